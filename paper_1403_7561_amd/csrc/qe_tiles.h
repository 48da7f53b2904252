// Wave-level element tiles shared by the single-instance kernels and the
// batched persistent kernel.
//
// A wave owns an 8 x 8 column of elements -- lane (lx, ly) = element
// (7 wx - 1 + lx, 7 wy - 1 + ly) -- and the 7 x 7 node columns that are the
// (1,1) corner of its elements with lx, ly < 7.  It marches up node planes
// k0 .. k0+kz-1, computing element layers k0-1 .. k0+kz-1.  The four
// contributions an owned node receives from one element layer come from
// lanes +0, +1, +8 and +9 (cross-lane shuffles); the one from the layer below
// is carried in a register.  Every nodal sum is formed in a fixed order, and
// every element is "owned" (written / counted) by exactly one wave: the one in
// which it has lx, ly >= 1 and a layer >= k0.
#pragma once

#include "qe_device.h"

namespace qe {

template <typename T>
__device__ __forceinline__ void load8(const T* __restrict__ p, T out[8]);

template <>
__device__ __forceinline__ void load8<double>(const double* __restrict__ p, double out[8]) {
  const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 v = q[i];
    out[2 * i] = v.x;
    out[2 * i + 1] = v.y;
  }
}

template <>
__device__ __forceinline__ void load8<float>(const float* __restrict__ p, float out[8]) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float4 v = q[i];
    out[4 * i] = v.x;
    out[4 * i + 1] = v.y;
    out[4 * i + 2] = v.z;
    out[4 * i + 3] = v.w;
  }
}

__device__ __forceinline__ void store8(double* p, const double v[8]) {
  double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
  for (int i = 0; i < 4; ++i) q[i] = make_double2(v[2 * i], v[2 * i + 1]);
}

__device__ __forceinline__ void store8(float* p, const double v[8]) {
  float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
  for (int i = 0; i < 2; ++i)
    q[i] = make_float4((float)v[4 * i], (float)v[4 * i + 1], (float)v[4 * i + 2], (float)v[4 * i + 3]);
}

template <typename T>
__device__ __forceinline__ T shfl_down_t(T v, int d) {
  return __shfl_down(v, d, 64);
}

// Sum of the four contributions of one element layer to this lane's owned node.
template <typename T>
__device__ __forceinline__ void gather_faces(const T out[8], T& bot, T& top) {
  bot = out[3] + shfl_down_t(out[2], 1) + shfl_down_t(out[1], 8) + shfl_down_t(out[0], 9);
  top = out[7] + shfl_down_t(out[6], 1) + shfl_down_t(out[5], 8) + shfl_down_t(out[4], 9);
}

// Geometry of one wave tile.
struct WaveTile {
  int lane, lx, ly, ex, ey, gi, gj, k0, Lbeg, Lend;
  bool active, col_ok, own_el, node_ok;
  long n00, ecol, elayer, sxy;
  long slot0, slot_layer;   // tile-major slot of this lane's element at layer 0, stride per layer
  double x0, x1, y0, y1;    // element corners: loaded here, first used once the sweep's first loads are issued

  __device__ __forceinline__ WaveTile(const Geom& g, int wx, int wy, int wz, int kz, int lane_, bool active_) {
    lane = lane_;
    active = active_;
    lx = lane & 7;
    ly = lane >> 3;
    ex = 7 * wx - 1 + lx;
    ey = 7 * wy - 1 + ly;
    col_ok = active_ && ex >= 0 && ex < g.nx - 1 && ey >= 0 && ey < g.ny - 1;
    own_el = col_ok && lx >= 1 && ly >= 1;
    gi = 7 * wx + lx;
    gj = 7 * wy + ly;
    node_ok = active_ && lx < 7 && ly < 7 && gi < g.nx && gj < g.ny;
    k0 = wz * kz;
    Lbeg = k0 - 1;
    Lend = min(k0 + kz - 1, g.nz - 1);
    sxy = (long)g.nx * g.ny;
    n00 = col_ok ? (long)ex + (long)g.nx * ey : 0;
    elayer = (long)(g.nx - 1) * (g.ny - 1);
    ecol = col_ok ? (long)ex + (long)(g.nx - 1) * ey : 0;
    const int tgx = (g.nx + 6) / 7, tgy = (g.ny + 6) / 7;
    slot_layer = (long)tgx * tgy * 49;
    slot0 = col_ok ? tile_slot(ex, ey, 0, tgx, tgy) : 0;
    // loaded in every lane (outside the mesh: the nearest element's, never
    // used), so that no branch leaves the count of loads in flight unknown
    const int cx = min(max(ex, 0), g.nx - 2), cy = min(max(ey, 0), g.ny - 2);
    x0 = g.x[cx];
    x1 = g.x[cx + 1];
    y0 = g.y[cy];
    y1 = g.y[cy + 1];
  }
  // the element's stiffness weights are eps * (ahx hz, ahy hz, axy / hz)
  __device__ __forceinline__ void weights(double& ahx, double& ahy, double& axy) const {
    const double hx = x1 - x0, hy = y1 - y0;
    ahx = hy / hx;
    ahy = hx / hy;
    axy = hx * hy;
  }
  __device__ __forceinline__ long slot(int L) const { return slot0 + slot_layer * L; }
  __device__ __forceinline__ long node(const Geom& g, int L) const { return (long)gi + (long)g.nx * gj + sxy * L; }
  // semiconductor flags of this column over the chunk, bit (L - Lbeg); the
  // byte loads are issued in groups of eight before any is waited for
  __device__ __forceinline__ unsigned int semi_bits(const Geom& g, const uint8_t* __restrict__ semi) const {
    unsigned int b = 0;
    if (col_ok) {
      const int lo = max(Lbeg, 0), hi = min(Lend, g.nz - 2);
      for (int L0 = lo; L0 <= hi; L0 += 8) {
        uint8_t f[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) f[j] = (L0 + j <= hi) ? semi[ecol + elayer * (L0 + j)] : 0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (f[j]) b |= 1u << (L0 + j - Lbeg);
      }
    }
    return b;
  }
};

// ---------------------------------------------------------------------------
// J.v on one wave tile (see k_jv_wave).  eps_t, cq and cflag are in
// tile-major order (tile_slot); cflag marks the elements whose Gauss-point
// coefficients are not all exactly zero, and only those read cq (a zero
// coefficient adds exactly nothing).  Modes:
//   JV_PLAIN  y = J v with v read as 0 on Dirichlet nodes; identity_rows
//             (1: y = v on Dirichlet rows, 2: y = 0 there).
//   JV_DOT    v = a CG direction (zero on Dirichlet nodes); y = J v on every
//             owned row; dot += v^T J v over the elements this wave owns.
//   JV_SMOOTH as JV_PLAIN with identity_rows = 2, then a smoothing step:
//             y = v + S (b - J v) on every owned node (S is 0 on Dirichlet
//             nodes), y a buffer other than v; dot += b^T y over them.
// In the CG mode the Dirichlet flag is not read at all: the vectors vanish
// on Dirichlet nodes and D^-1 is 0 there, so whatever y holds on those rows
// never reaches z, p or x.  (The single-instance CG uses jv_tile_cg below.)
enum JvMode { JV_PLAIN = 0, JV_DOT = 1, JV_SMOOTH = 2 };

// cbits: this lane's coefficient flags over the chunk (bit L - Lbeg), as
// written by residual_tile for the same wave tile.
template <typename T, int kMode>
__device__ __forceinline__ void jv_tile(const Geom& g, const WaveTile& w, const T* __restrict__ eps_t,
                                        unsigned int cbits, const T* __restrict__ cq,
                                        const uint8_t* __restrict__ mask, const T* __restrict__ v,
                                        T* __restrict__ y, int identity_rows, double& dot,
                                        const T* __restrict__ sm_b = nullptr, const T* __restrict__ sm_S = nullptr) {
  constexpr bool kPlain = kMode != JV_DOT;
  constexpr bool kSmooth = kMode == JV_SMOOTH;
  const unsigned int sbits = cbits;
  auto face = [&](int P, T f[4]) {
    const long b = w.n00 + w.sxy * P;
    const long o[4] = {0, 1, g.nx, g.nx + 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      T val = v[b + o[k]];
      if (kPlain && mask[b + o[k]]) val = T(0);
      f[k] = val;
    }
  };
  // Everything a layer's elements need is loaded one layer ahead and consumed
  // only in the next iteration, and no load is issued after those prefetches
  // inside an iteration: a wait for any later load would drain them (loads
  // retire in order).
  T fb[4], ft[4], fn[4];
  T cc[8], cn[8], ee = T(0), en = T(0);
  uint8_t mk = 0, mkn = 0;
  T xs = T(0), bs = T(0), ss = T(0), xsn = T(0), bsn = T(0), ssn = T(0);  // JV_SMOOTH: v, b, S at the owned node
#pragma unroll
  for (int k = 0; k < 4; ++k) fb[k] = ft[k] = fn[k] = T(0);
#pragma unroll
  for (int k = 0; k < 8; ++k) cc[k] = cn[k] = T(0);
  if (w.col_ok && w.Lbeg >= 0) face(w.Lbeg, fb);
  if (w.col_ok && w.Lbeg + 1 <= g.nz - 1) face(w.Lbeg + 1, ft);
  if (w.col_ok && w.Lbeg >= 0 && w.Lbeg <= g.nz - 2) {
    const long sl = w.slot(w.Lbeg);
    ee = eps_t[sl];
    if (sbits & 1u) load8(cq + 8 * sl, cc);
  }
  if (kPlain && w.node_ok && w.Lbeg >= 0) mk = mask[w.node(g, w.Lbeg)];
  // the chunk's z spacings: lane j holds layer Lbeg + j, read per layer with
  // readlane (scalar, no memory access in the sweep)
  double zlo = 0.0, zhi = 1.0, rdzl = 1.0;
  {
    const int L = w.Lbeg + w.lane;
    if (L >= 0 && L <= min(w.Lend, g.nz - 2)) {
      zlo = g.z[L];
      zhi = g.z[L + 1];
      rdzl = g.rdz[L];
    }
  }
  double ahx, ahy, axy;
  w.weights(ahx, ahy, axy);
  const double hzl = zhi - zlo;
  T carry = T(0);
  // Retire the loads above before the loop.  Otherwise the first iteration's
  // operands are still in flight on entry, and the wait inserted for them
  // inside the loop body (a vmcnt wait, which retires in order) also drains
  // every prefetch of every later iteration.  An empty asm that reads and
  // writes each value forces that wait here without touching memory.
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    asm("" : "+v"(fb[k]));
    asm("" : "+v"(ft[k]));
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) asm("" : "+v"(cc[k]));
  asm("" : "+v"(ee));
  for (int L = w.Lbeg; L <= w.Lend; ++L) {
    const bool layer_ok = (L >= 0 && L <= g.nz - 2);
    const int L1 = L + 1;
    const double hz = lane_value(hzl, L - w.Lbeg);    // 1 outside [0, nz-2]
    const double rhz = lane_value(rdzl, L - w.Lbeg);
    // prefetch the next top face, the next layer's data and the next flag
    if (w.col_ok && L1 <= w.Lend && L1 + 1 <= g.nz - 1) face(L1 + 1, fn);
    if (w.col_ok && L1 <= w.Lend && L1 <= g.nz - 2) {
      const long sl = w.slot(L1);
      en = eps_t[sl];
      if ((sbits >> (L1 - w.Lbeg)) & 1u) load8(cq + 8 * sl, cn);
    }
    if (kPlain && w.node_ok && L1 <= w.Lend) mkn = mask[w.node(g, L1)];
    if (kSmooth && w.node_ok && L1 <= w.Lend) {
      const long n1 = w.node(g, L1);
      xsn = v[n1];
      bsn = sm_b[n1];
      ssn = sm_S[n1];
    }
    T out[8];
    if (w.col_ok && layer_ok) {
      const T sx = ee * T(ahx * hz), sy = ee * T(ahy * hz), sz = ee * T(axy * rhz);
      const T ve[8] = {fb[0], fb[1], fb[2], fb[3], ft[0], ft[1], ft[2], ft[3]};
      const double d =
          jv_element<T, kMode == JV_DOT>(ve, sx, sy, sz, cc, ((sbits >> (L - w.Lbeg)) & 1u) != 0, out);
      if (kMode == JV_DOT && w.own_el && L >= w.k0) dot += d;
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) out[k] = T(0);
    }
    T bot, top;
    gather_faces(out, bot, top);
    if (w.node_ok && L >= w.k0) {
      const long n = w.node(g, L);
      T val = carry + bot;
      if (kPlain && mk && identity_rows) val = identity_rows == 1 ? v[n] : T(0);
      if (kSmooth) {
        val = xs + ss * (bs - val);
        dot += (double)bs * (double)val;
      }
      y[n] = val;
    }
    carry = top;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      fb[k] = ft[k];
      ft[k] = fn[k];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) cc[k] = cn[k];
    ee = en;
    mk = mkn;
    xs = xsn;
    bs = bsn;
    ss = ssn;
  }
}

// What the CG sweep learns once its first loads are in flight: whether to go
// on (the solve has not stopped), beta, and whether this is the first
// iteration (p = z, y = J z).
// Whether the CG loop's first kernel also takes the previous iteration's
// solution step x += alpha p (it reads p anyway): in FP64 this saves the
// second kernel a read of p and a read and write of x; the FP32 sweep
// measured slower with it, so there the second kernel keeps the step.
template <typename T>
constexpr bool cg_jv_steps_x() {
  return sizeof(T) == 8;
}

template <typename T>
struct JvGo {
  bool go;
  T beta;
  bool first;
  T alpha;   // the previous iteration's step length (not read on the first)
};

// ---------------------------------------------------------------------------
// The CG sweep on raw buffer resources.
//
// Every load and store of this sweep is a raw buffer access.  A lane whose
// access is not wanted passes an offset beyond the resource's range; the
// hardware then returns zeros (load) or drops the write (store) without
// touching memory.  So the sweep issues the same memory instructions in every
// layer step and in every lane, with no branch around any of them, and the
// compiler's wait counts stay exact: the wait for one layer's operands never
// drains the loads already issued for the next layer (vector memory counts
// retire in order, and a load under a branch leaves the count after the join
// unknown, which forces a full drain).
//
// Each wave's resources start at its lowest layer, and per-layer steps are
// scalar offsets, so per-lane offsets are 32-bit and fixed over the sweep.
typedef unsigned int qe_u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int qe_u32x4 __attribute__((ext_vector_type(4)));
constexpr unsigned int kBufOob = 0x80000000u;     // offset past every range below
constexpr long kBufRangeMax = 0x7fffffffL;
constexpr unsigned int kBufConfig = 0x00020000u;  // raw 32-bit dword data format

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_res(const void* base, long bytes) {
  const long n = bytes <= 0 ? 0 : (bytes < kBufRangeMax ? bytes : kBufRangeMax);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)n, (int)kBufConfig);
}

template <typename T>
struct BufIO;

template <>
struct BufIO<double> {
  static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, unsigned int v, unsigned int s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, double x, unsigned int v, unsigned int s) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(qe_u32x2, x), r, v, s, 0);
  }
  // eight consecutive values (one element's Gauss-point coefficients)
  static __device__ __forceinline__ void ld8(__amdgpu_buffer_rsrc_t r, unsigned int v, unsigned int s, double o[8]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const qe_u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, v + 16 * i, s, 0);
      o[2 * i] = __builtin_bit_cast(double, (qe_u32x2){q.x, q.y});
      o[2 * i + 1] = __builtin_bit_cast(double, (qe_u32x2){q.z, q.w});
    }
  }
};

template <>
struct BufIO<float> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, unsigned int v, unsigned int s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, float x, unsigned int v, unsigned int s) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, v, s, 0);
  }
  static __device__ __forceinline__ void ld8(__amdgpu_buffer_rsrc_t r, unsigned int v, unsigned int s, float o[8]) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const qe_u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, v + 16 * i, s, 0);
      // by value: a bit cast of a vector element reads element 0
      o[4 * i] = __uint_as_float(q.x);
      o[4 * i + 1] = __uint_as_float(q.y);
      o[4 * i + 2] = __uint_as_float(q.z);
      o[4 * i + 3] = __uint_as_float(q.w);
    }
  }
};

// The value of lane + 1 (DPP row shift: lanes 15, 31, 47, 63 read 0).  In a
// wave tile the lanes with lx = 7, the only ones whose lane + 1 is in another
// row of 8, own no node.
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x101, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x101, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 2D Haar butterflies of one face (index bit 0 = x, bit 1 = y); the same
// transform inverts itself up to a factor 4.
template <typename T>
__device__ __forceinline__ void haar2(const T f[4], T u[4]) {
  const T a0 = f[0] + f[1], a1 = f[0] - f[1], a2 = f[2] + f[3], a3 = f[2] - f[3];
  u[0] = a0 + a2;
  u[1] = a1 + a3;
  u[2] = a0 - a2;
  u[3] = a1 - a3;
}

// What one layer step needs from memory, loaded one step ahead: the top face
// of the element layer (raw z values at its corners), the element's
// permittivity and Gauss-point coefficients and, at the lane's owned node of
// that layer, y, p and x.
template <typename T>
struct CgStage {
  T f[4];
  T e;
  T yv, pv, xv;
  T c[8];
};

// CG sweep on one wave tile: v = z (zero on Dirichlet nodes); on owned rows
// y = J z + beta y and p = z + beta p (first: y = J z, p = z), so y = J p by
// recurrence, and (when cg_jv_steps_x<T>()) the previous iteration's
// solution step x += alpha p with the p read before its update (not on the
// first); dot += p^T y over owned nodes.  pre() is called by every wave
// once the first loads are issued (it may synchronise the block); false: the
// solve has stopped and nothing was stored.  The element operator is
// jv_element's, with the partial sums grouped per face.  The bottom face of each element layer is kept in
// the 2D Haar basis from the step before, and the top-face output of one
// element layer is added to the bottom-face output of the next in that basis,
// so each face is transformed, inverse-transformed and gathered across lanes
// once.  Layer steps run in pairs over kz + 1 layers rounded up to even (the
// last step loads nothing ahead); a step beyond the chunk or the mesh loads
// in-range data it does not use (its z spacing is 0, its coefficient flag is
// clear) and stores nothing.
template <typename T, typename Pre>
__device__ __forceinline__ bool jv_tile_cg(const Geom& g, const WaveTile& w, int kz, const T* __restrict__ eps_t,
                                           unsigned int cbits, const T* __restrict__ cq, const T* __restrict__ z,
                                           T* __restrict__ y, T* __restrict__ p, T* __restrict__ x, double& dot,
                                           Pre pre) {
  using IO = BufIO<T>;
  constexpr unsigned int B = sizeof(T);
  const long sxy = w.sxy, sl = w.slot_layer;
  // lowest node (and element) layer the sweep reads; an idle wave (past the
  // last tile, its chunk above the mesh) gets the top element layer, so that
  // every range below is positive and it reads only zeros
  const int Pb = min(max(w.Lbeg, 0), g.nz - 2);
  const __amdgpu_buffer_rsrc_t rz = buf_res(z + sxy * Pb, (long)(g.nz - Pb) * sxy * B);
  const __amdgpu_buffer_rsrc_t ry = buf_res(y + sxy * Pb, (long)(g.nz - Pb) * sxy * B);
  const __amdgpu_buffer_rsrc_t rp = buf_res(p + sxy * Pb, (long)(g.nz - Pb) * sxy * B);
  const __amdgpu_buffer_rsrc_t rx = buf_res(x + sxy * Pb, (long)(g.nz - Pb) * sxy * B);
  const __amdgpu_buffer_rsrc_t re = buf_res(eps_t + sl * Pb, (long)(g.nz - 1 - Pb) * sl * B);
  const __amdgpu_buffer_rsrc_t rc = buf_res(cq + 8 * sl * Pb, (long)(g.nz - 1 - Pb) * sl * 8 * B);
  // per-lane byte offsets within a layer; corner 3 of the face is the owned
  // node, also read by lanes that own a node but no element (mesh edge x = 0
  // or y = 0), whose element terms are zero (their permittivity reads 0)
  const long nxy = (long)w.gi + (long)g.nx * w.gj;
  const unsigned int o_f[4] = {w.col_ok ? (unsigned int)(w.n00 * B) : kBufOob,
                               w.col_ok ? (unsigned int)((w.n00 + 1) * B) : kBufOob,
                               w.col_ok ? (unsigned int)((w.n00 + g.nx) * B) : kBufOob,
                               (w.col_ok || w.node_ok) ? (unsigned int)(nxy * B) : kBufOob};
  const unsigned int o_n = w.node_ok ? (unsigned int)(nxy * B) : kBufOob;
  const unsigned int o_e = w.col_ok ? (unsigned int)(w.slot0 * B) : kBufOob;
  const unsigned int o_c = (unsigned int)(w.slot0 * 8 * B);
  // scalar offset of node layer P / element layer L (clamped into the mesh)
  auto s_node = [&](int P) -> unsigned int { return (unsigned int)((min(max(P, 0), g.nz - 1) - Pb) * sxy * B); };
  auto s_elem = [&](int L) -> unsigned int { return (unsigned int)((min(max(L, 0), g.nz - 2) - Pb) * sl * B); };

  // The prologue's loads are all unconditional, so that pre() can wait for
  // loads its caller issued before them without waiting for them.  First the
  // chunk's z spacings: lane j holds layer Lbeg + j (clamped into the mesh),
  // read per step with readlane.
  double hzl, rdzl;
  {
    const int L = min(max(w.Lbeg + w.lane, 0), g.nz - 2);
    hzl = g.hz[L];
    rdzl = g.rdz[L];
  }
  CgStage<T> A, Bs;
  T fb[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) fb[k] = IO::ld(rz, o_f[k], s_node(w.Lbeg));
#pragma unroll
  for (int k = 0; k < 4; ++k) A.f[k] = IO::ld(rz, o_f[k], s_node(w.Lbeg + 1));
  A.e = IO::ld(re, o_e, s_elem(w.Lbeg));
  A.yv = A.pv = A.xv = T(0);   // node layer Lbeg is never owned
  // the flag word is first used here, after the loads above are issued (an
  // idle wave's word is not its own: cleared)
  __builtin_amdgcn_sched_barrier(0);
  if (!w.active) cbits = 0u;
  IO::ld8(rc, (cbits & 1u) ? o_c : kBufOob, 8 * s_elem(w.Lbeg), A.c);
  const JvGo<T> go = pre();
  if (!go.go) return false;
  double ahx, ahy, axy;
  w.weights(ahx, ahy, axy);
  const T beta = go.beta, alpha = go.alpha;
  const bool rec_old = !go.first;
  // retire the prologue's loads before the loop (see jv_tile)
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    asm("" : "+v"(fb[k]));
    asm("" : "+v"(A.f[k]));
  }
  asm("" : "+v"(A.e));
  T Tb[4], carry[4] = {T(0), T(0), T(0), T(0)};
  haar2(fb, Tb);
  T zb = fb[3];
  const bool own_lane = w.node_ok;

  // kNext: load the next step's operands (the chunk's last step has none)
  auto step = [&](int L, CgStage<T>& cur, CgStage<T>& nxt, auto next_tag) {
    constexpr bool kNext = decltype(next_tag)::value;
    const int j = L - w.Lbeg;
    const bool flag = (cbits >> j) & 1u;
    // The next step's operands.  Its Gauss-point coefficients are loaded by
    // the flagged lanes only (the one conditional access of the step) and
    // issued first: a wait that the compiler sizes for the path without them
    // then waits at most for them early, never for the loads issued after
    // them (scheduling barriers keep this order).
    if constexpr (kNext) {
#pragma unroll
      for (int k = 0; k < 8; ++k) nxt.c[k] = T(0);
      if ((cbits >> (j + 1)) & 1u) IO::ld8(rc, o_c, 8 * s_elem(L + 1), nxt.c);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) nxt.f[k] = IO::ld(rz, o_f[k], s_node(L + 2));
      nxt.e = IO::ld(re, o_e, s_elem(L + 1));
      nxt.yv = IO::ld(ry, o_n, s_node(L + 1));
      nxt.pv = IO::ld(rp, o_n, s_node(L + 1));
      if constexpr (cg_jv_steps_x<T>()) nxt.xv = IO::ld(rx, o_n, s_node(L + 1));
      __builtin_amdgcn_sched_barrier(0);
    }
    // element layer L: Haar coefficients, diagonal stiffness, mass term
    // 0 off the mesh (a scalar select)
    const bool lay_ok = L >= 0 && L <= g.nz - 2;
    const double hz = lay_ok ? lane_value(hzl, j) : 0.0, rhz = lay_ok ? lane_value(rdzl, j) : 0.0;
    const T sx = cur.e * T(ahx * hz), sy = cur.e * T(ahy * hz), sz = cur.e * T(axy * rhz);
    T Tt[4];
    haar2(cur.f, Tt);
    T vt[8], out[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      vt[k] = Tb[k] + Tt[k];
      vt[k + 4] = Tb[k] - Tt[k];
    }
    const T k2 = T(1.0 / 16.0), k6 = T(1.0 / 48.0), k18 = T(1.0 / 144.0);
    out[0] = T(0);
    out[1] = (sx * k2) * vt[1];
    out[2] = (sy * k2) * vt[2];
    out[3] = ((sx + sy) * k6) * vt[3];
    out[4] = (sz * k2) * vt[4];
    out[5] = ((sx + sz) * k6) * vt[5];
    out[6] = ((sy + sz) * k6) * vt[6];
    out[7] = ((sx + sy + sz) * k18) * vt[7];
    if (flag) {
      const T b0 = T(0.125), b1 = T(0.07216878364870322), b2 = T(0.041666666666666664),
              b3 = T(0.024056261216234407);
      const T db[8] = {b0, b1, b1, b2, b1, b2, b2, b3};
      T q[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) q[k] = db[k] * vt[k];
      haar3(q);
#pragma unroll
      for (int k = 0; k < 8; ++k) q[k] *= cur.c[k];
      haar3(q);
#pragma unroll
      for (int k = 0; k < 8; ++k) out[k] += db[k] * q[k];
    }
    // bottom-face output joins the top-face output of the layer below, then
    // one inverse face transform and one gather give node layer L
    T on[4], corner[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      on[k] = carry[k] + (out[k] + out[k + 4]);
      carry[k] = out[k] - out[k + 4];
    }
    haar2(on, corner);
    const T u = corner[3] + lane_next(corner[2]);
    const T v2 = corner[1] + lane_next(corner[0]);
    T val = u + shfl_down_t(v2, 8);
    T pv = zb;
    if (rec_old) {
      val += beta * cur.yv;
      pv += beta * cur.pv;
    }
    const bool st = L >= w.k0 && L <= w.Lend;
    IO::st(ry, val, st ? o_n : kBufOob, s_node(L));
    IO::st(rp, pv, st ? o_n : kBufOob, s_node(L));
    if constexpr (cg_jv_steps_x<T>()) IO::st(rx, cur.xv + alpha * cur.pv, (st && rec_old) ? o_n : kBufOob, s_node(L));
    if (st && own_lane) dot += (double)pv * (double)val;
#pragma unroll
    for (int k = 0; k < 4; ++k) Tb[k] = Tt[k];
    zb = cur.f[3];
  };
  using Next = std::integral_constant<bool, true>;
  using Last = std::integral_constant<bool, false>;
  const int nsteps = (kz + 2) & ~1;
  for (int s = 0; s < nsteps - 2; s += 2) {
    step(w.Lbeg + s, A, Bs, Next());
    step(w.Lbeg + s + 1, Bs, A, Next());
  }
  step(w.Lbeg + nsteps - 2, A, Bs, Next());
  step(w.Lbeg + nsteps - 1, Bs, A, Last());
  return true;
}

// ---------------------------------------------------------------------------
// H v and M v of the generalized Schrodinger eigenproblem for two columns at
// once, on raw buffer resources like jv_tile_cg.  H's element operator is the
// stiffness with per-element weights eH along x, y and z (a diagonal mass
// tensor, Eq. Schrodinger3D) plus the Gauss-point coefficients cH (eight per
// element); M's is the consistent mass matrix, which in the Haar
// basis is diagonal, (V / 64) (1/3)^(number of difference axes) for an
// element of volume V, so it costs eight products and no memory.  Both share
// the face loads, the forward transforms and the first Gauss-point transform;
// the element data (eH, cH) are loaded once for both columns.
//
// The input columns must vanish on the fixed nodes (the eigensolver keeps its
// basis in that subspace); outputs are 0 on owned nodes whose bit in mbits
// (bit L - Lbeg: the node of layer L is fixed) is set.  col_ok[1] = false:
// the second column is absent (its resources are empty: zeros in, no stores).
struct HmStage {
  double f[2][4];
  double e[3];   // kinetic weights along x, y, z
  double c[8];
};

__device__ __forceinline__ void jv_tile_hm(const Geom& g, const WaveTile& w, int kz, const double* __restrict__ eH,
                                           const double* __restrict__ cH, unsigned int mbits,
                                           const double* const zc[2], double* const yh[2], double* const ym[2],
                                           const bool col_ok[2]) {
  using IO = BufIO<double>;
  constexpr unsigned int B = 8;
  const long sxy = w.sxy, sl = w.slot_layer;
  const int Pb = min(max(w.Lbeg, 0), g.nz - 2);
  const long vbytes = (long)(g.nz - Pb) * sxy * B;
  __amdgpu_buffer_rsrc_t rz[2], rh[2], rm[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    rz[c] = buf_res(zc[c] + sxy * Pb, col_ok[c] ? vbytes : 0);
    rh[c] = buf_res(yh[c] + sxy * Pb, col_ok[c] ? vbytes : 0);
    rm[c] = buf_res(ym[c] + sxy * Pb, col_ok[c] ? vbytes : 0);
  }
  // eH holds three planes of tile-major weights (x, y, z), nslots apart
  const long nslots = sl * (g.nz - 1);
  __amdgpu_buffer_rsrc_t re[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) re[a] = buf_res(eH + a * nslots + sl * Pb, (long)(g.nz - 1 - Pb) * sl * B);
  const __amdgpu_buffer_rsrc_t rc = buf_res(cH + 8 * sl * Pb, (long)(g.nz - 1 - Pb) * sl * 8 * B);
  const long nxy = (long)w.gi + (long)g.nx * w.gj;
  const unsigned int o_f[4] = {w.col_ok ? (unsigned int)(w.n00 * B) : kBufOob,
                               w.col_ok ? (unsigned int)((w.n00 + 1) * B) : kBufOob,
                               w.col_ok ? (unsigned int)((w.n00 + g.nx) * B) : kBufOob,
                               w.col_ok ? (unsigned int)((w.n00 + g.nx + 1) * B) : kBufOob};
  const unsigned int o_n = w.node_ok ? (unsigned int)(nxy * B) : kBufOob;
  const unsigned int o_e = w.col_ok ? (unsigned int)(w.slot0 * B) : kBufOob;
  const unsigned int o_c = w.col_ok ? (unsigned int)(w.slot0 * 8 * B) : kBufOob;
  auto s_node = [&](int P) -> unsigned int { return (unsigned int)((min(max(P, 0), g.nz - 1) - Pb) * sxy * B); };
  auto s_elem = [&](int L) -> unsigned int { return (unsigned int)((min(max(L, 0), g.nz - 2) - Pb) * sl * B); };
  // element data of layer L: zeros off the mesh (the coefficients are not
  // scaled by the layer's z spacing, so they need their own guard)
  auto o_cl = [&](int L) -> unsigned int { return (L >= 0 && L <= g.nz - 2) ? o_c : kBufOob; };
  if (!w.active) mbits = 0u;

  double hzl, rdzl;
  {
    const int L = min(max(w.Lbeg + w.lane, 0), g.nz - 2);
    hzl = g.hz[L];
    rdzl = g.rdz[L];
  }
  HmStage A, Bs;
  double fb[2][4];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      fb[c][k] = IO::ld(rz[c], o_f[k], s_node(w.Lbeg));
      A.f[c][k] = IO::ld(rz[c], o_f[k], s_node(w.Lbeg + 1));
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) A.e[a] = IO::ld(re[a], o_e, s_elem(w.Lbeg));
  IO::ld8(rc, o_cl(w.Lbeg), 8 * s_elem(w.Lbeg), A.c);
  double ahx, ahy, axy;
  w.weights(ahx, ahy, axy);
  // retire the prologue's loads before the loop (see jv_tile)
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      asm("" : "+v"(fb[c][k]));
      asm("" : "+v"(A.f[c][k]));
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) asm("" : "+v"(A.e[a]));
#pragma unroll
  for (int k = 0; k < 8; ++k) asm("" : "+v"(A.c[k]));
  double Tb[2][4], carH[2][4], carM[2][4];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    haar2(fb[c], Tb[c]);
#pragma unroll
    for (int k = 0; k < 4; ++k) carH[c][k] = carM[c][k] = 0.0;
  }

  auto step = [&](int L, HmStage& cur, HmStage& nxt, auto next_tag) {
    constexpr bool kNext = decltype(next_tag)::value;
    const int j = L - w.Lbeg;
    if constexpr (kNext) {
      IO::ld8(rc, o_cl(L + 1), 8 * s_elem(L + 1), nxt.c);
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) nxt.f[c][k] = IO::ld(rz[c], o_f[k], s_node(L + 2));
#pragma unroll
      for (int a = 0; a < 3; ++a) nxt.e[a] = IO::ld(re[a], o_e, s_elem(L + 1));
      __builtin_amdgcn_sched_barrier(0);
    }
    const bool lay_ok = L >= 0 && L <= g.nz - 2;
    const double hz = lay_ok ? lane_value(hzl, j) : 0.0, rhz = lay_ok ? lane_value(rdzl, j) : 0.0;
    const double sx = cur.e[0] * (ahx * hz), sy = cur.e[1] * (ahy * hz), sz = cur.e[2] * (axy * rhz);
    const double k2 = 1.0 / 16.0, k6 = 1.0 / 48.0, k18 = 1.0 / 144.0;
    const double d1 = sx * k2, d2 = sy * k2, d3 = (sx + sy) * k6, d4 = sz * k2, d5 = (sx + sz) * k6,
                 d6 = (sy + sz) * k6, d7 = (sx + sy + sz) * k18;
    // M in the Haar basis (volume axy hz), with the final transform's 1/8
    const double V = axy * hz;
    const double m0 = V * (1.0 / 64.0), m1 = V * (1.0 / 192.0), m2 = V * (1.0 / 576.0), m3 = V * (1.0 / 1728.0);
    const double db[8] = {0.125, 0.07216878364870322, 0.07216878364870322, 0.041666666666666664,
                          0.07216878364870322, 0.041666666666666664, 0.041666666666666664, 0.024056261216234407};
    const bool st = L >= w.k0 && L <= w.Lend;
    const bool fixed = (mbits >> j) & 1u;
    const unsigned int os = st ? o_n : kBufOob;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double Tt[4], vt[8], oh[8], om[8], q[8];
      haar2(cur.f[c], Tt);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        vt[k] = Tb[c][k] + Tt[k];
        vt[k + 4] = Tb[c][k] - Tt[k];
      }
      om[0] = m0 * vt[0];
      om[1] = m1 * vt[1];
      om[2] = m1 * vt[2];
      om[3] = m2 * vt[3];
      om[4] = m1 * vt[4];
      om[5] = m2 * vt[5];
      om[6] = m2 * vt[6];
      om[7] = m3 * vt[7];
#pragma unroll
      for (int k = 0; k < 8; ++k) q[k] = db[k] * vt[k];
      haar3(q);   // Gauss-point values
#pragma unroll
      for (int k = 0; k < 8; ++k) q[k] *= cur.c[k];
      haar3(q);
      oh[0] = db[0] * q[0];
      oh[1] = d1 * vt[1] + db[1] * q[1];
      oh[2] = d2 * vt[2] + db[2] * q[2];
      oh[3] = d3 * vt[3] + db[3] * q[3];
      oh[4] = d4 * vt[4] + db[4] * q[4];
      oh[5] = d5 * vt[5] + db[5] * q[5];
      oh[6] = d6 * vt[6] + db[6] * q[6];
      oh[7] = d7 * vt[7] + db[7] * q[7];
      double onH[4], onM[4], crH[4], crM[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        onH[k] = carH[c][k] + (oh[k] + oh[k + 4]);
        carH[c][k] = oh[k] - oh[k + 4];
        onM[k] = carM[c][k] + (om[k] + om[k + 4]);
        carM[c][k] = om[k] - om[k + 4];
      }
      haar2(onH, crH);
      haar2(onM, crM);
      double vh = (crH[3] + lane_next(crH[2])) + shfl_down_t(crH[1] + lane_next(crH[0]), 8);
      double vm = (crM[3] + lane_next(crM[2])) + shfl_down_t(crM[1] + lane_next(crM[0]), 8);
      if (fixed) vh = vm = 0.0;
      IO::st(rh[c], vh, os, s_node(L));
      IO::st(rm[c], vm, os, s_node(L));
#pragma unroll
      for (int k = 0; k < 4; ++k) Tb[c][k] = Tt[k];
    }
  };
  using Next = std::integral_constant<bool, true>;
  using Last = std::integral_constant<bool, false>;
  const int nsteps = (kz + 2) & ~1;
  for (int s = 0; s < nsteps - 2; s += 2) {
    step(w.Lbeg + s, A, Bs, Next());
    step(w.Lbeg + s + 1, Bs, A, Next());
  }
  step(w.Lbeg + nsteps - 2, A, Bs, Next());
  step(w.Lbeg + nsteps - 1, Bs, A, Last());
}

// ---------------------------------------------------------------------------
// Predictor-corrector electrons of one element at its Gauss points (Sec.
// II.B.2): nq_q = P sum_i |psi_i|^2_q G(x_iq) and dnq_q = P/kT sum_i
// |psi_i|^2_q G'(x_iq), x_iq = (phi_q - phi^(k)_q - E_i)/kT, over the states
// in act (wave-uniform); |psi_i|^2 and phi^(k) are interpolated from the
// nodes like phi, and src holds phi at the Gauss points.
//
// 3D confinement (G = 1/(1 + e^-x)): e^-x_iq = e^-y_q e^(E_i/kT) with y_q =
// (phi_q - phi^(k)_q)/kT, so one exponential per Gauss point serves every
// state.  An element with some |y_q| > kPcExpMax (and 1D confinement) takes
// the per-state form, so that no product leaves the double range.  The form
// is chosen per element, never per wave: the owner of an element and the
// waves that see it as a halo get the same coefficients, zeros included (the
// J.v of a wave reads the owner's coefficients where its own are nonzero).
//
// The |psi_i|^2 loads are buffer loads with one per-lane offset (the
// element's first node; 8 N < 2^31 bytes, checked on the host) and scalar
// layer, corner and state steps; the next state's eight loads are issued
// before the current state is used, into the other of two register sets.
__device__ __forceinline__ void pc_electrons(const Geom& g, const WaveTile& w, int L, const Quantum& qm,
                                             unsigned int act, const double src[8], double nq[8],
                                             double dnq[8]) {
  const long b0 = w.n00 + w.sxy * L;
  double u[8];
  {
    const long o[8] = {0, 1, g.nx, g.nx + 1, w.sxy, w.sxy + 1, w.sxy + g.nx, w.sxy + g.nx + 1};
#pragma unroll
    for (int k = 0; k < 8; ++k) u[k] = qm.phik[b0 + o[k]];
  }
  gauss_interp(u);
  bool fast = qm.fast != 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    u[q] = (src[q] - u[q]) * qm.inv_kT;   // y_q
    fast = fast && fabs(u[q]) <= kPcExpMax;
  }
  if (fast) {
#pragma unroll
    for (int q = 0; q < 8; ++q) u[q] = exp(-u[q]);   // e^-y_q
  }
  const bool all_fast = __builtin_amdgcn_ballot_w64(!fast) == 0;
  const unsigned int vo = (unsigned int)(w.n00 * 8);
  const unsigned int s0 = (unsigned int)(w.sxy * L * 8), sy = (unsigned int)(g.nx * 8),
                     sz = (unsigned int)(w.sxy * 8);
  const long nbytes = qm.N * 8;
  auto load = [&](int i, double s2[8]) {
    const __amdgpu_buffer_rsrc_t r = buf_res(qm.psi2 + qm.N * i, nbytes);
    s2[0] = BufIO<double>::ld(r, vo, s0);
    s2[1] = BufIO<double>::ld(r, vo + 8, s0);
    s2[2] = BufIO<double>::ld(r, vo, s0 + sy);
    s2[3] = BufIO<double>::ld(r, vo + 8, s0 + sy);
    s2[4] = BufIO<double>::ld(r, vo, s0 + sz);
    s2[5] = BufIO<double>::ld(r, vo + 8, s0 + sz);
    s2[6] = BufIO<double>::ld(r, vo, s0 + sz + sy);
    s2[7] = BufIO<double>::ld(r, vo + 8, s0 + sz + sy);
  };
  // G = 1/(1 + t), t = e^-x in [e^-600, e^600]: a reciprocal refined twice
  // by Newton's iteration; dG/dx = t G^2 = G (t G), in that order so that it
  // does not underflow; P and 1/kT are applied after the sum.  Written with
  // explicit fma so that every copy rounds alike.
  auto fast_terms = [&](int i, const double s2[8]) {
    const double Bi = qm.B[i];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double t = u[q] * Bi;
      const double d = fma(u[q], Bi, 1.0);
      double G = __builtin_amdgcn_rcp(d);
      G = fma(G, fma(-d, G, 1.0), G);
      G = fma(G, fma(-d, G, 1.0), G);
      nq[q] = fma(s2[q], G, nq[q]);
      dnq[q] = fma(s2[q], G * (t * G), dnq[q]);
    }
  };
  auto slow_terms = [&](int i, const double s2[8]) {
    const double ei = qm.E[i] * qm.inv_kT;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double G, dG;
      pc_occupation(qm.conf, u[q] - ei, G, dG);
      nq[q] = fma(s2[q], G, nq[q]);
      dnq[q] = fma(s2[q], dG, dnq[q]);
    }
  };
  // one state's terms; the loop over states has one copy for waves whose
  // elements all take the one-exponential form and one that chooses per lane
  auto add = [&](auto kAllFast, int i, double s2[8]) {
    gauss_interp(s2);
    if constexpr (decltype(kAllFast)::value) {
      fast_terms(i, s2);
    } else {
      if (fast)
        fast_terms(i, s2);
      else
        slow_terms(i, s2);
    }
  };
  // states in increasing order; the pass for the last state reloads it into
  // the idle set (not used), so that every pass issues its loads unconditionally
  auto states = [&](auto kAllFast) {
    unsigned int m = act;
    int i = __builtin_ctz(m);
    m &= m - 1;
    double sa[8], sb[8];
    load(i, sa);
    for (;;) {
      int j = m ? __builtin_ctz(m) : i;
      load(j, sb);
      add(kAllFast, i, sa);
      if (!m) break;
      m &= m - 1;
      i = j;
      j = m ? __builtin_ctz(m) : i;
      load(j, sa);
      add(kAllFast, i, sb);
      if (!m) break;
      m &= m - 1;
      i = j;
    }
  };
  if (all_fast)
    states(std::integral_constant<bool, true>());
  else
    states(std::integral_constant<bool, false>());
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    nq[q] *= qm.pref;
    dnq[q] *= qm.pref * qm.inv_kT;
  }
}

// ---------------------------------------------------------------------------
// Residual F(phi + lam delta), Jacobi diagonal and Gauss-point coefficients
// c_q = -KAPPA semi W rho'(phi_q) (= KAPPA semi W n'(phi_q) with electrons
// alone) on one wave tile.  F and the diagonal are
// written on owned nodes (0 and 1 on Dirichlet rows, where the stored inverse
// diagonal is 0).  The owning wave writes, in tile-major order, cflag = 1 for
// an element with a nonzero c_q and then its c_q, else cflag = 0 and nothing
// (depleted silicon, where n' underflows to exactly 0, and insulators).
// norm2 accumulates F_i^2 over owned free nodes.
template <typename TD, bool kQ = false>
__device__ __forceinline__ void residual_tile(const Geom& g, const WaveTile& w, const Charge& ch,
                                              const double* __restrict__ eps, const uint8_t* __restrict__ semi,
                                              const Doping dop, const uint8_t* __restrict__ mask,
                                              const double* __restrict__ phi, const TD* __restrict__ delta,
                                              double lam, const double* __restrict__ fsheet,
                                              const double* __restrict__ fdiag, double* __restrict__ F,
                                              double* __restrict__ invdiag,
                                              double* __restrict__ diag_out, double* __restrict__ cq,
                                              float* __restrict__ cq32, uint8_t* __restrict__ cflag,
                                              unsigned int* __restrict__ cbits, float* __restrict__ invdiag32,
                                              double& norm2, const Quantum* qm = nullptr) {
  const unsigned int sbits = w.semi_bits(g, semi);
  double ahx, ahy, axy;
  w.weights(ahx, ahy, axy);
  // eigenstates whose support box meets a column of this wave (wave-uniform)
  unsigned int qcols = 0;
  if (kQ && qm->n > 0) {
    for (int i = 0; i < qm->n; ++i) {
      const int* bx = qm->sbox + 6 * i;
      const bool in = w.col_ok && w.ex + 1 >= bx[0] && w.ex <= bx[1] && w.ey + 1 >= bx[2] && w.ey <= bx[3];
      if (__builtin_amdgcn_ballot_w64(in)) qcols |= 1u << i;
    }
  }
  auto face = [&](int P, double f[4]) {
    const long b = w.n00 + w.sxy * P;
    const long o[4] = {0, 1, g.nx, g.nx + 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double val = phi[b + o[k]];
      if (delta) val += lam * (double)delta[b + o[k]];
      f[k] = val;
    }
  };
  double fb[4], ft[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) fb[k] = ft[k] = 0.0;
  if (w.col_ok && w.Lbeg >= 0) face(w.Lbeg, fb);
  double carryF = 0.0, carryD = 0.0;
  unsigned int cb = 0;
  for (int L = w.Lbeg; L <= w.Lend; ++L) {
    const bool layer_ok = (L >= 0 && L <= g.nz - 2);
    if (w.col_ok && L + 1 <= g.nz - 1) face(L + 1, ft);
    double outF[8], outD[8];
    if (w.col_ok && layer_ok) {
      const long el = w.ecol + w.elayer * L;
      const double hz = g.z[L + 1] - g.z[L];
      const double ee = eps[el];
      const double sx = ee * (ahx * hz), sy = ee * (ahy * hz), sz = ee * (axy * g.rdz[L]);
      const double ve[8] = {fb[0], fb[1], fb[2], fb[3], ft[0], ft[1], ft[2], ft[3]};
      const double dg = (sx + sy + sz) * (1.0 / 9.0);
      // eps Khat phi: with eigenstates it is formed after the charge, so that
      // it is not live across the states' loop
      if (kQ) {
#pragma unroll
        for (int k = 0; k < 8; ++k) outF[k] = 0.0;
      } else {
        jv_element(ve, sx, sy, sz, outF, false, outF);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) outD[k] = dg;
      const bool own = w.own_el && L >= w.k0;
      bool nzc = false;  // some c_q of this element is nonzero
      if ((sbits >> (L - w.Lbeg)) & 1u) {
        const double kw = ch.kappa * axy * hz * 0.125;
        double net = 0.0, ndo = 0.0, nac = 0.0;
        if (ch.incomplete) {
          ndo = dop.donors[el];
          nac = dop.acceptors[el];
        } else if (dop.net) {
          net = dop.net[el];
        } else if (dop.donors) {
          net = dop.donors[el] - dop.acceptors[el];
        }
        double src[8], cc[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) src[k] = ve[k];
        gauss_interp(src);
        double nq[8], dnq[8];
        const bool qel = kQ && (!qm->region || qm->region[el]);   // electrons from the states
        if (qel) {
#pragma unroll
          for (int q = 0; q < 8; ++q) nq[q] = dnq[q] = 0.0;
          // states whose support box meets this layer of the wave's columns
          // (wave-uniform); in a lane outside a state's box all eight |psi_i|^2
          // read are exactly 0, and so is what the state adds there
          unsigned int act = 0;
          for (unsigned int m = qcols; m; m &= m - 1) {
            const int i = __builtin_ctz(m);
            if (L + 1 >= qm->sbox[6 * i + 4] && L <= qm->sbox[6 * i + 5]) act |= 1u << i;
          }
          if (act) pc_electrons(g, w, L, *qm, act, src, nq, dnq);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          double rho, drho;
          if (qel)
            space_charge_n(ch, src[q], nq[q], dnq[q], net, ndo, nac, rho, drho);
          else
            space_charge(ch, src[q], net, ndo, nac, rho, drho);
          src[q] = kw * rho;
          cc[q] = -kw * drho;
          nzc |= cc[q] != 0.0;
        }
        if (own && nzc) {
          const long sl = w.slot(L);
          store8(cq + 8 * sl, cc);
          if (cq32) store8(cq32 + 8 * sl, cc);
        }
        gauss_interp(src);
        gauss_sq_project(cc);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          outF[k] -= src[k];
          outD[k] += cc[k];
        }
      }
      if (kQ) {
        double kf[8];
        jv_element(ve, sx, sy, sz, kf, false, kf);
#pragma unroll
        for (int k = 0; k < 8; ++k) outF[k] += kf[k];
      }
      if (own) cflag[w.slot(L)] = nzc ? 1 : 0;
      if (nzc) cb |= 1u << (L - w.Lbeg);
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) outF[k] = outD[k] = 0.0;
    }
    double bF, tF, bD, tD;
    gather_faces(outF, bF, tF);
    gather_faces(outD, bD, tD);
    if (w.node_ok && L >= w.k0) {
      const long n = w.node(g, L);
      double f = carryF + bF, d = carryD + bD;
      const bool dir = mask[n] != 0;
      if (dir) {
        f = 0.0;
        d = 1.0;
      } else if (fsheet) {
        f += fsheet[n];   // interface-charge / Robin face terms
        d += fdiag[n];
      }
      F[n] = f;
      const double id = dir ? 0.0 : 1.0 / d;  // 0 keeps CG vectors at 0 on Dirichlet rows
      invdiag[n] = id;
      if (diag_out) diag_out[n] = d;
      if (invdiag32) invdiag32[n] = (float)id;
      norm2 += f * f;
    }
    carryF = tF;
    carryD = tD;
#pragma unroll
    for (int k = 0; k < 4; ++k) fb[k] = ft[k];
  }
  if (cbits) *cbits = cb;
}

}  // namespace qe
