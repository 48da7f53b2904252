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
  bool col_ok, own_el, node_ok;
  long n00, ecol, elayer, sxy;
  long slot0, slot_layer;   // tile-major slot of this lane's element at layer 0, stride per layer
  double x0, x1, y0, y1;    // element corners: loaded here, first used once the sweep's first loads are issued

  __device__ __forceinline__ WaveTile(const Geom& g, int wx, int wy, int wz, int kz, int lane_, bool active) {
    lane = lane_;
    lx = lane & 7;
    ly = lane >> 3;
    ex = 7 * wx - 1 + lx;
    ey = 7 * wy - 1 + ly;
    col_ok = active && ex >= 0 && ex < g.nx - 1 && ey >= 0 && ey < g.ny - 1;
    own_el = col_ok && lx >= 1 && ly >= 1;
    gi = 7 * wx + lx;
    gj = 7 * wy + ly;
    node_ok = active && lx < 7 && ly < 7 && gi < g.nx && gj < g.ny;
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
    x0 = y0 = 0.0;
    x1 = y1 = 1.0;
    if (col_ok) {
      x0 = g.x[ex];
      x1 = g.x[ex + 1];
      y0 = g.y[ey];
      y1 = g.y[ey + 1];
    }
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
//             (1: y = v on Dirichlet rows, 2: y = 0 there):
//             Dirichlet rows return v_i.
//   JV_DOT    v = a CG direction (zero on Dirichlet nodes); y = J v on every
//             owned row; dot += v^T J v over the elements this wave owns.
//   JV_REC    v = z (zero on Dirichlet nodes); on owned rows
//             y = J z + beta y and p = z + beta p (first: y = J z, p = z),
//             so y = J p by recurrence; dot += p^T y over owned nodes.
// In the CG modes the Dirichlet flag is not read at all: the vectors vanish
// on Dirichlet nodes and D^-1 is 0 there, so whatever y holds on those rows
// never reaches z, p or x.
enum JvMode { JV_PLAIN = 0, JV_DOT = 1, JV_REC = 2 };

// What a CG-mode sweep learns once its first loads are in flight: whether to
// go on (the solve has not stopped), and beta / first for JV_REC.
template <typename T>
struct JvGo {
  bool go;
  T beta;
  bool first;
};

template <typename T>
struct JvAlways {
  __device__ __forceinline__ JvGo<T> operator()() const { return {true, T(0), true}; }
};

// cbits: this lane's coefficient flags over the chunk (bit L - Lbeg), as
// written by residual_tile for the same wave tile.  pre() is called by every
// wave once the first layer's loads are issued (it may synchronise the block).
// Returns pre().go (false: nothing was stored).
template <typename T, int kMode, typename Pre = JvAlways<T>>
__device__ __forceinline__ bool jv_tile(const Geom& g, const WaveTile& w, const T* __restrict__ eps_t,
                                        unsigned int cbits, const T* __restrict__ cq,
                                        const uint8_t* __restrict__ mask, const T* __restrict__ v,
                                        T* __restrict__ y, int identity_rows, double& dot,
                                        T* __restrict__ p = nullptr, Pre pre = Pre()) {
  constexpr bool kPlain = kMode == JV_PLAIN, kRec = kMode == JV_REC;
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
  const bool z_own = kRec && !w.col_ok && w.node_ok;   // owned node outside every element face loaded
  T fb[4], ft[4], fn[4];
  T cc[8], cn[8], ee = T(0), en = T(0);
  T yc = T(0), pc = T(0), zc = T(0);
  uint8_t mk = 0, mkn = 0;
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
  const JvGo<T> go = pre();
  if (!go.go) return false;
  double ahx, ahy, axy;
  w.weights(ahx, ahy, axy);
  const double hzl = zhi - zlo;
  const T beta = go.beta;
  const bool rec_old = kRec && !go.first;
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
    // the recurrence mode's y, p (and z) at this layer's owned node, issued
    // before the prefetches so that their wait does not drain them (loading
    // them a layer ahead too costs registers: spills at 4 waves per SIMD,
    // measured slower, as is 3 waves per SIMD)
    if (kRec && w.node_ok && L >= w.k0) {
      const long n = w.node(g, L);
      if (rec_old) {
        yc = y[n];
        pc = p[n];
      }
      if (z_own) zc = v[n];
    }
    // prefetch the next top face, the next layer's data and the next flag
    if (w.col_ok && L1 <= w.Lend && L1 + 1 <= g.nz - 1) face(L1 + 1, fn);
    if (w.col_ok && L1 <= w.Lend && L1 <= g.nz - 2) {
      const long sl = w.slot(L1);
      en = eps_t[sl];
      if ((sbits >> (L1 - w.Lbeg)) & 1u) load8(cq + 8 * sl, cn);
    }
    if (kPlain && w.node_ok && L1 <= w.Lend) mkn = mask[w.node(g, L1)];
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
      if (kRec) {
        const T zo = w.col_ok ? fb[3] : zc;   // z at the owned node (gi, gj, L)
        T pv = zo;
        if (rec_old) {
          val += beta * yc;
          pv += beta * pc;
        }
        p[n] = pv;
        dot += (double)pv * (double)val;
      }
      if (kPlain && mk && identity_rows) val = identity_rows == 1 ? v[n] : T(0);
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
  }
  return true;
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
      double zero[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) zero[k] = 0.0;
      jv_element(ve, sx, sy, sz, zero, false, outF);          // eps Khat phi
      const double dg = (sx + sy + sz) * (1.0 / 9.0);
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
          // predictor-corrector electrons: |psi_i|^2 and phi^(k) interpolated
          // to the Gauss points like phi
          const long b0 = w.n00 + w.sxy * L;
          const long o[8] = {0, 1, g.nx, g.nx + 1, w.sxy, w.sxy + 1, w.sxy + g.nx, w.sxy + g.nx + 1};
          double dph[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) dph[k] = qm->phik[b0 + o[k]];
          gauss_interp(dph);
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            dph[q] = src[q] - dph[q];
            nq[q] = dnq[q] = 0.0;
          }
          for (int i = 0; i < qm->n; ++i) {
            double s2[8];
            const double* ps = qm->psi2 + qm->N * i + b0;
#pragma unroll
            for (int k = 0; k < 8; ++k) s2[k] = ps[o[k]];
            gauss_interp(s2);
            const double Ei = qm->E[i];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              double G, dG;
              pc_occupation(qm->conf, (dph[q] - Ei) * qm->inv_kT, G, dG);
              nq[q] += qm->pref * s2[q] * G;
              dnq[q] += qm->pref * s2[q] * dG * qm->inv_kT;
            }
          }
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
