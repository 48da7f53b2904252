// HIP kernels (gfx950) of the Q1 nonlinear-Poisson Newton-Krylov path.
//
// Element sweeps (residual, J.v, adjoint) share one tiling.  A block of 256
// threads owns a 16 x 16 column of nodes over kz node planes.  It marches up
// the planes; at each element layer it stages the next node plane of the
// input field in LDS (with a one-node halo), computes the (16+1) x (16+1)
// elements that touch its nodes (the halo column is recomputed by the
// neighbouring tile), writes each element's 8 corner contributions to LDS and
// lets every owned node gather its 4 + 4 contributions from the elements
// below and above it.  There are no atomics: every nodal sum is formed in a
// fixed order, so results are bitwise reproducible.
#include "qe_kernels.h"

namespace qe {

// ---------------------------------------------------------------------------
// helpers for the element sweeps
template <typename T, typename Load>
__device__ __forceinline__ void stage_plane(T* dst, int P, int i0, int j0, const Geom& g, Load load) {
  if (P < 0 || P >= g.nz) return;
  for (int s = threadIdx.x; s < kNNL; s += kThreads) {
    const int la = s % kNXL, lb = s / kNXL;
    const int gi = i0 - 1 + la, gj = j0 - 1 + lb;
    T val = T(0);
    if (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny)
      val = load((long)gi + (long)g.nx * ((long)gj + (long)g.ny * P));
    dst[s] = val;
  }
}

template <typename T>
__device__ __forceinline__ void corners(const T* p0, const T* p1, int ea, int eb, T ve[8]) {
  const int s = eb * kNXL + ea;
  ve[0] = p0[s];
  ve[1] = p0[s + 1];
  ve[2] = p0[s + kNXL];
  ve[3] = p0[s + kNXL + 1];
  ve[4] = p1[s];
  ve[5] = p1[s + 1];
  ve[6] = p1[s + kNXL];
  ve[7] = p1[s + kNXL + 1];
}

// Sums the four bottom (plane L) and four top (plane L+1) contributions of
// layer L at owned node (na, nb).
template <typename T>
__device__ __forceinline__ void gather4(T (*so)[kNEL], int na, int nb, T& bot, T& top) {
  const int e = nb * kEX + na;
  bot = so[3][e] + so[2][e + 1] + so[1][e + kEX] + so[0][e + kEX + 1];
  top = so[7][e] + so[6][e + 1] + so[5][e + kEX] + so[4][e + kEX + 1];
}

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

__device__ __forceinline__ long elem_index(const Geom& g, int ex, int ey, int ez) {
  return (long)ex + (long)(g.nx - 1) * ((long)ey + (long)(g.ny - 1) * ez);
}

// ---------------------------------------------------------------------------
// Residual F(phi + lam*delta), Jacobi diagonal and per-Gauss-point charge
// linearisation c_q = KAPPA semi W n'(phi_q) (written once per element, by the
// tile that owns it).  Also ||F_free||^2 (last block).
template <typename TD>
__global__ __launch_bounds__(kThreads) void k_residual(
    Geom g, TileMap tm, Charge ch, const double* __restrict__ eps, const uint8_t* __restrict__ semi,
    const double* __restrict__ netdop, const uint8_t* __restrict__ mask, const double* __restrict__ phi,
    const TD* __restrict__ delta, double lam, double* __restrict__ F, double* __restrict__ invdiag,
    double* __restrict__ diag_out, double* __restrict__ cq, float* __restrict__ cq32,
    float* __restrict__ invdiag32, double* __restrict__ partial, unsigned int* counter,
    double* __restrict__ norm2) {
  __shared__ double sv[2][kNNL];
  __shared__ double sF[8][kNEL];
  __shared__ double sD[8][kNEL];
  __shared__ double sred[kThreads / 64];
  int tx, ty, tz;
  tile_of_block(blockIdx.x, tm, tx, ty, tz);
  const int i0 = tx * kTX, j0 = ty * kTY, k0 = tz * tm.kz;
  const int t = threadIdx.x;
  const int na = t % kTX, nb = t / kTX;
  const int gi = i0 + na, gj = j0 + nb;
  const bool node_ok = gi < g.nx && gj < g.ny;
  auto ld = [&](long n) -> double {
    double v = phi[n];
    if (delta) v += lam * (double)delta[n];
    return v;
  };
  double carryF = 0.0, carryD = 0.0, acc = 0.0;
  const int Lend = min(k0 + tm.kz - 1, g.nz - 1);
  stage_plane(sv[(k0 - 1) & 1], k0 - 1, i0, j0, g, ld);
  for (int L = k0 - 1; L <= Lend; ++L) {
    stage_plane(sv[(L + 1) & 1], L + 1, i0, j0, g, ld);
    __syncthreads();
    const bool layer_ok = (L >= 0 && L <= g.nz - 2);
    if (layer_ok) {
      const double hz = g.z[L + 1] - g.z[L];
      for (int e = t; e < kNEL; e += kThreads) {
        const int ea = e % kEX, eb = e / kEX;
        const int ex = i0 - 1 + ea, ey = j0 - 1 + eb;
        double outF[8], outD[8];
        if (ex >= 0 && ex < g.nx - 1 && ey >= 0 && ey < g.ny - 1) {
          const long el = elem_index(g, ex, ey, L);
          const bool owned = (ea >= 1 && eb >= 1 && L >= k0);
          const double hx = g.x[ex + 1] - g.x[ex], hy = g.y[ey + 1] - g.y[ey];
          const double ee = eps[el];
          const double sx = ee * hy * hz / hx, sy = ee * hx * hz / hy, sz = ee * hx * hy / hz;
          double ve[8];
          corners(sv[L & 1], sv[(L + 1) & 1], ea, eb, ve);
          stiff_apply(ve, sx, sy, sz, outF);
          const double dg = (sx + sy + sz) * (1.0 / 9.0);
#pragma unroll
          for (int k = 0; k < 8; ++k) outD[k] = dg;
          if (semi[el]) {
            const double kw = ch.kappa * hx * hy * hz * 0.125;
            const double nd = netdop ? netdop[el] : 0.0;
            double src[8], cc[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) src[k] = ve[k];
            gauss_interp(src);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              double n, dn;
              electron_density(ch, src[q], n, dn);
              src[q] = kw * (nd - n);
              cc[q] = kw * dn;
            }
            if (owned) {
              store8(cq + 8 * el, cc);
              if (cq32) store8(cq32 + 8 * el, cc);
            }
            gauss_interp(src);
            gauss_sq_project(cc);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              outF[k] -= src[k];
              outD[k] += cc[k];
            }
          }
        } else {
#pragma unroll
          for (int k = 0; k < 8; ++k) outF[k] = outD[k] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          sF[k][e] = outF[k];
          sD[k][e] = outD[k];
        }
      }
    }
    __syncthreads();
    if (node_ok) {
      double bF = 0.0, tF = 0.0, bD = 0.0, tD = 0.0;
      if (layer_ok) {
        gather4(sF, na, nb, bF, tF);
        gather4(sD, na, nb, bD, tD);
      }
      if (L >= k0) {
        const long n = (long)gi + (long)g.nx * ((long)gj + (long)g.ny * L);
        double f = carryF + bF, d = carryD + bD;
        if (mask[n]) {
          f = 0.0;
          d = 1.0;
        }
        F[n] = f;
        const double id = 1.0 / d;
        invdiag[n] = id;
        if (diag_out) diag_out[n] = d;
        if (invdiag32) invdiag32[n] = (float)id;
        acc += f * f;
      }
      carryF = tF;
      carryD = tD;
    }
  }
  const double s = block_sum(acc, sred);
  if (t == 0) partial[blockIdx.x] = s;
  if (last_block_done(counter)) {
    const double tot = reduce_partials(partial, gridDim.x, sred);
    if (t == 0) {
      *norm2 = tot;
      *counter = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// y = J v (masked).  With kPcg the block also forms p^T J p and the last
// block sets alpha = r^T z / p^T J p (or flags a breakdown).
template <typename T, bool kPcg>
__global__ __launch_bounds__(kThreads) void k_jv(
    Geom g, TileMap tm, const T* __restrict__ eps, const uint8_t* __restrict__ semi,
    const T* __restrict__ cq, const uint8_t* __restrict__ mask, const T* __restrict__ v,
    T* __restrict__ y, int identity_rows, PcgCtx* ctx, double* __restrict__ partial) {
  if (kPcg && ctx->done) return;
  __shared__ T sv[2][kNNL];
  __shared__ T so[8][kNEL];
  __shared__ double sred[kThreads / 64];
  int tx, ty, tz;
  tile_of_block(blockIdx.x, tm, tx, ty, tz);
  const int i0 = tx * kTX, j0 = ty * kTY, k0 = tz * tm.kz;
  const int t = threadIdx.x;
  const int na = t % kTX, nb = t / kTX;
  const int gi = i0 + na, gj = j0 + nb;
  const bool node_ok = gi < g.nx && gj < g.ny;
  auto ld = [&](long n) -> T { return mask[n] ? T(0) : v[n]; };
  T carry = T(0);
  double dot = 0.0;
  const int Lend = min(k0 + tm.kz - 1, g.nz - 1);
  stage_plane(sv[(k0 - 1) & 1], k0 - 1, i0, j0, g, ld);
  for (int L = k0 - 1; L <= Lend; ++L) {
    stage_plane(sv[(L + 1) & 1], L + 1, i0, j0, g, ld);
    __syncthreads();
    const bool layer_ok = (L >= 0 && L <= g.nz - 2);
    if (layer_ok) {
      const double hz = g.z[L + 1] - g.z[L];
      for (int e = t; e < kNEL; e += kThreads) {
        const int ea = e % kEX, eb = e / kEX;
        const int ex = i0 - 1 + ea, ey = j0 - 1 + eb;
        T out[8];
        if (ex >= 0 && ex < g.nx - 1 && ey >= 0 && ey < g.ny - 1) {
          const long el = elem_index(g, ex, ey, L);
          const double hx = g.x[ex + 1] - g.x[ex], hy = g.y[ey + 1] - g.y[ey];
          const T ee = eps[el];
          const T sx = ee * T(hy * hz / hx), sy = ee * T(hx * hz / hy), sz = ee * T(hx * hy / hz);
          T ve[8];
          corners(sv[L & 1], sv[(L + 1) & 1], ea, eb, ve);
          stiff_apply(ve, sx, sy, sz, out);
          if (semi[el]) {
            T c8[8];
            load8(cq + 8 * el, c8);
            gauss_interp(ve);
#pragma unroll
            for (int q = 0; q < 8; ++q) ve[q] *= c8[q];
            gauss_interp(ve);
#pragma unroll
            for (int k = 0; k < 8; ++k) out[k] += ve[k];
          }
        } else {
#pragma unroll
          for (int k = 0; k < 8; ++k) out[k] = T(0);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) so[k][e] = out[k];
      }
    }
    __syncthreads();
    if (node_ok) {
      T bot = T(0), top = T(0);
      if (layer_ok) gather4(so, na, nb, bot, top);
      if (L >= k0) {
        const long n = (long)gi + (long)g.nx * ((long)gj + (long)g.ny * L);
        T val = carry + bot;
        if (mask[n]) {
          if (identity_rows) val = v[n];
        } else if (kPcg) {
          dot += (double)sv[L & 1][(nb + 1) * kNXL + na + 1] * (double)val;
        }
        y[n] = val;
      }
      carry = top;
    }
  }
  if (kPcg) {
    const double s = block_sum(dot, sred);
    if (t == 0) partial[blockIdx.x] = s;
    if (last_block_done(&ctx->cnt_jv)) {
      const double pAp = reduce_partials(partial, gridDim.x, sred);
      if (t == 0) {
        ctx->pAp = pAp;
        if (!(pAp > 0.0) || !isfinite(pAp)) {
          ctx->done = 1;
          ctx->status = PCG_BREAKDOWN;
          ctx->alpha = 0.0;
        } else {
          ctx->alpha = ctx->rz / pAp;
        }
        ctx->cnt_jv = 0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint right-hand side g = dQ/dphi (all nodes) and Q = electrons in the box.
__global__ __launch_bounds__(kThreads) void k_adj_rhs(
    Geom g, TileMap tm, Charge ch, Box box, const uint8_t* __restrict__ semi,
    const double* __restrict__ phi, double* __restrict__ gvec, double* __restrict__ partial,
    unsigned int* counter, double* __restrict__ Qout) {
  __shared__ double sv[2][kNNL];
  __shared__ double so[8][kNEL];
  __shared__ double sred[kThreads / 64];
  int tx, ty, tz;
  tile_of_block(blockIdx.x, tm, tx, ty, tz);
  const int i0 = tx * kTX, j0 = ty * kTY, k0 = tz * tm.kz;
  const int t = threadIdx.x;
  const int na = t % kTX, nb = t / kTX;
  const int gi = i0 + na, gj = j0 + nb;
  const bool node_ok = gi < g.nx && gj < g.ny;
  auto ld = [&](long n) -> double { return phi[n]; };
  double carry = 0.0, qacc = 0.0;
  const int Lend = min(k0 + tm.kz - 1, g.nz - 1);
  stage_plane(sv[(k0 - 1) & 1], k0 - 1, i0, j0, g, ld);
  for (int L = k0 - 1; L <= Lend; ++L) {
    stage_plane(sv[(L + 1) & 1], L + 1, i0, j0, g, ld);
    __syncthreads();
    const bool layer_ok = (L >= 0 && L <= g.nz - 2);
    if (layer_ok) {
      const double zc = 0.5 * (g.z[L + 1] + g.z[L]), hz = g.z[L + 1] - g.z[L];
      for (int e = t; e < kNEL; e += kThreads) {
        const int ea = e % kEX, eb = e / kEX;
        const int ex = i0 - 1 + ea, ey = j0 - 1 + eb;
        double out[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) out[k] = 0.0;
        if (ex >= 0 && ex < g.nx - 1 && ey >= 0 && ey < g.ny - 1) {
          const long el = elem_index(g, ex, ey, L);
          const double xc = 0.5 * (g.x[ex + 1] + g.x[ex]), yc = 0.5 * (g.y[ey + 1] + g.y[ey]);
          if (semi[el] && box.contains(xc, yc, zc)) {
            const double W = (g.x[ex + 1] - g.x[ex]) * (g.y[ey + 1] - g.y[ey]) * hz * 0.125;
            corners(sv[L & 1], sv[(L + 1) & 1], ea, eb, out);
            gauss_interp(out);
            double qs = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              double n, dn;
              electron_density(ch, out[q], n, dn);
              qs += n;
              out[q] = W * dn;
            }
            if (ea >= 1 && eb >= 1 && L >= k0) qacc += W * qs;
            gauss_interp(out);
          }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) so[k][e] = out[k];
      }
    }
    __syncthreads();
    if (node_ok) {
      double bot = 0.0, top = 0.0;
      if (layer_ok) gather4(so, na, nb, bot, top);
      if (L >= k0) gvec[(long)gi + (long)g.nx * ((long)gj + (long)g.ny * L)] = carry + bot;
      carry = top;
    }
  }
  const double s = block_sum(qacc, sred);
  if (t == 0) partial[blockIdx.x] = s;
  if (last_block_done(counter)) {
    const double tot = reduce_partials(partial, gridDim.x, sred);
    if (t == 0) {
      *Qout = tot;
      *counter = 0;
    }
  }
}

// Adjoint gradients: dQ/deps_e = -lam_e^T Khat_e phi_e for owned elements and
// tcon_i = g_i - (J lam)_i on Dirichlet nodes (0 on free nodes); lam is zero
// on Dirichlet nodes.
__global__ __launch_bounds__(kThreads) void k_adj_grad(
    Geom g, TileMap tm, const double* __restrict__ eps, const uint8_t* __restrict__ semi,
    const double* __restrict__ cq, const uint8_t* __restrict__ mask, const double* __restrict__ lam,
    const double* __restrict__ phi, const double* __restrict__ gvec, double* __restrict__ dQdeps,
    double* __restrict__ tcon) {
  __shared__ double sl[2][kNNL];
  __shared__ double sp[2][kNNL];
  __shared__ double so[8][kNEL];
  int tx, ty, tz;
  tile_of_block(blockIdx.x, tm, tx, ty, tz);
  const int i0 = tx * kTX, j0 = ty * kTY, k0 = tz * tm.kz;
  const int t = threadIdx.x;
  const int na = t % kTX, nb = t / kTX;
  const int gi = i0 + na, gj = j0 + nb;
  const bool node_ok = gi < g.nx && gj < g.ny;
  auto ldl = [&](long n) -> double { return mask[n] ? 0.0 : lam[n]; };
  auto ldp = [&](long n) -> double { return phi[n]; };
  double carry = 0.0;
  const int Lend = min(k0 + tm.kz - 1, g.nz - 1);
  stage_plane(sl[(k0 - 1) & 1], k0 - 1, i0, j0, g, ldl);
  stage_plane(sp[(k0 - 1) & 1], k0 - 1, i0, j0, g, ldp);
  for (int L = k0 - 1; L <= Lend; ++L) {
    stage_plane(sl[(L + 1) & 1], L + 1, i0, j0, g, ldl);
    stage_plane(sp[(L + 1) & 1], L + 1, i0, j0, g, ldp);
    __syncthreads();
    const bool layer_ok = (L >= 0 && L <= g.nz - 2);
    if (layer_ok) {
      const double hz = g.z[L + 1] - g.z[L];
      for (int e = t; e < kNEL; e += kThreads) {
        const int ea = e % kEX, eb = e / kEX;
        const int ex = i0 - 1 + ea, ey = j0 - 1 + eb;
        double out[8];
        if (ex >= 0 && ex < g.nx - 1 && ey >= 0 && ey < g.ny - 1) {
          const long el = elem_index(g, ex, ey, L);
          const double hx = g.x[ex + 1] - g.x[ex], hy = g.y[ey + 1] - g.y[ey];
          const double ux = hy * hz / hx, uy = hx * hz / hy, uz = hx * hy / hz;
          double le[8], pe[8], kp[8];
          corners(sl[L & 1], sl[(L + 1) & 1], ea, eb, le);
          if (ea >= 1 && eb >= 1 && L >= k0) {
            corners(sp[L & 1], sp[(L + 1) & 1], ea, eb, pe);
            stiff_apply(pe, ux, uy, uz, kp);
            double d = 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) d += le[k] * kp[k];
            dQdeps[el] = -d;
          }
          const double ee = eps[el];
          stiff_apply(le, ee * ux, ee * uy, ee * uz, out);
          if (semi[el]) {
            double c8[8];
            load8(cq + 8 * el, c8);
            gauss_interp(le);
#pragma unroll
            for (int q = 0; q < 8; ++q) le[q] *= c8[q];
            gauss_interp(le);
#pragma unroll
            for (int k = 0; k < 8; ++k) out[k] += le[k];
          }
        } else {
#pragma unroll
          for (int k = 0; k < 8; ++k) out[k] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) so[k][e] = out[k];
      }
    }
    __syncthreads();
    if (node_ok) {
      double bot = 0.0, top = 0.0;
      if (layer_ok) gather4(so, na, nb, bot, top);
      if (L >= k0) {
        const long n = (long)gi + (long)g.nx * ((long)gj + (long)g.ny * L);
        tcon[n] = mask[n] ? gvec[n] - (carry + bot) : 0.0;
      }
      carry = top;
    }
  }
}

// Per-contact sums of tcon (fixed order).  Grid-stride over nodes; partial
// layout [block][contact].
__global__ __launch_bounds__(kVecThreads) void k_contact_sum(
    long N, int n_dir, const int32_t* __restrict__ dir_id, const double* __restrict__ tcon,
    double* __restrict__ partial, unsigned int* counter, double* __restrict__ out) {
  __shared__ double sred[kVecThreads / 64];
  for (int c = 0; c < n_dir; ++c) {
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
      if (dir_id[i] == c) acc += tcon[i];
    const double s = block_sum(acc, sred);
    if (threadIdx.x == 0) partial[(long)blockIdx.x * n_dir + c] = s;
  }
  if (last_block_done(counter)) {
    for (int c = 0; c < n_dir; ++c) {
      double acc = 0.0;
      const volatile double* p = partial;
      for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) acc += p[(long)b * n_dir + c];
      const double s = block_sum(acc, sred);
      if (threadIdx.x == 0) out[c] = s;
    }
    if (threadIdx.x == 0) *counter = 0;
  }
}

// ---------------------------------------------------------------------------
// Electron counts in up to kMaxBoxes boxes; one grid-stride pass over elements.
__global__ __launch_bounds__(kVecThreads) void k_count(
    Geom g, Charge ch, BoxSet boxes, const uint8_t* __restrict__ semi, const double* __restrict__ phi,
    double* __restrict__ partial, unsigned int* counter, double* __restrict__ out) {
  __shared__ double sred[kVecThreads / 64];
  double acc[kMaxBoxes];
#pragma unroll
  for (int r = 0; r < kMaxBoxes; ++r) acc[r] = 0.0;
  const long ex = g.nx - 1, ey = g.ny - 1;
  const long E = ex * ey * (g.nz - 1);
  for (long el = (long)blockIdx.x * blockDim.x + threadIdx.x; el < E; el += (long)gridDim.x * blockDim.x) {
    if (!semi[el]) continue;
    const int i = (int)(el % ex);
    const int j = (int)((el / ex) % ey);
    const int k = (int)(el / (ex * ey));
    const double xc = 0.5 * (g.x[i] + g.x[i + 1]), yc = 0.5 * (g.y[j] + g.y[j + 1]),
                 zc = 0.5 * (g.z[k] + g.z[k + 1]);
    bool any = false;
    for (int r = 0; r < boxes.n; ++r) any |= boxes.b[r].contains(xc, yc, zc);
    if (!any) continue;
    double ve[8];
    const long n0 = (long)i + (long)g.nx * ((long)j + (long)g.ny * k);
    const long sy = g.nx, sz = (long)g.nx * g.ny;
    ve[0] = phi[n0];
    ve[1] = phi[n0 + 1];
    ve[2] = phi[n0 + sy];
    ve[3] = phi[n0 + sy + 1];
    ve[4] = phi[n0 + sz];
    ve[5] = phi[n0 + sz + 1];
    ve[6] = phi[n0 + sz + sy];
    ve[7] = phi[n0 + sz + sy + 1];
    gauss_interp(ve);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += electron_density_only(ch, ve[q]);
    s *= (g.x[i + 1] - g.x[i]) * (g.y[j + 1] - g.y[j]) * (g.z[k + 1] - g.z[k]) * 0.125;
    for (int r = 0; r < boxes.n; ++r)
      if (boxes.b[r].contains(xc, yc, zc)) acc[r] += s;
  }
  for (int r = 0; r < boxes.n; ++r) {
    const double s = block_sum(acc[r], sred);
    if (threadIdx.x == 0) partial[(long)blockIdx.x * boxes.n + r] = s;
  }
  if (last_block_done(counter)) {
    for (int r = 0; r < boxes.n; ++r) {
      double a = 0.0;
      const volatile double* p = partial;
      for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) a += p[(long)b * boxes.n + r];
      const double s = block_sum(a, sred);
      if (threadIdx.x == 0) out[r] = s;
    }
    if (threadIdx.x == 0) *counter = 0;
  }
}

// Nodal density: n(phi_i) if node i touches a semiconductor element, else 0.
__global__ __launch_bounds__(kVecThreads) void k_density(Geom g, Charge ch, const uint8_t* __restrict__ semi,
                                                        const double* __restrict__ phi, double* __restrict__ nout) {
  const long N = (long)g.nx * g.ny * g.nz;
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    const int i = (int)(n % g.nx);
    const int j = (int)((n / g.nx) % g.ny);
    const int k = (int)(n / ((long)g.nx * g.ny));
    bool touch = false;
    for (int dk = -1; dk <= 0; ++dk)
      for (int dj = -1; dj <= 0; ++dj)
        for (int di = -1; di <= 0; ++di) {
          const int ei = i + di, ej = j + dj, ek = k + dk;
          if (ei >= 0 && ei < g.nx - 1 && ej >= 0 && ej < g.ny - 1 && ek >= 0 && ek < g.nz - 1)
            touch |= semi[elem_index(g, ei, ej, ek)] != 0;
        }
    nout[n] = touch ? electron_density_only(ch, phi[n]) : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Input validation.  Sets bits of *flags: 1 eps not finite/positive,
// 2 net doping not finite, 4 dir_id out of range, 8 phi not finite.
__global__ __launch_bounds__(kVecThreads) void k_validate(long N, long E, int n_dir, const double* __restrict__ eps,
                                                         const double* __restrict__ netdop,
                                                         const int32_t* __restrict__ dir_id,
                                                         const double* __restrict__ phi, int* flags) {
  int f = 0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (long)gridDim.x * blockDim.x) {
    const double v = eps[e];
    if (!(v > 0.0) || !isfinite(v)) f |= 1;
    if (netdop && !isfinite(netdop[e])) f |= 2;
  }
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    const int d = dir_id[n];
    if (d < -1 || d >= n_dir) f |= 4;
    if (phi && !isfinite(phi[n])) f |= 8;
  }
  if (f) atomicOr(flags, f);
}

// mask[i] = node i is Dirichlet.  Optionally sets phi on Dirichlet nodes to
// its value and (zero_free) free nodes to 0.
__global__ __launch_bounds__(kVecThreads) void k_stage(long N, const int32_t* __restrict__ dir_id,
                                                      const double* __restrict__ dir_val, uint8_t* __restrict__ mask,
                                                      double* __restrict__ phi, int apply, int zero_free) {
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    const int d = dir_id[n];
    mask[n] = d >= 0 ? 1 : 0;
    if (apply) {
      if (d >= 0)
        phi[n] = dir_val[d];
      else if (zero_free)
        phi[n] = 0.0;
    }
  }
}

template <typename TS, typename TD>
__global__ __launch_bounds__(kVecThreads) void k_cast(long n, const TS* __restrict__ a, TD* __restrict__ b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = (TD)a[i];
}

// phi += lam * delta
template <typename TD>
__global__ __launch_bounds__(kVecThreads) void k_axpy_phi(long N, double* __restrict__ phi,
                                                         const TD* __restrict__ delta, double lam) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
    phi[i] += lam * (double)delta[i];
}

// ---------------------------------------------------------------------------
// Jacobi-preconditioned CG, scalars kept on the device in PcgCtx.
// init: x = 0, r = sign*b on free nodes, p = z = D^-1 r; rz, rr0, tol2.
template <typename T, typename TB>
__global__ __launch_bounds__(kVecThreads) void k_pcg_init(long N, double sign, const TB* __restrict__ b,
                                                         const uint8_t* __restrict__ mask,
                                                         const T* __restrict__ invdiag, T* __restrict__ x,
                                                         T* __restrict__ r, T* __restrict__ p, PcgCtx* ctx,
                                                         double* __restrict__ partial, double rtol) {
  __shared__ double sred[kVecThreads / 64];
  double rz = 0.0, rr = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
    const T ri = mask[i] ? T(0) : (T)(sign * (double)b[i]);
    const T zi = invdiag[i] * ri;
    x[i] = T(0);
    r[i] = ri;
    p[i] = zi;
    rz += (double)ri * (double)zi;
    rr += (double)ri * (double)ri;
  }
  const double s1 = block_sum(rz, sred);
  const double s2 = block_sum(rr, sred);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s1;
    partial[2 * blockIdx.x + 1] = s2;
  }
  if (last_block_done(&ctx->cnt_init)) {
    double a = 0.0, c = 0.0;
    const volatile double* pp = partial;
    for (int k = threadIdx.x; k < (int)gridDim.x; k += blockDim.x) {
      a += pp[2 * k];
      c += pp[2 * k + 1];
    }
    const double RZ = block_sum(a, sred);
    const double RR = block_sum(c, sred);
    if (threadIdx.x == 0) {
      ctx->rz = RZ;
      ctx->rr = RR;
      ctx->rr0 = RR;
      ctx->tol2 = rtol * rtol * RR;
      ctx->iters = 0;
      ctx->alpha = ctx->beta = 0.0;
      if (!isfinite(RR) || !isfinite(RZ)) {
        ctx->done = 1;
        ctx->status = PCG_NONFINITE;
      } else if (RR == 0.0) {
        ctx->done = 1;
        ctx->status = PCG_CONVERGED;
      } else {
        ctx->done = 0;
        ctx->status = PCG_RUNNING;
      }
      ctx->cnt_init = 0;
    }
  }
}

// x += alpha p; r -= alpha y; then rz_new = r^T D^-1 r, rr = r^T r; the last
// block sets beta and decides convergence.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_pcg_update(long N, T* __restrict__ x, T* __restrict__ r,
                                                           const T* __restrict__ p, const T* __restrict__ y,
                                                           const T* __restrict__ invdiag, PcgCtx* ctx,
                                                           double* __restrict__ partial) {
  if (ctx->done) return;
  __shared__ double sred[kVecThreads / 64];
  const T alpha = (T)ctx->alpha;
  double rz = 0.0, rr = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * y[i];
    r[i] = ri;
    const T zi = invdiag[i] * ri;
    rz += (double)ri * (double)zi;
    rr += (double)ri * (double)ri;
  }
  const double s1 = block_sum(rz, sred);
  const double s2 = block_sum(rr, sred);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s1;
    partial[2 * blockIdx.x + 1] = s2;
  }
  if (last_block_done(&ctx->cnt_upd)) {
    double a = 0.0, c = 0.0;
    const volatile double* pp = partial;
    for (int k = threadIdx.x; k < (int)gridDim.x; k += blockDim.x) {
      a += pp[2 * k];
      c += pp[2 * k + 1];
    }
    const double RZ = block_sum(a, sred);
    const double RR = block_sum(c, sred);
    if (threadIdx.x == 0) {
      ctx->beta = RZ / ctx->rz;
      ctx->rz = RZ;
      ctx->rr = RR;
      ctx->iters += 1;
      if (!isfinite(RR) || !isfinite(RZ)) {
        ctx->done = 1;
        ctx->status = PCG_NONFINITE;
      } else if (RR <= ctx->tol2) {
        ctx->done = 1;
        ctx->status = PCG_CONVERGED;
      } else if (ctx->iters >= ctx->maxit) {
        ctx->done = 1;
        ctx->status = PCG_MAXIT;
      }
      ctx->cnt_upd = 0;
    }
  }
}

// p = D^-1 r + beta p
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_pcg_dir(long N, const T* __restrict__ r,
                                                        const T* __restrict__ invdiag, T* __restrict__ p,
                                                        const PcgCtx* ctx) {
  if (ctx->done) return;
  const T beta = (T)ctx->beta;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
    p[i] = invdiag[i] * r[i] + beta * p[i];
}

// ---------------------------------------------------------------------------
// Launchers (host side, same translation unit so the templates instantiate).
#define QE_LAUNCH(kernel, grid, block, stream, ...) \
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, (hipStream_t)(stream), __VA_ARGS__)

void launch_residual(hipStream_t s, const Geom& g, const TileMap& tm, const Charge& ch, const double* eps,
                     const uint8_t* semi, const double* netdop, const uint8_t* mask, const double* phi,
                     const double* delta64, const float* delta32, double lam, double* F, double* invdiag,
                     double* diag_out, double* cq, float* cq32, float* invdiag32, double* partial,
                     unsigned int* counter, double* norm2) {
  if (delta32)
    QE_LAUNCH(k_residual<float>, tm.nblocks, kThreads, s, g, tm, ch, eps, semi, netdop, mask, phi, delta32, lam, F,
              invdiag, diag_out, cq, cq32, invdiag32, partial, counter, norm2);
  else
    QE_LAUNCH(k_residual<double>, tm.nblocks, kThreads, s, g, tm, ch, eps, semi, netdop, mask, phi, delta64, lam, F,
              invdiag, diag_out, cq, cq32, invdiag32, partial, counter, norm2);
}

void launch_jv64(hipStream_t s, const Geom& g, const TileMap& tm, const double* eps, const uint8_t* semi,
                 const double* cq, const uint8_t* mask, const double* v, double* y, int identity_rows, PcgCtx* ctx,
                 double* partial) {
  if (ctx)
    QE_LAUNCH((k_jv<double, true>), tm.nblocks, kThreads, s, g, tm, eps, semi, cq, mask, v, y, identity_rows, ctx,
              partial);
  else
    QE_LAUNCH((k_jv<double, false>), tm.nblocks, kThreads, s, g, tm, eps, semi, cq, mask, v, y, identity_rows, ctx,
              partial);
}

void launch_jv32(hipStream_t s, const Geom& g, const TileMap& tm, const float* eps, const uint8_t* semi,
                 const float* cq, const uint8_t* mask, const float* v, float* y, int identity_rows, PcgCtx* ctx,
                 double* partial) {
  if (ctx)
    QE_LAUNCH((k_jv<float, true>), tm.nblocks, kThreads, s, g, tm, eps, semi, cq, mask, v, y, identity_rows, ctx,
              partial);
  else
    QE_LAUNCH((k_jv<float, false>), tm.nblocks, kThreads, s, g, tm, eps, semi, cq, mask, v, y, identity_rows, ctx,
              partial);
}

void launch_adj_rhs(hipStream_t s, const Geom& g, const TileMap& tm, const Charge& ch, const Box& box,
                    const uint8_t* semi, const double* phi, double* gvec, double* partial, unsigned int* counter,
                    double* Q) {
  QE_LAUNCH(k_adj_rhs, tm.nblocks, kThreads, s, g, tm, ch, box, semi, phi, gvec, partial, counter, Q);
}

void launch_adj_grad(hipStream_t s, const Geom& g, const TileMap& tm, const double* eps, const uint8_t* semi,
                     const double* cq, const uint8_t* mask, const double* lam, const double* phi,
                     const double* gvec, double* dQdeps, double* tcon) {
  QE_LAUNCH(k_adj_grad, tm.nblocks, kThreads, s, g, tm, eps, semi, cq, mask, lam, phi, gvec, dQdeps, tcon);
}

void launch_contact_sum(hipStream_t s, int nblocks, long N, int n_dir, const int32_t* dir_id, const double* tcon,
                        double* partial, unsigned int* counter, double* out) {
  QE_LAUNCH(k_contact_sum, nblocks, kVecThreads, s, N, n_dir, dir_id, tcon, partial, counter, out);
}

void launch_count(hipStream_t s, int nblocks, const Geom& g, const Charge& ch, const BoxSet& boxes,
                  const uint8_t* semi, const double* phi, double* partial, unsigned int* counter, double* out) {
  QE_LAUNCH(k_count, nblocks, kVecThreads, s, g, ch, boxes, semi, phi, partial, counter, out);
}

void launch_density(hipStream_t s, int nblocks, const Geom& g, const Charge& ch, const uint8_t* semi,
                    const double* phi, double* nout) {
  QE_LAUNCH(k_density, nblocks, kVecThreads, s, g, ch, semi, phi, nout);
}

void launch_validate(hipStream_t s, int nblocks, long N, long E, int n_dir, const double* eps, const double* netdop,
                     const int32_t* dir_id, const double* phi, int* flags) {
  QE_LAUNCH(k_validate, nblocks, kVecThreads, s, N, E, n_dir, eps, netdop, dir_id, phi, flags);
}

void launch_stage(hipStream_t s, int nblocks, long N, const int32_t* dir_id, const double* dir_val, uint8_t* mask,
                  double* phi, int apply, int zero_free) {
  QE_LAUNCH(k_stage, nblocks, kVecThreads, s, N, dir_id, dir_val, mask, phi, apply, zero_free);
}

void launch_cast_d2f(hipStream_t s, int nblocks, long n, const double* a, float* b) {
  QE_LAUNCH((k_cast<double, float>), nblocks, kVecThreads, s, n, a, b);
}

void launch_axpy_phi(hipStream_t s, int nblocks, long N, double* phi, const double* d64, const float* d32,
                     double lam) {
  if (d32)
    QE_LAUNCH(k_axpy_phi<float>, nblocks, kVecThreads, s, N, phi, d32, lam);
  else
    QE_LAUNCH(k_axpy_phi<double>, nblocks, kVecThreads, s, N, phi, d64, lam);
}

void launch_pcg_init64(hipStream_t s, int nblocks, long N, double sign, const double* b, const uint8_t* mask,
                       const double* invdiag, double* x, double* r, double* p, PcgCtx* ctx, double* partial,
                       double rtol) {
  QE_LAUNCH((k_pcg_init<double, double>), nblocks, kVecThreads, s, N, sign, b, mask, invdiag, x, r, p, ctx, partial,
            rtol);
}

void launch_pcg_init32(hipStream_t s, int nblocks, long N, double sign, const double* b, const uint8_t* mask,
                       const float* invdiag, float* x, float* r, float* p, PcgCtx* ctx, double* partial,
                       double rtol) {
  QE_LAUNCH((k_pcg_init<float, double>), nblocks, kVecThreads, s, N, sign, b, mask, invdiag, x, r, p, ctx, partial,
            rtol);
}

void launch_pcg_iter64(hipStream_t s, const Geom& g, const TileMap& tm, int vblocks, long N, const double* eps,
                       const uint8_t* semi, const double* cq, const uint8_t* mask, const double* invdiag, double* x,
                       double* r, double* p, double* y, PcgCtx* ctx, double* partial) {
  QE_LAUNCH((k_jv<double, true>), tm.nblocks, kThreads, s, g, tm, eps, semi, cq, mask, p, y, 1, ctx, partial);
  QE_LAUNCH(k_pcg_update<double>, vblocks, kVecThreads, s, N, x, r, p, y, invdiag, ctx, partial);
  QE_LAUNCH(k_pcg_dir<double>, vblocks, kVecThreads, s, N, r, invdiag, p, ctx);
}

void launch_pcg_iter32(hipStream_t s, const Geom& g, const TileMap& tm, int vblocks, long N, const float* eps,
                       const uint8_t* semi, const float* cq, const uint8_t* mask, const float* invdiag, float* x,
                       float* r, float* p, float* y, PcgCtx* ctx, double* partial) {
  QE_LAUNCH((k_jv<float, true>), tm.nblocks, kThreads, s, g, tm, eps, semi, cq, mask, p, y, 1, ctx, partial);
  QE_LAUNCH(k_pcg_update<float>, vblocks, kVecThreads, s, N, x, r, p, y, invdiag, ctx, partial);
  QE_LAUNCH(k_pcg_dir<float>, vblocks, kVecThreads, s, N, r, invdiag, p, ctx);
}

}  // namespace qe
