// HIP kernels (gfx950) of the Q1 nonlinear-Poisson Newton-Krylov path.
//
// The residual, J.v and CG sweeps run on wave tiles (qe_tiles.h): a wave owns
// a 7 x 7 column of nodes, computes the 8 x 8 elements that touch them while
// it marches up a chunk of node planes, and gathers each owned node's sums
// across lanes, with no LDS and no block barrier.  The adjoint's two
// element sweeps (k_adj_rhs, k_adj_grad) use block tiles instead: 256
// threads own a 16 x 16 column of nodes, stage each node plane of the input
// field in LDS with a one-node halo, compute the 17 x 17 elements around
// their nodes (the halo column is recomputed by the neighbouring tile) and
// gather the 4 + 4 corner contributions of every owned node from LDS.
// There are no atomics in any sweep: every nodal sum is formed in a fixed
// order, so results are bitwise reproducible.
#include "qe_kernels.h"
#include "qe_tiles.h"

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

__device__ __forceinline__ long elem_index(const Geom& g, int ex, int ey, int ez) {
  return (long)ex + (long)(g.nx - 1) * ((long)ey + (long)(g.ny - 1) * ez);
}

// Sum over the block of one value per thread, the same in every thread
// (NT = 0: blockDim.x threads, read from the dispatch packet).
template <int NT = 0>
__device__ __forceinline__ double block_sum_all(double a, double* sred) {
  a = wave_sum(a);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sred[wid] = a;
  __syncthreads();
  double r = 0.0;
  const int nw = ((NT ? NT : (int)blockDim.x) + 63) >> 6;
  for (int w = 0; w < nw; ++w) r += sred[w];
  return r;
}

// Sum of n partials (stride, offset) in a fixed order; the result is the
// same in every thread of the block.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n, int stride, int off,
                                               double* sred) {
  // eight loads in flight per thread before any is added (a load-add loop
  // would wait for each in turn)
  double a = 0.0;
  const int bs = blockDim.x;
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * bs) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (i0 + j * bs < n) ? part[(long)(i0 + j * bs) * stride + off] : 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) a += v[j];
  }
  return block_sum_all(a, sred);
}

// ---------------------------------------------------------------------------
// Wave-tiled kernels: four independent waves per block, one wave tile each
// (see qe_tiles.h).  No LDS and no block barrier in the sweep, so memory
// latency is hidden by the other waves on the SIMD.
__device__ __forceinline__ void wave_coords(const WaveMap& wm, int& wx, int& wy, int& wz, bool& active, int& wid) {
  // wave-uniform (scalar registers): the layer loop, z spacings and tile
  // bounds are then scalar and never wait on vector loads
  const int w = __builtin_amdgcn_readfirstlane(wave_of_block(blockIdx.x, wm) * 4 + (threadIdx.x >> 6));
  wid = w;
  active = w < wm.nwaves;
  wave_tile_of(w, wm, wx, wy, wz);
}

#ifndef QE_JV_MIN_WAVES
#define QE_JV_MIN_WAVES 4
#endif
// y = J v (JV_PLAIN: v read as 0 on Dirichlet nodes, identity_rows optional).
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QE_JV_MIN_WAVES, 8))) void k_jv_wave(
    Geom g, WaveMap wm, const T* __restrict__ eps, const unsigned int* __restrict__ cbits,
    const T* __restrict__ cq, const uint8_t* __restrict__ mask, const T* __restrict__ v,
    T* __restrict__ y, int identity_rows) {
  int wx, wy, wz, wid;
  bool active;
  wave_coords(wm, wx, wy, wz, active, wid);
  const WaveTile w(g, wx, wy, wz, wm.kz, threadIdx.x & 63, active);
  const unsigned int cb = active ? cbits[64L * wid + (threadIdx.x & 63)] : 0u;
  double dot = 0.0;
  jv_tile<T, JV_PLAIN>(g, w, eps, cb, cq, mask, v, y, identity_rows, dot);
}

// Posts a CG decision to host-coherent memory (one vector store, system scope).
__device__ __forceinline__ void post_progress(CgProgress* prog, int iters, int done, int status) {
  __hip_atomic_store(&prog->word, ((iters + 1) << 4) | (status << 1) | done, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
}

// CG iteration k, first kernel.  Once each wave's first loads are in flight,
// the block re-adds the r^T z partials of the previous kernel (rz_k) and
// stops the solve on convergence / non-finite values / the iteration limit
// (block 0 records the decision; every block takes the same one).  Then
// beta = rz_k / rz_{k-1} and, on the wave tiles, y = J z + beta y,
// p = z + beta p and, in FP64, the previous iteration's x += alpha p
// (jv_tile_cg); one p^T y partial per block.  rz_k goes to ctx->rzs[k & 1]
// and rz_{k-1} is read from the other slot.  A stopping kernel stores
// nothing, so the last step x += alpha p is left to k_cg_finish_x.
#ifndef QE_CG_MIN_WAVES
#define QE_CG_MIN_WAVES 3
#endif
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QE_CG_MIN_WAVES, 8))) void k_cg_jv(
    Geom g, WaveMap wm, const T* __restrict__ eps, const unsigned int* __restrict__ cbits,
    const T* __restrict__ cq, const T* __restrict__ z, T* __restrict__ y, T* __restrict__ p, T* __restrict__ x,
    int k, PcgCtx* __restrict__ ctx, CgProgress* __restrict__ prog, const double* __restrict__ part_rz, int n_rz,
    double* __restrict__ part_py) {
  if (ctx->done) return;
  __shared__ double sred[4];
  // the previous kernel's r^T z partials, loaded before anything else so
  // that waiting for them never waits for the sweep's first loads (the
  // block size is the constant 256: reading blockDim.x is a load too)
  constexpr int NT = 256;
  double rz_part[8];
  const bool rz_one = n_rz <= 8 * NT;
#pragma unroll
  for (int j = 0; j < 8; ++j) rz_part[j] = part_rz[min((int)threadIdx.x + j * NT, n_rz - 1)];
  int wx, wy, wz, wid;
  bool active;
  wave_coords(wm, wx, wy, wz, active, wid);
  const WaveTile w(g, wx, wy, wz, wm.kz, threadIdx.x & 63, active);
  // loaded unconditionally: an idle wave reads the last wave's word, which is
  // harmless (its lanes own nothing, read zeros and store nothing)
  const unsigned int cb = cbits[64L * min(wid, wm.nwaves - 1) + (threadIdx.x & 63)];
  int stop_status = PCG_RUNNING, stop_iters = 0;
  double* const sp = sred;
  // pointers captured by value keep their no-alias qualification, so the
  // sweep's z-spacing loads stay scalar
  auto decide = [=, &stop_status, &stop_iters]() -> JvGo<T> {
    double RZ;
    if (rz_one) {
      // the same fixed-order sum as sum_partials
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < 8; ++j) a += ((int)threadIdx.x + j * NT < n_rz) ? rz_part[j] : 0.0;
      RZ = uniform(block_sum_all<NT>(a, sp));
    } else {
      RZ = uniform(sum_partials(part_rz, n_rz, 1, 0, sp));
    }
    const int it = ctx->iters;
    const double rzprev = ctx->rzs[(k + 1) & 1];
    const bool bad = !isfinite(RZ), conv = !bad && RZ <= ctx->tol2, maxed = it >= ctx->maxit;
    const bool first = it == 0;
    const double b = uniform(first ? 0.0 : RZ / rzprev), al = first ? 0.0 : ctx->alpha;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctx->rzs[k & 1] = RZ;
      if (bad) {
        ctx->done = 1;
        ctx->status = PCG_NONFINITE;
      } else if (conv) {
        ctx->done = 1;
        ctx->status = PCG_CONVERGED;
      } else if (maxed) {
        ctx->done = 1;
        ctx->status = PCG_MAXIT;
      } else {
        ctx->beta = b;
      }
    }
    stop_status = bad ? PCG_NONFINITE : conv ? PCG_CONVERGED : PCG_MAXIT;
    stop_iters = it;
    return {!(bad || conv || maxed), (T)b, first, (T)al};
  };
  double dot = 0.0;
  if (!jv_tile_cg<T>(g, w, wm.kz, eps, cb, cq, z, y, p, x, dot, decide)) {  // uniform
    // posted after the sweep's code, so no store the sweep's loads must be
    // ordered against precedes them
    if (prog && blockIdx.x == 0 && threadIdx.x == 0) post_progress(prog, stop_iters, 1, stop_status);
    return;
  }
  const double d = wave_sum(dot);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) part_py[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

template <typename TD, bool kQ>
__device__ __forceinline__ void residual_wave(
    Geom g, WaveMap wm, Charge ch, const double* __restrict__ eps, const uint8_t* __restrict__ semi,
    const Doping dop, const uint8_t* __restrict__ mask, const double* __restrict__ phi,
    const TD* __restrict__ delta, double lam, const double* __restrict__ fsheet,
    const double* __restrict__ fdiag, double* __restrict__ F, double* __restrict__ invdiag,
    double* __restrict__ diag_out, double* __restrict__ cq, float* __restrict__ cq32,
    uint8_t* __restrict__ cflag, unsigned int* __restrict__ cbits, float* __restrict__ invdiag32,
    double* __restrict__ part, Quantum qm) {
  __shared__ double sred[4];
  int wx, wy, wz, wid;
  bool active;
  wave_coords(wm, wx, wy, wz, active, wid);
  if constexpr (kQ) {
    // the waves whose chunks hold the states' support loop over the states
    // and take longest: the chunk order is rotated so that they come first
    // in block order and start at once
    int zlo = 0x7fffffff;
    for (int i = 0; i < qm.n; ++i) zlo = min(zlo, qm.sbox[6 * i + 4]);
    if (zlo != 0x7fffffff) wz = (wz + max(zlo - 1, 0) / wm.kz) % wm.gz;
  }
  const WaveTile w(g, wx, wy, wz, wm.kz, threadIdx.x & 63, active);
  double acc = 0.0;
  residual_tile<TD, kQ>(g, w, ch, eps, semi, dop, mask, phi, delta, lam, fsheet, fdiag, F, invdiag, diag_out, cq, cq32,
                        cflag, (active && cbits) ? cbits + 64L * wid + (threadIdx.x & 63) : nullptr, invdiag32,
                        acc, &qm);
  const double d = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// The statistics residual runs at most 168 VGPRs (3 waves per SIMD) and the
// residual with eigenstates at most 256 (2 waves): the fastest caps measured
// at 129x129x65 (without one they take 190 and 257, 2 and 1 waves).
template <typename TD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_residual_wave(
    Geom g, WaveMap wm, Charge ch, const double* __restrict__ eps, const uint8_t* __restrict__ semi,
    const Doping dop, const uint8_t* __restrict__ mask, const double* __restrict__ phi,
    const TD* __restrict__ delta, double lam, const double* __restrict__ fsheet,
    const double* __restrict__ fdiag, double* __restrict__ F, double* __restrict__ invdiag,
    double* __restrict__ diag_out, double* __restrict__ cq, float* __restrict__ cq32,
    uint8_t* __restrict__ cflag, unsigned int* __restrict__ cbits, float* __restrict__ invdiag32,
    double* __restrict__ part, Quantum qm) {
  residual_wave<TD, false>(g, wm, ch, eps, semi, dop, mask, phi, delta, lam, fsheet, fdiag, F, invdiag, diag_out, cq,
                          cq32, cflag, cbits, invdiag32, part, qm);
}

template <typename TD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_residual_wave_q(
    Geom g, WaveMap wm, Charge ch, const double* __restrict__ eps, const uint8_t* __restrict__ semi,
    const Doping dop, const uint8_t* __restrict__ mask, const double* __restrict__ phi,
    const TD* __restrict__ delta, double lam, const double* __restrict__ fsheet,
    const double* __restrict__ fdiag, double* __restrict__ F, double* __restrict__ invdiag,
    double* __restrict__ diag_out, double* __restrict__ cq, float* __restrict__ cq32,
    uint8_t* __restrict__ cflag, unsigned int* __restrict__ cbits, float* __restrict__ invdiag32,
    double* __restrict__ part, Quantum qm) {
  residual_wave<TD, true>(g, wm, ch, eps, semi, dop, mask, phi, delta, lam, fsheet, fdiag, F, invdiag, diag_out, cq,
                          cq32, cflag, cbits, invdiag32, part, qm);
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
    Geom g, TileMap tm, const double* __restrict__ eps, const uint8_t* __restrict__ cflag,
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
          const long tsl = tile_slot(ex, ey, L, (g.nx + 6) / 7, (g.ny + 6) / 7);
          if (cflag[tsl]) {
            double c8[8];
            load8(cq + 8 * tsl, c8);
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
    double* __restrict__ partial, unsigned int* counter, double* __restrict__ out, Quantum qm) {
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
    if (qm.n > 0 && (!qm.region || qm.region[el])) {
      const long o[8] = {0, 1, sy, sy + 1, sz, sz + 1, sz + sy, sz + sy + 1};
      double dph[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) dph[k] = qm.phik[n0 + o[k]];
      gauss_interp(dph);
      double nq[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        dph[q] = ve[q] - dph[q];
        nq[q] = 0.0;
      }
      for (int st = 0; st < qm.n; ++st) {
        double s2[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) s2[k] = qm.psi2[qm.N * st + n0 + o[k]];
        gauss_interp(s2);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          double G, dG;
          pc_occupation(qm.conf, (dph[q] - qm.E[st]) * qm.inv_kT, G, dG);
          nq[q] += qm.pref * s2[q] * G;
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) s += nq[q];
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) s += electron_density_only(ch, ve[q]);
    }
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
                                                        const double* __restrict__ phi, double* __restrict__ nout,
                                                        Quantum qm) {
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
    double nn = 0.0;
    bool qnode = qm.n > 0 && !qm.region;   // touches a quantum-region element
    if (qm.n > 0 && qm.region)
      for (int dk = -1; dk <= 0; ++dk)
        for (int dj = -1; dj <= 0; ++dj)
          for (int di = -1; di <= 0; ++di) {
            const int ei = i + di, ej = j + dj, ek = k + dk;
            if (ei >= 0 && ei < g.nx - 1 && ej >= 0 && ej < g.ny - 1 && ek >= 0 && ek < g.nz - 1)
              qnode |= qm.region[elem_index(g, ei, ej, ek)] != 0;
          }
    if (touch && qnode) {
      const double dph = phi[n] - qm.phik[n];
      for (int st = 0; st < qm.n; ++st) {
        double G, dG;
        pc_occupation(qm.conf, (dph - qm.E[st]) * qm.inv_kT, G, dG);
        nn += qm.pref * qm.psi2[qm.N * st + n] * G;
      }
    } else if (touch) {
      nn = electron_density_only(ch, phi[n]);
    }
    nout[n] = nn;
  }
}

// ---------------------------------------------------------------------------
// Input validation.  Sets bits of *flags: 1 eps not finite/positive,
// 2 net doping not finite or a dopant density not finite and >= 0,
// 4 dir_id out of range, 8 phi not finite.
__global__ __launch_bounds__(kVecThreads) void k_validate(long N, long E, int n_dir, const double* __restrict__ eps,
                                                         const Doping dop, const int32_t* __restrict__ dir_id,
                                                         const double* __restrict__ phi, int* flags) {
  int f = 0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (long)gridDim.x * blockDim.x) {
    const double v = eps[e];
    if (!(v > 0.0) || !isfinite(v)) f |= 1;
    if (dop.net && !isfinite(dop.net[e])) f |= 2;
    if (dop.donors && !(dop.donors[e] >= 0.0 && isfinite(dop.donors[e]))) f |= 2;
    if (dop.acceptors && !(dop.acceptors[e] >= 0.0 && isfinite(dop.acceptors[e]))) f |= 2;
  }
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    const int d = dir_id[n];
    if (d < -1 || d >= n_dir) f |= 4;
    if (phi && !isfinite(phi[n])) f |= 8;
  }
  if (f) atomicOr(flags, f);
}

// Mesh coordinates and Dirichlet values: bits 128 / 256 / 512 of *flags when
// x / y / z has a value that is not finite or not above the one before it,
// 1024 when a Dirichlet value is not finite.
__global__ __launch_bounds__(kVecThreads) void k_validate_mesh(int nx, int ny, int nz, const double* __restrict__ x,
                                                              const double* __restrict__ y,
                                                              const double* __restrict__ z, int n_dir,
                                                              const double* __restrict__ dir_val, int* flags) {
  const int n[3] = {nx, ny, nz};
  const double* c[3] = {x, y, z};
  int f = 0;
  for (int a = 0; a < 3; ++a)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n[a]; i += gridDim.x * blockDim.x) {
      const double v = c[a][i];
      if (!isfinite(v) || (i > 0 && !(v > c[a][i - 1]))) f |= 128 << a;
    }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_dir; i += gridDim.x * blockDim.x)
    if (!isfinite(dir_val[i])) f |= 1024;
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

// Inverse z spacings 1 / (z[k+1] - z[k]) for the element stiffness weights,
// then the spacings themselves (rdz holds 2 (nz - 1) values).
__global__ __launch_bounds__(kVecThreads) void k_stage_rdz(int nz, const double* __restrict__ z,
                                                          double* __restrict__ rdz) {
  for (int k = (int)(blockIdx.x * blockDim.x + threadIdx.x); k < nz - 1; k += (int)(gridDim.x * blockDim.x)) {
    const double h = z[k + 1] - z[k];
    rdz[k] = 1.0 / h;
    rdz[nz - 1 + k] = h;
  }
}

template <typename TS, typename TD>
__global__ __launch_bounds__(kVecThreads) void k_cast(long n, const TS* __restrict__ a, TD* __restrict__ b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = (TD)a[i];
}

// b = a with Dirichlet entries zeroed (converted to TD)
template <typename TS, typename TD>
__global__ __launch_bounds__(kVecThreads) void k_masked_copy(long n, const uint8_t* __restrict__ mask,
                                                            const TS* __restrict__ a, TD* __restrict__ b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = mask[i] ? TD(0) : (TD)a[i];
}

// Tile-major copy of the per-element permittivity (padding slots 0).
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_stage_eps(Geom g, const double* __restrict__ eps,
                                                          T* __restrict__ eps_t, long nslots) {
  const int gx = (g.nx + 6) / 7, gy = (g.ny + 6) / 7;
  for (long sl = (long)blockIdx.x * blockDim.x + threadIdx.x; sl < nslots; sl += (long)gridDim.x * blockDim.x) {
    const int j = (int)(sl % 49);
    const long blk = sl / 49;
    const int tx = (int)(blk % gx), ty = (int)((blk / gx) % gy), L = (int)(blk / ((long)gx * gy));
    const int ex = 7 * tx + j % 7, ey = 7 * ty + j / 7;
    T v = T(0);
    if (ex < g.nx - 1 && ey < g.ny - 1 && L < g.nz - 1) v = (T)eps[elem_index(g, ex, ey, L)];
    eps_t[sl] = v;
  }
}

// Number of real elements whose tile-major flag is set (padding slots of
// ragged tiles are skipped: they are never written).
__global__ __launch_bounds__(kVecThreads) void k_count_flags(Geom g, const uint8_t* __restrict__ flag, long nslots,
                                                            unsigned long long* __restrict__ out) {
  __shared__ double sred[kVecThreads / 64];
  const int gx = (g.nx + 6) / 7, gy = (g.ny + 6) / 7;
  double cnt = 0.0;
  for (long sl = (long)blockIdx.x * blockDim.x + threadIdx.x; sl < nslots; sl += (long)gridDim.x * blockDim.x) {
    const int j = (int)(sl % 49);
    const long blk = sl / 49;
    const int tx = (int)(blk % gx), ty = (int)((blk / gx) % gy), L = (int)(blk / ((long)gx * gy));
    const int ex = 7 * tx + j % 7, ey = 7 * ty + j / 7;
    if (ex < g.nx - 1 && ey < g.ny - 1 && L < g.nz - 1 && flag[sl]) cnt += 1.0;
  }
  const double s = block_sum(cnt, sred);
  if (threadIdx.x == 0 && s > 0.0) atomicAdd(out, (unsigned long long)s);
}

// phi += lam * delta
template <typename TD>
__global__ __launch_bounds__(kVecThreads) void k_axpy_phi(long N, double* __restrict__ phi,
                                                         const TD* __restrict__ delta, double lam) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
    phi[i] += lam * (double)delta[i];
}

// ---------------------------------------------------------------------------
// Jacobi-preconditioned CG with its scalars on the device.  No kernel of the
// loop ends with a grid-wide reduction: each block publishes a partial sum and
// every block of the *next* kernel re-adds all partials in the same fixed
// order, so all blocks agree on alpha / beta bit for bit.  Iteration k keeps
// r^T z in ctx->rzs[k & 1]; the host passes the parity of k with every launch
// (chunks of iterations have even length, so a captured chunk can be replayed),
// and block 0 of the direction kernel counts the iterations.

// Four consecutive entries per thread ("chunk"), loaded with 16-byte vector
// loads when the chunk is whole.  The arrays are 256-byte aligned.
template <typename T>
struct Quad {
  T v[4];
};

template <typename T>
__device__ __forceinline__ Quad<T> ld4(const T* __restrict__ a, long c, long N) {
  Quad<T> q;
  const long i = 4 * c;
  if (i + 3 < N) {
    if constexpr (sizeof(T) == 8) {
      const double2* p2 = reinterpret_cast<const double2*>(a + i);
      const double2 u = p2[0], w = p2[1];
      q.v[0] = u.x; q.v[1] = u.y; q.v[2] = w.x; q.v[3] = w.y;
    } else {
      const float4 u = *reinterpret_cast<const float4*>(a + i);
      q.v[0] = u.x; q.v[1] = u.y; q.v[2] = u.z; q.v[3] = u.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) q.v[j] = (i + j < N) ? a[i + j] : T(0);
  }
  return q;
}

template <typename T>
__device__ __forceinline__ void st4(T* __restrict__ a, long c, long N, const Quad<T>& q) {
  const long i = 4 * c;
  if (i + 3 < N) {
    if constexpr (sizeof(T) == 8) {
      double2* p2 = reinterpret_cast<double2*>(a + i);
      p2[0] = make_double2(q.v[0], q.v[1]);
      p2[1] = make_double2(q.v[2], q.v[3]);
    } else {
      *reinterpret_cast<float4*>(a + i) = make_float4(q.v[0], q.v[1], q.v[2], q.v[3]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (i + j < N) a[i + j] = q.v[j];
  }
}

// x = 0, r = sign*b on free nodes, z = D^-1 r; partials of r^T z.
template <typename T, typename TB>
__global__ __launch_bounds__(kVecThreads) void k_pcg_init(long N, double sign, const TB* __restrict__ b,
                                                         const uint8_t* __restrict__ mask,
                                                         const T* __restrict__ invdiag, T* __restrict__ x,
                                                         T* __restrict__ r, T* __restrict__ z,
                                                         double* __restrict__ part) {
  __shared__ double sred[kVecThreads / 64];
  double rz = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
    const T ri = mask[i] ? T(0) : (T)(sign * (double)b[i]);
    const T zi = invdiag[i] * ri;
    x[i] = T(0);
    r[i] = ri;
    z[i] = zi;
    rz += (double)ri * (double)zi;
  }
  const double s1 = block_sum(rz, sred);
  if (threadIdx.x == 0) part[blockIdx.x] = s1;
}

// One block: the starting scalars of a solve.
__global__ __launch_bounds__(kVecThreads) void k_pcg_init_fin(PcgCtx* ctx, const double* __restrict__ part, int n,
                                                             double rtol, int maxit) {
  __shared__ double sred[kVecThreads / 64];
  const double RZ = sum_partials(part, n, 1, 0, sred);
  if (threadIdx.x == 0) {
    ctx->rzs[0] = RZ;
    ctx->rzs[1] = 0.0;
    ctx->tol2 = rtol * rtol * RZ;
    ctx->iters = 0;
    ctx->maxit = maxit;
    ctx->alpha = ctx->beta = ctx->pAp = 0.0;
    if (!isfinite(RZ)) {
      ctx->done = 1;
      ctx->status = PCG_NONFINITE;
    } else if (RZ == 0.0) {
      ctx->done = 1;
      ctx->status = PCG_CONVERGED;
    } else {
      ctx->done = 0;
      ctx->status = PCG_RUNNING;
    }
  }
}

// CG iteration k, second kernel: alpha = rz_k / p^T y (re-adding the
// partials of k_cg_jv); r -= alpha y; z = D^-1 r; partials of r^T z; in FP32
// also x += alpha p (in FP64 the next k_cg_jv takes that step).  Each thread first issues the loads of its first chunk, then re-adds
// the partials while they are in flight; later chunks are loaded one ahead.
// A launch after the solve has stopped returns at once.  Block 0 counts the
// iteration.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_cg_update(long N, int k, T* __restrict__ x, T* __restrict__ r,
                                                          T* __restrict__ z, const T* __restrict__ p,
                                                          const T* __restrict__ y, const T* __restrict__ invdiag,
                                                          PcgCtx* ctx, CgProgress* prog,
                                                          const double* __restrict__ part_py, int n_py,
                                                          double* __restrict__ part_rz) {
  if (ctx->done) return;
  __shared__ double sred[kVecThreads / 64];
  // the J.v kernel's p^T y partials first, so that waiting for them does not
  // wait for the vector loads below (the block size is the constant
  // kVecThreads: reading blockDim.x is a load too)
  constexpr int NT = kVecThreads;
  double py_part[8];
  const bool py_one = n_py <= 8 * NT;
#pragma unroll
  for (int j = 0; j < 8; ++j) py_part[j] = part_py[min((int)threadIdx.x + j * NT, n_py - 1)];
  const long nc = (N + 3) / 4, stride = (long)gridDim.x * NT;
  long c = (long)blockIdx.x * NT + threadIdx.x;
  constexpr bool kX = !cg_jv_steps_x<T>();
  Quad<T> qx, qr, qp, qy, qd;
  if (c < nc) {
    if constexpr (kX) qx = ld4(x, c, N);
    qr = ld4(r, c, N);
    if constexpr (kX) qp = ld4(p, c, N);
    qy = ld4(y, c, N);
    qd = ld4(invdiag, c, N);
  }
  const double rzk = ctx->rzs[k & 1];
  double pAp;
  if (py_one) {
    // the same fixed-order sum as sum_partials
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) a += ((int)threadIdx.x + j * NT < n_py) ? py_part[j] : 0.0;
    pAp = block_sum_all<NT>(a, sred);
  } else {
    pAp = sum_partials(part_py, n_py, 1, 0, sred);
  }
  if (!(pAp > 0.0) || !isfinite(pAp)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctx->pAp = pAp;
      ctx->done = 1;
      ctx->status = PCG_BREAKDOWN;
      if (prog) post_progress(prog, ctx->iters, 1, PCG_BREAKDOWN);
    }
    return;
  }
  const double a = rzk / pAp;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctx->pAp = pAp;
    ctx->alpha = a;
    ctx->iters += 1;
  }
  const T alpha = (T)a;
  double rz = 0.0;
  while (c < nc) {
    Quad<T> qz;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (kX) qx.v[j] += alpha * qp.v[j];
      qr.v[j] -= alpha * qy.v[j];
      qz.v[j] = qd.v[j] * qr.v[j];
      rz += (double)qr.v[j] * (double)qz.v[j];
    }
    if constexpr (kX) st4(x, c, N, qx);
    st4(r, c, N, qr);
    st4(z, c, N, qz);
    c += stride;
    if (c < nc) {
      if constexpr (kX) qx = ld4(x, c, N);
      qr = ld4(r, c, N);
      if constexpr (kX) qp = ld4(p, c, N);
      qy = ld4(y, c, N);
      qd = ld4(invdiag, c, N);
    }
  }
  const double s1 = block_sum(rz, sred);
  if (threadIdx.x == 0) part_rz[blockIdx.x] = s1;
}

// After an FP64 CG loop: the step x += alpha p of the last iteration whose
// alpha was formed, which no k_cg_jv took (the one after it stopped the
// solve, or none ran).  A breakdown forms no alpha: its step was taken.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_cg_finish_x(long N, const PcgCtx* __restrict__ ctx,
                                                            const T* __restrict__ p, T* __restrict__ x) {
  static_assert(cg_jv_steps_x<T>(), "only the sweep that takes the step leaves one to finish");
  if (ctx->status == PCG_BREAKDOWN || ctx->iters < 1) return;
  const T alpha = (T)ctx->alpha;
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x)
    x[n] += alpha * p[n];
}

// One block: sum of n partials (fixed order) into *out.
__global__ __launch_bounds__(kVecThreads) void k_sum_partials(const double* __restrict__ part, int n,
                                                             double* __restrict__ out) {
  __shared__ double sred[kVecThreads / 64];
  const double s = sum_partials(part, n, 1, 0, sred);
  if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------------------
// Launchers (host side, same translation unit so the templates instantiate).
#define QE_LAUNCH(kernel, grid, block, stream, ...) \
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, (hipStream_t)(stream), __VA_ARGS__)

void launch_adj_rhs(hipStream_t s, const Geom& g, const TileMap& tm, const Charge& ch, const Box& box,
                    const uint8_t* semi, const double* phi, double* gvec, double* partial, unsigned int* counter,
                    double* Q) {
  QE_LAUNCH(k_adj_rhs, tm.nblocks, kThreads, s, g, tm, ch, box, semi, phi, gvec, partial, counter, Q);
}

void launch_adj_grad(hipStream_t s, const Geom& g, const TileMap& tm, const double* eps, const uint8_t* cflag,
                     const double* cq, const uint8_t* mask, const double* lam, const double* phi,
                     const double* gvec, double* dQdeps, double* tcon) {
  QE_LAUNCH(k_adj_grad, tm.nblocks, kThreads, s, g, tm, eps, cflag, cq, mask, lam, phi, gvec, dQdeps, tcon);
}

void launch_contact_sum(hipStream_t s, int nblocks, long N, int n_dir, const int32_t* dir_id, const double* tcon,
                        double* partial, unsigned int* counter, double* out) {
  QE_LAUNCH(k_contact_sum, nblocks, kVecThreads, s, N, n_dir, dir_id, tcon, partial, counter, out);
}

void launch_count(hipStream_t s, int nblocks, const Geom& g, const Charge& ch, const BoxSet& boxes,
                  const uint8_t* semi, const double* phi, double* partial, unsigned int* counter, double* out,
                  const Quantum& qm) {
  QE_LAUNCH(k_count, nblocks, kVecThreads, s, g, ch, boxes, semi, phi, partial, counter, out, qm);
}

void launch_density(hipStream_t s, int nblocks, const Geom& g, const Charge& ch, const uint8_t* semi,
                    const double* phi, double* nout, const Quantum& qm) {
  QE_LAUNCH(k_density, nblocks, kVecThreads, s, g, ch, semi, phi, nout, qm);
}

__global__ __launch_bounds__(kVecThreads) void k_validate_quantum(Quantum qm, int* flags) {
  int f = 0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < qm.N; i += (long)gridDim.x * blockDim.x) {
    if (!isfinite(qm.phik[i])) f |= 64;
    for (int st = 0; st < qm.n; ++st) {
      const double v = qm.psi2[qm.N * st + i];
      if (!(v >= 0.0 && isfinite(v))) f |= 32;
    }
  }
  if (f) atomicOr(flags, f);
}

// Node-index bounding box of the nonzero |psi_i|^2 of every state (Quantum.sbox):
// an empty box per state, then per-wave minima / maxima merged by atomics
// (min / max are order independent).
__global__ __launch_bounds__(64) void k_state_boxes_init(int n, int* __restrict__ box) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    int* b = box + 6 * t;
    b[0] = b[2] = b[4] = 0x7fffffff;
    b[1] = b[3] = b[5] = -1;
  }
}

__global__ __launch_bounds__(256) void k_state_boxes(Geom g, Quantum qm, int* __restrict__ box) {
  // one wave per x row (j, k) of state blockIdx.y, rows strided over the
  // grid's waves; lanes step along x, so the reads are coalesced and the
  // only index arithmetic is per row
  const int st = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const long rows = (long)g.ny * g.nz;
  const long wave0 = (long)blockIdx.x * 4 + (threadIdx.x >> 6), nwav = (long)gridDim.x * 4;
  const double* ps = qm.psi2 + qm.N * st;
  int lo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, hi[3] = {-1, -1, -1};
  for (long r = wave0; r < rows; r += nwav) {
    const int j = (int)(r % g.ny), k = (int)(r / g.ny);
    const double* row = ps + r * g.nx;
    bool any = false;
    for (int i = lane; i < g.nx; i += 64) {
      if (row[i] != 0.0) {
        lo[0] = min(lo[0], i);
        hi[0] = max(hi[0], i);
        any = true;
      }
    }
    if (any) {
      lo[1] = min(lo[1], j);
      hi[1] = max(hi[1], j);
      lo[2] = min(lo[2], k);
      hi[2] = max(hi[2], k);
    }
  }
  // wave, then block minima / maxima; one set of atomics per block (the
  // grid keeps few blocks per state, so they do not queue on one address)
  __shared__ int sb[4][6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    for (int off = 32; off > 0; off >>= 1) {
      lo[a] = min(lo[a], __shfl_down(lo[a], off, 64));
      hi[a] = max(hi[a], __shfl_down(hi[a], off, 64));
    }
  }
  if (lane == 0)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      sb[threadIdx.x >> 6][2 * a] = lo[a];
      sb[threadIdx.x >> 6][2 * a + 1] = hi[a];
    }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = min(min(sb[0][2 * a], sb[1][2 * a]), min(sb[2][2 * a], sb[3][2 * a]));
      hi[a] = max(max(sb[0][2 * a + 1], sb[1][2 * a + 1]), max(sb[2][2 * a + 1], sb[3][2 * a + 1]));
    }
    if (hi[0] >= 0)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        atomicMin(box + 6 * st + 2 * a, lo[a]);
        atomicMax(box + 6 * st + 2 * a + 1, hi[a]);
      }
  }
}

void launch_state_boxes(hipStream_t s, int nblocks, const Geom& g, const Quantum& qm, int* box) {
  QE_LAUNCH(k_state_boxes_init, 1, 64, s, qm.n, box);
  // 64 blocks per state: 256 waves over the state's rows
  const long rows = (long)g.ny * g.nz;
  const int bx = (int)std::max(1L, std::min((rows + 3) / 4, 64L));
  (void)nblocks;
  hipLaunchKernelGGL(k_state_boxes, dim3(bx, qm.n), dim3(256), 0, s, g, qm, box);
}

void launch_validate_quantum(hipStream_t s, int nblocks, const Quantum& qm, int* flags) {
  QE_LAUNCH(k_validate_quantum, nblocks, kVecThreads, s, qm, flags);
}

void launch_validate(hipStream_t s, int nblocks, long N, long E, int n_dir, const double* eps, const Doping& dop,
                     const int32_t* dir_id, const double* phi, int* flags) {
  QE_LAUNCH(k_validate, nblocks, kVecThreads, s, N, E, n_dir, eps, dop, dir_id, phi, flags);
}

void launch_validate_mesh(hipStream_t s, int nx, int ny, int nz, const double* x, const double* y, const double* z,
                          int n_dir, const double* dir_val, int* flags) {
  const int longest = std::max(std::max(nx, ny), std::max(nz, n_dir));
  QE_LAUNCH(k_validate_mesh, std::max(1, std::min((longest + kVecThreads - 1) / kVecThreads, 64)), kVecThreads, s, nx,
            ny, nz, x, y, z, n_dir, dir_val, flags);
}

void launch_stage(hipStream_t s, int nblocks, long N, const int32_t* dir_id, const double* dir_val, uint8_t* mask,
                  double* phi, int apply, int zero_free) {
  QE_LAUNCH(k_stage, nblocks, kVecThreads, s, N, dir_id, dir_val, mask, phi, apply, zero_free);
}

void launch_stage_rdz(hipStream_t s, int nz, const double* z, double* rdz) {
  QE_LAUNCH(k_stage_rdz, 1, kVecThreads, s, nz, z, rdz);
}

void launch_cast_d2f(hipStream_t s, int nblocks, long n, const double* a, float* b) {
  QE_LAUNCH((k_cast<double, float>), nblocks, kVecThreads, s, n, a, b);
}

void launch_masked_copy_d2d(hipStream_t s, int nblocks, long n, const uint8_t* mask, const double* a, double* b) {
  QE_LAUNCH((k_masked_copy<double, double>), nblocks, kVecThreads, s, n, mask, a, b);
}

void launch_masked_copy_d2f(hipStream_t s, int nblocks, long n, const uint8_t* mask, const double* a, float* b) {
  QE_LAUNCH((k_masked_copy<double, float>), nblocks, kVecThreads, s, n, mask, a, b);
}

// J.v lanes' coefficient flags from the owners' element flags: bit L - Lbeg
// of a lane is set when its column's element of layer L has a nonzero c_q.
__global__ __launch_bounds__(256) void k_cbits_from_cflag(Geom g, WaveMap wm, const uint8_t* __restrict__ cflag,
                                                         unsigned int* __restrict__ cbits) {
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= wm.nwaves) return;
  int wx, wy, wz;
  wave_tile_of(w, wm, wx, wy, wz);
  const WaveTile t(g, wx, wy, wz, wm.kz, threadIdx.x & 63, true);
  unsigned int b = 0;
  if (t.col_ok) {
    const int lo = max(t.Lbeg, 0), hi = min(t.Lend, g.nz - 2);
    for (int L = lo; L <= hi; ++L)
      if (cflag[t.slot(L)]) b |= 1u << (L - t.Lbeg);
  }
  cbits[64L * w + (threadIdx.x & 63)] = b;
}

void launch_residual_wave(hipStream_t s, const Geom& g, const WaveMap& wm, const WaveMap& wmq, const Charge& ch,
                          const double* eps, const uint8_t* semi, const Doping& dop, const uint8_t* mask,
                          const double* phi, const double* delta64, const float* delta32, double lam,
                          const double* fsheet, const double* fdiag, double* F, double* invdiag, double* diag_out,
                          double* cq, float* cq32, uint8_t* cflag, unsigned int* cbits, float* invdiag32,
                          double* partial, double* norm2, const Quantum& qm) {
  const bool q = qm.n > 0;
  if (delta32 && q)
    QE_LAUNCH((k_residual_wave_q<float>), wmq.nblocks, 256, s, g, wmq, ch, eps, semi, dop, mask, phi, delta32, lam,
              fsheet, fdiag, F, invdiag, diag_out, cq, cq32, cflag, nullptr, invdiag32, partial, qm);
  else if (delta32)
    QE_LAUNCH((k_residual_wave<float>), wm.nblocks, 256, s, g, wm, ch, eps, semi, dop, mask, phi, delta32, lam,
              fsheet, fdiag, F, invdiag, diag_out, cq, cq32, cflag, cbits, invdiag32, partial, qm);
  else if (q)
    QE_LAUNCH((k_residual_wave_q<double>), wmq.nblocks, 256, s, g, wmq, ch, eps, semi, dop, mask, phi, delta64, lam,
              fsheet, fdiag, F, invdiag, diag_out, cq, cq32, cflag, nullptr, invdiag32, partial, qm);
  else
    QE_LAUNCH((k_residual_wave<double>), wm.nblocks, 256, s, g, wm, ch, eps, semi, dop, mask, phi, delta64, lam,
              fsheet, fdiag, F, invdiag, diag_out, cq, cq32, cflag, cbits, invdiag32, partial, qm);
  if (q) QE_LAUNCH(k_cbits_from_cflag, wm.nblocks, 256, s, g, wm, cflag, cbits);
  QE_LAUNCH(k_sum_partials, 1, kVecThreads, s, partial, q ? wmq.nblocks : wm.nblocks, norm2);
}

void launch_jv_wave64(hipStream_t s, const Geom& g, const WaveMap& wm, const double* eps, const unsigned int* cbits,
                      const double* cq, const uint8_t* mask, const double* v, double* y, int identity_rows) {
  QE_LAUNCH(k_jv_wave<double>, wm.nblocks, 256, s, g, wm, eps, cbits, cq, mask, v, y, identity_rows);
}

void launch_jv_wave32(hipStream_t s, const Geom& g, const WaveMap& wm, const float* eps, const unsigned int* cbits,
                      const float* cq, const uint8_t* mask, const float* v, float* y, int identity_rows) {
  QE_LAUNCH(k_jv_wave<float>, wm.nblocks, 256, s, g, wm, eps, cbits, cq, mask, v, y, identity_rows);
}

void launch_cg_jv64(hipStream_t s, const Geom& g, const WaveMap& wm, int cgblocks, int k, const double* eps_t,
                    const unsigned int* cbits, const double* cq, const double* z, double* y, double* p, double* x,
                    PcgCtx* ctx, CgProgress* prog, const double* part_rz, double* part_py) {
  QE_LAUNCH(k_cg_jv<double>, wm.nblocks, 256, s, g, wm, eps_t, cbits, cq, z, y, p, x, k, ctx, prog, part_rz, cgblocks,
            part_py);
}

void launch_cg_jv32(hipStream_t s, const Geom& g, const WaveMap& wm, int cgblocks, int k, const float* eps_t,
                    const unsigned int* cbits, const float* cq, const float* z, float* y, float* p, float* x,
                    PcgCtx* ctx, CgProgress* prog, const double* part_rz, double* part_py) {
  QE_LAUNCH(k_cg_jv<float>, wm.nblocks, 256, s, g, wm, eps_t, cbits, cq, z, y, p, x, k, ctx, prog, part_rz, cgblocks,
            part_py);
}

void launch_stage_eps64(hipStream_t s, int nblocks, const Geom& g, const double* eps, double* eps_t, long nslots) {
  QE_LAUNCH(k_stage_eps<double>, nblocks, kVecThreads, s, g, eps, eps_t, nslots);
}

void launch_stage_eps32(hipStream_t s, int nblocks, const Geom& g, const double* eps, float* eps_t, long nslots) {
  QE_LAUNCH(k_stage_eps<float>, nblocks, kVecThreads, s, g, eps, eps_t, nslots);
}

void launch_count_flags(hipStream_t s, int nblocks, const Geom& g, const uint8_t* flag, long nslots,
                        unsigned long long* out) {
  QE_LAUNCH(k_count_flags, nblocks, kVecThreads, s, g, flag, nslots, out);
}

void launch_axpy_phi(hipStream_t s, int nblocks, long N, double* phi, const double* d64, const float* d32,
                     double lam) {
  if (d32)
    QE_LAUNCH(k_axpy_phi<float>, nblocks, kVecThreads, s, N, phi, d32, lam);
  else
    QE_LAUNCH(k_axpy_phi<double>, nblocks, kVecThreads, s, N, phi, d64, lam);
}

void launch_pcg_start64(hipStream_t s, int cgblocks, long N, double sign, const double* b, const uint8_t* mask,
                        const double* invdiag, double* x, double* r, double* z, PcgCtx* ctx, double* part_rz,
                        double rtol, int maxit) {
  QE_LAUNCH((k_pcg_init<double, double>), cgblocks, kVecThreads, s, N, sign, b, mask, invdiag, x, r, z, part_rz);
  QE_LAUNCH(k_pcg_init_fin, 1, kVecThreads, s, ctx, part_rz, cgblocks, rtol, maxit);
}

void launch_pcg_start32(hipStream_t s, int cgblocks, long N, double sign, const double* b, const uint8_t* mask,
                        const float* invdiag, float* x, float* r, float* z, PcgCtx* ctx, double* part_rz,
                        double rtol, int maxit) {
  QE_LAUNCH((k_pcg_init<float, double>), cgblocks, kVecThreads, s, N, sign, b, mask, invdiag, x, r, z, part_rz);
  QE_LAUNCH(k_pcg_init_fin, 1, kVecThreads, s, ctx, part_rz, cgblocks, rtol, maxit);
}

void launch_pcg_iter64(hipStream_t s, const Geom& g, const WaveMap& wm, int cgblocks, long N, int k,
                       const double* eps_t, const unsigned int* cbits, const double* cq, const double* invdiag, double* x,
                       double* r, double* z, double* p, double* y, PcgCtx* ctx, CgProgress* prog, double* part_py,
                       double* part_rz, const SheetSet* S, const int4* items, const uint8_t* mask) {
  launch_cg_jv64(s, g, wm, cgblocks, k, eps_t, cbits, cq, z, y, p, x, ctx, prog, part_rz, part_py);
  int n_py = wm.nblocks;
  if (S && S->any_robin) {
    launch_sheet_jv64(s, *S, items, mask, z, y, p, ctx, part_py + wm.nblocks);
    n_py += sheet_blocks(*S);
  }
  QE_LAUNCH(k_cg_update<double>, cgblocks, kVecThreads, s, N, k, x, r, z, p, y, invdiag, ctx, prog, part_py, n_py,
            part_rz);
}

void launch_pcg_iter32(hipStream_t s, const Geom& g, const WaveMap& wm, int cgblocks, long N, int k,
                       const float* eps_t, const unsigned int* cbits, const float* cq, const float* invdiag, float* x,
                       float* r, float* z, float* p, float* y, PcgCtx* ctx, CgProgress* prog, double* part_py,
                       double* part_rz, const SheetSet* S, const int4* items, const uint8_t* mask) {
  launch_cg_jv32(s, g, wm, cgblocks, k, eps_t, cbits, cq, z, y, p, x, ctx, prog, part_rz, part_py);
  int n_py = wm.nblocks;
  if (S && S->any_robin) {
    launch_sheet_jv32(s, *S, items, mask, z, y, p, ctx, part_py + wm.nblocks);
    n_py += sheet_blocks(*S);
  }
  QE_LAUNCH(k_cg_update<float>, cgblocks, kVecThreads, s, N, k, x, r, z, p, y, invdiag, ctx, prog, part_py, n_py,
            part_rz);
}

void launch_cg_finish_x64(hipStream_t s, int nblocks, long N, const PcgCtx* ctx, const double* p, double* x) {
  QE_LAUNCH(k_cg_finish_x<double>, nblocks, kVecThreads, s, N, ctx, p, x);
}

}  // namespace qe
