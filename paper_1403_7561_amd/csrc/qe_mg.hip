// Geometric multigrid preconditioner of the CG (kernels and host
// launchers).  The paper solves each Newton step with a preconditioned
// Krylov method from its solver library and names no preconditioner
// (Sec. II.A.3 and II.C); this one is a symmetric V-cycle on the meshes of
// the coarse-mesh sequence:
//
//   level l + 1 keeps the fine nodes f(I) = min(2 I, n - 1) of level l along
//   each axis; its Jacobian is the coarse problem's own (rediscretised) at
//   the potential injected from level l;
//   prolongation P: trilinear interpolation in the fine coordinates;
//   restriction: exactly P^T;
//   smoother: x += S (b - J x) with S = omega / sum_j |J_ij| (weighted
//   l1-Jacobi, 0 < omega < 2), the same before and after the coarse
//   correction;
//   coarsest level: a fixed number of smoother steps from x = S b;
//   on very large meshes the finest level only adds its correction,
//   z = S r + P B_1 P^T r (no smoothing products there).
//
// With R = P^T, one smoother S on both sides and an SPD coarse operator, the
// V-cycle is symmetric; the row bound puts every eigenvalue of S J / omega
// in (0, 1], so 2 S^-1 - J is positive definite for omega < 2, and so is
// the V-cycle (and the additive form, a sum of positive definite and
// semidefinite parts): plain CG with it stays CG (no flexible variant).
// The l1 sums are formed element by element: sum_j |Khat_ij| of the box
// element from its three stiffness weights, and for the Gauss-point
// coefficient term, whose entries are all >= 0 and whose trilinear weights
// sum to 1, the row sum B^T c.  Both bound the assembled row's absolute sum
// from above.
//
// The V-cycle runs in the CG's own precision: FP64, or FP32 inside the
// mixed-precision Newton (FP32 coefficients, permittivities, smoother
// weights and vectors; restriction sums and the r^T z partials in FP64).
//
// A smoothing step after the coarse correction, and each of the coarsest
// level's, is one launch: the level's wave-tiled J.v in a smoothing mode
// writes x + S (b - J x) into the level's other vector as each row
// completes, so a level's x and y take turns holding its iterate.
//
// Every kernel here returns at once when the CG it serves has stopped
// (ctx->done), like the CG loop's own kernels, so launches queued after the
// stop cost only their dispatch.
#include <algorithm>

#include "qe_kernels.h"
#include "qe_tiles.h"

namespace qe {

#define QE_LAUNCH(kernel, grid, block, stream, ...) \
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, (hipStream_t)(stream), __VA_ARGS__)

__device__ __forceinline__ int mg_fine(int I, int n) { return min(2 * I, n - 1); }

// One axis of the interpolation: the coarse interval holding fine node i and
// the weight of its upper end (fine node i takes (1 - w) of coarse I and w
// of coarse I + 1).
__device__ __forceinline__ void mg_weight(int i, int nf, int nc, const double* __restrict__ xf, int& I, double& w) {
  I = min(i >> 1, nc - 2);
  const double a = xf[mg_fine(I, nf)], b = xf[mg_fine(I + 1, nf)];
  w = (xf[i] - a) / (b - a);
}

// One axis of the restriction: the fine nodes f(I) - 1, f(I), f(I) + 1 and
// their weights on coarse node I, the transpose of mg_weight's (a fine node
// strictly inside the coarse interval [I - 1, I] takes w of coarse I, one
// inside [I, I + 1] takes 1 - w).  A missing neighbour (the mesh's end, or
// a fine node that is itself a coarse node, as at the even count's last
// interval) gets weight 0 and the centre's index.
__device__ __forceinline__ void mg_taps(int I, int nf, int nc, const double* __restrict__ xf, int idx[3], double wt[3]) {
  const int c = mg_fine(I, nf);
  const double X = xf[c];
  idx[0] = idx[1] = idx[2] = c;
  wt[0] = wt[2] = 0.0;
  wt[1] = 1.0;
  if (I > 0) {
    const int lo = mg_fine(I - 1, nf);
    if (c - 1 > lo) {
      const double a = xf[lo];
      idx[0] = c - 1;
      wt[0] = (xf[c - 1] - a) / (X - a);
    }
  }
  if (I < nc - 1) {
    const int hi = mg_fine(I + 1, nf);
    if (c + 1 < hi) {
      const double b = xf[hi];
      idx[2] = c + 1;
      wt[2] = (b - xf[c + 1]) / (b - X);
    }
  }
}

// y = J v on one level, as the library's plain J.v (v read as 0 on Dirichlet
// nodes, y = 0 on their rows).
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_mg_jv(
    Geom g, WaveMap wm, const T* __restrict__ eps, const unsigned int* __restrict__ cbits,
    const T* __restrict__ cq, const uint8_t* __restrict__ mask, const T* __restrict__ v,
    T* __restrict__ y, const PcgCtx* __restrict__ ctx) {
  if (ctx->done) return;
  const int w = __builtin_amdgcn_readfirstlane(wave_of_block(blockIdx.x, wm) * 4 + (threadIdx.x >> 6));
  const bool active = w < wm.nwaves;
  int wx, wy, wz;
  wave_tile_of(w, wm, wx, wy, wz);
  const WaveTile t(g, wx, wy, wz, wm.kz, threadIdx.x & 63, active);
  const unsigned int cb = active ? cbits[64L * w + (threadIdx.x & 63)] : 0u;
  double dot = 0.0;
  jv_tile<T, JV_PLAIN>(g, t, eps, cb, cq, mask, v, y, 2, dot);
}

// One smoothing step in one launch: xo = x + S (b - J x) on every node (J x
// as k_mg_jv's, S = 0 on Dirichlet nodes), xo a buffer other than x; with
// part, one b^T xo partial per block, and blocks past the wave map's (the
// grid may be larger, to give the count a reader expects) write 0.  Its
// meshes give about 3 waves per SIMD or fewer, so it may take the registers
// of 3 (with 4 the FP64 form spills).
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_mg_jv_smooth(
    Geom g, WaveMap wm, const T* __restrict__ eps, const unsigned int* __restrict__ cbits,
    const T* __restrict__ cq, const uint8_t* __restrict__ mask, const T* __restrict__ x,
    const T* __restrict__ b, const T* __restrict__ S, T* __restrict__ xo, double* __restrict__ part,
    const PcgCtx* __restrict__ ctx) {
  if (ctx->done) return;
  if ((int)blockIdx.x >= wm.nblocks) {
    if (part && threadIdx.x == 0) part[blockIdx.x] = 0.0;
    return;
  }
  __shared__ double sred[4];
  const int w = __builtin_amdgcn_readfirstlane(wave_of_block(blockIdx.x, wm) * 4 + (threadIdx.x >> 6));
  const bool active = w < wm.nwaves;
  int wx, wy, wz;
  wave_tile_of(w, wm, wx, wy, wz);
  const WaveTile t(g, wx, wy, wz, wm.kz, threadIdx.x & 63, active);
  const unsigned int cb = active ? cbits[64L * w + (threadIdx.x & 63)] : 0u;
  double dot = 0.0;
  jv_tile<T, JV_SMOOTH>(g, t, eps, cb, cq, mask, x, xo, 2, dot, b, S);
  if (part) {
    const double s1 = block_sum(dot, sred);
    if (threadIdx.x == 0) part[blockIdx.x] = s1;
  }
}

// Tiles of the tiled restriction: along each axis ceil(n / w) tiles of w
// nodes, the last one shorter.  (Letting the last tile take one node more,
// so that 2^k + 1 meshes get no one-node tiles, needs a larger LDS window:
// 3 blocks per CU instead of 6, measured slower.)
__device__ __forceinline__ void mg_tile(int t, int n, int w, int& lo, int& hi) {
  lo = t * w;
  hi = min(lo + w, n);
}
static inline int mg_ntiles(int n, int w) { return (n + w - 1) / w; }

// Restriction tiles of 32 x 4 x 2 coarse nodes, one per thread.  The taps of
// coarse node I lie in [f(I) - 1, f(I) + 1] and move forward with I, so a
// tile of w coarse nodes reads a window of at most 2 w + 1 fine nodes, from
// the first tap of its first node to the last tap of its last.
constexpr int kRtX = 32, kRtY = 4, kRtZ = 2;
constexpr int kRwX = 2 * kRtX + 1, kRwY = 2 * kRtY + 1, kRwZ = 2 * kRtZ + 1;
constexpr int kRowsPer = (kRwY * kRwZ + 3) / 4;

// The restriction, one thread per coarse node (I, J, K): b_c = sum over fine
// nodes of P_fine,coarse (r - y) (y = NULL: r alone) with fine Dirichlet
// nodes counted as 0 (the CG's own r is not zero on their rows: its J.v
// writes them), 0 on coarse Dirichlet nodes; x_c = S_c b_c, the
// pre-smoothing step from zero.  The taps and weights per axis come from the
// level's tables (mg_taps, formed once per setup).  The block's fine window
// of r - y (0 on fine Dirichlet nodes) is staged in LDS by coalesced loads,
// and the 27 taps then read LDS.  Every load is issued before its first use (lanes past the
// window read a node inside it; the masks are applied as selects), so a
// block waits for memory twice, not once per element.
template <typename T, bool HAS_Y>
__global__ __launch_bounds__(kVecThreads) void k_mg_restrict_tile(int nxf, int nyf, int nzf, int nxc, int nyc, int nzc,
                                                                   int tnx, int tny, int tnz, MgAxes tab,
                                                                   const uint8_t* __restrict__ maskf,
                                                                   const T* __restrict__ r, const T* __restrict__ y,
                                                                   const uint8_t* __restrict__ maskc,
                                                                   const T* __restrict__ Sc, T* __restrict__ bc,
                                                                   T* __restrict__ xc, const PcgCtx* __restrict__ ctx) {
  if (ctx->done) return;
  __shared__ double sv[kRwX * kRwY * kRwZ];
  const int tx = blockIdx.x % tnx, ty = (blockIdx.x / tnx) % tny, tz = blockIdx.x / (tnx * tny);
  int I0, I1, J0, J1, K0, K1;
  mg_tile(tx, nxc, kRtX, I0, I1);
  mg_tile(ty, nyc, kRtY, J0, J1);
  mg_tile(tz, nzc, kRtZ, K0, K1);
  // window [f(I0) - 1, f(I1 - 1) + 1] clipped to the mesh: it holds every
  // tap of the tile (a tap that is no neighbour of a coarse node is staged
  // but not read)
  const int fx = max(mg_fine(I0, nxf) - 1, 0), fy = max(mg_fine(J0, nyf) - 1, 0), fz = max(mg_fine(K0, nzf) - 1, 0);
  const int wx = min(mg_fine(I1 - 1, nxf) + 1, nxf - 1) - fx + 1;
  const int wy = min(mg_fine(J1 - 1, nyf) + 1, nyf - 1) - fy + 1;
  const int rows = wy * (min(mg_fine(K1 - 1, nzf) + 1, nzf - 1) - fz + 1);
  const long base = (long)fx + (long)nxf * ((long)fy + (long)nyf * fz);
  // one window row per wave and step (lanes along x), all loads issued
  // before the first use; the 65th column of a full tile's window follows,
  // one node per thread
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ex = min(lane, wx - 1);
  uint8_t m[kRowsPer];
  T rv[kRowsPer], yv[kRowsPer];
#pragma unroll
  for (int p = 0; p < kRowsPer; ++p) {
    const int row = min(wv + 4 * p, rows - 1), ez = row / wy, ey = row - ez * wy;
    const long n = base + ex + (long)nxf * ((long)ey + (long)nyf * ez);
    m[p] = maskf[n];
    rv[p] = r[n];
    if (HAS_Y) yv[p] = y[n];
  }
  const int extra = wx > 64 ? (wx - 64) * rows : 0;
  const int xe = threadIdx.x < extra ? threadIdx.x : 0;
  const int xrow = xe / max(wx - 64, 1), xcol = 64 + xe - xrow * max(wx - 64, 1);
  const int xez = xrow / wy, xey = xrow - xez * wy;
  const long xn = base + (threadIdx.x < extra ? xcol + (long)nxf * ((long)xey + (long)nyf * xez) : 0);
  const uint8_t xm = maskf[xn];
  const T xr = r[xn], xy = HAS_Y ? y[xn] : T(0);
  // the taps, weights, flag and S of a coarse node, and its sum from LDS
  struct Taps {
    int ix[3], iy[3], iz[3];
    double wx[3], wy[3], wz[3];
    uint8_t mc;
    T st;
  };
  auto load_taps = [&](int I, int J, int K, Taps& q) {
    const long t = (long)I + (long)nxc * ((long)J + (long)nyc * K);
    q.mc = maskc[t];
    q.st = Sc[t];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      q.ix[k] = tab.rI[0][3 * I + k] - fx;
      q.iy[k] = tab.rI[1][3 * J + k] - fy;
      q.iz[k] = tab.rI[2][3 * K + k] - fz;
      q.wx[k] = tab.rw[0][3 * I + k];
      q.wy[k] = tab.rw[1][3 * J + k];
      q.wz[k] = tab.rw[2][3 * K + k];
    }
  };
  auto sum_taps = [&](int I, int J, int K, const Taps& q) {
    double v[27];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int bq = 0; bq < 3; ++bq) {
        const double* row = sv + (q.iz[c] * kRwY + q.iy[bq]) * kRwX;
#pragma unroll
        for (int a = 0; a < 3; ++a) v[(c * 3 + bq) * 3 + a] = row[q.ix[a]];
      }
    double b = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int bq = 0; bq < 3; ++bq) {
        const double wyz = q.wy[bq] * q.wz[c];
#pragma unroll
        for (int a = 0; a < 3; ++a) b += (wyz * q.wx[a]) * v[(c * 3 + bq) * 3 + a];
      }
    const long t = (long)I + (long)nxc * ((long)J + (long)nyc * K);
    const T bt = q.mc ? T(0) : (T)b;
    bc[t] = bt;
    xc[t] = q.st * bt;
  };
  // this thread's coarse node (one per thread: a tile has at most 256) is
  // loaded with the window
  const int li = threadIdx.x % kRtX, lj = (threadIdx.x / kRtX) % kRtY, lk = threadIdx.x / (kRtX * kRtY);
  const int Io = I0 + li, Jo = J0 + lj, Ko = K0 + lk;
  const bool own = Io < I1 && Jo < J1 && Ko < K1;
  Taps qo;
  load_taps(min(Io, I1 - 1), min(Jo, J1 - 1), min(Ko, K1 - 1), qo);
#pragma unroll
  for (int p = 0; p < kRowsPer; ++p) {
    const int row = wv + 4 * p;
    if (row < rows && lane < wx) {
      const int ez = row / wy, ey = row - ez * wy;
      const double v = (double)rv[p] - (HAS_Y ? (double)yv[p] : 0.0);
      sv[(ez * kRwY + ey) * kRwX + lane] = m[p] ? 0.0 : v;
    }
  }
  if (threadIdx.x < extra) {
    const double v = (double)xr - (HAS_Y ? (double)xy : 0.0);
    sv[(xez * kRwY + xey) * kRwX + xcol] = xm ? 0.0 : v;
  }
  __syncthreads();
  if (own) sum_taps(Io, Jo, Ko, qo);
}

// Fine node: xo = x + P x_c on free nodes, 0 on Dirichlet nodes (the
// coarse interval and weight per axis from the level's tables; xo may be
// x); with part, one partial of bdot^T xo per block.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_mg_prolong(int nxf, int nyf, long Nf, int nxc, int nyc, MgAxes tab,
                                                             const uint8_t* __restrict__ maskf,
                                                             const T* __restrict__ xcv, const T* x, T* xo,
                                                             const T* __restrict__ bdot, double* __restrict__ part,
                                                             const PcgCtx* __restrict__ ctx) {
  if (ctx->done) return;
  __shared__ double sred[kVecThreads / 64];
  double bz = 0.0;
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < Nf; n += (long)gridDim.x * blockDim.x) {
    if (maskf[n]) {
      xo[n] = T(0);
      continue;
    }
    const int i = (int)(n % nxf), j = (int)((n / nxf) % nyf), k = (int)(n / ((long)nxf * nyf));
    const int I = tab.pI[0][i], J = tab.pI[1][j], K = tab.pI[2][k];
    const double wx = tab.pw[0][i], wy = tab.pw[1][j], wz = tab.pw[2][k];
    const long c0 = (long)I + (long)nxc * ((long)J + (long)nyc * K), sy = nxc, sz = (long)nxc * nyc;
    double c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = (double)xcv[c0 + (q & 1) + ((q & 2) ? sy : 0) + ((q & 4) ? sz : 0)];
    const double v00 = c[0] + wx * (c[1] - c[0]), v10 = c[2] + wx * (c[3] - c[2]);
    const double v01 = c[4] + wx * (c[5] - c[4]), v11 = c[6] + wx * (c[7] - c[6]);
    const double v0 = v00 + wy * (v10 - v00), v1 = v01 + wy * (v11 - v01);
    const T xn = (T)((double)x[n] + (v0 + wz * (v1 - v0)));
    xo[n] = xn;
    if (part) bz += (double)bdot[n] * (double)xn;
  }
  if (part) {
    const double s1 = block_sum(bz, sred);
    if (threadIdx.x == 0) part[blockIdx.x] = s1;
  }
}

// The interpolation and restriction tables of a level pair, per axis: for
// each fine index its coarse interval and upper-end weight (mg_weight), for
// each coarse index its three fine taps and weights (mg_taps).
__global__ __launch_bounds__(kVecThreads) void k_mg_tables(int nxf, int nyf, int nzf, int nxc, int nyc, int nzc,
                                                            const double* __restrict__ xf,
                                                            const double* __restrict__ yf,
                                                            const double* __restrict__ zf, MgAxes tab) {
  const int nf[3] = {nxf, nyf, nzf}, nc[3] = {nxc, nyc, nzc};
  const double* co[3] = {xf, yf, zf};
  for (int a = 0; a < 3; ++a) {
    for (int i = threadIdx.x; i < nf[a]; i += blockDim.x) {
      int I;
      double w;
      mg_weight(i, nf[a], nc[a], co[a], I, w);
      tab.pI[a][i] = I;
      tab.pw[a][i] = w;
    }
    for (int I = threadIdx.x; I < nc[a]; I += blockDim.x) {
      int idx[3];
      double wt[3];
      mg_taps(I, nf[a], nc[a], co[a], idx, wt);
      for (int k = 0; k < 3; ++k) {
        tab.rI[a][3 * I + k] = idx[k];
        tab.rw[a][3 * I + k] = wt[k];
      }
    }
  }
}

// x += S (b - y) (S is 0 on Dirichlet nodes); with part, one partial of
// b^T x per block (the CG's r^T z after the fine level's last step).
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_mg_smooth(long N, const T* __restrict__ b, const T* __restrict__ y,
                                                            const T* __restrict__ S, T* __restrict__ x,
                                                            double* __restrict__ part, const PcgCtx* __restrict__ ctx) {
  if (ctx->done) return;
  __shared__ double sred[kVecThreads / 64];
  double bz = 0.0;
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    const T bn = b[n];
    const T xn = x[n] + S[n] * (bn - y[n]);
    x[n] = xn;
    bz += (double)bn * (double)xn;
  }
  if (part) {
    const double s1 = block_sum(bz, sred);
    if (threadIdx.x == 0) part[blockIdx.x] = s1;
  }
}

// After the V-cycle on the CG's starting residual: r_0^T z_0 from its
// partials replaces the Jacobi one (the tolerance keeps its ratio rtol^2).
__global__ __launch_bounds__(kVecThreads) void k_mg_start_fin(PcgCtx* ctx, const double* __restrict__ part, int n) {
  if (ctx->done) return;
  __shared__ double sred[kVecThreads / 64];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += kVecThreads) a += part[i];
  const double RZ = block_sum(a, sred);   // complete in thread 0
  if (threadIdx.x == 0) {
    const double ratio = ctx->tol2 / ctx->rzs[0];   // rtol^2 (rzs[0] > 0: the start did not stop)
    ctx->rzs[0] = RZ;
    ctx->tol2 = ratio * RZ;
    if (!isfinite(RZ)) {
      ctx->done = 1;
      ctx->status = PCG_NONFINITE;
    } else if (RZ <= 0.0) {
      // r != 0 (the start did not stop) and the V-cycle is positive definite:
      // r^T z <= 0 can only come from a broken linearisation
      ctx->done = 1;
      ctx->status = PCG_BREAKDOWN;
    }
  }
}

// A coarse level's eigenstates by injection (n_states planes of |psi|^2 and
// phi^(k)); each coarse element takes the region flag of its first fine
// element, as the coarse problem takes its materials.
__global__ __launch_bounds__(kVecThreads) void k_mg_coarsen_states(int nxf, int nyf, int nzf, int nxc, int nyc,
                                                                    int nzc, int n_states,
                                                                    const double* __restrict__ psi2f,
                                                                    const double* __restrict__ phikf,
                                                                    const uint8_t* __restrict__ regf,
                                                                    double* __restrict__ psi2c,
                                                                    double* __restrict__ phikc,
                                                                    uint8_t* __restrict__ regc) {
  const long Nf = (long)nxf * nyf * nzf, Nc = (long)nxc * nyc * nzc;
  const long Ec = (long)(nxc - 1) * (nyc - 1) * (nzc - 1);
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < Nc; t += (long)gridDim.x * blockDim.x) {
    const int I = (int)(t % nxc), J = (int)((t / nxc) % nyc), K = (int)(t / ((long)nxc * nyc));
    const long f = (long)mg_fine(I, nxf) + (long)nxf * ((long)mg_fine(J, nyf) + (long)nyf * mg_fine(K, nzf));
    phikc[t] = phikf[f];
    for (int st = 0; st < n_states; ++st) psi2c[(long)st * Nc + t] = psi2f[(long)st * Nf + f];
    if (regc && t < Ec) {
      const int ei = (int)(t % (nxc - 1)), ej = (int)((t / (nxc - 1)) % (nyc - 1)),
                ek = (int)(t / ((long)(nxc - 1) * (nyc - 1)));
      regc[t] = regf[(long)(2 * ei) + (long)(nxf - 1) * ((long)(2 * ej) + (long)(nyf - 1) * (2 * ek))];
    }
  }
}

// Coarse potential by injection: phi_c(I, J, K) = phi_f(f(I), f(J), f(K)).
__global__ __launch_bounds__(kVecThreads) void k_mg_inject(int nxf, int nyf, int nzf, int nxc, int nyc, int nzc,
                                                            const double* __restrict__ phif,
                                                            double* __restrict__ phic) {
  const long Nc = (long)nxc * nyc * nzc;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < Nc; t += (long)gridDim.x * blockDim.x) {
    const int I = (int)(t % nxc), J = (int)((t / nxc) % nyc), K = (int)(t / ((long)nxc * nyc));
    phic[t] = phif[(long)mg_fine(I, nxf) + (long)nxf * ((long)mg_fine(J, nyf) + (long)nyf * mg_fine(K, nzf))];
  }
}

// Smoother weights S_i = omega / (sum over the elements of node i of
// sum_j |Khat_ij| + (B^T c)_i) on free nodes, 0 on Dirichlet nodes.
// Khat's entry between local nodes that differ along the axes in d is
// sx kx(dx) my(dy) mz(dz) + sy mx(dx) ky(dy) mz(dz) + sz mx(dx) my(dy) kz(dz)
// with k(same) = 1, k(diff) = -1, m(same) = 1/3, m(diff) = 1/6 (the box
// element's stiffness in the weights sx = eps h_y h_z / h_x, ...).  B^T c is
// the coefficient term's product with the all-ones vector (the stiffness
// rows sum to zero), so jv_element gives it.
// One thread per node column (i, j) and chunk of kc node layers: it walks
// up the column, and each element layer's (up to) four elements around the
// column give the row sums of the node below them and of the node above
// (carried to the next layer).  The box element's stiffness rows all have the
// same absolute sum, so that part is formed once per element.
__global__ __launch_bounds__(kVecThreads) void k_mg_l1(Geom g, const double* __restrict__ eps,
                                                        const uint8_t* __restrict__ cflag,
                                                        const double* __restrict__ cq,
                                                        const uint8_t* __restrict__ mask, double omega, int kc,
                                                        double* __restrict__ S, float* __restrict__ S32) {
  const int nchunks = (g.nz + kc - 1) / kc;
  const int gx = (g.nx + 6) / 7, gy = (g.ny + 6) / 7;
  const int ncols = g.nx * g.ny;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ncols * nchunks; t += gridDim.x * blockDim.x) {
    const int i = t % g.nx, r = t / g.nx, j = r % g.ny, ch = r / g.ny;
    const int k0 = ch * kc, k1 = min(k0 + kc, g.nz);
    // the four element columns around node column (i, j): ex = i - 1 + a,
    // ey = j - 1 + b; this node is their local corner (1 - a, 1 - b)
    bool ok[4];
    double ahx[4], ahy[4], axy[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ex = i - 1 + (q & 1), ey = j - 1 + (q >> 1);
      ok[q] = ex >= 0 && ex <= g.nx - 2 && ey >= 0 && ey <= g.ny - 2;
      const int cx = min(max(ex, 0), g.nx - 2), cy = min(max(ey, 0), g.ny - 2);
      const double hx = g.x[cx + 1] - g.x[cx], hy = g.y[cy + 1] - g.y[cy];
      ahx[q] = hy / hx;
      ahy[q] = hx / hy;
      axy[q] = hx * hy;
    }
    // the row sums layer ez gives the node column's nodes at ez (bottom) and
    // ez + 1 (top)
    auto layer = [&](int ez, double& bot, double& top) {
      bot = top = 0.0;
      const double hz = g.z[ez + 1] - g.z[ez];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!ok[q]) continue;
        const int ex = i - 1 + (q & 1), ey = j - 1 + (q >> 1);
        const double e = eps[(long)ex + (long)(g.nx - 1) * ((long)ey + (long)(g.ny - 1) * ez)];
        const double sx = e * ahx[q] * hz, sy = e * ahy[q] * hz, sz = e * axy[q] / hz;
        double st = 0.0;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
          const bool dx = d & 1, dy = d & 2, dz = d & 4;
          const double kx = dx ? -1.0 : 1.0, ky = dy ? -1.0 : 1.0, kz = dz ? -1.0 : 1.0;
          const double mx = dx ? 1.0 / 6.0 : 1.0 / 3.0, my = dy ? 1.0 / 6.0 : 1.0 / 3.0,
                       mz = dz ? 1.0 / 6.0 : 1.0 / 3.0;
          st += fabs(sx * kx * my * mz + sy * mx * ky * mz + sz * mx * my * kz);
        }
        bot += st;
        top += st;
        const long sl = tile_slot(ex, ey, ez, gx, gy);
        if (cflag[sl]) {
          double c[8], ones[8], out[8];
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            c[m] = cq[8 * sl + m];
            ones[m] = 1.0;
          }
          jv_element<double, false>(ones, 0.0, 0.0, 0.0, c, true, out);
          const int li = (1 - (q & 1)) + 2 * (1 - (q >> 1));
          bot += out[li];
          top += out[li + 4];
        }
      }
    };
    double carry = 0.0, bot, top;
    if (k0 > 0) layer(k0 - 1, bot, carry);
    for (int k = k0; k < k1; ++k) {
      bot = top = 0.0;
      if (k <= g.nz - 2) layer(k, bot, top);
      const double sum = carry + bot;
      carry = top;
      const long n = (long)i + (long)g.nx * ((long)j + (long)g.ny * k);
      const double sn = mask[n] || !(sum > 0.0) ? 0.0 : omega / sum;
      S[n] = sn;
      if (S32) S32[n] = (float)sn;
    }
  }
}

static int mg_blocks(long n, long cap) {
  return (int)std::max(1L, std::min((n + kVecThreads - 1) / kVecThreads, cap));
}

void launch_mg_inject(hipStream_t s, const MgGrid& f, const MgGrid& c, const double* phif, double* phic) {
  QE_LAUNCH(k_mg_inject, mg_blocks(c.N, 4096), kVecThreads, s, f.g.nx, f.g.ny, f.g.nz, c.g.nx, c.g.ny, c.g.nz, phif,
            phic);
}

void launch_mg_l1(hipStream_t s, const MgGrid& L, const double* eps_natural, const uint8_t* cflag, double omega,
                  bool fp32) {
  // chunks of 8 layers on large meshes, shorter (more threads) on small ones
  const int kc = (int)std::max(1L, std::min(8L, L.N / 262144));
  const long threads = (long)L.g.nx * L.g.ny * ((L.g.nz + kc - 1) / kc);
  QE_LAUNCH(k_mg_l1, mg_blocks(threads, 8192), kVecThreads, s, L.g, eps_natural, cflag, L.cq, L.mask, omega, kc, L.S,
            fp32 ? L.S32 : nullptr);
}

void launch_mg_coarsen_states(hipStream_t s, const qe_problem* f, const qe_problem* c) {
  const long Nc = (long)c->nx * c->ny * c->nz;
  const qe_quantum& qf = *f->quantum;
  const qe_quantum& qc = *c->quantum;
  QE_LAUNCH(k_mg_coarsen_states, mg_blocks(Nc, 4096), kVecThreads, s, f->nx, f->ny, f->nz, c->nx, c->ny, c->nz,
            qf.n_states, qf.psi2, qf.phi_k, qf.region, const_cast<double*>(qc.psi2), const_cast<double*>(qc.phi_k),
            const_cast<uint8_t*>(qc.region));
}

void launch_mg_tables(hipStream_t s, const MgGrid& f, const MgGrid& c) {
  QE_LAUNCH(k_mg_tables, 1, kVecThreads, s, f.g.nx, f.g.ny, f.g.nz, c.g.nx, c.g.ny, c.g.nz, f.g.x, f.g.y, f.g.z, c.tab);
}

void launch_mg_start_fin(hipStream_t s, PcgCtx* ctx, const double* part, int n) {
  QE_LAUNCH(k_mg_start_fin, 1, kVecThreads, s, ctx, part, n);
}

// A level's arrays in the V-cycle's precision.
template <typename T>
struct MgView;
template <>
struct MgView<double> {
  const double *eps, *cq, *S;
  double *b, *x, *y;
  explicit MgView(const MgGrid& G) : eps(G.eps_t), cq(G.cq), S(G.S), b(G.b), x(G.x), y(G.y) {}
};
template <>
struct MgView<float> {
  const float *eps, *cq, *S;
  float *b, *x, *y;
  explicit MgView(const MgGrid& G) : eps(G.eps32), cq(G.cq32), S(G.S32), b(G.b32), x(G.x32), y(G.y32) {}
};

// b_c = P^T (b - y) and x_c = S_c b_c from level A onto level C (y = NULL:
// P^T b).  The tiled form on every level: one thread per coarse node
// gathering its 27 taps from memory took 17.3 us onto 65x65x33 against 11.3,
// and a group of 16 lanes per coarse node on the levels below 65536 nodes
// made the 129x129x65 adjoint 1 % slower.
template <typename T>
static void restrict_to(hipStream_t s, const MgGrid& A, const MgGrid& C, const T* b, const T* y, const MgView<T>& c,
                        const PcgCtx* ctx) {
  const int tnx = mg_ntiles(C.g.nx, kRtX), tny = mg_ntiles(C.g.ny, kRtY), tnz = mg_ntiles(C.g.nz, kRtZ);
  if (y)
    QE_LAUNCH((k_mg_restrict_tile<T, true>), tnx * tny * tnz, kVecThreads, s, A.g.nx, A.g.ny, A.g.nz, C.g.nx, C.g.ny,
              C.g.nz, tnx, tny, tnz, C.tab, A.mask, b, y, C.mask, c.S, c.b, c.x, ctx);
  else
    QE_LAUNCH((k_mg_restrict_tile<T, false>), tnx * tny * tnz, kVecThreads, s, A.g.nx, A.g.ny, A.g.nz, C.g.nx,
              C.g.ny, C.g.nz, tnx, tny, tnz, C.tab, A.mask, b, y, C.mask, c.S, c.b, c.x, ctx);
}

// xo = x + P x_c from level C onto level A (xo may be x); with part (grid
// = nb blocks), one b^T xo partial per block.
template <typename T>
static void prolong_to(hipStream_t s, const MgGrid& A, const MgGrid& C, const T* xc, const T* x, T* xo,
                       const T* bdot, double* part, int nb, const PcgCtx* ctx) {
  QE_LAUNCH(k_mg_prolong<T>, part ? nb : mg_blocks(A.N, 8192), kVecThreads, s, A.g.nx, A.g.ny, A.N, C.g.nx, C.g.ny,
            C.tab, A.mask, xc, x, xo, bdot, part, ctx);
}

// The V-cycle below level l (levels l .. nlev-1).  On entry level l holds
// b (its right-hand side) and x = S b; returns the array that holds B_l b
// (x or y: a smoothing step writes the other one).  Level 0's last
// smoothing step writes one b^T x partial per block into part (cgblocks
// blocks), and its result is always x.
template <typename T>
static T* vcycle(hipStream_t s, const MgGrid* L, int l, int nlev, int sweeps, bool add_top, int cgblocks,
                 double* part, const PcgCtx* ctx) {
  const MgGrid& A = L[l];
  const MgView<T> a(A);
  auto jv = [&]() {
    QE_LAUNCH(k_mg_jv<T>, A.wm.nblocks, 256, s, A.g, A.wm, a.eps, A.cbits, a.cq, A.mask, a.x, a.y, ctx);
  };
  auto jv_smooth = [&](const T* xin, T* xout, double* p, int nb) {
    QE_LAUNCH(k_mg_jv_smooth<T>, nb, 256, s, A.g, A.wm, a.eps, A.cbits, a.cq, A.mask, xin, (const T*)a.b, a.S, xout,
              p, ctx);
  };
  if (l == nlev - 1) {
    T* cur = a.x;
    T* nxt = a.y;
    for (int k = 1; k < sweeps; ++k) {
      jv_smooth(cur, nxt, nullptr, A.wm.nblocks);
      std::swap(cur, nxt);
    }
    return cur;
  }
  const MgGrid& C = L[l + 1];
  const MgView<T> c(C);
  if (l == 0 && add_top) {
    // additive top level: z = S r + P B_1 P^T r, no smoothing products on
    // the finest mesh (positive definite as a sum of positive definite and
    // semidefinite parts)
    restrict_to(s, A, C, a.b, (const T*)nullptr, c, ctx);
    const T* xc = vcycle<T>(s, L, l + 1, nlev, sweeps, add_top, cgblocks, part, ctx);
    prolong_to<T>(s, A, C, xc, a.x, a.x, (const T*)a.b, part, cgblocks, ctx);
    return a.x;
  }
  jv();
  restrict_to(s, A, C, a.b, (const T*)a.y, c, ctx);
  const T* xc = vcycle<T>(s, L, l + 1, nlev, sweeps, add_top, cgblocks, part, ctx);
  if (l > 0) {
    prolong_to<T>(s, A, C, xc, a.x, a.x, (const T*)nullptr, (double*)nullptr, 0, ctx);
    jv_smooth(a.x, a.y, nullptr, A.wm.nblocks);
    return a.y;
  }
  if (A.wm.nblocks <= cgblocks) {
    // the finest level's last step in one launch too: interpolate into y,
    // smooth from y into x (the CG's z), with the r^T z partials in the
    // CG's block count
    prolong_to<T>(s, A, C, xc, a.x, a.y, (const T*)nullptr, (double*)nullptr, 0, ctx);
    jv_smooth(a.y, a.x, part, cgblocks);
    return a.x;
  }
  prolong_to<T>(s, A, C, xc, a.x, a.x, (const T*)nullptr, (double*)nullptr, 0, ctx);
  jv();
  QE_LAUNCH(k_mg_smooth<T>, cgblocks, kVecThreads, s, A.N, a.b, a.y, a.S, a.x, part, ctx);
  return a.x;
}

void launch_mg_vcycle(hipStream_t s, const MgGrid* levels, int nlev, int sweeps, bool add_top, int cgblocks,
                      double* part_rz, const PcgCtx* ctx, bool fp32) {
  if (fp32)
    vcycle<float>(s, levels, 0, nlev, sweeps, add_top, cgblocks, part_rz, ctx);
  else
    vcycle<double>(s, levels, 0, nlev, sweeps, add_top, cgblocks, part_rz, ctx);
}

}  // namespace qe
