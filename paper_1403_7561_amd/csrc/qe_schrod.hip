// Effective-mass Schrodinger eigenpairs on the Q1 mesh (Sec. II.B, Eqs.
// SchrodEqn, SchrodEqnWeakForm) by block LOBPCG.
//
// Both operators of H psi = E M psi go through the wave-tiled J.v kernel:
// H' = H - sigma M is "stiffness weighted by (hbar^2/2m0)(m0/m*) plus Gauss-
// point coefficients W (V_q - sigma)", M is "zero stiffness plus
// coefficients W" -- the same element operator as the Poisson Jacobian.
// sigma lies below every V, so H' is SPD and the Jacobi preconditioner is
// positive.  Fixed nodes (psi = 0) are masked: every block vector is zero
// there and the J.v writes zero rows.
//
// One LOBPCG iteration: residuals R = H'X - M X diag(lambda) and their norms
// (device), soft locking of converged columns (host decision), W = D^-1 R
// for the active ones and its H', M products, the Gram matrices of
// [X, W, P] under H' and M (one pass over the three blocks on the FP64
// matrix cores), the small
// generalized eigenproblem on the host (column scaling, Cholesky, cyclic
// Jacobi), and the new X, P (with their products) in one streaming pass
// (the update is memory bound: k reads and 2 nb writes per row).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/qe.h"
#include "qe_kernels.h"
#include "qe_runtime.h"
#include "qe_tiles.h"

namespace qe {

// hbar^2 / (2 m0) in eV nm^2 (CODATA 2018)
static const double kHB2M = 1.054571817e-34 * 1.054571817e-34 / (2.0 * 9.1093837015e-31) / 1.602176634e-19 * 1e18;
constexpr int kSchBlocks = 256;
constexpr int kMaxCols = QE_MAX_EIG + 2;
constexpr int kGramBlocks = 512;   // row ranges of the Gram matrices

// Input checks: bit 1 inv_mass not finite / positive, 2 v0 not finite, 4 phi not finite.
__global__ __launch_bounds__(kVecThreads) void k_sch_validate(long E, long N, const double* __restrict__ inv_mass,
                                                             const double* __restrict__ v0,
                                                             const double* __restrict__ phi, int* flags) {
  int f = 0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double m = inv_mass[a * E + e];
      if (!(m > 0.0) || !isfinite(m)) f |= 1;
    }
    if (!isfinite(v0[e])) f |= 2;
  }
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x)
    if (!isfinite(phi[n])) f |= 4;
  if (f) atomicOr(flags, f);
}

__device__ __forceinline__ void elem_ijk(const Geom& g, long e, int& i, int& j, int& k) {
  const long ex = g.nx - 1, ey = g.ny - 1;
  i = (int)(e % ex);
  j = (int)((e / ex) % ey);
  k = (int)(e / (ex * ey));
}

// Per block: min over elements of v0_e - phi at the element's corners (a
// lower bound of V at every Gauss point, which interpolates phi).
__global__ __launch_bounds__(kVecThreads) void k_sch_vmin(Geom g, const double* __restrict__ v0,
                                                         const double* __restrict__ phi, double* __restrict__ part) {
  __shared__ double sred[kVecThreads / 64];
  const long E = (long)(g.nx - 1) * (g.ny - 1) * (g.nz - 1);
  double m = INFINITY;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (long)gridDim.x * blockDim.x) {
    int i, j, k;
    elem_ijk(g, e, i, j, k);
    const long n0 = (long)i + (long)g.nx * ((long)j + (long)g.ny * k);
    const long sy = g.nx, sz = (long)g.nx * g.ny;
    double pm = phi[n0];
    pm = fmax(pm, phi[n0 + 1]);
    pm = fmax(pm, phi[n0 + sy]);
    pm = fmax(pm, phi[n0 + sy + 1]);
    pm = fmax(pm, phi[n0 + sz]);
    pm = fmax(pm, phi[n0 + sz + 1]);
    pm = fmax(pm, phi[n0 + sz + sy]);
    pm = fmax(pm, phi[n0 + sz + sy + 1]);
    m = fmin(m, v0[e] - pm);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_down(m, o, 64));
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sred[0];
    for (int w = 1; w < kVecThreads / 64; ++w) r = fmin(r, sred[w]);
    part[blockIdx.x] = r;
  }
}

// Tile-major operator data: kinetic weights (hbar^2/2m0)(m0/m*_a) along
// a = x, y, z (three planes of nslots) and the Gauss-point coefficients
// W (V_q - sigma) of H', W of M.
__global__ __launch_bounds__(kVecThreads) void k_sch_coef(Geom g, const double* __restrict__ inv_mass,
                                                         const double* __restrict__ v0,
                                                         const double* __restrict__ phi, double sigma, double hb2m,
                                                         double* __restrict__ eH, double* __restrict__ cH) {
  const long E = (long)(g.nx - 1) * (g.ny - 1) * (g.nz - 1);
  const int tgx = (g.nx + 6) / 7, tgy = (g.ny + 6) / 7;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (long)gridDim.x * blockDim.x) {
    int i, j, k;
    elem_ijk(g, e, i, j, k);
    const long n0 = (long)i + (long)g.nx * ((long)j + (long)g.ny * k);
    const long sy = g.nx, sz = (long)g.nx * g.ny;
    double q[8] = {phi[n0], phi[n0 + 1], phi[n0 + sy], phi[n0 + sy + 1],
                   phi[n0 + sz], phi[n0 + sz + 1], phi[n0 + sz + sy], phi[n0 + sz + sy + 1]};
    gauss_interp(q);
    const double W = (g.x[i + 1] - g.x[i]) * (g.y[j + 1] - g.y[j]) * (g.z[k + 1] - g.z[k]) * 0.125;
    const double ve = v0[e];
    double ch[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) ch[t] = W * (ve - q[t] - sigma);
    const long sl = tile_slot(i, j, k, tgx, tgy);
    const long nslots = (long)tgx * tgy * 49 * (g.nz - 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) eH[a * nslots + sl] = hb2m * inv_mass[a * E + e];
    store8(cH + 8 * sl, ch);
  }
}

// Fixed-node flags of every lane of the operator sweep: bit L - Lbeg is set
// when the lane's owned node of layer L is fixed.
__global__ __launch_bounds__(256) void k_sch_mbits(Geom g, WaveMap wm, const uint8_t* __restrict__ mask,
                                                   unsigned int* __restrict__ mbits) {
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= wm.nwaves) return;
  int wx, wy, wz;
  wave_tile_of(w, wm, wx, wy, wz);
  const WaveTile t(g, wx, wy, wz, wm.kz, threadIdx.x & 63, true);
  unsigned int b = 0;
  if (t.node_ok)
    for (int L = t.k0; L <= t.Lend; ++L)
      if (mask[t.node(g, L)]) b |= 1u << (L - t.Lbeg);
  mbits[64L * w + (threadIdx.x & 63)] = b;
}

// H and M applied to columns c0 .. c0 + ncols - 1 of Z (column stride N):
// block (bx, by) sweeps four wave tiles for columns c0 + 2 by and the next.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_sch_apply(
    Geom g, WaveMap wm, const double* __restrict__ eH, const double* __restrict__ cH,
    const unsigned int* __restrict__ mbits, long N, int c0, int ncols, const double* __restrict__ Z,
    double* __restrict__ HZ, double* __restrict__ MZ) {
  const int w = __builtin_amdgcn_readfirstlane(wave_of_block(blockIdx.x, wm) * 4 + (threadIdx.x >> 6));
  const bool active = w < wm.nwaves;
  int wx, wy, wz;
  wave_tile_of(w, wm, wx, wy, wz);
  const WaveTile t(g, wx, wy, wz, wm.kz, threadIdx.x & 63, active);
  const unsigned int mb = mbits[64L * min(w, wm.nwaves - 1) + (threadIdx.x & 63)];
  const int ca = c0 + 2 * (int)blockIdx.y;
  const bool ok[2] = {true, ca + 1 < c0 + ncols};
  const int cb = ok[1] ? ca + 1 : ca;
  const double* const zc[2] = {Z + (long)ca * N, Z + (long)cb * N};
  double* const yh[2] = {HZ + (long)ca * N, HZ + (long)cb * N};
  double* const ym[2] = {MZ + (long)ca * N, MZ + (long)cb * N};
  jv_tile_hm(g, t, wm.kz, eH, cH, mb, zc, yh, ym, ok);
}

// Jacobi preconditioner: 1 / (kinetic diagonal + consistent-mass diagonal
// times (v0_e - phi_n - sigma)) on free nodes, 0 on fixed ones.
__global__ __launch_bounds__(kVecThreads) void k_sch_diag(Geom g, const double* __restrict__ inv_mass,
                                                         const double* __restrict__ v0,
                                                         const double* __restrict__ phi,
                                                         const uint8_t* __restrict__ mask, double sigma,
                                                         double hb2m, double* __restrict__ dinv) {
  const long N = (long)g.nx * g.ny * g.nz, Ecount = (long)(g.nx - 1) * (g.ny - 1) * (g.nz - 1);
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    if (mask[n]) {
      dinv[n] = 0.0;
      continue;
    }
    const int i = (int)(n % g.nx), j = (int)((n / g.nx) % g.ny), k = (int)(n / ((long)g.nx * g.ny));
    double d = 0.0;
    for (int dk = -1; dk <= 0; ++dk)
      for (int dj = -1; dj <= 0; ++dj)
        for (int di = -1; di <= 0; ++di) {
          const int ei = i + di, ej = j + dj, ek = k + dk;
          if (ei < 0 || ei >= g.nx - 1 || ej < 0 || ej >= g.ny - 1 || ek < 0 || ek >= g.nz - 1) continue;
          const long e = (long)ei + (long)(g.nx - 1) * ((long)ej + (long)(g.ny - 1) * ek);
          const double hx = g.x[ei + 1] - g.x[ei], hy = g.y[ej + 1] - g.y[ej], hz = g.z[ek + 1] - g.z[ek];
          d += hb2m * (inv_mass[e] * (hy * hz / hx) + inv_mass[Ecount + e] * (hx * hz / hy) +
                       inv_mass[2 * Ecount + e] * (hx * hy / hz)) * (1.0 / 9.0);
          d += hx * hy * hz * (1.0 / 27.0) * fmax(v0[e] - phi[n] - sigma, 0.0);
        }
    dinv[n] = d > 0.0 ? 1.0 / d : 0.0;
  }
}

// Starting block: SplitMix64 (Steele, Lea, Flood 2014) of (seed, column,
// node) mapped to [-1, 1), zero on fixed nodes.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// A box of nodes [i0, i0 + bx) x [j0, j0 + by) x [k0, k0 + bz) of a gx x gy x gz
// mesh, x fastest in both numberings.
struct BoxMap {
  int bx, by, bz, i0, j0, k0, gx, gy;
};
__device__ __forceinline__ long box_to_mesh(const BoxMap& b, long n) {
  const int i = (int)(n % b.bx), j = (int)((n / b.bx) % b.by), k = (int)(n / ((long)b.bx * b.by));
  return (long)(i + b.i0) + (long)b.gx * ((long)(j + b.j0) + (long)b.gy * (k + b.k0));
}

// The random numbers are drawn by mesh node index, so a box's block equals
// the mesh's block restricted to it.
__global__ __launch_bounds__(kVecThreads) void k_sch_rand(long N, int ncol, uint64_t seed, BoxMap bm,
                                                         const uint8_t* __restrict__ mask, double* __restrict__ X) {
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x)
    for (int c = 0; c < ncol; ++c) {
      const uint64_t r = splitmix64(seed ^ splitmix64((uint64_t)c * 0x100000001B3ull + (uint64_t)box_to_mesh(bm, n)));
      const double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);   // [0, 1)
      X[(long)c * N + n] = mask[n] ? 0.0 : 2.0 * u - 1.0;
    }
}

__global__ __launch_bounds__(kVecThreads) void k_sch_mask(long N, int ncol, const uint8_t* __restrict__ mask,
                                                         double* __restrict__ X) {
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x)
    if (mask[n])
      for (int c = 0; c < ncol; ++c) X[(long)c * N + n] = 0.0;
}

// Bounding box of the nodes that are not fixed, as maxima that start at 0:
// b[d] = max (n_d - 1 - i_d) and b[3 + d] = max (i_d + 1) over those nodes.
__global__ __launch_bounds__(kVecThreads) void k_sch_box(int nx, int ny, long N, const uint8_t* __restrict__ fixed,
                                                        int* __restrict__ b) {
  const int nz = (int)(N / ((long)nx * ny));
  int m[6] = {0, 0, 0, 0, 0, 0};
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    if (fixed[n]) continue;
    const int i = (int)(n % nx), j = (int)((n / nx) % ny), k = (int)(n / ((long)nx * ny));
    m[0] = max(m[0], nx - 1 - i);
    m[1] = max(m[1], ny - 1 - j);
    m[2] = max(m[2], nz - 1 - k);
    m[3] = max(m[3], i + 1);
    m[4] = max(m[4], j + 1);
    m[5] = max(m[5], k + 1);
  }
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    for (int o = 32; o > 0; o >>= 1) m[d] = max(m[d], __shfl_xor(m[d], o, 64));
    if ((threadIdx.x & 63) == 0 && m[d] > 0) atomicMax(b + d, m[d]);
  }
}

// dst[c][n] = src[c][mesh index of box node n] for the ncol columns.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_sch_box_gather(BoxMap bm, int ncol, long sstride,
                                                               const T* __restrict__ src, T* __restrict__ dst) {
  const long nb = (long)bm.bx * bm.by * bm.bz;
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < nb; n += (long)gridDim.x * blockDim.x) {
    const long m = box_to_mesh(bm, n);
    for (int c = 0; c < ncol; ++c) dst[c * nb + n] = src[c * sstride + m];
  }
}

// The box's columns back on the whole mesh, 0 outside the box; psi2 (if
// not NULL) receives their squares.
__global__ __launch_bounds__(kVecThreads) void k_sch_box_scatter(BoxMap bm, long N, int ncol,
                                                                const double* __restrict__ src,
                                                                double* __restrict__ psi, double* __restrict__ psi2) {
  const long nb = (long)bm.bx * bm.by * bm.bz;
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    const int i = (int)(n % bm.gx) - bm.i0, j = (int)((n / bm.gx) % bm.gy) - bm.j0,
              k = (int)(n / ((long)bm.gx * bm.gy)) - bm.k0;
    const bool in = i >= 0 && i < bm.bx && j >= 0 && j < bm.by && k >= 0 && k < bm.bz;
    const long l = in ? (long)i + (long)bm.bx * ((long)j + (long)bm.by * k) : 0;
    for (int c = 0; c < ncol; ++c) {
      const double v = in ? src[c * nb + l] : 0.0;
      psi[c * N + n] = v;
      if (psi2) psi2[c * N + n] = v * v;
    }
  }
}

struct ColMap {
  int n;
  int src[kMaxCols];
  int dst[kMaxCols];
  double lam[kMaxCols];
};

// Columns of the Rayleigh-Ritz basis: 0 .. k0-1 are those of Z (and H'Z, MZ);
// k0 + i is column src[i] of P (and HP, MP), read in place.  P is stored
// right after its block's K columns, so basis column c is column
// basis_col(c) of the block.
struct PCols {
  int k0, K;
  int src[kMaxCols];
};
__device__ __forceinline__ long basis_col(const PCols& pc, int c) {
  return c < pc.k0 ? c : pc.K + pc.src[c - pc.k0];
}

// Per block and column c of the map: partial sums of |r|^2, |H'x|^2, |Mx|^2
// with r = H'x - lam M x (blockIdx.y = column).
__global__ __launch_bounds__(kVecThreads) void k_sch_norms(long N, ColMap cm, const double* __restrict__ HX,
                                                          const double* __restrict__ MX, double* __restrict__ part) {
  __shared__ double sred[kVecThreads / 64];
  const int c = blockIdx.y;
  const long o = (long)cm.src[c] * N;
  const double lam = cm.lam[c];
  double r2 = 0.0, h2 = 0.0, m2 = 0.0;
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    const double h = HX[o + n], m = MX[o + n];
    const double r = h - lam * m;
    r2 += r * r;
    h2 += h * h;
    m2 += m * m;
  }
  const double a = block_sum(r2, sred), b = block_sum(h2, sred), d = block_sum(m2, sred);
  if (threadIdx.x == 0) {
    double* p = part + ((long)c * 3) * gridDim.x + blockIdx.x;
    p[0] = a;
    p[gridDim.x] = b;
    p[2 * gridDim.x] = d;
  }
}

// out[c] = sum of the gridDim-wide partial rows (fixed order), one block per row.
__global__ __launch_bounds__(kVecThreads) void k_sch_rowsum(const double* __restrict__ part, int nper,
                                                           double* __restrict__ out) {
  __shared__ double sred[kVecThreads / 64];
  double a = 0.0;
  for (int i = threadIdx.x; i < nper; i += blockDim.x) a += part[(long)blockIdx.x * nper + i];
  const double s = block_sum(a, sred);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// W[dst] = D^-1 (H'x - lam M x) for the mapped columns.
__global__ __launch_bounds__(kVecThreads) void k_sch_precond(long N, ColMap cm, const double* __restrict__ HX,
                                                            const double* __restrict__ MX,
                                                            const double* __restrict__ dinv, double* __restrict__ Z) {
  const int c = blockIdx.y;
  const long o = (long)cm.src[c] * N, d = (long)cm.dst[c] * N;
  const double lam = cm.lam[c];
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x)
    Z[d + n] = dinv[n] * (HX[o + n] - lam * MX[o + n]);
}

// The Rayleigh-Ritz update of one operator's block (blockIdx.y: the block
// vectors Z, H'Z, MZ): X <- S C, in place in Z's first nb columns, and
// (with_p) P <- S[:, nb:k] C[nb:k, :], where S is the basis [X W P] (pc:
// P's columns read in place, before this thread overwrites its rows of P), formed first so that X = P +
// Z[:, :nb] C[:nb, :] takes k nb products per row, not (2k - nb) nb.  C (k x
// nb, column-major) is staged in LDS transposed (row j's nb coefficients
// adjacent, rows padded to even), so one 16-byte LDS read serves two
// products; each thread owns whole rows, so reading a row before writing it
// back is safe.  A streaming pass: k reads and 2 nb writes per row.
__global__ __launch_bounds__(kVecThreads) void k_sch_update(long N, int k, int nb, int with_p, PCols pc,
                                                           const double* __restrict__ C, double* Z, double* HZ,
                                                           double* MZ, double* P, double* HP, double* MP) {
  constexpr int kLd = (kMaxCols + 1) & ~1;
  __shared__ __attribute__((aligned(16))) double sc[3 * kMaxCols * kLd];
  for (int i = threadIdx.x; i < 3 * kMaxCols * kLd; i += blockDim.x) {
    const int j = i / kLd, c = i % kLd;
    sc[i] = (j < k && c < nb) ? C[c * k + j] : 0.0;
  }
  __syncthreads();
  double* const Zs[3] = {Z, HZ, MZ};
  double* const Ps[3] = {P, HP, MP};
  double* const B = Zs[blockIdx.y];
  double* const Pb = Ps[blockIdx.y];
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    double ax[kMaxCols];
#pragma unroll
    for (int c = 0; c < kMaxCols; ++c) ax[c] = 0.0;
    // columns nb .. k-1 (P's part), then 0 .. nb-1 on top of it
    auto accumulate = [&](int jb, int je) {
      for (int j0 = jb; j0 < je; j0 += 6) {
        double z[6];   // six loads in flight before any is used
#pragma unroll
        for (int u = 0; u < 6; ++u) z[u] = j0 + u < je ? B[basis_col(pc, j0 + u) * N + n] : 0.0;
#pragma unroll
        for (int u = 0; u < 6; ++u) {
          const int j = j0 + u;
          if (j >= je) break;
          const double2* row = reinterpret_cast<const double2*>(sc + j * kLd);
#pragma unroll
          for (int c = 0; c < kMaxCols; c += 2)
            if (c < nb) {
              const double2 cc = row[c / 2];
              ax[c] += z[u] * cc.x;
              if (c + 1 < kMaxCols) ax[c + 1] += z[u] * cc.y;
            }
        }
      }
    };
    accumulate(nb, k);
    double ap[kMaxCols];
#pragma unroll
    for (int c = 0; c < kMaxCols; ++c) ap[c] = ax[c];
    accumulate(0, nb);
#pragma unroll
    for (int c = 0; c < kMaxCols; ++c) {
      if (c < nb) {
        B[(long)c * N + n] = ax[c];
        if (with_p) Pb[(long)c * N + n] = ap[c];
      }
    }
  }
}

// Both Gram matrices of the basis S = [X W P], S^T H'S and S^T MS (k x k each,
// k <= 54; pc: P's columns read in place),
// on the FP64 matrix cores: per block over its rows, slabs of kGramRows rows
// of Z, H'Z and MZ are staged in LDS (columns padded to 64 with zeros), and
// each wave accumulates 16 x 16 output tiles with v_mfma_f64_16x16x4f64,
// four rows per instruction.  Operand layout of that instruction (checked on
// the device): lane l supplies A[l % 16][l / 16] of the 16 x 4 left operand
// and B[l / 16][l % 16] of the 4 x 16 right one, and holds
// D[l / 16 + 4 r][l % 16] in accumulator element r.  Both matrices are
// symmetric, so only the tiles on and above the diagonal are formed (10 of
// 16) and mirrored on output: waves 0, 1 take Z^T H'Z, waves 2, 3 Z^T MZ,
// five tiles each.  The next slab's loads are in flight (in registers) while
// the current one is multiplied.  One partial per block and entry, summed in
// a fixed order afterwards.
constexpr int kGramRows = 32, kGramLd = 64;
constexpr int kGramPer = (kGramRows * kGramLd + 255) / 256;   // staged values per thread and array
typedef double qe_v4d __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_sch_gram(long N, int k, PCols pc, const double* __restrict__ Z,
                                                  const double* __restrict__ HZ, const double* __restrict__ MZ,
                                                  double* __restrict__ part) {
  __shared__ double sz[kGramRows * kGramLd], sh[kGramRows * kGramLd], sm[kGramRows * kGramLd];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int e = t; e < kGramRows * kGramLd; e += 256) sz[e] = sh[e] = sm[e] = 0.0;
  const int KT = (k + 15) / 16;
  const int g = wave >> 1;                 // 0: Z^T H'Z, 1: Z^T MZ
  const double* sb = g == 0 ? sh : sm;
  // this wave's tiles (I, J), J >= I: (0,0..3), (3,3) or (1,1..3), (2,2..3)
  const int sub = wave & 1;
  const int TI[5] = {sub, sub, sub, sub == 0 ? 0 : 2, sub == 0 ? 3 : 2};
  const int TJ[5] = {sub == 0 ? 0 : 1, sub == 0 ? 1 : 2, sub == 0 ? 2 : 3, sub == 0 ? 3 : 2, 3};
  qe_v4d acc[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) acc[q] = qe_v4d{0.0, 0.0, 0.0, 0.0};
  const long per = (N + gridDim.x - 1) / gridDim.x;
  const long r0 = (long)blockIdx.x * per, r1 = min(N, r0 + per);
  const int li = lane & 15, lk = lane >> 4;
  const int ne = kGramRows * k;             // staged values per array
  double nz[kGramPer], nh[kGramPer], nm[kGramPer];
  auto load_slab = [&](long base) {
    const int rows = (int)min((long)kGramRows, r1 - base);
#pragma unroll
    for (int i = 0; i < kGramPer; ++i) {
      const int e = t + 256 * i;           // e = c * kGramRows + r: coalesced along rows
      const int c = e / kGramRows, r = e % kGramRows;
      const bool in = e < ne && r < rows;
      const long o = in ? basis_col(pc, c) * N + base + r : 0;
      nz[i] = in ? Z[o] : 0.0;
      nh[i] = in ? HZ[o] : 0.0;
      nm[i] = in ? MZ[o] : 0.0;
    }
  };
  if (r0 < r1) load_slab(r0);
  for (long base = r0; base < r1; base += kGramRows) {
    __syncthreads();   // the previous slab's products have read the LDS
#pragma unroll
    for (int i = 0; i < kGramPer; ++i) {
      const int e = t + 256 * i;
      if (e < ne) {
        const int c = e / kGramRows, r = e % kGramRows;
        sz[r * kGramLd + c] = nz[i];
        sh[r * kGramLd + c] = nh[i];
        sm[r * kGramLd + c] = nm[i];
      }
    }
    __syncthreads();
    if (base + kGramRows < r1) load_slab(base + kGramRows);
#pragma unroll 2
    for (int r4 = 0; r4 < kGramRows; r4 += 4) {
      const int row = r4 + lk;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        if (TJ[q] < KT) {   // uniform (J >= I, so I < KT too)
          const double a = sz[row * kGramLd + TI[q] * 16 + li];
          const double b = sb[row * kGramLd + TJ[q] * 16 + li];
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
        }
      }
    }
  }
  double* out = part + ((long)blockIdx.x * 2 + g) * k * k;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    if (TJ[q] >= KT) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = TI[q] * 16 + lk + 4 * r, j = TJ[q] * 16 + li;
      if (i < k && j < k) {
        out[(long)j * k + i] = acc[q][r];   // column-major
        if (TI[q] != TJ[q]) out[(long)i * k + j] = acc[q][r];
      }
    }
  }
}

// G[m * len + i] = sum over the n blocks of part[(b * 2 + m) * len + i], for
// the two matrices m.  A block takes 64 consecutive entries of the two
// matrices; its wave w adds the partials of blocks w, w + 16, ... in order and
// the 16 wave sums are added in wave order: a fixed order, with 16 times the
// loads in flight of one thread per entry.
constexpr int kSumWaves = 16;
__global__ __launch_bounds__(64 * kSumWaves) void k_sch_sum_parts2(const double* __restrict__ part, int n, int len,
                                                                  double* __restrict__ out) {
  __shared__ double acc[kSumWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const bool ok = i < 2 * len;
  const int m = ok ? i / len : 0, e = ok ? i % len : 0;
  double a = 0.0;
  int b = w;
  for (; b + 7 * kSumWaves < n; b += 8 * kSumWaves) {   // eight loads in flight
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[((long)(b + u * kSumWaves) * 2 + m) * len + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) a += v[u];
  }
  for (; b < n; b += kSumWaves) a += part[((long)b * 2 + m) * len + e];
  acc[w][lane] = a;
  __syncthreads();
  if (w == 0 && ok) {
    double t = acc[0][lane];
    for (int j = 1; j < kSumWaves; ++j) t += acc[j][lane];
    out[i] = t;
  }
}

__global__ __launch_bounds__(kVecThreads) void k_sch_square(long n, const double* __restrict__ a,
                                                           double* __restrict__ b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = a[i] * a[i];
}

// ---------------------------------------------------------------- host side
// Eigen-decomposition of the symmetric k x k matrix A (row-major, destroyed):
// Householder reduction to tridiagonal form with the transformations
// accumulated, then the implicit QL iteration with Wilkinson-type shifts on
// the tridiagonal matrix, each plane rotation also applied to the
// accumulated basis (Golub and Van Loan, Matrix Computations, Secs. 8.3.1
// and 8.3.5; Bowdler, Martin, Reinsch and Wilkinson, Numer. Math. 11, 1968).
// V receives the eigenvectors as columns (row-major), w the eigenvalues.
static void sym_eig(int k, std::vector<double>& A, std::vector<double>& V, std::vector<double>& w) {
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * k + j]; };
  // the basis is accumulated transposed (row i = column i of V), so that
  // each transformation updates contiguous rows
  std::vector<double> Qt((size_t)k * k, 0.0);
  auto q = [&](int i, int j) -> double& { return Qt[(size_t)j * k + i]; };
  for (int i = 0; i < k; ++i) q(i, i) = 1.0;
  std::vector<double> v(k), p(k), d(k), e(k, 0.0);
  // reduction: column j's part below the subdiagonal is annihilated by
  // H = I - 2 v v^T / (v^T v) acting on rows / columns j+1 .. k-1
  for (int j = 0; j + 2 < k; ++j) {
    double nx = 0.0;
    for (int i = j + 1; i < k; ++i) nx += a(i, j) * a(i, j);
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    const double x0 = a(j + 1, j);
    const double alpha = x0 >= 0.0 ? -nx : nx;
    double vv = 0.0;
    for (int i = j + 1; i < k; ++i) {
      v[i] = a(i, j);
      if (i == j + 1) v[i] -= alpha;
      vv += v[i] * v[i];
    }
    if (vv == 0.0) continue;
    const double tau = 2.0 / vv;
    // H A H = A - v w^T - w v^T with p = tau A v, w = p - (tau/2)(v^T p) v
    double vp = 0.0;
    for (int i = j + 1; i < k; ++i) {
      double s = 0.0;
      for (int t = j + 1; t < k; ++t) s += a(i, t) * v[t];
      p[i] = tau * s;
      vp += v[i] * p[i];
    }
    const double h = 0.5 * tau * vp;
    for (int i = j + 1; i < k; ++i) p[i] -= h * v[i];
    for (int i = j + 1; i < k; ++i)
      for (int t = j + 1; t < k; ++t) a(i, t) -= v[i] * p[t] + p[i] * v[t];
    a(j + 1, j) = a(j, j + 1) = alpha;
    for (int i = j + 2; i < k; ++i) a(i, j) = a(j, i) = 0.0;
    // V <- V H, i.e. rows j+1 .. k-1 of Qt <- H (those rows)
    for (int r = 0; r < k; ++r) p[r] = 0.0;
    for (int t = j + 1; t < k; ++t) {
      const double* qt = &Qt[(size_t)t * k];
      for (int r = 0; r < k; ++r) p[r] += v[t] * qt[r];
    }
    for (int t = j + 1; t < k; ++t) {
      double* qt = &Qt[(size_t)t * k];
      const double f = tau * v[t];
      for (int r = 0; r < k; ++r) qt[r] -= f * p[r];
    }
  }
  for (int i = 0; i < k; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < k; ++i) e[i] = a(i + 1, i);   // e[i] couples i and i+1
  // implicit QL on (d, e)
  for (int l = 0; l < k; ++l) {
    for (int iter = 0; iter < 60; ++iter) {
      int m = l;
      for (; m + 1 < k; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-16 * dd) break;
      }
      if (m == l) break;
      // shift from the leading 2 x 2 block, the eigenvalue closer to d[l]
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {   // underflow: the chain splits here
          d[i + 1] -= pp;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        double* qi = &Qt[(size_t)i * k];   // the same rotation on columns i, i+1 of V
        double* qi1 = &Qt[(size_t)(i + 1) * k];
        for (int t = 0; t < k; ++t) {
          const double vi = qi[t], vi1 = qi1[t];
          qi1[t] = s * vi + c * vi1;
          qi[t] = c * vi - s * vi1;
        }
      }
      if (deflated) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  w = d;
  V.resize((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) V[(size_t)i * k + j] = Qt[(size_t)j * k + i];
}

// Rayleigh-Ritz on the k x k pencil (GA, GB) (column-major, symmetric):
// the nb lowest eigenvalues into lam and the coefficient matrix C (k x nb,
// column-major) with C^T GB C = I.  The basis [X W P] loses rank as the
// iteration converges (a residual direction falls into the span of the
// others), so GB, scaled to a unit diagonal, is diagonalised and only its
// eigendirections above kRankTol of the largest are kept (the SVQB basis of
// Stathopoulos and Wu, SIAM J. Sci. Comput. 23, 2002): the pencil reduced
// to that range is a standard symmetric eigenproblem.  False if fewer than
// nb directions remain (or GB has a diagonal entry that is not positive).
constexpr double kRankTol = 1e-12;

static bool rayleigh_ritz(int k, int nb, const double* GA, const double* GB, std::vector<double>& lam,
                          std::vector<double>& C) {
  std::vector<double> d(k), B((size_t)k * k), A((size_t)k * k);
  for (int i = 0; i < k; ++i) {
    const double b = GB[(size_t)i * k + i];
    if (!(b > 0.0) || !std::isfinite(b)) return false;
    d[i] = 1.0 / std::sqrt(b);
  }
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      // symmetrised and scaled to a unit diagonal of B
      B[(size_t)i * k + j] = 0.5 * (GB[(size_t)j * k + i] + GB[(size_t)i * k + j]) * d[i] * d[j];
      A[(size_t)i * k + j] = 0.5 * (GA[(size_t)j * k + i] + GA[(size_t)i * k + j]) * d[i] * d[j];
    }
  // B = U diag(mu) U^T; T = U_r diag(mu_r)^-1/2 over the kept directions
  std::vector<double> U, mu;
  sym_eig(k, B, U, mu);
  double mu_max = 0.0;
  for (int i = 0; i < k; ++i) mu_max = std::max(mu_max, mu[i]);
  std::vector<int> keep;
  for (int i = 0; i < k; ++i)
    if (mu[i] > kRankTol * mu_max) keep.push_back(i);
  const int r = (int)keep.size();
  if (r < nb || !(mu_max > 0.0) || !std::isfinite(mu_max)) return false;
  std::vector<double> T((size_t)k * r);   // row-major k x r
  for (int j = 0; j < r; ++j) {
    const double sc = 1.0 / std::sqrt(mu[keep[j]]);
    for (int i = 0; i < k; ++i) T[(size_t)i * r + j] = U[(size_t)i * k + keep[j]] * sc;
  }
  // A_r = T^T A T (r x r), symmetrised
  std::vector<double> AT((size_t)k * r, 0.0), Ar((size_t)r * r, 0.0);
  for (int i = 0; i < k; ++i)
    for (int t = 0; t < k; ++t) {
      const double a = A[(size_t)i * k + t];
      for (int j = 0; j < r; ++j) AT[(size_t)i * r + j] += a * T[(size_t)t * r + j];
    }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double acc = 0.0;
      for (int t = 0; t < k; ++t) acc += T[(size_t)t * r + i] * AT[(size_t)t * r + j];
      Ar[(size_t)i * r + j] = acc;
    }
  for (int i = 0; i < r; ++i)
    for (int j = i + 1; j < r; ++j) {
      const double m = 0.5 * (Ar[(size_t)i * r + j] + Ar[(size_t)j * r + i]);
      Ar[(size_t)i * r + j] = Ar[(size_t)j * r + i] = m;
    }
  std::vector<double> V, w;
  sym_eig(r, Ar, V, w);
  std::vector<int> ord(r);
  for (int i = 0; i < r; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return w[a] < w[b]; });
  lam.resize(nb);
  C.assign((size_t)k * nb, 0.0);
  for (int c = 0; c < nb; ++c) {
    lam[c] = w[ord[c]];
    // C = D T v
    for (int i = 0; i < k; ++i) {
      double acc = 0.0;
      for (int j = 0; j < r; ++j) acc += T[(size_t)i * r + j] * V[(size_t)j * r + ord[c]];
      C[(size_t)c * k + i] = acc * d[i];
    }
  }
  return true;
}

struct SchLayout {
  size_t eH, cH, rdz, mbits, mask, dinv, Z, HZ, MZ, P, HP, MP, G, gpart, C, part, sums, flags;
  size_t total;
};

static SchLayout sch_layout(long N, long nslots, int nz, long nwaves, int nb) {
  SchLayout L;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = (off + b + 255) & ~size_t(255);
    return o;
  };
  const int K = 3 * nb;
  L.eH = take(3 * nslots * 8);
  L.cH = take(nslots * 64);
  L.rdz = take((size_t)(nz - 1) * 16);
  L.mbits = take(nwaves * 64 * 4);
  L.mask = take(N);
  L.dinv = take(N * 8);
  // each block's P follows it: P's column i is the block's column K + i
  L.Z = take((size_t)(K + nb) * N * 8);
  L.P = L.Z + (size_t)K * N * 8;
  L.HZ = take((size_t)(K + nb) * N * 8);
  L.HP = L.HZ + (size_t)K * N * 8;
  L.MZ = take((size_t)(K + nb) * N * 8);
  L.MP = L.MZ + (size_t)K * N * 8;
  L.G = take((size_t)2 * K * K * 8);
  L.gpart = take((size_t)kGramBlocks * 2 * K * K * 8);
  L.C = take((size_t)K * nb * 8);
  L.part = take((size_t)kSchBlocks * 3 * kMaxCols * 8);
  L.sums = take((size_t)3 * kMaxCols * 8);
  L.flags = take(64);
  L.total = off;
  return L;
}

static bool mesh_ok(const qe_problem* p) {
  return p && p->nx >= 2 && p->ny >= 2 && p->nz >= 2 && p->x && p->y && p->z &&
         (long)p->nx * p->ny * p->nz <= (1L << 31) - 1;
}


// LOBPCG on the mesh of p, which is the caller's mesh or a box of it: the
// operators, the iteration and the results (psi, psi2: column stride p's
// node count).  bm places p's nodes in the caller's mesh for the random
// starting block.
static qe_status sch_core(const qe_problem* p, const double* inv_mass, const double* v0, const uint8_t* fixed,
                          const double* phi, double sigma, const BoxMap& bm, int32_t n_states, double tol,
                          int32_t maxit, uint64_t seed, int32_t guess, double* E, double* psi, double* psi2,
                          int32_t* iters, char* ws, size_t ws_bytes, hipStream_t s) {
  const long N = (long)p->nx * p->ny * p->nz;
  const int nb = n_states + 2, K = 3 * nb;
  Geom g{p->nx, p->ny, p->nz, p->x, p->y, p->z, nullptr};
  const WaveMap wm = make_wavemap(p->nx, p->ny, p->nz, 0);
  const SchLayout L = sch_layout(N, tile_slots(p->nx, p->ny, p->nz), p->nz, wm.nwaves, nb);
  if (ws_bytes < L.total) return fail(QE_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  auto f64 = [&](size_t o) { return reinterpret_cast<double*>(ws + o); };
  auto ck = [&](hipError_t e, const char* what) -> qe_status {
    return e == hipSuccess ? QE_OK : fail(QE_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  };
  const int vb = vec_blocks(N);
  // ---- operators
  g.rdz = f64(L.rdz);
  g.hz = g.rdz + (p->nz - 1);
  launch_stage_rdz(s, p->nz, p->z, f64(L.rdz));
  hipLaunchKernelGGL(k_sch_coef, dim3(vb), dim3(kVecThreads), 0, s, g, inv_mass, v0, phi, sigma, kHB2M,
                     f64(L.eH), f64(L.cH));
  uint8_t* mask = reinterpret_cast<uint8_t*>(ws + L.mask);
  if (fixed)
    QE_TRY(ck(hipMemcpyAsync(mask, fixed, N, hipMemcpyDeviceToDevice, s), "copy"));
  else
    QE_TRY(ck(hipMemsetAsync(mask, 0, N, s), "memset"));
  unsigned int* mbits = reinterpret_cast<unsigned int*>(ws + L.mbits);
  hipLaunchKernelGGL(k_sch_mbits, dim3(wm.nblocks), dim3(256), 0, s, g, wm, mask, mbits);
  hipLaunchKernelGGL(k_sch_diag, dim3(vb), dim3(kVecThreads), 0, s, g, inv_mass, v0, phi, mask, sigma, kHB2M,
                     f64(L.dinv));
  double *Z = f64(L.Z), *HZ = f64(L.HZ), *MZ = f64(L.MZ);
  // H and M of columns c0 .. c0 + n - 1 of Z into HZ, MZ (one launch; the
  // columns vanish on the fixed nodes, and so do their images)
  auto apply = [&](int c0, int n) {
    hipLaunchKernelGGL(k_sch_apply, dim3(wm.nblocks, (n + 1) / 2), dim3(256), 0, s, g, wm, f64(L.eH), f64(L.cH),
                       mbits, N, c0, n, Z, HZ, MZ);
  };
  std::vector<double> hG(2 * (size_t)K * K), lam, Cm;
  // Gram matrices of the first k columns, Rayleigh-Ritz, and the new X (and
  // P from columns nb.. when with_p).
  // pc: the basis' P columns (none: pc.k0 = k)
  auto rr_update = [&](int k, bool with_p, const PCols& pc) -> qe_status {
    double* G = f64(L.G);
    hipLaunchKernelGGL(k_sch_gram, dim3(kGramBlocks), dim3(256), 0, s, N, k, pc, Z, HZ, MZ, f64(L.gpart));
    // G (both matrices, column-major, one after the other) = fixed-order sum of the block partials
    hipLaunchKernelGGL(k_sch_sum_parts2, dim3((2 * k * k + 63) / 64), dim3(64 * kSumWaves), 0, s, f64(L.gpart),
                       kGramBlocks, k * k, G);
    QE_TRY(ck(hipGetLastError(), "Gram launch"));
    QE_TRY(ck(hipMemcpyAsync(hG.data(), G, 2 * (size_t)k * k * 8, hipMemcpyDeviceToHost, s), "copy"));
    QE_TRY(ck(hipStreamSynchronize(s), "sync"));
    if (!rayleigh_ritz(k, nb, hG.data(), hG.data() + (size_t)k * k, lam, Cm)) return QE_ERR_KRYLOV_BREAKDOWN;
    QE_TRY(ck(hipMemcpyAsync(f64(L.C), Cm.data(), Cm.size() * 8, hipMemcpyHostToDevice, s), "copy"));
    const int ub = (int)std::max(1L, std::min((N + kVecThreads - 1) / kVecThreads, 1024L));
    hipLaunchKernelGGL(k_sch_update, dim3(ub, 3), dim3(kVecThreads), 0, s, N, k, nb, with_p ? 1 : 0, pc,
                       f64(L.C), Z, HZ, MZ, f64(L.P), f64(L.HP), f64(L.MP));
    return ck(hipGetLastError(), "update launch");
  };
  // ---- starting block
  hipLaunchKernelGGL(k_sch_rand, dim3(vb), dim3(kVecThreads), 0, s, N, nb, seed, bm, mask, Z);
  if (guess) {   // the caller's vectors start the first n_states columns (guards stay random)
    QE_TRY(ck(hipMemcpyAsync(Z, psi, (size_t)n_states * N * 8, hipMemcpyDeviceToDevice, s), "copy"));
    hipLaunchKernelGGL(k_sch_mask, dim3(vb), dim3(kVecThreads), 0, s, N, n_states, mask, Z);
  }
  apply(0, nb);
  PCols nopc;
  std::memset(&nopc, 0, sizeof(nopc));
  nopc.k0 = nb;
  nopc.K = K;
  qe_status st = rr_update(nb, false, nopc);
  if (st != QE_OK) return st == QE_ERR_KRYLOV_BREAKDOWN ? fail(st, "starting block is rank deficient") : st;
  bool have_p = false;
  int it = 0;
  std::vector<double> sums(3 * kMaxCols);
  std::vector<int> active;
  bool converged = false;
  for (it = 1; it <= maxit; ++it) {
    // residual norms of every column
    ColMap cm;
    std::memset(&cm, 0, sizeof(cm));
    cm.n = nb;
    for (int c = 0; c < nb; ++c) {
      cm.src[c] = c;
      cm.lam[c] = lam[c];
    }
    hipLaunchKernelGGL(k_sch_norms, dim3(kSchBlocks, nb), dim3(kVecThreads), 0, s, N, cm, HZ, MZ, f64(L.part));
    hipLaunchKernelGGL(k_sch_rowsum, dim3(3 * nb), dim3(kVecThreads), 0, s, f64(L.part), kSchBlocks, f64(L.sums));
    QE_TRY(ck(hipMemcpyAsync(sums.data(), f64(L.sums), 3 * nb * 8, hipMemcpyDeviceToHost, s), "copy"));
    QE_TRY(ck(hipStreamSynchronize(s), "sync"));
    active.clear();
    bool done = true;
    for (int c = 0; c < nb; ++c) {
      const double r = std::sqrt(sums[3 * c]), h = std::sqrt(sums[3 * c + 1]), m = std::sqrt(sums[3 * c + 2]);
      const double rel = r / std::max(h + std::fabs(lam[c]) * m, 1e-300);
      if (!std::isfinite(rel)) return fail(QE_ERR_NONFINITE, "non-finite residual in the eigensolver");
      if (rel > tol) {
        active.push_back(c);
        if (c < n_states) done = false;
      }
    }
    if (done) {
      converged = true;
      break;
    }
    if (it == maxit) break;
    // W = D^-1 R for the active columns, after X in Z; P's active columns after W
    const int na = (int)active.size();
    ColMap wmap;
    std::memset(&wmap, 0, sizeof(wmap));
    wmap.n = na;
    for (int a = 0; a < na; ++a) {
      wmap.src[a] = active[a];
      wmap.dst[a] = nb + a;
      wmap.lam[a] = lam[active[a]];
    }
    hipLaunchKernelGGL(k_sch_precond, dim3(kSchBlocks, na), dim3(kVecThreads), 0, s, N, wmap, HZ, MZ, f64(L.dinv), Z);
    apply(nb, na);
    const int k = nb + na;
    PCols pc;
    std::memset(&pc, 0, sizeof(pc));
    pc.k0 = k;
    pc.K = K;
    if (have_p) {
      // P's active columns join the basis where they are (no copy)
      for (int a = 0; a < na; ++a) pc.src[a] = active[a];
      st = rr_update(k + na, true, pc);
      if (st == QE_ERR_KRYLOV_BREAKDOWN) st = rr_update(k, true, pc);   // drop P when [X W P] lost rank
    } else {
      st = rr_update(k, true, pc);
    }
    if (st == QE_ERR_KRYLOV_BREAKDOWN) return fail(st, "the LOBPCG basis lost rank at iteration %d", it);
    if (st != QE_OK) return st;
    have_p = true;
  }
  // ---- results: X's first n_states columns
  for (int c = 0; c < n_states; ++c) E[c] = lam[c] + sigma;
  QE_TRY(ck(hipMemcpyAsync(psi, Z, (size_t)n_states * N * 8, hipMemcpyDeviceToDevice, s), "copy"));
  if (psi2) hipLaunchKernelGGL(k_sch_square, dim3(vb), dim3(kVecThreads), 0, s, (long)n_states * N, Z, psi2);
  QE_TRY(ck(hipGetLastError(), "launch"));
  QE_TRY(ck(hipStreamSynchronize(s), "sync"));
  if (iters) *iters = it;
  return converged ? QE_OK : fail(QE_ERR_NOT_CONVERGED, "eigensolver hit maxit (%d)", maxit);
}


}  // namespace qe

using namespace qe;

extern "C" {

size_t qe_schrodinger_workspace_bytes(const qe_problem* p, int32_t n_states) {
  if (!mesh_ok(p) || n_states < 1 || n_states > QE_MAX_EIG) return 0;
  const long N = (long)p->nx * p->ny * p->nz;
  const WaveMap wm = make_wavemap(p->nx, p->ny, p->nz, 0);
  return sch_layout(N, tile_slots(p->nx, p->ny, p->nz), p->nz, wm.nwaves, n_states + 2).total;
}

qe_status qe_schrodinger_solve(const qe_problem* p, const qe_schrodinger* sp, const double* phi, int32_t n_states,
                               double tol, int32_t maxit, uint64_t seed, int32_t guess, double* E, double* psi,
                               double* psi2, int32_t* iters, void* ws_, size_t ws_bytes, void* stream) {
  clear_error();
  if (!mesh_ok(p)) return fail(QE_ERR_INVALID_ARG, "bad mesh (nx, ny, nz >= 2 and x, y, z needed)");
  if (!sp || !sp->inv_mass || !sp->v0) return fail(QE_ERR_INVALID_ARG, "inv_mass / v0 is NULL");
  if (!phi || !E || !psi) return fail(QE_ERR_INVALID_ARG, "phi / E / psi is NULL");
  if (n_states < 1 || n_states > QE_MAX_EIG) return fail(QE_ERR_INVALID_ARG, "n_states outside [1, %d]", QE_MAX_EIG);
  if (!(tol > 0.0 && tol < 1.0)) return fail(QE_ERR_INVALID_ARG, "tol must be in (0, 1)");
  if (maxit < 1) return fail(QE_ERR_INVALID_ARG, "maxit < 1");
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const long N = (long)nx * ny * nz, Ecount = (long)(nx - 1) * (ny - 1) * (nz - 1);
  const int nb = n_states + 2;
  if (N < 4L * nb) return fail(QE_ERR_INVALID_ARG, "mesh too small for %d states", n_states);
  const Geom g{nx, ny, nz, p->x, p->y, p->z, nullptr};
  const WaveMap wm = make_wavemap(nx, ny, nz, 0);
  const SchLayout L = sch_layout(N, tile_slots(nx, ny, nz), nz, wm.nwaves, nb);
  if (!ws_) return fail(QE_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws_) & 255) return fail(QE_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < L.total) return fail(QE_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  char* ws = reinterpret_cast<char*>(ws_);
  hipStream_t s = (hipStream_t)stream;
  auto ck = [&](hipError_t e, const char* what) -> qe_status {
    return e == hipSuccess ? QE_OK : fail(QE_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  };
  const int vb = vec_blocks(N);
  // ---- checks, the shift sigma below every V, and the box of the free nodes
  int* dflags = reinterpret_cast<int*>(ws + L.flags);
  QE_TRY(ck(hipMemsetAsync(dflags, 0, 7 * sizeof(int), s), "memset"));
  double* part = reinterpret_cast<double*>(ws + L.part);
  hipLaunchKernelGGL(k_sch_validate, dim3(vb), dim3(kVecThreads), 0, s, Ecount, N, sp->inv_mass, sp->v0, phi, dflags);
  hipLaunchKernelGGL(k_sch_vmin, dim3(kSchBlocks), dim3(kVecThreads), 0, s, g, sp->v0, phi, part);
  if (sp->fixed) hipLaunchKernelGGL(k_sch_box, dim3(vb), dim3(kVecThreads), 0, s, nx, ny, N, sp->fixed, dflags + 1);
  std::vector<double> hp(kSchBlocks);
  int hf[7] = {0, 0, 0, 0, 0, 0, 0};
  QE_TRY(ck(hipMemcpyAsync(hf, dflags, sizeof(hf), hipMemcpyDeviceToHost, s), "copy"));
  QE_TRY(ck(hipMemcpyAsync(hp.data(), part, kSchBlocks * 8, hipMemcpyDeviceToHost, s), "copy"));
  QE_TRY(ck(hipStreamSynchronize(s), "sync"));
  if (hf[0] & 1) return fail(QE_ERR_INVALID_ARG, "inv_mass must be finite and > 0");
  if (hf[0] & 2) return fail(QE_ERR_NONFINITE, "v0 not finite");
  if (hf[0] & 4) return fail(QE_ERR_NONFINITE, "phi not finite");
  double vmin = INFINITY;
  for (double v : hp) vmin = std::min(vmin, v);
  const double sigma = vmin - 0.1;   // eV below every V: H - sigma M is SPD
  const BoxMap whole{nx, ny, nz, 0, 0, 0, nx, ny};
  // Every node outside the free nodes' bounding box grown by one node is
  // fixed and touches only elements whose nodes are all fixed, so psi is 0
  // there and the box (with its own fixed nodes, and the natural condition
  // wherever it meets the mesh boundary) has the same eigenpairs.
  if (sp->fixed && hf[4] > 0) {
    const int n[3] = {nx, ny, nz};
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::max(n[d] - 1 - hf[1 + d] - 1, 0);
      hi[d] = std::min(hf[4 + d] - 1 + 1, n[d] - 1);
    }
    const BoxMap bm{hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1, lo[0], lo[1], lo[2], nx, ny};
    const long Nb = (long)bm.bx * bm.by * bm.bz, Eb = (long)(bm.bx - 1) * (bm.by - 1) * (bm.bz - 1);
    size_t off = 0;
    auto take = [&](size_t b) {
      const size_t o = off;
      off = (off + b + 255) & ~size_t(255);
      return o;
    };
    const size_t o_psi = take((size_t)n_states * Nb * 8), o_im = take(3 * Eb * 8), o_v0 = take(Eb * 8),
                 o_phi = take(Nb * 8), o_fx = take(Nb);
    const WaveMap wmb = make_wavemap(bm.bx, bm.by, bm.bz, 0);
    const size_t need = off + sch_layout(Nb, tile_slots(bm.bx, bm.by, bm.bz), bm.bz, wmb.nwaves, nb).total;
    if (Nb < N && Nb >= 4L * nb && need <= ws_bytes) {
      qe_problem pb = *p;
      pb.nx = bm.bx;
      pb.ny = bm.by;
      pb.nz = bm.bz;
      pb.x = p->x + bm.i0;
      pb.y = p->y + bm.j0;
      pb.z = p->z + bm.k0;
      const BoxMap em{bm.bx - 1, bm.by - 1, bm.bz - 1, bm.i0, bm.j0, bm.k0, nx - 1, ny - 1};
      double *psib = reinterpret_cast<double*>(ws + o_psi), *imb = reinterpret_cast<double*>(ws + o_im),
             *v0b = reinterpret_cast<double*>(ws + o_v0), *phib = reinterpret_cast<double*>(ws + o_phi);
      uint8_t* fxb = reinterpret_cast<uint8_t*>(ws + o_fx);
      const int gb = vec_blocks(Nb);
      hipLaunchKernelGGL(k_sch_box_gather<double>, dim3(gb), dim3(kVecThreads), 0, s, em, 3, Ecount, sp->inv_mass, imb);
      hipLaunchKernelGGL(k_sch_box_gather<double>, dim3(gb), dim3(kVecThreads), 0, s, em, 1, Ecount, sp->v0, v0b);
      hipLaunchKernelGGL(k_sch_box_gather<double>, dim3(gb), dim3(kVecThreads), 0, s, bm, 1, N, phi, phib);
      hipLaunchKernelGGL(k_sch_box_gather<uint8_t>, dim3(gb), dim3(kVecThreads), 0, s, bm, 1, N, sp->fixed, fxb);
      if (guess)
        hipLaunchKernelGGL(k_sch_box_gather<double>, dim3(gb), dim3(kVecThreads), 0, s, bm, n_states, N, psi, psib);
      QE_TRY(ck(hipGetLastError(), "box launch"));
      const qe_status st = sch_core(&pb, imb, v0b, fxb, phib, sigma, bm, n_states, tol, maxit, seed, guess, E, psib,
                                    nullptr, iters, ws + off, ws_bytes - off, s);
      if (st != QE_OK && st != QE_ERR_NOT_CONVERGED) return st;
      hipLaunchKernelGGL(k_sch_box_scatter, dim3(vb), dim3(kVecThreads), 0, s, bm, N, n_states, psib, psi, psi2);
      QE_TRY(ck(hipGetLastError(), "launch"));
      QE_TRY(ck(hipStreamSynchronize(s), "sync"));
      return st;
    }
  }
  return sch_core(p, sp->inv_mass, sp->v0, sp->fixed, phi, sigma, whole, n_states, tol, maxit, seed, guess, E, psi,
                  psi2, iters, ws, ws_bytes, s);
}

}  // extern "C"
