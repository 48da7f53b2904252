// Interface-charge and Robin face terms (Sec. II.A.5) on mesh-plane sheets.
//
// On a face f (a rectangle of a node plane, sides ha x hb) the weak form
// gains alpha int_f (phi - phi0) w_i - KAPPA sigma_f int_f w_i.  With bilinear
// traces the integrals are exact: int_f w_i = A/4 and int_f w_i w_j = A/36
// times 4 (j = i), 2 (j shares a side with i) or 1 (j is diagonal to i).
// Each node of a sheet is handled by one thread of the first sheet that
// contains it, which sums over every sheet containing it and over the (up to
// four) faces of each around the node, in a fixed order: no atomics, and the
// result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "qe_kernels.h"

namespace qe {

// Position (a, b) of global node n in sheet t, if t contains it.
__device__ __forceinline__ bool sheet_pos(const SheetSet& S, const SheetDev& t, long n, int& a, int& b) {
  const long nxy = (long)S.nx * S.ny;
  const int i = (int)(n % S.nx), j = (int)((n / S.nx) % S.ny), k = (int)(n / nxy);
  int c;
  if (t.axis == 2) {
    c = k; a = i; b = j;
  } else if (t.axis == 1) {
    c = j; a = i; b = k;
  } else {
    c = i; a = j; b = k;
  }
  return c == t.plane && a >= t.a0 && a <= t.a1 && b >= t.b0 && b <= t.b1;
}

// Sheet s and node (a, b) of flat slot t over all sheets' nodes.
__device__ __forceinline__ void sheet_slot(const SheetSet& S, long t, int& s, int& a, int& b) {
  s = 0;
  while (t >= S.start[s + 1]) ++s;
  const SheetDev& d = S.s[s];
  const long loc = t - S.start[s];
  const int na = d.a1 - d.a0 + 1;
  a = d.a0 + (int)(loc % na);
  b = d.b0 + (int)(loc / na);
}

__device__ __forceinline__ long sheet_node(const SheetDev& d, int a, int b) { return d.base + a * d.sa + b * d.sb; }

// Owner test: no sheet before s contains node n.
__device__ __forceinline__ bool sheet_owner(const SheetSet& S, int s, long n) {
  for (int t = 0; t < s; ++t) {
    int a, b;
    if (sheet_pos(S, S.s[t], n, a, b)) return false;
  }
  return true;
}

// The face terms at node n (one of the sheets' nodes): Robin mass product
// sum alpha int_f w_n v (v read through `val`), the constant load
// sum (alpha phi0 + KAPPA sigma) int_f w_n and the diagonal sum alpha int_f w_n^2.
template <typename Val>
__device__ __forceinline__ void sheet_terms_at(const SheetSet& S, int s0, long n, double kappa, Val val,
                                               double& mv, double& load, double& diag) {
  mv = load = diag = 0.0;
  const double vn = val(n);
  for (int t = s0; t < S.n; ++t) {
    const SheetDev& d = S.s[t];
    int a, b;
    if (!sheet_pos(S, d, n, a, b)) continue;
    const int na = d.a1 - d.a0;
    for (int fb = b - 1; fb <= b; ++fb) {
      if (fb < d.b0 || fb >= d.b1) continue;
      const int b2 = fb == b ? b + 1 : b - 1;
      const double hb = d.cb[fb + 1] - d.cb[fb];
      for (int fa = a - 1; fa <= a; ++fa) {
        if (fa < d.a0 || fa >= d.a1) continue;
        const int a2 = fa == a ? a + 1 : a - 1;
        const double A = (d.ca[fa + 1] - d.ca[fa]) * hb;
        const double sg = d.sigma ? d.sigma[(fa - d.a0) + (long)na * (fb - d.b0)] : 0.0;
        load += (d.alpha * d.phi0 + kappa * sg) * (0.25 * A);
        if (d.alpha != 0.0) {
          const double m = d.alpha * A * (1.0 / 36.0);
          mv += m * (4.0 * vn + 2.0 * val(sheet_node(d, a2, b)) + 2.0 * val(sheet_node(d, a, b2)) +
                     val(sheet_node(d, a2, b2)));
          diag += 4.0 * m;
        }
      }
    }
  }
}

// Face contributions to F(phi + lam delta) and to the Jacobian diagonal, on
// free sheet nodes (fsheet, fdiag are read by the residual kernel there).
template <typename TD>
__global__ __launch_bounds__(kVecThreads) void k_sheet_residual(SheetSet S, double kappa,
                                                               const uint8_t* __restrict__ mask,
                                                               const double* __restrict__ phi,
                                                               const TD* __restrict__ delta, double lam,
                                                               double* __restrict__ fsheet,
                                                               double* __restrict__ fdiag) {
  const long total = S.start[S.n];
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    int s, a, b;
    sheet_slot(S, t, s, a, b);
    const long n = sheet_node(S.s[s], a, b);
    if (mask[n] || !sheet_owner(S, s, n)) continue;
    auto val = [=](long j) { return delta ? phi[j] + lam * (double)delta[j] : phi[j]; };
    double mv, load, diag;
    sheet_terms_at(S, s, n, kappa, val, mv, load, diag);
    fsheet[n] = mv - load;
    fdiag[n] = diag;
  }
}

// y_n += (R v)_n on free sheet nodes with v read as 0 on Dirichlet nodes
// (dir_rows: y_n -= (R v)_n on Dirichlet sheet nodes instead, the Robin part
// of the adjoint's contact terms).  In the CG (ctx set) the kernel does
// nothing once the solve has stopped, and writes one partial of p^T (R v) per
// block (appended to the J.v's partials).
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_sheet_jv(SheetSet S, const uint8_t* __restrict__ mask,
                                                         const T* __restrict__ v, T* __restrict__ y,
                                                         const T* __restrict__ p, const PcgCtx* __restrict__ ctx,
                                                         double* __restrict__ part, int dir_rows) {
  if (ctx && ctx->done) return;
  __shared__ double sred[kVecThreads / 64];
  const long total = S.start[S.n];
  double dot = 0.0;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    int s, a, b;
    sheet_slot(S, t, s, a, b);
    const long n = sheet_node(S.s[s], a, b);
    if ((mask[n] != 0) != (dir_rows != 0) || !sheet_owner(S, s, n)) continue;
    auto val = [=](long j) { return mask[j] ? 0.0 : (double)v[j]; };
    double mv, load, diag;
    sheet_terms_at(S, s, n, 0.0, val, mv, load, diag);
    if (dir_rows) mv = -mv;
    const T yn = (T)((double)y[n] + mv);
    y[n] = yn;
    if (p) dot += (double)p[n] * mv;
  }
  if (part) {
    const double sum = block_sum(dot, sred);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

// Bit 16 of *flags: a sheet's sigma is not finite.
__global__ __launch_bounds__(kVecThreads) void k_validate_sheets(SheetSet S, int* flags) {
  int f = 0;
  for (int s = 0; s < S.n; ++s) {
    const SheetDev& d = S.s[s];
    if (!d.sigma) continue;
    const long nf = (long)(d.a1 - d.a0) * (d.b1 - d.b0);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += (long)gridDim.x * blockDim.x)
      if (!isfinite(d.sigma[i])) f = 16;
  }
  if (f) atomicOr(flags, f);
}

int sheet_blocks(const SheetSet& S) {
  const long b = (S.start[S.n] + kVecThreads - 1) / kVecThreads;
  return (int)std::max(1L, std::min(b, (long)kSheetBlocks));
}

void launch_sheet_residual(hipStream_t s, const SheetSet& S, double kappa, const uint8_t* mask, const double* phi,
                           const double* delta64, const float* delta32, double lam, double* fsheet, double* fdiag) {
  if (delta32)
    hipLaunchKernelGGL(k_sheet_residual<float>, dim3(sheet_blocks(S)), dim3(kVecThreads), 0, s, S, kappa, mask, phi,
                       delta32, lam, fsheet, fdiag);
  else
    hipLaunchKernelGGL(k_sheet_residual<double>, dim3(sheet_blocks(S)), dim3(kVecThreads), 0, s, S, kappa, mask, phi,
                       delta64, lam, fsheet, fdiag);
}

void launch_sheet_jv64(hipStream_t s, const SheetSet& S, const uint8_t* mask, const double* v, double* y,
                       const double* p, const PcgCtx* ctx, double* part) {
  hipLaunchKernelGGL(k_sheet_jv<double>, dim3(sheet_blocks(S)), dim3(kVecThreads), 0, s, S, mask, v, y, p, ctx, part, 0);
}

void launch_sheet_jv32(hipStream_t s, const SheetSet& S, const uint8_t* mask, const float* v, float* y,
                       const float* p, const PcgCtx* ctx, double* part) {
  hipLaunchKernelGGL(k_sheet_jv<float>, dim3(sheet_blocks(S)), dim3(kVecThreads), 0, s, S, mask, v, y, p, ctx, part, 0);
}

void launch_sheet_contact(hipStream_t s, const SheetSet& S, const uint8_t* mask, const double* lam, double* tcon) {
  hipLaunchKernelGGL(k_sheet_jv<double>, dim3(sheet_blocks(S)), dim3(kVecThreads), 0, s, S, mask, lam, tcon, nullptr,
                     nullptr, nullptr, 1);
}

void launch_validate_sheets(hipStream_t s, const SheetSet& S, int* flags) {
  hipLaunchKernelGGL(k_validate_sheets, dim3(64), dim3(kVecThreads), 0, s, S, flags);
}

}  // namespace qe
