// Interface-charge and Robin face terms (Sec. II.A.4) on mesh-plane sheets.
//
// On a face f (a rectangle of a node plane, sides ha x hb) the weak form
// gains alpha int_f (phi - phi0) w_i - KAPPA sigma_f int_f w_i.  With bilinear
// traces the integrals are exact: int_f w_i = A/4 and int_f w_i w_j = A/36
// times 4 (j = i), 2 (j shares a side with i) or 1 (j is diagonal to i).
// Each distinct node of the sheets is one work item (listed on the host from
// the sheets' index ranges), handled by one thread that sums over every sheet
// containing it and over the (up to four) faces of each around the node, in a
// fixed order: no atomics, and the result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "qe_kernels.h"

namespace qe {

// Node (i, j, k) of position (a, b) in sheet d, and the position of node
// (i, j, k) in sheet t if t contains it.
__device__ __forceinline__ void sheet_ijk(const SheetDev& d, int a, int b, int& i, int& j, int& k) {
  if (d.axis == 2) {
    i = a; j = b; k = d.plane;
  } else if (d.axis == 1) {
    i = a; j = d.plane; k = b;
  } else {
    i = d.plane; j = a; k = b;
  }
}

__device__ __forceinline__ bool sheet_pos(const SheetDev& t, int i, int j, int k, int& a, int& b) {
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

__device__ __forceinline__ long sheet_node(const SheetDev& d, int a, int b) { return d.base + a * d.sa + b * d.sb; }

// The face terms at position (a, b) of sheet d: the Robin mass product
// sum alpha int_f w_n v over its (up to four) faces around the node, the
// constant load sum (alpha phi0 + KAPPA sigma) int_f w_n and the diagonal
// sum alpha int_f w_n^2.  The nine stencil values are loaded first, all
// independent of each other.
template <typename Val>
__device__ __forceinline__ void sheet_terms_one(const SheetDev& d, int a, int b, double kappa, Val val,
                                                double& mv, double& load, double& diag) {
  // indices clamped into the sheet so that every load is valid and none
  // waits behind a branch; values outside the sheet are then zeroed
  double vv[3][3];
#pragma unroll
  for (int db = 0; db < 3; ++db)
#pragma unroll
    for (int da = 0; da < 3; ++da) {
      const int aa = min(max(a + da - 1, d.a0), d.a1), bb = min(max(b + db - 1, d.b0), d.b1);
      vv[db][da] = val(sheet_node(d, aa, bb));
    }
#pragma unroll
  for (int db = 0; db < 3; ++db)
#pragma unroll
    for (int da = 0; da < 3; ++da) {
      const int aa = a + da - 1, bb = b + db - 1;
      if (!(aa >= d.a0 && aa <= d.a1 && bb >= d.b0 && bb <= d.b1)) vv[db][da] = 0.0;
    }
  const int na = d.a1 - d.a0;
#pragma unroll
  for (int fb = 0; fb < 2; ++fb) {
    const int f_b = b - 1 + fb;           // face index along b
    if (f_b < d.b0 || f_b >= d.b1) continue;
    const int ob = fb == 0 ? 0 : 2;       // the stencil row of the face's other nodes
    const double hb = d.cb[f_b + 1] - d.cb[f_b];
#pragma unroll
    for (int fa = 0; fa < 2; ++fa) {
      const int f_a = a - 1 + fa;
      if (f_a < d.a0 || f_a >= d.a1) continue;
      const int oa = fa == 0 ? 0 : 2;
      const double A = (d.ca[f_a + 1] - d.ca[f_a]) * hb;
      const double sg = d.sigma ? d.sigma[(f_a - d.a0) + (long)na * (f_b - d.b0)] : 0.0;
      load += (d.alpha * d.phi0 + kappa * sg) * (0.25 * A);
      const double m = d.alpha * A * (1.0 / 36.0);
      mv += m * (4.0 * vv[1][1] + 2.0 * vv[1][oa] + 2.0 * vv[ob][1] + vv[ob][oa]);
      diag += 4.0 * m;
    }
  }
}

// Sum over every sheet from item.s on that contains the item's node (the
// later ones only when the item is flagged as shared).
template <typename Val>
__device__ __forceinline__ void sheet_terms_at(const SheetSet& S, const int4 it, double kappa, Val val, double& mv,
                                               double& load, double& diag) {
  mv = load = diag = 0.0;
  const int s0 = it.y & 0xff;
  sheet_terms_one(S.s[s0], it.z, it.w, kappa, val, mv, load, diag);
  if (it.y >> 8) {
    int i, j, k;
    sheet_ijk(S.s[s0], it.z, it.w, i, j, k);
    for (int t = s0 + 1; t < S.n; ++t) {
      int a, b;
      if (sheet_pos(S.s[t], i, j, k, a, b)) sheet_terms_one(S.s[t], a, b, kappa, val, mv, load, diag);
    }
  }
}

// Face contributions to F(phi + lam delta) and to the Jacobian diagonal, on
// free sheet nodes (fsheet, fdiag are read by the residual kernel there).
// items: one per distinct sheet node (x: node, y: sheet | shared << 8,
// z, w: position in that sheet).
template <typename TD>
__global__ __launch_bounds__(kVecThreads) void k_sheet_residual(SheetSet S, const int4* __restrict__ items,
                                                               double kappa, const uint8_t* __restrict__ mask,
                                                               const double* __restrict__ phi,
                                                               const TD* __restrict__ delta, double lam,
                                                               double* __restrict__ fsheet,
                                                               double* __restrict__ fdiag) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S.n_items; t += gridDim.x * blockDim.x) {
    const int4 it = items[t];
    const long n = it.x;
    auto val = [=](long j) { return delta ? phi[j] + lam * (double)delta[j] : phi[j]; };
    const bool row_dir = mask[n] != 0;
    double mv, load, diag;
    sheet_terms_at(S, it, kappa, val, mv, load, diag);
    if (row_dir) continue;
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
__global__ __launch_bounds__(kVecThreads) void k_sheet_jv(SheetSet S, const int4* __restrict__ items,
                                                         const uint8_t* __restrict__ mask,
                                                         const T* __restrict__ v, T* __restrict__ y,
                                                         const T* __restrict__ p, const PcgCtx* __restrict__ ctx,
                                                         double* __restrict__ part, int dir_rows) {
  if (ctx && ctx->done) return;
  __shared__ double sred[kVecThreads / 64];
  double dot = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S.n_items; t += gridDim.x * blockDim.x) {
    const int4 it = items[t];
    const long n = it.x;
    // v and the flag loaded side by side (not one after the other)
    auto val = [=](long j) {
      const double vj = (double)v[j];
      return mask[j] ? 0.0 : vj;
    };
    const bool row_dir = mask[n] != 0;
    const double yo = (double)y[n];
    const double pn = p ? (double)p[n] : 0.0;
    double mv, load, diag;
    sheet_terms_at(S, it, 0.0, val, mv, load, diag);
    if (row_dir != (dir_rows != 0)) continue;
    if (dir_rows) mv = -mv;
    y[n] = (T)(yo + mv);
    dot += pn * mv;
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
  const long b = ((long)S.n_items + kVecThreads - 1) / kVecThreads;
  return (int)std::max(1L, std::min(b, (long)kSheetBlocks));
}

void launch_sheet_residual(hipStream_t s, const SheetSet& S, const int4* items, double kappa, const uint8_t* mask, const double* phi,
                           const double* delta64, const float* delta32, double lam, double* fsheet, double* fdiag) {
  if (delta32)
    hipLaunchKernelGGL(k_sheet_residual<float>, dim3(sheet_blocks(S)), dim3(kVecThreads), 0, s, S, items, kappa, mask,
                       phi, delta32, lam, fsheet, fdiag);
  else
    hipLaunchKernelGGL(k_sheet_residual<double>, dim3(sheet_blocks(S)), dim3(kVecThreads), 0, s, S, items, kappa, mask,
                       phi, delta64, lam, fsheet, fdiag);
}

void launch_sheet_jv64(hipStream_t s, const SheetSet& S, const int4* items, const uint8_t* mask, const double* v, double* y,
                       const double* p, const PcgCtx* ctx, double* part) {
  hipLaunchKernelGGL(k_sheet_jv<double>, dim3(sheet_blocks(S)), dim3(kVecThreads), 0, s, S, items, mask, v, y, p, ctx, part, 0);
}

void launch_sheet_jv32(hipStream_t s, const SheetSet& S, const int4* items, const uint8_t* mask, const float* v, float* y,
                       const float* p, const PcgCtx* ctx, double* part) {
  hipLaunchKernelGGL(k_sheet_jv<float>, dim3(sheet_blocks(S)), dim3(kVecThreads), 0, s, S, items, mask, v, y, p, ctx, part, 0);
}

void launch_sheet_contact(hipStream_t s, const SheetSet& S, const int4* items, const uint8_t* mask, const double* lam, double* tcon) {
  hipLaunchKernelGGL(k_sheet_jv<double>, dim3(sheet_blocks(S)), dim3(kVecThreads), 0, s, S, items, mask, lam, tcon,
                     nullptr, nullptr, nullptr, 1);
}

void launch_validate_sheets(hipStream_t s, const SheetSet& S, int* flags) {
  hipLaunchKernelGGL(k_validate_sheets, dim3(64), dim3(kVecThreads), 0, s, S, flags);
}

}  // namespace qe
