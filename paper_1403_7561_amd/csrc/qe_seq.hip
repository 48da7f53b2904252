// Coarse-mesh sequence of the nonlinear solve's initial guess: the coarse
// problem's arrays from the fine one, and the coarse potential interpolated
// back onto the fine nodes (kernels and host launchers).
#include <algorithm>

#include "qe_kernels.h"

namespace qe {

#define QE_LAUNCH(kernel, grid, block, stream, ...) \
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, (hipStream_t)(stream), __VA_ARGS__)

// ---------------------------------------------------------------------------
// Coarse-mesh sequence for the initial guess: the coarse mesh keeps fine
// nodes f(I) = min(2 I, n - 1) along each axis; coarse element (I, J, K)
// takes the materials of fine element (f(I), f(J), f(K)), its first fine
// element; the potential returns by trilinear interpolation in the fine
// coordinates.
__device__ __forceinline__ int seq_fine(int I, int n) { return min(2 * I, n - 1); }

__global__ __launch_bounds__(kVecThreads) void k_seq_coarsen(int nxf, int nyf, int nzf, int nxc, int nyc, int nzc,
                                                              const double* __restrict__ xf, const double* __restrict__ yf,
                                                              const double* __restrict__ zf, const double* __restrict__ epsf,
                                                              const uint8_t* __restrict__ semif,
                                                              const double* __restrict__ netf, const double* __restrict__ donf,
                                                              const double* __restrict__ accf, const int32_t* __restrict__ dirf,
                                                              double* __restrict__ xc, double* __restrict__ yc,
                                                              double* __restrict__ zc, double* __restrict__ epsc,
                                                              uint8_t* __restrict__ semic, double* __restrict__ netc,
                                                              double* __restrict__ donc, double* __restrict__ accc,
                                                              int32_t* __restrict__ dirc) {
  const long Nc = (long)nxc * nyc * nzc, Ec = (long)(nxc - 1) * (nyc - 1) * (nzc - 1);
  const long stride = (long)gridDim.x * blockDim.x;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < Nc; t += stride) {
    const int I = (int)(t % nxc), J = (int)((t / nxc) % nyc), K = (int)(t / ((long)nxc * nyc));
    dirc[t] = dirf[(long)seq_fine(I, nxf) + (long)nxf * ((long)seq_fine(J, nyf) + (long)nyf * seq_fine(K, nzf))];
    if (t < nxc) xc[t] = xf[seq_fine((int)t, nxf)];
    if (t < nyc) yc[t] = yf[seq_fine((int)t, nyf)];
    if (t < nzc) zc[t] = zf[seq_fine((int)t, nzf)];
    if (t < Ec) {
      const int ei = (int)(t % (nxc - 1)), ej = (int)((t / (nxc - 1)) % (nyc - 1)),
                ek = (int)(t / ((long)(nxc - 1) * (nyc - 1)));
      const long ef = (long)(2 * ei) + (long)(nxf - 1) * ((long)(2 * ej) + (long)(nyf - 1) * (2 * ek));
      epsc[t] = epsf[ef];
      semic[t] = semif[ef];
      if (netc) netc[t] = netf[ef];
      if (donc) donc[t] = donf[ef];
      if (accc) accc[t] = accf[ef];
    }
  }
}

// One axis of the interpolation: the coarse interval holding fine node i and
// the weight of its upper end.
__device__ __forceinline__ void seq_weight(int i, int nf, int nc, const double* __restrict__ xf, int& I, double& w) {
  I = min(i >> 1, nc - 2);
  const double a = xf[seq_fine(I, nf)], b = xf[seq_fine(I + 1, nf)];
  w = (xf[i] - a) / (b - a);
}

__global__ __launch_bounds__(kVecThreads) void k_seq_prolong(int nxf, int nyf, int nzf, int nxc, int nyc, int nzc,
                                                              const double* __restrict__ xf, const double* __restrict__ yf,
                                                              const double* __restrict__ zf, const double* __restrict__ phic,
                                                              double* __restrict__ phif) {
  const long Nf = (long)nxf * nyf * nzf;
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < Nf; n += (long)gridDim.x * blockDim.x) {
    const int i = (int)(n % nxf), j = (int)((n / nxf) % nyf), k = (int)(n / ((long)nxf * nyf));
    int I, J, K;
    double wx, wy, wz;
    seq_weight(i, nxf, nxc, xf, I, wx);
    seq_weight(j, nyf, nyc, yf, J, wy);
    seq_weight(k, nzf, nzc, zf, K, wz);
    const long c0 = (long)I + (long)nxc * ((long)J + (long)nyc * K), sy = nxc, sz = (long)nxc * nyc;
    const double v00 = phic[c0] + wx * (phic[c0 + 1] - phic[c0]);
    const double v10 = phic[c0 + sy] + wx * (phic[c0 + sy + 1] - phic[c0 + sy]);
    const double v01 = phic[c0 + sz] + wx * (phic[c0 + sz + 1] - phic[c0 + sz]);
    const double v11 = phic[c0 + sz + sy] + wx * (phic[c0 + sz + sy + 1] - phic[c0 + sz + sy]);
    const double v0 = v00 + wy * (v10 - v00), v1 = v01 + wy * (v11 - v01);
    phif[n] = v0 + wz * (v1 - v0);
  }
}

void launch_seq_coarsen(hipStream_t s, const qe_problem* f, const qe_problem* c) {
  const long Nc = (long)c->nx * c->ny * c->nz;
  const int nb = (int)std::max(1L, std::min((Nc + kVecThreads - 1) / kVecThreads, 4096L));
  QE_LAUNCH(k_seq_coarsen, nb, kVecThreads, s, f->nx, f->ny, f->nz, c->nx, c->ny, c->nz, f->x, f->y, f->z, f->eps_r,
            f->semi, f->net_doping, f->donors, f->acceptors, f->dir_id, const_cast<double*>(c->x),
            const_cast<double*>(c->y), const_cast<double*>(c->z), const_cast<double*>(c->eps_r),
            const_cast<uint8_t*>(c->semi), const_cast<double*>(c->net_doping), const_cast<double*>(c->donors),
            const_cast<double*>(c->acceptors), const_cast<int32_t*>(c->dir_id));
}

void launch_seq_prolong(hipStream_t s, const qe_problem* f, const qe_problem* c, const double* phic, double* phif) {
  const long Nf = (long)f->nx * f->ny * f->nz;
  const int nb = (int)std::max(1L, std::min((Nf + kVecThreads - 1) / kVecThreads, 8192L));
  QE_LAUNCH(k_seq_prolong, nb, kVecThreads, s, f->nx, f->ny, f->nz, c->nx, c->ny, c->nz, f->x, f->y, f->z, phic, phif);
}

}  // namespace qe
