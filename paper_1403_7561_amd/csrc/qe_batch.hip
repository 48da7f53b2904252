// Batched solve of many independent devices (a gate-voltage sweep over
// uneven meshes) in one persistent launch.
//
// Every workgroup repeatedly takes the next instance from a device queue
// (instances ordered largest first) and runs that instance's whole solve --
// linear initial guess, Newton with backtracking, Jacobi CG, electron counts --
// on the device.  Its waves share the instance's wave tiles (qe_tiles.h);
// phases are separated by block barriers and every scalar comes from a block
// reduction in a fixed order, so the Newton and CG decisions are uniform over
// the block.  Workgroups never wait for each other: no co-residency is
// assumed and every loop is bounded by an iteration limit.
//
// The host validates the instances, lays out the workspace, picks the block
// size and chunk height (autotuned, cached in a file), and captures the queue
// reset and the persistent kernel in a hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "qe_runtime.h"
#include "qe_tiles.h"

namespace qe {

// One instance as the device sees it.
struct BatchInst {
  Geom g;
  const double* eps;
  const uint8_t* semi;
  Doping dop;
  const int32_t* dir_id;
  const double* dir_val;
  double* phi;
  double *F, *x, *r, *p, *y, *invdiag, *c, *eps_t;   // c, eps_t, cflag tile-major (tile_slot)
  uint8_t *mask, *cflag;
  unsigned int* cbits;   // [ntiles][64] per-lane coefficient flags over the chunk
  double* rdz;   // [nz-1] inverse z spacings (g.rdz points here)
  long N, nslots;
  int gx, gy, gz, kz, ntiles;
};

struct BatchOut {
  int status, newton_iters, krylov_iters, ls_halvings, init_krylov_iters, n_residual_evals;
  double res0, res_final;
  double counts[kMaxBoxes];
};

struct BatchParams {
  int n_inst;
  const BatchInst* inst;
  const int* order;
  BatchOut* out;
  int* queue;
  Charge ch;
  double atol, rtol_max;
  int newton_maxit, ls_max, krylov_maxit;
  BoxSet boxes;
};

// ------------------------------------------------------------ block helpers
template <int NT>
__device__ __forceinline__ double bsum(double v, double* sred) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) r += sred[w];
  return r;
}

template <int NT>
__device__ __forceinline__ void bsum2(double& a, double& b, double* sred) {
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sred[threadIdx.x >> 6] = a;
    sred[NT / 64 + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  double ra = 0.0, rb = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    ra += sred[w];
    rb += sred[NT / 64 + w];
  }
  a = ra;
  b = rb;
}

__device__ __forceinline__ WaveTile tile_at(const BatchInst& I, int t) {
  t = __builtin_amdgcn_readfirstlane(t);   // wave-uniform: scalar layer loop
  const int wx = t % I.gx, wy = (t / I.gx) % I.gy, wz = t / (I.gx * I.gy);
  return WaveTile(I.g, wx, wy, wz, I.kz, threadIdx.x & 63, true);
}

// ||F(phi + lam delta)||^2 with F, invdiag and c written for that point.
template <int NT>
__device__ double b_residual(const BatchInst& I, const Charge& ch, const double* delta, double lam, double* sred) {
  double acc = 0.0;
  for (int t = threadIdx.x >> 6; t < I.ntiles; t += NT / 64) {
    const WaveTile w = tile_at(I, t);
    residual_tile<double>(I.g, w, ch, I.eps, I.semi, I.dop, I.mask, I.phi, delta, lam, nullptr, nullptr, I.F, I.invdiag, nullptr,
                          I.c, nullptr, I.cflag, I.cbits + 64L * t + (threadIdx.x & 63), nullptr, acc);
  }
  return bsum<NT>(acc, sred);
}

// Jacobi CG on J x = sign b over the free nodes; returns the iteration count,
// *st = PCG_CONVERGED / PCG_MAXIT / PCG_BREAKDOWN / PCG_NONFINITE.
template <int NT>
__device__ int b_pcg(const BatchInst& I, const double* b, double sign, double rtol, int maxit, int* st,
                     double* sred) {
  double rz = 0.0, rr = 0.0;
  for (long n = threadIdx.x; n < I.N; n += NT) {
    const double ri = I.mask[n] ? 0.0 : sign * b[n];
    const double zi = I.invdiag[n] * ri;
    I.x[n] = 0.0;
    I.r[n] = ri;
    I.p[n] = zi;
    rz += ri * zi;
    rr += ri * ri;
  }
  bsum2<NT>(rz, rr, sred);
  if (!isfinite(rz) || !isfinite(rr)) {
    *st = PCG_NONFINITE;
    return 0;
  }
  if (rz == 0.0) {
    *st = PCG_CONVERGED;
    return 0;
  }
  const double tol2 = rtol * rtol * rz;
  for (int it = 0; it < maxit; ++it) {
    double dot = 0.0;
    for (int t = threadIdx.x >> 6; t < I.ntiles; t += NT / 64) {
      const WaveTile w = tile_at(I, t);
      jv_tile<double, JV_DOT>(I.g, w, I.eps_t, I.cbits[64L * t + (threadIdx.x & 63)], I.c, nullptr, I.p, I.y, 1,
                              dot);
    }
    const double pAp = bsum<NT>(dot, sred);
    if (!(pAp > 0.0) || !isfinite(pAp)) {
      *st = PCG_BREAKDOWN;
      return it;
    }
    const double alpha = rz / pAp;
    double rzn = 0.0, rrn = 0.0;
    for (long n = threadIdx.x; n < I.N; n += NT) {
      I.x[n] += alpha * I.p[n];
      const double ri = I.r[n] - alpha * I.y[n];
      I.r[n] = ri;
      const double zi = I.invdiag[n] * ri;
      rzn += ri * zi;
      rrn += ri * ri;
    }
    bsum2<NT>(rzn, rrn, sred);
    if (!isfinite(rzn) || !isfinite(rrn)) {
      *st = PCG_NONFINITE;
      return it + 1;
    }
    if (rzn <= tol2) {
      *st = PCG_CONVERGED;
      return it + 1;
    }
    const double beta = rzn / rz;
    rz = rzn;
    for (long n = threadIdx.x; n < I.N; n += NT) I.p[n] = I.invdiag[n] * I.r[n] + beta * I.p[n];
    __syncthreads();
  }
  *st = PCG_MAXIT;
  return maxit;
}

template <int NT>
__device__ void b_axpy_phi(const BatchInst& I, double lam) {
  for (long n = threadIdx.x; n < I.N; n += NT) I.phi[n] += lam * I.x[n];
  __syncthreads();
}

template <int NT>
__device__ void b_solve(const BatchParams& bp, const BatchInst& I, BatchOut& o, double* sred) {
  // stage: Dirichlet mask, Dirichlet values, zeros elsewhere; tile-major eps;
  // inverse z spacings
  for (int k = threadIdx.x; k < I.g.nz - 1; k += NT) I.rdz[k] = 1.0 / (I.g.z[k + 1] - I.g.z[k]);
  for (long n = threadIdx.x; n < I.N; n += NT) {
    const int d = I.dir_id[n];
    I.mask[n] = d >= 0 ? 1 : 0;
    I.phi[n] = d >= 0 ? I.dir_val[d] : 0.0;
  }
  {
    const int gx = (I.g.nx + 6) / 7, gy = (I.g.ny + 6) / 7;
    for (long sl = threadIdx.x; sl < I.nslots; sl += NT) {
      const int j = (int)(sl % 49);
      const long blk = sl / 49;
      const int tx = (int)(blk % gx), ty = (int)((blk / gx) % gy), L = (int)(blk / ((long)gx * gy));
      const int ex = 7 * tx + j % 7, ey = 7 * ty + j / 7;
      double e = 0.0;
      if (ex < I.g.nx - 1 && ey < I.g.ny - 1)
        e = I.eps[(long)ex + (long)(I.g.nx - 1) * ((long)ey + (long)(I.g.ny - 1) * L)];
      I.eps_t[sl] = e;
    }
  }
  __syncthreads();
  int status = QE_OK, newton = 0, kry = 0, halv = 0, nres = 0, pst = 0;
  // charge-free linear initial guess
  const Charge lin = linear_charge(bp.ch);
  double n2 = b_residual<NT>(I, lin, nullptr, 0.0, sred);
  if (n2 > 0.0 && isfinite(n2)) {
    const int its = b_pcg<NT>(I, I.F, -1.0, QE_INIT_RTOL, bp.krylov_maxit, &pst, sred);
    o.init_krylov_iters = its;
    kry += its;
    if (pst == PCG_CONVERGED || pst == PCG_MAXIT) b_axpy_phi<NT>(I, 1.0);
  }
  n2 = b_residual<NT>(I, bp.ch, nullptr, 0.0, sred);
  ++nres;
  double nrm = sqrt(n2), prev = -1.0;
  o.res0 = nrm;
  if (!isfinite(nrm)) status = QE_ERR_NONFINITE;
  if (status == QE_OK) {
    status = QE_ERR_NOT_CONVERGED;
    for (int it = 0; it <= bp.newton_maxit; ++it) {
      if (nrm <= bp.atol) {
        status = QE_OK;
        break;
      }
      if (it == bp.newton_maxit) break;
      double eta = prev < 0.0 ? bp.rtol_max : fmin(bp.rtol_max, QE_EW_GAMMA * (nrm / prev) * (nrm / prev));
      eta = fmax(eta, 0.5 * bp.atol / nrm);
      eta = fmin(eta, bp.rtol_max);
      eta = fmax(eta, 1e-13);
      kry += b_pcg<NT>(I, I.F, -1.0, eta, bp.krylov_maxit, &pst, sred);
      if (pst == PCG_BREAKDOWN || pst == PCG_NONFINITE) {
        status = pst == PCG_BREAKDOWN ? QE_ERR_KRYLOV_BREAKDOWN : QE_ERR_NONFINITE;
        break;
      }
      double lam = 1.0, nt = 0.0;
      bool ok = false;
      for (int hv = 0; hv <= bp.ls_max; ++hv) {
        nt = sqrt(b_residual<NT>(I, bp.ch, I.x, lam, sred));
        ++nres;
        if (isfinite(nt) && nt <= (1.0 - 1e-4 * lam) * nrm) {
          ok = true;
          break;
        }
        lam *= 0.5;
        ++halv;
      }
      if (!ok) {
        status = QE_ERR_LINESEARCH;
        break;
      }
      b_axpy_phi<NT>(I, lam);
      prev = nrm;
      nrm = nt;
      newton = it + 1;
    }
  }
  // electron counts in the boxes (owned elements only)
  for (int r = 0; r < bp.boxes.n; ++r) {
    double acc = 0.0;
    const long ex = I.g.nx - 1, ey = I.g.ny - 1, E = ex * ey * (I.g.nz - 1);
    const Box bx = bp.boxes.b[r];
    for (long el = threadIdx.x; el < E; el += NT) {
      if (!I.semi[el]) continue;
      const int i = (int)(el % ex), j = (int)((el / ex) % ey), k = (int)(el / (ex * ey));
      const double xc = 0.5 * (I.g.x[i] + I.g.x[i + 1]), yc = 0.5 * (I.g.y[j] + I.g.y[j + 1]),
                   zc = 0.5 * (I.g.z[k] + I.g.z[k + 1]);
      if (!bx.contains(xc, yc, zc)) continue;
      const long n0 = (long)i + (long)I.g.nx * ((long)j + (long)I.g.ny * k);
      const long sy = I.g.nx, sz = (long)I.g.nx * I.g.ny;
      double ve[8] = {I.phi[n0], I.phi[n0 + 1], I.phi[n0 + sy], I.phi[n0 + sy + 1],
                      I.phi[n0 + sz], I.phi[n0 + sz + 1], I.phi[n0 + sz + sy], I.phi[n0 + sz + sy + 1]};
      gauss_interp(ve);
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) s += electron_density_only(bp.ch, ve[q]);
      acc += s * (I.g.x[i + 1] - I.g.x[i]) * (I.g.y[j + 1] - I.g.y[j]) * (I.g.z[k + 1] - I.g.z[k]) * 0.125;
    }
    const double tot = bsum<NT>(acc, sred);
    if (threadIdx.x == 0) o.counts[r] = tot;
  }
  if (threadIdx.x == 0) {
    o.status = status;
    o.newton_iters = newton;
    o.krylov_iters = kry;
    o.ls_halvings = halv;
    o.n_residual_evals = nres;
    o.res_final = nrm;
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_batch_solve(BatchParams bp) {
  __shared__ double sred[2 * NT / 64];
  __shared__ int s_next;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(bp.queue, 1);
    __syncthreads();
    const int k = s_next;
    __syncthreads();
    if (k >= bp.n_inst) break;
    const int id = bp.order[k];
    BatchOut o;
    o.init_krylov_iters = 0;
    b_solve<NT>(bp, bp.inst[id], o, sred);
    if (threadIdx.x == 0) bp.out[id] = o;
    __syncthreads();
  }
}

__global__ void k_reset_queue(int* q) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0;
}

// ------------------------------------------------------------ host side
struct BatchConfig {
  int threads = 512;  // 256, 512 or 1024
  int kz = 8;
};

static size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

static const int kTuneKz[3] = {4, 8, 16};   // chunk heights the tuner tries
static const int kMinKz = 4;

static size_t inst_bytes(const qe_problem& p) {
  const long N = (long)p.nx * p.ny * p.nz;
  const long S = tile_slots(p.nx, p.ny, p.nz);
  // per-lane coefficient words for the shortest chunk height the tuner uses
  const long tiles = (long)((p.nx + 6) / 7) * ((p.ny + 6) / 7) * ((p.nz + kMinKz - 1) / kMinKz);
  return 6 * al256(N * 8) + al256(S * 64) + al256(S * 8) + al256(S) + al256(N) + al256((p.nz - 1) * 8) +
         al256(tiles * 64 * 4);
}

static size_t batch_bytes(int n, const qe_problem* probs) {
  size_t t = al256(sizeof(BatchInst) * n) + al256(sizeof(BatchOut) * n) + al256(sizeof(int) * n) + 256;
  for (int i = 0; i < n; ++i) t += inst_bytes(probs[i]);
  return t;
}

static qe_status launch_batch(const BatchParams& bp, const BatchConfig& cfg, int grid, hipStream_t s,
                              bool use_graph) {
  auto enqueue = [&](hipStream_t st) {
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, st, bp.queue);
    switch (cfg.threads) {
      case 256:
        hipLaunchKernelGGL(k_batch_solve<256>, dim3(grid), dim3(256), 0, st, bp);
        break;
      case 1024:
        hipLaunchKernelGGL(k_batch_solve<1024>, dim3(grid), dim3(1024), 0, st, bp);
        break;
      default:
        hipLaunchKernelGGL(k_batch_solve<512>, dim3(grid), dim3(512), 0, st, bp);
        break;
    }
  };
  if (!use_graph) {
    enqueue(s);
    if (hipGetLastError() != hipSuccess) return fail(QE_ERR_HIP, "batch launch failed");
    return QE_OK;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(QE_ERR_HIP, "hipStreamBeginCapture failed");
  enqueue(s);
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (e != hipSuccess) return fail(QE_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e == hipSuccess) e = hipGraphLaunch(exec, s);
  // the executable graph is released only after the launch has finished
  const hipError_t es = hipStreamSynchronize(s);
  if (e == hipSuccess) e = es;
  if (exec) (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(QE_ERR_HIP, "graph launch failed: %s", hipGetErrorString(e));
  return QE_OK;
}

static int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
  return cus;
}

static std::string tune_key(int n, const std::vector<long>& sizes) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  const long tot = std::accumulate(sizes.begin(), sizes.end(), 0L);
  const long mx = sizes.empty() ? 0 : *std::max_element(sizes.begin(), sizes.end());
  // bucket the workload: instance count and mean / max size to ~powers of two
  auto b2 = [](long v) {
    int k = 0;
    while ((1L << k) < v) ++k;
    return k;
  };
  std::ostringstream os;
  os << arch << ";cu=" << device_cus() << ";n=" << b2(n) << ";mean=" << b2(n ? tot / n : 0) << ";max=" << b2(mx);
  std::string k = os.str();
  for (auto& ch : k)
    if (ch == ' ' || ch == '\n') ch = '_';
  return k;
}

static bool read_cache(const char* path, const std::string& key, BatchConfig& cfg) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string k;
    int t, kz;
    if (is >> k >> t >> kz && k == key && (t == 256 || t == 512 || t == 1024) &&
        (kz == kTuneKz[0] || kz == kTuneKz[1] || kz == kTuneKz[2])) {
      cfg.threads = t;
      cfg.kz = kz;
      return true;
    }
  }
  return false;
}

static void write_cache(const char* path, const std::string& key, const BatchConfig& cfg) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << cfg.threads << " " << cfg.kz << "\n";
}

}  // namespace qe

using namespace qe;

extern "C" {

size_t qe_batch_workspace_bytes(int32_t n_inst, const qe_problem* probs, const qe_options* o) {
  (void)o;
  if (n_inst < 1 || !probs) return 0;
  for (int i = 0; i < n_inst; ++i)
    if (check_problem(&probs[i]) != QE_OK) return 0;
  return batch_bytes(n_inst, probs);
}

qe_status qe_solve_batch(int32_t n_inst, const qe_problem* probs, const qe_physics* ph, const qe_options* o,
                         double* const* phi, int32_t n_boxes, const double* boxes, double* counts,
                         const char* tune_cache, void* ws_, size_t ws_bytes, void* stream, qe_report* reps) {
  clear_error();
  if (n_inst < 1 || !probs || !phi) return fail(QE_ERR_INVALID_ARG, "need n_inst >= 1, probs and phi");
  qe_status st;
  if ((st = check_options(o)) != QE_OK) return st;
  if (o->precision != QE_PREC_FP64) return fail(QE_ERR_INVALID_ARG, "the batched solve runs in FP64");
  // every instance starts from the linear guess (a coarse-mesh sequence is
  // for meshes far larger than the sweep's)
  if (o->init_guess == 1) return fail(QE_ERR_INVALID_ARG, "the batched solve starts from the linear guess");
  Charge ch;
  if ((st = make_charge(ph, ch)) != QE_OK) return st;
  if (n_boxes < 0 || n_boxes > kMaxBoxes) return fail(QE_ERR_INVALID_ARG, "n_boxes must be in [0, %d]", kMaxBoxes);
  if (n_boxes > 0 && (!boxes || !counts)) return fail(QE_ERR_INVALID_ARG, "boxes/counts is NULL");
  BoxSet bs;
  bs.n = n_boxes;
  for (int r = 0; r < n_boxes; ++r) {
    const double* b = boxes + 6 * r;
    for (int k = 0; k < 6; ++k)
      if (std::isnan(b[k])) return fail(QE_ERR_INVALID_ARG, "box %d has NaN", r);
    bs.b[r] = Box{b[0], b[1], b[2], b[3], b[4], b[5]};
  }
  for (int i = 0; i < n_inst; ++i) {
    if ((st = check_problem(&probs[i])) != QE_OK) return fail(st, "instance %d: %s", i, qe_last_error());
    if (!phi[i]) return fail(QE_ERR_INVALID_ARG, "phi[%d] is NULL", i);
    if (probs[i].quantum)
      return fail(QE_ERR_INVALID_ARG, "instance %d: predictor-corrector states are not supported by the batch", i);
    if (probs[i].n_sheets > 0)
      return fail(QE_ERR_INVALID_ARG, "instance %d: interface / Robin sheets are not supported by the batch", i);
    if (ch.incomplete && !probs[i].donors)
      return fail(QE_ERR_INVALID_ARG, "instance %d: incomplete ionization needs donors and acceptors", i);
  }
  const size_t need = batch_bytes(n_inst, probs);
  if (!ws_) return fail(QE_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws_) & 255) return fail(QE_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < need) return fail(QE_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  // per-instance host-side and device-side validation (coordinates, values)
  {
    std::vector<double> c;
    for (int i = 0; i < n_inst; ++i) {
      const qe_problem& p = probs[i];
      const double* arrs[3] = {p.x, p.y, p.z};
      const int lens[3] = {p.nx, p.ny, p.nz};
      for (int a = 0; a < 3; ++a) {
        c.resize(lens[a]);
        if (hipMemcpyAsync(c.data(), arrs[a], lens[a] * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return fail(QE_ERR_HIP, "instance %d: coordinate copy failed", i);
        for (int k = 1; k < lens[a]; ++k)
          if (!(c[k] > c[k - 1]) || !std::isfinite(c[k]))
            return fail(QE_ERR_INVALID_ARG, "instance %d: coordinates %c not strictly increasing", i, "xyz"[a]);
      }
    }
  }
  char* ws = reinterpret_cast<char*>(ws_);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o2 = off;
    off = al256(off + bytes);
    return ws + o2;
  };
  BatchInst* d_inst = reinterpret_cast<BatchInst*>(take(sizeof(BatchInst) * n_inst));
  BatchOut* d_out = reinterpret_cast<BatchOut*>(take(sizeof(BatchOut) * n_inst));
  int* d_order = reinterpret_cast<int*>(take(sizeof(int) * n_inst));
  int* d_queue = reinterpret_cast<int*>(take(256));
  std::vector<long> sizes(n_inst);
  for (int i = 0; i < n_inst; ++i) sizes[i] = (long)probs[i].nx * probs[i].ny * probs[i].nz;
  BatchConfig cfg;
  const std::string key = tune_key(n_inst, sizes);
  const bool cached = read_cache(tune_cache, key, cfg);
  std::vector<BatchInst> hinst(n_inst);
  auto build = [&](const BatchConfig& cf) {
    size_t o2 = off;
    for (int i = 0; i < n_inst; ++i) {
      const qe_problem& p = probs[i];
      BatchInst& I = hinst[i];
      const long N = (long)p.nx * p.ny * p.nz, S = tile_slots(p.nx, p.ny, p.nz);
      I.g = Geom{p.nx, p.ny, p.nz, p.x, p.y, p.z, nullptr, nullptr};
      I.eps = p.eps_r;
      I.semi = p.semi;
      I.dop = Doping{p.net_doping, p.donors, p.acceptors};
      I.dir_id = p.dir_id;
      I.dir_val = p.dir_val;
      I.phi = phi[i];
      I.N = N;
      auto tk = [&](size_t bytes) {
        char* q = ws + o2;
        o2 = al256(o2 + bytes);
        return q;
      };
      I.F = reinterpret_cast<double*>(tk(N * 8));
      I.x = reinterpret_cast<double*>(tk(N * 8));
      I.r = reinterpret_cast<double*>(tk(N * 8));
      I.p = reinterpret_cast<double*>(tk(N * 8));
      I.y = reinterpret_cast<double*>(tk(N * 8));
      I.invdiag = reinterpret_cast<double*>(tk(N * 8));
      I.c = reinterpret_cast<double*>(tk(S * 64));
      I.eps_t = reinterpret_cast<double*>(tk(S * 8));
      I.cflag = reinterpret_cast<uint8_t*>(tk(S));
      I.rdz = reinterpret_cast<double*>(tk((p.nz - 1) * 8));
      I.cbits = reinterpret_cast<unsigned int*>(
          tk((size_t)((p.nx + 6) / 7) * ((p.ny + 6) / 7) * ((p.nz + kMinKz - 1) / kMinKz) * 64 * 4));
      I.g.rdz = I.rdz;
      I.nslots = S;
      I.mask = reinterpret_cast<uint8_t*>(tk(N));
      I.kz = cf.kz;
      I.gx = (p.nx + 6) / 7;
      I.gy = (p.ny + 6) / 7;
      I.gz = (p.nz + cf.kz - 1) / cf.kz;
      I.ntiles = I.gx * I.gy * I.gz;
    }
  };
  // device-side value checks (eps, doping, dir_id) for every instance
  {
    int* dflags = d_queue + 1;
    if (hipMemsetAsync(dflags, 0, sizeof(int), s) != hipSuccess) return fail(QE_ERR_HIP, "memset failed");
    for (int i = 0; i < n_inst; ++i) {
      const qe_problem& p = probs[i];
      const long N = (long)p.nx * p.ny * p.nz, E = (long)(p.nx - 1) * (p.ny - 1) * (p.nz - 1);
      launch_validate(s, vec_blocks(N), N, E, p.n_dir, p.eps_r, Doping{p.net_doping, p.donors, p.acceptors},
                      p.dir_id, nullptr, dflags);
    }
    int f = 0;
    if (hipMemcpyAsync(&f, dflags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(QE_ERR_HIP, "validation failed to run");
    if (f & 1) return fail(QE_ERR_INVALID_ARG, "eps_r must be finite and > 0");
    if (f & 2) return fail(QE_ERR_NONFINITE, "net_doping not finite or donors / acceptors not finite and >= 0");
    if (f & 4) return fail(QE_ERR_INVALID_ARG, "dir_id outside [-1, n_dir)");
  }
  // largest instances first
  std::vector<int> order(n_inst);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sizes[a] > sizes[b]; });
  if (hipMemcpy(d_order, order.data(), sizeof(int) * n_inst, hipMemcpyHostToDevice) != hipSuccess)
    return fail(QE_ERR_HIP, "order upload failed");
  BatchParams bp;
  bp.n_inst = n_inst;
  bp.inst = d_inst;
  bp.order = d_order;
  bp.out = d_out;
  bp.queue = d_queue;
  bp.ch = ch;
  bp.atol = o->newton_atol;
  bp.rtol_max = o->krylov_rtol_max;
  bp.newton_maxit = o->newton_maxit;
  bp.ls_max = o->ls_max_halvings;
  bp.krylov_maxit = o->krylov_maxit;
  bp.boxes = bs;
  const int cus = device_cus();
  // a private stream for the capture when the caller passed the null stream
  hipStream_t cs = s;
  bool own = false;
  if (!cs) {
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(QE_ERR_HIP, "stream create failed");
    own = true;
  }
  auto run = [&](const BatchConfig& cf, int n_run, bool graph) -> qe_status {
    build(cf);
    if (hipMemcpy(d_inst, hinst.data(), sizeof(BatchInst) * n_inst, hipMemcpyHostToDevice) != hipSuccess)
      return fail(QE_ERR_HIP, "descriptor upload failed");
    BatchParams b2 = bp;
    b2.n_inst = n_run;
    const int grid = std::max(1, std::min(n_run, cus));
    qe_status r = launch_batch(b2, cf, grid, cs, graph);
    if (r != QE_OK) return r;
    if (hipStreamSynchronize(cs) != hipSuccess) return fail(QE_ERR_HIP, "batch kernel failed");
    return QE_OK;
  };
  qe_status result = QE_OK;
  if (!cached) {
    // autotune on the largest instances (the ones that bound the sweep)
    const int n_try = std::min(n_inst, std::max(1, cus / 8));
    const int cand_t[3] = {256, 512, 1024};
    const int* cand_kz = kTuneKz;
    double best = 1e300;
    BatchConfig bestc = cfg;
    for (int ti = 0; ti < 3 && result == QE_OK; ++ti)
      for (int ki = 0; ki < 3 && result == QE_OK; ++ki) {
        BatchConfig cf;
        cf.threads = cand_t[ti];
        cf.kz = cand_kz[ki];
        auto t0 = std::chrono::steady_clock::now();
        result = run(cf, n_try, false);
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (result == QE_OK && dt < best) {
          best = dt;
          bestc = cf;
        }
      }
    cfg = bestc;
    if (result == QE_OK) write_cache(tune_cache, key, cfg);
  }
  if (result == QE_OK) result = run(cfg, n_inst, true);
  if (own) (void)hipStreamDestroy(cs);
  if (result != QE_OK) return result;
  std::vector<BatchOut> hout(n_inst);
  if (hipMemcpy(hout.data(), d_out, sizeof(BatchOut) * n_inst, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(QE_ERR_HIP, "result read-back failed");
  qe_status worst = QE_OK;
  for (int i = 0; i < n_inst; ++i) {
    if (reps) {
      qe_report& r = reps[i];
      std::memset(&r, 0, sizeof(r));
      r.status = hout[i].status;
      r.newton_iters = hout[i].newton_iters;
      r.krylov_iters = hout[i].krylov_iters;
      r.ls_halvings = hout[i].ls_halvings;
      r.init_krylov_iters = hout[i].init_krylov_iters;
      r.n_residual_evals = hout[i].n_residual_evals;
      r.res0 = hout[i].res0;
      r.res_final = hout[i].res_final;
    }
    for (int b = 0; b < n_boxes; ++b) counts[(long)i * n_boxes + b] = hout[i].counts[b];
    if (hout[i].status != QE_OK && worst == QE_OK) worst = (qe_status)hout[i].status;
  }
  if (worst != QE_OK) return fail(worst, "at least one instance did not converge (see the reports)");
  return QE_OK;
}

}  // extern "C"
