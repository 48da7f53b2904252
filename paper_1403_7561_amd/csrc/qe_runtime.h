// Host-side context shared by the entry points of the nonlinear-Poisson library.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/qe.h"
#include "qe_kernels.h"

// Relative CG tolerance of the charge-free initial guess: the first Newton
// step corrects its error, so it is solved only roughly.  And the factor of
// the Eisenstat-Walker forcing term eta_k = gamma (|F_k| / |F_k-1|)^2
// (their second choice, with gamma = 0.9, alpha = 2), capped by
// qe_options.krylov_rtol_max.
#ifndef QE_INIT_RTOL
#define QE_INIT_RTOL 1e-2
#endif
#ifndef QE_EW_GAMMA
#define QE_EW_GAMMA 0.9
#endif

// Returns the status of `expr` from the enclosing function unless it is QE_OK.
#define QE_TRY(expr)              \
  do {                            \
    qe_status s_ = (expr);        \
    if (s_ != QE_OK) return s_;   \
  } while (0)

namespace qe {

struct HostMirror;
qe_status fail(qe_status st, const char* fmt, ...);
void clear_error();
qe_status make_charge(const qe_physics* ph, Charge& ch);
qe_status check_problem(const qe_problem* p);
qe_status check_options(const qe_options* o);
int vec_blocks(long N);
int cg_blocks(long N);
TileMap make_tilemap(int nx, int ny, int nz, int kz);

// Byte offsets of the workspace carve-out.
struct Layout {
  size_t F, x, r, p, y, z, invdiag, gvec, c, cflag, rdz, cbits, mask, fsheet, fdiag, sheet_items;
  size_t x32, r32, p32, y32, z32, invdiag32, c32, eps32, eps_t;
  size_t partial, partial2, ctx, scal, counters, flags, sbox;
  long n_partial;
  size_t total;
};
Layout make_layout(long N, long E, long nslots, long nz_elems, long nwaves, int nblocks_tile, int vblocks,
                   int n_dir, long sheet_slots, long nwaves_q);
long sheet_slots(const qe_problem* p);
qe_status make_quantum(const qe_problem* p, const Charge& ch, Quantum& Q);
SheetSet make_sheets(const qe_problem* p, std::vector<int4>& items);

// The multigrid preconditioner as the CG loop sees it: the levels (0 = the
// Context's own mesh) and the coarsest level's smoothing steps.
struct MgRun {
  const MgGrid* lv;
  int nlev;
  int sweeps;
  bool add_top;   // additive finest level (no smoothing products there)
};

// One call's view of a problem, its workspace and its stream.
struct Context {
  qe_problem prob;
  Geom g;
  TileMap tm;
  WaveMap wm;
  WaveMap wmq;   // the residual with eigenstates (wm without them)
  SheetSet sheets{};
  Quantum quantum{};
  static constexpr int kEventRing = 8;
  hipEvent_t events[kEventRing] = {};   // CG progress markers, created on first use
  ~Context() {
    for (hipEvent_t e : events)
      if (e) (void)hipEventDestroy(e);
  }
  long N = 0, E = 0, nslots = 0;
  int vblocks = 0;
  Layout lay;
  char* ws = nullptr;
  hipStream_t s = nullptr;

  double* f64(size_t off) const { return reinterpret_cast<double*>(ws + off); }
  float* f32(size_t off) const { return reinterpret_cast<float*>(ws + off); }
  uint8_t* u8(size_t off) const { return reinterpret_cast<uint8_t*>(ws + off); }
  unsigned int* u32(size_t off) const { return reinterpret_cast<unsigned int*>(ws + off); }
  const int4* sheet_items() const { return reinterpret_cast<const int4*>(ws + lay.sheet_items); }

  bool no_alloc = false;                // host read-backs in static storage, no events
  HostMirror* hm = nullptr;
  // wave_kz > 0: the J.v / residual wave tiles' chunk height (else the
  // library's choice for the mesh)
  qe_status init(const qe_problem* p, const Charge& ch, void* ws, size_t ws_bytes, void* stream, int kz = 0,
                 bool no_alloc = false, int wave_kz = 0);
  Doping doping() const;
  // Device-side checks of the problem's arrays (coordinates, Dirichlet ids
  // and values, eps_r, doping, sheets, states) and of phi: one round trip.
  qe_status validate(const double* phi);
  qe_status stage(double* phi, int apply, int zero_free);
  qe_status residual(const Charge& ch, const double* phi, const double* d64, const float* d32, double lam, bool mixed,
                     double* diag_out, double* norm2_host);
  // mg: the multigrid preconditioner, or nullptr for Jacobi
  qe_status pcg(bool mixed, const double* b, double sign, double rtol, int maxit, int check_every, int* pcg_status,
                int* iters, const MgRun* mg = nullptr);
  qe_status pcg_polled(bool mixed, const double* b, double sign, double rtol, int maxit, int* pcg_status,
                       int* iters);
};

}  // namespace qe
