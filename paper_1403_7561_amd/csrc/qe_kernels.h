// Kernel-side types and host launchers of the Q1 nonlinear-Poisson path.
#pragma once

#include "../../include/qe.h"
#include "qe_device.h"

namespace qe {

constexpr int kMaxBoxes = 16;

// Closed axis-aligned box (nm); an element belongs to it when its centroid does.
struct Box {
  double x0, x1, y0, y1, z0, z1;
  __host__ __device__ bool contains(double x, double y, double z) const {
    return x >= x0 && x <= x1 && y >= y0 && y <= y1 && z >= z0 && z <= z1;
  }
};

struct BoxSet {
  int n;
  Box b[kMaxBoxes];
};

enum PcgStatus : int { PCG_RUNNING = 0, PCG_CONVERGED = 1, PCG_BREAKDOWN = 2, PCG_MAXIT = 3, PCG_NONFINITE = 4 };

// The stop of a CG solve, posted by the kernel that takes it into
// host-coherent memory so the host learns it without copies, as one word:
// ((iterations + 1) << 4) | (status << 1) | 1.
struct CgProgress {
  int word;
};

// Conjugate-gradient scalars, kept on the device between kernels.
struct PcgCtx {
  double rzs[2], pAp, alpha, beta, tol2;
  int iters, maxit, done, status;
};

void launch_adj_rhs(hipStream_t s, const Geom& g, const TileMap& tm, const Charge& ch, const Box& box,
                    const uint8_t* semi, const double* phi, double* gvec, double* partial, unsigned int* counter,
                    double* Q);
void launch_adj_grad(hipStream_t s, const Geom& g, const TileMap& tm, const double* eps, const uint8_t* cflag,
                     const double* cq, const uint8_t* mask, const double* lam, const double* phi,
                     const double* gvec, double* dQdeps, double* tcon);
void launch_contact_sum(hipStream_t s, int nblocks, long N, int n_dir, const int32_t* dir_id, const double* tcon,
                        double* partial, unsigned int* counter, double* out);
// Electrons per box / at the nodes: from the statistics, or from the
// predictor-corrector states when qm.n > 0.
void launch_count(hipStream_t s, int nblocks, const Geom& g, const Charge& ch, const BoxSet& boxes,
                  const uint8_t* semi, const double* phi, double* partial, unsigned int* counter, double* out,
                  const Quantum& qm);
void launch_density(hipStream_t s, int nblocks, const Geom& g, const Charge& ch, const uint8_t* semi,
                    const double* phi, double* nout, const Quantum& qm);
// Quantum.sbox: per state, the node-index box of its nonzero |psi|^2 (box: [n][6]).
void launch_state_boxes(hipStream_t s, int nblocks, const Geom& g, const Quantum& qm, int* box);
// Bits 32 (|psi|^2 not finite or negative) and 64 (phi^(k) not finite) of *flags.
void launch_validate_quantum(hipStream_t s, int nblocks, const Quantum& qm, int* flags);
void launch_validate(hipStream_t s, int nblocks, long N, long E, int n_dir, const double* eps, const Doping& dop,
                     const int32_t* dir_id, const double* phi, int* flags);
// Coordinates finite and strictly increasing, Dirichlet values finite
// (flag bits 128 / 256 / 512 for x / y / z, 1024 for the values).
void launch_validate_mesh(hipStream_t s, int nx, int ny, int nz, const double* x, const double* y, const double* z,
                          int n_dir, const double* dir_val, int* flags);
void launch_stage(hipStream_t s, int nblocks, long N, const int32_t* dir_id, const double* dir_val, uint8_t* mask,
                  double* phi, int apply, int zero_free);
// Inverse z spacings, then the spacings, into g.rdz's buffer (2 (nz - 1) values).
void launch_stage_rdz(hipStream_t s, int nz, const double* z, double* rdz);
void launch_cast_d2f(hipStream_t s, int nblocks, long n, const double* a, float* b);
void launch_masked_copy_d2d(hipStream_t s, int nblocks, long n, const uint8_t* mask, const double* a, double* b);
void launch_masked_copy_d2f(hipStream_t s, int nblocks, long n, const uint8_t* mask, const double* a, float* b);
// Coarse-mesh sequence: the coarse problem's coordinates, materials and
// Dirichlet ids from the fine one (c's arrays are device memory the caller
// owns), and the coarse potential interpolated onto the fine nodes.
void launch_seq_coarsen(hipStream_t s, const qe_problem* f, const qe_problem* c);
void launch_seq_prolong(hipStream_t s, const qe_problem* f, const qe_problem* c, const double* phic, double* phif);
// Per-axis tables between a level and the next finer one: for each fine
// index its coarse interval pI and upper-end weight pw (interpolation), for
// each coarse index its three fine taps rI and weights rw (restriction).
struct MgAxes {
  int* pI[3];
  double* pw[3];
  int* rI[3];
  double* rw[3];
};
// Multigrid preconditioner of the CG (qe_mg.hip): one level's mesh,
// linearisation (the arrays of its residual) and vectors, in FP64 and, for
// the mixed-precision CG, FP32.  On level 0, b is the CG's r, x its z and S
// the array the CG kernels use in place of D^-1.
struct MgGrid {
  Geom g;
  WaveMap wm;
  long N;
  const unsigned int* cbits;   // J.v lanes' coefficient flags
  const uint8_t* mask;         // Dirichlet nodes
  const double* eps_t;         // tile-major permittivity
  const double* cq;            // tile-major Gauss-point coefficients
  double* S;                   // l1-Jacobi smoother weights (0 on Dirichlet nodes)
  double *b, *x, *y;           // right-hand side, iterate, J x
  const float* eps32;          // the same in FP32
  const float* cq32;
  float* S32;
  float *b32, *x32, *y32;
  MgAxes tab;                  // tables to the next finer level (levels >= 1)
};
// The tables of the level pair (f finer, c coarser) into c.tab.
void launch_mg_tables(hipStream_t s, const MgGrid& f, const MgGrid& c);
// The coarse problem's eigenstate arrays from the fine one's (|psi|^2 and
// phi^(k) at the coarse nodes, each coarse element's region flag from its
// first fine element); c->quantum's arrays are device memory the caller owns.
void launch_mg_coarsen_states(hipStream_t s, const qe_problem* f, const qe_problem* c);
// phi_c = phi_f at the coarse level's nodes f(I) = min(2 I, n - 1).
void launch_mg_inject(hipStream_t s, const MgGrid& f, const MgGrid& c, const double* phif, double* phic);
// L.S (and L.S32 with fp32) from the level's permittivity (natural element
// order), coefficient flags and FP64 coefficients.
void launch_mg_l1(hipStream_t s, const MgGrid& L, const double* eps_natural, const uint8_t* cflag, double omega,
                  bool fp32);
// z = B r on level 0 (x = S r on entry), in FP32 with fp32; one r^T z
// partial per block of the last kernel (cgblocks blocks) into part_rz.
// add_top: the finest level adds the coarse correction to S r instead of
// smoothing around it.  Skipped once ctx->done.
void launch_mg_vcycle(hipStream_t s, const MgGrid* levels, int nlev, int sweeps, bool add_top, int cgblocks,
                      double* part_rz, const PcgCtx* ctx, bool fp32);
// After a CG start with z = S r and the V-cycle: r_0^T z_0 and the
// tolerance from the V-cycle's partials.
void launch_mg_start_fin(hipStream_t s, PcgCtx* ctx, const double* part, int n);
WaveMap make_wavemap(int nx, int ny, int nz, int kz);
// The residual with eigenstates (qm.n > 0) runs on the wave map wmq (shorter
// chunks: the states' loop makes the waves over the dot the slowest) and
// leaves the J.v lanes' coefficient flags (cbits, wave map wm) to a pass
// over the owners' element flags.
void launch_residual_wave(hipStream_t s, const Geom& g, const WaveMap& wm, const WaveMap& wmq, const Charge& ch,
                          const double* eps, const uint8_t* semi, const Doping& dop, const uint8_t* mask,
                          const double* phi, const double* delta64, const float* delta32, double lam,
                          const double* fsheet, const double* fdiag, double* F, double* invdiag, double* diag_out,
                          double* cq, float* cq32, uint8_t* cflag, unsigned int* cbits, float* invdiag32,
                          double* partial, double* norm2, const Quantum& qm);
// y = J v with v read as 0 on Dirichlet nodes (identity_rows: y_i = v_i there).
void launch_jv_wave64(hipStream_t s, const Geom& g, const WaveMap& wm, const double* eps, const unsigned int* cbits,
                      const double* cq, const uint8_t* mask, const double* v, double* y, int identity_rows);
void launch_jv_wave32(hipStream_t s, const Geom& g, const WaveMap& wm, const float* eps, const unsigned int* cbits,
                      const float* cq, const uint8_t* mask, const float* v, float* y, int identity_rows);
// First kernel of CG iteration k: stopping test, beta, y = J z + beta y,
// p = z + beta p, in FP64 the previous iteration's x += alpha p (x is not
// touched in FP32), p^T y partials.
void launch_cg_jv64(hipStream_t s, const Geom& g, const WaveMap& wm, int cgblocks, int k, const double* eps_t,
                    const unsigned int* cbits, const double* cq, const double* z, double* y, double* p, double* x,
                    PcgCtx* ctx, CgProgress* prog, const double* part_rz, double* part_py);
void launch_cg_jv32(hipStream_t s, const Geom& g, const WaveMap& wm, int cgblocks, int k, const float* eps_t,
                    const unsigned int* cbits, const float* cq, const float* z, float* y, float* p, float* x,
                    PcgCtx* ctx, CgProgress* prog, const double* part_rz, double* part_py);
// After an FP64 CG loop: the last iteration's x += alpha p (none after a
// breakdown).
void launch_cg_finish_x64(hipStream_t s, int nblocks, long N, const PcgCtx* ctx, const double* p, double* x);
// Tile-major permittivity copy for the wave-tiled J.v (see tile_slot).
void launch_stage_eps64(hipStream_t s, int nblocks, const Geom& g, const double* eps, double* eps_t, long nslots);
void launch_stage_eps32(hipStream_t s, int nblocks, const Geom& g, const double* eps, float* eps_t, long nslots);
// Count of real elements with a set tile-major flag, added to *out.
void launch_count_flags(hipStream_t s, int nblocks, const Geom& g, const uint8_t* flag, long nslots,
                        unsigned long long* out);
void launch_axpy_phi(hipStream_t s, int nblocks, long N, double* phi, const double* d64, const float* d32,
                     double lam);
// CG start: x = 0, r = sign*b (free rows), z = D^-1 r, then the scalars
// (cgblocks r^T z partials).
void launch_pcg_start64(hipStream_t s, int cgblocks, long N, double sign, const double* b, const uint8_t* mask,
                        const double* invdiag, double* x, double* r, double* z, PcgCtx* ctx, double* part_rz,
                        double rtol, int maxit);
void launch_pcg_start32(hipStream_t s, int cgblocks, long N, double sign, const double* b, const uint8_t* mask,
                        const float* invdiag, float* x, float* r, float* z, PcgCtx* ctx, double* part_rz,
                        double rtol, int maxit);
// CG iteration (parity k): k_cg_jv, the Robin faces' product when S has any
// (its partials appended after the J.v's), then k_cg_update on cgblocks blocks.
void launch_pcg_iter64(hipStream_t s, const Geom& g, const WaveMap& wm, int cgblocks, long N, int k,
                       const double* eps_t, const unsigned int* cbits, const double* cq, const double* invdiag, double* x,
                       double* r, double* z, double* p, double* y, PcgCtx* ctx, CgProgress* prog, double* part_py,
                       double* part_rz, const SheetSet* S, const int4* items, const uint8_t* mask);
void launch_pcg_iter32(hipStream_t s, const Geom& g, const WaveMap& wm, int cgblocks, long N, int k,
                       const float* eps_t, const unsigned int* cbits, const float* cq, const float* invdiag, float* x,
                       float* r, float* z, float* p, float* y, PcgCtx* ctx, CgProgress* prog, double* part_py,
                       double* part_rz, const SheetSet* S, const int4* items, const uint8_t* mask);

// ---- interface-charge / Robin sheets (qe_sheets.hip)
constexpr int kSheetBlocks = 256;
int sheet_blocks(const SheetSet& S);
// fsheet[n] = face terms of F(phi + lam delta) at free sheet nodes, fdiag[n]
// their Jacobian diagonal (other entries untouched).
void launch_sheet_residual(hipStream_t s, const SheetSet& S, const int4* items, double kappa, const uint8_t* mask,
                           const double* phi, const double* delta64, const float* delta32, double lam, double* fsheet,
                           double* fdiag);
// y += R v on free sheet nodes (v masked); with ctx, skipped once the CG has
// stopped and one p^T R v partial per block into part.
void launch_sheet_jv64(hipStream_t s, const SheetSet& S, const int4* items, const uint8_t* mask, const double* v,
                       double* y, const double* p, const PcgCtx* ctx, double* part);
void launch_sheet_jv32(hipStream_t s, const SheetSet& S, const int4* items, const uint8_t* mask, const float* v,
                       float* y, const float* p, const PcgCtx* ctx, double* part);
// tcon -= R lam on Dirichlet sheet nodes (the adjoint's contact terms).
void launch_sheet_contact(hipStream_t s, const SheetSet& S, const int4* items, const uint8_t* mask, const double* lam,
                          double* tcon);
void launch_validate_sheets(hipStream_t s, const SheetSet& S, int* flags);

}  // namespace qe
