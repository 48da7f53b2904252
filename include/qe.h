/*
 * qe.h -- C ABI of the MI355X semiclassical nonlinear-Poisson library.
 *
 * The library solves the discrete Galerkin form (Eq. PoissonWeakForm, Sec.
 * II.A) of
 *
 *     -div(eps_r grad phi) = KAPPA * (p - n + N_D+ - N_A-),   KAPPA = q/eps0
 *
 * (Eq. Poisson) on a rectilinear Q1 hexahedral mesh of a Si/SiO2 gate stack.
 * Carriers follow Thomas-Fermi (T = 0), Maxwell-Boltzmann (Eq. MBstatistics)
 * or Fermi-Dirac statistics with the Bednarczyk F_1/2 form (Eqs.
 * FDstatistics, EffectiveDOS, FDIntApprox, with exp(x) below x = -50).  By
 * default holes are absent and dopants fully ionised (p = 0, N_D+ - N_A- =
 * net_doping); qe_physics switches on holes and incomplete ionization
 * (Eqs. Ionization, FinalIonization).  Gate electrodes and contacts are
 * Dirichlet nodes (Eq. ContOnIns with a mid-gap work function, so a gate node
 * carries its applied voltage; Ohmic contacts take qe_ohmic_potential);
 * every other outer face is the default zero-flux Neumann boundary (Sec.
 * II.A.4).
 * Newton's method with the exact Jacobian (Sec. II.A.3, II.C) is globalised
 * by backtracking; the linear systems are solved by Jacobi-preconditioned
 * conjugate gradients, all on the GPU.
 *
 * Units: lengths nm, potentials V, energies eV, densities nm^-3
 * (1 cm^-3 = 1e-21 nm^-3), temperatures K.  The residual is in V*nm.
 *
 * Layout: node (i, j, k) is i + nx*(j + ny*k) (x fastest); element (i, j, k),
 * whose lowest corner is node (i, j, k), is i + (nx-1)*(j + (ny-1)*k).
 * E_F = 0 (grounded substrate, Sec. II.A.2), E_F - E_C = phi - Ec0 and, with
 * holes, E_V - E_F = Ec0 - Eg - phi (Eq. EcEv_phi with the constant offset
 * folded into Ec0).
 *
 * Conventions shared by every entry point:
 *  - Every array pointer in qe_problem and every "device" argument is DEVICE
 *    memory allocated and owned by the caller; "host" arguments are host
 *    memory.  The library never frees caller memory.
 *  - `ws` is caller-owned device scratch of at least qe_workspace_bytes()
 *    bytes, 256-byte aligned; its contents on entry are irrelevant and on
 *    return unspecified.  Concurrent calls must not share a workspace.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    device work is enqueued on it; every entry point returns after
 *    synchronising that stream (the Newton decisions are taken on the host).
 *  - Errors never abort: a negative qe_status is returned and
 *    qe_last_error() describes it.  Invalid arguments are detected before any
 *    device work is enqueued, except the device-array checks (eps_r > 0,
 *    finiteness, dir_id range), which a validation kernel performs first.
 *    On QE_ERR_NOT_CONVERGED / QE_ERR_LINESEARCH / QE_ERR_KRYLOV_* the last
 *    iterate is still written to phi and the report.
 */
#ifndef QE_H
#define QE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QE_OK = 0,
  QE_ERR_INVALID_ARG = -1,       /* bad sizes, NULL pointers, options out of range */
  QE_ERR_HIP = -2,               /* a HIP runtime call failed */
  QE_ERR_WORKSPACE = -3,         /* ws NULL, misaligned or smaller than required */
  QE_ERR_NOT_CONVERGED = -4,     /* Newton hit newton_maxit above newton_atol */
  QE_ERR_LINESEARCH = -5,        /* no sufficient decrease after ls_max_halvings */
  QE_ERR_KRYLOV_BREAKDOWN = -6,  /* p^T J p <= 0 or non-finite inside CG */
  QE_ERR_NONFINITE = -7,         /* NaN/Inf in inputs or in the residual */
  QE_ERR_KRYLOV_MAXIT = -8       /* a linear solve hit krylov_maxit (adjoint only) */
} qe_status;

typedef enum {
  QE_STAT_LINEAR = 0,            /* no mobile charge (doping only) */
  QE_STAT_TF = 1,                /* Thomas-Fermi: n = C_TF max(0, phi-Ec0)^(3/2) */
  QE_STAT_FD12 = 2,              /* n = N_C F_1/2((phi-Ec0)/kT), Eq. FDIntApprox */
  QE_STAT_MB = 3                 /* n = N_C exp((phi-Ec0)/kT), Eq. MBstatistics */
} qe_statistics;

typedef enum {
  QE_ION_COMPLETE = 0,           /* N_D+ - N_A- = net_doping */
  QE_ION_INCOMPLETE = 1          /* Eq. FinalIonization from donors / acceptors */
} qe_ionization;

typedef enum {
  QE_PREC_FP64 = 0,              /* everything in FP64 */
  QE_PREC_MIXED = 1              /* J.v and CG in FP32; residual, charge, line search,
                                    Newton update in FP64 */
} qe_precision;

/* Preconditioner of the CG (the paper's solver library leaves it to
 * the user; Sec. II.A.3).  Jacobi: z = D^-1 r.  Multigrid: a symmetric
 * V-cycle on the meshes of the coarse-mesh sequence (every other node along
 * each axis, the last kept, while the coarser mesh keeps at least 2000
 * nodes), each with the coarse problem's own Jacobian at the injected
 * potential; trilinear prolongation P, restriction P^T, one weighted
 * l1-Jacobi smoothing step (S = 1.8 / sum_j |J_ij|) before and one after the
 * coarse correction, four on the coarsest mesh; on meshes of 4M nodes and
 * more the finest level only adds its correction (z = S r + P B_1 P^T r).
 * It is symmetric positive definite (any weight below 2 keeps it so), so
 * the CG stays plain CG.  AUTO takes multigrid for the Newton steps whose
 * CG tolerance is at most 3e-2 (1e-1 on meshes of 4M nodes and more, where
 * a V-cycle costs less relative to a Jacobi iteration) and for the adjoint,
 * where one V-cycle saves more iterations than it costs, and Jacobi
 * otherwise.  In mixed precision the
 * V-cycle runs in FP32 like the CG it serves.  With sheets the V-cycle
 * leaves out the Robin face term (it stays positive definite); with
 * eigenstates every coarse mesh carries them, injected like the potential.
 * Multigrid needs a mesh of at least 250000 nodes and an entry point that
 * allocates; elsewhere every choice runs Jacobi. */
typedef enum {
  QE_PC_AUTO = 0,
  QE_PC_JACOBI = 1,
  QE_PC_MULTIGRID = 2            /* multigrid for every CG solve it can serve */
} qe_precond;

/* A rectangle of mesh faces carrying a surface charge and / or a Robin
 * condition (Sec. II.A.4).  The sheet lies in the node plane
 * x_axis = coordinate[plane] (axis 0: x, 1: y, 2: z) and covers faces a0..a1-1
 * along its first in-plane axis and b0..b1-1 along its second (axis 2: x then
 * y; axis 1: x then z; axis 0: y then z); a face is the rectangle between
 * nodes a..a+1 and b..b+1 of that plane.  It may lie inside the mesh (an
 * interface) or on its outer boundary.  On every face f the weak form gains
 *  - the surface-charge load KAPPA sigma_f int_f w_i (Eq. NeuBC4fc: the flux
 *    jump across the face is q sigma_f; positive sigma = positive charge);
 *  - with robin_d > 0, the Robin term alpha int_f (phi - phi0) w_i with
 *    alpha = robin_eps / robin_d: the potential is pinned to phi0 on a plane
 *    robin_d beyond the face, through a layer of relative permittivity
 *    robin_eps (the charged-gate construction of Sec. II.A.4, d = 10 nm there).
 * Both integrals are exact (bilinear traces on rectangles).  Rows of
 * Dirichlet nodes are unaffected.  Sheets may share nodes and planes. */
typedef struct {
  int32_t axis;                  /* 0, 1 or 2 */
  int32_t plane;                 /* node index along `axis`, in [0, n_axis) */
  int32_t a0, a1;                /* 0 <= a0 < a1 <= n_a - 1 */
  int32_t b0, b1;                /* 0 <= b0 < b1 <= n_b - 1 */
  const double* sigma;           /* DEVICE [(a1-a0)*(b1-b0)], a fastest, nm^-2,
                                    finite; NULL = no surface charge */
  double robin_d;                /* nm, finite, >= 0; 0 = no Robin term */
  double robin_eps;              /* > 0 when robin_d > 0 */
  double phi0;                   /* V, finite */
} qe_sheet;

#define QE_MAX_SHEETS 16

/* Eigenstates of an earlier outer Schrodinger-Poisson iteration k, for the
 * predictor step of the predictor-corrector method (Eq. pcPoisson): the
 * electron density becomes
 *   n~(phi) = sum_i P |psi_i|^2 G((E_F - E_i + (phi - phi^(k))) / kT)
 * with 3D confinement (Eq. ApproxEDens3DConfined) P = 4, G(x) = 1/(1 + e^-x)
 * -- the printed minus sign in front of q(phi - phi^(k)) in its exponent --
 * and with 1D confinement (Eq. ApproxEDens1DConfined)
 * P = 2 m_t kT / (pi hbar^2), G(x) = ln(1 + e^x).  |psi_i|^2 and phi^(k) are
 * nodal fields interpolated to the Gauss points like phi.  n~ replaces the
 * electron statistics in the quantum region (holes and dopants stay as
 * qe_physics says; nodal densities take n~ at nodes touching the region);
 * T_K > 0 is needed.  Supported by qe_solve, qe_residual, qe_jv, qe_jv_f32,
 * qe_density and qe_count_electrons (which then report n~); qe_adjoint and
 * qe_solve_batch reject it. */
#define QE_MAX_STATES 32
typedef struct {
  int32_t n_states;              /* 1 .. QE_MAX_STATES */
  int32_t confinement;           /* 3 or 1 */
  const double* psi2;            /* DEVICE [n_states][N] nodal |psi_i^(k)|^2, finite,
                                    >= 0 (nm^-3 for 3D, nm^-1 for 1D) */
  const double* phi_k;           /* DEVICE [N] the potential phi^(k), V */
  const double* E_i;             /* HOST [n_states] levels E_i^(k) - E_F, eV, finite */
  double m_t;                    /* transverse mass / m0, > 0 (1D form) */
  const uint8_t* region;         /* DEVICE [E] nonzero: the element's electrons are n~
                                    (the quantum region); elsewhere the statistics;
                                    NULL = every element */
} qe_quantum;

/* One device.  All pointers are DEVICE memory, read only, except `sheets`
 * and `quantum`. */
typedef struct {
  int32_t nx, ny, nz;            /* nodes per axis, each >= 2 */
  const double* x;               /* [nx] nm, strictly increasing */
  const double* y;               /* [ny] */
  const double* z;               /* [nz] */
  const double* eps_r;           /* [E] relative permittivity, finite, > 0 */
  const uint8_t* semi;           /* [E] 1 = semiconductor (carries electrons and
                                    doping), 0 = insulator */
  const double* net_doping;      /* [E] N_D - N_A in nm^-3 (complete ionization);
                                    NULL means donors - acceptors when those are
                                    given, else 0 */
  const int32_t* dir_id;         /* [N] -1 = free node, else index < n_dir */
  const double* dir_val;         /* [n_dir] Dirichlet potential in V */
  int32_t n_dir;                 /* >= 0; a problem with no Dirichlet node needs
                                    n'(phi) > 0 somewhere to be solvable */
  const double* donors;          /* [E] N_D in nm^-3, finite, >= 0, or NULL; required
                                    with QE_ION_INCOMPLETE */
  const double* acceptors;       /* [E] N_A in nm^-3, likewise; NULL exactly when
                                    donors is NULL */
  int32_t n_sheets;              /* 0 .. QE_MAX_SHEETS; not supported by
                                    qe_solve_batch */
  const qe_sheet* sheets;        /* HOST array [n_sheets] (its sigma arrays are
                                    device memory); NULL when n_sheets = 0 */
  const qe_quantum* quantum;     /* HOST, or NULL: electrons from the statistics */
} qe_problem;

typedef struct {
  int32_t stat;                  /* qe_statistics (electrons and holes) */
  double T_K;                    /* > 0 for QE_STAT_FD12 / QE_STAT_MB and for
                                    incomplete ionization, ignored otherwise */
  double m_eff;                  /* conduction DOS mass / m0 (Eq. EffectiveMass), > 0 */
  double Ec0_eV;                 /* E_C - E_F at phi = 0 */
  int32_t holes;                 /* 1: p(phi) from the same statistics (Eq. Poisson) */
  double m_h;                    /* valence DOS mass / m0 (Eq. EffectiveMass), > 0 with holes */
  double Eg_eV;                  /* band gap, E_V = E_C - Eg (Eq. EcEv_phi), >= 0 */
  int32_t ionization;            /* qe_ionization; incomplete needs T > 0 and
                                    QE_STAT_FD12 or QE_STAT_MB */
  double Ed_eV, Ea_eV;           /* donor / acceptor ionization energies (Sec. II.A.3) */
  double gD, gA;                 /* ground-state degeneracy factors, > 0 (2 and 4 for Si) */
} qe_physics;

typedef struct {
  double newton_atol;            /* stop when ||F_free||_2 <= atol (V nm), > 0 */
  int32_t newton_maxit;          /* >= 0 */
  int32_t ls_max_halvings;       /* >= 0 */
  double krylov_rtol_max;        /* cap of the inexact-Newton forcing term, (0, 1) */
  int32_t krylov_maxit;          /* CG iterations per linear solve, >= 1 */
  int32_t precision;             /* qe_precision */
  int32_t init_guess;            /* 0: linear (charge-free) Poisson solve;
                                    1: start from the phi passed in;
                                    2: coarse-mesh sequence (see qe_solve) */
  int32_t check_every;           /* CG iterations the host keeps queued beyond
                                    those known to have finished (0 = 9;
                                    clamped to [9, 56]) */
  int32_t precond;               /* CG preconditioner (qe_precond) */
} qe_options;

typedef struct {
  int32_t status;                /* qe_status of the call */
  int32_t newton_iters;
  int32_t krylov_iters;          /* total CG iterations incl. the initial guess */
  int32_t ls_halvings;
  int32_t init_krylov_iters;
  int32_t n_residual_evals;
  double res0;                   /* ||F_free|| at the first Newton iterate */
  double res_final;              /* ||F_free|| at the returned phi */
  int32_t seq_levels;            /* coarse meshes solved for the initial guess
                                    (init_guess = 2), 0 for the linear guess */
  int32_t mg_levels;             /* meshes of the multigrid preconditioner when
                                    it served a CG solve of the call, else 0 */
  int32_t mg_krylov_iters;       /* CG iterations preconditioned by multigrid
                                    (part of krylov_iters) */
} qe_report;

/* Fill `o` with defaults (atol 1e-8, 100 Newton steps, 30 halvings, forcing
 * cap 0.3, 20000 CG iterations, FP64, coarse-mesh sequence, QE_PC_AUTO).  The forcing
 * term is eta_k = min(cap, 0.9 (|F_k| / |F_k-1|)^2) (Eisenstat-Walker), and
 * the linear initial guess is solved to a relative CG residual of 1e-2. */
void qe_default_options(qe_options* o);

/* Bytes of workspace any entry point below needs for this problem. */
size_t qe_workspace_bytes(const qe_problem* p, const qe_options* o);

/* Nonlinear solve (Sec. II.A; initial guess, residual, Jacobian, CG, line
 * search, Newton update).  phi: device [N]; on entry the guess when
 * init_guess = 1 (its Dirichlet entries are overwritten), on return the
 * solution.  n_nodal: device [N] or NULL; receives n(phi_i) at nodes that
 * touch a semiconductor element, 0 elsewhere.  rep: host, may be NULL.
 * The paper leaves Newton's start open (Sec. II.A.3).  With init_guess = 2
 * a mesh of at least 250000 nodes without sheets or eigenstates is first
 * coarsened (every other node along each axis, the last one kept; each
 * coarse element takes the materials of its first fine element), that
 * problem is solved from the linear guess until ||F|| falls to a fraction
 * 1e-3 (139425 / N_coarse)^(1/3) of its initial value (a finer coarse mesh
 * is worth solving further; measured; its CG runs in FP32 inside its FP64
 * Newton, as in mixed precision), and its potential, interpolated
 * trilinearly, starts Newton here; the solution is the same (the discrete problem has one
 * solution), only the iteration counts change.  Smaller meshes, sheets,
 * eigenstates, a coarse solve that fails, or a workspace without room for
 * the coarse levels (qe_workspace_bytes counts them) take the linear
 * guess. */
qe_status qe_solve(const qe_problem* p, const qe_physics* ph, const qe_options* o,
                   double* phi, double* n_nodal, void* ws, size_t ws_bytes,
                   void* stream, qe_report* rep);

/* qe_solve for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid allocation).  The same
 * problem, options, results and errors as qe_solve, without a caller
 * workspace: the library uses a static device array of QE_STATIC_WS_BYTES
 * bytes (256 MiB, enough for 129 x 129 x 65 nodes) that it holds on each GPU
 * it runs on until the process ends.  The call allocates no device or
 * pinned host memory and creates no HIP event (its CG loop is polled by
 * stream synchronisations instead of events and a posted host word).
 * QE_ERR_WORKSPACE, before any device work, when qe_workspace_bytes(p, o)
 * exceeds QE_STATIC_WS_BYTES.  Every call on one GPU uses that GPU's array,
 * which keeps the last call's contents (a solve writes every part it reads
 * first), so calls that overlap on one GPU race. */
#define QE_STATIC_WS_BYTES (256u << 20)
qe_status qe_solve_static(const qe_problem* p, const qe_physics* ph, const qe_options* o, double* phi,
                          double* n_nodal, void* stream, qe_report* rep);

/* Residual of Eq. PoissonWeakForm at phi (device [N], used as given, Dirichlet
 * entries included): F device [N] (free rows; 0 on Dirichlet rows).
 * diag: device [N] or NULL, the Jacobian diagonal (1 on Dirichlet rows).
 * norm2: host scalar or NULL, ||F_free||_2^2. */
qe_status qe_residual(const qe_problem* p, const qe_physics* ph, const double* phi,
                      double* F, double* diag, double* norm2,
                      void* ws, size_t ws_bytes, void* stream);

/* Jacobian-vector product at phi (exact derivative of the coded residual):
 * y = J(phi) v with v masked to 0 on Dirichlet nodes, and y_i = v_i on
 * Dirichlet rows.  phi, v, y: device [N]. */
qe_status qe_jv(const qe_problem* p, const qe_physics* ph, const double* phi,
                const double* v, double* y, void* ws, size_t ws_bytes, void* stream);

/* The same product computed in FP32 (the mixed-precision inner operator):
 * the linearisation is formed in FP64 at phi, then rounded to FP32. */
qe_status qe_jv_f32(const qe_problem* p, const qe_physics* ph, const double* phi,
                    const float* v, float* y, void* ws, size_t ws_bytes, void* stream);

/* Electron count in boxes (Sec. III: N = integral of n over the dot region):
 * sum over semiconductor elements whose centroid lies in the closed box of
 * sum_q W_q n(phi_q).  boxes: host [n_boxes][6] = x0,x1,y0,y1,z0,z1 (nm);
 * counts: host [n_boxes].  1 <= n_boxes <= 16. */
qe_status qe_count_electrons(const qe_problem* p, const qe_physics* ph, const double* phi,
                             int32_t n_boxes, const double* boxes, double* counts,
                             void* ws, size_t ws_bytes, void* stream);

/* Nodal electron density (as qe_solve's n_nodal) at phi.  n: device [N]. */
qe_status qe_density(const qe_problem* p, const qe_physics* ph, const double* phi,
                     double* n, void* ws, size_t ws_bytes, void* stream);

/* Adjoint gradient of Q = electrons in `box` (host [6]) at a converged phi
 * (device [N]), for the capacitance C_g = q dQ/dV_g of Sec. III and gate
 * design loops (Sec. IV):
 *   J_ff lam = dQ/dphi_f (same CG, J symmetric),
 *   dQ/dV_c   = sum_{i in contact c} (dQ/dphi_i - (J lam)_i),
 *   dQ/deps_e = -lam_e^T Khat_e phi_e.
 * Q: host scalar or NULL.  dQ_ddir: host [n_dir] (per Dirichlet value).
 * dQ_deps: device [E] or NULL.  lam: device [N] or NULL (adjoint state).
 * opts: krylov_maxit and precision (must be FP64) are used; the adjoint CG
 * stops when the preconditioned residual norm (r^T D^-1 r)^(1/2) falls to
 * 1e-12 of its initial value.  rep: host or NULL. */
qe_status qe_adjoint(const qe_problem* p, const qe_physics* ph, const qe_options* o,
                     const double* phi, const double* box, double* Q, double* dQ_ddir,
                     double* dQ_deps, double* lam, void* ws, size_t ws_bytes,
                     void* stream, qe_report* rep);

/* Batched solve of many independent devices in one persistent launch: the
 * design searches of Sec. IV run many device simulations at once (gate
 * voltages varied as parameters, many layouts side by side, each device the
 * nonlinear Poisson problem of Sec. II.A), which here becomes a gate-voltage
 * sweep over uneven meshes on one GPU.  Newton, line search and CG run on
 * the device for every instance, with the same algorithm and stopping rules
 * as qe_solve.
 *   probs: host [n_inst] of qe_problem (device arrays inside);
 *   phi: host [n_inst] of device pointers, each [N_k]; out: solutions;
 *   boxes: host [n_boxes][6]; counts: host [n_inst][n_boxes] (may be NULL
 *     when n_boxes = 0);
 *   tune_cache: path of the autotuner's cache file (NULL = no cache);
 *   reps: host [n_inst] or NULL.
 * All instances share ph and o; o->precision must be FP64. */
size_t qe_batch_workspace_bytes(int32_t n_inst, const qe_problem* probs, const qe_options* o);
qe_status qe_solve_batch(int32_t n_inst, const qe_problem* probs, const qe_physics* ph,
                         const qe_options* o, double* const* phi, int32_t n_boxes,
                         const double* boxes, double* counts, const char* tune_cache,
                         void* ws, size_t ws_bytes, void* stream, qe_report* reps);

/* Benchmark helper: forms the linearisation at phi (device [N]), sets up a
 * CG state from v (device [N], FP64): z = D^-1 v on free rows and 0 on
 * Dirichlet rows, y = p = 0, beta = 1 (FP32 copies with QE_PREC_MIXED), then
 * launches the first kernel of a CG iteration -- y = J z + beta y,
 * p = z + beta p and the p^T y partial sums -- `reps` times between two HIP
 * events on `stream`.
 * ms_per_apply: host, mean kernel time per launch.
 * n_coef_elems: host or NULL; the number of elements whose Gauss-point
 *   coefficients are not all exactly zero at phi, i.e. the elements whose
 *   coefficients the kernel reads (the others add exactly nothing). */
qe_status qe_time_jv(const qe_problem* p, const qe_physics* ph, const double* phi, const double* v,
                     int32_t precision, int32_t reps, double* ms_per_apply, int64_t* n_coef_elems,
                     void* ws, size_t ws_bytes, void* stream);

/* Dirichlet value of an Ohmic contact on semiconductor (Sec. II.A.4, second
 * case): thermal equilibrium and charge neutrality of the majority carriers
 * at the contact, in this library's convention (E_F = 0, E_C = Ec0 - phi).
 * n-type when N_D >= N_A, else p-type (densities in nm^-3, host scalars).
 *  - complete ionization, QE_STAT_MB: Eq. PotBC4MBCompIon with the net
 *    doping |N_D - N_A| as the majority density;
 *  - complete ionization, QE_STAT_FD12: Eq. PotBC4FDCompIon with eta from the
 *    Nilsson inverse (Eq. FDintInverse), likewise;
 *  - incomplete ionization (MB or FD, as the paper does for FD): Eqs.
 *    Yval4MBIncompIon and PotBC4MBIncompIon with the majority dopant alone,
 *    ln y from Eq. ApproxLogTerms once exp(E_d/kT) terms exceed 1e300; the
 *    p-type form carries +E_a, which the definitions of y_p and E_a give.
 * V_a: applied voltage (V), added as printed.  phi: host, out.
 * Errors: QE_ERR_INVALID_ARG for TF or linear statistics, T <= 0, a zero or
 * negative majority density, or NULL pointers. */
qe_status qe_ohmic_potential(const qe_physics* ph, double N_D, double N_A, double V_a, double* phi);

/* Effective-mass Schrodinger eigenproblem on the same Q1 mesh (Sec. II.B,
 * Eqs. SchrodEqn, SchrodEqnWeakForm, and Eq. Schrodinger3D's per-axis masses,
 * Sec. II.C): H psi = E M psi with
 *   H_ij = sum_e (hbar^2/2m0) sum_a (m0/m*_e,a) int_e d_a w_i d_a w_j + int V w_i w_j,
 *   M_ij = int w_i w_j,  V = v0_e - phi (eV; phi interpolated to the Gauss
 * points), a over x, y, z (a diagonal mass tensor per element: m_t, m_t, m_l
 * for the Delta_2 valleys of a Si dot), psi = 0 on the `fixed` nodes and
 * natural (Neumann) conditions on every other boundary.  Only nx, ny, nz,
 * x, y, z of the qe_problem are read. */
typedef struct {
  const double* inv_mass;        /* DEVICE [3][E] m0 / m*_e along x, then y, then z
                                    (three planes of E), finite, > 0 */
  const double* v0;              /* DEVICE [E] conduction-band edge at phi = 0 relative
                                    to E_F, eV, finite (Ec0 in Si, plus the band
                                    offset in an insulator) */
  const uint8_t* fixed;          /* DEVICE [N] nonzero: psi = 0 there; or NULL */
} qe_schrodinger;

#define QE_MAX_EIG 16

/* Device scratch of qe_schrodinger_solve for n_states states (0 if invalid). */
size_t qe_schrodinger_workspace_bytes(const qe_problem* p, int32_t n_states);

/* Lowest n_states (1 .. QE_MAX_EIG) eigenpairs by block LOBPCG (Knyazev's
 * locally optimal block preconditioned CG) on H - sigma M with sigma below
 * every V (so the operator is SPD), two guard vectors, the Jacobi
 * preconditioner, soft locking of converged vectors, and Rayleigh-Ritz on
 * the block [X, W, P] (Gram matrices on the GPU; the small dense generalized
 * eigenproblem on the host).  Operators use the wave-tiled J.v.
 * The iteration runs on the bounding box of the free nodes grown by one
 * node whenever that box is smaller than the mesh and the workspace holds
 * it next to the box's copies of the inputs (the eigenpairs are the same:
 * psi vanishes outside it); psi and psi2 are written on the whole mesh.
 * phi: device [N].  Stops when every wanted pair has
 * ||H x - E M x||_2 <= tol (||H x||_2 + |E| ||M x||_2) or after maxit
 * iterations (QE_ERR_NOT_CONVERGED, results still written).
 * E: host [n_states] ascending, eV.  psi: device [n_states][N], M-orthonormal,
 * 0 on fixed nodes (sign arbitrary).  psi2: device [n_states][N] or NULL,
 * receives psi^2 (the input of qe_quantum).  iters: host or NULL.
 * seed: the starting block's counter-based random numbers (SplitMix64).
 * guess: nonzero = psi holds starting vectors on entry (e.g. the previous
 * outer iteration's states; the two guard vectors stay random). */
qe_status qe_schrodinger_solve(const qe_problem* p, const qe_schrodinger* s, const double* phi,
                               int32_t n_states, double tol, int32_t maxit, uint64_t seed, int32_t guess,
                               double* E, double* psi, double* psi2, int32_t* iters,
                               void* ws, size_t ws_bytes, void* stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char* qe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QE_H */
