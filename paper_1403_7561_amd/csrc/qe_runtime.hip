// Host runtime and C ABI of the Q1 nonlinear-Poisson library (see qe.h).
//
// The Newton iteration is driven from the host: one scalar read per residual
// evaluation and one per block of CG iterations.  Inside a linear solve every
// scalar (alpha, beta, residual norms, the stop flag) lives on the device, so
// a block of CG iterations is a plain sequence of kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qe.h"
#include "qe_kernels.h"
#include "qe_runtime.h"

namespace qe {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

qe_status fail(qe_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

void clear_error() { g_last_error.clear(); }

#define QE_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(QE_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                                \
  } while (0)


// ------------------------------------------------------------------ physics
// CODATA 2018 values (q, hbar, kB exact).
static const double kQ = 1.602176634e-19, kEps0 = 8.8541878128e-12, kHbar = 1.054571817e-34,
                    kM0 = 9.1093837015e-31, kKB = 1.380649e-23, kPi = 3.14159265358979323846;

// Effective density of states (Eq. EffectiveDOS) in nm^-3 and the T = 0
// density prefactor C (n = C u^(3/2), u in eV) from integrating the 3D
// density of states up to E_F.
static double effective_dos(double m_eff, double T_K) {
  const double m = m_eff * kM0, kT_J = kKB * T_K;
  return 2.0 * std::pow(m * kT_J / (2.0 * kPi * kHbar * kHbar), 1.5) * 1e-27;
}

static double tf_prefactor(double m_eff) {
  const double m = m_eff * kM0;
  return std::pow(2.0 * m * kQ, 1.5) / (3.0 * kPi * kPi * kHbar * kHbar * kHbar) * 1e-27;
}

static bool positive(double v) { return v > 0.0 && std::isfinite(v); }

qe_status make_charge(const qe_physics* ph, Charge& ch) {
  if (!ph) return fail(QE_ERR_INVALID_ARG, "physics is NULL");
  std::memset(&ch, 0, sizeof(ch));
  ch.kappa = kQ / kEps0 * 1e9;  // V nm: Poisson divided by eps0, nm units
  ch.Ec0 = ph->Ec0_eV;
  ch.T_K = ph->T_K;
  if (!std::isfinite(ph->Ec0_eV)) return fail(QE_ERR_INVALID_ARG, "Ec0_eV not finite");
  if (ph->holes != 0 && ph->holes != 1) return fail(QE_ERR_INVALID_ARG, "holes must be 0 or 1");
  if (ph->ionization != QE_ION_COMPLETE && ph->ionization != QE_ION_INCOMPLETE)
    return fail(QE_ERR_INVALID_ARG, "unknown ionization %d", ph->ionization);
  const bool holes = ph->holes == 1 && ph->stat != QE_STAT_LINEAR;
  const bool incomplete = ph->ionization == QE_ION_INCOMPLETE;
  if (holes && !positive(ph->m_h)) return fail(QE_ERR_INVALID_ARG, "m_h must be > 0 with holes");
  if ((holes || incomplete) && !(ph->Eg_eV >= 0.0 && std::isfinite(ph->Eg_eV)))
    return fail(QE_ERR_INVALID_ARG, "Eg_eV must be finite and >= 0");
  switch (ph->stat) {
    case QE_STAT_LINEAR:
      ch.stat = STAT_LINEAR;
      break;
    case QE_STAT_TF:
      if (!positive(ph->m_eff)) return fail(QE_ERR_INVALID_ARG, "m_eff must be > 0");
      ch.stat = STAT_TF;
      ch.Ctf = tf_prefactor(ph->m_eff);
      if (holes) ch.Ctf_h = tf_prefactor(ph->m_h);
      break;
    case QE_STAT_FD12:
    case QE_STAT_MB:
      if (!positive(ph->m_eff)) return fail(QE_ERR_INVALID_ARG, "m_eff must be > 0");
      if (!positive(ph->T_K))
        return fail(QE_ERR_INVALID_ARG, "Fermi-Dirac and Boltzmann statistics need T_K > 0");
      ch.stat = ph->stat == QE_STAT_MB ? STAT_MB : STAT_FD;
      ch.inv_kT = kQ / (kKB * ph->T_K);  // 1/eV
      ch.Nc = effective_dos(ph->m_eff, ph->T_K);
      if (holes) ch.Nv = effective_dos(ph->m_h, ph->T_K);
      break;
    default:
      return fail(QE_ERR_INVALID_ARG, "unknown statistics %d", ph->stat);
  }
  if (holes) {
    ch.holes = 1;
    ch.Eg = ph->Eg_eV;
  }
  if (incomplete) {
    if (ch.stat != STAT_FD && ch.stat != STAT_MB)
      return fail(QE_ERR_INVALID_ARG, "incomplete ionization needs Fermi-Dirac or Boltzmann statistics");
    if (!std::isfinite(ph->Ed_eV) || !std::isfinite(ph->Ea_eV))
      return fail(QE_ERR_INVALID_ARG, "Ed_eV and Ea_eV must be finite");
    if (!positive(ph->gD) || !positive(ph->gA)) return fail(QE_ERR_INVALID_ARG, "gD and gA must be > 0");
    ch.incomplete = 1;
    ch.Eg = ph->Eg_eV;
    ch.ed_kT = ph->Ed_eV * ch.inv_kT;
    ch.ea_kT = ph->Ea_eV * ch.inv_kT;
    ch.ln_gD = std::log(ph->gD);
    ch.ln_gA = std::log(ph->gA);
  }
  return QE_OK;
}

// ------------------------------------------------------------------ sizes
static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Blocks of the CG vector kernels: one 4-entry chunk per thread up to 2048
// blocks (every block re-adds all partials of the previous kernel).
int cg_blocks(long N) {
  long b = (N + (long)kVecThreads * 4 - 1) / ((long)kVecThreads * 4);
  return (int)std::max(1L, std::min(b, 2048L));
}

int vec_blocks(long N) {
  long b = (N + (long)kVecThreads * 8 - 1) / ((long)kVecThreads * 8);
  return (int)std::max(1L, std::min(b, 1024L));
}

TileMap make_tilemap(int nx, int ny, int nz, int kz) {
  TileMap tm;
  tm.gx = (nx + kTX - 1) / kTX;
  tm.gy = (ny + kTY - 1) / kTY;
  if (kz <= 0) {
    // enough blocks to cover the chip a few times, but chunks long enough that
    // the recomputed halo layer stays a small fraction
    kz = 8;
    while (kz > 4 && (long)tm.gx * tm.gy * ((nz + kz - 1) / kz) < 512) kz >>= 1;
  }
  tm.kz = std::max(1, std::min(kz, kMaxKz));
  kz = tm.kz;
  tm.gz = (nz + kz - 1) / kz;
  tm.nblocks = tm.gx * tm.gy * tm.gz;
  return tm;
}

WaveMap make_wavemap(int nx, int ny, int nz, int kz) {
  WaveMap wm;
  wm.gx = (nx + 6) / 7;
  wm.gy = (ny + 6) / 7;
  if (kz <= 0) {
    // taller chunks recompute fewer halo layers and, at 9, put a
    // 129x129x65 mesh's CG sweep in one round of 3 waves per SIMD
    // (measured fastest there and at 257x257x129); a small mesh gets
    // shorter chunks, hence more waves, down to 3 (the 65x65x33 coarse
    // start: 1100 waves; its solve with chunks of 4 / 3 / 2 / 1 made the
    // 129x129x65 solve 9.69 / 9.57 / 9.75 / 9.90 ms)
    kz = 9;
    while (kz > 3 && (long)wm.gx * wm.gy * ((nz + kz - 1) / kz) < 2048) --kz;
  }
  wm.kz = std::max(1, std::min(kz, 31));
  wm.gz = (nz + wm.kz - 1) / wm.kz;
  wm.nwaves = wm.gx * wm.gy * wm.gz;
  wm.nblocks = (wm.nwaves + 3) / 4;
  return wm;
}

static int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return v ? atoi(v) : dflt;
}
static long env_long(const char* name, long dflt) {
  const char* v = getenv(name);
  return v ? atol(v) : dflt;
}
static double env_double(const char* name, double dflt) {
  const char* v = getenv(name);
  return v ? atof(v) : dflt;
}

static const int kCountBlocks = 256;

// Chunk height of the residual with eigenstates (QE_Q_KZ overrides it).
static const int kQResidualKz = 4;
static WaveMap quantum_wavemap(const qe_problem* p) {
  return make_wavemap(p->nx, p->ny, p->nz, std::max(1, env_int("QE_Q_KZ", kQResidualKz)));
}
static const int kContactBlocks = 256;

Layout make_layout(long N, long E, long nslots, long nz_elems, long nwaves, int nblocks_tile, int vblocks,
                   int n_dir, long sheet_slots, long nwaves_q) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.F = take(N * 8);
  L.x = take(N * 8);
  L.r = take(N * 8);
  L.p = take(N * 8);
  L.y = take(N * 8);
  L.z = take(N * 8);
  L.invdiag = take(N * 8);
  L.gvec = take(N * 8);
  L.c = take(nslots * 64);     // tile-major (tile_slot)
  L.eps_t = take(nslots * 8);
  L.cflag = take(nslots);      // tile-major: element has a nonzero c_q
  L.rdz = take(2 * nz_elems * 8);  // inverse z spacings, then the spacings
  L.cbits = take(nwaves * 64 * 4);  // per J.v lane: coefficient flags over its chunk
  L.mask = take(N);
  L.fsheet = sheet_slots ? take(N * 8) : 0;   // face terms of F at sheet nodes, 0 elsewhere
  L.fdiag = sheet_slots ? take(N * 8) : 0;
  L.sheet_items = sheet_slots ? take(sheet_slots * 16) : 0;   // int4 per distinct sheet node
  L.x32 = take(N * 4);
  L.r32 = take(N * 4);
  L.p32 = take(N * 4);
  L.y32 = take(N * 4);
  L.z32 = take(N * 4);
  L.invdiag32 = take(N * 4);
  L.c32 = take(nslots * 32);
  L.eps32 = take(nslots * 4);
  long np = std::max<long>(nblocks_tile, 2L * vblocks);
  np = std::max<long>(np, (long)N / 64 + 64);   // wave-tiled J.v: one partial per block
  np = std::max<long>(np, (nwaves + 3) / 4 + kSheetBlocks);   // ... then the Robin faces' partials
  np = std::max<long>(np, (nwaves_q + 3) / 4);                 // the residual with eigenstates
  np = std::max<long>(np, (long)kCountBlocks * kMaxBoxes);
  np = std::max<long>(np, (long)kContactBlocks * std::max(1, n_dir));
  L.n_partial = np;
  L.partial = take(np * 8);
  L.partial2 = take(std::max<long>(vblocks, cg_blocks(N)) * 8);
  L.ctx = take(sizeof(PcgCtx));
  L.scal = take(64 * 8);
  L.counters = take(16 * sizeof(unsigned int));
  L.flags = take(16);
  L.sbox = take(kMaxStates * 6 * sizeof(int));   // support boxes of the predictor's states
  L.total = off;
  return L;
}

// ------------------------------------------------------------------ problem
qe_status check_problem(const qe_problem* p) {
  if (!p) return fail(QE_ERR_INVALID_ARG, "problem is NULL");
  if (p->nx < 2 || p->ny < 2 || p->nz < 2) return fail(QE_ERR_INVALID_ARG, "need nx, ny, nz >= 2");
  const long N = (long)p->nx * p->ny * p->nz;
  if (N > (1L << 31) - 1) return fail(QE_ERR_INVALID_ARG, "mesh too large");
  if (!p->x || !p->y || !p->z || !p->eps_r || !p->semi || !p->dir_id)
    return fail(QE_ERR_INVALID_ARG, "NULL array in problem");
  if (p->n_dir < 0) return fail(QE_ERR_INVALID_ARG, "n_dir < 0");
  if (p->n_dir > 0 && !p->dir_val) return fail(QE_ERR_INVALID_ARG, "dir_val is NULL");
  if ((p->donors == nullptr) != (p->acceptors == nullptr))
    return fail(QE_ERR_INVALID_ARG, "donors and acceptors must be given together");
  if (p->n_sheets < 0 || p->n_sheets > QE_MAX_SHEETS)
    return fail(QE_ERR_INVALID_ARG, "n_sheets outside [0, %d]", QE_MAX_SHEETS);
  if (p->n_sheets > 0 && !p->sheets) return fail(QE_ERR_INVALID_ARG, "sheets is NULL");
  for (int i = 0; i < p->n_sheets; ++i) {
    const qe_sheet& h = p->sheets[i];
    const int n[3] = {p->nx, p->ny, p->nz};
    if (h.axis < 0 || h.axis > 2) return fail(QE_ERR_INVALID_ARG, "sheet %d: axis must be 0, 1 or 2", i);
    const int na = n[h.axis == 0 ? 1 : 0], nb = n[h.axis == 2 ? 1 : 2];
    if (h.plane < 0 || h.plane >= n[h.axis]) return fail(QE_ERR_INVALID_ARG, "sheet %d: plane out of range", i);
    if (!(0 <= h.a0 && h.a0 < h.a1 && h.a1 <= na - 1 && 0 <= h.b0 && h.b0 < h.b1 && h.b1 <= nb - 1))
      return fail(QE_ERR_INVALID_ARG, "sheet %d: face range out of range", i);
    if (!(h.robin_d >= 0.0 && std::isfinite(h.robin_d)) || !std::isfinite(h.phi0))
      return fail(QE_ERR_INVALID_ARG, "sheet %d: robin_d must be finite and >= 0, phi0 finite", i);
    if (h.robin_d > 0.0 && !(h.robin_eps > 0.0 && std::isfinite(h.robin_eps)))
      return fail(QE_ERR_INVALID_ARG, "sheet %d: robin_eps must be > 0", i);
  }
  return QE_OK;
}

// Kernel view of the predictor-corrector states, checked on the host.
qe_status make_quantum(const qe_problem* p, const Charge& ch, Quantum& Q) {
  std::memset(&Q, 0, sizeof(Q));
  const qe_quantum* q = p->quantum;
  if (!q) return QE_OK;
  if (q->n_states < 1 || q->n_states > QE_MAX_STATES)
    return fail(QE_ERR_INVALID_ARG, "quantum: n_states outside [1, %d]", QE_MAX_STATES);
  if (q->confinement != 3 && q->confinement != 1) return fail(QE_ERR_INVALID_ARG, "quantum: confinement must be 3 or 1");
  if (!q->psi2 || !q->phi_k || !q->E_i) return fail(QE_ERR_INVALID_ARG, "quantum: NULL array");
  if (!positive(ch.T_K)) return fail(QE_ERR_INVALID_ARG, "quantum: the predictor-corrector density needs T_K > 0");
  if (q->confinement == 1 && !positive(q->m_t)) return fail(QE_ERR_INVALID_ARG, "quantum: m_t must be > 0");
  for (int i = 0; i < q->n_states; ++i)
    if (!std::isfinite(q->E_i[i])) return fail(QE_ERR_INVALID_ARG, "quantum: E_i[%d] not finite", i);
  Q.n = q->n_states;
  Q.conf = q->confinement;
  Q.N = (long)p->nx * p->ny * p->nz;
  // the kernels address one state's |psi|^2 with 32-bit byte offsets
  if (Q.N * 8 > 0x7fffffffL) return fail(QE_ERR_INVALID_ARG, "quantum: more than 2^28 - 1 nodes");
  Q.psi2 = q->psi2;
  Q.phik = q->phi_k;
  Q.region = q->region;
  const double kT_J = kKB * ch.T_K;
  Q.inv_kT = kQ / kT_J;
  // 3D: two spins x two valleys; 1D: 2 m_t kT / (pi hbar^2) in nm^-2
  Q.pref = q->confinement == 3 ? 4.0 : 2.0 * q->m_t * kM0 * kT_J / (kPi * kHbar * kHbar) * 1e-18;
  for (int i = 0; i < q->n_states; ++i) Q.E[i] = q->E_i[i];
  // e^(E_i/kT) for the one-exponential form of the 3D occupation
  Q.fast = q->confinement == 3;
  for (int i = 0; i < q->n_states; ++i) {
    const double e = q->E_i[i] * Q.inv_kT;
    if (!(std::fabs(e) <= kPcExpMax)) Q.fast = 0;
    Q.B[i] = Q.fast ? std::exp(e) : 0.0;
  }
  return QE_OK;
}

// Nodes of all sheets counted with multiplicity (an upper bound of the
// distinct ones).
long sheet_slots(const qe_problem* p) {
  long n = 0;
  for (int i = 0; i < p->n_sheets; ++i)
    n += (long)(p->sheets[i].a1 - p->sheets[i].a0 + 1) * (p->sheets[i].b1 - p->sheets[i].b0 + 1);
  return n;
}

// Kernel view of a problem's sheets (checked by check_problem) and the list
// of their distinct nodes: index bookkeeping only, from the sheets' ranges.
SheetSet make_sheets(const qe_problem* p, std::vector<int4>& items) {
  SheetSet S;
  std::memset(&S, 0, sizeof(S));
  S.n = p->n_sheets;
  const long nxy = (long)p->nx * p->ny;
  const double* c[3] = {p->x, p->y, p->z};
  const long stride[3] = {1, p->nx, nxy};
  for (int i = 0; i < S.n; ++i) {
    const qe_sheet& h = p->sheets[i];
    SheetDev& d = S.s[i];
    const int ia = h.axis == 0 ? 1 : 0, ib = h.axis == 2 ? 1 : 2;   // in-plane axes
    d.axis = h.axis;
    d.plane = h.plane;
    d.a0 = h.a0;
    d.a1 = h.a1;
    d.b0 = h.b0;
    d.b1 = h.b1;
    d.base = h.plane * stride[h.axis];
    d.sa = stride[ia];
    d.sb = stride[ib];
    d.ca = c[ia];
    d.cb = c[ib];
    d.sigma = h.sigma;
    d.alpha = h.robin_d > 0.0 ? h.robin_eps / h.robin_d : 0.0;
    d.phi0 = h.phi0;
    S.any_robin |= d.alpha != 0.0;
  }
  // a node belongs to sheet t when it lies in t's plane inside t's node range
  auto contains = [&](int t, int ijk[3]) {
    const qe_sheet& h = p->sheets[t];
    const int ia = h.axis == 0 ? 1 : 0, ib = h.axis == 2 ? 1 : 2;
    return ijk[h.axis] == h.plane && ijk[ia] >= h.a0 && ijk[ia] <= h.a1 && ijk[ib] >= h.b0 && ijk[ib] <= h.b1;
  };
  items.clear();
  for (int i = 0; i < S.n; ++i) {
    const qe_sheet& h = p->sheets[i];
    const int ia = h.axis == 0 ? 1 : 0, ib = h.axis == 2 ? 1 : 2;
    for (int b = h.b0; b <= h.b1; ++b)
      for (int a = h.a0; a <= h.a1; ++a) {
        int ijk[3];
        ijk[h.axis] = h.plane;
        ijk[ia] = a;
        ijk[ib] = b;
        bool first = true, shared = false;
        for (int t = 0; t < S.n && first; ++t)
          if (t != i && contains(t, ijk)) {
            if (t < i) first = false;
            else shared = true;
          }
        if (!first) continue;
        const long n = ijk[0] + p->nx * ((long)ijk[1] + (long)p->ny * ijk[2]);
        items.push_back(make_int4((int)n, i | (shared ? 256 : 0), a, b));
      }
  }
  S.n_items = (int)items.size();
  return S;
}

qe_status check_options(const qe_options* o) {
  if (!o) return fail(QE_ERR_INVALID_ARG, "options are NULL");
  if (!(o->newton_atol > 0) || !std::isfinite(o->newton_atol)) return fail(QE_ERR_INVALID_ARG, "newton_atol must be > 0");
  if (o->newton_maxit < 0) return fail(QE_ERR_INVALID_ARG, "newton_maxit < 0");
  if (o->ls_max_halvings < 0 || o->ls_max_halvings > 60) return fail(QE_ERR_INVALID_ARG, "ls_max_halvings out of range");
  if (!(o->krylov_rtol_max > 0 && o->krylov_rtol_max < 1)) return fail(QE_ERR_INVALID_ARG, "krylov_rtol_max not in (0,1)");
  if (o->krylov_maxit < 1) return fail(QE_ERR_INVALID_ARG, "krylov_maxit < 1");
  if (o->precision != QE_PREC_FP64 && o->precision != QE_PREC_MIXED) return fail(QE_ERR_INVALID_ARG, "bad precision");
  if (o->init_guess < 0 || o->init_guess > 2) return fail(QE_ERR_INVALID_ARG, "bad init_guess");
  if (o->check_every < 0) return fail(QE_ERR_INVALID_ARG, "check_every < 0");
  if (o->precond < QE_PC_AUTO || o->precond > QE_PC_MULTIGRID) return fail(QE_ERR_INVALID_ARG, "bad precond");
  return QE_OK;
}

// Host memory for scalar read-backs (one per thread): pinned, with a
// host-coherent word the CG's stopping kernel posts to; or, for the entry
// point that allocates nothing, the thread's own static storage (no posted
// word: that CG loop is polled by stream synchronisations).
struct HostMirror {
  PcgCtx* ctx = nullptr;
  double* scal = nullptr;
  int* flags = nullptr;
  volatile CgProgress* prog = nullptr;   // host-coherent: written by the device while it runs
  CgProgress* prog_dev = nullptr;        // the same memory as the device addresses it
  bool ok = false;
};

static HostMirror make_pinned_mirror() {
  HostMirror m;
  void* a = nullptr;
  void* b = nullptr;
  if (hipHostMalloc(&a, 4096, hipHostMallocDefault) != hipSuccess) return m;
  m.ctx = reinterpret_cast<PcgCtx*>(a);
  m.scal = reinterpret_cast<double*>(reinterpret_cast<char*>(a) + 1024);
  m.flags = reinterpret_cast<int*>(reinterpret_cast<char*>(a) + 3072);
  if (hipHostMalloc(&b, 256, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) return m;
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, b, 0) != hipSuccess) return m;
  m.prog = reinterpret_cast<volatile CgProgress*>(b);
  m.prog_dev = reinterpret_cast<CgProgress*>(d);
  m.ok = true;
  return m;
  // never freed: thread-exit destructors may run after the HIP runtime is gone
}

HostMirror& mirror() {
  static thread_local HostMirror m = make_pinned_mirror();
  return m;
}

static HostMirror& plain_mirror() {
  struct Store {
    PcgCtx ctx;
    double scal[64];
    int flags[4];
  };
  static thread_local Store st;
  static thread_local HostMirror m{&st.ctx, st.scal, st.flags, nullptr, nullptr, true};
  return m;
}

qe_status Context::init(const qe_problem* p, const Charge& ch, void* ws_, size_t ws_bytes, void* stream_, int kz,
                        bool no_alloc_, int wave_kz) {
  no_alloc = no_alloc_;
  QE_TRY(check_problem(p));
  if (ch.incomplete && !p->donors)
    return fail(QE_ERR_INVALID_ARG, "incomplete ionization needs donors and acceptors");
  QE_TRY(make_quantum(p, ch, quantum));
  prob = *p;
  s = (hipStream_t)stream_;
  N = (long)p->nx * p->ny * p->nz;
  E = (long)(p->nx - 1) * (p->ny - 1) * (p->nz - 1);
  g.nx = p->nx;
  g.ny = p->ny;
  g.nz = p->nz;
  g.x = p->x;
  g.y = p->y;
  g.z = p->z;
  tm = make_tilemap(p->nx, p->ny, p->nz, kz);
  wm = make_wavemap(p->nx, p->ny, p->nz, wave_kz > 0 ? wave_kz : env_int("QE_JV_KZ", 0));
  // with eigenstates the waves over the dot loop over every state on each of
  // their layers; chunks of kQResidualKz layers shorten that critical path
  wmq = quantum.n > 0 ? quantum_wavemap(p) : wm;
  vblocks = vec_blocks(N);
  nslots = tile_slots(p->nx, p->ny, p->nz);
  lay = make_layout(N, E, nslots, p->nz - 1, wm.nwaves, tm.nblocks, vblocks, p->n_dir, sheet_slots(p),
                    quantum.n > 0 ? wmq.nwaves : 0);
  if (!ws_) return fail(QE_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws_) & 255) return fail(QE_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < lay.total)
    return fail(QE_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, lay.total);
  ws = reinterpret_cast<char*>(ws_);
  hm = no_alloc ? &plain_mirror() : &mirror();
  if (!hm->ok) return fail(QE_ERR_HIP, "pinned host buffer allocation failed");
  g.rdz = f64(lay.rdz);
  g.hz = g.rdz + (p->nz - 1);
  launch_stage_rdz(s, p->nz, p->z, f64(lay.rdz));
  std::vector<int4> items;
  sheets = make_sheets(p, items);
  if (sheets.n > 0) {
    QE_HIP(hipMemsetAsync(ws + lay.fsheet, 0, N * sizeof(double), s));
    QE_HIP(hipMemsetAsync(ws + lay.fdiag, 0, N * sizeof(double), s));
    QE_HIP(hipMemcpyAsync(ws + lay.sheet_items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    QE_HIP(hipStreamSynchronize(s));   // `items` is a host temporary
  }
  if (quantum.n > 0) {
    quantum.sbox = reinterpret_cast<const int*>(ws + lay.sbox);
    launch_state_boxes(s, vblocks, g, quantum, reinterpret_cast<int*>(ws + lay.sbox));
  }
  // reset device scalars and reduction counters
  QE_HIP(hipMemsetAsync(ws + lay.ctx, 0, sizeof(PcgCtx), s));
  QE_HIP(hipMemsetAsync(ws + lay.counters, 0, 16 * sizeof(unsigned int), s));
  QE_HIP(hipMemsetAsync(ws + lay.flags, 0, 16, s));
  return QE_OK;
}

// Doping arrays of the problem (the species only when both are given).
Doping Context::doping() const {
  return Doping{prob.net_doping, prob.donors, prob.acceptors};
}

// Device-side checks of the coordinates, Dirichlet ids and values, eps_r,
// doping, sheets, states and (optionally) phi.
qe_status Context::validate(const double* phi) {
  int* dflags = reinterpret_cast<int*>(ws + lay.flags);
  launch_validate_mesh(s, prob.nx, prob.ny, prob.nz, prob.x, prob.y, prob.z, prob.n_dir, prob.dir_val, dflags);
  launch_validate(s, vblocks, N, E, prob.n_dir, prob.eps_r, doping(), prob.dir_id, phi, dflags);
  if (sheets.n > 0) launch_validate_sheets(s, sheets, dflags);
  if (quantum.n > 0) launch_validate_quantum(s, vblocks, quantum, dflags);
  QE_HIP(hipGetLastError());
  QE_HIP(hipMemcpyAsync(hm->flags, dflags, sizeof(int), hipMemcpyDeviceToHost, s));
  QE_HIP(hipStreamSynchronize(s));
  const int f = *hm->flags;
  for (int a = 0; a < 3; ++a)
    if (f & (128 << a)) return fail(QE_ERR_INVALID_ARG, "coordinates %c not finite or not strictly increasing", "xyz"[a]);
  if (f & 1024) return fail(QE_ERR_NONFINITE, "dir_val not finite");
  if (f & 1) return fail(QE_ERR_INVALID_ARG, "eps_r must be finite and > 0");
  if (f & 2) return fail(QE_ERR_NONFINITE, "net_doping not finite or donors / acceptors not finite and >= 0");
  if (f & 4) return fail(QE_ERR_INVALID_ARG, "dir_id outside [-1, n_dir)");
  if (f & 8) return fail(QE_ERR_NONFINITE, "phi not finite");
  if (f & 16) return fail(QE_ERR_NONFINITE, "sheet sigma not finite");
  if (f & 32) return fail(QE_ERR_NONFINITE, "quantum psi2 not finite and >= 0");
  if (f & 64) return fail(QE_ERR_NONFINITE, "quantum phi_k not finite");
  return QE_OK;
}

qe_status Context::stage(double* phi, int apply, int zero_free) {
  launch_stage(s, vblocks, N, prob.dir_id, prob.dir_val, u8(lay.mask), phi, apply, zero_free);
  launch_stage_eps64(s, vblocks, g, prob.eps_r, f64(lay.eps_t), nslots);
  QE_HIP(hipGetLastError());
  return QE_OK;
}

qe_status Context::residual(const Charge& ch, const double* phi, const double* d64, const float* d32, double lam,
                            bool mixed, double* diag_out, double* norm2_host) {
  const bool sh = sheets.n > 0;
  if (sh) launch_sheet_residual(s, sheets, sheet_items(), ch.kappa, u8(lay.mask), phi, d64, d32, lam, f64(lay.fsheet), f64(lay.fdiag));
  launch_residual_wave(s, g, wm, wmq, ch, prob.eps_r, prob.semi, doping(), u8(lay.mask), phi, d64, d32, lam,
                       sh ? f64(lay.fsheet) : nullptr, sh ? f64(lay.fdiag) : nullptr, f64(lay.F), f64(lay.invdiag), diag_out, f64(lay.c), mixed ? f32(lay.c32) : nullptr,
                       u8(lay.cflag), u32(lay.cbits), mixed ? f32(lay.invdiag32) : nullptr, f64(lay.partial),
                       f64(lay.scal), quantum);
  QE_HIP(hipGetLastError());
  if (norm2_host) {
    QE_HIP(hipMemcpyAsync(hm->scal, ws + lay.scal, sizeof(double), hipMemcpyDeviceToHost, s));
    QE_HIP(hipStreamSynchronize(s));
    *norm2_host = hm->scal[0];
  }
  return QE_OK;
}

// Jacobi-PCG on J x = sign*b (free rows).  Returns the CG status through
// *pcg_status and the iteration count through *iters.
qe_status Context::pcg(bool mixed, const double* b, double sign, double rtol, int maxit, int check_every,
                       int* pcg_status, int* iters, const MgRun* mg) {
  PcgCtx* dctx = reinterpret_cast<PcgCtx*>(ws + lay.ctx);
  if (no_alloc) return pcg_polled(mixed, b, sign, rtol, maxit, pcg_status, iters);
  if (mg && mg->nlev < 2) mg = nullptr;
  HostMirror& hm = *this->hm;
  volatile CgProgress* hp = hm.prog;
  hp->word = 0;  // the last decision of an earlier solve has been read: no write is pending
  const int cgb = cg_blocks(N);
  // with multigrid the CG kernels' z = D^-1 r becomes the V-cycle's first
  // smoothing step z = S r; the V-cycle then turns z into B r and replaces
  // the r^T z partials
  const double* dinv = mg ? mg->lv[0].S : f64(lay.invdiag);
  const float* dinv32 = mg ? mg->lv[0].S32 : f32(lay.invdiag32);
  if (mixed)
    launch_pcg_start32(s, cgb, N, sign, b, u8(lay.mask), dinv32, f32(lay.x32), f32(lay.r32), f32(lay.z32), dctx,
                       f64(lay.partial2), rtol, maxit);
  else
    launch_pcg_start64(s, cgb, N, sign, b, u8(lay.mask), dinv, f64(lay.x), f64(lay.r), f64(lay.z), dctx,
                       f64(lay.partial2), rtol, maxit);
  if (mg) {
    launch_mg_vcycle(s, mg->lv, mg->nlev, mg->sweeps, mg->add_top, cgb, f64(lay.partial2), dctx, mixed);
    launch_mg_start_fin(s, dctx, f64(lay.partial2), cgb);
  }
  QE_HIP(hipGetLastError());
  auto queue_iter = [&](int k) {
    if (mixed)
      launch_pcg_iter32(s, g, wm, cgb, N, k & 1, f32(lay.eps32), u32(lay.cbits), f32(lay.c32), dinv32, f32(lay.x32),
                        f32(lay.r32), f32(lay.z32), f32(lay.p32), f32(lay.y32), dctx, hm.prog_dev, f64(lay.partial),
                        f64(lay.partial2), sheets.any_robin ? &sheets : nullptr, sheet_items(), u8(lay.mask));
    else
      launch_pcg_iter64(s, g, wm, cgb, N, k & 1, f64(lay.eps_t), u32(lay.cbits), f64(lay.c), dinv, f64(lay.x),
                        f64(lay.r), f64(lay.z), f64(lay.p), f64(lay.y), dctx, hm.prog_dev, f64(lay.partial),
                        f64(lay.partial2), sheets.any_robin ? &sheets : nullptr, sheet_items(), u8(lay.mask));
    if (mg) launch_mg_vcycle(s, mg->lv, mg->nlev, mg->sweeps, mg->add_top, cgb, f64(lay.partial2), dctx, mixed);
  };
  // The host keeps `ahead` iterations queued beyond those it knows have
  // finished (an event is recorded after every kEv-th iteration), so the
  // device never waits for the host.  The first kernel posts to host-coherent
  // memory only when it stops the solve (convergence, non-finite values, the
  // iteration limit in iteration maxit; the second kernel on breakdown), once
  // per solve; the queued iterations after that return at once.
#ifndef QE_CG_EVENT_EVERY
#define QE_CG_EVENT_EVERY 8
#endif
  constexpr int kRing = kEventRing;
  // a multigrid iteration (~25 launches) outlasts the host's reaction to an
  // event several times over: an event after each, two iterations ahead
  // (three measured no faster)
  const int kEv = mg ? 1 : QE_CG_EVENT_EVERY;
  hipEvent_t* ring = events;
  for (int e = 0; e < kRing; ++e)
    if (!ring[e]) QE_HIP(hipEventCreateWithFlags(&ring[e], hipEventDisableTiming));
  // kEv + 1 by default: one iteration (~30 us at 129x129x65) covers the
  // host's reaction to an event, and fewer launches return at once after
  // the stop (measured: 0.5 % faster solves than kEv + 4; events every 4 or
  // 2 iterations cost more than they save)
  const int ahead =
      mg ? std::min(std::max(1, env_int("QE_MG_AHEAD", 2)), kRing - 1) : std::min(std::max(check_every > 0 ? check_every : kEv + 1, kEv + 1), kEv * (kRing - 1));
  int queued = 0, finished = 0, head = 0, tail = 0;  // events [head, tail) pending, in ring order
  // FP64: the last x += alpha p, queued after every launch of the loop
  auto finish = [&]() -> qe_status {
    if (!mixed) {
      launch_cg_finish_x64(s, vblocks, N, dctx, f64(lay.p), f64(lay.x));
      QE_HIP(hipGetLastError());
    }
    return QE_OK;
  };
  for (;;) {
    while (queued <= maxit && queued < finished + ahead) {
      queue_iter(queued++);
      if (queued % kEv == 0 || queued > maxit) {
        QE_HIP(hipEventRecord(ring[tail % kRing], s));
        ++tail;
      }
    }
    QE_HIP(hipGetLastError());
    const int wd = hp->word;
    if (wd & 1) {
      *pcg_status = (wd >> 1) & 7;
      *iters = (wd >> 4) - 1;
      return finish();
    }
    if (head < tail) {
      const hipError_t e = hipEventQuery(ring[head % kRing]);
      if (e == hipSuccess) {
        ++head;
        finished = std::min(queued, head * kEv);
      } else if (e != hipErrorNotReady) {
        return fail(QE_ERR_HIP, "CG stream failed: %s", hipGetErrorString(e));
      }
      continue;
    }
    // everything queued has finished without a posted stop: read the
    // scalars (a stop may also have been posted after the check above)
    PcgCtx& h = *hm.ctx;
    QE_HIP(hipMemcpyAsync(&h, dctx, sizeof(PcgCtx), hipMemcpyDeviceToHost, s));
    QE_HIP(hipStreamSynchronize(s));
    if (h.done || queued > maxit) {
      *pcg_status = h.done ? h.status : PCG_MAXIT;
      *iters = h.iters;
      return finish();
    }
  }
}

// The same CG loop without events or a posted stop: chunks of iterations are
// queued, the stream synchronised and the scalars read back after each.  For
// the entry point that allocates nothing (a queued launch after the stop
// returns at once, as in pcg).
qe_status Context::pcg_polled(bool mixed, const double* b, double sign, double rtol, int maxit, int* pcg_status,
                              int* iters) {
  PcgCtx* dctx = reinterpret_cast<PcgCtx*>(ws + lay.ctx);
  const int cgb = cg_blocks(N);
  if (mixed)
    launch_pcg_start32(s, cgb, N, sign, b, u8(lay.mask), f32(lay.invdiag32), f32(lay.x32), f32(lay.r32),
                       f32(lay.z32), dctx, f64(lay.partial2), rtol, maxit);
  else
    launch_pcg_start64(s, cgb, N, sign, b, u8(lay.mask), f64(lay.invdiag), f64(lay.x), f64(lay.r), f64(lay.z),
                       dctx, f64(lay.partial2), rtol, maxit);
  QE_HIP(hipGetLastError());
  constexpr int kChunk = 16;
  int queued = 0;
  for (;;) {
    for (int c = 0; c < kChunk && queued <= maxit; ++c, ++queued) {
      if (mixed)
        launch_pcg_iter32(s, g, wm, cgb, N, queued & 1, f32(lay.eps32), u32(lay.cbits), f32(lay.c32),
                          f32(lay.invdiag32), f32(lay.x32), f32(lay.r32), f32(lay.z32), f32(lay.p32), f32(lay.y32),
                          dctx, nullptr, f64(lay.partial), f64(lay.partial2), sheets.any_robin ? &sheets : nullptr,
                          sheet_items(), u8(lay.mask));
      else
        launch_pcg_iter64(s, g, wm, cgb, N, queued & 1, f64(lay.eps_t), u32(lay.cbits), f64(lay.c), f64(lay.invdiag),
                          f64(lay.x), f64(lay.r), f64(lay.z), f64(lay.p), f64(lay.y), dctx, nullptr, f64(lay.partial),
                          f64(lay.partial2), sheets.any_robin ? &sheets : nullptr, sheet_items(), u8(lay.mask));
    }
    QE_HIP(hipGetLastError());
    PcgCtx& h = *hm->ctx;
    QE_HIP(hipMemcpyAsync(&h, dctx, sizeof(PcgCtx), hipMemcpyDeviceToHost, s));
    QE_HIP(hipStreamSynchronize(s));
    if (h.done || queued > maxit) {
      *pcg_status = h.done ? h.status : PCG_MAXIT;
      *iters = h.iters;
      if (!mixed) {   // the last x += alpha p, as in pcg (none after a breakdown)
        launch_cg_finish_x64(s, vblocks, N, dctx, f64(lay.p), f64(lay.x));
        QE_HIP(hipGetLastError());
      }
      return QE_OK;
    }
  }
}

}  // namespace qe

using namespace qe;

static size_t fine_layout_bytes(const qe_problem* p);
static size_t seq_extra_bytes(const qe_problem* p, int levels);
static size_t extra_bytes(const qe_problem* p, int seq_levels);
static int seq_levels_wanted();

// ====================================================================== C ABI
// ------------------------------------------------------------------ contacts
// eta with F_1/2(eta) ~= u: the Nilsson inverse of Eq. FDintInverse (the
// first term tends to -1/2 at u = 1).
static double nilsson_eta(double u) {
  const double nu = std::cbrt(std::pow(0.75 * std::sqrt(kPi) * u, 2.0));
  const double lead = std::fabs(u - 1.0) < 1e-8 ? -0.5 : std::log(u) / (1.0 - u * u);
  const double t = 0.24 + 1.08 * nu;
  return lead + nu / (1.0 + 1.0 / (t * t));
}

// ln y of the neutral contact with incomplete ionization (Eqs. Yval4MBIncompIon
// and ApproxLogTerms): y = e^((E_F - E_D)/kT) solves g y^2 + y = K with
// K = (N / N_band) e^(E_level/kT) (the paper's factors 8 and 16 are 4g for
// g_D = 2 and g_A = 4).  The root is taken in the rationalised form
// 2K / (1 + sqrt(1 + 4gK)); once 4gK passes 1e300 only the leading term
// ln y = (ln(K/g))/2 is kept.
static double incomplete_ln_y(double N, double Nband, double level_kT, double g) {
  const double lnK = std::log(N / Nband) + level_kT;
  const double ln4gK = std::log(4.0 * g) + lnK;
  if (ln4gK < std::log(1e300)) {
    const double K = std::exp(lnK);
    return std::log(2.0 * K / (1.0 + std::sqrt(1.0 + 4.0 * g * K)));
  }
  return 0.5 * (lnK - std::log(g));
}

extern "C" {

void qe_default_options(qe_options* o) {
  if (!o) return;
  o->newton_atol = 1e-8;
  o->newton_maxit = 100;
  o->ls_max_halvings = 30;
  o->krylov_rtol_max = 0.3;
  o->krylov_maxit = 20000;
  o->precision = QE_PREC_FP64;
  o->init_guess = 2;
  o->check_every = 0;
  o->precond = QE_PC_AUTO;
}

size_t qe_workspace_bytes(const qe_problem* p, const qe_options* o) {
  (void)o;
  if (check_problem(p) != QE_OK) return 0;
  return fine_layout_bytes(p) + extra_bytes(p, seq_levels_wanted());
}

}  // extern "C"

// The largest layout Context::init takes for this problem with this wave
// chunk height (0: the library's choice), checked there.
static size_t layout_bytes(const qe_problem* p, int wave_kz) {
  const long N = (long)p->nx * p->ny * p->nz;
  const long E = (long)(p->nx - 1) * (p->ny - 1) * (p->nz - 1);
  // the tile map with the smallest chunk height has the most blocks
  TileMap tm = make_tilemap(p->nx, p->ny, p->nz, 1);
  const WaveMap wm = make_wavemap(p->nx, p->ny, p->nz, wave_kz > 0 ? wave_kz : env_int("QE_JV_KZ", 0));
  const long nwq = p->quantum ? quantum_wavemap(p).nwaves : 0;
  return make_layout(N, E, tile_slots(p->nx, p->ny, p->nz), p->nz - 1, wm.nwaves, tm.nblocks, vec_blocks(N),
                     p->n_dir, sheet_slots(p), nwq).total;
}

static size_t fine_layout_bytes(const qe_problem* p) { return layout_bytes(p, 0); }

// ---------------------------------------------------------------------------
// Coarse-mesh sequence (init_guess = 2).  The problem coarsened by taking
// every other node along each axis (the last node kept) is solved first, to
// the relative residual seq_rtol (from its linear guess, or a further level
// when QE_SEQ_LEVELS asks for more than one), and its potential, interpolated
// trilinearly, starts Newton here.  Only for meshes of at least
// kSeqMinNodes nodes (measured faster from 269k nodes up; smaller solves are
// launch-bound) without sheets or eigenstates; otherwise, or when the
// workspace has no room for the coarse levels, the linear guess.  The coarse arrays and the coarse
// solve's workspace follow the fine layout in the caller's workspace.
static const long kSeqMinNodes = 250000;
static const int kSeqLevels = 1;

// The coarse solve need not be much more accurate than the coarse mesh's
// own error against the fine one: 1e-3 for a coarse mesh of 139,425 nodes
// (the 129x129x65 problem's), scaled by (139425 / N_c)^(1/3), the scaling
// that fits the optima measured on the two stacks below.
// Measured at 129x129x65: 1e-2 / 3e-3 / 1e-3 / 1e-4 gave 20.1 / 19.2 / 17.9 /
// 18.7 ms (with the V-cycle: 3e-3 / 1e-3 / 3e-4 gave 10.6 / 9.4 / 10.5 ms);
// at 257x257x129 (coarse 1.08M nodes), with the V-cycle, 1e-3 / 5e-4 / 2.6e-4
// / 1e-4 gave 46.2 / 43.1 / 46.0 / 50.2 ms (the scaling was (.)^(2/3), giving
// 2.6e-4, before the V-cycle took the fine Newton's last steps).
static double seq_rtol(long n_coarse) {
  const double r = 1e-3 * std::pow(139425.0 / (double)n_coarse, 1.0 / 3.0);
  return env_double("QE_SEQ_RTOL", std::min(1e-2, std::max(1e-5, r)));
}

struct SeqPlan {
  qe_problem pc;       // the coarse problem (device pointers into the plan's region)
  size_t o_phi, o_ws, total;
};

// The problem coarsened by every other node along each axis (the last node
// kept): its arrays are carved from base + off (off advances, 256-aligned);
// false if a dimension would not shrink or would fall below 3 nodes.
static bool carve_coarse(const qe_problem* p, char* base, size_t& off, qe_problem& c) {
  c = *p;
  c.nx = p->nx / 2 + 1;
  c.ny = p->ny / 2 + 1;
  c.nz = p->nz / 2 + 1;
  if (c.nx < 3 || c.ny < 3 || c.nz < 3 || c.nx >= p->nx || c.ny >= p->ny || c.nz >= p->nz) return false;
  const long Nc = (long)c.nx * c.ny * c.nz, Ec = (long)(c.nx - 1) * (c.ny - 1) * (c.nz - 1);
  auto take = [&](size_t b) {
    const size_t o = off;
    off = align256(off + b);
    return o;
  };
  c.x = reinterpret_cast<const double*>(base + take(c.nx * 8));
  c.y = reinterpret_cast<const double*>(base + take(c.ny * 8));
  c.z = reinterpret_cast<const double*>(base + take(c.nz * 8));
  c.eps_r = reinterpret_cast<const double*>(base + take(Ec * 8));
  c.semi = reinterpret_cast<const uint8_t*>(base + take(Ec));
  c.net_doping = p->net_doping ? reinterpret_cast<const double*>(base + take(Ec * 8)) : nullptr;
  c.donors = p->donors ? reinterpret_cast<const double*>(base + take(Ec * 8)) : nullptr;
  c.acceptors = p->acceptors ? reinterpret_cast<const double*>(base + take(Ec * 8)) : nullptr;
  c.dir_id = reinterpret_cast<const int32_t*>(base + take(Nc * 4));
  c.n_sheets = 0;
  c.sheets = nullptr;
  c.quantum = nullptr;
  return check_problem(&c) == QE_OK;
}

static bool seq_plan(const qe_problem* p, char* base, SeqPlan& sp, int levels) {
  if (levels < 1 || p->n_sheets > 0 || p->quantum) return false;
  const long N = (long)p->nx * p->ny * p->nz;
  if (N < env_long("QE_SEQ_MIN_NODES", kSeqMinNodes)) return false;
  qe_problem& c = sp.pc;
  size_t off = 0;
  if (!carve_coarse(p, base, off, c)) return false;
  const long Nc = (long)c.nx * c.ny * c.nz;
  sp.o_phi = off;
  off = align256(off + Nc * 8);
  sp.o_ws = off;
  // the coarse solve's workspace: its own layout and room for its own
  // sequence or multigrid levels
  off += fine_layout_bytes(&c) + extra_bytes(&c, levels - 1);
  sp.total = off;
  return true;
}

static int seq_levels_wanted() { return env_int("QE_SEQ_LEVELS", kSeqLevels); }

static size_t seq_extra_bytes(const qe_problem* p, int levels) {
  SeqPlan sp;
  // sizes only: a dummy base that no pointer derived from it is read through
  return seq_plan(p, reinterpret_cast<char*>(size_t(1) << 20), sp, levels) ? sp.total : 0;
}

// ---------------------------------------------------------------------------
// Multigrid preconditioner of the CG (qe_precond; kernels in
// qe_mg.hip).  With sheets the fine level is the problem's own Jacobian
// without the Robin face term (the V-cycle stays positive definite, it only
// approximates J less closely) and the coarse levels carry no sheets; with
// eigenstates every coarse level has them too, injected like the potential
// (|psi|^2 and phi^(k) at its nodes, each coarse element the region flag
// of its first fine element).  The levels are the meshes of the coarse-mesh sequence, down
// to the last one with at least kMgMinCoarse nodes; each coarse level has
// its problem arrays, its potential, its smoother weights and a Context
// layout (whose r, x and y hold the V-cycle's b, x and J x), after the fine
// layout in the caller's workspace (the region the sequence's coarse solve
// used before Newton started).  Level 0 adds its smoother weights and a J x
// vector there; its b and x are the CG's r and z.
static const long kMgMinNodes = 250000;
static const long kMgMinCoarse = 2000;
static const int kMgMaxLevels = 6;
// AUTO: multigrid for CG tolerances at or below this one.  At the
// 129x129x65 stack a V-cycle costs ~7 Jacobi iterations (its small levels
// are launch- and latency-bound) and saves ~10x the iterations on the last
// Newton steps; measured there, 1e-2 / 3e-2 / 1e-1 / every step gave
// 13.4 / 13.4 / 13.5 / 15.0 ms per solve against 17.8 ms with Jacobi only.
static const double kMgEta = 3e-2;
// Smoothing steps on the coarsest mesh (at 129x129x65 with the weight below,
// 2 / 4 / 6 gave 37 / 30 / 28 adjoint iterations in 7.6 / 6.9 / 6.9 ms and
// solves of 12.0 / 11.0 / 11.3 ms; a fifth level, down to 9x9x5, measured
// slower).
static const int kMgSweeps = 4;
// Chunk height of the coarse levels' wave tiles: their meshes are small, so
// short chunks give the J.v and the residual more waves (latency, not
// bandwidth, bounds them there; 1 / 2 / 4 measured 8.8 / 9.0 / 9.5 ms for
// the adjoint above).
static const int kMgCoarseKz = 1;
// Coarse levels of this many nodes and more keep the default chunks (a
// 129x129x65 level under 257x257x129: its J.v took 34.8 us with chunks of
// 1, against ~19 us with the default).
static const long kMgCoarseKzMaxNodes = 500000;
static int mg_coarse_kz(long nodes) {
  if (nodes >= env_long("QE_MG_KZ_MAX_NODES", kMgCoarseKzMaxNodes)) return 0;
  return std::max(1, env_int("QE_MG_KZ", kMgCoarseKz));
}
// Smoother weight: S = omega / (row's absolute-sum bound).  Since that bound
// puts every eigenvalue of S J / omega in (0, 1], any omega < 2 keeps
// 2 S^-1 - J positive definite, hence the V-cycle; for the stiffness rows the
// bound is about twice the diagonal, so omega = 1 would damp like Jacobi
// with 0.5.  Measured at 129x129x65: omega 1.0 / 1.2 / 1.4 / 1.6 / 1.8 / 1.9
// gave solves of 13.3 / 12.9 / 11.8 / 12.0 / 11.0 / 10.9 ms and adjoints of
// 8.6 / 8.2 / 7.7 / 7.3 / 6.9 / 6.9 ms; at 257x257x129 1.8 against 1.0 took
// 88 against 104 ms.
static const double kMgOmega = 1.8;
// From this many nodes the finest level is additive (z = S r + P B_1 P^T r):
// there its two smoothing J.v products cost more than the iterations they
// save (257x257x129: solve 88 -> 76 ms, adjoint 39 -> 34 ms; at 129x129x65
// the multiplicative form is faster, 11.3 against 11.9 ms).
static const long kMgAddTopNodes = 4000000;
// On those meshes a V-cycle costs about two Jacobi iterations, so the AUTO
// rule takes it from this CG tolerance on (257x257x129: 3e-2 / 5e-2 / 1e-1
// / 2e-1 gave FP64 solves of 71.5 / 48.0 / 46.8 / 46.8 ms, mixed 50.4 /
// 37.3 / 37.3 / 37.3; the same on its 129x129x65 coarse start as well
// measured slower, 47.7, and at 129x129x65 itself 1e-1 made the solve 3 %
// slower).
static const double kMgEtaLarge = 1e-1;
static double mg_omega() {
  const double w = env_double("QE_MG_OMEGA", kMgOmega);
  return (w > 0.0 && w < 2.0) ? w : kMgOmega;
}

struct MgPlan {
  int nlev = 0;
  qe_problem pc[kMgMaxLevels];
  size_t o_y0 = 0, o_y0_32 = 0, o_S[kMgMaxLevels] = {}, o_S32[kMgMaxLevels] = {}, o_phi[kMgMaxLevels] = {},
         o_ws[kMgMaxLevels] = {}, ws_bytes[kMgMaxLevels] = {};
  size_t o_pI[kMgMaxLevels][3] = {}, o_pw[kMgMaxLevels][3] = {}, o_rI[kMgMaxLevels][3] = {},
         o_rw[kMgMaxLevels][3] = {};
  // with eigenstates: each coarse level's states (|psi|^2 and phi^(k) at its
  // nodes, the region flag of its elements; the levels E_i are shared)
  qe_quantum qc[kMgMaxLevels] = {};
  size_t total = 0;
};

static bool mg_plan(const qe_problem* p, char* base, MgPlan& mp) {
  mp.nlev = 0;
  const long N = (long)p->nx * p->ny * p->nz;
  if (N < env_long("QE_MG_MIN_NODES", kMgMinNodes)) return false;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = align256(off + b);
    return o;
  };
  mp.pc[0] = *p;
  mp.o_S[0] = take(N * 8);
  mp.o_y0 = take(N * 8);
  mp.o_S32[0] = take(N * 4);
  mp.o_y0_32 = take(N * 4);
  int L = 1;
  while (L < kMgMaxLevels) {
    qe_problem c;
    size_t o2 = off;
    if (!carve_coarse(&mp.pc[L - 1], base, o2, c)) break;
    const long Nc = (long)c.nx * c.ny * c.nz;
    if (Nc < env_long("QE_MG_MIN_COARSE", kMgMinCoarse)) break;
    off = o2;
    if (p->quantum) {
      const qe_quantum& qf = *mp.pc[L - 1].quantum;
      qe_quantum& q = mp.qc[L];
      q = qf;
      const long Ec = (long)(c.nx - 1) * (c.ny - 1) * (c.nz - 1);
      q.psi2 = reinterpret_cast<const double*>(base + take((size_t)qf.n_states * Nc * 8));
      q.phi_k = reinterpret_cast<const double*>(base + take(Nc * 8));
      q.region = qf.region ? reinterpret_cast<const uint8_t*>(base + take(Ec)) : nullptr;
      c.quantum = &q;
    }
    mp.pc[L] = c;
    mp.o_phi[L] = take(Nc * 8);
    mp.o_S[L] = take(Nc * 8);
    mp.o_S32[L] = take(Nc * 4);
    const int nf[3] = {mp.pc[L - 1].nx, mp.pc[L - 1].ny, mp.pc[L - 1].nz}, nc[3] = {c.nx, c.ny, c.nz};
    for (int a = 0; a < 3; ++a) {
      mp.o_pI[L][a] = take(nf[a] * 4);
      mp.o_pw[L][a] = take(nf[a] * 8);
      mp.o_rI[L][a] = take(nc[a] * 3 * 4);
      mp.o_rw[L][a] = take(nc[a] * 3 * 8);
    }
    mp.ws_bytes[L] = layout_bytes(&c, mg_coarse_kz(Nc));
    mp.o_ws[L] = take(mp.ws_bytes[L]);
    ++L;
  }
  if (L < 2) return false;
  mp.nlev = L;
  mp.total = off;
  return true;
}

static size_t mg_extra_bytes(const qe_problem* p) {
  MgPlan mp;
  return mg_plan(p, reinterpret_cast<char*>(size_t(1) << 20), mp) ? mp.total : 0;
}

// Room after the fine layout: the sequence's coarse solve before Newton and
// the multigrid levels during it use the same region.
static size_t extra_bytes(const qe_problem* p, int seq_levels) {
  return std::max(seq_extra_bytes(p, seq_levels), mg_extra_bytes(p));
}

// The AUTO threshold for a mesh of this many nodes (QE_MG_ETA overrides it
// for every mesh).
static double mg_eta(long nodes) {
  const char* v = getenv("QE_MG_ETA");
  if (v) return atof(v);
  return nodes >= env_long("QE_MG_ADD_NODES", kMgAddTopNodes) ? kMgEtaLarge : kMgEta;
}

// One call's multigrid levels: planned when the call may use them, set up
// on first use, linearised at each potential a CG solve with them starts
// from.
struct MgState {
  MgPlan plan;
  char* base = nullptr;
  bool possible = false, ready = false;
  Context cx[kMgMaxLevels];   // levels 1 .. nlev - 1
  MgGrid lv[kMgMaxLevels];
  MgRun run{};

  bool fp32 = false;   // the CG it serves runs in FP32 (mixed precision)

  // Whether multigrid can serve this call (an allocating entry point, a
  // large enough plain mesh, room in the workspace).
  void plan_for(const qe_problem* p, const qe_options* o, void* ws, size_t ws_bytes, bool mixed, bool no_alloc) {
    possible = false;
    fp32 = mixed;
    if (no_alloc || o->precond == QE_PC_JACOBI) return;
    const size_t fine = align256(fine_layout_bytes(p));
    if (ws_bytes < fine) return;
    base = reinterpret_cast<char*>(ws) + fine;
    possible = mg_plan(p, base, plan) && ws_bytes - fine >= plan.total;
  }
  bool wanted(const qe_options* o, double eta) const {
    return possible && (o->precond == QE_PC_MULTIGRID || eta <= mg_eta(plan.pc[0].nx * (long)plan.pc[0].ny * plan.pc[0].nz));
  }
  qe_status setup(Context& fine, const Charge& ch) {
    for (int l = 1; l < plan.nlev; ++l) {
      launch_seq_coarsen(fine.s, &plan.pc[l - 1], &plan.pc[l]);
      if (plan.pc[l].quantum) launch_mg_coarsen_states(fine.s, &plan.pc[l - 1], &plan.pc[l]);
      QE_HIP(hipGetLastError());
      const long nl = (long)plan.pc[l].nx * plan.pc[l].ny * plan.pc[l].nz;
      QE_TRY(cx[l].init(&plan.pc[l], ch, base + plan.o_ws[l], plan.ws_bytes[l], fine.s, 0, false, mg_coarse_kz(nl)));
      QE_TRY(cx[l].stage(nullptr, 0, 0));
      if (fp32) launch_stage_eps32(fine.s, cx[l].vblocks, cx[l].g, plan.pc[l].eps_r, cx[l].f32(cx[l].lay.eps32),
                                   cx[l].nslots);
    }
    for (int l = 0; l < plan.nlev; ++l) {
      Context& c = l == 0 ? fine : cx[l];
      MgGrid& G = lv[l];
      G.g = c.g;
      G.wm = c.wm;
      G.N = c.N;
      G.eps_t = c.f64(c.lay.eps_t);
      G.cbits = c.u32(c.lay.cbits);
      G.cq = c.f64(c.lay.c);
      G.mask = c.u8(c.lay.mask);
      G.S = reinterpret_cast<double*>(base + plan.o_S[l]);
      G.b = c.f64(c.lay.r);
      G.x = l == 0 ? c.f64(c.lay.z) : c.f64(c.lay.x);
      G.y = l == 0 ? reinterpret_cast<double*>(base + plan.o_y0) : c.f64(c.lay.y);
      G.eps32 = c.f32(c.lay.eps32);
      G.cq32 = c.f32(c.lay.c32);
      G.S32 = reinterpret_cast<float*>(base + plan.o_S32[l]);
      G.b32 = c.f32(c.lay.r32);
      G.x32 = l == 0 ? c.f32(c.lay.z32) : c.f32(c.lay.x32);
      G.y32 = l == 0 ? reinterpret_cast<float*>(base + plan.o_y0_32) : c.f32(c.lay.y32);
      for (int a = 0; a < 3 && l > 0; ++a) {
        G.tab.pI[a] = reinterpret_cast<int*>(base + plan.o_pI[l][a]);
        G.tab.pw[a] = reinterpret_cast<double*>(base + plan.o_pw[l][a]);
        G.tab.rI[a] = reinterpret_cast<int*>(base + plan.o_rI[l][a]);
        G.tab.rw[a] = reinterpret_cast<double*>(base + plan.o_rw[l][a]);
      }
    }
    for (int l = 1; l < plan.nlev; ++l) launch_mg_tables(fine.s, lv[l - 1], lv[l]);
    QE_HIP(hipGetLastError());
    run = MgRun{lv, plan.nlev, std::max(1, env_int("QE_MG_SWEEPS", kMgSweeps)),
                fine.N >= env_long("QE_MG_ADD_NODES", kMgAddTopNodes)};
    ready = true;
    return QE_OK;
  }
  // The coarse levels' Jacobians at the potential injected from phi (the
  // fine level's was formed by the caller's last residual at phi), then
  // every level's smoother weights.
  qe_status linearize(Context& fine, const Charge& ch, const double* phi) {
    const double* src = phi;
    for (int l = 1; l < plan.nlev; ++l) {
      double* ph = reinterpret_cast<double*>(base + plan.o_phi[l]);
      launch_mg_inject(fine.s, lv[l - 1], lv[l], src, ph);
      QE_TRY(cx[l].residual(ch, ph, nullptr, nullptr, 0.0, fp32, nullptr, nullptr));
      src = ph;
    }
    for (int l = 0; l < plan.nlev; ++l) {
      Context& c = l == 0 ? fine : cx[l];
      launch_mg_l1(fine.s, lv[l], c.prob.eps_r, c.u8(c.lay.cflag), mg_omega(), fp32);
    }
    QE_HIP(hipGetLastError());
    return QE_OK;
  }
  // Ready to serve a CG solve at phi (set up on first use).
  qe_status prepare(Context& fine, const Charge& ch, const double* phi) {
    if (!ready) QE_TRY(setup(fine, ch));
    return linearize(fine, ch, phi);
  }
};

extern "C" {

const char* qe_last_error(void) { return g_last_error.c_str(); }

static void fill_report(qe_report* rep, const qe_report& r) {
  if (rep) *rep = r;
}

static qe_status finish(qe_status st, qe_report& r, qe_report* rep) {
  r.status = st;
  fill_report(rep, r);
  return st;
}

}  // extern "C"

// qe_solve's body; no_alloc: host read-backs in static storage and the CG
// polled without events (qe_solve_static).  newton_rtol > 0 (the coarse
// levels of a sequence) also stops Newton once ||F|| falls below that
// fraction of its initial value.
static qe_status solve_impl(const qe_problem* p, const qe_physics* ph, const qe_options* o, double* phi,
                            double* n_nodal, void* ws, size_t ws_bytes, void* stream, qe_report* rep, bool no_alloc,
                            double newton_rtol = 0.0, int seq_levels = -1, bool trusted = false) {
  clear_error();
  qe_report r;
  std::memset(&r, 0, sizeof(r));
  Charge ch, lin;
  qe_status st;
  if ((st = check_options(o)) != QE_OK) return finish(st, r, rep);
  if ((st = make_charge(ph, ch)) != QE_OK) return finish(st, r, rep);
  if (!phi) return finish(fail(QE_ERR_INVALID_ARG, "phi is NULL"), r, rep);
  Context cx;
  if ((st = cx.init(p, ch, ws, ws_bytes, stream, 0, no_alloc)) != QE_OK) return finish(st, r, rep);
  const bool mixed = o->precision == QE_PREC_MIXED;
  // (trusted: a coarse problem built here from a checked one needs no
  // checks, each a round trip to the device)
  if (!trusted && (st = cx.validate(o->init_guess == 1 ? phi : nullptr)) != QE_OK) return finish(st, r, rep);
  // coarse-mesh sequence: the coarse problem's arrays are built from this
  // one's (validated above), solved, and its potential interpolated into phi
  bool linear = o->init_guess == 0;
  if (o->init_guess == 2) {
    SeqPlan sp;
    const size_t fine = align256(fine_layout_bytes(p));
    char* base = reinterpret_cast<char*>(ws) + fine;
    const int levels = seq_levels < 0 ? seq_levels_wanted() : seq_levels;
    if (ws_bytes >= fine && seq_plan(p, base, sp, levels) && ws_bytes - fine >= sp.total) {
      launch_seq_coarsen(cx.s, p, &sp.pc);
      if (hipGetLastError() != hipSuccess) return finish(fail(QE_ERR_HIP, "coarsening launch failed"), r, rep);
      qe_report rc;
      double* phic = reinterpret_cast<double*>(base + sp.o_phi);
      // the coarse solve only starts this one: its CG runs in FP32 (inside
      // its FP64 Newton), as in mixed precision (the 129x129x65 solve's
      // step: 9.46-9.57 -> 9.20-9.43 ms, the same iteration counts, phi equal
      // to 1e-15)
      qe_options oc = *o;
      oc.precision = QE_PREC_MIXED;
      const qe_status sc = solve_impl(&sp.pc, ph, &oc, phic, nullptr, base + sp.o_ws, sp.total - sp.o_ws, stream, &rc,
                                      no_alloc, seq_rtol((long)sp.pc.nx * sp.pc.ny * sp.pc.nz), levels - 1, true);
      if (sc == QE_ERR_HIP) return finish(sc, r, rep);
      if (sc == QE_OK || sc == QE_ERR_NOT_CONVERGED) {
        launch_seq_prolong(cx.s, p, &sp.pc, phic, phi);
        if (hipGetLastError() != hipSuccess) return finish(fail(QE_ERR_HIP, "interpolation launch failed"), r, rep);
        r.seq_levels = rc.seq_levels + 1;
        r.init_krylov_iters = rc.krylov_iters;
        r.krylov_iters += rc.krylov_iters;
      }
      clear_error();   // a coarse solve that failed leaves the linear guess, not an error
    }
    linear = r.seq_levels == 0;
  }
  if ((st = cx.stage(phi, 1, linear ? 1 : 0)) != QE_OK) return finish(st, r, rep);
  if (mixed) {
    launch_stage_eps32(cx.s, cx.vblocks, cx.g, p->eps_r, cx.f32(cx.lay.eps32), cx.nslots);
    if (hipGetLastError() != hipSuccess) return finish(fail(QE_ERR_HIP, "cast launch failed"), r, rep);
  }
  const int check = o->check_every;
  int pst = 0, its = 0;
  MgState mg;
  mg.plan_for(p, o, ws, ws_bytes, mixed, no_alloc);
  if (linear) {
    // charge-free linear Poisson with the doping kept: one Newton step from
    // phi = (Dirichlet values, 0) on the linear problem
    lin = linear_charge(ch);
    double n2;
    if ((st = cx.residual(lin, phi, nullptr, nullptr, 0.0, mixed, nullptr, &n2)) != QE_OK) return finish(st, r, rep);
    if (!std::isfinite(n2)) return finish(fail(QE_ERR_NONFINITE, "initial residual not finite"), r, rep);
    if (n2 > 0) {
      if ((st = cx.pcg(mixed, cx.f64(cx.lay.F), -1.0, mixed ? std::max(1e-6, QE_INIT_RTOL) : QE_INIT_RTOL,
                       o->krylov_maxit, check, &pst, &its)) != QE_OK)
        return finish(st, r, rep);
      r.init_krylov_iters = its;
      r.krylov_iters += its;
      if (pst == PCG_BREAKDOWN || pst == PCG_NONFINITE)
        return finish(fail(pst == PCG_BREAKDOWN ? QE_ERR_KRYLOV_BREAKDOWN : QE_ERR_NONFINITE,
                           "linear initial guess: CG failed (status %d)", pst), r, rep);
      launch_axpy_phi(cx.s, cx.vblocks, cx.N, phi, mixed ? nullptr : cx.f64(cx.lay.x),
                      mixed ? cx.f32(cx.lay.x32) : nullptr, 1.0);
    }
  }
  double n2;
  if ((st = cx.residual(ch, phi, nullptr, nullptr, 0.0, mixed, nullptr, &n2)) != QE_OK) return finish(st, r, rep);
  r.n_residual_evals++;
  double nrm = std::sqrt(n2), prev = -1.0;
  r.res0 = nrm;
  r.res_final = nrm;
  if (!std::isfinite(nrm)) return finish(fail(QE_ERR_NONFINITE, "residual not finite at the initial guess"), r, rep);
  st = QE_ERR_NOT_CONVERGED;
  for (int it = 0; it <= o->newton_maxit; ++it) {
    if (nrm <= o->newton_atol || nrm <= newton_rtol * r.res0) {
      st = QE_OK;
      break;
    }
    if (it == o->newton_maxit) break;
    double eta = prev < 0 ? o->krylov_rtol_max
                          : std::min(o->krylov_rtol_max, QE_EW_GAMMA * (nrm / prev) * (nrm / prev));
    eta = std::max(eta, 0.5 * o->newton_atol / nrm);
    eta = std::min(eta, o->krylov_rtol_max);
    eta = std::max(eta, mixed ? 1e-6 : 1e-13);
    const bool use_mg = mg.wanted(o, eta);
    if (use_mg && (st = mg.prepare(cx, ch, phi)) != QE_OK) return finish(st, r, rep);
    qe_status s2 = cx.pcg(mixed, cx.f64(cx.lay.F), -1.0, eta, o->krylov_maxit, check, &pst, &its,
                          use_mg ? &mg.run : nullptr);
    if (s2 != QE_OK) return finish(s2, r, rep);
    r.krylov_iters += its;
    if (use_mg) {
      r.mg_krylov_iters += its;
      r.mg_levels = mg.plan.nlev;
    }
    if (pst == PCG_BREAKDOWN || pst == PCG_NONFINITE) {
      st = fail(pst == PCG_BREAKDOWN ? QE_ERR_KRYLOV_BREAKDOWN : QE_ERR_NONFINITE, "Newton step %d: CG failed (status %d)",
                it, pst);
      break;
    }
    double lam = 1.0, nt = 0.0;
    bool ok = false;
    for (int hv = 0; hv <= o->ls_max_halvings; ++hv) {
      if ((s2 = cx.residual(ch, phi, mixed ? nullptr : cx.f64(cx.lay.x), mixed ? cx.f32(cx.lay.x32) : nullptr, lam,
                            mixed, nullptr, &n2)) != QE_OK)
        return finish(s2, r, rep);
      r.n_residual_evals++;
      nt = std::sqrt(n2);
      if (std::isfinite(nt) && nt <= (1.0 - 1e-4 * lam) * nrm) {
        ok = true;
        break;
      }
      lam *= 0.5;
      r.ls_halvings++;
    }
    if (!ok) {
      st = fail(QE_ERR_LINESEARCH, "line search failed at Newton step %d (||F|| = %.3e)", it, nrm);
      break;
    }
    launch_axpy_phi(cx.s, cx.vblocks, cx.N, phi, mixed ? nullptr : cx.f64(cx.lay.x),
                    mixed ? cx.f32(cx.lay.x32) : nullptr, lam);
    prev = nrm;
    nrm = nt;
    r.newton_iters = it + 1;
    r.res_final = nrm;
  }
  if (st == QE_ERR_NOT_CONVERGED)
    fail(st, "Newton did not reach atol %.3e in %d steps (||F|| = %.3e)", o->newton_atol, o->newton_maxit, nrm);
  if (n_nodal) launch_density(cx.s, cx.vblocks, cx.g, ch, p->semi, phi, n_nodal, cx.quantum);
  if (hipStreamSynchronize(cx.s) != hipSuccess || hipGetLastError() != hipSuccess)
    return finish(fail(QE_ERR_HIP, "stream error at the end of the solve"), r, rep);
  return finish(st, r, rep);
}

// The workspace of qe_solve_static on each GPU: a file-scope device array
// (QE_STATIC_WS_BYTES), whose address is taken once per device with that
// device current; host code passes that address, never the array's name.
static __device__ __align__(256) char scratch[QE_STATIC_WS_BYTES];
static void* g_scratch_ptr[64] = {};
static std::mutex g_scratch_mutex;

static qe_status scratch_ptr(void** out) {
  int dev = -1;
  QE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(QE_ERR_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    QE_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(QE_ERR_HIP, "hipGetSymbolAddress returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return QE_OK;
}

extern "C" {

qe_status qe_solve(const qe_problem* p, const qe_physics* ph, const qe_options* o, double* phi, double* n_nodal,
                   void* ws, size_t ws_bytes, void* stream, qe_report* rep) {
  return solve_impl(p, ph, o, phi, n_nodal, ws, ws_bytes, stream, rep, false);
}

qe_status qe_solve_static(const qe_problem* p, const qe_physics* ph, const qe_options* o, double* phi,
                          double* n_nodal, void* stream, qe_report* rep) {
  clear_error();
  qe_report r;
  std::memset(&r, 0, sizeof(r));
  qe_status st;
  if ((st = check_problem(p)) != QE_OK) return finish(st, r, rep);
  // the coarse levels of a sequence are used when the static array has room
  // for them as well, the linear guess otherwise
  const size_t need = fine_layout_bytes(p);
  if (need > (size_t)QE_STATIC_WS_BYTES)
    return finish(fail(QE_ERR_WORKSPACE, "the problem needs %zu bytes of workspace, more than the %zu of the static "
                                         "workspace (use qe_solve with a caller workspace)",
                       need, (size_t)QE_STATIC_WS_BYTES),
                  r, rep);
  void* ws = nullptr;
  if ((st = scratch_ptr(&ws)) != QE_OK) return finish(st, r, rep);
  return solve_impl(p, ph, o, phi, n_nodal, ws, QE_STATIC_WS_BYTES, stream, rep, true);
}

qe_status qe_residual(const qe_problem* p, const qe_physics* ph, const double* phi, double* F, double* diag,
                      double* norm2, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  Charge ch;
  QE_TRY(make_charge(ph, ch));
  if (!phi || !F) return fail(QE_ERR_INVALID_ARG, "phi/F is NULL");
  Context cx;
  QE_TRY(cx.init(p, ch, ws, ws_bytes, stream));
  QE_TRY(cx.validate(phi));
  QE_TRY(cx.stage(nullptr, 0, 0));
  double n2;
  QE_TRY(cx.residual(ch, phi, nullptr, nullptr, 0.0, false, diag, &n2));
  QE_HIP(hipMemcpyAsync(F, cx.ws + cx.lay.F, cx.N * sizeof(double), hipMemcpyDeviceToDevice, cx.s));
  QE_HIP(hipStreamSynchronize(cx.s));
  if (norm2) *norm2 = n2;
  return QE_OK;
}

qe_status qe_jv(const qe_problem* p, const qe_physics* ph, const double* phi, const double* v, double* y, void* ws,
                size_t ws_bytes, void* stream) {
  clear_error();
  Charge ch;
  QE_TRY(make_charge(ph, ch));
  if (!phi || !v || !y) return fail(QE_ERR_INVALID_ARG, "phi/v/y is NULL");
  Context cx;
  QE_TRY(cx.init(p, ch, ws, ws_bytes, stream));
  QE_TRY(cx.validate(phi));
  QE_TRY(cx.stage(nullptr, 0, 0));
  QE_TRY(cx.residual(ch, phi, nullptr, nullptr, 0.0, false, nullptr, nullptr));
  launch_jv_wave64(cx.s, cx.g, cx.wm, cx.f64(cx.lay.eps_t), cx.u32(cx.lay.cbits), cx.f64(cx.lay.c), cx.u8(cx.lay.mask), v,
                   y, 1);
  if (cx.sheets.any_robin) launch_sheet_jv64(cx.s, cx.sheets, cx.sheet_items(), cx.u8(cx.lay.mask), v, y, nullptr, nullptr, nullptr);
  QE_HIP(hipGetLastError());
  QE_HIP(hipStreamSynchronize(cx.s));
  return QE_OK;
}

qe_status qe_jv_f32(const qe_problem* p, const qe_physics* ph, const double* phi, const float* v, float* y, void* ws,
                    size_t ws_bytes, void* stream) {
  clear_error();
  Charge ch;
  QE_TRY(make_charge(ph, ch));
  if (!phi || !v || !y) return fail(QE_ERR_INVALID_ARG, "phi/v/y is NULL");
  Context cx;
  QE_TRY(cx.init(p, ch, ws, ws_bytes, stream));
  QE_TRY(cx.validate(phi));
  QE_TRY(cx.stage(nullptr, 0, 0));
  QE_TRY(cx.residual(ch, phi, nullptr, nullptr, 0.0, true, nullptr, nullptr));
  launch_stage_eps32(cx.s, cx.vblocks, cx.g, p->eps_r, cx.f32(cx.lay.eps32), cx.nslots);
  launch_jv_wave32(cx.s, cx.g, cx.wm, cx.f32(cx.lay.eps32), cx.u32(cx.lay.cbits), cx.f32(cx.lay.c32), cx.u8(cx.lay.mask), v,
                   y, 1);
  if (cx.sheets.any_robin) launch_sheet_jv32(cx.s, cx.sheets, cx.sheet_items(), cx.u8(cx.lay.mask), v, y, nullptr, nullptr, nullptr);
  QE_HIP(hipGetLastError());
  QE_HIP(hipStreamSynchronize(cx.s));
  return QE_OK;
}

qe_status qe_time_jv(const qe_problem* p, const qe_physics* ph, const double* phi, const double* v,
                     int32_t precision, int32_t reps, double* ms_per_apply, int64_t* n_coef_elems,
                     void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  Charge ch;
  QE_TRY(make_charge(ph, ch));
  if (!phi || !v || !ms_per_apply) return fail(QE_ERR_INVALID_ARG, "phi/v/ms_per_apply is NULL");
  if (reps < 1) return fail(QE_ERR_INVALID_ARG, "reps < 1");
  if (precision != QE_PREC_FP64 && precision != QE_PREC_MIXED) return fail(QE_ERR_INVALID_ARG, "bad precision");
  const bool mixed = precision == QE_PREC_MIXED;
  Context cx;
  QE_TRY(cx.init(p, ch, ws, ws_bytes, stream));
  QE_TRY(cx.validate(phi));
  QE_TRY(cx.stage(nullptr, 0, 0));
  QE_TRY(cx.residual(ch, phi, nullptr, nullptr, 0.0, mixed, nullptr, nullptr));
  // The CG loop's first kernel in its steady state (iteration >= 1,
  // beta = 1): z = D^-1 v on free rows (0 on Dirichlet rows, as CG keeps it),
  // y = p = 0, and scalars that never stop the solve.
  const int cgb = cg_blocks(cx.N);
  PcgCtx* dctx = reinterpret_cast<PcgCtx*>(cx.ws + cx.lay.ctx);
  if (mixed) {
    launch_stage_eps32(cx.s, cx.vblocks, cx.g, p->eps_r, cx.f32(cx.lay.eps32), cx.nslots);
    launch_pcg_start32(cx.s, cgb, cx.N, 1.0, v, cx.u8(cx.lay.mask), cx.f32(cx.lay.invdiag32), cx.f32(cx.lay.x32),
                       cx.f32(cx.lay.r32), cx.f32(cx.lay.z32), dctx, cx.f64(cx.lay.partial2), 0.0, 1 << 30);
    QE_HIP(hipMemsetAsync(cx.ws + cx.lay.y32, 0, cx.N * 4, cx.s));
    QE_HIP(hipMemsetAsync(cx.ws + cx.lay.p32, 0, cx.N * 4, cx.s));
  } else {
    launch_pcg_start64(cx.s, cgb, cx.N, 1.0, v, cx.u8(cx.lay.mask), cx.f64(cx.lay.invdiag), cx.f64(cx.lay.x),
                       cx.f64(cx.lay.r), cx.f64(cx.lay.z), dctx, cx.f64(cx.lay.partial2), 0.0, 1 << 30);
    QE_HIP(hipMemsetAsync(cx.ws + cx.lay.y, 0, cx.N * 8, cx.s));
    QE_HIP(hipMemsetAsync(cx.ws + cx.lay.p, 0, cx.N * 8, cx.s));
  }
  PcgCtx& hc = *mirror().ctx;
  QE_HIP(hipMemcpyAsync(&hc, dctx, sizeof(PcgCtx), hipMemcpyDeviceToHost, cx.s));
  QE_HIP(hipStreamSynchronize(cx.s));
  if (hc.done) return fail(QE_ERR_INVALID_ARG, "v vanishes on the free nodes");
  hc.iters = 1;
  hc.rzs[1] = hc.rzs[0];
  hc.tol2 = 0.0;
  hc.alpha = 0.0;   // the fused solution step leaves x = 0
  QE_HIP(hipMemcpyAsync(dctx, &hc, sizeof(PcgCtx), hipMemcpyHostToDevice, cx.s));
  QE_HIP(hipStreamSynchronize(cx.s));
  hipEvent_t e0, e1;
  QE_HIP(hipEventCreate(&e0));
  QE_HIP(hipEventCreate(&e1));
  auto once = [&]() {
    if (mixed)
      launch_cg_jv32(cx.s, cx.g, cx.wm, cgb, 0, cx.f32(cx.lay.eps32), cx.u32(cx.lay.cbits), cx.f32(cx.lay.c32),
                     cx.f32(cx.lay.z32), cx.f32(cx.lay.y32), cx.f32(cx.lay.p32), cx.f32(cx.lay.x32), dctx,
                     mirror().prog_dev,
                     cx.f64(cx.lay.partial2), cx.f64(cx.lay.partial));
    else
      launch_cg_jv64(cx.s, cx.g, cx.wm, cgb, 0, cx.f64(cx.lay.eps_t), cx.u32(cx.lay.cbits), cx.f64(cx.lay.c),
                     cx.f64(cx.lay.z), cx.f64(cx.lay.y), cx.f64(cx.lay.p), cx.f64(cx.lay.x), dctx,
                     mirror().prog_dev,
                     cx.f64(cx.lay.partial2), cx.f64(cx.lay.partial));
  };
  once();  // warm-up
  hipError_t e = hipEventRecord(e0, cx.s);
  for (int k = 0; k < reps && e == hipSuccess; ++k) once();
  if (e == hipSuccess) e = hipEventRecord(e1, cx.s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(QE_ERR_HIP, "timing failed: %s", hipGetErrorString(e));
  *ms_per_apply = (double)ms / reps;
  if (n_coef_elems) {
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(cx.ws + cx.lay.scal) + 63;
    QE_HIP(hipMemsetAsync(cnt, 0, sizeof(*cnt), cx.s));
    launch_count_flags(cx.s, cx.vblocks, cx.g, cx.u8(cx.lay.cflag), cx.nslots, cnt);
    QE_HIP(hipGetLastError());
    QE_HIP(hipMemcpyAsync(mirror().scal, cnt, sizeof(*cnt), hipMemcpyDeviceToHost, cx.s));
    QE_HIP(hipStreamSynchronize(cx.s));
    unsigned long long v64;
    std::memcpy(&v64, mirror().scal, sizeof(v64));
    *n_coef_elems = (int64_t)v64;
  }
  return QE_OK;
}

qe_status qe_count_electrons(const qe_problem* p, const qe_physics* ph, const double* phi, int32_t n_boxes,
                             const double* boxes, double* counts, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  Charge ch;
  QE_TRY(make_charge(ph, ch));
  if (!phi || !boxes || !counts) return fail(QE_ERR_INVALID_ARG, "phi/boxes/counts is NULL");
  if (n_boxes < 1 || n_boxes > kMaxBoxes) return fail(QE_ERR_INVALID_ARG, "n_boxes must be in [1, %d]", kMaxBoxes);
  BoxSet bs;
  bs.n = n_boxes;
  for (int r = 0; r < n_boxes; ++r) {
    const double* b = boxes + 6 * r;
    for (int k = 0; k < 6; ++k)
      if (std::isnan(b[k])) return fail(QE_ERR_INVALID_ARG, "box %d has NaN", r);
    bs.b[r] = Box{b[0], b[1], b[2], b[3], b[4], b[5]};
  }
  Context cx;
  QE_TRY(cx.init(p, ch, ws, ws_bytes, stream));
  QE_TRY(cx.validate(phi));
  launch_count(cx.s, kCountBlocks, cx.g, ch, bs, p->semi, phi, cx.f64(cx.lay.partial),
               reinterpret_cast<unsigned int*>(cx.ws + cx.lay.counters) + 1, cx.f64(cx.lay.scal), cx.quantum);
  QE_HIP(hipGetLastError());
  QE_HIP(hipMemcpyAsync(mirror().scal, cx.ws + cx.lay.scal, n_boxes * sizeof(double), hipMemcpyDeviceToHost, cx.s));
  QE_HIP(hipStreamSynchronize(cx.s));
  for (int r = 0; r < n_boxes; ++r) counts[r] = mirror().scal[r];
  return QE_OK;
}

qe_status qe_density(const qe_problem* p, const qe_physics* ph, const double* phi, double* n, void* ws,
                     size_t ws_bytes, void* stream) {
  clear_error();
  Charge ch;
  QE_TRY(make_charge(ph, ch));
  if (!phi || !n) return fail(QE_ERR_INVALID_ARG, "phi/n is NULL");
  Context cx;
  QE_TRY(cx.init(p, ch, ws, ws_bytes, stream));
  QE_TRY(cx.validate(phi));
  launch_density(cx.s, cx.vblocks, cx.g, ch, p->semi, phi, n, cx.quantum);
  QE_HIP(hipGetLastError());
  QE_HIP(hipStreamSynchronize(cx.s));
  return QE_OK;
}

qe_status qe_adjoint(const qe_problem* p, const qe_physics* ph, const qe_options* o, const double* phi,
                     const double* box, double* Q, double* dQ_ddir, double* dQ_deps, double* lam, void* ws,
                     size_t ws_bytes, void* stream, qe_report* rep) {
  clear_error();
  qe_report r;
  std::memset(&r, 0, sizeof(r));
  Charge ch;
  qe_status st;
  if ((st = check_options(o)) != QE_OK) return finish(st, r, rep);
  if (o->precision != QE_PREC_FP64) return finish(fail(QE_ERR_INVALID_ARG, "the adjoint runs in FP64"), r, rep);
  if ((st = make_charge(ph, ch)) != QE_OK) return finish(st, r, rep);
  if (!phi || !box || !dQ_ddir) return finish(fail(QE_ERR_INVALID_ARG, "phi/box/dQ_ddir is NULL"), r, rep);
  if (p && p->quantum)
    return finish(fail(QE_ERR_INVALID_ARG, "the adjoint does not support predictor-corrector states"), r, rep);
  for (int k = 0; k < 6; ++k)
    if (std::isnan(box[k])) return finish(fail(QE_ERR_INVALID_ARG, "box has NaN"), r, rep);
  Context cx;
  if ((st = cx.init(p, ch, ws, ws_bytes, stream)) != QE_OK) return finish(st, r, rep);
  if ((st = cx.validate(phi)) != QE_OK) return finish(st, r, rep);
  if (p->n_dir > 56) return finish(fail(QE_ERR_INVALID_ARG, "the adjoint supports at most 56 contacts"), r, rep);
  if ((st = cx.stage(nullptr, 0, 0)) != QE_OK) return finish(st, r, rep);
  double n2;
  if ((st = cx.residual(ch, phi, nullptr, nullptr, 0.0, false, nullptr, &n2)) != QE_OK) return finish(st, r, rep);
  r.res0 = r.res_final = std::sqrt(n2);
  unsigned int* counters = reinterpret_cast<unsigned int*>(cx.ws + cx.lay.counters);
  const Box bx{box[0], box[1], box[2], box[3], box[4], box[5]};
  launch_adj_rhs(cx.s, cx.g, cx.tm, ch, bx, p->semi, phi, cx.f64(cx.lay.gvec), cx.f64(cx.lay.partial), counters + 2,
                 cx.f64(cx.lay.scal) + 1);
  int pst = 0, its = 0;
  MgState mg;
  mg.plan_for(p, o, ws, ws_bytes, false, false);
  const bool use_mg = mg.wanted(o, 1e-12);
  if (use_mg && (st = mg.prepare(cx, ch, phi)) != QE_OK) return finish(st, r, rep);
  if ((st = cx.pcg(false, cx.f64(cx.lay.gvec), 1.0, 1e-12, o->krylov_maxit, o->check_every, &pst, &its,
                   use_mg ? &mg.run : nullptr)) != QE_OK)
    return finish(st, r, rep);
  r.krylov_iters = its;
  if (use_mg) {
    r.mg_krylov_iters = its;
    r.mg_levels = mg.plan.nlev;
  }
  if (pst == PCG_BREAKDOWN || pst == PCG_NONFINITE)
    return finish(fail(pst == PCG_BREAKDOWN ? QE_ERR_KRYLOV_BREAKDOWN : QE_ERR_NONFINITE, "adjoint CG failed (status %d)",
                       pst), r, rep);
  // dQ/deps goes to the caller's buffer or to scratch (the y vector; E < N)
  double* deps_buf = dQ_deps ? dQ_deps : cx.f64(cx.lay.y);
  launch_adj_grad(cx.s, cx.g, cx.tm, p->eps_r, cx.u8(cx.lay.cflag), cx.f64(cx.lay.c), cx.u8(cx.lay.mask), cx.f64(cx.lay.x), phi,
                  cx.f64(cx.lay.gvec), deps_buf, cx.f64(cx.lay.r));
  if (cx.sheets.any_robin) launch_sheet_contact(cx.s, cx.sheets, cx.sheet_items(), cx.u8(cx.lay.mask), cx.f64(cx.lay.x), cx.f64(cx.lay.r));
  if (p->n_dir > 0)
    launch_contact_sum(cx.s, kContactBlocks, cx.N, p->n_dir, p->dir_id, cx.f64(cx.lay.r), cx.f64(cx.lay.partial),
                       counters + 3, cx.f64(cx.lay.scal) + 8);
  if (hipGetLastError() != hipSuccess) return finish(fail(QE_ERR_HIP, "adjoint launch failed"), r, rep);
  if (lam && hipMemcpyAsync(lam, cx.ws + cx.lay.x, cx.N * sizeof(double), hipMemcpyDeviceToDevice, cx.s) != hipSuccess)
    return finish(fail(QE_ERR_HIP, "copy of lam failed"), r, rep);
  const int nd = p->n_dir;
  if (hipMemcpyAsync(mirror().scal, cx.ws + cx.lay.scal, 64 * sizeof(double), hipMemcpyDeviceToHost, cx.s) != hipSuccess ||
      hipStreamSynchronize(cx.s) != hipSuccess)
    return finish(fail(QE_ERR_HIP, "adjoint read-back failed"), r, rep);
  if (Q) *Q = mirror().scal[1];
  for (int c = 0; c < nd; ++c) dQ_ddir[c] = mirror().scal[8 + c];
  st = (pst == PCG_MAXIT) ? fail(QE_ERR_KRYLOV_MAXIT, "adjoint CG hit krylov_maxit (%d)", its) : QE_OK;
  return finish(st, r, rep);
}

qe_status qe_ohmic_potential(const qe_physics* ph, double N_D, double N_A, double V_a, double* phi) {
  clear_error();
  if (!ph || !phi) return fail(QE_ERR_INVALID_ARG, "NULL argument");
  if (ph->stat != QE_STAT_MB && ph->stat != QE_STAT_FD12)
    return fail(QE_ERR_INVALID_ARG, "Ohmic contacts need Boltzmann or Fermi-Dirac statistics");
  if (!positive(ph->T_K)) return fail(QE_ERR_INVALID_ARG, "T_K must be > 0");
  if (!(N_D >= 0.0 && std::isfinite(N_D)) || !(N_A >= 0.0 && std::isfinite(N_A)))
    return fail(QE_ERR_INVALID_ARG, "N_D and N_A must be finite and >= 0");
  if (!std::isfinite(V_a) || !std::isfinite(ph->Ec0_eV)) return fail(QE_ERR_INVALID_ARG, "V_a and Ec0_eV must be finite");
  const bool ntype = N_D >= N_A;
  const double m = ntype ? ph->m_eff : ph->m_h;
  if (!positive(m)) return fail(QE_ERR_INVALID_ARG, ntype ? "m_eff must be > 0" : "m_h must be > 0");
  if (!ntype && !(ph->Eg_eV >= 0.0 && std::isfinite(ph->Eg_eV)))
    return fail(QE_ERR_INVALID_ARG, "Eg_eV must be finite and >= 0");
  const double kT = kKB * ph->T_K / kQ;  // eV
  const double Nband = effective_dos(m, ph->T_K);
  const double Ev0 = ph->Ec0_eV - ph->Eg_eV;   // E_V - E_F at phi = 0
  double v;
  if (ph->ionization == QE_ION_COMPLETE) {
    // majority carriers balance the net doping: n = N_D - N_A or p = N_A - N_D
    const double net = std::fabs(N_D - N_A);
    if (!(net > 0.0)) return fail(QE_ERR_INVALID_ARG, "net doping at the contact is zero");
    const double eta = ph->stat == QE_STAT_MB ? std::log(net / Nband) : nilsson_eta(net / Nband);
    v = ntype ? ph->Ec0_eV + kT * eta : Ev0 - kT * eta;   // Eqs. PotBC4MBCompIon, PotBC4FDCompIon
  } else if (ph->ionization == QE_ION_INCOMPLETE) {
    const double N = ntype ? N_D : N_A;
    const double E = ntype ? ph->Ed_eV : ph->Ea_eV, g = ntype ? ph->gD : ph->gA;
    if (!(N > 0.0)) return fail(QE_ERR_INVALID_ARG, "majority dopant density at the contact is zero");
    if (!std::isfinite(E) || !positive(g)) return fail(QE_ERR_INVALID_ARG, "bad ionization energy or degeneracy");
    const double ln_y = incomplete_ln_y(N, Nband, E / kT, g);
    // E_F - E_D = kT ln y_n with E_D = E_C - E_d; E_A - E_F = kT ln y_p with
    // E_A = E_V + E_a (Eq. PotBC4MBIncompIon)
    v = ntype ? ph->Ec0_eV - E + kT * ln_y : Ev0 + E - kT * ln_y;
  } else {
    return fail(QE_ERR_INVALID_ARG, "unknown ionization %d", ph->ionization);
  }
  *phi = v + V_a;
  return QE_OK;
}

}  // extern "C"
