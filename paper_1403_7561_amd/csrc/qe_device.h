// Device-side building blocks of the Q1 nonlinear-Poisson kernels (gfx950).
//
// Element-local algebra uses the local corner index a + 2b + 4c (x fastest).
// On a box element (hx, hy, hz) the unit-permittivity stiffness is
//   Khat = (hy hz/hx) A(x)M(y)M(z) + (hx hz/hy) M(x)A(y)M(z) + (hx hy/hz) M(x)M(y)A(z)
// with the unit 1D stiffness A = [[1,-1],[-1,1]] and mass M = [[2,1],[1,2]]/6;
// it is applied axis by axis (sum factorisation), never formed.  Gauss-point
// interpolation with the 2-point rule is the tensor product of the symmetric
// 1D matrix B = [[g1, g0], [g0, g1]], g1,0 = (1 +- 1/sqrt(3))/2, so the same
// routine also performs the projection back to the corners.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qe {

// Block tiles of the adjoint sweeps (k_adj_rhs, k_adj_grad).
constexpr int kTX = 16;               // owned node columns per tile in x
constexpr int kTY = 16;               // ... in y
constexpr int kEX = kTX + 1;          // element columns per tile (one halo column)
constexpr int kEY = kTY + 1;
constexpr int kNXL = kTX + 2;         // staged node columns
constexpr int kNYL = kTY + 2;
constexpr int kNEL = kEX * kEY;       // elements per tile layer (289)
constexpr int kNNL = kNXL * kNYL;     // staged nodes per plane (324)
constexpr int kThreads = 256;         // 4 waves of 64
constexpr int kJvThreads = 320;       // 5 waves: one thread per tile element (289)
constexpr int kMaxKz = 16;            // node planes per chunk, at most
constexpr int kVecThreads = 256;

constexpr double kG1 = 0.78867513459481288225;   // (1 + 1/sqrt(3)) / 2
constexpr double kG0 = 0.21132486540518711775;   // (1 - 1/sqrt(3)) / 2

enum Stat : int { STAT_LINEAR = 0, STAT_TF = 1, STAT_FD = 2, STAT_MB = 3 };

// Mesh geometry (device pointers to the caller's coordinate arrays).
struct Geom {
  int nx, ny, nz;
  const double* x;
  const double* y;
  const double* z;
  const double* rdz;   // [nz-1] 1 / (z[k+1] - z[k]), staged in the workspace
  const double* hz;    // [nz-1] z[k+1] - z[k], staged after rdz (NULL where unused)
};

// Electron statistics constants (derived on the host from CODATA values).
struct Charge {
  int stat;
  double Ec0;      // eV
  double inv_kT;   // 1/eV
  double Nc;       // nm^-3
  double Ctf;      // nm^-3 eV^-3/2
  double kappa;    // q/eps0 in V nm
  // the rest of the space charge of Eq. Poisson
  int holes;       // p(phi) with E_V - E_F = Ec0 - Eg - phi
  int incomplete;  // Eq. FinalIonization from per-element N_D, N_A
  double Nv;       // valence effective DOS, nm^-3
  double Ctf_h;    // valence Thomas-Fermi prefactor
  double Eg;       // eV
  double ed_kT, ea_kT;   // E_d / kT, E_a / kT
  double ln_gD, ln_gA;   // ln of the degeneracy factors
  double T_K;
};

// Charge of the linear initial-guess problem: no mobile charge, dopants fully
// ionised (N_D - N_A from the species when no net doping is given).
__host__ __device__ inline Charge linear_charge(const Charge& ch) {
  Charge lin = ch;
  lin.stat = STAT_LINEAR;
  lin.holes = 0;
  lin.incomplete = 0;
  return lin;
}

// Tile decomposition of the node grid: gx*gy tiles of kTX x kTY node columns,
// gz chunks of kz node planes.
struct TileMap {
  int gx, gy, gz, kz;
  int nblocks;
};

// Block b is dispatched to XCD b % 8; hand each XCD a contiguous run of tiles
// so that neighbouring tiles (which re-read each other's halo) share an L2.
__device__ __forceinline__ void tile_of_block(int b, const TileMap& tm, int& tx, int& ty, int& tz) {
  const int per = tm.nblocks >> 3, rem = tm.nblocks & 7;
  const int xcd = b & 7, loc = b >> 3;
  int t = (xcd < rem) ? xcd * (per + 1) + loc : rem * (per + 1) + (xcd - rem) * per + loc;
  tx = t % tm.gx;
  t /= tm.gx;
  ty = t % tm.gy;
  tz = t / tm.gy;
}

// Wave tiles of the J.v kernel: gx*gy tiles of 7 x 7 owned node columns,
// gz chunks of kz node planes, four waves per block.
struct WaveMap {
  int gx, gy, gz, kz;
  int nwaves, nblocks;
};

// Wave tile (wx, wy, wz) of wave index w: x fastest, so a block's four
// waves are neighbours in x (measured faster at 129x129x65 than z fastest).
__host__ __device__ __forceinline__ void wave_tile_of(int w, const WaveMap& wm, int& wx, int& wy, int& wz) {
  wx = w % wm.gx;
  wy = (w / wm.gx) % wm.gy;
  wz = w / (wm.gx * wm.gy);
}

// Block order of the wave-tiled kernels: chunks of 16 consecutive blocks
// (64 wave tiles, neighbours in x) dealt round-robin to the 8 XCDs (the
// hardware sends block b to XCD b % 8).  Neighbouring tiles then share an
// XCD's L2, and at any moment all XCDs work in one band of the mesh; one
// contiguous range per XCD instead measured 188 against 145 us for the CG
// J.v at 257x257x129 (chunks of 8 to 64 blocks measure alike).  Blocks past
// the last whole round of chunks keep their order.
__device__ __forceinline__ int wave_of_block(int b, const WaveMap& wm) {
  constexpr int C = 16;
  const int full = (wm.nblocks / (8 * C)) * 8 * C;
  if (b >= full) return b;
  const int xcd = b & 7, loc = b >> 3;
  return ((loc / C) * 8 + xcd) * C + loc % C;
}

// Tile-major order of the per-element work arrays (Gauss-point coefficients,
// staged permittivity): element (ex, ey, L) of 7 x 7 tile (ex/7, ey/7) goes to
// slot ((L gy + ty) gx + tx) 49 + (ex - 7 tx) + 7 (ey - 7 ty), gx = ceil(nx/7).
// A wave then reads its 49 owned elements of a layer as one contiguous block.
__host__ __device__ __forceinline__ long tile_slot(int ex, int ey, int L, int gx, int gy) {
  const int tx = ex / 7, ty = ey / 7;
  return ((long)L * gy + ty) * gx * 49L + (long)tx * 49 + (ex - 7 * tx) + 7 * (ey - 7 * ty);
}

__host__ __device__ __forceinline__ long tile_slots(int nx, int ny, int nz) {
  return (long)((nx + 6) / 7) * ((ny + 6) / 7) * 49L * (nz - 1);
}

__device__ __forceinline__ int ci(int a, int b, int c) { return a + 2 * b + 4 * c; }

// ---- 1D operators -------------------------------------------------------
template <typename T>
__device__ __forceinline__ void mass1(T u0, T u1, T& o0, T& o1) {
  const T s = T(1) / T(6);
  o0 = (T(2) * u0 + u1) * s;
  o1 = (u0 + T(2) * u1) * s;
}

// out = (sx A(x)M(y)M(z) + sy M(x)A(y)M(z) + sz M(x)M(y)A(z)) v
template <typename T>
__device__ __forceinline__ void stiff_apply(const T v[8], T sx, T sy, T sz, T out[8]) {
  T mz[8], dz[8];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const T u0 = v[ci(a, b, 0)], u1 = v[ci(a, b, 1)];
      mass1(u0, u1, mz[ci(a, b, 0)], mz[ci(a, b, 1)]);
      const T d = u0 - u1;
      dz[ci(a, b, 0)] = d;
      dz[ci(a, b, 1)] = -d;
    }
  T myz[8], t[8];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const T m0 = mz[ci(a, 0, c)], m1 = mz[ci(a, 1, c)];
      mass1(m0, m1, myz[ci(a, 0, c)], myz[ci(a, 1, c)]);
      const T d = m0 - m1;
      T e0, e1;
      mass1(dz[ci(a, 0, c)], dz[ci(a, 1, c)], e0, e1);
      t[ci(a, 0, c)] = sy * d + sz * e0;
      t[ci(a, 1, c)] = -sy * d + sz * e1;
    }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const T d = sx * (myz[ci(0, b, c)] - myz[ci(1, b, c)]);
      T o0, o1;
      mass1(t[ci(0, b, c)], t[ci(1, b, c)], o0, o1);
      out[ci(0, b, c)] = d + o0;
      out[ci(1, b, c)] = -d + o1;
    }
}

// Tensor-product application of [[p, q], [q, p]] along x, y and z (in place).
template <typename T>
__device__ __forceinline__ void tensor_sym(T u[8], T p, T q) {
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const T u0 = u[ci(0, b, c)], u1 = u[ci(1, b, c)];
      u[ci(0, b, c)] = p * u0 + q * u1;
      u[ci(1, b, c)] = q * u0 + p * u1;
    }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const T u0 = u[ci(a, 0, c)], u1 = u[ci(a, 1, c)];
      u[ci(a, 0, c)] = p * u0 + q * u1;
      u[ci(a, 1, c)] = q * u0 + p * u1;
    }
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const T u0 = u[ci(a, b, 0)], u1 = u[ci(a, b, 1)];
      u[ci(a, b, 0)] = p * u0 + q * u1;
      u[ci(a, b, 1)] = q * u0 + p * u1;
    }
}

// Corner values -> Gauss-point values (and, being symmetric, the projection
// sum_q f_q w_a(q) back to the corners).
template <typename T>
__device__ __forceinline__ void gauss_interp(T u[8]) { tensor_sym(u, T(kG1), T(kG0)); }

// sum_q f_q w_a(q)^2 : the Gauss-point weights of the mass diagonal.
template <typename T>
__device__ __forceinline__ void gauss_sq_project(T u[8]) { tensor_sym(u, T(kG1 * kG1), T(kG0 * kG0)); }

// ---- sum/difference (Haar) form of the element Jacobian ---------------------
// With H = [[1, 1], [1, -1]] along each axis (H^-1 = H/2):
//   A = H^-1 diag(0, 2) H,  M = H^-1 diag(1/2, 1/6) H,  B = H^-1 diag(1, 1/sqrt(3)) H,
// so in the basis H3 = H(x)H(y)H(z) the box-element stiffness is diagonal and
// the Gauss-point interpolation is diagonal too.  J_e v = Khat v + B3 (c . B3 v)
// then costs four 8-point transforms, a few scalings and the 8 coefficient
// products, instead of the axis-by-axis matrices above.
template <typename T>
__device__ __forceinline__ void haar3(T u[8]) {
#pragma unroll
  for (int p = 0; p < 8; p += 2) {
    const T a = u[p], b = u[p + 1];
    u[p] = a + b;
    u[p + 1] = a - b;
  }
#pragma unroll
  for (int p = 0; p < 8; p += 4)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const T a = u[p + q], b = u[p + q + 2];
      u[p + q] = a + b;
      u[p + q + 2] = a - b;
    }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const T a = u[q], b = u[q + 4];
    u[q] = a + b;
    u[q + 4] = a - b;
  }
}

// out = (eps Khat + B3 diag(c) B3) v on one box element; sx = eps hy hz / hx,
// sy = eps hx hz / hy, sz = eps hx hy / hz; c may be skipped (insulator).
// With kDot, also returns v^T out, taken in the Haar basis before the last
// transform (H3 is symmetric), so v need not stay live.
template <typename T, bool kDot = false>
__device__ __forceinline__ double jv_element(const T v[8], T sx, T sy, T sz, const T c[8], bool have_c, T out[8]) {
  // Khat diagonal in the Haar basis, times the 1/8 of the final inverse transform
  const T k2 = T(1.0 / 16.0), k6 = T(1.0 / 48.0), k18 = T(1.0 / 144.0);
  T vt[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) vt[k] = v[k];
  haar3(vt);
  out[0] = T(0);
  out[1] = (sx * k2) * vt[1];
  out[2] = (sy * k2) * vt[2];
  out[3] = ((sx + sy) * k6) * vt[3];
  out[4] = (sz * k2) * vt[4];
  out[5] = ((sx + sz) * k6) * vt[5];
  out[6] = ((sy + sz) * k6) * vt[6];
  out[7] = ((sx + sy + sz) * k18) * vt[7];
  if (have_c) {
    // D_B / 8 : (1/sqrt3)^(number of difference axes) / 8
    const T b0 = T(0.125), b1 = T(0.07216878364870322), b2 = T(0.041666666666666664),
            b3 = T(0.024056261216234407);
    const T db[8] = {b0, b1, b1, b2, b1, b2, b2, b3};
    T q[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) q[k] = db[k] * vt[k];
    haar3(q);  // Gauss-point values
#pragma unroll
    for (int k = 0; k < 8; ++k) q[k] *= c[k];
    haar3(q);
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] += db[k] * q[k];
  }
  double d = 0.0;
  if (kDot) {
#pragma unroll
    for (int k = 0; k < 8; ++k) d += (double)vt[k] * (double)out[k];
  }
  haar3(out);
  return d;
}

// Interface-charge / Robin sheets as the kernels see them.  Node (a, b) of
// sheet s (a in [a0, a1], b in [b0, b1]) is base + a*sa + b*sb; ca / cb are
// the coordinates along the two in-plane axes.  The kernels work on a list of
// the distinct sheet nodes (int4: node, sheet | shared << 8, a, b), where
// `sheet` is the first sheet containing the node and `shared` says that a
// later one does too.
constexpr int kMaxSheets = 16;
struct SheetDev {
  int axis, plane;
  int a0, a1, b0, b1;
  long base, sa, sb;
  const double* ca;
  const double* cb;
  const double* sigma;   // [(a1-a0)*(b1-b0)] or NULL
  double alpha;          // robin_eps / robin_d, 0 = no Robin term
  double phi0;
};
struct SheetSet {
  int n;
  int any_robin;
  int n_items;   // distinct sheet nodes (work items)
  SheetDev s[kMaxSheets];
};

// Per-element doping: the net N_D - N_A (complete ionization; NULL = 0, or
// donors - acceptors when only those are given) or the two species.
struct Doping {
  const double* net;
  const double* donors;
  const double* acceptors;
};

// ---- charge statistics ----------------------------------------------------
// Density of one band, N F(u/kT), and its derivative in u, where u is
// E_F minus the band edge (V): Fermi-Dirac uses Bednarczyk's F_1/2 with its
// exact derivative and exp(eta) below eta = -50; Boltzmann is exp; Thomas-
// Fermi is the T -> 0 limit with prefactor C.
__device__ __forceinline__ void band_density(const Charge& ch, double u, double N, double C, double& f,
                                             double& df) {
  if (ch.stat == STAT_TF) {
    const double up = fmax(u, 0.0);
    const double s = sqrt(up);
    f = C * up * s;
    df = 1.5 * C * s;
  } else if (ch.stat == STAT_FD || ch.stat == STAT_MB) {
    const double eta = u * ch.inv_kT;
    if (ch.stat == STAT_MB || eta < -50.0) {
      const double e = exp(eta);
      f = N * e;
      df = N * e * ch.inv_kT;
    } else {
      const double a = 1.3293403881791355;          // 3 sqrt(pi) / 4
      const double xp1 = eta + 1.0;
      const double g = exp(-0.17 * xp1 * xp1);
      const double eta2 = eta * eta;
      const double v = eta2 * eta2 + 50.0 + 33.6 * eta * (1.0 - 0.68 * g);
      const double dv = 4.0 * eta2 * eta + 33.6 * (1.0 - 0.68 * g) + 7.76832 * eta * xp1 * g;
      const double em = exp(-eta);
      const double vp = exp(-0.375 * log(v));          // v^(-3/8)
      const double F = 1.0 / (em + a * vp);
      const double Fp = (em + 0.375 * a * (vp / v) * dv) * F * F;
      f = N * F;
      df = N * Fp * ch.inv_kT;
    }
  } else {
    f = 0.0;
    df = 0.0;
  }
}

// n(phi) and dn/dphi (E_F - E_C = phi - Ec0).
__device__ __forceinline__ void electron_density(const Charge& ch, double phi, double& n, double& dn) {
  band_density(ch, phi - ch.Ec0, ch.Nc, ch.Ctf, n, dn);
}

// 1 / (1 + exp(A)) and its derivative in A, without overflow.
__device__ __forceinline__ void fermi_factor(double A, double& f, double& df) {
  if (A > 0.0) {
    const double e = exp(-A);
    f = e / (1.0 + e);
  } else {
    f = 1.0 / (1.0 + exp(A));
  }
  df = -f * (1.0 - f);
}

// Space charge rho = p - n + N_D+ - N_A- (nm^-3) and drho/dphi at one point
// for a given electron density n and dn/dphi: net = N_D - N_A with complete
// ionization; nd, na per element otherwise.
__device__ __forceinline__ void space_charge_n(const Charge& ch, double phi, double n, double dn, double net,
                                               double nd, double na, double& rho, double& drho) {
  rho = -n;
  drho = -dn;
  if (ch.holes) {
    double p, dp;
    band_density(ch, ch.Ec0 - ch.Eg - phi, ch.Nv, ch.Ctf_h, p, dp);  // u = E_V - E_F
    rho += p;
    drho -= dp;
  }
  if (ch.incomplete) {
    // N_D+ = N_D / (1 + g_D exp((E_F - E_D)/kT)), E_F - E_D = phi - Ec0 + E_d
    double fd, dfd, fa, dfa;
    fermi_factor((phi - ch.Ec0) * ch.inv_kT + ch.ed_kT + ch.ln_gD, fd, dfd);
    // N_A- = N_A / (1 + g_A exp((E_A - E_F)/kT)), E_A - E_F = Ec0 - Eg - phi + E_a
    fermi_factor((ch.Ec0 - ch.Eg - phi) * ch.inv_kT + ch.ea_kT + ch.ln_gA, fa, dfa);
    rho += nd * fd - na * fa;
    drho += (nd * dfd + na * dfa) * ch.inv_kT;
  } else {
    rho += net;
  }
}

// The same with the electrons of the charge statistics.
__device__ __forceinline__ void space_charge(const Charge& ch, double phi, double net, double nd, double na,
                                             double& rho, double& drho) {
  double n, dn;
  electron_density(ch, phi, n, dn);
  space_charge_n(ch, phi, n, dn, net, nd, na, rho, drho);
}

// Predictor-corrector electrons from the eigenstates of an earlier outer
// iteration (Eq. pcPoisson): n~ = sum_i P |psi_i|^2 G(x_i) with
// x_i = (E_F - E_i + (phi - phi^(k)))/kT, E_F = 0.  3D confinement (Eq.
// ApproxEDens3DConfined): P = 4, G = 1/(1 + e^-x); 1D confinement (Eq.
// ApproxEDens1DConfined): P = 2 m_t kT/(pi hbar^2), G = ln(1 + e^x).
constexpr int kMaxStates = 32;
struct Quantum {
  int n;                 // states; 0 = electrons from the statistics
  int conf;              // 3 or 1
  long N;                // stride of psi2 between states
  const double* psi2;    // [n][N] nodal |psi_i|^2
  const double* phik;    // [N] phi^(k)
  const uint8_t* region; // [E] quantum-region elements, NULL = all
  // [n][6] node-index box (i0, i1, j0, j1, k0, k1, inclusive) holding every
  // node where |psi_i|^2 is not zero (empty when i0 > i1); an element outside
  // it gets exactly nothing from state i
  const int* sbox;
  double pref;           // P
  double inv_kT;         // 1/eV
  double E[kMaxStates];  // E_i - E_F, eV
  // 3D confinement with every |E_i/kT| <= kPcExpMax: e^(E_i/kT), so that
  // e^-x_i = e^-y e^(E_i/kT) with one exponential per Gauss point
  int fast;
  double B[kMaxStates];
};
constexpr double kPcExpMax = 300.0;

// G(x) and G'(x) of the confinement's occupation.
__device__ __forceinline__ void pc_occupation(int conf, double x, double& G, double& dG) {
  const double e = exp(-fabs(x));
  const double s = x >= 0.0 ? 1.0 / (1.0 + e) : e / (1.0 + e);   // 1/(1 + e^-x)
  if (conf == 3) {
    G = s;
    dG = s * (1.0 - s);
  } else {
    G = fmax(x, 0.0) + log1p(e);   // ln(1 + e^x)
    dG = s;
  }
}
__device__ __forceinline__ double electron_density_only(const Charge& ch, double phi) {
  double n, dn;
  electron_density(ch, phi, n, dn);
  return n;
}

// Block barrier that orders LDS only: unlike __syncthreads() it does not wait
// for outstanding global loads, so prefetches stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---- reductions -------------------------------------------------------------
// A value known to be the same in every lane, moved to scalar registers.
__device__ __forceinline__ double uniform(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)b);
  const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Lane `idx` (wave-uniform) of v, in scalar registers.
__device__ __forceinline__ double lane_value(double v, int idx) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned int lo = __builtin_amdgcn_readlane((unsigned int)b, idx);
  const unsigned int hi = __builtin_amdgcn_readlane((unsigned int)(b >> 32), idx);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over the block (fixed order); the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sred) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sred[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) r += sred[w];
  }
  __syncthreads();
  return r;
}

// Publishes partial[blockIdx] (already written by thread 0) and reports
// whether this block is the last to finish; the last block then sees every
// partial.  The counter is reset by the caller's last block.
__device__ __forceinline__ bool last_block_done(unsigned int* counter) {
  __shared__ int am_last;
  __threadfence();
  if (threadIdx.x == 0) {
    const unsigned int prev = atomicAdd(counter, 1u);
    am_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (am_last) __threadfence();
  return am_last != 0;
}

// Sum of partial[0..n) in a fixed order by one block; valid in thread 0.
__device__ __forceinline__ double reduce_partials(const double* partial, int n, double* sred) {
  double v = 0.0;
  const volatile double* p = partial;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += p[i];
  return block_sum(v, sred);
}

}  // namespace qe
