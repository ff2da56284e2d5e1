// The general model of the class (Sec. II.A-C) given by polynomial term
// lists: D discrete states, M modes, P partial waves.  Device form of the
// model and the per-point stencil arithmetic shared by the operator kernel
// and the batched solver (terms.hip) and the level-shift plane kernel.
//
// Layout: a vector holds D blocks of npts = prod_k n_k points, point index
// i = ((n_0 n_1 + n_1') ...) with the last mode fastest.
//
// Every monomial c prod_k q_k^p_k is the Kronecker product of the powers of
// the truncated coordinate (P q P)^p (products of truncated matrices), a
// banded matrix per mode; its rows are tabulated (qtab: row n of mode k's
// p-th power, columns n + delta for delta = -4..4).  An operator (a block
// U_dd' of the direct coupling, or a discrete-continuum factor O_d^mu) is
// compiled on the host into stencil points: the distinct offset vectors
// delta of its monomials, each with the monomials that reach it; at output
// point n its coefficient is sum_t c_t prod_k (P q_k P)^{p_tk}[n_k][n_k + delta_k].
// Every such matrix is symmetric, so the coefficient of O at (n, n + delta)
// is also that of O^T and of O at (n + delta, n).
//
// A x at total energy E (Eqs. (18), (21), (23), (28)):
//   u_d^mu   = O_d^mu x_d                      (stencil)
//   w_d^mu   = sum_d' F^mu_dd'(eps_nu) u_d'^mu  (pointwise, eps_nu = E - E_nu)
//   (A x)_d  = (E - E_nu - E_d) x_d - sum_d' U_dd' x_d' - sum_mu (O_d^mu)^T w_d^mu.
#pragma once
#include "internal.h"

namespace vdc {

constexpr int kGenMaxStates = 4;
constexpr int kGenMaxModes = 8;
constexpr int kGenMaxWaves = 4;
constexpr int kGenMaxPow = 4;
constexpr int kGenQW = 2 * kGenMaxPow + 1;   // tabulated offsets per row

// One monomial: coefficient and the power of each mode.
struct GenTerm {
  double c;
  signed char pw[kGenMaxModes];
};

// One stencil point of an operator: flat offset, per-mode offsets and the
// range of its monomials in the term array.
struct GenPoint {
  int off;
  int t0, nt;
  int zero;                       // all offsets are 0 (the diagonal)
  signed char dl[kGenMaxModes];
};

struct GenOp {
  int p0, np;                     // range of points; np = 0: the operator is 0
};

// Per-model data of the kernels (host-filled; pointers to device arrays the
// model owns).
struct DevGen {
  int D, M, P, npts;
  int n[kGenMaxModes];
  int stride[kGenMaxModes];
  double omega[kGenMaxModes];
  double e_state[kGenMaxStates];
  double A[kGenMaxStates][kGenMaxWaves], B[kGenMaxStates][kGenMaxWaves];
  int l[kGenMaxWaves];
  GenOp uop[kGenMaxStates][kGenMaxStates];   // U_dd' (both orders)
  GenOp vop[kGenMaxStates][kGenMaxWaves];    // O_d^mu
  // level-shift plane of F^mu_dd' in an energy's table (both orders), -1: 0
  int fplane[kGenMaxWaves][kGenMaxStates][kGenMaxStates];
  int nplanes;
  // plane of w_d^mu in the work array, -1 where O_d^mu = 0
  int wplane[kGenMaxWaves][kGenMaxStates];
  int nw;
  const double* qtab;             // rows of (P q P)^p per mode and power
  int qoff[kGenMaxModes];         // start of mode k's [p][n][kGenQW] block
  const GenPoint* pts;
  const GenTerm* terms;
  const double* Enu;              // [npts] E_nu of each point
  // level-shift transform: models of two states each (see the planes kernel)
  const DevModel* lsm;
  const int* lsmap;               // [nlsm][kNumF] -> plane, or -1
  int nlsm;
  const int* perm;                // points in order of E_nu
};

// Multi-index of point i.
__device__ inline void gen_index(const DevGen& g, int i, int* nk) {
  for (int k = g.M - 1; k >= 0; --k) {
    const int q = i / g.n[k];
    nk[k] = i - q * g.n[k];
    i = q;
  }
}

// Coefficient of stencil point pt at the output point with multi-index nk;
// false when the neighbour n + delta lies outside the basis.
__device__ inline bool gen_coef(const DevGen& g, const GenPoint& pt, const int* nk, double& c) {
  for (int k = 0; k < g.M; ++k) {
    const int m = nk[k] + pt.dl[k];
    if (m < 0 || m >= g.n[k]) return false;
  }
  double s = 0.0;
  for (int t = pt.t0; t < pt.t0 + pt.nt; ++t) {
    const GenTerm tm = g.terms[t];
    double v = tm.c;
    for (int k = 0; k < g.M; ++k)
      v *= g.qtab[g.qoff[k] + ((size_t)tm.pw[k] * g.n[k] + nk[k]) * kGenQW + pt.dl[k] + kGenMaxPow];
    s += v;
  }
  c = s;
  return true;
}

// (Op v)(i) for the operator op on one block of v (npts points).
__device__ inline c64 gen_stencil(const DevGen& g, const GenOp& op, const int* nk, int i,
                                  const c64* __restrict__ v) {
  c64 acc{0.0, 0.0};
  for (int q = op.p0; q < op.p0 + op.np; ++q) {
    const GenPoint pt = g.pts[q];
    double c;
    if (gen_coef(g, pt, nk, c)) acc = acc + c * v[i + pt.off];
  }
  return acc;
}

// Pass 1 at point i: w_d^mu(i) for every (mu, d) with O_d^mu != 0.
// F: the energy's level-shift planes [nplanes][npts]; x: [D][npts].
__device__ inline void gen_pass1(const DevGen& g, const c64* __restrict__ F,
                                 const c64* __restrict__ x, c64* __restrict__ w, int i) {
  int nk[kGenMaxModes];
  gen_index(g, i, nk);
  for (int mu = 0; mu < g.P; ++mu) {
    c64 u[kGenMaxStates];
    for (int d = 0; d < kGenMaxStates; ++d) u[d] = c64{0.0, 0.0};
    for (int d = 0; d < g.D; ++d)
      if (g.vop[d][mu].np) u[d] = gen_stencil(g, g.vop[d][mu], nk, i, x + (size_t)d * g.npts);
    for (int d = 0; d < g.D; ++d) {
      const int wp = g.wplane[mu][d];
      if (wp < 0) continue;
      c64 s{0.0, 0.0};
      for (int e = 0; e < g.D; ++e) {
        const int fp = g.fplane[mu][d][e];
        if (fp >= 0) s = s + F[(size_t)fp * g.npts + i] * u[e];
      }
      w[(size_t)wp * g.npts + i] = s;
    }
  }
}

// Pass 2 at point i: (A x)_d(i) for every state d into y.
__device__ inline void gen_pass2(const DevGen& g, double E, const c64* __restrict__ x,
                                 const c64* __restrict__ w, c64* __restrict__ y, int i) {
  int nk[kGenMaxModes];
  gen_index(g, i, nk);
  const double Ev = g.Enu[i];
  for (int d = 0; d < g.D; ++d) {
    c64 s = (E - Ev - g.e_state[d]) * x[(size_t)d * g.npts + i];
    for (int e = 0; e < g.D; ++e)
      if (g.uop[d][e].np) s = s - gen_stencil(g, g.uop[d][e], nk, i, x + (size_t)e * g.npts);
    for (int mu = 0; mu < g.P; ++mu) {
      const int wp = g.wplane[mu][d];
      if (wp >= 0) s = s - gen_stencil(g, g.vop[d][mu], nk, i, w + (size_t)wp * g.npts);
    }
    y[(size_t)d * g.npts + i] = s;
  }
}

// Diagonal of A at (d, i):  E - E_nu - E_d - U_dd(i, i)
//   - sum_mu sum_delta O_d^mu(i + delta, i)^2 F^mu_dd(i + delta).
__device__ inline c64 gen_diag(const DevGen& g, double E, const c64* __restrict__ F, int d, int i) {
  int nk[kGenMaxModes];
  gen_index(g, i, nk);
  double re = E - g.Enu[i] - g.e_state[d];
  const GenOp& u = g.uop[d][d];
  for (int q = u.p0; q < u.p0 + u.np; ++q) {
    const GenPoint pt = g.pts[q];
    double c;
    if (pt.zero && gen_coef(g, pt, nk, c)) re -= c;
  }
  c64 s{re, 0.0};
  for (int mu = 0; mu < g.P; ++mu) {
    const int fp = g.fplane[mu][d][d];
    if (fp < 0 || !g.vop[d][mu].np) continue;
    const GenOp& o = g.vop[d][mu];
    for (int q = o.p0; q < o.p0 + o.np; ++q) {
      const GenPoint pt = g.pts[q];
      double c;
      if (gen_coef(g, pt, nk, c)) s = s - (c * c) * F[(size_t)fp * g.npts + i + pt.off];
    }
  }
  return s;
}

// f_d^mu(eps) = sqrt(Gamma / 2 pi), Gamma = A eps^(l + 1/2) exp(-eps/B) (Eq. (22)).
__host__ __device__ inline double gen_f(const DevGen& g, int d, int mu, double eps) {
  if (!(eps > 0.0) || !(g.A[d][mu] > 0.0)) return 0.0;
  const double G = g.A[d][mu] * pow(eps, g.l[mu] + 0.5) * exp(-eps / g.B[d][mu]);
  return sqrt(G / (2.0 * kPi));
}

// Flat index of multi-index v, or -1 outside the basis.
__host__ __device__ inline int gen_flat(const DevGen& g, const int* v) {
  int i = 0;
  for (int k = 0; k < g.M; ++k) {
    if (v[k] < 0 || v[k] >= g.n[k]) return -1;
    i = i * g.n[k] + v[k];
  }
  return i;
}

__host__ __device__ inline double gen_vib_energy(const DevGen& g, const int* v) {
  double e = 0.0;
  for (int k = 0; k < g.M; ++k) e += g.omega[k] * (v[k] + 0.5);
  return e;
}

// Amplitude T^mu_f = Phi^{v_f mu T} psi = sum_d f_d^mu(E - E_vf) (O_d^mu psi_d)(v_f)
// (Eqs. (24), (25)); psi: [D][npts].
__device__ inline c64 gen_amplitude(const DevGen& g, double E, const int* vf, int mu,
                                    const c64* __restrict__ psi) {
  const int i = gen_flat(g, vf);
  if (i < 0) return c64{0.0, 0.0};
  const double eps = E - gen_vib_energy(g, vf);
  c64 T{0.0, 0.0};
  for (int d = 0; d < g.D; ++d) {
    const double f = gen_f(g, d, mu, eps);
    if (f == 0.0 || !g.vop[d][mu].np) continue;
    T = T + f * gen_stencil(g, g.vop[d][mu], vf, i, psi + (size_t)d * g.npts);
  }
  return T;
}

}  // namespace vdc
