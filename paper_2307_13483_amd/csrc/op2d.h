// The operator A = E - H_ef(E) of the generalized two-state model (Sec. II.C,
// Eqs. (18), (21), (23), (28)) applied as a stencil in one symmetry block.
//
// Symmetry blocks.  The operator commutes with s_d (-1)^{n_u} (s_1 = +1,
// s_2 = -1): every coupling either keeps (d, n_u) parity (H_0, k_d q_g,
// (1 + lam_d q_g) F (1 + lam_d q_g)) or flips both d and the parity of n_u
// (lam q_u and the q_u-sandwiches).  Every right-hand side Phi^{v mu} lies in
// one block, so a solve only needs one unknown per (n_g, n_u): at each grid
// point exactly one state is "active".  In block p, state 1 is active where
// n_u + p is even and state 2 where it is odd.  This halves the unknowns and
// the bytes of every vector; the gerade/ungerade split of the spectra
// (Sec. IV) is exactly this decomposition.
//
// With z the block vector, at a point where state d is active (A = d, B = the
// other state) the level-shift term of Eq. (23) reads
//     u_A = (1 + lam_d q_g) z,     u_B = q_u z,
//     (w_A, w_B) = [[F_AA, F_AB], [F_AB, F_BB]] (u_A, u_B)      (pointwise)
//     (F z)      = (1 + lam_d q_g) w_A + q_u w_B,
// where the 2x2 level-shift block is that of the even partial wave where
// state 1 is active and of the odd partial wave where state 2 is active
// (F_AA, F_AB, F_BB) = (F[1e1e], F[1e2e], F[2e2e]) or (F[2o2o], F[1o2o], F[1o1o]).
// Together with the diagonal (E - E_nu - E_d) and the direct couplings
//     y = (E - E_nu - E_d) z - k_d q_g z - lam q_u z - F z.
// q acts as [q w]_n = (sqrt(n) w_{n-1} + sqrt(n+1) w_{n+1}) / sqrt 2,
// truncated at the basis edge (Sec. III).
#pragma once
#include "internal.h"

namespace vdc {

template <typename R> struct CT;
template <> struct CT<double> { using C = c64; };
template <> struct CT<float> { using C = c32; };

template <typename R>
__device__ inline typename CT<R>::C cz() { return typename CT<R>::C{R(0), R(0)}; }

template <typename R>
__device__ inline typename CT<R>::C cfrom(c64 a) { return typename CT<R>::C{R(a.x), R(a.y)}; }

// Per-job view of the operator, precision R.
template <typename R>
struct OpJob {
  using C = typename CT<R>::C;
  int Ng, Nu, Nc, p;
  double dbase0, dbase1;   // E - E_d - (w_g + w_u)/2, by active state (FP64)
  double omega_g, omega_u;
  R kappa0, kappa1, lamd0, lamd1, lam;
  const C* AA;             // level-shift planes of this job's block
  const C* AB;
  const C* BB;
};

// Per-state coefficient by active state a in {0, 1}.  The pairs are kept as
// separate scalars and chosen by a select: a runtime index into an array
// member would keep the whole struct in private (scratch) memory.
template <typename T>
__device__ inline T by_state(T v0, T v1, int a) { return a ? v1 : v0; }

template <typename R>
__device__ inline OpJob<R> make_op(const DevModel& m, const DevJob& jb,
                                   const typename CT<R>::C* table_block) {
  OpJob<R> op;
  op.Ng = m.Ng;
  op.Nu = m.Nu;
  op.Nc = m.Nc;
  op.p = jb.parity;
  const double half = 0.5 * (m.omega_g + m.omega_u);
  op.dbase0 = jb.E - m.E1 - half;
  op.dbase1 = jb.E - m.E2 - half;
  op.omega_g = m.omega_g;
  op.omega_u = m.omega_u;
  op.kappa0 = R(m.kappa[0]);
  op.kappa1 = R(m.kappa[1]);
  op.lamd0 = R(m.lamd[0]);
  op.lamd1 = R(m.lamd[1]);
  op.lam = R(m.lam);
  op.AA = table_block;
  op.AB = table_block + m.Nc;
  op.BB = table_block + 2 * (size_t)m.Nc;
  return op;
}

// sqrt(n/2) for n = 0..kSqMax, filled into LDS once per workgroup.
constexpr int kSqMax = 1024;

template <typename R>
__device__ inline void fill_sq(R* sq) {
  for (int n = threadIdx.x; n <= kSqMax; n += blockDim.x) sq[n] = R(sqrt(0.5 * n));
}

template <typename R>
__device__ inline typename CT<R>::C load_z(const typename CT<R>::C* __restrict__ v,
                                           const typename CT<R>::C* __restrict__ dinv, int j) {
  return dinv ? dinv[j] * v[j] : v[j];
}

// Phase 1 at point i: the local part of y and the pointwise level-shift
// products (w_A, w_B).
template <typename R>
__device__ inline void op_phase1(const OpJob<R>& op, const R* sq, const typename CT<R>::C* v,
                                 const typename CT<R>::C* dinv, int i,
                                 typename CT<R>::C& yloc, typename CT<R>::C& wA,
                                 typename CT<R>::C& wB) {
  using C = typename CT<R>::C;
  const int ng = i / op.Nu, nu = i - ng * op.Nu;
  const int a = (nu + op.p) & 1;
  const C z = load_z<R>(v, dinv, i);
  C zg = cz<R>(), zu = cz<R>();
  if (ng > 0) zg = sq[ng] * load_z<R>(v, dinv, i - op.Nu);
  if (ng + 1 < op.Ng) zg = zg + sq[ng + 1] * load_z<R>(v, dinv, i + op.Nu);
  if (nu > 0) zu = sq[nu] * load_z<R>(v, dinv, i - 1);
  if (nu + 1 < op.Nu) zu = zu + sq[nu + 1] * load_z<R>(v, dinv, i + 1);
  const R d = R(by_state(op.dbase0, op.dbase1, a) - op.omega_g * ng - op.omega_u * nu);
  yloc = d * z - by_state(op.kappa0, op.kappa1, a) * zg - op.lam * zu;
  const C uA = z + by_state(op.lamd0, op.lamd1, a) * zg;
  const C uB = zu;
  const C fab = op.AB[i];
  wA = op.AA[i] * uA + fab * uB;
  wB = fab * uA + op.BB[i] * uB;
}

// Phase 2 at point i: y = yloc - (1 + lam_d q_g) w_A - q_u w_B.
template <typename R>
__device__ inline typename CT<R>::C op_phase2(const OpJob<R>& op, const R* sq,
                                              const typename CT<R>::C* __restrict__ wA,
                                              const typename CT<R>::C* __restrict__ wB, int i,
                                              typename CT<R>::C yloc) {
  using C = typename CT<R>::C;
  const int ng = i / op.Nu, nu = i - ng * op.Nu;
  const int a = (nu + op.p) & 1;
  C g = cz<R>(), u = cz<R>();
  if (ng > 0) g = sq[ng] * wA[i - op.Nu];
  if (ng + 1 < op.Ng) g = g + sq[ng + 1] * wA[i + op.Nu];
  if (nu > 0) u = sq[nu] * wB[i - 1];
  if (nu + 1 < op.Nu) u = u + sq[nu + 1] * wB[i + 1];
  return yloc - wA[i] - by_state(op.lamd0, op.lamd1, a) * g - u;
}

// Diagonal of A at point i (the M^{dg} preconditioner of Sec. III.B):
// D = E - E_nu - E_d - F_AA(nu) - lam_d^2 sum_{nu' = nu +- g} (q_g)^2 F_AA(nu')
//     - sum_{nu' = nu +- u} (q_u)^2 F_BB(nu'),
// the neighbours nu +- u carrying the other state's entry in their BB slot.
template <typename R>
__device__ inline typename CT<R>::C op_diag(const OpJob<R>& op, int i) {
  using C = typename CT<R>::C;
  const int ng = i / op.Nu, nu = i - ng * op.Nu;
  const int a = (nu + op.p) & 1;
  const R d = R(by_state(op.dbase0, op.dbase1, a) - op.omega_g * ng - op.omega_u * nu);
  C s = op.AA[i];
  C sg = cz<R>();
  if (ng > 0) sg = R(0.5 * ng) * op.AA[i - op.Nu];
  if (ng + 1 < op.Ng) sg = sg + R(0.5 * (ng + 1)) * op.AA[i + op.Nu];
  s = s + (by_state(op.lamd0, op.lamd1, a) * by_state(op.lamd0, op.lamd1, a)) * sg;
  if (nu > 0) s = s + R(0.5 * nu) * op.BB[i - 1];
  if (nu + 1 < op.Nu) s = s + R(0.5 * (nu + 1)) * op.BB[i + 1];
  return C{d - s.x, -s.y};
}

template <typename R>
__device__ inline typename CT<R>::C cinv(typename CT<R>::C a) {
  const R n = a.x * a.x + a.y * a.y;
  return typename CT<R>::C{a.x / n, -a.y / n};
}

// Width Gamma_d^mu(eps) and the coupling f = sqrt(Gamma / 2 pi) (Eq. (22)).
__device__ inline double coupling_f(const DevModel& m, int d, int mu, double eps) {
  if (!(eps > 0.0)) return 0.0;
  const double G = m.A[d][mu] * pow(eps, m.l[mu] + 0.5) * exp(-eps / m.B[d][mu]);
  return sqrt(G / (2.0 * kPi));
}

// Nonzero components of Phi^{v mu} = f_d^mu(eps) <nu|O_d^mu|v> (Eq. (25)), with
// O_1^e = 1 + lam_1 q_g, O_2^e = q_u, O_1^o = q_u, O_2^o = 1 + lam_2 q_g.
// Writes up to 6 entries (state index d in {0,1}, n_g, n_u, value).
struct PhiEntry { int d, g, u; double val; };

__device__ inline int phi_entries(const DevModel& m, int mu, double eps, int g, int u,
                                  PhiEntry* e) {
  int n = 0;
  for (int d = 0; d < 2; ++d) {
    const double f = coupling_f(m, d, mu, eps);
    if (f == 0.0) continue;
    const bool G = (d == mu);   // (1,e) and (2,o) carry 1 + lam_d q_g
    if (G) {
      e[n++] = PhiEntry{d, g, u, f};
      if (g + 1 < m.Ng) e[n++] = PhiEntry{d, g + 1, u, f * m.lamd[d] * sqrt(0.5 * (g + 1))};
      if (g > 0) e[n++] = PhiEntry{d, g - 1, u, f * m.lamd[d] * sqrt(0.5 * g)};
    } else {
      if (u + 1 < m.Nu) e[n++] = PhiEntry{d, g, u + 1, f * sqrt(0.5 * (u + 1))};
      if (u > 0) e[n++] = PhiEntry{d, g, u - 1, f * sqrt(0.5 * u)};
    }
  }
  return n;
}

// Symmetry block of Phi^{v mu}: state 1 sits on n_u = v_u (mu = e) or v_u +- 1.
__host__ __device__ inline int block_parity(int vi_u, int mu) { return (vi_u + mu) & 1; }

}  // namespace vdc
