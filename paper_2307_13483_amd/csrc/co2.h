// The CO2-like three-state, four-mode model on the device: the operator
// A = E - H_0 - U - F of Sec. III.C's model class (three discrete states
// sigma, Pi_x, Pi_y; modes s, bend x and y, a; partial waves s, p_x, p_y;
// couplings up to second order), applied in one reflection sector, and the
// paper's preconditioner for this class: one block per (n_s, n_a) holding the
// whole bend plane, factored by complex-symmetric L D L^T.
//
// Reflection sectors.  A commutes with the reflections x -> -x and y -> -y
// (q_x, Pi_x and p_x change sign under the first, q_y, Pi_y and p_y under the
// second), and every right-hand side lies in one sector (px, py): the
// sector's eigenvalues are (-1)^{v_x + [mu = p_x]} and (-1)^{v_y + [mu = p_y]}.
// In a sector every bend point (n_x, n_y) carries at most one state, fixed
// by the parities t_x = (n_x + px) & 1, t_y = (n_y + py) & 1:
//   (0, 0) sigma, (1, 0) Pi_x, (0, 1) Pi_y, (1, 1) none.
// A vector is one complex value per point of the grid [n_s][n_a][n_x][n_y]
// (n_y fastest), zero at the "none" points: three quarters of the grid carry
// a state, a quarter of the full basis of three states.  The continuum channel that can reach a point is fixed by
// its type as well: the s wave at sigma points, p_x at Pi_x points, p_y at
// Pi_y points, so the level-shift sandwich has exactly two pointwise
// components per point (a sigma part w_A and a Pi part w_B), as in the
// two-state model:
//   sigma point:  u_A = (1 + l_s q_s) z,  u_B = h_p (q_x + q_y) z   (F^s)
//   Pi_x point:   u_A = h_s q_x z,        u_B = (1 + l_p q_s) z      (F^p)
//   Pi_y point:   u_A = h_s q_y z,        u_B = (1 + l_p q_s) z      (F^p)
//   (w_A, w_B) = [[F_ss, F_sp], [F_sp, F_pp]] (u_A, u_B),
// and F z is the transposed sandwich of the neighbours' (w_A, w_B).  q acts
// as [q w]_n = sqrt(n/2) w_{n-1} + sqrt((n+1)/2) w_{n+1} and q^2 is the
// product of two truncated q.
//
// Level shift.  The six functions F[f_d f_d'] (state classes sigma, Pi; wave
// classes s, p) depend on a point only through eps_nu = E - E_nu, and E_nu
// through (n_s, n_x + n_y, n_a): one table row per such triple and energy.
#pragma once
#include "internal.h"

namespace vdc {

struct Co2Model {
  int Ns, Nx, Ny, Na;
  int npts;              // Ns * Na * Nx * Ny
  int nb;                // Nx + Ny - 1 values of n_x + n_y
  int ntab;              // Ns * nb * Na table rows per energy
  double omega_s, omega_b, omega_a;
  double E_sigma, E_pi;
  double k_sigma, k_pi;
  double gs[2], gb[2], ga[2];   // [0] sigma, [1] Pi
  double c_rt, c_sp, c_sp2;
  double l_sigma, l_pi, h_sigma, h_pi;
};

struct Co2Job {
  double eps_i, E;
  int v[4];              // initial state (n_s, n_x, n_y, n_a)
  int mu;                // 0 s, 1 p_x, 2 p_y
  int px, py;            // sector bits
  int table;             // index of the job's energy in the table array
  int out;               // index in the caller's arrays
};

__host__ __device__ inline int co2_type(int x, int y, int px, int py) {
  return ((x + px) & 1) | (((y + py) & 1) << 1);
}

__host__ __device__ inline int co2_sector_x(const int* v, int mu) { return (v[1] + (mu == 1)) & 1; }
__host__ __device__ inline int co2_sector_y(const int* v, int mu) { return (v[2] + (mu == 2)) & 1; }

// c ? a : b on complex values, component by component (keeps the choice a
// choice of values, never of the addresses they were read from)
__device__ __forceinline__ c64 co2_sel(bool c, c64 a, c64 b) {
  return c64{c ? a.x : b.x, c ? a.y : b.y};
}

// A model coefficient as a wavefront-uniform value.  Choices between two
// coefficients by a lane's class are made between such values: a choice
// between the fields themselves is compiled into a per-lane choice of
// address and a vector load.
__device__ inline double co2_uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ inline double co2_pick(bool first, double a, double b) {
  return first ? co2_uniform(a) : co2_uniform(b);
}

// (q^2)_{n n} and (q^2)_{n, n+2} of the truncated product
__device__ inline double q2_diag(int n, int N) { return 0.5 * n + (n + 1 < N ? 0.5 * (n + 1) : 0.0); }

// The bend-mode weights of a point (n_x, n_y) = (x, y), from sq[n] = sqrt(n/2):
// of q_x at x - 1, x + 1 (xl, xh), of q_x^2 at x - 2, x + 2 (x2l, x2h) and
// its diagonal x2d; the same along n_y.  Zero where the neighbour lies past
// the basis edge.  Co2BendSq reads each from the table where it is used;
// Co2BendW holds them (the march keeps them in registers).
struct Co2BendSq {
  const double* sq;
  int x, y, Nx, Ny;
  __device__ double xl() const { return sq[x > 0 ? x : 0]; }
  __device__ double xh() const { return sq[x + 1 < Nx ? x + 1 : 0]; }
  __device__ double yl() const { return sq[y > 0 ? y : 0]; }
  __device__ double yh() const { return sq[y + 1 < Ny ? y + 1 : 0]; }
  __device__ double x2l() const { return sq[x >= 2 ? x - 1 : 0] * sq[x >= 2 ? x : 0]; }
  __device__ double x2h() const { return sq[x + 2 < Nx ? x + 1 : 0] * sq[x + 2 < Nx ? x + 2 : 0]; }
  __device__ double y2l() const { return sq[y >= 2 ? y - 1 : 0] * sq[y >= 2 ? y : 0]; }
  __device__ double y2h() const { return sq[y + 2 < Ny ? y + 1 : 0] * sq[y + 2 < Ny ? y + 2 : 0]; }
  __device__ double x2d() const { return q2_diag(x, Nx); }
  __device__ double y2d() const { return q2_diag(y, Ny); }
};

struct Co2BendW {
  double w[10];
  __device__ explicit Co2BendW(const Co2BendSq& b)
      : w{b.xl(), b.xh(), b.yl(), b.yh(), b.x2l(), b.x2h(), b.y2l(), b.y2h(), b.x2d(), b.y2d()} {}
  __device__ double xl() const { return w[0]; }
  __device__ double xh() const { return w[1]; }
  __device__ double yl() const { return w[2]; }
  __device__ double yh() const { return w[3]; }
  __device__ double x2l() const { return w[4]; }
  __device__ double x2h() const { return w[5]; }
  __device__ double y2l() const { return w[6]; }
  __device__ double y2h() const { return w[7]; }
  __device__ double x2d() const { return w[8]; }
  __device__ double y2d() const { return w[9]; }
};

struct Co2Point {
  int s, a, x, y, t;
};

__device__ inline Co2Point co2_point(const Co2Model& m, int i) {
  Co2Point p;
  p.y = i % m.Ny;
  int r = i / m.Ny;
  p.x = r % m.Nx;
  r /= m.Nx;
  p.a = r % m.Na;
  p.s = r / m.Na;
  p.t = 0;
  return p;
}

// One job's operator: model, sector, energy, table rows of its energy.
struct Co2Op {
  const Co2Model* m;
  const c64* tab;        // [Ns][nb][Na][6]
  double E;
  int px, py;
};

// Level-shift value at point (s, x, y, a) for the wave class of point type t
// and pair k (0: sigma sigma, 1: sigma Pi, 2: Pi Pi).
__device__ inline c64 co2_tab(const Co2Op& o, int s, int x, int y, int a, int t, int k) {
  const Co2Model& m = *o.m;
  const int w = t == 0 ? 0 : 1;
  return o.tab[((size_t)(s * m.nb + x + y) * m.Na + a) * kNumF + 3 * w + k];
}

// The operator at one point is branch-free in its memory accesses: every
// neighbour is loaded unconditionally, from the point itself where the
// neighbour lies past the basis edge, and weighted by zero there (the
// weights are sqrt(n/2) read at index 0 = 0), so that all loads of a point
// can be in flight together.  Terms are added in the same order as a
// branchy evaluation would add them (a skipped term adds zero).
//
// The point arithmetic takes its neighbours from an accessor: z(ok, ds, da,
// dx, dy) is vs v at the point offset by (ds, da, dx, dy) in (n_s, n_a, n_x,
// n_y) when ok, else at the point itself; w(ok, ds, dx, dy) the level-shift
// product of the point's own channel class (w_A at a sigma point, w_B at a Pi
// point) at the offset point, else at the point itself; tab(o, p, t, k) the
// level-shift value co2_tab at the point; pick(first, a, b) and cls(c2, c)
// one of two model coefficients by the point's class; bend(sq, m, p) the
// point's bend-mode weights (Co2BendSq or Co2BendW).  Co2Flat reads a whole
// vector and its w planes from memory.
struct Co2Flat {
  const c64* v;
  double vs;
  const c64* wc;             // w_A or w_B, by the point's class (phase 2)
  int i, ss, sa, sx, sy;
  __device__ c64 z(bool ok, int ds, int da, int dx, int dy) const {
    return vs * v[ok ? i + ds * ss + da * sa + dx * sx + dy * sy : i];
  }
  __device__ c64 w(bool ok, int ds, int dx, int dy) const {
    return wc[ok ? i + ds * ss + dx * sx + dy * sy : i];
  }
  __device__ c64 tab(const Co2Op& o, const Co2Point& p, int t, int k) const {
    return co2_tab(o, p.s, p.x, p.y, p.a, t, k);
  }
  __device__ double pick(bool first, double a, double b) const { return first ? a : b; }
  __device__ double cls(const double* c2, int c) const { return c2[c]; }
  __device__ Co2BendSq bend(const double* sq, const Co2Model& m, const Co2Point& p) const {
    return Co2BendSq{sq, p.x, p.y, m.Nx, m.Ny};
  }
};

// Phase 1 at point p: the pointwise level-shift products (w_A, w_B) of the
// channel that reaches the point.
template <typename Acc>
__device__ inline void co2_point1(const Co2Op& o, const double* sq, const Acc& Z, const Co2Point& p,
                                  c64& wa, c64& wb) {
  const Co2Model& m = *o.m;
  const int t = co2_type(p.x, p.y, o.px, o.py);
  // sqrt(n/2) z(n - 1) + sqrt((n + 1)/2) z(n + 1) along one mode
  const bool slo = p.s > 0, shi = p.s + 1 < m.Ns, xlo = p.x > 0, xhi = p.x + 1 < m.Nx;
  const bool ylo = p.y > 0, yhi = p.y + 1 < m.Ny;
  const auto W = Z.bend(sq, m, p);
  const c64 z0 = Z.z(true, 0, 0, 0, 0);
  const c64 qs = sq[slo ? p.s : 0] * Z.z(slo, -1, 0, 0, 0) + sq[shi ? p.s + 1 : 0] * Z.z(shi, 1, 0, 0, 0);
  const c64 qx = W.xl() * Z.z(xlo, 0, 0, -1, 0) + W.xh() * Z.z(xhi, 0, 0, 1, 0);
  const c64 qy = W.yl() * Z.z(ylo, 0, 0, 0, -1) + W.yh() * Z.z(yhi, 0, 0, 0, 1);
  const int tt = t == 3 ? 0 : t;
  const c64 T0 = Z.tab(o, p, tt, 0);
  const c64 T1 = Z.tab(o, p, tt, 1);
  const c64 T2 = Z.tab(o, p, tt, 2);
  const c64 us = t == 0 ? z0 + m.l_sigma * qs : m.h_sigma * (t == 1 ? qx : qy);
  const c64 up = t == 0 ? m.h_pi * (qx + qy) : z0 + m.l_pi * qs;
  wa = T0 * us + T1 * up;
  wb = T1 * us + T2 * up;
  if (t == 3) wa = wb = c64{0.0, 0.0};
}

// Phase 2 at point p: y = (E - E_nu) z - U z - F z.
template <typename Acc>
__device__ inline c64 co2_point2(const Co2Op& o, const double* sq, const Acc& Z, const Co2Point& p) {
  const Co2Model& m = *o.m;
  const int t = co2_type(p.x, p.y, o.px, o.py);
  const int s = p.s, a = p.a, x = p.x, y = p.y;
  const c64 z0 = Z.z(true, 0, 0, 0, 0);
  const int c = t == 0 ? 0 : 1;
  const double rt = t == 0 ? 0.0 : Z.pick(t == 1, m.c_rt, -m.c_rt);
  // diagonal-state polynomial: E_d + k q_s + g_s q_s^2 + (g_b + rt) q_x^2 + (g_b - rt) q_y^2 + g_a q_a^2
  const bool s_lo = s > 0, s_hi = s + 1 < m.Ns;
  const double ws_lo = sq[s_lo ? s : 0], ws_hi = sq[s_hi ? s + 1 : 0];
  const c64 qs1 = ws_lo * Z.z(s_lo, -1, 0, 0, 0) + ws_hi * Z.z(s_hi, 1, 0, 0, 0);
  // (q^2 z) along mode k: n, its basis size N, unit offset (ds, da, dx, dy)
  auto q2 = [&](int n, int N, int us, int ua, int ux, int uy) {
    const bool lo = n >= 2, hi = n + 2 < N;
    return q2_diag(n, N) * z0 + (sq[lo ? n - 1 : 0] * sq[lo ? n : 0]) * Z.z(lo, -2 * us, -2 * ua, -2 * ux, -2 * uy) +
           (sq[hi ? n + 1 : 0] * sq[hi ? n + 2 : 0]) * Z.z(hi, 2 * us, 2 * ua, 2 * ux, 2 * uy);
  };
  // the same along a bend mode, with the point's bend weights
  const auto W = Z.bend(sq, m, p);
  auto q2b = [&](double d, double wl, double wh, bool lo, bool hi, int ux, int uy) {
    return d * z0 + wl * Z.z(lo, 0, 0, -2 * ux, -2 * uy) + wh * Z.z(hi, 0, 0, 2 * ux, 2 * uy);
  };
  const double gs = Z.cls(m.gs, c), gb = Z.cls(m.gb, c), ga = Z.cls(m.ga, c);
  c64 U = Z.pick(c == 0, m.E_sigma, m.E_pi) * z0 + Z.pick(c == 0, m.k_sigma, m.k_pi) * qs1 +
          gs * q2(s, m.Ns, 1, 0, 0, 0) + (gb + rt) * q2b(W.x2d(), W.x2l(), W.x2h(), x >= 2, x + 2 < m.Nx, 1, 0) +
          (gb - rt) * q2b(W.y2d(), W.y2l(), W.y2h(), y >= 2, y + 2 < m.Ny, 0, 1) + ga * q2(a, m.Na, 0, 1, 0, 0);
  // sigma - Pi couplings c (1 + c' q_s) q_x and c (1 + c' q_s) q_y, at the
  // point's s - 1, s, s + 1
  const bool x_lo = x > 0, x_hi = x + 1 < m.Nx, y_lo = y > 0, y_hi = y + 1 < m.Ny;
  const double wx_lo = W.xl(), wx_hi = W.xh(), wy_lo = W.yl(), wy_hi = W.yh();
  auto qx_at = [&](bool ok, int ds) {
    return wx_lo * Z.z(ok && x_lo, ds, 0, -1, 0) + wx_hi * Z.z(ok && x_hi, ds, 0, 1, 0);
  };
  auto qy_at = [&](bool ok, int ds) {
    return wy_lo * Z.z(ok && y_lo, ds, 0, 0, -1) + wy_hi * Z.z(ok && y_hi, ds, 0, 0, 1);
  };
  const c64 cx = m.c_sp * (qx_at(true, 0) + m.c_sp2 * (ws_lo * qx_at(s_lo, -1) + ws_hi * qx_at(s_hi, 1)));
  const c64 cy = m.c_sp * (qy_at(true, 0) + m.c_sp2 * (ws_lo * qy_at(s_lo, -1) + ws_hi * qy_at(s_hi, 1)));
  // Pi_x - Pi_y: 2 c_rt q_x q_y
  const c64 xy = (wx_lo * wy_lo) * Z.z(x_lo && y_lo, 0, 0, -1, -1) + (wx_lo * wy_hi) * Z.z(x_lo && y_hi, 0, 0, -1, 1) +
                 (wx_hi * wy_lo) * Z.z(x_hi && y_lo, 0, 0, 1, -1) + (wx_hi * wy_hi) * Z.z(x_hi && y_hi, 0, 0, 1, 1);
  U = t == 0 ? (U + cx) + cy : (U + (t == 1 ? cx : cy)) + (2.0 * m.c_rt) * xy;
  // F z: transposed sandwich of the neighbours' (w_A, w_B)
  const c64 sl = ws_lo * Z.w(s_lo, -1, 0, 0) + ws_hi * Z.w(s_hi, 1, 0, 0);
  const c64 rx = wx_lo * Z.w(x_lo, 0, -1, 0) + wx_hi * Z.w(x_hi, 0, 1, 0);
  const c64 ry = wy_lo * Z.w(y_lo, 0, 0, -1) + wy_hi * Z.w(y_hi, 0, 0, 1);
  c64 Fz = Z.w(true, 0, 0, 0) + Z.pick(t == 0, m.l_sigma, m.l_pi) * sl;
  if (t == 0 || t == 1) Fz = Fz + Z.pick(t == 0, m.h_sigma, m.h_pi) * rx;
  if (t == 0 || t == 2) Fz = Fz + Z.pick(t == 0, m.h_sigma, m.h_pi) * ry;
  const double Ev = m.omega_s * (s + 0.5) + m.omega_b * (x + y + 1.0) + m.omega_a * (a + 0.5);
  const c64 out = (o.E - Ev) * z0 - U - Fz;
  return t == 3 ? c64{0.0, 0.0} : out;
}

// The two phases at flat point i of a vector v in memory (wA, wB its w planes).
__device__ inline void co2_phase1(const Co2Op& o, const double* sq, const c64* v, double vs,
                                  int i, c64& wa, c64& wb) {
  const Co2Model& m = *o.m;
  const Co2Flat Z{v, vs, nullptr, i, m.Na * m.Nx * m.Ny, m.Nx * m.Ny, m.Ny, 1};
  co2_point1(o, sq, Z, co2_point(m, i), wa, wb);
}

__device__ inline c64 co2_phase2(const Co2Op& o, const double* sq, const c64* v, double vs,
                                 const c64* wA, const c64* wB, int i) {
  const Co2Model& m = *o.m;
  const Co2Point p = co2_point(m, i);
  const int t = co2_type(p.x, p.y, o.px, o.py);
  const Co2Flat Z{v, vs, t == 0 ? wA : wB, i, m.Na * m.Nx * m.Ny, m.Nx * m.Ny, m.Ny, 1};
  return co2_point2(o, sq, Z, p);
}

// y = A (vs v) over the whole vector by one workgroup; wA, wB are scratch
// vectors.  Begins with a barrier (v may have just been written by other
// threads) and ends with one.  With red given, also returns ||y||^2 (to every
// thread) and with bsub, y = bsub - A (vs v); with bdot given as well,
// bdot[0..1] receives sum_i (vs v_i) y_i (the bilinear form, no conjugate).
__device__ inline double co2_apply(const Co2Op& o, const double* sq, const c64* v, double vs,
                                   c64* y, c64* wA, c64* wB, const c64* bsub = nullptr,
                                   double* red = nullptr, double* bdot = nullptr);

// One job's block factor storage in bytes, for planes of n points and W1 =
// 2 Ny + 1: L by columns (F) and by rows (G), complex FP16 [planes][n][W1];
// 1/D, complex FP32 [planes][n]; the band staging of the factor kernel,
// complex FP32 [planes][n][7]; 256 bytes of padding.
struct Co2FacLayout {
  size_t F, G, Dinv, S, total;
};

__host__ __device__ inline Co2FacLayout co2_fac_layout(int planes, int n, int W1) {
  Co2FacLayout l;
  const size_t pn = (size_t)planes * n;
  l.F = 0;
  l.G = l.F + pn * W1 * sizeof(c16);
  l.Dinv = l.G + pn * W1 * sizeof(c16);
  l.S = (l.Dinv + pn * sizeof(c32) + 255) / 256 * 256;
  l.total = (l.S + pn * 7 * sizeof(c32) + 256 + 255) / 256 * 256;
  return l;
}

// Launch arguments of the solver and of the operator / preconditioner apply.
struct Co2Args {
  const Co2Model* model;
  const DevModel* ls;        // level-shift functions (widths, transform nodes)
  const Co2Job* jobs;
  int n_jobs;
  const c64* tables;         // [n_energies][ntab][6]
  int* counter;
  c64* scratch;
  size_t slot_elems, ld;
  const unsigned char* fac;  // block factors, one Co2FacLayout per job (job order of jobs)
  size_t fac_job_bytes;
  int m, max_iter, precond, method;   // method: VDC_GMRES or VDC_COCG
  double tol;
  int n_final;
  const int* finals;         // [n_final][4]
  c64* T_out;                // [n_jobs][n_final][3]
  double* sigma_out;         // [n_jobs][n_final]
  c64* psi_out;              // [n_jobs][npts] or null
  DevInfo* info;
};

// The bend-plane block factorisation of every (job, plane): one wavefront
// per plane.
struct Co2FactorArgs {
  const Co2Model* model;
  const Co2Job* jobs;        // E, sector and table row of each job
  int n_jobs;
  const c64* tables;
  unsigned char* fac;        // one Co2FacLayout per job
  size_t fac_job_bytes;
};

struct Co2OpsArgs {
  const Co2Model* model;
  const c64* tab;            // the energy's table rows
  double E;
  const int* sectors;        // [n_vec][2]
  int n_vec, which;          // 0: operator, 1: block preconditioner
  const c64* x;
  c64* y;
  c64* scratch;              // per workgroup: wA, wB (2 npts)
  size_t slot_elems;
  const unsigned char* fac;  // which == 1: the factor of every vector
  size_t fac_job_bytes;
};

// ------------------------------------------------------------------ blocks

// In-plane element A((x, y), (x + dx, y + dy)) of the block (s, a), |dx|, |dy|
// <= 2; zero where a point carries no state.
__device__ inline c64 co2_band_entry(const Co2Op& o, const double* sq, int s, int a, int x, int y,
                                     int dx, int dy) {
  const Co2Model& m = *o.m;
  const int t = co2_type(x, y, o.px, o.py);
  const int x2 = x + dx, y2 = y + dy;
  if (t == 3 || x2 < 0 || x2 >= m.Nx || y2 < 0 || y2 >= m.Ny) return c64{0.0, 0.0};
  const int t2 = co2_type(x2, y2, o.px, o.py);
  if (t2 == 3) return c64{0.0, 0.0};
  auto Tt = [&](int xx, int yy, int k) { return co2_tab(o, s, xx, yy, a, co2_type(xx, yy, o.px, o.py), k); };
  const double hs2 = m.h_sigma * m.h_sigma, hp2 = m.h_pi * m.h_pi;
  if (dx == 0 && dy == 0) {
    const int c = t == 0 ? 0 : 1;
    const double rt = t == 0 ? 0.0 : (t == 1 ? m.c_rt : -m.c_rt);
    const double U = (c == 0 ? m.E_sigma : m.E_pi) + m.gs[c] * q2_diag(s, m.Ns) +
                     (m.gb[c] + rt) * q2_diag(x, m.Nx) + (m.gb[c] - rt) * q2_diag(y, m.Ny) +
                     m.ga[c] * q2_diag(a, m.Na);
    const double Ev = m.omega_s * (s + 0.5) + m.omega_b * (x + y + 1.0) + m.omega_a * (a + 0.5);
    const int k = t == 0 ? 0 : 2;     // the point's own pair
    auto along_s = [&]() {
      c64 r = c64{0.0, 0.0};
      if (s > 0) r = (0.5 * s) * co2_tab(o, s - 1, x, y, a, t, k);
      if (s + 1 < m.Ns) r = r + (0.5 * (s + 1)) * co2_tab(o, s + 1, x, y, a, t, k);
      return r;
    };
    auto along_x = [&](int kk) {
      c64 r = c64{0.0, 0.0};
      if (x > 0) r = (0.5 * x) * Tt(x - 1, y, kk);
      if (x + 1 < m.Nx) r = r + (0.5 * (x + 1)) * Tt(x + 1, y, kk);
      return r;
    };
    auto along_y = [&](int kk) {
      c64 r = c64{0.0, 0.0};
      if (y > 0) r = (0.5 * y) * Tt(x, y - 1, kk);
      if (y + 1 < m.Ny) r = r + (0.5 * (y + 1)) * Tt(x, y + 1, kk);
      return r;
    };
    c64 F;
    if (t == 0)
      F = Tt(x, y, 0) + (m.l_sigma * m.l_sigma) * along_s() + hs2 * (along_x(0) + along_y(0));
    else
      F = Tt(x, y, 2) + (m.l_pi * m.l_pi) * along_s() + hp2 * (t == 1 ? along_x(2) : along_y(2));
    return c64{(o.E - Ev - U) - F.x, -F.y};
  }
  auto q1 = [&](int n1, int n2) { return sq[n1 > n2 ? n1 : n2]; };   // |n1 - n2| = 1
  if ((dx == 0) != (dy == 0) && (dx == 1 || dx == -1 || dy == 1 || dy == -1)) {
    if (t != 0 && t2 != 0) return c64{0.0, 0.0};
    const int xs = t == 0 ? x : x2, ys = t == 0 ? y : y2;    // the sigma point
    const int xp = t == 0 ? x2 : x, yp = t == 0 ? y2 : y;    // the Pi point
    const double q = dx ? q1(x, x2) : q1(y, y2);
    const c64 ch = m.h_pi * Tt(xs, ys, 1) + m.h_sigma * Tt(xp, yp, 1);
    return c64{-(m.c_sp + ch.x) * q, -ch.y * q};
  }
  if (dy == 0 && (dx == 2 || dx == -2)) {
    if (t != t2) return c64{0.0, 0.0};
    const int xm = (x + x2) / 2;
    const double q = q1(x, xm) * q1(xm, x2);
    const int c = t == 0 ? 0 : 1;
    const double rt = t == 0 ? 0.0 : (t == 1 ? m.c_rt : -m.c_rt);
    c64 f = c64{0.0, 0.0};
    if (t == 0) f = hs2 * Tt(xm, y, 0);
    if (t == 1) f = hp2 * Tt(xm, y, 2);
    return c64{-(m.gb[c] + rt + f.x) * q, -f.y * q};
  }
  if (dx == 0 && (dy == 2 || dy == -2)) {
    if (t != t2) return c64{0.0, 0.0};
    const int ym = (y + y2) / 2;
    const double q = q1(y, ym) * q1(ym, y2);
    const int c = t == 0 ? 0 : 1;
    const double rt = t == 0 ? 0.0 : (t == 1 ? m.c_rt : -m.c_rt);
    c64 f = c64{0.0, 0.0};
    if (t == 0) f = hs2 * Tt(x, ym, 0);
    if (t == 2) f = hp2 * Tt(x, ym, 2);
    return c64{-(m.gb[c] - rt + f.x) * q, -f.y * q};
  }
  if ((dx == 1 || dx == -1) && (dy == 1 || dy == -1)) {
    if (!((t == 1 && t2 == 2) || (t == 2 && t2 == 1))) return c64{0.0, 0.0};
    const int xpx = t == 1 ? x : x2, ypx = t == 1 ? y : y2;   // Pi_x point
    const int xpy = t == 1 ? x2 : x, ypy = t == 1 ? y2 : y;   // Pi_y point
    const int kx = xpy, ky = ypx;                             // the sigma point between
    const double q = q1(xpx, kx) * q1(ky, ypy);
    const c64 f = hp2 * Tt(kx, ky, 2);
    return c64{-(2.0 * m.c_rt + f.x) * q, -f.y * q};
  }
  return c64{0.0, 0.0};
}

}  // namespace vdc
