// Barrier-free sweep of the operator of op2d.h by one wavefront.
//
// A wavefront owns a strip of 60 consecutive n_u columns (plus two halo
// columns on each side) and walks down the n_g rows of a slab.  The stencil
// couples n_g +- 1 and n_u +- 1 in each of its two passes (the direct terms
// and u_A, u_B; then the two sides of the level-shift sandwich of Eq. (23)),
// so a lane keeps its own column's last rows in registers and takes the
// n_u neighbours from the adjacent lanes.  The two halo columns absorb the
// radius-two reach in n_u: the outer halo lane's own neighbours are not
// valid, but only halo lanes use them.  Nothing goes through LDS and there
// is no barrier, so the many independent wavefronts of a launch hide the
// memory latency among themselves; on top of that each lane requests the
// rows it will need several steps ahead.
//
// Values outside the basis (n < 0 or n >= N) are zeros, which reproduces
// the truncation of q at the basis edge.
#pragma once
#include <type_traits>

#include "op2d.h"

namespace vdc {

constexpr int kStripHalo = 2;
constexpr int kStripWidth = 64 - 2 * kStripHalo;   // owned columns per wavefront

__host__ __device__ inline int strip_count(int Nu) {
  return (Nu + kStripWidth - 1) / kStripWidth;
}

// Lane moves by one position across the whole wavefront (DPP wave_shr:1 /
// wave_shl:1): lane_prev gives lane i the value of lane i - 1, lane_next
// that of lane i + 1.  With bound_ctrl set, lanes 0 and 63 (both halo
// lanes) receive zero.
__device__ inline int dpp_prev(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ inline int dpp_next(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ inline double lane_prev(double v) {
  return __hiloint2double(dpp_prev(__double2hiint(v)), dpp_prev(__double2loint(v)));
}
__device__ inline double lane_next(double v) {
  return __hiloint2double(dpp_next(__double2hiint(v)), dpp_next(__double2loint(v)));
}
__device__ inline float lane_prev(float v) { return __int_as_float(dpp_prev(__float_as_int(v))); }
__device__ inline float lane_next(float v) { return __int_as_float(dpp_next(__float_as_int(v))); }
__device__ inline c64 lane_prev(c64 a) { return c64{lane_prev(a.x), lane_prev(a.y)}; }
__device__ inline c64 lane_next(c64 a) { return c64{lane_next(a.x), lane_next(a.y)}; }
__device__ inline c32 lane_prev(c32 a) { return c32{lane_prev(a.x), lane_prev(a.y)}; }
__device__ inline c32 lane_next(c32 a) { return c32{lane_next(a.x), lane_next(a.y)}; }

template <typename R>
struct StripTab { typename CT<R>::C aa, ab, bb; };

// Registers of one lane: z at rows r-1 and r, the level-shift products w_A
// at rows r-2 and r-1 (w_B at r-1), the local part of the output at row r-1
// (every term but the n_g and n_u neighbours of w_A and w_B) and sqrt(n/2)
// at n = r-1 and r.
template <typename R>
struct StripState {
  using C = typename CT<R>::C;
  C zc, zn, wam, wac, wbc, ylc;
  R sqm, sqc;
};

// y[i] = A (vscale dinv v) [i] for rows g0 .. g1-1 of the wavefront's strip
// (bsub given: y = bsub - A(...)); returns the lane's sum of |y|^2 over the
// elements it wrote.  sq holds sqrt(n/2) for n = 0..kSqMax (LDS).  z is
// requested ZA rows ahead, the level-shift tables TA rows ahead (more rows
// in flight against more registers).  Control flow is uniform across the wavefront except
// for the masked store.  Every load is issued unconditionally from a clamped
// address and masked afterwards, so the loop body is straight-line code and
// the loads for the rows ahead stay in flight across steps.
template <typename R, int ZA = 2, int TA = 1>
__device__ inline R strip_sweep(const OpJob<R>& op, const R* sq,
                                const typename CT<R>::C* __restrict__ v,
                                R vscale, const typename CT<R>::C* __restrict__ dinv,
                                typename CT<R>::C* __restrict__ y,
                                const typename CT<R>::C* __restrict__ bsub, int strip, int g0,
                                int g1) {
  using C = typename CT<R>::C;
  const int Ng = op.Ng, Nu = op.Nu;
  const int lane = threadIdx.x & 63;
  const int nu = strip * kStripWidth - kStripHalo + lane;
  const bool col = nu >= 0 && nu < Nu;
  const bool own = col && lane >= kStripHalo && lane < 64 - kStripHalo;
  const int cc = min(max(nu, 0), Nu - 1);
  const int a = (nu + op.p) & 1;
  const R sql = col ? R(sqrt(0.5 * nu)) : R(0);         // sqrt(n_u / 2)
  const R sqr = col ? R(sqrt(0.5 * (nu + 1))) : R(0);   // sqrt((n_u + 1) / 2)
  const R lda = by_state(op.lamd0, op.lamd1, a);
  const R kap = by_state(op.kappa0, op.kappa1, a);
  const double dcol = by_state(op.dbase0, op.dbase1, a) - op.omega_u * nu;
  const int zmax = min(Ng - 1, g1 + 1), tmax = min(Ng - 1, g1);   // last rows used

  // z at row r of this lane's column (zero outside the basis); rows past
  // the slab's last use are clamped and never consumed
  auto load_row = [&](int r) -> C {
    const int i = min(max(r, 0), zmax) * Nu + cc;
    const C z = vscale * load_z<R>(v, dinv, i);
    return (col && r >= 0 && r < Ng) ? z : cz<R>();
  };
  auto load_tab = [&](int r) -> StripTab<R> {
    const int i = min(max(r, 0), tmax) * Nu + cc;
    return StripTab<R>{op.AA[i], op.AB[i], op.BB[i]};
  };
  // sqrt(n/2) for a row index n; rows past N_g only ever scale zeros
  auto sqg = [&](int n) { return sq[min(max(n, 0), kSqMax)]; };

  StripState<R> s;
  s.zc = load_row(g0 - 2);
  s.zn = load_row(g0 - 1);
  s.wam = s.wac = s.wbc = s.ylc = cz<R>();
  s.sqm = sqg(g0 - 2);
  s.sqc = sqg(g0 - 1);
  // Prefetch slots: slot k of pz serves the steps j = r - g0 + 1 with
  // j % ZA == k, likewise pt.  The loop below is unrolled by 4.
  static_assert(4 % ZA == 0 && 4 % TA == 0, "prefetch distances must divide the unroll");
  constexpr int kZAhead = ZA, kTAhead = TA;
  C pz[kZAhead];
  for (int k = 0; k < kZAhead; ++k) pz[k] = load_row(g0 + k);
  StripTab<R> pt[kTAhead];
  for (int k = 0; k < kTAhead; ++k) pt[k] = load_tab(g0 - 1 + k);
  R acc = R(0);

  // One step at lead row r: the level-shift products at row r and, with
  // OUT, the output row r - 1.
  auto step = [&](auto out_tag, int r, C& zslot, StripTab<R>& tslot) {
    constexpr bool OUT = decltype(out_tag)::value;
    const C zp = zslot;
    const StripTab<R> tr = tslot;
    zslot = load_row(r + 1 + kZAhead);
    tslot = load_tab(r + kTAhead);
    const R sqn = sqg(r + 1);
    const C zl = lane_prev(s.zn), zr = lane_next(s.zn);
    const C zg = s.sqc * s.zc + sqn * zp;
    const C zu = sql * zl + sqr * zr;
    const C uA = s.zn + lda * zg;
    const bool live = col && r >= 0 && r < Ng;
    const C wan = live ? tr.aa * uA + tr.ab * zu : cz<R>();
    const C wbn = live ? tr.ab * uA + tr.bb * zu : cz<R>();
    const R d = R(dcol - op.omega_g * r);
    const C yln = d * s.zn - kap * zg - op.lam * zu - wan;
    if constexpr (OUT) {
      const int q = r - 1;
      const C bl = lane_prev(s.wbc), br = lane_next(s.wbc);
      const C ag = s.sqm * s.wam + s.sqc * wan;
      const C bu = sql * bl + sqr * br;
      C out = s.ylc - lda * ag - bu;
      if (own) {
        const int i = q * Nu + nu;
        if (bsub) out = bsub[i] - out;
        y[i] = out;
        acc += norm2(out);
      }
    }
    s.wam = s.wac;
    s.wac = wan;
    s.wbc = wbn;
    s.ylc = yln;
    s.zc = s.zn;
    s.zn = zp;
    s.sqm = s.sqc;
    s.sqc = sqn;
  };
  using no = std::integral_constant<bool, false>;
  using yes = std::integral_constant<bool, true>;

  // steps j = r - g0 + 1 = 0, 1 only fill the registers; from j = 2 on each
  // step also writes row r - 1
  step(no{}, g0 - 1, pz[0], pt[0]);
  step(no{}, g0, pz[1 % kZAhead], pt[1 % kTAhead]);
  int r = g0 + 1;
  for (; r + 3 <= g1; r += 4) {
    step(yes{}, r, pz[2 % kZAhead], pt[2 % kTAhead]);
    step(yes{}, r + 1, pz[3 % kZAhead], pt[3 % kTAhead]);
    step(yes{}, r + 2, pz[4 % kZAhead], pt[4 % kTAhead]);
    step(yes{}, r + 3, pz[5 % kZAhead], pt[5 % kTAhead]);
  }
  if (r <= g1) step(yes{}, r, pz[2 % kZAhead], pt[2 % kTAhead]);
  if (r + 1 <= g1) step(yes{}, r + 1, pz[3 % kZAhead], pt[3 % kTAhead]);
  if (r + 2 <= g1) step(yes{}, r + 2, pz[4 % kZAhead], pt[4 % kTAhead]);
  return acc;
}

}  // namespace vdc
