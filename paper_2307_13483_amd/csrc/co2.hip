// Kernels of the CO2-like model (co2.h): the persistent batched GMRES with
// the bend-plane block preconditioner (Sec. III.B; the block choice the paper
// makes for its CO2 model in Sec. III.C), and the operator and preconditioner
// applied to given vectors.
#include "co2.h"
#include "krylov.h"
#include "strip.h"

namespace vdc {

__device__ inline double co2_apply(const Co2Op& o, const double* sq, const c64* v, double vs,
                                   c64* y, c64* wA, c64* wB, const c64* bsub, double* red,
                                   double* bdot) {
  const int n = o.m->npts;
  __syncthreads();
#pragma unroll 1
  for (int i = threadIdx.x; i < n; i += kBlock) {
    c64 a, b;
    co2_phase1(o, sq, v, vs, i, a, b);
    wA[i] = a;
    wB[i] = b;
  }
  __syncthreads();
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
  for (int i = threadIdx.x; i < n; i += kBlock) {
    c64 r = co2_phase2(o, sq, v, vs, wA, wB, i);
    if (bsub) r = bsub[i] - r;
    y[i] = r;
    acc[0] += norm2(r);
    if (bdot) {
      const c64 t = (vs * v[i]) * r;
      acc[1] += t.x;
      acc[2] += t.y;
    }
  }
  if (!red) {
    __syncthreads();
    return 0.0;
  }
  block_sum<3, double>(acc, red, red + 3 * kWaves);
  const double s = red[3 * kWaves];
  if (bdot && threadIdx.x < 2) bdot[threadIdx.x] = red[3 * kWaves + 1 + threadIdx.x];
  __syncthreads();
  return s;
}

// Block element A(r, c) of plane (s, a) in the plane's point order j = x Ny + y;
// rows and columns of points without a state are those of the identity.
__device__ inline c64 co2_plane_entry(const Co2Op& o, const double* sq, int s, int a, int r, int c) {
  const Co2Model& m = *o.m;
  const int xr = r / m.Ny, yr = r - xr * m.Ny, xc = c / m.Ny, yc = c - xc * m.Ny;
  if (co2_type(xr, yr, o.px, o.py) == 3 || co2_type(xc, yc, o.px, o.py) == 3)
    return c64{r == c ? 1.0 : 0.0, 0.0};
  const int dx = xc - xr, dy = yc - yr;
  if (dx < -2 || dx > 2 || dy < -2 || dy > 2) return c64{0.0, 0.0};
  return co2_band_entry(o, sq, s, a, xr, yr, dx, dy);
}

// ------------------------------------------------------------------ block factorisation
//
// Each plane block (fixed n_s, n_a; points j = x Ny + y, y fastest) is
// banded with half bandwidth w = 2 Ny and complex symmetric; it is factored
// A = L D L^T without pivoting (Sec. III.B), the band and its updates in
// FP32 (pivots and multipliers formed in FP64).  L is stored in FP16 twice,
// by columns, F[j][k] = L(j + k, j), and by rows, G[i][k] = L(i, i - k),
// k = 1..w (entry 0 and entries before column 0 are zero), so that both
// triangular sweeps of the apply read contiguous rows; 1/D is stored in
// FP32 (Co2FacLayout).  The applied preconditioner is the exact inverse of
// the stored L D L^T, applied in FP64: a fixed linear operator (its
// distance from the block's inverse only changes the iteration count), so
// GMRES sees no rounding-dependent preconditioner.
//
// One wavefront per plane.  First the wavefront writes the plane's nonzero
// band entries to the staging area S: for column c and the seven stencil
// offsets o, (dx', dy') with dx' >= 0 of |dx'| + |dy'| <= 2, the entry
// A(c + dx' Ny + dy', c) (zero where that point lies outside the plane;
// points without a state carry the identity).  Then the elimination runs
// with the active part of the band in registers: lane (R mod 64) holds row
// R, register c the column j0 + c (j0 the first pivot of the current group
// of kFacU pivots), and each lane updates its own row.  After
// kFacU pivots the registers move down by kFacU (the columns just eliminated
// leave) and the kFacU rows that become active enter through LDS; their
// band entries were fetched one group earlier.  The pivot column reaches
// the lanes through LDS (each lane writes its entry, every lane reads the
// entries after the pivot as broadcast loads) rather than by readlane: 48
// complex values per pivot as scalars would not fit the scalar registers.

constexpr int kFacU = 4;                          // pivots per register shift
constexpr int kFacMaxW = 48;                      // largest half bandwidth: Ny <= 24
constexpr int kFacSlots = kFacMaxW + kFacU;       // register columns per row
constexpr int kFacWaves = 4;                      // planes per workgroup
constexpr int kFacStencil = 7;                    // stencil offsets per column
constexpr int kFacChunk = 16;                     // pivot-row entries per load chunk
static_assert(kFacMaxW % kFacChunk == 0, "the pivot row is read in whole chunks");
// a pivot below this fraction of its original diagonal entry (squared
// magnitudes) sends the plane to its diagonal
constexpr double kFacPivotTol = 1e-10;

// Stencil offset o = 0..6: (dx', dy') = (0,0) (0,1) (0,2) (1,-1) (1,0) (1,1) (2,0).
__host__ __device__ inline int stencil_dx(int o) { return (o >= 3) + (o >= 6); }
__host__ __device__ inline int stencil_dy(int o) { return o < 3 ? o : (o < 6 ? o - 4 : 0); }

__device__ inline double rlane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ inline c64 rlane(c64 v, int l) { return c64{rlane(v.x, l), rlane(v.y, l)}; }
__device__ inline float rlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline c32 rlane(c32 v, int l) { return c32{rlane(v.x, l), rlane(v.y, l)}; }
__device__ inline c32 to32(c64 v) { return c32{(float)v.x, (float)v.y}; }
__device__ inline c64 to64(c32 v) { return c64{(double)v.x, (double)v.y}; }
__device__ inline c16 to16(c64 v) { return c16{(_Float16)(float)v.x, (_Float16)(float)v.y}; }
__device__ inline c64 to64(c16 v) { return c64{(double)(float)v.x, (double)(float)v.y}; }

// Orders this wavefront's LDS writes before its later LDS reads.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(64 * kFacWaves) co2_factor_kernel(Co2FactorArgs a) {
  __shared__ double sq[kSqMax + 1];
  __shared__ c32 stage[kFacWaves][kFacU * kFacSlots];
  // the pivot column of each wavefront, twice over (lanes 0..63 at k and
  // k + 64), in two buffers used by alternate pivots
  __shared__ c32 colbuf[kFacWaves][2][128];
  fill_sq<double>(sq);
  __syncthreads();
  const Co2Model& m = *a.model;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int planes = m.Ns * m.Na, per_job = (planes + kFacWaves - 1) / kFacWaves;
  const int job = blockIdx.x / per_job, P = (blockIdx.x - job * per_job) * kFacWaves + wv;
  if (job >= a.n_jobs || P >= planes) return;
  const Co2Job& jb = a.jobs[job];
  const Co2Op op{a.model, a.tables + (size_t)jb.table * m.ntab * kNumF, jb.E, jb.px, jb.py};
  const int n = m.Nx * m.Ny, w = 2 * m.Ny, W1 = w + 1;
  const int ps = P / m.Na, pa = P - ps * m.Na;
  const Co2FacLayout lay = co2_fac_layout(planes, n, W1);
  unsigned char* base = a.fac + (size_t)job * a.fac_job_bytes;
  c16* F = reinterpret_cast<c16*>(base + lay.F) + (size_t)P * n * W1;
  c16* G = reinterpret_cast<c16*>(base + lay.G) + (size_t)P * n * W1;
  c32* Dinv = reinterpret_cast<c32*>(base + lay.Dinv) + (size_t)P * n;
  c32* S = reinterpret_cast<c32*>(base + lay.S) + (size_t)P * n * kFacStencil;
  // entries of G before column 0, and the staged band
  for (int q = lane; q < min(w, n) * W1; q += 64) {
    const int i = q / W1, k = q - i * W1;
    if (k > i) G[q] = c16{0, 0};
  }
  for (int e = lane; e < n * kFacStencil; e += 64) {
    const int c = e / kFacStencil, o = e - kFacStencil * c;
    const int xc = c / m.Ny, yc = c - xc * m.Ny;
    const int xr = xc + stencil_dx(o), yr = yc + stencil_dy(o);
    c64 v = c64{0.0, 0.0};
    if (xr < m.Nx && yr >= 0 && yr < m.Ny) v = co2_plane_entry(op, sq, ps, pa, xr * m.Ny + yr, c);
    S[e] = to32(v);
  }
  __threadfence_block();   // written by every lane, read back by other lanes below
  c32* st = stage[wv];
  // this lane's entry of a group's band: (row b, offset o), lane = b 7 + o
  // (lanes from kFacU 7 on hold none)
  const int fb = lane / kFacStencil, fo = lane - kFacStencil * fb;
  const int foff = stencil_dx(fo) * m.Ny + stencil_dy(fo);
  c32 T = c32{0.f, 0.f};
  auto fetch = [&](int r0, int cnt) {
    const int R = r0 + fb, c = R - foff;
    T = (fb < cnt && R < n && c >= 0) ? S[(size_t)c * kFacStencil + fo] : c32{0.f, 0.f};
  };
  c32 A[kFacSlots];
#pragma unroll
  for (int c = 0; c < kFacSlots; ++c) A[c] = c32{0.f, 0.f};
  float d0 = 0.f;   // |original diagonal entry|^2 of this lane's row
  // the fetched rows r0 .. r0 + cnt - 1 into their lanes, register c =
  // column j0 + c, through LDS laid out by register (where two offsets of a
  // small plane name the same column, at most one of them is nonzero)
  auto enter = [&](int r0, int cnt, int j0) {
    for (int q = lane; q < kFacU * kFacSlots; q += 64) st[q] = c32{0.f, 0.f};
    wave_lds_sync();
    const int c = r0 - j0 + fb - foff;
    if (fb < cnt && c >= 0 && c < kFacSlots && (T.x != 0.f || T.y != 0.f)) st[fb * kFacSlots + c] = T;
    wave_lds_sync();
    const int b = (lane - r0) & 63;
    if (b < cnt) {
#pragma unroll
      for (int cc = 0; cc < kFacSlots; ++cc) A[cc] = st[b * kFacSlots + cc];
      d0 = norm2(st[b * kFacSlots + (r0 + b - j0)]);
    }
    wave_lds_sync();
  };
  for (int r0 = 0; r0 < w + kFacU && r0 < n; r0 += kFacU) {
    const int cnt = min(kFacU, min(w + kFacU, n) - r0);
    fetch(r0, cnt);
    enter(r0, cnt, 0);
  }
  if (kFacU < n - w) fetch(kFacU + w, min(kFacU, n - kFacU - w));
  bool ok = true;
#pragma unroll 1
  for (int j0 = 0; j0 < n; j0 += kFacU) {
    // the last group may run past n: such pivots store nothing and update
    // no row
#pragma unroll
    for (int t = 0; t < kFacU; ++t) {
      const int j = j0 + t;
      // every lane's entry of column j, A(R, j) of its row R, into LDS: the
      // pivot row's entries A(j, j + c') = A(j + c', j) (A is symmetric) are
      // then read back by every lane as broadcast loads, pc[c' - 1]
      c32* col = colbuf[wv][t & 1];
      col[lane] = A[t];
      col[lane + 64] = A[t];
      wave_lds_sync();
      const c32* pc = col + ((j + 1) & 63);
      const c64 D = to64(col[j & 63]);
      const double nd = norm2(D);
      if (j < n) ok = ok && isfinite(nd) && nd > kFacPivotTol * (double)rlane(d0, j & 63);
      const c64 Di = cinv<double>(D);
      const int r = (lane - j) & 63;            // this lane's row is j + r
      const bool act = r >= 1 && r <= w && j + r < n;
      const c64 L = act ? to64(A[t]) * Di : c64{0.0, 0.0};
      if (r <= w && j < n) {
        const c16 o = to16(L);
        F[(size_t)j * W1 + r] = o;
        if (j + r < n) G[(size_t)(j + r) * W1 + r] = o;
        if (r == 0) Dinv[j] = to32(Di);
      }
      // A(j + r, j + c') -= L(j + r, j) A(j + c', j), c' = 1..48, in every
      // lane (L = 0 in rows outside the pivot's band; offsets past w and
      // entries right of a row's diagonal land in registers no live row
      // uses)
      const c32 Lf = to32(L);
      // (in chunks of kFacChunk: their broadcast loads, then their updates;
      // the scheduling barrier keeps the chunks' loads from all being hoisted
      // ahead, which would take kFacMaxW complex registers at once)
#pragma unroll
      for (int c0 = 1; c0 <= kFacMaxW; c0 += kFacChunk) {
        c32 scv[kFacChunk];
#pragma unroll
        for (int q = 0; q < kFacChunk; ++q) scv[q] = pc[c0 - 1 + q];
#pragma unroll
        for (int q = 0; q < kFacChunk; ++q) {
          const c32 sc = scv[q];
          c32& e = A[t + c0 + q];
          e.x = fmaf(-Lf.x, sc.x, e.x);
          e.x = fmaf(Lf.y, sc.y, e.x);
          e.y = fmaf(-Lf.x, sc.y, e.y);
          e.y = fmaf(-Lf.y, sc.x, e.y);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int c = 0; c + kFacU < kFacSlots; ++c) A[c] = A[c + kFacU];
    // rows j0 + U + w .. enter now (their first pivot is in the next
    // group); the group after that is fetched for the next round
    const int nj0 = j0 + kFacU, r0 = nj0 + w;
    if (r0 < n) {
      enter(r0, min(kFacU, n - r0), nj0);
      if (r0 + kFacU < n) fetch(r0 + kFacU, min(kFacU, n - r0 - kFacU));
    }
  }
  if (!ok) {
    // a vanishing pivot: the plane falls back to its diagonal
    for (int q = lane; q < n * W1; q += 64) {
      F[q] = c16{0, 0};
      G[q] = c16{0, 0};
    }
    for (int j = lane; j < n; j += 64) Dinv[j] = to32(cinv<double>(co2_plane_entry(op, sq, ps, pa, j, j)));
  }
}

// Lane i takes the value of lane i + 1, lane 63 that of lane 0 (DPP
// wave_rol:1).
__device__ inline int dpp_rot(int v) { return __builtin_amdgcn_mov_dpp(v, 0x134, 0xf, 0xf, false); }
__device__ inline double lane_rot(double v) {
  return __hiloint2double(dpp_rot(__double2hiint(v)), dpp_rot(__double2loint(v)));
}
__device__ inline c64 lane_rot(c64 a) { return c64{lane_rot(a.x), lane_rot(a.y)}; }

// Vector values enter the sweeps through the lanes past the band: w + Q <= 63.
constexpr int kApplyQ = 15;

// z = M^{-1} (vs v) (z may be v): one wavefront per plane, two sweeps of the
// same form.  Forward L y = vs v over the columns of L (F): lane k carries
// the running value of row j + k; at step j lane 0 holds y_j, every other
// lane subtracts L(j + k, j) y_j, and the lanes rotate down by one, so y_j
// goes to lane 63.  Backward L^T z = D^{-1} y over the rows of L (G): lane k
// carries row j - k; lane 0 holds z_j, every other lane subtracts
// L(j, j - k) z_j, the lanes rotate.  The lanes past the band (k > w) carry
// the next kApplyQ starting values, which enter at lane w without a
// per-step select; after kApplyQ steps the results of the chunk sit in
// lanes 64 - kApplyQ .. 63 and are stored, and the starting lanes are
// refilled (a value above them needs more than kApplyQ steps to reach the
// band).  Factor rows are loaded kApplyQ steps ahead by all 64 lanes (the
// lanes outside the band read the row's entry 0, which the factor stores as
// zero).  Steps past the plane's end only touch
// values that are never stored.  Begins and ends with a barrier.
__device__ __attribute__((always_inline)) inline void co2_block_apply(
    const Co2Model& m, const unsigned char* fac, const c64* v, double vs, c64* z) {
  __syncthreads();
  constexpr int Q = kApplyQ;
  const int n = m.Nx * m.Ny, w = 2 * m.Ny, W1 = w + 1, planes = m.Ns * m.Na;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool feed = lane > w && lane <= w + Q;   // refilled per chunk
  const int outq = lane - (64 - Q);              // the chunk step this lane holds at its end
  // the lanes outside the band (lane 0 and lanes past w) read entry 0 of a
  // factor row, which is zero, so their running values stay as they are
  // without a per-step mask; the row is addressed as a uniform base plus the
  // lane's byte offset
  const unsigned loff = (unsigned)(lane >= 1 && lane <= w ? lane : 0) * (unsigned)sizeof(c16);
  const Co2FacLayout lay = co2_fac_layout(planes, n, W1);
  auto step = [&](c64& acc, c16& Lq, const c16* next_row) {
    const c64 x = rlane(acc, 0);
    const c16 Lh = Lq;
    Lq = *reinterpret_cast<const c16*>(reinterpret_cast<const char*>(next_row) + loff);
    const double lx = (double)(float)Lh.x, ly = (double)(float)Lh.y;
    acc.x = fma(-lx, x.x, acc.x);
    acc.x = fma(ly, x.y, acc.x);
    acc.y = fma(-lx, x.y, acc.y);
    acc.y = fma(-ly, x.x, acc.y);
    acc = lane_rot(acc);
  };
  for (int P = wave; P < planes; P += kWaves) {
    const c16* F = reinterpret_cast<const c16*>(fac + lay.F) + (size_t)P * n * W1;
    const c16* G = reinterpret_cast<const c16*>(fac + lay.G) + (size_t)P * n * W1;
    const c32* Dinv = reinterpret_cast<const c32*>(fac + lay.Dinv) + (size_t)P * n;
    const c64* vp = v + (size_t)P * n;
    c64* zp = z + (size_t)P * n;
    // forward: lane k starts with row k
    c16 Lr[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q)
      Lr[q] = *reinterpret_cast<const c16*>(reinterpret_cast<const char*>(F + (size_t)min(q, n - 1) * W1) + loff);
    c64 acc = lane < n && lane <= w + Q ? vs * vp[lane] : c64{0.0, 0.0};
    for (int j0 = 0; j0 < n; j0 += Q) {
      const int e = j0 + Q + lane;   // starting values of the next chunk
      const c64 vnext = feed && e < n ? vs * vp[e] : c64{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < Q; ++q) step(acc, Lr[q], F + (size_t)min(j0 + q + Q, n - 1) * W1);
      if (outq >= 0 && j0 + outq < n) zp[j0 + outq] = acc;
      if (feed) acc = vnext;
    }
    __threadfence_block();   // y, written above by several lanes, is read back below
    // backward: lane k starts with row n - 1 - k, D^{-1} y
#pragma unroll
    for (int q = 0; q < Q; ++q)
      Lr[q] = *reinterpret_cast<const c16*>(reinterpret_cast<const char*>(G + (size_t)max(n - 1 - q, 0) * W1) + loff);
    auto start = [&](int i) { return i >= 0 ? to64(Dinv[i]) * zp[i] : c64{0.0, 0.0}; };
    acc = lane <= w + Q ? start(n - 1 - lane) : c64{0.0, 0.0};
    for (int j1 = n - 1; j1 >= 0; j1 -= Q) {
      const c64 snext = feed ? start(j1 - Q - lane) : c64{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < Q; ++q) step(acc, Lr[q], G + (size_t)max(j1 - q - Q, 0) * W1);
      if (outq >= 0 && j1 - outq >= 0) zp[j1 - outq] = acc;
      if (feed) acc = snext;
    }
  }
  __syncthreads();
}

// Jacobi: dinv = 1 / diag(A) at points with a state, 0 elsewhere.
__device__ inline void co2_jacobi(const Co2Op& o, const double* sq, c64* dinv) {
  const Co2Model& m = *o.m;
  for (int i = threadIdx.x; i < m.npts; i += kBlock) {
    const Co2Point p = co2_point(m, i);
    dinv[i] = co2_type(p.x, p.y, o.px, o.py) == 3
                  ? c64{0.0, 0.0}
                  : cinv<double>(co2_band_entry(o, sq, p.s, p.a, p.x, p.y, 0, 0));
  }
}

// Nonzero entries of Phi^{v mu} in the sector (px, py): f_d^mu(eps) O_d^mu |v>
// (Eq. (25)); at most 7 entries (index into the sector vector, value).
struct Co2PhiEntry { int i; double val; };

__device__ inline int co2_phi_entries(const Co2Model& m, const DevModel& ls, const int* v, int mu,
                                      double eps, int px, int py, Co2PhiEntry* e) {
  int n = 0;
  auto idx = [&](int s, int x, int y, int a) { return ((s * m.Na + a) * m.Nx + x) * m.Ny + y; };
  auto add = [&](int d, int s, int x, int y, int a, double val) {
    if (s < 0 || s >= m.Ns || x < 0 || x >= m.Nx || y < 0 || y >= m.Ny || a < 0 || a >= m.Na) return;
    if (co2_type(x, y, px, py) != d || val == 0.0) return;
    e[n++] = Co2PhiEntry{idx(s, x, y, a), val};
  };
  const int s = v[0], x = v[1], y = v[2], a = v[3];
  const int w = mu == 0 ? 0 : 1;
  for (int d = 0; d < 3; ++d) {
    const double f = coupling_f(ls, d == 0 ? 0 : 1, w, eps);
    if (f == 0.0) continue;
    const bool gs = (mu == 0 && d == 0) || (mu == 1 && d == 1) || (mu == 2 && d == 2);
    if (gs) {   // (1 + l q_s)
      const double l = d == 0 ? m.l_sigma : m.l_pi;
      add(d, s, x, y, a, f);
      add(d, s + 1, x, y, a, f * l * sqrt(0.5 * (s + 1)));
      add(d, s - 1, x, y, a, f * l * sqrt(0.5 * s));
    } else if ((mu == 0 && d == 1) || (mu == 1 && d == 0)) {   // h q_x
      const double h = d == 0 ? m.h_sigma : m.h_pi;
      add(d, s, x + 1, y, a, f * h * sqrt(0.5 * (x + 1)));
      add(d, s, x - 1, y, a, f * h * sqrt(0.5 * x));
    } else if ((mu == 0 && d == 2) || (mu == 2 && d == 0)) {   // h q_y
      const double h = d == 0 ? m.h_sigma : m.h_pi;
      add(d, s, x, y + 1, a, f * h * sqrt(0.5 * (y + 1)));
      add(d, s, x, y - 1, a, f * h * sqrt(0.5 * y));
    }
  }
  return n;
}

struct Co2Lds {
  KrylovLds<double> K;
  double red[kRedSize];
  double sq[kSqMax + 1];
  double dot[2];
  int job;
};

// Byte model (passes over a sector vector of npts complex FP64 values; the
// factor, W1 = 2 Ny + 1 complex FP16 multipliers per point by columns and
// again by rows plus 1/D in FP32, is M = W1 / 2 + 1 / 2 passes): setup: x, b
// written, b read, V_0 copied (5), plus the factor written by the factor
// kernel (M) or dinv written (1); Arnoldi step: M^{-1} (the columns read
// forward, the rows and 1/D backward, and the vector in, y out, y in, zt
// out: M + 4) or the diagonal (v, dinv read, zt written: 3), then the
// operator (zt read twice, w_A, w_B written and read, y written: 7), and the
// projection passes of cycle_passes (which counts 6 for an operator of its
// own); cycle end with k steps: the update (basis k and zt out, M^{-1} in
// place, x in/out and zt in: k + M + 8; with the diagonal: k + 3) and the
// true residual (x twice, w_A, w_B twice, b, residual out: 8).  COCG: setup
// as above plus r = b (2), K^{-1} r (block M + 4, diagonal 3) and <r|z>_S
// (2); per step the operator with <p|Ap>_S (7), x and r (6), K^{-1} r, its
// <r|z>_S (2) and p = z + beta p (3); a true-residual check 8.
__global__ void __launch_bounds__(kBlock) co2_gmres_kernel(Co2Args a) {
  __shared__ Co2Lds L;
  fill_sq<double>(L.sq);
  const Co2Model& md = *a.model;
  const int tid = threadIdx.x;
  const int npts = md.npts;
  const size_t ld = a.ld;
  const int m = a.m;
  c64* slot = a.scratch + (size_t)blockIdx.x * a.slot_elems;
  c64* V = slot;
  c64* x = V + (size_t)(m + 1) * ld;
  c64* b = x + ld;
  c64* zt = b + ld;
  c64* wA = zt + ld;
  c64* wB = wA + ld;
  c64* dinv = wB + ld;
  c64* Rm = dinv + ld;
  const bool blk = a.precond == VDC_PREC_BLOCK;
  const double W1 = 2.0 * md.Ny + 1.0;
  for (;;) {
    __syncthreads();
    if (tid == 0) L.job = atomicAdd(a.counter, 1);
    __syncthreads();
    const int js = L.job;
    if (js >= a.n_jobs) break;
    const Co2Job jb = a.jobs[js];
    const Co2Op op{a.model, a.tables + (size_t)jb.table * md.ntab * kNumF, jb.E, jb.px, jb.py};
    const unsigned char* fac = blk ? a.fac + (size_t)js * a.fac_job_bytes : nullptr;
    double passes = 5.0;
    const double Mp = 0.5 * W1 + 0.5;   // the factor, in passes
    if (blk) {
      passes += Mp;
    } else if (a.precond == VDC_PREC_JACOBI) {
      co2_jacobi(op, L.sq, dinv);
      passes += 1.0;
    }
    for (int i = tid; i < npts; i += kBlock) {
      x[i] = c64{0.0, 0.0};
      b[i] = c64{0.0, 0.0};
    }
    __syncthreads();
    if (tid == 0) {
      Co2PhiEntry e[8];
      const int ne = co2_phi_entries(md, *a.ls, jb.v, jb.mu, jb.eps_i, jb.px, jb.py, e);
      for (int q = 0; q < ne; ++q) b[e[q].i] = b[e[q].i] + c64{e[q].val, 0.0};
    }
    __syncthreads();
    const double bnorm = sqrt(norm_sq<double>(b, npts, L.red));
    double beta = bnorm;
    int iters = 0, cycles = 0, status = VDC_NOT_CONVERGED;
    if (!(bnorm > 0.0) || !isfinite(bnorm)) {
      status = isfinite(bnorm) ? VDC_CONVERGED : VDC_NONFINITE;
      beta = 0.0;
    } else if (a.method == VDC_COCG) {
      // COCG (Sec. III.A) preconditioned as M^{-1} A M^{-T} with K = M M^T
      // the block L D L^T or the diagonal (both symmetric), in the two-term
      // form; r, p, q, z in V_0..V_3.  The true residual decides; the
      // iteration restarts from it when only the updated one has converged,
      // and after one breakdown of the bilinear form.
      c64* r = V;
      c64* p = V + ld;
      c64* q = V + 2 * ld;
      c64* z = V + 3 * ld;
      auto kinv = [&](const c64* src, c64* dst) {   // dst = K^{-1} src, then a barrier
        if (blk) {
          co2_block_apply(md, fac, src, 1.0, dst);
          passes += Mp + 4.0;
        } else {
          for (int i = tid; i < npts; i += kBlock)
            dst[i] = a.precond == VDC_PREC_JACOBI ? dinv[i] * src[i] : src[i];
          __syncthreads();
          passes += 3.0;
        }
      };
      auto bilin = [&](const c64* u, const c64* w) {   // <u|w>_S over own elements
        double acc[2] = {0.0, 0.0};
        for (int i = tid; i < npts; i += kBlock) {
          const c64 t = u[i] * w[i];
          acc[0] += t.x;
          acc[1] += t.y;
        }
        block_sum<2, double>(acc, L.red, L.red + 2 * kWaves);
        const c64 v = c64{L.red[2 * kWaves], L.red[2 * kWaves + 1]};
        __syncthreads();
        passes += 2.0;
        return v;
      };
      for (int i = tid; i < npts; i += kBlock) r[i] = b[i];
      passes += 2.0;
      kinv(r, p);
      c64 rho = bilin(r, p);
      bool fresh = true;
      for (;;) {
        co2_apply(op, L.sq, p, 1.0, q, wA, wB, nullptr, L.red, L.dot);
        passes += 7.0;
        const c64 mu = c64{L.dot[0], L.dot[1]};
        const double mn = norm2(mu), rn = norm2(rho);
        if (!(mn > 0.0) || !(rn > 0.0) || !isfinite(mn) || !isfinite(rn)) {
          if (fresh) {
            status = (isfinite(mn) && isfinite(rn)) ? VDC_BREAKDOWN : VDC_NONFINITE;
            break;
          }
          beta = sqrt(co2_apply(op, L.sq, x, 1.0, r, wA, wB, b, L.red));
          passes += 8.0;
          ++cycles;
          if (beta <= a.tol * bnorm) {
            status = VDC_CONVERGED;
            break;
          }
          kinv(r, p);
          rho = bilin(r, p);
          fresh = true;
          continue;
        }
        const c64 alpha = cdiv(rho, mu);
        double acc[1] = {0.0};
        for (int i = tid; i < npts; i += kBlock) {
          x[i] = x[i] + alpha * p[i];
          const c64 ri = r[i] - alpha * q[i];
          r[i] = ri;
          acc[0] += norm2(ri);
        }
        block_sum<1, double>(acc, L.red, L.red + kWaves);
        const double rr = L.red[kWaves];
        __syncthreads();
        passes += 6.0;
        ++iters;
        fresh = false;
        if (!isfinite(rr)) {
          status = VDC_NONFINITE;
          break;
        }
        if (sqrt(rr) <= a.tol * bnorm || iters >= a.max_iter) {
          beta = sqrt(co2_apply(op, L.sq, x, 1.0, r, wA, wB, b, L.red));
          passes += 8.0;
          ++cycles;
          if (beta <= a.tol * bnorm) {
            status = VDC_CONVERGED;
            break;
          }
          if (!isfinite(beta)) {
            status = VDC_NONFINITE;
            break;
          }
          if (iters >= a.max_iter) break;
          kinv(r, p);
          rho = bilin(r, p);
          fresh = true;
          continue;
        }
        kinv(r, z);
        const c64 rho_new = bilin(r, z);
        const c64 bt = cdiv(rho_new, rho);
        rho = rho_new;
        for (int i = tid; i < npts; i += kBlock) p[i] = z[i] + bt * p[i];
        passes += 3.0;
      }
    } else {
      for (int i = tid; i < npts; i += kBlock) V[i] = b[i];
      auto apply = [&](int j, double sc, c64* out) {
        const c64* vj = V + (size_t)j * ld;
        if (blk) {
          co2_block_apply(md, fac, vj, sc, zt);
        } else {
          for (int i = tid; i < npts; i += kBlock)
            zt[i] = a.precond == VDC_PREC_JACOBI ? sc * (dinv[i] * vj[i]) : sc * vj[i];
        }
        co2_apply(op, L.sq, zt, 1.0, out, wA, wB);
      };
      for (;;) {
        if (tid == 0) {
          L.K.g[0] = c64{beta, 0.0};
          L.K.vs[0] = 1.0 / beta;
        }
        __syncthreads();
        const CycleResult cr = krylov_cycle<double>(L.K, L.red, V, ld, npts, m, a.tol * bnorm,
                                                    a.max_iter, iters, Rm, apply);
        passes += cycle_passes(cr.k, cr.reorth_passes) + cr.k * ((blk ? Mp + 4.0 : 3.0) + 1.0) +
                  (blk ? cr.k + Mp + 8.0 : cr.k + 3.0) + 8.0;
        if (blk) {
          update_x<double>(V, ld, cr.k, L.K.y, L.K.vs, nullptr, zt, npts, true);
          co2_block_apply(md, fac, zt, 1.0, zt);
          for (int i = tid; i < npts; i += kBlock) x[i] = x[i] + zt[i];
        } else {
          update_x<double>(V, ld, cr.k, L.K.y, L.K.vs,
                           a.precond == VDC_PREC_JACOBI ? dinv : nullptr, x, npts);
        }
        beta = sqrt(co2_apply(op, L.sq, x, 1.0, V, wA, wB, b, L.red));
        ++cycles;
        if (!isfinite(beta) || cr.nonfinite) {
          status = VDC_NONFINITE;
          break;
        }
        if (beta <= a.tol * bnorm) {
          status = VDC_CONVERGED;
          break;
        }
        if (cr.breakdown) {
          status = VDC_BREAKDOWN;
          break;
        }
        if (iters >= a.max_iter) {
          status = VDC_NOT_CONVERGED;
          break;
        }
      }
    }
    __syncthreads();
    // amplitudes T = Phi_f^T psi for each final state and partial wave, and
    // the job's share of sigma (Eqs. (15), (16))
    const int out = jb.out;
    const double c = 2.0 * kPi * kPi * kPi / (jb.eps_i / kHartreeEV);
    for (int q = tid; q < a.n_final * 3; q += kBlock) {
      const int f = q / 3, mu = q - 3 * f;
      const int* vf = a.finals + 4 * f;
      const double Ef = md.omega_s * (vf[0] + 0.5) + md.omega_b * (vf[1] + vf[2] + 1.0) +
                        md.omega_a * (vf[3] + 0.5);
      Co2PhiEntry e[8];
      const int ne = co2_phi_entries(md, *a.ls, vf, mu, jb.E - Ef, jb.px, jb.py, e);
      c64 T = c64{0.0, 0.0};
      for (int r = 0; r < ne; ++r) T = T + e[r].val * x[e[r].i];
      a.T_out[((size_t)out * a.n_final + f) * 3 + mu] = T;
    }
    __syncthreads();
    for (int f = tid; f < a.n_final; f += kBlock) {
      double s2 = 0.0;
      for (int mu = 0; mu < 3; ++mu) s2 += norm2(a.T_out[((size_t)out * a.n_final + f) * 3 + mu]);
      a.sigma_out[(size_t)out * a.n_final + f] = c * s2;
    }
    if (a.psi_out)
      for (int i = tid; i < npts; i += kBlock) a.psi_out[(size_t)out * npts + i] = x[i];
    if (tid == 0)
      a.info[out] = DevInfo{status, iters, cycles, 0, bnorm > 0.0 ? beta / bnorm : 0.0,
                            passes * 16.0 * npts};
  }
}

// y = A x or y = M^{-1} x for given sector vectors (one workgroup per vector).

__global__ void __launch_bounds__(kBlock) co2_ops_kernel(Co2OpsArgs a) {
  __shared__ double sq[kSqMax + 1];
  fill_sq<double>(sq);
  const Co2Model& md = *a.model;
  c64* slot = a.scratch + (size_t)blockIdx.x * a.slot_elems;
  for (int v = blockIdx.x; v < a.n_vec; v += gridDim.x) {
    const Co2Op op{a.model, a.tab, a.E, a.sectors[2 * v], a.sectors[2 * v + 1]};
    const c64* xv = a.x + (size_t)v * md.npts;
    c64* yv = a.y + (size_t)v * md.npts;
    if (a.which == 0) {
      co2_apply(op, sq, xv, 1.0, yv, slot, slot + md.npts);
    } else {
      co2_block_apply(md, a.fac + (size_t)v * a.fac_job_bytes, xv, 1.0, yv);
    }
  }
}

int co2_factor_max_ny() { return kFacMaxW / 2; }

hipError_t launch_co2_factor(const Co2FactorArgs& a, int Ns, int Na, hipStream_t s) {
  const int per_job = (Ns * Na + kFacWaves - 1) / kFacWaves;
  const size_t groups = (size_t)per_job * a.n_jobs;
  if (groups == 0) return hipSuccess;
  if (groups > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(co2_factor_kernel, dim3((unsigned)groups), dim3(64 * kFacWaves), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_co2_gmres(const Co2Args& a, int n_groups, hipStream_t s) {
  hipLaunchKernelGGL(co2_gmres_kernel, dim3(n_groups), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// The operator on many sector vectors at once (vdc_co2_apply, which = 0) as
// two grid-wide passes, one thread per (vector, point) in workgroups of
// kCo2Threads: the first writes every point's (w_A, w_B), the second every
// point's y from its neighbours' z and (w_A, w_B).  The same per-point
// arithmetic as the solver's operator (co2_phase1, co2_phase2); here every
// point of every vector is independent work, so the loads of many
// wavefronts are in flight per CU instead of those of one workgroup per
// vector.  Vectors are taken in batches (the w planes of a batch are
// scratch): vector v0 + blockIdx.y.
constexpr int kCo2Threads = 256;

__device__ inline void fill_sq_small(double* sq, int nmax) {
  for (int n = threadIdx.x; n <= nmax; n += blockDim.x) sq[n] = sqrt(0.5 * n);
  __syncthreads();
}

__global__ void __launch_bounds__(kCo2Threads) co2_w_kernel(Co2OpsArgs a, int v0) {
  __shared__ double sq[kSqMax + 1];
  const Co2Model& md = *a.model;
  fill_sq_small(sq, max(max(md.Ns, md.Nx), max(md.Ny, md.Na)) + 2);
  const int i = blockIdx.x * kCo2Threads + threadIdx.x;
  if (i >= md.npts) return;
  const int v = v0 + blockIdx.y;
  const Co2Op op{a.model, a.tab, a.E, a.sectors[2 * v], a.sectors[2 * v + 1]};
  c64 wa, wb;
  co2_phase1(op, sq, a.x + (size_t)v * md.npts, 1.0, i, wa, wb);
  c64* w = a.scratch + (size_t)blockIdx.y * 2 * md.npts;
  w[i] = wa;
  w[md.npts + i] = wb;
}

__global__ void __launch_bounds__(kCo2Threads) co2_y_kernel(Co2OpsArgs a, int v0) {
  __shared__ double sq[kSqMax + 1];
  const Co2Model& md = *a.model;
  fill_sq_small(sq, max(max(md.Ns, md.Nx), max(md.Ny, md.Na)) + 2);
  const int i = blockIdx.x * kCo2Threads + threadIdx.x;
  if (i >= md.npts) return;
  const int v = v0 + blockIdx.y;
  const Co2Op op{a.model, a.tab, a.E, a.sectors[2 * v], a.sectors[2 * v + 1]};
  const c64* w = a.scratch + (size_t)blockIdx.y * 2 * md.npts;
  a.y[(size_t)v * md.npts + i] =
      co2_phase2(op, sq, a.x + (size_t)v * md.npts, 1.0, w, w + md.npts, i);
}

// The operator on many sector vectors at once by marching along n_s
// (vdc_co2_apply, which = 0, for bend planes of Nx Ny <= kMarchMaxPlane
// points): one workgroup per (vector, n_a), one thread per bend point that
// carries a state (co2_live_point).  Step s of the march
//   stores z and the level-shift rows of plane s + 1 into LDS rings (four
//   z planes, two planes of rows),
//   computes (w_A, w_B) at s + 1 (co2_point1; its bend neighbours from LDS),
//   stores the component the point's bend neighbours read into a ring of two
//   LDS planes,
//   computes y at s (co2_point2; the bend neighbours of z at s - 1 .. s + 1
//   and of w at s from LDS, the own column and z at n_a -+ 2 from
//   registers) and stores it,
// with one barrier per step: a z slot written in step s was last read in
// step s - 2, a w or row slot in step s - 1, before the barrier of step s.
// A bend neighbour (n_x +- 1 or n_y +- 1) flips one parity, so it is of the
// other class or carries no state: each point stores only the component of
// the other class (w_B at sigma points, w_A at Pi points).  Every x value is
// read from memory three times (own column, and as the n_a +- 2 neighbour of
// two workgroups of the same vector), y written once (its zeros at the
// points that carry no state after the march), and no w leaves the chip.  The loads a step needs (z of the own column at s + 2, z at n_a -+ 2,
// the level-shift rows of s + 1) are issued at the top of the step before.
// Workgroups are dealt to the eight XCDs in turn (workgroup b to XCD b mod
// 8); the workgroups of one vector are numbered so that they share an XCD and
// follow each other there, and their n_a +- 2 reads meet one L2.  The same
// per-point arithmetic as the solver's operator and the split passes.
constexpr int kMarchMaxPlane = 1024;

// The launch's dynamic LDS (the same array the solver kernels tile into).
extern __shared__ __align__(16) char vdc_tile_lds[];

// A complex value in the march's LDS rings, read and written as one 16-byte
// vector access (c64 itself is 8-byte aligned, and a pair of doubles may be
// split into two 8-byte accesses at a 16-byte lane stride: two-way bank
// conflicts).  Every access to the rings goes through these.
typedef double c64v __attribute__((ext_vector_type(2)));

__device__ inline c64 ld16(const c64* p) {
  const c64v v = *reinterpret_cast<const c64v*>(p);
  return c64{v.x, v.y};
}

__device__ inline void st16(c64* p, c64 v) { *reinterpret_cast<c64v*>(p) = c64v{v.x, v.y}; }

// The bend points of a plane that carry a state (types 0, 1, 2): every row
// holds the ne points with n_y + py even, a row with n_x + px even also the
// Ny - ne others, and the remaining points (type 3) carry none.  They are
// ordered in two parts: the points with n_y + py even, row by row (Nx ne),
// then the others, row by row over the rows that hold them.  Ordered so, the
// bend neighbours of a run of consecutive points in one row are consecutive
// points of one row, or all the one zero entry.
__host__ __device__ inline int co2_row_even(int Ny, int py) { return (Ny + 1 - py) / 2; }

__host__ __device__ inline int co2_live_count(int Nx, int Ny, int px, int py) {
  const int full = (Nx + 1 - px) / 2;
  return full * Ny + (Nx - full) * co2_row_even(Ny, py);
}

// The k-th point that carries a state (k < co2_live_count).
__host__ __device__ inline void co2_live_point(int k, int Nx, int Ny, int px, int py, int& x,
                                               int& y) {
  const int ne = co2_row_even(Ny, py), no = Ny - ne;
  if (k < Nx * ne) {
    x = k / ne;
    y = 2 * (k - x * ne) + py;
  } else {
    const int q = (k - Nx * ne) / no;
    x = 2 * q + px;
    y = 2 * (k - Nx * ne - q * no) + 1 - py;
  }
}

// The k-th point that carries none (k < Nx Ny - co2_live_count): n_x + px and
// n_y + py both odd.
__host__ __device__ inline void co2_dead_point(int k, int Ny, int px, int py, int& x, int& y) {
  const int nd = Ny - co2_row_even(Ny, py);
  const int h = k / nd;
  x = 2 * h + 1 - px;
  y = 2 * (k - h * nd) + 1 - py;
}

// Threads of a march workgroup: one per point that carries a state, and at
// least as many as the points that carry none (each stores the zeros of one),
// over the four sectors.
inline int co2_march_threads(int Nx, int Ny) {
  int n = 0;
  for (int p = 0; p < 4; ++p) {
    const int live = co2_live_count(Nx, Ny, p & 1, p >> 1);
    n = max(n, max(live, Nx * Ny - live));
  }
  return (n + 63) / 64 * 64;
}

// The march's rings hold a plane's points that carry a state in the order
// of co2_live_point, then one zero entry.  Co2Nbr: the ring indices of a
// point's twelve bend neighbours (n_x, n_y offsets of co2_nbr_slot), the
// zero entry for a neighbour outside the plane or one that carries no state.
struct Co2Nbr {
  int i[12];
};

__host__ __device__ constexpr int co2_nbr_slot(int dx, int dy) {
  return dy == 0   ? (dx == -1 ? 0 : dx == 1 ? 1 : dx == -2 ? 4 : 5)
         : dx == 0 ? (dy == -1 ? 2 : dy == 1 ? 3 : dy == -2 ? 6 : 7)
                   : 8 + (dx > 0 ? 2 : 0) + (dy > 0 ? 1 : 0);
}

// Ring index of point (x, y) (the inverse of co2_live_point), or zslot.
__host__ __device__ inline int co2_ring_index(int x, int y, int Nx, int Ny, int px, int py,
                                              int zslot) {
  if (x < 0 || x >= Nx || y < 0 || y >= Ny || (((x + px) & (y + py)) & 1)) return zslot;
  const int ne = co2_row_even(Ny, py);
  if (((y + py) & 1) == 0) return x * ne + ((y - py) >> 1);
  return Nx * ne + (x >> 1) * (Ny - ne) + ((y + py - 1) >> 1);
}

// Neighbour accessor of the march for a centre at plane s (see co2_point1,
// co2_point2): LDS planes of z at s - 2 (own column only) and s - 1 .. s + 1,
// of the neighbour components of w at s and the point's level-shift values;
// in registers the own column's z at s .. s + 2, z at n_a -+ 2 and the own
// class's w at s - 1 .. s + 1; model coefficients picked as uniform values
// (co2_pick: the march's loop would reload a per-lane choice after every
// store of y).  A neighbour that is not in the basis is not selected away:
// every such term carries a zero weight (sqrt(0/2) of the basis edge), and the
// value read there is finite for a finite input (the ring's zero entry, its
// zero planes before the first n_s, an earlier plane of the input after the
// last, or zeros past either end of n_a), so the product is zero without a
// select.  A neighbour that carries no state reads the zero entry; the terms
// that read one are those the point's type does not use.
struct Co2Ring {
  const c64* zm2;
  const c64* zp[3];
  const c64* wn;
  const c64* T;
  c64 z0, z1, z2, za[2], wc[3];
  int k;                     // the point's ring index
  Co2Nbr nb;                 // ring indices of its bend neighbours
  Co2BendW W;                // its bend-mode weights
  __device__ c64 z(bool, int ds, int da, int dx, int dy) const {
    if (da != 0) return za[da > 0 ? 1 : 0];
    if (dx == 0 && dy == 0) {
      if (ds == 0) return z0;
      if (ds == 1) return z1;
      if (ds == 2) return z2;
      return ld16((ds == -1 ? zp[0] : zm2) + k);
    }
    return ld16(zp[1 + ds] + nb.i[co2_nbr_slot(dx, dy)]);
  }
  __device__ c64 w(bool, int ds, int dx, int dy) const {
    if (dx == 0 && dy == 0) return wc[1 + ds];
    return ld16(wn + nb.i[co2_nbr_slot(dx, dy)]);
  }
  __device__ c64 tab(const Co2Op&, const Co2Point&, int, int k) const { return ld16(T + k); }
  __device__ double pick(bool first, double a, double b) const { return co2_pick(first, a, b); }
  __device__ double cls(const double* c2, int c) const { return co2_pick(c == 0, c2[0], c2[1]); }
  __device__ Co2BendW bend(const double*, const Co2Model&, const Co2Point&) const { return W; }
};

// Doubles of sqrt(n/2) at the head of the march's dynamic LDS (even, so the
// planes after them stay 16-byte aligned), and the whole dynamic LDS: sqrt
// values, z ring [4][Nx Ny], w ring [2][Nx Ny], row ring [2][6 (Nx + Ny - 1)].
__host__ __device__ inline int co2_march_sq(int Ns, int Nx, int Ny, int Na) {
  const int nmax = max(max(Ns, Nx), max(Ny, Na));
  return (nmax + 4) & ~1;
}

__host__ __device__ inline size_t co2_march_lds(int Ns, int Nx, int Ny, int Na) {
  return (size_t)co2_march_sq(Ns, Nx, Ny, Na) * sizeof(double) +
         ((size_t)6 * (Nx * Ny + 1) + (size_t)2 * kNumF * (Nx + Ny - 1)) * sizeof(c64);
}

// The model, vectors and rows come as separate kernel arguments, none aliasing
// another, so that the model's fields are read once into scalar registers
// and no store of y orders the loads of x.
template <int kThreads>
__global__ void __launch_bounds__(kThreads)
    co2_march_kernel(const Co2Model* __restrict__ model, const c64* __restrict__ tab,
                     const int* __restrict__ sectors, int n_vec, double E,
                     const c64* __restrict__ x_in, c64* __restrict__ y_out) {
  const Co2Model& md = *model;
  const int Ns = md.Ns, Na = md.Na, Ny = md.Ny, NP = md.Nx * md.Ny;
  const int b = blockIdx.x, slot = b >> 3;
  const int ia = slot % Na;
  const int v = (slot / Na) * 8 + (b & 7);
  if (v >= n_vec) return;
  const int tid = threadIdx.x;
  const int nsq = co2_march_sq(Ns, md.Nx, Ny, Na);
  const int ntp = kNumF * md.nb;              // level-shift values of one plane's rows
  double* sq = reinterpret_cast<double*>(vdc_tile_lds);
  const int PS = NP + 1;                      // ring plane: the points, one zero
  c64* zl = reinterpret_cast<c64*>(vdc_tile_lds + nsq * sizeof(double));   // [4][PS]
  c64* wl = zl + 4 * PS;                                                   // [2][PS]
  c64* tl = wl + 2 * PS;                                                   // [2][ntp]
  for (int n = tid; n < nsq; n += blockDim.x) sq[n] = sqrt(0.5 * n);
  // the rings start at zero: planes -2 and -1, and the zero entries
  for (int i = tid; i < 6 * PS; i += blockDim.x) st16(zl + i, c64{0.0, 0.0});
  const int px = sectors[2 * v] & 1, py = sectors[2 * v + 1] & 1;
  // one lane per point that carries a state; lanes past them compute the
  // first such point (or point 0 if there is none) and store nothing
  const int n_live = co2_live_count(md.Nx, Ny, px, py), n_dead = NP - n_live;
  const bool live = tid < n_live;
  int x = 0, y = 0;
  if (n_live > 0) co2_live_point(live ? tid : 0, md.Nx, Ny, px, py, x, y);
  const int j = x * Ny + y;                   // in the vector
  const int k = live ? tid : 0;               // in the rings
  Co2Nbr nb;
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const int dx = i < 8 ? (i < 4 ? (i < 2 ? 2 * i - 1 : 0) : (i < 6 ? 4 * i - 18 : 0)) : (i < 10 ? -1 : 1);
    const int dy = i < 8 ? (i < 4 ? (i < 2 ? 0 : 2 * i - 5) : (i < 6 ? 0 : 4 * i - 26)) : ((i & 1) ? 1 : -1);
    nb.i[i] = co2_ring_index(x + dx, y + dy, md.Nx, Ny, px, py, NP);
  }
  // the model's fields read once, before the loop (read in the loop's
  // branches, the compiler would load them again at every step)
  const Co2Model mloc = md;
  const Co2Op op{&mloc, tab, E, px, py};
  const int t = co2_type(x, y, op.px, op.py);
  const int trow_off = (x + y) * kNumF + (t == 0 || t == 3 ? 0 : 3);   // co2_tab's row and class
  const int ss = Na * NP;                     // stride of n_s
  // this workgroup's column block of the vector: point (s, n_a, j) at s ss + j
  const c64* xv = x_in + (size_t)v * md.npts + (size_t)ia * NP;
  c64* yv = y_out + (size_t)v * md.npts + (size_t)ia * NP;
  const c64* tab_a = tab + (size_t)ia * kNumF;
  const bool alo = ia >= 2, ahi = ia + 2 < Na;
  const c64 zero{0.0, 0.0};
  // z of the own column at plane s (0 past the last), and at s, n_a + da
  auto zat = [&](int s) {
    c64 r{0.0, 0.0};
    if (s < Ns) r = xv[s * ss + j];
    return r;
  };
  auto zna = [&](bool ok, int s, int da) {
    c64 r{0.0, 0.0};
    if (ok && s < Ns) r = xv[s * ss + da * NP + j];
    return r;
  };
  // value i of the level-shift rows of plane s (co2_tab at n_x + n_y = i / 6)
  auto trow = [&](int s, int i) {
    return tab_a[(size_t)(s * md.nb + i / kNumF) * Na * kNumF + i % kNumF];
  };
  auto trow_ahead = [&](int s) {
    c64 r{0.0, 0.0};
    if (tid < ntp && s < Ns) r = trow(s, tid);
    return r;
  };
  // z(s), z(s + 1), z(s + 2) of the own column; z(s, n_a -+ 2); the own
  // class's w(s - 1), w(s); the rows of plane s + 1 in flight.  The loads of a
  // step are issued at its top and waited for at its end, where the registers
  // move down; moving the freshest load waits for everything in flight, so in
  // this rolled loop loading further ahead would only hold registers.
  c64 z0 = zat(0), z1 = zat(1), z2 = zat(2);
  c64 zam = zna(alo, 0, -2), zap = zna(ahi, 0, 2);
  c64 wo0 = zero, wo1 = zero, yprev = zero;
  for (int i = tid; i < ntp; i += blockDim.x) st16(tl + i, trow(0, i));
  c64 tq = trow_ahead(1);
  // plane 0 and its w
  __syncthreads();
  // the point's bend weights, held in registers for the march
  const Co2BendW bw(Co2BendSq{sq, x, y, md.Nx, Ny});
  if (live) st16(zl + k, z0);
  __syncthreads();
  {
    const Co2Ring R{zl, {zl, zl, zl}, wl, tl + trow_off, z0, z1, zero, {zero, zero}, {zero, zero, zero},
                    k, nb, bw};
    c64 wa, wb;
    co2_point1(op, sq, R, Co2Point{0, ia, x, y, 0}, wa, wb);
    wo1 = co2_sel(t == 0, wa, wb);
    if (live) st16(wl + k, co2_sel(t == 0, wb, wa));
  }
#pragma unroll 1
  for (int s = 0; s < Ns; ++s) {
    c64* zs1 = zl + ((s + 1) & 3) * PS;
    c64* w1 = wl + ((s + 1) & 1) * PS;
    c64* t1 = tl + ((s + 1) & 1) * ntp;
    if (s + 1 < Ns) {
      if (live) st16(zs1 + k, z1);
      if (tid < ntp) st16(t1 + tid, tq);
      for (int i = tid + blockDim.x; i < ntp; i += blockDim.x) st16(t1 + i, trow(s + 1, i));
    }
    const c64 tq2 = trow_ahead(s + 2);
    const c64 zam2 = zna(alo, s + 1, -2), zap2 = zna(ahi, s + 1, 2);
    const c64 z3 = zat(s + 3);
    // y of the previous step, stored at the top of this step: the wait at a
    // step's end covers every memory operation in flight (stores count with
    // the loads on this target), so a store issued just before it would be
    // waited for at once
    if (live && s > 0) yv[(s - 1) * ss + j] = yprev;
    __syncthreads();
    c64 wn1 = zero;
    if (s + 1 < Ns) {
      const Co2Ring R{zl, {zl + (s & 3) * PS, zs1, zs1}, w1, t1 + trow_off, z1, z2, zero, {zero, zero},
                      {zero, zero, zero}, k, nb, bw};
      c64 wa, wb;
      co2_point1(op, sq, R, Co2Point{s + 1, ia, x, y, 0}, wa, wb);
      wn1 = co2_sel(t == 0, wa, wb);
      if (live) st16(w1 + k, co2_sel(t == 0, wb, wa));
    }
    {
      const Co2Ring R{zl + ((s + 2) & 3) * PS, {zl + ((s + 3) & 3) * PS, zl + (s & 3) * PS, zs1},
                      wl + (s & 1) * PS, tl, z0, z1, z2, {zam, zap}, {wo0, wo1, wn1}, k, nb, bw};
      yprev = co2_point2(op, sq, R, Co2Point{s, ia, x, y, 0});
    }
    z0 = z1;
    z1 = z2;
    z2 = z3;
    zam = zam2;
    zap = zap2;
    tq = tq2;
    wo0 = wo1;
    wo1 = wn1;
  }
  if (live) yv[(Ns - 1) * ss + j] = yprev;
  // y is zero at the points that carry no state
  if (tid < n_dead) {
    int xd, yd;
    co2_dead_point(tid, Ny, px, py, xd, yd);
    for (int sd = 0; sd < Ns; ++sd) yv[sd * ss + xd * Ny + yd] = zero;
  }
}

// Whether the march takes a model: planes up to kMarchMaxPlane points and
// its rings within 96 KiB of LDS.
bool co2_march_fits(int Ns, int Nx, int Ny, int Na) {
  return Nx * Ny <= kMarchMaxPlane && co2_march_lds(Ns, Nx, Ny, Na) <= 96 * 1024;
}

// Groups of the march: eight per (n_a, group of eight vectors).
hipError_t launch_co2_march(const Co2OpsArgs& a, int Ns, int Nx, int Ny, int Na, hipStream_t s) {
  if (a.n_vec == 0) return hipSuccess;
  const size_t groups = (size_t)8 * Na * ((a.n_vec + 7) / 8);
  if (!co2_march_fits(Ns, Nx, Ny, Na) || groups > 0x7fffffff) return hipErrorInvalidValue;
  const int threads = co2_march_threads(Nx, Ny);
  // up to 512 threads (8 wavefronts, at most 2 per SIMD) the kernel may use
  // 256 VGPRs, wider ones 128
  if (threads <= 512)
    hipLaunchKernelGGL(co2_march_kernel<512>, dim3((unsigned)groups), dim3(threads),
                       co2_march_lds(Ns, Nx, Ny, Na), s, a.model, a.tab, a.sectors, a.n_vec, a.E,
                       a.x, a.y);
  else
    hipLaunchKernelGGL(co2_march_kernel<kMarchMaxPlane>, dim3((unsigned)groups), dim3(threads),
                       co2_march_lds(Ns, Nx, Ny, Na), s, a.model, a.tab, a.sectors, a.n_vec, a.E,
                       a.x, a.y);
  return hipGetLastError();
}

// npts: points per vector (host copy of the model's), batch: vectors whose w
// planes fit the scratch.
hipError_t launch_co2_apply_split(const Co2OpsArgs& a, int npts, int batch, hipStream_t s) {
  for (int v0 = 0; v0 < a.n_vec; v0 += batch) {
    const int nb = min(batch, a.n_vec - v0);
    const dim3 grid((npts + kCo2Threads - 1) / kCo2Threads, nb);
    hipLaunchKernelGGL(co2_w_kernel, grid, dim3(kCo2Threads), 0, s, a, v0);
    hipLaunchKernelGGL(co2_y_kernel, grid, dim3(kCo2Threads), 0, s, a, v0);
  }
  return hipGetLastError();
}

hipError_t launch_co2_ops(const Co2OpsArgs& a, int n_groups, hipStream_t s) {
  hipLaunchKernelGGL(co2_ops_kernel, dim3(n_groups), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace vdc
