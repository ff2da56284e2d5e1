// Workgroup-level building blocks of the on-chip Krylov solver: fixed-order
// (deterministic) reductions, multi-vector projections and updates.
//
// Element ownership: thread t of the workgroup owns block elements
// i = t, t + kBlock, t + 2 kBlock, ...  Every pass over a vector uses the same
// ownership, so outside the stencil a thread only reads elements it wrote
// itself and needs no barrier; the stencil (which reads neighbours) starts
// with one.
#pragma once
#include "op2d.h"

namespace vdc {

constexpr int kChunk = 4;   // basis vectors per projection chunk (register budget)

// Sum NV values over the workgroup.  Wave sums by xor-butterfly, then the
// per-wave partials are added in wave order by NV threads (fixed order, so
// the result is bitwise reproducible).  Result in out[0..NV-1] (LDS).
template <int NV, typename R>
__device__ inline void block_sum(R (&v)[NV], R* red, R* out) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] += __shfl_xor(v[q], s, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[wave * NV + q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    R s = R(0);
    for (int w = 0; w < kWaves; ++w) s += red[w * NV + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Values reduced per projection chunk: kChunk complex dot products plus ||w||^2.
constexpr int kRedNV = 2 * kChunk + 1;
// LDS scratch needed by block_sum/project.
constexpr int kRedSize = kWaves * kRedNV + kRedNV;

// h[l] = sum_i conj(V_l[i]) w[i] for l = 0..nv-1 (interleaved re/im in LDS);
// with wnorm2 given, ||w||^2 is accumulated in the same pass (first chunk).
template <typename R>
__device__ inline void project(const typename CT<R>::C* __restrict__ V, size_t ld, int nv,
                               const typename CT<R>::C* __restrict__ w, int Nc, R* red, R* hout,
                               R* wnorm2 = nullptr) {
  using C = typename CT<R>::C;
  for (int l0 = 0; l0 < nv; l0 += kChunk) {
    const int nl = min(kChunk, nv - l0);
    R acc[kRedNV];
#pragma unroll
    for (int q = 0; q < kRedNV; ++q) acc[q] = R(0);
    const bool want_norm = wnorm2 != nullptr && l0 == 0;
    for (int i = threadIdx.x; i < Nc; i += kBlock) {
      const C wi = w[i];
      C vv[kChunk];
#pragma unroll
      for (int q = 0; q < kChunk; ++q) vv[q] = (q < nl) ? V[(size_t)(l0 + q) * ld + i] : cz<R>();
#pragma unroll
      for (int q = 0; q < kChunk; ++q) {
        const C t = conjmul(vv[q], wi);
        acc[2 * q] += t.x;
        acc[2 * q + 1] += t.y;
      }
      if (want_norm) acc[2 * kChunk] += norm2(wi);
    }
    block_sum<kRedNV, R>(acc, red, red + kWaves * kRedNV);
    if (threadIdx.x < 2 * nl) hout[2 * l0 + threadIdx.x] = red[kWaves * kRedNV + threadIdx.x];
    if (want_norm && threadIdx.x == 2 * kChunk) *wnorm2 = red[kWaves * kRedNV + 2 * kChunk];
    __syncthreads();
  }
}

// w[i] -= sum_l V_l[i] h[l], l = 0..nv-1 (h interleaved in LDS), own elements;
// with red given, returns ||w||^2 of the result (reduced in the same pass,
// returned to every thread), else 0.
template <typename R>
__device__ inline R subtract(const typename CT<R>::C* __restrict__ V, size_t ld, int nv,
                             typename CT<R>::C* __restrict__ w, int Nc, const R* h,
                             R* red = nullptr) {
  using C = typename CT<R>::C;
  R acc[1] = {R(0)};
  for (int i = threadIdx.x; i < Nc; i += kBlock) {
    C s = w[i];
    int l = 0;
    for (; l + kChunk <= nv; l += kChunk) {
      C vv[kChunk];
#pragma unroll
      for (int q = 0; q < kChunk; ++q) vv[q] = V[(size_t)(l + q) * ld + i];
#pragma unroll
      for (int q = 0; q < kChunk; ++q) s = s - vv[q] * C{h[2 * (l + q)], h[2 * (l + q) + 1]};
    }
    for (; l < nv; ++l) s = s - V[(size_t)l * ld + i] * C{h[2 * l], h[2 * l + 1]};
    w[i] = s;
    acc[0] += norm2(s);
  }
  if (!red) return R(0);
  block_sum<1, R>(acc, red, red + kWaves);
  const R v = red[kWaves];
  __syncthreads();   // every thread has read v before red is reused
  return v;
}

// ||w||^2 over the workgroup (own elements), returned to every thread.
template <typename R>
__device__ inline R norm_sq(const typename CT<R>::C* __restrict__ w, int Nc, R* red) {
  R acc[1] = {R(0)};
  for (int i = threadIdx.x; i < Nc; i += kBlock) acc[0] += norm2(w[i]);
  block_sum<1, R>(acc, red, red + kWaves);
  const R v = red[kWaves];
  __syncthreads();   // every thread has read v before red is reused
  return v;
}

// y = A (vscale * dinv * v) (dinv may be null), one fused pass through LDS.
// The block is walked in tiles of T rows of n_g: the tile's rows of
// z = vscale dinv v plus two halo rows on each side are staged in LDS (the
// halo rows were just read by the previous tile, so they come from cache),
// the pointwise level-shift products (w_A, w_B) of the rows the tile needs
// are formed in LDS, and y is written once.  lds must hold
// (3 T + 8) * Nu complex values of precision R.  With bsub given the pass
// writes y = bsub - A(...) instead (a residual), and with red given it also
// returns ||y||^2; with bdot given as well, bdot[0..1] receives the bilinear
// form sum_i z_i y_i (no conjugate) of the staged input z = vscale dinv v
// and the output.  Ends with a barrier (y is written by threads other than
// the element owners).
template <typename R>
__device__ inline R matvec_tiled(const OpJob<R>& op, const R* sq,
                                 const typename CT<R>::C* __restrict__ v, R vscale,
                                 const typename CT<R>::C* __restrict__ dinv,
                                 typename CT<R>::C* __restrict__ y,
                                 typename CT<R>::C* lds, int T,
                                 const typename CT<R>::C* __restrict__ bsub = nullptr,
                                 R* red = nullptr, R* bdot = nullptr) {
  using C = typename CT<R>::C;
  R acc[3] = {R(0), R(0), R(0)};
  const int Ng = op.Ng, Nu = op.Nu;
  C* zt = lds;                          // rows g0-2 .. g0+T+1
  C* wa = lds + (size_t)(T + 4) * Nu;   // rows g0-1 .. g0+T
  C* wb = wa + (size_t)(T + 2) * Nu;
  __syncthreads();
  for (int g0 = 0; g0 < Ng; g0 += T) {
    const int t = min(T, Ng - g0);
    const int zr0 = max(0, g0 - 2), zr1 = min(Ng, g0 + t + 2);
    for (int q = threadIdx.x; q < (zr1 - zr0) * Nu; q += kBlock) {
      const int i = zr0 * Nu + q;
      zt[(zr0 - g0 + 2) * Nu + q] = vscale * load_z<R>(v, dinv, i);
    }
    __syncthreads();
    const int wr0 = max(0, g0 - 1), wr1 = min(Ng, g0 + t + 1);
    for (int q = threadIdx.x; q < (wr1 - wr0) * Nu; q += kBlock) {
      const int row = wr0 + q / Nu, nu = q - (q / Nu) * Nu;
      const int a = (nu + op.p) & 1;
      const C* zr = zt + (row - g0 + 2) * Nu;
      C zg = cz<R>(), zu = cz<R>();
      if (row > 0) zg = sq[row] * zr[nu - Nu];
      if (row + 1 < Ng) zg = zg + sq[row + 1] * zr[nu + Nu];
      if (nu > 0) zu = sq[nu] * zr[nu - 1];
      if (nu + 1 < Nu) zu = zu + sq[nu + 1] * zr[nu + 1];
      const C uA = zr[nu] + by_state(op.lamd0, op.lamd1, a) * zg;
      const int i = row * Nu + nu;
      const C fab = op.AB[i];
      wa[(row - g0 + 1) * Nu + nu] = op.AA[i] * uA + fab * zu;
      wb[(row - g0 + 1) * Nu + nu] = fab * uA + op.BB[i] * zu;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < t * Nu; q += kBlock) {
      const int row = g0 + q / Nu, nu = q - (q / Nu) * Nu;
      const int a = (nu + op.p) & 1;
      const C* zr = zt + (row - g0 + 2) * Nu;
      const C* ar = wa + (row - g0 + 1) * Nu;
      const C* br = wb + (row - g0 + 1) * Nu;
      C zg = cz<R>(), zu = cz<R>(), ag = cz<R>(), bu = cz<R>();
      if (row > 0) {
        zg = sq[row] * zr[nu - Nu];
        ag = sq[row] * ar[nu - Nu];
      }
      if (row + 1 < Ng) {
        zg = zg + sq[row + 1] * zr[nu + Nu];
        ag = ag + sq[row + 1] * ar[nu + Nu];
      }
      if (nu > 0) {
        zu = sq[nu] * zr[nu - 1];
        bu = sq[nu] * br[nu - 1];
      }
      if (nu + 1 < Nu) {
        zu = zu + sq[nu + 1] * zr[nu + 1];
        bu = bu + sq[nu + 1] * br[nu + 1];
      }
      const R d = R(by_state(op.dbase0, op.dbase1, a) - op.omega_g * row - op.omega_u * nu);
      C out = d * zr[nu] - by_state(op.kappa0, op.kappa1, a) * zg - op.lam * zu - ar[nu] - by_state(op.lamd0, op.lamd1, a) * ag - bu;
      if (bsub) out = bsub[row * Nu + nu] - out;
      y[row * Nu + nu] = out;
      acc[0] += norm2(out);
      if (bdot) {
        const C t = zr[nu] * out;
        acc[1] += t.x;
        acc[2] += t.y;
      }
    }
    __syncthreads();
  }
  if (!red) return R(0);
  if (bdot) {
    block_sum<3, R>(acc, red, red + kWaves * 3);
    const R s = red[kWaves * 3];
    if (threadIdx.x < 2) bdot[threadIdx.x] = red[kWaves * 3 + 1 + threadIdx.x];
    __syncthreads();
    return s;
  }
  R a1[1] = {acc[0]};
  block_sum<1, R>(a1, red, red + kWaves);
  const R s = red[kWaves];
  __syncthreads();
  return s;
}

// Rows per tile of matvec_tiled for a block of width Nu and lds_bytes of LDS
// (0 when even one row does not fit: use matvec_block instead).
__host__ __device__ inline int tile_rows(int Nu, size_t elem_bytes, size_t lds_bytes) {
  const long per_row = (long)Nu * (long)elem_bytes;
  const long t = ((long)(lds_bytes / per_row) - 8) / 3;
  return t < 1 ? 0 : (t > 32 ? 32 : (int)t);
}

// y = A (dinv * v) (dinv may be null); y, wA, wB are vectors of Nc elements.
// Begins with a barrier so v may have just been written by other threads;
// on return y holds the result at the calling thread's own elements (no
// trailing barrier needed for own-element consumers).
template <typename R>
__device__ inline void matvec_block(const OpJob<R>& op, const R* sq,
                                    const typename CT<R>::C* v,
                                    const typename CT<R>::C* dinv,
                                    typename CT<R>::C* wA, typename CT<R>::C* wB,
                                    typename CT<R>::C* y, R vscale = R(1)) {
  __syncthreads();
  for (int i = threadIdx.x; i < op.Nc; i += kBlock) {
    typename CT<R>::C yl, a, b;
    op_phase1<R>(op, sq, v, dinv, i, yl, a, b);
    y[i] = vscale * yl;
    wA[i] = vscale * a;
    wB[i] = vscale * b;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < op.Nc; i += kBlock) y[i] = op_phase2<R>(op, sq, wA, wB, i, y[i]);
}

// y = A (vscale dinv v): the LDS-tiled pass when tile rows T > 0, else the two
// global phases; ends with a barrier either way.
template <typename R>
__device__ inline void apply_A(const OpJob<R>& op, const R* sq, const typename CT<R>::C* v,
                               R vscale, const typename CT<R>::C* dinv, typename CT<R>::C* y,
                               typename CT<R>::C* lds, int T, typename CT<R>::C* wA,
                               typename CT<R>::C* wB) {
  if (T > 0) {
    matvec_tiled<R>(op, sq, v, vscale, dinv, y, lds, T);
  } else {
    matvec_block<R>(op, sq, v, dinv, wA, wB, y, vscale);
    __syncthreads();
  }
}

// y = b - A x and ||y||^2 (returned to every thread); ends with a barrier.
template <typename R>
__device__ inline R residual_A(const OpJob<R>& op, const R* sq, const typename CT<R>::C* x,
                               const typename CT<R>::C* b, typename CT<R>::C* y,
                               typename CT<R>::C* lds, int T, typename CT<R>::C* wA,
                               typename CT<R>::C* wB, R* red) {
  if (T > 0) return matvec_tiled<R>(op, sq, x, R(1), nullptr, y, lds, T, b, red);
  matvec_block<R>(op, sq, x, nullptr, wA, wB, y);
  R acc[1] = {R(0)};
  for (int i = threadIdx.x; i < op.Nc; i += kBlock) {
    const typename CT<R>::C r = b[i] - y[i];
    y[i] = r;
    acc[0] += norm2(r);
  }
  block_sum<1, R>(acc, red, red + kWaves);
  const R s = red[kWaves];
  __syncthreads();
  return s;
}

}  // namespace vdc
