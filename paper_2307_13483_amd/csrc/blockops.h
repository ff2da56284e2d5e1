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

// y = A (dinv * v) (dinv may be null); y, wA, wB are vectors of Nc elements.
// Begins with a barrier so v may have just been written by other threads;
// on return y holds the result at the calling thread's own elements (no
// trailing barrier needed for own-element consumers).
template <typename R>
__device__ inline void matvec_block(const OpJob<R>& op, const R* sq,
                                    const typename CT<R>::C* v,
                                    const typename CT<R>::C* dinv,
                                    typename CT<R>::C* wA, typename CT<R>::C* wB,
                                    typename CT<R>::C* y) {
  __syncthreads();
  for (int i = threadIdx.x; i < op.Nc; i += kBlock) {
    typename CT<R>::C yl, a, b;
    op_phase1<R>(op, sq, v, dinv, i, yl, a, b);
    y[i] = yl;
    wA[i] = a;
    wB[i] = b;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < op.Nc; i += kBlock) y[i] = op_phase2<R>(op, sq, wA, wB, i, y[i]);
}

}  // namespace vdc
