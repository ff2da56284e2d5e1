// Block-diagonal preconditioner built from sections of A (Sec. III.B): the
// blocks hold the points of one n_u column and kSegRows consecutive n_g, in
// the job's symmetry block.  With the segment as long as the column this is
// the paper's M^u; the segmentation keeps every block small enough for one
// thread's registers.
//
// Band of A inside a column (one active state a along it, op2d.h): the
// direct terms give -k_a q_g, and the sandwich (1 + lam_a q_g) F_AA
// (1 + lam_a q_g) reaches n_g +- 2; every q_u path leaves the column except
// q_u F_BB q_u, which returns and only adds to the diagonal.  With
// q(n) = sqrt(n/2):
//   A(g, g)     = the diagonal of op_diag,
//   A(g, g + 1) = -k_a q(g+1) - lam_a q(g+1) (F_AA(g) + F_AA(g+1)),
//   A(g, g + 2) = -lam_a^2 q(g+1) q(g+2) F_AA(g+1).
// A block is complex symmetric (A^T = A), factored as L D L^T without
// pivoting; a block whose pivot falls below 1e-12 of its diagonal entry is
// replaced by its diagonal.
#pragma once
#include "op2d.h"

namespace vdc {

constexpr int kSegRows = 8;

// L and D^{-1} of every block, one entry per point (block layout).
template <typename R>
struct SegFactor {
  typename CT<R>::C* l1;     // L(g + 1, g) inside the block (0 at its last row)
  typename CT<R>::C* l2;     // L(g + 2, g)
  typename CT<R>::C* dinv;   // 1 / D(g)
};

__host__ __device__ inline int seg_blocks(int Ng, int Nu) {
  return Nu * ((Ng + kSegRows - 1) / kSegRows);
}

__device__ inline c64 col_off1(const OpJob<double>& op, const double* sq, int g, int u, int a) {
  const double q = sq[g + 1];
  const c64 f = op.AA[g * op.Nu + u] + op.AA[(g + 1) * op.Nu + u];
  const double lq = by_state(op.lamd0, op.lamd1, a) * q;
  return c64{-by_state(op.kappa0, op.kappa1, a) * q - lq * f.x, -lq * f.y};
}

__device__ inline c64 col_off2(const OpJob<double>& op, const double* sq, int g, int u, int a) {
  const double l = by_state(op.lamd0, op.lamd1, a);
  return (-l * l * sq[g + 1] * sq[g + 2]) * op.AA[(g + 1) * op.Nu + u];
}

template <typename R>
__device__ inline typename CT<R>::C narrow(c64 a) { return cfrom<R>(a); }

// Factor block c (FP64 arithmetic, stored in precision R), one thread.
template <typename R>
__device__ inline void seg_factor_block(const OpJob<double>& op, const double* sq,
                                        const SegFactor<R>& f, int c) {
  const int Ng = op.Ng, Nu = op.Nu;
  const int u = c % Nu, g0 = (c / Nu) * kSegRows, L = min(kSegRows, Ng - g0);
  const int a = (u + op.p) & 1;
  c64 D[kSegRows], l1[kSegRows], l2[kSegRows];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < kSegRows; ++k) {
    l1[k] = l2[k] = D[k] = c64{0.0, 0.0};
    if (k < L) {
      const int g = g0 + k;
      const c64 akk = op_diag<double>(op, g * Nu + u);
      c64 d = akk;
      if (k >= 1) d = d - (l1[k - 1] * l1[k - 1]) * D[k - 1];
      if (k >= 2) d = d - (l2[k - 2] * l2[k - 2]) * D[k - 2];
      const double nd = sqrt(norm2(d));
      ok = ok && isfinite(nd) && nd > 1e-12 * sqrt(norm2(akk));
      D[k] = d;
      const c64 di = cinv<double>(d);
      if (k + 1 < L) {
        c64 t = col_off1(op, sq, g, u, a);
        if (k >= 1) t = t - (l2[k - 1] * l1[k - 1]) * D[k - 1];
        l1[k] = t * di;
      }
      if (k + 2 < L) l2[k] = col_off2(op, sq, g, u, a) * di;
    }
  }
#pragma unroll
  for (int k = 0; k < kSegRows; ++k) {
    if (k < L) {
      const int i = (g0 + k) * Nu + u;
      if (ok) {
        f.l1[i] = narrow<R>(l1[k]);
        f.l2[i] = narrow<R>(l2[k]);
        f.dinv[i] = narrow<R>(cinv<double>(D[k]));
      } else {
        f.l1[i] = cz<R>();
        f.l2[i] = cz<R>();
        f.dinv[i] = narrow<R>(cinv<double>(op_diag<double>(op, i)));
      }
    }
  }
}

// Factor every block, spread over the workgroup's threads.  No barrier.
template <typename R>
__device__ inline void seg_factor(const OpJob<double>& op, const double* sq,
                                  const SegFactor<R>& f) {
  const int nb = seg_blocks(op.Ng, op.Nu);
  for (int c = threadIdx.x; c < nb; c += kBlock) seg_factor_block<R>(op, sq, f, c);
}

// Block c of z = M^{-1} (vscale v), or of z += M^{-1} (vscale v) with
// accumulate, one thread: forward L, D^{-1}, backward L^T.  z may be v: the
// block's v is read in full before any of it is written.
template <typename R>
__device__ inline void seg_apply_block(const SegFactor<R>& f, int Ng, int Nu,
                                       const typename CT<R>::C* v, R vscale,
                                       typename CT<R>::C* z, bool accumulate, int c) {
  using C = typename CT<R>::C;
  const int u = c % Nu, g0 = (c / Nu) * kSegRows, L = min(kSegRows, Ng - g0);
  C y[kSegRows];
#pragma unroll
  for (int k = 0; k < kSegRows; ++k) {
    y[k] = cz<R>();
    if (k < L) {
      const int i = (g0 + k) * Nu + u;
      C t = vscale * v[i];
      if (k >= 1) t = t - f.l1[i - Nu] * y[k - 1];
      if (k >= 2) t = t - f.l2[i - 2 * Nu] * y[k - 2];
      y[k] = t;
    }
  }
#pragma unroll
  for (int k = kSegRows - 1; k >= 0; --k) {
    if (k < L) {
      const int i = (g0 + k) * Nu + u;
      C t = f.dinv[i] * y[k];
      if (k + 1 < L) t = t - f.l1[i] * y[k + 1];
      if (k + 2 < L) t = t - f.l2[i] * y[k + 2];
      y[k] = t;
      z[i] = accumulate ? z[i] + t : t;
    }
  }
}

// The whole vector, blocks spread over the workgroup's threads.  Begins with
// a barrier (v may have just been written by other threads), ends without.
template <typename R>
__device__ inline void seg_apply(const SegFactor<R>& f, int Ng, int Nu,
                                 const typename CT<R>::C* v, R vscale,
                                 typename CT<R>::C* z, bool accumulate) {
  __syncthreads();
  const int nb = seg_blocks(Ng, Nu);
  for (int c = threadIdx.x; c < nb; c += kBlock)
    seg_apply_block<R>(f, Ng, Nu, v, vscale, z, accumulate, c);
}

// One COCG step's vector work over the column blocks, each block by one
// thread: x += alpha p and r -= alpha q on the block's elements, then
// z = M^{-1} r from the updated r held in registers; acc[0] += ||r||^2 and
// acc[1] + i acc[2] += <r|z>_S (no conjugate) over the thread's blocks.
// Begins with a barrier (p, q may have just been written by other threads);
// x, r and z are then owned by blocks, so a barrier must precede element
// ownership again.
template <typename R>
__device__ inline void seg_cocg_step(const SegFactor<R>& f, int Ng, int Nu,
                                     typename CT<R>::C alpha,
                                     const typename CT<R>::C* __restrict__ p,
                                     const typename CT<R>::C* __restrict__ q,
                                     typename CT<R>::C* __restrict__ x,
                                     typename CT<R>::C* __restrict__ r,
                                     typename CT<R>::C* __restrict__ z, R* acc) {
  using C = typename CT<R>::C;
  __syncthreads();
  const int nb = seg_blocks(Ng, Nu);
  for (int c = threadIdx.x; c < nb; c += kBlock) {
    const int u = c % Nu, g0 = (c / Nu) * kSegRows, L = min(kSegRows, Ng - g0);
    C rv[kSegRows], y[kSegRows];
#pragma unroll
    for (int k = 0; k < kSegRows; ++k) {
      rv[k] = y[k] = cz<R>();
      if (k < L) {
        const int i = (g0 + k) * Nu + u;
        x[i] = x[i] + alpha * p[i];
        const C ri = r[i] - alpha * q[i];
        r[i] = ri;
        rv[k] = ri;
        acc[0] += norm2(ri);
        C t = ri;
        if (k >= 1) t = t - f.l1[i - Nu] * y[k - 1];
        if (k >= 2) t = t - f.l2[i - 2 * Nu] * y[k - 2];
        y[k] = t;
      }
    }
#pragma unroll
    for (int k = kSegRows - 1; k >= 0; --k) {
      if (k < L) {
        const int i = (g0 + k) * Nu + u;
        C t = f.dinv[i] * y[k];
        if (k + 1 < L) t = t - f.l1[i] * y[k + 1];
        if (k + 2 < L) t = t - f.l2[i] * y[k + 2];
        y[k] = t;
        z[i] = t;
        const C rz = rv[k] * t;
        acc[1] += rz.x;
        acc[2] += rz.y;
      }
    }
  }
}

}  // namespace vdc
