// Block-diagonal preconditioners built from sections of A (Sec. III.B), in
// the job's symmetry block.  Column blocks (VDC_PREC_BLOCK): the points of
// one n_u column and kSegRows consecutive n_g; with the segment as long as
// the column this is the paper's M^u, and the segmentation keeps every block
// small enough for one thread's registers.  Row blocks (VDC_PREC_ROWS, the
// second half of this file): the whole n_u row of one n_g, the paper's M^g.
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
// pivoting; a block whose pivot falls below 1e-12 of its diagonal entry, or
// whose multipliers do not fit their storage, is replaced by its diagonal.
#pragma once
#include "op2d.h"

namespace vdc {

constexpr int kSegRows = 8;

// Storage of the multipliers: complex FP64 for the FP64 solvers, complex
// FP16 for the FP32 ones (halves the bytes and registers of their sweeps;
// the stored values define the preconditioner exactly, so it stays
// symmetric).  D^{-1} keeps the solver's precision.
template <typename R> struct FacT { using S = typename CT<R>::C; };
template <> struct FacT<float> { using S = c16; };

template <typename R>
__device__ inline typename CT<R>::C lw(typename CT<R>::C a) { return a; }
template <typename R>
__device__ inline typename CT<R>::C lw(c16 a) {
  return typename CT<R>::C{R((float)a.x), R((float)a.y)};
}
template <typename R>
__host__ __device__ inline typename FacT<R>::S lnarrow(c64 a) {
  if constexpr (sizeof(typename FacT<R>::S) == sizeof(c16))
    return c16{(_Float16)(float)a.x, (_Float16)(float)a.y};
  else
    return cfrom<R>(a);
}
// Whether a multiplier is representable in the storage: FP16 ends at 65504.
template <typename R>
__host__ __device__ inline bool lfits(c64 a) {
  if constexpr (sizeof(typename FacT<R>::S) == sizeof(c16))
    return fabs(a.x) < 6.0e4 && fabs(a.y) < 6.0e4;
  else
    return true;
}

// L and D^{-1} of every block, one entry per point (block layout).
template <typename R>
struct SegFactor {
  typename FacT<R>::S* l1;   // L(g + 1, g) inside the block (0 at its last row)
  typename FacT<R>::S* l2;   // L(g + 2, g)
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
      ok = ok && lfits<R>(l1[k]) && lfits<R>(l2[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < kSegRows; ++k) {
    if (k < L) {
      const int i = (g0 + k) * Nu + u;
      if (ok) {
        f.l1[i] = lnarrow<R>(l1[k]);
        f.l2[i] = lnarrow<R>(l2[k]);
        f.dinv[i] = narrow<R>(cinv<double>(D[k]));
      } else {
        f.l1[i] = lnarrow<R>(c64{0.0, 0.0});
        f.l2[i] = lnarrow<R>(c64{0.0, 0.0});
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
      if (k >= 1) t = t - lw<R>(f.l1[i - Nu]) * y[k - 1];
      if (k >= 2) t = t - lw<R>(f.l2[i - 2 * Nu]) * y[k - 2];
      y[k] = t;
    }
  }
#pragma unroll
  for (int k = kSegRows - 1; k >= 0; --k) {
    if (k < L) {
      const int i = (g0 + k) * Nu + u;
      C t = f.dinv[i] * y[k];
      if (k + 1 < L) t = t - lw<R>(f.l1[i]) * y[k + 1];
      if (k + 2 < L) t = t - lw<R>(f.l2[i]) * y[k + 2];
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
// ownership again.  z may be q: a block reads all of its q before it writes
// any of its z, and no block reads another block's q.
template <typename R>
__device__ inline void seg_cocg_step(const SegFactor<R>& f, int Ng, int Nu,
                                     typename CT<R>::C alpha,
                                     const typename CT<R>::C* __restrict__ p,
                                     const typename CT<R>::C* q,
                                     typename CT<R>::C* __restrict__ x,
                                     typename CT<R>::C* __restrict__ r,
                                     typename CT<R>::C* z, R* acc) {
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
        if (k >= 1) t = t - lw<R>(f.l1[i - Nu]) * y[k - 1];
        if (k >= 2) t = t - lw<R>(f.l2[i - 2 * Nu]) * y[k - 2];
        y[k] = t;
      }
    }
#pragma unroll
    for (int k = kSegRows - 1; k >= 0; --k) {
      if (k < L) {
        const int i = (g0 + k) * Nu + u;
        C t = f.dinv[i] * y[k];
        if (k + 1 < L) t = t - lw<R>(f.l1[i]) * y[k + 1];
        if (k + 2 < L) t = t - lw<R>(f.l2[i]) * y[k + 2];
        y[k] = t;
        z[i] = t;
        const C rz = rv[k] * t;
        acc[1] += rz.x;
        acc[2] += rz.y;
      }
    }
  }
}


// The same step split in two (the FP32 solvers' form): x += alpha p,
// r -= alpha q and acc[0] += ||r||^2 element by element over all threads
// (kBatch elements per thread in flight; elements past the end re-load the
// last one and store nothing), a barrier, then block by block z = M^{-1} r with acc[1] + i acc[2] +=
// <r|z>_S.  A block's r and factor entries are all loaded before its
// recurrences start (rows past a short block's end re-load its last row and
// are not used), so a thread waits for memory once per block instead of once
// per row; the update pass keeps every wavefront's loads independent.  r is
// read once more than in the fused form.  Begins with a barrier; z may be q.
template <typename R>
__device__ inline void seg_cocg_step_split(const SegFactor<R>& f, int Ng, int Nu,
                                           typename CT<R>::C alpha,
                                           const typename CT<R>::C* __restrict__ p,
                                           const typename CT<R>::C* q,
                                           typename CT<R>::C* __restrict__ x,
                                           typename CT<R>::C* __restrict__ r,
                                           typename CT<R>::C* z, R* acc) {
  using C = typename CT<R>::C;
  __syncthreads();
  const int Nc = Ng * Nu;
  // kBatch elements per thread at a time, all loads before any store
  for (int i0 = threadIdx.x; i0 < Nc; i0 += kBatch * kBlock) {
    C xv[kBatch], pv[kBatch], rv[kBatch], qv[kBatch];
#pragma unroll
    for (int e = 0; e < kBatch; ++e) {
      const int i = min(i0 + e * kBlock, Nc - 1);
      xv[e] = x[i];
      pv[e] = p[i];
      rv[e] = r[i];
      qv[e] = q[i];
    }
#pragma unroll
    for (int e = 0; e < kBatch; ++e) {
      const int i = i0 + e * kBlock;
      if (i < Nc) {
        x[i] = xv[e] + alpha * pv[e];
        const C ri = rv[e] - alpha * qv[e];
        r[i] = ri;
        acc[0] += norm2(ri);
      }
    }
  }
  __syncthreads();
  const int nb = seg_blocks(Ng, Nu);
  for (int c = threadIdx.x; c < nb; c += kBlock) {
    const int u = c % Nu, g0 = (c / Nu) * kSegRows, L = min(kSegRows, Ng - g0);
    C rv[kSegRows], a1[kSegRows], a2[kSegRows], di[kSegRows];
#pragma unroll
    for (int k = 0; k < kSegRows; ++k) {
      const int i = (g0 + min(k, L - 1)) * Nu + u;
      rv[k] = r[i];
      a1[k] = lw<R>(f.l1[i]);
      a2[k] = lw<R>(f.l2[i]);
      di[k] = f.dinv[i];
    }
    C y[kSegRows];
#pragma unroll
    for (int k = 0; k < kSegRows; ++k) {
      C t = rv[k];
      if (k >= 1) t = t - a1[k - 1] * y[k - 1];
      if (k >= 2) t = t - a2[k - 2] * y[k - 2];
      y[k] = t;
    }
#pragma unroll
    for (int k = kSegRows - 1; k >= 0; --k) {
      if (k < L) {
        C t = di[k] * y[k];
        if (k + 1 < L) t = t - a1[k] * y[k + 1];
        if (k + 2 < L) t = t - a2[k] * y[k + 2];
        y[k] = t;
        z[(g0 + k) * Nu + u] = t;
        const C rz = rv[k] * t;
        acc[1] += rz.x;
        acc[2] += rz.y;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Row blocks: the paper's M^g (Sec. III.B), one block per n_g holding its
// whole n_u row (both states; in the symmetry block one point per n_u).
// Inside a row the state alternates with n_u; the couplings that stay in the
// row are the direct -lam q_u, the q_u parts of the sandwiches next to their
// (1 + lam_d q_g) partners (F_AB at either end of the step) and the
// returning q_u F_BB q_u, which reaches n_u +- 2:
//   A(u, u + 1) = -q(u+1) (lam + F_AB(u) + F_AB(u+1)),
//   A(u, u + 2) = -q(u+1) q(u+2) F_BB(u+1),
// with each point's F_AB, F_BB those of its own active state (op2d.h).  The
// rows are factored whole (L D L^T, no pivoting, the same diagonal fallback
// as the column blocks), one thread per row, and stored in the SegFactor
// planes at the points' own positions: l1 = L(u+1, u), l2 = L(u+2, u).
// A row is a serial recurrence of length N_u, so only N_g threads work; the
// paper finds these blocks the most effective for models whose strongest
// coupling runs along q_u (lam of Eq. (18)).

__device__ inline c64 row_off1(const OpJob<double>& op, const double* sq, int i, int u) {
  const double q = sq[u + 1];
  const c64 f = op.AB[i] + op.AB[i + 1];
  return c64{-q * (op.lam + f.x), -q * f.y};
}

__device__ inline c64 row_off2(const OpJob<double>& op, const double* sq, int i, int u) {
  return (-sq[u + 1] * sq[u + 2]) * op.BB[i + 1];
}

// Factor row g (FP64 arithmetic, stored in precision R), one thread.
template <typename R>
__device__ inline void row_factor_row(const OpJob<double>& op, const double* sq,
                                      const SegFactor<R>& f, int g) {
  const int Nu = op.Nu, base = g * Nu;
  c64 Dm1{0.0, 0.0}, Dm2{0.0, 0.0}, l1m1{0.0, 0.0}, l2m1{0.0, 0.0}, l2m2{0.0, 0.0};
  bool ok = true;
  for (int u = 0; u < Nu; ++u) {
    const int i = base + u;
    const c64 akk = op_diag<double>(op, i);
    const c64 d = akk - (l1m1 * l1m1) * Dm1 - (l2m2 * l2m2) * Dm2;
    const double nd = sqrt(norm2(d));
    ok = ok && isfinite(nd) && nd > 1e-12 * sqrt(norm2(akk));
    const c64 di = cinv<double>(d);
    c64 l1{0.0, 0.0}, l2{0.0, 0.0};
    if (u + 1 < Nu) l1 = (row_off1(op, sq, i, u) - (l2m1 * l1m1) * Dm1) * di;
    if (u + 2 < Nu) l2 = row_off2(op, sq, i, u) * di;
    ok = ok && lfits<R>(l1) && lfits<R>(l2);
    f.l1[i] = lnarrow<R>(l1);
    f.l2[i] = lnarrow<R>(l2);
    f.dinv[i] = narrow<R>(di);
    Dm2 = Dm1;
    Dm1 = d;
    l2m2 = l2m1;
    l2m1 = l2;
    l1m1 = l1;
  }
  if (!ok) {
    for (int u = 0; u < Nu; ++u) {
      const int i = base + u;
      f.l1[i] = lnarrow<R>(c64{0.0, 0.0});
      f.l2[i] = lnarrow<R>(c64{0.0, 0.0});
      f.dinv[i] = narrow<R>(cinv<double>(op_diag<double>(op, i)));
    }
  }
}

// Factor every row, spread over the workgroup's threads.  No barrier.
template <typename R>
__device__ inline void row_factor(const OpJob<double>& op, const double* sq,
                                  const SegFactor<R>& f) {
  for (int g = threadIdx.x; g < op.Ng; g += blockDim.x) row_factor_row<R>(op, sq, f, g);
}

// Row g of z = M^{-1} (vscale v), or z += M^{-1} (vscale v) with accumulate,
// one thread.  The forward sweep's L^{-1} values y are parked in z, or in the
// vector park when accumulating (park may be v, which is then overwritten);
// the backward sweep keeps its last two results in registers.  z may be v.
// With dot, acc[0] + i acc[1] += sum_u y_u^2 / D_u = v^T M^{-1} v (vscale
// 1), formed in the backward sweep from the values it loads anyway.
// Every row has the same length, so the loops run in step across a
// wavefront; the loads of RowChunk<R>::K points (4 in FP64, 8 in FP32) are
// issued together, so a sweep waits for memory once per chunk rather than
// once per point.
template <typename R>
struct RowChunk { static constexpr int K = 4; };
template <>
struct RowChunk<float> { static constexpr int K = 8; };

template <typename R, bool dot>
__device__ inline void row_sweep(const SegFactor<R>& f, int Nu, const typename CT<R>::C* v,
                                 R vscale, typename CT<R>::C* z, bool accumulate,
                                 typename CT<R>::C* park, int g, R* acc) {
  using C = typename CT<R>::C;
  constexpr int K = RowChunk<R>::K;
  if (!accumulate) park = z;
  const int base = g * Nu, last = base + Nu - 1;
  C y1 = cz<R>(), y2 = cz<R>();
  for (int u0 = 0; u0 < Nu; u0 += K) {
    C vv[K], a1[K], a2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = min(base + u0 + k, last);
      vv[k] = v[i];
      a1[k] = lw<R>(f.l1[max(i - 1, base)]);
      a2[k] = lw<R>(f.l2[max(i - 2, base)]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int u = u0 + k;
      if (u < Nu) {
        C t = vscale * vv[k];
        if (u >= 1) t = t - a1[k] * y1;
        if (u >= 2) t = t - a2[k] * y2;
        park[base + u] = t;
        y2 = y1;
        y1 = t;
      }
    }
  }
  C z1 = cz<R>(), z2 = cz<R>();
  for (int u0 = Nu - 1; u0 >= 0; u0 -= K) {
    C yy[K], dd[K], a1[K], a2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = max(base + u0 - k, base);
      yy[k] = park[i];
      dd[k] = f.dinv[i];
      a1[k] = lw<R>(f.l1[i]);
      a2[k] = lw<R>(f.l2[i]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int u = u0 - k;
      if (u >= 0) {
        const C w = dd[k] * yy[k];
        if (dot) {
          const C yw = yy[k] * w;
          acc[0] += yw.x;
          acc[1] += yw.y;
        }
        C t = w;
        if (u + 1 < Nu) t = t - a1[k] * z1;
        if (u + 2 < Nu) t = t - a2[k] * z2;
        const int i = base + u;
        z[i] = accumulate ? z[i] + t : t;
        z2 = z1;
        z1 = t;
      }
    }
  }
}

template <typename R>
__device__ inline void row_apply_row(const SegFactor<R>& f, int Nu, const typename CT<R>::C* v,
                                     R vscale, typename CT<R>::C* z, bool accumulate,
                                     typename CT<R>::C* park, int g) {
  row_sweep<R, false>(f, Nu, v, vscale, z, accumulate, park, g, nullptr);
}

// The whole vector, rows spread over the workgroup's threads.  Begins with a
// barrier, ends without.
template <typename R>
__device__ inline void row_apply(const SegFactor<R>& f, int Ng, int Nu,
                                 const typename CT<R>::C* v, R vscale, typename CT<R>::C* z,
                                 bool accumulate, typename CT<R>::C* park) {
  __syncthreads();
  for (int g = threadIdx.x; g < Ng; g += blockDim.x)
    row_apply_row<R>(f, Nu, v, vscale, z, accumulate, park, g);
}

// seg_cocg_step with rows: x += alpha p, r -= alpha q and acc[0] += ||r||^2
// element by element over all threads, a barrier, then z = M^{-1} r row by
// row with acc[1] + i acc[2] += <r|z>_S = r^T (L D L^T)^{-1} r, summed as
// y^T D^{-1} y with y = L^{-1} r.  Begins with a barrier; x and r are read
// once more by the rows than in the fused column version.  z may be q (q is
// read only before the barrier).
template <typename R>
__device__ inline void row_cocg_step(const SegFactor<R>& f, int Ng, int Nu,
                                     typename CT<R>::C alpha,
                                     const typename CT<R>::C* __restrict__ p,
                                     const typename CT<R>::C* q,
                                     typename CT<R>::C* __restrict__ x,
                                     typename CT<R>::C* __restrict__ r,
                                     typename CT<R>::C* z, R* acc) {
  using C = typename CT<R>::C;
  __syncthreads();
  const int Nc = Ng * Nu;
  for (int i = threadIdx.x; i < Nc; i += blockDim.x) {
    x[i] = x[i] + alpha * p[i];
    const C ri = r[i] - alpha * q[i];
    r[i] = ri;
    acc[0] += norm2(ri);
  }
  __syncthreads();
  for (int g = threadIdx.x; g < Ng; g += blockDim.x)
    row_sweep<R, true>(f, Nu, r, R(1), z, false, nullptr, g, acc + 1);
}

// Dispatch on the preconditioner: VDC_PREC_BLOCK (column segments) or
// VDC_PREC_ROWS (whole rows) share the factor planes.  The solver kernels are
// instantiated per choice (rows true or false), so neither pays registers for
// the other's code.
__host__ __device__ inline bool prec_has_factor(int precond) {
  return precond == VDC_PREC_BLOCK || precond == VDC_PREC_ROWS;
}

template <bool rows, typename R>
__device__ inline void prec_factor(const OpJob<double>& op, const double* sq,
                                   const SegFactor<R>& f) {
  if constexpr (rows) row_factor<R>(op, sq, f);
  else seg_factor<R>(op, sq, f);
}

// park: scratch for the row variant's forward sweep when accumulating (may
// be v); unused otherwise.
template <bool rows, typename R>
__device__ inline void prec_apply(const SegFactor<R>& f, int Ng, int Nu,
                                  const typename CT<R>::C* v, R vscale, typename CT<R>::C* z,
                                  bool accumulate, typename CT<R>::C* park = nullptr) {
  if constexpr (rows) row_apply<R>(f, Ng, Nu, v, vscale, z, accumulate, park);
  else seg_apply<R>(f, Ng, Nu, v, vscale, z, accumulate);
}

template <bool rows, typename R>
__device__ inline void prec_cocg_step(const SegFactor<R>& f, int Ng, int Nu,
                                      typename CT<R>::C alpha,
                                      const typename CT<R>::C* __restrict__ p,
                                      const typename CT<R>::C* q,
                                      typename CT<R>::C* __restrict__ x,
                                      typename CT<R>::C* __restrict__ r,
                                      typename CT<R>::C* z, R* acc) {
  if constexpr (rows) row_cocg_step<R>(f, Ng, Nu, alpha, p, q, x, r, z, acc);
  else if constexpr (sizeof(R) == 4) seg_cocg_step_split<R>(f, Ng, Nu, alpha, p, q, x, r, z, acc);
  else seg_cocg_step<R>(f, Ng, Nu, alpha, p, q, x, r, z, acc);
}

}  // namespace vdc
