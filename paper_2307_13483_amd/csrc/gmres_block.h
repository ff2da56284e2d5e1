// Restarted GMRES(m) in complex FP64 on one symmetry block, run by a whole
// workgroup (Sec. III.A, right preconditioning of Sec. III.B by the diagonal
// of A or by its column or row blocks, segprec.h): cycles of krylov_cycle,
// x += M^{-1} V y, and the FP64 true residual b - A x deciding convergence
// (the stopping rule of Sec. III).  Shared by the forward solver and the
// adjoint (transposed) solve: A^T = A, and M^T = M for both preconditioners.
#pragma once
#include "krylov.h"
#include "segprec.h"

namespace vdc {

struct Fp64Lds {
  KrylovLds<double> K;
  double red[kRedSize];
  double sq[kSqMax + 1];
  int job;
};

// Per-workgroup vectors of the FP64 solver (leading dimension ld): dinv is
// 1/diag(A) for the diagonal preconditioner and D^{-1} of the block factors
// (with l1, l2) for the block one; zt holds M^{-1} of the vector in work.
struct Fp64Slot {
  c64 *V, *x, *b, *dinv, *w, *wA, *wB, *l1, *l2, *zt, *Rm, *extra;
};

__device__ inline Fp64Slot fp64_slot(c64* slot, size_t ld, int m) {
  Fp64Slot s;
  s.V = slot;
  s.x = slot + (size_t)(m + 1) * ld;
  s.b = s.x + ld;
  s.dinv = s.b + ld;
  s.w = s.dinv + ld;
  s.wA = s.w + ld;
  s.wB = s.wA + ld;
  s.l1 = s.wB + ld;
  s.l2 = s.l1 + ld;
  s.zt = s.l2 + ld;
  s.Rm = s.zt + ld;
  s.extra = s.Rm + (size_t)(m + 1) * m;
  return s;
}

struct BlockSolve {
  int status, iters, cycles;
  double bnorm, beta, passes;
};

// The preconditioner (dinv = 1/diag(A) or 1, or the block factors) and
// x = 0, b = 0 over the block.  No barrier.
template <bool rows>
__device__ inline void fp64_prepare(const OpJob<double>& op, const double* sq, const Fp64Slot& s,
                                    int precond) {
  const bool blk = prec_has_factor(precond);
  if (blk) prec_factor<rows, double>(op, sq, SegFactor<double>{s.l1, s.l2, s.dinv});
  for (int i = threadIdx.x; i < op.Nc; i += kBlock) {
    if (!blk)
      s.dinv[i] = precond == VDC_PREC_JACOBI ? cinv<double>(op_diag<double>(op, i)) : c64{1.0, 0.0};
    s.x[i] = c64{0.0, 0.0};
    s.b[i] = c64{0.0, 0.0};
  }
}

// Dynamic LDS of the solver kernels: the tiles of matvec_tiled.
extern __shared__ __align__(16) char vdc_tile_lds[];

// Solves A x = b with b in s.b (complete and visible: call after a barrier).
// Byte model (passes over a block vector of Nc complex FP64 values): setup 8
// (two table planes read for the diagonal; dinv, x, b written; b read for its
// norm and copied to V_0), each cycle of k steps cycle_passes(k) + k + 9:
// x update k + 3 (basis, dinv, x in; x out) and the true residual b - A x
// written into V_0 in the operator's pass (x, 3 table planes, b in; V_0 out).
// The block preconditioner adds 4 passes to every step (M^{-1} reads the
// vector and three factor planes and writes zt, the operator reads zt but no
// dinv), 4 to the x update (sum written to zt and read back with the factor,
// x in and out) and 3 to the setup (factor: one more table plane, three
// planes written instead of one).
template <bool rows>
__device__ inline BlockSolve gmres_fp64_block(Fp64Lds& L, const OpJob<double>& op,
                                              const Fp64Slot& s, size_t ld, int m, double tol,
                                              int max_iter, int T, int precond,
                                              double* hist = nullptr, int hist_len = 0) {
  const int Nc = op.Nc;
  const bool blk = prec_has_factor(precond);
  const SegFactor<double> fac{s.l1, s.l2, s.dinv};
  c64* lds = reinterpret_cast<c64*>(vdc_tile_lds);
  BlockSolve r{VDC_NOT_CONVERGED, 0, 0, 0.0, 0.0, blk ? 11.0 : 8.0};
  r.bnorm = sqrt(norm_sq<double>(s.b, Nc, L.red));
  r.beta = r.bnorm;
  if (!(r.bnorm > 0.0) || !isfinite(r.bnorm)) {
    r.status = isfinite(r.bnorm) ? VDC_CONVERGED : VDC_NONFINITE;
    r.beta = 0.0;
    return r;
  }
  for (int i = threadIdx.x; i < Nc; i += kBlock) s.V[i] = s.b[i];
  auto apply = [&](int j, double sc, c64* out) {
    if (blk) {
      prec_apply<rows, double>(fac, op.Ng, op.Nu, s.V + (size_t)j * ld, sc, s.zt, false);
      apply_A<double>(op, L.sq, s.zt, 1.0, nullptr, out, lds, T, s.wA, s.wB);
    } else {
      apply_A<double>(op, L.sq, s.V + (size_t)j * ld, sc, s.dinv, out, lds, T, s.wA, s.wB);
    }
  };
  for (;;) {
    if (threadIdx.x == 0) {
      L.K.g[0] = c64{r.beta, 0.0};
      L.K.vs[0] = 1.0 / r.beta;
    }
    __syncthreads();
    const CycleResult cr = krylov_cycle<double>(L.K, L.red, s.V, ld, Nc, m, tol * r.bnorm,
                                                max_iter, r.iters, s.Rm, apply, hist, hist_len,
                                                1.0 / r.bnorm);
    r.passes += cycle_passes(cr.k, cr.reorth_passes) + cr.k + 9.0 + (blk ? 4.0 * cr.k + 4.0 : 0.0);
    if (blk) {
      // zt = V y (own elements), then x += M^{-1} zt (block ownership)
      update_x<double>(s.V, ld, cr.k, L.K.y, L.K.vs, nullptr, s.zt, Nc, true);
      prec_apply<rows, double>(fac, op.Ng, op.Nu, s.zt, 1.0, s.x, true, s.zt);
    } else {
      update_x<double>(s.V, ld, cr.k, L.K.y, L.K.vs, s.dinv, s.x, Nc);
    }
    // true residual b - A x, written into V_0 (the next cycle's start)
    r.beta = sqrt(residual_A<double>(op, L.sq, s.x, s.b, s.V, lds, T, s.wA, s.wB, L.red));
    ++r.cycles;
    if (!isfinite(r.beta) || cr.nonfinite) {
      r.status = VDC_NONFINITE;
      break;
    }
    if (r.beta <= tol * r.bnorm) {
      r.status = VDC_CONVERGED;
      break;
    }
    if (cr.breakdown) {
      r.status = VDC_BREAKDOWN;
      break;
    }
    if (r.iters >= max_iter) {
      r.status = VDC_NOT_CONVERGED;
      break;
    }
  }
  return r;
}

}  // namespace vdc
