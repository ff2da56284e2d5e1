// Complex FP64 COCG (Sec. III.A) for one job by one workgroup, on chip:
// conjugate gradients with the symmetrized bilinear form <a|b>_S =
// sum_i a_i b_i, for the complex symmetric A of the model, preconditioned as
// M^{-1} A M^{-T} (Sec. III.B) with K = M M^T the diagonal of A, its column
// blocks or its rows (segprec.h; all symmetric), in the coupled two-term
// form:
//   r = b, z = K^{-1} r, p = z, rho = <r|z>_S;
//   repeat: q = A p, mu = <p|q>_S (in the operator's pass), alpha = rho/mu,
//           x += alpha p, r -= alpha q, z = K^{-1} r, rho' = <r|z>_S,
//           p = z + (rho'/rho) p.
// Short recurrences: no basis is stored and no orthogonalisation pass is
// made.  When ||r|| <= tol ||b|| the FP64 true residual b - A x decides
// (stopping rule of Sec. III); if it is larger the iteration restarts from
// it.  A vanishing <p|q>_S or <r|z>_S (the form is not definite) restarts
// from the true residual once, and is reported as a breakdown if it recurs
// at once.  Used by the forward solver and by the adjoint (A^T = A).
#pragma once
#include "gmres_block.h"

namespace vdc {

// Byte model (passes over a block vector of Nc complex FP64 values):
// setup: the preconditioner and x, b (as the FP64 GMRES: 5, block 8), ||b||
// (1), r = b (2), z = K^{-1} r into p with rho (diagonal: r, dinv in, p out:
// 3; block: r and 3 factor planes in, p out, then r, p for rho: 7);
// iteration: the operator (p and 3 table planes in, q out: 5, <p|q>_S from
// the staged p), the update of x and r with rho' (x, p, r, q in, x, r out,
// and dinv in: 7; column blocks, fused with z = K^{-1} r: 3 factor planes
// in and z out as well: 10; rows: the update element by element, then the
// row sweeps (r and 2 factor planes in, L^{-1} r parked in z; z and 3 factor
// planes in, z out): 15), the next direction (diagonal: r, dinv, p in, p
// out: 4; block: z, p in, p out: 3); a true-residual check 6 (+ the setup's
// z, rho and p passes on a restart).
//
// Solves A x = b with b in s.b (complete and visible: call after a barrier)
// and s.x = 0 and the preconditioner prepared (fp64_prepare); r, p, q, z are
// the slot's first four basis vectors.  red: kRedSize doubles of LDS, dot:
// 2 doubles of LDS, sq: the sqrt table in LDS.  "cycles" of the result
// counts the restarts from the true residual.
template <bool rows>
__device__ inline BlockSolve cocg_fp64_block(double* red, double* dot, const double* sq,
                                             const OpJob<double>& op, const Fp64Slot& s,
                                             size_t ld, double tol, int max_iter, int T,
                                             int precond, double* hist = nullptr,
                                             int hist_len = 0) {
  const int tid = threadIdx.x;
  const int Nc = op.Nc;
  c64* lds = reinterpret_cast<c64*>(vdc_tile_lds);
  c64* r = s.V;
  c64* p = s.V + ld;
  c64* q = s.V + 2 * ld;
  c64* z = s.V + 3 * ld;
  const bool blk = prec_has_factor(precond);
  const SegFactor<double> fac{s.l1, s.l2, s.dinv};
  double passes = blk ? 9.0 : 6.0;
  const double bnorm = sqrt(norm_sq<double>(s.b, Nc, red));
  for (int i = tid; i < Nc; i += kBlock) r[i] = s.b[i];
  passes += 2.0;
  // p = z = K^{-1} r and rho = <r|z>_S (own elements; block: after its
  // own barrier)
  auto restart_direction = [&]() -> c64 {
    double acc[2] = {0.0, 0.0};
    if (blk) {
      prec_apply<rows, double>(fac, op.Ng, op.Nu, r, 1.0, p, false);
      __syncthreads();
      for (int i = tid; i < Nc; i += kBlock) {
        const c64 t = r[i] * p[i];
        acc[0] += t.x;
        acc[1] += t.y;
      }
      passes += 7.0;
    } else {
      for (int i = tid; i < Nc; i += kBlock) {
        const c64 zi = s.dinv[i] * r[i];
        p[i] = zi;
        const c64 t = r[i] * zi;
        acc[0] += t.x;
        acc[1] += t.y;
      }
      passes += 3.0;
    }
    block_sum<2, double>(acc, red, red + kWaves * 2);
    const c64 rho = c64{red[kWaves * 2], red[kWaves * 2 + 1]};
    __syncthreads();
    return rho;
  };
  int iters = 0, restarts = 0, status = VDC_NOT_CONVERGED;
  double beta_true = bnorm;
  if (!(bnorm > 0.0) || !isfinite(bnorm)) {
    status = isfinite(bnorm) ? VDC_CONVERGED : VDC_NONFINITE;
    beta_true = 0.0;
  } else {
    c64 rho = restart_direction();
    bool fresh = true;   // p was just reset from the true residual
    for (;;) {
      // q = A p and mu = <p|q>_S
      double mu[2] = {0.0, 0.0};
      if (T > 0) {
        matvec_tiled<double>(op, sq, p, 1.0, nullptr, q, lds, T, nullptr, red, dot);
        mu[0] = dot[0];
        mu[1] = dot[1];
      } else {
        matvec_block<double>(op, sq, p, nullptr, s.wA, s.wB, q);
        double acc[2] = {0.0, 0.0};
        for (int i = tid; i < Nc; i += kBlock) {
          const c64 t = p[i] * q[i];
          acc[0] += t.x;
          acc[1] += t.y;
        }
        block_sum<2, double>(acc, red, red + kWaves * 2);
        mu[0] = red[kWaves * 2];
        mu[1] = red[kWaves * 2 + 1];
        __syncthreads();
        passes += 2.0;
      }
      passes += 5.0;
      const c64 muc = c64{mu[0], mu[1]};
      const double mn = norm2(muc), rn = norm2(rho);
      if (!(mn > 0.0) || !(rn > 0.0) || !isfinite(mn) || !isfinite(rn)) {
        // breakdown of the bilinear form: restart from the true residual
        // once; at once again, give up
        if (fresh) {
          status = (isfinite(mn) && isfinite(rn)) ? VDC_BREAKDOWN : VDC_NONFINITE;
          break;
        }
        beta_true = sqrt(residual_A<double>(op, sq, s.x, s.b, r, lds, T, s.wA, s.wB, red));
        passes += 6.0;
        if (beta_true <= tol * bnorm) {
          status = VDC_CONVERGED;
          break;
        }
        rho = restart_direction();
        ++restarts;
        fresh = true;
        continue;
      }
      const c64 alpha = cdiv(rho, muc);
      // x += alpha p, r -= alpha q, ||r||^2 and rho' = <r|K^{-1} r>_S in one
      // pass (block: by column blocks or rows, z = K^{-1} r stored)
      double acc[3] = {0.0, 0.0, 0.0};
      if (blk) {
        prec_cocg_step<rows, double>(fac, op.Ng, op.Nu, alpha, p, q, s.x, r, z, acc);
      } else {
        for (int i = tid; i < Nc; i += kBlock) {
          s.x[i] = s.x[i] + alpha * p[i];
          const c64 ri = r[i] - alpha * q[i];
          r[i] = ri;
          acc[0] += norm2(ri);
          const c64 t = ri * (s.dinv[i] * ri);
          acc[1] += t.x;
          acc[2] += t.y;
        }
      }
      block_sum<3, double>(acc, red, red + kWaves * 3);
      const double rr = red[kWaves * 3];
      const c64 rho_new = c64{red[kWaves * 3 + 1], red[kWaves * 3 + 2]};
      __syncthreads();
      passes += blk ? (rows ? 15.0 : 10.0) : 7.0;
      ++iters;
      if (hist && tid == 0 && iters <= hist_len) hist[iters - 1] = sqrt(rr) / bnorm;
      fresh = false;
      if (!isfinite(rr)) {
        status = VDC_NONFINITE;
        break;
      }
      if (sqrt(rr) <= tol * bnorm || iters >= max_iter) {
        // the true residual decides; restart from it if needed
        beta_true = sqrt(residual_A<double>(op, sq, s.x, s.b, r, lds, T, s.wA, s.wB, red));
        passes += 6.0;
        if (beta_true <= tol * bnorm) {
          status = VDC_CONVERGED;
          break;
        }
        if (!isfinite(beta_true)) {
          status = VDC_NONFINITE;
          break;
        }
        if (iters >= max_iter) break;
        rho = restart_direction();
        ++restarts;
        fresh = true;
        continue;
      }
      const c64 beta = cdiv(rho_new, rho);
      rho = rho_new;
      for (int i = tid; i < Nc; i += kBlock) {
        const c64 zi = blk ? z[i] : s.dinv[i] * r[i];
        p[i] = zi + beta * p[i];
      }
      passes += blk ? 3.0 : 4.0;
    }
  }

  return BlockSolve{status, iters, restarts, bnorm, beta_true, passes};
}

}  // namespace vdc
