// Mixed precision on chip: flexible GMRES in complex FP64 (outer) whose
// variable right preconditioner is one cycle of GMRES run entirely in complex
// FP32 (inner: FP32 basis, FP32 level-shift tables, FP32 stencil, FP32 dot
// products accumulated in FP32, FP32 preconditioner: the diagonal or the
// column- or row-block factors of segprec.h).  The outer level keeps
// everything that decides the answer in FP64: the operator applied to the
// inner results, its Gram-Schmidt, the Hessenberg least squares by Givens, the
// solution update, the true residual b - A x and the amplitudes.  Because
// the outer basis Z of preconditioned vectors is stored (A Z_k = V_{k+1} H_k),
// the inner solve may differ from step to step and the outer residual
// estimate stays that of the FP64 operator.
//
// One job per workgroup, jobs popped from a device queue as in the FP64
// solver; "iters" counts inner FP32 Arnoldi steps (the bulk of the bytes),
// "outer" the FP64 outer steps.
#include "gmres_block.h"
#include "solve_args.h"

namespace vdc {

struct MixedLds {
  KrylovLds<double> Ko;
  KrylovLds<float> Ki;
  double red[kRedSize];
  float redf[kRedSize];
  double sq[kSqMax + 1];
  float sqf[kSqMax + 1];
  int job;
};

template <bool rows, bool diag>
__global__ void __launch_bounds__(kBlock)
fgmres_mixed_kernel(SolveArgs a) {
  __shared__ MixedLds L;
  fill_sq<double>(L.sq);
  fill_sq<float>(L.sqf);
  const int tid = threadIdx.x;
  const int m = a.m, mi = a.m_in;
  const size_t ld = a.ncap;
  c64* lds64 = reinterpret_cast<c64*>(vdc_tile_lds);
  c32* lds32 = reinterpret_cast<c32*>(vdc_tile_lds);
  c64* slot = a.scratch + (size_t)blockIdx.x * a.slot_elems;
  // FP64 part
  c64* Vo = slot;                                 // (m+1) x ld
  c64* Z = Vo + (size_t)(m + 1) * ld;             // m x ld
  c64* x = Z + (size_t)m * ld;
  c64* b = x + ld;
  c64* w = b + ld;                                // unused by the tiled operator
  c64* wA = w + ld;
  c64* wB = wA + ld;
  c64* Ro = wB + ld;                              // (m+1) x m
  c64* Ri = Ro + (size_t)(m + 1) * m;             // (mi+1) x mi
  // FP32 part
  c32* Vi = reinterpret_cast<c32*>(Ri + (size_t)(mi + 1) * mi);   // (mi+1) x ld
  c32* dinv = Vi + (size_t)(mi + 1) * ld;        // 1/diag(A), or D^{-1} of the blocks
  c32* w32 = dinv + ld;
  c32* wA32 = w32 + ld;
  c32* wB32 = wA32 + ld;
  c16* l1 = reinterpret_cast<c16*>(wB32 + ld);  // block multipliers (segprec.h), FP16:
  c16* l2 = l1 + ld;                             //   both in one plane
  c32* zt = wB32 + 2 * ld;                             // M^{-1} of the inner vector in work
  (void)w;
  (void)w32;
  const bool blk = prec_has_factor(a.precond);
  const SegFactor<float> fac{l1, l2, dinv};

  for (;;) {
    __syncthreads();
    if (tid == 0) L.job = atomicAdd(a.counter, 1);
    __syncthreads();
    const int js = L.job;
    if (js >= a.n_jobs) break;
    const DevJob jb = a.jobs[js];
    const DevModel& md = a.models[jb.model];
    const DevTable tb = a.tabs[jb.table];
    const size_t toff = tb.offset + (size_t)(jb.parity * a.planes) * md.Nc;
    const OpJob<double> op = make_op<double>(md, jb, a.tables + toff);
    const OpJob<float> op32 = make_op<float>(md, jb, a.tables32 + toff);
    const int Nc = md.Nc;

    if (blk) prec_factor<rows, float>(op, L.sq, fac);
    for (int i = tid; i < Nc; i += kBlock) {
      if (!blk) {
        const c64 d = a.precond == VDC_PREC_JACOBI ? cinv<double>(op_diag<double>(op, i))
                                                    : c64{1.0, 0.0};
        dinv[i] = c32{(float)d.x, (float)d.y};
      }
      x[i] = c64{0.0, 0.0};
      b[i] = c64{0.0, 0.0};
    }
    __syncthreads();
    if (tid == 0) {
      PhiEntry e[6];
      const int n = phi_entries(md, jb.mu, jb.eps_i, jb.vi_g, jb.vi_u, e);
      for (int q = 0; q < n; ++q) b[e[q].g * md.Nu + e[q].u] = c64{e[q].val, 0.0};
    }
    __syncthreads();
    const double bnorm = sqrt(norm_sq<double>(b, Nc, L.red));
    double beta = bnorm;
    int iters = 0, outer = 0, cycles = 0, status = VDC_NOT_CONVERGED;
    // byte model in passes over a block vector of Nc values, p64 in complex
    // FP64 (16 B) and p32 in complex FP32 (8 B):
    //   setup: two FP64 table planes (diagonal), x, b written, b read, V_0
    //     copied (p64 7); FP32 dinv written (p32 1)
    //   outer step (cycle_passes counts 6 p64 for its operator: v_j read in
    //     the cast and the FP64 operator on z_j): v_j cast (1 p32), inner
    //     cycle of k steps (cycle_passes(k) p32), z_j = dinv V y (k + 1 p32,
    //     1 p64)
    //   outer cycle of k_o steps: x += Z y (k_o + 2 p64), residual (6 p64)
    // The block preconditioner adds: setup one more FP64 table plane and the
    // two FP16 multiplier planes written (p64 1, p32 1); every inner step
    // M^{-1} (vector, 1/D and the multipliers read: 2, zt written) before an
    // operator that reads zt but no dinv (p32 3); z_j: the sum written to
    // zt, M^{-1} in place (zt and the factor read, zt written), zt read for
    // the widening (p32 6 instead of 1).
    double p64 = blk ? 8.0 : 7.0, p32 = blk ? 2.0 : 1.0;
    if (!(bnorm > 0.0) || !isfinite(bnorm)) {
      status = isfinite(bnorm) ? VDC_CONVERGED : VDC_NONFINITE;
      beta = 0.0;
    } else {
      for (int i = tid; i < Nc; i += kBlock) Vo[i] = b[i];
      // inner FP32 operator: A (s dinv v)
      auto apply_in = [&](int j, float sc, c32* out) {
        if (blk) {
          prec_apply<rows, float>(fac, md.Ng, md.Nu, Vi + (size_t)j * ld, sc, zt, false);
          apply_A<float>(op32, L.sqf, zt, 1.0f, nullptr, out, lds32, a.tileT32, wA32, wB32);
        } else {
          apply_A<float>(op32, L.sqf, Vi + (size_t)j * ld, sc, dinv, out, lds32, a.tileT32, wA32,
                         wB32);
        }
      };
      // outer step j: Z_j = inner(s V_j), out = A Z_j in FP64
      auto apply_out = [&](int j, double sc, c64* out) {
        const c64* v = Vo + (size_t)j * ld;
        float acc[1] = {0.f};
        for (int i = tid; i < Nc; i += kBlock) {
          const c32 t = c32{(float)(sc * v[i].x), (float)(sc * v[i].y)};
          Vi[i] = t;
          acc[0] += norm2(t);
        }
        block_sum<1, float>(acc, L.redf, L.redf + kWaves);
        const double n0 = sqrt((double)L.redf[kWaves]);
        __syncthreads();
        c64* z = Z + (size_t)j * ld;
        p32 += 1.0;
        if (n0 > 0.0) {
          if (tid == 0) {
            L.Ki.g[0] = c64{n0, 0.0};
            L.Ki.vs[0] = (float)(1.0 / n0);
          }
          __syncthreads();
          const CycleResult ci = krylov_cycle<float>(L.Ki, L.redf, Vi, ld, Nc, mi,
                                                     a.tol_in * n0, a.max_iter, iters, Ri,
                                                     apply_in);
          // z = M^{-1} sum_l (vs_l Vi_l) y_l, widened to FP64
          for (int i = tid; i < Nc; i += kBlock) {
            c32 s = c32{0.f, 0.f};
            int l = 0;
            for (; l + kChunk <= ci.k; l += kChunk) {
              c32 vv[kChunk];
#pragma unroll
              for (int q = 0; q < kChunk; ++q) vv[q] = Vi[(size_t)(l + q) * ld + i];
#pragma unroll
              for (int q = 0; q < kChunk; ++q) {
                const float f = L.Ki.vs[l + q];
                s = s + vv[q] * c32{(float)L.Ki.y[l + q].x * f, (float)L.Ki.y[l + q].y * f};
              }
            }
            for (; l < ci.k; ++l) {
              const float f = L.Ki.vs[l];
              s = s + Vi[(size_t)l * ld + i] * c32{(float)L.Ki.y[l].x * f, (float)L.Ki.y[l].y * f};
            }
            if (blk) {
              zt[i] = s;
            } else {
              const c32 t = dinv[i] * s;
              z[i] = c64{(double)t.x, (double)t.y};
            }
          }
          if (blk) {
            prec_apply<rows, float>(fac, md.Ng, md.Nu, zt, 1.0f, zt, false);
            __syncthreads();
            for (int i = tid; i < Nc; i += kBlock) z[i] = c64{(double)zt[i].x, (double)zt[i].y};
          }
          p32 += cycle_passes(ci.k, ci.reorth_passes) + ci.k + 1.0 +
                 (blk ? 3.0 * ci.k + 5.0 : 0.0);
        } else {
          for (int i = tid; i < Nc; i += kBlock) z[i] = c64{0.0, 0.0};
        }
        p64 += 1.0;
        apply_A<double>(op, L.sq, z, 1.0, nullptr, out, lds64, a.tileT, wA, wB);
        ++outer;
      };
      int ocount = 0;
      for (;;) {
        if (tid == 0) {
          L.Ko.g[0] = c64{beta, 0.0};
          L.Ko.vs[0] = 1.0 / beta;
        }
        __syncthreads();
        const CycleResult cr = krylov_cycle<double>(L.Ko, L.red, Vo, ld, Nc, m, a.tol * bnorm,
                                                    1 << 30, ocount, Ro, apply_out,
                                                    hist_row<diag>(a, jb), a.hist_len, 1.0 / bnorm);
        p64 += cycle_passes(cr.k, cr.reorth_passes) + cr.k + 2.0 + 6.0;
        // x += Z y (Z_l is the preconditioned unit basis vector l)
        update_x<double>(Z, ld, cr.k, L.Ko.y, nullptr, nullptr, x, Nc);
        // FP64 true residual into V_0
        beta = sqrt(residual_A<double>(op, L.sq, x, b, Vo, lds64, a.tileT, wA, wB, L.red));
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
    finish_job<diag>(a, md, jb, x, tid, status, iters, cycles, outer,
               bnorm > 0.0 ? beta / bnorm : 0.0, (16.0 * p64 + 8.0 * p32) * Nc);
  }
}

hipError_t launch_fgmres_mixed(const SolveArgs& a, int n_groups, size_t dyn_lds, hipStream_t s) {
  const bool rows = a.precond == VDC_PREC_ROWS, diag = a.check_optical || a.hist;
  if (rows && diag)
    hipLaunchKernelGGL((fgmres_mixed_kernel<true, true>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else if (rows)
    hipLaunchKernelGGL((fgmres_mixed_kernel<true, false>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else if (diag)
    hipLaunchKernelGGL((fgmres_mixed_kernel<false, true>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else
    hipLaunchKernelGGL((fgmres_mixed_kernel<false, false>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  return hipGetLastError();
}

int fgmres_mixed_occupancy(size_t dyn_lds) {
  return std::min(std::min(occupancy_of(fgmres_mixed_kernel<true, true>, dyn_lds),
                           occupancy_of(fgmres_mixed_kernel<true, false>, dyn_lds)),
                  std::min(occupancy_of(fgmres_mixed_kernel<false, true>, dyn_lds),
                           occupancy_of(fgmres_mixed_kernel<false, false>, dyn_lds)));
}

}  // namespace vdc
