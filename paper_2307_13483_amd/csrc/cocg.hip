// Persistent batched COCG in complex FP64 (Sec. III.A), one job per
// workgroup at a time, the whole solve on chip (cocg_block.h).  Every wave
// reaches the queue-exhausted exit.
#include "cocg_block.h"
#include "solve_args.h"

namespace vdc {

struct CocgLds {
  double red[kRedSize];
  double sq[kSqMax + 1];
  double dot[2];
  int job;
};

template <bool rows, bool diag>
__global__ void __launch_bounds__(kBlock) cocg_fp64_kernel(SolveArgs a) {
  __shared__ CocgLds L;
  fill_sq<double>(L.sq);
  const int tid = threadIdx.x;
  const Fp64Slot s = fp64_slot(a.scratch + (size_t)blockIdx.x * a.slot_elems, a.ncap, 4);
  for (;;) {
    __syncthreads();
    if (tid == 0) L.job = atomicAdd(a.counter, 1);
    __syncthreads();
    const int js = L.job;
    if (js >= a.n_jobs) break;
    const DevJob jb = a.jobs[js];
    const DevModel& md = a.models[jb.model];
    const DevTable tb = a.tabs[jb.table];
    const OpJob<double> op = make_op<double>(
        md, jb, a.tables + tb.offset + (size_t)(jb.parity * a.planes) * md.Nc);
    fp64_prepare<rows>(op, L.sq, s, a.precond);
    __syncthreads();
    if (tid == 0) {
      PhiEntry e[6];
      const int n = phi_entries(md, jb.mu, jb.eps_i, jb.vi_g, jb.vi_u, e);
      for (int k = 0; k < n; ++k) s.b[e[k].g * md.Nu + e[k].u] = c64{e[k].val, 0.0};
    }
    __syncthreads();
    const BlockSolve r = cocg_fp64_block<rows>(L.red, L.dot, L.sq, op, s, a.ncap, a.tol,
                                               a.max_iter, a.tileT, a.precond,
                                               hist_row<diag>(a, jb), a.hist_len);
    __syncthreads();
    finish_job<diag>(a, md, jb, s.x, tid, r.status, r.iters, r.cycles, 0,
               r.bnorm > 0.0 ? r.beta / r.bnorm : 0.0, r.passes * 16.0 * md.Nc);
  }
}

// Mixed precision (the pattern of the FP32-inner solver): FP64 iterative
// refinement whose correction equations A d = r / ||r|| are solved by COCG
// entirely in complex FP32 (FP32 tables, stencil, preconditioner and
// bilinear forms accumulated in FP32) to the relative residual tol_in, or
// m_in steps: every outer step forms the FP64 true residual b - A x, which
// decides convergence, casts it to FP32, runs the inner COCG from d = 0 and
// adds ||r|| d to x in FP64.  "iters" counts inner FP32 steps, "outer" the
// refinement steps.
//
// Byte model (p64: passes of complex FP64, p32 of complex FP32): setup as the
// FP64 COCG's preconditioner (p64 5, block: p64 1 and p32 2 for the FP32
// factors: 1/D, and the two FP16 multiplier planes, each half a p32) plus
// x, b; per outer step the residual (x, 3 table planes, b in, r out: p64 6),
// its cast (p64 1, p32 1), the inner start (r, dinv in, p out, then r, p for
// rho: p32 3; column blocks: r and the factor in, p out, r and p: 6; rows:
// the forward sweeps parking L^{-1} r in p and the backward sweeps, then r
// and p: 9) and x += ||r|| d (p64 2, p32 1); per inner step the operator
// (p32 5), the update of d and r with rho' (diagonal: d, p, r, q, dinv in, d,
// r out: p32 7; column blocks: d, p, r, q in, d, r out, then the sweeps with
// r and the factor (2) in, z out: p32 10; rows: the same update, then the
// forward sweeps (r and the multipliers in, L^{-1} r parked in z: 3) and the
// backward sweeps (z and the factor in, z out: 4): p32 13) and the next
// direction (diagonal: r, dinv, p in, p out: p32 4; block: z, p in, p out:
// p32 3).
struct CocgMixedLds {
  double red[kRedSize];
  float redf[kRedSize];
  double sq[kSqMax + 1];
  float sqf[kSqMax + 1];
  float dot[2];
  int job;
};

template <bool rows, bool diag>
__global__ void __launch_bounds__(kBlock) cocg_mixed_kernel(SolveArgs a) {
  __shared__ CocgMixedLds L;
  fill_sq<double>(L.sq);
  fill_sq<float>(L.sqf);
  const int tid = threadIdx.x;
  const size_t ld = a.ncap;
  c64* lds64 = reinterpret_cast<c64*>(vdc_tile_lds);
  c32* lds32 = reinterpret_cast<c32*>(vdc_tile_lds);
  c64* slot = a.scratch + (size_t)blockIdx.x * a.slot_elems;
  c64* x = slot;                      // FP64
  c64* b = x + ld;
  c64* r64 = b + ld;
  c64* wA = r64 + ld;
  c64* wB = wA + ld;
  c32* r = reinterpret_cast<c32*>(wB + ld);   // FP32
  c32* p = r + ld;
  c32* q = p + ld;
  c32* z = q;                         // K^{-1} r over q, which the update has consumed
  c32* d = q + ld;
  c32* dinv = d + ld;
  c16* l1 = reinterpret_cast<c16*>(dinv + ld);   // FP16 multipliers: both in one plane
  c16* l2 = l1 + ld;
  c32* wA32 = dinv + 2 * ld;
  c32* wB32 = wA32 + ld;
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
        const c64 dd = a.precond == VDC_PREC_JACOBI ? cinv<double>(op_diag<double>(op, i))
                                                     : c64{1.0, 0.0};
        dinv[i] = c32{(float)dd.x, (float)dd.y};
      }
      x[i] = c64{0.0, 0.0};
      b[i] = c64{0.0, 0.0};
    }
    __syncthreads();
    if (tid == 0) {
      PhiEntry e[6];
      const int n = phi_entries(md, jb.mu, jb.eps_i, jb.vi_g, jb.vi_u, e);
      for (int k = 0; k < n; ++k) b[e[k].g * md.Nu + e[k].u] = c64{e[k].val, 0.0};
    }
    __syncthreads();
    double p64 = blk ? 6.0 : 7.0, p32 = blk ? 2.0 : 1.0;
    const double bnorm = sqrt(norm_sq<double>(b, Nc, L.red));
    double* hist = hist_row<diag>(a, jb);
    p64 += 1.0;
    int iters = 0, outer = 0, status = VDC_NOT_CONVERGED;
    double beta = bnorm;
    // z = K^{-1} src (FP32), then a barrier
    auto kinv = [&](const c32* src, c32* dst) {
      if (blk) {
        prec_apply<rows, float>(fac, op.Ng, op.Nu, src, 1.0f, dst, false);
        __syncthreads();
      } else {
        for (int i = tid; i < Nc; i += kBlock) dst[i] = dinv[i] * src[i];
        __syncthreads();
      }
    };
    auto bilin = [&](const c32* u, const c32* w) {
      float acc[2] = {0.f, 0.f};
      for (int i = tid; i < Nc; i += kBlock) {
        const c32 t = u[i] * w[i];
        acc[0] += t.x;
        acc[1] += t.y;
      }
      block_sum<2, float>(acc, L.redf, L.redf + 2 * kWaves);
      const c32 v = c32{L.redf[2 * kWaves], L.redf[2 * kWaves + 1]};
      __syncthreads();
      return v;
    };
    if (!(bnorm > 0.0) || !isfinite(bnorm)) {
      status = isfinite(bnorm) ? VDC_CONVERGED : VDC_NONFINITE;
      beta = 0.0;
    } else {
      for (int i = tid; i < Nc; i += kBlock) r64[i] = b[i];
      p64 += 2.0;
      for (;;) {
        // r64 holds the FP64 true residual, beta its norm
        if (beta <= a.tol * bnorm) {
          status = VDC_CONVERGED;
          break;
        }
        if (iters >= a.max_iter) break;
        const double sc = 1.0 / beta;
        for (int i = tid; i < Nc; i += kBlock) {
          const c64 t = sc * r64[i];
          r[i] = c32{(float)t.x, (float)t.y};
          d[i] = c32{0.f, 0.f};
        }
        p64 += 1.0;
        p32 += 2.0;
        __syncthreads();
        // inner COCG on A d = r (unit norm) in FP32
        kinv(r, p);
        c32 rho = bilin(r, p);
        p32 += blk ? (rows ? 9.0 : 6.0) : 3.0;
        int k = 0;
        bool bad = false;
        for (;;) {
          if (a.tileT32 > 0) {
            matvec_tiled<float>(op32, L.sqf, p, 1.0f, nullptr, q, lds32, a.tileT32, nullptr,
                                L.redf, L.dot);
          } else {
            matvec_block<float>(op32, L.sqf, p, nullptr, wA32, wB32, q);
            float acc[2] = {0.f, 0.f};
            for (int i = tid; i < Nc; i += kBlock) {
              const c32 t = p[i] * q[i];
              acc[0] += t.x;
              acc[1] += t.y;
            }
            block_sum<2, float>(acc, L.redf, L.redf + 2 * kWaves);
            if (tid < 2) L.dot[tid] = L.redf[2 * kWaves + tid];
            __syncthreads();
            p32 += 2.0;
          }
          p32 += 5.0;
          const c32 mu = c32{L.dot[0], L.dot[1]};
          const float mn = norm2(mu), rn = norm2(rho);
          if (!(mn > 0.f) || !(rn > 0.f) || !isfinite(mn) || !isfinite(rn)) {
            bad = k == 0;
            break;
          }
          const c32 alpha = cinv<float>(mu) * rho;
          // d += alpha p, r -= alpha q, ||r||^2 and rho' = <r|K^{-1} r>_S in
          // one pass (block: by column blocks or rows, z = K^{-1} r stored)
          float acc[3] = {0.f, 0.f, 0.f};
          if (blk) {
            prec_cocg_step<rows, float>(fac, op.Ng, op.Nu, alpha, p, q, d, r, z, acc);
          } else {
            for (int i = tid; i < Nc; i += kBlock) {
              d[i] = d[i] + alpha * p[i];
              const c32 ri = r[i] - alpha * q[i];
              r[i] = ri;
              acc[0] += norm2(ri);
              const c32 t = ri * (dinv[i] * ri);
              acc[1] += t.x;
              acc[2] += t.y;
            }
          }
          block_sum<3, float>(acc, L.redf, L.redf + 3 * kWaves);
          const float rr = L.redf[3 * kWaves];
          const c32 rho_new = c32{L.redf[3 * kWaves + 1], L.redf[3 * kWaves + 2]};
          __syncthreads();
          p32 += blk ? (rows ? 13.0 : 10.0) : 7.0;
          ++k;
          ++iters;
          if (hist && tid == 0 && iters <= a.hist_len)
            hist[iters - 1] = sqrt((double)rr) * beta / bnorm;
          if (rr <= (float)(a.tol_in * a.tol_in) || k >= a.m_in || iters >= a.max_iter ||
              !isfinite(rr))
            break;
          const c32 bt = cinv<float>(rho) * rho_new;
          rho = rho_new;
          for (int i0 = tid; i0 < Nc; i0 += kBatch * kBlock) {
            c32 zv[kBatch], pv[kBatch];
#pragma unroll
            for (int e = 0; e < kBatch; ++e) {
              const int i = min(i0 + e * kBlock, Nc - 1);
              zv[e] = blk ? z[i] : dinv[i] * r[i];
              pv[e] = p[i];
            }
#pragma unroll
            for (int e = 0; e < kBatch; ++e)
              if (i0 + e * kBlock < Nc) p[i0 + e * kBlock] = zv[e] + bt * pv[e];
          }
          p32 += blk ? 3.0 : 4.0;
        }
        if (bad) {
          status = VDC_BREAKDOWN;
          break;
        }
        // x += ||r|| d in FP64, then the true residual
        for (int i = tid; i < Nc; i += kBlock)
          x[i] = x[i] + beta * c64{(double)d[i].x, (double)d[i].y};
        p64 += 2.0;
        p32 += 1.0;
        ++outer;
        beta = sqrt(residual_A<double>(op, L.sq, x, b, r64, lds64, a.tileT, wA, wB, L.red));
        p64 += 6.0;
        if (!isfinite(beta)) {
          status = VDC_NONFINITE;
          break;
        }
      }
    }
    __syncthreads();
    finish_job<diag>(a, md, jb, x, tid, status, iters, outer, outer,
               bnorm > 0.0 ? beta / bnorm : 0.0, (p64 * 16.0 + p32 * 8.0) * md.Nc);
  }
}

hipError_t launch_cocg_mixed(const SolveArgs& a, int n_groups, size_t dyn_lds, hipStream_t s) {
  const bool rows = a.precond == VDC_PREC_ROWS, diag = a.check_optical || a.hist;
  if (rows && diag)
    hipLaunchKernelGGL((cocg_mixed_kernel<true, true>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else if (rows)
    hipLaunchKernelGGL((cocg_mixed_kernel<true, false>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else if (diag)
    hipLaunchKernelGGL((cocg_mixed_kernel<false, true>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else
    hipLaunchKernelGGL((cocg_mixed_kernel<false, false>), dim3(n_groups), dim3(kBlock), dyn_lds, s,
                       a);
  return hipGetLastError();
}

int cocg_mixed_occupancy(size_t dyn_lds) {
  return std::min(std::min(occupancy_of(cocg_mixed_kernel<true, true>, dyn_lds),
                           occupancy_of(cocg_mixed_kernel<true, false>, dyn_lds)),
                  std::min(occupancy_of(cocg_mixed_kernel<false, true>, dyn_lds),
                           occupancy_of(cocg_mixed_kernel<false, false>, dyn_lds)));
}

hipError_t launch_cocg_fp64(const SolveArgs& a, int n_groups, size_t dyn_lds, hipStream_t s) {
  const bool rows = a.precond == VDC_PREC_ROWS, diag = a.check_optical || a.hist;
  if (rows && diag)
    hipLaunchKernelGGL((cocg_fp64_kernel<true, true>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else if (rows)
    hipLaunchKernelGGL((cocg_fp64_kernel<true, false>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else if (diag)
    hipLaunchKernelGGL((cocg_fp64_kernel<false, true>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else
    hipLaunchKernelGGL((cocg_fp64_kernel<false, false>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  return hipGetLastError();
}

int cocg_fp64_occupancy(size_t dyn_lds) {
  return std::min(std::min(occupancy_of(cocg_fp64_kernel<true, true>, dyn_lds),
                           occupancy_of(cocg_fp64_kernel<true, false>, dyn_lds)),
                  std::min(occupancy_of(cocg_fp64_kernel<false, true>, dyn_lds),
                           occupancy_of(cocg_fp64_kernel<false, false>, dyn_lds)));
}

}  // namespace vdc
