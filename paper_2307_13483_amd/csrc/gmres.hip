// Persistent batched restarted GMRES in complex FP64 (Sec. III.A), one job
// per workgroup at a time, the whole solve on chip.
//
// Each workgroup pops jobs from a device counter (the host orders the job
// array longest-first), then for its job:
//   1. the diagonal preconditioner 1/diag(A) (Sec. III.B) and the right-hand
//      side Phi^{v_i mu_i} (Eq. (25)) in the job's symmetry block;
//   2. restarted GMRES(m) with right preconditioning (krylov.h), then
//      x += M^{-1} V y and the FP64 true residual b - A x, which decides
//      convergence (stopping rule of Sec. III);
//   3. the amplitudes T = Phi_f^T Psi (Eq. (24)) and the job's share of
//      sigma (Eq. (16)).
// Every wave reaches the queue-exhausted exit; there is no inter-workgroup
// waiting, so the grid drains whether or not all workgroups are resident.
#include "krylov.h"
#include "solve_args.h"

namespace vdc {

struct Fp64Lds {
  KrylovLds<double> K;
  double red[kRedSize];
  double sq[kSqMax + 1];
  int job;
};

__global__ void __launch_bounds__(kBlock)
gmres_fp64_kernel(SolveArgs a) {
  __shared__ Fp64Lds L;
  fill_sq<double>(L.sq);
  const int tid = threadIdx.x;
  const int m = a.m;
  c64* slot = a.scratch + (size_t)blockIdx.x * a.slot_elems;
  const size_t ld = a.ncap;
  c64* V = slot;
  c64* x = slot + (size_t)(m + 1) * ld;
  c64* b = x + ld;
  c64* dinv = b + ld;
  c64* w = dinv + ld;
  c64* wA = w + ld;
  c64* wB = wA + ld;
  c64* Rm = wB + ld;

  for (;;) {
    __syncthreads();
    if (tid == 0) L.job = atomicAdd(a.counter, 1);
    __syncthreads();
    const int js = L.job;
    if (js >= a.n_jobs) break;
    const DevJob jb = a.jobs[js];
    const DevModel& md = a.models[jb.model];
    const DevTable tb = a.tabs[jb.table];
    const OpJob<double> op =
        make_op<double>(md, jb, a.tables + tb.offset + (size_t)(jb.parity * 3) * md.Nc);
    const int Nc = md.Nc;

    // ---- preconditioner, x = 0, b = 0
    for (int i = tid; i < Nc; i += kBlock) {
      dinv[i] = a.precond ? cinv<double>(op_diag<double>(op, i)) : c64{1.0, 0.0};
      x[i] = c64{0.0, 0.0};
      b[i] = c64{0.0, 0.0};
    }
    __syncthreads();
    // ---- right-hand side Phi^{v_i mu_i} in the block (<= 5 nonzeros)
    if (tid == 0) {
      PhiEntry e[6];
      const int n = phi_entries(md, jb.mu, jb.eps_i, jb.vi_g, jb.vi_u, e);
      for (int q = 0; q < n; ++q) b[e[q].g * md.Nu + e[q].u] = c64{e[q].val, 0.0};
    }
    __syncthreads();
    const double bnorm = sqrt(norm_sq<double>(b, Nc, L.red));
    double beta = bnorm;
    int iters = 0, cycles = 0, status = VDC_NOT_CONVERGED;
    // byte model (passes over a block vector of Nc complex FP64 values):
    // setup 7 (3 table planes read; dinv, x, b, v_0 written), each cycle of k
    // steps cycle_passes(k) + k + 10 (x update k + 3, true residual 7)
    double passes = 7.0;
    if (!(bnorm > 0.0) || !isfinite(bnorm)) {
      status = isfinite(bnorm) ? VDC_CONVERGED : VDC_NONFINITE;
      beta = 0.0;
    } else {
      for (int i = tid; i < Nc; i += kBlock) V[i] = (1.0 / beta) * b[i];
      auto apply = [&](int j, c64* out) {
        matvec_block<double>(op, L.sq, V + (size_t)j * ld, dinv, wA, wB, out);
      };
      for (;;) {
        if (tid == 0) L.K.g[0] = c64{beta, 0.0};
        const CycleResult cr = krylov_cycle<double>(L.K, L.red, V, ld, Nc, m, a.tol * bnorm,
                                                    a.max_iter, iters, Rm, w, apply);
        passes += cycle_passes(cr.k) + cr.k + 10.0;
        // ---- x += M^{-1} V y
        combine_neg<double>(V, ld, cr.k, L.K.y, w, Nc);
        for (int i = tid; i < Nc; i += kBlock) x[i] = x[i] - dinv[i] * w[i];
        // ---- true residual r = b - A x (FP64)
        matvec_block<double>(op, L.sq, x, nullptr, wA, wB, w);
        for (int i = tid; i < Nc; i += kBlock) w[i] = b[i] - w[i];
        beta = sqrt(norm_sq<double>(w, Nc, L.red));
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
        for (int i = tid; i < Nc; i += kBlock) V[i] = (1.0 / beta) * w[i];
      }
    }
    __syncthreads();
    finish_job(a, md, jb, x, tid, status, iters, cycles, 0, bnorm > 0.0 ? beta / bnorm : 0.0,
               passes * 16.0 * Nc);
  }
}

hipError_t launch_gmres_fp64(const SolveArgs& a, int n_groups, hipStream_t s) {
  hipLaunchKernelGGL(gmres_fp64_kernel, dim3(n_groups), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

int gmres_fp64_occupancy() {
  int n = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gmres_fp64_kernel, kBlock, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace vdc
