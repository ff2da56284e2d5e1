// Persistent batched restarted GMRES in complex FP64 (Sec. III.A), one job
// per workgroup at a time, the whole solve on chip.
//
// Each workgroup pops jobs from a device counter (the host orders the job
// array longest-first), then for its job:
//   1. the preconditioner (Sec. III.B: 1/diag(A), or the LDL^T factors of the
//      column or row blocks of segprec.h) and the right-hand side Phi^{v_i mu_i}
//      (Eq. (25)) in the job's symmetry block;
//   2. restarted GMRES(m) with right preconditioning (krylov.h), then
//      x += M^{-1} V y and the FP64 true residual b - A x, which decides
//      convergence (stopping rule of Sec. III);
//   3. the amplitudes T = Phi_f^T Psi (Eq. (24)) and the job's share of
//      sigma (Eq. (16)).
// Every wave reaches the queue-exhausted exit; there is no inter-workgroup
// waiting, so the grid drains whether or not all workgroups are resident.
#include "gmres_block.h"
#include "solve_args.h"

namespace vdc {

template <bool rows, bool diag>
__global__ void __launch_bounds__(kBlock)
gmres_fp64_kernel(SolveArgs a) {
  __shared__ Fp64Lds L;
  fill_sq<double>(L.sq);
  const int tid = threadIdx.x;
  const Fp64Slot s = fp64_slot(a.scratch + (size_t)blockIdx.x * a.slot_elems, a.ncap, a.m);
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
    // right-hand side Phi^{v_i mu_i} in the block (<= 5 nonzeros)
    if (tid == 0) {
      PhiEntry e[6];
      const int n = phi_entries(md, jb.mu, jb.eps_i, jb.vi_g, jb.vi_u, e);
      for (int q = 0; q < n; ++q) s.b[e[q].g * md.Nu + e[q].u] = c64{e[q].val, 0.0};
    }
    __syncthreads();
    const BlockSolve r =
        gmres_fp64_block<rows>(L, op, s, a.ncap, a.m, a.tol, a.max_iter, a.tileT, a.precond,
                               hist_row<diag>(a, jb), a.hist_len);
    __syncthreads();
    finish_job<diag>(a, md, jb, s.x, tid, r.status, r.iters, r.cycles, 0,
               r.bnorm > 0.0 ? r.beta / r.bnorm : 0.0, r.passes * 16.0 * md.Nc);
  }
}

hipError_t launch_gmres_fp64(const SolveArgs& a, int n_groups, size_t dyn_lds, hipStream_t s) {
  const bool rows = a.precond == VDC_PREC_ROWS, diag = a.check_optical || a.hist;
  if (rows && diag)
    hipLaunchKernelGGL((gmres_fp64_kernel<true, true>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else if (rows)
    hipLaunchKernelGGL((gmres_fp64_kernel<true, false>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else if (diag)
    hipLaunchKernelGGL((gmres_fp64_kernel<false, true>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else
    hipLaunchKernelGGL((gmres_fp64_kernel<false, false>), dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  return hipGetLastError();
}

int gmres_fp64_occupancy(size_t dyn_lds) {
  return std::min(std::min(occupancy_of(gmres_fp64_kernel<true, true>, dyn_lds),
                           occupancy_of(gmres_fp64_kernel<true, false>, dyn_lds)),
                  std::min(occupancy_of(gmres_fp64_kernel<false, true>, dyn_lds),
                           occupancy_of(gmres_fp64_kernel<false, false>, dyn_lds)));
}

}  // namespace vdc
