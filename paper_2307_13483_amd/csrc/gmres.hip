// Persistent batched restarted GMRES in complex FP64 (Sec. III.A), one job
// per workgroup at a time, the whole solve on chip.
//
// Each workgroup pops jobs from a device counter (the host orders the job
// array longest-first), then for its job:
//   1. the diagonal preconditioner 1/diag(A) and the right-hand side
//      Phi^{v_i mu_i} (Eq. (25)) in the job's symmetry block;
//   2. restarted GMRES(m) with right preconditioning: Arnoldi with classical
//      Gram-Schmidt applied twice (the vector being orthogonalised stays in
//      registers), Givens rotations on the Hessenberg column (one thread),
//      x += M^{-1} V y at the end of a cycle, then the FP64 true residual
//      b - A x decides convergence (stopping rule of Sec. III);
//   3. the amplitudes T = Phi_f^T Psi (Eq. (24)) and the job's share of
//      sigma (Eq. (16)).
// Every wave reaches the queue-exhausted exit; there is no inter-workgroup
// waiting, so the grid drains whether or not all workgroups are resident.
#include "blockops.h"
#include "solve_args.h"

namespace vdc {

struct GivensLds {
  double cs[kMaxRestart];
  c64 sn[kMaxRestart];
  c64 g[kMaxRestart + 1];
  c64 y[kMaxRestart];
  double h1[2 * (kMaxRestart + 1)];
  double h2[2 * (kMaxRestart + 1)];
  c64 hc[kMaxRestart + 1];
  double red[kWaves * 2 * kChunk + 2 * kChunk];
  double sq[kSqMax + 1];
  double resid;
  double nrm;
  int flag;
  int job;
};

__device__ inline c64 cdiv(c64 a, c64 b) {
  const double n = b.x * b.x + b.y * b.y;
  return c64{(a.x * b.x + a.y * b.y) / n, (a.y * b.x - a.x * b.y) / n};
}

// Thread-0 Givens update of Hessenberg column j (Saad & Schultz): apply the
// previous rotations, build rotation j from (h_jj, h_{j+1,j}), store the R
// column and update the right-hand side g.  Returns |g_{j+1}|.
__device__ inline double givens_step(GivensLds& L, int j, double hnext, c64* Rcol) {
  c64* col = L.hc;
  for (int i = 0; i <= j; ++i)
    col[i] = c64{L.h1[2 * i] + L.h2[2 * i], L.h1[2 * i + 1] + L.h2[2 * i + 1]};
  for (int i = 0; i < j; ++i) {
    const c64 a = col[i], b = col[i + 1];
    const c64 s = L.sn[i];
    const double c = L.cs[i];
    col[i] = c * a + s * b;
    col[i + 1] = c * b - c64{s.x, -s.y} * a;
  }
  const c64 a = col[j];
  const double aa = sqrt(norm2(a));
  const double den = hypot(aa, hnext);
  double c;
  c64 s;
  if (den == 0.0) {
    c = 1.0;
    s = c64{0.0, 0.0};
  } else if (aa == 0.0) {
    c = 0.0;
    s = c64{1.0, 0.0};
  } else {
    c = aa / den;
    s = c64{a.x / aa * hnext / den, a.y / aa * hnext / den};  // (a/|a|) conj(h) / den, h real
  }
  L.cs[j] = c;
  L.sn[j] = s;
  col[j] = c * a + hnext * s;
  for (int i = 0; i <= j; ++i) Rcol[i] = col[i];
  const c64 gj = L.g[j];
  L.g[j + 1] = -1.0 * (c64{s.x, -s.y} * gj);
  L.g[j] = c * gj;
  return sqrt(norm2(L.g[j + 1]));
}

// Back substitution R y = g for the k x k upper triangle (columns in Rm,
// leading dimension ldr).  Thread 0.
__device__ inline void back_substitute(GivensLds& L, int k, const c64* Rm, int ldr) {
  for (int i = k - 1; i >= 0; --i) {
    c64 s = L.g[i];
    for (int l = i + 1; l < k; ++l) s = s - Rm[(size_t)l * ldr + i] * L.y[l];
    L.y[i] = cdiv(s, Rm[(size_t)i * ldr + i]);
  }
}

__global__ void __launch_bounds__(kBlock)
gmres_fp64_kernel(SolveArgs a) {
  __shared__ GivensLds L;
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
  const int ldr = m + 1;

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
    // ---- right-hand side Phi^{v_i mu_i} in the block (<= 6 nonzeros)
    if (tid == 0) {
      PhiEntry e[6];
      const int n = phi_entries(md, jb.mu, jb.eps_i, jb.vi_g, jb.vi_u, e);
      for (int q = 0; q < n; ++q) b[e[q].g * md.Nu + e[q].u] = c64{e[q].val, 0.0};
    }
    __syncthreads();
    const double bnorm = sqrt(norm_sq<double>(b, Nc, L.red));
    double beta = bnorm;
    int iters = 0, cycles = 0, status = VDC_NOT_CONVERGED;
    bool breakdown = false;
    if (!(bnorm > 0.0) || !isfinite(bnorm)) {
      status = isfinite(bnorm) ? VDC_CONVERGED : VDC_NONFINITE;
      beta = 0.0;
    } else {
      // V_0 = r_0 / beta with r_0 = b (x_0 = 0)
      for (int i = tid; i < Nc; i += kBlock) V[i] = (1.0 / beta) * b[i];
      for (;;) {
        if (tid == 0) L.g[0] = c64{beta, 0.0};
        int kdim = 0;
        for (int j = 0; j < m; ++j) {
          matvec_block<double>(op, L.sq, V + (size_t)j * ld, dinv, wA, wB, w);
          // classical Gram-Schmidt, twice
          project<double>(V, ld, j + 1, w, Nc, L.red, L.h1);
          subtract<double>(V, ld, j + 1, w, Nc, L.h1);
          project<double>(V, ld, j + 1, w, Nc, L.red, L.h2);
          subtract<double>(V, ld, j + 1, w, Nc, L.h2);
          const double hn = sqrt(norm_sq<double>(w, Nc, L.red));
          if (tid == 0) {
            L.resid = givens_step(L, j, hn, Rm + (size_t)j * ldr);
            L.nrm = hn;
          }
          __syncthreads();
          const double res = L.resid;
          ++iters;
          kdim = j + 1;
          if (!isfinite(res) || !isfinite(hn)) break;
          if (hn == 0.0) {
            breakdown = true;
            break;
          }
          if (res <= a.tol * bnorm || iters >= a.max_iter) break;
          if (j + 1 < m)
            for (int i = tid; i < Nc; i += kBlock) V[(size_t)(j + 1) * ld + i] = (1.0 / hn) * w[i];
        }
        // ---- x += M^{-1} V y
        if (tid == 0) back_substitute(L, kdim, Rm, ldr);
        __syncthreads();
        for (int i = tid; i < Nc; i += kBlock) w[i] = c64{0.0, 0.0};
        subtract<double>(V, ld, kdim, w, Nc, reinterpret_cast<const double*>(L.y));
        for (int i = tid; i < Nc; i += kBlock) x[i] = x[i] - dinv[i] * w[i];
        // ---- true residual r = b - A x (FP64)
        matvec_block<double>(op, L.sq, x, nullptr, wA, wB, w);
        for (int i = tid; i < Nc; i += kBlock) w[i] = b[i] - w[i];
        beta = sqrt(norm_sq<double>(w, Nc, L.red));
        ++cycles;
        if (!isfinite(beta)) {
          status = VDC_NONFINITE;
          break;
        }
        if (beta <= a.tol * bnorm) {
          status = VDC_CONVERGED;
          break;
        }
        if (breakdown) {
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
    // ---- outputs: amplitudes, sigma share, Psi, info
    finish_job(a, md, jb, x, tid, status, iters, cycles, 0, bnorm > 0.0 ? beta / bnorm : 0.0);
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
