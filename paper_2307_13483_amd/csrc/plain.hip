// The plain single-solve path: the same restarted GMRES as the persistent
// solver (Sec. III.A; CGS2, Givens, FP64 true residual), but one job at a
// time with every step a separate grid-wide kernel issued from the host:
// stencil phases, multi-vector dot products (block partials + a fixed-order
// reduction kernel), updates, norms and a one-thread Givens kernel.  The host
// issues a whole cycle of m steps without waiting; kernels after convergence
// return at once on a device flag, and the host reads the status back once
// per cycle.  This is the reference point for the batched launch.
#include <string>
#include <vector>

#include "segprec.h"
#include "solve_args.h"

namespace vdc {

constexpr int kPT = 256;   // threads per block of the plain kernels

// Device-resident state of one plain solve (slot space from plain_extra_elems).
struct PlainState {
  double h1[2 * (kMaxRestart + 1)];
  double h2[2 * (kMaxRestart + 1)];
  c64 g[kMaxRestart + 1];
  c64 sn[kMaxRestart];
  c64 y[kMaxRestart];
  double cs[kMaxRestart];
  double hn, resid, beta, bnorm, passes;
  int k, done, status, iters, cycles, breakdown, stop_cycle;
};

struct PlainArgs {
  DevModel md;
  DevJob jb;
  const c64* tab;       // block tables of the job (3 planes)
  c64 *V, *x, *b, *dinv, *w, *wA, *wB, *l1, *l2, *zt, *Rm;
  c64* part;            // [m+1][nblk] partial dots
  double* partn;        // [nblk] partial norms
  PlainState* st;
  size_t ld;
  int m, nblk, max_iter, precond;
  double tol;
};

__device__ inline OpJob<double> plain_op(const PlainArgs& a) { return make_op<double>(a.md, a.jb, a.tab); }

__global__ void __launch_bounds__(kPT) p_init(PlainArgs a) {
  const int i = blockIdx.x * kPT + threadIdx.x;
  if (i >= a.md.Nc) return;
  const OpJob<double> op = plain_op(a);
  if (!prec_has_factor(a.precond))
    a.dinv[i] = a.precond == VDC_PREC_JACOBI ? cinv<double>(op_diag<double>(op, i)) : c64{1.0, 0.0};
  a.x[i] = c64{0.0, 0.0};
  a.b[i] = c64{0.0, 0.0};
}

// block preconditioner factors (segprec.h), one thread per column block or
// per row
__global__ void __launch_bounds__(kPT) p_factor(PlainArgs a) {
  __shared__ double sq[kSqMax + 1];
  fill_sq<double>(sq);
  __syncthreads();
  const int c = blockIdx.x * kPT + threadIdx.x;
  const SegFactor<double> f{a.l1, a.l2, a.dinv};
  if (a.precond == VDC_PREC_ROWS) {
    if (c < a.md.Ng) row_factor_row<double>(plain_op(a), sq, f, c);
    return;
  }
  if (c >= seg_blocks(a.md.Ng, a.md.Nu)) return;
  seg_factor_block<double>(plain_op(a), sq, f, c);
}

// z = M^{-1} v, or z += M^{-1} v with accumulate, one thread per block; the
// end-of-cycle call runs until the job is done, the step call until the
// cycle stops
__global__ void __launch_bounds__(kPT) p_papply(PlainArgs a, const c64* v, c64* z, int accumulate,
                                                int end_of_cycle) {
  if (end_of_cycle ? a.st->done : a.st->stop_cycle) return;
  const int c = blockIdx.x * kPT + threadIdx.x;
  const SegFactor<double> f{a.l1, a.l2, a.dinv};
  if (a.precond == VDC_PREC_ROWS) {
    // accumulating calls pass v = zt, which parks the forward sweep
    if (c < a.md.Ng) row_apply_row<double>(f, a.md.Nu, v, 1.0, z, accumulate != 0, a.zt, c);
    return;
  }
  if (c >= seg_blocks(a.md.Ng, a.md.Nu)) return;
  seg_apply_block<double>(f, a.md.Ng, a.md.Nu, v, 1.0, z, accumulate != 0, c);
}

__global__ void p_rhs(PlainArgs a) {
  PhiEntry e[6];
  const int n = phi_entries(a.md, a.jb.mu, a.jb.eps_i, a.jb.vi_g, a.jb.vi_u, e);
  for (int q = 0; q < n; ++q) a.b[e[q].g * a.md.Nu + e[q].u] = c64{e[q].val, 0.0};
  PlainState& s = *a.st;
  s.k = 0;
  s.done = 0;
  s.status = VDC_NOT_CONVERGED;
  s.iters = 0;
  s.cycles = 0;
  s.breakdown = 0;
  s.stop_cycle = 0;
  s.passes = prec_has_factor(a.precond) ? 10.0 : 7.0;
}

// per-block partial sums of |v|^2 (the v is w or b)
__global__ void __launch_bounds__(kPT) p_norm_part(PlainArgs a, const c64* v) {
  if (a.st->stop_cycle) return;
  __shared__ double red[kPT];
  const int i = blockIdx.x * kPT + threadIdx.x;
  red[threadIdx.x] = (i < a.md.Nc) ? norm2(v[i]) : 0.0;
  __syncthreads();
  for (int s = kPT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partn[blockIdx.x] = red[0];
}

// what: 0 = ||b|| (start), 1 = ||w|| (Arnoldi), 2 = ||r|| (end of cycle)
__global__ void p_norm_final(PlainArgs a, int what) {
  PlainState& s = *a.st;
  if (s.stop_cycle) return;
  double t = 0.0;
  for (int k = 0; k < a.nblk; ++k) t += a.partn[k];
  const double n = sqrt(t);
  if (what == 0) {
    s.bnorm = n;
    s.beta = n;
    s.g[0] = c64{n, 0.0};
    if (!(n > 0.0) || !isfinite(n)) {
      s.status = isfinite(n) ? VDC_CONVERGED : VDC_NONFINITE;
      s.done = 1;
      s.stop_cycle = 1;
      s.beta = 0.0;
    }
  } else if (what == 1) {
    s.hn = n;
  } else {
    s.beta = n;
  }
}

// v_out = v_in / (what ? hn : beta)
__global__ void __launch_bounds__(kPT) p_scale(PlainArgs a, const c64* vin, c64* vout, int use_hn) {
  if (a.st->stop_cycle) return;
  const int i = blockIdx.x * kPT + threadIdx.x;
  if (i >= a.md.Nc) return;
  const double d = use_hn ? a.st->hn : a.st->beta;
  vout[i] = (1.0 / d) * vin[i];
}

__global__ void __launch_bounds__(kPT) p_phase1(PlainArgs a, const c64* v, int scaled) {
  if (a.st->stop_cycle) return;
  __shared__ double sq[kSqMax + 1];
  fill_sq<double>(sq);
  __syncthreads();
  const int i = blockIdx.x * kPT + threadIdx.x;
  if (i >= a.md.Nc) return;
  const OpJob<double> op = plain_op(a);
  c64 y, wa, wb;
  op_phase1<double>(op, sq, v, scaled ? a.dinv : nullptr, i, y, wa, wb);
  a.w[i] = y;
  a.wA[i] = wa;
  a.wB[i] = wb;
}

__global__ void __launch_bounds__(kPT) p_phase2(PlainArgs a) {
  if (a.st->stop_cycle) return;
  __shared__ double sq[kSqMax + 1];
  fill_sq<double>(sq);
  __syncthreads();
  const int i = blockIdx.x * kPT + threadIdx.x;
  if (i >= a.md.Nc) return;
  const OpJob<double> op = plain_op(a);
  a.w[i] = op_phase2<double>(op, sq, a.wA, a.wB, i, a.w[i]);
}

// partial dots: block (b, l) -> part[l][b] = sum_{i in block b} conj(V_l[i]) w[i]
__global__ void __launch_bounds__(kPT) p_dot_part(PlainArgs a, int nv) {
  if (a.st->stop_cycle) return;
  __shared__ double rr[kPT], ri[kPT];
  const int l = blockIdx.y;
  if (l >= nv) return;
  const int i = blockIdx.x * kPT + threadIdx.x;
  c64 t = c64{0.0, 0.0};
  if (i < a.md.Nc) t = conjmul(a.V[(size_t)l * a.ld + i], a.w[i]);
  rr[threadIdx.x] = t.x;
  ri[threadIdx.x] = t.y;
  __syncthreads();
  for (int s = kPT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      rr[threadIdx.x] += rr[threadIdx.x + s];
      ri[threadIdx.x] += ri[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) a.part[(size_t)l * a.nblk + blockIdx.x] = c64{rr[0], ri[0]};
}

// h[l] = sum_b part[l][b] in block order; which = 1 -> h1, 2 -> h2
__global__ void p_dot_final(PlainArgs a, int nv, int which) {
  if (a.st->stop_cycle) return;
  const int l = threadIdx.x;
  if (l >= nv) return;
  c64 s = c64{0.0, 0.0};
  for (int b = 0; b < a.nblk; ++b) s = s + a.part[(size_t)l * a.nblk + b];
  double* h = which == 1 ? a.st->h1 : a.st->h2;
  h[2 * l] = s.x;
  h[2 * l + 1] = s.y;
}

// w -= sum_l V_l h[l]
__global__ void __launch_bounds__(kPT) p_axpy(PlainArgs a, int nv, int which) {
  if (a.st->stop_cycle) return;
  const int i = blockIdx.x * kPT + threadIdx.x;
  if (i >= a.md.Nc) return;
  const double* h = which == 1 ? a.st->h1 : a.st->h2;
  c64 s = a.w[i];
  for (int l = 0; l < nv; ++l) s = s - a.V[(size_t)l * a.ld + i] * c64{h[2 * l], h[2 * l + 1]};
  a.w[i] = s;
}

// Givens update of column j, convergence / breakdown flags (one thread)
__global__ void p_givens(PlainArgs a, int j) {
  PlainState& s = *a.st;
  if (s.stop_cycle) return;
  c64 col[kMaxRestart + 1];
  for (int i = 0; i <= j; ++i) col[i] = c64{s.h1[2 * i] + s.h2[2 * i], s.h1[2 * i + 1] + s.h2[2 * i + 1]};
  for (int i = 0; i < j; ++i) {
    const c64 x = col[i], y = col[i + 1];
    col[i] = s.cs[i] * x + s.sn[i] * y;
    col[i + 1] = s.cs[i] * y - c64{s.sn[i].x, -s.sn[i].y} * x;
  }
  const double hn = s.hn;
  const c64 x = col[j];
  const double ax = sqrt(norm2(x));
  const double den = hypot(ax, hn);
  double c;
  c64 sn;
  if (den == 0.0) {
    c = 1.0;
    sn = c64{0.0, 0.0};
  } else if (ax == 0.0) {
    c = 0.0;
    sn = c64{1.0, 0.0};
  } else {
    c = ax / den;
    sn = c64{x.x / ax * hn / den, x.y / ax * hn / den};
  }
  s.cs[j] = c;
  s.sn[j] = sn;
  col[j] = c * x + hn * sn;
  for (int i = 0; i <= j; ++i) a.Rm[(size_t)j * (a.m + 1) + i] = col[i];
  const c64 gj = s.g[j];
  s.g[j + 1] = -1.0 * (c64{sn.x, -sn.y} * gj);
  s.g[j] = c * gj;
  const double res = sqrt(norm2(s.g[j + 1]));
  s.resid = res;
  s.iters += 1;
  s.k = j + 1;
  if (!isfinite(res) || !isfinite(hn)) {
    s.stop_cycle = 1;
  } else if (hn == 0.0) {
    s.breakdown = 1;
    s.stop_cycle = 1;
  } else if (res <= a.tol * s.bnorm || s.iters >= a.max_iter) {
    s.stop_cycle = 1;
  }
}

// back substitution and cycle start bookkeeping (one thread)
__global__ void p_backsub(PlainArgs a) {
  PlainState& s = *a.st;
  if (s.done) return;
  const int k = s.k;
  const int ldr = a.m + 1;
  for (int i = k - 1; i >= 0; --i) {
    c64 t = s.g[i];
    for (int l = i + 1; l < k; ++l) t = t - a.Rm[(size_t)l * ldr + i] * s.y[l];
    const c64 d = a.Rm[(size_t)i * ldr + i];
    const double n = d.x * d.x + d.y * d.y;
    s.y[i] = c64{(t.x * d.x + t.y * d.y) / n, (t.y * d.x - t.x * d.y) / n};
  }
  s.stop_cycle = 0;   // the end-of-cycle kernels run
}

// x += dinv * sum_l V_l y_l (block preconditioner: zt = sum_l V_l y_l)
__global__ void __launch_bounds__(kPT) p_update(PlainArgs a) {
  if (a.st->done) return;
  const int i = blockIdx.x * kPT + threadIdx.x;
  if (i >= a.md.Nc) return;
  c64 t = c64{0.0, 0.0};
  for (int l = 0; l < a.st->k; ++l) t = t + a.V[(size_t)l * a.ld + i] * a.st->y[l];
  if (prec_has_factor(a.precond))
    a.zt[i] = t;
  else
    a.x[i] = a.x[i] + a.dinv[i] * t;
}

// w = b - w (true residual after the matvec of x)
__global__ void __launch_bounds__(kPT) p_resid(PlainArgs a) {
  if (a.st->done) return;
  const int i = blockIdx.x * kPT + threadIdx.x;
  if (i >= a.md.Nc) return;
  a.w[i] = a.b[i] - a.w[i];
}

// status after the true residual (one thread)
__global__ void p_status(PlainArgs a) {
  PlainState& s = *a.st;
  if (s.done) return;
  s.cycles += 1;
  s.passes += 7.0 * s.k + 2.0 * s.k * (s.k + 1.0) + s.k + 10.0 +
              (prec_has_factor(a.precond) ? 4.0 * s.k + 4.0 : 0.0);
  const double beta = s.beta;
  if (!isfinite(beta)) {
    s.status = VDC_NONFINITE;
    s.done = 1;
  } else if (beta <= a.tol * s.bnorm) {
    s.status = VDC_CONVERGED;
    s.done = 1;
  } else if (s.breakdown) {
    s.status = VDC_BREAKDOWN;
    s.done = 1;
  } else if (s.iters >= a.max_iter) {
    s.status = VDC_NOT_CONVERGED;
    s.done = 1;
  }
  s.stop_cycle = s.done;
  s.g[0] = c64{beta, 0.0};
}

__global__ void __launch_bounds__(kBlock) p_finish(SolveArgs sa, PlainArgs a) {
  __syncthreads();
  const PlainState& s = *a.st;
  finish_job<true>(sa, a.md, a.jb, a.x, threadIdx.x, s.status, s.iters, s.cycles, 0,
                   s.bnorm > 0.0 ? s.beta / s.bnorm : 0.0, s.passes * 16.0 * a.md.Nc);
}

size_t plain_extra_elems(size_t ncap, int m) {
  const size_t nblk = (ncap + kPT - 1) / kPT;
  return (size_t)(m + 1) * nblk + (nblk + 32) / 2 + 1 + (sizeof(PlainState) + 15) / 16 + 16;
}

vdc_status solve_plain_impl(const SolveArgs& sa, const std::vector<DevJob>& jobs,
                            const std::vector<DevModel>& models, hipStream_t st,
                            std::string& err) {
  const int n_jobs = (int)jobs.size();
  const int m = sa.m;
  c64* slot = sa.scratch;
  const size_t ld = sa.ncap;
  PlainArgs a{};
  a.V = slot;
  a.x = slot + (size_t)(m + 1) * ld;
  a.b = a.x + ld;
  a.dinv = a.b + ld;
  a.w = a.dinv + ld;
  a.wA = a.w + ld;
  a.wB = a.wA + ld;
  a.l1 = a.wB + ld;
  a.l2 = a.l1 + ld;
  a.zt = a.l2 + ld;
  a.Rm = a.zt + ld;
  const int nblk_max = (int)((ld + kPT - 1) / kPT);
  a.part = a.Rm + (size_t)(m + 1) * m;
  a.partn = reinterpret_cast<double*>(a.part + (size_t)(m + 1) * nblk_max);
  a.st = reinterpret_cast<PlainState*>(a.partn + nblk_max + 32);
  a.ld = ld;
  a.m = m;
  a.max_iter = sa.max_iter;
  a.precond = sa.precond;
  a.tol = sa.tol;
  // the per-energy table offsets, to point each job at its block tables
  std::vector<DevTable> htabs;
  {
    int nt = 0;
    for (const DevJob& j : jobs) nt = std::max(nt, j.table + 1);
    htabs.resize(nt);
    if (hipMemcpyAsync(htabs.data(), sa.tabs, sizeof(DevTable) * nt, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      err = "plain path: table read-back failed";
      return VDC_ERR_HIP;
    }
  }
  PlainState hs;
  for (int q = 0; q < n_jobs; ++q) {
    const DevJob& jb = jobs[q];
    a.md = models[jb.model];
    a.jb = jb;
    a.tab = sa.tables + htabs[jb.table].offset + (size_t)(jb.parity * sa.planes) * a.md.Nc;
    a.nblk = (a.md.Nc + kPT - 1) / kPT;
    const dim3 g1(a.nblk), b1(kPT);
    const bool blk = prec_has_factor(a.precond);
    const int n_fac = a.precond == VDC_PREC_ROWS ? a.md.Ng : seg_blocks(a.md.Ng, a.md.Nu);
    const dim3 gs((n_fac + kPT - 1) / kPT);
    hipLaunchKernelGGL(p_init, g1, b1, 0, st, a);
    if (blk) hipLaunchKernelGGL(p_factor, gs, b1, 0, st, a);
    hipLaunchKernelGGL(p_rhs, dim3(1), dim3(1), 0, st, a);
    hipLaunchKernelGGL(p_norm_part, g1, b1, 0, st, a, (const c64*)a.b);
    hipLaunchKernelGGL(p_norm_final, dim3(1), dim3(1), 0, st, a, 0);
    hipLaunchKernelGGL(p_scale, g1, b1, 0, st, a, (const c64*)a.b, a.V, 0);
    for (;;) {
      for (int j = 0; j < m; ++j) {
        if (blk) {
          hipLaunchKernelGGL(p_papply, gs, b1, 0, st, a, (const c64*)(a.V + (size_t)j * ld), a.zt, 0,
                             0);
          hipLaunchKernelGGL(p_phase1, g1, b1, 0, st, a, (const c64*)a.zt, 0);
        } else {
          hipLaunchKernelGGL(p_phase1, g1, b1, 0, st, a, (const c64*)(a.V + (size_t)j * ld), 1);
        }
        hipLaunchKernelGGL(p_phase2, g1, b1, 0, st, a);
        for (int pass = 1; pass <= 2; ++pass) {
          hipLaunchKernelGGL(p_dot_part, dim3(a.nblk, j + 1), b1, 0, st, a, j + 1);
          hipLaunchKernelGGL(p_dot_final, dim3(1), dim3(kMaxRestart + 1), 0, st, a, j + 1, pass);
          hipLaunchKernelGGL(p_axpy, g1, b1, 0, st, a, j + 1, pass);
        }
        hipLaunchKernelGGL(p_norm_part, g1, b1, 0, st, a, (const c64*)a.w);
        hipLaunchKernelGGL(p_norm_final, dim3(1), dim3(1), 0, st, a, 1);
        hipLaunchKernelGGL(p_givens, dim3(1), dim3(1), 0, st, a, j);
        if (j + 1 < m)
          hipLaunchKernelGGL(p_scale, g1, b1, 0, st, a, (const c64*)a.w, a.V + (size_t)(j + 1) * ld, 1);
      }
      hipLaunchKernelGGL(p_backsub, dim3(1), dim3(1), 0, st, a);
      hipLaunchKernelGGL(p_update, g1, b1, 0, st, a);
      if (blk) hipLaunchKernelGGL(p_papply, gs, b1, 0, st, a, (const c64*)a.zt, a.x, 1, 1);
      hipLaunchKernelGGL(p_phase1, g1, b1, 0, st, a, (const c64*)a.x, 0);
      hipLaunchKernelGGL(p_phase2, g1, b1, 0, st, a);
      hipLaunchKernelGGL(p_resid, g1, b1, 0, st, a);
      hipLaunchKernelGGL(p_norm_part, g1, b1, 0, st, a, (const c64*)a.w);
      hipLaunchKernelGGL(p_norm_final, dim3(1), dim3(1), 0, st, a, 2);
      hipLaunchKernelGGL(p_status, dim3(1), dim3(1), 0, st, a);
      hipLaunchKernelGGL(p_scale, g1, b1, 0, st, a, (const c64*)a.w, a.V, 0);
      // one status read-back per cycle
      if (hipMemcpyAsync(&hs, a.st, sizeof(PlainState), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        err = "plain path: status read-back failed";
        return VDC_ERR_HIP;
      }
      if (hs.done) break;
    }
    hipLaunchKernelGGL(p_finish, dim3(1), dim3(kBlock), 0, st, sa, a);
    if (hipGetLastError() != hipSuccess) {
      err = "plain path: kernel launch failed";
      return VDC_ERR_HIP;
    }
  }
  return VDC_OK;
}

}  // namespace vdc
