// Kernels of the general (term-list) model: the operator on full-layout
// vectors, and the batched persistent solve (one job per workgroup, COCG or
// restarted GMRES in complex FP64, right-preconditioned by diag(A) or not),
// followed by the amplitudes and cross-section shares.  Stencil arithmetic
// in terms.h.
#include "blockops.h"
#include "krylov.h"
#include "terms.h"
#include "terms_args.h"

namespace vdc {

constexpr int kGenThreads = 256;

// y = A x, pass 1 (w planes) and pass 2 (y), one thread per (point, vector).
__global__ void __launch_bounds__(kGenThreads)
gen_pass1_kernel(const DevGen* __restrict__ gm, const c64* __restrict__ F,
                 const c64* __restrict__ x, c64* __restrict__ w, size_t xld, size_t wld) {
  const DevGen& g = *gm;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.npts) return;
  gen_pass1(g, F, x + blockIdx.y * xld, w + blockIdx.y * wld, i);
}

__global__ void __launch_bounds__(kGenThreads)
gen_pass2_kernel(const DevGen* __restrict__ gm, double E, const c64* __restrict__ x,
                 const c64* __restrict__ w, c64* __restrict__ y, size_t xld, size_t wld) {
  const DevGen& g = *gm;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.npts) return;
  gen_pass2(g, E, x + blockIdx.y * xld, w + blockIdx.y * wld, y + blockIdx.y * xld, i);
}

hipError_t launch_gen_apply(const DevGen* gm_dev, int npts, double E, const c64* F, int n_vec,
                            const c64* x, c64* w, c64* y, size_t xld, size_t wld, hipStream_t s) {
  if (n_vec <= 0) return hipSuccess;
  const dim3 grid((npts + kGenThreads - 1) / kGenThreads, n_vec);
  hipLaunchKernelGGL(gen_pass1_kernel, grid, dim3(kGenThreads), 0, s, gm_dev, F, x, w, xld, wld);
  hipLaunchKernelGGL(gen_pass2_kernel, grid, dim3(kGenThreads), 0, s, gm_dev, E, x, w, y, xld, wld);
  return hipGetLastError();
}

// ------------------------------------------------------------ batched solve

struct GenLds {
  KrylovLds<double> K;
  double red[kRedSize];
  int job;
};

// y = A v for one job, by the whole workgroup: pass 1 writes the w planes,
// pass 2 reads them (barriers before, between and after).
__device__ inline void gen_apply_block(const DevGen& g, double E, const c64* F, const c64* v,
                                       c64* w, c64* y) {
  __syncthreads();
  for (int i = threadIdx.x; i < g.npts; i += kBlock) gen_pass1(g, F, v, w, i);
  __syncthreads();
  for (int i = threadIdx.x; i < g.npts; i += kBlock) gen_pass2(g, E, v, w, y, i);
  __syncthreads();
}

// Byte model, in passes over a job vector of N = D npts complex FP64 values:
// the operator reads its input and the level-shift planes (nplanes npts
// values), writes and reads the w planes (2 nw npts) and writes y:
//   op = 2 + (nplanes + 2 nw) npts / N;
// COCG step: operator, <p|q> (p, q), the update of x and r with rho'
// (x, p, r, q, dinv in, x, r out: 7), the next direction (r, dinv, p in, p
// out: 4); GMRES step j: scaling z = dinv s V_j (2), operator, classical
// Gram-Schmidt (2 (j + 1), twice when repeated); cycle end: x update
// (k + 3), the true residual (operator + b in, V_0 out: op + 2).
__device__ inline double gen_op_passes(const DevGen& g) {
  return 2.0 + (double)(g.nplanes + 2 * g.nw) / (double)g.D;
}

__global__ void __launch_bounds__(kBlock) gen_solve_kernel(GenArgs a) {
  __shared__ GenLds L;
  const int tid = threadIdx.x;
  c64* slot = a.scratch + (size_t)blockIdx.x * a.slot_elems;
  const size_t ld = a.ld;
  c64* x = slot;
  c64* b = x + ld;
  c64* dinv = b + ld;
  c64* z = dinv + ld;                 // scaled operator input / residual work
  c64* W = z + ld;                    // w planes (wld values)
  c64* V = W + a.wld;                 // COCG: r, p, q; GMRES: the basis (m + 1)
  c64* Rm = V + (size_t)(a.method == VDC_COCG ? 3 : a.m + 1) * ld;
  for (;;) {
    __syncthreads();
    if (tid == 0) L.job = atomicAdd(a.counter, 1);
    __syncthreads();
    const int js = L.job;
    if (js >= a.n_jobs) break;
    const GenJob jb = a.jobs[js];
    const DevGen& g = a.models[jb.model];
    const GenTab tb = a.tabs[jb.table];
    const c64* F = a.tables + tb.offset;
    const int N = g.D * g.npts;
    const double E = jb.E;
    // preconditioner and b = Phi^{v_i mu_i}
    for (int i = tid; i < N; i += kBlock) {
      const int d = i / g.npts, p = i - d * g.npts;
      dinv[i] = a.precond == VDC_PREC_JACOBI ? cinv<double>(gen_diag(g, E, F, d, p))
                                             : c64{1.0, 0.0};
      x[i] = c64{0.0, 0.0};
      b[i] = c64{0.0, 0.0};
    }
    __syncthreads();
    if (tid == 0) {
      const int vi = gen_flat(g, jb.v);
      const double eps = E - gen_vib_energy(g, jb.v);
      for (int d = 0; d < g.D; ++d) {
        const double f = gen_f(g, d, jb.mu, eps);
        const GenOp& o = g.vop[d][jb.mu];
        if (f == 0.0 || !o.np) continue;
        for (int q = o.p0; q < o.p0 + o.np; ++q) {
          const GenPoint pt = g.pts[q];
          double c;
          if (gen_coef(g, pt, jb.v, c)) b[(size_t)d * g.npts + vi + pt.off] = c64{f * c, 0.0};
        }
      }
    }
    __syncthreads();
    const double opp = gen_op_passes(g);
    double passes = 5.0;
    const double bnorm = sqrt(norm_sq<double>(b, N, L.red));
    int status = VDC_NOT_CONVERGED, iters = 0, cycles = 0;
    double beta = bnorm;
    // true residual b - A x into r (and its norm)
    auto true_residual = [&](c64* r) -> double {
      gen_apply_block(g, E, F, x, W, z);
      double acc[1] = {0.0};
      for (int i = tid; i < N; i += kBlock) {
        const c64 t = b[i] - z[i];
        r[i] = t;
        acc[0] += norm2(t);
      }
      block_sum<1, double>(acc, L.red, L.red + kWaves);
      const double v = L.red[kWaves];
      __syncthreads();
      passes += opp + 3.0;
      return sqrt(v);
    };
    if (!(bnorm > 0.0) || !isfinite(bnorm)) {
      status = isfinite(bnorm) ? VDC_CONVERGED : VDC_NONFINITE;
      beta = 0.0;
    } else if (a.method == VDC_COCG) {
      c64* r = V;
      c64* p = V + ld;
      c64* q = V + 2 * ld;
      for (int i = tid; i < N; i += kBlock) r[i] = b[i];
      auto restart_dir = [&]() -> c64 {
        double acc[2] = {0.0, 0.0};
        for (int i = tid; i < N; i += kBlock) {
          const c64 zi = dinv[i] * r[i];
          p[i] = zi;
          const c64 t = r[i] * zi;
          acc[0] += t.x;
          acc[1] += t.y;
        }
        block_sum<2, double>(acc, L.red, L.red + 2 * kWaves);
        const c64 rho = c64{L.red[2 * kWaves], L.red[2 * kWaves + 1]};
        __syncthreads();
        passes += 3.0;
        return rho;
      };
      c64 rho = restart_dir();
      bool fresh = true;
      for (;;) {
        gen_apply_block(g, E, F, p, W, q);
        double acc2[2] = {0.0, 0.0};
        for (int i = tid; i < N; i += kBlock) {
          const c64 t = p[i] * q[i];
          acc2[0] += t.x;
          acc2[1] += t.y;
        }
        block_sum<2, double>(acc2, L.red, L.red + 2 * kWaves);
        const c64 mu = c64{L.red[2 * kWaves], L.red[2 * kWaves + 1]};
        __syncthreads();
        passes += opp + 2.0;
        const double mn = norm2(mu), rn = norm2(rho);
        if (!(mn > 0.0) || !(rn > 0.0) || !isfinite(mn) || !isfinite(rn)) {
          if (fresh) {
            status = (isfinite(mn) && isfinite(rn)) ? VDC_BREAKDOWN : VDC_NONFINITE;
            break;
          }
          beta = true_residual(r);
          if (beta <= a.tol * bnorm) {
            status = VDC_CONVERGED;
            break;
          }
          rho = restart_dir();
          ++cycles;
          fresh = true;
          continue;
        }
        const c64 alpha = cdiv(rho, mu);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int i = tid; i < N; i += kBlock) {
          x[i] = x[i] + alpha * p[i];
          const c64 ri = r[i] - alpha * q[i];
          r[i] = ri;
          acc[0] += norm2(ri);
          const c64 t = ri * (dinv[i] * ri);
          acc[1] += t.x;
          acc[2] += t.y;
        }
        block_sum<3, double>(acc, L.red, L.red + 3 * kWaves);
        const double rr = L.red[3 * kWaves];
        const c64 rho_new = c64{L.red[3 * kWaves + 1], L.red[3 * kWaves + 2]};
        __syncthreads();
        passes += 7.0;
        ++iters;
        fresh = false;
        if (!isfinite(rr)) {
          status = VDC_NONFINITE;
          break;
        }
        if (sqrt(rr) <= a.tol * bnorm || iters >= a.max_iter) {
          beta = true_residual(r);
          if (beta <= a.tol * bnorm) {
            status = VDC_CONVERGED;
            break;
          }
          if (!isfinite(beta)) {
            status = VDC_NONFINITE;
            break;
          }
          if (iters >= a.max_iter) break;
          rho = restart_dir();
          ++cycles;
          fresh = true;
          continue;
        }
        const c64 bt = cdiv(rho_new, rho);
        rho = rho_new;
        for (int i = tid; i < N; i += kBlock) p[i] = dinv[i] * r[i] + bt * p[i];
        passes += 4.0;
      }
    } else {
      // restarted GMRES(m), right preconditioning by dinv
      for (int i = tid; i < N; i += kBlock) V[i] = b[i];
      auto apply = [&](int j, double sc, c64* out) {
        const c64* vj = V + (size_t)j * ld;
        for (int i = tid; i < N; i += kBlock) z[i] = (sc * dinv[i]) * vj[i];
        gen_apply_block(g, E, F, z, W, out);
      };
      for (;;) {
        if (tid == 0) {
          L.K.g[0] = c64{beta, 0.0};
          L.K.vs[0] = 1.0 / beta;
        }
        __syncthreads();
        const CycleResult cr = krylov_cycle<double>(L.K, L.red, V, ld, N, a.m, a.tol * bnorm,
                                                    a.max_iter, iters, Rm, apply);
        passes += cycle_passes(cr.k, cr.reorth_passes) + cr.k * (opp - 4.0) + cr.k + 3.0;
        update_x<double>(V, ld, cr.k, L.K.y, L.K.vs, dinv, x, N);
        beta = true_residual(V);
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
        if (iters >= a.max_iter) break;
      }
    }
    __syncthreads();
    // amplitudes and the cross-section share (Eqs. (15), (16), (24))
    const int out = jb.out;
    if (tid < a.n_final) {
      const int* vf = a.finals + (size_t)tid * kGenMaxModes;
      double s2 = 0.0;
      for (int mu = 0; mu < a.n_pw; ++mu) {
        const c64 T = mu < g.P ? gen_amplitude(g, E, vf, mu, x) : c64{0.0, 0.0};
        a.T_out[((size_t)out * a.n_final + tid) * a.n_pw + mu] = T;
        s2 += norm2(T);
      }
      a.sigma_out[(size_t)out * a.n_final + tid] =
          2.0 * kPi * kPi * kPi / (jb.eps_i / kHartreeEV) * s2;
    }
    if (a.psi_out) {
      c64* psi = a.psi_out + (size_t)out * a.psi_ld;
      for (int i = tid; i < N; i += kBlock) psi[i] = x[i];
    }
    // optical theorem: -Im T_ii = pi sum over open (v_f, mu_f) |T_f|^2 in the
    // truncated basis (A = R + i pi sum Phi Phi^T, Eqs. (19), (23), (25));
    // when asked for (a uniform branch: every thread or none)
    double defect = -1.0;
    if (a.check_optical) {
      double acc[1] = {0.0};
      for (int i = tid; i < g.npts; i += kBlock) {
        if (!(E - g.Enu[i] > 0.0)) continue;
        int nk[kGenMaxModes];
        gen_index(g, i, nk);
        for (int k = g.M; k < kGenMaxModes; ++k) nk[k] = 0;
        for (int mu = 0; mu < g.P; ++mu) acc[0] += norm2(gen_amplitude(g, E, nk, mu, x));
      }
      block_sum<1, double>(acc, L.red, L.red + kWaves);
      const double S = L.red[kWaves];
      __syncthreads();
      const c64 Tii = gen_amplitude(g, E, jb.v, jb.mu, x);
      const double ti = sqrt(norm2(Tii));
      defect = ti > 0.0 ? fabs(-Tii.y - kPi * S) / ti : 0.0;
    }
    if (tid == 0)
      a.info[out] = DevInfo{status, iters, cycles, 0, bnorm > 0.0 ? beta / bnorm : 0.0,
                            passes * 16.0 * N, defect};
  }
}

// Cross sections of Eq. (16): sigma[c][f] = sum of the shares of the jobs j
// with collision[j] = c (their mu_i differ), added in job order.
__global__ void __launch_bounds__(kGenThreads)
sum_waves_kernel(int n_jobs, const int* __restrict__ coll, int n_coll, int n_final,
                 const double* __restrict__ share, double* __restrict__ sigma) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_coll * n_final) return;
  const int c = t / n_final, f = t - c * n_final;
  double s = 0.0;
  for (int j = 0; j < n_jobs; ++j)
    if (coll[j] == c) s += share[(size_t)j * n_final + f];
  sigma[t] = s;
}

hipError_t launch_sum_waves(int n_jobs, const int* coll, int n_coll, int n_final,
                            const double* share, double* sigma, hipStream_t s) {
  const int n = n_coll * n_final;
  hipLaunchKernelGGL(sum_waves_kernel, dim3((n + kGenThreads - 1) / kGenThreads),
                     dim3(kGenThreads), 0, s, n_jobs, coll, n_coll, n_final, share, sigma);
  return hipGetLastError();
}

hipError_t launch_gen_solve(const GenArgs& a, int n_groups, hipStream_t s) {
  hipLaunchKernelGGL(gen_solve_kernel, dim3(n_groups), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

int gen_solve_occupancy() { return occupancy_of(gen_solve_kernel, 0); }

}  // namespace vdc
