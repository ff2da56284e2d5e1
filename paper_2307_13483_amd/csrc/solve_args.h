// Arguments of the solver kernels and the per-job epilogue (amplitudes,
// cross-section share, solution, status) shared by every solve path.
#pragma once
#include "op2d.h"

namespace vdc {

// Sum of NV values over a workgroup of blockDim.x <= kBlock threads (a
// multiple of 64): wave xor-butterflies, then the wave partials in wave
// order (fixed order).  Result in out[0..NV-1] after a barrier.
template <int NV>
__device__ inline void block_sum_any(double (&v)[NV], double* red, double* out) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] += __shfl_xor(v[q], s, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[wave * NV + q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w * NV + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

struct SolveArgs {
  const DevModel* models;
  const DevJob* jobs;
  int n_jobs;
  const DevTable* tabs;
  const c64* tables;        // FP64 level-shift tables
  const c32* tables32;      // FP32 copy (mixed precision only)
  int* counter;             // job queue head
  c64* scratch;             // per-workgroup slots
  size_t slot_elems;        // c64 elements per slot
  size_t ncap;              // leading dimension of slot vectors (>= max Nc)
  int m;                    // restart length (outer length for FP32_INNER)
  int max_iter;
  double tol;
  int precond;
  int method;               // VDC_GMRES or VDC_COCG (the adjoint's solve)
  int m_in;                 // FP32_INNER: inner restart length
  double tol_in;            // FP32_INNER: inner relative tolerance
  int n_final;
  const int* finals;        // device [n_final][2]
  c64* T_out;               // [n_jobs][n_final][2]
  double* sigma_out;        // [n_jobs][n_final]
  c64* psi_out;             // [n_jobs][2 Nc] or null (row length of the job's model)
  size_t psi_ld;            // row length of psi_out (2 * max Nc)
  DevInfo* info;            // [n_jobs], indexed by the caller's job order
  int planes;               // table planes per parity (3, or 9 for the adjoint)
  int tileT;                // rows per LDS tile of the FP64 matvec (0: two-phase)
  int tileT32;              // the same for the FP32 inner matvec
  // adjoint inputs/outputs
  const c64* psi_in;        // forward solutions, full layout, row length psi_ld
  const c64* T_in;          // forward amplitudes [n_jobs][n_final][2]
  const double* dsig;       // dL/dsigma [n_jobs][n_final]
  double* grad;             // [n_jobs][16] per-job gradient contributions
  // residual histories (vdc_solve_history): [n_jobs][hist_len] or null
  double* hist;
  int hist_len;
  int check_optical;        // compute the optical-theorem defect of each solution
};

// The solver kernels come in two instantiations: diag = false (the default
// launch: no defect pass, no history stores, nothing of either in the
// kernel) and diag = true (the launch when the defect or histories are asked
// for), so that the default kernel's register allocation is not burdened by
// code it does not run.

// This job's history row, or null (always null in a diag = false kernel).
template <bool diag>
__device__ inline double* hist_row(const SolveArgs& a, const DevJob& jb) {
  if constexpr (!diag) return nullptr;
  return a.hist ? a.hist + (size_t)jb.out * a.hist_len : nullptr;
}

// Optical-theorem defect of the solution x of the job's symmetry block,
// |-Im T_ii - pi sum_{open v_f} sum_{mu_f} |T_f|^2| / |T_ii|, where T_ii is the
// job's elastic amplitude and the sum runs over every open final state of
// the basis: the truncated-basis identity that follows from A = R + i pi
// sum Phi Phi^T (Eqs. (19), (23), (25)), exact for the exact solution.  In
// the block at a point where state a is active only the wave mu = a has an
// amplitude, T = f_a^a(eps) (1 + lam_a q_g) x + f_b^a(eps) q_u x (b the
// other state), from the same neighbours as the operator.  All threads,
// after a barrier; returned to every thread.
__device__ inline double optical_defect(const DevModel& md, const DevJob& jb, const c64* x,
                                        double Tii_im, double Tii_abs) {
  __shared__ double red[kWaves + 1];
  double acc[1] = {0.0};
  const int Nu = md.Nu;
  for (int i = threadIdx.x; i < md.Nc; i += blockDim.x) {
    const int ng = i / Nu, nu = i - ng * Nu;
    const double eps = jb.E - (md.omega_g * (ng + 0.5) + md.omega_u * (nu + 0.5));
    if (!(eps > 0.0)) continue;
    const int act = (nu + jb.parity) & 1;
    const double fa = coupling_f(md, act, act, eps), fb = coupling_f(md, 1 - act, act, eps);
    c64 zg = c64{0.0, 0.0}, zu = c64{0.0, 0.0};
    if (ng > 0) zg = sqrt(0.5 * ng) * x[i - Nu];
    if (ng + 1 < md.Ng) zg = zg + sqrt(0.5 * (ng + 1)) * x[i + Nu];
    if (nu > 0) zu = sqrt(0.5 * nu) * x[i - 1];
    if (nu + 1 < Nu) zu = zu + sqrt(0.5 * (nu + 1)) * x[i + 1];
    const c64 T = fa * (x[i] + md.lamd[act] * zg) + fb * zu;
    acc[0] += norm2(T);
  }
  block_sum_any<1>(acc, red, red + kWaves);
  const double S = red[kWaves];
  __syncthreads();
  return Tii_abs > 0.0 ? fabs(-Tii_im - kPi * S) / Tii_abs : 0.0;
}

// Amplitudes T_{mu_f v_f <- mu_i v_i} = Phi^{v_f mu_f T} Psi (Eq. (24)) for the
// solution x of the job's symmetry block, the share 2 pi^3/eps_i sum_{mu_f}|T|^2
// of sigma_{v_f <- v_i} (Eq. (16), eps_i in hartree), the full-layout Psi, the
// optical-theorem defect (diag kernels with check_optical set; else -1) and
// the status.  Called by all threads of the workgroup after a barrier.
template <bool diag>
__device__ inline void finish_job(const SolveArgs& a, const DevModel& md, const DevJob& jb,
                                  const c64* x, int tid, int status, int iters, int cycles,
                                  int outer, double rel_res, double alg_bytes) {
  const int out = jb.out;
  double defect = -1.0;
  if constexpr (diag) {
    if (a.check_optical) {
      // the elastic amplitude T_ii (every thread, from the few entries of Phi_i)
      c64 Tii = c64{0.0, 0.0};
      PhiEntry e[6];
      const int n = phi_entries(md, jb.mu, jb.eps_i, jb.vi_g, jb.vi_u, e);
      for (int q = 0; q < n; ++q)
        if (((e[q].u + jb.parity) & 1) == e[q].d)
          Tii = Tii + e[q].val * x[e[q].g * md.Nu + e[q].u];
      defect = optical_defect(md, jb, x, Tii.y, sqrt(norm2(Tii)));
      // the defect pass reads x once more (16 B per block unknown)
      alg_bytes += 16.0 * md.Nc;
    }
  }
  if (tid < a.n_final) {
    const int g = a.finals[2 * tid], u = a.finals[2 * tid + 1];
    const double eps_f = jb.E - (md.omega_g * (g + 0.5) + md.omega_u * (u + 0.5));
    double s2 = 0.0;
    for (int mu = 0; mu < 2; ++mu) {
      c64 T = c64{0.0, 0.0};
      if (g >= 0 && g < md.Ng && u >= 0 && u < md.Nu) {
        PhiEntry e[6];
        const int n = phi_entries(md, mu, eps_f, g, u, e);
        for (int q = 0; q < n; ++q)
          if (((e[q].u + jb.parity) & 1) == e[q].d) T = T + e[q].val * x[e[q].g * md.Nu + e[q].u];
      }
      a.T_out[((size_t)out * a.n_final + tid) * 2 + mu] = T;
      s2 += norm2(T);
    }
    a.sigma_out[(size_t)out * a.n_final + tid] = 2.0 * kPi * kPi * kPi / (jb.eps_i / kHartreeEV) * s2;
  }
  if (a.psi_out) {
    c64* psi = a.psi_out + (size_t)out * a.psi_ld;
    for (int i = tid; i < md.Nc; i += blockDim.x) {
      const int nu = i % md.Nu;
      const int act = (nu + jb.parity) & 1;
      psi[(size_t)act * md.Nc + i] = x[i];
      psi[(size_t)(1 - act) * md.Nc + i] = c64{0.0, 0.0};
    }
  }
  if (tid == 0) a.info[out] = DevInfo{status, iters, cycles, outer, rel_res, alg_bytes, defect};
}

}  // namespace vdc
