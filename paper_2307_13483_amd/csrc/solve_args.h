// Arguments of the solver kernels and the per-job epilogue (amplitudes,
// cross-section share, solution, status) shared by every solve path.
#pragma once
#include "op2d.h"

namespace vdc {

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
};

// Amplitudes T_{mu_f v_f <- mu_i v_i} = Phi^{v_f mu_f T} Psi (Eq. (24)) for the
// solution x of the job's symmetry block, the share 2 pi^3/eps_i sum_{mu_f}|T|^2
// of sigma_{v_f <- v_i} (Eq. (16), eps_i in hartree), the full-layout Psi and
// the status.  Called by all threads of the workgroup after a barrier.
__device__ inline void finish_job(const SolveArgs& a, const DevModel& md, const DevJob& jb,
                                  const c64* x, int tid, int status, int iters, int cycles,
                                  int outer, double rel_res, double alg_bytes) {
  const int out = jb.out;
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
  if (tid == 0) a.info[out] = DevInfo{status, iters, cycles, outer, rel_res, alg_bytes};
}

}  // namespace vdc
