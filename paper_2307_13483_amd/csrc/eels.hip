// Two-dimensional electron energy-loss spectra (Eq. (17)) from solutions of
// the two-state model: for each right-hand side (eps_i, v_i, mu_i) its share
// of sigma_{v_f <- v_i} for every final state v_f of the basis (Eqs. (15),
// (16) with T = Phi_f^T Psi, Eq. (24)), spread over the energy-loss grid by
// the spectrometer's resolution, a Gaussian of the given full width at half
// maximum with unit area:
//   S(eps_i, d) = sum_{v_f} sigma_{v_f <- v_i}(eps_i) rho(d - (E_{v_f} - E_{v_i})).
// One workgroup per right-hand side at a time (persistent, jobs from a
// counter): the shares of all final states, in order of their vibrational
// energy, into the workgroup's scratch row; then one thread per grid point
// sums the final states within 8 standard deviations of the Gaussian (the
// rest contributes below 1e-13 of the peak), found by binary search in the
// sorted energies, in that fixed order.
#include "eels.h"

namespace vdc {

__global__ void __launch_bounds__(kBlock) eels_kernel(EelsArgs a) {
  __shared__ int job;
  const DevModel& md = *a.model;
  const int Nc = md.Nc, tid = threadIdx.x;
  double* sh = a.share + (size_t)blockIdx.x * Nc;
  const double c4 = 4.0 * log(2.0) / (a.fwhm * a.fwhm);
  const double norm = 2.0 * sqrt(log(2.0) / kPi) / a.fwhm;
  const double cut = 8.0 * a.fwhm / (2.0 * sqrt(2.0 * log(2.0)));
  for (;;) {
    __syncthreads();
    if (tid == 0) job = atomicAdd(a.counter, 1);
    __syncthreads();
    const int js = job;
    if (js >= a.n_jobs) break;
    const EelsJob jb = a.jobs[js];
    const c64* psi = a.psi + (size_t)js * a.psi_ld;
    const double pref = 2.0 * kPi * kPi * kPi / (jb.eps_i / kHartreeEV);
    for (int k = tid; k < Nc; k += kBlock) {
      const int s = a.order[k], g = s / md.Nu, u = s - g * md.Nu;
      const double eps_f = jb.E - a.Evf[k];
      double s2 = 0.0;
      for (int mu = 0; mu < 2; ++mu) {
        PhiEntry e[6];
        const int n = phi_entries(md, mu, eps_f, g, u, e);
        c64 T = c64{0.0, 0.0};
        for (int q = 0; q < n; ++q)
          T = T + e[q].val * psi[(size_t)e[q].d * Nc + e[q].g * md.Nu + e[q].u];
        s2 += norm2(T);
      }
      sh[k] = pref * s2;
    }
    __syncthreads();
    for (int k = tid; k < a.n_grid; k += kBlock) {
      const double d = a.d0 + k * a.dd;
      const double lo = jb.Evi + d - cut, hi = jb.Evi + d + cut;
      int l = 0, r = Nc;   // first final state with energy >= lo
      while (l < r) {
        const int mid = (l + r) >> 1;
        if (a.Evf[mid] < lo) l = mid + 1; else r = mid;
      }
      double acc = 0.0;
      for (int f = l; f < Nc && a.Evf[f] <= hi; ++f) {
        const double x = d - (a.Evf[f] - jb.Evi);
        acc += sh[f] * (norm * exp(-c4 * x * x));
      }
      a.S[(size_t)jb.out * a.n_grid + k] = acc;
    }
  }
}

hipError_t launch_eels(const EelsArgs& a, int n_groups, hipStream_t s) {
  hipLaunchKernelGGL(eels_kernel, dim3(n_groups), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace vdc
