// Level-shift tables: the six functions F[f_d^mu f_d'^mu](eps) of Eq. (19)
// at eps = E - E_nu for every basis point nu and every total energy E of a
// batch, stored in the symmetry-block layout the solver reads.
//
// Real part: principal value of the piecewise-linear interpolant L of
// g = sqrt(Gamma_d Gamma_d') on the model's nodes x_k, in closed form
//     2 pi Delta(eps) = sum_k c_k psi(eps - x_k) - g_{K-1} (ln|eps - x_{K-1}| + 1),
// psi(t) = t ln|t|, c_k = s_k - s_{k-1} the jumps of the interpolant's slope
// (s_{-1} = s_{K-1} = 0; g_0 = 0 because Gamma(0) = 0).  This follows from
// integrating L(x)/(eps - x) segment by segment and summing by parts.
// All six functions share the same psi(eps - x_k), so each node costs one
// logarithm and six fused multiply-adds.
// Imaginary part: -g(eps)/2 = -pi f_d f_d' for eps > 0, else 0 (analytic).
#include "internal.h"

namespace vdc {

__device__ inline double width_pair(const DevModel& m, int mu, int d1, int d2, double eps) {
  if (!(eps > 0.0)) return 0.0;
  const double A = sqrt(m.A[d1][mu] * m.A[d2][mu]);
  const double rB = 0.5 / m.B[d1][mu] + 0.5 / m.B[d2][mu];
  return A * pow(eps, m.l[mu] + 0.5) * exp(-eps * rB);
}

// The six complex values at one electron energy eps.
__device__ inline void level_shift6(const DevModel& m, double eps, c64 out[kNumF]) {
  double acc[kNumF];
#pragma unroll
  for (int f = 0; f < kNumF; ++f) acc[f] = 0.0;
  const double* __restrict__ xk = m.nodes;
  const double* __restrict__ ck = m.coef;
  for (int k = 0; k < m.K; ++k) {
    const double t = eps - xk[k];
    const double psi = (t == 0.0) ? 0.0 : t * log(fabs(t));
#pragma unroll
    for (int f = 0; f < kNumF; ++f) acc[f] = fma(ck[k * kNumF + f], psi, acc[f]);
  }
  const double tl = eps - xk[m.K - 1];
  const double lnl = (tl == 0.0) ? 0.0 : log(fabs(tl));
  const double inv2pi = 1.0 / (2.0 * kPi);
#pragma unroll
  for (int f = 0; f < kNumF; ++f) out[f].x = (acc[f] - m.glast[f] * (lnl + 1.0)) * inv2pi;
  // imaginary parts, pairs (1,1), (1,2), (2,2) per mu
#pragma unroll
  for (int mu = 0; mu < 2; ++mu) {
    out[fidx(mu, 0)].y = -0.5 * width_pair(m, mu, 0, 0, eps);
    out[fidx(mu, 1)].y = -0.5 * width_pair(m, mu, 0, 1, eps);
    out[fidx(mu, 2)].y = -0.5 * width_pair(m, mu, 1, 1, eps);
  }
}

// One thread per (energy, basis point).  Writes both parity tables:
// table[(p*3 + slot)*Nc + i], slots (AA, AB, BB) of the active state at i:
// state 1 active (n_u + p even): (F[1e1e], F[1e2e], F[2e2e]);
// state 2 active:               (F[2o2o], F[1o2o], F[1o1o]).
__global__ void __launch_bounds__(256)
level_shift_tables_kernel(const DevModel* __restrict__ models, const DevTable* __restrict__ tabs,
                          int max_nc, c64* __restrict__ base, c32* __restrict__ base32) {
  const int t = blockIdx.y;
  const DevTable tb = tabs[t];
  const DevModel& m = models[tb.model];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.Nc) return;
  const int ng = i / m.Nu, nu = i - ng * m.Nu;
  const double Ev = m.omega_g * (ng + 0.5) + m.omega_u * (nu + 0.5);
  c64 F[kNumF];
  level_shift6(m, tb.E - Ev, F);
  for (int p = 0; p < 2; ++p) {
    const bool s1 = ((nu + p) & 1) == 0;
    const c64 aa = s1 ? F[0] : F[5];
    const c64 ab = s1 ? F[1] : F[4];
    const c64 bb = s1 ? F[2] : F[3];
    c64* dst = base + tb.offset + (size_t)(p * 3) * m.Nc;
    dst[i] = aa;
    dst[m.Nc + i] = ab;
    dst[2 * (size_t)m.Nc + i] = bb;
    if (base32) {
      c32* d32 = base32 + tb.offset + (size_t)(p * 3) * m.Nc;
      d32[i] = c32{(float)aa.x, (float)aa.y};
      d32[m.Nc + i] = c32{(float)ab.x, (float)ab.y};
      d32[2 * (size_t)m.Nc + i] = c32{(float)bb.x, (float)bb.y};
    }
  }
}

__global__ void __launch_bounds__(256)
level_shift_points_kernel(DevModel m, int n, const double* __restrict__ eps, c64* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  c64 F[kNumF];
  level_shift6(m, eps[i], F);
#pragma unroll
  for (int f = 0; f < kNumF; ++f) out[(size_t)i * kNumF + f] = F[f];
}

hipError_t launch_level_shift_tables(const DevModel* models_dev, const DevTable* tables_dev,
                                     int n_tables, int max_nc, c64* table_base,
                                     c32* table32_base, hipStream_t s) {
  if (n_tables <= 0) return hipSuccess;
  dim3 grid((max_nc + 255) / 256, n_tables);
  hipLaunchKernelGGL(level_shift_tables_kernel, grid, dim3(256), 0, s, models_dev, tables_dev,
                     max_nc, table_base, table32_base);
  return hipGetLastError();
}

hipError_t launch_level_shift_points(const DevModel& m, int n_eps, const double* eps, c64* out,
                                     hipStream_t s) {
  if (n_eps <= 0) return hipSuccess;
  hipLaunchKernelGGL(level_shift_points_kernel, dim3((n_eps + 255) / 256), dim3(256), 0, s, m,
                     n_eps, eps, out);
  return hipGetLastError();
}

}  // namespace vdc
