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
//
// Far field: for a cluster of kClus consecutive nodes with centre x_c and
// half-width r, and t = eps - x_c with |t| >= 3 r, the cluster's part of the
// sum is the convergent series (psi^(n)(t) = (-1)^n (n-2)! / t^(n-1), n >= 2)
//     sum_k c_k psi(t - d_k) = t ln|t| M_0 - (ln|t| + 1) M_1
//                              + sum_{n>=2} M_n / (n (n-1)) t^-(n-1),
// M_n = sum_k c_k d_k^n, d_k = x_k - x_c, truncated at n = 30 (remainder
// below 3^-31 / 900 of the cluster's magnitude); its eps derivative follows
// term by term.  Near clusters are summed node by node; groups of kSup
// clusters have moments of their own for points far from the whole group.
// Points are processed in order of eps (a permutation per offset
// rectangle), so the lanes of a wave agree on which clusters are far; a
// cluster is expanded only if it is far for every lane of the wave.
//
// Sharing across initial states: eps_nu = eps_i + w_g (v_g - n_g) + w_u (v_u - n_u)
// depends on (n_g, n_u) only through the offsets (v_g - n_g, v_u - n_u), so
// the jobs with one incident energy eps_i evaluate the transform once on the
// rectangle of offsets they need ("shift table"), and a gather pass writes
// each total energy's block tables from it.
#include "internal.h"
#include "terms_args.h"

namespace vdc {

constexpr int kLsThreads = 256;

// ln|t| for t != 0, finite: t = m 2^e with m in [1/sqrt2, sqrt2),
// ln m = 2 atanh(s), s = (m-1)/(m+1), |s| <= 0.1716, by its odd power series
// (11 terms: the remainder is below 2^-56 relative), plus e ln 2 with ln 2
// split into a 32-bit head and a tail so e*ln2_hi is exact.
__device__ inline double ln_abs(double t) {
  int e;
  double m = frexp(fabs(t), &e);            // [0.5, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double num = m - 1.0;               // exact
  const double den = m + 1.0;
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  r = fma(r, fma(-den, r, 1.0), r);
  double s = num * r;
  s = fma(r, fma(-s, den, num), s);         // one residual correction
  const double z = s * s;
  double p = 1.0 / 23.0;
  p = fma(p, z, 1.0 / 21.0);
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double lnm = fma(2.0 * s * z, p, 2.0 * s);
  const double ln2_hi = 6.93147180369123816490e-01;   // 32 significant bits
  const double ln2_lo = 1.90821492927058770002e-10;
  const double de = (double)e;
  return fma(de, ln2_hi, fma(de, ln2_lo, lnm));
}

__device__ inline double width_pair(const DevModel& m, int mu, int d1, int d2, double eps) {
  if (!(eps > 0.0)) return 0.0;
  const double A = sqrt(m.A[d1][mu] * m.A[d2][mu]);
  const double rB = 0.5 / m.B[d1][mu] + 0.5 / m.B[d2][mu];
  return A * pow(eps, m.l[mu] + 0.5) * exp(-eps * rB);
}

// A pointer that is the same for every lane, moved to scalar registers and
// to the constant address space so that reads through it with lane-uniform
// offsets become scalar loads (the data is read-only during the kernel).
typedef const __attribute__((address_space(4))) double* uniform_dptr;
__device__ inline uniform_dptr uniform_ptr(const double* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (uniform_dptr)(((uint64_t)hi << 32) | lo);
}

// Far-field terms of one cluster (or super-cluster) C at t = eps - x_c,
// added to the sums (see the series above).
template <bool DERIV>
__device__ inline void far_terms(uniform_dptr C, double t, double* aF, double* aD, double* aX) {
  const double L = ln_abs(t);
  double u = __builtin_amdgcn_rcp(t);
  u = fma(u, fma(-t, u, 1.0), u);
  u = fma(u, fma(-t, u, 1.0), u);
  const double tl = t * L, l1 = L + 1.0;
#pragma unroll
  for (int f = 0; f < kNumF; ++f) {
    const uniform_dptr M = C + 2 + f * (kClusP + 1);
    double ser = M[kClusP];
    for (int n = kClusP - 1; n >= 2; --n) ser = fma(ser, u, M[n]);
    aF[f] += fma(tl, M[0], fma(-l1, M[1], u * ser));
    if (DERIV) {
      double sd = (kClusP - 1) * M[kClusP];
      for (int n = kClusP - 1; n >= 2; --n) sd = fma(sd, u, (n - 1) * M[n]);
      aD[f] += fma(L, M[0], -u * fma(u, sd, M[1]));
      const uniform_dptr MX = C + 2 + (kNumF + f) * (kClusP + 1);
      double sx = MX[kClusP];
      for (int n = kClusP - 1; n >= 2; --n) sx = fma(sx, u, MX[n]);
      aX[f] += fma(tl, MX[0], fma(-l1, MX[1], u * sx));
    }
  }
}

// Sums over the nodes of the transform for one electron energy: aF[f] =
// sum_k c_k psi(eps - x_k) (g's slope jumps), with DERIV also
// aD[f] = sum_k c_k ln|eps - x_k| and aX[f] = sum_k cx_k psi(eps - x_k)
// (x g's slope jumps).  Called by every lane of a wave (inactive lanes pass
// active = false and vote "far").  Two levels: a super-cluster of kSup
// clusters far for the whole wave takes one expansion (away from the nodes'
// range, where most points of a workload lie, 8 instead of 64), else each of
// its clusters is expanded or, where near, summed node by node.
template <bool DERIV>
__device__ inline void node_sums(const DevModel& m, double eps, bool active, double* aF,
                                 double* aD, double* aX) {
#pragma unroll
  for (int f = 0; f < kNumF; ++f) aF[f] = aD[f] = aX[f] = 0.0;
  const uniform_dptr clus = uniform_ptr(m.clus);
  const uniform_dptr sup = uniform_ptr(m.sup);
  const uniform_dptr nodes = uniform_ptr(m.nodes);
  const uniform_dptr coef = uniform_ptr(m.coef);
  const uniform_dptr coefx = uniform_ptr(m.coefx);
  const int nclust = __builtin_amdgcn_readfirstlane(m.nclust);
  const int nsup = __builtin_amdgcn_readfirstlane(m.nsup);
  const int K = __builtin_amdgcn_readfirstlane(m.K);
  for (int sc = 0; sc < nsup; ++sc) {
    const uniform_dptr S = sup + (size_t)sc * kClusStride;
    const double ts = eps - S[0];
    if (__all(!active || (fabs(ts) >= 3.0 * S[1] && ts != 0.0))) {
      far_terms<DERIV>(S, ts, aF, aD, aX);
      continue;
    }
    const int c1 = min(nclust, (sc + 1) * kSup);
    for (int c = sc * kSup; c < c1; ++c) {
      const uniform_dptr C = clus + (size_t)c * kClusStride;
      const double t = eps - C[0];
      if (__all(!active || (fabs(t) >= 3.0 * C[1] && t != 0.0))) {
        far_terms<DERIV>(C, t, aF, aD, aX);
      } else if (active) {
        const int k1 = min(K, (c + 1) * kClus);
        for (int k = c * kClus; k < k1; ++k) {
          const double tk = eps - nodes[k];
          const double ln = (tk == 0.0) ? 0.0 : ln_abs(tk);
          const double psi = tk * ln;
#pragma unroll
          for (int f = 0; f < kNumF; ++f) {
            const double ck = coef[(size_t)k * kNumF + f];
            aF[f] = fma(ck, psi, aF[f]);
            if (DERIV) {
              aD[f] = fma(ck, ln, aD[f]);
              aX[f] = fma(coefx[(size_t)k * kNumF + f], psi, aX[f]);
            }
          }
        }
      }
    }
  }
}

// The six complex level shifts at eps (Re from the node sums, Im analytic).
__device__ inline void level_shift6(const DevModel& m, double eps, bool active, c64 out[kNumF]) {
  double aF[kNumF], aD[kNumF], aX[kNumF];
  node_sums<false>(m, eps, active, aF, aD, aX);
  const double tl = eps - m.nodes[m.K - 1];
  const double lnl = (tl == 0.0) ? 0.0 : ln_abs(tl);
  const double inv2pi = 1.0 / (2.0 * kPi);
#pragma unroll
  for (int f = 0; f < kNumF; ++f) out[f].x = (aF[f] - m.glast[f] * (lnl + 1.0)) * inv2pi;
#pragma unroll
  for (int mu = 0; mu < 2; ++mu) {
    out[fidx(mu, 0)].y = -0.5 * width_pair(m, mu, 0, 0, eps);
    out[fidx(mu, 1)].y = -0.5 * width_pair(m, mu, 0, 1, eps);
    out[fidx(mu, 2)].y = -0.5 * width_pair(m, mu, 1, 1, eps);
  }
}

// Shift tables: one thread per (group, offset point).  Group g covers offsets
// a in [a_min, a_min + na), b in [b_min, b_min + nb) at eps_i + w_g a + w_u b,
// stored [point][6] from the group's offset.
__global__ void __launch_bounds__(kLsThreads)
shift_table_kernel(const DevModel* __restrict__ models, const DevGroup* __restrict__ groups,
                   const int* __restrict__ perm, c64* __restrict__ shift) {
  const DevGroup gr = groups[blockIdx.y];
  const DevModel& m = models[gr.model];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int npts = gr.na * gr.nb;
  if (blockIdx.x * blockDim.x >= npts) return;   // whole workgroup beyond the rectangle
  const bool active = s < npts;
  int i = 0;
  double eps = 0.0;
  if (active) {
    i = perm[gr.perm_off + s];
    const int ia = i / gr.nb, ib = i - ia * gr.nb;
    eps = gr.eps_i + m.omega_g * (gr.a_min + ia) + m.omega_u * (gr.b_min + ib);
  }
  c64 F[kNumF];
  level_shift6(m, eps, active, F);
  if (active) {
#pragma unroll
    for (int f = 0; f < kNumF; ++f) shift[gr.offset + (size_t)i * kNumF + f] = F[f];
  }
}

// Block tables of one total energy from its group's shift table:
// table[(p*3 + slot)*Nc + i], slots (AA, AB, BB) of the active state at i:
// state 1 active (n_u + p even): (F[1e1e], F[1e2e], F[2e2e]);
// state 2 active:               (F[2o2o], F[1o2o], F[1o1o]).
__global__ void __launch_bounds__(kLsThreads)
gather_tables_kernel(const DevModel* __restrict__ models, const DevGroup* __restrict__ groups,
                     const DevTable* __restrict__ tabs, const c64* __restrict__ shift,
                     c64* __restrict__ base, c32* __restrict__ base32) {
  const DevTable tb = tabs[blockIdx.y];
  const DevModel& m = models[tb.model];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.Nc) return;
  const DevGroup gr = groups[tb.group];
  const int ng = i / m.Nu, nu = i - ng * m.Nu;
  const int ia = tb.vg - ng - gr.a_min, ib = tb.vu - nu - gr.b_min;
  const c64* F = shift + gr.offset + (size_t)(ia * gr.nb + ib) * kNumF;
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

// Level shift, its eps derivative and the transform of x g(x) (for the
// derivatives in the width scales B), from the same node sums:
//   2 pi dDelta/deps = sum_k c_k ln|eps - x_k| - g_{K-1}/(eps - x_{K-1})
// (the "+1" of d psi/dt drops out because the slope jumps sum to zero), and
// the x g transform is the level shift with the slope jumps of x g.
// Imaginary parts: -g'(eps)/2 and -eps g(eps)/2 (analytic).
__device__ inline void level_shift18(const DevModel& m, double eps, bool active, c64 F[kNumF],
                                     c64 D[kNumF], c64 X[kNumF]) {
  double aF[kNumF], aD[kNumF], aX[kNumF];
  node_sums<true>(m, eps, active, aF, aD, aX);
  const double tl = eps - m.nodes[m.K - 1];
  const double lnl = (tl == 0.0) ? 0.0 : ln_abs(tl);
  const double itl = (tl == 0.0) ? 0.0 : 1.0 / tl;
  const double inv2pi = 1.0 / (2.0 * kPi);
#pragma unroll
  for (int f = 0; f < kNumF; ++f) {
    F[f].x = (aF[f] - m.glast[f] * (lnl + 1.0)) * inv2pi;
    D[f].x = (aD[f] - m.glast[f] * itl) * inv2pi;
    X[f].x = (aX[f] - m.glastx[f] * (lnl + 1.0)) * inv2pi;
  }
  const int pairs[3][2] = {{0, 0}, {0, 1}, {1, 1}};
#pragma unroll
  for (int mu = 0; mu < 2; ++mu) {
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int d1 = pairs[pq][0], d2 = pairs[pq][1];
      const double g = width_pair(m, mu, d1, d2, eps);
      const double rate = (eps > 0.0) ? (m.l[mu] + 0.5) / eps - (0.5 / m.B[d1][mu] + 0.5 / m.B[d2][mu])
                                      : 0.0;
      F[fidx(mu, pq)].y = -0.5 * g;
      D[fidx(mu, pq)].y = -0.5 * g * rate;
      X[fidx(mu, pq)].y = -0.5 * eps * g;
    }
  }
}

__global__ void __launch_bounds__(kLsThreads)
shift_table_deriv_kernel(const DevModel* __restrict__ models, const DevGroup* __restrict__ groups,
                         const int* __restrict__ perm, c64* __restrict__ shift) {
  const DevGroup gr = groups[blockIdx.y];
  const DevModel& m = models[gr.model];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int npts = gr.na * gr.nb;
  if (blockIdx.x * blockDim.x >= npts) return;
  const bool active = s < npts;
  int i = 0;
  double eps = 0.0;
  if (active) {
    i = perm[gr.perm_off + s];
    const int ia = i / gr.nb, ib = i - ia * gr.nb;
    eps = gr.eps_i + m.omega_g * (gr.a_min + ia) + m.omega_u * (gr.b_min + ib);
  }
  c64 F[kNumF], D[kNumF], X[kNumF];
  level_shift18(m, eps, active, F, D, X);
  if (active) {
    c64* o = shift + gr.offset + (size_t)i * 3 * kNumF;
#pragma unroll
    for (int f = 0; f < kNumF; ++f) {
      o[f] = F[f];
      o[kNumF + f] = D[f];
      o[2 * kNumF + f] = X[f];
    }
  }
}

// Adjoint table sets: per parity 9 planes (F, dF/deps, X) x (AA, AB, BB).
__global__ void __launch_bounds__(kLsThreads)
gather_tables_deriv_kernel(const DevModel* __restrict__ models,
                           const DevGroup* __restrict__ groups,
                           const DevTable* __restrict__ tabs, const c64* __restrict__ shift,
                           c64* __restrict__ base) {
  const DevTable tb = tabs[blockIdx.y];
  const DevModel& m = models[tb.model];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.Nc) return;
  const DevGroup gr = groups[tb.group];
  const int ng = i / m.Nu, nu = i - ng * m.Nu;
  const int ia = tb.vg - ng - gr.a_min, ib = tb.vu - nu - gr.b_min;
  const c64* S = shift + gr.offset + (size_t)(ia * gr.nb + ib) * 3 * kNumF;
  for (int p = 0; p < 2; ++p) {
    const bool s1 = ((nu + p) & 1) == 0;
    c64* dst = base + tb.offset + (size_t)(p * kPlanesDeriv) * m.Nc;
    for (int kind = 0; kind < 3; ++kind) {
      const c64* F = S + kind * kNumF;
      dst[(size_t)(3 * kind) * m.Nc + i] = s1 ? F[0] : F[5];
      dst[(size_t)(3 * kind + 1) * m.Nc + i] = s1 ? F[1] : F[4];
      dst[(size_t)(3 * kind + 2) * m.Nc + i] = s1 ? F[2] : F[3];
    }
  }
}

__global__ void __launch_bounds__(kLsThreads)
level_shift_points_kernel(DevModel m, int n, const double* __restrict__ eps, c64* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < n;
  c64 F[kNumF];
  level_shift6(m, active ? eps[i] : 0.0, active, F);
  if (active) {
#pragma unroll
    for (int f = 0; f < kNumF; ++f) out[(size_t)i * kNumF + f] = F[f];
  }
}

// Level-shift planes of the general model at total energy E (one table per
// (model, E)): each of the model's two-state transform models c evaluates
// its six functions at eps_nu = E - E_nu, and lsmap[c][f] names the plane
// F^mu_dd' that function f of c supplies (-1: a duplicate, not stored).
// Points are visited in order of E_nu (perm), so a wave's lanes agree on
// which node clusters are far.
__global__ void __launch_bounds__(kLsThreads)
gen_planes_kernel(const DevGen* __restrict__ gens, const GenTab* __restrict__ tabs,
                  c64* __restrict__ base) {
  const GenTab tb = tabs[blockIdx.z];
  const DevGen& g = gens[tb.model];
  const int c = blockIdx.y;
  if (c >= g.nlsm || blockIdx.x * blockDim.x >= g.npts) return;   // whole workgroup
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = s < g.npts;
  const int i = active ? g.perm[s] : 0;
  const double eps = active ? tb.E - g.Enu[i] : 0.0;
  c64 F[kNumF];
  level_shift6(g.lsm[c], eps, active, F);
  if (active) {
#pragma unroll
    for (int f = 0; f < kNumF; ++f) {
      const int pl = g.lsmap[c * kNumF + f];
      if (pl >= 0) base[tb.offset + (size_t)pl * g.npts + i] = F[f];
    }
  }
}

hipError_t launch_gen_planes(const DevGen* gens, const GenTab* tabs, int n_tabs, int max_npts,
                             int max_nlsm, c64* base, hipStream_t s) {
  if (n_tabs <= 0 || max_nlsm <= 0) return hipSuccess;
  const dim3 grid((max_npts + kLsThreads - 1) / kLsThreads, max_nlsm, n_tabs);
  hipLaunchKernelGGL(gen_planes_kernel, grid, dim3(kLsThreads), 0, s, gens, tabs, base);
  return hipGetLastError();
}

hipError_t launch_level_shift_tables(const DevModel* models_dev, const DevGroup* groups_dev,
                                     int n_groups, int max_group_pts, const int* perm,
                                     const DevTable* tables_dev, int n_tables, int max_nc,
                                     c64* shift, c64* table_base, c32* table32_base,
                                     hipStream_t s, bool deriv) {
  if (n_tables <= 0) return hipSuccess;
  dim3 g1((max_group_pts + kLsThreads - 1) / kLsThreads, n_groups);
  if (deriv) {
    hipLaunchKernelGGL(shift_table_deriv_kernel, g1, dim3(kLsThreads), 0, s, models_dev,
                       groups_dev, perm, shift);
    dim3 g2((max_nc + kLsThreads - 1) / kLsThreads, n_tables);
    hipLaunchKernelGGL(gather_tables_deriv_kernel, g2, dim3(kLsThreads), 0, s, models_dev,
                       groups_dev, tables_dev, shift, table_base);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(shift_table_kernel, g1, dim3(kLsThreads), 0, s, models_dev, groups_dev, perm,
                     shift);
  dim3 g2((max_nc + kLsThreads - 1) / kLsThreads, n_tables);
  hipLaunchKernelGGL(gather_tables_kernel, g2, dim3(kLsThreads), 0, s, models_dev, groups_dev,
                     tables_dev, shift, table_base, table32_base);
  return hipGetLastError();
}

hipError_t launch_level_shift_points(const DevModel& m, int n_eps, const double* eps, c64* out,
                                     hipStream_t s) {
  if (n_eps <= 0) return hipSuccess;
  hipLaunchKernelGGL(level_shift_points_kernel, dim3((n_eps + kLsThreads - 1) / kLsThreads),
                     dim3(kLsThreads), 0, s, m, n_eps, eps, out);
  return hipGetLastError();
}

}  // namespace vdc
