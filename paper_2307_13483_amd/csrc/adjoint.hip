// Adjoint gradient of cross sections with respect to the 16 model parameters
// (w_g, w_u, k_1, k_2, lam, lam_1, lam_2, gap, A_1e, A_2e, A_1o, A_2o, B_1e,
// B_2e, B_1o, B_2o), one workgroup per job as in the forward solver.
//
// For a job (eps_i, v_i, mu_i) with forward solution Psi and amplitudes T_f,
// and dL/dsigma_f given per final state, the complex weights
//     W_f = 2 c (dL/dsigma_f) conj(T_f),  c = 2 pi^3 / eps_i  (Eq. (16)),
// make dL = Re sum_f W_f dT_f.  With T_f = Phi_f^T A^-1 Phi_i (Eq. (24)) and
// A^T = A (complex symmetric, Sec. III.A) one extra solve with the same
// operator,  A zeta = sum_f W_f Phi_f,  gives
//     dL/dp = Re[ sum_f W_f (dPhi_f/dp)^T Psi + zeta^T dPhi_i/dp - zeta^T (dA/dp) Psi ].
// zeta^T (dA/dp) Psi is a sum over grid points of bilinear forms in the
// block stencil quantities (u_A, u_B of both vectors, as in op2d.h): the
// diagonal E - E_nu - E_d (w_g, w_u, gap), the direct couplings (k_d, lam),
// the (1 + lam_d q_g) factors of the sandwich (lam_d), and the level-shift
// diagonals through dF/deps (w_g, w_u), F/A (A) and the transform of x g (B).
#include "cocg_block.h"
#include "solve_args.h"

namespace vdc {

constexpr int kNumParams = 16;
constexpr int kRedA = kWaves * 16 + 16;

struct AdjLds {
  Fp64Lds S;
  double dot[2];
  double redA[kRedA];
  c64 W[2 * kMaxFinal];
  int job;
};

struct PhiTerm { int d, g, u, kind; double f, o, sfac; };

// Components of Phi^{v mu} = f_d^mu(eps) <nu|O_d^mu|v> split into the coupling
// f and the matrix element o (kind 0: the 1 of 1 + lam_d q_g, kind 1: its
// lam_d q_g part with sfac = <nu|q_g|v>, kind 2: q_u).
__device__ inline int phi_terms(const DevModel& m, int mu, double eps, int g, int u, PhiTerm* t) {
  int n = 0;
  for (int d = 0; d < 2; ++d) {
    const double f = coupling_f(m, d, mu, eps);
    if (f == 0.0) continue;
    if (d == mu) {
      t[n++] = PhiTerm{d, g, u, 0, f, 1.0, 0.0};
      if (g + 1 < m.Ng) {
        const double q = sqrt(0.5 * (g + 1));
        t[n++] = PhiTerm{d, g + 1, u, 1, f, m.lamd[d] * q, q};
      }
      if (g > 0) {
        const double q = sqrt(0.5 * g);
        t[n++] = PhiTerm{d, g - 1, u, 1, f, m.lamd[d] * q, q};
      }
    } else {
      if (u + 1 < m.Nu) t[n++] = PhiTerm{d, g, u + 1, 2, f, sqrt(0.5 * (u + 1)), 0.0};
      if (u > 0) t[n++] = PhiTerm{d, g, u - 1, 2, f, sqrt(0.5 * u), 0.0};
    }
  }
  return n;
}

// Adds coef * d(Phi entry)/dp * vec(entry) to G for every parameter p; deps_dw
// are d eps/d w_g and d eps/d w_u of the entry's electron energy.
__device__ inline void phi_param_terms(const DevModel& m, int mu, double eps, int g, int u,
                                       int parity, const c64* vec, c64 coef, double de_g,
                                       double de_u, c64* G) {
  PhiTerm t[6];
  const int n = phi_terms(m, mu, eps, g, u, t);
  for (int q = 0; q < n; ++q) {
    if (((t[q].u + parity) & 1) != t[q].d) continue;   // outside the job's block
    const c64 v = coef * vec[t[q].g * m.Nu + t[q].u];
    const int d = t[q].d;
    const double A = m.A[d][mu], B = m.B[d][mu];
    const double val = t[q].f * t[q].o;
    G[8 + 2 * mu + d] = G[8 + 2 * mu + d] + (val / (2.0 * A)) * v;
    G[12 + 2 * mu + d] = G[12 + 2 * mu + d] + (val * eps / (2.0 * B * B)) * v;
    if (t[q].kind == 1) G[5 + d] = G[5 + d] + (t[q].f * t[q].sfac) * v;
    if (de_g != 0.0 || de_u != 0.0) {
      const double fp = t[q].f * ((m.l[mu] + 0.5) / (2.0 * eps) - 1.0 / (2.0 * B));
      G[0] = G[0] + (fp * de_g * t[q].o) * v;
      G[1] = G[1] + (fp * de_u * t[q].o) * v;
    }
  }
}

// G[idx[q]] -= (workgroup sum of the q-th complex accumulator)
template <int NC>
__device__ inline void subtract_sums(double (&acc)[2 * NC], double* red, c64* G, const int* idx) {
  block_sum<2 * NC, double>(acc, red, red + kWaves * 2 * NC);
  if (threadIdx.x == 0)
    for (int q = 0; q < NC; ++q)
      G[idx[q]] = G[idx[q]] - c64{red[kWaves * 2 * NC + 2 * q], red[kWaves * 2 * NC + 2 * q + 1]};
  __syncthreads();
}

__device__ inline void cacc(double* acc, int q, c64 v) {
  acc[2 * q] += v.x;
  acc[2 * q + 1] += v.y;
}

// Sums over the block of the bilinear forms S_p = zeta^T (dA/dp) psi; G -= S_p.
// A = (E - E_nu - E_d) - k_d q_g - lam q_u - F, so each S_p below carries the
// sign of its term in A; the level-shift part of zeta^T F psi is
// sum_nu [u_A(zeta) F_AA u_A(psi) + u_A(zeta) F_AB u_B(psi) + u_B(zeta) F_AB u_A(psi)
//         + u_B(zeta) F_BB u_B(psi)] = t_AA + t_AB + t_BB, with F_AA ~ A_A,
// F_AB ~ sqrt(A_A A_B), F_BB ~ A_B, and d/dB of the three from the x g
// transform divided by B^2 (diagonal) or 2 B^2 (cross).
__device__ void sweep_dA(const OpJob<double>& op, const DevJob& jb, const DevModel& md,
                         const double* sq, const c64* z, const c64* y, const c64* tab,
                         double* red, c64* G) {
  const int Nc = op.Nc, Nu = op.Nu, Ng = op.Ng;
  const c64* Dt = tab + 3 * (size_t)Nc;   // dF/deps planes
  const c64* Xt = tab + 6 * (size_t)Nc;   // transform of x g
  for (int pass = 0; pass < 3; ++pass) {
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    for (int i = threadIdx.x; i < Nc; i += kBlock) {
      const int ng = i / Nu, nu = i - ng * Nu;
      const int a = (nu + op.p) & 1;
      c64 zg = c64{0, 0}, zu = c64{0, 0}, yg = c64{0, 0}, yu = c64{0, 0};
      if (ng > 0) {
        zg = sq[ng] * z[i - Nu];
        yg = sq[ng] * y[i - Nu];
      }
      if (ng + 1 < Ng) {
        zg = zg + sq[ng + 1] * z[i + Nu];
        yg = yg + sq[ng + 1] * y[i + Nu];
      }
      if (nu > 0) {
        zu = sq[nu] * z[i - 1];
        yu = sq[nu] * y[i - 1];
      }
      if (nu + 1 < Nu) {
        zu = zu + sq[nu + 1] * z[i + 1];
        yu = yu + sq[nu + 1] * y[i + 1];
      }
      const c64 zi = z[i], yi = y[i];
      const double ld = by_state(op.lamd0, op.lamd1, a);
      const c64 uAz = zi + ld * zg, uBz = zu, uAy = yi + ld * yg, uBy = yu;
      if (pass == 0) {
        const c64 FAA = op.AA[i], FAB = op.AB[i];
        const c64 wAz = FAA * uAz + FAB * uBz, wAy = FAA * uAy + FAB * uBy;
        const c64 DAA = Dt[i], DAB = Dt[Nc + i], DBB = Dt[2 * (size_t)Nc + i];
        const c64 dF = uAy * (DAA * uAz + DAB * uBz) + uBy * (DAB * uAz + DBB * uBz);
        const c64 yz = yi * zi;
        const double dg = (double)(jb.vi_g - ng), du = (double)(jb.vi_u - nu);
        cacc(acc, 0, dg * (yz - dF));                       // w_g
        cacc(acc, 1, du * (yz - dF));                       // w_u
        if (a == 1) cacc(acc, 2, -1.0 * yz);                // gap (state 2 diagonal)
        cacc(acc, 3 + a, -1.0 * (yi * zg));                 // k_d
        cacc(acc, 5, -1.0 * (yi * zu));                     // lam
        cacc(acc, 6 + a, -1.0 * (yg * wAz + wAy * zg));     // lam_d
      } else {
        const c64* P = (pass == 1) ? op.AA : Xt;            // F (A terms) or X (B terms)
        const c64 PAA = P[i], PAB = P[Nc + i], PBB = P[2 * (size_t)Nc + i];
        const c64 tAA = uAy * PAA * uAz;
        const c64 tAB = uAy * PAB * uBz + uBy * PAB * uAz;
        const c64 tBB = uBy * PBB * uBz;
        cacc(acc, 3 * a + 0, tAA);
        cacc(acc, 3 * a + 1, tAB);
        cacc(acc, 3 * a + 2, tBB);
      }
    }
    // map the raw sums to parameters; A and B terms are scaled on thread 0
    if (pass == 0) {
      const int idx[8] = {0, 1, 7, 2, 3, 4, 5, 6};
      subtract_sums<8>(acc, red, G, idx);
    } else {
      block_sum<16, double>(acc, red, red + kWaves * 16);
      if (threadIdx.x == 0) {
        const double* r = red + kWaves * 16;
        // a = 0: state 1 active, even wave: AA <-> (1e), BB <-> (2e)
        // a = 1: state 2 active, odd wave:  AA <-> (2o), BB <-> (1o)
        for (int a = 0; a < 2; ++a) {
          const c64 tAA{r[6 * a + 0], r[6 * a + 1]};
          const c64 tAB{r[6 * a + 2], r[6 * a + 3]};
          const c64 tBB{r[6 * a + 4], r[6 * a + 5]};
          const int mu = a;
          const int dA = a, dB = 1 - a;   // the active and the other state
          // dA/dp = -dF/dp here, so G -= S_p adds the F derivatives
          if (pass == 1) {
            const double AA = md.A[dA][mu], AB = md.A[dB][mu];
            G[8 + 2 * mu + dA] = G[8 + 2 * mu + dA] + ((1.0 / AA) * tAA + (0.5 / AA) * tAB);
            G[8 + 2 * mu + dB] = G[8 + 2 * mu + dB] + ((1.0 / AB) * tBB + (0.5 / AB) * tAB);
          } else {
            const double BA = md.B[dA][mu], BB = md.B[dB][mu];
            G[12 + 2 * mu + dA] =
                G[12 + 2 * mu + dA] + ((1.0 / (BA * BA)) * tAA + (0.5 / (BA * BA)) * tAB);
            G[12 + 2 * mu + dB] =
                G[12 + 2 * mu + dB] + ((1.0 / (BB * BB)) * tBB + (0.5 / (BB * BB)) * tAB);
          }
        }
      }
      __syncthreads();
    }
  }
}

template <bool rows>
__global__ void __launch_bounds__(kBlock)
adjoint_kernel(SolveArgs a) {
  __shared__ AdjLds L;
  __shared__ c64 G[kNumParams];
  fill_sq<double>(L.S.sq);
  const int tid = threadIdx.x;
  const Fp64Slot s = fp64_slot(a.scratch + (size_t)blockIdx.x * a.slot_elems, a.ncap, a.m);
  c64* z = s.extra;   // forward solution in the block
  for (;;) {
    __syncthreads();
    if (tid == 0) L.job = atomicAdd(a.counter, 1);
    __syncthreads();
    const int js = L.job;
    if (js >= a.n_jobs) break;
    const DevJob jb = a.jobs[js];
    const DevModel& md = a.models[jb.model];
    const DevTable tb = a.tabs[jb.table];
    const c64* tab = a.tables + tb.offset + (size_t)(jb.parity * a.planes) * md.Nc;
    const OpJob<double> op = make_op<double>(md, jb, tab);
    const int Nc = md.Nc, out = jb.out;
    fp64_prepare<rows>(op, L.S.sq, s, a.precond);
    const c64* psi = a.psi_in + (size_t)out * a.psi_ld;
    for (int i = tid; i < Nc; i += kBlock) {
      const int act = ((i % md.Nu) + jb.parity) & 1;
      z[i] = psi[(size_t)act * Nc + i];
    }
    if (tid < kNumParams) G[tid] = c64{0.0, 0.0};
    __syncthreads();
    // adjoint right-hand side sum_f W_f Phi_f (entries in the block)
    const double c = 2.0 * kPi * kPi * kPi / (jb.eps_i / kHartreeEV);
    if (tid == 0) {
      for (int f = 0; f < a.n_final; ++f) {
        const int g = a.finals[2 * f], u = a.finals[2 * f + 1];
        const double eps_f = jb.E - (md.omega_g * (g + 0.5) + md.omega_u * (u + 0.5));
        for (int mu = 0; mu < 2; ++mu) {
          const c64 T = a.T_in[((size_t)out * a.n_final + f) * 2 + mu];
          const double wr = 2.0 * c * a.dsig[(size_t)out * a.n_final + f];
          const c64 W = c64{wr * T.x, -wr * T.y};
          L.W[2 * f + mu] = W;
          if (g < 0 || g >= md.Ng || u < 0 || u >= md.Nu) continue;
          PhiEntry e[6];
          const int n = phi_entries(md, mu, eps_f, g, u, e);
          for (int q = 0; q < n; ++q)
            if (((e[q].u + jb.parity) & 1) == e[q].d)
              s.b[e[q].g * md.Nu + e[q].u] = s.b[e[q].g * md.Nu + e[q].u] + e[q].val * W;
        }
      }
    }
    __syncthreads();
    const BlockSolve r =
        a.method == VDC_COCG
            ? cocg_fp64_block<rows>(L.S.red, L.dot, L.S.sq, op, s, a.ncap, a.tol, a.max_iter,
                                    a.tileT, a.precond)
            : gmres_fp64_block<rows>(L.S, op, s, a.ncap, a.m, a.tol, a.max_iter, a.tileT,
                                     a.precond);
    __syncthreads();
    // -zeta^T (dA/dp) psi
    sweep_dA(op, jb, md, L.S.sq, z, s.x, tab, L.redA, G);
    // Phi derivative terms (thread 0): zeta^T dPhi_i/dp and sum_f W_f (dPhi_f/dp)^T psi
    if (tid == 0) {
      phi_param_terms(md, jb.mu, jb.eps_i, jb.vi_g, jb.vi_u, jb.parity, s.x, c64{1.0, 0.0}, 0.0,
                      0.0, G);
      for (int f = 0; f < a.n_final; ++f) {
        const int g = a.finals[2 * f], u = a.finals[2 * f + 1];
        if (g < 0 || g >= md.Ng || u < 0 || u >= md.Nu) continue;
        const double eps_f = jb.E - (md.omega_g * (g + 0.5) + md.omega_u * (u + 0.5));
        for (int mu = 0; mu < 2; ++mu)
          phi_param_terms(md, mu, eps_f, g, u, jb.parity, z, L.W[2 * f + mu],
                          (double)(jb.vi_g - g), (double)(jb.vi_u - u), G);
      }
      for (int p = 0; p < kNumParams; ++p) a.grad[(size_t)out * kNumParams + p] = G[p].x;
      // byte model: solve as in the forward solver, plus psi gathered (2 passes)
      // and three sweeps reading psi, zeta and 3 table planes (15 passes)
      a.info[out] = DevInfo{r.status, r.iters, r.cycles, 0,
                            r.bnorm > 0.0 ? r.beta / r.bnorm : 0.0,
                            (r.passes + 2.0 + 15.0) * 16.0 * Nc};
    }
  }
}

hipError_t launch_adjoint(const SolveArgs& a, int n_groups, size_t dyn_lds, hipStream_t s) {
  if (a.precond == VDC_PREC_ROWS)
    hipLaunchKernelGGL(adjoint_kernel<true>, dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  else
    hipLaunchKernelGGL(adjoint_kernel<false>, dim3(n_groups), dim3(kBlock), dyn_lds, s, a);
  return hipGetLastError();
}

int adjoint_occupancy(size_t dyn_lds) {
  return std::min(occupancy_of(adjoint_kernel<true>, dyn_lds),
                  occupancy_of(adjoint_kernel<false>, dyn_lds));
}

}  // namespace vdc
