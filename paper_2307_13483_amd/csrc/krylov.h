// One restarted-GMRES cycle run by a whole workgroup (Sec. III.A): Arnoldi
// with classical Gram-Schmidt applied twice, a one-thread Givens update of
// each Hessenberg column, and the back substitution R y = g at the end.
// Generic in the precision R of the basis vectors and their dot products; the
// small Hessenberg least-squares problem is always FP64.
#pragma once
#include "blockops.h"

namespace vdc {

template <typename R>
struct KrylovLds {
  double cs[kMaxRestart];
  c64 sn[kMaxRestart];
  c64 g[kMaxRestart + 1];
  c64 y[kMaxRestart];
  R h1[2 * (kMaxRestart + 1)];   // projection coefficients onto the unit basis
  R h2[2 * (kMaxRestart + 1)];
  R hs[2 * (kMaxRestart + 1)];   // the same times the stored vectors' scales
  R vs[kMaxRestart + 1];         // basis vector l is vs[l] * V_l (lazy normalisation)
  c64 hc[kMaxRestart + 1];
  double resid;
  R wnorm2;
};

__device__ inline c64 cdiv(c64 a, c64 b) {
  const double n = b.x * b.x + b.y * b.y;
  return c64{(a.x * b.x + a.y * b.y) / n, (a.y * b.x - a.x * b.y) / n};
}

// Thread-0 Givens update of Hessenberg column j: apply the previous
// rotations, build rotation j from (h_jj, h_{j+1,j}), store the R column and
// update the right-hand side g.  Returns |g_{j+1}| (the residual norm of the
// least-squares problem).
template <typename R>
__device__ inline double givens_step(KrylovLds<R>& L, int j, double hnext, c64* Rcol) {
  c64* col = L.hc;
  for (int i = 0; i <= j; ++i)
    col[i] = c64{(double)L.h1[2 * i] + (double)L.h2[2 * i],
                 (double)L.h1[2 * i + 1] + (double)L.h2[2 * i + 1]};
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
    s = c64{a.x / aa * hnext / den, a.y / aa * hnext / den};  // (a/|a|) conj(h)/den, h real
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
template <typename R>
__device__ inline void back_substitute(KrylovLds<R>& L, int k, const c64* Rm, int ldr) {
  for (int i = k - 1; i >= 0; --i) {
    c64 s = L.g[i];
    for (int l = i + 1; l < k; ++l) s = s - Rm[(size_t)l * ldr + i] * L.y[l];
    L.y[i] = cdiv(s, Rm[(size_t)i * ldr + i]);
  }
}

// Vector passes of one Arnoldi cycle of k steps by design: per step j the
// operator reads v_j, the Jacobi scaling and three level-shift planes and
// writes w into the basis slot j+1 (5 + 1 = 6, orthogonalised in place, so
// no separate normalisation pass); classical Gram-Schmidt reads the basis
// twice (2 (j+1)), twice more when repeated (reorth_passes, the sum of
// 2 (j+1) over the repeated steps).
__host__ __device__ inline double cycle_passes(int k, double reorth_passes) {
  return 6.0 * k + 1.0 * k * (k + 1.0) + reorth_passes;
}

struct CycleResult {
  int k;           // Arnoldi steps taken
  bool breakdown;  // h_{k,k-1} == 0 (Krylov space exhausted)
  bool nonfinite;
  double reorth_passes;   // basis passes of the repeated Gram-Schmidt steps
  int reorth;             // number of repeated steps
};

// Selective reorthogonalisation (after Daniel, Gragg, Kaufman & Stewart
// 1976): classical Gram-Schmidt loses orthogonality in proportion to
// ||w|| / ||w'||, so the second pass runs only when the first removed more
// than 1 - eta^2 of ||w||^2.  With eta = 0.1 the loss per step stays below
// ~10 ulp; on these operators ||w'||/||w|| is 0.2-0.9 in almost all steps and
// iteration counts are unchanged.  ||w'|| is always computed from the vector
// itself (fused into the update pass): the Pythagorean shortcut
// ||w||^2 - sum |h|^2 makes the GMRES residual estimate stall near 1e-8.
constexpr double kReorthEta2 = 0.01;

// h (coefficients on the unit basis) = raw projections on the stored
// vectors times their scales; hs = h times the scales again (the
// coefficients of the stored vectors in the update).  Threads < 2 nv.
template <typename R>
__device__ inline void scale_coeffs(R* h, R* hs, const R* vs, int nv) {
  if (threadIdx.x < 2 * nv) {
    const R s = vs[threadIdx.x >> 1];
    h[threadIdx.x] *= s;
    hs[threadIdx.x] = h[threadIdx.x] * s;
  }
  __syncthreads();
}

// Runs up to m Arnoldi steps.  On entry the stored vector V_0 and its scale
// L.vs[0] (V_0 * vs[0] has unit norm) and L.g[0] = beta are set (by thread 0
// for the LDS values, followed by a barrier).  apply(j, s, out) must write
// the preconditioned operator applied to s * V_j into out = V_{j+1} and end
// with a barrier.  Stops when the least-squares residual drops to tol_abs or
// iters reaches max_iter.  On return L.y holds the least-squares
// coefficients on the unit basis (after a barrier).
// With hist, thread 0 writes the least-squares residual times hscale after
// every step to hist[iters - 1] while iters <= hist_len.
template <typename R, typename Apply>
__device__ inline CycleResult krylov_cycle(KrylovLds<R>& L, R* red, typename CT<R>::C* V,
                                           size_t ld, int Nc, int m, double tol_abs,
                                           int max_iter, int& iters, c64* Rm, Apply apply,
                                           double* hist = nullptr, int hist_len = 0,
                                           double hscale = 0.0) {
  using C = typename CT<R>::C;
  CycleResult res{0, false, false, 0.0, 0};
  for (int j = 0; j < m; ++j) {
    C* w = V + (size_t)(j + 1) * ld;
    apply(j, L.vs[j], w);
    project<R>(V, ld, j + 1, w, Nc, red, L.h1, &L.wnorm2);
    scale_coeffs<R>(L.h1, L.hs, L.vs, j + 1);
    const double rest = (double)subtract<R>(V, ld, j + 1, w, Nc, L.hs, red);
    // every thread takes the same decision from the same reduced values
    const double wn2 = (double)L.wnorm2;
    double hn;
    if (rest >= kReorthEta2 * wn2) {
      hn = sqrt(rest);
      if (threadIdx.x < 2 * (j + 1)) L.h2[threadIdx.x] = R(0);
      __syncthreads();
    } else {
      project<R>(V, ld, j + 1, w, Nc, red, L.h2);
      scale_coeffs<R>(L.h2, L.hs, L.vs, j + 1);
      hn = sqrt((double)subtract<R>(V, ld, j + 1, w, Nc, L.hs, red));
      res.reorth_passes += 2.0 * (j + 1);
      res.reorth += 1;
    }
    if (threadIdx.x == 0) {
      L.resid = givens_step<R>(L, j, hn, Rm + (size_t)j * (m + 1));
      L.vs[j + 1] = R(hn > 0.0 ? 1.0 / hn : 0.0);
    }
    __syncthreads();
    const double r = L.resid;
    ++iters;
    if (hist && threadIdx.x == 0 && iters <= hist_len) hist[iters - 1] = r * hscale;
    res.k = j + 1;
    if (!isfinite(r) || !isfinite(hn)) {
      res.nonfinite = true;
      break;
    }
    if (hn == 0.0) {
      res.breakdown = true;
      break;
    }
    if (r <= tol_abs || iters >= max_iter) break;
  }
  if (threadIdx.x == 0) back_substitute<R>(L, res.k, Rm, m + 1);
  __syncthreads();
  return res;
}

// x += dinv * sum_l (vs[l] V_l) y_l (own elements; dinv, vs may be null), y from
// L.y (FP64), in precision R: reads the k basis vectors, dinv and x once.
// With assign, x = dinv * sum ... instead (x not read).
template <typename R>
__device__ inline void update_x(const typename CT<R>::C* V, size_t ld, int k, const c64* y,
                                const R* vs, const typename CT<R>::C* dinv,
                                typename CT<R>::C* x, int Nc, bool assign = false) {
  using C = typename CT<R>::C;
  for (int i = threadIdx.x; i < Nc; i += kBlock) {
    C s = cz<R>();
    int l = 0;
    for (; l + kChunk <= k; l += kChunk) {
      C vv[kChunk];
#pragma unroll
      for (int q = 0; q < kChunk; ++q) vv[q] = V[(size_t)(l + q) * ld + i];
#pragma unroll
      for (int q = 0; q < kChunk; ++q)
        s = s + vv[q] * C{R(y[l + q].x) * (vs ? vs[l + q] : R(1)),
                          R(y[l + q].y) * (vs ? vs[l + q] : R(1))};
    }
    for (; l < k; ++l)
      s = s + V[(size_t)l * ld + i] * C{R(y[l].x) * (vs ? vs[l] : R(1)),
                                        R(y[l].y) * (vs ? vs[l] : R(1))};
    const C t = dinv ? dinv[i] * s : s;
    x[i] = assign ? t : x[i] + t;
  }
}

}  // namespace vdc
