// Kernels of the CO2-like model (co2.h): the persistent batched GMRES with
// the bend-plane block preconditioner (Sec. III.B; the block choice the paper
// makes for its CO2 model in Sec. III.C), and the operator and preconditioner
// applied to given vectors.
#include "co2.h"
#include "krylov.h"
#include "strip.h"

namespace vdc {

// LDS of the block factorisation: a ring of w + 1 band columns.
extern __shared__ __align__(16) char vdc_co2_lds[];

__device__ inline double co2_apply(const Co2Op& o, const double* sq, const c64* v, double vs,
                                   c64* y, c64* wA, c64* wB, const c64* bsub, double* red) {
  const int n = o.m->npts;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    c64 a, b;
    co2_phase1(o, sq, v, vs, i, a, b);
    wA[i] = a;
    wB[i] = b;
  }
  __syncthreads();
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += kBlock) {
    c64 r = co2_phase2(o, sq, v, vs, wA, wB, i);
    if (bsub) r = bsub[i] - r;
    y[i] = r;
    acc[0] += norm2(r);
  }
  if (!red) {
    __syncthreads();
    return 0.0;
  }
  block_sum<1, double>(acc, red, red + kWaves);
  const double s = red[kWaves];
  __syncthreads();
  return s;
}

// Block element A(r, c) of plane (s, a) in the plane's point order j = x Ny + y;
// rows and columns of points without a state are those of the identity.
__device__ inline c64 co2_plane_entry(const Co2Op& o, const double* sq, int s, int a, int r, int c) {
  const Co2Model& m = *o.m;
  const int xr = r / m.Ny, yr = r - xr * m.Ny, xc = c / m.Ny, yc = c - xc * m.Ny;
  if (co2_type(xr, yr, o.px, o.py) == 3 || co2_type(xc, yc, o.px, o.py) == 3)
    return c64{r == c ? 1.0 : 0.0, 0.0};
  const int dx = xc - xr, dy = yc - yr;
  if (dx < -2 || dx > 2 || dy < -2 || dy > 2) return c64{0.0, 0.0};
  return co2_band_entry(o, sq, s, a, xr, yr, dx, dy);
}

// Factor every plane block into fac ([plane][j][w + 1]: 1/D_j, then
// L(j + k, j) for k = 1..w), w = 2 Ny the half bandwidth.
//   1. The band of every block, A(c + k, c), is written into fac by all
//      threads at once (only the in-plane neighbour offsets can be nonzero).
//   2. Each plane is eliminated right-looking on a ring of w + 1 + kCo2Cols
//      columns in LDS (column c holds A(c + k, c), k = 0..w, as updated so
//      far); the band columns are fetched kCo2Cols at a time, and the factor
//      rows are staged in LDS and written back kCo2Cols at a time (over band
//      columns already in the ring), so memory waits at one barrier in
//      kCo2Cols rather than at every pivot.
// A plane whose pivot falls below 1e-14 of its diagonal entry is replaced by
// its diagonal.  Barriers inside.
constexpr int kCo2Cols = 16;

size_t co2_factor_lds_bytes(int Ny) {
  const size_t W1 = 2 * (size_t)Ny + 1, R = W1 + kCo2Cols;
  return (R * W1 + W1 + R + (size_t)kCo2Cols * W1) * sizeof(c64);
}

__device__ inline void co2_factor_planes(const Co2Op& o, const double* sq, c64* fac, int* flag) {
  const Co2Model& m = *o.m;
  const int n = m.Nx * m.Ny, w = 2 * m.Ny, W1 = w + 1, R = W1 + kCo2Cols;
  const int planes = m.Ns * m.Na;
  c64* ring = reinterpret_cast<c64*>(vdc_co2_lds);   // [R][W1]
  c64* lrow = ring + R * W1;                           // [W1]
  c64* diag0 = lrow + W1;                              // [R] original diagonal per slot
  c64* fbuf = diag0 + R;                               // [kCo2Cols][W1] factor rows
  const int tid = threadIdx.x;
  __syncthreads();
  for (size_t q = tid; q < (size_t)planes * n * W1; q += kBlock) {
    const int k = (int)(q % W1);
    const size_t cq = q / W1;
    const int c = (int)(cq % n), P = (int)(cq / n);
    const int r = c + k;
    c64 v = c64{0.0, 0.0};
    if (r < n) {
      const int xr = r / m.Ny, xc = c / m.Ny;
      const int dx = xc - xr, dy = (c - xc * m.Ny) - (r - xr * m.Ny);
      if (dx >= -2 && dy >= -2 && dy <= 2) v = co2_plane_entry(o, sq, P / m.Na, P % m.Na, r, c);
    }
    fac[q] = v;
  }
  __syncthreads();
  // this thread's share of the rank-one update: the pairs (column offset
  // co, row offset k), co = 1..w, k = 0..w - co, of q = tid + u kBlock; the
  // same for every pivot (w W1 <= 62 * 63 < kUpd kBlock for Ny <= 31)
  constexpr int kUpd = 4;
  int uco[kUpd], uk[kUpd];
#pragma unroll
  for (int u = 0; u < kUpd; ++u) {
    const int q = tid + u * kBlock;
    const int co = q / W1 + 1, k = q - (co - 1) * W1;
    const bool ok = q < w * W1 && k <= w - co;
    uco[u] = ok ? co : 0;
    uk[u] = k;
  }
  for (int P = 0; P < planes; ++P) {
    c64* F = fac + (size_t)P * n * W1;
    if (tid == 0) *flag = 1;
    // columns 0 .. R-1 into the ring
    for (int q = tid; q < R * W1; q += kBlock) {
      const int c = q / W1;
      ring[q] = c < n ? F[q] : c64{0.0, 0.0};
      if (q % W1 == 0) diag0[c] = ring[q];
    }
    __syncthreads();
    int sl = 0;                           // ring slot of the pivot column, j % R
    for (int j = 0; j < n; ++j) {
      const c64 D = ring[sl * W1];
      const c64 Di = cinv<double>(D);
      const int jb = j % kCo2Cols;
      if (tid <= w) {
        const c64 L = tid == 0 ? Di : ring[sl * W1 + tid] * Di;
        lrow[tid] = L;
        fbuf[jb * W1 + tid] = L;
      }
      if (tid == 0) {
        const double nd = sqrt(norm2(D));
        if (!(isfinite(nd) && nd > 1e-14 * sqrt(norm2(diag0[sl])))) *flag = 0;
      }
      __syncthreads();
      // A(c + k, c) -= L(c, j) D L(c + k, j) for the next w columns
#pragma unroll
      for (int u = 0; u < kUpd; ++u) {
        if (uco[u] == 0) continue;
        int slot = sl + uco[u];
        if (slot >= R) slot -= R;
        c64* e = ring + slot * W1 + uk[u];
        *e = *e - (lrow[uco[u]] * D) * lrow[uco[u] + uk[u]];
      }
      // every kCo2Cols pivots (and at the end): the staged factor rows out,
      // and the next kCo2Cols band columns into the slots of the columns just
      // eliminated
      if (jb == kCo2Cols - 1 || j + 1 == n) {
        const int j0 = j - jb;
        for (int q = tid; q < (j + 1 - j0) * W1; q += kBlock)
          F[(size_t)j0 * W1 + q] = fbuf[q];
        if (jb == kCo2Cols - 1) {
          for (int q = tid; q < kCo2Cols * W1; q += kBlock) {
            const int c = j + 1 - kCo2Cols + R + q / W1, k = q % W1;
            const int slot = c % R;
            const c64 v = c < n ? F[(size_t)c * W1 + k] : c64{0.0, 0.0};
            ring[slot * W1 + k] = v;
            if (k == 0) diag0[slot] = v;
          }
        }
      }
      __syncthreads();
      if (++sl == R) sl = 0;
    }
    if (!*flag) {
      for (int j = tid; j < n; j += kBlock) {
        F[(size_t)j * W1] = cinv<double>(co2_plane_entry(o, sq, P / m.Na, P % m.Na, j, j));
        for (int k = 1; k <= w; ++k) F[(size_t)j * W1 + k] = c64{0.0, 0.0};
      }
    }
    __syncthreads();
  }
}

__device__ inline c64 lane0(c64 v) {
  return c64{__shfl(v.x, 0), __shfl(v.y, 0)};
}

__device__ inline c64 wave_sum(c64 v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  return v;
}

constexpr int kCo2Chunk = 4;   // factor rows loaded ahead per wavefront

// z = M^{-1} (vs v) (z may be v): one wavefront per plane, forward L, D^{-1},
// backward L^T; lane k holds the running value of row j + k.  Begins and ends
// with a barrier.
__device__ inline void co2_block_apply(const Co2Model& m, const c64* fac, const c64* v, double vs,
                                       c64* z) {
  __syncthreads();
  const int n = m.Nx * m.Ny, w = 2 * m.Ny, W1 = w + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool band = lane >= 1 && lane <= w;
  for (int P = wave; P < m.Ns * m.Na; P += kWaves) {
    const c64* F = fac + (size_t)P * n * W1;
    const c64* vp = v + (size_t)P * n;
    c64* zp = z + (size_t)P * n;
    c64 acc = (lane <= w && lane < n) ? vs * vp[lane] : c64{0.0, 0.0};
    for (int j0 = 0; j0 < n; j0 += kCo2Chunk) {
      c64 Lr[kCo2Chunk];
#pragma unroll
      for (int q = 0; q < kCo2Chunk; ++q)
        Lr[q] = (band && j0 + q < n) ? F[(size_t)(j0 + q) * W1 + lane] : c64{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < kCo2Chunk; ++q) {
        const int j = j0 + q;
        if (j >= n) break;
        const c64 yj = lane0(acc);
        if (lane == 0) zp[j] = yj;
        acc = acc - Lr[q] * yj;
        acc = lane_next(acc);
        if (lane == w) acc = (j + 1 + w < n) ? vs * vp[j + 1 + w] : c64{0.0, 0.0};
      }
    }
    c64 zw = c64{0.0, 0.0};
    for (int j1 = n - 1; j1 >= 0; j1 -= kCo2Chunk) {
      // lane 0 holds D^{-1}_j y_j, lanes 1..w the row of L^T
      c64 Lr[kCo2Chunk];
#pragma unroll
      for (int q = 0; q < kCo2Chunk; ++q) {
        const int j = j1 - q;
        Lr[q] = c64{0.0, 0.0};
        if (j >= 0 && lane <= w) Lr[q] = F[(size_t)j * W1 + lane];
        if (j >= 0 && lane == 0) Lr[q] = Lr[q] * zp[j];
      }
#pragma unroll
      for (int q = 0; q < kCo2Chunk; ++q) {
        const int j = j1 - q;
        if (j < 0) break;
        const c64 dot = wave_sum(band ? Lr[q] * zw : c64{0.0, 0.0});
        const c64 zj = lane0(Lr[q]) - dot;
        if (lane == 0) zp[j] = zj;
        zw = lane_prev(zw);
        if (lane == 1) zw = zj;
      }
    }
  }
  __syncthreads();
}

// Jacobi: dinv = 1 / diag(A) at points with a state, 0 elsewhere.
__device__ inline void co2_jacobi(const Co2Op& o, const double* sq, c64* dinv) {
  const Co2Model& m = *o.m;
  for (int i = threadIdx.x; i < m.npts; i += kBlock) {
    const Co2Point p = co2_point(m, i);
    dinv[i] = co2_type(p.x, p.y, o.px, o.py) == 3
                  ? c64{0.0, 0.0}
                  : cinv<double>(co2_band_entry(o, sq, p.s, p.a, p.x, p.y, 0, 0));
  }
}

// Nonzero entries of Phi^{v mu} in the sector (px, py): f_d^mu(eps) O_d^mu |v>
// (Eq. (25)); at most 7 entries (index into the sector vector, value).
struct Co2PhiEntry { int i; double val; };

__device__ inline int co2_phi_entries(const Co2Model& m, const DevModel& ls, const int* v, int mu,
                                      double eps, int px, int py, Co2PhiEntry* e) {
  int n = 0;
  auto idx = [&](int s, int x, int y, int a) { return ((s * m.Na + a) * m.Nx + x) * m.Ny + y; };
  auto add = [&](int d, int s, int x, int y, int a, double val) {
    if (s < 0 || s >= m.Ns || x < 0 || x >= m.Nx || y < 0 || y >= m.Ny || a < 0 || a >= m.Na) return;
    if (co2_type(x, y, px, py) != d || val == 0.0) return;
    e[n++] = Co2PhiEntry{idx(s, x, y, a), val};
  };
  const int s = v[0], x = v[1], y = v[2], a = v[3];
  const int w = mu == 0 ? 0 : 1;
  for (int d = 0; d < 3; ++d) {
    const double f = coupling_f(ls, d == 0 ? 0 : 1, w, eps);
    if (f == 0.0) continue;
    const bool gs = (mu == 0 && d == 0) || (mu == 1 && d == 1) || (mu == 2 && d == 2);
    if (gs) {   // (1 + l q_s)
      const double l = d == 0 ? m.l_sigma : m.l_pi;
      add(d, s, x, y, a, f);
      add(d, s + 1, x, y, a, f * l * sqrt(0.5 * (s + 1)));
      add(d, s - 1, x, y, a, f * l * sqrt(0.5 * s));
    } else if ((mu == 0 && d == 1) || (mu == 1 && d == 0)) {   // h q_x
      const double h = d == 0 ? m.h_sigma : m.h_pi;
      add(d, s, x + 1, y, a, f * h * sqrt(0.5 * (x + 1)));
      add(d, s, x - 1, y, a, f * h * sqrt(0.5 * x));
    } else if ((mu == 0 && d == 2) || (mu == 2 && d == 0)) {   // h q_y
      const double h = d == 0 ? m.h_sigma : m.h_pi;
      add(d, s, x, y + 1, a, f * h * sqrt(0.5 * (y + 1)));
      add(d, s, x, y - 1, a, f * h * sqrt(0.5 * y));
    }
  }
  return n;
}



struct Co2Lds {
  KrylovLds<double> K;
  double red[kRedSize];
  double sq[kSqMax + 1];
  int job, flag;
};

// Byte model (passes over a sector vector of npts complex FP64 values, W1 =
// 2 Ny + 1 factor entries per point): setup: x, b written, b read, V_0
// copied (5), plus the factor written (W1) or dinv written (1); Arnoldi step:
// M^{-1} (vector and factor read, zt written: W1 + 2) or the diagonal (v,
// dinv read, zt written: 3), then the operator (zt read twice, w_A, w_B
// written and read, y written: 7), and the projection passes of
// cycle_passes (which counts 6 for an operator of its own); cycle end with k
// steps: the update (basis k and x in/out, with M^{-1}: zt written and read
// back, W1 + 2 for M^{-1}: k + W1 + 6; with the diagonal: k + 3) and the true
// residual (x twice, w_A, w_B twice, b, residual out: 8).
__global__ void __launch_bounds__(kBlock) co2_gmres_kernel(Co2Args a) {
  __shared__ Co2Lds L;
  fill_sq<double>(L.sq);
  const Co2Model& md = *a.model;
  const int tid = threadIdx.x;
  const int npts = md.npts;
  const size_t ld = a.ld;
  const int m = a.m;
  c64* slot = a.scratch + (size_t)blockIdx.x * a.slot_elems;
  c64* V = slot;
  c64* x = V + (size_t)(m + 1) * ld;
  c64* b = x + ld;
  c64* zt = b + ld;
  c64* wA = zt + ld;
  c64* wB = wA + ld;
  c64* dinv = wB + ld;
  c64* Rm = dinv + ld;
  c64* fac = slot + a.fac_off;
  const bool blk = a.precond == VDC_PREC_BLOCK;
  const double W1 = 2.0 * md.Ny + 1.0;
  for (;;) {
    __syncthreads();
    if (tid == 0) L.job = atomicAdd(a.counter, 1);
    __syncthreads();
    const int js = L.job;
    if (js >= a.n_jobs) break;
    const Co2Job jb = a.jobs[js];
    const Co2Op op{a.model, a.tables + (size_t)jb.table * md.ntab * kNumF, jb.E, jb.px, jb.py};
    double passes = 5.0;
    if (blk) {
      co2_factor_planes(op, L.sq, fac, &L.flag);
      passes += W1;
    } else if (a.precond == VDC_PREC_JACOBI) {
      co2_jacobi(op, L.sq, dinv);
      passes += 1.0;
    }
    for (int i = tid; i < npts; i += kBlock) {
      x[i] = c64{0.0, 0.0};
      b[i] = c64{0.0, 0.0};
    }
    __syncthreads();
    if (tid == 0) {
      Co2PhiEntry e[8];
      const int ne = co2_phi_entries(md, *a.ls, jb.v, jb.mu, jb.eps_i, jb.px, jb.py, e);
      for (int q = 0; q < ne; ++q) b[e[q].i] = b[e[q].i] + c64{e[q].val, 0.0};
    }
    __syncthreads();
    const double bnorm = sqrt(norm_sq<double>(b, npts, L.red));
    double beta = bnorm;
    int iters = 0, cycles = 0, status = VDC_NOT_CONVERGED;
    if (!(bnorm > 0.0) || !isfinite(bnorm)) {
      status = isfinite(bnorm) ? VDC_CONVERGED : VDC_NONFINITE;
      beta = 0.0;
    } else {
      for (int i = tid; i < npts; i += kBlock) V[i] = b[i];
      auto apply = [&](int j, double sc, c64* out) {
        const c64* vj = V + (size_t)j * ld;
        if (blk) {
          co2_block_apply(md, fac, vj, sc, zt);
        } else {
          for (int i = tid; i < npts; i += kBlock)
            zt[i] = a.precond == VDC_PREC_JACOBI ? sc * (dinv[i] * vj[i]) : sc * vj[i];
        }
        co2_apply(op, L.sq, zt, 1.0, out, wA, wB);
      };
      for (;;) {
        if (tid == 0) {
          L.K.g[0] = c64{beta, 0.0};
          L.K.vs[0] = 1.0 / beta;
        }
        __syncthreads();
        const CycleResult cr = krylov_cycle<double>(L.K, L.red, V, ld, npts, m, a.tol * bnorm,
                                                    a.max_iter, iters, Rm, apply);
        passes += cycle_passes(cr.k, cr.reorth_passes) + cr.k * ((blk ? W1 + 2.0 : 3.0) + 1.0) +
                  (blk ? cr.k + W1 + 6.0 : cr.k + 3.0) + 8.0;
        if (blk) {
          update_x<double>(V, ld, cr.k, L.K.y, L.K.vs, nullptr, zt, npts, true);
          co2_block_apply(md, fac, zt, 1.0, zt);
          for (int i = tid; i < npts; i += kBlock) x[i] = x[i] + zt[i];
        } else {
          update_x<double>(V, ld, cr.k, L.K.y, L.K.vs,
                           a.precond == VDC_PREC_JACOBI ? dinv : nullptr, x, npts);
        }
        beta = sqrt(co2_apply(op, L.sq, x, 1.0, V, wA, wB, b, L.red));
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
        if (iters >= a.max_iter) {
          status = VDC_NOT_CONVERGED;
          break;
        }
      }
    }
    __syncthreads();
    // amplitudes T = Phi_f^T psi for each final state and partial wave, and
    // the job's share of sigma (Eqs. (15), (16))
    const int out = jb.out;
    const double c = 2.0 * kPi * kPi * kPi / (jb.eps_i / kHartreeEV);
    for (int q = tid; q < a.n_final * 3; q += kBlock) {
      const int f = q / 3, mu = q - 3 * f;
      const int* vf = a.finals + 4 * f;
      const double Ef = md.omega_s * (vf[0] + 0.5) + md.omega_b * (vf[1] + vf[2] + 1.0) +
                        md.omega_a * (vf[3] + 0.5);
      Co2PhiEntry e[8];
      const int ne = co2_phi_entries(md, *a.ls, vf, mu, jb.E - Ef, jb.px, jb.py, e);
      c64 T = c64{0.0, 0.0};
      for (int r = 0; r < ne; ++r) T = T + e[r].val * x[e[r].i];
      a.T_out[((size_t)out * a.n_final + f) * 3 + mu] = T;
    }
    __syncthreads();
    for (int f = tid; f < a.n_final; f += kBlock) {
      double s2 = 0.0;
      for (int mu = 0; mu < 3; ++mu) s2 += norm2(a.T_out[((size_t)out * a.n_final + f) * 3 + mu]);
      a.sigma_out[(size_t)out * a.n_final + f] = c * s2;
    }
    if (a.psi_out)
      for (int i = tid; i < npts; i += kBlock) a.psi_out[(size_t)out * npts + i] = x[i];
    if (tid == 0)
      a.info[out] = DevInfo{status, iters, cycles, 0, bnorm > 0.0 ? beta / bnorm : 0.0,
                            passes * 16.0 * npts};
  }
}

// y = A x or y = M^{-1} x for given sector vectors (one workgroup per vector).

__global__ void __launch_bounds__(kBlock) co2_ops_kernel(Co2OpsArgs a) {
  __shared__ double sq[kSqMax + 1];
  __shared__ int flag;
  fill_sq<double>(sq);
  const Co2Model& md = *a.model;
  c64* slot = a.scratch + (size_t)blockIdx.x * a.slot_elems;
  for (int v = blockIdx.x; v < a.n_vec; v += gridDim.x) {
    const Co2Op op{a.model, a.tab, a.E, a.sectors[2 * v], a.sectors[2 * v + 1]};
    const c64* xv = a.x + (size_t)v * md.npts;
    c64* yv = a.y + (size_t)v * md.npts;
    if (a.which == 0) {
      co2_apply(op, sq, xv, 1.0, yv, slot, slot + md.npts);
    } else {
      co2_factor_planes(op, sq, slot, &flag);
      co2_block_apply(md, slot, xv, 1.0, yv);
    }
  }
}

size_t co2_factor_lds(int Ny) { return co2_factor_lds_bytes(Ny); }

hipError_t launch_co2_gmres(const Co2Args& a, int n_groups, size_t dyn, hipStream_t s) {
  hipLaunchKernelGGL(co2_gmres_kernel, dim3(n_groups), dim3(kBlock), dyn, s, a);
  return hipGetLastError();
}

hipError_t launch_co2_ops(const Co2OpsArgs& a, int n_groups, size_t dyn, hipStream_t s) {
  hipLaunchKernelGGL(co2_ops_kernel, dim3(n_groups), dim3(kBlock), dyn, s, a);
  return hipGetLastError();
}

}  // namespace vdc
