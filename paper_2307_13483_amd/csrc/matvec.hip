// Grid-wide application of A = E - H_ef(E) (Eq. (28)) to a batch of
// full-layout vectors, one symmetry block each: gather the block, the two
// stencil phases of op2d.h as separate grid-wide passes, scatter back.
#include "op2d.h"
#include "strip.h"

namespace vdc {

__global__ void zero_int_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t launch_zero_int(int* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(zero_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
gather_block_kernel(const DevModel* __restrict__ md, const int* __restrict__ par, int n_vec,
                    const c64* __restrict__ x, c64* __restrict__ z) {
  const int Nc = md->Nc, Nu = md->Nu;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (i >= Nc || v >= n_vec) return;
  const int act = ((i % Nu) + par[v]) & 1;
  z[(size_t)v * Nc + i] = x[(size_t)v * 2 * Nc + (size_t)act * Nc + i];
}

__global__ void __launch_bounds__(256)
scatter_block_kernel(const DevModel* __restrict__ md, const int* __restrict__ par, int n_vec,
                     const c64* __restrict__ yc, c64* __restrict__ y) {
  const int Nc = md->Nc, Nu = md->Nu;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (i >= Nc || v >= n_vec) return;
  const int act = ((i % Nu) + par[v]) & 1;
  y[(size_t)v * 2 * Nc + (size_t)act * Nc + i] = yc[(size_t)v * Nc + i];
  y[(size_t)v * 2 * Nc + (size_t)(1 - act) * Nc + i] = c64{0.0, 0.0};
}

__global__ void __launch_bounds__(256)
matvec_phase1_kernel(const DevModel* __restrict__ md, const DevTable* __restrict__ tab,
                     const c64* __restrict__ tables, const int* __restrict__ par, int n_vec,
                     const c64* __restrict__ z, c64* __restrict__ yc, c64* __restrict__ wA,
                     c64* __restrict__ wB) {
  __shared__ double sq[kSqMax + 1];
  fill_sq<double>(sq);
  __syncthreads();
  const DevModel& m = *md;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (i >= m.Nc || v >= n_vec) return;
  DevJob jb{};
  jb.E = tab->E;
  jb.parity = par[v];
  const OpJob<double> op =
      make_op<double>(m, jb, tables + tab->offset + (size_t)(jb.parity * 3) * m.Nc);
  const size_t o = (size_t)v * m.Nc;
  c64 y, a, b;
  op_phase1<double>(op, sq, z + o, nullptr, i, y, a, b);
  yc[o + i] = y;
  wA[o + i] = a;
  wB[o + i] = b;
}

__global__ void __launch_bounds__(256)
matvec_phase2_kernel(const DevModel* __restrict__ md, const DevTable* __restrict__ tab,
                     const c64* __restrict__ tables, const int* __restrict__ par, int n_vec,
                     c64* __restrict__ yc, const c64* __restrict__ wA,
                     const c64* __restrict__ wB) {
  __shared__ double sq[kSqMax + 1];
  fill_sq<double>(sq);
  __syncthreads();
  const DevModel& m = *md;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (i >= m.Nc || v >= n_vec) return;
  DevJob jb{};
  jb.E = tab->E;
  jb.parity = par[v];
  const OpJob<double> op =
      make_op<double>(m, jb, tables + tab->offset + (size_t)(jb.parity * 3) * m.Nc);
  const size_t o = (size_t)v * m.Nc;
  yc[o + i] = op_phase2<double>(op, sq, wA + o, wB + o, i, yc[o + i]);
}

// Batched operator on block vectors (n_g-major, n_u contiguous), all at one
// total energy.  One wavefront per (vector, row slab, column strip), four
// wavefronts per workgroup; after the sqrt table is in LDS the sweep of
// strip.h needs no barrier, so a wavefront past the end simply returns.
__global__ void __launch_bounds__(256, 4)
matvec_strip_kernel(const DevModel* __restrict__ md, const DevTable* __restrict__ tab,
                    const c64* __restrict__ tables, const int* __restrict__ par, int n_vec,
                    const c64* __restrict__ x, c64* __restrict__ y, int S, int n_slabs,
                    int n_strips) {
  __shared__ double sq[kSqMax + 1];
  fill_sq<double>(sq);
  __syncthreads();
  const long task = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const long per_vec = (long)n_slabs * n_strips;
  if (task >= (long)n_vec * per_vec) return;
  const int v = (int)(task / per_vec);
  const int rem = (int)(task - (long)v * per_vec);
  const int slab = rem / n_strips, strip = rem - slab * n_strips;
  const DevModel& m = *md;
  DevJob jb{};
  jb.E = tab->E;
  jb.parity = par[v];
  const OpJob<double> op =
      make_op<double>(m, jb, tables + tab->offset + (size_t)(jb.parity * 3) * m.Nc);
  const size_t o = (size_t)v * m.Nc;
  const int g0 = slab * S, g1 = min(m.Ng, g0 + S);
  strip_sweep<double>(op, sq, x + o, 1.0, nullptr, y + o, nullptr, strip, g0, g1);
}

hipError_t launch_matvec_strip(const DevModel* md, const DevTable* tab, const c64* tables,
                               const int* par, int n_vec, const c64* x, c64* y, int Ng, int Nu,
                               int S, hipStream_t s) {
  if (S < 1) return hipErrorInvalidValue;
  const int n_slabs = (Ng + S - 1) / S, n_strips = strip_count(Nu);
  const long tasks = (long)n_vec * n_slabs * n_strips;
  const long blocks = (tasks + 3) / 4;
  if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(matvec_strip_kernel, dim3((unsigned)blocks), dim3(256), 0, s, md, tab, tables,
                     par, n_vec, x, y, S, n_slabs, n_strips);
  return hipGetLastError();
}

hipError_t launch_matvec_full(const DevModel* md, const DevTable* tab, const c64* tables,
                              int n_vec, const int* par, const c64* x, c64* y, c64* z, c64* yc,
                              c64* wA, c64* wB, int Nc, hipStream_t s) {
  if (n_vec > 65535) return hipErrorInvalidValue;
  dim3 grid((Nc + 255) / 256, n_vec);
  hipLaunchKernelGGL(gather_block_kernel, grid, dim3(256), 0, s, md, par, n_vec, x, z);
  hipLaunchKernelGGL(matvec_phase1_kernel, grid, dim3(256), 0, s, md, tab, tables, par, n_vec, z,
                     yc, wA, wB);
  hipLaunchKernelGGL(matvec_phase2_kernel, grid, dim3(256), 0, s, md, tab, tables, par, n_vec,
                     yc, wA, wB);
  hipLaunchKernelGGL(scatter_block_kernel, grid, dim3(256), 0, s, md, par, n_vec, yc, y);
  return hipGetLastError();
}

}  // namespace vdc
