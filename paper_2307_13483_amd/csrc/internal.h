// Internal declarations shared by the HIP translation units of libvdc.
// Not part of the C ABI (see include/vdc.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "vdc.h"

namespace vdc {

constexpr double kHartreeEV = 27.211386245988;
constexpr double kPi = 3.14159265358979323846;
constexpr int kBlock = 1024;      // threads per workgroup of the persistent solver
// elements per thread whose loads a streaming loop issues together before it
// stores any: one wait for memory per batch instead of one per element
constexpr int kBatch = 4;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxRestart = 128;
// Slot vectors of length ncap besides the basis: FP64 solver (x, b, dinv, w,
// wA, wB and the block factors l1, l2 with zt), FP32 inner solver (dinv, w,
// wA, wB, l1, l2, zt).
constexpr int kFp64SlotVectors = 9;
constexpr int kFp32SlotVectors = 7;
constexpr int kMaxFinal = 64;
constexpr int kNumF = 6;          // level-shift functions per energy
// Far-field expansion of the transform's node sum: clusters of kClus
// consecutive nodes, moments up to kClusP; per cluster: centre, half-width,
// then for the 6 functions g and the 6 functions x g: M_0, M_1 and
// mu_n = M_n / (n (n-1)), n = 2..kClusP.
// kSup consecutive clusters form a super-cluster with moments of its own,
// used where a whole wave's points are far from it.
constexpr int kClus = 64;
constexpr int kSup = 8;
constexpr int kClusP = 30;
constexpr int kClusStride = 2 + 2 * kNumF * (kClusP + 1);

// Resident workgroups of kBlock threads per CU for a solver kernel with
// dyn_lds bytes of dynamic LDS (1 when the runtime cannot tell).
template <typename Kernel>
inline int occupancy_of(Kernel k, size_t dyn_lds) {
  int n = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kBlock, dyn_lds);
  return (e == hipSuccess && n > 0) ? n : 1;
}

// Level-shift function index: mu-major, pairs (11, 12, 22).
//   0: F[f1e f1e]  1: F[f1e f2e]  2: F[f2e f2e]
//   3: F[f1o f1o]  4: F[f1o f2o]  5: F[f2o f2o]
__host__ __device__ constexpr int fidx(int mu, int pair) { return 3 * mu + pair; }

// Model parameters in the form the kernels read them (plain values + device
// pointers to the transform data owned by the model).
// Complex FP16: stored multipliers of the block factors.
struct c16 { _Float16 x, y; };

struct DevModel {
  int Ng, Nu, Nc;        // Nc = Ng*Nu unknowns per symmetry block
  int K;                 // transform nodes
  double omega_g, omega_u;
  double E1, E2;
  double kappa[2];       // [d]
  double lam;            // direct q_u coupling
  double lamd[2];        // continuum-coupling slopes lam_1, lam_2
  double A[2][2], B[2][2];
  int l[2];
  double glast[kNumF];   // interpolated width product at the last node
  double glastx[kNumF];  // the same for x g(x)
  const double* nodes;   // [K]            device
  const double* coef;    // [K][kNumF]     device: slope jumps c_k of g
  const double* coefx;   // [K][kNumF]     device: slope jumps of x g(x)
  int nclust;            // ceil(K / kClus)
  const double* clus;    // [nclust][kClusStride] device: far-field moments
  int nsup;              // ceil(nclust / kSup)
  const double* sup;     // [nsup][kClusStride] device: super-cluster moments
};

// One job as the kernels see it (host-filled, device-resident array).
struct DevJob {
  double eps_i;          // incident electron energy
  double E;              // total energy eps_i + E_{v_i}
  int vi_g, vi_u, mu;
  int parity;            // 0: state 1 on even n_u; 1: state 1 on odd n_u
  int model;             // index into the DevModel array
  int table;             // index of the per-energy table pair
  int out;               // index of the job in the caller's arrays
  int pad;
};

// Per-energy table set: 2 parities x 3 planes (AA, AB, BB) x Nc complex.
struct DevTable {
  double E;
  int model;
  int group;             // shift table it is gathered from
  int vg, vu;            // initial state of a job with this energy
  size_t offset;         // in complex elements from the table base
};

// Shift table of one (model, eps_i): level shifts at eps_i + w_g a + w_u b for
// the offsets a = v_g - n_g in [a_min, a_min + na), b = v_u - n_u in
// [b_min, b_min + nb), stored [point][6] from offset (complex elements).
struct DevGroup {
  double eps_i;
  int model;
  int a_min, na, b_min, nb;
  int perm_off;          // start of its point order (sorted by eps) in the perm array
  size_t offset;
};

// Planes per parity of a table set: 3 (level shift AA, AB, BB) or, for the
// adjoint, 9 (level shift, its eps derivative, and the transform of x g).
constexpr int kPlanesSolve = 3;
constexpr int kPlanesDeriv = 9;

// Per-job results written by the kernels, copied to vdc_job_info on the host.
struct DevInfo {
  int status, iters, restarts, outer;
  double rel_res;
  double alg_bytes;
  double defect = -1.0;  // optical-theorem defect of the solution (-1: not computed)
};

struct c64 { double x, y; };
struct c32 { float x, y; };

__host__ __device__ inline c64 mk(double a, double b) { return c64{a, b}; }
__host__ __device__ inline c64 operator+(c64 a, c64 b) { return c64{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline c64 operator-(c64 a, c64 b) { return c64{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline c64 operator*(c64 a, c64 b) {
  return c64{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ inline c64 operator*(double s, c64 a) { return c64{s * a.x, s * a.y}; }
__host__ __device__ inline c64 conjmul(c64 a, c64 b) {  // conj(a) * b
  return c64{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__host__ __device__ inline double norm2(c64 a) { return a.x * a.x + a.y * a.y; }

__host__ __device__ inline c32 operator+(c32 a, c32 b) { return c32{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline c32 operator-(c32 a, c32 b) { return c32{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline c32 operator*(c32 a, c32 b) {
  return c32{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ inline c32 operator*(float s, c32 a) { return c32{s * a.x, s * a.y}; }
__host__ __device__ inline c32 conjmul(c32 a, c32 b) {
  return c32{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__host__ __device__ inline float norm2(c32 a) { return a.x * a.x + a.y * a.y; }

// Launchers (defined in the .hip files).
hipError_t launch_level_shift_tables(const DevModel* models_dev, const DevGroup* groups_dev,
                                     int n_groups, int max_group_pts, const int* perm,
                                     const DevTable* tables_dev, int n_tables, int max_nc,
                                     c64* shift, c64* table_base, c32* table32_base,
                                     hipStream_t s, bool deriv = false);
hipError_t launch_level_shift_points(const DevModel& m, int n_eps, const double* eps,
                                     c64* out, hipStream_t s);

}  // namespace vdc
