// C ABI of libvdc: model build, workspace layout, job ordering and launches.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"
#include "co2.h"
#include "eels.h"
#include "blockops.h"
#include "solve_args.h"
#include "strip.h"
#include "terms_args.h"

namespace vdc {
hipError_t launch_gmres_fp64(const SolveArgs& a, int n_groups, size_t dyn_lds, hipStream_t s);
int gmres_fp64_occupancy(size_t dyn_lds);
hipError_t launch_cocg_fp64(const SolveArgs& a, int n_groups, size_t dyn_lds, hipStream_t s);
int cocg_fp64_occupancy(size_t dyn_lds);
hipError_t launch_cocg_mixed(const SolveArgs& a, int n_groups, size_t dyn_lds, hipStream_t s);
int cocg_mixed_occupancy(size_t dyn_lds);
hipError_t launch_fgmres_mixed(const SolveArgs& a, int n_groups, size_t dyn_lds, hipStream_t s);
int fgmres_mixed_occupancy(size_t dyn_lds);
hipError_t launch_zero_int(int* p, int n, hipStream_t s);
hipError_t launch_adjoint(const SolveArgs& a, int n_groups, size_t dyn_lds, hipStream_t s);
int adjoint_occupancy(size_t dyn_lds);
hipError_t launch_matvec_strip(const DevModel* md, const DevTable* tab, const c64* tables,
                               const int* par, int n_vec, const c64* x, c64* y, int Ng, int Nu,
                               int S, hipStream_t s);
hipError_t launch_matvec_full(const DevModel* md, const DevTable* tab, const c64* tables,
                              int n_vec, const int* parity_dev, const c64* x, c64* y, c64* z,
                              c64* yc, c64* wA, c64* wB, int Nc, hipStream_t s);
size_t plain_extra_elems(size_t ncap, int m);
hipError_t launch_co2_factor(const Co2FactorArgs& a, int Ns, int Na, hipStream_t s);
hipError_t launch_co2_gmres(const Co2Args& a, int n_groups, hipStream_t s);
hipError_t launch_co2_ops(const Co2OpsArgs& a, int n_groups, hipStream_t s);
hipError_t launch_co2_apply_split(const Co2OpsArgs& a, int npts, int batch, hipStream_t s);
hipError_t launch_co2_march(const Co2OpsArgs& a, int Ns, int Nx, int Ny, int Na, hipStream_t s);
bool co2_march_fits(int Ns, int Nx, int Ny, int Na);
constexpr int kCo2ApplyBatch = 128;   // vectors per pass pair of the split operator
int co2_factor_max_ny();
vdc_status solve_plain_impl(const SolveArgs& a, const std::vector<DevJob>& jobs,
                            const std::vector<DevModel>& models, hipStream_t s,
                            std::string& err);
}  // namespace vdc

using namespace vdc;

// Device memory of vdc_solve_noalloc: one array per GPU, allocated when the
// code object is loaded on it and held until the process ends.  Host code
// never uses the name as an address (it is a host-side stand-in); it takes
// the device address from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[VDC_NOALLOC_SCRATCH_BYTES];

// Term-list form of a model (vdc_model_create): the device model of the
// general kernels and the device memory it points to.
struct GenHost {
  DevGen dev{};
  int N = 0;                       // D npts
  std::vector<void*> mem;          // device allocations
  std::vector<vdc_model_t> ls;     // two-state transform models of the level shifts
  ~GenHost();
};

struct vdc_model {
  vdc_model2d_desc desc;
  DevModel dev;
  double* d_nodes = nullptr;
  double* d_coef = nullptr;
  double* d_coefx = nullptr;
  double* d_clus = nullptr;
  int kind = 0;                    // 0: two-state kernels available; 1: term lists only
  GenHost* gen = nullptr;          // term-list form (models from vdc_model_create)
};

GenHost::~GenHost() {
  for (void* p : mem)
    if (p) (void)hipFree(p);
  for (vdc_model_t m : ls) vdc_model_destroy(m);
}

namespace {

thread_local std::string g_err = "no error";
thread_local double g_ms_tables = 0.0, g_ms_solver = 0.0;

// Events bracketing the table kernel and the solver on the call's stream.
struct EventSet {
  hipEvent_t e[3] = {nullptr, nullptr, nullptr};
  bool ok = false;
  explicit EventSet(bool want = true) {
    if (!want) return;   // no events: nothing is created
    ok = true;
    for (auto& x : e) ok = ok && hipEventCreate(&x) == hipSuccess;
  }
  ~EventSet() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

vdc_status fail(vdc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

vdc_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return VDC_ERR_HIP;
}

#define HIPCHK(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// sqrt(Gamma_d Gamma_d') on the host, for the transform coefficients.
double width_pair_host(const vdc_model2d_desc& d, int mu, int d1, int d2, double x) {
  if (!(x > 0.0)) return 0.0;
  const double A = std::sqrt(d.A[d1][mu] * d.A[d2][mu]);
  const double rB = 0.5 / d.B[d1][mu] + 0.5 / d.B[d2][mu];
  return A * std::pow(x, d.l[mu] + 0.5) * std::exp(-x * rB);
}

double vib_energy(const vdc_model2d_desc& d, int g, int u) {
  return d.omega_g * (g + 0.5) + d.omega_u * (u + 0.5);
}

struct Plan {
  std::vector<DevModel> models;
  std::vector<DevJob> jobs;       // sorted, longest first
  std::vector<DevTable> tabs;
  std::vector<DevGroup> groups;
  int max_nc = 0;
  int max_nu = 0;
  int tileT = 0, tileT32 = 0;
  size_t dyn_lds = 0;
  int max_group_pts = 0;
  size_t shift_elems = 0;
  std::vector<int> perm;          // per rectangle shape: points in order of eps
  bool deriv = false;
  size_t table_elems = 0;
  int n_groups = 0;
  size_t ncap = 0, slot_elems = 0;
  // byte offsets
  size_t off_counter, off_models, off_jobs, off_tabs, off_groups, off_perm, off_finals, off_info,
      off_shift, off_tables, off_tables32, off_scratch, total;
};

int cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
  return n > 0 ? n : 256;
}

// Optional plan settings: an output index per job (a re-solve of some jobs
// of a larger call writes their rows of the caller's arrays), the length of
// those arrays, and a cap on the resident workgroups (fewer slots, so that a
// plan fits a given amount of memory).
struct PlanExtra {
  const int* out_map = nullptr;
  int n_out = -1;
  int max_groups = 0;
  bool untimed = false;   // record no kernel-time events (creates none)
  double* hist = nullptr; // residual histories [n_out][hist_len] (device)
  int hist_len = 0;
};

vdc_status make_plan(int n_models, const vdc_model_t* models, const vdc_solve_opts* o,
                     int n_jobs, const vdc_job* jobs, int n_final, bool plain, Plan& P,
                     bool adjoint = false, const PlanExtra* ex = nullptr) {
  const int n_out = (ex && ex->out_map) ? ex->n_out : n_jobs;
  if (n_models <= 0 || !models) return fail(VDC_ERR_INVALID_ARG, "no models");
  if (!o) return fail(VDC_ERR_INVALID_ARG, "opts is NULL");
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(VDC_ERR_INVALID_ARG, "bad job list");
  if (n_final < 0 || n_final > kMaxFinal) return fail(VDC_ERR_INVALID_ARG, "n_final must be 0..64");
  if (o->restart < 1 || o->restart > kMaxRestart) return fail(VDC_ERR_INVALID_ARG, "restart must be 1..128");
  if (o->max_iter < 1) return fail(VDC_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (!(o->tol > 0.0)) return fail(VDC_ERR_INVALID_ARG, "tol must be > 0");
  if (o->precond != VDC_PREC_NONE && o->precond != VDC_PREC_JACOBI &&
      o->precond != VDC_PREC_BLOCK && o->precond != VDC_PREC_ROWS)
    return fail(VDC_ERR_INVALID_ARG, "unknown preconditioner");
  if (o->precision != VDC_FP64 && o->precision != VDC_FP32_INNER)
    return fail(VDC_ERR_INVALID_ARG, "unknown precision");
  if (o->method != VDC_GMRES && o->method != VDC_COCG)
    return fail(VDC_ERR_INVALID_ARG, "unknown method");
  const bool mixed = o->precision == VDC_FP32_INNER;
  const bool cocg = o->method == VDC_COCG;
  if (cocg && plain) return fail(VDC_ERR_UNSUPPORTED, "COCG runs in the batched solves only");
  if (mixed && adjoint) return fail(VDC_ERR_UNSUPPORTED, "the adjoint solve is FP64 only");
  P.deriv = adjoint;
  const int planes = adjoint ? kPlanesDeriv : kPlanesSolve;
  const int shift_per_point = adjoint ? 3 * kNumF : kNumF;
  if (mixed) {
    if (plain) return fail(VDC_ERR_UNSUPPORTED, "the plain path is FP64 only");
    if (o->inner_restart < 1 || (!cocg && o->inner_restart > kMaxRestart))
      return fail(VDC_ERR_INVALID_ARG, "inner_restart must be 1..128 (>= 1 for COCG)");
    if (o->outer_restart < 1 || o->outer_restart > 32)
      return fail(VDC_ERR_INVALID_ARG, "outer_restart must be 1..32");
    if (!(o->inner_tol > 0.0) || !(o->inner_tol < 1.0))
      return fail(VDC_ERR_INVALID_ARG, "inner_tol must be in (0, 1)");
  }
  P.models.resize(n_models);
  for (int k = 0; k < n_models; ++k) {
    if (!models[k]) return fail(VDC_ERR_INVALID_ARG, "NULL model");
    if (models[k]->kind != 0)
      return fail(VDC_ERR_INVALID_ARG, "a model built from term lists without the two-state form: "
                                       "use vdc_model_solve");
    P.models[k] = models[k]->dev;
    P.max_nc = std::max(P.max_nc, models[k]->dev.Nc);
    P.max_nu = std::max(P.max_nu, models[k]->dev.Nu);
  }
  // LDS tiles of the fused operator pass (96 KB budget next to the static LDS)
  const size_t kTileBudget = 96 * 1024;
  if (o->tile_rows < 0) return fail(VDC_ERR_INVALID_ARG, "tile_rows must be >= 0");
  P.tileT = tile_rows(P.max_nu, sizeof(c64), kTileBudget);
  P.tileT32 = mixed ? tile_rows(P.max_nu, sizeof(c32), kTileBudget) : 0;
  if (o->tile_rows > 0) {
    P.tileT = std::min(P.tileT, o->tile_rows);
    P.tileT32 = std::min(P.tileT32, o->tile_rows);
  }
  P.dyn_lds = std::max((size_t)(3 * P.tileT + 8) * P.max_nu * sizeof(c64) * (P.tileT > 0),
                       (size_t)(3 * P.tileT32 + 8) * P.max_nu * sizeof(c32) * (P.tileT32 > 0));
  std::map<std::pair<int, double>, int> tab_index;
  // jobs sharing (model, eps_i) share one shift table over the offsets they need
  std::map<std::pair<int, double>, int> grp_index;
  std::vector<int> gvmin_g, gvmax_g, gvmin_u, gvmax_u;
  for (int j = 0; j < n_jobs; ++j) {
    const vdc_job& jb = jobs[j];
    if (jb.model < 0 || jb.model >= n_models) return fail(VDC_ERR_INVALID_ARG, "job model index out of range");
    auto key = std::make_pair(jb.model, jb.eps_i);
    auto it = grp_index.find(key);
    if (it == grp_index.end()) {
      it = grp_index.emplace(key, (int)P.groups.size()).first;
      DevGroup g{};
      g.eps_i = jb.eps_i;
      g.model = jb.model;
      P.groups.push_back(g);
      gvmin_g.push_back(jb.vi_g);
      gvmax_g.push_back(jb.vi_g);
      gvmin_u.push_back(jb.vi_u);
      gvmax_u.push_back(jb.vi_u);
    } else {
      const int g = it->second;
      gvmin_g[g] = std::min(gvmin_g[g], jb.vi_g);
      gvmax_g[g] = std::max(gvmax_g[g], jb.vi_g);
      gvmin_u[g] = std::min(gvmin_u[g], jb.vi_u);
      gvmax_u[g] = std::max(gvmax_u[g], jb.vi_u);
    }
  }
  std::map<std::tuple<int, int, int>, int> perm_index;   // (model, na, nb) -> offset
  for (size_t g = 0; g < P.groups.size(); ++g) {
    DevGroup& G = P.groups[g];
    const DevModel& md = P.models[G.model];
    G.a_min = gvmin_g[g] - (md.Ng - 1);
    G.na = gvmax_g[g] - G.a_min + 1;
    G.b_min = gvmin_u[g] - (md.Nu - 1);
    G.nb = gvmax_u[g] - G.b_min + 1;
    const auto pk = std::make_tuple(G.model, G.na, G.nb);
    auto pit = perm_index.find(pk);
    if (pit == perm_index.end()) {
      // eps = eps_i + w_g a + w_u b: order the rectangle's points by w_g ia + w_u ib
      const int off = (int)P.perm.size();
      const int npts = G.na * G.nb;
      std::vector<std::pair<double, int>> key(npts);
      for (int ia = 0; ia < G.na; ++ia)
        for (int ib = 0; ib < G.nb; ++ib)
          key[ia * G.nb + ib] = std::make_pair(md.omega_g * ia + md.omega_u * ib, ia * G.nb + ib);
      std::sort(key.begin(), key.end());
      for (int q = 0; q < npts; ++q) P.perm.push_back(key[q].second);
      pit = perm_index.emplace(pk, off).first;
    }
    G.perm_off = pit->second;
    G.offset = P.shift_elems;
    P.shift_elems += (size_t)G.na * G.nb * shift_per_point;
    P.max_group_pts = std::max(P.max_group_pts, G.na * G.nb);
  }
  if (P.groups.size() > 65535) return fail(VDC_ERR_INVALID_ARG, "more than 65535 distinct incident energies");
  P.jobs.resize(n_jobs);
  for (int j = 0; j < n_jobs; ++j) {
    const vdc_job& jb = jobs[j];
    if (jb.model < 0 || jb.model >= n_models) return fail(VDC_ERR_INVALID_ARG, "job model index out of range");
    const vdc_model2d_desc& d = models[jb.model]->desc;
    if (!(jb.eps_i > 0.0) || !std::isfinite(jb.eps_i))
      return fail(VDC_ERR_INVALID_ARG, "eps_i must be > 0 (open entrance channel)");
    if (jb.vi_g < 0 || jb.vi_g >= d.Ng || jb.vi_u < 0 || jb.vi_u >= d.Nu)
      return fail(VDC_ERR_INVALID_ARG, "v_i outside the basis");
    if (jb.mu_i != 0 && jb.mu_i != 1) return fail(VDC_ERR_INVALID_ARG, "mu_i must be 0 or 1");
    DevJob& o2 = P.jobs[j];
    o2.eps_i = jb.eps_i;
    o2.E = jb.eps_i + vib_energy(d, jb.vi_g, jb.vi_u);
    o2.vi_g = jb.vi_g;
    o2.vi_u = jb.vi_u;
    o2.mu = jb.mu_i;
    o2.parity = (jb.vi_u + jb.mu_i) & 1;
    o2.model = jb.model;
    o2.out = (ex && ex->out_map) ? ex->out_map[j] : j;
    o2.pad = 0;
    auto key = std::make_pair(jb.model, o2.E);
    auto it = tab_index.find(key);
    if (it == tab_index.end()) {
      DevTable t;
      t.E = o2.E;
      t.model = jb.model;
      t.group = grp_index.at(std::make_pair(jb.model, jb.eps_i));
      t.vg = jb.vi_g;
      t.vu = jb.vi_u;
      t.offset = P.table_elems;
      P.table_elems += 2 * planes * (size_t)P.models[jb.model].Nc;
      it = tab_index.emplace(key, (int)P.tabs.size()).first;
      P.tabs.push_back(t);
    }
    o2.table = it->second;
  }
  if ((int)P.tabs.size() > 65535) return fail(VDC_ERR_INVALID_ARG, "more than 65535 distinct energies");
  // longest first: cost ~ unknowns x (iterations grow with the total energy)
  std::stable_sort(P.jobs.begin(), P.jobs.end(), [&](const DevJob& a, const DevJob& b) {
    const double ca = P.models[a.model].Nc * (0.5 + a.E);
    const double cb = P.models[b.model].Nc * (0.5 + b.E);
    return ca > cb;
  });
  const int m = cocg ? 4 : (mixed ? o->outer_restart : o->restart);
  P.ncap = (size_t)((P.max_nc + 63) / 64) * 64;
  if (mixed && cocg) {
    // FP64 refinement over FP32 COCG (cocg_mixed_kernel): FP64 x, b, r, wA,
    // wB; FP32 (in c64 units) r, p, q, d, 1/D, the two FP16 multiplier
    // planes (one FP32 plane together), wA, wB.  No basis and no Hessenberg:
    // inner_restart is only a step limit and does not enter the size.
    P.slot_elems = (size_t)5 * P.ncap + ((size_t)8 * P.ncap + 1) / 2;
  } else if (mixed) {
    // FP64: Vout (m+1), Z (m), x, b, w, wA, wB, R_out, R_in;
    // FP32 (in c64 units): Vin (m_in+1) and the inner solver's vectors
    const int mi = o->inner_restart;
    P.slot_elems = (size_t)(2 * m + 6) * P.ncap + (size_t)(m + 1) * m + (size_t)(mi + 1) * mi +
                   ((size_t)(mi + 1 + kFp32SlotVectors) * P.ncap + 1) / 2;
  } else {
    // V (m+1), the solver's vectors, R (+ the forward solution for the adjoint)
    P.slot_elems = (size_t)(m + 1 + kFp64SlotVectors) * P.ncap + (size_t)(m + 1) * m;
    if (plain) P.slot_elems += plain_extra_elems(P.ncap, m);
    if (adjoint) P.slot_elems += P.ncap;
  }
  P.slot_elems = (P.slot_elems + 31) / 32 * 32;
  int occ = 1;
  if (!plain)
    occ = adjoint ? adjoint_occupancy(P.dyn_lds)
                  : (mixed ? (cocg ? cocg_mixed_occupancy(P.dyn_lds) : fgmres_mixed_occupancy(P.dyn_lds))
                           : (cocg ? cocg_fp64_occupancy(P.dyn_lds) : gmres_fp64_occupancy(P.dyn_lds)));
  P.n_groups = plain ? 1 : std::max(1, std::min(n_jobs, cu_count() * occ));
  if (ex && ex->max_groups > 0) P.n_groups = std::min(P.n_groups, ex->max_groups);
  size_t off = 0;
  P.off_counter = off; off += 256;
  P.off_models = off; off = align256(off + sizeof(DevModel) * n_models);
  P.off_jobs = off; off = align256(off + sizeof(DevJob) * std::max(1, n_jobs));
  P.off_tabs = off; off = align256(off + sizeof(DevTable) * std::max<size_t>(1, P.tabs.size()));
  P.off_groups = off; off = align256(off + sizeof(DevGroup) * std::max<size_t>(1, P.groups.size()));
  P.off_perm = off; off = align256(off + sizeof(int) * std::max<size_t>(1, P.perm.size()));
  P.off_finals = off; off = align256(off + sizeof(int) * 2 * std::max(1, n_final));
  P.off_info = off; off = align256(off + sizeof(DevInfo) * std::max(1, n_out));
  P.off_shift = off; off = align256(off + sizeof(c64) * P.shift_elems);
  P.off_tables = off; off = align256(off + sizeof(c64) * P.table_elems);
  P.off_tables32 = off; off = align256(off + (mixed ? sizeof(c32) * P.table_elems : 0));
  P.off_scratch = off; off = align256(off + sizeof(c64) * P.slot_elems * P.n_groups);
  P.total = off;
  return VDC_OK;
}

struct AdjointIO {
  const double* psi;
  const double* T;
  const double* dsig;
  double* grad_jobs;
  double* grad;
};

// A solve as it sits in the workspace: the plan, the kernels' arguments and
// what the table kernels need.  Filled by prepare_solve, launched by
// enqueue_solve (kernels only: no copy, no memset, no host synchronisation).
struct Prepared {
  Plan P;
  SolveArgs a{};
  char* ws = nullptr;
  bool mixed = false, cocg = false, plain = false, adjoint = false;
  int n_jobs = 0;
  std::vector<int> out_map;   // caller index of each job (empty: the identity)
  int n_out = 0;              // entries of the info array in the workspace
};

vdc_status prepare_solve(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                         int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                         void* workspace, size_t ws_bytes, double* T_out, double* sigma_out,
                         double* psi_out, hipStream_t s, bool plain, const AdjointIO* adj,
                         Prepared& R, const PlanExtra* ex = nullptr) {
  Plan& P = R.P;
  vdc_status st = make_plan(n_models, models, opts, n_jobs, jobs, n_final, plain, P, adj != nullptr,
                            ex);
  if (st != VDC_OK) return st;
  R.n_jobs = n_jobs;
  R.n_out = n_jobs;
  if (ex && ex->out_map) {
    R.out_map.assign(ex->out_map, ex->out_map + n_jobs);
    R.n_out = ex->n_out;
  }
  if (n_jobs == 0) return VDC_OK;
  if (!workspace) return fail(VDC_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(VDC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < P.total)
    return fail(VDC_ERR_WORKSPACE, "workspace too small: need " + std::to_string(P.total) +
                                       " bytes, got " + std::to_string(ws_bytes));
  if (!adj && n_final > 0 && (!finals || !T_out || !sigma_out))
    return fail(VDC_ERR_INVALID_ARG, "finals/T_out/sigma_out must be non-NULL when n_final > 0");
  if (adj && (!adj->psi || !adj->grad_jobs || (n_final > 0 && (!finals || !adj->T || !adj->dsig))))
    return fail(VDC_ERR_INVALID_ARG, "psi, T, dL_dsigma, finals and grad_jobs must be non-NULL");
  char* ws = static_cast<char*>(workspace);
  R.ws = ws;
  R.mixed = opts->precision == VDC_FP32_INNER;
  R.cocg = opts->method == VDC_COCG;
  R.plain = plain;
  R.adjoint = adj != nullptr;
  const bool mixed = R.mixed;

  HIPCHK(hipMemcpyAsync(ws + P.off_models, P.models.data(), sizeof(DevModel) * n_models,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + P.off_jobs, P.jobs.data(), sizeof(DevJob) * n_jobs,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + P.off_tabs, P.tabs.data(), sizeof(DevTable) * P.tabs.size(),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + P.off_groups, P.groups.data(), sizeof(DevGroup) * P.groups.size(),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + P.off_perm, P.perm.data(), sizeof(int) * P.perm.size(),
                        hipMemcpyHostToDevice, s));
  if (n_final > 0)
    HIPCHK(hipMemcpyAsync(ws + P.off_finals, finals, sizeof(int) * 2 * n_final,
                          hipMemcpyHostToDevice, s));

  SolveArgs& a = R.a;
  a.models = reinterpret_cast<const DevModel*>(ws + P.off_models);
  a.jobs = reinterpret_cast<const DevJob*>(ws + P.off_jobs);
  a.n_jobs = n_jobs;
  a.tabs = reinterpret_cast<const DevTable*>(ws + P.off_tabs);
  a.tables = reinterpret_cast<const c64*>(ws + P.off_tables);
  a.tables32 = mixed ? reinterpret_cast<const c32*>(ws + P.off_tables32) : nullptr;
  a.counter = reinterpret_cast<int*>(ws + P.off_counter);
  a.scratch = reinterpret_cast<c64*>(ws + P.off_scratch);
  a.slot_elems = P.slot_elems;
  a.ncap = P.ncap;
  a.m = opts->method == VDC_COCG ? 4 : (mixed ? opts->outer_restart : opts->restart);
  a.max_iter = opts->max_iter;
  a.tol = opts->tol;
  a.precond = opts->precond;
  a.method = opts->method;
  a.m_in = opts->inner_restart;
  a.tol_in = opts->inner_tol;
  a.n_final = n_final;
  a.finals = reinterpret_cast<const int*>(ws + P.off_finals);
  a.T_out = reinterpret_cast<c64*>(T_out);
  a.sigma_out = sigma_out;
  a.psi_out = reinterpret_cast<c64*>(psi_out);
  a.psi_ld = 2 * (size_t)P.max_nc;
  a.info = reinterpret_cast<DevInfo*>(ws + P.off_info);
  a.planes = adj ? kPlanesDeriv : kPlanesSolve;
  a.tileT = P.tileT;
  a.tileT32 = P.tileT32;
  a.check_optical = opts->check_optical != 0;
  if (adj) {
    a.psi_in = reinterpret_cast<const c64*>(adj->psi);
    a.T_in = reinterpret_cast<const c64*>(adj->T);
    a.dsig = adj->dsig;
    a.grad = adj->grad_jobs;
  }
  if (ex && ex->hist) {
    a.hist = ex->hist;
    a.hist_len = ex->hist_len;
  }
  return VDC_OK;
}

// The counter reset, the level-shift tables and the persistent solver kernel
// (not the plain path, which reads status back between its kernels).  With
// ev, events bracket the tables and the solver.
vdc_status enqueue_solve(const Prepared& R, hipStream_t s, EventSet* ev) {
  const Plan& P = R.P;
  const SolveArgs& a = R.a;
  char* ws = R.ws;
  HIPCHK(launch_zero_int(reinterpret_cast<int*>(ws + P.off_counter), 64, s));
  if (ev) HIPCHK(hipEventRecord(ev->e[0], s));
  HIPCHK(launch_level_shift_tables(a.models, reinterpret_cast<const DevGroup*>(ws + P.off_groups),
                                   (int)P.groups.size(), P.max_group_pts,
                                   reinterpret_cast<const int*>(ws + P.off_perm), a.tabs,
                                   (int)P.tabs.size(), P.max_nc,
                                   reinterpret_cast<c64*>(ws + P.off_shift),
                                   reinterpret_cast<c64*>(ws + P.off_tables),
                                   R.mixed ? reinterpret_cast<c32*>(ws + P.off_tables32) : nullptr,
                                   s, P.deriv));
  if (ev) HIPCHK(hipEventRecord(ev->e[1], s));
  if (R.adjoint) {
    HIPCHK(launch_adjoint(a, P.n_groups, P.dyn_lds, s));
  } else if (R.mixed && R.cocg) {
    HIPCHK(launch_cocg_mixed(a, P.n_groups, P.dyn_lds, s));
  } else if (R.mixed) {
    HIPCHK(launch_fgmres_mixed(a, P.n_groups, P.dyn_lds, s));
  } else if (R.cocg) {
    HIPCHK(launch_cocg_fp64(a, P.n_groups, P.dyn_lds, s));
  } else {
    HIPCHK(launch_gmres_fp64(a, P.n_groups, P.dyn_lds, s));
  }
  if (ev) HIPCHK(hipEventRecord(ev->e[2], s));
  return VDC_OK;
}

// Per-job results from the workspace (synchronises the stream).
vdc_status read_info(const Prepared& R, vdc_job_info* info, hipStream_t s) {
  std::vector<DevInfo> hinfo(R.n_out);
  HIPCHK(hipMemcpyAsync(hinfo.data(), R.ws + R.P.off_info, sizeof(DevInfo) * R.n_out,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (info) {
    for (int k = 0; k < R.n_jobs; ++k) {
      const int j = R.out_map.empty() ? k : R.out_map[k];
      info[j].retried = 0;
      info[j].status = hinfo[j].status;
      info[j].iters = hinfo[j].iters;
      info[j].restarts = hinfo[j].restarts;
      info[j].outer_iters = hinfo[j].outer;
      info[j].rel_res = hinfo[j].rel_res;
      info[j].alg_bytes = hinfo[j].alg_bytes;
      info[j].optical_defect = hinfo[j].defect;
    }
  }
  return VDC_OK;
}

vdc_status run_solve(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                     int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                     void* workspace, size_t ws_bytes, double* T_out, double* sigma_out,
                     double* psi_out, vdc_job_info* info, void* stream, bool plain,
                     const AdjointIO* adj = nullptr, const PlanExtra* ex = nullptr) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Prepared R;
  vdc_status st = prepare_solve(n_models, models, opts, n_jobs, jobs, n_final, finals, workspace,
                                ws_bytes, T_out, sigma_out, psi_out, s, plain, adj, R, ex);
  if (st != VDC_OK || n_jobs == 0) return st;
  EventSet ev(!(ex && ex->untimed));
  if (plain) {
    HIPCHK(launch_zero_int(reinterpret_cast<int*>(R.ws + R.P.off_counter), 64, s));
    if (ev.ok) HIPCHK(hipEventRecord(ev.e[0], s));
    const Plan& P = R.P;
    const SolveArgs& a = R.a;
    HIPCHK(launch_level_shift_tables(a.models, reinterpret_cast<const DevGroup*>(R.ws + P.off_groups),
                                     (int)P.groups.size(), P.max_group_pts,
                                     reinterpret_cast<const int*>(R.ws + P.off_perm), a.tabs,
                                     (int)P.tabs.size(), P.max_nc,
                                     reinterpret_cast<c64*>(R.ws + P.off_shift),
                                     reinterpret_cast<c64*>(R.ws + P.off_tables), nullptr, s,
                                     P.deriv));
    if (ev.ok) HIPCHK(hipEventRecord(ev.e[1], s));
    std::string err;
    st = solve_plain_impl(a, P.jobs, P.models, s, err);
    if (st != VDC_OK) return fail(st, err);
    if (ev.ok) HIPCHK(hipEventRecord(ev.e[2], s));
  } else {
    st = enqueue_solve(R, s, ev.ok ? &ev : nullptr);
    if (st != VDC_OK) return st;
  }
  st = read_info(R, info, s);
  if (st != VDC_OK) return st;
  if (ev.ok) {
    float t1 = 0.f, t2 = 0.f;
    HIPCHK(hipEventElapsedTime(&t1, ev.e[0], ev.e[1]));
    HIPCHK(hipEventElapsedTime(&t2, ev.e[1], ev.e[2]));
    g_ms_tables = t1;
    g_ms_solver = t2;
  }
  if (adj && adj->grad) {
    // per-job contributions summed in job order on the host (fixed order)
    std::vector<double> g((size_t)n_jobs * 16);
    HIPCHK(hipMemcpy(g.data(), adj->grad_jobs, sizeof(double) * g.size(), hipMemcpyDeviceToHost));
    for (int p = 0; p < 16; ++p) {
      double t = 0.0;
      for (int j = 0; j < n_jobs; ++j) t += g[(size_t)j * 16 + p];
      adj->grad[p] = t;
    }
  }
  return VDC_OK;
}

// FP32-inner jobs that did not converge (stagnation, breakdown or a
// non-finite value in FP32) are solved again in FP64 with the same method,
// preconditioner and limits, into their own rows of the caller's outputs,
// using the caller's workspace (the first solve is complete: read_info
// synchronised the stream).  With fewer slots when the FP64 plan of these jobs
// does not fit the workspace; a job is marked retried = 1, or 2 when not even
// one slot fits.  The kernel timings of the first solve are kept.
vdc_status retry_fp64(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                      int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                      void* workspace, size_t ws_bytes, double* T_out, double* sigma_out,
                      double* psi_out, vdc_job_info* info, void* stream,
                      bool untimed = false) {
  std::vector<int> idx;
  for (int j = 0; j < n_jobs; ++j)
    if (info[j].status != VDC_CONVERGED) idx.push_back(j);
  if (idx.empty()) return VDC_OK;
  std::vector<vdc_job> sub(idx.size());
  for (size_t k = 0; k < idx.size(); ++k) sub[k] = jobs[idx[k]];
  vdc_solve_opts o64 = *opts;
  o64.precision = VDC_FP64;
  PlanExtra ex;
  ex.out_map = idx.data();
  ex.n_out = n_jobs;
  ex.untimed = untimed;
  Plan P;
  vdc_status st = make_plan(n_models, models, &o64, (int)sub.size(), sub.data(), n_final, false, P,
                            false, &ex);
  if (st != VDC_OK) return st;
  if (P.total > ws_bytes) {
    const size_t slot = sizeof(c64) * P.slot_elems;
    const size_t avail = ws_bytes > P.off_scratch + 256 ? ws_bytes - P.off_scratch - 256 : 0;
    const int g = (int)std::min<size_t>(avail / slot, (size_t)P.n_groups);
    if (g < 1) {
      for (int j : idx) info[j].retried = 2;
      return VDC_OK;
    }
    ex.max_groups = g;
  }
  const double t1 = g_ms_tables, t2 = g_ms_solver;
  st = run_solve(n_models, models, &o64, (int)sub.size(), sub.data(), n_final, finals, workspace,
                 ws_bytes, T_out, sigma_out, psi_out, info, stream, false, nullptr, &ex);
  g_ms_tables = t1;
  g_ms_solver = t2;
  if (st != VDC_OK) return st;
  for (int j : idx) info[j].retried = 1;
  return VDC_OK;
}

// Device address of this GPU's scratch array (looked up with the device
// current, once per device, then cached).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

vdc_status scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(VDC_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(VDC_ERR_HIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return VDC_OK;
}

}  // namespace

struct vdc_batch {
  Prepared R;
  EventSet ev;             // bracket the tables and the solver of each eager launch
  bool timed = false;      // an eager launch has recorded them
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};

extern "C" {

const char* vdc_last_error(void) { return g_err.c_str(); }

vdc_status vdc_last_kernel_times(double* ms_tables, double* ms_solver) {
  if (ms_tables) *ms_tables = g_ms_tables;
  if (ms_solver) *ms_solver = g_ms_solver;
  return VDC_OK;
}

const char* vdc_version(void) { return "vdc 0.1 gfx950"; }

vdc_status vdc_model2d_create(const vdc_model2d_desc* d, vdc_model_t* out) {
  if (!d || !out) return fail(VDC_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (d->Ng < 1 || d->Nu < 1 || d->Ng > kSqMax || d->Nu > kSqMax)
    return fail(VDC_ERR_INVALID_ARG, "Ng and Nu must be 1..1024");
  if (d->hilbert_nodes < 16 || d->hilbert_nodes > 65536)
    return fail(VDC_ERR_INVALID_ARG, "hilbert_nodes must be 16..65536");
  if (!(d->hilbert_xmax > 0.0) || !std::isfinite(d->hilbert_xmax))
    return fail(VDC_ERR_INVALID_ARG, "hilbert_xmax must be > 0");
  for (int mu = 0; mu < 2; ++mu) {
    if (d->l[mu] < 0 || d->l[mu] > 4) return fail(VDC_ERR_INVALID_ARG, "l must be 0..4");
    for (int s = 0; s < 2; ++s) {
      if (!(d->A[s][mu] >= 0.0) || !std::isfinite(d->A[s][mu]))
        return fail(VDC_ERR_INVALID_ARG, "width amplitudes A must be finite and >= 0");
      if (!(d->B[s][mu] > 0.0) || !std::isfinite(d->B[s][mu]))
        return fail(VDC_ERR_INVALID_ARG, "width scales B must be finite and > 0");
    }
  }
  const double scal[] = {d->omega_g, d->omega_u, d->kappa1, d->kappa2, d->lam,
                         d->lam1,    d->lam2,    d->E1,     d->gap};
  for (double v : scal)
    if (!std::isfinite(v)) return fail(VDC_ERR_INVALID_ARG, "non-finite model parameter");
  if (!(d->omega_g > 0.0) || !(d->omega_u > 0.0))
    return fail(VDC_ERR_INVALID_ARG, "vibrational frequencies must be > 0");
  if (!std::isfinite(d->E1 + d->gap))
    return fail(VDC_ERR_INVALID_ARG, "E1 + gap overflows");
  if ((size_t)d->Ng * d->Nu > (size_t)1 << 26) return fail(VDC_ERR_INVALID_ARG, "basis too large");

  vdc_model* m = new vdc_model();
  m->desc = *d;
  DevModel& dm = m->dev;
  dm.Ng = d->Ng;
  dm.Nu = d->Nu;
  dm.Nc = d->Ng * d->Nu;
  dm.K = d->hilbert_nodes;
  dm.omega_g = d->omega_g;
  dm.omega_u = d->omega_u;
  dm.E1 = d->E1;
  dm.E2 = d->E1 + d->gap;
  dm.kappa[0] = d->kappa1;
  dm.kappa[1] = d->kappa2;
  dm.lam = d->lam;
  dm.lamd[0] = d->lam1;
  dm.lamd[1] = d->lam2;
  for (int s = 0; s < 2; ++s)
    for (int mu = 0; mu < 2; ++mu) {
      dm.A[s][mu] = d->A[s][mu];
      dm.B[s][mu] = d->B[s][mu];
    }
  dm.l[0] = d->l[0];
  dm.l[1] = d->l[1];
  // transform data: nodes, slope jumps c_k of the interpolated width products
  const int K = dm.K;
  std::vector<double> x(K), coef((size_t)K * kNumF, 0.0), coefx((size_t)K * kNumF, 0.0);
  for (int k = 0; k < K; ++k) {
    const double t = k * std::sqrt(d->hilbert_xmax) / (K - 1);
    x[k] = t * t;
  }
  for (int mu = 0; mu < 2; ++mu) {
    const int pairs[3][2] = {{0, 0}, {0, 1}, {1, 1}};
    for (int pq = 0; pq < 3; ++pq) {
      const int f = fidx(mu, pq);
      std::vector<double> g(K);
      for (int k = 0; k < K; ++k) g[k] = width_pair_host(*d, mu, pairs[pq][0], pairs[pq][1], x[k]);
      double sprev = 0.0, sxprev = 0.0;
      for (int k = 0; k < K; ++k) {
        const double s = (k + 1 < K) ? (g[k + 1] - g[k]) / (x[k + 1] - x[k]) : 0.0;
        const double sx =
            (k + 1 < K) ? (x[k + 1] * g[k + 1] - x[k] * g[k]) / (x[k + 1] - x[k]) : 0.0;
        coef[(size_t)k * kNumF + f] = s - sprev;
        coefx[(size_t)k * kNumF + f] = sx - sxprev;
        sprev = s;
        sxprev = sx;
      }
      dm.glast[f] = g[K - 1];
      dm.glastx[f] = x[K - 1] * g[K - 1];
    }
  }
  // far-field moments per cluster of nodes and per super-cluster of kSup
  // clusters (see levelshift.hip), summed in extended precision and rounded
  // once: the super-clusters' sums run over 512 nodes
  const int nclust = (K + kClus - 1) / kClus;
  const int nsup = (nclust + kSup - 1) / kSup;
  std::vector<double> clus((size_t)(nclust + nsup) * kClusStride, 0.0);
  auto moments = [&](int k0, int k1, double* C) {
    const double xc = 0.5 * (x[k0] + x[k1 - 1]);
    C[0] = xc;
    C[1] = 0.5 * (x[k1 - 1] - x[k0]);
    for (int kind = 0; kind < 2; ++kind) {
      const std::vector<double>& cf = kind == 0 ? coef : coefx;
      for (int f = 0; f < kNumF; ++f) {
        long double M[kClusP + 1] = {};
        for (int k = k0; k < k1; ++k) {
          const long double ck = cf[(size_t)k * kNumF + f], d = (long double)x[k] - xc;
          long double dn = 1.0L;
          for (int n = 0; n <= kClusP; ++n) {
            M[n] += ck * dn;
            dn *= d;
          }
        }
        double* out = C + 2 + (kind * kNumF + f) * (kClusP + 1);
        for (int n = 0; n <= kClusP; ++n)
          out[n] = (double)(n >= 2 ? M[n] / ((long double)n * (n - 1)) : M[n]);
      }
    }
  };
  for (int c = 0; c < nclust; ++c)
    moments(c * kClus, std::min(K, (c + 1) * kClus), clus.data() + (size_t)c * kClusStride);
  for (int sc = 0; sc < nsup; ++sc)
    moments(sc * kSup * kClus, std::min(K, (sc + 1) * kSup * kClus),
            clus.data() + (size_t)(nclust + sc) * kClusStride);
  hipError_t e = hipMalloc(&m->d_nodes, sizeof(double) * K);
  if (e == hipSuccess) e = hipMalloc(&m->d_coef, sizeof(double) * K * kNumF);
  if (e == hipSuccess) e = hipMalloc(&m->d_coefx, sizeof(double) * K * kNumF);
  if (e == hipSuccess) e = hipMalloc(&m->d_clus, sizeof(double) * clus.size());
  if (e == hipSuccess) e = hipMemcpy(m->d_nodes, x.data(), sizeof(double) * K, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(m->d_coef, coef.data(), sizeof(double) * K * kNumF, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(m->d_coefx, coefx.data(), sizeof(double) * K * kNumF, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(m->d_clus, clus.data(), sizeof(double) * clus.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (m->d_nodes) (void)hipFree(m->d_nodes);
    if (m->d_coef) (void)hipFree(m->d_coef);
    if (m->d_coefx) (void)hipFree(m->d_coefx);
    if (m->d_clus) (void)hipFree(m->d_clus);
    delete m;
    return hip_fail(e, "model upload");
  }
  dm.nodes = m->d_nodes;
  dm.coef = m->d_coef;
  dm.coefx = m->d_coefx;
  dm.nclust = nclust;
  dm.clus = m->d_clus;
  dm.nsup = nsup;
  dm.sup = m->d_clus + (size_t)nclust * kClusStride;
  *out = m;
  return VDC_OK;
}

vdc_status vdc_model_destroy(vdc_model_t m) {
  if (!m) return VDC_OK;
  if (m->d_nodes) (void)hipFree(m->d_nodes);
  if (m->d_coef) (void)hipFree(m->d_coef);
  if (m->d_coefx) (void)hipFree(m->d_coefx);
  if (m->d_clus) (void)hipFree(m->d_clus);
  delete m->gen;
  delete m;
  return VDC_OK;
}

vdc_status vdc_workspace_size(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                              int n_jobs, const vdc_job* jobs, size_t* bytes) {
  if (!bytes) return fail(VDC_ERR_INVALID_ARG, "bytes is NULL");
  // size for the larger of the two paths so one workspace serves both
  Plan P;
  vdc_status st = make_plan(n_models, models, opts, n_jobs, jobs, kMaxFinal, false, P);
  if (st != VDC_OK) return st;
  size_t total = P.total;
  if (opts->precision == VDC_FP64 && opts->method == VDC_GMRES) {
    Plan Q;
    st = make_plan(n_models, models, opts, n_jobs, jobs, kMaxFinal, true, Q);
    if (st != VDC_OK) return st;
    total = std::max(total, Q.total);
  }
  *bytes = total;
  return VDC_OK;
}

vdc_status vdc_solve(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                     int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                     void* workspace, size_t ws_bytes, double* T_out, double* sigma_out,
                     double* psi_out, vdc_job_info* info, void* stream) {
  const bool mixed = opts && opts->precision == VDC_FP32_INNER;
  std::vector<vdc_job_info> own;
  if (mixed && !info && n_jobs > 0) {
    own.resize(n_jobs);
    info = own.data();
  }
  const vdc_status st = run_solve(n_models, models, opts, n_jobs, jobs, n_final, finals, workspace,
                                  ws_bytes, T_out, sigma_out, psi_out, info, stream, false);
  if (st != VDC_OK || !mixed || n_jobs == 0) return st;
  return retry_fp64(n_models, models, opts, n_jobs, jobs, n_final, finals, workspace, ws_bytes,
                    T_out, sigma_out, psi_out, info, stream);
}

vdc_status vdc_solve_history(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                             int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                             void* workspace, size_t ws_bytes, double* T_out, double* sigma_out,
                             double* psi_out, vdc_job_info* info, double* hist, int hist_len,
                             void* stream) {
  if (!hist || hist_len < 1) return fail(VDC_ERR_INVALID_ARG, "hist must be non-NULL, hist_len >= 1");
  PlanExtra ex;
  ex.hist = hist;
  ex.hist_len = hist_len;
  return run_solve(n_models, models, opts, n_jobs, jobs, n_final, finals, workspace, ws_bytes,
                   T_out, sigma_out, psi_out, info, stream, false, nullptr, &ex);
}

vdc_status vdc_solve_noalloc(int n_models, const vdc_model_t* models,
                             const vdc_solve_opts* opts, int n_jobs, const vdc_job* jobs,
                             int n_final, const int* finals, double* T_out, double* sigma_out,
                             double* psi_out, vdc_job_info* info, void* stream) {
  const size_t cap = VDC_NOALLOC_SCRATCH_BYTES;
  Plan P;
  vdc_status st = make_plan(n_models, models, opts, n_jobs, jobs, n_final, false, P);
  if (st != VDC_OK || n_jobs == 0) return st;
  PlanExtra ex;
  ex.untimed = true;
  if (P.total > cap) {
    // fewer resident workgroups (slots) until the plan fits, if one does
    const size_t slot = sizeof(c64) * P.slot_elems;
    const size_t fixed = P.off_scratch + 256;
    if (fixed + slot > cap)
      return fail(VDC_ERR_WORKSPACE,
                  "vdc_solve_noalloc: this call needs " + std::to_string(fixed + slot) +
                      " bytes of device scratch with one resident workgroup, more than the " +
                      std::to_string(cap) + " bytes the library holds; use vdc_solve");
    ex.max_groups = (int)std::min<size_t>((cap - fixed) / slot, (size_t)P.n_groups);
  }
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st != VDC_OK) return st;
  const bool mixed = opts->precision == VDC_FP32_INNER;
  std::vector<vdc_job_info> own;
  if (mixed && !info) {
    own.resize(n_jobs);
    info = own.data();
  }
  st = run_solve(n_models, models, opts, n_jobs, jobs, n_final, finals, ws, cap, T_out, sigma_out,
                 psi_out, info, stream, false, nullptr, &ex);
  if (st != VDC_OK || !mixed) return st;
  return retry_fp64(n_models, models, opts, n_jobs, jobs, n_final, finals, ws, cap, T_out,
                    sigma_out, psi_out, info, stream, true);
}

vdc_status vdc_batch_create(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                            int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                            void* workspace, size_t ws_bytes, double* T_out, double* sigma_out,
                            double* psi_out, void* stream, vdc_batch_t* out) {
  if (!out) return fail(VDC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_jobs < 1) return fail(VDC_ERR_INVALID_ARG, "a batch needs at least one job");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  vdc_batch* b = new vdc_batch();
  vdc_status st = prepare_solve(n_models, models, opts, n_jobs, jobs, n_final, finals, workspace,
                                ws_bytes, T_out, sigma_out, psi_out, s, false, nullptr, b->R);
  if (st == VDC_OK && hipStreamSynchronize(s) != hipSuccess)
    st = fail(VDC_ERR_HIP, "batch upload failed");
  if (st != VDC_OK) {
    delete b;
    return st;
  }
  *out = b;
  return VDC_OK;
}

vdc_status vdc_batch_launch(vdc_batch_t b, void* stream) {
  if (!b) return fail(VDC_ERR_INVALID_ARG, "NULL batch");
  const vdc_status st =
      enqueue_solve(b->R, reinterpret_cast<hipStream_t>(stream), b->ev.ok ? &b->ev : nullptr);
  b->timed = st == VDC_OK && b->ev.ok;
  return st;
}

vdc_status vdc_batch_kernel_times(vdc_batch_t b, double* ms_tables, double* ms_solver) {
  if (!b) return fail(VDC_ERR_INVALID_ARG, "NULL batch");
  if (!b->timed) return fail(VDC_ERR_INVALID_ARG, "no timed launch: call vdc_batch_launch first");
  HIPCHK(hipEventSynchronize(b->ev.e[2]));
  float t1 = 0.f, t2 = 0.f;
  HIPCHK(hipEventElapsedTime(&t1, b->ev.e[0], b->ev.e[1]));
  HIPCHK(hipEventElapsedTime(&t2, b->ev.e[1], b->ev.e[2]));
  if (ms_tables) *ms_tables = t1;
  if (ms_solver) *ms_solver = t2;
  return VDC_OK;
}

vdc_status vdc_batch_capture(vdc_batch_t b, void* stream) {
  if (!b) return fail(VDC_ERR_INVALID_ARG, "NULL batch");
  if (!stream) return fail(VDC_ERR_INVALID_ARG, "capture needs a stream other than the null stream");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  b->drop_graph();
  HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const vdc_status st = enqueue_solve(b->R, s, nullptr);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (st != VDC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  b->graph = g;
  const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    b->drop_graph();
    return hip_fail(ei, "hipGraphInstantiate");
  }
  return VDC_OK;
}

vdc_status vdc_batch_replay(vdc_batch_t b, void* stream) {
  if (!b) return fail(VDC_ERR_INVALID_ARG, "NULL batch");
  if (!b->exec) return fail(VDC_ERR_INVALID_ARG, "no captured graph: call vdc_batch_capture first");
  HIPCHK(hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream)));
  return VDC_OK;
}

vdc_status vdc_batch_info(vdc_batch_t b, vdc_job_info* info, void* stream) {
  if (!b) return fail(VDC_ERR_INVALID_ARG, "NULL batch");
  return read_info(b->R, info, reinterpret_cast<hipStream_t>(stream));
}

vdc_status vdc_batch_destroy(vdc_batch_t b) {
  if (!b) return VDC_OK;
  b->drop_graph();
  delete b;
  return VDC_OK;
}

vdc_status vdc_solve_plain(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                           int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                           void* workspace, size_t ws_bytes, double* T_out, double* sigma_out,
                           double* psi_out, vdc_job_info* info, void* stream) {
  return run_solve(n_models, models, opts, n_jobs, jobs, n_final, finals, workspace, ws_bytes,
                   T_out, sigma_out, psi_out, info, stream, true);
}

vdc_status vdc_adjoint_workspace_size(int n_models, const vdc_model_t* models,
                                      const vdc_solve_opts* opts, int n_jobs,
                                      const vdc_job* jobs, size_t* bytes) {
  if (!bytes) return fail(VDC_ERR_INVALID_ARG, "bytes is NULL");
  Plan P;
  vdc_status st = make_plan(n_models, models, opts, n_jobs, jobs, kMaxFinal, false, P, true);
  if (st != VDC_OK) return st;
  *bytes = P.total;
  return VDC_OK;
}

vdc_status vdc_solve_adjoint(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                             int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                             const double* psi, const double* T, const double* dL_dsigma,
                             void* workspace, size_t ws_bytes, double* grad_jobs, double* grad,
                             vdc_job_info* info, void* stream) {
  AdjointIO io{psi, T, dL_dsigma, grad_jobs, grad};
  return run_solve(n_models, models, opts, n_jobs, jobs, n_final, finals, workspace, ws_bytes,
                   nullptr, nullptr, nullptr, info, stream, false, &io);
}

vdc_status vdc_level_shift(vdc_model_t m, int n_eps, const double* eps, double* out, void* stream) {
  if (!m) return fail(VDC_ERR_INVALID_ARG, "NULL model");
  if (m->kind != 0) return fail(VDC_ERR_INVALID_ARG, "a model built from term lists without the two-state form");
  if (n_eps < 0) return fail(VDC_ERR_INVALID_ARG, "n_eps < 0");
  if (n_eps == 0) return VDC_OK;
  if (!eps || !out) return fail(VDC_ERR_INVALID_ARG, "NULL buffer");
  HIPCHK(launch_level_shift_points(m->dev, n_eps, eps, reinterpret_cast<c64*>(out),
                                   reinterpret_cast<hipStream_t>(stream)));
  return VDC_OK;
}

static size_t matvec_ws(const vdc_model* m, int n_vec) {
  const size_t Nc = (size_t)m->dev.Nc;
  size_t off = 0;
  off = align256(off + sizeof(DevModel));
  off = align256(off + sizeof(DevTable));
  off = align256(off + sizeof(DevGroup));
  off = align256(off + sizeof(int) * Nc);
  off = align256(off + sizeof(c64) * kNumF * Nc);
  off = align256(off + sizeof(int) * std::max(1, n_vec));
  off = align256(off + sizeof(c64) * 6 * Nc);
  off = align256(off + sizeof(c64) * 4 * Nc * std::max(1, n_vec));
  return off;
}

vdc_status vdc_matvec_workspace_size(vdc_model_t m, int n_vec, size_t* bytes) {
  if (!m || !bytes || n_vec < 0) return fail(VDC_ERR_INVALID_ARG, "bad argument");
  if (m->kind != 0) return fail(VDC_ERR_INVALID_ARG, "a model built from term lists without the two-state form");
  *bytes = matvec_ws(m, n_vec);
  return VDC_OK;
}

// Batched operator on block vectors (the solvers' layout); tables for E are
// built into the workspace first, then one strip sweep per (vector, slab,
// strip).
static size_t matvec_block_ws(const vdc_model* m) {
  const size_t Nc = (size_t)m->dev.Nc;
  size_t off = 0;
  off = align256(off + sizeof(DevModel));
  off = align256(off + sizeof(DevTable));
  off = align256(off + sizeof(DevGroup));
  off = align256(off + sizeof(int) * Nc);
  off = align256(off + sizeof(c64) * kNumF * Nc);   // shift table
  off = align256(off + sizeof(c64) * 6 * Nc);       // block tables
  return off;
}

// Rows per slab: enough wavefronts to fill the chip several times over
// (about 16 per CU), but slabs of at least 8 rows so that the two halo rows
// re-read at each slab edge stay a small overhead.
static int strip_slab_rows(int Ng, int Nu, int n_vec) {
  const long columns = (long)n_vec * strip_count(Nu);
  const long want = 16L * cu_count();
  long slabs = (want + columns - 1) / columns;
  slabs = std::max(1L, std::min<long>(slabs, Ng / 8 > 0 ? Ng / 8 : 1));
  return (int)((Ng + slabs - 1) / slabs);
}

vdc_status vdc_matvec_block_workspace_size(vdc_model_t m, int n_vec, size_t* bytes) {
  if (!m || !bytes || n_vec < 0) return fail(VDC_ERR_INVALID_ARG, "bad argument");
  if (m->kind != 0) return fail(VDC_ERR_INVALID_ARG, "a model built from term lists without the two-state form");
  *bytes = matvec_block_ws(m) + align256(sizeof(int) * std::max(1, n_vec));
  return VDC_OK;
}

vdc_status vdc_matvec_block(vdc_model_t m, double E, int n_vec, const int* parity,
                            const double* x, double* y, void* workspace, size_t ws_bytes,
                            void* stream) {
  if (!m) return fail(VDC_ERR_INVALID_ARG, "NULL model");
  if (m->kind != 0) return fail(VDC_ERR_INVALID_ARG, "a model built from term lists without the two-state form");
  if (n_vec < 0 || !std::isfinite(E)) return fail(VDC_ERR_INVALID_ARG, "bad n_vec or E");
  if (n_vec == 0) return VDC_OK;
  if (!parity || !x || !y || !workspace) return fail(VDC_ERR_INVALID_ARG, "NULL buffer");
  for (int v = 0; v < n_vec; ++v)
    if (parity[v] != 0 && parity[v] != 1) return fail(VDC_ERR_INVALID_ARG, "parity must be 0 or 1");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(VDC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  const size_t need = matvec_block_ws(m) + align256(sizeof(int) * n_vec);
  if (ws_bytes < need) return fail(VDC_ERR_WORKSPACE, "workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t Nc = (size_t)m->dev.Nc;
  char* ws = static_cast<char*>(workspace);
  size_t off = 0;
  DevModel* dmod = reinterpret_cast<DevModel*>(ws + off); off = align256(off + sizeof(DevModel));
  DevTable* dtab = reinterpret_cast<DevTable*>(ws + off); off = align256(off + sizeof(DevTable));
  DevGroup* dgrp = reinterpret_cast<DevGroup*>(ws + off); off = align256(off + sizeof(DevGroup));
  int* dperm = reinterpret_cast<int*>(ws + off); off = align256(off + sizeof(int) * Nc);
  c64* shift = reinterpret_cast<c64*>(ws + off); off = align256(off + sizeof(c64) * kNumF * Nc);
  c64* tables = reinterpret_cast<c64*>(ws + off); off = align256(off + sizeof(c64) * 6 * Nc);
  int* dpar = reinterpret_cast<int*>(ws + off);
  DevGroup g{};
  g.eps_i = E - 0.5 * (m->dev.omega_g + m->dev.omega_u);
  g.a_min = -(m->dev.Ng - 1);
  g.na = m->dev.Ng;
  g.b_min = -(m->dev.Nu - 1);
  g.nb = m->dev.Nu;
  DevTable t{};
  t.E = E;
  std::vector<std::pair<double, int>> key(Nc);
  for (int ia = 0; ia < g.na; ++ia)
    for (int ib = 0; ib < g.nb; ++ib)
      key[ia * g.nb + ib] = std::make_pair(m->dev.omega_g * ia + m->dev.omega_u * ib, ia * g.nb + ib);
  std::sort(key.begin(), key.end());
  std::vector<int> hperm(Nc);
  for (size_t q = 0; q < Nc; ++q) hperm[q] = key[q].second;
  HIPCHK(hipMemcpyAsync(dmod, &m->dev, sizeof(DevModel), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dtab, &t, sizeof(DevTable), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dgrp, &g, sizeof(DevGroup), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dperm, hperm.data(), sizeof(int) * Nc, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dpar, parity, sizeof(int) * n_vec, hipMemcpyHostToDevice, s));
  EventSet ev;
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[0], s));
  HIPCHK(launch_level_shift_tables(dmod, dgrp, 1, m->dev.Nc, dperm, dtab, 1, m->dev.Nc, shift,
                                   tables, nullptr, s));
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[1], s));
  const int S = strip_slab_rows(m->dev.Ng, m->dev.Nu, n_vec);
  HIPCHK(launch_matvec_strip(dmod, dtab, tables, dpar, n_vec, reinterpret_cast<const c64*>(x),
                             reinterpret_cast<c64*>(y), m->dev.Ng, m->dev.Nu, S, s));
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[2], s));
  HIPCHK(hipStreamSynchronize(s));
  if (ev.ok) {
    float t1 = 0.f, t2 = 0.f;
    HIPCHK(hipEventElapsedTime(&t1, ev.e[0], ev.e[1]));
    HIPCHK(hipEventElapsedTime(&t2, ev.e[1], ev.e[2]));
    g_ms_tables = t1;
    g_ms_solver = t2;
  }
  return VDC_OK;
}

vdc_status vdc_matvec(vdc_model_t m, double E, int n_vec, const int* parity, const double* x,
                      double* y, void* workspace, size_t ws_bytes, void* stream) {
  if (!m) return fail(VDC_ERR_INVALID_ARG, "NULL model");
  if (m->kind != 0) return fail(VDC_ERR_INVALID_ARG, "a model built from term lists without the two-state form");
  if (n_vec < 0 || !std::isfinite(E)) return fail(VDC_ERR_INVALID_ARG, "bad n_vec or E");
  if (n_vec == 0) return VDC_OK;
  if (!parity || !x || !y || !workspace) return fail(VDC_ERR_INVALID_ARG, "NULL buffer");
  for (int v = 0; v < n_vec; ++v)
    if (parity[v] != 0 && parity[v] != 1) return fail(VDC_ERR_INVALID_ARG, "parity must be 0 or 1");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(VDC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < matvec_ws(m, n_vec)) return fail(VDC_ERR_WORKSPACE, "workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t Nc = (size_t)m->dev.Nc;
  char* ws = static_cast<char*>(workspace);
  size_t off = 0;
  DevModel* dmod = reinterpret_cast<DevModel*>(ws + off); off = align256(off + sizeof(DevModel));
  DevTable* dtab = reinterpret_cast<DevTable*>(ws + off); off = align256(off + sizeof(DevTable));
  DevGroup* dgrp = reinterpret_cast<DevGroup*>(ws + off); off = align256(off + sizeof(DevGroup));
  int* dperm = reinterpret_cast<int*>(ws + off); off = align256(off + sizeof(int) * Nc);
  c64* shift = reinterpret_cast<c64*>(ws + off); off = align256(off + sizeof(c64) * kNumF * Nc);
  int* dpar = reinterpret_cast<int*>(ws + off); off = align256(off + sizeof(int) * n_vec);
  c64* tables = reinterpret_cast<c64*>(ws + off); off = align256(off + sizeof(c64) * 6 * Nc);
  c64* z = reinterpret_cast<c64*>(ws + off);
  c64* yc = z + Nc * n_vec;
  c64* wA = yc + Nc * n_vec;
  c64* wB = wA + Nc * n_vec;
  // one energy: a shift table over offsets a = -n_g, b = -n_u at
  // eps = E - (w_g + w_u)/2 + w_g a + w_u b = E - E_nu, read with v = (0, 0)
  DevGroup g{};
  g.eps_i = E - 0.5 * (m->dev.omega_g + m->dev.omega_u);
  g.model = 0;
  g.a_min = -(m->dev.Ng - 1);
  g.na = m->dev.Ng;
  g.b_min = -(m->dev.Nu - 1);
  g.nb = m->dev.Nu;
  g.perm_off = 0;
  g.offset = 0;
  std::vector<std::pair<double, int>> key(Nc);
  for (int ia = 0; ia < g.na; ++ia)
    for (int ib = 0; ib < g.nb; ++ib)
      key[ia * g.nb + ib] = std::make_pair(m->dev.omega_g * ia + m->dev.omega_u * ib, ia * g.nb + ib);
  std::sort(key.begin(), key.end());
  std::vector<int> hperm(Nc);
  for (size_t q = 0; q < Nc; ++q) hperm[q] = key[q].second;
  DevTable t{};
  t.E = E;
  t.model = 0;
  t.group = 0;
  t.vg = 0;
  t.vu = 0;
  t.offset = 0;
  HIPCHK(hipMemcpyAsync(dmod, &m->dev, sizeof(DevModel), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dtab, &t, sizeof(DevTable), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dgrp, &g, sizeof(DevGroup), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dperm, hperm.data(), sizeof(int) * Nc, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dpar, parity, sizeof(int) * n_vec, hipMemcpyHostToDevice, s));
  HIPCHK(launch_level_shift_tables(dmod, dgrp, 1, m->dev.Nc, dperm, dtab, 1, m->dev.Nc, shift,
                                   tables, nullptr, s));
  HIPCHK(launch_matvec_full(dmod, dtab, tables, n_vec, dpar, reinterpret_cast<const c64*>(x),
                            reinterpret_cast<c64*>(y), z, yc, wA, wB, m->dev.Nc, s));
  // the host-side staging buffers above are read by the copies before return
  HIPCHK(hipStreamSynchronize(s));
  return VDC_OK;
}

// 2D electron energy-loss spectra (Eq. (17)) from full-layout solutions.
namespace {
size_t eels_groups(int n_jobs) { return (size_t)std::max(1, std::min(n_jobs, cu_count())); }
}  // namespace

vdc_status vdc_eels_workspace_size(vdc_model_t model, int n_jobs, size_t* bytes) {
  if (!model || !bytes || n_jobs < 0) return fail(VDC_ERR_INVALID_ARG, "bad argument");
  if (model->kind != 0) return fail(VDC_ERR_INVALID_ARG, "a model built from term lists without the two-state form");
  const int Nc = model->dev.Nc;
  size_t off = 0;
  off = align256(off + sizeof(DevModel));
  off = align256(off + sizeof(EelsJob) * std::max(1, n_jobs));
  off = align256(off + sizeof(int) * Nc);
  off = align256(off + sizeof(double) * Nc);
  off = align256(off + sizeof(int));
  off = align256(off + sizeof(double) * Nc * eels_groups(n_jobs));
  *bytes = off;
  return VDC_OK;
}

vdc_status vdc_eels(vdc_model_t model, int n_jobs, const vdc_job* jobs, const double* psi,
                    size_t psi_ld, int n_grid, double loss0, double dloss, double fwhm,
                    double* S_out, void* workspace, size_t ws_bytes, void* stream) {
  size_t need = 0;
  vdc_status st = vdc_eels_workspace_size(model, n_jobs, &need);
  if (st != VDC_OK) return st;
  if (n_jobs == 0) return VDC_OK;
  const DevModel& md = model->dev;
  if (!jobs || !psi || !S_out || !workspace) return fail(VDC_ERR_INVALID_ARG, "NULL buffer");
  if (n_grid < 1) return fail(VDC_ERR_INVALID_ARG, "n_grid must be >= 1");
  if (!(fwhm > 0.0) || !(dloss > 0.0) || !std::isfinite(loss0) || !std::isfinite(fwhm) ||
      !std::isfinite(dloss))
    return fail(VDC_ERR_INVALID_ARG, "fwhm and dloss must be > 0, loss0 finite");
  if (psi_ld < 2 * (size_t)md.Nc) return fail(VDC_ERR_INVALID_ARG, "psi_ld must be >= 2 Ng Nu");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(VDC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < need) return fail(VDC_ERR_WORKSPACE, "workspace too small");
  std::vector<EelsJob> ej(n_jobs);
  for (int k = 0; k < n_jobs; ++k) {
    const vdc_job& j = jobs[k];
    if (!(j.eps_i > 0.0) || !std::isfinite(j.eps_i)) return fail(VDC_ERR_INVALID_ARG, "eps_i must be > 0");
    if (j.vi_g < 0 || j.vi_g >= md.Ng || j.vi_u < 0 || j.vi_u >= md.Nu)
      return fail(VDC_ERR_INVALID_ARG, "initial state outside the basis");
    if (j.model != 0) return fail(VDC_ERR_INVALID_ARG, "jobs of vdc_eels refer to its one model (0)");
    const double Evi = md.omega_g * (j.vi_g + 0.5) + md.omega_u * (j.vi_u + 0.5);
    ej[k] = EelsJob{j.eps_i, j.eps_i + Evi, Evi, k};
  }
  // final states by vibrational energy (ties by index)
  std::vector<int> order(md.Nc);
  std::vector<double> Evf(md.Nc);
  for (int q = 0; q < md.Nc; ++q) order[q] = q;
  auto energy = [&](int q) {
    const int g = q / md.Nu, u = q - g * md.Nu;
    return md.omega_g * (g + 0.5) + md.omega_u * (u + 0.5);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return energy(a) < energy(b); });
  for (int q = 0; q < md.Nc; ++q) Evf[q] = energy(order[q]);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  size_t off = 0;
  DevModel* d_model = reinterpret_cast<DevModel*>(ws + off); off = align256(off + sizeof(DevModel));
  EelsJob* d_jobs = reinterpret_cast<EelsJob*>(ws + off); off = align256(off + sizeof(EelsJob) * n_jobs);
  int* d_order = reinterpret_cast<int*>(ws + off); off = align256(off + sizeof(int) * md.Nc);
  double* d_Evf = reinterpret_cast<double*>(ws + off); off = align256(off + sizeof(double) * md.Nc);
  int* d_counter = reinterpret_cast<int*>(ws + off); off = align256(off + sizeof(int));
  double* d_share = reinterpret_cast<double*>(ws + off);
  HIPCHK(hipMemcpyAsync(d_model, &md, sizeof(DevModel), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d_jobs, ej.data(), sizeof(EelsJob) * n_jobs, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d_order, order.data(), sizeof(int) * md.Nc, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d_Evf, Evf.data(), sizeof(double) * md.Nc, hipMemcpyHostToDevice, s));
  HIPCHK(launch_zero_int(d_counter, 1, s));
  EelsArgs a{};
  a.model = d_model;
  a.jobs = d_jobs;
  a.n_jobs = n_jobs;
  a.psi = reinterpret_cast<const c64*>(psi);
  a.psi_ld = psi_ld;
  a.order = d_order;
  a.Evf = d_Evf;
  a.share = d_share;
  a.counter = d_counter;
  a.n_grid = n_grid;
  a.d0 = loss0;
  a.dd = dloss;
  a.fwhm = fwhm;
  a.S = S_out;
  EventSet ev;
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[0], s));
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[1], s));
  HIPCHK(launch_eels(a, (int)eels_groups(n_jobs), s));
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[2], s));
  HIPCHK(hipStreamSynchronize(s));
  if (ev.ok) {
    float t2 = 0.f;
    HIPCHK(hipEventElapsedTime(&t2, ev.e[1], ev.e[2]));
    g_ms_tables = 0.f;
    g_ms_solver = t2;
  }
  return VDC_OK;
}

}  // extern "C"


// ------------------------------------------------------------------ CO2-like model


struct vdc_co2 {
  vdc_co2_desc desc;
  Co2Model dev;
  vdc_model_t ls = nullptr;   // the six level-shift functions (state classes x wave classes)
};

namespace {

double co2_vib(const Co2Model& m, int s, int b, int a) {
  return m.omega_s * (s + 0.5) + m.omega_b * (b + 1.0) + m.omega_a * (a + 0.5);
}

size_t co2_ld(const Co2Model& m) { return ((size_t)m.npts + 63) / 64 * 64; }

// Bytes of one job's block factor (Co2FacLayout)
size_t co2_fac_bytes(const Co2Model& m) {
  return co2_fac_layout(m.Ns * m.Na, m.Nx * m.Ny, 2 * m.Ny + 1).total;
}

struct Co2Plan {
  std::vector<Co2Job> jobs;
  std::vector<double> energies;
  size_t ld = 0, slot_elems = 0, fac_job_bytes = 0;
  int n_groups = 1, m = 0;
  size_t off_model = 0, off_ls = 0, off_jobs = 0, off_eps = 0, off_tab = 0, off_counter = 0,
         off_finals = 0, off_info = 0, off_fac = 0, off_scratch = 0, total = 0;
};

vdc_status co2_plan(vdc_co2_t model, const vdc_solve_opts* o, int n_jobs, const vdc_co2_job* jobs,
                    int n_final, Co2Plan& P) {
  if (!model || !o) return fail(VDC_ERR_INVALID_ARG, "NULL model or opts");
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(VDC_ERR_INVALID_ARG, "bad job list");
  if (n_final < 0 || n_final > kMaxFinal) return fail(VDC_ERR_INVALID_ARG, "n_final must be 0..64");
  if (o->restart < 1 || o->restart > kMaxRestart) return fail(VDC_ERR_INVALID_ARG, "restart must be 1..128");
  if (o->max_iter < 1) return fail(VDC_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (!(o->tol > 0.0)) return fail(VDC_ERR_INVALID_ARG, "tol must be > 0");
  if (o->precision != VDC_FP64) return fail(VDC_ERR_INVALID_ARG, "this model solves in FP64 only");
  if (o->precond == VDC_PREC_ROWS)
    return fail(VDC_ERR_UNSUPPORTED, "row blocks are the two-state model's M^g; use VDC_PREC_BLOCK here");
  if (o->precond != VDC_PREC_NONE && o->precond != VDC_PREC_JACOBI && o->precond != VDC_PREC_BLOCK)
    return fail(VDC_ERR_INVALID_ARG, "unknown preconditioner");
  if (o->method != VDC_GMRES && o->method != VDC_COCG)
    return fail(VDC_ERR_INVALID_ARG, "unknown method");
  const Co2Model& md = model->dev;
  if (o->precond == VDC_PREC_BLOCK && md.Ny > co2_factor_max_ny())
    return fail(VDC_ERR_UNSUPPORTED, "the block preconditioner needs Ny <= 24");
  std::map<double, int> eidx;
  for (int k = 0; k < n_jobs; ++k) {
    const vdc_co2_job& j = jobs[k];
    if (!(j.eps_i > 0.0) || !std::isfinite(j.eps_i)) return fail(VDC_ERR_INVALID_ARG, "eps_i must be > 0");
    const int lim[4] = {md.Ns, md.Nx, md.Ny, md.Na};
    for (int q = 0; q < 4; ++q)
      if (j.v[q] < 0 || j.v[q] >= lim[q]) return fail(VDC_ERR_INVALID_ARG, "initial state outside the basis");
    if (j.mu_i < 0 || j.mu_i > 2) return fail(VDC_ERR_INVALID_ARG, "mu_i must be 0, 1 or 2");
    Co2Job c{};
    c.eps_i = j.eps_i;
    c.E = j.eps_i + co2_vib(md, j.v[0], j.v[1] + j.v[2], j.v[3]);
    for (int q = 0; q < 4; ++q) c.v[q] = j.v[q];
    c.mu = j.mu_i;
    c.px = co2_sector_x(j.v, j.mu_i);
    c.py = co2_sector_y(j.v, j.mu_i);
    auto it = eidx.find(c.E);
    if (it == eidx.end()) it = eidx.emplace(c.E, (int)eidx.size()).first;
    c.table = it->second;
    c.out = k;
    P.jobs.push_back(c);
  }
  P.energies.assign(eidx.size(), 0.0);
  for (auto& kv : eidx) P.energies[kv.second] = kv.first;
  // higher energies first (more open channels, longer solves on these models)
  std::stable_sort(P.jobs.begin(), P.jobs.end(),
                   [](const Co2Job& a, const Co2Job& b) { return a.E > b.E; });
  P.m = o->method == VDC_COCG ? 4 : o->restart;   // COCG keeps r, p, q, z in V_0..V_3
  P.ld = co2_ld(md);
  P.slot_elems = ((size_t)(P.m + 1 + 6) * P.ld + (size_t)(P.m + 1) * P.m + 31) / 32 * 32;
  P.fac_job_bytes = o->precond == VDC_PREC_BLOCK ? co2_fac_bytes(md) : 0;
  P.n_groups = std::max(1, std::min(n_jobs, cu_count()));
  size_t off = 0;
  P.off_model = off; off = align256(off + sizeof(Co2Model));
  P.off_ls = off; off = align256(off + sizeof(DevModel));
  P.off_jobs = off; off = align256(off + sizeof(Co2Job) * std::max(1, n_jobs));
  P.off_eps = off; off = align256(off + sizeof(double) * std::max<size_t>(1, P.energies.size()) * md.ntab);
  P.off_tab = off; off = align256(off + sizeof(c64) * kNumF * std::max<size_t>(1, P.energies.size()) * md.ntab);
  P.off_counter = off; off = align256(off + sizeof(int));
  P.off_finals = off; off = align256(off + sizeof(int) * 4 * std::max(1, n_final));
  P.off_info = off; off = align256(off + sizeof(DevInfo) * std::max(1, n_jobs));
  P.off_fac = off; off = align256(off + P.fac_job_bytes * n_jobs);
  P.off_scratch = off; off = align256(off + sizeof(c64) * P.slot_elems * P.n_groups);
  P.total = off;
  return VDC_OK;
}

// Level-shift rows of every distinct energy: eps = E - E_nu for each
// (n_s, n_x + n_y, n_a), the six functions at each.
vdc_status co2_tables(vdc_co2_t model, const std::vector<double>& energies, double* d_eps, c64* d_tab,
                      hipStream_t s) {
  const Co2Model& md = model->dev;
  std::vector<double> eps(energies.size() * (size_t)md.ntab);
  for (size_t e = 0; e < energies.size(); ++e)
    for (int si = 0; si < md.Ns; ++si)
      for (int b = 0; b < md.nb; ++b)
        for (int a = 0; a < md.Na; ++a)
          eps[e * md.ntab + ((size_t)si * md.nb + b) * md.Na + a] = energies[e] - co2_vib(md, si, b, a);
  if (eps.empty()) return VDC_OK;
  HIPCHK(hipMemcpyAsync(d_eps, eps.data(), sizeof(double) * eps.size(), hipMemcpyHostToDevice, s));
  HIPCHK(launch_level_shift_points(model->ls->dev, (int)eps.size(), d_eps, d_tab, s));
  return VDC_OK;
}

}  // namespace

vdc_status vdc_co2_create(const vdc_co2_desc* d, vdc_co2_t* out) {
  if (!d || !out) return fail(VDC_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  const int sz[4] = {d->Ns, d->Nx, d->Ny, d->Na};
  for (int v : sz)
    if (v < 1 || v > kSqMax - 2) return fail(VDC_ERR_INVALID_ARG, "basis sizes must be 1..1022");
  if (d->Ny > 31) return fail(VDC_ERR_INVALID_ARG, "Ny must be <= 31 (band of the bend blocks)");
  if ((size_t)d->Ns * d->Nx * d->Ny * d->Na > (size_t)1 << 26)
    return fail(VDC_ERR_INVALID_ARG, "basis too large");
  const double scal[] = {d->omega_s, d->omega_b, d->omega_a, d->E_sigma, d->E_pi, d->k_sigma,
                         d->k_pi, d->gs_sigma, d->gb_sigma, d->ga_sigma, d->gs_pi, d->gb_pi,
                         d->ga_pi, d->c_rt, d->c_sp, d->c_sp2, d->l_sigma, d->l_pi, d->h_sigma,
                         d->h_pi};
  for (double v : scal)
    if (!std::isfinite(v)) return fail(VDC_ERR_INVALID_ARG, "non-finite model parameter");
  if (!(d->omega_s > 0.0) || !(d->omega_b > 0.0) || !(d->omega_a > 0.0))
    return fail(VDC_ERR_INVALID_ARG, "vibrational frequencies must be > 0");
  // the level-shift functions through a two-state descriptor: "state" d =
  // state class (sigma, pi), "partial wave" mu = wave class (s, p)
  vdc_model2d_desc ld{};
  ld.omega_g = d->omega_s;
  ld.omega_u = d->omega_b;
  ld.E1 = d->E_sigma;
  ld.gap = d->E_pi - d->E_sigma;
  for (int c = 0; c < 2; ++c)
    for (int w = 0; w < 2; ++w) {
      ld.A[c][w] = d->A[c][w];
      ld.B[c][w] = d->B[c][w];
    }
  ld.l[0] = 0;
  ld.l[1] = 1;
  ld.Ng = ld.Nu = 1;
  ld.hilbert_nodes = d->hilbert_nodes;
  ld.hilbert_xmax = d->hilbert_xmax;
  vdc_model_t lsm = nullptr;
  const vdc_status st = vdc_model2d_create(&ld, &lsm);
  if (st != VDC_OK) return st;
  vdc_co2* m = new vdc_co2();
  m->desc = *d;
  m->ls = lsm;
  Co2Model& c = m->dev;
  c.Ns = d->Ns;
  c.Nx = d->Nx;
  c.Ny = d->Ny;
  c.Na = d->Na;
  c.npts = d->Ns * d->Na * d->Nx * d->Ny;
  c.nb = d->Nx + d->Ny - 1;
  c.ntab = d->Ns * c.nb * d->Na;
  c.omega_s = d->omega_s;
  c.omega_b = d->omega_b;
  c.omega_a = d->omega_a;
  c.E_sigma = d->E_sigma;
  c.E_pi = d->E_pi;
  c.k_sigma = d->k_sigma;
  c.k_pi = d->k_pi;
  c.gs[0] = d->gs_sigma;
  c.gb[0] = d->gb_sigma;
  c.ga[0] = d->ga_sigma;
  c.gs[1] = d->gs_pi;
  c.gb[1] = d->gb_pi;
  c.ga[1] = d->ga_pi;
  c.c_rt = d->c_rt;
  c.c_sp = d->c_sp;
  c.c_sp2 = d->c_sp2;
  c.l_sigma = d->l_sigma;
  c.l_pi = d->l_pi;
  c.h_sigma = d->h_sigma;
  c.h_pi = d->h_pi;
  *out = m;
  return VDC_OK;
}

vdc_status vdc_co2_destroy(vdc_co2_t m) {
  if (!m) return VDC_OK;
  vdc_model_destroy(m->ls);
  delete m;
  return VDC_OK;
}

vdc_status vdc_co2_workspace_size(vdc_co2_t model, const vdc_solve_opts* opts, int n_jobs,
                                  const vdc_co2_job* jobs, size_t* bytes) {
  if (!bytes) return fail(VDC_ERR_INVALID_ARG, "NULL bytes");
  Co2Plan P;
  const vdc_status st = co2_plan(model, opts, n_jobs, jobs, 0, P);
  if (st != VDC_OK) return st;
  *bytes = P.total + align256(sizeof(int) * 4 * kMaxFinal);
  return VDC_OK;
}

vdc_status vdc_co2_solve(vdc_co2_t model, const vdc_solve_opts* opts, int n_jobs,
                         const vdc_co2_job* jobs, int n_final, const int* finals, double* T_out,
                         double* sigma_out, double* psi_out, vdc_job_info* info, void* workspace,
                         size_t ws_bytes, void* stream) {
  Co2Plan P;
  vdc_status st = co2_plan(model, opts, n_jobs, jobs, n_final, P);
  if (st != VDC_OK) return st;
  if (n_jobs == 0) return VDC_OK;
  if (!T_out || !sigma_out || !info || !workspace || (n_final > 0 && !finals))
    return fail(VDC_ERR_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(VDC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < P.total) return fail(VDC_ERR_WORKSPACE, "workspace too small");
  const Co2Model& md = model->dev;
  for (int f = 0; f < n_final; ++f) {
    const int lim[4] = {md.Ns, md.Nx, md.Ny, md.Na};
    for (int q = 0; q < 4; ++q)
      if (finals[4 * f + q] < 0 || finals[4 * f + q] >= lim[q])
        return fail(VDC_ERR_INVALID_ARG, "final state outside the basis");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  Co2Model* d_model = reinterpret_cast<Co2Model*>(ws + P.off_model);
  DevModel* d_ls = reinterpret_cast<DevModel*>(ws + P.off_ls);
  Co2Job* d_jobs = reinterpret_cast<Co2Job*>(ws + P.off_jobs);
  double* d_eps = reinterpret_cast<double*>(ws + P.off_eps);
  c64* d_tab = reinterpret_cast<c64*>(ws + P.off_tab);
  int* d_counter = reinterpret_cast<int*>(ws + P.off_counter);
  int* d_finals = reinterpret_cast<int*>(ws + P.off_finals);
  DevInfo* d_info = reinterpret_cast<DevInfo*>(ws + P.off_info);
  unsigned char* d_fac = reinterpret_cast<unsigned char*>(ws + P.off_fac);
  c64* d_scratch = reinterpret_cast<c64*>(ws + P.off_scratch);
  HIPCHK(hipMemcpyAsync(d_model, &md, sizeof(Co2Model), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d_ls, &model->ls->dev, sizeof(DevModel), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d_jobs, P.jobs.data(), sizeof(Co2Job) * n_jobs, hipMemcpyHostToDevice, s));
  if (n_final > 0)
    HIPCHK(hipMemcpyAsync(d_finals, finals, sizeof(int) * 4 * n_final, hipMemcpyHostToDevice, s));
  HIPCHK(launch_zero_int(d_counter, 1, s));
  EventSet ev;
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[0], s));
  st = co2_tables(model, P.energies, d_eps, d_tab, s);
  if (st != VDC_OK) return st;
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[1], s));
  if (opts->precond == VDC_PREC_BLOCK) {
    Co2FactorArgs f{};
    f.model = d_model;
    f.jobs = d_jobs;
    f.n_jobs = n_jobs;
    f.tables = d_tab;
    f.fac = d_fac;
    f.fac_job_bytes = P.fac_job_bytes;
    HIPCHK(launch_co2_factor(f, md.Ns, md.Na, s));
  }
  Co2Args a{};
  a.model = d_model;
  a.ls = d_ls;
  a.jobs = d_jobs;
  a.n_jobs = n_jobs;
  a.tables = d_tab;
  a.counter = d_counter;
  a.scratch = d_scratch;
  a.slot_elems = P.slot_elems;
  a.ld = P.ld;
  a.fac = d_fac;
  a.fac_job_bytes = P.fac_job_bytes;
  a.m = P.m;
  a.max_iter = opts->max_iter;
  a.precond = opts->precond;
  a.method = opts->method;
  a.tol = opts->tol;
  a.n_final = n_final;
  a.finals = d_finals;
  a.T_out = reinterpret_cast<c64*>(T_out);
  a.sigma_out = sigma_out;
  a.psi_out = reinterpret_cast<c64*>(psi_out);
  a.info = d_info;
  HIPCHK(launch_co2_gmres(a, P.n_groups, s));
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[2], s));
  std::vector<DevInfo> hinfo(n_jobs);
  HIPCHK(hipMemcpyAsync(hinfo.data(), d_info, sizeof(DevInfo) * n_jobs, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (ev.ok) {
    float t1 = 0.f, t2 = 0.f;
    HIPCHK(hipEventElapsedTime(&t1, ev.e[0], ev.e[1]));
    HIPCHK(hipEventElapsedTime(&t2, ev.e[1], ev.e[2]));
    g_ms_tables = t1;
    g_ms_solver = t2;
  }
  for (int k = 0; k < n_jobs; ++k)
    info[k] = vdc_job_info{hinfo[k].status, hinfo[k].iters, hinfo[k].restarts, 0, hinfo[k].rel_res,
                           hinfo[k].alg_bytes, 0, 0, -1.0};
  return VDC_OK;
}

vdc_status vdc_co2_ops_workspace_size(vdc_co2_t model, int n_vec, int which, size_t* bytes) {
  if (!model || !bytes || n_vec < 0 || (which != 0 && which != 1))
    return fail(VDC_ERR_INVALID_ARG, "bad argument");
  const Co2Model& md = model->dev;
  if (which == 1 && md.Ny > co2_factor_max_ny())
    return fail(VDC_ERR_UNSUPPORTED, "the block preconditioner needs Ny <= 24");
  // which = 0: none for the march along n_s (co2_march_fits), else the
  // split operator's w planes for a batch of vectors; which = 1: one slot per
  // workgroup (the block apply needs none, kept small)
  const bool march = co2_march_fits(md.Ns, md.Nx, md.Ny, md.Na);
  const int groups = which == 0 ? (march ? 0 : std::max(1, std::min(n_vec, kCo2ApplyBatch)))
                                : std::max(1, std::min(n_vec, cu_count()));
  const size_t fac = which == 1 ? co2_fac_bytes(md) : 0;
  size_t off = 0;
  off = align256(off + sizeof(Co2Model));
  off = align256(off + sizeof(double) * md.ntab);
  off = align256(off + sizeof(c64) * kNumF * md.ntab);
  off = align256(off + sizeof(int) * 2 * std::max(1, n_vec));
  off = align256(off + sizeof(Co2Job) * std::max(1, n_vec));
  off = align256(off + fac * std::max(1, n_vec));
  off = align256(off + sizeof(c64) * 2 * (size_t)md.npts * groups);
  *bytes = off;
  return VDC_OK;
}

vdc_status vdc_co2_apply(vdc_co2_t model, double E, int which, int n_vec, const int* sectors,
                         const double* x, double* y, void* workspace, size_t ws_bytes, void* stream) {
  size_t need = 0;
  vdc_status st = vdc_co2_ops_workspace_size(model, n_vec, which, &need);
  if (st != VDC_OK) return st;
  if (!std::isfinite(E)) return fail(VDC_ERR_INVALID_ARG, "non-finite E");
  if (n_vec == 0) return VDC_OK;
  if (!sectors || !x || !y || !workspace) return fail(VDC_ERR_INVALID_ARG, "NULL buffer");
  for (int v = 0; v < 2 * n_vec; ++v)
    if (sectors[v] != 0 && sectors[v] != 1) return fail(VDC_ERR_INVALID_ARG, "sector bits must be 0 or 1");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(VDC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < need) return fail(VDC_ERR_WORKSPACE, "workspace too small");
  const Co2Model& md = model->dev;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  size_t off = 0;
  Co2Model* d_model = reinterpret_cast<Co2Model*>(ws + off); off = align256(off + sizeof(Co2Model));
  double* d_eps = reinterpret_cast<double*>(ws + off); off = align256(off + sizeof(double) * md.ntab);
  c64* d_tab = reinterpret_cast<c64*>(ws + off); off = align256(off + sizeof(c64) * kNumF * md.ntab);
  int* d_sec = reinterpret_cast<int*>(ws + off); off = align256(off + sizeof(int) * 2 * n_vec);
  Co2Job* d_jobs = reinterpret_cast<Co2Job*>(ws + off); off = align256(off + sizeof(Co2Job) * n_vec);
  const size_t fac_job = which == 1 ? co2_fac_bytes(md) : 0;
  unsigned char* d_fac = reinterpret_cast<unsigned char*>(ws + off); off = align256(off + fac_job * n_vec);
  c64* d_scratch = reinterpret_cast<c64*>(ws + off);
  const int groups = std::max(1, std::min(n_vec, cu_count()));
  std::vector<Co2Job> vj(n_vec);
  for (int v = 0; v < n_vec; ++v) {
    vj[v] = Co2Job{};
    vj[v].E = E;
    vj[v].px = sectors[2 * v];
    vj[v].py = sectors[2 * v + 1];
    vj[v].table = 0;
  }
  HIPCHK(hipMemcpyAsync(d_model, &md, sizeof(Co2Model), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d_sec, sectors, sizeof(int) * 2 * n_vec, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d_jobs, vj.data(), sizeof(Co2Job) * n_vec, hipMemcpyHostToDevice, s));
  EventSet ev;
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[0], s));
  st = co2_tables(model, std::vector<double>{E}, d_eps, d_tab, s);
  if (st != VDC_OK) return st;
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[1], s));
  if (which == 1) {
    Co2FactorArgs f{};
    f.model = d_model;
    f.jobs = d_jobs;
    f.n_jobs = n_vec;
    f.tables = d_tab;
    f.fac = d_fac;
    f.fac_job_bytes = fac_job;
    HIPCHK(launch_co2_factor(f, md.Ns, md.Na, s));
  }
  Co2OpsArgs a{};
  a.model = d_model;
  a.tab = d_tab;
  a.E = E;
  a.sectors = d_sec;
  a.n_vec = n_vec;
  a.which = which;
  a.x = reinterpret_cast<const c64*>(x);
  a.y = reinterpret_cast<c64*>(y);
  a.scratch = d_scratch;
  a.slot_elems = 2 * (size_t)md.npts;
  a.fac = d_fac;
  a.fac_job_bytes = fac_job;
  if (which == 0 && co2_march_fits(md.Ns, md.Nx, md.Ny, md.Na))
    HIPCHK(launch_co2_march(a, md.Ns, md.Nx, md.Ny, md.Na, s));
  else if (which == 0)
    HIPCHK(launch_co2_apply_split(a, md.npts, std::max(1, std::min(n_vec, kCo2ApplyBatch)), s));
  else
    HIPCHK(launch_co2_ops(a, groups, s));
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[2], s));
  HIPCHK(hipStreamSynchronize(s));
  if (ev.ok) {
    float t1 = 0.f, t2 = 0.f;
    HIPCHK(hipEventElapsedTime(&t1, ev.e[0], ev.e[1]));
    HIPCHK(hipEventElapsedTime(&t2, ev.e[1], ev.e[2]));
    g_ms_tables = t1;
    g_ms_solver = t2;
  }
  return VDC_OK;
}

// ---------------------------------------------------------------------------
// The general model given by polynomial term lists (vdc_model_create etc.)

namespace {

using PowKey = std::array<int, kGenMaxModes>;

// Canonical form of a term list: coefficients summed per (state pair or
// state and wave, powers); zero sums dropped.
struct Canon {
  std::map<std::tuple<int, int, PowKey>, double> u;   // (d <= e, powers)
  std::map<std::tuple<int, int, PowKey>, double> v;   // (d, mu, powers)
};

PowKey powkey(const vdc_term& t) {
  PowKey k{};
  for (int i = 0; i < kGenMaxModes; ++i) k[i] = t.pow[i];
  return k;
}

vdc_status check_desc(const vdc_model_desc* d, Canon& c) {
  if (d->n_states < 1 || d->n_states > VDC_MAX_STATES)
    return fail(VDC_ERR_INVALID_ARG, "n_states must be 1..4");
  if (d->n_modes < 1 || d->n_modes > VDC_MAX_MODES)
    return fail(VDC_ERR_INVALID_ARG, "n_modes must be 1..8");
  if (d->n_pw < 1 || d->n_pw > VDC_MAX_WAVES) return fail(VDC_ERR_INVALID_ARG, "n_pw must be 1..4");
  if (!d->omega || !d->nbasis || !d->e_state || !d->width)
    return fail(VDC_ERR_INVALID_ARG, "omega, nbasis, e_state and width must be non-NULL");
  if (d->n_uterms < 0 || d->n_vterms < 0 || (d->n_uterms > 0 && !d->uterms) ||
      (d->n_vterms > 0 && !d->vterms))
    return fail(VDC_ERR_INVALID_ARG, "bad term list");
  if (d->hilbert_nodes < 16 || d->hilbert_nodes > 65536)
    return fail(VDC_ERR_INVALID_ARG, "hilbert_nodes must be 16..65536");
  if (!(d->hilbert_xmax > 0.0) || !std::isfinite(d->hilbert_xmax))
    return fail(VDC_ERR_INVALID_ARG, "hilbert_xmax must be > 0");
  size_t npts = 1;
  for (int k = 0; k < d->n_modes; ++k) {
    if (!(d->omega[k] > 0.0) || !std::isfinite(d->omega[k]))
      return fail(VDC_ERR_INVALID_ARG, "vibrational frequencies must be finite and > 0");
    if (d->nbasis[k] < 1 || d->nbasis[k] > kSqMax)
      return fail(VDC_ERR_INVALID_ARG, "basis sizes must be 1..1024");
    npts *= (size_t)d->nbasis[k];
  }
  if (npts * d->n_states > ((size_t)1 << 26)) return fail(VDC_ERR_INVALID_ARG, "basis too large");
  for (int s = 0; s < d->n_states; ++s)
    if (!std::isfinite(d->e_state[s])) return fail(VDC_ERR_INVALID_ARG, "non-finite state energy");
  for (int mu = 0; mu < d->n_pw; ++mu) {
    int lmu = -1;
    for (int s = 0; s < d->n_states; ++s) {
      const vdc_width& w = d->width[s * d->n_pw + mu];
      if (!(w.A >= 0.0) || !std::isfinite(w.A))
        return fail(VDC_ERR_INVALID_ARG, "width amplitudes A must be finite and >= 0");
      if (!(w.B > 0.0) || !std::isfinite(w.B))
        return fail(VDC_ERR_INVALID_ARG, "width scales B must be finite and > 0");
      if (w.l < 0 || w.l > 4) return fail(VDC_ERR_INVALID_ARG, "l must be 0..4");
      if (w.A > 0.0) {
        if (lmu >= 0 && w.l != lmu)
          return fail(VDC_ERR_INVALID_ARG, "the threshold exponent l belongs to the partial wave: "
                                           "equal for every state coupled to it");
        lmu = w.l;
      }
    }
  }
  auto check_term = [&](const vdc_term& t, int emax) -> bool {
    if (t.d < 0 || t.d >= d->n_states || t.e < 0 || t.e >= emax) return false;
    if (!std::isfinite(t.coeff)) return false;
    for (int k = 0; k < kGenMaxModes; ++k) {
      if (t.pow[k] < 0 || t.pow[k] > VDC_MAX_POWER) return false;
      if (k >= d->n_modes && t.pow[k] != 0) return false;
    }
    return true;
  };
  for (int i = 0; i < d->n_uterms; ++i) {
    const vdc_term& t = d->uterms[i];
    if (!check_term(t, d->n_states))
      return fail(VDC_ERR_INVALID_ARG, "bad U term " + std::to_string(i) +
                                           ": states, finite coefficient, powers 0..4 on the modes");
    c.u[std::make_tuple(std::min(t.d, t.e), std::max(t.d, t.e), powkey(t))] += t.coeff;
  }
  for (int i = 0; i < d->n_vterms; ++i) {
    const vdc_term& t = d->vterms[i];
    if (!check_term(t, d->n_pw))
      return fail(VDC_ERR_INVALID_ARG, "bad V term " + std::to_string(i) +
                                           ": state, wave, finite coefficient, powers 0..4");
    c.v[std::make_tuple(t.d, t.e, powkey(t))] += t.coeff;
  }
  for (auto it = c.u.begin(); it != c.u.end();) it = it->second == 0.0 ? c.u.erase(it) : std::next(it);
  for (auto it = c.v.begin(); it != c.v.end();) it = it->second == 0.0 ? c.v.erase(it) : std::next(it);
  return VDC_OK;
}

// The two-state generalized model in the descriptor (and the caller allows
// its kernels): fill the two-state descriptor.
bool as_two_state(const vdc_model_desc* d, const Canon& c, vdc_model2d_desc& o) {
  if (!d->dispatch || d->n_states != 2 || d->n_modes != 2 || d->n_pw != 2) return false;
  const PowKey g{1, 0}, u{0, 1}, one{};
  double kap[2] = {0.0, 0.0}, lam = 0.0;
  for (const auto& t : c.u) {
    const int a = std::get<0>(t.first), b = std::get<1>(t.first);
    const PowKey& p = std::get<2>(t.first);
    if (a == b && p == g) kap[a] = t.second;
    else if (a == 0 && b == 1 && p == u) lam = t.second;
    else return false;
  }
  double lamd[2] = {0.0, 0.0};
  int seen = 0;
  for (const auto& t : c.v) {
    const int a = std::get<0>(t.first), mu = std::get<1>(t.first);
    const PowKey& p = std::get<2>(t.first);
    if (a == mu && p == one && t.second == 1.0) seen |= 1 << (2 * a + mu);
    else if (a == mu && p == g) lamd[a] = t.second;
    else if (a != mu && p == u && t.second == 1.0) seen |= 1 << (2 * a + mu);
    else return false;
  }
  if (seen != 15) return false;
  o = vdc_model2d_desc{};
  o.omega_g = d->omega[0];
  o.omega_u = d->omega[1];
  o.kappa1 = kap[0];
  o.kappa2 = kap[1];
  o.lam = lam;
  o.lam1 = lamd[0];
  o.lam2 = lamd[1];
  o.E1 = d->e_state[0];
  o.gap = d->e_state[1] - d->e_state[0];
  for (int s = 0; s < 2; ++s)
    for (int mu = 0; mu < 2; ++mu) {
      o.A[s][mu] = d->width[s * 2 + mu].A;
      o.B[s][mu] = d->width[s * 2 + mu].B;
    }
  for (int mu = 0; mu < 2; ++mu)
    o.l[mu] = d->width[0 * 2 + mu].A > 0.0 ? d->width[mu].l : d->width[2 + mu].l;
  o.Ng = d->nbasis[0];
  o.Nu = d->nbasis[1];
  o.hilbert_nodes = d->hilbert_nodes;
  o.hilbert_xmax = d->hilbert_xmax;
  return true;
}

template <typename T>
vdc_status upload(GenHost& G, const std::vector<T>& h, const T** out) {
  void* p = nullptr;
  const size_t n = std::max<size_t>(1, h.size()) * sizeof(T);
  HIPCHK(hipMalloc(&p, n));
  G.mem.push_back(p);
  if (!h.empty()) HIPCHK(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = reinterpret_cast<const T*>(p);
  return VDC_OK;
}

// Rows of (P q P)^p for p = 0..4 on an n-function basis: table[(p n + m) kGenQW
// + delta + 4] = <m|(P q P)^p|m + delta>.
std::vector<double> power_rows(int n) {
  std::vector<double> t((size_t)(kGenMaxPow + 1) * n * kGenQW, 0.0);
  auto at = [&](int p, int m, int dl) -> double& {
    return t[((size_t)p * n + m) * kGenQW + dl + kGenMaxPow];
  };
  for (int m = 0; m < n; ++m) at(0, m, 0) = 1.0;
  // (M q)[m][j] = sum_i M[m][i] q[i][j], q[i][i+1] = q[i+1][i] = sqrt((i+1)/2)
  for (int p = 1; p <= kGenMaxPow; ++p)
    for (int m = 0; m < n; ++m)
      for (int dl = -p; dl <= p; ++dl) {
        const int j = m + dl;
        if (j < 0 || j >= n) continue;
        double s = 0.0;
        for (int dd = -(p - 1); dd <= p - 1; ++dd) {
          const int i = m + dd;
          if (i < 0 || i >= n || std::abs(i - j) != 1) continue;
          s += at(p - 1, m, dd) * std::sqrt(0.5 * std::max(i, j));
        }
        at(p, m, dl) = s;
      }
  return t;
}

// Compile one operator (monomials with their coefficients) into stencil
// points: the distinct offset vectors, each with the monomials reaching it.
GenOp compile_op(const std::vector<std::pair<PowKey, double>>& mono, const DevGen& g,
                 std::vector<GenPoint>& pts, std::vector<GenTerm>& terms) {
  std::map<std::array<int, kGenMaxModes>, std::vector<int>> by_off;
  for (size_t t = 0; t < mono.size(); ++t) {
    const PowKey& p = mono[t].first;
    std::array<int, kGenMaxModes> dl{};
    // odometer over delta_k in {-p_k, -p_k + 2, ..., p_k}
    for (int k = 0; k < kGenMaxModes; ++k) dl[k] = -p[k];
    for (;;) {
      by_off[dl].push_back((int)t);
      int k = g.M - 1;
      while (k >= 0) {
        dl[k] += 2;
        if (dl[k] <= p[k]) break;
        dl[k] = -p[k];
        --k;
      }
      if (k < 0) break;
    }
  }
  GenOp op{(int)pts.size(), (int)by_off.size()};
  for (const auto& e : by_off) {
    GenPoint pt{};
    pt.off = 0;
    pt.zero = 1;
    for (int k = 0; k < kGenMaxModes; ++k) {
      pt.dl[k] = (signed char)e.first[k];
      if (k < g.M) pt.off += e.first[k] * g.stride[k];
      if (e.first[k] != 0) pt.zero = 0;
    }
    pt.t0 = (int)terms.size();
    pt.nt = (int)e.second.size();
    for (int t : e.second) {
      GenTerm tm{};
      tm.c = mono[t].second;
      for (int k = 0; k < kGenMaxModes; ++k) tm.pw[k] = (signed char)mono[t].first[k];
      terms.push_back(tm);
    }
    pts.push_back(pt);
  }
  return op;
}

vdc_status build_gen(const vdc_model_desc* d, const Canon& c, GenHost& G) {
  DevGen& g = G.dev;
  g.D = d->n_states;
  g.M = d->n_modes;
  g.P = d->n_pw;
  g.npts = 1;
  for (int k = 0; k < g.M; ++k) {
    g.n[k] = d->nbasis[k];
    g.omega[k] = d->omega[k];
    g.npts *= g.n[k];
  }
  int st = 1;
  for (int k = g.M - 1; k >= 0; --k) {
    g.stride[k] = st;
    st *= g.n[k];
  }
  G.N = g.D * g.npts;
  for (int s = 0; s < g.D; ++s) g.e_state[s] = d->e_state[s];
  for (int s = 0; s < g.D; ++s)
    for (int mu = 0; mu < g.P; ++mu) {
      g.A[s][mu] = d->width[s * g.P + mu].A;
      g.B[s][mu] = d->width[s * g.P + mu].B;
    }
  for (int mu = 0; mu < g.P; ++mu) {
    g.l[mu] = 0;
    for (int s = 0; s < g.D; ++s)
      if (d->width[s * g.P + mu].A > 0.0) g.l[mu] = d->width[s * g.P + mu].l;
  }
  // operators
  std::vector<GenPoint> pts;
  std::vector<GenTerm> terms;
  for (int a = 0; a < g.D; ++a)
    for (int b = a; b < g.D; ++b) {
      std::vector<std::pair<PowKey, double>> mono;
      for (const auto& t : c.u)
        if (std::get<0>(t.first) == a && std::get<1>(t.first) == b)
          mono.emplace_back(std::get<2>(t.first), t.second);
      GenOp op{0, 0};
      if (!mono.empty()) op = compile_op(mono, g, pts, terms);
      g.uop[a][b] = g.uop[b][a] = op;
    }
  for (int a = 0; a < g.D; ++a)
    for (int mu = 0; mu < g.P; ++mu) {
      std::vector<std::pair<PowKey, double>> mono;
      for (const auto& t : c.v)
        if (std::get<0>(t.first) == a && std::get<1>(t.first) == mu)
          mono.emplace_back(std::get<2>(t.first), t.second);
      g.vop[a][mu] = mono.empty() ? GenOp{0, 0} : compile_op(mono, g, pts, terms);
    }
  // level-shift planes F^mu_de: both states couple to mu (O != 0, A > 0)
  g.nplanes = 0;
  auto couples = [&](int s, int mu) { return g.vop[s][mu].np > 0 && g.A[s][mu] > 0.0; };
  for (int mu = 0; mu < kGenMaxWaves; ++mu)
    for (int a = 0; a < kGenMaxStates; ++a)
      for (int b = 0; b < kGenMaxStates; ++b) g.fplane[mu][a][b] = -1;
  for (int mu = 0; mu < g.P; ++mu)
    for (int a = 0; a < g.D; ++a)
      for (int b = a; b < g.D; ++b)
        if (couples(a, mu) && couples(b, mu)) g.fplane[mu][a][b] = g.fplane[mu][b][a] = g.nplanes++;
  g.nw = 0;
  for (int mu = 0; mu < kGenMaxWaves; ++mu)
    for (int a = 0; a < kGenMaxStates; ++a) g.wplane[mu][a] = -1;
  for (int mu = 0; mu < g.P; ++mu)
    for (int a = 0; a < g.D; ++a)
      if (couples(a, mu)) g.wplane[mu][a] = g.nw++;
  // two-state transform models: slots (mu, a, b) covering F_aa, F_ab, F_bb,
  // two slots (waves mu' = 0, 1 of the descriptor) per model
  struct Slot { int mu, a, b; };
  std::vector<Slot> slots;
  std::vector<char> covered(g.nplanes > 0 ? g.nplanes : 1, 0);
  for (int mu = 0; mu < g.P; ++mu) {
    for (int a = 0; a < g.D; ++a)
      for (int b = a + 1; b < g.D; ++b)
        if (g.fplane[mu][a][b] >= 0) slots.push_back(Slot{mu, a, b});
    for (int a = 0; a < g.D; ++a)
      if (g.fplane[mu][a][a] >= 0) slots.push_back(Slot{mu, a, a});
  }
  std::vector<DevModel> lsm;
  std::vector<int> lsmap;
  for (size_t s0 = 0; s0 < slots.size(); s0 += 2) {
    vdc_model2d_desc ld{};
    ld.omega_g = ld.omega_u = 1.0;
    ld.Ng = ld.Nu = 1;
    ld.hilbert_nodes = d->hilbert_nodes;
    ld.hilbert_xmax = d->hilbert_xmax;
    std::array<int, kNumF> map;
    map.fill(-1);
    for (int w = 0; w < 2; ++w) {
      ld.A[0][w] = ld.A[1][w] = 0.0;
      ld.B[0][w] = ld.B[1][w] = 1.0;
      ld.l[w] = 0;
      if (s0 + w >= slots.size()) continue;
      const Slot& sl = slots[s0 + w];
      ld.A[0][w] = g.A[sl.a][sl.mu];
      ld.B[0][w] = g.B[sl.a][sl.mu];
      ld.A[1][w] = g.A[sl.b][sl.mu];
      ld.B[1][w] = g.B[sl.b][sl.mu];
      ld.l[w] = g.l[sl.mu];
      const int pairs[3][2] = {{sl.a, sl.a}, {sl.a, sl.b}, {sl.b, sl.b}};
      for (int pq = 0; pq < 3; ++pq) {
        const int pl = g.fplane[sl.mu][pairs[pq][0]][pairs[pq][1]];
        if (pl >= 0 && !covered[pl]) {
          covered[pl] = 1;
          map[fidx(w, pq)] = pl;
        }
      }
    }
    vdc_model_t m2 = nullptr;
    const vdc_status st2 = vdc_model2d_create(&ld, &m2);
    if (st2 != VDC_OK) return st2;
    G.ls.push_back(m2);
    lsm.push_back(m2->dev);
    for (int f = 0; f < kNumF; ++f) lsmap.push_back(map[f]);
  }
  g.nlsm = (int)lsm.size();
  // tables of powers of the truncated coordinate, E_nu and the point order
  std::vector<double> qtab;
  for (int k = 0; k < g.M; ++k) {
    g.qoff[k] = (int)qtab.size();
    const std::vector<double> t = power_rows(g.n[k]);
    qtab.insert(qtab.end(), t.begin(), t.end());
  }
  std::vector<double> Enu(g.npts);
  for (int i = 0; i < g.npts; ++i) {
    int r = i;
    double e = 0.0;
    for (int k = g.M - 1; k >= 0; --k) {
      const int nk = r % g.n[k];
      r /= g.n[k];
      e += g.omega[k] * (nk + 0.5);
    }
    Enu[i] = e;
  }
  std::vector<int> perm(g.npts);
  for (int i = 0; i < g.npts; ++i) perm[i] = i;
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return Enu[a] < Enu[b]; });
  vdc_status st3;
  if ((st3 = upload(G, qtab, &g.qtab)) != VDC_OK) return st3;
  if ((st3 = upload(G, pts, &g.pts)) != VDC_OK) return st3;
  if ((st3 = upload(G, terms, &g.terms)) != VDC_OK) return st3;
  if ((st3 = upload(G, Enu, &g.Enu)) != VDC_OK) return st3;
  if ((st3 = upload(G, perm, &g.perm)) != VDC_OK) return st3;
  if ((st3 = upload(G, lsm, &g.lsm)) != VDC_OK) return st3;
  if ((st3 = upload(G, lsmap, &g.lsmap)) != VDC_OK) return st3;
  return VDC_OK;
}

// Plan of a batched solve of term-list models (workspace layout).
struct GenPlan {
  std::vector<DevGen> models;
  std::vector<GenJob> jobs;
  std::vector<GenTab> tabs;
  size_t table_elems = 0, ld = 0, wld = 0, slot_elems = 0;
  int n_groups = 0, max_npts = 0, max_nlsm = 0, n_pw = 0;
  size_t off_counter, off_models, off_jobs, off_tabs, off_finals, off_info, off_tables,
      off_scratch, total;
};

vdc_status gen_plan(int n_models, const vdc_model_t* models, const vdc_solve_opts* o, int n_jobs,
                    const vdc_mjob* jobs, int n_final, GenPlan& P) {
  if (n_models <= 0 || !models) return fail(VDC_ERR_INVALID_ARG, "no models");
  if (!o) return fail(VDC_ERR_INVALID_ARG, "opts is NULL");
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(VDC_ERR_INVALID_ARG, "bad job list");
  if (n_final < 0 || n_final > kMaxFinal) return fail(VDC_ERR_INVALID_ARG, "n_final must be 0..64");
  if (o->method != VDC_GMRES && o->method != VDC_COCG)
    return fail(VDC_ERR_INVALID_ARG, "unknown method");
  if (o->method == VDC_GMRES && (o->restart < 1 || o->restart > kMaxRestart))
    return fail(VDC_ERR_INVALID_ARG, "restart must be 1..128");
  if (o->max_iter < 1) return fail(VDC_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (!(o->tol > 0.0)) return fail(VDC_ERR_INVALID_ARG, "tol must be > 0");
  if (o->precision != VDC_FP64)
    return fail(VDC_ERR_UNSUPPORTED, "term-list models are solved in FP64 only");
  if (o->precond != VDC_PREC_NONE && o->precond != VDC_PREC_JACOBI)
    return fail(VDC_ERR_UNSUPPORTED, "term-list models take VDC_PREC_NONE or VDC_PREC_JACOBI");
  size_t maxN = 1, maxW = 1;
  for (int k = 0; k < n_models; ++k) {
    if (!models[k] || !models[k]->gen)
      return fail(VDC_ERR_INVALID_ARG, "every model must come from vdc_model_create");
    const DevGen& g = models[k]->gen->dev;
    P.models.push_back(g);
    maxN = std::max(maxN, (size_t)g.D * g.npts);
    maxW = std::max(maxW, (size_t)g.nw * g.npts);
    P.max_npts = std::max(P.max_npts, g.npts);
    P.max_nlsm = std::max(P.max_nlsm, g.nlsm);
    P.n_pw = std::max(P.n_pw, g.P);
  }
  std::map<std::pair<int, double>, int> tab_index;
  P.jobs.resize(n_jobs);
  for (int j = 0; j < n_jobs; ++j) {
    const vdc_mjob& jb = jobs[j];
    if (jb.model < 0 || jb.model >= n_models)
      return fail(VDC_ERR_INVALID_ARG, "job model index out of range");
    const DevGen& g = P.models[jb.model];
    if (!(jb.eps_i > 0.0) || !std::isfinite(jb.eps_i))
      return fail(VDC_ERR_INVALID_ARG, "eps_i must be > 0 (open entrance channel)");
    if (jb.mu_i < 0 || jb.mu_i >= g.P) return fail(VDC_ERR_INVALID_ARG, "mu_i outside the model's waves");
    GenJob& o2 = P.jobs[j];
    for (int k = 0; k < kGenMaxModes; ++k) {
      o2.v[k] = k < g.M ? jb.v[k] : 0;
      if (k >= g.M && jb.v[k] != 0) return fail(VDC_ERR_INVALID_ARG, "v_i has entries past n_modes");
    }
    if (gen_flat(g, o2.v) < 0) return fail(VDC_ERR_INVALID_ARG, "v_i outside the basis");
    o2.eps_i = jb.eps_i;
    o2.E = jb.eps_i + gen_vib_energy(g, o2.v);
    o2.mu = jb.mu_i;
    o2.model = jb.model;
    o2.out = j;
    auto key = std::make_pair(jb.model, o2.E);
    auto it = tab_index.find(key);
    if (it == tab_index.end()) {
      GenTab t{};
      t.E = o2.E;
      t.model = jb.model;
      t.offset = P.table_elems;
      P.table_elems += (size_t)g.nplanes * g.npts;
      it = tab_index.emplace(key, (int)P.tabs.size()).first;
      P.tabs.push_back(t);
    }
    o2.table = it->second;
  }
  if (P.tabs.size() > 65535) return fail(VDC_ERR_INVALID_ARG, "more than 65535 distinct energies");
  // longest first: unknowns x energy
  std::stable_sort(P.jobs.begin(), P.jobs.end(), [&](const GenJob& a, const GenJob& b) {
    const DevGen& ga = P.models[a.model];
    const DevGen& gb = P.models[b.model];
    return (double)ga.D * ga.npts * (0.5 + a.E) > (double)gb.D * gb.npts * (0.5 + b.E);
  });
  P.ld = (maxN + 63) / 64 * 64;
  P.wld = (maxW + 63) / 64 * 64;
  const int m = o->method == VDC_COCG ? 3 : o->restart + 1;
  P.slot_elems = 4 * P.ld + P.wld + (size_t)m * P.ld +
                 (o->method == VDC_COCG ? 0 : (size_t)(o->restart + 1) * o->restart);
  P.slot_elems = (P.slot_elems + 31) / 32 * 32;
  P.n_groups = std::max(1, std::min(n_jobs, cu_count() * gen_solve_occupancy()));
  size_t off = 0;
  P.off_counter = off; off += 256;
  P.off_models = off; off = align256(off + sizeof(DevGen) * n_models);
  P.off_jobs = off; off = align256(off + sizeof(GenJob) * std::max(1, n_jobs));
  P.off_tabs = off; off = align256(off + sizeof(GenTab) * std::max<size_t>(1, P.tabs.size()));
  P.off_finals = off; off = align256(off + sizeof(int) * kGenMaxModes * std::max(1, n_final));
  P.off_info = off; off = align256(off + sizeof(DevInfo) * std::max(1, n_jobs));
  P.off_tables = off; off = align256(off + sizeof(c64) * P.table_elems);
  P.off_scratch = off; off = align256(off + sizeof(c64) * P.slot_elems * P.n_groups);
  P.total = off;
  return VDC_OK;
}

// All models have the two-state form: the job list in that form.
bool all_two_state(int n_models, const vdc_model_t* models) {
  for (int k = 0; k < n_models; ++k)
    if (!models[k] || models[k]->kind != 0) return false;
  return true;
}

vdc_status to_two_state_jobs(int n_jobs, const vdc_mjob* jobs, int n_final, const int* finals,
                             std::vector<vdc_job>& j2, std::vector<int>& f2) {
  j2.resize(n_jobs);
  for (int j = 0; j < n_jobs; ++j) {
    for (int k = 2; k < VDC_MAX_MODES; ++k)
      if (jobs[j].v[k] != 0) return fail(VDC_ERR_INVALID_ARG, "v_i has entries past n_modes");
    j2[j] = vdc_job{jobs[j].eps_i, jobs[j].v[0], jobs[j].v[1], jobs[j].mu_i, jobs[j].model};
  }
  f2.resize(2 * std::max(1, n_final));
  for (int f = 0; f < n_final; ++f) {
    f2[2 * f] = finals[f * VDC_MAX_MODES];
    f2[2 * f + 1] = finals[f * VDC_MAX_MODES + 1];
  }
  return VDC_OK;
}

}  // namespace

extern "C" {

vdc_status vdc_model_create(const vdc_model_desc* d, vdc_model_t* out) {
  if (!d || !out) return fail(VDC_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  Canon c;
  vdc_status st = check_desc(d, c);
  if (st != VDC_OK) return st;
  vdc_model2d_desc d2;
  vdc_model_t m = nullptr;
  if (as_two_state(d, c, d2)) {
    st = vdc_model2d_create(&d2, &m);
    if (st != VDC_OK) return st;
  } else {
    m = new vdc_model();
    m->desc = vdc_model2d_desc{};
    m->dev = DevModel{};
    m->kind = 1;
  }
  m->gen = new GenHost();
  st = build_gen(d, c, *m->gen);
  if (st != VDC_OK) {
    vdc_model_destroy(m);
    return st;
  }
  *out = m;
  return VDC_OK;
}

vdc_status vdc_model_kind(vdc_model_t m, int* kind) {
  if (!m || !kind) return fail(VDC_ERR_INVALID_ARG, "NULL argument");
  *kind = m->kind;
  return VDC_OK;
}

vdc_status vdc_model_workspace_size(int n_models, const vdc_model_t* models,
                                    const vdc_solve_opts* opts, int n_jobs, const vdc_mjob* jobs,
                                    size_t* bytes) {
  if (!bytes) return fail(VDC_ERR_INVALID_ARG, "bytes is NULL");
  if (n_models > 0 && models && all_two_state(n_models, models)) {
    std::vector<vdc_job> j2;
    std::vector<int> f2;
    vdc_status st = to_two_state_jobs(n_jobs, jobs, 0, nullptr, j2, f2);
    if (st != VDC_OK) return st;
    return vdc_workspace_size(n_models, models, opts, n_jobs, j2.data(), bytes);
  }
  GenPlan P;
  vdc_status st = gen_plan(n_models, models, opts, n_jobs, jobs, kMaxFinal, P);
  if (st != VDC_OK) return st;
  *bytes = P.total;
  return VDC_OK;
}

vdc_status vdc_model_solve(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                           int n_jobs, const vdc_mjob* jobs, int n_final, const int* finals,
                           void* workspace, size_t ws_bytes, double* T_out, double* sigma_out,
                           double* psi_out, vdc_job_info* info, void* stream) {
  if (n_final > 0 && !finals) return fail(VDC_ERR_INVALID_ARG, "finals is NULL");
  if (n_models > 0 && models && all_two_state(n_models, models)) {
    std::vector<vdc_job> j2;
    std::vector<int> f2;
    vdc_status st = to_two_state_jobs(n_jobs, jobs, n_final, finals, j2, f2);
    if (st != VDC_OK) return st;
    return vdc_solve(n_models, models, opts, n_jobs, j2.data(), n_final, f2.data(), workspace,
                     ws_bytes, T_out, sigma_out, psi_out, info, stream);
  }
  GenPlan P;
  vdc_status st = gen_plan(n_models, models, opts, n_jobs, jobs, n_final, P);
  if (st != VDC_OK || n_jobs == 0) return st;
  if (!workspace) return fail(VDC_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(VDC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < P.total)
    return fail(VDC_ERR_WORKSPACE, "workspace too small: need " + std::to_string(P.total) +
                                       " bytes, got " + std::to_string(ws_bytes));
  if (n_final > 0 && (!T_out || !sigma_out))
    return fail(VDC_ERR_INVALID_ARG, "T_out/sigma_out must be non-NULL when n_final > 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  std::vector<int> fin((size_t)kGenMaxModes * std::max(1, n_final), 0);
  for (int f = 0; f < n_final; ++f)
    for (int k = 0; k < kGenMaxModes; ++k) fin[(size_t)f * kGenMaxModes + k] = finals[f * VDC_MAX_MODES + k];
  HIPCHK(hipMemcpyAsync(ws + P.off_models, P.models.data(), sizeof(DevGen) * n_models,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + P.off_jobs, P.jobs.data(), sizeof(GenJob) * n_jobs,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + P.off_tabs, P.tabs.data(), sizeof(GenTab) * P.tabs.size(),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + P.off_finals, fin.data(), sizeof(int) * fin.size(),
                        hipMemcpyHostToDevice, s));
  GenArgs a{};
  a.models = reinterpret_cast<const DevGen*>(ws + P.off_models);
  a.jobs = reinterpret_cast<const GenJob*>(ws + P.off_jobs);
  a.n_jobs = n_jobs;
  a.tabs = reinterpret_cast<const GenTab*>(ws + P.off_tabs);
  a.tables = reinterpret_cast<const c64*>(ws + P.off_tables);
  a.counter = reinterpret_cast<int*>(ws + P.off_counter);
  a.scratch = reinterpret_cast<c64*>(ws + P.off_scratch);
  a.slot_elems = P.slot_elems;
  a.ld = P.ld;
  a.wld = P.wld;
  a.method = opts->method;
  a.m = opts->restart;
  a.max_iter = opts->max_iter;
  a.tol = opts->tol;
  a.precond = opts->precond;
  a.n_final = n_final;
  a.finals = reinterpret_cast<const int*>(ws + P.off_finals);
  a.n_pw = P.n_pw;
  a.T_out = reinterpret_cast<c64*>(T_out);
  a.sigma_out = sigma_out;
  a.psi_out = reinterpret_cast<c64*>(psi_out);
  a.psi_ld = P.ld;
  size_t maxN = 0;
  for (const DevGen& g : P.models) maxN = std::max(maxN, (size_t)g.D * g.npts);
  a.psi_ld = maxN;
  a.info = reinterpret_cast<DevInfo*>(ws + P.off_info);
  a.check_optical = opts->check_optical != 0;
  EventSet ev;
  HIPCHK(launch_zero_int(a.counter, 64, s));
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[0], s));
  HIPCHK(launch_gen_planes(a.models, a.tabs, (int)P.tabs.size(), P.max_npts, P.max_nlsm,
                           reinterpret_cast<c64*>(ws + P.off_tables), s));
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[1], s));
  HIPCHK(launch_gen_solve(a, P.n_groups, s));
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[2], s));
  std::vector<DevInfo> hinfo(n_jobs);
  HIPCHK(hipMemcpyAsync(hinfo.data(), ws + P.off_info, sizeof(DevInfo) * n_jobs,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (ev.ok) {
    float t1 = 0.f, t2 = 0.f;
    HIPCHK(hipEventElapsedTime(&t1, ev.e[0], ev.e[1]));
    HIPCHK(hipEventElapsedTime(&t2, ev.e[1], ev.e[2]));
    g_ms_tables = t1;
    g_ms_solver = t2;
  }
  if (info)
    for (int j = 0; j < n_jobs; ++j)
      info[j] = vdc_job_info{hinfo[j].status, hinfo[j].iters, hinfo[j].restarts, 0,
                             hinfo[j].rel_res, hinfo[j].alg_bytes, 0, 0, hinfo[j].defect};
  return VDC_OK;
}

static size_t gen_apply_ws(const GenHost& G, int n_vec, size_t* off_tab, size_t* off_tables,
                           size_t* off_w) {
  size_t off = align256(sizeof(DevGen));
  *off_tab = off;
  off = align256(off + sizeof(GenTab));
  *off_tables = off;
  off = align256(off + sizeof(c64) * (size_t)std::max(1, G.dev.nplanes) * G.dev.npts);
  *off_w = off;
  off = align256(off + sizeof(c64) * (size_t)std::max(1, G.dev.nw) * G.dev.npts *
                           std::max(1, n_vec));
  return off;
}

vdc_status vdc_model_apply_workspace_size(vdc_model_t m, int n_vec, size_t* bytes) {
  if (!m || !bytes || n_vec < 0) return fail(VDC_ERR_INVALID_ARG, "bad argument");
  if (!m->gen) return fail(VDC_ERR_UNSUPPORTED, "the model has no term-list form (vdc_model2d_create)");
  size_t a, b, c;
  *bytes = gen_apply_ws(*m->gen, n_vec, &a, &b, &c);
  return VDC_OK;
}

vdc_status vdc_model_apply(vdc_model_t m, double E, int n_vec, const double* x, double* y,
                           void* workspace, size_t ws_bytes, void* stream) {
  size_t need = 0;
  vdc_status st = vdc_model_apply_workspace_size(m, n_vec, &need);
  if (st != VDC_OK) return st;
  if (n_vec == 0) return VDC_OK;
  if (!std::isfinite(E)) return fail(VDC_ERR_INVALID_ARG, "E must be finite");
  if (!x || !y || !workspace) return fail(VDC_ERR_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(VDC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < need) return fail(VDC_ERR_WORKSPACE, "workspace too small");
  const GenHost& G = *m->gen;
  const size_t N = (size_t)G.N;
  if (reinterpret_cast<const char*>(x) < reinterpret_cast<const char*>(y) + sizeof(c64) * N * n_vec &&
      reinterpret_cast<const char*>(y) < reinterpret_cast<const char*>(x) + sizeof(c64) * N * n_vec)
    return fail(VDC_ERR_INVALID_ARG, "x and y must not overlap");
  size_t off_tab, off_tables, off_w;
  gen_apply_ws(G, n_vec, &off_tab, &off_tables, &off_w);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  GenTab tb{};
  tb.E = E;
  tb.model = 0;
  tb.offset = 0;
  HIPCHK(hipMemcpyAsync(ws, &G.dev, sizeof(DevGen), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + off_tab, &tb, sizeof(GenTab), hipMemcpyHostToDevice, s));
  const DevGen* gd = reinterpret_cast<const DevGen*>(ws);
  c64* F = reinterpret_cast<c64*>(ws + off_tables);
  EventSet ev;
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[0], s));
  HIPCHK(launch_gen_planes(gd, reinterpret_cast<const GenTab*>(ws + off_tab), 1, G.dev.npts,
                           G.dev.nlsm, F, s));
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[1], s));
  HIPCHK(launch_gen_apply(gd, G.dev.npts, E, F, n_vec, reinterpret_cast<const c64*>(x),
                          reinterpret_cast<c64*>(ws + off_w), reinterpret_cast<c64*>(y), N,
                          (size_t)std::max(1, G.dev.nw) * G.dev.npts, s));
  if (ev.ok) HIPCHK(hipEventRecord(ev.e[2], s));
  HIPCHK(hipStreamSynchronize(s));
  if (ev.ok) {
    float t1 = 0.f, t2 = 0.f;
    HIPCHK(hipEventElapsedTime(&t1, ev.e[0], ev.e[1]));
    HIPCHK(hipEventElapsedTime(&t2, ev.e[1], ev.e[2]));
    g_ms_tables = t1;
    g_ms_solver = t2;
  }
  return VDC_OK;
}

vdc_status vdc_sum_partial_waves(int n_jobs, const int* collision, int n_coll, int n_final,
                                 const double* share, double* sigma, void* stream) {
  if (n_jobs < 0 || n_coll < 0 || n_final < 0)
    return fail(VDC_ERR_INVALID_ARG, "negative size");
  if (n_coll == 0 || n_final == 0) return VDC_OK;
  if (!sigma || (n_jobs > 0 && (!collision || !share)))
    return fail(VDC_ERR_INVALID_ARG, "NULL buffer");
  HIPCHK(launch_sum_waves(n_jobs, collision, n_coll, n_final, share, sigma,
                          reinterpret_cast<hipStream_t>(stream)));
  return VDC_OK;
}

}  // extern "C"
