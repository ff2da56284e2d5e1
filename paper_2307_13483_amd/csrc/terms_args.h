// Job, table and argument structs of the general model's batched solve.
#pragma once
#include "terms.h"

namespace vdc {

struct GenJob {
  double eps_i;            // incident electron energy
  double E;                // total energy eps_i + E_{v_i}
  int v[kGenMaxModes];     // initial vibrational state
  int mu;                  // incoming partial wave
  int model, table, out;
};

// Level-shift planes of one (model, total energy): [nplanes][npts] complex
// from offset (complex elements from the table base).
struct GenTab {
  double E;
  int model;
  int pad;
  size_t offset;
};

struct GenArgs {
  const DevGen* models;
  const GenJob* jobs;
  int n_jobs;
  const GenTab* tabs;
  const c64* tables;
  int* counter;
  c64* scratch;
  size_t slot_elems;       // complex elements per workgroup slot
  size_t ld;               // leading dimension of slot vectors (>= max D npts)
  size_t wld;              // w planes per slot (>= max nw npts)
  int method, m, max_iter;
  double tol;
  int precond;
  int n_final;
  const int* finals;       // [n_final][kGenMaxModes]
  int n_pw;                // partial waves per amplitude row (max P)
  c64* T_out;              // [n_jobs][n_final][n_pw]
  double* sigma_out;       // [n_jobs][n_final]
  c64* psi_out;            // [n_jobs][psi_ld] or null
  size_t psi_ld;
  DevInfo* info;
  int check_optical;       // compute the optical-theorem defect of each solution
};

hipError_t launch_gen_apply(const DevGen* gm_dev, int npts, double E, const c64* F, int n_vec,
                            const c64* x, c64* w, c64* y, size_t xld, size_t wld, hipStream_t s);
hipError_t launch_gen_solve(const GenArgs& a, int n_groups, hipStream_t s);
int gen_solve_occupancy();
hipError_t launch_sum_waves(int n_jobs, const int* coll, int n_coll, int n_final,
                            const double* share, double* sigma, hipStream_t s);
hipError_t launch_gen_planes(const DevGen* gens, const GenTab* tabs, int n_tabs, int max_npts,
                             int max_nlsm, c64* base, hipStream_t s);

}  // namespace vdc
