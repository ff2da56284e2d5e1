// Runs one case through the library built for the CPU stand-in of HIP and
// writes its results: "solve CASE OUT" (vdc_solve: two-state models),
// "co2 DESC X N_VEC WHICH E OUT" (vdc_co2_apply on the vectors in X),
// "co2solve DESC CASE OUT" (vdc_co2_solve) and "terms CASE DISPATCH OUT"
// (vdc_model_create + vdc_model_solve).  Case
// files hold the C structs of include/vdc.h as the tests write them.
// Prints one line per job; exits non-zero when a call fails.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "vdc.h"

namespace {

void* dev_alloc(size_t n) {
  void* p = nullptr;
  if (posix_memalign(&p, 256, n ? n : 1) != 0) abort();
  memset(p, 0, n);
  return p;
}

template <typename T> void rd(FILE* f, T* p, size_t n) {
  if (n && fread(p, sizeof(T), n, f) != n) {
    printf("case file: short read\n");
    exit(2);
  }
}

void put(FILE* g, const void* p, size_t bytes) {
  if (bytes && fwrite(p, 1, bytes, g) != bytes) exit(2);
}

void report(const std::vector<vdc_job_info>& info) {
  int bad = 0;
  for (size_t j = 0; j < info.size(); ++j) {
    printf("job %zu status %d iters %d outer %d rel_res %.6e retried %d\n", j, info[j].status,
           info[j].iters, info[j].outer_iters, info[j].rel_res, info[j].retried);
    bad += info[j].status != VDC_CONVERGED;
  }
  printf("done: %d not converged\n", bad);
}

// solve: n_models, descs, n_jobs, jobs, n_final, finals [2], opts
int run_solve(const char* path, const char* out) {
  FILE* f = fopen(path, "rb");
  if (!f) return 2;
  int nm = 0, nj = 0, nf = 0;
  rd(f, &nm, 1);
  std::vector<vdc_model2d_desc> descs(nm);
  rd(f, descs.data(), nm);
  rd(f, &nj, 1);
  std::vector<vdc_job> jobs(nj);
  rd(f, jobs.data(), nj);
  rd(f, &nf, 1);
  std::vector<int> finals(2 * nf);
  rd(f, finals.data(), 2 * nf);
  vdc_solve_opts o;
  rd(f, &o, 1);
  fclose(f);
  std::vector<vdc_model_t> models(nm);
  int max_nc = 0;
  for (int k = 0; k < nm; ++k) {
    if (vdc_model2d_create(&descs[k], &models[k]) != VDC_OK) {
      printf("vdc_model2d_create: %s\n", vdc_last_error());
      return 3;
    }
    max_nc = std::max(max_nc, descs[k].Ng * descs[k].Nu);
  }
  size_t ws = 0;
  if (vdc_workspace_size(nm, models.data(), &o, nj, jobs.data(), &ws) != VDC_OK) {
    printf("vdc_workspace_size: %s\n", vdc_last_error());
    return 3;
  }
  void* w = dev_alloc(ws);
  const size_t nT = 4 * (size_t)nj * nf, nS = (size_t)nj * nf, nP = 4 * (size_t)nj * max_nc;
  double* T = (double*)dev_alloc(sizeof(double) * nT);
  double* sig = (double*)dev_alloc(sizeof(double) * nS);
  double* psi = (double*)dev_alloc(sizeof(double) * nP);
  std::vector<vdc_job_info> info(nj);
  if (vdc_solve(nm, models.data(), &o, nj, jobs.data(), nf, finals.data(), w, ws, T, sig, psi,
                info.data(), nullptr) != VDC_OK) {
    printf("vdc_solve: %s\n", vdc_last_error());
    return 3;
  }
  report(info);
  FILE* g = fopen(out, "wb");
  put(g, T, sizeof(double) * nT);
  put(g, sig, sizeof(double) * nS);
  put(g, psi, sizeof(double) * nP);
  fclose(g);
  free(w);
  free(T);
  free(sig);
  free(psi);
  for (vdc_model_t m : models) vdc_model_destroy(m);
  return 0;
}

// co2: desc; x from a file (complex [n_vec][npts]); sector of vector v:
// (v & 1, (v >> 1) & 1)
int run_co2(const char* path, const char* xpath, int n_vec, int which, double E, const char* out) {
  vdc_co2_desc d;
  FILE* f = fopen(path, "rb");
  if (!f) return 2;
  rd(f, &d, 1);
  fclose(f);
  vdc_co2_t m;
  if (vdc_co2_create(&d, &m) != VDC_OK) {
    printf("vdc_co2_create: %s\n", vdc_last_error());
    return 3;
  }
  const size_t npts = (size_t)d.Ns * d.Nx * d.Ny * d.Na, nx = 2 * npts * n_vec;
  std::vector<int> sec(2 * n_vec);
  for (int v = 0; v < n_vec; ++v) {
    sec[2 * v] = v & 1;
    sec[2 * v + 1] = (v >> 1) & 1;
  }
  double* x = (double*)dev_alloc(sizeof(double) * nx);
  double* y = (double*)dev_alloc(sizeof(double) * nx);
  FILE* fx = fopen(xpath, "rb");
  if (!fx) return 2;
  rd(fx, x, nx);
  fclose(fx);
  size_t ws = 0;
  if (vdc_co2_ops_workspace_size(m, n_vec, which, &ws) != VDC_OK) {
    printf("vdc_co2_ops_workspace_size: %s\n", vdc_last_error());
    return 3;
  }
  void* w = dev_alloc(ws);
  if (vdc_co2_apply(m, E, which, n_vec, sec.data(), x, y, w, ws, nullptr) != VDC_OK) {
    printf("vdc_co2_apply: %s\n", vdc_last_error());
    return 3;
  }
  printf("done: co2 apply, %zu points, %d vectors\n", npts, n_vec);
  FILE* g = fopen(out, "wb");
  put(g, y, sizeof(double) * nx);
  fclose(g);
  free(x);
  free(y);
  free(w);
  vdc_co2_destroy(m);
  return 0;
}

// co2solve: desc; n_jobs, jobs (vdc_co2_job), n_final, finals [4], opts.
// Writes T (complex [n_jobs][n_final][3]), sigma [n_jobs][n_final] and psi
// (complex [n_jobs][npts]).
int run_co2_solve(const char* dpath, const char* cpath, const char* out) {
  vdc_co2_desc d;
  FILE* f = fopen(dpath, "rb");
  if (!f) return 2;
  rd(f, &d, 1);
  fclose(f);
  vdc_co2_t m;
  if (vdc_co2_create(&d, &m) != VDC_OK) {
    printf("vdc_co2_create: %s\n", vdc_last_error());
    return 3;
  }
  FILE* c = fopen(cpath, "rb");
  if (!c) return 2;
  int nj = 0, nf = 0;
  rd(c, &nj, 1);
  std::vector<vdc_co2_job> jobs(nj);
  rd(c, jobs.data(), nj);
  rd(c, &nf, 1);
  std::vector<int> finals(4 * nf);
  rd(c, finals.data(), 4 * nf);
  vdc_solve_opts o;
  rd(c, &o, 1);
  fclose(c);
  const size_t npts = (size_t)d.Ns * d.Nx * d.Ny * d.Na;
  size_t ws = 0;
  if (vdc_co2_workspace_size(m, &o, nj, jobs.data(), &ws) != VDC_OK) {
    printf("vdc_co2_workspace_size: %s\n", vdc_last_error());
    return 3;
  }
  void* w = dev_alloc(ws);
  double* T = (double*)dev_alloc(sizeof(double) * 2 * nj * nf * 3);
  double* sig = (double*)dev_alloc(sizeof(double) * nj * nf);
  double* psi = (double*)dev_alloc(sizeof(double) * 2 * nj * npts);
  std::vector<vdc_job_info> info(nj);
  if (vdc_co2_solve(m, &o, nj, jobs.data(), nf, finals.data(), T, sig, psi, info.data(), w, ws,
                    nullptr) != VDC_OK) {
    printf("vdc_co2_solve: %s\n", vdc_last_error());
    return 3;
  }
  report(info);
  FILE* g = fopen(out, "wb");
  put(g, T, sizeof(double) * 2 * nj * nf * 3);
  put(g, sig, sizeof(double) * nj * nf);
  put(g, psi, sizeof(double) * 2 * nj * npts);
  fclose(g);
  free(w);
  free(T);
  free(sig);
  free(psi);
  vdc_co2_destroy(m);
  return 0;
}

// terms: D M P, omega[M], nbasis[M], e_state[D], n_u, uterms, n_v, vterms,
// width[D P], K, X, n_jobs, jobs, n_final, finals [VDC_MAX_MODES], opts
int run_terms(const char* path, int dispatch, const char* out) {
  FILE* f = fopen(path, "rb");
  if (!f) return 2;
  int D, M, P;
  rd(f, &D, 1);
  rd(f, &M, 1);
  rd(f, &P, 1);
  std::vector<double> omega(M), es(D);
  std::vector<int> nb(M);
  rd(f, omega.data(), M);
  rd(f, nb.data(), M);
  rd(f, es.data(), D);
  int nu = 0, nv = 0;
  rd(f, &nu, 1);
  std::vector<vdc_term> ut(nu);
  rd(f, ut.data(), nu);
  rd(f, &nv, 1);
  std::vector<vdc_term> vt(nv);
  rd(f, vt.data(), nv);
  std::vector<vdc_width> wd(D * P);
  rd(f, wd.data(), D * P);
  int K = 0;
  double X = 0.0;
  rd(f, &K, 1);
  rd(f, &X, 1);
  int nj = 0;
  rd(f, &nj, 1);
  std::vector<vdc_mjob> jobs(nj);
  rd(f, jobs.data(), nj);
  int nf = 0;
  rd(f, &nf, 1);
  std::vector<int> fin(nf * VDC_MAX_MODES);
  rd(f, fin.data(), fin.size());
  vdc_solve_opts o;
  rd(f, &o, 1);
  fclose(f);
  vdc_model_desc d{D, M, P, omega.data(), nb.data(), es.data(), nu, ut.data(), nv, vt.data(),
                   wd.data(), K, X, dispatch};
  vdc_model_t m;
  if (vdc_model_create(&d, &m) != VDC_OK) {
    printf("vdc_model_create: %s\n", vdc_last_error());
    return 3;
  }
  int kind = -1;
  vdc_model_kind(m, &kind);
  size_t ws = 0;
  if (vdc_model_workspace_size(1, &m, &o, nj, jobs.data(), &ws) != VDC_OK) {
    printf("vdc_model_workspace_size: %s\n", vdc_last_error());
    return 3;
  }
  size_t N = D;
  for (int k = 0; k < M; ++k) N *= nb[k];
  const int npw = kind == 0 ? 2 : P;
  void* w = dev_alloc(ws);
  const size_t nT = 2 * (size_t)nj * nf * npw, nS = (size_t)nj * nf, nP = 2 * (size_t)nj * N;
  double* T = (double*)dev_alloc(sizeof(double) * nT);
  double* sig = (double*)dev_alloc(sizeof(double) * nS);
  double* psi = (double*)dev_alloc(sizeof(double) * nP);
  std::vector<vdc_job_info> info(nj);
  if (vdc_model_solve(1, &m, &o, nj, jobs.data(), nf, fin.data(), w, ws, T, sig, psi,
                      info.data(), nullptr) != VDC_OK) {
    printf("vdc_model_solve: %s\n", vdc_last_error());
    return 3;
  }
  printf("kind %d\n", kind);
  report(info);
  FILE* g = fopen(out, "wb");
  put(g, T, sizeof(double) * nT);
  put(g, sig, sizeof(double) * nS);
  put(g, psi, sizeof(double) * nP);
  fclose(g);
  free(w);
  free(T);
  free(sig);
  free(psi);
  vdc_model_destroy(m);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  setvbuf(stdout, nullptr, _IOLBF, 0);
  const std::string cmd = argc > 1 ? argv[1] : "";
  if (cmd == "solve" && argc == 4) return run_solve(argv[2], argv[3]);
  if (cmd == "co2" && argc == 8)
    return run_co2(argv[2], argv[3], atoi(argv[4]), atoi(argv[5]), atof(argv[6]), argv[7]);
  if (cmd == "terms" && argc == 5) return run_terms(argv[2], atoi(argv[3]), argv[4]);
  if (cmd == "co2solve" && argc == 5) return run_co2_solve(argv[2], argv[3], argv[4]);
  fprintf(stderr, "usage: solve CASE OUT | co2 DESC X N_VEC WHICH E OUT | terms CASE DISPATCH OUT\n");
  return 2;
}
