// Launch arguments of the energy-loss spectrum kernel (eels.hip).
#pragma once
#include "internal.h"
#include "op2d.h"

namespace vdc {

struct EelsJob {
  double eps_i, E, Evi;   // incident energy, total energy, E_{v_i}
  int out;                // row of S
};

struct EelsArgs {
  const DevModel* model;
  const EelsJob* jobs;
  int n_jobs;
  const c64* psi;         // [job][2 Nc] full layout, row length psi_ld
  size_t psi_ld;
  const int* order;       // [Nc] final states g Nu + u, by vibrational energy
  const double* Evf;      // [Nc] their energies, ascending
  double* share;          // [groups][Nc] scratch
  int* counter;
  int n_grid;
  double d0, dd, fwhm;
  double* S;              // [n_jobs][n_grid]
};

hipError_t launch_eels(const EelsArgs& a, int n_groups, hipStream_t s);

}  // namespace vdc
