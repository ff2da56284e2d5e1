// FGMRES with an FP32 inner GMRES (placeholder until the kernel lands).
#include "solve_args.h"

namespace vdc {
hipError_t launch_fgmres_mixed(const SolveArgs&, int, hipStream_t) { return hipErrorNotSupported; }
int fgmres_mixed_occupancy() { return 1; }
}  // namespace vdc
