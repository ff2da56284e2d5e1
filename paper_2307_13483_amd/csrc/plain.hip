// Plain single-solve path (placeholder until the kernels land).
#include <string>
#include <vector>
#include "solve_args.h"

namespace vdc {
vdc_status solve_plain_impl(const SolveArgs&, const std::vector<DevJob>&,
                            const std::vector<DevModel>&, hipStream_t, std::string& err) {
  err = "plain path not built yet";
  return VDC_ERR_UNSUPPORTED;
}
}  // namespace vdc
