// Entry points whose kernels are not written yet.
#include "plan.hpp"

namespace shg {
size_t adjoint_ws_bytes(const Plan&) { return 0; }
void free_adjoint(Plan&) {}
int propagate_temp(Plan&, void*, void*, const double*, const void*, int, int, void*, double*,
                   hipStream_t) {
  return fail(SHG_EUNSUPPORTED, "temperature fields are not supported yet");
}
}  // namespace shg

using namespace shg;
extern "C" {
int shg_propagate_adjoint(shg_plan*, const void*, const void*, const double*, const void*,
                          const void*, const void*, const double*, void*, void*, double*, double*,
                          void*, void*, double*, void*, void*) {
  return fail(SHG_EUNSUPPORTED, "adjoint not supported yet");
}
int shg_propagate_batch(int32_t n, shg_plan* const*, void* const*, void* const*,
                        const double* const*, void*, double*, void*) {
  if (n < 1) return fail(SHG_EINVAL, "n=%d must be >= 1", n);
  return fail(SHG_EUNSUPPORTED, "batch not supported yet");
}
size_t shg_batch_workspace_bytes(int32_t, shg_plan* const*) { return 0; }
}
