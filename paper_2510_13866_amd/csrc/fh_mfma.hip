// Placeholder until the MFMA forward filter lands.
#include "fh_internal.h"
namespace fh {
hipError_t launch_forward_mfma(fh_plan, const void*, const int32_t*, hipStream_t) { return hipErrorNotSupported; }
}  // namespace fh
