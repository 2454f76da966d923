// Error-driven adaptive refinement (placeholder until the policy lands).
#include "runtime.h"

using namespace bfi;

extern "C" {

bfi_status bfi_integrate_adaptive(bfi_context *, const bfi_lattice *, bfi_precision, uint64_t,
                                  const double *, const double *, const bfi_adaptive_config *,
                                  const bfi_launch *, bfi_result *, bfi_adaptive_stats *,
                                  uint64_t *, double *, double *, uint64_t *, uint64_t *, size_t,
                                  size_t *)
{
    return fail(BFI_EUNSUPPORTED, "adaptive refinement not built yet");
}

bfi_status bfi_adaptive_decide(const bfi_lattice *, const bfi_subvolumes *, const double *,
                               const double *, const bfi_adaptive_config *, int32_t *)
{
    return fail(BFI_EUNSUPPORTED, "adaptive refinement not built yet");
}

}  // extern "C"
