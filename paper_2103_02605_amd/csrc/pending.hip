// Entry points still to be written: they validate nothing yet and report EINVAL.
#include <hip/hip_runtime.h>

#include "host.hpp"

namespace fcirc {
}  // namespace fcirc

extern "C" {
fcirc_status fcirc_matvec_fwd_shared(fcirc_ctx*, const void*, const void*, void*, uint64_t, uint32_t, fcirc_ring, void*) {
  return FCIRC_EINVAL;
}
fcirc_status fcirc_matvec_backward(fcirc_ctx*, const void*, const void*, const void*, void*, void*, uint64_t, uint32_t,
                                   fcirc_ring, void*) {
  return FCIRC_EINVAL;
}
}
