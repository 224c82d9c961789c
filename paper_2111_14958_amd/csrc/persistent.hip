// Persistent chunk kernel (placeholder until the grid-barrier kernel lands).
#include "cg_host.h"

namespace wd {
int record_persistent_chunk(int, const LaunchSet &, hipStream_t, const Prob *, int, int, void *) {
    return fail(WD_EINVAL, "persistent CG kernel not available in this build");
}
}  // namespace wd
