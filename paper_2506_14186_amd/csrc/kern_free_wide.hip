// Free-body kernels (one body on a free joint, sphere/capsule/box geoms
// against world planes) with sixteen contact slots, for each compiled team size.
#include "dmx_launch.hpp"

namespace dmx_host {

static const KernelEntry kEntries[] = {
    FREE_ENTRY(16, 8), FREE_ENTRY(16, 16),
};

KernelTable free_kernels_wide() { return {kEntries, (int)(sizeof(kEntries) / sizeof(kEntries[0]))}; }

}  // namespace dmx_host
