// Free-body kernels (one body on a free joint, sphere/capsule/box geoms
// against world planes) with eight contact slots (the corner-sphere cube), for each compiled team size.
#include "dmx_launch.hpp"

namespace dmx_host {

static const KernelEntry kEntries[] = {
    FREE_ENTRY(8, 1), FREE_ENTRY(8, 2), FREE_ENTRY(8, 4), FREE_ENTRY(8, 8), FREE_ENTRY(8, 16),
};

KernelTable free_kernels() { return {kEntries, (int)(sizeof(kEntries) / sizeof(kEntries[0]))}; }

}  // namespace dmx_host
