// Free-body kernels (one body on a free joint, sphere/capsule/box geoms
// against world planes) with one to four contact slots (the sphere, the capsule, the box geom), for each compiled team size.
#include "dmx_launch.hpp"

namespace dmx_host {

static const KernelEntry kEntries[] = {
    FREE_ENTRY(1, 1), FREE_ENTRY(2, 1), FREE_ENTRY(2, 2), FREE_ENTRY(4, 1), FREE_ENTRY(4, 4), FREE_ENTRY(4, 8),
};

KernelTable free_kernels_small() { return {kEntries, (int)(sizeof(kEntries) / sizeof(kEntries[0]))}; }

}  // namespace dmx_host
