// Articulated-tree kernels (hinge/slide joints, sphere/capsule geoms against
// world planes): the planar legged chain (7 joints, 5 bodies, 4 foot contact
// slots) and a 3-link test pendulum.
#include "dmx_tree.hpp"
#include "dmx_launch.hpp"

namespace dmx_host {

static const KernelEntry kTree[] = {
    TREE_ENTRY(7, 5, 4, 4), TREE_ENTRY(7, 5, 4, 8), TREE_ENTRY(7, 5, 4, 16), TREE_ENTRY(4, 3, 1, 4),
};

KernelTable tree_kernels() { return {kTree, (int)(sizeof(kTree) / sizeof(kTree[0]))}; }

}  // namespace dmx_host
