// edge_peel_2_7.hip - peeling kernels for 2 to 7 levels.
#include "edge_peel.hpp"

namespace edgeh {

int peel_launch_2_7(const Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels, int vw,
                    bool edge_out, hipStream_t s) {
    return launch_peel_range<2, 7>(g, c, bw, levels, vw, edge_out, s);
}

}  // namespace edgeh
