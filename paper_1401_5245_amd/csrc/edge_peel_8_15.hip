// edge_peel_8_15.hip - peeling kernels for 8 to 15 levels.
#include "edge_peel.hpp"

namespace edgeh {

int peel_launch_8_15(const Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels, int vw,
                     bool edge_out, hipStream_t s) {
    return launch_peel_range<8, 15>(g, c, bw, levels, vw, edge_out, s);
}

}  // namespace edgeh
