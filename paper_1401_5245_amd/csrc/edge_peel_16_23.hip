// edge_peel_16_23.hip - peeling kernels for 16 to 23 levels.
#include "edge_peel.hpp"

namespace edgeh {

int peel_launch_16_23(const Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels, int vw,
                      bool edge_out, hipStream_t s) {
    return launch_peel_range<16, 23>(g, c, bw, levels, vw, edge_out, s);
}

}  // namespace edgeh
