// edge_peel_24_31.hip - peeling kernels for 24 to 31 levels.
#include "edge_peel.hpp"

namespace edgeh {

int peel_launch_24_31(const Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels, int vw,
                      bool edge_out, hipStream_t s) {
    return launch_peel_range<24, 31>(g, c, bw, levels, vw, edge_out, s);
}

}  // namespace edgeh
