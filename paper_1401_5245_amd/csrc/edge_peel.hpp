// edge_peel.hpp - iterated peeling kernels and their launchers, included by
// the units that instantiate each range of level counts (one kernel per
// level count keeps every level's rows in registers; splitting the counts
// over several units lets them compile in parallel).
#pragma once

#include "edge_host.hpp"

namespace edgeh {

using namespace edgek;

// Iterated peeling of one image: strips of `rows` rows x kPeelSpan words,
// one wavefront per strip, L levels.
template <int L, bool EDGEOUT, class Pol>
__global__ void __launch_bounds__(512) k_peel(Geom g, int64_t chunks, int rows, int64_t nunits,
                                              uint32_t bw, int wpb) {
    const int64_t unit = (int64_t)xcd_block(blockIdx.x, gridDim.x) * wpb +
                         wave_uniform(threadIdx.x / kWave);
    if (unit >= nunits) return;
    const int64_t strip = unit / chunks;
    const int64_t chunk = unit - strip * chunks;
    const int64_t y0 = strip * rows;
    const int64_t y1 = y0 + rows < g.height ? y0 + rows : g.height;
    peel_unit<L, EDGEOUT, Pol>(g, chunk, (int)y0, (int)y1, bw);
}

// Iterated peeling with VW words per lane: strips of `rows` rows x 64*VW
// words, one wavefront per strip, L levels.
template <int L, bool EDGEOUT, int VW>
__global__ void __launch_bounds__(512) k_peel_vec(Geom g, int64_t chunks, int rows,
                                                  int64_t nunits, uint32_t bw, int wpb) {
    const int64_t unit = (int64_t)xcd_block(blockIdx.x, gridDim.x) * wpb +
                         wave_uniform(threadIdx.x / kWave);
    if (unit >= nunits) return;
    const int64_t strip = unit / chunks;
    const int64_t chunk = unit - strip * chunks;
    const int64_t y0 = strip * rows;
    const int64_t y1 = y0 + rows < g.height ? y0 + rows : g.height;
    const int j0 = (int)(chunk * kWave * VW);
    if (j0 + kWave * VW <= g.wd)
        peel_vec_unit<L, EDGEOUT, VW, true, CachedStrip>(g, j0, (int)y0, (int)y1, bw);
    else
        peel_vec_unit<L, EDGEOUT, VW, false, CachedStrip>(g, j0, (int)y0, (int)y1, bw);
}

// Iterated peeling with a strip's levels split over the two wavefronts of
// a workgroup (one strip per workgroup, so both leave together).
template <int LA, int LB, bool EDGEOUT>
__global__ void __launch_bounds__(2 * kWave) k_peel_split(Geom g, int64_t chunks, int rows,
                                                         int64_t nunits, uint32_t bw) {
    __shared__ uint32_t xfer[2 * kPeelSplitGroup][kWave];
    const int64_t unit = (int64_t)xcd_block(blockIdx.x, gridDim.x);
    if (unit >= nunits) return;
    const int role = wave_uniform(threadIdx.x / kWave);
    const int64_t strip = unit / chunks;
    const int64_t chunk = unit - strip * chunks;
    const int64_t y0 = strip * rows;
    const int64_t y1 = y0 + rows < g.height ? y0 + rows : g.height;
    peel_split_unit<LA, LB, EDGEOUT, CachedStrip>(g, chunk, (int)y0, (int)y1, bw, role, xfer);
}

template <int L, bool EDGEOUT>
int launch_peel_kernel(const Geom& g, const edge_launch_cfg& c, uint32_t bw, hipStream_t s) {
    const int64_t chunks = ceil_div(g.wd, (int64_t)kPeelSpan);
    const int64_t nunits = chunks * ceil_div(g.height, c.rows_per_tile);
    const int64_t blocks = ceil_div(nunits, c.waves_per_block);
    if (!grid_fits(blocks, c.waves_per_block * kWave)) return EDGE_ERR_UNSUPPORTED;
    hipLaunchKernelGGL((k_peel<L, EDGEOUT, CachedStrip>), dim3((uint32_t)blocks),
                       dim3(c.waves_per_block * kWave), 0, s, g, chunks, c.rows_per_tile, nunits,
                       bw, c.waves_per_block);
    return launch_status();
}

template <int L, bool EDGEOUT, int VW>
int launch_peel_vec_kernel(const Geom& g, const edge_launch_cfg& c, uint32_t bw, hipStream_t s) {
    const int64_t chunks = ceil_div(g.wd, (int64_t)kWave * VW);
    const int64_t nunits = chunks * ceil_div(g.height, c.rows_per_tile);
    const int64_t blocks = ceil_div(nunits, c.waves_per_block);
    if (!grid_fits(blocks, c.waves_per_block * kWave)) return EDGE_ERR_UNSUPPORTED;
    hipLaunchKernelGGL((k_peel_vec<L, EDGEOUT, VW>), dim3((uint32_t)blocks),
                       dim3(c.waves_per_block * kWave), 0, s, g, chunks, c.rows_per_tile, nunits,
                       bw, c.waves_per_block);
    return launch_status();
}

template <int L, bool EDGEOUT>
int launch_peel_split_kernel(const Geom& g, const edge_launch_cfg& c, uint32_t bw,
                             hipStream_t s) {
    const int64_t chunks = ceil_div(g.wd, (int64_t)kPeelSpan);
    const int64_t nunits = chunks * ceil_div(g.height, c.rows_per_tile);
    if (!grid_fits(nunits, 2 * kWave)) return EDGE_ERR_UNSUPPORTED;
    constexpr int LA = peel_split_first(L);
    hipLaunchKernelGGL((k_peel_split<LA, L - LA, EDGEOUT>), dim3((uint32_t)nunits),
                       dim3(2 * kWave), 0, s, g, chunks, c.rows_per_tile, nunits, bw);
    return launch_status();
}

// One instantiation per level count LO..HI (levels are a template constant
// so that every level's rows stay in registers).
// vw: words per lane that the image's alignment allows (2 or 4 select the
// vector-width unit up to kPeelVecLevels levels).
template <int L, int HI, bool EDGEOUT>
int launch_peel(const Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels, int vw,
                hipStream_t s) {
    if constexpr (L > HI) {
        return EDGE_ERR_INVALID;
    } else {
        if (levels == L) {
            if constexpr (L >= kPeelSplitLevels) {
                return launch_peel_split_kernel<L, EDGEOUT>(g, c, bw, s);
            } else if constexpr (L <= kPeelVecLevels) {
                if (vw == 4) return launch_peel_vec_kernel<L, EDGEOUT, 4>(g, c, bw, s);
                if (vw == 2) return launch_peel_vec_kernel<L, EDGEOUT, 2>(g, c, bw, s);
                return launch_peel_kernel<L, EDGEOUT>(g, c, bw, s);
            } else {
                return launch_peel_kernel<L, EDGEOUT>(g, c, bw, s);
            }
        }
        return launch_peel<L + 1, HI, EDGEOUT>(g, c, bw, levels, vw, s);
    }
}

template <int LO, int HI>
int launch_peel_range(const Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels, int vw,
                      bool edge_out, hipStream_t s) {
    if (edge_out) return launch_peel<LO, HI, true>(g, c, bw, levels, vw, s);
    return launch_peel<LO, HI, false>(g, c, bw, levels, vw, s);
}

}  // namespace edgeh
