// edge_host.hpp - host-side helpers shared by the library's translation
// units (argument checks, launch status, device attributes) and the
// launchers that live in their own units (peeling, grey input).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <stdint.h>

#include "edge_device.hpp"
#include "edge_masks.h"

namespace edgeh {

using namespace edgek;

// hipError_t of the last EDGE_ERR_HIP on this thread (one variable for the
// whole library).
inline thread_local int g_last_hip = 0;

inline int hip_failed(hipError_t e) {
    g_last_hip = (int)e;
    return EDGE_ERR_HIP;
}

inline int launch_status() {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? EDGE_OK : hip_failed(e);
}

constexpr int kMaxDevices = 64;
inline std::atomic<int> g_cu_count[kMaxDevices];

inline int cu_count(int* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_failed(e);
    if (dev >= 0 && dev < kMaxDevices) {
        const int c = g_cu_count[dev].load(std::memory_order_relaxed);
        if (c > 0) { *out = c; return EDGE_OK; }
    }
    int n = 0;
    e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_failed(e);
    if (n <= 0) n = 1;
    if (dev >= 0 && dev < kMaxDevices) g_cu_count[dev].store(n, std::memory_order_relaxed);
    *out = n;
    return EDGE_OK;
}

inline bool cfg_ok(const edge_launch_cfg& c) {
    return (c.vec_words == 1 || c.vec_words == 2 || c.vec_words == 4) && c.rows_per_tile >= 1 &&
           c.rows_per_tile <= 1024 &&
           (c.waves_per_block == 1 || c.waves_per_block == 2 || c.waves_per_block == 4 ||
            c.waves_per_block == 8) &&
           c.blocks_per_cu >= 1 && c.blocks_per_cu <= 32 && c.cache_policy >= EDGE_CACHE_AUTO &&
           c.cache_policy <= EDGE_CACHE_STREAM &&
           (c.shape == EDGE_SHAPE_STRIP ||
            ((c.shape == EDGE_SHAPE_TILE || c.shape == EDGE_SHAPE_TILE_XCD) &&
             c.rows_per_tile <= EDGE_TILE_MAX_ROWS) ||
            ((c.shape == EDGE_SHAPE_BAND || c.shape == EDGE_SHAPE_BAND_XCD) &&
             (c.rows_per_tile == 1 || c.rows_per_tile == 2 || c.rows_per_tile == 4) &&
             c.waves_per_block * c.rows_per_tile >= 3));
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// A dispatch carries its grid size in work-items as a 32-bit number.
inline bool grid_fits(int64_t blocks, int64_t threads_per_block) {
    return blocks >= 0 && blocks * threads_per_block <= (int64_t)UINT32_MAX;
}

inline int64_t pow2_floor(int64_t v) {
    int64_t p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

inline int common_checks(int word_bits, int border, int mode, uint32_t flags, bool batch = false) {
    if (word_bits != 32 && word_bits != 64) return EDGE_ERR_INVALID;
    if (border != EDGE_BORDER_WHITE && border != EDGE_BORDER_BLACK) return EDGE_ERR_INVALID;
    if (mode != EDGE_MODE_MASKS && mode != EDGE_MODE_FULL) return EDGE_ERR_INVALID;
    const uint32_t known = EDGE_FLAG_CLAUSE2_ONLY | EDGE_FLAG_INVERT_OUT |
                           (batch ? (uint32_t)EDGE_FLAG_PLANNED : 0u);
    if (flags & ~known) return EDGE_ERR_INVALID;
    if ((flags & EDGE_FLAG_CLAUSE2_ONLY) && mode != EDGE_MODE_FULL) return EDGE_ERR_INVALID;
    return EDGE_OK;
}

inline int kernel_mode(int mode, uint32_t flags) {
    if (mode == EDGE_MODE_MASKS) return kModePlain;
    return (flags & EDGE_FLAG_CLAUSE2_ONLY) ? kModeClause2 : kModeFull;
}

inline uint32_t border_word(int border) { return border == EDGE_BORDER_WHITE ? 0xffffffffu : 0u; }

inline bool ranges_overlap(uintptr_t a, uint64_t na, uintptr_t b, uint64_t nb) {
    return a < b + nb && b < a + na;
}

inline int alignment_words(uintptr_t p) {
    if (p % 16 == 0) return 4;
    if (p % 8 == 0) return 2;
    return 1;
}

// From this many levels a peel strip's levels are split over two wavefronts.
constexpr int kPeelSplitLevels = 16;

}  // namespace edgeh

namespace edgeh {

// Peeling with 2..31 levels (edge_peel.hip and its level-range units):
// `levels` levels, vw the words per lane the image's alignment allows.
int peel_launch(const edgek::Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels, int vw,
                bool edge_out, hipStream_t s);
int peel_launch_2_7(const edgek::Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels,
                    int vw, bool edge_out, hipStream_t s);
int peel_launch_8_15(const edgek::Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels,
                     int vw, bool edge_out, hipStream_t s);
int peel_launch_16_23(const edgek::Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels,
                      int vw, bool edge_out, hipStream_t s);
int peel_launch_24_31(const edgek::Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels,
                      int vw, bool edge_out, hipStream_t s);

// Grey input (edge_grey.hip): the fused threshold -> edges bands, with the
// kernel mode (kModePlain / kModeFull / kModeClause2) chosen at run time.
int grey_edges_launch(const edgek::Geom& g, const edge_launch_cfg& c, uint32_t bw, int invert,
                      bool aligned, int kmode, hipStream_t s);
// Threshold + pack: one thread per 32-bit output word, `blocks` blocks of
// 256; nt: non-temporal stores.
int pack_launch(const uint8_t* grey, int64_t gstride, uint32_t* out, int64_t stride,
                int32_t height, int32_t width, int32_t wd32, uint32_t thr, bool aligned, bool nt,
                int64_t blocks, hipStream_t s);

}  // namespace edgeh
