// edge_grey.hip - grey-image kernels (section 7: a grey image is made binary
// by a threshold): threshold + pack, and the threshold fused into the edge
// pass so that the binary image never reaches memory.
#include "edge_host.hpp"

namespace edgeh {

using namespace edgek;

// Grey image in, edge map out: units are bands of nw * RW - 2 output rows
// of one 64-word chunk, one per workgroup; a grid smaller than the unit
// count (very tall images) takes them in turns, the LDS tile reused after
// a barrier.
template <int MODE, int RW, bool ALIGNED, class Pol>
__global__ void __launch_bounds__(512) k_grey_band(Geom g, int64_t chunks, int64_t nunits,
                                                   uint32_t bw, int invert, int nw) {
    extern __shared__ uint32_t band_tile[];
    for (int64_t unit = xcd_block(blockIdx.x, gridDim.x); unit < nunits; unit += gridDim.x) {
        const int64_t band = unit / chunks;
        const int64_t chunk = unit - band * chunks;
        const int j0 = (int)(chunk * kWave);
        if (32ll * (j0 + kWave) <= g.width)
            grey_band_unit<MODE, RW, ALIGNED, true, Pol>(g, band_tile, nw, j0, band * (nw * RW - 2),
                                                         bw, invert != 0);
        else
            grey_band_unit<MODE, RW, ALIGNED, false, Pol>(g, band_tile, nw, j0, band * (nw * RW - 2),
                                                          bw, invert != 0);
        if (unit + gridDim.x < nunits) __syncthreads();
    }
}

// Threshold binarisation + packing (section 7: a grey image is first made
// binary by a threshold): one 32-bit output word per thread, from the 16-byte
// blocks that hold its 32 grey bytes; a byte >= thr becomes white (1). Rows
// of `gstride` bytes in, packed rows of `stride` 32-bit words out; bits past
// the width are 0. ALIGNED: the grey pointer and pitch are 16-byte aligned.
// NT: non-temporal stores (packed images too large to stay cached for the
// pass that reads them next).
template <bool ALIGNED, bool NT>
__global__ void __launch_bounds__(256) k_pack(const uint8_t* grey, int64_t gstride, uint32_t* out,
                                              int64_t stride, int32_t height, int32_t width,
                                              int32_t wd, uint32_t thr) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;    // launched with 256 threads
    if (t >= (int64_t)height * wd) return;
    const int64_t y = t / wd;
    const int j = (int)(t - y * wd);
    const uint8_t* rp = grey + y * gstride;
    const GreyBlocks<ALIGNED> q = load_grey_word<ALIGNED, false>(rp, j, width);
    const uint32_t v = grey_word<ALIGNED>(q, rp, thr) & valid_bits(j, width);
    if constexpr (NT) __builtin_nontemporal_store(v, out + y * stride + j);
    else out[y * stride + j] = v;
}

// Workgroups of one grey-band launch at most (2^22 x 512 threads stays
// below the grid's 2^32 threads); beyond, each takes several bands.
constexpr int64_t kMaxBandBlocks = int64_t(1) << 22;

template <int MODE, int RW, bool ALIGNED, class Pol>
int launch_grey_band_rw(const Geom& g, int nw, int64_t chunks, uint32_t bw, int invert,
                        hipStream_t stream) {
    const int64_t nunits = chunks * ceil_div(g.height, (int64_t)(nw * RW - 2));
    const int64_t blocks = std::min<int64_t>(nunits, kMaxBandBlocks);
    const size_t lds = (size_t)nw * RW * kBandPitch * sizeof(uint32_t);
    hipLaunchKernelGGL((k_grey_band<MODE, RW, ALIGNED, Pol>), dim3((uint32_t)blocks),
                       dim3(nw * kWave), lds, stream, g, chunks, nunits, bw, invert, nw);
    return launch_status();
}

// Band shape from the launch shape: waves_per_block wavefronts, each
// loading rows_per_tile rows rounded down to 2, 4 or 8 (a band loads at
// least four rows).
template <int MODE, bool ALIGNED, class Pol>
int launch_grey_band(const Geom& g, const edge_launch_cfg& c, uint32_t bw, int invert,
                     hipStream_t stream) {
    const int64_t chunks = ceil_div(g.wd, (int64_t)kWave);
    const int nw = c.waves_per_block;
    int rw = c.rows_per_tile >= 8 ? 8 : (c.rows_per_tile >= 4 ? 4 : 2);
    while (nw * rw < 4) rw *= 2;
    if (rw == 8) return launch_grey_band_rw<MODE, 8, ALIGNED, Pol>(g, nw, chunks, bw, invert, stream);
    if (rw == 4) return launch_grey_band_rw<MODE, 4, ALIGNED, Pol>(g, nw, chunks, bw, invert, stream);
    return launch_grey_band_rw<MODE, 2, ALIGNED, Pol>(g, nw, chunks, bw, invert, stream);
}

// Rows that start on 16-byte boundaries (pointer and pitch) load two
// blocks per word, others three. The cache policy: AUTO (the built-in)
// keeps the loads cached, since bands re-read their first and last rows
// from the cache, and makes the stores non-temporal, since the edge map is
// not read back (8192^2 / 16384^2 / 65536^2: 17.3 / 54.5 / 835 us against
// 18.5 / 58.3 / 864 us with cached stores); NORMAL keeps both cached;
// STREAM makes both non-temporal (slower at every size measured: a lane's
// two loads take alternate 16-byte halves of the same cache lines in two
// instructions, and non-temporal loads fetch such lines again for the
// second; a wavefront reading 1 KiB contiguous per load with non-temporal
// loads, its lanes then exchanging half-words, ran at the AUTO policy's
// speed, not faster).
template <int MODE, bool ALIGNED>
int launch_grey_aligned(const Geom& g, const edge_launch_cfg& c, uint32_t bw, int invert,
                        hipStream_t stream) {
    if (c.cache_policy == EDGE_CACHE_STREAM)
        return launch_grey_band<MODE, ALIGNED, StreamingStrip>(g, c, bw, invert, stream);
    if (c.cache_policy == EDGE_CACHE_NORMAL)
        return launch_grey_band<MODE, ALIGNED, CachedStrip>(g, c, bw, invert, stream);
    return launch_grey_band<MODE, ALIGNED, StreamOutStrip>(g, c, bw, invert, stream);
}

template <int MODE>
int launch_grey(const Geom& g, const edge_launch_cfg& c, uint32_t bw, int invert, bool aligned,
                hipStream_t stream) {
    return aligned ? launch_grey_aligned<MODE, true>(g, c, bw, invert, stream)
                   : launch_grey_aligned<MODE, false>(g, c, bw, invert, stream);
}

int grey_edges_launch(const Geom& g, const edge_launch_cfg& c, uint32_t bw, int invert,
                      bool aligned, int kmode, hipStream_t s) {
    switch (kmode) {
        case kModePlain: return launch_grey<kModePlain>(g, c, bw, invert, aligned, s);
        case kModeFull: return launch_grey<kModeFull>(g, c, bw, invert, aligned, s);
        default: return launch_grey<kModeClause2>(g, c, bw, invert, aligned, s);
    }
}

int pack_launch(const uint8_t* grey, int64_t gstride, uint32_t* out, int64_t stride,
                int32_t height, int32_t width, int32_t wd, uint32_t thr, bool aligned, bool nt,
                int64_t blocks, hipStream_t s) {
    const dim3 grid((uint32_t)blocks), block(256);
    if (aligned && nt)
        hipLaunchKernelGGL((k_pack<true, true>), grid, block, 0, s, grey, gstride, out, stride,
                           height, width, wd, thr);
    else if (aligned)
        hipLaunchKernelGGL((k_pack<true, false>), grid, block, 0, s, grey, gstride, out, stride,
                           height, width, wd, thr);
    else if (nt)
        hipLaunchKernelGGL((k_pack<false, true>), grid, block, 0, s, grey, gstride, out, stride,
                           height, width, wd, thr);
    else
        hipLaunchKernelGGL((k_pack<false, false>), grid, block, 0, s, grey, gstride, out, stride,
                           height, width, wd, thr);
    return launch_status();
}

}  // namespace edgeh
