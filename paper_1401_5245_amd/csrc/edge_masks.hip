// edge_masks.hip - kernels and C ABI of libedgemask (gfx950).
//
// Entry points are declared and documented in include/edge_masks.h. Every
// entry point validates its arguments on the host before any HIP call,
// chooses a launch shape, and enqueues asynchronously on the caller's
// stream. The library allocates no device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <stdint.h>
#include <string.h>

#include "edge_host.hpp"

using namespace edgek;
using namespace edgeh;

static_assert(kTileMaxRows == EDGE_TILE_MAX_ROWS, "tile height of the kernels and the ABI");

static_assert(kMaxHeight == EDGE_MAX_HEIGHT, "one height limit for the header and the kernels");

// ================================================================ kernels ===

// One image, strips of `rows` rows x 64*VW words, one wavefront per strip
// (for a tile policy, rows <= its height). by_xcd: workgroups regrouped by
// XCD, so that vertically adjacent strips share one L2 (always for strips);
// else the dispatch order. wpb: wavefronts per workgroup, passed in
// (reading the workgroup size costs every wavefront a dependent load
// before its first unit).
template <int VW, int MODE, class Pol>
__global__ void __launch_bounds__(512) k_strip(Geom g, int64_t chunks, int rows, int64_t nunits,
                                               uint32_t bw, int invert, int wpb, int by_xcd) {
    const uint32_t b = by_xcd ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int64_t unit = (int64_t)b * wpb + wave_uniform(threadIdx.x / kWave);
    if (unit >= nunits) return;
    const int64_t strip = unit / chunks;
    const int64_t chunk = unit - strip * chunks;
    const int64_t y0 = strip * rows;
    const int64_t y1 = y0 + rows < g.height ? y0 + rows : g.height;
    strip_unit<VW, MODE, Pol>(g, (int)(chunk * kWave * VW), (int)y0, (int)y1, bw, invert != 0);
}

// One image in bands (band_unit): one band of one chunk per workgroup of nw
// wavefronts, nw * RW - 2 rows per band; by_xcd as for k_strip.
template <int VW, int RW, int MODE>
__global__ void __launch_bounds__(512) k_band(Geom g, int64_t chunks, int64_t nunits, uint32_t bw,
                                              int invert, int nw, int by_xcd) {
    extern __shared__ __align__(16) uint32_t band_lds[];
    const uint32_t b = by_xcd ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    if ((int64_t)b >= nunits) return;      // the whole workgroup: no barrier is split
    const int64_t band = (int64_t)b / chunks;
    const int64_t chunk = (int64_t)b - band * chunks;
    band_unit<VW, RW, MODE>(g, band_lds, nw, (int)(chunk * kWave * VW), band * (nw * RW - 2), bw,
                            invert != 0);
}

// One image with rows of <= 32 words, `band` rows per wavefront.
template <int MODE>
__global__ void __launch_bounds__(512) k_narrow(Geom g, int64_t band, int64_t nunits, uint32_t bw,
                                                int invert, int wpb) {
    const int64_t unit = (int64_t)xcd_block(blockIdx.x, gridDim.x) * wpb +
                         wave_uniform(threadIdx.x / kWave);
    if (unit >= nunits) return;
    const int64_t ya = unit * band;
    const int64_t yb = ya + band < g.height ? ya + band : g.height;
    narrow_unit<MODE>(g, (int)ya, (int)yb, bw, invert != 0);
}

// Descriptor check shared by the host validator and the device planner:
// sizes and offset non-negative, stride >= the row's words, and every word
// of the image inside the arena. Division-free for strides below 2^32.
__host__ __device__ static inline bool desc_ok(const edge_image_desc& d, int64_t arena_words,
                                               int word_bits) {
    if (d.height < 0 || d.width < 0 || d.offset_words < 0 || d.stride_words < 0) return false;
    if (d.height > kMaxHeight) return false;
    if (d.height == 0 || d.width == 0) return true;
    const int shift = word_bits == 64 ? 6 : 5;
    const int64_t wd = ((int64_t)d.width + word_bits - 1) >> shift;
    if (d.stride_words < wd || wd > arena_words || d.offset_words > arena_words) return false;
    if (d.stride_words < (1ll << 32)) {
        const int64_t span = (int64_t)(d.height - 1) * d.stride_words + wd;   // < 2^63
        return span <= arena_words - d.offset_words;
    }
    if ((int64_t)(d.height - 1) > (arena_words - wd) / d.stride_words) return false;
    const int64_t span = (int64_t)(d.height - 1) * d.stride_words + wd;
    return d.offset_words <= arena_words - span;
}

// Work plan (the batch workspace), int64 words:
//   [0] total units, [1] skipped descriptors, [2] kPlanMagic ^ n,
//   [3] persistent wavefronts the plan was made for (nw), [4..7] reserved;
//   [8 ...] n + 1 image records (PlanImage, 6 words each; record n holds
//   only the total, as the first unit past the last image);
//   then nw + 1 wavefront entries (PlanWave, 9 words each): wavefront w
//   starts at unit floor(total * w / nw), and its entry also holds the
//   image of that unit, the first unit of the next image and a copy of the
//   image's record, so that a wavefront reaches its first unit's geometry
//   with the loads of the header (entry nw: first unit = total).
// Either planner writes it: the device planner (k_plan) or the host planner
// (edge_batch_plan). The batch kernel reads only the plan, never the table.
constexpr int kWsHeader = 8;
constexpr int64_t kPlanMagic = 0x45444745504c414ell;   // "EDGEPLAN"
constexpr int kMaxBatchWaves = 65536;
constexpr int kPlanThreads = 1024;

// One image of the plan: its geometry in 32-bit words and how it is cut
// into units, so that the batch kernel does no division or re-validation
// of the descriptor beyond one bounds test.
struct PlanImage {
    int64_t first;      // first unit of the image
    int64_t off32;      // first word of the image (32-bit words from the arena start)
    int64_t stride32;   // row pitch (32-bit words)
    int32_t height, width;
    int32_t wd32;       // 32-bit words per row
    int32_t band;       // rows per unit
    int32_t split;      // strips: 64*vw-word chunks per row; narrow units: rows per step
    uint32_t kind;      // bits 0-2: strip words per lane (1, 2, 4), 0 for narrow
                        // units, 7 for an image without work; bits 8-31
                        // (narrow units): ceil(2^16 / wd32), so that
                        // lane / wd32 = (lane * that) >> 16 for lanes < 64
};
static_assert(sizeof(PlanImage) == 48, "six int64 words per image record");
constexpr int kPlanRecWords = sizeof(PlanImage) / 8;
constexpr uint32_t kKindIdle = 7;

struct PlanWave {
    int64_t first;      // first unit of the wavefront
    int64_t next;       // first unit of the image after `image`
    int32_t image;      // image holding unit `first`
    int32_t reserved;
    PlanImage rec;      // that image's record
};
static_assert(sizeof(PlanWave) == 72, "nine int64 words per wavefront entry");
constexpr int kPlanWaveWords = sizeof(PlanWave) / 8;

__host__ __device__ constexpr int64_t ws_wave_offset(int32_t n) {
    return kWsHeader + (int64_t)(n + 1) * kPlanRecWords;
}
// Bytes of the plan for n images and nw wavefronts; the workspace holds the
// plan of the largest grid.
__host__ __device__ constexpr int64_t ws_plan_bytes(int32_t n, int64_t nw) {
    return (ws_wave_offset(n) + (nw + 1) * kPlanWaveWords) * 8;
}
__host__ __device__ constexpr int64_t ws_bytes(int32_t n) {
    return ws_plan_bytes(n, kMaxBatchWaves);
}

// Record of descriptor d (kind kKindIdle when it has no work); returns its
// units. *bad is set when the descriptor fails the checks of desc_ok.
__host__ __device__ inline int64_t plan_image(const edge_image_desc& d, int64_t arena_words,
                                              int word_bits, int vmax, int rows, PlanImage* r,
                                              int* bad) {
    *r = PlanImage{0, 0, 0, 0, 0, 0, 1, 1, kKindIdle};
    if (!desc_ok(d, arena_words, word_bits)) {
        *bad = 1;
        return 0;
    }
    if (d.height == 0 || d.width == 0) return 0;
    const int per = word_bits / 32;
    const int shift = word_bits == 64 ? 6 : 5;
    const int64_t wd32 = (((int64_t)d.width + word_bits - 1) >> shift) * per;
    const UnitShape s = unit_shape(d.height, d.width, wd32, d.offset_words * per,
                                   d.stride_words * per, vmax, rows);
    r->off32 = d.offset_words * per;
    r->stride32 = d.stride_words * per;
    r->height = d.height;
    r->width = d.width;
    r->wd32 = (int32_t)wd32;
    r->band = (int32_t)s.band;
    if (s.narrow) {
        r->split = kWave / (int)wd32;
        r->kind = (uint32_t)((65536 + wd32 - 1) / wd32) << 8;
    } else {
        r->split = (int32_t)s.chunks;
        r->kind = (uint32_t)s.vw;
    }
    return s.count;
}

// Units of descriptor d (0 when it fails the checks; *bad counts those).
__device__ __forceinline__ int64_t desc_units(const edge_image_desc& d, int64_t arena_words,
                                              int word_bits, int vmax, int rows, int* bad) {
    if (!desc_ok(d, arena_words, word_bits)) {
        ++*bad;
        return 0;
    }
    const int per = word_bits / 32;
    const int shift = word_bits == 64 ? 6 : 5;
    const int64_t wd = (((int64_t)d.width + word_bits - 1) >> shift) * per;
    return unit_shape(d.height, d.width, wd, d.offset_words * per, d.stride_words * per, vmax,
                      rows).count;
}

// Batch planner: one workgroup; thread t owns the contiguous images
// [t*per, (t+1)*per). It counts their work units (the first kKeep counts
// stay in registers), one workgroup scan turns the chunk sums into each
// image's first unit, each thread writes its images' records, and then the
// wavefront map for the wavefronts whose first unit falls inside its chunk
// (wavefront w's first unit is floor(total * w / nw)).
constexpr int kKeep = 8;

__global__ void __launch_bounds__(kPlanThreads) k_plan(const edge_image_desc* tab, int n,
                                                       int64_t arena_words, int word_bits,
                                                       int vmax, int rows, int nw, int64_t* ws) {
    __shared__ int64_t wave_sum[kPlanThreads / kWave];
    __shared__ int bad_count;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int per = (n + kPlanThreads - 1) / kPlanThreads;
    const int i0 = min(n, tid * per), i1 = min(n, i0 + per);
    PlanImage* rec = reinterpret_cast<PlanImage*>(ws + kWsHeader);
    PlanWave* wv = reinterpret_cast<PlanWave*>(ws + ws_wave_offset(n));
    if (n == 0) {               // nothing to plan (a graph may be captured with n = 0)
        if (tid == 0) {
            ws[0] = 0;
            ws[1] = 0;
            ws[2] = kPlanMagic;
            ws[3] = nw;
        }
        return;
    }
    if (tid == 0) bad_count = 0;
    __syncthreads();

    // All descriptor loads first (clamped indices, no branches), then the
    // arithmetic, so the loads overlap instead of completing one by one.
    edge_image_desc dd[kKeep];
#pragma unroll
    for (int k = 0; k < kKeep; ++k) dd[k] = tab[min(i0 + k, n - 1)];
    int bad = 0;
    int64_t mine = 0;
    int64_t cnt[kKeep];
#pragma unroll
    for (int k = 0; k < kKeep; ++k) {
        int b = 0;
        const int64_t c = desc_units(dd[k], arena_words, word_bits, vmax, rows, &b);
        const bool mine_k = i0 + k < i1;
        cnt[k] = mine_k ? c : 0;
        bad += mine_k ? b : 0;
        mine += cnt[k];
    }
    for (int i = i0 + kKeep; i < i1; ++i)
        mine += desc_units(tab[i], arena_words, word_bits, vmax, rows, &bad);
    if (bad) atomicAdd(&bad_count, bad);

    int64_t x = mine;                                  // inclusive scan of the chunk sums
    for (int off = 1; off < kWave; off <<= 1) {
        const int64_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) wave_sum[wave] = x;
    __syncthreads();
    int64_t before = 0, total = 0;
    for (int w = 0; w < kPlanThreads / kWave; ++w) {
        const int64_t v = wave_sum[w];
        if (w < wave) before += v;
        total += v;
    }
    const int64_t u_first = before + x - mine;         // first unit of image i0

    int unused = 0;
    int64_t u = u_first;
#pragma unroll
    for (int k = 0; k < kKeep; ++k) {
        if (i0 + k < i1) {
            PlanImage r;
            plan_image(dd[k], arena_words, word_bits, vmax, rows, &r, &unused);
            r.first = u;
            rec[i0 + k] = r;
        }
        u += cnt[k];
    }
    for (int i = i0 + kKeep; i < i1; ++i) {
        PlanImage r;
        const int64_t c = plan_image(tab[i], arena_words, word_bits, vmax, rows, &r, &unused);
        r.first = u;
        rec[i] = r;
        u += c;
    }

    const PlanImage idle{0, 0, 0, 0, 0, 0, 1, 1, kKindIdle};
    if (total == 0) {                                  // no work: every wavefront empty
        for (int w = tid; w <= nw; w += kPlanThreads) wv[w] = PlanWave{0, 0, 0, 0, idle};
    } else if (mine > 0) {
        // wavefronts w with floor(total*w/nw) in [u_first, u_first + mine)
        const int64_t w_lo = (u_first * nw + total - 1) / total;
        const int64_t w_hi = min((int64_t)nw, ((u_first + mine) * nw + total - 1) / total);
        int i = i0;
        int64_t s_i = u_first;                            // first unit of image i
        for (int64_t w = w_lo; w < w_hi; ++w) {
            const int64_t uw = total * w / nw;
            int64_t c;                                     // units of image i
            for (;;) {
                const int k = i - i0;
                c = 0;
#pragma unroll
                for (int q = 0; q < kKeep; ++q) c = (q == k) ? cnt[q] : c;
                if (k >= kKeep) c = desc_units(tab[i], arena_words, word_bits, vmax, rows, &unused);
                if (uw < s_i + c) break;
                s_i += c;
                ++i;
            }
            // image i's record was written above by this same thread; copied
            // word by word (a whole record in registers spills here)
            wv[w].first = uw;
            wv[w].next = s_i + c;
            wv[w].image = i;
            wv[w].reserved = 0;
            const int64_t* src = reinterpret_cast<const int64_t*>(rec + i);
            int64_t* dst = reinterpret_cast<int64_t*>(&wv[w].rec);
            for (int k = 0; k < kPlanRecWords; ++k) dst[k] = src[k];
        }
    }
    if (tid == 0) {
        PlanImage end = idle;
        end.first = total;
        rec[n] = end;
        wv[nw] = PlanWave{total, total, n, 0, end};
        ws[0] = total;
        ws[1] = bad_count;     // every atomicAdd precedes the scan's barrier
        ws[2] = kPlanMagic ^ n;
        ws[3] = nw;
    }
}

// Accepts a plan record only if every word it makes the kernel touch lies
// inside the arena and its unit shape fits the kernel's paths, whatever
// the record holds (a plan written for another table gives wrong output,
// never an access outside the arena).
__device__ __forceinline__ bool record_ok(const PlanImage& r, int64_t arena32, int vmax) {
    const uint32_t vw = r.kind & 7u;
    if (vw == kKindIdle || r.height < 1 || r.height > kMaxHeight || r.width < 1 || r.wd32 < 1 ||
        r.band < 1 || r.split < 1 || r.off32 < 0 || r.stride32 < r.wd32 ||
        r.stride32 > (1ll << 32))
        return false;
    // (height - 1) * stride32 + wd32 < 2^30 * 2^32 + 2^31: no overflow
    if ((int64_t)(r.height - 1) * r.stride32 + r.wd32 > arena32 - r.off32) return false;
    if (vw == 0) return r.wd32 <= kNarrowMaxWords && r.split * r.wd32 <= kWave;
    return r.wd32 > kNarrowMaxWords && (vw == 1 || vw == 2 || vw == 4) && (int)vw <= vmax &&
           ((r.off32 | r.stride32 | r.wd32) & (vw - 1)) == 0;
}

// Persistent batch kernel body: wavefront gw of nw processes the contiguous unit
// range [first of entry gw, first of entry gw + 1) across the images of the
// plan, starting with the image and record its entry holds. The header and
// the two entries are loaded together; records of later images are loaded
// when the range reaches them. A unit is a strip or a group of narrow rows
// of one image, located by one division (none for images one chunk wide).
// VMAX: the widest strip vector width compiled in. VMAX = 1 leaves out the
// wide strip paths, whose registers would otherwise limit how many
// wavefronts of small crops a compute unit keeps in flight.
template <int MODE, int VMAX>
__device__ __forceinline__ void batch_body(const uint32_t* in, uint32_t* out, int n,
                                           int64_t arena32, const int64_t* ws, int vmax,
                                           uint32_t bw, int invert, int wpb, uint32_t nblocks) {
    const uint32_t lb = xcd_block(blockIdx.x, nblocks);
    const int64_t nw = (int64_t)nblocks * wpb;
    const int64_t gw = (int64_t)lb * wpb + wave_uniform(threadIdx.x / kWave);
    // Every load of the header and of this wavefront's map entries first
    // (all inside the workspace: n >= 0 and nw <= kMaxBatchWaves are checked
    // on the host), then one combined test, so that the loads are in flight
    // together rather than one after another behind early exits.
    const PlanWave* wv = reinterpret_cast<const PlanWave*>(ws + ws_wave_offset(n));
    const int64_t total = ws[0], magic = ws[2], plan_nw = ws[3];
    const int64_t u0 = wv[gw].first, u1 = wv[gw + 1].first;
    int64_t next = wv[gw].next;
    int i = wv[gw].image;
    PlanImage r = wv[gw].rec;
    // the entry's fields count as used here (no instruction results), so
    // that their loads are issued with the header's; left alone, the
    // compiler sinks them below the exit test, one more round trip
    asm volatile("" ::"s"(next), "s"(r.first), "s"(r.off32), "s"(r.stride32), "s"(r.height),
                 "s"(r.width), "s"(r.wd32), "s"(r.band), "s"(r.split), "s"(r.kind), "s"(in),
                 "s"(out));
    const bool bad = (n <= 0) | (magic != (kPlanMagic ^ n)) | (plan_nw != nw) | (u0 < 0) |
                     (u0 >= u1) | (u1 > total) | (i < 0) | (i >= n);
    if (bad) return;
    const PlanImage* rec = reinterpret_cast<const PlanImage*>(ws + kWsHeader);
    int cur = -1;
    bool ok = false;
    Geom g;
    g.plane = 0;
    g.grey = nullptr;
    g.grey_stride = 0;
    g.thr = 0;
    int band = 1, split = 1, vw = 1;
    uint32_t qmagic = 0;
    for (int64_t u = u0; u < u1; ++u) {
        while (next <= u) {
            if (++i >= n) return;
            r = rec[i];
            next = rec[i + 1].first;
        }
        if (i != cur) {
            cur = i;
            ok = record_ok(r, arena32, vmax);
            if (ok) {
                // wave-uniform by construction; stated, so that the
                // geometry stays in scalar registers through the unit loops
                const int64_t off = wave_uniform64(r.off32);
                g.in = in + off;
                g.out = out + off;
                g.stride = wave_uniform64(r.stride32);
                g.height = wave_uniform(r.height);
                g.width = wave_uniform(r.width);
                g.wd = wave_uniform(r.wd32);
                band = wave_uniform(r.band);
                split = wave_uniform(r.split);
                vw = (int)(r.kind & 7u);
                qmagic = r.kind >> 8;
            }
        }
        if (!ok) continue;
        const int64_t local = u - r.first;
        if (local < 0 || local >= (1ll << 31)) continue;
        if (vw == 0) {
            const int64_t y0 = local * band;
            if (y0 >= g.height) continue;
            const int64_t y1 = y0 + band < g.height ? y0 + band : g.height;
            // lane layout per unit (a few VALU operations): kept across
            // units it would hold registers through the strip paths too
            narrow_rows<MODE>(g, narrow_lanes_q(g, split, qmagic, bw), (int)y0, (int)y1, bw,
                              invert != 0);
            continue;
        }
        const uint32_t strip = split == 1 ? (uint32_t)local : (uint32_t)local / (uint32_t)split;
        const uint32_t chunk = (uint32_t)local - strip * (uint32_t)split;
        const int64_t y0 = (int64_t)strip * band;
        const int64_t j0 = (int64_t)chunk * kWave * vw;
        if (y0 >= g.height || j0 >= g.wd) continue;
        const int64_t y1 = y0 + band < g.height ? y0 + band : g.height;
        if (VMAX >= 4 && vw == 4) {
            strip_unit<(VMAX >= 4 ? 4 : 1), MODE>(g, (int)j0, (int)y0, (int)y1, bw, invert != 0);
        } else if (VMAX >= 2 && vw == 2) {
            strip_unit<(VMAX >= 2 ? 2 : 1), MODE>(g, (int)j0, (int)y0, (int)y1, bw, invert != 0);
        } else {
            strip_unit<1, MODE>(g, (int)j0, (int)y0, (int)y1, bw, invert != 0);
        }
    }
}

// The batch kernels: one word per lane only (the shape for small crops,
// few enough registers for eight wavefronts per SIMD), and with the wide
// strip paths. The grid's workgroup count and size come in as arguments
// (no argument beyond the explicit ones is read).
template <int MODE>
__global__ void __launch_bounds__(512) k_batch_narrow(const uint32_t* in, uint32_t* out, int n,
                                                         int64_t arena32, const int64_t* ws,
                                                         int vmax, uint32_t bw, int invert, int wpb,
                                                         uint32_t nblocks) {
    batch_body<MODE, 1>(in, out, n, arena32, ws, vmax, bw, invert, wpb, nblocks);
}

template <int MODE>
__global__ void __launch_bounds__(512) k_batch_wide(const uint32_t* in, uint32_t* out, int n,
                                                    int64_t arena32, const int64_t* ws, int vmax,
                                                    uint32_t bw, int invert, int wpb,
                                                    uint32_t nblocks) {
    batch_body<MODE, 4>(in, out, n, arena32, ws, vmax, bw, invert, wpb, nblocks);
}

// The paper's method as separate whole-image passes (sections 3-5), each a
// block operation over 32-bit words, one word per thread. Used as the
// unfused ablation of the fused kernels. Pixels past the width read as the
// border colour (bw) in every pass.
enum { kStageMask = 0, kStageLeft, kStageRight, kStageUp, kStageDown, kStageOr, kStageOrLast };

__device__ __forceinline__ uint32_t stage_pixel_word(const uint32_t* in, int64_t stride,
                                                     int32_t height, int32_t width, int32_t wd,
                                                     int64_t y, int j, uint32_t bw) {
    if (y < 0 || y >= height || j < 0 || j >= wd) return bw;
    const uint32_t vm = valid_bits(j, width);
    return (in[y * stride + j] & vm) | (bw & ~vm);
}

template <int STAGE>
__global__ void __launch_bounds__(256) k_stage(const uint32_t* img, const uint32_t* src,
                                               uint32_t* dst, int64_t stride, int32_t height,
                                               int32_t width, int32_t wd, uint32_t bw) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;    // launched with 256 threads
    if (t >= (int64_t)height * wd) return;
    const int64_t y = t / wd;
    const int j = (int)(t - y * wd);
    const int64_t o = y * stride + j;
    if constexpr (STAGE == kStageMask) {                 // section 3: the negative image
        dst[o] = ~stage_pixel_word(img, stride, height, width, wd, y, j, bw);
    } else if constexpr (STAGE <= kStageDown) {          // section 4: shifted image AND mask
        const uint32_t c = stage_pixel_word(img, stride, height, width, wd, y, j, bw);
        uint32_t shifted;
        if constexpr (STAGE == kStageLeft)               // image shifted right: sees x - 1
            shifted = west_of(c, stage_pixel_word(img, stride, height, width, wd, y, j - 1, bw));
        else if constexpr (STAGE == kStageRight)         // image shifted left: sees x + 1
            shifted = east_of(c, stage_pixel_word(img, stride, height, width, wd, y, j + 1, bw));
        else if constexpr (STAGE == kStageUp)            // image shifted down: sees y - 1
            shifted = stage_pixel_word(img, stride, height, width, wd, y - 1, j, bw);
        else                                             // image shifted up: sees y + 1
            shifted = stage_pixel_word(img, stride, height, width, wd, y + 1, j, bw);
        dst[o] = src[o] & shifted;
    } else {                                             // section 5: OR of the edges
        uint32_t v = dst[o] | src[o];
        if constexpr (STAGE == kStageOrLast) v &= valid_bits(j, width);
        dst[o] = v;
    }
}

// Plain 128-bit copy: the bandwidth reference.
__global__ void __launch_bounds__(256) k_copy(const u32x4* in, u32x4* out, int64_t n16) {
    constexpr int kPer = 4, kThreads = 256;                          // launched with 256 threads
    const int64_t base = (int64_t)blockIdx.x * kThreads * kPer + threadIdx.x;
    u32x4 v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = base + (int64_t)k * kThreads;
        if (i < n16) v[k] = __builtin_nontemporal_load(in + i);
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = base + (int64_t)k * kThreads;
        if (i < n16) __builtin_nontemporal_store(v[k], out + i);
    }
}

// ============================================================== host side ===

namespace {

using namespace edgeh;

// Built-in single-image shape, from the tuned shapes of square images of
// 2048^2 .. 65536^2 on gfx950. Rows of <= 32 words: narrow units of up to 16
// steps. Wider rows: four words per lane when the row fills at least 75% of
// its 256-word spans, else two (a half-used 4-word span loses to twice the
// wavefronts: 3.1 against 4.4 us at 4096^2, 5.2 against 7.1 us at 6000^2).
// Images of under 3 MiB of traffic are bound by launch latency and take
// 2-row strips (the most wavefronts); larger ones take tiles in dispatch
// order, 4 wavefronts per workgroup, of 4 rows up to 12 MiB and 8 rows up
// to 64 MiB, then 16-row tiles of 8 wavefronts regrouped by XCD up to 96 MiB
// (uint64 squares, full definition, against the strips these replace:
// 4096^2 2.99 / 3.15 us, 8192^2 4.58 / 5.43, 16384^2 13.3 / 14.2; at
// 16384^2 the 16-row tiles take 13.5 us in dispatch order with 4
// wavefronts); from 96 MiB, bands of 8 wavefronts x 2 rows
// regrouped by XCD (against 16-row tiles: 23168^2 27.3 / 30.9 us, 32768^2
// 49.5 / 49.9, 65536^2 166.7 / 188.5; 65536 x 16384 51.1 / 48.3). With 4
// wavefronts per band the 65536^2 time varied from 172 to 208 us between
// allocations and runs; with 8 it stays within 1%.
edge_launch_cfg default_single(int64_t height, int64_t wd32) {
    edge_launch_cfg c{};
    c.blocks_per_cu = 1;
    c.cache_policy = EDGE_CACHE_AUTO;
    if (wd32 <= kNarrowMaxWords) {
        const int64_t grp = kWave / wd32;
        c.vec_words = 1;
        c.waves_per_block = 4;
        c.rows_per_tile = (int32_t)pow2_floor(std::max<int64_t>(1, std::min<int64_t>(16, height / (grp * 2048))));
    } else {
        const int64_t span4 = (int64_t)kWave * 4;
        c.vec_words = 4 * wd32 >= 3 * span4 * ceil_div(wd32, span4) ? 4 : 2;
        const int64_t traffic = 2 * height * wd32 * 4;
        c.waves_per_block = 4;
        if (traffic < (3ll << 20)) {
            c.rows_per_tile = 2;
        } else if (traffic < (64ll << 20)) {
            c.shape = EDGE_SHAPE_TILE;
            c.rows_per_tile = traffic < (12ll << 20) ? 4 : 8;
        } else if (traffic < (96ll << 20)) {
            c.shape = EDGE_SHAPE_TILE_XCD;
            c.rows_per_tile = 16;
            c.waves_per_block = 8;
        } else {
            c.shape = EDGE_SHAPE_BAND_XCD;
            c.rows_per_tile = 2;
            c.waves_per_block = 8;
            // a band grid past the dispatch limit (images of tens of GB):
            // long strips, whose grid is 128 times smaller
            const int64_t span = (int64_t)kWave * strip_vw(wd32, c.vec_words, 0, 0);
            const int64_t bands = ceil_div(wd32, span) * ceil_div(height, (int64_t)(8 * 2 - 2));
            if (!grid_fits(bands, 8 * kWave)) {
                c.shape = EDGE_SHAPE_STRIP;
                c.rows_per_tile = 256;
            }
        }
    }
    return c;
}

// Strips only (four fundamental-edge planes, single peels): about 1024
// strips of at most 256 rows above 16 MiB of traffic, else 2-row strips.
edge_launch_cfg default_strips(int64_t height, int64_t wd32) {
    edge_launch_cfg c = default_single(height, wd32);
    if (wd32 <= kNarrowMaxWords) return c;
    const int v = strip_vw(wd32, c.vec_words, 0, 0);
    const int64_t chunks = ceil_div(wd32, (int64_t)kWave * v);
    const bool small = 2 * height * wd32 * 4 <= (16ll << 20);
    c.shape = EDGE_SHAPE_STRIP;
    c.rows_per_tile = small ? 2 : (int32_t)pow2_floor(std::max<int64_t>(2, std::min<int64_t>(256, chunks * height / 1024)));
    c.waves_per_block = c.rows_per_tile >= 256 ? 8 : 4;
    return c;
}

// Streaming (non-temporal) loads and stores pay off from a few MiB of
// traffic up (measured: 3.12 against 3.30 us at 4096^2, 4 MiB; equal at
// 3000^2); smaller images stay cached.
constexpr int64_t kStreamBytes = 4ll << 20;
// Threshold + pack: packed output bytes from which its stores stream.
constexpr int64_t kPackStreamBytes = 16ll << 20;

edge_launch_cfg default_batch() {
    edge_launch_cfg c{};
    c.vec_words = 4;
    c.rows_per_tile = 8;
    c.waves_per_block = 4;
    c.blocks_per_cu = 8;
    c.cache_policy = EDGE_CACHE_NORMAL;
    return c;
}

template <int MODE, class Pol>
int launch_strip(const Geom& g, int vw, int64_t chunks, const edge_launch_cfg& c, int64_t nunits,
                 int64_t blocks, uint32_t bw, int invert, hipStream_t stream) {
    const int by_xcd = Pol::oneshot ? c.shape == EDGE_SHAPE_TILE_XCD : 1;
    const int threads = c.waves_per_block * kWave;
    switch (vw) {
        case 4:
            hipLaunchKernelGGL((k_strip<4, MODE, Pol>), dim3((uint32_t)blocks), dim3(threads), 0,
                               stream, g, chunks, c.rows_per_tile, nunits, bw, invert,
                               c.waves_per_block, by_xcd);
            break;
        case 2:
            hipLaunchKernelGGL((k_strip<2, MODE, Pol>), dim3((uint32_t)blocks), dim3(threads), 0,
                               stream, g, chunks, c.rows_per_tile, nunits, bw, invert,
                               c.waves_per_block, by_xcd);
            break;
        default:
            hipLaunchKernelGGL((k_strip<1, MODE, Pol>), dim3((uint32_t)blocks), dim3(threads), 0,
                               stream, g, chunks, c.rows_per_tile, nunits, bw, invert,
                               c.waves_per_block, by_xcd);
            break;
    }
    return launch_status();
}

template <int MODE, int RW>
int launch_band(const Geom& g, int vw, const edge_launch_cfg& c, uint32_t bw, int invert,
                hipStream_t stream) {
    const int nw = c.waves_per_block;
    const int64_t chunks = ceil_div(g.wd, (int64_t)kWave * vw);
    const int64_t nunits = chunks * ceil_div(g.height, (int64_t)(nw * RW - 2));
    if (!grid_fits(nunits, nw * kWave)) return EDGE_ERR_UNSUPPORTED;
    const size_t lds = (size_t)nw * RW * band_pitch(vw) * sizeof(uint32_t);
    const int by_xcd = c.shape == EDGE_SHAPE_BAND_XCD;
    const dim3 grid((uint32_t)nunits), block(nw * kWave);
    switch (vw) {
        case 4:
            hipLaunchKernelGGL((k_band<4, RW, MODE>), grid, block, lds, stream, g, chunks, nunits,
                               bw, invert, nw, by_xcd);
            break;
        case 2:
            hipLaunchKernelGGL((k_band<2, RW, MODE>), grid, block, lds, stream, g, chunks, nunits,
                               bw, invert, nw, by_xcd);
            break;
        default:
            hipLaunchKernelGGL((k_band<1, RW, MODE>), grid, block, lds, stream, g, chunks, nunits,
                               bw, invert, nw, by_xcd);
            break;
    }
    return launch_status();
}

template <int MODE>
int launch_single(const Geom& g, int vw, const edge_launch_cfg& c, uint32_t bw, int invert,
                  hipStream_t stream) {
    const int threads = c.waves_per_block * kWave;
    if (g.wd <= kNarrowMaxWords) {
        const int64_t band = (int64_t)(kWave / g.wd) * c.rows_per_tile;
        const int64_t nunits = ceil_div(g.height, band);
        const int64_t blocks = ceil_div(nunits, c.waves_per_block);
        if (!grid_fits(blocks, c.waves_per_block * kWave)) return EDGE_ERR_UNSUPPORTED;
        hipLaunchKernelGGL(k_narrow<MODE>, dim3((uint32_t)blocks), dim3(threads), 0, stream, g,
                           band, nunits, bw, invert, c.waves_per_block);
        return launch_status();
    }
    const int64_t chunks = ceil_div(g.wd, (int64_t)kWave * vw);
    const int64_t nunits = chunks * ceil_div(g.height, c.rows_per_tile);
    const int64_t blocks = ceil_div(nunits, c.waves_per_block);
    if (!grid_fits(blocks, c.waves_per_block * kWave)) return EDGE_ERR_UNSUPPORTED;
    // bands and tiles for the edge map, its diagnostic and the direction
    // planes; the single-level peels (copy, one peel) always walk strips
    if constexpr (MODE == kModePlain || MODE == kModeFull || MODE == kModeClause2 ||
                  MODE == kModeDirections) {
        const bool band = c.shape == EDGE_SHAPE_BAND || c.shape == EDGE_SHAPE_BAND_XCD;
        if (band && c.rows_per_tile == 1) return launch_band<MODE, 1>(g, vw, c, bw, invert, stream);
        if (band && c.rows_per_tile == 2) return launch_band<MODE, 2>(g, vw, c, bw, invert, stream);
        if (band) return launch_band<MODE, 4>(g, vw, c, bw, invert, stream);
    }
    if constexpr (MODE != kModeCopy && MODE != kModePeel) {
        const bool tile = c.shape == EDGE_SHAPE_TILE || c.shape == EDGE_SHAPE_TILE_XCD;
        if (tile && c.rows_per_tile <= 8)
            return launch_strip<MODE, TileStrip<8>>(g, vw, chunks, c, nunits, blocks, bw, invert,
                                                    stream);
        if (tile)
            return launch_strip<MODE, TileStrip<kTileMaxRows>>(g, vw, chunks, c, nunits, blocks,
                                                               bw, invert, stream);
    }
    bool stream_mode = c.cache_policy == EDGE_CACHE_STREAM;
    if (c.cache_policy == EDGE_CACHE_AUTO)
        stream_mode = 2 * (int64_t)g.height * g.wd * 4 >= kStreamBytes;
    if (stream_mode)
        return launch_strip<MODE, StreamingStrip>(g, vw, chunks, c, nunits, blocks, bw, invert,
                                                  stream);
    return launch_strip<MODE, CachedStrip>(g, vw, chunks, c, nunits, blocks, bw, invert, stream);
}

// Single-image launch. planes = 1 for the edge map; 4 for the fundamental
// edges (kModeDirections), written plane_words B-bit words apart.
int image_launch(const void* in, void* out, int64_t height, int64_t width, int64_t stride_words,
                 int word_bits, int border, int mode, uint32_t flags, const edge_launch_cfg* cfg,
                 void* hip_stream, int planes = 1, int64_t plane_words = 0) {
    int rc = common_checks(word_bits, border, mode, flags);
    if (rc) return rc;
    if (height < 0 || width < 0 || stride_words < 0 || plane_words < 0) return EDGE_ERR_INVALID;
    if (height > kMaxHeight || width > 0x7fffffff) return EDGE_ERR_INVALID;
    if (cfg && !cfg_ok(*cfg)) return EDGE_ERR_INVALID;
    if (height == 0 || width == 0) return EDGE_OK;
    if (!in || !out) return EDGE_ERR_INVALID;
    const int64_t wd = ceil_div(width, word_bits);
    if (stride_words < wd) return EDGE_ERR_INVALID;
    const int word_bytes = word_bits / 8;
    const uintptr_t pin = (uintptr_t)in, pout = (uintptr_t)out;
    if (pin % word_bytes || pout % word_bytes) return EDGE_ERR_ALIGN;
    if (stride_words > (int64_t)(INT64_MAX / 8) / height) return EDGE_ERR_INVALID;
    const int64_t span_words = (height - 1) * stride_words + wd;
    if (planes > 1 && plane_words < span_words) return EDGE_ERR_INVALID;
    if (planes > 1 && plane_words > (int64_t)(INT64_MAX / 64)) return EDGE_ERR_INVALID;
    const uint64_t span = (uint64_t)span_words * word_bytes;
    const uint64_t out_span = (uint64_t)((planes - 1) * plane_words + span_words) * word_bytes;
    if (ranges_overlap(pin, span, pout, out_span)) return EDGE_ERR_ALIAS;

    const int per = word_bits / 32;
    Geom g;
    g.in = (const uint32_t*)in;
    g.out = (uint32_t*)out;
    g.stride = stride_words * per;
    g.height = (int32_t)height;
    g.width = (int32_t)width;
    g.wd = (int32_t)(wd * per);
    g.plane = plane_words * per;
    g.grey = nullptr;
    g.grey_stride = 0;
    g.thr = 0;
    edge_launch_cfg c = cfg ? *cfg : planes == 4 ? default_strips(height, g.wd)
                                                : default_single(height, g.wd);
    // four planes out per row in: 2-row strips keep more stores in flight
    // (measured at 8192^2: 9.9 us against 11.0 us with the plain shape)
    if (!cfg && planes == 4 && g.wd > kNarrowMaxWords) c.rows_per_tile = 2;
    // and once the traffic outgrows the 256 MB last-level cache, cached
    // stores beat non-temporal ones (measured: 32768^2 129 against 136 us,
    // 65536^2 492 against 553 us; up to 16384^2 streaming is as fast or
    // faster)
    if (!cfg && planes == 4 && (uint64_t)(planes + 1) * span > (256ull << 20))
        c.cache_policy = EDGE_CACHE_NORMAL;
    int vmax = c.vec_words;
    vmax = std::min(vmax, alignment_words(pin));
    vmax = std::min(vmax, alignment_words(pout));
    if (planes > 1) vmax = std::min(vmax, alignment_words((uintptr_t)(plane_words * word_bytes)));
    const int vw = strip_vw(g.wd, vmax, 0, g.stride);
    // four planes from rows of four words per lane: 8-row tiles for 12 MiB
    // - 1 GiB of image traffic (against the 2-row strips: 8192^2 8.1 /
    // 10.2 us, 16384^2 34.7 / 38.2, 23168^2 83.9 / 88.8, 32768^2 125 /
    // 151), bands of 8 wavefronts x 2 rows from there (65536^2: 481 against
    // 499-520 us); at 4096^2 and with two words per lane (11584^2) the
    // strips are as fast or faster
    const int64_t image_traffic = (int64_t)2 * span_words * word_bytes;
    if (!cfg && planes == 4 && g.wd > kNarrowMaxWords && vw == 4 &&
        image_traffic >= (12ll << 20)) {
        if (image_traffic < (1ll << 30)) {
            c.shape = EDGE_SHAPE_TILE;
            c.rows_per_tile = 8;
            c.waves_per_block = 4;
        } else {
            c.shape = EDGE_SHAPE_BAND;
            c.rows_per_tile = 2;
            c.waves_per_block = 8;
            const int64_t bands = ceil_div(g.wd, (int64_t)kWave * 4) * ceil_div(height, (int64_t)14);
            if (!grid_fits(bands, 8 * kWave)) {         // as in default_single
                c.shape = EDGE_SHAPE_STRIP;
                c.rows_per_tile = 2;
                c.waves_per_block = 4;
            }
        }
    }
    const uint32_t bw = border_word(border);
    const int inv = (flags & EDGE_FLAG_INVERT_OUT) ? 1 : 0;
    hipStream_t s = (hipStream_t)hip_stream;
    if (planes == 4) return launch_single<kModeDirections>(g, vw, c, bw, 0, s);
    switch (kernel_mode(mode, flags)) {
        case kModePlain: return launch_single<kModePlain>(g, vw, c, bw, inv, s);
        case kModeFull: return launch_single<kModeFull>(g, vw, c, bw, inv, s);
        default: return launch_single<kModeClause2>(g, vw, c, bw, inv, s);
    }
}

struct BatchArgs {
    const void* in;
    void* out;
    int64_t arena_words;
    const edge_image_desc* table;
    int32_t n;
    int word_bits, border, mode;
    uint32_t flags;
    edge_launch_cfg cfg;
    void* ws;
};

int batch_validate(const void* in_arena, void* out_arena, int64_t arena_words,
                   const edge_image_desc* table_dev, int32_t n_images, int word_bits, int border,
                   int mode, uint32_t flags, const edge_launch_cfg* cfg, void* workspace_dev,
                   int64_t workspace_bytes, BatchArgs* a) {
    int rc = common_checks(word_bits, border, mode, flags, true);
    if (rc) return rc;
    if (n_images < 0 || arena_words < 0) return EDGE_ERR_INVALID;
    if (cfg && !cfg_ok(*cfg)) return EDGE_ERR_INVALID;
    if (!in_arena || !out_arena || !table_dev) return EDGE_ERR_INVALID;
    const int word_bytes = word_bits / 8;
    if ((uintptr_t)in_arena % word_bytes || (uintptr_t)out_arena % word_bytes ||
        (uintptr_t)table_dev % 8)
        return EDGE_ERR_ALIGN;
    if (arena_words > INT64_MAX / 8) return EDGE_ERR_INVALID;
    const uint64_t bytes = (uint64_t)arena_words * word_bytes;
    if (ranges_overlap((uintptr_t)in_arena, bytes, (uintptr_t)out_arena, bytes))
        return EDGE_ERR_ALIAS;
    if (!workspace_dev || workspace_bytes < ws_bytes(n_images) || (uintptr_t)workspace_dev % 256)
        return EDGE_ERR_WORKSPACE;
    a->in = in_arena;
    a->out = out_arena;
    a->arena_words = arena_words;
    a->table = table_dev;
    a->n = n_images;
    a->word_bits = word_bits;
    a->border = border;
    a->mode = mode;
    a->flags = flags;
    a->cfg = cfg ? *cfg : default_batch();
    a->ws = workspace_dev;
    return EDGE_OK;
}

template <int MODE>
int launch_batch_kernel(const BatchArgs& a, int vmax, int blocks, hipStream_t s) {
    const uint32_t bw = border_word(a.border);
    const int inv = (a.flags & EDGE_FLAG_INVERT_OUT) ? 1 : 0;
    const int64_t arena32 = a.arena_words * (a.word_bits / 32);
    if (vmax == 1)
        hipLaunchKernelGGL((k_batch_narrow<MODE>), dim3(blocks), dim3(a.cfg.waves_per_block * kWave), 0,
                           s, (const uint32_t*)a.in, (uint32_t*)a.out, a.n, arena32,
                           (const int64_t*)a.ws, vmax, bw, inv, a.cfg.waves_per_block,
                           (uint32_t)blocks);
    else
        hipLaunchKernelGGL((k_batch_wide<MODE>), dim3(blocks), dim3(a.cfg.waves_per_block * kWave), 0,
                           s, (const uint32_t*)a.in, (uint32_t*)a.out, a.n, arena32,
                           (const int64_t*)a.ws, vmax, bw, inv, a.cfg.waves_per_block,
                           (uint32_t)blocks);
    return launch_status();
}

// Vector width limit and persistent grid of a batch (same on host and device plans).
int batch_shape(const void* in, const void* out, const edge_launch_cfg& cfg, int* vmax,
                int* blocks) {
    int cus = 0;
    const int rc = cu_count(&cus);
    if (rc) return rc;
    int v = cfg.vec_words;
    v = std::min(v, alignment_words((uintptr_t)in));
    v = std::min(v, alignment_words((uintptr_t)out));
    *vmax = v;
    *blocks = std::min(cfg.blocks_per_cu * cus, kMaxBatchWaves / cfg.waves_per_block);
    return EDGE_OK;
}

int batch_enqueue(const BatchArgs& a, hipStream_t s) {
    int vmax = 1, blocks = 1;
    int rc = batch_shape(a.in, a.out, a.cfg, &vmax, &blocks);
    if (rc) return rc;
    if (!(a.flags & EDGE_FLAG_PLANNED)) {
        hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, s, a.table, a.n,
                           a.arena_words, a.word_bits, vmax, a.cfg.rows_per_tile,
                           blocks * a.cfg.waves_per_block, (int64_t*)a.ws);
        rc = launch_status();
        if (rc) return rc;
    }
    switch (kernel_mode(a.mode, a.flags)) {
        case kModePlain: return launch_batch_kernel<kModePlain>(a, vmax, blocks, s);
        case kModeFull: return launch_batch_kernel<kModeFull>(a, vmax, blocks, s);
        default: return launch_batch_kernel<kModeClause2>(a, vmax, blocks, s);
    }
}

struct EdgeGraph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

// ------------------------------------------------- library-held workspace ---

// The workspace of edge_batch_noalloc: a fixed device array, one instance
// per GPU the code object is loaded on, sized for the largest batch that
// entry point accepts. Host code never passes the array's name to a kernel
// or a copy (on the host it is only a stand-in for the device symbol); it
// uses the device address looked up per device by noalloc_workspace().
}  // namespace

constexpr int64_t kNoAllocBytes = ws_bytes(EDGE_BATCH_NOALLOC_MAX_IMAGES);
static_assert(kNoAllocBytes % 8 == 0 && kNoAllocBytes <= (8 << 20),
              "a modest fixed workspace: at most 8 MiB per GPU");
static __device__ __align__(256) int64_t g_noalloc_ws[kNoAllocBytes / 8];

namespace {

std::atomic<void*> g_noalloc_addr[kMaxDevices];
std::mutex g_noalloc_mu;

// Device address of the current device's array (hipGetSymbolAddress once
// per device, with that device current; later calls read the cache).
int noalloc_workspace(void** addr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_failed(e);
    if (dev < 0 || dev >= kMaxDevices) return EDGE_ERR_UNSUPPORTED;
    void* p = g_noalloc_addr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        p = g_noalloc_addr[dev].load(std::memory_order_relaxed);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_noalloc_ws));
            if (e != hipSuccess) return hip_failed(e);
            if (!p || (uintptr_t)p % 256) return EDGE_ERR_WORKSPACE;
            g_noalloc_addr[dev].store(p, std::memory_order_release);
        }
    }
    *addr = p;
    return EDGE_OK;
}

// Built-in peel shape, from sweeps at 8192^2 and 16384^2: a unit walks
// 2 * levels halo rows besides its strip (the first half of them with few
// levels formed), so strips are the smallest power of two above the level
// count (at least 8, at most 64 rows), doubled once when the image would
// still give more than 8192 strips (4096 when each strip takes two
// wavefronts); 4 wavefronts per workgroup. cache_policy is not used: peel
// units load through the caches, which keep the halo rows that
// neighbouring strips share.
// Two or three levels: four words per lane at any size. Four to seven
// levels on images of 2^30 pixels and more: four words per lane in 32-row
// strips (measured, against the one-word unit in its built-in strips:
// 32768^2 4 / 7 peels about 49 / 66 against 53 / 73 us, 65536^2 216 / 277
// against 238-264 / 295-298 us; at 16384^2 level, at 8192^2 slower), when
// the image's alignment allows it (vec_ok), else the one-word shape.
edge_launch_cfg default_peel(int64_t height, int64_t wd32, int levels, bool vec_ok = true) {
    edge_launch_cfg c{};
    const bool large = vec_ok && levels >= 4 && levels <= kPeelVecLevels &&
                       height * wd32 * 32 >= (int64_t(1) << 30);
    c.vec_words = (vec_ok && levels <= 3) || large ? 4 : 1;
    c.blocks_per_cu = 1;
    c.cache_policy = EDGE_CACHE_NORMAL;
    c.waves_per_block = 4;
    const int64_t chunks = ceil_div(wd32, (int64_t)kPeelSpan);
    int64_t rows = 8;
    while (rows <= levels && rows < 64) rows *= 2;
    const int64_t many = levels >= kPeelSplitLevels ? 4096 : 8192;
    if (rows < 64 && chunks * ceil_div(height, rows) > many) rows *= 2;
    if (large) rows = 32;
    // keep the grid (one or two wavefronts per strip) within 2^32 work-items
    const int64_t max_units = levels >= kPeelSplitLevels ? (1ll << 25) : (1ll << 26);
    while (chunks * ceil_div(height, rows) >= max_units && rows < 1024) rows *= 2;
    c.rows_per_tile = (int32_t)rows;
    return c;
}

}  // namespace

int edgeh::peel_launch(const Geom& g, const edge_launch_cfg& c, uint32_t bw, int levels, int vw,
                       bool edge_out, hipStream_t s) {
    if (levels >= 2 && levels <= 7) return peel_launch_2_7(g, c, bw, levels, vw, edge_out, s);
    if (levels >= 8 && levels <= 15) return peel_launch_8_15(g, c, bw, levels, vw, edge_out, s);
    if (levels >= 16 && levels <= 23) return peel_launch_16_23(g, c, bw, levels, vw, edge_out, s);
    if (levels >= 24 && levels <= 31) return peel_launch_24_31(g, c, bw, levels, vw, edge_out, s);
    return EDGE_ERR_INVALID;
}

namespace {

template <int STAGE>
int launch_stage(const uint32_t* img, const uint32_t* src, uint32_t* dst, int64_t stride,
                 int32_t height, int32_t width, int32_t wd, uint32_t bw, hipStream_t s) {
    const int64_t blocks = ceil_div((int64_t)height * wd, 256);
    if (!grid_fits(blocks, 256)) return EDGE_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_stage<STAGE>, dim3((uint32_t)blocks), dim3(256), 0, s, img, src, dst,
                       stride, height, width, wd, bw);
    return launch_status();
}

}  // namespace

// ================================================================== C ABI ===

extern "C" {

int edge_abi_version(void) { return EDGE_MASKS_ABI_VERSION; }

int edge_last_hip_error(void) { return g_last_hip; }

const char* edge_status_string(int status) {
    switch (status) {
        case EDGE_OK: return "ok";
        case EDGE_ERR_INVALID: return "invalid argument";
        case EDGE_ERR_ALIGN: return "pointer not aligned to the word size";
        case EDGE_ERR_ALIAS: return "input and output overlap";
        case EDGE_ERR_HIP: return "HIP runtime error";
        case EDGE_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
        case EDGE_ERR_UNSUPPORTED: return "launch configuration not supported";
        default: return "unknown status";
    }
}

int edge_masks(const void* in, void* out, int64_t height, int64_t width, int64_t stride_words,
               int word_bits, int border, void* hip_stream) {
    return image_launch(in, out, height, width, stride_words, word_bits, border, EDGE_MODE_MASKS,
                        0u, nullptr, hip_stream);
}

int edge_full(const void* in, void* out, int64_t height, int64_t width, int64_t stride_words,
              int word_bits, int border, uint32_t flags, void* hip_stream) {
    return image_launch(in, out, height, width, stride_words, word_bits, border, EDGE_MODE_FULL,
                        flags, nullptr, hip_stream);
}

int edge_image_launch(const void* in, void* out, int64_t height, int64_t width,
                      int64_t stride_words, int word_bits, int border, int mode, uint32_t flags,
                      const edge_launch_cfg* cfg, void* hip_stream) {
    return image_launch(in, out, height, width, stride_words, word_bits, border, mode, flags, cfg,
                        hip_stream);
}

int edge_directions(const void* in, void* out4, int64_t plane_words, int64_t height,
                    int64_t width, int64_t stride_words, int word_bits, int border,
                    const edge_launch_cfg* cfg, void* hip_stream) {
    return image_launch(in, out4, height, width, stride_words, word_bits, border,
                        EDGE_MODE_MASKS, 0u, cfg, hip_stream, 4, plane_words);
}

int edge_threshold_pack(const void* grey, int64_t grey_stride_bytes, int threshold, void* out,
                        int64_t height, int64_t width, int64_t stride_words, int word_bits,
                        void* hip_stream) {
    if (word_bits != 32 && word_bits != 64) return EDGE_ERR_INVALID;
    if (threshold < 0 || threshold > 256) return EDGE_ERR_INVALID;
    if (height < 0 || width < 0 || stride_words < 0 || grey_stride_bytes < 0)
        return EDGE_ERR_INVALID;
    if (height > kMaxHeight || width > 0x7fffffff) return EDGE_ERR_INVALID;
    if (height == 0 || width == 0) return EDGE_OK;
    if (!grey || !out) return EDGE_ERR_INVALID;
    const int64_t wd = ceil_div(width, word_bits);
    if (stride_words < wd || grey_stride_bytes < width) return EDGE_ERR_INVALID;
    const int word_bytes = word_bits / 8;
    if ((uintptr_t)out % word_bytes) return EDGE_ERR_ALIGN;
    if (stride_words > (int64_t)(INT64_MAX / 8) / height ||
        grey_stride_bytes > (int64_t)(INT64_MAX / 2) / height)
        return EDGE_ERR_INVALID;
    const uint64_t gspan = (uint64_t)((height - 1) * grey_stride_bytes + width);
    const uint64_t ospan = (uint64_t)((height - 1) * stride_words + wd) * word_bytes;
    if (ranges_overlap((uintptr_t)grey, gspan, (uintptr_t)out, ospan)) return EDGE_ERR_ALIAS;
    const int per = word_bits / 32;
    const int32_t wd32 = (int32_t)(wd * per);
    const int64_t threads = height * (int64_t)wd32;
    const int64_t blocks = ceil_div(threads, 256);
    if (!grid_fits(blocks, 256)) return EDGE_ERR_UNSUPPORTED;
    const bool aligned = (uintptr_t)grey % 16 == 0 && grey_stride_bytes % 16 == 0;
    // packed output from 16 MiB up stored non-temporally (16384^2 / 32768^2
    // / 65536^2: 52.3 / 204 / 807 us against 53.4 / 213 / 844 us; equal up
    // to 8192^2, where a following edge pass still finds the output cached)
    const bool nt = (int64_t)height * wd32 * 4 >= kPackStreamBytes;
    hipStream_t s = (hipStream_t)hip_stream;
    return pack_launch((const uint8_t*)grey, grey_stride_bytes, (uint32_t*)out, stride_words * per,
                       (int32_t)height, (int32_t)width, wd32, (uint32_t)threshold, aligned, nt,
                       blocks, s);
}

int edge_threshold_edges(const void* grey, int64_t grey_stride_bytes, int threshold, void* out,
                         int64_t height, int64_t width, int64_t stride_words, int word_bits,
                         int border, int mode, uint32_t flags, const edge_launch_cfg* cfg,
                         void* hip_stream) {
    int rc = common_checks(word_bits, border, mode, flags);
    if (rc) return rc;
    if (threshold < 0 || threshold > 256) return EDGE_ERR_INVALID;
    if (height < 0 || width < 0 || stride_words < 0 || grey_stride_bytes < 0)
        return EDGE_ERR_INVALID;
    if (height > kMaxHeight || width > 0x7fffffff) return EDGE_ERR_INVALID;
    if (cfg && !cfg_ok(*cfg)) return EDGE_ERR_INVALID;
    if (height == 0 || width == 0) return EDGE_OK;
    if (!grey || !out) return EDGE_ERR_INVALID;
    const int64_t wd = ceil_div(width, word_bits);
    if (stride_words < wd || grey_stride_bytes < width) return EDGE_ERR_INVALID;
    const int word_bytes = word_bits / 8;
    if ((uintptr_t)out % word_bytes) return EDGE_ERR_ALIGN;
    if (stride_words > (int64_t)(INT64_MAX / 8) / height ||
        grey_stride_bytes > (int64_t)(INT64_MAX / 2) / height)
        return EDGE_ERR_INVALID;
    const uint64_t gspan = (uint64_t)((height - 1) * grey_stride_bytes + width);
    const uint64_t ospan = (uint64_t)((height - 1) * stride_words + wd) * word_bytes;
    if (ranges_overlap((uintptr_t)grey, gspan, (uintptr_t)out, ospan)) return EDGE_ERR_ALIAS;
    const int per = word_bits / 32;
    Geom g;
    g.in = nullptr;
    g.out = (uint32_t*)out;
    g.stride = stride_words * per;
    g.height = (int32_t)height;
    g.width = (int32_t)width;
    g.wd = (int32_t)(wd * per);
    g.plane = 0;
    g.grey = (const uint8_t*)grey;
    g.grey_stride = grey_stride_bytes;
    g.thr = (uint32_t)threshold;
    edge_launch_cfg c{};
    if (cfg) {
        c = *cfg;
    } else {
        // bands of 8 wavefronts x 2 rows (16 rows loaded, 14 out), cached
        // loads and non-temporal stores: within 1-2% of the best band shape
        // at 8192^2, 16384^2 and 65536^2, and faster than threshold-and-pack
        // alone at each
        c.vec_words = 1;
        c.blocks_per_cu = 1;
        c.cache_policy = EDGE_CACHE_AUTO;
        c.rows_per_tile = 2;
        c.waves_per_block = 8;
    }
    const bool aligned = (uintptr_t)grey % 16 == 0 && grey_stride_bytes % 16 == 0;
    const uint32_t bw = border_word(border);
    const int inv = (flags & EDGE_FLAG_INVERT_OUT) ? 1 : 0;
    hipStream_t s = (hipStream_t)hip_stream;
    return grey_edges_launch(g, c, bw, inv, aligned, kernel_mode(mode, flags), s);
}

int edge_peel(const void* in, void* out, int64_t height, int64_t width, int64_t stride_words,
              int word_bits, int border, int iterations, uint32_t flags,
              const edge_launch_cfg* cfg, void* hip_stream) {
    if (word_bits != 32 && word_bits != 64) return EDGE_ERR_INVALID;
    if (border != EDGE_BORDER_WHITE && border != EDGE_BORDER_BLACK) return EDGE_ERR_INVALID;
    if (flags & ~(uint32_t)EDGE_FLAG_PEEL_EDGE) return EDGE_ERR_INVALID;
    if (iterations < 0 || iterations > EDGE_PEEL_MAX_ITERATIONS) return EDGE_ERR_INVALID;
    if (height < 0 || width < 0 || stride_words < 0) return EDGE_ERR_INVALID;
    if (height > kMaxHeight || width > 0x7fffffff) return EDGE_ERR_INVALID;
    if (cfg && !cfg_ok(*cfg)) return EDGE_ERR_INVALID;
    if (height == 0 || width == 0) return EDGE_OK;
    if (!in || !out) return EDGE_ERR_INVALID;
    const int64_t wd = ceil_div(width, word_bits);
    if (stride_words < wd) return EDGE_ERR_INVALID;
    const int word_bytes = word_bits / 8;
    const uintptr_t pin = (uintptr_t)in, pout = (uintptr_t)out;
    if (pin % word_bytes || pout % word_bytes) return EDGE_ERR_ALIGN;
    if (stride_words > (int64_t)(INT64_MAX / 8) / height) return EDGE_ERR_INVALID;
    const uint64_t span = (uint64_t)((height - 1) * stride_words + wd) * word_bytes;
    if (ranges_overlap(pin, span, pout, span)) return EDGE_ERR_ALIAS;
    const int per = word_bits / 32;
    Geom g;
    g.in = (const uint32_t*)in;
    g.out = (uint32_t*)out;
    g.stride = stride_words * per;
    g.height = (int32_t)height;
    g.width = (int32_t)width;
    g.wd = (int32_t)(wd * per);
    g.plane = 0;
    g.grey = nullptr;
    g.grey_stride = 0;
    g.thr = 0;
    const bool edge_out = (flags & EDGE_FLAG_PEEL_EDGE) != 0;
    const int levels = iterations + (edge_out ? 1 : 0);
    const uint32_t bw = border_word(border);
    hipStream_t s = (hipStream_t)hip_stream;
    if (levels <= 1) {
        // One level (one peel, or the edge map of the image) or none: the
        // strip loop of the single-image kernels with that word function.
        edge_launch_cfg c = cfg ? *cfg : default_strips(height, g.wd);
        c.shape = EDGE_SHAPE_STRIP;
        int vmax = std::min(c.vec_words, std::min(alignment_words(pin), alignment_words(pout)));
        const int vw = strip_vw(g.wd, vmax, 0, g.stride);
        if (levels == 0) return launch_single<kModeCopy>(g, vw, c, bw, 0, s);
        if (edge_out) return launch_single<kModePlain>(g, vw, c, bw, 0, s);
        return launch_single<kModePeel>(g, vw, c, bw, 0, s);
    }
    edge_launch_cfg c = cfg ? *cfg : default_peel(height, g.wd, levels);
    const int vmax = std::min(c.vec_words, std::min(alignment_words(pin), alignment_words(pout)));
    const int vw = pick_vw(g.wd, vmax, 0, g.stride);
    // the built-in shape for four words per lane, but the image allows one
    if (!cfg && vw < 2 && levels >= 4) c = default_peel(height, g.wd, levels, false);
    return peel_launch(g, c, bw, levels, vw, edge_out, s);
}

int edge_masks_staged(const void* in, void* out, void* scratch, int64_t scratch_bytes,
                      int64_t height, int64_t width, int64_t stride_words, int word_bits,
                      int border, void* hip_stream) {
    if (word_bits != 32 && word_bits != 64) return EDGE_ERR_INVALID;
    if (border != EDGE_BORDER_WHITE && border != EDGE_BORDER_BLACK) return EDGE_ERR_INVALID;
    if (height < 0 || width < 0 || stride_words < 0 || scratch_bytes < 0) return EDGE_ERR_INVALID;
    if (height > kMaxHeight || width > 0x7fffffff) return EDGE_ERR_INVALID;
    if (height == 0 || width == 0) return EDGE_OK;
    if (!in || !out) return EDGE_ERR_INVALID;
    const int64_t wd = ceil_div(width, word_bits);
    if (stride_words < wd) return EDGE_ERR_INVALID;
    const int word_bytes = word_bits / 8;
    if ((uintptr_t)in % word_bytes || (uintptr_t)out % word_bytes) return EDGE_ERR_ALIGN;
    if (stride_words > (int64_t)(INT64_MAX / 64) / height) return EDGE_ERR_INVALID;
    const int64_t plane = height * stride_words * word_bytes;     // bytes per scratch plane
    const uint64_t span = (uint64_t)((height - 1) * stride_words + wd) * word_bytes;
    if (!scratch || scratch_bytes < 4 * plane || (uintptr_t)scratch % 4)
        return EDGE_ERR_WORKSPACE;
    const uintptr_t pin = (uintptr_t)in, pout = (uintptr_t)out, ps = (uintptr_t)scratch;
    if (ranges_overlap(pin, span, pout, span) || ranges_overlap(pin, span, ps, 4 * plane) ||
        ranges_overlap(pout, span, ps, 4 * plane))
        return EDGE_ERR_ALIAS;
    const int per = word_bits / 32;
    const int64_t stride = stride_words * per;
    const int32_t wd32 = (int32_t)(wd * per), H = (int32_t)height, W = (int32_t)width;
    const uint32_t bw = border_word(border);
    const uint32_t* img = (const uint32_t*)in;
    uint32_t* mask = (uint32_t*)scratch;
    uint32_t* f_right = (uint32_t*)(ps + plane);
    uint32_t* f_up = (uint32_t*)(ps + 2 * plane);
    uint32_t* f_down = (uint32_t*)(ps + 3 * plane);
    uint32_t* f_left = (uint32_t*)out;                  // the left edge accumulates the OR
    hipStream_t s = (hipStream_t)hip_stream;
    int rc;
    if ((rc = launch_stage<kStageMask>(img, nullptr, mask, stride, H, W, wd32, bw, s))) return rc;
    if ((rc = launch_stage<kStageLeft>(img, mask, f_left, stride, H, W, wd32, bw, s))) return rc;
    if ((rc = launch_stage<kStageRight>(img, mask, f_right, stride, H, W, wd32, bw, s))) return rc;
    if ((rc = launch_stage<kStageUp>(img, mask, f_up, stride, H, W, wd32, bw, s))) return rc;
    if ((rc = launch_stage<kStageDown>(img, mask, f_down, stride, H, W, wd32, bw, s))) return rc;
    if ((rc = launch_stage<kStageOr>(img, f_right, f_left, stride, H, W, wd32, bw, s))) return rc;
    if ((rc = launch_stage<kStageOr>(img, f_up, f_left, stride, H, W, wd32, bw, s))) return rc;
    return launch_stage<kStageOrLast>(img, f_down, f_left, stride, H, W, wd32, bw, s);
}

int edge_default_cfg(int64_t height, int64_t width, int word_bits, int mode, int batch,
                     edge_launch_cfg* cfg_out) {
    if (!cfg_out || height < 0 || width < 0) return EDGE_ERR_INVALID;
    if (common_checks(word_bits, EDGE_BORDER_WHITE, mode, 0u)) return EDGE_ERR_INVALID;
    const int64_t wd32 = ceil_div(width, word_bits) * (word_bits / 32);
    *cfg_out = batch ? default_batch() : default_single(height, std::max<int64_t>(wd32, 1));
    return EDGE_OK;
}

int64_t edge_batch_workspace_bytes(int32_t n_images) {
    if (n_images < 0) return EDGE_ERR_INVALID;
    return ws_bytes(n_images);
}

int edge_batch_check(const edge_image_desc* table_host, int32_t n_images, int64_t arena_words,
                     int word_bits) {
    if (n_images < 0 || arena_words < 0) return EDGE_ERR_INVALID;
    if (word_bits != 32 && word_bits != 64) return EDGE_ERR_INVALID;
    if (n_images > 0 && !table_host) return EDGE_ERR_INVALID;
    for (int32_t i = 0; i < n_images; ++i)
        if (!desc_ok(table_host[i], arena_words, word_bits)) return EDGE_ERR_INVALID;
    return EDGE_OK;
}

int edge_batch_plan(const void* in_arena, const void* out_arena, int64_t arena_words,
                    const edge_image_desc* table_host, int32_t n_images, int word_bits,
                    const edge_launch_cfg* cfg, void* plan_host, int64_t plan_bytes,
                    int64_t* plan_used_bytes) {
    if (n_images < 0 || arena_words < 0 || !plan_used_bytes) return EDGE_ERR_INVALID;
    if (word_bits != 32 && word_bits != 64) return EDGE_ERR_INVALID;
    if (cfg && !cfg_ok(*cfg)) return EDGE_ERR_INVALID;
    if (!in_arena || !out_arena || (n_images > 0 && !table_host)) return EDGE_ERR_INVALID;
    if (!plan_host || plan_bytes < edge_batch_workspace_bytes(n_images) ||
        (uintptr_t)plan_host % 8)
        return EDGE_ERR_WORKSPACE;
    int rc = edge_batch_check(table_host, n_images, arena_words, word_bits);
    if (rc) return rc;
    const edge_launch_cfg c = cfg ? *cfg : default_batch();
    int vmax = 1, blocks = 1;
    rc = batch_shape(in_arena, out_arena, c, &vmax, &blocks);
    if (rc) return rc;
    const int64_t nw = (int64_t)blocks * c.waves_per_block;
    int64_t* ws = (int64_t*)plan_host;
    PlanImage* rec = (PlanImage*)(ws + kWsHeader);
    int64_t total = 0;
    for (int32_t i = 0; i < n_images; ++i) {
        PlanImage r;
        int bad = 0;
        const int64_t units = plan_image(table_host[i], arena_words, word_bits, vmax,
                                         c.rows_per_tile, &r, &bad);
        r.first = total;
        rec[i] = r;
        total += units;
    }
    rec[n_images] = PlanImage{total, 0, 0, 0, 0, 0, 1, 1, kKindIdle};
    for (int k = 0; k < kWsHeader; ++k) ws[k] = 0;
    ws[0] = total;
    ws[2] = kPlanMagic ^ n_images;
    ws[3] = nw;
    PlanWave* wv = (PlanWave*)(ws + ws_wave_offset(n_images));
    int32_t i = 0;
    for (int64_t w = 0; w < nw; ++w) {
        const int64_t uw = total * w / nw;
        // the last image starting at or before uw: the one holding it
        while (i + 1 < n_images && rec[i + 1].first <= uw) ++i;
        wv[w] = PlanWave{uw, i < n_images ? rec[i + 1].first : total, i, 0, rec[i]};
    }
    wv[nw] = PlanWave{total, total, n_images, 0, rec[n_images]};
    *plan_used_bytes = ws_plan_bytes(n_images, nw);
    return EDGE_OK;
}

int edge_batch(const void* in_arena, void* out_arena, int64_t arena_words,
               const edge_image_desc* table_dev, int32_t n_images, int word_bits, int border,
               int mode, uint32_t flags, const edge_launch_cfg* cfg, void* workspace_dev,
               int64_t workspace_bytes, void* hip_stream) {
    BatchArgs a;
    int rc = batch_validate(in_arena, out_arena, arena_words, table_dev, n_images, word_bits,
                            border, mode, flags, cfg, workspace_dev, workspace_bytes, &a);
    if (rc) return rc;
    if (n_images == 0) return EDGE_OK;
    return batch_enqueue(a, (hipStream_t)hip_stream);
}

int edge_batch_noalloc(const void* in_arena, void* out_arena, int64_t arena_words,
                       const edge_image_desc* table_dev, int32_t n_images, int word_bits,
                       int border, int mode, uint32_t flags, const edge_launch_cfg* cfg,
                       void* hip_stream) {
    if (n_images > EDGE_BATCH_NOALLOC_MAX_IMAGES) return EDGE_ERR_WORKSPACE;
    if (flags & EDGE_FLAG_PLANNED) return EDGE_ERR_INVALID;
    // every argument check first (with a stand-in workspace of the right
    // size and alignment), then the one HIP query for the array's address
    BatchArgs a;
    int rc = batch_validate(in_arena, out_arena, arena_words, table_dev, n_images, word_bits,
                            border, mode, flags, cfg, (void*)(uintptr_t)256, kNoAllocBytes, &a);
    if (rc) return rc;
    if (n_images == 0) return EDGE_OK;
    rc = noalloc_workspace(&a.ws);
    if (rc) return rc;
    return batch_enqueue(a, (hipStream_t)hip_stream);
}

int edge_batch_graph_create(const void* in_arena, void* out_arena, int64_t arena_words,
                            const edge_image_desc* table_dev, int32_t n_images, int word_bits,
                            int border, int mode, uint32_t flags, const edge_launch_cfg* cfg,
                            void* workspace_dev, int64_t workspace_bytes, void** graph_out) {
    if (!graph_out) return EDGE_ERR_INVALID;
    *graph_out = nullptr;
    BatchArgs a;
    int rc = batch_validate(in_arena, out_arena, arena_words, table_dev, n_images, word_bits,
                            border, mode, flags, cfg, workspace_dev, workspace_bytes, &a);
    if (rc) return rc;
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_failed(e);
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return hip_failed(e);
    }
    rc = batch_enqueue(a, s);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    (void)hipStreamDestroy(s);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_failed(e);
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_failed(e);
    }
    EdgeGraph* h = new (std::nothrow) EdgeGraph{graph, exec};
    if (!h) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return EDGE_ERR_INVALID;
    }
    *graph_out = h;
    return EDGE_OK;
}

int edge_graph_launch(void* graph, void* hip_stream) {
    if (!graph) return EDGE_ERR_INVALID;
    const hipError_t e = hipGraphLaunch(((EdgeGraph*)graph)->exec, (hipStream_t)hip_stream);
    return e == hipSuccess ? EDGE_OK : hip_failed(e);
}

int edge_graph_destroy(void* graph) {
    if (!graph) return EDGE_OK;
    EdgeGraph* h = (EdgeGraph*)graph;
    hipError_t e1 = hipGraphExecDestroy(h->exec);
    hipError_t e2 = hipGraphDestroy(h->graph);
    delete h;
    if (e1 != hipSuccess) return hip_failed(e1);
    if (e2 != hipSuccess) return hip_failed(e2);
    return EDGE_OK;
}

int edge_copy_bytes(const void* in, void* out, int64_t n_bytes, void* hip_stream) {
    if (n_bytes < 0 || n_bytes % 16) return EDGE_ERR_INVALID;
    if (n_bytes == 0) return EDGE_OK;
    if (!in || !out) return EDGE_ERR_INVALID;
    if ((uintptr_t)in % 16 || (uintptr_t)out % 16) return EDGE_ERR_ALIGN;
    if (ranges_overlap((uintptr_t)in, (uint64_t)n_bytes, (uintptr_t)out, (uint64_t)n_bytes))
        return EDGE_ERR_ALIAS;
    const int64_t n16 = n_bytes / 16;
    const int64_t blocks = ceil_div(n16, 256 * 4);
    if (!grid_fits(blocks, 256)) return EDGE_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_copy, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                       (const u32x4*)in, (u32x4*)out, n16);
    return launch_status();
}

}  // extern "C"
