// edge_device.hpp - gfx950 device code of libedgemask: the fused method of
// masks on packed binary rows.
//
// The paper's three stages (mask = negative image, section 3; four
// fundamental edges = image shifted one pixel ANDed with the mask, section 4;
// edge = OR of the four, section 5) are fused into one pass. Per 32-bit word
// c of a row, with u and d the words above and below and w, e the image
// shifted by one pixel to the right and to the left:
//     edge = ~c & (u | d | w | e)
// which is the Boolean function Edge(p) of section 1 for 32 pixels at once
// (distributivity turns the OR of four masked shifts into one mask).
//
// Layout: rows of 32-bit words, LSB first (pixel x is bit x % 32 of word
// x / 32). 64-bit words have the same byte layout, so the host passes every
// image as 32-bit words with the row length rounded up to whole 64-bit words.
// Bits at x >= width take the border colour on input and are 0 on output.
//
// Work decomposition: one wavefront (64 lanes) per work unit.
//   - strip unit: 64 * VW consecutive words of each of `rows` consecutive
//     rows; each lane owns VW words and walks down the rows keeping the rows
//     above and below in registers, so every input word is loaded once per
//     strip (plus one halo row above and below). West/east carries between
//     lanes move with DPP wavefront shifts; the words just outside the
//     wavefront's span are loaded by lanes 0 and 63.
//   - narrow unit (rows of <= 32 words): several whole rows side by side in
//     one wavefront, one word per lane, rows above and below read directly.
//   - peel unit (iterated peeling, below): a strip of one word per lane
//     with the rows of every peel level in registers; from 16 levels the
//     levels of one strip are shared by two wavefronts of a workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace edgek {

constexpr int kWave = 64;
// Row indices are 32-bit in the kernels, and the row loops look a few
// hundred rows ahead of the last row; images are limited to 2^30 rows.
constexpr int32_t kMaxHeight = 1 << 30;
constexpr int kNarrowSteps = 4; // narrow-unit steps loaded ahead of use
constexpr int kNarrowMaxWords = 32;

// kModeDirections writes the four fundamental edges of section 4 (left,
// right, up, down: the edge types of Fig. 2) to four output planes.
// kModePeel writes the image after one peel (its edge points turned white)
// and kModeCopy the image itself: the single-level cases of iterated
// peeling, which run the strip loop of the edge kernels.
enum { kModePlain = 0, kModeFull = 1, kModeClause2 = 2, kModeDirections = 3, kModePeel = 4,
       kModeCopy = 5 };

// Compile-time choices of the strip loop: rows kept in flight per lane,
// non-temporal (streaming) cache policy for the row loads and stores, and
// ONESHOT: the unit's rows are all requested at the start and the ring is
// never refilled, so a unit holds at most PREFETCH rows.
template <int PREFETCH, bool NT_LOAD, bool NT_STORE, bool ONESHOT = false>
struct StripPolicy {
    static constexpr int prefetch = PREFETCH;
    static constexpr bool nt_load = NT_LOAD;
    static constexpr bool nt_store = NT_STORE;
    static constexpr bool oneshot = ONESHOT;
};
// Images that fit in the caches keep normal loads and stores (halo rows and
// the output stay cached for the next consumer); large images stream.
using CachedStrip = StripPolicy<4, false, false>;
using StreamingStrip = StripPolicy<4, true, true>;
// Rows that are re-read from the cache (the halo rows of grey bands) but
// whose output is not: cached loads, non-temporal stores.
using StreamOutStrip = StripPolicy<4, false, true>;
// Tiles: a wavefront requests all rows of its tile and the two halo rows
// at once, computes the rows as they arrive and ends. Short-lived
// wavefronts with their whole input in flight keep the memory system's
// queues fuller than long strips walking a few rows ahead. Tiles keep the
// dispatcher's workgroup order (no regrouping by XCD): the workgroups in
// flight then form one window sweeping down the image.
constexpr int kTileMaxRows = 16;
template <int R>
using TileStrip = StripPolicy<R, true, true, true>;

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One image in 32-bit word units.
struct Geom {
    const uint32_t* in;
    uint32_t* out;
    int64_t stride;   // words between rows
    int32_t height;   // rows
    int32_t width;    // pixels per row
    int32_t wd;       // words per row the kernels touch (whole B-bit words)
    int64_t plane;    // words between output planes (kModeDirections only)
    // grey input (threshold then edges): rows of grey_stride bytes; a byte
    // >= thr is white. Used by the grey kernels.
    const uint8_t* grey;
    int64_t grey_stride;
    uint32_t thr;
};

// Four grey bytes against the threshold at once, in one 32-bit word. With
// k = 256 - thr, a byte is >= thr exactly when byte + k carries out of its
// eight bits. The low seven bits of all four bytes are added in one go
// (their sums stay inside the byte), and the carry out of each byte is the
// majority of its top bit, k's top bit and the carry into them. Bit 8i + 7
// of the result is set when byte i >= thr; the other bits are junk. kk is k
// in every byte and kk7 its low seven bits; thr = 256 gives k = 0 (no byte
// reaches it), thr = 0 is the caller's (every byte reaches it).
__device__ __forceinline__ uint32_t ge_top4(uint32_t four, uint32_t kk, uint32_t kk7) {
    const uint32_t lo = (four & 0x7f7f7f7fu) + kk7;
    return (four & kk) | ((four | kk) & lo);
}

// Exchange the bits selected by m with those d places above them.
__device__ __forceinline__ uint32_t swap_bits(uint32_t x, int d, uint32_t m) {
    const uint32_t t = ((x >> d) ^ x) & m;
    return x ^ t ^ (t << d);
}

// One packed word from 32 grey bytes held in two 128-bit values: bit x is
// white (1) when byte x >= thr (0 <= thr <= 256). Dword m holds pixels
// 4m..4m+3, each flag at bit 8b + 7 (b = pixel - 4m); shifting dword m's
// flags down by 7 - m gathers pixel 4m + b at bit 8b + m, and moving every
// bit from 8b + m to 4m + b (a rotation of the five bit-index bits by two
// places) takes four exchanges of index bits: 2 and 4, 1 and 3, 0 and 2,
// 0 and 1. About 55 bitwise operations per word instead of a compare and
// a select per byte.
__device__ __forceinline__ uint32_t threshold_word(const u32x4& a, const u32x4& b, uint32_t thr) {
    const uint32_t kk = ((256u - thr) & 0xffu) * 0x01010101u, kk7 = kk & 0x7f7f7f7fu;
    const uint32_t d[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t t = ge_top4(d[7], kk, kk7) & 0x80808080u;
#pragma unroll
    for (int m = 0; m < 7; ++m) t |= (ge_top4(d[m], kk, kk7) >> (7 - m)) & (0x01010101u << m);
    t = swap_bits(t, 12, 0x0000f0f0u);
    t = swap_bits(t, 6, 0x00cc00ccu);
    t = swap_bits(t, 3, 0x0a0a0a0au);
    t = swap_bits(t, 1, 0x22222222u);
    return thr == 0 ? 0xffffffffu : t;
}

// The 32 grey bytes of packed word j of a row, as 16-byte blocks counted
// from the 16-byte boundary at or before the row start (r = the row
// start's offset from it): block b starts 32j + 16b bytes after that
// boundary, clamped to the row's last block, so every block loaded holds at
// least one byte of the row and lies in the same memory page as that byte
// (no load can fault, whatever the row's alignment or the word's place).
// Bytes at or past the width come out as junk bits that the caller masks.
// ALIGNED (r = 0): the word is two blocks; otherwise three, and the word's
// bytes start r bytes into the first. INSIDE: all 32 bytes of the word lie
// in the row; aligned, both blocks then hold only row bytes and need no
// clamp (unaligned, the third block of a row that happens to start on a
// boundary holds none, so it stays clamped).
template <bool ALIGNED>
struct GreyBlocks {
    u32x4 q[ALIGNED ? 2 : 3];
};

template <bool ALIGNED, bool NT, bool INSIDE = false>
__device__ __forceinline__ GreyBlocks<ALIGNED> load_grey_word(const uint8_t* row, int j,
                                                              int32_t width) {
    const uint32_t r = ALIGNED ? 0u : (uint32_t)((uintptr_t)row & 15u);
    const uint8_t* base = row - r;
    const uint32_t last = (r + (uint32_t)width - 1u) & ~15u;
    GreyBlocks<ALIGNED> gb;
#pragma unroll
    for (int b = 0; b < (ALIGNED ? 2 : 3); ++b) {
        uint32_t off = 32u * (uint32_t)j + 16u * b;
        if constexpr (!(INSIDE && ALIGNED)) off = off < last ? off : last;
        const u32x4* p = reinterpret_cast<const u32x4*>(base + off);
        gb.q[b] = NT ? __builtin_nontemporal_load(p) : *p;
    }
    return gb;
}

// The packed word of unaligned blocks whose word starts QD dwords and rb
// bytes into the first block: each of its dwords is a funnel of two loaded
// neighbours (constant indices, so the blocks stay in registers).
template <int QD>
__device__ __forceinline__ uint32_t grey_word_at(const GreyBlocks<false>& gb, uint32_t rb,
                                                 uint32_t thr) {
    const uint32_t d[12] = {gb.q[0].x, gb.q[0].y, gb.q[0].z, gb.q[0].w,
                            gb.q[1].x, gb.q[1].y, gb.q[1].z, gb.q[1].w,
                            gb.q[2].x, gb.q[2].y, gb.q[2].z, gb.q[2].w};
    uint32_t o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = __builtin_amdgcn_alignbyte(d[QD + k + 1], d[QD + k], rb);
    const u32x4 a = {o[0], o[1], o[2], o[3]}, b = {o[4], o[5], o[6], o[7]};
    return threshold_word(a, b, thr);
}

// The packed word of those blocks (bit k: byte 32j + k >= thr). Unaligned:
// the word starts r bytes into the first block, r being the same for every
// lane of a row (so the switch is uniform).
template <bool ALIGNED>
__device__ __forceinline__ uint32_t grey_word(const GreyBlocks<ALIGNED>& gb, const uint8_t* row,
                                              uint32_t thr) {
    if constexpr (ALIGNED) {
        return threshold_word(gb.q[0], gb.q[1], thr);
    } else {
        const uint32_t r = (uint32_t)((uintptr_t)row & 15u), rb = r & 3u;
        switch (r >> 2) {
            case 0: return grey_word_at<0>(gb, rb, thr);
            case 1: return grey_word_at<1>(gb, rb, thr);
            case 2: return grey_word_at<2>(gb, rb, thr);
            default: return grey_word_at<3>(gb, rb, thr);
        }
    }
}

// ------------------------------------------------------------ word helpers --

// Bits of word j that hold pixels x < width.
__device__ __forceinline__ uint32_t valid_bits(int j, int32_t width) {
    const int64_t v = (int64_t)width - 32ll * j;
    if (v >= 32) return 0xffffffffu;
    if (v <= 0) return 0u;
    return (1u << (uint32_t)v) - 1u;
}

// Image shifted right by one pixel (section 4): bit x of the result holds
// pixel x - 1, the left neighbour n4 of Fig. 1. `prev` is the word before c.
__device__ __forceinline__ uint32_t west_of(uint32_t c, uint32_t prev) {
    return __builtin_amdgcn_alignbit(c, prev, 31);
}

// Image shifted left by one pixel: bit x holds pixel x + 1, neighbour n8.
__device__ __forceinline__ uint32_t east_of(uint32_t c, uint32_t next) {
    return __builtin_amdgcn_alignbit(next, c, 1);
}

// Lane i receives v of lane i - 1; lane 0 receives `fill` (DPP wave_shr:1).
__device__ __forceinline__ uint32_t from_lower_lane(uint32_t v, uint32_t fill) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x138, 0xf, 0xf, false);
}

// Lane i receives v of lane i + 1; lane 63 receives `fill` (DPP wave_shl:1).
__device__ __forceinline__ uint32_t from_upper_lane(uint32_t v, uint32_t fill) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x130, 0xf, 0xf, false);
}

// The same shifts with 0 shifted in (bound_ctrl), one instruction each.
__device__ __forceinline__ uint32_t from_lower_lane0(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t from_upper_lane0(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xf, 0xf, true);
}

// Second clause of the definition in section 1, bit-sliced over 32 pixels:
// bit x is 1 when at most one of the eight neighbour words has a 0 (black)
// at bit x. `none` tracks "no black so far", `one` "at most one so far".
__device__ __forceinline__ uint32_t at_most_one_black(uint32_t a1, uint32_t a2, uint32_t a3,
                                                      uint32_t a4, uint32_t a5, uint32_t a6,
                                                      uint32_t a7, uint32_t a8) {
    uint32_t none = a1 & a2;
    uint32_t one = a1 | a2;
    one = (one & a3) | none; none &= a3;
    one = (one & a4) | none; none &= a4;
    one = (one & a5) | none; none &= a5;
    one = (one & a6) | none; none &= a6;
    one = (one & a7) | none; none &= a7;
    one = (one & a8) | none;
    return one;
}

// Output word for pixel word c with its eight neighbour words (Fig. 1
// numbering: n1 NE, n2 N, n3 NW, n4 W, n5 SW, n6 S, n7 SE, n8 E).
template <int MODE>
__device__ __forceinline__ uint32_t edge_word(uint32_t c, uint32_t n1, uint32_t n2, uint32_t n3,
                                              uint32_t n4, uint32_t n5, uint32_t n6, uint32_t n7,
                                              uint32_t n8) {
    const uint32_t white4 = n2 | n4 | n6 | n8;                 // section 1, Edge(p)
    if constexpr (MODE == kModePlain) {
        return ~c & white4;
    } else if constexpr (MODE == kModePeel) {
        return c | white4;                                      // c | Edge(c)
    } else if constexpr (MODE == kModeCopy) {
        return c;
    } else {
        const uint32_t few = at_most_one_black(n1, n2, n3, n4, n5, n6, n7, n8);
        if constexpr (MODE == kModeFull) return ~c & (white4 | few);
        else return ~c & few;
    }
}

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t wave_uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Spread consecutive workgroups over the eight XCDs in contiguous ranges:
// the dispatcher sends workgroup b to XCD b % 8, so logical block order
// b' keeps neighbouring tiles (which share halo rows) in one XCD's L2.
// XCD x takes the q + (x < rem) consecutive logical blocks from
// x * q + min(x, rem); written without a branch, so that the kernel's
// argument loads are issued together.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
    constexpr uint32_t X = 8;
    const uint32_t xcd = b % X, idx = b / X, q = nb / X, rem = nb % X;
    return xcd * q + (xcd < rem ? xcd : rem) + idx;
}

template <int VW, bool NT>
__device__ __forceinline__ void load_words(const uint32_t* p, uint32_t (&w)[VW]) {
    if constexpr (VW == 4) {
        const u32x4* vp = reinterpret_cast<const u32x4*>(p);
        const u32x4 v = NT ? __builtin_nontemporal_load(vp) : *vp;
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    } else if constexpr (VW == 2) {
        const u32x2* vp = reinterpret_cast<const u32x2*>(p);
        const u32x2 v = NT ? __builtin_nontemporal_load(vp) : *vp;
        w[0] = v.x; w[1] = v.y;
    } else {
        w[0] = NT ? __builtin_nontemporal_load(p) : *p;
    }
}

template <int VW, bool NT>
__device__ __forceinline__ void store_words(uint32_t* p, const uint32_t (&w)[VW]) {
    if constexpr (VW == 4) {
        u32x4 v; v.x = w[0]; v.y = w[1]; v.z = w[2]; v.w = w[3];
        if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(p));
        else *reinterpret_cast<u32x4*>(p) = v;
    } else if constexpr (VW == 2) {
        u32x2 v; v.x = w[0]; v.y = w[1];
        if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<u32x2*>(p));
        else *reinterpret_cast<u32x2*>(p) = v;
    } else {
        if constexpr (NT) __builtin_nontemporal_store(w[0], p);
        else *p = w[0];
    }
}

// --------------------------------------------------------------- strips ----

// Rows [y0, y1) of words [j0, j0 + 64*VW) of image g, by the calling
// wavefront (all 64 lanes active; every branch below is wave-uniform).
// WHOLE: the span lies inside the row. Otherwise (the row's last chunk)
// VW divides the row's word count (strip_vw), so each lane's words lie
// either all inside the row or all past its end. Either way a lane inside
// moves its VW words with one vector load and store; lanes past the end
// load the chunk's first words instead (an address inside the row; their
// words become border words) and store nothing.
// `bw` is the border word (all ones for a white border, zero for black).
//
// EDGES: some word just outside the span lies inside the row, so lanes 0
// and 63 load it with each row; otherwise both carries are border words.
//
// Each lane keeps Pol::prefetch rows in flight in the ring q[]: the slot of
// the row just consumed is refilled with the row that many rows further down.
// With Pol::oneshot the unit is a tile of at most Pol::prefetch rows
// (y1 - y0 <= Pol::prefetch, kept by the caller) whose rows are all loaded
// before the first is used.
// Loads never branch: rows past y1 re-read row y1 (an L1 hit) and rows
// outside the image are clamped into it and replaced by the border after
// the load, so the hardware's in-order load counter waits exactly for the
// row being consumed.
template <int VW, int MODE, bool WHOLE, bool EDGES, class Pol>
__device__ __forceinline__ void strip_body(const Geom& g, int j0, int y0, int y1, uint32_t bw,
                                           bool invert) {
    constexpr int P = Pol::prefetch;
    const int lane = threadIdx.x & (kWave - 1);
    const int jl = j0 + lane * VW;
    // the display inversion as a mask: (x ^ inv) & vm is the edge word,
    // inverted or not, with its pad bits cleared (one three-input operation)
    const uint32_t inv = invert ? 0xffffffffu : 0u;

    uint32_t vm[VW], om[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        vm[k] = valid_bits(jl + k, g.width);
        om[k] = bw & ~vm[k];
    }

    // Words just outside the wavefront's span: lane 0 needs the word on the
    // left, lane 63 the word on the right. Other lanes load a harmless word.
    const int je = lane == 0 ? j0 - 1 : j0 + kWave * VW;
    const bool has_e = (lane == 0 && j0 > 0) || (lane == kWave - 1 && je < g.wd);
    const int je_load = has_e ? je : j0;
    const uint32_t vme = valid_bits(je, g.width), ome = bw & ~vme;

    struct Raw { uint32_t w[VW]; uint32_t e; };
    struct Row { uint32_t c[VW], w[VW], e[VW]; };

    const bool inside_row = WHOLE || jl < g.wd;   // the lane's VW words are in the row
    const int jv = inside_row ? jl : j0;
    auto load_raw = [&](int y) {
        const int yc = y < 0 ? 0 : (y >= g.height ? g.height - 1 : y);
        Raw r;
        const uint32_t* rp = g.in + (int64_t)yc * g.stride;
        load_words<VW, Pol::nt_load>(rp + jv, r.w);
        if constexpr (EDGES) r.e = rp[je_load];
        else r.e = bw;
        return r;
    };

    // Pad bits take the border colour, rows outside the image become border
    // rows; then the row shifted right (west neighbours, n4) and shifted
    // left (east neighbours, n8) are formed with funnel shifts, the carry
    // words crossing lanes by DPP.
    auto shift_row = [&](const Raw& r, int y) {
        const bool inside = (unsigned)y < (unsigned)g.height;
        Row o;
#pragma unroll
        for (int k = 0; k < VW; ++k) o.c[k] = inside ? ((r.w[k] & vm[k]) | om[k]) : bw;
        const uint32_t e = (EDGES && inside && has_e) ? ((r.e & vme) | ome) : bw;
        const uint32_t left = from_lower_lane(o.c[VW - 1], e);
        const uint32_t right = from_upper_lane(o.c[0], e);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            o.w[k] = west_of(o.c[k], k > 0 ? o.c[k - 1] : left);
            o.e[k] = east_of(o.c[k], k + 1 < VW ? o.c[k + 1] : right);
        }
        return o;
    };

    auto store_row = [&](uint32_t* op, const uint32_t (&res)[VW]) {
        if (inside_row) store_words<VW, Pol::nt_store>(op + jl, res);
    };

    auto emit = [&](int y, const Row& up, const Row& cur, const Row& dn) {
        uint32_t* op = g.out + (int64_t)y * g.stride;
        if constexpr (MODE == kModeDirections) {
            // fundamental edges (section 4): the mask ANDed with the image
            // shifted right (left edge, n4), left (right edge, n8), down
            // (up edge, n2) and up (down edge, n6)
            uint32_t l[VW], r[VW], u[VW], d[VW];
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                const uint32_t m = ~cur.c[k] & vm[k];
                l[k] = m & cur.w[k];
                r[k] = m & cur.e[k];
                u[k] = m & up.c[k];
                d[k] = m & dn.c[k];
            }
            store_row(op, l);
            store_row(op + g.plane, r);
            store_row(op + 2 * g.plane, u);
            store_row(op + 3 * g.plane, d);
        } else {
            uint32_t res[VW];
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                res[k] = (edge_word<MODE>(cur.c[k], up.e[k], up.c[k], up.w[k], cur.w[k], dn.w[k],
                                          dn.c[k], dn.e[k], cur.e[k]) ^ inv) & vm[k];
            }
            store_row(op, res);
        }
    };

    if constexpr (Pol::oneshot) {
        // every row of the tile and its two halo rows requested at once
        // (rows past y1 re-read row y1); then each row as it arrives
        Raw t[P + 2];
#pragma unroll
        for (int i = 0; i < P + 2; ++i) t[i] = load_raw(min(y0 - 1 + i, y1));
        __builtin_amdgcn_sched_barrier(0);
        Row up = shift_row(t[0], y0 - 1);
        Row cur = shift_row(t[1], y0);
#pragma unroll
        for (int o = 0; o < P; ++o) {
            const int y = y0 + o;
            if (y < y1) {
                const Row dn = shift_row(t[o + 2], y + 1);
                emit(y, up, cur, dn);
                up = cur;
                cur = dn;
            }
        }
        return;
    }
    const Raw ra = load_raw(y0 - 1);
    const Raw rb = load_raw(y0);
    Raw q[P];
#pragma unroll
    for (int u = 0; u < P; ++u) q[u] = load_raw(min(y0 + 1 + u, y1));
    Row up = shift_row(ra, y0 - 1);
    Row cur = shift_row(rb, y0);
    int r = y0;
    for (; r + P <= y1; r += P) {   // whole groups
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int y = r + u;
            const Row dn = shift_row(q[u], y + 1);
            q[u] = load_raw(min(y + 1 + P, y1));
            emit(y, up, cur, dn);
            up = cur;
            cur = dn;
            // Keep each row's work in its own slot of the schedule; hoisting
            // a later row's arithmetic would make the wavefront wait for
            // every load in flight.
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int u = 0; u + 1 < P; ++u) {        // last partial group
        const int y = r + u;
        if (y < y1) {
            const Row dn = shift_row(q[u], y + 1);
            emit(y, up, cur, dn);
            up = cur;
            cur = dn;
        }
    }
}

// Grey input as bands (section 7's threshold fused into the edge pass; the
// binary image is never stored). A workgroup of nw wavefronts loads the
// nw * RW consecutive rows y0 - 1 .. y0 + nw * RW - 2 of one 64-word chunk,
// every row's 32 bytes per lane in flight at once, thresholds them into
// packed words in LDS, and then computes the nw * RW - 2 rows between the
// first and the last from LDS. Concurrent workgroups take consecutive
// chunks and bands, so the rows in flight form one compact window of the
// image; a wavefront walking a long strip of its own keeps its next rows
// in flight at a different place of the image from every other, which
// measured slower for grey rows (32 bytes per lane and row, eight times a
// packed row). An LDS row holds, in this order, the pixel left of the chunk
// (replicated over the word), the 64 words and the pixel right of it, so
// the west and east neighbour words of every lane come from LDS. Words
// past the row end hold the border colour, pad bits too.
constexpr int kBandPitch = kWave + 2;

// WHOLE: every pixel of the chunk lies inside the row (no clamps, no pad
// bits); otherwise the row's last chunk.
template <int MODE, int RW, bool ALIGNED, bool WHOLE, class Pol>
__device__ __forceinline__ void grey_band_unit(const Geom& g, uint32_t* tile, int nw, int j0,
                                               int64_t y0, uint32_t bw, bool invert) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = wave_uniform(threadIdx.x / kWave);
    const int jl = j0 + lane;
    const uint32_t vm = WHOLE ? 0xffffffffu : valid_bits(jl, g.width), om = bw & ~vm;
    const int64_t xl = 32ll * j0 - 1, xr = 32ll * (j0 + kWave);
    const bool has_l = j0 > 0, has_r = xr < g.width;
    const bool edge_lane = lane == 0 || lane == kWave - 1;
    const int64_t xe = lane == 0 ? (has_l ? xl : 0) : (has_r ? xr : 0);

    GreyBlocks<ALIGNED> q[RW];
    uint32_t eb[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int64_t y = y0 - 1 + i * nw + w;
        const int64_t yc = y < 0 ? 0 : (y >= g.height ? g.height - 1 : y);
        const uint8_t* rp = g.grey + yc * g.grey_stride;
        q[i] = load_grey_word<ALIGNED, Pol::nt_load, WHOLE>(rp, jl, g.width);
        eb[i] = edge_lane ? rp[xe] : 0u;
    }
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int l = i * nw + w;
        const int64_t y = y0 - 1 + l;
        const int64_t yc = y < 0 ? 0 : (y >= g.height ? g.height - 1 : y);
        const bool inside = y >= 0 && y < g.height;
        uint32_t* t = tile + l * kBandPitch;
        const uint32_t word = grey_word<ALIGNED>(q[i], g.grey + yc * g.grey_stride, g.thr);
        t[1 + lane] = inside ? (WHOLE ? word : ((word & vm) | om)) : bw;
        const uint32_t side = eb[i] >= g.thr ? 0xffffffffu : 0u;
        if (lane == 0) t[0] = inside && has_l ? side : bw;
        if (lane == kWave - 1) t[kBandPitch - 1] = inside && has_r ? side : bw;
    }
    __syncthreads();

    // output rows y0 + o, o = 0 .. nw * RW - 3; wavefront w takes a
    // contiguous share
    const int ob = nw * RW - 2;
    const int o0 = w * ob / nw, o1 = (w + 1) * ob / nw;
    auto row = [&](int l, uint32_t& c, uint32_t& wv, uint32_t& ev) {
        const uint32_t* t = tile + l * kBandPitch + lane;
        c = t[1];
        wv = west_of(c, t[0]);
        ev = east_of(c, t[2]);
    };
    uint32_t uc, uw, ue, cc, cw, ce;
    row(o0, uc, uw, ue);
    row(o0 + 1, cc, cw, ce);
    for (int o = o0; o < o1; ++o) {
        uint32_t dc, dw, de;
        row(o + 2, dc, dw, de);
        const int64_t y = y0 + o;
        if (y < g.height && (WHOLE || jl < g.wd)) {
            const uint32_t v = edge_word<MODE>(cc, ue, uc, uw, cw, dw, dc, de, ce) & vm;
            uint32_t* op = g.out + y * g.stride + jl;
            const uint32_t res = invert ? (v ^ vm) : v;
            if constexpr (Pol::nt_store) __builtin_nontemporal_store(res, op);
            else *op = res;
        }
        uc = cc; uw = cw; ue = ce;
        cc = dc; cw = dw; ce = de;
    }
}

template <int VW, int MODE, class Pol = CachedStrip>
__device__ __forceinline__ void strip_unit(const Geom& g, int j0, int y0, int y1, uint32_t bw,
                                           bool invert) {
    const bool whole = j0 + kWave * VW <= g.wd;
    const bool edges = j0 > 0 || j0 + kWave * VW < g.wd;
    if (whole) {
        if (edges) strip_body<VW, MODE, true, true, Pol>(g, j0, y0, y1, bw, invert);
        else strip_body<VW, MODE, true, false, Pol>(g, j0, y0, y1, bw, invert);
    } else {
        if (edges) strip_body<VW, MODE, false, true, Pol>(g, j0, y0, y1, bw, invert);
        else strip_body<VW, MODE, false, false, Pol>(g, j0, y0, y1, bw, invert);
    }
}

// ------------------------------------------------------------------ bands ----

// Bands: a workgroup of nw wavefronts loads the nw * RW consecutive rows
// y0 - 1 .. y0 + nw * RW - 2 of one chunk of 64 * VW words (wavefront w the
// rows w, w + nw, ...), every row in flight at once; writes them to LDS with
// pad bits and rows outside the image set to the border, together with the
// word just left and the word just right of the chunk; and computes the
// nw * RW - 2 rows between the first and the last from LDS, each wavefront a
// contiguous share. Neighbouring bands overlap by two rows, so the halo
// rows cost 2 / (nw * RW) of the reads. VW divides the row's word count
// (strip_vw): a lane's words are all inside the row or all past its end.
// An LDS row holds the left word at kBandLeft, the chunk's words from
// kBandBody (16-byte aligned) and the right word after them.
constexpr int kBandLeft = 3, kBandBody = 4;
__host__ __device__ constexpr int band_pitch(int vw) { return kWave * vw + 8; }

template <int VW, int RW, int MODE>
__device__ __forceinline__ void band_unit(const Geom& g, uint32_t* lds, int nw, int j0,
                                          int64_t y0, uint32_t bw, bool invert) {
    constexpr int PITCH = band_pitch(VW), RIGHT = kBandBody + kWave * VW;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = wave_uniform(threadIdx.x / kWave);
    const int jl = j0 + lane * VW;
    const bool inside_row = jl < g.wd;
    const int jv = inside_row ? jl : j0;
    uint32_t vm[VW], om[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        vm[k] = valid_bits(jl + k, g.width);
        om[k] = bw & ~vm[k];
    }
    const uint32_t inv = invert ? 0xffffffffu : 0u;    // as in strip_body
    const bool has_l = j0 > 0, has_r = j0 + kWave * VW < g.wd;
    // lane 0 loads the word left of the chunk, lane 63 the word right of it
    // (when inside the row); the other lanes load the chunk's first word
    const int je = (lane == 0 && has_l) ? j0 - 1 : ((lane == kWave - 1 && has_r) ? j0 + kWave * VW : j0);
    const uint32_t vme = valid_bits(j0 + kWave * VW, g.width), ome = bw & ~vme;

    uint32_t q[RW][VW], e[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int64_t y = y0 - 1 + (int64_t)i * nw + w;
        const int64_t yc = y < 0 ? 0 : (y >= g.height ? g.height - 1 : y);
        const uint32_t* rp = g.in + yc * g.stride;
        load_words<VW, true>(rp + jv, q[i]);
        e[i] = rp[je];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int l = i * nw + w;
        const int64_t y = y0 - 1 + l;
        const bool inside = y >= 0 && y < g.height;
        uint32_t v[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) v[k] = inside ? ((q[i][k] & vm[k]) | om[k]) : bw;
        uint32_t* t = lds + l * PITCH;
        store_words<VW, false>(t + kBandBody + lane * VW, v);
        if (lane == 0) t[kBandLeft] = inside && has_l ? e[i] : bw;
        if (lane == kWave - 1) t[RIGHT] = inside && has_r ? ((e[i] & vme) | ome) : bw;
    }
    __syncthreads();

    struct Row { uint32_t c[VW], wv[VW], ev[VW]; };
    auto row = [&](int l) {
        const uint32_t* t = lds + l * PITCH;
        Row r;
        load_words<VW, false>(t + kBandBody + lane * VW, r.c);
        const uint32_t left = from_lower_lane(r.c[VW - 1], t[kBandLeft]);
        const uint32_t right = from_upper_lane(r.c[0], t[RIGHT]);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            r.wv[k] = west_of(r.c[k], k > 0 ? r.c[k - 1] : left);
            r.ev[k] = east_of(r.c[k], k + 1 < VW ? r.c[k + 1] : right);
        }
        return r;
    };
    const int ob = nw * RW - 2;
    const int o0 = w * ob / nw, o1 = (w + 1) * ob / nw;
    Row up = row(o0), cur = row(o0 + 1);
    for (int o = o0; o < o1; ++o) {
        const Row dn = row(o + 2);
        const int64_t y = y0 + o;
        if (y < g.height && inside_row) {
            uint32_t* op = g.out + y * g.stride + jl;
            if constexpr (MODE == kModeDirections) {
                // the four fundamental edges (section 4), as in strip_body
                uint32_t l[VW], r[VW], u[VW], d[VW];
#pragma unroll
                for (int k = 0; k < VW; ++k) {
                    const uint32_t m = ~cur.c[k] & vm[k];
                    l[k] = m & cur.wv[k];
                    r[k] = m & cur.ev[k];
                    u[k] = m & up.c[k];
                    d[k] = m & dn.c[k];
                }
                store_words<VW, true>(op, l);
                store_words<VW, true>(op + g.plane, r);
                store_words<VW, true>(op + 2 * g.plane, u);
                store_words<VW, true>(op + 3 * g.plane, d);
            } else {
                uint32_t res[VW];
#pragma unroll
                for (int k = 0; k < VW; ++k)
                    res[k] = (edge_word<MODE>(cur.c[k], up.ev[k], up.c[k], up.wv[k], cur.wv[k],
                                              dn.wv[k], dn.c[k], dn.ev[k], cur.ev[k]) ^ inv) &
                             vm[k];
                store_words<VW, true>(op, res);
            }
        }
        up = cur;
        cur = dn;
    }
}

// ---------------------------------------------------------------- peeling ----

// Iterated peeling of the edge (edge detection as the step that thinning
// repeats, section 1): one peel turns every edge point white. Since
// Edge(p) = ~p & (n2 | n4 | n6 | n8), the peeled pixel is p | n2 | n4 | n6 | n8:
// one level of white dilation by the 4-neighbour cross. A peel unit forms L
// levels in registers while its wavefront walks down the rows, so L peels
// cost one read and one write of the image.
//
// Lanes: a wavefront covers 64 consecutive 32-bit words of each row, one per
// lane, and stores lanes 1..62 only (kPeelSpan words per chunk); lanes 0 and
// 63 hold the words on either side as a halo. Their outer neighbours are
// never loaded (black is shifted in), so after j levels the bits within j
// pixels of a halo word's far side may be wrong; with L <= 31 the bit next
// to the stored span never is.
//
// Outside the image: words past the row ends and rows above and below start
// as border words and are then dilated like the image itself. The region
// that evolves is a rectangle containing the image, and in a rectangle the
// shortest 4-connected path between two pixels inside never needs to leave
// the image, so the stored words equal those of the definition in which
// outside pixels keep the border colour at every step (white outside stays
// white in both readings).
//
// Level j of row r is L_j(r) = c | W(c) | E(c) | L_{j-1}(r-1) | L_{j-1}(r+1)
// with c = L_{j-1}(r) and W, E its one-pixel shifts (carries from the
// neighbouring lanes by DPP): six VALU operations per word and level. It is
// formed at the step where level 0 reaches row r + j; each level keeps its
// two most recent rows. EDGEOUT stores L_L & ~L_{L-1}, the edge map of the
// image after L - 1 peels.
constexpr int kPeelSpan = kWave - 2;
// Steps per loop body of peel_unit, and rows loaded ahead of use (groups
// of 6, 9 and 12 steps measured no faster at 8192^2 and 16384^2).
constexpr int kPeelGroup = 3;

// Warm-up. A strip's walk starts at t0 = y0 - L, and level j first reaches
// a row the strip needs (row y0 - L + j, which level j + 1 needs for its
// own first such row) at relative step s = t - t0 = 2j. Until then its rows
// are never used, so in the first 2L steps the levels above s / 2 are not
// formed: they only pass their input rows along (register renaming), which
// hands each level the two rows below before it starts forming. Levels are
// switched on kPeelPhase at a time, once per group of steps; this removes
// about a fifth of the work of a strip about 2L rows tall.
constexpr int kPeelPhase = 3;

// How many of the n levels lo+1..lo+n of one wavefront the group of p
// steps from relative step s forms: those that the group's last step
// (s + p - 1) needs, rounded up to a multiple of kPeelPhase (at most n).
__device__ __forceinline__ int peel_formed(int s, int p, int lo, int n) {
    int need = (s + p - 1) / 2 - lo;
    need = need < 0 ? 0 : need;
    need = (need + kPeelPhase - 1) / kPeelPhase * kPeelPhase;
    return need < n ? need : n;
}

// f(std::integral_constant<int, A>{}) for the phase count A = act, where
// act is a count peel_formed returns for n = N (a multiple of kPeelPhase
// below N, or N).
template <int N, int K = 0, class F>
__device__ __forceinline__ void peel_phase(int act, F&& f) {
    if constexpr (K * kPeelPhase >= N) {
        f(std::integral_constant<int, N>{});
    } else {
        if (act <= K * kPeelPhase) f(std::integral_constant<int, K * kPeelPhase>{});
        else peel_phase<N, K + 1>(act, f);
    }
}

template <int L, bool EDGEOUT, class Pol>
__device__ __forceinline__ void peel_unit(const Geom& g, int64_t chunk, int y0, int y1,
                                          uint32_t bw) {
    static_assert(L >= 1 && L <= 31, "the halo lanes carry 32 pixels");
    // P rows in flight, P a multiple of three: each level's rows rotate
    // through three registers, so a loop body of P steps needs no moves
    constexpr int P = kPeelGroup;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t j = chunk * kPeelSpan - 1 + lane;      // may lie outside the row
    const bool inrow = j >= 0 && j < g.wd;
    const bool keep = inrow && lane >= 1 && lane <= kWave - 2;
    const uint32_t vm = inrow ? valid_bits((int)j, g.width) : 0u;
    const uint32_t om = bw & ~vm;                        // outside the row: all border
    const int64_t jl = inrow ? j : (j < 0 ? 0 : (int64_t)g.wd - 1);

    auto load = [&](int y) -> uint32_t {
        const int yc = y < 0 ? 0 : (y >= g.height ? g.height - 1 : y);
        const uint32_t* p = g.in + (int64_t)yc * g.stride + jl;
        return Pol::nt_load ? __builtin_nontemporal_load(p) : *p;
    };

    uint32_t A[L], B[L];     // level i: rows t-i-2 and t-i-1 at the start of step t
#pragma unroll
    for (int i = 0; i < L; ++i) { A[i] = bw; B[i] = bw; }

    // one step forming levels 1..ACT (the levels above only pass rows along)
    auto step = [&](auto act_tag, int t, uint32_t raw) {
        constexpr int ACT = decltype(act_tag)::value;
        uint32_t n = (unsigned)t < (unsigned)g.height ? ((raw & vm) | om) : bw;   // L_0(t)
#pragma unroll
        for (int i = 0; i < L; ++i) {
            // level i + 1 at row t - i - 1 from level i rows t-i-2, t-i-1, t-i
            const uint32_t c = B[i];
            uint32_t v = c;
            if (i < ACT) {
                const uint32_t lw = from_lower_lane0(c), le = from_upper_lane0(c);
                v = (c | west_of(c, lw) | east_of(c, le)) | (A[i] | n);
            }
            A[i] = c;
            B[i] = n;
            n = v;
        }
        const int y = t - L;                  // n = L_L(y); A[L-1] = L_{L-1}(y)
        if (y >= y0 && keep) {
            const uint32_t res = (EDGEOUT ? (n & ~A[L - 1]) : n) & vm;
            uint32_t* op = g.out + (int64_t)y * g.stride + j;
            if constexpr (Pol::nt_store) __builtin_nontemporal_store(res, op);
            else *op = res;
        }
    };

    const int t0 = y0 - L, tlast = y1 - 1 + L;
    uint32_t q[P];
#pragma unroll
    for (int u = 0; u < P; ++u) q[u] = load(min(t0 + u, tlast));
    auto group = [&](auto act_tag, int t) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const uint32_t w = q[u];
            q[u] = load(min(t + u + P, tlast));
            step(act_tag, t + u, w);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    constexpr auto all = std::integral_constant<int, L>{};
    int t = t0;
    if constexpr (L > kPeelPhase) {
        for (; t - t0 < 2 * L && t + P <= tlast + 1; t += P)
            peel_phase<L>(peel_formed(t - t0, P, 0, L), [&](auto a) { group(a, t); });
    }
    for (; t + P <= tlast + 1; t += P) group(all, t);
#pragma unroll
    for (int u = 0; u + 1 < P; ++u)
        if (t + u <= tlast) step(all, t + u, q[u]);
}

// Peeling with VW consecutive words per lane (one 64- or 128-bit load and
// store per row, VW = 2 or 4) for up to kPeelVecLevels levels: the
// wavefront covers 64 * VW words of each row and has no halo lanes. The word
// just left of its span (held by lane 0) and the word just right of it
// (lane 63) sit in one more register per level and form their levels too,
// with black shifted in from beyond them; the error that brings starts at
// their far bits and moves one pixel per level, so with L <= 31 the bit next
// to the span stays exact (the argument of the halo lanes of peel_unit).
// Per level and row: the words' funnel shifts and ORs as in peel_unit, the
// DPP carries once per lane, the halo word's own level. Warm-up as in
// peel_unit. WHOLE: the span lies inside the row (vector loads and stores).
// Built for up to seven levels. Its loop body ends in a scheduling barrier
// only up to three levels: with the barrier and the warm-up switch-on
// together, the four-level instantiation came out of -O3 giving wrong
// words (exact at -O1, or with either taken out), and from four levels on
// the barrier does not pay anyway.
constexpr int kPeelVecLevels = 7;
constexpr int kPeelVecBarrierLevels = 3;
// The cause of the wrong four-level words was never shown; until it is, the
// barrier stays out of every instantiation from four levels up.
static_assert(kPeelVecBarrierLevels < 4,
              "four or more levels with the loop-body barrier gave wrong words at -O3");

template <int L, bool EDGEOUT, int VW, bool WHOLE, class Pol>
__device__ __forceinline__ void peel_vec_unit(const Geom& g, int j0, int y0, int y1,
                                              uint32_t bw) {
    static_assert(L >= 1 && L <= 31, "the halo words carry 32 pixels");
    constexpr int P = kPeelGroup;
    const int lane = threadIdx.x & (kWave - 1);
    const int jl = j0 + lane * VW;
    uint32_t vm[VW], om[VW];
    int jw[VW];
    bool inrow[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        vm[k] = valid_bits(jl + k, g.width);
        om[k] = bw & ~vm[k];
        inrow[k] = jl + k < g.wd;
        jw[k] = inrow[k] ? jl + k : g.wd - 1;
    }
    const bool first = lane == 0;
    const int jh = first ? j0 - 1 : j0 + kWave * VW;     // lanes 0 and 63; the rest unused
    const bool hin = jh >= 0 && jh < g.wd;
    const uint32_t vmh = hin ? valid_bits(jh, g.width) : 0u;
    const uint32_t omh = bw & ~vmh;
    const int jhl = hin ? jh : (jh < 0 ? 0 : g.wd - 1);

    struct Raw { uint32_t w[VW]; uint32_t h; };
    auto load = [&](int y) -> Raw {
        const int yc = y < 0 ? 0 : (y >= g.height ? g.height - 1 : y);
        const uint32_t* rp = g.in + (int64_t)yc * g.stride;
        Raw r;
        if constexpr (WHOLE) {
            load_words<VW, Pol::nt_load>(rp + jl, r.w);
        } else {
#pragma unroll
            for (int k = 0; k < VW; ++k) r.w[k] = rp[jw[k]];
        }
        r.h = rp[jhl];
        return r;
    };

    uint32_t A[L][VW], B[L][VW], Ah[L], Bh[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
#pragma unroll
        for (int k = 0; k < VW; ++k) { A[i][k] = bw; B[i][k] = bw; }
        Ah[i] = bw;
        Bh[i] = bw;
    }

    // one step forming levels 1..ACT (the levels above only pass rows along)
    auto step = [&](auto act_tag, int t, const Raw& raw) {
        constexpr int ACT = decltype(act_tag)::value;
        const bool inside = (unsigned)t < (unsigned)g.height;
        uint32_t n[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) n[k] = inside ? ((raw.w[k] & vm[k]) | om[k]) : bw;
        uint32_t nh = inside ? ((raw.h & vmh) | omh) : bw;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            uint32_t c[VW], v[VW];
#pragma unroll
            for (int k = 0; k < VW; ++k) { c[k] = B[i][k]; v[k] = c[k]; }
            const uint32_t ch = Bh[i];
            uint32_t vh = ch;
            if (i < ACT) {
                // lane 0 takes its left halo word, lane 63 its right one
                const uint32_t wi = from_lower_lane(c[VW - 1], ch);
                const uint32_t ei = from_upper_lane(c[0], ch);
#pragma unroll
                for (int k = 0; k < VW; ++k) {
                    const uint32_t w = west_of(c[k], k > 0 ? c[k - 1] : wi);
                    const uint32_t e = east_of(c[k], k + 1 < VW ? c[k + 1] : ei);
                    v[k] = (c[k] | w | e) | (A[i][k] | n[k]);
                }
                const uint32_t hx = first ? 0u : c[VW - 1], hy = first ? c[0] : 0u;
                vh = (ch | west_of(ch, hx) | east_of(ch, hy)) | (Ah[i] | nh);
            }
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                A[i][k] = c[k];
                B[i][k] = n[k];
                n[k] = v[k];
            }
            Ah[i] = ch;
            Bh[i] = nh;
            nh = vh;
        }
        const int y = t - L;                  // n = L_L(y); A[L-1] = L_{L-1}(y)
        if (y >= y0) {
            uint32_t res[VW];
#pragma unroll
            for (int k = 0; k < VW; ++k) res[k] = (EDGEOUT ? (n[k] & ~A[L - 1][k]) : n[k]) & vm[k];
            uint32_t* op = g.out + (int64_t)y * g.stride;
            if constexpr (WHOLE) {
                store_words<VW, Pol::nt_store>(op + jl, res);
            } else {
#pragma unroll
                for (int k = 0; k < VW; ++k)
                    if (inrow[k]) op[jl + k] = res[k];
            }
        }
    };

    const int t0 = y0 - L, tlast = y1 - 1 + L;
    Raw q[P];
#pragma unroll
    for (int u = 0; u < P; ++u) q[u] = load(min(t0 + u, tlast));
    auto group = [&](auto act_tag, int t) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const Raw w = q[u];
            q[u] = load(min(t + u + P, tlast));
            step(act_tag, t + u, w);
            if constexpr (L <= kPeelVecBarrierLevels) __builtin_amdgcn_sched_barrier(0);
        }
    };
    constexpr auto all = std::integral_constant<int, L>{};
    int t = t0;
    if constexpr (L > kPeelPhase) {
        for (; t - t0 < 2 * L && t + P <= tlast + 1; t += P)
            peel_phase<L>(peel_formed(t - t0, P, 0, L), [&](auto a) { group(a, t); });
    }
    for (; t + P <= tlast + 1; t += P) group(all, t);
#pragma unroll
    for (int u = 0; u + 1 < P; ++u)
        if (t + u <= tlast) step(all, t + u, q[u]);
}

// Peeling with the levels of one strip split over two wavefronts of a
// workgroup (twice the wavefronts for the same halo rows, half the
// registers each). Wavefront 0 loads the rows and forms levels 1..LA for a
// group of P steps, writing each step's top row (level LA) to LDS; after
// the workgroup barrier wavefront 1 forms levels LA+1..LA+LB from those P
// rows while wavefront 0 goes on with the next group. The LDS ring holds two
// groups: a group's rows are overwritten two groups later, after wavefront 1
// has passed the barrier that follows its reading them. Both wavefronts run
// the same groups, one barrier each, so the barrier count always matches.
// A group is six steps: a multiple of three, so that each level's three
// rows rotate through the same registers, and half the barriers of a
// three-step group (8-15% faster for 20 to 30 levels, measured).
// Both parts skip the warm-up like peel_unit; wavefront 1's levels start
// later, so it is given more of them (peel_split_first).
// The stored words equal those of peel_unit<LA + LB, ...>.
constexpr int kPeelSplitGroup = 6;

// Levels of wavefront 0 when a strip's L levels are split: with the
// warm-up skipped this balances the levels formed by the two wavefronts
// for strips about 2L rows tall (counted over L = 16..31).
constexpr int peel_split_first(int L) { return (3 * L + 3) / 7; }

template <int LA, int LB, bool EDGEOUT, class Pol>
__device__ __forceinline__ void peel_split_unit(const Geom& g, int64_t chunk, int y0, int y1,
                                                uint32_t bw, int role,
                                                uint32_t (*lds)[kWave]) {
    static_assert(LA >= 1 && LB >= 1 && LA + LB <= 31, "the halo lanes carry 32 pixels");
    constexpr int L = LA + LB;
    constexpr int P = kPeelSplitGroup;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t j = chunk * kPeelSpan - 1 + lane;
    const bool inrow = j >= 0 && j < g.wd;
    const bool keep = inrow && lane >= 1 && lane <= kWave - 2;
    const uint32_t vm = inrow ? valid_bits((int)j, g.width) : 0u;
    const uint32_t om = bw & ~vm;
    const int64_t jl = inrow ? j : (j < 0 ? 0 : (int64_t)g.wd - 1);

    auto load = [&](int y) -> uint32_t {
        const int yc = y < 0 ? 0 : (y >= g.height ? g.height - 1 : y);
        const uint32_t* p = g.in + (int64_t)yc * g.stride + jl;
        return Pol::nt_load ? __builtin_nontemporal_load(p) : *p;
    };

    constexpr int LM = LA > LB ? LA : LB;
    uint32_t A[LM], B[LM];
#pragma unroll
    for (int i = 0; i < LM; ++i) { A[i] = bw; B[i] = bw; }

    // the C levels of this wavefront's part fed with row n, of which the
    // first ACT are formed and the rest only pass rows along
    auto levels = [&](uint32_t n, auto count_tag, auto act_tag) -> uint32_t {
        constexpr int C = decltype(count_tag)::value;
        constexpr int ACT = decltype(act_tag)::value;
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const uint32_t c = B[i];
            uint32_t v = c;
            if (i < ACT) {
                const uint32_t lw = from_lower_lane0(c), le = from_upper_lane0(c);
                v = (c | west_of(c, lw) | east_of(c, le)) | (A[i] | n);
            }
            A[i] = c;
            B[i] = n;
            n = v;
        }
        return n;
    };

    auto finish = [&](int t, uint32_t n) {     // n = L_L(t - L); A[LB-1] = L_{L-1}(t - L)
        const int y = t - L;
        if (y >= y0 && keep) {
            const uint32_t res = (EDGEOUT ? (n & ~A[LB - 1]) : n) & vm;
            uint32_t* op = g.out + (int64_t)y * g.stride + j;
            if constexpr (Pol::nt_store) __builtin_nontemporal_store(res, op);
            else *op = res;
        }
    };

    const int t0 = y0 - L, tlast = y1 - 1 + L;
    uint32_t q[P];
#pragma unroll
    for (int u = 0; u < P; ++u) q[u] = role == 0 ? load(min(t0 + u, tlast)) : 0u;
    // one group of P steps of either part, forming ACT of its levels
    auto part0 = [&](int t, int half, auto act_tag) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int tt = t + u;
            const uint32_t raw = q[u];
            q[u] = load(min(tt + P, tlast));
            const uint32_t n0 = (unsigned)tt < (unsigned)g.height ? ((raw & vm) | om) : bw;
            if (tt <= tlast)
                lds[half * P + u][lane] = levels(n0, std::integral_constant<int, LA>{}, act_tag);
        }
    };
    auto part1 = [&](int t, int half, auto act_tag) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int tt = t + u;
            if (tt <= tlast)
                finish(tt, levels(lds[half * P + u][lane], std::integral_constant<int, LB>{},
                                  act_tag));
        }
    };
    int half = 0;
    for (int t = t0; t <= tlast; t += P, half ^= 1) {
        const bool warm = t - t0 < 2 * L;
        if (role == 0) {
            if (warm) peel_phase<LA>(peel_formed(t - t0, P, 0, LA), [&](auto a) { part0(t, half, a); });
            else part0(t, half, std::integral_constant<int, LA>{});
        }
        __syncthreads();
        if (role == 1) {
            if (warm) peel_phase<LB>(peel_formed(t - t0, P, LA, LB), [&](auto a) { part1(t, half, a); });
            else part1(t, half, std::integral_constant<int, LB>{});
        }
    }
}

// --------------------------------------------------------- narrow units ----

// Rows [ya, yb) of an image whose rows have g.wd <= 32 words: 64 / wd rows
// side by side per wavefront step, one word per lane, kNarrowSteps steps
// loaded before any is used. Lanes past the last row load a safe word and
// store nothing. A group of kNarrowSteps steps is split into its loads
// (narrow_load) and its arithmetic and stores (narrow_emit), so that a caller
// can issue the next group's loads before finishing the current one.
struct NarrowLanes {
    int wd, grp, q, j;
    bool used;
    uint32_t vm, om;
};

__device__ __forceinline__ NarrowLanes narrow_lanes(const Geom& g, uint32_t bw) {
    const int lane = threadIdx.x & (kWave - 1);
    NarrowLanes l;
    l.wd = g.wd;
    l.grp = kWave / l.wd;
    l.q = lane / l.wd;
    l.used = l.q < l.grp;
    l.j = l.used ? lane - l.q * l.wd : 0;
    l.vm = valid_bits(l.j, g.width);
    l.om = bw & ~l.vm;
    return l;
}

// The same lane layout from a planned image: grp rows per step and the
// quotient lane / wd as (lane * qmagic) >> 16 with qmagic = ceil(2^16 / wd)
// (exact for lane < 64 and wd <= 32: the error is below 64 / 2^16, less than
// the 1 / wd that separates lane / wd from the next integer). A lane whose
// word index falls outside [0, wd), as an inconsistent plan could make it,
// stays unused.
__device__ __forceinline__ NarrowLanes narrow_lanes_q(const Geom& g, int grp, uint32_t qmagic,
                                                      uint32_t bw) {
    const int lane = threadIdx.x & (kWave - 1);
    NarrowLanes l;
    l.wd = g.wd;
    l.grp = wave_uniform(grp);      // a wave-uniform loop step
    l.q = (int)(((uint32_t)lane * qmagic) >> 16);
    const int j = lane - l.q * l.wd;
    l.used = l.q < l.grp && j >= 0 && j < l.wd;
    l.j = l.used ? j : 0;
    l.vm = valid_bits(l.j, g.width);
    l.om = bw & ~l.vm;
    return l;
}

struct NarrowGroup {
    uint32_t c[kNarrowSteps], u[kNarrowSteps], d[kNarrowSteps];
};

// Loads of the group starting at row y of the unit [ya, yb). Each lane's
// row pointer is formed once and advanced by grp rows per step; lanes past
// the unit's last row read row ya instead.
__device__ __forceinline__ void narrow_load(const Geom& g, const NarrowLanes& l, int ya, int yb,
                                            int y, NarrowGroup& r) {
    const int64_t step = (int64_t)l.grp * g.stride;
    const uint32_t* row = g.in + (int64_t)(y + l.q) * g.stride + l.j;
    const uint32_t* safe = g.in + (int64_t)ya * g.stride + l.j;
#pragma unroll
    for (int i = 0; i < kNarrowSteps; ++i) {
        const int yy = y + i * l.grp + l.q;
        const bool live = l.used && yy < yb;
        const int ys = live ? yy : ya;
        const uint32_t* p = live ? row : safe;
        r.c[i] = p[0];
        r.u[i] = p[ys > 0 ? -g.stride : 0];
        r.d[i] = p[ys + 1 < g.height ? g.stride : 0];
        row += step;
    }
}

// Edge word of one lane in one step (every mode but the direction planes):
// the loaded words of its row (c), the row above (u) and the row below (d),
// pad bits and rows outside the image taken as the border; row yy.
template <int MODE>
__device__ __forceinline__ uint32_t narrow_word(const NarrowLanes& l, int yy, int height,
                                                uint32_t c, uint32_t u, uint32_t d, uint32_t bw) {
    const int j = l.j, wd = l.wd;
    const uint32_t vm = l.vm, om = l.om;
    const uint32_t cc = (c & vm) | om;
    const uint32_t uu = yy > 0 ? ((u & vm) | om) : bw;
    const uint32_t dd = yy + 1 < height ? ((d & vm) | om) : bw;
    uint32_t cl = from_lower_lane(cc, bw), cr = from_upper_lane(cc, bw);
    if (j == 0) cl = bw;
    if (j == wd - 1) cr = bw;
    uint32_t ul = bw, ur = bw, dl = bw, dr = bw;
    if constexpr (MODE == kModeFull || MODE == kModeClause2) {
        ul = from_lower_lane(uu, bw); ur = from_upper_lane(uu, bw);
        dl = from_lower_lane(dd, bw); dr = from_upper_lane(dd, bw);
        if (j == 0) { ul = bw; dl = bw; }
        if (j == wd - 1) { ur = bw; dr = bw; }
    }
    return edge_word<MODE>(cc, east_of(uu, ur), uu, west_of(uu, ul), west_of(cc, cl),
                           west_of(dd, dl), dd, east_of(dd, dr), east_of(cc, cr)) & vm;
}

// Edge words of the group starting at row y, from its loaded words.
template <int MODE>
__device__ __forceinline__ void narrow_emit(const Geom& g, const NarrowLanes& l, int yb, int y,
                                            const NarrowGroup& r, uint32_t bw, bool invert) {
    const int j = l.j, wd = l.wd;
    const uint32_t vm = l.vm, om = l.om;
    const int64_t step = (int64_t)l.grp * g.stride;
    uint32_t* row = g.out + (int64_t)(y + l.q) * g.stride + j;
#pragma unroll
    for (int i = 0; i < kNarrowSteps; ++i) {
        const int yy = y + i * l.grp + l.q;
        const bool live = l.used && yy < yb;
        uint32_t* op = row;                       // row yy of this lane
        row += step;
        if constexpr (MODE == kModeDirections) {
            const uint32_t cc = (r.c[i] & vm) | om;
            const uint32_t uu = yy > 0 ? ((r.u[i] & vm) | om) : bw;
            const uint32_t dd = yy + 1 < g.height ? ((r.d[i] & vm) | om) : bw;
            uint32_t cl = from_lower_lane(cc, bw), cr = from_upper_lane(cc, bw);
            if (j == 0) cl = bw;
            if (j == wd - 1) cr = bw;
            const uint32_t m = ~cc & vm;
            if (live) {
                op[0] = m & west_of(cc, cl);
                op[g.plane] = m & east_of(cc, cr);
                op[2 * g.plane] = m & uu;
                op[3 * g.plane] = m & dd;
            }
        } else {
            const uint32_t v = narrow_word<MODE>(l, yy, g.height, r.c[i], r.u[i], r.d[i], bw);
            if (live) op[0] = invert ? (v ^ vm) : v;
        }
    }
}

// Rows [ya, yb) by 32-bit byte offsets from one scalar base row (the row
// above ya, or row 0), for units whose rows span less than 2^32 bytes (any
// mode but the direction planes). A lane's word in its row is the base plus
// its offset, clamped to the last word the unit may read (so that lanes
// past the unit read a valid word); the rows above and below are that
// offset minus or plus the pitch, clamped to the same range. Words so read
// from outside the image are replaced by the border in narrow_word. No
// 64-bit address arithmetic and no per-row selects of pointers remain.
template <int MODE>
__device__ __forceinline__ void narrow_rows32(const Geom& g, const NarrowLanes& l, int ya, int yb,
                                              uint32_t bw, bool invert) {
    const int base_row = ya > 0 ? ya - 1 : 0;
    const int last_row = yb < g.height ? yb : g.height - 1;
    const uint32_t pitch = (uint32_t)g.stride * 4u;
    const char* in = reinterpret_cast<const char*>(g.in + (int64_t)base_row * g.stride);
    char* out = reinterpret_cast<char*>(g.out + (int64_t)base_row * g.stride);
    const uint32_t last = (uint32_t)(last_row - base_row) * pitch + (uint32_t)(l.wd - 1) * 4u;
    const uint32_t lane0 =
        l.used ? (uint32_t)(ya - base_row + l.q) * pitch + (uint32_t)l.j * 4u : 0u;
    const uint32_t step = (uint32_t)l.grp * pitch;
    for (int y = ya; y < yb; y += l.grp * kNarrowSteps) {
        const uint32_t o0 = (uint32_t)(y - ya) * pitch;
        uint32_t oc[kNarrowSteps], c[kNarrowSteps], u[kNarrowSteps], d[kNarrowSteps];
#pragma unroll
        for (int i = 0; i < kNarrowSteps; ++i) {
            oc[i] = min(lane0 + (o0 + (uint32_t)i * step), last);
            const uint32_t ou = max(oc[i], pitch) - pitch;
            const uint32_t od = min(oc[i] + pitch, last);
            c[i] = *reinterpret_cast<const uint32_t*>(in + oc[i]);
            u[i] = *reinterpret_cast<const uint32_t*>(in + ou);
            d[i] = *reinterpret_cast<const uint32_t*>(in + od);
        }
#pragma unroll
        for (int i = 0; i < kNarrowSteps; ++i) {
            const int yy = y + i * l.grp + l.q;
            uint32_t v = narrow_word<MODE>(l, yy, g.height, c[i], u[i], d[i], bw);
            v = invert ? (v ^ l.vm) : v;
            // formed in every lane before the store's branch: left to the
            // compiler, the word (and the loads of its rows above and
            // below) sink into the branch, a second round trip per group
            asm volatile("" : "+v"(v));
            if (l.used && yy < yb) *reinterpret_cast<uint32_t*>(out + oc[i]) = v;
        }
    }
}

template <int MODE>
__device__ __forceinline__ void narrow_rows(const Geom& g, const NarrowLanes& l, int ya, int yb,
                                            uint32_t bw, bool invert) {
    if constexpr (MODE != kModeDirections) {
        if ((int64_t)(yb - ya + 2) * g.stride * 4 < (int64_t(1) << 32)) {
            narrow_rows32<MODE>(g, l, ya, yb, bw, invert);
            return;
        }
    }
    for (int y = ya; y < yb; y += l.grp * kNarrowSteps) {
        NarrowGroup r;
        narrow_load(g, l, ya, yb, y, r);
        narrow_emit<MODE>(g, l, yb, y, r, bw, invert);
    }
}

template <int MODE>
__device__ __forceinline__ void narrow_unit(const Geom& g, int ya, int yb, uint32_t bw,
                                            bool invert) {
    narrow_rows<MODE>(g, narrow_lanes(g, bw), ya, yb, bw, invert);
}

// Vector width actually used for a wide image: the largest v <= vmax whose
// alignment holds (offset and stride in words divisible by v) and whose
// span 64*v does not leave more than half of the wavefront idle.
__host__ __device__ inline int pick_vw(int64_t wd, int vmax, int64_t offset_words,
                                       int64_t stride_words) {
    int v = vmax;
    while (v > 1 && ((offset_words & (v - 1)) != 0 || (stride_words & (v - 1)) != 0 ||
                     wd < 32 * v))
        v /= 2;
    return v;
}

// Words per lane of the strip and tile kernels: as pick_vw, and a divisor
// of the row's word count, so that no lane's words straddle the row's end.
__host__ __device__ inline int strip_vw(int64_t wd, int vmax, int64_t offset_words,
                                        int64_t stride_words) {
    int v = pick_vw(wd, vmax, offset_words, stride_words);
    while (v > 1 && (wd & (v - 1)) != 0) v /= 2;
    return v;
}

// Work units of one image (0 for an empty image). All quotients fit 32 bits
// (height < 2^31, wd < 2^26, band <= 64 * 1024), so they use 32-bit division.
struct UnitShape {
    int narrow;        // 1: narrow units, 0: strips
    int vw;            // strip vector width
    uint32_t chunks;   // word chunks per row (1 for narrow units)
    uint32_t band;     // rows per unit
    int64_t count;     // units
};

__host__ __device__ inline UnitShape unit_shape(int64_t height, int64_t width, int64_t wd,
                                                int64_t offset_words, int64_t stride_words,
                                                int vmax, int rows) {
    UnitShape s{0, 1, 1, 1, 0};
    if (height <= 0 || width <= 0) return s;
    if (wd <= kNarrowMaxWords) {
        s.narrow = 1;
        s.band = (uint32_t)(kWave / wd) * (uint32_t)rows;
    } else {
        s.vw = strip_vw(wd, vmax, offset_words, stride_words);
        const uint32_t span = (uint32_t)kWave * (uint32_t)s.vw;
        s.chunks = ((uint32_t)wd - 1u) / span + 1u;
        s.band = (uint32_t)rows;
    }
    s.count = (int64_t)s.chunks * (int64_t)(((uint32_t)height - 1u) / s.band + 1u);
    return s;
}

}  // namespace edgek
