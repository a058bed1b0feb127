/*
 * edge_masks.h - C ABI of libedgemask, a gfx950 (MI355X) library for edge
 * detection of binary images by the method of masks (Sadeq, Wahdan, Mahdi,
 * "Edge Detection of Binary Images Using the Method of Masks", 2000).
 *
 * WHAT IS COMPUTED
 *   An image is a monochrome bit-stream, one bit per pixel, 0 = black and
 *   1 = white (paper, section 2). A pixel p is an edge point when
 *       Edge(p) = (NOT p) AND (n2 OR n4 OR n6 OR n8)
 *   (Boolean function of section 1), with n2, n4, n6, n8 the up, left, down
 *   and right neighbours of the numbering of Fig. 1:
 *        n3 n2 n1
 *        n4  P n8
 *        n5 n6 n7
 *   The paper gets there in three stages: the mask is the negative image
 *   (section 3); each of the four fundamental edges is the image shifted by
 *   one pixel in one direction ANDed with the mask (section 4); the edge is
 *   the OR of the four (section 5). The library fuses the three stages into
 *   one pass over the packed words: by distributivity the OR of the four
 *   masked shifts equals the mask ANDed with the OR of the four shifts.
 *
 *   The full definition of section 1 also counts as an edge point a black
 *   pixel with at most one black 8-neighbour ("full mode"). Such a pixel
 *   always has at least three white 4-neighbours, so the full-mode output
 *   equals the plain output bit for bit; EDGE_FLAG_CLAUSE2_ONLY exposes the
 *   second clause on its own.
 *
 * PACKED LAYOUT (every entry point)
 *   Rows of B-bit words, B = word_bits = 32 or 64, little-endian, LSB first:
 *   pixel (x, y) is bit (x mod B) of word (y * stride_words + x / B).
 *   A row has Wd = ceil(width / B) valid words; stride_words >= Wd.
 *   - Input bits at x >= width inside the valid words are ignored.
 *   - Output bits at x >= width inside the valid words are written as 0.
 *   - Stride words Wd .. stride_words-1 are neither read nor written.
 *   The byte layout of a row is the same for B = 32 and B = 64.
 *
 * OUTSIDE THE IMAGE
 *   The paper does not say what a shifted block brings in at the frame.
 *   `border` chooses: EDGE_BORDER_WHITE (default; out-of-image pixels are
 *   white, so black pixels on the frame are edge points) or
 *   EDGE_BORDER_BLACK. Both clauses use the same convention.
 *
 * CALLING RULES
 *   - All device pointers are caller-owned device memory. The library
 *     allocates no device memory; graph handles are the only objects it owns.
 *     (edge_batch_noalloc's workspace is a fixed array inside the library's
 *     code object, one per GPU, that exists once the library is loaded.)
 *   - Every call is asynchronous on `hip_stream` (a hipStream_t; NULL = the
 *     null stream) and returns once the work is enqueued. Inputs must stay
 *     valid and unmodified until the stream reaches the work.
 *   - Argument errors are returned before any HIP call is made.
 *   - height == 0 or width == 0 is a no-op returning EDGE_OK. Heights above
 *     EDGE_MAX_HEIGHT and widths above 2^31 - 1 pixels are rejected.
 *   - In-place operation is not supported: overlapping input and output
 *     byte ranges return EDGE_ERR_ALIAS.
 *   - Pointers must be aligned to B/8 bytes (EDGE_ERR_ALIGN otherwise).
 *     16-byte alignment of the pointers and of the row pitch enables 128-bit
 *     loads and stores.
 *   - Functions are reentrant and keep no mutable global state apart from a
 *     per-device compute-unit count and a per-device address of the
 *     edge_batch_noalloc workspace, each cached on first use.
 */
#ifndef EDGE_MASKS_H
#define EDGE_MASKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EDGE_MASKS_ABI_VERSION 2

/* Largest image height (rows) any entry point accepts. */
#define EDGE_MAX_HEIGHT (1 << 30)

/* Status codes returned by every int-returning entry point. */
enum {
    EDGE_OK = 0,
    EDGE_ERR_INVALID = -1,     /* bad size, stride, enum, flag or descriptor */
    EDGE_ERR_ALIGN = -2,       /* pointer not aligned to the word size */
    EDGE_ERR_ALIAS = -3,       /* input and output byte ranges overlap */
    EDGE_ERR_HIP = -4,         /* a HIP call failed; see edge_last_hip_error() */
    EDGE_ERR_WORKSPACE = -5,   /* workspace missing, too small or misaligned */
    EDGE_ERR_UNSUPPORTED = -6  /* launch configuration outside what is built */
};

/* Colour of pixels outside the image. */
enum { EDGE_BORDER_WHITE = 0, EDGE_BORDER_BLACK = 1 };

/* Which definition of section 1: clause 1 only, or clause 1 OR clause 2. */
enum { EDGE_MODE_MASKS = 0, EDGE_MODE_FULL = 1 };

/* Flags. CLAUSE2_ONLY (full mode only): output the black pixels with at
 * most one black 8-neighbour, without clause 1. INVERT_OUT: the display
 * polarity of section 5 (edge pixels 0, others 1); padding bits stay 0.
 * PLANNED (batch calls only): the workspace already holds the plan that
 * edge_batch_plan made for this table, arenas, word size and cfg, so the
 * device planner is skipped. PEEL_EDGE (edge_peel only): output the edge
 * map of the peeled image. */
enum { EDGE_FLAG_CLAUSE2_ONLY = 1u << 0, EDGE_FLAG_INVERT_OUT = 1u << 1,
       EDGE_FLAG_PLANNED = 1u << 2, EDGE_FLAG_PEEL_EDGE = 1u << 3 };

/* Most peels edge_peel does in one call. */
#define EDGE_PEEL_MAX_ITERATIONS 30

/* One image of a batch. Offsets and strides count B-bit words from the
 * start of the arena; in and out arenas share the same descriptors. */
typedef struct edge_image_desc {
    int64_t offset_words;
    int32_t height;
    int32_t width;
    int64_t stride_words;
} edge_image_desc;

/* Launch configuration (NULL selects the built-in choice).
 *   vec_words       32-bit words per lane for wide rows: 1, 2 or 4.
 *   rows_per_tile   rows one wavefront walks down per work unit, 1..1024
 *                   (1..EDGE_TILE_MAX_ROWS for tiles; for bands, the rows
 *                   each wavefront loads: 1, 2 or 4, with
 *                   waves_per_block * rows_per_tile >= 3).
 *   waves_per_block wavefronts per workgroup: 1, 2, 4 or 8.
 *   blocks_per_cu   persistent workgroups per compute unit (batch only),
 *                   1..32; ignored by the single-image calls.
 *   cache_policy    EDGE_CACHE_AUTO (by image size), EDGE_CACHE_NORMAL or
 *                   EDGE_CACHE_STREAM (non-temporal loads and stores);
 *                   single images only, batches use EDGE_CACHE_NORMAL;
 *                   edge_threshold_edges reads AUTO as cached loads with
 *                   non-temporal stores.
 *   shape           how a single image's rows of more than 32 words are
 *                   cut into work: EDGE_SHAPE_STRIP (a wavefront walks its
 *                   rows with a few rows in flight), EDGE_SHAPE_TILE (a
 *                   wavefront requests all rows of its unit at once, always
 *                   with non-temporal loads and stores; cache_policy is not
 *                   used; workgroups in dispatch order) or
 *                   EDGE_SHAPE_TILE_XCD (the same tiles, workgroups
 *                   regrouped so that each XCD takes a contiguous part of
 *                   the image, as strips always are), or EDGE_SHAPE_BAND /
 *                   EDGE_SHAPE_BAND_XCD (a workgroup loads
 *                   waves_per_block * rows_per_tile consecutive rows of one
 *                   chunk into LDS at once and computes all but the first
 *                   and last; non-temporal loads and stores). Used by the
 *                   edge-map calls and edge_directions; ignored by batches,
 *                   by rows of at most 32 words and by the grey-input and
 *                   peeling calls. */
typedef struct edge_launch_cfg {
    int32_t vec_words;
    int32_t rows_per_tile;
    int32_t waves_per_block;
    int32_t blocks_per_cu;
    int32_t cache_policy;
    int32_t shape;
} edge_launch_cfg;

enum { EDGE_CACHE_AUTO = 0, EDGE_CACHE_NORMAL = 1, EDGE_CACHE_STREAM = 2 };
enum { EDGE_SHAPE_STRIP = 0, EDGE_SHAPE_TILE = 1, EDGE_SHAPE_TILE_XCD = 2, EDGE_SHAPE_BAND = 3,
       EDGE_SHAPE_BAND_XCD = 4 };

/* Most rows of one EDGE_SHAPE_TILE work unit. */
#define EDGE_TILE_MAX_ROWS 16

/* Plain method (Boolean function Edge(p), section 1; stages of sections
 * 3-5). `in`, `out`: device pointers to height rows of stride_words words.
 * Returns EDGE_OK or an error status. */
int edge_masks(const void* in, void* out, int64_t height, int64_t width,
               int64_t stride_words, int word_bits, int border, void* hip_stream);

/* Full definition of an edge point (section 1, both clauses). `flags` may
 * hold EDGE_FLAG_CLAUSE2_ONLY and EDGE_FLAG_INVERT_OUT. */
int edge_full(const void* in, void* out, int64_t height, int64_t width,
              int64_t stride_words, int word_bits, int border, uint32_t flags,
              void* hip_stream);

/* Single image with an explicit mode, flags and launch configuration
 * (cfg == NULL: built-in choice). Same computation as edge_masks /
 * edge_full; used by the autotuner to time candidate configurations.
 * EDGE_FLAG_CLAUSE2_ONLY requires mode == EDGE_MODE_FULL. */
int edge_image_launch(const void* in, void* out, int64_t height, int64_t width,
                      int64_t stride_words, int word_bits, int border, int mode,
                      uint32_t flags, const edge_launch_cfg* cfg, void* hip_stream);

/* The four fundamental edges of section 4 - the edge types of Fig. 2 -
 * as four planes: out4 + 0, 1, 2, 3 x plane_words hold the left, right, up
 * and down edges (the mask ANDed with the image shifted right, left, down
 * and up by one pixel: black pixels whose n4, n8, n2 or n6 neighbour is
 * white). Their OR is edge_masks's output. Each plane has the input's
 * layout; plane_words >= (height - 1) * stride_words + ceil(width / B).
 * cfg: NULL or as for edge_image_launch. */
int edge_directions(const void* in, void* out4, int64_t plane_words, int64_t height,
                    int64_t width, int64_t stride_words, int word_bits, int border,
                    const edge_launch_cfg* cfg, void* hip_stream);

/* Binarisation by a threshold (section 7: a non-binary image is made
 * binary first) and packing. grey: device bytes, height rows of
 * grey_stride_bytes (>= width) bytes. A grey value >= threshold becomes white
 * (1), a smaller one black (0); threshold 0..256 (0: all white, 256: all
 * black). out: packed rows in the layout above (stride_words words of
 * word_bits), bits past the width written 0, stride words untouched.
 * Any pointer and pitch: bytes load in the 16-byte aligned blocks that hold
 * them (two per 32 pixels where rows start on 16-byte boundaries, three
 * otherwise); a block can reach up to 15 bytes before a row's first byte
 * or after its last, never outside the memory pages of the row. Packed
 * output of 16 MiB or more (height x row words) is stored non-temporally. */
int edge_threshold_pack(const void* grey, int64_t grey_stride_bytes, int threshold, void* out,
                        int64_t height, int64_t width, int64_t stride_words, int word_bits,
                        void* hip_stream);

/* Threshold and edges in one pass: the grey image of edge_threshold_pack
 * is binarised in registers and its edge map (mode, flags and border as
 * for edge_image_launch) written in the packed layout; the binary image is
 * never stored. Equals edge_threshold_pack followed by edge_image_launch.
 * Grey bytes load as for edge_threshold_pack. The image runs as bands of
 * 2048-pixel chunks: a workgroup of waves_per_block wavefronts loads
 * waves_per_block x r rows of a chunk at once (r = rows_per_tile rounded
 * down to 2, 4 or 8, raised until a band loads four rows) and writes the
 * rows between the first and the last. cfg: NULL for the built-in shape
 * (8 wavefronts, r = 2, cache_policy AUTO), or a configuration; vec_words
 * and blocks_per_cu are ignored; cache_policy AUTO keeps the loads cached
 * and makes the stores non-temporal, NORMAL keeps both cached, STREAM makes
 * both non-temporal. */
int edge_threshold_edges(const void* grey, int64_t grey_stride_bytes, int threshold, void* out,
                         int64_t height, int64_t width, int64_t stride_words, int word_bits,
                         int border, int mode, uint32_t flags, const edge_launch_cfg* cfg,
                         void* hip_stream);

/* The paper's three stages as separate whole-image passes, the unfused
 * form of edge_masks kept as an ablation: mask = negative image
 * (section 3); four fundamental edges = mask AND the image shifted by one
 * pixel (section 4); three ORs into the left edge (section 5; the display
 * inversion is left out). Eight launches, about 23 image-sized transfers
 * against 2 for the fused kernel. Same output as edge_masks.
 * scratch: device buffer of >= 4 * height * stride_words * word_bits / 8
 * bytes (mask and three edge planes), 4-byte aligned, disjoint from in and
 * out. */
int edge_masks_staged(const void* in, void* out, void* scratch, int64_t scratch_bytes,
                      int64_t height, int64_t width, int64_t stride_words, int word_bits,
                      int border, void* hip_stream);

/* Iterated peeling of the edge: `iterations` times, every edge point of
 * the current image (Edge(p) of section 1) turns white, pixels outside the
 * image keeping the border colour; thinning repeats this step (section 1).
 * A black pixel is left after k peels exactly when no white pixel (nor,
 * under the white border, the outside) lies within taxicab distance k of it.
 * out receives the peeled image, or with EDGE_FLAG_PEEL_EDGE its edge map
 * (the pixels the next peel would remove; iterations = 0 then gives the
 * output of edge_masks). Layout, padding and alias rules as edge_masks;
 * 0 <= iterations <= EDGE_PEEL_MAX_ITERATIONS, all done in one pass over
 * the image. cfg: NULL, or a configuration. With two or more levels
 * (iterations, plus one with EDGE_FLAG_PEEL_EDGE) its rows_per_tile and
 * waves_per_block are used, and with two to seven levels also vec_words
 * (words per lane, narrowed as the pointers and stride require; the
 * built-in shape takes four words per lane for two or three levels, and for
 * four to seven on images of 2^30 pixels or more); loads
 * always go through the caches, and from 16 levels each strip takes one
 * workgroup of two wavefronts. One level or none runs the strip loop of
 * edge_image_launch, which reads every field as that call does. */
int edge_peel(const void* in, void* out, int64_t height, int64_t width, int64_t stride_words,
              int word_bits, int border, int iterations, uint32_t flags,
              const edge_launch_cfg* cfg, void* hip_stream);

/* Built-in launch configuration for an image shape (batch != 0: for the
 * persistent batch kernel). Returns EDGE_OK and fills *cfg_out. */
int edge_default_cfg(int64_t height, int64_t width, int word_bits, int mode,
                     int batch, edge_launch_cfg* cfg_out);

/* Bytes of device workspace edge_batch needs for n_images descriptors.
 * Returns a negative status for n_images < 0. */
int64_t edge_batch_workspace_bytes(int32_t n_images);

/* Host-side check of a descriptor table (host memory) against arenas of
 * arena_words words: sizes >= 0, height <= EDGE_MAX_HEIGHT, stride >= Wd,
 * every image inside the arena. Returns EDGE_OK or EDGE_ERR_INVALID. */
int edge_batch_check(const edge_image_desc* table_host, int32_t n_images,
                     int64_t arena_words, int word_bits);

/* Host-side work plan for a batch: writes into plan_host (>=
 * edge_batch_workspace_bytes(n_images) bytes, 8-byte aligned, host memory)
 * the plan the device planner would write for table_host, and the number
 * of leading bytes that matter in *plan_used_bytes. The caller copies those
 * bytes into the device workspace and calls edge_batch with
 * EDGE_FLAG_PLANNED. in_arena/out_arena are the device arenas (only their
 * alignment is read) and cfg must equal the one given to edge_batch.
 * Returns EDGE_ERR_INVALID when a descriptor fails edge_batch_check. Makes
 * one HIP query (the compute-unit count, cached). The batch kernel checks
 * the plan's header and every unit against its image, so a plan that does
 * not belong to the table gives wrong output but no access outside valid
 * images of the arenas. */
int edge_batch_plan(const void* in_arena, const void* out_arena, int64_t arena_words,
                    const edge_image_desc* table_host, int32_t n_images, int word_bits,
                    const edge_launch_cfg* cfg, void* plan_host, int64_t plan_bytes,
                    int64_t* plan_used_bytes);

/* Many independent images in one persistent launch (each image as in
 * edge_masks / edge_full; no bits cross between images).
 *   in_arena, out_arena: device arenas of arena_words B-bit words each.
 *   table_dev: device array of n_images descriptors (read by the device
 *     when the stream reaches the work, so it may be rewritten in place
 *     between graph replays).
 *   workspace_dev: device scratch of >= edge_batch_workspace_bytes(n)
 *     bytes, 256-byte aligned, owned by the caller; overwritten each call.
 *   mode, flags: as edge_image_launch. cfg: NULL = built-in choice.
 * A descriptor that fails the checks of edge_batch_check is skipped on the
 * device (its output untouched) and flagged in the workspace; callers
 * should run edge_batch_check on the host copy first. Two calls that share
 * a workspace must not overlap in time. */
int edge_batch(const void* in_arena, void* out_arena, int64_t arena_words,
               const edge_image_desc* table_dev, int32_t n_images, int word_bits,
               int border, int mode, uint32_t flags, const edge_launch_cfg* cfg,
               void* workspace_dev, int64_t workspace_bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): edge_batch
 * with the workspace held by the library. The work plan goes into a fixed
 * device array in the library's code object, 256-byte aligned, one per GPU
 * (about 5.3 MiB each, held until the process ends), sized for at most
 * EDGE_BATCH_NOALLOC_MAX_IMAGES images; its device address is looked up
 * once per GPU, on the first call with that GPU current.
 *   Arguments as edge_batch, without the workspace. The current device must
 *   be the one the arenas, the table and hip_stream belong to.
 *   n_images > EDGE_BATCH_NOALLOC_MAX_IMAGES returns EDGE_ERR_WORKSPACE,
 *   and EDGE_FLAG_PLANNED returns EDGE_ERR_INVALID (there is no way to put
 *   a host plan into the array without a copy), both before any HIP call.
 *   Allocates nothing: no hipMalloc, hipFree or allocating library call.
 *   Every call on a GPU shares that GPU's array: the device planner
 *   rewrites every word the kernel reads on each call, so nothing has to be
 *   cleared between calls, but calls that overlap in time on one GPU (other
 *   streams, other threads) race on the plan and give wrong output; order
 *   them on one stream or with events. */
#define EDGE_BATCH_NOALLOC_MAX_IMAGES 16384
int edge_batch_noalloc(const void* in_arena, void* out_arena, int64_t arena_words,
                       const edge_image_desc* table_dev, int32_t n_images, int word_bits,
                       int border, int mode, uint32_t flags, const edge_launch_cfg* cfg,
                       void* hip_stream);

/* Capture the work of one edge_batch call (same arguments) into an
 * instantiated HIP graph. *graph_out receives an opaque handle. */
int edge_batch_graph_create(const void* in_arena, void* out_arena, int64_t arena_words,
                            const edge_image_desc* table_dev, int32_t n_images,
                            int word_bits, int border, int mode, uint32_t flags,
                            const edge_launch_cfg* cfg, void* workspace_dev,
                            int64_t workspace_bytes, void** graph_out);

/* Replay a captured batch on `hip_stream`. */
int edge_graph_launch(void* graph, void* hip_stream);

/* Free a graph handle (NULL is a no-op). */
int edge_graph_destroy(void* graph);

/* Plain device copy of n_bytes (multiple of 16, 16-byte aligned pointers,
 * no overlap): the bandwidth ceiling that the edge kernels are compared to. */
int edge_copy_bytes(const void* in, void* out, int64_t n_bytes, void* hip_stream);

/* Text for a status code (static storage). */
const char* edge_status_string(int status);

/* hipError_t of the last EDGE_ERR_HIP on the calling thread (0 if none). */
int edge_last_hip_error(void);

/* EDGE_MASKS_ABI_VERSION of the built library. */
int edge_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EDGE_MASKS_H */
