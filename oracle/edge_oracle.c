/*
 * edge_oracle.c - CPU oracle for edge detection of binary images
 * (Sadeq, Wahdan, Mahdi, "Edge Detection of Binary Images Using the Method
 * of Masks", Sci. Bull. Fac. Eng. Ain Shams Univ. 35(3), 2000).
 *
 * TEST INFRASTRUCTURE. This file is the slow, obviously correct reference
 * that the GPU library is checked against. Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg load it. It includes no header of the
 * GPU library and shares no code, table or helper with it.
 *
 * What it is: the "traditional scanning algorithm" of section 1 - visit every
 * pixel, evaluate the edge predicate, write the answer - on a byte-per-pixel
 * image. It does no bit packing and no word tricks.
 *
 * Conventions:
 *   - A pixel byte of 0 is black, any other value is white (section 2: the
 *     colour bit of a monochrome image is 0 for black and 1 for white).
 *   - Neighbours are numbered as in Fig. 1 (see DY/DX below).
 *   - A neighbour outside the image takes the value `border_pixel`
 *     (1 = white, 0 = black). The paper does not say what lies outside the
 *     image; the caller chooses.
 *   - Output byte 1 = edge point, 0 = not (the value of Edge(p) in the
 *     Boolean function of section 1). With `invert` set the byte is flipped,
 *     which is the display polarity of section 5, where the ORed edges are
 *     inverted so that edges show black.
 *
 * Clauses (definition of a binary edge point, section 1):
 *   ORACLE_CLAUSE1: a black point with at least one white 4-neighbour
 *                   (neighbours 2, 4, 6 and 8 of Fig. 1).
 *   ORACLE_CLAUSE2: a black point with at most one black 8-neighbour
 *                   (any of the eight neighbours of Fig. 1).
 * A pixel is an edge point when it satisfies any selected clause.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

#define ORACLE_CLAUSE1 1
#define ORACLE_CLAUSE2 2

/* Fig. 1: neighbour k of P (k = 1..8; entry 0 unused) sits at row offset
 * DY[k] and column offset DX[k]. Rows grow downwards, columns rightwards.
 * The figure lays the neighbours out as
 *        3 2 1
 *        4 P 8
 *        5 6 7
 */
static const int DY[9] = {0, -1, -1, -1, 0, +1, +1, +1, 0};
static const int DX[9] = {0, +1, 0, -1, -1, -1, 0, +1, +1};

/* The four 4-neighbours named in the Boolean function Edge(p) of section 1. */
static const int FOUR_NEIGHBOURS[4] = {2, 4, 6, 8};

/* Colour of pixel (y, x): 1 = white, 0 = black; outside -> border_pixel. */
static int pixel(const uint8_t* img, int64_t H, int64_t W, int64_t y, int64_t x,
                 int border_pixel) {
    if (y < 0 || y >= H || x < 0 || x >= W) return border_pixel;
    return img[y * W + x] != 0;
}

/* Edge map of one H x W image (row-major bytes). Returns 0, or -1 on bad
 * arguments (negative size, unknown clause bits, null pointer with pixels). */
int oracle_edge_image(const uint8_t* img, uint8_t* out, int64_t H, int64_t W,
                      int border_pixel, int clauses, int invert) {
    if (H < 0 || W < 0) return -1;
    if (clauses & ~(ORACLE_CLAUSE1 | ORACLE_CLAUSE2)) return -1;
    if (border_pixel != 0 && border_pixel != 1) return -1;
    if (H * W > 0 && (img == NULL || out == NULL)) return -1;

    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            int p = pixel(img, H, W, y, x, border_pixel);
            int edge = 0;
            if (p == 0) { /* only a black point can be an edge point */
                if (clauses & ORACLE_CLAUSE1) {
                    int white_4 = 0;
                    for (int i = 0; i < 4; ++i) {
                        int k = FOUR_NEIGHBOURS[i];
                        if (pixel(img, H, W, y + DY[k], x + DX[k], border_pixel) == 1)
                            white_4 = 1;
                    }
                    if (white_4) edge = 1;
                }
                if (clauses & ORACLE_CLAUSE2) {
                    int black_8 = 0;
                    for (int k = 1; k <= 8; ++k)
                        if (pixel(img, H, W, y + DY[k], x + DX[k], border_pixel) == 0)
                            ++black_8;
                    if (black_8 <= 1) edge = 1;
                }
            }
            out[y * W + x] = (uint8_t)(invert ? !edge : edge);
        }
    }
    return 0;
}

/* The four fundamental edges of section 4, as four byte planes of H x W
 * in the order the section names them: left, right, up, down. The left
 * edge is the image shifted right by one pixel ANDed with the mask (the
 * negative image, section 3): a black point whose left neighbour (n4 of
 * Fig. 1) is white. Likewise right uses n8, up uses n2 and down uses n6;
 * these are the four types of Fig. 2. */
int oracle_fundamental_edges(const uint8_t* img, uint8_t* out4, int64_t H, int64_t W,
                             int border_pixel) {
    static const int DIRECTION_NEIGHBOUR[4] = {4, 8, 2, 6};   /* left, right, up, down */
    if (H < 0 || W < 0) return -1;
    if (border_pixel != 0 && border_pixel != 1) return -1;
    if (H * W > 0 && (img == NULL || out4 == NULL)) return -1;
    for (int plane = 0; plane < 4; ++plane) {
        const int k = DIRECTION_NEIGHBOUR[plane];
        uint8_t* out = out4 + (int64_t)plane * H * W;
        for (int64_t y = 0; y < H; ++y)
            for (int64_t x = 0; x < W; ++x) {
                const int mask = 1 - pixel(img, H, W, y, x, border_pixel);   /* section 3 */
                const int shifted = pixel(img, H, W, y + DY[k], x + DX[k], border_pixel);
                out[y * W + x] = (uint8_t)(mask & shifted);
            }
    }
    return 0;
}

/* Binarisation of a grey image by a threshold (section 7: non-binary images
 * are first converted to binary by thresholding). A grey value >= threshold
 * becomes white (1), a smaller one black (0), so dark strokes stay black.
 * threshold 0 makes every pixel white, 256 every pixel black. */
int oracle_threshold(const uint8_t* grey, uint8_t* out, int64_t H, int64_t W, int threshold) {
    if (H < 0 || W < 0 || threshold < 0 || threshold > 256) return -1;
    if (H * W > 0 && (grey == NULL || out == NULL)) return -1;
    for (int64_t i = 0; i < H * W; ++i) out[i] = (uint8_t)(grey[i] >= threshold ? 1 : 0);
    return 0;
}

/* Iterated peeling of the edge, the step that thinning repeats (section 1
 * names edge detection as part of thinning): `iterations` times, find the
 * edge points of the current image (clause 1, the Boolean function Edge(p))
 * and make them white. Pixels outside the image keep the border colour at
 * every step. out receives the image after the last peel or, with
 * `edge_out` set, the edge map of that image (the next layer to be peeled).
 * Returns 0, or -1 on bad arguments or when scratch memory is unavailable. */
int oracle_peel(const uint8_t* img, uint8_t* out, int64_t H, int64_t W, int border_pixel,
                int iterations, int edge_out) {
    if (H < 0 || W < 0 || iterations < 0) return -1;
    if (border_pixel != 0 && border_pixel != 1) return -1;
    if (H * W == 0) return 0;
    if (img == NULL || out == NULL) return -1;
    uint8_t* cur = (uint8_t*)malloc((size_t)(H * W));
    uint8_t* edge = (uint8_t*)malloc((size_t)(H * W));
    if (cur == NULL || edge == NULL) {
        free(cur);
        free(edge);
        return -1;
    }
    for (int64_t i = 0; i < H * W; ++i) cur[i] = img[i] != 0;
    for (int t = 0; t < iterations; ++t) {
        oracle_edge_image(cur, edge, H, W, border_pixel, ORACLE_CLAUSE1, 0);
        for (int64_t i = 0; i < H * W; ++i)
            if (edge[i]) cur[i] = 1;          /* an edge point is peeled: it turns white */
    }
    if (edge_out) oracle_edge_image(cur, out, H, W, border_pixel, ORACLE_CLAUSE1, 0);
    else
        for (int64_t i = 0; i < H * W; ++i) out[i] = cur[i];
    free(cur);
    free(edge);
    return 0;
}

/* The same for n images of equal shape stored one after another. */
int oracle_edge_stack(const uint8_t* imgs, uint8_t* outs, int64_t n, int64_t H,
                      int64_t W, int border_pixel, int clauses, int invert) {
    if (n < 0) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int rc = oracle_edge_image(imgs + i * H * W, outs + i * H * W, H, W,
                                   border_pixel, clauses, invert);
        if (rc) return rc;
    }
    return 0;
}
