/* The oracle's C functions on every shape up to 9 x 9 and a few long thin
 * ones, under AddressSanitizer and UndefinedBehaviorSanitizer: inputs and
 * outputs are exact-size heap blocks, so that any access past an image is
 * caught. Also checks E within the black pixels and the bad-argument
 * returns. Prints "oracle ok" and exits 0 on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_edge_image(const uint8_t* img, uint8_t* out, int64_t H, int64_t W, int border_pixel,
                      int clauses, int invert);
int oracle_fundamental_edges(const uint8_t* img, uint8_t* out4, int64_t H, int64_t W,
                             int border_pixel);
int oracle_threshold(const uint8_t* grey, uint8_t* out, int64_t H, int64_t W, int threshold);
int oracle_peel(const uint8_t* img, uint8_t* out, int64_t H, int64_t W, int border_pixel,
                int iterations, int edge_out);
int oracle_edge_stack(const uint8_t* imgs, uint8_t* outs, int64_t n, int64_t H, int64_t W,
                      int border_pixel, int clauses, int invert);

static int failures = 0;
static uint64_t rng = 0x9E3779B97F4A7C15ull;

static unsigned next_bit(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (unsigned)(rng >> 63);
}

static void run_shape(int64_t H, int64_t W) {
    const size_t n = (size_t)(H * W);
    uint8_t* img = (uint8_t*)malloc(n ? n : 1);
    uint8_t* out = (uint8_t*)malloc(n ? n : 1);
    uint8_t* out4 = (uint8_t*)malloc(4 * n ? 4 * n : 1);
    uint8_t* stack_in = (uint8_t*)malloc(3 * n ? 3 * n : 1);
    uint8_t* stack_out = (uint8_t*)malloc(3 * n ? 3 * n : 1);
    for (size_t i = 0; i < n; ++i) img[i] = (uint8_t)next_bit();
    for (size_t i = 0; i < 3 * n; ++i) stack_in[i] = (uint8_t)next_bit();
    for (int border = 0; border <= 1; ++border) {
        for (int clauses = 0; clauses <= 3; ++clauses)
            for (int invert = 0; invert <= 1; ++invert) {
                if (oracle_edge_image(img, out, H, W, border, clauses, invert)) ++failures;
                for (size_t i = 0; i < n && !invert; ++i)
                    if (out[i] && img[i]) ++failures;   /* edge points are black */
            }
        if (oracle_fundamental_edges(img, out4, H, W, border)) ++failures;
        for (int k = 0; k <= 3; ++k)
            for (int edge_out = 0; edge_out <= 1; ++edge_out)
                if (oracle_peel(img, out, H, W, border, k, edge_out)) ++failures;
        if (oracle_edge_stack(stack_in, stack_out, 3, H, W, border, 3, 0)) ++failures;
    }
    const int thresholds[] = {0, 1, 128, 255, 256};
    for (unsigned t = 0; t < sizeof thresholds / sizeof thresholds[0]; ++t)
        if (oracle_threshold(img, out, H, W, thresholds[t])) ++failures;
    free(img);
    free(out);
    free(out4);
    free(stack_in);
    free(stack_out);
}

int main(void) {
    for (int64_t H = 0; H <= 9; ++H)
        for (int64_t W = 0; W <= 9; ++W) run_shape(H, W);
    run_shape(1, 1000);
    run_shape(1000, 1);
    run_shape(37, 129);
    /* bad arguments return -1 without touching memory */
    uint8_t b[4] = {0, 1, 0, 1};
    if (oracle_edge_image(b, b, -1, 2, 1, 1, 0) != -1) ++failures;
    if (oracle_edge_image(b, b, 2, 2, 2, 1, 0) != -1) ++failures;
    if (oracle_edge_image(b, b, 2, 2, 1, 4, 0) != -1) ++failures;
    if (oracle_edge_image(NULL, b, 2, 2, 1, 1, 0) != -1) ++failures;
    if (oracle_threshold(b, b, 2, 2, 257) != -1) ++failures;
    if (oracle_peel(b, b, 2, 2, 1, -1, 0) != -1) ++failures;
    if (oracle_edge_stack(b, b, -1, 2, 2, 1, 1, 0) != -1) ++failures;
    if (failures) {
        printf("FAIL: %d\n", failures);
        return 1;
    }
    printf("oracle ok\n");
    return 0;
}
