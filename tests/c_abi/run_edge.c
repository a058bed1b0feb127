/* The library driven from plain C: device memory from the HIP runtime's C
 * API, no Python and no PyTorch. Each case runs an entry point on a seeded
 * random image (or a batch of them) and compares every pixel with the
 * oracle's C functions (this program is test infrastructure, so it may call
 * both). Prints one line per case; exits 0 when every case matches. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "edge_masks.h"

/* oracle/edge_oracle.c */
int oracle_edge_image(const uint8_t* img, uint8_t* out, int64_t H, int64_t W, int border_pixel,
                      int clauses, int invert);
int oracle_peel(const uint8_t* img, uint8_t* out, int64_t H, int64_t W, int border_pixel,
                int iterations, int edge_out);
int oracle_threshold(const uint8_t* grey, uint8_t* out, int64_t H, int64_t W, int threshold);

static uint64_t rng_state;

static uint64_t next_u64(void) { /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

#define HIP_OK(x)                                                             \
    do {                                                                      \
        hipError_t e_ = (x);                                                  \
        if (e_ != hipSuccess) {                                               \
            printf("HIP error %d at line %d\n", (int)e_, __LINE__);          \
            return 0;                                                         \
        }                                                                     \
    } while (0)

enum { KIND_MASKS, KIND_FULL, KIND_PEEL };

/* One case: returns 1 when the device output equals the oracle's. */
static int run_case(int64_t H, int64_t W, int border, int kind, uint64_t seed) {
    const int64_t wd = (W + 63) / 64, S = wd + 1, n = H * S;
    const uint64_t sentinel = 0xA5A5A5A5A5A5A5A5ull;
    uint64_t* words = malloc((size_t)n * 8);
    uint64_t* back = malloc((size_t)n * 8);
    uint8_t* img = malloc((size_t)(H * W));
    uint8_t* want = malloc((size_t)(H * W));
    void *din = NULL, *dout = NULL;
    int ok = 1, rc = EDGE_OK;
    int64_t y, x;
    rng_state = seed;
    for (int64_t i = 0; i < n; ++i) words[i] = next_u64() & next_u64(); /* ~25% white */
    for (y = 0; y < H; ++y)
        for (x = 0; x < W; ++x) img[y * W + x] = (uint8_t)((words[y * S + x / 64] >> (x % 64)) & 1);
    HIP_OK(hipMalloc(&din, (size_t)n * 8));
    HIP_OK(hipMalloc(&dout, (size_t)n * 8));
    HIP_OK(hipMemcpy(din, words, (size_t)n * 8, hipMemcpyHostToDevice));
    HIP_OK(hipMemset(dout, 0xA5, (size_t)n * 8));
    if (kind == KIND_MASKS) {
        rc = edge_masks(din, dout, H, W, S, 64, border, NULL);
        oracle_edge_image(img, want, H, W, border == EDGE_BORDER_WHITE, 1, 0);
    } else if (kind == KIND_FULL) {
        rc = edge_full(din, dout, H, W, S, 64, border, 0u, NULL);
        oracle_edge_image(img, want, H, W, border == EDGE_BORDER_WHITE, 3, 0);
    } else {
        rc = edge_peel(din, dout, H, W, S, 64, border, 3, 0u, NULL, NULL);
        oracle_peel(img, want, H, W, border == EDGE_BORDER_WHITE, 3, 0);
    }
    if (rc != EDGE_OK) {
        printf("entry point returned %d (%s)\n", rc, edge_status_string(rc));
        ok = 0;
    }
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(back, dout, (size_t)n * 8, hipMemcpyDeviceToHost));
    for (y = 0; y < H && ok; ++y) {
        for (x = 0; x < W; ++x)
            if ((uint8_t)((back[y * S + x / 64] >> (x % 64)) & 1) != want[y * W + x]) {
                printf("pixel (%lld, %lld) differs\n", (long long)y, (long long)x);
                ok = 0;
                break;
            }
        if (ok && W % 64 && (back[y * S + wd - 1] >> (W % 64)) != 0) {
            printf("row %lld: pad bits not zero\n", (long long)y);
            ok = 0;
        }
        if (ok && back[y * S + wd] != sentinel) {
            printf("row %lld: stride word written\n", (long long)y);
            ok = 0;
        }
    }
    /* in place is refused before any HIP call */
    if (ok && edge_masks(din, din, H, W, S, 64, border, NULL) != EDGE_ERR_ALIAS) ok = 0;
    HIP_OK(hipFree(din));
    HIP_OK(hipFree(dout));
    free(words);
    free(back);
    free(img);
    free(want);
    printf("%s %lld x %lld border %d kind %d\n", ok ? "match" : "MISMATCH", (long long)H,
           (long long)W, border, kind);
    return ok;
}

/* One batch of uneven images (32-bit words) in one arena, run with the
 * device planner and again with the host plan (EDGE_FLAG_PLANNED); every
 * image compared with the oracle. Returns 1 when both runs match. */
static int run_batch_case(int border, uint64_t seed) {
    enum { N = 24 };
    edge_image_desc tab[N];
    int64_t off = 0, i, y, x;
    int ok = 1, pass;
    rng_state = seed;
    for (i = 0; i < N; ++i) {
        const int64_t h = 1 + (int64_t)(next_u64() % 150), w = 1 + (int64_t)(next_u64() % 600);
        const int64_t s = (w + 31) / 32 + (int64_t)(next_u64() % 3);
        off = (off + 3) / 4 * 4; /* 16-byte aligned images */
        tab[i].offset_words = off;
        tab[i].height = (int32_t)h;
        tab[i].width = (int32_t)w;
        tab[i].stride_words = s;
        off += h * s;
    }
    const int64_t words = (off + 3) / 4 * 4;
    uint32_t* arena = malloc((size_t)words * 4);
    uint32_t* back = malloc((size_t)words * 4);
    const int64_t ws_bytes = edge_batch_workspace_bytes(N);
    void* plan = malloc((size_t)ws_bytes);
    void *din = NULL, *dout = NULL, *dtab = NULL, *dws = NULL;
    int64_t used = 0;
    for (i = 0; i < words; ++i) arena[i] = (uint32_t)(next_u64() & next_u64());
    if (edge_batch_check(tab, N, words, 32) != EDGE_OK) {
        printf("batch table rejected\n");
        return 0;
    }
    HIP_OK(hipMalloc(&din, (size_t)words * 4));
    HIP_OK(hipMalloc(&dout, (size_t)words * 4));
    HIP_OK(hipMalloc(&dtab, sizeof(tab)));
    HIP_OK(hipMalloc(&dws, (size_t)ws_bytes));
    HIP_OK(hipMemcpy(din, arena, (size_t)words * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dtab, tab, sizeof(tab), hipMemcpyHostToDevice));
    for (pass = 0; pass < 2 && ok; ++pass) {
        int rc;
        uint32_t flags = 0u;
        HIP_OK(hipMemset(dout, 0, (size_t)words * 4));
        if (pass == 1) {
            rc = edge_batch_plan(din, dout, words, tab, N, 32, NULL, plan, ws_bytes, &used);
            if (rc != EDGE_OK) {
                printf("edge_batch_plan returned %d (%s)\n", rc, edge_status_string(rc));
                ok = 0;
                break;
            }
            HIP_OK(hipMemcpy(dws, plan, (size_t)used, hipMemcpyHostToDevice));
            flags = EDGE_FLAG_PLANNED;
        }
        rc = edge_batch(din, dout, words, (const edge_image_desc*)dtab, N, 32, border,
                        EDGE_MODE_MASKS, flags, NULL, dws, ws_bytes, NULL);
        if (rc != EDGE_OK) {
            printf("edge_batch returned %d (%s)\n", rc, edge_status_string(rc));
            ok = 0;
            break;
        }
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipMemcpy(back, dout, (size_t)words * 4, hipMemcpyDeviceToHost));
        for (i = 0; i < N && ok; ++i) {
            const int64_t h = tab[i].height, w = tab[i].width, s = tab[i].stride_words;
            const uint32_t* in = arena + tab[i].offset_words;
            const uint32_t* got = back + tab[i].offset_words;
            uint8_t* img = malloc((size_t)(h * w));
            uint8_t* want = malloc((size_t)(h * w));
            for (y = 0; y < h; ++y)
                for (x = 0; x < w; ++x) img[y * w + x] = (uint8_t)((in[y * s + x / 32] >> (x % 32)) & 1);
            oracle_edge_image(img, want, h, w, border == EDGE_BORDER_WHITE, 1, 0);
            for (y = 0; y < h && ok; ++y)
                for (x = 0; x < w; ++x)
                    if ((uint8_t)((got[y * s + x / 32] >> (x % 32)) & 1) != want[y * w + x]) {
                        printf("batch pass %d image %lld pixel (%lld, %lld) differs\n", pass,
                               (long long)i, (long long)y, (long long)x);
                        ok = 0;
                        break;
                    }
            free(img);
            free(want);
        }
    }
    HIP_OK(hipFree(din));
    HIP_OK(hipFree(dout));
    HIP_OK(hipFree(dtab));
    HIP_OK(hipFree(dws));
    free(arena);
    free(back);
    free(plan);
    printf("%s batch of %d images border %d\n", ok ? "match" : "MISMATCH", N, border);
    return ok;
}

/* Grey input, thresholded and edge-detected in one call, from rows that
 * start `offset` bytes past a 16-byte boundary with a pitch of W + pad
 * bytes, the device buffer ending at the image's last byte. */
static int run_grey_case(int64_t H, int64_t W, int64_t offset, int64_t pad, int threshold,
                         uint64_t seed) {
    const int64_t gs = W + pad, span = (H - 1) * gs + W;
    const int64_t wd = (W + 31) / 32, n = H * wd;
    uint8_t* grey = malloc((size_t)span);
    uint8_t* dense = malloc((size_t)(H * W));
    uint8_t* binary = malloc((size_t)(H * W));
    uint8_t* want = malloc((size_t)(H * W));
    uint32_t* back = malloc((size_t)n * 4);
    uint8_t* dgrey = NULL;
    void* dout = NULL;
    int ok = 1, rc;
    int64_t y, x;
    rng_state = seed;
    for (int64_t i = 0; i < span; ++i) grey[i] = (uint8_t)next_u64();
    for (y = 0; y < H; ++y)
        for (x = 0; x < W; ++x) dense[y * W + x] = grey[y * gs + x];
    oracle_threshold(dense, binary, H, W, threshold);
    oracle_edge_image(binary, want, H, W, 1, 1, 0);
    HIP_OK(hipMalloc((void**)&dgrey, (size_t)(offset + span)));
    HIP_OK(hipMalloc(&dout, (size_t)n * 4));
    HIP_OK(hipMemcpy(dgrey + offset, grey, (size_t)span, hipMemcpyHostToDevice));
    rc = edge_threshold_edges(dgrey + offset, gs, threshold, dout, H, W, wd, 32, EDGE_BORDER_WHITE,
                              EDGE_MODE_MASKS, 0, NULL, NULL);
    if (rc != EDGE_OK) {
        printf("edge_threshold_edges: %s\n", edge_status_string(rc));
        ok = 0;
    } else {
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipMemcpy(back, dout, (size_t)n * 4, hipMemcpyDeviceToHost));
        for (y = 0; y < H && ok; ++y)
            for (x = 0; x < W; ++x)
                if ((uint8_t)((back[y * wd + x / 32] >> (x % 32)) & 1) != want[y * W + x]) {
                    ok = 0;
                    break;
                }
    }
    HIP_OK(hipFree(dgrey));
    HIP_OK(hipFree(dout));
    free(grey);
    free(dense);
    free(binary);
    free(want);
    free(back);
    printf("%s grey %lld x %lld offset %lld pitch %lld threshold %d\n", ok ? "match" : "MISMATCH",
           (long long)H, (long long)W, (long long)offset, (long long)gs, threshold);
    return ok;
}

int main(void) {
    static const int64_t shapes[][2] = {{1, 1}, {3, 33}, {5, 64}, {70, 1000}, {257, 2049},
                                        {33, 8193}};
    int all = 1, cases = 0;
    if (edge_abi_version() != EDGE_MASKS_ABI_VERSION) {
        printf("ABI version mismatch\n");
        return 1;
    }
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s)
        for (int border = 0; border < 2; ++border)
            for (int kind = 0; kind < 3; ++kind) {
                all &= run_case(shapes[s][0], shapes[s][1], border, kind,
                                1000u * (uint64_t)s + 10u * (uint64_t)border + (uint64_t)kind);
                ++cases;
            }
    for (int border = 0; border < 2; ++border) {
        all &= run_batch_case(border, 77u + (uint64_t)border);
        ++cases;
    }
    {
        static const int64_t grey[][4] = {{1, 1, 0, 0}, {9, 100, 5, 3}, {17, 2048, 3, 0},
                                          {15, 4133, 11, 13}, {30, 4096, 8, 8}};
        for (size_t s = 0; s < sizeof(grey) / sizeof(grey[0]); ++s) {
            all &= run_grey_case(grey[s][0], grey[s][1], grey[s][2], grey[s][3], 97 + 20 * (int)s,
                                 500u + (uint64_t)s);
            ++cases;
        }
    }
    printf("%s: %d cases\n", all ? "all match" : "FAILED", cases);
    return all ? 0 : 1;
}
