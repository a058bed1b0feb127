/* Host-side argument validation of every libedgemask entry point, for a
 * build of the library whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer. Device pointers here are fake (never
 * dereferenced: each call returns from its checks before any HIP call);
 * host tables are exact-size heap blocks, so that a read past one is caught.
 * Prints "validate ok" and exits 0 when every status is as expected. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "edge_masks.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
    if (got != want) {
        printf("FAIL %s: got %d want %d\n", what, got, want);
        ++failures;
    }
}

#define A ((void*)(uintptr_t)0x10000000u)
#define B ((void*)(uintptr_t)0x20000000u)
#define W0 ((uintptr_t)0x30000000u)

static edge_image_desc* table_of(const int64_t (*rows)[4], int n) {
    edge_image_desc* t = (edge_image_desc*)malloc(sizeof(edge_image_desc) * (size_t)(n ? n : 1));
    for (int i = 0; i < n; ++i) {
        t[i].offset_words = rows[i][0];
        t[i].height = (int32_t)rows[i][1];
        t[i].width = (int32_t)rows[i][2];
        t[i].stride_words = rows[i][3];
    }
    return t;
}

int main(void) {
    /* statuses and strings */
    const int codes[] = {EDGE_OK, EDGE_ERR_INVALID, EDGE_ERR_ALIGN, EDGE_ERR_ALIAS, EDGE_ERR_HIP,
                         EDGE_ERR_WORKSPACE, EDGE_ERR_UNSUPPORTED, -99};
    for (unsigned i = 0; i < sizeof codes / sizeof codes[0]; ++i)
        if (!edge_status_string(codes[i])[0]) expect(1, 0, "status string");
    expect(edge_last_hip_error(), 0, "last hip error");
    expect(edge_abi_version(), EDGE_MASKS_ABI_VERSION, "abi version");

    /* single images */
    expect(edge_masks(A, B, 4, 100, 4, 16, 0, NULL), EDGE_ERR_INVALID, "word bits");
    expect(edge_masks(A, B, 4, 100, 4, 32, 2, NULL), EDGE_ERR_INVALID, "border");
    expect(edge_masks(A, B, -1, 100, 4, 32, 0, NULL), EDGE_ERR_INVALID, "height");
    expect(edge_masks(A, B, 4, 100, 3, 32, 0, NULL), EDGE_ERR_INVALID, "stride");
    expect(edge_masks(NULL, B, 4, 100, 4, 32, 0, NULL), EDGE_ERR_INVALID, "null in");
    expect(edge_masks((char*)A + 2, B, 4, 100, 4, 32, 0, NULL), EDGE_ERR_ALIGN, "align");
    expect(edge_masks(A, (char*)A + 16, 4, 100, 4, 32, 0, NULL), EDGE_ERR_ALIAS, "alias");
    expect(edge_masks(A, B, (int64_t)1 << 31, 100, 4, 32, 0, NULL), EDGE_ERR_INVALID, "tall");
    expect(edge_masks(A, B, 4, (int64_t)1 << 31, (int64_t)1 << 26, 32, 0, NULL), EDGE_ERR_INVALID,
           "wide");
    expect(edge_masks(A, B, 4, 100, INT64_MAX / 2, 32, 0, NULL), EDGE_ERR_INVALID, "huge stride");
    expect(edge_masks(NULL, NULL, 0, 100, 4, 32, 0, NULL), EDGE_OK, "empty");
    expect(edge_full(A, B, 4, 100, 4, 32, 0, 8u, NULL), EDGE_ERR_INVALID, "full flags");
    expect(edge_image_launch(A, B, 4, 100, 4, 32, 0, 2, 0u, NULL, NULL), EDGE_ERR_INVALID, "mode");
    expect(edge_image_launch(A, B, 4, 100, 4, 32, 0, 0, EDGE_FLAG_CLAUSE2_ONLY, NULL, NULL),
           EDGE_ERR_INVALID, "clause 2 in plain mode");
    {
        const edge_launch_cfg bad[] = {{3, 4, 4, 1, 0, 0},   {4, 0, 4, 1, 0, 0},
                                       {4, 4, 3, 1, 0, 0},   {4, 4, 4, 0, 0, 0},
                                       {4, 2000, 4, 1, 0, 0}, {4, 4, 4, 33, 0, 0},
                                       {4, 4, 4, 1, 3, 0},   {4, 4, 4, 1, -1, 0},
                                       {4, EDGE_TILE_MAX_ROWS + 1, 4, 1, 0, EDGE_SHAPE_TILE},
                                       {4, 4, 4, 1, 0, 5},   {4, 4, 4, 1, 0, -1},
                                       {4, 3, 4, 1, 0, EDGE_SHAPE_BAND}, {4, 2, 1, 1, 0, EDGE_SHAPE_BAND}};
        for (unsigned i = 0; i < sizeof bad / sizeof bad[0]; ++i) {
            edge_launch_cfg* c = (edge_launch_cfg*)malloc(sizeof *c);
            *c = bad[i];
            expect(edge_image_launch(A, B, 4, 100, 4, 32, 0, 0, 0u, c, NULL), EDGE_ERR_INVALID,
                   "cfg");
            free(c);
        }
    }
    expect(edge_directions(A, B, 3, 4, 100, 4, 32, 0, NULL, NULL), EDGE_ERR_INVALID,
           "plane too small");
    expect(edge_threshold_pack(A, 100, 257, B, 4, 100, 4, 32, NULL), EDGE_ERR_INVALID,
           "threshold");
    expect(edge_threshold_pack(A, 99, 128, B, 4, 100, 4, 32, NULL), EDGE_ERR_INVALID,
           "grey pitch");
    expect(edge_threshold_edges(A, 100, -1, B, 4, 100, 4, 32, 0, 0, 0u, NULL, NULL),
           EDGE_ERR_INVALID, "grey threshold");
    expect(edge_peel(A, B, 4, 100, 4, 32, 0, EDGE_PEEL_MAX_ITERATIONS + 1, 0u, NULL, NULL),
           EDGE_ERR_INVALID, "peel count");
    expect(edge_peel(A, B, 4, 100, 4, 32, 0, 3, 1u, NULL, NULL), EDGE_ERR_INVALID, "peel flags");
    expect(edge_masks_staged(A, B, (void*)W0, 8, 4, 100, 4, 32, 0, NULL), EDGE_ERR_WORKSPACE,
           "staged scratch");
    expect(edge_copy_bytes(A, B, 15, NULL), EDGE_ERR_INVALID, "copy size");
    expect(edge_copy_bytes(A, (char*)A + 16, 64, NULL), EDGE_ERR_ALIAS, "copy alias");
    {
        edge_launch_cfg* c = (edge_launch_cfg*)malloc(sizeof *c);
        expect(edge_default_cfg(8192, 8192, 64, 0, 0, c), EDGE_OK, "default cfg");
        expect(edge_default_cfg(8192, 8192, 48, 0, 0, c), EDGE_ERR_INVALID, "default cfg bits");
        expect(edge_default_cfg(100, 100, 32, 0, 1, c), EDGE_OK, "default batch cfg");
        free(c);
    }

    /* batches: descriptor tables in exact-size host blocks */
    {
        const int64_t ok_rows[2][4] = {{0, 4, 100, 4}, {16, 3, 500, 18}};
        edge_image_desc* ok = table_of(ok_rows, 2);
        expect(edge_batch_check(ok, 2, 16 + 2 * 18 + 16, 32), EDGE_OK, "batch check");
        expect(edge_batch_check(ok, 2, 16 + 2 * 18 + 15, 32), EDGE_ERR_INVALID, "overrun");
        free(ok);
        const int64_t bad_rows[][4] = {{-1, 1, 1, 1}, {0, -1, 1, 1}, {0, 1, -1, 1},
                                       {0, 2, 100, 3}, {0, (int64_t)1 << 30, 1, 1},
                                       {901, 1, 3200, 100}};
        for (unsigned i = 0; i < sizeof bad_rows / sizeof bad_rows[0]; ++i) {
            edge_image_desc* t = table_of(&bad_rows[i], 1);
            expect(edge_batch_check(t, 1, 1000, 32), EDGE_ERR_INVALID, "bad descriptor");
            free(t);
        }
        expect(edge_batch_check(NULL, 0, 0, 32), EDGE_OK, "empty table");
        expect(edge_batch_check(NULL, 1, 10, 32), EDGE_ERR_INVALID, "null table");
    }
    {
        const int64_t need = edge_batch_workspace_bytes(4);
        expect(need > 0, 1, "workspace bytes");
        expect(edge_batch_workspace_bytes(-1) < 0, 1, "negative count");
        const edge_image_desc* tab = (const edge_image_desc*)(W0 + 0x1000);
        expect(edge_batch(A, B, 1000, tab, -1, 32, 0, 0, 0u, NULL, (void*)W0, need, NULL),
               EDGE_ERR_INVALID, "batch count");
        expect(edge_batch(A, B, 1000, tab, 4, 8, 0, 0, 0u, NULL, (void*)W0, need, NULL),
               EDGE_ERR_INVALID, "batch bits");
        expect(edge_batch(A, B, 1000, (const edge_image_desc*)((char*)tab + 4), 4, 32, 0, 0, 0u, NULL, (void*)W0, need,
                          NULL), EDGE_ERR_ALIGN, "table align");
        expect(edge_batch(A, (char*)A + 400, 1000, tab, 4, 32, 0, 0, 0u, NULL, (void*)W0, need,
                          NULL), EDGE_ERR_ALIAS, "arena alias");
        expect(edge_batch(A, B, 1000, tab, 4, 32, 0, 0, 0u, NULL, (void*)W0, need - 8, NULL),
               EDGE_ERR_WORKSPACE, "small workspace");
        expect(edge_batch(A, B, 1000, tab, 0, 32, 0, 0, 0u, NULL, (void*)W0, need, NULL), EDGE_OK,
               "empty batch");
        void* g = NULL;
        expect(edge_batch_graph_create(A, B, 1000, tab, 4, 32, 0, 0, 0u, NULL, (void*)W0,
                                       need - 8, &g), EDGE_ERR_WORKSPACE, "graph workspace");
        expect(g == NULL, 1, "no graph");
        expect(edge_graph_destroy(NULL), EDGE_OK, "destroy null");
        expect(edge_graph_launch(NULL, NULL), EDGE_ERR_INVALID, "launch null");
        expect(edge_batch_noalloc(A, B, 1000, tab, EDGE_BATCH_NOALLOC_MAX_IMAGES + 1, 32, 0, 0,
                                  0u, NULL, NULL), EDGE_ERR_WORKSPACE, "noalloc count");
        expect(edge_batch_noalloc(A, B, 1000, tab, 4, 32, 0, 0, EDGE_FLAG_PLANNED, NULL, NULL),
               EDGE_ERR_INVALID, "noalloc planned");
        expect(edge_batch_noalloc(A, B, 1000, tab, 0, 32, 0, 0, 0u, NULL, NULL), EDGE_OK,
               "noalloc empty");
        int64_t used = 0;
        const int64_t one[1][4] = {{0, 4, 100, 4}};
        edge_image_desc* t = table_of(one, 1);
        int64_t* plan = (int64_t*)malloc(16);
        expect(edge_batch_plan(A, B, 100, t, 1, 32, NULL, plan, 16, &used), EDGE_ERR_WORKSPACE,
               "plan size");
        expect(edge_batch_plan(A, B, 100, t, 1, 48, NULL, plan, 16, &used), EDGE_ERR_INVALID,
               "plan bits");
        expect(edge_batch_plan(A, B, 100, t, 1, 32, NULL, plan, 16, NULL), EDGE_ERR_INVALID,
               "plan used");
        free(plan);
        free(t);
    }
    if (failures) return 1;
    printf("validate ok\n");
    return 0;
}
