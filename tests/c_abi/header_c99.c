/* The public header is plain C: this file compiles as strict C99 and takes
 * the address of every entry point with its declared type. Compiled by
 * tests/test_c_abi.py with gcc -std=c99 -pedantic -Werror -fsyntax-only. */
#include <stddef.h>
#include "edge_masks.h"

typedef int (*image_fn)(const void*, void*, int64_t, int64_t, int64_t, int, int, void*);
typedef void (*any_fn)(void);

int main(void) {
    image_fn masks = edge_masks;
    any_fn all[] = {
        (any_fn)edge_masks, (any_fn)edge_full, (any_fn)edge_image_launch,
        (any_fn)edge_directions, (any_fn)edge_threshold_pack, (any_fn)edge_threshold_edges,
        (any_fn)edge_masks_staged, (any_fn)edge_peel, (any_fn)edge_default_cfg,
        (any_fn)edge_batch_workspace_bytes, (any_fn)edge_batch_check, (any_fn)edge_batch_plan,
        (any_fn)edge_batch, (any_fn)edge_batch_graph_create, (any_fn)edge_graph_launch,
        (any_fn)edge_graph_destroy, (any_fn)edge_copy_bytes, (any_fn)edge_status_string,
        (any_fn)edge_last_hip_error, (any_fn)edge_abi_version};
    edge_image_desc d = {0, 1, 1, 1};
    edge_launch_cfg c = {4, 8, 4, 1, EDGE_CACHE_AUTO, EDGE_SHAPE_STRIP};
    (void)masks;
    (void)d;
    (void)c;
    return (int)(sizeof(all) / sizeof(all[0])) == 20 ? 0 : 1;
}
