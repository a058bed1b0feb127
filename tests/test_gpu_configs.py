"""Whole-image parity at the benchmark workloads' own sizes, seeds and
launch shapes, and of the wide strip kernel (four words per lane, whole
256-word spans with neighbour words on both sides, the steady-state group
loop) that those workloads run.

Workloads: a 512x512 stroke image (seed 1, uint32 rows); an 8192x8192 glyph
page (seed 2, uint64 rows) with the built-in and the autotuned shape; a
16384x16384 skeleton page (seed 4, uint64 rows) in full mode and its
clause-2 diagnostic; a 12800x32768 glyph page (seed 12) in the built-in
band shape; 4096 glyph crops (seed 3, uint32 rows) in one
persistent launch with the autotuned shape, replayed from a captured graph.
Every output word is compared with the oracle's edge map of section 1."""
import numpy as np
import pytest
import torch

import oracle
from synth import images, pack_rows, row_words, unpack_rows
from tests.gpu_util import assert_same, expect, log, run_single

pytestmark = pytest.mark.gpu


def _whole(img, word_bits, *, mode="masks", clause2_only=False, border="white", cfg=None):
    import paper_1401_5245_amd as em
    H, W = img.shape
    words = pack_rows(img, word_bits, pad="random", seed=H + W)
    dt = np.int64 if word_bits == 64 else np.int32
    inp = torch.from_numpy(words.view(dt)).cuda()
    out = torch.full_like(inp, -1)
    em.edge_image(inp, out, H, W, mode=mode, clause2_only=clause2_only, border=border, cfg=cfg)
    torch.cuda.synchronize()
    got = unpack_rows(out.cpu().numpy().view(words.dtype), W)
    del inp, out
    return got


def test_stroke_image_512_u32():
    img, _ = images.strokes_image(512, 512, seed=1)
    want = oracle.edge(img)
    for cfg in (None, "tuned"):
        log(f"512^2 u32 strokes cfg={cfg}")
        assert_same(_whole(img, 32, cfg=cfg), want, f"512^2 cfg={cfg}")


def test_glyph_page_8192_u64():
    img = images.glyph_page(8192, 8192, seed=2)
    for border in ("white", "black"):
        want = oracle.edge(img, border=border)
        for cfg in (None, "tuned"):
            log(f"8192^2 u64 glyph page {border} cfg={cfg}")
            assert_same(_whole(img, 64, border=border, cfg=cfg), want, f"8192^2 {border} {cfg}")


def test_skeleton_page_16384_u64_full_and_clause2():
    img = images.skeleton_page(16384, 16384, seed=4)
    want_c2 = oracle.edge(img, clauses=oracle.CLAUSE2)
    assert want_c2.sum() > 1000          # the page has clause-2 pixels to find
    for cfg in ("tuned", None):
        log(f"16384^2 u64 skeleton page full cfg={cfg}")
        got = _whole(img, 64, mode="full", cfg=cfg)
        assert_same(got, oracle.edge(img, clauses=oracle.CLAUSE1 | oracle.CLAUSE2),
                    f"16384^2 full cfg={cfg}")
        del got
        log(f"16384^2 u64 skeleton page clause 2 cfg={cfg}")
        assert_same(_whole(img, 64, mode="full", clause2_only=True, cfg=cfg), want_c2,
                    f"16384^2 clause 2 cfg={cfg}")


def test_glyph_page_12800x32768_u64_builtin_band():
    """From 96 MiB of traffic the built-in shape is a band (a workgroup's
    rows staged in LDS): a whole 12800 x 32768 page in full mode."""
    import ctypes
    from paper_1401_5245_amd import _abi
    c = _abi.EdgeLaunchCfg()
    assert _abi.load().edge_default_cfg(12800, 32768, 64, 1, 0, ctypes.byref(c)) == 0
    assert c.shape == _abi.EDGE_SHAPE_BAND_XCD
    img = images.glyph_page(12800, 32768, seed=12)
    log("12800x32768 u64 glyph page full, built-in band")
    assert_same(_whole(img, 64, mode="full"),
                oracle.edge(img, clauses=oracle.CLAUSE1 | oracle.CLAUSE2), "12800x32768 band")


def test_4096_glyph_crops_tuned_graph_replays():
    import paper_1401_5245_amd as em
    crops = images.glyph_crops(4096, seed=3)
    wants = [oracle.edge(c) for c in crops]
    packed = [(pack_rows(c, 32, pad="random", seed=i), c.shape[1]) for i, c in enumerate(crops)]
    for plan in ("host", "device"):
        b = em.Batch(packed, 32, "cuda", cfg="tuned", plan=plan)
        g = b.graph()
        for replay in range(3):
            log(f"4096 crops tuned plan={plan} replay {replay}")
            b.out.fill_(-1)          # eager work between replays
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            host = b.out.cpu().numpy().view(np.uint32)
            for i, c in enumerate(crops):
                got = unpack_rows(b.output_words(i, host), c.shape[1])
                assert_same(got, wants[i], f"crop {i} {c.shape} plan={plan} replay {replay}")
        g.close()


# Rows of at least two whole 256-word spans of four words per lane (uint64:
# 64 pixels per word), with and without a partial span at the end, tall
# enough that strips of 4..64 rows run the loop over whole groups of rows.
WIDE = [(100, 3 * 16384 + 37), (300, 4 * 16384), (71, 2 * 16384 + 64 * 129)]


@pytest.mark.parametrize("rows", [4, 8, 17, 64])
@pytest.mark.parametrize("cache", [1, 2])
@pytest.mark.parametrize("waves", [4, 8])
def test_wide_rows_vec4_whole_spans(rows, cache, waves):
    cfg = dict(vec_words=4, rows_per_tile=rows, waves_per_block=waves, blocks_per_cu=1,
               cache_policy=cache)
    for k, (H, W) in enumerate(WIDE):
        img = images.bernoulli_image(H, W, 0.35 + 0.1 * k, seed=H * 3 + W + rows)
        for mode, c2 in (("masks", False), ("full", False), ("full", True)):
            for border in ("white", "black"):
                log(f"wide {H}x{W} {mode} c2={c2} {border} {cfg}")
                # an even stride in 64-bit words keeps every row 16-byte aligned
                _, got = run_single(img, 64, border=border, mode=mode, clause2_only=c2, cfg=cfg,
                                    stride_extra=row_words(W, 64) % 2)
                assert_same(got, expect(img, border=border, mode=mode, clause2_only=c2),
                            f"{H}x{W} {mode} c2={c2} {border} {cfg}")
