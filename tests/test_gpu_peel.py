"""Iterated edge peeling on the GPU (edge_peel), bit-exact against the
oracle's repeated peel, plus properties that hold at any size."""
import functools

import numpy as np
import pytest
import torch

import oracle
from synth import images, pack_rows, pad_bits_zero, row_words, unpack_rows
from tests.gpu_util import SENTINEL32, assert_same, log, to_device_words

pytestmark = pytest.mark.gpu

ITERS = [0, 1, 2, 3, 5, 8, 9, 16, 17, 30]
# widths around the 62-word chunk of a peel wavefront (32-bit words): 1984
# pixels fill one chunk exactly, 1985 spill one word into the next
SHAPES = [(1, 1), (1, 70), (5, 31), (3, 33), (40, 257), (17, 1000), (9, 1984), (12, 1985),
          (33, 4100), (70, 8193), (130, 64)]


def sparse_white(H, W, seed, p=0.004):
    """Mostly black with scattered white pixels, so deep peels still
    change the image."""
    rng = np.random.default_rng(seed)
    return (rng.random((H, W)) < p).astype(np.uint8)


def run_peel(img, word_bits, k, *, border="white", edge_out=False, stride_extra=1, cfg=None):
    import paper_1401_5245_amd as em
    H, W = img.shape
    S = row_words(W, word_bits) + stride_extra
    words = pack_rows(img, word_bits, S, pad="random", seed=H + 3 * W)
    inp = to_device_words(words)
    sent = words.dtype.type(SENTINEL32 if word_bits == 32 else 0xA5A5A5A5A5A5A5A5)
    out = to_device_words(np.full_like(words, sent))
    em.peel(inp, out, H, W, k, border=border, edge_out=edge_out, cfg=cfg, stride_words=S)
    torch.cuda.synchronize()
    ow = out.cpu().numpy().view(words.dtype).reshape(H, S)
    assert (ow[:, row_words(W, word_bits):] == sent).all(), "stride padding was written"
    assert pad_bits_zero(ow, W), "output pad bits are not zero"
    return unpack_rows(ow, W)


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("H,W", SHAPES)
def test_peel_matches_oracle(word_bits, H, W):
    log(f"peel B={word_bits} {H}x{W}")
    img = sparse_white(H, W, seed=H * 131 + W)
    for border in ("white", "black"):
        for k in ITERS:
            for edge_out in (False, True):
                got = run_peel(img, word_bits, k, border=border, edge_out=edge_out)
                want = oracle.peel(img, k, border=border, edge_out=edge_out)
                assert_same(got, want, f"k={k} edge_out={edge_out} {border}")


@pytest.mark.parametrize("cfg", [dict(rows_per_tile=1, waves_per_block=1),
                                 dict(rows_per_tile=3, waves_per_block=2),
                                 dict(rows_per_tile=7, waves_per_block=8, cache_policy=2),
                                 dict(rows_per_tile=64, waves_per_block=4, cache_policy=1),
                                 dict(rows_per_tile=256, waves_per_block=4)])
def test_peel_cfgs(cfg):
    img = images.glyph_page(300, 3000, seed=8, noise=0.02)
    img = np.where(sparse_white(300, 3000, seed=2, p=0.001) == 1, 1, img).astype(np.uint8)
    full = dict(vec_words=1, blocks_per_cu=1, cache_policy=0)
    full.update(cfg)
    for k in (1, 7, 30):
        for edge_out in (False, True):
            got = run_peel(img, 64, k, edge_out=edge_out, cfg=full, stride_extra=0)
            assert_same(got, oracle.peel(img, k, edge_out=edge_out), f"{cfg} k={k}")


def test_peel_zero_is_input_and_edge_is_edge_masks():
    import paper_1401_5245_amd as em
    img = images.glyph_page(257, 1111, seed=3, noise=0.01)
    assert_same(run_peel(img, 32, 0), img, "zero peels")
    words = pack_rows(img, 32)
    inp = to_device_words(words)
    a, b = torch.empty_like(inp), torch.empty_like(inp)
    em.peel(inp, a, *img.shape, 0, edge_out=True)
    em.edge_masks(inp, b, *img.shape)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def oracle_rows(img, k, rows, border="white", edge_out=False):
    """Rows of the oracle's peel of a tall image, each from a window of
    k + 2 rows on either side: a peel moves information one row, so the
    window's cut edges cannot reach the middle row."""
    H = img.shape[0]
    out = []
    for y in rows:
        lo, hi = max(0, y - k - 2), min(H, y + k + 3)
        out.append(oracle.peel(img[lo:hi], k, border=border, edge_out=edge_out)[y - lo])
    return np.stack(out)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 7, 8, 30])
def test_peel_8192_sampled_rows(k):
    """The 8192^2 glyph page in uint64 words, in the built-in launch shape:
    sampled rows against the oracle on row windows."""
    import paper_1401_5245_amd as em
    H = W = 8192
    log(f"peel 8192^2 k={k}")
    img = images.glyph_page(H, W, seed=2)
    inp = to_device_words(pack_rows(img, 64))
    out = torch.empty_like(inp)
    rows = [0, 1, 2, 31, 32, 33, 4095, 4096, 8159, 8190, 8191]
    for edge_out in (False, True):
        em.peel(inp, out, H, W, k, edge_out=edge_out)
        torch.cuda.synchronize()
        got = unpack_rows(out[rows].cpu().numpy().view(np.uint64), W)
        assert_same(got, oracle_rows(img, k, rows, edge_out=edge_out), f"k={k} {edge_out}")


@functools.lru_cache(maxsize=1)
def _page_32768():
    """The 8192^2 glyph page of seed 5 tiled 4 x 4, and its uint64 words."""
    img = np.tile(images.glyph_page(8192, 8192, seed=5), (4, 4))
    return img, pack_rows(img, 64)


@pytest.mark.parametrize("k", [4, 5, 6, 7])
def test_peel_32768_sampled_rows(k):
    """A 32768^2 image (2^30 pixels: four to seven levels take four words
    per lane in the built-in shape), uint64 words, and the same image in
    uint32 words from a start that is 4 bytes off an 8-byte boundary (one
    word per lane, the one-word shape): sampled rows against the oracle on
    row windows."""
    import paper_1401_5245_amd as em
    H = W = 32768
    log(f"peel 32768^2 k={k}")
    img, words = _page_32768()
    rows = [0, 1, 2, 31, 32, 33, 16383, 16384, 32735, 32766, 32767]
    inp = to_device_words(words)
    out = torch.empty_like(inp)
    w32 = words.view(np.uint32)
    flat = torch.zeros(w32.size + 1, dtype=torch.int32, device="cuda")
    flat[1:] = torch.from_numpy(w32.reshape(-1).view(np.int32)).cuda()
    inp_odd = flat[1:].view(H, -1)                         # 4 bytes past an 8-byte boundary
    out_odd = torch.empty_like(inp_odd)
    for edge_out in (False, True):
        want = oracle_rows(img, k, rows, edge_out=edge_out)
        em.peel(inp, out, H, W, k, edge_out=edge_out)
        em.peel(inp_odd, out_odd, H, W, k, edge_out=edge_out)
        torch.cuda.synchronize()
        got = unpack_rows(out[rows].cpu().numpy().view(np.uint64), W)
        assert_same(got, want, f"k={k} {edge_out} uint64")
        got = unpack_rows(out_odd[rows].cpu().numpy().view(np.uint32), W)
        assert_same(got, want, f"k={k} {edge_out} uint32, odd start")


def test_peel_composes():
    """k peels in one call equal k single peels, and a peels then b peels
    equal a + b peels (2048^2, random sparse-white content, both borders)."""
    import paper_1401_5245_amd as em
    H = W = 2048
    img = sparse_white(H, W, seed=11, p=0.002)
    inp = to_device_words(pack_rows(img, 64))
    for border in ("white", "black"):
        a, b, c = (torch.empty_like(inp) for _ in range(3))
        em.peel(inp, a, H, W, 12, border=border)
        src, dst = inp, b
        for i in range(12):
            em.peel(src, dst, H, W, 1, border=border)
            src, dst = dst, (c if dst is b else b)
        torch.cuda.synchronize()
        assert torch.equal(a, src), f"one call of 12 != 12 single peels ({border})"
        em.peel(inp, b, H, W, 5, border=border)
        em.peel(b, c, H, W, 7, border=border)
        torch.cuda.synchronize()
        assert torch.equal(a, c), f"5 then 7 != 12 ({border})"


def white_seeds(H, W, n, seed):
    """A black image with n isolated white pixels. Each peel grows their
    diamonds by one pixel, so every level up to 30 still changes rows near
    them; on images whose deep levels have turned all white, a level formed
    wrongly (or not at all) would not show."""
    rng = np.random.default_rng(seed)
    img = np.zeros((H, W), np.uint8)
    img[rng.integers(0, H, n), rng.integers(0, W, n)] = 1
    return img


@pytest.mark.parametrize("k", [6, 7, 14, 15, 16, 17, 22, 29, 30])
def test_peel_deep_levels(k):
    """Levels that are still changing at every depth, through both the
    one-wavefront and the split strip units, with strips short enough that
    every strip starts in a different phase of the level switch-on."""
    for (H, W, n, wb) in ((90, 3000, 6, 32), (130, 200, 3, 64)):
        img = white_seeds(H, W, n, seed=H + k)
        for border in ("black", "white"):
            for edge_out in (False, True):
                want = oracle.peel(img, k, border=border, edge_out=edge_out)
                prev = oracle.peel(img, k - 1, border=border, edge_out=edge_out)
                assert not np.array_equal(want, prev), "the input does not exercise level k"
                for rows in (None, 3, 7, 32, 64):
                    cfg = None if rows is None else dict(
                        vec_words=1, rows_per_tile=rows, waves_per_block=2, blocks_per_cu=1,
                        cache_policy=0)
                    got = run_peel(img, wb, k, border=border, edge_out=edge_out, cfg=cfg)
                    assert_same(got, want, f"{H}x{W} k={k} {border} edge_out={edge_out} rows={rows}")


@pytest.mark.parametrize("k,edge_out", [(0, False), (1, False), (0, True)])
@pytest.mark.parametrize("cfg", [None,
                                 dict(vec_words=4, rows_per_tile=2, waves_per_block=4,
                                      blocks_per_cu=1, cache_policy=2),
                                 dict(vec_words=2, rows_per_tile=7, waves_per_block=1,
                                      blocks_per_cu=1, cache_policy=1)])
def test_single_level_on_strip_loop(k, edge_out, cfg):
    """One level or none runs the edge kernels' strip loop (any vector
    width, narrow rows included); odd strides force narrower loads."""
    for (H, W, wb, extra) in ((70, 8193, 32, 1), (33, 4100, 64, 0), (41, 900, 32, 3),
                              (9, 20000, 64, 1)):
        img = sparse_white(H, W, seed=H + W + k, p=0.05)
        for border in ("white", "black"):
            got = run_peel(img, wb, k, border=border, edge_out=edge_out, cfg=cfg,
                           stride_extra=extra)
            assert_same(got, oracle.peel(img, k, border=border, edge_out=edge_out),
                        f"{H}x{W} B={wb} k={k} edge_out={edge_out} {border} cfg={cfg}")


@pytest.mark.parametrize("vec", [1, 2, 4])
@pytest.mark.parametrize("edge_out", [False, True])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
def test_peel_vector_widths(vec, k, edge_out):
    """Up to seven levels with one, two or four words per lane (strides that
    do not divide by the width fall back to narrower loads), sparse content
    so that every level still changes the image."""
    for (H, W, wb, extra) in ((70, 8193, 32, 0), (33, 4100, 64, 0), (41, 900, 32, 3),
                              (9, 20000, 64, 1), (130, 2100, 32, 4)):
        img = sparse_white(H, W, seed=H + W + k, p=0.003)
        for border in ("white", "black"):
            want = oracle.peel(img, k, border=border, edge_out=edge_out)
            for rows in (3, 8):
                cfg = dict(vec_words=vec, rows_per_tile=rows, waves_per_block=2, blocks_per_cu=1,
                           cache_policy=0)
                got = run_peel(img, wb, k, border=border, edge_out=edge_out, cfg=cfg,
                               stride_extra=extra)
                assert_same(got, want, f"{H}x{W} B={wb} k={k} {border} vec={vec} rows={rows}")


@pytest.mark.parametrize("edge_out", [False, True])
def test_every_level_count(edge_out):
    """Every peel count 0..30 with both outputs, so that every kernel
    instantiation (one per level count and output, and the vector-width
    ones) runs: on seeded images whose every level still changes, with the
    built-in shape and with one word per lane."""
    one = dict(vec_words=1, rows_per_tile=8, waves_per_block=4, blocks_per_cu=1, cache_policy=0)
    for (H, W, n, wb) in ((200, 3000, 6, 32), (150, 1000, 3, 64)):
        img = white_seeds(H, W, n, seed=H + W)
        for border in ("black", "white"):
            for k in range(0, 31):
                want = oracle.peel(img, k, border=border, edge_out=edge_out)
                for cfg in (None, one):
                    got = run_peel(img, wb, k, border=border, edge_out=edge_out, cfg=cfg)
                    assert_same(got, want, f"{H}x{W} k={k} {border} cfg={cfg}")
