"""Direction planes (section 4) and threshold packing (section 7) on the
GPU, bit-exact against the oracle."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from synth import images, pack_rows, row_words, unpack_rows
from tests.gpu_util import assert_same, log, to_device_words

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (1, 70), (5, 31), (3, 33), (40, 257), (17, 1000), (9, 2049), (33, 4100),
          (70, 8193)]


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("H,W", SHAPES)
def test_direction_planes(word_bits, H, W):
    import paper_1401_5245_amd as em
    img = images.bernoulli_image(H, W, 0.45, seed=H * 31 + W)
    for border in ("white", "black"):
        for extra in (0, 3):
            S = row_words(W, word_bits) + extra
            words = pack_rows(img, word_bits, S, pad="random", seed=W)
            inp = to_device_words(words)
            plane = H * S + 5                        # planes with a gap between them
            dt = inp.dtype
            out = torch.full((4 * plane,), -1, dtype=dt, device="cuda")
            em.edge_directions(inp, out, H, W, border=border, stride_words=S)
            mask = torch.zeros_like(inp)
            em.edge_masks(inp, mask, H, W, border=border)
            torch.cuda.synchronize()
            host = out.cpu().numpy().view(words.dtype)
            want = oracle.fundamental_edges(img, border=border)
            ors = np.zeros((H, W), np.uint8)
            for k in range(4):
                pw = host[k * plane:k * plane + H * S].reshape(H, S)
                got = unpack_rows(pw, W)
                assert_same(got, want[k], f"plane {oracle.DIRECTIONS[k]} B={word_bits} {border}")
                assert (pw[:, row_words(W, word_bits):] == ~words.dtype.type(0)).all()
                ors |= got
            assert_same(ors, unpack_rows(mask.cpu().numpy().view(words.dtype), W), "OR of planes")


def test_direction_planes_builtin_tiles():
    """From 12 MiB of image traffic, rows of four words per lane take 8-row
    tiles by default: a whole 3200 x 16384 page against the oracle."""
    import paper_1401_5245_amd as em
    img = images.glyph_page(3200, 16384, seed=9, noise=0.02)
    words = pack_rows(img, 64, pad="random", seed=9)
    inp = to_device_words(words)
    out = torch.empty((4,) + tuple(inp.shape), dtype=inp.dtype, device="cuda")
    em.edge_directions(inp, out, *img.shape)
    torch.cuda.synchronize()
    want = oracle.fundamental_edges(img)
    host = out.cpu().numpy().view(np.uint64)
    for k in range(4):
        assert_same(unpack_rows(host[k], img.shape[1]), want[k], oracle.DIRECTIONS[k])


@pytest.mark.parametrize("cfg", [dict(vec_words=1, rows_per_tile=3, waves_per_block=2),
                                 dict(vec_words=4, rows_per_tile=16, waves_per_block=8,
                                      cache_policy=2),
                                 dict(vec_words=4, rows_per_tile=7, waves_per_block=4, shape=1),
                                 dict(vec_words=2, rows_per_tile=16, waves_per_block=2, shape=2),
                                 dict(vec_words=4, rows_per_tile=2, waves_per_block=8, shape=4),
                                 dict(vec_words=2, rows_per_tile=4, waves_per_block=2, shape=3),
                                 dict(vec_words=1, rows_per_tile=1, waves_per_block=4, shape=3)])
def test_direction_planes_cfgs(cfg):
    import paper_1401_5245_amd as em
    img = images.glyph_page(300, 3000, seed=8, noise=0.02)
    words = pack_rows(img, 64)
    inp = to_device_words(words)
    out = torch.empty((4,) + tuple(inp.shape), dtype=inp.dtype, device="cuda")
    em.edge_directions(inp, out, *img.shape, cfg=cfg)
    torch.cuda.synchronize()
    want = oracle.fundamental_edges(img)
    host = out.cpu().numpy().view(np.uint64)
    for k in range(4):
        assert_same(unpack_rows(host[k], img.shape[1]), want[k], oracle.DIRECTIONS[k])


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("H,W", [(1, 1), (3, 31), (5, 32), (7, 33), (20, 100), (64, 1000),
                                 (9, 4097)])
def test_threshold_pack(word_bits, H, W):
    import paper_1401_5245_amd as em
    grey = images.grey_image(H, W, seed=H + W)
    for gpad in (0, 16, 5):                        # aligned and unaligned grey pitches
        gs = W + gpad
        g = np.zeros((H, gs), np.uint8)
        g[:, :W] = grey
        gt = torch.from_numpy(g).cuda()
        for t in (0, 1, 97, 128, 255, 256):
            S = row_words(W, word_bits) + 1
            out = to_device_words(np.full((H, S), 0x5A5A5A5A, dtype=np.uint32 if word_bits == 32
                                          else np.uint64))
            em.threshold_pack(gt, out, H, W, t, grey_stride=gs, stride_words=S)
            torch.cuda.synchronize()
            host = out.cpu().numpy().view(np.uint32 if word_bits == 32 else np.uint64)
            assert_same(unpack_rows(host, W), oracle.threshold(grey, t), f"t={t} gs={gs}")
            np.testing.assert_array_equal(pack_rows(oracle.threshold(grey, t), word_bits, S)[:, :-1],
                                          host[:, :-1])


@pytest.mark.parametrize("gpad", [0, 5])
def test_threshold_pack_streaming_stores(gpad):
    """Packed output of 16 MiB or more is stored non-temporally: 8192 rows
    of 16448 pixels (16.4 MiB packed) with an aligned and an unaligned grey
    pitch, the stride word after each row left untouched."""
    import paper_1401_5245_amd as em
    H, W = 8192, 16448
    grey = images.grey_image(H, W, seed=41 + gpad)
    gs = W + gpad
    g = np.zeros((H, gs), np.uint8)
    g[:, :W] = grey
    gt = torch.from_numpy(g).cuda()
    S = row_words(W, 64) + 1
    log(f"threshold pack with streaming stores: {H} x {W}, grey pitch {gs}")
    out = to_device_words(np.full((H, S), 0x5A5A5A5A5A5A5A5A, dtype=np.uint64))
    em.threshold_pack(gt, out, H, W, 128, grey_stride=gs, stride_words=S)
    torch.cuda.synchronize()
    host = out.cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(pack_rows(oracle.threshold(grey, 128), 64, S)[:, :-1],
                                  host[:, :-1])
    assert (host[:, -1] == np.uint64(0x5A5A5A5A5A5A5A5A)).all()


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("H,W", [(1, 1), (2, 31), (5, 33), (9, 1000), (4, 2048), (7, 2049),
                                 (33, 4100), (3, 8200)])
def test_threshold_edges_fused(word_bits, H, W):
    import paper_1401_5245_amd as em
    grey = images.grey_image(H, W, seed=2 * H + W)
    for gpad in (0, 16, 3):
        gs = W + gpad
        g = np.zeros((H, gs), np.uint8)
        g[:, :W] = grey
        gt = torch.from_numpy(g).cuda()
        for t in (0, 100, 128, 256):
            binary = oracle.threshold(grey, t)
            for border, mode, c2, inv in (("white", "masks", False, False),
                                          ("black", "full", True, False),
                                          ("white", "full", False, True)):
                S = row_words(W, word_bits)
                out = to_device_words(np.zeros((H, S), dtype=np.uint32 if word_bits == 32
                                               else np.uint64))
                em.threshold_edges(gt, out, H, W, t, grey_stride=gs, border=border, mode=mode,
                                   clause2_only=c2, invert=inv)
                torch.cuda.synchronize()
                host = out.cpu().numpy().view(np.uint32 if word_bits == 32 else np.uint64)
                clauses = oracle.CLAUSE2 if c2 else (3 if mode == "full" else oracle.CLAUSE1)
                want = oracle.edge(binary, border=border, clauses=clauses, invert=inv)
                assert_same(unpack_rows(host, W), want, f"t={t} gs={gs} {border} {mode}")


@pytest.mark.parametrize("W", [1, 31, 100, 2048, 2053, 4096, 4133])
def test_grey_rows_at_every_alignment(W):
    """Grey rows starting at every byte offset mod 16 (a base offset of
    0..15 bytes and pitches of W + 0, 1, 3, 8 and 13 bytes), read from a
    buffer that ends at the image's last byte: both threshold kernels equal
    the oracle."""
    import paper_1401_5245_amd as em
    H = 19
    grey = images.grey_image(H, W, seed=W)
    want_pack = oracle.threshold(grey, 131)
    want_edges = oracle.edge(want_pack, border="black")
    S = row_words(W, 32)
    packed = torch.zeros((H, S), dtype=torch.int32, device="cuda")
    edges = torch.zeros((H, S), dtype=torch.int32, device="cuda")
    for pad in (0, 1, 3, 8, 13):
        gs = W + pad
        for off in range(16):
            flat = np.zeros(off + (H - 1) * gs + W, np.uint8)
            for y in range(H):
                flat[off + y * gs:off + y * gs + W] = grey[y]
            buf = torch.from_numpy(flat).cuda()
            view = buf[off:]
            em.threshold_pack(view, packed, H, W, 131, grey_stride=gs)
            em.threshold_edges(view, edges, H, W, 131, grey_stride=gs, border="black")
            torch.cuda.synchronize()
            tag = f"W={W} pitch={gs} offset={off}"
            assert_same(unpack_rows(packed.cpu().numpy().view(np.uint32), W), want_pack, tag)
            assert_same(unpack_rows(edges.cpu().numpy().view(np.uint32), W), want_edges, tag)


def test_every_threshold_every_byte_value():
    """Every threshold 0..256 against a grey image that puts every byte
    value at every bit position of a 32-pixel word (value (x + 37y) mod 256
    over 32 rows), 2304 pixels wide: the fused kernel's first chunk lies
    wholly inside the row, its second is the partial last chunk."""
    import paper_1401_5245_amd as em
    H, W = 32, 2304
    y, x = np.mgrid[0:H, 0:W]
    grey = ((x + 37 * y) % 256).astype(np.uint8)
    gt = torch.from_numpy(grey).cuda()
    S = row_words(W, 64)
    packed = torch.zeros((H, S), dtype=torch.int64, device="cuda")
    edges = torch.zeros((H, S), dtype=torch.int64, device="cuda")
    for t in range(257):
        em.threshold_pack(gt, packed, H, W, t)
        em.threshold_edges(gt, edges, H, W, t)
        torch.cuda.synchronize()
        binary = oracle.threshold(grey, t)
        assert_same(unpack_rows(packed.cpu().numpy().view(np.uint64), W), binary, f"pack t={t}")
        assert_same(unpack_rows(edges.cpu().numpy().view(np.uint64), W), oracle.edge(binary),
                    f"edges t={t}")


@pytest.mark.parametrize("waves,rows", [(1, 1), (1, 8), (2, 2), (2, 4), (4, 4), (4, 8), (8, 2),
                                       (8, 8)])
def test_threshold_edges_band_heights(waves, rows):
    """The fused grey kernel runs bands of waves * rows' loaded rows (rows
    rounded to 2, 4 or 8, at least four rows a band) less two: heights
    around one and two bands, in every mode, with and without a partial
    last chunk."""
    import paper_1401_5245_amd as em
    rw = 8 if rows >= 8 else (4 if rows >= 4 else 2)
    while waves * rw < 4:
        rw *= 2
    ob = waves * rw - 2
    for H, cache in itertools.product(sorted({1, 2, 3, ob - 1, ob, ob + 1, 2 * ob - 1,
                                              2 * ob + 1} - {0}), (0, 1)):
        cfg = dict(vec_words=1, rows_per_tile=rows, waves_per_block=waves, cache_policy=cache)
        for W in (2048, 4096 + 37):
            grey = images.grey_image(H, W, seed=H * 3 + W + waves)
            gt = torch.from_numpy(np.ascontiguousarray(grey)).cuda()
            binary = oracle.threshold(grey, 128)
            for border, mode, c2, inv in (("white", "masks", False, False),
                                          ("black", "full", False, True),
                                          ("white", "full", True, False)):
                out = torch.full((H, row_words(W, 64)), -1, dtype=torch.int64, device="cuda")
                em.threshold_edges(gt, out, H, W, 128, border=border, mode=mode,
                                   clause2_only=c2, invert=inv, cfg=cfg)
                torch.cuda.synchronize()
                clauses = oracle.CLAUSE2 if c2 else (3 if mode == "full" else oracle.CLAUSE1)
                want = oracle.edge(binary, border=border, clauses=clauses, invert=inv)
                assert_same(unpack_rows(out.cpu().numpy().view(np.uint64), W), want,
                            f"H={H} W={W} {border} {mode} c2={c2} cache={cache}")


@pytest.mark.parametrize("rows,waves,cache", [(1, 1, 1), (3, 2, 2), (16, 8, 1), (64, 4, 2),
                                              (2, 8, 0), (4, 4, 0)])
def test_threshold_edges_cfgs(rows, waves, cache):
    import paper_1401_5245_amd as em
    H, W = 130, 5000
    grey = images.grey_image(H, W, seed=rows)
    gt = torch.from_numpy(np.ascontiguousarray(grey)).cuda()
    S = row_words(W, 64)
    out = torch.zeros((H, S), dtype=torch.int64, device="cuda")
    em.threshold_edges(gt, out, H, W, 120, cfg=dict(vec_words=1, rows_per_tile=rows,
                                                    waves_per_block=waves, cache_policy=cache))
    torch.cuda.synchronize()
    want = oracle.edge(oracle.threshold(grey, 120))
    assert_same(unpack_rows(out.cpu().numpy().view(np.uint64), W), want, "cfg")


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("H,W", [(1, 1), (1, 65), (6, 31), (5, 100), (40, 1000), (9, 4100)])
def test_staged_pipeline_equals_fused_and_oracle(word_bits, H, W):
    import paper_1401_5245_amd as em
    img = images.bernoulli_image(H, W, 0.5, seed=H + 7 * W)
    for border in ("white", "black"):
        S = row_words(W, word_bits) + 1
        words = pack_rows(img, word_bits, S, pad="random", seed=3)
        inp = to_device_words(words)
        out = torch.full_like(inp, -1)
        scratch = torch.full((em.staged_scratch_bytes(H, S, word_bits) // 4,), 7,
                             dtype=torch.int32, device="cuda")
        em.edge_masks_staged(inp, out, H, W, scratch, border=border)
        fused = torch.zeros_like(inp)
        em.edge_masks(inp, fused, H, W, border=border)
        torch.cuda.synchronize()
        host = out.cpu().numpy().view(words.dtype)
        assert_same(unpack_rows(host, W), oracle.edge(img, border=border), f"staged {border}")
        wd = row_words(W, word_bits)
        np.testing.assert_array_equal(host[:, :wd], fused.cpu().numpy().view(words.dtype)[:, :wd])
        assert (host[:, wd:] == ~words.dtype.type(0)).all()        # stride padding untouched
