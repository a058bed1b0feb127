"""Bit-exact parity of the HIP path with the CPU oracle (needs a gfx950 GPU).

Sizes span several wavefront spans and a ragged tail; every case compares
the whole edge map with the oracle's, checks that stride padding is never
written and that output pad bits are zero."""
import numpy as np
import pytest

from synth import images
from tests.gpu_util import assert_same, expect, log, run_single

pytestmark = pytest.mark.gpu

WIDTHS = [1, 5, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 1000, 1024, 2049, 4100,
          8191, 8193, 16500]
HEIGHTS = [1, 2, 3, 7, 33]


def rand_img(H, W, q=0.5, seed=0):
    return images.bernoulli_image(H, W, q, seed)


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("W", WIDTHS)
def test_plain_shapes(word_bits, W):
    for H in HEIGHTS:
        img = rand_img(H, W, 0.5, seed=H * 1000 + W)
        for border in ("white", "black"):
            log(f"plain B={word_bits} H={H} W={W} border={border}")
            _, got = run_single(img, word_bits, border=border, api="masks")
            assert_same(got, expect(img, border=border), f"H={H} W={W} {border}")


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("W", [1, 33, 100, 257, 1000, 2049, 8193])
@pytest.mark.parametrize("clause2_only", [False, True])
def test_full_mode_shapes(word_bits, W, clause2_only):
    for H in (1, 2, 5, 40):
        img = rand_img(H, W, 0.7, seed=W + H)   # mostly black: clause 2 fires often
        for border in ("white", "black"):
            log(f"full B={word_bits} H={H} W={W} c2={clause2_only} {border}")
            _, got = run_single(img, word_bits, border=border, mode="full",
                                clause2_only=clause2_only, api="full")
            assert_same(got, expect(img, border=border, mode="full", clause2_only=clause2_only),
                        f"H={H} W={W} {border}")


@pytest.mark.parametrize("mode,c2", [("masks", False), ("full", False), ("full", True)])
def test_invert_flag(mode, c2):
    img = rand_img(37, 700, 0.4, seed=3)
    for border in ("white", "black"):
        _, got = run_single(img, 64, border=border, mode=mode, clause2_only=c2, invert=True)
        assert_same(got, expect(img, border=border, mode=mode, clause2_only=c2, invert=True))


@pytest.mark.parametrize("word_bits", [32, 64])
def test_strides_pads_and_alignment(word_bits):
    img = rand_img(50, 3000, 0.5, seed=9)
    want = expect(img)
    for stride_extra in (0, 1, 2, 3, 7):
        for offset_w in (0, 1, 2, 3):     # misaligns the pointers for 128-bit access
            for pad in ("zero", "ones", "random"):
                _, got = run_single(img, word_bits, stride_extra=stride_extra, pad=pad,
                                    offset_words=offset_w)
                assert_same(got, want, f"stride+{stride_extra} off{offset_w} pad={pad}")


@pytest.mark.parametrize("cfg", [dict(vec_words=4, rows_per_tile=16, waves_per_block=8, shape=2),
                                 dict(vec_words=4, rows_per_tile=7, waves_per_block=2, shape=1),
                                 dict(vec_words=4, rows_per_tile=2, waves_per_block=8, shape=4),
                                 dict(vec_words=2, rows_per_tile=4, waves_per_block=1, shape=3)])
@pytest.mark.parametrize("word_bits", [32, 64])
def test_strides_pads_and_alignment_tiles_bands(cfg, word_bits):
    """Tiles and bands over garbage pad bits, stride padding (never written)
    and pointers off the 16-byte boundary (fewer words per lane)."""
    img = rand_img(50, 3000, 0.5, seed=19)
    for mode, c2 in (("masks", False), ("full", True)):
        want = expect(img, mode=mode, clause2_only=c2)
        for stride_extra in (0, 1, 3):
            for offset_w in (0, 1, 2, 3):
                for pad in ("ones", "random"):
                    _, got = run_single(img, word_bits, stride_extra=stride_extra, pad=pad,
                                        offset_words=offset_w, mode=mode, clause2_only=c2,
                                        cfg=cfg)
                    assert_same(got, want, f"{cfg} B{word_bits} stride+{stride_extra} "
                                           f"off{offset_w} pad={pad} {mode}")


@pytest.mark.parametrize("vec", [1, 2, 4])
@pytest.mark.parametrize("rows", [1, 3, 4, 5, 8, 17, 64])
@pytest.mark.parametrize("waves", [1, 2, 4, 8])
@pytest.mark.parametrize("cache", [1, 2])
def test_launch_configs(vec, rows, waves, cache):
    cfg = dict(vec_words=vec, rows_per_tile=rows, waves_per_block=waves, blocks_per_cu=1,
               cache_policy=cache)
    for (H, W, wb) in ((70, 4100, 64), (33, 1000, 32), (9, 300, 32), (100, 700, 64)):
        img = rand_img(H, W, 0.5, seed=H + W + vec)
        for mode, c2 in (("masks", False), ("full", True)):
            _, got = run_single(img, wb, mode=mode, clause2_only=c2, cfg=cfg)
            assert_same(got, expect(img, mode=mode, clause2_only=c2), f"{cfg} {H}x{W}")


# Tiles: a multi-chunk row with a partial last chunk (33000 pixels), whole
# 256-word chunks (16384 pixels of uint64), rows of one partial chunk, one
# row, rows of at most 32 words (which take the narrow kernel whatever the
# shape) and uint32 rows that split a 64-bit word
TILE_IMAGES = ((70, 4100, 64), (100, 33000, 64), (17, 16384, 64), (1, 2000, 32), (5, 700, 64),
               (33, 1000, 32), (40, 16416, 32))
TILE_CASES = (("masks", False, "white", False), ("full", False, "black", True),
              ("full", True, "white", False))
_tile_expected = {}


def _tile_case(H, W, mode, c2, border, inv):
    key = (H, W, mode, c2, border, inv)
    if key not in _tile_expected:
        img = rand_img(H, W, 0.45, seed=H * 7 + W)
        _tile_expected[key] = (img, expect(img, border=border, mode=mode, clause2_only=c2,
                                           invert=inv))
    return _tile_expected[key]


@pytest.mark.parametrize("vec", [1, 2, 4])
@pytest.mark.parametrize("rows", [1, 2, 7, 8, 9, 16])
@pytest.mark.parametrize("waves", [1, 4, 8])
@pytest.mark.parametrize("shape", [1, 2])
def test_tile_configs(vec, rows, waves, shape):
    """Tiles (every row of a unit requested at once) of every height up to
    the most, in both workgroup orders, against the oracle."""
    cfg = dict(vec_words=vec, rows_per_tile=rows, waves_per_block=waves, blocks_per_cu=1,
               cache_policy=0, shape=shape)
    for (H, W, wb) in TILE_IMAGES:
        for (mode, c2, border, inv) in TILE_CASES:
            img, want = _tile_case(H, W, mode, c2, border, inv)
            _, got = run_single(img, wb, mode=mode, clause2_only=c2, border=border, invert=inv,
                                cfg=cfg)
            assert_same(got, want, f"{cfg} {H}x{W} B{wb} {mode} c2={c2} {border} inv={inv}")


@pytest.mark.parametrize("vec", [1, 2, 4])
@pytest.mark.parametrize("rows", [1, 2, 4])
@pytest.mark.parametrize("waves", [1, 2, 4, 8])
@pytest.mark.parametrize("shape", [3, 4])
def test_band_configs(vec, rows, waves, shape):
    """Bands (a workgroup's rows staged in LDS, all loaded at once) of every
    height, in both workgroup orders, against the oracle."""
    if waves * rows < 3:
        pytest.skip("a band computes waves * rows - 2 >= 1 rows")
    cfg = dict(vec_words=vec, rows_per_tile=rows, waves_per_block=waves, blocks_per_cu=1,
               cache_policy=0, shape=shape)
    for (H, W, wb) in TILE_IMAGES:
        for (mode, c2, border, inv) in TILE_CASES:
            img, want = _tile_case(H, W, mode, c2, border, inv)
            _, got = run_single(img, wb, mode=mode, clause2_only=c2, border=border, invert=inv,
                                cfg=cfg)
            assert_same(got, want, f"{cfg} {H}x{W} B{wb} {mode} c2={c2} {border} inv={inv}")


@pytest.mark.parametrize("H,W,wb", [(1600, 8200, 64), (1200, 12000, 32), (3300, 4100, 64)])
def test_builtin_tiles(H, W, wb):
    """Images of 3 MiB of traffic and more take tiles by default: whole
    images against the oracle, in both modes, strides and pads too."""
    img = rand_img(H, W, 0.3, seed=H + W)
    for mode in ("masks", "full"):
        _, got = run_single(img, wb, mode=mode, stride_extra=3 if wb == 64 else 5)
        assert_same(got, expect(img, mode=mode), f"{H}x{W} B{wb} {mode}")


def test_translation_every_bit_offset():
    """A fixed pattern at every x offset across two 64-bit words and several
    rows: catches carry and direction mistakes."""
    rng = np.random.default_rng(1)
    pat = (rng.random((6, 7)) >= 0.5).astype(np.uint8)
    for wb in (32, 64):
        for dy in (0, 1, 5):
            for dx in range(0, 2 * wb + 2):
                img = np.ones((16, 3 * wb), np.uint8)
                img[dy:dy + 6, dx:dx + 7] = pat
                for border in ("white", "black"):
                    _, got = run_single(img, wb, border=border, mode="full")
                    assert_same(got, expect(img, border=border), f"dx={dx} dy={dy}")


def test_d4_symmetry():
    img = images.glyph_page(300, 513, seed=7, noise=0.01)
    for f in (np.fliplr, np.flipud, np.transpose):
        t = np.ascontiguousarray(f(img))
        _, a = run_single(img, 64)
        _, b = run_single(t, 64)
        assert_same(np.ascontiguousarray(f(a)), b, f.__name__)


def test_closed_forms_on_gpu():
    for (H, W) in ((1, 1), (2, 2), (5, 300), (300, 5), (64, 4096)):
        white = np.ones((H, W), np.uint8)
        black = np.zeros((H, W), np.uint8)
        assert run_single(white, 64)[1].sum() == 0
        frame = H * W if min(H, W) <= 2 else 2 * (H + W) - 4
        assert run_single(black, 64, border="white")[1].sum() == frame
        assert run_single(black, 64, border="black")[1].sum() == 0
    img = np.ones((40, 300), np.uint8)
    img[10:30, 100:250] = 0
    assert run_single(img, 32)[1].sum() == 2 * (20 + 150) - 4
