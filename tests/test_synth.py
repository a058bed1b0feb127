"""Packing and generator checks (CPU)."""
import numpy as np
import pytest

from synth import images, pack_rows, pad_bits_zero, row_words, unpack_rows


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("W", [1, 31, 32, 33, 63, 64, 65, 200])
def test_pack_roundtrip_and_layout(word_bits, W):
    rng = np.random.default_rng(W)
    img = (rng.random((5, W)) >= 0.5).astype(np.uint8)
    for stride in (None, row_words(W, word_bits) + 3):
        for pad in ("zero", "ones", "random"):
            words = pack_rows(img, word_bits, stride, pad=pad, seed=1)
            assert words.dtype == (np.uint32 if word_bits == 32 else np.uint64)
            np.testing.assert_array_equal(unpack_rows(words, W), img)
            if pad == "zero" or W % word_bits == 0:
                assert pad_bits_zero(words, W)
            elif pad == "ones":
                assert not pad_bits_zero(words, W)
    # explicit layout: pixel x of row y is bit x mod B of word y*S + x // B
    words = pack_rows(img, word_bits)
    for y in range(5):
        for x in range(W):
            w = int(words[y, x // word_bits])
            assert (w >> (x % word_bits)) & 1 == img[y, x]
    # same bytes as numpy.packbits(..., bitorder='little') per row
    np.testing.assert_array_equal(
        words.view(np.uint8)[:, :-(-W // 8)], np.packbits(img, axis=1, bitorder="little"))


def test_pad_bits_zero():
    img = np.ones((2, 40), np.uint8)
    assert pad_bits_zero(pack_rows(img, 32), 40)
    assert not pad_bits_zero(pack_rows(img, 32, pad="ones"), 40)
    # stride padding words are not inspected
    w = pack_rows(img, 32, stride_words=4)
    w[:, 3] = 0xFFFFFFFF
    assert pad_bits_zero(w, 40)


def test_generators_are_seeded_and_in_band():
    a, k = images.strokes_image(512, 512, seed=1)
    b, k2 = images.strokes_image(512, 512, seed=1)
    np.testing.assert_array_equal(a, b)
    assert k == k2 and 0.15 <= images.black_fraction(a) <= 0.25
    p = images.glyph_page(1024, 1536, seed=2)
    np.testing.assert_array_equal(p, images.glyph_page(1024, 1536, seed=2))
    assert 0.12 <= images.black_fraction(p) <= 0.28
    s = images.skeleton_page(1024, 1024, seed=4)
    assert 0.04 <= images.black_fraction(s) <= 0.16
    crops = images.glyph_crops(64, seed=3)
    assert all(24 <= c.shape[0] <= 256 and 24 <= c.shape[1] <= 256 for c in crops)
    assert 0.15 <= np.mean([images.black_fraction(c) for c in crops]) <= 0.45
    bern = images.bernoulli_image(512, 512, 0.3, seed=9)
    assert abs(images.black_fraction(bern) - 0.3) < 0.01


def test_skeleton_page_has_isolated_pixels():
    s = images.skeleton_page(512, 512, seed=4, isolated=1e-3)
    from scipy import ndimage
    K = (s == 0).astype(np.int32)
    n = ndimage.convolve(K, np.ones((3, 3), np.int32), mode="constant")
    assert ((K == 1) & (n == 1)).sum() > 0
