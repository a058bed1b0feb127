"""Pins for the oracle's fundamental-edge planes (section 4, Fig. 2) and
its threshold binarisation (section 7)."""
import itertools
import os

import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import BORDERS, _all_images, _read_grids

NAME_TO_PLANE = {"(a) Right": "right", "(b) Left": "left", "(c) Up": "up", "(d) Down": "down"}


def shifted_and_planes(img, border):
    """Section 4 with numpy arrays: each fundamental edge is the image
    shifted by one pixel ANDed with the mask (negative image, section 3)."""
    I = (np.asarray(img) != 0).astype(np.uint8)
    P = np.pad(I, 1, constant_values=1 if border == "white" else 0)
    M = 1 - P[1:-1, 1:-1]
    return np.stack([M & P[1:-1, :-2],    # left: image shifted right, pixel sees x-1
                     M & P[1:-1, 2:],     # right
                     M & P[:-2, 1:-1],    # up
                     M & P[2:, 1:-1]])    # down


def test_fig2_names_match_planes(golden_dir):
    """Each Fig. 2 pattern fires its own direction plane for every filling
    of its don't-care cells."""
    names, grids = _read_grids(os.path.join(golden_dir, "fig2_patterns.txt"))
    for name, g in zip(names, grids):
        plane = oracle.DIRECTIONS.index(NAME_TO_PLANE[name])
        cells = [(r, c) for r in range(3) for c in range(3) if g[r][c] in ("x", "X")]
        for bits in itertools.product((0, 1), repeat=len(cells)):
            img = np.array([[0 if v == "0" else 1 for v in row] for row in g], np.uint8)
            for (r, c), b in zip(cells, bits):
                img[r, c] = b
            assert oracle.fundamental_edges(img)[plane, 1, 1] == 1, (name, bits)


def test_single_white_neighbour_fires_one_plane(golden_dir):
    """Fig. 1 positions: with only neighbour k white around a black centre,
    exactly the plane of k fires (4 left, 8 right, 2 up, 6 down)."""
    _, (fig,) = _read_grids(os.path.join(golden_dir, "fig1_neighbours.txt"))
    pos = {int(fig[r][c]): (r, c) for r in range(3) for c in range(3) if fig[r][c] != "P"}
    want = {4: "left", 8: "right", 2: "up", 6: "down"}
    for k, (r, c) in pos.items():
        img = np.zeros((3, 3), np.uint8)
        img[r, c] = 1
        fired = oracle.fundamental_edges(img, border="black")[:, 1, 1]
        expect = np.zeros(4, np.uint8)
        if k in want:
            expect[oracle.DIRECTIONS.index(want[k])] = 1
        np.testing.assert_array_equal(fired, expect, err_msg=f"neighbour {k}")


@pytest.mark.parametrize("border", BORDERS)
@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (9, 1), (17, 33), (64, 65)])
def test_planes_match_shifted_ands_and_or_to_edge(shape, border):
    rng = np.random.default_rng(sum(shape))
    img = (rng.random(shape) >= 0.5).astype(np.uint8)
    f = oracle.fundamental_edges(img, border=border)
    np.testing.assert_array_equal(f, shifted_and_planes(img, border))
    np.testing.assert_array_equal(f.max(axis=0), oracle.edge(img, border=border))  # section 5


@pytest.mark.parametrize("shape", [(2, 3), (3, 3), (1, 8), (4, 3)])
def test_planes_exhaustive(shape):
    for border in BORDERS:
        for img in _all_images(*shape):
            np.testing.assert_array_equal(oracle.fundamental_edges(img, border=border),
                                          shifted_and_planes(img, border))


def test_planes_d4():
    rng = np.random.default_rng(4)
    img = (rng.random((23, 31)) >= 0.45).astype(np.uint8)
    L, R, U, D = range(4)
    f = oracle.fundamental_edges(img)
    g = oracle.fundamental_edges(np.ascontiguousarray(np.fliplr(img)))
    np.testing.assert_array_equal(g[[R, L, U, D]], f[:, :, ::-1])
    g = oracle.fundamental_edges(np.ascontiguousarray(np.flipud(img)))
    np.testing.assert_array_equal(g[[L, R, D, U]], f[:, ::-1, :])
    g = oracle.fundamental_edges(np.ascontiguousarray(img.T))
    np.testing.assert_array_equal(g[[U, D, L, R]], f.transpose(0, 2, 1))


def test_threshold_by_histogram_and_bounds():
    rng = np.random.default_rng(9)
    grey = rng.integers(0, 256, size=(37, 53), dtype=np.uint8)
    hist = np.bincount(grey.ravel(), minlength=256)
    above = np.concatenate([np.cumsum(hist[::-1])[::-1], [0]])   # pixels >= t, t = 0..256
    prev = None
    for t in range(0, 257):
        b = oracle.threshold(grey, t)
        assert b.sum() == above[t], t
        if prev is not None:
            assert not (b & ~prev.astype(bool)).any()          # monotone in t
            np.testing.assert_array_equal((prev != b), grey == t - 1)   # t-1 -> t flips value t-1
        prev = b
    assert oracle.threshold(grey, 0).all() and not oracle.threshold(grey, 256).any()
    with pytest.raises(ValueError):
        oracle.threshold(grey, 257)


# ---------------------------------------------------------------- peeling --
# One peel turns the current edge points white. A black pixel is an edge
# point exactly when a 4-neighbour is white, so after k peels a black pixel
# is left exactly when no white pixel (or white outside, under the white
# border) lies within taxicab distance k of it. On a rectangular grid the
# taxicab distance inside the image equals the distance in the plane, so the
# black-border case needs no path argument either.

CROSS = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]], bool)


def taxicab_to_white(img, border):
    """Taxicab distance from each pixel to the nearest white pixel (0 on
    white pixels), from scipy's exact city-block distance transform; a
    white border adds a white frame around the image. None when no white
    pixel exists at all."""
    from scipy import ndimage
    black = np.asarray(img) == 0
    if border == "white":
        black = np.pad(black, 1, constant_values=False)
    if black.all():
        return None
    d = ndimage.distance_transform_cdt(black, metric="taxicab")
    return d[1:-1, 1:-1] if border == "white" else d


@pytest.mark.parametrize("border", BORDERS)
@pytest.mark.parametrize("shape", [(1, 1), (1, 13), (13, 1), (9, 9), (24, 37), (40, 33)])
@pytest.mark.parametrize("q", [0.15, 0.5, 0.9])
def test_peel_by_taxicab_distance(shape, border, q):
    rng = np.random.default_rng(int(q * 100) + shape[0] * 97 + shape[1])
    img = (rng.random(shape) >= q).astype(np.uint8)      # q = black fraction
    d = taxicab_to_white(img, border)
    for k in range(0, 7):
        got = oracle.peel(img, k, border=border)
        lay = oracle.peel(img, k, border=border, edge_out=True)
        if d is None:       # all black under a black border: nothing ever peels
            assert not got.any() and not lay.any()
            continue
        np.testing.assert_array_equal(got, (d <= k).astype(np.uint8), err_msg=f"k={k}")
        np.testing.assert_array_equal(lay, (d == k + 1).astype(np.uint8), err_msg=f"k={k}")


@pytest.mark.parametrize("border", BORDERS)
def test_peel_equals_iterated_textbook_erosion(border):
    """k peels = k erosions of the black set by the 4-connected cross with
    the outside held at the border colour (scipy, one call per k)."""
    from scipy import ndimage
    rng = np.random.default_rng(12)
    img = (rng.random((31, 45)) >= 0.8).astype(np.uint8)
    black = img == 0
    for k in range(1, 6):
        er = ndimage.binary_erosion(black, structure=CROSS, iterations=k,
                                    border_value=0 if border == "white" else 1)
        np.testing.assert_array_equal(oracle.peel(img, k, border=border), (~er).astype(np.uint8))


def test_peel_rectangle_closed_form():
    """A filled w x h black rectangle on white shrinks by one pixel on every
    side per peel: (w - 2k)(h - 2k) pixels are left while both are positive,
    and the k-th layer holds the rest of the (w - 2k + 2)(h - 2k + 2) ring."""
    for (w, h) in [(1, 1), (2, 5), (7, 7), (11, 6), (20, 3)]:
        img = np.ones((h + 6, w + 6), np.uint8)
        img[3:3 + h, 3:3 + w] = 0
        for k in range(0, max(w, h) + 2):
            left = max(0, w - 2 * k) * max(0, h - 2 * k)
            assert int((oracle.peel(img, k) == 0).sum()) == left, (w, h, k)


def test_peel_zero_steps_and_layers():
    rng = np.random.default_rng(3)
    img = (rng.random((19, 27)) >= 0.7).astype(np.uint8)
    for border in BORDERS:
        np.testing.assert_array_equal(oracle.peel(img, 0, border=border), img)
        np.testing.assert_array_equal(oracle.peel(img, 0, border=border, edge_out=True),
                                      oracle.edge(img, border=border))
        for k in range(0, 5):   # the edge of the k-times peeled image is the (k+1)-th peel
            a, b = oracle.peel(img, k, border=border), oracle.peel(img, k + 1, border=border)
            np.testing.assert_array_equal(oracle.peel(img, k, border=border, edge_out=True),
                                          b & (1 - a))
            np.testing.assert_array_equal(oracle.peel(a, 2, border=border),
                                          oracle.peel(img, k + 2, border=border))
    with pytest.raises(ValueError):
        oracle.peel(img, -1)
