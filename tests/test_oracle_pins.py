"""Pins for the CPU oracle: each test checks it against something other than
itself - the paper's figures, textbook morphology from scipy, the paper's own
three-stage construction, brute force over every tiny image, closed forms and
invariants of the definition in section 1.

A plausible mistake in the oracle (a dropped neighbour, a diagonal used in
place of a 4-neighbour, a sign flip that marks white points, a swapped row and
column index, a wrong border value) fails at least one test here.
"""
import itertools
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle

CROSS = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]], bool)
RING8 = np.array([[1, 1, 1], [1, 0, 1], [1, 1, 1]], np.int32)
BORDERS = ("white", "black")


# ------------------------------------------------------------ fixtures ----

def _read_grids(path):
    """Parse a fixture of 3x3 grids; '# name:' lines start a new grid."""
    grids, names, cur, name = [], [], [], None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("# name:"):
                name = line.split(":", 1)[1].strip()
                continue
            if not line or line.startswith("#"):
                continue
            cur.append(line.split())
            if len(cur) == 3:
                grids.append(cur)
                names.append(name)
                cur = []
    return names, grids


def _neighbourhood(center, values):
    """3x3 image with `center` and the 8 ring pixels (row-major, centre skipped)."""
    img = np.empty((3, 3), np.uint8)
    it = iter(values)
    for r in range(3):
        for c in range(3):
            img[r, c] = center if (r, c) == (1, 1) else next(it)
    return img


# ---------------------------------------------- textbook cross-checks ----

def _black(img):
    return np.asarray(img) == 0


def morph_edge(img, border):
    """Black pixels not in the erosion of the black set by the 4-connected
    cross: the textbook inner boundary. Outside pixels are black for the
    black border (border_value=1) and white otherwise."""
    K = _black(img)
    if K.ndim == 3:
        st = CROSS[None]
    else:
        st = CROSS
    er = ndimage.binary_erosion(K, structure=st, border_value=1 if border == "black" else 0)
    return (K & ~er).astype(np.uint8)


def count_black8(img, border):
    """Number of black pixels among the eight neighbours (outside counted
    by the border colour)."""
    K = _black(img).astype(np.int32)
    w = RING8[None] if K.ndim == 3 else RING8
    return ndimage.convolve(K, w, mode="constant", cval=1 if border == "black" else 0)


def clause2_ref(img, border):
    return (_black(img) & (count_black8(img, border) <= 1)).astype(np.uint8)


def three_stage(img, border):
    """The paper's method on whole arrays: mask = negative image (section 3),
    four fundamental edges = image shifted one pixel ANDed with the mask
    (section 4), edge = OR of the four (section 5, display inversion off)."""
    I = (np.asarray(img) != 0).astype(np.uint8)
    P = np.pad(I, 1, constant_values=1 if border == "white" else 0)
    M = 1 - P
    core = (slice(1, -1), slice(1, -1))
    left = M[core] & P[1:-1, :-2]    # image shifted right by one: sees x-1
    right = M[core] & P[1:-1, 2:]    # image shifted left by one: sees x+1
    up = M[core] & P[:-2, 1:-1]      # image shifted down by one: sees y-1
    down = M[core] & P[2:, 1:-1]     # image shifted up by one: sees y+1
    return left | right | up | down


# ------------------------------------------------------------- figures ----

def test_fig1_four_neighbours_are_2_4_6_8(golden_dir):
    """Fig. 1 numbering + the Boolean function of section 1: with a black
    centre and only neighbour k white, the centre is an edge iff k is one of
    2, 4, 6, 8. Positions come from the figure, not from the oracle."""
    _, grids = _read_grids(os.path.join(golden_dir, "fig1_neighbours.txt"))
    (fig,) = grids
    pos = {}
    for r in range(3):
        for c in range(3):
            if fig[r][c] != "P":
                pos[int(fig[r][c])] = (r, c)
    assert sorted(pos) == list(range(1, 9))
    for border in BORDERS:
        for k, (r, c) in pos.items():
            img = np.zeros((3, 3), np.uint8)
            img[r, c] = 1
            e = oracle.edge(img, border=border)
            assert e[1, 1] == (1 if k in (2, 4, 6, 8) else 0), (k, border)
            # clause 2: a black centre with exactly one black neighbour (k)
            img2 = np.ones((3, 3), np.uint8)
            img2[1, 1] = 0
            img2[r, c] = 0
            assert oracle.edge(img2, border=border, clauses=oracle.CLAUSE2)[1, 1] == 1
            # two black neighbours: not clause 2
            other = pos[(k % 8) + 1]
            img2[other] = 0
            assert oracle.edge(img2, border=border, clauses=oracle.CLAUSE2)[1, 1] == 0


def test_fig2_patterns_are_edge_points(golden_dir):
    """Every filling of the don't-care cells of each Fig. 2 pattern gives an
    edge point at the centre."""
    names, grids = _read_grids(os.path.join(golden_dir, "fig2_patterns.txt"))
    assert len(grids) == 4
    for name, g in zip(names, grids):
        cells = [(r, c) for r in range(3) for c in range(3) if g[r][c] in ("x", "X")]
        assert g[1][1] == "0"
        for bits in itertools.product((0, 1), repeat=len(cells)):
            img = np.array([[0 if v == "0" else 1 for v in row] for row in g], np.uint8)
            for (r, c), b in zip(cells, bits):
                img[r, c] = b
            assert oracle.edge(img)[1, 1] == 1, (name, bits)


def test_fig2_patterns_cover_every_edge_point(golden_dir):
    """Section 1: the four types of Fig. 2 are all the edge points. Over all
    256 rings around a black centre, the oracle marks the centre iff the ring
    matches one of the patterns; a white centre is never marked."""
    _, grids = _read_grids(os.path.join(golden_dir, "fig2_patterns.txt"))

    def matches(img, g):
        return all(g[r][c] in ("x", "X") or int(g[r][c]) == img[r, c]
                   for r in range(3) for c in range(3))

    n_edges = 0
    for ring in itertools.product((0, 1), repeat=8):
        img = _neighbourhood(0, ring)
        want = int(any(matches(img, g) for g in grids))
        assert oracle.edge(img, border="black")[1, 1] == want, ring
        n_edges += want
        assert oracle.edge(_neighbourhood(1, ring))[1, 1] == 0
    # the four 4-neighbours are free in 16 ways, of which one (all black) is no edge
    assert n_edges == 256 - 16


# ------------------------------------------------ library / brute force ----

@pytest.mark.parametrize("border", BORDERS)
@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (2, 2), (3, 5), (17, 33),
                                   (64, 65), (100, 31)])
@pytest.mark.parametrize("q", [0.1, 0.5, 0.9])
def test_matches_textbook_morphology(shape, border, q):
    rng = np.random.default_rng(hash((shape, border, q)) & 0xFFFF)
    img = (rng.random(shape) >= q).astype(np.uint8)
    e = oracle.edge(img, border=border)
    np.testing.assert_array_equal(e, morph_edge(img, border))
    np.testing.assert_array_equal(e, three_stage(img, border))
    np.testing.assert_array_equal(
        oracle.edge(img, border=border, clauses=oracle.CLAUSE2), clause2_ref(img, border))


def _all_images(H, W):
    n = H * W
    codes = np.arange(2 ** n, dtype=np.int64)
    bits = (codes[:, None] >> np.arange(n)) & 1
    return bits.astype(np.uint8).reshape(-1, H, W)


EXHAUSTIVE_SHAPES = [(H, W) for H in range(1, 13) for W in range(1, 13) if H * W <= 12] + \
                    [(4, 4), (2, 8), (8, 2), (1, 16), (16, 1)]


@pytest.mark.parametrize("shape", EXHAUSTIVE_SHAPES)
def test_exhaustive_tiny_images(shape):
    """Every image with up to 12 pixels (and every 16-pixel image of five
    shapes), both borders, all three clause selections, against scipy."""
    H, W = shape
    imgs = _all_images(H, W)
    for border in BORDERS:
        c1 = morph_edge(imgs, border)
        c2 = clause2_ref(imgs, border)
        np.testing.assert_array_equal(oracle.edge_stack(imgs, border=border), c1)
        np.testing.assert_array_equal(
            oracle.edge_stack(imgs, border=border, clauses=oracle.CLAUSE2), c2)
        full = oracle.edge_stack(imgs, border=border, clauses=oracle.CLAUSE1 | oracle.CLAUSE2)
        np.testing.assert_array_equal(full, c1 | c2)
        # clause 2 never adds a pixel to clause 1 (section 1: "other cases are
        # included in these cases"), under either border
        np.testing.assert_array_equal(full, c1)


# --------------------------------------------------------- closed forms ----

@pytest.mark.parametrize("H,W", [(1, 1), (1, 9), (9, 1), (2, 2), (5, 8), (64, 33)])
def test_closed_forms_whole_image(H, W):
    white = np.ones((H, W), np.uint8)
    black = np.zeros((H, W), np.uint8)
    for border in BORDERS:
        assert oracle.edge(white, border=border).sum() == 0
    frame = H * W if min(H, W) <= 2 else 2 * (W + H) - 4
    assert oracle.edge(black, border="white").sum() == frame
    assert oracle.edge(black, border="black").sum() == 0


@pytest.mark.parametrize("w,h", [(1, 1), (1, 5), (5, 1), (2, 2), (2, 7), (9, 4), (30, 30)])
def test_rectangle_edge_count(w, h):
    img = np.ones((h + 10, w + 12), np.uint8)
    img[5:5 + h, 6:6 + w] = 0
    want = w * h if min(w, h) == 1 else 2 * (w + h) - 4
    for border in BORDERS:
        e = oracle.edge(img, border=border)
        assert e.sum() == want
        assert oracle.edge(img, border=border, clauses=3).sum() == want


def test_lone_pixel_and_checkerboard():
    img = np.ones((9, 11), np.uint8)
    img[4, 3] = 0
    assert oracle.edge(img).sum() == 1 and oracle.edge(img)[4, 3] == 1
    assert oracle.edge(img, clauses=oracle.CLAUSE2)[4, 3] == 1
    cb = ((np.indices((13, 14)).sum(0)) % 2).astype(np.uint8)
    for border in BORDERS:
        np.testing.assert_array_equal(oracle.edge(cb, border=border), (cb == 0).astype(np.uint8))


def test_clause2_closed_forms():
    """Clause 2 alone: segment end points, 2x2 block, line interiors."""
    for seg in ("h", "v", "d"):
        for n in (2, 3, 10):
            img = np.ones((16, 16), np.uint8)
            for i in range(n):
                y, x = {"h": (5, 2 + i), "v": (2 + i, 5), "d": (2 + i, 2 + i)}[seg]
                img[y, x] = 0
            c2 = oracle.edge(img, clauses=oracle.CLAUSE2)
            assert c2.sum() == 2, (seg, n)
            ends = {"h": [(5, 2), (5, 1 + n)], "v": [(2, 5), (1 + n, 5)],
                    "d": [(2, 2), (1 + n, 1 + n)]}[seg]
            for y, x in ends:
                assert c2[y, x] == 1
    blk = np.ones((8, 8), np.uint8)
    blk[3:5, 3:5] = 0
    assert oracle.edge(blk, clauses=oracle.CLAUSE2).sum() == 0


def test_one_row_image_black_border():
    """With a black border every neighbour of a 1-row all-black image is
    black, so neither clause fires; with a white border all pixels fire."""
    img = np.zeros((1, 5), np.uint8)
    assert oracle.edge(img, border="black", clauses=3).sum() == 0
    assert oracle.edge(img, border="white", clauses=3).sum() == 5


# ----------------------------------------------------------- invariants ----

@pytest.mark.parametrize("border", BORDERS)
def test_invariants(border):
    rng = np.random.default_rng(7)
    img = (rng.random((61, 47)) >= 0.4).astype(np.uint8)
    e = oracle.edge(img, border=border)
    c2 = oracle.edge(img, border=border, clauses=oracle.CLAUSE2)
    full = oracle.edge(img, border=border, clauses=3)
    assert not (e & img).any()                      # edges are black pixels
    np.testing.assert_array_equal(full, e)          # clause 2 is subsumed
    assert not (c2 & ~e.astype(bool)).any()         # clause-2 set within E
    np.testing.assert_array_equal(oracle.edge(img, border=border, invert=True), 1 - e)
    # D4 equivariance: flips and transposition commute with the detector
    for f in (np.fliplr, np.flipud, np.transpose, lambda a: np.rot90(a, 1)):
        np.testing.assert_array_equal(oracle.edge(np.ascontiguousarray(f(img)), border=border),
                                      f(e))
        np.testing.assert_array_equal(
            oracle.edge(np.ascontiguousarray(f(img)), border=border, clauses=2), f(c2))


def test_translation():
    """A fixed pattern placed at every offset gives the shifted edge map."""
    rng = np.random.default_rng(11)
    pat = (rng.random((5, 6)) >= 0.5).astype(np.uint8)
    pat[0, :] = pat[-1, :] = 1
    pat[:, 0] = pat[:, -1] = 1
    base = oracle.edge(pat)
    for dy in range(0, 4):
        for dx in range(0, 70):
            img = np.ones((12, 80), np.uint8)
            img[dy:dy + 5, dx:dx + 6] = pat
            e = oracle.edge(img)
            assert e.sum() == base.sum()
            np.testing.assert_array_equal(e[dy:dy + 5, dx:dx + 6], base)


def test_bernoulli_edge_density():
    """Interior pixels of a Bernoulli(q) image are edges with probability
    q (1 - q^4); clause-2 points with q [(1-q)^8 + 8 q (1-q)^7]."""
    q = 0.3
    rng = np.random.default_rng(5)
    img = (rng.random((1024, 1024)) >= q).astype(np.uint8)
    e = oracle.edge(img)[1:-1, 1:-1]
    c2 = oracle.edge(img, clauses=2)[1:-1, 1:-1]
    n = e.size
    for got, p in ((e.mean(), q * (1 - q ** 4)),
                   (c2.mean(), q * ((1 - q) ** 8 + 8 * q * (1 - q) ** 7))):
        sd = np.sqrt(p * (1 - p) / n)
        assert abs(got - p) < 5 * sd, (got, p)


def test_edge_rows_window_matches_whole_image():
    rng = np.random.default_rng(3)
    img = (rng.random((40, 70)) >= 0.5).astype(np.uint8)
    for clauses in (1, 2, 3):
        whole = oracle.edge(img, clauses=clauses)
        rows = np.array([0, 1, 17, 38, 39])
        np.testing.assert_array_equal(
            oracle.edge_rows(img, 0, rows, 40, clauses=clauses), whole[rows])
        np.testing.assert_array_equal(
            oracle.edge_rows(img[16:19], 16, np.array([17]), 40, clauses=clauses), whole[[17]])


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.edge(np.ones((3, 3, 3), np.uint8))
    with pytest.raises(ValueError):
        oracle.edge(np.ones((3, 3), np.uint8), clauses=4)
    assert oracle.edge(np.ones((0, 5), np.uint8)).shape == (0, 5)
