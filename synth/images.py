"""Seeded synthetic binary images shaped like the paper's workloads.

The paper measures on images of Arabic letters (50x50 to 300x300) and on a
thresholded photograph (sections 7-8, Figs. 6-11). Those images are not
available, so thick-stroke glyphs on a white background stand in for them:
single images of random strokes, pages tiled from a seeded glyph alphabet,
small glyph crops, 1-pixel skeleton lines, and Bernoulli noise.

Every function returns a uint8 array with 0 = black and 1 = white and is a
pure function of its arguments (seeded ``numpy.random.Generator``). Nothing
here computes edges.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------- drawing ----

def _draw_segment(canvas: np.ndarray, x0: float, y0: float, x1: float, y1: float,
                  width: float) -> None:
    """Paint black every pixel centre within width/2 of the segment."""
    H, W = canvas.shape
    r = width / 2.0
    xa = max(0, int(math.floor(min(x0, x1) - r)))
    xb = min(W, int(math.ceil(max(x0, x1) + r)) + 1)
    ya = max(0, int(math.floor(min(y0, y1) - r)))
    yb = min(H, int(math.ceil(max(y0, y1) + r)) + 1)
    if xa >= xb or ya >= yb:
        return
    yy, xx = np.mgrid[ya:yb, xa:xb].astype(np.float32)
    dx, dy = x1 - x0, y1 - y0
    l2 = dx * dx + dy * dy
    if l2 == 0.0:
        t = np.zeros_like(xx)
    else:
        t = np.clip(((xx - x0) * dx + (yy - y0) * dy) / l2, 0.0, 1.0)
    d2 = (xx - (x0 + t * dx)) ** 2 + (yy - (y0 + t * dy)) ** 2
    canvas[ya:yb, xa:xb][d2 <= r * r] = 0


def _draw_ellipse_outline(canvas: np.ndarray, cx: float, cy: float, a: float, b: float,
                          width: float) -> None:
    """Paint black a ring of about `width` pixels along an axis-aligned ellipse."""
    H, W = canvas.shape
    r = width / 2.0
    xa = max(0, int(math.floor(cx - a - r)))
    xb = min(W, int(math.ceil(cx + a + r)) + 1)
    ya = max(0, int(math.floor(cy - b - r)))
    yb = min(H, int(math.ceil(cy + b + r)) + 1)
    if xa >= xb or ya >= yb:
        return
    yy, xx = np.mgrid[ya:yb, xa:xb].astype(np.float32)
    rho = np.sqrt(((xx - cx) / a) ** 2 + ((yy - cy) / b) ** 2)
    canvas[ya:yb, xa:xb][np.abs(rho - 1.0) * min(a, b) <= r] = 0


def _draw_line_1px(canvas: np.ndarray, x0: int, y0: int, x1: int, y1: int) -> None:
    """Bresenham's line: an 8-connected black line one pixel wide."""
    H, W = canvas.shape
    dx, dy = abs(x1 - x0), -abs(y1 - y0)
    sx = 1 if x0 < x1 else -1
    sy = 1 if y0 < y1 else -1
    err = dx + dy
    while True:
        if 0 <= x0 < W and 0 <= y0 < H:
            canvas[y0, x0] = 0
        if x0 == x1 and y0 == y1:
            return
        e2 = 2 * err
        if e2 >= dy:
            err += dy
            x0 += sx
        if e2 <= dx:
            err += dx
            y0 += sy


def black_fraction(img: np.ndarray) -> float:
    return float((np.asarray(img) == 0).mean()) if np.asarray(img).size else 0.0


# ------------------------------------------------------ single-image shapes --

def strokes_image(height: int = 512, width: int = 512, seed: int = 1, n_shapes: int = 40,
                  stroke=(3, 12), band=(0.15, 0.25), max_redraws: int = 64):
    """Random thick polylines and ellipse outlines, black on white.

    Returns ``(img, k)``: the first draw with seed ``seed + k`` whose black
    fraction lies in ``band``.
    """
    for k in range(max_redraws):
        rng = np.random.default_rng(seed + k)
        img = np.ones((height, width), np.uint8)
        for _ in range(n_shapes):
            w = float(rng.integers(stroke[0], stroke[1] + 1))
            if rng.random() < 0.5:
                nv = int(rng.integers(2, 7))
                x, y = rng.uniform(0, width), rng.uniform(0, height)
                for _ in range(nv - 1):
                    ang = rng.uniform(0, 2 * math.pi)
                    step = rng.uniform(0.04, 0.2) * min(height, width)
                    nx, ny = x + step * math.cos(ang), y + step * math.sin(ang)
                    _draw_segment(img, x, y, nx, ny, w)
                    x, y = nx, ny
            else:
                s = min(height, width)
                a, b = rng.uniform(0.02, 0.12) * s, rng.uniform(0.02, 0.12) * s
                _draw_ellipse_outline(img, rng.uniform(0, width), rng.uniform(0, height),
                                      max(a, 2.0), max(b, 2.0), w)
        if band[0] <= black_fraction(img) <= band[1]:
            return img, k
    raise RuntimeError("no draw fell inside the black-fraction band")


def bernoulli_image(height: int, width: int, q: float, seed: int) -> np.ndarray:
    """Each pixel independently black with probability q."""
    rng = np.random.default_rng(seed)
    return (rng.random((height, width), dtype=np.float32) >= q).astype(np.uint8)


# --------------------------------------------------------- glyph alphabets --

def glyph_alphabet(rng: np.random.Generator, n: int = 256, size: int = 96,
                   strokes=(1, 6), stroke=(2, 10), thin_lines=(0, 0)) -> np.ndarray:
    """n square glyphs, each 1-6 thick polyline strokes (optionally plus
    1-pixel Bresenham lines), black on white. Shape (n, size, size)."""
    out = np.ones((n, size, size), np.uint8)
    m = 0.12 * size
    for g in range(n):
        c = out[g]
        for _ in range(int(rng.integers(strokes[0], strokes[1] + 1))):
            w = float(rng.integers(stroke[0], stroke[1] + 1))
            nv = int(rng.integers(2, 5))
            pts = rng.uniform(m, size - m, size=(nv, 2))
            for i in range(nv - 1):
                _draw_segment(c, pts[i, 0], pts[i, 1], pts[i + 1, 0], pts[i + 1, 1], w)
        for _ in range(int(rng.integers(thin_lines[0], thin_lines[1] + 1))):
            p = rng.integers(int(m), int(size - m), size=4)
            _draw_line_1px(c, int(p[0]), int(p[1]), int(p[2]), int(p[3]))
    return out


def _tile_page(rng: np.random.Generator, height: int, width: int, alphabet: np.ndarray,
               box=(48, 96), gap=(2, 12)) -> np.ndarray:
    """Lay glyphs from `alphabet` in text lines: each line has a height in
    `box`, each glyph box a width in `box`, separated by small white gaps."""
    n, gs, _ = alphabet.shape
    page = np.ones((height, width), np.uint8)
    y = int(rng.integers(0, gap[1] + 1))
    while y < height:
        lh = int(rng.integers(box[0], box[1] + 1))
        x = int(rng.integers(0, gap[1] + 1))
        while x < width:
            gw = int(rng.integers(box[0], box[1] + 1))
            gi = int(rng.integers(0, n))
            h = min(lh, height - y, gs)
            w = min(gw, width - x, gs)
            page[y:y + h, x:x + w] = alphabet[gi, :h, :w]
            x += gw + int(rng.integers(gap[0], gap[1] + 1))
        y += lh + int(rng.integers(gap[0], gap[1] + 1))
    return page


def salt_and_pepper(img: np.ndarray, p: float, rng: np.random.Generator) -> np.ndarray:
    """Flip each pixel with probability p (in place; also returned)."""
    flat = img.reshape(-1)
    n = int(rng.binomial(flat.size, p)) if flat.size else 0
    if n:
        idx = rng.integers(0, flat.size, size=n)
        flat[idx] = 1 - flat[idx]
    return img


def glyph_page(height: int = 8192, width: int = 8192, seed: int = 2,
               noise: float = 0.005) -> np.ndarray:
    """A page of glyph-like strokes (width 2-10 px, about 20% black) with
    salt-and-pepper noise that flips a fraction `noise` of the pixels."""
    rng = np.random.default_rng(seed)
    alphabet = glyph_alphabet(rng, n=256, size=96, strokes=(3, 6), stroke=(2, 10))
    page = _tile_page(rng, height, width, alphabet)
    if noise:
        salt_and_pepper(page, noise, rng)
    return page


def skeleton_page(height: int = 16384, width: int = 16384, seed: int = 4,
                  isolated: float = 1e-5) -> np.ndarray:
    """1-pixel Bresenham lines plus thick strokes (width 3-12), about 10%
    black, plus isolated black pixels at density `isolated` whose eight
    neighbours are white, so line end points and lone pixels occur."""
    rng = np.random.default_rng(seed)
    alphabet = glyph_alphabet(rng, n=256, size=96, strokes=(1, 2), stroke=(3, 12),
                              thin_lines=(1, 4))
    page = _tile_page(rng, height, width, alphabet)
    n = int(rng.binomial(height * width, isolated)) if height * width else 0
    if n and height >= 3 and width >= 3:
        ys = rng.integers(1, height - 1, size=n)
        xs = rng.integers(1, width - 1, size=n)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                page[ys + dy, xs + dx] = 1
        page[ys, xs] = 0
    return page


def glyph_crops(n: int = 4096, seed: int = 3, side=(24, 256), strokes=(1, 6),
                stroke_frac=(0.08, 0.15)) -> list:
    """n independent glyph crops: H and W log-uniform in `side`, 1-6 thick
    strokes of width 8-15% of the short side (about 30% black)."""
    rng = np.random.default_rng(seed)
    lo, hi = math.log(side[0]), math.log(side[1])
    crops = []
    for _ in range(n):
        H = int(round(math.exp(rng.uniform(lo, hi))))
        W = int(round(math.exp(rng.uniform(lo, hi))))
        c = np.ones((H, W), np.uint8)
        s = min(H, W)
        for _ in range(int(rng.integers(strokes[0], strokes[1] + 1))):
            w = max(1.0, rng.uniform(*stroke_frac) * s)
            nv = int(rng.integers(2, 5))
            xs = rng.uniform(0, W, size=nv)
            ys = rng.uniform(0, H, size=nv)
            for i in range(nv - 1):
                _draw_segment(c, xs[i], ys[i], xs[i + 1], ys[i + 1], w)
        crops.append(c)
    return crops


def serving_pool(n: int = 64, seed: int = 5, side=(64, 4096), q: float = 0.3) -> list:
    """Request images: H and W log-uniform in `side`; half glyph pages, half
    Bernoulli(q) black noise. Returns a list of (img, kind)."""
    rng = np.random.default_rng(seed)
    lo, hi = math.log(side[0]), math.log(side[1])
    pool = []
    for i in range(n):
        H = int(round(math.exp(rng.uniform(lo, hi))))
        W = int(round(math.exp(rng.uniform(lo, hi))))
        sub = int(rng.integers(0, 2**31))
        if i % 2 == 0:
            pool.append((glyph_page(H, W, seed=sub, noise=0.0), "glyph"))
        else:
            pool.append((bernoulli_image(H, W, q, seed=sub), "bernoulli"))
    return pool


def log_uniform_sides(rng: np.random.Generator, n: int, side) -> np.ndarray:
    lo, hi = math.log(side[0]), math.log(side[1])
    return np.rint(np.exp(rng.uniform(lo, hi, size=n))).astype(np.int64)


def grey_image(height: int, width: int, seed: int, blobs: int = 24) -> np.ndarray:
    """A grey uint8 image standing in for the photograph of section 7:
    a smooth field of random Gaussian blobs over a gradient, plus noise.
    (Grey values are not binary; threshold them first.)"""
    rng = np.random.default_rng(seed)
    yy = np.linspace(0.0, 1.0, height, dtype=np.float32)[:, None]
    xx = np.linspace(0.0, 1.0, width, dtype=np.float32)[None, :]
    f = 0.3 * xx + 0.2 * yy
    for _ in range(blobs):
        cy, cx = rng.uniform(0, 1, size=2)
        r = rng.uniform(0.02, 0.2)
        f = f + rng.uniform(-0.6, 0.6) * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * r * r))
    f = f + rng.normal(0.0, 0.03, size=(height, width)).astype(np.float32)
    lo, hi = float(f.min()), float(f.max())
    return np.clip((f - lo) / max(hi - lo, 1e-6) * 255.0, 0, 255).astype(np.uint8)
