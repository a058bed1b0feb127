"""CPU oracle for binary-image edge detection by the method of masks.

TEST INFRASTRUCTURE. Only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg may import this package. The GPU library never imports,
links or calls it, and it imports nothing from the GPU library.

The arithmetic lives in ``edge_oracle.c`` (the per-pixel scan of section 1 of
the paper, on a byte image). This module only compiles it with the host C
compiler and marshals numpy arrays to it.

Parity status: every function here is pinned by the CPU tests in
``tests/test_oracle_pins.py`` (Fig. 1 and Fig. 2 fixtures, textbook
morphology, the paper's literal three-stage construction, exhaustive tiny
images, closed forms and invariants) and ``tests/test_oracle_pins_next.py``
(direction planes, threshold, peeling against the taxicab distance
transform and iterated textbook erosion).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "edge_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CLAUSE1 = 1  # black with >= 1 white 4-neighbour (section 1)
CLAUSE2 = 2  # black with <= 1 black 8-neighbour (section 1)

_BORDER_PIXEL = {"white": 1, "black": 0}

_lib = None


def build() -> str:
    """Compile edge_oracle.c into liboracle.so with the host C compiler."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    argt = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_edge_image.argtypes = argt
    lib.oracle_edge_image.restype = ctypes.c_int
    lib.oracle_edge_stack.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64] + argt[2:]
    lib.oracle_edge_stack.restype = ctypes.c_int
    lib.oracle_fundamental_edges.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_int64, ctypes.c_int]
    lib.oracle_fundamental_edges.restype = ctypes.c_int
    lib.oracle_threshold.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_int]
    lib.oracle_threshold.restype = ctypes.c_int
    lib.oracle_peel.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_peel.restype = ctypes.c_int
    _lib = lib
    return lib


def _as_bytes(img: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(img)
    if a.dtype != np.uint8:
        a = (a != 0).astype(np.uint8)
    return a


def edge(img: np.ndarray, border: str = "white", clauses: int = CLAUSE1,
         invert: bool = False) -> np.ndarray:
    """Edge map of an (H, W) byte image; 0 = black, nonzero = white.

    Returns an (H, W) uint8 array, 1 = edge point (0 = edge when ``invert``).
    ``clauses`` selects clause 1 (plain), clause 1 | clause 2 (full
    definition) or clause 2 alone, per the definition in section 1.
    """
    a = _as_bytes(img)
    if a.ndim != 2:
        raise ValueError("expected a 2-D image")
    H, W = a.shape
    out = np.empty((H, W), dtype=np.uint8)
    rc = _load().oracle_edge_image(a.ctypes.data, out.ctypes.data, H, W,
                                   _BORDER_PIXEL[border], int(clauses), int(bool(invert)))
    if rc != 0:
        raise ValueError(f"oracle_edge_image rejected its arguments ({rc})")
    return out


def edge_stack(imgs: np.ndarray, border: str = "white", clauses: int = CLAUSE1,
               invert: bool = False) -> np.ndarray:
    """Edge maps of an (n, H, W) stack of equally shaped byte images."""
    a = _as_bytes(imgs)
    if a.ndim != 3:
        raise ValueError("expected an (n, H, W) stack")
    n, H, W = a.shape
    out = np.empty_like(a)
    rc = _load().oracle_edge_stack(a.ctypes.data, out.ctypes.data, n, H, W,
                                   _BORDER_PIXEL[border], int(clauses), int(bool(invert)))
    if rc != 0:
        raise ValueError(f"oracle_edge_stack rejected its arguments ({rc})")
    return out


DIRECTIONS = ("left", "right", "up", "down")


def fundamental_edges(img: np.ndarray, border: str = "white") -> np.ndarray:
    """The four fundamental edges of section 4 of an (H, W) byte image:
    a (4, H, W) uint8 array, planes ordered left, right, up, down."""
    a = _as_bytes(img)
    if a.ndim != 2:
        raise ValueError("expected a 2-D image")
    H, W = a.shape
    out = np.empty((4, H, W), dtype=np.uint8)
    rc = _load().oracle_fundamental_edges(a.ctypes.data, out.ctypes.data, H, W,
                                          _BORDER_PIXEL[border])
    if rc != 0:
        raise ValueError(f"oracle_fundamental_edges rejected its arguments ({rc})")
    return out


def threshold(grey: np.ndarray, t: int) -> np.ndarray:
    """Binary image of a uint8 grey image: 1 (white) where grey >= t."""
    g = np.ascontiguousarray(grey, dtype=np.uint8)
    if g.ndim != 2:
        raise ValueError("expected a 2-D image")
    H, W = g.shape
    out = np.empty((H, W), dtype=np.uint8)
    rc = _load().oracle_threshold(g.ctypes.data, out.ctypes.data, H, W, int(t))
    if rc != 0:
        raise ValueError(f"oracle_threshold rejected its arguments ({rc})")
    return out


def peel(img: np.ndarray, iterations: int, border: str = "white",
         edge_out: bool = False) -> np.ndarray:
    """The (H, W) byte image after `iterations` peels (each peel turns the
    current edge points white), or with ``edge_out`` the edge map of that
    image. uint8, 1 = white (image) or 1 = edge (edge map)."""
    a = _as_bytes(img)
    if a.ndim != 2:
        raise ValueError("expected a 2-D image")
    H, W = a.shape
    out = np.empty((H, W), dtype=np.uint8)
    rc = _load().oracle_peel(a.ctypes.data, out.ctypes.data, H, W, _BORDER_PIXEL[border],
                             int(iterations), int(bool(edge_out)))
    if rc != 0:
        raise ValueError(f"oracle_peel rejected its arguments ({rc})")
    return out


def edge_rows(img_rows: np.ndarray, first_row: int, rows: np.ndarray, height: int,
              border: str = "white", clauses: int = CLAUSE1, invert: bool = False) -> np.ndarray:
    """Edge map of selected rows of a tall image, from a window of it.

    ``img_rows`` holds image rows ``first_row .. first_row + len - 1`` of an
    image with ``height`` rows. Each requested row must have its upper and
    lower neighbour rows inside the window (or be the image's top or bottom
    row). Each output row is the oracle run on the three-row window around
    it, whose middle row sees exactly the neighbours it sees in the whole
    image.
    """
    a = _as_bytes(img_rows)
    out = []
    for y in rows:
        lo = max(0, y - 1)
        hi = min(height, y + 2)
        if lo < first_row or hi > first_row + a.shape[0]:
            raise ValueError(f"row {y} needs rows {lo}..{hi - 1} in the window")
        win = a[lo - first_row:hi - first_row]
        e = edge(win, border=border, clauses=clauses, invert=invert)
        out.append(e[y - lo])
    return np.stack(out) if out else np.zeros((0, a.shape[1]), np.uint8)
