"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/edge_masks.h, and rejects bad arguments on the host
before any HIP call. The pointers passed here are never dereferenced: every
call below returns from argument validation."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1401_5245_amd import _abi
from paper_1401_5245_amd.batch import DESC_DTYPE

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "edge_masks.h")

lib = _abi.load()
OK, INVALID, ALIGN, ALIAS, WS = (_abi.EDGE_OK, _abi.EDGE_ERR_INVALID, _abi.EDGE_ERR_ALIGN,
                                 _abi.EDGE_ERR_ALIAS, _abi.EDGE_ERR_WORKSPACE)
A, B = 0x10000000, 0x20000000  # fake, 256-byte aligned, far apart


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(edge_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 14, names
    for n in names:
        assert hasattr(lib, n), n
        assert n in _abi._SIGNATURES, f"binding lacks {n}"


def test_version_and_strings():
    assert lib.edge_abi_version() == 2
    for s in (OK, INVALID, ALIGN, ALIAS, _abi.EDGE_ERR_HIP, WS, _abi.EDGE_ERR_UNSUPPORTED):
        assert lib.edge_status_string(s)
    assert lib.edge_status_string(-99) == b"unknown status"
    assert lib.edge_last_hip_error() == 0


def masks(inp=A, out=B, H=4, W=100, S=4, wb=32, border=0):
    return lib.edge_masks(inp, out, H, W, S, wb, border, None)


def launch(inp=A, out=B, H=4, W=100, S=4, wb=32, border=0, mode=0, flags=0, cfg=None):
    return lib.edge_image_launch(inp, out, H, W, S, wb, border, mode, flags, cfg, None)


@pytest.mark.parametrize("kw,want", [
    (dict(wb=16), INVALID), (dict(wb=0), INVALID), (dict(border=2), INVALID),
    (dict(H=-1), INVALID), (dict(W=-5), INVALID), (dict(S=3), INVALID),
    (dict(inp=None), INVALID), (dict(out=None), INVALID),
    (dict(inp=A + 2), ALIGN), (dict(out=B + 4, wb=64, S=2), ALIGN),
    (dict(out=A + 16), ALIAS), (dict(out=A - 4 * 15), ALIAS),
    (dict(H=1 << 31), INVALID), (dict(H=_abi.EDGE_MAX_HEIGHT + 1), INVALID),
    (dict(W=1 << 31, S=1 << 26), INVALID),
])
def test_image_validation(kw, want):
    assert masks(**kw) == want


def test_empty_images_are_no_ops():
    assert masks(H=0) == OK and masks(W=0) == OK
    assert masks(inp=None, out=None, H=0) == OK


def test_mode_flag_and_cfg_validation():
    assert launch(mode=2) == INVALID
    assert launch(flags=4) == INVALID
    assert launch(mode=0, flags=_abi.EDGE_FLAG_CLAUSE2_ONLY) == INVALID
    assert lib.edge_full(A, B, 4, 100, 4, 32, 0, 8, None) == INVALID
    for bad in ((3, 4, 4, 1, 0), (4, 0, 4, 1, 0), (4, 4, 3, 1, 0), (4, 4, 4, 0, 0),
                (4, 2000, 4, 1, 0), (4, 4, 16, 1, 0), (4, 4, 4, 33, 0), (4, 4, 4, 1, 3),
                (4, 4, 4, 1, -1), (4, _abi.EDGE_TILE_MAX_ROWS + 1, 4, 1, 0, _abi.EDGE_SHAPE_TILE),
                (4, 4, 4, 1, 0, 5), (4, 4, 4, 1, 0, -1),
                (4, 3, 4, 1, 0, _abi.EDGE_SHAPE_BAND), (4, 8, 4, 1, 0, _abi.EDGE_SHAPE_BAND_XCD),
                (4, 2, 1, 1, 0, _abi.EDGE_SHAPE_BAND)):
        cfg = _abi.EdgeLaunchCfg(*bad)
        assert launch(cfg=ctypes.byref(cfg)) == INVALID, bad
    # tiles up to EDGE_TILE_MAX_ROWS rows pass the checks (the launch
    # itself is not reached: H = 0)
    ok = _abi.EdgeLaunchCfg(4, _abi.EDGE_TILE_MAX_ROWS, 4, 1, 0, _abi.EDGE_SHAPE_TILE)
    assert launch(cfg=ctypes.byref(ok), H=0) == OK
    # adjacent, non-overlapping buffers are fine up to the launch; exactly
    # touching ranges (out right after in) must not be reported as aliasing
    assert launch(out=A + 4 * 16, H=0) == OK


def peel(inp=A, out=B, H=4, W=100, S=4, wb=32, border=0, k=3, flags=0, cfg=None):
    return lib.edge_peel(inp, out, H, W, S, wb, border, k, flags, cfg, None)


@pytest.mark.parametrize("kw,want", [
    (dict(wb=16), INVALID), (dict(border=2), INVALID), (dict(H=-1), INVALID),
    (dict(S=3), INVALID), (dict(inp=None), INVALID), (dict(out=None), INVALID),
    (dict(inp=A + 2), ALIGN), (dict(out=A + 16), ALIAS), (dict(k=-1), INVALID),
    (dict(k=_abi.EDGE_PEEL_MAX_ITERATIONS + 1), INVALID), (dict(flags=1), INVALID),
    (dict(flags=_abi.EDGE_FLAG_PEEL_EDGE | _abi.EDGE_FLAG_INVERT_OUT), INVALID),
    (dict(cfg=ctypes.byref(_abi.EdgeLaunchCfg(4, 0, 4, 1, 0))), INVALID),
    (dict(H=0), OK), (dict(W=0, inp=None, out=None), OK),
    (dict(H=_abi.EDGE_MAX_HEIGHT + 1), INVALID),
])
def test_peel_validation(kw, want):
    assert peel(**kw) == want


def test_default_cfg():
    c = _abi.EdgeLaunchCfg()
    assert lib.edge_default_cfg(8192, 8192, 64, 0, 0, ctypes.byref(c)) == OK
    assert c.vec_words in (1, 2, 4) and c.rows_per_tile >= 1 and c.waves_per_block >= 1
    assert lib.edge_default_cfg(8192, 8192, 48, 0, 0, ctypes.byref(c)) == INVALID
    assert lib.edge_default_cfg(-1, 8, 32, 0, 0, ctypes.byref(c)) == INVALID
    assert lib.edge_default_cfg(100, 100, 32, 0, 1, ctypes.byref(c)) == OK
    assert c.blocks_per_cu >= 1
    # built-in shape of uint64 squares: 2-row strips under 3 MiB of traffic,
    # then tiles of 4 rows (to 12 MiB), 8 rows (to 64 MiB) and 16 rows
    # regrouped by XCD (to 96 MiB), then 2-row bands
    for side, shape, rows in ((2048, _abi.EDGE_SHAPE_STRIP, 2), (4096, _abi.EDGE_SHAPE_TILE, 4),
                              (8192, _abi.EDGE_SHAPE_TILE, 8), (11584, _abi.EDGE_SHAPE_TILE, 8),
                              (16384, _abi.EDGE_SHAPE_TILE_XCD, 16),
                              (23168, _abi.EDGE_SHAPE_BAND_XCD, 2),
                              (65536, _abi.EDGE_SHAPE_BAND_XCD, 2)):
        assert lib.edge_default_cfg(side, side, 64, 0, 0, ctypes.byref(c)) == OK
        assert (c.shape, c.rows_per_tile) == (shape, rows), (side, c.shape, c.rows_per_tile)
        assert c.rows_per_tile <= _abi.EDGE_TILE_MAX_ROWS or c.shape == _abi.EDGE_SHAPE_STRIP
        assert c.shape != _abi.EDGE_SHAPE_BAND_XCD or c.waves_per_block * c.rows_per_tile >= 3
    # past the dispatch limit of a band grid (2^32 work-items), long strips
    assert lib.edge_default_cfg(1 << 25, 65536, 64, 0, 0, ctypes.byref(c)) == OK
    assert (c.shape, c.rows_per_tile) == (_abi.EDGE_SHAPE_STRIP, 256)
    assert lib.edge_default_cfg(1 << 20, 65536, 64, 0, 0, ctypes.byref(c)) == OK
    assert c.shape == _abi.EDGE_SHAPE_BAND_XCD
    # rows of at most 32 words: narrow units whatever the size
    assert lib.edge_default_cfg(65536, 1024, 32, 0, 0, ctypes.byref(c)) == OK
    assert c.vec_words == 1 and c.shape == _abi.EDGE_SHAPE_STRIP
    # four words per lane only when the rows fill 75% of their 256-word spans
    for side, vec in ((4096, 2), (6000, 2), (6200, 4), (8192, 4), (9600, 2), (12800, 4)):
        assert lib.edge_default_cfg(side, side, 64, 0, 0, ctypes.byref(c)) == OK
        assert c.vec_words == vec, (side, c.vec_words)


def table(rows):
    t = np.zeros(len(rows), dtype=DESC_DTYPE)
    for i, r in enumerate(rows):
        t[i] = r
    return t


def test_batch_check():
    ok = table([(0, 10, 40, 2), (20, 5, 64, 2), (30, 0, 0, 0), (31, 3, 1, 1)])
    assert lib.edge_batch_check(ok.ctypes.data, len(ok), 34, 32) == OK
    assert lib.edge_batch_check(ok.ctypes.data, len(ok), 33, 32) == INVALID  # last image overruns
    tall = (0, _abi.EDGE_MAX_HEIGHT + 1, 1, 1)             # inside an arena of 2^30 + 1 words
    assert lib.edge_batch_check(table([tall]).ctypes.data, 1, (1 << 30) + 1, 32) == INVALID
    assert lib.edge_batch_check(table([(0, 1 << 30, 1, 1)]).ctypes.data, 1, (1 << 30) + 1,
                                32) == OK
    for bad in [(0, -1, 4, 1), (0, 1, -4, 1), (-1, 1, 4, 1), (0, 2, 40, 1), (0, 2, 32, 1 << 40)]:
        t = table([bad])
        assert lib.edge_batch_check(t.ctypes.data, 1, 1000, 32) == INVALID, bad
    assert lib.edge_batch_check(None, 0, 0, 32) == OK
    assert lib.edge_batch_check(None, 1, 10, 32) == INVALID
    assert lib.edge_batch_check(ok.ctypes.data, len(ok), 34, 16) == INVALID


def test_batch_validation():
    need = lib.edge_batch_workspace_bytes(4)
    # header, 5 image records of 48 bytes, 65537 wavefront entries of 72 bytes
    # (the largest grid)
    assert need == (8 + 5 * 6 + 65537 * 9) * 8
    assert lib.edge_batch_workspace_bytes(-1) < 0
    W = 0x30000000

    def batch(inp=A, out=B, words=1000, tab=W + 0x1000, n=4, wb=32, border=0, mode=0, flags=0,
              ws=W, wsb=need):
        return lib.edge_batch(inp, out, words, tab, n, wb, border, mode, flags, None, ws, wsb,
                              None)

    assert batch(n=-1) == INVALID
    assert batch(wb=8) == INVALID
    assert batch(mode=3) == INVALID
    assert batch(tab=None) == INVALID
    assert batch(tab=W + 0x1004) == ALIGN
    assert batch(inp=A + 2) == ALIGN
    assert batch(out=A + 400) == ALIAS
    assert batch(wsb=need - 8) == WS
    assert batch(ws=None) == WS
    assert batch(ws=W + 128) == WS
    assert batch(n=0) == OK
    h = ctypes.c_void_p()
    assert lib.edge_batch_graph_create(A, B, 1000, W + 0x1000, 4, 32, 0, 0, 0, None, W, need - 8,
                                       ctypes.byref(h)) == WS
    assert not h.value
    assert lib.edge_graph_destroy(None) == OK
    assert lib.edge_graph_launch(None, None) == INVALID


def test_batch_noalloc_validation():
    # every case returns before the one HIP query (the array's address)
    W = 0x30000000
    PLANNED = 1 << 2

    def noalloc(inp=A, out=B, words=1000, tab=W + 0x1000, n=4, wb=32, border=0, mode=0, flags=0):
        return lib.edge_batch_noalloc(inp, out, words, tab, n, wb, border, mode, flags, None, None)

    assert _abi.EDGE_BATCH_NOALLOC_MAX_IMAGES == 16384
    assert noalloc(n=16385) == WS
    assert noalloc(n=1 << 30) == WS
    assert noalloc(flags=PLANNED) == INVALID
    assert noalloc(n=-1) == INVALID
    assert noalloc(wb=8) == INVALID
    assert noalloc(tab=None) == INVALID
    assert noalloc(inp=A + 2) == ALIGN
    assert noalloc(out=A + 400) == ALIAS
    assert noalloc(n=0) == OK
    assert noalloc(n=0, flags=PLANNED) == INVALID


def test_copy_validation():
    assert lib.edge_copy_bytes(A, B, 15, None) == INVALID
    assert lib.edge_copy_bytes(A + 8, B, 16, None) == ALIGN
    assert lib.edge_copy_bytes(A, A + 16, 64, None) == ALIAS
    assert lib.edge_copy_bytes(A, B, 0, None) == OK


def test_planned_flag_and_host_plan_validation():
    planned = _abi.EDGE_FLAG_PLANNED
    assert launch(flags=planned) == INVALID          # single-image calls reject it
    used = ctypes.c_int64()
    P = 0x40000000
    big = 1 << 20
    assert lib.edge_batch_plan(A, B, 100, None, 1, 32, None, P, big, ctypes.byref(used)) == INVALID
    assert lib.edge_batch_plan(A, B, 100, None, 0, 48, None, P, big, ctypes.byref(used)) == INVALID
    assert lib.edge_batch_plan(A, B, 100, None, 0, 32, None, P, 8, ctypes.byref(used)) == WS
    assert lib.edge_batch_plan(A, B, 100, None, 0, 32, None, P + 4, big, ctypes.byref(used)) == WS
    assert lib.edge_batch_plan(A, B, -1, None, 0, 32, None, P, big, ctypes.byref(used)) == INVALID
    assert lib.edge_batch_plan(A, B, 100, None, 0, 32, None, P, big, None) == INVALID
    bad = table([(0, 2, 40, 1)])                      # stride below the row's words
    buf = np.zeros(lib.edge_batch_workspace_bytes(1) // 8, np.int64)
    assert lib.edge_batch_plan(A, B, 100, bad.ctypes.data, 1, 32, None, buf.ctypes.data,
                               buf.nbytes, ctypes.byref(used)) == INVALID


def test_binding_rejects_host_tensors():
    """The C ABI takes bare pointers and cannot tell host memory from
    device memory; the Python binding refuses host tensors before the call."""
    import torch
    import paper_1401_5245_amd as em
    a, b = torch.zeros(64, dtype=torch.int64), torch.zeros(64, dtype=torch.int64)
    with pytest.raises(ValueError):
        em.copy_bytes(a, b, 16)
    with pytest.raises(ValueError):
        em.edge_masks(a.view(4, 16), b.view(4, 16), 4, 64)
    with pytest.raises(ValueError):
        em.peel(a.view(4, 16), b.view(4, 16), 4, 64, 2)
    ws = torch.zeros(em.batch_workspace_bytes(1), dtype=torch.uint8)
    table = torch.zeros(3, dtype=torch.int64)
    with pytest.raises(ValueError):
        em.edge_batch(a, b, table, 1, ws)
