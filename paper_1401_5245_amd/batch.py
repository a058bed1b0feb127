"""Many images in one persistent launch: arenas, descriptor tables, graphs.

A batch is two device arenas of packed words (input and output, same
layout), a device table of ``edge_image_desc`` records (offset, height,
width, stride; offsets and strides in words) and a small device workspace
the library writes its work plan into. ``edge_batch`` enqueues the planner
and the persistent kernel; ``BatchGraph`` captures the same work once in a
HIP graph and replays it.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._abi import (EDGE_FLAG_CLAUSE2_ONLY, EDGE_FLAG_INVERT_OUT, EDGE_FLAG_PLANNED,
                   EdgeImageDesc, EdgeLaunchCfg, check, load)

_lib = load()

DESC_DTYPE = np.dtype([("offset_words", "<i8"), ("height", "<i4"), ("width", "<i4"),
                       ("stride_words", "<i8")])
assert DESC_DTYPE.itemsize == ctypes.sizeof(EdgeImageDesc)

_BORDERS = {"white": 0, "black": 1}
_MODES = {"masks": 0, "full": 1}
_NP_WORDS = {32: np.uint32, 64: np.uint64}
_TORCH_WORDS = {32: torch.int32, 64: torch.int64}


def _flags(clause2_only: bool, invert: bool, planned: bool = False) -> int:
    return ((EDGE_FLAG_CLAUSE2_ONLY if clause2_only else 0) |
            (EDGE_FLAG_INVERT_OUT if invert else 0) | (EDGE_FLAG_PLANNED if planned else 0))


def _cfg_ptr(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, dict):
        cfg = EdgeLaunchCfg.from_dict(cfg)
    return ctypes.byref(cfg)


def _resolve(cfg, n_images, arena_words, word_bits, mode):
    """cfg "tuned": the autotuned batch entry for this size class (or None)."""
    if isinstance(cfg, str):
        if cfg != "tuned":
            raise ValueError(f"unknown cfg {cfg!r}")
        from . import tune
        return tune.lookup_batch(n_images, arena_words, word_bits, mode)
    return cfg


def _word_bits(t: torch.Tensor) -> int:
    from . import word_bits_of
    return word_bits_of(t)


def batch_workspace_bytes(n_images: int) -> int:
    v = int(_lib.edge_batch_workspace_bytes(n_images))
    if v < 0:
        check(v)
    return v


def pack_arena(images, word_bits: int, align_words: int | None = None):
    """Concatenate packed images into one arena.

    ``images``: sequence of ``(words, width)`` with ``words`` an (H, S)
    array of packed rows. Each image starts at a multiple of
    ``align_words`` (default: 16 bytes). Returns ``(arena, table)``: a 1-D
    word array and a structured array of descriptors.
    """
    if align_words is None:
        align_words = 128 // word_bits
    n = len(images)
    table = np.zeros(n, dtype=DESC_DTYPE)
    off = 0
    for i, (w, width) in enumerate(images):
        H, S = w.shape
        off = -(-off // align_words) * align_words
        table[i] = (off, H, width, S)
        off += H * S
    total = -(-off // align_words) * align_words
    arena = np.zeros(max(total, align_words), dtype=_NP_WORDS[word_bits])
    for i, (w, _) in enumerate(images):
        o = int(table[i]["offset_words"])
        arena[o:o + w.size] = w.reshape(-1)
    return arena, table


def check_table(table: np.ndarray, arena_words: int, word_bits: int) -> None:
    """Host-side validation of a descriptor table (raises EdgeError)."""
    t = np.ascontiguousarray(table, dtype=DESC_DTYPE)
    check(_lib.edge_batch_check(t.ctypes.data if len(t) else None, len(t), arena_words, word_bits))


def table_to_device(table: np.ndarray, device="cuda") -> torch.Tensor:
    t = np.ascontiguousarray(table, dtype=DESC_DTYPE)
    return torch.from_numpy(t.view(np.int64).reshape(-1, 3).copy()).to(device)


def plan_batch(in_arena: torch.Tensor, out_arena: torch.Tensor, table: np.ndarray, *,
               mode: str = "masks", cfg=None, out: np.ndarray | None = None):
    """Host-side work plan for `table` (host descriptors of the device table)
    and these device arenas. Returns (plan words, used bytes): copy the first
    `used bytes` into the workspace and launch with planned=True."""
    wb = _word_bits(in_arena)
    t = np.ascontiguousarray(table, dtype=DESC_DTYPE)
    cfg = _resolve(cfg, len(t), in_arena.numel(), wb, mode)
    nbytes = batch_workspace_bytes(len(t))
    if out is None:
        out = np.zeros(-(-nbytes // 8), dtype=np.int64)
    used = ctypes.c_int64()
    check(_lib.edge_batch_plan(in_arena.data_ptr(), out_arena.data_ptr(), in_arena.numel(),
                               t.ctypes.data if len(t) else None, len(t), wb, _cfg_ptr(cfg),
                               out.ctypes.data, out.nbytes, ctypes.byref(used)))
    return out, int(used.value)


def _check_batch_tensors(in_arena, out_arena, table_dev, n_images, workspace) -> None:
    """Device placement and sizes that the C ABI cannot see (it takes bare
    pointers): arenas of one type and size, a table of at least n_images
    descriptors, all contiguous device tensors."""
    for name, t in (("in_arena", in_arena), ("out_arena", out_arena), ("table", table_dev),
                    ("workspace", workspace)):
        if t is None and name == "workspace":
            continue
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous device tensor")
    if out_arena.dtype != in_arena.dtype or out_arena.numel() != in_arena.numel():
        raise ValueError("input and output arenas must match in type and size")
    if table_dev.numel() * table_dev.element_size() < int(n_images) * DESC_DTYPE.itemsize:
        raise ValueError(f"the table holds fewer than {n_images} descriptors")


def edge_batch(in_arena: torch.Tensor, out_arena: torch.Tensor, table_dev: torch.Tensor,
               n_images: int, workspace: torch.Tensor, *, border: str = "white",
               mode: str = "masks", clause2_only: bool = False, invert: bool = False, cfg=None,
               planned: bool = False, stream=None) -> None:
    """Enqueue one batched launch: the device planner then the persistent
    kernel, or (planned=True) the kernel alone on a plan already in the
    workspace (see plan_batch)."""
    from . import stream_handle
    wb = _word_bits(in_arena)
    _check_batch_tensors(in_arena, out_arena, table_dev, n_images, workspace)
    cfg = _resolve(cfg, n_images, in_arena.numel(), wb, mode)
    check(_lib.edge_batch(in_arena.data_ptr(), out_arena.data_ptr(), in_arena.numel(),
                          table_dev.data_ptr(), n_images, wb, _BORDERS[border], _MODES[mode],
                          _flags(clause2_only, invert, planned), _cfg_ptr(cfg),
                          workspace.data_ptr(),
                          workspace.numel() * workspace.element_size(), stream_handle(stream)))


def edge_batch_noalloc(in_arena: torch.Tensor, out_arena: torch.Tensor, table_dev: torch.Tensor,
                       n_images: int, *, border: str = "white", mode: str = "masks",
                       clause2_only: bool = False, invert: bool = False, cfg=None,
                       stream=None) -> None:
    """edge_batch with the workspace held by the library (a fixed array per
    GPU, at most EDGE_BATCH_NOALLOC_MAX_IMAGES images): for callers that
    cannot allocate. Calls that overlap in time on one GPU race."""
    from . import stream_handle
    wb = _word_bits(in_arena)
    _check_batch_tensors(in_arena, out_arena, table_dev, n_images, None)
    cfg = _resolve(cfg, n_images, in_arena.numel(), wb, mode)
    check(_lib.edge_batch_noalloc(in_arena.data_ptr(), out_arena.data_ptr(), in_arena.numel(),
                                  table_dev.data_ptr(), n_images, wb, _BORDERS[border],
                                  _MODES[mode], _flags(clause2_only, invert), _cfg_ptr(cfg),
                                  stream_handle(stream)))


class BatchGraph:
    """One batched launch captured in a HIP graph; replay with launch().

    The graph reads the descriptor table when it runs, so the table's
    contents (not its size or address) may be rewritten between replays.
    The tensors passed in are kept alive by this object.
    """

    def __init__(self, in_arena, out_arena, table_dev, n_images, workspace, *,
                 border="white", mode="masks", clause2_only=False, invert=False, cfg=None,
                 planned=False):
        wb = _word_bits(in_arena)
        _check_batch_tensors(in_arena, out_arena, table_dev, n_images, workspace)
        cfg = _resolve(cfg, n_images, in_arena.numel(), wb, mode)
        self._keep = (in_arena, out_arena, table_dev, workspace)
        h = ctypes.c_void_p()
        check(_lib.edge_batch_graph_create(
            in_arena.data_ptr(), out_arena.data_ptr(), in_arena.numel(), table_dev.data_ptr(),
            n_images, wb, _BORDERS[border], _MODES[mode], _flags(clause2_only, invert, planned),
            _cfg_ptr(cfg), workspace.data_ptr(), workspace.numel() * workspace.element_size(),
            ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None) -> None:
        from . import stream_handle
        if not self._h:
            raise RuntimeError("graph destroyed")
        check(_lib.edge_graph_launch(self._h, stream_handle(stream)))

    def close(self) -> None:
        if getattr(self, "_h", None):
            check(_lib.edge_graph_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Packed images resident in device arenas, ready to launch.

    ``images``: sequence of ``(words, width)`` (see pack_arena).
    ``plan``: "host" (default) plans once on the host and launches the
    persistent kernel alone; "device" runs the device planner on every
    launch (needed when the device table is rewritten between launches).
    """

    def __init__(self, images, word_bits: int, device="cuda", *, border="white",
                 mode="masks", clause2_only=False, invert=False, cfg=None, align_words=None,
                 plan: str = "host"):
        if plan not in ("host", "device"):
            raise ValueError("plan must be 'host' or 'device'")
        arena, table = pack_arena(images, word_bits, align_words)
        check_table(table, arena.size, word_bits)
        self.word_bits = word_bits
        self.table = table
        self.n = len(table)
        host = torch.from_numpy(arena.view(np.int64 if word_bits == 64 else np.int32))
        self.inp = host.to(device)
        self.out = torch.zeros_like(self.inp)
        self.table_dev = table_to_device(table, device)
        nb = batch_workspace_bytes(self.n)
        self.workspace = torch.zeros(-(-nb // 8), dtype=torch.int64, device=device)
        cfg = _resolve(cfg, self.n, self.inp.numel(), word_bits, mode)
        self.kw = dict(border=border, mode=mode, clause2_only=clause2_only, invert=invert,
                       cfg=cfg, planned=plan == "host")
        if plan == "host":
            words, used = plan_batch(self.inp, self.out, table, mode=mode, cfg=cfg)
            self.workspace[:-(-used // 8)].copy_(torch.from_numpy(words[:-(-used // 8)]))
        self._graph = None

    def run(self, stream=None) -> None:
        edge_batch(self.inp, self.out, self.table_dev, self.n, self.workspace, stream=stream,
                   **self.kw)

    def graph(self) -> BatchGraph:
        if self._graph is None:
            self._graph = BatchGraph(self.inp, self.out, self.table_dev, self.n, self.workspace,
                                     **self.kw)
        return self._graph

    def output_words(self, i: int, out_host: np.ndarray | None = None) -> np.ndarray:
        """Packed output rows (H, S) of image i (copies the arena if needed)."""
        if out_host is None:
            out_host = self.out.cpu().numpy().view(_NP_WORDS[self.word_bits])
        d = self.table[i]
        o, H, S = int(d["offset_words"]), int(d["height"]), int(d["stride_words"])
        return out_host[o:o + H * S].reshape(H, S)
