"""MI355X (gfx950) edge detection of binary images by the method of masks.

Thin Python binding of libedgemask (C ABI in include/edge_masks.h). Every
step of the computation runs in the library's HIP kernels; this module only
checks tensors and passes device pointers, sizes and the current HIP stream.
PyTorch provides device memory and streams.

Images are packed rows of 32- or 64-bit words (pixel x of row y is bit
x % B of word y * stride + x // B, black = 0, white = 1), held in torch
tensors of dtype int32/uint32 (B = 32) or int64/uint64 (B = 64).
"""
from __future__ import annotations

import ctypes

import torch

from ._abi import (EDGE_BORDER_BLACK, EDGE_BORDER_WHITE, EDGE_FLAG_CLAUSE2_ONLY,  # noqa: F401
                   EDGE_FLAG_INVERT_OUT, EDGE_FLAG_PEEL_EDGE, EDGE_MODE_FULL, EDGE_MODE_MASKS,
                   EDGE_PEEL_MAX_ITERATIONS, EdgeError, EdgeImageDesc, EdgeLaunchCfg, check, load)

_lib = load()

BORDERS = {"white": EDGE_BORDER_WHITE, "black": EDGE_BORDER_BLACK}
MODES = {"masks": EDGE_MODE_MASKS, "full": EDGE_MODE_FULL}
_WORD_DTYPES = {torch.int32: 32, torch.int64: 64}
for _name, _bits in (("uint32", 32), ("uint64", 64)):
    if hasattr(torch, _name):
        _WORD_DTYPES[getattr(torch, _name)] = _bits


def word_bits_of(t: torch.Tensor) -> int:
    try:
        return _WORD_DTYPES[t.dtype]
    except KeyError:
        raise TypeError(f"packed words must be 32- or 64-bit integers, got {t.dtype}") from None


def stream_handle(stream=None) -> int:
    """HIP stream handle of `stream` (default: torch's current stream)."""
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _image_args(inp: torch.Tensor, out: torch.Tensor, height: int, width: int,
                stride_words):
    if not (inp.is_cuda and out.is_cuda):
        raise ValueError("input and output must be device tensors")
    if inp.dtype != out.dtype:
        raise TypeError("input and output must have the same word type")
    if not (inp.is_contiguous() and out.is_contiguous()):
        raise ValueError("input and output must be contiguous")
    wb = word_bits_of(inp)
    if stride_words is None:
        if inp.dim() != 2:
            raise ValueError("pass stride_words for a tensor that is not (H, stride)")
        stride_words = inp.shape[1]
    need = (height - 1) * stride_words + -(-width // wb) if height and width else 0
    if inp.numel() < need or out.numel() < need:
        raise ValueError(f"tensors hold fewer than the {need} words the image spans")
    return wb, int(stride_words)


def _resolve_cfg(cfg, height, width, word_bits, mode):
    """None / a dict / an EdgeLaunchCfg, or "tuned": the autotuned entry for
    this shape class (None when the table has none)."""
    if isinstance(cfg, str):
        if cfg != "tuned":
            raise ValueError(f"unknown cfg {cfg!r}")
        from . import tune
        cfg = tune.lookup_image(height, width, word_bits, mode)
    if cfg is None or isinstance(cfg, EdgeLaunchCfg):
        return cfg
    return EdgeLaunchCfg.from_dict(cfg)


def _cfg_ptr(cfg):
    return None if cfg is None else ctypes.byref(cfg)


def edge_masks(inp: torch.Tensor, out: torch.Tensor, height: int, width: int, *,
               border: str = "white", stride_words=None, stream=None) -> torch.Tensor:
    """Plain method: out = NOT(p) AND (n2 OR n4 OR n6 OR n8) for every pixel."""
    wb, s = _image_args(inp, out, height, width, stride_words)
    check(_lib.edge_masks(inp.data_ptr(), out.data_ptr(), height, width, s, wb, BORDERS[border],
                          stream_handle(stream)))
    return out


def edge_full(inp: torch.Tensor, out: torch.Tensor, height: int, width: int, *,
              border: str = "white", clause2_only: bool = False, invert: bool = False,
              stride_words=None, stream=None) -> torch.Tensor:
    """Full definition: clause 1 OR black pixels with <= 1 black 8-neighbour."""
    wb, s = _image_args(inp, out, height, width, stride_words)
    flags = (EDGE_FLAG_CLAUSE2_ONLY if clause2_only else 0) | (EDGE_FLAG_INVERT_OUT if invert else 0)
    check(_lib.edge_full(inp.data_ptr(), out.data_ptr(), height, width, s, wb, BORDERS[border],
                         flags, stream_handle(stream)))
    return out


def edge_image(inp: torch.Tensor, out: torch.Tensor, height: int, width: int, *,
               mode: str = "masks", border: str = "white", clause2_only: bool = False,
               invert: bool = False, cfg=None, stride_words=None, stream=None) -> torch.Tensor:
    """Single image with explicit mode, flags and launch configuration
    (cfg: None = built-in, "tuned" = autotuned table entry, or a dict)."""
    wb, s = _image_args(inp, out, height, width, stride_words)
    flags = (EDGE_FLAG_CLAUSE2_ONLY if clause2_only else 0) | (EDGE_FLAG_INVERT_OUT if invert else 0)
    c = _resolve_cfg(cfg, height, width, wb, mode)
    check(_lib.edge_image_launch(inp.data_ptr(), out.data_ptr(), height, width, s, wb,
                                 BORDERS[border], MODES[mode], flags, _cfg_ptr(c),
                                 stream_handle(stream)))
    return out


def edge_directions(inp: torch.Tensor, out4: torch.Tensor, height: int, width: int, *,
                    border: str = "white", cfg=None, stride_words=None, stream=None):
    """The four fundamental edges of section 4 (the edge types of Fig. 2).

    ``out4`` holds four planes of the input's layout, in the order left,
    right, up, down: a (4, H, stride) tensor, or one whose numel is a
    multiple of 4 (planes back to back). Their OR equals edge_masks."""
    wb, s = _image_args(inp, out4.view(4, -1)[0], height, width, stride_words)
    plane = out4.numel() // 4
    c = _resolve_cfg(cfg, height, width, wb, "masks")
    check(_lib.edge_directions(inp.data_ptr(), out4.data_ptr(), plane, height, width, s, wb,
                               BORDERS[border], _cfg_ptr(c), stream_handle(stream)))
    return out4


def threshold_pack(grey: torch.Tensor, out: torch.Tensor, height: int, width: int,
                   threshold: int, *, grey_stride=None, stride_words=None, stream=None):
    """Binarise a uint8 grey image (white where grey >= threshold) into
    packed rows (section 7's conversion of a non-binary image)."""
    if grey.dtype != torch.uint8 or not grey.is_cuda or not grey.is_contiguous():
        raise TypeError("grey must be a contiguous uint8 device tensor")
    gs = int(grey_stride if grey_stride is not None else grey.shape[-1])
    if height and width and grey.numel() < (height - 1) * gs + width:
        raise ValueError("grey tensor smaller than the image")
    wb, s = _image_args(out, out, height, width, stride_words)
    check(_lib.edge_threshold_pack(grey.data_ptr(), gs, int(threshold), out.data_ptr(), height,
                                   width, s, wb, stream_handle(stream)))
    return out


def threshold_edges(grey: torch.Tensor, out: torch.Tensor, height: int, width: int,
                    threshold: int, *, mode: str = "masks", border: str = "white",
                    clause2_only: bool = False, invert: bool = False, cfg=None,
                    grey_stride=None, stride_words=None, stream=None):
    """Edge map of a uint8 grey image binarised at `threshold`, in one pass
    (the binary image is never written)."""
    if grey.dtype != torch.uint8 or not grey.is_cuda or not grey.is_contiguous():
        raise TypeError("grey must be a contiguous uint8 device tensor")
    gs = int(grey_stride if grey_stride is not None else grey.shape[-1])
    if height and width and grey.numel() < (height - 1) * gs + width:
        raise ValueError("grey tensor smaller than the image")
    wb, s = _image_args(out, out, height, width, stride_words)
    flags = (EDGE_FLAG_CLAUSE2_ONLY if clause2_only else 0) | (EDGE_FLAG_INVERT_OUT if invert else 0)
    c = None if cfg is None else (EdgeLaunchCfg.from_dict(cfg) if isinstance(cfg, dict) else cfg)
    check(_lib.edge_threshold_edges(grey.data_ptr(), gs, int(threshold), out.data_ptr(), height,
                                    width, s, wb, BORDERS[border], MODES[mode], flags,
                                    _cfg_ptr(c), stream_handle(stream)))
    return out


def peel(inp: torch.Tensor, out: torch.Tensor, height: int, width: int, iterations: int, *,
         border: str = "white", edge_out: bool = False, cfg=None, stride_words=None,
         stream=None) -> torch.Tensor:
    """`iterations` peels of the edge in one pass (each turns the current
    edge points white; at most EDGE_PEEL_MAX_ITERATIONS). With ``edge_out``
    the output is the edge map of the peeled image (the next layer)."""
    wb, s = _image_args(inp, out, height, width, stride_words)
    c = None if cfg is None else (EdgeLaunchCfg.from_dict(cfg) if isinstance(cfg, dict) else cfg)
    check(_lib.edge_peel(inp.data_ptr(), out.data_ptr(), height, width, s, wb, BORDERS[border],
                         int(iterations), EDGE_FLAG_PEEL_EDGE if edge_out else 0, _cfg_ptr(c),
                         stream_handle(stream)))
    return out


def staged_scratch_bytes(height: int, stride_words: int, word_bits: int) -> int:
    return 4 * height * stride_words * word_bits // 8


def edge_masks_staged(inp: torch.Tensor, out: torch.Tensor, height: int, width: int,
                      scratch: torch.Tensor, *, border: str = "white", stride_words=None,
                      stream=None) -> torch.Tensor:
    """The paper's three stages as eight separate passes (the unfused
    ablation of edge_masks; same output)."""
    wb, s = _image_args(inp, out, height, width, stride_words)
    if not scratch.is_cuda or not scratch.is_contiguous():
        raise ValueError("scratch must be a contiguous device tensor")
    check(_lib.edge_masks_staged(inp.data_ptr(), out.data_ptr(), scratch.data_ptr(),
                                 scratch.numel() * scratch.element_size(), height, width, s, wb,
                                 BORDERS[border], stream_handle(stream)))
    return out


def default_cfg(height: int, width: int, word_bits: int, mode: str = "masks",
                batch: bool = False) -> dict:
    c = EdgeLaunchCfg()
    check(_lib.edge_default_cfg(height, width, word_bits, MODES[mode], int(batch), ctypes.byref(c)))
    return c.as_dict()


def prepare(inp: torch.Tensor, out: torch.Tensor, height: int, width: int, *,
            mode: str = "masks", border: str = "white", clause2_only: bool = False,
            invert: bool = False, cfg=None, stride_words=None, stream=None):
    """Check the arguments once and return a no-argument callable that
    enqueues the same launch again (for tight launch loops). The tensors
    must stay alive while the callable is used."""
    wb, s = _image_args(inp, out, height, width, stride_words)
    flags = (EDGE_FLAG_CLAUSE2_ONLY if clause2_only else 0) | (EDGE_FLAG_INVERT_OUT if invert else 0)
    c = _resolve_cfg(cfg, height, width, wb, mode)
    args = (inp.data_ptr(), out.data_ptr(), height, width, s, wb, BORDERS[border], MODES[mode],
            flags, _cfg_ptr(c), stream_handle(stream))
    fn = _lib.edge_image_launch

    def launch():
        rc = fn(*args)
        if rc:
            check(rc)
    launch.keep = (inp, out, c)
    return launch


def copy_bytes(src: torch.Tensor, dst: torch.Tensor, n_bytes: int, stream=None) -> None:
    """Plain 128-bit device copy (the bandwidth reference for the kernels)."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("source and destination must be contiguous device tensors")
    if n_bytes > min(src.numel() * src.element_size(), dst.numel() * dst.element_size()):
        raise ValueError(f"{n_bytes} bytes exceed the source or destination tensor")
    check(_lib.edge_copy_bytes(src.data_ptr(), dst.data_ptr(), n_bytes, stream_handle(stream)))


from .batch import (Batch, BatchGraph, batch_workspace_bytes, edge_batch,  # noqa: E402,F401
                    edge_batch_noalloc, pack_arena)
