"""Shared helpers of the GPU tests: pack, upload, run through the C ABI,
download, and compare with the oracle bit for bit."""
import sys

import numpy as np
import torch

import oracle
from synth import pack_rows, pad_bits_zero, row_words, unpack_rows

SENTINEL32 = np.uint32(0xA5A5A5A5)
CLAUSES = {("masks", False): oracle.CLAUSE1, ("full", False): oracle.CLAUSE1 | oracle.CLAUSE2,
           ("full", True): oracle.CLAUSE2}


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def to_device_words(words: np.ndarray, offset_words: int = 0) -> torch.Tensor:
    """Upload packed words; with offset_words > 0 the tensor is a view that
    starts that many words into a larger allocation (misaligned pointer)."""
    wb = words.dtype.itemsize * 8
    tdt = torch.int64 if wb == 64 else torch.int32
    host = torch.from_numpy(words.view(np.int64 if wb == 64 else np.int32).copy())
    if offset_words == 0:
        return host.cuda()
    flat = torch.zeros(host.numel() + offset_words + 8, dtype=tdt, device="cuda")
    flat[offset_words:offset_words + host.numel()] = host.reshape(-1).cuda()
    return flat[offset_words:offset_words + host.numel()].view(host.shape)


def run_single(img: np.ndarray, word_bits: int = 32, *, border="white", mode="masks",
               clause2_only=False, invert=False, stride_extra=0, pad="random", cfg=None,
               offset_words=0, api="image"):
    """Run one image through the library; returns (out_words, out_image)."""
    import paper_1401_5245_amd as em
    H, W = img.shape
    S = row_words(W, word_bits) + stride_extra
    words = pack_rows(img, word_bits, S, pad=pad, seed=H * 7 + W)
    inp = to_device_words(words, offset_words)
    out = to_device_words(np.full_like(words, SENTINEL32 if word_bits == 32 else
                                       np.uint64(0xA5A5A5A5A5A5A5A5)), offset_words)
    if api == "masks":
        em.edge_masks(inp, out, H, W, border=border)
    elif api == "full":
        em.edge_full(inp, out, H, W, border=border, clause2_only=clause2_only, invert=invert)
    else:
        em.edge_image(inp, out, H, W, mode=mode, border=border, clause2_only=clause2_only,
                      invert=invert, cfg=cfg)
    torch.cuda.synchronize()
    ow = out.cpu().numpy().view(words.dtype).reshape(H, S)
    # stride padding words are never written
    wd = row_words(W, word_bits)
    sent = words.dtype.type(SENTINEL32 if word_bits == 32 else 0xA5A5A5A5A5A5A5A5)
    assert (ow[:, wd:] == sent).all(), "stride padding was written"
    assert pad_bits_zero(ow, W), "output pad bits are not zero"
    return ow, unpack_rows(ow, W)


def expect(img, *, border="white", mode="masks", clause2_only=False, invert=False):
    return oracle.edge(img, border=border, clauses=CLAUSES[(mode, clause2_only)], invert=invert)


def assert_same(got: np.ndarray, want: np.ndarray, what: str = "") -> None:
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        y, x = bad[0]
        raise AssertionError(f"{what}: {len(bad)} pixels differ; first at (y={y}, x={x}): "
                             f"got {got[y, x]} want {want[y, x]}")
