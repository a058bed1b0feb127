"""Bit packing of binary images into row words, and back.

Layout (shared by every consumer of packed images here): pixel (x, y) is bit
``x mod B`` of word ``y * S + x // B`` with B = 32 or 64 word bits, LSB first,
little-endian words. The byte image is the same for B = 32 and B = 64; only the
row padding differs. This is ``numpy.packbits(..., bitorder='little')`` with
each row padded to S words. No edge arithmetic lives here.
"""
from __future__ import annotations

import numpy as np

_DTYPES = {32: np.uint32, 64: np.uint64}


def row_words(width: int, word_bits: int) -> int:
    """Valid words per row: ceil(W / B)."""
    return -(-int(width) // int(word_bits))


def pack_rows(img: np.ndarray, word_bits: int = 32, stride_words: int | None = None,
              pad: str = "zero", seed: int = 0) -> np.ndarray:
    """Pack an (H, W) image with values 0 (black) / 1 (white) into (H, S) words.

    ``pad`` fills the bits past W in the last valid word and the stride words
    beyond it: ``"zero"``, ``"ones"`` or ``"random"`` (seeded), so tests can
    check that the consumer ignores them.
    """
    if word_bits not in _DTYPES:
        raise ValueError("word_bits must be 32 or 64")
    img = np.asarray(img)
    H, W = img.shape
    wd = row_words(W, word_bits)
    S = wd if stride_words is None else int(stride_words)
    if S < wd:
        raise ValueError("stride_words < words per row")
    nbytes = S * word_bits // 8
    bits = (img != 0).astype(np.uint8)
    packed = np.packbits(bits, axis=1, bitorder="little") if W else np.zeros((H, 0), np.uint8)
    out = np.zeros((H, nbytes), dtype=np.uint8)
    out[:, :packed.shape[1]] = packed
    if pad != "zero" and H:
        if pad == "ones":
            fill = np.full((H, nbytes), 0xFF, np.uint8)
        elif pad == "random":
            fill = np.random.default_rng(seed).integers(0, 256, (H, nbytes), dtype=np.uint8)
        else:
            raise ValueError(f"unknown pad {pad!r}")
        valid = np.zeros(nbytes * 8, dtype=np.uint8)
        valid[:W] = 1
        vmask = np.packbits(valid, bitorder="little")
        out = (out & vmask) | (fill & ~vmask)
    return np.ascontiguousarray(out).view(_DTYPES[word_bits]).reshape(H, S)


def unpack_rows(words: np.ndarray, width: int) -> np.ndarray:
    """Inverse of pack_rows: (H, S) words -> (H, W) uint8 image in {0, 1}."""
    words = np.ascontiguousarray(words)
    H = words.shape[0]
    as_bytes = words.view(np.uint8).reshape(H, -1)
    bits = np.unpackbits(as_bytes, axis=1, bitorder="little")
    return bits[:, :width].copy()


def pad_bits_zero(words: np.ndarray, width: int) -> bool:
    """True when every bit at x >= width of each row's valid words is 0.

    Only the valid words (the first ceil(W / B) of each row) are inspected;
    stride words beyond them belong to the caller.
    """
    words = np.ascontiguousarray(words)
    H = words.shape[0]
    word_bits = words.dtype.itemsize * 8
    wd = row_words(width, word_bits)
    bits = np.unpackbits(words[:, :wd].view(np.uint8).reshape(H, -1), axis=1,
                         bitorder="little")
    return not bits[:, width:].any()
