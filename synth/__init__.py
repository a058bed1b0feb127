"""Seeded synthetic inputs and the packed-row layout.

Shared by the tests, the smoke check and the benchmark, for both the GPU path
and the CPU oracle. Holds no edge arithmetic.
"""
from .packing import pack_rows, unpack_rows, row_words, pad_bits_zero  # noqa: F401
from . import images  # noqa: F401
