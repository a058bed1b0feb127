"""The largest images the entry points accept: 2^31 - 1 pixels per row and
EDGE_MAX_HEIGHT rows, bit-exact against the oracle on windows around
sampled positions (each window keeps enough margin that its cut edges
cannot reach the compared pixels; at the image's own edges the window edge
is the true border)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1401_5245_amd import _abi
from synth import unpack_rows
from tests.gpu_util import assert_same, log

pytestmark = pytest.mark.gpu

PEELS = 3
DEEP = 20          # levels split over two wavefronts per strip


def random_words(shape):
    n = int(np.prod(shape))
    return torch.randint(0, 256, (n * 8,), dtype=torch.uint8,
                         device="cuda").view(torch.int64).view(*shape)


def run_all(inp, H, W):
    """Plain, full definition and peel (image and layer) of one image."""
    import paper_1401_5245_amd as em
    outs = {}
    for name in ("plain", "full", "peel", "layer", "deep"):
        out = torch.empty_like(inp)
        if name == "plain":
            em.edge_masks(inp, out, H, W)
        elif name == "full":
            em.edge_full(inp, out, H, W)
        elif name == "deep":
            em.peel(inp, out, H, W, DEEP)
        else:
            em.peel(inp, out, H, W, PEELS, edge_out=name == "layer")
        outs[name] = out
    torch.cuda.synchronize()
    return outs


def oracle_of(name, win):
    if name == "plain":
        return oracle.edge(win)
    if name == "full":
        return oracle.edge(win, clauses=oracle.CLAUSE1 | oracle.CLAUSE2)
    if name == "deep":
        return oracle.peel(win, DEEP)
    return oracle.peel(win, PEELS, edge_out=name == "layer")


def test_widest_rows():
    H, W = 3, 2**31 - 1
    wd = (W + 63) // 64                              # 2^25 words of 64 bits per row
    log(f"widest rows: {H} x {W}")
    inp = random_words((H, wd))
    outs = run_all(inp, H, W)
    for a, b in ((0, 2), (wd // 2 - 1, wd // 2 + 1), (wd - 2, wd)):
        lo, hi = max(0, a - 1), min(wd, b + 1)       # one word of margin where the row goes on
        width = min(W, 64 * hi) - 64 * lo
        win = unpack_rows(inp[:, lo:hi].cpu().numpy().view(np.uint64), width)
        x0, x1 = 64 * (a - lo), min(W, 64 * b) - 64 * lo
        for name, out in outs.items():
            got = unpack_rows(out[:, lo:hi].cpu().numpy().view(np.uint64), width)
            assert_same(got[:, x0:x1], oracle_of(name, win)[:, x0:x1], f"{name} words {a}..{b}")


def test_tallest_image():
    H, W = _abi.EDGE_MAX_HEIGHT, 64                  # one 64-bit word per row: 8 GiB
    log(f"tallest image: {H} x {W}")
    inp = random_words((H, 1))
    outs = run_all(inp, H, W)
    m = DEEP + 2
    for y in (0, 1, 2, H // 2, H - 3, H - 2, H - 1):
        lo, hi = max(0, y - m), min(H, y + m + 1)
        win = unpack_rows(inp[lo:hi].cpu().numpy().view(np.uint64), W)
        for name, out in outs.items():
            got = unpack_rows(out[y:y + 1].cpu().numpy().view(np.uint64), W)
            assert_same(got, oracle_of(name, win)[y - lo:y - lo + 1], f"{name} row {y}")
