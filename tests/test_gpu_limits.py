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


def test_widest_rows_planes_and_grey():
    """Direction planes and grey input (threshold fused into the edge pass)
    on 3 rows of 2^31 - 1 pixels: 3 GiB of planes, 6 GiB of grey bytes."""
    import paper_1401_5245_amd as em
    torch.cuda.empty_cache()
    H, W = 3, 2**31 - 1
    wd = (W + 63) // 64
    log(f"widest rows, planes and grey: {H} x {W}")
    inp = random_words((H, wd))
    planes = torch.empty((4, H, wd), dtype=torch.int64, device="cuda")
    em.edge_directions(inp, planes, H, W)
    gs = 2**31                                       # 16-byte aligned grey rows
    grey = torch.randint(0, 256, (H, gs), dtype=torch.uint8, device="cuda")
    gout = torch.empty((H, wd), dtype=torch.int64, device="cuda")
    em.threshold_edges(grey, gout, H, W, 128, grey_stride=gs)
    torch.cuda.synchronize()
    for a, b in ((0, 2), (wd // 2 - 1, wd // 2 + 1), (wd - 2, wd)):
        lo, hi = max(0, a - 1), min(wd, b + 1)       # one word of margin where the row goes on
        width = min(W, 64 * hi) - 64 * lo
        x0, x1 = 64 * (a - lo), min(W, 64 * b) - 64 * lo
        win = unpack_rows(inp[:, lo:hi].cpu().numpy().view(np.uint64), width)
        want = oracle.fundamental_edges(win)
        for p in range(4):
            got = unpack_rows(planes[p, :, lo:hi].cpu().numpy().view(np.uint64), width)
            assert_same(got[:, x0:x1], want[p][:, x0:x1], f"plane {p} words {a}..{b}")
        gwin = grey[:, 64 * lo:64 * lo + width].cpu().numpy()
        want = oracle.edge(oracle.threshold(gwin, 128))
        got = unpack_rows(gout[:, lo:hi].cpu().numpy().view(np.uint64), width)
        assert_same(got[:, x0:x1], want[:, x0:x1], f"grey words {a}..{b}")
    del inp, planes, grey, gout
    torch.cuda.empty_cache()


def test_tallest_image_planes_and_grey():
    """Direction planes and grey input on EDGE_MAX_HEIGHT rows of 64 pixels:
    32 GiB of planes, 64 GiB of grey bytes."""
    import paper_1401_5245_amd as em
    torch.cuda.empty_cache()
    H, W = _abi.EDGE_MAX_HEIGHT, 64
    log(f"tallest image, planes and grey: {H} x {W}")
    inp = random_words((H, 1))
    planes = torch.empty((4, H, 1), dtype=torch.int64, device="cuda")
    em.edge_directions(inp, planes, H, W)
    torch.cuda.synchronize()
    rows = (0, 1, 2, H // 2, H - 3, H - 2, H - 1)
    for y in rows:
        lo, hi = max(0, y - 2), min(H, y + 3)
        want = oracle.fundamental_edges(unpack_rows(inp[lo:hi].cpu().numpy().view(np.uint64), W))
        for p in range(4):
            got = unpack_rows(planes[p, y:y + 1].cpu().numpy().view(np.uint64), W)
            assert_same(got, want[p][y - lo:y - lo + 1], f"plane {p} row {y}")
    del inp, planes
    torch.cuda.empty_cache()
    grey = torch.randint(0, 256, (H, W), dtype=torch.uint8, device="cuda")
    gout = torch.empty((H, 1), dtype=torch.int64, device="cuda")
    em.threshold_edges(grey, gout, H, W, 128)
    torch.cuda.synchronize()
    for y in rows:
        lo, hi = max(0, y - 2), min(H, y + 3)
        want = oracle.edge(oracle.threshold(grey[lo:hi].cpu().numpy(), 128))
        got = unpack_rows(gout[y:y + 1].cpu().numpy().view(np.uint64), W)
        assert_same(got, want[y - lo:y - lo + 1], f"grey row {y}")
    del grey, gout
    torch.cuda.empty_cache()


def test_batch_with_extreme_images():
    """One persistent batch launch over a table that holds the tallest image
    (EDGE_MAX_HEIGHT rows of 64 pixels) and the widest one (3 rows of
    2^31 - 1 pixels) between small crops: 64-bit arena offsets and millions
    of work units per image, with the host and the device planner."""
    import paper_1401_5245_amd as em
    from paper_1401_5245_amd import batch as B
    torch.cuda.empty_cache()
    tall, wide = _abi.EDGE_MAX_HEIGHT, 2**31 - 1
    shapes = [(5, 70), (tall, 64), (3, 33), (3, wide), (40, 257)]
    table = np.zeros(len(shapes), dtype=B.DESC_DTYPE)
    off = 0
    for i, (h, w) in enumerate(shapes):
        s = -(-w // 64)
        off = -(-off // 2) * 2                       # 16-byte aligned images
        table[i] = (off, h, w, s)
        off += h * s
    total = -(-off // 2) * 2
    log(f"batch with extreme images: {total} words")
    B.check_table(table, total, 64)
    inp = random_words((total,))
    out = torch.zeros_like(inp)
    table_dev = B.table_to_device(table)
    ws = torch.zeros(-(-B.batch_workspace_bytes(len(table)) // 8), dtype=torch.int64,
                     device="cuda")

    def image(t, i):
        o, h, s = int(table[i]["offset_words"]), int(table[i]["height"]), int(table[i]["stride_words"])
        return t[o:o + h * s].view(h, s)

    for plan in ("host", "device"):
        out.zero_()
        if plan == "host":
            words, used = B.plan_batch(inp, out, table)
            ws[:-(-used // 8)].copy_(torch.from_numpy(words[:-(-used // 8)]))
        em.edge_batch(inp, out, table_dev, len(table), ws, planned=plan == "host")
        torch.cuda.synchronize()
        for i in (0, 2, 4):
            h, w = shapes[i]
            want = oracle.edge(unpack_rows(image(inp, i).cpu().numpy().view(np.uint64), w))
            got = unpack_rows(image(out, i).cpu().numpy().view(np.uint64), w)
            assert_same(got, want, f"{plan} plan: crop {i}")
        ti, to = image(inp, 1), image(out, 1)
        for y in (0, 1, tall // 2, tall - 2, tall - 1):
            lo, hi = max(0, y - 1), min(tall, y + 2)
            want = oracle.edge(unpack_rows(ti[lo:hi].cpu().numpy().view(np.uint64), 64))
            got = unpack_rows(to[y:y + 1].cpu().numpy().view(np.uint64), 64)
            assert_same(got, want[y - lo:y - lo + 1], f"{plan} plan: tall image row {y}")
        wi, wo = image(inp, 3), image(out, 3)
        wd = wi.shape[1]
        for a, b in ((0, 2), (wd // 2 - 1, wd // 2 + 1), (wd - 2, wd)):
            lo, hi = max(0, a - 1), min(wd, b + 1)
            width = min(wide, 64 * hi) - 64 * lo
            x0, x1 = 64 * (a - lo), min(wide, 64 * b) - 64 * lo
            want = oracle.edge(unpack_rows(wi[:, lo:hi].cpu().numpy().view(np.uint64), width))
            got = unpack_rows(wo[:, lo:hi].cpu().numpy().view(np.uint64), width)
            assert_same(got[:, x0:x1], want[:, x0:x1], f"{plan} plan: wide image words {a}..{b}")
    del inp, out
    torch.cuda.empty_cache()
