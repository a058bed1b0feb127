"""Single-image entry points captured in a HIP graph (as the benchmark
times them) and replayed several times, with eager work and
synchronisation between replays: every replay must equal the eager
result."""
import numpy as np
import pytest
import torch

from synth import images, pack_rows
from tests.gpu_util import log, to_device_words

pytestmark = pytest.mark.gpu


def test_captured_launches_replay_exactly():
    import paper_1401_5245_amd as em
    H, W = 700, 3000
    img = images.glyph_page(H, W, seed=12, noise=0.01)
    grey = images.grey_image(H, W, seed=13)
    inp = to_device_words(pack_rows(img, 64))
    gt = torch.from_numpy(grey).cuda()
    flat = np.zeros(5 + (H - 1) * (W + 3) + W, np.uint8)    # rows off 16-byte boundaries
    for y in range(H):
        flat[5 + y * (W + 3):5 + y * (W + 3) + W] = grey[y]
    gu = torch.from_numpy(flat).cuda()[5:]
    outs = {k: torch.empty_like(inp)
            for k in ("masks", "full", "thr", "thr_unaligned", "pack", "peel", "layer")}
    planes = torch.empty((4,) + tuple(inp.shape), dtype=inp.dtype, device="cuda")

    def launches():
        em.edge_masks(inp, outs["masks"], H, W)
        em.edge_full(inp, outs["full"], H, W)
        em.edge_directions(inp, planes, H, W)
        em.threshold_edges(gt, outs["thr"], H, W, 128)
        em.threshold_edges(gu, outs["thr_unaligned"], H, W, 128, grey_stride=W + 3)
        em.threshold_pack(gu, outs["pack"], H, W, 128, grey_stride=W + 3)
        em.peel(inp, outs["peel"], H, W, 6)
        em.peel(inp, outs["layer"], H, W, 6, edge_out=True)

    launches()
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in outs.items()}
    ref_planes = planes.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        launches()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        launches()
    scratch = torch.empty_like(inp)
    for rep in range(5):
        log(f"replay {rep}")
        for v in outs.values():
            v.fill_(-1)
        planes.fill_(-1)
        em.edge_masks(inp, scratch, H, W)          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in outs.items():
            assert torch.equal(v, ref[k]), f"replay {rep}: {k}"
        assert torch.equal(planes, ref_planes), f"replay {rep}: planes"
        assert torch.equal(scratch, ref["masks"])
    assert torch.equal(ref["thr"], ref["thr_unaligned"])
    del g
