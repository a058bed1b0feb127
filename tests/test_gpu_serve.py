"""Serving: every result is the same alone and in the mix, under budget
pressure, in both batched and per-request modes."""
import numpy as np
import pytest
import torch

import oracle
from synth import images, pack_rows, unpack_rows
from tests.gpu_util import assert_same, log

pytestmark = pytest.mark.gpu


def make_pool(n=24, seed=21, side=(16, 600)):
    from paper_1401_5245_amd.serve import Pool
    rng = np.random.default_rng(seed)
    imgs = []
    for i in range(n):
        H, W = (int(v) for v in rng.integers(side[0], side[1] + 1, size=2))
        imgs.append(images.glyph_page(H, W, seed=seed + i, noise=0.01) if i % 2 == 0 else
                    images.bernoulli_image(H, W, 0.3, seed + i))
    pool = Pool.from_images([(pack_rows(im, 64), im.shape[1]) for im in imgs], 64)
    return imgs, pool


def alone(img):
    import paper_1401_5245_amd as em
    words = pack_rows(img, 64)
    inp = torch.from_numpy(words.view(np.int64)).cuda()
    out = torch.zeros_like(inp)
    em.edge_masks(inp, out, *img.shape)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("per_request", [False, True])
@pytest.mark.parametrize("budget_kib", [64, 4096])
@pytest.mark.parametrize("copy", ["sdma", "kernel"])
def test_results_same_alone_and_in_mix(per_request, budget_kib, copy):
    from paper_1401_5245_amd.serve import Server, poisson_arrivals
    imgs, pool = make_pool()
    singles = [alone(im) for im in imgs]
    n = 150
    arrivals = poisson_arrivals(n, 20000.0, seed=1)
    idx = np.random.default_rng(2).integers(0, len(imgs), size=n)
    budget = budget_kib << 10
    maxw = max(pool.words(i) for i in range(len(imgs)))
    need = (maxw + maxw % 2) * 8 * 2          # blocks are rounded to 16 bytes
    if need > budget:   # keep every request servable under the small budget
        budget = need
    srv = Server(pool, budget, max_inflight=3, copy=copy)
    log(f"serve per_request={per_request} budget={budget} copy={copy}")
    st = srv.run(arrivals, idx, per_request=per_request, record_outputs=True)
    assert st.rejected == 0 and st.latencies_ms.size == n
    outs = st.extra["outputs"]
    # every request's own output slice: equal to the image run alone, and
    # every pool image's edge map equal to the oracle's
    wants = [oracle.edge(im) for im in imgs]
    for i in range(len(imgs)):
        assert_same(unpack_rows(singles[i], imgs[i].shape[1]), wants[i], f"image {i} alone")
    for r in range(n):
        i = int(idx[r])
        got = outs[r].numpy().view(np.uint64).reshape(singles[i].shape)
        np.testing.assert_array_equal(got, singles[i], err_msg=f"request {r} (image {i})")
        assert_same(unpack_rows(got, imgs[i].shape[1]), wants[i], f"request {r} (image {i})")
    s = st.summary()
    assert s["p50_ms"] > 0 and s["p99_ms"] >= s["p50_ms"]
    if not per_request and budget_kib == 4096:
        assert s["batches"] < n      # arrivals were batched


def test_oversize_request_is_rejected_others_served():
    from paper_1401_5245_amd.serve import Server, poisson_arrivals
    imgs, pool = make_pool(n=6, seed=31, side=(20, 200))
    big = max(range(len(imgs)), key=pool.words)
    budget = (pool.words(big) - 2) * 8 * 2      # the largest image does not fit
    srv = Server(pool, budget)
    idx = np.arange(len(imgs))
    st = srv.run(poisson_arrivals(len(idx), 1000.0, seed=3), idx, record_outputs=True)
    assert st.rejected == 1
    assert st.latencies_ms.size == len(imgs) - 1
    for r, i in enumerate(idx):
        if i == big:
            assert st.extra["outputs"][r] is None
            continue
        got = st.extra["outputs"][r].numpy().view(np.uint64)
        np.testing.assert_array_equal(got.reshape(-1), alone(imgs[i]).reshape(-1))
