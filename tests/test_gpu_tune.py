"""The autotuner on small shapes with short candidate lists, gated by the
oracle's output; its JSON table round trip; and every launch shape in the
shipped table run against the oracle."""
import json

import numpy as np
import pytest
import torch

import oracle
from synth import images, pack_rows, row_words, unpack_rows
from tests.gpu_util import CLAUSES, assert_same, log

pytestmark = pytest.mark.gpu

_DT = {32: np.int32, 64: np.int64}


def _device(words):
    return torch.from_numpy(words.view(_DT[words.dtype.itemsize * 8]).copy()).cuda()


def _expected_words(img, word_bits, stride, **kw):
    """The oracle's edge map packed like the kernels' output (pad bits and
    stride words zero)."""
    return _device(pack_rows(oracle.edge(img, **kw), word_bits, stride, pad="zero"))


IMAGE_CANDIDATES = [
    dict(vec_words=2, rows_per_tile=2, waves_per_block=4, blocks_per_cu=1, cache_policy=1),
    dict(vec_words=4, rows_per_tile=8, waves_per_block=4, blocks_per_cu=1, cache_policy=2),
    dict(vec_words=4, rows_per_tile=32, waves_per_block=8, blocks_per_cu=1, cache_policy=1),
]


@pytest.mark.parametrize("mode", ["masks", "full"])
def test_tune_image_oracle_gate_and_table_round_trip(tmp_path, mode):
    import paper_1401_5245_amd as em
    from paper_1401_5245_amd import tune
    H, W = 300, 3 * 16384 + 37
    img = images.glyph_page(H, W, seed=41, noise=0.01)
    S = row_words(W, 64) + row_words(W, 64) % 2
    inp = _device(pack_rows(img, 64, S, pad="random", seed=5))
    out = torch.zeros_like(inp)
    clauses = CLAUSES[(mode, False)]
    ref = _expected_words(img, 64, S, clauses=clauses)
    path = str(tmp_path / "tune.json")
    cache = tune.TuneCache(path)
    log(f"tune_image {H}x{W} {mode}")
    cfg, us = tune.tune_image(inp, out, H, W, mode=mode, candidates=IMAGE_CANDIDATES, cache=cache,
                              launches=4, reps=2, cold_bytes=0, reference=ref)
    assert cfg in IMAGE_CANDIDATES and us > 0
    # the winner, run on its own, gives the oracle's edge map
    out.fill_(-1)
    em.edge_image(inp, out, H, W, mode=mode, stride_words=S, cfg=cfg)
    torch.cuda.synchronize()
    assert_same(unpack_rows(out.cpu().numpy().view(np.uint64), W),
                oracle.edge(img, clauses=clauses), f"tuned {cfg}")
    # JSON round trip: a fresh table read from the file returns the winner
    cache.save()
    key = tune.image_key(H, W, 64, mode)
    assert tune.TuneCache(path).get(key) == cfg
    with open(path) as f:
        assert json.load(f)[key]["candidates"] == len(IMAGE_CANDIDATES)


def test_tune_image_rejects_every_candidate_against_a_wrong_reference():
    from paper_1401_5245_amd import tune
    H, W = 40, 5000
    img = images.bernoulli_image(H, W, 0.3, seed=42)
    S = row_words(W, 64)
    inp = _device(pack_rows(img, 64, S))
    out = torch.zeros_like(inp)
    ref = _expected_words(img, 64, S)
    ref.view(-1)[S * 7 + 3] ^= 1 << 9          # one wrong pixel inside the image
    with pytest.raises(RuntimeError, match="reference"):
        tune.tune_image(inp, out, H, W, candidates=IMAGE_CANDIDATES[:2], launches=2, reps=1,
                        cold_bytes=0, reference=ref)


def test_tune_batch_oracle_gate_and_table_round_trip(tmp_path):
    import paper_1401_5245_amd as em
    from paper_1401_5245_amd import tune
    crops = images.glyph_crops(300, seed=43)
    b = em.Batch([(pack_rows(c, 32, pad="random", seed=i), c.shape[1])
                  for i, c in enumerate(crops)], 32, "cuda")
    want_arena, _ = em.pack_arena([(pack_rows(oracle.edge(c), 32, pad="zero"), c.shape[1])
                                   for c in crops], 32)
    ref = torch.from_numpy(want_arena.view(np.int32).copy()).cuda()
    cands = [dict(vec_words=1, rows_per_tile=4, waves_per_block=4, blocks_per_cu=8,
                  cache_policy=1),
             dict(vec_words=4, rows_per_tile=8, waves_per_block=2, blocks_per_cu=4,
                  cache_policy=1)]
    path = str(tmp_path / "tune.json")
    cache = tune.TuneCache(path)
    log("tune_batch 300 crops")
    cfg, us = tune.tune_batch(b, candidates=cands, cache=cache, launches=4, reps=2, reference=ref)
    assert cfg in cands and us > 0
    # the batch's own plan is back in its workspace: its launch still matches
    b.out.zero_()
    b.run()
    torch.cuda.synchronize()
    assert torch.equal(b.out, ref)
    cache.save()
    assert tune.TuneCache(path).get(tune.batch_key(b.n, b.inp.numel(), 32)) == cfg


def _shipped():
    from paper_1401_5245_amd import tune
    with open(tune.SHIPPED_TABLE) as f:
        return sorted(json.load(f).items())


def test_every_shipped_launch_shape_matches_the_oracle():
    """Each shipped entry's launch shape, run on an image of its size
    class's row width (which picks the kernel: narrow units or strips) with
    a ragged last word, at most 150 rows tall (the height only sets the
    grid)."""
    import paper_1401_5245_amd as em
    for key, entry in _shipped():
        _, kind, b, mode, cls = key.split("|")
        wb, cfg = int(b[1:]), entry["cfg"]
        log(f"shipped {key}: {cfg}")
        if kind == "image":
            w_log, h_log = (int(v[1:]) for v in cls.split("_"))
            W = (3 << w_log) // 2 * 32 - 5         # 1.5 * 2^w 32-bit words per row
            H = min(1 << h_log, 150)
            img = images.glyph_page(H, W, seed=44, noise=0.01)
            S = row_words(W, wb) + row_words(W, wb) % (128 // wb)
            inp = _device(pack_rows(img, wb, S, pad="random", seed=6))
            for c2 in ((False, True) if mode == "full" else (False,)):
                out = torch.full_like(inp, -1)
                em.edge_image(inp, out, H, W, mode=mode, clause2_only=c2, stride_words=S,
                              cfg=cfg)
                torch.cuda.synchronize()
                got = unpack_rows(out.cpu().numpy().view(np.uint64 if wb == 64 else np.uint32), W)
                assert_same(got, oracle.edge(img, clauses=CLAUSES[(mode, c2)]), f"{key} c2={c2}")
        else:
            crops = images.glyph_crops(400, seed=45)
            bt = em.Batch([(pack_rows(c, wb, pad="random", seed=i), c.shape[1])
                           for i, c in enumerate(crops)], wb, "cuda", mode=mode, cfg=cfg)
            bt.run()
            torch.cuda.synchronize()
            host = bt.out.cpu().numpy().view(np.uint64 if wb == 64 else np.uint32)
            for i, c in enumerate(crops):
                assert_same(unpack_rows(bt.output_words(i, host), c.shape[1]),
                            oracle.edge(c, clauses=CLAUSES[(mode, False)]), f"{key} crop {i}")
