"""edge_batch_noalloc (the batch entry point whose workspace is the
library's own fixed device array) against edge_batch with a caller
workspace, bit for bit, on calls in a row: the second call of each pair has
fewer and smaller images than the first, so it runs on the array the first
call left behind. Both outputs are also compared with the oracle."""
import numpy as np
import pytest
import torch

import oracle
from synth import images, pack_rows, unpack_rows
from tests.gpu_util import CLAUSES, assert_same, log

pytestmark = pytest.mark.gpu

_NP = {32: np.uint32, 64: np.uint64}


def _arena(imgs, word_bits):
    import paper_1401_5245_amd as em
    from paper_1401_5245_amd.batch import table_to_device
    packed = [(pack_rows(im, word_bits, pad="random", seed=i), im.shape[1])
              for i, im in enumerate(imgs)]
    arena, table = em.pack_arena(packed, word_bits)
    host = torch.from_numpy(arena.view(np.int64 if word_bits == 64 else np.int32))
    inp = host.cuda()
    return inp, table, table_to_device(table, "cuda")


def _outputs(out, table, imgs, word_bits):
    host = out.cpu().numpy().view(_NP[word_bits])
    res = []
    for d, im in zip(table, imgs):
        o, H, S = int(d["offset_words"]), int(d["height"]), int(d["stride_words"])
        res.append(unpack_rows(host[o:o + H * S].reshape(H, S), im.shape[1]))
    return res


def _one_call(imgs, word_bits, mode, c2):
    import paper_1401_5245_amd as em
    inp, table, tdev = _arena(imgs, word_bits)
    n = len(imgs)
    ref = torch.full_like(inp, 0x5A)
    got = torch.full_like(inp, 0x5A)
    ws = torch.zeros(-(-em.batch_workspace_bytes(n) // 8), dtype=torch.int64, device="cuda")
    em.edge_batch(inp, ref, tdev, n, ws, mode=mode, clause2_only=c2)
    em.edge_batch_noalloc(inp, got, tdev, n, mode=mode, clause2_only=c2)
    torch.cuda.synchronize()
    # the whole arena, stride and alignment gaps included, equals edge_batch's
    assert torch.equal(got, ref), "edge_batch_noalloc differs from edge_batch"
    for i, (g, im) in enumerate(zip(_outputs(got, table, imgs, word_bits), imgs)):
        assert_same(g, oracle.edge(im, clauses=CLAUSES[(mode, c2)]), f"image {i} {im.shape}")


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("mode,c2", [("masks", False), ("full", True)])
def test_noalloc_equals_edge_batch_twice(word_bits, mode, c2):
    big = images.glyph_crops(300, seed=31)
    rng = np.random.default_rng(32)
    small = [images.bernoulli_image(int(rng.integers(1, 60)), int(rng.integers(1, 200)), 0.3, i)
             for i in range(17)]
    log(f"noalloc B={word_bits} {mode} c2={c2}: {len(big)} crops, then {len(small)} smaller")
    _one_call(big, word_bits, mode, c2)
    _one_call(small, word_bits, mode, c2)


def test_noalloc_largest_batch_then_one_image():
    from paper_1401_5245_amd import _abi
    rng = np.random.default_rng(33)
    n = _abi.EDGE_BATCH_NOALLOC_MAX_IMAGES
    imgs = [images.bernoulli_image(int(rng.integers(1, 9)), int(rng.integers(1, 70)), 0.4, i)
            for i in range(n)]
    log(f"noalloc: {n} tiny images, then one")
    _one_call(imgs, 32, "masks", False)
    _one_call(imgs[:1], 32, "masks", False)
    # one image more than the array holds: refused before any device work
    inp, _, tdev = _arena(imgs[:1], 32)
    out = torch.empty_like(inp)
    rc = _abi.load().edge_batch_noalloc(inp.data_ptr(), out.data_ptr(), inp.numel(),
                                        tdev.data_ptr(), n + 1, 32, 0, 0, 0, None, None)
    assert rc == _abi.EDGE_ERR_WORKSPACE
