"""Batched path (planner + persistent kernel, HIP graph) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from synth import images, pack_rows, unpack_rows
from tests.gpu_util import CLAUSES, assert_same, log

pytestmark = pytest.mark.gpu


def mixed_images(n, seed, side=(1, 700)):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        H = int(rng.integers(side[0], side[1] + 1))
        W = int(rng.integers(side[0], side[1] + 1))
        if i % 7 == 0:
            H = int(rng.integers(0, 3))      # includes empty images
        if i % 11 == 0:
            W = int(rng.integers(1, 40))     # narrow rows
        out.append(images.bernoulli_image(H, W, float(rng.uniform(0.1, 0.9)), seed + i))
    return out


def run_batch(imgs, word_bits, *, border="white", mode="masks", clause2_only=False,
              invert=False, cfg=None, pad="random", align_words=None, plan="host"):
    import paper_1401_5245_amd as em
    packed = [(pack_rows(im, word_bits, pad=pad, seed=i), im.shape[1]) for i, im in enumerate(imgs)]
    b = em.Batch(packed, word_bits, "cuda", border=border, mode=mode, clause2_only=clause2_only,
                 invert=invert, cfg=cfg, align_words=align_words, plan=plan)
    b.run()
    torch.cuda.synchronize()
    return b


def check_batch(b, imgs, **kw):
    host = b.out.cpu().numpy().view(np.uint64 if b.word_bits == 64 else np.uint32)
    for i, im in enumerate(imgs):
        if im.size == 0:
            continue
        got = unpack_rows(b.output_words(i, host), im.shape[1])
        want = oracle.edge(im, border=kw.get("border", "white"),
                           clauses=CLAUSES[(kw.get("mode", "masks"), kw.get("clause2_only", False))],
                           invert=kw.get("invert", False))
        assert_same(got, want, f"image {i} {im.shape}")


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("mode,c2,inv", [("masks", False, False), ("full", False, False),
                                         ("full", True, False), ("masks", False, True)])
@pytest.mark.parametrize("border", ["white", "black"])
@pytest.mark.parametrize("plan", ["host", "device"])
def test_mixed_batch_matches_oracle(word_bits, mode, c2, inv, border, plan):
    imgs = mixed_images(60, seed=word_bits + len(mode) + int(c2) + int(inv))
    log(f"batch B={word_bits} {mode} c2={c2} inv={inv} {border} plan={plan}")
    b = run_batch(imgs, word_bits, border=border, mode=mode, clause2_only=c2, invert=inv,
                  plan=plan)
    check_batch(b, imgs, border=border, mode=mode, clause2_only=c2, invert=inv)


def test_glyph_crops_batch():
    crops = images.glyph_crops(600, seed=3)
    b = run_batch(crops, 32, pad="zero")
    check_batch(b, crops)


@pytest.mark.parametrize("align", [1, 2])
def test_unaligned_offsets(align):
    imgs = mixed_images(40, seed=99, side=(30, 900))
    b = run_batch(imgs, 64, align_words=align)
    check_batch(b, imgs)


@pytest.mark.parametrize("vec", [1, 2, 4])
@pytest.mark.parametrize("rows", [1, 2, 5, 16])
@pytest.mark.parametrize("waves", [1, 4, 8])
@pytest.mark.parametrize("bpc", [1, 3, 8])
def test_batch_launch_configs(vec, rows, waves, bpc):
    imgs = mixed_images(25, seed=5, side=(1, 1500))
    cfg = dict(vec_words=vec, rows_per_tile=rows, waves_per_block=waves, blocks_per_cu=bpc,
               cache_policy=1)
    b = run_batch(imgs, 64, cfg=cfg, mode="full", clause2_only=(rows % 2 == 1),
                  plan="host" if (vec + rows + waves + bpc) % 2 else "device")
    check_batch(b, imgs, mode="full", clause2_only=(rows % 2 == 1))


def test_host_plan_graph_replays():
    """A host-planned batch captured in a graph: replays (with eager work in
    between) equal the eager launch, which equals the device-planned one."""
    imgs = mixed_images(50, seed=17, side=(1, 900))
    b = run_batch(imgs, 64, plan="host")
    d = run_batch(imgs, 64, plan="device")
    assert torch.equal(b.out, d.out)
    eager = b.out.clone()
    g = b.graph()
    for rep in range(4):
        b.out.zero_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(b.out, eager), f"replay {rep}"
    check_batch(b, imgs)


def test_batch_equals_single_image_path():
    import paper_1401_5245_amd as em
    imgs = mixed_images(30, seed=7, side=(1, 1200))
    b = run_batch(imgs, 64)
    host = b.out.cpu().numpy().view(np.uint64)
    for i, im in enumerate(imgs):
        if im.size == 0:
            continue
        words = pack_rows(im, 64)
        inp = torch.from_numpy(words.view(np.int64)).cuda()
        out = torch.zeros_like(inp)
        em.edge_masks(inp, out, *im.shape)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(b.output_words(i, host), out.cpu().numpy().view(np.uint64))


def test_graph_replays_with_eager_work_between():
    """Replay the captured batch several times; between replays run eager
    device work (clearing the output, unrelated kernels, a synchronize) and
    rewrite the descriptor table in place. Every replay must equal the
    eager result for the table it saw."""
    import paper_1401_5245_amd as em
    from paper_1401_5245_amd.batch import DESC_DTYPE
    imgs = mixed_images(40, seed=11, side=(10, 600))
    b = run_batch(imgs, 64, plan="device")     # the table is rewritten on the device below
    eager = b.out.clone()
    g = b.graph()
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(5):
        b.out.zero_()
        junk.mul_(1.0001).add_(0.5)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(b.out, eager), f"replay {rep} differs from the eager result"
    # rewrite the table in place: reverse the descriptor order (same images,
    # same arena), which changes the work plan the graph computes on device
    rev = np.ascontiguousarray(b.table[::-1]).view(np.int64).reshape(-1, 3)
    b.table_dev.copy_(torch.from_numpy(rev.copy()))
    b.out.zero_()
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(b.out, eager)
    # a table that drops half the images: their outputs stay untouched
    half = b.table.copy()
    half["height"][::2] = 0
    b.table_dev.copy_(torch.from_numpy(np.ascontiguousarray(half).view(np.int64).reshape(-1, 3)))
    b.out.zero_()
    g.launch()
    torch.cuda.synchronize()
    host = b.out.cpu().numpy().view(np.uint64)
    ref = eager.cpu().numpy().view(np.uint64)
    for i in range(len(imgs)):
        got = b.output_words(i, host)
        if i % 2 == 0:
            assert not got.any()
        else:
            np.testing.assert_array_equal(got, b.output_words(i, ref))
    assert DESC_DTYPE.itemsize == 24


def test_invalid_descriptor_is_skipped_on_device():
    import paper_1401_5245_amd as em
    from paper_1401_5245_amd.batch import table_to_device, batch_workspace_bytes
    imgs = mixed_images(6, seed=13, side=(5, 200))
    packed = [(pack_rows(im, 64), im.shape[1]) for im in imgs]
    arena, table = em.pack_arena(packed, 64)
    bad = table.copy()
    bad[2]["offset_words"] = arena.size * 4          # far outside the arena
    with pytest.raises(em.EdgeError):
        em.batch.check_table(bad, arena.size, 64)
    inp = torch.from_numpy(arena.view(np.int64)).cuda()
    out = torch.zeros_like(inp)
    tdev = table_to_device(bad)
    ws = torch.zeros(batch_workspace_bytes(len(bad)) // 8 + 1, dtype=torch.int64, device="cuda")
    em.edge_batch(inp, out, tdev, len(bad), ws)
    torch.cuda.synchronize()
    assert int(ws[1]) == 1                            # one descriptor skipped
    host = out.cpu().numpy().view(np.uint64)
    for i, im in enumerate(imgs):
        d = table[i]
        o, H, S = int(d["offset_words"]), int(d["height"]), int(d["stride_words"])
        got = unpack_rows(host[o:o + H * S].reshape(H, S), im.shape[1]) if H else None
        if i == 2 or H == 0:
            continue
        assert_same(got, oracle.edge(im), f"image {i}")


@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("mode", ["masks", "full"])
@pytest.mark.parametrize("plan", ["host", "device"])
def test_narrow_only_kernel_variant(word_bits, mode, plan):
    """vec_words = 1 selects the batch kernel built without wide strip paths
    (more wavefronts per compute unit): glyph crops mixed with a few wide
    images (one-word strips), many persistent workgroups."""
    from synth import images
    crops = images.glyph_crops(300, seed=21)
    imgs = list(crops) + mixed_images(6, seed=22, side=(300, 2500))
    for rows, bpc in ((4, 8), (8, 24), (1, 32)):
        cfg = dict(vec_words=1, rows_per_tile=rows, waves_per_block=4, blocks_per_cu=bpc,
                   cache_policy=1)
        b = run_batch(imgs, word_bits, mode=mode, cfg=cfg, plan=plan)
        check_batch(b, imgs, mode=mode)
