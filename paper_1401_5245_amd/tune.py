"""Autotuner for launch configurations (words per lane, rows per tile,
wavefronts per workgroup, persistent workgroups per CU, cache policy, strip,
tile or band shape).

Each candidate is timed on the device from a captured graph of repeated
launches (so host launch overhead does not decide), and is admitted only
when its output equals, bit for bit, a reference output: the expected words
the caller passes (its tests pass the CPU oracle's, packed), or else the
output of the library's built-in configuration on the same input. Winners
are cached in a JSON file keyed by GPU architecture, word size, mode and a
size class.
"""
from __future__ import annotations

import functools
import itertools
import json
import math
import os
import threading

import torch

from . import _abi

_lock = threading.Lock()

DEFAULT_CACHE = os.environ.get(
    "EDGEMASK_TUNE_CACHE",
    os.path.join(os.path.expanduser("~"), ".cache", "edgemask", "tune.json"))
SHIPPED_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")


@functools.lru_cache(maxsize=None)
def arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def size_class(height: int, width: int, word_bits: int) -> str:
    """Coarse shape bucket: log2 of the 32-bit words per row and of the rows."""
    wd32 = max(1, -(-width // word_bits) * (word_bits // 32))
    return f"w{int(math.log2(wd32))}_h{int(math.log2(max(1, height)))}"


def image_key(height, width, word_bits, mode="masks") -> str:
    return f"{arch()}|image|B{word_bits}|{mode}|{size_class(height, width, word_bits)}"


def batch_key(n_images, total_words, word_bits, mode="masks") -> str:
    return (f"{arch()}|batch|B{word_bits}|{mode}|n{int(math.log2(max(1, n_images)))}"
            f"_s{int(math.log2(max(1, total_words)))}")


_shared = None


def shared_cache() -> "TuneCache":
    """The process-wide table (shipped table + user cache), loaded once."""
    global _shared
    with _lock:
        if _shared is None:
            _shared = TuneCache()
        return _shared


class TuneCache:
    """JSON table of tuned configurations (shipped table + user cache)."""

    def __init__(self, path: str = DEFAULT_CACHE):
        self.path = path
        self.table = {}
        for p in (SHIPPED_TABLE, path):
            if os.path.exists(p):
                with open(p) as f:
                    self.table.update(json.load(f))

    def get(self, key):
        return self.table.get(key, {}).get("cfg")

    def put(self, key, cfg, us, candidates):
        self.table[key] = {"cfg": cfg, "us": round(us, 3), "candidates": candidates}

    def save(self, path: str | None = None):
        path = path or self.path
        with _lock:
            os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
            tmp = path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)
            os.replace(tmp, path)


def _graph_time_us(fn, launches: int, reps: int) -> float:
    """Device time per call of fn, from a graph of `launches` calls."""
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        for _ in range(launches):
            fn()
    g.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        g.replay()
    b.record()
    b.synchronize()
    del g
    return a.elapsed_time(b) * 1e3 / (reps * launches)


def image_candidates(height: int, width: int, word_bits: int):
    wd32 = -(-width // word_bits) * (word_bits // 32)
    if wd32 <= 32:
        for rows, waves in itertools.product((1, 2, 4, 8, 16), (1, 2, 4, 8)):
            yield dict(vec_words=1, rows_per_tile=rows, waves_per_block=waves, blocks_per_cu=1,
                       cache_policy=1)
        return
    for vec, rows, waves, cache in itertools.product((2, 4), (2, 4, 8, 16, 32, 64, 128, 256),
                                                     (2, 4, 8), (1, 2)):
        if rows > max(2, height):
            continue
        yield dict(vec_words=vec, rows_per_tile=rows, waves_per_block=waves, blocks_per_cu=1,
                   cache_policy=cache, shape=_abi.EDGE_SHAPE_STRIP)
    # tiles (all rows of a unit requested at once), in dispatch order or
    # regrouped by XCD
    for vec, rows, waves, shape in itertools.product(
            (2, 4), (4, 8, 16), (2, 4, 8), (_abi.EDGE_SHAPE_TILE, _abi.EDGE_SHAPE_TILE_XCD)):
        if rows > max(4, height):
            continue
        yield dict(vec_words=vec, rows_per_tile=rows, waves_per_block=waves, blocks_per_cu=1,
                   cache_policy=0, shape=shape)
    # bands (a workgroup's rows staged in LDS)
    for vec, rows, waves, shape in itertools.product(
            (2, 4), (1, 2, 4), (4, 8), (_abi.EDGE_SHAPE_BAND, _abi.EDGE_SHAPE_BAND_XCD)):
        if waves * rows > max(4, height + 2):
            continue
        yield dict(vec_words=vec, rows_per_tile=rows, waves_per_block=waves, blocks_per_cu=1,
                   cache_policy=0, shape=shape)


def _rotate_time_us(fns, reps: int) -> float:
    """Device time per launch of a graph that calls each of fns once."""
    return _graph_time_us(lambda: [f() for f in fns], 1, reps) / len(fns)


def tune_image(inp, out, height, width, *, mode="masks", border="white", candidates=None,
               cache: TuneCache | None = None, launches=20, reps=3, cold_bytes=512 << 20,
               reference=None, verbose=False, finalists_n=3, finalist_rounds=4):
    """Time every candidate on (inp, out) whose output equals `reference` (a
    tensor like `out` holding the expected words, the words out of the
    image's rows zero), or when it is None the output of the built-in
    configuration; time the `finalists_n` fastest `finalist_rounds` more
    times each and keep the one with the lowest median. Returns (cfg,
    microseconds).

    Timing rotates over copies of the buffers until `cold_bytes` are
    touched per round, so images smaller than the last-level cache are
    timed from HBM, as a stream of distinct images would be."""
    import paper_1401_5245_amd as em
    if reference is None:
        out.zero_()
        em.edge_image(inp, out, height, width, mode=mode, border=border)
        torch.cuda.synchronize()
        ref = out.clone()
    else:
        if reference.shape != out.shape or reference.dtype != out.dtype:
            raise ValueError("reference must match out in shape and type")
        ref = reference.to(out.device)
    per_pair = 2 * inp.numel() * inp.element_size()
    copies = max(1, min(launches, -(-cold_bytes // per_pair)))
    ins = [inp] + [inp.clone() for _ in range(copies - 1)]
    outs = [out] + [torch.empty_like(out) for _ in range(copies - 1)]
    timed, tried = [], 0
    cands = list(candidates) if candidates is not None else list(
        image_candidates(height, width, em.word_bits_of(inp)))

    def time_us(c):
        fns = [(lambda i=i: em.edge_image(ins[i], outs[i], height, width, mode=mode,
                                          border=border, cfg=c)) for i in range(copies)]
        return _rotate_time_us(fns * max(1, launches // copies), reps)

    for c in cands:
        out.zero_()
        em.edge_image(inp, out, height, width, mode=mode, border=border, cfg=c)
        torch.cuda.synchronize()
        if not torch.equal(out, ref):
            if verbose:
                print("rejected (output differs):", c)
            continue
        us = time_us(c)
        tried += 1
        if verbose:
            print(f"{us:9.2f} us  {c}")
        timed.append((us, c))
    if not timed:
        raise RuntimeError("no candidate configuration matched the reference output")
    # one timing can flatter a shape whose speed varies from launch to
    # launch: the fastest few are timed again, in turn, and the best median
    # of all their timings wins
    ranked = sorted(timed, key=lambda t: t[0])[:finalists_n]
    finalists = [c for _, c in ranked]
    runs = {i: [us] for i, (us, _) in enumerate(ranked)}
    for _ in range(finalist_rounds):
        for i, c in enumerate(finalists):
            runs[i].append(time_us(c))
    medians = {i: sorted(v)[len(v) // 2] for i, v in runs.items()}
    pick = min(medians, key=medians.get)
    best, best_us = finalists[pick], medians[pick]
    if verbose:
        for i, c in enumerate(finalists):
            print(f"finalist {medians[i]:9.2f} us (of {[round(x, 2) for x in runs[i]]})  {c}")
    if cache is not None:
        cache.put(image_key(height, width, em.word_bits_of(inp), mode), best, best_us, tried)
    return best, best_us


def batch_candidates():
    # vec 1 builds the batch kernel without its wide strip paths (fewer
    # registers, more wavefronts per compute unit): best for small crops
    for vec, rows, waves, bpc in itertools.product((1, 4), (1, 2, 4, 8, 16), (1, 2, 4, 8),
                                                   (4, 8, 12, 16, 24, 32)):
        yield dict(vec_words=vec, rows_per_tile=rows, waves_per_block=waves, blocks_per_cu=bpc,
                   cache_policy=1)


def tune_batch(batch, *, candidates=None, cache: TuneCache | None = None, launches=10, reps=3,
               reference=None, verbose=False):
    """Tune the persistent batch launch of a Batch (its table and arenas):
    keep the fastest candidate whose output arena equals `reference` (a
    tensor like batch.out, zero outside the images' rows), or when it is
    None the output of the built-in configuration. Returns (cfg,
    microseconds per batched launch)."""
    from .batch import edge_batch, plan_batch
    kw = dict(batch.kw)
    kw.pop("cfg", None)
    kw.pop("planned", None)
    if reference is None:
        batch.out.zero_()
        edge_batch(batch.inp, batch.out, batch.table_dev, batch.n, batch.workspace, **kw)
        torch.cuda.synchronize()
        ref = batch.out.clone()
    else:
        if reference.shape != batch.out.shape or reference.dtype != batch.out.dtype:
            raise ValueError("reference must match the output arena in shape and type")
        ref = reference.to(batch.out.device)
    best, best_us, tried = None, float("inf"), 0
    ws = batch.workspace
    for c in (list(candidates) if candidates is not None else list(batch_candidates())):
        # each candidate gets its own host plan; the timed launches are the
        # persistent kernel alone, as Batch runs them
        words, used = plan_batch(batch.inp, batch.out, batch.table, mode=kw.get("mode", "masks"),
                                 cfg=c)
        ws[:-(-used // 8)].copy_(torch.from_numpy(words[:-(-used // 8)]))
        kw["planned"] = True
        batch.out.zero_()
        edge_batch(batch.inp, batch.out, batch.table_dev, batch.n, ws, cfg=c, **kw)
        torch.cuda.synchronize()
        if not torch.equal(batch.out, ref):
            if verbose:
                print("rejected (output differs):", c)
            continue
        us = _graph_time_us(lambda: edge_batch(batch.inp, batch.out, batch.table_dev, batch.n,
                                               ws, cfg=c, **kw), launches, reps)
        tried += 1
        if verbose:
            print(f"{us:9.2f} us  {c}")
        if us < best_us:
            best, best_us = c, us
    # leave the batch's own plan in its workspace again
    if batch.kw.get("planned"):
        words, used = plan_batch(batch.inp, batch.out, batch.table, mode=kw.get("mode", "masks"),
                                 cfg=batch.kw.get("cfg"))
        ws[:-(-used // 8)].copy_(torch.from_numpy(words[:-(-used // 8)]))
    if best is None:
        raise RuntimeError("no candidate configuration matched the reference output")
    if cache is not None:
        total = int(batch.inp.numel())
        cache.put(batch_key(batch.n, total, batch.word_bits, kw.get("mode", "masks")), best,
                  best_us, tried)
    return best, best_us


def lookup_image(height, width, word_bits, mode="masks", cache: TuneCache | None = None):
    cache = cache or shared_cache()
    return cache.get(image_key(height, width, word_bits, mode))


def lookup_batch(n_images, total_words, word_bits, mode="masks", cache: TuneCache | None = None):
    cache = cache or shared_cache()
    return cache.get(batch_key(n_images, total_words, word_bits, mode))


def _main(argv=None):
    """Tune the benchmark's workloads on this GPU and write a table."""
    import argparse
    import numpy as np
    import paper_1401_5245_amd as em
    ap = argparse.ArgumentParser(description="tune libedgemask launch configurations")
    ap.add_argument("--out", default=DEFAULT_CACHE,
                    help="JSON table to write (default: the user cache, %(default)s)")
    ap.add_argument("--seed", type=int, default=0, help="seed of the random test images")
    ap.add_argument("--verbose", action="store_true", help="print every candidate's time")
    ap.add_argument("--squares", default="",
                    help="comma-separated sides of square uint64 plain-method images to tune "
                         "instead of the default workloads (no batch)")
    ap.add_argument("--batch-only", action="store_true",
                    help="tune only the batch of 4096 glyph crops")
    a = ap.parse_args(argv)
    cache = TuneCache(a.out)
    rng = np.random.default_rng(a.seed)
    shapes = ((512, 512, 32, "masks"), (8192, 8192, 64, "masks"),
              (16384, 16384, 64, "full"), (65536, 65536, 64, "masks"))
    if a.squares:
        shapes = tuple((int(v), int(v), 64, "masks") for v in a.squares.split(","))
    if a.batch_only:
        shapes = ()
    for (H, W, wb, mode) in shapes:
        words = -(-W // wb) * (wb // 32) * H
        inp = torch.from_numpy(rng.integers(0, 2**31, size=words, dtype=np.int64)
                               .astype(np.int32)).cuda()
        if wb == 64:
            inp = inp.view(torch.int64)
        inp = inp.view(H, -1)
        out = torch.empty_like(inp)
        cfg, us = tune_image(inp, out, H, W, mode=mode, cache=cache, verbose=a.verbose,
                             launches=4 if H >= 65536 else 20)
        print(f"image {H}x{W} B{wb} {mode}: {us:.2f} us  {cfg}", flush=True)
        del inp, out
        torch.cuda.empty_cache()
    if a.squares:
        cache.save(a.out)
        print("wrote", a.out)
        return
    from synth import images, pack_rows
    crops = images.glyph_crops(4096, seed=3)
    b = em.Batch([(pack_rows(c, 32), c.shape[1]) for c in crops], 32)
    cfg, us = tune_batch(b, cache=cache, verbose=a.verbose)
    print(f"batch 4096 crops: {us:.2f} us  {cfg}", flush=True)
    cache.save(a.out)
    print("wrote", a.out)


if __name__ == "__main__":
    _main()


__all__ = ["TuneCache", "tune_image", "tune_batch", "lookup_image", "lookup_batch",
           "image_candidates", "batch_candidates", "_abi"]
