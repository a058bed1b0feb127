#!/usr/bin/env python3
"""Edge Gpixel/s and fraction of HBM peak of the method-of-masks kernels on
one MI355X, with the CPU oracle timed beside them.

Headline workload: the full definition (clause 1 OR clause 2 of section 1)
on one 16384x16384 binary page packed in uint64 row words (seeded 1-pixel
skeleton lines and thick strokes, about 10% black, isolated pixels), white
border. One step = one edge_full launch over the whole image; steps rotate
over 10 input/output buffer pairs (640 MiB) so that every launch reads from
HBM rather than the 256 MB last-level cache. Exactly --steps launches are
timed, after a warm-up of at least --warmup launches and 20 ms.

The last line on stdout is ONE compact JSON line (the headline, its
roofline, the CPU baseline and a summary of the other workloads); the full
results of every section go to the --detail file; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "edge Gpixel/s & % HBM peak; batched/served vs plain, p50/p99 ms"


VERBOSE = False


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def vlog(*a):
    """Progress detail, printed with --verbose only (the default stderr stays
    a few lines long)."""
    if VERBOSE:
        log(*a)


def parse(argv=None):
    p = argparse.ArgumentParser(description=" ".join(__doc__.split("\n\n")[0].split()))
    p.add_argument("--gpus", type=int, default=1,
                   help="GPUs to use; only 1 is supported (the benchmark runs on one GPU)")
    p.add_argument("--steps", type=int, default=2000,
                   help="timed launches of the headline workload (exactly this many)")
    p.add_argument("--warmup", type=int, default=200,
                   help="untimed launches before the timed region (at least 20 ms of them)")
    p.add_argument("--headline-only", action="store_true",
                   help="time only the headline workload (no other configs, no CPU baseline)")
    p.add_argument("--quick", action="store_true",
                   help="headline, the summarised workloads and the CPU baseline only "
                        "(skip the sweeps and widened rows of the detail file)")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="length of the one-thread oracle sample (the cpu_baseline field)")
    p.add_argument("--detail", default=os.path.join(ROOT, "gpurun_out", "bench_detail.json"),
                   help="file the full results of every section are written to")
    p.add_argument("--verbose", action="store_true", help="per-step progress on stderr")
    p.add_argument("--serve-copy", choices=("sdma", "kernel"), default="kernel",
                   help="host copies of the server: the copy kernel (default) or hipMemcpyAsync")
    p.add_argument("--serve-only", action="store_true",
                   help="run only the serving sweep (prints its JSON)")
    p.add_argument("--batch-only", action="store_true",
                   help="run only the batched-crops workload (prints its JSON)")
    p.add_argument("--next-only", action="store_true",
                   help="run only the widened rows (prints their JSON)")
    p.add_argument("--only", type=lambda v: v.split(","),
                   help="comma-separated sections to run alone, printing their JSON "
                        "(for profiling): " + ", ".join(SECTIONS))
    return p.parse_args(argv)


def ensure_built():
    import __graft_entry__
    __graft_entry__.ensure_built()


class Timer:
    """HIP events on torch's current stream, the stream every launch uses."""

    def __init__(self, torch):
        self.torch = torch

    def kernel_ms(self, fn, n: int) -> float:
        """Mean duration of fn's launch alone: an event pair around each of
        n launches on the current stream (host gaps between launches are
        outside every pair)."""
        t = self.torch
        s = t.cuda.current_stream()
        ev = [(t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True))
              for _ in range(n)]
        for i in range(n):
            ev[i][0].record(s)
            fn(i)
            ev[i][1].record(s)
        ev[-1][1].synchronize()
        return sum(a.elapsed_time(b) for a, b in ev) / n

    def per_call_ms(self, fn, n: int) -> float:
        t = self.torch
        s = t.cuda.current_stream()
        a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        a.record(s)
        for i in range(n):
            fn(i)
        b.record(s)
        b.synchronize()
        return a.elapsed_time(b) / n


def words_tensor(torch, words):
    wb = words.dtype.itemsize * 8
    return torch.from_numpy(words.view(np.int64 if wb == 64 else np.int32).copy()).cuda()


PROFILE = os.path.join(ROOT, "profiles", "k_strip_full_16384x16384_u64.md")
# every kernel source of the library (a change to any of them voids the
# traffic figures of the profile summaries)
KERNEL_SOURCES = tuple(sorted(
    "paper_1401_5245_amd/csrc/" + f for f in os.listdir(os.path.join(ROOT, "paper_1401_5245_amd", "csrc"))
    if f.endswith((".hip", ".hpp"))))


def measured_traffic(path: str = PROFILE, index: int = 0):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary (its
    index-th counter table, for profiles covering several kernels), or None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", path) if os.sep not in path else path).read()
    except OSError:
        return None
    fields = {"traffic_bytes_per_launch": [], "kernel_source_sha256_16": []}
    for line in text.splitlines():
        key, _, value = line.partition(": ")
        if key in fields:
            fields[key].append(value.strip())
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if index >= len(fields["traffic_bytes_per_launch"]) or \
            fields["kernel_source_sha256_16"][index] != h.hexdigest()[:16]:
        return None
    return int(fields["traffic_bytes_per_launch"][index])


def roofline(bytes_per_launch: float, ms: float, traffic=None) -> dict:
    gbs = bytes_per_launch / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic}


def check_rows(img, out_words, width, rows, border="white", clauses=1):
    """Compare sampled output rows with the oracle run on windows of img."""
    import oracle
    from synth import unpack_rows
    got = unpack_rows(out_words[rows], width)
    want = oracle.edge_rows(img, 0, rows, img.shape[0], border=border, clauses=clauses)
    return bool(np.array_equal(got, want))


# ------------------------------------------------------------ workloads ----

def graph_of(torch, launch_all, nstreams: int = 1, fns=None):
    """Capture library launches into a graph.

    Either launch_all() issues them all on the current stream, or `fns` is a
    list of launches dealt round-robin over `nstreams` streams forked from
    and joined back to the capture stream (independent images may then
    overlap on the device). Returns the torch.cuda.CUDAGraph."""
    def issue():
        if fns is None:
            launch_all()
            return
        cs = torch.cuda.current_stream()
        side = [torch.cuda.Stream() for _ in range(nstreams - 1)]
        streams = [cs] + side
        for s in side:
            s.wait_stream(cs)
        for i, f in enumerate(fns):
            with torch.cuda.stream(streams[i % nstreams]):
                f()
        for s in side:
            cs.wait_stream(s)

    g = torch.cuda.CUDAGraph()
    warm = torch.cuda.Stream()
    warm.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(warm):
        issue()                 # warm-up outside capture
    torch.cuda.current_stream().wait_stream(warm)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        issue()
    torch.cuda.synchronize()
    return g


class StepTimer:
    """Times exactly `steps` launches on torch's current stream, the stream
    every launch runs on, cycling over the rotating buffer pairs: replayed
    from one captured graph, or (eager=True) issued from the host one call
    at a time, for kernels that take longer than a host call.

    Warm-up replays the graph (launches back to back whatever the host's
    speed, also under a tracing profiler) until at least `warmup` launches
    and `warm_ms` of them have run. Before each timed region a spin kernel
    keeps the GPU busy while the host submits the graph or the calls
    (eager: long enough for all of them, from the host time of one pass of
    the calls after the warm-up), so the two events bracket device time
    only: event -> launches -> event. A graph replay adds about 10 us per
    region (20 launches of the headline: 13.4 us per launch replayed, 13.1
    us issued; equal over 200)."""

    def __init__(self, torch, fns, steps: int, eager: bool = False):
        self.torch = torch
        self.steps = steps
        self.eager = eager
        self.seq = [fns[i % len(fns)] for i in range(steps)]
        self.graph = graph_of(torch, None, nstreams=1, fns=self.seq)
        self.sleep_cycles = self._calibrate_sleep()

    def _run(self):
        if self.eager:
            for f in self.seq:
                f()
        else:
            self.graph.replay()

    def _calibrate_sleep(self, target_ms: float = 0.5) -> int:
        t = self.torch
        if not hasattr(t.cuda, "_sleep"):
            return 0
        a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        n = 100000
        a.record()
        t.cuda._sleep(n)
        b.record()
        b.synchronize()
        ms = max(a.elapsed_time(b), 1e-3)
        return int(min(max(n * target_ms / ms, 1000), 1 << 30))

    def warm(self, warmup: int, warm_ms: float = 20.0) -> int:
        t = self.torch
        done, t0 = 0, time.perf_counter()
        while done < max(warmup, 1) or (time.perf_counter() - t0) * 1e3 < warm_ms:
            self.graph.replay()
            done += self.steps
            t.cuda.synchronize()
        if self.eager:
            # one pass of the calls, its host time sizing the spin: the spin
            # must outlast the host's submission of every call of a region
            if self.sleep_cycles:
                t.cuda._sleep(self.sleep_cycles)
            h0 = time.perf_counter()
            self._run()
            host_ms = (time.perf_counter() - h0) * 1e3
            t.cuda.synchronize()
            done += self.steps
            if self.sleep_cycles:
                need_ms = 1.5 * host_ms + 0.5
                self.sleep_cycles = int(min(self.sleep_cycles * max(1.0, need_ms / 0.5),
                                            1 << 31))
        return done

    def region_ms(self) -> float:
        """Milliseconds of one timed region (all `steps` launches)."""
        t = self.torch
        s = t.cuda.current_stream()
        a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        t.cuda.synchronize()
        if self.sleep_cycles:
            t.cuda._sleep(self.sleep_cycles)
        a.record(s)
        self._run()
        b.record(s)
        b.synchronize()
        return a.elapsed_time(b)

    def close(self):
        self.graph = None
        self.torch.cuda.synchronize()


HEAD_SIDE = 16384
HEAD_PAIRS = 10


def headline_full(torch, em, args) -> dict:
    """The headline: full definition on the 16384^2 skeleton page (seed 4),
    u64 rows, 10 rotating buffer pairs; whole-image parity of the full map
    and of the clause-2 diagnostic against the oracle."""
    from synth import images, pack_rows, unpack_rows
    import oracle
    from paper_1401_5245_amd import tune
    H = W = HEAD_SIDE
    log("headline: full definition, 16384x16384 skeleton page (seed 4), uint64")
    img = images.skeleton_page(H, W, seed=4)
    src = words_tensor(torch, pack_rows(img, 64))
    ins = [src] + [src.clone() for _ in range(HEAD_PAIRS - 1)]
    outs = [torch.empty_like(src) for _ in range(HEAD_PAIRS)]
    cfg = tune.lookup_image(H, W, 64, "full")          # autotuned entry (None: built-in)
    em.edge_image(ins[0], outs[0], H, W, mode="full", cfg=cfg)
    torch.cuda.synchronize()
    got = unpack_rows(outs[0].cpu().numpy().view(np.uint64), W)
    want_full = oracle.edge(img, clauses=oracle.CLAUSE1 | oracle.CLAUSE2)
    exact_full = bool(np.array_equal(got, want_full))
    em.edge_full(ins[0], outs[1], H, W, clause2_only=True)
    torch.cuda.synchronize()
    got2 = unpack_rows(outs[1].cpu().numpy().view(np.uint64), W)
    want2 = oracle.edge(img, clauses=oracle.CLAUSE2)
    exact_c2 = bool(np.array_equal(got2, want2))
    n_clause2 = int(want2.sum())
    del got, got2, want2
    log(f"headline parity vs oracle (whole image): full {exact_full}, clause-2 {exact_c2} "
        f"({n_clause2} clause-2 pixels)")
    fns = [(lambda i=i: em.edge_image(ins[i], outs[i], H, W, mode="full", cfg=cfg))
           for i in range(HEAD_PAIRS)]
    st = StepTimer(torch, fns, args.steps, eager=True)
    warmed = st.warm(args.warmup)
    region = st.region_ms()                 # the timed region: exactly args.steps launches
    trials = [st.region_ms() / args.steps for _ in range(10)]
    st.close()
    replay_ok = args.steps < HEAD_PAIRS or all(bool(torch.equal(o, outs[0])) for o in outs[1:])
    ms = region / args.steps
    nbytes = 2 * H * (W // 64) * 8
    del ins, outs, src
    torch.cuda.empty_cache()
    return {"ms_per_step": ms, "region_ms": region, "warmup_launches": warmed,
            "trials_ms": trials, "bytes_per_step": nbytes, "pixels_per_step": H * W,
            "cfg": cfg, "bit_exact_full": exact_full, "bit_exact_clause2": exact_c2,
            "replays_equal": replay_ok, "clause2_pixels": n_clause2, "img": img}


def plain_8192(torch, em, tm, steps=4000, stream_counts=(1, 2, 4)):
    """Plain method on the 8192^2 glyph page (seed 2), u64 rows, 40 rotating
    buffer pairs; whole-image parity. Per-launch time of a one-stream graph
    (launches do not overlap), and graphs whose launches are dealt over 2 or
    4 streams (independent images may overlap) beside it."""
    from synth import images, pack_rows, unpack_rows
    import oracle
    from paper_1401_5245_amd import tune
    H = W = 8192
    NB = 40
    img = images.glyph_page(H, W, seed=2)
    src = words_tensor(torch, pack_rows(img, 64))
    ins = [src] + [src.clone() for _ in range(NB - 1)]
    outs = [torch.empty_like(src) for _ in range(NB)]
    cfg = tune.lookup_image(H, W, 64, "masks")
    em.edge_image(ins[0], outs[0], H, W, cfg=cfg)
    torch.cuda.synchronize()
    ref = outs[0].cpu().numpy().view(np.uint64)
    exact = bool(np.array_equal(unpack_rows(ref, W), oracle.edge(img)))
    fns = [(lambda i=i: em.edge_image(ins[i], outs[i], H, W, cfg=cfg)) for i in range(NB)]
    st = StepTimer(torch, fns, steps)
    st.warm(steps)
    trials = [st.region_ms() / steps for _ in range(5)]
    st.close()
    ms = float(np.median(trials))
    per_streams = {}
    for ns in stream_counts[1:]:
        g = graph_of(torch, None, nstreams=ns, fns=fns * 10)
        for _ in range(5):
            g.replay()
        per_streams[ns] = float(np.median([tm.per_call_ms(lambda i: g.replay(), 10) / (NB * 10)
                                           for _ in range(3)]))
        del g
    replay_ok = all(bool(torch.equal(o, outs[0])) for o in outs[1:])
    eager_ms = tm.per_call_ms(lambda i: em.edge_masks(ins[i % NB], outs[i % NB], H, W), 400)
    del ins, outs, src
    torch.cuda.empty_cache()
    nbytes = 2 * H * (W // 64) * 8
    return {"workload": "plain, 8192x8192 glyph page (seed 2, ~19% black, 0.5% salt-and-pepper), "
                        "uint64 rows, white border, 40 rotating buffer pairs, one-stream graph of "
                        f"{steps} launches",
            "launch_cfg": cfg or "built-in",
            "us_per_launch": round(ms * 1e3, 3), "gpx_s": round(H * W / (ms * 1e-3) / 1e9, 1),
            "roofline": roofline(nbytes, ms, measured_traffic("k_strip_plain_8192x8192_u64.md")),
            "bit_exact": exact and replay_ok,
            "trials_us": [round(t * 1e3, 3) for t in trials],
            "graph_streams_us_per_launch": {str(k): round(v * 1e3, 3)
                                            for k, v in per_streams.items()},
            "eager_python_us_per_launch": round(eager_ms * 1e3, 3)}


def copy_ceiling(torch, em, tm, nbytes, nb, steps):
    """GB/s (read + write) of the library's plain 128-bit copy over nb
    rotating buffer pairs of nbytes, launches replayed from a graph."""
    srcs = [torch.empty(nbytes // 8, dtype=torch.int64, device="cuda") for _ in range(nb)]
    dsts = [torch.empty_like(s) for s in srcs]
    for s in srcs:
        s.fill_(1)
    g = graph_of(torch, lambda: [em.copy_bytes(srcs[i], dsts[i], nbytes) for i in range(nb)])
    g.replay()
    reps = max(1, steps // nb)
    ms = tm.per_call_ms(lambda i: g.replay(), reps) / nb
    del srcs, dsts, g
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def launch_floor_ms(torch, em, tm, nl=40, reps=10, trials=7, warm=50):
    """Per-launch time of a near-empty kernel (the library's copy of 16
    bytes: one workgroup) replayed from a one-stream graph, launches back
    to back as the headline's are: the fixed cost any launch pays. (Issued
    one call at a time, a launch this short would be bound by the host.)
    Warmed up first (it may
    follow seconds of host-only work, after which the GPU idles at lower
    clocks) and the median of several trials."""
    a = torch.zeros(2, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    g = graph_of(torch, lambda: [em.copy_bytes(a, b, 16) for _ in range(nl)])
    for _ in range(warm):
        g.replay()
    ms = float(np.median([tm.per_call_ms(lambda i: g.replay(), reps) / nl
                          for _ in range(trials)]))
    del g
    return ms


def warm_by_time(torch, fn, ms=25.0):
    """Call fn (one launch) until about `ms` of device time has passed, at
    least 3 times: after seconds of host-only work (oracle checks) the GPU
    runs at lower clocks, and a few launches do not bring them back."""
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    fn()
    b.record(s)
    b.synchronize()
    for _ in range(max(3, int(ms / max(a.elapsed_time(b), 1e-3)))):
        fn()
    torch.cuda.synchronize()


def plain_512(torch, em, tm, steps):
    from synth import images, pack_rows, unpack_rows
    import oracle
    img, k = images.strokes_image(512, 512, seed=1)
    words = pack_rows(img, 32)
    inp = words_tensor(torch, words)
    out = torch.empty_like(inp)
    em.edge_image(inp, out, 512, 512, cfg="tuned")
    torch.cuda.synchronize()
    exact = bool(np.array_equal(unpack_rows(out.cpu().numpy().view(np.uint32), 512),
                                oracle.edge(img)))
    NL = 50
    g = graph_of(torch, lambda: [em.edge_image(inp, out, 512, 512, cfg="tuned")
                                 for _ in range(NL)])
    for _ in range(3):
        g.replay()
    reps = max(1, steps // NL)
    ms = tm.per_call_ms(lambda i: g.replay(), reps) / NL
    eager = tm.per_call_ms(lambda i: em.edge_masks(inp, out, 512, 512), steps)
    return {"workload": "plain, 512x512 strokes (seed 1, redraw k=%d), uint32" % k,
            "gpx_s": round(512 * 512 / (ms * 1e-3) / 1e9, 2), "us_per_launch": round(ms * 1e3, 2),
            "us_per_launch_eager_python": round(eager * 1e3, 2), "bit_exact": exact,
            "note": "latency-bound: 64 KiB per launch; graph-replayed launches"}


def plain_65536(torch, em, tm, steps):
    from synth import images, pack_rows, unpack_rows
    import oracle
    H = W = 65536
    log("building 65536x65536 page (8x8 tiles of an 8192^2 glyph page, seed 22)")
    tile_img = images.glyph_page(8192, 8192, seed=22)
    words = np.tile(pack_rows(tile_img, 64), (8, 8))
    inp = words_tensor(torch, words)
    del words
    out = torch.empty_like(inp)
    em.edge_image(inp, out, H, W, cfg="tuned")
    torch.cuda.synchronize()
    # image row y is tile row y % 8192 repeated 8 times across
    ok = True
    for r in (0, 1, 8191, 8192, 30000, 65534, 65535):
        lo, hi = max(0, r - 1), min(H, r + 2)
        win = np.tile(np.stack([tile_img[y % 8192] for y in range(lo, hi)]), (1, 8))
        want = oracle.edge(win)[r - lo]
        got = unpack_rows(out[r:r + 1].cpu().numpy().view(np.uint64), W)[0]
        ok &= bool(np.array_equal(got, want))
    warm_by_time(torch, lambda: em.edge_image(inp, out, H, W, cfg="tuned"))
    ms = tm.per_call_ms(lambda i: em.edge_image(inp, out, H, W, cfg="tuned"), steps)
    nbytes = 2 * H * (W // 64) * 8
    del inp, out
    torch.cuda.empty_cache()
    return {"workload": "plain, 65536x65536 tiled glyph page (seed 22), uint64, 1 GiB per launch",
            "gpx_s": round(H * W / (ms * 1e-3) / 1e9, 1), "ms_per_launch": round(ms, 4),
            "roofline": roofline(nbytes, ms, measured_traffic("k_band_plain_65536x65536_u64.md")),
            "sampled_rows_bit_exact": ok}


def full_65536(torch, em, tm, steps=10):
    """Full definition at 65536^2 (1 GiB each way: past every cache), the
    16384^2 skeleton page of seed 44 tiled 4x4; sampled rows of the full map
    and of the clause-2 diagnostic against the oracle on windows of the
    tiled image, and the plain method on the same image beside it."""
    from synth import images, pack_rows, unpack_rows
    import oracle
    H = W = 65536
    T = 16384
    log("full mode at 65536x65536 (4x4 tiles of a 16384^2 skeleton page, seed 44)")
    tile_img = images.skeleton_page(T, T, seed=44)
    words = np.tile(pack_rows(tile_img, 64), (4, 4))
    inp = words_tensor(torch, words)
    del words
    out = torch.empty_like(inp)
    rows = (0, 1, T - 1, T, 30000, H - 2, H - 1)

    def sampled_ok(clauses):
        ok = True
        for r in rows:
            lo, hi = max(0, r - 1), min(H, r + 2)
            win = np.tile(np.stack([tile_img[y % T] for y in range(lo, hi)]), (1, 4))
            want = oracle.edge(win, clauses=clauses)[r - lo]
            got = unpack_rows(out[r:r + 1].cpu().numpy().view(np.uint64), W)[0]
            ok &= bool(np.array_equal(got, want))
        return ok

    # one launch shape for the three modes (the plain method's tuned one),
    # so that their times differ only by what each mode computes
    from paper_1401_5245_amd import tune
    cfg = tune.lookup_image(H, W, 64, "masks")
    em.edge_image(inp, out, H, W, mode="full", clause2_only=True, cfg=cfg)
    torch.cuda.synchronize()
    ok2 = sampled_ok(oracle.CLAUSE2)
    res = {"workload": "65536x65536 tiled skeleton page (seed 44), uint64, 1 GiB per launch",
           "launch_cfg": cfg or "built-in"}
    nbytes = 2 * H * (W // 64) * 8
    for mode in ("full", "masks"):
        em.edge_image(inp, out, H, W, mode=mode, cfg=cfg)
        torch.cuda.synchronize()
        ok = sampled_ok(oracle.CLAUSE1 | (oracle.CLAUSE2 if mode == "full" else 0))
        warm_by_time(torch, lambda: em.edge_image(inp, out, H, W, mode=mode, cfg=cfg))
        ms = float(np.median([tm.per_call_ms(lambda i: em.edge_image(inp, out, H, W, mode=mode,
                                                                      cfg=cfg), steps)
                              for _ in range(3)]))
        key = "full" if mode == "full" else "plain"
        res[key] = {"ms_per_launch": round(ms, 4), "gpx_s": round(H * W / (ms * 1e-3) / 1e9, 1),
                    "roofline": roofline(nbytes, ms, measured_traffic(
                        "k_band_full_65536x65536_u64.md") if mode == "full" else None),
                    "sampled_rows_bit_exact": ok and (ok2 if mode == "full" else True)}
    res["full_vs_plain_time"] = round(res["full"]["ms_per_launch"] / res["plain"]["ms_per_launch"],
                                      4)
    # The full-mode kernel compiles to the plain kernel's instructions (the
    # compiler finds the second clause absorbed by the first); the clause-2
    # diagnostic evaluates the bit-sliced count in full, so its time is what
    # evaluating clause 2 costs on this image.
    def clause2(i=0):
        em.edge_image(inp, out, H, W, mode="full", clause2_only=True, cfg=cfg)

    warm_by_time(torch, clause2)
    ms2 = float(np.median([tm.per_call_ms(clause2, steps) for _ in range(3)]))
    res["clause2"] = {"ms_per_launch": round(ms2, 4), "roofline": roofline(nbytes, ms2),
                      "sampled_rows_bit_exact": ok2}
    res["clause2_vs_plain_time"] = round(ms2 / res["plain"]["ms_per_launch"], 4)
    del inp, out
    torch.cuda.empty_cache()
    return res


def next_rows_65536(torch, em, tm, steps=20):
    """Direction planes and the fused threshold -> edges at 65536^2, where
    every launch streams from HBM (2.7 GB and 4.8 GB per launch); sampled
    rows against the oracle on windows."""
    from synth import images, pack_rows, unpack_rows
    import oracle
    H = W = 65536
    rows = (0, 1, 8191, 8192, 30000, 65534, 65535)

    def window(tile, r):
        lo, hi = max(0, r - 1), min(H, r + 2)
        return lo, np.tile(np.stack([tile[y % 8192] for y in range(lo, hi)]), (1, 8))

    res = {}
    log("building 65536x65536 page (8x8 tiles of an 8192^2 glyph page, seed 22)")
    tile_img = images.glyph_page(8192, 8192, seed=22)
    words = np.tile(pack_rows(tile_img, 64), (8, 8))
    inp = words_tensor(torch, words)
    del words
    out4 = torch.empty((4,) + tuple(inp.shape), dtype=inp.dtype, device="cuda")
    em.edge_directions(inp, out4, H, W)
    torch.cuda.synchronize()
    ok = True
    for r in rows:
        lo, win = window(tile_img, r)
        fe = oracle.fundamental_edges(win)
        for p in range(4):
            got = unpack_rows(out4[p, r:r + 1].cpu().numpy().view(np.uint64), W)[0]
            ok &= bool(np.array_equal(got, fe[p][r - lo]))
    warm_by_time(torch, lambda: em.edge_directions(inp, out4, H, W))
    ms = tm.per_call_ms(lambda i: em.edge_directions(inp, out4, H, W), steps)
    nbytes = 5 * H * (W // 8)
    res["directions"] = {"workload": "65536x65536 tiled glyph page (seed 22), uint64: four "
                                     "fundamental-edge planes", "ms": round(ms, 4),
                         "roofline": roofline(nbytes, ms,
                                              measured_traffic("next_rows_65536x65536.md", 0)),
                         "sampled_rows_bit_exact": ok}
    del inp, out4
    torch.cuda.empty_cache()
    log("building 65536x65536 grey image (8x8 tiles of the 8192^2 grey image, seed 7)")
    grey_tile = images.grey_image(8192, 8192, seed=7)
    gt = torch.from_numpy(grey_tile).cuda().repeat(8, 8)       # 4 GiB of grey bytes
    out = torch.empty((H, W // 64), dtype=torch.int64, device="cuda")
    em.threshold_edges(gt, out, H, W, 128)
    torch.cuda.synchronize()
    binary_tile = oracle.threshold(grey_tile, 128)
    ok = True
    for r in rows:
        lo, win = window(binary_tile, r)
        got = unpack_rows(out[r:r + 1].cpu().numpy().view(np.uint64), W)[0]
        ok &= bool(np.array_equal(got, oracle.edge(win)[r - lo]))
    warm_by_time(torch, lambda: em.threshold_edges(gt, out, H, W, 128))
    ms = tm.per_call_ms(lambda i: em.threshold_edges(gt, out, H, W, 128), steps)
    nbytes = H * W + H * (W // 8)
    res["threshold_edges"] = {"workload": "65536x65536 tiled grey image (seed 7), threshold 128, "
                                          "uint64 out", "ms": round(ms, 4),
                              "gpx_s": round(H * W / (ms * 1e-3) / 1e9, 1),
                              "roofline": roofline(nbytes, ms,
                                                   measured_traffic("next_rows_65536x65536.md", 1)),
                              "sampled_rows_bit_exact": ok}
    del gt, out
    torch.cuda.empty_cache()
    return res


def batched_crops(torch, em, tm, steps):
    from synth import images, pack_rows, unpack_rows
    import oracle
    from paper_1401_5245_amd import _abi, tune
    log("generating 4096 glyph crops (seed 3)")
    crops = images.glyph_crops(4096, seed=3)
    b = em.Batch([(pack_rows(c, 32), c.shape[1]) for c in crops], 32, "cuda", cfg="tuned")
    g = b.graph()
    g.launch()
    torch.cuda.synchronize()
    host = b.out.cpu().numpy().view(np.uint32)
    exact = all(np.array_equal(unpack_rows(b.output_words(i, host), c.shape[1]), oracle.edge(c))
                for i, c in enumerate(crops))
    px = int(sum(c.size for c in crops))
    for _ in range(10):
        g.launch()
    ms_graph = tm.per_call_ms(lambda i: g.launch(), steps)
    ms_eager = tm.per_call_ms(lambda i: b.run(), steps)
    # baseline: one edge_masks launch per crop, same arenas, one stream
    lib = _abi.load()
    base_in, base_out = b.inp.data_ptr(), b.out.data_ptr()
    stream = int(torch.cuda.current_stream().cuda_stream)
    calls = [(base_in + int(d["offset_words"]) * 4, base_out + int(d["offset_words"]) * 4,
              int(d["height"]), int(d["width"]), int(d["stride_words"])) for d in b.table]

    def per_image(_):
        for (pi, po, h, w, s) in calls:
            lib.edge_masks(pi, po, h, w, s, 32, 0, stream)

    per_image(0)
    ms_plain = tm.per_call_ms(per_image, max(3, min(20, steps // 50)))
    # Device rates with the host out of the loop: one graph holding 20
    # launches of the batch, and one graph holding the 4096 per-crop
    # launches (each call above is one host submission, which a graph of
    # a single node does not make cheaper).
    from paper_1401_5245_amd.tune import _graph_time_us

    def per_image_here():
        st = int(torch.cuda.current_stream().cuda_stream)
        for (pi, po, h, w, s) in calls:
            lib.edge_masks(pi, po, h, w, s, 32, 0, st)

    us_graph20 = _graph_time_us(lambda: b.run(), 20, max(5, steps // 200))
    us_plain_graph = _graph_time_us(per_image_here, 1, 3)
    return {"workload": "batched, 4096 glyph crops H,W log-uniform [24,256] (seed 3), uint32, "
                        "%.1f Mpx" % (px / 1e6),
            "gpx_s_graph": round(px / (ms_graph * 1e-3) / 1e9, 1),
            "gpx_s_eager": round(px / (ms_eager * 1e-3) / 1e9, 1),
            "gpx_s_per_image_launches": round(px / (ms_plain * 1e-3) / 1e9, 2),
            "speedup_vs_per_image": round(ms_plain / ms_graph, 1),
            "us_graph": round(ms_graph * 1e3, 2),
            "us_per_launch_graph_of_20": round(us_graph20, 2),
            "gpx_s_graph_of_20": round(px / (us_graph20 * 1e-6) / 1e9, 1),
            "gpx_s_per_image_launches_in_one_graph": round(px / (us_plain_graph * 1e-6) / 1e9, 2),
            "speedup_graph_of_20_vs_per_image_graph": round(us_plain_graph / us_graph20, 1),
            "cfg": tune.lookup_batch(b.n, b.inp.numel(), 32) or em.default_cfg(0, 0, 32, batch=True),
            "bit_exact_all_crops": exact}


def host_link_ceiling(torch, nbytes=256 << 20, reps=5):
    """GB/s of pinned host <-> device copies on the serving path's copy call
    (hipMemcpyAsync): host to device, device to host, and both at once on
    two streams (each way)."""
    from paper_1401_5245_amd.serve import _copy_async
    n = nbytes // 8
    host_a = torch.empty(n, dtype=torch.int64).pin_memory()
    host_b = torch.empty(n, dtype=torch.int64).pin_memory()
    dev_a = torch.empty(n, dtype=torch.int64, device="cuda")
    dev_b = torch.empty(n, dtype=torch.int64, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    h2d = timed(lambda: _copy_async(dev_a, 0, host_a, 0, n, s1))
    d2h = timed(lambda: _copy_async(host_b, 0, dev_b, 0, n, s2))
    both = timed(lambda: (_copy_async(dev_a, 0, host_a, 0, n, s1),
                          _copy_async(host_b, 0, dev_b, 0, n, s2)))
    del host_a, host_b, dev_a, dev_b
    torch.cuda.empty_cache()
    return {"h2d_gbs": round(nbytes / h2d / 1e9, 1), "d2h_gbs": round(nbytes / d2h / 1e9, 1),
            "both_each_way_gbs": round(nbytes / both / 1e9, 1),
            "note": "256 MiB pinned copies with hipMemcpyAsync, host-timed"}


def sustained(runs, p99_bound_ms):
    """The highest offered rate below which every tested rate, itself
    included, met the p99 bound (runs in increasing rate order), and the
    rates that passed again above the first failure (reported, not taken)."""
    best, failed, later = None, False, []
    for st in runs:
        ok = st["p99_ms"] <= p99_bound_ms
        if ok and not failed:
            best = st
        elif ok:
            later.append(st["offered_rps"])
        else:
            failed = True
    return best, later


def serving(torch, em, p99_bound_ms=20.0, budget=4 << 30, copy="kernel"):
    """Poisson request stream over a 64-image pool (sides log-uniform in
    [64, 4096], half glyph pages, half Bernoulli(0.3)); sweep the offered
    rate for the batched server and the per-request-launch server; report
    the highest rate each sustains with p99 latency within the bound."""
    from synth import images, pack_rows, row_words
    from paper_1401_5245_amd.serve import Pool, Server, poisson_arrivals
    log("generating the serving pool (seed 5)")
    pool_imgs = images.serving_pool(64, seed=5)
    packed = []
    for im, _ in pool_imgs:
        wd = row_words(im.shape[1], 64)
        packed.append((pack_rows(im, 64, wd + wd % 2), im.shape[1]))
    pool = Pool.from_images(packed, 64)
    mean_px = float(pool.pixels.mean())
    srv = Server(pool, budget, max_inflight=3, copy=copy)
    rng = np.random.default_rng(55)
    out = {"workload": "serving: Poisson arrivals, 64-image pinned ingress ring (sides "
                       "log-uniform [64,4096], half glyph / half Bernoulli(0.3)), uint64; HBM "
                       "budget %d GiB, 3 batches in flight; latency = result in host memory "
                       "- scheduled arrival; host copies by %s" % (
                           budget >> 30, "the copy kernel" if copy == "kernel" else
                           "hipMemcpyAsync"),
           "mean_mpx_per_request": round(mean_px / 1e6, 3), "p99_bound_ms": p99_bound_ms}
    # steps of 20 000 req/s around the knee (about 85% of the batched
    # server's saturation rate), where doubling steps left the result to
    # whether one trial tipped into a growing queue
    for name, per_req, rates in (("batched", False, (1e4, 2e4, 4e4, 8e4, 1e5, 1.2e5, 1.4e5,
                                                     1.6e5, 2.4e5, 3.2e5, 4.8e5, 6.4e5)),
                                 ("per_request", True, (2e3, 5e3, 1e4, 1.5e4, 2e4, 3e4))):
        runs = []
        for rate in rates:
            n = int(min(max(400, rate * 0.3), 100000))
            trials = []
            for trial in range(2):
                arr = poisson_arrivals(n, rate, seed=int(rate) + trial)
                # the pool is an ingress ring: consecutive requests are
                # consecutive pool images (random sizes, random start)
                idx = (int(rng.integers(0, len(pool_imgs))) + np.arange(n)) % len(pool_imgs)
                srv.run(arr[:50], idx[:50], per_request=per_req)          # warm-up
                trials.append(srv.run(arr, idx, per_request=per_req).summary())
            st = max(trials, key=lambda t: t["p99_ms"])   # the worse of two trials
            st["offered_rps"] = rate
            st["trials_p99_ms"] = [t["p99_ms"] for t in trials]
            runs.append(st)
            st["trials_host_stall_ms"] = [max(t["max_loop_pass_ms"], t["max_oversleep_ms"])
                                          for t in trials]
            vlog(f"serve {name} rate={rate:.0f}/s p50={st['p50_ms']} p99={st['trials_p99_ms']} "
                 f"gpx_s={st['gpx_s']} batches={st['batches']} "
                 f"host stall ms={st['trials_host_stall_ms']} "
                 f"sections={[t['max_section_ms'] for t in trials]}")
        best, passes_above_failure = sustained(runs, p99_bound_ms)
        out[name] = {"runs": runs, "passing_rates_above_first_failure": passes_above_failure,
                     "max_sustained": None if best is None else {
                         "offered_rps": best["offered_rps"], "gpx_s": best["gpx_s"],
                         "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"],
                         "host_link_gbs_each_way": best["host_link_gbs_each_way"],
                         "stages_p50_p99": best["stages_p50_p99"]}}
    out["host_link_ceiling"] = host_link_ceiling(torch)
    log(f"host link: {out['host_link_ceiling']}")
    b, p = out["batched"]["max_sustained"], out["per_request"]["max_sustained"]
    if b and p:
        out["speedup_at_p99_bound"] = round(b["gpx_s"] / p["gpx_s"], 2)
    return out


def next_rows(torch, em, tm, steps):
    """The widened rows at 8192^2: the paper's unfused stages against the
    fused kernel, the four fundamental-edge planes, and thresholding a grey
    image (two passes against the fused pass). Every output is checked
    against the oracle on the whole image."""
    from synth import images, pack_rows, unpack_rows
    import oracle
    H = W = 8192
    img = images.glyph_page(H, W, seed=2)
    words = pack_rows(img, 64)
    inp = words_tensor(torch, words)
    out = torch.empty_like(inp)
    px = H * W
    packed_bytes = H * (W // 8)
    res = {}

    def graph_time(fns, reps):
        g = graph_of(torch, None, nstreams=1, fns=fns)
        g.replay()
        ms = tm.per_call_ms(lambda i: g.replay(), reps) / len(fns)
        del g
        return ms

    # NEXT-1: unfused stages
    scratch = torch.empty(em.staged_scratch_bytes(H, W // 64, 64) // 8, dtype=torch.int64,
                          device="cuda")
    em.edge_masks_staged(inp, out, H, W, scratch)
    torch.cuda.synchronize()
    want = oracle.edge(img)
    ok = bool(np.array_equal(unpack_rows(out.cpu().numpy().view(np.uint64), W), want))
    ms_staged = graph_time([lambda: em.edge_masks_staged(inp, out, H, W, scratch)] * 10, 3)
    ms_fused = graph_time([lambda: em.edge_image(inp, out, H, W, cfg="tuned")] * 10, 3)
    res["staged_vs_fused"] = {
        "workload": "8192x8192 glyph page, uint64: the three stages as 8 passes vs one fused pass",
        "ms_staged": round(ms_staged, 4), "ms_fused": round(ms_fused, 4),
        "fusion_speedup": round(ms_staged / ms_fused, 2),
        "staged_bytes_moved": 23 * packed_bytes, "fused_bytes_moved": 2 * packed_bytes,
        "staged_gbs_of_moved_bytes": round(23 * packed_bytes / (ms_staged * 1e-3) / 1e9, 1),
        "bit_exact": ok}
    del scratch
    # NEXT-3: direction planes
    out4 = torch.empty((4,) + tuple(inp.shape), dtype=inp.dtype, device="cuda")
    em.edge_directions(inp, out4, H, W)
    torch.cuda.synchronize()
    planes = out4.cpu().numpy().view(np.uint64)
    fe = oracle.fundamental_edges(img)
    ok = all(np.array_equal(unpack_rows(planes[k], W), fe[k]) for k in range(4))
    ms_dir = graph_time([lambda: em.edge_directions(inp, out4, H, W)] * 10, 3)
    res["directions"] = {
        "workload": "8192x8192 glyph page, uint64: four fundamental-edge planes (left, right, up, "
                    "down)", "ms": round(ms_dir, 4),
        "gbs": round(5 * packed_bytes / (ms_dir * 1e-3) / 1e9, 1), "bytes_moved": 5 * packed_bytes,
        "bit_exact": ok}
    del out4
    # NEXT-2: grey image -> threshold -> edges
    grey = images.grey_image(H, W, seed=7)
    gt = torch.from_numpy(grey).cuda()
    binary = torch.empty_like(inp)
    em.threshold_edges(gt, out, H, W, 128)
    torch.cuda.synchronize()
    want = oracle.edge(oracle.threshold(grey, 128))
    ok = bool(np.array_equal(unpack_rows(out.cpu().numpy().view(np.uint64), W), want))
    ms_fused_t = graph_time([lambda: em.threshold_edges(gt, out, H, W, 128)] * 10, 3)

    def two_pass():
        em.threshold_pack(gt, binary, H, W, 128)
        em.edge_image(binary, out, H, W, cfg="tuned")

    ms_two = graph_time([two_pass] * 10, 3)
    res["threshold_edges"] = {
        "workload": "8192x8192 grey image (smooth blobs + noise, seed 7), threshold 128, uint64",
        "ms_fused": round(ms_fused_t, 4), "ms_two_pass": round(ms_two, 4),
        "gbs_fused": round((px + packed_bytes) / (ms_fused_t * 1e-3) / 1e9, 1),
        "gpx_s_fused": round(px / (ms_fused_t * 1e-3) / 1e9, 1), "bit_exact": ok}
    del gt, binary, inp, out
    torch.cuda.empty_cache()
    return res


def peel_65536(torch, em, tm, steps=10):
    """Iterated peeling at 65536^2 (1 GiB each way), where one pass of k
    peels is bound by HBM rather than by the launch or the number of
    wavefronts: k = 1, 2, 4 and 8, sampled rows checked against the oracle
    run on full-width windows reaching k rows to either side (the k-th peel
    of a pixel depends on nothing farther away)."""
    from synth import images, pack_rows, unpack_rows
    import oracle
    H = W = 65536
    log("building 65536x65536 page (8x8 tiles of an 8192^2 glyph page, seed 22)")
    tile_img = images.glyph_page(8192, 8192, seed=22)
    words = np.tile(pack_rows(tile_img, 64), (8, 8))
    inp = words_tensor(torch, words)
    del words
    out = torch.empty_like(inp)
    rows = (0, 1, 8191, 8192, 30000, 65534, 65535)
    nbytes = 2 * H * (W // 64) * 8
    runs = []
    for k in (1, 2, 4, 8):
        em.peel(inp, out, H, W, k)
        torch.cuda.synchronize()
        ok = True
        for r in rows:
            lo, hi = max(0, r - k), min(H, r + k + 1)
            win = np.tile(np.stack([tile_img[y % 8192] for y in range(lo, hi)]), (1, 8))
            got = unpack_rows(out[r:r + 1].cpu().numpy().view(np.uint64), W)[0]
            ok &= bool(np.array_equal(got, oracle.peel(win, k)[r - lo]))
        warm_by_time(torch, lambda: em.peel(inp, out, H, W, k))
        ms = tm.per_call_ms(lambda i: em.peel(inp, out, H, W, k), steps)
        runs.append({"k": k, "ms": round(ms, 4),
                     "gpx_peels_s": round(H * W * k / (ms * 1e-3) / 1e9, 1),
                     "roofline": roofline(nbytes, ms), "sampled_rows_bit_exact": ok})
    del inp, out
    torch.cuda.empty_cache()
    return {"workload": "iterated peeling of the 65536x65536 tiled glyph page (seed 22), uint64, "
                        "white border; one edge_peel call of k peels, 1 GiB each way",
            "runs": runs}


def peel_section(torch, em, tm, ks=(1, 2, 4, 8, 16, 30)):
    """Iterated peeling of the 8192^2 glyph page (uint64): k peels in one
    fused pass against k launches of a single peel (ping-pong buffers);
    sampled rows checked against the oracle, the fused result against the
    repeated one on the whole image."""
    from synth import images, pack_rows, unpack_rows
    import oracle
    H = W = 8192
    img = images.glyph_page(H, W, seed=2)
    src = words_tensor(torch, pack_rows(img, 64))
    NB = 10
    ins = [src] + [src.clone() for _ in range(NB - 1)]
    outs = [torch.empty_like(src) for _ in range(NB)]
    tmp = [torch.empty_like(src) for _ in range(2)]
    nbytes = 2 * H * (W // 64) * 8
    rows = [0, 1, 4095, 8190, 8191]
    res = {"workload": "iterated peeling of the 8192x8192 glyph page (seed 2), uint64, white "
                       "border, 10 rotating buffer pairs; fused = one edge_peel call of k peels",
           "runs": []}
    for k in ks:
        fns = [(lambda i=i: em.peel(ins[i], outs[i], H, W, k)) for i in range(NB)]
        ms = rotation_time_ms(torch, tm, fns, 20, 5)

        def repeated(i=0):
            a = ins[i]
            for s_ in range(k):
                em.peel(a, tmp[s_ % 2], H, W, 1)
                a = tmp[s_ % 2]
            return a

        ms_rep = rotation_time_ms(torch, tm, [lambda: repeated()], 5, 3)
        em.peel(ins[0], outs[0], H, W, k)
        last = repeated()
        torch.cuda.synchronize()
        same = bool(torch.equal(outs[0], last))
        got = unpack_rows(outs[0][rows].cpu().numpy().view(np.uint64), W)
        want = np.stack([oracle.peel(img[max(0, y - k - 2):min(H, y + k + 3)], k)
                         [y - max(0, y - k - 2)] for y in rows])
        ok = bool(np.array_equal(got, want)) and same
        res["runs"].append({"k": k, "us_fused": round(ms * 1e3, 2), "us_repeated": round(ms_rep * 1e3, 2),
                            "speedup": round(ms_rep / ms, 2),
                            "gbs_fused": round(nbytes / (ms * 1e-3) / 1e9, 1),
                            "gpx_peels_s": round(H * W * k / (ms * 1e-3) / 1e9, 1),
                            "bit_exact": ok})
        log(f"peel k={k}: fused {ms * 1e3:.2f} us, repeated {ms_rep * 1e3:.2f} us, ok={ok}")
    del ins, outs, tmp, src
    torch.cuda.empty_cache()
    return res


def random_words(torch, side: int):
    """A side x side image of independent fair random bits (Bernoulli(0.5)),
    packed uint64, drawn on the device."""
    return torch.randint(0, 256, (side * side // 8,), dtype=torch.uint8,
                         device="cuda").view(torch.int64).view(side, side // 64)


def sample_check(inp, out, height, width, rows, word_bits=64) -> bool:
    """Compare sampled output rows of a device image with the oracle run on
    the input rows around them (copied back from the device)."""
    import oracle
    from synth import unpack_rows
    ok = True
    dt = np.uint64 if word_bits == 64 else np.uint32
    for r in rows:
        lo, hi = max(0, r - 1), min(height, r + 2)
        win = unpack_rows(inp[lo:hi].cpu().numpy().view(dt), width)
        want = oracle.edge_rows(win, lo, [r], height)[0]
        got = unpack_rows(out[r:r + 1].cpu().numpy().view(dt), width)[0]
        ok &= bool(np.array_equal(got, want))
    return ok


def rotation_time_ms(torch, tm, fns, min_launches: int, reps: int) -> float:
    """Per-launch time of launches replayed from one graph on one stream;
    the list is repeated until the graph holds at least min_launches."""
    seq = fns * max(1, -(-min_launches // len(fns)))
    g = graph_of(torch, None, nstreams=1, fns=seq)
    g.replay()
    torch.cuda.synchronize()
    ms = tm.per_call_ms(lambda i: g.replay(), reps) / len(seq)
    del g
    return ms


def size_sweep(torch, em, tm, sides=(1024, 2048, 4096, 8192, 16384, 32768, 65536)):
    """Plain method on square uint64 images of fair random bits, sides 2^10
    .. 2^16, rotating over buffer pairs until at least 640 MiB are touched
    per round (so every launch reads HBM): per-launch time, Gpx/s, GB/s and
    the plain copy of the same bytes. Section 6 claims time at most linear in
    the image size; the fixed launch cost dominates below about 8192^2."""
    res = []
    for side in sides:
        img_bytes = side * side // 8
        nb = int(min(40, max(1, -(-(640 << 20) // (2 * img_bytes)))))
        src = random_words(torch, side)
        ins = [src] + [src.clone() for _ in range(nb - 1)]
        outs = [torch.empty_like(src) for _ in range(nb)]
        em.edge_image(ins[0], outs[0], side, side, cfg="tuned")
        torch.cuda.synchronize()
        ok = sample_check(ins[0], outs[0], side, side, (0, 1, side // 2, side - 2, side - 1))
        fns = [(lambda i=i: em.edge_image(ins[i], outs[i], side, side, cfg="tuned"))
               for i in range(nb)]
        ms = rotation_time_ms(torch, tm, fns, 40 if side <= 16384 else 4,
                              5 if side <= 16384 else 3)
        del ins, outs, src
        torch.cuda.empty_cache()
        copy = copy_ceiling(torch, em, tm, img_bytes, nb, 40 if side <= 16384 else 4)
        gbs = 2 * img_bytes / (ms * 1e-3) / 1e9
        res.append({"side": side, "us_per_launch": round(ms * 1e3, 2),
                    "gpx_s": round(side * side / (ms * 1e-3) / 1e9, 1), "gbs": round(gbs, 1),
                    "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                    "copy_gbs_same_bytes": round(copy, 1),
                    "frac_of_copy": round(gbs / copy, 3), "buffer_pairs": nb,
                    "sampled_rows_bit_exact": ok})
        log(f"sweep {side}^2: {ms * 1e3:.2f} us, {gbs:.0f} GB/s, copy {copy:.0f} GB/s, ok={ok}")
    return {"workload": "plain, square uint64 images of fair random bits, sides 2^10..2^16, "
                        "white border, graph-replayed launches over rotating buffer pairs",
            "sizes": res}


def content_independence(torch, em, tm):
    """Plain-method launch time at 8192^2 (40 rotating pairs) and 65536^2
    for all-white, all-black, fair random and glyph-stroke images (section 7
    reports equal times for equally sized images of different content)."""
    from synth import images, pack_rows
    res = {}
    for side, nb in ((8192, 40), (65536, 1)):
        if side == 8192:
            strokes = words_tensor(torch, pack_rows(images.glyph_page(8192, 8192, seed=2), 64))
        else:
            tile = pack_rows(images.glyph_page(8192, 8192, seed=22), 64)
            strokes = torch.from_numpy(tile.view(np.int64)).cuda().repeat(8, 8)
        contents = {"white": lambda t: t.fill_(-1), "black": lambda t: t.zero_(),
                    "random": lambda t: t.copy_(random_words(torch, side)),
                    "strokes": lambda t: t.copy_(strokes)}
        per = {}
        for name, fill in contents.items():
            ins = [torch.empty_like(strokes) for _ in range(nb)]
            for t in ins:
                fill(t)
            outs = [torch.empty_like(strokes) for _ in range(nb)]
            em.edge_image(ins[0], outs[0], side, side, cfg="tuned")
            torch.cuda.synchronize()
            o = outs[0]
            if name == "white":
                ok = bool((o == 0).all())
            elif name == "black":   # white border: exactly the frame is edge
                ok = bool((o[0] == -1).all() and (o[-1] == -1).all()
                          and (o[1:-1, 0] == 1).all() and (o[1:-1, -1] == (-1 << 63)).all()
                          and (o[1:-1, 1:-1] == 0).all()) if side >= 128 else None
            else:
                ok = sample_check(ins[0], o, side, side, (0, side // 3, side - 1))
            fns = [(lambda i=i: em.edge_image(ins[i], outs[i], side, side, cfg="tuned"))
                   for i in range(nb)]
            ms = rotation_time_ms(torch, tm, fns, 40 if side <= 8192 else 10, 5)
            per[name] = {"us_per_launch": round(ms * 1e3, 2), "bit_exact": ok}
            log(f"content {side}^2 {name}: {ms * 1e3:.2f} us ok={ok}")
            del ins, outs
            torch.cuda.empty_cache()
        t = [v["us_per_launch"] for v in per.values()]
        res[f"{side}"] = dict(per, spread=round((max(t) - min(t)) / min(t), 4))
        del strokes
        torch.cuda.empty_cache()
    return dict(workload="plain, uint64, white border: all-white, all-black, fair random and "
                         "glyph-stroke images of one size; spread = (max - min) / min time",
                **res)


def host_cores() -> int:
    """Threads the CPU baseline may use: the cores this process may run on,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_banded(img, threads: int, clauses: int = 1):
    """The oracle on row bands of img, one band per thread (the oracle's C
    call releases the interpreter lock). Each band is computed with one halo
    row above and below from the image, so its rows see exactly their
    neighbours in the whole image; the oracle itself is unchanged."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    H = img.shape[0]
    cuts = np.linspace(0, H, threads + 1).astype(int)
    out = np.empty_like(img)

    def band(k):
        lo, hi = cuts[k], cuts[k + 1]
        if hi <= lo:
            return
        a, b = max(0, lo - 1), min(H, hi + 1)
        e = oracle.edge(img[a:b], clauses=clauses)
        out[lo:hi] = e[lo - a:lo - a + (hi - lo)]

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(band, range(threads)))
    return out


def cpu_oracle_configs(img8192, budget_s: float = 4.0):
    """The oracle at each workload size, on one thread and on all host cores
    (bands of rows in threads), packing excluded; bounded repetitions."""
    import oracle
    from synth import images
    threads = host_cores()

    def rate(fn, px, budget):
        t0, reps = time.perf_counter(), 0
        while True:
            fn()
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget or reps >= 50:
                return px * reps / el / 1e9

    if img8192 is None:
        img8192 = images.glyph_page(8192, 8192, seed=2)
    res = {"cores_all": threads, "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    img512, _ = images.strokes_image(512, 512, seed=1)
    crops = images.glyph_crops(4096, seed=3)
    page16k = images.skeleton_page(16384, 16384, seed=4)
    big = np.tile(images.glyph_page(8192, 8192, seed=22), (8, 8))
    cases = (("plain_512", img512, 1, budget_s / 4), ("plain_8192", img8192, 1, budget_s),
             ("full_16384", page16k, 3, budget_s), ("plain_65536", big, 1, 0.0))
    for name, im, cl, bud in cases:
        one = rate(lambda: oracle.edge(im, clauses=cl), im.size, bud)
        allc = rate(lambda: oracle_banded(im, threads, cl), im.size, bud)
        res[name] = {"gpx_s_1_thread": round(one, 4), "gpx_s_all_cores": round(allc, 4)}
        log(f"cpu oracle {name}: {one:.3f} Gpx/s on 1 thread, {allc:.3f} on {threads}")
    del big
    px = int(sum(c.size for c in crops))

    def crops_all():
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(oracle.edge, crops))

    res["batched_4096"] = {"gpx_s_1_thread": round(rate(lambda: [oracle.edge(c) for c in crops],
                                                        px, budget_s / 2), 4),
                           "gpx_s_all_cores": round(rate(crops_all, px, budget_s / 2), 4)}
    return res


def cpu_baseline(img, seconds):
    """The oracle (full definition: both clauses) on the headline image, one
    thread, repeated for about `seconds`; packing excluded."""
    import oracle
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.edge(img, clauses=oracle.CLAUSE1 | oracle.CLAUSE2)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds or reps >= 400:
            break
    gpx = img.size * reps / el / 1e9
    return {"value": round(gpx, 4), "unit": "Gpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} x the 16384x16384 headline image, full definition, byte image in "
                      f"and out (packing excluded), {el:.1f} s on one thread of {cpu_model()}"}


# Sections whose results are summarised in the final line (and written in
# full to the detail file), in the order they run.
def headline_section(torch, em, tm, args) -> dict:
    """The headline workload on its own (for profiling runs)."""
    res = headline_full(torch, em, args)
    res.pop("img")
    return res


SUMMARY_SECTIONS = {
    "plain_512": lambda torch, em, tm, a: plain_512(torch, em, tm, 2000),
    "plain_8192": lambda torch, em, tm, a: plain_8192(torch, em, tm),
    "plain_65536": lambda torch, em, tm, a: plain_65536(torch, em, tm, 20),
    "full_65536": lambda torch, em, tm, a: full_65536(torch, em, tm),
    "batched_4096": lambda torch, em, tm, a: batched_crops(torch, em, tm, 200),
    "serving": lambda torch, em, tm, a: serving(torch, em, copy=a.serve_copy),
}
# Sections written to the detail file only.
DETAIL_SECTIONS = {
    "next_rows": lambda torch, em, tm, a: next_rows(torch, em, tm, 200),
    "next_rows_65536": lambda torch, em, tm, a: next_rows_65536(torch, em, tm),
    "size_sweep": lambda torch, em, tm, a: size_sweep(torch, em, tm),
    "content": lambda torch, em, tm, a: content_independence(torch, em, tm),
    "peel": lambda torch, em, tm, a: peel_section(torch, em, tm),
    "peel_65536": lambda torch, em, tm, a: peel_65536(torch, em, tm),
    "cpu_configs": lambda torch, em, tm, a: cpu_oracle_configs(None),
}
SECTIONS = dict(SUMMARY_SECTIONS, **DETAIL_SECTIONS, **{
    "full_16384": headline_section,
    # the plain copy of 8, 64 or 512 MiB: the reference reading that scales
    # hardware counters of the edge kernels in the same profiled run
    "copy_8MiB": lambda torch, em, tm, a: round(copy_ceiling(torch, em, tm, 8 << 20, 40, 40), 1),
    "copy_64MiB": lambda torch, em, tm, a: round(copy_ceiling(torch, em, tm, 64 << 20, 10, 40), 1),
    "copy_512MiB": lambda torch, em, tm, a: round(copy_ceiling(torch, em, tm, 512 << 20, 2, 4),
                                                  1),
})


def device_clock_mhz(attr: int):
    """Peak clock of device 0 in MHz from hipDeviceGetAttribute (attribute 5:
    engine clock, 60: memory clock; both reported in kHz), None if unknown."""
    import ctypes
    try:
        lib = ctypes.CDLL("libamdhip64.so")
        v = ctypes.c_int(0)
        if lib.hipDeviceGetAttribute(ctypes.byref(v), ctypes.c_int(attr), ctypes.c_int(0)) != 0:
            return None
        return v.value // 1000 or None
    except OSError:
        return None


def versions(torch) -> dict:
    p = torch.cuda.get_device_properties(0)
    return {"torch": torch.__version__, "hip": torch.version.hip, "device": p.name,
            "arch": getattr(p, "gcnArchName", "?"), "compute_units": p.multi_processor_count,
            "hbm_gib": round(p.total_memory / 2**30, 1),
            "clock_mhz": device_clock_mhz(5), "memory_clock_mhz": device_clock_mhz(60)}


def _pick(d, *path):
    for k in path:
        if not isinstance(d, dict) or k not in d:
            return None
        d = d[k]
    return d


def summarise(detail: dict) -> dict:
    """A few numbers per summarised workload for the final line."""
    out = {}
    d = detail.get("plain_512")
    if d:
        out["cfg1_plain_512_u32"] = {"us": d["us_per_launch"], "gpx_s": d["gpx_s"],
                                     "exact": d["bit_exact"]}
    d = detail.get("plain_8192")
    if d:
        out["cfg2_plain_8192_u64"] = {"us": d["us_per_launch"], "gpx_s": d["gpx_s"],
                                      "frac": d["roofline"]["frac"], "exact": d["bit_exact"]}
    d = detail.get("plain_65536")
    if d:
        out["plain_65536_u64"] = {"gpx_s": d["gpx_s"], "frac": d["roofline"]["frac"],
                                  "exact": d["sampled_rows_bit_exact"]}
    d = detail.get("full_65536")
    if d:
        out["full_65536_u64"] = {"gpx_s": d["full"]["gpx_s"], "frac": d["full"]["roofline"]["frac"],
                                 "vs_plain_time": d["full_vs_plain_time"],
                                 "clause2_vs_plain_time": d.get("clause2_vs_plain_time"),
                                 "exact": d["full"]["sampled_rows_bit_exact"]}
    d = detail.get("batched_4096")
    if d:
        out["cfg3_batched_4096_u32"] = {"gpx_s": d["gpx_s_graph_of_20"],
                                        "x_vs_per_image": d["speedup_graph_of_20_vs_per_image_graph"],
                                        "exact": d["bit_exact_all_crops"]}
    d = detail.get("serving")
    if d:
        b = _pick(d, "batched", "max_sustained") or {}
        out["cfg5_served_u64"] = {"gpx_s": b.get("gpx_s"), "p50_ms": b.get("p50_ms"),
                                  "p99_ms": b.get("p99_ms"), "p99_bound_ms": d["p99_bound_ms"],
                                  "x_vs_per_request": d.get("speedup_at_p99_bound")}
    return out


def compact_line(head: dict, args, traffic, cpu, summary: dict, detail_path) -> dict:
    """The final JSON line: contract fields, the headline's roofline and CPU
    baseline, and the summary of the other workloads (a few hundred bytes
    each way; kept well under 2 KB)."""
    ms = head["ms_per_step"]
    nbytes = head["bytes_per_step"]
    gbs = nbytes / (ms * 1e-3) / 1e9
    exact = head["bit_exact_full"] and head["bit_exact_clause2"] and head["replays_equal"]
    trials = head["trials_ms"]
    line = {
        "metric": METRIC, "value": round(head["pixels_per_step"] / (ms * 1e-3) / 1e9, 1),
        "unit": "Gpixel/s", "n_gpus": 1, "steps": args.steps, "warmup": head["warmup_launches"],
        "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32 bitwise ops on u64-packed rows", "data": "synthetic",
        "config": {"workload": "full definition (clause 1 OR clause 2), one 16384x16384 skeleton "
                               "page (seed 4, ~10% black), uint64 rows, white border, 10 rotating "
                               "buffer pairs, the timed launches issued back to back on one "
                               "stream",
                   "launch_cfg": head["cfg"] or "built-in", "bytes_per_step": nbytes},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic},
        "cpu_baseline": cpu,
        "bit_exact": exact,
        "trials_ms": {"n": len(trials), "median": round(float(np.median(trials)), 5),
                      "p90": round(float(np.percentile(trials, 90)), 5)},
        "others": summary,
        "detail": os.path.relpath(detail_path, ROOT) if detail_path else None,
    }
    return line


def main(argv=None):
    global VERBOSE
    args = parse(argv)
    VERBOSE = args.verbose
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (a run "
                                   "on more GPUs is not supported)"}))
        sys.exit(2)
    if args.steps < 1:
        print(json.dumps({"error": "--steps must be at least 1"}))
        sys.exit(2)
    ensure_built()
    import torch
    import paper_1401_5245_amd as em
    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    tm = Timer(torch)
    only = args.only or (["serving"] if args.serve_only else ["batched_4096"] if args.batch_only
                         else ["next_rows"] if args.next_only else None)
    if only is not None:
        bad = [k for k in only if k not in SECTIONS]
        if bad:
            log(f"unknown section(s) {bad}; known: {list(SECTIONS)}")
            sys.exit(2)
        print(json.dumps({k: SECTIONS[k](torch, em, tm, args) for k in only}), flush=True)
        return
    head = headline_full(torch, em, args)
    img = head.pop("img")
    traffic = measured_traffic("k_strip_full_16384x16384_u64.md")
    log(f"headline: {head['ms_per_step'] * 1e3:.2f} us/step over {args.steps} steps")
    detail = {"headline": dict(head), "versions": versions(torch)}
    cpu = None
    if not args.headline_only:
        floor = launch_floor_ms(torch, em, tm)
        detail["launch_floor_us"] = round(floor * 1e3, 3)
        detail["copy_gbs_64MiB"] = round(copy_ceiling(torch, em, tm, 64 << 20, 10, 40), 1)
        for name, fn in SUMMARY_SECTIONS.items():
            log(f"section: {name}")
            detail[name] = fn(torch, em, tm, args)
        if not args.quick:
            for name, fn in DETAIL_SECTIONS.items():
                if name == "cpu_configs" and args.no_cpu:
                    continue
                log(f"section: {name}")
                detail[name] = fn(torch, em, tm, args)
        # after the GPU measurements: seconds of host-only work let the GPU idle down
        if not args.no_cpu:
            log("timing the CPU oracle")
            cpu = cpu_baseline(img, args.cpu_seconds)
            detail["cpu_baseline"] = cpu
    line = compact_line(head, args, traffic, cpu, summarise(detail),
                        args.detail if not args.headline_only else None)
    detail["line"] = line
    if args.detail:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
        with open(args.detail, "w") as f:
            json.dump(detail, f, indent=1, default=str)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
