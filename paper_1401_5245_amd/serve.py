"""Continuous-batching server for binary edge maps on one GPU.

Requests (packed images already in pinned host memory) arrive on a
schedule. The server admits them in arrival order while the device ring
arena (the HBM budget) has room, copies each admitted group to the device
with as few copies as the layout allows, and whenever a launch slot is free
sends every admitted request not yet launched into one persistent batched
launch (``edge_batch``). Up to ``max_inflight`` batches are on the device at
once, each moving through three streams: copy-in, compute, copy-out.
Results come back into a pinned host ring laid out like the device arena,
so each request has its own output slice for as long as its arena block is
live; a batch's block is released once its results are in host memory
(and, with ``record_outputs``, copied out of the ring), and the next
arrivals are admitted into it. Latency is measured from a request's
scheduled arrival to the moment its result is in host memory.

Copies between pinned host memory and the arena go either through the
runtime's copy engines (``copy="sdma"``: hipMemcpyAsync) or through the
library's 128-bit copy kernel reading and writing the pinned host memory
directly (``copy="kernel"``: edge_copy_bytes), an ordinary kernel launch on
the copy streams.

``per_request=True`` runs the same loop with one plain ``edge_image``
launch (and its own copy-out) per request: the per-request-launch server
that batching is compared against.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import batch as _batch
from ._abi import EdgeError, EDGE_ERR_INVALID, check, load

_HIP = None
_HIP_MEMCPY_DEFAULT = 4     # direction inferred from the pointers (unified addressing)
_HIP_EVENT_DISABLE_TIMING = 2
_HIP_ERROR_NOT_READY = 600


def _hip():
    """The HIP runtime already loaded by torch. Copies, events and waits go
    to it directly: torch's non-blocking copies into pinned memory also
    record a tracking event per copy, which can stall the host. ctypes
    releases the GIL for the duration of each call."""
    global _HIP
    if _HIP is None:
        lib = ctypes.CDLL("libamdhip64.so")
        vp = ctypes.c_void_p
        for name, args in (("hipMemcpyAsync", [vp, vp, ctypes.c_size_t, ctypes.c_int, vp]),
                           ("hipEventCreateWithFlags", [ctypes.POINTER(vp), ctypes.c_uint]),
                           ("hipEventRecord", [vp, vp]),
                           ("hipStreamWaitEvent", [vp, vp, ctypes.c_uint]),
                           ("hipEventQuery", [vp]),
                           ("hipEventDestroy", [vp]),
                           ("hipHostGetDevicePointer", [ctypes.POINTER(vp), vp, ctypes.c_uint])):
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _HIP = lib
    return _HIP


def _hip_ok(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"{what} failed (hipError {rc})")


def _copy_async(dst: torch.Tensor, dst_off: int, src: torch.Tensor, src_off: int, n: int,
                stream) -> None:
    """Copy n elements src[src_off:] -> dst[dst_off:] on `stream` (a torch
    stream or a raw hipStream_t handle)."""
    if not (0 <= src_off and src_off + n <= src.numel() and 0 <= dst_off
            and dst_off + n <= dst.numel()):
        raise ValueError("copy outside its tensors")
    if dst.element_size() != src.element_size():
        raise ValueError("source and destination differ in element size")
    es = src.element_size()
    handle = stream if isinstance(stream, int) else stream.cuda_stream
    _hip_ok(_hip().hipMemcpyAsync(dst.data_ptr() + dst_off * es, src.data_ptr() + src_off * es,
                                  n * es, _HIP_MEMCPY_DEFAULT, handle), "hipMemcpyAsync")


def _device_mapped(t: torch.Tensor) -> bool:
    """True when pinned host tensor t is mapped into the device's address
    space at its own address (what a kernel reading it directly needs)."""
    d = ctypes.c_void_p()
    if _hip().hipHostGetDevicePointer(ctypes.byref(d), t.data_ptr(), 0) != 0:
        return False
    return d.value == t.data_ptr()


def _copy_kernel(dst: torch.Tensor, dst_off: int, src: torch.Tensor, src_off: int, n: int,
                 stream: int) -> None:
    """The same copy with the library's copy kernel (edge_copy_bytes): 16-byte
    aligned ends and a multiple of 16 bytes, host side pinned."""
    if not (0 <= src_off and src_off + n <= src.numel() and 0 <= dst_off
            and dst_off + n <= dst.numel()):
        raise ValueError("copy outside its tensors")
    es = src.element_size()
    check(load().edge_copy_bytes(src.data_ptr() + src_off * es, dst.data_ptr() + dst_off * es,
                                 n * es, stream))


class _Event:
    """A raw HIP event (no timing), re-recorded on every use."""

    def __init__(self):
        h = ctypes.c_void_p()
        _hip_ok(_hip().hipEventCreateWithFlags(ctypes.byref(h), _HIP_EVENT_DISABLE_TIMING),
                "hipEventCreateWithFlags")
        self.h = h

    def record(self, stream: int) -> None:
        _hip_ok(_hip().hipEventRecord(self.h, stream), "hipEventRecord")

    def wait_on(self, stream: int) -> None:
        """Make `stream` wait for the last record of this event."""
        _hip_ok(_hip().hipStreamWaitEvent(stream, self.h, 0), "hipStreamWaitEvent")

    def done(self) -> bool:
        rc = _hip().hipEventQuery(self.h)
        if rc == _HIP_ERROR_NOT_READY:
            return False
        _hip_ok(rc, "hipEventQuery")
        return True

    def __del__(self):
        try:
            if self.h:
                _hip().hipEventDestroy(self.h)
        except Exception:
            pass


class RingArena:
    """FIFO ring allocator over [0, capacity) words.

    Blocks are taken at the head and released oldest first; a block never
    straddles the end of the ring (the tail gap is skipped). Offsets are
    rounded up to `align` words.
    """

    def __init__(self, capacity: int, align: int = 2):
        self.capacity = int(capacity)
        self.align = int(align)
        self.blocks = collections.deque()   # (offset, size)
        self.head = 0
        self.used = 0

    def _round(self, n):
        return -(-int(n) // self.align) * self.align

    def alloc(self, n: int):
        """Offset of a new block of n words, or None when it does not fit now."""
        n = self._round(n)
        if n <= 0 or n > self.capacity:
            raise ValueError(f"block of {n} words cannot fit a ring of {self.capacity}")
        if not self.blocks:
            off = 0
        else:
            first = self.blocks[0][0]
            if self.head > first:                 # live region [first, head)
                if self.head + n <= self.capacity:
                    off = self.head
                elif n <= first:
                    off = 0
                else:
                    return None
            else:                                 # wrapped: free [head, first)
                if self.head + n <= first:
                    off = self.head
                else:
                    return None
        self.blocks.append((off, n))
        self.head = off + n
        self.used += n
        return off

    def free_oldest(self):
        off, n = self.blocks.popleft()
        self.used -= n
        if not self.blocks:
            self.head = 0
        return off, n


@dataclass
class Request:
    rid: int
    pool_index: int
    arrival: float                   # scheduled arrival, seconds from start
    admitted: float = -1.0
    launched: float = -1.0
    kernel_done: float = -1.0
    done: float = -1.0
    offset: int = -1                 # device arena offset (words)
    rejected: bool = False


@dataclass
class Pool:
    """Packed request images in one pinned host buffer.

    host_in: pinned words of every pool image back to back (16-byte aligned
    offsets).
    """
    host_in: torch.Tensor
    table: np.ndarray                # DESC_DTYPE, offsets into host_in
    word_bits: int
    pixels: np.ndarray               # H*W per image

    @classmethod
    def from_images(cls, packed, word_bits: int):
        arena, table = _batch.pack_arena(packed, word_bits)
        view = np.int64 if word_bits == 64 else np.int32
        host_in = torch.from_numpy(arena.view(view)).pin_memory()
        pixels = table["height"].astype(np.int64) * table["width"].astype(np.int64)
        return cls(host_in, table, word_bits, pixels)

    def words(self, i: int) -> int:
        d = self.table[i]
        return int(d["height"]) * int(d["stride_words"])


@dataclass
class _Batch:
    reqs: list
    slot: int
    ev_kernel: _Event
    ev_done: _Event


@dataclass
class Stats:
    latencies_ms: np.ndarray
    latencies_no_d2h_ms: np.ndarray
    queue_ms: np.ndarray
    pixels: int
    duration_s: float
    n_batches: int
    rejected: int
    extra: dict = field(default_factory=dict)

    def summary(self) -> dict:
        lat = self.latencies_ms
        q = (lambda a, p: float(np.percentile(a, p)) if a.size else float("nan"))
        return {"requests": int(lat.size), "rejected": self.rejected, "batches": self.n_batches,
                "p50_ms": round(q(lat, 50), 3), "p99_ms": round(q(lat, 99), 3),
                "max_ms": round(float(lat.max()) if lat.size else float("nan"), 3),
                "p50_ms_no_d2h": round(q(self.latencies_no_d2h_ms, 50), 3),
                "p99_ms_no_d2h": round(q(self.latencies_no_d2h_ms, 99), 3),
                "p50_queue_ms": round(q(self.queue_ms, 50), 3),
                "gpx_s": round(self.pixels / self.duration_s / 1e9, 3) if self.duration_s else 0.0,
                "duration_s": round(self.duration_s, 4), **self.extra}


def _runs(src_offs, dst_offs, sizes):
    """Merge (src, dst, n) copies into runs contiguous on both sides."""
    runs = []
    for s, d, n in zip(src_offs, dst_offs, sizes):
        if runs and runs[-1][0] + runs[-1][2] == s and runs[-1][1] + runs[-1][2] == d:
            runs[-1][2] += n
        else:
            runs.append([s, d, n])
    return runs




class Server:
    """One-GPU continuous-batching server over a pinned request pool."""

    def __init__(self, pool: Pool, budget_bytes: int, *, max_inflight: int = 3,
                 max_batch: int = 4096, max_batch_bytes: int = 64 << 20,
                 border: str = "white", mode: str = "masks",
                 cfg=None, copy: str = "kernel", device="cuda"):
        if copy not in ("sdma", "kernel"):
            raise ValueError("copy must be 'sdma' or 'kernel'")
        self.pool = pool
        wb = pool.word_bits
        self.word_bytes = wb // 8
        cap = int(budget_bytes) // 2 // self.word_bytes      # each of in and out arenas
        align = 128 // wb
        cap -= cap % align
        self.ring = RingArena(cap, align)
        dt = torch.int64 if wb == 64 else torch.int32
        self.dev_in = torch.zeros(cap, dtype=dt, device=device)
        self.dev_out = torch.zeros(cap, dtype=dt, device=device)
        # results land in a pinned host ring with the device arena's layout:
        # a request's output slice is its own until its block is released
        self.host_out = torch.zeros(cap, dtype=dt).pin_memory()
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        # bytes of input per batch: a burst of arrivals then becomes several
        # pipelined batches instead of one whose copies hold up the rest
        self.max_batch_words = max(1, int(max_batch_bytes) // self.word_bytes)
        self.kw = dict(border=border, mode=mode, cfg=cfg)
        self.copy_engine = copy
        self._copy = _copy_kernel if copy == "kernel" else _copy_async
        self.s_in = torch.cuda.Stream(device)
        self.s_k = torch.cuda.Stream(device)
        self.s_out = torch.cuda.Stream(device)
        self.h_in, self.h_k, self.h_out = (self.s_in.cuda_stream, self.s_k.cuda_stream,
                                           self.s_out.cuda_stream)
        nb = _batch.batch_workspace_bytes(max_batch)
        # table and plan are copied in whole 16-byte units (the kernel copy's
        # granule): one spare word past the largest size each
        self.slots = []
        for _ in range(max_inflight):
            self.slots.append({
                "table_host": torch.zeros(max_batch * 3 + 1, dtype=torch.int64).pin_memory(),
                "table_dev": torch.zeros(max_batch * 3 + 1, dtype=torch.int64, device=device),
                "plan_host": torch.zeros(-(-nb // 8) + 1, dtype=torch.int64).pin_memory(),
                "ws": torch.zeros(-(-nb // 8) + 1, dtype=torch.int64, device=device),
                # created once and re-recorded each time the slot is used: the
                # slot is reused only after its last batch is back on the host
                "ev_in": _Event(), "ev_k": _Event(), "ev_d": _Event(),
                "busy": False})
        self._tab = np.zeros(max_batch, dtype=_batch.DESC_DTYPE)
        if copy == "kernel":
            host = [self.pool.host_in, self.host_out] + [
                S[k] for S in self.slots for k in ("table_host", "plan_host")]
            if not all(t.is_pinned() and _device_mapped(t) for t in host):
                raise RuntimeError("copy='kernel' needs pinned host buffers mapped at their "
                                   "own address on the device")
        self.warmup()

    def warmup(self):
        """Run the copy paths once at full size (pool to arena, arena to the
        host ring, on the serving streams) so that first-use set-up in the
        runtime is not paid by a request."""
        n = min(self.pool.host_in.numel(), self.dev_in.numel())
        n -= n % (16 // self.word_bytes)
        self._copy(self.dev_in, 0, self.pool.host_in, 0, n, self.h_in)
        self.s_out.wait_stream(self.s_in)
        self._copy(self.host_out, 0, self.dev_in, 0, n, self.h_out)
        for S in self.slots:
            for k in ("ev_in", "ev_k", "ev_d"):
                S[k].record(self.h_out)
        torch.cuda.synchronize()

    # ---------------------------------------------------------------- loop --

    def run(self, arrivals: np.ndarray, pool_index: np.ndarray, *, per_request: bool = False,
            record_outputs: bool = False) -> Stats:
        """Serve requests r = 0..n-1 arriving at `arrivals[r]` seconds with
        image pool_index[r]. Blocks until every request is answered."""
        import gc
        import paper_1401_5245_amd as em
        gc_was_enabled = gc.isenabled()
        gc.disable()            # no collector pauses inside the serving loop
        try:
            return self._run(em, arrivals, pool_index, per_request, record_outputs)
        finally:
            if gc_was_enabled:
                gc.enable()

    def _run(self, em, arrivals, pool_index, per_request, record_outputs) -> Stats:
        pool = self.pool
        n = len(arrivals)
        reqs = [Request(i, int(pool_index[i]), float(arrivals[i])) for i in range(n)]
        words = np.array([pool.words(int(p)) for p in pool_index], dtype=np.int64)
        waiting = collections.deque(range(n))
        admitted = collections.deque()
        inflight = collections.deque()
        out_of = [None] * n if record_outputs else None
        nbatches = 0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        dev_in, dev_out, host_in, host_out = self.dev_in, self.dev_out, pool.host_in, self.host_out
        copy = self._copy
        table = pool.table
        rejected = 0
        # host-side stalls: the longest pass through the loop, and the most a
        # sleep overran what it asked for
        max_pass, max_oversleep, stalls_over_1ms = 0.0, 0.0, 0
        sect = collections.defaultdict(float)       # longest time in each part of a pass

        def mark(name, t_from):
            t_to = now()
            if t_to - t_from > sect[name]:
                sect[name] = t_to - t_from
            return t_to

        while waiting or admitted or inflight:
            progressed = False
            it = now()
            # 1. completions, oldest first (the ring frees in order)
            while inflight and inflight[0].ev_done.done():
                b = inflight.popleft()
                t = now()
                for r in b.reqs:
                    r.done = t
                    if record_outputs:
                        out_of[r.rid] = host_out[r.offset:r.offset + words[r.rid]].clone()
                    self.ring.free_oldest()
                self.slots[b.slot]["busy"] = False
                progressed = True
            for b in inflight:
                if b.reqs[0].kernel_done < 0 and b.ev_kernel.done():
                    t = now()
                    for r in b.reqs:
                        r.kernel_done = t
            # 2. admission in arrival order while the ring has room
            t = mark("completions", it)
            newly = []
            while waiting and reqs[waiting[0]].arrival <= t:
                r = reqs[waiting[0]]
                if self.ring._round(words[r.rid]) > self.ring.capacity:
                    r.rejected = True          # larger than the whole budget
                    rejected += 1
                    waiting.popleft()
                    continue
                if words[r.rid] == 0:          # empty image: nothing to compute
                    r.admitted = r.launched = r.kernel_done = r.done = t
                    waiting.popleft()
                    continue
                off = self.ring.alloc(words[r.rid])
                if off is None:
                    break                      # wait for space to free up
                r.offset = off
                r.admitted = t
                waiting.popleft()
                newly.append(r)
            if newly:
                # whole 16-byte units (the ring's and the pool's alignment):
                # neighbouring blocks then merge into one copy
                runs = _runs([int(table[r.pool_index]["offset_words"]) for r in newly],
                             [r.offset for r in newly],
                             [self.ring._round(words[r.rid]) for r in newly])
                for s, d, m in runs:
                    copy(dev_in, d, host_in, s, m, self.h_in)
                admitted.extend(newly)
                progressed = True
            # 3. launch: every admitted request not yet launched (continuous batching)
            t_s = mark("admission", t)
            if admitted:
                slot = next((i for i, s in enumerate(self.slots) if not s["busy"]), None)
                if slot is not None:
                    if per_request:
                        group = [admitted.popleft()]
                    else:
                        group, gw = [], 0
                        while admitted and len(group) < self.max_batch and (
                                not group or gw + words[admitted[0].rid] <= self.max_batch_words):
                            r = admitted.popleft()
                            gw += words[r.rid]
                            group.append(r)
                    S = self.slots[slot]
                    # the copy-in stream is in order: one event recorded now
                    # covers the copies of every request admitted so far
                    S["ev_in"].record(self.h_in)
                    S["ev_in"].wait_on(self.h_k)
                    t = now()
                    t_s = mark("launch_wait", t_s)
                    if per_request:
                        r = group[0]
                        d = table[r.pool_index]
                        m = int(words[r.rid])
                        em.edge_image(dev_in[r.offset:r.offset + m], dev_out[r.offset:r.offset + m],
                                      int(d["height"]), int(d["width"]),
                                      stride_words=int(d["stride_words"]),
                                      border=self.kw["border"], mode=self.kw["mode"],
                                      stream=self.s_k)
                        t_s = mark("launch", t_s)
                    else:
                        k = len(group)
                        tab = self._tab[:k]
                        pidx = np.fromiter((r.pool_index for r in group), np.int64, k)
                        tab["offset_words"] = np.fromiter((r.offset for r in group), np.int64, k)
                        tab["height"] = table["height"][pidx]
                        tab["width"] = table["width"][pidx]
                        tab["stride_words"] = table["stride_words"][pidx]
                        S["table_host"][:k * 3].numpy()[:] = tab.view(np.int64)
                        _, used = _batch.plan_batch(dev_in, dev_out, tab, mode=self.kw["mode"],
                                                    cfg=self.kw["cfg"],
                                                    out=S["plan_host"].numpy())
                        t_s = mark("plan", t_s)
                        nt, nw = k * 3, -(-used // 8)
                        copy(S["table_dev"], 0, S["table_host"], 0, nt + nt % 2, self.h_k)
                        copy(S["ws"], 0, S["plan_host"], 0, nw + nw % 2, self.h_k)
                        t_s = mark("plan_copy", t_s)
                        _batch.edge_batch(dev_in, dev_out, S["table_dev"], k, S["ws"],
                                          planned=True, stream=self.s_k, **self.kw)
                        t_s = mark("launch", t_s)
                    S["ev_k"].record(self.h_k)
                    S["ev_k"].wait_on(self.h_out)
                    # results to the same offsets of the host ring
                    for s, d, m in _runs([r.offset for r in group], [r.offset for r in group],
                                         [self.ring._round(words[r.rid]) for r in group]):
                        copy(host_out, d, dev_out, s, m, self.h_out)
                    S["ev_d"].record(self.h_out)
                    mark("copy_out", t_s)
                    for r in group:
                        r.launched = t
                    S["busy"] = True
                    inflight.append(_Batch(group, slot, S["ev_k"], S["ev_d"]))
                    nbatches += 1
                    progressed = True
            t_end = now()
            if t_end - it > max_pass:
                max_pass = t_end - it
            stalls_over_1ms += t_end - it > 1e-3
            if not progressed:
                want = 0.0
                if not admitted and not inflight and waiting:
                    gap = reqs[waiting[0]].arrival - t_end
                    if gap > 2e-4:
                        want = gap - 1e-4
                time.sleep(want)
                over = now() - t_end - want
                if over > max_oversleep:
                    max_oversleep = over
                stalls_over_1ms += over > 1e-3
        served = [r for r in reqs if not r.rejected and words[r.rid] > 0]
        lat = np.array([(r.done - r.arrival) * 1e3 for r in served])
        lat_k = np.array([((r.kernel_done if r.kernel_done >= 0 else r.done) - r.arrival) * 1e3
                          for r in served])
        queue_ms = np.array([(r.launched - r.arrival) * 1e3 for r in served])
        # stages: waiting for a launch slot (and its copy-in), copy-in +
        # kernel as seen by the host, copy-out
        k_seen = np.array([((r.kernel_done if r.kernel_done >= 0 else r.done) - r.launched) * 1e3
                           for r in served])
        d2h = np.array([(r.done - (r.kernel_done if r.kernel_done >= 0 else r.done)) * 1e3
                        for r in served])
        pixels = int(sum(int(pool.pixels[r.pool_index]) for r in served))
        copied = int(sum(int(words[r.rid]) for r in served)) * self.word_bytes   # each way
        t_first = min((r.arrival for r in served), default=0.0)
        t_last = max((r.done for r in served), default=0.0)
        pct = (lambda a, p: round(float(np.percentile(a, p)), 3) if a.size else None)
        stages = {"launch_to_kernel_done_ms": [pct(k_seen, 50), pct(k_seen, 99)],
                  "copy_out_ms": [pct(d2h, 50), pct(d2h, 99)],
                  "queue_ms": [pct(queue_ms, 50), pct(queue_ms, 99)]}
        dur = t_last - t_first
        st = Stats(lat, lat_k, queue_ms, pixels, dur, nbatches, rejected,
                   {"copy": self.copy_engine, "stages_p50_p99": stages,
                    "host_link_gbs_each_way": round(copied / dur / 1e9, 2) if dur > 0 else 0.0,
                    "max_loop_pass_ms": round(max_pass * 1e3, 3),
                    "max_oversleep_ms": round(max_oversleep * 1e3, 3),
                    "host_stalls_over_1ms": int(stalls_over_1ms),
                    "max_section_ms": {k: round(v * 1e3, 3) for k, v in sect.items()}})
        if record_outputs:
            st.extra["outputs"] = out_of
        return st


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of `rate` requests/s."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


__all__ = ["RingArena", "Pool", "Server", "Stats", "poisson_arrivals", "EdgeError",
           "EDGE_ERR_INVALID"]
