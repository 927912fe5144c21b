"""Continuous-batching request loop over the encoder library.

Requests (each a handful of images at one resolution) arrive over time.  The
scheduler admits queued requests, oldest first, into a new device batch
whenever an execution slot is free and the batch's activation workspace fits
in the remaining HBM budget; admitted batches run concurrently on separate
HIP streams, so requests arriving while others are on the GPU start as soon
as a slot and memory free up.  Weights and text embeddings stay resident.

The scheduling state machine is independent of the device: it drives an
`Executor` (workspace_bytes / launch / poll / collect) against a `Clock`.
`GpuExecutor` runs vl_encode_images + vl_score on MI355X; tests drive the
same loop with a simulated executor and clock on the CPU.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional, Sequence, Tuple

__all__ = ["Request", "Result", "Clock", "RealClock", "SimClock", "Executor", "Scheduler",
           "ServeStats", "GpuExecutor", "percentile"]


@dataclass
class Request:
    rid: int
    arrival: float                       # seconds since the start of the run
    sizes: List[Tuple[int, int]]         # (H, W) of each image
    payload: Any = None                  # executor-specific input handle


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    n_images: int
    output: Any = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Clock:
    def now(self) -> float:
        raise NotImplementedError

    def wait(self, until: float) -> None:
        raise NotImplementedError


class RealClock(Clock):
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait(self, until: float) -> None:
        dt = until - self.now()
        if dt > 0:
            time.sleep(min(dt, 0.0005))


class SimClock(Clock):
    """Deterministic clock for tests: wait() jumps straight to the target."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def wait(self, until: float) -> None:
        self.t = max(self.t, until)


class Executor:
    """Device side of the loop.  launch() must not block on the device."""

    def workspace_bytes(self, sizes: Sequence[Tuple[int, int]]) -> int:
        raise NotImplementedError

    def launch(self, reqs: Sequence[Request], slot: int) -> Any:
        raise NotImplementedError

    def poll(self, handle: Any) -> bool:
        raise NotImplementedError

    def collect(self, handle: Any) -> List[Any]:
        """Per-request outputs of a finished launch, in launch order."""
        raise NotImplementedError

    def next_event_time(self) -> Optional[float]:
        """Earliest time a running launch may finish (simulated executors);
        None when unknown."""
        return None


@dataclass
class ServeStats:
    results: List[Result] = field(default_factory=list)
    batches: int = 0
    max_inflight: int = 0               # batches on the device at once
    max_inflight_images: int = 0        # images in those batches
    peak_budget: int = 0
    rejected: List[int] = field(default_factory=list)   # requests larger than the budget
    wall: float = 0.0

    def images_per_s(self) -> float:
        n = sum(r.n_images for r in self.results)
        return n / self.wall if self.wall > 0 else 0.0

    def latency_ms(self, q: float) -> float:
        return 1e3 * percentile([r.latency for r in self.results], q)


def percentile(xs: Sequence[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    if not xs:
        return float("nan")
    s = sorted(xs)
    k = max(1, int(math.ceil(q / 100.0 * len(s))))
    return s[k - 1]


class Scheduler:
    """Admission: FIFO; a batch takes queued requests while (a) the image
    count stays <= max_batch_images and (b) the batch workspace plus the
    workspaces of running batches stays <= budget_bytes.  A request whose
    workspace alone exceeds the budget is rejected.  At most `slots` batches
    run at once."""

    def __init__(self, executor: Executor, budget_bytes: int, slots: int = 2,
                 max_batch_images: int = 32):
        if slots < 1 or budget_bytes <= 0 or max_batch_images < 1:
            raise ValueError("slots, budget and batch limit must be positive")
        self.ex = executor
        self.budget = budget_bytes
        self.slots = slots
        self.max_batch_images = max_batch_images

    def run(self, requests: Sequence[Request], clock: Clock) -> ServeStats:
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        st = ServeStats()
        queue: List[Request] = []
        running: Dict[int, Tuple[Any, List[Request], int, float]] = {}
        free_slots = list(range(self.slots))
        used = 0
        i = 0
        t_start = clock.now()
        while i < len(pending) or queue or running:
            now = clock.now() - t_start
            while i < len(pending) and pending[i].arrival <= now:
                queue.append(pending[i])
                i += 1
            # Retire finished batches: free their slot and budget.
            for slot in list(running):
                h, reqs, ws, t_adm = running[slot]
                if self.ex.poll(h):
                    t_fin = clock.now() - t_start
                    outs = self.ex.collect(h)
                    for r, o in zip(reqs, outs):
                        st.results.append(Result(r.rid, r.arrival, t_adm, t_fin,
                                                 len(r.sizes), o))
                    used -= ws
                    del running[slot]
                    free_slots.append(slot)
            # Admit a new batch into each free slot while the budget allows.
            while free_slots and queue:
                batch: List[Request] = []
                sizes: List[Tuple[int, int]] = []
                ws = 0
                for r in list(queue):
                    if self.ex.workspace_bytes(r.sizes) > self.budget:
                        queue.remove(r)
                        st.rejected.append(r.rid)
                        continue
                    if len(sizes) + len(r.sizes) > self.max_batch_images and batch:
                        break
                    w = self.ex.workspace_bytes(sizes + r.sizes)
                    if used + w > self.budget:
                        break
                    batch.append(r)
                    sizes += r.sizes
                    ws = w
                    queue.remove(r)
                if not batch:
                    break
                slot = free_slots.pop(0)
                h = self.ex.launch(batch, slot)
                running[slot] = (h, batch, ws, clock.now() - t_start)
                used += ws
                st.batches += 1
                st.max_inflight = max(st.max_inflight, len(running))
                st.max_inflight_images = max(
                    st.max_inflight_images,
                    sum(len(r.sizes) for _, rs, _, _ in running.values() for r in rs))
                st.peak_budget = max(st.peak_budget, used)
            # Idle: wait for the next arrival or completion.
            nxt = [t_start + pending[i].arrival] if i < len(pending) else []
            ev = self.ex.next_event_time()
            if ev is not None:
                nxt.append(ev)
            if nxt:
                clock.wait(min(nxt))
            elif running:
                clock.wait(clock.now() + 1e-5)
        st.wall = clock.now() - t_start
        st.results.sort(key=lambda r: r.rid)
        return st


class GpuExecutor(Executor):
    """Runs each batch as vl_encode_images + vl_score on its slot's stream.
    A request payload is a flat FP32 device tensor of the request's images,
    or a list of such tensors (one per image); the batch's images are
    gathered into one packed buffer on the slot's stream.  Texts stay
    resident.  Outputs per request: (embeddings, top-1)."""

    def __init__(self, encoder, texts, head: str, scale: float, bias: float, slots: int,
                 keep_workspaces: bool = False):
        """keep_workspaces: each slot keeps its encoder workspace across
        batches (grown to the largest batch it has run), so an encoder with
        graph replay on replays one graph per (slot, capacity bucket); the
        device memory held is then up to `slots` of the largest workspace
        admitted, beyond what the admission budget counts per batch."""
        import torch
        from . import vl
        self.torch, self.vl = torch, vl
        self.enc = encoder
        self.texts = texts
        self.head, self.scale, self.bias = head, scale, bias
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.keep = keep_workspaces
        self.ws = [None] * slots

    def workspace_bytes(self, sizes):
        """Device bytes a batch holds while it runs: the encoder workspace
        plus the buffers launch() allocates (the packed pixels, counted even
        when a single request's tensor is used as is, the embeddings, the
        scores and the top-1 indices)."""
        n = len(sizes)
        chans = getattr(self.enc.cfg, "channels", 3)
        io = 4 * chans * sum(h * w for h, w in sizes)
        io += 4 * n * (self.enc.cfg.proj_dim + self.texts.shape[0] + 1)
        return self.enc.workspace_bytes(sizes) + io

    def launch(self, reqs, slot):
        torch, vl = self.torch, self.vl
        s = self.streams[slot]
        sizes = [hw for r in reqs for hw in r.sizes]
        n = len(sizes)
        with torch.cuda.stream(s):
            parts = []
            for r in reqs:
                parts.extend(r.payload if isinstance(r.payload, (list, tuple)) else [r.payload])
            pix = torch.cat(parts) if len(parts) > 1 else parts[0]
            need = self.enc.workspace_bytes(sizes)
            if self.keep:
                if self.ws[slot] is None or self.ws[slot].numel() < need:
                    self.ws[slot] = torch.empty(need, dtype=torch.uint8, device="cuda")
                ws = self.ws[slot]
            else:
                ws = torch.empty(need, dtype=torch.uint8, device="cuda")
            emb = torch.empty((n, self.enc.cfg.proj_dim), dtype=torch.float32, device="cuda")
            sc = torch.empty((n, self.texts.shape[0]), dtype=torch.float32, device="cuda")
            top = torch.empty(n, dtype=torch.int32, device="cuda")
            vl.vl_encode_images(self.enc.handle, pix, [h for h, _ in sizes],
                                [w for _, w in sizes], emb, ws, s,
                                channels=getattr(self.enc.cfg, "channels", 3),
                                proj_dim=self.enc.cfg.proj_dim)
            vl.vl_score(emb, self.texts, self.head, self.scale, self.bias, sc, top, s)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, reqs, emb, top, (pix, ws, sc))

    def poll(self, handle):
        return handle[0].query()

    def collect(self, handle):
        ev, reqs, emb, top, _ = handle
        out, o = [], 0
        for r in reqs:
            k = len(r.sizes)
            out.append((emb[o:o + k], top[o:o + k]))
            o += k
        return out
