"""Continuous-batching server for watershed + waterfall partition jobs.

Jobs (a quantised gradient already on the device, a connectivity and NL) arrive
at any time. A dispatcher admits them into micro-batches (2D and 3D jobs of any
connectivity together; one NL and grey type per micro-batch) while an execution
slot is free and the device-memory budget holds their footprint
(ws_footprint_bytes: outputs plus the library's scratch). Each slot owns a
library context (its own scratch) and a HIP stream and is driven by its own
host thread, so micro-batches of different slots run concurrently on the GPU.
Jobs that arrive while others are on the GPU wait for the next free slot and
join the next micro-batch. A job whose footprint alone exceeds the budget is
rejected without affecting any other job.

Every slot reserves the scratch of a max_batch_pixels batch up front, so
serving allocates no library scratch (device allocation and freeing wait for
the whole device). A micro-batch can exceed that only through one job larger
than the cap; such jobs run alone on slot 0, which also reserves
max_job_pixels when that is given, so the other slots never reallocate. While
an oversized job waits for slot 0, the other slots take the ordinary jobs
queued behind it.

All arithmetic is in the library (ws_batch); this module only schedules. The
result of a job is bit-identical to running it alone: the batched kernels
never mix images (see include/ws.h, ws_batch).
"""
from __future__ import annotations

import collections
import threading
import time
import traceback
from dataclasses import dataclass, field
from typing import Callable, List, Optional

from .binding import Context, WSError, load_library, _dims


@dataclass
class Job:
    grad: object                 # device tensor, uint8/uint16, (ny, nx) or (nz, ny, nx)
    conn: int
    NL: int = 4
    jid: int = 0
    t_arrival: float = 0.0       # time.perf_counter() when submitted
    t_start: float = 0.0         # admitted into a micro-batch
    t_done: float = 0.0          # labels ready on the device
    out: object = None           # int32 [NL, ...] device tensor
    nregions: object = None      # int64 [NL] device tensor
    error: Optional[str] = None
    slot: int = -1
    footprint: int = 0
    done: threading.Event = field(default_factory=threading.Event)
    on_done: Optional[Callable[["Job"], None]] = None  # called by the slot's thread once the labels are ready


def job_footprint(job: Job) -> int:
    lib = load_library()
    nx, ny, nz = _dims(tuple(job.grad.shape))
    code = 1 if job.grad.element_size() == 1 else 2
    return int(lib.ws_footprint_bytes(nx, ny, nz, int(job.conn), code, int(job.NL)))


class Server:
    """K execution slots, micro-batches of queued jobs, footprint admission."""

    def __init__(self, slots: int = 4, budget_bytes: Optional[int] = None, max_batch_jobs: int = 64,
                 max_batch_pixels: int = 1 << 26, max_job_pixels: Optional[int] = None, device: int = 0,
                 warm_layers: int = 4):
        import torch
        self.device = torch.device("cuda", device)
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(free * 0.6)
        self.budget = int(budget_bytes)
        self.max_batch_jobs = int(max_batch_jobs)
        self.max_batch_pixels = int(max_batch_pixels)
        self.in_use = 0
        self.queue: collections.deque = collections.deque()
        self.lock = threading.Condition()
        self.running = True
        self.completed: List[Job] = []
        self.batches = 0
        self.max_concurrent = 0
        self._busy = 0
        self.slots = []
        for k in range(slots):
            ctx = Context(device)
            reserve = self.max_batch_pixels
            if k == 0 and max_job_pixels:
                reserve = max(reserve, int(max_job_pixels))
            ctx.set_option("reserve_pixels", min(reserve, (1 << 31) - 1))
            stream = torch.cuda.Stream(device=self.device)  # default priority
            if warm_layers > 0:
                # the outputs are torch tensors allocated on the slot's stream:
                # leave a block of warm_layers int32 layers of the reserve in
                # that stream's cache, so outputs are carved from it rather than
                # allocated (allocation stalls every slot)
                with torch.cuda.stream(stream):
                    warm = torch.empty(int(warm_layers) * reserve, dtype=torch.int32, device=self.device)
                    del warm
            slot = {"k": k, "ctx": ctx, "stream": stream, "work": None, "cv": threading.Condition()}
            slot["thread"] = threading.Thread(target=self._worker, args=(slot,), daemon=True)
            self.slots.append(slot)
        for s in self.slots:
            s["thread"].start()
        self.dispatcher = threading.Thread(target=self._dispatch, daemon=True)
        self.dispatcher.start()

    # -- client side --------------------------------------------------------
    def submit(self, job: Job) -> Job:
        job.t_arrival = time.perf_counter()
        job.footprint = job_footprint(job)
        with self.lock:
            if job.footprint > self.budget:
                job.error = "footprint %d exceeds the device budget %d" % (job.footprint, self.budget)
                job.t_done = time.perf_counter()
                job.done.set()
                self.completed.append(job)
                return job
            self.queue.append(job)
            self.lock.notify_all()
        return job

    def drain(self, timeout: Optional[float] = None) -> bool:
        t_end = None if timeout is None else time.perf_counter() + timeout
        with self.lock:
            while self.queue or self._busy:
                left = None if t_end is None else t_end - time.perf_counter()
                if left is not None and left <= 0:
                    return False
                self.lock.wait(left if left is not None else 1.0)
        return True

    def close(self):
        self.drain()
        with self.lock:
            self.running = False
            self.lock.notify_all()
        for s in self.slots:
            with s["cv"]:
                s["cv"].notify_all()
        self.dispatcher.join(timeout=5)
        for s in self.slots:
            s["thread"].join(timeout=5)
            s["ctx"].close()

    # -- scheduling ---------------------------------------------------------
    def _oversized(self, job: Job) -> bool:
        return int(job.grad.numel()) > self.max_batch_pixels

    def _take_batch(self, allow_big: bool):
        """Under the lock: the longest compatible micro-batch that fits, led by
        the oldest queued job (the oldest ordinary one unless allow_big)."""
        batch, pix, foot = [], 0, 0
        head = None
        rest = collections.deque()
        while self.queue and len(batch) < self.max_batch_jobs:
            j = self.queue.popleft()
            if not allow_big and self._oversized(j):
                rest.append(j)
                continue
            if head is None:
                head = j
            n = int(j.grad.numel())
            # one ws_batch call takes any mix of 2D and 3D images and
            # connectivities; its NL and grey type are shared
            same = j.NL == head.NL and j.grad.dtype == head.grad.dtype
            fits = self.in_use + foot + j.footprint <= self.budget and (not batch or pix + n <= self.max_batch_pixels)
            if same and fits:
                batch.append(j)
                pix += n
                foot += j.footprint
            else:
                rest.append(j)
                if not fits and same:
                    break
        while rest:
            self.queue.appendleft(rest.pop())
        return batch, foot

    def _pick_slot(self):
        """Under the lock: (slot, allow_big) for the next micro-batch, or None.
        Oversized jobs run on slot 0 only; ordinary batches prefer the other
        slots, so an oversized job at the head of the queue delays no one."""
        zero = self.slots[0]
        if zero["work"] is None and self._oversized(self.queue[0]):
            return zero, True
        for s in self.slots[1:]:
            if s["work"] is None:
                return s, False
        if zero["work"] is None:
            return zero, True
        return None

    def _dispatch(self):
        while True:
            with self.lock:
                while self.running and not (self.queue and any(s["work"] is None for s in self.slots)):
                    self.lock.wait(0.05)
                if not self.running:
                    return
                pick = self._pick_slot()
                batch, foot = self._take_batch(pick[1]) if pick else ([], 0)
                if not batch:
                    # only oversized jobs wait for slot 0, or memory is busy:
                    # every completion and submission notifies
                    self.lock.wait(0.05)
                    continue
                slot = pick[0]
                self.in_use += foot
                self._busy += 1
                self.max_concurrent = max(self.max_concurrent, self._busy)
                self.batches += 1
                now = time.perf_counter()
                for j in batch:
                    j.t_start = now
                    j.slot = slot["k"]
                with slot["cv"]:
                    slot["work"] = (batch, foot)
                    slot["cv"].notify()

    def _worker(self, slot):
        import torch
        ctx, stream = slot["ctx"], slot["stream"]
        while True:
            with slot["cv"]:
                while slot["work"] is None and self.running:
                    slot["cv"].wait(0.05)
                if slot["work"] is None:
                    return
                batch, foot = slot["work"]
            outs = nregs = None
            try:
                with torch.cuda.stream(stream):
                    grads = [j.grad for j in batch]
                    NL = batch[0].NL
                    outs = [torch.empty((NL,) + tuple(g.shape), dtype=torch.int32, device=self.device) for g in grads]
                    nregs = [torch.zeros(NL, dtype=torch.int64, device=self.device) for _ in grads]
                    ctx.batch(grads, [j.conn for j in batch], NL, outs=outs, nregions=nregs)
                stream.synchronize()
                t = time.perf_counter()
                for j, o, n in zip(batch, outs, nregs):
                    j.out, j.nregions, j.t_done = o, n, t
            except WSError as e:
                t = time.perf_counter()
                for j in batch:
                    j.error, j.t_done = str(e), t
            outs = nregs = None  # the jobs hold the results now
            for j in batch:
                if j.on_done is not None:
                    try:
                        j.on_done(j)
                    except Exception:  # a client's callback must not stop the slot
                        traceback.print_exc()
            with self.lock:
                self.in_use -= foot
                self._busy -= 1
                self.completed.extend(batch)
                with slot["cv"]:
                    slot["work"] = None
                self.lock.notify_all()
            for j in batch:
                j.done.set()


def percentile(xs, q):
    if not xs:
        return float("nan")
    s = sorted(xs)
    k = min(len(s) - 1, max(0, int(round(q / 100.0 * (len(s) - 1)))))
    return s[k]
