"""Continuous-batching colouring server on one GPU.

Jobs (one graph each) arrive at any time.  The server keeps an arena of
device memory of a fixed budget and a table of at most `max_slots` resident
jobs:

* admission -- a waiting job is admitted, in arrival order, when a slot is
  free and its footprint (rowptr + colidx + colour/state words) fits in the
  arena (first-fit); its CSR is copied into the arena on a copy stream while
  the GPU keeps computing (from pinned host memory, or device to device when
  the request already lives on the GPU), and the compute stream waits for
  that copy only before the first step that includes the job;
* step -- one gc_batch_step launch advances every resident job by at most
  `rounds_per_step` rounds (each job keeps its own round count; a job's whole
  state between steps is its colour array), so new jobs start as soon as
  they are admitted instead of waiting for the batch to drain;
* retirement -- a job whose round had no loser is done: its colours are
  final, its memory and slot are freed at once and go to waiting jobs.

The resident table is kept host-side in exactly the layout of the
descriptors gc_batch_step reads, so a step costs one small host-to-device
copy of the table, one launch, and one copy back.

Each job's colouring is exactly the one gc_color gives for its graph alone
(the rounds of a job never depend on the other jobs).  Latency is measured
from a job's arrival to the end of the step that finished it.
"""
from __future__ import annotations

import bisect
import collections
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import gc


class ArenaAllocator:
    """First-fit allocator over [0, capacity) in units of int32 words, with
    coalescing of freed neighbours."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self._starts = [0] if capacity > 0 else []   # free blocks, sorted by start
        self._sizes = {0: self.capacity} if capacity > 0 else {}
        self.used = 0

    def alloc(self, size: int):
        size = int(size)
        if size <= 0:
            raise ValueError("allocation size must be positive")
        for i, s in enumerate(self._starts):
            have = self._sizes[s]
            if have >= size:
                del self._sizes[s]
                self._starts.pop(i)
                if have > size:
                    self._starts.insert(i, s + size)
                    self._sizes[s + size] = have - size
                self.used += size
                return s
        return None

    def release(self, start: int, size: int):
        start, size = int(start), int(size)
        i = bisect.bisect_left(self._starts, start)
        if i < len(self._starts) and self._starts[i] < start + size:
            raise ValueError("double free or overlapping release")
        if i > 0:
            p = self._starts[i - 1]
            if p + self._sizes[p] > start:
                raise ValueError("double free or overlapping release")
        self._starts.insert(i, start)
        self._sizes[start] = size
        self.used -= size
        if i + 1 < len(self._starts) and start + size == self._starts[i + 1]:
            nxt = self._starts.pop(i + 1)
            self._sizes[start] += self._sizes.pop(nxt)
        if i > 0:
            prv = self._starts[i - 1]
            if prv + self._sizes[prv] == start:
                self._sizes[prv] += self._sizes.pop(start)
                self._starts.pop(i)

    def largest_free(self) -> int:
        return max(self._sizes.values(), default=0)

    def free_blocks(self):
        return [(s, self._sizes[s]) for s in self._starts]


def _round64(w: int) -> int:
    return (w + 63) // 64 * 64


def job_words(n: int, nnz: int) -> int:
    """Arena footprint of a job in int32 words: rowptr, colidx, colours,
    each rounded up to a multiple of 64 words (256 bytes)."""
    return _round64(n + 1) + _round64(max(nnz, 1)) + _round64(max(n, 1))


@dataclass
class Job:
    id: int
    rowptr: torch.Tensor      # int32, pinned host or device
    colidx: torch.Tensor      # int32, pinned host or device
    arrival: float
    n: int
    nnz: int
    words: int
    offset: int = -1
    rounds: int = 0
    admitted_at: float = -1.0
    admitted_step: int = -1
    finished_at: float = -1.0
    finished_step: int = -1
    colors: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.finished_at - self.arrival


def _as_int32_tensor(a) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        t = a if a.dtype == torch.int32 else a.to(torch.int32)
        t = t.contiguous()
        if t.device.type == "cpu" and not t.is_pinned():
            t = t.pin_memory()
        return t
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).pin_memory()


class Server:
    """Continuous batching of colouring jobs on one device."""

    def __init__(self, budget_bytes: int, max_slots: int = 1024, rounds_per_step: int = 4,
                 device=None, keep_colors: bool = True):
        if budget_bytes < 4096:
            raise ValueError("budget too small")
        self.device = torch.device(device or "cuda:0")
        self.words = budget_bytes // 4
        self.arena = torch.empty(self.words, dtype=torch.int32, device=self.device)
        self.alloc = ArenaAllocator(self.words)
        self.max_slots = int(max_slots)
        self.rounds_per_step = int(rounds_per_step)
        self.keep_colors = keep_colors
        self.compute = torch.cuda.Stream(self.device)
        self.copy = torch.cuda.Stream(self.device)
        self.waiting: collections.deque[Job] = collections.deque()
        self.jobs: list[Job] = []                       # resident, in table order
        self.table = gc.desc_array([])                  # resident descriptors
        self.done: dict[int, Job] = {}
        self.steps = 0
        self._next_id = 0
        self._ws = None
        self._pending_copy = None                       # event of the last admission copy
        self._pending_desc = None                       # its segment descriptors (device)
        self.clock = time.perf_counter

    # -------------------------------------------------------------- API --
    def submit(self, rowptr, colidx, arrival: float | None = None) -> int:
        """Queue one graph (simple, symmetric, sorted rows; int32 CSR as
        numpy arrays or torch tensors, host or device)."""
        rp = _as_int32_tensor(rowptr)
        ci = _as_int32_tensor(colidx)
        n = rp.numel() - 1
        nnz = ci.numel()
        if n < 0:
            raise ValueError("rowptr needs at least one entry")
        words = job_words(n, nnz)
        if words > self.words:
            raise gc.GCError(gc.GC_ETOOBIG, f"job needs {words * 4} bytes, budget is "
                                            f"{self.words * 4}")
        job = Job(self._next_id, rp, ci, self.clock() if arrival is None else arrival, n, nnz, words)
        self._next_id += 1
        self.waiting.append(job)
        return job.id

    def idle(self) -> bool:
        return not self.waiting and not self.jobs

    def result(self, job_id: int) -> Job:
        return self.done[job_id]

    # ---------------------------------------------------------- machinery --
    def _admit(self, now: float):
        new = []
        while self.waiting and len(self.jobs) + len(new) < self.max_slots:
            job = self.waiting[0]
            if job.arrival > now:
                break
            off = self.alloc.alloc(job.words)
            if off is None:
                break  # admission stays in arrival order
            self.waiting.popleft()
            job.offset = off
            job.admitted_at = self.clock()
            job.admitted_step = self.steps
            new.append(job)
        if not new:
            return
        # the request tensors may still be being written by work queued on the
        # caller's stream: the copies start after it
        self.copy.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.copy):
            # CSR already on the device: every array of the admitted jobs in
            # one gc_copy_segments launch; host arrays: one copy each
            staged = []
            for job in new:
                rpw = _round64(job.n + 1)
                rp_dst = self.arena[job.offset:job.offset + job.n + 1]
                ci_dst = self.arena[job.offset + rpw:job.offset + rpw + job.nnz]
                for src, dst in ((job.rowptr, rp_dst), (job.colidx, ci_dst)):
                    if src.numel() == 0:
                        continue
                    if src.is_cuda and src.device == self.device:
                        staged.append((src, dst))
                    else:
                        dst.copy_(src, non_blocking=True)
            self._pending_desc = gc.copy_segments(staged, stream=self.copy)
            ev = torch.cuda.Event()
            ev.record(self.copy)
        self._pending_copy = ev
        rows = []
        for job in new:
            rpw = _round64(job.n + 1)
            ciw = _round64(max(job.nnz, 1))
            rows.append((job.offset, job.offset + rpw, job.offset + rpw + ciw, job.n, 0))
        self.table = np.concatenate([self.table, gc.desc_array(rows)])
        self.jobs.extend(new)

    def step(self) -> int:
        """Admit what fits, advance every resident job by at most
        rounds_per_step rounds, retire finished jobs.  Returns the number of
        jobs finished by this step."""
        self._admit(self.clock())
        if not self.jobs:
            return 0
        with torch.cuda.stream(self.compute):
            if self._pending_copy is not None:
                self.compute.wait_event(self._pending_copy)
                self._pending_copy = None
                self._pending_desc = None  # the copy stream has it; the step waits for it
            d_dev = torch.from_numpy(self.table.view(np.uint8)).to(self.device, non_blocking=False)
            self._ws = gc.batch_step(d_dev, self.arena, self.arena, self.arena,
                                     self.rounds_per_step, workspace=self._ws,
                                     stream=self.compute)
            back = d_dev.cpu()   # waits for the step
        self.steps += 1
        now = self.clock()
        table = back.numpy().view(gc.DESC_DTYPE).copy()
        fin = np.nonzero(table["active"] == 0)[0]
        if fin.size:
            if self.keep_colors:
                spans = [(int(table["color_off"][i]), int(table["n"][i])) for i in fin]
                idx = torch.from_numpy(np.concatenate(
                    [np.arange(o, o + n, dtype=np.int64) for o, n in spans] or
                    [np.zeros(0, np.int64)])).to(self.device)
                with torch.cuda.stream(self.compute):
                    flat = self.arena.index_select(0, idx).cpu().numpy()
                pos = 0
            for k, i in enumerate(fin):
                j = self.jobs[i]
                j.rounds = int(table["rounds"][i])
                j.finished_at = now
                j.finished_step = self.steps
                if self.keep_colors:
                    j.colors = flat[pos:pos + j.n]
                    pos += j.n
                self.alloc.release(j.offset, j.words)
                j.offset = -1
                j.rowptr = j.colidx = None
                self.done[j.id] = j
            keep = table["active"] != 0
            self.jobs = [j for j, k in zip(self.jobs, keep) if k]
            self.table = table[keep]
        else:
            self.table = table
        for j, r in zip(self.jobs, self.table["rounds"]):
            j.rounds = int(r)
        return int(fin.size)

    def run_until_idle(self, max_steps: int = 1_000_000):
        for _ in range(max_steps):
            if self.idle():
                return
            if not self.jobs and self.waiting and self.waiting[0].arrival > self.clock():
                time.sleep(max(0.0, self.waiting[0].arrival - self.clock()))
            self.step()
        raise RuntimeError("server did not drain")

    def serve(self, graphs, arrivals, t0: float | None = None):
        """Submit graphs[i] (objects with .rowptr, .colidx) at time
        t0 + arrivals[i] (seconds, non-decreasing) while stepping; returns the
        finished jobs in submission order."""
        payload = [(_as_int32_tensor(g.rowptr), _as_int32_tensor(g.colidx)) for g in graphs]
        t0 = self.clock() if t0 is None else t0
        ids = [self.submit(rp, ci, arrival=t0 + float(a)) for (rp, ci), a in zip(payload, arrivals)]
        self.run_until_idle()
        return [self.done[i] for i in ids]


def latency_summary(jobs):
    lat = np.array([j.latency for j in jobs], dtype=np.float64)
    if lat.size == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3), "jobs": int(lat.size)}
