"""Continuous-batching colouring server on one GPU.

Jobs (one graph each) arrive at any time.  The server keeps an arena of
device memory of a fixed budget and a table of at most `max_slots` resident
jobs:

* admission -- a waiting job is admitted, in arrival order, when a slot is
  free and its footprint (rowptr + colidx + colour/state words) fits in the
  arena (first-fit); its CSR is copied into the arena on a copy stream while
  the GPU keeps computing (from pinned host memory, or, when the request
  already lives on the GPU, by one gc_copy_segments launch for all the jobs
  admitted together), and the compute stream waits for that copy only before
  the first step that includes the job;
* step -- one gc_batch_step launch advances every resident job by at most
  `rounds_per_step` rounds (each job keeps its own round count; a job's whole
  state between steps is its colour array), so new jobs start as soon as
  they are admitted instead of waiting for the batch to drain.  A step
  launched while jobs that have arrived are still waiting (for a slot, for
  arena space, or for this step's admission, which has already happened)
  runs up to `backlog_rounds_per_step` rounds instead: under a steady stream
  of arrivals that is nearly every step, and fewer, longer steps carry less
  per-step overhead, which raises the rate the server sustains; a step with
  no one waiting keeps the short round count, so an isolated job is
  returned after fewer rounds of its neighbours' work;
* pipelining -- the descriptor table lives on the device and each step
  updates it in place; a step is queued before the previous one has been
  waited for, so the host admits, copies and retires while the GPU runs, and
  blocks only on the oldest of the two steps in flight.  A step's rounds and
  uncoloured counts come back by an asynchronous copy into pinned memory;
* retirement -- a job whose round had no loser is done: its completion time
  is when the host sees the step that finished it; it leaves the table at
  the next launch, and its memory and slot are reused once the step queued
  behind it (which still lists it, and leaves its colours unchanged) has run.

Each job's colouring is exactly the one gc_color gives for its graph alone
(the rounds of a job never depend on the other jobs).  Latency is measured
from a job's arrival to the host seeing the end of the step that finished it.
"""
from __future__ import annotations

import bisect
import collections
import gc as pygc
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import gc


class ArenaAllocator:
    """Best-fit allocator over [0, capacity) in units of int32 words: a
    request takes the smallest free block that holds it (the lowest such on
    ties), and freed neighbours coalesce.  Free blocks are indexed twice,
    by start and by (size, start), in sorted lists searched by bisection,
    so a call costs a binary search and a list insertion whatever the
    number of free blocks (a first-fit walk over a few thousand fragments
    once held a serving step for over 100 ms)."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self._starts = []      # free blocks, sorted by start
        self._sizes = {}       # start -> size
        self._by_size = []     # (size, start), sorted
        self.used = 0
        if self.capacity > 0:
            self._add(0, self.capacity)

    def _add(self, start: int, size: int):
        bisect.insort(self._starts, start)
        self._sizes[start] = size
        bisect.insort(self._by_size, (size, start))

    def _remove(self, start: int) -> int:
        size = self._sizes.pop(start)
        del self._starts[bisect.bisect_left(self._starts, start)]
        del self._by_size[bisect.bisect_left(self._by_size, (size, start))]
        return size

    def alloc(self, size: int):
        size = int(size)
        if size <= 0:
            raise ValueError("allocation size must be positive")
        i = bisect.bisect_left(self._by_size, (size, -1))
        if i == len(self._by_size):
            return None
        have, s = self._by_size[i]
        self._remove(s)
        if have > size:
            self._add(s + size, have - size)
        self.used += size
        return s

    def release(self, start: int, size: int):
        start, size = int(start), int(size)
        i = bisect.bisect_left(self._starts, start)
        if i < len(self._starts) and self._starts[i] < start + size:
            raise ValueError("double free or overlapping release")
        if i > 0:
            p = self._starts[i - 1]
            if p + self._sizes[p] > start:
                raise ValueError("double free or overlapping release")
        self.used -= size
        if i < len(self._starts) and start + size == self._starts[i]:
            size += self._remove(self._starts[i])
        if i > 0:
            prv = self._starts[i - 1]
            if prv + self._sizes[prv] == start:
                size += self._remove(prv)
                start = prv
        self._add(start, size)

    def release_many(self, starts, sizes):
        """Free several blocks at once (a serving step's finished jobs): the
        free list and the released blocks are merged, checked for overlap
        and coalesced in one sorted pass, and both indexes rebuilt; a
        handful of blocks take the per-block path instead."""
        st = np.asarray(starts, np.int64).ravel()
        sz = np.asarray(sizes, np.int64).ravel()
        if st.size != sz.size:
            raise ValueError("starts and sizes differ in length")
        if st.size < 32:
            for a, b in zip(st.tolist(), sz.tolist()):
                self.release(a, b)
            return
        if np.any(sz <= 0) or np.any(st < 0) or np.any(st + sz > self.capacity):
            raise ValueError("release outside the arena")
        nf = len(self._starts)
        fs = np.fromiter(self._starts, np.int64, nf)
        fz = np.fromiter((self._sizes[a] for a in self._starts), np.int64, nf)
        allst = np.concatenate([fs, st])
        allsz = np.concatenate([fz, sz])
        order = np.argsort(allst, kind="stable")
        allst, allsz = allst[order], allsz[order]
        ends = allst + allsz
        if np.any(ends[:-1] > allst[1:]):
            raise ValueError("double free or overlapping release")
        head = np.ones(allst.size, bool)
        head[1:] = ends[:-1] != allst[1:]          # a block not touching the previous one
        first = np.nonzero(head)[0]
        rs = allst[first]
        rz = np.add.reduceat(allsz, first)
        by = np.lexsort((rs, rz))
        self._starts = rs.tolist()
        self._sizes = dict(zip(self._starts, rz.tolist()))
        self._by_size = list(zip(rz[by].tolist(), rs[by].tolist()))
        self.used -= int(sz.sum())

    def largest_free(self) -> int:
        return self._by_size[-1][0] if self._by_size else 0

    def free_blocks(self):
        return [(s, self._sizes[s]) for s in self._starts]


def _round64(w: int) -> int:
    return (w + 63) // 64 * 64


def job_words(n: int, nnz: int) -> int:
    """Arena footprint of a job in int32 words: rowptr, colidx, colours,
    each rounded up to a multiple of 64 words (256 bytes)."""
    return _round64(n + 1) + _round64(max(nnz, 1)) + _round64(max(n, 1))


@dataclass(slots=True)
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
    on_device: bool = False   # both arrays live on the server's device
    rp_ptr: int = 0           # their device addresses (when on_device)
    ci_ptr: int = 0

    @property
    def latency(self) -> float:
        return self.finished_at - self.arrival


def _as_int32_tensor(a) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        t = a if a.dtype == torch.int32 else a.to(torch.int32)
        if not t.is_contiguous():
            t = t.contiguous()
        if not t.is_cuda and not t.is_pinned():
            t = t.pin_memory()
        return t
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).pin_memory()


class _Step:
    """A launched step: its completion event, the pinned copy of the table it
    wrote, and the job ids of its table rows in order."""

    def __init__(self, number, event, table_host, row_ids):
        self.number = number
        self.event = event
        self.table_host = table_host
        self.row_ids = row_ids


class Server:
    """Continuous batching of colouring jobs on one device."""

    PIPELINE = 2  # steps in flight

    def __init__(self, budget_bytes: int, max_slots: int = 1024, rounds_per_step: int = 4,
                 device=None, keep_colors: bool = True, backlog_rounds_per_step: int | None = None):
        if budget_bytes < 4096:
            raise ValueError("budget too small")
        self.device = torch.device(device or "cuda:0")
        self.words = budget_bytes // 4
        self.arena = torch.empty(self.words, dtype=torch.int32, device=self.device)
        self.alloc = ArenaAllocator(self.words)
        self.max_slots = int(max_slots)
        self.rounds_per_step = int(rounds_per_step)
        self.backlog_rounds_per_step = int(4 * rounds_per_step if backlog_rounds_per_step is None
                                           else backlog_rounds_per_step)
        self.backlog_steps = 0             # steps launched with the backlog's round count
        self.max_wait_s = 0.0              # longest wait for a step's completion event
        self.max_host_s = 0.0              # longest host time of one step() outside that wait
        self.keep_colors = keep_colors
        self.compute = torch.cuda.Stream(self.device)
        self.copy = torch.cuda.Stream(self.device)
        self.readback = torch.cuda.Stream(self.device)
        self.waiting: collections.deque[Job] = collections.deque()
        self.jobs: dict[int, Job] = {}     # admitted and not yet released, by id
        self.row_ids = np.zeros(0, np.int64)  # job ids of the device table, in row order
        self.table = None                  # device table (uint8, rows * desc size)
        self.finished = np.zeros(1024, bool)  # by job id: found finished
        self.dead = 0                      # finished jobs still in row_ids
        self.inflight: collections.deque[_Step] = collections.deque()
        self.free_after_next: list[Job] = []  # finished, still listed by a step in flight
        self.done: dict[int, Job] = {}
        self.steps = 0
        self._next_id = 0
        self._pending_copy = None          # event of the last admission copy
        self._keep = []                    # staging tensors alive until their copy has run
        self._resident = 0                 # admitted and not yet finished
        self._waited = 0.0                 # event waits of the current step()
        self.clock = time.perf_counter
        gc.desc_array([])                  # the record layout (gc.DESC_DTYPE)
        # Pinned host staging, allocated once: a ring of PIPELINE + 1 sets,
        # set k used by the steps numbered k mod (PIPELINE + 1).  A set is
        # rewritten only when the step that used it last has completed (the
        # loop waits for step s - 1 before queueing step s + 1).  Pinned
        # allocations inside the loop went to the system allocator whenever a
        # new size appeared, and one took 147 ms (measured).
        ring = self.PIPELINE + 1
        rec = gc.DESC_DTYPE.itemsize
        self._pin_table = [torch.empty(self.max_slots * rec, dtype=torch.uint8, pin_memory=True)
                           for _ in range(ring)]
        self._pin_rows = [torch.empty(self.max_slots * rec, dtype=torch.uint8, pin_memory=True)
                          for _ in range(ring)]
        # descriptors of the table compaction: one segment per run of kept rows
        self._pin_kdesc = [torch.empty(self.max_slots * 4, dtype=torch.int64, pin_memory=True)
                           for _ in range(ring)]
        if rec % 4:
            raise RuntimeError("descriptor records must be whole int32 words")
        self._pin_desc = [torch.empty(2 * self.max_slots * 4, dtype=torch.int64, pin_memory=True)
                          for _ in range(ring)]
        # Device buffers, allocated once as well (a new size class inside the
        # loop reached the device allocator, and one step's set-up took 64 ms,
        # measured): the descriptor table in one of two buffers (a step's
        # kept rows are copied into the other; both are used only on the
        # compute stream, in order), the descriptors of that copy (compute
        # stream) and of the admission copies (copy stream), and the step
        # workspace.
        self._dtab = [torch.empty(self.max_slots * rec, dtype=torch.uint8, device=self.device)
                      for _ in range(2)]
        self._dcur = 0                     # the buffer holding the table
        self._rows = 0                     # rows of the table
        self._dkdesc = torch.empty(self.max_slots * 4, dtype=torch.int64, device=self.device)
        self._ddesc = torch.empty(2 * self.max_slots * 4, dtype=torch.int64, device=self.device)
        self._ws = torch.empty(max(gc.gc_batch_step_workspace_bytes(self.max_slots, 0), 1),
                               dtype=torch.uint8, device=self.device)

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
        if rp.is_cuda and ci.is_cuda and rp.device == self.device and ci.device == self.device:
            job.on_device = True
            job.rp_ptr = rp.data_ptr()
            job.ci_ptr = ci.data_ptr()
        self._next_id += 1
        if self._next_id > self.finished.size:
            self.finished = np.concatenate([self.finished, np.zeros(self.finished.size, bool)])
        self.waiting.append(job)
        return job.id

    def submit_packed(self, voff, eoff, rowptr_local, colidx_local, arrivals) -> range:
        """Queue every graph of a packed batch already on this device, in the
        layout of gc_color_batch (graph g: rowptr_local[voff[g] + g ..
        voff[g + 1] + g], colidx_local[eoff[g] .. eoff[g + 1]]; voff, eoff
        host arrays), graph g arriving at arrivals[g] (absolute times on the
        server's clock).  Returns the job ids.  The caller keeps the tensors
        alive and unchanged until the jobs are admitted."""
        voff = np.asarray(voff, np.int64)
        eoff = np.asarray(eoff, np.int64)
        G = voff.size - 1
        if not (rowptr_local.is_cuda and colidx_local.is_cuda
                and rowptr_local.device == self.device and colidx_local.device == self.device
                and rowptr_local.dtype == torch.int32 and colidx_local.dtype == torch.int32
                and rowptr_local.is_contiguous() and colidx_local.is_contiguous()):
            raise ValueError("submit_packed takes contiguous int32 tensors on the server's device")
        n = np.diff(voff)
        nnz = np.diff(eoff)
        if G and (n.min() < 0 or nnz.min() < 0 or voff[-1] + G > rowptr_local.numel()
                  or eoff[-1] > colidx_local.numel()):
            raise ValueError("offsets do not fit the packed arrays")
        words = (n + 1 + 63) // 64 * 64 + (np.maximum(nnz, 1) + 63) // 64 * 64 \
            + (np.maximum(n, 1) + 63) // 64 * 64
        if G and words.max() > self.words:
            raise gc.GCError(gc.GC_ETOOBIG, f"a job needs {int(words.max()) * 4} bytes, budget is "
                                            f"{self.words * 4}")
        rp_ptr = rowptr_local.data_ptr() + 4 * (voff[:-1] + np.arange(G))
        ci_ptr = colidx_local.data_ptr() + 4 * eoff[:-1]
        arrivals = np.asarray(arrivals, np.float64)
        first = self._next_id
        need = first + G
        if need > self.finished.size:
            self.finished = np.concatenate([self.finished,
                                            np.zeros(max(need, 2 * self.finished.size)
                                                     - self.finished.size, bool)])
        for g, (ng, eg, wg, a, rpp, cip) in enumerate(zip(n.tolist(), nnz.tolist(), words.tolist(),
                                                          arrivals.tolist(), rp_ptr.tolist(),
                                                          ci_ptr.tolist())):
            job = Job(first + g, None, None, a, ng, eg, wg)
            job.on_device = True
            job.rp_ptr = rpp
            job.ci_ptr = cip
            self.waiting.append(job)
        self._next_id = need
        return range(first, need)

    def idle(self) -> bool:
        return not self.waiting and self._resident == 0 and not self.inflight

    def result(self, job_id: int) -> Job:
        return self.done[job_id]

    # ---------------------------------------------------------- machinery --
    def _admit(self, now: float):
        new = []
        while self.waiting and self._resident + len(new) < self.max_slots:
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
            self.jobs[job.id] = job
            new.append(job)
        if not new:
            return new
        # the request tensors may still be being written by work queued on the
        # caller's stream: the copies start after it
        self.copy.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.copy):
            # CSR already on the device: every array of the admitted jobs in
            # one gc_copy_segments launch, its descriptors built from the
            # addresses recorded at submission; host arrays: one copy each
            dev_jobs = [j for j in new if j.on_device]
            desc = None
            if dev_jobs:
                base = self.arena.data_ptr()
                off = np.fromiter((j.offset for j in dev_jobs), np.int64, len(dev_jobs))
                n = np.fromiter((j.n for j in dev_jobs), np.int64, len(dev_jobs))
                nnz = np.fromiter((j.nnz for j in dev_jobs), np.int64, len(dev_jobs))
                rpw = (n + 1 + 63) // 64 * 64
                src = np.empty(2 * len(dev_jobs), np.int64)
                dst = np.empty_like(src)
                words = np.empty_like(src)
                src[0::2] = np.fromiter((j.rp_ptr for j in dev_jobs), np.int64, len(dev_jobs))
                src[1::2] = np.fromiter((j.ci_ptr for j in dev_jobs), np.int64, len(dev_jobs))
                dst[0::2] = base + 4 * off
                dst[1::2] = base + 4 * (off + rpw)
                words[0::2] = n + 1
                words[1::2] = nnz
                desc = gc.copy_segments_raw(src, dst, words, self.device, stream=self.copy,
                                            host_buf=self._pin_desc[self.steps % len(self._pin_desc)],
                                            dev_buf=self._ddesc)
            for job in new:
                if job.on_device:
                    continue
                rpw = _round64(job.n + 1)
                self.arena[job.offset:job.offset + job.n + 1].copy_(job.rowptr, non_blocking=True)
                if job.nnz:
                    self.arena[job.offset + rpw:job.offset + rpw + job.nnz].copy_(
                        job.colidx, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy)
        # descriptors and sources stay referenced until the step that waits
        # for this copy has been queued behind it
        self._keep.append((desc, [(j.rowptr, j.colidx) for j in new]))
        self._pending_copy = ev
        self._resident += len(new)
        return new

    def _launch(self, new):
        """Queue one step over the table: finished rows dropped, new rows
        appended, then gc_batch_step in place and the table copied back."""
        slot = self.steps % len(self._pin_table)
        rec = gc.DESC_DTYPE.itemsize
        with torch.cuda.stream(self.compute):
            if self.dead:
                keep = np.nonzero(~self.finished[self.row_ids])[0]
                self.row_ids = self.row_ids[keep]
                self.dead = 0
                if keep.size:
                    # the kept rows move to the other buffer, one segment per
                    # run of consecutive rows, with the library's segment copy
                    # (descriptors staged in the pinned ring: nothing here
                    # waits for the step in flight).  torch.index_select did
                    # this before and once held the host for 149 ms inside
                    # the call (measured), which every job in flight waited out.
                    brk = np.flatnonzero(np.diff(keep) != 1) + 1
                    first = np.concatenate(([0], brk))
                    last = np.concatenate((brk, [keep.size]))
                    gc.copy_segments_raw(
                        self._dtab[self._dcur].data_ptr() + keep[first] * rec,
                        self._dtab[1 - self._dcur].data_ptr() + first * rec,
                        (last - first) * (rec // 4), self.device, stream=self.compute,
                        host_buf=self._pin_kdesc[slot], dev_buf=self._dkdesc)
                    self._dcur = 1 - self._dcur
                self._rows = int(keep.size)
            if new:
                k = len(new)
                off = np.fromiter((j.offset for j in new), np.int64, k)
                n = np.fromiter((j.n for j in new), np.int64, k)
                nnz = np.fromiter((j.nnz for j in new), np.int64, k)
                rpw = (n + 1 + 63) // 64 * 64
                ciw = (np.maximum(nnz, 1) + 63) // 64 * 64
                rows = np.zeros(k, gc.DESC_DTYPE)
                rows["rowptr_off"] = off
                rows["colidx_off"] = off + rpw
                rows["color_off"] = off + rpw + ciw
                rows["n"] = n
                h = self._pin_rows[slot][:rows.nbytes]
                h.numpy()[:] = rows.view(np.uint8)
                dst = self._dtab[self._dcur].view(self.max_slots, rec)[self._rows:self._rows + k]
                dst.view(-1).copy_(h, non_blocking=True)
                self._rows += k
                self.row_ids = np.concatenate([self.row_ids,
                                               np.array([j.id for j in new], np.int64)])
            self.table = self._dtab[self._dcur][:self._rows * rec]
            if self._pending_copy is not None:
                self.compute.wait_event(self._pending_copy)
                self._pending_copy = None
            # a backlog: jobs that have arrived and were not admitted
            backlog = bool(self.waiting) and self.waiting[0].arrival <= self.clock()
            rounds = self.backlog_rounds_per_step if backlog else self.rounds_per_step
            self.backlog_steps += backlog
            self._ws = gc.batch_step(self.table, self.arena, self.arena, self.arena,
                                     rounds, workspace=self._ws, stream=self.compute)
            host = self._pin_table[slot][:self.table.numel()]
            host.copy_(self.table, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.compute)
        self.steps += 1
        self.inflight.append(_Step(self.steps, ev, host, self.row_ids))
        self._keep = []  # queued behind the waits above: safe to drop on the host

    def _complete_oldest(self) -> int:
        st = self.inflight.popleft()
        t0 = self.clock()
        st.event.synchronize()
        now = self.clock()
        self._waited += now - t0
        table = st.table_host.numpy().view(gc.DESC_DTYPE)
        # jobs found finished at the previous completion were still listed by
        # this step; it has run, so their memory can be reused now
        self._release(self.free_after_next)
        self.free_after_next = []
        ids = st.row_ids
        rows = np.nonzero((table["active"] == 0) & ~self.finished[ids])[0]
        finished = []
        jobs, done, number = self.jobs, self.done, st.number
        # whole columns read once: a step can finish thousands of jobs
        for jid, r in zip(ids[rows].tolist(), table["rounds"][rows].tolist()):
            job = jobs[jid]
            job.rounds = r
            job.finished_at = now
            job.finished_step = number
            finished.append(job)
            done[jid] = job
        if rows.size:
            self.finished[ids[rows]] = True
            self.dead += rows.size
            self._resident -= rows.size
        # a step queued behind this one still lists them (its write-back leaves
        # their colours as they are); without one, nothing does
        if self.inflight:
            self.free_after_next = finished
        else:
            self._release(finished)
        return len(finished)

    def _release(self, jobs):
        if not jobs:
            return
        if self.keep_colors:
            # every step that touched these jobs has run; the read uses its own
            # stream, so it does not wait for the step in flight
            h = torch.from_numpy(np.concatenate(
                [np.arange(j.offset + _round64(j.n + 1) + _round64(max(j.nnz, 1)),
                           j.offset + _round64(j.n + 1) + _round64(max(j.nnz, 1)) + j.n,
                           dtype=np.int64) for j in jobs])).pin_memory()
            with torch.cuda.stream(self.readback):
                idx = h.to(self.device, non_blocking=True)
                flat = self.arena.index_select(0, idx).cpu().numpy()
            pos = 0
            for j in jobs:
                j.colors = flat[pos:pos + j.n]
                pos += j.n
        self.alloc.release_many([j.offset for j in jobs], [j.words for j in jobs])
        for j in jobs:
            j.offset = -1
            j.rowptr = j.colidx = None
            del self.jobs[j.id]

    def step(self) -> int:
        """Admit what fits, queue one step over every resident job (at most
        rounds_per_step rounds each), and wait for the oldest step in flight
        once the pipeline is full.  Returns the number of jobs found finished."""
        t0 = self.clock()
        self._waited = 0.0
        new = self._admit(t0)
        finished = 0
        if self._resident > 0 and (new or self.row_ids.size > self.dead):
            self._launch(new)
            while len(self.inflight) >= self.PIPELINE:
                finished += self._complete_oldest()
        elif self.inflight:
            finished += self._complete_oldest()
        self.max_wait_s = max(self.max_wait_s, self._waited)
        self.max_host_s = max(self.max_host_s, self.clock() - t0 - self._waited)
        return finished

    def reset_peaks(self):
        """Zero max_wait_s and max_host_s (for instance between two
        measured arrival streams on one long-lived server)."""
        self.max_wait_s = 0.0
        self.max_host_s = 0.0

    def run_until_idle(self, max_steps: int = 1_000_000):
        # Python's cyclic garbage collector is paused while the loop runs: a
        # full collection in a process holding a few hundred thousand objects
        # stalled the loop for tens of milliseconds (measured), which every
        # job in flight would wait out; the loop itself creates no cycles
        was_enabled = pygc.isenabled()
        pygc.disable()
        try:
            for _ in range(max_steps):
                if self.idle():
                    return
                if (self._resident == 0 and not self.inflight and self.waiting
                        and self.waiting[0].arrival > self.clock()):
                    time.sleep(max(0.0, self.waiting[0].arrival - self.clock()))
                self.step()
            raise RuntimeError("server did not drain")
        finally:
            if was_enabled:
                pygc.enable()

    def serve_packed(self, voff, eoff, rowptr_local, colidx_local, arrivals, repeats: int = 1):
        """serve() for a packed batch already on this device (submit_packed),
        its graphs submitted `repeats` times over: job r * G + g is graph g,
        arriving arrivals[r * G + g] seconds after the submission of all the
        jobs is complete (the schedule is registered first, so its cost does
        not delay the arrivals).  Returns the finished jobs in job order."""
        G = len(voff) - 1
        arrivals = np.asarray(arrivals, np.float64)
        if arrivals.size != repeats * G:
            raise ValueError("one arrival per graph and repetition")
        ids = []
        for r in range(repeats):
            ids += list(self.submit_packed(voff, eoff, rowptr_local, colidx_local,
                                           arrivals[r * G:(r + 1) * G]))
        t0 = self.clock()
        first = ids[0] if ids else self._next_id
        for job in self.waiting:
            if job.id >= first:
                job.arrival += t0
        self.run_until_idle()
        return [self.done[i] for i in ids]

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
