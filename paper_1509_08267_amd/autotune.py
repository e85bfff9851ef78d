"""Autotuner for the per-graph colouring path.

It picks, for one graph on one device:

* ``lanes``: lanes per light vertex in the pull speculate, so 64 / lanes
  vertices per wavefront;
* ``medium_degree``: the light/medium split (above it, a wavefront per vertex);
* ``heavy_degree``: the medium/heavy split (from it, a 256-thread workgroup per
  vertex);
* ``blocks_per_cu``: workgroups per compute unit in the round kernels.

It times colourings of the graph itself and walks the knobs one at a time
(coordinate descent: each knob is set to its fastest candidate with the others
held, in the order above).  The choice is cached in a JSON file keyed by the
device (architecture, compute units, memory) and a graph class (id width, log2
buckets of n, average and maximum degree, algorithm), so later graphs of the
same class reuse it without timing.

Every setting must give the same colours: a round's outcome depends only on
the state at the start of the round, never on how vertices are mapped to
lanes, wavefronts or workgroups.  ``tune`` checks this on every colouring it
times and raises if a candidate disagrees.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass, field

import torch

from . import gc

KNOBS = ("lanes", "medium_degree", "heavy_degree", "blocks_per_cu")

DEFAULT_CANDIDATES = {
    "lanes": [2, 4, 8, 16, 32],
    "medium_degree": [0, 32, 64, 128, 256, 512],   # 0: the library's rule
    "heavy_degree": [1024, 2048, 4096, 8192, 16384],
    "blocks_per_cu": [2, 3, 4, 6, 8, 12, 16],
}

_OPT_IDS = {"lanes": gc.GC_OPT_LANES, "medium_degree": gc.GC_OPT_MEDIUM_DEGREE,
            "heavy_degree": gc.GC_OPT_HEAVY_DEGREE, "blocks_per_cu": gc.GC_OPT_BLOCKS_PER_CU}


# Settings the autotuner chose on the devices it was run on, shipped with the
# library (same layout as the user cache, read-only): a graph class found
# here is not tuned again unless the caller asks for it.
SHIPPED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def default_cache_path() -> str:
    return os.environ.get("GC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache",
                                       "paper_1509_08267_amd", "autotune.json"))


def _bucket(x: float) -> int:
    return int(math.floor(math.log2(x))) if x >= 1 else 0


def graph_class(n: int, nnz: int, max_degree: int, rowptr_i64: bool, algorithm: str) -> str:
    """Key of the graph class a tuned setting is reused for."""
    avg = nnz / n if n else 0.0
    return (f"rp{64 if rowptr_i64 else 32}-n{_bucket(n)}-avg{_bucket(avg)}"
            f"-max{_bucket(max_degree)}-{algorithm}")


def device_key(device: int = 0) -> str:
    """Architecture, compute units and memory size (the marketing name is
    left out: it is not reported the same way under every tool)."""
    p = torch.cuda.get_device_properties(device)
    arch = getattr(p, "gcnArchName", "")
    return f"{arch}|cu{p.multi_processor_count}|mem{p.total_memory >> 30}GiB"


def coordinate_descent(knobs, candidates, measure, start):
    """Pure search: ``measure(setting) -> seconds``; returns (best, table).

    Knobs are visited in order; each takes the candidate with the lowest
    measured time while the others are held at their current best, and the
    start setting's own value competes as a candidate."""
    best = dict(start)
    table = []
    best_t = measure(dict(best))
    table.append((dict(best), best_t))
    for k in knobs:
        for c in candidates.get(k, []):
            if c == best.get(k):
                continue
            trial = dict(best)
            trial[k] = c
            t = measure(trial)
            table.append((trial, t))
            if t < best_t:
                best, best_t = trial, t
    return best, best_t, table


@dataclass
class TuneResult:
    setting: dict
    seconds: float
    baseline_seconds: float
    table: list = field(default_factory=list)
    cached: bool = False

    @property
    def speedup(self) -> float:
        return self.baseline_seconds / self.seconds if self.seconds > 0 else 1.0


class Cache:
    """JSON file: {device_key: {graph_class: {"setting": {...}, "seconds": t}}}."""

    def __init__(self, path: str | None = None, shipped: str | None = SHIPPED_PATH):
        self.path = path or default_cache_path()
        self.data = {}
        self.shipped = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.data = json.load(f)
        if shipped and os.path.exists(shipped):
            with open(shipped) as f:
                self.shipped = json.load(f)

    def get(self, dev: str, cls: str):
        """The user cache's entry, else the shipped one (or None)."""
        hit = self.data.get(dev, {}).get(cls)
        return hit if hit is not None else self.shipped.get(dev, {}).get(cls)

    def put(self, dev: str, cls: str, setting: dict, seconds: float) -> None:
        self.data.setdefault(dev, {})[cls] = {"setting": setting, "seconds": seconds}
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def apply(graph: "gc.Graph", setting: dict) -> None:
    for k, v in setting.items():
        gc.gc_set_option(graph.h, _OPT_IDS[k], int(v))


def current_setting(graph: "gc.Graph") -> dict:
    """The search's starting point: the library's automatic lanes and
    light/medium split (0), and the handle's current heavy split and
    workgroups per CU."""
    return {"lanes": 0, "medium_degree": 0,
            "heavy_degree": graph.get(gc.GC_OPT_HEAVY_DEGREE),
            "blocks_per_cu": graph.get(gc.GC_OPT_BLOCKS_PER_CU)}


def _class_of(graph: "gc.Graph") -> str:
    algo = "push" if graph.get(gc.GC_OPT_ALGORITHM) == gc.GC_ALGO_PUSH else "pull"
    return graph_class(graph.n, graph.m, graph.get(gc.GC_OPT_MAX_DEGREE),
                       graph.rowptr.dtype == torch.int64, algo)


def tune(graph: "gc.Graph", *, reps: int = 5, batch: int = 0, budget_s: float = 20.0,
         candidates: dict | None = None, cache: Cache | None = None,
         use_cache: bool = True) -> TuneResult:
    """Tune ``graph`` in place (its options end at the best setting found).

    ``batch`` colourings are timed per measurement (0: enough for ~2 ms) and
    the median of ``reps`` measurements is the setting's time.  Knobs that
    cannot matter for this graph are skipped (heavy_degree when no vertex
    reaches the smallest candidate).  Tuning stops early, keeping the best so
    far, once ``budget_s`` seconds have passed."""
    cands = {k: list(v) for k, v in (candidates or DEFAULT_CANDIDATES).items()}
    maxdeg = graph.get(gc.GC_OPT_MAX_DEGREE)
    if cands.get("heavy_degree") and maxdeg < min(cands["heavy_degree"]):
        cands["heavy_degree"] = []
    # a light/medium split at or above the maximum degree leaves every vertex
    # light, which the automatic rule already covers when it is that high
    cands["medium_degree"] = [c for c in cands.get("medium_degree", []) if c == 0 or c < maxdeg]
    cache = cache if cache is not None else Cache()
    dev, cls = device_key(graph.colidx.device.index or 0), _class_of(graph)
    if use_cache:
        hit = cache.get(dev, cls)
        if hit is not None:
            apply(graph, hit["setting"])
            return TuneResult(dict(hit["setting"]), hit["seconds"], float("nan"), [], True)

    if graph.n == 0:
        return TuneResult(current_setting(graph), 0.0, 0.0, [], False)
    out = torch.empty(graph.n, dtype=torch.int32, device=graph.colidx.device)
    ref = torch.empty_like(out)
    start = current_setting(graph)
    graph.color(ref)
    graph.stats()
    t0 = time.perf_counter()
    graph.color(out)
    torch.cuda.synchronize()
    one = max(time.perf_counter() - t0, 1e-6)
    nb = batch or max(1, min(50, int(2e-3 / one)))
    deadline = time.perf_counter() + budget_s
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def measure(setting):
        if time.perf_counter() > deadline:
            return float("inf")
        apply(graph, setting)
        graph.color(out)          # first call after a change re-plans the launches
        graph.stats()
        if not torch.equal(out, ref):
            raise RuntimeError(f"autotune: setting {setting} changed the colouring")
        times = []
        for _ in range(reps):
            ev0.record()
            for _ in range(nb):
                graph.color(out)
            ev1.record()
            ev1.synchronize()
            times.append(ev0.elapsed_time(ev1) / 1e3 / nb)
        graph.stats()
        times.sort()
        return times[len(times) // 2]

    best, best_t, table = coordinate_descent(KNOBS, cands, measure, start)
    apply(graph, best)
    base_t = table[0][1]
    if best_t < float("inf"):
        cache.put(dev, cls, best, best_t)
    return TuneResult(best, best_t, base_t, table, False)


def main(argv=None) -> int:
    """Tune the named synthetic workloads on this device and write the
    settings in the cache layout (the shipped table is made this way):

        python -m paper_1509_08267_amd.autotune --out tuning.json er_1m_16m ...
    """
    import argparse

    import numpy as np

    import graphgen
    p = argparse.ArgumentParser(description=main.__doc__)
    p.add_argument("--out", required=True)
    p.add_argument("--budget", type=float, default=25.0)
    p.add_argument("workloads", nargs="+")
    args = p.parse_args(argv)
    cache = Cache(args.out, shipped=None)
    for name in args.workloads:
        g = graphgen.workload(name)
        rp64 = g.nnz > 2**31 - 1 or name == "rmat22_ef16"
        rp = torch.from_numpy(g.rowptr.astype(np.int64 if rp64 else np.int32)).cuda()
        ci = torch.from_numpy(g.colidx).cuda()
        with gc.Graph(rp, ci) as G:
            res = tune(G, budget_s=args.budget, cache=cache, use_cache=False)
            print(f"{name} {_class_of(G)} {res.setting} {res.seconds * 1e3:.4f} ms "
                  f"(start {res.baseline_seconds * 1e3:.4f} ms)", flush=True)
        del rp, ci, g
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
