"""Write ``workloads.json``: the oracle's answers on the full-size workloads.

Every value in the output comes from ``graphgen`` (the inputs) and ``oracle``
(the answers) only.  Run from the repository root:

    python tests/golden/make_golden.py [workload ...]
    python tests/golden/make_golden.py --seq-only [workload ...]
    python tests/golden/make_golden.py --blocks-only [workload ...]
    python tests/golden/make_golden.py --orders-only [workload ...]

Per workload it records the input's SHA-256 and shape, the oracle's round
count, colour count and the SHA-256 of its colour vector, the per-round
totals used for algorithmic byte counts (sum over rounds of |U_r|, of the
degrees of U_r and of the lower-neighbour counts of U_r), the sequential
First-Fit colour count, and the oracle's single-thread time.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workloads.json")


def colors_sha(c: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(c, dtype=np.int32).tobytes()).hexdigest()


def skip_fields(g, r):
    """Lower bounds on the row entries a scan must read when rows are sorted.

    With ascending rows the lower neighbours of v form a prefix of its row.
    A lower neighbour whose colour was final before round r cannot conflict
    with v in round r, so a scan that remembers how far the leading run of
    such neighbours reaches reads, in round r >= 2, only the entries from the
    first lower neighbour still uncoloured at the start of round r up to the
    first conflict; and once v's colour is final in round r, only the
    entries from the first lower neighbour still uncoloured after round r
    can need a push.  Both counts come from the oracle's round_of alone:
    with M_p the largest round_of over the first p+1 lower neighbours,

      sum_active_scan_skip = sum over rounds >= 2 of the early-stop scan
          count, minus sum over v, p of max(0, round_of[v] - max(M_p, 1));
      push_rows_skip_after_round1 = sum over v final in round >= 2 of
          deg(v) - #{p : M_p <= round_of[v]}.
    """
    n, nnz = g.n, g.nnz
    if n == 0 or nnz == 0:
        return {"rows_sorted": True, "sum_active_scan_skip": 0, "push_rows_skip_after_round1": 0}
    deg = np.diff(g.rowptr).astype(np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    dst = g.colidx.astype(np.int64)
    same_row = src[1:] == src[:-1]
    rows_sorted = bool(np.all(dst[1:][same_row] > dst[:-1][same_row]))
    ro = r.round_of.astype(np.int64)
    R = int(r.rounds)
    lower = dst < src
    ls, lu = src[lower], dst[lower]
    # segmented running maximum of round_of over each row's lower prefix
    key = ls * (R + 1) + ro[lu]
    M = np.maximum.accumulate(key) - ls * (R + 1)
    skipped = np.maximum(0, ro[ls] - np.maximum(M, 1)).sum()
    scan = int(r.trace[1:, 3].sum()) - int(skipped)
    head = np.bincount(ls[M <= ro[ls]], minlength=n)
    late = ro >= 2
    push = int((deg[late] - head[late]).sum())
    return {"rows_sorted": rows_sorted, "sum_active_scan_skip": scan,
            "push_rows_skip_after_round1": push}


def one(name):
    inp = graphgen.workload(name)
    rec = {"description": graphgen.WORKLOADS[name]}
    if isinstance(inp, graphgen.Batch):
        rec.update(input_sha256=inp.sha256(), num_graphs=inp.num_graphs,
                   n=int(inp.voff[-1]), nnz=int(inp.eoff[-1]))
        t = time.perf_counter()
        colors, rounds = oracle.rsc_batch(inp.voff, inp.eoff, inp.rowptr_local, inp.colidx_local)
        rec["oracle_seconds"] = time.perf_counter() - t
        # per-round totals over all graphs (for algorithmic byte counts)
        sa = sd = sl = ss = 0
        for g in range(inp.num_graphs):
            sub = inp.graph(g)
            r = oracle.rsc(sub.rowptr, sub.colidx)
            assert np.array_equal(r.colors, colors[inp.voff[g]:inp.voff[g + 1]])
            sa += int(r.trace[:, 0].sum())
            sd += int(r.trace[:, 1].sum())
            sl += int(r.trace[:, 2].sum())
            ss += int(r.trace[:, 3].sum())
        rec["sum_active"] = sa
        rec["sum_active_deg"] = sd
        rec["sum_active_lower_deg"] = sl
        rec["sum_active_scan"] = ss
        rec["colors_sha256"] = colors_sha(colors)
        rec["rounds_sha256"] = hashlib.sha256(rounds.astype(np.int64).tobytes()).hexdigest()
        rec["rounds_max"] = int(rounds.max())
        rec["rounds_sum"] = int(rounds.sum())
        ncol = np.zeros(inp.num_graphs, np.int64)
        for g in range(inp.num_graphs):
            a, b = int(inp.voff[g]), int(inp.voff[g + 1])
            ncol[g] = int(colors[a:b].max()) + 1 if b > a else 0
        rec["num_colors_sum"] = int(ncol.sum())
        rec["num_colors_max"] = int(ncol.max())
        return rec
    g = inp
    rec.update(input_sha256=g.sha256(), n=g.n, nnz=g.nnz, max_degree=g.max_degree())
    t = time.perf_counter()
    r = oracle.rsc(g.rowptr, g.colidx)
    rec["oracle_seconds"] = time.perf_counter() - t
    rec["rounds"] = r.rounds
    rec["num_colors"] = r.num_colors
    rec["colors_sha256"] = colors_sha(r.colors)
    rec["round_sizes"] = [int(x) for x in r.trace[:, 0]]
    rec["sum_active"] = int(r.trace[:, 0].sum())
    rec["sum_active_deg"] = int(r.trace[:, 1].sum())
    rec["sum_active_lower_deg"] = int(r.trace[:, 2].sum())
    rec["sum_active_scan"] = int(r.trace[:, 3].sum())
    # CSR entries (v, u) whose u is still uncoloured after v's colour is
    # final: the pushes a push-based colouring has to store
    deg = np.diff(g.rowptr)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    ro = r.round_of.astype(np.int64)
    useful = ro[g.colidx.astype(np.int64)] > ro[src]
    rec["push_useful"] = int(useful.sum())
    # the same restricted to vertices whose colour became final after round 1
    # (round 1 runs in its own kernel)
    late = ro[src] >= 2
    rec["push_rows_after_round1"] = int(late.sum())
    rec["push_useful_after_round1"] = int((useful & late).sum())
    rec.update(skip_fields(g, r))
    assert oracle.check_proper(g.rowptr, g.colidx, r.colors) == 0
    assert oracle.check_grundy(g.rowptr, g.colidx, r.colors) == 0
    rec.update(seq_fields(g))
    return rec


BLOCKS_P = 16384  # blocks of the recorded p-block colourings (64 per CU on 256 CUs)


def order_fields(g):
    """The speculative colouring in the largest-first and seed-0 random
    vertex orders (relabel, colour, map back)."""
    from oracle import ordering
    rec = {}
    for kind in ("largest_first", "random"):
        col, (_, res) = ordering.colour_in_order(
            g.rowptr, g.colidx, kind, 0, lambda rp, ci: (lambda r: (r.colors, r))(oracle.rsc(rp, ci)))
        rec[f"order_{kind}_colors_sha256"] = colors_sha(col)
        rec[f"order_{kind}_rounds"] = res.rounds
        rec[f"order_{kind}_num_colors"] = res.num_colors
        rec[f"order_{kind}_sum_active"] = int(res.trace[:, 0].sum())
    return rec


def blocks_fields(g):
    """Algorithm 1 read literally with BLOCKS_P blocks."""
    t = time.perf_counter()
    col, R, rec = oracle.blocks(g.rowptr, g.colidx, BLOCKS_P)
    return {"blocks_p": BLOCKS_P, "blocks_seconds": time.perf_counter() - t,
            "blocks_colors_sha256": colors_sha(col), "blocks_rounds": R,
            "blocks_num_colors": int(col.max()) + 1 if col.size else 0,
            "blocks_sum_active": int((rec.astype(np.int64) + 1).sum()),
            # a vertex is pending in rounds 1 .. recolours + 1: the rows those
            # rounds read
            "blocks_sum_active_deg": int(((rec.astype(np.int64) + 1)
                                          * np.diff(g.rowptr).astype(np.int64)).sum())}


def seq_fields(g):
    """Sequential First Fit (the Section 5 baseline) and the rounds of the
    id-priority schedule that reproduces it."""
    t = time.perf_counter()
    s = oracle.seq(g.rowptr, g.colidx)
    rec = {"seq_seconds": time.perf_counter() - t,
           "seq_num_colors": int(s.max()) + 1 if s.size else 0,
           "seq_colors_sha256": colors_sha(s)}
    R, ro = oracle.seq_rounds(g.rowptr, g.colidx)
    ro = ro.astype(np.int64)
    deg = np.diff(g.rowptr).astype(np.int64)
    rec["seq_rounds"] = R
    # a vertex is uncoloured in rounds 1 .. round_of(v): sum of |U_r|
    rec["seq_sum_active"] = int(ro.sum())
    # the same counts restricted to rounds >= 2 (round 1 has its own launch):
    # visits, visits of vertices still waiting, and the rows of the vertices
    # coloured then (each read once for the least absent colour)
    rec["seq_visits_after_round1"] = int(np.maximum(ro - 1, 0).sum())
    rec["seq_waiting_visits_after_round1"] = int(np.maximum(ro - 2, 0).sum())
    rec["seq_rows_after_round1"] = int(deg[ro >= 2].sum())
    rec["seq_coloured_after_round1"] = int((ro >= 2).sum())
    return rec


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    if names and names[0] == "--orders-only":
        for name in names[1:] or ["er_10k_100k", "er_1m_16m"]:
            g = graphgen.workload(name)
            assert g.sha256() == data[name]["input_sha256"]
            data[name].update(order_fields(g))
            print(f"[golden] {name}: orders", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        return
    if names and names[0] == "--blocks-only":
        # (re)compute only the p-block fields of recorded workloads
        for name in names[1:] or ["er_10k_100k", "er_1m_16m"]:
            g = graphgen.workload(name)
            assert g.sha256() == data[name]["input_sha256"]
            data[name].update(blocks_fields(g))
            print(f"[golden] {name}: blocks rounds {data[name]['blocks_rounds']}", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        return
    if names and names[0] == "--seq-only":
        # refresh only the sequential-baseline fields of recorded workloads
        for name in names[1:] or [k for k in data if k != "er_batch_4096"]:
            g = graphgen.workload(name)
            assert g.sha256() == data[name]["input_sha256"]
            data[name].update(seq_fields(g))
            print(f"[golden] {name}: seq rounds {data[name]['seq_rounds']}", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        return
    for name in names:
        print(f"[golden] {name} ...", flush=True)
        data[name] = one(name)
        print(f"[golden] {name}: {json.dumps(data[name])[:300]}", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(graphgen.WORKLOADS))
