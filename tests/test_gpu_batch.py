"""GPU parity of the batched path (gc_color_batch, gc_batch_step): every
graph of a batch is coloured bit for bit as the oracle colours it alone
(colours and round count), whatever the batch around it, its position in
the batch, the state placement (LDS int8 / int16 / int32, or global), or how
the rounds are split into resumable steps."""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from conftest import ROOT

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1509_08267_amd import gc as gcmod
    gcmod.load()
    return gcmod


def pack(graphs):
    voff, eoff, rps, cis = [0], [0], [], []
    for g in graphs:
        voff.append(voff[-1] + g.n)
        eoff.append(eoff[-1] + g.nnz)
        rps.append(g.rowptr.astype(np.int32))
        cis.append(g.colidx.astype(np.int32))
    return graphgen.Batch(np.array(voff, np.int64), np.array(eoff, np.int64),
                          np.concatenate(rps) if rps else np.zeros(0, np.int32),
                          np.concatenate(cis) if cis else np.zeros(0, np.int32))


def dev(b):
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()
    return (t(b.voff, np.int64), t(b.eoff, np.int64), t(b.rowptr_local, np.int32),
            t(b.colidx_local if b.colidx_local.size else np.zeros(1, np.int32), np.int32))


def run_batch(gc, b):
    colors, rounds = gc.color_batch(*dev(b), voff_host=b.voff, eoff_host=b.eoff)
    torch.cuda.synchronize()
    return colors.cpu().numpy(), rounds.cpu().numpy()


def check_against_oracle(b, colors, rounds):
    for i in range(b.num_graphs):
        g = b.graph(i)
        ref = oracle.rsc(g.rowptr, g.colidx)
        got = colors[b.voff[i]:b.voff[i + 1]]
        assert rounds[i] == ref.rounds, (i, g.n, rounds[i], ref.rounds)
        assert np.array_equal(got, ref.colors), (i, g.n)


def mixed_graphs():
    rng = np.random.default_rng(3)
    gs = [graphgen.complete(1), graphgen.CSR(np.zeros(1, np.int64), np.zeros(0, np.int32)),
          graphgen.path(50), graphgen.cycle(5), graphgen.cycle(9),
          graphgen.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 5), (4, 5)]),
          graphgen.star(300, 0), graphgen.star(300, 300), graphgen.complete(130),
          graphgen.crown(8), graphgen.empty(17), graphgen.path(3001)]
    for k in range(40):
        n = int(rng.integers(2, 3000))
        m = int(min(n * (n - 1) // 2, rng.integers(1, 20) * n))
        gs.append(graphgen.er(n, m, 1000 + k))
    return gs


def test_mixed_batch_matches_oracle(gc):
    b = pack(mixed_graphs())
    colors, rounds = run_batch(gc, b)
    check_against_oracle(b, colors, rounds)


def test_state_placements(gc):
    # int8 in LDS, int16 in LDS (max degree > 127), int32 in LDS (> 32767),
    # and global int32 state (n beyond the LDS slice)
    gs = [graphgen.er(20000, 200000, 1),          # int8, LDS
          graphgen.star(1000, 5),                 # int16, LDS
          graphgen.star(40000, 3),                # int32 (degree 40000), global (4n > 64 KB)
          graphgen.er(100000, 500000, 2),         # int8 but n > 64K: global
          graphgen.star(14000, 9)]                # int16, LDS (2n <= 64 KB)
    b = pack(gs)
    colors, rounds = run_batch(gc, b)
    check_against_oracle(b, colors, rounds)


def test_batch_equals_alone_and_any_order(gc):
    gs = mixed_graphs()[:30]
    b = pack(gs)
    colors, rounds = run_batch(gc, b)
    perm = np.random.default_rng(8).permutation(len(gs))
    bp = pack([gs[i] for i in perm])
    cp, rp_ = run_batch(gc, bp)
    for j, i in enumerate(perm):
        assert rp_[j] == rounds[i]
        assert np.array_equal(cp[bp.voff[j]:bp.voff[j + 1]], colors[b.voff[i]:b.voff[i + 1]])
    # alone, through the per-graph path
    for i in (2, 6, 8, 20):
        g = gs[i]
        rp = torch.from_numpy(g.rowptr.astype(np.int32)).cuda()
        ci = torch.from_numpy(g.colidx).cuda()
        with gc.Graph(rp, ci) as G:
            out = G.color()
            assert G.stats()[0] == rounds[i]
        assert np.array_equal(out.cpu().numpy(), colors[b.voff[i]:b.voff[i + 1]])


@pytest.mark.parametrize("step_rounds", [1, 2, 3, 7])
def test_resumable_steps(gc, step_rounds):
    gs = mixed_graphs()
    b = pack(gs)
    ref_colors, ref_rounds = run_batch(gc, b)
    voff, eoff, rpl, cil = dev(b)
    colors = torch.full((int(b.voff[-1]),), 777, dtype=torch.int32, device="cuda")
    rows = [(int(b.voff[i] + i), int(b.eoff[i]), int(b.voff[i]), gs[i].n, 0)
            for i in range(len(gs))]
    descs = torch.from_numpy(gc.desc_array(rows).view(np.uint8)).cuda()
    steps = 0
    while True:
        gc.batch_step(descs, rpl, cil, colors, step_rounds)
        torch.cuda.synchronize()
        d = descs.cpu().numpy().view(gc.DESC_DTYPE)
        steps += 1
        if not d["active"].any():
            break
        assert steps < 10000
    assert np.array_equal(d["rounds"], ref_rounds)
    assert np.array_equal(colors.cpu().numpy(), ref_colors)
    assert steps >= int(np.ceil(ref_rounds.max() / step_rounds))


def team_graphs():
    """A batch in which the large graphs are coloured by teams of
    workgroups: each has at least a workgroup's fair share of the batch's
    work and 2 x 65,536 units of it (the team size is
    min(2 work / fair share, work / 65,536, grid))."""
    gs = [graphgen.er(60000, 600000, 11), graphgen.er(150000, 900000, 12),
          graphgen.star(200000, 77)]
    gs += mixed_graphs()[:20]
    return gs


def team_size(gs, i, grid):
    work = [int(g.nnz) + g.n + 1 for g in gs]
    fair = sum(work) // grid + 1
    return min(2 * work[i] // fair, grid, work[i] // 65536)


def test_teams_of_workgroups_match_oracle(gc):
    gs = team_graphs()
    grid = 2 * torch.cuda.get_device_properties(0).multi_processor_count
    assert all(team_size(gs, i, grid) >= 2 for i in range(3))
    assert all(team_size(gs, i, grid) < 2 for i in range(3, len(gs)))
    b = pack(gs)
    colors, rounds = run_batch(gc, b)
    check_against_oracle(b, colors, rounds)
    # one graph alone takes every workgroup it can use; a second launch on
    # the same buffers gives the same bits
    b1 = pack([gs[1]])
    c1, r1 = run_batch(gc, b1)
    assert r1[0] == rounds[1] and np.array_equal(c1, colors[b.voff[1]:b.voff[2]])


def test_team_colouring_is_fast(gc):
    """400,000 vertices and 6 M edges alone in a batch: one workgroup needs
    tens of milliseconds, a team of ~190 about a millisecond."""
    import time
    gcmod = gc
    g = graphgen.er(400000, 6000000, 13)
    b = pack([g])
    args = dev(b)
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        colors, rounds = gcmod.color_batch(*args, voff_host=b.voff, eoff_host=b.eoff)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    ref = oracle.rsc(g.rowptr, g.colidx)
    assert rounds.cpu().numpy()[0] == ref.rounds
    assert np.array_equal(colors.cpu().numpy(), ref.colors)
    print(f"one 400k-vertex graph in a batch: {dt * 1e3:.2f} ms")
    assert dt < 0.030


@pytest.mark.parametrize("step_rounds", [1, 3])
def test_resumable_steps_with_teams(gc, step_rounds):
    gs = team_graphs()
    b = pack(gs)
    ref_colors, ref_rounds = run_batch(gc, b)
    voff, eoff, rpl, cil = dev(b)
    colors = torch.full((int(b.voff[-1]),), 777, dtype=torch.int32, device="cuda")
    rows = [(int(b.voff[i] + i), int(b.eoff[i]), int(b.voff[i]), gs[i].n, 0)
            for i in range(len(gs))]
    descs = torch.from_numpy(gc.desc_array(rows).view(np.uint8)).cuda()
    steps = 0
    while True:
        gc.batch_step(descs, rpl, cil, colors, step_rounds)
        torch.cuda.synchronize()
        d = descs.cpu().numpy().view(gc.DESC_DTYPE)
        steps += 1
        if not d["active"].any():
            break
        assert steps < 10000
    assert np.array_equal(d["rounds"], ref_rounds)
    assert np.array_equal(colors.cpu().numpy(), ref_colors)
    maxdeg = [int(np.diff(g.rowptr).max()) if g.n and g.nnz else 0 for g in gs]
    assert np.array_equal(d["max_degree"], maxdeg)


def test_empty_batch_and_bad_workspace(gc):
    b = pack([])
    colors, rounds = gc.color_batch(*dev(pack([graphgen.path(3)])), voff_host=np.array([0, 3]),
                                    eoff_host=np.array([0, 4]))
    torch.cuda.synchronize()
    assert colors.cpu().tolist() == [0, 1, 0]
    voff, eoff, rpl, cil = dev(pack([graphgen.path(3)]))
    with pytest.raises(gc.GCError) as ei:
        gc.gc_color_batch(1, voff, eoff, rpl, cil, torch.zeros(3, dtype=torch.int32, device="cuda"),
                          None, torch.zeros(8, dtype=torch.uint8, device="cuda"), 8)
    assert ei.value.code == gc.GC_EINVAL and "workspace" in str(ei.value)
    assert b.num_graphs == 0


@pytest.mark.slow
def test_workload_er_batch_4096(gc):
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "workloads.json")))["er_batch_4096"]
    b = graphgen.workload("er_batch_4096")
    assert b.sha256() == golden["input_sha256"]
    colors, rounds = run_batch(gc, b)
    assert hashlib.sha256(colors.astype(np.int32).tobytes()).hexdigest() == golden["colors_sha256"]
    assert hashlib.sha256(rounds.astype(np.int64).tobytes()).hexdigest() == golden["rounds_sha256"]
