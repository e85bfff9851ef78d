"""Continuous batching on the GPU: jobs queue under a small memory budget,
jobs arriving while others run are admitted mid-flight, and every job's
colouring equals the oracle's for its graph alone (tolerance 0)."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1509_08267_amd import gc, serve as srv
    gc.load()
    return srv


def graphs(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(np.exp(rng.uniform(np.log(50), np.log(20000))))
        m = int(min(n * (n - 1) // 2, n * rng.uniform(2, 20)))
        out.append(graphgen.er(n, m, seed * 1000 + k))
    out += [graphgen.path(501), graphgen.complete(150), graphgen.star(400, 0), graphgen.empty(3)]
    return out


def test_queueing_midflight_admission_and_parity(serve):
    gs = graphs(60, 1)
    biggest = max(serve.job_words(g.n, g.nnz) for g in gs)
    srv = serve.Server(budget_bytes=4 * 3 * biggest, max_slots=16, rounds_per_step=2)
    # half arrive at once, the rest while those are running
    arrivals = np.concatenate([np.zeros(32), 0.002 + np.sort(np.random.default_rng(2).uniform(0, 0.05, len(gs) - 32))])
    jobs = srv.serve(gs, arrivals)
    for g, j in zip(gs, jobs):
        ref = oracle.rsc(g.rowptr, g.colidx)
        assert j.rounds == ref.rounds
        assert np.array_equal(j.colors, ref.colors)
    # the budget forced queueing: some job waited for memory or a slot, and
    # the steps taken while jobs waited ran the backlog's round count
    assert any(j.admitted_step > 0 for j in jobs)
    assert 0 < srv.backlog_steps < srv.steps
    # continuous batching: some job was admitted at a step where another job,
    # admitted earlier, was still being coloured
    midflight = [j for j in jobs
                 if any(k.admitted_step < j.admitted_step < k.finished_step for k in jobs)]
    assert midflight
    s = serve.latency_summary(jobs)
    assert 0 < s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]
    assert srv.alloc.used == 0 and srv.idle()


def test_alone_equals_in_the_mix(serve):
    gs = graphs(20, 3)
    alone = []
    for g in gs:
        srv = serve.Server(budget_bytes=64 << 20, rounds_per_step=3)
        alone.append(srv.serve([g], [0.0])[0])
    srv = serve.Server(budget_bytes=64 << 20, max_slots=8, rounds_per_step=1)
    mixed = srv.serve(gs, np.linspace(0, 0.01, len(gs)))
    for a, b in zip(alone, mixed):
        assert a.rounds == b.rounds and np.array_equal(a.colors, b.colors)


def test_oversized_job_is_rejected(serve):
    from paper_1509_08267_amd import gc
    srv = serve.Server(budget_bytes=1 << 16)
    g = graphgen.er(20000, 100000, 1)
    with pytest.raises(gc.GCError) as ei:
        srv.submit(g.rowptr, g.colidx)
    assert ei.value.code == gc.GC_ETOOBIG


def test_copy_segments_exact(serve):
    # many int32 arrays copied by one gc_copy_segments launch: lengths around
    # the 4096-word piece, empty and large ones; the words between the
    # destinations stay untouched
    from paper_1509_08267_amd import gc
    rng = np.random.default_rng(5)
    lens = [0, 1, 63, 4095, 4096, 4097, 8192, 12289, 0, 200_001, 7, 3]
    dev = torch.device("cuda:0")
    srcs = [torch.from_numpy(rng.integers(-2**31, 2**31 - 1, size=n, dtype=np.int64)
                             .astype(np.int32)).to(dev) for n in lens]
    gap = 17
    total = sum(lens) + gap * (len(lens) + 1)
    out = torch.full((total,), -7, dtype=torch.int32, device=dev)
    pairs, pos, spans = [], gap, []
    for s in srcs:
        pairs.append((s, out[pos:pos + s.numel()]))
        spans.append((pos, s.numel()))
        pos += s.numel() + gap
    keep = gc.copy_segments(pairs)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    mask = np.ones(total, bool)
    for (p, n), s in zip(spans, srcs):
        assert np.array_equal(got[p:p + n], s.cpu().numpy()), n
        mask[p:p + n] = False
    assert (got[mask] == -7).all()
    del keep


def test_copy_segments_inconsistent_pieces_stay_in_bounds(serve):
    # a descriptor whose first_piece values do not match the lengths copies
    # less, never more: every write stays inside its destination
    from paper_1509_08267_amd import gc
    dev = torch.device("cuda:0")
    a = torch.arange(10000, dtype=torch.int32, device=dev)
    out = torch.full((30000,), -1, dtype=torch.int32, device=dev)
    # segment 0 claims one piece but has three; segment 1 starts at piece 1
    desc = np.array([[a.data_ptr(), out.data_ptr(), 10000, 0],
                     [a.data_ptr(), out[20000:].data_ptr(), 5000, 1]], dtype=np.int64)
    d = torch.from_numpy(desc).to(dev)
    gc.gc_copy_segments(2, d, 3)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got[:4096], np.arange(4096))      # piece 0 of segment 0
    assert (got[4096:20000] == -1).all()                    # its other pieces were not listed
    assert np.array_equal(got[20000:25000], np.arange(5000))  # segment 1, pieces 1..2
    assert (got[25000:] == -1).all()


class _DevReq:
    def __init__(self, rowptr, colidx):
        self.rowptr, self.colidx = rowptr, colidx


def _device_requests(gs, stream):
    # the request tensors are written by work queued on `stream` (a copy
    # from pageable memory and an in-place add), as a producer would
    reqs = []
    with torch.cuda.stream(stream):
        for g in gs:
            rp = torch.from_numpy(g.rowptr.astype(np.int32)).cuda(non_blocking=False)
            ci = torch.from_numpy(g.colidx.astype(np.int32) - 1).cuda()
            ci.add_(1)
            reqs.append(_DevReq(rp, ci))
    return reqs


@pytest.mark.parametrize("midflight", [False, True])
def test_device_staged_requests(serve, midflight):
    # requests whose CSR already lives on the GPU are admitted by one copy
    # launch per admission; the copy waits for the producer's stream
    gs = graphs(40, 7)
    producer = torch.cuda.current_stream()
    reqs = _device_requests(gs, producer)
    biggest = max(serve.job_words(g.n, g.nnz) for g in gs)
    srv = serve.Server(budget_bytes=4 * 4 * biggest, max_slots=12, rounds_per_step=2)
    arrivals = (np.sort(np.random.default_rng(8).uniform(0, 0.03, len(gs))) if midflight
                else np.zeros(len(gs)))
    jobs = srv.serve(reqs, arrivals)
    for g, j in zip(gs, jobs):
        ref = oracle.rsc(g.rowptr, g.colidx)
        assert j.rounds == ref.rounds
        assert np.array_equal(j.colors, ref.colors)
    assert srv.alloc.used == 0 and srv.idle()


@pytest.mark.parametrize("midflight", [False, True])
def test_packed_submission(serve, midflight):
    # a packed batch on the device (the layout of gc_color_batch), submitted
    # as a whole: every job equals the oracle, under a budget that queues
    gs = graphs(40, 11)
    voff = np.concatenate([[0], np.cumsum([g.n for g in gs])]).astype(np.int64)
    eoff = np.concatenate([[0], np.cumsum([g.nnz for g in gs])]).astype(np.int64)
    rpl = torch.from_numpy(np.concatenate([g.rowptr.astype(np.int32) for g in gs])).cuda()
    cil = torch.from_numpy(np.concatenate([g.colidx.astype(np.int32) for g in gs])).cuda()
    biggest = max(serve.job_words(g.n, g.nnz) for g in gs)
    srv = serve.Server(budget_bytes=4 * 4 * biggest, max_slots=12, rounds_per_step=3)
    arrivals = (np.sort(np.random.default_rng(9).uniform(0, 0.03, len(gs))) if midflight
                else np.zeros(len(gs)))
    jobs = srv.serve_packed(voff, eoff, rpl, cil, arrivals)
    for g, j in zip(gs, jobs):
        ref = oracle.rsc(g.rowptr, g.colidx)
        assert j.rounds == ref.rounds
        assert np.array_equal(j.colors, ref.colors)
    assert srv.alloc.used == 0 and srv.idle()
    with pytest.raises(ValueError):
        srv.submit_packed(voff, eoff, rpl.cpu(), cil, np.zeros(len(gs)))
    with pytest.raises(ValueError):
        srv.submit_packed(voff, eoff + 5, rpl, cil, np.zeros(len(gs)))


def test_step_loop_allocates_nothing(serve):
    # once built (and warmed by one stream), the server's loop takes no device
    # memory from the caching allocator and no pinned host memory: the table,
    # the workspace and every staging buffer were allocated by the constructor
    gs = graphs(60, 13)
    voff = np.concatenate([[0], np.cumsum([g.n for g in gs])]).astype(np.int64)
    eoff = np.concatenate([[0], np.cumsum([g.nnz for g in gs])]).astype(np.int64)
    rpl = torch.from_numpy(np.concatenate([g.rowptr.astype(np.int32) for g in gs])).cuda()
    cil = torch.from_numpy(np.concatenate([g.colidx.astype(np.int32) for g in gs])).cuda()
    srv = serve.Server(budget_bytes=64 << 20, max_slots=16, rounds_per_step=2, keep_colors=False)
    arrivals = np.sort(np.random.default_rng(5).uniform(0, 0.01, len(gs)))
    srv.serve_packed(voff, eoff, rpl, cil, arrivals)
    torch.cuda.synchronize()

    def counts():
        dev = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
        host = torch.cuda.host_memory_stats().get("allocation.allocated", 0) \
            if hasattr(torch.cuda, "host_memory_stats") else 0
        return dev, host

    before = counts()
    steps0 = srv.steps
    jobs = srv.serve_packed(voff, eoff, rpl, cil, arrivals)
    torch.cuda.synchronize()
    assert srv.steps > steps0 + 5
    assert counts() == before
    assert all(j.finished_at > 0 for j in jobs) and srv.idle()
    # (the device counter does see an allocation)
    x = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    assert counts()[0] > before[0]
    del x
