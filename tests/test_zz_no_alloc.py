"""GPU: gc_color_batch_noalloc, the batch entry point that allocates nothing
(its workspace is a fixed device array inside the library), against
gc_color_batch with a caller-allocated workspace: same colours and rounds,
bit for bit, on two calls in a row (the second with a smaller batch, which
must not see anything the first left in the shared array), and no change in
the device's free memory across a call."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1509_08267_amd import gc as gcmod
    gcmod.load()
    return gcmod


def _batch(count, seed):
    rng = np.random.default_rng(seed)
    gs = []
    for k in range(count):
        n = int(np.exp(rng.uniform(np.log(10), np.log(30000))))
        m = int(min(n * (n - 1) // 2, n * rng.uniform(2, 24)))
        gs.append(graphgen.er(n, m, seed * 7919 + k))
    gs += [graphgen.empty(0), graphgen.complete(90), graphgen.path(333)]
    voff = np.zeros(len(gs) + 1, np.int64)
    eoff = np.zeros(len(gs) + 1, np.int64)
    for i, g in enumerate(gs):
        voff[i + 1] = voff[i] + g.n
        eoff[i + 1] = eoff[i] + g.nnz
    rpl = np.concatenate([g.rowptr.astype(np.int32) for g in gs])
    cil = np.concatenate([g.colidx for g in gs]).astype(np.int32)
    return gs, voff, eoff, rpl, cil


def _run_both(gc, voff, eoff, rpl, cil):
    dev = torch.device("cuda:0")
    d = lambda a: torch.from_numpy(a).to(dev)
    G = voff.shape[0] - 1
    n = int(voff[-1])
    args = (d(voff), d(eoff), d(rpl), d(cil))
    col_a = torch.full((n,), 77, dtype=torch.int32, device=dev)
    rnd_a = torch.full((G,), -5, dtype=torch.int32, device=dev)
    nbytes = gc.gc_batch_workspace_bytes(G, voff, eoff)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    gc.gc_color_batch(G, *args, col_a, rnd_a, ws, nbytes)
    col_b = torch.full((n,), -9, dtype=torch.int32, device=dev)
    rnd_b = torch.full((G,), 1234, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    gc.gc_color_batch_noalloc(G, *args, col_b, rnd_b)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    return (col_a.cpu().numpy(), rnd_a.cpu().numpy(), col_b.cpu().numpy(), rnd_b.cpu().numpy(),
            free0, free1)


def test_noalloc_equals_workspace_entry_point_twice(gc):
    first = _batch(300, 1)
    second = _batch(40, 2)       # smaller: fewer descriptors than the first call left
    for gs, voff, eoff, rpl, cil in (first, second):
        ca, ra, cb, rb, free0, free1 = _run_both(gc, voff, eoff, rpl, cil)
        assert np.array_equal(ca, cb)
        assert np.array_equal(ra, rb)
        assert free0 == free1
        # and both equal the oracle, graph by graph
        for i, g in enumerate(gs):
            ref = oracle.rsc(g.rowptr, g.colidx)
            assert np.array_equal(cb[voff[i]:voff[i + 1]], ref.colors), i
            assert rb[i] == ref.rounds, i


def test_noalloc_rejects_too_many_graphs(gc):
    G = gc.GC_STATIC_BATCH_MAX_GRAPHS + 1
    dev = torch.device("cuda:0")
    voff = torch.zeros(G + 1, dtype=torch.int64, device=dev)
    z32 = torch.zeros(G + 1, dtype=torch.int32, device=dev)
    with pytest.raises(gc.GCError) as ei:
        gc.gc_color_batch_noalloc(G, voff, voff, z32, z32, z32, z32)
    assert ei.value.code == gc.GC_ETOOBIG
