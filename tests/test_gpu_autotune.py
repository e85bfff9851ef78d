"""GPU: the autotuner times real colourings, keeps every colouring bit-exact
with the oracle, writes its cache and reuses it."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1509_08267_amd import autotune, gc
    gc.load()
    return gc, autotune


@pytest.mark.parametrize("name,g,rp64", [
    ("er", graphgen.er(20000, 200000, 7), False),
    ("rmat14", graphgen.rmat(14, 16, seed=3), True),
])
def test_tune_keeps_colours_and_caches(mods, tmp_path, name, g, rp64):
    gc, autotune = mods
    ref = oracle.rsc(g.rowptr, g.colidx)
    rp = torch.from_numpy(g.rowptr.astype(np.int64 if rp64 else np.int32)).cuda()
    ci = torch.from_numpy(g.colidx).cuda()
    cache = autotune.Cache(str(tmp_path / "tune.json"), shipped=None)
    with gc.Graph(rp, ci) as G:
        res = autotune.tune(G, reps=2, budget_s=15.0, cache=cache)
        assert not res.cached
        assert set(res.setting) == set(autotune.KNOBS)
        assert len(res.table) >= 2 and res.seconds <= res.baseline_seconds
        print(f"[autotune] {name}: {res.setting} {res.seconds * 1e3:.3f} ms "
              f"(start {res.baseline_seconds * 1e3:.3f} ms)", flush=True)
        out = G.color()
        r, k = G.stats()
        assert np.array_equal(out.cpu().numpy(), ref.colors)
        assert r == ref.rounds
        cls = autotune._class_of(G)
    assert autotune.Cache(cache.path, shipped=None).get(autotune.device_key(), cls) is not None
    # a second graph of the same class takes the cached setting without timing
    with gc.Graph(rp, ci) as G2:
        res2 = autotune.tune(G2, cache=autotune.Cache(cache.path, shipped=None))
        assert res2.cached and res2.setting == res.setting
        out = G2.color()
        G2.stats()
        assert np.array_equal(out.cpu().numpy(), ref.colors)
