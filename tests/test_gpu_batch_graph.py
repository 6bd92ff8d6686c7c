"""A batch macro-step captured once into a HIP graph and replayed: every replay
continues every lattice, bit-identical to the same lattice run alone, with the
program's own eager work and synchronisations between the replays."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spkmc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1005_4713_amd import spkmc as mod
    return mod


def _mix(d, Ls, seed0):
    rng = np.random.default_rng(seed0)
    return [dict(L=L, domain=d, T=float(rng.uniform(4.0, 5.0)), H=float(rng.choice([0.0, 0.05, -0.05])),
                 seed=seed0 * 100 + i, init=["random", "up", "down"][i % 3], rates=["glauber", "metropolis"][i % 2])
            for i, L in enumerate(Ls)]


def _sims(spkmc, mix):
    return [spkmc.Sim(m["L"], m["domain"], T=m["T"], H=m["H"], seed=m["seed"], init=m["init"], rates=m["rates"],
                      layout="packed", engine="persistent", record_cap=256) for m in mix]


def _same(a, b):
    assert a.state() == b.state()
    assert a.records() == b.records()
    assert np.array_equal(a.spins(), b.spins())


@pytest.mark.parametrize("d,Ls", [(16, [32, 48, 64, 96, 32]), (32, [64, 128, 64])])
def test_graph_replays_equal_solo(spkmc, d, Ls):
    import torch
    print("case graph", d, Ls, flush=True)
    mix = _mix(d, Ls, 3 + d)
    batch, solo = _sims(spkmc, mix), _sims(spkmc, mix)
    ncyc = [20 + 7 * i for i in range(len(mix))]
    g = spkmc.BatchGraph(batch, ncyc, obs_every=5)
    assert g.info["lattices"] == len(mix)
    x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
    for rep in range(3):
        g.launch(1)
        # the program's own eager work between replays, then a full synchronisation
        x = (x * 1.0001 + 1.0).sqrt_()
        torch.cuda.synchronize()
        for s, n in zip(solo, ncyc):
            s.run(n, obs_every=5)
        for b, s in zip(batch, solo):
            _same(b, s)
    # several replays in one call
    g.launch(4)
    for s, n in zip(solo, ncyc):
        s.run(4 * n, obs_every=5)
    for b, s in zip(batch, solo):
        _same(b, s)
    g.close()
    # after the graph: the lattices go on with eager batches and solo runs alike
    spkmc.run_batch(batch, 30, obs_every=5)
    for s in solo:
        s.run(30, obs_every=5)
    for b, s in zip(batch, solo):
        _same(b, s)


def test_graph_rejects_outside_progress(spkmc):
    mix = _mix(16, [32, 48], 5)
    batch = _sims(spkmc, mix)
    g = spkmc.BatchGraph(batch, [10, 10])
    g.launch(1)
    batch[0].run(3)  # advanced outside the graph
    with pytest.raises(spkmc.SpkmcError):
        g.launch(1)
    g.close()
    with pytest.raises(spkmc.SpkmcError):
        spkmc.BatchGraph(batch, [0, 0])  # nothing to capture
