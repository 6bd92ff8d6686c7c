"""GPU parity of the method variants against the CPU oracle: two colours
(octant parity), the all-octant R_max and the optimistic bound R'_max, on the
per-cycle engine (every variant, both layouts) and on the persistent engines
(two colours and the bound on the re-binning kernel and in batches, the
all-octant maximum on the incremental one).  Bar: spins, fired/null counts, M and B bit-exact; clock within 1e-12
relative."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
T_REL = 1e-12

RMAX_ALL, TWO, BOUND = 1, 2, 4


@pytest.fixture(scope="module")
def spkmc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1005_4713_amd import spkmc as mod
    return mod


def _same(g, o):
    assert g[0] == o[0] and g[1] == o[1] and g[2] == o[2], (g, o)
    assert g[4] == o[4] and g[5] == o[5], (g, o)
    assert abs(g[3] - o[3]) <= T_REL * abs(o[3]), (g, o)


def _oracle(L, d, variant, **kw):
    scope = 1 if variant & RMAX_ALL else 2 if variant & BOUND else 0
    colours = 2 if variant & TWO else 8
    kw = dict(kw)
    kw["rates"] = {"glauber": 0, "metropolis": 1}[kw.get("rates", "glauber")]
    kw["init"] = {"random": 0, "up": 1, "down": 2}[kw.get("init", "random")]
    return oracle.Sim(L=L, d=d, colours=colours, rmax_scope=scope, **kw)


def _compare(spkmc, L, d, layout, engine, variant, launches=(23, 40, 57), obs=5, **kw):
    kw.setdefault("T", 4.5115)
    gpu = spkmc.Sim(L, d, layout=layout, engine=engine, variant=variant, seed=19, record_cap=512, **kw)
    orc = _oracle(L, d, variant, seed=19, **kw)
    _same(gpu.state(), orc.state())
    for n in launches:
        gpu.run(n, obs_every=obs)
        ro = orc.run(n, obs_every=obs)
        rg = gpu.records(len(ro)) if ro else []
        assert len(rg) == len(ro)
        for g_, o_ in zip(rg, ro):
            _same(g_, o_)
        _same(gpu.state(), orc.state())
        assert np.array_equal(gpu.spins(), orc.spins())
    assert orc.check_failures() == 0
    return gpu


@pytest.mark.parametrize("variant", [RMAX_ALL, TWO, BOUND, TWO | RMAX_ALL, TWO | BOUND])
@pytest.mark.parametrize("L,d,layout,kw", [
    (16, 8, "int8", dict(H=0.05)),
    (16, 4, "int8", dict(rates="metropolis")),
    (32, 16, "packed", dict(init="up", T=4.4)),
    (64, 32, "packed", dict(H=-0.05)),
    (24, 8, "packed", dict()),                    # h = 4: several domains share a word
])
def test_cycle_engine_variants(spkmc, variant, L, d, layout, kw):
    print("case cycle", variant, L, d, layout, kw, flush=True)
    g = _compare(spkmc, L, d, layout, "cycle", variant, **kw)
    assert g.info()["engine"] == spkmc.ENGINES["cycle"]


@pytest.mark.parametrize("L,d,kw", [
    (64, 32, dict()),
    (128, 32, dict(H=0.05, rates="metropolis")),
    (64, 16, dict(init="up")),
    (128, 16, dict(T=4.6)),
])
def test_persistent_bound(spkmc, L, d, kw):
    """The fixed bound on the re-binning persistent kernel: no R_max exchange,
    neighbour-local waits, records appended by workgroup 0 as they complete."""
    print("case persistent bound", L, d, kw, flush=True)
    g = _compare(spkmc, L, d, "packed", "persistent", BOUND, **kw)
    assert g.info()["engine"] == spkmc.ENGINES["persistent"]


def test_persistent_bound_every_cycle_records(spkmc):
    """A record every cycle: the record banks are reused every four cycles."""
    print("case persistent bound obs 1", flush=True)
    _compare(spkmc, 128, 16, "packed", "persistent", BOUND, launches=(150,), obs=1)


@pytest.mark.parametrize("L,d,kw", [
    (64, 32, dict()),
    (128, 32, dict(H=0.05)),
    (128, 16, dict(rates="metropolis", init="down")),
])
def test_incremental_all_octants(spkmc, L, d, kw):
    """The all-octant maximum from the resident histograms of every octant."""
    print("case incremental rmax_all", L, d, kw, flush=True)
    g = _compare(spkmc, L, d, "packed", "incremental", RMAX_ALL, **kw)
    assert g.info()["engine"] == spkmc.ENGINES["incremental"]


@pytest.mark.parametrize("variant", [TWO, TWO | BOUND])
@pytest.mark.parametrize("L,d,kw", [
    (64, 32, dict()),
    (128, 32, dict(H=0.05)),
    (64, 16, dict(init="up", rates="metropolis")),
    (128, 16, dict(T=4.6)),
])
def test_persistent_two_colours(spkmc, variant, L, d, kw):
    """Two colours on the re-binning persistent kernel: four frequency lines per
    domain, a wait on every neighbour after each colour change."""
    print("case persistent two colours", variant, L, d, kw, flush=True)
    g = _compare(spkmc, L, d, "packed", "persistent", variant, **kw)
    assert g.info()["engine"] == spkmc.ENGINES["persistent"]


def test_auto_engine_choice(spkmc):
    pick = lambda v: spkmc.Sim(64, 16, variant=v, seed=1).info()["engine"]  # noqa: E731
    assert spkmc.Sim(64, 32, variant=RMAX_ALL, seed=1).info()["engine"] == spkmc.ENGINES["slab"]
    assert spkmc.Sim(64, 32, seed=1).info()["engine"] == spkmc.ENGINES["persistent"]
    assert pick(0) == spkmc.ENGINES["persistent"]
    assert pick(BOUND) == spkmc.ENGINES["persistent"]
    assert pick(RMAX_ALL) == spkmc.ENGINES["incremental"]
    assert pick(TWO) == spkmc.ENGINES["persistent"]
    assert pick(TWO | BOUND) == spkmc.ENGINES["persistent"]
    assert pick(TWO | RMAX_ALL) == spkmc.ENGINES["cycle"]
    with pytest.raises(spkmc.SpkmcError):
        spkmc.Sim(64, 16, variant=TWO, engine="incremental", seed=1)
    with pytest.raises(spkmc.SpkmcError):
        spkmc.Sim(64, 16, variant=BOUND, engine="incremental", seed=1)


def test_variants_in_one_batch(spkmc):
    """Batches run the re-binning kernel, so lattices of different variants
    (contract, bound, two colours, both) share one launch, each bit-identical
    to its solo run."""
    specs = [(64, 16, 0.0, 3, 0), (32, 16, 0.05, 4, BOUND), (128, 16, -0.05, 5, TWO), (64, 16, 0.0, 6, TWO | BOUND)]
    solo, batch = [], []
    for L, d, H, seed, v in specs:
        a = spkmc.Sim(L, d, H=H, seed=seed, variant=v, record_cap=64)
        a.run(60, obs_every=6)
        solo.append((a.state(), a.records(), a.spins().tobytes()))
        batch.append(spkmc.Sim(L, d, H=H, seed=seed, variant=v, record_cap=64))
    spkmc.run_batch(batch, 60, obs_every=6)
    for s_, b in zip(solo, batch):
        assert (b.state(), b.records(), b.spins().tobytes()) == s_


def test_eight_colour_batch_with_a_bound_member(spkmc):
    """Eight-colour lattices alone run a batch kernel with one line per domain
    and the fixed bound's code compiled out; one member with the bound moves the
    whole batch to the kernel that reads both at run time.  Either way every
    member ends bit-identical to its solo run."""
    for specs in ([(64, 16, 0.0, 7, 0), (48, 16, 0.05, 8, 0), (32, 16, -0.05, 9, 0)],
                  [(64, 16, 0.0, 7, 0), (48, 16, 0.05, 8, BOUND), (32, 16, -0.05, 9, 0)]):
        print("case eight-colour batch", [s[4] for s in specs], flush=True)
        solo, batch = [], []
        for L, d, H, seed, v in specs:
            a = spkmc.Sim(L, d, H=H, seed=seed, variant=v, record_cap=64)
            a.run(50, obs_every=5)
            solo.append((a.state(), a.records(), a.spins().tobytes()))
            batch.append(spkmc.Sim(L, d, H=H, seed=seed, variant=v, record_cap=64))
        spkmc.run_batch(batch, 50, obs_every=5)
        for s_, b in zip(solo, batch):
            assert (b.state(), b.records(), b.spins().tobytes()) == s_
