"""GPU parity of the slab engine (class counts of every octant, per slab of
four z-planes, kept in device memory and moved by every flip; only the slab
holding the selected site is classified): against the CPU oracle, and against
the re-binning persistent engine at sizes the oracle would take minutes for.
Bar: spins, fired/null counts, M and B bit-exact; clock within 1e-12 relative.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
T_REL = 1e-12


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


def _orc(L, d, **kw):
    kw = dict(kw)
    kw["rates"] = {"glauber": 0, "metropolis": 1}[kw.get("rates", "glauber")]
    kw["init"] = {"random": 0, "up": 1, "down": 2}[kw.get("init", "random")]
    return oracle.Sim(L=L, d=d, **kw)


@pytest.mark.parametrize("L,kw", [
    (32, dict()),                                  # one domain: every neighbour domain is itself
    (64, dict(H=0.05)),                            # two domains per edge
    (96, dict(rates="metropolis")),                # 27 domains, one partly filled workgroup
    (128, dict(init="up", T=4.4)),                 # 64 domains
    (160, dict(H=-0.05, rates="metropolis")),      # 125 domains: three idle rows
    (256, dict(init="down", T=4.6)),               # 512 domains, four workgroups
])
def test_slab_vs_oracle(spkmc, L, kw):
    print("case slab", L, kw, flush=True)
    kw.setdefault("T", 4.5115)
    gpu = spkmc.Sim(L, 32, layout="packed", engine="slab", seed=7, record_cap=256, **kw)
    assert gpu.info()["engine"] == spkmc.ENGINES["slab"]
    orc = _orc(L, 32, seed=7, **kw)
    for n in (37, 63, 100):  # the slab counts are binned afresh at every launch
        gpu.run(n, obs_every=10)
        ro = orc.run(n, obs_every=10)
        rg = gpu.records(len(ro)) if ro else []
        assert len(rg) == len(ro)
        for g_, o_ in zip(rg, ro):
            _same(g_, o_)
        _same(gpu.state(), orc.state())
        assert np.array_equal(gpu.spins(), orc.spins())
    assert orc.check_failures() == 0


@pytest.mark.parametrize("L,cycles", [(512, 300), (1024, 120)])
def test_slab_vs_persistent(spkmc, L, cycles):
    """Beyond the oracle's reach: the same trajectory as the re-binning engine,
    including at the full 1024^3 size, in one launch and across two."""
    print("case slab vs persistent", L, cycles, flush=True)
    a = spkmc.Sim(L, 32, engine="slab", seed=11, record_cap=64)
    b = spkmc.Sim(L, 32, engine="persistent", seed=11, record_cap=64)
    a.run(cycles // 3, obs_every=20)
    a.run(cycles - cycles // 3, obs_every=20)
    b.run(cycles, obs_every=20)
    assert a.records() == b.records()
    assert a.state() == b.state()
    assert np.array_equal(a.spins(), b.spins())
    del a, b


def test_slab_unsupported(spkmc):
    with pytest.raises(spkmc.SpkmcError):
        spkmc.Sim(64, 16, engine="slab", seed=1)                     # octant edge 8
    with pytest.raises(spkmc.SpkmcError):
        spkmc.Sim(64, 32, engine="slab", seed=1, variant=2)          # two colours
    with pytest.raises(spkmc.SpkmcError):
        spkmc.Sim(64, 32, engine="slab", seed=1, variant=4)          # the fixed bound
    with pytest.raises(spkmc.SpkmcError):
        spkmc.Sim(64, 32, engine="slab", seed=1, layout="int8")


@pytest.mark.parametrize("L,kw", [
    (32, dict()),
    (64, dict(H=0.05, rates="metropolis")),
    (128, dict(init="up", T=4.4)),
    (160, dict(H=-0.05)),
])
def test_slab_rmax_all_vs_oracle(spkmc, L, kw):
    """The all-octant R_max (variant A) from the counts of every octant."""
    print("case slab rmax_all", L, kw, flush=True)
    kw.setdefault("T", 4.5115)
    gpu = spkmc.Sim(L, 32, layout="packed", engine="slab", variant=1, seed=13, record_cap=256, **kw)
    assert gpu.info()["engine"] == spkmc.ENGINES["slab"]
    orc = _orc(L, 32, seed=13, rmax_scope=1, **kw)
    for n in (37, 63, 100):
        gpu.run(n, obs_every=10)
        ro = orc.run(n, obs_every=10)
        rg = gpu.records(len(ro)) if ro else []
        assert len(rg) == len(ro)
        for g_, o_ in zip(rg, ro):
            _same(g_, o_)
        _same(gpu.state(), orc.state())
        assert np.array_equal(gpu.spins(), orc.spins())
    assert orc.check_failures() == 0


def test_slab_rmax_all_vs_incremental(spkmc):
    print("case slab rmax_all vs incremental 512", flush=True)
    a = spkmc.Sim(512, 32, engine="slab", variant=1, seed=17, record_cap=64)
    b = spkmc.Sim(512, 32, engine="incremental", variant=1, seed=17, record_cap=64)
    a.run(150, obs_every=25)
    b.run(150, obs_every=25)
    assert a.records() == b.records()
    assert a.state() == b.state()
    assert np.array_equal(a.spins(), b.spins())
