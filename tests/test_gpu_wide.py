"""The persistent engine's wide mode (octant edge 16): each workgroup runs two or
four rounds of four passes of lines; the bin keeps only the moments, and once
the true R_max is known every round's class planes are derived again from the
spins for the selection.  It takes the lattices whose lines are too many for one
round (two colours at 1024^3; eight colours up to 131 072 domains).
Bar: spins, fired/null counts, M and B bit-exact; clock within 1e-12 relative."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
T_REL = 1e-12
TWO, BOUND = 2, 4


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


@pytest.mark.parametrize("L,variant,wg", [
    (256, 0, 256),             # 512 lines: two workgroups of two rounds
    (384, 0, 512),             # 1728 lines: three full workgroups of four rounds, one part-filled
    (256, TWO, 512),           # 2048 lines: four workgroups
    (256, TWO, 256),           # eight workgroups of two rounds
    (256, BOUND, 512),         # the fixed bound: no exchange
    (256, TWO | BOUND, 256),
])
def test_wide_against_oracle(spkmc, L, variant, wg):
    print("case wide oracle", L, variant, wg, flush=True)
    gpu = spkmc.Sim(L, 32, layout="packed", engine="persistent", wg_domains=wg, variant=variant, T=4.5115,
                    seed=29, record_cap=64)
    info = gpu.info()
    assert info["engine"] == spkmc.ENGINES["persistent"] and info["wg_domains"] == wg
    orc = oracle.Sim(L=L, d=32, colours=2 if variant & TWO else 8, rmax_scope=2 if variant & BOUND else 0,
                     T=4.5115, seed=29)
    for n in (5, 9):  # two launches
        gpu.run(n, obs_every=2)
        ro = orc.run(n, obs_every=2)
        rg = gpu.records(len(ro)) if ro else []
        assert len(rg) == len(ro)
        for g_, o_ in zip(rg, ro):
            _same(g_, o_)
        _same(gpu.state(), orc.state())
        assert np.array_equal(gpu.spins(), orc.spins())


@pytest.mark.parametrize("L,variant,wg,spins", [
    (1024, TWO, 512, True),    # 131 072 lines: 256 workgroups of four rounds
    (1280, 0, 256, False),     # 64 000 lines: 250 workgroups of two rounds
])
def test_wide_equals_cycle_engine(spkmc, L, variant, wg, spins):
    """AUTO takes the wide mode; it agrees bit for bit with the per-cycle engine
    over 40 cycles in two launches, records every 5 cycles."""
    import torch
    print("case wide vs cycle", L, variant, flush=True)
    a = spkmc.Sim(L, 32, layout="packed", variant=variant, T=4.5115, seed=31, record_cap=16)
    info = a.info()
    assert info["engine"] == spkmc.ENGINES["persistent"] and info["wg_domains"] == wg
    b = spkmc.Sim(L, 32, layout="packed", engine="cycle", variant=variant, T=4.5115, seed=31, record_cap=16)
    for n in (15, 25):
        a.run(n, obs_every=5)
        b.run(n, obs_every=5)
    assert a.state() == b.state()
    assert a.records() == b.records() and len(a.records()) == 8
    if spins:
        assert np.array_equal(a.spins(), b.spins())
    del a, b
    torch.cuda.empty_cache()
