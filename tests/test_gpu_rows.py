"""The per-cycle engine's row kernels (PACKED, octant edge 8 or 16): one cycle
in two launches, bit-identical to the oracle and to the persistent engine.
Lattices here span several workgroups of lines (h = 8: 256 lines per
workgroup; h = 16: 128), with eight and with two colours and the fixed bound.
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


@pytest.mark.parametrize("variant", [0, TWO, BOUND, TWO | BOUND])
@pytest.mark.parametrize("L,d,kw", [
    (128, 16, dict()),                                # h = 8: 512 lines, 2 workgroups (8 with two colours)
    (96, 16, dict(H=0.05, rates="metropolis")),       # 216 lines: a part-filled workgroup
    (128, 32, dict(init="up", T=4.4)),                # h = 16: 64 lines
])
def test_rows_against_oracle(spkmc, variant, L, d, kw):
    print("case rows oracle", variant, L, d, kw, flush=True)
    kw = dict(kw)
    kw.setdefault("T", 4.5115)
    gpu = spkmc.Sim(L, d, layout="packed", engine="cycle", variant=variant, seed=23, record_cap=256, **kw)
    okw = dict(kw)
    okw["rates"] = {"glauber": 0, "metropolis": 1}[okw.get("rates", "glauber")]
    okw["init"] = {"random": 0, "up": 1, "down": 2}[okw.get("init", "random")]
    orc = oracle.Sim(L=L, d=d, colours=2 if variant & TWO else 8, rmax_scope=2 if variant & BOUND else 0,
                     seed=23, **okw)
    for n in (7, 12):
        gpu.run(n, obs_every=3)
        ro = orc.run(n, obs_every=3)
        rg = gpu.records(len(ro)) if ro else []
        assert len(rg) == len(ro)
        for g_, o_ in zip(rg, ro):
            _same(g_, o_)
        _same(gpu.state(), orc.state())
        assert np.array_equal(gpu.spins(), orc.spins())
    assert gpu.info()["engine"] == spkmc.ENGINES["cycle"]


@pytest.mark.parametrize("variant", [0, TWO, BOUND])
@pytest.mark.parametrize("L,d", [(256, 32), (256, 16)])
def test_rows_equal_persistent(spkmc, variant, L, d):
    """Larger lattices (2^24 spins, up to 32 768 lines): the row kernels and the
    persistent kernel agree bit for bit over 60 cycles with records."""
    print("case rows vs persistent", variant, L, d, flush=True)
    a = spkmc.Sim(L, d, layout="packed", engine="cycle", variant=variant, seed=31, record_cap=64)
    b = spkmc.Sim(L, d, layout="packed", engine="persistent", variant=variant, seed=31, record_cap=64)
    for n in (25, 35):
        a.run(n, obs_every=5)
        b.run(n, obs_every=5)
    assert a.state() == b.state()
    assert a.records() == b.records()
    assert np.array_equal(a.spins(), b.spins())


def test_headline_size_engines_agree(spkmc):
    """L = 1024, d = 32, T_c, seed 42 (the benchmark's lattice), 200 cycles with a
    record every 10: the persistent kernel and the row kernels agree bit for bit,
    and the incremental M and B equal M and B recomputed from the final spins."""
    from paper_1005_4713_amd import workloads
    w = workloads.HEADLINE_L1024
    print("case headline engines 200 cycles", flush=True)
    runs = []
    for engine in ("persistent", "cycle"):
        sim = spkmc.Sim(w["L"], w["domain"], layout="packed", engine=engine, T=w["T"], seed=w["seed"],
                        record_cap=32)
        sim.run(200, obs_every=10)
        runs.append((sim.state(), sim.records(), sim))
    (sa, ra, a), (sb, rb, b) = runs
    assert sa == sb and ra == rb
    s = a.spins().reshape(w["L"], w["L"], w["L"])  # int8, one byte per site
    assert np.array_equal(s, b.spins().reshape(w["L"], w["L"], w["L"]))
    M = int(s.sum(dtype=np.int64))
    B = sum(int((s * np.roll(s, 1, ax)).sum(dtype=np.int64)) for ax in range(3))
    assert (sa[4], sa[5]) == (M, B)


def test_largest_power_of_two_lattice(spkmc):
    """L = 2048 (2^33 sites: 1 GiB packed, 8 GiB as int8), d = 32, T_c: the
    per-cycle slab kernels (packed, word offsets up to 2^28) and the generic
    kernels (int8) agree record for record over four cycles, and every cycle
    accounts for each of the 2^18 domains once (an event or a null)."""
    import torch
    L, d, cycles = 2048, 32, 4
    print("case L2048 packed vs int8", flush=True)
    runs = []
    for layout in ("packed", "int8"):
        sim = spkmc.Sim(L, d, layout=layout, T=4.5115, seed=5, record_cap=8)
        assert sim.info()["engine"] == spkmc.ENGINES["cycle"]
        sim.run(cycles, obs_every=1)
        runs.append((sim.state(), sim.records()))
        del sim
        torch.cuda.empty_cache()
    (sa, ra), (sb, rb) = runs
    assert sa == sb and ra == rb and len(ra) == cycles
    K = (L // d) ** 3
    for i, r in enumerate(ra):
        assert r[0] == i + 1 and r[1] + r[2] == (i + 1) * K
