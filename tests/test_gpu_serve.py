"""The request server on the GPU: continuous batching (requests admitted while
others run, by pool footprint, advanced in macro-steps) leaves every lattice
bit-identical to running it alone with the plain path."""
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


MIX = [
    # (L, domain, layout, T, H, seed, ncycles, obs_every)
    (32, 16, "packed", 4.5115, 0.0, 11, 120, 10),
    (48, 16, "packed", 4.2, 0.05, 12, 37, 10),
    (64, 16, "packed", 4.9, -0.05, 13, 260, 10),
    (64, 32, "packed", 4.5115, 0.0, 14, 150, 10),
    (96, 32, "packed", 4.0, 0.05, 15, 75, 10),
    (32, 8, "packed", 4.5115, 0.0, 16, 90, 10),   # octant edge 4: runs alone
    (16, 8, "int8", 4.5115, 0.05, 17, 64, 10),    # int8: runs alone
    (128, 16, "packed", 4.6, 0.0, 18, 200, 10),
    (48, 16, "packed", 4.4, 0.0, 19, 0, 10),      # no cycles: the initial state
    (64, 16, "packed", 4.5115, 0.05, 20, 101, 7),  # another observation interval
]


def _solo(spkmc, L, d, layout, T, H, seed, n, obs):
    s = spkmc.Sim(L, d, layout=layout, T=T, H=H, seed=seed, record_cap=64)
    s.run(n, obs_every=obs)
    return s.state(), s.spins(), s.records()


def test_served_equals_solo(spkmc):
    print("serve: 10-request mix, macro 50, staggered submission", flush=True)
    srv = spkmc.Server(64 << 20, macro_cycles=50, max_live=8, inflight=2)
    ids = []
    for i, (L, d, lay, T, H, seed, n, obs) in enumerate(MIX):
        ids.append(srv.submit(L, d, n, obs_every=obs, keep=True, layout=lay, T=T, H=H, seed=seed, record_cap=64))
        if i % 3 == 2:
            srv.step()  # later requests arrive while earlier ones run
    st = srv.drain()
    assert st["done"] == len(MIX) and st["failed"] == 0
    assert st["pool_peak"] <= 64 << 20
    for rid, (L, d, lay, T, H, seed, n, obs) in zip(ids, MIX):
        want_state, want_spins, want_recs = _solo(spkmc, L, d, lay, T, H, seed, n, obs)
        info = srv.poll(rid)
        assert info["state"] == spkmc.REQ_DONE
        assert info["state_tuple"] == want_state, (L, d, lay)
        assert info["t_done"] >= info["t_admit"] >= info["t_arrival"] - 1e-9
        v = srv.lattice(rid, L, record_cap=64)
        assert v.state() == want_state
        assert np.array_equal(v.spins(), want_spins), (L, d, lay)
        assert v.records() == want_recs, (L, d, lay)
        srv.release(rid)
    srv.close()


def test_served_requests_vs_oracle(spkmc):
    """Requests served in the mix (admitted while others run, advanced in shared
    batch launches or alone) against the CPU oracle directly: the record of
    every observation cycle, the final state and every spin.  The three cover a
    batched octant edge 8, a batched octant edge 16 and an int8 lattice that
    runs alone."""
    import oracle
    print("serve: mix, three requests checked against the oracle", flush=True)
    srv = spkmc.Server(64 << 20, macro_cycles=40, max_live=8, inflight=2)
    ids = []
    for i, (L, d, lay, T, H, seed, n, obs) in enumerate(MIX):
        ids.append(srv.submit(L, d, n, obs_every=obs, keep=True, layout=lay, T=T, H=H, seed=seed, record_cap=64))
        if i % 2 == 1:
            srv.step()
    st = srv.drain()
    assert st["done"] == len(MIX) and st["failed"] == 0
    for k in (2, 4, 6):
        L, d, lay, T, H, seed, n, obs = MIX[k]
        orc = oracle.Sim(L=L, d=d, T=T, H=H, seed=seed)
        ro = orc.run(n, obs_every=obs)
        v = srv.lattice(ids[k], L, record_cap=64)
        rg = v.records()
        assert len(rg) == len(ro) == n // obs, (L, d, lay)
        for g, o in zip(rg, ro):
            assert g[:3] == o[:3] and g[4:] == o[4:], (L, d, lay, g, o)
            assert abs(g[3] - o[3]) <= 1e-12 * abs(o[3]), (g, o)
        so = orc.state()
        sg = srv.poll(ids[k])["state_tuple"]
        assert sg[:3] == so[:3] and sg[4:] == so[4:] and abs(sg[3] - so[3]) <= 1e-12 * abs(so[3])
        assert np.array_equal(v.spins(), orc.spins()), (L, d, lay)
        srv.release(ids[k])
    srv.close()


def test_admission_by_footprint(spkmc):
    print("serve: admission under a pool that holds two lattices", flush=True)
    one = spkmc.state_bytes(spkmc.make_params(64, 16))
    pool = 2 * ((one + 255) // 256 * 256) + 256
    srv = spkmc.Server(pool, macro_cycles=40, max_live=16, inflight=2)
    specs = [(64, 4.3 + 0.05 * i, 100 + i, 60 + 13 * i) for i in range(7)]
    ids = [srv.submit(L, 16, n, T=T, seed=seed) for (L, T, seed, n) in specs]
    st = srv.step()
    assert st["live"] <= 2 and st["queued"] >= 1
    while True:
        st = srv.step(wait=True)
        assert st["live"] <= 2 and st["pool_in_use"] <= pool
        if st["queued"] == 0 and st["live"] == 0 and st["inflight"] == 0:
            break
    assert st["pool_peak"] <= pool and st["pool_in_use"] == 0
    assert st["done"] == len(specs)
    for rid, (L, T, seed, n) in zip(ids, specs):
        info = srv.poll(rid)
        want = spkmc.Sim(L, 16, T=T, seed=seed)
        want.run(n)
        assert info["state_tuple"] == want.state()
        srv.release(rid)
    srv.close()


def test_server_errors(spkmc):
    srv = spkmc.Server(1 << 20, macro_cycles=10, max_live=4, inflight=1)
    with pytest.raises(spkmc.SpkmcError):
        srv.submit(16, 3, 10)  # odd domain
    with pytest.raises(spkmc.SpkmcError):
        srv.submit(256, 16, 10)  # larger than the pool
    rid = srv.submit(32, 16, 30, keep=True)
    with pytest.raises(spkmc.SpkmcError):
        srv.release(rid)  # still queued
    srv.drain()
    assert srv.poll(rid)["state"] == spkmc.REQ_DONE
    srv.release(rid)
    with pytest.raises(spkmc.SpkmcError):
        srv.poll(rid)
    srv.close()


def test_served_wide_lattice_runs_alone(spkmc):
    """A lattice with more lines than one batch launch holds (two colours at 1024^3:
    131 072 lines) is served alone through spkmc_run, which takes the persistent
    kernel's wide mode, beside a small batched request; both results equal their
    solo runs (the server's 20-cycle macro-steps against one 40-cycle run)."""
    print("serve: wide lattice beside a batched one", flush=True)
    big = spkmc.state_bytes(spkmc.make_params(1024, 32, variant=2, record_cap=16))
    srv = spkmc.Server(big + (256 << 20), macro_cycles=20, max_live=4, inflight=2)
    rb = srv.submit(1024, 32, 40, obs_every=10, variant=2, T=4.5115, seed=8, record_cap=16)
    rs = srv.submit(64, 16, 40, obs_every=10, T=4.5115, seed=9, record_cap=16)
    st = srv.drain()
    assert st["done"] == 2 and st["failed"] == 0
    got_big, got_small = srv.poll(rb)["state_tuple"], srv.poll(rs)["state_tuple"]
    srv.close()
    a = spkmc.Sim(1024, 32, variant=2, T=4.5115, seed=8, record_cap=16)
    assert a.info()["engine"] == spkmc.ENGINES["persistent"] and a.info()["wg_domains"] == 512
    a.run(40, obs_every=10)
    assert got_big == a.state()
    b = spkmc.Sim(64, 16, T=4.5115, seed=9, record_cap=16)
    b.run(40, obs_every=10)
    assert got_small == b.state()
