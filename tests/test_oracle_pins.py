"""Deterministic pins of the CPU oracle against things other than itself.

* Philox4x32-10 against rocRAND's independent open-source engine.
* the uniform conversions against their exact closed forms.
* the rate table against detailed balance with eq. 1 and against flip energies
  evaluated from the Hamiltonian on explicit configurations.
* site classes and octant histograms against a numpy (np.roll) count.
* the chessboard geometry (octants of one colour never interact) by brute force.
* the frequency-line selection against the probabilities of steps 3, 4 and 4b,
  measured exactly over a fine grid of uniforms.
* invariants, order independence and resume of the spkMC cycle.
* spkMC with one active region equals serial BKL driven by the same draws.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TC = 1.0 / 0.2216546


# --------------------------------------------------------------------------- Philox
@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("kat") / "kat")
    src = os.path.join(ROOT, "tests", "golden", "philox_rocrand_kat.cpp")
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_kat):
    rng = np.random.default_rng(12345)
    cases = [((0, 0, 0, 0), (0, 0)), ((0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF, 0xFFFFFFFF))]
    for _ in range(64):
        c = [int(v) for v in rng.integers(0, 2 ** 32, 4)]
        c[1] &= 0x3FFFFFFF  # the engine reaches the counter through a 64-bit offset of 4 c_lo
        k = [int(v) for v in rng.integers(0, 2 ** 32, 2)]
        cases.append((tuple(c), tuple(k)))
    inp = "".join(f"{c[0]} {c[1]} {c[2]} {c[3]} {k[0]} {k[1]}\n" for c, k in cases)
    out = subprocess.run([rocrand_kat], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [tuple(int(v) for v in line.split()) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for (c, k), r in zip(cases, ref):
        assert oracle.philox(c, k) == r, (c, k)


# --------------------------------------------------------------------------- conversions
def test_uniform_conversions_closed_forms():
    assert oracle.u53(0, 0) == 0.0
    assert oracle.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert oracle.uopen52(0, 0) == 2.0 ** -53
    assert oracle.uopen52(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    rng = np.random.default_rng(7)
    for a, b in rng.integers(0, 2 ** 32, (200, 2)):
        a, b = int(a), int(b)
        m53 = ((a >> 5) << 26) | (b >> 6)
        assert oracle.u53(a, b) == m53 / 2.0 ** 53
        m52 = ((a >> 6) << 26) | (b >> 6)
        assert oracle.uopen52(a, b) == (m52 + 0.5) / 2.0 ** 52
        assert 0.0 < oracle.uopen52(a, b) < 1.0
    for n in (1, 2, 3, 7, 64, 4096, 2 ** 31 + 5):
        assert oracle.idx(0, n) == 0
        assert oracle.idx(0xFFFFFFFF, n) == n - 1
        assert oracle.idx(0x80000000, n) == n // 2
        for w in rng.integers(0, 2 ** 32, 50):
            assert oracle.idx(int(w), n) == (int(w) * n) >> 32


# --------------------------------------------------------------------------- rates
def _energy(sp, J, H):
    B = 0
    for ax in range(3):
        B += int((sp * np.roll(sp, -1, axis=ax)).sum())
    return -J * B - H * int(sp.sum())


@pytest.mark.parametrize("rates", [0, 1])
@pytest.mark.parametrize("J,H", [(1.0, 0.0), (1.0, 0.05), (1.0, -0.05), (0.0, 0.3), (-0.5, 0.1)])
@pytest.mark.parametrize("T", [4.40, TC, 4.60, 1.0e3, 1.7])
def test_rate_table_detailed_balance(rates, J, H, T):
    r = oracle.rate_table(J, H, T, rates)
    beta = 1.0 / T
    for c in range(14):
        sgn = 1 if c >= 7 else -1
        a = c % 7
        # the reverse move: the flipped spin has the opposite sign and 6 - a aligned neighbours
        c_rev = (0 if sgn == 1 else 7) + (6 - a)
        dE = 2.0 * J * (2 * a - 6) + 2.0 * H * sgn
        ratio = r[c] / r[c_rev]
        assert ratio == pytest.approx(math.exp(-beta * dE), rel=1e-13)
        if rates == 1:
            assert r[c] == (1.0 if dE <= 0 else pytest.approx(math.exp(-beta * dE), rel=1e-15))
        assert 0.0 < r[c] <= 1.0


def test_rate_classes_match_hamiltonian():
    """The class -> flip energy map of the table agrees with eq. 1 evaluated on
    explicit lattices: for every site, E(flipped) - E(original) must make the
    Glauber rate of the site's class (detailed balance then fixes the rest)."""
    rng = np.random.default_rng(3)
    for (J, H, T) in [(1.0, 0.0, TC), (1.0, 0.05, 4.4), (0.7, -0.2, 2.5)]:
        r = oracle.rate_table(J, H, T, 0)
        for L in (2, 3, 4):
            sp = rng.choice(np.array([-1, 1], dtype=np.int8), size=(L, L, L))
            flat = np.ascontiguousarray(sp.transpose(2, 1, 0)).reshape(-1)  # index x + L(y + Lz)
            E0 = _energy(sp.astype(np.int64), J, H)
            for x in range(L):
                for y in range(L):
                    for z in range(L):
                        sp2 = sp.astype(np.int64).copy()
                        sp2[x, y, z] *= -1
                        dE = _energy(sp2, J, H) - E0
                        c = oracle.site_class(flat, x, y, z)
                        assert r[c] == pytest.approx(1.0 / (1.0 + math.exp(dE / T)), rel=1e-12)


def test_rate_table_rejects_degenerate():
    with pytest.raises(ValueError):
        oracle.rate_table(1.0, 0.0, 0.0)
    with pytest.raises(ValueError):
        oracle.rate_table(1.0, 0.0, -1.0)
    with pytest.raises(ValueError):
        oracle.rate_table(1.0, 0.0, 1e-3)  # exp overflows: some rates are exactly 0
    with pytest.raises(ValueError):
        oracle.rate_table(1.0, 0.0, 4.5, rates=3)


# --------------------------------------------------------------------------- classes
def _classes_numpy(sp):
    """class of every site: 7 [s=+1] + number of the 6 periodic neighbours equal to s."""
    a = np.zeros(sp.shape, dtype=np.int64)
    for ax in range(3):
        for sh in (1, -1):
            a += (np.roll(sp, sh, axis=ax) == sp)
    return 7 * (sp > 0) + a


@pytest.mark.parametrize("L", [2, 3, 5, 8])
def test_site_classes_vs_numpy(L):
    rng = np.random.default_rng(L)
    sp = rng.choice(np.array([-1, 1], dtype=np.int8), size=(L, L, L))  # sp[x, y, z]
    flat = np.ascontiguousarray(sp.transpose(2, 1, 0)).reshape(-1)
    cls = _classes_numpy(sp)
    for x in range(L):
        for y in range(L):
            for z in range(L):
                assert oracle.site_class(flat, x, y, z) == cls[x, y, z]
    M, B = oracle.observables(flat)
    assert M == int(sp.astype(np.int64).sum())
    assert B == sum(int((sp.astype(np.int64) * np.roll(sp, -1, axis=ax)).sum()) for ax in range(3))


def _octant_sites(L, d, k, s):
    nd = L // d
    h = d // 2
    kx, ky, kz = k % nd, (k // nd) % nd, k // (nd * nd)
    ox, oy, oz = kx * d + (s & 1) * h, ky * d + ((s >> 1) & 1) * h, kz * d + ((s >> 2) & 1) * h
    return [(ox + lx, oy + ly, oz + lz) for lz in range(h) for ly in range(h) for lx in range(h)]


@pytest.mark.parametrize("L,d", [(8, 4), (16, 8), (12, 4), (8, 2)])
def test_octant_histograms_vs_numpy(L, d):
    sim = oracle.Sim(L=L, d=d, seed=99)
    flat = sim.spins()
    sp = flat.reshape(L, L, L).transpose(2, 1, 0)  # sp[x, y, z]
    cls = _classes_numpy(sp)
    K = (L // d) ** 3
    for k in range(K):
        for s in range(8):
            want = np.bincount([cls[p] for p in _octant_sites(L, d, k, s)], minlength=14)
            assert list(want) == sim.octant_hist(k, s)


@pytest.mark.parametrize("L,d", [(8, 4), (12, 4), (16, 8), (8, 2), (4, 2), (24, 6)])
def test_same_colour_octants_do_not_interact(L, d):
    """No site of one active octant, nor of its 1-site halo, lies in another
    active octant of the same colour (Sec. 3.2: subcells larger than the
    interaction range)."""
    K = (L // d) ** 3
    for s in range(8):
        owner = {}
        for k in range(K):
            for p in _octant_sites(L, d, k, s):
                assert p not in owner
                owner[p] = k
        for k in range(K):
            for (x, y, z) in _octant_sites(L, d, k, s):
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    q = ((x + dx) % L, (y + dy) % L, (z + dz) % L)
                    assert owner.get(q, k) == k


# --------------------------------------------------------------------------- selection
def test_frequency_line_probabilities_exact():
    """Steps 3, 4, 4b: with a uniform u the chosen class c has probability
    n_c r_c / R_max and the null event (R_max - R_k) / R_max; the in-class index
    is uniform.  Measured exactly over a grid of u and w."""
    rng = np.random.default_rng(5)
    r = oracle.rate_table(1.0, 0.05, TC, 0)
    for trial in range(6):
        hist = rng.integers(0, 40, 14).astype(np.uint32)
        hist[rng.integers(0, 14, 3)] = 0
        Rk = float((hist * r).sum())
        Rmax = Rk * (1.0 + 0.5 * trial / 5)
        G = 1 << 16
        counts = np.zeros(15)
        for i in range(G):
            u = (i + 0.5) / G
            got = oracle.select(hist, r, Rmax, u, 0)
            counts[14 if got is None else got[0]] += 1
        want = np.append(hist * r / Rmax, (Rmax - Rk) / Rmax)
        assert np.all(np.abs(counts / G - want) <= 2.0 / G + 1e-12), (counts / G, want)
        for c in np.nonzero(hist)[0]:
            # the j drawn inside the class covers 0..n-1 uniformly
            n = int(hist[c])
            js = np.bincount([oracle.idx(int(w), n) for w in np.linspace(0, 2 ** 32 - 1, 4096).astype(np.uint64)],
                             minlength=n)
            assert js.min() >= 4096 // n - 1 and js.max() <= 4096 // n + 2


# --------------------------------------------------------------------------- random start
@pytest.mark.parametrize("seed", [1, 2, 42])
def test_random_start_is_iid_half(seed):
    """init = random gives iid +-1 spins with p = 1/2 (the workloads' random
    start): the magnetisation, the correlation at every lag that the block and
    word structure of the draws could repeat at (1, the 32-bit word, the
    128-bit block, one x row, one plane), the nearest-neighbour correlation on
    the periodic lattice along each axis, the up count of every 128-site block
    against Binomial(128, 1/2), and no block repeated."""
    from scipy import stats
    L = 64
    N = L ** 3
    s = oracle.init_spins(L, seed, 0).astype(np.float64)
    assert set(np.unique(s)) == {-1.0, 1.0}
    lim = 5.0 / math.sqrt(N)
    assert abs(s.mean()) < lim
    for lag in (1, 2, 31, 32, 33, 64, 96, 127, 128, 129, 256, 512, L, L * L, 4096):
        assert abs(np.mean(s[:-lag] * s[lag:])) < 5.0 / math.sqrt(N - lag), lag
    cube = s.reshape(L, L, L)  # [z, y, x]
    for ax in range(3):
        assert abs(np.mean(cube * np.roll(cube, 1, axis=ax))) < lim, ax
    blocks = (s.reshape(-1, 128) > 0)
    ups = blocks.sum(axis=1)
    obs = np.bincount(ups, minlength=129)
    # pool the tails so every expected count is at least 5
    pmf = stats.binom.pmf(np.arange(129), 128, 0.5)
    lo, hi = 46, 82
    o = np.concatenate([[obs[:lo].sum()], obs[lo:hi + 1], [obs[hi + 1:].sum()]])
    e = np.concatenate([[pmf[:lo].sum()], pmf[lo:hi + 1], [pmf[hi + 1:].sum()]]) * len(ups)
    assert stats.chisquare(o, e).pvalue > 1e-4
    packed = np.packbits(blocks, axis=1)
    assert len({row.tobytes() for row in packed}) == len(packed)  # no Philox block repeats
    # a different key gives an uncorrelated lattice
    s2 = oracle.init_spins(L, seed + 1000, 0).astype(np.float64)
    assert abs(np.mean(s * s2)) < lim


# --------------------------------------------------------------------------- cycle invariants
@pytest.mark.parametrize("L,d,init", [(16, 8, 0), (16, 4, 1), (12, 6, 2), (8, 2, 0)])
def test_cycle_invariants(L, d, init):
    sim = oracle.Sim(L=L, d=d, seed=11, init=init, check=1, H=0.05)
    K = (L // d) ** 3
    recs = sim.run(300, obs_every=1)
    assert sim.check_failures() == 0  # incremental M, B equal a full recompute every cycle
    prev = (0, 0, 0)
    for (n, fired, nulls, t, M, B) in recs:
        assert fired + nulls == K * n
        assert fired - prev[0] <= K
        assert t > prev[2]
        assert (L ** 3 - M) % 2 == 0 and abs(M) <= L ** 3 and abs(B) <= 3 * L ** 3
        prev = (fired, nulls, t)
    M, B = oracle.observables(sim.spins())
    assert (M, B) == (recs[-1][4], recs[-1][5])


@pytest.mark.parametrize("colours,scope", [(8, 0), (2, 0), (8, 1), (2, 2)])
def test_thread_count_independence(colours, scope):
    """The opt-in parallel-for over domains gives the single-threaded
    trajectory bit for bit (records and final spins)."""
    out = []
    before = oracle.get_threads()
    for nt in (1, 4):
        oracle.set_threads(nt)
        try:
            sim = oracle.Sim(L=16, d=4, seed=19, H=0.05, colours=colours, rmax_scope=scope, check=1)
            recs = sim.run(200, obs_every=7)
            assert sim.check_failures() == 0
            out.append((recs, sim.spins()))
        finally:
            oracle.set_threads(before)
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])


def test_order_independence():
    """Deciding every domain first and applying after, applying at once in
    domain order, and applying at once in a shuffled order give the same
    trajectory bit for bit: active octants never read what another writes."""
    for L, d in [(16, 4), (12, 6), (16, 8)]:
        outs = []
        for order in (0, 1, 2):
            sim = oracle.Sim(L=L, d=d, seed=5, order=order)
            recs = sim.run(200, obs_every=10)
            outs.append((recs, sim.spins().tobytes()))
            assert sim.check_failures() == 0
        assert outs[0] == outs[1] == outs[2]


@pytest.mark.parametrize("scope", [0, 1, 2])
def test_two_colour_lines_independent(scope):
    """Two colours: the four active octants of a domain (and of every domain)
    never touch, so applying each flip at once, in domain order or shuffled,
    gives the trajectory of deciding every line first; every line's histogram
    is recomputed before its decision and must be unchanged."""
    for L, d in [(16, 4), (12, 6), (8, 2)]:
        outs = []
        for order in (0, 1, 2):
            sim = oracle.Sim(L=L, d=d, seed=7, order=order, colours=2, rmax_scope=scope, check=1)
            recs = sim.run(150, obs_every=10)
            outs.append((recs, sim.spins().tobytes()))
            assert sim.check_failures() == 0
        assert outs[0] == outs[1] == outs[2]
        K = (L // d) ** 3
        for (n, fired, nulls, t, M, B) in outs[0][0]:
            assert fired + nulls == 4 * K * n  # four lines per domain and cycle


def test_bound_lowers_utilisation_not_the_law():
    """R'_max >= R_max: the same trajectory law with more null events; the mean
    cycle length is 1 / (8 R'_max) exactly."""
    a = oracle.Sim(L=16, d=8, seed=9, rmax_scope=0)
    b = oracle.Sim(L=16, d=8, seed=9, rmax_scope=2)
    ra, rb = a.run(400), b.run(400)
    sa, sb = a.state(), b.state()
    assert sb[1] / (sb[1] + sb[2]) < sa[1] / (sa[1] + sa[2])
    assert abs(sb[3] - 400 / (8 * b.rbound())) < 0.15 * 400 / (8 * b.rbound())


def test_resume_is_exact():
    a = oracle.Sim(L=16, d=8, seed=21)
    a.run(300)
    b = oracle.Sim(L=16, d=8, seed=21)
    b.run(150)
    st = b.state()
    c = oracle.Sim(L=16, d=8, seed=21, init=1)
    c.set_state(b.spins(), cycle=st[0], fired=st[1], nulls=st[2], t=st[3])
    c.run(150)
    assert a.state() == c.state()
    assert np.array_equal(a.spins(), c.spins())


def test_high_symmetry_all_rates_half():
    """J = H = 0: every rate is 1/2, every R_k = h^3/2 = R_max, so every domain
    fires every cycle (utilisation 1) and E[dt] = 1 / (8 R_max) = 1 / (4 h^3)."""
    L, d = 16, 4
    h = d // 2
    sim = oracle.Sim(L=L, d=d, J=0.0, H=0.0, seed=3)
    n = 4000
    recs = sim.run(n, obs_every=n)
    K = (L // d) ** 3
    assert recs[-1][1] == K * n and recs[-1][2] == 0
    mean_dt = recs[-1][3] / n
    se = (1.0 / (4 * h ** 3)) / math.sqrt(n)
    assert abs(mean_dt - 1.0 / (4 * h ** 3)) < 5 * se


def test_one_region_equals_serial_bkl_with_same_draws():
    """With one domain and one colour the frequency line is the whole lattice
    and R_max = R_tot: the spkMC cycle is then the serial BKL step.  Driven by
    the same draws, the two simulators agree bit for bit (spins and clock)."""
    for L, seed, init in [(4, 1, 0), (6, 2, 1), (4, 9, 2)]:
        sim = oracle.Sim(L=L, d=L, colours=1, seed=seed, init=init, H=0.05)
        bkl = oracle.Bkl(L=L, canonical=1, draw_mode=1, seed=seed, init=init, H=0.05)
        for _ in range(5):
            sim.run(100)
            bkl.run(100)
            assert np.array_equal(sim.spins(), bkl.spins())
            s, b = sim.state(), bkl.state()
            assert s[3] == b[3] and s[4:] == b[4:] and s[1] == b[1]


def test_bkl_list_mode_counts_consistent():
    bkl = oracle.Bkl(L=8, seed=4)
    bkl.run(20000)
    sp = bkl.spins()
    cls = _classes_numpy(sp.reshape(8, 8, 8).transpose(2, 1, 0))
    assert list(np.bincount(cls.reshape(-1), minlength=14)) == bkl.counts()
    M, B = oracle.observables(sp)
    assert (M, B) == bkl.state()[4:]


def test_invalid_geometry_rejected():
    for kw in [dict(L=16, d=3), dict(L=16, d=6), dict(L=1, d=2), dict(L=16, d=0), dict(L=8, d=4, colours=1),
               dict(L=8, d=4, colours=3), dict(L=8, d=4, rmax_scope=3)]:
        with pytest.raises(ValueError):
            oracle.Sim(**kw)
