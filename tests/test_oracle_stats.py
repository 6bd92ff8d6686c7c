"""Statistical pins of the CPU oracle against closed forms.

* L = 2 exact enumeration (oracle.enumerate2, computed from eq. 1 alone):
  serial BKL and the spkMC cycle with R_max over all octants reach the
  Boltzmann law; the spkMC cycle with R_max over the active octant reaches the
  closed-form law proportional to sum_s 1/r_s.
* J = 0: independent spins relax as m(t) = m_inf + (m0 - m_inf) exp(-Gamma t)
  with m_inf = tanh(beta H); this fixes the time normalisation of step 5.
* the paper's central claim (Sec. 4): the bias of the parallel method against
  the serial mean stays within the combined standard deviation (eqs. 6-7).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import enumerate2

TC = 1.0 / 0.2216546


def _batch_means(run_batch, nbatch):
    vals = np.array([run_batch() for _ in range(nbatch)])
    return vals.mean(axis=0), vals.std(axis=0, ddof=1) / math.sqrt(nbatch)


def _tw_batch(sim_or_bkl, n):
    tw, _ = sim_or_bkl.run_tw(n)
    return tw[1:] / tw[0]  # <E>, <|M|>, <M^2> time-weighted


@pytest.mark.parametrize("T,H,rates", [(TC, 0.0, 0), (3.0, 0.2, 0), (TC, 0.0, 1)])
def test_l2_bkl_reaches_boltzmann(T, H, rates):
    ex = enumerate2.averages(1.0, H, T, rates)["boltzmann"]
    bkl = oracle.Bkl(L=2, T=T, H=H, rates=rates, seed=17)
    bkl.run(1000)
    mean, se = _batch_means(lambda: _tw_batch(bkl, 20000), 30)
    for v, m, s in zip((ex["E"], ex["absM"], ex["M2"]), mean, se):
        assert abs(m - v) < 5 * s + 1e-9, (m, v, s)


@pytest.mark.parametrize("T,H,rates", [(TC, 0.0, 0), (3.0, 0.2, 0), (TC, 0.0, 1)])
def test_l2_spkmc_active_reaches_closed_form(T, H, rates):
    laws = enumerate2.averages(1.0, H, T, rates)
    ex = laws["spkmc_active"]
    sim = oracle.Sim(L=2, d=2, T=T, H=H, rates=rates, seed=23)
    sim.run(1000)
    mean, se = _batch_means(lambda: _tw_batch(sim, 20000), 30)
    for v, m, s in zip((ex["E"], ex["absM"], ex["M2"]), mean, se):
        assert abs(m - v) < 5 * s + 1e-9, (m, v, s)
    # and the test can tell the two laws apart
    assert abs(laws["boltzmann"]["E"] - ex["E"]) > 20 * se[0]


def test_l2_state_distribution():
    """The whole 256-state time-weighted law, not only three moments."""
    T, H = TC, 0.1
    laws = enumerate2.averages(1.0, H, T, 0)
    for scope, key in ((0, "spkmc_active"), (1, "boltzmann")):
        sim = oracle.Sim(L=2, d=2, T=T, H=H, seed=31, rmax_scope=scope)
        _, hist = sim.run_tw(4000000, state_hist=True)
        p = hist / hist.sum()
        tv = 0.5 * np.abs(p - laws[key]["p"]).sum()
        assert tv < 0.01, (scope, tv)
    # the two laws are far apart compared with that tolerance
    assert 0.5 * np.abs(laws["spkmc_active"]["p"] - laws["boltzmann"]["p"]).sum() > 0.2
    bkl = oracle.Bkl(L=2, T=T, H=H, seed=37)
    _, hist = bkl.run_tw(4000000, state_hist=True)
    p = hist / hist.sum()
    assert 0.5 * np.abs(p - laws["boltzmann"]["p"]).sum() < 0.01


def test_l2_spkmc_all_octants_reaches_boltzmann():
    T, H = TC, 0.0
    ex = enumerate2.averages(1.0, H, T, 0)["boltzmann"]
    sim = oracle.Sim(L=2, d=2, T=T, H=H, seed=29, rmax_scope=1)
    sim.run(1000)
    mean, se = _batch_means(lambda: _tw_batch(sim, 20000), 30)
    for v, m, s in zip((ex["E"], ex["absM"], ex["M2"]), mean, se):
        assert abs(m - v) < 5 * s + 1e-9, (m, v, s)


def _j0_curve(make, grid, runs):
    ms = []
    for r in range(runs):
        obj = make(r)
        M, _ = obj.run_grid(grid)
        assert len(M) == len(grid)
        ms.append(M / obj.N)
    return np.array(ms)


def _j0_check(curves, want, N):
    """Mean of the runs against the closed form.  Every run shares one clock
    over all its domains, so the run-to-run scatter of m(t) exceeds that of N
    independent spins; the error bar is the larger of the empirical standard
    error and the independent-spin one."""
    runs = curves.shape[0]
    se = np.maximum(curves.std(axis=0, ddof=1), np.sqrt((1 - want ** 2) / N)) / math.sqrt(runs)
    dev = np.abs(curves.mean(axis=0) - want)
    assert np.all(dev < 5 * se), (curves.mean(axis=0), want, se)


J0_T, J0_H = 1.0, 0.3
J0_GRID = np.array([0.05, 0.2, 0.5, 1.0, 2.0, 4.0])


def _j0_want(rates):
    beta = 1.0 / J0_T
    minf = math.tanh(beta * J0_H)
    gamma = 1.0 if rates == 0 else 1.0 + math.exp(-2 * beta * abs(J0_H))
    return minf + (1 - minf) * np.exp(-gamma * J0_GRID)


@pytest.mark.parametrize("rates", [0, 1])
def test_j0_relaxation_closed_form(rates):
    """J = 0, field H, from all +1: every spin is an independent two-state
    process, m(t) = m_inf + (1 - m_inf) exp(-Gamma t) with m_inf = tanh(beta H),
    Gamma = 1 (Glauber) or 1 + exp(-2 beta |H|) (Metropolis).  A wrong colour
    factor in the clock would change Gamma eightfold."""
    want = _j0_want(rates)
    N, runs = 32 ** 3, 8
    _j0_check(_j0_curve(lambda r: oracle.Sim(L=32, d=16, J=0.0, H=J0_H, T=J0_T, rates=rates, init=1,
                                             seed=100 + r), J0_GRID, runs), want, N)
    _j0_check(_j0_curve(lambda r: oracle.Bkl(L=32, J=0.0, H=J0_H, T=J0_T, rates=rates, init=1, seed=200 + r),
                        J0_GRID, runs), want, N)


@pytest.mark.parametrize("colours,scope", [(8, 1), (8, 2), (2, 0), (2, 1), (2, 2)])
def test_j0_relaxation_variant_clocks(colours, scope):
    """The clock of every variant (Sec. 3.1 step 5 with S colours, reading R5):
    two colours (S = 2, four lines per domain), R_max over all octants, and the
    fixed bound R'_max.  At J = 0 the drift of M is linear in the spins, so
    d<M>/dt takes the physical value for any R_max rule that the clock divides
    out: m(t) follows the closed form exactly in expectation.  S = 8 left in
    for two colours would slow the decay fourfold; a clock that ignored the
    larger all-octant or bound R_max would speed it up."""
    want = _j0_want(0)
    N, runs = 32 ** 3, 8
    curves = _j0_curve(lambda r: oracle.Sim(L=32, d=16, J=0.0, H=J0_H, T=J0_T, init=1, seed=300 + r,
                                            colours=colours, rmax_scope=scope), J0_GRID, runs)
    _j0_check(curves, want, N)
    # the same runs are far from the curve of a clock off by a factor of four
    minf = math.tanh(J0_H / J0_T)
    wrong = minf + (1 - minf) * np.exp(-4.0 * J0_GRID)
    assert abs(curves.mean(axis=0)[2] - wrong[2]) > 0.1


def test_spkmc_bias_within_serial_deviation():
    """Eqs. 6-7 on the oracle: m(t) from all +1 at T_c, L = 32 (2^15 spins),
    512 sites per octant; the time-integrated bias of the parallel mean against
    the serial mean is smaller than 3 sigma_b, sigma_b^2 = sigma_p^2 + sigma_s^2
    (standard errors of the two means)."""
    L, d, runs = 32, 16, 12
    grid = np.linspace(0.5, 8.0, 16)

    def integ(make):
        vals = []
        for r in range(runs):
            M, _ = make(r).run_grid(grid)
            vals.append(np.trapezoid(M / L ** 3, grid) / (grid[-1] - grid[0]))
        return np.mean(vals), np.std(vals, ddof=1) / math.sqrt(runs)

    mp, sp = integ(lambda r: oracle.Sim(L=L, d=d, T=TC, init=1, seed=1000 + r))
    ms, ss = integ(lambda r: oracle.Bkl(L=L, T=TC, init=1, seed=2000 + r))
    sigma_b = math.sqrt(sp ** 2 + ss ** 2)
    assert abs(mp - ms) < 3 * sigma_b, (mp, ms, sigma_b)


# --- the paper-literal variants: two colours (octant parity) and the optimistic
# bound R'_max; exact laws from the 256-state transition matrix built from eq. 1

def test_cycle_law_solver_matches_closed_forms():
    """The matrix solver reproduces the two closed forms it generalises."""
    T, H = TC, 0.1
    laws = enumerate2.averages(1.0, H, T, 0)
    assert np.abs(enumerate2.cycle_law(1.0, H, T, 0, 8, 0) - laws["spkmc_active"]["p"]).max() < 1e-10
    assert np.abs(enumerate2.cycle_law(1.0, H, T, 0, 8, 1) - laws["boltzmann"]["p"]).max() < 1e-10
    # the bound is exact uniformisation: Boltzmann for both colourings
    assert np.abs(enumerate2.cycle_law(1.0, H, T, 0, 8, 2) - laws["boltzmann"]["p"]).max() < 1e-10
    assert np.abs(enumerate2.cycle_law(1.0, H, T, 0, 2, 2) - laws["boltzmann"]["p"]).max() < 1e-10
    # two colours with a state-dependent R_max is a different law
    p2 = enumerate2.cycle_law(1.0, H, T, 0, 2, 0)
    assert 0.5 * np.abs(p2 - laws["boltzmann"]["p"]).sum() > 0.05


@pytest.mark.parametrize("colours,scope", [(2, 0), (2, 1), (2, 2), (8, 2)])
def test_l2_variant_state_distribution(colours, scope):
    T, H = TC, 0.1
    law = enumerate2.cycle_law(1.0, H, T, 0, colours, scope)
    sim = oracle.Sim(L=2, d=2, T=T, H=H, seed=41 + scope, colours=colours, rmax_scope=scope)
    _, hist = sim.run_tw(2000000, state_hist=True)
    p = hist / hist.sum()
    tv = 0.5 * np.abs(p - law).sum()
    assert tv < 0.01, (colours, scope, tv)
    assert sim.check_failures() == 0


def test_bound_is_the_largest_line_rate():
    """R'_max = n_k max_c r_c: reached by a region whose every site is in the
    fastest class, never exceeded by any line during a run."""
    for rates, H in ((0, 0.0), (0, 0.3), (1, 0.0)):
        sim = oracle.Sim(L=16, d=8, T=TC, H=H, rates=rates, seed=3, rmax_scope=2, check=1)
        r = sim.rates()
        assert sim.rbound() == 64 * r.max()
        # class 0 (a down spin whose six neighbours are up) is the fastest
        # Glauber class for H >= 0
        if rates == 0:
            assert r.argmax() == 0
        sim.run(300)
        assert sim.check_failures() == 0
