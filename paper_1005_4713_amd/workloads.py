"""Seeded synthetic workloads (parameter sets only, no arithmetic of the method).

The lattices of the paper are synthetic Ising systems: a workload is fully
described by (L, d, J, H, T, rates, init, seed, cycles).  Both the GPU tests,
the benchmark and the oracle-based tests take their parameters from here.
"""
BETA_C = 0.2216546          # most accurate estimate quoted in Sec. 2 / Sec. 6
T_C = 1.0 / BETA_C

# The configurations the hot path is measured and checked on.
SMALL_L16 = dict(name="L16_d8_int8", L=16, domain=8, J=1.0, H=0.0, T=4.5115, rates="glauber", init="random",
                 seed=1, layout="int8", cycles=1000, obs_every=1)
MEDIUM_L128 = dict(name="L128_d8_int8", L=128, domain=8, J=1.0, H=0.0, T=4.5115, rates="glauber",
                   init="random", seed=2, layout="int8", cycles=10000, obs_every=10)
LARGE_L512 = [dict(name=f"L512_d16_T{T}_{r}_{i}", L=512, domain=16, J=1.0, H=0.0, T=T, rates=r, init=i,
                   seed=3 + n, layout="packed", cycles=2000, obs_every=10)
              for n, (T, r, i) in enumerate((T, r, i) for T in (4.40, 4.5115, 4.60)
                                            for r in ("metropolis", "glauber") for i in ("up", "random"))]
HEADLINE_L1024 = dict(name="L1024_d32_packed_Tc", L=1024, domain=32, J=1.0, H=0.0, T=4.5115, rates="glauber",
                      init="random", seed=42, layout="packed", cycles=500, obs_every=10)


def replica_mix(n=256, seed=5):
    """The batched/served mix: L from {32,48,64,96,128,192,256}, T uniform in
    [4.0, 5.0], H in {0, +0.05, -0.05}, each replica with its own seed.
    Drawn with numpy's Philox generator (a library RNG, not the method's)."""
    import numpy as np
    g = np.random.Generator(np.random.Philox(seed))
    Ls = [32, 48, 64, 96, 128, 192, 256]
    out = []
    for i in range(n):
        L = int(g.choice(Ls))
        T = float(g.uniform(4.0, 5.0))
        H = float(g.choice([0.0, 0.05, -0.05]))
        out.append(dict(name=f"replica{i}", L=L, J=1.0, H=H, T=T, rates="glauber", init="random",
                        seed=1000 + i, layout="packed", cycles=1000))
    return out


def arrivals(n=256, rate=50.0, seed=6):
    """Poisson arrival times (exponential gaps at `rate` per second)."""
    import numpy as np
    g = np.random.Generator(np.random.Philox(seed))
    return np.cumsum(g.exponential(1.0 / rate, n))
