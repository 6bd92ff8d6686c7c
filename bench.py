"""Benchmark of the spkMC hot path on one MI355X.

A step is one spkMC cycle over the whole lattice (sublattice draw, class
binning and frequency lines of every domain, the device-wide R_max, the
event selection and flips, the clock and the counters).  The default workload
is the headline configuration: L = 1024 (2^30 spins, bit-packed), domains of
32^3, T = 4.5115, Glauber rates, random start (seed 42).

Prints one JSON line: spin-flip events per second of simulated dynamics with
the lattice resident in HBM, the roofline of the dominant kernel (algorithmic
bytes per cycle from the method: every domain reads its active octant and its
1-site halo at one bit per site and writes one flip, K ((h^3 + 6 h^2)/8 + 8)
bytes), the batched and served forms on the replica mix (throughput, p50/p99
latency of the served requests, each against the plain path and the plain
1024^3 kernel), and the CPU oracle timed on a bounded sample of the same
workload (on all host threads, and on one).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-flip events/s + achieved HBM GB/s at 1024^3, T=T_c; p50/p99 latency (served)"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed cycles")
    ap.add_argument("--warmup", type=int, default=50, help="untimed cycles before the timed region")
    ap.add_argument("--workload", default="headline", choices=["headline", "l512", "l512_sweep", "l128", "batch", "serve", "zeff"])
    ap.add_argument("--variant", default="", help="method variant bits by name, e.g. rmax_bound or two_colours|rmax_all")
    ap.add_argument("--zeff-L", type=int, default=512, help="zeff: lattice edge")
    ap.add_argument("--zeff-tmax", type=float, default=400.0, help="zeff: simulated time to reach")
    ap.add_argument("--replicas", type=int, default=256, help="batch / serve: lattices in the replica mix")
    ap.add_argument("--cycles", type=int, default=1000, help="batch / serve: cycles per lattice")
    ap.add_argument("--macro-cycles", type=int, default=100,
                    help="serve: cycles per macro-step; batch: cycles per eager or graph macro-step")
    ap.add_argument("--engine", default="auto", choices=["auto", "cycle", "persistent", "incremental", "slab"])
    ap.add_argument("--wg-domains", type=int, default=0)
    ap.add_argument("--obs-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mix", action="store_true", help="headline: skip the batched and served replica-mix legs")
    ap.add_argument("--cpu-cycles", type=int, default=0, help="oracle cycles for the CPU baseline (0 = auto)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="instead of the benchmark, copy this many MiB with a plain device copy (for counter scaling)")
    return ap.parse_args()


def workload(name):
    from paper_1005_4713_amd import workloads as W
    if name == "headline":
        return dict(W.HEADLINE_L1024)
    if name == "l512":
        return dict(W.LARGE_L512[2])
    return dict(W.MEDIUM_L128)


def calibrate_copy(mib):
    import torch
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": n, "copies": 3, "read_bytes_per_copy": n, "write_bytes_per_copy": n}))


def source_hash(names):
    """Hash of kernel sources with their comments and layout removed, so that an
    edit of comments alone does not retire a profile taken with that code."""
    import hashlib
    import re
    m = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        m.update(" ".join(text.split()).encode())
    return m.hexdigest()[:16]


def measured_traffic(workload_name, kernel, variant, steps):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary of this kernel and workload (each scaled by the reading of a plain
    copy of known size); None if there is none or the kernel source changed
    since the counters were taken."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json")):
        with open(path) as f:
            rec = json.load(f)
        if (rec.get("workload") != workload_name or rec.get("kernel") != kernel
                or rec.get("variant", "contract") != variant):
            continue
        if source_hash(rec["source_files"]) != rec["source_hash"]:
            return None, None
        rec["path"] = os.path.relpath(path, ROOT)
        return rec["hbm_bytes_per_cycle"] * steps, rec
    return None, None


def measured_valu(workload_name, kernel):
    """Vector-issue counters of this kernel and workload from the committed
    rocprofv3 SQ_INSTS_VALU / SQ_ACTIVE_INST_VALU summary; None if there is none
    or the kernel source changed since they were taken."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_valu.json")):
        with open(path) as f:
            rec = json.load(f)
        if rec.get("workload") != workload_name or rec.get("kernel") != kernel:
            continue
        if source_hash(rec["source_files"]) != rec["source_hash"]:
            return None
        return {"busy": rec["valu_busy"], "insts_per_wave_cycle": rec["valu_insts_per_wave_cycle"],
                "source": os.path.relpath(path, ROOT)}
    return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        return ""


def cpu_baseline(w, cycles, threads=1):
    """The oracle as it stands on a bounded sample of the workload: `cycles`
    spkMC cycles of the full lattice (initialisation not timed), its per-domain
    loops on `threads` host threads (1 = the plain serial loops; the trajectory
    is the same for every thread count)."""
    import oracle
    oracle.set_threads(threads)
    try:
        t0 = time.perf_counter()
        sim = oracle.Sim(L=w["L"], d=w["domain"], J=w["J"], H=w["H"], T=w["T"], seed=w["seed"],
                         rates=0 if w["rates"] == "glauber" else 1,
                         init={"random": 0, "up": 1, "down": 2}[w["init"]])
        t_init = time.perf_counter() - t0
        st0 = sim.state()
        t0 = time.perf_counter()
        sim.run(cycles)
        dt = time.perf_counter() - t0
        st1 = sim.state()
        del sim
    finally:
        oracle.set_threads(1)
    fired = st1[1] - st0[1]
    return {"value": fired / dt, "unit": "spin-flip events/s", "cores": oracle_threads_used(threads), "kind": "oracle",
            "host": {"cpu": _cpu_model(), "logical_cpus": os.cpu_count()},
            "sample": f"{cycles} cycles of the same L={w['L']} d={w['domain']} lattice from the same seed on "
                      f"{threads} thread(s) ({fired} events in {dt:.2f} s; initialisation {t_init:.1f} s not timed)",
            "attempts_per_s": (st1[1] + st1[2] - st0[1] - st0[2]) / dt}


def oracle_threads_used(threads):
    return max(1, min(int(threads), os.cpu_count() or 1))


def serial_bkl_baseline(events=2_500_000):
    """The oracle's serial rejection-free (BKL) simulator, single-threaded, at
    L = 128, T_c: the classic serial method, for reference beside the oracle's
    spkMC (a bounded number of events from a random start)."""
    import oracle
    b = oracle.Bkl(L=128, d=8, J=1.0, H=0.0, T=4.5115, seed=2)
    t0 = time.perf_counter()
    b.run(events)
    dt = time.perf_counter() - t0
    return {"value": events / dt, "unit": "spin-flip events/s", "cores": 1, "kind": "oracle serial BKL",
            "sample": f"{events} events of L=128, T=4.5115 from a random start in {dt:.2f} s"}


def _serve_run(spkmc, specs, doms, arrivals, pool_bytes, macro, max_live, log):
    """Submit request i at arrivals[i] seconds (real time) and step the server
    until every request is done; returns per-request latencies and totals."""
    srv = spkmc.Server(pool_bytes, macro_cycles=macro, max_live=max_live, inflight=2)
    n = len(specs)
    ids = [None] * n
    t0 = srv.clock()
    i = 0
    steps = 0
    while True:
        now = srv.clock() - t0
        while i < n and arrivals[i] <= now:
            sp = specs[i]
            ids[i] = srv.submit(sp["L"], doms[i], sp["cycles"], T=sp["T"], H=sp["H"], seed=sp["seed"],
                                t_arrival=t0 + arrivals[i], record_cap=0)
            i += 1
        st = srv.step(wait=False)
        steps += 1
        busy = st["queued"] or st["live"] or st["inflight"]
        if i == n and not busy:
            break
        if not busy and i < n:
            gap = arrivals[i] - (srv.clock() - t0)
            if gap > 2e-4:
                time.sleep(gap - 1e-4)
    res = [srv.poll(r) for r in ids]
    srv.close()
    lat = np.array([r["t_done"] - r["t_arrival"] for r in res])
    wait = np.array([r["t_admit"] - r["t_arrival"] for r in res])
    fired = sum(r["state_tuple"][1] for r in res)
    attempts = sum(r["state_tuple"][1] + r["state_tuple"][2] for r in res)
    span = max(r["t_done"] for r in res) - (t0 + float(arrivals[0]))
    out = {"requests": n, "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3),
           "admission_wait_p99_ms": float(np.percentile(wait, 99) * 1e3),
           "makespan_s": span, "events_per_s": fired / span, "attempts_per_s": attempts / span,
           "pool_bytes": pool_bytes, "pool_peak": st["pool_peak"], "macro_cycles": macro,
           "macro_steps": st["macro_steps"], "launches": st["launches"], "host_steps": steps}
    log(f"serve: {n} requests, p50 {out['p50_ms']:.2f} ms p99 {out['p99_ms']:.2f} ms, "
        f"makespan {span:.3f} s, pool peak {st['pool_peak'] / 2**20:.1f} MiB")
    return out, [r["state_tuple"] for r in res]


def replica_mix_legs(args, plain_kernel_events, log):
    """The batched and served forms on the replica mix (256 lattices, L in
    {32..256}, T in [4, 5], H in {0, +-0.05}, 1000 cycles each), each against
    the plain path (every lattice alone, one launch after another) and against
    the plain single-lattice kernel at 1024^3 of the same run; every batched and
    served lattice is checked bit for bit against its plain run."""
    import torch
    from paper_1005_4713_amd import spkmc, tune, workloads
    specs = workloads.replica_mix(args.replicas)
    for sp in specs:
        sp["cycles"] = args.cycles
    plan, table = tune.tune(specs, probe_cycles=20, log=log)
    doms = plan["domains"]
    log("bench: replica mix, plain path")
    solo = tune.build(specs, doms)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sim in solo:
        sim.run(args.cycles)
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t0
    plain = [sim.state() for sim in solo]
    del solo
    fired = sum(st[1] for st in plain)
    plain_rate = fired / dt_plain
    log("bench: replica mix, batched")
    sims = tune.build(specs, doms)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tune.run_plan(plan, sims, args.cycles)
    torch.cuda.synchronize()
    dt_batch = time.perf_counter() - t0
    batched = [sim.state() for sim in sims]
    del sims
    log("bench: replica mix, served (Poisson arrivals)")
    foot = sum((spkmc.state_bytes(spkmc.make_params(sp["L"], d)) + 255) // 256 * 256 for sp, d in zip(specs, doms))
    cap = int(200e9)
    served, st_served = _serve_run(spkmc, specs, doms, workloads.arrivals(len(specs), rate=50.0, seed=6),
                                   min(cap, foot), args.macro_cycles, 512, log)
    return {
        "batched": {"value": fired / dt_batch, "unit": "spin-flip events/s", "seconds": dt_batch,
                    "launches": len(plan["launches"]), "domains_policy": plan["policy"], "passes": plan["passes"],
                    "vs_plain_path": dt_plain / dt_batch, "vs_plain_1024_kernel": fired / dt_batch / plain_kernel_events,
                    "bit_identical_to_plain": batched == plain},
        "served": {"p50_ms": served["p50_ms"], "p99_ms": served["p99_ms"], "mean_ms": served["mean_ms"],
                   "max_ms": served["max_ms"], "events_per_s": served["events_per_s"],
                   "vs_plain_path": served["events_per_s"] / plain_rate,
                   "vs_plain_1024_kernel": served["events_per_s"] / plain_kernel_events,
                   "makespan_s": served["makespan_s"], "arrivals": "Poisson 50/s, seed 6",
                   "admission_cap_bytes": cap, "mix_footprint_bytes": foot, "macro_cycles": args.macro_cycles,
                   "bit_identical_to_plain": st_served == plain},
        "plain_path": {"value": plain_rate, "unit": "spin-flip events/s", "seconds": dt_plain,
                       "kind": "each lattice alone, one launch after another"},
        "workload": f"replica_mix_{len(specs)}x{args.cycles}_cycles",
    }


def bench_zeff(args):
    """Sec. 6 analysis (eqs. 16-17): magnetisation relaxation from all +1 at
    T_c, m(t) ~ t^(-beta / (nu z)); the effective exponent from the log-slope
    over sliding windows, z_eff = -(beta/nu) / (d ln m / d ln t), with the
    paper's beta/nu = 0.515.  Time in units of 1/lambda (lambda = 1)."""
    import torch
    from paper_1005_4713_amd import spkmc
    L = args.zeff_L
    d = 32 if L >= 1024 else 16
    sim = spkmc.Sim(L, d, layout="packed", init="up", T=4.5115, seed=77, variant=args.variant or 0,
                    record_cap=1 << 16)
    obs = 50 if L >= 1024 else 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chunk = 20000
    recs = []
    while sim.state()[3] < args.zeff_tmax:
        sim.run(chunk, obs_every=obs)
        recs += sim.records(chunk // obs)
        print(f"zeff: t = {sim.state()[3]:.1f}", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    t = np.array([r[3] for r in recs])
    m = np.array([r[4] for r in recs], dtype=np.float64) / float(L) ** 3
    beta_over_nu = 0.515
    windows = []
    lo = 1.0
    while lo * 2 <= t[-1]:
        sel = (t >= lo) & (t <= 2 * lo) & (m > 0)
        if sel.sum() >= 5:
            slope = np.polyfit(np.log(t[sel]), np.log(m[sel]), 1)[0]
            windows.append({"t_lo": lo, "t_hi": 2 * lo, "inv_t_mid": 1.0 / (1.5 * lo), "slope": slope,
                            "z_eff": -beta_over_nu / slope if slope < 0 else None})
        lo *= 2 ** 0.5
    st = sim.state()
    out = {"metric": "z_eff(t) from m(t) ~ t^(-beta/(nu z)), all +1 start at T_c", "value": windows[-1]["z_eff"],
           "unit": "dimensionless", "n_gpus": 1, "higher_is_better": None, "data": "synthetic", "dtype": "u32+f64",
           "config": {"workload": f"L{L}_d{d}_packed_Tc_up", "variant": args.variant or "contract",
                      "beta_over_nu": beta_over_nu, "cycles": st[0], "t_end": st[3]},
           "wall_s": wall, "events_per_s": st[1] / wall, "windows": windows,
           "m_t": [[float(a), float(b)] for a, b in zip(t[::max(1, len(t) // 200)], m[::max(1, len(m) // 200)])]}
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """The replica mix served as requests: Poisson arrivals at 50/s (seed 6)
    into the request server with the admission cap at 200 GB (the whole mix
    needs far less, so it never binds: the pool is the mix's total footprint);
    the same mix arriving at once; and at once under a 16 MiB cap, which makes
    admission wait for memory.  Latency = completion seen by the host minus
    arrival.  Every served result is checked against the plain path."""
    import torch
    from paper_1005_4713_amd import spkmc, tune, workloads
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    specs = workloads.replica_mix(args.replicas)
    for sp in specs:
        sp["cycles"] = args.cycles
    plan, _ = tune.tune(specs, probe_cycles=20, log=log)
    doms = plan["domains"]
    foot = sum((spkmc.state_bytes(spkmc.make_params(sp["L"], d)) + 255) // 256 * 256 for sp, d in zip(specs, doms))
    cap = int(200e9)
    arr = workloads.arrivals(len(specs), rate=50.0, seed=6)
    # plain path: each lattice alone, in turn
    solo = tune.build(specs, doms)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in solo:
        s.run(args.cycles)
    torch.cuda.synchronize()
    dt_solo = time.perf_counter() - t1
    plain_states = [s.state() for s in solo]
    del solo
    fired_plain = sum(s[1] for s in plain_states)
    macro = args.macro_cycles
    poisson, st_p = _serve_run(spkmc, specs, doms, arr, min(cap, foot), macro, 512, log)
    burst, st_b = _serve_run(spkmc, specs, doms, np.zeros(len(specs)), min(cap, foot), macro, 512, log)
    capped, st_c = _serve_run(spkmc, specs, doms, np.zeros(len(specs)), 16 << 20, macro, 512, log)
    same = st_p == plain_states and st_b == plain_states and st_c == plain_states
    out = {"metric": "served replica mix: p50/p99 latency", "value": poisson["p99_ms"], "unit": "ms (p99)",
           "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "u32+f64",
           "config": {"workload": f"replica_mix_{args.replicas}_served", "cycles": args.cycles,
                      "arrivals": "Poisson 50/s, seed 6", "admission_cap_bytes": cap, "mix_footprint_bytes": foot,
                      "domains_policy": plan["policy"]},
           "p50_ms": poisson["p50_ms"], "p99_ms": poisson["p99_ms"],
           "poisson_50_per_s": poisson, "burst": burst, "burst_cap_16MiB": capped,
           "plain": {"events_per_s": fired_plain / dt_solo, "seconds": dt_solo, "kind": "each lattice alone, in turn"},
           "burst_vs_plain": burst["events_per_s"] / (fired_plain / dt_solo),
           "bit_identical_to_plain": same}
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """The replica mix (L in {32..256}, T in [4, 5], H in {0, +-0.05}, 1000 cycles
    each) run as tuned batched launches, against the plain single-lattice path
    (every lattice alone, one launch per lattice, one after another)."""
    import torch
    from paper_1005_4713_amd import spkmc, tune, workloads
    specs = workloads.replica_mix(args.replicas)
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    plan, table = tune.tune(specs, probe_cycles=20, log=log)
    sims = tune.build(specs, plan["domains"])
    torch.cuda.synchronize()
    s0 = [s.state() for s in sims]
    t0 = time.perf_counter()
    tune.run_plan(plan, sims, args.cycles)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s1 = [s.state() for s in sims]
    fired = sum(b[1] - a[1] for a, b in zip(s0, s1))
    attempts = sum(b[1] + b[2] - a[1] - a[2] for a, b in zip(s0, s1))
    del sims
    # plain path: the same lattices, one at a time
    solo = tune.build(specs, plan["domains"])
    torch.cuda.synchronize()
    q0 = [s.state() for s in solo]
    t1 = time.perf_counter()
    for s in solo:
        s.run(args.cycles)
    torch.cuda.synchronize()
    dt_solo = time.perf_counter() - t1
    q1 = [s.state() for s in solo]
    fired_solo = sum(b[1] - a[1] for a, b in zip(q0, q1))
    same = all(a == b for a, b in zip(s1, q1))
    del solo
    # macro-steps of `macro` cycles: eager batch launches, then the same steps as
    # batch graphs captured once and replayed
    macro = args.macro_cycles
    timed = {}
    for kind in ("eager", "graph"):
        sims = tune.build(specs, plan["domains"])
        torch.cuda.synchronize()
        a0 = [s.state() for s in sims]
        tk = time.perf_counter()
        if kind == "eager":
            tune.run_plan(plan, sims, args.cycles, macro=macro)
        else:
            graphs = tune.run_plan_graph(plan, sims, args.cycles, macro)
        torch.cuda.synchronize()
        secs = time.perf_counter() - tk
        if kind == "graph":
            for g in graphs:
                g.close()
        a1 = [s.state() for s in sims]
        timed[kind] = {"value": sum(b[1] - a[1] for a, b in zip(a0, a1)) / secs, "seconds": secs,
                       "bit_identical_to_plain": all(a == b for a, b in zip(a1, q1))}
        del sims
    out = {"metric": "spin-flip events/s, batched replica mix", "value": fired / dt, "unit": "spin-flip events/s",
           "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "u32+f64",
           "config": {"workload": f"replica_mix_{args.replicas}", "cycles": args.cycles,
                      "domains_policy": plan["policy"], "passes": plan["passes"],
                      "launches": len(plan["launches"]),
                      "sites": sum(sp["L"] ** 3 for sp in specs)},
           "seconds": dt, "attempts_per_s": attempts / dt,
           "plain": {"value": fired_solo / dt_solo, "seconds": dt_solo, "kind": "each lattice alone, in turn"},
           "speedup_vs_plain": (fired / dt) / (fired_solo / dt_solo), "bit_identical_to_plain": same,
           "macro_steps": {"cycles_per_step": macro, "eager_batches": timed["eager"],
                           "batch_graphs": timed["graph"]},
           "tuner": table}
    print(json.dumps(out), flush=True)


def bench_l512_sweep(args):
    """The L = 512, d = 16 sweep: three temperatures around T_c, both rate
    families, both starts, 2000 cycles each with a record every 10.  Per
    configuration: throughput, UR, and from the records of cycles 1001-2000 the
    moments of m = M/N: <|m|>, Q = <m^4>/<m^2>^2 and 1 - Q/3 (the ratio the paper
    prints for U4 and the cumulant it says goes to 0 at low T)."""
    import numpy as np
    import torch
    from paper_1005_4713_amd import spkmc, workloads
    rows = []
    for w in workloads.LARGE_L512:
        print(f"bench: {w['name']}", file=sys.stderr, flush=True)
        sim = spkmc.Sim(w["L"], w["domain"], J=w["J"], H=w["H"], T=w["T"], seed=w["seed"], rates=w["rates"],
                        init=w["init"], layout=w["layout"], record_cap=w["cycles"] // w["obs_every"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(w["cycles"], obs_every=w["obs_every"])
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        st = sim.state()
        recs = [r for r in sim.records() if r[0] > w["cycles"] // 2]
        m = np.array([r[4] for r in recs], dtype=np.float64) / float(w["L"]) ** 3
        m2, m4 = float(np.mean(m ** 2)), float(np.mean(m ** 4))
        q = m4 / (m2 * m2) if m2 > 0 else float("nan")
        rows.append({"name": w["name"], "T": w["T"], "rates": w["rates"], "init": w["init"],
                     "engine": ["auto", "cycle", "persistent", "incremental", "slab"][sim.info()["engine"]],
                     "flips_per_s": st[1] / secs, "us_per_cycle": secs / w["cycles"] * 1e6,
                     "ur": st[1] / max(st[1] + st[2], 1), "t_end": st[3], "abs_m": float(np.mean(np.abs(m))),
                     "Q": q, "one_minus_Q_over_3": 1.0 - q / 3.0, "records_used": len(recs)})
        del sim
    total_flips = sum(r["flips_per_s"] * r["us_per_cycle"] * 1e-6 * 2000 for r in rows)
    total_secs = sum(r["us_per_cycle"] * 1e-6 * 2000 for r in rows)
    print(json.dumps({"metric": "L=512 d=16 sweep: spin-flip events/s over 12 runs of 2000 cycles; Q per run",
                      "value": total_flips / total_secs, "unit": "spin-flip events/s", "n_gpus": 1,
                      "higher_is_better": True, "data": "synthetic", "dtype": "u32+f64",
                      "config": {"workload": "L512_d16_sweep", "runs": len(rows), "cycles": 2000, "obs_every": 10},
                      "runs": rows}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    from paper_1005_4713_amd import spkmc

    if args.workload == "batch":
        torch.cuda.set_device(0)
        bench_batch(args)
        return
    if args.workload == "serve":
        torch.cuda.set_device(0)
        bench_serve(args)
        return
    if args.workload == "zeff":
        torch.cuda.set_device(0)
        bench_zeff(args)
        return
    if args.workload == "l512_sweep":
        torch.cuda.set_device(0)
        bench_l512_sweep(args)
        return
    w = workload(args.workload)
    torch.cuda.set_device(0)
    print(f"bench: workload {w['name']} engine={args.engine} warmup={args.warmup} steps={args.steps}",
          file=sys.stderr, flush=True)
    sim = spkmc.Sim(w["L"], w["domain"], J=w["J"], H=w["H"], T=w["T"], seed=w["seed"], rates=w["rates"],
                    init=w["init"], layout=w["layout"], engine=args.engine, wg_domains=args.wg_domains,
                    variant=args.variant or 0,
                    record_cap=max(1, (args.warmup + args.steps) // max(args.obs_every, 1) + 1))
    info = sim.info()
    stream = sim.stream
    torch.cuda.synchronize()
    if args.warmup:
        sim.run(args.warmup, obs_every=args.obs_every)
    torch.cuda.synchronize()
    s0 = sim.state()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.run(args.steps, obs_every=args.obs_every)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    s1 = sim.state()
    fired = s1[1] - s0[1]
    nulls = s1[2] - s0[2]
    secs = gpu_ms / 1e3
    value = fired / secs
    bytes_cycle = info["bytes_per_cycle"]
    launches = 1 if info["engine"] in (spkmc.ENGINES["persistent"], spkmc.ENGINES["incremental"],
                                       spkmc.ENGINES["slab"]) else 3 * args.steps
    achieved = bytes_cycle * args.steps / secs / 1e9
    inc = info["engine"] == spkmc.ENGINES["incremental"]
    lpd = 4 if sim.params.variant & spkmc.VARIANTS["two_colours"] else 1
    passes = info["wg_domains"] * 16 // info["block"] if info["block"] else 0
    bnd = int(bool(sim.params.variant & spkmc.VARIANTS["rmax_bound"]) and not inc)  # the bound compiled in
    kernel = (f"k_persistent<{info['h']}, {passes}, {info['block']}, "
              f"{str(inc).lower()}, {lpd}, {bnd}>" if launches == 1 else "whole cycle (3 launches)")
    if launches == 1 and passes > 4:  # the wide mode: rounds of four passes
        kernel = f"k_persistent_wide<{passes // 4}, {lpd}, {bnd}>"
    if info["engine"] == spkmc.ENGINES["slab"]:
        kernel = f"k_slab<{str(bool(sim.params.variant & spkmc.VARIANTS['rmax_all'])).lower()}>"
    traffic, traffic_rec = (None, None)
    if launches == 1:
        traffic, traffic_rec = measured_traffic(w["name"], kernel, args.variant or "contract", args.steps)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spin-flip events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32+f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "L": w["L"], "domain": w["domain"], "T": w["T"], "J": w["J"],
                   "H": w["H"], "rates": w["rates"], "init": w["init"], "seed": w["seed"],
                   "layout": w["layout"], "engine": ["auto", "cycle", "persistent", "incremental", "slab"][info["engine"]],
                   "grid": info["grid"], "block": info["block"], "wg_domains": info["wg_domains"],
                   "K": info["K"], "h": info["h"], "obs_every": args.obs_every,
                   "variant": args.variant or "contract"},
        "attempts_per_s": (fired + nulls) / secs,
        "ur": fired / max(fired + nulls, 1),
        "wall_s": wall,
        "sim_time": [s0[3], s1[3]],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel,
                     "bytes_per_cycle": bytes_cycle, "launches": launches,
                     "avg_launch_ms": gpu_ms / launches,
                     "traffic_source": None if traffic is None else traffic_rec["path"],
                     "valu": measured_valu(w["name"], kernel) if launches == 1 and not args.variant else None,
                     # the lower bound of the bytes a cycle must move: the active octants'
                     # own bits only (class masks without a halo), K l h^3 / 8 (l active octants per domain)
                     "frac_lower_bound_bytes": (info["K"] * lpd * info["h"] ** 3 / 8.0) * args.steps / secs / 1e9
                     / HBM_PEAK_GBS},
    }
    del sim
    torch.cuda.synchronize()
    if args.workload == "headline" and not args.no_mix:
        log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
        out["replica_mix"] = replica_mix_legs(args, value, log)
    if not args.no_cpu_baseline:
        cyc = args.cpu_cycles or (12 if w["L"] >= 1024 else 80 if w["L"] >= 512 else 4000)
        nthr = min(16, os.cpu_count() or 1)
        print(f"bench: cpu baseline, {3 * cyc} oracle cycles on {nthr} threads", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, 3 * cyc, threads=nthr)
        print(f"bench: cpu baseline, {cyc} oracle cycles on one thread", file=sys.stderr, flush=True)
        out["cpu_baseline"]["single_thread"] = cpu_baseline(w, cyc, threads=1)
        out["cpu_baseline"]["serial_bkl"] = serial_bkl_baseline()
    print(json.dumps(out), flush=True)


def _shutdown():
    """Release every device object of the library and wait for the device
    before the interpreter exits (nothing is left for exit-time handlers)."""
    import gc
    import torch
    from paper_1005_4713_amd import spkmc
    gc.collect()
    spkmc.release_cached()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
    if "torch" in sys.modules and sys.modules["torch"].cuda.is_initialized():
        _shutdown()
