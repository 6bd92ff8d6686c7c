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
bytes), and the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-flip events/s + achieved HBM GB/s at 1024^3, T=T_c; p50/p99 latency (served)"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed cycles")
    ap.add_argument("--warmup", type=int, default=50, help="untimed cycles before the timed region")
    ap.add_argument("--workload", default="headline", choices=["headline", "l512", "l128", "batch", "serve"])
    ap.add_argument("--replicas", type=int, default=256, help="batch / serve: lattices in the replica mix")
    ap.add_argument("--cycles", type=int, default=1000, help="batch / serve: cycles per lattice")
    ap.add_argument("--engine", default="auto", choices=["auto", "cycle", "persistent"])
    ap.add_argument("--wg-domains", type=int, default=0)
    ap.add_argument("--obs-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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


def measured_traffic(workload_name, steps):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary of this kernel and workload (each scaled by the reading of a plain
    copy of known size); None if there is none or the kernel source changed
    since the counters were taken."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json")):
        with open(path) as f:
            rec = json.load(f)
        if rec.get("workload") != workload_name:
            continue
        m = hashlib.sha256()
        for name in rec["source_files"]:
            with open(os.path.join(ROOT, name), "rb") as f:
                m.update(f.read())
        if m.hexdigest()[:16] != rec["source_hash"]:
            return None, None
        return rec["hbm_bytes_per_cycle"] * steps, rec
    return None, None


def cpu_baseline(w, cycles):
    """The oracle as it stands, single-threaded, on a bounded sample of the
    workload: `cycles` spkMC cycles of the full lattice (initialisation not timed)."""
    import oracle
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
    fired = st1[1] - st0[1]
    return {"value": fired / dt, "unit": "spin-flip events/s", "cores": 1, "kind": "oracle",
            "sample": f"{cycles} cycles of the same L={w['L']} d={w['domain']} lattice from the same seed "
                      f"({fired} events in {dt:.2f} s; initialisation {t_init:.1f} s not timed)",
            "attempts_per_s": (st1[1] + st1[2] - st0[1] - st0[2]) / dt}


def bench_serve(args):
    raise SystemExit("serving benchmark not built yet")


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
    out = {"metric": "spin-flip events/s, batched replica mix", "value": fired / dt, "unit": "spin-flip events/s",
           "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "u32+f64",
           "config": {"workload": f"replica_mix_{args.replicas}", "cycles": args.cycles,
                      "domains_policy": plan["policy"], "passes": plan["passes"],
                      "launches": len(plan["launches"]),
                      "sites": sum(sp["L"] ** 3 for sp in specs)},
           "seconds": dt, "attempts_per_s": attempts / dt,
           "plain": {"value": fired_solo / dt_solo, "seconds": dt_solo, "kind": "each lattice alone, in turn"},
           "speedup_vs_plain": (fired / dt) / (fired_solo / dt_solo), "bit_identical_to_plain": same,
           "tuner": table}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus above 1 is not supported",
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
    w = workload(args.workload)
    torch.cuda.set_device(0)
    print(f"bench: workload {w['name']} engine={args.engine} warmup={args.warmup} steps={args.steps}",
          file=sys.stderr, flush=True)
    sim = spkmc.Sim(w["L"], w["domain"], J=w["J"], H=w["H"], T=w["T"], seed=w["seed"], rates=w["rates"],
                    init=w["init"], layout=w["layout"], engine=args.engine, wg_domains=args.wg_domains,
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
    launches = 1 if info["engine"] == spkmc.ENGINES["persistent"] else 3 * args.steps
    achieved = bytes_cycle * args.steps / secs / 1e9
    traffic, traffic_rec = (None, None)
    if launches == 1:
        traffic, traffic_rec = measured_traffic(w["name"], args.steps)
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
                   "layout": w["layout"], "engine": ["auto", "cycle", "persistent"][info["engine"]],
                   "grid": info["grid"], "block": info["block"], "wg_domains": info["wg_domains"],
                   "K": info["K"], "h": info["h"], "obs_every": args.obs_every},
        "attempts_per_s": (fired + nulls) / secs,
        "ur": fired / max(fired + nulls, 1),
        "wall_s": wall,
        "sim_time": [s0[3], s1[3]],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "spkmc_persistent" if launches == 1 else "whole cycle (3 launches)",
                     "bytes_per_cycle": bytes_cycle, "launches": launches,
                     "avg_launch_ms": gpu_ms / launches,
                     "traffic_source": None if traffic is None else "profiles/persistent_L1024_d32_traffic.json"},
    }
    if not args.no_cpu_baseline:
        cyc = args.cpu_cycles or (3 if w["L"] >= 1024 else 20 if w["L"] >= 512 else 2000)
        print(f"bench: cpu baseline, {cyc} oracle cycles", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, cyc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
