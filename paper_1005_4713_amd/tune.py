"""Launch planner and autotuner for batches of independent lattices.

A batch launch holds lattices of one octant edge h (8 or 16, domain 16 or 32)
and must fit on the device at once: lattice i takes ceil(K_i / (rows * P))
workgroups (rows = 64 domains per pass for h = 8, 32 for h = 16; P passes per
workgroup), one workgroup per CU at most.  The tuner chooses

* the domain size of each lattice (16, or 32 where L allows it),
* the passes per workgroup P of each launch (1, 2 or 4: more passes pack more
  domains, hence more small lattices, onto each CU),

by timing short probe runs of every candidate plan on throw-away copies of the
lattices (objective: event attempts, i.e. domain-cycles, per second), and packs
the lattices into launches first-fit by decreasing size.
Changing the domain size changes a lattice's trajectory (it is a parameter of
the method); the launch shape never does.
"""
import time

import torch

from . import spkmc

ROWS = {8: 64, 16: 32}
MAX_PASSES = {8: 2, 16: 4}  # batches of octant edge 8 stop at two passes (registers)


def domain_choices(L):
    return [d for d in (16, 32) if L % d == 0]


def wgs(L, d, P):
    K = (L // d) ** 3
    D = ROWS[d // 2] * P
    return -(-K // D)


def pack(items, capacity):
    """items: (index, workgroups); first-fit decreasing into bins of `capacity`."""
    bins = []
    for idx, w in sorted(items, key=lambda x: -x[1]):
        if w > capacity:
            raise ValueError(f"lattice {idx} needs {w} workgroups, more than fit at once ({capacity})")
        for b in bins:
            if b["wgs"] + w <= capacity:
                b["members"].append(idx)
                b["wgs"] += w
                break
        else:
            bins.append({"members": [idx], "wgs": w})
    return bins


def make_plan(specs, policy, passes, capacity):
    """policy: 16 (every lattice on domains of 16) or 32 (32 where L allows);
    passes: {h: P}.  Returns the domain of each lattice and the launches."""
    doms = []
    for sp in specs:
        ch = domain_choices(sp["L"])
        doms.append(32 if policy == 32 and 32 in ch else 16)
    launches = []
    for h in (8, 16):
        idx = [i for i, d in enumerate(doms) if d // 2 == h]
        if not idx:
            continue
        P = min(passes[h], MAX_PASSES[h])
        for b in pack([(i, wgs(specs[i]["L"], doms[i], P)) for i in idx], capacity):
            launches.append({"h": h, "P": P, "wg_domains": ROWS[h] * P, "members": b["members"], "wgs": b["wgs"]})
    return {"policy": policy, "passes": {h: min(P, MAX_PASSES[h]) for h, P in passes.items()}, "domains": doms,
            "launches": launches}


def build(specs, doms, record_cap=0, device=None):
    return [spkmc.Sim(sp["L"], d, J=sp.get("J", 1.0), H=sp["H"], T=sp["T"], seed=sp["seed"],
                      rates=sp.get("rates", "glauber"), init=sp.get("init", "random"), layout="packed",
                      engine="persistent", record_cap=record_cap, device=device)
            for sp, d in zip(specs, doms)]


def run_plan(plan, sims, ncycles, obs_every=0, macro=None):
    """Run every lattice `ncycles` cycles with the plan's launches (each launch
    in macro-steps of `macro` cycles, or all at once)."""
    for ln in plan["launches"]:
        members = [sims[i] for i in ln["members"]]
        left = ncycles
        while left > 0:
            step = left if macro is None else min(macro, left)
            spkmc.run_batch(members, step, obs_every=obs_every, wg_domains=ln["wg_domains"])
            left -= step


def run_plan_graph(plan, sims, ncycles, macro, obs_every=0):
    """The plan's launches as batch graphs of one `macro`-cycle macro-step each,
    every graph replayed ncycles // macro times (ncycles a multiple of macro);
    returns the graphs, which the caller closes once the replays are done."""
    if ncycles % macro:
        raise ValueError("ncycles must be a multiple of macro")
    graphs = [spkmc.BatchGraph([sims[i] for i in ln["members"]], macro, obs_every=obs_every,
                               wg_domains=ln["wg_domains"]) for ln in plan["launches"]]
    for g in graphs:
        g.launch(ncycles // macro)
    return graphs


def capacity():
    return torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count


def tune(specs, probe_cycles=20, policies=(16, 32), pass_options=(1, 2, 4), log=None):
    """Time every (domain policy, passes) candidate on throw-away lattices and
    return the fastest plan with the measurements."""
    cap = capacity()
    results = []
    for policy in policies:
        base = make_plan(specs, policy, {8: 1, 16: 1}, cap)
        sims = build(specs, base["domains"])
        torch.cuda.synchronize()
        for P in pass_options:
            try:
                plan = make_plan(specs, policy, {8: P, 16: P}, cap)
            except ValueError:
                continue
            run_plan(plan, sims, 2)  # warm the kernels of this shape
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run_plan(plan, sims, probe_cycles)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            attempts = probe_cycles * sum((sp["L"] // d) ** 3 for sp, d in zip(specs, plan["domains"]))
            rate = sum(sp["L"] ** 3 for sp in specs) * probe_cycles / dt  # sites swept per second
            results.append({"policy": policy, "P": P, "seconds": dt, "launches": len(plan["launches"]),
                            "attempts_per_s": attempts / dt, "site_cycles_per_s": rate, "plan": plan})
            if log:
                log(f"tune: domains {policy} passes {P}: {len(plan['launches'])} launches, "
                    f"{dt * 1e3:.2f} ms for {probe_cycles} cycles")
        del sims
    # the plan with the most event attempts (domain-cycles) per second: a cycle
    # of a lattice on domains of 32 does an eighth of the attempts of one on 16
    best = max(results, key=lambda r: r["attempts_per_s"])
    return best["plan"], [{k: v for k, v in r.items() if k != "plan"} for r in results]
