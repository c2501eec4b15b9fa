"""Throughput of the particle-in-cell joint PDF step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload canyon1m|canyon10m|square40k]

One step = one pass of the whole hot path over every particle: statistics of
each element (means, Reynolds stresses, scalar moments, velocity-binned
<phi|V>), IECM, Langevin velocity, position, tracking with wall/periodic
conditions, source, re-binning into element segments.  Inputs are resident in
HBM before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s

WORKLOADS = {
    "canyon1m": ("config2", "street canyon, 9912-element Delaunay mesh, 1M particles, GLM, FP32 state"),
    "batched64": ("config4", "64 independent canyon runs on the 9912-element mesh, 12.2M particles in total "
                             "(10k-1M per run, log-uniform), distinct seeds and sources"),
    "canyon10m": ("config3", "wall-function canyon, 48618-element mesh, 10M particles, SLM, 4th moments + histograms"),
    "canyon10m_omega": ("config3w", "wall-function canyon, 48618-element mesh, 10M particles, SLM, 4th moments + "
                                    "histograms, stochastic turbulent frequency per particle"),
    "canyon10m_bins5": ("config3b", "wall-function canyon, 48618-element mesh, 10M particles, SLM, 4th moments + "
                                    "histograms, <phi|V> on 5x5x5 velocity bins"),
    "square40k": ("config1", "unit square 20x20x2, 40k particles, SLM, FP64"),
}


# Workloads whose configuration fixes the step count (the square case: 100 steps).
FIXED_STEPS = {"square40k": 100}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1003_4548_amd", "csrc")
    for fn in sorted(os.listdir(d)):
        if fn.endswith((".hip", ".hpp")):
            with open(os.path.join(d, fn), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(wl) -> dict:
    """Bytes one step must move at minimum in this design.

    Per particle: read x y u v w psi id (and omega when carried), write the
    same.  Per element cell: the statistics record written, the cell's
    start/capacity/count/rate words, its mesh record and an even share of the
    vertex coefficient table.
    """
    ts = 4 if wl.precision == "f32" else 8
    om = bool(getattr(wl, "omega", False))
    per_particle = 2 * ((7 if om else 6) * ts + 4)
    nstat = (86 if wl.moments >= 4 else 31) + wl.hist_bins + (3 if om else 0) + \
        (250 if getattr(wl, "vbins", 2) == 5 else 0)
    ne, nv = wl.mesh.nelem, wl.mesh.nvert
    ncell = ne * wl.nens
    per_cell = nstat * 8 + 4 * 4 + ts
    per_mesh = ne * (3 * 4 * 3 + 8 + 3 * 8 + (8 if om else 0)) + nv * (2 * 8 + 16 * ts)
    n = wl.n_total
    total = n * per_particle + ncell * per_cell + per_mesh
    return dict(per_particle=per_particle, per_cell=per_cell, per_step=total, particles=n)


def scope_bytes(wl) -> dict:
    """The scope table's algorithmic bytes per particle-step: one read of the
    particle state (x y u v w psi, element, id, and omega when carried), one write of
    its mutable part (x y u v w psi, element, and omega), one re-read of the
    statistics inputs (u v w psi, element, and omega); per element cell and
    mesh the same amortised terms as the design count."""
    ts = 4 if wl.precision == "f32" else 8
    om = 1 if getattr(wl, "omega", False) else 0
    # read: 6 (+1) state values, element and id; write: 6 (+1) values and the
    # element; re-read: u v w psi (+omega) and the element (f32: 32 + 28 + 20)
    per_particle = ((6 + om) * ts + 8) + ((6 + om) * ts + 4) + ((4 + om) * ts + 4)
    d = algorithmic_bytes(wl)
    n = wl.n_total
    amort = d["per_step"] - n * d["per_particle"]
    return dict(per_particle=per_particle, per_step=n * per_particle + amort,
                per_particle_with_amortised=round((n * per_particle + amort) / max(1, n), 2))


def host_cpu() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"host_cpus": os.cpu_count(), "cpu_model": model}


def read_profile(kind: str, workload: str, src_hash: str) -> dict:
    """Figures of a committed rocprofv3 summary ("key value" lines), if it was
    taken on the current kernel source; {} otherwise."""
    fn = os.path.join(ROOT, "profiles", f"{kind}_k_step_{workload}.txt")
    if not os.path.exists(fn):
        return {}
    vals = {}
    for line in open(fn):
        if line.startswith("#"):
            continue
        parts = line.replace(":", " ").split()
        if len(parts) == 2:
            vals[parts[0]] = parts[1]
    return vals if vals.get("kernel_source_hash") == src_hash else {}


def read_traffic(workload: str, src_hash: str):
    """HBM bytes per step of the step kernel from the calibrated counters."""
    try:
        return float(read_profile("hbm_traffic", workload, src_hash)["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wavefront-instruction
# (64 lanes on a 16-lane SIMD) every 4 cycles
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4


def read_valu(workload: str, src_hash: str):
    """VALU wavefront-instructions per step of the step kernel (SQ_INSTS_VALU)."""
    try:
        return float(read_profile("valu", workload, src_hash)["valu_wave_instructions_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(wl_fn, seconds: float = 15.0) -> dict:
    """The oracle on the host cores, on a bounded sample of the same workload:
    the full particle set, as many whole steps as fit in about `seconds`."""
    import oracle as O
    # a one-GPU job is allotted 16 host CPUs, whatever os.cpu_count() reports;
    # on a smaller host all of its cores
    threads = min(16, os.cpu_count() or 1)
    wl = wl_fn()
    orc = O.Oracle(wl, threads=threads)
    orc.step(1)                       # warm caches; the first step is not timed
    steps = 0
    t0 = time.perf_counter()
    while True:
        orc.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 2000:
            break
    n = wl.n_total
    res = {"value": n * steps / el, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
           "sample": f"{wl.name}: all {n} particles, {steps} steps after one untimed step, {el:.1f} s",
           "threads_note": "OpenMP threads = min(16, host CPUs): a one-GPU job is allotted 16 host CPUs",
           **host_cpu()}
    # one host thread on the same state, a few seconds
    O.lib().orc_set_threads(1)
    orc.step(1)
    s1 = 0
    t0 = time.perf_counter()
    while True:
        orc.step(1)
        s1 += 1
        el1 = time.perf_counter() - t0
        if el1 >= seconds / 3 or s1 >= 200:
            break
    res["single_thread"] = {"value": n * s1 / el1, "steps": s1, "seconds": round(el1, 1)}
    O.lib().orc_set_threads(threads)
    return res


def learned_leg(torch, W, Simulation) -> dict:
    """The learned conditional means on the 10k-element canyon with its street
    source.  Training rows: 20-particle subsamples of runs at 500 particles per
    element (seeds 1..4), taken every 100 steps from step 500 to 2000, eight
    draws each, the rows with scalar spread kept.  Compared with a run at
    4000 particles per element (seed 101) at the same steps, next to the
    binned estimate of 20- and 500-particle subsamples.  Then used inside the
    step of a 20-particle-per-element run on the 50k-element resolved-wall
    mesh."""
    from paper_1003_4548_amd import mlp as PM
    t_start = time.perf_counter()
    spin, every, snaps, draws = 500, 100, 16, 8

    rows = []
    for seed in (1, 2, 3, 4):
        sim = Simulation.from_workload(W.config5(ppe=500, seed=seed), device="cuda:0")
        sim.step_graph(spin)
        for k in range(snaps):
            if k:
                sim.step_graph(every)
            for d in range(draws):
                r = PM.dataset(sim, target=20, key=1000 + seed, draw=draws * k + d)
                rows.append(r[r[:, 40:48].sum(dim=1) > 0])
        sim.sync()
        sim.close()
    rows = torch.cat(rows)
    nrows = int(rows.shape[0])
    print(f"[bench] learned: {nrows} training rows", file=sys.stderr, flush=True)
    net = PM.ConditionalMeanNet(seed=0)
    net.fit_norm(rows)
    iters, batch = 6000, 2048
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(net.stream)
    loss = net.train(rows, iters=iters, batch=batch, lr=2e-3, seed=7)
    e1.record(net.stream)
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    loss = loss.cpu().numpy()
    del rows
    # compared with 4000 particles per element
    sim = Simulation.from_workload(W.config5(ppe=4000, seed=101), device="cuda:0")
    sim.step_graph(spin)
    r20, r500 = [], []
    sizes = (20, 40, 80, 160, 320, 500, 1000)
    rsz = {t: [] for t in sizes}
    for k in range(snaps):
        if k:
            sim.step_graph(every)
        r20.append(PM.dataset(sim, target=20, key=5555, draw=k))
        r500.append(PM.dataset(sim, target=500, key=6666, draw=k))
        for t in sizes:
            rsz[t].append(PM.dataset(sim, target=t, key=7777 + t, draw=k))
    sim.sync()
    sim.close()
    r20 = torch.cat(r20)
    r500 = torch.cat(r500)
    plain_by_size = {t: PM.estimate_error(torch.cat(rsz[t])) for t in sizes}
    del rsz
    rec = PM.records_from_rows(r20)
    cm, _ = net.infer(rec)
    domain = (r20[:, 0] > 0) & (r20[:, 31] > 1e-4)
    took = (cm != rec[:, 23:31]).any(dim=1)
    err = {"plain_20": PM.estimate_error(r20), "learned_20": PM.estimate_error(r20, cm),
           "plain_500": PM.estimate_error(r500)}
    served_frac = float((took & domain).sum()) / max(1, int(domain.sum()))
    n_domain = int(domain.sum())
    del r20, r500, rec, cm
    torch.cuda.empty_cache()
    # inside the step: 20 particles per element on the 50k-element resolved-wall canyon
    wl = W.config5(ppe=20, seed=101, target=50000)
    sim = Simulation.from_workload(wl, device="cuda:0")
    in_step_shape = sim.autotune(steps_per_trial=8)
    if in_step_shape[1]:
        in_step_shape = (in_step_shape[0], 0)      # the learned means run inside one-item-per-wavefront steps
        sim.set_launch(*in_step_shape)
    sim.step_graph(spin)
    steps = 200
    sim.sync()
    t0 = time.perf_counter()
    sim.step_graph(steps)
    sim.sync()
    plain_s = time.perf_counter() - t0
    lm = net.attach(sim)
    sim.step_graph(12)
    sim.sync()
    lm.served.zero_()
    t0 = time.perf_counter()
    sim.step_graph(steps)
    sim.sync()
    mlp_s = time.perf_counter() - t0
    st = sim.statistics_device()[0]
    in_domain = int(((st[:, 0] > 0) & (st[:, 14] > 1e-8)).sum())
    inloop_served = int(lm.served.cpu()[0]) / (steps * max(1, in_domain))
    lm.detach()
    sim.close()
    n, E = wl.n_total, wl.mesh.nelem
    # the subsample size at which the plain binned estimate reaches the
    # learned estimate's error (log-log interpolation between measured sizes)
    import math
    eq_ppe = None
    le = err["learned_20"]
    for a, b in zip(sizes[:-1], sizes[1:]):
        ea, eb = plain_by_size[a], plain_by_size[b]
        if ea >= le >= eb:
            f = (math.log(ea) - math.log(le)) / max(1e-30, math.log(ea) - math.log(eb))
            eq_ppe = round(math.exp(math.log(a) + f * (math.log(b) - math.log(a))), 1)
            break
    eq_res = None
    if eq_ppe is not None:
        # the plain step at that count on the same mesh, next to the learned step at 20
        wq = W.config5(ppe=int(round(eq_ppe)), seed=101, target=50000)
        sq = Simulation.from_workload(wq, device="cuda:0")
        shq = sq.autotune(steps_per_trial=8)
        sq.step_graph(20)
        sq.sync()
        t0 = time.perf_counter()
        sq.step_graph(steps)
        sq.sync()
        eq_s = time.perf_counter() - t0
        sq.close()
        eq_res = {"ppe": int(round(eq_ppe)), "particles": wq.n_total, "lanes_per_cell": shq[0],
                  "ms_per_step": round(1e3 * eq_s / steps, 5), "value": round(wq.n_total * steps / eq_s, 1),
                  "learned_20ppe_ms_per_step": round(1e3 * mlp_s / steps, 5),
                  "learned_faster_by": round(eq_s / mlp_s, 4)}
    res = {
        "error_metric": "population-weighted RMS of <phi|V> over (element, bin) against 4000 particles/element",
        "error_plain_20ppe": round(err["plain_20"], 6), "error_learned_20ppe": round(err["learned_20"], 6),
        "error_plain_500ppe": round(err["plain_500"], 6),
        "learned_vs_plain20": round(err["learned_20"] / err["plain_20"], 4),
        "learned_vs_plain500": round(err["learned_20"] / err["plain_500"], 4),
        "error_plain_by_ppe": {str(t): round(v, 6) for t, v in plain_by_size.items()},
        "plain_ppe_with_learned_error": eq_ppe,
        "equal_error_step": eq_res,
        "elements_with_scalar_spread": n_domain,
        "served_fraction_with_scalar_spread": round(served_frac, 4),
        "train": {"rows": nrows, "iters": iters, "batch": batch, "ms": round(train_ms, 2),
                  "loss_first": float(loss[:20].mean()), "loss_last": float(loss[-200:].mean())},
        "in_step": {"workload": wl.name, "particles": n, "elements": E, "steps": steps,
                    "lanes_per_cell": in_step_shape[0],
                    "value": round(n * steps / mlp_s, 1), "ms_per_step": round(1e3 * mlp_s / steps, 5),
                    "plain_value": round(n * steps / plain_s, 1),
                    "served_fraction_with_scalar_spread": round(inloop_served, 4)},
        "seconds": round(time.perf_counter() - t_start, 1),
    }
    print(f"[bench] learned: {res}", file=sys.stderr, flush=True)
    return res


def eulerian_leg(torch, W, Simulation, solve: str, cycles: int = 5, between: int = 6) -> dict:
    """An Eulerian solve on the 1M-particle, 10k-element canyon: the elliptic
    relaxation (eqs. 12-18; five components, warm-started from the last
    solution) or the mean-pressure projection (one component, from zero).
    A first solve, then solves every `between` steps at four tolerances.  GPU
    time per solve from HIP events on the simulation's stream around the call
    (statistics pass, assembly, iterations, the update that uses the
    solution).  The per-iteration cost and the per-solve set-up are the slope
    and intercept of a least-squares line through (iterations, solve time)
    of the solves after the first at each tolerance.  Bytes per iteration
    (algorithmic): per unknown and solved component, r w s p x read and
    p x s r w written (80 B), and per unknown the inverse diagonal and its
    padded row (8 + 12 W B); with the projection's coarse space, per
    aggregate its three sums and correction read and written (64 B) and per
    block the rows of E^+ its need list reads (32 na 4 B: float)."""
    wl = W.config2(steps=10)
    sim = Simulation.from_workload(wl, device="cuda:0")
    size = sim.relaxation_size()
    sim.step_graph(30)
    sim.sync()
    stream = sim.stream
    call = sim.elliptic_relaxation if solve == "relaxation" else sim.pressure_projection
    ncomp = 5 if solve == "relaxation" else 1

    def timed(tol):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        r = call(max_iters=20000, tol=tol, outputs=False)
        e1.record(stream)
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1)

    cold, cold_ms = timed(1e-8)
    warm = {}
    pts = []
    for tol in (1e-6, 1e-8, 1e-10, 1e-12):
        its, mss = [], []
        for k in range(cycles + 1):
            sim.step_graph(between)
            r, ms = timed(tol)
            assert r["converged"], r
            if k == 0:
                continue   # the first solve at a new tolerance sizes its batches from the last one
            its.append(r["iterations"])
            mss.append(ms)
            pts.append((r["iterations"], ms))
        warm[f"{tol:g}"] = {"iterations": round(sum(its) / len(its), 1), "ms": round(sum(mss) / len(mss), 4)}
    sim.close()
    n = len(pts)
    mx = sum(p[0] for p in pts) / n
    my = sum(p[1] for p in pts) / n
    slope = sum((p[0] - mx) * (p[1] - my) for p in pts) / sum((p[0] - mx) ** 2 for p in pts)
    icpt = my - slope * mx
    nc, w = size["unknowns"], size["row_width"]
    na = size["aggregates"] if solve == "projection" else 0
    nbx = -(-nc // 128)
    bytes_iter = nc * (ncomp * 80 + 8 + 12 * w) + (na * 64 + nbx * 32 * na * 4 if na else 0)
    achieved = bytes_iter / (slope * 1e-3) / 1e9
    res = {
        "workload": f"{wl.name}: the P1 system of its mesh, statistics of its 1M particles",
        "unknowns": nc, "nonzeros": size["nonzeros"], "row_width": w, "components": ncomp,
        "coarse_aggregates": na,
        "first_solve": {"tol": 1e-8, "iterations": cold["iterations"], "ms": round(cold_ms, 4)},
        "every_steps": between, "by_tol": warm,
        "per_iteration_us": round(1e3 * slope, 3), "per_solve_setup_us": round(1e3 * icpt, 1),
        "roofline": {"bound": "hbm", "kernel": "k_relax_iter" if solve == "relaxation" else "k_proj_iter", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes_per_iteration": bytes_iter,
                     "spmv_hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
                     "note": "the system is L2-resident (a few MB) and each iteration is one launch with two "
                             "dependent rounds of loads: launch latency and load latency bound it, not HBM"},
    }
    if solve == "projection":
        res["note"] = ("conjugate gradients preconditioned by the diagonal plus a coarse correction on "
                       f"{na} aggregates of 32 unknowns (one launch per iteration); each projection covers "
                       f"the {between} steps since the one before")
    print(f"[bench] {solve}: {res}", file=sys.stderr, flush=True)
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="canyon1m", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--secondary", default="canyon10m,batched64,canyon10m_omega,canyon10m_bins5,square40k",
                    help="further workloads reported in the same line, comma separated ('' for none)")
    ap.add_argument("--secondary-steps", type=int, default=1000)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed blocks of K steps on the main workload; the first is the reported one, "
                         "all are listed with their median")
    ap.add_argument("--no-graph", action="store_true", help="launch steps one by one instead of graph replays")
    ap.add_argument("--autotune-steps", type=int, default=8,
                    help="steps per trial of a candidate launch shape (two trials each) before warmup "
                         "(0: no tuning)")
    ap.add_argument("--launch", default="",
                    help="fixed launch shape 'lanes_per_cell,persistent' (e.g. 32,1) instead of tuning")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned conditional-mean leg (training, error, in-step throughput)")
    ap.add_argument("--no-relaxation", action="store_true",
                    help="skip the Eulerian legs (elliptic relaxation and mean-pressure projection: solve time "
                         "and per-iteration cost)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration under rocprofv3)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU; the batched-ensemble and mesh-partition "
              "designs for several GPUs are documented with the library but not launched", file=sys.stderr)
        return 2

    import torch
    import workloads as W
    from paper_1003_4548_amd import Simulation

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    src_hash = kernel_source_hash()

    autotune_steps = args.autotune_steps

    def valu_issue(name, kern_ms):
        """The bound the step kernel actually sits at: VALU issue, from the
        profiled instruction count over the live kernel time."""
        n = read_valu(name, src_hash)
        if n is None:
            return None
        rate = n / (kern_ms * 1e-3)
        return {"bound": "alu", "achieved": round(rate / 1e9, 2), "peak": round(VALU_PEAK_WAVE_INSTS / 1e9, 2),
                "unit": "G VALU wavefront-instructions/s", "frac": round(rate / VALU_PEAK_WAVE_INSTS, 4),
                "valu_wave_instructions_per_step": n}

    def run(name, steps, warmup, repeats=1):
        cfg_fn = getattr(W, WORKLOADS[name][0])
        wl = cfg_fn(steps=steps)
        sim = Simulation.from_workload(wl, device="cuda:0")
        print(f"[bench] {name}: {wl.n_total} particles, {wl.mesh.nelem} elements, warmup {warmup}", file=sys.stderr, flush=True)
        if args.launch:
            shape = tuple(int(v) for v in args.launch.split(","))
            sim.set_launch(*shape)
        elif autotune_steps > 0:
            shape = sim.autotune(steps_per_trial=autotune_steps)
        else:
            shape = (64, 0)
        print(f"[bench] {name}: launch shape group={shape[0]} persistent={shape[1]}", file=sys.stderr, flush=True)
        tuned = sim.steps_done()
        sim.step(warmup)
        sim.sync()
        stream = sim.stream
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        step_fn = sim.step if args.no_graph else sim.step_graph
        t0 = time.perf_counter()
        e0.record(stream)
        step_fn(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sim.sync()
        assert sim.steps_done() == tuned + warmup + steps
        # further timed blocks of the same length (spread of the measurement)
        rep_ms = [1e3 * (t1 - t0) / steps]
        for _ in range(repeats - 1):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            step_fn(steps)
            torch.cuda.synchronize()
            rep_ms.append(1e3 * (time.perf_counter() - ta) / steps)
        # the step kernels' own time, from HIP events around each step's
        # kernels on the simulation's stream (eager steps, same state)
        timed_steps = min(steps, 200)
        kern_ms = sim.step_timed(timed_steps) / timed_steps
        repacks = sim.repacks()
        metrics = sim.metrics()
        # the same steps with time averaging on (one merge launch per step)
        avg_steps = min(steps, 100)
        sim.average_attach()
        step_fn(avg_steps)
        sim.sync()
        t2 = time.perf_counter()
        step_fn(avg_steps)
        sim.sync()
        avg_wall = time.perf_counter() - t2
        sim.average_detach()
        wall = t1 - t0
        graph_ms = e0.elapsed_time(e1) / steps
        ab = algorithmic_bytes(wl)
        sb = scope_bytes(wl)
        achieved = sb["per_step"] / (kern_ms * 1e-3) / 1e9
        achieved_design = ab["per_step"] / (kern_ms * 1e-3) / 1e9
        traffic = read_traffic(name, src_hash)
        res = {
            "value": wl.n_total * steps / wall,
            "ms_per_step": 1e3 * wall / steps,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                         "kernel": "k_step (one or two launches per step)", "kernel_ms": round(kern_ms, 5),
                         "kernel_ms_source": f"HIP events around each step's kernels, {timed_steps} eager steps",
                         "graph_ms_per_step": round(graph_ms, 5),
                         "algorithmic_bytes": "scope table: state read + mutable write + statistics re-read "
                                              "per particle, plus amortised cell and mesh terms",
                         "algorithmic_bytes_per_step": sb["per_step"],
                         "algorithmic_bytes_per_particle": sb["per_particle"],
                         "design_bytes": {"per_particle": ab["per_particle"], "per_step": ab["per_step"],
                                          "achieved": round(achieved_design, 1),
                                          "frac": round(achieved_design / HBM_PEAK_GBS, 4),
                                          "note": "one state read and one write; estimation is fused with "
                                                  "the advance, so there is no separate re-read"},
                         "valu_issue": valu_issue(name, kern_ms)},
            "config": {"workload": WORKLOADS[name][1], "preset": name, "particles": wl.n_total,
                       "elements": wl.mesh.nelem, "vertices": wl.mesh.nvert, "ensembles": wl.nens,
                       "state_dtype": wl.precision, "statistics_dtype": "f64", "model": wl.describe()["model"],
                       "moments": wl.moments, "hist_bins": wl.hist_bins, "dt": wl.dt,
                       "turbulent_frequency": bool(getattr(wl, "omega", False)),
                       "velocity_bins": "5x5x5" if getattr(wl, "vbins", 2) == 5 else "2x2x2 (signs)",
                       "launch": {"lanes_per_cell": shape[0], "persistent": bool(shape[1]),
                                  "autotune_steps_per_candidate": 0 if args.launch else autotune_steps,
                                  "hip_graph": not args.no_graph},
                       "segment_repacks": repacks,
                       "repeat_ms_per_step": [round(v, 5) for v in rep_ms],
                       "median_ms_per_step": round(sorted(rep_ms)[len(rep_ms) // 2], 5),
                       "last_step": {"mover_fraction": round(metrics["arrivals_last_step"] / max(1, wl.n_total), 5),
                                     "min_per_cell": metrics["min_per_cell"],
                                     "max_per_cell": metrics["max_per_cell"]},
                       "with_time_averaging": {"steps": avg_steps, "ms_per_step": round(1e3 * avg_wall / avg_steps, 5),
                                               "value": round(wl.n_total * avg_steps / avg_wall, 1)},
                       "kernel_source_hash": src_hash},
            "wl_fn": (cfg_fn, steps),
        }
        sim.close()
        del sim
        torch.cuda.empty_cache()
        return res

    main_res = run(args.workload, args.steps, args.warmup, max(1, args.repeats))
    out = {
        "metric": "particle-steps/s",
        "value": round(main_res["value"], 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if main_res["config"]["state_dtype"] == "f32" else "f64",
        "data": "synthetic",
        "config": main_res["config"],
        "roofline": main_res["roofline"],
    }
    for name in [w for w in args.secondary.split(",") if w and w != args.workload]:
        sec_steps = FIXED_STEPS.get(name, args.secondary_steps)
        sec = run(name, sec_steps, max(5, args.warmup // 2))
        out.setdefault("secondary", {})[name] = {
            "value": round(sec["value"], 1), "unit": "particle-steps/s", "steps": sec_steps,
            "ms_per_step": round(sec["ms_per_step"], 5), "config": sec["config"], "roofline": sec["roofline"]}
    sec = out.get("secondary", {})
    if "batched64" in sec and "canyon10m" in sec:
        # the batched run's time against its particles at the large run's time per particle
        per_particle = sec["canyon10m"]["ms_per_step"] / sec["canyon10m"]["config"]["particles"]
        b = sec["batched64"]
        b["balance_efficiency"] = round(b["config"]["particles"] * per_particle / b["ms_per_step"], 4)
    if not args.no_learned:
        out["learned_phi_given_v"] = learned_leg(torch, W, Simulation)
    if not args.no_relaxation:
        out["elliptic_relaxation"] = eulerian_leg(torch, W, Simulation, "relaxation")
        out["pressure_projection"] = eulerian_leg(torch, W, Simulation, "projection")
    if args.calibrate_copy:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
        del a, b
    if not args.no_cpu_baseline:
        cfg_fn, _ = main_res["wl_fn"]
        out["cpu_baseline"] = cpu_baseline(lambda: cfg_fn(steps=1), args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
