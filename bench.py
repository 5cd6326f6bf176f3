"""Throughput of the cloning algorithm on one MI355X: clone-hops per second.

Workload (the L=100 transition sweep): periodic SSEP with L=100, N=50, 32
scaled biases lambda = s L^2 evenly spaced over [-10, 20], Nc = 1e5 clones
each, Delta t = 0.5, t_obs = 2000 (4000 cloning intervals), [eq] selection,
modified (e^{-s}-scaled) dynamics, uniform random initial configurations,
Philox seeds 2000 + i.  All 32 instances run as one batch: one step = one
cloning interval of the whole sweep (the dynamical stage of 3.2e6 clones,
then the cloning stage of each instance).  The reported value is the number of
hops performed in the timed steps divided by their wall time; the cloning
stage is inside the timed region.

Usage: python bench.py [--steps K] [--warmup W] [--nc NC] [--no-cpu-baseline]
By default W + K = 4000 so that the run covers exactly t_obs = 2000.

--workload batch: 64 uneven instances in one context against 64 sequential
contexts.  --workload guided-rate: guided against plain throughput at L=100,
lambda=15.  --workload large: the L=400, Nc=1e6 workload, plain and guided.  --workload guide: wall time to |delta psi| <= 1e-3, guided
against plain, at L=100 (lambda = 5, 10, 15, 20, Delta t = 0.5) and at the
paper's phase-separated state point L=50, lambda=50 (Delta t = 10,
t_obs = 1e4); see bench_guide.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1711_05095_amd import inputs, pd  # noqa: E402

# Published MI355X figures (vector ALU): 256 CUs x 64 lanes x 2.4 GHz.
PEAK_VALU_LANE_OPS = 256 * 64 * 2.4e9
PEAK_HBM_GBS = 8000.0
# VALU instructions in one pass of the event loop of the step kernel (W = 2),
# counted from its gfx950 assembly by paper_1711_05095_amd.isa_count (a test
# keeps this constant equal to that count).  It is the algorithmic work of an
# event for every variant (the compacting variant's loop has the same count;
# its rounds' bookkeeping lies outside the loop and counts as overhead).
VALU_PER_EVENT_W2 = 160
VALU_PER_EVENT_W7 = 285   # the same loop for 400-site states (7 words)
# HBM bytes the cloning stage must move per clone: ln Ups read (8) by the
# resample scan, ancestor written (4); the gather of the states is fused into
# the next dynamical stage's load.
RESAMPLE_BYTES_PER_CLONE = 12
# HBM bytes per launch of the step kernel on this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE runs scaled by a plain 1 GiB copy (factors 2 and
# 1), valid only for the kernel sources they were taken on (STEP_SOURCES).
STEP_TRAFFIC = {"bytes": 239.9e6, "kernels_sha1": "f643ba6df47a", "kernel": "k_step_c<2>"}
STEP_SOURCES = ["pd_kernels.hip", "pd_tile.hpp", "pd_device.hpp", "pd_internal.hpp"]


def step_sources_sha1():
    h = hashlib.sha1()
    for f in STEP_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1711_05095_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:12]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--nc", type=int, default=100_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cycles", type=int, default=8)
    ap.add_argument("--variant", type=int, default=None,
                    help="step kernel variant (default: chosen by the autotuner)")
    ap.add_argument("--refill", type=int, default=13,
                    help="variants 1-3: refill threshold; variant 4: first round in 16ths")
    ap.add_argument("--scan-tiles", type=int, default=1,
                    help="tiles of 256 clones per cloning-stage block (with --variant)")
    ap.add_argument("--workload", choices=["sweep", "batch", "guide", "guided-rate", "large"],
                    default="sweep",
                    help="sweep: the L=100 transition sweep (default); batch: 64 uneven "
                         "instances in one context against 64 sequential contexts")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (for PMC byte-counter scaling)")
    a = ap.parse_args()
    if a.steps is None:
        M = int(round(inputs.SWEEP["t_obs"] / inputs.SWEEP["dt"]))
        a.steps = max(1, M - a.warmup)
    return a


def calibrate_copy():
    import torch
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n}), flush=True)


def bench_batch(a):
    """64 uneven instances (L in {20..200}, N = L/2, lambda in [-10, 20], Nc
    log-uniform in [1e3, 1e5], dt = 0.5, t_obs = 1000): all in one context
    (one step launch per word count and one cloning launch per cycle, replayed
    from graphs), against the same 64 instances run one after another, each
    in its own context."""
    import torch
    specs = inputs.batched_instances()
    M = int(round(specs[0]["t_obs"] / specs[0]["dt"]))
    cycles = min(M, a.steps)
    params = [pd.make_params(d["L"], d["N"], d["s"], d["Nc"], d["t_obs"], d["dt"], seed=d["seed"],
                             instance=d["instance"]) for d in specs]
    B = pd.Sampler(params)
    tuning = B.autotune(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.run(cycles)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    hops_b = sum(B.estimates(i)["hops"] for i in range(B.n))
    singles = [pd.Sampler(q) for q in params]
    for S in singles:
        S.set_tuning(tuning["step_variant"], tuning["refill"], tuning["graph_cycles"],
                     tuning["scan_tiles"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for S in singles:
        S.run(cycles)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    hops_s = sum(S.estimates()["hops"] for S in singles)
    same = all(B.estimates(i) == singles[i].estimates() for i in range(B.n))
    return {"metric": "clone-hops/s", "value": hops_b / t_batch, "unit": "clone-hops/s",
            "n_gpus": 1, "steps": cycles, "warmup": 0, "ms_per_step": t_batch / cycles * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "64 uneven instances: L in {20..200}, N=L/2, lambda in "
                                   "[-10,20], Nc log-uniform in [1e3,1e5], dt=0.5, %d intervals"
                                   % cycles, "total_clones": int(sum(d["Nc"] for d in specs))},
            "sequential": {"value": hops_s / t_sec if (t_sec := t_seq) else None,
                           "seconds": t_seq, "hops": hops_s},
            "batched_seconds": t_batch, "speedup_vs_sequential": t_seq / t_batch,
            "identical_results": same, "tuning": tuning}


def _estimates(L, N, lam, Nc, t_obs, dt, reps, mode, eg=None, seed=0, inst0=1):
    """psi-hat of `reps` independent runs (one batch) and the wall time."""
    import torch
    s = inputs.s_of_lambda(lam, L)
    ps = [pd.make_params(L, N, s, Nc, t_obs, dt, seed=seed, weight_mode=mode, instance=inst0 + r)
          for r in range(reps)]
    S = pd.Sampler(ps)
    if eg is not None:
        S.set_guide(eg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.run(int(round(t_obs / dt)))
    est = [S.estimates(i) for i in range(reps)]
    el = time.perf_counter() - t0
    S.close()
    return np.array([e["psi"] for e in est]), el


def bench_guide(a):
    """Wall time to |delta psi| <= 1e-3, guided against plain.

    For each state point and each form (plain: modified dynamics; guided: the
    learned guide, trained on the GPU from plain populations at Nc = 1e5 and
    distilled on them; at L = 400 the L = 100 guide fine-tuned on L = 400
    populations), the cheapest (Nc, t_obs) of a grid whose RMS error over
    8 seeds against psi_ref is <= 1e-3; psi_ref = mean of plain runs at
    Nc = 1e6 with the same t_obs (psi-hat's large-Nc limit depends on t_obs).
    The reported time is one run at that grid point (median of 3).  Guide
    training (collection, training, distillation) is timed separately."""
    import torch
    from paper_1711_05095_amd import guide
    points = [dict(L=100, N=50, lam=lam, dt=0.5, t_grid=[100.0, 500.0, 2000.0],
                   nc_grid=[100, 1000, 10000, 100000], lag=100, snapshots=10, burn=400)
              for lam in (5.0, 10.0, 15.0, 20.0)]
    points.append(dict(L=50, N=25, lam=50.0, dt=10.0, t_grid=[10000.0],
                       nc_grid=[1000, 3000, 10000, 30000, 100000], lag=5, snapshots=10,
                       burn=100))
    # L=400: the guide of the L=100, lambda=20 point, fine-tuned on L=400 populations
    points.append(dict(L=400, N=200, lam=20.0, dt=1.0, t_grid=[100.0, 500.0],
                       nc_grid=[100, 1000, 10000], lag=20, snapshots=4, burn=50,
                       finetune_from=(100, 20.0)))
    out = []
    trained = {}
    tol, reps = 1e-3, 8
    for P in points:
        L, N, lam, dt = P["L"], P["N"], P["lam"], P["dt"]
        t0 = time.perf_counter()
        if "finetune_from" in P:
            base = trained[P["finetune_from"]]
            states, counts = guide.collect(L, N, inputs.s_of_lambda(lam, L), 100_000, dt,
                                           P["lag"], P["snapshots"], P["burn"], seed=77)
            Sd, Cd = guide.Trainer.upload(states, counts, seed=1)
            tr = guide.Trainer(L, theta0=base.theta.cpu().numpy(), lr=5e-4)
            for e in range(3):
                tr.epoch(Sd, Cd, 5e-4 * 0.8 ** e)
            _, eg, _ = tr.tables_cond(Sd, 4, 1.0)
            g = {"trainer": tr, "eg": eg}
        else:
            g = guide.train_guide(L, N, inputs.s_of_lambda(lam, L), Nc=100_000, dt=dt,
                                  lag_cycles=P["lag"], snapshots=P["snapshots"],
                                  burn_cycles=P["burn"], epochs=10, lr=1e-3, decay=0.8,
                                  gmax=1.0, seed=9)
        trained[(L, lam)] = g["trainer"]
        t_train = time.perf_counter() - t0
        refs = {}
        for t_obs in P["t_grid"]:
            psi, _ = _estimates(L, N, lam, 1_000_000, t_obs, dt, 2, pd.PD_W_MODIFIED, seed=1,
                                inst0=100)
            refs[t_obs] = float(psi.mean())
        row = {"L": L, "lambda": lam, "dt": dt, "train_seconds": t_train, "psi_ref": refs,
               "guide": "fine-tuned from L=%d" % P["finetune_from"][0] if "finetune_from" in P
               else "trained at this point"}
        grid = sorted(((nc, t) for nc in P["nc_grid"] for t in P["t_grid"]),
                      key=lambda q: q[0] * q[1])
        for name, mode, eg in (("plain", pd.PD_W_MODIFIED, None),
                               ("guided", pd.PD_W_GUIDED, g["eg"])):
            found = None
            for nc, t_obs in grid:
                psi, _ = _estimates(L, N, lam, nc, t_obs, dt, reps, mode, eg, seed=2)
                rms = float(np.sqrt(np.mean((psi - refs[t_obs]) ** 2)))
                print("  L=%d lambda=%g %s Nc=%d t_obs=%g: rms %.2e" % (L, lam, name, nc, t_obs, rms),
                      file=sys.stderr, flush=True)
                if rms <= tol:
                    times = [_estimates(L, N, lam, nc, t_obs, dt, 1, mode, eg, seed=3)[1]
                             for _ in range(3)]
                    found = {"Nc": nc, "t_obs": t_obs, "rms": rms,
                             "seconds": float(np.median(times))}
                    break
            row[name] = found
        if row["plain"] and row["guided"]:
            row["plain_over_guided"] = row["plain"]["seconds"] / row["guided"]["seconds"]
        print(json.dumps(row), file=sys.stderr, flush=True)
        out.append(row)
    ratios = [r["plain_over_guided"] for r in out if "plain_over_guided" in r]
    return {"metric": "wall time to |dpsi|<=1e-3, plain/guided", "unit": "ratio",
            "value": float(np.exp(np.mean(np.log(ratios)))) if ratios else None,
            "higher_is_better": True, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
            "vs_baseline": None,
            "config": {"workload": "guided vs plain: L=100 lambda 5..20 dt=0.5; L=50 lambda=50 "
                                   "dt=10 t_obs=1e4; L=400 lambda=20 dt=1 (guide fine-tuned "
                                   "from L=100); RMS over 8 seeds vs plain Nc=1e6"},
            "points": out}


def bench_guided_rate(a):
    """Throughput of the guided dynamical stage against the plain one on the
    same workload: a guide trained at L=100, lambda=15 (Nc=1e5, 10 snapshots,
    lag 100 intervals), then 32 instances x Nc=1e5 (one lambda, 32 seeds),
    dt=0.5, a.steps cycles each after 8 warm-up cycles."""
    import torch
    from paper_1711_05095_amd import guide
    L, N, lam, dt = 100, 50, 15.0, 0.5
    s = inputs.s_of_lambda(lam, L)
    g = guide.train_guide(L, N, s, Nc=100_000, dt=dt, lag_cycles=100, snapshots=10,
                          burn_cycles=400, epochs=10, lr=1e-3, decay=0.8, gmax=1.0, seed=9)
    steps = min(a.steps, 200)
    out = {}
    for name, mode in (("plain", pd.PD_W_MODIFIED), ("guided", pd.PD_W_GUIDED)):
        ps = [pd.make_params(L, N, s, 100_000, (steps + 8) * dt, dt, seed=2000 + i, instance=i,
                             weight_mode=mode) for i in range(32)]
        S = pd.Sampler(ps)
        if mode == pd.PD_W_GUIDED:
            S.set_guide(g["eg"])
        S.run(8)
        torch.cuda.synchronize()
        h0 = sum(S.estimates(i)["hops"] for i in range(S.n))
        t0 = time.perf_counter()
        S.run(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        h = sum(S.estimates(i)["hops"] for i in range(S.n)) - h0
        out[name] = {"hops_per_second": h / el, "ms_per_cycle": el / steps * 1e3,
                     "hops_per_clone_interval": h / (steps * 32 * 100_000)}
        S.close()
    return {"metric": "clone-hops/s, guided", "value": out["guided"]["hops_per_second"],
            "unit": "clone-hops/s", "n_gpus": 1, "steps": steps, "warmup": 8,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic", "vs_baseline": None,
            "config": {"workload": "L=100 N=50 lambda=15: 32 instances x Nc=1e5, dt=0.5, "
                                   "trained guide vs plain"},
            "plain": out["plain"], "guided": out["guided"],
            "guided_over_plain": out["guided"]["hops_per_second"] / out["plain"]["hops_per_second"]}


def _timed_cycles(S, steps, res_bytes):
    """Runs `steps` cycles with HIP events around every stage on the sampler's
    stream; returns (hops/s, mean step ms, mean resample ms, resample GB/s)."""
    import torch
    st = S.stream
    torch.cuda.synchronize()
    h0 = sum(S.estimates(i)["hops"] for i in range(S.n))
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(st)
        S.step()
        ev[k][1].record(st)
        S.resample()
        ev[k][2].record(st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h = sum(S.estimates(i)["hops"] for i in range(S.n)) - h0
    step_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    res_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    return h / el, step_ms, res_ms, res_bytes / (res_ms / 1e3) / 1e9, h / steps


def bench_large(a):
    """The L=400 workload: N=200, Nc=1e6 clones with 400-bit states (7 words),
    dt=1, lambda in {0, 10, 20}.  Per lambda: plain throughput over a.steps
    cycles (default 100, after 8, autotuned), the step kernel against the ALU
    roofline (events x the 7-word event loop's VALU count / step time) and the
    cloning stage's HBM rate; then guided throughput with a guide trained at
    L=100 (lambda=20) and fine-tuned on L=400 populations."""
    import torch
    from paper_1711_05095_amd import guide
    L, N, Nc, dt = 400, 200, 1_000_000, 1.0
    steps = min(a.steps, 100)
    rows = []
    g100 = guide.train_guide(100, 50, inputs.s_of_lambda(20.0, 100), Nc=100_000, dt=0.5,
                             lag_cycles=100, snapshots=10, burn_cycles=400, epochs=10, lr=1e-3,
                             decay=0.8, gmax=1.0, seed=9)
    for lam in inputs.LARGE["lambdas"]:
        s = inputs.s_of_lambda(lam, L)
        row = {"lambda": lam}
        P = pd.make_params(L, N, s, Nc, (steps + 8) * dt, dt, seed=5000 + int(lam))
        S = pd.Sampler(P)
        tuning = S.autotune(3)
        S.run(8)
        hs, sm, rm, gbs, hpc = _timed_cycles(S, steps, RESAMPLE_BYTES_PER_CLONE * Nc)
        ach = (hpc + Nc) * VALU_PER_EVENT_W7 / (sm / 1e3)
        row["plain"] = {"hops_per_second": hs, "step_ms": sm, "resample_ms": rm,
                        "resample_GBps": gbs, "hops_per_cycle": hpc, "tuning": tuning,
                        "roofline": {"bound": "alu", "achieved": ach / 1e12,
                                     "peak": PEAK_VALU_LANE_OPS / 1e12,
                                     "unit": "T VALU lane-instr/s",
                                     "frac": ach / PEAK_VALU_LANE_OPS,
                                     "per_unit": "%d VALU instr per event" % VALU_PER_EVENT_W7}}
        S.close()
        # fine-tune the L=100 guide on L=400 populations (1e5 clones, 4 snapshots)
        states, counts = guide.collect(L, N, s, 100_000, dt, 20, 4, 50, seed=77)
        Sd, Cd = guide.Trainer.upload(states, counts, seed=1)
        tr = guide.Trainer(L, theta0=g100["trainer"].theta.cpu().numpy(), lr=5e-4)
        t0 = time.perf_counter()
        for e in range(3):
            tr.epoch(Sd, Cd, 5e-4 * 0.8 ** e)
        _, eg, _ = tr.tables_cond(Sd, 4, 1.0)
        row["finetune_seconds"] = time.perf_counter() - t0
        P = pd.make_params(L, N, s, Nc, (steps + 8) * dt, dt, seed=5000 + int(lam),
                           weight_mode=pd.PD_W_GUIDED)
        S = pd.Sampler(P)
        S.set_guide(eg)
        S.run(8)
        hs, sm, rm, gbs, hpc = _timed_cycles(S, steps, RESAMPLE_BYTES_PER_CLONE * Nc)
        row["guided"] = {"hops_per_second": hs, "step_ms": sm, "resample_ms": rm,
                         "resample_GBps": gbs, "hops_per_cycle": hpc}
        S.close()
        print(json.dumps(row), file=sys.stderr, flush=True)
        rows.append(row)
    return {"metric": "clone-hops/s", "unit": "clone-hops/s", "n_gpus": 1, "dtype": "f64",
            "data": "synthetic", "vs_baseline": None, "higher_is_better": True,
            "value": float(np.mean([r["plain"]["hops_per_second"] for r in rows])),
            "steps": steps, "warmup": 8,
            "config": {"workload": "L=400 N=200 Nc=1e6 dt=1, lambda 0/10/20, one instance each; "
                                   "guide trained at L=100 lambda=20, fine-tuned at L=400"},
            "resample_peak_GBps": PEAK_HBM_GBS, "points": rows}


def cpu_baseline(nc, cycles):
    """The test oracle (plain single-threaded C) on a bounded sample of the
    same workload: instance lambda = 20, Nc clones, `cycles` intervals."""
    import oracle
    w = inputs.SWEEP
    s = inputs.s_of_lambda(20.0, w["L"])
    o = oracle.Oracle(w["L"], w["N"], s, nc, w["dt"], M=cycles, seed=w["seed0"])
    t0 = time.perf_counter()
    r = o.run()
    dt = time.perf_counter() - t0
    return {"value": r["hops"] / dt, "unit": "clone-hops/s", "cores": 1, "kind": "oracle",
            "sample": "lambda=20 instance of the sweep, Nc=%d, %d intervals (%d hops, "
                      "init included), %.1f s" % (nc, cycles, r["hops"], dt)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if a.calibrate_copy:
        calibrate_copy()
        return
    if a.workload == "batch":
        print(json.dumps(bench_batch(a)), flush=True)
        return
    if a.workload == "guide":
        print(json.dumps(bench_guide(a)), flush=True)
        return
    if a.workload == "guided-rate":
        print(json.dumps(bench_guided_rate(a)), flush=True)
        return
    if a.workload == "large":
        print(json.dumps(bench_large(a)), flush=True)
        return
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = inputs.SWEEP
    L, N, dt = w["L"], w["N"], w["dt"]
    total = a.warmup + a.steps
    params = [pd.make_params(L, N, inputs.s_of_lambda(lam, L), a.nc, total * dt, dt,
                             seed=w["seed0"] + i, instance=i)
              for i, lam in enumerate(w["lambdas"])]
    S = pd.Sampler(params)
    st = S.stream

    if a.variant is None:
        tuning = S.autotune(24)          # restores the population afterwards
    else:
        S.set_tuning(a.variant, a.refill, 16, a.scan_tiles)
        tuning = S.tuning()
    for _ in range(a.warmup):
        S.step()
        S.resample()
    torch.cuda.synchronize()
    hops0 = sum(S.estimates(i)["hops"] for i in range(S.n))

    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        ev[k][0].record(st)
        S.step()
        ev[k][1].record(st)
        S.resample()
        ev[k][2].record(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    est = [S.estimates(i) for i in range(S.n)]
    hops = sum(e["hops"] for e in est) - hops0
    step_ms = np.array([e0.elapsed_time(e1) for e0, e1, _ in ev])
    res_ms = np.array([e1.elapsed_time(e2) for _, e1, e2 in ev])
    res_bytes = RESAMPLE_BYTES_PER_CLONE * a.nc * S.n
    value = hops / elapsed
    # events of the step kernel = hops + one closing draw per clone per interval
    events_per_launch = (hops + a.steps * a.nc * S.n) / a.steps
    step_s = float(step_ms.mean()) / 1e3
    achieved = events_per_launch * VALU_PER_EVENT_W2 / step_s

    sha = step_sources_sha1()
    kname = {0: "k_step<2>", 4: "k_step_c<2>"}.get(tuning["step_variant"], "k_step_q<2>")
    traffic = STEP_TRAFFIC["bytes"] if (sha == STEP_TRAFFIC["kernels_sha1"] and a.nc == 100_000
                                        and kname == STEP_TRAFFIC["kernel"]) else None
    out = {
        "metric": "clone-hops/s",
        "value": value,
        "unit": "clone-hops/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "L=100 N=50 transition sweep: 32 lambdas in [-10,20], "
                               "Nc=%d each, dt=0.5, t_obs=%g, [eq], modified dynamics, "
                               "one batch" % (a.nc, total * dt),
                   "instances": S.n, "Nc": a.nc, "L": L, "N": N, "dt": dt,
                   "intervals": total},
        "roofline": {"bound": "alu", "kernel": kname,
                     "achieved": achieved / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12,
                     "unit": "T VALU lane-instr/s", "frac": achieved / PEAK_VALU_LANE_OPS,
                     "traffic": traffic,
                     "per_unit": "%d VALU instr per event" % VALU_PER_EVENT_W2,
                     "events_per_launch": events_per_launch,
                     "step_ms_mean": float(step_ms.mean()),
                     "step_ms_median": float(np.median(step_ms))},
        "resample": {"bound": "hbm", "kernel": "k_resample",
                     "achieved": res_bytes / (float(res_ms.mean()) / 1e3) / 1e9,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": res_bytes / (float(res_ms.mean()) / 1e3) / 1e9 / PEAK_HBM_GBS,
                     "bytes_per_launch": res_bytes, "ms_mean": float(res_ms.mean())},
        "tuning": tuning,
        "physics": {"lambda": w["lambdas"][::8],
                    "psi": [est[i]["psi"] for i in range(0, S.n, 8)],
                    "k_hat": [est[i]["k_hat"] for i in range(0, S.n, 8)]},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.nc, a.cpu_cycles)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
