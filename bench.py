"""Benchmark of the social-field tick on one MI355X.

Workload: the 1024x1024 hall (5% rectangle obstacles, two 16-su exits,
50,000 pedestrians, field radius 16, 500 ticks), synthetic and seeded.  A
"step" is one tick of the whole hot path: bin, decide + claim, commit,
superpose.  Inputs are resident in HBM when the timed region starts.

Prints one JSON line: pedestrian-steps/s (value) and su-field updates/s, the
roofline of the dominant kernel (field superposition) from HIP events recorded
around its launches, the CPU oracle timed on a bounded sample, and (object
"ensemble256") the batched-vs-plain comparison described below.

--workload serving runs the serving loop (Poisson arrivals at 50, 200 and 800
scenes/s, sizes from the same distribution, each scene to evacuation or 2000
ticks, admission by device footprint) and reports per-tick latency p50/p99
and scenes/s per rate.

--workload ensemble256 measures batching instead: 256 scenes of uneven size,
crowd and radius (sides 128..2048 su, 300 ticks), stepped once as a plain
loop of per-scene ticks and once as a batch (one decide, commit and field
launch per tick for all scenes, graph replays, autotuned tiling), with both
results checked to be identical and a lockstep tick of the smallest scenes
against the oracle.

--workload flow1000 runs the paper's own experiment scenario (section 5,
Table IV): a 1000x1000 torus, density 0.5, 8-directional flow, 7x7 fields,
1000 ticks, with the paper's time quoted beside it as context; --workload
flow-sweep runs its 360-combination grid (sides 100..1000, densities
0.1..0.9, 1/2/4/8 directions) and --workload flow-walk its walk-period
experiment (Table V: flow1000 with periods uniform in 1..max, max = 1..11).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pedestrian-steps/s + su-field updates/s; batched vs plain, 0 untied mismatches"
# Non-packed FP32 add rate of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 64 * 2.4e9 / 1e12
# back-to-back field launches timed for the roofline
FIELD_LOOP = 200
KERNEL_SRC = os.path.join(ROOT, "paper_1803_04782_amd", "csrc", "sf_kernels.hip")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "superpose_hall1024_pmc.json")


def kernel_source_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def window_contributions(sc) -> float:
    """Mean number of (pedestrian, su) pairs per pedestrian with the su inside
    the grid and the pedestrian's window, own su excluded, at the initial
    positions."""
    W, H, R = sc.width, sc.height, sc.radius
    if getattr(sc, "periodic", False):
        return float((2 * R + 1) ** 2 - 1)  # a torus: every window is whole
    x = sc.pos % W
    y = sc.pos // W
    wx = np.minimum(x + R, W - 1) - np.maximum(x - R, 0) + 1
    wy = np.minimum(y + R, H - 1) - np.maximum(y - R, 0) + 1
    return float(np.mean(wx * wy - 1))


def traffic_per_launch():
    """HBM bytes per superposition launch from the committed rocprofv3 PMC
    summary, if it was taken on the current kernel source."""
    try:
        d = json.load(open(PMC_SUMMARY))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(sc, gpu_state, seconds: float = 12.0):
    """The FP64 oracle as it stands (single thread) on a bounded sample of the
    workload, plus the same-run accuracy gate: one lockstep tick of the GPU
    state against the oracle."""
    import oracle

    st = oracle.statics(sc)
    pos = sc.pos.copy()
    live_sum = 0
    ticks = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and ticks < sc.steps:
        live_sum += int((pos >= 0).sum())
        pos = oracle.step(st, pos, sc.start_step + ticks).pos
        ticks += 1
    dt = time.perf_counter() - t0
    base = {"value": live_sum / dt, "unit": "pedestrian-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {ticks} ticks of the workload from its initial state "
                      f"(FP64 C oracle, one thread, {dt:.1f} s)"}
    # accuracy gate on the GPU's final state
    pos_g, P_g, t_g, tgt_g, flags_g, pos_next = gpu_state
    r = oracle.step(st, pos_g, t_g)
    free = sc.obstacle == 0
    err = float(np.max(np.abs(P_g[free] - r.P[free]) / np.maximum(np.abs(r.P[free]), 1.0)))
    live = pos_g >= 0
    won = (flags_g & 2) != 0
    bad = live & ((tgt_g != r.target) | (won != (r.moved == 1)) | (pos_next != r.pos))
    tied = set(r.target[live & (r.tied == 1)].tolist()) | set(tgt_g[live & (r.tied == 1)].tolist())
    untied = [j for j in np.flatnonzero(bad)
              if not r.tied[j] and r.target[j] not in tied and tgt_g[j] not in tied]
    gate = {"tick": int(t_g), "field_rel_err": err, "untied_mismatches": len(untied),
            "tied_mismatches": int(bad.sum()) - len(untied),
            "near_tie_decisions": int(r.tied[live].sum()), "decisions": int(live.sum())}
    return base, gate


def bench_ensemble(args, stream, steps=None, emit=True):
    """Batched vs plain on the uneven 256-scene ensemble; prints the JSON line
    (emit) and returns it."""
    import torch

    import oracle
    from paper_1803_04782_amd import scenes, sf

    def say(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    scs = scenes.ensemble(n_scenes=args.scenes, seed=3)
    if steps is None:
        steps = args.steps if args.steps is not None else scs[0].steps
    su_total = sum(s.width * s.height for s in scs)
    free_total = sum(int((s.obstacle == 0).sum()) for s in scs)
    peds_total = sum(s.n_peds for s in scs)
    say(f"ensemble of {len(scs)} scenes: {su_total:.3g} su, {peds_total} pedestrians "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    plain = [sf.GpuScene(s, stream=stream) for s in scs]
    member = [sf.GpuScene(s, stream=stream) for s in scs]
    say(f"created {2 * len(scs)} scenes in {time.perf_counter() - t0:.1f} s")
    b = sf.Batch(member, stream=stream)
    try:
        t0 = time.perf_counter()
        tiling = b.tune(reps=3)
        say(f"autotuned tiling {tiling} in {time.perf_counter() - t0:.1f} s")
        for _ in range(args.warmup):
            for g in plain:
                g.step(1)
        b.step(args.warmup)
        torch.cuda.synchronize()
        ps_plain0 = sum(g.stats()["ped_steps"] for g in plain)
        ps_batch0 = sum(x["ped_steps"] for x in b.stats())

        t0 = time.perf_counter()
        for _ in range(steps):
            for g in plain:
                g.step(1)
        torch.cuda.synchronize()
        dt_plain = time.perf_counter() - t0
        say(f"plain loop: {steps} ticks in {dt_plain:.2f} s")
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        dt_batch = time.perf_counter() - t0
        say(f"batched: {steps} ticks in {dt_batch:.2f} s")
        ps_plain = sum(g.stats()["ped_steps"] for g in plain) - ps_plain0
        totals = b.stats()
        ps_batch = sum(x["ped_steps"] for x in totals) - ps_batch0

        # the two runs must agree bit for bit (positions of every scene, fields
        # of the 16 smallest)
        order = np.argsort([s.width * s.height for s in scs])
        same_pos = all(np.array_equal(a.positions(), m.positions()) for a, m in zip(plain, member))
        same_field = all(np.array_equal(plain[j].field(), member[j].field()) for j in order[:16])
        # one lockstep tick of the 8 smallest scenes against the oracle
        small = [int(j) for j in order[:8]]
        before = []
        for j in small:
            st = oracle.statics(scs[j])
            pos = member[j].positions()
            before.append((j, st, pos, member[j].field(),
                           oracle.step(st, pos, totals[j]["step"])))
        b.step(1)
        err, untied, tied = 0.0, 0, 0
        for j, st, pos, P_g, r in before:
            free = st.obstacle == 0
            if free.any():
                err = max(err, float(np.max(np.abs(P_g[free] - r.P[free]) /
                                            np.maximum(np.abs(r.P[free]), 1.0))))
            tgt_g, flags_g = member[j].last_moves()
            pos_g = member[j].positions()
            live = pos >= 0
            won = (flags_g & 2) != 0
            bad = live & ((tgt_g != r.target) | (won != (r.moved == 1)) | (pos_g != r.pos))
            hot = set(r.target[live & (r.tied == 1)].tolist()) | \
                set(tgt_g[live & (r.tied == 1)].tolist())
            u = [k for k in np.flatnonzero(bad)
                 if not r.tied[k] and r.target[k] not in hot and tgt_g[k] not in hot
                 and pos[k] not in hot]
            untied += len(u)
            tied += int(bad.sum()) - len(u)
    finally:
        b.close()
        for g in plain + member:
            g.close()

    value = ps_batch / dt_batch
    out = {"metric": METRIC, "value": value, "unit": "pedestrian-steps/s", "n_gpus": 1,
           "steps": steps, "warmup": args.warmup, "ms_per_step": 1000.0 * dt_batch / steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"ensemble{len(scs)}", "scenes": len(scs), "su": su_total,
                      "pedestrians": peds_total, "ticks": steps, "sides": [128, 2048],
                      "radii": [4, 8, 16, 32], "parallelism": "single-gpu"},
           "su_field_updates_per_s": steps * free_total / dt_batch,
           "plain": {"value": ps_plain / dt_plain, "ms_per_step": 1000.0 * dt_plain / steps},
           "batched_vs_plain": (ps_batch / dt_batch) / (ps_plain / dt_plain),
           "tiling": tiling,
           "identical_to_plain": {"positions_all_scenes": bool(same_pos),
                                  "fields_16_smallest": bool(same_field)},
           "accuracy_gate": {"scenes": len(small), "field_rel_err": err,
                             "untied_mismatches": untied, "tied_mismatches": tied},
           "roofline": None, "cpu_baseline": None}
    if emit:
        print(json.dumps(out), flush=True)
    return out


# The paper's time for the same scenario (Table IV, 7x7 fields; 1000 ticks per
# reported run), on a GPU it does not name and with its own field laws: context
# only, not a target.
PAPER_FLOW1000 = {"seconds_per_1000_ticks": 62.0, "ms_per_tick": 62.0,
                  "pedestrian_steps_per_s": 500000 / 0.062,
                  "hardware": "unnamed GPU (OpenCL), FP32", "source": "Table IV, 7x7 column"}


def bench_flow_sweep(args, stream):
    """The paper's experiment grid (section 5): tori of 100^2 .. 1000^2 su,
    density 0.1 .. 0.9, 1/2/4/8-directional flows, 7x7 fields, `steps` ticks
    each (default 1000).  Prints one JSON line: aggregate pedestrian-steps/s
    and the ms per tick of every combination."""
    import torch

    from paper_1803_04782_amd import scenes, sf

    def say(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    steps = args.steps if args.steps is not None else 1000
    sides = [int(v) for v in args.sweep_sides.split(",")]
    dens = [float(v) for v in args.sweep_densities.split(",")]
    dirs = [int(v) for v in args.sweep_directions.split(",")]
    rows = []
    total_ps, total_t = 0, 0.0
    for n in sides:
        for d in dens:
            for k in dirs:
                sc = scenes.flow_scene(n, n, d, k, radius=3, seed=0, steps=steps)
                g = sf.GpuScene(sc, stream=stream)
                try:
                    g.step(5)
                    g.set_state(sc.pos, 0)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    g.step(steps)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    ps = g.stats()["ped_steps"]
                    moved = g.stats()["moved"]
                finally:
                    g.close()
                total_ps += ps
                total_t += dt
                rows.append({"side": n, "density": d, "directions": k, "pedestrians": sc.n_peds,
                             "ms_per_tick": 1000.0 * dt / steps, "pedestrian_steps_per_s": ps / dt,
                             "moved_fraction": moved / max(ps, 1)})
            say(f"side {n} density {d:g}: " + ", ".join(
                f"k{r['directions']} {r['ms_per_tick']:.4f} ms" for r in rows[-len(dirs):]))
    out = {"metric": METRIC, "value": total_ps / total_t, "unit": "pedestrian-steps/s",
           "n_gpus": 1, "steps": steps, "warmup": 5,
           "ms_per_step": 1000.0 * total_t / (steps * len(rows)), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "flow-sweep", "sides": sides, "densities": dens,
                      "directions": dirs, "radius": 3, "periodic": True, "ticks": steps,
                      "combinations": len(rows), "parallelism": "single-gpu"},
           "runs": rows, "paper_context": PAPER_FLOW1000, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


# The paper's times for flow1000 with walk periods uniform in 1..max (Table V,
# current GPU model; seconds per 1000 ticks): context only.
PAPER_WALK = {1: 62.0, 3: 64.0, 5: 64.0, 7: 63.0, 9: 62.0, 11: 62.0}


def bench_flow_walk(args, stream):
    """flow1000 with walk periods uniform in 1..max for max = 1, 3, ..., 11
    (the experiment of the paper's Table V); one JSON line with ms per tick
    per maximal period."""
    import torch

    from paper_1803_04782_amd import scenes, sf

    steps = args.steps if args.steps is not None else 1000
    rows = []
    total_ps, total_t = 0, 0.0
    for pmax in (1, 3, 5, 7, 9, 11):
        sc = scenes.flow_scene(1000, 1000, 0.5, 8, radius=3, seed=0, steps=steps,
                               max_walk_period=pmax)
        g = sf.GpuScene(sc, stream=stream)
        try:
            g.step(5)
            g.set_state(sc.pos, 0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = g.stats()
        finally:
            g.close()
        total_ps += st["ped_steps"]
        total_t += dt
        rows.append({"max_walk_period": pmax, "ms_per_tick": 1000.0 * dt / steps,
                     "pedestrian_steps_per_s": st["ped_steps"] / dt,
                     "registered_fraction": st["movers"] / max(st["ped_steps"], 1),
                     "paper_ms_per_tick": PAPER_WALK[pmax]})
        print(f"[bench] max walk period {pmax}: {rows[-1]['ms_per_tick']:.4f} ms per tick",
              file=sys.stderr, flush=True)
    out = {"metric": METRIC, "value": total_ps / total_t, "unit": "pedestrian-steps/s",
           "n_gpus": 1, "steps": steps, "warmup": 5,
           "ms_per_step": 1000.0 * total_t / (steps * len(rows)), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "flow-walk", "grid": [1000, 1000], "density": 0.5,
                      "directions": 8, "radius": 3, "periodic": True, "ticks": steps,
                      "max_walk_periods": [r["max_walk_period"] for r in rows],
                      "parallelism": "single-gpu"},
           "runs": rows, "paper_context": {"source": "Table V, current GPU model",
                                           "hardware": PAPER_FLOW1000["hardware"]},
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_serving(args, stream):
    """Serving loop under Poisson arrivals at several rates."""
    import torch

    from paper_1803_04782_amd import scenes, serve

    def say(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    # request sizes: a pool of scenes drawn from the uneven-ensemble
    # distribution (request i uses pool entry i mod pool size)
    t0 = time.perf_counter()
    pool = scenes.ensemble(n_scenes=args.pool, seed=4, steps=2000)
    say(f"request pool of {len(pool)} scenes generated in {time.perf_counter() - t0:.1f} s")
    rates = [float(r) for r in args.rates.split(",")]
    runs = []
    for lam in rates:
        arrivals = serve.poisson_arrivals(lam, args.serve_seconds, seed=4)
        reqs = [serve.Request(i, float(a), (lambda s=pool[i % len(pool)]: s), max_steps=2000)
                for i, a in enumerate(arrivals)]
        srv = serve.Server(int(args.budget_gib * (1 << 30)), max_scenes=args.max_scenes,
                           stream=stream, background_builds=not args.sync_builds)
        say(f"rate {lam:g}/s: {len(reqs)} requests over {args.serve_seconds:g} s")
        out = srv.run(reqs, stop_admitting_at=args.serve_seconds, drain=False,
                      deadline=args.serve_seconds)
        torch.cuda.synchronize()
        out.pop("results")
        out["rate_per_s"] = lam
        say(f"   {json.dumps(out)}")
        runs.append(out)
    best = max(runs, key=lambda r: r["ped_steps_per_s"])
    out = {"metric": METRIC, "value": best["ped_steps_per_s"], "unit": "pedestrian-steps/s",
           "n_gpus": 1, "steps": None, "warmup": 0, "ms_per_step": best["step_latency_ms_p50"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "serving", "rates_per_s": rates,
                      "window_s": args.serve_seconds, "max_steps": 2000,
                      "budget_gib": args.budget_gib, "max_scenes": args.max_scenes,
                      "request_pool": len(pool),
                      "builds": "between ticks" if args.sync_builds else "worker thread",
                      "parallelism": "single-gpu"},
           "runs": runs, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed ticks (default: the workload's own tick count)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="hall1024",
                    choices=["hall1024", "room64", "plaza8192", "flow1000", "flow-sweep",
                             "flow-walk", "ensemble256", "serving"])
    ap.add_argument("--scenes", type=int, default=256, help="ensemble size (ensemble256)")
    ap.add_argument("--rates", default="50,200,800", help="arrival rates per s (serving)")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="arrival window per rate (serving)")
    ap.add_argument("--sync-builds", action="store_true",
                    help="serving: build admitted scenes between ticks, not on a worker thread")
    ap.add_argument("--budget-gib", type=float, default=64.0,
                    help="device memory admitted scenes may hold (serving)")
    ap.add_argument("--max-scenes", type=int, default=256, help="resident slots (serving)")
    ap.add_argument("--pool", type=int, default=64, help="request pool size (serving)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--sweep-sides", default="100,200,300,400,500,600,700,800,900,1000",
                    help="flow-sweep: torus sides")
    ap.add_argument("--sweep-densities", default="0.1,0.2,0.3,0.4,0.5,0.6,0.7,0.8,0.9",
                    help="flow-sweep: pedestrians per su")
    ap.add_argument("--sweep-directions", default="1,2,4,8", help="flow-sweep: flow directions")
    ap.add_argument("--field-update", type=int, default=0,
                    help="K >= 2: incremental field update with a full superposition every K "
                         "ticks (sf_set_field_update); 0 = full superposition every tick")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="hall1024: skip the attached batched-vs-plain ensemble comparison")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (HBM "
                         "counter calibration under rocprofv3) and exit")
    args = ap.parse_args()
    if args.copy_probe_mib:
        import torch

        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "path is described in the design notes, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1803_04782_amd import scenes, sf

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.workload == "ensemble256":
        bench_ensemble(args, stream)
        return
    if args.workload == "serving":
        bench_serving(args, stream)
        return
    if args.workload == "flow-sweep":
        bench_flow_sweep(args, stream)
        return
    if args.workload == "flow-walk":
        bench_flow_walk(args, stream)
        return
    sc = scenes.WORKLOADS[args.workload]()
    if args.steps is None:
        args.steps = sc.steps
    print(f"[bench] workload {sc.name}: {sc.width}x{sc.height} su, {sc.n_peds} pedestrians, "
          f"R={sc.radius}", file=sys.stderr, flush=True)
    free_su = int((sc.obstacle == 0).sum())
    g = sf.GpuScene(sc, stream=stream)
    if args.field_update:
        g.set_field_update(args.field_update)
    try:
        # warm-up ticks, then back to the initial state for the timed run
        g.step(args.warmup)
        g.set_state(sc.pos, sc.start_step)
        torch.cuda.synchronize()

        t0 = time.perf_counter()
        g.step(args.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s = g.stats()
        ped_steps = s["ped_steps"]

        # same ticks again with HIP events around every kernel launch
        g.set_state(sc.pos, sc.start_step)
        g.set_timing(True)
        g.step(args.steps)
        torch.cuda.synchronize()
        ktimes = {}
        for name, kid in (("superpose", sf.SF_KERNEL_SUPERPOSE), ("decide", sf.SF_KERNEL_DECIDE),
                          ("commit", sf.SF_KERNEL_COMMIT)):
            ms, n = g.kernel_time(kid)
            ktimes[name] = {"avg_us": 1000.0 * ms / max(n, 1), "launches": n}
        g.set_timing(False)
        s2 = g.stats()

        # the field kernel alone, back to back: FIELD_LOOP superpositions of
        # the final state (sf_refresh_field; the field stays the same bit for
        # bit), two HIP events around the loop on the scene's stream.  The
        # per-launch events above cost the host more per launch than a tick
        # takes on the device, so those launches run with idle gaps before
        # them and their start-to-stop intervals read high.
        g.refresh_field(10)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.refresh_field(FIELD_LOOP)
        e1.record(stream)
        torch.cuda.synchronize()
        field_loop_us = 1000.0 * e0.elapsed_time(e1) / FIELD_LOOP

        # final state for the accuracy gate
        pos_g = g.positions()
        P_g = g.field()
        t_g = g.stats()["step"]
        g.step(1)
        tgt_g, flags_g = g.last_moves()
        pos_next = g.positions()
    finally:
        g.close()

    value = ped_steps / dt
    su_updates = args.steps * free_su / dt
    contrib_per_launch = (s2["ped_steps"] / max(args.steps, 1)) * window_contributions(sc)
    sup_us = field_loop_us
    achieved = contrib_per_launch / (sup_us * 1e-6) / 1e12
    # algorithmic bytes of one superposition launch: S (FP64) read and P
    # (FP32) written once, the bitmap read once
    # per su, the occupancy bitmap read once
    alg_bytes = 12.0 * sc.width * sc.height + 8.0 * ((sc.width + 63) // 64) * sc.height
    roofline = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / ALU_PEAK_TFLOPS,
                "traffic": traffic_per_launch(), "kernel": "superpose",
                "flop_per_launch": contrib_per_launch, "avg_launch_us": sup_us,
                "launch_timing": f"{FIELD_LOOP} back-to-back field launches on the final state, "
                                 "HIP events around the loop",
                "tick_launch_interval_us": ktimes["superpose"]["avg_us"],
                "algorithmic_bytes_per_launch": alg_bytes,
                "hbm_frac": alg_bytes / (sup_us * 1e-6) / 8.0e12}
    # measured HBM rate (calibrated counters over the launch duration) and the
    # launch's floor at peak: max(algorithmic bytes / 8 TB/s, adds / ALU rate)
    if roofline["traffic"] is not None:
        roofline["measured_hbm_GBps"] = roofline["traffic"] / (sup_us * 1e-6) / 1e9
    t_hbm = alg_bytes / 8.0e12
    t_alu = contrib_per_launch / (ALU_PEAK_TFLOPS * 1e12)
    roofline["floor_us"] = 1e6 * max(t_hbm, t_alu)
    roofline["floor_binding"] = "alu" if t_alu >= t_hbm else "hbm"

    out = {"metric": METRIC, "value": value, "unit": "pedestrian-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000.0 * dt / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "field_us_per_tick": ktimes["superpose"]["avg_us"] * ktimes["superpose"]["launches"]
           / max(args.steps, 1),
           "data": "synthetic", "config": {"workload": sc.name, "grid": [sc.width, sc.height],
                                           "field_update": args.field_update,
                                           "pedestrians": sc.n_peds, "radius": sc.radius,
                                           "ticks": args.steps, "parallelism": "single-gpu"},
           "su_field_updates_per_s": su_updates, "kernels": ktimes, "roofline": roofline,
           "stats": s}
    if args.workload == "flow1000":
        out["config"].update({"periodic": True, "density": 0.5, "directions": 8})
        out["paper_context"] = PAPER_FLOW1000
    if not args.no_cpu:
        base, gate = cpu_baseline(sc, (pos_g, P_g, t_g, tgt_g, flags_g, pos_next),
                                  args.cpu_seconds)
        out["cpu_baseline"] = base
        out["accuracy_gate"] = gate
    else:
        out["cpu_baseline"] = None
    if args.workload == "hall1024" and not args.no_ensemble:
        # the metric's batched-vs-plain half: the 256-scene ensemble, 300 ticks
        e = bench_ensemble(args, stream, steps=300, emit=False)
        out["ensemble256"] = {k: e[k] for k in ("value", "unit", "ms_per_step", "steps",
                                                "su_field_updates_per_s", "plain",
                                                "batched_vs_plain", "tiling",
                                                "identical_to_plain", "accuracy_gate")}
        out["ensemble256"]["config"] = e["config"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
