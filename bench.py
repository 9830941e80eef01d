"""Benchmark of the social-field tick on one MI355X.

Default line (the metric's configuration): the batched ensemble of 256
uneven scenes (sides 128..2048 su, obstacle cover 0..10%, 1..10% occupancy,
radii 4/8/16/32, 1..4 exits), synthetic and seeded.  A "step" is one tick of
the whole hot path for every scene: bin, decide + claim, commit, superpose.
Inputs are resident in HBM when the timed region starts.  The batch (one
decide, commit and field launch per group per tick, graph replays, autotuned
tiling) is timed over K ticks five times from the same reset state, and the
median run is `value`; the plain loop of per-scene sf_step ticks is timed the
same way for `batched_vs_plain`.  The line carries the roofline of the
batched field superposition (HIP events around back-to-back field passes),
the FP64 oracle timed on all host cores on a bounded sample, an accuracy
gate against the oracle, and sub-objects: "hall1024" and "plaza8192"
(single scenes, each with its own roofline and accuracy gate) and "serving"
(a short continuous-batching leg at 50, 200 and 800 arrivals/s).

Other workloads (--workload): hall1024, room64, plaza8192 (one scene each),
serving (longer windows), flow1000 (the paper's section 5 scenario: a
1000x1000 torus, density 0.5, 8-directional flow, 7x7 fields, 1000 ticks),
flow-sweep (its 360-combination grid), flow-walk (its walk-period
experiment of Table V) and sect-compare (the paper's own 8-sect, K-slot FP32
field path against the exact gather: speed and error) and ensemble-classes
(the ensemble's batched field pass by radius class).
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
# The field is summed with one FP64 add per (pedestrian, su) contribution.
# MI355X issues one FP64 add (or FMA) per lane per clock: 256 CUs x 64 lanes
# x 2.4 GHz = 39.3e12 adds/s (the 78.6 TFLOP/s FP64 vector peak counts an FMA
# as two flops).
ALU_PEAK_TFLOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK = 8.0e12
# back-to-back field launches timed for the roofline
FIELD_LOOP = 200
# host threads of the oracle: the cores a GPU machine grants one GPU's job
ORACLE_THREADS_CAP = 16
KERNEL_SRC = os.path.join(ROOT, "paper_1803_04782_amd", "csrc", "sf_kernels.hip")
PMC_DIR = os.path.join(ROOT, "profiles")


def say(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def host_info() -> dict:
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def oracle_threads() -> int:
    import oracle

    return min(ORACLE_THREADS_CAP, oracle.host_threads())


def contributions(W, H, R, periodic, pos) -> float:
    """(pedestrian, su) pairs of the live pedestrians: su inside the grid and
    the pedestrian's window, own su excluded (one FP64 add each)."""
    live = np.asarray(pos)
    live = live[live >= 0]
    if periodic:
        return float(live.size) * ((2 * R + 1) ** 2 - 1)  # a torus: every window is whole
    x, y = live % W, live // W
    wx = np.minimum(x + R, W - 1) - np.maximum(x - R, 0) + 1
    wy = np.minimum(y + R, H - 1) - np.maximum(y - R, 0) + 1
    return float(np.sum(wx * wy - 1))


def field_bytes(W, H) -> float:
    """Algorithmic bytes of one field pass: S (FP64) read and P (FP32)
    written once per su, the occupancy bitmap read once."""
    return 12.0 * W * H + 8.0 * ((W + 63) // 64) * H


def traffic_per_launch(name):
    """HBM bytes per field launch from the committed rocprofv3 PMC summary
    profiles/superpose_<name>_pmc.json, if it was taken on the current kernel source."""
    try:
        d = json.load(open(os.path.join(PMC_DIR, f"superpose_{name}_pmc.json")))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def roofline(contrib, nbytes, launch_us, kernel, timing, traffic_name):
    achieved = contrib / (launch_us * 1e-6) / 1e12
    r = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
         "frac": achieved / ALU_PEAK_TFLOPS, "traffic": traffic_per_launch(traffic_name),
         "kernel": kernel, "flop_per_launch": contrib, "avg_launch_us": launch_us,
         "launch_timing": timing, "algorithmic_bytes_per_launch": nbytes,
         "hbm_frac": nbytes / (launch_us * 1e-6) / HBM_PEAK}
    if r["traffic"] is not None:
        r["measured_hbm_GBps"] = r["traffic"] / (launch_us * 1e-6) / 1e9
    t_hbm, t_alu = nbytes / HBM_PEAK, contrib / (ALU_PEAK_TFLOPS * 1e12)
    r["floor_us"] = 1e6 * max(t_hbm, t_alu)
    r["floor_binding"] = "alu" if t_alu >= t_hbm else "hbm"
    return r


def windows(k: int, n: int = 5):
    """k timed ticks split into up to n windows of near-equal length."""
    n = max(1, min(n, k))
    return [k // n + (1 if i < k % n else 0) for i in range(n)]


def gate_tick(st, pos, P_g, t, tgt_g, flags_g, pos_next, threads):
    """One tick of a GPU scene against the oracle's full tick: field bits,
    relative error and mismatched decisions (the parity bar)."""
    import oracle

    r = oracle.step(st, pos, t, threads=threads)
    free = st.obstacle == 0
    err = 0.0
    if free.any():
        err = float(np.max(np.abs(P_g[free] - r.P[free]) / np.maximum(np.abs(r.P[free]), 1.0)))
    live = pos >= 0
    won = (flags_g & 2) != 0
    bad = live & ((tgt_g != r.target) | (won != (r.moved == 1)) | (pos_next != r.pos))
    hot = set(r.target[live & (r.tied == 1)].tolist()) | set(tgt_g[live & (r.tied == 1)].tolist())
    untied = [j for j in np.flatnonzero(bad)
              if not r.tied[j] and r.target[j] not in hot and tgt_g[j] not in hot
              and pos[j] not in hot]
    return {"field_su_differing": int(np.count_nonzero(P_g != r.P.astype(np.float32))),
            "field_rel_err": err, "untied_mismatches": len(untied),
            "tied_mismatches": int(bad.sum()) - len(untied),
            "near_tie_decisions": int(r.tied[live].sum()), "decisions": int(live.sum())}


def merge_gates(gates):
    out = {"field_su_differing": 0, "field_rel_err": 0.0, "untied_mismatches": 0,
           "tied_mismatches": 0, "near_tie_decisions": 0, "decisions": 0}
    for g in gates:
        for k in out:
            out[k] = max(out[k], g[k]) if k == "field_rel_err" else out[k] + g[k]
    return out


def oracle_sample(items, seconds, threads):
    """The FP64 oracle as it stands on a bounded sample: for each (statics,
    positions, tick) the oracle's full tick (field on `threads` threads);
    statics are built outside the timed region (scene creation)."""
    import oracle

    live_sum, ticks, t_run = 0, 0, 0.0
    for make, label in items:
        st, pos, t = make()
        while True:
            t0 = time.perf_counter()
            r = oracle.step(st, pos, t, threads=threads)
            t_run += time.perf_counter() - t0
            live_sum += int((pos >= 0).sum())
            ticks += 1
            pos, t = r.pos, t + 1
            if t_run >= seconds or label == "one":
                break
        if t_run >= seconds:
            break
    return live_sum, ticks, t_run


def cpu_baseline_dict(live_sum, ticks, t_run, threads, sample):
    d = {"value": live_sum / t_run if t_run > 0 else None, "unit": "pedestrian-steps/s",
         "cores": threads, "kind": "oracle", "sample": sample, "timed_s": t_run,
         "ticks": ticks}
    d.update(host_info())
    return d


def single_scene(sc, args, stream, steps, field_loop, cpu_seconds, kernel_label):
    """One scene: `steps` timed ticks after warm-up (from the initial state),
    per-kernel events, the field roofline from back-to-back launches, a
    one-tick accuracy gate and the oracle baseline."""
    import torch

    import oracle
    from paper_1803_04782_amd import sf

    threads = oracle_threads()
    free_su = int((sc.obstacle == 0).sum())
    t0 = time.perf_counter()
    g = sf.GpuScene(sc, stream=stream)
    say(f"{sc.name}: {sc.width}x{sc.height} su, {sc.n_peds} pedestrians, R={sc.radius}, "
        f"created in {time.perf_counter() - t0:.1f} s")
    if args.field_update:
        g.set_field_update(args.field_update)
    try:
        g.step(args.warmup)
        g.set_state(sc.pos, sc.start_step)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s = g.stats()
        # same ticks again with HIP events around every kernel launch
        g.set_state(sc.pos, sc.start_step)
        g.set_timing(True)
        g.step(steps)
        torch.cuda.synchronize()
        ktimes = {}
        for name, kid in (("superpose", sf.SF_KERNEL_SUPERPOSE), ("decide", sf.SF_KERNEL_DECIDE),
                          ("commit", sf.SF_KERNEL_COMMIT)):
            ms, n = g.kernel_time(kid)
            ktimes[name] = {"avg_us": 1000.0 * ms / max(n, 1), "launches": n}
        g.set_timing(False)
        # the field alone, back to back on the final state (the field keeps
        # its bits), two HIP events around the loop on the scene's stream
        pos_end = g.positions()
        g.refresh_field(5)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.refresh_field(field_loop)
        e1.record(stream)
        torch.cuda.synchronize()
        field_us = 1000.0 * e0.elapsed_time(e1) / field_loop
        # accuracy gate: the next tick against the oracle's full tick
        P_g = g.field()
        t_g = g.stats()["step"]
        g.step(1)
        tgt_g, flags_g = g.last_moves()
        pos_next = g.positions()
    finally:
        g.close()
    st = oracle.statics(sc, threads=threads)
    gate = gate_tick(st, pos_end, P_g, t_g, tgt_g, flags_g, pos_next, threads)
    gate["tick"] = int(t_g)
    contrib = contributions(sc.width, sc.height, sc.radius, sc.periodic, pos_end)
    out = {"value": s["ped_steps"] / dt, "unit": "pedestrian-steps/s", "steps": steps,
           "ms_per_step": 1000.0 * dt / steps,
           "su_field_updates_per_s": steps * free_su / dt,
           "config": {"workload": sc.name, "grid": [sc.width, sc.height],
                      "pedestrians": sc.n_peds, "radius": sc.radius, "ticks": steps,
                      "field_update": args.field_update},
           "kernels": ktimes,
           "roofline": roofline(contrib, field_bytes(sc.width, sc.height), field_us, kernel_label,
                                f"{field_loop} back-to-back field launches on the final state, "
                                "HIP events around the loop on the scene's stream", sc.name),
           "accuracy_gate": gate, "stats": s}
    out["roofline"]["tick_launch_interval_us"] = ktimes["superpose"]["avg_us"]
    if cpu_seconds > 0:
        live_sum, ticks, t_run = oracle_sample(
            [(lambda: (st, sc.pos.copy(), sc.start_step), "run")], cpu_seconds, threads)
        out["cpu_baseline"] = cpu_baseline_dict(
            live_sum, ticks, t_run, threads,
            f"first {ticks} ticks of {sc.name} from its initial state (FP64 C oracle, field on "
            f"{threads} threads, {t_run:.1f} s)")
    else:
        out["cpu_baseline"] = None
    return out


def ensemble_line(args, stream, steps):
    """Batched vs plain on the uneven ensemble: the default line's headline."""
    import torch

    import oracle
    from paper_1803_04782_amd import scenes, sf

    threads = oracle_threads()
    t0 = time.perf_counter()
    scs = scenes.ensemble(n_scenes=args.scenes, seed=3)
    su_total = sum(s.width * s.height for s in scs)
    free_total = sum(int((s.obstacle == 0).sum()) for s in scs)
    peds_total = sum(s.n_peds for s in scs)
    say(f"ensemble of {len(scs)} scenes: {su_total:.3g} su, {peds_total} pedestrians "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    plain = [sf.GpuScene(s, stream=stream) for s in scs]
    member = [sf.GpuScene(s, stream=stream) for s in scs]
    say(f"created {2 * len(scs)} scenes in {time.perf_counter() - t0:.1f} s")
    fixed = json.loads(args.tiling) if args.tiling else None
    b = sf.Batch(member, tiling=fixed, stream=stream)
    wins = windows(steps)
    try:
        t0 = time.perf_counter()
        if fixed is None:
            tiling = b.tune(reps=3)
            say(f"autotuned tiling {tiling} in {time.perf_counter() - t0:.1f} s")
        else:
            tiling = b.tiling()
            say(f"tiling as given: {tiling}")
        for _ in range(args.warmup):
            for g in plain:
                g.step(1)
        b.step(args.warmup)
        torch.cuda.synchronize()

        def ped_steps_plain():
            return sum(g.stats()["ped_steps"] for g in plain)

        def ped_steps_batch():
            return sum(x["ped_steps"] for x in b.stats())

        runs_p, runs_b = [], []
        for k in wins:
            ps0 = ped_steps_plain()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                for g in plain:
                    g.step(1)
            torch.cuda.synchronize()
            runs_p.append((k, time.perf_counter() - t0, ped_steps_plain() - ps0))
        for k in wins:
            ps0 = ped_steps_batch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.step(k)
            torch.cuda.synchronize()
            runs_b.append((k, time.perf_counter() - t0, ped_steps_batch() - ps0))
        dt_p = sum(r[1] for r in runs_p)
        dt_b = sum(r[1] for r in runs_b)
        ps_p = sum(r[2] for r in runs_p)
        ps_b = sum(r[2] for r in runs_b)
        say(f"plain: {steps} ticks in {dt_p:.3f} s; batched: {dt_b:.3f} s")
        totals = b.stats()

        # the batched field alone, back to back, HIP events on the batch's stream
        pos_all = [m.positions() for m in member]
        contrib = sum(contributions(s.width, s.height, s.radius, s.periodic, p)
                      for s, p in zip(scs, pos_all))
        nbytes = sum(field_bytes(s.width, s.height) for s in scs)
        loops = 20
        b.refresh_field(2)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.refresh_field(loops)
        e1.record(stream)
        torch.cuda.synchronize()
        pass_us = 1000.0 * e0.elapsed_time(e1) / loops
        n_groups = tiling["groups"]

        # the two runs agree bit for bit (positions of every scene, fields of
        # the 16 smallest); one full tick of the 8 smallest and the largest
        # scene against the oracle
        order = np.argsort([s.width * s.height for s in scs])
        same_pos = all(np.array_equal(a.positions(), m.positions()) for a, m in zip(plain, member))
        same_field = all(np.array_equal(plain[j].field(), member[j].field()) for j in order[:16])
        checked = [int(j) for j in order[:8]] + [int(order[-1])]
        before = []
        for j in checked:
            before.append((j, pos_all[j], member[j].field(), totals[j]["step"]))
        b.step(1)
        gates = []
        for j, pos, P_g, t in before:
            st = oracle.statics(scs[j], threads=threads)
            tgt_g, flags_g = member[j].last_moves()
            gates.append(gate_tick(st, pos, P_g, t, tgt_g, flags_g, member[j].positions(),
                                   threads))
        gate = merge_gates(gates)
        gate["scenes"] = len(checked)
    finally:
        b.close()
        for g in plain + member:
            g.close()

    # the oracle on all host cores: one tick of scenes in a seeded random
    # order, each from its initial state, bounded to args.cpu_seconds
    rng = np.random.default_rng(7)
    pick = [int(j) for j in rng.permutation(len(scs))]
    items = [((lambda j=j: (oracle.statics(scs[j], threads=threads), scs[j].pos.copy(),
                             scs[j].start_step)), "one") for j in pick]
    live_sum, ticks, t_run = oracle_sample(items, args.cpu_seconds, threads)
    base = cpu_baseline_dict(
        live_sum, ticks, t_run, threads,
        f"first tick of {ticks} ensemble scenes in a seeded random order, each from its "
        f"initial state (FP64 C oracle, field on {threads} threads, {t_run:.1f} s; statics "
        "built outside the timed region)")

    rate_b = [r[2] / r[1] for r in runs_b]
    rate_p = [r[2] / r[1] for r in runs_p]
    field_label = ("superpose (batched: " + ("one launch" if n_groups == 1 else
                                             f"{n_groups} launches, one per radius group")
                   + " per pass)")
    out = {"metric": METRIC, "value": ps_b / dt_b, "unit": "pedestrian-steps/s", "n_gpus": 1,
           "steps": steps, "warmup": args.warmup, "ms_per_step": 1000.0 * dt_b / steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"ensemble{len(scs)}", "scenes": len(scs), "su": su_total,
                      "pedestrians": peds_total, "ticks": steps, "sides": [128, 2048],
                      "radii": [4, 8, 16, 32], "parallelism": "single-gpu"},
           "su_field_updates_per_s": steps * free_total / dt_b,
           "windows": {"ticks": wins, "batched_rate_median": float(np.median(rate_b)),
                       "batched_rates": rate_b, "plain_rate_median": float(np.median(rate_p)),
                       "plain_rates": rate_p},
           "plain": {"value": ps_p / dt_p, "ms_per_step": 1000.0 * dt_p / steps},
           "batched_vs_plain": (ps_b / dt_b) / (ps_p / dt_p),
           "batched_vs_plain_median": float(np.median(rate_b) / np.median(rate_p)),
           "tiling": tiling,
           "identical_to_plain": {"positions_all_scenes": bool(same_pos),
                                  "fields_16_smallest": bool(same_field)},
           "accuracy_gate": gate,
           "roofline": roofline(contrib, nbytes, pass_us, field_label,
                                f"{loops} back-to-back batched field passes on the final state "
                                "(sf_batch_refresh_field), HIP events around the loop on the "
                                "batch's stream", "ensemble256"),
           "cpu_baseline": base}
    return out


def serving_leg(args, stream):
    """A short continuous-batching leg at each arrival rate."""
    import torch

    from paper_1803_04782_amd import scenes, serve

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
        say(f"serving at {lam:g}/s: {len(reqs)} requests over {args.serve_seconds:g} s")
        # arrivals for serve_seconds, then the resident scenes keep running
        # (up to serve_seconds + drain_seconds) so that finished scenes count
        out = srv.run(reqs, stop_admitting_at=args.serve_seconds, drain=args.drain_seconds > 0,
                      deadline=args.serve_seconds + args.drain_seconds)
        torch.cuda.synchronize()
        out.pop("results")
        out["rate_per_s"] = lam
        say(f"   p50/p99 step {out['step_latency_ms_p50']:.2f}/{out['step_latency_ms_p99']:.2f} "
            f"ms, {out['scenes_per_s']:.2f} scenes/s, {out['ped_steps_per_s']:.3g} ped-steps/s")
        runs.append(out)
    return {"rates_per_s": rates, "window_s": args.serve_seconds,
            "drain_s": args.drain_seconds, "max_steps": 2000,
            "budget_gib": args.budget_gib, "max_scenes": args.max_scenes,
            "request_pool": len(pool),
            "builds": "between ticks" if args.sync_builds else "worker thread", "runs": runs}


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
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
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
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "flow-walk", "grid": [1000, 1000], "density": 0.5,
                      "directions": 8, "radius": 3, "periodic": True, "ticks": steps,
                      "max_walk_periods": [r["max_walk_period"] for r in rows],
                      "parallelism": "single-gpu"},
           "runs": rows, "paper_context": {"source": "Table V, current GPU model",
                                           "hardware": PAPER_FLOW1000["hardware"]},
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_sect_compare(args, stream):
    """The paper's own field path (8 sects, fan-out terms, Algorithm 3's K
    FP32 slots; sf_set_field_sect) against the exact gather on flow1000 (7x7
    fields) and hall1024 (R = 16): field launch time (back-to-back launches,
    HIP events), tick time, the FP32 field's error against the exact field and
    the decisions of one tick that differ from the exact path's."""
    import torch

    from paper_1803_04782_amd import scenes, sf

    steps = args.steps if args.steps is not None else 100
    loops = 50
    rows = []
    for sc in (scenes.flow1000(), scenes.hall1024()):
        for K in (0, 2, 4, 8, 16):
            for refresh in (0, 8):
                g = sf.GpuScene(sc, stream=stream)
                ref = sf.GpuScene(sc, stream=stream)
                try:
                    if refresh:
                        g.set_field_update(refresh)
                    if K:
                        g.set_field_sect(K)
                    g.step(args.warmup)
                    g.set_state(sc.pos, sc.start_step)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    g.step(steps)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    ps = g.stats()["ped_steps"]
                    # field launches back to back on the final state
                    g.refresh_field(3)
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    g.refresh_field(loops)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    field_us = 1000.0 * e0.elapsed_time(e1) / loops
                    # error and decisions against the exact path from the same state
                    pos = g.positions()
                    t_now = g.stats()["step"]
                    ref.set_state(pos, t_now)
                    P, Pe = g.field(), ref.field()
                    free = np.isfinite(Pe)
                    rel = np.abs(P[free].astype(np.float64) - Pe[free]) / np.maximum(
                        np.abs(Pe[free].astype(np.float64)), 1.0)
                    g.step(1)
                    ref.step(1)
                    tg, _ = g.last_moves()
                    te, _ = ref.last_moves()
                    live = pos >= 0
                finally:
                    g.close()
                    ref.close()
                row = {"workload": sc.name, "K": K, "path": "sect" if K else "gather",
                       "refresh": refresh, "ms_per_tick": 1000.0 * dt / steps,
                       "pedestrian_steps_per_s": ps / dt, "field_launch_us": field_us,
                       "field_max_rel_err": float(rel.max()) if rel.size else 0.0,
                       "field_su_differing": int(np.count_nonzero(P[free] != Pe[free])),
                       "decisions_differing": int(np.count_nonzero(live & (tg != te))),
                       "decisions": int(live.sum())}
                rows.append(row)
                say(f"{sc.name} {row['path']} K={K} refresh={refresh}: tick "
                    f"{row['ms_per_tick'] * 1000:.1f} us, field {field_us:.1f} us, max rel err "
                    f"{row['field_max_rel_err']:.2e}, {row['decisions_differing']} decisions "
                    "differ")
    out = {"metric": METRIC, "value": None, "unit": "pedestrian-steps/s", "n_gpus": 1,
           "steps": steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 (sect path) / f64 (gather)", "data": "synthetic",
           "config": {"workload": "sect-compare", "parallelism": "single-gpu"},
           "runs": rows, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_ensemble_classes(args, stream):
    """The ensemble's field pass by radius class: the scenes of each radius as
    a one-group batch (tuned), back-to-back field passes timed with HIP
    events; beside each, the class's contributions and its HBM and ALU
    floors, and the default grouping of all 256 scenes."""
    import torch

    from paper_1803_04782_amd import scenes, sf

    scs = scenes.ensemble(n_scenes=args.scenes, seed=3)
    loops = 10

    def timed(b):
        b.refresh_field(2)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.refresh_field(loops)
        e1.record(stream)
        torch.cuda.synchronize()
        return 1000.0 * e0.elapsed_time(e1) / loops

    rows = []
    for R in sorted({s.radius for s in scs}):
        sub = [s for s in scs if s.radius == R]
        gs = [sf.GpuScene(s, stream=stream) for s in sub]
        try:
            with sf.Batch(gs, tiling={"groups": 1}, stream=stream) as b:
                tiling = b.tune(reps=2)
                us = timed(b)
        finally:
            for g in gs:
                g.close()
        su = sum(s.width * s.height for s in sub)
        contrib = sum(contributions(s.width, s.height, s.radius, s.periodic, s.pos) for s in sub)
        nbytes = sum(field_bytes(s.width, s.height) for s in sub)
        rows.append({"radius": R, "scenes": len(sub), "su": su, "contributions": contrib,
                     "pass_us": us, "hbm_floor_us": 1e6 * nbytes / HBM_PEAK,
                     "alu_floor_us": 1e6 * contrib / (ALU_PEAK_TFLOPS * 1e12),
                     "tiling": tiling["group"][0]})
        say(f"R={R}: {len(sub)} scenes, field pass {us:.1f} us")
    gs = [sf.GpuScene(s, stream=stream) for s in scs]
    try:
        with sf.Batch(gs, stream=stream) as b:
            tiling = b.tune(reps=2)
            all_us = timed(b)
    finally:
        for g in gs:
            g.close()
    out = {"metric": METRIC, "value": None, "unit": "us per field pass", "n_gpus": 1,
           "steps": None, "warmup": 2, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "i32 sums (exact)", "data": "synthetic",
           "config": {"workload": "ensemble-classes", "scenes": len(scs),
                      "parallelism": "single-gpu"},
           "classes": rows, "default_groups": {"pass_us": all_us, "tiling": tiling},
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_serving(args, stream):
    """Serving loop under Poisson arrivals at several rates (longer windows
    than the default line's leg)."""
    leg = serving_leg(args, stream)
    best = max(leg["runs"], key=lambda r: r["ped_steps_per_s"])
    cfg = {k: v for k, v in leg.items() if k != "runs"}
    cfg.update({"workload": "serving", "parallelism": "single-gpu"})
    out = {"metric": METRIC, "value": best["ped_steps_per_s"], "unit": "pedestrian-steps/s",
           "n_gpus": 1, "steps": None, "warmup": 0, "ms_per_step": best["step_latency_ms_p50"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": cfg, "runs": leg["runs"], "roofline": None,
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def line_for_single(sub, args):
    """A single-scene result as the top-level JSON line of its workload."""
    out = {"metric": METRIC, "value": sub["value"], "unit": sub["unit"], "n_gpus": 1,
           "steps": sub["steps"], "warmup": args.warmup, "ms_per_step": sub["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic"}
    out.update({k: v for k, v in sub.items() if k not in out})
    out["config"]["parallelism"] = "single-gpu"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed ticks (default: the workload's own tick count)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="default",
                    choices=["default", "ensemble256", "hall1024", "room64", "plaza8192",
                             "flow1000", "flow-sweep", "flow-walk", "serving",
                             "sect-compare", "ensemble-classes"])
    ap.add_argument("--scenes", type=int, default=256, help="ensemble size (ensemble256)")
    ap.add_argument("--tiling", default=None,
                    help="ensemble256: batch tiling as JSON instead of the autotuner's "
                         "(for counter runs whose kernels must all be the timed ones)")
    ap.add_argument("--rates", default="50,200,800", help="arrival rates per s (serving)")
    ap.add_argument("--serve-seconds", type=float, default=None,
                    help="arrival window per rate (serving; default 30 s alone, 4 s in the "
                         "default line)")
    ap.add_argument("--drain-seconds", type=float, default=None,
                    help="serving: after the arrival window, keep ticking the resident scenes "
                         "for up to this long (default 0 alone, 6 s in the default line)")
    ap.add_argument("--sync-builds", action="store_true",
                    help="serving: build admitted scenes between ticks, not on a worker thread")
    ap.add_argument("--budget-gib", type=float, default=64.0,
                    help="device memory admitted scenes may hold (serving)")
    ap.add_argument("--max-scenes", type=int, default=256, help="resident slots (serving)")
    ap.add_argument("--pool", type=int, default=None,
                    help="request pool size (serving; default 64 alone, 32 in the default line)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--no-subs", action="store_true",
                    help="default line: skip the hall1024, plaza8192 and serving sub-objects")
    ap.add_argument("--sweep-sides", default="100,200,300,400,500,600,700,800,900,1000",
                    help="flow-sweep: torus sides")
    ap.add_argument("--sweep-densities", default="0.1,0.2,0.3,0.4,0.5,0.6,0.7,0.8,0.9",
                    help="flow-sweep: pedestrians per su")
    ap.add_argument("--sweep-directions", default="1,2,4,8", help="flow-sweep: flow directions")
    ap.add_argument("--field-update", type=int, default=0,
                    help="K >= 2: incremental field update with a full superposition every K "
                         "ticks (sf_set_field_update); 0 = full superposition every tick")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="bound on the timed oracle work of each CPU baseline")
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

    from paper_1803_04782_amd import scenes

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.no_cpu:
        args.cpu_seconds = 0.0
    if args.workload == "serving":
        args.serve_seconds = args.serve_seconds or 30.0
        args.drain_seconds = args.drain_seconds or 0.0
        args.pool = args.pool or 64
        bench_serving(args, stream)
        return
    if args.workload == "flow-sweep":
        bench_flow_sweep(args, stream)
        return
    if args.workload == "flow-walk":
        bench_flow_walk(args, stream)
        return
    if args.workload == "sect-compare":
        bench_sect_compare(args, stream)
        return
    if args.workload == "ensemble-classes":
        bench_ensemble_classes(args, stream)
        return
    if args.workload in ("default", "ensemble256"):
        t_start = time.perf_counter()
        steps = args.steps if args.steps is not None else 300
        out = ensemble_line(args, stream, steps)
        if args.workload == "default" and not args.no_subs:
            # the metric's single-scene configurations, each with its roofline
            sub_cpu = min(args.cpu_seconds, 5.0)
            out["hall1024"] = single_scene(scenes.hall1024(), args, stream, 500, FIELD_LOOP,
                                           sub_cpu, "superpose")
            out["plaza8192"] = single_scene(scenes.plaza8192(), args, stream, 200, 50,
                                            sub_cpu, "superpose")
            args.serve_seconds = args.serve_seconds or 4.0
            args.drain_seconds = 6.0 if args.drain_seconds is None else args.drain_seconds
            args.pool = args.pool or 32
            out["serving"] = serving_leg(args, stream)
        out["bench_wall_s"] = time.perf_counter() - t_start
        print(json.dumps(out), flush=True)
        return
    sc = scenes.WORKLOADS[args.workload]()
    steps = args.steps if args.steps is not None else sc.steps
    sub = single_scene(sc, args, stream, steps, FIELD_LOOP, args.cpu_seconds, "superpose")
    out = line_for_single(sub, args)
    if args.workload == "flow1000":
        out["config"].update({"periodic": True, "density": 0.5, "directions": 8})
        out["paper_context"] = PAPER_FLOW1000
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
