"""Throughput of the constraint-matrix hot path on one MI355X.

One step = one time step of the fast scheme through the C ABI (icr_step):
free motion, contact selection, W_H = H A^-1 H^T, n_newton x (frames,
W = C W_H C^T, PGS, proximity GEMV), corrective motion.  The metric scope of
the paper's Table 1 ("Total" = build W_H + Newton iterations) is reported
beside the whole step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config precision]

Prints one JSON line.  Inputs are seeded synthetic scenes (see
paper_2306_06946_amd/scenes.py) resident on the GPU before timing starts.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def supernode_ranges(analysis, node_ids):
    """Number of contacts below every supernode (host bookkeeping for flop counts)."""
    perm, sup = analysis["perm"], analysis["sup"]
    N = len(perm)
    owner = np.empty(N, dtype=np.int64)
    for s, (c0, nc, _, _) in enumerate(sup):
        owner[perm[c0:c0 + nc]] = s
    keys = np.sort(owner[node_ids])
    first = sup[:, 3]
    idx = np.arange(len(sup))
    lo = np.searchsorted(keys, first, side="left")
    hi = np.searchsorted(keys, idx, side="right")
    return hi - lo


def build_WH_flops(analysis, node_ids):
    sup, rp = analysis["sup"], analysis["rows_ptr"]
    cnt = supernode_ranges(analysis, node_ids)
    n3 = 3.0 * sup[:, 1]
    b3 = 3.0 * np.diff(rp)
    r = 3.0 * cnt
    return float(np.sum(r * n3 * n3 + 2.0 * r * n3 * b3 + n3 * r * (r + 1.0)))


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc summary.

    The summary (profiles/hbm_traffic_precision.md) holds a line
    `traffic_bytes_per_launch <kernel> <bytes> <source hash>`; the value is
    used only while the kernel source hash matches the current source, else
    the traffic is unknown (None).  The caller applies it only to the
    workload the counters were taken on.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_precision.md")
    src = os.path.join(ROOT, "paper_2306_06946_amd", "csrc", "k_contact.hip")
    try:
        lines = open(path).read().splitlines()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    for ln in lines:
        f = ln.strip().strip("`").split()
        if len(f) == 4 and f[0] == "traffic_bytes_per_launch" and f[1] == kernel:
            return float(f[2]) if f[3] == digest else None
    return None


def profiled_issue(kernel):
    """Single-wave issue check of `kernel` from the committed rocprofv3 SQ
    counters (profiles/pgs_issue_precision.md, line `issue_check <kernel>
    <VALU instructions per launch> <busy cycles per launch> <cycles per FP64
    VALU instruction> <source hash>`), or None when the kernel source changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pgs_issue_precision.md")
    src = os.path.join(ROOT, "paper_2306_06946_amd", "csrc", "k_contact.hip")
    try:
        lines = open(path).read().splitlines()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    for ln in lines:
        f = ln.strip().strip("`").split()
        if len(f) == 6 and f[0] == "issue_check" and f[1] == kernel and f[5] == digest:
            valu, busy, cpi = float(f[2]), float(f[3]), float(f[4])
            return {"valu_insts_per_launch": valu, "busy_cycles_per_launch": busy, "cycles_per_valu": cpi,
                    "issue_bound_cycles": valu * cpi, "frac": valu * cpi / busy,
                    "note": "dependent chain of one solving wave at a time: FP64 VALU issue of the launch's "
                            "instructions (all waves) against its busy cycles, an upper bound of the chain's "
                            "share (profiles/pgs_issue_precision.md)"}
    return None


def serving_leg(n_scenes, rate, sweeps, slots, seconds=2.0, group=8, max_wait_ms=0.0):
    """Serving mix through icr_server: closed-loop saturation with 1, 4 and
    `slots` slots (Newton loops of the requests started together batched into
    one launch), the same at `slots` slots without batching, then Poisson
    arrivals at `rate` steps/s over `seconds` on `slots` slots, batched."""
    import torch
    from paper_2306_06946_amd import icr
    from paper_2306_06946_amd.scenes import make_scene
    t0 = time.perf_counter()
    scs = [make_scene("serving", 100 + i) for i in range(n_scenes)]
    scenes = []
    for sc in scs:
        s = icr.scene_from_dict(sc)
        s.step(sc["obstacle"], sc["n_contacts"], sc["n_newton"], sweeps, 0.0, sc["j_inner"], report=False)
        scenes.append(s)
    torch.cuda.synchronize()
    log(f"[bench] serving: {n_scenes} scenes ready in {time.perf_counter() - t0:.1f} s")
    out = {"scenes": n_scenes, "nodes": [len(sc["nodes"]) for sc in scs], "contacts": [sc["n_contacts"] for sc in scs],
           "pgs_sweeps": sweeps, "hbm_budget_bytes": 200 << 30}

    def closed_loop(slots, window, batching=True):
        # every scene keeps one request outstanding; count completions in a
        # fixed time window (fast scenes complete more steps than slow ones)
        srv = icr.Server(hbm_budget=200 << 30, slots=slots, batching=group if batching else 0,
                         max_wait_ms=max_wait_ms)
        ids = [srv.admit(s) for s in scenes]
        lat = []
        ts = time.perf_counter()
        for i, sc in zip(ids, scs):
            srv.submit(i, sc["obstacle"], sc["n_contacts"], sc["n_newton"], sweeps, 0.0, sc["j_inner"])
        done = 0
        while True:
            comp, _ = srv.poll(wait=True)
            el = time.perf_counter() - ts
            for c in comp:
                done += 1
                lat.append(c["latency_ms"])
                if el < window:
                    sc = scs[ids.index(c["scene"])]
                    srv.submit(c["scene"], sc["obstacle"], sc["n_contacts"], sc["n_newton"], sweeps, 0.0,
                               sc["j_inner"])
            if el >= window:
                break
        n_in_window = done
        while True:   # drain what is still in flight (not counted)
            comp, pend = srv.poll(wait=True)
            if pend == 0 and not comp:
                break
        used = srv.used()
        srv.close()
        for s in scenes:
            s.set_stream(torch.cuda.current_stream().cuda_stream)
        lat = np.array(lat)
        return dict(slots=slots, batching=batching, window_s=window, steps=int(n_in_window),
                    steps_per_s=n_in_window / el, p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), admitted_bytes=int(used))

    out["hw_queues"] = os.environ.get("GPU_MAX_HW_QUEUES")
    out["group"] = group
    out["max_wait_ms"] = max_wait_ms
    for k in sorted({1, 4, slots}):
        out[f"closed_loop_{k}_slot" + ("s" if k > 1 else "")] = closed_loop(k, seconds)
    out[f"closed_loop_{slots}_slots_unbatched"] = closed_loop(slots, seconds, batching=False)
    cap = out[f"closed_loop_{slots}_slot" + ("s" if slots > 1 else "")]["steps_per_s"]
    log("[bench] serving closed loop: " + ", ".join(
        f"{v['slots']} slots{'' if v['batching'] else ' unbatched'} {v['steps_per_s']:.0f} steps/s"
        for k, v in out.items() if k.startswith("closed_loop")) + f" (hardware queues {out['hw_queues']})")
    if rate <= 0:
        rate = 0.7 * cap   # an offered load the slots can carry
    # open loop: Poisson arrivals, random scene per arrival
    rng = np.random.default_rng(7)
    n_req = int(rate * seconds)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    which = rng.integers(0, n_scenes, size=n_req)
    srv = icr.Server(hbm_budget=200 << 30, slots=slots, batching=group, max_wait_ms=max_wait_ms)
    ids = [srv.admit(s) for s in scenes]
    lat = []
    k = 0
    ts = time.perf_counter()
    while len(lat) < n_req:
        now = time.perf_counter() - ts
        while k < n_req and arrivals[k] <= now:
            sc = scs[which[k]]
            srv.submit(ids[which[k]], sc["obstacle"], sc["n_contacts"], sc["n_newton"], sweeps, 0.0, sc["j_inner"],
                       tag=k)
            k += 1
        comp, _ = srv.poll(wait=False)
        lat += [c["latency_ms"] for c in comp]   # from submission, made as soon as the arrival time passes
    el = time.perf_counter() - ts
    srv.close()
    for s in scenes:
        s.set_stream(torch.cuda.current_stream().cuda_stream)
    lat = np.array(lat)
    out["poisson"] = dict(rate_steps_per_s=rate, requests=n_req, elapsed_s=el, achieved_steps_per_s=n_req / el,
                          p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)), slots=slots)
    log(f"[bench] serving poisson {rate:.0f}/s: achieved {n_req / el:.0f}/s p50 {out['poisson']['p50_ms']:.2f} ms "
        f"p99 {out['poisson']['p99_ms']:.2f} ms")
    for s in scenes:
        s.close()
    return out


def cpu_baseline(sc, sweeps):
    """The FP64 oracle on the same step: the first time step of the
    configuration's trajectory (the step the GPU's trajectory starts with),
    run whole by the oracle -- free motion, contact selection, W_H (as the
    inverse of the Schur complement onto the contact DOFs), the Newton loop
    with the same sweep count, corrective motion and integration.  Set-up
    (assembly, the banded factor of A for the single-RHS solves) is excluded
    and reported beside it."""
    import oracle.icr_oracle as O
    t0 = time.perf_counter()
    sim = O.Simulation(sc)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    out = sim.step(max_sweeps=sweeps, tol=0.0, wh="schur")
    per_step = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    nc = len(out["nodes_c"])
    return dict(value=1.0 / per_step, unit="time-steps/s", cores=cores, kind="oracle",
                sample=(f"one whole time step (the trajectory's first) of the same configuration: free motion, "
                        f"selection of {nc} contacts, W_H {3 * nc}x{3 * nc} by the Schur complement, "
                        f"{sc['n_newton']} Newton iterations x {sweeps} PGS sweeps, corrective motion; "
                        f"set-up (assembly + banded factor, {setup:.1f} s) excluded; BLAS threads = host cores"),
                seconds_per_step=per_step, setup_s=setup)


def copy_probe(mib):
    """Plain copy kernel of known size: reads and writes mib MiB per launch."""
    import torch
    torch.cuda.set_device(0)
    n = int(mib * 2 ** 20) // 8
    x = torch.arange(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_launch": 8 * n, "launches": 5}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="timed steps: repeats of the --trajectory-step trajectory from the initial state")
    ap.add_argument("--trajectory", type=int, default=0,
                    help="steps per trajectory; 0 = the configuration's own count (20 for precision)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="precision")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--sweeps", type=int, default=30, help="PGS sweeps per Newton iteration (paper: 30)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--standard-steps", type=int, default=20,
                    help="also time this many steps of the standard rebuild scheme (Algorithm 2); 0 = skip")
    ap.add_argument("--per-sweep-steps", type=int, default=0,
                    help="also time this many steps with the directions updated after every PGS sweep "
                         "(n_newton x sweeps iterations of one sweep); 0 = skip")
    ap.add_argument("--mixed-steps", type=int, default=20,
                    help="also time this many steps in mixed precision (FP32 multi-RHS solve with 0 and 1 FP64-"
                         "residual refinement steps, FP32 W_H / W storage) against the FP64 path; 0 = skip")
    ap.add_argument("--per-constraint-steps", type=int, default=0,
                    help="also time this many steps with the directions updated before every local solve; 0 = skip")
    ap.add_argument("--graph", action="store_true",
                    help="replay the captured step graph instead of launching every step eagerly (eager is about "
                         "1%% faster here: the graph replay loses part of the overlap of the W_H products)")
    ap.add_argument("--no-graph", action="store_true", help="eager launches (the default; kept for old commands)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the W_H products of a tree level on the scene's own stream instead of a second one")
    ap.add_argument("--serving", type=int, default=0, metavar="SCENES",
                    help="also run the serving mix: this many independent scenes (node count 500-8000, 10-500 "
                         "contacts) stepped through icr_server; 0 = skip")
    ap.add_argument("--serving-rate", type=float, default=0.0,
                    help="Poisson arrival rate (steps/s, all scenes); 0 = 70%% of the measured capacity")
    ap.add_argument("--serving-seconds", type=float, default=2.0,
                    help="length of each closed-loop window and of the Poisson run")
    ap.add_argument("--serving-group", type=int, default=8,
                    help="requests per slot and round of the serving mix, their Newton loops in one launch "
                         "(0: one whole step per slot)")
    ap.add_argument("--serving-max-wait", type=float, default=0.0,
                    help="ms a short serving group waits for more requests while a slot runs")
    ap.add_argument("--serving-slots", type=int, default=16,
                    help="server slots (streams) of the serving mix; HIP gets as many hardware queues (1..32)")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="MIB",
                    help="only run a plain device-to-device copy of this many MiB (5 launches) and exit: the "
                         "calibration kernel for HBM byte counters")
    args = ap.parse_args()
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; the multi-GPU sharding of build_WH is a "
                                   "design, not an implemented path", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.serving > 0:
        if not 1 <= args.serving_slots <= 32:
            ap.error("--serving-slots must be in 1..32")
        # streams beyond the process's hardware queues share a queue and run
        # one after another; must be set before HIP starts
        os.environ["GPU_MAX_HW_QUEUES"] = str(max(4, args.serving_slots))
    import torch
    from paper_2306_06946_amd import icr
    from paper_2306_06946_amd.scenes import make_scene

    torch.cuda.set_device(0)
    sc = make_scene(args.config, args.seed)
    nc = sc["n_contacts"]
    m = 3 * nc
    log(f"[bench] config={args.config} nodes={len(sc['nodes'])} dofs={3 * len(sc['nodes'])} contacts={nc}")
    stream = torch.cuda.current_stream().cuda_stream
    s = icr.scene_from_dict(sc, stream)
    if args.no_overlap:
        s.set_overlap(False)
    info = s.factor_info()
    log(f"[bench] factor: {info['n_supernodes']} supernodes, nnz(L)={info['nnz_L']/1e6:.1f}M, "
        f"{info['factor_flops']/1e9:.1f} GFLOP in {info['factor_ms']:.1f} ms")
    analysis = icr.analyze(sc["nodes"], sc["tets"])

    def one_step(timing):
        # timing = True: phase stamps and a report (synchronises the stream)
        return s.step(sc["obstacle"], nc, sc["n_newton"], args.sweeps, 0.0, sc["j_inner"], timing=timing,
                      report=timing, graph=args.graph and not args.no_graph)

    q0, v0, t_init = s.get_state()
    q0, v0 = q0.clone(), v0.clone()
    for i in range(args.warmup):
        r = one_step(True)
        log(f"[bench] warmup {i}: {r['ms_total']:.2f} ms")
    traj = max(1, min(args.trajectory or sc["n_steps"], args.steps))
    # timed region: the steps only (no phase stamps, no host synchronisation
    # between steps); each step's device time from events on the stream
    tstream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(tstream)
    for i in range(args.steps):
        if i % traj == 0:
            s.set_state(q0, v0, t_init)   # restart the trajectory (also clears the warm start)
        one_step(False)
        evs[i + 1].record(tstream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lat = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    # phase breakdown: one more trajectory with stamps (outside the timed region)
    s.set_state(q0, v0, t_init)
    reps = [one_step(True) for _ in range(traj)]
    torch.cuda.synchronize()
    res = s.step_results(nc)
    node_ids = res["node_ids"].cpu().numpy()

    steps_per_s = args.steps / elapsed
    ph = {k: float(np.mean([r[k] for r in reps])) for k in
          ("ms_total", "ms_free", "ms_contacts", "ms_build_WH", "ms_newton", "ms_update_W", "ms_pgs", "ms_corr",
           "ms_correct")}
    metric_ms = ph["ms_build_WH"] + ph["ms_newton"]
    sweeps = reps[-1]["sweeps"]
    n_newton = sc["n_newton"]
    pgs_ms_launch = ph["ms_pgs"] / n_newton
    wh_flops = build_WH_flops(analysis, node_ids)
    cand = {
        "pgs": (ph["ms_pgs"], dict(bound="hbm", achieved=args.sweeps * m * m * 8 / (pgs_ms_launch * 1e-3) / 1e9,
                                   peak=HBM_PEAK_GBS, unit="GB/s")),
        "build_WH": (ph["ms_build_WH"], dict(bound="mfma", achieved=wh_flops / (ph["ms_build_WH"] * 1e-3) / 1e12,
                                             peak=FP64_PEAK_TFLOPS, unit="TFLOP/s")),
        "update_W": (ph["ms_update_W"], dict(bound="hbm",
                                             achieved=2 * m * m * 8 / (ph["ms_update_W"] / n_newton * 1e-3) / 1e9,
                                             peak=HBM_PEAK_GBS, unit="GB/s")),
    }
    dom = max(cand, key=lambda k: cand[k][0])
    roof = dict(cand[dom][1])
    roof["kernel"] = {"pgs": "k_pgs_active", "build_WH": "k_rhs_*", "update_W": "k_update_W"}[dom]
    roof["frac"] = roof["achieved"] / roof["peak"]
    # the counters were taken on the precision workload at the default sweep count
    on_profiled = args.config == "precision" and args.sweeps == 30
    roof["traffic"] = profiled_traffic(roof["kernel"]) if on_profiled else None
    if dom == "pgs":
        # SURVEY's unit for PGS is the bytes a dense sweep streams (m^2 * 8 per
        # sweep); the kernel sweeps the active set in LDS and registers and is
        # bound by its sequential contact chain, so the HBM fraction is nominal
        roof["basis"] = "nominal: dense-sweep bytes 30 x m^2 x 8 per launch; the kernel is a latency-bound chain"
        roof["latency"] = profiled_issue("k_pgs_active") if on_profiled else None
    out = {
        "metric": ("time-steps/sec (W_H build + Newton W updates) at "
                   + ("60k" if args.config == "precision" else f"{3 * len(sc['nodes']) / 1000:.1f}k")
                   + " DOF; p50/p99 step latency"),
        "value": steps_per_s,
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "trajectory_steps": traj,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": ("synthetic seeded scene (jittered grid tet mesh, rigid sphere"
                 + (", two stacked bodies with interface pair contacts" if sc.get("pairs") is not None else "")
                 + "); no paper dataset exists"),
        "config": {"workload": f"{args.config}: {sc['grid'][0]}x{sc['grid'][1]}x{sc['grid'][2]} node grid, "
                               f"{3 * len(sc['nodes'])} DOF, {nc} contacts (W_H {m}x{m}), {n_newton} Newton x "
                               f"{args.sweeps} PGS sweeps, FP64",
                   "dofs": 3 * len(sc["nodes"]), "contacts": nc, "newton": n_newton, "pgs_sweeps": args.sweeps,
                   "parallelism": "single GPU"},
        "launch": "graph replay" if (args.graph and not args.no_graph) else "eager",
        "metric_scope_steps_per_s": 1e3 / metric_ms,
        "phases_ms": ph,
        "build_WH_gflop": wh_flops / 1e9,
        "status_counts": [reps[-1]["n_separate"], reps[-1]["n_stick"], reps[-1]["n_slip"]],
        "roofline": roof,
    }
    has_pairs = sc.get("pairs") is not None
    if has_pairs and (args.standard_steps > 0 or args.per_constraint_steps > 0):
        log("[bench] pair contacts run the fast scheme only: standard and per-constraint legs skipped")
        args.standard_steps = args.per_constraint_steps = 0
    if args.standard_steps > 0:
        # same trajectory: a second scene runs the standard scheme (warm-up,
        # then a restart from the initial state) and its steps are compared
        # with the same steps of the fast scheme (both schemes give the same
        # states up to rounding)
        log("[bench] standard rebuild scheme (Algorithm 2) for comparison...")
        ns = min(args.standard_steps, traj)
        s2 = icr.scene_from_dict(sc, stream)
        for _ in range(args.warmup):
            s2.step(sc["obstacle"], nc, n_newton, args.sweeps, 0.0, sc["j_inner"], timing=True, standard=True)
        s2.set_state(q0, v0, t_init)
        std = [s2.step(sc["obstacle"], nc, n_newton, args.sweeps, 0.0, sc["j_inner"], timing=True, standard=True)
               for _ in range(ns)]
        keys = ("ms_total", "ms_build_WH", "ms_newton", "ms_update_W", "ms_pgs", "ms_corr")
        sp = {k: float(np.mean([r[k] for r in std])) for k in keys}
        fp = {k: float(np.mean([r[k] for r in reps[:ns]])) for k in keys}
        out["standard_scheme"] = {
            "steps": ns, "same_steps_as_fast": f"trajectory steps 0..{ns - 1}",
            "ms_per_step": sp["ms_total"], "fast_ms_per_step": fp["ms_total"],
            "ms_per_newton_iteration": sp["ms_newton"] / n_newton,
            "ms_rebuild_W_per_iteration": sp["ms_update_W"] / n_newton,
            "ms_pgs_per_iteration": sp["ms_pgs"] / n_newton, "ms_corr_per_iteration": sp["ms_corr"] / n_newton,
            "fast_ms_per_newton_iteration": fp["ms_newton"] / n_newton,
            "fast_ms_update_W_per_iteration": fp["ms_update_W"] / n_newton,
            "fast_ms_build_WH": fp["ms_build_WH"],
            "newton_iteration_speedup": sp["ms_newton"] / fp["ms_newton"],
            "update_W_speedup": sp["ms_update_W"] / fp["ms_update_W"],
            "metric_scope_speedup": sp["ms_newton"] / (fp["ms_build_WH"] + fp["ms_newton"]),
        }
        s2.close()
    if args.per_sweep_steps > 0:
        # variant of the results section: directions (and W) updated after
        # every PGS sweep, i.e. n_newton x sweeps Newton iterations of one sweep
        nps = min(args.per_sweep_steps, traj)
        nk = n_newton * args.sweeps
        log(f"[bench] directions updated every sweep: {nk} iterations x 1 sweep, {nps} steps...")
        s.set_state(q0, v0, t_init)
        pr = [s.step(sc["obstacle"], nc, nk, 1, 0.0, sc["j_inner"], timing=True) for _ in range(nps)]
        keys = ("ms_total", "ms_build_WH", "ms_newton", "ms_update_W", "ms_pgs", "ms_corr")
        pp = {k: float(np.mean([r[k] for r in pr])) for k in keys}
        fp = {k: float(np.mean([r[k] for r in reps[:nps]])) for k in keys}
        out["per_sweep_directions"] = {
            "steps": nps, "newton_iterations": nk, "sweeps_per_iteration": 1,
            "ms_per_step": pp["ms_total"], "metric_scope_ms": pp["ms_build_WH"] + pp["ms_newton"],
            "ms_update_W": pp["ms_update_W"], "ms_pgs": pp["ms_pgs"], "ms_corr": pp["ms_corr"],
            "fast_ms_per_step": fp["ms_total"], "fast_metric_scope_ms": fp["ms_build_WH"] + fp["ms_newton"],
            "status_counts": [pr[-1]["n_separate"], pr[-1]["n_stick"], pr[-1]["n_slip"]],
        }
    if args.mixed_steps > 0:
        # mixed precision (FP32 solve + FP64-residual refinement, FP32 W_H / W)
        # on the same trajectory, against the FP64 path of the same GPU: time
        # per step and, on the trajectory's first step, errors against FP64
        nms = min(args.mixed_steps, traj)
        s.set_state(q0, v0, t_init)
        one_step(True)
        r64 = s.step_results(nc, with_WH=True)
        res64 = {k: r64[k].cpu().numpy() for k in ("WH", "lam", "p")}
        out["mixed_precision"] = {"steps": nms, "fp64_ms_per_step": ph["ms_total"],
                                  "fp64_ms_build_WH": ph["ms_build_WH"], "fp64_ms_newton": ph["ms_newton"]}
        for refine in (0, 1):
            log(f"[bench] mixed precision, {refine} refinement step(s): {nms} steps...")
            kw = dict(timing=True, graph=False, precision=icr.FP32_IR, refine=refine)
            s.set_state(q0, v0, t_init)
            s.step(sc["obstacle"], nc, n_newton, args.sweeps, 0.0, sc["j_inner"], **kw)
            r32 = s.step_results(nc, with_WH=True)
            err = {k: float(np.linalg.norm(r32[k].cpu().numpy() - res64[k]) / np.linalg.norm(res64[k]))
                   for k in ("WH", "lam")}
            s.set_state(q0, v0, t_init)
            mr = [s.step(sc["obstacle"], nc, n_newton, args.sweeps, 0.0, sc["j_inner"], **kw) for _ in range(nms)]
            keys = ("ms_total", "ms_build_WH", "ms_newton", "ms_update_W", "ms_pgs", "ms_corr")
            mp = {k: float(np.mean([r[k] for r in mr])) for k in keys}
            out["mixed_precision"][f"refine_{refine}"] = {
                "ms_per_step": mp["ms_total"], "steps_per_s": 1e3 / mp["ms_total"], "ms_build_WH": mp["ms_build_WH"],
                "ms_newton": mp["ms_newton"], "ms_update_W": mp["ms_update_W"], "ms_pgs": mp["ms_pgs"],
                "metric_scope_steps_per_s": 1e3 / (mp["ms_build_WH"] + mp["ms_newton"]),
                "rel_err_vs_fp64_first_step": err}
        s.set_state(q0, v0, t_init)
    if args.per_constraint_steps > 0:
        # variant of the results section: directions updated before every
        # local solve (one-workgroup Gauss-Seidel on world-frame forces), same
        # Newton and sweep counts
        npc = min(args.per_constraint_steps, traj)
        log(f"[bench] directions updated before every local solve: {npc} steps...")
        s.set_state(q0, v0, t_init)
        pr = [s.step(sc["obstacle"], nc, n_newton, args.sweeps, 0.0, sc["j_inner"], timing=True,
                     per_constraint=True, graph=False) for _ in range(npc)]
        keys = ("ms_total", "ms_build_WH", "ms_newton", "ms_pgs", "ms_corr")
        pp = {k: float(np.mean([r[k] for r in pr])) for k in keys}
        out["per_constraint_directions"] = {
            "steps": npc, "newton_iterations": n_newton, "sweeps_per_iteration": args.sweeps,
            "ms_per_step": pp["ms_total"], "metric_scope_ms": pp["ms_build_WH"] + pp["ms_newton"],
            "ms_pgs": pp["ms_pgs"], "ms_corr": pp["ms_corr"],
            "status_counts": [pr[-1]["n_separate"], pr[-1]["n_stick"], pr[-1]["n_slip"]],
        }
    if args.serving > 0:
        out["serving"] = serving_leg(args.serving, args.serving_rate, args.sweeps, args.serving_slots,
                                     seconds=args.serving_seconds, group=args.serving_group,
                                     max_wait_ms=args.serving_max_wait)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (the oracle's first step)...")
        out["cpu_baseline"] = cpu_baseline(sc, args.sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
