"""Benchmark of the tiled-sCOLA hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]

A benchmark "step" is one batch: the whole KDK evolution (initial deposit and Poisson solve,
then n_steps fused particle steps each followed by the Poisson solve of the next force) of
every sCOLA box of the workload, from inputs already resident in HBM (the set-up
Psi1/Psi2/Phi_BC^0 computed once before timing).  value = box particles x KDK steps per
second over the K timed batches.  One JSON line is printed.

Workloads (particles per side, box side, tiling):
  c2  500 Mpc/h, 128^3 particles, 4^3 tiles of 32^3 + 16 buffer (64^3 boxes), 20 steps, FP32
  c1  200 Mpc/h, 64^3 particles, 2^3 tiles of 32^3 + 8 buffer (48^3 boxes), 10 steps, FP64
      per-tile (the plain path)
Roofline: the dominant kernel is the fused particle step; its algorithmic traffic is 72 B
per particle (x_res and p_res read and written, Psi1 and Psi2 read, all FP32), timed
with HIP events around single launches on the stream it runs on.  roofline.whole_step adds
the Poisson solve (16 B per interior node) and takes the measured time of one KDK step of
the evolution, i.e. every kernel of the step.
CPU baseline: the FP64 oracle on a sample of c2 (16 of its 64 boxes, all steps) and on the
whole c1 workload, boxes in parallel processes.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PARTICLE_BYTES_FP32 = 72     # per particle and step: 4 x 12 B of x_res/p_res + 2 x 12 B of Psi
PARTICLE_BYTES_FP64 = 144


def build_sim(S, wl, precision=None, schedule=None):
    if wl.mixed:
        tiles = [((x, y, z), c, b) for x, y, z, c, b in wl.mixed]
    else:
        tiles = S.uniform_tiling(wl.Np, wl.tiles_per_side, wl.buffer)
    prec = precision or wl.precision
    sch = schedule or ("per_tile" if prec == "fp64" else "batched")
    return S.Simulation(wl.L, wl.Np, tiles, wl.n_steps, a_i=wl.a_i, a_f=wl.a_f,
                        precision=prec, schedule=sch)


def measured_traffic():
    """HBM bytes per launch of the fused particle step measured with rocprofv3 FETCH_SIZE and
    WRITE_SIZE (calibrated against a 1 GiB copy) on this workload, as recorded in
    profiles/k_particles_c2_hbm_traffic.txt -- or None when the kernel's sources have changed
    since the counters were taken (the file records their SHA-256)."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "k_particles_c2_hbm_traffic.txt")
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                      if line.startswith(("kernel_source_sha256:", "sources:",
                                          "traffic_bytes_per_launch:")))
        h = hashlib.sha256()
        for src in fields["sources"].split():
            h.update(open(os.path.join(here, src), "rb").read())
        if h.hexdigest() != fields["kernel_source_sha256"].strip():
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def whole_step(P, G, ms_per_kdk):
    """All kernels of one KDK step against the HBM roofline: algorithmic bytes 72 B per box
    particle (x_res, p_res read and written, Psi1, Psi2 read, FP32) + 16 B per interior mesh
    node (delta written and read, Phi written and read, FP32) over the measured time of one
    KDK step of the evolution."""
    b = PARTICLE_BYTES_FP32 * P + 16 * G
    gbs = b / (ms_per_kdk * 1e-3) / 1e9
    return {"bytes_per_kdk_step": b, "ms_per_kdk_step": ms_per_kdk, "achieved": gbs,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}


def time_evolve(torch, sim, steps, warmup):
    # the second call records the evolution as a hipGraph; timed calls replay it
    for _ in range(max(warmup, 2)):
        sim.evolve()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        sim.evolve()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / steps, wall


def time_kernel(torch, fn, reps, warmup=None):
    """Average duration of one launch, HIP events around each call on the current stream,
    after `warmup` untimed calls (default: as many as timed ones) so the clocks and caches
    have settled, as for the warm-up steps of the evolution."""
    for _ in range(reps if warmup is None else warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in evs)
    return sum(ts) / len(ts), ts[len(ts) // 2]


def time_batch(torch, fn, reps):
    """Average duration of one call within a run of `reps` back-to-back calls: HIP events
    around the whole run on the current stream (after as many untimed calls), so that the
    events' own overhead is spread over the run; the calls' kernels follow each other with
    only the launch gaps between them."""
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and its logical CPU count."""
    name = platform.processor() or "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, os.cpu_count() or 1


def _oracle_box(args):
    """One box of the oracle run (worker process): evolution of tile t, timed alone."""
    from threadpoolctl import threadpool_limits

    from oracle.scola import evolve_box
    s1, s2, bc0, steps = args
    with threadpool_limits(1):
        t0 = time.perf_counter()
        evolve_box(s1, s2, bc0, steps)
        return time.perf_counter() - t0


def oracle_rate(name, max_boxes=None, max_workers=16):
    """The FP64 oracle on the host's cores: workload `name` (its first max_boxes boxes, or
    all), the full-box set-up once, then the boxes evolved in parallel worker processes (one
    box per process, as the boxes are independent), single-threaded BLAS in each.
    value = box particles x steps / wall time of the parallel evolution."""
    import multiprocessing as mp

    import numpy as np

    import synthetic
    from oracle.cosmology import Cosmology, cola_schedule
    from oracle.run import box_inputs, setup_full_box
    from oracle.tiling import uniform_tiling

    wl = synthetic.WORKLOADS[name]
    c = Cosmology()
    t0 = time.perf_counter()
    phi1, phi2, psi1, psi2 = setup_full_box(synthetic.white_noise(wl.Np, 42), wl.L, c, wl.a_i)
    tiles = uniform_tiling(wl.Np, wl.tiles_per_side, wl.buffer)
    if max_boxes:
        tiles = tiles[:max_boxes]
    steps, _ = cola_schedule(c, wl.a_i, wl.a_f, wl.n_steps)
    jobs = [(*box_inputs(psi1, psi2, phi1, t), steps) for t in tiles]
    setup_s = time.perf_counter() - t0
    model, ncpu = cpu_model()
    workers = max(1, min(len(jobs), ncpu, max_workers))
    # fork: called before this process touches the GPU (see main)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        per_box = pool.map(_oracle_box, jobs)
    wall = time.perf_counter() - t0
    P = sum(t.M ** 3 for t in tiles)
    n_all = wl.tiles_per_side ** 3
    part = "in full" if len(tiles) == n_all else f"{len(tiles)} of its {n_all} boxes"
    return dict(value=P * wl.n_steps / wall, unit="particle-steps/s", cores=workers,
                kind="oracle",
                sample=f"{name} {part}: boxes of {tiles[0].M}^3, {wl.n_steps} KDK steps, FP64 "
                       f"NumPy, one box per worker process ({workers} processes, 1 BLAS "
                       f"thread each) on {model} ({ncpu} logical CPUs visible); evolution wall "
                       f"{wall:.1f} s (pool start included), CPU {np.sum(per_box):.1f} s in "
                       f"all, full-box set-up {setup_s:.1f} s",
                cpu_model=model, host_logical_cpus=ncpu, evolution_wall_s=wall,
                cpu_s=float(np.sum(per_box)), setup_s=setup_s)


def cpu_baseline():
    """The oracle on the benchmark's own workload c2 (a bounded sample: as many boxes as
    worker processes, up to 16, with all 20 steps, scaled to particle-steps/s), and on the
    plain FP64 workload c1 in full."""
    out = oracle_rate("c2", max_boxes=16)
    out["c1_full"] = oracle_rate("c1")
    return out


def adjoint_timing(torch, S, synthetic, name="c4", reps=3):
    """Forward with checkpoints (every 5 steps) and the reverse pass (segment recomputation
    + adjoint steps + FP64 set-up adjoint) of a density loss, HIP-event timed on the current
    stream: c4 (the c2 boxes, 20 FP32 steps) or c5 (512 boxes of 96^3, 30 FP32 steps)."""
    wl = synthetic.WORKLOADS[name]
    sim = S.Simulation(wl.L, wl.Np, S.uniform_tiling(wl.Np, wl.tiles_per_side, wl.buffer),
                       wl.n_steps, precision="fp32", checkpoint_every=5)
    w = torch.from_numpy(synthetic.white_noise(wl.Np, 42)).cuda()
    t = torch.from_numpy(synthetic.loss_target(wl.Np, 43)).cuda().float()
    sim.setup(w)
    sched = sim.tune(reps=3)
    dens = torch.empty((wl.Np,) * 3, dtype=torch.float32, device="cuda")
    ev = lambda: torch.cuda.Event(enable_timing=True)
    fw, bw = [], []
    for r in range(reps + 1):
        a, b, c = ev(), ev(), ev()
        a.record()
        sim.evolve()
        sim.output(density=dens)
        b.record()
        sim.backward(2.0 * (dens - t))
        c.record()
        torch.cuda.synchronize()
        if r:
            fw.append(a.elapsed_time(b))
            bw.append(b.elapsed_time(c))
    f, g = sum(fw) / reps, sum(bw) / reps
    ws_gb = sim.layout.total / 1e9
    groups = sim.groups
    del sim
    torch.cuda.empty_cache()
    return {"workload": f"{name}: {wl.Np}^3 particles, {wl.tiles_per_side ** 3} boxes of "
                        f"{wl.Np // wl.tiles_per_side + 2 * wl.buffer}^3, {wl.n_steps} FP32 "
                        f"steps, density loss, checkpoint every 5",
            "forward_ms": f, "backward_ms": g, "backward_over_forward": g / f,
            "workspace_GB": ws_gb, "launch_schedule": {str(k): v for k, v in sched.items()},
            "concurrent_box_groups": groups,
            "note": "backward = segment recomputation (one forward's worth of steps) + adjoint "
                    "steps + FP64 set-up adjoint"}


def workload_rate(torch, S, synthetic, name, steps=3, warmup=2):
    """Particle-steps/s of scola_evolve on one more workload (autotuned, graph replayed)."""
    wl = synthetic.WORKLOADS[name]
    sim = build_sim(S, wl)
    w = torch.from_numpy(synthetic.white_noise(wl.Np, 42)).cuda()
    sim.setup(w)
    sched = sim.tune(reps=3)
    ms, _ = time_evolve(torch, sim, steps, warmup)
    info = sim.info()
    nodes = sum((M - 1) ** 3 for _, M, _, _ in sim.box_slices())
    out = {"workload": f"{name}: L={wl.L:g} Mpc/h, {wl.Np}^3 particles, {info['n_tiles']} "
                       f"boxes, {wl.n_steps} steps, {sim.precision} batched",
           "value": info["n_particles"] * wl.n_steps / (ms * 1e-3), "unit": "particle-steps/s",
           "ms_per_evolve": ms, "box_particles": info["n_particles"],
           "useful_particle_steps_per_s": wl.Np ** 3 * wl.n_steps / (ms * 1e-3),
           "launch_schedule": {str(k): v for k, v in sched.items()},
           "concurrent_box_groups": sim.groups,
           "whole_step_roofline": whole_step(info["n_particles"], nodes, ms / wl.n_steps)}
    del sim
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the mixed-size (c3) and large (c5) workload lines")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the persistent-step comparison (cooperative launches)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the forward + reverse timing of the adjoint workload")
    ap.add_argument("--kernels-only", action="store_true",
                    help="set-up, then only the single-launch kernel timings and a "
                         "1 GiB device copy that calibrates the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the boxes are independent and the library has "
              "no multi-GPU path (see the design notes for how it would shard).",
              file=sys.stderr)
        sys.exit(2)

    # the CPU baseline runs first, before this process initialises the GPU, so that its
    # worker processes are forked from a process with no device state
    cpu = None
    if not args.no_cpu_baseline and not args.adjoint_only and not args.kernels_only \
            and args.workload == "c2":
        cpu = cpu_baseline()

    import torch

    import paper_2003_04925_amd as S
    import synthetic
    torch.cuda.set_device(0)
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_timing(torch, S, synthetic, "c4", reps=args.steps)}),
              flush=True)
        return
    wl = synthetic.WORKLOADS[args.workload]
    sim = build_sim(S, wl)
    info = sim.info()
    P = info["n_particles"]
    w = torch.from_numpy(synthetic.white_noise(wl.Np, 42)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.setup(w)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    if args.kernels_only:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        tab = sim.step_table()
        row = tab[wl.n_steps // 2]
        sim.evolve()
        for _ in range(args.steps):
            sim.op_poisson(row[3])
            sim.op_step(row[1], row[2], row[3], row[4], row[3], row[4], True)
        torch.cuda.synchronize()
        print(json.dumps({"kernels_only": True, "workload": wl.name}), flush=True)
        return
    block_schedule = sim.tune(reps=5)      # autotuned launch schedule, untimed
    ms, wall = time_evolve(torch, sim, args.steps, args.warmup)
    value = P * wl.n_steps / (ms * 1e-3)

    # end to end: set-up + evolution + outputs (positions and density)
    pos = torch.empty((3, wl.Np, wl.Np, wl.Np), dtype=sim.real, device="cuda")
    dens = torch.empty((wl.Np,) * 3, dtype=sim.real, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.setup(w)
    sim.evolve()
    sim.output(pos=pos, density=dens)
    torch.cuda.synchronize()
    e2e_s = time.perf_counter() - t0

    # dominant kernel: the fused particle step, single launches timed with events
    tab = sim.step_table()
    k = wl.n_steps // 2
    row = tab[k]
    sim.setup(w)
    sim.op_deposit(row[3], row[4])
    sim.op_poisson(row[3])
    step_fn = lambda: sim.op_step(row[1], 0.0, row[3], row[4], row[3], row[4], True)
    step_avg, step_med = time_kernel(torch, step_fn, 20)
    step_run = time_batch(torch, step_fn, 20)
    pois_avg, _ = time_kernel(torch, lambda: sim.op_poisson(row[3]), 20)
    algo_bytes = (PARTICLE_BYTES_FP32 if sim.precision == "fp32" else PARTICLE_BYTES_FP64) * P
    G = sum((M - 1) ** 3 for _, M, _, _ in sim.box_slices())
    traffic = measured_traffic() if wl.name == "c2" else None
    # the dominant kernel's launch duration: 20 back-to-back scola_op_step calls (each the
    # fused step and the small kernel that folds its dropped mass) between two events
    achieved = algo_bytes / (step_run * 1e-3) / 1e9

    result = {
        "metric": "particle-steps/s",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "step": f"one benchmark step = one whole evolution of every box ({wl.n_steps} KDK "
                f"steps: deposits, Poisson solves, fused particle steps)",
        "ms_per_kdk_step": ms / wl.n_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if sim.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: L={wl.L:g} Mpc/h, {wl.Np}^3 particles, "
                               f"{info['n_tiles']} boxes, {wl.n_steps} KDK steps, "
                               f"{sim.precision} {('per-tile' if sim.precision == 'fp64' else 'batched')}",
                   "box_particles": P, "n_tiles": info["n_tiles"],
                   "oversimulation_r": info["r"], "n_steps": wl.n_steps,
                   "launch_schedule": {str(k): v for k, v in block_schedule.items()},
                   "concurrent_box_groups": sim.groups},
        "useful_particle_steps_per_s": wl.Np ** 3 * wl.n_steps / (ms * 1e-3),
        "end_to_end_s": e2e_s,
        "setup_s_first_call": setup_s,
        "kernels_ms": {"particle_step": step_avg, "particle_step_median": step_med,
                       "particle_step_back_to_back": step_run, "poisson_3pass": pois_avg},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic if sim.precision == "fp32" else None,
                     "kernel": "k_particles<float,1> (fused interp+kick+drift+deposit)",
                     "algorithmic_bytes_per_launch": algo_bytes,
                     "whole_step": whole_step(P, G, ms / wl.n_steps)
                     if sim.precision == "fp32" else None},
    }
    # the same evolution with one persistent cooperative launch per KDK step (the batching
    # pattern of a single fused launch per step), for comparison with the default schedule
    try:
        if args.no_persistent:
            raise RuntimeError("skipped (--no-persistent)")
        sim.set_persistent(True)
        pms, _ = time_evolve(torch, sim, max(3, args.steps // 2), args.warmup)
        st = sim.persistent()
        sim.set_persistent(False)
        result["persistent_step"] = {
            "ms_per_evolve": pms, "value": P * wl.n_steps / (pms * 1e-3),
            "unit": "particle-steps/s", "vs_default": ms / pms, "grid": st["grid"],
            "barrier_failures": st["barrier_failures"],
            "note": "one cooperative launch per KDK step and class (particle step + the three "
                    "Poisson passes, grid-wide barriers), eager; the default is the "
                    "graph-replayed four-launch step"}
    except Exception as exc:          # noqa: BLE001 - reported in the JSON line
        result["persistent_step"] = {"error": f"{type(exc).__name__}: {exc}"}
    if not args.no_fp64 and args.workload == "c2":
        wl1 = synthetic.WORKLOADS["c1"]
        sim64 = build_sim(S, wl1)
        w1 = torch.from_numpy(synthetic.white_noise(wl1.Np, 42)).cuda()
        sim64.setup(w1)
        ms64, _ = time_evolve(torch, sim64, 3, 2)
        result["fp64_per_tile"] = {"workload": "c1: 64^3 particles, 8 boxes of 48^3, 10 "
                                               "steps, FP64 per-tile schedule",
                                   "value": sim64.info()["n_particles"] * wl1.n_steps /
                                   (ms64 * 1e-3), "unit": "particle-steps/s"}
        sim32 = build_sim(S, wl1, precision="fp32", schedule="batched")
        sim32.setup(w1)
        ms32, _ = time_evolve(torch, sim32, 3, 2)
        result["fp32_batched_same_workload"] = {
            "workload": "c1 in FP32 batched", "value": sim32.info()["n_particles"] *
            wl1.n_steps / (ms32 * 1e-3), "speedup_vs_fp64_per_tile": ms64 / ms32}
    if not args.no_adjoint and args.workload == "c2":
        result["adjoint"] = adjoint_timing(torch, S, synthetic, "c4")
    if not args.no_extra and args.workload == "c2":
        # the other workloads: each guarded so that a failure is reported, not fatal
        for key, fn in (("c3_mixed", lambda: workload_rate(torch, S, synthetic, "c3")),
                        ("c5_large", lambda: workload_rate(torch, S, synthetic, "c5", 2, 2)),
                        ("c5_adjoint", lambda: adjoint_timing(torch, S, synthetic, "c5", 1))):
            if key == "c5_adjoint" and args.no_adjoint:
                continue
            try:
                result[key] = fn()
            except Exception as exc:          # noqa: BLE001 - reported in the JSON line
                result[key] = {"error": f"{type(exc).__name__}: {exc}"}
                torch.cuda.empty_cache()
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
