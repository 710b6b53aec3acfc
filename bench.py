#!/usr/bin/env python3
"""Throughput of the full LB time step (collide-stream + particle phase) on one
MI355X, in million lattice-site updates per second (MLUPS), with the
collide-stream kernel's fraction of the HBM roofline and the FP64 CPU oracle
timed on the host beside it.

Headline workload: the batched ensemble of 256 independent periodic boxes
(edges 32-64, 29.5 M sites, one spheroid each), D3Q19 TRT (Lambda = 3/16,
tau+ = 1), FP16 storage of the scaled deviations with FP32 collision,
counter-force on: its 2.24 GB of population traffic per step is far beyond
the 256 MB last-level cache, so the roofline figure is an HBM figure.  Legs
beside it: the 256^3 suspension of 512 squirmers in FP16 and FP32 (HBM-sized),
its 6,400-squirmer variant (5 % volume fraction), and the 128^3 inclined
spheroid in FP32, FP16 and D3Q27, whose in-place population buffer fits the
last-level cache (labelled cache_resident).  Inputs are resident in device
memory before the timed region starts.

Prints one JSON line.  Only one GPU is used: --gpus above 1 is refused.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D3Q19 MLUPS + % HBM roofline; steps to steady state, plain vs surrogate"
HBM_PEAK_GBS = 8000.0
BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16": "f32", "bf16": "f32"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "collide_stream_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2403_05443_amd", "csrc", "k_stream.hip")


def build_lattice(W, device="cuda:0"):
    from paper_2403_05443_amd.runner import build_lattice as build
    return build(W, device)


def traffic_record(src_sha, workload, storage, variant):
    """HBM bytes per collide-stream launch from the committed counter
    summary, only if it was taken on this kernel source, workload and
    variant."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    key = f"{workload}/{storage}/v{variant}"
    ent = rec.get("entries", {}).get(key)
    if not ent or rec.get("source_sha256") != src_sha:
        return None
    return ent.get("traffic_bytes_per_launch")


MALL_BYTES = 256 * 2 ** 20   # the last-level (Infinity) cache of the MI355X


def workload_by_name(name, storage):
    """The synthetic workloads bench.py measures, by name."""
    from paper_2403_05443_amd import workloads
    table = {
        "c4_ensemble_256": lambda: workloads.c4(storage),
        "c2_inclined_128": lambda: workloads.c2(storage, 128),
        "c2_inclined_128_d3q27": lambda: workloads.c2(storage, 128, lattice=27),
        "c5_squirmers_256_512": lambda: workloads.c5(storage),
        "c5_squirmers_256_6400": lambda: workloads.c5(storage, n=6400),
        "empty_256": lambda: workloads.empty(storage),
    }
    if name not in table:
        raise SystemExit(f"unknown workload {name}; one of {sorted(table)}")
    return table[name]()


# legs reported beside the headline: workload, storage, timed steps, warm-up steps
LEGS = {
    "suspension_fp16": ("c5_squirmers_256_512", "fp16", 100, 10),
    "suspension_fp32": ("c5_squirmers_256_512", "fp32", 100, 10),
    "suspension_6400_fp16": ("c5_squirmers_256_6400", "fp16", 50, 10),
    "inclined_128_fp32": ("c2_inclined_128", "fp32", 1000, 50),
    "inclined_128_fp16": ("c2_inclined_128", "fp16", 1000, 50),
    "inclined_128_d3q27_fp32": ("c2_inclined_128_d3q27", "fp32", 500, 50),
    "empty_256_fp16": ("empty_256", "fp16", 200, 20),
    "empty_256_fp32": ("empty_256", "fp32", 200, 20),
}


def _omp():
    """libgomp of this process (the oracle is built with OpenMP), or None."""
    import ctypes
    try:
        return ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None


def cpu_baseline(W, seconds):
    """The oracle as it stands on a bounded sample of workload W, on every
    host core OpenMP gives it: box after box (each with its particles), a few
    steps each, until `seconds` of stepping are spent; MLUPS over the steps
    taken."""
    import oracle
    omp = _omp()
    cores = omp.omp_get_max_threads() if omp else int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    steps_per_box = 10 if len(W.boxes) > 1 else 0
    done, spent, nb = 0, 0.0, 0
    for bi, b in enumerate(W.boxes):
        o = oracle.OracleSim(b.shape, W.collision, W.tau, magic=W.magic, walls=b.walls, wall_lo=b.wall_lo,
                             wall_hi=b.wall_hi, init=b.init, counterforce=W.counterforce)
        for p in W.particles:
            if p.box == bi:
                pid = o.add_ellipsoid(p.centre, p.axes, p.quat)
                o.set_external(pid, p.force, p.torque)
        n3 = b.shape[0] * b.shape[1] * b.shape[2]
        n = steps_per_box
        if n == 0:  # a single box: size the run from one timed step
            t0 = time.perf_counter()
            o.step(1)
            n = max(1, int(seconds / max(time.perf_counter() - t0, 1e-6)))
        t0 = time.perf_counter()
        o.step(n)
        spent += time.perf_counter() - t0
        done += n3 * n
        nb += 1
        del o
        if spent >= seconds:
            break
    sample = (f"{W.name}: the first {nb} of its {len(W.boxes)} boxes, {steps_per_box} oracle steps each"
              if len(W.boxes) > 1 else f"{W.name}: {done // (W.boxes[0].shape[0] ** 3)} oracle steps")
    return {"value": round(done / spent / 1e6, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{sample} ({spent:.1f} s of stepping)"}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_reference():
    """The oracle on the host, one thread and all threads, on 64^3 and 128^3
    periodic boxes holding a static sphere of radius 4 (BGK tau = 1), with
    the CPU model: the single-thread and all-core figures beside the GPU's."""
    import oracle
    omp = _omp()
    allc = omp.omp_get_max_threads() if omp else 1
    out = {"cpu_model": _cpu_model(), "logical_cpus": os.cpu_count(), "threads_all": allc, "kind": "oracle",
           "workload": "periodic box, static sphere R = 4, BGK tau = 1, FP64, D3Q19"}
    plan = {1: {64: 20, 128: 5}, allc: {64: 100, 128: 40}}
    for threads, sizes in plan.items():
        if omp:
            omp.omp_set_num_threads(threads)
        key = "single_thread" if threads == 1 else "all_threads"
        out[key] = {}
        for L, n in sizes.items():
            o = oracle.OracleSim((L, L, L), "bgk", 1.0)
            o.add_ellipsoid((L / 2 - 0.3, L / 2 - 0.2, L / 2 - 0.1), (4.0, 4.0, 4.0), (1, 0, 0, 0))
            o.step(1)
            t0 = time.perf_counter()
            o.step(n)
            dt = time.perf_counter() - t0
            out[key][f"{L}^3"] = {"mlups": round(L ** 3 * n / dt / 1e6, 3), "steps": n}
            del o
    if omp:
        omp.omp_set_num_threads(allc)
    return out


def _pmc_rows(d):
    """(kernel name, counter value) of every dispatch in a rocprofv3 --pmc csv tree."""
    import csv
    import glob
    out = []
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(path)):
            out.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return out


def summarize_pmc(fetch_dir, write_dir, workload, storage, probe_bytes, variant):
    """HBM bytes per collide-stream launch from FETCH_SIZE and WRITE_SIZE (KiB
    per dispatch), each scaled by what the same counter reads for the copy
    probe of known size."""
    W = workload_by_name(workload, storage)
    res = {}
    for name, d in (("fetch", fetch_dir), ("write", write_dir)):
        rows = _pmc_rows(d)
        probe = [v for k, v in rows if "k_copy_probe" in k]
        names = [k for k, _ in rows if "collide_stream" in k]
        if not probe or not names:
            raise SystemExit(f"no copy-probe / collide-stream dispatches under {d}")
        # the counter runs force one variant, so every collide-stream dispatch
        # is of it (an in-place variant alternates its even and odd kernel)
        kname = " + ".join(sorted(set(names)))
        k1 = [v for k, v in rows if "collide_stream" in k]
        probe_kib = sorted(probe)[len(probe) // 2]
        scale = probe_bytes / (probe_kib * 1024.0)
        res[name] = {"kernel": kname, "launches": len(k1),
                     "counter_kib_per_launch": sum(k1) / len(k1), "probe_kib": probe_kib, "scale": scale,
                     "bytes_per_launch": sum(k1) / len(k1) * 1024.0 * scale}
    src_sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    try:
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("source_sha256") != src_sha:
            rec = {}
    except (OSError, ValueError):
        rec = {}
    rec["source_sha256"] = src_sha
    rec["kernel"] = "k_collide_stream / k_collide_stream_rows"
    rec.setdefault("entries", {})[f"{W.name}/{storage}/v{variant}"] = {
        "fetch": res["fetch"], "write": res["write"],
        "algorithmic_bytes_per_launch": 2 * W.lattice * BYTES[storage] * W.sites,
        "traffic_bytes_per_launch": round(res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]),
    }
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    json.dump(rec, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(rec["entries"][f"{W.name}/{storage}/v{variant}"]))


def measure(W, steps, warmup, graph_steps, variant=None, psteps=200):
    """Times `steps` steps of workload W after `warmup` steps (collide-stream
    variant from the tuner unless given); returns the lattice and a dict of
    the measured figures."""
    import torch
    if variant is not None:
        os.environ["LBELL_K1_VARIANT"] = str(variant)
    try:
        lat = build_lattice(W)
    finally:
        os.environ.pop("LBELL_K1_VARIANT", None)
    if variant is None:
        variant = lat.autotune(30)[0]  # 30 timed steps per candidate: a 2-3 % margin is resolved
    lat.set_graph(graph_steps)
    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    lat.step(steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    lat.sync()
    # collide-stream launch duration inside real steps: HIP events on the
    # library's stream around every launch (each launch reads the buffer the
    # step before wrote, as in the timed run)
    n = min(steps, psteps)
    ms_c, ms_p = lat.profile_step(n)
    k1 = ms_c / n
    alg = 2 * W.lattice * BYTES[W.storage] * W.sites  # Q reads + Q writes per site
    # population memory a step touches: one buffer in place (variants 11-14), two otherwise
    ws = W.lattice * BYTES[W.storage] * W.sites * (1 if 11 <= variant <= 14 else 2)
    return lat, {
        "mlups": W.sites * steps / (ms / 1e3) / 1e6, "ms_per_step": ms / steps, "wall_s": wall,
        "variant": variant, "k1_ms": k1, "alg_bytes": alg, "achieved_gbs": alg / (k1 / 1e3) / 1e9,
        "phase_ms": {"collide_stream": ms_c / n, "particle": ms_p / n}, "working_set": ws,
    }


def roofline_mlups(W):
    """Site updates per second (millions) at 8 TB/s with 2 Q s bytes per site."""
    return HBM_PEAK_GBS * 1e9 / (2 * W.lattice * BYTES[W.storage]) / 1e6


def leg_record(W, m, src_sha, steps):
    """One measured workload beside the headline."""
    return {"workload": W.name, "boxes": len(W.boxes), "sites": W.sites, "particles": len(W.particles),
            "lattice": f"D3Q{W.lattice}", "storage": W.storage, "steps": steps,
            "mlups": round(m["mlups"], 1), "ms_per_step": round(m["ms_per_step"], 5),
            "frac_of_roofline_mlups": round(m["mlups"] / roofline_mlups(W), 4),
            "k1_variant": m["variant"], "k1_avg_launch_ms": round(m["k1_ms"], 5),
            "k1_bytes_per_launch": m["alg_bytes"], "k1_achieved_gbs": round(m["achieved_gbs"], 1),
            "k1_frac": round(m["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "k1_traffic": traffic_record(src_sha, W.name, W.storage, m["variant"]),
            "working_set_bytes": m["working_set"], "cache_resident": m["working_set"] <= MALL_BYTES,
            "phase_ms_per_step": {k: round(v, 5) for k, v in m["phase_ms"].items()}}


def steps_to_steady(runs, eval_boxes, monitor_tol=0.1, wrong_tol=0.02):
    """The second half of the metric: train the warm-start network on `runs`
    256-box FP16 ensembles (alternately with and without torques; symmetry
    and linearity augmentation, 80/20 split), then count the steps a held-out
    force-driven FP16 ensemble needs to come within 0.5% of its steady
    velocity from a plain start, a surrogate warm start watched by the device
    monitor at monitor_tol, and the closed-form control.  A second surrogate
    leg starts the same ensemble from the network with its parameters
    doubled, watched at wrong_tol: its fallback rate and the steps to steady
    of the boxes that fell back, counted from the warm start (the steps spent
    before the fallback included)."""
    from paper_2403_05443_amd import lbell, runner, workloads
    t0 = time.perf_counter()
    sur, info = runner.train_warm_network(seeds=runs, boxes=256, epochs=1000, seed0=10)
    t_train = time.perf_counter() - t0
    We = workloads.c4("fp16", eval_boxes, seed_index=100, torque=False)
    res = runner.compare_starts(We, sur, monitor_tol=monitor_tol)
    wrong = lbell.Surrogate(max_samples=4096, params=2.0 * sur.params())
    bad = runner.compare_starts(We, wrong, monitor_tol=wrong_tol)
    t_eval = time.perf_counter() - t0 - t_train
    # the whole warm start (features, network, start field) of the headline
    # ensemble, best of three
    lat = runner.build_lattice(workloads.c4("fp16", 256))
    t_head = []
    for _ in range(3):
        lat.sync()
        t1 = time.perf_counter()
        lat.warm_start(sur)
        lat.sync()
        t_head.append(1e3 * (time.perf_counter() - t1))
    del lat
    m = res["median_steps"]
    rates = lambda r: {k: round(r[k + "_rate"], 4) for k in ("accepted", "fallback", "steady_miss")}  # noqa: E731
    return {"eval_workload": We.name, "storage": "fp16", "boxes": res["boxes"], "steady_boxes": res["steady_boxes"],
            "tol": res["tol"], "sample_every": res["every"],
            "median_steps_plain": m["plain"], "median_steps_surrogate": m["surrogate"],
            "median_steps_control": m["control"],
            "median_steps_exact_velocity": m["exact_velocity"],
            "surrogate_over_plain": round(res["surrogate_over_plain"], 4),
            "control_over_plain": round(res["control_over_plain"], 4),
            "median_prediction_error": round(res["median_prediction_error"], 5),
            "start_ms": {k: round(v, 2) for k, v in res["start_ms"].items()},
            "warm_start_ms_c4_ensemble_256": round(min(t_head), 2),
            "monitor": {"tol": monitor_tol, **rates(res), "queued_for_training": len(res["queued"])},
            "wrong_network": {"params": "trained x 2", "monitor_tol": wrong_tol, **rates(bad),
                              "median_prediction_error": round(bad["median_prediction_error"], 5),
                              "median_steps_surrogate": bad["median_steps"]["surrogate"],
                              "median_steps_fallback_boxes": bad["median_steps_fallback_boxes"],
                              "median_steps_plain_same_boxes": bad["median_steps_plain_fallback_boxes"],
                              "median_decision_step_fallback_boxes": bad["median_decision_step_fallback_boxes"],
                              "queued_for_training": len(bad["queued"])},
            "training": {"ensembles": runs, "lb_steps_per_ensemble": info["lb_steps_per_ensemble"],
                         "samples": info["samples"], "loss_val": info["loss_val"],
                         "val_target_variance": info["val_target_variance"]},
            "seconds": {"train": round(t_train, 2), "eval": round(t_eval, 2)}}


def _progress(msg):
    """One line on stderr per finished part of the run."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c4_ensemble_256",
                    help="headline workload (c4_ensemble_256, c5_squirmers_256_512, c5_squirmers_256_6400, "
                         "c2_inclined_128, c2_inclined_128_d3q27, empty_256)")
    ap.add_argument("--storage", default="fp16", choices=sorted(BYTES))
    ap.add_argument("--graph", type=int, default=50, help="steps per HIP graph replay (0: plain launches)")
    ap.add_argument("--variant", type=int, default=None,
                    help="collide-stream variant of the headline instead of the tuner's choice (see lb_autotune)")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated legs measured beside the headline ('none' for none): " + ", ".join(LEGS))
    ap.add_argument("--sweep-only", action="store_true",
                    help="run the domain-size (32^3-512^3) and resolution studies of the settling spheroid "
                         "instead of the benchmark and print their results as one JSON line")
    ap.add_argument("--studies", default="domain,resolution,sphere_array,jeffery_domain",
                    help="with --sweep-only: comma-separated studies to run (domain, resolution, sphere_array, "
                         "jeffery_domain, drift_superposition, squirmer_starts, squirmer_feedback: the network "
                         "retrained on the samples of a suspension it missed, stokes_start: the start field's "
                         "time on the 256-box ensemble)")
    ap.add_argument("--surrogate-runs", type=int, default=4,
                    help="256-box FP16 ensembles run to train the warm-start network (0: skip steps to steady)")
    ap.add_argument("--eval-boxes", type=int, default=64, help="held-out force-driven boxes for steps to steady")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe-bytes", type=int, default=1 << 30,
                    help="size of the copy used as the achievable-bandwidth reference")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script into "
                         "profiles/collide_stream_traffic.json and exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        if args.variant is None:
            raise SystemExit("--summarize-pmc needs the --variant the counter runs used")
        summarize_pmc(*args.summarize_pmc, workload=args.workload, storage=args.storage,
                      probe_bytes=args.probe_bytes, variant=args.variant)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not a measured path.", file=sys.stderr)
        sys.exit(2)

    from paper_2403_05443_amd import lbell
    lbell.load()
    if args.sweep_only:
        from paper_2403_05443_amd import runner, workloads
        t0 = time.perf_counter()
        studies = {
            "domain": lambda: runner.domain_sweep([32, 64, 128, 256, 512], a=7.5, b=2.5, nu=0.1, storage="fp32"),
            "resolution": lambda: runner.resolution_sweep([2.0, 2.5, 3.0, 4.0], r=3.0),
            "sphere_array": lambda: {L: runner.sphere_array_run(L) for L in (24, 32, 48, 64)},
            "jeffery_domain": lambda: [runner.jeffery_half_period(L) for L in (26, 32, 40, 48, 64)],
            "drift_superposition": lambda: runner.drift_superposition(bs=(2.0, 3.0, 4.0)),
            "stokes_start": lambda: runner.stokes_start_time(workloads.c4("fp16", 256)),
            "squirmer_feedback": lambda: runner.squirmer_feedback(
                lambda extra: runner.train_warm_network(seeds=4, boxes=256, epochs=1000, seed0=10, extra=extra)[0],
                workloads.c5("fp16"), workloads.c5("fp16", seed_index=1),
                log=lambda m: print(m, file=sys.stderr, flush=True)),
            "squirmer_starts": lambda: runner.squirmer_starts(
                workloads.c5("fp16"), runner.train_warm_network(seeds=4, boxes=256, epochs=1000, seed0=10)[0],
                log=lambda m: print(m, file=sys.stderr, flush=True)),
        }
        out = {"kind": "studies of the settling spheroid (Sec. III.A-C, Figs. 4 and 9) and of the squirmer "
                       "suspension's starts (Sec. III.D)", "data": "synthetic"}
        for name in args.studies.split(","):
            out[name] = studies[name]()
        out["seconds"] = round(time.perf_counter() - t0, 1)
        print(json.dumps(out), flush=True)
        return
    W = workload_by_name(args.workload, args.storage)
    copy_gbs = lbell.bandwidth_probe(args.probe_bytes, reps=5)
    lat, m = measure(W, args.steps, args.warmup, args.graph, variant=args.variant)
    del lat
    _progress(f"headline {W.name}/{args.storage}: {m['mlups']:.1f} MLUPS, variant {m['variant']}")
    src_sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    traffic = traffic_record(src_sha, W.name, args.storage, m["variant"])
    rm = roofline_mlups(W)
    out = {
        "metric": METRIC,
        "value": round(m["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.storage],
        "data": "synthetic",
        "config": {"workload": W.name, "boxes": len(W.boxes), "sites": W.sites, "particles": len(W.particles),
                   "lattice": f"D3Q{W.lattice}", "storage": args.storage, "collision": W.collision,
                   "tau_plus": W.tau, "lambda": W.magic, "graph_steps": args.graph, "parallelism": "1 GPU"},
        "roofline_mlups": round(rm, 1),
        "frac_of_roofline_mlups": round(m["mlups"] / rm, 4),
        "roofline": {"bound": "hbm", "achieved": round(m["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(m["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_collide_stream", "variant": m["variant"], "bytes_per_launch": m["alg_bytes"],
                     "avg_launch_ms": round(m["k1_ms"], 5), "copy_probe_gbs": round(copy_gbs, 1),
                     "source_sha256": src_sha,
                     "working_set_bytes": m["working_set"], "cache_resident": m["working_set"] <= MALL_BYTES},
        "phase_ms_per_step": {k: round(v, 5) for k, v in m["phase_ms"].items()},
        "wall_s": round(m["wall_s"], 3),
        "legs": {},
    }
    legs = [] if args.legs in ("", "none") else args.legs.split(",")
    for name in legs:
        wname, storage, steps, warm = LEGS[name]
        Wl = workload_by_name(wname, storage)
        lat, e = measure(Wl, steps, warm, args.graph)
        del lat
        out["legs"][name] = leg_record(Wl, e, src_sha, steps)
        _progress(f"leg {name}: {e['mlups']:.1f} MLUPS, variant {e['variant']}")
    if args.surrogate_runs > 0:
        out["steps_to_steady"] = steps_to_steady(args.surrogate_runs, args.eval_boxes)
        _progress("steps to steady done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_seconds)
        _progress("cpu baseline done")
        out["cpu_reference"] = cpu_reference()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
