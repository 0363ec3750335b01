"""Throughput of the explicit MPM step on one MI355X.

Workload (default, ``--workload batch``): the batched set -- 256 independent
scenes of 1k-250k particles each (log-uniform), elastic or Drucker-Prager
blocks on meshes of 0.02 m cells, CFL 0.3 -- advanced together, one launch per
stage, FP32 particle state with FP64 positions and nodal mass.  One "step" is
one full update-stress-first time step (reorder check, nodal clear, P2G,
stress + force, G2P) of every particle of every scene.  Inputs are resident in
device memory before timing starts.

Prints one JSON line: batched particle-updates/s over exactly K timed steps
(after an untimed warm-up call that tunes the launch shape and records the
K-step HIP graphs, and a second one that launches them once), the plain
one-scene-at-a-time rate over the same steps,
p50/p99 per-scene completion latency of both over the set's own 500 steps,
the dominant kernel's achieved bandwidth against the HBM peak (from a pass in
which every kernel is launched between two HIP events on the library's
stream), the FP64 oracle timed on a bounded sample on the host CPU, and the
granular column's full 1000-step run.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload batch|column|column_gimp|column_usl|column_musl|column_gimp_usl|column_gimp_musl|column_iso|plate|c1|c5|c5_linear|c5_compare|serve]
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
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ITEM_KERNELS = ("p2g", "stress", "g2p_p2g", "p2g_usl", "g2p_usl", "p2g_musl", "musl_g2p", "musl_stress")
METRIC = "particle-updates/s (FP32 batched vs plain) at stated error; p50/p99 scene latency"


def kernel_bytes(kernel: str, n_particles: int, n_nodes: int) -> int:
    """Algorithmic HBM bytes of one launch: every particle field the stage
    needs read once and written once, every touched node's fields once.
    Particle: x 24 B (FP64), v 12, sigma 24, vol 4, mass 4, cell 4.
    Node: mass 8 B (FP64), momentum 12, force 12."""
    per_particle = {
        "p2g": 24 + 12 + 4 + 4,                            # read x, v, mass, cell
        "stress": (24 + 4 + 4 + 4 + 24) + (24 + 4),        # read x, cell, mass, vol, sigma; write sigma, vol
        "g2p_p2g": (24 + 12 + 4 + 4) + (24 + 12 + 4),      # read x, v, cell, mass; write x, v, cell
        "p2g_usl": 24 + 12 + 4 + 4 + 24 + 4,
        "g2p_usl": (24 + 12 + 4 + 24 + 4) + (24 + 12 + 4 + 24 + 4),
        "p2g_musl": 24 + 12 + 4 + 4 + 24 + 4,
        "musl_g2p": (24 + 12 + 4 + 4) + 12,                 # read x, v, cell, mass; write v
        "musl_stress": (24 + 4 + 4 + 24) + (24 + 4 + 24 + 4),   # read x, cell, vol, sigma; write x, vol, sigma, cell
    }
    # MUSL nodes also carry the remapped momentum r (12 B): cleared by
    # p2g_musl, written by musl_g2p, read by musl_stress
    per_node = {"p2g": 20, "stress": 20 + 12 + 32, "g2p_p2g": 32 + 20, "p2g_usl": 32, "g2p_usl": 32 + 32,
                "p2g_musl": 32 + 12, "musl_g2p": 32 + 12, "musl_stress": 32 + 12 + 32}
    return per_particle.get(kernel, 0) * n_particles + per_node.get(kernel, 0) * n_nodes


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("mpmx_kernels.hip", "mpmx_api.hip", "mpmx_dev.h", "mpmx_launch.h"):
        with open(os.path.join(ROOT, "paper_1909_13380_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return None
    entry = data.get(workload, {}).get(kernel)
    if not entry or entry.get("source_hash") != source_hash():
        return None
    return entry.get("bytes_per_launch")


def make_workload(name: str):
    from paper_1909_13380_amd import scenes
    if name == "column":
        return scenes.c2(), "granular column, DP, 2,097,152 particles, 256x128x160 mesh, linear"
    if name == "column_gimp":
        sc = scenes.c2()
        sc["scheme"]["shape"] = scenes.SHAPE_GIMP
        return sc, "granular column, DP, 2,097,152 particles, 256x128x160 mesh, GIMP"
    if name == "column_usl":
        sc = scenes.c2()
        sc["scheme"]["algo"] = scenes.USL
        return sc, "granular column, DP, 2,097,152 particles, 256x128x160 mesh, linear, USL"
    if name in ("column_gimp_usl", "column_gimp_musl"):
        sc = scenes.c2()
        sc["scheme"]["shape"] = scenes.SHAPE_GIMP
        sc["scheme"]["algo"] = scenes.USL if name == "column_gimp_usl" else scenes.MUSL
        return sc, ("granular column, DP, 2,097,152 particles, 256x128x160 mesh, GIMP, "
                    + ("USL" if name == "column_gimp_usl" else "MUSL"))
    if name == "column_musl":
        sc = scenes.c2()
        sc["scheme"]["algo"] = scenes.MUSL
        return sc, "granular column, DP, 2,097,152 particles, 256x128x160 mesh, linear, MUSL"
    if name == "column_iso":
        return (scenes.distort(scenes.c2(), amp=0.25, seed=2),
                "granular column, DP, 2,097,152 particles, 256x128x160 isoparametric mesh (uniform grid moved by a "
                "smooth field of 0.25 h), linear")
    if name == "plate":
        return (scenes.plate_with_hole(),
                "plate with a hole (quarter strip), 40,153 particles, 66x41x1 mesh, linear, elastic, PIC")
    if name == "c1":
        return scenes.c1(), "elastic block, 4,096 particles, 16^3 mesh, linear"
    if name == "c5":
        return scenes.c5(), "large granular column, DP, 25,165,824 particles, 512x256x128 mesh, GIMP"
    if name == "c5_linear":
        return (scenes.c5(shape=scenes.SHAPE_LINEAR),
                "large granular column, DP, 25,165,824 particles, 512x256x128 mesh, linear")
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(sc: dict, steps: int) -> dict:
    import oracle
    grid = oracle.Grid(sc["mesh"], sc["scheme"]["shape"])
    oracle.run(sc, 1, grid=grid)          # first touch of the nodal arrays
    t0 = time.perf_counter()
    oracle.run(sc, steps, grid=grid)
    dt = time.perf_counter() - t0
    n = len(sc["x"])
    return {"value": n * steps / dt, "unit": "particle-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {steps} steps of the same scene ({n} particles), FP64, one thread",
            "seconds": round(dt, 3)}


def _oracle_job(job):
    import oracle
    sc, steps = job
    oracle.run(sc, steps)
    return len(sc["x"]) * steps


def cpu_baseline_parallel(scs: list, steps: int, cores: int) -> dict:
    """The oracle on `cores` host processes at once, one scene per task
    (scene-parallel), over the given sample; wall time of the whole pool,
    first touch of each scene's nodal arrays included.  Runs before the
    process touches the GPU (the workers are forked)."""
    import multiprocessing as mpr
    with mpr.get_context("fork").Pool(cores) as pool:
        t0 = time.perf_counter()
        jobs = sorted(((sc, steps) for sc in scs), key=lambda j: -len(j[0]["x"]))   # largest first
        pu = sum(pool.map(_oracle_job, jobs, chunksize=1))
        dt = time.perf_counter() - t0
    return {"value": pu / dt, "unit": "particle-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(scs)} scenes of the set spread over its sizes ({sum(len(s['x']) for s in scs)} "
                      f"particles), {steps} steps each, FP64, scene-parallel", "seconds": round(dt, 3)}


def _csv_rows(root: str, suffix: str):
    import csv
    for dirpath, _, files in os.walk(root):
        for f in files:
            if f.endswith(suffix):
                with open(os.path.join(dirpath, f), newline="") as fh:
                    yield from csv.DictReader(fh)


def _short(name: str) -> str:
    name = name.split("(")[0].replace("void ", "").replace("mpmx::", "")
    return name.strip()


def _base(name: str) -> str:
    """The library's name of a kernel instantiation: k_stress<float, 0, 256>
    is "stress"; k_p2g with the force (USL) is "p2g_usl", and with the force
    and the remap clear (MUSL) "p2g_musl"."""
    base = name.split("<")[0].replace("k_", "")
    targs = [a.strip() for a in name[len(name.split("<")[0]) + 1:-1].split(",")] if "<" in name else []
    if base == "p2g" and len(targs) > 2 and targs[2] == "true":
        return "p2g_musl" if len(targs) > 4 and targs[4] == "true" else "p2g_usl"
    return base


def _counter_means(root: str) -> dict:
    """Mean counter value per dispatch, per kernel and counter, from the
    counter_collection CSV files under root."""
    acc: dict = {}
    for r in _csv_rows(root, "counter_collection.csv"):
        key = (_short(r["Kernel_Name"]), r["Counter_Name"])
        tot = acc.setdefault(key, {})
        d = r.get("Dispatch_Id", str(len(tot)))
        tot[d] = tot.get(d, 0.0) + float(r["Counter_Value"])
    return {k: sum(v.values()) / len(v) for k, v in acc.items()}


def summarize(root: str, workload: str, commands: str, out_name: str = ""):
    """Kernel-trace statistics and HBM traffic per launch from rocprofv3 CSV
    output: root/trace (--kernel-trace --stats), root/copy_FETCH_SIZE,
    root/copy_WRITE_SIZE (the 1 GiB device copy of --calibrate-copy 1024),
    root/FETCH_SIZE, root/WRITE_SIZE (the step).  Counters are KiB per
    dispatch; each is scaled by (known bytes of the copy) / (what the same
    counter reads for the copy kernel).  `out_name`, if given, names the summary
    file and the traffic entry instead of the workload."""
    stats = list(_csv_rows(os.path.join(root, "trace"), "kernel_stats.csv"))
    lines = [f"# rocprofv3 kernel statistics: {workload}", "", "Commands (repository root, rocprofv3 from ROCm 7.2):", ""]
    lines += [f"    {c}" for c in commands.split(";;") if c.strip()] + [""]
    lines.append(f"{'kernel':34s} {'calls':>7s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_%':>8s}")
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"{_short(r['Name'])[:34]:34s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):8.2f}")
    bench_line = None
    log = os.path.join(root, "trace.log")
    if os.path.exists(log):
        for ln in open(log):
            if ln.startswith("{") and '"metric"' in ln:
                bench_line = json.loads(ln)
    if bench_line and "kernels" in bench_line:
        lines += ["", "Same run, HIP events around each launch on the library's stream (bench.py's own timing):",
                  f"ms_per_step {bench_line['ms_per_step']:.4f}, value {bench_line['value']:.4g} "
                  f"{bench_line['unit']}", ""]
        lines.append(f"{'kernel':34s} {'events_avg_us':>14s} {'rocprof_avg_us':>15s}")
        # item kernels exist per workgroup size: compare the instantiation the
        # tuned launch shape used
        launch = bench_line.get("config", {}).get("launch", {})
        want = {"stress": launch.get("stress_threads"), "g2p_p2g": launch.get("g2p_threads"),
                "p2g": launch.get("g2p_threads"), "p2g_usl": launch.get("stress_threads"),
                "g2p_usl": launch.get("g2p_threads"), "p2g_musl": launch.get("stress_threads"),
                "musl_g2p": launch.get("g2p_threads"), "musl_stress": launch.get("g2p_threads")}
        rp = {}
        for r in stats:
            name = _short(r["Name"])
            base = _base(name)
            targs = [a.strip() for a in name[len(name.split("<")[0]) + 1:-1].split(",")] if "<" in name else []
            threads = targs[3] if base in ("p2g", "p2g_usl", "p2g_musl") and len(targs) > 3 else (targs[-1] if targs else "")
            if base in want and want[base] is not None and threads != str(want[base]):
                continue
            rp[base] = (float(r["AverageNs"]) / 1e3, name)
        for k, v in sorted(bench_line["kernels"].items()):
            avg, name = rp.get(k, (float("nan"), ""))
            lines.append(f"{k:34s} {v['avg_us']:14.2f} {avg:15.2f}   {name}")
    traffic = {}
    copy_bytes = 1024 << 20
    scale = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        cm = _counter_means(os.path.join(root, "copy_" + c))
        kib = [v for (k, cn), v in cm.items() if cn == c and "copyBuffer" in k]
        if kib:
            scale[c] = copy_bytes / (max(kib) * 1024.0)
    if len(scale) == 2:
        lines += ["", "HBM traffic per launch (rocprofv3 --pmc, KiB per dispatch scaled by the copy calibration:",
                  f"FETCH_SIZE x {scale['FETCH_SIZE']:.4f}, WRITE_SIZE x {scale['WRITE_SIZE']:.4f}; "
                  f"the copy moves {copy_bytes} bytes each way)", ""]
        lines.append(f"{'kernel':34s} {'read_MB':>10s} {'write_MB':>10s} {'total_MB':>10s}")
        fm = _counter_means(os.path.join(root, "FETCH_SIZE"))
        wm = _counter_means(os.path.join(root, "WRITE_SIZE"))
        for k in sorted({k for k, _ in fm} & {k for k, _ in wm}):
            rd = fm[(k, "FETCH_SIZE")] * 1024.0 * scale["FETCH_SIZE"]
            wr = wm[(k, "WRITE_SIZE")] * 1024.0 * scale["WRITE_SIZE"]
            lines.append(f"{k[:34]:34s} {rd / 1e6:10.2f} {wr / 1e6:10.2f} {(rd + wr) / 1e6:10.2f}")
            base = _base(k)
            entry = {"bytes_per_launch": rd + wr, "read_bytes": rd, "write_bytes": wr, "source_hash": source_hash(),
                     "instantiation": k}
            # one entry per kernel: the tuned instantiation when there are several
            tw = (bench_line or {}).get("config", {}).get("launch", {})
            t_use = {"stress": tw.get("stress_threads"), "g2p_p2g": tw.get("g2p_threads"),
                     "p2g_usl": tw.get("stress_threads"), "g2p_usl": tw.get("g2p_threads"),
                     "p2g_musl": tw.get("stress_threads"), "musl_g2p": tw.get("g2p_threads"),
                     "musl_stress": tw.get("g2p_threads")}.get(base)
            targs = [a.strip() for a in k[len(k.split("<")[0]) + 1:-1].split(",")] if "<" in k else []
            threads = targs[3] if base in ("p2g", "p2g_usl", "p2g_musl") and len(targs) > 3 else (targs[-1] if targs else "")
            if base in traffic and t_use is not None and threads != str(t_use):
                continue
            traffic[base] = entry
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    default = {"column": "step_kernels_column_2m", "column_gimp": "step_kernels_column_2m_gimp",
               "column_usl": "step_kernels_column_2m_usl", "column_musl": "step_kernels_column_2m_musl",
               "plate": "step_kernels_plate_40k", "c1": "step_kernels_block_4k", "batch": "step_kernels_batch_256",
               "c5": "step_kernels_column_25m_gimp"}.get(workload, "step_kernels_" + workload)
    fname = out_name or default
    with open(os.path.join(ROOT, "profiles", fname + ".txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if traffic:
        path = os.path.join(ROOT, "profiles", "traffic.json")
        data = json.load(open(path)) if os.path.exists(path) else {}
        # the workload's own profile is what its bench line reads; other
        # profiles of it (e.g. a forced reorder every step) keep their name
        data[workload if fname == default else fname] = traffic
        with open(path, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
    print("\n".join(lines))


def summarize_counters(root: str, workload: str, commands: str, out_name: str):
    """SQ instruction counters per dispatch from rocprofv3 --pmc passes
    (root/pmc_*), with the kernel trace of the same command (root/trace):
    for each item kernel, instructions per particle (wave instructions x 64
    lanes / particles) and issue rates per CU and cycle (wave instructions /
    (256 CUs x average duration x 2.4 GHz)).  Counter values are summed over
    the counter's hardware instances within a dispatch, then averaged over
    dispatches."""
    import glob
    if workload == "batch":
        from paper_1909_13380_amd import scenes
        n = sum(len(sc["x"]) for sc in scenes.c3())
        desc = f"the batched set: 256 scenes, {n} particles"
    else:
        sc, desc = make_workload(workload)
        n = len(sc["x"])
    dur = {_short(r["Name"]): float(r["AverageNs"]) for r in _csv_rows(os.path.join(root, "trace"), "kernel_stats.csv")}
    means: dict = {}
    for d in sorted(glob.glob(os.path.join(root, "pmc_*"))):
        means.update(_counter_means(d))
    kernels = sorted({k for k, _ in means if _base(k) in ITEM_KERNELS})
    counters = sorted({c for _, c in means})
    lines = [f"# rocprofv3 SQ counters: {desc}", "", "Commands (repository root, rocprofv3 from ROCm 7.2):", ""]
    lines += [f"    {c}" for c in commands.split(";;") if c.strip()] + [""]
    lines.append("Per dispatch (wave instructions, or cycles for SQ_ACTIVE_* and SQ_BUSY_*):")
    lines.append("")
    lines.append(f"{'counter':32s} " + " ".join(f"{k[:26]:>26s}" for k in kernels))
    for c in counters:
        lines.append(f"{c:32s} " + " ".join(f"{means.get((k, c), float('nan')):26.4g}" for k in kernels))
    lines += ["", f"Derived ({n} particles; average durations from the trace):", ""]
    lines.append(f"{'':32s} " + " ".join(f"{k[:26]:>26s}" for k in kernels))
    lines.append(f"{'avg duration (us)':32s} " + " ".join(f"{dur.get(k, float('nan')) / 1e3:26.2f}" for k in kernels))
    for c, label in (("SQ_INSTS_LDS_ATOMIC", "LDS atomics per particle"), ("SQ_INSTS_LDS_LOAD", "LDS loads per particle"),
                     ("SQ_INSTS_VALU", "VALU instr per particle"), ("SQ_INSTS_SALU", "SALU instr per particle")):
        if any((k, c) in means for k in kernels):
            lines.append(f"{label:32s} " + " ".join(f"{means.get((k, c), float('nan')) * 64 / n:26.2f}" for k in kernels))
    for c, label in (("SQ_INSTS_LDS_ATOMIC", "LDS atomics / CU / cycle"), ("SQ_INSTS_LDS_LOAD", "LDS loads / CU / cycle"),
                     ("SQ_INSTS_VALU", "VALU instr / CU / cycle")):
        if any((k, c) in means for k in kernels):
            lines.append(f"{label:32s} " + " ".join(
                f"{means.get((k, c), float('nan')) / (256 * dur.get(k, float('nan')) * 2.4):26.4f}" for k in kernels))
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", out_name + ".txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def apply_launch_options(ctx, args):
    from paper_1909_13380_amd import mpmx
    for opt, val in ((mpmx.OPT_STRESS_THREADS, args.stress_threads), (mpmx.OPT_G2P_THREADS, args.g2p_threads),
                     (mpmx.OPT_BLOCKS_PER_CU, args.blocks_per_cu),
                     (mpmx.OPT_STRESS_BLOCKS_PER_CU, args.stress_blocks_per_cu),
                     (mpmx.OPT_G2P_BLOCKS_PER_CU, args.g2p_blocks_per_cu)):
        if val:
            ctx.set_option(opt, val)
    if args.graph_steps >= 0:
        ctx.set_option(mpmx.OPT_GRAPH_STEPS, args.graph_steps)


def _percentiles(vals):
    v = np.sort(np.asarray(vals, dtype=np.float64))
    return {"p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99)),
            "max_ms": float(v[-1]), "n": int(len(v))}


def host_identity() -> dict:
    """The host CPU the oracle baseline ran on: logical CPUs and model name."""
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    return {"host_cpus": os.cpu_count() or 1, "host_cpus_available": avail, "cpu_model": model}


def active_nodes(mesh: dict, counts: np.ndarray) -> int:
    """Nodes of the occupied cells (linear shape functions): the nodes a
    step's transfers touch."""
    nx, ny, nz = (int(c) for c in mesh["n"])
    cells = np.flatnonzero(counts)
    cx, cy, cz = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    ids = []
    for dk in (0, 1):
        for dj in (0, 1):
            for di in (0, 1):
                ids.append((cx + di) + (nx + 1) * ((cy + dj) + (ny + 1) * (cz + dk)))
    return int(np.unique(np.concatenate(ids)).size) if len(cells) else 0


def run_batch(args):
    """The batched set: 256 independent scenes (1k-250k particles, elastic
    or Drucker-Prager), FP32.  Batched: one launch per stage over all scenes.
    Plain: the same kernels per scene, scenes one after another in FIFO
    order.  Both legs first run an untimed warm-up call that tunes the launch
    shape and records the K-step HIP graphs; the batched leg then launches its
    graph once more untimed (a graph's first launch pays a one-time cost), so
    the timed call only replays.
    `value` is the batched rate over exactly K timed steps per scene; the
    plain rate over the same K steps stands beside it.  Latency: a second
    pair of runs over the set's own 500 steps, each scene's completion
    measured from the start of the run (HIP event after its last launch;
    in the batch every scene ends with the batch's last step)."""
    import torch
    from paper_1909_13380_amd import mpmx, scenes
    n_sc = args.scenes
    K = args.steps
    full_steps = 500
    scs = scenes.c3(n_sc, nsteps=full_steps)
    total = int(sum(len(sc["x"]) for sc in scs))
    print(f"# {n_sc} scenes, {total} particles", file=sys.stderr, flush=True)
    cb = cb_par = None
    if not args.no_cpu_baseline:
        # before anything touches the GPU: the pool forks
        ident = host_identity()
        by_size = sorted(scs, key=lambda sc: len(sc["x"]))
        one = by_size[:: max(1, len(by_size) // 8)][:8]
        print("# timing the oracle on the host", file=sys.stderr, flush=True)
        cb = cpu_baseline_scenes(one, args.cpu_steps * 40)
        cb.update(ident)
        cores = max(1, min(16, ident["host_cpus_available"]))
        sample = by_size[:: max(1, len(by_size) // (2 * cores))][: 2 * cores]
        cb_par = cpu_baseline_parallel(sample, 10, cores)
        cb_par.update(ident)
        cb_par["note"] = "16 worker processes at most: the CPU share of one GPU on the measurement host"
    torch.cuda.init()
    stream = torch.cuda.Stream()          # a real stream: the library and torch's events share it
    torch.cuda.set_stream(stream)
    ctx = mpmx.Context(0, stream=stream.cuda_stream)
    apply_launch_options(ctx, args)
    untimed = max(args.warmup, mpmx.TUNE_MIN_STEPS)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # --- batched: warm-up (tunes, records the graphs), then K timed steps
    batch = [ctx.create_scene(sc, precision=mpmx.FP32) for sc in scs]
    ctx.batch_step(batch, [untimed] * n_sc)
    gk = ctx.get_option(mpmx.OPT_GRAPH_STEPS)
    if gk > 0:   # the recorded graph's first launch, untimed
        ctx.batch_step(batch, [gk + 1] * n_sc)
        untimed += gk + 1
    g0 = ctx.get_option(mpmx.OPT_GRAPH_LAUNCHES)
    tb = timed(lambda: ctx.batch_step(batch, [K] * n_sc))
    launch_b = {"stress_threads": ctx.get_option(mpmx.OPT_STRESS_THREADS),
                "g2p_threads": ctx.get_option(mpmx.OPT_G2P_THREADS),
                "stress_blocks_per_cu": ctx.get_option(mpmx.OPT_STRESS_BLOCKS_PER_CU),
                "g2p_blocks_per_cu": ctx.get_option(mpmx.OPT_G2P_BLOCKS_PER_CU),
                "graph_steps": ctx.get_option(mpmx.OPT_GRAPH_STEPS),
                "graph_launches_in_timed_call": ctx.get_option(mpmx.OPT_GRAPH_LAUNCHES) - g0,
                "tune_runs": ctx.get_option(mpmx.OPT_TUNE_RUNS)}
    print(f"# batched: {K} steps in {tb * 1e3:.2f} ms", file=sys.stderr, flush=True)
    prof = {}
    if not args.no_profile:
        ctx.profile(True)
        ctx.profile_reset()
        ctx.batch_step(batch, [K] * n_sc)
        prof = ctx.profile_read()
        ctx.profile(False)
    n_nodes = 0
    for sc, b in zip(scs, batch):
        st = b.stats()
        if st["error_bits"]:
            raise SystemExit(f"batched scene {sc['name']} stopped with error bits {st['error_bits']}")
        n_nodes += active_nodes(sc["mesh"], b.cell_counts())
    for b in batch:
        b.destroy()
    if args.no_plain:
        ctx.close()
        out = {"metric": METRIC, "value": total * K / tb, "unit": "particle-updates/s", "n_gpus": 1, "steps": K,
               "warmup": args.warmup, "ms_per_step": 1e3 * tb / K, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
               "config": {"workload": f"batched: {n_sc} independent scenes (batched leg only)", "scenes": n_sc,
                          "particles": total, "touched_nodes": n_nodes, "launch": launch_b}}
        if prof:
            out["kernels"] = {k: {"launches": v[0], "avg_us": 1e3 * v[1] / max(v[0], 1), "total_ms": v[1]}
                              for k, v in prof.items()}
        print(json.dumps(out), flush=True)
        return
    # --- plain FIFO: same warm-up per scene, then K timed steps each
    plain = [ctx.create_scene(sc, precision=mpmx.FP32) for sc in scs]
    for s in plain:
        s.step(untimed)
    tp = timed(lambda: [s.step(K) for s in plain])
    print(f"# plain: {K} steps per scene in {tp * 1e3:.2f} ms", file=sys.stderr, flush=True)
    for s in plain:
        s.destroy()
    # --- latency over the set's own 500 steps, from the initial state
    lat = {}
    batch = [ctx.create_scene(sc, precision=mpmx.FP32) for sc in scs]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tfb = timed(lambda: (e0.record(), ctx.batch_step(batch, [full_steps] * n_sc), e1.record()))
    lat["batched"] = _percentiles([e0.elapsed_time(e1)] * n_sc)
    for b in batch:
        b.destroy()
    plain = [ctx.create_scene(sc, precision=mpmx.FP32) for sc in scs]
    evs = [torch.cuda.Event(enable_timing=True) for _ in plain]
    p0 = torch.cuda.Event(enable_timing=True)

    def fifo():
        p0.record()
        for s, e in zip(plain, evs):
            s.step(full_steps)
            e.record()
    tfp = timed(fifo)
    lat["plain"] = _percentiles([p0.elapsed_time(e) for e in evs])
    for s in plain:
        s.destroy()
    # --- the single large scene (granular column, 2.1M particles): its full
    # 1000-step run from the initial state in one call, reorders included
    col = None
    if not args.no_column:
        csc = scenes.c2()
        cs = ctx.create_scene(csc, precision=mpmx.FP32)
        tc = timed(lambda: cs.step(csc["nsteps"]))
        st = cs.stats()
        if st["error_bits"]:
            raise SystemExit(f"column stopped with error bits {st['error_bits']}")
        col = {"workload": "granular column, DP, 2,097,152 particles, 256x128x160 mesh, linear, USF, FP32",
               "steps": csc["nsteps"], "seconds": tc, "ms_per_step": 1e3 * tc / csc["nsteps"],
               "value": len(csc["x"]) * csc["nsteps"] / tc, "reorders": st["n_sorts"],
               "note": "one call from the initial state: first-step P2G, graph recording and every reorder "
                       "included"}
        cs.destroy()
        print(f"# column: {csc['nsteps']} steps in {tc * 1e3:.1f} ms, {st['n_sorts']} reorders",
              file=sys.stderr, flush=True)
    ctx.close()
    pu = total * K
    out = {"metric": METRIC, "value": pu / tb, "unit": "particle-updates/s", "n_gpus": 1, "steps": K,
           "warmup": args.warmup, "ms_per_step": 1e3 * tb / K, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"batched: {n_sc} independent scenes, 1k-250k particles each (log-uniform), "
                                  f"elastic or Drucker-Prager, 0.02 m cells, CFL 0.3, one launch per stage",
                      "scenes": n_sc, "particles": total, "touched_nodes": n_nodes,
                      "precision": "fp32 state, fp64 positions and nodal mass",
                      "untimed_steps_before": untimed, "launch": launch_b}}
    out["plain"] = {"value": pu / tp, "ms_per_step": 1e3 * tp / K,
                    "order": "FIFO, one scene at a time, same kernels, each scene warmed up alike"}
    out["speedup_vs_plain"] = tp / tb
    out["latency"] = {"steps": full_steps, "batched": lat["batched"], "plain": lat["plain"],
                      "batched_value": total * full_steps / tfb, "plain_value": total * full_steps / tfp,
                      "note": "per-scene completion from the start of a run from the initial state (first-call "
                              "work included); all scenes of the batch end with its last step"}
    if prof:
        kernels = {k: {"launches": v[0], "avg_us": 1e3 * v[1] / max(v[0], 1), "total_ms": v[1]}
                   for k, v in prof.items()}
        dom = max((k for k in kernels if k in ("stress", "g2p_p2g")), key=lambda k: kernels[k]["total_ms"])
        nbytes = kernel_bytes(dom, total, n_nodes)
        achieved = nbytes / (kernels[dom]["avg_us"] * 1e-6) / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, "batch"),
                           "algorithmic_bytes_per_launch": nbytes}
        out["kernels"] = kernels
        step_bytes = sum(kernel_bytes(k, total, n_nodes) for k in ("stress", "g2p_p2g"))
        out["step_algorithmic_GBs"] = step_bytes / (tb / K) / 1e9
    if cb is not None:
        out["cpu_baseline"] = cb
        out["cpu_baseline_parallel"] = cb_par
    if col is not None:
        out["column"] = col
    print(json.dumps(out), flush=True)


def cpu_baseline_scenes(scs: list, steps: int) -> dict:
    """The oracle on one host thread over a sample of the set's scenes, each
    for `steps` steps from its initial state (first touch of its nodal
    arrays outside the timing)."""
    import oracle
    pu, sec = 0, 0.0
    for sc in scs:
        grid = oracle.Grid(sc["mesh"], sc["scheme"]["shape"])
        oracle.run(sc, 1, grid=grid)
        t0 = time.perf_counter()
        oracle.run(sc, steps, grid=grid)
        sec += time.perf_counter() - t0
        pu += len(sc["x"]) * steps
    return {"value": pu / sec, "unit": "particle-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(scs)} scenes of the set spread over its sizes ({sum(len(s['x']) for s in scs)} "
                      f"particles), first {steps} steps of each, FP64, one thread", "seconds": round(sec, 3)}


def _serve_batched(mpmx, ctx, reqs, rate, tick_steps, budget, fill=0):
    """The request loop (continuous batching) on one arrival stream: submit
    each request at its arrival (particle arrays borrowed, results written to
    arrays allocated at submit, as the plain path's read allocates them),
    tick, collect completions.  Returns the
    latencies (arrival -> result on the host, ms), particle-updates and the
    span in seconds.  fill: the server's occupancy limit (particles; 0 off)."""
    srv = mpmx.Server(ctx, budget, max_tick_steps=tick_steps, fill_particles=fill)
    n_req = len(reqs)
    arrivals = [t / rate for t, _, _ in reqs]
    lat, pu, i, ticks = [], 0, 0, 0
    t0 = srv.clock()
    while len(lat) < n_req:
        now = srv.clock() - t0
        while i < n_req and arrivals[i] <= now:
            _, sc, k = reqs[i]
            srv.submit(sc, k, precision=mpmx.FP32, tag=i, borrow=True, out=True)
            i += 1
        r, q = srv.tick()
        ticks += 1
        for c in srv.poll(256, copy_state=False):
            if c["status"] != mpmx.OK:
                raise SystemExit(f"request {c['tag']} failed with status {c['status']}")
            lat.append(1e3 * (c["t_done"] - t0 - arrivals[c["tag"]]))
            pu += c["n"] * c["steps_done"]
        if r == 0 and q == 0 and i < n_req:
            time.sleep(max(0.0, min(0.002, arrivals[i] - (srv.clock() - t0))))
    span = srv.clock() - t0
    srv.close()
    return lat, pu, span, ticks


def _serve_plain(mpmx, ctx, reqs, rate):
    """The plain path on the same arrivals: one request at a time in arrival
    order, alone on the GPU (create, step, read back, free)."""
    import torch
    n_req = len(reqs)
    arrivals = [t / rate for t, _, _ in reqs]
    lat, pu = [], 0
    t0 = time.perf_counter()
    for i, (_, sc, k) in enumerate(reqs):
        wait = arrivals[i] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        s = ctx.create_scene(sc, precision=mpmx.FP32)
        s.step(k)
        s.read()
        s.destroy()
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - t0 - arrivals[i]))
        pu += len(sc["x"]) * k
    return lat, pu, time.perf_counter() - t0


def run_serve(args):
    """Serving: a Poisson stream of requests from the batched-scene
    generator (seed 4), steps uniform in 100..2000, admitted against a 64 GiB
    device budget by the library's request loop (continuous batching: uploads
    and read-backs overlap the running steps), final particle state returned
    to host memory; latency is arrival -> result on the host.  Beside it at
    every rate, the plain path on the same arrivals (one request at a time,
    alone on the GPU).  Then one rate of the stream of 2.1M-particle column
    requests, batched (without and with the occupancy limit) and plain."""
    import torch
    from paper_1909_13380_amd import mpmx, scenes
    n_req = args.requests
    rates = [float(r) for r in args.rates.split(",")]
    base = scenes.c4_requests(1.0, n_req)        # arrival times at 1/s; other rates scale them
    total_pu = int(sum(len(sc["x"]) * k for _, sc, k in base))
    print(f"# {n_req} requests generated, {total_pu:.3e} particle-updates", file=sys.stderr, flush=True)
    torch.cuda.init()
    ctx = mpmx.Context(0)
    apply_launch_options(ctx, args)
    budget = 64 << 30
    results = []
    for rate in rates:
        lat, pu, span, ticks = _serve_batched(mpmx, ctx, base, rate, args.tick_steps, budget, args.fill_particles)
        row = {"rate_per_s": rate, "requests": n_req, "seconds": span, "value": pu / span, "ticks": ticks,
               **_percentiles(lat)}
        if not args.no_plain:
            plat, ppu, pspan = _serve_plain(mpmx, ctx, base, rate)
            row["plain"] = {"seconds": pspan, "value": ppu / pspan, **_percentiles(plat)}
        print(f"# rate {rate}/s: {json.dumps(row)}", file=sys.stderr, flush=True)
        results.append(row)
    col = None
    if args.column_rate > 0:
        creqs = scenes.column_requests(1.0, args.column_requests)
        cpu_total = int(sum(len(sc["x"]) * k for _, sc, k in creqs))
        lat, pu, span, ticks = _serve_batched(mpmx, ctx, creqs, args.column_rate, args.tick_steps, budget)
        col = {"workload": f"serving: Poisson stream of {len(creqs)} granular-column requests (2,097,152 particles "
                           f"each, own jitter seed), 100-2000 steps each, 64 GiB budget",
               "rate_per_s": args.column_rate, "requests": len(creqs), "seconds": span, "value": pu / span,
               "ticks": ticks, "particle_updates": cpu_total, **_percentiles(lat)}
        if args.column_fill > 0:
            lat, pu, span, ticks = _serve_batched(mpmx, ctx, creqs, args.column_rate, args.tick_steps, budget,
                                                  args.column_fill)
            col["filled"] = {"fill_particles": args.column_fill, "seconds": span, "value": pu / span,
                             "ticks": ticks, **_percentiles(lat)}
        if not args.no_plain:
            plat, ppu, pspan = _serve_plain(mpmx, ctx, creqs, args.column_rate)
            col["plain"] = {"seconds": pspan, "value": ppu / pspan, **_percentiles(plat)}
        print(f"# column stream: {json.dumps(col)}", file=sys.stderr, flush=True)
    ctx.close()
    best = max(results, key=lambda r: r["value"])
    out = {"metric": METRIC, "value": best["value"], "unit": "particle-updates/s", "n_gpus": 1, "steps": None,
           "warmup": 0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
           "data": "synthetic",
           "config": {"workload": f"serving: Poisson stream of {n_req} requests per rate from the batched-scene "
                                  f"generator (seed 4), 1k-250k particles, 100-2000 steps each, 64 GiB budget",
                      "max_tick_steps": args.tick_steps, "fill_particles": args.fill_particles,
                      "particle_updates_per_rate": total_pu},
           "rates": results}
    if col is not None:
        out["column_stream"] = col
    print(json.dumps(out), flush=True)


def _shape_metrics(x0, x, v, mass, h):
    """Outcome measures of a column run: displacement, runout (front along x,
    the direction the column collapses), final height, kinetic energy."""
    u = x - x0
    return {"runout_m": float(x[:, 0].max() - x0[:, 0].max()), "height_m": float(x[:, 2].max()),
            "mean_settlement_m": float(-u[:, 2].mean()), "kinetic_energy_J": float(0.5 * (mass * (v * v).sum(1)).sum()),
            "moved_over_h": float((np.linalg.norm(u, axis=1) > h).mean())}


def run_c5_compare(args):
    """The large column with GIMP and with linear shape functions on the same
    inputs, all 500 steps each in FP32: throughput of each, and how the two
    results differ (relative L2 of the displacement difference, runout,
    height, settlement, kinetic energy).  Beside it, the same comparison on
    the 1/64 subsample scene: the GPU's GIMP and linear runs against the
    FP64 oracle's stored samples of both (tests/golden/c5sub_*_500.npz, made
    by tests/golden/make_c5sub_golden.py, which calls only the oracle)."""
    import torch
    from paper_1909_13380_amd import mpmx, scenes
    torch.cuda.init()
    ctx = mpmx.Context(0)
    apply_launch_options(ctx, args)
    out_runs = {}
    for name, shape in (("gimp", scenes.SHAPE_GIMP), ("linear", scenes.SHAPE_LINEAR)):
        sc = scenes.c5(shape=shape)
        k = sc["nsteps"]
        s = ctx.create_scene(sc, precision=mpmx.FP32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(k)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        got = s.read()
        st = s.stats()
        s.destroy()
        if st["error_bits"]:
            raise SystemExit(f"c5 {name} stopped with error bits {st['error_bits']}")
        out_runs[name] = {"x0": sc["x"], "x": got["x"], "v": got["v"], "mass": sc["mass"], "h": sc["mesh"]["h"],
                          "steps": k, "seconds": sec, "value": len(sc["x"]) * k / sec, "reorders": st["n_sorts"]}
        print(f"# c5 {name}: {k} steps in {sec:.3f} s", file=sys.stderr, flush=True)
    g, l = out_runs["gimp"], out_runs["linear"]
    ug, ul = g["x"] - g["x0"], l["x"] - l["x0"]
    full = {"particles": len(g["x0"]), "steps": g["steps"],
            "gimp": {"value": g["value"], "seconds": g["seconds"], "reorders": g["reorders"],
                     **_shape_metrics(g["x0"], g["x"], g["v"], g["mass"], g["h"])},
            "linear": {"value": l["value"], "seconds": l["seconds"], "reorders": l["reorders"],
                       **_shape_metrics(l["x0"], l["x"], l["v"], l["mass"], l["h"])},
            "displacement_difference_rel_l2": float(np.linalg.norm(ug - ul) / np.linalg.norm(ul))}
    # the 1/64 subsample: GPU runs of both shapes against the oracle's samples
    sub = {}
    gold_dir = os.path.join(ROOT, "tests", "golden")
    for name, shape in (("gimp", scenes.SHAPE_GIMP), ("linear", scenes.SHAPE_LINEAR)):
        path = os.path.join(gold_dir, f"c5sub_{name}_500.npz")
        if not os.path.exists(path):
            continue
        gold = np.load(path)
        sc = scenes.c5(subsample=True, shape=shape)
        s = ctx.create_scene(sc, precision=mpmx.FP32)
        s.step(int(gold["nsteps"]))
        got = s.read()
        s.destroy()
        idx = gold["index"]
        u_gpu, u_or = got["x"][idx] - gold["x0"], gold["x"] - gold["x0"]
        sub[name] = {"u_gpu": u_gpu, "u_oracle": u_or,
                     "err_u_vs_oracle": float(np.linalg.norm(u_gpu - u_or) / np.linalg.norm(u_or)),
                     "err_sigma_vs_oracle": float(np.linalg.norm(got["stress"][idx] - gold["stress"])
                                                  / np.linalg.norm(gold["stress"]))}
    ctx.close()
    subsample = None
    if len(sub) == 2:
        dg = sub["gimp"]["u_gpu"] - sub["linear"]["u_gpu"]
        do = sub["gimp"]["u_oracle"] - sub["linear"]["u_oracle"]
        subsample = {"sample": "every 64th of the 393,216 particles, 500 steps",
                     "gimp_err_u_vs_oracle": sub["gimp"]["err_u_vs_oracle"],
                     "linear_err_u_vs_oracle": sub["linear"]["err_u_vs_oracle"],
                     "gimp_err_sigma_vs_oracle": sub["gimp"]["err_sigma_vs_oracle"],
                     "linear_err_sigma_vs_oracle": sub["linear"]["err_sigma_vs_oracle"],
                     "oracle_displacement_difference_rel_l2": float(np.linalg.norm(do) /
                                                                    np.linalg.norm(sub["linear"]["u_oracle"])),
                     "gpu_displacement_difference_rel_l2": float(np.linalg.norm(dg) /
                                                                 np.linalg.norm(sub["linear"]["u_gpu"])),
                     "difference_of_differences_rel_l2": float(np.linalg.norm(dg - do) / np.linalg.norm(do))}
    line = {"metric": METRIC, "value": full["gimp"]["value"], "unit": "particle-updates/s", "n_gpus": 1,
            "steps": full["steps"], "warmup": 0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "fp32", "data": "synthetic",
            "config": {"workload": "large granular column, DP, 25,165,824 particles, 512x256x128 mesh, GIMP against "
                                   "linear on the same inputs, all 500 steps each, FP32"},
            "full_size": full, "subsample_vs_oracle": subsample}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="batch")
    ap.add_argument("--no-column", action="store_true",
                    help="--workload batch: skip the full 1000-step run of the granular column")
    ap.add_argument("--no-plain", action="store_true",
                    help="--workload batch: the batched leg only (no plain leg, latency runs or column), for profiling; "
                         "--workload serve: no plain path beside the request loop")
    ap.add_argument("--sort", default="on_demand", choices=["on_demand", "always"])
    ap.add_argument("--cpu-steps", type=int, default=5, help="oracle steps of the CPU baseline (batch: 40x this)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip per-kernel HIP event timing")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (a plain copy kernel of known size, for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--summarize", metavar="DIR",
                    help="only summarize the rocprofv3 CSV output under DIR (kernel trace + counter passes) "
                         "into profiles/ and exit; no GPU needed")
    ap.add_argument("--commands", default="", help="with --summarize: the commands that produced DIR")
    ap.add_argument("--profile-name", default="", help="with --summarize: name of the summary file and traffic entry")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="write the SQ counter summary of rocprofv3 --pmc passes DIR/pmc_* (with DIR/trace) to profiles/")
    ap.add_argument("--stress-threads", type=int, default=0, help="fixed workgroup size (turns autotuning off)")
    ap.add_argument("--g2p-threads", type=int, default=0, help="fixed workgroup size (turns autotuning off)")
    ap.add_argument("--blocks-per-cu", type=int, default=0,
                    help="fixed grid density of both item kernels (turns autotuning off)")
    ap.add_argument("--stress-blocks-per-cu", type=int, default=0,
                    help="fixed grid density of the stress-side kernel (turns autotuning off)")
    ap.add_argument("--g2p-blocks-per-cu", type=int, default=0,
                    help="fixed grid density of the G2P-side kernel (turns autotuning off)")
    ap.add_argument("--graph-steps", type=int, default=-1, help="steps per recorded HIP graph (0: none; default: the library's)")
    ap.add_argument("--scenes", type=int, default=256, help="--workload batch: number of scenes")
    ap.add_argument("--requests", type=int, default=2000, help="--workload serve: requests per arrival rate")
    ap.add_argument("--rates", default="50,100,150",
                    help="--workload serve: arrival rates (requests/s); about 0.3, 0.6 and 0.9 of the saturated rate")
    ap.add_argument("--tick-steps", type=int, default=64, help="--workload serve: most steps per server tick")
    ap.add_argument("--column-rate", type=float, default=0.0,
                    help="--workload serve: also run the stream of 2.1M-particle column requests at this rate (req/s)")
    ap.add_argument("--column-requests", type=int, default=40, help="--workload serve: column requests")
    ap.add_argument("--fill-particles", type=int, default=0,
                    help="--workload serve: the server's occupancy limit for the batched-scene stream (0: off)")
    ap.add_argument("--column-fill", type=int, default=2000000,
                    help="--workload serve: the column stream again with this occupancy limit (0: skip)")
    args = ap.parse_args()
    args.steps_given = any(a == "--steps" or a.startswith("--steps=") for a in sys.argv[1:])
    if args.summarize:
        summarize(args.summarize, args.workload, args.commands, args.profile_name)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.workload, args.commands,
                           args.profile_name or "sq_counters_" + args.workload)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        raise SystemExit(2)

    import torch
    if args.calibrate_copy:
        n = args.calibrate_copy << 18   # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes_each_way": n * 4, "launches": 3}))
        return
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "c5_compare":
        run_c5_compare(args)
        return
    from paper_1909_13380_amd import mpmx

    sc, desc = make_workload(args.workload)
    n = len(sc["x"])
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = mpmx.Context(0, stream=stream.cuda_stream)
    apply_launch_options(ctx, args)
    policy = mpmx.SORT_ALWAYS if args.sort == "always" else mpmx.SORT_ON_DEMAND
    s = ctx.create_scene(sc, precision=mpmx.FP32, sort_policy=policy)
    print(f"# scene created: {desc}", file=sys.stderr, flush=True)
    # untimed: the warm-up, which also runs the launch-shape tuner (it needs
    # a call of at least TUNE_MIN_STEPS steps)
    untimed = max(args.warmup, mpmx.TUNE_MIN_STEPS)
    s.step(untimed)
    gk = ctx.get_option(mpmx.OPT_GRAPH_STEPS)
    if gk > 0:   # the recorded graph's first launch, untimed
        s.step(gk + 1)
        untimed += gk + 1
    torch.cuda.synchronize()
    nodes = s.nodes()
    n_nodes = int(np.count_nonzero(nodes["m"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"# timed {args.steps} steps: {1e3 * (t1 - t0) / args.steps:.4f} ms/step", file=sys.stderr, flush=True)
    launch = {"stress_threads": ctx.get_option(mpmx.OPT_STRESS_THREADS),
              "g2p_threads": ctx.get_option(mpmx.OPT_G2P_THREADS),
              "stress_blocks_per_cu": ctx.get_option(mpmx.OPT_STRESS_BLOCKS_PER_CU),
              "g2p_blocks_per_cu": ctx.get_option(mpmx.OPT_G2P_BLOCKS_PER_CU),
              "graph_steps": ctx.get_option(mpmx.OPT_GRAPH_STEPS),
              "graph_launches": ctx.get_option(mpmx.OPT_GRAPH_LAUNCHES)}
    prof = {}
    if not args.no_profile:
        # per-kernel durations: the same number of steps again, every kernel
        # launched directly between a pair of HIP events on the library's stream
        ctx.profile(True)
        ctx.profile_reset()
        s.step(args.steps)
        prof = ctx.profile_read()
        ctx.profile(False)
    st = s.stats()
    if st["error_bits"]:
        raise SystemExit(f"scene stopped with error bits {st['error_bits']}")
    elapsed = t1 - t0
    value = n * args.steps / elapsed
    out = {"metric": METRIC, "value": value, "unit": "particle-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": desc, "particles": n, "mesh": list(sc["mesh"]["n"]), "dt": sc["scheme"]["dt"],
                      "precision": "fp32 state, fp64 positions and nodal mass", "sort_policy": args.sort,
                      "reorders_in_run": st["n_sorts"], "work_items": st["n_items"], "touched_nodes": n_nodes,
                      "untimed_steps_before": untimed, "launch": launch}}
    if prof:
        kernels = {k: {"launches": v[0], "avg_us": 1e3 * v[1] / max(v[0], 1), "total_ms": v[1]}
                   for k, v in prof.items()}
        dom = max((k for k in kernels if k in ITEM_KERNELS), key=lambda k: kernels[k]["total_ms"])
        avg_s = kernels[dom]["avg_us"] * 1e-6
        nbytes = kernel_bytes(dom, n, n_nodes)
        achieved = nbytes / avg_s / 1e9
        traffic = measured_traffic(dom, args.workload)
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "algorithmic_bytes_per_launch": nbytes}
        out["kernels"] = kernels
        # the kernels every step runs: USF stress + g2p_p2g, USL p2g_usl +
        # g2p_usl, MUSL p2g_musl + musl_g2p + musl_stress
        step_kernels = {0: ("stress", "g2p_p2g"), 1: ("p2g_usl", "g2p_usl"),
                        2: ("p2g_musl", "musl_g2p", "musl_stress")}[sc["scheme"]["algo"]]
        step_bytes = sum(kernel_bytes(k, n, n_nodes) for k in step_kernels)
        out["step_algorithmic_GBs"] = step_bytes / (elapsed / args.steps) / 1e9
    if not args.no_cpu_baseline:
        print("# timing the oracle on the host", file=sys.stderr, flush=True)
        if args.workload == "column_iso":
            # the oracle locates isoparametric particles by searching every
            # cell: a small distorted block stands in
            from paper_1909_13380_amd import scenes as _sc
            sub = _sc.distort(_sc.random_block(n_cells=(9, 7, 6), mesh_cells=(14, 11, 9), h=0.05, seed=21,
                                               material=_sc.drucker_prager()), amp=0.25, seed=2)
            cb = cpu_baseline(sub, args.cpu_steps * 4)
            cb["sample"] = (f"first {args.cpu_steps * 4} steps of a distorted Drucker-Prager block "
                            f"({len(sub['x'])} particles, 14x11x9 isoparametric mesh), FP64, one thread")
        elif args.workload in ("c5", "c5_linear"):
            from paper_1909_13380_amd import scenes as _sc
            sub = _sc.c5(subsample=True, shape=sc["scheme"]["shape"])
            cb = cpu_baseline(sub, args.cpu_steps)
            cb["sample"] = (f"first {args.cpu_steps} steps of the 1/64 subsample of the same column "
                            f"({len(sub['x'])} particles), FP64, one thread")
        else:
            cb = cpu_baseline(sc, args.cpu_steps)
        cb["cores"] = 1
        out["cpu_baseline"] = cb
    s.destroy()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
