"""Throughput of the spherical-harmonics hot path on one MI355X.

One step = the forward with gradients (Y[N,81] and dY[N,3,81] from xyz[N,3],
sph_compute_with_gradients) followed by the backward (grad_xyz[N,3] from the
stored dY and an upstream gradient grad_Y[N,81], sph_backward), for
N = 1,000,000 points with iid N(0,1) coordinates, l_max = 8, float32,
normalised harmonics.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line:  points/s (value), ms per step, the roofline of the
dominant kernel (algorithmic bytes per launch / mean launch time from HIP
events recorded around each launch on the launch stream), the per-kernel
figures, secondary measurements of the other workloads, and the oracle timed
on the host cores on a bounded sample; the oracle's results for 2048 rows of
that sample also check the GPU's rows (accuracy).

    python bench.py [--gpus 1] [--steps 50] [--warmup 10] [--no-cpu-baseline]

Profiling (rocprofv3 runs of `bench.py --profile`, commands in
PROFILE_COMMANDS) and their summaries under profiles/:

    python bench.py --summarize DIR    # DIR holds the rocprofv3 output folders
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

N_POINTS = 1_000_000
L_MAX = 8
NORMALIZE = True
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "points/s and HBM GB/s for Y+dY fwd+bwd, l_max=8 FP32; max err vs FP64 oracle"
# The sources of the headline step's two kernels (their code, tables and
# launch shapes): a change to any of them voids the committed byte counters.
KERNEL_SOURCES = ["sph_device.hpp", "sph_coeffs.hpp", "sph_fwd.inl", "sph_fwd1.inl", "sph_fwd4.inl", "sph_bwd.inl",
                  "sph_instances.inl", "sph_kernels_derivs_f32_n1_m0.hip", "sph_kernels_bwd_f32.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_l8_f32.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2302_08381_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kind: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if absent or taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    k = t.get("kernels", {}).get(kind)
    return None if k is None else float(k["hbm_bytes_per_launch"])


# The rocprofv3 runs whose output --summarize reads ({out}: output folder,
# {repo}: this repository).  Run from /tmp with TMPDIR=/tmp.  Counters are
# collected in runs of their own, one counter per run.
PROFILE_COMMANDS = {
    "trace": "rocprofv3 --kernel-trace --stats --output-format csv -d {out}/prof_trace -o run -- "
             "python3 {repo}/bench.py --profile --steps 20 --warmup 3",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}/pmc_fetch -o run -- "
             "python3 {repo}/bench.py --profile --steps 3 --warmup 1",
    "write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}/pmc_write -o run -- "
             "python3 {repo}/bench.py --profile --steps 3 --warmup 1",
}
KERNEL_ROLES = {"forward": "k_fwd4<", "backward": "k_bwd<"}
PROFILE_STEPS = 20  # the --steps of the kernel-trace command above
REFERENCE_COPY = "copyBuffer"  # torch's device-to-device copy of the profile run
REFERENCE_COPY_BYTES = 1 << 30


def _counter_per_dispatch(path: str) -> dict:
    """{kernel name: [counter value per dispatch]} from a rocprofv3 counter CSV."""
    import csv
    per = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            key = (r["Dispatch_Id"], r["Kernel_Name"])
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (_, name), v in per.items():
        out.setdefault(name, []).append(v)
    return out


def summarize(outdir: str) -> None:
    """Write profiles/kernels_l8_f32.md (kernel trace statistics) and
    profiles/traffic_l8_f32.{json,md} (HBM bytes per launch from FETCH_SIZE and
    WRITE_SIZE, each scaled by what the counter reads for the profile run's
    1 GiB reference copy)."""
    import csv
    prof = os.path.join(ROOT, "profiles")
    os.makedirs(prof, exist_ok=True)
    K = (L_MAX + 1) ** 2
    alg = N_POINTS * 4 * (3 + 4 * K)
    cmds = {k: v.format(out="/root/repo/gpurun_out", repo="/root/repo") for k, v in PROFILE_COMMANDS.items()}

    with open(os.path.join(outdir, "prof_trace", "run_kernel_stats.csv")) as f:
        stats = list(csv.DictReader(f))
    lines = ["# Kernel trace: forward (Y+dY) and backward, l_max = 8, float32, N = 1,000,000", "",
             "Command (from /tmp, TMPDIR=/tmp):", "", "    " + cmds["trace"], "",
            f"Kernel sources hash: {kernel_hash()}", "",
             "| kernel | calls | mean us | min us | max us | share % | algorithmic GB/s at mean |",
             "|---|---|---|---|---|---|---|"]
    for r in stats:
        name = r["Name"]
        mean = float(r["AverageNs"]) * 1e-9
        gbs = ""
        if any(tag in name for tag in KERNEL_ROLES.values()):
            gbs = f"{alg / mean / 1e9:.0f}"
        lines.append(f"| `{name}` | {r['Calls']} | {mean * 1e6:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} | {gbs} |")
    lines += ["", f"Algorithmic bytes per launch of either kernel: N * 4 * (3 + 4K) = {alg} (K = {K})."]
    # the timed region only: the last PROFILE_STEPS launches of each kernel
    # (the statistics above include the warm-up launches)
    with open(os.path.join(outdir, "prof_trace", "run_kernel_trace.csv")) as f:
        trace = list(csv.DictReader(f))
    lines += ["", f"Timed region (the last {PROFILE_STEPS} launches of each kernel, as bench.py times them):", "",
              "| kernel | launches | mean us | algorithmic GB/s |", "|---|---|---|---|"]
    for role, tag in KERNEL_ROLES.items():
        ds = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in trace if tag in r["Kernel_Name"])
        ds = ds[-PROFILE_STEPS:]
        if ds:
            m = sum(e - b for b, e in ds) / len(ds) * 1e-9
            lines.append(f"| {role} | {len(ds)} | {m * 1e6:.1f} | {alg / m / 1e9:.0f} |")
    with open(os.path.join(prof, "kernels_l8_f32.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    fetch = _counter_per_dispatch(os.path.join(outdir, "pmc_fetch", "run_counter_collection.csv"))
    write = _counter_per_dispatch(os.path.join(outdir, "pmc_write", "run_counter_collection.csv"))

    def mean_of(tbl, tag):
        vals = [v for name, vs in tbl.items() if tag in name for v in vs]
        return sum(vals) / len(vals) if vals else None

    fscale = REFERENCE_COPY_BYTES / (mean_of(fetch, REFERENCE_COPY) * 1024)
    wscale = REFERENCE_COPY_BYTES / (mean_of(write, REFERENCE_COPY) * 1024)
    t = {"kernel_hash": kernel_hash(), "commands": {"fetch": cmds["fetch"], "write": cmds["write"]},
         "reference_copy_bytes": REFERENCE_COPY_BYTES,
         "scale": {"FETCH_SIZE": fscale, "WRITE_SIZE": wscale}, "kernels": {}}
    md = ["# HBM traffic per launch: forward (Y+dY) and backward, l_max = 8, float32, N = 1,000,000", "",
          "Commands (from /tmp, TMPDIR=/tmp):", "", "    " + cmds["fetch"], "    " + cmds["write"], "",
          f"Kernel sources hash: {kernel_hash()}", "",
          f"Scale factors: bytes = counter KiB * 1024 * factor, with the factor set so that the "
          f"1 GiB reference copy reads and writes 1 GiB: FETCH_SIZE x{fscale:.3f}, WRITE_SIZE x{wscale:.3f}.", "",
          "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) | algorithmic bytes | ratio |",
          "|---|---|---|---|---|---|"]
    for role, tag in KERNEL_ROLES.items():
        fk, wk = mean_of(fetch, tag), mean_of(write, tag)
        if fk is None or wk is None:
            continue
        hbm = (fk * fscale + wk * wscale) * 1024
        t["kernels"][role] = {"fetch_kib": fk, "write_kib": wk, "hbm_bytes_per_launch": hbm,
                              "algorithmic_bytes": alg}
        md.append(f"| {role} | {fk:.0f} | {wk:.0f} | {hbm:.4g} | {alg:.4g} | {hbm / alg:.3f} |")
    with open(os.path.join(prof, "traffic_l8_f32.json"), "w") as f:
        json.dump(t, f, indent=1)
    with open(os.path.join(prof, "traffic_l8_f32.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(lines + [""] + md))


# ------------------------------------------------------------ host oracle
def host_cores() -> int:
    """Worker processes for the oracle: the CPUs this process may run on,
    at most 16 (one GPU's share of a host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_fwd_bwd(args):
    """One chunk of the headline step on the host: the oracle's harmonics and
    gradients, then its backward contraction (a pool worker)."""
    import oracle
    pts, gY = args
    _, G = oracle.real_sph(pts, L_MAX, NORMALIZE)
    oracle.backward(G, gY)
    return pts.shape[0]


def _per_l(gpu, ref, pts, l_max, normalize, kind):
    import oracle
    mx, rms = oracle.per_l_errors(gpu, ref, pts, l_max, normalize, kind)
    return {"max": [float(v) for v in mx], "rms": [float(v) for v in rms]}


def _contraction_err(gx, ref, gY, pts, l_max, normalize):
    """max and RMS of |grad_xyz - ref| / sum_k |gY_k| g_l(k)."""
    import numpy as np

    import oracle
    _, g, _ = oracle.component_scales(pts, l_max, normalize)
    e = np.abs(np.asarray(gx, float) - np.asarray(ref, float)) / (np.abs(gY) * g).sum(1)[:, None]
    return {"max": float(e.max()), "rms": float(np.sqrt((e ** 2).mean()))}


def cpu_baseline(pool, gpu_rows, gpu_rows_f64, gpu_c1, n_single: int = 200_000, chunk: int = 20_000):
    """The oracle (numpy longdouble recurrence tier) on the host:

    * all cores: the whole headline workload (1e6 points, forward with
      gradients and the backward contraction) over the worker pool;
    * one thread: its first n_single points, for comparison;
    * the CPU-sized workload (N = 1000, float64, l_max = 4, both kinds) in
      full, whose results also check the GPU's.

    The oracle's results for the first chunk (20 000 rows) check the GPU's
    rows at float32 and float64: per-l max and RMS of the scaled errors of Y
    and dY, and of grad_xyz.  gpu_rows(n) / gpu_rows_f64(n) return the GPU's
    (Y, dY, grad_xyz) for the first n rows as host arrays; gpu_c1(normalize)
    the GPU's (Y, dY) of the CPU-sized workload."""
    import numpy as np

    import oracle
    from workloads import SEEDS, standard_normal, standard_normal_points

    K = (L_MAX + 1) ** 2
    pts64 = standard_normal_points(N_POINTS, SEEDS["plain_gpu"])
    gY64 = standard_normal((N_POINTS, K), SEEDS["plain_gpu_grad"])
    pts = pts64.astype(np.float32)
    gY = gY64.astype(np.float32)

    # all cores, the whole workload
    cores = pool._processes
    t0 = time.perf_counter()
    done = sum(pool.imap_unordered(_oracle_fwd_bwd, ((pts[s:s + chunk], gY[s:s + chunk])
                                                     for s in range(0, N_POINTS, chunk))))
    t_all = time.perf_counter() - t0
    assert done == N_POINTS

    # one thread, the first n_single points; the first chunk's results kept
    kept = None
    t0 = time.perf_counter()
    for s in range(0, n_single, chunk):
        Yr, G = oracle.real_sph(pts[s:s + chunk], L_MAX, NORMALIZE)
        gr = oracle.backward(G, gY[s:s + chunk])
        if s == 0:
            kept = (Yr, G, gr)
    t_one = time.perf_counter() - t0

    # the GPU's first chunk against the oracle's, float32 (the oracle sees
    # the same rounded inputs) and float64
    acc = {"rows": f"the first {chunk} rows of the {N_POINTS}-point workload",
           "metric": "per-l max and RMS of |gpu - oracle| / s_l (values) or g_l (gradients), the addition-"
                     "theorem scales; grad_xyz: |gpu - oracle| / sum_k |grad_Y_k| g_l(k)",
           "tolerance": {"f32": 1e-5, "f64": 1e-12}}
    hp = pts[:chunk].astype(np.float64)
    Yg, dYg, gxg = gpu_rows(chunk)
    acc["f32"] = {"Y": _per_l(Yg, kept[0], hp, L_MAX, NORMALIZE, "Y"),
                  "dY": _per_l(dYg, kept[1], hp, L_MAX, NORMALIZE, "dY"),
                  "grad_xyz": _contraction_err(gxg, kept[2], gY[:chunk].astype(np.float64), hp, L_MAX, NORMALIZE)}
    Yr, G = oracle.real_sph(pts64[:chunk], L_MAX, NORMALIZE)
    gr = oracle.backward(G, gY64[:chunk])
    Yg, dYg, gxg = gpu_rows_f64(chunk)
    acc["f64"] = {"Y": _per_l(Yg, Yr, pts64[:chunk], L_MAX, NORMALIZE, "Y"),
                  "dY": _per_l(dYg, G, pts64[:chunk], L_MAX, NORMALIZE, "dY"),
                  "grad_xyz": _contraction_err(gxg, gr, gY64[:chunk], pts64[:chunk], L_MAX, NORMALIZE)}

    # the CPU-sized workload in full: N = 1000, float64, l_max = 4
    p1 = standard_normal_points(1000, SEEDS["plain_cpu"])
    c1 = {}
    for norm in (False, True):
        t0 = time.perf_counter()
        Yr, G = oracle.real_sph(p1, 4, norm)
        dt = time.perf_counter() - t0
        Yg, dYg = gpu_c1(norm)
        c1[f"normalize={int(norm)}"] = {"oracle_s": dt, "oracle_ns_per_point": dt / 1000 * 1e9,
                                        "Y": _per_l(Yg, Yr, p1, 4, norm, "Y"),
                                        "dY": _per_l(dYg, G, p1, 4, norm, "dY")}
    acc["plain_cpu_sized_f64_l4"] = c1

    base = {"value": N_POINTS / t_all, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": f"the whole workload ({N_POINTS} points, Y+dY and backward), numpy longdouble recurrence "
                      f"tier, {t_all:.1f} s wall on {cores} worker processes (one thread each)",
            "host": {"cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(), "workers": cores},
            "one_thread": {"value": n_single / t_one, "unit": "points/s",
                           "sample": f"first {n_single} points, {t_one:.1f} s wall, 1 thread"}}
    return base, acc


def _time(fn, reps: int, warm: int = 3) -> float:
    """Mean seconds per call of fn() on the current stream (HIP events)."""
    import torch
    for _ in range(warm):
        fn()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def _time_graph(fn, reps: int, replays: int = 3) -> float:
    """Mean GPU seconds per call of fn(): reps calls captured into one graph
    and replayed, so the host's per-call work (argument checks, the
    library's launch) does not leave the GPU idle between kernels.  For
    kernels shorter than that host work; fn must not allocate or
    synchronise."""
    import torch
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(replays):
        g.replay()
    e1.record(s)
    torch.cuda.synchronize()
    del g
    return e0.elapsed_time(e1) * 1e-3 / (reps * replays)


def extras(dev):
    """Secondary measurements of the other parts of the path (not the headline)."""
    import numpy as np
    import torch

    import paper_2302_08381_amd as sph
    from workloads import SEEDS, csr_environments, shell_points, standard_normal, standard_normal_points
    out = {}
    # float64, same workload as the headline
    K = (L_MAX + 1) ** 2
    x64 = torch.as_tensor(standard_normal_points(N_POINTS, SEEDS["plain_gpu"]), dtype=torch.float64).to(dev)
    g64 = torch.as_tensor(standard_normal((N_POINTS, K), SEEDS["plain_gpu_grad"]), dtype=torch.float64).to(dev)
    Y = torch.empty((N_POINTS, K), dtype=torch.float64, device=dev)
    dY = torch.empty((N_POINTS, 3, K), dtype=torch.float64, device=dev)
    gx = torch.empty((N_POINTS, 3), dtype=torch.float64, device=dev)
    tf = _time(lambda: sph.sph_compute_with_gradients(x64, L_MAX, NORMALIZE, Y=Y, dY=dY), 20)
    tb = _time(lambda: sph.sph_backward(dY, g64, L_MAX, grad_xyz=gx), 20)
    b = N_POINTS * 8 * (3 + 4 * K)
    out["f64_l8"] = {"forward_s": tf, "backward_s": tb, "points_per_s_fwd_bwd": N_POINTS / (tf + tb),
                     "forward_GB_per_s": b / tf / 1e9, "backward_GB_per_s": b / tb / 1e9}
    del x64, g64, Y, dY, gx
    # values only, float32
    x32 = torch.as_tensor(standard_normal_points(N_POINTS, SEEDS["plain_gpu"]), dtype=torch.float32).to(dev)
    Yv = torch.empty((N_POINTS, K), dtype=torch.float32, device=dev)
    tv = _time(lambda: sph.sph_compute(x32, L_MAX, NORMALIZE, Y=Yv), 30)
    out["values_only_l8_f32"] = {"s": tv, "points_per_s": N_POINTS / tv,
                                 "GB_per_s": N_POINTS * 4 * (3 + K) / tv / 1e9}
    # e3nn's conventions, Y+dY: permuted points, the forward, the in-place conversion
    xp = torch.empty_like(x32)
    Ye = torch.empty((N_POINTS, K), dtype=torch.float32, device=dev)
    dYe = torch.empty((N_POINTS, 3, K), dtype=torch.float32, device=dev)

    def e3nn_call():
        sph.sph_e3nn_coordinates(x32, out=xp)
        sph.sph_compute_with_gradients(xp, L_MAX, NORMALIZE, Y=Ye, dY=dYe)
        sph.sph_e3nn_convert(Ye, dYe, L_MAX, "component")
    te = _time(e3nn_call, 20)
    out["e3nn_component_l8_f32"] = {"s": te, "points_per_s": N_POINTS / te,
                                    "note": "Y+dY in e3nn's conventions; the conversion re-reads and rewrites Y, dY"}
    del x32, Yv, xp, Ye, dYe
    # double backward: 4e6 points in the ball 0.5..5, l_max = 6, float32, normalised
    n3, L3 = 4_000_000, 6
    K3 = (L3 + 1) ** 2
    xb = torch.as_tensor(shell_points(n3, 0.5, 5.0, SEEDS["diff"]), dtype=torch.float32).to(dev)
    gYb = torch.as_tensor(standard_normal((n3, K3), 31), dtype=torch.float32).to(dev)
    vb = torch.as_tensor(standard_normal((n3, 3), 32), dtype=torch.float32).to(dev)
    ggb = torch.empty((n3, K3), dtype=torch.float32, device=dev)
    g2b = torch.empty((n3, 3), dtype=torch.float32, device=dev)
    td = _time(lambda: sph.sph_double_backward(xb, gYb, vb, L3, True, grad_grad_Y=ggb, grad_xyz2=g2b), 10)
    out["double_backward_l6_f32_4M"] = {"s": td, "points_per_s": n3 / td,
                                        "GB_per_s": n3 * 4 * (3 + K3 + 3 + K3 + 3) / td / 1e9}
    # ... and its first backward, from the forward's stored dY
    Y3 = torch.empty((n3, K3), device=dev)
    dY3 = torch.empty((n3, 3, K3), device=dev)
    gx3 = torch.empty((n3, 3), device=dev)
    sph.sph_compute_with_gradients(xb, L3, True, Y=Y3, dY=dY3)
    tb3 = _time(lambda: sph.sph_backward(dY3, gYb, L3, grad_xyz=gx3), 10)
    out["backward_l6_f32_4M"] = {"s": tb3, "points_per_s": n3 / tb3,
                                 "GB_per_s": n3 * 4 * (4 * K3 + 3) / tb3 / 1e9}
    # explicit second derivatives on the same points: Y, dY and d2Y [n,3,3,K]
    # (two launches: the forward, then the second-derivative kernel)
    d2Y3 = torch.empty((n3, 3, 3, K3), device=dev)
    th = _time(lambda: sph.sph_compute_with_hessians(xb, L3, True, Y=Y3, dY=dY3, d2Y=d2Y3), 5)
    out["hessians_l6_f32_4M"] = {"s": th, "points_per_s": n3 / th,
                                 "GB_per_s": n3 * 4 * (3 + 13 * K3) / th / 1e9,
                                 "bytes": "read xyz, write Y, dY and d2Y: N*4*(3 + 13K)"}
    del xb, gYb, vb, Y3, dY3, gx3, d2Y3, ggb, g2b
    # plain method, CPU-sized: N = 1000, float64, l_max = 4 (launch-bound)
    x1 = torch.as_tensor(standard_normal_points(1000, SEEDS["plain_cpu"]), dtype=torch.float64).to(dev)
    t1 = _time(lambda: sph.sph_compute_with_gradients(x1, 4, True), 50)
    Y1 = torch.empty((1000, 25), dtype=torch.float64, device=dev)
    dY1 = torch.empty((1000, 3, 25), dtype=torch.float64, device=dev)
    t1g = _time_graph(lambda: sph.sph_compute_with_gradients(x1, 4, True, Y=Y1, dY=dY1), 50)
    out["plain_l4_f64_1000"] = {"forward_s": t1, "points_per_s": 1000 / t1,
                                "gpu_s_graph_replay": t1g, "note": "forward_s includes the host's work per call"}
    # precision workload: l_max = 32, N = 200 000 (unit sphere, near the poles,
    # radii 1e-6..1e3), float32 and float64; errors are checked by the tests
    from workloads import precision_stress_points
    pts5, _ = precision_stress_points(200_000, SEEDS["precision"])
    n5, K5 = pts5.shape[0], 33 ** 2
    p5 = {}
    for dt5, w5, name in ((torch.float32, 4, "f32"), (torch.float64, 8, "f64")):
        x5 = torch.as_tensor(pts5, dtype=dt5).to(dev)
        Y5 = torch.empty((n5, K5), dtype=dt5, device=dev)
        dY5 = torch.empty((n5, 3, K5), dtype=dt5, device=dev)
        t5 = _time(lambda: sph.sph_compute_with_gradients(x5, 32, True, Y=Y5, dY=dY5), 5)
        p5[name] = {"forward_s": t5, "points_per_s": n5 / t5, "GB_per_s": n5 * w5 * (3 + 4 * K5) / t5 / 1e9}
        del x5, Y5, dY5
    out["precision_l32_200k"] = p5
    # batched: 20 000 environments, fused forward + backward with dY, per l_max
    pts, offs = csr_environments(20_000, 8, 128, 0.5, 5.0, SEEDS["batched"])
    nb = int(offs[-1])
    xc = torch.as_tensor(pts, dtype=torch.float32).to(dev)
    oc = torch.as_tensor(offs, device=dev)
    bat = {}
    for Lb in (3, 6, 8, 12):
        Kb = (Lb + 1) ** 2
        gYc = torch.as_tensor(standard_normal((nb, Kb), 1000 + Lb), dtype=torch.float32).to(dev)
        o = {"Y": torch.empty((nb, Kb), device=dev), "dY": torch.empty((nb, 3, Kb), device=dev),
             "grad_xyz": torch.empty((nb, 3), device=dev)}
        tbat = _time(lambda: sph.sph_batched_compute(xc, oc, Lb, True, store_dY=True, grad_Y=gYc, out=o,
                                                          check=False), 20)
        Yp = torch.empty((nb, Kb), device=dev)
        dYp = torch.empty((nb, 3, Kb), device=dev)
        gxp = torch.empty((nb, 3), device=dev)

        def plain():
            sph.sph_compute_with_gradients(xc, Lb, True, Y=Yp, dY=dYp)
            sph.sph_backward(dYp, gYc, Lb, grad_xyz=gxp)
        tpl = _time(plain, 20)
        bat[str(Lb)] = {"batched_fused_s": tbat, "plain_fwd_bwd_s": tpl, "points": nb,
                        "batched_points_per_s": nb / tbat, "plain_points_per_s": nb / tpl,
                        "config": sph.sph_batched_get_config(Lb, True, torch.float32, True, True)}
    out["batched_20k_envs_f32"] = bat
    # radial expansion of the same environments: c[e,n,lm] = sum_j R_nl(r_j)
    # Y_lm(x_j), 8 radial channels (Gaussian basis, cutoff 5), fused against
    # the harmonics stored by the values-only kernel and contracted by torch
    from workloads import gaussian_radial_basis
    env_of = torch.repeat_interleave(torch.arange(offs.size - 1, device=dev), oc[1:] - oc[:-1])
    exp = {}
    NMX = 8
    for Lb in (3, 6, 8, 12):
        Kb = (Lb + 1) ** 2
        Rc = torch.as_tensor(gaussian_radial_basis(pts, Lb, NMX, 5.0), dtype=torch.float32).to(dev)
        cc = torch.empty((offs.size - 1, NMX, Kb), device=dev)
        tex = _time(lambda: sph.sph_radial_expansion(xc, oc, Rc, Lb, True, out=cc, check=False), 20)
        lk = torch.tensor([l for l in range(Lb + 1) for _ in range(2 * l + 1)], device=dev)
        Yu = torch.empty((nb, Kb), device=dev)
        acc = torch.empty((offs.size - 1, Kb, NMX), device=dev)

        def unfused():
            sph.sph_compute(xc, Lb, True, Y=Yu)
            acc.zero_()
            acc.index_add_(0, env_of, Rc[:, lk, :] * Yu[:, :, None])
        tun = _time(unfused, 5)
        byts = nb * 4 * (3 + (Lb + 1) * NMX) + (offs.size - 1) * (8 + 4 * NMX * Kb)
        Gc = torch.as_tensor(standard_normal((offs.size - 1, NMX, Kb), 700 + Lb), dtype=torch.float32).to(dev)
        tbw = _time(lambda: sph.sph_radial_expansion_backward(xc, oc, Rc, Gc, Lb, True, check=False), 10)
        exp[str(Lb)] = {"fused_s": tex, "unfused_s": tun, "backward_s": tbw, "points": nb, "n_max": NMX,
                        "fused_points_per_s": nb / tex, "fused_GB_per_s": byts / tex / 1e9,
                        "backward_points_per_s": nb / tbw}
    out["radial_expansion_20k_envs_f32"] = exp
    # compile-time (unrolled, literal coefficients) against run-time-degree
    # kernels at low l_max, and the one-lane kernel: the batched path on the
    # same environments, Y and dY stored, one tile per block, each variant
    # pinned.  GPU time from graph replays: at l_max <= 2 a kernel is shorter
    # than the host's work per call
    spec = {}
    for Ls in range(0, 7):
        Ks = (Ls + 1) ** 2
        o = {"Y": torch.empty((nb, Ks), device=dev), "dY": torch.empty((nb, 3, Ks), device=dev)}
        row = {}
        # tile16: the compile-time quad-lane kernel on a 16-point tile; one_lane
        # (l_max <= 3): one lane per point
        for variant in ("default", "tile16", "runtime_degree") + (("one_lane",) if Ls <= 3 else ()):
            sph.sph_batched_set_config(Ls, True, torch.float32, True, False, variant, 0)
            row[variant + "_s"] = _time_graph(lambda: sph.sph_batched_compute(xc, oc, Ls, True, store_dY=True,
                                                                                    out=o, check=False), 20)
        row["GB_per_s_default"] = nb * 4 * (3 + 4 * Ks) / row["default_s"] / 1e9
        sph.sph_batched_set_config(Ls, True, torch.float32, True, False, "default", 0)
        if Ls <= 3:  # with the fused backward as well
            gYs = torch.as_tensor(standard_normal((nb, Ks), 1100 + Ls), dtype=torch.float32).to(dev)
            o["grad_xyz"] = torch.empty((nb, 3), device=dev)
            for variant in ("default", "tile16", "one_lane"):
                sph.sph_batched_set_config(Ls, True, torch.float32, True, True, variant, 0)
                row[variant + "_with_backward_s"] = _time_graph(
                    lambda: sph.sph_batched_compute(xc, oc, Ls, True, store_dY=True, grad_Y=gYs, out=o,
                                                    check=False), 20)
            sph.sph_batched_set_config(Ls, True, torch.float32, True, True, "default", 0)
        spec[str(Ls)] = row
    out["low_lmax_variants_f32"] = spec
    return out


# ------------------------------------------------------------ kernel suite profile
# One program that launches every kernel of the path on its workload, for
# rocprofv3 runs: a kernel trace, the two HBM byte counters, and the SQ
# counters that show what bounds each kernel (VALU activity, occupancy, LDS
# bank conflicts).  Counters are collected in runs of their own.
SUITE_COMMANDS = {
    "trace": "rocprofv3 --kernel-trace --stats --output-format csv -d {out}/suite_trace -o run -- "
             "python3 {repo}/bench.py --profile-suite --steps 5 --warmup 2",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}/suite_fetch -o run -- "
             "python3 {repo}/bench.py --profile-suite --steps 2 --warmup 1",
    "write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}/suite_write -o run -- "
             "python3 {repo}/bench.py --profile-suite --steps 2 --warmup 1",
    "sq": "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAVE_CYCLES SQ_LDS_BANK_CONFLICT "
          "SQ_INSTS_LDS SQ_BUSY_CYCLES GRBM_GUI_ACTIVE --output-format csv -d {out}/suite_sq -o run -- "
          "python3 {repo}/bench.py --profile-suite --steps 2 --warmup 1",
    "tcc": "rocprofv3 --pmc TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum TCC_EA0_WRREQ_LEVEL_sum GRBM_GUI_ACTIVE "
           "--output-format csv -d {out}/suite_tcc -o run -- "
           "python3 {repo}/bench.py --profile-suite --steps 2 --warmup 1",
    "wait": "rocprofv3 --pmc SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_LDS_IDX_ACTIVE SQ_WAVE_CYCLES GRBM_GUI_ACTIVE "
            "--output-format csv -d {out}/suite_wait -o run -- "
            "python3 {repo}/bench.py --profile-suite --steps 2 --warmup 1",
}
SUITE_STEPS = 5  # the --steps of the trace command


def _suite_workloads():
    """(role, kernel-name tag, algorithmic bytes per launch, workload) of the
    suite's kernels."""
    from workloads import SEEDS, csr_environments
    K8, K6 = 81, 49
    n3 = 4_000_000
    _, offs = csr_environments(20_000, 8, 128, 0.5, 5.0, SEEDS["batched"])
    ne, npt = offs.size - 1, int(offs[-1])
    L, NM = EXPANSION_L, EXPANSION_CHANNELS
    return [
        ("forward", "k_fwd4<float, 8, 8,", N_POINTS * 4 * (3 + 4 * K8),
         "Y+dY, N = 1e6, l_max = 8, float32, normalised"),
        ("backward", "k_bwd<float", N_POINTS * 4 * (4 * K8 + 3), "grad_xyz from dY, same workload"),
        ("double backward", "k_dbwd<float", n3 * 4 * ((3 + K6 + 3) + (K6 + 3)),
         "ggY and grad_xyz2, N = 4e6 in the ball 0.5..5, l_max = 6, float32, normalised"),
        ("hessian: Y+dY", "k_fwd4<float, 6, 6,", n3 * 4 * (3 + 4 * K6),
         "the forward half of sph_compute_with_hessians, same 4e6 points, l_max = 6"),
        ("hessian: d2Y", "k_hess<float", n3 * 4 * (3 + 9 * K6), "d2Y [n,3,3,K], same points"),
        ("radial expansion", "k_expand<float", npt * 4 * (3 + (L + 1) * NM) + ne * (8 + 4 * NM * K8),
         f"{ne} environments ({npt} points), l_max = 8, 8 channels, float32"),
        ("radial expansion backward", "k_expand_bwd<float",
         npt * 4 * (3 + 2 * (L + 1) * NM + 3) + ne * (8 + 4 * NM * K8), "grad_xyz and grad_R, same environments"),
    ]


def suite_hash() -> str:
    """Hash of every kernel source and the C ABI (the suite covers all of them)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2302_08381_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


CU_NUM, XCD_NUM, CLOCK_GHZ = 256, 8, 2.4


def _per_dispatch(path: str) -> dict:
    """{dispatch id: (kernel name, {counter: value}, row)} from a rocprofv3
    counter CSV (one row per dispatch and counter)."""
    import csv
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            d = out.setdefault(int(r["Dispatch_Id"]), (r["Kernel_Name"], {}, r))
            d[1][r["Counter_Name"]] = d[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def summarize_suite(outdir: str) -> None:
    """profiles/kernel_suite.md: per kernel of the path, its mean duration
    (kernel trace), algorithmic and HBM bytes (FETCH_SIZE / WRITE_SIZE scaled
    by the 1 GiB reference copy), and what the SQ counters say bounds it:
    VALU instructions per wave and the share of the CUs' VALU issue slots
    they fill, mean resident waves per CU, LDS instructions and bank-conflict
    cycles.  GRBM_GUI_ACTIVE is summed over the 8 XCDs, so the kernel's
    cycles are GRBM_GUI_ACTIVE / 8; SQ_WAVE_CYCLES counts quad-cycles."""
    import csv
    cmds = {k: v.format(out="/root/repo/gpurun_out", repo="/root/repo") for k, v in SUITE_COMMANDS.items()}
    with open(os.path.join(outdir, "suite_trace", "run_kernel_trace.csv")) as f:
        trace = list(csv.DictReader(f))
    fetch = _per_dispatch(os.path.join(outdir, "suite_fetch", "run_counter_collection.csv"))
    write = _per_dispatch(os.path.join(outdir, "suite_write", "run_counter_collection.csv"))
    sq = _per_dispatch(os.path.join(outdir, "suite_sq", "run_counter_collection.csv"))
    tcc_path = os.path.join(outdir, "suite_tcc", "run_counter_collection.csv")
    tcc = _per_dispatch(tcc_path) if os.path.exists(tcc_path) else {}
    wait_path = os.path.join(outdir, "suite_wait", "run_counter_collection.csv")
    wait = _per_dispatch(wait_path) if os.path.exists(wait_path) else {}

    def mean_counter(tbl, tag, name):
        v = [c[name] for k, c, _ in tbl.values() if tag in k and name in c]
        return sum(v) / len(v) if v else None

    fs = REFERENCE_COPY_BYTES / (mean_counter(fetch, REFERENCE_COPY, "FETCH_SIZE") * 1024)
    ws = REFERENCE_COPY_BYTES / (mean_counter(write, REFERENCE_COPY, "WRITE_SIZE") * 1024)
    lines = ["# Kernel suite: time, bytes and SQ counters of every kernel of the path", "",
             "Commands (from /tmp, TMPDIR=/tmp), each in a run of its own:", ""]
    lines += ["    " + cmds[k] for k in ("trace", "fetch", "write", "sq") + (("tcc",) if tcc else ())
              + (("wait",) if wait else ())]
    # the hash the profiled runs printed (the sources they ran), not the tree's
    run_hashes = set()
    for k in ("trace", "fetch", "write", "sq", "tcc", "wait"):
        log = os.path.join(outdir, f"suite_{k}.log")
        if os.path.exists(log):
            with open(log) as f:
                for line in f:
                    if line.startswith('{"profile_run": "suite"'):
                        run_hashes.add(json.loads(line)["kernel_sources"])
    if len(run_hashes) != 1:
        raise SystemExit(f"suite runs printed kernel source hashes {sorted(run_hashes)}: expected exactly one")
    run_hash = run_hashes.pop()
    note = "" if run_hash == suite_hash() else " (the sources have changed since: the figures are of the earlier ones)"
    lines += ["", f"Kernel sources hash: {run_hash}{note}", "",
              f"HBM bytes = counter KiB * 1024 * factor, the factor set so that the 1 GiB reference copy reads and "
              f"writes 1 GiB: FETCH_SIZE x{fs:.3f}, WRITE_SIZE x{ws:.3f}.  Cycles = GRBM_GUI_ACTIVE / {XCD_NUM} "
              f"(the counter is summed over the XCDs).  VALU slots: one wave64 VALU instruction per SIMD per 4 "
              f"cycles, i.e. one per CU per cycle over {CU_NUM} CUs.  Waves per CU: 4 * SQ_WAVE_CYCLES "
              f"(quad-cycles) / ({CU_NUM} * cycles), of at most 32.  LDS conflict: SQ_LDS_BANK_CONFLICT cycles "
              f"per CU-cycle.", "",
              "| kernel | workload | mean us | alg. bytes | alg. GB/s | HBM bytes / alg. | VALU instr / wave | "
              "VALU slots used | waves / CU | LDS instr / wave | LDS conflict | VGPR, AGPR | block x grid |",
              "|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for role, tag, alg, what in _suite_workloads():
        ds = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r) for r in trace if tag in r["Kernel_Name"])
        ds = ds[-SUITE_STEPS:]
        if not ds:
            continue
        mean = sum(e - b for b, e, _ in ds) / len(ds) * 1e-9
        row = ds[-1][2]
        fk, wk = mean_counter(fetch, tag, "FETCH_SIZE"), mean_counter(write, tag, "WRITE_SIZE")
        hbm = (fk * fs + wk * ws) * 1024 if fk is not None and wk is not None else None
        c = {n: mean_counter(sq, tag, n) for n in ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_WAVE_CYCLES", "SQ_INSTS_LDS",
                                                  "SQ_LDS_BANK_CONFLICT", "GRBM_GUI_ACTIVE")}
        cyc = c["GRBM_GUI_ACTIVE"] / XCD_NUM
        lines.append(
            f"| {role} (`{row['Kernel_Name'].split('(')[0].replace('void sph::', '')}`) | {what} | {mean * 1e6:.1f} | "
            f"{alg:.4g} | {alg / mean / 1e9:.0f} | {hbm / alg:.3f} | {c['SQ_INSTS_VALU'] / c['SQ_WAVES']:.0f} | "
            f"{100 * c['SQ_INSTS_VALU'] / (CU_NUM * cyc):.0f} % | {4 * c['SQ_WAVE_CYCLES'] / (CU_NUM * cyc):.1f} | "
            f"{c['SQ_INSTS_LDS'] / c['SQ_WAVES']:.0f} | {100 * c['SQ_LDS_BANK_CONFLICT'] / (CU_NUM * cyc):.1f} % | "
            f"{row['VGPR_Count']}, {row['Accum_VGPR_Count']} | {row['Workgroup_Size_X']} x "
            f"{int(row['Grid_Size_X']) // max(1, int(row['Workgroup_Size_X']))} |")
    lines += ["", "Means over the last %d launches of each kernel in the trace run; counters from the last "
              "launches of the counter runs (counter runs serialise the launches)." % SUITE_STEPS]
    if tcc:
        # write path to HBM: requests from L2 to the memory fabric and how many
        # are in flight on average, for the store-bound kernels and torch's
        # fill of 1 GiB (the write-only reference of the same run)
        lines += ["", "Writes from L2 to memory (TCC_EA0_WRREQ: requests, of them 64-byte; WRREQ_LEVEL: "
                  "requests in flight summed over cycles, so LEVEL / cycles is the mean number in flight):", "",
                  "| kernel | mean us | write requests | 64-byte share | mean in flight | written GB/s |",
                  "|---|---|---|---|---|---|"]
        refs = [(r, t, a) for r, t, a, _ in _suite_workloads() if r in ("forward", "hessian: d2Y",
                                                                        "hessian: Y+dY")]
        refs.append(("torch fill, 1 GiB", "FillFunctor", float(REFERENCE_COPY_BYTES)))
        for role, tag, alg in refs:
            ds = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in trace if tag in r["Kernel_Name"])
            ds = ds[-SUITE_STEPS:]
            req = mean_counter(tcc, tag, "TCC_EA0_WRREQ_sum")
            if not ds or req is None:
                continue
            mean = sum(e - b for b, e in ds) / len(ds) * 1e-9
            r64 = mean_counter(tcc, tag, "TCC_EA0_WRREQ_64B_sum")
            lvl = mean_counter(tcc, tag, "TCC_EA0_WRREQ_LEVEL_sum")
            cyc = mean_counter(tcc, tag, "GRBM_GUI_ACTIVE") / XCD_NUM
            wk = mean_counter(write, tag, "WRITE_SIZE")
            wgbs = f"{wk * ws * 1024 / mean / 1e9:.0f}" if wk is not None else ""
            lines.append(f"| {role} | {mean * 1e6:.1f} | {req:.4g} | {r64 / req:.3f} | {lvl / cyc:.0f} | {wgbs} |")
    if wait:
        # where the waves' time goes: waiting on results of memory, LDS or
        # scalar loads (s_waitcnt), waiting to issue, and how busy the LDS is
        lines += ["", "Wave time (SQ_WAIT_ANY: wave quad-cycles waiting on outstanding memory, LDS or scalar "
                  "results; SQ_WAIT_INST_ANY: waiting to issue; both over SQ_WAVE_CYCLES) and LDS busy "
                  "(SQ_LDS_IDX_ACTIVE cycles per CU-cycle):", "",
                  "| kernel | waiting on results | waiting to issue | LDS busy |", "|---|---|---|---|"]
        for role, tag, _, _ in _suite_workloads():
            w = {n: mean_counter(wait, tag, n) for n in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_LDS_IDX_ACTIVE",
                                                        "SQ_WAVE_CYCLES", "GRBM_GUI_ACTIVE")}
            if any(v is None for v in w.values()):
                continue
            cyc = w["GRBM_GUI_ACTIVE"] / XCD_NUM
            lines.append(f"| {role} | {100 * w['SQ_WAIT_ANY'] / w['SQ_WAVE_CYCLES']:.0f} % | "
                         f"{100 * w['SQ_WAIT_INST_ANY'] / w['SQ_WAVE_CYCLES']:.0f} % | "
                         f"{100 * w['SQ_LDS_IDX_ACTIVE'] / (CU_NUM * cyc):.0f} % |")
    with open(os.path.join(ROOT, "profiles", "kernel_suite.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def profile_suite(dev, steps: int, warmup: int) -> None:
    import torch

    import paper_2302_08381_amd as sph
    from workloads import SEEDS, shell_points, standard_normal, standard_normal_points
    K = 81
    x = torch.as_tensor(standard_normal_points(N_POINTS, SEEDS["plain_gpu"]), dtype=torch.float32).to(dev)
    gY = torch.as_tensor(standard_normal((N_POINTS, K), SEEDS["plain_gpu_grad"]), dtype=torch.float32).to(dev)
    Y = torch.empty((N_POINTS, K), device=dev)
    dY = torch.empty((N_POINTS, 3, K), device=dev)
    gx = torch.empty((N_POINTS, 3), device=dev)
    n3, L3, K3 = 4_000_000, 6, 49
    xb = torch.as_tensor(shell_points(n3, 0.5, 5.0, SEEDS["diff"]), dtype=torch.float32).to(dev)
    gYb = torch.as_tensor(standard_normal((n3, K3), 31), dtype=torch.float32).to(dev)
    vb = torch.as_tensor(standard_normal((n3, 3), 32), dtype=torch.float32).to(dev)
    Y3 = torch.empty((n3, K3), device=dev)
    dY3 = torch.empty((n3, 3, K3), device=dev)
    d2Y3 = torch.empty((n3, 3, 3, K3), device=dev)
    xe, oe, Re, Ge, ne_pts, ne = _expansion_inputs(dev)
    ce = torch.empty((ne, EXPANSION_CHANNELS, K), device=dev)

    def step():
        sph.sph_compute_with_gradients(x, L_MAX, True, Y=Y, dY=dY)
        sph.sph_backward(dY, gY, L_MAX, grad_xyz=gx)
        sph.sph_double_backward(xb, gYb, vb, L3, True)
        sph.sph_compute_with_hessians(xb, L3, True, Y=Y3, dY=dY3, d2Y=d2Y3)
        sph.sph_radial_expansion(xe, oe, Re, EXPANSION_L, True, out=ce, check=False)
        sph.sph_radial_expansion_backward(xe, oe, Re, Ge, EXPANSION_L, True, check=False)
    for _ in range(warmup + steps):
        step()
    # reference copy of known size for scaling the HBM byte counters
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": "suite", "steps": steps, "kernel_sources": suite_hash()}), flush=True)


# ------------------------------------------------------------ precision report
PRECISION_COMMAND = "python3 bench.py --precision-report gpurun_out/precision_l32.md"
PRECISION_CLASSES = ("unit sphere", "near the poles", "radii 1e-6..1e3")


def _precision_chunk(args):
    """Per class: (points, Y max[l], Y rms[l], dY max[l], dY rms[l]) of one
    chunk of GPU rows against the oracle (a pool worker)."""
    import oracle
    pts, Yg, dYg, cls = args
    Yr, G = oracle.real_sph(pts, 32, True)
    out = {}
    for c in range(len(PRECISION_CLASSES)):
        m = cls == c
        if m.any():
            my, ry = oracle.per_l_errors(Yg, Yr, pts, 32, True, "Y", mask=m)
            md, rd = oracle.per_l_errors(dYg, G, pts, 32, True, "dY", mask=m)
            out[c] = (int(m.sum()), my, ry, md, rd)
    return out


def precision_report(dev, pool, path: str, per_class: int = 20_000, chunk: int = 1000) -> None:
    """Per-l max and RMS of the scaled errors of Y and dY against the oracle
    on the l_max = 32 stress workload (N = 200 000, normalised), float32 and
    float64, per sub-population: the GPU computes all 200 000 points in one
    call; per_class points of each class are checked."""
    import numpy as np
    import torch

    import paper_2302_08381_amd as sph
    from workloads import SEEDS, precision_stress_points

    L = 32
    pts, cls = precision_stress_points(200_000, SEEDS["precision"])
    rng = np.random.default_rng(55)
    idx = np.sort(np.concatenate([rng.choice(np.flatnonzero(cls == c), per_class, replace=False)
                                  for c in range(len(PRECISION_CLASSES))]))
    ii = torch.as_tensor(idx, device=dev)
    head = ["# Per-l accuracy at l_max = 32: the precision stress workload", "",
            "Command (repository root, one GPU):", "", "    " + PRECISION_COMMAND, "",
            f"Kernel sources hash: {kernel_hash()}", "",
            f"Workload: N = 200 000 points, normalised harmonics, l_max = 32 (K = 1089): 100 000 on the unit "
            f"sphere, 50 000 with |x|, |y| ~ 10^U(-12,-3) and z = +-1, 50 000 isotropic with r ~ 10^U(-6,3) "
            f"(seed {SEEDS['precision']}).  The GPU computes Y and dY for all 200 000 points in one call; "
            f"{per_class} points of each class (seeded choice) are compared with the oracle (numpy longdouble "
            f"recurrence tier) on the inputs the kernel saw (float32-rounded for the float32 run).", "",
            "Error: |gpu - oracle| / s_l for values and / g_l for gradients, with the addition-theorem scales "
            "s_l = sqrt((2l+1)/4pi) and g_l = sqrt(l(l+1)(2l+1)/4pi)/r; max and RMS over the class's points, "
            "the 2l+1 orders and (for dY) the three axes.  Tolerances: float32 1e-5, float64 1e-12.", ""]
    summary, tables = [], []
    for dt, name in ((torch.float32, "float32"), (torch.float64, "float64")):
        x = torch.as_tensor(pts, dtype=dt).to(dev)
        Y, dY = sph.sph_compute_with_gradients(x, L, True)
        ph = x[ii].double().cpu().numpy()
        Yh = Y[ii].double().cpu().numpy()
        dYh = dY[ii].double().cpu().numpy()
        del x, Y, dY
        torch.cuda.empty_cache()
        ch = cls[idx]
        nc = len(PRECISION_CLASSES)
        ymax = np.zeros((nc, L + 1))
        dmax = np.zeros((nc, L + 1))
        ysq = np.zeros((nc, L + 1))
        dsq = np.zeros((nc, L + 1))
        npts = np.zeros(nc, np.int64)
        ls = np.arange(L + 1)
        jobs = ((ph[s:s + chunk], Yh[s:s + chunk], dYh[s:s + chunk], ch[s:s + chunk])
                for s in range(0, idx.size, chunk))
        for res in pool.imap_unordered(_precision_chunk, jobs):
            for c, (n, my, ry, md, rd) in res.items():
                npts[c] += n
                ymax[c] = np.maximum(ymax[c], my)
                dmax[c] = np.maximum(dmax[c], md)
                ysq[c] += ry ** 2 * n * (2 * ls + 1)
                dsq[c] += rd ** 2 * n * 3 * (2 * ls + 1)
        for c, cname in enumerate(PRECISION_CLASSES):
            yr = np.sqrt(ysq[c] / (npts[c] * (2 * ls + 1)))
            dr = np.sqrt(dsq[c] / (npts[c] * 3 * (2 * ls + 1)))
            summary.append(f"| {name} | {cname} | {npts[c]} | {ymax[c].max():.2e} | {dmax[c].max():.2e} | "
                           f"{yr.max():.2e} | {dr.max():.2e} |")
            tables += [f"## {name}, {cname} ({npts[c]} points)", "",
                       "| l | Y max | Y RMS | dY max | dY RMS |", "|---|---|---|---|---|"]
            tables += [f"| {l} | {ymax[c, l]:.2e} | {yr[l]:.2e} | {dmax[c, l]:.2e} | {dr[l]:.2e} |"
                       for l in range(L + 1)]
            tables.append("")
        print(f"precision report: {name} done", flush=True)
    table_head = ["| dtype | class | points | Y max | dY max | Y RMS | dY RMS |", "|---|---|---|---|---|---|---|"]
    lines = head + ["Summary (largest over l):", ""] + table_head + summary + [""] + tables
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(table_head + summary), flush=True)


EXPANSION_L, EXPANSION_CHANNELS = 8, 8


def _expansion_inputs(dev):
    import numpy as np
    import torch

    from workloads import SEEDS, csr_environments, gaussian_radial_basis, standard_normal
    pts, offs = csr_environments(20_000, 8, 128, 0.5, 5.0, SEEDS["batched"])
    K = (EXPANSION_L + 1) ** 2
    xyz = torch.as_tensor(pts, dtype=torch.float32).to(dev)
    o = torch.as_tensor(offs, device=dev)
    R = torch.as_tensor(gaussian_radial_basis(pts, EXPANSION_L, EXPANSION_CHANNELS, 5.0), dtype=torch.float32).to(dev)
    G = torch.as_tensor(standard_normal((offs.size - 1, EXPANSION_CHANNELS, K), 700 + EXPANSION_L),
                        dtype=torch.float32).to(dev)
    return xyz, o, R, G, int(offs[-1]), int(np.asarray(offs).size - 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--profile", action="store_true",
                    help="only run warmup + steps (and a 1 GiB reference copy), for rocprofv3")
    ap.add_argument("--summarize", metavar="DIR",
                    help="write the profiles/ summaries from the rocprofv3 output in DIR (no GPU)")
    ap.add_argument("--profile-suite", action="store_true",
                    help="only run warmup + steps of every kernel of the path on its workload (and a 1 GiB "
                         "reference copy), for rocprofv3")
    ap.add_argument("--summarize-suite", metavar="DIR",
                    help="write profiles/kernel_suite.md from the rocprofv3 output folders in DIR (no GPU)")
    ap.add_argument("--precision-report", metavar="PATH",
                    help="write the per-l accuracy tables of the l_max = 32 stress workload (float32 and float64, "
                         "per sub-population) to PATH")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize)
        return
    if args.summarize_suite:
        summarize_suite(args.summarize_suite)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the path has no "
              "cross-GPU step; each GPU would run the same kernels on its own shard of points.",
              file=sys.stderr)
        sys.exit(2)

    # The oracle's worker processes are forked before anything touches the
    # GPU, so they hold no device state.
    pool = None
    if args.precision_report or not (args.no_cpu_baseline or args.profile or args.profile_suite):
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(host_cores())

    import torch

    import paper_2302_08381_amd as sph
    from workloads import SEEDS, standard_normal, standard_normal_points

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.profile_suite:
        profile_suite(dev, args.steps, args.warmup)
        return
    if args.precision_report:
        precision_report(dev, pool, args.precision_report)
        pool.close()
        pool.join()
        return
    K = (L_MAX + 1) ** 2
    xyz = torch.as_tensor(standard_normal_points(N_POINTS, SEEDS["plain_gpu"]), dtype=torch.float32).to(dev)
    gY = torch.as_tensor(standard_normal((N_POINTS, K), SEEDS["plain_gpu_grad"]), dtype=torch.float32).to(dev)
    Y = torch.empty((N_POINTS, K), dtype=torch.float32, device=dev)
    dY = torch.empty((N_POINTS, 3, K), dtype=torch.float32, device=dev)
    gx = torch.empty((N_POINTS, 3), dtype=torch.float32, device=dev)

    def step():
        sph.sph_compute_with_gradients(xyz, L_MAX, NORMALIZE, Y=Y, dY=dY)
        sph.sph_backward(dY, gY, L_MAX, grad_xyz=gx)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    if args.profile:
        for _ in range(args.steps):
            step()
        # reference copy of known size for scaling the HBM byte counters
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "steps": args.steps, "reference_copy_bytes_each_way": a.numel() * 4,
                          "kernel_sources": kernel_hash()}))
        return

    stream = torch.cuda.current_stream(dev)  # the launch stream of both kernels
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record(stream)
        sph.sph_compute_with_gradients(xyz, L_MAX, NORMALIZE, Y=Y, dY=dY)
        ev[s][1].record(stream)
        sph.sph_backward(dY, gY, L_MAX, grad_xyz=gx)
        ev[s][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_fwd = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps * 1e-3
    t_bwd = sum(e[1].elapsed_time(e[2]) for e in ev) / args.steps * 1e-3
    ms_per_step = wall / args.steps * 1e3
    value = N_POINTS * args.steps / wall

    w = 4
    bytes_fwd = N_POINTS * w * (3 + 4 * K)   # read xyz, write Y and dY
    bytes_bwd = N_POINTS * w * (4 * K + 3)   # read dY and grad_Y, write grad_xyz
    per_kernel = {
        "forward_Y_dY": {"kernel": "k_fwd4<float,8,8,true>", "mean_s": t_fwd, "bytes": bytes_fwd,
                         "GB_per_s": bytes_fwd / t_fwd / 1e9, "traffic": load_traffic("forward")},
        "backward": {"kernel": "k_bwd<float>", "mean_s": t_bwd, "bytes": bytes_bwd,
                     "GB_per_s": bytes_bwd / t_bwd / 1e9, "traffic": load_traffic("backward")},
    }
    dom_name = max(per_kernel, key=lambda k: per_kernel[k]["mean_s"])
    dom = per_kernel[dom_name]
    achieved = dom["GB_per_s"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": dom["traffic"], "kernel": dom_name}

    # practical ceilings on this GPU: torch's write-only fill and copy kernels
    # over buffers of the forward's size
    big = torch.empty(bytes_fwd // 4, dtype=torch.float32, device=dev)
    half = torch.empty(bytes_fwd // 8, dtype=torch.float32, device=dev)
    half2 = torch.empty_like(half)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    for _ in range(3):
        big.fill_(1.0)
        half2.copy_(half)
    e0.record(stream)
    for _ in range(10):
        big.fill_(1.0)
    e1.record(stream)
    for _ in range(10):
        half2.copy_(half)
    e2.record(stream)
    torch.cuda.synchronize()
    fill_gbs = bytes_fwd * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    copy_gbs = 2 * half.numel() * 4 * 10 / (e1.elapsed_time(e2) * 1e-3) / 1e9
    del big, half, half2

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain forward Y+dY then backward, N=1,000,000 points, xyz iid N(0,1) "
                               "(seed 2), grad_Y iid N(0,1) (seed 12), l_max=8, normalize=true, float32",
                   "n_points": N_POINTS, "l_max": L_MAX, "normalize": NORMALIZE},
        "GB_per_s_fwd_bwd": round((bytes_fwd + bytes_bwd) * args.steps / wall / 1e9, 1),
        "roofline": roofline,
        "kernels": {k: {kk: (round(vv, 7) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in per_kernel.items()},
        "ceilings_GB_per_s": {"torch_fill_write_only": round(fill_gbs, 1), "torch_copy": round(copy_gbs, 1)},
        "kernel_sources": kernel_hash(),
    }
    if not args.no_extras:
        out["extra"] = extras(dev)
    if pool is not None:
        def gpu_rows(n):
            return Y[:n].double().cpu().numpy(), dY[:n].double().cpu().numpy(), gx[:n].double().cpu().numpy()

        def gpu_rows_f64(n):
            # the float64 run of the same workload, whole, sliced
            x64 = torch.as_tensor(standard_normal_points(N_POINTS, SEEDS["plain_gpu"]), dtype=torch.float64).to(dev)
            g64 = torch.as_tensor(standard_normal((N_POINTS, K), SEEDS["plain_gpu_grad"]),
                                  dtype=torch.float64).to(dev)
            Y64, dY64 = sph.sph_compute_with_gradients(x64, L_MAX, NORMALIZE)
            gx64 = sph.sph_backward(dY64, g64, L_MAX)
            return Y64[:n].cpu().numpy(), dY64[:n].cpu().numpy(), gx64[:n].cpu().numpy()

        def gpu_c1(norm):
            x1 = torch.as_tensor(standard_normal_points(1000, SEEDS["plain_cpu"]), dtype=torch.float64).to(dev)
            Y1, dY1 = sph.sph_compute_with_gradients(x1, 4, norm)
            return Y1.cpu().numpy(), dY1.cpu().numpy()
        out["cpu_baseline"], out["accuracy"] = cpu_baseline(pool, gpu_rows, gpu_rows_f64, gpu_c1)
        pool.close()
        pool.join()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
