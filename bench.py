"""Throughput of the refined KBC hot path on one MI355X.

Workload (default): D3Q27 KBC flow past a sphere -- three nested 2x levels, coarse
256x128x128, sphere diameter 20 finest units, uniform inlet u = 0.05, outflow,
Re = 300 -- with FP32 populations (the headline) and weight-shifted FP16 populations
(alongside).  One step = one coarse step of the whole refined path (four finest
ticks: every level's stream-collide, interface gather/reconstruction/coalescence,
every collision), replayed from HIP graphs.  The four-level block forest (512 blocks
of 16^3 cells) is measured as a second workload in both storage forms.

Metric: fine-equivalent MLUPS = sum_l N_l 2^l x coarse steps / s / 1e6 (N_l: fluid
nodes of level l), i.e. the paper's time-step-weighted "equivalent fine level
points" per second; the median of five timed windows of K coarse steps each.  Also
reported: HBM fractions (algorithmic bytes per coarse step, and the dominant
stream-collide kernel's roofline measured with HIP events), the adjoint/forward time
ratio (two-level D2Q9 cylinder, mean drag over 2000 coarse steps, checkpoints every
100) and the FP64 CPU oracle on the same workload (OpenMP build on every host core,
and single-thread).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sphere3d]
"""
from __future__ import annotations

import argparse
import faulthandler
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "fine-equiv MLUPS & HBM % (FP32 vs FP16 store); adjoint/forward time ratio"
STORE_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in ("kernels.hip", "lbm_device.hpp", "elbm_dev.hpp"):
        with open(os.path.join(ROOT, "paper_1608_06915_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name, storage):
    """HBM bytes per stream-collide launch from the committed FETCH_SIZE/WRITE_SIZE
    summary of this workload, or None if there is none or the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_stream_collide.%s.%s.hbm_counters.md" % (workload_name, storage))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("source_sha256", "traffic_bytes_per_launch"):
                k, v = line.split(":", 1)
                vals[k] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def workload(name):
    from paper_1608_06915_amd import synth

    if name == "channel3d":
        return synth.channel3d(), ("D3Q27 KBC two-level channel 128x64x64 coarse, periodic x/z, bounce-back y, "
                                   "refined near-wall slabs 8 coarse rows, body force Re_tau~180, 5% seeded "
                                   "velocity perturbations")
    if name == "sphere3d":
        return synth.sphere3d(), ("D3Q27 KBC flow past a sphere, 3 nested 2x levels, coarse 256x128x128, D=20 "
                                  "finest units, inlet u=0.05, outflow, Re=300")
    if name == "sphere_paper3d":
        return synth.sphere_paper3d(), ("D3Q27 KBC flow past a sphere at the paper's scale: 4 nested 2x levels, coarse "
                                        "448x296x296, D=120 finest units, inlet u=0.05, outflow, Re=3700")
    if name == "forest3d":
        return synth.forest3d(), ("D3Q27 KBC periodic block forest, 4 levels, 512 blocks of 16^3 cells "
                                  "(204/154/106/48), 2:1 balanced, seeded |u|<=0.05")
    if name == "tgv2d":
        return synth.tgv2d(), "D2Q9 KBC two-level Taylor-Green 64x64 coarse, refined [16,48]^2"
    if name == "cylinder2d":
        return synth.cylinder2d(), "D2Q9 KBC two-level channel 256x128 with cylinder D=32 fine, Re=100"
    raise SystemExit("unknown workload " + name)


def mode_counts(lat, sp):
    """Nodes stream-collided per level and substep kind, from the node classes:
    returns per level (first-substep count, every-step count)."""
    out = []
    for l in range(sp.levels):
        c = lat.node_class(l)
        fluid = (c >= 0) & ((c & 1) == 0)
        ring = (c & 2) != 0
        pd = (c >> 2) & 3
        bulk = fluid & ~ring & ((pd >= 2) | (l == 0))
        inner = fluid & ~ring & (pd == 1) & (l > 0)
        out.append((int(bulk.sum() + inner.sum()), int(bulk.sum())))
    return out


def sc_bytes_per_coarse_step(sp, counts, sbytes):
    """Algorithmic bytes of the stream-collide launches in one coarse step: each
    processed node reads Q and writes Q populations."""
    L = sp.levels
    T = 1 << (L - 1)
    per_node = 2 * sp.Q * sbytes
    total_nodes, launches = 0, 0
    for t in range(1, T + 1):
        lmin = min(l for l in range(L) if t % (1 << (L - 1 - l)) == 0)
        for l in range(lmin, L):
            first = l == lmin and l > 0
            total_nodes += counts[l][0] if first else counts[l][1]
        launches += 1
    return total_nodes * per_node, launches, total_nodes


def fine_equiv_updates(lat, sp):
    return sum(lat.level_info(l)[1] * (1 << l) for l in range(sp.levels))


def owned_fine_equiv_updates(lat, sp):
    """The owned-node variant: level-l nodes counted by their owned volume (coarse units,
    child nodes 2^-D each, the overlap split at the cut), converted back to level-l
    nodes and weighted by the level's 2^l substeps."""
    return sum(float(np.nansum(lat.weights(l))) * (1 << (l * sp.D)) * (1 << l) for l in range(sp.levels))


def copy_ceiling_gbs(mib=1024, reps=10):
    """Read + write bandwidth of a plain streaming copy of `mib` MiB: the library's copy
    kernel (16-byte accesses, non-temporal stores, four workgroups per compute unit) and
    torch's copy_, each the median of three timings of `reps` copies."""
    import torch

    from paper_1608_06915_amd import elbm

    n = (mib << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, fn in (("stream_copy", lambda: elbm.stream_copy(b, a)), ("torch_copy", lambda: b.copy_(a))):
        for _ in range(3):
            fn()
        t = []
        for _ in range(3):
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            for _ in range(reps):
                fn()
            e.record()
            e.synchronize()
            t.append(s.elapsed_time(e))
        out[name] = 2 * (mib << 20) * reps / (float(np.median(t)) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


def run_gpu(sp, storage, steps, warmup, tune, launch=None, windows=5):
    """Set up the workload, then time `windows` windows of exactly `steps` coarse
    steps each (HIP events on the bound stream, synchronised on both sides)."""
    import torch

    from paper_1608_06915_amd import elbm

    lat = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, storage)
    from paper_1608_06915_amd import synth

    synth.apply(sp, lat)
    lat.bind()
    for l in range(sp.levels):
        lo, n = lat.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        lat.init(l, rho, u, nz)
    if launch:
        lat.set_launch(**launch)
    elif tune:
        # launch configuration chosen by the tuner (paper_1608_06915_amd/tune.py) and kept
        # in the tuning cache; the library default when the cache has none
        if not lat.use_cached_launch(os.environ.get("ELBM_TUNE_CACHE")):
            print("bench: no cached launch configuration, library default", file=sys.stderr, flush=True)
    print("bench: %s %s launch %s" % (sp.name, storage, lat.get_launch()), file=sys.stderr, flush=True)
    lat.advance(warmup)
    lat.synchronize()
    torch.cuda.synchronize()
    win = []
    for _ in range(windows):
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(lat.stream)
        lat.advance(steps)
        end.record(lat.stream)
        end.synchronize()
        torch.cuda.synchronize()
        win.append(start.elapsed_time(end))
    # the same number of steps again with HIP events around every stream-collide
    # launch, on the stream the kernels are launched on
    tot_ms, sc_ms, n_launch = lat.profile(steps)
    ok = lat.check()
    return lat, win, sc_ms, n_launch, tot_ms, ok


def measure(name, sp, storage, steps, warmup, tune, launch=None, windows=5):
    """One workload in one storage form: throughput, HBM fractions, roofline."""
    lat, win, sc_ms, n_launch, _, ok = run_gpu(sp, storage, steps, warmup, tune, launch, windows)
    ms = float(np.median(win))
    fe = fine_equiv_updates(lat, sp)
    value = fe * steps / (ms / 1e3) / 1e6
    counts = mode_counts(lat, sp)
    sbytes = STORE_BYTES[storage]
    bytes_step, launches_step, _ = sc_bytes_per_coarse_step(sp, counts, sbytes)
    per_launch_bytes = bytes_step / launches_step
    avg_launch_ms = sc_ms / max(n_launch, 1)
    achieved = per_launch_bytes / (avg_launch_ms / 1e3) / 1e9
    # whole-step HBM fraction with algorithmic bytes (every fluid node of every level
    # reads and writes Q populations per level step)
    step_bytes = fe * 2 * sp.Q * sbytes
    hbm_pct = step_bytes / (ms / steps / 1e3) / 1e9 / PEAK_HBM_GBS * 100
    print("bench: %s %s %.1f MLUPS_fe (median of %d windows), %.4f ms/step, stream-collide %.4f ms/launch %.0f GB/s, "
          "stable=%s" % (name, storage, value, len(win), ms / steps, avg_launch_ms, achieved, ok),
          file=sys.stderr, flush=True)
    out = {"value": round(value, 2), "ms_per_step": round(ms / steps, 5),
           "windows_ms": [round(w, 4) for w in win], "hbm_pct_alg": round(hbm_pct, 2),
           "mlups_fe_owned": round(owned_fine_equiv_updates(lat, sp) * steps / (ms / 1e3) / 1e6, 2),
           "stable": ok, "launch": lat.get_launch(),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(name, storage),
                        "kernel": "k_stream_collide", "bytes_per_launch": int(per_launch_bytes),
                        "avg_launch_ms": round(avg_launch_ms, 5), "launches": n_launch,
                        "bytes_per_node_update": 2 * sp.Q * sbytes}}
    info = {"levels": sp.levels, "fluid_nodes_per_level": [lat.level_info(l)[1] for l in range(sp.levels)],
            "fine_equiv_updates_per_step": fe}
    return lat, out, info


def _init(lat, sp):
    for l in range(sp.levels):
        lo, n = lat.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        lat.init(l, rho, u, nz)


def run_adjoint(name, storage, n, K):
    """Forward time of n coarse steps vs a full adjoint run (forward with checkpoints
    every K, recomputation, reverse sweep) of the mean drag on the body level, or of
    the final kinetic energy when the workload has no body."""
    import torch

    from paper_1608_06915_amd import elbm, synth

    sp, desc = workload(name)
    lat = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, storage)
    synth.apply(sp, lat)
    lat.bind()
    # the forward and the adjoint's checkpointed forward both take the cached launch
    # configuration of the workload
    if not lat.use_cached_launch(os.environ.get("ELBM_TUNE_CACHE")):
        print("bench: adjoint workload: no cached launch configuration, library default", file=sys.stderr, flush=True)
    _init(lat, sp)
    obj, bl = ("drag", sp.body_level) if sp.body_level is not None else ("ke", 0)
    lat.adjoint_bind(n, K)
    lat.adjoint_forward(min(n, K), obj, bl, (1.0, 0.0, 0.0))  # warm-up: graphs, code paths
    lat.adjoint_backward()
    _init(lat, sp)
    lat.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    lat.advance(n)
    end.record(lat.stream)
    end.synchronize()
    fwd_ms = start.elapsed_time(end)
    _init(lat, sp)
    lat.synchronize()
    t0 = time.time()
    J = lat.adjoint_forward(n, obj, bl, (1.0, 0.0, 0.0))
    lat.adjoint_backward()
    wall_ms = (time.time() - t0) * 1e3
    ms = lat.adjoint_timing()
    fe = fine_equiv_updates(lat, sp)
    # forward with checkpoints, then the backward pass (recomputation of a segment
    # overlapping the reverse sweep of the next), each timed on the stream
    adj_ms = ms[0] + ms[3]
    print("bench: adjoint %s %s n=%d K=%d forward %.1f ms, adjoint %.1f ms (fwd+ckpt %.1f, backward %.1f: recompute "
          "%.1f overlapping reverse %.1f), ratio %.2f" % (name, storage, n, K, fwd_ms, adj_ms, ms[0], ms[3], ms[1],
                                                         ms[2], adj_ms / fwd_ms),
          file=sys.stderr, flush=True)
    return {"workload": desc, "storage": storage, "objective": obj, "coarse_steps": n, "checkpoint_every": K,
            "forward_ms": round(fwd_ms, 3), "adjoint_ms": round(adj_ms, 3),
            "adjoint_breakdown_ms": {"forward_with_checkpoints": round(ms[0], 3), "backward": round(ms[3], 3),
                                     "recompute": round(ms[1], 3), "reverse": round(ms[2], 3)},
            "ratio": round(adj_ms / fwd_ms, 3), "ratio_wall": round(wall_ms / fwd_ms, 3),
            "forward_MLUPS_fe": round(fe * n / (fwd_ms / 1e3) / 1e6, 1), "J": J, "launch": lat.get_launch()}


def _plane_value(field, x, y):
    """bilinear value of a 2-D plane field (numpy order y, x) at fractional (x, y), over the
    corners that hold a value (NaN marks solid or absent nodes)"""
    x0, y0 = int(math.floor(x)), int(math.floor(y))
    acc, wsum = 0.0, 0.0
    for dy in (0, 1):
        for dx in (0, 1):
            w = (1 - abs(x - (x0 + dx))) * (1 - abs(y - (y0 + dy)))
            yy, xx = y0 + dy, x0 + dx
            if 0 <= yy < field.shape[0] and 0 <= xx < field.shape[1] and np.isfinite(field[yy, xx]) and w > 0:
                acc += w * field[yy, xx]
                wsum += w
    return acc / wsum if wsum > 0 else float("nan")


def wake_statistics(lat, sp, steps, every):
    """Time-averaged sphere-wake quantities over `steps` coarse steps, sampled every
    `every` steps on the z-plane through the sphere centre (body level, the level above
    it for the wake axis, level 0 for the free stream): the mean drag coefficient
    C_d = F_x / (rho U^2 pi R^2 / 2); the base pressure coefficient C_pb = (p_b - p_inf) /
    (rho U^2 / 2) with p = rho / 3, p_b at the first fluid node behind the sphere on the
    axis and p_inf on the axis 5 D upstream; the recirculation length L_r / D from the
    sphere's rear to where the mean axial velocity on the axis turns positive; the
    separation angle, from the front stagnation point, where the mean tangential
    velocity one node off the surface changes sign (both half-planes averaged)."""
    import torch

    bl = sp.body_level
    cb, R = sp.bodies[bl][0], sp.body_diameter / 2.0
    levels = sorted({0, max(bl - 1, 0), bl})
    planes = {}
    for l in levels:
        lo, n = lat.level_box(l)
        s = 2.0 ** (bl - l)
        planes[l] = {"lo": lo, "k": int(round(cb[2] / s)) - int(lo[2]), "rho": None, "u": None}
    lat.drag(bl, reset=True)
    done, samples = 0, 0
    while done < steps:
        k = min(every, steps - done)
        lat.advance(k)
        done += k
        for l in levels:
            rho, u = lat.moments_device(l)
            p = planes[l]
            r2, u2 = rho[p["k"]].clone(), u[:, p["k"]].clone()
            p["rho"] = r2 if p["rho"] is None else p["rho"] + r2
            p["u"] = u2 if p["u"] is None else p["u"] + u2
            del rho, u
        samples += 1
        if done % 1000 < every:
            print("bench: wake averaging %d / %d coarse steps" % (done, steps), file=sys.stderr, flush=True)
    F, nst = lat.drag(bl, reset=True)
    lat.synchronize()
    for l in levels:
        planes[l]["rho"] = (planes[l]["rho"] / samples).cpu().numpy()
        planes[l]["u"] = (planes[l]["u"] / samples).cpu().numpy()
    U = sp.U
    cd = 2.0 * (F[0] / nst) / (U ** 2 * math.pi * R * R)

    def at(l, X, Y, what, comp=0):
        """mean field of level l at body-level position (X, Y) on the plane"""
        s = 2.0 ** (bl - l)
        p = planes[l]
        f = p["rho"] if what == "rho" else p["u"][comp]
        return _plane_value(f, X / s - p["lo"][0], Y / s - p["lo"][1])

    # free stream: level 0, 5 D upstream on the axis; base: first fluid node behind the sphere
    D = 2.0 * R
    rho_inf = at(0, cb[0] - 5 * D, cb[1], "rho")
    xb = math.floor(cb[0] + R) + 1.0
    rho_b = at(bl, xb, cb[1], "rho")
    cpb = (rho_b - rho_inf) / 3.0 / (0.5 * rho_inf * U * U)
    # recirculation length on the axis, finest level holding the point
    lr = float("nan")
    prev = None
    X = xb
    while X < cb[0] + 8 * D:
        v = at(bl, X, cb[1], "u", 0)
        if not np.isfinite(v) and bl > 0:
            v = at(bl - 1, X, cb[1], "u", 0)
        if not np.isfinite(v):
            break
        if prev is not None and prev[1] < 0.0 <= v:
            x0 = prev[0] + (X - prev[0]) * (-prev[1]) / (v - prev[1])
            lr = (x0 - (cb[0] + R)) / D
            break
        prev = (X, v)
        X += 1.0
    # separation angle one node off the surface, in both half-planes
    angles = []
    for sgn in (1.0, -1.0):
        prev = None
        for th in np.arange(20.0, 170.0, 0.25):
            t = math.radians(th)
            r = R + 1.0
            Xp, Yp = cb[0] - r * math.cos(t), cb[1] + sgn * r * math.sin(t)
            ut = at(bl, Xp, Yp, "u", 0) * math.sin(t) + at(bl, Xp, Yp, "u", 1) * sgn * math.cos(t)
            if prev is not None and np.isfinite(ut) and np.isfinite(prev[1]) and prev[1] > 0.0 >= ut:
                angles.append(prev[0] + (th - prev[0]) * prev[1] / (prev[1] - ut))
                break
            prev = (th, ut)
    phis = float(np.mean(angles)) if angles else float("nan")
    return {"C_d": round(float(cd), 5), "C_pb": round(float(cpb), 5), "L_r_over_D": round(float(lr), 4),
            "phi_s_deg": round(phis, 3), "window_coarse_steps": steps, "samples": samples,
            "paper": {"C_d": 0.383, "C_pb": -0.220, "L_r_over_D": 2.51, "phi_s_deg": 89.993},
            "note": "halfway bounce-back walls (the paper uses Grad's wall condition); separation angle "
                    "measured one node off the surface in the plane through the centre"}


def cpu_baseline(sp, fe_updates, steps, library):
    """The FP64 oracle on the same workload: `steps` coarse steps after its set-up."""
    import oracle

    t0 = time.time()
    o = oracle.Oracle(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, library=library)
    from paper_1608_06915_amd import synth

    synth.apply(sp, o)
    for l in range(sp.levels):
        lo, n = o.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        o.init(l, rho, u, nz)
    setup = time.time() - t0
    t0 = time.time()
    o.advance(steps)
    dt = time.time() - t0
    return fe_updates * steps / dt / 1e6, dt, setup


def host_cores():
    """(threads the OpenMP oracle uses, logical CPUs this process may run on, lscpu model line)"""
    import subprocess

    import oracle

    threads = oracle.omp_threads()
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = ""
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return threads, avail, model


def main():
    faulthandler.enable()  # a fatal signal prints the Python stack of every thread
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="coarse steps per timed window")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--windows", type=int, default=5, help="timed windows (the median is reported)")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--workload", default="sphere3d")
    ap.add_argument("--extra-workload", default="forest3d",
                    help="second workload measured in FP32 and FP16s ('' for none)")
    ap.add_argument("--cpu-steps", type=int, default=8, help="coarse steps of the OpenMP oracle leg")
    ap.add_argument("--cpu-steps-serial", type=int, default=1, help="coarse steps of the single-thread oracle leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-half", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the library default launch configuration (ignore the tuning cache)")
    ap.add_argument("--launch", default=None,
                    help='fixed launch configuration as JSON, e.g. {"threads": 128} (ignores the tuning cache)')
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--drag-steps", type=int, default=0,
                    help="after the timed steps, report the body's mean drag coefficient over this many coarse steps")
    ap.add_argument("--wake-steps", type=int, default=0,
                    help="after the drag window, time-average the sphere wake over this many coarse steps (C_d, C_pb, "
                         "L_r, separation angle)")
    ap.add_argument("--wake-every", type=int, default=10, help="coarse steps between wake samples")
    ap.add_argument("--adjoint-workload", default="cylinder2d")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--adjoint-K", type=int, default=100)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (scale for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        n = args.copy_calibration << 20
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": n, "copy_bytes_written_per_launch": n, "launches": 5}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU; multi-GPU runs are not supported", file=sys.stderr)
        raise SystemExit(2)

    import torch

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    sp, desc = workload(args.workload)
    print("bench: workload=%s storage=%s steps=%d x %d windows warmup=%d" % (
        args.workload, args.storage, args.steps, args.windows, args.warmup), file=sys.stderr, flush=True)
    launch = json.loads(args.launch) if args.launch else None
    lat, head, info = measure(args.workload, sp, args.storage, args.steps, args.warmup, not args.no_tune, launch,
                              args.windows)
    fe = info["fine_equiv_updates_per_step"]
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "MLUPS (fine-equivalent)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": dict({"workload": desc}, **info, storage=args.storage,
                       compute="f32" if args.storage != "f64" else "f64", launch=head["launch"]),
        "windows": args.windows,
        "windows_ms": head["windows_ms"],
        "hbm_pct_alg": head["hbm_pct_alg"],
        "mlups_fe_owned": head["mlups_fe_owned"],
        "stable": head["stable"],
        "roofline": head["roofline"],
    }
    if args.drag_steps > 0 and sp.body_level is not None:
        # mean drag coefficient of the body over the next drag_steps coarse steps:
        # C_d = F_x / (rho U^2 pi R^2 / 2), F the momentum exchanged per body-level step
        bl = sp.body_level
        R = sp.body_diameter / 2.0
        lat.drag(bl, reset=True)
        done, fx, nst, wins = 0, 0.0, 0, []
        while done < args.drag_steps:
            n = min(1000, args.drag_steps - done)
            lat.advance(n)
            F, k = lat.drag(bl, reset=True)  # synchronous
            fx, nst, done = fx + F[0], nst + k, done + n
            wins.append(round(float(2.0 * (F[0] / k) / (sp.U ** 2 * math.pi * R * R)), 5))
            print("bench: drag window %d / %d coarse steps, C_d of the last %d: %.4f" % (done, args.drag_steps, n,
                                                                                      wins[-1]),
                  file=sys.stderr, flush=True)
        cd = 2.0 * (fx / nst) / (sp.U ** 2 * math.pi * R * R)
        before = args.warmup + (args.windows + 1) * args.steps  # warm-up, timed windows and the profiling pass
        out["drag"] = {"C_d": round(float(cd), 5), "after_coarse_steps": before,
                       "window_coarse_steps": args.drag_steps, "C_d_per_1000_coarse_steps": wins,
                       "stable": bool(lat.check())}
        print("bench: C_d %.4f over coarse steps %d-%d" % (cd, before, before + args.drag_steps),
              file=sys.stderr, flush=True)
    if args.wake_steps > 0 and sp.body_level is not None and sp.D == 3:
        out["wake"] = wake_statistics(lat, sp, args.wake_steps, args.wake_every)
        out["wake"]["stable"] = bool(lat.check())
        print("bench: wake " + json.dumps(out["wake"]), file=sys.stderr, flush=True)
    del lat
    torch.cuda.empty_cache()
    cc = copy_ceiling_gbs()
    out["roofline"]["copy_ceiling_GBs"] = round(cc["stream_copy"], 1)
    out["roofline"]["torch_copy_GBs"] = round(cc["torch_copy"], 1)
    out["roofline"]["frac_of_copy_ceiling"] = round(out["roofline"]["achieved"] / cc["stream_copy"], 4)
    print("bench: plain streaming copy %.0f GB/s read + write (torch copy_ %.0f GB/s); stream-collide at %.2f of it"
          % (cc["stream_copy"], cc["torch_copy"], out["roofline"]["frac_of_copy_ceiling"]), file=sys.stderr, flush=True)
    if not args.no_half and args.storage == "f32" and not launch:
        lat2, half, _ = measure(args.workload, sp, "f16s", args.steps, args.warmup, not args.no_tune, None,
                                args.windows)
        out["f16s"] = half
        del lat2
        torch.cuda.empty_cache()
    if args.extra_workload and not launch:
        sp2, desc2 = workload(args.extra_workload)
        extra = {"workload": desc2}
        for st in ("f32", "f16s") if not args.no_half else ("f32",):
            lat3, res, info2 = measure(args.extra_workload, sp2, st, args.steps, args.warmup, not args.no_tune, None,
                                       args.windows)
            extra.update(info2)
            extra[st] = res
            del lat3
            torch.cuda.empty_cache()
        out[args.extra_workload] = extra
    if not args.no_adjoint:
        out["adjoint"] = run_adjoint(args.adjoint_workload, args.storage, args.adjoint_steps, args.adjoint_K)
    if not args.no_cpu:
        threads, avail, model = host_cores()
        mlups, dt, setup = cpu_baseline(sp, fe, args.cpu_steps, "omp")
        m1, dt1, setup1 = cpu_baseline(sp, fe, args.cpu_steps_serial, None)
        out["cpu_baseline"] = {
            "value": round(mlups, 4), "unit": "MLUPS (fine-equivalent)", "cores": threads, "kind": "oracle",
            "sample": "%d coarse steps of the same workload, FP64 oracle built with OpenMP, %d threads on %d "
                      "available logical CPUs (%s): %.1f s after a %.1f s set-up" % (
                          args.cpu_steps, threads, avail, model or "lscpu model unknown", dt, setup),
            "single_thread": {"value": round(m1, 4), "cores": 1,
                              "sample": "%d coarse step(s), the same oracle built without OpenMP: %.1f s after a "
                                        "%.1f s set-up" % (args.cpu_steps_serial, dt1, setup1)}}
        print("bench: oracle %.3f MLUPS_fe on %d threads, %.3f single-thread" % (mlups, threads, m1),
              file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
