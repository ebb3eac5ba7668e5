"""Launch-configuration tuner: times candidate configurations of a workload, each in a
fresh child process, and writes the fastest to the tuning cache that elbm_tune reads.

    python -m paper_1608_06915_amd.tune --workload sphere3d --storage f32 [--cache PATH]

Every candidate runs in a process of its own: the child sets the workload up, applies
the candidate (elbm_set_launch), warms up (graph capture), times the median of a few
windows of coarse steps with HIP events on the bound stream, checks stability and
prints one JSON line.  A candidate whose child fails, is unstable or exceeds its time
limit is dropped.  All candidates give bitwise identical populations (the library's
launch configurations are tested for that), so the choice is on time alone.

Cache format (one line per workload shape, the key built as elbm_tune builds it):
    "d<dim>s<storage>_<bricks of level 0>_<bricks of level 1>...": [graph, wg_per_cu, xcd, threads, occupancy, pipeline]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEFAULT_CACHE = os.path.join(HERE, "launch_cache.txt")
FIELDS = ("use_graph", "wg_per_cu", "xcd_remap", "threads", "occupancy", "pipeline")

_LINE = re.compile(r'^\s*"([^"]+)"\s*:\s*\[\s*(-?\d+)\s*,\s*(-?\d+)\s*,\s*(-?\d+)\s*,\s*(-?\d+)\s*,\s*(-?\d+)\s*,\s*(-?\d+)\s*\]')


def candidates(kind: str = "default"):
    """Launch configurations to time (dicts of elbm_set_launch arguments)."""
    out = []
    if kind == "small":
        for x in (1, 32):
            out.append(dict(use_graph=10, wg_per_cu=0, xcd_remap=x, threads=256, occupancy=1, pipeline=0))
        out.append(dict(use_graph=0, wg_per_cu=0, xcd_remap=1, threads=256, occupancy=1, pipeline=0))
        return out
    for x in (1, 32):
        for t in (128, 256):
            for p in (0, 2):
                out.append(dict(use_graph=10, wg_per_cu=0, xcd_remap=x, threads=t, occupancy=1, pipeline=p))
    out.append(dict(use_graph=10, wg_per_cu=0, xcd_remap=8, threads=256, occupancy=1, pipeline=0))
    out.append(dict(use_graph=10, wg_per_cu=0, xcd_remap=32, threads=256, occupancy=4, pipeline=0))
    out.append(dict(use_graph=10, wg_per_cu=2, xcd_remap=1, threads=256, occupancy=1, pipeline=1))
    out.append(dict(use_graph=1, wg_per_cu=0, xcd_remap=32, threads=256, occupancy=1, pipeline=0))
    out.append(dict(use_graph=0, wg_per_cu=0, xcd_remap=1, threads=256, occupancy=1, pipeline=0))
    return out


def read_cache(path: str):
    """{key: [6 ints]} from a cache file (missing file: empty)."""
    out = {}
    if not os.path.exists(path):
        return out
    with open(path) as fh:
        for line in fh:
            m = _LINE.match(line)
            if m:
                out[m.group(1)] = [int(v) for v in m.groups()[1:]]
    return out


def format_entry(key: str, cfg) -> str:
    vals = [int(cfg[f]) for f in FIELDS] if isinstance(cfg, dict) else [int(v) for v in cfg]
    if len(vals) != 6:
        raise ValueError("a launch configuration has six fields")
    return '"%s": [%s]' % (key, ", ".join(str(v) for v in vals))


def write_entry(path: str, key: str, cfg, comment: str = "") -> None:
    """Replace the line of `key` (or append one), keeping every other line; the file is
    rewritten through a temporary file and renamed."""
    if not re.fullmatch(r"[A-Za-z0-9_]+", key):
        raise ValueError("bad cache key %r" % key)
    lines = []
    if os.path.exists(path):
        with open(path) as fh:
            lines = fh.read().splitlines()
    entry = format_entry(key, cfg)
    kept = []
    for line in lines:
        m = _LINE.match(line)
        if m and m.group(1) == key:
            continue
        if comment and line.strip() == "# " + comment.strip():
            continue
        kept.append(line)
    if comment:
        kept.append("# " + comment.strip())
    kept.append(entry)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        fh.write("\n".join(kept) + "\n")
    os.replace(tmp, path)


def _spec(name: str):
    from paper_1608_06915_amd import synth

    if ":" in name:  # module:function returning a synth.Spec
        mod, fn = name.split(":", 1)
        import importlib

        return getattr(importlib.import_module(mod), fn)()
    return getattr(synth, name)()


def child(args) -> int:
    """Time one candidate configuration; print one JSON line."""
    import numpy as np
    import torch

    from paper_1608_06915_amd import elbm, synth

    torch.cuda.set_device(0)
    sp = _spec(args.workload)
    lat = elbm.Lattice(sp.D, sp.N, sp.periodic, sp.nu0, sp.levels, args.storage)
    synth.apply(sp, lat)
    lat.bind()
    for l in range(sp.levels):
        lo, n = lat.level_box(l)
        rho, u, nz = sp.init(l, lo, n)
        lat.init(l, rho, u, nz)
    cfg = json.loads(args.launch)
    lat.set_launch(**cfg)
    lat.advance(args.warmup)
    lat.synchronize()
    win = []
    for _ in range(args.windows):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(lat.stream)
        lat.advance(args.steps)
        b.record(lat.stream)
        b.synchronize()
        win.append(a.elapsed_time(b) / args.steps)
    key = "d%ds%d" % (sp.D, elbm.STORAGE[args.storage]) + "".join(
        "_%d" % lat.level_info(l)[3] for l in range(sp.levels))
    print(json.dumps({"key": key, "launch": cfg, "ms_per_step": float(np.median(win)),
                      "windows_ms_per_step": win, "stable": bool(lat.check())}), flush=True)
    return 0


def tune(workload: str, storage: str, cache: str = DEFAULT_CACHE, kind: str = "default", steps: int = 40,
         warmup: int = 10, windows: int = 3, timeout: float = 180.0, write: bool = True, log=sys.stderr):
    """Time every candidate in a child process; write the fastest to `cache`.
    Returns (key, best configuration, per-candidate results)."""
    results = []
    key = None
    env = dict(os.environ)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    for cfg in candidates(kind):
        cmd = [sys.executable, "-m", "paper_1608_06915_amd.tune", "--child", "--workload", workload, "--storage",
               storage, "--launch", json.dumps(cfg), "--steps", str(steps), "--warmup", str(warmup), "--windows",
               str(windows)]
        t0 = time.time()
        try:
            p = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env, cwd=ROOT)
            rec = None
            if p.returncode == 0:
                for line in p.stdout.splitlines()[::-1]:
                    if line.startswith("{"):
                        rec = json.loads(line)
                        break
            if rec is None:
                res = {"launch": cfg, "error": "exit %d: %s" % (p.returncode, (p.stderr or "")[-300:])}
            elif not rec["stable"]:
                res = {"launch": cfg, "error": "unstable"}
            else:
                res = {"launch": cfg, "ms_per_step": rec["ms_per_step"]}
                key = rec["key"]
        except subprocess.TimeoutExpired:
            res = {"launch": cfg, "error": "time limit %.0f s" % timeout}
        res["wall_s"] = round(time.time() - t0, 1)
        results.append(res)
        print("tune: %s %s %s -> %s" % (workload, storage, json.dumps(cfg),
                                         "%.5f ms/step" % res["ms_per_step"] if "ms_per_step" in res else res["error"]),
              file=log, flush=True)
    ok = [r for r in results if "ms_per_step" in r]
    if not ok:
        raise RuntimeError("tune: no candidate ran for %s %s" % (workload, storage))
    best = min(ok, key=lambda r: r["ms_per_step"])
    if write:
        write_entry(cache, key, best["launch"], comment="%s %s (paper_1608_06915_amd/tune.py, %d candidates)" % (
            workload, storage, len(results)))
    return key, best["launch"], results


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", required=True, help="synth workload name or module:function returning a Spec")
    ap.add_argument("--storage", default="f32", choices=("f64", "f32", "f16s", "bf16s"))
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--candidates", default="default", choices=("default", "small"))
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--windows", type=int, default=3)
    ap.add_argument("--timeout", type=float, default=180.0, help="seconds per candidate")
    ap.add_argument("--no-write", action="store_true")
    ap.add_argument("--child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--launch", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args(argv)
    if args.child:
        return child(args)
    key, best, results = tune(args.workload, args.storage, args.cache, args.candidates, args.steps, args.warmup,
                              args.windows, args.timeout, not args.no_write)
    print(json.dumps({"workload": args.workload, "storage": args.storage, "key": key, "best": best,
                      "candidates": results}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
