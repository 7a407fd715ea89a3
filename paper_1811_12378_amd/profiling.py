"""Profiling workloads and rocprofv3 summaries for libhfci.

    python -m paper_1811_12378_amd.profiling stage [--n 256] [--poles 16] [--nrhs 1] [--steps 2] [--prec 32]
        Runs the batched fixed-point iteration for a fixed number of steps on the
        256^3 layered benchmark medium, so the middle-factor kernel runs
        (steps-1)*(q-2) + (q-3) launches over poles*nrhs systems, all active.
    python -m paper_1811_12378_amd.profiling net [--n 256] [--reps 5]
        Applies an (untrained) learned preconditioner to a random vector on the 256^3
        layered medium: the BF16-MFMA convolution kernels of one forward pass per rep.
    python -m paper_1811_12378_amd.profiling copy [--mib 2048]
        A device-to-device copy of known size (read + write) for calibrating
        the FETCH_SIZE / WRITE_SIZE counters.
    python -m paper_1811_12378_amd.profiling summarize --stats DIR [--fetch DIR --write DIR
        --copy-fetch DIR --copy-write DIR --copy-mib M] --kernel SUBSTR --out FILE [--cmd CMD ...]
        Reads rocprofv3 CSV output and writes a short text summary (and, with
        counters, the per-launch HBM traffic JSON next to it).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _stage(a):
    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import workloads as W
    from paper_1811_12378_amd import hfci

    wl = W.config_layered_256(n=a.n, nrhs=a.nrhs)
    ctx = hfci.Context(0)
    op = hfci.Operator(ctx, torch.from_numpy(wl.c).cuda(), wl.h, wl.omega, wl.damp_cells, wl.damp_rho2)
    if a.tune:
        op.set_tune(a.prec, *a.tune)
    cont = hfci.Contour(op, a.poles, 1.0, 0.5, a.q)
    dt = torch.complex64 if a.prec == 32 else torch.complex128
    f = torch.from_numpy(np.stack(wl.rhs)).cuda().to(dt)
    ctx.profile(True)
    y, steps = hfci.shifted_solve(op, cont, f, steps=a.steps)
    prof = ctx.profile_read()
    st = prof["fp_stage"]
    avg = st["total_ms"] / max(1, st["launches"])
    gbs = st["alg_bytes"] / max(1e-12, st["total_ms"] * 1e-3) / 1e9
    print(json.dumps({"n": a.n, "tune": op.get_tune(a.prec), "systems": a.poles * a.nrhs, "steps": a.steps,
                      "stage_launches": st["launches"],
                      "stage_avg_ms": avg, "stage_alg_bytes_per_launch": st["alg_bytes"] / max(1, st["launches"]),
                      "stage_alg_gbs": gbs}), flush=True)


def _net(a):
    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import workloads as W
    from paper_1811_12378_amd import hfci

    wl = W.config_layered_256(n=a.n, nrhs=1)
    ctx = hfci.Context(0)
    op = hfci.Operator(ctx, torch.from_numpy(wl.c).cuda(), wl.h, wl.omega, wl.damp_cells, wl.damp_rho2)
    net = hfci.Net(ctx, seed=1)
    r = torch.randn((1, a.n, a.n, a.n), dtype=torch.complex128, device="cuda")
    net.apply(op, r)
    torch.cuda.synchronize()
    import time
    t0 = time.perf_counter()
    for _ in range(a.reps):
        net.apply(op, r)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.reps
    print(json.dumps({"n": a.n, "reps": a.reps, "apply_ms": dt * 1e3}), flush=True)


def _copy(a):
    import torch
    n = a.mib * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}), flush=True)


def _read_csv(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find(d, pattern):
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise FileNotFoundError("no %s under %s" % (pattern, d))
    return hits[-1]


def _counter_per_dispatch(d, counter, kernel_sub):
    """Mean over dispatches of `counter` (summed over its instances) for kernels matching kernel_sub."""
    rows = _read_csv(_find(d, "*counter_collection.csv"))
    per = {}
    for r in rows:
        name = r.get("Kernel_Name", "")
        if kernel_sub not in name or r.get("Counter_Name") != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    if not per:
        raise RuntimeError("counter %s not found for %s" % (counter, kernel_sub))
    vals = list(per.values())
    return sum(vals) / len(vals), len(vals)


def source_hash():
    h = hashlib.sha256()
    for name in ("stencil.hip", "kernels.h"):
        with open(os.path.join(HERE, "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _summarize(a):
    rows = _read_csv(_find(a.stats, "*kernel_stats.csv"))
    lines = ["# rocprofv3 summary", ""]
    if a.cmd:
        lines += ["command:", "", "    " + " ".join(a.cmd), ""]
    lines += ["| kernel | calls | total ms | average us | % |", "|---|---:|---:|---:|---:|"]
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:12]:
        name = r["Name"]
        short = name if len(name) < 110 else name[:107] + "..."
        lines.append("| `%s` | %s | %.3f | %.2f | %.1f |" % (short, r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                                                             float(r["AverageNs"]) / 1e3,
                                                             100.0 * float(r["TotalDurationNs"]) / total))
    out = {}
    if a.fetch and a.write:
        fetch_k, nf = _counter_per_dispatch(a.fetch, "FETCH_SIZE", a.kernel)
        write_k, nw = _counter_per_dispatch(a.write, "WRITE_SIZE", a.kernel)
        cf, _ = _counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
        cw, _ = _counter_per_dispatch(a.copy_write, "WRITE_SIZE", a.copy_kernel)
        copy_bytes = a.copy_mib * 1024 * 1024
        # counters are in KiB; the copy kernel moves copy_bytes each way
        sf = copy_bytes / (cf * 1024.0)
        sw = copy_bytes / (cw * 1024.0)
        fetch_b = fetch_k * 1024.0 * sf
        write_b = write_k * 1024.0 * sw
        out = {"kernel": a.kernel, "source_hash": source_hash(), "shape": a.shape or [],
               "bytes_per_launch": fetch_b + write_b, "alg_bytes_per_launch": a.alg_bytes,
               "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
               "copy_scale_fetch": sf, "copy_scale_write": sw, "dispatches": [nf, nw]}
        lines += ["", "HBM traffic of `%s` per launch (FETCH_SIZE, WRITE_SIZE in KiB, each scaled by the "
                      "copy-kernel calibration factor):" % a.kernel, "",
                  "* fetch %.1f MB, write %.1f MB, total %.1f MB (factors %.4f / %.4f)"
                  % (fetch_b / 1e6, write_b / 1e6, (fetch_b + write_b) / 1e6, sf, sw)]
        if a.alg_bytes:
            lines += ["* algorithmic bytes per launch in the same runs %.1f MB: measured / algorithmic = %.3f"
                      % (a.alg_bytes / 1e6, (fetch_b + write_b) / a.alg_bytes)]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if out and a.traffic_json:
        with open(a.traffic_json, "w") as fh:
            json.dump(out, fh, indent=1)
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    s = sub.add_parser("stage")
    s.add_argument("--n", type=int, default=256)
    s.add_argument("--poles", type=int, default=16)
    s.add_argument("--nrhs", type=int, default=1)
    s.add_argument("--steps", type=int, default=2)
    s.add_argument("--q", type=int, default=8)
    s.add_argument("--prec", type=int, default=32)
    s.add_argument("--tune", type=int, nargs="+", metavar="V",
                   help="kern ty pd cz fuse [sg]: the stencil launch shape")
    nn = sub.add_parser("net")
    nn.add_argument("--n", type=int, default=256)
    nn.add_argument("--reps", type=int, default=5)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=2048)
    m = sub.add_parser("summarize")
    m.add_argument("--stats", required=True)
    m.add_argument("--fetch")
    m.add_argument("--write")
    m.add_argument("--copy-fetch")
    m.add_argument("--copy-write")
    m.add_argument("--copy-mib", type=int, default=2048)
    m.add_argument("--copy-kernel", default="copy")
    m.add_argument("--kernel", required=True)
    m.add_argument("--out", required=True)
    m.add_argument("--traffic-json")
    m.add_argument("--shape", type=int, nargs="+", help="stencil launch shape the counters were taken with")
    m.add_argument("--alg-bytes", type=float, help="algorithmic bytes per launch of the counter runs")
    m.add_argument("--cmd", nargs=argparse.REMAINDER)
    a = ap.parse_args(argv)
    {"stage": _stage, "net": _net, "copy": _copy, "summarize": _summarize}[a.cmd_name](a)


if __name__ == "__main__":
    main()
