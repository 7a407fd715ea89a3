"""Training pipeline of the learned preconditioner (all compute in libhfci's kernels).

    python -m paper_1811_12378_amd.learned train --out net.bin [--n 64] [--media 24] [--pairs 48]
                                                 [--steps 4000] [--crop 64]
    python -m paper_1811_12378_amd.learned eval --net net.bin [--n 256] [--medium grf|layered]

Pairs: on each random medium (Gaussian random field wavespeed, 10 points per
wavelength), FGMRES with the FCI preconditioner solves for a random right-hand side
and hands back every Arnoldi pair (v_j, FCI(v_j)) - the shifted polynomial iteration
generates the corrections the network learns.  Training: Adam on whole volumes (or
crops) with a random global phase per step.  FCI(v) = d(v) w(v) where the step size d
of Alg. 1 is a global complex scalar that a local network cannot see, and FGMRES only
uses the direction of its search vectors, so the default loss is the scale- and
phase-invariant 1 - |<o, t>|^2 / (|o|^2 |t|^2).  Use: FGMRES with
precond = learned keeps the best multiple of N(v_j) when its residual ||v_j - d A N(v_j)|| is
within tau times FCI's mean residual on the same solve, and falls back to FCI(v_j) otherwise.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def harvest_pairs(ctx, n=64, media=24, pairs=48, J=16, eps=0.25, q=8, ppw=10.0, seed=100):
    """(v, e, kch, medium_of_pair) on the device from FGMRES runs on `media` random media."""
    import torch

    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import workloads as W
    from . import hfci

    v = torch.empty((media * pairs, n, n, n), dtype=torch.complex64, device="cuda")
    e = torch.empty_like(v)
    kch = torch.empty((media, n, n, n), dtype=torch.float32, device="cuda")
    mop = np.zeros(media * pairs, dtype=np.int32)
    got = 0
    for m in range(media):
        c = W.grf_medium(n, seed + m)
        omega = W.omega_for_ppw(float(c.min()), n, ppw)
        op = hfci.Operator(ctx, torch.from_numpy(c).cuda(), 1.0 / n, omega, 8, 1.0)
        cont = hfci.Contour(op, J, 1.0, eps, q)
        kch[m] = hfci.medium_channel(op)
        if m % 2 == 0:
            f = W.point_source(n, tuple(int(x) for x in W.source_nodes(n, 1, seed + m, 9)[0]))
        else:
            f = W.gaussian_rhs(n, seed + 1000 + m)
        fd = torch.from_numpy(f[None]).cuda()
        opts = hfci.default_opts(precision=32, tol=1e-9, max_it=pairs)
        opts.harvest_cap = pairs
        opts.harvest_v = v[got].data_ptr()
        opts.harvest_z = e[got].data_ptr()
        _, st = hfci.solve(op, cont, fd, opts=opts)
        k = st["harvested"]
        mop[got:got + k] = m
        got += k
        log("medium %d: %d pairs (relres %.2e after %d its)" % (m, k, st["final_relres"], st["its"]))
        cont.close()
        op.close()
    return v[:got], e[:got], kch, mop[:got]


def train(ctx, out, n=64, media=24, pairs=48, steps=4000, crop=64, lr=1e-3, lr_min=1e-5, seed=0, J=16, eps=0.25,
          loss_kind=1):
    from . import hfci
    t0 = time.perf_counter()
    v, e, kch, mop = harvest_pairs(ctx, n=n, media=media, pairs=pairs, J=J, eps=eps)
    t1 = time.perf_counter()
    net = hfci.Net(ctx, seed=seed)
    final, curve = net.train(v, e, kch, mop, crop=crop, steps=steps, lr=lr, lr_min=lr_min, log_every=max(1, steps // 20),
                             seed=seed, verbose=True, loss_kind=loss_kind)
    t2 = time.perf_counter()
    if out:
        net.save(out)
    info = {"pairs": int(v.shape[0]), "harvest_s": t1 - t0, "train_s": t2 - t1, "final_loss": final,
            "curve": [float(x) for x in curve], "steps": steps, "crop": crop}
    del v, e, kch
    return net, info


def compare(ctx, net, n=256, medium="grf", seed=777, J=16, eps=0.25, tol=1e-6, taus=(0.9,), max_it=1500,
            nrhs=1, verbose=1):
    """Time-to-tol with FCI only versus the learned preconditioner (FCI as fallback)."""
    import torch

    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import workloads as W
    from . import hfci

    if medium == "layered":
        wl = W.config_layered_256(n=n, nrhs=nrhs, seed=seed)
    else:
        c = W.grf_medium(n, seed)
        nodes = W.source_nodes(n, nrhs, seed + 5, 9)
        wl = W.Workload("grf_%d" % n, c, W.omega_for_ppw(float(c.min()), n, 10.0), 8, 1.0,
                        [W.point_source(n, p) for p in nodes])
    op = hfci.Operator(ctx, torch.from_numpy(wl.c).cuda(), wl.h, wl.omega, wl.damp_cells, wl.damp_rho2)
    cont = hfci.Contour(op, J, 1.0, eps, 8)
    f = torch.from_numpy(np.stack(wl.rhs)).cuda()
    res = {}
    hfci.solve(op, cont, f, opts=hfci.default_opts(precision=32, tol=tol, max_it=1))  # allocate
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = hfci.solve(op, cont, f, opts=hfci.default_opts(precision=32, tol=tol, max_it=max_it, verbose=verbose))
    torch.cuda.synchronize()
    res["fci"] = dict(st, time_s=time.perf_counter() - t0)
    log("fci only: %.2f s, %d its, relres %.2e" % (res["fci"]["time_s"], st["its"], st["final_relres"]))
    for tau in taus:
        o = hfci.default_opts(precision=32, tol=tol, max_it=max_it, precond=2, learned_tau=tau, verbose=verbose)
        o.net = net.h.value
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = hfci.solve(op, cont, f, opts=o)
        torch.cuda.synchronize()
        res["learned_tau_%g" % tau] = dict(st, time_s=time.perf_counter() - t0)
        log("learned tau %g: %.2f s, %d its (%d kept, %d fallbacks), relres %.2e, net %.0f ms, "
            "mean scaled residual net %.3f / fci %.3f"
            % (tau, res["learned_tau_%g" % tau]["time_s"], st["its"], st["learned_accepted"],
               st["learned_fallbacks"], st["final_relres"], st["time_net_ms"], st["net_rho_mean"],
               st["fci_rho_mean"]))
    cont.close()
    op.close()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--n", type=int, default=64)
    t.add_argument("--media", type=int, default=24)
    t.add_argument("--pairs", type=int, default=48)
    t.add_argument("--steps", type=int, default=4000)
    t.add_argument("--crop", type=int, default=64)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--seed", type=int, default=0)
    e = sub.add_parser("eval")
    e.add_argument("--net", required=True)
    e.add_argument("--n", type=int, default=256)
    e.add_argument("--medium", default="grf")
    e.add_argument("--taus", type=float, nargs="+", default=[0.9])
    a = ap.parse_args(argv)
    from . import hfci
    ctx = hfci.Context(0)
    if a.cmd == "train":
        _, info = train(ctx, a.out, n=a.n, media=a.media, pairs=a.pairs, steps=a.steps, crop=a.crop, lr=a.lr,
                        seed=a.seed)
        print(json.dumps(info))
    else:
        net = hfci.Net(ctx)
        net.load(a.net)
        print(json.dumps(compare(ctx, net, n=a.n, medium=a.medium, taus=a.taus), default=float))


if __name__ == "__main__":
    main()
