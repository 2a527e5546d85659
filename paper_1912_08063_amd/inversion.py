"""Full-waveform inversion outer loop: L-BFGS with a backtracking line search.

Each iteration minimises the least-squares misfit of Eq. 1 over the velocity
model: the misfit and its gradient come from fwi_gradient (forward,
checkpointed adjoint and imaging condition in the HIP library), trial models
of the line search from fwi_forward.  The model is kept inside [vmin, vmax]
and the sponge damping is held fixed across iterations, as the gradient
assumes.

    python -m paper_1912_08063_amd.inversion --iters 10 --shots 32
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _dot(a, b):
    return float((a.double() * b.double()).sum())


def misfit(v, obs, src, src_pos, rec_pos, cfg, workspace=None):
    """Eq. 1 for a trial model: forward traces, then sum (d - obs)^2 in fp64."""
    from . import api
    d = api.forward(v, src, src_pos, rec_pos, cfg, workspace=workspace)
    return float(((d.double() - obs.double()) ** 2).sum())


def lbfgs(v0, obs, src, src_pos, rec_pos, cfg, iters=10, memory=5, vmin=None, vmax=None,
          first_step=20.0, c1=1e-4, max_backtracks=8, log=None, steps=None):
    """Returns (v, history) with history[i] = misfit before iteration i (and the last).
    If `steps` is a list, the accepted step length of each iteration is appended."""
    import torch

    from . import api
    v = v0.clone()
    vmin = float(v0.min()) if vmin is None else vmin
    vmax = float(v0.max()) if vmax is None else vmax
    ws, wf = api.Workspace(), api.Workspace()
    phi, g = api.gradient(v, obs, src, src_pos, rec_pos, cfg, workspace=ws)
    hist = [phi]
    S, Y = [], []
    for it in range(iters):
        # two-loop recursion for the L-BFGS direction d = -H g
        q = g.clone()
        alphas = []
        for s, y in reversed(list(zip(S, Y))):
            rho = 1.0 / _dot(y, s)
            a = rho * _dot(s, q)
            alphas.append((a, rho, s, y))
            q -= a * y
        if S:
            q *= _dot(S[-1], Y[-1]) / _dot(Y[-1], Y[-1])
        for a, rho, s, y in reversed(alphas):
            b = rho * _dot(y, q)
            q += (a - b) * s
        d = -q
        gd = _dot(g, d)
        if gd >= 0:                      # not a descent direction: restart
            S, Y = [], []
            d = -g
            gd = _dot(g, d)
        # first trial: unit step for quasi-Newton directions, else a step that
        # changes the model by at most `first_step` m/s
        step = 1.0 if S else first_step / max(float(d.abs().max()), 1e-30)
        accepted = False
        for _ in range(max_backtracks):
            vt = torch.clamp(v + step * d, vmin, vmax)
            pt = misfit(vt, obs, src, src_pos, rec_pos, cfg, workspace=wf)
            if pt <= phi + c1 * step * gd:
                accepted = True
                break
            step *= 0.5
        if not accepted:
            if log:
                log("iteration %d: line search failed, stopping" % it)
            break
        pn, gn = api.gradient(vt, obs, src, src_pos, rec_pos, cfg, workspace=ws)
        s, y = vt - v, gn - g
        if _dot(s, y) > 1e-30 * max(_dot(y, y), 1e-300):
            S.append(s)
            Y.append(y)
            if len(S) > memory:
                S.pop(0)
                Y.pop(0)
        v, g, phi = vt, gn, pn
        hist.append(phi)
        if steps is not None:
            steps.append(step)
        if log:
            log("iteration %d: misfit %.6e (step %.3g)" % (it, phi, step))
    return v, hist


def main(argv=None):
    import torch

    from . import api, workloads as wl
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--shots", type=int, default=32)
    ap.add_argument("--nt", type=int, default=3000)
    ap.add_argument("--every", type=int, default=50)
    args = ap.parse_args(argv)
    log = lambda m: print("[fwi] " + m, file=sys.stderr, flush=True)
    P = wl.shots_2d(nt=args.nt, nshots=args.shots)
    dev = torch.device("cuda:0")
    t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(d)
    w, s, r = t(P.wavelet, torch.float32), t(P.src_pos, torch.int32), t(P.rec_pos, torch.int32)
    cfg = api.Config(dt=P.dt, dx=P.dx, order=P.order, nsponge=P.nb, eta_max=P.eta_max,
                     ckpt="every:%d" % args.every)
    truth = t(P.v, torch.float32)
    obs = api.forward(truth, w, s, r, cfg)
    v0 = t(P.v_start, torch.float32)
    t0 = time.perf_counter()
    v, hist = lbfgs(v0, obs, w, s, r, cfg, iters=args.iters, vmin=1500.0, vmax=4500.0, log=log)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    err0 = float((v0 - truth).norm() / truth.norm())
    err = float((v - truth).norm() / truth.norm())
    print(json.dumps({"workload": P.name, "iterations": len(hist) - 1, "misfit": hist,
                      "relative_misfit": [h / hist[0] for h in hist],
                      "model_error_start": err0, "model_error_end": err, "seconds": secs}),
          flush=True)


if __name__ == "__main__":
    main()
