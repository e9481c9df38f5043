"""Sweeps of the decoder over the axes of the paper's experiments (Sec. 4):

* ``fig2``: u = 1, 2, 3 matrices at rate 0.5 over a grid of BSC error rates
  (throughput and success rate against e, the shape of Fig. 2);
* ``table3``: u = 3 at rates 0.5-0.8, each at the error rate where the
  efficiency f = m/(n h(e)) of eq. (3) sits in the paper's bins (Table 3).

Every point decodes 256 frames of n = 65536 bits from Bob's bits and error
rates (mbp_decode_from_bits, FP32 sum-product, T = 100, early exit) with the
inputs resident on the GPU, and reports throughput, frame error rate against
Alice's key, success rate, average iterations and f. Run as
``python -m paper_2001_07979_amd.sweep [fig2|table3|all] [--out FILE]``; one
JSON object per point goes to stdout (and FILE).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

FIG2_E = (0.04, 0.05, 0.06, 0.07, 0.08, 0.09, 0.10)
# (rate, f) pairs: the middle of each efficiency bin of Table 3
TABLE3 = ((0.5, 1.125), (0.5, 1.175), (0.5, 1.3), (0.6, 1.125), (0.7, 1.125), (0.8, 1.125))


def points(which: str):
    from .inputs import workloads as W
    out = []
    if which in ("fig2", "all"):
        out += [("fig2", 0.5, u, e) for u in (1, 2, 3) for e in FIG2_E]
    if which in ("table3", "all"):
        out += [("table3", r, 3, W.e_for_efficiency(r, f)) for r, f in TABLE3]
    return out


def measure(ctx, wl, reps: int = 5, schedule: str = "flooding") -> dict:
    import torch
    from . import mbp
    from .inputs import workloads as W
    fr = wl.frames()
    dc = mbp.Code.from_inputs(ctx, wl.code)
    dev = torch.device("cuda", ctx.device)
    y = torch.from_numpy(fr.y).to(dev)
    e = torch.from_numpy(fr.p.astype(np.float64)).to(dev)
    z = torch.from_numpy(fr.z).to(dev)

    def step():
        return mbp.decode_from_bits(ctx, dc, y, e, z, algo=wl.algo, max_iter=wl.max_iter, alpha=wl.alpha,
                                    clip=wl.clip, want_llr=False, schedule=schedule)

    out = step()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = step()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    bits = out["bits"].cpu().numpy()
    ok = out["ok"].cpu().numpy()
    m = wl.code.m[0]
    p = float(np.mean(fr.p))
    h = W.binary_entropy(p)
    code = wl.code
    return {"workload": wl.name, "rate": round(1 - m / code.n, 4), "u": code.u, "e": round(p, 5),
            "frames": fr.nframes, "mbps": round(fr.nframes * code.n / dt / 1e6, 1),
            "ms_per_step": round(dt * 1e3, 4), "fer": float(np.any(bits != fr.x, axis=1).mean()),
            "success": float(ok.mean()), "avg_iters": float(out["iters"].float().mean().item()),
            "f": round(m / (code.n * h), 4), "f_leak": round(code.u * m / (code.n * h), 4),
            "schedule": schedule}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("which", nargs="?", default="all", choices=["fig2", "table3", "all"])
    ap.add_argument("--frames", type=int, default=256)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--schedule", default="flooding", choices=["flooding", "serial"])
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    from . import mbp
    from .inputs import workloads as W
    ctx = mbp.Context(0)
    sink = open(args.out, "w") if args.out else None
    for kind, rate, u, e in points(args.which):
        wl = W.sweep_workload(rate, u, e, nframes=args.frames)
        rec = dict(sweep=kind, **measure(ctx, wl, args.reps, args.schedule))
        line = json.dumps(rec)
        print(line, flush=True)
        if sink:
            sink.write(line + "\n")
            sink.flush()
    if sink:
        sink.close()
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
