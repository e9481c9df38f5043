"""Run the HIP decoder and the FP64 oracle on the same seeded inputs, and
compare them under the parity protocol.

Protocol (GPU against the FP64 oracle):
* a frame the oracle decodes without a near tie (its flag is 0) must match
  exactly in success, iteration count and every decided bit;
* its final soft decisions must agree to `rtol` (1e-4 for FP32) relative,
  plus ATOL32 = 1e-5 absolute for FP32 (the representation limit of the
  summed messages where they cancel), wherever |L| >= 1e-3, whatever the
  frame's iteration count. A test may name a longer-decode bound instead
  (`long_after`, `long_rtol`) where its inputs include decodes long enough
  for FP32 to drift from FP64 by more than that; each such bound is a
  measured one, recorded with its evidence beside the test;
* FP32 min-sum frames that stop after `long_after` iterations with
  `long_rtol=None` are held bit for bit to the oracle's binary32 min-sum by
  their test, and against FP64 only counted: at most `long_budget` of the
  frames may disagree (min-sum's rounding grows by about alpha (d_v - 1) per
  iteration, enough to move a long decode's stopping iteration or outcome);
* a frame the oracle fails must fail on the GPU too with iters = T;
* flagged frames (a soft decision within 1e-3 of zero at a point where FP32
  rounding could change the outcome) are compared and counted; together with
  failed-frame disagreements they may not exceed 1% of the frames.
"""
from __future__ import annotations

import numpy as np

import oracle

SMALL = 1e-3
# Longer-decode bounds, measured (GPU against the FP64 oracle on the tests'
# own inputs; the largest relative difference of L beyond ATOL32):
# * FP32 sum-product stays within 1e-4 for frames that stop within
#   SPA_LONG_AFTER = 16 iterations (largest 9.6e-5, at 13 iterations, among
#   300 stragglers up to BSC 0.09); beyond, single frames near a code's
#   threshold drift further (1.5e-4 to 0.10 between 18 and 47 iterations)
#   with every decision the same, so those tests name their own bound.
# * FP32 min-sum amplifies rounding by about alpha (d_v - 1) per iteration:
#   within 1e-4 up to 7 flooding iterations (largest 2.1e-5) and 5 serial
#   iterations of u = 2 (3.5e-5), 1.3e-4 already at 6. Later frames are held
#   bit for bit to the binary32 oracle and only counted against FP64.
SPA_LONG_AFTER = 16
NMS_LONG_AFTER = 7


def nms_long_after(schedule: str = "flooding", u: int = 1) -> int:
    """Iterations within which FP32 min-sum is held to 1e-4 against FP64."""
    if schedule == "flooding" or u <= 1:
        return NMS_LONG_AFTER
    return 5 if u == 2 else 3
# FP32 holds a check message of size up to C = 20 only to 20 * 2^-24 = 1.2e-6;
# a soft decision adds up to ~16 of them, so where they cancel to a small
# |L| its FP32 value is good to about 1e-5 absolute, not 1e-4 relative.
ATOL32 = 1e-5
_SCHEDULES = {"flooding": oracle.FLOODING, "serial": oracle.SERIAL}
_COUPLINGS = {"joint": oracle.JOINT, "independent": oracle.INDEPENDENT}


def gpu_run(ctx, dcode, frames, algo, dtype, max_iter, early_exit=True, alpha=0.75,
            clip=20.0, llr=None, schedule="flooding", coupling="joint", compact=True, msg="f32"):
    import torch
    from paper_2001_07979_amd import mbp
    dev = torch.device("cuda", ctx.device)
    y = torch.from_numpy(frames.y).to(dev)
    e = torch.from_numpy(frames.p.astype(np.float64)).to(dev)
    if llr is None:
        llr = mbp.llr_from_bits(ctx, y, e, dtype=dtype)
    else:
        llr = torch.from_numpy(llr).to(dev)
    z = torch.from_numpy(frames.z).to(dev)
    out = mbp.decode(ctx, dcode, llr, z, algo=algo, max_iter=max_iter, early_exit=early_exit,
                     alpha=alpha, clip=clip, schedule=schedule, coupling=coupling, compact=compact, msg=msg)
    torch.cuda.synchronize()
    return dict(llr_in=llr.cpu().numpy(), bits=out["bits"].cpu().numpy(),
                iters=out["iters"].cpu().numpy(), ok=out["ok"].cpu().numpy(),
                L=out["llr"].cpu().numpy().astype(np.float64))


def oracle_llr(frames, dtype):
    lam = oracle.llr_from_bits(frames.y, frames.p)
    if dtype == "f32":
        lam = lam.astype(np.float32).astype(np.float64)
    return lam


def oracle_run(code, frames, algo, dtype, max_iter, early_exit=True, alpha=0.75, clip=20.0,
               idx=None, lam=None, schedule="flooding", coupling="joint", msg="f32"):
    if lam is None:
        lam = oracle_llr(frames, dtype)
    z = frames.z
    if idx is not None:
        lam, z = lam[idx], z[idx]
    r = oracle.decode(code, lam, z, algo=oracle.SPA if algo == "spa" else oracle.NMS,
                      max_iter=max_iter, early_exit=early_exit, alpha=alpha, clip=clip,
                      schedule=_SCHEDULES[schedule], coupling=_COUPLINGS[coupling], msg_half=msg == "f16")
    r["llr_in"] = lam
    return r


def compare(gpu, orc, max_iter, rtol, idx=None, exact_all=False, atol=0.0, long_after=None,
            long_rtol=None, long_budget=0.05):
    """Apply the protocol; returns a summary dict, raising AssertionError on a bug.

    long_after=None: every strict frame is held to rtol. long_after=t with a
    long_rtol: strict frames that stop after t iterations are held to
    long_rtol instead. long_after=t with long_rtol=None: those frames are
    counted against FP64 (long_mismatch, at most long_budget of the frames),
    for FP32 min-sum runs whose tests hold them bit for bit to the binary32
    oracle.
    """
    sel = (lambda a: a[idx]) if idx is not None else (lambda a: a)
    g = {k: sel(v) for k, v in gpu.items() if k != "llr_in"}
    F = len(orc["ok"])
    summary = dict(frames=F, oracle_ok=int(orc["ok"].sum()), flagged=int(orc["flag"].sum()),
                   flagged_mismatch=0, failed_mismatch=0, long_mismatch=0, max_rel=0.0,
                   max_rel_long=0.0, hamming_failed=[])
    for f in range(F):
        o_ok, o_it = int(orc["ok"][f]), int(orc["iters"][f])
        g_ok, g_it = int(g["ok"][f]), int(g["iters"][f])
        same_bits = np.array_equal(orc["bits"][f], g["bits"][f])
        same = g_ok == o_ok and g_it == o_it and same_bits
        long = long_after is not None and o_it > long_after and not exact_all
        if long and long_rtol is None:
            # FP32 min-sum past long_after: a disagreement with FP64 (a decode
            # the oracle completes that differs, or one it fails that the GPU
            # completes or stops early) is counted
            summary["long_mismatch"] += int(not same if o_ok else (g_ok or g_it != max_iter))
            continue
        strict = exact_all or (o_ok and not orc["flag"][f])
        if strict:
            assert g_ok == o_ok and g_it == o_it, (
                f"frame {f}: gpu ok={g_ok} iters={g_it}, oracle ok={o_ok} iters={o_it}")
            assert same_bits, f"frame {f}: {int((orc['bits'][f] != g['bits'][f]).sum())} bits differ"
            Lo, Lg = orc["L"][f], g["L"][f]
            tol = long_rtol if long else rtol
            mask = np.abs(Lo) >= SMALL
            err = np.abs(Lg[mask] - Lo[mask])
            rel = err / np.abs(Lo[mask])
            if rel.size:
                key = "max_rel_long" if long else "max_rel"
                summary[key] = max(summary[key], float(rel.max()))
                k = int(np.argmax(err - tol * np.abs(Lo[mask])))
                Lo_k, Lg_k = Lo[mask][k], Lg[mask][k]
                assert np.all(err <= tol * np.abs(Lo[mask]) + atol), (
                    f"frame {f} (iters {o_it}): L differs by {rel.max():.3g} relative at "
                    f"L={Lo_k:.6g} (gpu {Lg_k:.6g}, abs {abs(Lg_k - Lo_k):.3g}); "
                    f"median rel {np.median(rel):.3g}, 99th pct {np.percentile(rel, 99):.3g}, "
                    f"max |L| {np.abs(Lo).max():.4g}")
        elif not o_ok:
            if g_ok or g_it != max_iter:
                summary["failed_mismatch"] += 1
            summary["hamming_failed"].append(int((orc["bits"][f] != g["bits"][f]).sum()))
        else:
            summary["flagged_mismatch"] += int(not same)
    bad = summary["flagged_mismatch"] + summary["failed_mismatch"]
    assert bad <= 0.01 * F, f"{bad} of {F} frames disagree: {summary}"
    assert summary["long_mismatch"] <= long_budget * F, (
        f"{summary['long_mismatch']} of {F} long min-sum decodes disagree with FP64: {summary}")
    return summary


def oracle_f32_run(code, frames, max_iter, early_exit=True, alpha=0.75, clip=20.0, idx=None,
                   lam=None, schedule="flooding", coupling="joint", msg="f32"):
    if lam is None:
        lam = oracle_llr(frames, "f32")
    z = frames.z
    if idx is not None:
        lam, z = lam[idx], z[idx]
    return oracle.decode_nms_f32(code, lam, z, max_iter=max_iter, early_exit=early_exit,
                                 alpha=alpha, clip=clip, schedule=_SCHEDULES[schedule],
                                 coupling=_COUPLINGS[coupling], msg_half=msg == "f16")


def assert_bitwise(gpu, ref, idx=None):
    """GPU outputs equal to a reference bit for bit (bits, iters, ok, L)."""
    sel = (lambda a: a[idx]) if idx is not None else (lambda a: a)
    for k in ("bits", "iters", "ok", "L"):
        a, b = sel(gpu[k]), ref[k]
        if not np.array_equal(a, b):
            bad = np.nonzero(np.any((a != b).reshape(a.shape[0], -1), axis=1))[0]
            raise AssertionError(f"{k} differs on frames {bad[:10].tolist()} ({bad.size} in all)")
