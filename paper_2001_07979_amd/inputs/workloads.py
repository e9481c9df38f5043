"""The decoder's workloads, built from seeded synthetic inputs.

Each one names its code (PEG matrices and degree profile), its frames (key
bits, BSC noise, syndromes) and its decoder settings. They stand in for the
paper's QKD keys and PEG matrices (Sec. 3A splits a 2^20-bit sifted key into
frames of n bits; Sec. 4 runs rates 0.5-0.8 at efficiency 1.1-1.4), neither of
which is published.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import Code, Frames, bsc_frames, peg_code

IRREGULAR_238 = {2: 0.25, 3: 0.45, 8: 0.30}
IRREGULAR_2310 = {2: 0.25, 3: 0.45, 10: 0.30}


def peg_depth(n: int) -> int:
    """Breadth-first depth bound of the PEG construction (-1 = none)."""
    if n <= 8192:
        return -1
    if n <= 65536:
        return 2
    return 1


@dataclass
class Workload:
    name: str
    code: Code
    nframes: int
    p: object
    seed: int
    algo: str
    dtype: str
    max_iter: int
    early_exit: bool = True
    alpha: float = 0.75
    clip: float = 20.0
    meta: dict = field(default_factory=dict)

    def frames(self, nframes: int | None = None) -> Frames:
        return bsc_frames(self.code, nframes or self.nframes, self.p, self.seed)


def fp64_n4096(nframes: int = 16) -> Workload:
    """u=2 regular (3,6) PEG matrices, n=4096, rate 1/2, BSC 0.05, FP64 sum-product."""
    code = peg_code(4096, 2048, 2, {3: 1.0}, seed_base=1000, max_depth=peg_depth(4096),
                    name="peg-n4096-r050-u2-dv3")
    return Workload("mbp-spa-f64-n4096-u2-p0.05", code, nframes, 0.05, 1, "spa", "f64", 50)


def qkd_n65536(nframes: int = 256, algo: str = "spa") -> Workload:
    """u=2 irregular {2,3,8} PEG matrices, n=65536, rate 3/4, BSC 0.02, FP32."""
    code = peg_code(65536, 16384, 2, IRREGULAR_238, seed_base=2000,
                    max_depth=peg_depth(65536), name="peg-n65536-r075-u2-d238")
    return Workload(f"mbp-{algo}-f32-n65536-r075-u2-p0.02", code, nframes, 0.02, 2, algo,
                    "f32", 100)


QKD_262K_POINTS = {0.5: 0.08, 0.7: 0.04, 0.85: 0.02}


def qkd_n262144(rate: float, nframes: int = 64, algo: str = "spa") -> Workload:
    """u=3 irregular {2,3,10} PEG matrices, n=2^18, one of three (rate, p) points."""
    n = 262144
    m = int(round((1.0 - rate) * n))
    p = QKD_262K_POINTS[rate]
    code = peg_code(n, m, 3, IRREGULAR_2310, seed_base=3000 + int(round(rate * 100)),
                    max_depth=peg_depth(n), name=f"peg-n262144-r{rate}-u3-d2310")
    return Workload(f"mbp-{algo}-f32-n262144-r{rate}-u3-p{p}", code, nframes, p, 3, algo,
                    "f32", 100)


def unrolled_n16384(nframes: int = 512) -> Workload:
    """u=2 irregular {2,3,8} PEG matrices, n=16384, rate 1/2, BSC p ~ U[0.04, 0.08]."""
    code = peg_code(16384, 8192, 2, IRREGULAR_238, seed_base=5000, max_depth=peg_depth(16384),
                    name="peg-n16384-r050-u2-d238")
    p = np.random.default_rng(5).uniform(0.04, 0.08, size=nframes)
    return Workload("mbp-nms-unrolled-k20-n16384-u2", code, nframes, p, 5, "nms", "f32", 20,
                    early_exit=False)


MIXED_N = (16384, 65536, 262144)
MIXED_RATES = (0.5, 0.7, 0.85)


def mixed_code(n: int, rate: float, u: int) -> Code:
    """Code of one cell of the mixed queue: the first u of three {2,3,10} PEG
    matrices of that (n, rate), so u=2 and u=3 frames share matrices."""
    m = int(round((1.0 - rate) * n))
    depth = 2 if n <= 16384 else 1
    full = peg_code(n, m, 3, IRREGULAR_2310, seed_base=4000 + 10 * MIXED_N.index(n)
                    + MIXED_RATES.index(rate) * 100, max_depth=depth,
                    name=f"peg-n{n}-r{rate}-u3-d2310")
    return Code(n=n, row_ptr=full.row_ptr[:u], col_idx=full.col_idx[:u],
                name=f"peg-n{n}-r{rate}-u{u}-d2310", meta=dict(full.meta, u=u))


@dataclass
class QueueFrame:
    cell: tuple  # (n, rate, u)
    p: float
    arrival_s: float


def mixed_queue(nframes: int = 2048, seed: int = 4, rate_fps: float = None):
    """Frame list of the heterogeneous queue: n, rate and u drawn uniformly,
    BSC p log-uniform in [0.01, 0.08], Poisson arrivals (rate_fps frames per
    second; None puts every arrival at t = 0)."""
    rng = np.random.default_rng(seed)
    cells = [(n, r, u) for n in MIXED_N for r in MIXED_RATES for u in (2, 3)]
    pick = rng.integers(0, len(cells), nframes)
    p = np.exp(rng.uniform(np.log(0.01), np.log(0.08), nframes))
    if rate_fps:
        t = np.cumsum(rng.exponential(1.0 / rate_fps, nframes))
    else:
        t = np.zeros(nframes)
    return [QueueFrame(cells[k], float(pp), float(tt)) for k, pp, tt in zip(pick, p, t)]


def queue_frames(queue, seed: int = 4):
    """The queue's frames grouped by cell, each group in arrival order:
    {cell: (code, queue indices, Frames)}.  A cell draws its frames from
    SeedSequence(1000 * seed + cell index)."""
    cells = sorted({q.cell for q in queue})
    out = {}
    for k, cell in enumerate(cells):
        idx = np.array([i for i, q in enumerate(queue) if q.cell == cell], dtype=np.int64)
        code = mixed_code(*cell)
        p = np.array([queue[i].p for i in idx])
        out[cell] = (code, idx, bsc_frames(code, len(idx), p, 1000 * seed + k))
    return out


# ------------------------------------------------------------------- sweeps
# The axes of the paper's experiments (Sec. 4, Figs. 2-3, Table 3): the number
# of matrices u, the error rate e and the code rate R, on n = 65536 frames of
# {2,3,10} PEG matrices. The codes for u = 1, 2, 3 at one rate share their
# matrices (u takes the first u of three).
SWEEP_N = 65536
SWEEP_RATES = (0.5, 0.6, 0.7, 0.8)


def sweep_code(rate: float, u: int):
    n = SWEEP_N
    m = int(round((1.0 - rate) * n))
    return peg_code(n, m, u, IRREGULAR_2310, seed_base=6000 + 10 * int(round(rate * 10)),
                    max_depth=peg_depth(n), name=f"peg-n{n}-r{rate}-u{u}-d2310")


def binary_entropy(e: float) -> float:
    return float(-e * np.log2(e) - (1 - e) * np.log2(1 - e))


def e_for_efficiency(rate: float, f: float) -> float:
    """The BSC error rate e <= 1/2 at which f = m / (n h(e)) (eq. (3), m of
    one matrix) equals f for a code of rate R = 1 - m/n: h(e) = (1 - R)/f,
    solved by bisection."""
    target = (1.0 - rate) / f
    lo, hi = 1e-12, 0.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if binary_entropy(mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def sweep_workload(rate: float, u: int, e: float, nframes: int = 256, algo: str = "spa") -> Workload:
    code = sweep_code(rate, u)
    return Workload(f"mbp-{algo}-f32-n{SWEEP_N}-r{rate}-u{u}-p{e:.4f}", code, nframes, float(e),
                    7000 + int(round(e * 1e4)), algo, "f32", 100, meta=dict(rate=rate, u=u))
