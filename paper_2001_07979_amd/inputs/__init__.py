"""Seeded synthetic inputs for multi-matrix syndrome BP decoding.

This module draws what a decode is run on, and nothing else:

* the u parity-check matrices, built by progressive edge growth (PEG) as the
  paper does (Sec. 2) from a degree profile and a seed;
* per frame, Alice's key x (iid uniform bits), Bob's key y = x xor BSC(p)
  noise, and Alice's u syndromes z^l = H_l x mod 2 (Sec. 2, eq. (1)).

It holds none of the decoder's arithmetic (no LLRs, no message updates, no
stopping rule); the GPU path and the CPU oracle each compute those on their
own from these inputs.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_PEG_LIB = os.path.join(_HERE, "libpeg.so")
_REPO = os.path.dirname(os.path.dirname(_HERE))
CACHE_DIR = os.environ.get("MBP_PEG_CACHE", os.path.join(_REPO, ".cache", "peg"))

_peg = None


def _peg_lib():
    global _peg
    if _peg is None:
        if not os.path.exists(_PEG_LIB):
            raise RuntimeError(
                f"{_PEG_LIB} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(_PEG_LIB)
        lib.peg_build.restype = ctypes.c_int
        lib.peg_build.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        _peg = lib
    return _peg


def degree_sequence(n: int, m: int, fractions: Dict[int, float]) -> np.ndarray:
    """Variable degrees, non-decreasing, from degree -> node-fraction.

    Counts are rounded by largest remainder so they sum to n. Degree-2 nodes
    are capped at m-1 (more of them would close a cycle made only of degree-2
    nodes); the excess moves to the next degree up.
    """
    degs = sorted(fractions)
    raw = np.array([fractions[d] * n for d in degs], dtype=np.float64)
    cnt = np.floor(raw).astype(np.int64)
    short = n - int(cnt.sum())
    order = np.argsort(-(raw - cnt), kind="stable")
    for k in range(short):
        cnt[order[k % len(degs)]] += 1
    counts = dict(zip(degs, (int(c) for c in cnt)))
    if 2 in counts and counts[2] > m - 1:
        spill = counts[2] - (m - 1)
        counts[2] = m - 1
        up = [d for d in degs if d > 2]
        if not up:
            raise ValueError("degree-2 cap needs a higher degree class")
        counts[up[0]] += spill
    seq = np.concatenate([np.full(counts[d], d, dtype=np.int32) for d in degs])
    assert seq.size == n
    return seq


def peg_matrix(n: int, m: int, var_deg: np.ndarray, seed: int,
               max_depth: int = -1, cache: bool = True):
    """CSR (row_ptr[m+1], col_idx[E]) of an m x n PEG matrix.

    Results are cached on disk under CACHE_DIR, keyed by every argument.
    """
    var_deg = np.ascontiguousarray(var_deg, dtype=np.int32)
    key = hashlib.sha1(
        var_deg.tobytes() + f"|{n}|{m}|{seed}|{max_depth}|peg1".encode()).hexdigest()[:20]
    path = os.path.join(CACHE_DIR, f"peg_n{n}_m{m}_s{seed}_d{max_depth}_{key}.npz")
    if cache and os.path.exists(path):
        with np.load(path, allow_pickle=False) as f:
            return f["row_ptr"].copy(), f["col_idx"].copy()
    E = int(var_deg.sum())
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    col_idx = np.zeros(E, dtype=np.int32)
    rc = _peg_lib().peg_build(n, m, var_deg.ctypes.data, ctypes.c_uint64(seed),
                              int(max_depth), row_ptr.ctypes.data, col_idx.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"peg_build failed with code {rc}")
    if cache:
        os.makedirs(CACHE_DIR, exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, row_ptr=row_ptr, col_idx=col_idx)
        os.replace(tmp, path)
    return row_ptr, col_idx


@dataclass
class Code:
    """u sparse parity-check matrices H_1..H_u over the same n key bits."""

    n: int
    row_ptr: List[np.ndarray]
    col_idx: List[np.ndarray]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def u(self) -> int:
        return len(self.row_ptr)

    @property
    def m(self) -> List[int]:
        return [int(r.size - 1) for r in self.row_ptr]

    @property
    def M(self) -> int:
        return sum(self.m)

    @property
    def E(self) -> int:
        return sum(int(c.size) for c in self.col_idx)

    def stacked(self):
        """CSR of the stacked (sum m_l) x n matrix [H_1; ...; H_u]."""
        ptrs, off = [], 0
        for l, rp in enumerate(self.row_ptr):
            ptrs.append((rp[:-1] if l < self.u - 1 else rp) + off)
            off += int(rp[-1])
        return np.concatenate(ptrs).astype(np.int32), np.concatenate(self.col_idx).astype(np.int32)

    def dense(self, l: Optional[int] = None) -> np.ndarray:
        """Dense 0/1 matrix (small codes only): H_l, or the stack if l is None."""
        rp, ci = (self.row_ptr[l], self.col_idx[l]) if l is not None else self.stacked()
        H = np.zeros((rp.size - 1, self.n), dtype=np.uint8)
        for j in range(rp.size - 1):
            H[j, ci[rp[j]:rp[j + 1]]] = 1
        return H


def peg_code(n: int, m: int, u: int, fractions: Dict[int, float], seed_base: int,
             max_depth: int = -1, name: str = "") -> Code:
    """u PEG matrices with one degree profile; matrix l uses seed seed_base + l.

    Every matrix gives variable i the same degree (PEG takes variables in
    ascending degree order), so the stacked variable degree is u times it.
    """
    dv = degree_sequence(n, m, fractions)
    rps, cis = [], []
    for l in range(u):
        rp, ci = peg_matrix(n, m, dv, seed_base + l, max_depth)
        rps.append(rp)
        cis.append(ci)
    return Code(n=n, row_ptr=rps, col_idx=cis, name=name,
                meta=dict(m=m, u=u, fractions=dict(fractions), seed_base=seed_base,
                          max_depth=max_depth))


def code_from_dense(Hs: Sequence[np.ndarray], name: str = "") -> Code:
    """Code from dense 0/1 matrices (tests and tiny examples)."""
    n = int(Hs[0].shape[1])
    rps, cis = [], []
    for H in Hs:
        H = np.asarray(H, dtype=np.uint8)
        assert H.shape[1] == n
        rp = np.zeros(H.shape[0] + 1, dtype=np.int32)
        cols = []
        for j in range(H.shape[0]):
            c = np.nonzero(H[j])[0].astype(np.int32)
            cols.append(c)
            rp[j + 1] = rp[j] + c.size
        rps.append(rp)
        cis.append(np.concatenate(cols) if cols else np.zeros(0, np.int32))
    return Code(n=n, row_ptr=rps, col_idx=cis, name=name)


def syndromes(code: Code, x: np.ndarray) -> np.ndarray:
    """Alice's syndromes z = [H_1 x; ...; H_u x] mod 2, eq. (1); x is [F, n]."""
    x = np.atleast_2d(np.asarray(x, dtype=np.uint8))
    out = []
    for rp, ci in zip(code.row_ptr, code.col_idx):
        starts = rp[:-1]
        nonempty = rp[1:] > starts
        s = np.zeros((x.shape[0], rp.size - 1), dtype=np.uint8)
        if ci.size:
            at = np.minimum(starts, ci.size - 1)
            for f in range(x.shape[0]):  # one row at a time: contiguous gathers
                s[f, nonempty] = np.bitwise_xor.reduceat(x[f].take(ci), at)[nonempty]
        out.append(s)
    return np.concatenate(out, axis=1)


@dataclass
class Frames:
    """A batch of key frames: Alice's x, Bob's y, the syndromes z, BSC p."""

    x: np.ndarray  # [F, n] uint8
    y: np.ndarray  # [F, n] uint8
    z: np.ndarray  # [F, M] uint8
    p: np.ndarray  # [F] float64

    @property
    def nframes(self) -> int:
        return int(self.x.shape[0])


def bsc_frames(code: Code, nframes: int, p, seed: int) -> Frames:
    """nframes frames: x ~ iid Bernoulli(1/2), y = x xor Bernoulli(p_f) noise.

    Frame f draws its key and its noise from two separate child streams of
    SeedSequence(seed), so a frame does not depend on the batch size.
    """
    n = code.n
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), (nframes,)).copy()
    x = np.empty((nframes, n), dtype=np.uint8)
    y = np.empty((nframes, n), dtype=np.uint8)
    children = np.random.SeedSequence(seed).spawn(nframes)
    for f, ss in enumerate(children):
        kss, nss = ss.spawn(2)
        x[f] = np.random.Generator(np.random.PCG64(kss)).integers(0, 2, n, dtype=np.uint8)
        noise = np.random.Generator(np.random.PCG64(nss)).random(n) < p[f]
        y[f] = x[f] ^ noise.astype(np.uint8)
    z = syndromes(code, x)
    return Frames(x=x, y=y, z=z, p=p)
