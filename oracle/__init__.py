"""FP64 CPU oracle for multi-matrix syndrome BP — test infrastructure only.

Thin ctypes wrapper over ``liboracle.so`` (built from ``mbp_oracle.c`` by
``__graft_entry__.build()``). Only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it; the decoder never does.

A code is any object with ``n``, ``row_ptr`` (list of u int32 arrays) and
``col_idx`` (list of u int32 arrays), e.g. the input generator's ``Code``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

SPA, NMS = 0, 1


class _Code(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("u", ctypes.c_int32),
                ("m", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("early_exit", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("clip", ctypes.c_double), ("alpha_tl", ctypes.c_void_p),
                ("margin", ctypes.c_double), ("schedule", ctypes.c_int32),
                ("coupling", ctypes.c_int32), ("msg_half", ctypes.c_int32)]

FLOODING, SERIAL = 0, 1  # schedules: flooding, matrix-serial
JOINT, INDEPENDENT = 0, 1  # how the u matrices combine: one stacked graph, or u decoders joined by eq. (2)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(_LIB_PATH)
        L.oracle_binary_entropy.restype = ctypes.c_double
        L.oracle_binary_entropy.argtypes = [ctypes.c_double]
        L.oracle_efficiency.restype = ctypes.c_double
        L.oracle_efficiency.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double]
        L.oracle_llr_from_bits.restype = None
        L.oracle_llr_from_bits.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                           ctypes.c_void_p]
        L.oracle_mbp_decode.restype = ctypes.c_int32
        L.oracle_mbp_decode.argtypes = [ctypes.POINTER(_Code), ctypes.POINTER(_Params),
                                        ctypes.c_int32] + [ctypes.c_void_p] * 7 + [ctypes.c_int32]
        L.oracle_mbp_decode_nms_f32.restype = ctypes.c_int32
        L.oracle_mbp_decode_nms_f32.argtypes = [ctypes.POINTER(_Code), ctypes.POINTER(_Params),
                                                ctypes.c_int32] + [ctypes.c_void_p] * 6 + [ctypes.c_int32]
        L.oracle_syndrome.restype = ctypes.c_int32
        L.oracle_syndrome.argtypes = [ctypes.POINTER(_Code), ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p]
        L.oracle_unsatisfied.restype = ctypes.c_int32
        L.oracle_unsatisfied.argtypes = [ctypes.POINTER(_Code), ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_nms_unrolled.restype = ctypes.c_int32
        L.oracle_nms_unrolled.argtypes = [ctypes.POINTER(_Code), ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_double, ctypes.c_int32] + [ctypes.c_void_p] * 6 \
            + [ctypes.c_int32]
        L.oracle_default_threads.restype = ctypes.c_int32
        L.oracle_default_threads.argtypes = []
        L.oracle_round_binary16.restype = ctypes.c_double
        L.oracle_round_binary16.argtypes = [ctypes.c_double]
        _lib = L
    return _lib


def _pack(code):
    m = np.array([int(r.size - 1) for r in code.row_ptr], dtype=np.int32)
    rp = np.ascontiguousarray(np.concatenate([np.asarray(r, np.int32) for r in code.row_ptr]))
    ci = np.ascontiguousarray(np.concatenate([np.asarray(c, np.int32) for c in code.col_idx]))
    keep = (m, rp, ci)
    s = _Code(int(code.n), int(m.size), m.ctypes.data, rp.ctypes.data, ci.ctypes.data)
    return s, keep


def binary_entropy(e: float) -> float:
    return float(lib().oracle_binary_entropy(float(e)))


def efficiency(m: int, n: int, e: float) -> float:
    return float(lib().oracle_efficiency(int(m), int(n), float(e)))


def default_threads() -> int:
    return int(lib().oracle_default_threads())


def round_binary16(x: float) -> float:
    """The binary16 value nearest to x (ties to even), as the decode's
    msg_half option stores check messages."""
    return float(lib().oracle_round_binary16(float(x)))


def llr_from_bits(y: np.ndarray, e) -> np.ndarray:
    """Channel LLRs [F, n] (FP64) from Bob's bits [F, n] and per-frame error rate."""
    y = np.ascontiguousarray(np.atleast_2d(y), dtype=np.uint8)
    F, n = y.shape
    e = np.broadcast_to(np.asarray(e, dtype=np.float64), (F,))
    out = np.empty((F, n), dtype=np.float64)
    for f in range(F):
        lib().oracle_llr_from_bits(y[f].ctypes.data, n, float(e[f]), out[f].ctypes.data)
    return out


def decode(code, llr: np.ndarray, synd: np.ndarray, algo: int = SPA, max_iter: int = 50,
           early_exit: bool = True, alpha: float = 0.75, clip: float = 20.0,
           alpha_tl: Optional[np.ndarray] = None, margin: float = 1e-3,
           nthreads: int = 0, schedule: int = FLOODING, coupling: int = JOINT,
           msg_half: bool = False) -> dict:
    """FP64 MBP decode of every frame; returns bits, iters, ok, L, flag.
    msg_half stores every check message rounded to binary16."""
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float64)
    synd = np.ascontiguousarray(np.atleast_2d(synd), dtype=np.uint8)
    F, n = llr.shape
    assert n == code.n and synd.shape[0] == F
    cs, keep = _pack(code)
    atl = None
    if alpha_tl is not None:
        atl = np.ascontiguousarray(alpha_tl, dtype=np.float64)
        assert atl.shape == (max_iter, len(code.row_ptr))
    P = _Params(int(algo), int(max_iter), int(bool(early_exit)), float(alpha), float(clip),
                atl.ctypes.data if atl is not None else None, float(margin), int(schedule), int(coupling),
                int(bool(msg_half)))
    bits = np.zeros((F, n), dtype=np.uint8)
    iters = np.zeros(F, dtype=np.int32)
    ok = np.zeros(F, dtype=np.uint8)
    L = np.zeros((F, n), dtype=np.float64)
    flag = np.zeros(F, dtype=np.uint8)
    rc = lib().oracle_mbp_decode(ctypes.byref(cs), ctypes.byref(P), F, llr.ctypes.data,
                                 synd.ctypes.data, bits.ctypes.data, iters.ctypes.data,
                                 ok.ctypes.data, L.ctypes.data, flag.ctypes.data, int(nthreads))
    del keep
    if rc != 0:
        raise ValueError("oracle_mbp_decode rejected its input")
    return dict(bits=bits, iters=iters, ok=ok, L=L, flag=flag)


def decode_nms_f32(code, llr: np.ndarray, synd: np.ndarray, max_iter: int = 50,
                   early_exit: bool = True, alpha: float = 0.75, clip: float = 20.0,
                   alpha_tl: Optional[np.ndarray] = None, nthreads: int = 0,
                   schedule: int = FLOODING, coupling: int = JOINT, msg_half: bool = False) -> dict:
    """Normalized min-sum decode with every operation in binary32 (see the C source);
    msg_half stores every check message rounded to binary16."""
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float64)
    synd = np.ascontiguousarray(np.atleast_2d(synd), dtype=np.uint8)
    F, n = llr.shape
    assert n == code.n and synd.shape[0] == F
    cs, keep = _pack(code)
    atl = None
    if alpha_tl is not None:
        atl = np.ascontiguousarray(alpha_tl, dtype=np.float64)
        assert atl.shape == (max_iter, len(code.row_ptr))
    P = _Params(NMS, int(max_iter), int(bool(early_exit)), float(alpha), float(clip),
                atl.ctypes.data if atl is not None else None, 1e-3, int(schedule), int(coupling),
                int(bool(msg_half)))
    bits = np.zeros((F, n), dtype=np.uint8)
    iters = np.zeros(F, dtype=np.int32)
    ok = np.zeros(F, dtype=np.uint8)
    L = np.zeros((F, n), dtype=np.float64)
    rc = lib().oracle_mbp_decode_nms_f32(ctypes.byref(cs), ctypes.byref(P), F, llr.ctypes.data,
                                         synd.ctypes.data, bits.ctypes.data, iters.ctypes.data,
                                         ok.ctypes.data, L.ctypes.data, int(nthreads))
    del keep
    if rc != 0:
        raise ValueError("oracle_mbp_decode_nms_f32 rejected its input")
    return dict(bits=bits, iters=iters, ok=ok, L=L)


def syndrome(code, x: np.ndarray) -> np.ndarray:
    """Eq. (1): the stacked syndromes [H_1 x; ...; H_u x] mod 2 of each frame."""
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.uint8)
    cs, keep = _pack(code)
    z = np.zeros((x.shape[0], int(sum(code.m))), dtype=np.uint8)
    rc = lib().oracle_syndrome(ctypes.byref(cs), x.shape[0], x.ctypes.data, z.ctypes.data)
    del keep
    if rc != 0:
        raise ValueError("oracle_syndrome rejected its input")
    return z


def unsatisfied(code, x: np.ndarray, synd: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.uint8)
    synd = np.ascontiguousarray(np.atleast_2d(synd), dtype=np.uint8)
    cs, keep = _pack(code)
    w = np.zeros(x.shape[0], dtype=np.int32)
    rc = lib().oracle_unsatisfied(ctypes.byref(cs), x.shape[0], x.ctypes.data,
                                  synd.ctypes.data, w.ctypes.data)
    del keep
    if rc != 0:
        raise ValueError("oracle_unsatisfied rejected its input")
    return w


def nms_unrolled(code, K: int, alpha: np.ndarray, llr: np.ndarray, synd: np.ndarray,
                 clip: float = 20.0, gL: Optional[np.ndarray] = None, binary32: bool = False):
    """Unrolled min-sum: L^K, and with gL = dJ/dL^K also (dJ/dllr, dJ/dalpha).

    binary32=True runs the forward in float arithmetic and differentiates
    that trajectory (the reverse sweep itself stays FP64)."""
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float64)
    synd = np.ascontiguousarray(np.atleast_2d(synd), dtype=np.uint8)
    F, n = llr.shape
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    assert alpha.shape == (K, len(code.row_ptr))
    cs, keep = _pack(code)
    Lout = np.zeros((F, n), dtype=np.float64)
    glam = galpha = None
    gptr = None
    if gL is not None:
        gL = np.ascontiguousarray(np.atleast_2d(gL), dtype=np.float64)
        glam = np.zeros((F, n), dtype=np.float64)
        galpha = np.zeros_like(alpha)
        gptr = gL.ctypes.data
    rc = lib().oracle_nms_unrolled(ctypes.byref(cs), int(K), alpha.ctypes.data, float(clip), F,
                                   llr.ctypes.data, synd.ctypes.data, gptr, Lout.ctypes.data,
                                   glam.ctypes.data if glam is not None else None,
                                   galpha.ctypes.data if galpha is not None else None,
                                   int(bool(binary32)))
    del keep
    if rc != 0:
        raise ValueError("oracle_nms_unrolled rejected its input")
    return (Lout, glam, galpha) if gL is not None else Lout
