"""Python binding of the MBP decoder library (``libmbp.so``, ``include/mbp.h``).

Argument marshalling only: every step of a decode runs in the library's HIP
kernels. Device buffers are torch tensors on the GPU (PyTorch provides the
device memory and the stream); results come back as torch tensors.
The binding fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbp.so")

MBP_OK = 0
MBP_EINVAL, MBP_ENOMEM, MBP_EDEVICE, MBP_ESTATE, MBP_EUNSUPPORTED = -1, -2, -3, -4, -5
MBP_ALGO_SPA, MBP_ALGO_NMS = 0, 1
MBP_F32, MBP_F64 = 0, 1
KERNEL_IDS = {"check": 0, "variable": 1, "syndrome": 2, "staging": 3}

_lib = None


class MbpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class mbp_params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("early_exit", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("llr_clip", ctypes.c_double)]


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        sig = {
            "mbp_last_error": (ctypes.c_char_p, []),
            "mbp_version": (i32, []),
            "mbp_ctx_create": (ctypes.c_int, [i32, ctypes.POINTER(vp)]),
            "mbp_ctx_destroy": (None, [vp]),
            "mbp_code_create": (ctypes.c_int, [vp, i32, i32, vp, vp, vp, ctypes.POINTER(vp)]),
            "mbp_code_destroy": (None, [vp]),
            "mbp_code_info": (ctypes.c_int, [vp] + [vp] * 6),
            "mbp_llr_from_bits": (ctypes.c_int, [vp, i32, i32, vp, vp, i32, vp, vp]),
            "mbp_decode": (ctypes.c_int, [vp, vp, ctypes.POINTER(mbp_params), i32] + [vp] * 7),
            "mbp_profile_enable": (ctypes.c_int, [vp, i32]),
            "mbp_profile_reset": (ctypes.c_int, [vp]),
            "mbp_profile_get": (ctypes.c_int, [vp, i32, ctypes.POINTER(i64),
                                               ctypes.POINTER(ctypes.c_double)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().mbp_last_error().decode()


def _check(rc: int, what: str):
    if rc != MBP_OK:
        raise MbpError(rc, f"{what}: {last_error()}")


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev_ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Context:
    """A decoder context on one GPU (owns the decode workspace)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().mbp_ctx_create(int(device), ctypes.byref(h)), "mbp_ctx_create")
        self.handle = h
        self.device = int(device)

    def close(self):
        if self.handle:
            lib().mbp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile_enable(self, on: bool = True):
        _check(lib().mbp_profile_enable(self.handle, int(bool(on))), "mbp_profile_enable")

    def profile_reset(self):
        _check(lib().mbp_profile_reset(self.handle), "mbp_profile_reset")

    def profile_get(self, kernel: str):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(lib().mbp_profile_get(self.handle, KERNEL_IDS[kernel], ctypes.byref(n),
                                     ctypes.byref(ms)), "mbp_profile_get")
        return int(n.value), float(ms.value)


class Code:
    """u parity-check matrices uploaded to the device (mbp_code_create)."""

    def __init__(self, ctx: Context, n: int, row_ptr: Sequence[np.ndarray],
                 col_idx: Sequence[np.ndarray]):
        u = len(row_ptr)
        rps = [np.ascontiguousarray(r, dtype=np.int32) for r in row_ptr]
        cis = [np.ascontiguousarray(c, dtype=np.int32) for c in col_idx]
        m = np.array([r.size - 1 for r in rps], dtype=np.int32)
        rp_arr = (ctypes.c_void_p * u)(*[r.ctypes.data for r in rps])
        ci_arr = (ctypes.c_void_p * u)(*[c.ctypes.data for c in cis])
        h = ctypes.c_void_p()
        _check(lib().mbp_code_create(ctx.handle, int(n), u, m.ctypes.data,
                                     ctypes.cast(rp_arr, ctypes.c_void_p),
                                     ctypes.cast(ci_arr, ctypes.c_void_p), ctypes.byref(h)),
               "mbp_code_create")
        self.ctx = ctx
        self.handle = h
        self.n, self.u, self.m = int(n), u, m.tolist()
        self.M = int(m.sum())
        info = self.info()
        self.E, self.max_check_deg, self.max_var_deg = info["E"], info["max_check_deg"], info["max_var_deg"]

    @classmethod
    def from_inputs(cls, ctx: Context, code) -> "Code":
        return cls(ctx, code.n, code.row_ptr, code.col_idx)

    def info(self) -> dict:
        n, u, M = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        E = ctypes.c_int64()
        dc, dv = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().mbp_code_info(self.handle, *(ctypes.addressof(x) for x in (n, u, M, E, dc, dv))),
               "mbp_code_info")
        return dict(n=n.value, u=u.value, M=M.value, E=E.value, max_check_deg=dc.value,
                    max_var_deg=dv.value)

    def close(self):
        if self.handle:
            lib().mbp_code_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dtype_code(dtype) -> int:
    import torch
    if dtype in (torch.float32, "f32", "float32", MBP_F32):
        return MBP_F32
    if dtype in (torch.float64, "f64", "float64", MBP_F64):
        return MBP_F64
    raise ValueError(f"unsupported dtype {dtype}")


def _torch_dtype(code: int):
    import torch
    return torch.float32 if code == MBP_F32 else torch.float64


def llr_from_bits(ctx: Context, y, e, dtype="f32", out=None, stream=None):
    """Channel LLRs (1-2y) ln((1-e)/e) of Bob's bits y [F, n] (uint8, GPU) and
    per-frame error rates e [F] (float64, GPU)."""
    import torch
    dt = _dtype_code(dtype)
    F, n = y.shape
    if out is None:
        out = torch.empty((F, n), dtype=_torch_dtype(dt), device=y.device)
    _check(lib().mbp_llr_from_bits(ctx.handle, F, n, _dev_ptr(y), _dev_ptr(e), dt, _dev_ptr(out),
                                   _stream_ptr(stream)), "mbp_llr_from_bits")
    return out


def decode(ctx: Context, code: Code, llr, synd, algo: str = "spa", max_iter: int = 50,
           early_exit: bool = True, alpha: float = 0.75, clip: float = 20.0,
           want_llr: bool = True, out: Optional[dict] = None, stream=None) -> dict:
    """Decode every frame: llr [F, n] (float32/float64, GPU), synd [F, M] (uint8, GPU).

    Returns dict(bits [F, n] uint8, iters [F] int32, ok [F] uint8, llr [F, n] or None).
    """
    import torch
    dt = _dtype_code(llr.dtype)
    F = int(llr.shape[0])
    if llr.shape[1] != code.n or tuple(synd.shape) != (F, code.M):
        raise ValueError("llr must be [F, n] and synd [F, M]")
    if not (llr.is_contiguous() and synd.is_contiguous()):
        raise ValueError("llr and synd must be contiguous")
    if synd.dtype != torch.uint8:
        raise ValueError("synd must be uint8")
    dev = llr.device
    if out is None:
        out = dict(bits=torch.empty((F, code.n), dtype=torch.uint8, device=dev),
                   iters=torch.empty(F, dtype=torch.int32, device=dev),
                   ok=torch.empty(F, dtype=torch.uint8, device=dev),
                   llr=torch.empty((F, code.n), dtype=llr.dtype, device=dev) if want_llr else None)
    p = mbp_params(MBP_ALGO_SPA if algo == "spa" else MBP_ALGO_NMS, dt, int(max_iter),
                   int(bool(early_exit)), float(alpha), float(clip))
    _check(lib().mbp_decode(ctx.handle, code.handle, ctypes.byref(p), F, _dev_ptr(llr),
                            _dev_ptr(synd), _dev_ptr(out["bits"]), _dev_ptr(out["iters"]),
                            _dev_ptr(out["ok"]), _dev_ptr(out.get("llr")), _stream_ptr(stream)),
           "mbp_decode")
    return out
