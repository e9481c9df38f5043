"""Python binding of the MBP decoder library (``libmbp.so``, ``include/mbp.h``).

Argument marshalling only: every step of a decode runs in the library's HIP
kernels. Device buffers are torch tensors on the GPU (PyTorch provides the
device memory and the stream); results come back as torch tensors.
The binding fails loudly when the library has not been built.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbp.so")

MBP_OK = 0
MBP_EINVAL, MBP_ENOMEM, MBP_EDEVICE, MBP_ESTATE, MBP_EUNSUPPORTED = -1, -2, -3, -4, -5
MBP_ALGO_SPA, MBP_ALGO_NMS = 0, 1
MBP_F32, MBP_F64 = 0, 1
MBP_FLOODING, MBP_MATRIX_SERIAL = 0, 1
MBP_JOINT, MBP_INDEPENDENT = 0, 1
MBP_MSG_F32, MBP_MSG_F16 = 0, 1
ABI_VERSION = 3  # mbp_version() of the library this binding marshals for
_COUPLINGS = {"joint": MBP_JOINT, "independent": MBP_INDEPENDENT}
_MSGS = {"f32": MBP_MSG_F32, "f16": MBP_MSG_F16}
KERNEL_IDS = {"check": 0, "variable": 1, "syndrome": 2, "staging": 3, "first": 4, "second": 5}

_lib = None


class MbpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class mbp_batch(ctypes.Structure):
    _fields_ = [("code", ctypes.c_void_p), ("nframes", ctypes.c_int32),
                ("llr", ctypes.c_void_p), ("synd", ctypes.c_void_p),
                ("bits_out", ctypes.c_void_p), ("iters_out", ctypes.c_void_p),
                ("ok_out", ctypes.c_void_p), ("llr_out", ctypes.c_void_p)]


class mbp_tuning(ctypes.Structure):
    _fields_ = [("rows_per_wave", ctypes.c_int32), ("vars_per_wave", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("compact", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class mbp_params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("early_exit", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("llr_clip", ctypes.c_double),
                ("compact", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("coupling", ctypes.c_int32), ("msg_dtype", ctypes.c_int32)]


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # torch first: the library then binds to the HIP runtime torch loaded,
        # so the process holds one runtime (loaded the other way round, torch
        # finds no GPU)
        import torch  # noqa: F401
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
            "mbp_decode_from_bits": (ctypes.c_int, [vp, vp, ctypes.POINTER(mbp_params), i32] + [vp] * 8),
            "mbp_syndrome": (ctypes.c_int, [vp, vp, i32, vp, vp, vp]),
            "mbp_syndrome_noalloc": (ctypes.c_int, [vp, vp, i32, vp, vp, vp]),
            "mbp_peg_build": (ctypes.c_int, [vp, i32, i32, i32, vp, vp, i32, vp, vp]),
            "mbp_unrolled_workspace_bytes": (ctypes.c_int, [vp, i32, i32, i32,
                                                             ctypes.POINTER(ctypes.c_uint64)]),
            "mbp_nms_unrolled_fwd": (ctypes.c_int, [vp, vp, i32, i32, i32, ctypes.c_double] + [vp] * 5
                                     + [ctypes.c_uint64, vp]),
            "mbp_nms_unrolled_bwd": (ctypes.c_int, [vp, vp, i32, i32, i32, ctypes.c_double] + [vp] * 7
                                     + [ctypes.c_uint64, vp]),
            "mbp_tuning_default": (ctypes.c_int, [ctypes.POINTER(mbp_tuning)]),
            "mbp_decode_batched": (ctypes.c_int, [vp, i32, ctypes.POINTER(mbp_batch),
                                                  ctypes.POINTER(mbp_params),
                                                  ctypes.POINTER(mbp_tuning), vp]),
            "mbp_plan_create": (ctypes.c_int, [vp, i32, ctypes.POINTER(mbp_batch),
                                               ctypes.POINTER(mbp_params), ctypes.POINTER(mbp_tuning),
                                               ctypes.POINTER(vp)]),
            "mbp_plan_launch": (ctypes.c_int, [vp, vp]),
            "mbp_plan_wait": (ctypes.c_int, [vp, vp]),
            "mbp_plan_destroy": (None, [vp]),
            "mbp_queue_create": (ctypes.c_int, [vp, ctypes.POINTER(mbp_params), ctypes.POINTER(mbp_tuning),
                                                ctypes.POINTER(vp)]),
            "mbp_queue_submit": (ctypes.c_int, [vp, i32, ctypes.POINTER(mbp_batch)]),
            "mbp_queue_flush": (ctypes.c_int, [vp, vp]),
            "mbp_queue_poll": (ctypes.c_int, [vp, ctypes.POINTER(i64)]),
            "mbp_queue_wait": (ctypes.c_int, [vp]),
            "mbp_queue_destroy": (None, [vp]),
            "mbp_autotune": (ctypes.c_int, [vp, i32, ctypes.POINTER(mbp_batch),
                                            ctypes.POINTER(mbp_params), ctypes.c_char_p,
                                            ctypes.POINTER(mbp_tuning)]),
            "mbp_profile_enable": (ctypes.c_int, [vp, i32]),
            "mbp_profile_reset": (ctypes.c_int, [vp]),
            "mbp_profile_get": (ctypes.c_int, [vp, i32, ctypes.POINTER(i64),
                                               ctypes.POINTER(ctypes.c_double)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.mbp_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {L.mbp_version()}, this binding expects "
                               f"{ABI_VERSION}: rebuild it with __graft_entry__.build()")
        _lib = L
        # library objects still open when the interpreter exits are closed
        # while the HIP runtime is still up (before C-level exit handlers)
        atexit.register(close_all)
    return _lib


# Every open Plan, Queue, Code and Context, by kind, for close_all().
_open = {kind: weakref.WeakSet() for kind in ("plan", "queue", "code", "ctx")}


def close_all():
    """Close every Plan and Queue, then every Code, then every Context that
    is still open (each close is idempotent)."""
    for kind in ("plan", "queue", "code", "ctx"):
        for obj in list(_open[kind]):
            try:
                obj.close()
            except Exception:  # noqa: BLE001 - teardown goes on with the rest
                pass


def last_error() -> str:
    return lib().mbp_last_error().decode()


def _check(rc: int, what: str):
    if rc != MBP_OK:
        raise MbpError(rc, f"{what}: {last_error()}")


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev(t, name: str, device: int, dtypes=None, shape=None, optional: bool = False) -> Optional[int]:
    """Device address of a tensor the library will read or write, after
    checking that it is a contiguous torch tensor on GPU `device` with one of
    `dtypes` and, if given, exactly `shape`. A host tensor, a tensor of
    another device or a strided view would hand the kernels an address they
    cannot use, so every such case is rejected here, before any launch."""
    import torch
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor, not {type(t).__name__}")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name} must be on cuda:{device} (it is on {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtypes is not None and t.dtype not in dtypes:
        raise ValueError(f"{name} must be {' or '.join(str(d) for d in dtypes)} (it is {t.dtype})")
    if shape is not None and tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (it has {tuple(t.shape)})")
    return t.data_ptr()


def _u8():
    import torch
    return (torch.uint8,)


def _f32():
    import torch
    return (torch.float32,)


def _f64():
    import torch
    return (torch.float64,)


def _out_ptrs(out: dict, device: int, F: int, n: int, llr_dtype) -> tuple:
    import torch
    return (_dev(out.get("bits"), "out['bits']", device, _u8(), (F, n)),
            _dev(out.get("iters"), "out['iters']", device, (torch.int32,), (F,)),
            _dev(out.get("ok"), "out['ok']", device, _u8(), (F,)),
            _dev(out.get("llr"), "out['llr']", device, (llr_dtype,), (F, n), optional=True))


class Context:
    """A decoder context on one GPU (owns the decode workspace)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().mbp_ctx_create(int(device), ctypes.byref(h)), "mbp_ctx_create")
        self.handle = h
        self.device = int(device)
        _open["ctx"].add(self)

    def close(self):
        if self.handle:
            lib().mbp_ctx_destroy(self.handle)
            self.handle = None
        _open["ctx"].discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile_enable(self, on: bool = True, kernels=None):
        """Time every kernel (on=True), none (on=False), or only the named
        kernels (a list of KERNEL_IDS keys)."""
        if not on:
            mask = 0
        elif kernels is None:
            mask = 0x3F
        else:
            mask = 0
            for k in kernels:
                mask |= 1 << KERNEL_IDS[k]
        _check(lib().mbp_profile_enable(self.handle, mask), "mbp_profile_enable")

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
        self.device = ctx.device
        self.handle = h
        self.n, self.u, self.m = int(n), u, m.tolist()
        self.M = int(m.sum())
        info = self.info()
        self.E, self.max_check_deg, self.max_var_deg = info["E"], info["max_check_deg"], info["max_var_deg"]
        _open["code"].add(self)

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
        _open["code"].discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

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
    if y.dim() != 2:
        raise ValueError("y must be [F, n]")
    F, n = (int(x) for x in y.shape)
    py = _dev(y, "y", ctx.device, _u8())
    pe = _dev(e, "e", ctx.device, _f64(), (F,))
    if out is None:
        out = torch.empty((F, n), dtype=_torch_dtype(dt), device=y.device)
    po = _dev(out, "out", ctx.device, (_torch_dtype(dt),), (F, n))
    _check(lib().mbp_llr_from_bits(ctx.handle, F, n, py, pe, dt, po, _stream_ptr(stream)), "mbp_llr_from_bits")
    return out


def _params(algo, dt, max_iter, early_exit, alpha, clip, compact, schedule, coupling="joint", msg="f32"):
    if coupling not in _COUPLINGS:
        raise ValueError(f"unknown coupling {coupling!r}")
    if msg not in _MSGS:
        raise ValueError(f"unknown message storage {msg!r}")
    return mbp_params(MBP_ALGO_SPA if algo == "spa" else MBP_ALGO_NMS, dt, int(max_iter),
                      int(bool(early_exit)), float(alpha), float(clip), int(bool(compact)),
                      {"flooding": MBP_FLOODING, "serial": MBP_MATRIX_SERIAL}[schedule],
                      _COUPLINGS[coupling], _MSGS[msg])


def _decode_outputs(F, n, dtype, dev, want_llr):
    import torch
    return dict(bits=torch.empty((F, n), dtype=torch.uint8, device=dev),
                iters=torch.empty(F, dtype=torch.int32, device=dev),
                ok=torch.empty(F, dtype=torch.uint8, device=dev),
                llr=torch.empty((F, n), dtype=dtype, device=dev) if want_llr else None)


def syndrome(ctx: Context, code: Code, x, out=None, stream=None):
    """Alice's syndromes, eq. (1): x [F, n] uint8 key bits (GPU) -> [F, M] uint8
    (the u syndromes of each frame back to back), computed on the GPU."""
    import torch
    if x.dim() != 2:
        raise ValueError("x must be [F, n]")
    F = int(x.shape[0])
    px = _dev(x, "x", ctx.device, _u8(), (F, code.n))
    if out is None:
        out = torch.empty((F, code.M), dtype=torch.uint8, device=x.device)
    po = _dev(out, "out", ctx.device, _u8(), (F, code.M))
    _check(lib().mbp_syndrome(ctx.handle, code.handle, F, px, po, _stream_ptr(stream)), "mbp_syndrome")
    return out


def syndrome_noalloc(ctx: Context, code: Code, x, out, stream=None):
    """syndrome() with no allocation and no wait (mbp_syndrome_noalloc): the
    caller passes the output [F, M] uint8; at most 2^21 / n groups of 64 frames."""
    if x.dim() != 2:
        raise ValueError("x must be [F, n]")
    F = int(x.shape[0])
    px = _dev(x, "x", ctx.device, _u8(), (F, code.n))
    po = _dev(out, "out", ctx.device, _u8(), (F, code.M))
    _check(lib().mbp_syndrome_noalloc(ctx.handle, code.handle, F, px, po, _stream_ptr(stream)),
           "mbp_syndrome_noalloc")
    return out


def peg_build(ctx: Context, n: int, m: int, var_deg, seeds, max_depth: int = -1):
    """u PEG matrices built on the GPU (mbp_peg_build), matrix l from
    seeds[l]: returns ([row_ptr] * u, [col_idx] * u) as int32 numpy arrays."""
    dv = np.ascontiguousarray(var_deg, dtype=np.int32)
    if dv.shape != (int(n),):
        raise ValueError("var_deg must have n entries")
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64).reshape(-1))
    u = int(sd.size)
    E = int(dv.sum())
    rp = np.zeros((u, int(m) + 1), dtype=np.int32)
    ci = np.zeros((u, E), dtype=np.int32)
    _check(lib().mbp_peg_build(ctx.handle, int(n), int(m), u, dv.ctypes.data, sd.ctypes.data, int(max_depth),
                               rp.ctypes.data, ci.ctypes.data), "mbp_peg_build")
    return [rp[l] for l in range(u)], [ci[l] for l in range(u)]


def decode(ctx: Context, code: Code, llr, synd, algo: str = "spa", max_iter: int = 50,
           early_exit: bool = True, alpha: float = 0.75, clip: float = 20.0,
           want_llr: bool = True, out: Optional[dict] = None, stream=None,
           compact: bool = True, schedule: str = "flooding", coupling: str = "joint",
           msg: str = "f32") -> dict:
    """Decode every frame: llr [F, n] (float32/float64, GPU), synd [F, M] (uint8, GPU).

    schedule: "flooding" or "serial" (Algorithm 1's per-matrix loop);
    coupling: "joint" (one stacked graph) or "independent" (one decoder per
    matrix, joined by eq. (2)); msg: "f32", or "f16" to store the check
    messages as binary16 (FP32 flooding joint decodes only).
    Returns dict(bits [F, n] uint8, iters [F] int32, ok [F] uint8, llr [F, n] or None).
    """
    import torch
    dt = _dtype_code(llr.dtype)
    if llr.dim() != 2:
        raise ValueError("llr must be [F, n]")
    F = int(llr.shape[0])
    pl = _dev(llr, "llr", ctx.device, (torch.float32, torch.float64), (F, code.n))
    pz = _dev(synd, "synd", ctx.device, _u8(), (F, code.M))
    if out is None:
        out = _decode_outputs(F, code.n, llr.dtype, llr.device, want_llr)
    pb, pi, pk, plo = _out_ptrs(out, ctx.device, F, code.n, llr.dtype)
    p = _params(algo, dt, max_iter, early_exit, alpha, clip, compact, schedule, coupling, msg)
    _check(lib().mbp_decode(ctx.handle, code.handle, ctypes.byref(p), F, pl, pz, pb, pi, pk, plo,
                            _stream_ptr(stream)), "mbp_decode")
    return out


def decode_from_bits(ctx: Context, code: Code, y, e, synd, dtype: str = "f32", algo: str = "spa",
                     max_iter: int = 50, early_exit: bool = True, alpha: float = 0.75,
                     clip: float = 20.0, want_llr: bool = True, out: Optional[dict] = None,
                     stream=None, compact: bool = True, schedule: str = "flooding",
                     coupling: str = "joint", msg: str = "f32") -> dict:
    """decode() with the channel given as Bob's bits y [F, n] (uint8, GPU) and
    error rates e [F] (float64, GPU); the LLRs are formed inside the decoder.
    Same outputs as llr_from_bits followed by decode, bit for bit."""
    import torch
    if y.dim() != 2:
        raise ValueError("y must be [F, n]")
    F = int(y.shape[0])
    py = _dev(y, "y", ctx.device, _u8(), (F, code.n))
    pe = _dev(e, "e", ctx.device, _f64(), (F,))
    pz = _dev(synd, "synd", ctx.device, _u8(), (F, code.M))
    tdt = _torch_dtype(_dtype_code(dtype))
    if out is None:
        out = _decode_outputs(F, code.n, tdt, y.device, want_llr)
    pb, pi, pk, plo = _out_ptrs(out, ctx.device, F, code.n, tdt)
    p = _params(algo, _dtype_code(tdt), max_iter, early_exit, alpha, clip, compact, schedule, coupling, msg)
    _check(lib().mbp_decode_from_bits(ctx.handle, code.handle, ctypes.byref(p), F, py, pe, pz, pb, pi, pk,
                                      plo, _stream_ptr(stream)), "mbp_decode_from_bits")
    return out


# ------------------------------------------------------------ unrolled min-sum
def unrolled_workspace_bytes(code: Code, nframes: int, K: int, ckpt_every: int) -> int:
    b = ctypes.c_uint64()
    _check(lib().mbp_unrolled_workspace_bytes(code.handle, int(nframes), int(K), int(ckpt_every),
                                              ctypes.byref(b)), "mbp_unrolled_workspace_bytes")
    return int(b.value)


def nms_unrolled_fwd(ctx: Context, code: Code, llr, synd, alpha, ckpt_every: int, clip: float,
                     workspace, out=None, stream=None):
    """L^K of K = alpha.shape[0] unrolled min-sum iterations (FP32, GPU tensors)."""
    import torch
    if llr.dim() != 2 or alpha.dim() != 2:
        raise ValueError("llr must be [F, n] and alpha [K, u]")
    F = int(llr.shape[0])
    K = int(alpha.shape[0])
    pl = _dev(llr, "llr", ctx.device, _f32(), (F, code.n))
    pz = _dev(synd, "synd", ctx.device, _u8(), (F, code.M))
    pa = _dev(alpha, "alpha", ctx.device, _f32(), (K, code.u))
    pw = _dev(workspace, "workspace", ctx.device, _u8())
    if out is None:
        out = torch.empty_like(llr)
    po = _dev(out, "out", ctx.device, _f32(), (F, code.n))
    _check(lib().mbp_nms_unrolled_fwd(ctx.handle, code.handle, F, K, int(ckpt_every), float(clip),
                                      pl, pz, pa, po, pw, int(workspace.numel()), _stream_ptr(stream)),
           "mbp_nms_unrolled_fwd")
    return out


def nms_unrolled_bwd(ctx: Context, code: Code, llr, synd, alpha, grad_out, ckpt_every: int,
                     clip: float, workspace, stream=None):
    """(dJ/dllr, dJ/dalpha) of the unrolled forward for dJ/dL^K = grad_out."""
    import torch
    if llr.dim() != 2 or alpha.dim() != 2:
        raise ValueError("llr must be [F, n] and alpha [K, u]")
    F = int(llr.shape[0])
    K = int(alpha.shape[0])
    pl = _dev(llr, "llr", ctx.device, _f32(), (F, code.n))
    pz = _dev(synd, "synd", ctx.device, _u8(), (F, code.M))
    pa = _dev(alpha, "alpha", ctx.device, _f32(), (K, code.u))
    pg = _dev(grad_out, "grad_out", ctx.device, _f32(), (F, code.n))
    pw = _dev(workspace, "workspace", ctx.device, _u8())
    grad_llr = torch.empty_like(llr)
    grad_alpha = torch.empty_like(alpha)
    _check(lib().mbp_nms_unrolled_bwd(ctx.handle, code.handle, F, K, int(ckpt_every), float(clip),
                                      pl, pz, pa, pg, grad_llr.data_ptr(), grad_alpha.data_ptr(), pw,
                                      int(workspace.numel()), _stream_ptr(stream)), "mbp_nms_unrolled_bwd")
    return grad_llr, grad_alpha


def _autograd_function():
    import torch

    class MbpUnrolledNMS(torch.autograd.Function):
        """L^K = unrolled min-sum(llr, alpha[K, u]); gradients from the HIP adjoint."""

        @staticmethod
        def forward(fctx, llr, alpha, ctx, code, synd, ckpt_every, clip):
            llr = llr.contiguous()
            alpha = alpha.contiguous()
            nbytes = unrolled_workspace_bytes(code, llr.shape[0], alpha.shape[0], ckpt_every)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=llr.device)
            out = nms_unrolled_fwd(ctx, code, llr, synd, alpha, ckpt_every, clip, ws)
            fctx.save_for_backward(llr, alpha, synd, ws)
            fctx.meta = (ctx, code, ckpt_every, clip)
            return out

        @staticmethod
        def backward(fctx, grad_out):
            llr, alpha, synd, ws = fctx.saved_tensors
            ctx, code, ckpt_every, clip = fctx.meta
            g_llr, g_alpha = nms_unrolled_bwd(ctx, code, llr, synd, alpha, grad_out.contiguous(),
                                              ckpt_every, clip, ws)
            return g_llr, g_alpha, None, None, None, None, None

    return MbpUnrolledNMS


_unrolled_fn = None


def unrolled_nms(ctx: Context, code: Code, llr, synd, alpha, ckpt_every: int = 5,
                 clip: float = 20.0):
    """Differentiable unrolled min-sum: returns L^K with autograd to llr and alpha."""
    global _unrolled_fn
    if _unrolled_fn is None:
        _unrolled_fn = _autograd_function()
    return _unrolled_fn.apply(llr, alpha, ctx, code, synd, int(ckpt_every), float(clip))


# ----------------------------------------------------------- batched decode
def _batched_params(algo, max_iter, early_exit, alpha, clip):
    if algo not in ("spa", "nms"):
        raise ValueError(f"unknown algo {algo!r}")
    return mbp_params(MBP_ALGO_SPA if algo == "spa" else MBP_ALGO_NMS, MBP_F32, int(max_iter),
                      int(bool(early_exit)), float(alpha), float(clip), 0, MBP_FLOODING, MBP_JOINT)


def batch_outputs(code: Code, llr, want_llr: bool = True) -> dict:
    import torch
    F = int(llr.shape[0])
    dev = llr.device
    return dict(bits=torch.empty((F, code.n), dtype=torch.uint8, device=dev),
                iters=torch.empty(F, dtype=torch.int32, device=dev),
                ok=torch.empty(F, dtype=torch.uint8, device=dev),
                llr=torch.empty((F, code.n), dtype=torch.float32, device=dev) if want_llr else None)


def _batches(items, outs):
    if len(items) != len(outs):
        raise ValueError("one output dict per batch")
    arr = (mbp_batch * len(items))()
    for k, ((code, llr, synd), o) in enumerate(zip(items, outs)):
        if llr.dim() != 2:
            raise ValueError(f"batch {k}: llr must be [F, n]")
        F, dev = int(llr.shape[0]), code.device
        pl = _dev(llr, f"batch {k} llr", dev, _f32(), (F, code.n))
        pz = _dev(synd, f"batch {k} synd", dev, _u8(), (F, code.M))
        pb, pi, pk, plo = _out_ptrs(o, dev, F, code.n, llr.dtype)
        arr[k] = mbp_batch(code.handle.value, F, pl, pz, pb, pi, pk, plo)
    return arr


def _tuning(t):
    if t is None:
        return None
    if isinstance(t, mbp_tuning):
        return t
    return mbp_tuning(int(t["rows_per_wave"]), int(t["vars_per_wave"]), int(t["blocks_per_cu"]),
                      int(t["schedule"]), int(t.get("compact", 1)))


def default_tuning() -> dict:
    t = mbp_tuning()
    _check(lib().mbp_tuning_default(ctypes.byref(t)), "mbp_tuning_default")
    return t.as_dict()


def decode_batched(ctx: Context, items, max_iter: int = 100, early_exit: bool = True,
                   alpha: float = 0.75, clip: float = 20.0, tuning=None, outs=None,
                   want_llr: bool = True, stream=None, algo: str = "nms"):
    """Decode [(Code, llr [F, n] f32, synd [F, M] u8), ...] in one persistent launch
    (FP32, min-sum or sum-product). Returns one output dict per item."""
    if outs is None:
        outs = [batch_outputs(c, l, want_llr) for c, l, _ in items]
    arr = _batches(items, outs)
    p = _batched_params(algo, max_iter, early_exit, alpha, clip)
    tu = _tuning(tuning)
    _check(lib().mbp_decode_batched(ctx.handle, len(items), arr, ctypes.byref(p),
                                    ctypes.byref(tu) if tu is not None else None,
                                    _stream_ptr(stream)), "mbp_decode_batched")
    return outs


def autotune(ctx: Context, items, max_iter: int = 100, early_exit: bool = True,
             alpha: float = 0.75, clip: float = 20.0, cache_path: Optional[str] = None,
             outs=None, algo: str = "nms") -> dict:
    if outs is None:
        outs = [batch_outputs(c, l) for c, l, _ in items]
    arr = _batches(items, outs)
    p = _batched_params(algo, max_iter, early_exit, alpha, clip)
    t = mbp_tuning()
    _check(lib().mbp_autotune(ctx.handle, len(items), arr, ctypes.byref(p),
                              cache_path.encode() if cache_path else None, ctypes.byref(t)),
           "mbp_autotune")
    return t.as_dict()


class Plan:
    """A captured hipGraph of a batched decode over fixed buffers."""

    def __init__(self, ctx: Context, items, outs, max_iter: int = 100, early_exit: bool = True,
                 alpha: float = 0.75, clip: float = 20.0, tuning=None, algo: str = "nms"):
        arr = _batches(items, outs)
        p = _batched_params(algo, max_iter, early_exit, alpha, clip)
        tu = _tuning(tuning)
        h = ctypes.c_void_p()
        _check(lib().mbp_plan_create(ctx.handle, len(items), arr, ctypes.byref(p),
                                     ctypes.byref(tu) if tu is not None else None, ctypes.byref(h)),
               "mbp_plan_create")
        self.handle = h
        self.ctx, self.items, self.outs = ctx, items, outs
        _open["plan"].add(self)

    def launch(self, stream=None):
        _check(lib().mbp_plan_launch(self.handle, _stream_ptr(stream)), "mbp_plan_launch")

    def wait(self, stream=None):
        _check(lib().mbp_plan_wait(self.handle, _stream_ptr(stream)), "mbp_plan_wait")

    def close(self):
        if self.handle:
            lib().mbp_plan_destroy(self.handle)
            self.handle = None
        _open["plan"].discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Queue:
    """Serving queue over the batched decode (mbp_queue_*): submit batches of
    frames as they arrive, flush to decode everything pending in one batched
    launch, poll for the frames done. Submitted tensors must stay alive until
    their flush completes; the queue keeps references to them until then."""

    def __init__(self, ctx: Context, max_iter: int = 100, early_exit: bool = True, alpha: float = 0.75,
                 clip: float = 20.0, tuning=None, algo: str = "nms"):
        p = _batched_params(algo, max_iter, early_exit, alpha, clip)
        tu = _tuning(tuning)
        h = ctypes.c_void_p()
        _check(lib().mbp_queue_create(ctx.handle, ctypes.byref(p), ctypes.byref(tu) if tu is not None else None,
                                      ctypes.byref(h)), "mbp_queue_create")
        self.handle = h
        self.ctx = ctx
        self._pending, self._flights, self._done = [], [], 0
        _open["queue"].add(self)

    def submit(self, items, outs):
        """items: [(Code, llr [F, n] f32, synd [F, M] u8)], outs: batch_outputs(...) per item."""
        arr = _batches(items, outs)
        _check(lib().mbp_queue_submit(self.handle, len(items), arr), "mbp_queue_submit")
        self._pending.append((items, outs, sum(int(llr.shape[0]) for _, llr, _ in items)))

    def flush(self, stream=None):
        _check(lib().mbp_queue_flush(self.handle, _stream_ptr(stream)), "mbp_queue_flush")
        if self._pending:
            self._flights.append(self._pending)
            self._pending = []

    def _release(self, done: int):
        # drop the references of flushes whose frames are all done
        while self._flights and done - self._done >= sum(f for _, _, f in self._flights[0]):
            self._done += sum(f for _, _, f in self._flights.pop(0))

    def poll(self) -> int:
        n = ctypes.c_int64()
        _check(lib().mbp_queue_poll(self.handle, ctypes.byref(n)), "mbp_queue_poll")
        self._release(int(n.value))
        return int(n.value)

    def wait(self):
        _check(lib().mbp_queue_wait(self.handle), "mbp_queue_wait")
        return self.poll()

    def close(self):
        if self.handle:
            lib().mbp_queue_destroy(self.handle)
            self.handle = None
            self._flights = []
        _open["queue"].discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
