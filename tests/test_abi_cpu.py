"""The C-ABI library loads and exports what include/mbp.h declares (CPU only).

No call here reaches a GPU: only symbol lookups, the version, and argument
checks that fail before any device work.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mbp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(mbp_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("mbp_ctx_create", "mbp_code_create", "mbp_decode", "mbp_llr_from_bits",
               "mbp_last_error"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    from paper_2001_07979_amd import mbp
    L = mbp.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_error_paths_without_device():
    from paper_2001_07979_amd import mbp
    L = mbp.lib()
    assert L.mbp_version() == 3
    h = ctypes.c_void_p()
    assert L.mbp_ctx_create(0, None) == mbp.MBP_EINVAL
    assert "NULL" in mbp.last_error()
    assert L.mbp_code_create(None, 8, 1, None, None, None, ctypes.byref(h)) == mbp.MBP_EINVAL
    assert "ctx" in mbp.last_error()
    p = mbp.mbp_params(0, 0, 10, 1, 0.75, 20.0)
    assert L.mbp_decode(None, None, ctypes.byref(p), 1, *([None] * 7)) == mbp.MBP_EINVAL
    assert L.mbp_llr_from_bits(None, 1, 1, None, None, 0, None, None) == mbp.MBP_EINVAL
    assert L.mbp_decode_from_bits(None, None, ctypes.byref(p), 1, *([None] * 8)) == mbp.MBP_EINVAL
    assert "mbp_decode_from_bits" in mbp.last_error()
    dv = (ctypes.c_int32 * 4)(2, 2, 2, 2)
    seeds = (ctypes.c_uint64 * 1)(1)
    assert L.mbp_peg_build(None, 4, 2, 1, dv, seeds, 1, None, None) == mbp.MBP_EINVAL
    assert "mbp_peg_build" in mbp.last_error()
    assert L.mbp_syndrome(None, None, 1, None, None, None) == mbp.MBP_EINVAL
    qh = ctypes.c_void_p()
    assert L.mbp_queue_create(None, ctypes.byref(p), None, ctypes.byref(qh)) == mbp.MBP_EINVAL
    assert L.mbp_queue_submit(None, 1, None) == mbp.MBP_EINVAL
    L.mbp_queue_destroy(None)
    n, ms = ctypes.c_int64(), ctypes.c_double()
    assert L.mbp_profile_get(None, 0, ctypes.byref(n), ctypes.byref(ms)) == mbp.MBP_EINVAL
    L.mbp_ctx_destroy(None)
    L.mbp_code_destroy(None)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2001_07979_amd import mbp
    monkeypatch.setattr(mbp, "_lib", None)
    monkeypatch.setattr(mbp, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        mbp.lib()


def test_binding_rejects_host_and_misshaped_tensors(monkeypatch):
    """Every device buffer is checked in the binding before the library is
    called: a host tensor (a GPU page fault if its address reached a kernel),
    a strided view, a wrong dtype or shape, and an alpha that is not [K, u]
    are all refused with ValueError, and no library call happens."""
    import types

    import torch
    from paper_2001_07979_amd import mbp

    def no_call():
        raise AssertionError("the library was called")

    monkeypatch.setattr(mbp, "lib", no_call)
    ctx = types.SimpleNamespace(device=0, handle=None)
    code = types.SimpleNamespace(n=8, M=4, u=2, device=0, handle=types.SimpleNamespace(value=None))
    F = 3
    y = torch.zeros((F, 8), dtype=torch.uint8)
    e = torch.full((F,), 0.05, dtype=torch.float64)
    z = torch.zeros((F, 4), dtype=torch.uint8)
    lam = torch.zeros((F, 8), dtype=torch.float32)
    with pytest.raises(ValueError, match="cuda:0"):
        mbp.llr_from_bits(ctx, y, e)
    with pytest.raises(ValueError, match="cuda:0"):
        mbp.decode(ctx, code, lam, z)
    with pytest.raises(ValueError, match="cuda:0"):
        mbp.decode_from_bits(ctx, code, y, e, z)
    with pytest.raises(ValueError, match="cuda:0"):
        mbp.syndrome(ctx, code, y)
    with pytest.raises(ValueError, match="cuda:0"):
        mbp.nms_unrolled_fwd(ctx, code, lam, z, torch.zeros((5, 2)), 1, 20.0, torch.zeros(4, dtype=torch.uint8))
    with pytest.raises(ValueError, match="cuda:0"):
        mbp.decode_batched(ctx, [(code, lam, z)], outs=[{}])


def test_device_check_order_on_fake_cuda_tensors(monkeypatch):
    """The device check itself, with the CUDA test answered by a stand-in so
    it runs without a GPU: strided views, wrong dtypes and shapes, and an
    alpha of the wrong [K, u] shape are rejected."""
    import torch
    from paper_2001_07979_amd import mbp

    class FakeCuda(torch.Tensor):
        @property
        def is_cuda(self):
            return True

        @property
        def device(self):
            return torch.device("cuda", 0)

    def fake(t):
        return t.as_subclass(FakeCuda)

    a = fake(torch.zeros((4, 6), dtype=torch.float32))
    assert mbp._dev(a, "a", 0, (torch.float32,), (4, 6)) == a.data_ptr()
    with pytest.raises(ValueError, match="cuda:1"):
        mbp._dev(a, "a", 1)
    with pytest.raises(ValueError, match="contiguous"):
        mbp._dev(fake(torch.zeros((6, 4)).t()), "a", 0)
    with pytest.raises(ValueError, match="torch.float64"):
        mbp._dev(a, "a", 0, (torch.float64,))
    with pytest.raises(ValueError, match="shape"):
        mbp._dev(a, "alpha", 0, (torch.float32,), (5, 2))
    with pytest.raises(TypeError):
        mbp._dev([1, 2], "a", 0)


def test_close_all_order():
    """close_all() closes plans and queues before codes and codes before
    contexts, once each, and leaves nothing registered."""
    from paper_2001_07979_amd import mbp

    closed = []

    class Obj:
        def __init__(self, kind):
            self.kind = kind

        def close(self):
            closed.append(self.kind)
            mbp._open[self.kind].discard(self)

    objs = [Obj(k) for k in ("ctx", "code", "plan", "queue", "code", "ctx")]
    for o in objs:
        mbp._open[o.kind].add(o)
    mbp.close_all()
    assert closed == ["plan", "queue", "code", "code", "ctx", "ctx"]
    assert all(len(s) == 0 for s in mbp._open.values())
