"""GPU parity of the independent-decoder coupling (Sec. 2 forms the LLRs and
messages of each of the u matrices respectively: matrix l's variable-to-check
message is lambda plus matrix l's other check messages at the variable, and
only the soft decision of eq. (2) joins the matrices) against the oracle's
coupling of the same name, through the C-ABI, under both schedules."""
import ctypes

import numpy as np
import pytest

from paper_2001_07979_amd.inputs import bsc_frames, peg_code
from paper_2001_07979_amd.inputs import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu

RTOL32 = 1e-4
RTOL64 = 1e-9
IND = "independent"


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2001_07979_amd import mbp
    c = mbp.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def codes():
    """Two matrices (n = 1000, ragged) and three (n = 640), as the serial tests."""
    return {2: peg_code(1000, 260, 2, W.IRREGULAR_238, seed_base=7100, name="peg-n1000"),
            3: peg_code(640, 200, 3, {2: 0.3, 3: 0.7}, seed_base=7300, name="peg-n640-u3")}


def _upload(ctx, code):
    from paper_2001_07979_amd import mbp
    return mbp.Code.from_inputs(ctx, code)


@pytest.mark.parametrize("schedule", ["flooding", "serial"])
@pytest.mark.parametrize("u", [2, 3])
@pytest.mark.parametrize("algo,dtype", [("nms", "f32"), ("spa", "f32"), ("spa", "f64"),
                                        ("nms", "f64")])
@pytest.mark.parametrize("F", [1, 65, 130])
def test_independent_parity(ctx, codes, schedule, u, algo, dtype, F):
    """FP32 min-sum bit for bit with the binary32 oracle, FP64 min-sum bit for
    bit with the FP64 oracle, sum-product under the parity protocol."""
    code = codes[u]
    hi = 0.03 if u == 2 else 0.025
    fr = bsc_frames(code, F, np.linspace(0.005, hi, F), seed=500 + F + u)
    dc = _upload(ctx, code)
    lam = parity.oracle_llr(fr, dtype)
    kw = dict(schedule=schedule, coupling=IND)
    if dtype == "f32":
        g = parity.gpu_run(ctx, dc, fr, algo, dtype, 40, **kw)
        assert np.array_equal(g["llr_in"].astype(np.float64), lam)
    else:
        g = parity.gpu_run(ctx, dc, fr, algo, dtype, 40, llr=lam, **kw)
    o = parity.oracle_run(code, fr, algo, dtype, 40, lam=lam, **kw)
    if (algo, dtype) == ("nms", "f32"):
        parity.assert_bitwise(g, parity.oracle_f32_run(code, fr, 40, lam=lam, **kw))
    if (algo, dtype) == ("nms", "f64"):
        parity.assert_bitwise(g, o)
    long = dict(long_after=parity.nms_long_after(schedule, u)) if (algo, dtype) == ("nms", "f32") else {}
    s = parity.compare(g, o, 40, RTOL32 if dtype == "f32" else RTOL64,
                       atol=parity.ATOL32 if dtype == "f32" else 0.0, **long)
    assert s["oracle_ok"] >= F // 2


@pytest.mark.parametrize("schedule", ["flooding", "serial"])
@pytest.mark.parametrize("u", [2, 3])
def test_independent_fixed_iterations(ctx, codes, schedule, u):
    """Without early exit, T = 1, 2 and 7: FP32 min-sum bit for bit with the
    binary32 oracle, FP64 sum-product on every frame within 1e-9."""
    code = codes[u]
    fr = bsc_frames(code, 70, 0.04, seed=29 + u)
    dc = _upload(ctx, code)
    kw = dict(schedule=schedule, coupling=IND)
    for T in (1, 2, 7):
        g = parity.gpu_run(ctx, dc, fr, "nms", "f32", T, early_exit=False, **kw)
        assert np.all(g["iters"] == T)
        parity.assert_bitwise(g, parity.oracle_f32_run(code, fr, T, early_exit=False, **kw))
        o = parity.oracle_run(code, fr, "spa", "f64", T, early_exit=False, **kw)
        g64 = parity.gpu_run(ctx, dc, fr, "spa", "f64", T, early_exit=False, llr=o["llr_in"], **kw)
        parity.compare(g64, o, T, RTOL64, exact_all=True)


@pytest.mark.parametrize("schedule", ["flooding", "serial"])
@pytest.mark.parametrize("algo", ["spa", "nms"])
def test_independent_from_bits_and_compaction(ctx, codes, schedule, algo):
    """From Bob's bits equals the LLR path bit for bit; compaction on and off
    give the same outputs (300 frames with spread-out stopping iterations)."""
    import torch
    from paper_2001_07979_amd import mbp
    code = codes[2]
    fr = bsc_frames(code, 300, np.linspace(0.002, 0.04, 300), seed=77)
    dc = _upload(ctx, code)
    dev = torch.device("cuda", ctx.device)
    y = torch.from_numpy(fr.y).to(dev)
    e = torch.from_numpy(fr.p).to(dev)
    z = torch.from_numpy(fr.z).to(dev)
    lam = mbp.llr_from_bits(ctx, y, e)
    kw = dict(algo=algo, max_iter=50, schedule=schedule, coupling=IND)
    a = mbp.decode(ctx, dc, lam, z, **kw)
    b = mbp.decode_from_bits(ctx, dc, y, e, z, **kw)
    c = mbp.decode(ctx, dc, lam, z, compact=False, **kw)
    torch.cuda.synchronize()
    for k in ("bits", "iters", "ok", "llr"):
        assert torch.equal(a[k], b[k]), f"from bits: {k}"
        assert torch.equal(a[k], c[k]), f"compaction: {k}"
    its = a["iters"].cpu().numpy()
    assert its.max() > its.min() + 2, "frames should stop at different iterations"


@pytest.mark.parametrize("u", [2, 3])
def test_independent_schedules_agree(ctx, codes, u):
    """Independent decoders do not exchange messages, so visiting the
    matrices in turn changes nothing: matrix l's check pass reads lambda plus
    its own messages of the previous iteration under either schedule, and the
    soft decisions and stopping test come after the last matrix. The two
    schedules give the same outputs bit for bit."""
    code = codes[u]
    fr = bsc_frames(code, 130, np.linspace(0.005, 0.04, 130), seed=600 + u)
    dc = _upload(ctx, code)
    for algo, dtype in (("spa", "f32"), ("nms", "f32"), ("spa", "f64")):
        a = parity.gpu_run(ctx, dc, fr, algo, dtype, 40, coupling=IND)
        b = parity.gpu_run(ctx, dc, fr, algo, dtype, 40, coupling=IND, schedule="serial")
        for k in ("bits", "iters", "ok", "L"):
            assert np.array_equal(a[k], b[k]), (algo, dtype, k)


def test_independent_one_matrix_is_joint(ctx):
    """With u = 1 the two couplings are the same decoder."""
    code = peg_code(1000, 260, 1, W.IRREGULAR_238, seed_base=7500, name="peg-n1000-u1")
    fr = bsc_frames(code, 64, np.linspace(0.01, 0.03, 64), seed=31)
    dc = _upload(ctx, code)
    for algo in ("spa", "nms"):
        a = parity.gpu_run(ctx, dc, fr, algo, "f32", 30)
        b = parity.gpu_run(ctx, dc, fr, algo, "f32", 30, coupling=IND)
        for k in ("bits", "iters", "ok", "L"):
            assert np.array_equal(a[k], b[k]), (algo, k)


def test_independent_is_not_joint(ctx, codes):
    """The couplings are different decoders: their soft decisions differ."""
    code = codes[2]
    fr = bsc_frames(code, 64, 0.03, seed=41)
    dc = _upload(ctx, code)
    a = parity.gpu_run(ctx, dc, fr, "spa", "f32", 3, early_exit=False)
    b = parity.gpu_run(ctx, dc, fr, "spa", "f32", 3, early_exit=False, coupling=IND)
    assert not np.array_equal(a["L"], b["L"])


def test_independent_n65536_every_frame(ctx):
    """The 256-frame u = 2 n = 65536 batch with independent decoders,
    flooding, FP32 sum-product: every frame against the FP64 oracle under the
    parity protocol, and min-sum bit for bit with the binary32 oracle."""
    wl = W.qkd_n65536(nframes=256, algo="spa")
    code, fr = wl.code, wl.frames()
    dc = _upload(ctx, code)
    kw = dict(coupling=IND)
    g = parity.gpu_run(ctx, dc, fr, "spa", "f32", 100, **kw)
    o = parity.oracle_run(code, fr, "spa", "f32", 100, **kw)
    s = parity.compare(g, o, 100, RTOL32, atol=parity.ATOL32)
    assert s["oracle_ok"] == 256
    gn = parity.gpu_run(ctx, dc, fr, "nms", "f32", 100, **kw)
    parity.assert_bitwise(gn, parity.oracle_f32_run(code, fr, 100, **kw))


def test_independent_rejections(ctx, codes):
    """Codes of more than four matrices and the batched decode refuse the
    independent coupling (EUNSUPPORTED); an unknown coupling is EINVAL."""
    import torch
    from paper_2001_07979_amd import mbp
    dev = torch.device("cuda", ctx.device)
    code5 = peg_code(400, 60, 5, {2: 0.3, 3: 0.7}, seed_base=7700, name="peg-n400-u5")
    dc5 = _upload(ctx, code5)
    fr = bsc_frames(code5, 4, 0.01, seed=3)
    lam = torch.zeros((4, code5.n), dtype=torch.float32, device=dev)
    z = torch.from_numpy(fr.z).to(dev)
    with pytest.raises(RuntimeError, match="at most 4 matrices"):
        mbp.decode(ctx, dc5, lam, z, coupling=IND)
    with pytest.raises(ValueError):
        mbp.decode(ctx, dc5, lam, z, coupling="stacked")
    # raw parameters through the C-ABI: coupling 7, and the batched decode
    dc = _upload(ctx, codes[2])
    fr2 = bsc_frames(codes[2], 4, 0.01, seed=4)
    lam2 = torch.zeros((4, codes[2].n), dtype=torch.float32, device=dev)
    z2 = torch.from_numpy(fr2.z).to(dev)
    o = mbp.batch_outputs(dc, lam2)
    p = mbp.mbp_params(mbp.MBP_ALGO_NMS, mbp.MBP_F32, 10, 1, 0.75, 20.0, 1, mbp.MBP_FLOODING, 7)
    rc = mbp.lib().mbp_decode(ctx.handle, dc.handle, ctypes.byref(p), 4, lam2.data_ptr(), z2.data_ptr(),
                              o["bits"].data_ptr(), o["iters"].data_ptr(), o["ok"].data_ptr(), None, None)
    assert rc == -1 and b"coupling" in mbp.lib().mbp_last_error()
    b = mbp.mbp_batch(dc.handle, 4, lam2.data_ptr(), z2.data_ptr(), o["bits"].data_ptr(),
                      o["iters"].data_ptr(), o["ok"].data_ptr(), o["llr"].data_ptr())
    p.coupling = mbp.MBP_INDEPENDENT
    t = mbp.mbp_tuning()
    assert mbp.lib().mbp_tuning_default(ctypes.byref(t)) == 0
    rc = mbp.lib().mbp_decode_batched(ctx.handle, 1, ctypes.byref(b), ctypes.byref(p), ctypes.byref(t), None)
    assert rc == -5 and b"joint" in mbp.lib().mbp_last_error()
    torch.cuda.synchronize()
