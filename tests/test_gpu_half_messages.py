"""GPU parity of binary16 message storage (msg="f16"): every new check
message is computed in FP32 and stored rounded to the nearest binary16, and
every later read uses the stored value; the soft decisions stay FP32. The
oracle's decoders have the same option (each new message rounded to
binary16 before it is stored). Min-sum is held bit for bit to the binary32
oracle with binary16 storage; sum-product to the FP64 oracle with binary16
storage under the parity protocol, with the bound below."""
import numpy as np
import pytest

from paper_2001_07979_amd.inputs import bsc_frames, peg_code
from paper_2001_07979_amd.inputs import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu

# Sum-product: the GPU forms each message in FP32 with hardware exp2/log2,
# the oracle in FP64; the two round to the same binary16 value except where
# the FP32 value sits within its own error of a binary16 rounding boundary,
# where they differ by one binary16 step (2^-11 relative). Such a step moves
# the soft decisions it enters by up to 2^-11 |c| (1e-2 near the clip: the
# absolute term), and later iterations carry it on. Measured on this file's
# inputs: largest relative difference of L 3.7e-4 (u = 2 and 3, 130
# frames; 3.5e-4 on the first 64 headline frames); the bound keeps 5x.
RTOL16 = 2e-3
ATOL16 = 1e-2
F16 = dict(msg="f16")


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
    return {2: peg_code(1000, 260, 2, W.IRREGULAR_238, seed_base=7100, name="peg-n1000"),
            3: peg_code(640, 200, 3, {2: 0.3, 3: 0.7}, seed_base=7300, name="peg-n640-u3")}


def _upload(ctx, code):
    from paper_2001_07979_amd import mbp
    return mbp.Code.from_inputs(ctx, code)


@pytest.mark.parametrize("u", [2, 3])
@pytest.mark.parametrize("F", [1, 65, 130])
def test_half_min_sum_bitwise(ctx, codes, u, F):
    """FP32 min-sum with binary16 messages, bit for bit with the binary32
    oracle's min-sum with binary16 storage (bits, iterations, flags, L)."""
    code = codes[u]
    hi = 0.03 if u == 2 else 0.025
    fr = bsc_frames(code, F, np.linspace(0.005, hi, F), seed=900 + F + u)
    dc = _upload(ctx, code)
    g = parity.gpu_run(ctx, dc, fr, "nms", "f32", 40, **F16)
    lam = parity.oracle_llr(fr, "f32")
    parity.assert_bitwise(g, parity.oracle_f32_run(code, fr, 40, lam=lam, **F16))
    # binary16 storage is a different decoder from FP32 storage
    if F > 1:
        g32 = parity.gpu_run(ctx, dc, fr, "nms", "f32", 40)
        assert not np.array_equal(g["L"], g32["L"])


@pytest.mark.parametrize("u", [2, 3])
@pytest.mark.parametrize("F", [1, 65, 130])
def test_half_sum_product(ctx, codes, u, F):
    """FP32 sum-product with binary16 messages against the FP64 oracle with
    binary16 storage: every strict frame equal in bits, iterations and
    success, its soft decisions within RTOL16 relative plus ATOL16."""
    code = codes[u]
    hi = 0.03 if u == 2 else 0.025
    fr = bsc_frames(code, F, np.linspace(0.005, hi, F), seed=950 + F + u)
    dc = _upload(ctx, code)
    g = parity.gpu_run(ctx, dc, fr, "spa", "f32", 40, **F16)
    o = parity.oracle_run(code, fr, "spa", "f32", 40, lam=parity.oracle_llr(fr, "f32"), **F16)
    s = parity.compare(g, o, 40, RTOL16, atol=ATOL16)
    print("half sum-product", u, F, s)
    assert s["oracle_ok"] >= F // 2


def test_half_fixed_iterations(ctx, codes):
    """Without early exit, T = 1, 2 and 7: min-sum bit for bit with the
    binary32 oracle with binary16 storage; at T = 1 sum-product equals the
    FP64 oracle's binary16 messages to within one binary16 step per message."""
    code = codes[2]
    fr = bsc_frames(code, 70, 0.04, seed=31)
    dc = _upload(ctx, code)
    lam = parity.oracle_llr(fr, "f32")
    for T in (1, 2, 7):
        g = parity.gpu_run(ctx, dc, fr, "nms", "f32", T, early_exit=False, **F16)
        assert np.all(g["iters"] == T)
        parity.assert_bitwise(g, parity.oracle_f32_run(code, fr, T, early_exit=False, lam=lam, **F16))
    g = parity.gpu_run(ctx, dc, fr, "spa", "f32", 1, early_exit=False, **F16)
    o = parity.oracle_run(code, fr, "spa", "f32", 1, early_exit=False, lam=lam, **F16)
    deg = np.zeros(code.n)
    for ci in code.col_idx:
        np.add.at(deg, ci, 1)
    step = deg * 20.0 * 2.0 ** -10 + 1e-5  # one binary16 step of the largest message, per edge
    assert np.all(np.abs(g["L"] - o["L"]) <= step[None, :])


@pytest.mark.parametrize("algo", ["spa", "nms"])
def test_half_from_bits_and_compaction(ctx, codes, algo):
    """From Bob's bits equals the LLR path bit for bit, and compaction on and
    off give the same outputs, with binary16 messages (300 frames whose
    stopping iterations spread out)."""
    import torch
    from paper_2001_07979_amd import mbp
    code = codes[2]
    fr = bsc_frames(code, 300, np.linspace(0.002, 0.04, 300), seed=78)
    dc = _upload(ctx, code)
    dev = torch.device("cuda", ctx.device)
    y = torch.from_numpy(fr.y).to(dev)
    e = torch.from_numpy(fr.p).to(dev)
    z = torch.from_numpy(fr.z).to(dev)
    lam = mbp.llr_from_bits(ctx, y, e)
    kw = dict(algo=algo, max_iter=50, msg="f16")
    a = mbp.decode(ctx, dc, lam, z, **kw)
    b = mbp.decode_from_bits(ctx, dc, y, e, z, **kw)
    c = mbp.decode(ctx, dc, lam, z, compact=False, **kw)
    torch.cuda.synchronize()
    for k in ("bits", "iters", "ok", "llr"):
        assert torch.equal(a[k], b[k]), f"from bits: {k}"
        assert torch.equal(a[k], c[k]), f"compaction: {k}"
    its = a["iters"].cpu().numpy()
    assert its.max() > its.min() + 2


def test_half_n262144_headline_frames(ctx):
    """The headline workload (n = 2^18, u = 3, rate 0.85, p = 0.02): all 1024
    frames decode with binary16 messages (FER 0, as with FP32 storage), and
    every frame of the first group (64) matches the FP64 oracle with binary16
    storage under the protocol."""
    import torch
    from paper_2001_07979_amd import mbp
    wl = W.qkd_n262144(0.85, nframes=1024)
    code, fr = wl.code, wl.frames()
    dc = _upload(ctx, code)
    dev = torch.device("cuda", ctx.device)
    y = torch.from_numpy(fr.y).to(dev)
    e = torch.from_numpy(fr.p).to(dev)
    z = torch.from_numpy(fr.z).to(dev)
    out = mbp.decode_from_bits(ctx, dc, y, e, z, algo="spa", max_iter=100, msg="f16")
    torch.cuda.synchronize()
    bits = out["bits"].cpu().numpy()
    assert np.array_equal(bits, fr.x), "every frame decodes"
    idx = np.arange(64)
    g = {k: v.cpu().numpy() for k, v in (("bits", out["bits"]), ("iters", out["iters"]), ("ok", out["ok"]))}
    g["L"] = out["llr"].cpu().numpy().astype(np.float64)
    o = parity.oracle_run(code, fr, "spa", "f32", 100, idx=idx, **F16)
    s = parity.compare(g, o, 100, RTOL16, idx=idx, atol=ATOL16)
    print("half headline", s)
    assert s["oracle_ok"] == 64


def test_half_rejections(ctx, codes):
    """Binary16 messages need FP32, flooding and the joint coupling; the
    batched decode refuses them."""
    import ctypes

    import torch
    from paper_2001_07979_amd import mbp
    code = codes[2]
    dc = _upload(ctx, code)
    dev = torch.device("cuda", ctx.device)
    fr = bsc_frames(code, 4, 0.01, seed=5)
    z = torch.from_numpy(fr.z).to(dev)
    lam32 = torch.zeros((4, code.n), dtype=torch.float32, device=dev)
    lam64 = torch.zeros((4, code.n), dtype=torch.float64, device=dev)
    for kw, lam in ((dict(schedule="serial"), lam32), (dict(coupling="independent"), lam32), ({}, lam64)):
        with pytest.raises(RuntimeError, match="binary16"):
            mbp.decode(ctx, dc, lam, z, msg="f16", **kw)
    with pytest.raises(ValueError):
        mbp.decode(ctx, dc, lam32, z, msg="bf16")
    o = mbp.batch_outputs(dc, lam32)
    b = mbp.mbp_batch(dc.handle, 4, lam32.data_ptr(), z.data_ptr(), o["bits"].data_ptr(),
                      o["iters"].data_ptr(), o["ok"].data_ptr(), o["llr"].data_ptr())
    p = mbp.mbp_params(mbp.MBP_ALGO_SPA, mbp.MBP_F32, 10, 1, 0.75, 20.0, 0, mbp.MBP_FLOODING, mbp.MBP_JOINT,
                       mbp.MBP_MSG_F16)
    t = mbp.mbp_tuning()
    assert mbp.lib().mbp_tuning_default(ctypes.byref(t)) == 0
    rc = mbp.lib().mbp_decode_batched(ctx.handle, 1, ctypes.byref(b), ctypes.byref(p), ctypes.byref(t), None)
    assert rc == -5 and b"FP32 messages" in mbp.lib().mbp_last_error()
    torch.cuda.synchronize()
