"""GPU parity of the matrix-serial schedule (Algorithm 1: within an iteration
the matrices are visited in turn, each check pass followed by a variable
pass, so matrix l + 1 already sees what matrix l sent) against the oracle's
schedule of the same name, through the C-ABI."""
import numpy as np
import pytest

from paper_2001_07979_amd.inputs import bsc_frames, peg_code, syndromes
from paper_2001_07979_amd.inputs import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu

RTOL32 = 1e-4
RTOL64 = 1e-9
S = "serial"


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
    """Two matrices (n = 1000, ragged) and three (n = 640, the middle one's
    first-iteration pass sees one earlier matrix and leaves one out)."""
    return {2: peg_code(1000, 260, 2, W.IRREGULAR_238, seed_base=7100, name="peg-n1000"),
            3: peg_code(640, 200, 3, {2: 0.3, 3: 0.7}, seed_base=7300, name="peg-n640-u3")}


def _upload(ctx, code):
    from paper_2001_07979_amd import mbp
    return mbp.Code.from_inputs(ctx, code)


@pytest.mark.parametrize("u", [2, 3])
@pytest.mark.parametrize("algo,dtype", [("nms", "f32"), ("spa", "f32"), ("spa", "f64"),
                                        ("nms", "f64")])
@pytest.mark.parametrize("F", [1, 65, 130])
def test_serial_parity(ctx, codes, u, algo, dtype, F):
    code = codes[u]
    hi = 0.035 if u == 2 else 0.03
    fr = bsc_frames(code, F, np.linspace(0.01, hi, F), seed=300 + F + u)
    dc = _upload(ctx, code)
    lam = parity.oracle_llr(fr, dtype)
    if dtype == "f32":
        g = parity.gpu_run(ctx, dc, fr, algo, dtype, 40, schedule=S)
        assert np.array_equal(g["llr_in"].astype(np.float64), lam)
    else:
        g = parity.gpu_run(ctx, dc, fr, algo, dtype, 40, llr=lam, schedule=S)
    o = parity.oracle_run(code, fr, algo, dtype, 40, lam=lam, schedule=S)
    if (algo, dtype) == ("nms", "f32"):
        parity.assert_bitwise(g, parity.oracle_f32_run(code, fr, 40, lam=lam, schedule=S))
    if (algo, dtype) == ("nms", "f64"):
        parity.assert_bitwise(g, o)
    # every frame at 1e-4 / 1e-9 whatever its iteration count (sum-product
    # stops within 6 here); FP32 min-sum past nms_long_after iterations is held
    # bit for bit to the binary32 oracle above and counted against FP64
    long = dict(long_after=parity.nms_long_after(S, u)) if (algo, dtype) == ("nms", "f32") else {}
    s = parity.compare(g, o, 40, RTOL32 if dtype == "f32" else RTOL64,
                       atol=parity.ATOL32 if dtype == "f32" else 0.0, **long)
    assert s["oracle_ok"] >= F // 2


@pytest.mark.parametrize("u", [2, 3])
def test_serial_fixed_iterations(ctx, codes, u):
    """Without early exit: T = 1 (only the first iteration's partial sums), 2
    and 7 iterations, FP32 min-sum bit for bit against the binary32 oracle."""
    code = codes[u]
    fr = bsc_frames(code, 70, 0.04, seed=19 + u)
    dc = _upload(ctx, code)
    for T in (1, 2, 7):
        g = parity.gpu_run(ctx, dc, fr, "nms", "f32", T, early_exit=False, schedule=S)
        assert np.all(g["iters"] == T)
        parity.assert_bitwise(g, parity.oracle_f32_run(code, fr, T, early_exit=False, schedule=S))
        o = parity.oracle_run(code, fr, "spa", "f64", T, early_exit=False, schedule=S)
        g64 = parity.gpu_run(ctx, dc, fr, "spa", "f64", T, early_exit=False, llr=o["llr_in"],
                             schedule=S)
        parity.compare(g64, o, T, RTOL64, exact_all=True)


def test_serial_one_matrix_is_flooding(ctx):
    """With u = 1 there is one phase: the two schedules are the same decoder."""
    code = peg_code(1000, 260, 1, W.IRREGULAR_238, seed_base=7500, name="peg-n1000-u1")
    fr = bsc_frames(code, 64, np.linspace(0.01, 0.03, 64), seed=31)
    dc = _upload(ctx, code)
    for algo in ("spa", "nms"):
        a = parity.gpu_run(ctx, dc, fr, algo, "f32", 30)
        b = parity.gpu_run(ctx, dc, fr, algo, "f32", 30, schedule=S)
        for k in ("bits", "iters", "ok", "L"):
            assert np.array_equal(a[k], b[k]), (algo, k)


@pytest.mark.parametrize("algo,dtype", [("spa", "f32"), ("nms", "f32"), ("spa", "f64")])
def test_serial_compaction_keeps_results(ctx, codes, algo, dtype):
    """300 frames with spread-out stopping iterations: regrouping the running
    frames into spare groups changes no output of the serial schedule."""
    import torch
    from paper_2001_07979_amd import mbp
    code = codes[2]
    p = np.random.default_rng(911).permutation(np.geomspace(0.02, 0.09, 300))
    fr = bsc_frames(code, 300, p, seed=911)
    dc = _upload(ctx, code)
    lam = parity.oracle_llr(fr, dtype)
    llr = torch.from_numpy(lam.astype(np.float32 if dtype == "f32" else np.float64)).cuda()
    z = torch.from_numpy(fr.z).cuda()
    T = 60
    outs = [mbp.decode(ctx, dc, llr, z, algo=algo, max_iter=T, compact=cp, schedule=S)
            for cp in (True, False)]
    torch.cuda.synchronize()
    a, b = ({k: v.cpu().numpy() for k, v in o.items()} for o in outs)
    for k in ("bits", "iters", "ok", "llr"):
        assert np.array_equal(a[k], b[k]), k
    its = a["iters"]
    assert (its == T).sum() > 30 and (its <= 5).sum() > 40
    g = dict(bits=a["bits"], iters=a["iters"], ok=a["ok"], L=a["llr"].astype(np.float64))
    # every frame against the oracle, failed or not
    if algo == "nms":
        parity.assert_bitwise(g, parity.oracle_f32_run(code, fr, T, lam=lam, schedule=S))
    o = parity.oracle_run(code, fr, algo, dtype, T, lam=lam, schedule=S)
    # stragglers up to T = 60 near the code's threshold; measured beyond 16
    # iterations: FP32 sum-product L within 5.6e-3 (a frame at 29
    # iterations), FP64 within 2.1e-5 (a frame at 56); FP32 min-sum against
    # FP64: 23 of 300 long decodes differ
    long = {("spa", "f32"): dict(long_after=parity.SPA_LONG_AFTER, long_rtol=2e-2),
            ("spa", "f64"): dict(long_after=parity.SPA_LONG_AFTER, long_rtol=1e-4),
            ("nms", "f32"): dict(long_after=parity.nms_long_after(S, 2), long_budget=0.1)}[(algo, dtype)]
    parity.compare(g, o, T, RTOL32 if dtype == "f32" else RTOL64,
                   atol=parity.ATOL32 if dtype == "f32" else 0.0, **long)


@pytest.mark.parametrize("algo", ["spa", "nms"])
def test_serial_n65536_every_frame(ctx, algo):
    """The u = 2 n = 65536, 256-frame workload under the serial schedule:
    every frame against the oracle (min-sum also bit for bit with the
    binary32 oracle), properties on all, and fewer iterations on average
    than flooding."""
    wl = W.qkd_n65536(algo=algo)
    fr = wl.frames()
    dc = _upload(ctx, wl.code)
    g = parity.gpu_run(ctx, dc, fr, algo, "f32", wl.max_iter, alpha=wl.alpha, schedule=S)
    o = parity.oracle_run(wl.code, fr, algo, "f32", wl.max_iter, alpha=wl.alpha, schedule=S)
    if algo == "nms":
        parity.assert_bitwise(g, parity.oracle_f32_run(wl.code, fr, wl.max_iter, schedule=S))
    s = parity.compare(g, o, wl.max_iter, RTOL32, atol=parity.ATOL32)
    assert s["oracle_ok"] == 256
    okf = g["ok"] == 1
    assert np.array_equal(syndromes(wl.code, g["bits"][okf]), fr.z[okf])
    assert np.all(g["iters"][~okf] == wl.max_iter)
    assert okf.mean() > 0.99 and np.array_equal(g["bits"][okf], fr.x[okf])
    flood = parity.gpu_run(ctx, dc, fr, algo, "f32", wl.max_iter, alpha=wl.alpha)
    assert g["iters"].mean() < flood["iters"].mean()


@pytest.mark.parametrize("rate", [0.5, 0.7, 0.85])
def test_serial_u3_n262144_every_frame(ctx, rate):
    """Three matrices at QKD scale (n = 2^18, the three (rate, p) points),
    sum-product: all 64 frames against the oracle."""
    wl = W.qkd_n262144(rate, algo="spa")
    fr = wl.frames()
    dc = _upload(ctx, wl.code)
    g = parity.gpu_run(ctx, dc, fr, "spa", "f32", wl.max_iter, alpha=wl.alpha, schedule=S)
    o = parity.oracle_run(wl.code, fr, "spa", "f32", wl.max_iter, alpha=wl.alpha, schedule=S)
    s = parity.compare(g, o, wl.max_iter, RTOL32, atol=parity.ATOL32)
    assert s["oracle_ok"] == 64
    okf = g["ok"] == 1
    assert np.array_equal(syndromes(wl.code, g["bits"][okf]), fr.z[okf])
    assert np.all(g["iters"][~okf] == wl.max_iter)


def test_schedule_is_validated(ctx, codes):
    """An unknown schedule is an argument error; the batched decoder runs
    flooding only and says so."""
    import ctypes
    import torch
    from paper_2001_07979_amd import mbp
    code = codes[2]
    dc = _upload(ctx, code)
    F = 2
    llr = torch.zeros((F, code.n), device="cuda")
    z = torch.zeros((F, code.M), dtype=torch.uint8, device="cuda")
    out = [torch.empty((F, code.n), dtype=torch.uint8, device="cuda"),
           torch.empty(F, dtype=torch.int32, device="cuda"),
           torch.empty(F, dtype=torch.uint8, device="cuda")]
    for sched in (2, -1):
        p = mbp.mbp_params(mbp.MBP_ALGO_SPA, mbp.MBP_F32, 10, 1, 0.75, 20.0, 1, sched)
        rc = mbp.lib().mbp_decode(ctx.handle, dc.handle, ctypes.byref(p), F, llr.data_ptr(),
                                  z.data_ptr(), out[0].data_ptr(), out[1].data_ptr(),
                                  out[2].data_ptr(), None, None)
        assert rc == mbp.MBP_EINVAL
    items = [(dc, llr, z)]
    outs = [mbp.batch_outputs(dc, llr)]
    p = mbp.mbp_params(mbp.MBP_ALGO_NMS, mbp.MBP_F32, 10, 1, 0.75, 20.0, 1, 1)
    rc = mbp.lib().mbp_decode_batched(ctx.handle, 1, mbp._batches(items, outs), ctypes.byref(p),
                                      None, None)
    assert rc == mbp.MBP_EUNSUPPORTED


@pytest.mark.parametrize("u", [4, 5])
def test_serial_many_matrices(ctx, u):
    """Four matrices (the most whose per-matrix sums the serial variable
    passes keep) and five (every message summed again each phase): min-sum
    bit for bit against the binary32 oracle, sum-product FP64 against the
    oracle, both with compaction on a spread of stopping iterations."""
    code = peg_code(512, 96, u, {2: 0.3, 3: 0.7}, seed_base=7600 + u, name=f"peg-n512-u{u}")
    F = 140
    p = np.random.default_rng(u).permutation(np.geomspace(0.01, 0.09, F))
    fr = bsc_frames(code, F, p, seed=40 + u)
    dc = _upload(ctx, code)
    lam = parity.oracle_llr(fr, "f32")
    g = parity.gpu_run(ctx, dc, fr, "nms", "f32", 50, schedule=S)
    parity.assert_bitwise(g, parity.oracle_f32_run(code, fr, 50, lam=lam, schedule=S))
    lam64 = parity.oracle_llr(fr, "f64")
    g64 = parity.gpu_run(ctx, dc, fr, "spa", "f64", 50, llr=lam64, schedule=S)
    o64 = parity.oracle_run(code, fr, "spa", "f64", 50, lam=lam64, schedule=S)
    # FP64: 1e-9 within 8 iterations; these codes run frames to 35-50
    # iterations, where the two FP64 check rules' last-bit differences
    # (prefix/suffix products against the direct product) grow to ~1e-6
    # absolute around small L
    parity.compare(g64, o64, 50, RTOL64, long_after=8, long_rtol=1e-4, atol=1e-9)
    its = g["iters"]
    assert (its == 50).sum() > 20 and (its <= 4).sum() > 50  # the oracle: 39/34 and 75/77
