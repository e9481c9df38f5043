"""GPU parity of the unrolled min-sum forward and its hand-written adjoint.

The forward is held bit for bit to the plain decoder and to the oracle's
binary32 min-sum; the gradients to the FP64 oracle's exact reverse-mode
gradient, to central differences of the GPU forward, and to themselves under
a different checkpoint spacing.
"""
import numpy as np
import pytest

import oracle
from paper_2001_07979_amd.inputs import bsc_frames, peg_code
from paper_2001_07979_amd.inputs import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2001_07979_amd import mbp
    c = mbp.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ragged_code():
    return peg_code(1000, 260, 2, W.IRREGULAR_238, seed_base=7100, name="peg-n1000")


def _tensors(fr, alpha):
    import torch
    lam = oracle.llr_from_bits(fr.y, fr.p).astype(np.float32)
    return (torch.from_numpy(lam).cuda(), torch.from_numpy(fr.z).cuda(),
            torch.from_numpy(alpha.astype(np.float32)).cuda(), lam.astype(np.float64))


def _run(ctx, dc, llr, z, alpha, gL=None, ckpt=5, clip=20.0):
    import torch
    from paper_2001_07979_amd import mbp
    K = alpha.shape[0]
    ws = torch.empty(mbp.unrolled_workspace_bytes(dc, llr.shape[0], K, ckpt), dtype=torch.uint8,
                     device="cuda")
    L = mbp.nms_unrolled_fwd(ctx, dc, llr, z, alpha, ckpt, clip, ws)
    if gL is None:
        torch.cuda.synchronize()
        return L.cpu().numpy().astype(np.float64)
    g_llr, g_alpha = mbp.nms_unrolled_bwd(ctx, dc, llr, z, alpha, gL, ckpt, clip, ws)
    torch.cuda.synchronize()
    return (L.cpu().numpy().astype(np.float64), g_llr.cpu().numpy().astype(np.float64),
            g_alpha.cpu().numpy().astype(np.float64))


def test_forward_is_the_plain_decoder_and_binary32_oracle(ctx, ragged_code):
    from paper_2001_07979_amd import mbp
    fr = bsc_frames(ragged_code, 70, np.linspace(0.02, 0.05, 70), seed=600)
    K = 7
    dc = mbp.Code.from_inputs(ctx, ragged_code)
    alpha = np.full((K, 2), 0.75)
    llr, z, a, lam = _tensors(fr, alpha)
    L = _run(ctx, dc, llr, z, a)
    g = parity.gpu_run(ctx, dc, fr, "nms", "f32", K, early_exit=False)
    assert np.array_equal(L, g["L"])
    alpha = np.random.default_rng(2).uniform(0.5, 1.0, (K, 2)).astype(np.float32).astype(np.float64)
    llr, z, a, lam = _tensors(fr, alpha)
    L = _run(ctx, dc, llr, z, a)
    ref = oracle.decode_nms_f32(ragged_code, lam, fr.z, max_iter=K, early_exit=False, alpha_tl=alpha)
    assert np.array_equal(L, ref["L"])


def _grad_close(g, ref, rtol, floor):
    """Coordinates within rtol of the reference plus floor x its rms."""
    return np.abs(g - ref) <= rtol * np.abs(ref) + floor * np.sqrt(np.mean(ref ** 2))


@pytest.mark.parametrize("ties", [False, True])
def test_gradient_matches_fp64_oracle(ctx, ragged_code, ties):
    """Against the oracle's FP64 reverse sweep of the same binary32 forward
    trajectory (same minima, signs and caps): every coordinate to 1e-4.
    Against the all-FP64 oracle, whose trajectory rounds differently: tie-free
    LLRs (a continuous random gain on each) agree on nearly every frame; BSC
    LLRs, which all share one magnitude per frame, make the minima exact ties
    that the two trajectories later resolve differently, so there the
    subgradients differ and only the forward is compared."""
    from paper_2001_07979_amd import mbp
    import torch
    fr = bsc_frames(ragged_code, 32, np.linspace(0.03, 0.06, 32), seed=500)
    K = 5
    rng = np.random.default_rng(1)
    alpha = rng.uniform(0.6, 0.9, (K, 2)).astype(np.float32).astype(np.float64)
    dc = mbp.Code.from_inputs(ctx, ragged_code)
    _, z, a, lam = _tensors(fr, alpha)
    if not ties:
        lam = (lam * rng.uniform(0.7, 1.3, size=lam.shape)).astype(np.float32).astype(np.float64)
    llr = torch.from_numpy(lam.astype(np.float32)).cuda()
    w = np.random.default_rng(3).normal(size=lam.shape)  # J = sum w * L^K
    L, g_llr, g_alpha = _run(ctx, dc, llr, z, a, gL=torch.from_numpy(w.astype(np.float32)).cuda())

    L32, glam32, galpha32 = oracle.nms_unrolled(ragged_code, K, alpha, lam, fr.z, gL=w, binary32=True)
    assert np.array_equal(L, L32)
    close = _grad_close(g_llr, glam32, 1e-4, 1e-5)
    assert close.all(), f"{(~close).sum()} of {close.size} coordinates differ"
    np.testing.assert_allclose(g_alpha, galpha32, rtol=1e-4, atol=1e-5 * np.abs(galpha32).max())

    L64, glam64, galpha64 = oracle.nms_unrolled(ragged_code, K, alpha, lam, fr.z, gL=w)
    # the FP32 forward drifts from FP64 by rounding amplified over K checks
    # (measured up to 8.5e-5 at |L| up to 25 here)
    np.testing.assert_allclose(L, L64, rtol=1e-5, atol=2e-4)
    if not ties:
        frames_ok = _grad_close(g_llr, glam64, 1e-4, 1e-4).all(axis=1)
        assert frames_ok.mean() >= 0.9, f"{(~frames_ok).sum()} of {frames_ok.size} frames differ"
        assert np.linalg.norm(g_llr - glam64) <= 2e-2 * np.linalg.norm(glam64)
        np.testing.assert_allclose(g_alpha, galpha64, rtol=1e-1, atol=1e-3 * np.abs(galpha64).max())


def test_checkpoint_spacing_does_not_change_gradients(ctx, ragged_code):
    from paper_2001_07979_amd import mbp
    import torch
    fr = bsc_frames(ragged_code, 40, 0.05, seed=501)
    K = 9
    alpha = np.random.default_rng(4).uniform(0.6, 0.9, (K, 2))
    dc = mbp.Code.from_inputs(ctx, ragged_code)
    llr, z, a, lam = _tensors(fr, alpha)
    gL = torch.from_numpy(np.random.default_rng(5).normal(size=lam.shape).astype(np.float32)).cuda()
    ref = _run(ctx, dc, llr, z, a, gL=gL, ckpt=K)
    for ck in (1, 2, 4, 5):
        got = _run(ctx, dc, llr, z, a, gL=gL, ckpt=ck)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), f"ckpt_every={ck}"


def test_gradient_matches_central_differences(ctx):
    """Central differences of the GPU forward on a small code, where the map
    is linear across the step (both one-sided slopes agree)."""
    from paper_2001_07979_amd import mbp
    import torch
    code = peg_code(48, 24, 2, {3: 1.0}, seed_base=9100)
    fr = bsc_frames(code, 2, 0.08, seed=41)
    K = 5
    rng = np.random.default_rng(1)
    alpha = rng.uniform(0.6, 0.9, (K, 2))
    dc = mbp.Code.from_inputs(ctx, code)
    llr, z, a, lam = _tensors(fr, alpha)
    lam = lam * rng.uniform(0.7, 1.3, size=lam.shape)
    llr = torch.from_numpy(lam.astype(np.float32)).cuda()
    lam = llr.cpu().numpy().astype(np.float64)
    w = rng.normal(size=lam.shape)
    _, g_llr, g_alpha = _run(ctx, dc, llr, z, a, gL=torch.from_numpy(w.astype(np.float32)).cuda())

    def J_lam(x):
        return float((_run(ctx, dc, torch.from_numpy(x.astype(np.float32)).cuda(), z, a) * w).sum())

    def J_alpha(x):
        return float((_run(ctx, dc, llr, z, torch.from_numpy(x.astype(np.float32)).cuda()) * w).sum())

    eps = 1e-3
    checked = 0
    for i in rng.choice(lam.size, 30, replace=False):
        xp, xm = lam.copy(), lam.copy()
        xp.flat[i] += eps
        xm.flat[i] -= eps
        jp, j0, jm = J_lam(xp), J_lam(lam), J_lam(xm)
        right, left = (jp - j0) / eps, (j0 - jm) / eps
        if abs(right - left) <= 2e-2 * (1 + abs(right)):
            fd = 0.5 * (right + left)
            assert g_llr.flat[i] == pytest.approx(fd, rel=2e-2, abs=2e-2)
            checked += 1
    assert checked >= 15
    checked = 0
    for i in range(alpha.size):
        xp, xm = alpha.copy(), alpha.copy()
        xp.flat[i] += eps
        xm.flat[i] -= eps
        jp, j0, jm = J_alpha(xp), J_alpha(alpha), J_alpha(xm)
        right, left = (jp - j0) / eps, (j0 - jm) / eps
        if abs(right - left) <= 2e-2 * (1 + abs(right)):
            assert g_alpha.flat[i] == pytest.approx(0.5 * (right + left), rel=2e-2, abs=5e-2)
            checked += 1
    assert checked >= 4


def test_autograd_bce_training_step(ctx):
    """K=20 unrolled min-sum on the n=16384 code as a torch autograd op: the
    BCE loss of sigma(-L^K) against Alice's bits back-propagates through the
    HIP adjoint into llr and alpha, and matches the oracle's FP64 reverse sweep of the
    same binary32 trajectory."""
    import torch
    from paper_2001_07979_amd import mbp
    wl = W.unrolled_n16384(nframes=8)
    fr = wl.frames()
    K = 20
    dc = mbp.Code.from_inputs(ctx, wl.code)
    lam = oracle.llr_from_bits(fr.y, fr.p).astype(np.float32)
    llr = torch.from_numpy(lam).cuda().requires_grad_(True)
    alpha = torch.full((K, 2), 0.75, device="cuda", requires_grad=True)
    z = torch.from_numpy(fr.z).cuda()
    x = torch.from_numpy(fr.x.astype(np.float32)).cuda()
    L = mbp.unrolled_nms(ctx, dc, llr, z, alpha, ckpt_every=5)
    loss = torch.nn.functional.binary_cross_entropy_with_logits(-L, x)
    loss.backward()
    a64 = np.full((K, 2), 0.75)
    L32 = oracle.nms_unrolled(wl.code, K, a64, lam.astype(np.float64), fr.z, binary32=True)
    Lg = L.detach().cpu().numpy().astype(np.float64)
    assert np.array_equal(Lg, L32)
    # dJ/dL^K of the mean BCE of sigma(-L) against x, from the binary32 L
    sig = 1.0 / (1.0 + np.exp(L32))
    gL = -(sig - fr.x) / fr.x.size
    _, glam32, galpha32 = oracle.nms_unrolled(wl.code, K, a64, lam.astype(np.float64), fr.z, gL=gL,
                                              binary32=True)
    g = llr.grad.cpu().numpy().astype(np.float64)
    # gL itself is computed in FP32 by torch here and in FP64 by the test
    close = _grad_close(g, glam32, 1e-3, 1e-4)
    assert close.mean() >= 0.999, f"{(~close).sum()} of {close.size} coordinates differ"
    np.testing.assert_allclose(alpha.grad.cpu().numpy(), galpha32, rtol=1e-3,
                               atol=1e-4 * np.abs(galpha32).max() + 1e-30)
    L64 = oracle.nms_unrolled(wl.code, K, a64, lam.astype(np.float64), fr.z)
    np.testing.assert_allclose(Lg, L64, rtol=1e-4, atol=1e-3)


def test_config_scale_gradients(ctx):
    """The configured training workload: the u=2 n=16384 rate-1/2 code, K=20,
    checkpoints every 5, 512 frames at BSC p ~ U[0.04, 0.08], weights alpha
    [20, 2] drawn in [0.65, 0.85], objective J = sum w * L^K with random w.

    * Forward and backward on all 512 frames; on 8 sampled frames L^K bit
      for bit against the oracle's binary32 forward and dJ/dllr against its
      FP64 reverse sweep of that trajectory; dJ/dalpha over all frames equal
      to the sum over 8 launches of 64 frames each (a different reduction
      grouping: FP32 rounding only) and, for the 8-frame launch, to the oracle.
    * Central differences (eps = 1e-3) of the GPU forward on 2 tie-free
      frames: 64 llr coordinates (32 where w is nonzero, 32 anywhere) and all
      40 weights, on coordinates where both one-sided slopes agree (the map
      is piecewise linear)."""
    import torch
    from paper_2001_07979_amd import mbp
    wl = W.unrolled_n16384(nframes=512)
    fr = wl.frames()
    code, K, F = wl.code, wl.max_iter, 512
    rng = np.random.default_rng(20)
    alpha = rng.uniform(0.65, 0.85, (K, 2)).astype(np.float32).astype(np.float64)
    with mbp.Code.from_inputs(ctx, code) as dc:
        llr, z, a, lam = _tensors(fr, alpha)
        w = rng.normal(size=lam.shape)
        wt = torch.from_numpy(w.astype(np.float32)).cuda()
        L, g_llr, g_alpha = _run(ctx, dc, llr, z, a, gL=wt)
        idx = np.array([0, 63, 64, 200, 317, 384, 450, 511])
        L32, glam32, galpha32 = oracle.nms_unrolled(code, K, alpha, lam[idx], fr.z[idx], gL=w[idx], binary32=True)
        assert np.array_equal(L[idx], L32)
        close = _grad_close(g_llr[idx], glam32, 1e-4, 1e-5)
        assert close.all(), f"{(~close).sum()} of {close.size} coordinates differ"
        assert np.abs(g_alpha).max() > 1.0  # a gradient that carries signal
        parts = np.zeros_like(g_alpha)
        for c0 in range(0, F, 64):
            parts += _run(ctx, dc, llr[c0:c0 + 64].contiguous(), z[c0:c0 + 64].contiguous(), a,
                          gL=wt[c0:c0 + 64].contiguous())[2]
        np.testing.assert_allclose(g_alpha, parts, rtol=1e-5, atol=1e-6 * np.abs(parts).max())
        sub = _run(ctx, dc, llr[idx].contiguous(), z[idx].contiguous(), a, gL=wt[idx].contiguous())
        np.testing.assert_allclose(sub[2], galpha32, rtol=1e-4, atol=1e-5 * np.abs(galpha32).max())

        # central differences on two tie-free frames with a sparse objective
        two = [np.argmax(fr.p), np.argsort(fr.p)[-2]]  # the two noisiest frames
        lam2 = (lam[two] * rng.uniform(0.7, 1.3, (2, code.n))).astype(np.float32).astype(np.float64)
        z2 = z[torch.tensor(two, device="cuda")].contiguous()
        w2 = np.zeros_like(lam2)
        sup = rng.choice(lam2.size, 256, replace=False)
        w2.flat[sup] = rng.normal(size=256)
        x2 = torch.from_numpy(lam2.astype(np.float32)).cuda()
        _, g2, ga2 = _run(ctx, dc, x2, z2, a, gL=torch.from_numpy(w2.astype(np.float32)).cuda())

        def J(l, al):
            return float((_run(ctx, dc, torch.from_numpy(l.astype(np.float32)).cuda(), z2,
                               torch.from_numpy(al.astype(np.float32)).cuda()) * w2).sum())

        eps = 1e-3
        j0 = J(lam2, alpha)
        coords = np.concatenate([sup[:32], rng.choice(lam2.size, 32, replace=False)])
        checked = 0
        for i in coords:
            xp, xm = lam2.copy(), lam2.copy()
            xp.flat[i] += eps
            xm.flat[i] -= eps
            right, left = (J(xp, alpha) - j0) / eps, (j0 - J(xm, alpha)) / eps
            if abs(right - left) <= 2e-2 * (1 + abs(right)):
                fd = 0.5 * (right + left)
                assert abs(g2.flat[i] - fd) <= 1e-2 * (1 + abs(fd)), (i, g2.flat[i], fd)
                checked += 1
        assert checked >= 48
        checked = 0
        for k in range(alpha.size):
            ap, am = alpha.copy(), alpha.copy()
            ap.flat[k] += eps
            am.flat[k] -= eps
            right, left = (J(lam2, ap) - j0) / eps, (j0 - J(lam2, am)) / eps
            if abs(right - left) <= 2e-2 * (1 + abs(right)):
                fd = 0.5 * (right + left)
                assert abs(ga2.flat[k] - fd) <= 1e-3 * (1 + abs(fd)), (k, ga2.flat[k], fd)
                checked += 1
        assert checked >= 30
