"""GPU tests of the batched persistent decode: frames of several codes in one
persistent launch, as eager calls, captured graphs and autotuned settings.
The reference is the plain decode of each batch alone (itself held to the
oracle by test_gpu_decode.py) plus the oracle's binary32 min-sum."""
import numpy as np
import pytest

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
def mix(ctx):
    """Three codes (n, u, rate and check degree all different) with 1, 70 and
    64 frames at mixed error rates."""
    import torch
    from paper_2001_07979_amd import mbp
    codes = [peg_code(1000, 260, 2, W.IRREGULAR_238, seed_base=7100, name="peg-n1000"),
             peg_code(640, 200, 3, {2: 0.3, 3: 0.7}, seed_base=7300, name="peg-n640-u3"),
             peg_code(2048, 256, 2, W.IRREGULAR_2310, seed_base=7400, name="peg-n2048")]
    nfr = [1, 70, 64]
    items, frames = [], []
    for k, (code, F) in enumerate(zip(codes, nfr)):
        fr = bsc_frames(code, F, np.geomspace(0.01, 0.06, F), seed=900 + k)
        dc = mbp.Code.from_inputs(ctx, code)
        lam = parity.oracle_llr(fr, "f32").astype(np.float32)
        items.append((dc, torch.from_numpy(lam).cuda(), torch.from_numpy(fr.z).cuda()))
        frames.append((code, fr, lam))
    return items, frames


def _np(o):
    return {k: (v.cpu().numpy().astype(np.float64) if k == "llr" else v.cpu().numpy())
            for k, v in o.items() if v is not None}


def _plain(ctx, items, T=60, early_exit=True):
    from paper_2001_07979_amd import mbp
    return [_np(mbp.decode(ctx, dc, llr, z, algo="nms", max_iter=T, early_exit=early_exit))
            for dc, llr, z in items]


def _same(a, b):
    for k in ("bits", "iters", "ok", "llr"):
        assert np.array_equal(a[k], b[k]), k


def test_batched_equals_plain_and_binary32_oracle(ctx, mix):
    from paper_2001_07979_amd import mbp
    import torch
    items, frames = mix
    outs = mbp.decode_batched(ctx, items, max_iter=60)
    torch.cuda.synchronize()
    got = [_np(o) for o in outs]
    for g, p in zip(got, _plain(ctx, items)):
        _same(g, p)
    for g, (code, fr, lam) in zip(got, frames):
        ref = parity.oracle_f32_run(code, fr, 60, lam=lam.astype(np.float64))
        parity.assert_bitwise(dict(bits=g["bits"], iters=g["iters"], ok=g["ok"], L=g["llr"]), ref)
    # the mix holds both outcomes (the oracle decodes 84 of the 135 frames)
    assert 60 < sum(int(g["ok"].sum()) for g in got) < sum(g["ok"].size for g in got)


@pytest.mark.parametrize("tuning", [dict(rows_per_wave=1, vars_per_wave=8, blocks_per_cu=1, schedule=1, compact=1),
                                    dict(rows_per_wave=8, vars_per_wave=1, blocks_per_cu=3, schedule=0, compact=0),
                                    dict(rows_per_wave=2, vars_per_wave=2, blocks_per_cu=4, schedule=1, compact=0),
                                    dict(rows_per_wave=4, vars_per_wave=4, blocks_per_cu=2, schedule=0, compact=1)])
def test_tunings_do_not_change_results(ctx, mix, tuning):
    from paper_2001_07979_amd import mbp
    items, _ = mix
    ref = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=60)]
    got = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=60, tuning=tuning)]
    for a, b in zip(got, ref):
        _same(a, b)


@pytest.fixture(scope="module")
def stragglers(ctx):
    """Batches whose frames converge at very different iterations or not at
    all (BSC p up to beyond the decoding threshold): 300 frames (5 groups) of
    the n=1000 code and 130 frames (3 groups) of the n=2048 rate-3/4 code, so
    the running frames shrink into fewer groups than they occupy."""
    import torch
    from paper_2001_07979_amd import mbp
    codes = [peg_code(1000, 260, 2, W.IRREGULAR_238, seed_base=7100, name="peg-n1000"),
             peg_code(2048, 256, 2, W.IRREGULAR_2310, seed_base=7400, name="peg-n2048")]
    specs = [(300, (0.02, 0.09), 910), (130, (0.004, 0.035), 911)]
    items, frames = [], []
    for code, (F, (p0, p1), seed) in zip(codes, specs):
        p = np.random.default_rng(seed).permutation(np.geomspace(p0, p1, F))
        fr = bsc_frames(code, F, p, seed=seed)
        dc = mbp.Code.from_inputs(ctx, code)
        lam = parity.oracle_llr(fr, "f32").astype(np.float32)
        items.append((dc, torch.from_numpy(lam).cuda(), torch.from_numpy(fr.z).cuda()))
        frames.append((code, fr, lam))
    return items, frames


def test_compaction_keeps_results(ctx, stragglers):
    """With compaction (running frames regrouped into spare groups as others
    retire) every output equals the decode without it, the plain decode, and,
    on sampled frames, the oracle's binary32 min-sum."""
    from paper_2001_07979_amd import mbp
    items, frames = stragglers
    T = 60
    on = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=T, tuning=dict(
        rows_per_wave=4, vars_per_wave=4, blocks_per_cu=2, schedule=0, compact=1))]
    off = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=T, tuning=dict(
        rows_per_wave=4, vars_per_wave=4, blocks_per_cu=2, schedule=0, compact=0))]
    for a, b in zip(on, off):
        _same(a, b)
    for a, b in zip(on, _plain(ctx, items, T=T)):
        _same(a, b)
    for g, (code, fr, lam) in zip(on, frames):
        idx = np.random.default_rng(5).choice(fr.nframes, 12, replace=False)
        ref = parity.oracle_f32_run(code, fr, T, idx=idx, lam=lam.astype(np.float64))
        parity.assert_bitwise(dict(bits=g["bits"], iters=g["iters"], ok=g["ok"], L=g["llr"]), ref, idx=idx)
    # the mix really has stragglers and failures
    its = np.concatenate([g["iters"] for g in on])
    assert (its == T).sum() > 100 and (its <= 5).sum() > 80


def test_edge_cases(ctx, mix, stragglers):
    """Iteration limits 1 and 2 (no room for compaction), a batch whose every
    frame fails (random syndromes), and many small batches at once: all equal
    to the plain decode."""
    import torch
    from paper_2001_07979_amd import mbp
    items, _ = mix
    for T in (1, 2):
        got = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=T)]
        for g, p in zip(got, _plain(ctx, items, T=T)):
            _same(g, p)
            assert np.all(g["iters"] <= T)
    dc, llr, z = stragglers[0][0]
    bad = torch.from_numpy(np.random.default_rng(8).integers(0, 2, tuple(z.shape)).astype(np.uint8)).cuda()
    got = _np(mbp.decode_batched(ctx, [(dc, llr, bad)], max_iter=12)[0])
    assert np.all(got["ok"] == 0) and np.all(got["iters"] == 12)
    _same(got, _plain(ctx, [(dc, llr, bad)], T=12)[0])
    many = []
    for k in range(20):
        d, l, zz = items[k % len(items)]
        F = 1 + (k * 7) % 5
        many.append((d, l[:F].contiguous(), zz[:F].contiguous()))
    got = [_np(o) for o in mbp.decode_batched(ctx, many, max_iter=30)]
    for g, p in zip(got, _plain(ctx, many, T=30)):
        _same(g, p)


def test_fixed_iterations(ctx, mix):
    from paper_2001_07979_amd import mbp
    items, _ = mix
    got = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=9, early_exit=False)]
    for g, p in zip(got, _plain(ctx, items, T=9, early_exit=False)):
        _same(g, p)
        assert np.all(g["iters"] == 9)


def test_graph_plan_replays(ctx, mix):
    """A captured plan, replayed three times with eager work in between,
    matches the eager decode every time."""
    import torch
    from paper_2001_07979_amd import mbp
    items, _ = mix
    ref = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=60)]
    outs = [mbp.batch_outputs(dc, llr) for dc, llr, _ in items]
    plan = mbp.Plan(ctx, items, outs, max_iter=60)
    for rep in range(3):
        for o in outs:
            for v in o.values():
                v.zero_()
        plan.launch()
        plan.wait()
        got = [_np(o) for o in outs]
        for a, b in zip(got, ref):
            _same(a, b)
        _plain(ctx, items[:1])  # eager work between replays
        torch.cuda.synchronize()
    plan.close()


def test_autotune_picks_a_valid_setting(ctx, mix, tmp_path):
    from paper_2001_07979_amd import mbp
    items, _ = mix
    cache = str(tmp_path / "tune.txt")
    t = mbp.autotune(ctx, items, max_iter=60, cache_path=cache)
    assert 1 <= t["rows_per_wave"] <= 64 and t["schedule"] in (0, 1)
    assert mbp.autotune(ctx, items, max_iter=60, cache_path=cache) == t  # cached
    ref = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=60)]
    got = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=60, tuning=t)]
    for a, b in zip(got, ref):
        _same(a, b)


def test_batched_rejects_what_it_does_not_run(ctx, mix):
    """FP64, the matrix-serial schedule and sum-product on checks of degree
    above 34 are refused before any launch (EUNSUPPORTED)."""
    import ctypes
    from paper_2001_07979_amd import mbp
    items, _ = mix
    outs = [mbp.batch_outputs(dc, llr) for dc, llr, _ in items]
    arr = mbp._batches(items, outs)
    for algo, dtype, sched in ((mbp.MBP_ALGO_SPA, mbp.MBP_F64, 0), (mbp.MBP_ALGO_NMS, mbp.MBP_F32, 1)):
        p = mbp.mbp_params(algo, dtype, 10, 1, 0.75, 20.0, 1, sched)
        rc = mbp.lib().mbp_decode_batched(ctx.handle, len(items), arr, ctypes.byref(p), None, None)
        assert rc == mbp.MBP_EUNSUPPORTED
    wide = peg_code(512, 32, 1, {3: 1.0}, seed_base=7500, name="peg-n512-dc48")  # check degree 48
    assert max(int(np.diff(r).max()) for r in wide.row_ptr) > 34
    import torch
    with mbp.Code.from_inputs(ctx, wide) as dc:
        llr = torch.ones((3, 512), dtype=torch.float32, device="cuda")
        z = torch.zeros((3, wide.M), dtype=torch.uint8, device="cuda")
        with pytest.raises(mbp.MbpError, match="34"):
            mbp.decode_batched(ctx, [(dc, llr, z)], algo="spa")
        mbp.decode_batched(ctx, [(dc, llr, z)], algo="nms")  # min-sum takes any degree


@pytest.fixture(scope="module")
def spa_mix(ctx):
    """Codes within the batched sum-product rule's check degree (<= 34):
    n=1000 (degrees 16-18), n=640 u=3, n=2048 rate 3/4 with 512 checks per
    matrix (degrees 19-20); 1, 70 and 64 frames at mixed error rates, and 300
    stragglers of the n=1000 code up to beyond its threshold."""
    import torch
    from paper_2001_07979_amd import mbp
    codes = [peg_code(1000, 260, 2, W.IRREGULAR_238, seed_base=7100, name="peg-n1000"),
             peg_code(640, 200, 3, {2: 0.3, 3: 0.7}, seed_base=7300, name="peg-n640-u3"),
             peg_code(2048, 512, 2, W.IRREGULAR_2310, seed_base=7600, name="peg-n2048-m512"),
             peg_code(1000, 260, 2, W.IRREGULAR_238, seed_base=7100, name="peg-n1000")]
    specs = [(1, (0.01, 0.06), 930), (70, (0.01, 0.06), 931), (64, (0.02, 0.12), 932), (300, (0.02, 0.09), 933)]
    items, frames = [], []
    for code, (F, (p0, p1), seed) in zip(codes, specs):
        assert max(int(np.diff(r).max()) for r in code.row_ptr) <= 34
        p = np.random.default_rng(seed).permutation(np.geomspace(p0, p1, F))
        fr = bsc_frames(code, F, p, seed=seed)
        dc = mbp.Code.from_inputs(ctx, code)
        lam = parity.oracle_llr(fr, "f32").astype(np.float32)
        items.append((dc, torch.from_numpy(lam).cuda(), torch.from_numpy(fr.z).cuda()))
        frames.append((code, fr, lam))
    yield items, frames
    for dc, _, _ in items:
        dc.close()


def test_batched_sum_product_equals_plain_and_oracle(ctx, spa_mix):
    """Sum-product in the persistent kernel: bit for bit the plain decode's
    sum-product (the same row rule), with and without compaction, over
    several tunings; and the FP64 oracle's results under the parity
    protocol."""
    from paper_2001_07979_amd import mbp
    for items, frames, T in ((spa_mix[0][:3], spa_mix[1][:3], 60), (spa_mix[0][3:], spa_mix[1][3:], 60)):
        plain = [_np(mbp.decode(ctx, dc, llr, z, algo="spa", max_iter=T)) for dc, llr, z in items]
        for tuning in (None, dict(rows_per_wave=1, vars_per_wave=8, blocks_per_cu=1, schedule=1, compact=1),
                       dict(rows_per_wave=8, vars_per_wave=2, blocks_per_cu=2, schedule=0, compact=0)):
            got = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=T, algo="spa", tuning=tuning)]
            for g, p in zip(got, plain):
                _same(g, p)
        # every frame against the oracle; the stragglers up to BSC 0.09 run to
        # T = 60, where L drifts to 2.9e-3 (measured, a frame at 41
        # iterations) with every decision the same
        for g, (code, fr, lam) in zip(got, frames):
            o = parity.oracle_run(code, fr, "spa", "f32", T, lam=lam.astype(np.float64))
            parity.compare(dict(bits=g["bits"], iters=g["iters"], ok=g["ok"], L=g["llr"]), o, T, 1e-4,
                           atol=parity.ATOL32, long_after=parity.SPA_LONG_AFTER, long_rtol=1e-2)


def test_graph_plan_sum_product(ctx, spa_mix):
    """A captured sum-product plan (its persistent node marked cooperative)
    replays twice to the eager result."""
    import torch
    from paper_2001_07979_amd import mbp
    items = spa_mix[0]
    ref = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=60, algo="spa")]
    outs = [mbp.batch_outputs(dc, llr) for dc, llr, _ in items]
    with mbp.Plan(ctx, items, outs, max_iter=60, algo="spa") as plan:
        for rep in range(2):
            for o in outs:
                for v in o.values():
                    v.zero_()
            plan.launch()
            plan.wait()
            for a, b in zip([_np(o) for o in outs], ref):
                _same(a, b)
            _plain(ctx, items[:1])
            torch.cuda.synchronize()


@pytest.fixture(scope="module")
def queue_cells(ctx):
    """One batch per (n, rate, u) cell of the mixed serving queue (n in
    {16384, 65536, 2^18}, rate in {0.5, 0.7, 0.85}, u in {2, 3}, the queue's
    own codes), 6 frames each at error rates spread log-uniformly over the
    queue's [0.01, 0.08], so every cell has frames that decode and, at the
    high rates, frames that fail."""
    import torch
    from paper_2001_07979_amd import mbp
    items, frames = [], []
    for k, (n, rate, u) in enumerate([(n, r, u) for n in W.MIXED_N for r in W.MIXED_RATES for u in (2, 3)]):
        code = W.mixed_code(n, rate, u)
        p = np.exp(np.random.default_rng(40 + k).uniform(np.log(0.01), np.log(0.08), 6))
        fr = bsc_frames(code, 6, p, seed=4000 + k)
        dc = mbp.Code.from_inputs(ctx, code)
        lam = parity.oracle_llr(fr, "f32").astype(np.float32)
        items.append((dc, torch.from_numpy(lam).cuda(), torch.from_numpy(fr.z).cuda()))
        frames.append((code, fr, lam))
    yield items, frames
    for dc, _, _ in items:
        dc.close()


def test_queue_cells_min_sum_bitwise_with_binary32_oracle(ctx, queue_cells):
    """All 18 cells in one batched launch (min-sum, alpha 0.75, T = 30):
    every frame bit for bit against the oracle's binary32 min-sum, and
    equal to the plain decode of each cell."""
    from paper_2001_07979_amd import mbp
    items, frames = queue_cells
    T = 30
    got = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=T)]
    for g, p in zip(got, _plain(ctx, items, T=T)):
        _same(g, p)
    for g, (code, fr, lam) in zip(got, frames):
        ref = parity.oracle_f32_run(code, fr, T, lam=lam.astype(np.float64))
        parity.assert_bitwise(dict(bits=g["bits"], iters=g["iters"], ok=g["ok"], L=g["llr"]), ref)
    oks = np.concatenate([g["ok"] for g in got])
    assert 0 < oks.sum() < oks.size


def test_queue_cells_sum_product_against_oracle(ctx, queue_cells):
    """The same 18 cells with sum-product (T = 30): equal to the plain
    decode bit for bit, and every frame under the parity protocol against
    the FP64 oracle."""
    from paper_2001_07979_amd import mbp
    items, frames = queue_cells
    T = 30
    got = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=T, algo="spa")]
    for g, (dc, llr, z) in zip(got, items):
        _same(g, _np(mbp.decode(ctx, dc, llr, z, algo="spa", max_iter=T)))
    for g, (code, fr, lam) in zip(got, frames):
        o = parity.oracle_run(code, fr, "spa", "f32", T, lam=lam.astype(np.float64))
        parity.compare(dict(bits=g["bits"], iters=g["iters"], ok=g["ok"], L=g["llr"]), o, T, 1e-4,
                       atol=parity.ATOL32)


def test_queue_matches_batched_decode(ctx, mix):
    """Frames submitted to the serving queue in two submits and flushes (and
    an empty flush) decode exactly as the batched call; poll reaches the
    frame count, wait returns it."""
    import time
    from paper_2001_07979_amd import mbp
    items, _ = mix
    ref = [_np(o) for o in mbp.decode_batched(ctx, items, max_iter=60)]
    q = mbp.Queue(ctx, max_iter=60)
    assert q.poll() == 0
    outs = [mbp.batch_outputs(dc, llr) for dc, llr, _ in items]
    q.submit(items[:1], outs[:1])
    q.flush()
    q.submit(items[1:], outs[1:])
    q.flush()
    q.flush()  # nothing pending
    total = sum(int(llr.shape[0]) for _, llr, _ in items)
    t0 = time.time()
    while q.poll() < total and time.time() - t0 < 60:
        time.sleep(0.001)
    assert q.wait() == total
    for a, b in zip([_np(o) for o in outs], ref):
        _same(a, b)
    q.close()
    with pytest.raises(mbp.MbpError):
        mbp.Queue(ctx, max_iter=0)
