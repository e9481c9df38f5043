"""CPU checks of the seeded input generators shared by the oracle tests, the
GPU parity tests and the benchmark (frames, syndromes, the mixed queue)."""
import numpy as np

from paper_2001_07979_amd.inputs import bsc_frames, code_from_dense, peg_code, syndromes
from paper_2001_07979_amd.inputs import workloads as W


def test_syndromes_are_the_dense_product():
    """Eq. (1): z^l = H_l x mod 2, against a dense matrix product, with an
    empty row in one matrix."""
    rng = np.random.default_rng(0)
    H1 = (rng.random((7, 23)) < 0.3).astype(np.uint8)
    H1[3] = 0
    H2 = (rng.random((5, 23)) < 0.4).astype(np.uint8)
    code = code_from_dense([H1, H2])
    x = rng.integers(0, 2, (9, 23), dtype=np.uint8)
    want = np.concatenate([(x.astype(np.int64) @ H.T.astype(np.int64)) % 2 for H in (H1, H2)], axis=1)
    assert np.array_equal(syndromes(code, x), want.astype(np.uint8))


def test_frames_do_not_depend_on_batch_size():
    code = peg_code(256, 64, 2, {3: 1.0}, seed_base=77)
    a = bsc_frames(code, 5, np.array([0.01, 0.02, 0.03, 0.04, 0.05]), seed=3)
    b = bsc_frames(code, 2, np.array([0.01, 0.02]), seed=3)
    assert np.array_equal(a.x[:2], b.x) and np.array_equal(a.y[:2], b.y)
    assert np.array_equal(a.z, syndromes(code, a.x))


def test_bsc_noise_rate():
    code = peg_code(4096, 1024, 1, {3: 1.0}, seed_base=78, max_depth=2)
    fr = bsc_frames(code, 8, 0.05, seed=4)
    rate = float((fr.x != fr.y).mean())
    assert abs(rate - 0.05) < 4 * np.sqrt(0.05 * 0.95 / fr.x.size)


def test_mixed_queue_shape():
    q = W.mixed_queue(2048, seed=4)
    cells = {f.cell for f in q}
    assert len(cells) == 18
    p = np.array([f.p for f in q])
    assert p.min() >= 0.01 and p.max() <= 0.08
    t = np.array([f.arrival_s for f in W.mixed_queue(2048, seed=4, rate_fps=1000.0)])
    assert np.all(np.diff(t) >= 0)
    assert abs(t[-1] - 2.048) < 0.3  # 2048 Poisson arrivals at 1000 per second
    # the arrival trace changes nothing else
    assert [f.cell for f in W.mixed_queue(2048, seed=4, rate_fps=1000.0)] == [f.cell for f in q]


def test_error_rate_for_an_efficiency():
    """e_for_efficiency inverts eq. (3) as the oracle computes it:
    f = m / (n h(e)) at the returned e, for the rates and bins of the sweeps."""
    import oracle
    n = 65536
    for rate in W.SWEEP_RATES:
        m = int(round((1 - rate) * n))
        for f in (1.1, 1.125, 1.3):
            e = W.e_for_efficiency(rate, f)
            assert 0 < e < 0.5
            assert abs(oracle.efficiency(m, n, e) - f) < 1e-4
