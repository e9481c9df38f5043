"""GPU parity at points of the sweeps (u = 1, 2, 3 matrices; error rates up
to and past where single-matrix decoding fails; rates 0.5-0.8): sampled
frames against the oracle under the parity protocol, properties on all."""
import numpy as np
import pytest

from paper_2001_07979_amd.inputs import syndromes
from paper_2001_07979_amd.inputs import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2001_07979_amd import mbp
    c = mbp.Context(0)
    yield c
    c.close()


def _run(ctx, wl):
    import torch
    from paper_2001_07979_amd import mbp
    fr = wl.frames()
    dc = mbp.Code.from_inputs(ctx, wl.code)
    o = mbp.decode_from_bits(ctx, dc, torch.from_numpy(fr.y).cuda(), torch.from_numpy(fr.p).cuda(),
                             torch.from_numpy(fr.z).cuda(), algo=wl.algo, max_iter=wl.max_iter)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in o.items()}
    return fr, dict(bits=g["bits"], iters=g["iters"], ok=g["ok"], L=g["llr"].astype(np.float64))


@pytest.mark.parametrize("rate,u,e", [(0.5, 1, 0.08), (0.5, 2, 0.09), (0.8, 3, None)])
def test_sweep_points_match_oracle(ctx, rate, u, e):
    if e is None:
        e = W.e_for_efficiency(rate, 1.125)
    wl = W.sweep_workload(rate, u, e)
    fr, g = _run(ctx, wl)
    # every frame against the oracle (256 frames of n = 65536); the u = 1
    # point runs 17 to 35 iterations, where L drifts to 1.5e-4 (measured, a
    # frame at 25 iterations) with every decision the same
    o = parity.oracle_run(wl.code, fr, "spa", "f32", wl.max_iter)
    parity.compare(g, o, wl.max_iter, 1e-4, atol=parity.ATOL32, long_after=parity.SPA_LONG_AFTER,
                   long_rtol=1e-3)
    okf = g["ok"] == 1
    assert np.array_equal(syndromes(wl.code, g["bits"][okf]), fr.z[okf])
    assert np.all(g["iters"][~okf] == wl.max_iter)


def test_more_matrices_decode_more_frames(ctx):
    """At e = 0.09 and rate 0.5 one matrix is near its limit (f = 1.15) while
    the stacked u = 3 graph, with more checks than bits, decodes nearly all."""
    _, one = _run(ctx, W.sweep_workload(0.5, 1, 0.09))
    _, three = _run(ctx, W.sweep_workload(0.5, 3, 0.09))
    assert three["ok"].mean() > one["ok"].mean() + 0.2
