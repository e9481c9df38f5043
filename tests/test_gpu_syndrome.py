"""GPU: Alice's syndromes (eq. (1), mbp_syndrome) bit for bit against the
oracle's, through the C-ABI, from one frame to a ragged partial group, and at
the benchmark's full size."""
import numpy as np
import pytest

import oracle
from paper_2001_07979_amd.inputs import bsc_frames, peg_code
from paper_2001_07979_amd.inputs import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2001_07979_amd import mbp
    c = mbp.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("F", [1, 63, 64, 65, 130])
@pytest.mark.parametrize("which", ["n1000-u2", "n640-u3"])
def test_syndrome_matches_oracle(ctx, F, which):
    import torch
    from paper_2001_07979_amd import mbp
    code = (peg_code(1000, 260, 2, W.IRREGULAR_238, seed_base=7100, name="peg-n1000") if which == "n1000-u2"
            else peg_code(640, 200, 3, {2: 0.3, 3: 0.7}, seed_base=7300, name="peg-n640-u3"))
    rng = np.random.default_rng(F)
    x = rng.integers(0, 2, (F, code.n), dtype=np.uint8)
    x[0] *= 5  # nonzero bytes are ones
    dc = mbp.Code.from_inputs(ctx, code)
    z = mbp.syndrome(ctx, dc, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy(), oracle.syndrome(code, x))


def test_syndrome_full_size_and_decoder_round_trip(ctx):
    """n = 65536, 256 frames: every syndrome equal to the oracle's, and
    feeding them to the decoder recovers Alice's frames."""
    import torch
    from paper_2001_07979_amd import mbp
    wl = W.qkd_n65536()
    fr = wl.frames()
    dc = mbp.Code.from_inputs(ctx, wl.code)
    z = mbp.syndrome(ctx, dc, torch.from_numpy(fr.x).cuda())
    torch.cuda.synchronize()
    zc = z.cpu().numpy()
    assert np.array_equal(zc, oracle.syndrome(wl.code, fr.x))
    y = torch.from_numpy(fr.y).cuda()
    e = torch.from_numpy(fr.p).cuda()
    o = mbp.decode_from_bits(ctx, dc, y, e, z, algo="spa", max_iter=wl.max_iter)
    ok = o["ok"].cpu().numpy() == 1
    assert ok.mean() > 0.99 and np.array_equal(o["bits"].cpu().numpy()[ok], fr.x[ok])


def test_syndrome_edges(ctx):
    import torch
    from paper_2001_07979_amd import mbp
    code = peg_code(1000, 260, 2, W.IRREGULAR_238, seed_base=7100, name="peg-n1000")
    dc = mbp.Code.from_inputs(ctx, code)
    zero = mbp.syndrome(ctx, dc, torch.zeros((3, code.n), dtype=torch.uint8, device="cuda"))
    assert not zero.any().item()
    empty = mbp.syndrome(ctx, dc, torch.zeros((0, code.n), dtype=torch.uint8, device="cuda"))
    assert empty.shape == (0, code.M)
    assert mbp.lib().mbp_syndrome(ctx.handle, dc.handle, 2, None, None, None) == mbp.MBP_EINVAL
