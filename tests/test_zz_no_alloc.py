"""The allocation-free syndrome call (mbp_syndrome_noalloc) against
mbp_syndrome, through the C-ABI: two calls in a row on one context, the
second with fewer frames, each bit for bit equal to the allocating call; a
size beyond the fixed scratch is refused before anything is enqueued."""
import numpy as np
import pytest

from paper_2001_07979_amd.inputs import bsc_frames
from paper_2001_07979_amd.inputs import workloads as W

pytestmark = pytest.mark.gpu


def test_noalloc_syndrome_equals_allocating_call():
    import torch
    from paper_2001_07979_amd import mbp
    ctx = mbp.Context(0)
    code = W.qkd_n65536(nframes=4).code
    dc = mbp.Code.from_inputs(ctx, code)
    dev = torch.device("cuda", 0)
    # 256 frames (4 groups), then 70 (2 groups, the second partly filled):
    # the second call reuses the scratch the first one left behind
    for F, seed in ((256, 901), (70, 902)):
        fr = bsc_frames(code, F, 0.02, seed=seed)
        x = torch.from_numpy(fr.x).to(dev)
        ref = mbp.syndrome(ctx, dc, x)
        out = torch.full((F, code.M), 7, dtype=torch.uint8, device=dev)
        mbp.syndrome_noalloc(ctx, dc, x, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"F={F}: syndromes differ"
        assert np.array_equal(out.cpu().numpy(), fr.z), f"F={F}: not Alice's syndromes"
    # ceil(2049 / 64) * 65536 words exceed the 2^21-word scratch
    big = torch.zeros((2049, code.n), dtype=torch.uint8, device=dev)
    zb = torch.zeros((2049, code.M), dtype=torch.uint8, device=dev)
    with pytest.raises(mbp.MbpError, match="exceed the scratch"):
        mbp.syndrome_noalloc(ctx, dc, big, zb)
    torch.cuda.synchronize()
    dc.close()
    ctx.close()
