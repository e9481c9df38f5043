"""GPU PEG construction (mbp_peg_build): the matrices it builds keep the
properties the PEG procedure guarantees (Sec. 2 names PEG, after Hu,
Eleftheriou and Arnold): every variable gets exactly its degree, no check
holds a variable twice, rows are ascending, the depth bound b leaves no
cycle shorter than 2 (b + 2), and lowest-degree choices keep the check
degrees close together. The result depends only on the arguments, and the
codes decode like the host generator's."""
from collections import deque

import numpy as np
import pytest

from paper_2001_07979_amd.inputs import Code, bsc_frames, degree_sequence, peg_code
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


def _shortest_other_path(rows, cols_of, c, v, limit):
    """Length of the shortest path from check c to variable v that does not
    use the edge (c, v), in edges, or None if longer than limit."""
    seen_c, seen_v = {c}, set()
    q = deque([(c, True, 0)])  # (node, is_check, distance)
    while q:
        x, is_check, d = q.popleft()
        if d >= limit:
            continue
        nbrs = rows[x] if is_check else cols_of[x]
        for y in nbrs:
            if is_check and x == c and y == v:
                continue  # the edge itself
            if is_check:
                if y == v:
                    return d + 1
                if y not in seen_v:
                    seen_v.add(y)
                    q.append((y, False, d + 1))
            elif y not in seen_c:
                seen_c.add(y)
                q.append((y, True, d + 1))
    return None


def _check_matrix(rp, ci, n, m, dv, bound):
    assert rp[0] == 0 and rp[-1] == ci.size == dv.sum()
    rows = [ci[rp[r]:rp[r + 1]] for r in range(m)]
    for r in rows:
        assert np.all(np.diff(r) > 0), "rows ascending, no variable twice"
    assert np.array_equal(np.bincount(ci, minlength=n), dv), "every variable gets its degree"
    deg = np.diff(rp)
    assert deg.max() - deg.min() <= 3, (deg.min(), deg.max())
    cols_of = [[] for _ in range(n)]
    for r, row in enumerate(rows):
        for v in row:
            cols_of[v].append(r)
    # the depth bound: the other path between an edge's ends is >= 2b + 3
    # edges, i.e. no cycle through the edge is shorter than 2 (b + 2)
    need = 2 * bound + 3
    for r, row in enumerate(rows):
        for v in row:
            d = _shortest_other_path(rows, cols_of, r, int(v), need - 1)
            assert d is None, f"edge ({r}, {v}) closes a cycle of {d + 1}"
    return deg


@pytest.mark.parametrize("depth", [0, 1, 2, -1])
def test_peg_properties(ctx, depth):
    """A sparse code (degrees 2 and 3, check degree 5), where two levels of
    the search reach about 130 of the 1000 checks, so every edge has
    unreached candidates and the bound holds for every edge."""
    from paper_2001_07979_amd import mbp
    n, m = 2000, 1000
    dv = degree_sequence(n, m, {2: 0.5, 3: 0.5})
    rps, cis = mbp.peg_build(ctx, n, m, dv, [11, 12], depth)
    for rp, ci in zip(rps, cis):
        # the unbounded search stops only at the farthest level: no 4-cycle
        _check_matrix(rp, ci, n, m, dv, depth if depth >= 0 else 1)
    assert not np.array_equal(cis[0], cis[1]), "different seeds, different matrices"


def test_peg_is_deterministic(ctx):
    from paper_2001_07979_amd import mbp
    n, m = 4096, 2048
    dv = degree_sequence(n, m, W.IRREGULAR_2310)
    a = mbp.peg_build(ctx, n, m, dv, [5, 6, 7], 2)
    b = mbp.peg_build(ctx, n, m, dv, [5, 6, 7], 2)
    for x, y in zip(a[0] + a[1], b[0] + b[1]):
        assert np.array_equal(x, y)


def test_peg_codes_decode_like_host_codes(ctx):
    """A u = 2 rate-1/2 code from the GPU builder and one from the host
    generator (same degrees, same depth bound) decode the same frames at BSC
    0.05 with the same success: every frame, in a similar number of
    iterations."""
    import torch
    from paper_2001_07979_amd import mbp
    n, m = 16384, 8192
    dv = degree_sequence(n, m, W.IRREGULAR_238)
    rps, cis = mbp.peg_build(ctx, n, m, dv, [900, 901], 2)
    gpu_code = Code(n=n, row_ptr=rps, col_idx=cis, name="gpu-peg")
    host_code = peg_code(n, m, 2, W.IRREGULAR_238, seed_base=900, max_depth=2, name="host-peg")
    dev = torch.device("cuda", ctx.device)
    its = []
    for code in (gpu_code, host_code):
        fr = bsc_frames(code, 128, 0.05, seed=17)
        dc = mbp.Code.from_inputs(ctx, code)
        out = mbp.decode_from_bits(ctx, dc, torch.from_numpy(fr.y).to(dev), torch.from_numpy(fr.p).to(dev),
                                   torch.from_numpy(fr.z).to(dev), algo="spa", max_iter=100)
        torch.cuda.synchronize()
        assert np.array_equal(out["bits"].cpu().numpy(), fr.x), code.name
        its.append(float(out["iters"].float().mean().item()))
        dc.close()
    assert abs(its[0] - its[1]) <= 0.25 * its[1] + 1.0, its


def test_peg_rejections(ctx):
    from paper_2001_07979_amd import mbp
    dv = np.full(64, 3, np.int32)
    with pytest.raises(RuntimeError, match="non-decreasing"):
        mbp.peg_build(ctx, 64, 32, dv[::-1].copy() - np.arange(64, dtype=np.int32) % 2, [1], 1)
    with pytest.raises(RuntimeError, match="degrees"):
        mbp.peg_build(ctx, 64, 2, dv, [1], 1)
