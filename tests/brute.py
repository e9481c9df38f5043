"""Brute-force references that pin the oracle on tiny codes.

Each one enumerates every assignment of a handful of bits, so it shares
nothing with belief propagation beyond the model it is exact for:

* bitwise MAP LLRs: ln( sum_{x: Hx=z, x_i=0} w(x) / sum_{x: Hx=z, x_i=1} w(x) )
  with w(x) = prod_i exp(-lambda_i x_i), i.e. lambda_i = ln P(x_i=0)/P(x_i=1);
* max-marginals: max_{x_i=0} l(x) - max_{x_i=1} l(x) with l(x) = -lambda . x;
* the exact root marginal of the depth-t computation tree of the Tanner graph
  (every copy of check j keeps z_j, every copy of bit i keeps lambda_i).
BP is exact on trees, min-sum with no normalization is exact max-product on
trees, and t flooding iterations compute the depth-t computation-tree
marginal; these are the facts the pins rest on.
"""
from __future__ import annotations

import numpy as np


def _bits(N: int) -> np.ndarray:
    ids = np.arange(1 << N, dtype=np.int64)
    return ((ids[:, None] >> np.arange(N)[None, :]) & 1).astype(np.uint8)


def _logsumexp(a: np.ndarray) -> float:
    m = a.max()
    return float(m + np.log(np.exp(a - m).sum()))


def _feasible(H: np.ndarray, z: np.ndarray, X: np.ndarray) -> np.ndarray:
    par = (X.astype(np.int64) @ H.T.astype(np.int64)) & 1
    return np.all(par == z[None, :].astype(np.int64), axis=1)


def map_llr(H: np.ndarray, z: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Exact bitwise MAP LLRs of every bit (n <= ~20)."""
    n = H.shape[1]
    X = _bits(n)
    ok = _feasible(H, z, X)
    X = X[ok]
    lw = -(X.astype(np.float64) @ lam)
    out = np.empty(n)
    for i in range(n):
        out[i] = _logsumexp(lw[X[:, i] == 0]) - _logsumexp(lw[X[:, i] == 1])
    return out


def max_marginal(H: np.ndarray, z: np.ndarray, lam: np.ndarray) -> np.ndarray:
    n = H.shape[1]
    X = _bits(n)
    X = X[_feasible(H, z, X)]
    lw = -(X.astype(np.float64) @ lam)
    return np.array([lw[X[:, i] == 0].max() - lw[X[:, i] == 1].max() for i in range(n)])


def computation_tree(H: np.ndarray, root: int, t: int):
    """Variable copies (original ids) and check copies (orig id, member copies)."""
    checks_of = [np.nonzero(H[:, i])[0].tolist() for i in range(H.shape[1])]
    vars_of = [np.nonzero(H[j])[0].tolist() for j in range(H.shape[0])]
    var_orig = [root]
    chk = []
    frontier = [(0, None)]
    for _ in range(t):
        nxt = []
        for vc, parent in frontier:
            v = var_orig[vc]
            for j in checks_of[v]:
                if j == parent:
                    continue
                members = [vc]
                for w in vars_of[j]:
                    if w == v:
                        continue
                    var_orig.append(w)
                    wc = len(var_orig) - 1
                    members.append(wc)
                    nxt.append((wc, j))
                chk.append((j, members))
        frontier = nxt
    return var_orig, chk


def tree_root_llr(H: np.ndarray, z: np.ndarray, lam: np.ndarray, root: int, t: int,
                  max_copies: int = 22) -> float:
    var_orig, chk = computation_tree(H, root, t)
    N = len(var_orig)
    if N > max_copies:
        raise ValueError(f"computation tree has {N} variable copies")
    X = _bits(N)
    ok = np.ones(X.shape[0], dtype=bool)
    for j, members in chk:
        par = np.bitwise_xor.reduce(X[:, members], axis=1)
        ok &= par == z[j]
    X = X[ok]
    lw = -(X.astype(np.float64) @ lam[np.array(var_orig)])
    return _logsumexp(lw[X[:, 0] == 0]) - _logsumexp(lw[X[:, 0] == 1])


def random_tree_code(rng: np.random.Generator, n: int, u: int = 2, max_extra: int = 2):
    """Dense u matrices whose stacked Tanner graph is a tree on n bits.

    Each new check joins one existing bit to 1..max_extra new bits; checks
    are dealt to the u matrices at random (each matrix gets at least one).
    """
    rows = []
    have = 1
    while have < n:
        k = int(rng.integers(1, max_extra + 1))
        k = min(k, n - have)
        anchor = int(rng.integers(0, have))
        r = np.zeros(n, dtype=np.uint8)
        r[anchor] = 1
        r[have:have + k] = 1
        rows.append(r)
        have += k
    owner = rng.integers(0, u, size=len(rows))
    owner[:u] = np.arange(u)[: min(u, len(rows))]
    return [np.array([rows[j] for j in range(len(rows)) if owner[j] == l]) for l in range(u)]
