"""Shared test helpers: tolerance scaffolding built from the clause lists."""
import sys

import numpy as np
import scipy.sparse as sp

import cnfgen


def w_abs_matrix(n, lits):
    """|W| (n x m, CSR) of the canonical clauses (repeats once, pairs cancel)."""
    lits = np.asarray(lits, dtype=np.int64)
    ends = np.nonzero(lits == 0)[0]
    m = ends.size
    cid = np.repeat(np.arange(m), np.diff(np.concatenate([[-1], ends])) - 1)
    nz = lits[lits != 0]
    var = np.abs(nz) - 1
    sign = np.sign(nz)
    # coefficient per (var, clause) after dedup: +1 pos only, -1 neg only, 0 both
    key = cid * (n + 1) + var
    order = np.argsort(key, kind="stable")
    key_s, sign_s = key[order], sign[order]
    uk, start = np.unique(key_s, return_index=True)
    has_pos = np.maximum.reduceat((sign_s > 0).astype(np.int8), start) if uk.size else np.zeros(0)
    has_neg = np.maximum.reduceat((sign_s < 0).astype(np.int8), start) if uk.size else np.zeros(0)
    coef = has_pos.astype(np.int64) - has_neg.astype(np.int64)
    keep = coef != 0
    rows = (uk % (n + 1))[keep]
    cols = (uk // (n + 1))[keep]
    return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(n, m))


def sech2(x):
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(-2.0 * np.abs(x))
    return 4.0 * e / (1.0 + e) ** 2


def tolerance_terms(Wabs, x, mu, m, weights=None):
    """Per restart: loss bound scale (1/m) sum mu w F^2 and S_i for the
    gradient, F_j = sum |tanh| over clause j (w = 1 without weights)."""
    X = np.asarray(x, dtype=np.float64).reshape(Wabs.shape[0], -1)
    T = np.abs(np.tanh(X))
    F = Wabs.T @ T                       # [m][R]
    mu = np.asarray(mu, dtype=np.float64).reshape(F.shape)
    if weights is not None:
        mu = mu * np.asarray(weights, dtype=np.float64).reshape(-1, 1)
    lscale = (mu * F * F).sum(axis=0) / max(m, 1)
    S = sech2(X) * (2.0 / max(m, 1)) * (Wabs @ (mu * F))
    return lscale, S


def assert_eval_parity(oc, Wabs, x_np, loss, grad, unsat, mode, rtol=1e-5, weights=None):
    """GPU (loss, grad, unsat) at float32 x vs the FP64 oracle."""
    lo, go, uo, fo, muo = oc.loss_grad(x_np, mode, want_f=True)
    np.testing.assert_array_equal(np.asarray(unsat), uo)
    lscale, S = tolerance_terms(Wabs, x_np, muo, oc.m, weights)
    lerr = np.abs(np.asarray(loss) - lo)
    assert np.all(lerr <= rtol * lscale + 1e-300), (loss, lo, lscale)
    msg = f"parity n={oc.n} m={oc.m}: loss err / scale max {np.max(lerr / np.maximum(lscale, 1e-300)):.2e}"
    if grad is not None:
        g = np.asarray(grad, dtype=np.float64).reshape(go.shape)
        err = np.abs(g - go)
        msg += f", grad err / S max {np.max(np.where(S > 0, err / np.maximum(S, 1e-300), 0.0)):.2e}"
        bound = rtol * S + 1e-30
        bad = np.argwhere(err > bound)
        assert bad.size == 0, (bad[:5], g[tuple(bad[0])], go[tuple(bad[0])], S[tuple(bad[0])])
        assert np.all(g[S == 0] == 0.0)
        G2 = go.reshape(go.shape[0], -1)
        for r in range(G2.shape[1]):
            nrm = np.linalg.norm(G2[:, r])
            assert np.linalg.norm(g.reshape(G2.shape)[:, r] - G2[:, r]) <= rtol * nrm + 1e-30
    print(msg, file=sys.stderr, flush=True)
    return lo, go, uo


def edge_case_cnf():
    clauses = [[1, -2, 3], [2, 2, -3], [], [1, -1, 4], [-4, 4], [5], [-5, 1, 1, 2], [3, -1],
               [6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, -1],
               [-6, -7], [7, 7, 7], [-20, 21, -22]]
    return 24, cnfgen.from_clauses(clauses)
