"""Differentiation: the hand-written adjoint behind torch.autograd.Function,
against the FP64 oracle gradient and central finite differences, with and
without activation checkpointing (bitwise equal)."""
import sys

import numpy as np
import pytest

import cnfgen
import oracle as O

from _helpers import assert_eval_parity, tolerance_terms, w_abs_matrix

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hm = pytest.importorskip("paper_2402_03640_amd")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _grad(cnf, x, mode, checkpoint, scale=None):
    from paper_2402_03640_amd.autograd import maxsat_loss
    xt = x.clone().requires_grad_(True)
    loss, unsat = maxsat_loss(cnf, xt, loss_mode=mode, checkpoint=checkpoint)
    (loss * (scale if scale is not None else 1.0)).sum().backward()
    return loss.detach().cpu().numpy(), unsat.cpu().numpy(), xt.grad.detach().cpu().numpy()


@pytest.mark.parametrize("mode", [hm.LOSS_UNSAT, hm.LOSS_ALL])
def test_autograd_matches_oracle_cfg4(mode):
    """Mixed 2/3/4-CNF n=1000 m=4200 with 16 restarts."""
    n, m, R = 1000, 4200, 16
    lits = cnfgen.mixed_kcnf(n, m, seed=4)
    cnf = hm.load_cnf(n, lits)
    x_np = cnfgen.random_x(n, R, seed=41, lo=-2, hi=2)
    x = torch.from_numpy(x_np).cuda()
    loss, unsat, g = _grad(cnf, x, mode, checkpoint=False)
    oc = O.OracleCNF(n, lits)
    assert_eval_parity(oc, w_abs_matrix(n, lits), x_np, loss, g, unsat, mode)
    loss2, unsat2, g2 = _grad(cnf, x, mode, checkpoint=True)
    np.testing.assert_array_equal(g.view(np.uint32), g2.view(np.uint32))
    np.testing.assert_array_equal(loss, loss2)


def test_autograd_heavy_rows_and_scaling():
    n, m = 20000, 100000
    lits = cnfgen.structured_cnf(n, m, seed=12)
    cnf = hm.load_cnf(n, lits)
    assert cnf.info["n_heavy"] > 0
    x_np = cnfgen.random_x(n, 2, seed=5)
    x = torch.from_numpy(x_np).cuda()
    loss, unsat, g = _grad(cnf, x, hm.LOSS_UNSAT, checkpoint=False)
    oc = O.OracleCNF(n, lits)
    assert_eval_parity(oc, w_abs_matrix(n, lits), x_np, loss, g, unsat, hm.LOSS_UNSAT)
    _, _, g2 = _grad(cnf, x, hm.LOSS_UNSAT, checkpoint=True)
    np.testing.assert_array_equal(g.view(np.uint32), g2.view(np.uint32))
    # an incoming gradient of 2 doubles every entry exactly; per-restart scales apply per column
    _, _, g3 = _grad(cnf, x, hm.LOSS_UNSAT, checkpoint=False,
                     scale=torch.tensor([2.0, -0.5], dtype=torch.float64, device="cuda"))
    np.testing.assert_array_equal(g3[:, 0], 2.0 * g[:, 0])
    np.testing.assert_array_equal(g3[:, 1], -0.5 * g[:, 1])


def test_autograd_finite_differences():
    """Central differences (h = 1e-4) of the GPU loss itself, on coordinates far
    from 0 so the mask is locally constant: agreement to the FP32 noise floor."""
    n, m = 200, 860
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=3)
    cnf = hm.load_cnf(n, lits)
    rng = np.random.default_rng(0)
    x_np = (rng.uniform(0.2, 1.5, n) * np.where(rng.random(n) < 0.5, -1, 1)).astype(np.float32)
    x = torch.from_numpy(x_np).cuda()
    for mode in (hm.LOSS_UNSAT, hm.LOSS_ALL):
        loss, unsat, g = _grad(cnf, x, mode, checkpoint=True)
        g = g.reshape(-1)
        oc = O.OracleCNF(n, lits)
        _, _, _, _, mu = oc.loss_grad(x_np, mode, want_f=True)
        _, S = tolerance_terms(w_abs_matrix(n, lits), x_np, mu, m)
        S = S.reshape(-1)
        h = 1e-4
        idx = rng.choice(n, size=40, replace=False)
        X = np.repeat(x_np[:, None], 2 * idx.size, axis=1)
        for k, i in enumerate(idx):
            X[i, 2 * k] += h
            X[i, 2 * k + 1] -= h
        Xt = torch.from_numpy(np.ascontiguousarray(X)).cuda()
        lp, _, _ = hm.eval_relaxed(cnf, Xt, loss_mode=mode, want_grad=False)
        for k, i in enumerate(idx):
            dx = float(np.float32(X[i, 2 * k]) - np.float32(X[i, 2 * k + 1]))
            fd = (lp[2 * k] - lp[2 * k + 1]) / dx
            # FP32 scores: the loss difference carries ~1e-7 relative noise of L
            noise = 4e-7 * max(lp[2 * k], 1e-12) / dx
            assert abs(fd - g[i]) <= 1e-3 * S[i] + noise + 1e-12, (mode, i, fd, g[i], S[i])


def test_torch_driven_descent_reduces_unsat():
    """x as a torch parameter optimised by torch.optim.Adam through the custom
    function: the rounded cost goes down."""
    from paper_2402_03640_amd.autograd import maxsat_loss
    n, m = 2000, 8600
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=21)
    cnf = hm.load_cnf(n, lits)
    x = torch.nn.Parameter(torch.from_numpy(cnfgen.random_x(n, 1, seed=2)).cuda())
    opt = torch.optim.Adam([x], lr=1e-2)
    first = None
    for it in range(60):
        opt.zero_grad()
        loss, unsat = maxsat_loss(cnf, x)
        if first is None:
            first = int(unsat.item())
        loss.sum().backward()
        opt.step()
    last = int(maxsat_loss(cnf, x)[1].item())
    _say(f"torch-driven: unsat {first} -> {last}")
    assert last < 0.7 * first


def test_concurrent_evaluations_bitwise():
    """Sixteen threads on their own streams evaluate the loss, gradient and
    unsat counts (eval_relaxed, and the autograd loss with and without
    recomputation) of random instances at once: every result equals the one
    computed alone, bit for bit."""
    import threading

    from paper_2402_03640_amd.autograd import maxsat_loss
    rng = np.random.default_rng(5)
    cases = []
    for i in range(24):
        n = int(np.exp(rng.uniform(np.log(30), np.log(20000))))
        lits = (cnfgen.structured_cnf(n, int(n * rng.uniform(2, 5)), seed=900 + i) if i % 2
                else cnfgen.uniform_kcnf(n, int(n * 4.2), 3, seed=900 + i))
        c = hm.load_cnf(n, lits)
        x = torch.from_numpy(cnfgen.random_x(n, int(rng.choice([1, 4, 16, 64])), seed=i)).cuda()
        mode, ck = int(rng.choice([hm.LOSS_UNSAT, hm.LOSS_ALL])), bool(rng.random() < 0.5)
        l0, g0, u0 = hm.eval_relaxed(c, x, loss_mode=mode)
        cases.append((c, x, mode, ck, l0.copy(), g0.clone(), u0.copy(), _grad(c, x, mode, ck)[2]))
    torch.cuda.synchronize()
    bad, lock = [], threading.Lock()

    def worker(w):
        try:
            torch.cuda.set_device(0)
            st = torch.cuda.Stream()
            r = np.random.default_rng(w)
            with torch.cuda.stream(st):
                for _ in range(40):
                    c, x, mode, ck, l0, g0, u0, ag0 = cases[int(r.integers(0, len(cases)))]
                    l, g, u = hm.eval_relaxed(c, x, loss_mode=mode, stream=st)
                    xt = x.clone().requires_grad_(True)
                    loss, _ = maxsat_loss(c, xt, loss_mode=mode, checkpoint=ck)
                    loss.sum().backward()
                    st.synchronize()
                    ok = (np.array_equal(l, l0) and np.array_equal(u, u0)
                          and torch.equal(g.view(torch.int32), g0.view(torch.int32))
                          and np.array_equal(xt.grad.cpu().numpy().view(np.uint32), ag0.view(np.uint32)))
                    if not ok:
                        with lock:
                            bad.append((w, c.n))
        except Exception as e:  # reported on the test's thread
            with lock:
                bad.append((w, repr(e)))

    th = [threading.Thread(target=worker, args=(w,)) for w in range(16)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not bad, bad[:10]
