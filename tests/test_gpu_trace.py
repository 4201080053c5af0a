"""The trajectory of a solve: the (step, cost, loss) of every counted iterate,
kept on the device in a ring and read at the end, through the C ABI."""
import sys

import numpy as np
import pytest

import cnfgen
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hm = pytest.importorskip("paper_2402_03640_amd")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hm.lib()
    yield
    torch.cuda.synchronize()


def _counted(s0, T, K):
    """Iterations a solve of T steps from s0 counts: multiples of K, and the last."""
    return [t for t in range(s0, s0 + T) if t % K == 0] + [s0 + T]


@pytest.mark.parametrize("sched", [1, 255], ids=["tiled", "resident"])
def test_trace_records_every_count(sched):
    n, m, R, T, K = 200, 860, 3, 230, 20
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, m, 3, seed=3))
    out = hm.solve(cnf, steps=T, restarts=R, eval_every=K, seed=4, lr=1e-2, schedule=sched, autotune=False,
                   trace_cap=64)
    tr = out.trace
    steps = _counted(0, T, K)
    assert tr.shape == (len(steps), R)
    for r in range(R):
        assert tr["step"][:, r].tolist() == steps
        costs = tr["cost"][:, r]
        # the best is the first strictly lowest count below m
        lo = int(costs.min())
        assert out.restart_best[r] == min(lo, m)
        if lo < m:
            assert out.restart_step[r] == steps[int(np.argmin(costs))]
        # the last row is the count and loss at x_T
        assert tr["loss"][-1, r] == out.restart_loss[r]
    _say(f"trace ({'resident' if sched == 255 else 'tiled'}): costs of restart 0 {tr['cost'][:, 0].tolist()}")


@pytest.mark.parametrize("sched", [1, 255], ids=["tiled", "resident"])
def test_trace_of_a_weighted_solve(sched):
    """Weighted MaxSAT: each recorded cost is the total weight of the
    unsatisfied clauses (int64, hard clauses past 2^31), the best is the
    lowest one, and the oracle weighs the returned assignment at it."""
    n, m, R, T, K = 200, 860, 2, 120, 10
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=13)
    rng = np.random.default_rng(13)
    w = rng.integers(1, 500, size=m).astype(np.int64)
    w[rng.choice(m, size=20, replace=False)] = 3 * 10 ** 11
    cnf = hm.load_cnf(n, lits, weights=w)
    out = hm.solve(cnf, steps=T, restarts=R, eval_every=K, seed=6, lr=1e-2, schedule=sched, autotune=False,
                   trace_cap=64)
    tr = out.trace
    assert tr.shape == (len(_counted(0, T, K)), R)
    for r in range(R):
        costs = tr["cost"][:, r]
        assert out.restart_best[r] == min(int(costs.min()), int(w.sum()))
    assert O.OracleCNF(n, lits, weights=w).count(out.best_assignment) == out.best_cost
    _say(f"weighted trace ({'resident' if sched == 255 else 'tiled'}): restart 0 {tr['cost'][:, 0].tolist()[:6]}")


def test_trace_tiled_equals_resident():
    n, m, R, T, K = 60, 258, 2, 150, 7
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, m, 3, seed=5))
    kw = dict(steps=T, restarts=R, eval_every=K, seed=1, lr=5e-2, autotune=False, trace_cap=100)
    a = hm.solve(cnf, schedule=2, **kw)
    b = hm.solve(cnf, schedule=255, **kw)
    np.testing.assert_array_equal(a.trace["step"], b.trace["step"])
    np.testing.assert_array_equal(a.trace["cost"], b.trace["cost"])
    # the FP64 loss totals are summed in schedule-dependent order
    np.testing.assert_allclose(a.trace["loss"], b.trace["loss"], rtol=1e-12, atol=0)


@pytest.mark.parametrize("n,R,sched", [(500, 4, 3), (5000, 1, 42), (5000, 1, 41)],
                         ids=["tiled", "slot-one-tile", "slot-two-tiles"])
def test_trace_matches_the_oracle_for_short_solves(n, R, sched):
    """Six Adam steps at lr 1e-4, counted every other step: each count equals
    the oracle's count of its own iterate, each loss is within the parity
    tolerance (the FP32 and FP64 iterates agree to far below a rounding
    flip at this step size); also under the occurrence-slot schedules."""
    m, T, K = int(4.3 * n), 6, 2
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=8)
    cnf = hm.load_cnf(n, lits)
    out = hm.solve(cnf, steps=T, restarts=R, eval_every=K, seed=2, lr=1e-4, autotune=False, schedule=sched,
                   trace_cap=8)
    assert out.schedule & 0xFF == sched
    oc = O.OracleCNF(n, lits)
    st = oc.init_state(restarts=R, seed=2)
    prev = 0
    for row, t in enumerate(_counted(0, T, K)):
        if t > prev:
            st = oc.run(st, t - prev, eval_every=K, lr=1e-4)
            prev = t
        for r in range(R):
            a = (st["x"][:, r] > 0).astype(np.uint8)
            assert out.trace["cost"][row, r] == oc.count(a)
        lo = oc.loss_grad(st["x"], O.UNSAT)[0]
        np.testing.assert_allclose(out.trace["loss"][row], lo, rtol=1e-5)


@pytest.mark.parametrize("sched", [1, 255], ids=["tiled", "resident"])
def test_trace_ring_keeps_the_last_rows(sched):
    n, m, R, T, K = 120, 516, 2, 400, 10
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, m, 3, seed=6))
    kw = dict(steps=T, restarts=R, eval_every=K, seed=3, lr=1e-2, schedule=sched, autotune=False)
    full = hm.solve(cnf, trace_cap=1000, **kw).trace
    for cap in (1, 7, 41):
        part = hm.solve(cnf, trace_cap=cap, **kw).trace
        assert part.shape == (min(cap, full.shape[0]), R)
        np.testing.assert_array_equal(part, full[-cap:])


@pytest.mark.parametrize("sched", [1, 255], ids=["tiled", "resident"])
def test_trace_of_a_resumed_solve(sched):
    """Resumed off the counting period: its rows continue the numbering, and
    the two pieces' rows together are the uninterrupted solve's (the split
    iterate is counted once more, at the end of the first piece)."""
    n, m, R, K = 150, 645, 2, 25
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, m, 3, seed=7))
    kw = dict(restarts=R, eval_every=K, seed=5, lr=1e-2, schedule=sched, autotune=False, trace_cap=100)
    full = hm.solve(cnf, steps=300, **kw).trace
    a = hm.solve(cnf, steps=137, want_state=True, **kw)
    b = hm.solve(cnf, steps=163, resume=a.state, **kw)
    assert a.trace["step"][:, 0].tolist() == _counted(0, 137, K)
    assert b.trace["step"][:, 0].tolist() == _counted(137, 163, K)
    joined = np.concatenate([a.trace[:-1], b.trace])  # the split iterate's second count dropped
    np.testing.assert_array_equal(joined["step"], full["step"])
    np.testing.assert_array_equal(joined["cost"], full["cost"])
    np.testing.assert_allclose(joined["loss"], full["loss"], rtol=1e-12, atol=0)
