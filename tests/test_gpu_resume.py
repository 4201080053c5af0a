"""Resume: the state Algorithm 1 carries between iterations (relaxed values,
Adam moments, iteration count, best so far) handed back by one solve and
continued by another, through the C ABI, on the tiled and the resident
solver.  T1 steps then T2 more equal T1 + T2 steps bit for bit when T1 is a
multiple of the counting period; a resumed step agrees with the oracle's
step from the same state."""
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


def _bits(t):
    return t.cpu().numpy().view(np.uint32) if t.dtype == torch.float32 else t.cpu().numpy()


def _same_state(a, b):
    for k in ("x", "m", "v", "best_assignment"):
        ta, tb = getattr(a, k), getattr(b, k)
        assert (ta is None) == (tb is None), k
        if ta is not None:
            np.testing.assert_array_equal(_bits(ta), _bits(tb), err_msg=k)
    np.testing.assert_array_equal(a.best, b.best)
    np.testing.assert_array_equal(a.best_step, b.best_step)
    assert a.step == b.step


def _same_out(a, b):
    np.testing.assert_array_equal(a.restart_best, b.restart_best)
    np.testing.assert_array_equal(a.restart_step, b.restart_step)
    np.testing.assert_array_equal(a.best_assignment, b.best_assignment)
    assert a.best_cost == b.best_cost and a.best_restart == b.best_restart and a.best_step == b.best_step


# (name, n, m, R, K, schedule): the tiled kernels with graph replay, the
# bitset schedule at one restart, and the resident solver
CASES = [("tiled", 3000, 12900, 4, 25, 0), ("bitset", 20000, 86000, 1, 50, 37), ("resident", 50, 215, 4, 10, 255)]


@pytest.mark.parametrize("opt", [hm.ADAM, hm.SGD])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_resume_equals_uninterrupted(case, opt):
    name, n, m, R, K, sched = case
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, m, 3, seed=n))
    lr = 1e-2 if opt == hm.ADAM else 0.5
    kw = dict(restarts=R, eval_every=K, seed=7, optimizer=opt, lr=lr, schedule=sched, autotune=False)
    _say(f"resume {name} n={n} R={R} K={K} opt={opt}")
    full = hm.solve(cnf, steps=1000, want_state=True, want_x=True, **kw)
    one = hm.solve(cnf, steps=500, want_state=True, **kw)
    assert one.state.step == 500
    two = hm.solve(cnf, steps=500, resume=one.state, want_state=True, want_x=True, **kw)
    assert two.state.step == 1000 and two.steps_done == 500
    _same_out(full, two)
    _same_state(full.state, two.state)
    np.testing.assert_array_equal(_bits(full.x_final), _bits(two.x_final))
    np.testing.assert_array_equal(_bits(full.state.x), _bits(full.x_final))
    # three pieces, the middle one not a multiple of K: x, m, v still equal
    a = hm.solve(cnf, steps=137, want_state=True, **kw)
    b = hm.solve(cnf, steps=463, resume=a.state, want_state=True, **kw)
    c = hm.solve(cnf, steps=400, resume=b.state, want_state=True, **kw)
    for k in ("x", "m", "v"):
        if getattr(full.state, k) is not None:
            np.testing.assert_array_equal(_bits(getattr(full.state, k)), _bits(getattr(c.state, k)), err_msg=k)
    assert c.state.step == 1000
    assert np.all(c.state.best <= full.state.best)
    _say(f"  best {full.best_cost} at step {full.best_step} (schedule {full.schedule})")


@pytest.mark.parametrize("sched", [37, 42, 255], ids=["tiled-bitset", "tiled-slot", "resident"])
def test_weighted_resume_equals_uninterrupted(sched):
    """Weighted MaxSAT with hard clauses: the best so far is a total weight
    (int64, past 2^31) and enters a resumed solve as one; 200 + 200 steps
    equal 400 bit for bit, and the oracle weighs the returned assignment at
    the reported cost."""
    if sched in (37, 42):
        n, R, lits = 20000, 1, cnfgen.structured_cnf(20000, 100000, seed=9)
    else:
        n, R, lits = 60, 3, cnfgen.uniform_kcnf(60, 300, 3, seed=9)
    m = int(np.count_nonzero(lits == 0))
    rng = np.random.default_rng(9)
    w = rng.integers(1, 1000, size=m).astype(np.int64)
    w[rng.choice(m, size=max(m // 50, 1), replace=False)] = 10 ** 12  # hard clauses
    cnf = hm.load_cnf(n, lits, weights=w)
    kw = dict(restarts=R, eval_every=10, seed=2, lr=1e-2, schedule=sched, autotune=False)
    full = hm.solve(cnf, steps=400, want_state=True, **kw)
    a = hm.solve(cnf, steps=200, want_state=True, **kw)
    b = hm.solve(cnf, steps=200, resume=a.state, want_state=True, **kw)
    assert b.schedule == full.schedule == (sched if sched == 255 else b.schedule)
    _same_out(full, b)
    _same_state(full.state, b.state)
    assert O.OracleCNF(n, lits, weights=w).count(b.best_assignment) == b.best_cost
    _say(f"weighted resume {sched}: best {b.best_cost} at step {b.best_step}")


def test_resume_across_solvers():
    """500 steps on the tiled kernels, then 500 on the resident solver from
    the state they left (and the other way round): the same as 1000 on
    either, since both sum in the instance's order."""
    n, m, R = 400, 1720, 2
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, m, 3, seed=5))
    kw = dict(restarts=R, eval_every=20, seed=3, lr=1e-2, autotune=False)
    full = hm.solve(cnf, steps=1000, schedule=255, want_state=True, **kw)
    for s1, s2 in ((2, 255), (255, 2)):
        a = hm.solve(cnf, steps=500, schedule=s1, want_state=True, **kw)
        b = hm.solve(cnf, steps=500, schedule=s2, resume=a.state, want_state=True, **kw)
        assert a.schedule != b.schedule
        _same_out(full, b)
        _same_state(full.state, b.state)


def test_resumed_step_matches_the_oracle_step():
    """One Adam step from a state 300 steps in (nonzero moments, step count
    301): x, m and v against the oracle's step from the same FP32 state,
    within the step tolerance (1e-5 of each update's terms)."""
    n, m, R = 500, 2150, 3
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=9)
    cnf = hm.load_cnf(n, lits)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    kw = dict(restarts=R, eval_every=1, seed=11, lr=lr, schedule=2, autotune=False)
    a = hm.solve(cnf, steps=300, want_state=True, **kw)
    b = hm.solve(cnf, steps=1, resume=a.state, want_state=True, **kw)
    x0 = a.state.x.cpu().numpy().astype(np.float64)
    m0 = a.state.m.cpu().numpy().astype(np.float64)
    v0 = a.state.v.cpu().numpy().astype(np.float64)
    oc = O.OracleCNF(n, lits)
    st = dict(x=x0, m=m0, v=v0, step=300, best=a.state.best.copy(), best_step=a.state.best_step.copy(),
              best_assignment=a.state.best_assignment.cpu().numpy())
    o = oc.run(st, 1, eval_every=1, lr=lr, beta1=b1, beta2=b2, eps=eps)
    g = oc.loss_grad(a.state.x.cpu().numpy(), O.UNSAT)[1]
    bc1, bc2 = 1 - b1 ** 301, 1 - b2 ** 301
    mg, vg, xg = (t.cpu().numpy().astype(np.float64) for t in (b.state.m, b.state.v, b.state.x))
    m_scale = b1 * np.abs(m0) + (1 - b1) * np.abs(g)
    assert np.all(np.abs(mg - o["m"]) <= 1e-5 * m_scale + 1e-30)
    v_scale = b2 * v0 + (1 - b2) * g * g
    assert np.all(np.abs(vg - o["v"]) <= 1e-5 * v_scale + 1e-30)
    step_scale = (lr / bc1) * m_scale / (np.sqrt(o["v"] / bc2) + eps)
    ulp = np.abs(x0) * 2.0 ** -23
    assert np.all(np.abs(xg - o["x"]) <= 1e-5 * step_scale + ulp + 1e-30)
    np.testing.assert_array_equal(b.state.best, o["best"])
    np.testing.assert_array_equal(b.state.best_step, o["best_step"])
    _say(f"resumed step: max |dx - dx_oracle| {np.max(np.abs(xg - o['x'])):.2e}")


def test_resume_argument_errors():
    n = 60
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, 258, 3, seed=2))
    a = hm.solve(cnf, steps=10, restarts=2, want_state=True, autotune=False)
    with pytest.raises(hm.HipMsatError) as e:
        hm.solve(cnf, steps=10, restarts=2, resume=a.state, x0=a.state.x, autotune=False)
    assert e.value.name == "HMS_ERR_ARG"
    bad = hm.SolverState(a.state.x, None, None, a.state.best_assignment, a.state.best, a.state.best_step, 10)
    with pytest.raises(hm.HipMsatError) as e:  # Adam needs the moments
        hm.solve(cnf, steps=10, restarts=2, resume=bad, autotune=False)
    assert e.value.name == "HMS_ERR_ARG"
    big = hm.SolverState(a.state.x, a.state.m, a.state.v, a.state.best_assignment, a.state.best,
                         a.state.best_step, 2 ** 31 - 5)
    with pytest.raises(hm.HipMsatError) as e:
        hm.solve(cnf, steps=10, restarts=2, resume=big, autotune=False)
    assert e.value.name == "HMS_ERR_ARG"
    # SGD needs no moments, in or out
    s = hm.solve(cnf, steps=10, restarts=2, optimizer=hm.SGD, lr=0.1, want_state=True, autotune=False)
    assert s.state.m is None
    hm.solve(cnf, steps=10, restarts=2, optimizer=hm.SGD, lr=0.1, resume=s.state, autotune=False)


def test_cancel_returns_a_resumable_state():
    """A cancelled solve hands back the state after the steps it took; the
    rest of the steps from it give the uninterrupted result."""
    n, m = 3000, 12900
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, m, 3, seed=12))
    kw = dict(restarts=2, eval_every=10, seed=5, lr=1e-2, autotune=False, schedule=3)
    full = hm.solve(cnf, steps=400, want_state=True, **kw)
    flag = hm.CancelFlag()
    flag.set()
    with pytest.raises(hm.HipMsatError) as e:
        hm.solve(cnf, steps=400, cancel=flag, want_state=True, **kw)
    part = e.value.result
    # the flag is polled where a replayed graph body ends (a multiple of K)
    assert e.value.name == "HMS_ERR_CANCELLED" and part.state.step == part.steps_done
    assert 0 < part.steps_done < 400 and part.steps_done % 10 == 0
    rest = hm.solve(cnf, steps=400 - part.steps_done, resume=part.state, want_state=True, **kw)
    _same_out(full, rest)
    _same_state(full.state, rest.state)


def test_tuned_resident_choice_yields_to_a_time_limit_and_a_cancel_flag():
    """Once the tuner has picked the resident solver for an instance, a solve
    of that instance with a time limit or a cancel flag (which the resident
    solver cannot honour) takes a tiled schedule instead of failing."""
    n, m = 50, 215
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, m, 3, seed=1))
    code, _ = hm.tune(cnf, restarts=1, eval_every=1)
    assert code == hm.RESIDENT, code
    r0 = hm.solve(cnf, steps=100, eval_every=1, seed=2, lr=1e-2)
    assert r0.schedule == hm.RESIDENT
    r1 = hm.solve(cnf, steps=100, eval_every=1, seed=2, lr=1e-2, time_limit_s=1000.0)
    r2 = hm.solve(cnf, steps=100, eval_every=1, seed=2, lr=1e-2, cancel=hm.CancelFlag())
    for r in (r1, r2):
        assert r.schedule != hm.RESIDENT and r.steps_done == 100
        _same_out(r0, r)
