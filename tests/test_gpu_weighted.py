"""Weighted MaxSAT (clause weights; hard clauses as large weights) on the
GPU path against the weighted FP64 oracle: costs exact, loss and gradient to
the same tolerance as the unweighted path, unit weights bitwise equal to the
unweighted path, every schedule bitwise equal to every other."""
import sys

import numpy as np
import pytest

import cnfgen
import oracle as O

from _helpers import assert_eval_parity, edge_case_cnf, w_abs_matrix

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


def _weights(m, seed, hi=100):
    return np.random.default_rng(seed).integers(1, hi, size=m).astype(np.int64)


def test_unit_weights_equal_unweighted_bitwise():
    n, m, R = 3000, 12900, 4
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=31)
    a = hm.load_cnf(n, lits)
    b = hm.load_cnf(n, lits, weights=np.ones(m, np.int64))
    assert b.info["weighted"] == 1 and b.info["total_weight"] == m and a.info["weighted"] == 0
    x = torch.from_numpy(cnfgen.random_x(n, R, seed=3, specials=True)).cuda()
    for mode in (hm.LOSS_UNSAT, hm.LOSS_ALL):
        la, ga, ua = hm.eval_relaxed(a, x, loss_mode=mode)
        lb, gb, ub = hm.eval_relaxed(b, x, loss_mode=mode)
        np.testing.assert_array_equal(la, lb)
        np.testing.assert_array_equal(ua, ub)
        np.testing.assert_array_equal(ga.cpu().numpy().view(np.uint32), gb.cpu().numpy().view(np.uint32))
    kw = dict(steps=60, restarts=R, eval_every=7, seed=5, lr=1e-2, want_x=True)
    for sched in (0, 255):  # the automatic (tiled) choice and the resident solver
        ra, rb = hm.solve(a, schedule=sched, **kw), hm.solve(b, schedule=sched, **kw)
        assert ra.schedule == rb.schedule and (ra.schedule == 255) == (sched == 255)
        np.testing.assert_array_equal(ra.restart_best, rb.restart_best)
        np.testing.assert_array_equal(ra.x_final.cpu().numpy().view(np.uint32),
                                      rb.x_final.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("mode", [hm.LOSS_UNSAT, hm.LOSS_ALL])
@pytest.mark.parametrize("kind", ["mixed", "edge", "skewed"])
def test_weighted_eval_parity(mode, kind):
    if kind == "mixed":
        n, R = 1000, 16
        lits = cnfgen.mixed_kcnf(n, 4200, seed=4)
    elif kind == "edge":
        (n, lits), R = edge_case_cnf(), 3
    else:
        n, R = 20000, 2
        lits = cnfgen.structured_cnf(n, 100000, seed=12)
    m = int(np.count_nonzero(np.asarray(lits) == 0))
    w = _weights(m, seed=7)
    x = cnfgen.random_x(n, R, seed=8, lo=-2, hi=2, specials=(kind == "edge"))
    cnf = hm.load_cnf(n, lits, weights=w)
    loss, g, u = hm.eval_relaxed(cnf, torch.from_numpy(x).cuda(), loss_mode=mode)
    oc = O.OracleCNF(n, lits, weights=w)
    assert_eval_parity(oc, w_abs_matrix(n, lits), x, loss, g.cpu().numpy(), u, mode, weights=w)
    assert cnf.info["total_weight"] == oc.total_weight


def test_weighted_schedules_bitwise():
    n, m, R = 1000, 4200, 16
    lits = cnfgen.mixed_kcnf(n, m, seed=4)
    cnf = hm.load_cnf(n, lits, weights=_weights(m, seed=9))
    xt = torch.from_numpy(cnfgen.random_x(n, R, seed=44, lo=-2, hi=2)).cuda()
    ref = None
    for sched in list(range(1, hm.schedule_count() + 1)) + [34 | (32 << 8) | (8 << 16), 255]:
        res = hm.solve(cnf, steps=5, restarts=R, eval_every=1, x0=xt, schedule=sched, want_x=True)
        cur = (res.restart_best.copy(), res.restart_step.copy(), res.x_final.cpu().numpy().view(np.uint32))
        if ref is None:
            ref = cur
        else:
            for a, b in zip(cur, ref):
                np.testing.assert_array_equal(a, b)


def test_weighted_steps_match_oracle():
    n, m, R = 400, 1720, 4
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=6)
    w = _weights(m, seed=6, hi=10)
    rng = np.random.default_rng(6)
    x0 = (rng.uniform(0.05, 1.0, (n, R)) * np.where(rng.random((n, R)) < 0.5, -1, 1)).astype(np.float32)
    oc = O.OracleCNF(n, lits, weights=w)
    cnf = hm.load_cnf(n, lits, weights=w)
    xt = torch.from_numpy(x0).cuda()
    for steps in (1, 2, 3):
        res = hm.solve(cnf, steps=steps, restarts=R, eval_every=1, x0=xt, lr=1e-4, want_x=True)
        ro = oc.solve(steps=steps, restarts=R, eval_every=1, x0=x0, lr=1e-4, want_x=True)
        d_g = res.x_final.cpu().numpy().astype(np.float64) - x0
        d_o = ro["x"] - x0
        assert np.all(np.abs(d_g - d_o) <= 1e-5 * np.abs(d_o) * steps + 2e-7 * np.abs(x0) + 1e-12), steps
        np.testing.assert_array_equal(res.restart_best, ro["restart_best"])


@pytest.mark.parametrize("seed", [0, 1])
def test_weighted_never_beats_bruteforce(seed):
    n, m = 16, 70
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=50 + seed)
    w = _weights(m, seed=seed, hi=50)
    oc = O.OracleCNF(n, lits, weights=w)
    opt, _, _ = oc.bruteforce()
    cnf = hm.load_cnf(n, lits, weights=w)
    res = hm.solve(cnf, steps=400, restarts=8, eval_every=1, seed=seed, lr=0.05)
    _say(f"weighted n={n}: GPU best {res.best_cost}, optimum {opt}, total {oc.total_weight}")
    assert opt <= res.best_cost <= oc.total_weight
    assert hm.evaluate(cnf, res.best_assignment) == res.best_cost == oc.count(res.best_assignment)


def test_wcnf_files(tmp_path):
    rng = np.random.default_rng(3)
    n = 30
    clauses = cnfgen.to_clauses(cnfgen.uniform_kcnf(n, 120, 3, seed=3))
    w = [int(v) for v in rng.integers(1, 20, size=len(clauses))]
    top = sum(w) + 1
    # classic: "p wcnf n m top", weight first on each clause line
    p1 = tmp_path / "a.wcnf"
    with open(p1, "w") as f:
        f.write(f"c weighted\np wcnf {n} {len(clauses)} {top}\n")
        for c, wj in zip(clauses, w):
            f.write(f"{wj} " + " ".join(map(str, c)) + " 0\n")
    a = hm.load_cnf_dimacs(str(p1))
    assert a.info["weighted"] == 1 and a.info["total_weight"] == sum(w)
    # header-less: hard clauses marked "h" weigh 1 + the total soft weight
    hard = clauses[:10]
    p2 = tmp_path / "b.wcnf"
    with open(p2, "w") as f:
        for c in hard:
            f.write("h " + " ".join(map(str, c)) + " 0\n")
        for c, wj in zip(clauses[10:], w[10:]):
            f.write(f"{wj} " + " ".join(map(str, c)) + " 0\n")
    b = hm.load_cnf_dimacs(str(p2))
    soft = sum(w[10:])
    assert b.info["total_weight"] == soft + 10 * (soft + 1)
    oa = O.OracleCNF(n, cnfgen.from_clauses(clauses), weights=w)
    ob = O.OracleCNF(n, cnfgen.from_clauses(clauses), weights=[soft + 1] * 10 + w[10:])
    for _ in range(10):
        x = rng.integers(0, 2, size=n).astype(np.uint8)
        assert hm.evaluate(a, x) == oa.count(x)
        assert hm.evaluate(b, x) == ob.count(x)
    # a clause line without its weight is rejected
    p3 = tmp_path / "c.wcnf"
    p3.write_text(f"p wcnf 3 1 10\n0\n")
    with pytest.raises(hm.HipMsatError):
        hm.load_cnf_dimacs(str(p3))
    with pytest.raises(hm.HipMsatError):
        hm.load_cnf(3, cnfgen.from_clauses([[1, 2], [-3]]), weights=[1, 0])


def _weighted_oracle_check(n, lits, w, out):
    """The oracle weighs the returned assignment at the reported cost, and
    (n <= 18) no restart reports less than the exact weighted optimum."""
    oc = O.OracleCNF(n, lits, weights=w)
    assert oc.count(out.best_assignment) == out.best_cost == int(np.min(out.restart_best))
    if n <= 18:
        assert np.all(out.restart_best >= oc.bruteforce()[0])


def test_weighted_batch_equals_solo():
    reqs = []
    for i, (n, m) in enumerate([(50, 215), (3000, 12900), (20000, 86000), (40, 170), (15000, 64000), (14, 60),
                                (18, 77)]):
        lits = cnfgen.uniform_kcnf(n, m, 3, seed=60 + i)
        reqs.append((n, lits, _weights(m, seed=i)))
    cnfs = [hm.load_cnf(n, lits, weights=w) for n, lits, w in reqs]
    kw = dict(steps=80, restarts=2, eval_every=5)
    batch = hm.solve_batch(cnfs, seeds=list(range(len(cnfs))), lr=1e-2, **kw)
    for i, (c, b) in enumerate(zip(cnfs, batch)):
        a = hm.solve(c, seed=i, lr=1e-2, autotune=False, **kw)
        np.testing.assert_array_equal(a.restart_best, b.restart_best)
        np.testing.assert_array_equal(a.best_assignment, b.best_assignment)
        assert hm.evaluate(c, b.best_assignment) == b.best_cost
        _weighted_oracle_check(reqs[i][0], reqs[i][1], reqs[i][2], b)


def test_weighted_served_equals_solo():
    from paper_2402_03640_amd.serve import Server
    reqs = []
    for i, (n, m) in enumerate([(50, 215), (3000, 12900), (8000, 34400), (60, 250), (16, 68)]):
        lits = cnfgen.uniform_kcnf(n, m, 3, seed=80 + i)
        reqs.append((n, lits, _weights(m, seed=80 + i)))
    kw = dict(steps=60, restarts=1, eval_every=6, lr=1e-2)
    solo = [hm.solve(hm.load_cnf(n, l, weights=w), seed=i, **kw) for i, (n, l, w) in enumerate(reqs)]
    with Server(workers=2) as srv:
        futs = [srv.submit(n, l, weights=w, seed=i, **kw) for i, (n, l, w) in enumerate(reqs)]
        res = [f.result(timeout=120) for f in futs]
    for a, r, (n, l, w) in zip(solo, res, reqs):
        np.testing.assert_array_equal(a.restart_best, r.output.restart_best)
        np.testing.assert_array_equal(a.best_assignment, r.output.best_assignment)
        _weighted_oracle_check(n, l, w, r.output)
