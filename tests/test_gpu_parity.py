"""GPU parity: the HIP solve loop against the FP64 oracle, through the C ABI.

Per evaluation (same FP32 x bits in): unsat counts bit-exact, loss within
1e-5 of (1/m) sum mu F^2 and each gradient entry within 1e-5 S_i (see
_helpers.tolerance_terms).  Trajectory-level checks are invariants: brute-force
optimum, evaluate(best) == best, determinism across schedules, restarts and
graph replay, and the SplitMix64 initial values.
"""
import sys

import numpy as np
import pytest

import cnfgen
import oracle as O

from _helpers import assert_eval_parity, edge_case_cnf, tolerance_terms, w_abs_matrix

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


def _x(n, R, seed, **kw):
    return cnfgen.random_x(n, R, seed, **kw)


def _eval_both(n, lits, x_np, mode, schedule_check=True):
    oc = O.OracleCNF(n, lits)
    W = w_abs_matrix(n, lits)
    cnf = hm.load_cnf(n, lits)
    xt = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    loss, g, u = hm.eval_relaxed(cnf, xt, loss_mode=mode)
    torch.cuda.synchronize()
    gn = g.cpu().numpy()
    assert_eval_parity(oc, W, x_np, loss, gn, u, mode)
    return cnf, loss, gn, u


@pytest.mark.parametrize("mode", [hm.LOSS_UNSAT, hm.LOSS_ALL])
@pytest.mark.parametrize("R", [1, 3, 16])
def test_eval_edge_cases(mode, R):
    n, lits = edge_case_cnf()
    _say(f"edge cases n={n} R={R} mode={mode}")
    x = _x(n, R, seed=R, lo=-3, hi=3, specials=True)
    _eval_both(n, lits, x, mode)


def _random_formula(rng, n, m):
    """Clauses of 0..20 literals (some past the 16 of the FP32 score path),
    with repeated literals and complementary pairs."""
    clauses = []
    for _ in range(m):
        k = int(rng.choice([0, 1, 2, 3, 3, 4, 5, 8, 17, 20], p=[.02, .05, .2, .3, .15, .1, .08, .05, .03, .02]))
        vs = rng.integers(1, n + 1, k)
        clauses.append([int(v) * (1 if rng.random() < 0.5 else -1) for v in vs])
    return cnfgen.from_clauses(clauses)


@pytest.mark.parametrize("seed", range(12))
def test_eval_random_formulas(seed):
    """Seeded random formulas of mixed shape, 1 to 5 restarts, both loss
    modes (special x values included): counts exact, loss and gradient within
    tolerance of the oracle."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 300))
    m = int(rng.integers(1, 6 * n))
    lits = _random_formula(rng, n, m)
    R = int(rng.integers(1, 6))
    for mode in (hm.LOSS_UNSAT, hm.LOSS_ALL):
        _eval_both(n, lits, _x(n, R, seed=2000 + seed, lo=-3, hi=3, specials=True), mode)


@pytest.mark.parametrize("mode", [hm.LOSS_UNSAT, hm.LOSS_ALL])
def test_eval_nan_inputs(mode):
    """NaN relaxed values round to false (a NaN is not > 0), so counts stay
    exact; a NaN reaches the loss of a restart and the gradient entries of the
    variables that share a loss clause with it, on both sides alike.  Finite
    entries keep the parity tolerance."""
    rng = np.random.default_rng(77 + mode)
    n, m, R = 120, 500, 6
    lits = _random_formula(rng, n, m)
    x = _x(n, R, seed=78, lo=-2, hi=2, specials=True, nan=9)
    x[:, 0] = np.where(np.isnan(x[:, 0]), np.float32(0.5), x[:, 0])  # restart 0 has no NaN
    oc = O.OracleCNF(n, lits)
    cnf = hm.load_cnf(n, lits)
    loss, g, u = hm.eval_relaxed(cnf, torch.from_numpy(x).cuda(), loss_mode=mode)
    torch.cuda.synchronize()
    gn = g.cpu().numpy().astype(np.float64)
    lo, go, uo = oc.loss_grad(x, mode)
    np.testing.assert_array_equal(u, uo)
    np.testing.assert_array_equal(np.isnan(loss), np.isnan(lo))
    np.testing.assert_array_equal(np.isnan(gn), np.isnan(go))
    assert not np.isnan(loss[0]) and np.isnan(loss).sum() >= 1
    fin = ~np.isnan(lo)
    W = w_abs_matrix(n, lits)
    _, _, _, _, muo = oc.loss_grad(x[:, fin], mode, want_f=True)
    lscale, S = tolerance_terms(W, x[:, fin], muo, oc.m)
    assert np.all(np.abs(loss[fin] - lo[fin]) <= 1e-5 * lscale + 1e-300)
    gf, gof = gn[:, fin], go[:, fin]
    assert np.all(np.abs(gf - gof) <= 1e-5 * S + 1e-30)
    _say(f"nan inputs: {int(np.isnan(loss).sum())} of {R} losses NaN, "
         f"{int(np.isnan(gn).sum())} gradient entries NaN, counts {u.tolist()}")


@pytest.mark.parametrize("mode", [hm.LOSS_UNSAT, hm.LOSS_ALL])
def test_eval_worked_example(mode, golden):
    g = golden("worked_example.txt")
    lits = np.array(g["clauses"], np.int32)
    x = np.array(g["x"], np.float32).reshape(2, 1)
    cnf, loss, gn, u = _eval_both(2, lits, x, mode)
    assert u[0] == g["unsat_count"]


def test_eval_cfg1_shape():
    n, m = 50, 215
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=1)
    for R in (1, 8):
        _say(f"cfg1 shape R={R}")
        _eval_both(n, lits, _x(n, R, seed=10 + R), hm.LOSS_UNSAT)


def test_eval_cfg4_all_schedules():
    """Mixed 2/3/4-CNF n=1000 m=4200 R=16: parity, and every schedule gives the
    bitwise same gradient and counts."""
    n, m, R = 1000, 4200, 16
    lits = cnfgen.mixed_kcnf(n, m, seed=4)
    x = _x(n, R, seed=44, lo=-2, hi=2)
    for mode in (hm.LOSS_UNSAT, hm.LOSS_ALL):
        cnf, loss0, g0, u0 = _eval_both(n, lits, x, mode)
    cnf = hm.load_cnf(n, lits)
    xt = torch.from_numpy(x).cuda()
    ref = None
    codes = list(range(1, hm.schedule_count() + 1)) + [34 | (32 << 8) | (8 << 16), 26 | (32 << 8) | (64 << 16),
                                  25 | (32 << 8) | (16 << 16), 14 | (16 << 8), 14 | (64 << 8), 11 | (1 << 8), 16 | (32 << 8),
                                  7 | (64 << 8), 1 | (64 << 8), 255]
    for sched in codes:
        res = hm.solve(cnf, steps=3, restarts=R, eval_every=1, x0=xt, schedule=sched, want_x=True)
        xf = res.x_final.cpu().numpy()
        cur = (res.restart_best.copy(), res.restart_step.copy(), xf)
        _say(f"cfg4 schedule {sched}: best {res.restart_best[:4]}")
        if ref is None:
            ref = cur
        else:
            np.testing.assert_array_equal(cur[0], ref[0])
            np.testing.assert_array_equal(cur[1], ref[1])
            np.testing.assert_array_equal(cur[2].view(np.uint32), ref[2].view(np.uint32))


def test_single_restart_schedules_bitwise():
    """R = 1 on a skewed instance (heavy rows): every schedule, with and
    without the unsat bitset, gives the same trajectory bit for bit."""
    n, m = 20000, 100000
    lits = cnfgen.structured_cnf(n, m, seed=12)
    cnf = hm.load_cnf(n, lits)
    assert cnf.info["n_heavy"] > 0
    ref = None
    for sched in [1, 2, 3, 4, 11, 23, 24, 25, 24 | (32 << 8), 25 | (64 << 8), 2 | (32 << 8), 36, 37, 38, 39, 40, 41, 42]:
        res = hm.solve(cnf, steps=60, restarts=1, eval_every=7, seed=5, lr=1e-2, schedule=sched,
                       want_x=True)
        cur = (res.restart_best.copy(), res.restart_step.copy(),
               res.x_final.cpu().numpy().view(np.uint32).copy(), res.best_assignment.copy())
        _say(f"R=1 schedule {sched}: best {res.best_cost} at {res.best_step}")
        if ref is None:
            ref = cur
        else:
            for a, b in zip(cur, ref):
                np.testing.assert_array_equal(a, b)


def _slot_instances(rng):
    """One-restart instances for the slot schedule: uniform, skewed (heavy
    rows in segments), mixed, dense 5-CNF (rows kept whole), and one with
    long clauses, repeats, tautologies and empty clauses."""
    out = [(3000, cnfgen.uniform_kcnf(3000, 12900, 3, seed=1)),
           (20000, cnfgen.structured_cnf(20000, 90000, seed=2)),
           (2000, cnfgen.mixed_kcnf(2000, 8400, seed=3)),
           (1200, cnfgen.uniform_kcnf(1200, 20400, 5, seed=4))]
    n = 500
    cl = cnfgen.to_clauses(cnfgen.uniform_kcnf(n, 2000, 3, seed=5))
    for _ in range(12):  # long clauses (FP64 scores past 16 columns)
        vs = rng.choice(n, size=int(rng.integers(17, 40)), replace=False) + 1
        cl.append([int(v) if rng.random() < 0.5 else -int(v) for v in vs])
    cl += [[], [7, -7, 9], [4, 4, -5], [-11, 12, 12, -11], [], [300, -300]]
    out.append((n, cnfgen.from_clauses(cl)))
    # three variables in 3000 clauses: every variable row is split into
    # segments and there are no light rows
    out.append((3, cnfgen.uniform_kcnf(3, 3000, 2, seed=6)))
    return out


def test_device_slot_map_equals_host_scan():
    """The occurrence map the library builds on the device at load equals
    the host scan of the plan view (checked against the layouts on the CPU),
    on instances with heavy rows in segments, dense rows kept whole, long
    clauses, repeats, tautologies and empty clauses."""
    rng = np.random.default_rng(5)
    for n, lits in _slot_instances(rng):
        cnf = hm.load_cnf(n, lits)
        dev = cnf.slot_map()
        plan = hm.Plan(n, lits)
        host = plan.c_slot
        assert dev.size == host.size > 0
        np.testing.assert_array_equal(dev, host)
        assert cnf.info["slot_bytes"] == 4 * plan.v_ent.size
        _say(f"slot map n={n}: {dev.size} entries, {int(np.count_nonzero(dev != 0xFFFFFFFF))} real")
        cnf.free()
    empty = hm.load_cnf(5, np.zeros(0, dtype=np.int32))
    assert empty.slot_map().size == 0 and empty.info["slot_bytes"] == 0


def test_slot_schedule_bitwise():
    """The slot schedule (the forward leaves each occurrence's adjoint in
    the slot of its variable-side entry, the backward reads them in entry
    order) gives the trajectory of its twin and of the bitset schedule bit
    for bit, while clauses enter and leave the loss every step (large steps,
    both optimizers, weights, hard clauses), in solo and grouped solves; with
    several restarts or the unmasked loss it falls back to its twin."""
    rng = np.random.default_rng(77)
    for idx, (n, lits) in enumerate(_slot_instances(rng)):
        m = int(np.count_nonzero(lits == 0))
        for weighted in (False, True):
            w = None
            if weighted:
                w = rng.integers(1, 30, size=m).astype(np.int64)
                w[rng.random(m) < 0.02] = 10 ** 6  # hard clauses
            cnf = hm.load_cnf(n, lits, weights=w)
            for opt, lr, K in ((hm.SGD, 0.3, 3), (hm.ADAM, 5e-2, 1)):
                kw = dict(steps=40, restarts=1, eval_every=K, optimizer=opt, lr=lr, seed=idx, want_x=True)
                runs = {s: hm.solve(cnf, schedule=s, **kw) for s in (40, 37, 41, 42)}
                ref = runs[40]
                for s, o in runs.items():
                    np.testing.assert_array_equal(o.restart_best, ref.restart_best, err_msg=str(s))
                    np.testing.assert_array_equal(o.restart_step, ref.restart_step)
                    np.testing.assert_array_equal(o.best_assignment, ref.best_assignment)
                    np.testing.assert_array_equal(o.x_final.cpu().numpy().view(np.uint32),
                                                  ref.x_final.cpu().numpy().view(np.uint32))
                _say(f"slot schedule, instance {idx} weighted={weighted} opt={opt}: best {ref.best_cost}")
            cnf.free()
    # grouped one-restart solves under the slot schedule equal their solo solves
    inst = _slot_instances(rng)[:3]
    cnfs = [hm.load_cnf(n, lits) for n, lits in inst]
    outs = hm.solve_batch(cnfs, steps=30, restarts=1, eval_every=5, seeds=[3, 4, 5], lr=5e-2, schedule=41,
                          want_x=True)
    for c, o, sd in zip(cnfs, outs, (3, 4, 5)):
        a = hm.solve(c, steps=30, restarts=1, eval_every=5, seed=sd, lr=5e-2, schedule=40, want_x=True)
        assert o.best_cost == a.best_cost and o.best_step == a.best_step
        np.testing.assert_array_equal(o.x_final.cpu().numpy().view(np.uint32),
                                      a.x_final.cpu().numpy().view(np.uint32))
    # several restarts and the unmasked loss: the twin runs
    c = cnfs[0]
    for kw in (dict(restarts=4), dict(restarts=1, loss_mode=hm.LOSS_ALL)):
        a = hm.solve(c, steps=20, eval_every=4, seed=9, lr=5e-2, schedule=41, want_x=True, **kw)
        b = hm.solve(c, steps=20, eval_every=4, seed=9, lr=5e-2, schedule=40, want_x=True, **kw)
        assert a.schedule == b.schedule
        np.testing.assert_array_equal(a.x_final.cpu().numpy().view(np.uint32),
                                      b.x_final.cpu().numpy().view(np.uint32))
    for c in cnfs:
        c.free()


def test_schedule_id_errors():
    n, lits = 200, cnfgen.uniform_kcnf(200, 860, 3, seed=1)
    cnf = hm.load_cnf(n, lits)
    for bad in (26 | (32 << 8) | (3 << 16), 26 | (3 << 8), 1 << 24, hm.schedule_count() + 1, 26 | (128 << 8),
                36 | (32 << 8)):
        with pytest.raises(hm.HipMsatError):
            hm.solve(cnf, steps=2, restarts=8, schedule=bad)
    code, ms = hm.tune(cnf, restarts=8, iters=3)
    res = hm.solve(cnf, steps=2, restarts=8)
    assert res.schedule == code and ms > 0


def test_restart_group_bitset_bitwise():
    """Several restarts on a skewed instance (heavy rows): the bitset
    schedules, one bit per clause and restart group, give the trajectory of
    the plain schedules bit for bit."""
    n, m, R = 20000, 100000, 8
    lits = cnfgen.structured_cnf(n, m, seed=12)
    cnf = hm.load_cnf(n, lits)
    assert cnf.info["n_heavy"] > 0
    ref = None
    for sched in [4, 26, 23 | (64 << 8), 24 | (32 << 8), 25 | (32 << 8), 25 | (64 << 8), 29 | (64 << 8),
                  30 | (64 << 8), 31 | (32 << 8), 32 | (64 << 8)]:
        res = hm.solve(cnf, steps=60, restarts=R, eval_every=7, seed=5, lr=1e-2, schedule=sched,
                       want_x=True)
        cur = (res.restart_best.copy(), res.restart_step.copy(),
               res.x_final.cpu().numpy().view(np.uint32).copy(), res.best_assignment.copy())
        _say(f"R={R} schedule {sched}: best {res.best_cost} at {res.best_step} (ran {res.schedule})")
        assert res.schedule & 0xFF == sched & 0xFF
        if ref is None:
            ref = cur
        else:
            for a, b in zip(cur, ref):
                np.testing.assert_array_equal(a, b)


RESIDENT = 255


@pytest.mark.parametrize("kind,R,opt,mode", [
    ("uniform", 1, hm.ADAM, hm.LOSS_UNSAT), ("uniform", 4, hm.SGD, hm.LOSS_ALL),
    ("mixed", 16, hm.ADAM, hm.LOSS_UNSAT), ("mixed", 8, hm.SGD, hm.LOSS_ALL), ("skewed", 1, hm.ADAM, hm.LOSS_UNSAT),
    ("skewed", 3, hm.SGD, hm.LOSS_UNSAT), ("edge", 2, hm.ADAM, hm.LOSS_ALL), ("dense", 2, hm.ADAM, hm.LOSS_UNSAT)])
def test_resident_matches_tiled(kind, R, opt, mode):
    """The resident solver (whole loop in one workgroup, state in LDS) is
    bitwise equal to the tiled kernels: per-restart bests, steps, final x and
    best assignment."""
    if kind == "uniform":
        n, lits = 50, cnfgen.uniform_kcnf(50, 215, 3, seed=1)
    elif kind == "mixed":
        n, lits = 1000, cnfgen.mixed_kcnf(1000, 4200, seed=4)
    elif kind == "skewed":
        n, lits = 3000, cnfgen.structured_cnf(3000, 15000, seed=4)
    elif kind == "dense":  # rows of about 85 entries, kept whole
        n, lits = 400, cnfgen.uniform_kcnf(400, 6800, 5, seed=6)
    else:
        n, lits = edge_case_cnf()
    cnf = hm.load_cnf(n, lits)
    lr = 0.05 if opt == hm.SGD else 1e-2
    kw = dict(steps=150, restarts=R, eval_every=5, seed=9, optimizer=opt, lr=lr, loss_mode=mode,
              want_x=True)
    a = hm.solve(cnf, schedule=RESIDENT, **kw)
    b = hm.solve(cnf, schedule={1: 1, 2: 2, 3: 3, 4: 3, 8: 4, 16: 4}[R], **kw)
    _say(f"resident {kind} R={R}: best {a.best_cost} vs tiled {b.best_cost} (sched {b.schedule})")
    assert a.schedule == RESIDENT and b.schedule != RESIDENT
    np.testing.assert_array_equal(a.restart_best, b.restart_best)
    np.testing.assert_array_equal(a.restart_step, b.restart_step)
    np.testing.assert_array_equal(a.x_final.cpu().numpy().view(np.uint32),
                                  b.x_final.cpu().numpy().view(np.uint32))
    np.testing.assert_array_equal(a.best_assignment, b.best_assignment)
    assert hm.evaluate(cnf, a.best_assignment) == a.best_cost
    np.testing.assert_allclose(a.restart_loss, b.restart_loss, rtol=1e-12)


def test_random_instances_schedule_independent():
    """Random instances (uniform k-CNF with k from 2 to 7, skewed, mixed, a
    third weighted) with random restart counts, counting periods, optimizers
    and loss modes: three random tuner schedules and the resident solver all
    give the automatic schedule's result bit for bit."""
    rng = np.random.default_rng(2026)
    checked = 0
    for it in range(120):
        kind = rng.choice(["uniform", "structured", "mixed"])
        n = int(rng.integers(30, 6000))
        if kind == "uniform":
            k = int(rng.integers(2, 8))
            lits = cnfgen.uniform_kcnf(n, max(int(n * rng.uniform(1.5, 0.6 * 2 ** k)), 1), k, seed=it)
        elif kind == "structured":
            lits = cnfgen.structured_cnf(n, int(n * rng.uniform(2, 6)), seed=it)
        else:
            lits = cnfgen.mixed_kcnf(n, int(n * rng.uniform(2, 5)), seed=it)
        m = int(np.count_nonzero(lits == 0))
        weights = rng.integers(1, 50, size=m).astype(np.int64) if rng.random() < 0.3 else None
        cnf = hm.load_cnf(n, lits, weights=weights)
        R = int(rng.choice([1, 2, 3, 5, 8, 16, 33, 64]))
        opt = int(rng.choice([hm.ADAM, hm.SGD]))
        mode = int(rng.choice([hm.LOSS_UNSAT, hm.LOSS_ALL]))
        kw = dict(steps=int(rng.integers(20, 120)), restarts=R, eval_every=int(rng.choice([1, 3, 10, 25])),
                  optimizer=opt, loss_mode=mode, lr=0.05 if opt == hm.SGD else 1e-2, seed=it, want_x=True,
                  autotune=False)
        ref = hm.solve(cnf, **kw)
        cands = hm.tune_candidates(R, mode)
        for s in list(rng.choice(cands, size=min(3, len(cands)), replace=False)) + [RESIDENT]:
            try:
                o = hm.solve(cnf, schedule=int(s), **kw)
            except hm.HipMsatError:
                continue  # the resident solver does not fit this instance
            np.testing.assert_array_equal(o.restart_best, ref.restart_best)
            np.testing.assert_array_equal(o.restart_step, ref.restart_step)
            np.testing.assert_array_equal(o.best_assignment, ref.best_assignment)
            np.testing.assert_array_equal(o.x_final.cpu().numpy().view(np.uint32),
                                          ref.x_final.cpu().numpy().view(np.uint32))
            checked += 1
        assert hm.evaluate(cnf, ref.best_assignment) == ref.best_cost
        cnf.free()
    _say(f"{checked} schedule pairs checked")


def test_binding_rejects_bad_points():
    """Relaxed points that the kernels cannot take are refused before any
    launch: wrong dtype, not contiguous, wrong row count, a gradient buffer of
    another shape, an initial point with the wrong restart count."""
    import torch
    n = 50
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, 215, 3, seed=1))
    good = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(TypeError):
        hm.eval_relaxed(cnf, good.double())
    with pytest.raises(ValueError, match="contiguous"):
        hm.eval_relaxed(cnf, torch.zeros((4, n), dtype=torch.float32, device="cuda").t())
    with pytest.raises(ValueError, match="shape"):
        hm.eval_relaxed(cnf, torch.zeros((n + 1, 4), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="grad_out"):
        hm.eval_relaxed(cnf, good, grad_out=torch.zeros((n, 3), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="restarts"):
        hm.solve(cnf, steps=2, restarts=3, x0=good)
    loss, g, unsat = hm.eval_relaxed(cnf, good)  # the good one still works
    assert g.shape == (n, 4) and unsat.shape == (4,)


def test_untimed_choice_of_resident():
    """Without timing, the resident solver takes instances of at most 2^15
    nonzeros (2^16 when every step is counted); larger ones run tiled."""
    small = hm.load_cnf(50, cnfgen.uniform_kcnf(50, 215, 3, seed=1))
    mid = hm.load_cnf(4000, cnfgen.uniform_kcnf(4000, 17200, 3, seed=2))  # 51600 nonzeros
    assert 1 << 15 < mid.info["nnz"] <= 1 << 16
    kw = dict(steps=20, restarts=1, seed=0, autotune=False)
    assert hm.solve(small, eval_every=5, **kw).schedule == RESIDENT
    assert hm.solve(mid, eval_every=5, **kw).schedule != RESIDENT
    assert hm.solve(mid, eval_every=1, **kw).schedule == RESIDENT
    # the batch path routes the same way
    out = hm.solve_batch([small, mid], steps=20, eval_every=5, seeds=[0, 1])
    assert out[0].schedule == RESIDENT and out[1].schedule != RESIDENT


def test_untimed_tiled_schedule_at_one_restart():
    """Without timing, one-restart tiled solves with the unsat-masked loss
    take: above 2^22 nonzeros the slot schedule with two clause tiles per
    forward wavefront (table entry 41), above 2^17 the one with one tile
    (entry 42); below, 16-column backward batches with four lanes per
    variable row (entry 39) up to 2^14 active variables, else two (entry
    38).  With the unmasked loss above 2^20 nonzeros: two tiles per forward
    wavefront, no slots (entry 36).  Every choice gives the same result bit
    for bit."""
    kw = dict(steps=12, restarts=1, eval_every=4, seed=0, autotune=False, want_x=True)
    for n, m, k, mode, want in ((400000, 1720000, 3, hm.LOSS_UNSAT, 41), (40000, 340000, 4, hm.LOSS_UNSAT, 42),
                                (20000, 86000, 3, hm.LOSS_UNSAT, 42), (8000, 34400, 3, hm.LOSS_UNSAT, 39),
                                (30000, 40000, 3, hm.LOSS_UNSAT, 38), (40000, 340000, 4, hm.LOSS_ALL, 36)):
        lits = cnfgen.uniform_kcnf(n, m, k, seed=n)
        cnf = hm.load_cnf(n, lits)
        a = hm.solve(cnf, loss_mode=mode, **kw)
        _say(f"n={n} m={m} k={k} nnz={cnf.info['nnz']} mode {mode}: untimed schedule {a.schedule}")
        assert a.schedule & 0xFF == want
        b = hm.solve(cnf, schedule=1, loss_mode=mode, **kw)
        np.testing.assert_array_equal(a.x_final.cpu().numpy().view(np.uint32), b.x_final.cpu().numpy().view(np.uint32))
        np.testing.assert_array_equal(a.restart_best, b.restart_best)
        cnf.free()


def test_resident_concurrent_threads():
    """Resident solves of different LDS sizes on several threads at once (the
    kernel's dynamic-LDS attribute is shared by all of them): every result
    equals the same solve alone, bit for bit."""
    import threading

    import torch
    inst = [(50, cnfgen.uniform_kcnf(50, 215, 3, seed=1)), (400, cnfgen.uniform_kcnf(400, 1700, 3, seed=2)),
            (1000, cnfgen.mixed_kcnf(1000, 4200, seed=4)), (120, cnfgen.uniform_kcnf(120, 510, 3, seed=3))]
    cnfs = [hm.load_cnf(n, lits) for n, lits in inst]
    kw = dict(steps=200, restarts=2, eval_every=5, seed=3, lr=1e-2, schedule=RESIDENT, want_x=True)
    solo = [hm.solve(c, **kw) for c in cnfs]
    _say("resident solves on 4 threads, 3 rounds each")
    errors = []

    def run(i):
        try:
            torch.cuda.set_device(0)
            st = torch.cuda.Stream()
            for _ in range(3):
                r = hm.solve(cnfs[i], stream=st, **kw)
                if not (np.array_equal(r.restart_best, solo[i].restart_best)
                        and np.array_equal(r.best_assignment, solo[i].best_assignment)
                        and np.array_equal(r.x_final.cpu().numpy().view(np.uint32),
                                           solo[i].x_final.cpu().numpy().view(np.uint32))):
                    errors.append(f"instance {i} differs from its solo solve")
        except Exception as e:  # reported below, on the test's thread
            errors.append(f"instance {i}: {e!r}")

    th = [threading.Thread(target=run, args=(i,)) for i in range(len(cnfs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors


def test_eval_cfg2_full_size():
    n, m, R = 20000, 86000, 64
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=2)
    x = _x(n, R, seed=22)
    _say("cfg2 full size R=64")
    _eval_both(n, lits, x, hm.LOSS_UNSAT)


def test_eval_structured_heavy_rows():
    n, m = 60000, 300000
    lits = cnfgen.structured_cnf(n, m, seed=3)
    cnf = hm.load_cnf(n, lits)
    assert cnf.info["n_heavy"] > 0
    for R in (1, 4):
        _say(f"structured n={n} m={m} R={R} heavy={cnf.info['n_heavy']}")
        _eval_both(n, lits, _x(n, R, seed=33 + R), hm.LOSS_UNSAT)
    _eval_both(n, lits, _x(n, 1, seed=35), hm.LOSS_ALL)


def test_eval_dense_rows_whole():
    """Uniform 5-CNF at ratio 17: every variable has about 85 entries and no
    row is split (one lane sums a whole row of up to 256 entries)."""
    n, m = 20000, 340000
    lits = cnfgen.uniform_kcnf(n, m, 5, seed=5)
    cnf = hm.load_cnf(n, lits)
    assert cnf.info["n_heavy"] == 0
    for R, mode in ((1, hm.LOSS_UNSAT), (4, hm.LOSS_UNSAT), (1, hm.LOSS_ALL)):
        _say(f"dense 5-CNF n={n} m={m} R={R}")
        _eval_both(n, lits, _x(n, R, seed=55 + R), mode)


def test_eval_very_long_clause():
    """One clause over 20000 distinct variables (one FP64 row of 20000
    columns; its tile pads the other 63 rows to that length) among short ones."""
    n = 30000
    rng = np.random.default_rng(41)
    long = (rng.permutation(n)[:20000] + 1) * np.where(rng.random(20000) < 0.5, -1, 1)
    lits = np.concatenate([cnfgen.uniform_kcnf(n, 60000, 3, seed=41), long.astype(np.int32), [0]]).astype(np.int32)
    for R, mode in ((1, hm.LOSS_ALL), (2, hm.LOSS_UNSAT)):
        _eval_both(n, lits, _x(n, R, seed=410 + R), mode)


def test_eval_cfg3_full_size():
    n, m = 500000, 2500000
    lits = cnfgen.structured_cnf(n, m, seed=3)
    _say("cfg3 full size")
    _eval_both(n, lits, _x(n, 1, seed=333), hm.LOSS_UNSAT)


def test_evaluate_counts_bit_exact():
    n, lits = edge_case_cnf()
    oc = O.OracleCNF(n, lits)
    cnf = hm.load_cnf(n, lits)
    rng = np.random.default_rng(0)
    for _ in range(20):
        a = (rng.random(n) < 0.5).astype(np.uint8)
        assert hm.evaluate(cnf, a) == oc.count(a)
    n, m = 3000, 12900
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=9)
    oc = O.OracleCNF(n, lits)
    cnf = hm.load_cnf(n, lits)
    for _ in range(5):
        a = (rng.random(n) < 0.5).astype(np.uint8)
        assert hm.evaluate(cnf, a) == oc.count(a)


def test_init_matches_splitmix_oracle():
    n, R, seed = 777, 5, 123456789
    lits = cnfgen.uniform_kcnf(n, 3000, 3, seed=5)
    cnf = hm.load_cnf(n, lits)
    res = hm.solve(cnf, steps=0, restarts=R, seed=seed, want_x=True)
    xg = res.x_final.cpu().numpy()
    xo = O.init_x(n, R, seed)
    np.testing.assert_array_equal(xg.view(np.uint32), xo.view(np.uint32))
    oc = O.OracleCNF(n, lits)
    for r in range(R):
        assert res.restart_best[r] == oc.count((xo[:, r] > 0).astype(np.uint8))


def test_step_parity_adam():
    """Steps from the same x0 (|x| >= 0.05, no rounding flips within 3 steps of
    lr 1e-4): x after each step within tolerance of the FP64 oracle."""
    n, m, R = 400, 1720, 4
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=6)
    rng = np.random.default_rng(6)
    x0 = (rng.uniform(0.05, 1.0, (n, R)) * np.where(rng.random((n, R)) < 0.5, -1, 1)).astype(np.float32)
    oc = O.OracleCNF(n, lits)
    cnf = hm.load_cnf(n, lits)
    xt = torch.from_numpy(x0).cuda()
    for steps in (1, 2, 3):
        res = hm.solve(cnf, steps=steps, restarts=R, eval_every=1, x0=xt, lr=1e-4, want_x=True)
        xg = res.x_final.cpu().numpy().astype(np.float64)
        ro = oc.solve(steps=steps, restarts=R, eval_every=1, x0=x0, lr=1e-4, want_x=True)
        d_g = xg - x0
        d_o = ro["x"] - x0
        assert np.all(np.abs(d_g - d_o) <= 1e-5 * np.abs(d_o) * steps + 2e-7 * np.abs(x0) + 1e-12), steps
        np.testing.assert_array_equal(res.restart_best, ro["restart_best"])


@pytest.mark.parametrize("kind", ["headline", "structured"])
def test_bench_schedule_full_size_step(kind):
    """At the benchmark sizes and in the schedules the benchmark times (64
    restarts: table entry 34 with 32/8 rows per unit; one restart on the
    structured instance: entry 41, occurrence slots), one Adam step from x0 with |x| >= 0.05:
    bitwise equal to another schedule's step, counts equal to the
    oracle's, and the step within tolerance of the oracle's wherever the
    gradient's sign is well determined (|g| > 1e-3 S_i)."""
    if kind == "headline":
        n, m, R, sched, other = 20000, 86000, 64, 34 | (32 << 8) | (8 << 16), 15
        lits = cnfgen.uniform_kcnf(n, m, 3, seed=21)
    else:
        n, m, R, sched, other = 500000, 2500000, 1, 41, 37
        lits = cnfgen.structured_cnf(n, m, seed=3)
    rng = np.random.default_rng(77)
    x0 = (rng.uniform(0.05, 1.0, (n, R)) * np.where(rng.random((n, R)) < 0.5, -1, 1)).astype(np.float32)
    cnf = hm.load_cnf(n, lits)
    xt = torch.from_numpy(x0).cuda()
    kw = dict(steps=1, restarts=R, eval_every=1, x0=xt, lr=1e-4, want_x=True)
    a = hm.solve(cnf, schedule=sched, **kw)
    b = hm.solve(cnf, schedule=other, **kw)
    _say(f"{kind}: schedule {a.schedule} vs {b.schedule}")
    assert (a.schedule & 0xff) == (sched & 0xff) and (b.schedule & 0xff) == other
    xa = a.x_final.cpu().numpy()
    np.testing.assert_array_equal(xa.view(np.uint32), b.x_final.cpu().numpy().view(np.uint32))
    np.testing.assert_array_equal(a.restart_best, b.restart_best)
    oc = O.OracleCNF(n, lits)
    ro = oc.solve(steps=1, restarts=R, eval_every=1, x0=x0, lr=1e-4, want_x=True)
    np.testing.assert_array_equal(a.restart_best, ro["restart_best"])
    _, go, _, _, muo = oc.loss_grad(x0, hm.LOSS_UNSAT, want_f=True)
    _, S = tolerance_terms(w_abs_matrix(n, lits), x0, muo, m)
    go = go.reshape(n, R)
    robust = np.abs(go) > 1e-3 * S
    d_g = xa.astype(np.float64) - x0
    d_o = ro["x"].reshape(n, R) - x0
    err = np.abs(d_g - d_o)[robust]
    bound = (1e-5 * np.abs(d_o) + 2e-7 * np.abs(x0) + 1e-12)[robust]
    _say(f"{kind}: {robust.sum()} of {robust.size} coordinates compared, max err / bound {np.max(err / bound):.2e}")
    assert robust.sum() >= 0.5 * np.count_nonzero(S)
    assert np.all(err <= bound)


def test_state_past_2_31_elements():
    """64-bit indexing: 4.2M variables x 512 restarts puts 2.15e9 elements in
    each state array, past 2^31.  Restarts of the batched solve equal
    single-restart solves with seed + r, bit for bit, at sampled r."""
    n, m, R = 4_200_000, 1_000_000, 512
    assert n * R > 2 ** 31
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=31)
    cnf = hm.load_cnf(n, lits)
    kw = dict(steps=2, eval_every=1, lr=1e-2, want_x=True, autotune=False)
    a = hm.solve(cnf, restarts=R, seed=7, **kw)
    _say(f"n={n} R={R}: schedule {a.schedule}, best {a.best_cost}")
    for r in (0, 1, 257, 511):
        b = hm.solve(cnf, restarts=1, seed=7 + r, **kw)
        assert a.restart_best[r] == b.restart_best[0]
        np.testing.assert_array_equal(a.x_final[:, r].cpu().numpy().view(np.uint32),
                                      b.x_final[:, 0].cpu().numpy().view(np.uint32))
    del a
    torch.cuda.empty_cache()


def test_sgd_worked_example_step(golden):
    g = golden("worked_example.txt")
    lits = np.array(g["clauses"], np.int32)
    cnf = hm.load_cnf(2, lits)
    x0 = torch.tensor(np.array(g["x"], np.float32).reshape(2, 1)).cuda()
    res = hm.solve(cnf, steps=1, restarts=1, optimizer=hm.SGD, lr=g["lr"], loss_mode=hm.LOSS_ALL,
                   x0=x0, want_x=True)
    x1 = res.x_final.cpu().numpy()[:, 0]
    np.testing.assert_allclose(x1, g["x_after_one_step"], atol=0.005)
    oc = O.OracleCNF(2, lits)
    ro = oc.solve(steps=1, restarts=1, optimizer=O.SGD, lr=g["lr"], mode=O.ALL,
                  x0=np.array(g["x"], np.float32), want_x=True)
    np.testing.assert_allclose(x1, ro["x"][:, 0], rtol=1e-6)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_solve_never_beats_bruteforce(seed):
    n = 18
    lits = cnfgen.uniform_kcnf(n, 90, 3, seed=seed)
    oc = O.OracleCNF(n, lits)
    opt, _, _ = oc.bruteforce()
    cnf = hm.load_cnf(n, lits)
    res = hm.solve(cnf, steps=400, restarts=8, eval_every=1, seed=seed, lr=0.05)
    _say(f"brute force seed {seed}: opt {opt} best {res.best_cost}")
    assert res.best_cost >= opt
    assert hm.evaluate(cnf, res.best_assignment) == res.best_cost
    assert oc.count(res.best_assignment) == res.best_cost
    assert res.best_cost == res.restart_best.min()
    assert res.best_restart == int(np.argmin(res.restart_best))


def test_plain_vs_batched_bitwise():
    """Restart r of a batched solve with seed s equals the plain solve with
    seed s + r, bitwise (state and best)."""
    n, m, R, s = 2000, 8600, 8, 40
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=7)
    cnf = hm.load_cnf(n, lits)
    big = hm.solve(cnf, steps=120, restarts=R, eval_every=10, seed=s, want_x=True, lr=1e-2)
    xb = big.x_final.cpu().numpy()
    for r in range(R):
        one = hm.solve(cnf, steps=120, restarts=1, eval_every=10, seed=s + r, want_x=True, lr=1e-2)
        assert one.restart_best[0] == big.restart_best[r]
        assert one.restart_step[0] == big.restart_step[r]
        np.testing.assert_array_equal(one.x_final.cpu().numpy()[:, 0].view(np.uint32),
                                      xb[:, r].view(np.uint32))


def test_graph_and_direct_launch_identical():
    n, m, R = 5000, 21500, 16
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=8)
    cnf = hm.load_cnf(n, lits)
    a = hm.solve(cnf, steps=150, restarts=R, eval_every=50, seed=3, use_graph=True, want_x=True)
    b = hm.solve(cnf, steps=150, restarts=R, eval_every=50, seed=3, use_graph=False, want_x=True)
    c = hm.solve(cnf, steps=150, restarts=R, eval_every=50, seed=3, use_graph=True, want_x=True)
    for o in (b, c):
        np.testing.assert_array_equal(a.restart_best, o.restart_best)
        np.testing.assert_array_equal(a.restart_step, o.restart_step)
        np.testing.assert_array_equal(a.x_final.cpu().numpy().view(np.uint32),
                                      o.x_final.cpu().numpy().view(np.uint32))


def test_solve_best_monotone_and_consistent():
    n, m = 3000, 12900
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=10)
    cnf = hm.load_cnf(n, lits)
    prev = m
    for T in (0, 50, 100, 200):
        res = hm.solve(cnf, steps=T, restarts=2, eval_every=10, seed=1, lr=1e-2)
        assert res.best_cost <= prev
        assert hm.evaluate(cnf, res.best_assignment) == res.best_cost
        prev = res.best_cost


def test_degenerate_instances():
    cnf = hm.load_cnf(0, np.zeros(0, np.int32))
    res = hm.solve(cnf, steps=5, restarts=2)
    assert res.best_cost == 0
    cnf = hm.load_cnf(3, np.array([0, 0, 0], np.int32))
    res = hm.solve(cnf, steps=5, restarts=1)
    assert res.best_cost == 3 and res.best_step == -1
    assert hm.evaluate(cnf, np.zeros(3, np.uint8)) == 3
    cnf = hm.load_cnf(2, np.array([1, -1, 0, 2, 0], np.int32))
    res = hm.solve(cnf, steps=20, restarts=1, lr=0.1)
    assert res.best_cost == 0
    lo, g, u = hm.eval_relaxed(cnf, torch.tensor([[0.3], [-0.2]], device="cuda"))
    assert u[0] == 1


def test_time_limit_stops_at_a_counting_boundary():
    """A wall-clock limit (the paper runs Algorithm 1 under time limits) stops
    the loop at a K-step boundary; the steps taken are exactly those of a
    fixed-step solve of the same length (bitwise), and the best is consistent."""
    n, m = 20000, 86000
    lits = cnfgen.uniform_kcnf(n, m, 3, seed=2)
    cnf = hm.load_cnf(n, lits)
    K = 25
    a = hm.solve(cnf, steps=10 ** 7, restarts=4, eval_every=K, seed=3, lr=1e-2, time_limit_s=0.05, want_x=True)
    _say(f"time limit: {a.steps_done} steps, best {a.best_cost}")
    assert 0 < a.steps_done < 10 ** 7 and a.steps_done % K == 0
    b = hm.solve(cnf, steps=a.steps_done, restarts=4, eval_every=K, seed=3, lr=1e-2, want_x=True)
    np.testing.assert_array_equal(a.restart_best, b.restart_best)
    np.testing.assert_array_equal(a.restart_step, b.restart_step)
    np.testing.assert_array_equal(a.x_final.cpu().numpy().view(np.uint32), b.x_final.cpu().numpy().view(np.uint32))
    assert hm.evaluate(cnf, a.best_assignment) == a.best_cost


def test_cancel_flag_returns_best_so_far():
    """Failure handling forced from the host: a cancel flag set by another
    thread stops the solve at a counting boundary with HMS_ERR_CANCELLED and
    the best so far, which is consistent and equals the fixed-step solve of
    that length."""
    import threading
    import time
    n, m = 20000, 86000
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, m, 3, seed=2))
    flag = hm.CancelFlag()
    threading.Thread(target=lambda: (time.sleep(0.05), flag.set()), daemon=True).start()
    with pytest.raises(hm.HipMsatError) as ei:
        hm.solve(cnf, steps=10 ** 7, restarts=2, eval_every=10, seed=1, lr=1e-2, cancel=flag, want_x=True)
    assert ei.value.name == "HMS_ERR_CANCELLED"
    a = ei.value.result
    assert 0 < a.steps_done < 10 ** 7 and a.steps_done % 10 == 0
    assert hm.evaluate(cnf, a.best_assignment) == a.best_cost
    b = hm.solve(cnf, steps=a.steps_done, restarts=2, eval_every=10, seed=1, lr=1e-2, want_x=True)
    np.testing.assert_array_equal(a.restart_best, b.restart_best)
    np.testing.assert_array_equal(a.x_final.cpu().numpy().view(np.uint32), b.x_final.cpu().numpy().view(np.uint32))
    # a flag set before the solve stops it at the first boundary
    flag2 = hm.CancelFlag()
    flag2.set()
    with pytest.raises(hm.HipMsatError) as ei:
        hm.solve(cnf, steps=1000, restarts=1, eval_every=10, cancel=flag2)
    assert ei.value.result.steps_done <= 32 * 2


def test_nonfinite_x0_reported():
    n, lits = 3, np.array([1, 2, 0, -3, 0], np.int32)
    cnf = hm.load_cnf(n, lits)
    x0 = torch.tensor([[float("nan")], [-0.5], [0.5]], device="cuda")
    with pytest.raises(hm.HipMsatError) as e:
        hm.solve(cnf, steps=3, restarts=1, x0=x0)
    assert e.value.name == "HMS_ERR_NONFINITE"
    assert e.value.result.best_cost >= 0


def test_dimacs_file(tmp_path):
    p = tmp_path / "f.cnf"
    p.write_text("c comment\np cnf 3 3\n1 -2 0\n2 3\n 0\n-1 -3 0\n")
    cnf = hm.load_cnf_dimacs(str(p))
    assert cnf.n == 3 and cnf.m == 3
    assert hm.evaluate(cnf, np.array([0, 0, 0], np.uint8)) == 1
