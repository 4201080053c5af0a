"""Batching and serving: each instance's result is the same alone, in a
batched launch, and served in a mix with others (bitwise)."""
import sys
import time

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
    yield


def _requests(count, seed, n_hi=6000):
    reqs = cnfgen.serving_stream(count, seed=seed, rate=400.0, n_lo=50, n_hi=n_hi)
    return [(r.n, r.cnf(), dict(steps=120, restarts=1 + (r.index % 3), eval_every=10, seed=r.index,
                                lr=1e-2)) for r in reqs]


def _oracle_check(n, lits, out, weights=None):
    """The method's own checks of a batched or served result: the oracle
    counts the returned assignment at the reported cost, and no cost is below
    the exact optimum (brute force for n <= 18)."""
    oc = O.OracleCNF(n, lits, weights=weights)
    assert oc.count(out.best_assignment) == out.best_cost
    assert out.best_cost == int(np.min(out.restart_best))
    if n <= 18:
        opt, _, _ = oc.bruteforce()
        assert np.all(out.restart_best >= opt)
        return opt
    return None


def _tiny_requests(seed):
    """Requests small enough to brute-force (n <= 18)."""
    out = []
    for i, n in enumerate((8, 12, 15, 18)):
        out.append((n, cnfgen.uniform_kcnf(n, int(4.3 * n), 3, seed=seed * 100 + i),
                    dict(steps=120, restarts=1 + i % 3, eval_every=10, seed=900 + i, lr=1e-2)))
    return out


def _same(a, b):
    np.testing.assert_array_equal(a.restart_best, b.restart_best)
    np.testing.assert_array_equal(a.restart_step, b.restart_step)
    np.testing.assert_array_equal(a.best_assignment, b.best_assignment)
    # the FP64 loss total may differ in the last bits between schedules
    np.testing.assert_allclose(a.restart_loss, b.restart_loss, rtol=1e-12, atol=0)


def test_solve_batch_equals_solo():
    reqs = _requests(24, seed=1) + _tiny_requests(1)
    cnfs = [hm.load_cnf(n, lits) for n, lits, _ in reqs]
    solo = [hm.solve(c, **p) for c, (_, _, p) in zip(cnfs, reqs)]
    batch = hm.solve_batch(cnfs, steps=[p["steps"] for *_, p in reqs],
                           restarts=[p["restarts"] for *_, p in reqs],
                           eval_every=[p["eval_every"] for *_, p in reqs],
                           seeds=[p["seed"] for *_, p in reqs], lr=[p["lr"] for *_, p in reqs])
    kinds = {}
    for c, a, b, (n, lits, _) in zip(cnfs, solo, batch, reqs):
        assert b.status == 0
        _same(a, b)
        kinds[b.schedule == 255] = kinds.get(b.schedule == 255, 0) + 1
        assert hm.evaluate(c, b.best_assignment) == b.best_cost
        _oracle_check(n, lits, b)
    _say(f"batch: resident {kinds.get(True, 0)}, tiled {kinds.get(False, 0)}")
    assert kinds.get(True, 0) > 0 and kinds.get(False, 0) > 0


@pytest.mark.parametrize("opt,mode", [(hm.ADAM, hm.LOSS_UNSAT), (hm.SGD, hm.LOSS_ALL)])
def test_grouped_tiled_batch_equals_solo(opt, mode):
    """Instances too large for the resident solver, of uneven sizes (some with
    heavy rows), solved in grouped launches: each result is bitwise the solo
    result, with per-instance learning rates and seeds."""
    # the largest has more than 2^21 literals: its automatic schedule differs
    # from the others', and the group runs them all with the largest's
    sizes = [(20000, 86000, "u"), (9000, 40000, "s"), (15000, 64000, "u"), (30000, 120000, "s"),
             (12000, 50000, "u"), (200000, 860000, "u")]
    cnfs, lrs, all_lits = [], [], []
    for i, (n, m, kind) in enumerate(sizes):
        lits = (cnfgen.uniform_kcnf(n, m, 3, seed=40 + i) if kind == "u"
                else cnfgen.structured_cnf(n, m, seed=40 + i))
        all_lits.append(lits)
        cnfs.append(hm.load_cnf(n, lits))
        lrs.append((1e-2 if opt == hm.ADAM else 0.5) * (1 + 0.1 * i))
    assert any(c.info["n_heavy"] > 0 for c in cnfs)
    # one restart with the masked loss: the largest instance's automatic
    # schedule (bitset) differs from the others'
    kw = dict(steps=75, restarts=1 if mode == hm.LOSS_UNSAT else 2, eval_every=7, optimizer=opt, loss_mode=mode)
    batch = hm.solve_batch(cnfs, seeds=list(range(len(cnfs))), lr=lrs, want_x=True, **kw)
    for i, (c, b) in enumerate(zip(cnfs, batch)):
        assert b.status == 0 and b.schedule != 255
        _oracle_check(sizes[i][0], all_lits[i], b)
        a = hm.solve(c, seed=i, lr=lrs[i], want_x=True, autotune=False, **kw)
        _same(a, b)
        np.testing.assert_array_equal(a.x_final.cpu().numpy().view(np.uint32),
                                      b.x_final.cpu().numpy().view(np.uint32))
        assert b.steps_done == 75
    _say(f"grouped batch of {len(cnfs)}: device {batch[0].device_ms:.2f} ms, schedule {batch[0].schedule}")


@pytest.mark.parametrize("sched", [36, 37, 41, 42])
def test_grouped_batch_multi_tile_schedules(sched):
    """Grouped launches under the schedules that give each forward wavefront
    whole tiles (several tiles, or one with occurrence slots): each result is
    bitwise the solo result under the default schedule."""
    sizes = [(9000, 40000, "s"), (20000, 86000, "u"), (30000, 120000, "s"), (3000, 12000, "u")]
    cnfs = []
    for i, (n, m, kind) in enumerate(sizes):
        lits = (cnfgen.uniform_kcnf(n, m, 3, seed=60 + i) if kind == "u"
                else cnfgen.structured_cnf(n, m, seed=60 + i))
        cnfs.append(hm.load_cnf(n, lits))
    kw = dict(steps=40, restarts=1, eval_every=5, lr=1e-2)
    batch = hm.solve_batch(cnfs, seeds=list(range(len(cnfs))), schedule=sched, want_x=True, **kw)
    for i, (c, b) in enumerate(zip(cnfs, batch)):
        assert b.status == 0 and (b.schedule & 0xff) == sched
        a = hm.solve(c, seed=i, want_x=True, autotune=False, **kw)
        _same(a, b)
        np.testing.assert_array_equal(a.x_final.cpu().numpy().view(np.uint32),
                                      b.x_final.cpu().numpy().view(np.uint32))


def test_served_equals_solo_and_overlaps():
    """Requests of mixed kinds (default and other Adam constants, explicit
    start points, instances small enough to brute-force) served together:
    each equals its solo solve and passes the oracle's checks."""
    from paper_2402_03640_amd.serve import Server
    reqs = _requests(40, seed=2) + _tiny_requests(2)
    for i in range(0, 40, 5):  # other Adam constants: batched among themselves
        reqs[i][2].update(beta1=0.8, beta2=0.99, eps=1e-7)
    for i in range(3, 40, 9):  # a start point of its own: solved alone
        n, p = reqs[i][0], reqs[i][2]
        p["x0"] = torch.from_numpy(cnfgen.random_x(n, p["restarts"], seed=500 + i)).cuda()
    torch.cuda.synchronize()  # the workers read x0 from their own streams
    solo = []
    for n, lits, p in reqs:
        c = hm.load_cnf(n, lits)
        solo.append(hm.solve(c, **p))
        c.free()
    t0 = time.perf_counter()
    with Server(workers=4) as srv:
        futs = []
        for i, (n, lits, p) in enumerate(reqs):
            futs.append(srv.submit(n, lits, **p))
            time.sleep(0.001 * (i % 3))
        res = [f.result(timeout=120) for f in futs]
    wall = time.perf_counter() - t0
    for a, r, (n, lits, _) in zip(solo, res, reqs):
        _same(a, r.output)
        assert r.latency > 0 and r.done >= r.admitted >= r.arrival
        _oracle_check(n, lits, r.output)
    # requests were in flight together: latencies overlap in time
    spans = sorted((r.admitted, r.done) for r in res)
    overlap = sum(1 for (a0, a1), (b0, b1) in zip(spans, spans[1:]) if b0 < a1)
    _say(f"served {len(res)} in {wall:.3f} s, overlapping pairs {overlap}")
    assert overlap > 0


def test_admission_respects_budget():
    """Admission by footprint: with room for about two requests, the
    footprint in flight never exceeds the budget, requests wait for room (at
    least one deferral), and a request larger than the whole budget runs only
    on an idle device, with nothing beside it.  Results equal the solo ones."""
    from paper_2402_03640_amd.serve import Server, footprint_bytes
    reqs = _requests(16, seed=3, n_hi=3000)

    def foot(n, l, p):
        return footprint_bytes(n, int(np.count_nonzero(l == 0)), l.size - int(np.count_nonzero(l == 0)),
                               p["restarts"])

    budget = int(2.2 * max(foot(*r) for r in reqs))
    nb, lb = 60000, cnfgen.uniform_kcnf(60000, 258000, 3, seed=33)
    big = (nb, lb, dict(steps=60, restarts=2, eval_every=10, seed=77, lr=1e-2))
    assert foot(*big) > budget
    reqs = reqs[:8] + [big] + reqs[8:]
    solo = []
    for n, lits, p in reqs:
        c = hm.load_cnf(n, lits)
        solo.append(hm.solve(c, **p))
        c.free()
    with Server(workers=4, hbm_budget=budget, trace=True) as srv:
        futs = [srv.submit(n, lits, **p) for n, lits, p in reqs]
        res = [f.result(timeout=300) for f in futs]
    for a, r in zip(solo, res):
        _same(a, r.output)
    assert srv.in_use == 0 and srv.deferrals >= 1
    # replay the admissions and completions (both stamped under the server's lock)
    # (a completion sorts before an admission stamped at the same instant)
    ev = sorted([(a, 1, f, over) for a, d, f, over in srv.jobs] + [(d, 0, -f, over) for a, d, f, over in srv.jobs])
    in_use, running_over = 0, 0
    for t, kind, df, over in ev:
        if kind == 1 and over:
            assert in_use == 0, "an over-budget request was admitted beside others"
        if kind == 1 and not over:
            assert running_over == 0, "a request was admitted beside an over-budget one"
        in_use += df
        running_over += (1 if df > 0 else -1) if over else 0
        if not running_over:
            assert in_use <= budget, (in_use, budget)
    assert any(over for *_, over in srv.jobs)
    _say(f"admission: budget {budget / 2**20:.1f} MiB, peak {srv.peak_in_use / 2**20:.1f} MiB, "
         f"deferrals {srv.deferrals}, jobs {len(srv.jobs)}")


def test_short_groups_match_the_oracle():
    """Three Adam steps (lr 1e-4, counting every step) of a batched group and
    of a served mix: each instance's per-restart best costs and steps equal
    the oracle's from the same seeds, and the batched x_T is within the step
    tolerance of the oracle's x_T (FP32 rounding of three updates)."""
    from paper_2402_03640_amd.serve import Server
    T, lr = 3, 1e-4
    inst = []
    for i, n in enumerate((12, 90, 700, 3000, 9000, 24000)):
        inst.append((n, cnfgen.uniform_kcnf(n, int(4.3 * n), 3, seed=300 + i), 1 + i % 3, 40 + 7 * i))
    cnfs = [hm.load_cnf(n, lits) for n, lits, _, _ in inst]
    kw = dict(steps=T, eval_every=1, lr=lr)
    batch = hm.solve_batch(cnfs, restarts=[R for *_, R, _ in inst], seeds=[s for *_, s in inst], want_x=True, **kw)
    with Server(workers=3) as srv:
        futs = [srv.submit(n, lits, restarts=R, seed=s, **kw) for n, lits, R, s in inst]
        served = [f.result(timeout=120).output for f in futs]
    for (n, lits, R, s), b, v in zip(inst, batch, served):
        oc = O.OracleCNF(n, lits)
        o = oc.solve(steps=T, restarts=R, eval_every=1, seed=s, lr=lr, want_x=True)
        for out in (b, v):
            np.testing.assert_array_equal(out.restart_best, o["restart_best"])
            np.testing.assert_array_equal(out.restart_step, o["restart_step"])
            assert oc.count(out.best_assignment) == out.best_cost
        xg = b.x_final.cpu().numpy().astype(np.float64)
        tol = T * (2.0 ** -23 * (np.abs(o["x"]) + 4 * lr * T) + 1e-5 * 4 * lr)
        assert np.all(np.abs(xg - o["x"]) <= tol), np.max(np.abs(xg - o["x"]) / tol)
    _say(f"short groups: {len(inst)} instances, batched schedules {[b.schedule for b in batch]}")


def test_large_tiled_group_equals_solo():
    """Sixteen uneven tiled instances (3- to 5-CNF, 20k to 4M literals) in
    one grouped launch: each result is bitwise its solo result, the group
    running the schedule of its largest instance."""
    rng = np.random.default_rng(77)
    cnfs, seeds, inst = [], [], []
    for i in range(16):
        k = int(rng.integers(3, 6))
        n = int(rng.integers(2000, 40000))
        m = int(n * (3.5 + 1.5 * rng.random()) * 2 ** k / 8)
        inst.append((n, cnfgen.uniform_kcnf(n, m, k, seed=100 + i)))
        cnfs.append(hm.load_cnf(*inst[-1]))
        seeds.append(1000 + i)
    kw = dict(steps=80, restarts=1, eval_every=10, lr=1e-2)
    batch = hm.solve_batch(cnfs, seeds=seeds, want_x=True, **kw)
    tiled = 0
    for c, s, b, (n, lits) in zip(cnfs, seeds, batch, inst):
        a = hm.solve(c, seed=s, autotune=False, want_x=True, **kw)
        assert b.status == 0
        _same(a, b)
        _oracle_check(n, lits, b)
        np.testing.assert_array_equal(a.x_final.cpu().numpy().view(np.uint32),
                                      b.x_final.cpu().numpy().view(np.uint32))
        tiled += b.schedule != 255
    _say(f"large group: {tiled} of 16 tiled")
    assert tiled >= 9


def test_large_requests_run_alone():
    """Requests of more than 2^21 literals form jobs of their own, while the
    smaller requests of the same kind queued with them are still grouped; every
    result equals its solo solve."""
    from paper_2402_03640_amd.serve import GROUP_MAX_LITS, Server
    kw = dict(steps=20, restarts=1, eval_every=10, lr=1e-2)
    reqs = []
    for i in range(8):
        n = 250000 if i % 4 == 0 else 3000
        lits = cnfgen.uniform_kcnf(n, int(4.3 * n), 3, seed=300 + i)
        reqs.append((n, lits, dict(seed=i, **kw)))
    big = {i for i, (n, lits, p) in enumerate(reqs) if lits.size - np.count_nonzero(lits == 0) > GROUP_MAX_LITS}
    assert len(big) == 2
    solo = []
    for n, lits, p in reqs:
        c = hm.load_cnf(n, lits)
        solo.append(hm.solve(c, **p))
        c.free()
    with Server(workers=1, trace=True) as srv:
        futs = [srv.submit(n, lits, **p) for n, lits, p in reqs]
        res = [f.result(timeout=300) for f in futs]
    for a, r in zip(solo, res):
        _same(a, r.output)
    for rids in srv.job_rids:
        if any(r in big for r in rids):
            assert len(rids) == 1, srv.job_rids
    assert any(len(rids) > 1 for rids in srv.job_rids), srv.job_rids
    _say(f"jobs: {srv.job_rids}")


def test_queued_requests_are_taken_together():
    """With its one worker busy, requests of one kind that queue up are taken
    together when the worker frees (one job, shared launches), and each
    result still equals its solo solve."""
    from paper_2402_03640_amd import serve as S
    n0, lits0 = 3000, cnfgen.uniform_kcnf(3000, 12900, 3, seed=60)
    reqs = [(400 + 10 * i, cnfgen.uniform_kcnf(400 + 10 * i, 1700 + 43 * i, 3, seed=61 + i)) for i in range(12)]
    kw = dict(steps=150, restarts=1, eval_every=10, lr=1e-2, autotune=False)
    solo = []
    for i, (n, lits) in enumerate(reqs):
        c = hm.load_cnf(n, lits)
        solo.append(hm.solve(c, seed=i, **kw))
        c.free()
    sizes = []

    class Logged(S.Server):
        def _run(self, job, stream):
            sizes.append(len(job))
            return super()._run(job, stream)

    with Logged(workers=1) as srv:
        first = srv.submit(n0, lits0, seed=99, **dict(kw, steps=3000))  # keeps the worker busy
        futs = [srv.submit(n, lits, seed=i, **kw) for i, (n, lits) in enumerate(reqs)]
        res = [f.result(timeout=120) for f in futs]
        first.result(timeout=120)
    _say(f"job sizes {sizes}")
    for a, r in zip(solo, res):
        _same(a, r.output)
    assert sizes[0] == 1 and max(sizes[1:]) >= 6 and len(sizes) <= 4


def test_concurrent_batches_equal_solo():
    """Sixteen threads, each on its own stream, solve random groups of one to
    sixteen instances at once (resident and tiled): every result equals the
    instance's solo solve.  Concurrent kernels make a workgroup's wavefronts
    progress unevenly, which exposes a missing barrier inside a workgroup."""
    import threading

    import torch
    rng = np.random.default_rng(3)
    cnfs = []
    for i in range(80):
        n = int(np.exp(rng.uniform(np.log(30), np.log(6000))))
        k = int(rng.integers(3, 6))
        cnfs.append(hm.load_cnf(n, cnfgen.uniform_kcnf(n, max(int(n * rng.uniform(3.5, 5) * 2 ** k / 8), 1), k,
                                                       seed=5000 + i)))
    kw = dict(steps=200, restarts=1, eval_every=50, lr=1e-4)
    solo = [hm.solve(c, seed=i, autotune=False, **kw) for i, c in enumerate(cnfs)]
    bad, done, lock = [], [0], threading.Lock()

    def worker(w):
        try:
            torch.cuda.set_device(0)
            st = torch.cuda.Stream()
            r = np.random.default_rng(100 + w)
            for _ in range(20):
                idx = [int(x) for x in r.choice(len(cnfs), size=int(r.integers(1, 17)), replace=False)]
                if len(idx) == 1:
                    outs = [hm.solve(cnfs[idx[0]], seed=idx[0], stream=st, autotune=False, **kw)]
                else:
                    outs = hm.solve_batch([cnfs[i] for i in idx], seeds=idx, stream=st, **kw)
                with lock:
                    for i, o in zip(idx, outs):
                        done[0] += 1
                        if not (o.best_cost == solo[i].best_cost
                                and np.array_equal(o.best_assignment, solo[i].best_assignment)):
                            bad.append((w, i, len(idx), o.schedule))
        except Exception as e:  # reported on the test's thread
            with lock:
                bad.append((w, repr(e)))

    th = [threading.Thread(target=worker, args=(w,)) for w in range(16)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    _say(f"{done[0]} concurrent results")
    assert not bad, bad[:10]


def test_repeated_solves_do_not_grow_device_memory():
    """Loading, solving (alone and batched) and freeing the same instances
    twice over: device memory after the second pass equals that after the
    first (the stream-ordered pool keeps its high-water mark, nothing more)."""
    import torch
    rng = np.random.default_rng(1)
    inst = []
    for i in range(20):
        n = int(np.exp(rng.uniform(np.log(30), np.log(20000))))
        inst.append((n, cnfgen.uniform_kcnf(n, int(n * 4.2), 3, seed=i)))

    def one_pass():
        for _ in range(8):
            cnfs = [hm.load_cnf(n, lits) for n, lits in inst]
            for i, c in enumerate(cnfs):
                hm.solve(c, steps=30, restarts=1 + i % 4, eval_every=10, seed=i, autotune=False)
            hm.solve_batch(cnfs, steps=30, eval_every=10, seeds=list(range(len(cnfs))))
            for c in cnfs:
                c.free()
        torch.cuda.synchronize()
        return torch.cuda.mem_get_info()[0]

    f1 = one_pass()
    f2 = one_pass()
    _say(f"free after pass 1: {f1 / 2**20:.0f} MiB, after pass 2: {f2 / 2**20:.0f} MiB")
    assert f1 - f2 <= 16 << 20
