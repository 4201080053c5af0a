"""Host-side tests of the C ABI library: it loads, exports every declared
symbol, and builds instance plans whose two sparse layouts are exact
transposes of the canonical W (no GPU needed)."""
import os
import re

import numpy as np
import pytest

import cnfgen
import paper_2402_03640_amd as hm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIGN = np.uint32(0x80000000)
IDX = np.uint32(0x7FFFFFFF)


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "hipmsat.h")).read()
    declared = set(re.findall(r"\b(hms_[a-z_]+)\s*\(", header))
    assert declared, "no declarations found"
    L = hm.lib()
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} is declared but not exported"
    assert set(hm._lib.EXPORTS) == declared
    assert hm.version().startswith("hipmsat")


def test_probe_library_exports_every_declared_symbol():
    from paper_2402_03640_amd import probe
    header = open(os.path.join(ROOT, "include", "hipmsat_probe.h")).read()
    declared = set(re.findall(r"\b(hmsp_[a-z_]+)\s*\(", header))
    assert declared
    L = probe.lib()
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} is declared but not exported"
    assert set(probe.EXPORTS) == declared


def _canonical(clauses):
    """Canonical W entries per clause: (var0, sign) in first-appearance order."""
    out, taut = [], []
    for cl in clauses:
        pos, neg, order = set(), set(), []
        for l in cl:
            v = abs(l) - 1
            (pos if l > 0 else neg).add(v)
            if v not in order:
                order.append(v)
        ents = [(v, -1 if v in neg else 1) for v in order if not (v in pos and v in neg)]
        out.append(ents)
        taut.append(any(v in pos and v in neg for v in order))
    return out, taut


def _decode_tiles(tiles, ent):
    """Rows of a tiled layout: list of entry lists (padding kept) and nreal."""
    rows = []
    for base, ln, nreal, flags in tiles:
        for q in range(64):
            rows.append([int(ent[base + c * 64 + q]) for c in range(ln)])
    return rows


def _check_plan(n, lits):
    clauses = cnfgen.to_clauses(lits)
    P = hm.Plan(n, lits)
    canon, taut = _canonical(clauses)
    assert P.m == len(clauses)
    assert P.n_empty == sum(1 for c in clauses if len(c) == 0)
    assert P.n_taut == sum(taut)
    assert P.nnz == sum(len(e) for e in canon)
    var_old = P.var_old
    assert sorted(var_old.tolist()) == list(range(n))
    var_new = np.empty(n, np.int64)
    var_new[var_old] = np.arange(n)
    # ---- clause side: each kernel row is a canonical clause, padding inert
    rows = _decode_tiles(P.c_tile, P.c_ent)
    seen = set()
    for r, orig in enumerate(P.c_row_orig.tolist()):
        t, q = divmod(r, 64)
        base, ln, nreal, flags = P.c_tile[t]
        ents = rows[r]
        if orig < 0:
            assert q >= nreal
            assert all(e == n for e in ents)  # dummy variable, positive sign
            continue
        assert q < nreal and orig not in seen
        seen.add(orig)
        want = [(int(var_new[v]), s) for v, s in canon[orig]]
        got = [(e & 0x7FFFFFFF, -1 if e & 0x80000000 else 1) for e in ents if e != n]
        assert got == want
        assert all(e == n for e in ents[len(want):])
        assert bool(flags & 1) == taut[orig]
    assert seen == {j for j in range(len(clauses)) if canon[j]}
    # lengths sorted descending within each flag class
    # ---- variable side: exact transpose, clause rows ascending per variable
    krow_of = {orig: r for r, orig in enumerate(P.c_row_orig.tolist()) if orig >= 0}
    occ = [[] for _ in range(n)]
    for r, orig in sorted((r, o) for o, r in krow_of.items()):
        for e in rows[r]:
            if e == n:
                continue
            occ[e & 0x7FFFFFFF].append(r | (e & 0x80000000))
    deg = [len(o) for o in occ]
    assert deg == sorted(deg, reverse=True)
    assert P.n_act == sum(1 for d in deg if d > 0)
    assert P.n_heavy == sum(1 for d in deg if d > P.split_len)
    long = sum(1 for d in deg if d > P.seg_len)
    dense = long > 0 and 4 * long >= P.n_act and max(deg) <= 256
    assert P.split_len == (max(deg) if dense else P.seg_len)
    vrows = _decode_tiles(P.v_tile, P.v_ent)
    azero = P.c_tiles * 64
    seg_rows_pad = P.seg_tiles * 64
    for i in range(P.n_heavy):
        # segment s of ns holds entries s, s + ns, s + 2 ns, ... of the list
        segs = P.seg_row[P.seg_first[i]:P.seg_first[i + 1]].tolist()
        ns = len(segs)
        assert ns == -(-deg[i] // P.seg_len)
        for s, sr in enumerate(segs):
            assert sr < P.seg_rows
            got = [e for e in vrows[sr] if e != azero]
            assert got == occ[i][s::ns]
            assert all(e == azero for e in vrows[sr][len(got):])
    assert P.seg_row.tolist() == list(range(P.seg_rows))
    for i in range(P.n_heavy, P.n_act):
        r = seg_rows_pad + (i - P.n_heavy)
        got = [e for e in vrows[r] if e != azero]
        assert got == occ[i]
        assert all(e == azero for e in vrows[r][len(got):])
    _check_slots(P, n)
    return P


def _check_slots(P, n):
    """The clause-side -> variable-side occurrence map: every real clause
    entry names the variable-side entry of the same (variable, clause row,
    sign), each variable-side entry is named once, padding names none."""
    assert P.c_slot.size == P.c_ent.size
    # variable and row of every variable-side entry
    v_var = np.full(P.v_ent.size, -1, dtype=np.int64)
    v_real = np.zeros(P.v_ent.size, dtype=bool)
    for t, (base, ln, nreal, _) in enumerate(P.v_tile.tolist()):
        for q in range(nreal):
            row = t * 64 + q
            if row < P.seg_rows:
                var = int(np.searchsorted(P.seg_first, row, side="right")) - 1
            else:
                var = P.n_heavy + row - P.seg_tiles * 64
            pos = base + q + 64 * np.arange(ln)
            v_var[pos] = var
            v_real[pos] = P.v_ent[pos] != P.c_tiles * 64
    hits = np.zeros(P.v_ent.size, dtype=np.int64)
    for t, (base, ln, nreal, _) in enumerate(P.c_tile.tolist()):
        for q in range(64):
            for c in range(ln):
                p = base + 64 * c + q
                e, sl = int(P.c_ent[p]), int(P.c_slot[base + q * ln + c])  # the map is row by row
                if e == n:
                    assert sl == 0xFFFFFFFF
                    continue
                vp = sl & 0x7FFFFFFF
                assert sl & 0x80000000 == e & 0x80000000
                assert int(P.v_ent[vp]) == (t * 64 + q) | (e & 0x80000000)
                assert v_var[vp] == e & 0x7FFFFFFF
                hits[vp] += 1
    assert np.array_equal(hits, v_real.astype(np.int64))


def test_plan_small_edge_cases():
    clauses = [[1, -2, 3], [2, 2, -3], [], [1, -1, 4], [-4, 4], [5], [-5, 1, 1, 2], [3, -1]]
    P = _check_plan(6, cnfgen.from_clauses(clauses))
    assert P.n_empty == 1 and P.n_taut == 2
    assert P.n_act == 5  # variable 6 appears nowhere


def test_plan_random_mixed():
    _check_plan(200, cnfgen.mixed_kcnf(200, 900, seed=2))


def test_plan_skewed_heavy_rows():
    lits = cnfgen.structured_cnf(3000, 15000, seed=4)
    P = _check_plan(3000, lits)
    assert P.n_heavy > 0 and P.seg_rows > P.n_heavy and P.split_len == P.seg_len


def test_plan_dense_rows_kept_whole():
    """Dense uniform 5-CNF: every variable has about 85 entries, so no row is
    split; a denser one with rows above 256 entries splits them."""
    P = _check_plan(2000, cnfgen.uniform_kcnf(2000, 34000, 5, seed=7))
    assert P.n_heavy == 0 and P.seg_rows == 0 and P.split_len > P.seg_len
    P = _check_plan(300, cnfgen.uniform_kcnf(300, 20000, 5, seed=8))
    assert P.split_len == P.seg_len and P.n_heavy > 0


def _random_clauses(data, n, m, lo, hi):
    """Clauses of lo..hi literals over n variables, with repeats, complementary
    pairs and empty clauses all possible."""
    from hypothesis import strategies as st
    lit = st.integers(1, n).flatmap(lambda v: st.sampled_from([v, -v]))
    return data.draw(st.lists(st.lists(lit, min_size=lo, max_size=hi), min_size=m, max_size=m))


def test_plan_random_formulas_property():
    """Random formulas (any mix of lengths, repeats, tautologies and empty
    clauses; sparse and dense): both layouts are exact, the interleaved
    segments hold every entry once, and the split threshold follows the rule."""
    from hypothesis import HealthCheck, given, settings
    from hypothesis import strategies as st

    @settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
    @given(st.data())
    def run(data):
        n = data.draw(st.integers(1, 40))
        m = data.draw(st.integers(0, 120))
        if data.draw(st.booleans()):
            clauses = _random_clauses(data, n, m, 0, 14)
        else:  # few variables, many long clauses: long rows, heavy or dense
            clauses = _random_clauses(data, min(n, 6), max(m, 60), 3, 14)
            n = min(n, 6)
        _check_plan(n, cnfgen.from_clauses(clauses))

    run()


def _with_plan_threads(threads, fn):
    """fn() with HIPMSAT_PLAN_THREADS set to `threads` (the setting before is restored)."""
    old = os.environ.get("HIPMSAT_PLAN_THREADS")
    os.environ["HIPMSAT_PLAN_THREADS"] = str(threads)
    try:
        return fn()
    finally:
        if old is None:
            del os.environ["HIPMSAT_PLAN_THREADS"]
        else:
            os.environ["HIPMSAT_PLAN_THREADS"] = old


def _plan_arrays(n, lits, threads):
    P = _with_plan_threads(threads, lambda: hm.Plan(n, lits))
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in vars(P).items()}


@pytest.mark.parametrize("threads", [2, 3, 7, 16])
def test_plan_is_the_same_for_any_thread_count(threads):
    """The host plan build splits its phases over threads; the plan (every
    array and counter) is bitwise the one-thread plan, on formulas with
    tautologies, repeats, empty clauses, clauses past the 16-literal fast path,
    heavy segmented rows and dense unsplit rows, and with a tiny formula that
    leaves most threads an empty share."""
    rng = np.random.default_rng(threads)
    cases = [(1, cnfgen.from_clauses([[1], [-1, 1]])),
             (24, cnfgen.from_clauses([[1, -2, 3], [2, 2, -3], [], [1, -1, 4], [-4, 4], [5], [-5, 1, 1, 2],
                                       list(range(1, 21)) + [-7, 7, 3], [-20, 21, -22], []]))]
    clauses = []
    for _ in range(3000):
        k = int(rng.choice([0, 1, 2, 3, 5, 17, 30], p=[.02, .05, .2, .5, .15, .05, .03]))
        clauses.append([int(v) * (1 if rng.random() < 0.5 else -1) for v in rng.integers(1, 400, k)])
    cases.append((400, cnfgen.from_clauses(clauses)))
    cases.append((3000, cnfgen.structured_cnf(3000, 15000, seed=4)))
    cases.append((2000, cnfgen.uniform_kcnf(2000, 34000, 5, seed=7)))
    for n, lits in cases:
        a, b = _plan_arrays(n, lits, 1), _plan_arrays(n, lits, threads)
        assert a.keys() == b.keys()
        for k in a:
            if isinstance(a[k], np.ndarray):
                np.testing.assert_array_equal(a[k], b[k], err_msg=k)
            else:
                assert a[k] == b[k], k
    # parse errors name the same first bad literal
    bad = cnfgen.from_clauses([[1, 2]] * 500 + [[3, 99]] + [[1]] * 500 + [[-98]])
    msgs = []
    for th in (1, threads):
        with pytest.raises(hm.HipMsatError) as e:
            _with_plan_threads(th, lambda: hm.Plan(50, bad))
        msgs.append(str(e.value))
    assert msgs[0] == msgs[1] and "literal 99 at position 1501" in msgs[0]


def test_tune_candidates():
    """The autotuner's candidate list (host only): valid table entries and
    rows per unit, bitset variants only with the unsat-masked loss."""
    nsched = hm.schedule_count()
    assert nsched == 42
    for R, mode in ((1, hm.LOSS_UNSAT), (1, hm.LOSS_ALL), (3, hm.LOSS_UNSAT), (64, hm.LOSS_UNSAT)):
        codes = hm.tune_candidates(R, mode)
        assert codes and len(set(codes)) == len(codes)
        for c in codes:
            idx, U = c & 0xFF, c >> 8
            assert 1 <= idx <= nsched and U >= 1 and 64 % U == 0
        has_mask = any((c & 0xFF) in (23, 24, 25, 29, 30, 31, 32) for c in codes)
        assert has_mask == (mode == hm.LOSS_UNSAT)
        # the slot schedule: one restart and the unsat-masked loss only
        assert any((c & 0xFF) in (41, 42) for c in codes) == (R == 1 and mode == hm.LOSS_UNSAT)
    assert (26 | (32 << 8)) in hm.tune_candidates(64)
    with pytest.raises(hm.HipMsatError):
        hm.tune_candidates(0)


def test_plan_empty_instance():
    P = hm.Plan(0, np.zeros(0, np.int32))
    assert P.m == 0 and P.c_tiles == 0 and P.v_tiles == 0
    P = hm.Plan(3, np.array([0, 0], np.int32))
    assert P.m == 2 and P.n_empty == 2 and P.n_act == 0


def test_plan_errors():
    with pytest.raises(hm.HipMsatError) as e:
        hm.Plan(3, np.array([1, 2], np.int32))
    assert e.value.name == "HMS_ERR_PARSE"
    with pytest.raises(hm.HipMsatError) as e:
        hm.Plan(3, np.array([1, -4, 0], np.int32))
    assert e.value.name == "HMS_ERR_LITERAL_RANGE"
    with pytest.raises(hm.HipMsatError) as e:
        hm.Plan(-1, np.array([0], np.int32))
    assert e.value.name == "HMS_ERR_ARG"


def test_load_without_gpu_reports_device_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(hm.HipMsatError) as e:
        hm.load_cnf(3, np.array([1, 2, 0], np.int32), stream=0)
    assert e.value.name == "HMS_ERR_DEVICE"


def test_weights_count_checked_before_any_device_call():
    """A weight array whose length is not the clause count is refused by the
    binding (the C entry point reads one weight per clause)."""
    import paper_2402_03640_amd as hm
    with pytest.raises(ValueError, match="2 clause weights for 3 clauses"):
        hm.load_cnf(3, [1, 2, 0, -1, 3, 0, 2, 0], weights=[1, 2])
