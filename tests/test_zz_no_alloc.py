"""The allocation-free evaluation (hms_eval_relaxed_noalloc), through the C ABI:
its loss, gradient and counts equal hms_eval_relaxed's bit for bit on calls in
a row over one fixed workspace (a large input, then a smaller one, then the
large one again), they pass the oracle's parity bar, the call allocates no
device memory, and an input too large for the workspace is refused."""
import sys

import numpy as np
import pytest

import cnfgen
import oracle as O

from _helpers import assert_eval_parity, w_abs_matrix

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


def _noalloc(cnf, xt, mode):
    R = xt.shape[1]
    loss = torch.full((R,), -1.0, dtype=torch.float64, device="cuda")
    grad = torch.full_like(xt, 7.0)
    unsat = torch.full((R,), -1, dtype=torch.int64, device="cuda")
    hm.eval_relaxed_noalloc(cnf, xt, loss, grad, unsat, loss_mode=mode)
    torch.cuda.synchronize()
    return loss.cpu().numpy(), grad.cpu().numpy(), unsat.cpu().numpy()


def _case(n, m, R, seed, kind):
    lits = (cnfgen.uniform_kcnf(n, m, 3, seed=seed) if kind == "u" else cnfgen.structured_cnf(n, m, seed=seed))
    x = cnfgen.random_x(n, R, seed=seed + 1, lo=-2, hi=2, specials=True)
    return n, lits, x


# a large input, a smaller one, the large one again: each call finds the
# previous call's contents in the workspace
CASES = [(20000, 86000, 8, 1, "u"), (1000, 4200, 16, 2, "u"), (20000, 86000, 8, 1, "u"), (9000, 40000, 1, 3, "s")]


@pytest.mark.parametrize("mode", [hm.LOSS_UNSAT, hm.LOSS_ALL])
def test_noalloc_equals_eval_relaxed_on_calls_in_a_row(mode):
    for n, m, R, seed, kind in CASES:
        n, lits, x = _case(n, m, R, seed, kind)
        _say(f"noalloc n={n} m={m} R={R} kind={kind} mode={mode}")
        cnf = hm.load_cnf(n, lits)
        xt = torch.from_numpy(x).cuda()
        lo, go, uo = _noalloc(cnf, xt, mode)
        lr, gr, ur = hm.eval_relaxed(cnf, xt, loss_mode=mode)
        gr = gr.cpu().numpy()
        np.testing.assert_array_equal(uo, ur)
        np.testing.assert_array_equal(lo.view(np.uint64), lr.view(np.uint64))
        np.testing.assert_array_equal(go.view(np.uint32), gr.view(np.uint32))
        if n <= 1000:
            assert_eval_parity(O.OracleCNF(n, lits), w_abs_matrix(n, lits), x, lo, go, uo, mode)
        cnf.free()


def test_noalloc_optional_outputs_and_no_device_allocation():
    n, lits, x = _case(3000, 12900, 4, 5, "u")
    cnf = hm.load_cnf(n, lits)
    xt = torch.from_numpy(x).cuda()
    lr, gr, ur = hm.eval_relaxed(cnf, xt)
    loss = torch.empty(4, dtype=torch.float64, device="cuda")
    unsat = torch.empty(4, dtype=torch.int64, device="cuda")
    grad = torch.empty_like(xt)
    hm.eval_relaxed_noalloc(cnf, xt, loss, None, None)  # loss only
    hm.eval_relaxed_noalloc(cnf, xt, None, None, unsat)  # count only
    torch.cuda.synchronize()
    np.testing.assert_array_equal(loss.cpu().numpy(), lr)
    np.testing.assert_array_equal(unsat.cpu().numpy(), ur)
    hm.eval_relaxed_noalloc(cnf, xt, loss, grad, unsat)  # warm: every kernel of the call has run
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(5):
        hm.eval_relaxed_noalloc(cnf, xt, loss, grad, unsat)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    np.testing.assert_array_equal(grad.cpu().numpy().view(np.uint32), gr.cpu().numpy().view(np.uint32))
    _say(f"noalloc: device free memory {free0 / 2**20:.1f} -> {free1 / 2**20:.1f} MiB over 5 calls")
    assert free1 == free0


def test_noalloc_refuses_an_input_past_its_workspace():
    n, m, R = 20000, 86000, 256
    cnf = hm.load_cnf(n, cnfgen.uniform_kcnf(n, m, 3, seed=1))
    xt = torch.zeros((n, R), dtype=torch.float32, device="cuda")
    loss = torch.empty(R, dtype=torch.float64, device="cuda")
    with pytest.raises(hm.HipMsatError) as e:
        hm.eval_relaxed_noalloc(cnf, xt, loss, None, None)
    assert e.value.name == "HMS_ERR_TOO_LARGE"
    # the allocating variant has no such limit
    lr, _, ur = hm.eval_relaxed(cnf, xt, want_grad=False)
    assert np.all(ur == ur[0])
