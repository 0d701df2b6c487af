"""The termination rule of Sec. V on the device (spgm_solve_tol) against the oracle.

The rule stops at the first iteration k with || |s^k| - |s^{k-1}| ||_2 < tol || |s^{k-1}| ||_2.
The stopping iteration is an integer decided by floating point: the GPU iterates carry float32
rounding, so the comparison is made only where the oracle's relative changes stay clear of tol
by a margin (0.2 %) up to its stopping iteration, which the test asserts first.  There the GPU
must stop at the same iteration, with the iterate within the float32 projector's tolerance
(rel-L2 <= 1e-5) of the oracle's, and its recorded changes within 0.2 % of the oracle's.  Group
size, graph replay and the roll-back to a stop inside a group must not change the result: the
iterate is bitwise that of spgm_solve with the same number of iterations.
"""
import json
import os

import numpy as np
import pytest

from oracle import Oracle, rel_l2
from paper_2509_00774_amd import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MARGIN = 2e-3


def say(*a):
    print("[gpu-tol]", *a, flush=True)


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_00774_amd import binding
    binding.load_library()
    return binding


@pytest.fixture(scope="module")
def c0():
    cfg = W.CONFIGS["c0"]
    geom = W.config_geometry("c0")
    orc = Oracle(geom)
    sj = json.load(open(os.path.join(ROOT, "tests", "golden", "step_sizes.json")))["c0"]
    eta = float(np.float32(sj["eta"]))
    alpha = float(np.float32(sj["lambda"] * eta))
    s_true, idx = W.config_scene("c0")
    y = W.add_noise(orc.forward_sparse(np.arange(orc.M), idx, s_true[idx]), cfg["snr_db"], seed=cfg["seed"] + 2)
    return geom, orc, y.astype(np.complex64), eta, alpha


def oracle_changes(orc, rows, y, eta, alpha, tol):
    """Oracle iterates until the rule holds; returns (stop k, iterates s^0..s^k, changes)."""
    s = np.zeros(orc.N, dtype=np.complex128)
    its, ch = [s], []
    for k in range(rows.shape[0]):
        sn = orc.step(rows[k], y, s, eta, alpha)
        o2 = np.sum(np.abs(s) ** 2)
        d2 = np.sum((np.abs(sn) - np.abs(s)) ** 2)
        ch.append(np.sqrt(d2 / o2) if o2 > 0 else np.inf)
        its.append(sn)
        s = sn
        if ch[-1] < tol:
            return k + 1, its, np.array(ch)
    return rows.shape[0], its, np.array(ch)


def run_case(bd, geom, orc, y, eta, alpha, rows, tol, what):
    y128 = y.astype(np.complex128)
    k_star, its, ch = oracle_changes(orc, rows, y128, eta, alpha, tol)
    assert k_star < rows.shape[0], "the rule must hold within the table"
    # the decision is clear of rounding: every change before the stop above tol, the stop below
    assert np.all(ch[:-1] > tol * (1 + MARGIN)) and ch[-1] < tol * (1 - MARGIN), (ch[-3:], tol)
    # the oracle's own termination routine agrees with the step-by-step reading of the rule
    s_o, k_o = orc.solve_tol(rows, y128, np.zeros(orc.N), eta, alpha, tol)
    assert k_o == k_star and rel_l2(s_o, its[k_star]) == 0.0
    plan = bd.Plan(geom)
    yd = torch.from_numpy(y).cuda()
    rows_d = torch.from_numpy(rows).cuda()
    results = {}
    for check_every, graph in ((7, True), (7, False), (50, True), (1, False)):
        s = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
        done, changes = plan.spgm_solve_tol(rows_d, yd, s, eta, alpha, tol, check_every=check_every,
                                            use_graph=graph)
        torch.cuda.synchronize()
        results[(check_every, graph)] = (done, s.cpu().numpy(), changes)
        say("%s: check_every %d graph %s -> stop %d (oracle %d)" % (what, check_every, graph, done, k_star))
    s_ref = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    plan.spgm_solve(rows_d[:k_star].contiguous(), yd, s_ref, eta, alpha)
    s_ref = s_ref.cpu().numpy()
    assert plan.spgm_plan_status() == 0
    plan.close()
    for key, (done, s, changes) in results.items():
        assert done == k_star, key
        assert np.array_equal(s, s_ref), key  # bitwise the solve of k_star iterations
        err = rel_l2(s.astype(np.complex128), its[k_star])
        assert err <= 1e-5, (key, err)
        assert changes.shape == (k_star,)
        assert np.isinf(changes[0])  # s^0 = 0
        assert np.allclose(changes[1:], ch[1:], rtol=MARGIN, atol=0), key
    say("%s: stop %d, iterate rel_l2 %.3e vs oracle" % (what, k_star, rel_l2(s_ref.astype(np.complex128), its[k_star])))


def test_spgm_stop_matches_oracle(bd, c0):
    """SPGM minibatches of the c0 workload: tol = 0.05 stops after about a dozen iterations."""
    geom, orc, y, eta, alpha = c0
    rows = W.draw_rows(orc.M, W.CONFIGS["c0"]["B"], 60, seed=77)
    run_case(bd, geom, orc, y, eta, alpha, rows, 0.05, "spgm c0")


def test_pgm_stop_matches_oracle(bd, c0):
    """Full-batch PGM (every row every iteration), a deterministic monotone approach: tol = 5e-3."""
    geom, orc, y, eta, alpha = c0
    rows = np.ascontiguousarray(np.broadcast_to(np.arange(orc.M, dtype=np.int32), (120, orc.M)))
    run_case(bd, geom, orc, y, eta, alpha, rows, 5e-3, "pgm c0")


def test_zero_tol_runs_every_iteration(bd, c0):
    geom, orc, y, eta, alpha = c0
    rows = torch.from_numpy(W.draw_rows(orc.M, 256, 23, seed=5)).cuda()
    yd = torch.from_numpy(y).cuda()
    plan = bd.Plan(geom)
    a = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    b = torch.zeros_like(a)
    done, changes = plan.spgm_solve_tol(rows, yd, a, eta, alpha, 0.0, check_every=10)
    plan.spgm_solve(rows, yd, b, eta, alpha)
    torch.cuda.synchronize()
    plan.close()
    assert done == 23 and changes.shape == (23,) and np.all(np.isfinite(changes[1:]))
    assert torch.equal(a, b)


def test_nonfinite_iterate_is_reported(bd, c0):
    """Measurements holding NaN make the first iterate non-finite: SPGM_E_NONFINITE at iteration 1."""
    geom, orc, y, eta, alpha = c0
    rows = torch.from_numpy(W.draw_rows(orc.M, 256, 5, seed=6)).cuda()
    yd = torch.full((orc.M,), float("nan"), dtype=torch.complex64, device="cuda")
    plan = bd.Plan(geom)
    s = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    with pytest.raises(bd.SpgmError) as exc:
        plan.spgm_solve_tol(rows, yd, s, eta, alpha, 1e-3, check_every=4)
    plan.close()
    assert exc.value.code == bd.SPGM_E_NONFINITE
    assert exc.value.iters_done == 1
