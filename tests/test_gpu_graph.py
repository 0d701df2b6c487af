"""hipGraph-captured solve: every replay equals the eager solve bit for bit, with the program's
own eager work and synchronisations between replays; new arguments re-capture; a workspace
that grows between replays invalidates the graph."""
import numpy as np
import pytest

from paper_2509_00774_amd import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_00774_amd import binding
    binding.load_library()
    return binding


def test_graph_replays_match_eager(bd):
    geom = W.config_geometry("c0")
    plan = bd.Plan(geom)
    rows = torch.from_numpy(W.config_rows("c0", K=20)).cuda()
    y = torch.from_numpy(W.random_complex(plan.M, seed=1).astype(np.complex64)).cuda()
    eta, alpha = 8e-3, 1e-3
    s_ref = torch.zeros(plan.N, dtype=torch.complex64, device="cuda")
    plan.spgm_solve(rows, y, s_ref, eta, alpha)
    torch.cuda.synchronize()
    ref = s_ref.cpu().numpy()
    s = torch.zeros(plan.N, dtype=torch.complex64, device="cuda")
    for rep in range(4):
        s.zero_()                      # eager work between replays
        plan.spgm_forward(rows[0].contiguous(), s_ref)
        plan.spgm_solve_graph(rows, y, s, eta, alpha)
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), ref), rep
    # other arguments re-capture
    s.zero_()
    plan.spgm_solve_graph(rows, y, s, eta, 2 * alpha)
    s2 = torch.zeros_like(s)
    plan.spgm_solve(rows, y, s2, eta, 2 * alpha)
    torch.cuda.synchronize()
    assert np.array_equal(s.cpu().numpy(), s2.cpu().numpy())
    # a larger minibatch elsewhere grows the workspace; the next replay must still be right
    big = torch.arange(plan.M, dtype=torch.int32, device="cuda")
    plan.spgm_forward(big, s_ref)
    s.zero_()
    plan.spgm_solve_graph(rows, y, s, eta, alpha)
    torch.cuda.synchronize()
    assert np.array_equal(s.cpu().numpy(), ref)
    assert plan.spgm_plan_status() == 0


@pytest.mark.parametrize("iters", [1, 2, 7])
def test_solve_equals_repeated_steps(bd, iters):
    """The solve defers each proximal step into the next forward (alternating iterate buffers);
    it must reproduce `iters` single steps bit for bit, eager and captured, from a nonzero start
    and with the autotuned row splits (several adjoint partial slices)."""
    geom = W.config_geometry("c0")
    plan = bd.Plan(geom)
    B = W.CONFIGS["c0"]["B"]
    plan.autotune(B)
    rows = torch.from_numpy(W.config_rows("c0", K=iters)).cuda()
    y = torch.from_numpy(W.random_complex(plan.M, seed=2).astype(np.complex64)).cuda()
    s0 = torch.from_numpy(W.random_complex(plan.N, seed=3).astype(np.complex64)).cuda()
    # the thresholds add up to 0.3 over the solve: a few percent of the unit-variance start end at 0
    eta, alpha = 8e-3, 0.3 / iters
    s_step = s0.clone()
    for k in range(iters):
        plan.spgm_step(rows[k].contiguous(), y, s_step, eta, alpha)
    s_solve = s0.clone()
    plan.spgm_solve(rows, y, s_solve, eta, alpha)
    s_graph = s0.clone()
    plan.spgm_solve_graph(rows, y, s_graph, eta, alpha)
    torch.cuda.synchronize()
    ref = s_step.cpu().numpy()
    assert np.count_nonzero(ref) not in (0, ref.size)  # the threshold is active
    assert np.array_equal(s_solve.cpu().numpy(), ref)
    assert np.array_equal(s_graph.cpu().numpy(), ref)
    assert plan.spgm_plan_status() == 0
