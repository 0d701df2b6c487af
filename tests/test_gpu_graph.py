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
