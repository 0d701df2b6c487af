"""spgm_step_noalloc: the SPGM step in the library's fixed scratch array, for callers that cannot
allocate device memory.  Two calls in a row on one plan (the second with a smaller minibatch) and
a third on another plan share the GPU's array; each must equal spgm_step on the same inputs bit
for bit (same kernels and launch shapes) and the oracle's step within the float32 projector's
tolerance (Sec. IV, Eq. 5 with the gradient of Eq. 6).  A minibatch whose workspace exceeds the
array is refused."""
import json
import os

import numpy as np
import pytest

from oracle import Oracle, rel_l2
from paper_2509_00774_amd import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_00774_amd import binding
    binding.load_library()
    return binding


def one_case(bd, plan, orc, rows, y, s0, eta, what):
    # threshold at the median magnitude of the oracle's gradient step, so that about half of the
    # voxels are set to zero by the prox
    v = s0.astype(np.complex128) - eta * orc.gradient(rows, y.astype(np.complex128), s0.astype(np.complex128))
    alpha = float(np.float32(np.median(np.abs(v))))
    rows_d = torch.from_numpy(rows).cuda()
    y_d = torch.from_numpy(y).cuda()
    a = torch.from_numpy(s0.copy()).cuda()
    b = torch.from_numpy(s0.copy()).cuda()
    plan.spgm_step_noalloc(rows_d, y_d, a, eta, alpha)
    plan.spgm_step(rows_d, y_d, b, eta, alpha)
    torch.cuda.synchronize()
    got, ref_gpu = a.cpu().numpy(), b.cpu().numpy()
    ref = orc.step(rows, y.astype(np.complex128), s0.astype(np.complex128), eta, alpha)
    err = rel_l2(got.astype(np.complex128), ref)
    print("[no-alloc] %s: B=%d, rel_l2 vs oracle %.3e, bitwise equal to spgm_step: %s" % (
        what, rows.size, err, np.array_equal(got, ref_gpu)), flush=True)
    assert np.array_equal(got, ref_gpu)
    assert err <= 1e-5
    assert 0.3 < np.mean(ref == 0) < 0.7  # the threshold is active


def test_noalloc_step_twice_then_other_plan(bd):
    steps = json.load(open(os.path.join(ROOT, "tests", "golden", "step_sizes.json")))
    geom1 = W.config_geometry("c1")
    orc1 = Oracle(geom1)
    plan1 = bd.Plan(geom1)
    eta = float(np.float32(steps["c1"]["eta"]))
    y1 = W.random_complex(orc1.M, seed=901).astype(np.complex64)
    s1 = (0.05 * W.random_complex(orc1.N, seed=902)).astype(np.complex64)
    one_case(bd, plan1, orc1, W.draw_rows(orc1.M, 4096, 1, seed=903)[0], y1, s1, eta, "c1 B=4096")
    one_case(bd, plan1, orc1, W.draw_rows(orc1.M, 1000, 1, seed=904)[0], y1, s1, eta, "c1 B=1000")
    plan1.close()
    geom0 = W.config_geometry("c0")
    orc0 = Oracle(geom0)
    plan0 = bd.Plan(geom0)
    eta = float(np.float32(steps["c0"]["eta"]))
    y0 = W.random_complex(orc0.M, seed=905).astype(np.complex64)
    s0 = (0.3 * W.random_complex(orc0.N, seed=906)).astype(np.complex64)
    one_case(bd, plan0, orc0, W.draw_rows(orc0.M, 256, 1, seed=907)[0], y0, s0, eta, "c0 B=256")
    plan0.close()


def test_noalloc_refuses_a_workspace_beyond_the_array(bd):
    geom = W.config_geometry("c2")
    plan = bd.Plan(geom)
    rows = torch.from_numpy(W.draw_rows(plan.M, 16384, 1, seed=908)[0]).cuda()
    y = torch.zeros(plan.M, dtype=torch.complex64, device="cuda")
    s = torch.zeros(plan.N, dtype=torch.complex64, device="cuda")
    with pytest.raises(bd.SpgmError) as exc:
        plan.spgm_step_noalloc(rows, y, s, 1e-3, 1e-4)
    assert exc.value.code == bd.SPGM_E_UNSUPPORTED
    assert "scratch" in str(exc.value)
    plan.close()
