"""GPU parity of the other regularisers (the prox of Eq. 5 swapped for the elastic net or for the
total variation of the magnitudes; Sec. III notes the extension) against the FP64 oracle.

Tolerances.  The elastic-net and l1 proxes are a few float32 operations per voxel: elementwise
|gpu - oracle| <= 1e-6 max|v|.  The TV prox runs K dual iterations in float32; the map is
continuous (projections on the unit ball and on u >= 0, no branch decides a discrete result), so
rounding errors accumulate slowly: a float32 emulation of the same iteration on the grids below
stays within 2.7e-6 max|v| at K = 100 and alpha = 0.5.  The bound used is rel L2 <= 1e-5 and
elementwise <= 2e-5 max|v|.  A step or solve adds the float32 projector's own bound
(rel L2 <= 1e-5, elementwise <= 1e-4 max, as for spgm_step).
"""
import numpy as np
import pytest

from oracle import Oracle, prox_elastic, prox_l1, prox_tv_magnitude, rel_l2
from paper_2509_00774_amd import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

PROX_ELEM = 1e-6
TV_TOL, TV_ELEM = 1e-5, 2e-5
TOL, ELEM = 1e-5, 1e-4


def say(*a):
    print("[gpu-reg]", *a, flush=True)


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_00774_amd import binding
    binding.load_library()
    return binding


def cdev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex64))).cuda()


def idev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.int32))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def check(got, ref, what, tol, elem):
    err = rel_l2(got, ref)
    emax = np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)
    say("%s: rel_l2=%.3e elem_max=%.3e" % (what, err, emax))
    assert err <= tol, (what, err)
    assert emax <= elem, (what, emax)


def geom_for(grid, T=4, R=5, F=6, seed=0):
    return W.make_geometry(T, R, F, (20e9, 30e9), grid, 5e-3, 0.25, 0.2, seed=seed)


GRIDS = [(16, 16, 8), (7, 5, 3), (1, 1, 17), (33, 1, 2), (61, 61, 21)]


@pytest.mark.parametrize("grid", GRIDS)
def test_tv_prox_parity(bd, grid):
    plan = bd.Plan(geom_for(grid))
    v = W.blocky_field(grid, seed=sum(grid)).astype(np.complex64)
    vmax = np.max(np.abs(v))
    for alpha, K in [(0.02, 1), (0.1, 2), (0.1, 7), (0.5, 40), (0.5, 100)]:
        say("grid %s alpha %.2f K %d" % (grid, alpha, K))
        got = host(plan.spgm_prox(cdev(v), alpha, bd.REG_TV_MAGNITUDE, tv_iters=K))
        ref = prox_tv_magnitude(v.astype(np.complex128), grid, alpha, K)
        check(got, ref, "tv grid %s alpha %.2f K %d" % (grid, alpha, K), TV_TOL, TV_ELEM * vmax / np.max(np.abs(ref)))
    plan.close()


def test_tv_prox_identities(bd):
    grid = (9, 7, 4)
    plan = bd.Plan(geom_for(grid))
    v = W.blocky_field(grid, seed=5).astype(np.complex64)
    v[::7] = 0  # exact zeros stay zero
    for alpha, K in [(0.0, 20), (0.3, 0)]:
        t = cdev(v)
        plan.spgm_prox(t, alpha, bd.REG_TV_MAGNITUDE, tv_iters=K)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), v), (alpha, K)
    got = host(plan.spgm_prox(cdev(v), 0.3, bd.REG_TV_MAGNITUDE, tv_iters=30))
    assert np.all(got[::7] == 0)
    # a constant-magnitude image is a fixed point; the phase of every voxel is kept
    ph = np.exp(1j * np.random.default_rng(1).uniform(0, 2 * np.pi, v.size))
    c = (0.75 * ph).astype(np.complex64)
    got = host(plan.spgm_prox(cdev(c), 0.3, bd.REG_TV_MAGNITUDE, tv_iters=30))
    assert np.max(np.abs(got - c)) < 1e-6
    plan.close()


@pytest.mark.parametrize("kind", ["l1", "elastic"])
def test_pointwise_prox_parity(bd, kind):
    grid = (13, 11, 5)
    plan = bd.Plan(geom_for(grid))
    v = W.random_complex(int(np.prod(grid)), seed=7).astype(np.complex64)
    for alpha, mu in [(0.0, 0.0), (0.4, 0.0), (0.9, 2.5), (3.0, 0.1)]:
        if kind == "l1":
            got = host(plan.spgm_prox(cdev(v), alpha, bd.REG_L1))
            ref = prox_l1(v.astype(np.complex128), alpha)
        else:
            got = host(plan.spgm_prox(cdev(v), alpha, bd.REG_ELASTIC_NET, mu=mu))
            ref = prox_elastic(v.astype(np.complex128), alpha, mu)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(v))
        say("%s alpha %.2f mu %.2f: elem_max %.2e, zeros gpu %d oracle %d" % (
            kind, alpha, mu, err, np.sum(got == 0), np.sum(ref == 0)))
        assert err <= PROX_ELEM
    plan.close()


def c0_tv_problem():
    """c0 geometry with a blocky random-phase scene (the image class TV priors suit)."""
    cfg = W.CONFIGS["c0"]
    geom = W.config_geometry("c0")
    orc = Oracle(geom)
    s_true = W.blocky_field(cfg["grid"], n_boxes=4, noise=0.0, seed=31)
    y = W.add_noise(orc.forward(np.arange(orc.M), s_true), cfg["snr_db"], seed=32)
    y = y.astype(np.complex64).astype(np.complex128)
    L = max(orc.lipschitz(r, iters=60, seed=k) for k, r in enumerate(W.draw_rows(orc.M, cfg["B"], 4, seed=77)))
    eta = float(np.float32(1.0 / L))
    return geom, orc, y, s_true, eta


def test_c0_step_reg_parity(bd):
    geom, orc, y, s_true, eta = c0_tv_problem()
    plan = bd.Plan(geom)
    rows = W.config_rows("c0")[0]
    s0 = W.random_complex(orc.N, seed=9).astype(np.complex64)
    gscale = np.max(np.abs(s0))
    cases = [(0, 0.02, 0.0, 0), (1, 0.02, 3.0, 0), (2, 0.05 * gscale, 0.0, 1), (2, 0.05 * gscale, 0.0, 25)]
    for kind, alpha, mu, K in cases:
        s_gpu = cdev(s0)
        plan.spgm_step_reg(idev(rows), cdev(y), s_gpu, eta, alpha, kind, mu=mu, tv_iters=K)
        ref = orc.step_reg(rows, y, s0.astype(np.complex128), eta, alpha, kind, mu=mu, tv_iters=K)
        check(host(s_gpu), ref, "c0 step kind %d alpha %.3g mu %.1f K %d" % (kind, alpha, mu, K), TOL, ELEM)
    assert plan.status() == 0
    plan.close()


def test_step_reg_l1_and_elastic_mu0_equal_spgm_step(bd):
    """The l1 kind runs the same kernels as spgm_step; the elastic net at mu = 0 performs the same
    float operations (scale 1), so both agree with spgm_step bit for bit."""
    geom, orc, y, s_true, eta = c0_tv_problem()
    plan = bd.Plan(geom)
    rows = W.config_rows("c0")[1]
    s0 = cdev(W.random_complex(orc.N, seed=4))
    a = plan.spgm_step(idev(rows), cdev(y), s0.clone(), eta, 0.03)
    b = plan.spgm_step_reg(idev(rows), cdev(y), s0.clone(), eta, 0.03, bd.REG_L1)
    c = plan.spgm_step_reg(idev(rows), cdev(y), s0.clone(), eta, 0.03, bd.REG_ELASTIC_NET, mu=0.0)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)
    plan.close()


def test_c0_tv_solve_parity(bd):
    """20 TV-regularised SPGM iterations from zero (10 dual iterations per prox), GPU vs oracle."""
    geom, orc, y, s_true, eta = c0_tv_problem()
    plan = bd.Plan(geom)
    rows = W.config_rows("c0", K=20)
    alpha = 0.02 * float(np.max(np.abs(orc.adjoint(np.arange(orc.M), y)))) / orc.M * eta
    s_gpu = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    plan.spgm_solve_reg(idev(rows), cdev(y), s_gpu, eta, alpha, bd.REG_TV_MAGNITUDE, tv_iters=10)
    s_ref = np.zeros(orc.N, dtype=np.complex128)
    for k in range(rows.shape[0]):
        s_ref = orc.step_reg(rows[k], y, s_ref, eta, alpha, 2, tv_iters=10)
    got = host(s_gpu)
    check(got, s_ref, "c0 TV solve K=20", TOL, ELEM)
    say("c0 TV solve: NMSE vs truth %.3e" % (np.sum(np.abs(got - s_true) ** 2) / np.sum(np.abs(s_true) ** 2)))
    assert plan.status() == 0
    plan.close()


def test_regularizer_validation(bd):
    plan = bd.Plan(geom_for((4, 4, 2)))
    v = torch.zeros(plan.N, dtype=torch.complex64, device="cuda")
    with pytest.raises(bd.SpgmError) as e:
        plan.spgm_prox(v, 0.1, 7)
    assert e.value.code == bd.SPGM_E_INVALID
    with pytest.raises(bd.SpgmError) as e:
        plan.spgm_prox(v, 0.1, bd.REG_ELASTIC_NET, mu=-1.0)
    assert e.value.code == bd.SPGM_E_INVALID
    with pytest.raises(bd.SpgmError) as e:
        plan.spgm_prox(v, 0.1, bd.REG_TV_MAGNITUDE, tv_iters=-1)
    assert e.value.code == bd.SPGM_E_INVALID
    with pytest.raises(bd.SpgmError) as e:
        plan.spgm_prox(v, float("nan"), bd.REG_TV_MAGNITUDE, tv_iters=3)
    assert e.value.code == bd.SPGM_E_INVALID
    plan.close()
