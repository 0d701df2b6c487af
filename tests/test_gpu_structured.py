"""GPU parity of the structured-minibatch path (frequency x transmitter x receiver subsets, the
separable factorisation of Eq. 2 with float32 GEMMs on the matrix cores) against the FP64 oracle
evaluated on the Cartesian-product rows, and against the pair kernels on the same rows.

Tolerance: the float32 projector's (relative L2 <= 1e-5 per output vector, elementwise
|gpu - oracle| <= 1e-4 max|oracle|); the factor phases are compensated per antenna exactly as
the pair phases are per antenna pair.
"""
import numpy as np
import pytest

from oracle import Oracle, rel_l2
from paper_2509_00774_amd import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-5
ELEM = 1e-4


def say(*a):
    print("[gpu-structured]", *a, flush=True)


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


def check(got, ref, what):
    err = rel_l2(got, ref)
    emax = np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)
    say("%s: rel_l2=%.3e elem_max=%.3e" % (what, err, emax))
    assert err <= TOL, (what, err)
    assert emax <= ELEM, (what, emax)


def subsets(geom, nf, nt, nr, seed):
    T, R, F = geom["tx"].shape[0], geom["rx"].shape[0], len(geom["freq"])
    fs, ts, rs = W.draw_structured_subsets(T, R, F, nf, nt, nr, 1, seed=seed)
    return fs[0], ts[0], rs[0], W.structured_rows(T, R, fs[0], ts[0], rs[0])


def structured_case(bd, geom, nf, nt, nr, seed, what):
    orc = Oracle(geom)
    plan = bd.Plan(geom)
    fs, ts, rs, rows = subsets(geom, nf, nt, nr, seed)
    s = W.random_complex(orc.N, seed=seed + 1).astype(np.complex64)
    r = W.random_complex(rows.size, seed=seed + 2).astype(np.complex64)
    y = host(plan.spgm_forward_structured(idev(fs), idev(ts), idev(rs), cdev(s)))
    g = host(plan.spgm_adjoint_structured(idev(fs), idev(ts), idev(rs), cdev(r)))
    check(y, orc.forward(rows, s.astype(np.complex128)), what + " forward")
    check(g, orc.adjoint(rows, r.astype(np.complex128)), what + " adjoint")
    # the pair kernels on the same rows give the same operator
    y_pair = host(plan.forward(idev(rows), cdev(s)))
    g_pair = host(plan.adjoint(idev(rows), cdev(r)))
    say("%s: structured vs pair kernels forward %.2e adjoint %.2e" % (what, rel_l2(y, y_pair), rel_l2(g, g_pair)))
    assert rel_l2(y, y_pair) <= TOL and rel_l2(g, g_pair) <= TOL
    assert plan.status() == 0
    plan.close()


@pytest.mark.parametrize("nf,nt,nr", [(4, 4, 3), (8, 8, 8), (16, 8, 8), (2, 7, 5)])
def test_c0_structured_projector(bd, nf, nt, nr):
    structured_case(bd, W.config_geometry("c0"), nf, nt, nr, 500 + nf * nt * nr, "c0 (%d,%d,%d)" % (nf, nt, nr))


@pytest.mark.parametrize("T,R,F,grid,nf,nt,nr", [
    (5, 7, 6, (13, 11, 6), 3, 5, 7),      # every Tx and Rx, ragged bricks, odd receiver count
    (33, 40, 4, (9, 8, 5), 2, 32, 31),    # largest subsets (32 Tx tiles, 31 Rx: padded k-step)
    (9, 3, 4, (8, 8, 4), 1, 1, 1),        # a single row
    (2, 1, 1, (3, 2, 1), 1, 2, 1),        # smallest grid
    (16, 9, 11, (17, 9, 12), 11, 16, 9),  # every row of the matrix (M = 1584)
    (20, 24, 3, (8, 8, 4), 2, 16, 20),    # 1 x 3 output tiles (two waves each, two idle)
    (20, 12, 3, (8, 8, 4), 2, 17, 9),     # 2 x 2 output tiles (two waves each)
    (24, 24, 3, (8, 8, 4), 2, 20, 24),    # 2 x 3 output tiles (one wave each, two idle)
])
def test_structured_ragged_shapes(bd, T, R, F, grid, nf, nt, nr):
    pulse = np.exp(1j * np.linspace(0, 2, F)) * np.linspace(1.0, 0.4, F)
    geom = W.make_geometry(T, R, F, (20e9, 30e9), grid, 4e-3, 0.22, 0.2, pulse=pulse, seed=T * 100 + R)
    structured_case(bd, geom, nf, nt, nr, 700 + T + R, "T%d R%d F%d grid%s (%d,%d,%d)" % (T, R, F, grid, nf, nt, nr))


def test_structured_bad_index_sets_status(bd):
    geom = W.make_geometry(4, 4, 4, (20e9, 30e9), (8, 8, 4), 5e-3, 0.25, 0.2, seed=3)
    plan = bd.Plan(geom)
    s = cdev(W.random_complex(plan.N, seed=4))
    plan.spgm_forward_structured(idev([0, 4]), idev([1]), idev([2]), s)  # frequency 4 is out of range
    assert plan.status() == bd.SPGM_E_BADROW
    assert plan.status() == 0
    with pytest.raises(bd.SpgmError) as e:
        plan.spgm_forward_structured(idev([0]), idev(np.zeros(33)), idev([0]), s)  # nt > 32
    assert e.value.code == bd.SPGM_E_INVALID


def test_c0_structured_step_and_solve(bd):
    cfg = W.CONFIGS["c0"]
    geom = W.config_geometry("c0")
    orc = Oracle(geom)
    plan = bd.Plan(geom)
    s_true, idx = W.config_scene("c0")
    y = W.add_noise(orc.forward_sparse(np.arange(orc.M), idx, s_true[idx]), cfg["snr_db"], seed=cfg["seed"] + 2)
    y = y.astype(np.complex64).astype(np.complex128)
    eta, alpha = 0.009, 0.0014
    T, R, F = cfg["T"], cfg["R"], cfg["F"]
    K = 60
    fs, ts, rs = W.draw_structured_subsets(T, R, F, 8, 4, 8, K, seed=41)  # B = 256, as the c0 minibatch
    rows = np.stack([W.structured_rows(T, R, fs[k], ts[k], rs[k]) for k in range(K)])
    s0 = W.random_complex(orc.N, seed=42).astype(np.complex64)
    s_gpu = cdev(s0)
    plan.spgm_step_structured(idev(fs[0]), idev(ts[0]), idev(rs[0]), cdev(y), s_gpu, eta, alpha)
    check(host(s_gpu), orc.step(rows[0], y, s0.astype(np.complex128), eta, alpha), "c0 structured step")
    s_gpu = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    plan.spgm_solve_structured(idev(fs), idev(ts), idev(rs), cdev(y), s_gpu, eta, alpha)
    check(host(s_gpu), orc.solve(rows, y, np.zeros(orc.N), eta, alpha), "c0 structured solve K=%d" % K)
    assert plan.status() == 0


@pytest.mark.parametrize("iters", [1, 2, 5])
def test_structured_solve_equals_repeated_steps(bd, iters):
    """The structured solve reproduces `iters` single structured steps bit for bit (nonzero
    start, active threshold)."""
    cfg = W.CONFIGS["c0"]
    geom = W.config_geometry("c0")
    plan = bd.Plan(geom)
    T, R, F = cfg["T"], cfg["R"], cfg["F"]
    fs, ts, rs = W.draw_structured_subsets(T, R, F, 4, 8, 6, iters, seed=51)
    y = cdev(W.random_complex(plan.M, seed=52))
    s0 = W.random_complex(plan.N, seed=53).astype(np.complex64)
    eta, alpha = 8e-3, 0.3 / iters
    s_step = cdev(s0)
    for k in range(iters):
        plan.spgm_step_structured(idev(fs[k]), idev(ts[k]), idev(rs[k]), y, s_step, eta, alpha)
    s_solve = cdev(s0)
    plan.spgm_solve_structured(idev(fs), idev(ts), idev(rs), y, s_solve, eta, alpha)
    ref = host(s_step)
    assert np.count_nonzero(ref) not in (0, ref.size)
    assert np.array_equal(host(s_solve), ref)
    assert plan.status() == 0


def test_c1_structured_full_size_sampled(bd):
    """c1 geometry with the structured minibatch (16 f, 16 Tx, 16 Rx; B = 4096 as the c1
    minibatch), full launch; the oracle evaluates 24 sampled rows and 64 sampled voxels."""
    geom = W.config_geometry("c1")
    orc = Oracle(geom)
    plan = bd.Plan(geom)
    fs, ts, rs, rows = subsets(geom, 16, 16, 16, 61)
    s = W.random_complex(orc.N, seed=62).astype(np.complex64)
    r = W.random_complex(rows.size, seed=63).astype(np.complex64)
    y = host(plan.spgm_forward_structured(idev(fs), idev(ts), idev(rs), cdev(s)))
    g = host(plan.spgm_adjoint_structured(idev(fs), idev(ts), idev(rs), cdev(r)))
    rng = np.random.default_rng(64)
    js = np.sort(rng.choice(rows.size, 24, replace=False))
    vs = np.sort(rng.choice(orc.N, 64, replace=False))
    check(y[js], orc.forward(rows[js], s.astype(np.complex128)), "c1 structured forward (24 sampled rows)")
    check(g[vs], orc.adjoint_voxels(rows, r.astype(np.complex128), vs), "c1 structured adjoint (64 sampled voxels)")
    assert plan.status() == 0
