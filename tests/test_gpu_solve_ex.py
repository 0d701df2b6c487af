"""spgm_solve_ex: the SPGM solve with options (Sec. IV, Eq. 5 iterated).  Minibatches drawn by the
library's seeded generator give the same iterate, bit for bit, as spgm_solve on the generator's
table, and match the FP64 oracle solve on the oracle's own draw of the same rows (rel-L2 <= 1e-5);
a solve split over calls at start_iter equals one call; the termination rule and structured
subsets go through the same generator."""
import json
import os

import numpy as np
import pytest

import oracle
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


def cdev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex64))).cuda()


def idev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.int32))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def c0_problem():
    cfg = W.CONFIGS["c0"]
    geom = W.config_geometry("c0")
    orc = Oracle(geom)
    st, idx = W.random_scene(orc.N, cfg["density"], seed=cfg["seed"] + 1)
    y = W.add_noise(orc.forward_sparse(np.arange(orc.M), idx, st[idx]), cfg["snr_db"], seed=cfg["seed"] + 2)
    y = y.astype(np.complex64)
    steps = json.load(open(os.path.join(ROOT, "tests", "golden", "step_sizes.json")))["c0"]
    return geom, orc, y, float(np.float32(steps["eta"])), float(steps["lambda"])


@pytest.mark.parametrize("use_graph", [False, True])
def test_generated_rows_match_table_and_oracle(bd, use_graph):
    geom, orc, y, eta, lam = c0_problem()
    plan = bd.Plan(geom)
    B, iters, seed = 256, 8, 4242
    yd = cdev(y)
    s = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    assert plan.spgm_solve_ex(yd, s, iters, eta, lam, B=B, seed=seed, use_graph=use_graph) == iters
    table = bd.rows_generate(seed, 0, iters, orc.M, B)
    s_ref = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    alpha = float(np.float32(lam * eta))
    plan.solve(idev(table), yd, s_ref, eta, alpha)
    assert np.array_equal(host(s), host(s_ref))
    ref = orc.solve(oracle.rows_generate(seed, 0, iters, orc.M, B), y.astype(np.complex128), np.zeros(orc.N), eta,
                    alpha)
    err = rel_l2(host(s), ref)
    print("[solve-ex] generated rows, graph=%s: rel_l2 vs oracle %.3e" % (use_graph, err), flush=True)
    assert err <= 1e-5
    assert plan.status() == 0


@pytest.mark.parametrize("use_graph", [False, True])
def test_resume_at_start_iter(bd, use_graph):
    """solve(K) equals solve(k) followed by solve(K - k, start_iter = k), bit for bit."""
    geom, orc, y, eta, lam = c0_problem()
    plan = bd.Plan(geom)
    yd = cdev(y)
    a = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    plan.spgm_solve_ex(yd, a, 10, eta, lam, B=200, seed=77, use_graph=use_graph)
    b = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    plan.spgm_solve_ex(yd, b, 4, eta, lam, B=200, seed=77, use_graph=use_graph)
    plan.spgm_solve_ex(yd, b, 6, eta, lam, B=200, seed=77, start_iter=4, use_graph=use_graph)
    assert np.array_equal(host(a), host(b))
    c = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    plan.spgm_solve_ex(yd, c, 10, eta, lam, B=200, seed=78, use_graph=use_graph)
    assert not np.array_equal(host(a), host(c))


def test_termination_rule_with_generated_rows(bd):
    geom, orc, y, eta, lam = c0_problem()
    plan = bd.Plan(geom)
    yd = cdev(y)
    B, iters, seed, tol = 256, 60, 9, 0.05  # SPGM at c0 meets tol = 0.05 after about a dozen iterations
    s = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    done = plan.spgm_solve_ex(yd, s, iters, eta, lam, B=B, seed=seed, tol=tol, check_every=5)
    table = idev(bd.rows_generate(seed, 0, iters, orc.M, B))
    s_ref = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    done_ref, _ = plan.spgm_solve_tol(table, yd, s_ref, eta, float(np.float32(lam * eta)), tol, check_every=5,
                                      use_graph=False)
    print("[solve-ex] termination after %d iterations (spgm_solve_tol: %d)" % (done, done_ref), flush=True)
    assert 1 <= done < iters and done == done_ref
    assert np.array_equal(host(s), host(s_ref))


def test_structured_sampling(bd):
    geom, orc, y, eta, lam = c0_problem()
    T, R, F = geom["tx"].shape[0], geom["rx"].shape[0], len(geom["freq"])
    nf, nt, nr, iters, seed = 8, 4, 6, 5, 31
    plan = bd.Plan(geom)
    yd = cdev(y)
    s = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    assert plan.spgm_solve_ex(yd, s, iters, eta, lam, sampling=1, nf=nf, nt=nt, nr=nr, seed=seed) == iters
    f, t, r = bd.subsets_generate(seed, 0, iters, F, T, R, nf, nt, nr)
    s_ref = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    alpha = float(np.float32(lam * eta))
    plan.spgm_solve_structured(idev(f), idev(t), idev(r), yd, s_ref, eta, alpha)
    assert np.array_equal(host(s), host(s_ref))
    fo, to, ro = oracle.subsets_generate(seed, 0, iters, F, T, R, nf, nt, nr)
    table = np.stack([W.structured_rows(T, R, fo[k], to[k], ro[k]) for k in range(iters)])
    ref = orc.solve(table, y.astype(np.complex128), np.zeros(orc.N), eta, alpha)
    err = rel_l2(host(s), ref)
    print("[solve-ex] structured subsets: rel_l2 vs oracle %.3e" % err, flush=True)
    assert err <= 1e-5


def test_given_rows_and_chunked_generation(bd):
    """Given rows run as spgm_solve; at c1 (B = 4096) 1030 drawn iterations span two chunks of
    the generator's staging (1024 iterations each) and still equal spgm_solve on the table."""
    geom, orc, y, eta, lam = c0_problem()
    plan = bd.Plan(geom)
    table = bd.rows_generate(5, 0, 6, orc.M, 128)
    yd = cdev(y)
    a = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    plan.spgm_solve_ex(yd, a, 6, eta, lam, rows=idev(table))
    b = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    plan.solve(idev(table), yd, b, eta, float(np.float32(lam * eta)))
    assert np.array_equal(host(a), host(b))
    g1 = W.config_geometry("c1")
    p1 = bd.Plan(g1)
    M1, N1 = W.dims(g1)
    y1 = cdev(W.random_complex(M1, seed=3))
    s1 = torch.zeros(N1, dtype=torch.complex64, device="cuda")
    p1.spgm_solve_ex(y1, s1, 1030, 1e-3, 0.01, B=4096, seed=11)
    s2 = torch.zeros(N1, dtype=torch.complex64, device="cuda")
    p1.solve(idev(bd.rows_generate(11, 0, 1030, M1, 4096)), y1, s2, 1e-3, float(np.float32(0.01 * 1e-3)))
    assert np.array_equal(host(s1), host(s2))
    assert p1.status() == 0


def test_bad_options(bd):
    geom, orc, y, eta, lam = c0_problem()
    plan = bd.Plan(geom)
    yd = cdev(y)
    s = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
    with pytest.raises(bd.SpgmError) as e:
        plan.spgm_solve_ex(yd, s, 3, eta, lam, B=orc.M + 1, seed=1)
    assert e.value.code == bd.SPGM_E_INVALID
    with pytest.raises(bd.SpgmError) as e:
        plan.spgm_solve_ex(yd, s, 3, -1.0, lam, B=16, seed=1)
    assert e.value.code == bd.SPGM_E_INVALID
    with pytest.raises(bd.SpgmError) as e:
        plan.spgm_solve_ex(yd, s, 3, eta, lam, sampling=1, nf=2, nt=2, nr=2, tol=1e-3)
    assert e.value.code == bd.SPGM_E_UNSUPPORTED
