"""GPU parity of the shared-geometry batched path (K right-hand sides through one set of entries,
16-bit operands on the matrix cores) against the FP64 oracle applied column by column.

Stated error bounds.
* Elementwise (every case): each product E * S (or conj(E) * R) carries two roundings to the
  16-bit type, one of the entry and one of the right-hand side, each of relative size <= u in
  complex modulus (u = 2^-8 for bfloat16, 2^-11 for half).  Products of 16-bit values are exact
  in float32, so
      |got - exact| <= (2u + u^2) * sum |A| |X|  +  1e-4 * sum |A| |X|,
  the last term an allowance for the float32 phase and the float32 accumulation order.
* Relative L2 of each output column (long sums only, c0 and c1): the roundings are independent,
  with relative RMS about 0.72 ulp(1) / sqrt(12) each (1.6e-3 bfloat16, 2.0e-4 half), about
  2.3e-3 and 2.9e-4 for a product, and sums of many terms keep that relative size:
      bfloat16: <= 6e-3,   half: <= 8e-4   (about 2.5x the estimate).
A full SPGM solve with the batched operators is compared with the float32 projector's solve at
matched reconstruction error: NMSE against the true scene within 0.1 dB, scene by scene.
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
TOL = {0: 6e-3, 1: 8e-4}
PREC_NAME = {0: "bf16", 1: "fp16"}


def say(*a):
    print("[gpu-batched]", *a, flush=True)


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


def rand_matrix(rows, cols, seed):
    return W.random_complex(rows * cols, seed=seed).reshape(rows, cols).astype(np.complex64)


def check_cols(got, ref, tol, what):
    """Relative L2 error of every column (and of the whole matrix) against the reference."""
    per = np.array([rel_l2(got[:, k], ref[:, k]) for k in range(ref.shape[1])])
    tot = rel_l2(got, ref)
    say("%s: rel_l2 all %.3e, worst column %.3e, mean column %.3e" % (what, tot, per.max(), per.mean()))
    assert per.max() <= tol, (what, per.max())
    return per


UNIT = {0: 2.0 ** -8, 1: 2.0 ** -11}
FP32_ALLOW = 1e-4


def check_bound(got, ref, weight, prec, what):
    """Elementwise |got - ref| <= (2u + u^2 + 1e-4) * weight with weight = sum |A| |X|."""
    u = UNIT[prec]
    lim = (2.0 * u + u * u + FP32_ALLOW) * weight
    ratio = float(np.max(np.abs(got - ref) / np.maximum(lim, 1e-300)))
    say("%s: worst |err| / bound = %.3f" % (what, ratio))
    assert ratio <= 1.0, (what, ratio)


def abs_entries(orc, geom, rows, voxels):
    """|A_{m,n}| = |p(f)| / (4 pi d_T d_R) for the given rows and voxels (error-bound weights)."""
    T, R = geom["tx"].shape[0], geom["rx"].shape[0]
    rows = np.asarray(rows, dtype=np.int64)
    f, t, r = rows // (T * R), (rows // R) % T, rows % R
    pf = np.ones(rows.size) if geom["pulse"] is None else np.abs(np.asarray(geom["pulse"]))[f]
    pos = np.stack([orc.voxel_position(int(n)) for n in voxels])
    dT = np.linalg.norm(geom["tx"][t][:, None, :] - pos[None], axis=2)
    dR = np.linalg.norm(geom["rx"][r][:, None, :] - pos[None], axis=2)
    return pf[:, None] / (4.0 * np.pi * dT * dR)


def oracle_forward(orc, rows, S):
    return np.stack([orc.forward(rows, S[:, k].astype(np.complex128)) for k in range(S.shape[1])], axis=1)


def oracle_adjoint(orc, rows, R):
    return np.stack([orc.adjoint(rows, R[:, k].astype(np.complex128)) for k in range(R.shape[1])], axis=1)


def batched_case(bd, geom, rows, K, prec, seed, what, long_sums=False):
    orc = Oracle(geom)
    plan = bd.Plan(geom)
    S = rand_matrix(orc.N, K, seed)
    R = rand_matrix(len(rows), K, seed + 1)
    Y = host(plan.spgm_forward_batched(idev(rows), cdev(S), precision=prec))
    G = host(plan.spgm_adjoint_batched(idev(rows), cdev(R), precision=prec))
    assert Y.shape == (len(rows), K) and G.shape == (orc.N, K)
    absA = np.abs(orc.dense(rows))
    y_ref, g_ref = oracle_forward(orc, rows, S), oracle_adjoint(orc, rows, R)
    name = PREC_NAME[prec]
    check_bound(Y, y_ref, absA @ np.abs(S), prec, what + " forward " + name)
    check_bound(G, g_ref, absA.T @ np.abs(R), prec, what + " adjoint " + name)
    if long_sums:
        check_cols(Y, y_ref, TOL[prec], what + " forward " + name)
        check_cols(G, g_ref, TOL[prec], what + " adjoint " + name)
    assert plan.status() == 0
    plan.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_c0_batched_projector(bd, prec):
    geom = W.config_geometry("c0")
    rows = W.config_rows("c0", K=1)[0]
    batched_case(bd, geom, rows, 32, prec, 300 + prec, "c0 K=32", long_sums=True)


@pytest.mark.parametrize("T,R,F,grid,B,K", [
    (5, 7, 6, (13, 11, 6), 37, 5),     # R > T, ragged bricks, K < 32
    (9, 3, 4, (8, 8, 4), 1, 1),        # a single row and a single right-hand side
    (6, 6, 3, (17, 9, 5), 108, 33),    # every row of the matrix, two passes (32 + 1)
    (2, 1, 1, (3, 2, 1), 2, 3),        # smallest grid
    (8, 8, 16, (16, 16, 8), 700, 40),  # several 32-row tiles and row groups, K = 40
])
def test_batched_ragged_shapes(bd, T, R, F, grid, B, K):
    pulse = np.exp(1j * np.linspace(0, 2, F)) * np.linspace(1.0, 0.4, F)
    geom = W.make_geometry(T, R, F, (20e9, 30e9), grid, 4e-3, 0.22, 0.2, pulse=pulse, seed=T * 100 + R)
    M = F * T * R
    rng = np.random.default_rng(B + K)
    rows = np.arange(M) if B == M else rng.integers(0, M, size=B)  # repeats allowed
    batched_case(bd, geom, rows.astype(np.int32), K, 0, 400 + B, "ragged T%d R%d grid%s B%d K%d" % (T, R, grid, B, K))


def test_batched_columns_match_single_rhs_calls(bd):
    """Column k of a K = 32 call equals a K = 1 call on that column (same entries, same sums)."""
    geom = W.config_geometry("c0")
    plan = bd.Plan(geom)
    rows = idev(W.config_rows("c0", K=1)[0])
    S = rand_matrix(plan.N, 32, 41)
    Y = host(plan.spgm_forward_batched(rows, cdev(S)))
    for k in (0, 17, 31):
        yk = host(plan.spgm_forward_batched(rows, cdev(S[:, k:k + 1].copy())))
        assert np.array_equal(yk[:, 0], Y[:, k])


def test_batched_bitwise_reproducible(bd):
    geom = W.config_geometry("c0")
    plan = bd.Plan(geom)
    rows = idev(W.config_rows("c0", K=1)[0])
    S = cdev(rand_matrix(plan.N, 32, 42))
    R = cdev(rand_matrix(rows.numel(), 32, 43))
    assert np.array_equal(host(plan.spgm_forward_batched(rows, S)), host(plan.spgm_forward_batched(rows, S)))
    assert np.array_equal(host(plan.spgm_adjoint_batched(rows, R)), host(plan.spgm_adjoint_batched(rows, R)))


def test_batched_bad_row_and_unsupported_mode(bd):
    geom = W.make_geometry(4, 4, 4, (20e9, 30e9), (8, 8, 4), 5e-3, 0.25, 0.2, seed=3)
    plan = bd.Plan(geom)
    S = cdev(rand_matrix(plan.N, 4, 44))
    plan.spgm_forward_batched(idev([0, 1, plan.M]), S)
    assert plan.status() == bd.SPGM_E_BADROW
    assert plan.status() == 0
    with pytest.raises(bd.SpgmError) as e:
        plan.spgm_forward_batched(idev([0, 1]), S, precision=7)
    assert e.value.code == bd.SPGM_E_INVALID
    f64 = bd.Plan(geom, phase_mode=bd.PHASE_F64)
    with pytest.raises(bd.SpgmError) as e:
        f64.spgm_forward_batched(idev([0, 1]), S)
    assert e.value.code == bd.SPGM_E_UNSUPPORTED


def test_c1_batched_full_size_sampled(bd):
    """Full c1 launch shape (B = 4096, N = 131072, K = 32) as timed by the batched benchmark; the
    oracle evaluates 16 sampled rows and 48 sampled voxels for every column."""
    geom = W.config_geometry("c1")
    orc = Oracle(geom)
    plan = bd.Plan(geom)
    rows = W.config_rows("c1", K=1)[0]
    K = 32
    S = rand_matrix(orc.N, K, 51)
    R = rand_matrix(rows.size, K, 52)
    Y = host(plan.spgm_forward_batched(idev(rows), cdev(S)))
    G = host(plan.spgm_adjoint_batched(idev(rows), cdev(R)))
    rng = np.random.default_rng(53)
    js = np.sort(rng.choice(rows.size, 16, replace=False))
    vs = np.sort(rng.choice(orc.N, 48, replace=False))
    say("c1: oracle on %d rows and %d voxels x %d columns" % (js.size, vs.size, K))
    y_ref = np.stack([orc.forward(rows[js], S[:, k].astype(np.complex128)) for k in range(K)], axis=1)
    g_ref = np.stack([orc.adjoint_voxels(rows, R[:, k].astype(np.complex128), vs) for k in range(K)], axis=1)
    check_cols(Y[js], y_ref, TOL[0], "c1 K=32 forward (16 sampled rows)")
    check_cols(G[vs], g_ref, TOL[0], "c1 K=32 adjoint (48 sampled voxels)")
    check_bound(Y[js], y_ref, np.abs(orc.dense(rows[js])) @ np.abs(S), 0, "c1 K=32 forward (16 sampled rows)")
    check_bound(G[vs], g_ref, abs_entries(orc, geom, rows, vs).T @ np.abs(R), 0, "c1 K=32 adjoint (48 sampled voxels)")
    assert plan.status() == 0


def c0_scenes(K):
    """K c0-shaped problems sharing the geometry: scene k from seed 1000 + k, 30 dB noise."""
    cfg = W.CONFIGS["c0"]
    geom = W.config_geometry("c0")
    orc = Oracle(geom)
    S_true = np.zeros((orc.N, K), dtype=np.complex128)
    Y = np.zeros((orc.M, K), dtype=np.complex128)
    for k in range(K):
        s, idx = W.random_scene(orc.N, cfg["density"], seed=1000 + k)
        S_true[:, k] = s
        Y[:, k] = W.add_noise(orc.forward_sparse(np.arange(orc.M), idx, s[idx]), cfg["snr_db"], seed=2000 + k)
    Y = Y.astype(np.complex64).astype(np.complex128)
    steps = json.load(open(os.path.join(ROOT, "tests", "golden", "step_sizes.json")))["c0"]
    eta = float(np.float32(steps["eta"]))
    alpha = float(np.float32(steps["lambda"] * eta))
    return geom, orc, S_true, Y, eta, alpha


@pytest.mark.parametrize("prec", [0, 1])
def test_c0_batched_step(bd, prec):
    geom, orc, S_true, Y, eta, alpha = c0_scenes(4)
    plan = bd.Plan(geom)
    rows = W.config_rows("c0", K=1)[0]
    S0 = rand_matrix(orc.N, 4, 61)
    S = cdev(S0)
    plan.spgm_step_batched(idev(rows), cdev(Y), S, eta, alpha, precision=prec)
    ref = np.stack([orc.step(rows, Y[:, k], S0[:, k].astype(np.complex128), eta, alpha) for k in range(4)], axis=1)
    check_cols(host(S), ref, TOL[prec], "c0 batched step " + PREC_NAME[prec])


def nmse_db(s, t):
    return 10.0 * np.log10(np.sum(np.abs(s - t) ** 2) / np.sum(np.abs(t) ** 2))


@pytest.mark.parametrize("prec", [0, 1])
def test_c0_batched_solve_matches_fp32_reconstruction(bd, prec):
    """K = 8 scenes, 200 SPGM iterations: batched 16-bit solve vs the float32 projector's solve of
    each scene (same rows, step and threshold).  NMSE to the true scene within 0.1 dB."""
    K = 8
    geom, orc, S_true, Y, eta, alpha = c0_scenes(K)
    plan = bd.Plan(geom)
    table = idev(W.config_rows("c0"))  # 200 x 256
    Sb = torch.zeros(orc.N, K, dtype=torch.complex64, device="cuda")
    plan.spgm_solve_batched(table, cdev(Y), Sb, eta, alpha, precision=prec)
    Sb = host(Sb)
    worst = 0.0
    for k in range(K):
        s32 = torch.zeros(orc.N, dtype=torch.complex64, device="cuda")
        plan.solve(table, cdev(Y[:, k]), s32, eta, alpha)
        s32 = host(s32)
        d = abs(nmse_db(Sb[:, k], S_true[:, k]) - nmse_db(s32, S_true[:, k]))
        worst = max(worst, d)
        say("%s scene %d: NMSE batched %.3f dB, float32 %.3f dB, iterate rel diff %.2e" % (
            PREC_NAME[prec], k, nmse_db(Sb[:, k], S_true[:, k]), nmse_db(s32, S_true[:, k]), rel_l2(Sb[:, k], s32)))
    assert worst <= 0.1
    assert plan.status() == 0


@pytest.mark.parametrize("K,B,iters", [
    (8, 256, 5),    # c0 (8 bricks, one row split): each step's adjoint hands the packed S to the next forward
    (40, 256, 3),   # two passes of right-hand sides: every forward packs S itself
    (8, 700, 3),    # 8 bricks and 700 rows: the adjoint splits the rows and sums the splits separately
])
def test_batched_solve_equals_repeated_steps(bd, K, B, iters):
    """spgm_solve_batched gives bit for bit the iterates of `iters` separate spgm_step_batched calls
    on the same row table; with several row splits, one step is also checked against the oracle."""
    geom = W.config_geometry("c0")
    orc = Oracle(geom)
    rng = np.random.default_rng(K * 1000 + B)
    table = rng.integers(0, orc.M, size=(iters, B)).astype(np.int32)
    Y = rand_matrix(orc.M, K, 71 + K).astype(np.complex128)
    S0 = rand_matrix(orc.N, K, 72 + K)
    steps = json.load(open(os.path.join(ROOT, "tests", "golden", "step_sizes.json")))["c0"]
    eta = float(np.float32(steps["eta"]))
    alpha = float(np.float32(0.02 * eta))
    plan = bd.Plan(geom)
    Yd = cdev(Y)
    Ss = cdev(S0)
    plan.spgm_solve_batched(idev(table), Yd, Ss, eta, alpha, precision=0)
    St = cdev(S0)
    for i in range(iters):
        plan.spgm_step_batched(idev(table[i]), Yd, St, eta, alpha, precision=0)
        if i == 0 and B > 512:
            ref = np.stack([orc.step(table[0], Y[:, k], S0[:, k].astype(np.complex128), eta, alpha)
                            for k in range(K)], axis=1)
            check_cols(host(St), ref, TOL[0], "c0 batched step, split rows")
    a, b = host(Ss), host(St)
    say("K=%d B=%d: solve vs steps max |diff| %.3g" % (K, B, float(np.max(np.abs(a - b)))))
    assert np.array_equal(a, b)
    assert plan.status() == 0
