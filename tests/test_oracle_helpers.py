"""Pins for the oracle's helper functions that set inputs or score results: the Lipschitz
estimate that fixes every step size, and the PSNR over normalised magnitudes (Sec. V's image
metric), plus the study's own copy of that metric.  Each test checks against something other
than the function's formula: an eigen-solve of the dense matrix, closed-form values and
invariances.

Planted mistakes each test is built to catch:
* lipschitz: dividing by M instead of B (value off by M/B), too few power iterations (an
  underestimate), forgetting the adjoint (A A^H is the wrong size);
* psnr_magnitude / psnr_normalised: dropping the max-normalisation (the value changes when an
  input is scaled), using the complex values instead of magnitudes (a phase rotation changes
  it), swapping mean for sum (the 9.03 dB case gives 6.02 dB).
"""
import numpy as np
import pytest

from oracle import Oracle, psnr_magnitude
from paper_2509_00774_amd import workloads as W
from paper_2509_00774_amd.study import psnr_normalised


def tiny_problem():
    geom = W.make_geometry(3, 4, 5, (20e9, 30e9), (4, 3, 2), 5e-3, 0.25, 0.2, seed=11)
    orc = Oracle(geom)
    rows = W.draw_rows(orc.M, 20, 1, seed=12)[0]
    return orc, rows


def test_lipschitz_equals_top_eigenvalue_of_dense_normal_matrix():
    """lipschitz(rows) is the largest eigenvalue of A_B^H A_B / B: compared with LAPACK's Hermitian
    eigen-solve of the dense 24 x 24 matrix built from the entries of Eq. 2 (whose closed forms are
    pinned separately).  A division by M instead of B would be off by a factor 3."""
    orc, rows = tiny_problem()
    A = orc.dense(rows)
    H = A.conj().T @ A / rows.size
    ev = np.linalg.eigvalsh(H)
    top, second = ev[-1], ev[-2]
    assert second / top < 0.99  # a spectral gap, so 600 power iterations converge far below 1e-8
    got = orc.lipschitz(rows, iters=600, seed=3)
    assert abs(got - top) <= 1e-8 * top, (got, top)
    # the planted mistake (1/M instead of 1/B) is far outside the tolerance
    assert abs(top * rows.size / orc.M - top) > 1e-3 * top


def test_lipschitz_few_iterations_never_overestimates():
    """A Rayleigh quotient of a Hermitian positive semi-definite matrix never exceeds its top
    eigenvalue: short power iterations can only underestimate L."""
    orc, rows = tiny_problem()
    A = orc.dense(rows)
    top = np.linalg.eigvalsh(A.conj().T @ A / rows.size)[-1]
    for iters in (1, 2, 5, 20):
        assert orc.lipschitz(rows, iters=iters, seed=5) <= top * (1 + 1e-12)


@pytest.mark.parametrize("psnr", [psnr_magnitude, psnr_normalised], ids=["oracle", "study"])
def test_psnr_closed_forms(psnr):
    """Identical inputs give infinity; |a| = [1, 0.5] against |b| = [1, 0] has mean squared error
    0.125 after normalisation to peak 1, i.e. 10 log10(8) = 9.0309 dB."""
    a = np.array([1.0, 0.5])
    b = np.array([1.0, 0.0])
    assert psnr(a, a) == float("inf")
    assert abs(psnr(a, b) - 10 * np.log10(8.0)) < 1e-12
    assert abs(10 * np.log10(8.0) - 9.030899869919435) < 1e-12


@pytest.mark.parametrize("psnr", [psnr_magnitude, psnr_normalised], ids=["oracle", "study"])
def test_psnr_invariances(psnr):
    """Scaling either input by a positive constant or rotating its phases changes nothing (the
    metric is over magnitudes normalised to peak 1)."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    ref = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    base = psnr(x, ref)
    assert np.isfinite(base)
    for sx, sr in ((3.7, 1.0), (1.0, 0.02), (1e-6, 1e6)):
        assert abs(psnr(sx * x, sr * ref) - base) < 1e-9
    rot = np.exp(1j * rng.uniform(0, 2 * np.pi, 50))
    assert abs(psnr(x * rot, ref) - base) < 1e-9
    # a metric without the normalisation would move by 20 log10(3.7) under the first scaling
    a, b = np.abs(x), np.abs(ref)
    raw = lambda u, v: 10 * np.log10(1.0 / np.mean((u - v) ** 2))  # noqa: E731
    assert abs(raw(3.7 * a, b) - raw(a, b)) > 1.0


@pytest.mark.parametrize("psnr", [psnr_magnitude, psnr_normalised], ids=["oracle", "study"])
def test_psnr_single_defect(psnr):
    """N magnitudes equal to 1 except one at 0: the mean squared error is 1/N, so the PSNR is
    10 log10(N) exactly (N = 1000: 30 dB)."""
    ref = np.ones(1000)
    x = ref.copy()
    x[17] = 0.0
    assert abs(psnr(x, ref) - 30.0) < 1e-9


# ---------------------------------------------------------------------------------------
# Termination rule of Sec. V (relative change of the magnitudes), on an iteration with a
# closed form: one voxel, every row in every iteration (B = M), no threshold.  Then
#     s_k - s* = q^k (s_0 - s*),  q = 1 - eta c,  c = (1/M) sum_m |A_m|^2,
# with s* the least-squares value, and |A_m| = 1/(4 pi d_T d_R) for p = 1 (Eq. 2).
# ---------------------------------------------------------------------------------------
def one_voxel_problem():
    tx = [[0.03, -0.02, 0.0], [-0.05, 0.04, 0.0], [0.01, 0.06, 0.0]]
    rx = [[0.02, 0.02, 0.0], [-0.04, -0.03, 0.0]]
    freq = np.linspace(20e9, 30e9, 4)
    geom = {"tx": np.asarray(tx), "rx": np.asarray(rx), "freq": freq, "pulse": None, "grid": (1, 1, 1),
            "centre": np.array([0.01, -0.01, 0.3]), "pitch": np.array([1e-3, 1e-3, 1e-3]), "c": 3.0e8}
    orc = Oracle(geom)
    # c from the geometry alone (numpy distances), not from the oracle's entries
    dT = np.linalg.norm(np.asarray(tx) - geom["centre"], axis=1)
    dR = np.linalg.norm(np.asarray(rx) - geom["centre"], axis=1)
    amp2 = (1.0 / (4 * np.pi * dT[:, None] * dR[None, :])) ** 2  # [t][r], same for every f
    c = float(np.mean(np.broadcast_to(amp2, (len(freq),) + amp2.shape)))
    rng = np.random.default_rng(4)
    y = rng.standard_normal(orc.M) + 1j * rng.standard_normal(orc.M)
    return orc, c, y


@pytest.mark.parametrize("tol,k_stop", [(0.6, 2), (0.4, 3), (0.1, 4), (0.05, 5), (0.02, 6), (0.01, 7)])
def test_solve_tol_stopping_iteration_by_hand(tol, k_stop):
    """eta c = 1/2 and s_0 = 0 give |s_k| = |s*| (1 - 2^-k), so the relative change of the
    magnitudes at iteration k is 2^-k / (1 - 2^-(k-1)): 0.5, 0.167, 0.0714, 0.0333, 0.0161,
    0.00794 for k = 2..7 (at k = 1 the previous iterate is zero and the rule is not met).  The
    stopping iterations follow by hand.  Planted mistakes caught: measuring the change against
    the new iterate (tol 0.4 would stop at k = 2), stopping at the first iteration after a zero
    iterate, or counting iterations from zero."""
    orc, c, y = one_voxel_problem()
    eta = 0.5 / c
    rows = np.tile(np.arange(orc.M, dtype=np.int32), (20, 1))
    s, k = orc.solve_tol(rows, y, np.zeros(1), eta, 0.0, tol)
    assert k == k_stop
    # the iterate returned is the one after k_stop iterations
    assert np.array_equal(s, orc.solve(rows[:k_stop], y, np.zeros(1), eta, 0.0))
    # and |s_k| = |s*| (1 - 2^-k) with s* the limit
    s_inf = orc.solve(rows, y, np.zeros(1), eta, 0.0)  # 20 iterations: 2^-20 from the limit
    assert abs(abs(s[0]) - abs(s_inf[0]) * (1 - 2.0 ** -k_stop) / (1 - 2.0 ** -20)) < 1e-12 * abs(s_inf[0])


def test_solve_tol_measures_magnitudes_not_complex_values():
    """s_0 = j s* rotates the phase along the way: s_k = s* (1 - q^k + j q^k), q = 1/2, so |s_k| =
    |s*| sqrt((1 - q^k)^2 + q^2k) = |s*| (1, 0.7071, 0.7906, ...).  The change of the magnitudes at
    k = 1 is 0.2929 (< 0.3: stop), while the change of the complex values is 0.7071 (a rule on
    complex values would run on to k = 3, where it is 0.2236)."""
    orc, c, y = one_voxel_problem()
    eta = 0.5 / c
    rows = np.tile(np.arange(orc.M, dtype=np.int32), (40, 1))
    s_star = orc.solve(rows, y, np.zeros(1), eta, 0.0)  # 2^-40 from the limit
    _, k = orc.solve_tol(rows, y, 1j * s_star, eta, 0.0, 0.3)
    assert k == 1
    _, k = orc.solve_tol(rows, y, 1j * s_star, eta, 0.0, 0.29)
    # magnitudes 0.7071, 0.7906, 0.8839, 0.9396: changes 0.1180, 0.1180, 0.0631 -> stops at k = 2
    assert k == 2


def test_solve_tol_zero_tolerance_and_zero_iterate():
    """tol = 0 runs every iteration; an iterate that stays at zero (lambda above lambda_max) never
    meets the rule, so the solve runs to the iteration cap."""
    orc, c, y = one_voxel_problem()
    eta = 0.5 / c
    rows = np.tile(np.arange(orc.M, dtype=np.int32), (6, 1))
    s, k = orc.solve_tol(rows, y, np.zeros(1), eta, 0.0, 0.0)
    assert k == 6 and np.array_equal(s, orc.solve(rows, y, np.zeros(1), eta, 0.0))
    big = 10.0 * orc.lambda_max(y) * eta
    s, k = orc.solve_tol(rows, y, np.zeros(1), eta, big, 0.5)
    assert k == 6 and s[0] == 0
