"""Pins for the oracle's other regularisers (the l1 prox of Eq. 5 swapped for another prox; the
paper notes the extension in Sec. III).  Each check rests on a fact of the mathematics, not on
the oracle's formula retyped:

* forward differences of a linear ramp are its slopes, zero on each upper face; the
  difference operator and its adjoint satisfy <D u, w> = <u, D^T w>;
* elastic net: closed form on a 3-4-5 value, zero inside the threshold, the l1 prox at mu = 0
  and the optimality condition of the prox at random points;
* magnitude TV: an image of constant magnitude and weight 0 are fixed points; a 1-D step of
  height h keeps its two levels at a + alpha/L and c - alpha/R (the exact minimiser) along
  each axis; a large weight gives the mean; a 1-D random signal agrees with an independent
  quadratic-programming solve of the same prox; on a 3-D grid the primal-dual gap closes,
  certifying the fixed point; the phase is kept.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import (Oracle, grad3, grad3_adjoint, prox_elastic, prox_l1,
                    prox_tv_magnitude)
from paper_2509_00774_amd import workloads as W


def _phases(rng, n):
    return np.exp(2j * np.pi * rng.random(n))


def _tv(u, grid):
    g = grad3(u, grid)
    return float(np.sum(np.sqrt(np.sum(g * g, axis=0))))


# ---------------------------------------------------------------------------------------
# Difference operator
# ---------------------------------------------------------------------------------------
def test_grad3_linear_ramp():
    nx, ny, nz = 5, 4, 3
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = (ix + 10 * iy + 100 * iz).astype(float)
    g = grad3(u, (nx, ny, nz)).reshape(3, nz, ny, nx)
    assert np.array_equal(g[0], np.where(ix < nx - 1, 1.0, 0.0))
    assert np.array_equal(g[1], np.where(iy < ny - 1, 10.0, 0.0))
    assert np.array_equal(g[2], np.where(iz < nz - 1, 100.0, 0.0))


@pytest.mark.parametrize("grid", [(5, 4, 3), (1, 1, 7), (6, 1, 1), (2, 9, 1)])
def test_grad3_adjoint_identity(grid):
    rng = np.random.default_rng(3)
    N = int(np.prod(grid))
    u = rng.standard_normal(N)
    w = rng.standard_normal((3, N))
    lhs = float(np.sum(grad3(u, grid) * w))
    rhs = float(np.dot(u, grad3_adjoint(w, grid)))
    assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))
    # D annihilates constants, so D^T w sums to zero
    assert abs(np.sum(grad3_adjoint(w, grid))) <= 1e-12 * np.sum(np.abs(w))


def test_grad3_adjoint_one_hot():
    """D^T of a unit dual value at voxel n, direction x, is +1 at n + e_x and -1 at n."""
    grid = (4, 3, 2)
    N = 24
    w = np.zeros((3, N))
    n = (1 * 3 + 2) * 4 + 1  # iz=1, iy=2, ix=1
    w[0, n] = 1.0
    out = grad3_adjoint(w, grid)
    expect = np.zeros(N)
    expect[n + 1] = 1.0
    expect[n] = -1.0
    assert np.array_equal(out, expect)


# ---------------------------------------------------------------------------------------
# Elastic net
# ---------------------------------------------------------------------------------------
def test_elastic_closed_form():
    v = np.array([3 + 4j, 0.3 - 0.4j, -6 + 8j])
    got = prox_elastic(v, 1.0, 0.5)
    # |v| = 5: shrink to 4/5 of v, then scale by 1/1.5; |v| = 0.5 <= 1: zero; |v| = 10: 9/10, /1.5
    expect = np.array([(3 + 4j) * 0.8 / 1.5, 0.0, (-6 + 8j) * 0.9 / 1.5])
    assert np.allclose(got, expect, rtol=0, atol=1e-15)


def test_elastic_mu_zero_is_l1_and_optimal():
    rng = np.random.default_rng(5)
    v = rng.standard_normal(400) + 1j * rng.standard_normal(400)
    assert np.array_equal(prox_elastic(v, 0.7, 0.0), prox_l1(v, 0.7))
    a, mu = 0.7, 2.5
    x = prox_elastic(v, a, mu)
    on = np.abs(x) > 0
    # stationarity of 1/2|x - v|^2 + a|x| + (a mu / 2)|x|^2 where x != 0
    res = x[on] - v[on] + a * x[on] / np.abs(x[on]) + a * mu * x[on]
    assert np.max(np.abs(res)) < 1e-12
    # x = 0 is optimal iff |v| <= a
    assert np.all(np.abs(v[~on]) <= a) and np.all(np.abs(v[on]) > a)


# ---------------------------------------------------------------------------------------
# Magnitude TV
# ---------------------------------------------------------------------------------------
def test_tv_constant_magnitude_and_zero_weight():
    rng = np.random.default_rng(7)
    grid = (4, 3, 2)
    v = 2.5 * _phases(rng, 24)
    assert np.allclose(prox_tv_magnitude(v, grid, 0.7, 50), v, rtol=0, atol=1e-14)
    v2 = rng.standard_normal(24) + 1j * rng.standard_normal(24)
    assert np.array_equal(prox_tv_magnitude(v2, grid, 0.0, 50), v2)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_tv_step_closed_form(axis):
    """A step of L voxels at a and R voxels at c > a keeps two levels: the minimiser of
    L/2 (x - a)^2 + R/2 (y - c)^2 + alpha (y - x) is x = a + alpha/L, y = c - alpha/R (valid while
    those do not cross)."""
    L, R, a, c, alpha = 6, 10, 1.0, 3.0, 0.6
    n = L + R
    grid = [1, 1, 1]
    grid[axis] = n
    rng = np.random.default_rng(11 + axis)
    ph = _phases(rng, n)
    mag = np.r_[np.full(L, a), np.full(R, c)]
    out = prox_tv_magnitude(mag * ph, tuple(grid), alpha, 3000)
    expect = np.r_[np.full(L, a + alpha / L), np.full(R, c - alpha / R)]
    assert np.max(np.abs(np.abs(out) - expect)) < 1e-9
    assert np.max(np.abs(out / np.abs(out) - ph)) < 1e-12


def test_tv_large_weight_gives_mean():
    rng = np.random.default_rng(13)
    grid = (4, 3, 2)
    mag = rng.random(24) + 0.1
    out = prox_tv_magnitude(mag * _phases(rng, 24), grid, 50.0, 4000)
    assert np.max(np.abs(np.abs(out) - mag.mean())) < 1e-6


def test_tv_1d_matches_qp():
    """Independent solve of the 1-D prox as a smooth QP with slack variables t_i >= |u_{i+1} - u_i|."""
    rng = np.random.default_rng(17)
    n, alpha = 12, 0.25
    b = rng.random(n) * 2.0
    out = np.abs(prox_tv_magnitude(b.astype(complex), (n, 1, 1), alpha, 4000))

    def obj(z):
        u, t = z[:n], z[n:]
        return 0.5 * np.sum((u - b) ** 2) + alpha * np.sum(t)

    def jac(z):
        return np.r_[z[:n] - b, np.full(n - 1, alpha)]

    Dm = np.diff(np.eye(n), axis=0)
    cons = [{"type": "ineq", "fun": lambda z: z[n:] - Dm @ z[:n], "jac": lambda z: np.c_[-Dm, np.eye(n - 1)]},
            {"type": "ineq", "fun": lambda z: z[n:] + Dm @ z[:n], "jac": lambda z: np.c_[Dm, np.eye(n - 1)]}]
    z0 = np.r_[b, np.abs(np.diff(b))]
    res = minimize(obj, z0, jac=jac, constraints=cons, method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
    assert res.success
    assert np.max(np.abs(out - res.x[:n])) < 1e-5
    assert 0.5 * np.sum((out - b) ** 2) + alpha * np.sum(np.abs(np.diff(out))) <= res.fun + 1e-9


def test_tv_3d_duality_gap_closes():
    """Primal P(u) = 1/2|u - b|^2 + alpha TV(u); for any dual field with |w_n| <= 1 the value
    q(w) = 1/2|u_w - b|^2 + alpha <D u_w, w>, u_w = max(0, b - alpha D^T w), is a lower bound.
    A vanishing gap certifies that the returned magnitude is the prox."""
    rng = np.random.default_rng(19)
    grid = (5, 4, 3)
    N = 60
    alpha = 0.3
    b = rng.random(N) * 2.0
    ph = _phases(rng, N)
    out, w = prox_tv_magnitude(b * ph, grid, alpha, 3000, return_dual=True)
    u = np.abs(out)
    assert np.max(np.sqrt(np.sum(w * w, axis=0))) <= 1.0 + 1e-12
    u_w = np.maximum(0.0, b - alpha * grad3_adjoint(w, grid))
    assert np.max(np.abs(u - u_w)) < 1e-12
    primal = 0.5 * np.sum((u - b) ** 2) + alpha * _tv(u, grid)
    dual = 0.5 * np.sum((u_w - b) ** 2) + alpha * float(np.sum(grad3(u_w, grid) * w))
    assert dual <= primal + 1e-12
    assert primal - dual < 1e-7 * primal
    # a prox never raises the objective over the input, and the phase is kept
    assert primal <= alpha * _tv(b, grid) + 1e-12
    assert np.max(np.abs(out / u - ph)) < 1e-12


# ---------------------------------------------------------------------------------------
# The iteration with a swapped prox
# ---------------------------------------------------------------------------------------
def test_step_reg_reduces_to_l1_step():
    g = W.make_geometry(3, 4, 5, (20e9, 30e9), (4, 3, 2), 5e-3, 0.25, 0.2, seed=0)
    orc = Oracle(g)
    rng = np.random.default_rng(23)
    y = rng.standard_normal(orc.M) + 1j * rng.standard_normal(orc.M)
    s = rng.standard_normal(orc.N) + 1j * rng.standard_normal(orc.N)
    rows = rng.choice(orc.M, 17, replace=False)
    eta, alpha = 3e-2, 0.4
    ref = orc.step(rows, y, s, eta, alpha)
    assert np.array_equal(orc.step_reg(rows, y, s, eta, alpha, 0), ref)
    assert np.array_equal(orc.step_reg(rows, y, s, eta, alpha, 1, mu=0.0), ref)
    # TV with zero weight and l1 with zero threshold are both the plain gradient step
    plain = orc.step(rows, y, s, eta, 0.0)
    assert np.allclose(orc.step_reg(rows, y, s, eta, 0.0, 2, tv_iters=10), plain, rtol=0, atol=1e-15)
