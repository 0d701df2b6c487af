"""GPU edge cases of the minibatch size: empty and oversize minibatches are refused before any
launch, and the largest minibatch the library accepts (2^24 rows) runs through sorting, the tile
kernels and the reductions with results equal to the FP64 oracle's.

At 2^24 rows of the c0 geometry (M = 1024 distinct rows) every row repeats about 16 000 times.
The forward output of a row depends only on the row, so every copy must equal the oracle's value
for that row (and the copies must agree bitwise: each is formed by the same kernels in the same
order).  For the adjoint only the first copy of each distinct row carries a residual value and
every other copy carries an exact zero, so A_B^H r equals the oracle's adjoint over the distinct
rows; the zeros add exactly in float32, so the float32 projector's bound (relative L2 1e-5,
elementwise 1e-4 of the largest output) applies unchanged while every kernel still walks all
2^24 rows.
"""
import numpy as np
import pytest

from oracle import Oracle, rel_l2
from paper_2509_00774_amd import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-5
ELEM = 1e-4
MAX_B = 1 << 24  # the library's largest minibatch (kMaxB)


def say(*a):
    print("[gpu-edges]", *a, flush=True)


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


def test_empty_and_oversize_minibatches_are_refused(bd):
    """B = 0 and B = 2^24 + 1 return SPGM_E_INVALID from forward, adjoint and step without
    touching the plan: a later call gives bitwise the result of a fresh plan."""
    geom = W.config_geometry("c0")
    plan = bd.Plan(geom)
    s = cdev(W.random_complex(plan.N, seed=11))
    y = cdev(W.random_complex(plan.M, seed=12))
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    say("B=0 and B=%d on forward, adjoint and step" % (MAX_B + 1))
    for call in (lambda rows: plan.forward(rows, s),
                 lambda rows: plan.adjoint(rows, torch.zeros(rows.numel(), dtype=torch.complex64, device="cuda")),
                 lambda rows: plan.spgm_step(rows, y, s.clone(), 1e-3, 0.0)):
        with pytest.raises(bd.SpgmError) as e:
            call(empty)
        assert e.value.code == bd.SPGM_E_INVALID
    big = torch.zeros(MAX_B + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(bd.SpgmError) as e:
        plan.forward(big, s)
    assert e.value.code == bd.SPGM_E_INVALID
    del big
    assert plan.status() == 0
    rows = idev(W.config_rows("c0", K=1)[0])
    got = host(plan.forward(rows, s))
    fresh = bd.Plan(geom)
    assert np.array_equal(got, host(fresh.forward(rows, s)))
    fresh.close()
    plan.close()


def test_largest_minibatch_against_the_oracle(bd):
    """2^24 rows (each of the 1024 distinct rows about 16 000 times, in random order): forward
    outputs equal the oracle's per row and agree bitwise across copies; the adjoint with one
    non-zero residual per distinct row equals the oracle's adjoint over the distinct rows."""
    geom = W.config_geometry("c0")
    orc = Oracle(geom)
    M, N = orc.M, orc.N
    rng = np.random.default_rng(2024)
    rows = rng.integers(0, M, size=MAX_B).astype(np.int32)
    rows[:M] = rng.permutation(M)  # every distinct row occurs
    s = W.random_complex(N, seed=13).astype(np.complex64)
    plan = bd.Plan(geom)
    say("forward with B=%d rows (M=%d, N=%d)" % (MAX_B, M, N))
    y = host(plan.forward(idev(rows), cdev(s)))
    assert plan.status() == 0
    ref_rows = orc.forward(np.arange(M, dtype=np.int32), s.astype(np.complex128))
    uniq, first = np.unique(rows, return_index=True)  # first occurrence of every row
    assert np.array_equal(uniq, np.arange(M))
    check(y[first], ref_rows, "forward, one copy per distinct row")
    assert np.array_equal(y, y[first][rows]), "copies of a row differ"

    rho = W.random_complex(M, seed=14).astype(np.complex64)
    r = np.zeros(MAX_B, dtype=np.complex64)
    r[first] = rho
    say("adjoint with B=%d rows, %d of them non-zero" % (MAX_B, M))
    g = host(plan.adjoint(idev(rows), cdev(r)))
    assert plan.status() == 0
    check(g, orc.adjoint(np.arange(M, dtype=np.int32), rho.astype(np.complex128)), "adjoint, zero residual copies")
    plan.close()
