"""Ragged batches: several scenes of different arrays, bands and grids advanced together by one
launch per phase; each scene's iterate matches the FP64 oracle (relative L2 <= 1e-5) and the
single-plan solve, with and without graph capture."""
import numpy as np
import pytest

from oracle import Oracle, rel_l2
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


SHAPES = [  # T, R, F, grid
    (6, 9, 8, (16, 16, 8)),     # R > T
    (10, 4, 5, (13, 11, 6)),    # ragged bricks
    (8, 8, 12, (8, 8, 4)),
    (5, 5, 3, (24, 8, 12)),
    (12, 7, 6, (17, 9, 5)),
    (3, 11, 9, (9, 16, 4)),
]


def test_ragged_batch_matches_oracle(bd):
    K = 4
    geoms, ys, rows, s_np, etas, alphas = [], [], [], [], [], []
    for i, (T, R, F, grid) in enumerate(SHAPES):
        geom = W.make_geometry(T, R, F, (20e9, 30e9), grid, 4e-3, 0.24, 0.2, seed=300 + i)
        M, N = W.dims(geom)
        B = int(np.ceil(M / 4))
        geoms.append(geom)
        ys.append(W.random_complex(M, seed=400 + i).astype(np.complex64))
        rows.append(W.draw_rows(M, B, K, seed=500 + i))
        s_np.append((0.1 * W.random_complex(N, seed=600 + i)).astype(np.complex64))
        etas.append(2e-3 * (1 + 0.1 * i))
        alphas.append(1e-4)
    batch = bd.Batch(geoms)
    results = {}
    for use_graph in (False, True):
        ss = [torch.from_numpy(v.copy()).cuda() for v in s_np]
        batch.solve([torch.from_numpy(r).cuda() for r in rows], [torch.from_numpy(v).cuda() for v in ys], ss, etas,
                    alphas, use_graph=use_graph)
        torch.cuda.synchronize()
        results[use_graph] = [t.cpu().numpy() for t in ss]
    assert batch.status() == 0
    for a, b in zip(results[False], results[True]):
        assert np.array_equal(a, b)
    for i, geom in enumerate(geoms):
        orc = Oracle(geom)
        ref = orc.solve(rows[i], ys[i].astype(np.complex128), s_np[i].astype(np.complex128), etas[i], alphas[i])
        err = rel_l2(results[False][i], ref)
        plan = bd.Plan(geom)
        s1 = torch.from_numpy(s_np[i].copy()).cuda()
        plan.solve(torch.from_numpy(rows[i]).cuda(), torch.from_numpy(ys[i]).cuda(), s1, etas[i], alphas[i])
        err_plan = rel_l2(results[False][i], s1.cpu().numpy())
        print("[gpu-batch] scene %d %s grid %s: rel_l2 vs oracle %.3e, vs single-plan solve %.3e" % (
            i, SHAPES[i][:3], SHAPES[i][3], err, err_plan), flush=True)
        assert err <= 1e-5
        assert err_plan <= 1e-6
    batch.close()
