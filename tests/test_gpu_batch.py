"""Ragged batches: several scenes of different arrays, bands and grids advanced together by one
launch per phase; each scene's iterate matches the FP64 oracle (relative L2 <= 1e-5) and the
single-plan solve, with and without graph capture."""
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


# Scenes that differ in T + R and in the smaller array (LDS layout of each item), one 64x64x32
# grid (512 bricks) and minibatches of up to 1 440 rows (several row ranges at 256 rows each).
WALK = [  # T, R, F, grid
    (6, 9, 8, (64, 64, 32)),
    (12, 12, 40, (16, 16, 8)),   # M = 5 760, B = 1 440: six row ranges of 256
    (20, 5, 6, (24, 8, 12)),
    (4, 16, 10, (13, 11, 6)),
    (9, 9, 16, (32, 16, 8)),
]


def walk_inputs(K):
    geoms, ys, rows, s0 = [], [], [], []
    for i, (T, R, F, grid) in enumerate(WALK):
        geom = W.make_geometry(T, R, F, (20e9, 30e9), grid, 4e-3, 0.24, 0.2, seed=700 + i)
        M, N = W.dims(geom)
        geoms.append(geom)
        ys.append(W.random_complex(M, seed=710 + i).astype(np.complex64))
        rows.append(W.draw_rows(M, int(np.ceil(M / 4)), K, seed=720 + i))
        s0.append((0.1 * W.random_complex(N, seed=730 + i)).astype(np.complex64))
    return geoms, ys, rows, s0


def test_persistent_work_groups_walk_many_items(bd):
    """Four persistent work-groups and 256-row items: every work-group walks well over three
    items across scenes of different antenna counts (LDS re-carved per item), and the column
    sums add several row ranges.  The iterate after two iterations with a non-zero threshold
    matches the oracle (rel-L2 <= 1e-5) for every scene, and does not depend on the grid size
    (bitwise the same as with a full-chip grid) (Sec. IV-A, Eq. 6)."""
    K, rps, wg = 2, 256, 4
    geoms, ys, rows, s0 = walk_inputs(K)
    n_items = 0
    for geom, r in zip(geoms, rows):
        nx, ny, nz = geom["grid"]
        n_items += (-(-nx // 8)) * (-(-ny // 8)) * (-(-nz // 4)) * (-(-r.shape[1] // rps))
    assert n_items >= 3 * wg
    assert max(-(-r.shape[1] // rps) for r in rows) >= 4
    etas = [2e-3 * (1 + 0.1 * i) for i in range(len(geoms))]
    # thresholds at the median magnitude of each scene's first gradient step (oracle), so that
    # the prox zeroes about half of the voxels
    alphas = []
    for i, geom in enumerate(geoms):
        s64 = s0[i].astype(np.complex128)
        v = s64 - etas[i] * Oracle(geom).gradient(rows[i][0], ys[i].astype(np.complex128), s64)
        alphas.append(float(np.float32(np.median(np.abs(v)))))
    batch = bd.Batch(geoms)
    out = {}
    for max_wg in (wg, 0):
        batch.options(max_workgroups=max_wg, rows_per_split=rps)
        ss = [torch.from_numpy(v.copy()).cuda() for v in s0]
        batch.solve([torch.from_numpy(r).cuda() for r in rows], [torch.from_numpy(v).cuda() for v in ys], ss, etas,
                    alphas, use_graph=True)
        torch.cuda.synchronize()
        out[max_wg] = [t.cpu().numpy() for t in ss]
    assert batch.status() == 0
    batch.close()
    for a, b in zip(out[wg], out[0]):
        assert np.array_equal(a, b)
    print("[gpu-batch] %d items on %d work-groups" % (n_items, wg), flush=True)
    for i, geom in enumerate(geoms):
        ref = Oracle(geom).solve(rows[i], ys[i].astype(np.complex128), s0[i].astype(np.complex128), etas[i],
                                 alphas[i])
        err = rel_l2(out[wg][i], ref)
        zeros = int(np.sum(ref == 0))
        print("[gpu-batch] walk scene %d %s: rel_l2 %.3e, %d thresholded voxels" % (i, WALK[i], err, zeros), flush=True)
        assert err <= 1e-5
        assert zeros > 0


def test_options_are_validated(bd):
    geoms, _, _, _ = walk_inputs(1)
    batch = bd.Batch(geoms[2:3])
    for bad in ((-1, 0), (0, -64), (0, 100)):
        with pytest.raises(bd.SpgmError):
            batch.options(*bad)
    batch.close()


def test_c3_scale_first_iteration(bd):
    """All 96 scenes of the ragged workload (T, R in 8..32, F in 16..64, grids up to 64x64x32,
    B = ceil(M/4)) in one batch: the first iteration from s = 0 with a threshold that zeroes
    about half of each scene's voxels, against the oracle on a seeded 1 % voxel sample of every
    scene (from zero the iterate needs only A_B^H y_B there).  Then two iterations of the
    scenes with the smallest grids, against the oracle's full iterates."""
    scenes = W.ragged_scenes()
    n = len(scenes)
    steps = json.load(open(os.path.join(ROOT, "tests", "golden", "step_sizes.json")))["c3"]["scenes"]
    ys, rows, etas, alphas, samples = [], [], [], [], []
    t_or = 0.0
    import time
    for i, sc in enumerate(scenes):
        orc = Oracle(sc["geom"])
        y = W.random_complex(sc["M"], seed=sc["seed"] + 40).astype(np.complex64)
        r = W.draw_rows(sc["M"], sc["B"], 2, seed=sc["seed"] + 41)
        vs = W.voxel_sample(sc["N"], 0.01, seed=sc["seed"] + 42)
        eta = float(np.float32(steps[i]["eta"]))
        t0 = time.perf_counter()
        v = (eta / sc["B"]) * orc.adjoint_voxels(r[0], y[r[0]].astype(np.complex128), vs)
        t_or += time.perf_counter() - t0
        alpha = float(np.float32(np.median(np.abs(v))))  # threshold from the oracle's own values
        ys.append(y)
        rows.append(r)
        etas.append(eta)
        alphas.append(alpha)
        samples.append((vs, v))
    print("[gpu-batch] c3: oracle first steps on 1%% samples: %.1f s" % t_or, flush=True)
    batch = bd.Batch([sc["geom"] for sc in scenes])
    ss = [torch.zeros(sc["N"], dtype=torch.complex64, device="cuda") for sc in scenes]
    yd = [torch.from_numpy(y).cuda() for y in ys]
    batch.solve([torch.from_numpy(r[:1].copy()).cuda() for r in rows], yd, ss, etas, alphas, use_graph=True)
    torch.cuda.synchronize()
    assert batch.status() == 0
    from oracle import prox_l1
    worst = 0.0
    for i in range(n):
        vs, v = samples[i]
        ref = prox_l1(v, alphas[i])
        got = ss[i].cpu().numpy()[vs]
        err = rel_l2(got, ref)
        worst = max(worst, err)
        assert err <= 1e-5, (i, err)
        assert 0.3 < np.mean(ref == 0) < 0.7
    print("[gpu-batch] c3 first iteration, %d scenes: worst rel_l2 %.3e" % (n, worst), flush=True)
    small = [i for i, sc in enumerate(scenes) if sc["N"] <= 2048]
    ss2 = [torch.zeros(sc["N"], dtype=torch.complex64, device="cuda") for sc in scenes]
    batch.solve([torch.from_numpy(r).cuda() for r in rows], yd, ss2, etas, alphas, use_graph=False)
    torch.cuda.synchronize()
    batch.close()
    for i in small:
        sc = scenes[i]
        ref = Oracle(sc["geom"]).solve(rows[i], ys[i].astype(np.complex128), np.zeros(sc["N"]), etas[i], alphas[i])
        err = rel_l2(ss2[i].cpu().numpy(), ref)
        assert err <= 1e-5, (i, err)
    print("[gpu-batch] c3 two iterations of the %d smallest scenes match" % len(small), flush=True)
