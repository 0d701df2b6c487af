"""Autotuner: chosen row splits are within range, parity holds with them, and a second plan with
the same key reads them back from the JSON cache."""
import json

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


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_autotune_and_cache(bd, name, tmp_path):
    geom = W.config_geometry(name)
    B = W.CONFIGS[name]["B"]
    cache = tmp_path / "tune.json"
    plan = bd.Plan(geom)
    fs, as_ = plan.autotune(B, str(cache))
    print("[autotune] %s B=%d: forward splits %d, adjoint splits %d" % (name, B, fs, as_), flush=True)
    assert 1 <= fs <= (B + 63) // 64 and 1 <= as_ <= (B + 63) // 64
    data = json.load(open(cache))
    assert len(data) == 1 and list(data.values())[0][:2] == [fs, as_]
    # parity with the tuned launch shapes
    orc = Oracle(geom)
    rows = W.config_rows(name, K=1)[0]
    s = W.random_complex(orc.N, seed=3).astype(np.complex64)
    r = W.random_complex(B, seed=4).astype(np.complex64)
    y = plan.forward(torch.from_numpy(rows).cuda(), torch.from_numpy(s).cuda()).cpu().numpy()
    g = plan.adjoint(torch.from_numpy(rows).cuda(), torch.from_numpy(r).cuda()).cpu().numpy()
    js = np.arange(0, B, max(1, B // 32))
    vs = np.arange(0, orc.N, max(1, orc.N // 64))
    assert rel_l2(y[js], orc.forward(rows[js], s.astype(np.complex128))) <= 1e-5
    assert rel_l2(g[vs], orc.adjoint_voxels(rows, r.astype(np.complex128), vs)) <= 1e-5
    # a second plan applies the cached choice
    plan2 = bd.Plan(geom)
    assert plan2.autotune(B, str(cache)) == (fs, as_)


def test_c1_every_candidate_split(bd, tmp_path):
    """Parity at full c1 size for every row split the autotuner may choose (forced through the
    cache file), so the launch shape a benchmark run ends up timing is covered whichever wins."""
    geom = W.config_geometry("c1")
    B = W.CONFIGS["c1"]["B"]
    cache = tmp_path / "tune.json"
    bd.Plan(geom).autotune(B, str(cache))
    key = list(json.load(open(cache)).keys())[0]
    orc = Oracle(geom)
    rows = W.config_rows("c1", K=1)[0]
    s = W.random_complex(orc.N, seed=5).astype(np.complex64)
    r = W.random_complex(B, seed=6).astype(np.complex64)
    js = np.arange(0, B, B // 32)
    vs = np.arange(0, orc.N, orc.N // 64)
    y_ref = orc.forward(rows[js], s.astype(np.complex128))
    g_ref = orc.adjoint_voxels(rows, r.astype(np.complex128), vs)
    rows_d, s_d, r_d = (torch.from_numpy(a).cuda() for a in (rows, s, r))
    shapes = [(split, 0) for split in (1, 2, 3, 4, 6, 9, 13, 19, 28, 64)]
    shapes += [(split, w) for w in (8, 16) for split in (1, 4, 19, 64)]
    for split, waves in shapes:
        entry = [split, split] if waves == 0 else [split, split, 0, 0, waves, waves]
        json.dump({key: entry}, open(cache, "w"))
        plan = bd.Plan(geom)
        assert plan.autotune(B, str(cache)) == (split, split)
        (fs, fw), (as_, aw) = plan.spgm_plan_launch_shape(B)
        assert (fs, as_) == (split, split)
        if waves:
            # 16 waves only where the brick tables fit the 16-wave LDS layout; else 8
            assert fw == aw and fw in (8, waves)
        y = plan.forward(rows_d, s_d).cpu().numpy()
        g = plan.adjoint(rows_d, r_d).cpu().numpy()
        ey, eg = rel_l2(y[js], y_ref), rel_l2(g[vs], g_ref)
        print("[split %d, waves %d] forward %.3e adjoint %.3e" % (split, fw, ey, eg), flush=True)
        assert ey <= 1e-5 and eg <= 1e-5
        assert plan.status() == 0
        plan.close()


def cdev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex64))).cuda()


def idev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.int32))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def col_rel(got, ref):
    """Largest relative L2 error over the columns."""
    return max(rel_l2(got[:, k], ref[:, k]) for k in range(ref.shape[1]))


@pytest.mark.parametrize("name,B", [("c0", 1000), ("c1", 4096)])
def test_batched_every_candidate(bd, name, B, tmp_path):
    """Every launch shape the batched autotuner may choose, forced through the cache file: the
    shape query reports it, and the batched forward and adjoint (bfloat16, K = 32) stay within the
    batched path's relative error bound of 6e-3 per column on sampled rows and voxels against the
    oracle.  The timed run picks one of the candidates and a second plan reads it back."""
    geom = W.config_geometry(name)
    orc = Oracle(geom)
    rng = np.random.default_rng(B + 7)
    rows = W.config_rows("c1", K=1)[0] if name == "c1" else rng.integers(0, orc.M, B).astype(np.int32)
    K = 32
    S = (W.random_complex(orc.N * K, seed=81).reshape(orc.N, K)).astype(np.complex64)
    R = (W.random_complex(B * K, seed=82).reshape(B, K)).astype(np.complex64)
    js = np.sort(rng.choice(B, 16, replace=False))
    vs = np.sort(rng.choice(orc.N, 32, replace=False))
    y_ref = np.stack([orc.forward(rows[js], S[:, k].astype(np.complex128)) for k in range(K)], axis=1)
    g_ref = np.stack([orc.adjoint_voxels(rows, R[:, k].astype(np.complex128), vs) for k in range(K)], axis=1)
    rows_d, S_d, R_d = idev(rows), cdev(S), cdev(R)
    cache = tmp_path / "tune.json"
    plan0 = bd.Plan(geom)
    fwd_c, adj_c = plan0.spgm_plan_batched_candidates(B)
    shape = plan0.spgm_plan_autotune_batched(B, 0, str(cache))
    print("[autotune-mm] %s B=%d: %d forward and %d adjoint candidates; chose %s" % (
        name, B, len(fwd_c), len(adj_c), shape), flush=True)
    assert tuple(shape[:4]) in fwd_c and tuple(shape[4:6]) in adj_c
    keys = [k for k in json.load(open(cache)) if k.endswith("|mm0")]
    assert len(keys) == 1
    assert bd.Plan(geom).spgm_plan_autotune_batched(B, 0, str(cache)) == shape
    combos = [(f, adj_c[0]) for f in fwd_c] + [(fwd_c[0], a) for a in adj_c[1:]]
    for f, a in combos:
        json.dump({keys[0]: list(f) + list(a)}, open(cache, "w"))
        plan = bd.Plan(geom)
        got = plan.spgm_plan_autotune_batched(B, 0, str(cache))
        assert got[:6] == tuple(f) + tuple(a), (got, f, a)
        Y = host(plan.spgm_forward_batched(rows_d, S_d))
        G = host(plan.spgm_adjoint_batched(rows_d, R_d))
        ey, eg = col_rel(Y[js], y_ref), col_rel(G[vs], g_ref)
        print("[autotune-mm] %s forward %s adjoint %s: %.2e %.2e" % (name, f, a, ey, eg), flush=True)
        assert ey <= 6e-3 and eg <= 6e-3
        assert plan.status() == 0
        plan.close()


@pytest.mark.parametrize("nf,nt,nr", [(16, 16, 16), (8, 20, 8)])
def test_structured_every_candidate(bd, nf, nt, nr, tmp_path):
    """Structured kernels with each instance the autotuner may choose (8 items per thread only
    where nt + nr <= 32 and nt <= 16), forced through the cache: parity with the oracle on the c1
    geometry (rel-L2 <= 1e-5 on sampled rows and voxels); a forced small instance that the subset
    does not allow falls back to the general one."""
    geom = W.config_geometry("c1")
    orc = Oracle(geom)
    T, R, F = geom["tx"].shape[0], geom["rx"].shape[0], len(geom["freq"])
    fss, tss, rss = W.draw_structured_subsets(T, R, F, nf, nt, nr, 1, seed=91)
    fs, ts, rs = fss[0], tss[0], rss[0]
    rows = W.structured_rows(T, R, fs, ts, rs)
    s = W.random_complex(orc.N, seed=92).astype(np.complex64)
    r = W.random_complex(rows.size, seed=93).astype(np.complex64)
    rng = np.random.default_rng(94)
    js = np.sort(rng.choice(rows.size, 16, replace=False))
    vs = np.sort(rng.choice(orc.N, 32, replace=False))
    y_ref = orc.forward(rows[js], s.astype(np.complex128))
    g_ref = orc.adjoint_voxels(rows, r.astype(np.complex128), vs)
    cache = tmp_path / "tune.json"
    items = bd.Plan(geom).spgm_plan_autotune_structured(nf, nt, nr, str(cache))
    small_ok = nt + nr <= 32 and nt <= 16
    assert items in ((8, 16) if small_ok else (16,))
    key = [k for k in json.load(open(cache)) if "|sf|" in k][0]
    for forced in (8, 16):
        json.dump({key: [forced]}, open(cache, "w"))
        plan = bd.Plan(geom)
        got = plan.spgm_plan_autotune_structured(nf, nt, nr, str(cache))
        assert got == (forced if small_ok else 16)
        assert plan.spgm_plan_structured_shape(nf, nt, nr) == got
        y = host(plan.spgm_forward_structured(idev(fs), idev(ts), idev(rs), cdev(s)))
        g = host(plan.spgm_adjoint_structured(idev(fs), idev(ts), idev(rs), cdev(r)))
        ey, eg = rel_l2(y[js], y_ref), rel_l2(g[vs], g_ref)
        print("[autotune-sf] (%d, %d, %d) items %d: %.2e %.2e" % (nf, nt, nr, got, ey, eg), flush=True)
        assert ey <= 1e-5 and eg <= 1e-5
        assert plan.status() == 0
        plan.close()


RAGGED = [  # T, R, F, grid
    (6, 9, 8, (32, 32, 16)),
    (12, 12, 40, (16, 16, 8)),
    (20, 5, 6, (24, 8, 12)),
]


def test_ragged_batch_every_candidate(bd, tmp_path):
    """Ragged batch with each rows-per-work-item value the autotuner may choose, forced through
    the cache: one SPGM iteration with a non-zero threshold matches the oracle for every scene
    (rel-L2 <= 1e-5)."""
    geoms, ys, rows, s0 = [], [], [], []
    for i, (T, R, F, grid) in enumerate(RAGGED):
        geom = W.make_geometry(T, R, F, (20e9, 30e9), grid, 4e-3, 0.24, 0.2, seed=800 + i)
        M, N = W.dims(geom)
        geoms.append(geom)
        ys.append(W.random_complex(M, seed=810 + i).astype(np.complex64))
        rows.append(W.draw_rows(M, int(np.ceil(M / 2)), 1, seed=820 + i))
        s0.append((0.1 * W.random_complex(N, seed=830 + i)).astype(np.complex64))
    Bs = [r.shape[1] for r in rows]
    etas = [2e-3] * len(geoms)
    alphas, refs = [], []
    for i, geom in enumerate(geoms):
        orc = Oracle(geom)
        s64 = s0[i].astype(np.complex128)
        v = s64 - etas[i] * orc.gradient(rows[i][0], ys[i].astype(np.complex128), s64)
        alphas.append(float(np.float32(np.median(np.abs(v)))))
        refs.append(orc.solve(rows[i], ys[i].astype(np.complex128), s64, etas[i], alphas[i]))
    cache = tmp_path / "tune.json"
    chosen = bd.Batch(geoms).autotune(Bs, str(cache))
    assert chosen in (256, 512, 1024, 2048, 4096, 8192, 16384)
    key = [k for k in json.load(open(cache)) if "|batch|" in k][0]
    for rps in (256, 512, 1024, 2048, 4096, 8192, 16384):
        json.dump({key: [rps]}, open(cache, "w"))
        batch = bd.Batch(geoms)
        assert batch.autotune(Bs, str(cache)) == rps
        ss = [torch.from_numpy(v.copy()).cuda() for v in s0]
        batch.solve([torch.from_numpy(r).cuda() for r in rows], [torch.from_numpy(v).cuda() for v in ys], ss, etas,
                    alphas)
        assert batch.status() == 0
        for i in range(len(geoms)):
            err = rel_l2(host(ss[i]), refs[i])
            print("[autotune-batch] rows per item %d scene %d: rel_l2 %.2e" % (rps, i, err), flush=True)
            assert err <= 1e-5
        batch.close()


def test_plan_options_device_and_cache(bd, tmp_path):
    """A plan made with spgm_plan_create_ex on device 0 with a cache file: its autotuners write
    to that file when given no path."""
    geom = W.config_geometry("c0")
    cache = tmp_path / "plan_cache.json"
    plan = bd.Plan(geom, device=0, tune_cache=str(cache))
    fs, as_ = plan.autotune(256)
    shape = plan.spgm_plan_autotune_batched(256)
    keys = list(json.load(open(cache)).keys())
    assert len(keys) == 2 and any(k.endswith("|mm0") for k in keys)
    assert plan.spgm_plan_launch_shape(256)[0][0] == fs and plan.spgm_plan_batched_shape(256) == shape
    plan.close()
