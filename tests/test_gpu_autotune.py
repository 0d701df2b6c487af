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
