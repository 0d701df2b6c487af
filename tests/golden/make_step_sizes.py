"""Write ``step_sizes.json``: the Lipschitz estimate L of the minibatch gradient per workload.

For each workload, L = max over a few seeded minibatches of the largest eigenvalue of
A_B^H A_B / B, by power iteration with the FP64 oracle.  The solver uses eta = 1/L (Sec. IV:
a proximal-gradient step size at most the inverse Lipschitz constant of the data-fidelity
gradient) and lambda = 0.05 * max|A^H y| / M.  The synthetic measurements y come from the
oracle as well (forward projection of the seeded scene plus seeded noise).

The largest workload (c2: B = 16384 rows of N = 1 048 576 voxels) is too large for FP64 power
iterations on the host (each costs 3.4e10 entry evaluations), so its L is the top edge of the
Marchenko-Pastur law for a B x N matrix of independent entries of variance sigma^2,
sigma^2 (1 + sqrt(N/B))^2, with sigma^2 the mean |A_mn|^2 of oracle rows, scaled by the ratio
of the power-iteration L to that edge on the mid-size workload c1 (neighbouring voxels give
correlated columns, which raise the top eigenvalue above the independent-entry edge) and by a
margin of 1.5.  Its lambda_max is taken over a seeded 1 % voxel sample of A^H y.  The 96 scenes
of the ragged batch (c3) take the same two estimates scene by scene.

Calls only the oracle and the seeded input generators.  Usage:
    python tests/golden/make_step_sizes.py [workload ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import Oracle  # noqa: E402
from paper_2509_00774_amd import workloads as W  # noqa: E402

# workload -> (minibatches, power iterations)
PLAN = {"c0": (8, 100), "c4": (4, 40), "c1": (1, 10)}
OUT = os.path.join(HERE, "step_sizes.json")


def measurements(name, orc):
    s, idx = W.config_scene(name)
    cfg = W.CONFIGS[name]
    y0 = orc.forward_sparse(np.arange(orc.M), idx, s[idx])
    return W.add_noise(y0, cfg["snr_db"], seed=cfg["seed"] + 2)


def entry_power(orc, n_rows=8, seed=0):
    """Mean |A_mn|^2 over all voxels of a few seeded rows."""
    rows = np.random.default_rng(seed).choice(orc.M, size=n_rows, replace=False)
    return float(np.mean(np.abs(orc.dense(rows)) ** 2))


def mp_edge(orc, B):
    """sigma^2 (1 + sqrt(N/B))^2: top eigenvalue of A_B^H A_B / B for independent entries."""
    return entry_power(orc) * (1.0 + np.sqrt(orc.N / B)) ** 2


def large_case(name, data, t0):
    cfg = W.CONFIGS[name]
    orc = Oracle(W.config_geometry(name))
    ref = W.CONFIGS["c1"]
    ratio = data["c1"]["L"] / mp_edge(Oracle(W.config_geometry("c1")), ref["B"])
    L = 1.5 * ratio * mp_edge(orc, cfg["B"])
    y = measurements(name, orc)
    vox = W.voxel_sample(orc.N, 0.01, seed=cfg["seed"] + 9)
    lam_max = float(np.max(np.abs(orc.adjoint_voxels(np.arange(orc.M), y, vox))) / orc.M)
    data[name] = {"L": L, "L_mp_ratio_c1": ratio, "lambda_max": lam_max, "eta": 1.0 / L, "lambda": 0.05 * lam_max,
                  "note": "L = 1.5 x (c1 power-iteration L / c1 independent-entry edge) x sigma^2 (1 + sqrt(N/B))^2; "
                          "lambda_max = max|A^H y|/M over a seeded 1% voxel sample, y from the oracle"}
    print(name, data[name], "%.1fs" % (time.time() - t0), flush=True)


def ragged_case(name, data, t0):
    """Per scene of the ragged batch: eta from the scaled independent-entry edge (as for c2) and
    lambda = 0.05 lambda_max over a seeded 1 % voxel sample, y from the oracle."""
    ratio = data["c1"]["L"] / mp_edge(Oracle(W.config_geometry("c1")), W.CONFIGS["c1"]["B"])
    out = []
    for i, sc in enumerate(W.ragged_scenes()):
        orc = Oracle(sc["geom"])
        st, idx = W.random_scene(sc["N"], sc["density"], seed=sc["seed"] + 1)
        y = W.add_noise(orc.forward_sparse(np.arange(orc.M), idx, st[idx]), sc["snr_db"], seed=sc["seed"] + 2)
        vox = W.voxel_sample(orc.N, 0.01, seed=sc["seed"] + 9)
        lam_max = float(np.max(np.abs(orc.adjoint_voxels(np.arange(orc.M), y, vox))) / orc.M)
        L = 1.5 * ratio * mp_edge(orc, sc["B"])
        out.append({"eta": 1.0 / L, "lambda": 0.05 * lam_max, "lambda_max": lam_max, "L": L})
    data[name] = {"scenes": out, "L_mp_ratio_c1": ratio,
                  "note": "per scene: L = 1.5 x (c1 power-iteration L / c1 independent-entry edge) x "
                          "sigma^2 (1 + sqrt(N/B))^2; lambda_max = max|A^H y|/M over a seeded 1% voxel sample"}
    print(name, len(out), "scenes", "%.1fs" % (time.time() - t0), flush=True)


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t0 = time.time()
        if name in ("c2", "c3"):
            (large_case if name == "c2" else ragged_case)(name, data, t0)
            json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
            continue
        cfg = W.CONFIGS[name]
        orc = Oracle(W.config_geometry(name))
        nb, iters = PLAN[name]
        rows = W.draw_rows(orc.M, cfg["B"], nb, seed=cfg["seed"] + 5)
        Ls = [orc.lipschitz(rows[k], iters=iters, seed=k) for k in range(nb)]
        y = measurements(name, orc)
        lam_max = orc.lambda_max(y)
        data[name] = {"L": max(Ls), "L_per_batch": Ls, "power_iters": iters, "lambda_max": lam_max,
                      "eta": 1.0 / max(Ls), "lambda": 0.05 * lam_max,
                      "note": "L = max over seeded minibatches of lambda_max(A_B^H A_B)/B (FP64 power "
                              "iteration); lambda_max = max|A^H y|/M with y from the oracle"}
        print(name, data[name], "%.1fs" % (time.time() - t0), flush=True)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c0", "c4", "c1"])
