"""Seeded synthetic inputs for the SPGM projector, shared by the tests, the benchmark and the
reference checks.

This module only draws random numbers and lays out arrays: array geometry, frequency grid,
pulse spectrum, voxel grid, sparse random-phase scenes, measurement noise at a stated SNR and
minibatch row tables.  It holds none of the method's arithmetic (no observation-matrix entry,
no projection, no proximal step), so the HIP path and the CPU reference can both consume it
without sharing code.

Workload recipe (shapes follow the paper's setting of a planar MIMO array facing a 3-D voxel
cube, Sec. II and Sec. V):

* Tx and Rx antennas at independent uniform-random (x, y) on the z = 0 plane inside a square
  aperture centred on the origin (the paper's spiral array coordinates are not published in
  the text, so a random planar layout stands in for it);
* frequencies equally spaced over a band, end points included;
* a regular voxel grid of a given pitch centred at (0, 0, z0), index n = (iz*ny + iy)*nx + ix;
* scenes with a given fraction of non-zero voxels, magnitudes uniform in [0.5, 1] and
  phases uniform in [0, 2 pi) (random-phase reflectivity, Sec. III);
* additive circular complex Gaussian noise with variance mean|y0|^2 * 10^(-SNR/10);
* minibatches of B distinct rows drawn uniformly without replacement, fresh for every
  iteration (Sec. IV-A); the structured form draws #f frequencies, #Tx transmitters and #Rx
  receivers and takes every combination (Sec. IV-A, minibatch size B = #f * #Tx * #Rx).
"""
from __future__ import annotations

import numpy as np

C0 = 3.0e8  # propagation speed used by every workload (m/s)

# name -> shape parameters.  "B" is the minibatch size, "K" the iteration count.
CONFIGS = {
    # 8 Tx + 8 Rx in 0.2 m, 16 f in 20-30 GHz, 16x16x8 voxels at 5 mm, z0 = 0.25 m.
    "c0": dict(T=8, R=8, aperture=0.2, F=16, band=(20e9, 30e9), pulse=None,
               grid=(16, 16, 8), pitch=5e-3, z0=0.25, density=0.05, snr_db=30.0,
               B=256, K=200, seed=1000),
    # 32 Tx + 32 Rx in 0.3 m, 64 f in 20-40 GHz with a Gaussian pulse spectrum,
    # 64x64x32 voxels at 3 mm, z0 = 0.3 m.
    "c1": dict(T=32, R=32, aperture=0.3, F=64, band=(20e9, 40e9), pulse="gauss",
               grid=(64, 64, 32), pitch=3e-3, z0=0.3, density=0.02, snr_db=20.0,
               B=4096, K=500, seed=1001),
    # 48 Tx + 48 Rx in 0.3 m, 100 f in 20-40 GHz, 128x128x64 voxels at 2 mm, z0 = 0.3 m,
    # 1 % points plus three 32x32 planar patches.
    "c2": dict(T=48, R=48, aperture=0.3, F=100, band=(20e9, 40e9), pulse=None,
               grid=(128, 128, 64), pitch=2e-3, z0=0.3, density=0.01, snr_db=20.0,
               B=16384, K=1, seed=1002, patches=True),
    # 16 Tx + 16 Rx in 0.2 m, 32 f in 20-30 GHz, 32x32x16 voxels at 5 mm, z0 = 0.25 m.
    "c4": dict(T=16, R=16, aperture=0.2, F=32, band=(20e9, 30e9), pulse=None,
               grid=(32, 32, 16), pitch=5e-3, z0=0.25, density=0.02, snr_db=25.0,
               B=2048, K=10, seed=1004),
    # Ragged batch: 96 scenes, per scene T, R ~ U{8..32}, F ~ U{16..64}, k ~ U{1..4} with a
    # (16k, 16k, 8k) grid at 3 mm, density ~ U[1 %, 5 %], B = ceil(M/4); see ragged_scenes().
    "c3": dict(n_scenes=96, aperture=0.3, band=(20e9, 40e9), pitch=3e-3, z0=0.3, snr_db=25.0,
               K=200, seed=1003),
    # Paper-shaped: 16 Tx + 9 Rx in 0.3 m, 11 f in 4-16 GHz, 61x61x21 voxels at 5 mm,
    # z0 = 0.5 m, structured minibatch (4, 4, 3).
    "P": dict(T=16, R=9, aperture=0.3, F=11, band=(4e9, 16e9), pulse=None,
              grid=(61, 61, 21), pitch=5e-3, z0=0.5, density=0.02, snr_db=30.0,
              B=48, K=200, seed=1005, structured=(4, 4, 3)),
}


def gaussian_pulse(freq, f0=30e9, width=8e9):
    """p(f) = exp(-((f - f0)/width)^2): the Gaussian pulse spectrum of the 20-40 GHz workload."""
    return np.exp(-((np.asarray(freq, dtype=np.float64) - f0) / width) ** 2).astype(np.complex128)


def make_geometry(T, R, F, band, grid, pitch, z0, aperture, pulse=None, seed=0, c=C0):
    """Array, band and voxel grid as the dict both the plan and the reference take."""
    rng = np.random.default_rng(seed)
    half = 0.5 * aperture
    tx = np.zeros((T, 3))
    rx = np.zeros((R, 3))
    tx[:, :2] = rng.uniform(-half, half, size=(T, 2))
    rx[:, :2] = rng.uniform(-half, half, size=(R, 2))
    freq = np.linspace(band[0], band[1], F)
    if isinstance(pulse, str) and pulse == "gauss":
        p = gaussian_pulse(freq)
    elif pulse is None:
        p = None
    else:
        p = np.asarray(pulse, dtype=np.complex128)
    pitch3 = np.full(3, float(pitch)) if np.isscalar(pitch) else np.asarray(pitch, dtype=np.float64)
    return {"tx": tx, "rx": rx, "freq": freq, "pulse": p,
            "grid": tuple(int(v) for v in grid), "centre": np.array([0.0, 0.0, float(z0)]),
            "pitch": pitch3, "c": float(c)}


def dims(geom):
    """(M, N) of a geometry dict: M = F*T*R measurements, N = nx*ny*nz voxels."""
    M = len(geom["freq"]) * geom["tx"].shape[0] * geom["rx"].shape[0]
    nx, ny, nz = geom["grid"]
    return M, nx * ny * nz


def random_scene(N, density, seed=0, mag=(0.5, 1.0)):
    """Sparse random-phase scene: round(density*N) non-zeros. Returns (s, idx)."""
    rng = np.random.default_rng(seed)
    k = max(1, int(round(density * N)))
    idx = np.sort(rng.choice(N, size=k, replace=False))
    s = np.zeros(N, dtype=np.complex128)
    s[idx] = rng.uniform(mag[0], mag[1], size=k) * np.exp(1j * rng.uniform(0.0, 2 * np.pi, size=k))
    return s, idx


def patch_scene(grid, density, seed=0, patch=32, depths=(16, 32, 48)):
    """Point scatterers plus three constant-magnitude z-plane patches (random phase, |s| = 1)."""
    nx, ny, nz = grid
    N = nx * ny * nz
    s, _ = random_scene(N, density, seed=seed)
    rng = np.random.default_rng(seed + 7)
    cube = s.reshape(nz, ny, nx)
    x0, y0 = (nx - patch) // 2, (ny - patch) // 2
    for d in depths:
        if d < nz:
            ph = rng.uniform(0.0, 2 * np.pi, size=(min(patch, ny), min(patch, nx)))
            cube[d, y0:y0 + patch, x0:x0 + patch] = np.exp(1j * ph)
    s = cube.reshape(-1)
    return s, np.flatnonzero(s)


def blocky_field(grid, n_boxes=6, noise=0.05, seed=0):
    """Complex volume whose magnitude is a sum of constant boxes plus |Gaussian| noise and whose
    phase is uniform: the piecewise-constant images total-variation priors are meant for."""
    nx, ny, nz = (int(v) for v in grid)
    rng = np.random.default_rng(seed)
    mag = np.zeros((nz, ny, nx))
    for _ in range(n_boxes):
        lo = [int(rng.integers(0, n)) for n in (nz, ny, nx)]
        hi = [int(rng.integers(l + 1, n + 1)) for l, n in zip(lo, (nz, ny, nx))]
        mag[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += rng.uniform(0.3, 1.0)
    mag = mag + noise * np.abs(rng.standard_normal(mag.shape))
    ph = rng.uniform(0.0, 2 * np.pi, size=mag.shape)
    return (mag * np.exp(1j * ph)).reshape(-1)


def add_noise(y0, snr_db, seed=0):
    """y0 + w, w circular complex Gaussian with variance mean|y0|^2 * 10^(-snr/10)."""
    rng = np.random.default_rng(seed)
    y0 = np.asarray(y0, dtype=np.complex128)
    sigma2 = float(np.mean(np.abs(y0) ** 2)) * 10.0 ** (-snr_db / 10.0)
    w = rng.standard_normal(y0.shape) + 1j * rng.standard_normal(y0.shape)
    return y0 + np.sqrt(sigma2 / 2.0) * w


def draw_rows(M, B, K, seed=0):
    """K x B table; row k holds B distinct measurement indices, uniform without replacement."""
    rng = np.random.default_rng(seed)
    out = np.empty((K, B), dtype=np.int32)
    for k in range(K):
        out[k] = rng.choice(M, size=B, replace=False)
    return out


def draw_structured_subsets(T, R, F, nf, nt, nr, K, seed=0):
    """K structured minibatches as subsets: (fs [K][nf], ts [K][nt], rs [K][nr]) int32, each drawn
    without replacement (frequencies, then transmitters, then receivers per minibatch)."""
    rng = np.random.default_rng(seed)
    fs = np.empty((K, nf), dtype=np.int32)
    ts = np.empty((K, nt), dtype=np.int32)
    rs = np.empty((K, nr), dtype=np.int32)
    for k in range(K):
        fs[k] = rng.choice(F, size=nf, replace=False)
        ts[k] = rng.choice(T, size=nt, replace=False)
        rs[k] = rng.choice(R, size=nr, replace=False)
    return fs, ts, rs


def structured_rows(T, R, fs, ts, rs):
    """Rows of the Cartesian product in minibatch order j = (i nt + a) nr + b:
    m = (fs[i] T + ts[a]) R + rs[b]."""
    fs, ts, rs = (np.asarray(x, dtype=np.int64) for x in (fs, ts, rs))
    return ((fs[:, None, None] * T + ts[None, :, None]) * R + rs[None, None, :]).reshape(-1).astype(np.int32)


def draw_structured_rows(T, R, F, nf, nt, nr, K, seed=0):
    """K x (nf*nt*nr) table of Cartesian-product minibatches: nf frequencies, nt Tx and nr Rx
    drawn without replacement; row index m = (i_f*T + i_t)*R + i_r."""
    fs, ts, rs = draw_structured_subsets(T, R, F, nf, nt, nr, K, seed=seed)
    return np.stack([structured_rows(T, R, fs[k], ts[k], rs[k]) for k in range(K)])


def voxel_sample(n, fraction, seed=0):
    """Sorted seeded sample of round(fraction * n) distinct indices in [0, n) (row or voxel
    subsamples on which the full-size results are checked)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=max(1, int(round(fraction * n))), replace=False))


def random_complex(n, seed=0, dtype=np.complex128):
    """Dense standard circular complex Gaussian vector (for projector parity inputs)."""
    rng = np.random.default_rng(seed)
    return ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2.0)).astype(dtype)


def config_geometry(name):
    cfg = CONFIGS[name]
    return make_geometry(cfg["T"], cfg["R"], cfg["F"], cfg["band"], cfg["grid"], cfg["pitch"],
                         cfg["z0"], cfg["aperture"], pulse=cfg["pulse"], seed=cfg["seed"])


def config_scene(name):
    cfg = CONFIGS[name]
    nx, ny, nz = cfg["grid"]
    if cfg.get("patches"):
        return patch_scene(cfg["grid"], cfg["density"], seed=cfg["seed"] + 1)
    return random_scene(nx * ny * nz, cfg["density"], seed=cfg["seed"] + 1)


def config_rows(name, K=None, B=None):
    cfg = CONFIGS[name]
    geom = config_geometry(name)
    M, _ = dims(geom)
    K = cfg["K"] if K is None else K
    if cfg.get("structured") and B is None:
        nf, nt, nr = cfg["structured"]
        return draw_structured_rows(cfg["T"], cfg["R"], cfg["F"], nf, nt, nr, K, seed=cfg["seed"] + 3)
    return draw_rows(M, cfg["B"] if B is None else B, K, seed=cfg["seed"] + 3)


def ragged_scenes(n=None, seed=None):
    """Scenes of the ragged batch: list of dicts with geometry, scene, minibatch size B and seed."""
    cfg = CONFIGS["c3"]
    n = cfg["n_scenes"] if n is None else n
    seed = cfg["seed"] if seed is None else seed
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        T, R = (int(v) for v in rng.integers(8, 33, size=2))
        F = int(rng.integers(16, 65))
        k = int(rng.integers(1, 5))
        density = float(rng.uniform(0.01, 0.05))
        sseed = seed * 1000 + i
        geom = make_geometry(T, R, F, cfg["band"], (16 * k, 16 * k, 8 * k), cfg["pitch"], cfg["z0"], cfg["aperture"],
                             seed=sseed)
        M, N = dims(geom)
        out.append(dict(geom=geom, density=density, snr_db=cfg["snr_db"], B=int(np.ceil(M / 4)), seed=sseed, M=M, N=N))
    return out
