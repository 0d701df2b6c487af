"""CPU FP64 oracle for the SPGM near-field MIMO projector (arXiv 2509.00774).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with the
HIP path: the arithmetic lives in ``spgm_oracle.c`` (plain double precision, OpenMP
over independent rows or voxels) and this module only marshals numpy arrays.

Functions and the passage each one follows:

* :meth:`Oracle.entry`, :meth:`Oracle.dense`            -- observation-matrix entry (Sec. II, Eq. 2)
* :meth:`Oracle.forward`, :meth:`Oracle.forward_sparse`  -- y_B = A_B s (Sec. II, Eq. 1)
* :meth:`Oracle.adjoint`, :meth:`Oracle.adjoint_voxels`  -- A_B^H r (conjugate transpose of Eq. 1)
* :func:`prox_l1`                                        -- prox of alpha*||.||_1 used in Eq. 5
* :meth:`Oracle.gradient`                                -- minibatch gradient (Sec. IV-A, Eq. 6)
* :meth:`Oracle.step`, :meth:`Oracle.solve`              -- SPGM / PGM iteration (Sec. IV, Eq. 5)
* :meth:`Oracle.solve_tol`                               -- the same until the termination rule of Sec. V
* :meth:`Oracle.lambda_max`                              -- smallest lambda with zero minimiser of Eq. 3 with Eq. 4
* :meth:`Oracle.lipschitz`                               -- power iteration on A_B^H A_B / B (step-size choice)
* :func:`prox_elastic`, :func:`prox_tv_magnitude`,
  :func:`grad3`, :func:`grad3_adjoint`, :meth:`Oracle.step_reg` -- other regularisers in place of the l1 prox
                                                            (Sec. III notes the extension; readings in spgm_oracle.c)
* :func:`nmse`, :func:`psnr_magnitude`                   -- error metrics (Sec. V, PSNR over normalised magnitudes)
* :func:`unrolled_forward`, :func:`unrolled_vjp`         -- K iterations of Eq. 5 with per-iteration step size
                                                            and threshold, and their chain-rule gradient
* :func:`splitmix64`, :func:`rows_generate`,
  :func:`subsets_generate`                               -- the seeded minibatch draw of each SPGM iteration
                                                            (Sec. IV: rows drawn uniformly at random), written
                                                            from the generator's published definition
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import ensure_oracle

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class _Geometry(C.Structure):
    _fields_ = [
        ("n_tx", C.c_int32), ("n_rx", C.c_int32), ("n_freq", C.c_int32),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("tx_xyz", _dp), ("rx_xyz", _dp), ("freq_hz", _dp), ("pulse", _dp),
        ("centre", C.c_double * 3), ("pitch", C.c_double * 3), ("c", C.c_double),
    ]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        lib = C.CDLL(ensure_oracle())
        g = C.POINTER(_Geometry)
        sig = {
            "ora_num_threads": (C.c_int, []),
            "ora_num_rows": (C.c_int64, [g]),
            "ora_num_voxels": (C.c_int64, [g]),
            "ora_voxel_position": (None, [g, C.c_int64, _dp]),
            "ora_entry": (None, [g, C.c_int64, C.c_int64, _dp]),
            "ora_dense": (None, [g, _ip, C.c_int32, _dp]),
            "ora_forward": (None, [g, _ip, C.c_int32, _dp, _dp]),
            "ora_forward_sparse": (None, [g, _ip, C.c_int32, _lp, _dp, C.c_int64, _dp]),
            "ora_adjoint": (None, [g, _ip, C.c_int32, _dp, _dp]),
            "ora_adjoint_voxels": (None, [g, _ip, C.c_int32, _dp, _lp, C.c_int64, _dp]),
            "ora_prox_l1": (None, [_dp, C.c_int64, C.c_double]),
            "ora_stochastic_gradient": (None, [g, _ip, C.c_int32, _dp, _dp, _dp]),
            "ora_step": (None, [g, _ip, C.c_int32, _dp, _dp, C.c_double, C.c_double]),
            "ora_solve": (None, [g, _ip, C.c_int32, C.c_int32, _dp, _dp, C.c_double, C.c_double]),
            "ora_solve_tol": (C.c_int32, [g, _ip, C.c_int32, C.c_int32, _dp, _dp, C.c_double, C.c_double,
                                          C.c_double]),
            "ora_grad3": (None, [C.c_int32, C.c_int32, C.c_int32, _dp, _dp]),
            "ora_grad3_adjoint": (None, [C.c_int32, C.c_int32, C.c_int32, _dp, _dp]),
            "ora_prox_elastic": (None, [_dp, C.c_int64, C.c_double, C.c_double]),
            "ora_prox_tv_magnitude": (None, [_dp, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_int32, _dp]),
            "ora_step_reg": (None, [g, _ip, C.c_int32, _dp, _dp, C.c_double, C.c_double, C.c_int32,
                                    C.c_double, C.c_int32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def num_threads() -> int:
    """OpenMP threads the oracle uses (``OMP_NUM_THREADS`` or the host's core count)."""
    return int(_lib().ora_num_threads())


def _c128(a) -> np.ndarray:
    """Complex array -> contiguous complex128 (interleaved re, im doubles)."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


class Oracle:
    """FP64 reference for one imaging geometry.

    ``geom`` is a mapping with keys ``tx`` (T x 3), ``rx`` (R x 3), ``freq`` (F,),
    ``pulse`` (F complex, or None for p = 1), ``grid`` (nx, ny, nz), ``centre`` (3,),
    ``pitch`` (3,) and ``c`` -- the same fields the C-ABI plan takes.
    """

    def __init__(self, geom):
        self._keep = []
        tx = _f64(geom["tx"]).reshape(-1, 3)
        rx = _f64(geom["rx"]).reshape(-1, 3)
        fr = _f64(geom["freq"]).reshape(-1)
        pulse = geom.get("pulse")
        pl = None if pulse is None else _f64(np.stack([np.real(pulse), np.imag(pulse)], -1).reshape(-1))
        self._keep += [tx, rx, fr, pl]
        nx, ny, nz = (int(v) for v in geom["grid"])
        g = _Geometry()
        g.n_tx, g.n_rx, g.n_freq = tx.shape[0], rx.shape[0], fr.shape[0]
        g.nx, g.ny, g.nz = nx, ny, nz
        g.tx_xyz, g.rx_xyz, g.freq_hz = _ptr(tx), _ptr(rx), _ptr(fr)
        g.pulse = _ptr(pl) if pl is not None else _dp()
        g.centre = (C.c_double * 3)(*[float(v) for v in geom["centre"]])
        g.pitch = (C.c_double * 3)(*[float(v) for v in geom["pitch"]])
        g.c = float(geom["c"])
        self._g = g
        self.T, self.R, self.F = g.n_tx, g.n_rx, g.n_freq
        self.M = int(_lib().ora_num_rows(C.byref(g)))
        self.N = int(_lib().ora_num_voxels(C.byref(g)))

    # --- Sec. II ---------------------------------------------------------------
    def voxel_position(self, n: int) -> np.ndarray:
        out = np.zeros(3)
        _lib().ora_voxel_position(C.byref(self._g), int(n), _ptr(out))
        return out

    def entry(self, m: int, n: int) -> complex:
        out = np.zeros(2)
        _lib().ora_entry(C.byref(self._g), int(m), int(n), _ptr(out))
        return complex(out[0], out[1])

    def dense(self, rows=None) -> np.ndarray:
        rows = np.arange(self.M) if rows is None else rows
        rows = _i32(rows)
        A = np.zeros((rows.size, self.N), dtype=np.complex128)
        _lib().ora_dense(C.byref(self._g), _ptr(rows, _ip), rows.size, _ptr(A))
        return A

    def forward(self, rows, s) -> np.ndarray:
        rows, s = _i32(rows), _c128(s).reshape(-1)
        assert s.size == self.N
        y = np.zeros(rows.size, dtype=np.complex128)
        _lib().ora_forward(C.byref(self._g), _ptr(rows, _ip), rows.size, _ptr(s), _ptr(y))
        return y

    def forward_sparse(self, rows, idx, vals) -> np.ndarray:
        rows = _i32(rows)
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        vals = _c128(vals).reshape(-1)
        y = np.zeros(rows.size, dtype=np.complex128)
        _lib().ora_forward_sparse(C.byref(self._g), _ptr(rows, _ip), rows.size, _ptr(idx, _lp),
                                  _ptr(vals), idx.size, _ptr(y))
        return y

    def adjoint(self, rows, r) -> np.ndarray:
        rows, r = _i32(rows), _c128(r).reshape(-1)
        assert r.size == rows.size
        g = np.zeros(self.N, dtype=np.complex128)
        _lib().ora_adjoint(C.byref(self._g), _ptr(rows, _ip), rows.size, _ptr(r), _ptr(g))
        return g

    def adjoint_voxels(self, rows, r, idx) -> np.ndarray:
        """(A_B^H r) at the listed voxel indices only."""
        rows, r = _i32(rows), _c128(r).reshape(-1)
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        out = np.zeros(idx.size, dtype=np.complex128)
        _lib().ora_adjoint_voxels(C.byref(self._g), _ptr(rows, _ip), rows.size, _ptr(r), _ptr(idx, _lp),
                                  idx.size, _ptr(out))
        return out

    # --- Sec. IV ---------------------------------------------------------------
    def gradient(self, rows, y, s) -> np.ndarray:
        rows, y, s = _i32(rows), _c128(y).reshape(-1), _c128(s).reshape(-1)
        assert y.size == self.M and s.size == self.N
        out = np.zeros(self.N, dtype=np.complex128)
        _lib().ora_stochastic_gradient(C.byref(self._g), _ptr(rows, _ip), rows.size, _ptr(y), _ptr(s), _ptr(out))
        return out

    def step(self, rows, y, s, eta: float, alpha: float) -> np.ndarray:
        rows, y = _i32(rows), _c128(y).reshape(-1)
        s = _c128(s).reshape(-1).copy()
        assert y.size == self.M and s.size == self.N
        _lib().ora_step(C.byref(self._g), _ptr(rows, _ip), rows.size, _ptr(y), _ptr(s), float(eta), float(alpha))
        return s

    def step_reg(self, rows, y, s, eta: float, alpha: float, kind: int, mu: float = 0.0,
                 tv_iters: int = 0) -> np.ndarray:
        """Eq. 5 with the prox of another regulariser: kind 0 = l1, 1 = elastic net, 2 = magnitude TV."""
        rows, y = _i32(rows), _c128(y).reshape(-1)
        s = _c128(s).reshape(-1).copy()
        assert y.size == self.M and s.size == self.N
        _lib().ora_step_reg(C.byref(self._g), _ptr(rows, _ip), rows.size, _ptr(y), _ptr(s), float(eta),
                            float(alpha), int(kind), float(mu), int(tv_iters))
        return s

    def solve(self, rows_table, y, s0, eta: float, alpha: float) -> np.ndarray:
        """K iterations; ``rows_table`` is K x B (iteration k uses row k)."""
        rows = _i32(rows_table)
        K, B = rows.shape
        y = _c128(y).reshape(-1)
        s = _c128(s0).reshape(-1).copy()
        _lib().ora_solve(C.byref(self._g), _ptr(rows, _ip), K, B, _ptr(y), _ptr(s), float(eta), float(alpha))
        return s

    def solve_tol(self, rows_table, y, s0, eta: float, alpha: float, tol: float):
        """Iterations of Eq. 5 until the termination rule of Sec. V (relative 2-norm change of the
        magnitudes below ``tol``), at most K = len(rows_table).  Returns (s, iterations)."""
        rows = _i32(rows_table)
        K, B = rows.shape
        y = _c128(y).reshape(-1)
        s = _c128(s0).reshape(-1).copy()
        done = _lib().ora_solve_tol(C.byref(self._g), _ptr(rows, _ip), K, B, _ptr(y), _ptr(s), float(eta),
                                    float(alpha), float(tol))
        return s, int(done)

    def lambda_max(self, y) -> float:
        """max_n |(A^H y)_n| / M: for lambda at or above it, s = 0 minimises Eq. 3 with Eq. 4."""
        g = self.adjoint(np.arange(self.M), y)
        return float(np.max(np.abs(g)) / self.M)

    def lipschitz(self, rows, iters: int = 100, seed: int = 0) -> float:
        """Largest eigenvalue of A_B^H A_B / B by power iteration (FP64)."""
        rng = np.random.default_rng(seed)
        rows = _i32(rows)
        v = rng.standard_normal(self.N) + 1j * rng.standard_normal(self.N)
        v /= np.linalg.norm(v)
        lam = 0.0
        for _ in range(iters):
            w = self.adjoint(rows, self.forward(rows, v)) / rows.size
            lam = float(np.real(np.vdot(v, w)))
            v = w / np.linalg.norm(w)
        return lam


def prox_l1(v, alpha: float) -> np.ndarray:
    """Complex soft threshold S_alpha(v) = v * max(0, 1 - alpha/|v|) (prox of alpha*||.||_1)."""
    v = _c128(v).reshape(-1).copy()
    _lib().ora_prox_l1(_ptr(v), v.size, float(alpha))
    return v


def prox_elastic(v, alpha: float, mu: float) -> np.ndarray:
    """Prox of alpha*(||.||_1 + (mu/2)||.||^2): S_alpha(v) / (1 + alpha mu)."""
    v = _c128(v).reshape(-1).copy()
    _lib().ora_prox_elastic(_ptr(v), v.size, float(alpha), float(mu))
    return v


def grad3(u, grid) -> np.ndarray:
    """Forward differences of a real (nz, ny, nx) volume, shape (3, N); zero on each upper face."""
    nx, ny, nz = (int(v) for v in grid)
    u = _f64(u).reshape(-1)
    assert u.size == nx * ny * nz
    w = np.zeros(3 * u.size)
    _lib().ora_grad3(nx, ny, nz, _ptr(u), _ptr(w))
    return w.reshape(3, -1)


def grad3_adjoint(w, grid) -> np.ndarray:
    """Adjoint of :func:`grad3` (minus the divergence), shape (N,)."""
    nx, ny, nz = (int(v) for v in grid)
    w = _f64(w).reshape(-1)
    assert w.size == 3 * nx * ny * nz
    out = np.zeros(nx * ny * nz)
    _lib().ora_grad3_adjoint(nx, ny, nz, _ptr(w), _ptr(out))
    return out


def prox_tv_magnitude(v, grid, alpha: float, iters: int, return_dual: bool = False):
    """Prox of alpha*TV(|.|) with the phase kept; ``iters`` dual fast-gradient-projection iterations.

    With ``return_dual`` also returns the final dual field w, shape (3, N)."""
    nx, ny, nz = (int(x) for x in grid)
    v = _c128(v).reshape(-1).copy()
    assert v.size == nx * ny * nz
    w = np.zeros(3 * v.size)
    _lib().ora_prox_tv_magnitude(_ptr(v), nx, ny, nz, float(alpha), int(iters), _ptr(w))
    return (v, w.reshape(3, -1)) if return_dual else v


def nmse(x, ref) -> float:
    """|x - ref|^2 / |ref|^2."""
    x, ref = np.asarray(x), np.asarray(ref)
    return float(np.sum(np.abs(x - ref) ** 2) / np.sum(np.abs(ref) ** 2))


def rel_l2(x, ref) -> float:
    return float(np.sqrt(nmse(x, ref)))


def psnr_magnitude(x, ref) -> float:
    """PSNR over magnitudes each normalised to peak 1, with ``ref`` as the reference (Sec. V)."""
    a = np.abs(np.asarray(x)).reshape(-1)
    b = np.abs(np.asarray(ref)).reshape(-1)
    a = a / a.max() if a.max() > 0 else a
    b = b / b.max() if b.max() > 0 else b
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def library_path() -> str:
    return os.path.abspath(ensure_oracle())


# ---------------------------------------------------------------------------------------------
# Unrolled SPGM with per-iteration step size eta_k and threshold tau_k (Eq. 5 with Eq. 6):
#     z_k = s_k - (eta_k/B) A_k^H (A_k s_k - y_k),   s_{k+1} = S_{tau_k}(z_k).
# Gradients of a real loss use the convention dL/dRe + j dL/dIm for complex quantities.
# ---------------------------------------------------------------------------------------------
def unrolled_forward(orc, rows_table, y, s0, eta, tau):
    """All iterates [s_0, ..., s_K] in FP64."""
    rows_table = np.asarray(rows_table)
    y = _c128(y).reshape(-1)
    s = _c128(s0).reshape(-1).copy()
    out = [s.copy()]
    for k in range(rows_table.shape[0]):
        rows = rows_table[k]
        g = orc.adjoint(rows, orc.forward(rows, s) - y[rows])
        z = s - (float(eta[k]) / rows.size) * g
        s = prox_l1(z, float(tau[k]))
        out.append(s.copy())
    return out


def unrolled_vjp(orc, rows_table, y, iterates, eta, tau, sbar):
    """Chain rule through the unrolled iterations, last to first.

    Prox: where |z| > tau with u = z/|z|, zbar = (1 - tau/|z|) sbar + (tau/|z|) u Re(conj(u) sbar)
    and dL/dtau = -sum Re(conj(u) sbar); where |z| <= tau the output is 0 and zbar = 0.
    Linear step: sbar_k = zbar - (eta/B) A^H A zbar and dL/deta = -(1/B) Re <zbar, A^H (A s - y)>.
    Returns (dL/ds_0, dL/deta, dL/dtau)."""
    rows_table = np.asarray(rows_table)
    y = _c128(y).reshape(-1)
    K = rows_table.shape[0]
    sbar = _c128(sbar).reshape(-1).copy()
    eta_bar = np.zeros(K)
    tau_bar = np.zeros(K)
    for k in range(K - 1, -1, -1):
        rows = rows_table[k]
        B = rows.size
        s = iterates[k]
        g = orc.adjoint(rows, orc.forward(rows, s) - y[rows])
        z = s - (float(eta[k]) / B) * g
        r = np.abs(z)
        on = r > float(tau[k])
        u = np.zeros_like(z)
        u[on] = z[on] / r[on]
        re = np.real(np.conj(u) * sbar)
        c = np.zeros_like(r)
        c[on] = float(tau[k]) / r[on]
        zbar = np.where(on, (1.0 - c) * sbar + c * u * re, 0.0)
        tau_bar[k] = -np.sum(re[on])
        eta_bar[k] = -np.real(np.vdot(zbar, g)) / B
        sbar = zbar - (float(eta[k]) / B) * orc.adjoint(rows, orc.forward(rows, zbar))
    return sbar, eta_bar, tau_bar


# ------------------------------------------------------------------------------------------
# Seeded minibatches (Sec. IV: every SPGM iteration draws its rows uniformly at random).
# SplitMix64 as published by Steele, Lea and Flood (OOPSLA 2014); iteration k of a solve uses
# outputs k * 2**32 + 1, k * 2**32 + 2, ... of the sequence seeded with `seed`; a partial
# Fisher-Yates shuffle of 0 .. n-1 maps the draws to m distinct indices (draw j swaps position j
# with position j + floor(hi32(u) * (n - j) / 2**32)).  Plain Python integers, small cases only.
# ------------------------------------------------------------------------------------------
_MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(state: int):
    """Generator of SplitMix64 outputs from the initial state `state` (one per next())."""
    while True:
        state = (state + _GAMMA) & _MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        yield z ^ (z >> 31)


def _iteration_stream(seed: int, k: int):
    """Outputs k * 2**32 + 1, ... of the sequence seeded with `seed`: skip k * 2**32 increments."""
    return splitmix64((seed + k * (1 << 32) * _GAMMA) & _MASK64)


def _partial_shuffle(gen, n: int, m: int) -> list:
    """m distinct indices of 0 .. n-1: the first m positions of a partial Fisher-Yates shuffle."""
    moved = {}  # positions that no longer hold their own index
    out = []
    for j in range(m):
        u = next(gen)
        r = j + (((u >> 32) * (n - j)) >> 32)
        vj, vr = moved.get(j, j), moved.get(r, r)
        moved[j], moved[r] = vr, vj
        out.append(moved[j])
    return out


def rows_generate(seed: int, start_iter: int, iters: int, M: int, B: int) -> np.ndarray:
    """(iters, B) int32 table: the rows of iterations start_iter .. start_iter + iters - 1."""
    if not 1 <= B <= M:
        raise ValueError("need 1 <= B <= M")
    return np.array([_partial_shuffle(_iteration_stream(seed, start_iter + i), M, B) for i in range(iters)],
                    dtype=np.int32).reshape(iters, B)


def subsets_generate(seed: int, start_iter: int, iters: int, F: int, T: int, R: int, nf: int, nt: int, nr: int):
    """Per iteration: nf of F frequencies, then nt of T transmitters, then nr of R receivers from
    the iteration's stream; three int32 tables (iters, nf), (iters, nt), (iters, nr)."""
    fs, ts, rs = [], [], []
    for i in range(iters):
        gen = _iteration_stream(seed, start_iter + i)
        fs.append(_partial_shuffle(gen, F, nf))
        ts.append(_partial_shuffle(gen, T, nt))
        rs.append(_partial_shuffle(gen, R, nr))
    return (np.array(fs, dtype=np.int32).reshape(iters, nf), np.array(ts, dtype=np.int32).reshape(iters, nt),
            np.array(rs, dtype=np.int32).reshape(iters, nr))
