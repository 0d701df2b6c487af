"""ctypes binding of ``libspgm.so`` (C ABI in ``include/spgm.h``), same names as the C calls.

Argument marshalling only: every step of the projector runs in the library's HIP kernels.
PyTorch supplies device memory (``torch.complex64`` / ``torch.int32`` CUDA tensors) and the
current HIP stream.  There is no fallback: if the library is not built, or the call fails,
an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspgm.so")

SPGM_OK = 0
SPGM_E_INVALID = 1
SPGM_E_NOMEM = 2
SPGM_E_DEVICE = 3
SPGM_E_NONFINITE = 4
SPGM_E_UNSUPPORTED = 5
SPGM_E_BADROW = 6

PHASE_COMP32 = 0
PHASE_F64 = 1
PHASE_NAIVE32 = 2

MM_BF16 = 0
MM_FP16 = 1

REG_L1 = 0
REG_ELASTIC_NET = 1
REG_TV_MAGNITUDE = 2

EXPORTED = ("spgm_plan_create", "spgm_plan_destroy", "spgm_plan_dims", "spgm_forward", "spgm_adjoint",
            "spgm_step", "spgm_solve", "spgm_plan_status", "spgm_last_error", "spgm_plan_timing",
            "spgm_plan_timing_read", "spgm_unrolled_vjp_step", "spgm_solve_graph", "spgm_plan_autotune",
            "spgm_batch_create", "spgm_batch_destroy", "spgm_batch_plan", "spgm_batch_solve", "spgm_batch_status",
            "spgm_forward_batched", "spgm_adjoint_batched", "spgm_step_batched", "spgm_solve_batched",
            "spgm_forward_structured", "spgm_adjoint_structured", "spgm_step_structured", "spgm_solve_structured",
            "spgm_prox", "spgm_step_reg", "spgm_solve_reg", "spgm_phase_window",
            "spgm_solve_tol", "spgm_batch_options", "spgm_step_noalloc", "spgm_step_grad",
            "spgm_unrolled_vjp_step_g", "spgm_plan_launch_shape", "spgm_calibrate", "spgm_plan_autotune_batched",
            "spgm_plan_batched_shape", "spgm_plan_batched_candidates", "spgm_plan_autotune_structured",
            "spgm_plan_structured_shape", "spgm_batch_autotune", "spgm_rows_generate", "spgm_subsets_generate",
            "spgm_solve_opts_init", "spgm_solve_ex", "spgm_plan_opts_init", "spgm_plan_create_ex")

_dp = C.POINTER(C.c_double)


COMP32_WINDOW_TURNS = 8.0


class SpgmGeometry(C.Structure):
    """Mirror of ``spgm_geometry``."""
    _fields_ = [
        ("n_tx", C.c_int32), ("n_rx", C.c_int32), ("n_freq", C.c_int32),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("tx_xyz", _dp), ("rx_xyz", _dp), ("freq_hz", _dp), ("pulse", _dp),
        ("centre", C.c_double * 3), ("pitch", C.c_double * 3), ("c", C.c_double),
    ]


class SpgmRegularizer(C.Structure):
    """Mirror of ``spgm_regularizer``."""
    _fields_ = [("kind", C.c_int32), ("mu", C.c_float), ("tv_iters", C.c_int32)]


class SpgmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("spgm error %d: %s" % (code, msg))
        self.code = code


_LIB = None


class SpgmPlanOpts(C.Structure):
    """spgm_plan_opts (include/spgm.h)."""
    _fields_ = [("phase_mode", C.c_int32), ("device", C.c_int32), ("tune_cache", C.c_char_p)]


class SpgmSolveOpts(C.Structure):
    """spgm_solve_opts (include/spgm.h)."""
    _fields_ = [("iters", C.c_int32), ("B", C.c_int32), ("lam", C.c_double), ("eta", C.c_double),
                ("rows_d", C.c_void_p), ("seed", C.c_uint64), ("sampling", C.c_int32), ("nf", C.c_int32),
                ("nt", C.c_int32), ("nr", C.c_int32), ("start_iter", C.c_int32), ("tol", C.c_double),
                ("check_every", C.c_int32), ("use_graph", C.c_int32), ("iters_done", C.POINTER(C.c_int32))]


def load_library(path: str = LIB_PATH):
    """Load libspgm.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError("libspgm.so is not built (%s); run __graft_entry__.build()" % path)
    lib = C.CDLL(path)
    vp, i32, f32 = C.c_void_p, C.c_int32, C.c_float
    sigs = {
        "spgm_plan_create": [C.POINTER(vp), C.POINTER(SpgmGeometry), i32],
        "spgm_plan_destroy": [vp],
        "spgm_plan_dims": [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
        "spgm_forward": [vp, vp, i32, vp, vp, vp],
        "spgm_adjoint": [vp, vp, i32, vp, vp, vp],
        "spgm_step": [vp, vp, i32, vp, vp, f32, f32, vp],
        "spgm_solve": [vp, vp, i32, i32, vp, vp, f32, f32, vp],
        "spgm_solve_graph": [vp, vp, i32, i32, vp, vp, f32, f32, vp],
        "spgm_plan_autotune": [vp, i32, C.c_char_p, C.POINTER(i32), C.POINTER(i32)],
        "spgm_batch_create": [C.POINTER(vp), C.POINTER(SpgmGeometry), i32, i32],
        "spgm_batch_destroy": [vp],
        "spgm_batch_plan": [vp, i32, C.POINTER(vp)],
        "spgm_batch_solve": [vp, i32, C.POINTER(i32), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                             C.POINTER(f32), C.POINTER(f32), i32, vp],
        "spgm_batch_status": [vp, C.POINTER(i32)],
        "spgm_plan_status": [vp, C.POINTER(i32)],
        "spgm_plan_timing": [vp, i32],
        "spgm_unrolled_vjp_step": [vp, vp, i32, vp, vp, f32, f32, vp, vp, vp, vp, vp],
        "spgm_plan_timing_read": [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                  C.POINTER(C.c_int64)],
        "spgm_forward_batched": [vp, vp, i32, i32, vp, vp, i32, vp],
        "spgm_adjoint_batched": [vp, vp, i32, i32, vp, vp, i32, vp],
        "spgm_step_batched": [vp, vp, i32, i32, vp, vp, f32, f32, i32, vp],
        "spgm_solve_batched": [vp, vp, i32, i32, i32, vp, vp, f32, f32, i32, vp],
        "spgm_forward_structured": [vp, vp, i32, vp, i32, vp, i32, vp, vp, vp],
        "spgm_adjoint_structured": [vp, vp, i32, vp, i32, vp, i32, vp, vp, vp],
        "spgm_step_structured": [vp, vp, i32, vp, i32, vp, i32, vp, vp, f32, f32, vp],
        "spgm_solve_structured": [vp, vp, i32, vp, i32, vp, i32, i32, vp, vp, f32, f32, vp],
        "spgm_prox": [vp, C.POINTER(SpgmRegularizer), vp, f32, vp],
        "spgm_step_reg": [vp, C.POINTER(SpgmRegularizer), vp, i32, vp, vp, f32, f32, vp],
        "spgm_solve_reg": [vp, C.POINTER(SpgmRegularizer), vp, i32, i32, vp, vp, f32, f32, vp],
        "spgm_phase_window": [C.POINTER(SpgmGeometry), C.POINTER(C.c_double)],
        "spgm_batch_options": [vp, i32, i32],
        "spgm_step_noalloc": [vp, vp, i32, vp, vp, f32, f32, vp],
        "spgm_step_grad": [vp, vp, i32, vp, vp, f32, f32, vp, vp],
        "spgm_plan_launch_shape": [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
        "spgm_plan_autotune_batched": [vp, i32, i32, C.c_char_p, C.POINTER(i32)],
        "spgm_plan_batched_shape": [vp, i32, C.POINTER(i32)],
        "spgm_plan_batched_candidates": [vp, i32, C.POINTER(i32), i32, C.POINTER(i32), C.POINTER(i32), i32,
                                         C.POINTER(i32)],
        "spgm_plan_autotune_structured": [vp, i32, i32, i32, C.c_char_p, C.POINTER(i32)],
        "spgm_plan_structured_shape": [vp, i32, i32, i32, C.POINTER(i32)],
        "spgm_batch_autotune": [vp, C.POINTER(i32), C.c_char_p, C.POINTER(i32)],
        "spgm_rows_generate": [C.c_uint64, i32, i32, C.c_int64, i32, C.POINTER(i32)],
        "spgm_subsets_generate": [C.c_uint64, i32, i32, i32, i32, i32, i32, i32, i32, C.POINTER(i32),
                                  C.POINTER(i32), C.POINTER(i32)],
        "spgm_solve_opts_init": [C.c_void_p],
        "spgm_solve_ex": [vp, vp, vp, C.c_void_p, vp],
        "spgm_plan_opts_init": [C.c_void_p],
        "spgm_plan_create_ex": [C.POINTER(vp), C.c_void_p, C.c_void_p],
        "spgm_calibrate": [i32, i32, C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "spgm_unrolled_vjp_step_g": [vp, vp, i32, vp, vp, f32, f32, vp, vp, vp, vp, vp],
        "spgm_solve_tol": [vp, vp, i32, i32, vp, vp, f32, f32, C.c_double, i32, i32, C.POINTER(i32),
                           C.POINTER(C.c_double), vp],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.spgm_last_error.argtypes = []
    lib.spgm_last_error.restype = C.c_char_p
    _LIB = lib
    return lib


def _check(rc):
    if rc != SPGM_OK:
        msg = load_library().spgm_last_error().decode(errors="replace")
        raise SpgmError(rc, msg)


def make_geometry_struct(geom):
    """Build an ``SpgmGeometry`` from the geometry dict of :mod:`.workloads`.
    Returns (struct, keep-alive list)."""
    tx = np.ascontiguousarray(np.asarray(geom["tx"], dtype=np.float64).reshape(-1, 3))
    rx = np.ascontiguousarray(np.asarray(geom["rx"], dtype=np.float64).reshape(-1, 3))
    fr = np.ascontiguousarray(np.asarray(geom["freq"], dtype=np.float64).reshape(-1))
    pulse = geom.get("pulse")
    pl = None
    if pulse is not None:
        pulse = np.asarray(pulse, dtype=np.complex128).reshape(-1)
        pl = np.ascontiguousarray(np.stack([pulse.real, pulse.imag], -1).reshape(-1))
    g = SpgmGeometry()
    g.n_tx, g.n_rx, g.n_freq = tx.shape[0], rx.shape[0], fr.shape[0]
    g.nx, g.ny, g.nz = (int(v) for v in geom["grid"])
    g.tx_xyz = tx.ctypes.data_as(_dp)
    g.rx_xyz = rx.ctypes.data_as(_dp)
    g.freq_hz = fr.ctypes.data_as(_dp)
    g.pulse = pl.ctypes.data_as(_dp) if pl is not None else _dp()
    g.centre = (C.c_double * 3)(*[float(v) for v in geom["centre"]])
    g.pitch = (C.c_double * 3)(*[float(v) for v in np.broadcast_to(geom["pitch"], (3,))])
    g.c = float(geom["c"])
    return g, [tx, rx, fr, pl]


def phase_window(geom):
    """Largest |sin/cos argument| in turns the compensated float32 phase can form for ``geom``."""
    g, keep = make_geometry_struct(geom)
    out = C.c_double()
    _check(load_library().spgm_phase_window(C.byref(g), C.byref(out)))
    del keep
    return out.value


def calibrate(kind, iters=4096):
    """(chain steps per second, launch ms) of the issue-rate probe `kind` (0 FMA, 1 sin, 2 cos,
    3 entry body) on the current device."""
    rate, ms = C.c_double(), C.c_double()
    _check(load_library().spgm_calibrate(int(kind), int(iters), C.byref(rate), C.byref(ms)))
    return rate.value, ms.value


def rows_generate(seed, start_iter, iters, M, B):
    """(iters, B) int32 rows of the library's seeded generator (host only)."""
    out = np.empty((int(iters), int(B)), dtype=np.int32)
    _check(load_library().spgm_rows_generate(C.c_uint64(int(seed) & (2 ** 64 - 1)), int(start_iter), int(iters),
                                             int(M), int(B), out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out


def subsets_generate(seed, start_iter, iters, F, T, R, nf, nt, nr):
    """(f (iters, nf), t (iters, nt), r (iters, nr)) int32 subsets of the seeded generator."""
    f = np.empty((int(iters), int(nf)), dtype=np.int32)
    t = np.empty((int(iters), int(nt)), dtype=np.int32)
    r = np.empty((int(iters), int(nr)), dtype=np.int32)
    ip = C.POINTER(C.c_int32)
    _check(load_library().spgm_subsets_generate(C.c_uint64(int(seed) & (2 ** 64 - 1)), int(start_iter), int(iters),
                                                int(F), int(T), int(R), int(nf), int(nt), int(nr),
                                                f.ctypes.data_as(ip), t.ctypes.data_as(ip), r.ctypes.data_as(ip)))
    return f, t, r


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t, dtype, name, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))
    return C.c_void_p(t.data_ptr())


class Plan:
    """A plan (``spgm_plan``) for one geometry on the current device (or on ``device``, with
    ``tune_cache`` as its autotuners' default cache file: spgm_plan_create_ex)."""

    def __init__(self, geom, phase_mode: int = PHASE_COMP32, _handle=None, device=None, tune_cache=None):
        lib = load_library()
        self._owned = _handle is None
        if _handle is None:
            g, keep = make_geometry_struct(geom)
            h = C.c_void_p()
            if device is None and tune_cache is None:
                _check(lib.spgm_plan_create(C.byref(h), C.byref(g), int(phase_mode)))
            else:
                o = SpgmPlanOpts()
                _check(lib.spgm_plan_opts_init(C.byref(o)))
                o.phase_mode = int(phase_mode)
                o.device = -1 if device is None else int(device)
                o.tune_cache = None if tune_cache is None else os.fsencode(tune_cache)
                _check(lib.spgm_plan_create_ex(C.byref(h), C.byref(g), C.byref(o)))
            del keep
        else:
            h = _handle
        self._h = h
        self._lib = lib
        M, N = C.c_int64(), C.c_int64()
        _check(lib.spgm_plan_dims(h, C.byref(M), C.byref(N)))
        self.M, self.N = M.value, N.value

    def close(self):
        if getattr(self, "_h", None):
            if self._owned:
                self._lib.spgm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --- calls ---------------------------------------------------------------------------
    def spgm_forward(self, rows, s, out=None, stream=None):
        import torch
        B = rows.numel()
        if out is None:
            out = torch.empty(B, dtype=torch.complex64, device=s.device)
        _check(self._lib.spgm_forward(self._h, _dev(rows, torch.int32, "rows"), B,
                                      _dev(s, torch.complex64, "s", self.N),
                                      _dev(out, torch.complex64, "out", B), _stream_ptr(stream)))
        return out

    def spgm_adjoint(self, rows, r, out=None, stream=None):
        import torch
        B = rows.numel()
        if out is None:
            out = torch.empty(self.N, dtype=torch.complex64, device=r.device)
        _check(self._lib.spgm_adjoint(self._h, _dev(rows, torch.int32, "rows"), B,
                                      _dev(r, torch.complex64, "r", B),
                                      _dev(out, torch.complex64, "out", self.N), _stream_ptr(stream)))
        return out

    def spgm_step(self, rows, y, s, eta, alpha, stream=None):
        import torch
        B = rows.numel()
        _check(self._lib.spgm_step(self._h, _dev(rows, torch.int32, "rows"), B,
                                   _dev(y, torch.complex64, "y", self.M), _dev(s, torch.complex64, "s", self.N),
                                   float(eta), float(alpha), _stream_ptr(stream)))
        return s

    def spgm_step_noalloc(self, rows, y, s, eta, alpha, stream=None):
        """spgm_step in the library's fixed scratch array (no device allocation in the call)."""
        import torch
        B = rows.numel()
        _check(self._lib.spgm_step_noalloc(self._h, _dev(rows, torch.int32, "rows"), B,
                                           _dev(y, torch.complex64, "y", self.M),
                                           _dev(s, torch.complex64, "s", self.N), float(eta), float(alpha),
                                           _stream_ptr(stream)))
        return s

    def spgm_solve(self, rows_table, y, s, eta, alpha, stream=None):
        """``rows_table``: int32 tensor of shape (iters, B)."""
        import torch
        if rows_table.dim() != 2:
            raise ValueError("rows_table must be 2-D (iters, B)")
        K, B = rows_table.shape
        _check(self._lib.spgm_solve(self._h, _dev(rows_table, torch.int32, "rows_table"), int(K), int(B),
                                    _dev(y, torch.complex64, "y", self.M), _dev(s, torch.complex64, "s", self.N),
                                    float(eta), float(alpha), _stream_ptr(stream)))
        return s

    def spgm_solve_tol(self, rows_table, y, s, eta, alpha, tol, check_every=50, use_graph=True, stream=None):
        """Iterations of ``rows_table`` (iters, B) until the relative change of the magnitudes is
        below ``tol``; returns (iterations performed, numpy array of their relative changes)."""
        import torch
        if rows_table.dim() != 2:
            raise ValueError("rows_table must be 2-D (iters, B)")
        K, B = rows_table.shape
        done = C.c_int32()
        changes = np.full(int(K), np.nan)
        rc = self._lib.spgm_solve_tol(self._h, _dev(rows_table, torch.int32, "rows_table"), int(K), int(B),
                                      _dev(y, torch.complex64, "y", self.M), _dev(s, torch.complex64, "s", self.N),
                                      float(eta), float(alpha), float(tol), int(check_every), 1 if use_graph else 0,
                                      C.byref(done), changes.ctypes.data_as(C.POINTER(C.c_double)),
                                      _stream_ptr(stream))
        if rc == SPGM_E_NONFINITE:
            err = SpgmError(rc, self._lib.spgm_last_error().decode(errors="replace"))
            err.iters_done = done.value
            raise err
        _check(rc)
        return done.value, changes[:done.value]

    def spgm_solve_ex(self, y, s, iters, eta, lam, B=0, rows=None, seed=0, sampling=0, nf=0, nt=0, nr=0,
                      start_iter=0, tol=0.0, check_every=50, use_graph=False, stream=None):
        """spgm_solve_ex: rows (iters, B) on the device or None (seeded generator); returns the
        number of iterations performed."""
        import torch
        o = SpgmSolveOpts()
        _check(self._lib.spgm_solve_opts_init(C.byref(o)))
        done = C.c_int32()
        o.iters, o.lam, o.eta = int(iters), float(lam), float(eta)
        o.B = int(B) if rows is None else int(rows.shape[1])
        o.rows_d = None if rows is None else _dev(rows, torch.int32, "rows").value
        o.seed, o.sampling, o.nf, o.nt, o.nr = int(seed) & (2 ** 64 - 1), int(sampling), int(nf), int(nt), int(nr)
        o.start_iter, o.tol, o.check_every, o.use_graph = int(start_iter), float(tol), int(check_every), int(use_graph)
        o.iters_done = C.pointer(done)
        _check(self._lib.spgm_solve_ex(self._h, _dev(y, torch.complex64, "y", self.M),
                                       _dev(s, torch.complex64, "s", self.N), C.byref(o), _stream_ptr(stream)))
        return done.value

    # --- other regularisers: kind REG_L1, REG_ELASTIC_NET (mu) or REG_TV_MAGNITUDE (tv_iters) ---
    def spgm_prox(self, v, alpha, kind, mu=0.0, tv_iters=0, stream=None):
        import torch
        reg = SpgmRegularizer(int(kind), float(mu), int(tv_iters))
        _check(self._lib.spgm_prox(self._h, C.byref(reg), _dev(v, torch.complex64, "v", self.N), float(alpha),
                                   _stream_ptr(stream)))
        return v

    def spgm_step_reg(self, rows, y, s, eta, alpha, kind, mu=0.0, tv_iters=0, stream=None):
        import torch
        reg = SpgmRegularizer(int(kind), float(mu), int(tv_iters))
        B = rows.numel()
        _check(self._lib.spgm_step_reg(self._h, C.byref(reg), _dev(rows, torch.int32, "rows"), B,
                                       _dev(y, torch.complex64, "y", self.M), _dev(s, torch.complex64, "s", self.N),
                                       float(eta), float(alpha), _stream_ptr(stream)))
        return s

    def spgm_solve_reg(self, rows_table, y, s, eta, alpha, kind, mu=0.0, tv_iters=0, stream=None):
        """``rows_table``: int32 tensor of shape (iters, B)."""
        import torch
        if rows_table.dim() != 2:
            raise ValueError("rows_table must be 2-D (iters, B)")
        K, B = rows_table.shape
        reg = SpgmRegularizer(int(kind), float(mu), int(tv_iters))
        _check(self._lib.spgm_solve_reg(self._h, C.byref(reg), _dev(rows_table, torch.int32, "rows_table"), int(K),
                                        int(B), _dev(y, torch.complex64, "y", self.M),
                                        _dev(s, torch.complex64, "s", self.N), float(eta), float(alpha),
                                        _stream_ptr(stream)))
        return s

    def spgm_unrolled_vjp_step(self, rows, y, s, eta, tau, sbar_next, sbar, eta_bar, tau_bar, stream=None):
        """Backward of one unrolled iteration; eta_bar / tau_bar: float64 device tensors of one element."""
        import torch
        B = rows.numel()
        _check(self._lib.spgm_unrolled_vjp_step(
            self._h, _dev(rows, torch.int32, "rows"), B, _dev(y, torch.complex64, "y", self.M),
            _dev(s, torch.complex64, "s", self.N), float(eta), float(tau),
            _dev(sbar_next, torch.complex64, "sbar_next", self.N), _dev(sbar, torch.complex64, "sbar", self.N),
            _dev(eta_bar, torch.float64, "eta_bar", 1), _dev(tau_bar, torch.float64, "tau_bar", 1),
            _stream_ptr(stream)))
        return sbar

    def spgm_unrolled_vjp_step_g(self, rows, s, g, eta, tau, sbar_next, sbar, eta_bar, tau_bar, stream=None):
        """spgm_unrolled_vjp_step given g = A_B^H (A_B s - y_B) at the entering iterate."""
        import torch
        B = rows.numel()
        _check(self._lib.spgm_unrolled_vjp_step_g(
            self._h, _dev(rows, torch.int32, "rows"), B, _dev(s, torch.complex64, "s", self.N),
            _dev(g, torch.complex64, "g", self.N), float(eta), float(tau),
            _dev(sbar_next, torch.complex64, "sbar_next", self.N), _dev(sbar, torch.complex64, "sbar", self.N),
            _dev(eta_bar, torch.float64, "eta_bar", 1), _dev(tau_bar, torch.float64, "tau_bar", 1),
            _stream_ptr(stream)))
        return sbar

    def spgm_step_grad(self, rows, y, s, eta, alpha, g, stream=None):
        """spgm_step that also writes g = A_B^H (A_B s - y_B) at the entering iterate."""
        import torch
        B = rows.numel()
        _check(self._lib.spgm_step_grad(self._h, _dev(rows, torch.int32, "rows"), B,
                                        _dev(y, torch.complex64, "y", self.M), _dev(s, torch.complex64, "s", self.N),
                                        float(eta), float(alpha), _dev(g, torch.complex64, "g", self.N),
                                        _stream_ptr(stream)))
        return s

    def spgm_solve_graph(self, rows_table, y, s, eta, alpha, stream=None):
        """spgm_solve replayed from a captured HIP graph (re-captured when arguments change)."""
        import torch
        if rows_table.dim() != 2:
            raise ValueError("rows_table must be 2-D (iters, B)")
        K, B = rows_table.shape
        _check(self._lib.spgm_solve_graph(self._h, _dev(rows_table, torch.int32, "rows_table"), int(K), int(B),
                                          _dev(y, torch.complex64, "y", self.M),
                                          _dev(s, torch.complex64, "s", self.N), float(eta), float(alpha),
                                          _stream_ptr(stream)))
        return s

    def spgm_plan_autotune(self, B, cache_path=None):
        """Tune the row splits for minibatch size B; returns (forward splits, adjoint splits)."""
        fs, as_ = C.c_int32(), C.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(self._lib.spgm_plan_autotune(self._h, int(B), path, C.byref(fs), C.byref(as_)))
        return fs.value, as_.value

    def spgm_plan_launch_shape(self, B):
        """((forward splits, waves), (adjoint splits, waves)) used for minibatches of B rows."""
        v = [C.c_int32() for _ in range(4)]
        _check(self._lib.spgm_plan_launch_shape(self._h, int(B), *[C.byref(x) for x in v]))
        return (v[0].value, v[1].value), (v[2].value, v[3].value)

    def spgm_plan_autotune_batched(self, B, precision=MM_BF16, cache_path=None):
        """Tune the shared-geometry batch kernels for B rows; returns the applied shape as
        spgm_plan_batched_shape does."""
        v = (C.c_int32 * 7)()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(self._lib.spgm_plan_autotune_batched(self._h, int(B), int(precision), path, v))
        return tuple(v)

    def spgm_plan_batched_shape(self, B):
        """(row tiles per wave, bricks per work-group, waves, z slices, adjoint splits, adjoint
        staged rows, 1 if entries are formed in A-operand order) for minibatches of B rows."""
        v = (C.c_int32 * 7)()
        _check(self._lib.spgm_plan_batched_shape(self._h, int(B), v))
        return tuple(v)

    def spgm_plan_batched_candidates(self, B):
        """(forward candidates [(nrt, bricks per work-group, waves, z slices)], adjoint candidates
        [(splits, staged rows)]) that the batched autotuner times for B rows."""
        nf, na = C.c_int32(), C.c_int32()
        _check(self._lib.spgm_plan_batched_candidates(self._h, int(B), None, 0, C.byref(nf), None, 0, C.byref(na)))
        f, a = (C.c_int32 * (4 * max(1, nf.value)))(), (C.c_int32 * (2 * max(1, na.value)))()
        _check(self._lib.spgm_plan_batched_candidates(self._h, int(B), f, nf.value, C.byref(nf), a, na.value,
                                                      C.byref(na)))
        return ([tuple(f[4 * i:4 * i + 4]) for i in range(nf.value)],
                [tuple(a[2 * i:2 * i + 2]) for i in range(na.value)])

    def spgm_plan_autotune_structured(self, nf, nt, nr, cache_path=None):
        """Tune the structured kernels for (nf, nt, nr); returns the items per thread applied."""
        v = C.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(self._lib.spgm_plan_autotune_structured(self._h, int(nf), int(nt), int(nr), path, C.byref(v)))
        return v.value

    def spgm_plan_structured_shape(self, nf, nt, nr):
        """Items per thread (8 or 16) of the structured kernels for (nf, nt, nr)."""
        v = C.c_int32()
        _check(self._lib.spgm_plan_structured_shape(self._h, int(nf), int(nt), int(nr), C.byref(v)))
        return v.value

    def spgm_plan_status(self):
        st = C.c_int32()
        _check(self._lib.spgm_plan_status(self._h, C.byref(st)))
        return st.value

    def spgm_plan_timing(self, enable=True):
        _check(self._lib.spgm_plan_timing(self._h, 1 if enable else 0))

    def spgm_plan_timing_read(self):
        """(forward-tile ms, launches, adjoint-tile ms, launches) since the last read."""
        fm, am = C.c_double(), C.c_double()
        fn, an = C.c_int64(), C.c_int64()
        _check(self._lib.spgm_plan_timing_read(self._h, C.byref(fm), C.byref(fn), C.byref(am), C.byref(an)))
        return fm.value, fn.value, am.value, an.value

    # --- shared-geometry batches (K right-hand sides, 16-bit operands on the matrix cores) ---
    @staticmethod
    def _cols(t, rows_expected, name):
        if t.dim() != 2 or t.shape[0] != rows_expected:
            raise ValueError("%s must have shape (%d, K)" % (name, rows_expected))
        return int(t.shape[1])

    def spgm_forward_batched(self, rows, S, out=None, precision=MM_BF16, stream=None):
        """Y = A_rows S for S of shape (N, K); returns Y of shape (B, K)."""
        import torch
        B = rows.numel()
        K = self._cols(S, self.N, "S")
        if out is None:
            out = torch.empty(B, K, dtype=torch.complex64, device=S.device)
        _check(self._lib.spgm_forward_batched(self._h, _dev(rows, torch.int32, "rows"), B, K,
                                              _dev(S, torch.complex64, "S"),
                                              _dev(out, torch.complex64, "out", B * K), int(precision),
                                              _stream_ptr(stream)))
        return out

    def spgm_adjoint_batched(self, rows, R, out=None, precision=MM_BF16, stream=None):
        """G = A_rows^H R for R of shape (B, K); returns G of shape (N, K)."""
        import torch
        B = rows.numel()
        K = self._cols(R, B, "R")
        if out is None:
            out = torch.empty(self.N, K, dtype=torch.complex64, device=R.device)
        _check(self._lib.spgm_adjoint_batched(self._h, _dev(rows, torch.int32, "rows"), B, K,
                                              _dev(R, torch.complex64, "R"),
                                              _dev(out, torch.complex64, "out", self.N * K), int(precision),
                                              _stream_ptr(stream)))
        return out

    def spgm_step_batched(self, rows, Ymeas, S, eta, alpha, precision=MM_BF16, stream=None):
        """One SPGM iteration of K problems in place: Ymeas (M, K), S (N, K)."""
        import torch
        K = self._cols(S, self.N, "S")
        if self._cols(Ymeas, self.M, "Ymeas") != K:
            raise ValueError("Ymeas and S must have the same number of columns")
        _check(self._lib.spgm_step_batched(self._h, _dev(rows, torch.int32, "rows"), rows.numel(), K,
                                           _dev(Ymeas, torch.complex64, "Ymeas"), _dev(S, torch.complex64, "S"),
                                           float(eta), float(alpha), int(precision), _stream_ptr(stream)))
        return S

    def spgm_solve_batched(self, rows_table, Ymeas, S, eta, alpha, precision=MM_BF16, stream=None):
        """``rows_table``: int32 tensor of shape (iters, B); Ymeas (M, K), S (N, K) in place."""
        import torch
        if rows_table.dim() != 2:
            raise ValueError("rows_table must be 2-D (iters, B)")
        iters, B = rows_table.shape
        K = self._cols(S, self.N, "S")
        if self._cols(Ymeas, self.M, "Ymeas") != K:
            raise ValueError("Ymeas and S must have the same number of columns")
        _check(self._lib.spgm_solve_batched(self._h, _dev(rows_table, torch.int32, "rows_table"), int(iters),
                                            int(B), K, _dev(Ymeas, torch.complex64, "Ymeas"),
                                            _dev(S, torch.complex64, "S"), float(eta), float(alpha),
                                            int(precision), _stream_ptr(stream)))
        return S

    # --- structured minibatches (frequency x Tx x Rx subsets, separable factorisation) --------
    @staticmethod
    def _subsets(fs, ts, rs):
        import torch
        return [(_dev(x, torch.int32, name), int(x.shape[-1])) for x, name in ((fs, "f_idx"), (ts, "t_idx"),
                                                                              (rs, "r_idx"))]

    def spgm_forward_structured(self, fs, ts, rs, s, out=None, stream=None):
        """y = A_rows s for the rows of fs x ts x rs (order (i, a, b)); returns complex64[nf*nt*nr]."""
        import torch
        (f, nf), (t, nt), (r, nr) = self._subsets(fs, ts, rs)
        B = nf * nt * nr
        if out is None:
            out = torch.empty(B, dtype=torch.complex64, device=s.device)
        _check(self._lib.spgm_forward_structured(self._h, f, nf, t, nt, r, nr, _dev(s, torch.complex64, "s", self.N),
                                                 _dev(out, torch.complex64, "out", B), _stream_ptr(stream)))
        return out

    def spgm_adjoint_structured(self, fs, ts, rs, r_vec, out=None, stream=None):
        import torch
        (f, nf), (t, nt), (r, nr) = self._subsets(fs, ts, rs)
        B = nf * nt * nr
        if out is None:
            out = torch.empty(self.N, dtype=torch.complex64, device=r_vec.device)
        _check(self._lib.spgm_adjoint_structured(self._h, f, nf, t, nt, r, nr, _dev(r_vec, torch.complex64, "r", B),
                                                 _dev(out, torch.complex64, "out", self.N), _stream_ptr(stream)))
        return out

    def spgm_step_structured(self, fs, ts, rs, y, s, eta, alpha, stream=None):
        import torch
        (f, nf), (t, nt), (r, nr) = self._subsets(fs, ts, rs)
        _check(self._lib.spgm_step_structured(self._h, f, nf, t, nt, r, nr, _dev(y, torch.complex64, "y", self.M),
                                              _dev(s, torch.complex64, "s", self.N), float(eta), float(alpha),
                                              _stream_ptr(stream)))
        return s

    def spgm_solve_structured(self, fs, ts, rs, y, s, eta, alpha, stream=None):
        """fs (iters, nf), ts (iters, nt), rs (iters, nr) int32 tensors."""
        import torch
        if fs.dim() != 2 or ts.dim() != 2 or rs.dim() != 2 or not (fs.shape[0] == ts.shape[0] == rs.shape[0]):
            raise ValueError("fs, ts, rs must be 2-D with the same number of iterations")
        (f, nf), (t, nt), (r, nr) = self._subsets(fs, ts, rs)
        _check(self._lib.spgm_solve_structured(self._h, f, nf, t, nt, r, nr, int(fs.shape[0]),
                                               _dev(y, torch.complex64, "y", self.M),
                                               _dev(s, torch.complex64, "s", self.N), float(eta), float(alpha),
                                               _stream_ptr(stream)))
        return s

    # short aliases
    forward = spgm_forward
    adjoint = spgm_adjoint
    step = spgm_step
    solve = spgm_solve
    status = spgm_plan_status
    autotune = spgm_plan_autotune


class Batch:
    """A ragged batch (``spgm_batch``) of independent scenes advanced by one launch per phase."""

    def __init__(self, geoms, phase_mode: int = PHASE_COMP32):
        lib = load_library()
        n = len(geoms)
        arr = (SpgmGeometry * n)()
        keep = []
        for i, geom in enumerate(geoms):
            g, k = make_geometry_struct(geom)
            arr[i] = g
            keep.append(k)
        h = C.c_void_p()
        _check(lib.spgm_batch_create(C.byref(h), arr, n, int(phase_mode)))
        del keep
        self._h, self._lib, self.n = h, lib, n
        self.plans = []
        for i in range(n):
            ph = C.c_void_p()
            _check(lib.spgm_batch_plan(h, i, C.byref(ph)))
            self.plans.append(Plan(None, _handle=ph))

    def close(self):
        if getattr(self, "_h", None):
            for p in self.plans:
                p.close()
            self._lib.spgm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def spgm_batch_solve(self, rows_tables, ys, ss, etas, alphas, use_graph=False, stream=None):
        """rows_tables[i]: int32 (iters, B_i); ys[i]: complex64 (M_i,); ss[i]: complex64 (N_i,) in/out."""
        import torch
        n = self.n
        if not (len(rows_tables) == len(ys) == len(ss) == len(etas) == len(alphas) == n):
            raise ValueError("one entry per scene is required")
        iters = int(rows_tables[0].shape[0])
        Bs = (C.c_int32 * n)()
        rp, yp, sp = (C.c_void_p * n)(), (C.c_void_p * n)(), (C.c_void_p * n)()
        for i in range(n):
            if rows_tables[i].dim() != 2 or int(rows_tables[i].shape[0]) != iters:
                raise ValueError("every rows table must be (iters, B_i) with the same iters")
            Bs[i] = int(rows_tables[i].shape[1])
            rp[i] = _dev(rows_tables[i], torch.int32, "rows")
            yp[i] = _dev(ys[i], torch.complex64, "y", self.plans[i].M)
            sp[i] = _dev(ss[i], torch.complex64, "s", self.plans[i].N)
        ea = (C.c_float * n)(*[float(v) for v in etas])
        aa = (C.c_float * n)(*[float(v) for v in alphas])
        _check(self._lib.spgm_batch_solve(self._h, iters, Bs, rp, yp, sp, ea, aa, 1 if use_graph else 0,
                                          _stream_ptr(stream)))

    def spgm_batch_options(self, max_workgroups=0, rows_per_split=0):
        """Launch shape of the tile phases: persistent work-groups (0: fill the chip) and rows per
        work item (0: 1024; else a multiple of 64)."""
        _check(self._lib.spgm_batch_options(self._h, int(max_workgroups), int(rows_per_split)))

    def spgm_batch_status(self):
        st = C.c_int32()
        _check(self._lib.spgm_batch_status(self._h, C.byref(st)))
        return st.value

    def spgm_batch_autotune(self, Bs, cache_path=None):
        """Tune the rows per work item for minibatch sizes Bs (one per scene); returns it."""
        if len(Bs) != self.n:
            raise ValueError("one minibatch size per scene is required")
        arr = (C.c_int32 * self.n)(*[int(b) for b in Bs])
        v = C.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(self._lib.spgm_batch_autotune(self._h, arr, path, C.byref(v)))
        return v.value

    solve = spgm_batch_solve
    status = spgm_batch_status
    options = spgm_batch_options
    autotune = spgm_batch_autotune
