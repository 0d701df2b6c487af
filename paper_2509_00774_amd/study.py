"""Paper-protocol study on the paper-shaped synthetic workload (Sec. V, Figs. 2-4).

Workload: 16 Tx + 9 Rx at seeded random positions in a 0.3 m aperture, 11 frequencies in
4-16 GHz, a 61 x 61 x 21 voxel cube at 5 mm centred 0.5 m from the array (the scenario of
Sec. V); a seeded 0.2 % random-phase scene and 30 dB noise stand in for the measured data.

Protocol (Sec. V): SPGM with structured minibatches (#f, #Tx, #Rx) drawn afresh every
iteration, and PGM (all 11 x 16 x 9 rows every iteration), each run until the change in
reflectivity magnitudes drops below 1e-3; runtime against composition (Fig. 2), convergence
(Fig. 3), PSNR over normalised magnitudes with the PGM reconstruction as reference (Fig. 4), and
PGM run under the time budget of SPGM (4, 4, 3) (PGM*).  Readings where the paper is silent:
the change is || |s_k+1| - |s_k| || / || |s_k| || in the 2-norm; the regularisation weight is
lambda = 0.05 max|A^H y| / M for every run (alpha = lambda eta); the step size is 1/L with L the
top eigenvalue of A_B^H A_B / B -- of the full matrix for PGM, and the largest over four sampled
minibatches of the composition for SPGM ("own step").  The paper uses one step size for every
run; that protocol is run as well ("PGM step": SPGM at the PGM step size), and it is reported
as diverged when the iterate grows without bound.  The synthetic scene has 0.2 % non-zero
voxels (156 points; with 1 584 measurements a 2 % scene is beyond what l1 recovers).
Runtime = measured wall-clock time of the library's solve to termination (spgm_solve_tol: the
termination rule evaluated on the device after every iteration, read back once per group of 50
iterations).  Beside the protocol's termination rule, every run
records the PSNR against a converged PGM reconstruction (5 000 full iterations) every 10
iterations, and the table gives the runtime until it first reaches 30 and 40 dB ("PGM to
convergence" is PGM's own approach to that reference).  Every iteration runs on the pair
kernels with the Cartesian-product rows of its minibatch (at these antenna counts they are
faster than the separable path; both compute the same minibatch gradient).

Usage:  python -m paper_2509_00774_amd.study [--out profiles/study_P]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import workloads as W

COMPOSITIONS = [(2, 4, 3), (4, 4, 3), (4, 8, 3), (11, 4, 3), (4, 8, 9), (8, 8, 9), (4, 16, 9), (11, 16, 3),
                (8, 16, 9)]


def psnr_normalised(x, ref):
    """PSNR (dB) of |x|/max|x| against |ref|/max|ref| (peak 1)."""
    a = np.abs(x) / max(np.max(np.abs(x)), 1e-30)
    b = np.abs(ref) / max(np.max(np.abs(ref)), 1e-30)
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def nmse_db(x, ref):
    return 10.0 * np.log10(float(np.sum(np.abs(x - ref) ** 2)) / float(np.sum(np.abs(ref) ** 2)))


class Problem:
    def __init__(self, torch, binding, dev, seed_offset=0):
        self.torch, self.bd, self.dev = torch, binding, dev
        cfg = W.CONFIGS["P"]
        self.cfg = cfg
        self.geom = W.config_geometry("P")
        self.T, self.R, self.F = cfg["T"], cfg["R"], cfg["F"]
        self.plan = binding.Plan(self.geom)
        self.M, self.N = self.plan.M, self.plan.N
        N = int(np.prod(cfg["grid"]))
        self.s_true, idx = W.random_scene(N, 0.002, seed=cfg["seed"] + 1)
        st = torch.from_numpy(self.s_true.astype(np.complex64)).to(dev)
        self.all_f = torch.arange(self.F, dtype=torch.int32, device=dev)
        self.all_t = torch.arange(self.T, dtype=torch.int32, device=dev)
        self.all_r = torch.arange(self.R, dtype=torch.int32, device=dev)
        y0 = self.plan.spgm_forward_structured(self.all_f, self.all_t, self.all_r, st)  # row order = m order
        y = W.add_noise(y0.cpu().numpy().astype(np.complex128), cfg["snr_db"], seed=cfg["seed"] + 2)
        self.y = torch.from_numpy(y.astype(np.complex64)).to(dev)
        g = self.plan.spgm_adjoint_structured(self.all_f, self.all_t, self.all_r, self.y)
        self.lambda_max = float(torch.max(torch.abs(g)).item()) / self.M

    def top_eigenvalue(self, fs, ts, rs, iters=25, seed=0):
        """Power iteration on A_B^H A_B / B for one structured minibatch."""
        torch = self.torch
        B = fs.numel() * ts.numel() * rs.numel()
        rng = np.random.default_rng(seed)
        v = torch.from_numpy((rng.standard_normal(self.N) + 1j * rng.standard_normal(self.N)).astype(np.complex64))
        v = v.to(self.dev)
        lam = 0.0
        for _ in range(iters):
            v = v / torch.linalg.vector_norm(v)
            u = self.plan.spgm_forward_structured(fs, ts, rs, v)
            w = self.plan.spgm_adjoint_structured(fs, ts, rs, u) / B
            lam = float(torch.real(torch.vdot(v, w)).item())
            v = w
        return lam

    def row_table(self, comp, K, seed):
        """K x B table of the Cartesian-product rows (the same subsets as `subsets`), or every row
        for the full composition.  The iterations run on the pair kernels, which take these rows
        faster than the separable path at the paper's antenna counts."""
        if comp == (self.F, self.T, self.R):
            rows = np.broadcast_to(np.arange(self.M, dtype=np.int32), (K, self.M))
        else:
            rows = W.draw_structured_rows(self.T, self.R, self.F, *comp, K, seed=seed)
        return self.torch.from_numpy(np.ascontiguousarray(rows, dtype=np.int32)).to(self.dev)

    def subsets(self, comp, K, seed):
        nf, nt, nr = comp
        fs, ts, rs = W.draw_structured_subsets(self.T, self.R, self.F, nf, nt, nr, K, seed=seed)
        return [self.torch.from_numpy(x).to(self.dev) for x in (fs, ts, rs)]

    def run(self, comp, eta, alpha, tol, max_iters, seed, record_every=10, ref=None):
        """SPGM (or PGM for the full composition) from zero until the library's termination rule
        holds (spgm_solve_tol, at most max_iters iterations).

        Returns (s, iterations, status, curve, wall_s): status is True when the rule was met,
        False at max_iters, "diverged" for a non-finite iterate; wall_s is the measured
        wall-clock time of one uninterrupted solve to termination (graph-replayed groups of 50
        iterations, one host read of the change records per group).  curve rows are
        [iteration, change, PSNR against `ref` or None] every `record_every` iterations, from a
        second pass in segments of `record_every` iterations that reproduces the same iterates
        (the kernels and the rule do not depend on how iterations are grouped; checked)."""
        torch = self.torch
        rows = self.row_table(comp, max_iters, seed)
        s = torch.zeros(self.N, dtype=torch.complex64, device=self.dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            k, changes = self.plan.spgm_solve_tol(rows, self.y, s, eta, alpha, tol, check_every=50, use_graph=True)
            status = bool(k < max_iters or (tol > 0 and k > 0 and changes[-1] < tol))
        except self.bd.SpgmError as e:
            if e.code != self.bd.SPGM_E_NONFINITE:
                raise
            k, status = e.iters_done, "diverged"
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        curve = []
        s2 = torch.zeros_like(s)
        ref_h = None if ref is None else ref.cpu().numpy()
        for k0 in range(0, k, record_every):
            n = min(record_every, k - k0)
            try:
                _, ch = self.plan.spgm_solve_tol(rows[k0:k0 + n], self.y, s2, eta, alpha, 0.0, check_every=n,
                                                 use_graph=True)
            except self.bd.SpgmError as e:
                if e.code != self.bd.SPGM_E_NONFINITE:
                    raise
                break
            if (k0 + n) % record_every == 0:
                p = None if ref_h is None else psnr_normalised(s2.cpu().numpy(), ref_h)
                curve.append([k0 + n, float(ch[-1]), p])
        if status != "diverged":
            assert torch.equal(s, s2), "segmented pass must reproduce the solve"
        return s, k, status, curve, wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="profiles/study_P")
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--max-iters", type=int, default=20000)
    args = ap.parse_args()
    import torch

    from . import binding
    dev = torch.device("cuda:0")
    P = Problem(torch, binding, dev)
    full = (P.F, P.T, P.R)
    print("[study] P: T=%d R=%d F=%d M=%d N=%d, lambda_max=%.4e" % (P.T, P.R, P.F, P.M, P.N, P.lambda_max), flush=True)
    L_full = P.top_eigenvalue(P.all_f, P.all_t, P.all_r)
    lam = 0.05 * P.lambda_max
    eta_pgm = float(np.float32(1.0 / L_full))
    print("[study] lambda %.4e; PGM step 1/L_full = %.4e" % (lam, eta_pgm), flush=True)

    # A converged PGM reference beside the protocol's (which stops at the 1e-3 change rule).
    s_conv, _, _, _, _ = P.run(full, eta_pgm, float(np.float32(lam * eta_pgm)), 0.0, 5000, 1, record_every=5000)
    s_conv_h = s_conv.cpu().numpy().astype(np.complex128)
    thresholds = (30.0, 40.0)

    def time_to(curve, t_it, db):
        """Runtime (s) until the recorded PSNR against the converged PGM first reaches db."""
        for it, _, p in curve:
            if p is not None and np.isfinite(p) and p >= db:
                return it * t_it
        return None

    def entry(name, comp, eta, k, term, t_it, s_h, curve, ref):
        B = comp[0] * comp[1] * comp[2]
        ok = bool(np.all(np.isfinite(s_h)))
        rec = {"composition": list(comp), "B": B, "eta": eta, "iterations": k, "epochs": k * B / P.M,
               "terminated": term, "s_per_iteration": t_it, "runtime_s": k * t_it,
               "nmse_db_vs_truth": nmse_db(s_h, P.s_true) if ok else None,
               "psnr_db_vs_pgm": None if ref is None or not ok else psnr_normalised(s_h, ref),
               "psnr_db_vs_pgm_converged": psnr_normalised(s_h, s_conv_h) if ok else None,
               "curve": curve}
        for db in thresholds:
            rec["runtime_s_to_%ddb_vs_converged" % db] = time_to(curve, t_it, db)
        return rec

    records = {}
    # PGM's own approach to the converged reconstruction (no termination rule), for the
    # time-to-quality columns
    _, k_c, _, curve_c, wall_c = P.run(full, eta_pgm, float(np.float32(lam * eta_pgm)), 0.0, 5000, 1, ref=s_conv)
    records["PGM to convergence"] = entry("PGM", full, eta_pgm, k_c, False, wall_c / k_c, s_conv_h, curve_c, None)
    s_pgm, k_pgm, term_pgm, curve_pgm, wall_pgm = P.run(full, eta_pgm, float(np.float32(lam * eta_pgm)), args.tol,
                                                        args.max_iters, 1, ref=s_conv)
    t_pgm = wall_pgm / max(k_pgm, 1)
    s_pgm_h = s_pgm.cpu().numpy().astype(np.complex128)
    records["PGM"] = entry("PGM", full, eta_pgm, k_pgm, term_pgm, t_pgm, s_pgm_h, curve_pgm, None)
    print("[study] PGM: %d iterations (terminated %s), %.1f us/iteration, runtime %.4f s, NMSE %.2f dB" % (
        k_pgm, term_pgm, 1e6 * t_pgm, k_pgm * t_pgm, records["PGM"]["nmse_db_vs_truth"]), flush=True)
    pgm_runtime = k_pgm * t_pgm
    for ci, comp in enumerate(COMPOSITIONS):
        fs, ts, rs = P.subsets(comp, 4, 9000 + ci)
        L_b = max(P.top_eigenvalue(fs[j], ts[j], rs[j], seed=ci * 4 + j) for j in range(4))
        for tag, eta in (("own step", float(np.float32(1.0 / L_b))), ("PGM step", eta_pgm)):
            alpha = float(np.float32(lam * eta))
            s, k, term, curve, wall = P.run(comp, eta, alpha, args.tol, args.max_iters, 100000 * (ci + 1), ref=s_conv)
            t_it = wall / max(k, 1)
            sh = s.cpu().numpy().astype(np.complex128)
            rec = entry("SPGM", comp, eta, k, term, t_it, sh, curve, s_pgm_h)
            rec["speedup_vs_pgm"] = pgm_runtime / max(k * t_it, 1e-30)
            records["SPGM %d,%d,%d %s" % (comp + (tag,))] = rec
            print("[study] SPGM %s %s (eta %.3e): %d iterations (%.1f epochs, terminated %s), %.1f us/iteration, "
                  "runtime %.4f s (%.2fx PGM), PSNR vs PGM %s dB, NMSE %s dB" % (
                      comp, tag, eta, k, rec["epochs"], term, 1e6 * t_it, k * t_it, rec["speedup_vs_pgm"],
                      rec["psnr_db_vs_pgm"], rec["nmse_db_vs_truth"]), flush=True)
            print("[study]     PSNR vs converged PGM %s dB" % rec["psnr_db_vs_pgm_converged"], flush=True)
    # PGM* : PGM under the time budget of SPGM (4, 4, 3) (own step)
    budget = records["SPGM 4,4,3 own step"]["runtime_s"]
    k_star = max(1, int(budget / t_pgm))
    s_star, _, _, _, _ = P.run(full, eta_pgm, float(np.float32(lam * eta_pgm)), 0.0, k_star, 1, record_every=k_star)
    sh = s_star.cpu().numpy().astype(np.complex128)
    records["PGM*"] = entry("PGM*", full, eta_pgm, k_star, False, t_pgm, sh, [], s_pgm_h)
    print("[study] PGM* (budget of SPGM (4,4,3), %.4f s): %d iterations, PSNR vs PGM %.2f dB, NMSE %.2f dB" % (
        budget, k_star, records["PGM*"]["psnr_db_vs_pgm"], records["PGM*"]["nmse_db_vs_truth"]), flush=True)

    out = {"workload": "P-shaped synthetic: 16 Tx + 9 Rx in 0.3 m, 11 f in 4-16 GHz, 61x61x21 voxels at 5 mm, "
                       "z0 = 0.5 m, 0.2 % random-phase scene, 30 dB",
           "M": P.M, "N": P.N, "lambda": lam, "lambda_max": P.lambda_max, "L_full": L_full, "tol": args.tol,
           "records": records}
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    # the JSON keeps every 1000th point of each curve (the table below reads the full curves)
    thin = {"records": {k: dict(r, curve=[c for c in r["curve"] if c[0] % 1000 == 0]) for k, r in records.items()}}
    json.dump(dict(out, **thin), open(args.out + ".json", "w"), indent=1)
    lines = ["| run | B | step | iterations | epochs | terminated | us / iteration | runtime (ms) | speedup vs PGM "
             "| PSNR vs PGM (dB) | PSNR vs converged PGM (dB) | NMSE vs truth (dB) "
             "| ms to 30 dB vs converged | ms to 40 dB vs converged |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    fmt = lambda v, f: "—" if v is None else f % v  # noqa: E731
    for name, r in records.items():
        ms = lambda v: None if v is None else 1e3 * v  # noqa: E731
        lines.append("| %s | %d | %.3e | %d | %.1f | %s | %.1f | %.2f | %s | %s | %s | %s | %s | %s |" % (
            name, r["B"], r["eta"], r["iterations"], r["epochs"], r["terminated"], 1e6 * r["s_per_iteration"],
            1e3 * r["runtime_s"], fmt(r.get("speedup_vs_pgm"), "%.2f"), fmt(r["psnr_db_vs_pgm"], "%.2f"),
            fmt(r["psnr_db_vs_pgm_converged"], "%.2f"), fmt(r["nmse_db_vs_truth"], "%.2f"),
            fmt(ms(r["runtime_s_to_30db_vs_converged"]), "%.1f"), fmt(ms(r["runtime_s_to_40db_vs_converged"]), "%.1f")))
    # Convergence against time (the counterpart of Fig. 3): PSNR against the converged PGM
    # reconstruction at fixed runtimes, from each run's recorded curve.
    marks_ms = (10, 25, 50, 100, 200, 400, 800, 1600)
    lines += ["", "PSNR (dB) against the converged PGM reconstruction after a given runtime:", "",
              "| run | " + " | ".join("%d ms" % m for m in marks_ms) + " |",
              "|---|" + "---|" * len(marks_ms)]
    for name, r in records.items():
        curve = r["curve"]
        if not curve or curve[0][2] is None:
            continue
        cells = []
        for m in marks_ms:
            k = int(m * 1e-3 / r["s_per_iteration"])
            pts = [c for c in curve if c[0] <= k]
            v = pts[-1][2] if pts else None
            cells.append("—" if v is None or not np.isfinite(v) or k > r["iterations"] else "%.1f" % v)
        lines.append("| %s | %s |" % (name, " | ".join(cells)))
    open(args.out + "_table.md", "w").write("\n".join(lines) + "\n")
    print("\n".join(lines), flush=True)


if __name__ == "__main__":
    main()
