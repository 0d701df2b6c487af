"""Learning the step sizes and thresholds of a 10-iteration unrolled SPGM (the differentiable
form of Sec. IV, Eq. 5 with the minibatch gradient of Eq. 6).

Workload (16 Tx + 16 Rx in 0.2 m, 32 frequencies in 20-30 GHz, 32 x 32 x 16 voxels at 5 mm,
B = 2048 rows per iteration, one row table fixed by seed for every scene): 256 seeded training
scenes at 2 % density and 25 dB SNR, 32 held-out scenes of the same kind.  Parameters: per
iteration eta_k = eta_0 exp(a_k) and tau_k = lambda eta_0 exp(b_k) (log-scales, so both stay
positive), initialised at the plain solver's eta_0 = 1/L and lambda = 5 % of lambda_max
(the oracle-written step-size table).  Loss: mean squared error of s_10 to the true scene,
averaged over a minibatch of scenes; Adam on (a, b).  The forward and backward passes run in
the library (UnrolledSPGMFn: spgm_step, spgm_step_grad and spgm_unrolled_vjp_step_g); PyTorch
only holds the 20 parameters and the optimiser state.

Reported: training loss per epoch, held-out NMSE against the truth of the learned 10-iteration
unroll, of the same unroll at the initial parameters, and the number of plain SPGM iterations
(float32 projector, the initial eta and lambda, same row sampling continued with fresh seeded
rows) needed to reach the learned unroll's NMSE, with the measured time of each (matched
reconstruction error).

Usage:  python -m paper_2509_00774_amd.train_unrolled [--epochs 4] [--out profiles/train_c4]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def nmse(x, ref):
    return float(np.sum(np.abs(x - ref) ** 2) / np.sum(np.abs(ref) ** 2))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--scenes", type=int, default=256)
    ap.add_argument("--held-out", type=int, default=32)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=0.05)
    ap.add_argument("--max-plain", type=int, default=400)
    ap.add_argument("--out", default="profiles/train_c4")
    args = ap.parse_args()
    import torch

    from . import binding
    from .autograd import unrolled_spgm

    dev = torch.device("cuda:0")
    cfg = W.CONFIGS["c4"]
    geom = W.config_geometry("c4")
    M, N = W.dims(geom)
    K = cfg["K"]
    B = cfg["B"]
    steps = json.load(open(os.path.join(ROOT, "tests", "golden", "step_sizes.json")))["c4"]
    eta0 = float(np.float32(steps["eta"]))
    lam = float(steps["lambda"])
    plan = binding.Plan(geom)
    rows = torch.from_numpy(W.config_rows("c4", K=K)).to(dev)
    all_rows = torch.arange(M, dtype=torch.int32, device=dev)

    def scene(i):
        st, _ = W.random_scene(N, cfg["density"], seed=20000 + i)
        y0 = plan.spgm_forward(all_rows, torch.from_numpy(st.astype(np.complex64)).to(dev))
        y = W.add_noise(y0.cpu().numpy().astype(np.complex128), cfg["snr_db"], seed=30000 + i)
        return torch.from_numpy(st.astype(np.complex64)).to(dev), torch.from_numpy(y.astype(np.complex64)).to(dev)

    n_all = args.scenes + args.held_out
    t0 = time.perf_counter()
    data = [scene(i) for i in range(n_all)]
    train, held = data[:args.scenes], data[args.scenes:]
    print("[train] %d training + %d held-out scenes generated in %.1f s (M=%d, N=%d, B=%d, K=%d)" % (
        args.scenes, args.held_out, time.perf_counter() - t0, M, N, B, K), flush=True)

    a = torch.zeros(K, dtype=torch.float64, device=dev, requires_grad=True)
    b = torch.zeros(K, dtype=torch.float64, device=dev, requires_grad=True)
    opt = torch.optim.Adam([a, b], lr=args.lr)
    zero = torch.zeros(N, dtype=torch.complex64, device=dev)

    def unroll(y, grad=True):
        eta = eta0 * torch.exp(a)
        tau = lam * eta0 * torch.exp(b)
        if not grad:
            eta, tau = eta.detach(), tau.detach()
        return unrolled_spgm(plan, rows, y, zero, eta, tau)

    def held_nmse():
        with torch.no_grad():
            return float(np.mean([nmse(unroll(y, grad=False).cpu().numpy(), st.cpu().numpy()) for st, y in held]))

    nmse_init = held_nmse()
    print("[train] held-out NMSE at the initial parameters: %.4f (%.2f dB)" % (nmse_init, 10 * np.log10(nmse_init)),
          flush=True)
    rng = np.random.default_rng(1)
    history = []
    t_train = 0.0
    n_steps = 0
    for ep in range(args.epochs):
        order = rng.permutation(len(train))
        losses = []
        for j in range(0, len(order), args.batch):
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            opt.zero_grad()
            loss = 0.0
            idx = order[j:j + args.batch]
            for i in idx:
                st, y = train[i]
                out = unroll(y)
                loss = loss + torch.mean(torch.abs(out - st) ** 2) / len(idx)
            loss.backward()
            opt.step()
            torch.cuda.synchronize()
            t_train += time.perf_counter() - c0
            n_steps += len(idx)
            losses.append(float(loss.item()))
        h = held_nmse()
        history.append({"epoch": ep + 1, "train_loss": float(np.mean(losses)), "held_out_nmse": h})
        print("[train] epoch %d: train loss %.6e, held-out NMSE %.4f (%.2f dB)" % (
            ep + 1, np.mean(losses), h, 10 * np.log10(h)), flush=True)
    nmse_learned = history[-1]["held_out_nmse"] if history else nmse_init

    # Plain SPGM at the initial parameters: iterations (and time) to the learned unroll's NMSE.
    alpha0 = float(np.float32(lam * eta0))
    plain_rows = torch.from_numpy(W.draw_rows(M, B, args.max_plain, seed=cfg["seed"] + 3)).to(dev)
    plain_rows[:K] = rows
    iters_to_match, t_plain = [], []
    for st, y in held:
        s = torch.zeros(N, dtype=torch.complex64, device=dev)
        st_h = st.cpu().numpy()
        hit = None
        for k in range(args.max_plain):
            plan.spgm_step(plain_rows[k], y, s, eta0, alpha0)
            if nmse(s.cpu().numpy(), st_h) <= nmse_learned:
                hit = k + 1
                break
        iters_to_match.append(hit)
    s = torch.zeros(N, dtype=torch.complex64, device=dev)
    plan.spgm_solve(plain_rows[:K].contiguous(), held[0][1], s, eta0, alpha0)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    for _ in range(20):
        plan.spgm_solve(plain_rows[:K].contiguous(), held[0][1], s, eta0, alpha0)
    torch.cuda.synchronize()
    t_plain_k = (time.perf_counter() - c0) / 20
    with torch.no_grad():
        unroll(held[0][1], grad=False)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        for _ in range(20):
            unroll(held[0][1], grad=False)
        torch.cuda.synchronize()
        t_unroll = (time.perf_counter() - c0) / 20
    reached = [v for v in iters_to_match if v is not None]
    eta_l = (eta0 * torch.exp(a)).detach().cpu().numpy()
    tau_l = (lam * eta0 * torch.exp(b)).detach().cpu().numpy()
    out = {
        "workload": "c4: 16 Tx + 16 Rx, 32 f in 20-30 GHz, 32x32x16 voxels at 5 mm, B=2048, K=10 unrolled iterations",
        "train_scenes": args.scenes, "held_out_scenes": args.held_out, "epochs": args.epochs,
        "batch": args.batch, "lr": args.lr, "eta0": eta0, "lambda": lam,
        "held_out_nmse_initial": nmse_init, "held_out_nmse_learned": nmse_learned, "history": history,
        "eta_learned": eta_l.tolist(), "tau_learned": tau_l.tolist(),
        "plain_iters_to_learned_nmse": iters_to_match,
        "plain_iters_to_learned_nmse_median": None if not reached else float(np.median(reached)),
        "plain_reached": len(reached),
        "ms_unrolled_forward": 1e3 * t_unroll, "ms_plain_10_iterations": 1e3 * t_plain_k,
        "ms_per_training_scene": 1e3 * t_train / max(n_steps, 1),
    }
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    json.dump(out, open(args.out + ".json", "w"), indent=1)
    med = out["plain_iters_to_learned_nmse_median"]
    lines = [
        "| quantity | value |", "|---|---|",
        "| held-out NMSE, 10 iterations at the initial eta, tau | %.4f (%.2f dB) |" % (nmse_init, 10 * np.log10(nmse_init)),
        "| held-out NMSE, 10 learned iterations | %.4f (%.2f dB) |" % (nmse_learned, 10 * np.log10(nmse_learned)),
        "| plain SPGM iterations to the learned NMSE (median over %d of %d held-out scenes) | %s |" % (
            len(reached), len(held), "—" if med is None else "%.0f" % med),
        "| unrolled forward (10 iterations), ms | %.3f |" % (1e3 * t_unroll),
        "| plain solve of 10 iterations, ms | %.3f |" % (1e3 * t_plain_k),
        "| training, forward + backward per scene, ms | %.3f |" % (1e3 * t_train / max(n_steps, 1)),
    ]
    open(args.out + ".md", "w").write("\n".join(lines) + "\n")
    print("\n".join(lines), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
