"""GPU differentiation: the autograd wrappers and the native unrolled-SPGM backward against the
FP64 oracle's chain-rule gradient (which the CPU tests pin to central finite differences).

Tolerances: projector VJPs 1e-5 relative L2 (same arithmetic as the projector); unrolled SPGM
gradients 1e-4 relative L2 (float32 iterates through 10 iterations of forward and backward).
"""
import json
import os

import numpy as np
import pytest

from oracle import Oracle, rel_l2, unrolled_forward, unrolled_vjp
from paper_2509_00774_amd import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print("[gpu-autograd]", *a, flush=True)


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_00774_amd import binding
    binding.load_library()
    return binding


def cdev(x, grad=False):
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex64))).cuda()
    return t.requires_grad_(grad)


def idev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.int32))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def test_projector_and_adjoint_vjps(bd):
    from paper_2509_00774_amd.autograd import adjoint, projector
    geom = W.config_geometry("c0")
    orc = Oracle(geom)
    plan = bd.Plan(geom)
    rows = W.config_rows("c0", K=1)[0]
    s = cdev(W.random_complex(orc.N, seed=1), grad=True)
    ybar = W.random_complex(rows.size, seed=2).astype(np.complex64)
    y = projector(plan, idev(rows), s)
    (gs,) = torch.autograd.grad(y, s, grad_outputs=cdev(ybar))
    e1 = rel_l2(host(gs), orc.adjoint(rows, ybar.astype(np.complex128)))
    r = cdev(W.random_complex(rows.size, seed=3), grad=True)
    gbar = W.random_complex(orc.N, seed=4).astype(np.complex64)
    g = adjoint(plan, idev(rows), r)
    (gr,) = torch.autograd.grad(g, r, grad_outputs=cdev(gbar))
    e2 = rel_l2(host(gr), orc.forward(rows, gbar.astype(np.complex128)))
    say("projector VJP %.3e, adjoint VJP %.3e" % (e1, e2))
    assert e1 <= 1e-5 and e2 <= 1e-5


def c4_problem(K=10):
    cfg = W.CONFIGS["c4"]
    geom = W.config_geometry("c4")
    orc = Oracle(geom)
    s_true, idx = W.config_scene("c4")
    y = W.add_noise(orc.forward_sparse(np.arange(orc.M), idx, s_true[idx]), cfg["snr_db"], seed=cfg["seed"] + 2)
    y = y.astype(np.complex64).astype(np.complex128)
    steps = json.load(open(os.path.join(ROOT, "tests", "golden", "step_sizes.json")))["c4"]
    eta = (steps["eta"] * (1.0 + 0.05 * np.arange(K))).astype(np.float32).astype(np.float64)
    tau = (steps["lambda"] * eta).astype(np.float32).astype(np.float64)
    rows = W.config_rows("c4", K=K)
    return geom, orc, y, s_true, rows, eta, tau


def test_unrolled_spgm_gradient_c4(bd):
    """Unrolled SPGM on the 16 + 16 antenna, 32 f, 32x32x16 workload, 10 iterations of B = 2048:
    MSE loss to the true scene, gradients in s0, eta (10) and tau (10) against the FP64 oracle."""
    from paper_2509_00774_amd.autograd import unrolled_spgm
    geom, orc, y, s_true, rows, eta, tau = c4_problem()
    plan = bd.Plan(geom)
    s0 = 0.1 * W.random_complex(orc.N, seed=5)
    s0 = s0.astype(np.complex64).astype(np.complex128)
    s0_d = cdev(s0, grad=True)
    eta_d = torch.tensor(eta, dtype=torch.float64, device="cuda", requires_grad=True)
    tau_d = torch.tensor(tau, dtype=torch.float64, device="cuda", requires_grad=True)
    st = cdev(s_true)
    out = unrolled_spgm(plan, idev(rows), cdev(y), s0_d, eta_d, tau_d)
    loss = torch.mean(torch.abs(out - st) ** 2)
    loss.backward()
    say("oracle: unrolled forward and chain rule (K=%d, B=%d, N=%d)" % (rows.shape[0], rows.shape[1], orc.N))
    it = unrolled_forward(orc, rows, y, s0, eta, tau)
    sbar = 2.0 * (it[-1] - s_true) / orc.N
    s0bar, eta_bar, tau_bar = unrolled_vjp(orc, rows, y, it, eta, tau, sbar)
    e_out = rel_l2(host(out), it[-1])
    e_s = rel_l2(host(s0_d.grad), s0bar)
    e_eta = rel_l2(eta_d.grad.cpu().numpy(), eta_bar)
    e_tau = rel_l2(tau_d.grad.cpu().numpy(), tau_bar)
    say("unrolled c4: s_K %.3e, ds0 %.3e, deta %.3e, dtau %.3e" % (e_out, e_s, e_eta, e_tau))
    assert e_out <= 1e-5
    assert e_s <= 1e-4 and e_eta <= 1e-4 and e_tau <= 1e-4


def test_unrolled_checkpointing_is_exact(bd):
    """Recomputation from checkpoints reproduces the stored-iterate gradients bit for bit."""
    from paper_2509_00774_amd.autograd import unrolled_spgm
    geom, orc, y, s_true, rows, eta, tau = c4_problem(K=6)
    plan = bd.Plan(geom)
    grads = []
    for every in (1, 2, 6):
        s0_d = cdev(np.zeros(orc.N), grad=True)
        eta_d = torch.tensor(eta, dtype=torch.float64, device="cuda", requires_grad=True)
        tau_d = torch.tensor(tau, dtype=torch.float64, device="cuda", requires_grad=True)
        out = unrolled_spgm(plan, idev(rows), cdev(y), s0_d, eta_d, tau_d, checkpoint_every=every)
        torch.mean(torch.abs(out - cdev(s_true)) ** 2).backward()
        grads.append((host(s0_d.grad), eta_d.grad.cpu().numpy(), tau_d.grad.cpu().numpy()))
    for g in grads[1:]:
        for a, b in zip(grads[0], g):
            assert np.array_equal(a, b)


def test_unrolled_gradient_step_reduces_loss(bd):
    """A small gradient step on log(eta), log(tau) lowers the training loss (sanity of signs)."""
    from paper_2509_00774_amd.autograd import unrolled_spgm
    geom, orc, y, s_true, rows, eta, tau = c4_problem(K=6)
    plan = bd.Plan(geom)
    a = torch.zeros(rows.shape[0], dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.zeros(rows.shape[0], dtype=torch.float64, device="cuda", requires_grad=True)
    eta0 = torch.tensor(eta, device="cuda")
    tau0 = torch.tensor(tau, device="cuda")
    st = cdev(s_true)

    def loss_of(a, b):
        out = unrolled_spgm(plan, idev(rows), cdev(y), cdev(np.zeros(orc.N)), eta0 * torch.exp(a), tau0 * torch.exp(b))
        return torch.mean(torch.abs(out - st) ** 2)

    l0 = loss_of(a, b)
    l0.backward()
    with torch.no_grad():
        ga, gb = a.grad.clone(), b.grad.clone()
        step = 0.05 / float(torch.sqrt(torch.sum(ga ** 2) + torch.sum(gb ** 2)))
        l1 = loss_of(-step * ga, -step * gb)
    say("loss %.6e -> %.6e after one normalised gradient step" % (float(l0), float(l1)))
    assert float(l1) < float(l0)


def test_backward_from_kept_gradient_is_bitwise_the_recomputing_one(bd):
    """spgm_step_grad returns the iterate of spgm_step and the gradient A_B^H (A_B s - y_B) at the
    entering iterate; the backward step given that gradient (two entry passes) equals the one
    that recomputes it from y (four entry passes) bit for bit, and the gradient matches the
    oracle's (Eq. 6 without the 1/B)."""
    geom = W.config_geometry("c4")
    orc = Oracle(geom)
    plan = bd.Plan(geom)
    rows = W.draw_rows(orc.M, 2048, 1, seed=61)[0]
    y = W.random_complex(orc.M, seed=62).astype(np.complex64)
    s0 = (0.1 * W.random_complex(orc.N, seed=63)).astype(np.complex64)
    sbar_next = W.random_complex(orc.N, seed=64).astype(np.complex64)
    eta, tau = 8e-3, 2e-3
    r_d, y_d = idev(rows), cdev(y)
    a, b = cdev(s0), cdev(s0)
    g = torch.empty_like(a)
    plan.spgm_step_grad(r_d, y_d, a, eta, tau, g)
    plan.spgm_step(r_d, y_d, b, eta, tau)
    assert torch.equal(a, b)
    g_ref = orc.adjoint(rows, orc.forward(rows, s0.astype(np.complex128)) - y.astype(np.complex128)[rows])
    e_g = rel_l2(host(g), g_ref)
    outs = []
    for use_g in (True, False):
        sb = cdev(sbar_next)
        eb = torch.zeros(1, dtype=torch.float64, device="cuda")
        tb = torch.zeros(1, dtype=torch.float64, device="cuda")
        if use_g:
            plan.spgm_unrolled_vjp_step_g(r_d, cdev(s0), g, eta, tau, sb, sb, eb, tb)
        else:
            plan.spgm_unrolled_vjp_step(r_d, y_d, cdev(s0), eta, tau, sb, sb, eb, tb)
        torch.cuda.synchronize()
        outs.append((sb.cpu().numpy(), float(eb.item()), float(tb.item())))
    plan.close()
    say("step_grad: gradient rel_l2 %.3e vs oracle; kept-gradient backward bitwise equal: %s" % (
        e_g, np.array_equal(outs[0][0], outs[1][0])))
    assert e_g <= 1e-5
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1:] == outs[1][1:]
