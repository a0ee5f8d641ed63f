"""GPU parity of the parameter adjoint (pa_param_backward) and of the
torch.autograd.Function built on it.

theta_bar = sum_q (dP_q/dtheta)^T P_bar_q is compared with the oracle's
vector-Jacobian product (PyTorch reverse mode on the CPU, FP64), with
central finite differences of the GPU's FP64 forward (h = 1e-6), and with
the oracle's calibration-loss gradient.  Tolerances (normwise): FP64 1e-10,
FP32 1e-4."""
import numpy as np
import pytest
import torch

from oracle import calib, ncm
from paper_2510_00884_amd import synth
from gpu_util import close, need_gpu, rel, say

pytestmark = pytest.mark.gpu


def oracle_vjp(theta, F, Pbar, Av, p, h, L, has_bias=True):
    K, g = calib.feature_grads(F, Av)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    P = calib.stress_from_theta(th, torch.tensor(K), torch.tensor(g), p, h, L, has_bias)
    out, = torch.autograd.grad(P, th, torch.tensor(Pbar))
    return out.numpy(), P.detach().numpy()


@pytest.mark.parametrize("n_sv,h,L,bias", [(2, 16, 2, True), (2, 64, 3, True), (1, 32, 3, True),
                                           (0, 32, 2, False), (2, 32, 2, True)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_param_backward_vs_oracle(n_sv, h, L, bias, prec, tol):
    api = need_gpu()
    say("param_backward", n_sv, h, L, bias, prec)
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    theta = synth.micnn_params(p, h, L, seed=1, has_bias=bias)
    n = 700  # 43 full tiles of 16 and a ragged tail
    F = synth.sample_F(n, seed=3)
    Pbar = synth.rng(7).normal(size=(n, 3, 3))
    ref, Pref = oracle_vjp(theta, F, Pbar, Av, p, h, L, bias)
    gm = api.Model(theta, n_sv, h, L, A=Av, normalize=False, has_bias=bias)
    tb = api.param_backward(gm, torch.tensor(F, device="cuda"), torch.tensor(Pbar, device="cuda"), prec=prec)
    e = close(tb.cpu().numpy(), ref, tol, "theta_bar")
    say("  err", e)
    # the stress the forward returns for this model
    out = api.energy_stress_tangent(gm, torch.tensor(F, device="cuda"), prec="fp64", A=False, psi=False)
    close(out["P"].cpu().numpy().T.reshape(n, 3, 3), Pref, 1e-12, "P")


def test_param_backward_deterministic_and_empty():
    api = need_gpu()
    p = synth.num_inputs(2)
    theta = synth.micnn_params(p, 32, 2, seed=1)
    gm = api.Model(theta, 2, 32, 2, A=synth.structural_vectors(2))
    F = torch.tensor(synth.sample_F(5000, seed=1), device="cuda")
    Pb = torch.tensor(synth.rng(2).normal(size=(5000, 3, 3)), device="cuda")
    a = api.param_backward(gm, F, Pb, prec="fp64")
    b = api.param_backward(gm, F, Pb, prec="fp64")
    assert torch.equal(a, b)
    z = api.param_backward(gm, F[:0], Pb[:0], prec="fp64")
    assert torch.count_nonzero(z).item() == 0


def test_autograd_function_and_finite_differences():
    api = need_gpu()
    say("autograd + FD")
    n_sv, h, L = 2, 16, 3
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    theta = synth.micnn_params(p, h, L, seed=1)
    theta_ref = synth.micnn_params(p, h, L, seed=4)
    n = 512
    F = synth.sample_F(n, seed=3)
    Pref = ncm.stress_stiffness(F, ncm.model_from_theta(theta_ref, p, h, L, Av))["P"]
    Pt = Pref + 0.01 * np.sqrt(np.mean(Pref ** 2)) * synth.rng(5).normal(size=Pref.shape)
    Lo, go = calib.loss_and_grad(theta, F, Pt, Av, p, h, L)
    gm = api.Model(theta, n_sv, h, L, A=Av)
    th = torch.tensor(theta, device="cuda", requires_grad=True)
    Ft = torch.tensor(F, device="cuda")
    Ptt = torch.tensor(Pt, device="cuda")
    P = api.stress(th, Ft, gm, prec="fp64")
    loss = ((P - Ptt) ** 2).sum() / n
    loss.backward()
    assert abs(loss.item() - Lo) < 1e-12 * abs(Lo)
    close(th.grad.cpu().numpy(), go, 1e-10, "dL/dtheta")

    def gpu_loss(tv):
        m = api.Model(tv, n_sv, h, L, A=Av)
        Pg = api.energy_stress_tangent(m, Ft, prec="fp64", psi=False, A=False)["P"].t().reshape(n, 3, 3)
        return (((Pg - Ptt) ** 2).sum() / n).item()

    hstep = 1e-6
    idx = synth.rng(9).choice(theta.size, 12, replace=False)
    g = th.grad.cpu().numpy()
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = hstep
        fd = (gpu_loss(theta + e) - gpu_loss(theta - e)) / (2 * hstep)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, np.abs(g).max()), (i, fd, g[i])


@pytest.mark.parametrize("kind,n,n_sv,h,L", [("hex8", 3, 2, 32, 2), ("tet10", 2, 1, 16, 3)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_residual_loss_gradient(kind, n, n_sv, h, L, prec, tol):
    """Loss of eq. (loss) and its parameter gradient through the GPU path
    (tangent build, loss cotangent, residual cotangent, parameter adjoint)
    against the oracle's reverse-mode gradient."""
    api = need_gpu()
    say("residual loss gradient", kind, n, n_sv, h, L, prec)
    X, conn, par = (synth.hex_mesh if kind == "hex8" else synth.tet10_mesh)(n)
    u = synth.displacement_modes(X, 1.0 / n, seed=0)
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    theta = synth.micnn_params(p, h, L, seed=1)
    grp = synth.reaction_groups(X)
    R = np.array([0.03, -0.02])
    Lo, go, ro = calib.residual_loss_and_grad(theta, X, conn, u, grp, R, Av, p, h, L)
    gm = api.Model(theta, n_sv, h, L, A=Av, normalize=False, algorithm="adjoint")
    mesh = api.FEMesh(X, conn, colour=par)
    loss, tb = api.residual_loss_and_grad(gm, mesh, torch.tensor(u, device="cuda"),
                                          torch.tensor(grp, device="cuda"), R, prec=prec)
    assert abs(loss.item() - Lo) <= (1e-12 if prec == "fp64" else 1e-5) * abs(Lo)
    close(tb.cpu().numpy(), go, tol, "theta_bar")


def test_residual_loss_cotangent_and_empty_groups():
    """pa_residual_loss against the definition on a random residual, with and
    without reaction boundaries."""
    api = need_gpu()
    X, _, _ = synth.hex_mesh(4)
    grp = synth.reaction_groups(X)
    r = synth.rng(3).normal(size=grp.size)
    R = np.array([0.5, -1.5])
    loss, rbar = api.residual_loss(torch.tensor(r, device="cuda"), torch.tensor(grp, device="cuda"), R)
    L_ref = np.sum(r[grp == -1] ** 2) + sum((R[b] - r[grp == b].sum()) ** 2 for b in range(2))
    rb_ref = np.where(grp == -1, 2 * r, 0.0)
    for b in range(2):
        rb_ref[grp == b] = -2 * (R[b] - r[grp == b].sum())
    assert abs(loss.item() - L_ref) <= 1e-13 * L_ref
    close(rbar.cpu().numpy(), rb_ref, 1e-14, "r_bar")
    free = np.full(grp.size, -1, dtype=np.int32)
    loss0, rbar0 = api.residual_loss(torch.tensor(r, device="cuda"), torch.tensor(free, device="cuda"), [])
    assert abs(loss0.item() - np.sum(r ** 2)) <= 1e-13 * np.sum(r ** 2)
    close(rbar0.cpu().numpy(), 2 * r, 1e-15, "r_bar free")


def test_autograd_two_thetas_in_one_graph():
    """Two stress() calls of one model with different parameters in one graph,
    and the model given a third parameter vector before backward(): each
    gradient is the oracle's VJP at the theta its own forward used."""
    api = need_gpu()
    say("autograd two thetas")
    n_sv, h, L = 2, 16, 2
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    th1 = synth.micnn_params(p, h, L, seed=1)
    th2 = synth.micnn_params(p, h, L, seed=4)
    n = 300
    F = synth.sample_F(n, seed=3)
    W1 = synth.rng(11).normal(size=(n, 3, 3))
    W2 = synth.rng(12).normal(size=(n, 3, 3))
    gm = api.Model(th1, n_sv, h, L, A=Av, algorithm="adjoint")
    Ft = torch.tensor(F, device="cuda")
    t1 = torch.tensor(th1, device="cuda", requires_grad=True)
    t2 = torch.tensor(th2, device="cuda", requires_grad=True)
    P1 = api.stress(t1, Ft, gm, prec="fp64")
    P2 = api.stress(t2, Ft, gm, prec="fp64")
    gm.set_params(synth.micnn_params(p, h, L, seed=9))  # the model moves on before backward
    loss = (P1 * torch.tensor(W1, device="cuda")).sum() + (P2 * torch.tensor(W2, device="cuda")).sum()
    loss.backward()
    ref1, Pr1 = oracle_vjp(th1, F, W1, Av, p, h, L)
    ref2, Pr2 = oracle_vjp(th2, F, W2, Av, p, h, L)
    close(P1.detach().cpu().numpy(), Pr1, 1e-12, "P(theta1)")
    close(P2.detach().cpu().numpy(), Pr2, 1e-12, "P(theta2)")
    close(t1.grad.cpu().numpy(), ref1, 1e-10, "grad theta1")
    close(t2.grad.cpu().numpy(), ref2, 1e-10, "grad theta2")


def test_binding_rejects_bad_tensors_before_launch():
    """A float32, host or wrongly sized tensor is refused on the host with a
    ValueError (nothing reaches a kernel)."""
    api = need_gpu()
    p = synth.num_inputs(2)
    gm = api.Model(synth.micnn_params(p, 16, 2, seed=1), 2, 16, 2, A=synth.structural_vectors(2))
    F = torch.tensor(synth.sample_F(64, seed=1), device="cuda")
    for bad in (F.float(), F.cpu()):
        with pytest.raises(ValueError):
            api.energy_stress_tangent(gm, bad)
        with pytest.raises(ValueError):
            api.param_backward(gm, bad, F)
    with pytest.raises(ValueError):
        api.param_backward(gm, F, F[:10])
    X, conn, par = synth.hex_mesh(2)
    mesh = api.FEMesh(X, conn, colour=par)
    u = torch.zeros(3 * mesh.n_nodes, device="cuda", dtype=torch.float64)
    for bad in (u.float(), u.cpu(), u[:-3]):
        with pytest.raises(ValueError):
            api.tangent_build(gm, mesh, bad)
    grp = torch.full((3 * mesh.n_nodes,), -1, dtype=torch.int32, device="cuda")
    grp[5] = 2  # only two reaction forces below
    with pytest.raises(ValueError):
        api.residual_loss(u, grp, [0.0, 1.0])
