"""GPU parity across network sizes outside the mesh configurations: widths
up to 8 (FP64 and FP32 on the vector ALUs, one point per lane; the BF16
modes and the forward mode zero-padded to one 16-row matrix-core tile),
widths 9..16 (padded) and four hidden layers, against the FP64 oracle on
seeded inputs with full 16-point tiles and a ragged tail.  Tolerances (normwise): FP64 1e-12
for Psi, P and the tangent, 1e-10 for the parameter adjoint; FP32 network
1e-5 (tangent) and 1e-4 (parameter adjoint)."""
import numpy as np
import pytest
import torch

from oracle import calib, fe, ncm
from paper_2510_00884_amd import synth
from paper_2510_00884_amd._lib import PaError
from gpu_util import close, need_gpu, rel, say

pytestmark = pytest.mark.gpu

# (n_sv, width, hidden layers)
SIZES = [(2, 8, 2), (1, 4, 3), (0, 2, 2), (2, 1, 2), (2, 5, 3), (1, 3, 2), (2, 8, 4), (2, 12, 2), (2, 16, 4),
         (1, 32, 4), (2, 64, 4)]


def build(api, n_sv, h, L, normalize=True, algorithm="adjoint", has_bias=True):
    p = synth.num_inputs(n_sv)
    theta = synth.micnn_params(p, h, L, seed=1, has_bias=has_bias)
    Av = synth.structural_vectors(n_sv)
    gm = api.Model(theta, n_sv, h, L, A=Av, normalize=normalize, algorithm=algorithm, has_bias=has_bias)
    om = ncm.model_from_theta(theta, p, h, L, Av, normalize=normalize, has_bias=has_bias)
    return gm, om, theta, p, Av


def unpack(out, n):
    return (out["psi"].cpu().numpy(), out["P"].cpu().numpy().T.reshape(n, 3, 3),
            out["A"].cpu().numpy().T.reshape(n, 3, 3, 3, 3))


@pytest.mark.parametrize("n_sv,h,L", SIZES)
def test_adjoint_fp64_sizes(n_sv, h, L):
    api = need_gpu()
    say("sizes adjoint fp64", n_sv, h, L)
    gm, om, *_ = build(api, n_sv, h, L)
    n = 1000
    F = synth.sample_F(n, seed=0)
    psi, P, A = unpack(api.energy_stress_tangent(gm, torch.tensor(F, device="cuda"), prec="fp64"), n)
    ref = ncm.stress_stiffness(F, om)
    close(psi, ref["psi"], 1e-12, "psi")
    close(P, ref["P"], 1e-12, "P")
    close(A, ref["A"], 1e-12, "A")


@pytest.mark.parametrize("n_sv,h,L", [(2, 8, 2), (2, 32, 4), (1, 2, 3), (2, 6, 4), (2, 64, 3), (1, 32, 3), (0, 16, 3)])
def test_adjoint_fp32_sizes(n_sv, h, L):
    api = need_gpu()
    say("sizes adjoint fp32", n_sv, h, L)
    gm, om, *_ = build(api, n_sv, h, L)
    n = 1000
    F = synth.sample_F(n, seed=5)
    psi, P, A = unpack(api.energy_stress_tangent(gm, torch.tensor(F, device="cuda"), prec="fp32"), n)
    ref = ncm.stress_stiffness(F, om)
    e = (rel(psi, ref["psi"]), rel(P, ref["P"]), rel(A, ref["A"]))
    say("  errors psi/P/A", e)
    assert max(e) < 1e-5


@pytest.mark.parametrize("n_sv,h,L", [(2, 8, 2), (1, 4, 3)])
def test_forward_mode_narrow(n_sv, h, L):
    """The forward-mode kernel (Alg. 4) on a zero-padded narrow network."""
    api = need_gpu()
    say("sizes forward fp64", n_sv, h, L)
    gm, om, *_ = build(api, n_sv, h, L, algorithm="forward")
    n = 1000
    F = synth.sample_F(n, seed=0)
    psi, P, A = unpack(api.energy_stress_tangent(gm, torch.tensor(F, device="cuda"), prec="fp64"), n)
    ref = ncm.stress_stiffness(F, om)
    close(psi, ref["psi"], 1e-12, "psi")
    close(A, ref["A"], 1e-12, "A")


def test_depth4_forward_mode_and_bf16_unsupported():
    api = need_gpu()
    say("sizes depth 4 unsupported paths")
    F = torch.tensor(synth.sample_F(32, seed=5), device="cuda")
    gm, *_ = build(api, 2, 16, 4, algorithm="forward")
    with pytest.raises(PaError):
        api.energy_stress_tangent(gm, F, prec="fp64")
    gm, *_ = build(api, 2, 16, 4, algorithm="adjoint")
    with pytest.raises(PaError):
        api.energy_stress_tangent(gm, F, prec="bf16")


@pytest.mark.parametrize("n_sv,h,L,bias", [(2, 8, 2, True), (1, 4, 3, False), (2, 16, 4, True), (1, 32, 4, True)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_param_backward_sizes(n_sv, h, L, bias, prec, tol):
    api = need_gpu()
    say("sizes param_backward", n_sv, h, L, bias, prec)
    gm, om, theta, p, Av = build(api, n_sv, h, L, normalize=False, has_bias=bias)
    n = 700
    F = synth.sample_F(n, seed=3)
    Pbar = synth.rng(7).normal(size=(n, 3, 3))
    K, g = calib.feature_grads(F, Av)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    Pt = calib.stress_from_theta(th, torch.tensor(K), torch.tensor(g), p, h, L, bias)
    ref, = torch.autograd.grad(Pt, th, torch.tensor(Pbar))
    tb = api.param_backward(gm, torch.tensor(F, device="cuda"), torch.tensor(Pbar, device="cuda"), prec=prec)
    assert tb.numel() == synth.num_params(p, h, L, bias)
    e = close(tb.cpu().numpy(), ref.numpy(), tol, "theta_bar")
    say("  err", e)


def test_tangent_build_depth4():
    """A hex8 tangent build with a four-layer network (adjoint form)."""
    api = need_gpu()
    say("sizes tangent build depth 4")
    n = 3
    X, conn, par = synth.hex_mesh(n)
    u = synth.displacement_modes(X, 1.0 / n, seed=0)
    gm, om, *_ = build(api, 2, 16, 4)
    mesh = api.FEMesh(X, conn, colour=par)
    cperm = conn[mesh.perm]
    dNdX, w, _ = fe.geometry(X, cperm)
    r_ref, K_ref, _ = fe.element_residual_stiffness(u, cperm, dNdX, w, om)
    rg, Kg = fe.assemble(cperm, r_ref, K_ref, X.shape[0])
    r, vals = api.tangent_build(gm, mesh, torch.tensor(u, device="cuda"), prec="fp64")
    close(r.cpu().numpy(), rg, 1e-12, "r")
    close(vals.cpu().numpy(), Kg.data, 1e-12, "vals")


@pytest.mark.parametrize("n_sv,h,L,prec", [(2, 32, 2, "fp64"), (2, 64, 3, "bf16"), (2, 8, 2, "fp32"),
                                            (1, 16, 3, "fp32")])
def test_batched_material_call_is_bitwise_batch_independent(n_sv, h, L, prec):
    """pa_energy_stress_tangent_batched: batches of 1,000 (ragged: not a
    multiple of the 16-point tile), 4,096 and 16,384 points give outputs
    bitwise equal to the one-launch call, with a workspace of one batch."""
    api = need_gpu()
    say("batched material call", n_sv, h, L, prec)
    gm, om, *_ = build(api, n_sv, h, L)
    n = 40_000
    Ft = torch.tensor(synth.sample_F(n, seed=21), device="cuda")
    ref = api.energy_stress_tangent(gm, Ft, prec=prec)
    for b in (1000, 4096, 16384, n + 7):
        got = api.energy_stress_tangent(gm, Ft, prec=prec, batch=b)
        for k in ("psi", "P", "A"):
            assert torch.equal(got[k], ref[k]), (b, k)
    with pytest.raises(PaError):
        api.energy_stress_tangent(gm, Ft, prec=prec, batch=0)


@pytest.mark.parametrize("n_sv,h,L", [(2, 16, 2), (2, 32, 2), (1, 32, 3), (2, 64, 2), (2, 64, 3), (2, 64, 4), (0, 16, 4)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16_corr"])
def test_stress_only_sizes(n_sv, h, L, prec):
    """Value and gradient without the tangent (the one-wave stress kernel, and
    the FP32 pass of BF16 + correction) against the FP64 oracle, 2,000 points
    (125 full tiles) plus a ragged tail of 7: FP64 1e-12 on Psi and P; FP32
    and the corrected BF16 run 1e-5 (their value and gradient come from the
    FP32 pass)."""
    api = need_gpu()
    say("sizes stress-only", prec, n_sv, h, L)
    gm, om, *_ = build(api, n_sv, h, L)
    n = 2007
    F = synth.sample_F(n, seed=11)
    if prec == "bf16_corr" and L > 3:  # the all-BF16 pass serves two and three hidden layers
        with pytest.raises(PaError):
            api.energy_stress_tangent(gm, torch.tensor(F, device="cuda"), prec=prec, A=False)
        return
    out = api.energy_stress_tangent(gm, torch.tensor(F, device="cuda"), prec=prec, A=False)
    psi, P = out["psi"].cpu().numpy(), out["P"].cpu().numpy().T.reshape(n, 3, 3)
    ref = ncm.stress_stiffness(F, om)
    tol = 1e-12 if prec == "fp64" else 1e-5
    e = (rel(psi, ref["psi"]), rel(P, ref["P"]))
    say("  errors psi/P", e)
    assert max(e) < tol


TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 2e-2, "bf16_corr": 2e-2}


@pytest.mark.parametrize("n", [1, 17])
@pytest.mark.parametrize("h,L", [(32, 2), (64, 3)])
@pytest.mark.parametrize("algorithm", ["adjoint", "forward"])
def test_tiny_batches_every_precision(n, h, L, algorithm):
    """One point, and one full tile plus one: every network kernel (persistent
    grids of a single workgroup, waves with no tile) at every precision, with
    and without the tangent, against the oracle at the precision's tolerance
    (BF16 + correction: P at the FP32 tolerance)."""
    api = need_gpu()
    gm, om, *_ = build(api, 2, h, L, algorithm=algorithm)
    F = synth.sample_F(n, seed=21)
    ref = ncm.stress_stiffness(F, om)
    Ft = torch.tensor(F, device="cuda")
    for prec, tol in TOL.items():
        say("tiny batch", algorithm, prec, n, h, L)
        psi, P, A = unpack(api.energy_stress_tangent(gm, Ft, prec=prec), n)
        ptol = 1e-5 if prec == "bf16_corr" else tol
        assert rel(P, ref["P"]) < ptol and rel(A, ref["A"]) < tol
        out = api.energy_stress_tangent(gm, Ft, prec=prec, A=False)
        P2 = out["P"].cpu().numpy().T.reshape(n, 3, 3)
        assert rel(P2, ref["P"]) < ptol
