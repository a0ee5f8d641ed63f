"""Pins of the oracle's constitutive model against facts that do not come from
the oracle itself: closed-form energies, complex-step and finite-difference
derivatives, objectivity, material symmetry, the reference state, tensor
symmetries and an independent PyTorch autograd route."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import ncm
from paper_2510_00884_amd import synth

HERE = os.path.dirname(__file__)
FACTS = json.load(open(os.path.join(HERE, "golden", "paper_facts.json")))
EPS_CS = 1e-20


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def make_model(n_sv=2, h=8, L=3, seed=1, normalize=False, sigma=0.3):
    p = synth.num_inputs(n_sv)
    theta = synth.micnn_params(p, h, L, seed=seed, sigma=sigma)
    return ncm.model_from_theta(theta, p, h, L, synth.structural_vectors(n_sv), normalize=normalize)


def rand_F(n, seed=0, sigma=0.15):
    return synth.sample_F(n, seed=seed, sigma=sigma)


def cs_grad(fun, X, eps=EPS_CS):
    """Complex-step gradient of a batched scalar function of (n, 3, 3)."""
    n = X.shape[0]
    g = np.empty((n, 3, 3))
    for i in range(3):
        for J in range(3):
            Xc = X.astype(complex)
            Xc[:, i, J] += 1j * eps
            g[:, i, J] = np.imag(fun(Xc)) / eps
    return g


def cs_jac(fun, X, eps=EPS_CS):
    """Complex-step Jacobian of a batched (n,3,3)->(n,3,3) map: out[n,i,J,k,L]."""
    n = X.shape[0]
    out = np.empty((n, 3, 3, 3, 3))
    for k in range(3):
        for L in range(3):
            Xc = X.astype(complex)
            Xc[:, k, L] += 1j * eps
            out[:, :, :, k, L] = np.imag(fun(Xc)) / eps
    return out


# ---------------------------------------------------------------- structure
def test_param_count_matches_paper_table():
    f = FACTS["micnn_3x16_param_count"]
    assert synth.num_params(f["inputs"], f["width"], f["hidden_layers"], has_bias=False) == f["value"]


def test_features_vanish_at_identity():
    for n_sv in (0, 1, 2):
        K = ncm.features(np.eye(3)[None], synth.structural_vectors(n_sv))
        np.testing.assert_allclose(K, 0.0, atol=1e-15)
    assert FACTS["kinematic_layer_at_identity"]["value"] == [0.0, 0.0, 0.0]


def test_invariants_closed_form_diagonal():
    lam = np.array([1.3, 0.8, 1.1])
    F = np.diag(lam)[None]
    inv = ncm.invariants(F, synth.structural_vectors(2))
    l2 = lam ** 2
    assert np.isclose(inv["I1"][0], l2.sum())
    assert np.isclose(inv["I2"][0], l2[0] * l2[1] + l2[1] * l2[2] + l2[0] * l2[2])
    assert np.isclose(inv["I3"][0], l2.prod())
    # pairs (0,0), (0,1), (1,1): A^i.C A^j and A^i.C^2 A^j with A = e1, e2
    np.testing.assert_allclose(inv["I4"], [[l2[0]], [0.0], [l2[1]]])
    np.testing.assert_allclose(inv["I5"], [[l2[0] ** 2], [0.0], [l2[1] ** 2]])
    ex = FACTS["isochoric_exponents"]["value"]
    K = ncm.features(F, synth.structural_vectors(2))[0]
    J = lam.prod()
    assert np.isclose(K[0], l2.sum() * J ** (2 * ex["I1"]) - 3)
    assert np.isclose(K[3], l2[0] * J ** (2 * ex["I4"]) - 1)
    assert np.isclose(K[6], l2[0] ** 2 * J ** (2 * ex["I5"]) - 1)


# ---------------------------------------------------------------- network derivatives (eq. icnn)
def test_single_unit_closed_form():
    """N = a softplus(w.K + c) + b.K has closed-form gradient and Hessian."""
    r = np.random.default_rng(3)
    p = 5
    w = r.normal(size=(1, p)); c = r.normal(size=1); a = np.abs(r.normal(size=1)); b = r.normal(size=p)
    K = r.normal(size=(7, p))
    N, dN, d2N = ncm.micnn(K, [(w, None, c)], a, b)
    y = K @ w[0] + c[0]
    s = 1 / (1 + np.exp(-y))
    np.testing.assert_allclose(N, a[0] * np.log1p(np.exp(y)) + K @ b, rtol=1e-14)
    np.testing.assert_allclose(dN, a[0] * s[:, None] * w + b, rtol=1e-14)
    np.testing.assert_allclose(d2N, a[0] * (s * (1 - s))[:, None, None] * np.outer(w, w)[None], rtol=1e-13)


@pytest.mark.parametrize("n_sv,h,L", [(0, 6, 2), (1, 16, 2), (2, 8, 3), (2, 4, 4)])
def test_network_derivatives_by_complex_step(n_sv, h, L):
    m = make_model(n_sv, h, L)
    p = m.p
    K = np.random.default_rng(5).normal(scale=0.4, size=(11, p))
    N, dN, d2N = ncm.micnn(K, m.hidden, m.a, m.b)
    np.testing.assert_allclose(N, ncm.micnn_value(K, m.hidden, m.a, m.b), rtol=1e-14)
    for j in range(p):
        Kc = K.astype(complex); Kc[:, j] += 1j * EPS_CS
        np.testing.assert_allclose(np.imag(ncm.micnn_value(Kc, m.hidden, m.a, m.b)) / EPS_CS, dN[:, j], rtol=1e-12)
        _, dNc, _ = ncm.micnn(Kc, m.hidden, m.a, m.b)
        np.testing.assert_allclose(np.imag(dNc) / EPS_CS, d2N[:, :, j], rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(d2N, np.swapaxes(d2N, 1, 2), rtol=1e-14, atol=1e-15)


def test_micnn_convex_monotone_with_nonneg_weights():
    """Non-negative A^k, B^k and a convex non-decreasing activation give a convex,
    non-decreasing network (App. B.2): Hessian PSD, gradient >= 0."""
    m = make_model(2, 16, 3)
    K = np.random.default_rng(8).normal(size=(50, m.p))
    _, dN, d2N = ncm.micnn(K, m.hidden, m.a, m.b)
    assert (dN >= 0).all()
    ev = np.linalg.eigvalsh(d2N)
    assert (ev >= -1e-10 * np.abs(ev).max()).all()


# ---------------------------------------------------------------- closed-form energies
def nh_closed(F, mu, kap):
    """Textbook compressible Neo-Hookean: Psi = mu/2 (I1~ - 3) + kap/2 (J-1)^2,
    P and dP/dF written out by hand."""
    J = np.linalg.det(F)
    Fi = np.linalg.inv(F)
    FiT = np.swapaxes(Fi, 1, 2)
    I1 = np.einsum("nij,nij->n", F, F)
    c = J ** (-2.0 / 3.0)
    psi = 0.5 * mu * (I1 * c - 3) + 0.5 * kap * (J - 1) ** 2
    P = (mu * c)[:, None, None] * (F - (I1 / 3)[:, None, None] * FiT) + (kap * (J - 1) * J)[:, None, None] * FiT
    d = np.eye(3)
    A = (mu * c)[:, None, None, None, None] * (
        np.einsum("ik,JL->iJkL", d, d)[None]
        - 2.0 / 3.0 * np.einsum("niJ,nLk->niJkL", F, Fi)
        - 2.0 / 3.0 * np.einsum("nkL,nJi->niJkL", F, Fi)
        + (2.0 / 9.0) * I1[:, None, None, None, None] * np.einsum("nJi,nLk->niJkL", Fi, Fi)
        + (1.0 / 3.0) * I1[:, None, None, None, None] * np.einsum("nJk,nLi->niJkL", Fi, Fi))
    A += kap * ((2 * J - 1) * J)[:, None, None, None, None] * np.einsum("nJi,nLk->niJkL", Fi, Fi)
    A -= kap * ((J - 1) * J)[:, None, None, None, None] * np.einsum("nJk,nLi->niJkL", Fi, Fi)
    return psi, P, A


@pytest.mark.parametrize("n_sv", [0, 2])
def test_neo_hookean_reduction(n_sv):
    """a = 0 and b = (mu/2, 0, kap/2, 0, ...) reduce the network exactly to NH."""
    mu, kap = 1.7, 5.3
    m = make_model(n_sv, 8, 2)
    m.a = np.zeros_like(m.a)
    b = np.zeros(m.p); b[0] = mu / 2; b[2] = kap / 2
    m.b = b
    F = rand_F(64, seed=2)
    out = ncm.stress_stiffness(F, m)
    psi, P, A = nh_closed(F, mu, kap)
    np.testing.assert_allclose(out["psi"], psi, rtol=1e-13, atol=1e-14)
    assert rel(out["P"], P) < 1e-13
    assert rel(out["A"], A) < 1e-13


def test_gent_thomas_inner_function():
    """Gent-Thomas (eq. gt) through the I2~ feature (reading R13): Psi =
    0.5 K1 + log(((K2 + 3^1.5)^(2/3))/3) + K3; stress and stiffness from the
    push-forward route against complex-step derivatives of Psi written
    directly in F."""
    def psi_F(F):
        J = ncm._det3(F)
        C = np.einsum("nki,nkj->nij", F, F)
        I1 = np.einsum("nii->n", C)
        I2 = 0.5 * (I1 ** 2 - np.einsum("nij,nji->n", C, C))
        I1t = I1 * (J * J) ** (-1.0 / 3.0)
        I2t = I2 * (J * J) ** (-2.0 / 3.0)
        return 0.5 * (I1t - 3) + np.log(I2t / 3) + (J - 1) ** 2

    m = ncm.ClosedModel(ncm.gent_thomas, (0.5, 1.0, 1.0), np.zeros((0, 3)))
    F = rand_F(40, seed=4)
    out = ncm.stress_stiffness(F, m)
    np.testing.assert_allclose(out["psi"], psi_F(F), rtol=1e-13, atol=1e-14)
    assert rel(out["P"], cs_grad(psi_F, F)) < 1e-12
    Pfun = lambda X: ncm.stress_stiffness(X, m)["P"]
    assert rel(out["A"], cs_jac(Pfun, F)) < 1e-12


def cann_theta(p, seed=3):
    return np.abs(np.random.default_rng(seed).normal(0.0, 0.3, size=8 * p))


@pytest.mark.parametrize("n_sv", [0, 2])
def test_cann_derivatives_by_complex_step(n_sv):
    """Gradient and (diagonal) Hessian of the CANN (eq. cann-chain-rule)
    against complex-step derivatives of its value (eq. cann-def)."""
    p = ncm.num_inputs(n_sv)
    th = cann_theta(p)
    K = np.abs(np.random.default_rng(5).normal(0.0, 0.4, size=(30, p)))
    N, dN, d2N = ncm.cann(K, th)
    h = 1e-20
    for m in range(p):
        E = np.zeros(p); E[m] = h
        Nc, dNc, _ = ncm.cann(K + 1j * E, th)
        assert np.max(np.abs(np.imag(Nc) / h - dN[:, m])) <= 1e-13 * max(1.0, np.abs(dN).max())
        assert np.max(np.abs(np.imag(dNc) / h - d2N[:, :, m])) <= 1e-13 * max(1.0, np.abs(d2N).max())
    off = d2N.copy()
    off[:, np.arange(p), np.arange(p)] = 0.0
    assert np.all(off == 0.0)


def test_cann_neo_hookean_reduction():
    """A CANN with only the linear power-1 branches of K1 (w1 w2 = mu/2) and
    K3 (w1 w2 = kappa/2) is the Neo-Hookean energy exactly."""
    mu, kap = 1.7, 5.3
    th = np.zeros((3, 4, 2))
    th[0, 0] = (2.0, mu / 4)
    th[2, 0] = (0.5, kap)
    m = ncm.ClosedModel(ncm.cann, th.reshape(-1), np.zeros((0, 3)))
    F = rand_F(64, seed=2)
    out = ncm.stress_stiffness(F, m)
    psi, P, A = nh_closed(F, mu, kap)
    np.testing.assert_allclose(out["psi"], psi, rtol=1e-13, atol=1e-14)
    assert rel(out["P"], P) < 1e-13
    assert rel(out["A"], A) < 1e-13


def test_cann_stress_and_tangent_by_complex_step():
    """P and AA of an orthotropic CANN with the normalised reference state
    against complex-step derivatives of Psi written in F."""
    Av = np.eye(3)[:2]
    p = ncm.num_inputs(2)
    th = cann_theta(p, seed=8)
    m = ncm.ClosedModel(ncm.cann, th, Av, normalize=True)

    def psi_F(F):
        N, _, _ = m.inner(ncm.features(F, Av))
        return N

    F = rand_F(30, seed=6)
    out = ncm.stress_stiffness(F, m)
    np.testing.assert_allclose(out["psi"], psi_F(F), rtol=1e-13, atol=1e-14)
    assert rel(out["P"], cs_grad(psi_F, F)) < 1e-12
    Pfun = lambda X: ncm.stress_stiffness(X, m)["P"]
    assert rel(out["A"], cs_jac(Pfun, F)) < 1e-12
    I = np.eye(3)[None]
    ref = ncm.stress_stiffness(I, m)
    assert abs(ref["psi"][0]) < 1e-14 and np.abs(ref["P"]).max() < 1e-14


# ---------------------------------------------------------------- derivative routes
@pytest.mark.parametrize("n_sv,normalize", [(1, False), (2, True), (2, False)])
def test_stress_and_tangent_by_complex_step(n_sv, normalize):
    m = make_model(n_sv, 8, 3, normalize=normalize)
    F = rand_F(32, seed=7)
    out = ncm.stress_stiffness(F, m)
    np.testing.assert_allclose(out["psi"], ncm.energy(F, m), rtol=1e-12, atol=1e-13)
    assert rel(out["P"], cs_grad(lambda X: ncm.energy(X, m), F)) < 1e-12
    Pfun = lambda X: ncm.stress_stiffness(X, m)["P"]
    assert rel(out["A"], cs_jac(Pfun, F)) < 1e-12


def test_central_differences():
    m = make_model(2, 8, 2, normalize=True)
    F = rand_F(8, seed=9)
    out = ncm.stress_stiffness(F, m)
    h = 1e-6
    Pfd = np.empty_like(out["P"]); Afd = np.empty_like(out["A"])
    for i in range(3):
        for J in range(3):
            E = np.zeros((3, 3)); E[i, J] = h
            Pfd[:, i, J] = (ncm.energy(F + E, m) - ncm.energy(F - E, m)) / (2 * h)
            Afd[:, :, :, i, J] = (ncm.stress_stiffness(F + E, m)["P"] - ncm.stress_stiffness(F - E, m)["P"]) / (2 * h)
    assert rel(out["P"], Pfd) < 1e-7
    assert rel(out["A"], Afd) < 1e-7


def test_torch_autograd_hessian():
    """The paper's non-CGO baseline: reverse-mode AD of the energy (written in
    torch) gives the same P and dP/dF as the push-forward route."""
    n_sv, h, L = 2, 8, 3
    p = synth.num_inputs(n_sv)
    theta = synth.micnn_params(p, h, L, seed=11)
    m = ncm.model_from_theta(theta, p, h, L, synth.structural_vectors(n_sv))
    Av = torch.tensor(synth.structural_vectors(n_sv))
    hid, a, b = synth.unpack_params(theta, p, h, L)

    def psi_t(F):
        C = F.T @ F
        I1 = torch.trace(C)
        I2 = 0.5 * (I1 ** 2 - torch.trace(C @ C))
        J = torch.det(F)
        I3 = J * J
        feats = [I1 * I3 ** (-1 / 3) - 3, (I2 * I3 ** (-2 / 3)) ** 1.5 - 3 ** 1.5, (J - 1) ** 2]
        prs = ncm.pairs(n_sv)
        for (i, j) in prs:
            feats.append(Av[i] @ C @ Av[j] * I3 ** (-1 / 3) - Av[i] @ Av[j])
        for (i, j) in prs:
            feats.append(Av[i] @ C @ C @ Av[j] * I3 ** (-2 / 3) - Av[i] @ Av[j])
        K = torch.stack(feats)
        z = K
        for (A_, B_, c_) in hid:
            y = torch.tensor(A_) @ z + torch.tensor(c_)
            if B_ is not None:
                y = y + torch.tensor(B_) @ K
            z = torch.clamp(y, min=0.0) + torch.log1p(torch.exp(-torch.abs(y)))  # exact softplus
        return torch.tensor(a) @ z + torch.tensor(b) @ K

    F = rand_F(16, seed=12)
    out = ncm.stress_stiffness(F, m)
    for n in range(F.shape[0]):
        Ft = torch.tensor(F[n], requires_grad=True)
        P = torch.autograd.functional.jacobian(psi_t, Ft)
        H = torch.autograd.functional.hessian(psi_t, Ft)
        assert rel(out["P"][n], P.numpy()) < 1e-12
        assert rel(out["A"][n], H.numpy()) < 1e-12


# ---------------------------------------------------------------- invariance properties
def rot(axis, th):
    axis = np.asarray(axis, float); axis /= np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K


def test_objectivity():
    m = make_model(2, 8, 3, normalize=True)
    F = rand_F(24, seed=13)
    Q = synth.sample_F(1, seed=99, sigma=0.0)[0]  # pure rotation (sigma = 0)
    assert np.allclose(Q @ Q.T, np.eye(3)) and np.isclose(np.linalg.det(Q), 1)
    a = ncm.stress_stiffness(F, m)
    b = ncm.stress_stiffness(np.einsum("ij,njK->niK", Q, F), m)
    np.testing.assert_allclose(b["psi"], a["psi"], rtol=1e-13, atol=1e-14)
    assert rel(b["P"], np.einsum("ij,njK->niK", Q, a["P"])) < 1e-13
    assert rel(b["A"], np.einsum("ip,kr,npJrL->niJkL", Q, Q, a["A"])) < 1e-13


def test_material_symmetry():
    F = rand_F(24, seed=14)
    m1 = make_model(1, 8, 2, normalize=True)   # transversely isotropic about e1
    base = ncm.energy(F, m1)
    for th in (0.3, 1.1, 2.5):
        np.testing.assert_allclose(ncm.energy(F @ rot([1, 0, 0], th), m1), base, rtol=1e-12, atol=1e-13)
    m2 = make_model(2, 8, 2, normalize=True)   # e1, e2 with the mixed I4,12 / I5,12 inputs
    base = ncm.energy(F, m2)
    # the half-turn about e3 maps (e1, e2) -> (-e1, -e2): every pair product is kept
    np.testing.assert_allclose(ncm.energy(F @ rot([0, 0, 1], np.pi), m2), base, rtol=1e-12, atol=1e-13)
    # a half-turn about e1 flips the sign of the mixed inputs, so it is not a symmetry
    assert not np.allclose(ncm.energy(F @ rot([1, 0, 0], np.pi), m2), base)
    # covariance: Psi(F Q; A) = Psi(F; Q A) for any rotation Q
    Q = rot([1, 2, 3], 0.9)
    m3 = make_model(2, 8, 2, normalize=True)
    m3.Avec = (Q @ m2.Avec.T).T
    np.testing.assert_allclose(ncm.energy(F @ Q, m2), ncm.energy(F, m3), rtol=1e-12, atol=1e-13)


def test_reference_state():
    m = make_model(2, 16, 3, normalize=True)
    out = ncm.stress_stiffness(np.eye(3)[None], m)
    assert abs(out["psi"][0]) < 1e-14
    assert np.abs(out["P"]).max() < 1e-13
    # isotropic NH: A(I) is the Lame tensor, lambda = kap - 2 mu / 3
    mu, kap = 2.0, 7.0
    mn = make_model(0, 4, 2)
    mn.a = np.zeros_like(mn.a); mn.b = np.array([mu / 2, 0, kap / 2])
    A = ncm.stress_stiffness(np.eye(3)[None], mn)["A"][0]
    d = np.eye(3)
    lame = mu * (np.einsum("ik,JL->iJkL", d, d) + np.einsum("iL,Jk->iJkL", d, d)) + (kap - 2 * mu / 3) * np.einsum("iJ,kL->iJkL", d, d)
    np.testing.assert_allclose(A, lame, atol=1e-13)


def test_tensor_symmetries():
    m = make_model(2, 8, 3, normalize=True)
    out = ncm.stress_stiffness(rand_F(20, seed=15), m)
    A, tau, cc = out["A"], out["tau"], out["cc"]
    assert rel(A, np.einsum("niJkL->nkLiJ", A)) < 1e-13            # major symmetry
    assert rel(tau, np.swapaxes(tau, 1, 2)) < 1e-13                 # tau = P F^T symmetric
    assert rel(cc, np.einsum("nijkl->njikl", cc)) < 1e-13           # minor
    assert rel(cc, np.einsum("nijkl->nijlk", cc)) < 1e-13
    assert rel(cc, np.einsum("nijkl->nklij", cc)) < 1e-13           # major


def test_inverted_element_values_are_defined():
    """J < 0 (reading R10): isochoric factors use I3 = J^2, values stay finite
    and still equal the complex-step derivative of the energy."""
    m = make_model(2, 8, 2)
    F = rand_F(6, seed=16)
    F[:, :, 0] *= -1  # det < 0
    out = ncm.stress_stiffness(F, m)
    assert np.isfinite(out["A"]).all()
    assert rel(out["P"], cs_grad(lambda X: ncm.energy(X, m), F)) < 1e-11


@pytest.mark.parametrize("kind", ["UT", "UC", "BT", "BC", "SS", "PS"])
def test_loading_paths(kind):
    """App. C loading paths: Psi(0) = 0 (normalised), smooth, dPsi/dgamma = P : dF/dgamma."""
    m = make_model(2, 16, 3, normalize=True)
    gs = np.linspace(0.0, 0.5, 11)
    F = np.stack([synth.loading_path(kind, g) for g in gs])
    out = ncm.stress_stiffness(F, m)
    assert abs(out["psi"][0]) < 1e-13
    h = 1e-6
    for g, P in zip(gs[1:], out["P"][1:]):
        dF = (synth.loading_path(kind, g + h) - synth.loading_path(kind, g - h)) / (2 * h)
        dpsi = (ncm.energy(synth.loading_path(kind, g + h)[None], m) - ncm.energy(synth.loading_path(kind, g - h)[None], m))[0] / (2 * h)
        assert abs(dpsi - np.sum(P * dF)) < 1e-7 * max(1.0, abs(dpsi))
