"""Pins of the oracle's stress-calibration gradient: complex-step directional
derivatives (exact), central finite differences (h = 1e-6, FP64), and the
consistency of the feature derivatives with the constitutive route."""
import numpy as np
import pytest

from oracle import calib, ncm
from paper_2510_00884_amd import synth


def setup(n=64, n_sv=2, h=8, L=3):
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    theta = synth.micnn_params(p, h, L, seed=1)
    theta_ref = synth.micnn_params(p, h, L, seed=4)
    F = synth.sample_F(n, seed=3)
    Pref = ncm.stress_stiffness(F, ncm.model_from_theta(theta_ref, p, h, L, Av))["P"]
    Pt = Pref + 0.01 * np.sqrt(np.mean(Pref ** 2)) * synth.rng(5).normal(size=Pref.shape)
    return theta, F, Pt, Av, p, h, L


def test_feature_gradients_match_stress_route():
    theta, F, Pt, Av, p, h, L = setup()
    m = ncm.model_from_theta(theta, p, h, L, Av)
    K, g = calib.feature_grads(F, Av)
    _, dN, _ = ncm.micnn(K, m.hidden, m.a, m.b)
    P = np.einsum("nm,nmiJ->niJ", dN, g)
    np.testing.assert_allclose(P, ncm.stress_stiffness(F, m)["P"], rtol=1e-12, atol=1e-13)


def test_gradient_complex_step():
    theta, F, Pt, Av, p, h, L = setup()
    Lval, grad = calib.loss_and_grad(theta, F, Pt, Av, p, h, L)
    assert np.isclose(Lval, calib.loss(theta, F, Pt, Av, p, h, L), rtol=1e-13)
    r = np.random.default_rng(0)
    eps = 1e-20
    for _ in range(5):
        v = r.normal(size=theta.shape)
        d = np.imag(calib.loss(theta + 1j * eps * v, F, Pt, Av, p, h, L)) / eps
        assert abs(d - grad @ v) <= 1e-12 * max(1.0, abs(d))


def test_gradient_central_differences():
    theta, F, Pt, Av, p, h, L = setup(n=32)
    _, grad = calib.loss_and_grad(theta, F, Pt, Av, p, h, L)
    r = np.random.default_rng(1)
    hstep = 1e-6
    for idx in r.choice(theta.size, 16, replace=False):
        e = np.zeros_like(theta); e[idx] = hstep
        fd = (calib.loss(theta + e, F, Pt, Av, p, h, L) - calib.loss(theta - e, F, Pt, Av, p, h, L)) / (2 * hstep)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(grad).max())


def test_gradient_large_preactivations_complex_step():
    """3 x 64 network with non-negative weights: layer-3 pre-activations reach
    the hundreds, where a linearised softplus would be off by e^{-y}; the
    gradient still matches exact complex-step directional derivatives."""
    theta, F, Pt, Av, p, h, L = setup(n=24, h=64, L=3)
    Lval, grad = calib.loss_and_grad(theta, F, Pt, Av, p, h, L)
    r = np.random.default_rng(3)
    for _ in range(3):
        v = r.normal(size=theta.shape)
        d = np.imag(calib.loss(theta + 1j * 1e-20 * v, F, Pt, Av, p, h, L)) / 1e-20
        assert abs(d - grad @ v) <= 1e-12 * max(1.0, abs(d))


def residual_setup(kind="hex8", n=2, n_sv=1, h=8, L=2):
    X, conn, _ = (synth.hex_mesh if kind == "hex8" else synth.tet10_mesh)(n)
    u = synth.displacement_modes(X, 1.0 / n, seed=0)
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    theta = synth.micnn_params(p, h, L, seed=1)
    grp = synth.reaction_groups(X)
    R = np.array([0.03, -0.02])
    return theta, X, conn, u, grp, R, Av, p, h, L


@pytest.mark.parametrize("kind", ["hex8", "tet10"])
def test_residual_loss_gradient_complex_step(kind):
    """dL/dtheta of eq. (loss) by reverse mode on the material-form residual
    equals exact complex-step directional derivatives of L computed through
    the spatial-form element residual."""
    theta, X, conn, u, grp, R, Av, p, h, L = residual_setup(kind)
    Lval, grad, _ = calib.residual_loss_and_grad(theta, X, conn, u, grp, R, Av, p, h, L)
    assert np.isclose(Lval, calib.residual_loss(theta, X, conn, u, grp, R, Av, p, h, L), rtol=1e-12)
    rng = np.random.default_rng(2)
    for _ in range(3):
        v = rng.normal(size=theta.shape)
        d = np.imag(calib.residual_loss(theta + 1j * 1e-20 * v, X, conn, u, grp, R, Av, p, h, L)) / 1e-20
        assert abs(d - grad @ v) <= 1e-12 * max(1.0, abs(d))


def test_residual_groups_cover_faces():
    X, _, _ = synth.hex_mesh(3)
    grp = synth.reaction_groups(X).reshape(-1, 3)
    assert np.all(grp[np.isclose(X[:, 0], 0.0)] == -2)
    assert np.all(grp[np.isclose(X[:, 0], 1.0), 0] == 0)
    on_y = np.isclose(X[:, 1], 1.0) & ~np.isclose(X[:, 0], 0.0)
    assert np.all(grp[on_y, 1] == 1)
    assert (grp == -1).sum() > 0
