"""Pins of the oracle's elements, quadrature, element integrals and assembly."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fe, ncm
from paper_2510_00884_amd import synth


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def model(n_sv=2, h=8, L=2, normalize=True, seed=1):
    p = synth.num_inputs(n_sv)
    th = synth.micnn_params(p, h, L, seed=seed)
    return ncm.model_from_theta(th, p, h, L, synth.structural_vectors(n_sv), normalize=normalize)


MESHES = {"hex8": lambda n: synth.hex_mesh(n)[:2], "tet10": lambda n: synth.tet10_mesh(n)[:2]}


@pytest.mark.parametrize("kind", ["hex8", "tet10"])
def test_shape_functions(kind):
    rule, shape = (fe.hex8_rule, fe.hex8_shape) if kind == "hex8" else (fe.tet10_rule, fe.tet10_shape)
    pts, w = rule()
    N, dN = shape(pts)
    np.testing.assert_allclose(N.sum(1), 1.0, atol=1e-15)        # partition of unity
    np.testing.assert_allclose(dN.sum(1), 0.0, atol=1e-14)
    # Kronecker property at the nodes
    if kind == "hex8":
        nodes = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1] for a in range(8)], float)
        vol = 8.0
    else:
        v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
        nodes = np.vstack([v] + [0.5 * (v[i] + v[j]) for (i, j) in fe.TET10_EDGES])
        vol = 1.0 / 6.0
    Nn, _ = shape(nodes)
    np.testing.assert_allclose(Nn, np.eye(nodes.shape[0]), atol=1e-14)
    assert np.isclose(w.sum(), vol)
    # the rule integrates a quadratic exactly
    f = lambda x: 1 + x[:, 0] + x[:, 1] * x[:, 2] + x[:, 0] ** 2
    if kind == "hex8":
        exact = 8 + 0 + 0 + 8.0 / 3.0
    else:
        exact = 1 / 6 + 1 / 24 + 1 / 120 + 1 / 60
    assert np.isclose((w * f(pts)).sum(), exact)


@pytest.mark.parametrize("kind,n", [("hex8", 3), ("tet10", 2)])
def test_geometry(kind, n):
    X, conn = MESHES[kind](n)
    dNdX, w, det = fe.geometry(X, conn)
    assert (det > 0).all()
    assert np.isclose(w.sum(), 1.0)                                  # volume of the unit cube
    G = np.einsum("eaJ,eqaK->eqJK", X[conn], dNdX)                   # grad of the identity map
    np.testing.assert_allclose(G, np.broadcast_to(np.eye(3), G.shape), atol=1e-13)


@pytest.mark.parametrize("kind,n", [("hex8", 2), ("tet10", 1)])
def test_homogeneous_and_rigid(kind, n):
    X, conn = MESHES[kind](n)
    dNdX, w, _ = fe.geometry(X, conn)
    F0 = synth.sample_F(1, seed=3)[0]
    F = fe.deformation_gradients(X @ (F0 - np.eye(3)).T, conn, dNdX)
    np.testing.assert_allclose(F, np.broadcast_to(F0, F.shape), atol=1e-13)
    m = model()
    Q = synth.sample_F(1, seed=5, sigma=0.0)[0]
    u = X @ (Q - np.eye(3)).T + np.array([0.1, -0.2, 0.3])
    r, K, _ = fe.element_residual_stiffness(u, conn, dNdX, w, m)
    assert np.abs(r).max() < 1e-12                                   # rigid motion: no residual


@pytest.mark.parametrize("kind,n", [("hex8", 2), ("tet10", 1)])
def test_element_stiffness_properties(kind, n):
    X, conn = MESHES[kind](n)
    dNdX, w, _ = fe.geometry(X, conn)
    m = model()
    u = synth.displacement_uniform(X.shape[0], 0.04, seed=1)
    r, K, _ = fe.element_residual_stiffness(u, conn, dNdX, w, m)
    assert rel(K, np.swapaxes(K, 1, 2)) < 1e-13                     # hyperelastic: symmetric
    nd = K.shape[1]
    t = np.tile(np.array([0.3, -1.1, 0.7]), nd // 3)
    assert np.abs(K @ t).max() < 1e-12 * np.abs(K).max()           # translations in the null space
    # K_e is the derivative of r_e in u_e (central differences)
    e = 0
    h = 1e-6
    nodes = conn[e]
    Kfd = np.empty((nd, nd))
    for a in range(nd // 3):
        for i in range(3):
            up = u.copy(); up[nodes[a], i] += h
            um = u.copy(); um[nodes[a], i] -= h
            rp, _, _ = fe.element_residual_stiffness(up, conn[e:e + 1], dNdX[e:e + 1], w[e:e + 1], m)
            rm, _, _ = fe.element_residual_stiffness(um, conn[e:e + 1], dNdX[e:e + 1], w[e:e + 1], m)
            Kfd[:, 3 * a + i] = (rp[0] - rm[0]) / (2 * h)
    assert rel(K[e], Kfd) < 1e-7


def test_material_form_equals_spatial_form():
    """K^ab_ik from the material form sum_q w Grad N^a_J A_iJkL Grad N^b_L equals
    the paper's spatial form (eq. k-quad); r from P Grad N equals tau grad N."""
    X, conn = MESHES["hex8"](2)
    dNdX, w, _ = fe.geometry(X, conn)
    m = model()
    u = synth.displacement_uniform(X.shape[0], 0.05, seed=2)
    r, K, extra = fe.element_residual_stiffness(u, conn, dNdX, w, m)
    Km = np.einsum("eq,eqaJ,eqiJkL,eqbL->eaibk", w, dNdX, extra["A"], dNdX).reshape(K.shape)
    rm = np.einsum("eq,eqiJ,eqaJ->eai", w, extra["P"], dNdX).reshape(r.shape)
    assert rel(Km, K) < 1e-13
    assert rel(rm, r) < 1e-13


def test_global_assembly():
    X, conn = MESHES["hex8"](3)
    dNdX, w, _ = fe.geometry(X, conn)
    m = model()
    u = synth.displacement_uniform(X.shape[0], 0.05, seed=0)
    r_e, K_e, _ = fe.element_residual_stiffness(u, conn, dNdX, w, m)
    r, K = fe.assemble(conn, r_e, K_e, X.shape[0])
    assert abs(K - K.T).max() < 1e-12 * abs(K).max()
    v = np.random.default_rng(0).normal(size=r.shape)
    dofs = fe.element_dofs(conn)
    Kv = np.zeros_like(v)
    np.add.at(Kv, dofs.ravel(), np.einsum("eij,ej->ei", K_e, v[dofs]).ravel())
    assert rel(K @ v, Kv) < 1e-13                                   # matrix-free product
    assert np.isclose(r.sum(), r_e.sum())
    # a hex8 interior node couples to 27 nodes -> 81 entries per interior row
    counts = np.diff(K.indptr)
    assert counts.max() == 81


def test_tet10_colouring_and_hex_colouring_are_valid():
    for kind, gen in (("hex8", synth.hex_mesh), ("tet10", synth.tet10_mesh)):
        X, conn, col = gen(3)
        for c in np.unique(col):
            nodes = conn[col == c].ravel()
            assert np.unique(nodes).size == nodes.size, kind
    assert np.unique(synth.tet10_mesh(2)[2]).size == 48
