"""Oracle: isoparametric elements, quadrature, element residual/stiffness and
global assembly.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (shared with the product path as an interface, not as code):
* hex8 local node a = a0 + 2*a1 + 4*a2 sits at reference corner
  (2*a0-1, 2*a1-1, 2*a2-1); 2x2x2 Gauss rule at +-1/sqrt(3), weights 1, point
  q = q0 + 2*q1 + 4*q2 at ((2*q0-1), (2*q1-1), (2*q2-1))/sqrt(3).
* tet10 local nodes: vertices 0..3 at reference (0,0,0), (1,0,0), (0,1,0),
  (0,0,1), then mid-edge nodes of edges (0,1), (1,2), (0,2), (0,3), (1,3),
  (2,3); 4-point rule, point q has barycentric coordinate alpha at vertex q and
  beta elsewhere, weight 1/24.
* Element dof 3*a + i; global dof 3*node + i (node-major order of Sec. 2.1).

Readings of the paper used here
-------------------------------
E1  The quadrature weight w^{e,q}, "the volume of the quadrature point", is the
    reference Gauss weight times det(dX/dxi) (eqs. r-quad, k-quad).
E2  No traction boundary (eq. apprx-r): the Neumann term is absent.
E3  Global vectors and matrices are indexed by node-major dofs (Sec. 2.1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import ncm

G8 = 1.0 / np.sqrt(3.0)
TET_ALPHA = 0.5854101966249685
TET_BETA = 0.1381966011250105
TET10_EDGES = [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]


# ----------------------------------------------------------------------------
# shape functions and rules
# ----------------------------------------------------------------------------
def hex8_rule():
    pts = np.array([[(2 * (q & 1) - 1), (2 * ((q >> 1) & 1) - 1), (2 * ((q >> 2) & 1) - 1)]
                    for q in range(8)], dtype=float) * G8
    return pts, np.ones(8)


def hex8_shape(pts):
    """N (nq, 8) and dN/dxi (nq, 8, 3) of the trilinear hexahedron."""
    s = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1]
                  for a in range(8)], dtype=float)
    f = 1.0 + pts[:, None, :] * s[None, :, :]          # (nq, 8, 3)
    N = 0.125 * f.prod(axis=2)
    dN = np.empty(f.shape)
    for d in range(3):
        others = [e for e in range(3) if e != d]
        dN[:, :, d] = 0.125 * s[None, :, d] * f[:, :, others[0]] * f[:, :, others[1]]
    return N, dN


def tet10_rule():
    L = np.full((4, 4), TET_BETA)
    np.fill_diagonal(L, TET_ALPHA)
    pts = L[:, 1:]  # reference coordinates (xi, eta, zeta) = (L1, L2, L3)
    return pts, np.full(4, 1.0 / 24.0)


def tet10_shape(pts):
    """N (nq, 10) and dN/dxi (nq, 10, 3) of the quadratic tetrahedron."""
    nq = pts.shape[0]
    L = np.empty((nq, 4))
    L[:, 1:] = pts
    L[:, 0] = 1.0 - pts.sum(axis=1)
    dL = np.zeros((4, 3))
    dL[0, :] = -1.0
    dL[1, 0] = dL[2, 1] = dL[3, 2] = 1.0
    N = np.empty((nq, 10))
    dN = np.empty((nq, 10, 3))
    for a in range(4):
        N[:, a] = L[:, a] * (2.0 * L[:, a] - 1.0)
        dN[:, a, :] = (4.0 * L[:, a] - 1.0)[:, None] * dL[a][None, :]
    for e, (i, j) in enumerate(TET10_EDGES):
        N[:, 4 + e] = 4.0 * L[:, i] * L[:, j]
        dN[:, 4 + e, :] = 4.0 * (L[:, j][:, None] * dL[i][None, :] + L[:, i][:, None] * dL[j][None, :])
    return N, dN


def element_kind(nen):
    if nen == 8:
        return hex8_rule, hex8_shape
    if nen == 10:
        return tet10_rule, tet10_shape
    raise ValueError(nen)


# ----------------------------------------------------------------------------
# geometry: reference gradients and quadrature-point volumes
# ----------------------------------------------------------------------------
def geometry(X, conn):
    """dN/dX at every quadrature point and w = w_hat * det(dX/dxi) (E1).

    Returns dNdX (n_el, nq, nen, 3), w (n_el, nq), detJ (n_el, nq)."""
    rule, shape = element_kind(conn.shape[1])
    pts, wq = rule()
    _, dNr = shape(pts)                                # (nq, nen, 3)
    Xe = X[conn]                                       # (n_el, nen, 3)
    jac = np.einsum("qad,eaJ->eqdJ", dNr, Xe)          # dX_J/dxi_d
    det = np.linalg.det(jac)
    jinv = np.linalg.inv(jac)                          # (jinv)_{J d}
    dNdX = np.einsum("eqJd,qad->eqaJ", jinv, dNr)
    return dNdX, wq[None, :] * det, det


# ----------------------------------------------------------------------------
# Alg. 2: deformation gradient table -> vectorised constitutive model ->
# element sums (spatial form, eqs. apprx-k, apprx-r, r-quad, k-quad)
# ----------------------------------------------------------------------------
def deformation_gradients(u, conn, dNdX):
    """F = I + sum_a u^a (x) Grad N^a at every quadrature point (Alg. 1/2)."""
    ue = u[conn]                                       # (n_el, nen, 3)
    return np.eye(3) + np.einsum("eai,eqaJ->eqiJ", ue, dNdX)


def element_residual_stiffness(u, conn, dNdX, w, model):
    """r_e (n_el, 3*nen) and K_e (n_el, 3*nen, 3*nen).

    r^a_i = sum_q w tau_ij grad N^a_j,
    K^ab_ij = sum_q w grad N^a_k (delta_ij tau_kl + cc_ikjl) grad N^b_l,
    with grad N = F^{-T} Grad N (spatial gradient) and tau, cc from the
    push-forward route of the constitutive model."""
    n_el, nq, nen, _ = dNdX.shape
    F = deformation_gradients(u, conn, dNdX)
    out = ncm.stress_stiffness(F.reshape(-1, 3, 3), model)
    tau = out["tau"].reshape(n_el, nq, 3, 3)
    cc = out["cc"].reshape(n_el, nq, 3, 3, 3, 3)
    Fi = ncm._inv3(F)
    gx = np.einsum("eqJj,eqaJ->eqaj", Fi, dNdX)        # spatial gradients
    r = np.einsum("eq,eqij,eqaj->eai", w, tau, gx).reshape(n_el, 3 * nen)
    geo = np.einsum("ij,eqkl->eqikjl", np.eye(3), tau)
    D = geo + cc                                        # delta_ij tau_kl + cc_ikjl
    K = np.einsum("eq,eqak,eqikjl,eqbl->eaibj", w, gx, D, gx).reshape(n_el, 3 * nen, 3 * nen)
    return r, K, dict(F=F, psi=out["psi"].reshape(n_el, nq), P=out["P"].reshape(n_el, nq, 3, 3),
                      A=out["A"].reshape(n_el, nq, 3, 3, 3, 3))


def element_dofs(conn):
    nen = conn.shape[1]
    return (3 * conn[:, :, None] + np.arange(3)[None, None, :]).reshape(conn.shape[0], 3 * nen)


def assemble(conn, r_e, K_e, n_nodes):
    """Global residual and stiffness (CSR) by summing element contributions
    over node-major dofs (E3); duplicates are summed by the sparse library."""
    dofs = element_dofs(conn)
    ndof = 3 * n_nodes
    r = np.zeros(ndof)
    np.add.at(r, dofs.ravel(), r_e.ravel())
    nd = dofs.shape[1]
    rows = np.repeat(dofs, nd, axis=1).ravel()
    cols = np.tile(dofs, (1, nd)).ravel()
    K = sp.coo_matrix((K_e.ravel(), (rows, cols)), shape=(ndof, ndof)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    return r, K
