"""Oracle: stress-calibration loss and its gradient with respect to the network
parameters.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The loss is the mean over samples of the squared Frobenius norm of the stress
misfit, L = (1/N) sum_q ||P(F_q; theta) - P_t,q||^2, for the raw (not
normalised) network.  P is linear in the network gradient,
P_q = sum_m dN/dK_m (K_q; theta) g_m(F_q) with g_m = dK_m/dF = 2 G^m F^{-T}
(eq. stress-cgo pulled back, App. A.1); the feature derivatives g_m do not
depend on theta and come from the push-forward tables of ``ncm``.  The network
value is written as plain PyTorch CPU operations in FP64; its input gradient
and the parameter gradient of L are taken by reverse-mode automatic
differentiation (the library primitive), so this route shares nothing with a
hand-written adjoint.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ncm


def feature_grads(F, Avec):
    """K (n, p) and g (n, p, 3, 3) with g_m = dK_m/dF."""
    K, G, _ = ncm.feature_tables(F, Avec)
    Fi = ncm._inv3(F)
    g = 2.0 * np.einsum("nmij,nJj->nmiJ", G, Fi)
    return K, g


def _unpack_torch(theta, p, h, L, has_bias=True):
    off = 0

    def take(shape):
        nonlocal off
        cnt = int(np.prod(shape))
        x = theta[off:off + cnt].reshape(shape)
        off += cnt
        return x

    W1 = take((h, p))
    c1 = take((h,)) if has_bias else torch.zeros(h, dtype=theta.dtype)
    layers = [(W1, None, c1)]
    for _ in range(2, L + 1):
        A = take((h, h)); B = take((h, p))
        c = take((h,)) if has_bias else torch.zeros(h, dtype=theta.dtype)
        layers.append((A, B, c))
    a = take((h,)); b = take((p,))
    assert off == theta.numel()
    return layers, a, b


def _softplus(y):
    """log(1 + e^y) in the overflow-free form max(y, 0) + log(1 + e^{-|y|});
    exact for every y (no linearisation above a threshold)."""
    return torch.clamp(y, min=0.0) + torch.log1p(torch.exp(-torch.abs(y)))


def _network_value(K, layers, a, b):
    """eq. (icnn): y^k = A^k z^{k-1} + B^k z^0 + c^k, z^k = softplus(y^k),
    N = a . z^{L} + b . z^0."""
    z = K
    for (A, B, c) in layers:
        y = z @ A.T + c
        if B is not None:
            y = y + K @ B.T
        z = _softplus(y)
    return z @ a + K @ b


def stress_from_theta(theta, K, g, p, h, L, has_bias=True):
    """P (n, 3, 3) as a differentiable function of theta (torch, FP64)."""
    layers, a, b = _unpack_torch(theta, p, h, L, has_bias)
    Kt = K.clone().requires_grad_(True)
    N = _network_value(Kt, layers, a, b)
    dN, = torch.autograd.grad(N.sum(), Kt, create_graph=True)
    return torch.einsum("nm,nmij->nij", dN, g)


def loss_and_grad(theta, F, P_target, Avec, p, h, L, has_bias=True):
    """L and dL/dtheta in FP64 (numpy in, numpy out)."""
    K, g = feature_grads(F, Avec)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    Kt = torch.tensor(K, dtype=torch.float64)
    gt = torch.tensor(g, dtype=torch.float64)
    P = stress_from_theta(th, Kt, gt, p, h, L, has_bias)
    Pt = torch.tensor(P_target, dtype=torch.float64)
    Lval = ((P - Pt) ** 2).sum() / F.shape[0]
    grad, = torch.autograd.grad(Lval, th)
    return float(Lval.detach()), grad.numpy()


def loss(theta, F, P_target, Avec, p, h, L, has_bias=True, normalize=False):
    """L evaluated through the NumPy model (real or complex theta); used by
    the finite-difference and complex-step pins."""
    model = ncm.model_from_theta(theta, p, h, L, Avec, normalize=normalize, has_bias=has_bias)
    K, g = feature_grads(F, Avec)
    _, dN, _ = ncm.micnn(K.astype(np.result_type(K, theta)), model.hidden, model.a, model.b)
    P = np.einsum("nm,nmiJ->niJ", dN, g)
    return np.sum((P - P_target) ** 2) / F.shape[0]


# ----------------------------------------------------------------------------
# residual (NN-EUCLID) loss, eq. (loss), one time step
# ----------------------------------------------------------------------------
def _residual_loss_value(r, dof_group, R, xp):
    """L = sum_{free} r_d^2 + sum_b (R_b - sum_{d in b} r_d)^2 (eq. loss);
    dof_group: -1 free, b >= 0 reaction boundary b, -2 constrained unobserved."""
    free = dof_group == -1
    L = (r[free] ** 2).sum()
    for b in range(len(R)):
        L = L + (R[b] - r[dof_group == b].sum()) ** 2
    return L


def residual_loss_and_grad(theta, X, conn, u, dof_group, R, Avec, p, h, L, has_bias=True):
    """L and dL/dtheta for the raw network (numpy in, numpy out): the
    residual r^a_i = sum_q w P_iJ(F_q; theta) dN^a/dX_J (eqs. r-quad,
    apprx-r, material form) assembled over node-major dofs with PyTorch on
    the CPU in FP64, the stress from stress_from_theta, and reverse-mode
    automatic differentiation for the gradient."""
    from . import fe
    dNdX, w, _ = fe.geometry(X, conn)                       # (n_el, nq, nen, 3), (n_el, nq)
    F = fe.deformation_gradients(u, conn, dNdX)             # (n_el, nq, 3, 3)
    n_el, nq = F.shape[:2]
    K, g = feature_grads(F.reshape(-1, 3, 3), Avec)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    P = stress_from_theta(th, torch.tensor(K), torch.tensor(g), p, h, L, has_bias).reshape(n_el, nq, 3, 3)
    G = torch.tensor(dNdX)
    wt = torch.tensor(w)
    r_e = torch.einsum("eq,eqiJ,eqaJ->eai", wt, P, G)      # (n_el, nen, 3)
    dofs = torch.tensor(fe.element_dofs(conn)).reshape(-1)
    r = torch.zeros(3 * X.shape[0], dtype=torch.float64).index_add(0, dofs, r_e.reshape(-1))
    Lval = _residual_loss_value(r, torch.tensor(dof_group), torch.tensor(np.asarray(R, dtype=np.float64)), torch)
    grad, = torch.autograd.grad(Lval, th)
    return float(Lval.detach()), grad.numpy(), r.detach().numpy()


def residual_loss(theta, X, conn, u, dof_group, R, Avec, p, h, L, has_bias=True):
    """L through the NumPy model and the oracle's element residual (spatial
    form); real or complex theta, for finite-difference and complex-step
    pins."""
    from . import fe
    model = ncm.model_from_theta(theta, p, h, L, Avec, normalize=False, has_bias=has_bias)
    dNdX, w, _ = fe.geometry(X, conn)
    r_e, _, _ = fe.element_residual_stiffness(u, conn, dNdX, w, model)
    dofs = fe.element_dofs(conn)
    r = np.zeros(3 * X.shape[0], dtype=np.result_type(r_e, np.float64))
    np.add.at(r, dofs.reshape(-1), r_e.reshape(-1))
    return _residual_loss_value(r, np.asarray(dof_group), np.asarray(R), np)
