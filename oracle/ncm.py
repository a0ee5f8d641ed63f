"""Oracle: neural constitutive model (kinematic layer + MICNN + CGO route).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything is batched over a leading axis of quadrature points and works for
real (float64) and complex (complex128) inputs, so that complex-step
differentiation can pin it.

Readings of the paper used here
-------------------------------
R1  I5,ij second-order tensor for i != j (App. A.2.1): the printed
    2 sym(a^i (x) B a^j) holds only for i = j; the derivative of
    I5,ij = A^i . C^2 A^j pushed forward is  B M + M B  with M = sym(a^i (x) a^j).
R2  Isochoric I5 table (App. A.2.2) uses the isochoric B~ = J^{-2/3} B and
    a~ = J^{-1/3} a throughout (the printed G~5 shows B).
R3  The stiffness sum over the network Hessian runs over m and n
    (eq. stiffnes-cgo prints d2N/dK_m dK_m).
R4  The symmetric product is the standard
    (A [x] B)_ijkl = (A_ik B_jl + A_il B_jk)/2; the printed B_kj index is
    equivalent for the symmetric arguments used.
R5  I4 and I5 inputs use unordered pairs i <= j of structural vectors.
R6  Features (extends the kinematic layer of App. C to anisotropy):
    K = [I1~ - 3, I2~^{3/2} - 3^{3/2}, (J - 1)^2,
         {I4~_ij - A^i.A^j}_{i<=j}, {I5~_ij - A^i.A^j}_{i<=j}],
    all zero at F = I.
R7  The first hidden layer has one matrix W1 (A^(1) and B^(1) multiply the same
    z^(0) = K); hidden layers carry biases c_k; the output layer has none.
R8  Activation: softplus F(y) = log(1 + e^y), F' = sigma(y),
    F'' = sigma(y)(1 - sigma(y)).
R9  Optional normalisation (energy- and stress-free reference state):
    Psi = N(K) - N(0) - sum_{i<=j} kappa_ij K_{4,ij},
    kappa_ij = dN/dK_{4,ij}(0) + 2 dN/dK_{5,ij}(0).
R10 J <= 0: the isochoric factors use I3 = J^2 > 0; values are still produced.
R12 CANN inner network (App. B.1, eq. cann-def) with the layers of the
    hyper-parameter table: f0 = identity; for every input m four branches,
    powers {1, 2} times functions {w1 x, exp(w1 x) - 1}, each with its own
    inner weight w1 and outer weight w2, so 8 parameters per input, ordered
    per input as (1, lin), (2, lin), (1, exp), (2, exp), each (w1, w2).  The
    table's count of 33 parameters for three inputs does not follow from the
    printed layers; that count is unpinned.
R13 Gent-Thomas (eq. gt) as an inner function of the isotropic features:
    N = c1 K1 + c2 ((2/3) log(K2 + 3^{3/2}) - log 3) + c3 K3, with
    (c1, c2, c3) = (0.5, 1, 1) for eq. gt; other features carry no weight.
"""
from __future__ import annotations

import numpy as np

EYE = np.eye(3)
S32 = 3.0 ** 1.5


# ----------------------------------------------------------------------------
# small tensor helpers (batched over the leading axis)
# ----------------------------------------------------------------------------
def _sym(A):
    return 0.5 * (A + np.swapaxes(A, -1, -2))


def _outer(A, B):
    """(A (x) B)_ijkl = A_ij B_kl."""
    return np.einsum("...ij,...kl->...ijkl", A, B)


def _boxtimes(A, B):
    """(A [x] B)_ijkl = (A_ik B_jl + A_il B_jk)/2   (reading R4)."""
    return 0.5 * (np.einsum("...ik,...jl->...ijkl", A, B)
                  + np.einsum("...il,...jk->...ijkl", A, B))


def _det3(F):
    return (F[..., 0, 0] * (F[..., 1, 1] * F[..., 2, 2] - F[..., 1, 2] * F[..., 2, 1])
            - F[..., 0, 1] * (F[..., 1, 0] * F[..., 2, 2] - F[..., 1, 2] * F[..., 2, 0])
            + F[..., 0, 2] * (F[..., 1, 0] * F[..., 2, 1] - F[..., 1, 1] * F[..., 2, 0]))


def _inv3(F):
    """Inverse by the adjugate (works for complex entries)."""
    a = F
    cof = np.empty_like(a)
    cof[..., 0, 0] = a[..., 1, 1] * a[..., 2, 2] - a[..., 1, 2] * a[..., 2, 1]
    cof[..., 0, 1] = -(a[..., 1, 0] * a[..., 2, 2] - a[..., 1, 2] * a[..., 2, 0])
    cof[..., 0, 2] = a[..., 1, 0] * a[..., 2, 1] - a[..., 1, 1] * a[..., 2, 0]
    cof[..., 1, 0] = -(a[..., 0, 1] * a[..., 2, 2] - a[..., 0, 2] * a[..., 2, 1])
    cof[..., 1, 1] = a[..., 0, 0] * a[..., 2, 2] - a[..., 0, 2] * a[..., 2, 0]
    cof[..., 1, 2] = -(a[..., 0, 0] * a[..., 2, 1] - a[..., 0, 1] * a[..., 2, 0])
    cof[..., 2, 0] = a[..., 0, 1] * a[..., 1, 2] - a[..., 0, 2] * a[..., 1, 1]
    cof[..., 2, 1] = -(a[..., 0, 0] * a[..., 1, 2] - a[..., 0, 2] * a[..., 1, 0])
    cof[..., 2, 2] = a[..., 0, 0] * a[..., 1, 1] - a[..., 0, 1] * a[..., 1, 0]
    det = _det3(F)
    return np.swapaxes(cof, -1, -2) / det[..., None, None]


def pairs(n_sv: int):
    """Unordered pairs (i, j), i <= j, of structural vectors (reading R5)."""
    return [(i, j) for i in range(n_sv) for j in range(i, n_sv)]


def num_inputs(n_sv: int) -> int:
    return 3 + 2 * len(pairs(n_sv))


# ----------------------------------------------------------------------------
# Kinematic layer: invariants (eq. standard-inv-I; App. A.2.1-A.2.2)
# ----------------------------------------------------------------------------
def invariants(F, Avec):
    """Raw invariants.  Returns dict with I1, I2, I3, J, I4[pair], I5[pair]."""
    C = np.einsum("...ki,...kj->...ij", F, F)
    I1 = np.einsum("...ii->...", C)
    C2 = np.einsum("...ij,...jk->...ik", C, C)
    I2 = 0.5 * (I1 ** 2 - np.einsum("...ii->...", C2))
    J = _det3(F)
    I3 = J * J  # det C = (det F)^2
    n_sv = Avec.shape[0]
    I4, I5 = [], []
    for (i, j) in pairs(n_sv):
        I4.append(np.einsum("i,...ij,j->...", Avec[i], C, Avec[j]))
        I5.append(np.einsum("i,...ij,j->...", Avec[i], C2, Avec[j]))
    return dict(C=C, I1=I1, I2=I2, I3=I3, J=J, I4=I4, I5=I5)


def features(F, Avec):
    """Feature vector K (reading R6) from the isochoric invariants
    I~_m = I_m I3^{alpha_m}, alpha = -1/3 for {1, (4,ij)}, -2/3 for {2, (5,ij)}."""
    inv = invariants(F, Avec)
    I3 = inv["I3"]
    p13 = I3 ** (-1.0 / 3.0)
    p23 = I3 ** (-2.0 / 3.0)
    I1t = inv["I1"] * p13
    I2t = inv["I2"] * p23
    J = inv["J"]
    feats = [I1t - 3.0, I2t ** 1.5 - S32, (J - 1.0) ** 2]
    n_sv = Avec.shape[0]
    prs = pairs(n_sv)
    for k, (i, j) in enumerate(prs):
        feats.append(inv["I4"][k] * p13 - Avec[i] @ Avec[j])
    for k, (i, j) in enumerate(prs):
        feats.append(inv["I5"][k] * p23 - Avec[i] @ Avec[j])
    return np.stack(feats, axis=-1)


def _softplus(y):
    if np.iscomplexobj(y):
        return np.log1p(np.exp(y))
    return np.maximum(y, 0.0) + np.log1p(np.exp(-np.abs(y)))


def _sigmoid(y):
    if np.iscomplexobj(y):
        return 1.0 / (1.0 + np.exp(-y))
    e = np.exp(-np.abs(y))
    return np.where(y >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


# ----------------------------------------------------------------------------
# Inner network: (M)ICNN value, input gradient and input Hessian (eq. icnn)
# ----------------------------------------------------------------------------
def micnn(K, hidden, a, b):
    """Value, input gradient and input Hessian of the network of eq. (icnn).

    ``hidden`` = [(W1, None, c1), (A2, B2, c2), ...]; ``a``, ``b`` output weights.
    K: (n, p).  Returns N (n,), dN (n, p), d2N (n, p, p).

    The derivatives are the plain chain and product rules applied to the layer
    recursion y_k = A_k z_{k-1} + B_k K + c_k, z_k = F(y_k), z_0 = K,
    N = a.z_L + b.K, organised as
      gradient: the reverse sweep lambda_L = a, mu_k = lambda_k * F'(y_k),
                lambda_{k-1} = A_k^T mu_k, dN/dK = b + sum_k B_k^T mu_k + lambda_0;
      Hessian:  column m is the derivative of that reverse sweep along the
                input direction e_m (tangents ydot_k of the layer recursion,
                then mudot_k = lambdadot_k * F'(y_k) + lambda_k * F''(y_k) * ydot_k,
                lambdadot_{k-1} = A_k^T mudot_k), i.e. one Hessian-vector
                product per input.
    The App. B.2 algorithm computes the same quantities by carrying the
    second-derivative columns forward instead; the complex-step and
    closed-form pins in the tests check these against the plain value pass.
    """
    n, p = K.shape
    # forward: pre-activations of every layer
    ys = []
    z = K
    for (A, B, c) in hidden:
        y = z @ A.T + c
        if B is not None:
            y = y + K @ B.T
        ys.append(y)
        z = _softplus(y)
    N = z @ a + K @ b
    s1 = [_sigmoid(y) for y in ys]          # F'(y_k)
    s2 = [s * (1.0 - s) for s in s1]        # F''(y_k)
    # reverse sweep (gradient)
    Lh = len(hidden)
    lams = [None] * Lh                      # lambda_k = dN/dz_k
    mus = [None] * Lh
    lam = np.broadcast_to(a, ys[-1].shape)
    dN = np.broadcast_to(b, (n, p)).astype(np.result_type(K, a, b)).copy()
    for k in range(Lh - 1, -1, -1):
        A, B, _ = hidden[k]
        lams[k] = lam
        mu = lam * s1[k]
        mus[k] = mu
        if B is not None:
            dN = dN + mu @ B
        lam = mu @ A                        # lambda_{k-1}; lambda_0 = dN/dz_0 through z_0 = K
    dN = dN + lam
    # tangent of the reverse sweep along every input direction (Hessian columns)
    d2N = np.zeros((n, p, p), dtype=dN.dtype)
    for m in range(p):
        e = np.zeros(p)
        e[m] = 1.0
        ydots = []
        zdot = np.broadcast_to(e, (n, p))
        for (A, B, _), s in zip(hidden, s1):
            yd = zdot @ A.T
            if B is not None:
                yd = yd + B @ e
            ydots.append(yd)
            zdot = s * yd
        col = np.zeros((n, p), dtype=dN.dtype)
        lamdot = np.zeros_like(ys[-1])
        for k in range(Lh - 1, -1, -1):
            A, B, _ = hidden[k]
            mudot = lamdot * s1[k] + lams[k] * s2[k] * ydots[k]
            if B is not None:
                col = col + mudot @ B
            lamdot = mudot @ A
        d2N[:, :, m] = col + lamdot
    return N, dN, d2N


def micnn_value(K, hidden, a, b):
    """Plain forward pass of eq. (icnn) (value only); the derivatives of
    ``micnn`` are pinned against it by complex steps."""
    z = K
    for (A, B, c) in hidden:
        y = np.einsum("jk,nk->nj", A, z) + c
        if B is not None:
            y = y + np.einsum("jk,nk->nj", B, K)
        z = _softplus(y)
    return z @ a + K @ b


class Model:
    """Network parameters plus structural vectors and the normalisation flag."""

    def __init__(self, hidden, a, b, Avec, normalize=False):
        self.hidden = hidden
        self.a = np.asarray(a)
        self.b = np.asarray(b)
        self.Avec = np.asarray(Avec, dtype=float).reshape(-1, 3)
        self.normalize = bool(normalize)
        self.p = self.b.shape[0]
        n_sv = self.Avec.shape[0]
        assert self.p == num_inputs(n_sv)
        self.kappa = np.zeros(len(pairs(n_sv)))
        self.N0 = 0.0
        if self.normalize:
            N0, dN0, _ = micnn(np.zeros((1, self.p)), hidden, self.a, self.b)
            npair = len(pairs(n_sv))
            self.N0 = float(np.real(N0[0]))
            self.kappa = np.real(dN0[0, 3:3 + npair] + 2.0 * dN0[0, 3 + npair:3 + 2 * npair])

    # inner function seen by the chain rule: value, gradient, Hessian in K
    def inner(self, K):
        N, dN, d2N = micnn(K, self.hidden, self.a, self.b)
        if self.normalize:
            npair = self.kappa.shape[0]
            N = N - self.N0 - K[:, 3:3 + npair] @ self.kappa
            dN = dN.copy()
            dN[:, 3:3 + npair] -= self.kappa
        return N, dN, d2N


def cann(K, theta):
    """CANN inner network (eq. cann-def) and its derivatives (eq.
    cann-chain-rule, diagonal Hessian) under reading R12.  theta: 8 p."""
    n, p = K.shape
    th = np.asarray(theta).reshape(p, 4, 2)
    N = np.zeros(n, dtype=np.result_type(K, th))
    dN = np.zeros((n, p), dtype=N.dtype)
    d2N = np.zeros((n, p, p), dtype=N.dtype)
    for m in range(p):
        x = K[:, m]
        for k, (e, kind) in enumerate([(1, 0), (2, 0), (1, 1), (2, 1)]):
            w1, w2 = th[m, k]
            f1 = x ** e                        # power layer
            d1 = e * x ** (e - 1)
            dd1 = e * (e - 1) * x ** max(e - 2, 0) if e >= 2 else 0.0 * x
            if kind == 0:                      # f2 = w1 f1
                f2, d2, dd2 = w1 * f1, w1 + 0.0 * x, 0.0 * x
            else:                              # f2 = exp(w1 f1) - 1
                ex = np.exp(w1 * f1)
                f2, d2, dd2 = ex - 1.0, w1 * ex, w1 * w1 * ex
            N = N + w2 * f2
            dN[:, m] += w2 * d2 * d1
            d2N[:, m, m] += w2 * (dd2 * d1 * d1 + d2 * dd1)
    return N, dN, d2N


def gent_thomas(K, coef):
    """Gent-Thomas inner function (eq. gt, reading R13)."""
    c1, c2, c3 = coef
    u = K[:, 1] + S32
    N = c1 * K[:, 0] + c2 * ((2.0 / 3.0) * np.log(u) - np.log(3.0)) + c3 * K[:, 2]
    dN = np.zeros_like(K, dtype=np.result_type(K, u))
    d2N = np.zeros(K.shape + (K.shape[1],), dtype=dN.dtype)
    dN[:, 0] = c1
    dN[:, 1] = c2 * (2.0 / 3.0) / u
    dN[:, 2] = c3
    d2N[:, 1, 1] = -c2 * (2.0 / 3.0) / u ** 2
    return N, dN, d2N


class ClosedModel:
    """An inner function other than the MICNN (CANN or Gent-Thomas) with the
    same structural vectors and normalisation (R9) as Model."""

    def __init__(self, fn, theta, Avec, normalize=False):
        self.fn = fn
        self.theta = theta
        self.Avec = np.asarray(Avec, dtype=float).reshape(-1, 3)
        self.normalize = bool(normalize)
        n_sv = self.Avec.shape[0]
        self.p = num_inputs(n_sv)
        self.kappa = np.zeros(len(pairs(n_sv)))
        self.N0 = 0.0
        if self.normalize:
            N0, dN0, _ = fn(np.zeros((1, self.p)), theta)
            npair = len(pairs(n_sv))
            self.N0 = float(np.real(N0[0]))
            self.kappa = np.real(dN0[0, 3:3 + npair] + 2.0 * dN0[0, 3 + npair:3 + 2 * npair])

    def inner(self, K):
        N, dN, d2N = self.fn(K, self.theta)
        if self.normalize:
            npair = self.kappa.shape[0]
            N = N - self.N0 - K[:, 3:3 + npair] @ self.kappa
            dN = dN.copy()
            dN[:, 3:3 + npair] -= self.kappa
        return N, dN, d2N


def energy(F, model):
    """Psi(F) = N(K(F)) (eq. comp-se), plus normalisation if enabled."""
    K = features(F, model.Avec)
    if model.normalize:
        npair = model.kappa.shape[0]
        return micnn_value(K, model.hidden, model.a, model.b) - model.N0 - K[:, 3:3 + npair] @ model.kappa
    return micnn_value(K, model.hidden, model.a, model.b)


# ----------------------------------------------------------------------------
# CGO push-forward tensors G^m, GG^m (eqs. second-and-fourth; App. A.2)
# ----------------------------------------------------------------------------
def _raw_tables(Bs, a_list, prs):
    """Standard-invariant tables of App. A.2.1 evaluated with left tensor Bs
    and current structural vectors a_list (the isochoric versions are the same
    tables with B~ and a~, App. A.2.2).  Returns dicts G, GG keyed by name."""
    n = Bs.shape[0]
    I = np.broadcast_to(EYE, Bs.shape)
    trB = np.einsum("...ii->...", Bs)
    B2 = np.einsum("...ij,...jk->...ik", Bs, Bs)
    O4 = np.zeros((n, 3, 3, 3, 3), dtype=Bs.dtype)
    G = {"1": Bs, "2": Bs * trB[:, None, None] - B2}
    GG = {"1": O4, "2": _outer(Bs, Bs) - _boxtimes(Bs, Bs)}
    for k, (i, j) in enumerate(prs):
        M = _sym(np.einsum("...i,...j->...ij", a_list[i], a_list[j]))
        G[("4", k)] = M
        GG[("4", k)] = O4
        G[("5", k)] = np.einsum("...ij,...jk->...ik", Bs, M) + np.einsum("...ij,...jk->...ik", M, Bs)  # R1
        GG[("5", k)] = _boxtimes(Bs, M) + _boxtimes(M, Bs)
    return G, GG


def feature_tables(F, Avec):
    """G^m and GG^m for every feature K_m (push-forward of dK_m/dC and
    d2K_m/dCdC), built from the isochoric tables (App. A.2.2, readings R1, R2)
    and the volumetric J table, chained through the feature transforms (R6).
    Returns K (n,p), G (n,p,3,3), GG (n,p,3,3,3,3)."""
    n = F.shape[0]
    J = _det3(F)
    I3 = J * J
    Bfull = np.einsum("...iK,...jK->...ij", F, F)
    Jm23 = I3 ** (-1.0 / 3.0)   # J^{-2/3}
    Jm13 = I3 ** (-1.0 / 6.0)   # J^{-1/3}
    Bt = Bfull * Jm23[:, None, None]
    n_sv = Avec.shape[0]
    prs = pairs(n_sv)
    a_cur = [np.einsum("...iJ,J->...i", F, Avec[i]) for i in range(n_sv)]
    at = [x * Jm13[:, None] for x in a_cur]
    Gt, GGt = _raw_tables(Bt, at, prs)
    I = np.broadcast_to(EYE, (n, 3, 3)).astype(F.dtype)
    IxI = _outer(I, I)
    IbI = _boxtimes(I, I)

    inv = invariants(F, Avec)
    Itil = {"1": inv["I1"] * Jm23, "2": inv["I2"] * Jm23 ** 2}
    alpha = {"1": -1.0 / 3.0, "2": -2.0 / 3.0}
    for k in range(len(prs)):
        Itil[("4", k)] = inv["I4"][k] * Jm23
        Itil[("5", k)] = inv["I5"][k] * Jm23 ** 2
        alpha[("4", k)] = -1.0 / 3.0
        alpha[("5", k)] = -2.0 / 3.0

    def iso(key):
        """G, GG of the isochoric invariant I~ (App. A.2.2)."""
        al = alpha[key]
        It = Itil[key][:, None, None]
        g = Gt[key] + al * It * I
        gg = GGt[key] + al * (_outer(I, Gt[key]) + _outer(Gt[key], I)
                              + It[..., None, None] * (al * IxI - IbI))
        return g, gg

    Gs, GGs, Ks = [], [], []
    # K1 = I1~ - 3
    g, gg = iso("1")
    Ks.append(Itil["1"] - 3.0); Gs.append(g); GGs.append(gg)
    # K2 = I2~^{3/2} - 3^{3/2}:  f' = 1.5 I~^{1/2}, f'' = 0.75 I~^{-1/2}
    g, gg = iso("2")
    I2t = Itil["2"]
    f1 = 1.5 * I2t ** 0.5
    f2 = 0.75 * I2t ** (-0.5)
    Ks.append(I2t ** 1.5 - S32)
    Gs.append(f1[:, None, None] * g)
    GGs.append(f1[:, None, None, None, None] * gg + f2[:, None, None, None, None] * _outer(g, g))
    # K3 = (J - 1)^2 with the J table G = J/2 I, GG = J/4 (I(x)I - 2 I[x]I)
    gJ = 0.5 * J[:, None, None] * I
    ggJ = 0.25 * J[:, None, None, None, None] * (IxI - 2.0 * IbI)
    f1 = 2.0 * (J - 1.0)
    Ks.append((J - 1.0) ** 2)
    Gs.append(f1[:, None, None] * gJ)
    GGs.append(f1[:, None, None, None, None] * ggJ + 2.0 * _outer(gJ, gJ))
    for kind in ("4", "5"):
        for k, (i, j) in enumerate(prs):
            g, gg = iso((kind, k))
            Ks.append(Itil[(kind, k)] - Avec[i] @ Avec[j])
            Gs.append(g)
            GGs.append(gg)
    return np.stack(Ks, -1), np.stack(Gs, 1), np.stack(GGs, 1)


def stress_stiffness(F, model, inner=None):
    """Psi, P = dPsi/dF and AA = d2Psi/dFdF (row-major F_iJ) via the paper's
    route: Kirchhoff tau = 2 sum N_m G^m (eq. stress-cgo), spatial stiffness
    cc = 4 sum N_mn G^m (x) G^n + 4 sum N_m GG^m (eq. stiffnes-cgo, R3), pulled
    back with App. A.1:  P = tau F^{-T},
    AA_iJkL = F^{-1}_Jj (cc_ijkl + delta_ik tau_jl) F^{-1}_Ll.

    ``inner`` optionally replaces the network by any callable K -> (N, dN, d2N).
    Returns dict(psi (n,), P (n,3,3), A (n,3,3,3,3), tau, cc, K, dN, d2N).
    """
    K, G, GG = feature_tables(F, model.Avec)
    fn = inner if inner is not None else model.inner
    N, dN, d2N = fn(K)
    tau = 2.0 * np.einsum("nm,nmij->nij", dN, G)
    GN = np.einsum("nmo,nokl->nmkl", d2N, G)
    cc = (4.0 * np.einsum("nmij,nmkl->nijkl", G, GN)
          + 4.0 * np.einsum("nm,nmijkl->nijkl", dN, GG))
    Fi = _inv3(F)
    P = np.einsum("nij,nJj->niJ", tau, Fi)
    I = np.eye(3)
    AA = np.einsum("nJj,nijkl,nLl->niJkL", Fi, cc + np.einsum("ik,njl->nijkl", I, tau), Fi)
    return dict(psi=N, P=P, A=AA, tau=tau, cc=cc, K=K, dN=dN, d2N=d2N)


def model_from_theta(theta, p, h, L, Avec, normalize=False, has_bias=True):
    """Unpack a parameter vector (layout documented in the input generators)."""
    theta = np.asarray(theta)
    off = 0

    def take(shape):
        nonlocal off
        cnt = int(np.prod(shape))
        x = theta[off:off + cnt].reshape(shape)
        off += cnt
        return x

    W1 = take((h, p))
    c1 = take((h,)) if has_bias else np.zeros(h, dtype=theta.dtype)
    hidden = [(W1, None, c1)]
    for _ in range(2, L + 1):
        A = take((h, h))
        B = take((h, p))
        c = take((h,)) if has_bias else np.zeros(h, dtype=theta.dtype)
        hidden.append((A, B, c))
    a = take((h,))
    b = take((p,))
    if off != theta.size:
        raise ValueError("parameter vector has the wrong length")
    return Model(hidden, a, b, Avec, normalize=normalize)
