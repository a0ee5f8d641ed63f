"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module draws random numbers and lays out meshes; it holds none of the
method's arithmetic (no invariants, no network, no shape functions, no
quadrature).  Every generator is seeded with NumPy's PCG64 so a given call
returns the same arrays on every machine.

Parameter packing of the inner network (the (M)ICNN of eq. (icnn), App. B.2),
with ``p`` inputs, ``L`` hidden layers of width ``h``:

    [W1 (h x p, row-major), c1 (h)]                  hidden layer 1
    for k = 2..L: [A_k (h x h), B_k (h x p), c_k (h)]  hidden layer k
    [a (h), b (p)]                                    output layer (no bias)

Layer 1 carries a single matrix because A^(1) and B^(1) both multiply the
input z^(0) (eq. icnn, Alg. 4).  With ``has_bias=False`` the c_k blocks are
omitted; this is the packing that reproduces the 675 parameters the paper lists
for a 3 x 16 MICNN on three inputs (Table "hyperparams", App. C).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "num_inputs", "num_params", "micnn_params", "unpack_params",
    "structural_vectors", "sample_F", "hex_mesh", "tet10_mesh",
    "displacement_uniform", "displacement_modes", "loading_path",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def num_inputs(n_sv: int) -> int:
    """p = 3 isotropic features + one I4 and one I5 feature per unordered pair."""
    npair = n_sv * (n_sv + 1) // 2
    return 3 + 2 * npair


def num_params(p: int, h: int, L: int, has_bias: bool = True) -> int:
    nb = 1 if has_bias else 0
    n = h * p + nb * h
    n += (L - 1) * (h * h + h * p + nb * h)
    n += h + p
    return n


def micnn_params(p: int, h: int, L: int, seed: int = 1, sigma: float = 0.3,
                 has_bias: bool = True, nonneg: bool = True) -> np.ndarray:
    """Weights ~ |N(0, sigma)| (non-negative where convexity and monotonicity
    need it, App. B.2), biases ~ N(0, sigma)."""
    r = rng(seed)

    def w(shape):
        x = r.normal(0.0, sigma, size=shape)
        return np.abs(x) if nonneg else x

    def c(shape):
        return r.normal(0.0, sigma, size=shape)

    parts = [w((h, p))]
    if has_bias:
        parts.append(c((h,)))
    for _ in range(2, L + 1):
        parts += [w((h, h)), w((h, p))]
        if has_bias:
            parts.append(c((h,)))
    parts += [w((h,)), w((p,))]
    theta = np.concatenate([x.ravel() for x in parts]).astype(np.float64)
    assert theta.size == num_params(p, h, L, has_bias)
    return theta


def unpack_params(theta: np.ndarray, p: int, h: int, L: int, has_bias: bool = True):
    """Split a packed parameter vector into per-layer arrays (views)."""
    theta = np.asarray(theta)
    off = 0

    def take(shape):
        nonlocal off
        n = int(np.prod(shape))
        x = theta[off:off + n].reshape(shape)
        off += n
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
    assert off == theta.size
    return hidden, a, b


def structural_vectors(n_sv: int) -> np.ndarray:
    """Unit reference vectors e1 (and e2)."""
    A = np.zeros((2, 3))
    A[0, 0] = 1.0
    A[1, 1] = 1.0
    return A[:n_sv].copy()


def sample_F(n: int, seed: int = 0, sigma: float = 0.15, jmin: float = 0.7,
             jmax: float = 1.4) -> np.ndarray:
    """F = R U with R Haar-random in SO(3) (normalised Gaussian quaternion) and
    U = exp(sym(G)), G ~ N(0, sigma^2)^{3x3}, rescaled so det F lies in
    [jmin, jmax].  Returns (n, 3, 3)."""
    r = rng(seed)
    q = r.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    G = r.normal(0.0, sigma, size=(n, 3, 3))
    S = 0.5 * (G + np.swapaxes(G, 1, 2))
    lam, V = np.linalg.eigh(S)
    U = np.einsum("nij,nj,nkj->nik", V, np.exp(lam), V)
    J = np.exp(lam.sum(axis=1))
    Jc = np.clip(J, jmin, jmax)
    U *= ((Jc / J) ** (1.0 / 3.0))[:, None, None]
    return np.einsum("nij,njk->nik", R, U)


def hex_mesh(n: int, length: float = 1.0):
    """Structured n^3 mesh of 8-node hexahedra on [0, length]^3.

    Node (i, j, k) has id (i*(n+1) + j)*(n+1) + k and position (i, j, k)*h.
    Element (ei, ej, ek) has id (ei*n + ej)*n + ek; its local node
    a = a0 + 2*a1 + 4*a2 sits at corner (ei+a0, ej+a1, ek+a2), i.e. at
    reference coordinates (2*a0-1, 2*a1-1, 2*a2-1).
    Returns (X [n_nodes, 3], conn [n_el, 8] int32, parity_colour [n_el] int32).
    """
    h = length / n
    m = n + 1
    i, j, k = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    X = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * h
    ei, ej, ek = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ei, ej, ek = ei.ravel(), ej.ravel(), ek.ravel()
    conn = np.empty((n ** 3, 8), dtype=np.int32)
    for a in range(8):
        a0, a1, a2 = a & 1, (a >> 1) & 1, (a >> 2) & 1
        conn[:, a] = ((ei + a0) * m + (ej + a1)) * m + (ek + a2)
    colour = ((ei & 1) + 2 * (ej & 1) + 4 * (ek & 1)).astype(np.int32)
    return X, conn, colour


# Kuhn subdivision: six tetrahedra per cube, all sharing the diagonal from the
# corner (0,0,0) to (1,1,1); tetrahedron t follows the axis permutation PERMS[t].
_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
# Local node order: vertices 0..3, then the mid-edge nodes of edges
# (0,1), (1,2), (0,2), (0,3), (1,3), (2,3).
TET10_EDGES = [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]


def tet10_mesh(n: int, length: float = 1.0):
    """Kuhn-subdivided n^3 cube mesh of 10-node tetrahedra on [0, length]^3.

    Nodes live on the half-step grid: node (I, J, K), 0 <= I,J,K <= 2n, has id
    (I*(2n+1) + J)*(2n+1) + K and position (I, J, K)*h/2.  Every half-grid
    point is a vertex or an edge midpoint of some tetrahedron.  Tetrahedra with
    a negative orientation have vertices 1 and 2 swapped so every element is
    positively oriented.  Element id = 6*cube_id + t.  Returns
    (X [n_nodes, 3], conn [n_el, 10] int32, parity_colour [n_el] int32 in 0..47).
    """
    h = length / n
    m = 2 * n + 1
    I, J, K = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    X = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1).astype(np.float64) * (h / 2)
    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    ncube = n ** 3
    conn = np.empty((ncube, 6, 10), dtype=np.int32)
    base = np.stack([ci, cj, ck], axis=1) * 2  # half-grid coords of corner 000
    colour = np.empty((ncube, 6), dtype=np.int32)
    par = (ci & 1) + 2 * (cj & 1) + 4 * (ck & 1)
    for t, perm in enumerate(_PERMS):
        verts = [np.zeros(3, dtype=np.int64)]
        cur = np.zeros(3, dtype=np.int64)
        for ax in perm:
            cur = cur.copy()
            cur[ax] += 2
            verts.append(cur)
        v = np.array(verts)  # (4, 3) offsets in half-grid units
        # orientation of the reference -> physical map
        d = np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]).astype(float))
        if d < 0:
            v = v[[0, 2, 1, 3]]
        pts = [v[a] for a in range(4)] + [(v[a] + v[b]) // 2 for (a, b) in TET10_EDGES]
        for a, off in enumerate(pts):
            g = base + off[None, :]
            conn[:, t, a] = (g[:, 0] * m + g[:, 1]) * m + g[:, 2]
        colour[:, t] = par * 6 + t
    return X, conn.reshape(ncube * 6, 10), colour.reshape(-1)


def displacement_uniform(n_nodes: int, amp: float, seed: int = 0) -> np.ndarray:
    """u = amp * U[-1, 1] per dof; dof order 3*node + i.  Returns (n_nodes, 3)."""
    return amp * rng(seed).uniform(-1.0, 1.0, size=(n_nodes, 3))


def displacement_modes(X: np.ndarray, h: float, seed: int = 0, amp: float = 0.05,
                       noise: float = 0.02) -> np.ndarray:
    """u_i = amp*sin(pi X_i) + amp*sin(pi X_{(i+1) mod 3}) + noise*h*U[-1, 1]."""
    u = amp * np.sin(np.pi * X) + amp * np.sin(np.pi * np.roll(X, -1, axis=1))
    u = u + noise * h * rng(seed).uniform(-1.0, 1.0, size=X.shape)
    return u


def loading_path(kind: str, gamma: float) -> np.ndarray:
    """Deformation gradients of the six loading paths of App. C."""
    g = float(gamma)
    F = np.eye(3)
    if kind == "UT":
        F[0, 0] = 1 + g
    elif kind == "UC":
        F[0, 0] = 1 / (1 + g)
    elif kind == "BT":
        F[0, 0] = F[1, 1] = 1 + g
    elif kind == "BC":
        F[0, 0] = F[1, 1] = 1 / (1 + g)
    elif kind == "SS":
        F[0, 1] = g
    elif kind == "PS":
        F[0, 0] = 1 + g
        F[1, 1] = 1 / (1 + g)
    else:
        raise ValueError(kind)
    return F


def reaction_groups(X: np.ndarray, tol: float = 1e-12):
    """Dof classes for the residual loss on a unit-cube mesh: the X_0 = 0
    face is clamped and unobserved (-2); on the X_0 = 1 face the dofs in
    direction 0 form reaction boundary 0; on the X_1 = 1 face the dofs in
    direction 1 form reaction boundary 1 (where not already taken); every
    other dof is free (-1).  Returns int32 [3 n_nodes], node-major."""
    n = X.shape[0]
    grp = np.full((n, 3), -1, dtype=np.int32)
    x1 = np.abs(X[:, 1] - 1.0) < tol
    grp[x1, 1] = 1
    x0 = np.abs(X[:, 0] - 1.0) < tol
    grp[x0, 0] = 0
    grp[np.abs(X[:, 0]) < tol, :] = -2
    return grp.reshape(-1)


def cann_params(p: int, seed: int = 1, sigma: float = 0.3) -> np.ndarray:
    """CANN weights (8 per input: (w1, w2) for the branches (power 1, linear),
    (power 2, linear), (power 1, exp), (power 2, exp)), all ~ |N(0, sigma)|."""
    return np.abs(rng(seed).normal(0.0, sigma, size=8 * p))


GENT_THOMAS = np.array([0.5, 1.0, 1.0])  # coefficients of eq. (gt)
