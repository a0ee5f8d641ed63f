"""Thin PyTorch binding of the C ABI (argument marshalling only).

Tensors carry device memory; every computation runs in the HIP kernels of
libpa.so on the caller's current stream.  Names follow the C entry points
without the ``pa_`` prefix.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

__all__ = ["Model", "FEMesh", "invariants", "energy_stress_tangent", "element_residual_stiffness",
           "assemble_csr", "tangent_build", "param_backward", "num_params", "num_inputs", "PaStress",
           "stress", "energy_stress_tangent_noalloc", "noalloc_max_points"]


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(device):
    """A device with its index filled in ("cuda" is the current device)."""
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def _need(t, name, numel, dtype=torch.float64, device=None):
    """Checks, before anything is launched, that a tensor handed to the
    library has the element type, device and size the C entry point reads or
    writes (a wrong one would make a kernel read or write past its end)."""
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (got device {t.device})")
    if device is not None and t.device != _dev(device):
        raise ValueError(f"{name} is on {t.device}, the model is on {_dev(device)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, {numel} expected")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _desc(n_sv, width, n_hidden, A=None, normalize=False, has_bias=True, algorithm="forward", kind="micnn"):
    d = L.ModelDesc()
    d.n_sv = int(n_sv)
    if A is not None:
        A = np.asarray(A, dtype=np.float64).reshape(-1, 3)
        for i in range(min(2, A.shape[0])):
            for j in range(3):
                d.A[i][j] = float(A[i, j])
    d.n_hidden = int(n_hidden)
    d.width = int(width)
    d.activation = L.PA_ACT_SOFTPLUS
    d.normalize = int(bool(normalize))
    d.has_bias = int(bool(has_bias))
    d.algorithm = L.ALGORITHMS[algorithm] if isinstance(algorithm, str) else int(algorithm)
    d.kind = L.MODEL_KINDS[kind] if isinstance(kind, str) else int(kind)
    return d


def num_inputs(n_sv: int) -> int:
    lib = L.load()
    return lib.pa_num_inputs(C.byref(_desc(n_sv, 16, 2)))


def num_params(n_sv: int, width: int, n_hidden: int, has_bias: bool = True) -> int:
    lib = L.load()
    return lib.pa_num_params(C.byref(_desc(n_sv, width, n_hidden, has_bias=has_bias)))


def _prec(prec):
    return L.PRECISIONS[prec] if isinstance(prec, str) else int(prec)


class Model:
    """A neural constitutive model resident on the GPU (parameters prepared
    once by ``pa_prepare_params``)."""

    def __init__(self, theta, n_sv, width=16, n_hidden=2, A=None, normalize=False, has_bias=True,
                 algorithm="forward", device="cuda", kind="micnn"):
        """kind: "micnn" (eq. icnn), "cann" (App. B.1) or "gent_thomas" (eq. gt);
        width (1..16, 32 or 64) and n_hidden (2..4) apply to the MICNN only.
        algorithm: "forward" (Alg. 4; 2-3 hidden layers, every precision) or
        "adjoint" (adjoint-form Hessian; every precision: "fp64", "fp32", "bf16",
        "bf16_corr" and the mixed one-pass "bf16_jac")."""
        self.lib = L.load()
        self.desc = _desc(n_sv, width, n_hidden, A, normalize, has_bias, algorithm, kind)
        self.n_sv, self.width, self.n_hidden = int(n_sv), int(width), int(n_hidden)
        self.p = self.lib.pa_num_inputs(C.byref(self.desc))
        self.n_params = self.lib.pa_num_params(C.byref(self.desc))
        if not self.lib.pa_supported(C.byref(self.desc)):
            raise L.PaError(f"unsupported model: {self.lib.pa_last_error().decode()}")
        self.device = _dev(device)
        self._key = None
        self.set_params(theta)

    def _prepare(self, th):
        nb = self.lib.pa_prepared_bytes(C.byref(self.desc))
        prepared = torch.empty(nb, dtype=torch.uint8, device=self.device)
        _need(th, "theta", self.n_params, device=self.device)
        L.check(self.lib.pa_prepare_params(C.byref(self.desc), _p(th), _p(prepared), _stream()),
                "pa_prepare_params")
        return prepared

    def set_params(self, theta):
        th = torch.as_tensor(theta, dtype=torch.float64, device=self.device).contiguous().reshape(-1)
        if th.numel() != self.n_params:
            raise ValueError(f"theta has {th.numel()} entries, model needs {self.n_params}")
        self.theta = th
        self.prepared = self._prepare(th)
        self._key = (th.data_ptr(), th._version)

    def prepared_for(self, theta):
        """Prepared buffer of this parameter tensor: the model's own when
        theta is the tensor it last prepared and has not been modified since,
        otherwise a new buffer prepared from theta (the model keeps it, so a
        later call with the same unmodified tensor reuses it).  The returned
        buffer is never written again, so a caller may hold on to it (the
        autograd Function keeps the one its forward used for its backward)."""
        th = theta.detach()
        if th.dtype != torch.float64 or th.device != self.device or not th.is_contiguous():
            th = th.to(device=self.device, dtype=torch.float64).contiguous()
        th = th.reshape(-1)
        if th.numel() != self.n_params:
            raise ValueError(f"theta has {th.numel()} entries, model needs {self.n_params}")
        key = (theta.data_ptr(), theta._version)
        if key != self._key:
            self.theta = th
            self.prepared = self._prepare(th)
            self._key = key
        return self.prepared

    @property
    def algorithm(self):
        return self.desc.algorithm

    @property
    def algorithm_name(self):
        return {v: k for k, v in L.ALGORITHMS.items()}[self.desc.algorithm]

    @algorithm.setter
    def algorithm(self, a):
        self.desc.algorithm = L.ALGORITHMS[a] if isinstance(a, str) else int(a)


def _soa9(F):
    """(n, 3, 3) or (n, 9) -> contiguous (9, n); (9, n) passes through."""
    if F.dim() == 3:
        return F.reshape(F.shape[0], 9).t().contiguous()
    if F.dim() == 2 and F.shape[0] == 9 and F.shape[1] != 9:
        return F.contiguous()
    return F.reshape(-1, 9).t().contiguous()


def invariants(model: Model, F, soa: bool = False):
    """I_raw (4 + 2 npair, n), K (p, n), dKdF (p, 9, n)."""
    Fs = F if soa else _soa9(F)
    n = Fs.shape[1]
    _need(Fs, "F", 9 * n, device=model.device)
    npair = model.n_sv * (model.n_sv + 1) // 2
    I_raw = torch.empty((4 + 2 * npair, n), dtype=torch.float64, device=Fs.device)
    K = torch.empty((model.p, n), dtype=torch.float64, device=Fs.device)
    dK = torch.empty((model.p, 9, n), dtype=torch.float64, device=Fs.device)
    L.check(model.lib.pa_invariants(C.byref(model.desc), n, _p(Fs), _p(I_raw), _p(K), _p(dK), _stream()),
            "pa_invariants")
    return I_raw, K, dK


def energy_stress_tangent(model: Model, F, prec="fp64", psi=True, P=True, A=True, soa=False,
                          n_bad=None, workspace=None, out=None, prepared=None, batch=None):
    """Psi (n,), P (9, n), AA (81, n) in SoA layout (as returned by the
    library).  ``F`` is (n, 3, 3) or, with soa=True, (9, n).  ``prepared``:
    a prepared-parameter buffer of this model (default: the model's own).
    ``batch``: evaluate in batches of that many points
    (pa_energy_stress_tangent_batched; same outputs, workspace of one batch)."""
    Fs = F if soa else _soa9(F)
    n = Fs.shape[1]
    dev = Fs.device
    _need(Fs, "F", 9 * n, device=model.device)
    if out is None:
        out = {}
        if psi:
            out["psi"] = torch.empty(n, dtype=torch.float64, device=dev)
        if P:
            out["P"] = torch.empty((9, n), dtype=torch.float64, device=dev)
        if A:
            out["A"] = torch.empty((81, n), dtype=torch.float64, device=dev)
    _need(out.get("psi"), "psi", n, device=model.device)
    _need(out.get("P"), "P", 9 * n, device=model.device)
    _need(out.get("A"), "A", 81 * n, device=model.device)
    _need(n_bad, "n_bad", 1, torch.int32, device=model.device)
    ws_bytes = model.lib.pa_material_workspace_bytes(C.byref(model.desc), n if batch is None else min(batch, n))
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    prep = model.prepared if prepared is None else prepared
    if batch is not None:
        L.check(model.lib.pa_energy_stress_tangent_batched(
            C.byref(model.desc), _p(prep), _prec(prec), n, int(batch), _p(Fs), _p(out.get("psi")),
            _p(out.get("P")), _p(out.get("A")), _p(n_bad), _p(workspace), workspace.numel(), _stream()),
            "pa_energy_stress_tangent_batched")
        return out
    L.check(model.lib.pa_energy_stress_tangent(
        C.byref(model.desc), _p(prep), _prec(prec), n, _p(Fs), _p(out.get("psi")), _p(out.get("P")),
        _p(out.get("A")), _p(n_bad), _p(workspace), workspace.numel(), _stream()), "pa_energy_stress_tangent")
    return out


def energy_stress_tangent_noalloc(model: Model, F, prec="fp64", psi=True, P=True, A=True, soa=False,
                                  n_bad=None, out=None):
    """``energy_stress_tangent`` through ``pa_energy_stress_tangent_noalloc``:
    the library takes no workspace from the caller and allocates nothing (its
    own device scratch array serves); at most ``noalloc_max_points(model)``
    points per call.  The outputs are the caller's (allocated here when
    ``out`` is None)."""
    Fs = F if soa else _soa9(F)
    n = Fs.shape[1]
    dev = Fs.device
    _need(Fs, "F", 9 * n, device=model.device)
    if out is None:
        out = {}
        if psi:
            out["psi"] = torch.empty(n, dtype=torch.float64, device=dev)
        if P:
            out["P"] = torch.empty((9, n), dtype=torch.float64, device=dev)
        if A:
            out["A"] = torch.empty((81, n), dtype=torch.float64, device=dev)
    _need(out.get("psi"), "psi", n, device=model.device)
    _need(out.get("P"), "P", 9 * n, device=model.device)
    _need(out.get("A"), "A", 81 * n, device=model.device)
    _need(n_bad, "n_bad", 1, torch.int32, device=model.device)
    L.check(model.lib.pa_energy_stress_tangent_noalloc(
        C.byref(model.desc), _p(model.prepared), _prec(prec), n, _p(Fs), _p(out.get("psi")), _p(out.get("P")),
        _p(out.get("A")), _p(n_bad), _stream()), "pa_energy_stress_tangent_noalloc")
    return out


def noalloc_max_points(model: Model) -> int:
    """Largest batch ``energy_stress_tangent_noalloc`` accepts for this model."""
    return int(model.lib.pa_noalloc_max_points(C.byref(model.desc)))


def energy_stress_tangent_voigt(model: Model, F, prec="fp64", psi=True, tau=True, cc=True, soa=False,
                                n_bad=None, workspace=None, out=None):
    """Psi (n,), Kirchhoff tau (6, n) and spatial tangent cc (21, n) in Voigt
    slots (11, 22, 33, 23, 13, 12); cc holds the upper triangle of the 6 x 6
    matrix row by row.  ``F`` is (n, 3, 3) or, with soa=True, (9, n)."""
    Fs = F if soa else _soa9(F)
    n = Fs.shape[1]
    dev = Fs.device
    _need(Fs, "F", 9 * n, device=model.device)
    if out is None:
        out = {}
        if psi:
            out["psi"] = torch.empty(n, dtype=torch.float64, device=dev)
        if tau:
            out["tau"] = torch.empty((6, n), dtype=torch.float64, device=dev)
        if cc:
            out["cc"] = torch.empty((21, n), dtype=torch.float64, device=dev)
    _need(out.get("psi"), "psi", n, device=model.device)
    _need(out.get("tau"), "tau", 6 * n, device=model.device)
    _need(out.get("cc"), "cc", 21 * n, device=model.device)
    _need(n_bad, "n_bad", 1, torch.int32, device=model.device)
    ws_bytes = model.lib.pa_material_workspace_bytes(C.byref(model.desc), n)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    L.check(model.lib.pa_energy_stress_tangent_voigt(
        C.byref(model.desc), _p(model.prepared), _prec(prec), n, _p(Fs), _p(out.get("psi")), _p(out.get("tau")),
        _p(out.get("cc")), _p(n_bad), _p(workspace), workspace.numel(), _stream()),
        "pa_energy_stress_tangent_voigt")
    return out


VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def voigt_unpack(tau, cc):
    """(6, n), (21, n) Voigt arrays -> tau (n, 3, 3), cc (n, 3, 3, 3, 3) with
    the minor and major symmetries restored (host helper for callers and
    tests)."""
    tau = tau.cpu().numpy() if hasattr(tau, "cpu") else np.asarray(tau)
    cc = cc.cpu().numpy() if hasattr(cc, "cpu") else np.asarray(cc)
    n = tau.shape[1]
    T = np.zeros((n, 3, 3))
    for a, (i, j) in enumerate(VOIGT):
        T[:, i, j] = T[:, j, i] = tau[a]
    Cm = np.zeros((n, 3, 3, 3, 3))
    t = 0
    for a in range(6):
        for b in range(a, 6):
            (i, j), (k, l) = VOIGT[a], VOIGT[b]
            for (p_, q_) in {(i, j), (j, i)}:
                for (r_, s_) in {(k, l), (l, k)}:
                    Cm[:, p_, q_, r_, s_] = cc[t]
                    Cm[:, r_, s_, p_, q_] = cc[t]
            t += 1
    return T, Cm


def _morton3(q):
    """Morton (Z-order) keys of non-negative integer triples q [n, 3] < 2^21."""
    key = np.zeros(q.shape[0], dtype=np.uint64)
    for b in range(21):
        for d in range(3):
            key |= ((q[:, d].astype(np.uint64) >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + d)
    return key


class FEMesh:
    """Device-resident mesh: geometry, CSR pattern, element->CSR map, node
    incidence and a colouring.  ``perm[i]`` is the original id of element i.

    order="colour": elements renumbered colour by colour, so every colour is
    a contiguous range (needed by the fused coloured build).
    order="morton": elements in the Z-order of their centroids, so elements
    that share nodes are close in memory and in launch order (the node
    gathers of the F pass and the element-table reads of the node-centric
    assembly then hit the caches); the coloured assembly of element tables
    walks the colours through ``elem_perm``.
    order="native": elements as given.
    ``inline_geometry``: the tangent builds recompute shape gradients and
    weights from the node coordinates instead of reading the stored ones
    (same values, less memory traffic)."""

    def __init__(self, X, conn, colour=None, device="cuda", inline_geometry=True, order="colour"):
        self.lib = lib = L.load()
        X = np.ascontiguousarray(X, dtype=np.float64)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        n_el, nen = conn.shape
        self.nen, self.n_el, self.n_nodes = nen, n_el, X.shape[0]
        self.nq = 8 if nen == 8 else 4
        self.nd = 3 * nen
        if colour is None:
            colour = np.empty(n_el, dtype=np.int32)
            nc = C.c_int32()
            L.check(lib.pa_colour_elements(nen, n_el, self.n_nodes, conn.ctypes.data_as(C.c_void_p),
                                           colour.ctypes.data_as(C.c_void_p), C.byref(nc)), "pa_colour_elements")
        colour = np.asarray(colour, dtype=np.int32)
        if order not in ("colour", "morton", "native"):
            raise ValueError(f"unknown element order {order!r}")
        self.order = order
        if order == "colour":
            self.perm = np.argsort(colour, kind="stable").astype(np.int64)
        elif order == "morton" and n_el:
            cen = X[conn].mean(axis=1)
            lo, span = cen.min(axis=0), np.ptp(cen, axis=0).max()
            qz = np.floor((cen - lo) / (span if span > 0 else 1.0) * ((1 << 20) - 1)).astype(np.int64)
            self.perm = np.argsort(_morton3(qz), kind="stable").astype(np.int64)
        else:
            self.perm = np.arange(n_el, dtype=np.int64)
        self.conn_host = np.ascontiguousarray(conn[self.perm])
        mcol = colour[self.perm]  # colour of element i of the mesh
        counts = np.bincount(mcol, minlength=int(mcol.max()) + 1 if n_el else 0)
        self.colour_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        self.n_colours = len(counts)
        dev = _dev(device)
        self.device = dev
        # elements of the mesh listed colour by colour (identity for order="colour")
        self.elem_perm = None if order == "colour" else torch.tensor(
            np.argsort(mcol, kind="stable").astype(np.int32), device=dev)
        self.X = torch.tensor(X.T.copy(), device=dev)
        self.conn = torch.tensor(self.conn_host.T.copy(), device=dev)
        self.dNdX = torch.empty((self.nq, nen, 3, n_el), dtype=torch.float64, device=dev)
        self.w = torch.empty((self.nq, n_el), dtype=torch.float64, device=dev)
        self.n_bad = torch.zeros(1, dtype=torch.int32, device=dev)
        L.check(lib.pa_mesh_geometry(nen, n_el, self.n_nodes, _p(self.X), _p(self.conn), _p(self.dNdX), _p(self.w),
                                     _p(self.n_bad), _stream()), "pa_mesh_geometry")
        nnz = C.c_int64()
        cp = self.conn_host.ctypes.data_as(C.c_void_p)
        L.check(lib.pa_csr_pattern(nen, n_el, self.n_nodes, cp, None, None, C.byref(nnz)), "pa_csr_pattern")
        self.nnz = nnz.value
        row_ptr = np.empty(3 * self.n_nodes + 1, dtype=np.int64)
        col = np.empty(self.nnz, dtype=np.int32)
        L.check(lib.pa_csr_pattern(nen, n_el, self.n_nodes, cp, row_ptr.ctypes.data_as(C.c_void_p),
                                   col.ctypes.data_as(C.c_void_p), C.byref(nnz)), "pa_csr_pattern")
        self.row_ptr_host, self.col_host = row_ptr, col
        self.row_ptr = torch.tensor(row_ptr, device=dev)
        self.col = torch.tensor(col, device=dev)
        self.e2csr = torch.empty((n_el, nen, nen), dtype=torch.int32, device=dev)
        self.c_mesh = L.Mesh(n_el, self.n_nodes, nen, self.nq, self.conn.data_ptr(), self.dNdX.data_ptr(),
                             self.w.data_ptr(), self.X.data_ptr() if inline_geometry else None)
        self.c_csr = L.Csr(3 * self.n_nodes, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                           self.e2csr.data_ptr())
        L.check(lib.pa_element_csr_map(C.byref(self.c_mesh), C.byref(self.c_csr), _p(self.e2csr), _stream()),
                "pa_element_csr_map")
        self.c_col = L.Colouring(self.n_colours, self.colour_ptr.ctypes.data_as(C.c_void_p).value,
                                 None if self.elem_perm is None else self.elem_perm.data_ptr())
        # node incidence for the gather assembly
        inc_ptr = np.empty(self.n_nodes + 1, dtype=np.int64)
        inc_ent = np.empty(n_el * nen, dtype=np.int32)
        L.check(lib.pa_node_incidence(nen, n_el, self.n_nodes, cp, inc_ptr.ctypes.data_as(C.c_void_p),
                                      inc_ent.ctypes.data_as(C.c_void_p)), "pa_node_incidence")
        self.inc_ptr_host, self.inc_ent_host = inc_ptr, inc_ent
        self.inc_ptr = torch.tensor(inc_ptr, device=dev)
        self.inc_ent = torch.tensor(inc_ent, device=dev)
        self.max_row = int(np.diff(row_ptr).max()) if self.n_nodes else 0
        self.c_inc = L.Incidence(self.n_nodes, n_el * nen, self.max_row, self.inc_ptr.data_ptr(),
                                 self.inc_ent.data_ptr())

    def workspace_bytes(self, model: Model, assembly: str = "coloured") -> int:
        if assembly == "gather":
            return self.lib.pa_gather_workspace_bytes(C.byref(model.desc), C.byref(self.c_mesh))
        return self.lib.pa_element_workspace_bytes(C.byref(model.desc), C.byref(self.c_mesh))


def element_residual_stiffness(model: Model, mesh: FEMesh, u, prec="fp64", stiffness=True, workspace=None,
                               r_e=None, K_e=None, n_bad=None):
    """r_e (nd, n_el) and K_e (nd, nd, n_el), element index fastest, for the
    mesh's (colour-ordered) elements.  u: (n_nodes, 3) or (3 n_nodes,)
    displacement, dof = 3*node + i."""
    u = u.reshape(-1).contiguous()
    dev = u.device
    _need(u, "u", 3 * mesh.n_nodes, device=mesh.device)
    if r_e is None:
        r_e = torch.empty((mesh.nd, mesh.n_el), dtype=torch.float64, device=dev)
    if stiffness and K_e is None:
        K_e = torch.empty((mesh.nd, mesh.nd, mesh.n_el), dtype=torch.float64, device=dev)
    _need(r_e, "r_e", mesh.nd * mesh.n_el, device=mesh.device)
    _need(K_e if stiffness else None, "K_e", mesh.nd * mesh.nd * mesh.n_el, device=mesh.device)
    _need(n_bad, "n_bad", 1, torch.int32, device=mesh.device)
    nb = mesh.workspace_bytes(model)
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(nb, dtype=torch.uint8, device=dev)
    L.check(model.lib.pa_element_residual_stiffness(
        C.byref(model.desc), _p(model.prepared), _prec(prec), C.byref(mesh.c_mesh), _p(u), _p(r_e),
        _p(K_e if stiffness else None), _p(n_bad), _p(workspace), workspace.numel(), _stream()),
        "pa_element_residual_stiffness")
    return r_e, K_e


def assemble_csr(mesh: FEMesh, r_e, K_e, r=None, vals=None, zero_first=True):
    """Coloured scatter-assembly into the global residual and CSR values."""
    dev = mesh.device
    if r is None and r_e is not None:
        r = torch.empty(3 * mesh.n_nodes, dtype=torch.float64, device=dev)
    if vals is None and K_e is not None:
        vals = torch.empty(mesh.nnz, dtype=torch.float64, device=dev)
    _need(r_e, "r_e", mesh.nd * mesh.n_el, device=dev)
    _need(K_e, "K_e", mesh.nd * mesh.nd * mesh.n_el, device=dev)
    _need(r, "r", 3 * mesh.n_nodes, device=dev)
    _need(vals, "vals", mesh.nnz, device=dev)
    L.check(mesh.lib.pa_assemble_csr(C.byref(mesh.c_mesh), C.byref(mesh.c_col), C.byref(mesh.c_csr), _p(r_e),
                                     _p(K_e), _p(r), _p(vals), int(bool(zero_first)), _stream()), "pa_assemble_csr")
    return r, vals


def tangent_build(model: Model, mesh: FEMesh, u, prec="fp64", workspace=None, bufs=None, fused=True,
                  n_bad=None, assembly="gather"):
    """One Newton tangent build: u -> (r, CSR values).

    assembly="gather" (default) runs pa_tangent_build_gather (element-major
    tables, then one pass per node writing its CSR rows once);
    assembly="coloured" with fused=True runs pa_tangent_build (element rows
    scattered straight into CSR colour by colour); fused=False runs
    pa_element_residual_stiffness then pa_assemble_csr."""
    bufs = bufs if bufs is not None else {}
    if assembly not in ("gather", "coloured"):
        raise ValueError(f"unknown assembly {assembly!r}")
    if assembly == "coloured" and not fused:
        r_e, K_e = element_residual_stiffness(model, mesh, u, prec, workspace=workspace,
                                              r_e=bufs.get("r_e"), K_e=bufs.get("K_e"), n_bad=n_bad)
        r, vals = assemble_csr(mesh, r_e, K_e, r=bufs.get("r"), vals=bufs.get("vals"))
        bufs.update(r_e=r_e, K_e=K_e, r=r, vals=vals)
        return r, vals
    if assembly == "coloured" and mesh.order != "colour":
        raise ValueError("the fused coloured build needs a mesh numbered colour by colour (order='colour')")
    u = u.reshape(-1).contiguous()
    dev = u.device
    r = bufs.get("r")
    vals = bufs.get("vals")
    if r is None:
        r = torch.empty(3 * mesh.n_nodes, dtype=torch.float64, device=dev)
    if vals is None:
        vals = torch.empty(mesh.nnz, dtype=torch.float64, device=dev)
    _need(u, "u", 3 * mesh.n_nodes, device=mesh.device)
    _need(r, "r", 3 * mesh.n_nodes, device=mesh.device)
    _need(vals, "vals", mesh.nnz, device=mesh.device)
    _need(n_bad, "n_bad", 1, torch.int32, device=mesh.device)
    if assembly == "gather":
        nb = mesh.workspace_bytes(model, "gather")
        if workspace is None or workspace.numel() < nb:
            workspace = torch.empty(nb, dtype=torch.uint8, device=dev)
        L.check(model.lib.pa_tangent_build_gather(
            C.byref(model.desc), _p(model.prepared), _prec(prec), C.byref(mesh.c_mesh), C.byref(mesh.c_inc),
            C.byref(mesh.c_csr), _p(u), _p(r), _p(vals), _p(n_bad), _p(workspace), workspace.numel(), _stream()),
            "pa_tangent_build_gather")
        bufs.update(r=r, vals=vals)
        return r, vals
    nb = mesh.workspace_bytes(model)
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(nb, dtype=torch.uint8, device=dev)
    L.check(model.lib.pa_tangent_build(C.byref(model.desc), _p(model.prepared), _prec(prec), C.byref(mesh.c_mesh),
                                       C.byref(mesh.c_col), C.byref(mesh.c_csr), _p(u), _p(r), _p(vals), _p(n_bad),
                                       _p(workspace), workspace.numel(), _stream()), "pa_tangent_build")
    bufs.update(r=r, vals=vals)
    return r, vals


def residual_loss(r, dof_group, R):
    """Residual loss of eq. (loss) for one time step and its cotangent:
    returns (L (1,) tensor, r_bar).  dof_group: int32 per dof, -1 free, b >= 0
    reaction boundary b, -2 constrained and unobserved; R: reaction forces."""
    lib = L.load()
    r = r.reshape(-1).contiguous()
    _need(r, "r", None)
    grp = dof_group.to(device=r.device, dtype=torch.int32).contiguous().reshape(-1)
    Rt = torch.as_tensor(R, dtype=torch.float64, device=r.device).reshape(-1).contiguous()
    _need(grp, "dof_group", r.numel(), torch.int32, device=r.device)
    if grp.numel() and (int(grp.min()) < -2 or int(grp.max()) >= Rt.numel()):
        raise ValueError(f"dof_group entries must lie in [-2, {Rt.numel()}) (one group per reaction force)")
    nb = lib.pa_residual_loss_workspace(r.numel(), Rt.numel())
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=r.device)
    loss = torch.empty(1, dtype=torch.float64, device=r.device)
    rbar = torch.empty_like(r)
    L.check(lib.pa_residual_loss(r.numel(), _p(r), _p(grp), Rt.numel(), _p(Rt), _p(loss), _p(rbar), _p(ws),
                                 ws.numel(), _stream()), "pa_residual_loss")
    return loss, rbar


def residual_param_backward(model: Model, mesh: FEMesh, u, r_bar, prec="fp64"):
    """theta_bar = (dr/dtheta)^T r_bar for the raw network."""
    u = u.reshape(-1).contiguous()
    rb = r_bar.reshape(-1).contiguous()
    _need(u, "u", 3 * mesh.n_nodes, device=model.device)
    _need(rb, "r_bar", 3 * mesh.n_nodes, device=model.device)
    out = torch.empty(model.n_params, dtype=torch.float64, device=u.device)
    nb = model.lib.pa_residual_param_backward_workspace(C.byref(model.desc), C.byref(mesh.c_mesh), _prec(prec))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=u.device)
    L.check(model.lib.pa_residual_param_backward(C.byref(model.desc), _p(model.prepared), _prec(prec),
                                                 C.byref(mesh.c_mesh), _p(u), _p(rb), _p(out), _p(ws), ws.numel(),
                                                 _stream()), "pa_residual_param_backward")
    return out


def residual_loss_and_grad(model: Model, mesh: FEMesh, u, dof_group, R, prec="fp64"):
    """Loss of eq. (loss) for one time step and its gradient in theta: the
    residual from the tangent build (node-centric assembly), the loss and
    its cotangent, then the residual's parameter adjoint."""
    r, _ = tangent_build(model, mesh, u, prec=prec, assembly="gather")
    loss, rbar = residual_loss(r, dof_group, R)
    return loss, residual_param_backward(model, mesh, u, rbar, prec)


def param_backward(model: Model, F, P_bar, prec="fp32", soa=False, workspace=None, prepared=None):
    """theta_bar = sum_q (dP_q/dtheta)^T P_bar_q (raw network).  ``prepared``:
    the prepared-parameter buffer of the theta to differentiate at (default:
    the model's own)."""
    Fs = F if soa else _soa9(F)
    Pb = P_bar if soa else _soa9(P_bar)
    n = Fs.shape[1]
    _need(Fs, "F", 9 * n, device=model.device)
    _need(Pb, "P_bar", 9 * n, device=model.device)
    out = torch.empty(model.n_params, dtype=torch.float64, device=Fs.device)
    nb = model.lib.pa_param_backward_workspace(C.byref(model.desc), _prec(prec), n)
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device=Fs.device)
    prep = model.prepared if prepared is None else prepared
    L.check(model.lib.pa_param_backward(C.byref(model.desc), _p(prep), _prec(prec), n, _p(Fs), _p(Pb),
                                        _p(out), _p(workspace), workspace.numel(), _stream()), "pa_param_backward")
    return out


class PaStress(torch.autograd.Function):
    """P(theta, F) with the hand-written parameter adjoint as its backward.

    forward: pa_energy_stress_tangent (stress only; no Hessian columns) with
    the prepared buffer of this theta (``Model.prepared_for``: prepared once
    per parameter version, reused while theta is unchanged);
    backward: pa_param_backward on that same prepared buffer (activations
    recomputed; nothing stored but theta, F and the prepared parameters), so
    the gradient is the one of the theta the forward used even when the model
    has since been given other parameters.  Gradients flow to theta only."""

    @staticmethod
    def forward(ctx, theta, F, model, prec):
        prep = model.prepared_for(theta)
        out = energy_stress_tangent(model, F, prec=prec, psi=False, P=True, A=False, prepared=prep)
        ctx.save_for_backward(theta, F)
        ctx.model, ctx.prec, ctx.prep = model, prec, prep
        return out["P"].t().reshape(-1, 3, 3)

    @staticmethod
    def backward(ctx, P_bar):
        theta, F = ctx.saved_tensors
        tb = param_backward(ctx.model, F, P_bar.contiguous(), prec=ctx.prec, prepared=ctx.prep)
        return tb.to(theta.dtype), None, None, None


def stress(theta, F, model, prec="fp32"):
    """Differentiable first Piola-Kirchhoff stress (n, 3, 3) of the raw network."""
    return PaStress.apply(theta, F, model, prec)
