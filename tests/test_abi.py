"""The C-ABI library loads and exports every symbol include/pa.h declares;
host-only entry points (sizes, CSR pattern, colouring, argument checks) are
exercised on the CPU.  No GPU compute call is made here."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fe
from paper_2510_00884_amd import _lib as L
from paper_2510_00884_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pa.h")


def header_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pa_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libpa.so not built")
    return L.load()


def test_exports_every_declared_symbol(lib):
    syms = header_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(L.SIGNATURES), set(syms) ^ set(L.SIGNATURES)


def _desc(n_sv=2, h=32, Ld=2, has_bias=1):
    d = L.ModelDesc()
    d.n_sv, d.width, d.n_hidden, d.has_bias = n_sv, h, Ld, has_bias
    d.A[0][0] = 1.0
    d.A[1][1] = 1.0
    return d


@pytest.mark.parametrize("n_sv,h,Ld,bias", [(0, 16, 2, 1), (1, 16, 2, 1), (2, 32, 2, 1), (2, 64, 3, 1), (0, 16, 3, 0),
                                            (2, 8, 2, 1), (1, 2, 3, 0), (2, 64, 4, 1), (0, 4, 4, 1)])
def test_sizes_match_generators(lib, n_sv, h, Ld, bias):
    d = _desc(n_sv, h, Ld, bias)
    p = synth.num_inputs(n_sv)
    assert lib.pa_num_inputs(C.byref(d)) == p
    assert lib.pa_num_params(C.byref(d)) == synth.num_params(p, h, Ld, bool(bias))
    assert lib.pa_supported(C.byref(d)) == 1
    assert lib.pa_prepared_bytes(C.byref(d)) > 0


def test_argument_errors_before_launch(lib):
    d = _desc()
    d.n_sv = 3
    assert lib.pa_supported(C.byref(d)) == 0
    assert lib.pa_prepare_params(C.byref(d), C.c_void_p(8), C.c_void_p(8), None) == L.PA_ERR_ARG
    assert b"n_sv" in lib.pa_last_error()
    d = _desc(h=48)
    assert lib.pa_prepare_params(C.byref(d), C.c_void_p(8), C.c_void_p(8), None) == L.PA_ERR_UNSUPPORTED
    d = _desc(h=20)  # above 16 a width must be a multiple of 16
    assert lib.pa_prepare_params(C.byref(d), C.c_void_p(8), C.c_void_p(8), None) == L.PA_ERR_ARG
    d = _desc(Ld=5)
    assert lib.pa_supported(C.byref(d)) == 0
    d = _desc()
    rc = lib.pa_energy_stress_tangent(C.byref(d), C.c_void_p(8), 0, -1, None, None, None, None, None, None, 0, None)
    assert rc == L.PA_ERR_ARG
    rc = lib.pa_energy_stress_tangent(C.byref(d), C.c_void_p(8), 7, 10, C.c_void_p(8), None, None, None, None, None, 0, None)
    assert rc == L.PA_ERR_ARG
    rc = lib.pa_energy_stress_tangent(C.byref(d), C.c_void_p(8), 0, 10, C.c_void_p(8), None, None, None, None, None, 0, None)
    assert rc == L.PA_ERR_WORKSPACE
    m = L.Mesh(1, 8, 9, 8, 8, 8, 8)
    rc = lib.pa_element_residual_stiffness(C.byref(d), C.c_void_p(8), 0, C.byref(m), C.c_void_p(8), C.c_void_p(8),
                                           None, None, None, 0, None)
    assert rc == L.PA_ERR_ARG
    assert lib.pa_status_string(L.PA_ERR_WORKSPACE) == b"workspace too small"


@pytest.mark.parametrize("kind,n", [("hex8", 3), ("tet10", 2)])
def test_csr_pattern_matches_oracle_assembly(lib, kind, n):
    X, conn, _ = (synth.hex_mesh if kind == "hex8" else synth.tet10_mesh)(n)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    nen = conn.shape[1]
    nnz = C.c_int64()
    assert lib.pa_csr_pattern(nen, conn.shape[0], X.shape[0], conn.ctypes.data_as(C.c_void_p), None, None,
                              C.byref(nnz)) == 0
    row_ptr = np.empty(3 * X.shape[0] + 1, dtype=np.int64)
    col = np.empty(nnz.value, dtype=np.int32)
    assert lib.pa_csr_pattern(nen, conn.shape[0], X.shape[0], conn.ctypes.data_as(C.c_void_p),
                              row_ptr.ctypes.data_as(C.c_void_p), col.ctypes.data_as(C.c_void_p), C.byref(nnz)) == 0
    # the oracle's assembled matrix with all-ones element blocks has exactly this pattern
    nd = 3 * nen
    _, K = fe.assemble(conn, np.zeros((conn.shape[0], nd)), np.ones((conn.shape[0], nd, nd)), X.shape[0])
    np.testing.assert_array_equal(row_ptr, K.indptr)
    np.testing.assert_array_equal(col, K.indices)


def test_csr_pattern_c0_size(lib):
    X, conn, _ = synth.hex_mesh(8)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    nnz = C.c_int64()
    lib.pa_csr_pattern(8, conn.shape[0], X.shape[0], conn.ctypes.data_as(C.c_void_p), None, None, C.byref(nnz))
    assert nnz.value == 140625  # 8^3 hex8 mesh: 2,187 dofs, 140,625 nonzeros


@pytest.mark.parametrize("kind,n", [("hex8", 4), ("tet10", 2)])
def test_greedy_colouring_is_valid(lib, kind, n):
    X, conn, _ = (synth.hex_mesh if kind == "hex8" else synth.tet10_mesh)(n)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    colour = np.empty(conn.shape[0], dtype=np.int32)
    nc = C.c_int32()
    assert lib.pa_colour_elements(conn.shape[1], conn.shape[0], X.shape[0], conn.ctypes.data_as(C.c_void_p),
                                  colour.ctypes.data_as(C.c_void_p), C.byref(nc)) == 0
    assert colour.min() == 0 and colour.max() == nc.value - 1
    for c in range(nc.value):
        nodes = conn[colour == c].ravel()
        assert np.unique(nodes).size == nodes.size
    bad = conn.copy()
    bad[0, 0] = X.shape[0]
    assert lib.pa_colour_elements(bad.shape[1], bad.shape[0], X.shape[0], bad.ctypes.data_as(C.c_void_p),
                                  colour.ctypes.data_as(C.c_void_p), C.byref(nc)) == L.PA_ERR_ARG


@pytest.mark.parametrize("kind,n", [("hex8", 3), ("tet10", 2)])
def test_node_incidence(lib, kind, n):
    """Every (element, local node) pair appears once, under its node, in
    ascending element order."""
    X, conn, _ = (synth.hex_mesh if kind == "hex8" else synth.tet10_mesh)(n)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    n_el, nen = conn.shape
    ptr = np.empty(X.shape[0] + 1, dtype=np.int64)
    ent = np.empty(n_el * nen, dtype=np.int32)
    cp = conn.ctypes.data_as(C.c_void_p)
    assert lib.pa_node_incidence(nen, n_el, X.shape[0], cp, ptr.ctypes.data_as(C.c_void_p),
                                 ent.ctypes.data_as(C.c_void_p)) == 0
    assert ptr[0] == 0 and ptr[-1] == n_el * nen
    for i in range(X.shape[0]):
        e, a = np.divmod(ent[ptr[i]:ptr[i + 1]], nen)
        assert np.all(conn[e, a] == i)
        assert np.all(np.diff(e) > 0)
        assert ptr[i + 1] - ptr[i] == np.count_nonzero(conn == i)
    bad = conn.copy()
    bad[0, 0] = -1
    assert lib.pa_node_incidence(nen, n_el, X.shape[0], bad.ctypes.data_as(C.c_void_p),
                                 ptr.ctypes.data_as(C.c_void_p), None) == L.PA_ERR_ARG


def test_model_kinds_sizes_and_errors(lib):
    """CANN: 8 parameters per input; Gent-Thomas: 3; unknown kinds rejected;
    the parameter adjoint refuses non-MICNN kinds before any launch."""
    for n_sv, p in [(0, 3), (1, 5), (2, 9)]:
        d = L.ModelDesc()
        d.n_sv = n_sv
        d.kind = L.PA_MODEL_CANN
        assert lib.pa_num_params(C.byref(d)) == 8 * p
        assert lib.pa_supported(C.byref(d)) == 1
        assert lib.pa_prepared_bytes(C.byref(d)) >= 8 * (8 * p)
        d.kind = L.PA_MODEL_GENT_THOMAS
        assert lib.pa_num_params(C.byref(d)) == 3
        assert lib.pa_supported(C.byref(d)) == 1
    d.kind = 7
    assert lib.pa_supported(C.byref(d)) == 0
    d.kind = L.PA_MODEL_CANN
    dummy = C.c_void_p(1)
    rc = lib.pa_param_backward(C.byref(d), dummy, L.PA_FP64, 0, None, None, dummy, dummy, 1 << 20, None)
    assert rc == L.PA_ERR_UNSUPPORTED


def test_empty_mesh_is_a_no_op(lib):
    """An empty mesh returns PA_OK from the tangent builds before any launch
    (no GPU needed), once the argument checks have passed."""
    d = _desc()
    m = L.Mesh(0, 8, 8, 8, None, None, None, None)
    inc = L.Incidence(8, 0, 81, 8, None)
    csr = L.Csr(24, 0, 8, 8, 8)
    rc = lib.pa_tangent_build_gather(C.byref(d), None, 0, C.byref(m), C.byref(inc), C.byref(csr), None,
                                     C.c_void_p(8), C.c_void_p(8), None, None, 0, None)
    assert rc == L.PA_OK, lib.pa_last_error()
    # the node and CSR arrays are still required
    csr = L.Csr(24, 0, None, 8, None)
    rc = lib.pa_tangent_build_gather(C.byref(d), None, 0, C.byref(m), C.byref(inc), C.byref(csr), None,
                                     C.c_void_p(8), C.c_void_p(8), None, None, 0, None)
    assert rc == L.PA_ERR_ARG


def test_binding_argument_checks_on_host():
    """The binding's tensor checks run on the host and refuse host memory,
    the wrong element type and the wrong size (no GPU needed to see it)."""
    import torch
    from paper_2510_00884_amd import api
    with pytest.raises(ValueError, match="GPU tensor"):
        api._need(torch.zeros(9, dtype=torch.float64), "F", 9)
    with pytest.raises(ValueError, match="float64"):
        api._need(torch.zeros(9, dtype=torch.float32), "F", 9)
    with pytest.raises(ValueError, match="int32"):
        api._need(torch.zeros(9, dtype=torch.int64), "dof_group", 9, torch.int32)


def test_noalloc_limit_checked_before_launch(lib):
    """The allocation-free material call states its batch limit and refuses a
    larger batch on the host (PA_ERR_WORKSPACE, nothing launched)."""
    for n_sv, p in ((0, 3), (1, 5), (2, 9)):
        d = _desc(n_sv=n_sv)
        nmax = lib.pa_noalloc_max_points(C.byref(d))
        need = lib.pa_material_workspace_bytes(C.byref(d), nmax)
        assert 0 < need <= L.PA_NOALLOC_SCRATCH_BYTES
        assert lib.pa_material_workspace_bytes(C.byref(d), nmax + 1) > L.PA_NOALLOC_SCRATCH_BYTES
    d = _desc(n_sv=2)
    assert lib.pa_noalloc_max_points(C.byref(d)) == 131072
    rc = lib.pa_energy_stress_tangent_noalloc(C.byref(d), C.c_void_p(8), 0, 131073, C.c_void_p(8), None, None, None,
                                             None, None)
    assert rc == L.PA_ERR_WORKSPACE
    assert b"131072" in lib.pa_last_error()
    rc = lib.pa_energy_stress_tangent_noalloc(C.byref(d), C.c_void_p(8), 0, -1, C.c_void_p(8), None, None, None,
                                             None, None)
    assert rc == L.PA_ERR_ARG
    assert lib.pa_energy_stress_tangent_noalloc(C.byref(d), C.c_void_p(8), 0, 0, None, None, None, None, None,
                                               None) == L.PA_OK


def test_batched_call_arguments_checked_before_launch(lib):
    d = _desc(n_sv=2)
    ws1 = lib.pa_material_workspace_bytes(C.byref(d), 1000)
    rc = lib.pa_energy_stress_tangent_batched(C.byref(d), C.c_void_p(8), 0, 5000, 0, C.c_void_p(8), None, None,
                                              None, None, C.c_void_p(8), ws1, None)
    assert rc == L.PA_ERR_ARG
    rc = lib.pa_energy_stress_tangent_batched(C.byref(d), C.c_void_p(8), 0, 5000, 1000, C.c_void_p(8), None,
                                              None, None, None, C.c_void_p(8), ws1 - 1, None)
    assert rc == L.PA_ERR_WORKSPACE
    assert lib.pa_energy_stress_tangent_batched(C.byref(d), C.c_void_p(8), 0, 0, 1000, None, None, None, None,
                                               None, None, 0, None) == L.PA_OK


def test_pipe_probe_rejects_bad_arguments(lib):
    """The measurement probe checks its arguments on the host (no launch)."""
    out = C.c_void_p(0)
    assert lib.pa_pipe_probe(6, 0, 10, 1, C.c_void_p(1), None) == L.PA_ERR_ARG
    assert lib.pa_pipe_probe(1, -1, 10, 1, C.c_void_p(1), None) == L.PA_ERR_ARG
    assert lib.pa_pipe_probe(1, 0, 0, 1, C.c_void_p(1), None) == L.PA_ERR_ARG
    assert lib.pa_pipe_probe(1, 0, 10, 0, C.c_void_p(1), None) == L.PA_ERR_ARG
    assert lib.pa_pipe_probe(1, 0, 10, 70000, C.c_void_p(1), None) == L.PA_ERR_ARG
    assert lib.pa_pipe_probe(1, 0, 10, 1, out, None) == L.PA_ERR_ARG
