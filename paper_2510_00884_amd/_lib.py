"""ctypes declarations of the C ABI in include/pa.h.

Loading fails loudly when the HIP library has not been built: there is no
CPU fallback anywhere in the product path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpa.so")

PA_OK, PA_ERR_ARG, PA_ERR_UNSUPPORTED, PA_ERR_HIP, PA_ERR_WORKSPACE = 0, -1, -2, -3, -4
PA_FP64, PA_FP32, PA_BF16, PA_BF16_CORR, PA_BF16_JAC = 0, 1, 2, 3, 4
PA_ALGO_FORWARD, PA_ALGO_ADJOINT = 0, 1
PA_ACT_SOFTPLUS = 0
PA_NOALLOC_SCRATCH_BYTES = 64 << 20

PRECISIONS = {"fp64": PA_FP64, "fp32": PA_FP32, "bf16": PA_BF16, "bf16_corr": PA_BF16_CORR, "bf16_jac": PA_BF16_JAC}
ALGORITHMS = {"forward": PA_ALGO_FORWARD, "adjoint": PA_ALGO_ADJOINT}
PA_MODEL_MICNN, PA_MODEL_CANN, PA_MODEL_GENT_THOMAS = 0, 1, 2
MODEL_KINDS = {"micnn": PA_MODEL_MICNN, "cann": PA_MODEL_CANN, "gent_thomas": PA_MODEL_GENT_THOMAS}


class ModelDesc(C.Structure):
    _fields_ = [("n_sv", C.c_int32), ("A", (C.c_double * 3) * 2), ("n_hidden", C.c_int32),
                ("width", C.c_int32), ("activation", C.c_int32), ("normalize", C.c_int32),
                ("has_bias", C.c_int32), ("algorithm", C.c_int32), ("kind", C.c_int32)]


class Mesh(C.Structure):
    _fields_ = [("n_el", C.c_int64), ("n_nodes", C.c_int64), ("nen", C.c_int32), ("nq", C.c_int32),
                ("conn", C.c_void_p), ("dNdX", C.c_void_p), ("w", C.c_void_p), ("X", C.c_void_p)]


class Csr(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("e2csr", C.c_void_p)]


class Incidence(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_ent", C.c_int64), ("max_row", C.c_int32), ("ptr", C.c_void_p),
                ("ent", C.c_void_p)]


class Colouring(C.Structure):
    _fields_ = [("n_colours", C.c_int32), ("colour_ptr", C.c_void_p), ("elem_perm", C.c_void_p)]


P = C.c_void_p
I32, I64, SZ = C.c_int32, C.c_int64, C.c_size_t
PDESC = C.POINTER(ModelDesc)
PMESH = C.POINTER(Mesh)
PCSR = C.POINTER(Csr)
PCOL = C.POINTER(Colouring)

SIGNATURES = {
    "pa_num_inputs": (I32, [PDESC]),
    "pa_num_params": (I64, [PDESC]),
    "pa_supported": (I32, [PDESC]),
    "pa_prepared_bytes": (SZ, [PDESC]),
    "pa_prepare_params": (C.c_int, [PDESC, P, P, P]),
    "pa_invariants": (C.c_int, [PDESC, I64, P, P, P, P, P]),
    "pa_material_workspace_bytes": (SZ, [PDESC, I64]),
    "pa_energy_stress_tangent": (C.c_int, [PDESC, P, C.c_int, I64, P, P, P, P, P, P, SZ, P]),
    "pa_energy_stress_tangent_batched": (C.c_int, [PDESC, P, C.c_int, I64, I64, P, P, P, P, P, P, SZ, P]),
    "pa_energy_stress_tangent_noalloc": (C.c_int, [PDESC, P, C.c_int, I64, P, P, P, P, P, P]),
    "pa_noalloc_max_points": (I64, [PDESC]),
    "pa_mesh_geometry": (C.c_int, [I32, I64, I64, P, P, P, P, P, P]),
    "pa_element_workspace_bytes": (SZ, [PDESC, PMESH]),
    "pa_element_residual_stiffness": (C.c_int, [PDESC, P, C.c_int, PMESH, P, P, P, P, P, SZ, P]),
    "pa_csr_pattern": (C.c_int, [I32, I64, I64, P, P, P, C.POINTER(I64)]),
    "pa_colour_elements": (C.c_int, [I32, I64, I64, P, P, C.POINTER(I32)]),
    "pa_element_csr_map": (C.c_int, [PMESH, PCSR, P, P]),
    "pa_assemble_csr": (C.c_int, [PMESH, PCOL, PCSR, P, P, P, P, I32, P]),
    "pa_tangent_build": (C.c_int, [PDESC, P, C.c_int, PMESH, PCOL, PCSR, P, P, P, P, P, SZ, P]),
    "pa_node_incidence": (C.c_int, [I32, I64, I64, P, P, P]),
    "pa_energy_stress_tangent_voigt": (C.c_int, [PDESC, P, C.c_int, I64, P, P, P, P, P, P, SZ, P]),
    "pa_residual_loss_workspace": (SZ, [I64, I32]),
    "pa_residual_loss": (C.c_int, [I64, P, P, I32, P, P, P, P, SZ, P]),
    "pa_residual_param_backward_workspace": (SZ, [PDESC, PMESH, C.c_int]),
    "pa_residual_param_backward": (C.c_int, [PDESC, P, C.c_int, PMESH, P, P, P, P, SZ, P]),
    "pa_gather_workspace_bytes": (SZ, [PDESC, PMESH]),
    "pa_tangent_build_gather": (C.c_int, [PDESC, P, C.c_int, PMESH, C.POINTER(Incidence), PCSR, P, P, P, P, P, SZ,
                                          P]),
    "pa_param_backward_workspace": (SZ, [PDESC, C.c_int, I64]),
    "pa_param_backward": (C.c_int, [PDESC, P, C.c_int, I64, P, P, P, P, SZ, P]),
    "pa_pipe_probe": (C.c_int, [I32, I32, I32, I32, P, P]),
    "pa_profile_enable": (C.c_int, [I32]),
    "pa_profile_count": (I32, []),
    "pa_profile_get": (C.c_int, [I32, C.POINTER(C.c_char_p), C.POINTER(C.c_double), C.POINTER(I64)]),
    "pa_status_string": (C.c_char_p, [C.c_int]),
    "pa_last_error": (C.c_char_p, []),
    "pa_version": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libpa.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PaError(RuntimeError):
    pass


def check(rc: int, what: str):
    if rc != PA_OK:
        lib = load()
        msg = lib.pa_last_error().decode()
        raise PaError(f"{what} failed: {lib.pa_status_string(rc).decode()} ({rc}): {msg}")
