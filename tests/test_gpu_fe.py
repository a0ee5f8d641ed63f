"""GPU parity of the element and assembly path (pa_mesh_geometry,
pa_element_residual_stiffness, pa_assemble_csr) against the FP64 oracle on
small hex8 and tet10 meshes; FP64 tolerance 1e-12 normwise."""
import numpy as np
import pytest
import torch

from oracle import fe, ncm
from paper_2510_00884_amd import synth
from gpu_util import close, need_gpu, rel, say

pytestmark = pytest.mark.gpu


def setup(api, kind, n, n_sv=1, h=16, L=2, amp=0.05, colour="parity"):
    X, conn, par = (synth.hex_mesh if kind == "hex8" else synth.tet10_mesh)(n)
    p = synth.num_inputs(n_sv)
    theta = synth.micnn_params(p, h, L, seed=1)
    Av = synth.structural_vectors(n_sv)
    gm = api.Model(theta, n_sv, h, L, A=Av, normalize=True)
    om = ncm.model_from_theta(theta, p, h, L, Av, normalize=True)
    mesh = api.FEMesh(X, conn, colour=par if colour == "parity" else None)
    # hex8: uniform nodal noise as in the 8^3 correctness case; tet10: smooth
    # modes plus noise relative to the mesh size as in the large tet10 case
    # (uniform noise on a coarse quadratic mesh drives points towards J = 0)
    if kind == "hex8":
        u = synth.displacement_uniform(X.shape[0], amp, seed=0)
    else:
        u = synth.displacement_modes(X, 1.0 / n, seed=0)
    return X, conn, gm, om, mesh, u


@pytest.mark.parametrize("kind,n", [("hex8", 3), ("tet10", 2)])
def test_geometry(kind, n):
    api = need_gpu()
    say("geometry", kind, n)
    X, conn, gm, om, mesh, u = setup(api, kind, n)
    dNdX, w, _ = fe.geometry(X, conn[mesh.perm])
    g_dN = mesh.dNdX.cpu().numpy().transpose(3, 0, 1, 2)
    g_w = mesh.w.cpu().numpy().T
    close(g_dN, dNdX, 1e-14, "g_dN")
    close(g_w, w, 1e-14, "g_w")
    assert int(mesh.n_bad.item()) == 0


@pytest.mark.parametrize("kind,n,n_sv,h,L", [("hex8", 8, 1, 16, 2), ("tet10", 3, 2, 32, 2), ("hex8", 3, 2, 64, 3)])
def test_element_residual_stiffness_and_assembly(kind, n, n_sv, h, L):
    api = need_gpu()
    say("element", kind, n, n_sv, h, L)
    X, conn, gm, om, mesh, u = setup(api, kind, n, n_sv, h, L)
    ut = torch.tensor(u, device="cuda")
    r_e, K_e = api.element_residual_stiffness(gm, mesh, ut, prec="fp64")
    cperm = conn[mesh.perm]
    dNdX, w, _ = fe.geometry(X, cperm)
    r_ref, K_ref, _ = fe.element_residual_stiffness(u, cperm, dNdX, w, om)
    close(r_e.cpu().numpy().T, r_ref, 1e-12, "r_e")
    close(K_e.cpu().numpy().transpose(2, 0, 1), K_ref, 1e-12, "K_e")
    r, vals = api.assemble_csr(mesh, r_e, K_e)
    rg, Kg = fe.assemble(cperm, r_ref, K_ref, X.shape[0])
    np.testing.assert_array_equal(mesh.row_ptr_host, Kg.indptr)
    np.testing.assert_array_equal(mesh.col_host, Kg.indices)
    close(r.cpu().numpy(), rg, 1e-12, "r.cpu().numpy()")
    close(vals.cpu().numpy(), Kg.data, 1e-12, "vals.cpu().numpy()")
    # fused coloured build scatters the same rows straight into CSR
    rf, vf = api.tangent_build(gm, mesh, ut, prec="fp64", fused=True, assembly="coloured")
    close(rf.cpu().numpy(), rg, 1e-12, "fused r")
    close(vf.cpu().numpy(), Kg.data, 1e-12, "fused vals")
    # node-centric gather build writes every CSR row once (poisoned buffers
    # first: nothing may be left from before)
    bufs = {"r": torch.full_like(rf, float("nan")), "vals": torch.full_like(vf, float("nan"))}
    rgt, vgt = api.tangent_build(gm, mesh, ut, prec="fp64", assembly="gather", bufs=bufs)
    close(rgt.cpu().numpy(), rg, 1e-12, "gather r")
    close(vgt.cpu().numpy(), Kg.data, 1e-12, "gather vals")


def test_assembly_greedy_colouring_and_determinism():
    api = need_gpu()
    say("assembly greedy colouring")
    X, conn, gm, om, mesh, u = setup(api, "hex8", 4, colour="greedy")
    ut = torch.tensor(u, device="cuda")
    r1, v1 = api.tangent_build(gm, mesh, ut, fused=False, assembly="coloured")
    r1, v1 = r1.clone(), v1.clone()
    r2, v2 = api.tangent_build(gm, mesh, ut, fused=False, assembly="coloured")
    assert torch.equal(r1, r2) and torch.equal(v1, v2)   # fixed colouring: bitwise deterministic
    r3, v3 = api.tangent_build(gm, mesh, ut, fused=True, assembly="coloured")
    r3, v3 = r3.clone(), v3.clone()
    r4, v4 = api.tangent_build(gm, mesh, ut, fused=True, assembly="coloured")
    assert torch.equal(r3, r4) and torch.equal(v3, v4)
    r5, v5 = api.tangent_build(gm, mesh, ut, assembly="gather")
    r5, v5 = r5.clone(), v5.clone()
    r6, v6 = api.tangent_build(gm, mesh, ut, assembly="gather")
    assert torch.equal(r5, r6) and torch.equal(v5, v6)   # incidence order: bitwise deterministic
    close(v5.cpu().numpy(), v1.cpu().numpy(), 1e-14, "gather vs coloured")
    cperm = conn[mesh.perm]
    dNdX, w, _ = fe.geometry(X, cperm)
    r_ref, K_ref, _ = fe.element_residual_stiffness(u, cperm, dNdX, w, om)
    rg, Kg = fe.assemble(cperm, r_ref, K_ref, X.shape[0])
    close(r1.cpu().numpy(), rg, 1e-12, "r")
    close(v1.cpu().numpy(), Kg.data, 1e-12, "vals")


def test_homogeneous_and_rigid_motion():
    api = need_gpu()
    say("patch tests")
    X, conn, gm, om, mesh, _ = setup(api, "hex8", 3)
    Q = synth.sample_F(1, seed=5, sigma=0.0)[0]
    u = X @ (Q - np.eye(3)).T + np.array([0.1, -0.2, 0.3])
    r_e, K_e = api.element_residual_stiffness(gm, mesh, torch.tensor(u, device="cuda"))
    assert r_e.abs().max().item() < 1e-12
    K_e = K_e.permute(2, 0, 1)
    t = torch.tensor(np.tile([0.3, -1.1, 0.7], 8), device="cuda")
    assert (K_e @ t).abs().max().item() < 1e-11 * K_e.abs().max().item()
    assert (K_e - K_e.transpose(1, 2)).abs().max().item() < 1e-12 * K_e.abs().max().item()


@pytest.mark.parametrize("kind,n,n_sv,h,L", [("hex8", 5, 2, 32, 2), ("tet10", 2, 2, 64, 3)])
def test_tangent_build_adjoint_hessian(kind, n, n_sv, h, L):
    """The fused tangent build with the adjoint-form network Hessian matches
    the oracle's assembled residual and tangent."""
    api = need_gpu()
    say("tangent_build adjoint", kind, n, n_sv, h, L)
    X, conn, gm, om, mesh, u = setup(api, kind, n, n_sv, h, L)
    gm.algorithm = "adjoint"
    cperm = conn[mesh.perm]
    dNdX, w, _ = fe.geometry(X, cperm)
    r_ref, K_ref, _ = fe.element_residual_stiffness(u, cperm, dNdX, w, om)
    rg, Kg = fe.assemble(cperm, r_ref, K_ref, X.shape[0])
    for assembly in ("gather", "coloured"):
        rf, vf = api.tangent_build(gm, mesh, torch.tensor(u, device="cuda"), prec="fp64", assembly=assembly)
        close(rf.cpu().numpy(), rg, 1e-12, f"r ({assembly})")
        close(vf.cpu().numpy(), Kg.data, 1e-12, f"vals ({assembly})")


def test_tangent_build_cann():
    """Tangent build of a hex8 mesh with the CANN inner function."""
    api = need_gpu()
    say("tangent_build cann")
    n, n_sv = 3, 2
    X, conn, par = synth.hex_mesh(n)
    u = synth.displacement_modes(X, 1.0 / n, seed=0)
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    theta = synth.cann_params(p, seed=2)
    gm = api.Model(theta, n_sv, A=Av, normalize=True, kind="cann")
    om = ncm.ClosedModel(ncm.cann, theta, Av, normalize=True)
    mesh = api.FEMesh(X, conn, colour=par)
    cperm = conn[mesh.perm]
    dNdX, w, _ = fe.geometry(X, cperm)
    r_ref, K_ref, _ = fe.element_residual_stiffness(u, cperm, dNdX, w, om)
    rg, Kg = fe.assemble(cperm, r_ref, K_ref, X.shape[0])
    rf, vf = api.tangent_build(gm, mesh, torch.tensor(u, device="cuda"), prec="fp64")
    close(rf.cpu().numpy(), rg, 1e-12, "r")
    close(vf.cpu().numpy(), Kg.data, 1e-12, "vals")


@pytest.mark.parametrize("kind,n", [("hex8", 4), ("tet10", 3)])
def test_inline_geometry_matches_stored(kind, n):
    """Shape gradients and weights recomputed from the node coordinates inside
    the tangent-build kernels give the same build, bit for bit, as the ones
    stored by the geometry kernel (one device function computes both)."""
    api = need_gpu()
    say("inline geometry", kind, n)
    X, conn, gm, om, mesh, u = setup(api, kind, n, n_sv=2, h=32, L=2)
    gm.algorithm = "adjoint"
    par = (synth.hex_mesh if kind == "hex8" else synth.tet10_mesh)(n)[2]
    inl = api.FEMesh(X, conn, colour=par, inline_geometry=True)
    sto = api.FEMesh(X, conn, colour=par, inline_geometry=False)
    ut = torch.tensor(u, device="cuda")
    for assembly in ("gather", "coloured"):
        r1, v1 = api.tangent_build(gm, inl, ut, prec="fp64", assembly=assembly)
        r1, v1 = r1.clone(), v1.clone()
        r2, v2 = api.tangent_build(gm, sto, ut, prec="fp64", assembly=assembly)
        assert torch.equal(r1, r2) and torch.equal(v1, v2), assembly
    cperm = conn[inl.perm]
    dNdX, w, _ = fe.geometry(X, cperm)
    r_ref, K_ref, _ = fe.element_residual_stiffness(u, cperm, dNdX, w, om)
    rg, Kg = fe.assemble(cperm, r_ref, K_ref, X.shape[0])
    close(r1.cpu().numpy(), rg, 1e-12, "r")
    close(v1.cpu().numpy(), Kg.data, 1e-12, "vals")


@pytest.mark.parametrize("kind", ["hex8", "tet10"])
def test_single_cube_and_orphan_node(kind):
    """Edge cases of the element and assembly path: one hex8 element (every
    node on the boundary, one partially filled workgroup) or one Kuhn cube
    of six tet10 elements, plus a node that no element references (its CSR
    rows are empty and its residual entries must come out as zero)."""
    api = need_gpu()
    say("single cube + orphan node", kind)
    X, conn, par = (synth.hex_mesh if kind == "hex8" else synth.tet10_mesh)(1)
    X = np.vstack([X, [[2.0, 2.0, 2.0]]])  # unreferenced node
    u = synth.displacement_uniform(X.shape[0], 0.05, seed=0)
    p = synth.num_inputs(2)
    theta = synth.micnn_params(p, 16, 2, seed=1)
    Av = synth.structural_vectors(2)
    gm = api.Model(theta, 2, 16, 2, A=Av, normalize=True, algorithm="adjoint")
    om = ncm.model_from_theta(theta, p, 16, 2, Av, normalize=True)
    mesh = api.FEMesh(X, conn, colour=par)
    cperm = conn[mesh.perm]
    dNdX, w, _ = fe.geometry(X, cperm)
    r_ref, K_ref, _ = fe.element_residual_stiffness(u, cperm, dNdX, w, om)
    rg, Kg = fe.assemble(cperm, r_ref, K_ref, X.shape[0])
    ut = torch.tensor(u, device="cuda")
    for assembly in ("gather", "coloured"):
        r, vals = api.tangent_build(gm, mesh, ut, prec="fp64", assembly=assembly)
        close(r.cpu().numpy(), rg, 1e-12, f"r ({assembly})")
        close(vals.cpu().numpy(), Kg.data, 1e-12, f"vals ({assembly})")
        assert np.all(r.cpu().numpy()[-3:] == 0.0)
    r_e, K_e = api.element_residual_stiffness(gm, mesh, ut, prec="fp64")
    close(K_e.cpu().numpy().transpose(2, 0, 1), K_ref, 1e-12, "K_e")


@pytest.mark.parametrize("kind,n", [("hex8", 4), ("tet10", 2)])
@pytest.mark.parametrize("order", ["native", "morton"])
def test_element_orders(kind, n, order):
    """Meshes numbered in the given order (native or Z-order of the element
    centroids): the node-centric build equals the oracle's assembled residual
    and tangent, and the element tables assembled colour by colour through
    elem_perm equal the node-centric build; the fused coloured build refuses
    a mesh not numbered colour by colour."""
    api = need_gpu()
    say("element order", kind, n, order)
    X, conn, par = (synth.hex_mesh if kind == "hex8" else synth.tet10_mesh)(n)
    n_sv, h, L = 2, 16, 2
    p = synth.num_inputs(n_sv)
    theta = synth.micnn_params(p, h, L, seed=1)
    Av = synth.structural_vectors(n_sv)
    gm = api.Model(theta, n_sv, h, L, A=Av, normalize=True, algorithm="adjoint")
    om = ncm.model_from_theta(theta, p, h, L, Av, normalize=True)
    mesh = api.FEMesh(X, conn, colour=par, order=order)
    if order == "native":
        assert np.array_equal(mesh.perm, np.arange(conn.shape[0]))
    assert sorted(mesh.perm.tolist()) == list(range(conn.shape[0]))
    u = synth.displacement_modes(X, 1.0 / n, seed=0)
    ut = torch.tensor(u, device="cuda")
    r, vals = api.tangent_build(gm, mesh, ut, prec="fp64", assembly="gather")
    dNdX, w, _ = fe.geometry(X, conn)
    r_ref, K_ref, _ = fe.element_residual_stiffness(u, conn, dNdX, w, om)
    rg, Kg = fe.assemble(conn, r_ref, K_ref, X.shape[0])
    close(r.cpu().numpy(), rg, 1e-12, "r")
    close(vals.cpu().numpy(), Kg.data, 1e-12, "vals")
    rt, vt = api.tangent_build(gm, mesh, ut, prec="fp64", assembly="coloured", fused=False)
    close(rt.cpu().numpy(), r.cpu().numpy(), 1e-13, "tables + coloured assembly r")
    close(vt.cpu().numpy(), vals.cpu().numpy(), 1e-13, "tables + coloured assembly vals")
    with pytest.raises(ValueError):
        api.tangent_build(gm, mesh, ut, prec="fp64", assembly="coloured", fused=True)
