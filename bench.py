#!/usr/bin/env python3
"""Benchmark of the hot path: one Newton tangent build per step.

Workload (the plain-method FP64 vs FP32 mesh case): 64^3 trilinear hex8
unit-cube mesh (262,144 elements, 2,097,152 quadrature points, 823,875
dofs), orthotropic with structural vectors e1 and e2 (9 inputs), MICNN with
2 hidden layers of width 32 and softplus, weights |N(0, 0.3)| and biases
N(0, 0.3) (seed 1), normalised reference state, displacement
u_i = 0.05 sin(pi X_i) + 0.05 sin(pi X_{i+1}) + 0.02 h U[-1, 1] (seed 0).

A step is the whole path u -> F -> features -> network (value, gradient,
Hessian) -> chain rule (P, dP/dF) -> element residual and stiffness ->
CSR assembly of r and K.  Inputs are resident on the GPU before the
timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "bf16_corr": 2.5e15, "bf16_jac": 2.5e15}
HBM_PEAK = 8.0e12


def measured_traffic(kernel_symbol):
    """HBM bytes per launch of a kernel from the committed FETCH_SIZE /
    WRITE_SIZE summary (profiles/traffic.json), or None when that summary is
    for another kernel or the kernel's sources have changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tr = json.load(fh)
    if tr.get("symbol") != kernel_symbol:
        return None
    h = hashlib.sha256()
    for src in tr["sources"]:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != tr["sources_sha256"]:
        return None
    return tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"]


def mlp_flops_per_point(h, L, p):
    """Alg. 4 forward mode: 2h^2 c (L-1) + 2hc + 2hpL + 4h P2 (L-1) + h P2,
    c = 1 + p + P2 columns, P2 = p(p+1)/2."""
    P2 = p * (p + 1) // 2
    c = 1 + p + P2
    return 2 * h * h * c * (L - 1) + 2 * h * c + 2 * h * p * L + 4 * h * P2 * (L - 1) + h * P2


def mlp_adjoint_flops_per_point(h, L, p):
    """Adjoint-form Hessian: value forward 2hp + (L-1)(2h^2 + 2hp), value
    adjoint (L-1) 2h^2, Jacobian forward (L-1) 2h^2 p, Gram sums 3 h P2 L,
    gradient 2hp."""
    P2 = p * (p + 1) // 2
    return 2 * h * p + (L - 1) * (2 * h * h + 2 * h * p) + (L - 1) * 2 * h * h + (L - 1) * 2 * h * h * p \
        + 3 * h * P2 * L + 2 * h * p


def mlp_flops(kernel, h, L, p):
    return (mlp_adjoint_flops_per_point if kernel == "mlp_adjoint" else mlp_flops_per_point)(h, L, p)


def kernel_bytes_total(name, mesh, p):
    """Algorithmic HBM bytes of one step for a bandwidth-bound kernel: every
    input read once and every output written once.  The mesh recomputes
    shape gradients and weights from the node coordinates inside gather_F and
    the element integration, so those kernels read conn and X instead of
    dN/dX and w."""
    nen, nq, nd = mesh.nen, mesh.nq, 3 * mesh.nen
    nodes = 8 * 3 * mesh.n_nodes                                  # one double triple per node (u or X)
    if name == "gather_assemble":
        return mesh.n_el * (72 * sym_blocks(nen) + 8 * nd + 4 * nen * nen + 4 * nen) \
            + 8 * mesh.nnz + 8 * 3 * mesh.n_nodes + 8 * (3 * mesh.n_nodes + 1) + 8 * (mesh.n_nodes + 1)
    if name == "gather_F":
        return mesh.n_el * (nq * (72 + 8 * p) + 4 * nen) + 2 * nodes  # F and K out; conn, u and X in
    if name == "integrate_elmajor":
        return mesh.n_el * (nq * (72 + 216) + 4 * nen + 72 * sym_blocks(nen) + 8 * nd) + nodes
    b = kernel_bytes(name, nen, nq, p)
    return None if b is None else b * mesh.n_el


def sym_blocks(nen):
    """Distinct 3 x 3 node blocks of a symmetric element tangent."""
    return nen * (nen + 1) // 2


def kernel_bytes(name, nen, nq, p):
    """Algorithmic HBM bytes per element for the bandwidth-bound kernels that
    read stored geometry (the coloured and table paths): every input read
    once and every output written once (read-modify-write counts twice)."""
    nd = 3 * nen
    nout = 1 + p + p * (p + 1) // 2
    per_qp = {"features": 72 + 8 * p, "chain": 72 + 8 * nout + 72 + 648}
    if name in per_qp:
        return nq * per_qp[name]
    if name == "material_cc":
        return nq * (72 + 8 * (nout - 1) + 8 * 27)              # F, network derivatives in; S~, CC~ out
    inputs = nq * (72 + 8 * 27) + 4 * nen                        # F, S~ and CC~, conn (geometry from X)
    if name == "integrate":
        return inputs + 8 * nd * nd + 8 * nd                     # K_e, r_e written
    if name == "integrate_scatter":
        return inputs + 16 * nd * nd + 16 * nd + 4 * nen * nen   # CSR and r read-modify-write, CSR map
    if name == "assemble":
        return 24 * nd * nd + 24 * nd
    return None


def cpu_baseline(X, conn, u, theta, p, h, L, Av, n_sample):
    """The oracle (plain FP64 NumPy, single thread) on a contiguous sample of
    elements: element residual/stiffness through the push-forward route and
    COO->CSR assembly of that sample."""
    from threadpoolctl import threadpool_limits

    from oracle import fe, ncm
    om = ncm.model_from_theta(theta, p, h, L, Av, normalize=True)
    sub = conn[:n_sample]
    with threadpool_limits(limits=1):  # BLAS pools pinned to one thread: the figure is one core's
        t0 = time.perf_counter()
        dNdX, w, _ = fe.geometry(X, sub)
        r_e, K_e, _ = fe.element_residual_stiffness(u, sub, dNdX, w, om)
        fe.assemble(sub, r_e, K_e, X.shape[0])
        dt = time.perf_counter() - t0
    nq = dNdX.shape[1]
    return {"value": n_sample * nq / dt, "unit": "qp evals/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample} elements ({n_sample * nq} points) of the same mesh, model and "
                      f"displacement; geometry + element residual/stiffness + assembly; {dt:.1f} s; "
                      f"NumPy single thread on {os.cpu_count()} host cores"}


def _profiled(lib, fn, steps, warmup):
    """ms per call of fn (HIP events on the current stream) and the library's
    per-kernel times."""
    import ctypes as C
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    lib.pa_profile_enable(1)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    lib.pa_profile_enable(0)
    kern = {}
    for i in range(lib.pa_profile_count()):
        nm, t, k = C.c_char_p(), C.c_double(), C.c_int64()
        lib.pa_profile_get(i, C.byref(nm), C.byref(t), C.byref(k))
        kern[nm.value.decode()] = round(t.value / max(k.value, 1), 4)
    return e0.elapsed_time(e1) / steps, kern


def other_workload(args):
    """The point-batch, calibration and large-mesh workloads (not the
    default bench line): prints one JSON line per workload."""
    import torch
    from paper_2510_00884_amd import api, synth
    from paper_2510_00884_amd import _lib as L
    lib = L.load()
    n_sv, h, Lh = 2, 64, 3
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    theta = synth.micnn_params(p, h, Lh, seed=1)
    steps, warmup = max(args.steps // 4, 2), 1
    if args.workload == "points_2pow22":
        n = 1 << 22
        F = torch.tensor(synth.sample_F(n, seed=0), device="cuda")
        res = {}
        ref = None
        for prec, algo in [("fp64", "adjoint"), ("fp32", "adjoint"), ("bf16", "adjoint"), ("bf16_corr", "adjoint"),
                           ("bf16_jac", "adjoint"), ("bf16", "forward"), ("bf16_corr", "forward"), ("fp64", "forward")]:
            gm = api.Model(theta, n_sv, h, Lh, A=Av, normalize=True, algorithm=algo)
            bufs = {}
            def call():
                bufs["out"] = api.energy_stress_tangent(gm, F, prec=prec)
            ms, kern = _profiled(lib, call, steps, warmup)
            out = bufs["out"]
            if ref is None:
                ref = {k: v.clone() for k, v in out.items()}
            err = {k: ((out[k] - ref[k]).norm() / ref[k].norm()).item() for k in ("psi", "P", "A")}
            res[f"{prec}/{algo}"] = {"ms": ms, "qp_per_s": n / (ms / 1e3), "kernels_ms": kern,
                                     "rel_err_vs_fp64": err}
            print(f"[bench] {prec}/{algo}: {ms:.3f} ms, {n / (ms / 1e3):.3e} qp/s", file=sys.stderr, flush=True)
            del out
            bufs.clear()
        for prec in ("fp64", "fp32"):  # the paper's storage: tau (6) and cc (21) per point
            gm = api.Model(theta, n_sv, h, Lh, A=Av, normalize=True, algorithm="adjoint")
            bufs = {}
            def call_v():
                bufs["out"] = api.energy_stress_tangent_voigt(gm, F, prec=prec)
            ms, kern = _profiled(lib, call_v, steps, warmup)
            res[f"{prec}/adjoint/voigt"] = {"ms": ms, "qp_per_s": n / (ms / 1e3), "kernels_ms": kern}
            print(f"[bench] {prec}/adjoint/voigt: {ms:.3f} ms, {n / (ms / 1e3):.3e} qp/s", file=sys.stderr, flush=True)
            bufs.clear()
        best = res["fp64/adjoint"]
        line = {"metric": "qp evals/s (Psi+P+tangent) & elements assembled/s, FP64 vs FP32/BF16 at stated error",
                "value": best["qp_per_s"], "unit": "qp evals/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
                "ms_per_step": best["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f64", "data": "synthetic",
                "config": {"workload": "2^22 independent points, orthotropic (9 inputs), MICNN 3x64 softplus: "
                                       "Psi, P and dP/dF per point"},
                "precisions": res}
    elif args.workload == "calib_2pow20":
        n = 1 << 20
        F = torch.tensor(synth.sample_F(n, seed=3), device="cuda")
        Pbar = torch.tensor(synth.rng(7).normal(size=(n, 9)) / n, device="cuda")
        gm = api.Model(theta, n_sv, h, Lh, A=Av, normalize=False, algorithm="adjoint")
        res = {}
        for prec in ("fp32", "fp64"):
            ms_f, kf = _profiled(lib, lambda: api.energy_stress_tangent(gm, F, prec=prec, psi=False, A=False),
                                 steps, warmup)
            ms_b, kb = _profiled(lib, lambda: api.param_backward(gm, F, Pbar, prec=prec), steps, warmup)
            res[prec] = {"forward_P_ms": ms_f, "adjoint_ms": ms_b, "step_ms": ms_f + ms_b,
                         "kernels_ms": {**kf, **kb}}
            print(f"[bench] calibration {prec}: forward {ms_f:.3f} ms + adjoint {ms_b:.3f} ms",
                  file=sys.stderr, flush=True)
        st = res["fp32"]["step_ms"]
        line = {"metric": "calibration samples/s (stress forward + parameter adjoint)", "value": n / (st / 1e3),
                "unit": "samples/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": st,
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                "data": "synthetic",
                "config": {"workload": "2^20-point stress calibration, MICNN 3x64 softplus, FP32 network"},
                "precisions": res}
    elif args.workload == "model_sweep":
        # the model-size study of App. E: constitutive update (Psi, P, AA) on
        # 2^20 points for every network size the kernels provide, and the
        # CANN and Gent-Thomas inner functions
        n = 1 << 20
        F = torch.tensor(synth.sample_F(n, seed=0), device="cuda")
        res = {}
        # widths below 16 run zero-padded to 16 neurons
        cases = [("micnn", w_, l_) for l_ in (2, 3, 4) for w_ in (2, 8, 16, 32, 64)] + [("cann", 0, 0), ("gent_thomas", 0, 0)]
        for kind, w_, l_ in cases:
            if kind == "micnn":
                th = synth.micnn_params(p, w_, l_, seed=1)
                gm = api.Model(th, n_sv, w_, l_, A=Av, normalize=True, algorithm="adjoint")
                tag = f"micnn {l_}x{w_}"
            else:
                th = synth.cann_params(p, seed=2) if kind == "cann" else synth.GENT_THOMAS
                gm = api.Model(th, n_sv, A=Av, normalize=True, kind=kind)
                tag = kind
            for prec in ("fp64", "fp32"):
                ms, kern = _profiled(lib, lambda: api.energy_stress_tangent(gm, F, prec=prec), steps, warmup)
                res[f"{tag}/{prec}"] = {"params": gm.n_params, "ms": ms, "qp_per_s": n / (ms / 1e3),
                                        "kernels_ms": kern}
                print(f"[bench] {tag} ({gm.n_params} params) {prec}: {ms:.3f} ms", file=sys.stderr, flush=True)
        best = res["micnn 2x32/fp64"]
        line = {"metric": "qp evals/s (Psi+P+tangent) & elements assembled/s, FP64 vs FP32/BF16 at stated error",
                "value": best["qp_per_s"], "unit": "qp evals/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
                "ms_per_step": best["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f64", "data": "synthetic",
                "config": {"workload": "model-size sweep: 2^20 independent points, orthotropic (9 inputs)"},
                "models": res}
    else:  # tet10_56
        n = 56
        X, conn, par = synth.tet10_mesh(n)
        u = torch.tensor(synth.displacement_modes(X, 1.0 / n, seed=0), device="cuda").reshape(-1)
        gm = api.Model(theta, n_sv, h, Lh, A=Av, normalize=True, algorithm="adjoint")
        mesh = api.FEMesh(X, conn, colour=par)
        ws = torch.empty(mesh.workspace_bytes(gm, "gather"), dtype=torch.uint8, device="cuda")
        bufs = {}
        res = {}
        ref = None
        for prec in ("fp64", "fp32", "bf16_corr"):
            ms, kern = _profiled(lib, lambda: api.tangent_build(gm, mesh, u, prec=prec, workspace=ws, bufs=bufs),
                                 steps, warmup)
            res[prec] = {"ms": ms, "qp_per_s": mesh.n_el * mesh.nq / (ms / 1e3), "kernels_ms": kern}
            if ref is None:
                ref = (bufs["r"].clone(), bufs["vals"].clone())
            else:
                res[prec]["rel_err_vs_fp64_r"] = ((bufs["r"] - ref[0]).norm() / ref[0].norm()).item()
                res[prec]["rel_err_vs_fp64_K"] = ((bufs["vals"] - ref[1]).norm() / ref[1].norm()).item()
            print(f"[bench] tet10 {prec}: {ms:.3f} ms", file=sys.stderr, flush=True)
        ms = res["fp32"]["ms"]
        line = {"metric": "qp evals/s (Psi+P+tangent) & elements assembled/s, FP64 vs FP32/BF16 at stated error",
                "value": mesh.n_el * mesh.nq / (ms / 1e3), "unit": "qp evals/s", "n_gpus": 1, "steps": steps,
                "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f32 network, f64 elsewhere", "data": "synthetic",
                "config": {"workload": f"tet10 Kuhn mesh of {n}^3 cubes ({mesh.n_el} elements, "
                                       f"{3 * mesh.n_nodes} dofs, {mesh.nnz} nonzeros), MICNN 3x64 softplus, "
                                       "one Newton tangent build"},
                "elements_per_s": mesh.n_el / (ms / 1e3), "precisions": res}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64, help="cubes per side of the hex8 mesh")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16", "bf16_corr", "bf16_jac"])
    ap.add_argument("--algo", default="adjoint", choices=["forward", "adjoint"],
                    help="network Hessian formation (BF16 variants always use forward)")
    ap.add_argument("--variants", default="fp32,bf16,bf16_corr,bf16_jac",
                    help="other precisions timed after the headline run ('' for none)")
    ap.add_argument("--workload", default="hex8_64",
                    choices=["hex8_64", "points_2pow22", "calib_2pow20", "tet10_56", "model_sweep"],
                    help="hex8_64 (default): the tangent-build bench line; the others measure the point-batch "
                         "precision ladder, the calibration step and the large tet10 mesh")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes three times (the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--cpu-sample", type=int, default=12288, help="elements in the oracle CPU sample (0: skip)")
    ap.add_argument("--assembly", default="gather", choices=["gather", "coloured", "tables"],
                    help="gather: element-major tables + one pass per node (default); coloured: element rows "
                         "scattered into CSR colour by colour; tables: element tables + coloured assembly")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding of the mesh is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_00884_amd import api, synth
    from paper_2510_00884_amd import _lib as L

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        nb = args.copy_probe << 20
        x = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nb, "copy_probe_bytes_written": nb, "launches": 3}), flush=True)
        return
    if args.workload != "hex8_64":
        other_workload(args)
        return
    n = args.n
    n_sv, h, Lh = 2, 32, 2
    p = synth.num_inputs(n_sv)
    X, conn, par = synth.hex_mesh(n)
    u = synth.displacement_modes(X, 1.0 / n, seed=0)
    theta = synth.micnn_params(p, h, Lh, seed=1)
    Av = synth.structural_vectors(n_sv)
    t_setup = time.perf_counter()
    model = api.Model(theta, n_sv, h, Lh, A=Av, normalize=True, algorithm=args.algo)
    mesh = api.FEMesh(X, conn, colour=par)
    ut = torch.tensor(u, device="cuda").reshape(-1).contiguous()
    ws = torch.empty(mesh.workspace_bytes(model, "gather" if args.assembly == "gather" else "coloured"),
                     dtype=torch.uint8, device="cuda")
    bufs = {}
    api.tangent_build(model, mesh, ut, prec=args.prec, workspace=ws, bufs=bufs, fused=args.assembly != "tables",
                          assembly="gather" if args.assembly == "gather" else "coloured")
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print(f"[bench] setup {t_setup:.1f} s: {mesh.n_el} elements, {mesh.n_el * mesh.nq} points, "
          f"{3 * mesh.n_nodes} dofs, {mesh.nnz} nonzeros, {mesh.n_colours} colours", file=sys.stderr, flush=True)

    lib = L.load()

    def run(prec, steps, warmup, profile):
        for _ in range(warmup):
            api.tangent_build(model, mesh, ut, prec=prec, workspace=ws, bufs=bufs, fused=args.assembly != "tables",
                          assembly="gather" if args.assembly == "gather" else "coloured")
        torch.cuda.synchronize()
        if profile:
            lib.pa_profile_enable(1)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            api.tangent_build(model, mesh, ut, prec=prec, workspace=ws, bufs=bufs, fused=args.assembly != "tables",
                          assembly="gather" if args.assembly == "gather" else "coloured")
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        kern = {}
        if profile:
            lib.pa_profile_enable(0)
            import ctypes as C
            cnt = lib.pa_profile_count()
            for i in range(cnt):
                nm = C.c_char_p()
                t = C.c_double()
                k = C.c_int64()
                lib.pa_profile_get(i, C.byref(nm), C.byref(t), C.byref(k))
                kern[nm.value.decode()] = {"ms_total": t.value, "launches": k.value,
                                           "ms_per_launch": t.value / max(k.value, 1)}
        return ms, kern

    ms, kern = run(args.prec, args.steps, args.warmup, True)
    n_qp = mesh.n_el * mesh.nq
    r_ref = bufs["r"].clone()
    v_ref = bufs["vals"].clone()
    print(f"[bench] {args.prec}: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    # per-kernel achieved rates against the algorithmic work
    for k, v in kern.items():
        per_step_ms = v["ms_total"] / args.steps
        if k.startswith("mlp"):
            v["tflops"] = mlp_flops(k, h, Lh, p) * n_qp / (per_step_ms / 1e3) / 1e12
        else:
            b = kernel_bytes_total(k, mesh, p)
            if b:
                v["algorithmic_gb_per_step"] = b / 1e9
                v["gb_s"] = b / (per_step_ms / 1e3) / 1e9

    # dominant kernel and its roofline
    dom = max(kern, key=lambda k: kern[k]["ms_total"]) if kern else None
    roof = None
    if dom:
        per_launch_s = kern[dom]["ms_per_launch"] / 1e3
        if dom.startswith("mlp"):
            fl = mlp_flops(dom, h, Lh, p) * n_qp
            ach = fl / per_launch_s
            pr = {"fp64": 0, "fp32": 1}.get(args.prec, -1)
            # two-layer networks up to width 32 run the single-wave kernel
            sym = None if dom != "mlp_adjoint" else (
                f"k_mlp_adj2<{h}, {p}, {pr}, true>" if Lh == 2 and h <= 32 else f"k_mlp_adj<{h}, {Lh}, {p}, {pr}, true>")
            roof = {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK[args.prec] / 1e12, "unit": "TFLOP/s",
                    "frac": ach / PEAK[args.prec], "traffic": measured_traffic(sym) if sym else None, "kernel": dom,
                    "algorithmic_per_launch": f"{mlp_flops(dom, h, Lh, p)} FLOP/point x {n_qp} points"}
        else:
            launches_per_step = kern[dom]["launches"] / args.steps
            b = kernel_bytes_total(dom, mesh, p) / launches_per_step
            per_launch_s = kern[dom]["ms_total"] / kern[dom]["launches"] / 1e3
            ach = b / per_launch_s
            roof = {"bound": "hbm", "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                    "frac": ach / HBM_PEAK, "traffic": None, "kernel": dom}

    variants = {}
    for vp in [x for x in args.variants.split(",") if x and x not in ("none", args.prec)]:
        # the adjoint form has FP64, FP32 and BF16-with-FP32-correction kernels
        model.algorithm = args.algo
        vms, vk = run(vp, max(args.steps // 2, 2), 1, True)
        err_r = (bufs["r"] - r_ref).norm().item() / r_ref.norm().item()
        err_K = (bufs["vals"] - v_ref).norm().item() / v_ref.norm().item()
        mk = next((k for k in vk if k.startswith("mlp")), None)
        variants[vp] = {"value": n_qp / (vms / 1e3), "ms_per_step": vms, "algorithm": model.algorithm_name,
                        "rel_err_vs_fp64_r": err_r, "rel_err_vs_fp64_K": err_K,
                        "mlp_ms": vk[mk]["ms_per_launch"] if mk else None,
                        "mlp_tflops": (mlp_flops(mk, h, Lh, p) * n_qp / (vk[mk]["ms_per_launch"] / 1e3) / 1e12) if mk else None}
        print(f"[bench] {vp}: {vms:.3f} ms/step, err r {err_r:.2e} K {err_K:.2e}", file=sys.stderr, flush=True)

    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(X, conn, u, theta, p, h, Lh, Av, min(args.cpu_sample, mesh.n_el))
        print(f"[bench] cpu oracle: {cpu['value']:.3e} qp/s ({cpu['sample']})", file=sys.stderr, flush=True)

    line = {
        "metric": "qp evals/s (Psi+P+tangent) & elements assembled/s, FP64 vs FP32/BF16 at stated error",
        "value": n_qp / (ms / 1e3),
        "unit": "qp evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16", "bf16_corr": "bf16+f32", "bf16_jac": "f32+bf16"}[args.prec],
        "data": "synthetic",
        "config": {"workload": f"hex8 {n}^3 unit cube, orthotropic e1/e2 (9 inputs), MICNN 2x32 softplus, "
                               "one Newton tangent build: residual + tangent + CSR assembly",
                   "assembly": {"gather": "element-major tables + node-centric gather",
                                "coloured": "fused per-colour scatter",
                                "tables": "element tables + coloured assembly"}[args.assembly],
                   "elements": mesh.n_el, "points": n_qp, "dofs": 3 * mesh.n_nodes, "nnz": mesh.nnz,
                   "colours": mesh.n_colours, "precision": args.prec, "algorithm": args.algo},
        "elements_per_s": mesh.n_el / (ms / 1e3),
        "kernels": kern,
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
