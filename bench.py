#!/usr/bin/env python3
"""Benchmark of the hot path on one GPU: prints one JSON line.

Headline (the FP64-vs-FP32 mesh case): one Newton tangent build per step on
a 64^3 trilinear hex8 unit-cube mesh (262,144 elements, 2,097,152 quadrature
points, 823,875 dofs), orthotropic with structural vectors e1 and e2 (9
inputs), MICNN with 2 hidden layers of width 32 and softplus, weights
|N(0, 0.3)| and biases N(0, 0.3) (seed 1), normalised reference state,
displacement u_i = 0.05 sin(pi X_i) + 0.05 sin(pi X_{i+1}) + 0.02 h U[-1, 1]
(seed 0).  A step is the whole path u -> F -> features -> network (value,
gradient, Hessian) -> chain rule -> element residual and stiffness -> CSR
assembly of r and K, FP64, inputs resident on the GPU.

The same line carries the other workloads (``workloads``): the precision
ladder on 2^22 independent points (MICNN 3x64), the 2^20-sample stress
calibration step (stress forward + parameter adjoint, 3x64) and one tangent
build on the 56^3 Kuhn tet10 mesh (3x64); each with per-kernel times (HIP
events on the launch stream), errors against its FP64 run and the roofline
fraction of its kernels.  ``cpu_baseline``: the FP64 oracle on bounded
samples of the headline mesh and of the point batch, on one core and on all
host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np  # noqa: F401  (host arrays of the synthetic inputs)

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense)
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15}
HBM_PEAK = 8.0e12
METRIC = "qp evals/s (Psi+P+tangent) & elements assembled/s, FP64 vs FP32/BF16 at stated error"


# ---------------------------------------------------------------- work models
def mlp_forward_flops(h, L, p):
    """Alg. 4 forward mode (value, gradient and Hessian columns):
    2h^2 c (L-1) + 2hc + 2hpL + 4h P2 (L-1) + h P2, c = 1 + p + P2."""
    P2 = p * (p + 1) // 2
    c = 1 + p + P2
    return 2 * h * h * c * (L - 1) + 2 * h * c + 2 * h * p * L + 4 * h * P2 * (L - 1) + h * P2


def mlp_adjoint_parts(h, L, p, hess=True):
    """Adjoint-form network FLOPs per point split by the contraction that
    carries them: value forward 2hp + (L-1)(2h^2 + 2hp), reverse sweep
    (L-1) 2h^2, gradient 2hpL; with the Hessian: Jacobian forward
    (L-1) 2h^2 p, and the Gram sums 2h P2 (layer 1) + (L-1) 2h P2.
    Returns (value/gradient part, Jacobian part, Gram part)."""
    P2 = p * (p + 1) // 2
    vg = 2 * h * p + (L - 1) * (2 * h * h + 2 * h * p) + (L - 1) * 2 * h * h + 2 * h * p * L
    if not hess:
        return vg, 0, 0
    return vg, (L - 1) * 2 * h * h * p, 2 * h * P2 + (L - 1) * 2 * h * P2


def mlp_adjoint_flops(h, L, p, hess=True):
    return sum(mlp_adjoint_parts(h, L, p, hess))


def param_bwd_flops(h, L, p):
    """Parameter adjoint (reverse over the value and its tangent along
    lambda): forward 4hp + (L-1)(4h^2 + 4hp), reverse (L-1)(8h^2 + 4hp) + 4hp."""
    return 8 * h * p + (L - 1) * (12 * h * h + 8 * h * p)


def sym_blocks(nen):
    """Distinct 3 x 3 node blocks of a symmetric element tangent."""
    return nen * (nen + 1) // 2


def mesh_kernel_bytes(name, mesh, p):
    """Algorithmic HBM bytes of one build for a bandwidth-bound mesh kernel:
    every input read once and every output written once (read-modify-write
    counts twice).  Shape gradients and weights are recomputed from the node
    coordinates, so the kernels read conn and X instead of dN/dX and w."""
    nen, nq, nd, n_el = mesh.nen, mesh.nq, 3 * mesh.nen, mesh.n_el
    nodes = 8 * 3 * mesh.n_nodes                                  # one double triple per node (u or X)
    nout = 1 + p + p * (p + 1) // 2
    if name == "gather_assemble":
        return n_el * (72 * sym_blocks(nen) + 8 * nd + 4 * nen * nen + 4 * nen) \
            + 8 * mesh.nnz + 8 * 3 * mesh.n_nodes + 8 * (3 * mesh.n_nodes + 1) + 8 * (mesh.n_nodes + 1)
    if name == "gather_F":
        return n_el * (nq * (72 + 8 * p) + 4 * nen) + 2 * nodes  # F and K out; conn, u and X in
    if name == "integrate_elmajor":
        return n_el * (nq * (72 + 216) + 4 * nen + 72 * sym_blocks(nen) + 8 * nd) + nodes
    if name == "material_cc":
        return n_el * nq * (72 + 8 * (nout - 1) + 216)               # F, network derivatives in; S~, CC~ out
    if name == "integrate_scatter":
        return n_el * (nq * (72 + 216) + 4 * nen + 16 * nd * nd + 16 * nd + 4 * nen * nen) + nodes
    return None


def measured_traffic(kernel_symbol):
    """HBM bytes per launch of a kernel from the committed FETCH_SIZE /
    WRITE_SIZE summaries (profiles/traffic.json, one entry per kernel
    symbol), or None when there is no entry or the kernel's sources have
    changed since it was measured."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tr = json.load(fh)
    entry = tr.get(kernel_symbol)
    if not entry:
        return None
    h = hashlib.sha256()
    for src in entry["sources"]:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != entry["sources_sha256"]:
        return None
    return entry["fetch_bytes_per_launch"] + entry["write_bytes_per_launch"]


def roof_mfma(kernel, ms_per_launch, flops, peak_key):
    """Roofline record of a matrix-core kernel: algorithmic FLOPs per launch
    over its HIP-event launch time, against the published dense peak."""
    if ms_per_launch is None or ms_per_launch <= 0:
        return None
    ach = flops / (ms_per_launch * 1e-3)
    return {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK[peak_key] / 1e12, "unit": "TFLOP/s",
            "frac": ach / PEAK[peak_key], "traffic": None, "kernel": kernel, "ms_per_launch": ms_per_launch,
            "flop_per_launch": flops}


def roof_mixed(kernel, ms_per_launch, flops_by_peak):
    """Roofline of a kernel whose contractions run at two precisions: the
    time bound is the sum of each part's FLOPs over its own peak."""
    t_bound = sum(f / PEAK[k] for k, f in flops_by_peak.items())
    t = ms_per_launch * 1e-3
    tot = sum(flops_by_peak.values())
    return {"bound": "mfma", "achieved": tot / t / 1e12, "peak": tot / t_bound / 1e12, "unit": "TFLOP/s",
            "frac": t_bound / t, "traffic": None, "kernel": kernel, "ms_per_launch": ms_per_launch,
            "flop_per_launch": dict(flops_by_peak)}


def roof_hbm(kernel, ms_per_launch, nbytes):
    ach = nbytes / (ms_per_launch * 1e-3)
    return {"bound": "hbm", "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": ach / HBM_PEAK,
            "traffic": None, "kernel": kernel, "ms_per_launch": ms_per_launch, "bytes_per_launch": nbytes}


# ---------------------------------------------------------------- CPU baseline (the oracle)
_CPU = {}


def _oracle_elements(args):
    """Oracle element residual/stiffness + COO->CSR assembly of a contiguous
    element range (one process, one BLAS thread)."""
    lo, hi = args
    from threadpoolctl import threadpool_limits

    from oracle import fe
    g = _CPU
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        sub = g["conn"][lo:hi]
        dNdX, w, _ = fe.geometry(g["X"], sub)
        r_e, K_e, _ = fe.element_residual_stiffness(g["u"], sub, dNdX, w, g["om"])
        fe.assemble(sub, r_e, K_e, g["X"].shape[0])
        return time.perf_counter() - t0


def _oracle_points(args):
    """Oracle Psi, P and AA (push-forward route) on a contiguous slice of the
    point batch (one process, one BLAS thread)."""
    lo, hi = args
    from threadpoolctl import threadpool_limits

    from oracle import ncm
    g = _CPU
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ncm.stress_stiffness(g["F"][lo:hi], g["om3"])
        return time.perf_counter() - t0


def cpu_baselines(X, conn, u, theta, theta3, p, Av, n_el_sample, n_pt_sample):
    """The oracle as it stands, timed before the GPU is touched: on one core
    and on every host core (one forked process per core, each with one BLAS
    thread), on contiguous samples of the headline mesh (elements) and of the
    2^22-point batch (its leading points)."""
    import multiprocessing as mp

    from oracle import ncm
    from paper_2510_00884_amd import synth
    ncores = max(1, min(16, os.cpu_count() or 1))
    _CPU.update(X=X, conn=conn, u=u, om=ncm.model_from_theta(theta, p, 32, 2, Av, normalize=True),
                om3=ncm.model_from_theta(theta3, p, 64, 3, Av, normalize=True),
                F=synth.sample_F(n_pt_sample * ncores, seed=0))
    t_el = _oracle_elements((0, n_el_sample))
    t_pt = _oracle_points((0, n_pt_sample))
    with mp.get_context("fork").Pool(ncores) as pool:
        pool.map(_oracle_points, [(0, 64)] * ncores)  # workers up, modules imported
        t0 = time.perf_counter()
        pool.map(_oracle_elements, [(i * n_el_sample, (i + 1) * n_el_sample) for i in range(ncores)])
        t_el_all = time.perf_counter() - t0
        t0 = time.perf_counter()
        pool.map(_oracle_points, [(i * n_pt_sample, (i + 1) * n_pt_sample) for i in range(ncores)])
        t_pt_all = time.perf_counter() - t0
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    _CPU.clear()
    return {
        "value": ncores * n_el_sample * 8 / t_el_all, "unit": "qp evals/s", "cores": ncores, "kind": "oracle",
        "sample": (f"headline 64^3 hex8 mesh, MICNN 2x32: {n_el_sample} contiguous elements per process "
                   f"(geometry, element residual and stiffness by the push-forward route, COO->CSR assembly) in "
                   f"{ncores} processes, one BLAS thread each, {os.cpu_count()} host threads ({cpu_model}); "
                   f"{t_el_all:.1f} s wall, one core alone {t_el:.1f} s"),
        "one_core": {"mesh_qp_per_s": n_el_sample * 8 / t_el, "points_qp_per_s": n_pt_sample / t_pt},
        "all_cores": {"mesh_qp_per_s": ncores * n_el_sample * 8 / t_el_all,
                      "points_qp_per_s": ncores * n_pt_sample / t_pt_all},
        "points_sample": (f"2^22-point batch, MICNN 3x64: Psi, P and AA for {n_pt_sample} points per process; "
                          f"{t_pt_all:.1f} s wall on {ncores} processes, one core alone {t_pt:.1f} s"),
    }


# ---------------------------------------------------------------- GPU timing
def timed(fn, steps, warmup):
    """ms per call of fn (HIP events around the loop on the current stream,
    library profiling off), then one profiled pass of as many calls: per
    kernel the ms per launch and the launches per call (HIP events that the
    library records on its launch stream around every kernel it launches)."""
    import ctypes as C

    import torch

    from paper_2510_00884_amd import _lib as L
    lib = L.load()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    lib.pa_profile_enable(1)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    kern = {}
    for i in range(lib.pa_profile_count()):
        nm, t, k = C.c_char_p(), C.c_double(), C.c_int64()
        lib.pa_profile_get(i, C.byref(nm), C.byref(t), C.byref(k))
        kern[nm.value.decode()] = {"ms_per_launch": t.value / max(k.value, 1), "launches_per_step": k.value / steps}
    lib.pa_profile_enable(0)
    return ms, kern


def say(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def rel(a, b):
    return ((a - b).norm() / b.norm()).item()


# ---------------------------------------------------------------- workloads
def network_roofline(kern, h, L, p, prec, algo, n, hess=True):
    """Roofline records of the network kernel(s) of one call or build."""
    out = {}
    if algo == "forward":
        k = kern.get("mlp_forward")
        if k:
            out["network"] = roof_mfma("mlp_forward", k["ms_per_launch"], mlp_forward_flops(h, L, p) * n,
                                       "bf16" if prec.startswith("bf16") else prec)
        return out
    vg, jac, gram = mlp_adjoint_parts(h, L, p, hess)
    k = kern.get("mlp_adjoint")
    if not k:
        return out
    t = k["ms_per_launch"]
    if prec in ("fp64", "fp32"):
        out["network"] = roof_mfma("mlp_adjoint", t, (vg + jac + gram) * n, prec)
    elif prec in ("bf16", "bf16_corr"):
        out["network"] = roof_mfma("mlp_adjoint", t, (vg + jac + gram) * n, "bf16")
        c = kern.get("mlp_correction")
        if c:
            out["correction"] = roof_mfma("mlp_correction", c["ms_per_launch"],
                                          mlp_adjoint_flops(h, L, p, hess=False) * n, "fp32")
    elif prec == "bf16_jac":
        out["network"] = roof_mixed("mlp_adjoint", t, {"fp32": (vg + gram) * n, "bf16": jac * n})
    return out


def build_roofline(kern, mesh, h, L, p, prec):
    """Roofline records of a tangent build: the network kernel(s) and every
    bandwidth-bound mesh kernel; ``dominant`` names the longest per step."""
    n = mesh.n_el * mesh.nq
    out = network_roofline(kern, h, L, p, prec, "adjoint", n)
    for k, v in kern.items():
        b = mesh_kernel_bytes(k, mesh, p)
        if b:
            out[k] = roof_hbm(k, v["ms_per_launch"], b / max(v["launches_per_step"], 1))
    dom = max(kern, key=lambda k: kern[k]["ms_per_launch"] * kern[k]["launches_per_step"]) if kern else None
    out["dominant"] = {"mlp_adjoint": "network"}.get(dom, dom)
    return out


def bench_points(args):
    """Precision ladder on 2^22 independent points, MICNN 3x64 (Psi, P, AA)."""
    import torch

    from paper_2510_00884_amd import api, synth
    n, n_sv, h, Lh = 1 << 22, 2, 64, 3
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    theta = synth.micnn_params(p, h, Lh, seed=1)
    t0 = time.perf_counter()
    F = torch.tensor(synth.sample_F(n, seed=0), device="cuda")
    say(f"points: 2^22 F drawn in {time.perf_counter() - t0:.1f} s")
    steps, warmup = max(args.steps // 4, 3), 1
    res, ref = {}, None
    models = {a: api.Model(theta, n_sv, h, Lh, A=Av, normalize=True, algorithm=a) for a in ("adjoint", "forward")}
    for prec, algo in [("fp64", "adjoint"), ("fp32", "adjoint"), ("bf16", "adjoint"), ("bf16_corr", "adjoint"),
                       ("bf16_jac", "adjoint"), ("fp64", "forward"), ("fp32", "forward"), ("bf16", "forward"),
                       ("bf16_corr", "forward")]:
        gm = models[algo]
        box = {}

        def call():
            box["out"] = api.energy_stress_tangent(gm, F, prec=prec, out=box.get("out"), workspace=box.get("ws"))
        box["ws"] = torch.empty(gm.lib.pa_material_workspace_bytes(api.C.byref(gm.desc), n), dtype=torch.uint8,
                                device="cuda")
        ms, kern = timed(call, steps, warmup)
        o = box["out"]
        if ref is None:
            ref = {k: v.clone() for k, v in o.items()}
        err = {k: rel(o[k], ref[k]) for k in ("psi", "P", "A")}
        res[f"{prec}/{algo}"] = {"ms": ms, "qp_per_s": n / (ms * 1e-3), "kernels": kern, "rel_err_vs_fp64": err,
                                 "roofline": network_roofline(kern, h, Lh, p, prec, algo, n)}
        say(f"points {prec}/{algo}: {ms:.3f} ms, {n / (ms * 1e-3):.3e} qp/s, err P {err['P']:.1e} A {err['A']:.1e}")
        del o, box
    del ref
    torch.cuda.empty_cache()
    return {"workload": "2^22 independent points F = R U (J in [0.7, 1.4]), orthotropic (9 inputs), MICNN 3x64 "
                        "softplus: Psi, P and dP/dF per point (pa_energy_stress_tangent); errors are normwise "
                        "against the FP64 adjoint-form run",
            "n_points": n, "steps": steps, "precisions": res,
            "value": res["fp64/adjoint"]["qp_per_s"], "unit": "qp evals/s"}


def bench_calib(args):
    """One stress-calibration step on 2^20 samples: stress forward (P only)
    and the parameter adjoint, MICNN 3x64, raw network."""
    import torch

    from paper_2510_00884_amd import api, synth
    n, n_sv, h, Lh = 1 << 20, 2, 64, 3
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    F = torch.tensor(synth.sample_F(n, seed=3), device="cuda").reshape(n, 9).t().contiguous()  # [9][n]
    hidden = api.Model(synth.micnn_params(p, h, Lh, seed=4), n_sv, h, Lh, A=Av, normalize=False,
                       algorithm="adjoint")
    Pref = api.energy_stress_tangent(hidden, F, prec="fp64", psi=False, A=False, soa=True)["P"]
    noise = torch.tensor(synth.rng(5).normal(size=(9, n)), device="cuda")
    Pt = Pref + 0.01 * Pref.pow(2).mean().sqrt() * noise
    gm = api.Model(synth.micnn_params(p, h, Lh, seed=1), n_sv, h, Lh, A=Av, normalize=False, algorithm="adjoint")
    steps, warmup = max(args.steps // 4, 3), 1
    res, grads = {}, {}
    for prec in ("fp32", "fp64"):
        P = api.energy_stress_tangent(gm, F, prec=prec, psi=False, A=False, soa=True)["P"]
        Pbar = (2.0 / n) * (P - Pt)            # dLoss/dP of the loss mean ||P - P_t||^2 (outside the timed path)
        box = {"ws": torch.empty(gm.lib.pa_param_backward_workspace(api.C.byref(gm.desc), api._prec(prec), n),
                                 dtype=torch.uint8, device="cuda")}

        def fwd():
            box["o"] = api.energy_stress_tangent(gm, F, prec=prec, psi=False, A=False, soa=True, out=box.get("o"))

        def bwd():
            box["g"] = api.param_backward(gm, F, Pbar, prec=prec, soa=True, workspace=box["ws"])
        ms_f, kf = timed(fwd, steps, warmup)
        ms_b, kb = timed(bwd, steps, warmup)
        grads[prec] = box["g"].clone()
        roof = network_roofline(kf, h, Lh, p, prec, "adjoint", n, hess=False)
        pb = kb.get("param_backward")
        if pb:
            roof["param_backward"] = roof_mfma("param_backward", pb["ms_per_launch"],
                                               param_bwd_flops(h, Lh, p) * n, prec)
        res[prec] = {"forward_P_ms": ms_f, "adjoint_ms": ms_b, "step_ms": ms_f + ms_b,
                     "samples_per_s": n / ((ms_f + ms_b) * 1e-3), "kernels": {**kf, **kb}, "roofline": roof}
        say(f"calibration {prec}: forward {ms_f:.3f} ms + adjoint {ms_b:.3f} ms")
    res["fp32"]["rel_err_theta_bar_vs_fp64"] = rel(grads["fp32"], grads["fp64"])
    return {"workload": "stress calibration, 2^20 sampled F (seed 3), targets from a hidden MICNN 3x64 (seed 4) "
                        "plus 1% noise; one step = stress forward (P, network value and gradient) + parameter "
                        "adjoint theta_bar; P_bar = dLoss/dP formed once outside the timed calls",
            "n_samples": n, "steps": steps, "precisions": res, "value": res["fp32"]["samples_per_s"],
            "unit": "samples/s"}


def bench_tet10(args):
    """One Newton tangent build on the 56^3 Kuhn tet10 mesh, MICNN 3x64."""
    import torch

    from paper_2510_00884_amd import api, synth
    nc, n_sv, h, Lh = 56, 2, 64, 3
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    t0 = time.perf_counter()
    X, conn, par = synth.tet10_mesh(nc)
    u = torch.tensor(synth.displacement_modes(X, 1.0 / nc, seed=0), device="cuda").reshape(-1)
    gm = api.Model(synth.micnn_params(p, h, Lh, seed=1), n_sv, h, Lh, A=Av, normalize=True, algorithm="adjoint")
    mesh = api.FEMesh(X, conn, colour=par, order="native")
    ws = torch.empty(mesh.workspace_bytes(gm, "gather"), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    say(f"tet10: setup {time.perf_counter() - t0:.1f} s ({mesh.n_el} elements, {mesh.nnz} nonzeros)")
    n_qp = mesh.n_el * mesh.nq
    steps, warmup = max(args.steps // 4, 3), 1
    res, ref = {}, None
    bufs = {}
    for prec in ("fp64", "fp32", "bf16", "bf16_corr", "bf16_jac"):
        ms, kern = timed(lambda: api.tangent_build(gm, mesh, u, prec=prec, workspace=ws, bufs=bufs), steps, warmup)
        e = {"ms": ms, "qp_per_s": n_qp / (ms * 1e-3), "elements_per_s": mesh.n_el / (ms * 1e-3), "kernels": kern}
        if ref is None:
            ref = (bufs["r"].clone(), bufs["vals"].clone())
        else:
            e["rel_err_vs_fp64_r"] = rel(bufs["r"], ref[0])
            e["rel_err_vs_fp64_K"] = rel(bufs["vals"], ref[1])
        e["roofline"] = build_roofline(kern, mesh, h, Lh, p, prec)
        res[prec] = e
        say(f"tet10 {prec}: {ms:.3f} ms")
    out = {"workload": f"Kuhn tet10 mesh of {nc}^3 cubes ({mesh.n_el} elements, {n_qp} points, {3 * mesh.n_nodes} "
                       f"dofs, {mesh.nnz} nonzeros), orthotropic, MICNN 3x64 softplus: one Newton tangent build "
                       "(gather assembly)", "steps": steps, "precisions": res,
           "value": res["fp32"]["qp_per_s"], "unit": "qp evals/s", "value_precision": "fp32"}
    del ref, bufs, ws, mesh
    torch.cuda.empty_cache()
    return out


def bench_sizes(args):
    """Model-size sweep of App. E: the constitutive update (Psi, P, AA) on
    2^20 points for MICNN depths 2-4 x widths 2-64, the CANN and Gent-Thomas.
    Widths up to 8 (FP64, FP32) run on the vector ALUs, wider ones on the
    matrix cores; BF16 on the matrix cores for depths 2-3."""
    import torch

    from paper_2510_00884_amd import api, synth
    n, n_sv = 1 << 20, 2
    p = synth.num_inputs(n_sv)
    Av = synth.structural_vectors(n_sv)
    F = torch.tensor(synth.sample_F(n, seed=0), device="cuda")
    steps, warmup = max(args.steps // 4, 3), 1
    res = {}
    cases = [("micnn", w_, l_) for l_ in (2, 3, 4) for w_ in (2, 4, 8, 16, 32, 64)] + [("cann", 0, 0),
                                                                                      ("gent_thomas", 0, 0)]
    for kind, w_, l_ in cases:
        if kind == "micnn":
            gm = api.Model(synth.micnn_params(p, w_, l_, seed=1), n_sv, w_, l_, A=Av, normalize=True,
                           algorithm="adjoint")
            tag, precs = f"micnn {l_}x{w_}", ("fp64", "fp32") + (("bf16",) if l_ <= 3 else ())
        else:
            th = synth.cann_params(p, seed=2) if kind == "cann" else synth.GENT_THOMAS
            gm = api.Model(th, n_sv, A=Av, normalize=True, kind=kind)
            tag, precs = kind, ("fp64",)
        for prec in precs:
            box = {}

            def call():
                box["o"] = api.energy_stress_tangent(gm, F, prec=prec, out=box.get("o"))
            ms, kern = timed(call, steps, warmup)
            e = {"params": gm.n_params, "ms": ms, "qp_per_s": n / (ms * 1e-3), "kernels": kern}
            k = kern.get("mlp_adjoint")
            if k:
                fl = mlp_adjoint_flops(w_, l_, p) * n
                if w_ <= 8 and prec != "bf16":  # vector-ALU kernel: its FLOPs against the vector peak
                    e["network"] = "valu"
                    t = k["ms_per_launch"] * 1e-3
                    e["roofline"] = {"bound": "alu", "achieved": fl / t / 1e12, "peak": PEAK[prec] / 1e12,
                                     "unit": "TFLOP/s", "frac": fl / t / PEAK[prec], "kernel": "mlp_adjoint",
                                     "ms_per_launch": k["ms_per_launch"], "flop_per_launch": fl}
                else:
                    e["network"] = "mfma"
                    e["roofline"] = network_roofline(kern, max(w_, 16), l_, p, prec, "adjoint", n)["network"]
            res[f"{tag}/{prec}"] = e
            say(f"sizes {tag} ({gm.n_params} params) {prec}: {ms:.3f} ms")
    return {"workload": "model-size sweep (App. E): 2^20 independent points, orthotropic (9 inputs), Psi, P and "
                        "dP/dF; MICNN 2-4 hidden layers x widths 2-64 (widths <= 8 in FP64/FP32 on the vector ALUs; "
                        "the matrix-core roofline of widths below 16 counts the padded width 16), CANN, Gent-Thomas",
            "n_points": n, "steps": steps, "models": res}


def bench_batch(args):
    """Batch-size sweep (Alg. 3 batches; the paper's optimal-batch study):
    the 2^22-point 3x64 constitutive update in batches of 2^10 .. 2^22
    points (pa_energy_stress_tangent_batched, workspace of one batch)."""
    import torch

    from paper_2510_00884_amd import api, synth
    n, n_sv, h, Lh = 1 << 22, 2, 64, 3
    p = synth.num_inputs(n_sv)
    gm = api.Model(synth.micnn_params(p, h, Lh, seed=1), n_sv, h, Lh, A=synth.structural_vectors(n_sv),
                   normalize=True, algorithm="adjoint")
    F = torch.tensor(synth.sample_F(n, seed=0), device="cuda")
    res = {}
    for prec in ("fp64", "bf16"):
        for lb in (10, 12, 14, 16, 18, 20, 22):
            box = {}

            def call():
                box["o"] = api.energy_stress_tangent(gm, F, prec=prec, out=box.get("o"), batch=1 << lb)
            ms, _ = timed(call, 2, 1)
            res[f"{prec}/2^{lb}"] = {"batch": 1 << lb, "ms": ms, "qp_per_s": n / (ms * 1e-3),
                                     "workspace_bytes": gm.lib.pa_material_workspace_bytes(
                                         api.C.byref(gm.desc), 1 << lb)}
            say(f"batch {prec} 2^{lb}: {ms:.3f} ms")
    return {"workload": "2^22 points, MICNN 3x64, Psi + P + dP/dF evaluated in batches of 2^10 .. 2^22 points "
                        "(outputs bitwise independent of the batch)", "n_points": n, "batches": res}


def pipe_probe(blocks=1024, iters=2000, reps=3):
    """Do the matrix cores and the vector ALUs of one SIMD run concurrently?
    Times kinds of work alone in waves 0-3 of 8-wave workgroups, and pairs of
    kinds split over waves 0-3 and 4-7 (two waves per SIMD); a pair taking
    the sum of its parts rather than the larger one means they do not
    overlap."""
    import ctypes as C

    import torch

    from paper_2510_00884_amd import _lib as L
    lib = L.load()
    out = torch.empty(blocks * 512, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    names = {1: "fp64_mfma", 2: "fp32_mfma", 3: "fp64_fma", 4: "fp32_fma", 5: "int_mad"}

    ptr, sp = C.c_void_p(out.data_ptr()), C.c_void_p(stream.cuda_stream)

    def run(lo, hi):
        L.check(lib.pa_pipe_probe(lo, hi, iters, blocks, ptr, sp), "pa_pipe_probe")  # warm-up launch
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            L.check(lib.pa_pipe_probe(lo, hi, iters, blocks, ptr, sp), "pa_pipe_probe")
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    alone = {names[k]: run(k, 0) for k in names}
    pairs = {}
    for lo, hi in ((1, 3), (2, 4), (1, 4), (2, 3), (1, 5), (2, 5)):
        t = run(lo, hi)
        a, b = alone[names[lo]], alone[names[hi]]
        pairs[f"{names[lo]}+{names[hi]}"] = {"ms": t, "sum_ms": a + b, "max_ms": max(a, b),
                                             "overlap": (a + b - t) / min(a, b)}
    return {"probe": "pipe_overlap", "blocks": blocks, "waves_per_block": 8, "iters": iters, "alone_ms": alone,
            "pairs": pairs, "note": "overlap = (sum - pair) / smaller part: 0 = run in turn, 1 = fully concurrent"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64, help="cubes per side of the headline hex8 mesh")
    ap.add_argument("--workloads", default="points,calib,tet10,sizes,batch",
                    help="other workloads carried in the line ('' for none): points, calib, tet10, sizes, batch")
    ap.add_argument("--variants", default="fp32,bf16,bf16_corr,bf16_jac,coloured",
                    help="headline-mesh variants after the FP64 build ('' for none)")
    ap.add_argument("--cpu-elements", type=int, default=2048,
                    help="headline-mesh elements per process in the oracle CPU baseline (0: skip the baseline)")
    ap.add_argument("--cpu-points", type=int, default=16384, help="points per process in the oracle point sample")
    ap.add_argument("--pipe-probe", action="store_true",
                    help="only time the matrix-core / vector-ALU overlap probe (pa_pipe_probe) and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes three times (the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding of the mesh is designed but not built)", file=sys.stderr)
        sys.exit(2)

    from paper_2510_00884_amd import synth
    n = args.n
    n_sv, h, Lh = 2, 32, 2
    p = synth.num_inputs(n_sv)
    X, conn, par = synth.hex_mesh(n)
    u = synth.displacement_modes(X, 1.0 / n, seed=0)
    theta = synth.micnn_params(p, h, Lh, seed=1)
    Av = synth.structural_vectors(n_sv)

    cpu = None
    if args.cpu_elements > 0 and not args.copy_probe:
        t0 = time.perf_counter()
        cpu = cpu_baselines(X, conn, u, theta, synth.micnn_params(p, 64, 3, seed=1), p, Av, args.cpu_elements,
                            args.cpu_points)
        say(f"cpu oracle: {cpu['value']:.3e} qp/s on {cpu['cores']} cores, one core "
            f"{cpu['one_core']['mesh_qp_per_s']:.3e} qp/s ({time.perf_counter() - t0:.1f} s)")

    import torch

    from paper_2510_00884_amd import api

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.pipe_probe:
        print(json.dumps(pipe_probe()), flush=True)
        return
    if args.copy_probe:
        nb = args.copy_probe << 20
        x = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nb, "copy_probe_bytes_written": nb, "launches": 3}), flush=True)
        return

    # ---- headline: 64^3 hex8 tangent build, FP64
    t_setup = time.perf_counter()
    model = api.Model(theta, n_sv, h, Lh, A=Av, normalize=True, algorithm="adjoint")
    mesh = api.FEMesh(X, conn, colour=par, order="native")  # gather build: elements in mesh order
    ut = torch.tensor(u, device="cuda").reshape(-1).contiguous()
    ws = torch.empty(mesh.workspace_bytes(model, "gather"), dtype=torch.uint8, device="cuda")
    bufs = {}
    api.tangent_build(model, mesh, ut, prec="fp64", workspace=ws, bufs=bufs)
    torch.cuda.synchronize()
    say(f"setup {time.perf_counter() - t_setup:.1f} s: {mesh.n_el} elements, {mesh.n_el * mesh.nq} points, "
        f"{3 * mesh.n_nodes} dofs, {mesh.nnz} nonzeros")
    n_qp = mesh.n_el * mesh.nq
    n_el, dofs, nnz = mesh.n_el, 3 * mesh.n_nodes, mesh.nnz

    def build(prec, assembly="gather", w=ws):
        return lambda: api.tangent_build(model, mesh, ut, prec=prec, workspace=w, bufs=bufs, assembly=assembly)

    ms, kern = timed(build("fp64"), args.steps, args.warmup)
    r_ref, v_ref = bufs["r"].clone(), bufs["vals"].clone()
    say(f"hex8 fp64: {ms:.3f} ms/step")
    roofs = build_roofline(kern, mesh, h, Lh, p, "fp64")
    dom = roofs["dominant"]
    roof = dict(roofs[dom])
    if dom == "network":
        sym = f"k_mlp_adj2<{h}, {p}, 0, true>"
        roof["traffic"] = measured_traffic(sym)
        roof["symbol"] = sym
        roof["algorithmic"] = (f"{mlp_adjoint_flops(h, Lh, p)} FLOP/point (adjoint-form value, gradient and "
                               f"Hessian) x {n_qp} points")

    variants = {}
    for vp in [v for v in args.variants.split(",") if v]:
        if vp == "coloured":
            # the fused coloured scatter needs elements numbered colour by colour
            mesh_c = api.FEMesh(X, conn, colour=par, order="colour")
            ws_c = torch.empty(mesh_c.workspace_bytes(model, "coloured"), dtype=torch.uint8, device="cuda")
            vms, vk = timed(lambda: api.tangent_build(model, mesh_c, ut, prec="fp64", workspace=ws_c, bufs=bufs,
                                                      assembly="coloured"), max(args.steps // 2, 3), 1)
            roofv = build_roofline(vk, mesh_c, h, Lh, p, "fp64")
            del ws_c, mesh_c
            key = "fp64_coloured"
        else:
            vms, vk = timed(build(vp), max(args.steps // 2, 3), 1)
            roofv = build_roofline(vk, mesh, h, Lh, p, vp)
            key = vp
        variants[key] = {"value": n_qp / (vms * 1e-3), "ms_per_step": vms,
                         "rel_err_vs_fp64_r": rel(bufs["r"], r_ref), "rel_err_vs_fp64_K": rel(bufs["vals"], v_ref),
                         "kernels": vk, "roofline": roofv}
        say(f"hex8 {key}: {vms:.3f} ms/step, err r {variants[key]['rel_err_vs_fp64_r']:.1e} "
            f"K {variants[key]['rel_err_vs_fp64_K']:.1e}")
    del bufs, ws, mesh, r_ref, v_ref
    torch.cuda.empty_cache()

    workloads = {}
    for wl in [w for w in args.workloads.split(",") if w]:
        fn = {"points": bench_points, "calib": bench_calib, "tet10": bench_tet10, "sizes": bench_sizes,
              "batch": bench_batch}[wl]
        workloads[wl] = fn(args)
        torch.cuda.empty_cache()

    line = {
        "metric": METRIC,
        "value": n_qp / (ms * 1e-3),
        "unit": "qp evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"hex8 {n}^3 unit cube, orthotropic e1/e2 (9 inputs), MICNN 2x32 softplus, one "
                               "Newton tangent build: residual + tangent + CSR assembly (node-centric gather)",
                   "elements": n_el, "points": n_qp, "dofs": dofs, "nnz": nnz},
        "elements_per_s": n_el / (ms * 1e-3),
        "kernels": kern,
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": variants,
        "workloads": workloads,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
