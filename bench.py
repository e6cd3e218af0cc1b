"""Benchmark: matrix-free variable-coefficient pressure-Poisson operator on one MI355X.

Workload (the configuration the headline metric is quoted on): unit cube,
64^3 cells, Q2 (129^3 = 2,146,689 DoFs), droplet phi = tanh((0.25-|x-c|)/(2 eps)),
eps = 2h, rho_l/rho_g = 1000/1, Dirichlet faces.

One step = 100 FP64 operator applies on seed-1 uniform[-1,1] vectors (every
apply reads its own x and phi copy and writes its own y, so the working set
streams from HBM instead of the 256 MB Infinity Cache), then one FP64 Jacobi-PCG
solve and one FP32/FP64 mixed-precision solve to rtol 1e-8 with the
manufactured right-hand side b = A_D p*, p* = sin(pi x) sin(pi y) sin(pi z).

value = operator MDoF/s of the applies (N * applies / apply time), timed with
HIP events on the stream the kernels run on.  After the timed steps the line
also carries the rest of the metric: the cold FP32 Q2 apply, the Q3 (43^3)
FP64 and FP32 applies under the same protocol and its FP64-vs-mixed PCG to
rtol 1e-8, the same solves on the 64^3 Q2 bubble, the adjoint kernels
against their algorithmic bytes, the once-refined mesh, the batched workload
(8 meshes of 16^3..64^3 Q2 with 4 right-hand sides each: one persistent graph
launch, and the batched FP64 PCG of its 32 systems) and FP64 vs mixed PCG on
96^3 Q3 (24.1M DoFs, 20 spheres, ratio 1e4).  After the timed steps the same
applies are also captured in one HIP graph and replayed (`apply_us_graph`,
each replay checked against the eager outputs); `value` stays the eager rate.  One apply is two launches: the
tile kernel and the shared-node assembly; `roofline` prices the pair against
24 algorithmic bytes per DoF (x and phi read, y written once).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6
BYTES_PER_DOF_F64 = 24.0      # x read, phi read, y written once per DoF
BYTES_PER_DOF_F32 = 12.0      # the same vectors in FP32
# Vector bytes per DoF of one FP64 PCG iteration as the three launches move
# them: the apply (p, phi read; q written: 24), the assembly + update (q, r,
# 1/diag read; r written: 32) and the x / p update (r, 1/diag, p, x read; p, x
# written: 48); the shared-node partials and the scalar reductions not counted.
CG_BYTES_PER_DOF_ITER_F64 = 104.0
# FP64 operations of the Q2 cell kernel per cell (coefficient: 3 value sweeps
# and the material law; operator: 3 value sweeps, 3 collocation-derivative
# line pairs with the Gauss-point scaling, 3 transposed value sweeps), counted
# from the compiled tile kernel's instruction mix with an FMA as two
# operations (625 FMAC + 50 FMA + 408 MUL); the slot sums of the write-out are
# not counted.
FLOPS_PER_CELL_Q2 = 1758.0
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "apply_q2_64cube_traffic.md")
KERNEL_SOURCES = ["apply_impl.h", "apply_configs.h", "apply_misc.hip", "apply_f64.hip", "apply_f64_k2.hip", "common.h",
                  "tables.h", "shared_nodes.h", "kernels.h", "bounds.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--applies", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="leave out the secondary figures (Q3, FP32, batch, solvers of the other rows)")
    ap.add_argument("--extras", action="store_true", help="also time FP32, Q3/Q4, hot-cache applies, bubble solves")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed steps, run a plain 512 MiB device copy (counter calibration)")
    ap.add_argument("--sweep", type=int, default=0, metavar="K",
                    help="instead of the bench line: time every apply configuration of degree K on the droplet "
                         "(cold, 100 applies) and print one JSON line per configuration")
    ap.add_argument("--variants", default="", help="with --sweep: comma-separated kernel variants to time")
    ap.add_argument("--figure", default="", choices=["", "closest_points", "filter", "adjoint", "amr", "c2", "batch"],
                    help="instead of the bench line: only this secondary figure, as one JSON line")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2401_07805_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(cfg):
    """HBM bytes per apply of kernel configuration cfg (FP64) from the committed
    counter summary, if it was taken on the current kernel sources and covers
    that configuration (else None)."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    mh = re.search(r"kernel sources hash:\s*([0-9a-f]+)", text)
    if not mh or mh.group(1) != kernel_hash():
        return None
    tile = ",".join(str(int(t)) for t in cfg["tile"])
    mb = re.search(r"apply traffic: variant %d tile %s bytes ([0-9.eE+]+)" % (int(cfg["variant"]), tile), text)
    return float(mb.group(1)) if mb else None


def lscpu_facts():
    """Model, sockets, cores and threads of the host from `lscpu` (empty if unavailable)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return {}
    keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket",
            "Thread(s) per core": "threads_per_core", "CPU(s)": "cpus"}
    facts = {}
    for line in out.splitlines():
        if ":" not in line:
            continue
        k, v = (t.strip() for t in line.split(":", 1))
        if k in keys:
            facts[keys[k]] = int(v) if v.isdigit() else v
    return facts


def cpu_baseline():
    """The FP64 oracle (CSR assembled by full quadrature; CSR SpMV; textbook
    Jacobi PCG) on the host cores, on a bounded sample of the same workload:
    32^3 cells Q2 of the droplet (r 0.25, eps = 2h, ratio 1000)."""
    import oracle
    import workloads as W
    wl = W.droplet_at_scale(k=2, n=32, nvec=1, seed=1)
    m = wl.mesh
    t0 = time.perf_counter()
    op = oracle.Operator(m, phi=wl.phi)
    t_asm = time.perf_counter() - t0
    x = wl.vectors[0]
    op.matvec(x)
    op.matvec(x)
    ts = []
    for _ in range(10):
        t0 = time.perf_counter()
        op.matvec(x)
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    b = oracle.manufactured_sine_rhs(m, 0.25, m.eps)
    t0 = time.perf_counter()
    _, pinfo = op.pcg(b, rtol=1e-8)
    t_pcg = time.perf_counter() - t0
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    ts1 = []
    for _ in range(3):
        t0 = time.perf_counter()
        op.matvec(x)
        ts1.append(time.perf_counter() - t0)
    oracle.set_num_threads(threads)
    t1 = float(np.median(ts1))
    return {"value": m.ndofs / t / 1e6, "unit": "MDoF/s", "cores": threads, "kind": "oracle",
            "value_1_thread": m.ndofs / t1 / 1e6, "lscpu": lscpu_facts(),
            "pcg_rtol_1e-8_s": t_pcg, "pcg_iterations": pinfo["iterations"],
            "pcg_us_per_iter": t_pcg / max(pinfo["iterations"], 1) * 1e6,
            "sample": f"FP64 CSR SpMV, median of 10 after 2 warm-ups, droplet 32^3 cells Q2 "
                      f"({m.ndofs} DoFs, nnz {op.nnz}); assembly {t_asm:.2f} s not included; "
                      f"value_1_thread: median of 3 on one thread; pcg: Jacobi PCG from 0 to rtol 1e-8 with "
                      f"the manufactured right-hand side, wall time on `cores` threads"}


def timed_applies(torch, probs, xs, ys, napp, stream, prec_tensor=None):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    npool = len(probs)
    e0.record(stream)
    for i in range(napp):
        probs[i % npool].apply(xs[i], out=ys[i])
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3


def graph_applies(torch, probs, xs, ys, napp, dev, reps=5):
    """The same applies captured in one HIP graph (torch's stream capture of the
    library's launches) and replayed `reps` times, outside the timed steps.
    Before every replay the outputs are cleared by eager work; after it they
    are compared with the eager applies' outputs.  Returns the median seconds
    per apply and the largest relative difference of any replay."""
    npool = len(probs)
    ref = ys.clone()
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        for i in range(napp):
            probs[i % npool].apply(xs[i], out=ys[i])
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for i in range(napp):
            probs[i % npool].apply(xs[i], out=ys[i])
    torch.cuda.synchronize()
    scale = float(ref.abs().max())
    ts, diff = [], 0.0
    for _ in range(reps):
        ys.zero_()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3 / napp)
        diff = max(diff, float((ys - ref).abs().max()) / scale)
    del g
    return float(np.median(ts)), diff


def cold_rate(torch, probs, X, Y, napp, reps=3):
    """Median seconds per apply of napp applies rotating over a pool of problems
    (each with its own phi copy) and over napp distinct x / y vectors."""
    npool = len(probs)
    for i in range(napp):
        probs[i % npool].apply(X[i], out=Y[i])
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(napp):
            probs[i % npool].apply(X[i], out=Y[i])
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3 / napp)
    return float(np.median(ts))


def solve_pair(p, b, rtol=1e-8):
    """Host wall time of FP64 and mixed PCG from 0 to rtol (the same FP64 true
    residual criterion), each after one untimed solve that builds its graphs."""
    out = {}
    for prec in ("fp64", "mixed"):
        p.cg_solve(b, rtol=rtol, precision=prec)
        t0 = time.perf_counter()
        _, info = p.cg_solve(b, rtol=rtol, precision=prec)
        out[f"cg_{prec}_s"] = time.perf_counter() - t0
        out[f"cg_{prec}_iters"] = info["iterations"]
        out[f"cg_{prec}_true_rel_res"] = info["true_rel_residual"]
        if prec == "mixed":
            out["cg_mixed_deflation_corrections"] = info["deflation_corrections"]
    return out


def secondary(torch, vpp, W, dev, cache, xs, ys, probs_q2):
    """Figures of the metric beyond the headline apply, outside the timed steps:
    the cold FP32 Q2 apply; the Q3 43^3 FP64 and FP32 applies (cold, same
    protocol) and its FP64-vs-mixed PCG to rtol 1e-8; the same solves on the 64^3
    Q2 bubble; dJ/dc (grad_coef) and dJ/dphi (grad_phi) at 64^3 Q2 against
    their algorithmic bytes; the once-refined mesh; the batched workload's
    aggregate apply rate and batched PCG; FP64 vs mixed PCG at 96^3 Q3."""
    out = {}
    napp = xs.shape[0]
    N2 = probs_q2[0].n
    x32, y32 = xs.float(), torch.empty(xs.shape, dtype=torch.float32, device=dev)
    t = cold_rate(torch, probs_q2, x32, y32, napp)
    out["q2_f32"] = {"apply_us": t * 1e6, "mdofs": N2 / t / 1e6,
                     "roofline_frac": BYTES_PER_DOF_F32 * N2 / t / 1e9 / HBM_PEAK_GBS,
                     "kernel": probs_q2[0].config_for("fp32")}
    del x32, y32
    # Q3, 43^3 cells (2,197,000 DoFs), same droplet and protocol
    wl = W.droplet_at_scale(k=3, nvec=0)
    m3 = wl.mesh
    N3 = m3.ndofs
    phi3 = torch.from_numpy(wl.phi).to(dev)
    npool = max(1, min(napp, math.ceil(600e6 / (BYTES_PER_DOF_F64 * N3))))
    p3 = []
    for i in range(npool):
        p = vpp.Problem.from_mesh(m3)
        p.set_phi(phi3)
        p3.append(p)
    c3 = p3[0].tune(cache)
    c332 = p3[0].config_for("fp32")
    for p in p3[1:]:
        p.set_config(c3["variant"], c3["tile"], "fp64")
        p.set_config(c332["variant"], c332["tile"], "fp32")
    X3 = torch.from_numpy(W.uniform_vectors(1, napp, N3)).to(dev)
    Y3 = torch.empty_like(X3)
    t64 = cold_rate(torch, p3, X3, Y3, napp)
    X3f = X3.float()
    del X3, Y3
    Y3f = torch.empty_like(X3f)
    t32 = cold_rate(torch, p3, X3f, Y3f, napp)
    del X3f, Y3f
    q3 = {"ndofs": N3, "f64_apply_us": t64 * 1e6, "f64_mdofs": N3 / t64 / 1e6,
          "f64_roofline_frac": BYTES_PER_DOF_F64 * N3 / t64 / 1e9 / HBM_PEAK_GBS,
          "f32_apply_us": t32 * 1e6, "f32_mdofs": N3 / t32 / 1e6,
          "f32_roofline_frac": BYTES_PER_DOF_F32 * N3 / t32 / 1e9 / HBM_PEAK_GBS,
          "kernel_fp64": c3, "kernel_fp32": c332}
    ps = torch.from_numpy(W.sine_field(m3)).to(dev)
    ps[torch.from_numpy(m3.boundary_mask()).to(dev)] = 0.0
    q3.update(solve_pair(p3[0], p3[0].apply(ps)))
    out["q3"] = q3
    del p3
    # bubble 64^3 Q2: the same solves
    wb = W.droplet_at_scale(k=2, nvec=0, bubble=True)
    pb = vpp.Problem.from_mesh(wb.mesh)
    pb.set_phi(torch.from_numpy(wb.phi).to(dev))
    pb.tune(cache)
    ps = torch.from_numpy(W.sine_field(wb.mesh)).to(dev)
    ps[torch.from_numpy(wb.mesh.boundary_mask()).to(dev)] = 0.0
    out["bubble_q2"] = solve_pair(pb, pb.apply(ps))
    del pb
    # adjoint kernels at 64^3 Q2 (hot: p, lam, g_q from the previous call)
    p0 = probs_q2[0]
    pv, lam = xs[0], xs[1]
    g = p0.grad_coef(pv, lam)
    gphi = p0.grad_phi(g)
    nq = p0.nq
    res = {}
    for name, fn, nbytes in (("grad_coef", lambda: p0.grad_coef(pv, lam), 16.0 * N2 + 8.0 * nq),
                             ("grad_phi", lambda: p0.grad_phi(g), 16.0 * N2 + 8.0 * nq)):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            fn()
        e1.record()
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 20
        res[name] = {"us": us, "algorithmic_bytes": nbytes, "achieved_gbs": nbytes / us / 1e3,
                     "roofline_frac": nbytes / us / 1e3 / HBM_PEAK_GBS}
    del gphi
    out["adjoint_q2"] = res
    out["amr_q2"] = amr_figures(torch, vpp, W, dev)
    # the batched workload (aggregate rate and batched PCG) and mixed precision
    # at scale (96^3 Q3, 24.1M DoFs)
    out["c3_batch"] = batch_figures(torch, vpp, W, dev, cache, per_mesh=False)
    out["c2_q3_96"] = c2_figures(torch, vpp, W, dev, cache)
    return out


def amr_figures(torch, vpp, W, dev):
    """Once-refined mesh with hanging nodes: 32^3 coarse Q2 cells, the cells
    within three cells of the droplet's interface (r 0.25) refined once, phi
    with eps = half the fine cell size on both lattices, ratio 1000.  Hot apply
    (HIP events, 20 applies) per free unknown, against 24 B per entry of the
    two-lattice vector (x, phi read, y written), and PCG from 0 to rtol 1e-8
    for the nodal values of sin(pi x) sin(pi y) sin(pi z) as a synthetic
    right-hand side."""
    n = 32
    m = W.unit_cube(n, 2, 1000.0, 1.0)
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    mask = (np.abs(np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2) - 0.25) < 3.0 * h).ravel()
    p = vpp.AmrProblem(m.ncells, 2, mask, m.origin, m.extent, m.bc, m.rho_l, m.rho_g, m.heaviside)
    # node coordinates of both lattices (Q2: equidistant support points)
    xs = []
    for nn in (2 * n + 1, 4 * n + 1):
        ax = np.linspace(0.0, 1.0, nn)
        Zz, Yy, Xx = np.meshgrid(ax, ax, ax, indexing="ij")
        xs.append((Xx.ravel(), Yy.ravel(), Zz.ravel()))
    x, y, z = (np.concatenate([xs[0][d], xs[1][d]]) for d in range(3))
    eps = 0.5 * h / 2.0
    phi = np.tanh((0.25 - np.sqrt((x - .5) ** 2 + (y - .5) ** 2 + (z - .5) ** 2)) / (2 * eps))
    p.set_phi(torch.from_numpy(phi).to(dev))
    xv = torch.from_numpy(W.uniform_vectors(1, 1, p.n)[0]).to(dev)
    yv = torch.empty_like(xv)
    p.apply(xv, out=yv)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        p.apply(xv, out=yv)
    e1.record()
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / 20
    b = torch.from_numpy(np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)).to(dev)
    p.cg_solve(b, rtol=1e-8)
    t0 = time.perf_counter()
    _, info = p.cg_solve(b, rtol=1e-8)
    t_cg = time.perf_counter() - t0
    nbytes = 24.0 * p.n
    return {"coarse_cells": n ** 3, "refined_cells": int(mask.sum()), "entries": p.n, "free": p.nfree,
            "apply_us": us, "mdofs_free": p.nfree / us, "bytes_per_apply_24_per_entry": nbytes,
            "roofline_frac_24_per_entry": nbytes / us / 1e3 / HBM_PEAK_GBS,
            "cg_s": t_cg, "cg_iters": info["iterations"], "cg_true_rel_res": info["true_rel_residual"]}


def extras(torch, vpp, W, dev, cache):
    """Secondary figures: FP32 and hot-cache applies at Q2, Q3/Q4 applies, bubble solves."""
    out = {}
    for k in (2, 3, 4):
        wl = W.droplet_at_scale(k=k, nvec=1, seed=1)
        p = vpp.Problem.from_mesh(wl.mesh)
        p.set_phi(torch.from_numpy(wl.phi).to(dev))
        p.tune(cache)
        x = torch.from_numpy(wl.vectors[0]).to(dev)
        for tag, xx in (("f64", x), ("f32", x.float())):
            yy = torch.empty_like(xx)
            for _ in range(3):
                p.apply(xx, out=yy)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(50):
                p.apply(xx, out=yy)
            e1.record()
            e1.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / 50
            out[f"q{k}_{tag}_hot_apply_us"] = us
            out[f"q{k}_{tag}_hot_mdofs"] = wl.mesh.ndofs / us
        if k == 3:
            ps = torch.from_numpy(W.sine_field(wl.mesh)).to(dev)
            ps[torch.from_numpy(wl.mesh.boundary_mask()).to(dev)] = 0.0
            b = p.apply(ps)
            for prec in ("fp64", "mixed"):
                t0 = time.perf_counter()
                _, info = p.cg_solve(b, rtol=1e-8, precision=prec)
                out[f"q3_cg_{prec}_s"] = time.perf_counter() - t0
                out[f"q3_cg_{prec}_iters"] = info["iterations"]
    out.update(batch_figures(torch, vpp, W, dev, cache))
    out.update(filter_figures(torch, vpp, W, dev, cache))
    out.update(adjoint_figures(torch, vpp, W, dev, cache))
    out.update(closest_point_figures(torch, vpp, W, dev))
    out.update(c2_figures(torch, vpp, W, dev, cache))
    wl = W.droplet_at_scale(k=2, nvec=0, bubble=True)
    p = vpp.Problem.from_mesh(wl.mesh)
    p.set_phi(torch.from_numpy(wl.phi).to(dev))
    p.tune(cache)
    ps = torch.from_numpy(W.sine_field(wl.mesh)).to(dev)
    ps[torch.from_numpy(wl.mesh.boundary_mask()).to(dev)] = 0.0
    b = p.apply(ps)
    for prec in ("fp64", "mixed"):
        p.cg_solve(b, rtol=1e-8, precision=prec)
        t0 = time.perf_counter()
        _, info = p.cg_solve(b, rtol=1e-8, precision=prec)
        out[f"bubble_q2_cg_{prec}_s"] = time.perf_counter() - t0
        out[f"bubble_q2_cg_{prec}_iters"] = info["iterations"]
    return out


def filter_figures(torch, vpp, W, dev, cache):
    """Level-set filter system at 64^3 Q2: (M + eta h^2 K) n = b with eta = 2 and
    pure Neumann faces (Eq. normal_vector_regularized in weak form); hot FP64
    apply of the mass-shifted operator, and Jacobi PCG to the tolerances of
    Table tab:solver_settings (rtol 1e-12, atol 1e-20) for the three components
    of a droplet's interface normal, each with b = A n (so n is the exact
    discrete solution)."""
    n = 64
    filt = 2.0 / (n * n)
    m = W.Mesh(ncells=(n, n, n), degree=2, bc=(1,) * 6, rho_l=1.0 / filt, rho_g=1.0 / filt, mass=1.0)
    p = vpp.Problem.from_mesh(m)
    p.set_phi(torch.zeros(m.ndofs, dtype=torch.float64, device=dev))
    p.set_mass(1.0)
    p.tune(cache)
    comps = [torch.from_numpy(c).to(dev) for c in W.normal_field(m)]
    yy = torch.empty_like(comps[0])
    for _ in range(3):
        p.apply(comps[0], out=yy)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(50):
        p.apply(comps[0], out=yy)
    e1.record()
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / 50
    bs = [p.apply(c) for c in comps]
    p.cg_solve(bs[0], rtol=1e-12, atol=1e-20, max_iter=2, raise_on_failure=False)   # graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sols = [p.cg_solve(b, rtol=1e-12, atol=1e-20) for b in bs]
    t = time.perf_counter() - t0
    err = max(float(torch.linalg.norm(x - c) / torch.linalg.norm(c)) for (x, _), c in zip(sols, comps))
    # the chain on a droplet (r 0.25, eps = 2h): phi -> (n_bar, v) -> normal filters
    # -> (-div n, v) -> curvature filter, each right-hand side formed on the GPU
    phi = torch.from_numpy(W.droplet_phi(m, 0.25, 2.0 / n)).to(dev)
    p.normal_rhs(phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bn = p.normal_rhs(phi)
    torch.cuda.synchronize()
    t_nrhs = time.perf_counter() - t0
    ns = [p.cg_solve(b, rtol=1e-12, atol=1e-20)[0] for b in bn]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bk = p.curvature_rhs(*ns)
    torch.cuda.synchronize()
    t_krhs = time.perf_counter() - t0
    t0 = time.perf_counter()
    kap, kinfo = p.cg_solve(bk, rtol=1e-12, atol=1e-20)
    t_k = time.perf_counter() - t0
    band = phi.abs() < 0.5
    # one reinitialization step of a too-sharp profile (eps/2) with the filtered
    # normal, pseudo-time step eps (Eq. reinitialization; Table tab:solver_settings)
    eps = 2.0 / n
    psi = torch.from_numpy(W.droplet_phi(m, 0.25, 0.5 * eps)).to(dev)
    p.reinit_step(psi, ns, eps, eps, max_iter=2, raise_on_failure=False)   # workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rinfo = p.reinit_step(psi, ns, eps, eps)
    t_r = time.perf_counter() - t0
    return {"reinit_step_s": t_r, "reinit_cg_iters": rinfo["iterations"],
            "filter_q2_config": p.config, "filter_q2_f64_hot_apply_us": us,
            "filter_q2_f64_hot_mdofs": m.ndofs / us, "filter_normal_cg_s": t,
            "filter_normal_cg_iters": [i["iterations"] for _, i in sols], "filter_normal_cg_max_rel_err": err,
            "filter_normal_rhs_us": t_nrhs * 1e6, "filter_curvature_rhs_us": t_krhs * 1e6,
            "filter_curvature_cg_s": t_k, "filter_curvature_cg_iters": kinfo["iterations"],
            "filter_curvature_band_mean_over_2_by_r": float(kap[band].mean()) / (2.0 / 0.25)}


def adjoint_figures(torch, vpp, W, dev, cache):
    """The adjoint workload: 48^3 Q2 droplet r 0.3 against the target r 0.28,
    J = 1/2 |p - p_t|^2; forward PCG, then the backward pass of the autograd
    Function (adjoint PCG, dJ/dc at every Gauss point, dJ/dphi at the nodes),
    both to rtol 1e-10.  b = A_D(phi_t) p* for the manufactured sine p*,
    formed once and then held fixed (an input independent of phi)."""
    m, phi, phit = W.adjoint_case(n=48, k=2)
    prob = vpp.Problem.from_mesh(m)
    prob.set_phi(torch.from_numpy(phit).to(dev))
    prob.tune(cache)
    ps = torch.from_numpy(W.sine_field(m)).to(dev)
    ps[torch.from_numpy(m.boundary_mask()).to(dev)] = 0.0
    b = prob.apply(ps)
    pt, _ = prob.cg_solve(b, rtol=1e-10)
    times = {}
    for rep in range(2):                       # the first pass builds the graphs
        phi_t = torch.from_numpy(phi).to(dev).requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = vpp.poisson_solve(phi_t, b, prob, rtol=1e-10)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J = 0.5 * ((p - pt) ** 2).sum()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times = {"forward": t1 - t0, "backward": t2 - t1}
    return {"adjoint_c4_ndofs": m.ndofs, "adjoint_c4_forward_s": times["forward"],
            "adjoint_c4_backward_s": times["backward"],
            "adjoint_c4_grad_norm": float(torch.linalg.norm(phi_t.grad))}


def closest_point_figures(torch, vpp, W, dev):
    """Closest-point projection of the narrow band |phi| < 0.9 of the 64^3 Q2
    droplet (r 0.25, eps = 2h) onto {phi_h = 0}: 3 normal corrections per outer
    step, tol 1e-11, at most 50 outer steps; one launch over all support points.
    Timed twice: with the normalised gradient of phi_h as the normal, and with
    the filtered normal field (the three normal-filter solves, eta = 2, are set
    up before and not timed)."""
    wl = W.droplet_at_scale(k=2, nvec=0)
    p = vpp.Problem.from_mesh(wl.mesh)
    p.set_phi(torch.from_numpy(wl.phi).to(dev))
    eps = wl.mesh.eps
    y, info = p.closest_points(eps)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 5
    for _ in range(reps):
        y, info = p.closest_points(eps)
    e1.record()
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    band = info >= 0
    nb = int(band.sum())
    out = {"cp_band_points": nb, "cp_us": us, "cp_mpoints_per_s": nb / us,
           "cp_converged_fraction": float((info > 0).sum()) / max(nb, 1),
           "cp_mean_outer_steps": float(info[info > 0].double().mean())}
    # the same band with the filtered normal (eta = 2) as the normal of the corrections
    n = wl.mesh.ncells[0]
    filt = 2.0 / n ** 2
    mf = W.Mesh(ncells=wl.mesh.ncells, degree=2, bc=(1,) * 6, rho_l=1 / filt, rho_g=1 / filt)
    pf = vpp.Problem.from_mesh(mf)
    pf.set_phi(torch.zeros(mf.ndofs, dtype=torch.float64, device=dev))
    pf.set_mass(1.0)
    comps = [pf.cg_solve(b, rtol=1e-12, atol=1e-20)[0] for b in pf.normal_rhs(torch.from_numpy(wl.phi).to(dev))]
    y, info = p.closest_points(eps, normal=comps)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        y, info = p.closest_points(eps, normal=comps)
    e1.record()
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    out.update({"cp_filtered_normal_us": us,
                "cp_filtered_normal_converged_fraction": float((info > 0).sum()) / max(nb, 1),
                "cp_filtered_normal_mean_outer_steps": float(info[info > 0].double().mean())})
    return out


def c2_figures(torch, vpp, W, dev, cache):
    """Mixed precision at scale: 96^3 Q3 (24.1M DoFs), union of 20 spheres, ratio
    1e4, eps = 1.5h; FP64 PCG and mixed PCG to rtol 1e-8 (same FP64 residual
    criterion), errors against a tight FP64 solve (rtol 1e-11)."""
    wl = W.spheres_mixed(n=96, k=3)
    m = wl.mesh
    p = vpp.Problem.from_mesh(m)
    p.set_phi(torch.from_numpy(wl.phi).to(dev))
    p.tune(cache)
    ps = torch.from_numpy(W.sine_field(m)).to(dev)
    ps[torch.from_numpy(m.boundary_mask()).to(dev)] = 0.0
    b = p.apply(ps)
    out = {"c2_ndofs": m.ndofs}
    pref, iref = p.cg_solve(b, rtol=1e-11)
    for prec in ("fp64", "mixed"):
        t0 = time.perf_counter()
        x, info = p.cg_solve(b, rtol=1e-8, precision=prec)
        out[f"c2_cg_{prec}_s"] = time.perf_counter() - t0
        out[f"c2_cg_{prec}_iters"] = info["iterations"]
        out[f"c2_cg_{prec}_true_rel_res"] = info["true_rel_residual"]
        out[f"c2_cg_{prec}_err_vs_tight_fp64"] = float(torch.linalg.norm(x - pref) / torch.linalg.norm(pref))
    return out


def batch_figures(torch, vpp, W, dev, cache, per_mesh=True):
    """The batched workload: 8 independent single-sphere meshes of 16..64 cells per
    side (Q2, 7.6M DoFs) with 4 right-hand sides each, applied by one persistent
    graph launch; aggregate (and with per_mesh, per-mesh) DoF-rhs rates, the
    batched FP64 PCG of its 32 systems, and a Q3 batch (8 meshes of 8..32 cells
    per side, 4 right-hand sides each) against its 32 single applies."""
    wls = W.batch_meshes()
    probs, xs = [], []
    for wl in wls:
        p = vpp.Problem.from_mesh(wl.mesh)
        p.set_phi(torch.from_numpy(wl.phi).to(dev))
        probs.append(p)
        xs += [torch.from_numpy(v).to(dev) for v in wl.vectors]
    ys = [torch.empty_like(x) for x in xs]
    nrhs = [len(wl.vectors) for wl in wls]
    bt = vpp.Batch(probs, nrhs, tune_cache=cache)

    def rate(batch, xx, yy, dofs, reps=20):
        batch.apply(xx, yy)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            batch.apply(xx, yy)
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / reps
        return t, dofs / t / 1e6

    total = sum(wl.mesh.ndofs * len(wl.vectors) for wl in wls)
    t, r = rate(bt, xs, ys, total)
    out = {"batch_config": bt.config, "batch_dof_rhs": total, "batch_apply_us": t * 1e6,
           "batch_aggregate_mdofs": r, "batch_per_mesh_mdofs": []}
    i = 0
    for p, wl, nr in zip(probs, wls, nrhs) if per_mesh else ():
        b1 = vpp.Batch([p], [nr], tune_cache=cache)
        _, r1 = rate(b1, xs[i:i + nr], ys[i:i + nr], wl.mesh.ndofs * nr)
        out["batch_per_mesh_mdofs"].append({"n": wl.mesh.ncells[0], "ratio": wl.extra["ratio"], "mdofs": r1})
        i += nr
    out.update(batch_cg_figures(torch, bt, probs, xs))
    # Q3 batches: eight meshes of 8..32 cells per side with four right-hand
    # sides each, batched against the same 32 single-problem applies
    q3 = W.batch_meshes(sizes=(8, 10, 12, 14, 16, 20, 24, 32), nrhs=4, k=3)
    qp, qx = [], []
    for wl in q3:
        p = vpp.Problem.from_mesh(wl.mesh)
        p.set_phi(torch.from_numpy(wl.phi).to(dev))
        qp.append(p)
        qx += [torch.from_numpy(v).to(dev) for v in wl.vectors]
    qy = [torch.empty_like(x) for x in qx]
    qb = vpp.Batch(qp, [4] * len(qp), tune_cache=cache)
    qtotal = sum(wl.mesh.ndofs * 4 for wl in q3)
    tq, rq = rate(qb, qx, qy, qtotal)

    class Singles:
        def apply(self, xx, yy):
            for j, (x, y) in enumerate(zip(xx, yy)):
                qp[j // 4].apply(x, out=y)

    ts, rs = rate(Singles(), qx, qy, qtotal)
    out.update({"q3_batch_config": qb.config, "q3_batch_dof_rhs": qtotal, "q3_batch_apply_us": tq * 1e6,
                "q3_batch_aggregate_mdofs": rq, "q3_single_applies_us": ts * 1e6, "q3_single_applies_mdofs": rs})
    return out


def batch_cg_figures(torch, bt, probs, bs):
    """Batched FP64 PCG of the 32 systems of the batched workload (its vectors
    as right-hand sides, rtol 1e-8), host call to return, against the same
    systems solved one after another with the single-problem solver."""
    owner = [p for p, nr in zip(probs, bt.nrhs) for _ in range(nr)]
    # warm-up: workspaces and graphs of both paths
    bt.cg_solve(bs, [torch.zeros_like(b) for b in bs], rtol=1e-8, max_iter=2, raise_on_failure=False)
    for p in probs:
        p.cg_solve(bs[owner.index(p)], rtol=1e-8, max_iter=2, raise_on_failure=False)
    xs = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = bt.cg_solve(bs, xs, rtol=1e-8)
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    seq = [p.cg_solve(b, rtol=1e-8)[1] for p, b in zip(owner, bs)]
    t_seq = time.perf_counter() - t0
    return {"batch_cg_fp64_s": t_batch, "batch_cg_iters_max": max(i["iterations"] for i in infos),
            "batch_cg_iters_sum": sum(i["iterations"] for i in infos),
            "batch_cg_worst_true_rel_res": max(i["true_rel_residual"] for i in infos),
            "batch_cg_sequential_fp64_s": t_seq,
            "batch_cg_sequential_iters_sum": sum(i["iterations"] for i in seq)}


def config_sweep(torch, vpp, W, k, variants):
    """Cold FP64 / FP32 apply time of every tuner candidate of degree k on the
    droplet at its full size (64^3 Q2, 43^3 Q3, 32^3 Q4), each configuration's
    FP64 output compared with the first one's.  FP32 is timed only for
    configurations that have an FP32 kernel."""
    dev = torch.device("cuda", 0)
    wl = W.droplet_at_scale(k=k, nvec=0)
    m = wl.mesh
    N = m.ndofs
    napp = 100
    npool = max(1, min(napp, math.ceil(600e6 / (BYTES_PER_DOF_F64 * N))))
    phi_t = torch.from_numpy(wl.phi).to(dev)
    probs = []
    for _ in range(npool):
        p = vpp.Problem.from_mesh(m)
        p.set_phi(phi_t)
        probs.append(p)
    xs = torch.from_numpy(W.uniform_vectors(1, napp, N)).to(dev)
    ys = torch.empty_like(xs)
    x32 = xs.float()
    y32 = torch.empty_like(x32)
    log(f"sweep k={k} N={N} pool={npool}")
    ref = None
    for cfg in vpp.config_candidates(k):
        if variants and int(cfg["variant"]) not in variants:
            continue
        for p in probs:
            p.set_config(cfg["variant"], cfg["tile"], "fp64")
        t64 = cold_rate(torch, probs, xs, ys, napp)
        line = {"k": k, "ndofs": N, "variant": int(cfg["variant"]), "tile": list(cfg["tile"]),
                "fp64_us": t64 * 1e6, "fp64_frac": BYTES_PER_DOF_F64 * N / t64 / 1e9 / HBM_PEAK_GBS}
        try:
            for p in probs:
                p.set_config(cfg["variant"], cfg["tile"], "fp32")
        except vpp.VppError:
            pass                      # an FP64-only configuration
        else:
            t32 = cold_rate(torch, probs, x32, y32, napp)
            line["fp32_us"] = t32 * 1e6
            line["fp32_frac"] = BYTES_PER_DOF_F32 * N / t32 / 1e9 / HBM_PEAK_GBS
        y0 = ys[0].clone()
        if ref is None:
            ref = y0
        line["rel_diff_vs_first"] = float(torch.linalg.norm(y0 - ref) / torch.linalg.norm(ref))
        print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (the operator's multi-GPU sharding is a design "
              "note); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.sweep:
        import workloads as W
        import paper_2401_07805_amd as vpp
        variants = {int(v) for v in args.variants.split(",") if v}
        config_sweep(torch, vpp, W, args.sweep, variants)
        return
    if args.figure:
        import workloads as W
        import paper_2401_07805_amd as vpp
        dev = torch.device("cuda", 0)
        cache = os.path.join(ROOT, "paper_2401_07805_amd", "tune_cache.json")
        fig = {"closest_points": lambda: closest_point_figures(torch, vpp, W, dev),
               "filter": lambda: filter_figures(torch, vpp, W, dev, cache),
               "adjoint": lambda: adjoint_figures(torch, vpp, W, dev, cache),
               "amr": lambda: amr_figures(torch, vpp, W, dev),
               "c2": lambda: c2_figures(torch, vpp, W, dev, cache),
               "batch": lambda: batch_figures(torch, vpp, W, dev, cache)}[args.figure]()
        print(json.dumps({"figure": args.figure, **fig}), flush=True)
        return
    import workloads as W
    import paper_2401_07805_amd as vpp

    dev = torch.device("cuda", 0)
    wl = W.droplet_at_scale(k=2, nvec=0)
    m = wl.mesh
    N = m.ndofs
    napp = args.applies
    log(f"workload {wl.name} N={N}")
    # one phi copy per problem handle; applies rotate over them so that x, phi
    # and y of consecutive applies do not share cache lines
    npool = max(1, min(napp, math.ceil(600e6 / (BYTES_PER_DOF_F64 * N))))
    phi_t = torch.from_numpy(wl.phi).to(dev)
    probs = []
    for i in range(npool):
        p = vpp.Problem.from_mesh(m)
        p.set_phi(phi_t)
        probs.append(p)
    cache = os.path.join(ROOT, "paper_2401_07805_amd", "tune_cache.json")
    cfg = probs[0].tune(cache)
    cfg32 = probs[0].config_for("fp32")
    for p in probs[1:]:
        p.set_config(cfg["variant"], cfg["tile"], "fp64")
        p.set_config(cfg32["variant"], cfg32["tile"], "fp32")
    log(f"kernel config fp64 {cfg} fp32 {cfg32}")
    xs_host = W.uniform_vectors(1, napp, N)
    xs = torch.from_numpy(xs_host).to(dev)
    del xs_host
    ys = torch.empty_like(xs)
    pstar = torch.from_numpy(W.sine_field(m)).to(dev)
    pstar[torch.from_numpy(m.boundary_mask()).to(dev)] = 0.0
    b = probs[0].apply(pstar)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)

    def step():
        t_apply = timed_applies(torch, probs, xs, ys, napp, stream)
        t0 = time.perf_counter()
        p64, i64 = probs[0].cg_solve(b, rtol=1e-8)
        t_cg64 = time.perf_counter() - t0
        t0 = time.perf_counter()
        pmx, imx = probs[0].cg_solve(b, rtol=1e-8, precision="mixed", inner_rtol=1e-2)
        t_cgmx = time.perf_counter() - t0
        return t_apply, t_cg64, i64, p64, t_cgmx, imx, pmx

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    t_apply = sum(r[0] for r in res)
    value = N * napp * args.steps / t_apply / 1e6
    per_apply = t_apply / (napp * args.steps)
    achieved = BYTES_PER_DOF_F64 * N / per_apply / 1e9
    last = res[-1]
    err64 = float(torch.linalg.norm(last[3] - pstar) / torch.linalg.norm(pstar))
    errmx = float(torch.linalg.norm(last[6] - pstar) / torch.linalg.norm(pstar))
    t_graph, graph_diff = graph_applies(torch, probs, xs, ys, napp, dev)
    traffic = measured_traffic(cfg)
    sec = {}
    if not args.no_secondary:
        log("secondary figures")
        sec = secondary(torch, vpp, W, dev, cache, xs, ys, probs)
    out = {
        "metric": "operator MDoF/s + CG time to rtol 1e-8, FP64 vs FP32-mixed, Q2/Q3 hex",
        "value": value,
        "unit": "MDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "droplet 64^3 cells Q2, rho 1000/1, eps=2h, 100 applies + FP64 and mixed PCG to 1e-8",
                   "ndofs": N, "applies_per_step": napp, "kernel_fp64": cfg, "kernel_fp32": cfg32},
        "apply_us": per_apply * 1e6,
        "cg_fp64_s": float(np.median([r[1] for r in res])),
        "cg_fp64_iters": last[2]["iterations"],
        "cg_fp64_true_rel_res": last[2]["true_rel_residual"],
        "cg_fp64_err_vs_exact": err64,
        "cg_mixed_s": float(np.median([r[4] for r in res])),
        "cg_mixed_fp32_iters": last[5]["iterations"],
        "cg_mixed_replacements": last[5]["outer_iterations"],
        "cg_mixed_true_rel_res": last[5]["true_rel_residual"],
        "cg_mixed_err_vs_exact": errmx,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic / per_apply / 1e9,
                     "kernel": "FP64 Q2 apply = tile kernel + shared-node assembly (2 launches)"},
    }
    if traffic is not None:
        out["roofline"]["traffic_bytes_per_apply"] = traffic
    out["apply_us_graph"] = t_graph * 1e6
    out["mdofs_graph"] = N / t_graph / 1e6
    out["graph_max_rel_diff_vs_eager"] = graph_diff
    it64 = max(out["cg_fp64_iters"], 1)
    t_it = out["cg_fp64_s"] / it64
    out["cg_fp64_us_per_iter"] = t_it * 1e6
    out["cg_fp64_bytes_per_dof_iter"] = CG_BYTES_PER_DOF_ITER_F64
    out["cg_fp64_effective_gbs"] = CG_BYTES_PER_DOF_ITER_F64 * N / t_it / 1e9
    out["cg_mixed_us_per_fp32_iter"] = out["cg_mixed_s"] / max(out["cg_mixed_fp32_iters"], 1) * 1e6
    ncells = m.ncells[0] * m.ncells[1] * m.ncells[2]
    tflops = FLOPS_PER_CELL_Q2 * ncells / per_apply / 1e12
    out["valu"] = {"achieved": tflops, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": tflops / FP64_VALU_PEAK_TFLOPS, "flops_per_apply": FLOPS_PER_CELL_Q2 * ncells}
    out.update(sec)
    if args.copy_probe:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        c = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 3 x copy of 512 MiB")
    if args.extras:
        log("extras")
        out["extras"] = extras(torch, vpp, W, dev, cache)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
