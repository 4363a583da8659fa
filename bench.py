#!/usr/bin/env python3
"""Benchmark of the hot path: energy + gradient + clamped block-CSR Hessian of
the elastic-shell objective (StVK membrane per triangle + dihedral bending per
interior-edge diamond) on a 1024 x 1024-vertex grid rolled into a half
cylinder with small Gaussian noise (2,093,058 triangles, 3,137,541 diamonds,
13,606,924 3x3 blocks), FP32 derivative arithmetic, FP64 energy.

One step = one mad_problem_eval(ENERGY | GRAD | HESS | SPD) over the whole
mesh with inputs resident in HBM (topology, patches and pattern are built
once, outside the timed region). Prints one JSON line.

  python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--precision f32|f64]
                  [--n 1024] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 flops per element of the clamped-Hessian element algorithm (counted: see the design doc)
FLOPS_PER_ELEM = {"stvk": 6.0e3, "bending": 2.6e4}

# MI355X published peaks used as roofline denominators
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3
FP64_VALU_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32")
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--patch-faces", type=int, default=0)
    ap.add_argument("--scatter", choices=["patch", "atomic"], default="patch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=80, help="grid rows of the oracle timing sample")
    return ap.parse_args()


def alg_bytes(prob_info, precision_bytes):
    """Algorithmic HBM bytes of one step (read inputs once, write outputs once)."""
    nv, nt, nd, nnzb = prob_info
    rd = nv * 3 * 8 + nt * 3 * 4 + nd * 4 * 4 + nt * 5 * 8 + nd * 2 * 8 + (nv + 1) * 4 + nnzb * 4
    wr = nv * 3 * precision_bytes + nnzb * 9 * precision_bytes + 8
    return rd + wr


def cpu_baseline(args, terms):
    """The FP64 oracle timed on a bounded strip of the same workload (first rows of the grid)."""
    import numpy as np
    from oracle import oracle as O
    from paper_2509_00406_amd import meshgen
    full = meshgen.shell_cylinder(n=args.n, seed=2001)
    n = args.n
    rows = min(args.cpu_rows, n)
    nv = rows * n
    sel = np.all(full.tris < nv, axis=1)
    P = O.Problem(full.tris[sel], full.rest[:nv], nv, 3)
    for k, prm in terms:
        P.add_term(k, prm)
    P.build_pattern()
    n_el = int(sel.sum()) + P.topo.diamonds.shape[0]
    t0 = time.perf_counter()
    P.eval(full.x[:nv], O.ENERGY | O.GRAD | O.HESS | O.SPD, scales=False)
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n_el / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"first {rows} of {n} grid rows of the same shell: {n_el} elements "
                      f"(StVK triangles + bending diamonds), energy+grad+clamped Hessian+assembly, "
                      f"FP64, serial, {dt:.1f} s on {cpu}; host nproc {os.cpu_count()}"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2509_00406_amd import mad, meshgen

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    prec = mad.F32 if args.precision == "f32" else mad.F64
    pb = 4 if prec == mad.F32 else 8
    inp = meshgen.shell_cylinder(n=args.n, seed=2001)
    terms = [(mad.STVK, (1.0, 1.0)), (mad.BENDING, (1.0, 1.0))]
    t0 = time.perf_counter()
    mesh = mad.Mesh(inp.tris, inp.n_verts)
    scatter = mad.SCATTER_PATCH if args.scatter == "patch" else mad.SCATTER_ATOMIC
    prob = mad.Problem(mesh, 3, prec, patch_faces=args.patch_faces, scatter=scatter)
    for k, prm in terms:
        prob.add_term(k, prm, inp.rest)
    stream = torch.cuda.current_stream()
    prob.finalize(stream)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    x = torch.from_numpy(inp.x.ravel().copy()).cuda()
    out = prob.outputs()
    mode = mad.ENERGY | mad.GRAD | mad.HESS | mad.SPD
    n_elem = mesh.n_tris + mesh.n_diamonds

    for _ in range(args.warmup):
        prob.eval(x, mode, out=out, stream=stream)
    torch.cuda.synchronize()
    mad.mad_problem_set_profiling(prob.handle, True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        prob.eval(x, mode, out=out, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mad.mad_problem_set_profiling(prob.handle, False)
    stage_ms, n_evals = mad.mad_problem_profile(prob.handle)
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = max(wall * 1e3, gpu_ms) / args.steps
    nonfinite, fallbacks = prob.status()

    term_ms = stage_ms[1:1 + len(terms)]
    if args.scatter == "patch":
        # one fused kernel evaluates both terms of every patch
        dom_name = "k_eval_patch (StVK + bending fused)"
        dom_ms = term_ms[0] / n_evals
        flops = FLOPS_PER_ELEM["stvk"] * mesh.n_tris + FLOPS_PER_ELEM["bending"] * mesh.n_diamonds
    else:
        dom = int(np.argmax(term_ms))
        dom_ms = term_ms[dom] / n_evals
        dom_name = ["k_eval<StVK>", "k_eval<bending>"][dom]
        flops = FLOPS_PER_ELEM["stvk"] * mesh.n_tris if dom == 0 else FLOPS_PER_ELEM["bending"] * mesh.n_diamonds
    achieved_tf = flops / (dom_ms * 1e-3) / 1e12
    peak = FP32_VALU_PEAK_TFLOPS if prec == mad.F32 else FP64_VALU_PEAK_TFLOPS
    step_bytes = alg_bytes((mesh.n_verts, mesh.n_tris, mesh.n_diamonds, prob.nnzb), pb)

    res = {
        "metric": "elements/s for energy+grad+sparse Hessian assembly",
        "value": n_elem / (ms_per_step * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"elastic shell StVK+bending, {args.n}x{args.n} grid cylinder, sigma=1e-3h, "
                               f"clamped Hessians, block-CSR 3x3",
                   "triangles": mesh.n_tris, "diamonds": mesh.n_diamonds, "elements": n_elem,
                   "nnzb": prob.nnzb, "precision": args.precision, "scatter": args.scatter,
                   "patches_faces": args.patch_faces or 512},
        "roofline": {"bound": "alu", "kernel": dom_name, "achieved": achieved_tf, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved_tf / peak, "traffic": None,
                     "kernel_ms": dom_ms},
        "hbm": {"alg_bytes_per_step": step_bytes, "alg_GBs": step_bytes / (ms_per_step * 1e-3) / 1e9,
                "frac_of_8TBs": step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "stages_ms_per_step": {"fill": stage_ms[0] / n_evals,
                               **({"fused": term_ms[0] / n_evals, "gather_and_fp64_redo": term_ms[1] / n_evals}
                                  if args.scatter == "patch" else
                                  {["stvk", "bending"][i]: term_ms[i] / n_evals for i in range(len(terms))}),
                               "energy": stage_ms[-1] / n_evals},
        "setup_s": setup_s,
        "fp64_fallbacks": fallbacks,
        "nonfinite": nonfinite,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(args, [(4, (1.0, 1.0)), (5, (1.0, 1.0))])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
