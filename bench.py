"""Benchmark of the explicit LES momentum-residual assembly on one MI355X.

A step is one assembly (gather, element residual, scatter) of the 2.0 M-element
hybrid FP64 workload: a z-graded, 10 %-perturbed box of 95 x 95 x 94 cells split
into TET04 / PEN06 / PYR05 / HEX08 (40 / 40 / 5 / 15 %), divergence-free random
Fourier velocity, smooth pressure, nu = 1.5e-5, Vreman c = 0.1.  Inputs are
resident in HBM before the timed region.  Prints one JSON line.
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

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (256 CU x 2.4 GHz x 128)
FP32_VECTOR_PEAK_TFLOPS = 157.3


def flops_per_element(t: int, n_gauss: int) -> int:
    """Algorithmic flops of one element as the kernel computes it (FMA = 2).

    Per Gauss point with n nodes (node 0 is the local origin, so its terms
    vanish): J, reference gradients of u and p, and u_g cost 24 (n-1) FMA;
    adjugate and det 32; G and grad p 72; Vreman 46 (sqrt and divide as 1);
    strain, divergence, EMAC term, f and weights 41; T = w (nu+nu_t) S adj^T 54;
    the residual update 8 per node and component (24 n).  Total 72 n + 198.
    """
    n = t
    return n_gauss * (72 * n + 198)


GAUSS = {4: 4, 5: 8, 6: 6, 8: 8}
SLOT = {4: "tet04", 5: "pyr05", 6: "pen06", 8: "hex08"}


def algorithmic_bytes(mesh, n_field: int, with_p: bool) -> dict:
    """Bytes one assembly must move with ideal reuse: connectivity once, each
    geometry node (24 B), field node (u 24 B, p 8 B, rhs written 24 B) and the
    per-element filter width (8 B) once."""
    conn = 4 * int(mesh.conn.size) * (2 if mesh.field_node is not None else 1)
    nodes = 24 * mesh.n_nodes + n_field * (24 + (8 if with_p else 0) + 24)
    return {"conn": conn, "nodes": nodes, "delta": 8 * mesh.n_elems, "total": conn + nodes + 8 * mesh.n_elems}


def cpu_baseline(case, target_s: float = 12.0) -> dict:
    """The FP64 oracle, single thread, on a stride sample of the same elements
    (same type mix), sized to about target_s seconds of CPU work."""
    import oracle
    from paper_2005_05899_amd import meshgen as mg
    m = case.mesh

    def sub(stride):
        idx = np.arange(0, m.n_elems, stride)
        lens = np.diff(m.conn_offsets)[idx]
        offs = np.zeros(len(idx) + 1, np.int64)
        np.cumsum(lens, out=offs[1:])
        conn = np.concatenate([m.conn[m.conn_offsets[e]:m.conn_offsets[e + 1]] for e in idx])
        return mg.Mesh(m.coords, m.types[idx], offs, conn, m.field_node, m.n_field_nodes)

    probe = sub(max(1, m.n_elems // 20000))
    t0 = time.perf_counter()
    oracle.assemble(probe, case.u, case.p, case.nu, case.vreman_c)
    rate = probe.n_elems / (time.perf_counter() - t0)
    stride = max(1, int(m.n_elems / (rate * target_s)))
    sample = sub(stride)
    t0 = time.perf_counter()
    oracle.assemble(sample, case.u, case.p, case.nu, case.vreman_c)
    dt = time.perf_counter() - t0
    return {"value": sample.n_elems / dt, "unit": "element-assemblies/s", "cores": 1, "kind": "oracle",
            "sample": f"every {stride}-th element of the same mesh ({sample.n_elems} elements, same type mix), "
                      f"one single-thread FP64 assembly, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--scatter", choices=["staged", "chunk_atomic", "colour", "direct"], default="staged")
    ap.add_argument("--chunk", type=int, default=None, help="elements per chunk (chunked scatter)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the assembly of one mesh partition is the single-GPU unit of work)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_05899_amd import lesasm, meshgen
    torch.cuda.set_device(0)

    case = meshgen.hybrid_2m_case()
    m = case.mesh
    mesh = lesasm.Mesh.from_arrays(m, case.vreman_c, scatter=args.scatter)
    mesh.precision = args.precision
    if args.chunk:
        mesh.set_option(lesasm.OPT_CHUNK, args.chunk)
    u = mesh.to_internal(torch.from_numpy(case.u).cuda())
    p = mesh.to_internal(torch.from_numpy(case.p).cuda())
    rhs = torch.empty_like(u)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        mesh.assemble_momentum_rhs(u, p, case.nu, out=rhs)
    torch.cuda.synchronize()
    mesh.set_option(lesasm.OPT_PROFILE, 1)
    mesh.kernel_times(reset=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mesh.assemble_momentum_rhs(u, p, case.nu, out=rhs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = mesh.kernel_times(reset=True)
    mesh.set_option(lesasm.OPT_PROFILE, 0)

    E = m.n_elems
    value = E * args.steps / elapsed
    flops = {t: flops_per_element(t, GAUSS[t]) * mesh.n_per_type[t] for t in GAUSS}
    per_kernel = {}
    for t, slot in SLOT.items():
        ms, n = kt[slot]
        if n:
            avg = ms / n
            per_kernel[slot] = {"avg_ms": avg, "elements": mesh.n_per_type[t],
                                "tflops": flops[t] / (avg * 1e-3) / 1e12}
    dominant = max(per_kernel, key=lambda k: per_kernel[k]["avg_ms"])
    dk = per_kernel[dominant]
    peak = FP64_VECTOR_PEAK_TFLOPS if args.precision == "fp64" else FP32_VECTOR_PEAK_TFLOPS
    ab = algorithmic_bytes(m, m.n_field_nodes, True)
    kernel_ms_total = sum(v[0] for v in kt.values()) / args.steps
    out = {
        "metric": "element-assemblies/s + % HBM peak; mixed/learned vs FP64 at stated error",
        "value": value,
        "unit": "element-assemblies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-contract/f64-accumulate",
        "data": "synthetic",
        "config": {"workload": "hybrid box 2.0M elements (TET04/PEN06/PYR05/HEX08 40/40/5/15 %), FP64, "
                               f"{args.scatter} scatter",
                   "elements": E, "field_nodes": m.n_field_nodes, "per_type": {SLOT[t]: mesh.n_per_type[t] for t in SLOT},
                   "nu": case.nu, "vreman_c": case.vreman_c, "seeds": case.meta},
        "roofline": {"bound": "alu", "kernel": f"k_assemble<{dominant}>", "achieved": dk["tflops"], "peak": peak,
                     "unit": "TFLOP/s", "frac": dk["tflops"] / peak, "traffic": None},
        "hbm": {"algorithmic_bytes": ab["total"], "achieved_GBs": ab["total"] / (1e-3 * kernel_ms_total) / 1e9,
                "frac_of_peak": ab["total"] / (1e-3 * kernel_ms_total) / 1e9 / HBM_PEAK_GBS},
        "kernels": per_kernel,
        "assembly_tflops": sum(flops.values()) / (1e-3 * kernel_ms_total) / 1e12,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)
    mesh.close()


if __name__ == "__main__":
    main()
