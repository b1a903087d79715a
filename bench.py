"""Benchmark of the explicit LES momentum-residual assembly on one MI355X.

A step is one assembly (gather, element residual, scatter) of the 20.0 M-element
hybrid FP64 workload: a z-graded, 10 %-perturbed box of 205 x 205 cells in the
plane split into TET04 / PEN06 / PYR05 / HEX08 layers (40 / 40 / 5 / 15 % of the
elements), divergence-free random Fourier velocity, smooth pressure,
nu = 1.5e-5, Vreman c = 0.1.  Inputs are resident in HBM before the timed
region.  Prints one JSON line.

Beside the FP64 value the line carries the mixed-precision form (FP32 element
contractions) and, if trained weights are present, the learned closure, each
with its error against the FP64 CPU oracle on the same inputs, and the 2.0 M
mesh of the same generator as a sub-record.  Other modes: --workload batch64
(64 partitions, about 25 M elements, persistent launch), tet20m (20.25 M TET04),
precision20m (FP32 contractions and a full time step in both precisions),
cg20m, partition20m, balance8, copy (the counter calibration).
"""
from __future__ import annotations

import argparse
import ctypes
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (256 CU x 2.4 GHz x 128 flop/clk)
FP32_VECTOR_PEAK_TFLOPS = 157.3
BF16_MATRIX_PEAK_TFLOPS = 2500.0  # dense
# the learned closure's network per Gauss point: 2 (10 x 64 + 64 x 64 + 64 x 6)
MLP_FLOPS_PER_POINT = 2 * (10 * 64 + 64 * 64 + 64 * 6)

# Algorithmic FP64 flops per element of the residual (per Gauss point about
# 90 n + 175 for n nodes; the affine TET04 evaluates its geometry once):
FLOPS_PER_ELEMENT = {4: 1000, 5: 5000, 6: 4300, 8: 7200}
GAUSS = {4: 4, 5: 8, 6: 6, 8: 8}
SLOT = {4: "tet04", 5: "pyr05", 6: "pen06", 8: "hex08"}
WEIGHTS = os.path.join(ROOT, "paper_2005_05899_amd", "data", "closure_weights.npy")
WEIGHTS_META = os.path.join(ROOT, "paper_2005_05899_amd", "data", "closure_weights.json")


# Sources each kernel is built from: counter summaries are valid for these only.
# (The C header is left out: it holds the ABI and comments; the kernels use
# only its fixed element-type codes.)  The mesh code is part of the assembly's
# set because it cuts the chunks, which fixes the staging rows' traffic.
ASSEMBLY_SOURCES = ("csrc/assemble.hip", "csrc/element.hpp", "csrc/modal.hpp", "csrc/refelem.hpp", "csrc/mlp.hpp",
                    "csrc/common.hpp", "csrc/mesh.hip")
PARTITION_SOURCES = ("csrc/partition.hip", "csrc/common.hpp")
CG_SOURCES = ("csrc/stepper.hip", "csrc/common.hpp")


def source_hash(files=ASSEMBLY_SOURCES) -> str:
    """Hash of a kernel's code (comments and whitespace removed): counter
    summaries are valid for this hash only."""
    import re
    h = hashlib.sha256()
    for f in files:
        text = open(os.path.join(ROOT, "paper_2005_05899_amd", f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def algorithmic_bytes(mesh, with_p: bool) -> int:
    """Bytes one assembly must move with ideal reuse: connectivity once (4 B per
    element node), each geometry node (24 B), each field node (u 24 B, p 8 B,
    rhs written 24 B) and the per-element filter width (8 B)."""
    n_field = mesh.n_field_nodes
    conn = 4 * int(mesh.conn.size) * (2 if mesh.field_node is not None else 1)
    nodes = 24 * mesh.n_nodes + n_field * (24 + (8 if with_p else 0) + 24)
    return conn + nodes + 8 * mesh.n_elems


def per_type_bytes(mesh, t: int) -> float:
    """Algorithmic bytes of the elements of one type: its connectivity, its
    share of the node traffic (by element-node incidences) and its widths."""
    ne_t = int((mesh.types == t).sum())
    inc_t = ne_t * t
    total = algorithmic_bytes(mesh, True)
    conn_all = 4 * int(mesh.conn.size)
    nodes = total - conn_all - 8 * mesh.n_elems
    return 4 * inc_t + nodes * inc_t / max(1, int(mesh.conn.size)) + 8 * ne_t


def field_errors(got, ref) -> dict:
    """Per component relative L2 and max errors (absolute ones where the
    reference component is identically zero)."""
    out = {}
    for i, name in enumerate("xyz"):
        d = got[:, i] - ref[:, i]
        nr, mr = np.linalg.norm(ref[:, i]), np.abs(ref[:, i]).max()
        if nr > 0:
            out[f"u{name}"] = {"rel_l2": float(np.linalg.norm(d) / nr), "rel_max": float(np.abs(d).max() / mr)}
        else:
            out[f"u{name}"] = {"abs_l2": float(np.linalg.norm(d)), "abs_max": float(np.abs(d).max())}
    return out


def time_assembly(torch, mesh, u, p, nu, steps, warmup, concurrent=True):
    """Wall time of `steps` assemblies between two synchronisations after
    `warmup` untimed ones (no instrumentation).  concurrent=False runs the
    element-type kernels one after another."""
    from paper_2005_05899_amd import lesasm
    mesh.set_option(lesasm.OPT_CONCURRENT, 1 if concurrent else 0)
    rhs = torch.empty_like(u)
    for _ in range(warmup):
        mesh.assemble_momentum_rhs(u, p, nu, out=rhs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mesh.assemble_momentum_rhs(u, p, nu, out=rhs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mesh.set_option(lesasm.OPT_CONCURRENT, 1)
    return elapsed, None, rhs


def time_graph_replay(torch, mesh, u, p, nu, steps, warmup) -> float:
    """Seconds for `steps` replays of one assembly captured in a HIP graph
    (the same launches: fork to the side streams, element kernels, join,
    gather), on a stream of its own."""
    s = torch.cuda.Stream()
    rhs = torch.empty_like(u)
    with torch.cuda.stream(s):
        mesh.assemble_momentum_rhs(u, p, nu, out=rhs)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        mesh.assemble_momentum_rhs(u, p, nu, out=rhs)
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    del g
    return el


def time_wall(torch, mesh, m, case, u, steps) -> dict:
    """The boundary assembly of the wall model (wall z = 0): time per call and
    error against the oracle."""
    import oracle
    from paper_2005_05899_amd import meshgen
    faces = meshgen.wall_faces(m)
    mesh.set_wall(*faces)
    out = torch.zeros_like(u)
    for _ in range(3):
        mesh.assemble_wall(u, case.nu, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mesh.assemble_wall(u, case.nu, out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out.zero_()
    mesh.assemble_wall(u, case.nu, out)
    ref, *_ = oracle.wall_assemble(m, case.u, case.nu, *faces)
    got = mesh.to_user(out).cpu().numpy()
    mesh.set_wall(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int64))
    return {"faces": int(len(faces[2])), "ms_per_call": 1e3 * el / steps,
            "error_vs_oracle": field_errors(got, ref)}


def fallback_fraction(mesh, u, p, nu) -> dict:
    """Fraction of elements that kept Vreman's stress in one assembly, in all
    and per element type (per-type counters of the library)."""
    from paper_2005_05899_amd import lesasm
    lesasm.closure_fallbacks_by_type(mesh)  # resets the counters
    mesh.assemble_momentum_rhs(u, p, nu)
    by_type = lesasm.closure_fallbacks_by_type(mesh)
    out = {"all": sum(by_type.values()) / mesh.n_elems}
    for t, slot in SLOT.items():
        if mesh.n_per_type[t]:
            out[slot] = by_type[t] / mesh.n_per_type[t]
    return out


def host_cpu() -> dict:
    """Model, sockets, physical and logical cores of the host (from
    /proc/cpuinfo) and the CPUs this process may run on."""
    model, sockets, cores = None, set(), set()
    phys = None
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name" and model is None:
                model = v
            elif k == "physical id":
                phys = v
                sockets.add(v)
            elif k == "core id":
                cores.add((phys, v))
    except OSError:
        pass
    return {"model": model, "sockets": len(sockets) or None, "physical_cores": len(cores) or None,
            "logical_cpus": os.cpu_count(), "cpus_allowed": len(os.sched_getaffinity(0))}


def child_processes() -> list:
    """Processes this one started that are still alive (the benchmark starts
    none: the oracle's timing leg runs as OpenMP threads in this process)."""
    try:
        import psutil
    except ImportError:
        return []
    return [{"pid": c.pid, "name": c.name()} for c in psutil.Process().children(recursive=True)]


def baseline_threads() -> int:
    """Threads for the all-core oracle leg: OMP_NUM_THREADS if set (the CPU
    share of this process), else every CPU it may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    return int(env) if env.isdigit() and int(env) > 0 else len(os.sched_getaffinity(0))


def cpu_baseline(case, single_thread_s=None, min_cpu_seconds: float = 20.0, max_reps: int = 5) -> dict:
    """The FP64 oracle on the host cores: the whole workload assembled by the
    oracle's threaded leg (the plain element loop over contiguous element
    ranges, one OpenMP thread per core of this process's CPU share), repeated
    until about min_cpu_seconds of CPU time; median rate.  single_thread_s, if
    given, is the time of one plain single-thread oracle assembly of the same
    workload (reported beside it)."""
    import oracle
    threads = baseline_threads()
    rates, wall, reps = [], 0.0, 0
    while (wall * threads < min_cpu_seconds or reps < 2) and reps < max_reps:
        t0 = time.perf_counter()
        oracle.assemble_threads(case.mesh, case.u, case.p, case.nu, case.vreman_c, threads=threads)
        dt = time.perf_counter() - t0
        rates.append(case.mesh.n_elems / dt)
        wall += dt
        reps += 1
    out = {"value": float(np.median(rates)), "unit": "element-assemblies/s", "cores": threads, "kind": "oracle",
           "sample": f"the whole {case.mesh.n_elems}-element workload, {reps} FP64 oracle assemblies on {threads} "
                     f"threads ({wall:.1f} s wall, about {wall * threads:.0f} s of CPU time), median rate",
           "host": host_cpu()}
    if single_thread_s:
        out["single_thread"] = {"value": case.mesh.n_elems / single_thread_s, "seconds": single_thread_s,
                                "sample": "one plain single-thread oracle assembly of the whole workload"}
    return out


def traffic_from_profiles(slot: str, workload: str = "hybrid2m", kernel: str = "k_assemble",
                          files=ASSEMBLY_SOURCES):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{slot}_{workload}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != source_hash(files):
        return None
    return d


WORKLOADS = {
    "hybrid20m": ("hybrid box, 20.0M elements (205 x 205 cells; TET04/PEN06/PYR05/HEX08 = 40/40/5/15 %)",
                  "hybrid_20m_case"),
    "hybrid2m": ("hybrid box, 2.0M elements (95 x 95 cells; TET04/PEN06/PYR05/HEX08 = 40/40/5/15 %)",
                 "hybrid_2m_case"),
    "tet20m": ("all-TET04 box, 20.25M elements (150^3 cells x 6)", None),
}


def make_case(workload: str):
    from paper_2005_05899_amd import meshgen
    if workload == "tet20m":
        return meshgen.tet_case(150)
    return getattr(meshgen, WORKLOADS[workload][1])()


def kernel_table(mesh, m, kt, peak) -> dict:
    """Per element-type kernel: average event duration, algorithmic TFLOP/s
    and GB/s; staged-row gather and zero-fill per assembly."""
    table = {}
    for t, slot in SLOT.items():
        ms, n = kt[slot]
        if n:
            avg = ms / n
            fl = FLOPS_PER_ELEMENT[t] * mesh.n_per_type[t]
            table[slot] = {"avg_ms": avg, "launches": n, "elements": mesh.n_per_type[t],
                           "algorithmic_tflops": fl / (avg * 1e-3) / 1e12,
                           "frac_of_peak": fl / (avg * 1e-3) / 1e12 / peak,
                           "algorithmic_GBs": per_type_bytes(m, t) / (avg * 1e-3) / 1e9}
    n_asm = max(kt[slot][1] for slot in SLOT.values())
    for extra in ("gather", "fill"):  # summed per assembly (the gather is one launch per node class)
        ms, n = kt[extra]
        if n:
            table[extra] = {"ms_per_assembly": ms / n_asm, "launches_per_assembly": n / n_asm,
                            "avg_ms_per_launch": ms / n}
    return table


WARM_SECONDS = 0.3


def profile_kernels(torch, mesh, u, p, nu, steps, concurrent):
    """Per-kernel HIP-event durations of `steps` assemblies, recorded by the
    library on the stream each kernel is launched on.  concurrent=False runs
    the element-type kernels one after another (isolated durations)."""
    from paper_2005_05899_amd import lesasm
    rhs = torch.empty_like(u)
    mesh.set_option(lesasm.OPT_CONCURRENT, 1 if concurrent else 0)
    # uninstrumented assemblies for at least WARM_SECONDS first, so that the
    # clocks have settled before the first recorded launch
    t0 = time.perf_counter()
    while True:
        for _ in range(4):
            mesh.assemble_momentum_rhs(u, p, nu, out=rhs)
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= WARM_SECONDS:
            break
    mesh.set_option(lesasm.OPT_PROFILE, 1)
    mesh.kernel_times(reset=True)
    for _ in range(steps):
        mesh.assemble_momentum_rhs(u, p, nu, out=rhs)
    torch.cuda.synchronize()
    kt = mesh.kernel_times(reset=True)
    mesh.set_option(lesasm.OPT_PROFILE, 0)
    mesh.set_option(lesasm.OPT_CONCURRENT, 1)
    return kt


def closure_delta_ref(mesh, meta: dict) -> float:
    """Width reference handed to the learned closure: the mesh's geometric
    mean Delta_e when the network was trained with that rule (recorded in its
    metadata), else the fixed reference the metadata holds."""
    from paper_2005_05899_amd import training
    if meta.get("delta_ref_rule"):
        return training.mesh_delta_ref(mesh)
    return meta.get("delta_ref", 0.1)


def closure_variants(torch, args, mesh, m, case, u, p, elapsed, ref, precisions=("fp32", "fp64")) -> dict:
    """The fused learned closure (committed network, 5 % fallback rule) in the
    given contraction precisions: rate, speed against plain FP64 Vreman,
    network rate on the matrix cores, fallback fraction per type, difference
    from the FP64 Vreman oracle."""
    from paper_2005_05899_amd import lesasm
    vr = {}
    if not os.path.exists(WEIGHTS):
        return vr
    E = m.n_elems
    params = np.load(WEIGHTS)
    meta = json.load(open(WEIGHTS_META)) if os.path.exists(WEIGHTS_META) else {}
    net = lesasm.MLP(params)
    dref = closure_delta_ref(mesh, meta)
    for prec in precisions:
        mesh.precision = prec
        lesasm.set_closure(mesh, net, dref, 0.05)
        el, _, rl = time_assembly(torch, mesh, u, p, case.nu, args.steps, args.warmup)
        npts = sum(int((m.types == t).sum()) * GAUSS[t] for t in GAUSS)
        mfma_tf = npts * MLP_FLOPS_PER_POINT * args.steps / el / 1e12
        vr[f"learned_closure_{prec}"] = {
            "value": E * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
            "speedup_vs_fp64_vreman": elapsed / el, "delta_ref": dref,
            "network_bf16_tflops": mfma_tf, "network_frac_of_bf16_peak": mfma_tf / BF16_MATRIX_PEAK_TFLOPS,
            "fallback_fraction": fallback_fraction(mesh, u, p, case.nu),
            "difference_vs_fp64_vreman_oracle": None if ref is None else
            field_errors(mesh.to_user(rl).cpu().numpy(), ref)}
        lesasm.set_closure(mesh, None)
    net.close()
    mesh.precision = args.precision
    return vr


def measure_workload(torch, args, workload, case, variants: bool, oracle_errors: bool, closure: bool = False):
    """One workload: per-kernel isolated durations, graph replay, then the
    timed region (W warm-up assemblies, K timed ones between two
    synchronisations, no instrumentation), then the concurrent per-kernel
    durations; optionally the errors against the plain oracle on every node,
    the FP32 and learned-closure variants and the wall model."""
    from paper_2005_05899_amd import lesasm
    m = case.mesh
    mesh = lesasm.Mesh.from_arrays(m, case.vreman_c, scatter=args.scatter)
    mesh.precision = args.precision
    if args.chunk is not None:
        mesh.set_option(lesasm.OPT_CHUNK, args.chunk)
    u = mesh.to_internal(torch.from_numpy(case.u).cuda())
    p = mesh.to_internal(torch.from_numpy(case.p).cuda())
    torch.cuda.synchronize()
    peak = FP64_VECTOR_PEAK_TFLOPS if args.precision == "fp64" else FP32_VECTOR_PEAK_TFLOPS
    E = m.n_elems

    # isolated kernel durations for the roofline, then the caller-captured graph
    # (measurements of their own that precede the timed region)
    kt = profile_kernels(torch, mesh, u, p, case.nu, args.steps, concurrent=False)
    el_graph = None if args.isolated else time_graph_replay(torch, mesh, u, p, case.nu, args.steps, args.warmup)
    # the timed region
    elapsed, _, rhs = time_assembly(torch, mesh, u, p, case.nu, args.steps, args.warmup,
                                    concurrent=not args.isolated)
    kt_conc = profile_kernels(torch, mesh, u, p, case.nu, args.steps, concurrent=not args.isolated)

    per_kernel = kernel_table(mesh, m, kt, peak)
    dominant = max((k for k in per_kernel if k in SLOT.values()), key=lambda k: per_kernel[k]["avg_ms"])
    dk = per_kernel[dominant]
    ab = algorithmic_bytes(m, True)
    step_s = elapsed / args.steps
    total_flops = sum(FLOPS_PER_ELEMENT[t] * mesh.n_per_type[t] for t in SLOT)
    # counter summaries exist per precision for the staged scatter only (other
    # scatters and precisions run other kernels)
    traffic = None if args.scatter != "staged" else \
        traffic_from_profiles(dominant, workload if args.precision == "fp64" else f"{workload}_{args.precision}")
    desc = WORKLOADS[workload][0]
    rec = {
        "value": E * args.steps / elapsed,
        "ms_per_step": 1e3 * step_s,
        "config": {"workload": f"{desc}, {args.precision}, {args.scatter} scatter",
                   "elements": E, "field_nodes": m.n_field_nodes,
                   "per_type": {SLOT[t]: mesh.n_per_type[t] for t in SLOT},
                   "nu": case.nu, "vreman_c": case.vreman_c, "seeds": case.meta},
        "roofline": {"bound": "alu", "kernel": f"k_assemble_chunk<{dominant}, {args.precision}> (isolated launches)",
                     "achieved": dk["algorithmic_tflops"], "peak": peak, "unit": "TFLOP/s",
                     "frac": dk["algorithmic_tflops"] / peak,
                     "traffic": None if traffic is None else traffic["bytes_per_launch"],
                     "algorithmic_flops_per_launch": FLOPS_PER_ELEMENT[[t for t in SLOT if SLOT[t] == dominant][0]]
                     * dk["elements"], "avg_ms": dk["avg_ms"]},
        "hbm": {"algorithmic_bytes_per_step": ab, "achieved_GBs": ab / step_s / 1e9,
                "frac_of_peak": ab / step_s / 1e9 / HBM_PEAK_GBS,
                "working_set_exceeds_infinity_cache": ab > 256e6},
        "assembly": {"algorithmic_tflops": total_flops / step_s / 1e12,
                     "frac_of_peak": total_flops / step_s / 1e12 / peak},
        "kernels_isolated": per_kernel,
        "kernels_concurrent": kernel_table(mesh, m, kt_conc, peak),
        "graph_replay": None if el_graph is None else {
            "value": E * args.steps / el_graph, "ms_per_step": 1e3 * el_graph / args.steps,
            "note": "the same assembly captured once in a HIP graph and replayed"},
    }
    t_oracle = None
    if oracle_errors:
        import oracle
        t1 = time.perf_counter()
        ref = oracle.assemble(m, case.u, case.p, case.nu, case.vreman_c)
        t_oracle = time.perf_counter() - t1
        print(f"  {workload}: oracle assembly {t_oracle:.1f} s", file=sys.stderr, flush=True)
        got64 = mesh.to_user(rhs).cpu().numpy()
        rec[f"{args.precision}_error_vs_oracle"] = field_errors(got64, ref)
        rec["error_nodes"] = f"every node ({m.n_field_nodes})"
    if variants:
        vr = {}
        mesh.precision = "fp32"
        el, _, r32 = time_assembly(torch, mesh, u, p, case.nu, args.steps, args.warmup)
        vr["fp32_contractions"] = {"value": E * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
                                   "speedup_vs_fp64": elapsed / el,
                                   "error_vs_fp64_oracle": field_errors(mesh.to_user(r32).cpu().numpy(), ref)}
        vr.update(closure_variants(torch, args, mesh, m, case, u, p, elapsed, ref))
        mesh.precision = args.precision
        rec["variants"] = vr
        rec["wall_model"] = time_wall(torch, mesh, m, case, u, args.steps)
    elif closure:
        rec["variants"] = closure_variants(torch, args, mesh, m, case, u, p, elapsed, ref if oracle_errors else None,
                                           precisions=("fp32",))
    mesh.close()
    return rec, t_oracle


def run_main(args):
    import torch
    torch.cuda.set_device(0)
    t0 = time.time()
    case = make_case(args.workload)
    print(f"  {args.workload}: {case.mesh.n_elems} elements generated ({time.time() - t0:.0f} s)",
          file=sys.stderr, flush=True)
    rec, t_oracle = measure_workload(torch, args, args.workload, case, args.variants, args.variants)
    out = {
        "metric": "element-assemblies/s + % HBM peak; mixed/learned vs FP64 at stated error",
        "value": rec.pop("value"),
        "unit": "element-assemblies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic (seeded hybrid mesh and random Fourier fields; the paper's airplane meshes are not used)",
        "config": rec.pop("config"),
        "roofline": rec.pop("roofline"),
    }
    out.update(rec)
    out["source_hash"] = source_hash()
    if args.workload == "hybrid20m" and args.variants:
        # the 2.0 M-element mesh of the same generator as a sub-record (FP64, same protocol)
        t1 = time.time()
        small = make_case("hybrid2m")
        sub, _ = measure_workload(torch, args, "hybrid2m", small, False, True, closure=True)
        sub.pop("kernels_concurrent")
        out["hybrid2m"] = sub
        print(f"  hybrid2m sub-record ({time.time() - t1:.0f} s)", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, t_oracle)
    out["child_processes_at_end"] = child_processes()
    print(json.dumps(out), flush=True)


def run_batch(args):
    """64 partitions, element counts log-uniform in [50k, 2M] (about 25 M
    elements), one persistent launch per assembly; autotuned; graph-captured
    three-stage Runge-Kutta update."""
    import torch
    from paper_2005_05899_amd import lesasm, meshgen
    torch.cuda.set_device(0)
    sizes = meshgen.partition_sizes(64, seed=6)
    meshes, us, ps, nus = [], [], [], []
    E = 0
    t0 = time.time()
    for i, e in enumerate(sizes):
        c = meshgen.hybrid_case(int(e), seed_mesh=6 + i, seed_u=100 + i, seed_p=200 + i, n_modes=64)
        mesh = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
        meshes.append(mesh)
        us.append(mesh.to_internal(torch.from_numpy(c.u).cuda()))
        ps.append(mesh.to_internal(torch.from_numpy(c.p).cuda()))
        nus.append(c.nu)
        E += c.mesh.n_elems
        print(f"  partition {i}: {c.mesh.n_elems} elements ({time.time() - t0:.0f} s)", file=sys.stderr, flush=True)
    b = lesasm.Batch(meshes)
    outs = [torch.empty_like(u) for u in us]
    for _ in range(100):  # settle the clocks before the tuner compares configurations
        b.assemble(us, ps, nus, outs)
    torch.cuda.synchronize()
    best = b.tune(us, ps, nus, outs, cache_path=None, reps=5)
    cfg = b.config()
    for _ in range(args.warmup):
        b.assemble(us, ps, nus, outs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        b.assemble(us, ps, nus, outs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    # the same work as one call per mesh, for comparison
    for _ in range(args.warmup):
        for mesh, u, p, nu, o in zip(meshes, us, ps, nus, outs):
            mesh.assemble_momentum_rhs(u, p, nu, out=o)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        for mesh, u, p, nu, o in zip(meshes, us, ps, nus, outs):
            mesh.assemble_momentum_rhs(u, p, nu, out=o)
    torch.cuda.synchronize()
    el_single = time.perf_counter() - t2
    # graph-captured three-stage step against the same sequence launched eagerly
    s = torch.cuda.Stream()
    uw = [u.clone() for u in us]
    torch.cuda.synchronize()
    b.rk3_graph(uw, ps, nus, 1e-4, s)
    b.rk3_launch(s)
    s.synchronize()
    t3 = time.perf_counter()
    for _ in range(args.steps):
        b.rk3_launch(s)
    s.synchronize()
    el_graph = time.perf_counter() - t3
    with torch.cuda.stream(s):
        t4 = time.perf_counter()
        for _ in range(args.steps):
            b.rk3_eager(uw, ps, nus, 1e-4)
        s.synchronize()
        el_eager = time.perf_counter() - t4
    out = {
        "metric": "element-assemblies/s (batched persistent launch)",
        "value": E * args.steps / el, "unit": "element-assemblies/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"64 hybrid partitions, {E} elements, log-uniform sizes in [50k, 2M]",
                   "tuned": cfg, "tune_best_ms": best},
        "per_mesh_launches": {"value": E * args.steps / el_single, "ms_per_step": 1e3 * el_single / args.steps},
        "rk3_step_graph_ms": 1e3 * el_graph / args.steps, "rk3_step_eager_ms": 1e3 * el_eager / args.steps,
    }
    print(json.dumps(out), flush=True)
    b.close()
    for mesh in meshes:
        mesh.close()


def run_precision(args):
    """The 20 M-element hybrid box (205 x 205 cells): FP64 and FP32-contraction
    assemblies, each against the FP64 oracle field by field; one full time step
    (three Runge-Kutta stages and the FP64 pressure projection) in both
    precisions; the learned closure if trained weights are present."""
    import torch
    import oracle
    from paper_2005_05899_amd import lesasm, meshgen
    torch.cuda.set_device(0)
    t0 = time.time()
    case = meshgen.hybrid_20m_case()
    m = case.mesh
    print(f"  20M case generated: {m.n_elems} elements ({time.time() - t0:.0f} s)", file=sys.stderr, flush=True)
    mesh = lesasm.Mesh.from_arrays(m, case.vreman_c)
    u = mesh.to_internal(torch.from_numpy(case.u).cuda())
    p = mesh.to_internal(torch.from_numpy(case.p).cuda())
    E = m.n_elems
    res = {}
    for prec in ("fp64", "fp32"):
        mesh.precision = prec
        el, kt, r = time_assembly(torch, mesh, u, p, case.nu, args.steps, args.warmup)
        res[prec] = {"value": E * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
                     "rhs": mesh.to_user(r).cpu().numpy()}
        print(f"  {prec}: {res[prec]['ms_per_step']:.3f} ms per assembly", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    ref = oracle.assemble(m, case.u, case.p, case.nu, case.vreman_c)
    t_oracle = time.perf_counter() - t1
    print(f"  oracle: {t_oracle:.1f} s", file=sys.stderr, flush=True)
    for prec in res:
        res[prec]["error_vs_fp64_oracle"] = field_errors(res[prec].pop("rhs"), ref)

    # one full step from the same state in both precisions
    dt = 1e-3
    step = {}
    for prec in ("fp64", "fp32"):
        mesh.precision = prec
        st = lesasm.Stepper(mesh, case.nu, dt, rtol=1e-10, maxit=20000)
        uu, pp = u.clone(), p.clone()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        st.step(uu, pp)
        torch.cuda.synchronize()
        it, rr = st.stats()
        step[prec] = {"ms": 1e3 * (time.perf_counter() - ts), "cg_iterations": it, "cg_relative_residual": rr,
                      "u": uu, "p": pp}
        st.close()
        print(f"  step {prec}: {step[prec]['ms']:.1f} ms, {it} CG iterations", file=sys.stderr, flush=True)
    # the same step (FP64) from the step graph: stages, divergence, the CG with
    # the eager step's iteration count plus a margin captured (iterations after
    # convergence return at once on the device), correction; one replay to warm
    # up, then one timed replay from the same state
    mesh.precision = "fp64"
    st = lesasm.Stepper(mesh, case.nu, dt, rtol=1e-10, maxit=20000)
    gs = torch.cuda.Stream()
    ug, pg = u.clone(), p.clone()
    torch.cuda.synchronize()
    tc = time.perf_counter()
    g = lesasm.StepGraph(st, ug, pg, step["fp64"]["cg_iterations"] + 64, gs)
    t_capture = time.perf_counter() - tc
    g.launch(gs)
    gs.synchronize()
    ug.copy_(u)
    pg.copy_(p)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    g.launch(gs)
    gs.synchronize()
    t_graph = time.perf_counter() - ts
    it_g, res_g, ok_g = g.stats()
    step["fp64_step_graph"] = {"ms": 1e3 * t_graph, "cg_iterations": it_g, "cg_relative_residual": res_g,
                               "converged": ok_g, "captured_cg_iterations": step["fp64"]["cg_iterations"] + 64,
                               "capture_and_instantiate_s": t_capture,
                               "velocity_vs_eager": field_errors(mesh.to_user(ug).cpu().numpy(),
                                                                 mesh.to_user(step["fp64"]["u"]).cpu().numpy())}
    print(f"  step graph fp64: {1e3 * t_graph:.1f} ms, {it_g} CG iterations", file=sys.stderr, flush=True)
    g.close()
    st.close()
    # the pressure CG alone: a fixed number of iterations on this mesh's Laplacian
    st = lesasm.Stepper(mesh, case.nu, dt, rtol=1e-30, maxit=300)
    b = lesasm.divergence(mesh, u)
    st.pressure_solve(b)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    st.pressure_solve(b)
    torch.cuda.synchronize()
    el_cg = time.perf_counter() - ts
    it_cg, _ = st.stats()
    nnz = ctypes.c_int64()
    lesasm.check(lesasm.load().lesasm_stepper_laplacian(st._h, None, None, None, ctypes.byref(nnz)))
    n_rows = m.n_field_nodes
    cg_bytes = cg_bytes_per_iteration(nnz.value, n_rows)
    ms_it = 1e3 * el_cg / it_cg
    step["pressure_cg"] = {"iterations": it_cg, "ms_per_iteration": ms_it, "rows": n_rows, "nonzeros": nnz.value,
                           "algorithmic_bytes_per_iteration": cg_bytes,
                           "achieved_GBs": cg_bytes / ms_it / 1e6, "frac_of_hbm": cg_bytes / ms_it / 1e6 / HBM_PEAK_GBS}
    st.close()
    du64 = mesh.to_user(step["fp64"]["u"] - u).cpu().numpy()
    du32 = mesh.to_user(step["fp32"]["u"] - u).cpu().numpy()
    u64 = mesh.to_user(step["fp64"]["u"]).cpu().numpy()
    u32 = mesh.to_user(step["fp32"]["u"]).cpu().numpy()
    for prec in ("fp64", "fp32"):
        del step[prec]["u"], step[prec]["p"]
    step_cmp = {"velocity_fp32_vs_fp64": field_errors(u32, u64),
                "increment_fp32_vs_fp64": field_errors(du32, du64), "dt": dt}

    variants = {}
    if os.path.exists(WEIGHTS):
        params = np.load(WEIGHTS)
        meta = json.load(open(WEIGHTS_META)) if os.path.exists(WEIGHTS_META) else {}
        net = lesasm.MLP(params)
        dref = closure_delta_ref(mesh, meta)
        for prec in ("fp32", "fp64"):
            mesh.precision = prec
            lesasm.set_closure(mesh, net, dref, 0.05)
            el, _, rl = time_assembly(torch, mesh, u, p, case.nu, args.steps, args.warmup)
            variants[f"learned_closure_{prec}"] = {
                "value": E * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
                "fallback_fraction": fallback_fraction(mesh, u, p, case.nu),
                "difference_vs_fp64_vreman_oracle": field_errors(mesh.to_user(rl).cpu().numpy(), ref)}
            lesasm.set_closure(mesh, None)
        net.close()
    out = {
        "metric": "element-assemblies/s + % HBM peak; mixed/learned vs FP64 at stated error",
        "value": res["fp64"]["value"], "unit": "element-assemblies/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["fp64"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded hybrid mesh and random Fourier fields)",
        "config": {"workload": "hybrid box, 20M elements (205 x 205 cells), precision comparison",
                   "elements": E, "field_nodes": m.n_field_nodes, "seeds": case.meta},
        "precisions": res, "full_step": step, "full_step_comparison": step_cmp, "variants": variants,
        "oracle_seconds_single_thread": t_oracle,
    }
    print(json.dumps(out), flush=True)
    mesh.close()


def spmv_bytes(nnz: int, n: int) -> int:
    """Algorithmic bytes of one product q = K p: 12 B per nonzero (value,
    column index), p read once and q written (8 B per row each); the storage
    format's own overhead (row pointers, padding) is not counted."""
    return 12 * nnz + 16 * n


def cg_bytes_per_iteration(nnz: int, n: int) -> int:
    """Algorithmic bytes of one Jacobi-CG iteration: the SpMV; the residual
    update reads r, q and the diagonal and writes r, z; the direction step
    reads x, p, z and writes x, p (8 B per row each)."""
    return spmv_bytes(nnz, n) + 8 * n * (5 + 5)


def run_cg(args):
    """The pressure solver (Section 3.2, Algorithm 1: Jacobi-preconditioned CG,
    one SpMV and two dot products per iteration) on the Laplacian of the 20 M
    hybrid box (the mesh of the precision workload).  A step is one CG
    iteration; --steps iterations run in one solve whose tolerance is never
    reached; right-hand side and matrix resident in HBM.  The dominant kernel
    is the SpMV, timed on its own by back-to-back products."""
    import torch
    from paper_2005_05899_amd import lesasm, meshgen
    torch.cuda.set_device(0)
    layers = meshgen.hybrid_layers(205 * 205, 20_000_000)
    mg_mesh = meshgen.hybrid_box(205, 205, layers, seed=4)
    mesh = lesasm.Mesh.from_arrays(mg_mesh, 0.1)
    n = mesh.n_field_nodes
    t0 = time.perf_counter()
    st = lesasm.Stepper(mesh, 1.5e-5, 1e-3, rtol=1e-300, maxit=args.steps)
    t_setup = time.perf_counter() - t0
    print(f"  stepper set up in {t_setup:.1f} s ({n} rows)", file=sys.stderr, flush=True)
    nnz = ctypes.c_int64()
    lesasm.check(lesasm.load().lesasm_stepper_laplacian(st._h, None, None, None, ctypes.byref(nnz)))
    nnz = nnz.value
    entries = st.sell_entries()
    b = mesh.to_internal(torch.from_numpy(np.random.default_rng(21).standard_normal(n)).cuda())
    if args.warmup:
        st.pressure_solve(b)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x = st.pressure_solve(b)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    it, res = st.stats()
    assert it == args.steps and np.isfinite(res) and torch.isfinite(x).all()
    # the SpMV alone: events on the stream the library launches on
    q = torch.empty_like(b)
    for _ in range(max(args.warmup, 1)):
        st.spmv(x, q)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(args.steps):
        st.spmv(x, q)
    ev[1].record()
    ev[1].synchronize()
    ms_spmv = ev[0].elapsed_time(ev[1]) / args.steps
    print(f"  {1e3 * el / it:.4f} ms per CG iteration, SpMV {ms_spmv:.4f} ms", file=sys.stderr, flush=True)
    sb = spmv_bytes(nnz, n)
    cb = cg_bytes_per_iteration(nnz, n)
    ms_it = 1e3 * el / it
    tr = traffic_from_profiles("all", "cg20m", "k_spmv_sell_dot", CG_SOURCES)
    out = {
        "metric": "pressure-CG row-iterations/s (Jacobi-PCG)", "value": n * it / el, "unit": "row-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_it, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded hybrid box, random b)",
        "config": {"workload": f"Laplacian of the hybrid box 205 x 205 cells ({mg_mesh.n_elems} elements): "
                               f"{n} rows, {nnz} nonzeros; {it} iterations per solve"},
        "roofline": {"bound": "hbm", "kernel": "k_spmv_sell_dot", "achieved": sb / ms_spmv / 1e6, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": sb / ms_spmv / 1e6 / HBM_PEAK_GBS,
                     "traffic": None if tr is None else tr["bytes_per_launch"], "bytes_per_launch": sb,
                     "avg_ms": ms_spmv},
        "source_hash": source_hash(CG_SOURCES),
        "iteration": {"algorithmic_bytes": cb, "GBs": cb / ms_it / 1e6, "frac_of_hbm": cb / ms_it / 1e6 / HBM_PEAK_GBS},
        "sliced_ellpack_entries": entries, "padding_fraction": entries / nnz - 1.0,
        "relative_residual_after": res, "setup_seconds": t_setup,
    }
    st.close()
    mesh.close()
    if not args.no_cpu_baseline:
        # the oracle's CG on a smaller box of the same construction (its
        # Laplacian assembly in the oracle takes minutes at 20 M); the rate is
        # per row-iteration, which scales linearly with the matrix
        from oracle import cg, step
        sm = meshgen.hybrid_case(500_000, seed_mesh=4, with_p=False, n_modes=8).mesh
        K = step.laplacian(sm)
        bs = np.random.default_rng(22).standard_normal(K.shape[0])
        iters = 0
        t2 = time.perf_counter()
        while time.perf_counter() - t2 < 10.0:
            cg.jacobi_pcg(K, bs, 100, rtol=0.0)
            iters += 100
        dt = time.perf_counter() - t2
        out["cpu_baseline"] = {"value": K.shape[0] * iters / dt, "unit": "row-iterations/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{iters} oracle CG iterations on the Laplacian of a {sm.n_elems}-element "
                                         f"hybrid box ({K.shape[0]} rows, {K.nnz} nonzeros), {dt:.1f} s"}
    print(json.dumps(out), flush=True)


def partition_bytes(mesh, nbins: int) -> dict:
    """Algorithmic bytes of the partitioner's kernels with ideal reuse.
    Locations: offsets (8 B per element), connectivity (4 B per element node),
    node coordinates once (24 B per node), location and weight written (28 B
    per element).  Split: locations read twice (bounding box, keys: 48 B),
    weights read (4 B), keys written and read (8 B), parts written (4 B) per
    element, plus the bins (8 B each) zeroed, scanned (read twice, written
    once) and read by the split (twice)."""
    E = mesh.n_elems
    return {"centroids": 8 * (E + 1) + 4 * int(mesh.conn.size) + 24 * mesh.n_nodes + 28 * E,
            "split": 64 * E + 8 * nbins * (1 + 3 + 2)}


def run_partition(args):
    """Space-filling-curve partition of the 20 M-element hybrid box (the mesh of
    the precision workload): element locations and Gauss-point weights on the
    GPU, then the Hilbert split into 8 parts on 128^3 bins.  A step is both
    calls; inputs (connectivity, coordinates) resident in HBM."""
    import torch
    from paper_2005_05899_amd import lesasm, meshgen
    torch.cuda.set_device(0)
    layers = meshgen.hybrid_layers(205 * 205, 20_000_000)
    mesh = meshgen.hybrid_box(205, 205, layers, seed=4)
    P, level = 8, 7
    off = torch.from_numpy(mesh.conn_offsets.astype(np.int64)).cuda()
    conn = torch.from_numpy(mesh.conn.astype(np.int32)).cuda()
    xyz = torch.from_numpy(mesh.coords).cuda()
    cen, w = lesasm.element_centroids(off, conn, xyz)
    part = lesasm.sfc_partition(cen, w, P, level=level)
    for _ in range(args.warmup):
        cen, w = lesasm.element_centroids(off, conn, xyz, check_input=False)
        part = lesasm.sfc_partition(cen, w, P, level=level)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cen, w = lesasm.element_centroids(off, conn, xyz, check_input=False)
        part = lesasm.sfc_partition(cen, w, P, level=level)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # kernel times: events on the stream the library launches on, around
    # back-to-back calls into preallocated buffers (the queue stays full)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    nbytes = ctypes.c_size_t()
    lesasm.check(lesasm.load().lesasm_sfc_workspace_bytes(mesh.n_elems, P, level, ctypes.byref(nbytes)))
    work = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(args.steps):
        lesasm.element_centroids(off, conn, xyz, check_input=False, out=(cen, w, status))
    ev[1].record()
    for _ in range(args.steps):
        part = lesasm.sfc_partition(cen, w, P, level=level, work=work)
    ev[2].record()
    ev[2].synchronize()
    assert int(status.item()) == 0
    E = mesh.n_elems
    nb = partition_bytes(mesh, 1 << (3 * level))
    ms_c, ms_p = ev[0].elapsed_time(ev[1]) / args.steps, ev[1].elapsed_time(ev[2]) / args.steps
    got = part.cpu().numpy()
    tr = traffic_from_profiles("all", "partition20m", "k_centroids", PARTITION_SOURCES)
    out = {
        "metric": "elements partitioned/s (SFC partitioner)", "value": E * args.steps / el,
        "unit": "elements/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 locations, int64 weights", "data": "synthetic",
        "config": {"workload": f"hybrid box 205 x 205 cells, {E} elements, {mesh.n_nodes} nodes; "
                               f"{P} parts, 2^{level} bins per axis, Gauss-point weights"},
        "roofline": {"bound": "hbm", "kernel": "k_centroids", "achieved": nb["centroids"] / ms_c / 1e6,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": nb["centroids"] / ms_c / 1e6 / HBM_PEAK_GBS,
                     "traffic": None if tr is None else tr["bytes_per_launch"],
                     "bytes_per_launch": nb["centroids"], "avg_ms": ms_c},
        "source_hash": source_hash(PARTITION_SOURCES),
        "split": {"ms": ms_p, "bytes": nb["split"], "GBs": nb["split"] / ms_p / 1e6},
        "part_elements": np.bincount(got, minlength=P).tolist(),
    }
    if not args.no_cpu_baseline:
        import oracle.partition as op
        t1 = time.perf_counter()
        rc, rw = op.element_centroids(mesh.coords, mesh.conn_offsets, mesh.conn)
        want, _, _ = op.sfc_partition(rc, rw, P, level=level)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": E / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
                               "sample": f"the whole {E}-element workload, one oracle run ({dt:.1f} s)"}
        out["parity_full"] = {"parts_identical": bool(np.array_equal(got, want)),
                              "centroids_identical": bool(np.array_equal(cen.cpu().numpy(), rc))}
    print(json.dumps(out), flush=True)


def run_balance(args):
    """Correction-coefficient load balancing (Section "Load balancing") on the
    2.0 M-element hybrid box: 8 parts from the GPU partitioner with
    Gauss-point weights, each part assembled as a mesh of its own (its
    interface nodes duplicated, as in the paper's substructuring) and timed;
    the weighted regression updates the coefficients and the mesh is split
    again.  Element-type kernels run one after another so that a part's time
    adds up its work.  --steps assemblies are timed per part and iteration."""
    import torch
    from paper_2005_05899_amd import lesasm, meshgen
    torch.cuda.set_device(0)
    case = meshgen.hybrid_2m_case()
    m = case.mesh
    P, level, iters = 8, 7, 8
    off = torch.from_numpy(m.conn_offsets.astype(np.int64)).cuda()
    conn = torch.from_numpy(m.conn.astype(np.int32)).cuda()
    xyz = torch.from_numpy(m.coords).cuda()
    cen, w = lesasm.element_centroids(off, conn, xyz)
    lam_hist, t_hist, lb, tsum, types = [], [], [], [], []
    lam = np.ones(P)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t0 = time.time()
    for it in range(iters):
        part = lesasm.sfc_partition(cen, w, P, lam=lam, level=level).cpu().numpy()
        times, mix = [], []
        for i in range(P):
            sub, fids = meshgen.submesh(m, np.where(part == i)[0])
            mesh = lesasm.Mesh.from_arrays(sub, case.vreman_c)
            mesh.set_option(lesasm.OPT_CONCURRENT, 0)
            u = mesh.to_internal(torch.from_numpy(case.u[fids]).cuda())
            p = mesh.to_internal(torch.from_numpy(case.p[fids]).cuda())
            rhs = torch.empty_like(u)
            for _ in range(args.warmup):
                mesh.assemble_momentum_rhs(u, p, case.nu, out=rhs)
            reps = []
            for _ in range(args.steps):
                ev[0].record()
                mesh.assemble_momentum_rhs(u, p, case.nu, out=rhs)
                ev[1].record()
                ev[1].synchronize()
                reps.append(ev[0].elapsed_time(ev[1]))
            times.append(float(np.median(reps)))
            mix.append(sub.type_counts())
            mesh.close()
        lam_hist.append(lam.copy())
        t_hist.append(times)
        lb.append(float(np.mean(times) / np.max(times)))
        tsum.append(float(np.sum(times)))
        types.append(mix)
        print(f"  iteration {it}: load balance {lb[-1]:.4f}, part times {np.round(times, 4).tolist()} ms "
              f"({time.time() - t0:.0f} s)", file=sys.stderr, flush=True)
        lam = lesasm.balance_update(lam_hist, t_hist, 1.5)
    import oracle.partition as op
    lam_oracle = op.balance_update(lam_hist, t_hist, 1.5)
    out = {
        "metric": "load balance (mean / max part assembly time, 8 parts)", "value": lb[-1], "unit": "ratio",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": tsum[-1] / P,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"hybrid box 95 x 95 x 94 cells, {m.n_elems} elements, 8 parts, weighted "
                               f"regression (weights x1.5 per iteration), {iters} iterations"},
        "load_balance_per_iteration": lb, "sum_of_part_times_ms": tsum,
        "lambda_per_iteration": [np.round(v, 5).tolist() for v in lam_hist],
        "part_types_first": types[0], "part_types_last": types[-1],
        "lambda_next_vs_oracle_max_abs": float(np.abs(lam - lam_oracle).max()),
    }
    print(json.dumps(out), flush=True)


def run_copy(args):
    """A plain device copy of 512 MiB per step: the calibration workload for
    the hardware byte counters (FETCH_SIZE and WRITE_SIZE should read 512 MiB
    each per copy)."""
    import torch
    torch.cuda.set_device(0)
    n = 64 << 20  # doubles: 512 MiB
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for _ in range(args.steps):  # the same bytes through an elementwise kernel (b = 1.0 * a)
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    nbytes = 2 * 8 * n
    print(json.dumps({"metric": "device copy bandwidth (counter calibration)", "value": nbytes * args.steps / el / 1e9,
                      "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "copy of 512 MiB (read 512 MiB, write 512 MiB per step)",
                                 "bytes_read_per_step": 8 * n, "bytes_written_per_step": 8 * n}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100, help="untimed steps first (lets the clocks settle)")
    ap.add_argument("--workload", choices=["hybrid20m", "hybrid2m", "tet20m", "batch64", "precision20m", "copy",
                                           "partition20m", "balance8", "cg20m"], default="hybrid20m")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--scatter", choices=["staged", "chunk_atomic", "colour", "direct"], default="staged")
    ap.add_argument("--chunk", type=int, default=None, help="elements per chunk (chunked scatters)")
    ap.add_argument("--no-variants", dest="variants", action="store_false")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--isolated", action="store_true",
                    help="run the element-type kernels one after another in the timed region too")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the assembly of one mesh "
              "partition is the single-GPU unit of work; multi-GPU sharding is described, not run)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch64":
        run_batch(args)
    elif args.workload == "precision20m":
        run_precision(args)
    elif args.workload == "copy":
        run_copy(args)
    elif args.workload == "partition20m":
        run_partition(args)
    elif args.workload == "balance8":
        run_balance(args)
    elif args.workload == "cg20m":
        run_cg(args)
    else:
        run_main(args)


if __name__ == "__main__":
    main()
