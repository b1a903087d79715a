"""The benchmark's host logic, on the CPU: the one-GPU rule, the byte counts
behind the roofline figures (checked on tiny meshes whose counts follow by
hand), and the source hash that decides whether committed counter summaries
still describe the kernels."""
import os
import subprocess
import sys

import numpy as np

import bench
from paper_2005_05899_amd import meshgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_single_hex_bytes_by_hand():
    # one HEX08 element: 8 connectivity entries, 8 nodes (24 B geometry,
    # 24 + 8 + 24 B fields) and one filter width
    m = mg.uniform_hex_box((1, 1, 1), (1.0, 1.0, 1.0))
    assert bench.algorithmic_bytes(m, True) == 4 * 8 + 24 * 8 + 8 * (24 + 8 + 24) + 8
    assert bench.algorithmic_bytes(m, False) == 4 * 8 + 24 * 8 + 8 * (24 + 24) + 8
    assert bench.per_type_bytes(m, mg.HEX08) == bench.algorithmic_bytes(m, True)


def test_per_type_bytes_add_up_to_the_mesh():
    c = mg.small_hybrid_case(nx=4, ny=3, layers=[(mg.PEN06, 1), (mg.TET04, 1), (mg.PYR05, 1), (mg.HEX08, 1)],
                             seed=3)
    parts = sum(bench.per_type_bytes(c.mesh, t) for t in (mg.TET04, mg.PYR05, mg.PEN06, mg.HEX08))
    assert abs(parts - bench.algorithmic_bytes(c.mesh, True)) <= 1e-6 * parts


def test_cg_byte_counts():
    # 10 nonzeros over 3 rows: values and columns 12 B each, p read and q
    # written once; the iteration adds 10 vector passes of 8 B per row
    assert bench.spmv_bytes(10, 3) == 120 + 48
    assert bench.cg_bytes_per_iteration(10, 3) == 120 + 48 + 8 * 3 * 10


def test_source_hash_ignores_comments_and_layout_but_not_code(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("// a comment\n__global__ void k(double *a) {\n    a[0] = 1.0; /* set */\n}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    pkg = tmp_path / "paper_2005_05899_amd"
    pkg.mkdir()
    (pkg / "k.hip").write_text(src.read_text())
    h0 = bench.source_hash(("k.hip",))
    (pkg / "k.hip").write_text("__global__ void k(double *a)\n{\n  a[0] = 1.0;  // set to one\n}\n")
    assert bench.source_hash(("k.hip",)) == h0
    (pkg / "k.hip").write_text("__global__ void k(double *a) {\n    a[0] = 2.0;\n}\n")
    assert bench.source_hash(("k.hip",)) != h0


def test_partition_byte_counts():
    m = mg.uniform_hex_box((2, 1, 1), (2.0, 1.0, 1.0))
    nb = bench.partition_bytes(m, 8)
    assert nb["centroids"] == 8 * 3 + 4 * 16 + 24 * 12 + 28 * 2
    assert nb["split"] == 64 * 2 + 8 * 8 * 6
    assert np.isfinite(list(nb.values())).all()


def test_cpu_baseline_uses_the_threads_it_reports(monkeypatch):
    # the all-core leg runs the oracle's threaded assembly on OMP_NUM_THREADS
    # threads (the CPU share of the process) and says so, with the host model
    c = mg.small_hybrid_case(nx=4, ny=3, seed=5)
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    assert bench.baseline_threads() == 3
    cb = bench.cpu_baseline(c, single_thread_s=0.5, min_cpu_seconds=0.0, max_reps=2)
    assert cb["cores"] == 3 and cb["kind"] == "oracle" and cb["value"] > 0
    assert "3 threads" in cb["sample"] and cb["host"]["logical_cpus"] >= 1
    assert abs(cb["single_thread"]["value"] - c.mesh.n_elems / 0.5) < 1e-9
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert bench.baseline_threads() == len(os.sched_getaffinity(0))


def test_kernel_table_rates_and_per_assembly_gather():
    """Per-kernel figures from summed event times: average per launch, flop
    rate from the nominal counts, and the gather summed per assembly (it runs
    as one launch per class of shared nodes)."""
    m = mg.uniform_hex_box((2, 1, 1), (2.0, 1.0, 1.0))  # two HEX08 elements

    class FakeMesh:
        n_per_type = {4: 0, 5: 0, 6: 0, 8: 2}

    kt = {"tet04": (0.0, 0), "pyr05": (0.0, 0), "pen06": (0.0, 0), "hex08": (3.0, 3),  # 3 launches, 1 ms each
          "gather": (1.5, 15), "fill": (0.0, 0)}                                        # 5 launches per assembly
    tab = bench.kernel_table(FakeMesh(), m, kt, 78.6)
    assert set(tab) == {"hex08", "gather"}
    h = tab["hex08"]
    assert h["avg_ms"] == 1.0 and h["launches"] == 3 and h["elements"] == 2
    assert abs(h["algorithmic_tflops"] - 2 * 7200 / 1e-3 / 1e12) < 1e-18
    assert abs(h["frac_of_peak"] - h["algorithmic_tflops"] / 78.6) < 1e-18
    g = tab["gather"]
    assert g["ms_per_assembly"] == 0.5 and g["launches_per_assembly"] == 5 and g["avg_ms_per_launch"] == 0.1
