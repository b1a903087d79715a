"""Writes the stored expected values under tests/golden/ from the FP64 oracle.

Only the oracle (oracle/) computes them; the inputs come from the seeded
generators in paper_2005_05899_amd/meshgen.py.  Run from the repository root:

    python tests/golden/make_golden.py

Fixtures (text, one row per field node: x y z components of the nodal
right-hand side of M_L du/dt = rhs, Algorithm 1 "Element assembly",
momentum equation of Section 3.2):
  small_hybrid_rhs.txt  -- every element type (TET04, PYR05, PEN06, HEX08),
                           3 x 2 cells x 7 layers, seed 7, nu 0.05, c 0.1
  tg16_rhs_sample.txt   -- periodic 16^3 HEX08 Taylor-Green cube with noise
                           (seed 1, nu 1e-5, c 0.1): rows of 97 sampled field
                           nodes (node id first), plus column norms
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2005_05899_amd import meshgen  # noqa: E402

SMALL = dict(nx=3, ny=2, seed=7)
TG_SAMPLE = np.arange(0, 4096, 43)  # 96 nodes spread over the cube
TG_SAMPLE = np.append(TG_SAMPLE, 4095)


def small_case():
    return meshgen.small_hybrid_case(**SMALL)


def tg_case():
    return meshgen.periodic_tg_case(16)


def main():
    c = small_case()
    rhs = oracle.assemble(c.mesh, c.u, c.p, c.nu, c.vreman_c)
    hdr = ("nodal rhs of the explicit momentum residual (Algorithm 1, element assembly; Section 3.2), FP64 oracle\n"
           f"case: meshgen.small_hybrid_case(nx=3, ny=2, seed=7): {c.mesh.n_elems} elements, "
           f"{c.mesh.n_field_nodes} field nodes, per type {c.mesh.type_counts()}\n"
           "written by tests/golden/make_golden.py; columns rhs_x rhs_y rhs_z")
    np.savetxt(os.path.join(HERE, "small_hybrid_rhs.txt"), rhs, fmt="%.17e", header=hdr)

    t = tg_case()
    rhs = oracle.assemble(t.mesh, t.u, t.p, t.nu, t.vreman_c)
    rows = np.column_stack([TG_SAMPLE.astype(float), rhs[TG_SAMPLE]])
    norms = np.linalg.norm(rhs, axis=0)
    hdr = ("nodal rhs of the explicit momentum residual (Algorithm 1, element assembly; Section 3.2), FP64 oracle\n"
           "case: meshgen.periodic_tg_case(16): 16^3 periodic HEX08, Taylor-Green + 1e-3 uniform noise (seed 1), "
           "nu 1e-5, c 0.1\n"
           f"column 2-norms over all 4096 field nodes: {norms[0]:.17e} {norms[1]:.17e} {norms[2]:.17e}\n"
           "written by tests/golden/make_golden.py; columns node rhs_x rhs_y rhs_z")
    np.savetxt(os.path.join(HERE, "tg16_rhs_sample.txt"), rows, fmt="%.17e", header=hdr)


if __name__ == "__main__":
    main()
