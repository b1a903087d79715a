"""The oracle's pins catch plausible mistakes.

Each mutant plants one bug in a copy of the oracle source (on the CPU), builds
it, and runs the pin suite against it in a subprocess; the suite must fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lesasm_oracle.c")
PINS = ["tests/test_oracle_refelem.py", "tests/test_oracle_vreman.py", "tests/test_oracle_exact.py",
        "tests/test_oracle_invariants.py", "tests/test_oracle_step.py", "tests/test_oracle_closure.py",
        "tests/test_oracle_wall.py"]

MUTANTS = {
    "gradient_uses_J_inverse_untransposed": ("s += K[j][i] * dN[3 * a + j];", "s += K[i][j] * dN[3 * a + j];"),
    "jacobian_transposed": ("s += x[3 * a + i] * dN[3 * a + j];", "s += x[3 * a + j] * dN[3 * a + i];"),
    "emac_drops_divergence_term": ("C[i] = s + divu * ug[i];", "C[i] = s;"),
    "strain_not_symmetrised": ("S[i][j] = G[i][j] + G[j][i];", "S[i][j] = 2.0 * G[i][j];"),
    "pressure_gradient_sign": ("if (terms & TERM_PRES) f += dp[i];", "if (terms & TERM_PRES) f -= dp[i];"),
    "residual_sign": ("R[3 * a + i] -= dV * (N[a] * f + s);", "R[3 * a + i] -= dV * (N[a] * f - s);"),
    "pyramid_weights_swapped": ("const double W[2] = {1.0 / 6.0 + sqrt(10.0) / 48.0, 1.0 / 6.0 - sqrt(10.0) / 48.0};",
                                "const double W[2] = {1.0 / 6.0 - sqrt(10.0) / 48.0, 1.0 / 6.0 + sqrt(10.0) / 48.0};"),
    "tet_rule_point": ("const double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0", "const double a = (5.0 + 3.0 * sqrt(5.0)) / 21.0"),
    "vreman_drops_minor": ("+ beta[1][1] * beta[2][2] - beta[1][2] * beta[1][2];", "+ beta[1][1] * beta[2][2];"),
    "filter_width_sqrt": ("const double delta = cbrt(vol);", "const double delta = sqrt(vol);"),
    "hex_zeta_derivative": ("dN[3 * a + 2] = 0.125 * za[a] * fx * fy;", "dN[3 * a + 2] = 0.125 * za[a] * fx * fz;"),
    "prism_zeta_derivative": ("dN[3 * a + 2] = L[i] * dZ[j];", "dN[3 * a + 2] = L[i] * Z[j];"),
    "pyramid_zeta_derivative": ("dN[3 * a + 2] = (-(A + B) * q + A * B) / (4.0 * q * q);",
                                "dN[3 * a + 2] = (-(A + B) * q - A * B) / (4.0 * q * q);"),
    "scatter_wrong_node": ("rhs[3 * fid[a] + i] += R[3 * a + i];", "rhs[3 * fid[(a + 1) % n] + i] += R[3 * a + i];"),
    "lumped_mass_ignores_jacobian": ("M[fid[a]] += w[q] * d * N[a];", "M[fid[a]] += w[q] * N[a];"),
    "viscosity_ignores_eddy": ("if (terms & TERM_SGS) visc += nut;", "if (terms & TERM_SGS) visc += 0.5 * nut;"),
    "laplacian_untransposed_inverse": ("s += Ki[j][i] * dN[3 * a + j];", "s += Ki[i][j] * dN[3 * a + j];"),
    "laplacian_drops_jacobian": ("K[a * n + b] += w[q] * det * s;", "K[a * n + b] += w[q] * s;"),
    "divergence_untransposed_inverse": ("div += ue[3 * a + i] * Ki[j][i] * dN[3 * a + j];",
                                        "div += ue[3 * a + i] * Ki[i][j] * dN[3 * a + j];"),
    "wall_traction_sign": ("t[k] = -utau * utau * ut[k] / U;", "t[k] = utau * utau * ut[k] / U;"),
    "wall_keeps_normal_velocity": ("ut[k] = uel[k] - un * nrm[k];", "ut[k] = uel[k];"),
    "wall_law_drops_damping": ("WALL_C1 * (1.0 - exp(-yp / WALL_CHI) - (yp / WALL_CHI) * exp(-yp / 3.0));",
                               "WALL_C1 * (1.0 - exp(-yp / WALL_CHI));"),
    "wall_quad_drops_jacobian": ("wa[a] += 0.25 * (1.0 + s[a] * xi) * (1.0 + t[a] * eta) * jac;",
                                 "wa[a] += 0.25 * (1.0 + s[a] * xi) * (1.0 + t[a] * eta);"),
    "wall_distance_from_origin": ("y += nrm[k] * (xe[k] - xc[k]);", "y += nrm[k] * xe[k];"),
    "wall_tau_not_squared": ("t[k] = -utau * utau * ut[k] / U;", "t[k] = -utau * ut[k] / U;"),
}


def _run_pins(src_text, tmp_path):
    sys.path.insert(0, ROOT)
    from oracle.oracle import build
    mut = tmp_path / "variant.c"
    mut.write_text(src_text)
    lib = build(str(mut), str(tmp_path / "libvariant.so"))
    env = dict(os.environ, LESASM_ORACLE_LIB=lib)
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.mark.slow
def test_unmodified_copy_passes(tmp_path):
    r = _run_pins(open(SRC).read(), tmp_path)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, name  # every copy of the line gets the same bug
    r = _run_pins(src.replace(old, new), tmp_path)
    assert r.returncode == 1, f"pins did not catch {name}:\n{r.stdout[-2000:]}"


# ---- the partitioner and balancing oracle (Python) ----------------------------

PART_SRC = os.path.join(ROOT, "oracle", "partition.py")
PART_PINS = "tests/test_oracle_partition.py"
PART_MUTANTS = {
    "hilbert_gray_code_skips_an_axis": ("X[2] = X[2] ^ X[1]", "X[2] = X[2] ^ X[0]"),
    "hilbert_no_inversion": ("x0_flipped = X[0] ^ low", "x0_flipped = X[0]"),
    "hilbert_excess_from_first_axis": ("t = np.where((X[2] & q) != 0, t ^ (q - 1), t)",
                                       "t = np.where((X[0] & q) != 0, t ^ (q - 1), t)"),
    "bins_not_clamped": ("out[:, k] = np.minimum(v, nb - 1)", "out[:, k] = v"),
    "targets_wrong_normalisation": ("out.append(acc * float(total) / float(n_parts))",
                                    "out.append(acc * float(total) / float(n_parts + 1))"),
    "split_at_bin_start": ("mid2 = (2 * before[key] + binw[key])", "mid2 = (2 * before[key])"),
    "inclusive_prefix": ("before = np.concatenate([[0], np.cumsum(binw)[:-1]])", "before = np.cumsum(binw)"),
    "centroid_wrong_divisor": ("cen[sel] = acc / n", "cen[sel] = acc / (n - 1)"),
    "upsilon_over_sum": ("Ups = np.cumsum(T, axis=1) / T.mean(axis=1, keepdims=True)",
                         "Ups = np.cumsum(T, axis=1) / T.sum(axis=1, keepdims=True)"),
    "regression_weights_reversed": ("wk = growth ** np.arange(K)", "wk = growth ** -np.arange(K)"),
    "regression_cut_off_by_one": ("nxt = (i - alpha) / beta", "nxt = (i - 1 - alpha) / beta"),
    "degenerate_spread_threshold_dropped": ("if x.max() - x.min() > 1e-12 * P and sxx > 0:", "if sxx > 0:"),
    "degenerate_spread_threshold_too_wide": ("if x.max() - x.min() > 1e-12 * P and sxx > 0:",
                                             "if x.max() - x.min() > 1e-6 * P and sxx > 0:"),
    "negative_slope_accepted": ("if beta > 0:", "if beta != 0:"),
    "fallback_keeps_the_newest_point": ("nxt = i * x[-1] / y[-1] if y[-1] > 0 else x[-1]", "nxt = x[-1]"),
}


def _run_partition_pins(src_text, tmp_path):
    mut = tmp_path / "partition_variant.py"
    mut.write_text(src_text)
    env = dict(os.environ, LESASM_PARTITION_ORACLE=str(mut))
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", PART_PINS],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_partition_unmodified_copy_passes(tmp_path):
    r = _run_partition_pins(open(PART_SRC).read(), tmp_path)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(PART_MUTANTS))
def test_partition_pins_catch_mutant(name, tmp_path):
    old, new = PART_MUTANTS[name]
    src = open(PART_SRC).read()
    assert src.count(old) >= 1, name
    r = _run_partition_pins(src.replace(old, new), tmp_path)
    assert r.returncode == 1, f"pins did not catch {name}:\n{r.stdout[-2000:]}"


# ---- the conjugate-gradient oracle (Python) -----------------------------------

CG_SRC = os.path.join(ROOT, "oracle", "cg.py")
CG_PINS = "tests/test_oracle_cg.py"

CG_MUTANTS = {
    "beta_inverted": ("p = z + (rz_new / rz) * p", "p = z + (rz / rz_new) * p"),
    "direction_from_unpreconditioned_residual": ("p = z + (rz_new / rz) * p", "p = r + (rz_new / rz) * p"),
    "alpha_from_r_dot_r": ("alpha = rz / float(p @ q)", "alpha = float(r @ r) / float(p @ q)"),
    "residual_update_sign": ("r = r - alpha * q", "r = r + alpha * q"),
    "rz_never_advanced": ("            rz = rz_new\n", "            pass\n"),
    "preconditioner_not_inverted": ("dinv = 1.0 / K.diagonal()", "dinv = K.diagonal()"),
    "right_hand_side_not_projected": ("        b = b - b.mean()\n", "        b = b + 0.0\n"),
    "solution_not_projected": ("        x = x - x.mean()\n", "        x = x + 0.0\n"),
    "stops_on_unchecked_iterations": ("if it % check_every == 0 or it == maxit:", "if True:"),
}


def _run_cg_pins(src_text, tmp_path):
    mut = tmp_path / "cg_variant.py"
    mut.write_text(src_text)
    env = dict(os.environ, LESASM_CG_ORACLE=str(mut))
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", CG_PINS],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_cg_unmodified_copy_passes(tmp_path):
    r = _run_cg_pins(open(CG_SRC).read(), tmp_path)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(CG_MUTANTS))
def test_cg_pins_catch_mutant(name, tmp_path):
    old, new = CG_MUTANTS[name]
    src = open(CG_SRC).read()
    assert src.count(old) == 1, name
    r = _run_cg_pins(src.replace(old, new), tmp_path)
    assert r.returncode == 1, f"pins did not catch {name}:\n{r.stdout[-2000:]}"


# ---- the learned-closure oracle (Python) -------------------------------------

CLOSURE_SRC = os.path.join(ROOT, "oracle", "closure.py")
CLOSURE_PINS = "tests/test_oracle_closure.py"
CLOSURE_MUTANTS = {
    "fallback_comparison_inverted": ("use[e] = np.linalg.norm(D) ** 2 <= tol * tol * nr * nr",
                                     "use[e] = np.linalg.norm(D) ** 2 >= tol * tol * nr * nr"),
    "vreman_stress_sign": ("tau_v = -nut[:, None] * np.stack(", "tau_v = nut[:, None] * np.stack("),
    "network_stress_drops_width_squared": ("tau_m = (dg ** 2 * g2)[:, None]", "tau_m = (g2)[:, None]"),
    "network_stress_drops_gradient_norm": ("tau_m = (dg ** 2 * g2)[:, None]", "tau_m = (dg ** 2)[:, None]"),
    "network_stress_keeps_trace": ("* _mlp.deviatoric(y)", "* y"),
    "kept_element_drops_vreman_residual": ("RV[e] + D if use[e] else RV[e]", "D if use[e] else RV[e]"),
    "strain_not_symmetrised": ("S = G + G.transpose(0, 2, 1)", "S = 2.0 * G"),
    "stress_components_swapped": ("S[:, 0, 1], S[:, 0, 2], S[:, 1, 2]]", "S[:, 0, 1], S[:, 1, 2], S[:, 0, 2]]"),
    "error_ratio_inverted": ("eps[e] = np.linalg.norm(D) / nr if", "eps[e] = nr / np.linalg.norm(D) if"),
    "reference_width_for_every_element": ("dg = np.repeat(deltas, ng)", "dg = np.repeat(deltas, ng) * 0 + delta_ref"),
    "network_sees_transposed_gradient": ("x, g2 = _mlp.features(G, dg, delta_ref)",
                                         "x, g2 = _mlp.features(G.transpose(0, 2, 1), dg, delta_ref)"),
}


def _run_closure_pins(src_text, tmp_path):
    mut = tmp_path / "closure_variant.py"
    mut.write_text(src_text)
    env = dict(os.environ, LESASM_CLOSURE_ORACLE=str(mut))
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", CLOSURE_PINS],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_closure_unmodified_copy_passes(tmp_path):
    r = _run_closure_pins(open(CLOSURE_SRC).read(), tmp_path)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(CLOSURE_MUTANTS))
def test_closure_pins_catch_mutant(name, tmp_path):
    old, new = CLOSURE_MUTANTS[name]
    src = open(CLOSURE_SRC).read()
    assert src.count(old) == 1, name
    r = _run_closure_pins(src.replace(old, new), tmp_path)
    assert r.returncode == 1, f"pins did not catch {name}:\n{r.stdout[-2000:]}"


# ---- the closure's training data (Python) -------------------------------------

TRAIN_SRC = os.path.join(ROOT, "paper_2005_05899_amd", "training.py")
TRAIN_PINS = "tests/test_training_data.py"
TRAIN_MUTANTS = {
    "filter_weights": ("f = 0.25 * np.roll(f, 1, axis=ax) + 0.5 * f + 0.25 * np.roll(f, -1, axis=ax)",
                       "f = 0.3 * np.roll(f, 1, axis=ax) + 0.4 * f + 0.3 * np.roll(f, -1, axis=ax)"),
    "filter_skips_an_axis": ("    for ax in range(3):\n        f = 0.25", "    for ax in range(2):\n        f = 0.25"),
    "velocity_restricted_off_grid": ("ub = box_filter(ub)[::2, ::2, ::2]", "ub = box_filter(ub)[::2, 1::2, ::2]"),
    "products_not_filtered": ("pb = box_filter(pb)[::2, ::2, ::2]", "pb = pb[::2, ::2, ::2]"),
    "stress_sign": ("tau = pb - np.stack(", "tau = pb + np.stack("),
    "stress_components_mismatched": (
        "ub[..., 0] * ub[..., 1], ub[..., 0] * ub[..., 2], ub[..., 1] * ub[..., 2]], axis=-1)\n    return",
        "ub[..., 0] * ub[..., 2], ub[..., 0] * ub[..., 1], ub[..., 1] * ub[..., 2]], axis=-1)\n    return"),
    "gradient_axes_reversed": ("np.stack([gxv, gyv, gzv], axis=-1)", "np.stack([gzv, gyv, gxv], axis=-1)"),
    "gradient_not_scaled_by_spacing": ("f.shape[-1], 3) / h)", "f.shape[-1], 3))"),
    "interpolation_weight_wrong_axis": ("wx = gx if dx else 1 - gx", "wx = gy if dx else 1 - gy"),
    "gauss_points_wrong": ("GAUSS_1D = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))",
                           "GAUSS_1D = (0.5 - 0.5 / math.sqrt(2.0), 0.5 + 0.5 / math.sqrt(2.0))"),
    "corner_shift_axes_swapped": ("np.roll(f, (-dz, -dy, -dx), axis=(0, 1, 2))",
                                  "np.roll(f, (-dx, -dy, -dz), axis=(0, 1, 2))"),
    "target_scaled_by_width_once": ("(tg / (h * h * g2)[:, None])", "(tg / (h * g2)[:, None])"),
    "width_feature_inverted": ("math.log(h / delta_ref)", "math.log(delta_ref / h)"),
    "target_keeps_trace": ("        tg = deviatoric(tg)\n", "        tg = tg\n"),
    "reference_width_of_the_fine_grid": ("delta_ref = length / (n // 2)", "delta_ref = length / n"),
}


def _run_training_pins(src_text, tmp_path):
    mut = tmp_path / "training_variant.py"
    mut.write_text(src_text)
    env = dict(os.environ, LESASM_TRAINING_MODULE=str(mut))
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", TRAIN_PINS],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_training_unmodified_copy_passes(tmp_path):
    r = _run_training_pins(open(TRAIN_SRC).read(), tmp_path)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(TRAIN_MUTANTS))
def test_training_pins_catch_mutant(name, tmp_path):
    old, new = TRAIN_MUTANTS[name]
    src = open(TRAIN_SRC).read()
    assert src.count(old) == 1, name
    r = _run_training_pins(src.replace(old, new), tmp_path)
    assert r.returncode == 1, f"pins did not catch {name}:\n{r.stdout[-2000:]}"
