"""Planted mistakes: every pin battery must catch each of them.

Each mutant is a copy of the oracle's C source with one plausible mistake
(a dropped term, a wrong sign, a transposed bit, an off-by-one).  It is
compiled to a temporary library and the full pin battery runs against it in
a child process (so that a crash counts as caught).  A mutant that passes
every pin would mean the pins cannot tell the mistake from the method.
"""

import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

MUTANTS = {
    "anchor_not_aligned": ("anchor[a] = p[a] - p[a] % size;", "anchor[a] = p[a];"),
    "far_plane_sign": ("int64_t plane = m[a] > 0.0 ? anchor[a] + size : anchor[a];",
                       "int64_t plane = anchor[a] + size;"),
    "morton_y_z_swapped": ("k |= (uint64_t)((y >> b) & 1) << (3 * b + 1);",
                           "k |= (uint64_t)((y >> b) & 1) << (3 * b + 2);"),
    "lookup_off_by_one": ("if (keys[mid] <= k) lo = mid; else hi = mid;",
                          "if (keys[mid] < k) lo = mid; else hi = mid;"),
    "t_in_not_advanced": ("            t_in = t_out;\n        }", "        }"),
    "dropped_accumulation": ("N = N + rho[i] * l;", "N = rho[i] * l;"),
    "negative_step_stays": ("p[a] = m[a] > 0.0 ? anchor[a] + size : anchor[a] - 1;",
                            "p[a] = m[a] > 0.0 ? anchor[a] + size : anchor[a];"),
    "single_axis_at_ties": ("if (bounding[a] && tf[a] == t_out) {",
                            "if (bounding[a] && tf[a] == t_out && !out) { out = 2;"),
    "kahan_no_compensation": ("c = (t - S) - y;", "c = 0.0f;"),
    "gradient_without_chord": ("grad[vis[j]] += gr * chords[j];", "grad[vis[j]] += gr;"),
    "belt_shift_parity": ("((i - nside) % 2 == 0) ? 0.5 * dphi : 0.0;",
                          "((i - nside) % 2 == 1) ? 0.5 * dphi : 0.0;"),
    "cap_z_linear": ("z = 1.0 - (double)(i * i) / (3.0 * ns * ns);",
                     "z = 1.0 - (double)(i) / (3.0 * ns * ns);"),
    "exit_misses_low_face": ("if (p[a] < 0 || p[a] >= side) out = 1;",
                             "if (p[a] >= side) out = 1;"),
    "first_probe_rounded": ("for (int a = 0; a < 3; ++a) p[a] = (int64_t)floor(Q[a] * scale);",
                            "for (int a = 0; a < 3; ++a) p[a] = (int64_t)floor(Q[a] * scale + 0.5);"),
    "non_exit_axis_frozen": ("double x = fma(m[a], t_out, Q[a]) * scale;",
                             "double x = (double)p[a];"),
    "tiling_gap_ignored": ("if (keys[i] != expect) return ORC_ERR_TILING;", ""),
    "fields_plane_major": ("I[f] = I[f] + fields[vis[j] * K + f] * chords[j];",
                           "I[f] = I[f] + fields[f * n + vis[j]] * chords[j];"),
    "length_unit_dropped": ("const double nh = length * I[0];", "const double nh = I[0];"),
    "line_nu_squared": ("(8.0 * pi * (nu * nu * nu))", "(8.0 * pi * (nu * nu))"),
    "line_drops_8pi": ("(8.0 * pi * (nu * nu * nu))", "(nu * nu * nu)"),
    "du_no_turbulence": ("/ (pi * ORC_MP) + vturb * vturb);", "/ (pi * ORC_MP));"),
    "du_no_pi": ("/ (pi * ORC_MP) + vturb * vturb);", "/ ORC_MP + vturb * vturb);"),
    "beta_naive_quotient": ("1.0 : -expm1(-tau) / tau;", "1.0 : (1.0 - exp(-tau)) / tau;"),
    "beta_zero_depth_term": ("tau == 0.0 ? 1.0 :", "tau == 0.0 ? 0.0 :"),
    "av_eff_shift_lost": ("(xmin - log(sum / (double)Dn)) / gamma", "(-log(sum / (double)Dn)) / gamma"),
    "av_eff_mean_not_sum": ("log(sum / (double)Dn)", "log(sum)"),
    "nested_x_y_swapped": ("x |= ((in_face >> (2 * b)) & 1) << b;", "x |= ((in_face >> (2 * b + 1)) & 1) << b;"),
    "nested_face_row": ("const double Y = Yc - 1.0 + (double)(x + y + 1) / ns;",
                        "const double Y = Yc + (double)(x + y + 1) / ns;"),
    "nested_face_col": ("Xc = 2.0 * (f - 4);", "Xc = 1.0 + 2.0 * (f - 4);"),
    "nested_polar_stretch": ("phi = pi * (Xc + (X - Xc) / sigma) / 4.0;", "phi = pi * X / 4.0;"),
    "nested_polar_z": ("z = (1.0 - sigma * sigma / 3.0)", "z = (1.0 - sigma / 3.0)"),
    "nested_belt_z": ("z = 2.0 * Y / 3.0;", "z = 3.0 * Y / 8.0;"),
    "nested_reference_strided": ("sum = sum + fine[s * Dfine + q * ratio + k];",
                                 "sum = sum + fine[s * Dfine + q + k * Dcoarse];"),
    "nested_reference_sum": ("const double r = sum / (double)ratio;", "const double r = sum;"),
    "grid_floor_exclusive": ("split = mx[at] >= floor_ && (mx[at] - mn[at]) >= rel * mx[at];",
                             "split = mx[at] > floor_ && (mx[at] - mn[at]) >= rel * mx[at];"),
    "grid_variation_over_min": ("split = mx[at] >= floor_ && (mx[at] - mn[at]) >= rel * mx[at];",
                                "split = mx[at] >= floor_ && (mx[at] - mn[at]) >= rel * mn[at];"),
    "grid_mean_not_divided": ("mean[at] = sum / 8.0;", "mean[at] = sum;"),
    "grid_children_reversed": ("emit_leaves(L + 1, 8 * c + j, D,", "emit_leaves(L + 1, 8 * c + 7 - j, D,"),
    "grid_key_coarse_shift": ("keys[*n] = (uint64_t)c << (3 * (D - L));", "keys[*n] = (uint64_t)c << (3 * (D - L - 1));"),
    "nested_diagonal_sign": ("const double X = Xc + (double)(x - y) / ns;",
                             "const double X = Xc + (double)(y - x) / ns;"),
}

BATTERY = """
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {here!r})
import oracle, oracle_pins
lib = oracle.load({lib!r})
failed = []
for pin in oracle_pins.ALL_PINS:
    try:
        pin(oracle, lib)
    except Exception as e:
        failed.append(pin.__name__)
print("FAILED", len(failed), " ".join(failed))
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, f"mutation site not found: {name}"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = oracle.build(source=str(path), output=str(tmp_path / "libmutant.so"))
    code = BATTERY.format(root=ROOT, here=HERE, lib=lib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    caught = r.returncode != 0 or ("FAILED 0" not in r.stdout)
    assert caught, f"mutant {name} passed every pin: {r.stdout}"
