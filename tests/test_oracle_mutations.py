"""The oracle's pins have teeth: each plausible mistake below, planted in a
temporary copy of the oracle's C source (never in the oracle itself), makes
at least one test of tests/test_oracle_pins.py (tests/test_oracle_tracking.py
for the cell tracking) fail.

Slow (every mutant is compiled and the pins run against it): set
SUBSURF4D_SLOW=1 to run it.  CPU only.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "subsurf4d_oracle.c")

PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")
TRACKING = os.path.join(ROOT, "tests", "test_oracle_tracking.py")

# name: (text of the oracle, mistaken text[, the test file whose pins must catch it])
MUTANTS = {
    # G on the "-e_d" face taken from the cell itself instead of P - e_d
    "minus_face_G_from_P": ("Gf[2 * d] = G[(size_t)d * np + pidx(n, Pm[0], Pm[1], Pm[2], Pm[3])];",
                            "Gf[2 * d] = G[(size_t)d * np + pidx(n, P[0], P[1], P[2], P[3])];"),
    # Abar averaged over 4 instead of the 8 faces
    "abar_over_4": ("qs / 8.0", "qs / 4.0"),
    # tangential difference divided by 2h instead of h
    "tangential_2h": ("g[t] = (up - dn) / h;", "g[t] = (up - dn) / (2.0*h);"),
    # Dirichlet neighbour term dropped from the right-hand side
    "drop_dirichlet_term": ("rhs += cf * ub[", "rhs += 0.0 * ub["),
    # tangential corner taken around P instead of the face's other cell
    "tangential_index": ("get(ctx, Q[0] - f[0], Q[1] - f[1], Q[2] - f[2], Q[3] - f[3])) / 4.0;",
                         "get(ctx, P[0] - f[0], P[1] - f[1], P[2] - f[2], P[3] - f[3])) / 4.0;"),
    # relaxation applied to the new value only (omega ignored)
    "sor_ignores_omega": ("u[p] = omega * ubar + (1.0 - omega) * u[p];",
                          "u[p] = omega * ubar + (1.0 - omega) * ubar;"),
    # Neumann heat step with the interior stencil count at the boundary
    "heat_boundary_count": ("*diag = 1.0 + a * cnt;", "*diag = 1.0 + a * 8;"),
    # edge detector of the norm of the combined gradients instead of the sum of norms
    "g_of_combined_norm": ("const double s = delta * n0 + vartheta * n1;",
                           "const double s = sqrt(delta*delta*n0*n0 + vartheta*vartheta*n1*n1);"),
    # strict comparison in the local threshold
    "threshold_strict": ("ITH[q] = (I0[q] >= th) ? beta[m] : alpha[m];",
                         "ITH[q] = (I0[q] > th) ? beta[m] : alpha[m];"),
    # ownership ties go to the last ball instead of the first
    "owner_tie_last": ("if (owner[q] < 0 || d2 < best[q])", "if (owner[q] < 0 || d2 <= best[q])"),
    # rescale divides by the maximum only
    "rescale_max_only": ("u[p] = (u[p] - mu[m]) / (xi[m] - mu[m]);", "u[p] = (u[p]) / (xi[m]);"),
    # eps instead of eps^2 in Abar
    "abar_eps_not_squared": ("const double Abar = sqrt(eps * eps + qs / 8.0);",
                             "const double Abar = sqrt(eps + qs / 8.0);"),
    # normal derivative in t divided by 2h
    "normal_t_2h": ("if (t == d) { g[t] = (vQ - vP) / h; continue; }",
                    "if (t == d) { g[t] = (vQ - vP) / (t==3 ? 2*h : h); continue; }"),
    # initial function without the cut-off shift 1/(R+v)
    "init_no_shift": ("double val = 1.0 / (dd + v) - 1.0 / (R + v);", "double val = 1.0 / (dd + v) - 0.0 / (R + v);"),
    # stopping rule against the absolute residual instead of tol * ||b||
    "stop_absolute": ("if (R <= tol * bn) return 0;", "if (R <= tol) return 0;"),
    # cell tracking: one face neighbour (+z) missing from the flood fill
    "label_no_plus_z": ("{ci, cj, ck - 1}, {ci, cj, ck + 1}};", "{ci, cj, ck - 1}, {ci, cj, ck - 1}};", TRACKING),
    # distances: the region outside the image not counted as outside
    "dist_no_outer_shell": ("for (long c = 0; c <= n[2] + 1; ++c)", "for (long c = 1; c <= n[2]; ++c)", TRACKING),
    # distances: the z offset not squared
    "dist_z_not_squared": ("+ (c - k) * (c - k);", "+ (c - k);", TRACKING),
    # backward link looked up in the cell's own frame instead of frame l-1
    "link_same_frame": ("const int32_t below = label[(size_t)r[2] - fsz];", "const int32_t below = label[(size_t)r[2]];",
                        TRACKING),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is missing")
    good, bad, pins = (MUTANTS[name] + (PINS,))[:3]
    src = open(SRC).read()
    assert src.count(good) >= 1, f"{name}: the oracle text it mutates has changed"
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(good, bad))
    lib = tmp_path / "libmutant.so"
    subprocess.run([gcc, "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-o", str(lib),
                    str(mutant), "-lm"], check=True)
    env = dict(os.environ, SUBSURF4D_ORACLE_LIB=str(lib))
    env.pop("SUBSURF4D_SLOW", None)
    r = subprocess.run([sys.executable, "-m", "pytest", pins, "-q", "-x",
                        "-m", "not gpu", "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    # exit status 1 with a failed test: a pin caught it (not a load or collection error)
    assert r.returncode == 1 and " failed" in r.stdout, f"{name}: no pin failed\n{r.stdout[-2000:]}"
