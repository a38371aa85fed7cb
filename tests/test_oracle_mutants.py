"""The oracle's pins catch plausible mistakes.

Each case copies oracle.c with one planted mistake, builds it (same flags as
the oracle), and runs the named pins of test_oracle_pins.py against that
library in a child process: at least one of them must fail.  The mistakes
are the kind a reading of the paper or a slip in the code could make.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = [
    # (name, original text, planted text, pins that must catch it)
    ("reflection without q on the spin",
     "p1 = (2.0 * psi - q * cur) / q;", "p1 = (2.0 * psi - cur) / q;",
     "over_relaxation_conserves_energy"),
    ("the printed reflection (q = 1 field, mod 2 pi)",
     "double psi = atan2(sy, sx);\n                p1 = (2.0 * psi - q * cur) / q;",
     "double cx = 0.0, cy = 0.0;\n"
     "                if (x > 0) { cx += cos(phi[i - 1]); cy += sin(phi[i - 1]); }\n"
     "                if (x + 1 < nx) { cx += cos(phi[i + 1]); cy += sin(phi[i + 1]); }\n"
     "                if (y > 0) { cx += cos(phi[i - nx]); cy += sin(phi[i - nx]); }\n"
     "                if (y + 1 < ny) { cx += cos(phi[i + nx]); cy += sin(phi[i + nx]); }\n"
     "                p1 = fmod(2.0 * atan2(cy, cx) - cur + 2.0 * O_TWO_PI, O_TWO_PI);",
     "over_relaxation_conserves_energy"),
    ("Delta H with the wrong sign",
     "double dH = local_energy(nx, ny, phi, x, y, p2, q) - local_energy(nx, ny, phi, x, y, p1, q);",
     "double dH = local_energy(nx, ny, phi, x, y, p1, q) - local_energy(nx, ny, phi, x, y, p2, q);",
     "single_site_chain_matches_conditional_density and not for_q"),
    ("a neighbour dropped from the local energy",
     "    if (y + 1 < ny) h -= cos(q * (v - phi[i + nx]));\n    return h;",
     "    return h;",
     "single_site_chain_matches_conditional_density and not for_q"),
    ("acceptance with T multiplied",
     "int acc = (dH <= 0.0) || (exp(-dH / T) > r);", "int acc = (dH <= 0.0) || (exp(-dH * T) > r);",
     "single_site_chain_matches_conditional_density and not for_q"),
    ("one-sided proposal",
     "double raw = p1 + O_TWO_PI * (u - 0.5) / a;", "double raw = p1 + O_TWO_PI * u / a;",
     "single_site_chain_matches_conditional_density and not for_q"),
    ("vertical bonds missing from the energy",
     "            if (y + 1 < ny) H -= cos(q * (phi[i] - phi[i + nx]));\n        }\n    return H;",
     "        }\n    return H;",
     "energy_and_sample_energy_against_direct_sums"),
    ("map scaled by z_max instead of the range",
     "O_TWO_PI * ((z[i] - zmin) / (zmax - zmin))", "O_TWO_PI * ((z[i] - zmin) / zmax)",
     "map_endpoints_and_round_trip"),
    ("temperature interpolated linearly in T",
     "double x0 = log(Tg[k]), x1 = log(Tg[k + 1]);\n        *T_hat = exp(x0 + (ys - yf[k]) * (x1 - x0) / (yf[k + 1] - yf[k]));",
     "double x0 = Tg[k], x1 = Tg[k + 1];\n        *T_hat = x0 + (ys - yf[k]) * (x1 - x0) / (yf[k + 1] - yf[k]);",
     "invert_temperature_on_exact_power_law"),
    ("a-rule indexed by i instead of i + 1",
     "if (A < p->a_targ) a = 1.0 + (double)(t + 1) / p->k_a;",
     "if (A < p->a_targ) a = 1.0 + (double)t / p->k_a;",
     "a_rule or control_trace"),
    ("acceptance ratio over all sites instead of the P gaps",
     "                A = (double)acc / (double)P;",
     "                A = (double)acc / (double)n;",
     "a_rule or control_trace"),
    ("final a carried into the equilibrium sweeps",
     "double a_eq = p->eq_a_mode ? a : 1.0;", "double a_eq = a;",
     "a_rule or control_trace"),
]


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new, pins):
    text = open(SRC).read()
    assert text.count(old) == 1, name
    src = tmp_path / "oracle_mutant.c"
    src.write_text(text.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
                           "-o", str(lib), str(src), "-lm"])
    env = dict(os.environ, MPR_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert "passed" in r.stdout or "failed" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
    assert r.returncode == 1, f"{name}: the pins {pins!r} did not catch it\n" + r.stdout[-1500:]
