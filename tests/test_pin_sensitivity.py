"""The oracle's pins must fail on plausible mistakes: each case below alters
one expression of the oracle (a copy of its source, built into a temporary
library; the oracle itself is untouched), and the pin tests that cover that
function are run against the altered build in a subprocess.  Every
alteration must make at least one of them fail.

The alterations are the slips a reader of the paper could make in the time
step (Algorithm 1, local-time-step reading), the residual norm, the forces
(postprocessor reading), the Venkatakrishnan limiter and the modified
q-variables of eq. (28)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "qlskum_oracle.c")
PINS = ["tests/test_oracle_pins_aux.py", "tests/test_oracle_pins_kobc.py"]

PLANTS = {
    "timestep: largest distance": (
        "if (d < dmin) dmin = d;", "if (d > dmin || dmin == INFINITY) dmin = d;"),
    "timestep: sound speed without gamma": (
        "double c = sqrt(prm->gamma * prim[3] / prim[0]);", "double c = sqrt(prim[3] / prim[0]);"),
    "timestep: CFL dropped": (
        "dt[p] = prm->cfl * dmin / (speed + c);", "dt[p] = dmin / (speed + c);"),
    "residue: outer points counted": (
        "        if (cl->kind[p] == KIND_OUTER && prm->outer_bc != 1) continue;\n        m++;",
        "        m++;\n        if (cl->kind[p] == KIND_OUTER && prm->outer_bc != 1) continue;"),
    "residue: outer points summed": (
        "        if (cl->kind[p] == KIND_OUTER && prm->outer_bc != 1) continue;\n        m++;",
        "        if (cl->kind[p] == KIND_OUTER && prm->outer_bc != 1) {}\n        m++;"),
    "forces: one-sided arc length": ("double ds = 0.5 * (ln + lp);", "double ds = ln;"),
    "forces: sign of the pressure force": (
        "F[h][0] += -(prim[3] - pinf) * cl->nx[p] * ds;",
        "F[h][0] += (prim[3] - pinf) * cl->nx[p] * ds;"),
    "forces: dynamic pressure without 1/2": (
        "double qinf = 0.5 * 1.0 * prm->mach * prm->mach;",
        "double qinf = 1.0 * prm->mach * prm->mach;"),
    "forces: drag rotation": (
        "*cd_out = (Fx * cos(al) + Fy * sin(al)) / qinf;",
        "*cd_out = (Fx * cos(al) - Fy * sin(al)) / qinf;"),
    "forces: lift rotation": (
        "*cl_out = (-Fx * sin(al) + Fy * cos(al)) / qinf;",
        "*cl_out = (Fx * sin(al) + Fy * cos(al)) / qinf;"),
    "limiter: bounds swapped": (
        "double D = (delta > 0.0) ? (qmx - q) : (qmn - q);",
        "double D = (delta > 0.0) ? (qmn - q) : (qmx - q);"),
    "limiter: upper bound always": (
        "double D = (delta > 0.0) ? (qmx - q) : (qmn - q);", "double D = (qmx - q);"),
    "limiter: 2 delta^2 -> delta^2": (
        "double den = D * D + 2.0 * delta * delta + delta * D + eps2;",
        "double den = D * D + delta * delta + delta * D + eps2;"),
    "limiter: 2 delta D -> delta D": (
        "double num = (D * D + eps2) + 2.0 * delta * D;",
        "double num = (D * D + eps2) + delta * D;"),
    "limiter: eps^2 = (K d)^2": ("return e * e * e;", "return e * e;"),
    "limiter: eps from dx only": (
        "double e = K * sqrt(dx * dx + dy * dy);", "double e = K * sqrt(dx * dx);"),
    "eq. (28): bounds swapped in the limited shift": (
        "phi = ora_venkat(d, q[r * n + j], qmax[r * n + j], qmin[r * n + j], eps2);",
        "phi = ora_venkat(d, q[r * n + j], qmin[r * n + j], qmax[r * n + j], eps2);"),
    "eq. (28): sign of the shift": (
        "double d = -0.5 * (dx * g[r * n + j] + dy * g[(4 + r) * n + j]);",
        "double d = 0.5 * (dx * g[r * n + j] + dy * g[(4 + r) * n + j]);"),
    "eq. (28): full instead of half shift": (
        "double d = -0.5 * (dx * g[r * n + j] + dy * g[(4 + r) * n + j]);",
        "double d = -1.0 * (dx * g[r * n + j] + dy * g[(4 + r) * n + j]);"),
    "eq. (28): point's own shift with the neighbour's derivatives": (
        "shifted_q(prm, cl->n, q, g, qmax, qmin, p, dx, dy, qt0);",
        "shifted_q(prm, cl->n, q, g, qmax, qmin, i, dx, dy, qt0); "
        "for (int r = 0; r < 4; ++r) qt0[r] += q[r * cl->n + p] - q[r * cl->n + i];"),
    "outer condition: mirror not applied": (
        "double dn = -(dx * nx + dy * ny);      /* mirrored */",
        "double dn = (dx * nx + dy * ny);      /* mirrored */"),
    "outer condition: entering flux G+ instead of G-": (
        "ora_split_flux(prinf, nx, ny, -1, gamma, Ginf);", "ora_split_flux(prinf, nx, ny, 1, gamma, Ginf);"),
    "outer condition: own state not shifted by the mirrored offset": (
        "shifted_q(prm, n, q, g, qmax, qmin, p, mx, my, qt0);",
        "shifted_q(prm, n, q, g, qmax, qmin, p, dx, dy, qt0);"),
    "outer condition: outer points not updated": (
        "if (cl->kind[p] == KIND_OUTER && prm->outer_bc != 1) continue; /* held */",
        "if (cl->kind[p] == KIND_OUTER) continue; /* held */"),
}


@pytest.mark.parametrize("name", list(PLANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = PLANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"the expression of '{name}' is no longer in the oracle"
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(lib), str(mutant), "-lm"], check=True)
    env = dict(os.environ, QL_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode == 1, f"no pin failed for '{name}':\n{r.stdout[-2000:]}"


def test_unaltered_oracle_passes(tmp_path):
    lib = tmp_path / "libsame.so"
    subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(lib), SRC, "-lm"], check=True)
    env = dict(os.environ, QL_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-2000:]
