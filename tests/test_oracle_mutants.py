"""The oracle's pins catch plausible mistakes.  Each case copies the oracle,
plants one mistake in the copy's C source (a transposed operand, a wrong index,
a dropped term, a flipped sign, the wrong Piola map, swapped spaces, the wrong
stress or strain product), and runs
the CPU pin suites against the copy in a subprocess: at least one pin must
fail.  An unmodified copy must pass the same suites (control).  The mistakes
are planted only in temporary copies; the repository's oracle is untouched.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("s += G[b][a] * g[b]; /* (G^T grad^)_a */", "s += G[a][b] * g[b];", "G transposed"),
    ("o[3] = (g[0] + g[4] + g[8]) / det;", "o[3] = (g[0] + g[4]) / det;", "div: dropped term"),
    ("cr[1] = g[3 * 0 + 2] - g[3 * 2 + 0];", "cr[1] = g[3 * 2 + 0] - g[3 * 0 + 2];", "curl: flipped sign"),
    ("s += G[c][a] * v[c];", "s += J[a][c] * v[c];", "H(curl): contravariant instead of covariant"),
    ("int pk_axis = (family == ORC_NCF) ? (a == c) : (a != c);",
     "int pk_axis = (family == ORC_NCF) ? (a != c) : (a == c);", "NCF/NCE spaces swapped"),
    ("J[a][b] += X[v * 3 + a] * dphi[b];", "J[a][b] += X[v * 3 + b] * dphi[a];", "J transposed"),
    ("*w = s->wq[q0] * s->wq[q1] * s->wq[q2];", "*w = s->wq[q0] * s->wq[q1] * s->wq[q1];", "weight: wrong index"),
    ("double term = 1.0 / (nodes[i] - nodes[k]);", "double term = 1.0 / (nodes[k] - nodes[i]);",
     "Lagrange derivative: flipped sign"),
    ("for (int k = 0; k < 3; ++k) t += F[a][k] * S[k][b];", "for (int k = 0; k < 3; ++k) t += S[a][k] * F[k][b];",
     "SVK: P = S F instead of F S"),
    ("c += F[k][a] * F[k][b]; /* C = F^T F */", "c += F[a][k] * F[b][k];", "SVK: F F^T instead of F^T F"),
    ("dS[a][b] = (a == b ? lambda * trdE : 0.0) + 2.0 * mu * dE[a][b];", "dS[a][b] = 2.0 * mu * dE[a][b];",
     "SVK linearisation: dropped lambda term"),
    ("t += dH[k][a] * F[k][b] + F[k][a] * dH[k][b];", "t += dH[a][k] * F[b][k] + F[a][k] * dH[b][k];",
     "SVK linearisation: transposed dE"),
    ("for (int b = 0; b < 3; ++b) s += g[3 * c + b] * G[b][a]; /* d v_c / d x_a */",
     "for (int b = 0; b < 3; ++b) s += g[3 * c + b] * G[a][b];", "vector element: G transposed"),
    ("e->b[c].offset = c * n * n * n;", "e->b[c].offset = 0;", "vector element: blocks overlap"),
    ("mu * (FFt[c][cc] * (e == ee ? 1.0 : 0.0) + F[c][ee] * F[cc][e]);",
     "mu * (FFt[c][cc] * (e == ee ? 1.0 : 0.0) + F[c][e] * F[cc][ee]);", "SVK tangent: swapped indices"),
]
PIN_SUITES = [os.path.join(ROOT, "tests", "test_oracle_pins.py"), os.path.join(ROOT, "tests", "test_golden.py"),
              os.path.join(ROOT, "tests", "test_oracle_svk.py"), os.path.join(ROOT, "tests", "test_oracle_vq.py")]


def run_pins_against_copy(tmp_path, old=None, new=None):
    dst = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    if old is not None:
        src = (dst / "sf_oracle.c").read_text()
        assert src.count(old) == 1, "mutation anchor not found: %s" % old
        (dst / "sf_oracle.c").write_text(src.replace(old, new))
    env = dict(os.environ)
    # the copy shadows the repository's oracle; the repository still provides the tests' helpers
    env["PYTHONPATH"] = os.pathsep.join([str(tmp_path), ROOT])
    which = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.__file__)"], cwd=str(tmp_path),
                           env=env, capture_output=True, text=True, timeout=60)
    assert which.stdout.strip().startswith(str(dst)), which.stdout + which.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "--import-mode=append",
                        "-m", "not gpu"]
                       + PIN_SUITES, cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=600)
    return r


def test_unmodified_copy_passes(tmp_path):
    r = run_pins_against_copy(tmp_path)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


@pytest.mark.parametrize("old,new,name", MUTANTS, ids=[m[2] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, old, new, name):
    r = run_pins_against_copy(tmp_path, old, new)
    assert r.returncode != 0 and "failed" in r.stdout, (name, r.stdout[-2000:])
