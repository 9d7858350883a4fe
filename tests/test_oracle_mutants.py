"""Planted mistakes in the oracle must fail its pins (CPU only).

Each mutant is oracle/fea_oracle.c with one plausible mistake (a dropped
term, a wrong sign, factor or index, a transposed operand, a skipped
colour), compiled on its own. The oracle's pins (tests/test_oracle.py) then
run against it in a process of their own, with FEA_ORACLE_LIB naming the
mutant library, and at least one pin must fail. A mutant that every pin
accepted would be a mistake the pins cannot see. The unmodified source,
built the same way, must pass them all.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fea_oracle.c")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")

# (name, text of the source, its replacement): each text occurs once
MUTANTS = [
    ("geometry: J^-1 transposed in grad N = J^-T grad_xi N",
     "acc += Ji[j][i] * dN[3 * a + j];", "acc += Ji[i][j] * dN[3 * a + j];"),
    ("geometry: sign of a cofactor in det J",
     "- A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])", "+ A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])"),
    ("Gauss rule: hexahedron points at 1/sqrt(2)",
     "const double g = 1.0 / sqrt(3.0);", "const double g = 1.0 / sqrt(2.0);"),
    ("Gauss rule: prism weights 1/3",
     "                w[q] = 1.0 / 6.0;", "                w[q] = 1.0 / 3.0;"),
    ("shape functions: prism t-derivative halved",
     "dN[3 * a + 2] = L[k] * dg;", "dN[3 * a + 2] = L[k] * dg * 0.5;"),
    ("shape functions: pyramid apex derivative 1/4",
     "dN[12] = 0.0; dN[13] = 0.0; dN[14] = 0.5;", "dN[12] = 0.0; dN[13] = 0.0; dN[14] = 0.25;"),
    ("Poisson: G_a . G_a instead of G_a . G_b",
     "double t = wd * G[a][k] * G[b][k];", "double t = wd * G[a][k] * G[a][k];"),
    ("elasticity: shear term with swapped indices",
     "double t2 = wd * mu * G[a][j] * G[b][i];", "double t2 = wd * mu * G[a][i] * G[b][j];"),
    ("elasticity: lambda term dropped",
     "double v = t1 + t2 + (i == j ? dot : 0.0);", "double v = t2 + (i == j ? dot : 0.0);"),
    ("elasticity: lambda with (1 - nu) for (1 - 2 nu)",
     "(1.0 - 2.0 * nu)", "(1.0 - nu)"),
    ("right-hand side: first source component for every component",
     "double t = wd * N[a] * f[i];", "double t = wd * N[a] * f[0];"),
    ("neo-Hookean tangent: identity part paired i-J, j-L",
     "AA[i][J][j][L] = mu * (i == j) * (J == L)", "AA[i][J][j][L] = mu * (i == J) * (j == L)"),
    ("neo-Hookean tangent: lambda part with transposed F^-1 indices",
     "+ lam * Fi[J][i] * Fi[L][j];", "+ lam * Fi[J][j] * Fi[L][i];"),
    ("neo-Hookean stress: sign of the lambda ln J term",
     "P[i][J] = mu * (F[i][J] - Fi[J][i]) + lam * lnJ * Fi[J][i];",
     "P[i][J] = mu * (F[i][J] - Fi[J][i]) - lam * lnJ * Fi[J][i];"),
    ("|term| sums: lambda term counted twice (elasticity)",
     "fabs(t1) + fabs(t2) + (i == j ? tdot : 0.0);", "2.0 * fabs(t1) + fabs(t2) + (i == j ? tdot : 0.0);"),
    ("|term| sums: third tangent part counted twice (neo-Hookean)",
     "+ fabs(lam * Fi[J][i] * Fi[L][j]));", "+ 2.0 * fabs(lam * Fi[J][i] * Fi[L][j]));"),
    ("graph: repeated columns kept in a row",
     "if (out == 0 || buf[p] != buf[out - 1]) buf[out++] = buf[p];", "buf[out++] = buf[p];"),
    ("graph: element-to-nonzero map transposed",
     "e2nnz[map_ptr[e] + a * nn + b] = (int32_t)found;", "e2nnz[map_ptr[e] + b * nn + a] = (int32_t)found;"),
    ("colouring: the previous element's colour ignored",
     "if (o < e) used[colour[o]] = 1;", "if (o < e - 1) used[colour[o]] = 1;"),
    ("assembly: right-hand side overwritten instead of added",
     "rhs[(int64_t)r * B + i] += fe[a * B + i];", "rhs[(int64_t)r * B + i] = fe[a * B + i];"),
    ("colour timing variant: last colour skipped",
     "for (c = 0; c < n_colours; ++c) {", "for (c = 0; c + 1 < n_colours; ++c) {"),
    ("residual: internal force added instead of subtracted",
     "rhs[(int64_t)r * 3 + i] += fe[3 * a + i] - fint[3 * a + i];",
     "rhs[(int64_t)r * 3 + i] += fe[3 * a + i] + fint[3 * a + i];"),
    ("subgrid scale: geometric second-derivative term dropped",
     "for (k = 0; k < 3; ++k) acc -= gu[c][k] * Hx_geo[k][j][l];", ";"),
    ("subgrid scale: lambda for lambda + mu in grad div",
     "(lam + mu) * gdiv", "lam * gdiv"),
    ("subgrid scale: h for h^2 in tau",
     "double tau = h * h / (4.0 * ", "double tau = h / (4.0 * "),
    ("subgrid scale: pyramid mixed second derivative doubled",
     "H[0][1] = H[1][0] = sx * sy * fz / 8.0;", "H[0][1] = H[1][0] = sx * sy * fz / 4.0;"),
]

ORIGINAL = "unmodified source"


def _compile(src_text, path):
    c_path = path + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    p = subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                        "-o", path, c_path, "-lm"], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    return p.returncode, p.stdout


def _pins(lib_path):
    env = dict(os.environ, FEA_ORACLE_LIB=lib_path, OMP_NUM_THREADS="2")
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=600)
    return p.returncode, p.stdout


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    """Every mutant (and the unmodified source) compiled and run against the
    pins, eight at a time: name -> (compile rc, pins rc, pins output)."""
    with open(SRC) as f:
        src = f.read()
    d = tmp_path_factory.mktemp("oracle_mutants")
    jobs = {ORIGINAL: src}
    for k, (name, old, new) in enumerate(MUTANTS):
        assert src.count(old) == 1, name
        jobs[name] = src.replace(old, new)

    def run(item):
        k, (name, text) = item
        lib = str(d / f"mutant{k}.so")
        crc, cout = _compile(text, lib)
        if crc != 0:
            return name, (crc, None, cout)
        prc, pout = _pins(lib)
        return name, (crc, prc, pout)

    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as pool:
        return dict(pool.map(run, enumerate(jobs.items())))


def test_unmodified_oracle_passes_the_pins(outcomes):
    crc, prc, out = outcomes[ORIGINAL]
    assert crc == 0, out[-2000:]
    assert prc == 0, out[-2000:]


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(outcomes, name):
    crc, prc, out = outcomes[name]
    assert crc == 0, out[-2000:]
    # pytest exits with 1 when a test failed (not 0: passed, not 2+: error)
    assert prc == 1 and " failed" in out, out[-2000:]
