"""The oracle's pins must catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of the oracle's C source (a wrong constant, a dropped
term, a flipped sign, a swapped axis, a wrong index), builds it, and runs the pin suite
against the broken copy in a subprocess.  The suite must fail for every mutant.  The real
oracle is never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pp_oracle.c")

MUTANTS = {
    "a_up constant 4 -> 2": ("return 4.0 * W * W * H * H /", "return 2.0 * W * W * H * H /"),
    "a_u0 constant 2 -> 4": ("if (p == 0) return 2.0 * W * W /", "if (p == 0) return 4.0 * W * W /"),
    "a_0p uses W^2 for H^2": ("if (u == 0) return 2.0 * H * H /", "if (u == 0) return 2.0 * W * W /"),
    "a_up denominator swaps W and H": ("(((double)u * u * H * H + (double)p * p * W * W) * (double)u",
                                       "(((double)u * u * W * W + (double)p * p * H * H) * (double)u"),
    "moment factor of the u-row": ("if (p == 0) return W / ((double)u * pi);",
                                   "if (p == 0) return H / ((double)u * pi);"),
    "energy drops the one half": ("return (double)(0.5L * e);", "return (double)(e);"),
    "half width taken as full width": ("sincos_kpi(k, centre - size / 2.0, L, &sm, &cm);",
                                       "sincos_kpi(k, centre - size, L, &sm, &cm);"),
    "cosine difference sign": ("*K = cp - cm;", "*K = cm - cp;"),
    "gradient uses the wrong axis integral": ("sx += Kx[u] * zy;", "sx += Kx[u] * zl;"),
    "mean not removed (a_00 kept)": ("if (u == 0 && p == 0) return 0.0;\n    if (p == 0) return 2.0",
                                     "if (u == 0 && p == 0) return 1e-3;\n    if (p == 0) return 2.0"),
    "u=0 column integral uses height": ("Sc[j * Mu + 0] = w[i];", "Sc[j * Mu + 0] = h[i];"),
    "frequency off by one": ("edge_diffs(u, x[i], w[i], W, &S, &K); Sc[j * Mu + u] = S;",
                             "edge_diffs(u + 1, x[i], w[i], W, &S, &K); Sc[j * Mu + u] = S;"),
    "point field drops the frequency factor": ("ex += ((double)u * ORACLE_PI / W) * su[u] * zc;",
                                               "ex += su[u] * zc;"),
    "bin centre without the half bin": ("long q = (k * (2 * s + 1)) % (4 * m);", "long q = (k * (2 * s)) % (4 * m);"),
    "bin a_up constant 16 -> 8": ("return 16.0 * W * W * H * H /", "return 8.0 * W * W * H * H /"),
    "bin sine factor uses pi/m": ("sin(u * pi / (2.0 * m)) * sin(p * pi / (2.0 * m));",
                                  "sin(u * pi / (1.0 * m)) * sin(p * pi / (2.0 * m));"),
    "bin density over the bin width only": ("P[k] = (double)(acc[k] / ((long double)wb * hb));",
                                            "P[k] = (double)(acc[k] / ((long double)wb));"),
    "bin field xi_y uses the x frequency": ("ey += (long double)((double)p * pi / H) * apu * cu[u] * sp[p];",
                                            "ey += (long double)((double)u * pi / W) * apu * cu[u] * sp[p];"),
    "bin interpolation swaps the bin axes": ("const size_t b = (size_t)l * m + j;", "const size_t b = (size_t)j * m + l;"),
    "bin interpolation drops the gradient sign": ("if (xix) gx[i] = (double)-sx;", "if (xix) gx[i] = (double)sx;"),
    "bin interpolation area uses the width twice": ("const long double area = (long double)ox * oy;",
                                                    "const long double area = (long double)ox * ox;"),
    "sampled absolute sums lose the absolute value": ("sa += fabsl((long double)Sx * (long double)Ty);",
                                                      "sa += (long double)Sx * (long double)Ty;"),
    "block potential y integral": ("for (int p = 0; p < Mp; ++p) Yb[p] = edge_integral(p, y[i], h[i], H);",
                                   "for (int p = 0; p < Mp; ++p) Yb[p] = edge_integral(p, y[i], w[i], H);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {old!r}"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", str(msrc), "-o", str(lib), "-lm"],
                   check=True)
    env = dict(os.environ, PP_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch mutant '{name}':\n{r.stdout[-2000:]}"
