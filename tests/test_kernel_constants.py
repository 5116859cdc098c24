"""The polynomial constants hard-coded in the bf16 kernels come from their derivation script (CPU).

sincospi_seed in csrc/basis_gen.h evaluates sin(pi f) and cos(pi f) on |f| <= 1/4 by odd and
even polynomials whose coefficients csrc/fit_sincospi.py derives (least squares, no library
constants).  This test re-runs the fit, checks that the kernel's literals are those coefficients
(to the ten digits printed) and that the fitted polynomials meet the accuracy the recurrence seeds
rely on (below 1e-7 absolute when evaluated in fp32).
"""
import importlib.util
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2307_12041_amd", "csrc")


def _fit_module():
    spec = importlib.util.spec_from_file_location("fit_sincospi", os.path.join(CSRC, "fit_sincospi.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _kernel_literals():
    src = open(os.path.join(CSRC, "basis_gen.h")).read()
    body = src[src.index("void sincospi_seed("):]
    body = body[:body.index("\n}\n")]
    lits = [float(v) for v in re.findall(r"([-+]?\d\.\d+e[-+]\d+)f", body)]
    sp = body[body.index("const float sp"):body.index("const float cp")]
    cp = body[body.index("const float cp"):body.index("const int iq")]
    s = [float(v) for v in re.findall(r"([-+]?\d\.\d+e[-+]\d+)f", sp)]
    c = [float(v) for v in re.findall(r"([-+]?\d\.\d+e[-+]\d+)f", cp)]
    assert len(lits) == len(s) + len(c)
    return s, c


def test_sincospi_seed_constants_match_the_fit():
    fit = _fit_module()
    s_fit, c_fit = fit.fit()
    s_k, c_k = _kernel_literals()
    # Horner order in the kernel: innermost (highest power) first
    assert np.allclose(sorted(s_k), sorted(s_fit), rtol=1e-9, atol=0), (s_k, s_fit)
    assert np.allclose(sorted(c_k), sorted(c_fit), rtol=1e-9, atol=0), (c_k, c_fit)
    assert np.allclose(s_k, list(s_fit[::-1]), rtol=1e-9, atol=0)
    assert np.allclose(c_k, list(c_fit[::-1]), rtol=1e-9, atol=0)
    es, ec = fit.check(s_fit, c_fit)
    assert es < 1e-7 and ec < 1e-7
