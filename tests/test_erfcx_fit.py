"""The pair kernel's short-range factor g(x) = erfc(x) + (2/sqrt(pi)) x e^{-x^2}
(eq:velocity_shortrange) is formed as e^{-x^2} (erfcx(x) + (2/sqrt(pi)) x)
with erfcx from the polynomial table in csrc/erfcx_fit.h.  This test reads
the table, evaluates it the way the kernel does (float64 Horner in
Z = (4 - x) / (4 + x)) and checks it against scipy's erfcx and erfc, and
that the header is what its generator script writes."""
import math
import os
import re
import subprocess
import sys

import numpy as np
from scipy.special import erfc, erfcx

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2406_07366_amd", "csrc")


def table():
    src = open(os.path.join(CSRC, "erfcx_fit.h")).read()
    shift = float(re.search(r"kErfcxShift = ([^;]+);", src).group(1))
    body = re.search(r"kErfcxP\[kErfcxDeg \+ 1\] = \{([^}]*)\}", src).group(1)
    coef = [float(v) for v in body.replace("\n", " ").split(",") if v.strip()]
    deg = int(re.search(r"kErfcxDeg = (\d+);", src).group(1))
    assert len(coef) == deg + 1
    return shift, coef


def erfcx_kernel(x):
    shift, coef = table()
    inv = 1.0 / (shift + x)
    z = (shift - x) * inv
    p = np.full_like(x, coef[-1])
    for c in coef[-2::-1]:
        p = p * z + c
    return p * inv


def test_table_matches_erfcx():
    x = np.linspace(0.0, 6.0, 200001)
    assert np.abs(erfcx_kernel(x) / erfcx(x) - 1).max() < 1e-14
    far = np.logspace(np.log10(6.0), 6, 20001)
    assert np.abs(erfcx_kernel(far) / erfcx(far) - 1).max() < 2e-13


def table32():
    src = open(os.path.join(CSRC, "erfcx_fit.h")).read()
    body = re.search(r"kErfcxP32\[kErfcxDeg32 \+ 1\] = \{([^}]*)\}", src).group(1)
    return [np.float32(v.strip().rstrip("f")) for v in body.replace("\n", " ").split(",")
            if v.strip()]


def test_float32_table_matches_erfcx():
    # the float32 kernel's evaluation: float32 reciprocal, Z and Horner
    f = np.float32
    shift, _ = table()
    coef = table32()
    x = np.linspace(0.0, 6.0, 200001).astype(f)
    inv = (f(1.0) / (f(shift) + x)).astype(f)
    z = ((f(shift) - x) * inv).astype(f)
    p = np.full_like(z, coef[-1])
    for c in coef[-2::-1]:
        p = (p * z + c).astype(f)
    got = (p * inv).astype(np.float64)
    assert np.abs(got / erfcx(x.astype(np.float64)) - 1).max() < 1e-6


def test_short_range_factor():
    x = np.linspace(0.0, 6.0, 100001)
    ref = erfc(x) + 2 / math.sqrt(math.pi) * x * np.exp(-x * x)
    got = np.exp(-x * x) * (erfcx_kernel(x) + 2 / math.sqrt(math.pi) * x)
    assert np.abs(got / ref - 1).max() < 1e-14


def test_header_is_the_generators_output():
    # the same coefficients (to the least-squares solver's rounding)
    out = subprocess.run([sys.executable, os.path.join(CSRC, "erfcx_fit.py")],
                         capture_output=True, text=True, check=True).stdout
    body = re.search(r"kErfcxP\[kErfcxDeg \+ 1\] = \{([^}]*)\}", out).group(1)
    fresh = np.array([float(v) for v in body.replace("\n", " ").split(",") if v.strip()])
    _, coef = table()
    assert np.allclose(fresh, coef, rtol=1e-9, atol=1e-15)
