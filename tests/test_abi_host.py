"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol of include/bs.h, and derives its parameters as the header states."""
import math
import os
import re
import json

import pytest

from paper_2406_07366_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "bs.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(bs_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 10
    lib = B.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTED) == sorted(names)


def test_header_is_plain_c(tmp_path):
    """The boundary takes no C++ or torch types: the header compiles as
    strict C99, and a C program that calls only host-side entry points
    links against the library."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi.c"
    src.write_text('#include "bs.h"\n#include <stdio.h>\n'
                   "int main(void) {\n"
                   "  bs_params p = {0}, r;\n"
                   "  p.L = 6.283185307179586; p.a = 1e-6; p.tol = 1e-6; p.grid_n = 64;\n"
                   "  int rc = bs_resolve_params(&p, &r);\n"
                   '  printf("%d %d %d\\n", rc, r.K, r.w);\n'
                   "  return rc;\n}\n")
    lib = os.path.dirname(B.LIB_PATH)
    exe = tmp_path / "abi"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                    "-L", lib, "-lbs", "-Wl,-rpath," + lib], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert out == ["0", "20", "8"]


def test_params_struct_matches_header_field_order():
    src = open(os.path.join(ROOT, "include", "bs.h")).read()
    body = src[src.index("typedef struct {"):src.index("} bs_params;")]
    fields = re.findall(r"^\s*(?:double|int|const void \*)\s*(\w+)", body, re.M)
    assert fields == [f for f, _ in B.BsParams._fields_]


def _table1():
    d = json.load(open(os.path.join(ROOT, "tests", "golden", "table1_parameters.json")))
    return d["rows"]


@pytest.mark.parametrize("row", _table1())
def test_beta_and_width_follow_table1(row):
    """Sec. 5.3, Table 1: beta and w per nominal tolerance (sigma = 1.5)."""
    tol, beta, _, sigma, w = row[:5]
    r = B.resolve_params(B.make_params(L=2 * math.pi, a=1e-6, tol=tol, grid_n=512))
    assert (r.beta, r.sigma, r.w) == (beta, sigma, w)


@pytest.mark.parametrize("tol,beta,w", [(1e-5, 3.5, 7), (3e-4, 2.5, 5), (1e-7, 4.0, 9),
                                        (1e-15, 5.5, 16), (0.5, 2.0, 4)])
def test_tolerances_between_table_rows(tol, beta, w):
    """Between Table 1 rows: beta of the row with the largest tolerance <= tol,
    w from the App. A decay 10^(-0.9 w) <= tol, ceil(-log10(tol)/0.9) + 1,
    clamped to 4..16."""
    r = B.resolve_params(B.make_params(L=2 * math.pi, a=1e-6, tol=tol, grid_n=512))
    assert (r.beta, r.w) == (beta, w)


def test_derived_parameters_of_the_workloads():
    L = 2 * math.pi
    # 64-node ring: n = 32 -> M = 21, K = 10, beta = 3.5 (tol 1e-6)
    r = B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-6, grid_n=32))
    assert (r.K, r.w, r.beta) == (10, 8, 3.5)
    assert math.isclose(r.alpha, 10 / 7, rel_tol=1e-14)          # K (2pi/L)/(2 beta)
    assert math.isclose(r.rcut, r.beta / r.alpha, rel_tol=1e-14)
    assert r.rcut <= L / 2
    assert r.ncell == 1                                           # 3 L / (2 r_c) < 4
    # 40 ellipses: n = 64 -> K = 20
    r = B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-6, grid_n=64))
    assert (r.K, r.w) == (20, 8) and math.isclose(r.alpha, 20 / 7, rel_tol=1e-14)
    assert r.ncell == 7                                           # edge >= 2 r_c / 3
    assert L / r.ncell >= 2 * r.rcut / 3
    # tangle: n = 256, tol 1e-5 -> beta 3.5 (next accurate-enough row), w = 7
    r = B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-5, grid_n=256))
    assert (r.K, r.w, r.beta) == (84, 7, 3.5)
    # k_max = 2 beta alpha (Sec. 4)
    assert math.isclose(2 * r.beta * r.alpha, r.K * 2 * math.pi / L, rel_tol=1e-14)
    # Kaiser-Bessel shape parameter zeta = 0.995 w pi (1 - 1/(2 sigma)) (App. A)
    assert math.isclose(r.zeta, 0.995 * 7 * math.pi * (1 - 1 / 3), rel_tol=1e-14)


def test_parameter_errors():
    L = 2 * math.pi
    with pytest.raises(B.BsError) as e:
        B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-6, grid_n=16))
    assert e.value.code == B.BS_ETOL                 # would need r_c > L/2
    with pytest.raises(B.BsError) as e:
        B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-6, grid_n=64, alpha=1.0, rcut=4.0))
    assert e.value.code == B.BS_EMINIMG
    for bad in (dict(grid_n=30), dict(grid_n=64, Q=5), dict(grid_n=64, w=20),
                dict(grid_n=64, sigma=0.9)):
        with pytest.raises(B.BsError) as e:
            B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-6, **bad))
        assert e.value.code == B.BS_EINVAL
    with pytest.raises(B.BsError) as e:
        B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-6, grid_n=1024, sigma=1.0001))
    assert e.value.code == B.BS_EKB
    B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-6, grid_n=64, spline_order=6,
                                   local_frac=0.1))
    for bad in (dict(spline_order=5), dict(spline_order=6, ns_mode=B.BS_NS_MLP),
                dict(local_frac=1.5), dict(local_frac=-0.1), dict(local_frac=1e-4)):
        with pytest.raises(B.BsError) as e:
            B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-6, grid_n=64, **bad))
        assert e.value.code == B.BS_EINVAL


def test_pruned_transforms_need_a_power_of_two_grid():
    L = 2 * math.pi
    B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-6, grid_n=64, fft_mode=B.BS_FFT_PRUNED))
    with pytest.raises(B.BsError) as e:
        B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-6, grid_n=48, fft_mode=B.BS_FFT_PRUNED))
    assert e.value.code == B.BS_EINVAL
    with pytest.raises(B.BsError):
        B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-6, grid_n=64, fft_mode=7))
    # two LDS buffers of the z pass must hold 3 columns + pad: float64 up to 512
    B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-5, grid_n=1024, fft_mode=B.BS_FFT_PRUNED,
                                   precision=B.BS_FP32_MIXED))
    with pytest.raises(B.BsError):
        B.resolve_params(B.make_params(L=L, a=1e-6, tol=1e-5, grid_n=1024,
                                       fft_mode=B.BS_FFT_PRUNED))
