"""Accuracy across the paper's tolerance settings (Sec. 5.3, Table 1): for
each nominal tolerance, the plan derives beta and the kernel width w from it
(sigma = 1.5), and the FP64 velocity of the 40-ellipse workload must meet that
tolerance against the converged oracle (the stored reference, beta = 6.5)."""
import json
import math
import os

import numpy as np
import pytest

from paper_2406_07366_amd import workloads as W

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rows():
    d = json.load(open(os.path.join(ROOT, "tests", "golden", "table1_parameters.json")))
    return [dict(zip(d["columns"], r)) for r in d["rows"]]


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_07366_amd import binding
    return binding


@pytest.fixture(scope="module")
def ref():
    z = np.load(os.path.join(ROOT, "tests", "golden", "ref_ellipses.npz"))
    return z["v"]


def rel_l2(a, b):
    return math.sqrt(((a - b) ** 2).sum(1).mean() / (b ** 2).sum(1).mean())


@pytest.mark.parametrize("row", _rows(), ids=lambda r: f"tol{r['tol']:g}")
def test_velocity_meets_nominal_tolerance(B, ref, row):
    fs = W.ellipses()
    fs.tol = row["tol"]
    print(f"\n[case] ellipses tol {row['tol']:g}", flush=True)
    plan = B.Plan(B.params_for(fs))
    p = plan.params()
    assert (p.beta, p.w) == (row["beta"], row["w"])
    xyz, g = B.load_workload(fs)
    plan.set_filaments(fs.offsets, xyz, g)
    v = plan.velocity().cpu().numpy()
    plan.status()
    plan.close()
    err = rel_l2(v, ref)
    print(f"  beta {p.beta} w {p.w} alpha {p.alpha:.4f} r_c {p.rcut:.4f}: rel_l2 {err:.2e}")
    # the float64 evaluation and the reference's own rounding floor
    assert err <= max(row["tol"], 2e-13)
