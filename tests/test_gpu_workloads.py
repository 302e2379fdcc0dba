"""The four single-solve workloads at full size, in the launch configuration
bench.py times, checked against the oracle on outputs it can compute one by
one: the first 16 C-points by sequential stage-by-stage stepping, and
C-points spread over the whole time range (a quarter, half, three quarters
and the final time) by the extended-precision closed form of Lemma 1 -- the
exact discrete solution MGRIT converges to (Sec. 2.2) -- plus conservation
of the mean (the theta = 0 eigenvalue of every stepper is 1).  Solves run to
tol 1e-14 so that the converged iterate's error |A^-1| |r| is far below the
1e-12 relative bar.
"""

import numpy as np
import pytest
import torch

from oracle import rk
from paper_1910_03726_amd import inputs, mgrit as M

pytestmark = pytest.mark.gpu


def _run(name, precision=None, tol=1e-13, maxit=60, psi_rule=None):
    w = dict(inputs.WORKLOADS[name])
    if psi_rule:
        w["psi_rule"] = psi_rule
    psi, mi = M.workload_psi(w)
    assert mi < 1e-8
    u0 = inputs.workload_u0(w)
    nc = w["nt"] // w["m"]
    uinit = inputs.random_iterate(nc + 1, w["nx"], w["init_seed"])
    dev = "cuda:0"
    with M.Plan(w["nx"], w["nt"], w["cfl"], w["scheme"], w["m"], w["levels"], psi,
                cycle=w["cycle"], precision=precision or w["precision"]) as P:
        r = P.solve(torch.tensor(u0, device=dev), torch.tensor(uinit, device=dev), tol=tol,
                    maxit=maxit, out="cpoints")
        desc = P.describe()
    return w, u0, r, r.out.cpu().numpy(), desc


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("name,precision", [
    ("erk1_u1_nx64_nt256_m4_2level", None),
    ("erk3_u3_nx4096_nt16384_m8_fcycle", None),
    ("sdirk3_u3_nx2048_nt8192_m16_2level", None),
    ("erk5_u5_nx8192_nt65536_m8_fp32relax", None),      # FP32 relaxation form
    ("erk5_u5_nx8192_nt65536_m8_fp32relax", "fp64"),
])
def test_workload_parity(name, precision):
    tol, rel = 1e-14, 1e-12
    w, u0, r, C, desc = _run(name, precision, tol)
    assert r.converged, r.hist
    d = rk.Discretization(w["scheme"], w["nx"], w["cfl"])
    m, nc = w["m"], C.shape[0] - 1
    k = min(16, nc)
    early = d.time_stepping(u0, k * m, every=m)
    errs = {"first16": _rel(C[:k + 1], early)}
    for j in sorted({nc // 4, nc // 2, 3 * nc // 4, nc}):
        errs[j] = _rel(C[j], d.spectral_propagate(u0, j * m))
    print(name, precision, r.iters, r.hist[-1], desc, errs)
    assert max(errs.values()) < rel, errs
    # mean conservation at every C-point
    means = C.sum(axis=1)
    assert np.max(np.abs(means - u0.sum())) < 1e-9 * np.abs(u0).sum()


def test_paper_iteration_counts():
    # Two-level counts printed in the paper for these discretizations:
    # ERK1+U1 m = 4: 6 (Table 3); SDIRK3+U3 m = 16: 4 (Table 6).
    _, _, r, _, _ = _run("erk1_u1_nx64_nt256_m4_2level", tol=1e-10)
    assert r.iters == 6
    _, _, r, _, _ = _run("sdirk3_u3_nx2048_nt8192_m16_2level", tol=1e-10)
    assert r.iters == 4


@pytest.mark.parametrize("name", ["erk3_u3_nx4096_nt16384_m8_fcycle",
                                  "erk5_u5_nx8192_nt65536_m8_fp32relax"])
def test_bound_rule_beats_the_width_rule(name):
    # windows widened until the eq. (7) bound reaches 1e-3 need fewer
    # iterations than the Sec. 4.4 width rule, to the same solution
    wb, u0, rb, Cb, _ = _run(name, tol=1e-10, psi_rule="bound")
    ww, _, rw, Cw, _ = _run(name, tol=1e-10, psi_rule="window")
    print(name, "bound", rb.iters, "window", rw.iters)
    assert rb.converged and rw.converged
    assert rb.iters < rw.iters
    assert _rel(Cb[-1], Cw[-1]) < 1e-6

