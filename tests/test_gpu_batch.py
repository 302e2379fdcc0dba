"""Batched solves (mgrit_solve_batch) on the GPU.

Several plans on one stream are stepped together and launches of the same
kernel and shape are merged into one grid.  Every block of a merged launch
runs the same code on its own plan's arguments as in a launch of its own,
so each result must equal mgrit_solve's on the same plan and inputs bit for
bit: residual histories, iteration counts and outputs.  Members that stop
early (converged, out of iterations) leave the batch while the others go on.
"""

import numpy as np
import pytest
import torch

from oracle import rk
from paper_1910_03726_amd import inputs, mgrit as M

pytestmark = pytest.mark.gpu


def _plan(scheme, nx, nt, m, levels, frac, precision="fp64", relax="FCF", cycle="V"):
    c = rk.paper_cfl(scheme, frac) if scheme.startswith("ERK") else frac
    psi, _ = M.psi_optimize(scheme, c, nx, m, levels)
    return M.Plan(nx, nt, c, scheme, m, levels, psi, precision=precision, relax=relax,
                  cycle=cycle)


def _u0(nx, seed):
    return torch.tensor(inputs.fourier_u0(nx, 6, seed), device="cuda")


def _alone(P, u0, seed, tol, maxit, out):
    P.set_seed(seed)
    return P.solve(u0, None, tol=tol, maxit=maxit, out=out)


def _check_same(a, b):
    assert a.status == b.status
    assert a.iters == b.iters
    assert a.hist == b.hist  # bit for bit
    if a.out is not None:
        assert torch.equal(a.out, b.out)


CASES = {
    # same shape: every relaxation pass merges
    "same_shape": [("ERK3", 1024, 2048, 4, 3, 0.55), ("ERK3", 1024, 2048, 4, 3, 0.7),
                   ("ERK3", 1024, 2048, 4, 3, 0.85), ("ERK3", 1024, 2048, 4, 3, 0.62)],
    # different schemes, sizes and depths: merged only where shapes agree
    "mixed": [("ERK1", 512, 4096, 4, 4, 0.8), ("ERK5", 2048, 1024, 8, 3, 0.6),
              ("ERK3", 512, 4096, 4, 4, 0.75), ("SDIRK3", 1024, 1024, 4, 3, 4.0),
              ("ERK1", 512, 4096, 4, 4, 0.6)],
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("precision,relax,cycle", [("fp64", "FCF", "V"), ("fp64", "FCF", "F"),
                                                   ("fp32", "FCF", "V"), ("fp32", "F", "V")])
def test_batch_equals_solo(case, precision, relax, cycle):
    specs = CASES[case]
    plans = [_plan(*s, precision=precision, relax=relax, cycle=cycle) for s in specs]
    try:
        u0s = [_u0(s[1], 100 + i) for i, s in enumerate(specs)]
        seeds = [7 + 11 * i for i in range(len(specs))]
        solo = [_alone(P, u, sd, 1e-10, 60, "final") for P, u, sd in zip(plans, u0s, seeds)]
        for P, sd in zip(plans, seeds):
            P.set_seed(sd)
        batch = M.solve_batch(plans, u0s, tol=1e-10, maxit=60, out="final")
        for a, b in zip(solo, batch):
            _check_same(a, b)
            assert a.status == M.OK
        merged = [P.stats().batched_launches for P in plans]
        if case == "same_shape":
            assert min(merged) > 0
    finally:
        for P in plans:
            P.close()


def test_members_stop_at_different_iterations():
    """One member runs out of iterations, one converges loosely early, one
    converges tightly: each as when solved alone."""
    specs = [("ERK3", 1024, 2048, 4, 3, 0.85)] * 3
    plans = [_plan(*s) for s in specs]
    try:
        u0s = [_u0(1024, 5 + i) for i in range(3)]
        tols, maxits = [1e-10, 1e-4, 1e-12], [2, 60, 60]
        solo = []
        for P, u, t, mi in zip(plans, u0s, tols, maxits):
            solo.append(_alone(P, u, 3, t, mi, "cpoints"))
        for P in plans:
            P.set_seed(3)
        batch = M.solve_batch(plans, u0s, tol=tols, maxit=maxits, out="cpoints")
        assert [r.status for r in batch] == [M.ENOTCONV, M.OK, M.OK]
        assert batch[1].iters < batch[2].iters
        for a, b in zip(solo, batch):
            _check_same(a, b)
    finally:
        for P in plans:
            P.close()


def test_all_outputs_and_one_member():
    P = _plan("ERK3", 512, 1024, 4, 3, 0.8)
    try:
        u0 = _u0(512, 1)
        a = _alone(P, u0, 9, 1e-11, 40, "all")
        P.set_seed(9)
        (b,) = M.solve_batch([P], [u0], tol=1e-11, maxit=40, out="all")
        _check_same(a, b)
        assert P.stats().batched_launches == 0
    finally:
        P.close()


def test_invalid_batches():
    P = _plan("ERK1", 256, 1024, 4, 2, 0.8)
    s = torch.cuda.Stream()
    c = rk.paper_cfl("ERK1", 0.8)
    psi, _ = M.psi_optimize("ERK1", c, 256, 4, 2)
    Q = M.Plan(256, 1024, c, "ERK1", 4, 2, psi, stream=s.cuda_stream)
    try:
        u0 = _u0(256, 2)
        with pytest.raises(M.MgritError):
            M.solve_batch([P, Q], [u0, u0])  # two streams
        with pytest.raises(M.MgritError):
            M.solve_batch([P, P], [u0, u0])  # one plan twice
    finally:
        P.close()
        Q.close()
