"""Edge cases of the GPU path: empty and one-step batches, the smallest and
largest spatial sizes, ragged n_x, iteration limits, an exact initial
iterate, and divergence."""

import numpy as np
import pytest
import torch

from oracle import rk
from paper_1910_03726_amd import inputs, mgrit as M

pytestmark = pytest.mark.gpu


def _psi(scheme, c, nx, m, levels):
    psi, _ = M.psi_optimize(scheme, c, nx, m, levels)
    return psi


def test_phi_apply_batch_empty_zero_and_one_step():
    c = rk.paper_cfl("ERK3")
    with M.Plan(256, 8, c, "ERK3", 4, 2, _psi("ERK3", c, 256, 4, 2)) as P:
        x = torch.tensor(np.stack([inputs.fourier_u0(256, 4, s) for s in range(3)]),
                         device="cuda")
        out = torch.full_like(x, 7.0)
        P.phi_apply_batch(x[:0], out[:0], 3)  # nothing to do
        torch.cuda.synchronize()
        assert torch.all(out == 7.0)
        P.phi_apply_batch(x, out, 0)  # zero steps: a copy
        torch.cuda.synchronize()
        assert torch.equal(out, x)
        P.phi_apply_batch(x, out, 1)
        torch.cuda.synchronize()
    d = rk.Discretization("ERK3", 256, c)
    ref = np.stack([d.step(r) for r in x.cpu().numpy()])
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("scheme,nx,nt,m,levels", [
    ("ERK1", 16, 8, 2, 2),       # smallest: generic kernel, 4 coarse intervals
    ("ERK3", 192, 768, 4, 3),    # n_x a multiple of 64, not a power of two
    ("ERK1", 16384, 64, 4, 2),   # largest register-resident line (K = 32, 512 lanes)
])
def test_extreme_sizes_match_sequential_stepping(scheme, nx, nt, m, levels):
    c = rk.paper_cfl(scheme)
    u0 = inputs.fourier_u0(nx, 3, 4)
    with M.Plan(nx, nt, c, scheme, m, levels, _psi(scheme, c, nx, m, levels)) as P:
        r = P.solve(torch.tensor(u0, device="cuda"), None, tol=1e-13, maxit=nt, out="final")
    assert r.status == M.OK
    ref = rk.Discretization(scheme, nx, c).propagate(u0, nt)
    assert np.max(np.abs(r.out.cpu().numpy()[0] - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_iteration_limits_and_exact_start():
    s, nx, nt, m = "ERK3", 512, 2048, 4
    c = rk.paper_cfl(s)
    u0 = inputs.fourier_u0(nx, 4, 2)
    with M.Plan(nx, nt, c, s, m, 3, _psi(s, c, nx, m, 3)) as P:
        u = torch.tensor(u0, device="cuda")
        r0 = P.solve(u, None, tol=1e-10, maxit=0)
        assert r0.status == M.ENOTCONV and r0.iters == 0 and len(r0.hist) == 1
        assert r0.hist[0] > 1e-3
        rbig = P.solve(u, None, tol=1e9, maxit=10)  # already below tol
        assert rbig.status == M.OK and rbig.iters == 0
        # the exact C-points as the initial iterate: converged at once
        exact = rk.Discretization(s, nx, c).time_stepping(u0, nt, every=m)
        re = P.solve(u, torch.tensor(exact, device="cuda"), tol=1e-12, maxit=5)
        assert re.status == M.OK and re.iters == 0
        assert re.hist[0] <= 1e-12


def test_diverging_coarse_operator_is_reported():
    s, nx, nt, m = "ERK1", 64, 256, 4
    c = rk.paper_cfl(s)
    bad = [(np.array([0]), np.array([1e300]))]
    with M.Plan(nx, nt, c, s, m, 2, bad) as P:
        r = P.solve(torch.tensor(inputs.fourier_u0(nx, 4, 1), device="cuda"), None,
                    tol=1e-10, maxit=20)
    assert r.status == M.EDIVERGED
    assert not np.isfinite(r.hist[-1])
