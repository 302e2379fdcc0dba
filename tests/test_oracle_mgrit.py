"""Pins for the oracle's MGRIT iteration (Sec. 2.2, Sec. 4.4).

* the fixed point is the exact discrete solution: sequential stepping and
  a dense space-time LU solve of the block-bidiagonal system of eq. (3);
* finite exactness: FCF exact after n_t/(2m) iterations and F-relaxation
  after n_t/m, whatever Psi is (Sec. 1, Table 2);
* Psi = Phi^m converges in one iteration (Sec. 2.2);
* iteration counts printed in Tables 2, 4 and 6.
"""

import json
import os

import numpy as np
import pytest

from oracle import coarse, mgrit, rk
from paper_1910_03726_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_tables.json")))


def _setup(scheme, nx, nt, m, levels=2, widths=None, psi=None, cycle="V",
           relax="FCF", cfl=None):
    c = rk.paper_cfl(scheme) if cfl is None else cfl
    d = rk.Discretization(scheme, nx, c)
    if psi is None:
        H = coarse.build_hierarchy(d, m, levels, widths=widths)
        ops = [d.step] + [mgrit.taps_op(h["offsets"], h["weights"]) for h in H]
    else:
        ops = [d.step] + psi(d)
    return d, mgrit.MGRIT(ops, m, nt, cycle=cycle, relax=relax)


def _redisc(m, levels=2):
    # Psi_l = Phi with time step m^(l-1) dt (rediscretization, Sec. 2.2)
    return lambda d: [(lambda X, k=l: d.step(X, dt=m ** k * d.dt))
                      for l in range(1, levels)]


def _solve(d, M, tol=1e-10, maxit=400, seed=1, u0=None):
    nc = M.nt // M.m
    u0 = np.sin(np.pi * d.x) ** 4 if u0 is None else u0
    uinit = inputs.random_iterate(nc + 1, d.nx, seed)
    return M.solve(u0, uinit, tol, maxit, mgrit.norm_scale(d))


@pytest.mark.parametrize("scheme,m", [("ERK1", 4), ("ERK3", 2), ("SDIRK3", 4)])
def test_fcf_exact_after_nt_over_2m(scheme, m):
    # FCF propagates the exact solution two C-intervals per iteration, so
    # the residual is exactly zero after n_t/(2m) iterations even with the
    # divergent rediscretized Psi (Table 2, right side).
    nx, nt = 32, 64
    d, M = _setup(scheme, nx, nt, m, psi=_redisc(m))
    R = _solve(d, M, tol=0.0, maxit=nt // (2 * m))
    assert R.hist[-1] == 0.0
    assert R.hist[-2] > 0.0


@pytest.mark.parametrize("scheme,m", [("ERK1", 4), ("SDIRK2", 2)])
def test_f_relaxation_exact_after_nt_over_m(scheme, m):
    # F-relaxation (Parareal) propagates one C-interval per iteration.  Its
    # correction u + (Phi^m u_prev - u) is exact only up to rounding, and a
    # Psi far from Phi^m lets intermediate iterates grow, so the test uses
    # Psi = 0 (no growth) and a rounding-level bound.
    nx, nt = 24, 48
    d, M = _setup(scheme, nx, nt, m, psi=lambda d: [lambda X: 0.0 * X],
                  relax="F")
    R = _solve(d, M, tol=0.0, maxit=nt // m)
    assert R.hist[-1] < 1e-14 * R.hist[0]
    assert R.hist[-2] > 1e-8 * R.hist[0]


@pytest.mark.parametrize("scheme", ["ERK3", "SDIRK3"])
def test_ideal_psi_one_iteration(scheme):
    # Psi = Phi^m: the coarse problem is the exact Schur complement.
    nx, nt, m = 32, 64, 4
    c = rk.paper_cfl(scheme)
    d = rk.Discretization(scheme, nx, c)
    col, _ = coarse.phi_m_first_column(d.eigenvalues(), m)
    M = mgrit.MGRIT([d.step, mgrit.taps_op(np.arange(nx), col)], m, nt)
    R = _solve(d, M, tol=1e-13)
    assert R.iters == 1
    assert R.hist[1] < 1e-13 * R.hist[0]


@pytest.mark.parametrize("scheme", ["ERK3", "SDIRK2"])
def test_fixed_point_is_dense_space_time_solution(scheme):
    # Eq. (3) as one block lower-bidiagonal system, solved by dense LU with
    # Phi from the block form of the Runge-Kutta step.
    nx, nt, m = 8, 32, 4
    d, M = _setup(scheme, nx, nt, m, levels=3, widths=[6, 8]
                  if scheme == "ERK3" else None)
    P = d.dense_phi()
    N = (nt + 1) * nx
    A = np.eye(N)
    for n in range(nt):
        A[(n + 1) * nx:(n + 2) * nx, n * nx:(n + 1) * nx] = -P
    rng = np.random.default_rng(0)
    u0 = rng.standard_normal(nx)
    b = np.zeros(N)
    b[:nx] = u0
    U = np.linalg.solve(A, b).reshape(nt + 1, nx)
    R = _solve(d, M, tol=1e-14, u0=u0)
    assert R.status == "converged"
    full = M.fill(R.cpoints)
    assert np.max(np.abs(full - U)) < 1e-12 * np.max(np.abs(U))


@pytest.mark.parametrize("cycle", ["V", "F"])
def test_multilevel_converges_to_sequential_solution(cycle):
    scheme, nx, nt, m = "ERK3", 64, 512, 4
    d, M = _setup(scheme, nx, nt, m, levels=4, cycle=cycle)
    u0 = inputs.fourier_u0(nx, 8, 0, decay=2.0)
    R = _solve(d, M, tol=1e-13, u0=u0)
    assert R.status == "converged"
    seq = d.time_stepping(u0, nt, every=m)
    assert np.max(np.abs(R.cpoints - seq)) < 1e-12 * np.max(np.abs(seq))


def test_f_cycle_no_more_iterations_than_v_cycle():
    scheme, nx, nt, m = "ERK3", 128, 2048, 8
    counts = {}
    for cyc in ("V", "F"):
        d, M = _setup(scheme, nx, nt, m, levels=3, cycle=cyc)
        counts[cyc] = _solve(d, M).iters
    assert counts["F"] <= counts["V"]


def test_config1_counts():
    # ERK1+U1, n_x = 64, n_t = 256, m = 4: 6 iterations with the 3-point
    # characteristic Psi (Table 3's m = 4 entry); the rediscretized Psi
    # (coarse CFL 3.4 > 1) diverges and is only exact at n_t/(2m) = 32.
    w = inputs.WORKLOADS["erk1_u1_nx64_nt256_m4_2level"]
    u0 = inputs.workload_u0(w)
    d, M = _setup("ERK1", 64, 256, 4, widths=[3], cfl=w["cfl"])
    R = _solve(d, M, u0=u0, seed=w["init_seed"])
    assert R.iters == 6 and R.status == "converged"
    d, M = _setup("ERK1", 64, 256, 4, psi=_redisc(4), cfl=w["cfl"])
    R = _solve(d, M, u0=u0, seed=w["init_seed"], maxit=40)
    assert R.iters == 32 and R.hist[-1] == 0.0
    assert max(R.hist) > 1e30


def test_table4_erk1_v_cycles():
    want = GOLD["table4_multilevel_v_m4"]["ERK1_2e8x2e10"]
    for L, widths in ((2, [3]), (3, [3, 6]), (4, [3, 6, 11]),
                      (5, [3, 6, 11, 21])):
        d, M = _setup("ERK1", 256, 1024, 4, levels=L, widths=widths)
        assert _solve(d, M).iters == want[L - 2]


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_table6_sdirk_lsq_counts(p):
    # Table 6: two-level, least-squares Psi with the eta_tol thresholding
    # of Sec. 4.6, n_x = n_t = 2^10, c = 4; all six coarsening factors.
    want = GOLD["table6_sdirk_lsq"][f"SDIRK{p}"]
    got = []
    for m in (2, 4, 8, 16, 32, 64):
        d, M = _setup(f"SDIRK{p}", 1024, 1024, m)
        got.append(_solve(d, M).iters)
    assert got == want


@pytest.mark.parametrize("p,m", [(1, 2), (1, 4), (3, 4)])
def test_table2_rediscretized_sdirk_counts(p, m):
    want = GOLD["table2_rediscretized_sdirk"][f"SDIRK{p}"][str(m)]
    d, M = _setup(f"SDIRK{p}", 1024, 1024, m, psi=_redisc(m))
    R = _solve(d, M, maxit=300)
    assert R.iters == want
