"""Pins for the oracle's inflow/outflow discretization (Sec. 4.5).

* global order p of ERKp+Up with the boundary closures, against the exact
  solution g(t - (x+1)/alpha) of the inflow problem;
* exactness (to rounding) for polynomial inflow data of degree p-1, which
  every closure (inflow ghosts by inverse Lax-Wendroff, stage data,
  outflow extrapolation) reproduces exactly: a dropped term, a wrong sign
  or a wrong stage coefficient breaks it;
* away from the boundaries Phi is the periodic stepper (Corollary 1's
  Toeplitz stencil); Phi is stable at the paper's Courant numbers;
* MGRIT with the truncated periodic Psi converges to sequential stepping,
  and reproduces the ERK1 entries of Table 5 that the width rule of
  Table 4 fixes.
"""

import json
import os

import numpy as np
import pytest

from oracle import coarse, inflow, mgrit, rk
from paper_1910_03726_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_tables.json")))["table5_inflow"]


def _exact(d, g, t):
    return g(t - (d.x + 1.0) / d.alpha)


@pytest.mark.parametrize("scheme,order", [("ERK1", 1), ("ERK3", 3), ("ERK5", 5)])
def test_global_order(scheme, order):
    c = rk.paper_cfl(scheme)
    g = lambda t: np.sin(np.pi * t) ** 4
    errs = []
    for nx in (64, 128, 256):
        d = inflow.InflowDiscretization(scheme, nx, c)
        nt = int(round(0.5 / d.dt))
        G = inputs.sin4_inflow_derivs(nt, d.dt, d.n_derivs())
        u = d.time_stepping(_exact(d, g, 0.0), G, every=nt)[-1]
        errs.append(np.max(np.abs(u - _exact(d, g, nt * d.dt))))
    rate = np.log2(errs[1] / errs[2])
    assert order - 0.15 < rate < order + 0.5, errs


@pytest.mark.parametrize("scheme", ["ERK1", "ERK2", "ERK3", "ERK4", "ERK5"])
def test_polynomial_inflow_is_exact(scheme):
    d = inflow.InflowDiscretization(scheme, 48, rk.paper_cfl(scheme), alpha=1.3)
    deg = d.p - 1
    co = np.random.default_rng(d.p).standard_normal(deg + 1)
    g = lambda t: sum(co[k] * t ** k for k in range(deg + 1))
    nt = 40
    G = inputs.poly_inflow_derivs(co, nt, d.dt, d.n_derivs())
    u = d.time_stepping(_exact(d, g, 0.0), G, every=nt)[-1]
    ref = _exact(d, g, nt * d.dt)
    assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(np.abs(ref))
    # one degree more is not reproduced (the pin has teeth) for p >= 3
    if d.p >= 3:
        co2 = np.append(co, 1.0)
        g2 = lambda t: sum(co2[k] * t ** k for k in range(deg + 2))
        G2 = inputs.poly_inflow_derivs(co2, nt, d.dt, d.n_derivs())
        u2 = d.time_stepping(_exact(d, g2, 0.0), G2, every=nt)[-1]
        assert np.max(np.abs(u2 - _exact(d, g2, nt * d.dt))) > 1e-11


@pytest.mark.parametrize("scheme", ["ERK1", "ERK3", "ERK5"])
def test_interior_is_the_periodic_stencil_and_phi_is_stable(scheme):
    c = rk.paper_cfl(scheme)
    nx = 64
    d = inflow.InflowDiscretization(scheme, nx, c)
    P = d.dense_phi()
    Pp = rk.Discretization(scheme, nx, c).dense_phi()
    reach = len(d.b) * max(d.rl, d.rr)
    for i in range(2 * reach, nx - 2 * reach):
        np.testing.assert_allclose(P[i], Pp[i], rtol=0, atol=1e-15)
    assert np.max(np.abs(np.linalg.eigvals(P))) < 1.0
    assert np.linalg.norm(np.linalg.matrix_power(P, 4 * nx), 2) < 1.0
    # the step is affine: Phi u + f
    u = np.random.default_rng(0).standard_normal(nx)
    gd = np.random.default_rng(1).standard_normal(d.n_derivs())
    np.testing.assert_allclose(d.step(u, gd), P @ u + d.forcing(gd), rtol=0, atol=1e-13)


def test_truncated_psi_is_the_truncated_toeplitz_matrix():
    nx = 16
    offs, w = np.array([-2, 0, 1, 3, 15]), np.array([0.1, 0.5, 0.3, -0.2, 0.05])
    X = np.random.default_rng(2).standard_normal((3, nx))
    T = np.zeros((nx, nx))
    for o, wt in zip(offs, w):
        o = o - nx if o > nx // 2 else o
        for a in range(nx):
            if 0 <= a - o < nx:
                T[a, a - o] += wt
    np.testing.assert_allclose(inflow.truncated_taps_op(offs, w)(X), X @ T.T, atol=1e-15)


def _inflow_mgrit(scheme, nx, nt, m, L, widths=None, cycle="V"):
    c = rk.paper_cfl(scheme)
    d = inflow.InflowDiscretization(scheme, nx, c)
    H = coarse.build_hierarchy(rk.Discretization(scheme, nx, c), m, L, widths=widths)
    P = d.dense_phi()
    ops = [lambda X: X @ P.T] + [inflow.truncated_taps_op(h["offsets"], h["weights"])
                                 for h in H]
    G = inputs.sin4_inflow_derivs(nt, d.dt, d.n_derivs())
    u0 = np.sin(np.pi * (d.x + 1.0)) ** 4
    return d, mgrit.MGRIT(ops, m, nt, cycle=cycle), u0, G


def test_mgrit_fixed_point_is_sequential_stepping():
    d, M, u0, G = _inflow_mgrit("ERK3", 64, 256, 4, 3)
    g = d.rhs(u0, G)
    R = M.solve(u0, inputs.random_iterate(65, 64, 3), 1e-13, 60, mgrit.norm_scale(d), g=g)
    assert R.status == "converged"
    seq = d.time_stepping(u0, G, every=4)
    assert np.max(np.abs(R.cpoints - seq)) < 1e-11
    # all points by F-relaxation from the C-points
    allp = M.fill(R.cpoints, g)
    assert np.max(np.abs(allp - d.time_stepping(u0, G))) < 1e-11
    # FCF is exact after n_t/(2m) iterations whatever Psi is (Sec. 1)
    R2 = M.solve(u0, inputs.random_iterate(65, 64, 3), 0.0, 256 // 8,
                 mgrit.norm_scale(d), g=g)
    assert R2.hist[-1] < 1e-12 * R2.hist[0]


def test_table5_erk1_counts():
    # two-level, m = 4, width 3 (the width that gives Table 3's periodic count)
    d, M, u0, G = _inflow_mgrit("ERK1", 256, 1024, 4, 2, widths=[3])
    R = M.solve(u0, inputs.random_iterate(257, 256, 1), 1e-10, 40, mgrit.norm_scale(d),
                g=d.rhs(u0, G))
    assert R.iters == GOLD["ERK1_2e8x2e10_two_level"][1]
    # V-cycles with the Table 4 widths, 2..5 levels
    want = GOLD["ERK1_2e8x2e10_multilevel"]
    for L in range(2, 6):
        d, M, u0, G = _inflow_mgrit("ERK1", 256, 1024, 4, L, widths=[3, 6, 11, 21][:L - 1])
        R = M.solve(u0, inputs.random_iterate(257, 256, 1), 1e-10, 40, mgrit.norm_scale(d),
                    g=d.rhs(u0, G))
        assert R.iters == want[L - 2], L


def test_truncated_psi_with_positive_offsets_is_nilpotent_and_chunks_are_exact():
    # every offset >= 1: Psi is strictly lower triangular, Psi^q = 0 for
    # q = ceil(n_x / smallest offset); the sweep x^s = Psi x^(s-1) + g^s
    # restarted from zero q steps before a row gives that row exactly
    nx, offs = 40, np.array([3, 4, 5, 6, 8])
    w = np.random.default_rng(4).standard_normal(len(offs))
    op = inflow.truncated_taps_op(offs, w)
    q = -(-nx // int(offs.min()))
    E = np.eye(nx)
    Pq = E
    for _ in range(q):
        Pq = op(Pq)
    assert np.all(Pq == 0.0)
    Pq1 = E
    for _ in range(q - 1):
        Pq1 = op(Pq1)
    assert np.any(Pq1 != 0.0)  # q is the nilpotency index here
    n = 50
    g = np.random.default_rng(5).standard_normal((n + 1, nx))
    g[0] = 0.0
    ref = mgrit.sequential_solve(op, g)
    for t in range(q, n + 1):
        x = np.zeros(nx)
        for s in range(t - q + 1, t + 1):
            x = op(x[None])[0] + g[s]
        assert np.array_equal(x, ref[t]), t
