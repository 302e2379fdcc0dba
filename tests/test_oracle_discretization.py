"""Pins for the oracle's discretization (Sec. 2.1, Appendix A, Table 1).

Each test ties the oracle to something other than itself: order
conditions of Runge-Kutta theory, the Taylor conditions of the upwind
formulas, values printed in Table 1 and in the Sec. 2.2 set-up, the
closed-form Fourier symbol of Lemma 1, and the observed order of
accuracy of Fig. 1.
"""

import json
import math
import os

import numpy as np
import pytest

from oracle import rk

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_tables.json")))

ERKS = ["ERK1", "ERK2", "ERK3", "ERK4", "ERK5"]
SDIRKS = ["SDIRK1", "SDIRK2", "SDIRK3", "SDIRK4"]


def _order_conditions(A, b, c):
    """(value, exact) pairs for the Butcher order conditions up to order 5."""
    e = np.ones_like(b)
    Ac = A @ c
    return {
        1: [(b @ e, 1.0)],
        2: [(b @ c, 1 / 2)],
        3: [(b @ c**2, 1 / 3), (b @ Ac, 1 / 6)],
        4: [(b @ c**3, 1 / 4), (b @ (c * Ac), 1 / 8), (b @ (A @ c**2), 1 / 12),
            (b @ (A @ Ac), 1 / 24)],
        5: [(b @ c**4, 1 / 5), (b @ (c**2 * Ac), 1 / 10),
            (b @ (c * (A @ c**2)), 1 / 15), (b @ (c * (A @ Ac)), 1 / 30),
            (b @ (Ac * Ac), 1 / 20), (b @ (A @ c**3), 1 / 20),
            (b @ (A @ (c * Ac)), 1 / 40), (b @ (A @ (A @ c**2)), 1 / 60),
            (b @ (A @ (A @ Ac)), 1 / 120)],
    }


@pytest.mark.parametrize("scheme", ERKS + SDIRKS)
def test_tableau_order_conditions(scheme):
    A, b, c = rk.TABLEAUX[scheme]
    p = rk.scheme_order(scheme)
    conds = _order_conditions(A, b, c)
    for q in range(1, p + 1):
        for val, exact in conds[q]:
            assert abs(val - exact) < 1e-14, (scheme, q, val, exact)
    if p < 5:
        # the method is of order exactly p: some order-(p+1) condition fails
        assert any(abs(v - x) > 1e-6 for v, x in conds[p + 1])


@pytest.mark.parametrize("scheme", ERKS)
def test_erk_is_explicit(scheme):
    A, _, _ = rk.TABLEAUX[scheme]
    assert np.allclose(np.triu(A), 0.0)


def test_erk5_stability_polynomial():
    # R(z) = sum_{k<=5} z^k/k! + z^6/1280 for Butcher's (236a) method.
    g = rk.stability_polynomial_coeffs("ERK5")
    want = [1 / math.factorial(k) for k in range(6)] + [1 / 1280]
    assert np.allclose(g, want, rtol=0, atol=1e-16)


def test_sdirk3_constant_is_the_l_stable_root():
    # Appendix A, Table 8's zeta is the root of z^3 - 3z^2 + 3z/2 - 1/6 in
    # (0, 1) that makes the 3-stage SDIRK method of order 3 L-stable.
    z = rk.TABLEAUX["SDIRK3"][0][0, 0]
    assert abs(z**3 - 3 * z**2 + 1.5 * z - 1.0 / 6.0) < 1e-15


@pytest.mark.parametrize("scheme", SDIRKS)
def test_sdirk_l_stable(scheme):
    A, b, _ = rk.TABLEAUX[scheme]
    # stiffly accurate: b equals the last row of A, hence R(-inf) = 0
    assert np.allclose(A[-1], b)
    assert abs(rk.stability_function(A, b, -1e9)) < 1e-6
    y = np.linspace(-50, 50, 2001)
    assert np.max(np.abs(rk.stability_function(A, b, 1j * y))) <= 1 + 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_upwind_taylor_conditions(p):
    # (1/dx) sum_j d_j v(x + j dx) = v'(x) + O(dx^p):  sum_j d_j j^q = [q==1]
    # for q = 0..p, and the p+1 condition fails (exact order p).
    d = rk.UPWIND[p]
    for q in range(p + 1):
        s = sum(c * j**q for j, c in d.items())
        assert abs(s - (1.0 if q == 1 else 0.0)) < 1e-14
    assert abs(sum(c * j**(p + 1) for j, c in d.items())) > 1e-6
    # upwind for alpha > 0: at most floor(p/2) points downwind
    assert max(d) <= p // 2


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_cfl_limits_table1_strict(p):
    # Largest c with |R| <= 1 (up to rounding) matches Table 1's digits.
    c = rk.cfl_limit(f"ERK{p}", slack=1e-14)
    want = GOLD["table1_cfl_limits"][f"ERK{p}"]
    assert abs(c - want) < 5e-6, (c, want)


def test_cfl_limit_erk5_reading():
    # Table 1 prints 1.96583 for ERK5+U5.  The strict limit is lower
    # (~1.9396); 1.96583 is the limit once |R| - 1 <= 4e-7 is tolerated.
    strict = rk.cfl_limit("ERK5", slack=1e-14)
    loose = rk.cfl_limit("ERK5", slack=4e-7)
    assert 1.93 < strict < 1.945
    assert abs(loose - GOLD["table1_cfl_limits"]["ERK5"]) < 5e-6
    # the experiments' c = 0.85 * 1.96583 is strictly stable
    assert rk.max_amplification("ERK5", 0.85 * 1.96583) <= 1 + 1e-15


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_integration_times(p):
    # Sec. 2.2: n_t is the largest power of two with T = n_t dt <= 8.
    s = f"ERK{p}"
    c = 0.85 * GOLD["table1_cfl_limits"][s]
    for nx in (256, 1024):
        nt = rk.paper_nt(s, nx, c)
        T = nt * c * 2.0 / nx
        assert abs(T - GOLD["integration_times"][s]) < 0.05


@pytest.mark.parametrize("scheme", ERKS + SDIRKS)
def test_phi_symbol_lemma1(scheme):
    # Lemma 1: Phi acts on the Fourier mode exp(i k pi x) as R(dt l(theta)).
    nx = 48
    c = rk.paper_cfl(scheme)
    d = rk.Discretization(scheme, nx, c)
    lam = d.eigenvalues()
    rng = np.random.default_rng(3)
    for k in rng.choice(nx, 6, replace=False):
        mode = np.exp(2j * np.pi * k * np.arange(nx) / nx)
        out = d.step(np.real(mode)) + 1j * d.step(np.imag(mode))
        assert np.max(np.abs(out - lam[k] * mode)) < 1e-13


@pytest.mark.parametrize("scheme", ["ERK3", "ERK5", "SDIRK2", "SDIRK3"])
def test_dense_phi_block_form_matches_step(scheme):
    nx = 20
    d = rk.Discretization(scheme, nx, rk.paper_cfl(scheme))
    P = d.dense_phi()
    rng = np.random.default_rng(4)
    U = rng.standard_normal((5, nx))
    assert np.max(np.abs(U @ P.T - d.step(U))) < 1e-13
    # Corollary 1: Phi is circulant
    for i in range(nx):
        assert np.allclose(np.roll(P[0], i), P[i], atol=1e-14)


def test_explicit_phi_is_sparse_stencil():
    # Corollary 1: for ERK, Phi is a sparse circulant with s*(stencil span)
    # + 1 non-zeros per row: 2, 5, 10, 17, 31 for ERK1..ERK5.
    want = {1: 2, 2: 5, 3: 10, 4: 17, 5: 31}
    for p, nnz in want.items():
        d = rk.Discretization(f"ERK{p}", 64, rk.paper_cfl(f"ERK{p}"))
        col = d.dense_phi()[:, 0]
        assert np.count_nonzero(np.abs(col) > 1e-14) == nnz


def test_shifted_solve_is_exact():
    d = rk.Discretization("SDIRK3", 64, 4.0)
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal((3, 64))
    y = d.solve_shifted(rhs, 0.7 * d.dt)
    assert np.max(np.abs(y - 0.7 * d.dt * d.apply_L(y) - rhs)) < 1e-13


@pytest.mark.parametrize("scheme", ["ERK1", "ERK3", "ERK5", "SDIRK3", "SDIRK4"])
def test_discretization_order(scheme):
    # Fig. 1: the error against the exact (shifted) solution of eq. (1)
    # decays at rate p under uniform space-time refinement at fixed CFL.
    p = rk.scheme_order(scheme)
    c = rk.paper_cfl(scheme)
    errs = []
    sizes = (64, 128, 256) if p <= 3 else (32, 64, 128)
    T = 1.0
    for nx in sizes:
        d = rk.Discretization(scheme, nx, c)
        nt = int(round(T / d.dt))
        d.dt = T / nt
        u = d.propagate(np.sin(np.pi * d.x) ** 4, nt)
        exact = np.sin(np.pi * (d.x - d.alpha * T)) ** 4
        errs.append(np.sqrt(d.dx * np.sum((u - exact) ** 2)))
    rate = np.log2(errs[-2] / errs[-1])
    assert rate > p - 0.35, (scheme, errs, rate)


# -- Lemma 1 closed form (spectral_propagate) ---------------------------------
def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("scheme,nsteps", [("ERK1", 3000), ("ERK2", 2000), ("ERK3", 3000),
                                           ("ERK4", 2000), ("ERK5", 3000), ("SDIRK1", 30),
                                           ("SDIRK2", 500), ("SDIRK3", 500),
                                           ("SDIRK4", 500)])
def test_closed_form_matches_staged_stepping(scheme, nsteps):
    # Lemma 1's Phi^n u0 against n stage-by-stage steps (a different
    # algorithm: no eigenvalues, no transforms).  FP64 stepping drifts by
    # ~eps per step; a dropped stage term, a wrong coefficient or a
    # conjugated symbol would be off by O(1).  (SDIRK1 at c = 4 damps the
    # modes below the rounding level within a few hundred steps: 30 steps.)
    nx = 64
    d = rk.Discretization(scheme, nx, rk.paper_cfl(scheme))
    u0 = np.cos(np.pi * d.x) + 0.5 * np.sin(3 * np.pi * d.x) - 0.2 * np.cos(4 * np.pi * d.x)
    assert _rel(d.spectral_propagate(u0, nsteps), d.propagate(u0, nsteps)) < 5e-16 * nsteps


@pytest.mark.parametrize("scheme", ["ERK3", "ERK5", "SDIRK3", "SDIRK4"])
def test_closed_form_matches_dense_phi_power(scheme):
    # against the n-th power of Phi built from the block form of the step
    nx, n = 16, 37
    d = rk.Discretization(scheme, nx, rk.paper_cfl(scheme))
    u0 = np.random.default_rng(9).standard_normal(nx)
    P = np.linalg.matrix_power(d.dense_phi(), n)
    # (the dense block solve rounds at the size of SDIRK4's entries, ~8)
    assert _rel(d.spectral_propagate(u0, n), P @ u0) < 1e-12


@pytest.mark.parametrize("scheme", ["ERK3", "SDIRK3"])
def test_closed_form_transports_to_the_right(scheme):
    # u_t + alpha u_x = 0 with alpha > 0 carries a bump to the right by
    # alpha t = n c dx: n c cells (Sec. 2.1)
    nx = 256
    c = rk.paper_cfl(scheme)
    d = rk.Discretization(scheme, nx, c)
    u0 = np.exp(-((d.x + 0.5) / 0.08) ** 2)
    n = 40
    u = d.spectral_propagate(u0, n)
    shift = (int(np.argmax(u)) - int(np.argmax(u0))) % nx
    assert abs(shift - n * c) <= 1.0, (shift, n * c)


def test_closed_form_is_extended_precision():
    # one Fourier mode over 10^5 steps against a 40-digit evaluation of the
    # same eigenvalue power: the FP64 closed form would be off by ~n eps
    import mpmath as mp
    mp.mp.dps = 40
    nx, k, n = 1024, 1, 100000
    scheme = "ERK3"
    c = rk.paper_cfl(scheme)
    d = rk.Discretization(scheme, nx, c)
    u0 = np.cos(np.pi * k * d.x)
    # R(z) = 1 + z + z^2/2 + z^3/6 for ERK3 (order 3, three stages)
    th = 2 * mp.pi * k / nx
    z = -mp.mpf(c) * sum(mp.mpf(num) / den * mp.exp(1j * j * th)
                         for j, (num, den) in rk.UPWIND_FRACTIONS[3].items())
    lam = 1 + z + z ** 2 / 2 + z ** 3 / 6
    ln = lam ** n
    want = np.array([float(mp.re(ln * mp.exp(1j * mp.pi * k * (mp.mpf(-1) + mp.mpf(2) * i / nx))))
                     for i in range(nx)])
    # n eps of extended precision is 1.1e-14; FP64 would give ~1e-11
    assert _rel(d.spectral_propagate(u0, n), want) < 5e-14
