"""libmgrit C-ABI on the host: symbols, and the host-only setup entry points
(stability, the collapsed ERK stepper, the least-squares coarse operators)
against the oracle.  No GPU work is launched here.
"""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import coarse, rk, inflow
from paper_1910_03726_amd import mgrit as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(",
                             src, flags=re.M):
            if m.group(1) not in ("defined",):
                names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = M.lib()
    names = _declared_functions()
    assert "mgrit_solve" in names and "phi_apply_batch" in names
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_version():
    lib = M.lib()
    assert lib.mgrit_version() >= 100
    for code in range(0, -11, -1):
        assert lib.mgrit_strerror(code)
    assert b"unknown" in lib.mgrit_strerror(-999)


@pytest.mark.parametrize("scheme", ["ERK1", "ERK2", "ERK3", "ERK4", "ERK5", "SDIRK3"])
def test_max_amplification_matches_oracle(scheme):
    c = rk.paper_cfl(scheme)
    assert abs(M.max_amplification(scheme, c) - rk.max_amplification(scheme, c)) < 1e-13
    if scheme.startswith("ERK"):
        # just above Table 1's limit the step amplifies
        cmax = rk.CFL_MAX_TABLE1[rk.scheme_order(scheme)]
        assert M.max_amplification(scheme, 1.01 * cmax) > 1 + 1e-6


@pytest.mark.parametrize("scheme,nx", [("ERK1", 16), ("ERK2", 64), ("ERK3", 64),
                                       ("ERK4", 50), ("ERK5", 64), ("ERK5", 20)])
def test_phi_taps_are_one_step(scheme, nx):
    # Corollary 1: the collapsed stencil applied to e_0 is one staged step
    c = rk.paper_cfl(scheme)
    d = rk.Discretization(scheme, nx, c)
    off, w = M.phi_taps(scheme, c, nx)
    col = np.zeros(nx)
    np.add.at(col, off, w)
    e0 = np.zeros(nx)
    e0[0] = 1.0
    assert np.max(np.abs(col - d.step(e0))) < 1e-14


def test_phi_taps_rejects_sdirk():
    with pytest.raises(M.MgritError):
        M.phi_taps("SDIRK3", 4.0, 64)


CASES = [
    ("ERK1", 64, 4, 2, "window", [3]),
    ("ERK1", 256, 4, 4, "window", [3, 6, 11]),
    ("ERK3", 512, 8, 4, "window", None),
    ("ERK5", 1024, 8, 4, "window", None),
    ("SDIRK1", 256, 8, 2, "eta", None),
    ("SDIRK2", 256, 4, 2, "eta", None),
    ("SDIRK3", 2048, 16, 2, "eta", None),
    ("SDIRK4", 256, 64, 2, "eta", None),
    ("ERK3", 96, 4, 3, "window", None),
]


@pytest.mark.parametrize("scheme,nx,m,L,rule,widths", CASES)
def test_psi_optimize_matches_oracle(scheme, nx, m, L, rule, widths):
    c = rk.paper_cfl(scheme)
    d = rk.Discretization(scheme, nx, c)
    got, mi = M.psi_optimize(scheme, c, nx, m, L, rule=rule, widths=widths)
    H = coarse.build_hierarchy(d, m, L, widths=widths)
    assert mi < 1e-8
    for (o, w), h in zip(got, H):
        assert sorted(o.tolist()) == sorted(h["offsets"].tolist())
        a = w[np.argsort(o)]
        b = h["weights"][np.argsort(h["offsets"])]
        # both solve the same weighted least-squares problem; agreement is
        # limited by its conditioning
        assert np.max(np.abs(a - b)) <= 1e-8 * np.max(np.abs(b))


@pytest.mark.parametrize("scheme,nx,nt,m,L,target", [("ERK3", 256, 4096, 4, 4, 1e-3),
                                                      ("ERK5", 128, 2048, 8, 3, 1e-3),
                                                      ("ERK1", 64, 2048, 4, 3, 1e-4)])
def test_psi_optimize_bound_matches_oracle(scheme, nx, nt, m, L, target):
    c = rk.paper_cfl(scheme)
    d = rk.Discretization(scheme, nx, c)
    got, bounds, mi = M.psi_optimize_bound(scheme, c, nx, nt, m, L, target)
    H = coarse.build_hierarchy_bound(d, m, L, nt, target)
    assert mi < 1e-8
    for (o, w), b, h in zip(got, bounds, H):
        assert sorted(o.tolist()) == sorted(h["offsets"].tolist())
        a = w[np.argsort(o)]
        ref = h["weights"][np.argsort(h["offsets"])]
        assert np.max(np.abs(a - ref)) <= 1e-8 * np.max(np.abs(ref))
        # a bound at rounding level (|lambda^m - mu| ~ eps) differs by rounding
        assert b == pytest.approx(h["bound"], rel=1e-6, abs=1e-10)


def test_psi_optimize_bound_unreachable_target_takes_the_smallest_bound():
    # no width reaches 1e-15: each level takes the width of smallest bound
    s, nx, nt, m, L = "ERK3", 128, 2048, 4, 3
    c = rk.paper_cfl(s)
    got, bounds, _ = M.psi_optimize_bound(s, c, nx, nt, m, L, 1e-15)
    H = coarse.build_hierarchy_bound(rk.Discretization(s, nx, c), m, L, nt, 1e-15)
    for (o, _), b, h in zip(got, bounds, H):
        assert sorted(o.tolist()) == sorted(h["offsets"].tolist())
        assert b > 1e-15
        assert b == pytest.approx(h["bound"], rel=1e-6, abs=1e-10)


def test_psi_optimize_bound_rejects_sdirk():
    with pytest.raises(M.MgritError):
        M.psi_optimize_bound("SDIRK3", 4.0, 256, 1024, 4, 2)


@pytest.mark.parametrize("scheme,nx,alpha", [("ERK1", 16, 1.0), ("ERK2", 40, 0.7),
                                             ("ERK3", 64, 1.0), ("ERK4", 200, 1.3),
                                             ("ERK5", 200, 1.0), ("ERK5", 700, 1.0),
                                             ("ERK3", 1000, 2.0)])
def test_inflow_operator_matches_oracle(scheme, nx, alpha):
    # Phi as the bounded kernel applies it (dense corner blocks + the
    # truncated periodic stencil) and the forcing matrix B, against the
    # oracle's staged step applied to unit vectors and unit data
    c = rk.paper_cfl(scheme)
    d = inflow.InflowDiscretization(scheme, nx, c, alpha=alpha)
    phi, B = M.inflow_operator(scheme, c, nx, alpha)
    assert np.max(np.abs(phi - d.dense_phi())) <= 4e-15
    nd = d.n_derivs()
    Bo = np.stack([d.forcing(np.eye(nd)[k]) for k in range(nd)], axis=1)
    assert np.max(np.abs(B - Bo)) <= 1e-14 * np.max(np.abs(Bo))


def test_inflow_operator_rejects_sdirk():
    with pytest.raises(M.MgritError):
        M.inflow_operator("SDIRK3", 4.0, 64)


def test_psi_redisc_is_erk_at_m_times_c():
    c = rk.paper_cfl("ERK1")
    got, _ = M.psi_optimize("ERK1", c, 64, 4, 3, rule="redisc")
    for l, (o, w) in enumerate(got, start=1):
        o2, w2 = M.phi_taps("ERK1", c * 4 ** l, 64)
        assert o.tolist() == o2.tolist() and np.allclose(w, w2, rtol=0, atol=1e-15)


def test_psi_capacity_error():
    lib = M.lib()
    arr = (M.Taps * 1)()
    o = (ctypes.c_int * 2)()
    w = (ctypes.c_double * 2)()
    arr[0].nnz, arr[0].offset, arr[0].weight = 2, o, w
    rc = lib.mgrit_psi_optimize(13, 4.0, 2048, 16, 2, 2, None, 0.0, arr, None)
    assert rc == M.ECAPACITY
    assert arr[0].nnz == 42  # the count needed


def test_invalid_arguments():
    with pytest.raises(M.MgritError):
        M.psi_optimize("ERK1", 0.85, 64, 1, 2)
    with pytest.raises(M.MgritError):
        M.psi_optimize("ERK3", 1.38, 64, 4, 2, rule="eta")  # no eta table for ERK
