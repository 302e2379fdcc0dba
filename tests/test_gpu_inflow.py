"""Inflow/outflow boundaries (Sec. 4.5) on the GPU, against the oracle.

The fine step is the affine map of the oracle's InflowDiscretization
(boundary closures and per-step inflow forcing), the coarse operators the
periodic Psi truncated to the interval.  MGRIT must take the oracle's
iterations with the same residual histories (to rounding), converge to
sequential stepping, and reproduce Table 5's ERK1 counts.
"""

import json
import os

import numpy as np
import pytest
import torch

from oracle import coarse, inflow, mgrit, rk
from paper_1910_03726_amd import inputs, mgrit as M

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_tables.json")))["table5_inflow"]


def _setup(scheme, nx, nt, m, levels, widths=None, alpha=1.0):
    c = rk.paper_cfl(scheme)
    d = inflow.InflowDiscretization(scheme, nx, c, alpha=alpha)
    H = coarse.build_hierarchy(rk.Discretization(scheme, nx, c, alpha=alpha), m, levels,
                               widths=widths)
    psi = [(h["offsets"], h["weights"]) for h in H]
    G = inputs.sin4_inflow_derivs(nt, d.dt, d.n_derivs())
    return d, c, H, psi, G


def _oracle(d, H, G, m, nt, u0, uinit, tol, maxit, cycle="V", relax="FCF"):
    P = d.dense_phi()
    ops = [lambda X: X @ P.T] + [inflow.truncated_taps_op(h["offsets"], h["weights"])
                                 for h in H]
    MG = mgrit.MGRIT(ops, m, nt, cycle=cycle, relax=relax)
    return MG.solve(u0, uinit, tol, maxit, mgrit.norm_scale(d), g=d.rhs(u0, G))


def test_phi_apply_batch_steps_with_inflow_data():
    s, nx, nt = "ERK3", 256, 64
    d, c, H, psi, G = _setup(s, nx, nt, 4, 2)
    rows = np.stack([inputs.fourier_u0(nx, 4, k) for k in range(3)])
    with M.Plan(nx, nt, c, s, 4, 2, psi, inflow=G) as P:
        x = torch.tensor(rows, device="cuda")
        out = torch.empty_like(x)
        for k in (0, 1, 37, nt):
            P.phi_apply_batch(x, out, k)
            torch.cuda.synchronize()
            ref = np.stack([d.time_stepping(r, G[:k], every=max(k, 1))[-1] for r in rows])
            got = out.cpu().numpy()
            assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)), k
        with pytest.raises(M.MgritError):
            P.phi_apply_batch(x, out, nt + 1)  # beyond the inflow data


LANE_CASES = [
    # scheme, nx, the chunk size the plan picks
    ("ERK1", 1003, 8),   # ragged last chunk
    ("ERK2", 777, 8),
    ("ERK3", 1040, 8),   # right region moved off a wavefront edge
    ("ERK3", 2500, 16),  # several wavefronts, ragged
    ("ERK1", 4096, 16),
    ("ERK3", 4096, 16),
]


@pytest.mark.parametrize("case", LANE_CASES, ids=[f"{c[0]}-{c[1]}" for c in LANE_CASES])
def test_lane_kernel_steps_like_the_oracle(case):
    # the fine level's lane-resident kernel: k steps of the bounded Phi with
    # the inflow forcing, from several start rows
    s, nx, K = case
    nt = 48
    d, c, H, psi, G = _setup(s, nx, nt, 4, 2)
    rows = np.stack([inputs.fourier_u0(nx, 4, k) for k in range(3)])
    rows[1] = inputs.random_iterate(1, nx, 11)[0]
    with M.Plan(nx, nt, c, s, 4, 2, psi, inflow=G) as P:
        assert f"bounded_lanes<K={K}," in P.describe()
        x = torch.tensor(rows, device="cuda")
        out = torch.empty_like(x)
        for k in (0, 1, 8, 37):
            P.phi_apply_batch(x, out, k)
            torch.cuda.synchronize()
            ref = np.stack([d.time_stepping(r, G[:k], every=max(k, 1))[-1] for r in rows])
            got = out.cpu().numpy()
            assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)), (k, s, nx)


@pytest.mark.parametrize("case", LANE_CASES[2:], ids=[f"{c[0]}-{c[1]}" for c in LANE_CASES[2:]])
def test_lane_kernel_full_output(case):
    # the whole space-time solution (out="all"): the converged C-points
    # F-relaxed by the lane-resident kernel, every state of every interval
    # stored (the interior by its lanes, the boundary regions by the extra
    # wavefront), against the oracle's sequential stepping
    s, nx, K = case
    nt, m = 48, 4
    d, c, H, psi, G = _setup(s, nx, nt, m, 2)
    u0 = inputs.fourier_u0(nx, 4, 2)
    with M.Plan(nx, nt, c, s, m, 2, psi, inflow=G) as P:
        assert f"bounded_lanes<K={K}," in P.describe()
        r = P.solve(torch.tensor(u0, device="cuda"), None, tol=1e-13, maxit=60, out="all")
    assert r.status == M.OK
    seq = d.time_stepping(u0, G, every=1)
    got = r.out.cpu().numpy()
    assert got.shape == seq.shape
    assert np.max(np.abs(got - seq)) <= 1e-11 * np.max(np.abs(seq))


CASES = [
    # scheme, nx, nt, m, levels, cycle, relax, widths
    ("ERK1", 256, 1024, 4, 2, "V", "FCF", [3]),
    ("ERK3", 128, 512, 4, 3, "V", "FCF", None),
    ("ERK5", 96, 384, 8, 2, "V", "FCF", None),
    ("ERK3", 200, 800, 4, 3, "F", "FCF", None),
    ("ERK3", 128, 512, 4, 2, "V", "F", None),
    ("ERK5", 1024, 1024, 4, 4, "V", "FCF", None),
    # grids smaller than the two boundary blocks: Phi stored densely
    ("ERK3", 24, 96, 4, 2, "V", "FCF", None),
    ("ERK5", 48, 192, 4, 2, "V", "FCF", None),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}x{c[2]}-m{c[3]}-L{c[4]}-{c[5]}{c[6]}"
                                             for c in CASES])
def test_inflow_mgrit_matches_oracle(case):
    s, nx, nt, m, L, cycle, relax, widths = case
    d, c, H, psi, G = _setup(s, nx, nt, m, L, widths)
    u0 = np.sin(np.pi * (d.x + 1.0)) ** 4
    uinit = inputs.random_iterate(nt // m + 1, nx, 5)
    ref = _oracle(d, H, G, m, nt, u0, uinit, 1e-11, 80, cycle, relax)
    assert ref.status == "converged"
    with M.Plan(nx, nt, c, s, m, L, psi, cycle=cycle, relax=relax, inflow=G) as P:
        assert "bounded" in P.describe()
        r = P.solve(torch.tensor(u0, device="cuda"), torch.tensor(uinit, device="cuda"),
                    tol=1e-11, maxit=80, out="cpoints")
    assert r.status == M.OK
    assert r.iters == ref.iters
    h0 = ref.hist[0]
    for a, b in zip(r.hist, ref.hist):
        assert abs(a - b) <= 1e-9 * h0 + 1e-6 * b
    seq = d.time_stepping(u0, G, every=m)
    got = r.out.cpu().numpy()
    assert np.max(np.abs(got - seq)) <= 1e-10 * np.max(np.abs(seq))


def test_table5_erk1_counts_on_the_gpu():
    nx, nt = 256, 1024
    want = GOLD["ERK1_2e8x2e10_multilevel"]
    for L in range(2, 6):
        d, c, H, psi, G = _setup("ERK1", nx, nt, 4, L, [3, 6, 11, 21][:L - 1])
        u0 = np.sin(np.pi * (d.x + 1.0)) ** 4
        uinit = inputs.random_iterate(nt // 4 + 1, nx, 1)
        with M.Plan(nx, nt, c, "ERK1", 4, L, psi, inflow=G) as P:
            r = P.solve(torch.tensor(u0, device="cuda"), torch.tensor(uinit, device="cuda"),
                        tol=1e-10, maxit=40)
        assert r.iters == want[L - 2], L
    assert GOLD["ERK1_2e8x2e10_two_level"][1] == want[0]


def test_inflow_full_size_against_sequential_stepping():
    # ERK3+U3 4096 x 16384, m = 8, 4-level V-cycles: sampled outputs (the
    # first C-points and the final time) against the oracle's stepping
    s, nx, nt, m, L = "ERK3", 4096, 16384, 8, 4
    d, c, H, psi, G = _setup(s, nx, nt, m, L)
    u0 = np.sin(np.pi * (d.x + 1.0)) ** 4
    with M.Plan(nx, nt, c, s, m, L, psi, inflow=G) as P:
        r = P.solve(torch.tensor(u0, device="cuda"), None, tol=1e-12, maxit=60, out="cpoints")
    assert r.status == M.OK
    C = r.out.cpu().numpy()
    k = 16
    early = d.time_stepping(u0, G[:k * m], every=m)
    assert np.max(np.abs(C[:k + 1] - early)) <= 1e-11
    final = d.time_stepping(u0, G, every=nt)[-1]
    assert np.max(np.abs(C[-1] - final)) <= 1e-10
    # and the discrete solution is third-order close to the exact one
    ex = np.sin(np.pi * (nt * d.dt - (d.x + 1.0))) ** 4
    assert np.max(np.abs(C[-1] - ex)) < 1e-6


def test_inflow_batch_equals_solo():
    specs = [("ERK3", 512, 2048, 4, 3), ("ERK3", 512, 2048, 4, 3), ("ERK1", 256, 1024, 4, 2)]
    plans, u0s, solo = [], [], []
    try:
        for i, (s, nx, nt, m, L) in enumerate(specs):
            d, c, H, psi, G = _setup(s, nx, nt, m, L, alpha=1.0 + 0.1 * i)
            # alpha changes dt (and the data) while keeping c
            plans.append(M.Plan(nx, nt, c, s, m, L, psi, alpha=1.0 + 0.1 * i, inflow=G))
            u0s.append(torch.tensor(inputs.fourier_u0(nx, 4, i), device="cuda"))
        for P, u in zip(plans, u0s):
            P.set_seed(3)
            solo.append(P.solve(u, None, tol=1e-10, maxit=40, out="final"))
        for P in plans:
            P.set_seed(3)
        batch = M.solve_batch(plans, u0s, tol=1e-10, maxit=40, out="final")
        for a, b in zip(solo, batch):
            assert a.status == b.status == M.OK
            assert a.iters == b.iters and a.hist == b.hist
            assert torch.equal(a.out, b.out)
        assert plans[0].stats().batched_launches > 0
    finally:
        for P in plans:
            P.close()


def test_inflow_plan_limits():
    d, c, H, psi, G = _setup("ERK3", 128, 512, 4, 2)
    with pytest.raises(M.MgritError):
        M.Plan(128, 512, c, "ERK3", 4, 2, psi, precision="fp32", inflow=G)
    with pytest.raises(M.MgritError):
        M.Plan(128, 512, 4.0, "SDIRK3", 4, 2, psi, inflow=G)
    with pytest.raises(M.MgritError):  # too few derivative columns
        M.Plan(128, 512, c, "ERK3", 4, 2, psi, inflow=G[:, :3])
    with M.Plan(128, 512, c, "ERK3", 4, 2, psi, inflow=G) as P:
        with pytest.raises(M.MgritError):
            P.set_coarse_solver("spectral")  # Psi is not circulant


def test_wide_window_uses_the_point_kernel():
    # a coarse operator spanning more than 64 points runs on the point-by-
    # point kernel; results as the oracle's
    s, nx, nt, m = "ERK1", 256, 256, 4
    d, c, H, psi, G = _setup(s, nx, nt, m, 2, [3])
    offs = np.array([0, 1, 2, 40, 79])
    w = np.array([0.2, 0.5, 0.25, 0.03, 0.02])
    H = [{"offsets": offs, "weights": w}]
    u0 = np.sin(np.pi * (d.x + 1.0)) ** 4
    uinit = inputs.random_iterate(nt // m + 1, nx, 2)
    ref = _oracle(d, H, G, m, nt, u0, uinit, 1e-11, 80)
    with M.Plan(nx, nt, c, s, m, 2, [(offs, w)], inflow=G) as P:
        assert "L2 n=64: bounded ntaps=5" in P.describe()
        r = P.solve(torch.tensor(u0, device="cuda"), torch.tensor(uinit, device="cuda"),
                    tol=1e-11, maxit=80, out="cpoints")
    assert r.iters == ref.iters
    for a, b in zip(r.hist, ref.hist):
        assert abs(a - b) <= 1e-9 * ref.hist[0] + 1e-6 * b


def test_several_chunks_per_thread():
    # n_x = 8192: the fine level on the lane-resident kernel (512 lanes of
    # 16 points), the coarse levels with more chunks than threads in the
    # register-blocked kernel
    s, nx, nt, m, L = "ERK3", 8192, 512, 4, 3
    d, c, H, psi, G = _setup(s, nx, nt, m, L)
    u0 = np.sin(np.pi * (d.x + 1.0)) ** 4
    with M.Plan(nx, nt, c, s, m, L, psi, inflow=G) as P:
        assert "bounded<K=" in P.describe() and "bounded_lanes<K=16," in P.describe()
        r = P.solve(torch.tensor(u0, device="cuda"), None, tol=1e-12, maxit=60, out="final")
    assert r.status == M.OK
    ref = d.time_stepping(u0, G, every=nt)[-1]
    assert np.max(np.abs(r.out.cpu().numpy()[0] - ref)) <= 1e-10


def test_chunked_coarsest_sweep_equals_the_sweep_bit_for_bit():
    # the truncated coarsest Psi of the 4096 x 16384 ERK3 V-cycle has every
    # offset >= 1, so Psi^q = 0: the chunked sweep gives the same values
    s, nx, nt, m, L = "ERK3", 4096, 16384, 8, 4
    d, c, H, psi, G = _setup(s, nx, nt, m, L)
    u0 = torch.tensor(np.sin(np.pi * (d.x + 1.0)) ** 4, device="cuda")
    res = {}
    with M.Plan(nx, nt, c, s, m, L, psi, inflow=G) as P:
        assert "(chunked sweep)" in P.describe()
        for mode in ("auto", "sweep"):
            P.set_coarse_solver(mode)
            assert ("(chunked sweep)" in P.describe()) == (mode == "auto")
            P.set_seed(4)
            res[mode] = P.solve(u0, None, tol=1e-12, maxit=60, out="cpoints")
    a, b = res["auto"], res["sweep"]
    assert a.status == b.status == M.OK
    assert a.iters == b.iters and a.hist == b.hist
    assert torch.equal(a.out, b.out)

