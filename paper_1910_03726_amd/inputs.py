"""Seeded synthetic inputs for MGRIT/Parareal on periodic linear advection.

This module holds no arithmetic of the method: it only draws the seeded
initial conditions and initial iterates that both the HIP path and the
CPU oracle are given, and names the workloads by their sizes.

Inputs (the paper's workload is itself synthetic, Sec. 2.1):
* grid x_i = -1 + i dx, dx = 2/n_x, periodic (Sec. 2.1);
* u0 = sum_{k=1}^{K} k^{-decay} (a_k cos(pi k x) + b_k sin(pi k x)),
  a_k, b_k ~ N(0, 1) from numpy's PCG64 ``default_rng(seed)``; the paper's
  own u0 = sin^4(pi x) is available as ``sin4``;
* initial iterate: uniform U[0, 1) at every C-point except t = 0
  (Sec. 2.2 set-up), from ``default_rng(seed)``.
"""

import numpy as np


def grid(nx):
    return -1.0 + (2.0 / nx) * np.arange(nx)


def fourier_u0(nx, nmodes, seed, decay=0.0):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(nmodes)
    b = rng.standard_normal(nmodes)
    x = grid(nx)
    u = np.zeros(nx)
    for k in range(1, nmodes + 1):
        amp = float(k) ** (-decay)
        u += amp * (a[k - 1] * np.cos(np.pi * k * x)
                    + b[k - 1] * np.sin(np.pi * k * x))
    return u


def sin4(nx):
    return np.sin(np.pi * grid(nx)) ** 4


def inflow_grid(nx):
    """Unknowns of the inflow/outflow problem: x_i = -1 + i dx, i = 1..n_x."""
    return -1.0 + (2.0 / nx) * np.arange(1, nx + 1)


def sin4_inflow_derivs(nt, dt, nderiv, t0=0.0):
    """Inflow data g(t) = sin^4(pi t) at x = -1: row n holds g^(d)(t0 + n dt),
    d = 0..nderiv-1, n = 0..nt-1 (sin^4 = 3/8 - cos(2 pi t)/2 + cos(4 pi t)/8)."""
    t = t0 + dt * np.arange(nt)
    out = np.empty((nt, nderiv))
    for d in range(nderiv):
        ph = d * np.pi / 2
        v = (-0.5 * (2 * np.pi) ** d * np.cos(2 * np.pi * t + ph)
             + 0.125 * (4 * np.pi) ** d * np.cos(4 * np.pi * t + ph))
        out[:, d] = v + (0.375 if d == 0 else 0.0)
    return out


def poly_inflow_derivs(coeffs, nt, dt, nderiv):
    """Inflow data g(t) = sum_k coeffs[k] t^k: row n holds g^(d)(n dt)."""
    t = dt * np.arange(nt)
    out = np.zeros((nt, nderiv))
    for d in range(nderiv):
        for k in range(d, len(coeffs)):
            out[:, d] += coeffs[k] * (np.prod(np.arange(k - d + 1, k + 1)) if d else 1.0) * t ** (k - d)
    return out


def random_iterate(npoints, nx, seed):
    """U[0,1) values for ``npoints`` time levels (row 0 is replaced by u0)."""
    return np.random.default_rng(seed).random((npoints, nx))


def splitmix_iterate(npoints, nx, seed):
    """U[0,1) values of the splitmix64 stream (Steele, Lea & Flood, 2014):
    value i = mix(seed + (i+1) * 0x9E3779B97F4A7C15) >> 11, times 2^-53.
    The same counter-based stream fills the initial iterate on the device
    when none is passed in."""
    with np.errstate(over="ignore"):
        i = np.arange(npoints * nx, dtype=np.uint64)
        z = np.uint64(seed) + (i + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return ((z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
            ).reshape(npoints, nx)


# Courant numbers c = alpha dt/dx of the workloads.  ERK: 85% of the Table 1
# CFL limit (1, 1/2, 1.62589, 1.04449, 1.96583); SDIRK: c = 4 (Sec. 2.1).
CFL_LIMIT_TABLE1 = {1: 1.0, 2: 0.5, 3: 1.62589, 4: 1.04449, 5: 1.96583}


def erk_cfl(p, fraction=0.85):
    return fraction * CFL_LIMIT_TABLE1[p]


# The four single-solve workloads (sizes, scheme, solver shape, seeds).
# psi_rule: "window" (contiguous window, Sec. 4.4 width rule, or psi_widths),
# "eta" (SDIRK thresholding, Sec. 4.6), "bound" (window widths chosen per
# level until the eq. (7) bound reaches psi_target).
WORKLOADS = {
    "erk1_u1_nx64_nt256_m4_2level": dict(
        scheme="ERK1", nx=64, nt=256, cfl=erk_cfl(1), m=4, levels=2,
        cycle="V", precision="fp64", psi_rule="window", psi_widths=[3],
        u0=dict(nmodes=4, decay=0.0, seed=0), init_seed=1),
    "erk3_u3_nx4096_nt16384_m8_fcycle": dict(
        scheme="ERK3", nx=4096, nt=16384, cfl=erk_cfl(3), m=8, levels=4,
        cycle="F", precision="fp64", psi_rule="bound", psi_widths=None, psi_target=1e-3,
        u0=dict(nmodes=8, decay=2.0, seed=0), init_seed=1),
    "sdirk3_u3_nx2048_nt8192_m16_2level": dict(
        scheme="SDIRK3", nx=2048, nt=8192, cfl=4.0, m=16, levels=2,
        cycle="V", precision="fp64", psi_rule="eta", psi_widths=None,
        u0=dict(nmodes=8, decay=0.0, seed=0), init_seed=1),
    "erk5_u5_nx8192_nt65536_m8_fp32relax": dict(
        scheme="ERK5", nx=8192, nt=65536, cfl=erk_cfl(5), m=8, levels=5,
        cycle="V", precision="fp32", psi_rule="bound", psi_widths=None, psi_target=1e-3,
        u0=dict(nmodes=16, decay=0.0, seed=0), init_seed=1),
    # inflow/outflow boundaries (Sec. 4.5): u(-1, t) = sin^4(pi t), u0 the
    # exact solution's initial profile, the periodic Psi truncated
    "erk3_u3_inflow_nx4096_nt16384_m8_vcycle": dict(
        scheme="ERK3", nx=4096, nt=16384, cfl=erk_cfl(3), m=8, levels=4,
        cycle="V", precision="fp64", psi_rule="window", psi_widths=None,
        boundary="inflow", init_seed=1),
}


def workload_u0(w):
    if w.get("boundary") == "inflow":
        return np.sin(np.pi * (inflow_grid(w["nx"]) + 1.0)) ** 4
    return fourier_u0(w["nx"], w["u0"]["nmodes"], w["u0"]["seed"],
                      w["u0"]["decay"])


def workload_inflow(w, alpha=1.0):
    """Inflow data rows of an inflow workload (sin^4(pi t), derivatives 0..p)."""
    p = int(w["scheme"][-1])
    dt = w["cfl"] * (2.0 / w["nx"]) / alpha
    return sin4_inflow_derivs(w["nt"], dt, p + 1)


def serving_requests(n, seed=7, nx_exps=range(8, 14), nt_exps=range(10, 16),
                     orders=(1, 3, 5), ms=(4, 8)):
    """The serving mix: n requests with n_x = 2^a (a in nx_exps), n_t = 2^b
    (b in nt_exps), ERKp+Up with p in orders, CFL fraction U[0.5, 0.9] of the
    Table 1 limit rounded to 0.01 (clients pick the Courant number from a
    menu of 41 values), m in ms, FP32 relaxation or FP64 with probability
    1/2 each, u0 = 8 seeded Fourier modes, and a seed for the initial
    iterate.  Arrival times are drawn separately (``poisson_arrivals``)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        p = int(rng.choice(orders))
        frac = round(float(rng.uniform(0.5, 0.9)), 2)
        out.append(dict(
            nx=int(2 ** rng.choice(list(nx_exps))),
            nt=int(2 ** rng.choice(list(nt_exps))),
            scheme=f"ERK{p}", p=p, cfl=erk_cfl(p, frac), cfl_fraction=frac,
            m=int(rng.choice(ms)),
            precision="fp32" if rng.random() < 0.5 else "fp64",
            u0_seed=int(rng.integers(1 << 31)), init_seed=int(rng.integers(1, 1 << 62))))
    return out


def poisson_arrivals(n, rate, seed=7):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed + 1)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def request_u0(req):
    return fourier_u0(req["nx"], 8, req["u0_seed"])
