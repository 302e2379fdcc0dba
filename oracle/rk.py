"""Spatial and temporal discretizations of u_t + alpha u_x = 0 (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Everything here follows Sec. 2.1 of the paper and its Appendix A:

* the grid has n_x unknowns on the periodic interval [-1, 1), spacing
  dx = 2/n_x (the n_x+1 points of Sec. 2.1 with the last one identified with
  the first by periodicity);
* the p-th order upwind formula Up approximates v'(x_i) by
  (1/dx) * sum_j d_j v_{i+j}; the semi-discrete operator L of eq. (2) is the
  discretization of -alpha d/dx, so (L u)_i = -(alpha/dx) sum_j d_j u_{i+j};
* a Runge-Kutta method with Butcher tableau (A, b, c) advances u' = L u by
  one step dt (eq. (3)); the CFL number is c = alpha dt / dx (eq. (5)).

Arrays holding several state vectors are shaped (batch, n_x) and every
operation acts on the last axis.
"""

import numpy as np

# ---------------------------------------------------------------------------
# Upwind stencils U1-U5 (Sec. 2.1, formulas tagged U1..U5).
# Map: offset j -> coefficient d_j in  v'_i ~ (1/dx) sum_j d_j v_{i+j},
# written as exact fractions (numerator, denominator).
# ---------------------------------------------------------------------------
UPWIND_FRACTIONS = {
    1: {0: (1, 1), -1: (-1, 1)},
    2: {0: (3, 2), -1: (-4, 2), -2: (1, 2)},
    3: {1: (2, 6), 0: (3, 6), -1: (-6, 6), -2: (1, 6)},
    4: {1: (3, 12), 0: (10, 12), -1: (-18, 12), -2: (6, 12), -3: (-1, 12)},
    5: {2: (-3, 60), 1: (30, 60), 0: (20, 60), -1: (-60, 60), -2: (15, 60),
        -3: (-2, 60)},
}
UPWIND = {p: {j: n / d for j, (n, d) in c.items()} for p, c in UPWIND_FRACTIONS.items()}

LD = np.longdouble  # x86 extended precision: 64-bit significand


def _frac_ld(n, d):
    return LD(n) / LD(d)


def _tableaux(frac, sqrt, sdirk3_root, dtype):
    """Butcher tableaux of Appendix A, Table 7 (ERK1-ERK5) and Table 8
    (SDIRK1-SDIRK4), with every entry built by frac(p, q) = p/q, sqrt and the
    SDIRK3 constant in one number type (FP64 or extended precision)."""
    def tab(rows, b):
        s = len(b)
        A = np.zeros((s, s), dtype=dtype)
        for i, row in enumerate(rows):
            for j, v in enumerate(row):
                A[i, j] = v
        b = np.array(b, dtype=dtype)
        return A, b, A.sum(axis=1)

    f = frac
    one, zero = f(1, 1), f(0, 1)
    r2 = sqrt(2) / f(2, 1)
    z = sdirk3_root
    # SDIRK3 (Table 8): the other constants are polynomials in z
    be = (one - z) / f(2, 1)
    ga = f(-3, 2) * z * z + f(4, 1) * z - f(1, 4)
    ep = f(3, 2) * z * z - f(5, 1) * z + f(5, 4)
    return {
        "ERK1": tab([[zero]], [one]),
        "ERK2": tab([[zero], [one, zero]], [f(1, 2), f(1, 2)]),
        "ERK3": tab([[zero], [one], [f(1, 4), f(1, 4)]], [f(1, 6), f(1, 6), f(2, 3)]),
        "ERK4": tab([[zero], [f(1, 2)], [zero, f(1, 2)], [zero, zero, one]],
                    [f(1, 6), f(1, 3), f(1, 3), f(1, 6)]),
        "ERK5": tab(
            [[zero],
             [f(1, 4)],
             [f(1, 8), f(1, 8)],
             [zero, zero, f(1, 2)],
             [f(3, 16), f(-3, 8), f(3, 8), f(9, 16)],
             [f(-3, 7), f(8, 7), f(6, 7), f(-12, 7), f(8, 7)]],
            [f(7, 90), zero, f(32, 90), f(12, 90), f(32, 90), f(7, 90)]),
        "SDIRK1": tab([[one]], [one]),
        "SDIRK2": tab([[one - r2], [r2, one - r2]], [r2, one - r2]),
        "SDIRK3": tab([[z], [be, z], [ga, ep, z]], [ga, ep, z]),
        "SDIRK4": tab(
            [[f(1, 4)],
             [f(1, 2), f(1, 4)],
             [f(17, 50), f(-1, 25), f(1, 4)],
             [f(371, 1360), f(-137, 2720), f(15, 544), f(1, 4)],
             [f(25, 24), f(-49, 48), f(125, 16), f(-85, 12), f(1, 4)]],
            [f(25, 24), f(-49, 48), f(125, 16), f(-85, 12), f(1, 4)]),
    }


# The SDIRK3 diagonal (Table 8), to the 20 digits printed.
SDIRK3_ROOT = "0.43586652150845899942"

# FP64 tableaux (the staged stepper below) and extended-precision ones (the
# closed form of Lemma 1, spectral_propagate).
TABLEAUX = _tableaux(lambda p, q: p / q, lambda x: np.sqrt(float(x)), float(SDIRK3_ROOT),
                     float)
TABLEAUX_LD = _tableaux(_frac_ld, lambda x: np.sqrt(LD(x)), LD(SDIRK3_ROOT), LD)

# CFL limits printed in Table 1 (ERKp+Up).
CFL_MAX_TABLE1 = {1: 1.0, 2: 0.5, 3: 1.62589, 4: 1.04449, 5: 1.96583}


def scheme_order(scheme):
    """'ERK3' -> 3, 'SDIRK2' -> 2 (the scheme name carries its order p)."""
    return int(scheme[-1])


def is_implicit(scheme):
    return scheme.startswith("SDIRK")


class Discretization:
    """ERKp+Up or SDIRKp+Up for u_t + alpha u_x = 0 on n_x periodic points.

    ``cfl`` is the Courant number c = alpha dt/dx of eq. (5).
    """

    def __init__(self, scheme, nx, cfl, alpha=1.0):
        self.scheme = scheme
        self.p = scheme_order(scheme)
        self.nx = int(nx)
        self.alpha = float(alpha)
        self.cfl = float(cfl)
        self.dx = 2.0 / self.nx
        self.dt = self.cfl * self.dx / self.alpha
        self.A, self.b, self.c = TABLEAUX[scheme]
        self.stencil = UPWIND[self.p]
        self.x = -1.0 + self.dx * np.arange(self.nx)

    # -- the semi-discrete operator L of eq. (2) -------------------------
    def apply_L(self, u):
        """(L u)_i = -(alpha/dx) sum_j d_j u_{i+j}, periodic in i."""
        out = np.zeros_like(u)
        for j, d in self.stencil.items():
            # np.roll(u, -j)[..., i] == u[..., i + j]
            out += d * np.roll(u, -j, axis=-1)
        return -(self.alpha / self.dx) * out

    def symbol_L(self, theta):
        """Eigenvalue of L on the Fourier mode exp(i k x_i pi), theta = k pi dx.

        L is circulant, so (L e)_i = l(theta) e_i with
        l(theta) = -(alpha/dx) sum_j d_j exp(i j theta).
        """
        theta = np.asarray(theta, dtype=float)
        s = np.zeros(theta.shape, dtype=complex)
        for j, d in self.stencil.items():
            s += d * np.exp(1j * j * theta)
        return -(self.alpha / self.dx) * s

    def solve_shifted(self, rhs, shift):
        """Solve (I - shift * L) y = rhs exactly (periodic, via the DFT).

        L is circulant and hence diagonalized by the DFT (Sec. 2.1), so the
        solve is a division by 1 - shift * l(theta_k) in Fourier space.
        """
        theta = 2.0 * np.pi * np.fft.fftfreq(self.nx)
        # fftfreq gives k/n for k in [-n/2, n/2); theta_k = 2 pi k / n.
        sym = 1.0 - shift * self.symbol_L(theta)
        return np.real(np.fft.ifft(np.fft.fft(rhs, axis=-1) / sym, axis=-1))

    # -- one Runge-Kutta step, eq. (3) ------------------------------------
    def step(self, u, dt=None):
        """u^{n+1} = Phi u^n by the stages of the Butcher tableau.

        Explicit: k_i = L(u + dt sum_{j<i} a_ij k_j).
        Diagonally implicit: (I - dt a_ii L) Y_i = u + dt sum_{j<i} a_ij L Y_j,
        k_i = L Y_i.  In both cases u^{n+1} = u + dt sum_i b_i k_i.
        """
        dt = self.dt if dt is None else float(dt)
        A, b = self.A, self.b
        s = len(b)
        ks = []
        for i in range(s):
            rhs = u.copy()
            for j in range(i):
                if A[i, j] != 0.0:
                    rhs = rhs + dt * A[i, j] * ks[j]
            if A[i, i] != 0.0:
                Y = self.solve_shifted(rhs, dt * A[i, i])
            else:
                Y = rhs
            ks.append(self.apply_L(Y))
        out = u.copy()
        for i in range(s):
            if b[i] != 0.0:
                out = out + dt * b[i] * ks[i]
        return out

    def propagate(self, u, nsteps, dt=None):
        for _ in range(int(nsteps)):
            u = self.step(u, dt)
        return u

    def time_stepping(self, u0, nt, every=1):
        """Sequential time-stepping, eq. (3): returns u^0, u^every, ...

        This is the exact discrete solution of the space-time system that
        MGRIT and Parareal converge to (Sec. 2.2).
        """
        u = np.array(u0, dtype=float)
        out = [u.copy()]
        for n in range(1, int(nt) + 1):
            u = self.step(u)
            if n % every == 0:
                out.append(u.copy())
        return np.array(out)

    # -- Lemma 1: Phi = R(dt L) ---------------------------------------------
    def stability_function(self, z):
        """R(z) = 1 + z b^T (I - z A)^{-1} 1 for the tableau (Lemma 1)."""
        return stability_function(self.A, self.b, z)

    def eigenvalues(self, nx=None, dt=None):
        """lambda_k = R(dt * l(theta_k)), theta_k = 2 pi k / n_x (Lemma 1).

        Ordered like numpy's DFT of the first column: k = 0, 1, ..., n_x-1.
        """
        n = self.nx if nx is None else int(nx)
        dt = self.dt if dt is None else float(dt)
        theta = 2.0 * np.pi * np.arange(n) / n
        # l(theta) uses this object's dx; only n_x = self.nx is meaningful.
        return self.stability_function(dt * self.symbol_L(theta))

    def spectral_propagate(self, u0, nsteps):
        """Phi^n u0 in closed form, in extended precision.

        Phi is circulant with eigenvalue lambda_k = R(dt l(theta_k)) on the
        DFT mode k (Lemma 1), so Phi^n u0 = F^{-1} diag(lambda^n) F u0.  The
        whole evaluation runs in x86 extended precision (64-bit significand,
        eps = 1.1e-19) from the exact stencil fractions and tableau entries:
        the angles 2 pi (j k mod n_x)/n_x, the symbol, R(z) by forward
        substitution (A is lower triangular), lambda^n by repeated squaring
        (relative error ~ n eps) and the transforms; the result is rounded
        to FP64 once.  It is the exact discrete solution of eq. (3) to
        ~1e-14 relative for n <= 65536, where FP64 stepping drifts by the
        rounding of its constants.
        """
        n = self.nx
        pi = np.arccos(LD(-1))
        k = np.arange(n)
        sym = np.zeros(n, dtype=np.clongdouble)
        for j, (num, den) in UPWIND_FRACTIONS[self.p].items():
            ang = (LD(2) * pi / LD(n)) * ((j * k) % n).astype(LD)
            sym += _frac_ld(num, den) * (np.cos(ang) + 1j * np.sin(ang))
        # dt l(theta) = -(alpha dt/dx) sum_j d_j e^{ij theta} = -c sum_j ...
        z = -(LD(self.alpha) * LD(self.dt) / LD(self.dx)) * sym
        A, b, _ = TABLEAUX_LD[self.scheme]
        y = []
        acc = np.zeros(n, dtype=np.clongdouble)
        for i in range(len(b)):
            r = np.ones(n, dtype=np.clongdouble)
            for j in range(i):
                if A[i, j] != 0:
                    r = r + z * A[i, j] * y[j]
            y.append(r / (1 - z * A[i, i]))
            acc = acc + b[i] * y[i]
        lam = 1 + z * acc
        p = np.ones(n, dtype=np.clongdouble)
        base = lam
        e = int(nsteps)
        while e:
            if e & 1:
                p = p * base
            base = base * base
            e >>= 1
        U = np.fft.fft(np.asarray(u0, dtype=LD), axis=-1)
        return np.real(np.fft.ifft(p * U, axis=-1)).astype(np.float64)

    def dense_phi(self):
        """Phi as a dense n_x x n_x matrix, built from the block form of the
        Runge-Kutta step rather than by stepping:
        with Z = dt L,  K = (I - A (x) Z)^{-1} (1 (x) Z) u,
        Phi = I + (b^T (x) I) (I - A (x) Z)^{-1} (1 (x) Z).
        """
        n = self.nx
        Lm = np.zeros((n, n))
        for j, d in self.stencil.items():
            for i in range(n):
                Lm[i, (i + j) % n] += -(self.alpha / self.dx) * d
        Z = self.dt * Lm
        s = len(self.b)
        big = np.eye(s * n) - np.kron(self.A, Z)
        ones = np.kron(np.ones((s, 1)), Z)
        K = np.linalg.solve(big, ones)
        return np.eye(n) + np.kron(self.b.reshape(1, s), np.eye(n)) @ K


def stability_function(A, b, z):
    """R(z) = 1 + z b^T (I - zA)^{-1} 1 for scalar or array z."""
    z = np.asarray(z, dtype=complex)
    s = len(b)
    flat = z.reshape(-1)
    out = np.empty(flat.shape, dtype=complex)
    one = np.ones(s)
    for idx, zz in enumerate(flat):
        out[idx] = 1.0 + zz * b @ np.linalg.solve(np.eye(s) - zz * A, one)
    return out.reshape(z.shape)


def stability_polynomial_coeffs(scheme):
    """Coefficients of R(z) = sum_k g_k z^k for an explicit tableau:
    g_0 = 1, g_k = b^T A^{k-1} 1 (k >= 1)."""
    A, b, _ = TABLEAUX[scheme]
    s = len(b)
    g = [1.0]
    v = np.ones(s)
    for _ in range(s):
        g.append(float(b @ v))
        v = A @ v
    return np.array(g)


def max_amplification(scheme, cfl, ntheta=20001):
    """max over theta in [0, pi] of |R(c * sym(theta))| for ERKp+Up."""
    p = scheme_order(scheme)
    A, b, _ = TABLEAUX[scheme]
    theta = np.linspace(0.0, np.pi, ntheta)
    s = np.zeros(theta.shape, dtype=complex)
    for j, d in UPWIND[p].items():
        s += d * np.exp(1j * j * theta)
    z = -cfl * s
    if not is_implicit(scheme):
        g = stability_polynomial_coeffs(scheme)
        R = np.polyval(g[::-1], z)
    else:
        R = stability_function(A, b, z)
    return float(np.max(np.abs(R)))


def cfl_limit(scheme, slack=0.0, ntheta=20001, hi=4.0):
    """Largest c with max_theta |R(z(theta; c))| <= 1 + slack (eq. (5)).

    Bisection on c over a fine theta grid.  ``slack`` loosens the test
    |R| <= 1; Table 1's ERK5+U5 entry needs slack ~ 3.3e-7 (see tests).
    """
    lo = 1e-6
    assert max_amplification(scheme, lo, ntheta) <= 1.0 + slack + 1e-12
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if max_amplification(scheme, mid, ntheta) <= 1.0 + slack:
            lo = mid
        else:
            hi = mid
    return lo


def paper_cfl(scheme, fraction=0.85):
    """The CFL number used in the paper's experiments (Sec. 2.1): 85% of the
    Table 1 limit for ERK, c = 4 for SDIRK."""
    if is_implicit(scheme):
        return 4.0
    return fraction * CFL_MAX_TABLE1[scheme_order(scheme)]


def paper_nt(scheme, nx, cfl):
    """Largest power of two n_t with T = n_t dt <= 8 (Sec. 2.2 set-up)."""
    dt = cfl * (2.0 / nx)
    nt = 1
    while (2 * nt) * dt <= 8.0 + 1e-12:
        nt *= 2
    return nt
