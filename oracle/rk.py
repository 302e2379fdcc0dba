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
# Map: offset j -> coefficient d_j in  v'_i ~ (1/dx) sum_j d_j v_{i+j}.
# ---------------------------------------------------------------------------
UPWIND = {
    1: {0: 1.0, -1: -1.0},
    2: {0: 3.0 / 2.0, -1: -4.0 / 2.0, -2: 1.0 / 2.0},
    3: {1: 2.0 / 6.0, 0: 3.0 / 6.0, -1: -6.0 / 6.0, -2: 1.0 / 6.0},
    4: {1: 3.0 / 12.0, 0: 10.0 / 12.0, -1: -18.0 / 12.0, -2: 6.0 / 12.0,
        -3: -1.0 / 12.0},
    5: {2: -3.0 / 60.0, 1: 30.0 / 60.0, 0: 20.0 / 60.0, -1: -60.0 / 60.0,
        -2: 15.0 / 60.0, -3: -2.0 / 60.0},
}


def _tableau(rows, b):
    s = len(b)
    A = np.zeros((s, s))
    for i, row in enumerate(rows):
        A[i, :len(row)] = row
    b = np.asarray(b, dtype=float)
    return A, b, A.sum(axis=1)


def _sdirk3():
    # Appendix A, Table 8: constants of the 3-stage, 3rd-order SDIRK method.
    z = 0.43586652150845899942
    al = (1.0 + z) / 2.0
    be = (1.0 - z) / 2.0
    ga = -1.5 * z * z + 4.0 * z - 0.25
    ep = 1.5 * z * z - 5.0 * z + 1.25
    A, b, c = _tableau([[z], [be, z], [ga, ep, z]], [ga, ep, z])
    assert abs(c[1] - al) < 1e-15
    return A, b, c


_R2 = np.sqrt(2.0) / 2.0

# Butcher tableaux: Appendix A, Table 7 (ERK1-ERK5) and Table 8 (SDIRK1-4).
TABLEAUX = {
    "ERK1": _tableau([[0.0]], [1.0]),
    "ERK2": _tableau([[0.0], [1.0, 0.0]], [0.5, 0.5]),
    "ERK3": _tableau([[0.0], [1.0], [0.25, 0.25]],
                     [1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0]),
    "ERK4": _tableau([[0.0], [0.5], [0.0, 0.5], [0.0, 0.0, 1.0]],
                     [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]),
    "ERK5": _tableau(
        [[0.0],
         [1.0 / 4.0],
         [1.0 / 8.0, 1.0 / 8.0],
         [0.0, 0.0, 1.0 / 2.0],
         [3.0 / 16.0, -3.0 / 8.0, 3.0 / 8.0, 9.0 / 16.0],
         [-3.0 / 7.0, 8.0 / 7.0, 6.0 / 7.0, -12.0 / 7.0, 8.0 / 7.0]],
        [7.0 / 90.0, 0.0, 32.0 / 90.0, 12.0 / 90.0, 32.0 / 90.0, 7.0 / 90.0]),
    "SDIRK1": _tableau([[1.0]], [1.0]),
    "SDIRK2": _tableau([[1.0 - _R2], [_R2, 1.0 - _R2]], [_R2, 1.0 - _R2]),
    "SDIRK3": _sdirk3(),
    "SDIRK4": _tableau(
        [[1.0 / 4.0],
         [1.0 / 2.0, 1.0 / 4.0],
         [17.0 / 50.0, -1.0 / 25.0, 1.0 / 4.0],
         [371.0 / 1360.0, -137.0 / 2720.0, 15.0 / 544.0, 1.0 / 4.0],
         [25.0 / 24.0, -49.0 / 48.0, 125.0 / 16.0, -85.0 / 12.0, 1.0 / 4.0]],
        [25.0 / 24.0, -49.0 / 48.0, 125.0 / 16.0, -85.0 / 12.0, 1.0 / 4.0]),
}

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
        """Phi^n u0 in closed form: Phi is circulant with eigenvalues lambda_k
        on the DFT modes (Lemma 1), so Phi^n u0 = F^{-1} diag(lambda^n) F u0.

        lambda^n is formed by repeated squaring; its relative rounding grows
        like n * eps, so this is for long horizons where stepping is slow.
        """
        lam = self.eigenvalues()
        p = np.ones_like(lam)
        base = lam.copy()
        n = int(nsteps)
        while n:
            if n & 1:
                p = p * base
            base = base * base
            n >>= 1
        return np.real(np.fft.ifft(p * np.fft.fft(u0, axis=-1), axis=-1))

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
