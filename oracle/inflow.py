"""Inflow/outflow boundaries for the ERK+U discretizations (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Sec. 4.5 replaces the periodic interval by [-1, 1] with inflow data
u(-1, t) = g(t) at x = -1 and no condition at the outflow x = 1.  It names
the ingredients and not the formulas; the readings taken here:

* grid: unknowns at x_i = -1 + i dx, i = 1..n_x, dx = 2/n_x (x_0 = -1 is
  the inflow point, whose value is prescribed; x_{n_x} = 1 is the last
  unknown).  Array index a = i - 1.
* the same Up stencil at every unknown; it reaches r_l points to the left
  and r_r to the right, so points outside the grid are ghosts.
* outflow ghosts x_{n_x+e}: the polynomial of degree p-1 through the last p
  unknowns, evaluated there (p-th order extrapolation).
* inflow ghosts x_{-k} (k = 0 is the inflow point itself): truncated Taylor
  series about x = -1 whose space derivatives are traded for time
  derivatives by the PDE (inverse Lax-Wendroff):
  d^r u/dx^r = (-1/alpha)^r d^r u/dt^r, so
  u(-1 - k dx) = sum_r (k dx/alpha)^r / r! g^(r).
* stage values at the inflow (Carpenter et al.): the stage U_j of an ERK
  step is P_j(dt L) u^n with P_1 = 1 and P_j(z) = 1 + z sum_k a_jk P_k(z);
  since d/dt acts as L on the exact solution, the boundary value of stage
  j is sum_q gamma_jq dt^q g^(q)(t_n) with gamma_jq the coefficients of
  P_j.  Combined with the Taylor series above, ghost k of stage j is
  sum_{q + r <= p} gamma_jq dt^q (k dx/alpha)^r / r! g^(q+r)(t_n).
* the inflow data enter only through g^(d)(t_n), d = 0..p (one row per
  step, given by the caller).

The step is affine: u^{n+1} = Phi u^n + f^{n+1} with Phi the step for
g = 0 and f^{n+1} the step of the zero state with the data of t_n.
"""

import math

import numpy as np

from .rk import TABLEAUX, UPWIND, scheme_order


def stage_polynomials(A):
    """gamma[j][q]: coefficients of P_j(z) = 1 + z sum_{k<j} a_jk P_k(z)."""
    s = A.shape[0]
    P = []
    for j in range(s):
        c = np.zeros(s)
        c[0] = 1.0
        for k in range(j):
            if A[j, k] != 0.0:
                c[1:] += A[j, k] * P[k][:-1]
        P.append(c)
    return np.array(P)


def extrapolation_weights(p, e):
    """Weights on the last p unknowns (oldest first) of the degree p-1
    polynomial through them, evaluated e points beyond the last one."""
    t = np.arange(p, dtype=float) - (p - 1)
    w = np.ones(p)
    for i in range(p):
        for k in range(p):
            if k != i:
                w[i] *= (e - t[k]) / (t[i] - t[k])
    return w


class InflowDiscretization:
    """ERKp+Up for u_t + alpha u_x = 0 on (-1, 1] with inflow at x = -1."""

    def __init__(self, scheme, nx, cfl, alpha=1.0):
        if not scheme.startswith("ERK"):
            raise ValueError("inflow/outflow boundaries are for ERK schemes (Sec. 4.5)")
        self.scheme = scheme
        self.p = scheme_order(scheme)
        self.nx = int(nx)
        self.alpha = float(alpha)
        self.cfl = float(cfl)
        self.dx = 2.0 / self.nx
        self.dt = self.cfl * self.dx / self.alpha
        self.A, self.b, self.c = TABLEAUX[scheme]
        self.stencil = UPWIND[self.p]
        self.rl = -min(self.stencil)          # reach to the left
        self.rr = max(0, max(self.stencil))   # reach to the right
        self.x = -1.0 + self.dx * np.arange(1, self.nx + 1)
        self.gamma = stage_polynomials(self.A)
        self.ext = [extrapolation_weights(self.p, e) for e in range(1, self.rr + 1)]

    def n_derivs(self):
        """Rows of inflow data per step: g^(d)(t_n), d = 0..p."""
        return self.p + 1

    def inflow_ghosts(self, j, gd):
        """Ghost values x_0, x_{-1}, ... (k = 0..r_l-1) of stage j."""
        out = np.zeros(self.rl)
        if gd is None:
            return out
        p = self.p
        for k in range(self.rl):
            tot = 0.0
            for q in range(min(j, p) + 1):
                for r in range(p - q + 1):
                    tot += (self.gamma[j][q] * self.dt ** q
                            * (k * self.dx / self.alpha) ** r / math.factorial(r)
                            * gd[q + r])
            out[k] = tot
        return out

    def apply_L(self, U, left):
        """(L U)_a = -(alpha/dx) sum_o d_o U_{a+o} with ghosts (one state)."""
        nx = self.nx
        right = np.array([w @ U[nx - self.p:] for w in self.ext])
        # padded[rl + a] = U_a; padded[rl - 1 - k] = left ghost k
        padded = np.concatenate([left[::-1], U, right])
        out = np.zeros(nx)
        for o, d in self.stencil.items():
            out += d * padded[self.rl + o: self.rl + o + nx]
        return -(self.alpha / self.dx) * out

    def step(self, u, gd=None):
        """One ERK step from t_n; gd: g^(d)(t_n), d = 0..p (None: g = 0)."""
        u = np.asarray(u, dtype=float)
        ks = []
        for j in range(len(self.b)):
            U = u.copy()
            for k in range(j):
                if self.A[j, k] != 0.0:
                    U = U + self.dt * self.A[j, k] * ks[k]
            ks.append(self.apply_L(U, self.inflow_ghosts(j, gd)))
        out = u.copy()
        for j in range(len(self.b)):
            if self.b[j] != 0.0:
                out = out + self.dt * self.b[j] * ks[j]
        return out

    def dense_phi(self):
        """Phi (the step for g = 0) column by column."""
        n = self.nx
        P = np.empty((n, n))
        for c in range(n):
            e = np.zeros(n)
            e[c] = 1.0
            P[:, c] = self.step(e)
        return P

    def forcing(self, gd):
        """f^{n+1} = step of the zero state with the inflow data of t_n."""
        return self.step(np.zeros(self.nx), gd)

    def time_stepping(self, u0, G, every=1):
        """Sequential stepping with inflow data rows G[n] (n = 0..n_t-1):
        u^0, u^every, ... (the exact discrete solution)."""
        u = np.array(u0, dtype=float)
        out = [u.copy()]
        for n in range(G.shape[0]):
            u = self.step(u, G[n])
            if (n + 1) % every == 0:
                out.append(u.copy())
        return np.array(out)

    def rhs(self, u0, G):
        """Right-hand side of the space-time system (eq. (3) with inflow):
        g^0 = u^0, g^{n+1} = f^{n+1}."""
        g = np.empty((G.shape[0] + 1, self.nx))
        g[0] = u0
        for n in range(G.shape[0]):
            g[n + 1] = self.forcing(G[n])
        return g


def truncated_taps_op(offsets, weights):
    """The coarse operator Psi truncated at the boundaries (Sec. 4.5):
    (Psi u)_a = sum_t w_t u_{a - o_t} over 0 <= a - o_t < n_x, with the
    periodic offsets o_t taken in (-n_x/2, n_x/2]."""
    offs = [int(o) for o in offsets]
    w = [float(x) for x in weights]

    def op(X):
        X = np.atleast_2d(X)
        n = X.shape[-1]
        out = np.zeros_like(X)
        for o, wt in zip(offs, w):
            o = o % n
            if o > n // 2:
                o -= n
            if o >= 0:
                out[:, o:] += wt * X[:, :n - o]
            else:
                out[:, :n + o] += wt * X[:, -o:]
        return out
    return op
