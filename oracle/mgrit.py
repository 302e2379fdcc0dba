"""Two-level and multilevel MGRIT / Parareal (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Follows Sec. 2.2 of the paper (and Sec. 4.4 for the multilevel recursion).
On level l the time grid has n_l steps and the system is the block
lower-bidiagonal one of eq. (3) with a right-hand side g:

    x^0 = g^0,    x^{n+1} = Phi_l x^n + g^{n+1},   n = 0..n_l-1,

where Phi_1 = Phi (the fine stepper, g = (u0, 0, ..., 0)) and Phi_{l+1} is
the coarse stepper Psi on level l+1.  C-points are every m-th point.

* F-relaxation: x^{jm+s} = Phi_l x^{jm+s-1} + g^{jm+s}, s = 1..m-1 (from
  each C-point across its F-interval); C-relaxation: the same step into
  the next C-point.  FCF = F, C, F (Sec. 2.2).
* After F-relaxation the residual vanishes at F-points, so the space-time
  residual is the C-point residual r^{(j+1)m} = g + Phi_l x^{(j+1)m-1}
  - x^{(j+1)m}; it is injected as the coarse right-hand side (eq. (6)).
* The coarse error system e^{j+1} = Psi e^j + r^{j+1}, e^0 = 0 (eq. (6)) is
  solved sequentially on the coarsest level or recursively (V- or
  F-cycle); ideal interpolation = correction at C-points then
  F-relaxation.
* Stopping test: discrete L2 norm of the space-time residual,
  sqrt(dx dt sum r^2) <= tol (Sec. 2.2 set-up).

An iterate is held by its C-point values only (F-points are recomputed by
F-relaxation from them).  Arrays are (points, n_x).
"""

import numpy as np


class Result:
    def __init__(self, cpoints, iters, hist, status):
        self.cpoints = cpoints      # (N_c+1, n_x) C-point values returned
        self.iters = iters          # coarse corrections applied
        self.hist = hist            # residual norm before each correction
        self.status = status        # "converged" | "maxit" | "diverged"


def _rhs(g, s, m, nc):
    """g^{jm+s} for j = 0..nc-1 (None: g^n = 0 for n > 0)."""
    if g is None:
        return 0.0
    return g[s:s + nc * m:m]


def fc_relax(op, u, g, m):
    """F- then C-relaxation from C-points u (N_c+1 rows).

    Returns the relaxed C-points v: v^0 = u^0 and
    v^{j+1} = Phi^m u^j + sum_{s=1..m} Phi^{m-s} g^{jm+s}.
    """
    nc = u.shape[0] - 1
    x = u[:-1].copy()
    for s in range(1, m + 1):
        x = op(x) + _rhs(g, s, m, nc)
    v = np.empty_like(u)
    v[0] = u[0]
    v[1:] = x
    return v


def c_residual(op, v, g, m):
    """F-relaxation from C-points v, then the C-point residual.

    r^0 = 0, r^{j+1} = g^{(j+1)m} + Phi x^{(j+1)m-1} - v^{j+1}.
    """
    nc = v.shape[0] - 1
    x = v[:-1].copy()
    for s in range(1, m + 1):
        x = op(x) + _rhs(g, s, m, nc)
    r = np.zeros_like(v)
    r[1:] = x - v[1:]
    return r


def f_interpolate(op, u, g, m):
    """Ideal interpolation: C-points u, F-points by F-relaxation (all points)."""
    nc = u.shape[0] - 1
    n = u.shape[1]
    X = np.empty((nc * m + 1, n))
    X[::m] = u
    x = u[:-1].copy()
    for s in range(1, m):
        x = op(x) + _rhs(g, s, m, nc)
        X[s::m][:nc] = x
    return X


def sequential_solve(op, g):
    """Coarsest level: x^0 = g^0, x^{n+1} = Phi_L x^n + g^{n+1}."""
    X = np.empty_like(g)
    X[0] = g[0]
    for n in range(g.shape[0] - 1):
        X[n + 1] = op(X[n:n + 1])[0] + g[n + 1]
    return X


class MGRIT:
    """MGRIT on a hierarchy of steppers ops[0] (fine Phi), ops[1] (Psi), ...

    ``ops[l]`` maps an array (batch, n_x) to Phi_{l+1} applied row-wise.
    cycle: "V" or "F"; relax: "FCF" (default of the paper) or "F"
    (Parareal-type F-relaxation).
    """

    def __init__(self, ops, m, nt, cycle="V", relax="FCF"):
        self.ops = list(ops)
        self.L = len(self.ops)
        self.m = int(m)
        self.nt = int(nt)
        if self.nt % self.m ** (self.L - 1) != 0:
            raise ValueError("n_t must be divisible by m^(L-1)")
        self.cycle_kind = cycle
        self.relax = relax

    # -- one level ---------------------------------------------------------
    def _pre(self, l, u, g):
        op = self.ops[l]
        v = fc_relax(op, u, g, self.m) if self.relax == "FCF" else u.copy()
        return v, c_residual(op, v, g, self.m)

    def _coarse(self, l, r, kind):
        """Solve level l's error system (rhs r, zero initial guess)."""
        if l == self.L - 1:
            return sequential_solve(self.ops[l], r)
        e = np.zeros_like(r)
        if kind == "F":
            e = self._cycle(l, r, e, "F")
            e = self._cycle(l, r, e, "V")
        else:
            e = self._cycle(l, r, e, "V")
        return e

    def _cycle(self, l, g, x, kind):
        """One V- or F-cycle on level l >= 1 with rhs g and guess x (all pts)."""
        m = self.m
        u = x[::m].copy()
        v, r = self._pre(l, u, g)
        e = self._coarse(l + 1, r, kind)
        return f_interpolate(self.ops[l], v + e, g, m)

    # -- the solver ----------------------------------------------------------
    def solve(self, u0, uinit, tol, maxit, norm_scale, g=None):
        """Iterate from C-points ``uinit`` (row 0 replaced by u0).

        Returns Result with the FCF-relaxed C-points whose residual passed
        the test (or the last ones).  ``norm_scale`` = sqrt(dx dt).  ``g``:
        the fine level's right-hand side rows g^0..g^{n_t} of eq. (3) (row 0
        unused, u0 takes its place); None for g^n = 0, n > 0 (periodic
        problems; inflow data make it nonzero, Sec. 4.5).
        """
        u = np.array(uinit, dtype=float, copy=True)
        u[0] = u0
        hist = []
        for it in range(maxit + 1):
            v, r = self._pre(0, u, g)
            res = norm_scale * float(np.sqrt(np.sum(r * r)))
            hist.append(res)
            if not np.isfinite(res):
                return Result(v, it, hist, "diverged")
            if res <= tol:
                return Result(v, it, hist, "converged")
            if it == maxit:
                return Result(v, it, hist, "maxit")
            e = self._coarse(1, r, self.cycle_kind)
            u = v + e
        raise AssertionError("unreachable")

    def fill(self, cpoints, g=None):
        """All n_t+1 time levels from C-points by F-relaxation (fine level,
        right-hand side ``g`` as in solve)."""
        nc = cpoints.shape[0] - 1
        return f_interpolate(self.ops[0], cpoints, g, self.m) if nc > 0 else cpoints


def norm_scale(disc):
    """sqrt(dx dt): the discrete space-time L2 norm weight (Sec. 2.2)."""
    return float(np.sqrt(disc.dx * disc.dt))


def taps_op(offsets, weights):
    from .coarse import apply_taps
    offs = [int(o) for o in offsets]
    w = [float(x) for x in weights]
    return lambda X: apply_taps(offs, w, X)
