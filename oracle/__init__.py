"""CPU oracle (FP64; Lemma 1's closed form in extended precision) for
MGRIT/Parareal on periodic linear advection.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path and imports nothing from it.

The oracle is written from De Sterck, Falgout, Friedhoff, Krzysik and
MacLachlan, "Optimizing MGRIT and Parareal coarse-grid operators for linear
advection" (Numer. Linear Algebra Appl., 2021; arXiv:1910.03726).  It is
plain, slow and meant to be checked by eye against the paper:

* ``rk``     -- upwind stencils U1-U5 (Sec. 2.1), Butcher tableaux
                (Appendix A, Tables 7 and 8), staged Runge-Kutta stepping
                (eq. (3)), the stability function of Lemma 1 / eq. (4) and
                the closed form Phi^n = F^-1 diag(lambda^n) F of Lemma 1 in
                extended precision (the exact discrete solution over long
                horizons), CFL limits (eq. (5), Table 1).  Stencil and
                tableau entries are written once, as exact fractions or
                formulas, and evaluated in FP64 and in extended precision.
* ``coarse`` -- first column of Phi^m, the weighted least-squares coarse
                operator of eqs. (8)-(9), sparsity-pattern rules (Sec. 4.3,
                Sec. 4.6), operator complexity eq. (10), the two-level
                bound eq. (7).
* ``mgrit``  -- two-level and multilevel MGRIT (F or FCF relaxation,
                V- or F-cycles) as described in Sec. 2.2 and Sec. 4.4,
                with the discrete L2 residual stopping test.
* ``inflow`` -- ERK+U with inflow/outflow boundaries (Sec. 4.5): inflow
                ghosts by inverse Lax-Wendroff, stage boundary data,
                outflow extrapolation, the truncated periodic Psi.

Pins (tests under ``tests/test_oracle_*.py``) tie each function to values
or identities the paper and the mathematics fix.  Functions whose output no
such pin fixes say "parity unpinned" in their docstring.
"""

from . import rk, coarse, mgrit, inflow  # noqa: F401
