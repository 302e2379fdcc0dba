"""Coarse-grid time steppers Psi (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

A periodic stencil ("taps") is a list of (offset o, weight w) meaning
(Psi u)_i = sum_t w_t u_{(i - o_t) mod n_x}: the circulant matrix whose
first column holds w_t at row o_t (Sec. 4.1).  Its eigenvalues are the DFT
of that first column, mu_k = sum_t w_t exp(-2 pi i k o_t / n_x).

Sec. 4 of the paper chooses Psi ~ Phi^m by the weighted least-squares
problem eq. (8), which for circulant Psi is the linear problem eq. (9)
over the non-zero entries of the first column.
"""

import numpy as np

EPS_WEIGHT = 1e-6  # epsilon of the weighting function w (Sec. 4)
IMAG_FLAG = 1e-8   # imaginary-part acceptance threshold (after Lemma 2)

# eta_tol for the SDIRK thresholding rule, Sec. 4.6: index p -> values for
# m = 2, 4, 8, 16, 32, 64.
ETA_TOL = {
    1: (0.1, 0.125, 0.25, 0.5, 0.5, 0.6),
    2: (0.05, 0.1, 0.1, 0.2, 0.2, 0.2),
    3: (0.005, 0.01, 0.02, 0.02, 0.02, 0.04),
    4: (0.005, 0.01, 0.01, 0.01, 0.02, 0.02),
}
ETA_M = (2, 4, 8, 16, 32, 64)


def eta_tol(p, m):
    return ETA_TOL[p][ETA_M.index(m)]


# ---------------------------------------------------------------------------
# Circulant helpers
# ---------------------------------------------------------------------------
def taps_eigenvalues(offsets, weights, nx):
    """mu_k = sum_t w_t exp(-2 pi i k o_t / n_x), k = 0..n_x-1."""
    k = np.arange(nx, dtype=np.int64)
    mu = np.zeros(nx, dtype=complex)
    for o, w in zip(offsets, weights):
        # reduce k*o mod n in integers so the angle stays in [0, 2 pi)
        mu += w * np.exp(-2j * np.pi * ((k * (int(o) % nx)) % nx) / nx)
    return mu


def apply_taps(offsets, weights, u):
    """(Psi u)_i = sum_t w_t u_{i - o_t} (periodic), on the last axis."""
    out = np.zeros_like(u)
    for o, w in zip(offsets, weights):
        out += w * np.roll(u, int(o), axis=-1)
    return out


def first_column_from_eigs(eigs):
    """First column of the circulant matrix with eigenvalues ``eigs``:
    the inverse DFT (Sec. 4.1: lambda = F phi~)."""
    col = np.fft.ifft(eigs)
    return np.real(col), float(np.max(np.abs(np.imag(col))))


def phi_m_first_column(eigs, m):
    """phi~^m: the first column of Phi^m from the eigenvalues of Phi."""
    return first_column_from_eigs(np.asarray(eigs) ** m)


# ---------------------------------------------------------------------------
# Weighted least squares, eqs. (8)-(9)
# ---------------------------------------------------------------------------
def weights(eigs, eps=EPS_WEIGHT):
    """w_k = w(|lambda_k|) with w(z) = 1/(1 - z + eps)^2 (Sec. 4)."""
    return 1.0 / (1.0 - np.abs(eigs) + eps) ** 2


def lsq_psi(eigs, m, offsets, w=None):
    """Solve eq. (9) for the non-zero first-column entries of Psi.

    Minimizes || W^{1/2} (lambda^m - F R^T psi) ||_2 over psi, where
    (F R^T psi)_k = sum_t psi_t exp(-2 pi i k o_t / n_x).  ``w`` defaults to
    the weights of Sec. 4; pass ones for Remark 1's unit weight.
    Returns (real part of the solution, max |imaginary part|); by Lemma 2
    the exact solution is real.
    """
    eigs = np.asarray(eigs, dtype=complex)
    n = eigs.size
    w = weights(eigs) if w is None else np.asarray(w, dtype=float)
    sw = np.sqrt(w)
    k = np.arange(n, dtype=np.int64)
    offs = np.asarray(offsets, dtype=np.int64) % n
    # exp(-2 pi i k o / n) with k*o reduced mod n in integers
    M = sw[:, None] * np.exp(-2j * np.pi * (np.outer(k, offs) % n) / n)
    rhs = sw * eigs ** m
    sol, *_ = np.linalg.lstsq(M, rhs, rcond=None)
    return np.real(sol), float(np.max(np.abs(np.imag(sol))))


# ---------------------------------------------------------------------------
# Sparsity patterns
# ---------------------------------------------------------------------------
def threshold_pattern(col, eta):
    """Sec. 4.6: offsets o with |phi~^m_o| >= eta * max |phi~^m|."""
    a = np.abs(col)
    return np.nonzero(a >= eta * a.max())[0]


def cyclic_span(offsets, n):
    """Length of the shortest cyclic window of [0, n) holding all offsets."""
    s = np.sort(np.unique(np.asarray(offsets) % n))
    if s.size == 1:
        return 1
    gaps = np.diff(np.concatenate([s, [s[0] + n]]))
    return int(n - gaps.max() + 1)


def best_window(col, width):
    """Contiguous cyclic window [a, a+width) maximizing sum |phi~^m| inside;
    the smallest such a on ties (sums within a relative 1e-12 of the
    maximum count as ties).  Returns the offsets a..a+width-1 (mod n).

    This is the deterministic stand-in for the paper's hand-chosen
    contiguous Phi^m-based patterns of Sec. 4.3 (the chosen patterns are
    shown only in a figure).  Parity unpinned against the paper's weights.
    """
    a = np.abs(col)
    n = a.size
    width = min(int(width), n)
    ext = np.concatenate([a, a[:width]])
    csum = np.concatenate([[0.0], np.cumsum(ext)])
    sums = csum[width:width + n] - csum[:n]
    start = int(np.nonzero(sums >= sums.max() * (1.0 - 1e-12))[0][0])
    return (start + np.arange(width)) % n


def window_rule_width(col, nnz_prev, eta=0.02):
    """Width of the ERK window: max(nnz(Phi_l), span of |phi~^m| >= eta max)."""
    n = col.size
    return max(int(nnz_prev), cyclic_span(threshold_pattern(col, eta), n))


def signed_offsets(offsets, n):
    """Map offsets in [0, n) to (-n/2, n/2] (display only)."""
    o = np.asarray(offsets) % n
    return np.where(o > n // 2, o - n, o)


# ---------------------------------------------------------------------------
# Coarse operators for a level hierarchy (Sec. 4.4)
# ---------------------------------------------------------------------------
def fine_nnz(disc):
    """nnz of the (ERK) fine operator: taps of R(dt L) as a polynomial.

    SDIRK steppers are dense (Corollary 1); the window rule then uses only
    the threshold span, so 0 is returned for them."""
    if disc.scheme.startswith("SDIRK"):
        return 0
    col, _ = first_column_from_eigs(disc.eigenvalues())
    return int(np.count_nonzero(np.abs(col) > 1e-13 * np.abs(col).max()))


def build_hierarchy(disc, m, levels, rule="auto", widths=None, eta=None):
    """Psi_2..Psi_L for an L-level hierarchy: Phi_{l+1} ~ Phi_l^m (Sec. 4.4).

    rule "window": ERK contiguous window of given ``widths`` (one per coarse
    level) or of the width rule; rule "eta": SDIRK thresholding of Sec. 4.6
    with the printed eta_tol (or ``eta``).  "auto" picks "eta" for SDIRK and
    "window" for ERK.  Returns a list of dicts with offsets, weights,
    max_imag and the eigenvalues of each coarse operator.
    """
    n = disc.nx
    if rule == "auto":
        rule = "eta" if disc.scheme.startswith("SDIRK") else "window"
    lam = disc.eigenvalues()
    nnz_prev = fine_nnz(disc) if rule == "window" else None
    out = []
    for lev in range(1, levels):
        col, _ = phi_m_first_column(lam, m)
        if rule == "eta":
            e = eta if eta is not None else eta_tol(disc.p, m)
            offs = threshold_pattern(col, e)
        elif rule == "window":
            if widths is not None:
                wdt = widths[lev - 1]
            else:
                wdt = window_rule_width(col, nnz_prev)
            offs = best_window(col, wdt)
        else:
            raise ValueError(rule)
        psi, im = lsq_psi(lam, m, offs)
        mu = taps_eigenvalues(offs, psi, n)
        out.append({"offsets": np.asarray(offs), "weights": psi,
                    "max_imag": im, "eigs": mu})
        lam = mu
        nnz_prev = len(offs)
    return out


def operator_complexity(nnz_levels, m):
    """Eq. (10): (1/nnz(Phi_1)) sum_l m^{1-l} nnz(Phi_l)."""
    return sum(m ** (-l) * z for l, z in enumerate(nnz_levels)) / nnz_levels[0]


def two_level_bound(lam, mu, m, nt):
    """Eq. (7): sqrt(m) |lam|^m |lam^m - mu| / (1 - |mu|) (1 - |mu|^(nt/m-1))."""
    lam = np.asarray(lam)
    mu = np.asarray(mu)
    am = np.abs(mu)
    return (np.sqrt(m) * np.abs(lam) ** m * np.abs(lam ** m - mu) / (1.0 - am)
            * (1.0 - am ** (nt / m - 1)))


# ---------------------------------------------------------------------------
# Bound-driven window widths (eq. (7) per level)
# ---------------------------------------------------------------------------
def geometric_sum(a, N):
    """sum_{j<N} a^j elementwise: the factor (1 - a^N)/(1 - a) of eq. (7),
    written so that a = 1 (where it equals N) needs no 0/0: within 1e-12 of
    1 the first-order expansion N + N(N-1)/2 (a - 1)."""
    a = np.asarray(a, dtype=float)
    out = N + 0.5 * N * (N - 1.0) * (a - 1.0)
    far = np.abs(1.0 - a) >= 1e-12
    with np.errstate(divide="ignore"):
        out[far] = np.expm1(N * np.log(a[far])) / (a[far] - 1.0)
    return out


def max_two_level_bound(lam, mu, m, nt):
    """max over the modes of eq. (7) for a level of nt steps; inf if any
    mode's value is not finite."""
    lam = np.asarray(lam)
    mu = np.asarray(mu)
    v = (np.sqrt(m) * np.abs(lam) ** m * np.abs(lam ** m - mu)
         * geometric_sum(np.abs(mu), nt // m - 1))
    return float(np.max(v)) if np.all(np.isfinite(v)) else float("inf")


def build_hierarchy_bound(disc, m, levels, nt, target=1e-3, max_width=64):
    """ERK coarse operators Psi_2..Psi_L with bound-driven windows.

    Level by level (Psi_{l+1} against Phi_l^m, Sec. 4.4) the contiguous
    window of phi~^m is placed as by the window rule (best_window), and its
    width is the narrowest from the window rule's width up to max_width for
    which max_two_level_bound(lambda_l, mu, m, n_l) <= max(target, 1e-10)
    (n_l the steps of level l, n_1 = nt; bounds below 1e-10 are at the
    rounding level of the fit and meet any target); if none does, the
    narrowest width whose bound is within 0.1 % of the smallest.  Returns
    dicts as build_hierarchy, with the level's "bound".
    """
    n = disc.nx
    lam = disc.eigenvalues()
    nnz_prev = fine_nnz(disc)
    nl = nt
    out = []
    for _ in range(1, levels):
        col, _ = phi_m_first_column(lam, m)
        w0 = window_rule_width(col, nnz_prev)
        cands = []
        pick = None
        for width in range(w0, max(w0, min(max_width, n)) + 1):
            offs = best_window(col, width)
            psi, im = lsq_psi(lam, m, offs)
            mu = taps_eigenvalues(offs, psi, n)
            b = max_two_level_bound(lam, mu, m, nl)
            cand = {"offsets": np.asarray(offs), "weights": psi, "max_imag": im,
                    "eigs": mu, "bound": b}
            cands.append(cand)
            if b <= max(target, 1e-10):
                pick = cand
                break
        if pick is None:
            bmin = min(c["bound"] for c in cands)
            pick = next(c for c in cands if c["bound"] <= (1.0 + 1e-3) * bmin)
        out.append(pick)
        lam = pick["eigs"]
        nnz_prev = len(pick["offsets"])
        nl //= m
    return out

