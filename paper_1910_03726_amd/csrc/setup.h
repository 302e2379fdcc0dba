// Host-side setup of libmgrit: discretizations, stencils, Fourier symbols,
// the least-squares coarse operators and the SDIRK stage factorization.
// Pure C++ (no HIP); everything here runs once per plan, off the hot path.
#pragma once

#include <complex>
#include <string>
#include <vector>

#include "common.h"

namespace mgr {

using cd = std::complex<double>;

struct Tableau {
  int s = 0;          // stages
  int p = 0;          // order (= index of the upwind formula Up)
  bool implicit = false;
  double A[MAX_STAGES][MAX_STAGES] = {};
  double b[MAX_STAGES] = {};
};

// Appendix A, Tables 7 (ERK1-5) and 8 (SDIRK1-4); scheme ids of mgrit.h.
bool get_tableau(int scheme, Tableau& t);

// Sec. 2.1, formulas U1-U5: v'_i ~ (1/dx) sum_j d[j] v_{i + off[j]}.
void upwind(int p, std::vector<int>& off, std::vector<double>& d);

// Stability function R(z) = 1 + z b^T (I - z A)^{-1} 1 (Lemma 1).
cd stability(const Tableau& t, cd z);

// Eigenvalue of Phi on Fourier mode theta: R(dt * l(theta)) with
// dt l(theta) = -c sum_j d_j exp(i j theta).
cd step_symbol(const Tableau& t, double cfl, double theta);

// max_theta |R| over a fine grid of [0, pi].
double max_amplification(const Tableau& t, double cfl);

struct Taps {
  std::vector<int> off;     // offsets in [0, nx)
  std::vector<double> w;
};

// Phi of an explicit scheme as a stencil: R(Z) with Z = dt L expanded as a
// polynomial of the shift operator (Corollary 1), offsets folded mod nx.
bool erk_taps(const Tableau& t, double cfl, int nx, Taps& out);

// In-place DFT (forward: exp(-2 pi i k n / N); inverse includes 1/N).
void dft(std::vector<cd>& a, bool inverse);

// Eigenvalues of a stencil: mu_k = sum_t w_t exp(-2 pi i k o_t / nx).
void taps_eigs(const Taps& t, int nx, std::vector<cd>& mu);

// Eq. (9): weighted least squares for the pattern `offs`; returns the real
// part of the solution in w and the largest imaginary part.
double lsq_psi(const std::vector<cd>& lam, int m, const std::vector<int>& offs,
               std::vector<double>& w);

// The coarse hierarchy of mgrit_psi_optimize (see mgrit.h).
// Eq. (7) maximised over the modes: the two-level FCF bound of the pair
// (eigenvalues lam of Phi_l, mu of Psi) on a level of nt steps.
double two_level_bound_max(const std::vector<cd>& lam, const std::vector<cd>& mu, int m,
                           long long nt);

// ERK coarse operators whose contiguous windows are as narrow as the two-
// level bound allows: per level the narrowest width from the window rule's
// up to max_width with bound <= target, or the width with the smallest bound.
int psi_hierarchy_bound(int scheme, double cfl, int nx, int nt, int m, int levels,
                        double target, int max_width, std::vector<Taps>& out,
                        std::vector<double>& bounds, double& max_imag);

int psi_hierarchy(int scheme, double cfl, int nx, int m, int levels, int rule,
                  const int* widths, double eta, std::vector<Taps>& out,
                  double& max_imag);

// Minimal cyclic window [omin, omin+W) of [0, nx) holding every offset;
// `dense` receives the W weights (zeros off-pattern).  Offsets are merged
// mod nx first.
void tap_window(const Taps& t, int nx, int& omin, int& W,
                std::vector<double>& dense);

// Sec. 4.5: the step of ERKp+Up on (-1, 1] with inflow data at x = -1 as
// u^{n+1} = Phi u^n + B gd_n, gd_n = g^(d)(t_n), d = 0..p (inflow_setup.cpp).
struct InflowOp {
  Taps interior;                 // Phi away from the ends, signed offsets
  int nl = 0, ncl = 0;           // rows 0..nl-1 over columns 0..ncl-1
  std::vector<double> lblk;      // nl x ncl, row-major
  int nr = 0, ncr = 0;           // rows nx-nr.. over columns nx-ncr..
  std::vector<double> rblk;      // nr x ncr
  int nf = 0, nd = 0;            // forcing rows 0..nf-1: B is nf x nd
  std::vector<double> B;
};
int inflow_setup(const Tableau& t, double cfl, double alpha, int nx, InflowOp& out,
                 std::string& err);
// Phi[i][c] as the bounded kernel applies it
double inflow_entry(const InflowOp& op, int nx, int i, int c);

// SDIRK: factor M = I - gamma dt L into cyclic recurrences (see common.h)
// and fill the stage data; scan constants for chunk K and NL lanes.
// The partial-fraction form (SdirkPfDev): false, with err set, when the
// stage matrix has a repeated or nearly repeated root (the terms would
// cancel: sum |terms| above 64 |M^{-1}| on some wave) or more than
// MAX_PF_TERMS terms; the factored form then applies.
bool sdirk_setup_pf(const Tableau& t, double cfl, int K, int NL, SdirkPfDev& out,
                    std::string& err);

bool sdirk_setup(const Tableau& t, double cfl, int K, int NL, SdirkDev& out,
                 std::string& err);

}  // namespace mgr
