// Host setup of the inflow/outflow step (Sec. 4.5): ERKp+Up on (-1, 1]
// with inflow data g at x = -1, as the affine map u^{n+1} = Phi u^n + f^{n+1}
// that the bounded relaxation kernel applies.
//
// Unknowns sit at x_i = -1 + i dx, i = 1..n_x (array index i - 1).  The Up
// stencil reaches r_l points left and r_r right; points off the grid are
// ghosts:
//  * outflow ghosts x_{n_x+e}: the degree p-1 polynomial through the last p
//    unknowns (p-th order extrapolation);
//  * inflow ghosts x_{-k}, k = 0..r_l-1 (k = 0: the inflow point): Taylor
//    series about x = -1 with d^r u/dx^r = (-1/alpha)^r d^r u/dt^r (inverse
//    Lax-Wendroff), using for stage j the stage-consistent boundary data
//    sum_q gamma_jq dt^q g^(q)(t_n), gamma_jq the coefficients of the stage
//    polynomial P_j(z) = 1 + z sum_k a_jk P_k(z); terms with q + r <= p.
// Phi is the step for g = 0, f^{n+1} = B (g^(0..p)(t_n)) the step of the zero
// state.  Away from the boundaries Phi is the periodic collapsed stencil
// (Corollary 1) truncated to the interval; rows near the ends are stored
// densely.
#include <algorithm>
#include <cmath>

#include "../../include/mgrit.h"
#include "setup.h"

namespace mgr {
namespace {

struct InflowStep {
  const Tableau& t;
  int nx, rl = 0, rr = 0, p;
  double alpha, dx, dt;
  std::vector<int> off;
  std::vector<double> d;
  std::vector<std::vector<double>> gamma;  // [stage][q]
  std::vector<std::vector<double>> ext;    // [e-1][i]: last p points, oldest first

  InflowStep(const Tableau& tab, int n, double a, double h, double k)
      : t(tab), nx(n), p(tab.p), alpha(a), dx(h), dt(k) {
    upwind(p, off, d);
    for (int o : off) {
      rl = std::max(rl, -o);
      rr = std::max(rr, o);
    }
    gamma.assign(t.s, std::vector<double>(t.s, 0.0));
    for (int j = 0; j < t.s; ++j) {
      gamma[j][0] = 1.0;
      for (int k = 0; k < j; ++k)
        for (int q = 0; q + 1 < t.s; ++q) gamma[j][q + 1] += t.A[j][k] * gamma[k][q];
    }
    for (int e = 1; e <= rr; ++e) {
      std::vector<double> w(p, 1.0);
      for (int i = 0; i < p; ++i)
        for (int k = 0; k < p; ++k)
          if (k != i) w[i] *= (double)(e + (p - 1) - k) / (double)(i - k);
      ext.push_back(w);
    }
  }

  // inflow ghosts x_{-k}, k < rl, of stage j from the data gd[0..p]
  void ghosts(int j, const double* gd, double* left) const {
    for (int k = 0; k < rl; ++k) {
      double tot = 0.0;
      if (gd) {
        const double h = k * dx / alpha;
        for (int q = 0; q <= std::min(j, p); ++q) {
          const double dq = gamma[j][q] * std::pow(dt, q);
          double hr = 1.0, fact = 1.0;
          for (int r = 0; q + r <= p; ++r) {
            if (r > 0) {
              hr *= h;
              fact *= r;
            }
            tot += dq * hr / fact * gd[q + r];
          }
        }
      }
      left[k] = tot;
    }
  }

  void apply_L(const double* U, const double* left, double* out) const {
    double right[8] = {0};
    for (int e = 0; e < rr; ++e)
      for (int i = 0; i < p; ++i) right[e] += ext[e][i] * U[nx - p + i];
    const double sc = -alpha / dx;
    for (int a = 0; a < nx; ++a) {
      double acc = 0.0;
      for (size_t j = 0; j < off.size(); ++j) {
        const int q = a + off[j];
        const double v = q < 0 ? left[-q - 1] : (q >= nx ? right[q - nx] : U[q]);
        acc += d[j] * v;
      }
      out[a] = sc * acc;
    }
  }

  void step(const double* u, const double* gd, double* out) const {
    std::vector<std::vector<double>> K(t.s, std::vector<double>(nx));
    std::vector<double> U(nx), left(std::max(rl, 1));
    for (int j = 0; j < t.s; ++j) {
      for (int a = 0; a < nx; ++a) U[a] = u[a];
      for (int k = 0; k < j; ++k)
        if (t.A[j][k] != 0.0)
          for (int a = 0; a < nx; ++a) U[a] += dt * t.A[j][k] * K[k][a];
      ghosts(j, gd, left.data());
      apply_L(U.data(), left.data(), K[j].data());
    }
    for (int a = 0; a < nx; ++a) out[a] = u[a];
    for (int j = 0; j < t.s; ++j)
      if (t.b[j] != 0.0)
        for (int a = 0; a < nx; ++a) out[a] += dt * t.b[j] * K[j][a];
  }
};

}  // namespace

int inflow_setup(const Tableau& t, double cfl, double alpha, int nx, InflowOp& out,
                 std::string& err) {
  if (t.implicit || t.p < 1 || nx < 2 * t.p + 2) {
    err = "inflow/outflow boundaries need an explicit scheme and n_x >= 2p+2";
    return MGRIT_EINVAL;
  }
  const double dx = 2.0 / nx, dt = cfl * dx / alpha;
  // interior: the periodic stencil with signed offsets
  Taps per;
  erk_taps(t, cfl, nx, per);
  out.interior.off.clear();
  out.interior.w.clear();
  for (size_t i = 0; i < per.off.size(); ++i) {
    const int o = per.off[i] > nx / 2 ? per.off[i] - nx : per.off[i];
    out.interior.off.push_back(o);
    out.interior.w.push_back(per.w[i]);
  }
  InflowStep probe_shape(t, nx, alpha, dx, dt);
  const int s = t.s, rl = probe_shape.rl, rr = probe_shape.rr, p = t.p;
  // rows whose paths through the s stages can leave the grid and come back
  // (or meet the extrapolation) differ from the truncated stencil; margins
  // cover them with room to spare
  int nl = s * (rl + rr) + p, nr = s * (rl + rr) + 2 * p;
  int ncl = nl + s * rr, ncr = nr + s * rl + p;
  if (nl + nr >= nx || ncl > nx || ncr > nx) {  // small grids: Phi stored densely
    nl = ncl = nx;
    nr = ncr = 0;
  }
  // probe grid holding both corner blocks apart (same dx, dt)
  const int np = std::min(nx, std::max(2 * (ncl + ncr) + 8, 64));
  InflowStep st(t, np, alpha, dx, dt);
  std::vector<double> e(np, 0.0), col(np);
  out.nl = nl;
  out.ncl = ncl;
  out.lblk.assign((size_t)nl * ncl, 0.0);
  for (int c = 0; c < ncl; ++c) {
    e[c] = 1.0;
    st.step(e.data(), nullptr, col.data());
    e[c] = 0.0;
    for (int i = 0; i < nl; ++i) out.lblk[(size_t)i * ncl + c] = col[i];
  }
  out.nr = nr;
  out.ncr = ncr;
  out.rblk.assign((size_t)nr * ncr, 0.0);
  for (int c = 0; c < ncr; ++c) {
    const int pc = np - ncr + c;
    e[pc] = 1.0;
    st.step(e.data(), nullptr, col.data());
    e[pc] = 0.0;
    for (int i = 0; i < nr; ++i) out.rblk[(size_t)i * ncr + c] = col[np - nr + i];
  }
  // forcing: f = B gd, column d of B the step of zero with unit datum d
  out.nd = p + 1;
  std::vector<double> zero(np, 0.0), gd(out.nd, 0.0);
  std::vector<std::vector<double>> Bc(out.nd);
  int nf = 0;
  for (int dd = 0; dd < out.nd; ++dd) {
    gd[dd] = 1.0;
    st.step(zero.data(), gd.data(), col.data());
    gd[dd] = 0.0;
    Bc[dd] = col;
    for (int i = 0; i < np; ++i)
      if (col[i] != 0.0) nf = std::max(nf, i + 1);
  }
  out.nf = nf;
  out.B.assign((size_t)nf * out.nd, 0.0);
  for (int i = 0; i < nf; ++i)
    for (int dd = 0; dd < out.nd; ++dd) out.B[(size_t)i * out.nd + dd] = Bc[dd][i];
  return MGRIT_OK;
}

double inflow_entry(const InflowOp& op, int nx, int i, int c) {
  if (i < op.nl) return c < op.ncl ? op.lblk[(size_t)i * op.ncl + c] : 0.0;
  if (i >= nx - op.nr) {
    const int cc = c - (nx - op.ncr);
    return cc >= 0 ? op.rblk[(size_t)(i - (nx - op.nr)) * op.ncr + cc] : 0.0;
  }
  double v = 0.0;
  for (size_t t = 0; t < op.interior.off.size(); ++t)
    if (i - op.interior.off[t] == c) v += op.interior.w[t];
  return v;
}

}  // namespace mgr
