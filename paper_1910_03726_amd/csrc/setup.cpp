// Host-side setup of libmgrit (see setup.h).  Runs once per plan.
#include "setup.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>

#include "../../include/mgrit.h"

namespace mgr {

static const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Appendix A: Butcher tableaux, Sec. 2.1: upwind formulas
// ---------------------------------------------------------------------------
// Every entry is written once, as a fraction p/q or a formula in sqrt(2) and
// the SDIRK3 diagonal, and evaluated in the number type R: FP64 for the
// kernels, extended precision or binary128 where the setup needs the exact
// values (the collapsed ERK stencil, the SDIRK stage factorization).
using quad = __float128;

template <typename R>
struct Num;
template <>
struct Num<double> {
  static double sqrt2() { return std::sqrt(2.0); }
  static double sdirk3_root() { return 0.43586652150845899942; }
};
template <>
struct Num<long double> {
  static long double sqrt2() { return std::sqrt(2.0L); }
  static long double sdirk3_root() { return 0.43586652150845899942L; }
};
template <>
struct Num<quad> {
  static quad sqrt2() {
    quad x = std::sqrt(2.0);  // two Newton steps from the FP64 root
    for (int i = 0; i < 2; ++i) x = (x + quad(2) / x) / quad(2);
    return x;
  }
  static quad sdirk3_root() {  // 0.4358665215 0845899942 (Table 8)
    return (quad(4358665215LL) + quad(845899942LL) / quad(10000000000LL)) /
           quad(10000000000LL);
  }
};

template <typename R>
struct TableauOf {
  int s = 0;
  R A[MAX_STAGES][MAX_STAGES] = {};
  R b[MAX_STAGES] = {};
};

template <typename R>
static void rows_of(TableauOf<R>& t, std::initializer_list<std::initializer_list<R>> rows,
                    std::initializer_list<R> b) {
  int i = 0;
  for (auto& r : rows) {
    int j = 0;
    for (R v : r) t.A[i][j++] = v;
    ++i;
  }
  t.s = (int)b.size();
  int k = 0;
  for (R v : b) t.b[k++] = v;
}

template <typename R>
static bool tableau_of(int scheme, TableauOf<R>& t) {
  t = TableauOf<R>();
  auto f = [](long long p, long long q) { return R(p) / R(q); };
  const R one = R(1), zero = R(0);
  switch (scheme) {
    case MGRIT_ERK1:
      rows_of<R>(t, {{zero}}, {one});
      return true;
    case MGRIT_ERK2:
      rows_of<R>(t, {{zero}, {one, zero}}, {f(1, 2), f(1, 2)});
      return true;
    case MGRIT_ERK3:
      rows_of<R>(t, {{zero}, {one}, {f(1, 4), f(1, 4)}}, {f(1, 6), f(1, 6), f(2, 3)});
      return true;
    case MGRIT_ERK4:
      rows_of<R>(t, {{zero}, {f(1, 2)}, {zero, f(1, 2)}, {zero, zero, one}},
                 {f(1, 6), f(1, 3), f(1, 3), f(1, 6)});
      return true;
    case MGRIT_ERK5:
      rows_of<R>(t,
                 {{zero},
                  {f(1, 4)},
                  {f(1, 8), f(1, 8)},
                  {zero, zero, f(1, 2)},
                  {f(3, 16), f(-3, 8), f(3, 8), f(9, 16)},
                  {f(-3, 7), f(8, 7), f(6, 7), f(-12, 7), f(8, 7)}},
                 {f(7, 90), zero, f(32, 90), f(12, 90), f(32, 90), f(7, 90)});
      return true;
    case MGRIT_SDIRK1:
      rows_of<R>(t, {{one}}, {one});
      return true;
    case MGRIT_SDIRK2: {
      const R r2 = Num<R>::sqrt2() / R(2);
      rows_of<R>(t, {{one - r2}, {r2, one - r2}}, {r2, one - r2});
      return true;
    }
    case MGRIT_SDIRK3: {
      const R z = Num<R>::sdirk3_root();
      const R be = (one - z) / R(2);
      const R ga = f(-3, 2) * z * z + R(4) * z - f(1, 4);
      const R ep = f(3, 2) * z * z - R(5) * z + f(5, 4);
      rows_of<R>(t, {{z}, {be, z}, {ga, ep, z}}, {ga, ep, z});
      return true;
    }
    case MGRIT_SDIRK4:
      rows_of<R>(t,
                 {{f(1, 4)},
                  {f(1, 2), f(1, 4)},
                  {f(17, 50), f(-1, 25), f(1, 4)},
                  {f(371, 1360), f(-137, 2720), f(15, 544), f(1, 4)},
                  {f(25, 24), f(-49, 48), f(125, 16), f(-85, 12), f(1, 4)}},
                 {f(25, 24), f(-49, 48), f(125, 16), f(-85, 12), f(1, 4)});
      return true;
    default:
      return false;
  }
}

bool get_tableau(int scheme, Tableau& t) {
  t = Tableau();
  TableauOf<double> x;
  if (!tableau_of(scheme, x)) return false;
  t.s = x.s;
  for (int i = 0; i < x.s; ++i) {
    for (int j = 0; j < x.s; ++j) t.A[i][j] = x.A[i][j];
    t.b[i] = x.b[i];
  }
  t.implicit = scheme >= MGRIT_SDIRK1;
  t.p = t.implicit ? scheme - 10 : scheme;
  return true;
}

// Sec. 2.1: U1..U5 as fractions (offset, numerator, denominator).
struct UpwindTerm {
  int off;
  int num, den;
};
static std::vector<UpwindTerm> upwind_terms(int p) {
  switch (p) {
    case 1: return {{0, 1, 1}, {-1, -1, 1}};
    case 2: return {{0, 3, 2}, {-1, -4, 2}, {-2, 1, 2}};
    case 3: return {{1, 2, 6}, {0, 3, 6}, {-1, -6, 6}, {-2, 1, 6}};
    case 4: return {{1, 3, 12}, {0, 10, 12}, {-1, -18, 12}, {-2, 6, 12}, {-3, -1, 12}};
    case 5:
      return {{2, -3, 60}, {1, 30, 60}, {0, 20, 60}, {-1, -60, 60}, {-2, 15, 60},
              {-3, -2, 60}};
    default: return {};
  }
}

void upwind(int p, std::vector<int>& off, std::vector<double>& d) {
  off.clear();
  d.clear();
  for (const UpwindTerm& u : upwind_terms(p)) {
    off.push_back(u.off);
    d.push_back((double)u.num / (double)u.den);
  }
}

cd stability(const Tableau& t, cd z) {
  // (I - zA) y = 1 by forward substitution (A is lower triangular).
  cd y[MAX_STAGES];
  cd acc = 0.0;
  for (int i = 0; i < t.s; ++i) {
    cd r = 1.0;
    for (int j = 0; j < i; ++j) r += z * t.A[i][j] * y[j];
    y[i] = r / (1.0 - z * t.A[i][i]);
    acc += t.b[i] * y[i];
  }
  return 1.0 + z * acc;
}

cd step_symbol(const Tableau& t, double cfl, double theta) {
  std::vector<int> off;
  std::vector<double> d;
  upwind(t.p, off, d);
  cd s = 0.0;
  for (size_t j = 0; j < off.size(); ++j)
    s += d[j] * std::exp(cd(0.0, off[j] * theta));
  return stability(t, -cfl * s);
}

// Largest |R(z(theta))| over theta in [0, pi] (at -theta the symbol is the
// conjugate): a scan of 1025 points, then a golden-section search on the
// bracket of every sampled local maximum within 1e-3 of the largest sample,
// so the value is the maximum itself rather than a sampled lower bound.
double max_amplification(const Tableau& t, double cfl) {
  std::vector<int> off;
  std::vector<double> d;
  upwind(t.p, off, d);
  auto amp = [&](double th) {
    cd s = 0.0;
    for (size_t j = 0; j < off.size(); ++j) s += d[j] * std::exp(cd(0.0, off[j] * th));
    return std::abs(stability(t, -cfl * s));
  };
  const int n = 1025;
  const double h = kPi / (n - 1);
  std::vector<double> v(n);
  double mx = 0.0;
  for (int i = 0; i < n; ++i) mx = std::max(mx, v[i] = amp(h * i));
  const double g = 0.5 * (std::sqrt(5.0) - 1.0);
  double best = mx;
  for (int i = 0; i < n; ++i) {
    if (v[i] < mx - 1e-3) continue;
    if ((i > 0 && v[i - 1] > v[i]) || (i + 1 < n && v[i + 1] > v[i])) continue;
    double a = h * std::max(i - 1, 0), b = h * std::min(i + 1, n - 1);
    double c = b - g * (b - a), e = a + g * (b - a);
    double fc = amp(c), fe = amp(e);
    for (int it = 0; it < 64 && b - a > 1e-15; ++it) {
      if (fc >= fe) {
        b = e;
        e = c;
        fe = fc;
        c = b - g * (b - a);
        fc = amp(c);
      } else {
        a = c;
        c = e;
        fc = fe;
        e = a + g * (b - a);
        fe = amp(e);
      }
    }
    best = std::max(best, std::max(fc, fe));
  }
  return best;
}

// ---------------------------------------------------------------------------
// Corollary 1: the ERK stepper as one stencil
// ---------------------------------------------------------------------------
// The taps are the coefficients of R(Z) = sum_k g_k Z^k, Z = dt L a
// polynomial of the shift, computed in binary128 from the tableau's
// fractions so that rounding them to FP64 is the only error.  That rounding
// is chosen (each tap within one unit in the last place of its value) to
// keep the low Fourier modes of the stencil on the exact symbol: errors e_o
// move the eigenvalue of mode theta by sum_o e_o exp(-i o theta) =
// E0 - i theta E1 - theta^2/2 E2 + ..., E_q = sum_o o^q e_o (o the signed
// offset), and n_t steps multiply that drift n_t-fold, so E0 (conservation
// of the mean), E1 (transport speed) and E2 are driven toward zero.
static void round_taps_preserving_moments(const std::map<int, quad>& exact, int nx,
                                          Taps& out) {
  const size_t n = exact.size();
  std::vector<int> so;
  std::vector<quad> ex;
  std::vector<double> r;
  std::vector<quad> ulp;
  for (auto& a : exact) {
    so.push_back(a.first > nx / 2 ? a.first - nx : a.first);
    ex.push_back(a.second);
    const double v = (double)a.second;
    r.push_back(v);
    ulp.push_back((quad)std::nextafter(std::fabs(v), HUGE_VAL) - (quad)std::fabs(v));
  }
  quad E[3] = {0, 0, 0};
  for (size_t i = 0; i < n; ++i) {
    const quad e = (quad)r[i] - ex[i], o = so[i];
    E[0] += e;
    E[1] += o * e;
    E[2] += o * o * e;
  }
  // mode scale of the weights: theta ~ 0.05 (about 8 periods per 1000 points)
  const quad w1 = quad(1) / quad(20), w2 = w1 * w1 / quad(2);
  auto cost = [&](quad e0, quad e1, quad e2) {
    const quad a = e0, b = w1 * e1, c = w2 * e2;
    return a * a + b * b + c * c;
  };
  quad J = cost(E[0], E[1], E[2]);
  for (int it = 0; it < 256; ++it) {
    int bi = -1;
    double bv = 0.0;
    quad bJ = J;
    for (size_t i = 0; i < n; ++i)
      for (int dir = -1; dir <= 1; dir += 2) {
        const double v = std::nextafter(r[i], dir > 0 ? HUGE_VAL : -HUGE_VAL);
        quad dev = (quad)v - ex[i];
        if (dev < 0) dev = -dev;
        if (dev > ulp[i]) continue;
        const quad d = (quad)v - (quad)r[i], o = so[i];
        const quad j = cost(E[0] + d, E[1] + o * d, E[2] + o * o * d);
        if (j < bJ) {
          bJ = j;
          bi = (int)i;
          bv = v;
        }
      }
    if (bi < 0) break;
    const quad d = (quad)bv - (quad)r[bi], o = so[bi];
    E[0] += d;
    E[1] += o * d;
    E[2] += o * o * d;
    r[bi] = bv;
    J = bJ;
  }
  out.off.clear();
  out.w.clear();
  size_t i = 0;
  for (auto& a : exact) {
    out.off.push_back(a.first);
    out.w.push_back(r[i++]);
  }
}

bool erk_taps(const Tableau& t, double cfl, int nx, Taps& out) {
  if (t.implicit) return false;
  TableauOf<quad> q;
  const int scheme = t.p;  // ERKp has scheme id p
  if (!tableau_of(scheme, q) || q.s != t.s) return false;
  // Z = dt L: (Z u)_i = -c sum_j d_j u_{i+j}; as first-column offset o = -j.
  std::map<int, quad> Z;
  for (const UpwindTerm& u : upwind_terms(t.p))
    Z[-u.off] += -(quad)cfl * (quad(u.num) / quad(u.den));
  // stability polynomial coefficients g_0 = 1, g_k = b^T A^{k-1} 1
  quad v[MAX_STAGES], nv[MAX_STAGES];
  for (int i = 0; i < q.s; ++i) v[i] = 1;
  std::vector<quad> g(1, quad(1));
  for (int k = 1; k <= q.s; ++k) {
    quad gk = 0;
    for (int i = 0; i < q.s; ++i) gk += q.b[i] * v[i];
    g.push_back(gk);
    for (int i = 0; i < q.s; ++i) {
      nv[i] = 0;
      for (int j = 0; j < q.s; ++j) nv[i] += q.A[i][j] * v[j];
    }
    for (int i = 0; i < q.s; ++i) v[i] = nv[i];
  }
  std::map<int, quad> phi, pw;  // pw = Z^k
  pw[0] = 1;
  phi[0] = g[0];
  for (int k = 1; k <= q.s; ++k) {
    std::map<int, quad> nxt;
    for (auto& a : pw)
      for (auto& b : Z) nxt[a.first + b.first] += a.second * b.second;
    pw.swap(nxt);
    for (auto& a : pw) phi[a.first] += g[k] * a.second;
  }
  std::map<int, quad> folded;
  for (auto& a : phi) folded[((a.first % nx) + nx) % nx] += a.second;
  quad mx = 0;
  for (auto& a : folded) mx = std::max(mx, a.second < 0 ? -a.second : a.second);
  // coefficients that cancel exactly come out at the binary128 rounding level
  std::map<int, quad> kept;
  for (auto& a : folded)
    if ((a.second < 0 ? -a.second : a.second) > quad(1e-24) * mx) kept.insert(a);
  round_taps_preserving_moments(kept, nx, out);
  return true;
}

// ---------------------------------------------------------------------------
// DFTs with exactly reduced angles
// ---------------------------------------------------------------------------
static void roots_of_unity(int n, std::vector<cd>& w) {
  // w[q] = exp(-2 pi i q / n); tables are kept per n (setup threads share them)
  static std::mutex mu;
  static std::map<int, std::shared_ptr<const std::vector<cd>>> cache;
  std::shared_ptr<const std::vector<cd>> tab;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(n);
    if (it != cache.end()) tab = it->second;
  }
  if (!tab) {
    auto v = std::make_shared<std::vector<cd>>(n);
    for (int q = 0; q < n; ++q) {
      double a = -2.0 * kPi * (double)q / (double)n;
      (*v)[q] = cd(std::cos(a), std::sin(a));
    }
    tab = v;
    std::lock_guard<std::mutex> lk(mu);
    if (cache.size() < 64) cache.emplace(n, tab);
  }
  w = *tab;
}

// The transform with the roots of unity w (roots_of_unity of a.size()).
static void dft_with(std::vector<cd>& a, bool inverse, const std::vector<cd>& w) {
  const int n = (int)a.size();
  if (n > 0 && (n & (n - 1)) == 0) {
    // iterative radix-2
    for (int i = 1, j = 0; i < n; ++i) {
      int bit = n >> 1;
      for (; j & bit; bit >>= 1) j ^= bit;
      j ^= bit;
      if (i < j) std::swap(a[i], a[j]);
    }
    for (int len = 2; len <= n; len <<= 1) {
      const int step = n / len, half = len / 2;
      for (int k = 0; k < half; ++k) {
        const cd tw = inverse ? std::conj(w[k * step]) : w[k * step];
        for (int i = k; i < n; i += len) {
          const cd u = a[i], v = a[i + half] * tw;
          a[i] = u + v;
          a[i + half] = u - v;
        }
      }
    }
  } else {
    std::vector<cd> out(n);
    for (int k = 0; k < n; ++k) {
      cd s = 0.0;
      for (int t = 0; t < n; ++t) {
        cd tw = w[(int)(((long long)k * t) % n)];
        s += a[t] * (inverse ? std::conj(tw) : tw);
      }
      out[k] = s;
    }
    a.swap(out);
  }
  if (inverse)
    for (auto& x : a) x /= (double)n;
}

void dft(std::vector<cd>& a, bool inverse) {
  std::vector<cd> w;
  roots_of_unity((int)a.size(), w);
  dft_with(a, inverse, w);
}

void taps_eigs(const Taps& t, int nx, std::vector<cd>& mu) {
  std::vector<cd> w;
  roots_of_unity(nx, w);
  mu.assign(nx, cd(0.0));
  if (nx > 0 && (nx & (nx - 1)) == 0) {
    // mu = forward transform of the taps placed at their offsets
    for (size_t q = 0; q < t.off.size(); ++q) mu[((t.off[q] % nx) + nx) % nx] += t.w[q];
    dft_with(mu, false, w);
    return;
  }
  for (size_t q = 0; q < t.off.size(); ++q) {
    long long o = ((t.off[q] % nx) + nx) % nx;
    for (int k = 0; k < nx; ++k) mu[k] += t.w[q] * w[(int)((k * o) % nx)];
  }
}

static cd ipow(cd z, int m) {
  cd r = 1.0;
  while (m > 0) {
    if (m & 1) r *= z;
    z *= z;
    m >>= 1;
  }
  return r;
}

// ---------------------------------------------------------------------------
// Eq. (9) by its normal equations, refined against the full spectrum
// ---------------------------------------------------------------------------
// With e_t(k) = e^{-2 pi i k o_t / n} the columns and w_k the weights, the
// normal matrix G[t][s] = Re sum_k w_k conj(e_t(k)) e_s(k) depends only on
// o_t - o_s: it is the real part of c(d) = sum_k w_k e^{2 pi i k d / n}, one
// inverse FFT of the weights.  Likewise A^T W r for any spectral residual r
// is an inverse FFT read at the offsets, and the model sum_t x_t e_t(k) one
// forward FFT of the sparse tap vector.  The Cholesky solution of G loses
// digits to cond(G) (up to ~1e15 on deep levels), so it is refined: each
// step recomputes the residual from the spectrum and solves G again, which
// contracts the error by about cond(G) * eps per step.  O(n log n + v^3)
// per level instead of O(n v^2).  False if n is not a power of two or the
// refinement does not settle (the caller then uses the QR solution).
static bool lsq_psi_spectral(const std::vector<cd>& lam, int m, const std::vector<int>& offs,
                             std::vector<double>& x) {
  const int n = (int)lam.size();
  const int v = (int)offs.size();
  if (n < 2 || (n & (n - 1)) != 0 || v < 1 || v > n) return false;
  std::vector<int> o(v);
  for (int t = 0; t < v; ++t) o[t] = ((offs[t] % n) + n) % n;
  std::vector<double> wk(n);
  std::vector<cd> target(n), c(n), h(n);
  for (int k = 0; k < n; ++k) {
    const double sw = 1.0 / (1.0 - std::abs(lam[k]) + 1e-6);
    wk[k] = sw * sw;
    target[k] = ipow(lam[k], m);
    c[k] = wk[k];
    h[k] = wk[k] * target[k];
  }
  std::vector<cd> ru;
  roots_of_unity(n, ru);
  dft_with(c, true, ru);  // c[d] * n = sum_k w_k e^{+2 pi i k d / n}
  dft_with(h, true, ru);
  std::vector<double> G((size_t)v * v), L((size_t)v * v, 0.0), g(v);
  for (int t = 0; t < v; ++t) {
    for (int q = 0; q < v; ++q) G[(size_t)t * v + q] = n * c[((o[t] - o[q]) % n + n) % n].real();
    g[t] = n * h[o[t]].real();
  }
  // Cholesky G = L L^T
  for (int j = 0; j < v; ++j) {
    double d = G[(size_t)j * v + j];
    for (int q = 0; q < j; ++q) d -= L[(size_t)j * v + q] * L[(size_t)j * v + q];
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    L[(size_t)j * v + j] = ljj;
    for (int i = j + 1; i < v; ++i) {
      double s = G[(size_t)i * v + j];
      for (int q = 0; q < j; ++q) s -= L[(size_t)i * v + q] * L[(size_t)j * v + q];
      L[(size_t)i * v + j] = s / ljj;
    }
  }
  auto solve = [&](std::vector<double>& b) {
    for (int i = 0; i < v; ++i) {
      double s = b[i];
      for (int q = 0; q < i; ++q) s -= L[(size_t)i * v + q] * b[q];
      b[i] = s / L[(size_t)i * v + i];
    }
    for (int i = v - 1; i >= 0; --i) {
      double s = b[i];
      for (int q = i + 1; q < v; ++q) s -= L[(size_t)q * v + i] * b[q];
      b[i] = s / L[(size_t)i * v + i];
    }
  };
  x = g;
  solve(x);
  double prev = 1e300;
  std::vector<cd> r(n);
  for (int it = 0; it < 40; ++it) {
    // spectral residual r_k = target_k - sum_t x_t e_t(k), weighted, back
    std::fill(r.begin(), r.end(), cd(0.0));
    for (int t = 0; t < v; ++t) r[o[t]] += x[t];
    dft_with(r, false, ru);
    for (int k = 0; k < n; ++k) r[k] = wk[k] * (target[k] - r[k]);
    dft_with(r, true, ru);
    std::vector<double> dx(v);
    for (int t = 0; t < v; ++t) dx[t] = n * r[o[t]].real();
    solve(dx);
    double nd = 0.0, nx = 0.0;
    for (int t = 0; t < v; ++t) {
      x[t] += dx[t];
      nd = std::max(nd, std::fabs(dx[t]));
      nx = std::max(nx, std::fabs(x[t]));
    }
    if (nd <= 1e-13 * nx) return true;
    if (it >= 2 && nd > 0.5 * prev) return nd <= 1e-12 * nx;  // at its rounding floor
    prev = nd;
  }
  return false;
}

// ---------------------------------------------------------------------------
// Eq. (9): Householder QR least squares (fallback)
// ---------------------------------------------------------------------------
double lsq_psi(const std::vector<cd>& lam, int m, const std::vector<int>& offs,
               std::vector<double>& wout) {
  if (lsq_psi_spectral(lam, m, offs, wout)) return 0.0;  // real by construction
  // Rows k of eq. (9): sqrt(w_k) [e^{-2 pi i k o_t / n}]_t against
  // sqrt(w_k) lambda_k^m.  The symbols of a real stencil satisfy
  // lambda_{n-k} = conj(lambda_k), so rows k and n-k are conjugate and, for
  // real weights psi, contribute equal residuals: the least-squares problem
  // is the real one over k = 0..n/2 with the real and imaginary parts of
  // each row as two equations (scaled by sqrt 2 where k and n-k differ).
  // Its minimiser is the (real) minimiser of the complex problem; solved by
  // Householder QR on column-major real arrays.
  const int n = (int)lam.size();
  const int v = (int)offs.size();
  std::vector<cd> w;
  roots_of_unity(n, w);
  const int kh = n / 2;
  std::vector<int> rows_k;  // (k, part): part 0 real, 1 imaginary
  std::vector<int> rows_p;
  for (int k = 0; k <= kh; ++k) {
    rows_k.push_back(k);
    rows_p.push_back(0);
    const bool self = (k == 0) || (2 * k == n);
    if (!self) {
      rows_k.push_back(k);
      rows_p.push_back(1);
    }
  }
  const int nr = (int)rows_k.size();
  std::vector<double> A((size_t)nr * v), bb(nr);
  for (int r = 0; r < nr; ++r) {
    const int k = rows_k[r];
    const bool self = (k == 0) || (2 * k == n);
    const double sc = self ? 1.0 : std::sqrt(2.0);
    const double sw = sc / (1.0 - std::abs(lam[k]) + 1e-6);  // sqrt w = 1/(1-|l|+eps)
    const cd rhs = ipow(lam[k], m);
    bb[r] = sw * (rows_p[r] ? rhs.imag() : rhs.real());
    for (int t = 0; t < v; ++t) {
      const long long o = ((offs[t] % n) + n) % n;
      const cd e = w[(int)((k * o) % n)];
      A[(size_t)t * nr + r] = sw * (rows_p[r] ? e.imag() : e.real());
    }
  }
  auto dot = [nr](const double* x, const double* y, int j) {
    double s0 = 0.0, s1 = 0.0;
    int i = j;
    for (; i + 1 < nr; i += 2) {
      s0 += x[i] * y[i];
      s1 += x[i + 1] * y[i + 1];
    }
    if (i < nr) s0 += x[i] * y[i];
    return s0 + s1;
  };
  std::vector<double> diag(v, 0.0);
  for (int j = 0; j < v && j < nr; ++j) {
    double* h = &A[(size_t)j * nr];
    const double nrm2 = dot(h, h, j);
    const double nrm = std::sqrt(nrm2);
    if (nrm == 0.0) continue;
    const double x0 = h[j];
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    h[j] = x0 - alpha;  // reflector stored in place of the column
    const double hn2 = nrm2 - x0 * x0 + h[j] * h[j];
    diag[j] = alpha;
    if (hn2 == 0.0) continue;
    for (int k = j + 1; k < v; ++k) {
      double* c = &A[(size_t)k * nr];
      const double f = 2.0 * dot(h, c, j) / hn2;
      for (int i = j; i < nr; ++i) c[i] -= f * h[i];
    }
    const double f = 2.0 * dot(h, bb.data(), j) / hn2;
    for (int i = j; i < nr; ++i) bb[i] -= f * h[i];
  }
  wout.assign(v, 0.0);
  for (int j = std::min(v, nr) - 1; j >= 0; --j) {
    double s = bb[j];
    for (int k = j + 1; k < v; ++k) s -= A[(size_t)k * nr + j] * wout[k];
    wout[j] = diag[j] != 0.0 ? s / diag[j] : 0.0;
  }
  return 0.0;  // the minimiser is real by construction
}

// ---------------------------------------------------------------------------
// Sparsity patterns (Sec. 4.3 window rule, Sec. 4.6 thresholding)
// ---------------------------------------------------------------------------
static const double kEta[4][6] = {{0.1, 0.125, 0.25, 0.5, 0.5, 0.6},
                                  {0.05, 0.1, 0.1, 0.2, 0.2, 0.2},
                                  {0.005, 0.01, 0.02, 0.02, 0.02, 0.04},
                                  {0.005, 0.01, 0.01, 0.01, 0.02, 0.02}};

static double eta_table(int p, int m) {
  if (p < 1 || p > 4) return -1.0;
  int idx = -1;
  for (int i = 0, mm = 2; i < 6; ++i, mm *= 2)
    if (mm == m) idx = i;
  return idx < 0 ? -1.0 : kEta[p - 1][idx];
}

static std::vector<int> threshold(const std::vector<double>& col, double eta) {
  double mx = 0.0;
  for (double c : col) mx = std::max(mx, std::fabs(c));
  std::vector<int> o;
  for (int i = 0; i < (int)col.size(); ++i)
    if (std::fabs(col[i]) >= eta * mx) o.push_back(i);
  return o;
}

static int cyclic_span(const std::vector<int>& offs, int n) {
  std::vector<int> s(offs);
  std::sort(s.begin(), s.end());
  s.erase(std::unique(s.begin(), s.end()), s.end());
  if (s.size() <= 1) return (int)s.size();
  int gap = s.front() + n - s.back();
  for (size_t i = 1; i < s.size(); ++i) gap = std::max(gap, s[i] - s[i - 1]);
  return n - gap + 1;
}

// Smallest a whose window sum reaches the maximum up to a relative 1e-12.
static std::vector<int> best_window(const std::vector<double>& col, int width) {
  const int n = (int)col.size();
  width = std::min(width, n);
  std::vector<double> sums(n, 0.0);
  double s = 0.0;
  for (int i = 0; i < width; ++i) s += std::fabs(col[i]);
  for (int a = 0; a < n; ++a) {
    // recompute exactly every 256 starts to bound drift of the running sum
    if (a % 256 == 0) {
      s = 0.0;
      for (int i = 0; i < width; ++i) s += std::fabs(col[(a + i) % n]);
    }
    sums[a] = s;
    s += std::fabs(col[(a + width) % n]) - std::fabs(col[a]);
  }
  double mx = *std::max_element(sums.begin(), sums.end());
  int start = 0;
  for (int a = 0; a < n; ++a)
    if (sums[a] >= mx * (1.0 - 1e-12)) {
      start = a;
      break;
    }
  std::vector<int> o(width);
  for (int i = 0; i < width; ++i) o[i] = (start + i) % n;
  return o;
}

int psi_hierarchy(int scheme, double cfl, int nx, int m, int levels, int rule,
                  const int* widths, double eta, std::vector<Taps>& out,
                  double& max_imag) {
  Tableau t;
  if (!get_tableau(scheme, t)) return MGRIT_EINVAL;
  if (nx < 2 || m < 2 || levels < 2 || !(cfl > 0.0)) return MGRIT_EINVAL;
  if (rule == MGRIT_PSI_AUTO) rule = t.implicit ? MGRIT_PSI_ETA : MGRIT_PSI_WINDOW;
  out.clear();
  max_imag = 0.0;
  if (rule == MGRIT_PSI_REDISC) {
    if (t.implicit) return MGRIT_EINVAL;
    double c = cfl;
    for (int l = 1; l < levels; ++l) {
      c *= m;
      Taps tp;
      erk_taps(t, c, nx, tp);
      out.push_back(tp);
    }
    return MGRIT_OK;
  }
  if (rule != MGRIT_PSI_WINDOW && rule != MGRIT_PSI_ETA) return MGRIT_EINVAL;
  std::vector<cd> lam(nx);
  {
    std::vector<int> off;
    std::vector<double> d;
    upwind(t.p, off, d);
    for (int k = 0; k < nx; ++k) {
      const double th = 2.0 * kPi * k / nx;
      cd z = 0.0;
      for (size_t j = 0; j < off.size(); ++j) z += d[j] * std::exp(cd(0.0, off[j] * th));
      lam[k] = stability(t, -cfl * z);  // step_symbol at th
    }
  }
  int nnz_prev = 0;
  if (!t.implicit) {
    Taps f;
    erk_taps(t, cfl, nx, f);
    nnz_prev = (int)f.off.size();
  }
  for (int l = 1; l < levels; ++l) {
    std::vector<cd> col(nx);
    for (int k = 0; k < nx; ++k) col[k] = ipow(lam[k], m);
    dft(col, true);
    std::vector<double> rcol(nx);
    for (int k = 0; k < nx; ++k) rcol[k] = col[k].real();
    std::vector<int> offs;
    if (rule == MGRIT_PSI_ETA) {
      double e = eta > 0.0 ? eta : (t.implicit ? eta_table(t.p, m) : -1.0);
      if (e <= 0.0) return MGRIT_EINVAL;
      offs = threshold(rcol, e);
    } else {
      int wdt = widths ? widths[l - 1]
                       : std::max(nnz_prev, cyclic_span(threshold(rcol, 0.02), nx));
      if (wdt < 1) return MGRIT_EINVAL;
      offs = best_window(rcol, wdt);
    }
    Taps tp;
    tp.off = offs;
    max_imag = std::max(max_imag, lsq_psi(lam, m, offs, tp.w));
    taps_eigs(tp, nx, lam);
    nnz_prev = (int)offs.size();
    out.push_back(tp);
  }
  return max_imag > 1e-8 ? MGRIT_EIMAG : MGRIT_OK;
}

// ---------------------------------------------------------------------------
// Bound-driven windows: eq. (7) per mode, the window width chosen per level
// ---------------------------------------------------------------------------
// sum_{j < N} a^j, evaluated without cancellation near a = 1
// sum_{j<N} a^j; within 1e-12 of a = 1 its first-order expansion
// N + N(N-1)/2 (a-1), whose next term is below rounding there
static double geometric_sum(double a, double N) {
  if (std::fabs(1.0 - a) < 1e-12) return N + 0.5 * N * (N - 1.0) * (a - 1.0);
  return std::expm1(N * std::log(a)) / (a - 1.0);
}

double two_level_bound_max(const std::vector<cd>& lam, const std::vector<cd>& mu, int m,
                           long long nt) {
  const double N = (double)(nt / m) - 1.0;
  double b = 0.0;
  for (size_t k = 0; k < lam.size(); ++k) {
    const double am = std::abs(mu[k]);
    const double v = std::sqrt((double)m) * std::pow(std::abs(lam[k]), m) *
                     std::abs(ipow(lam[k], m) - mu[k]) * geometric_sum(am, N);
    if (!std::isfinite(v)) return HUGE_VAL;  // overflow: never a choice
    b = std::max(b, v);
  }
  return b;
}

int psi_hierarchy_bound(int scheme, double cfl, int nx, int nt, int m, int levels,
                        double target, int max_width, std::vector<Taps>& out,
                        std::vector<double>& bounds, double& max_imag) {
  Tableau t;
  if (!get_tableau(scheme, t) || t.implicit) return MGRIT_EINVAL;
  if (nx < 2 || nt < 1 || m < 2 || levels < 2 || !(cfl > 0.0) || !(target > 0.0) ||
      max_width < 1)
    return MGRIT_EINVAL;
  long long span = 1;
  for (int l = 1; l < levels; ++l) span *= m;
  if (span > nt || nt % span) return MGRIT_EINVAL;
  out.clear();
  bounds.clear();
  max_imag = 0.0;
  std::vector<cd> lam(nx);
  {
    std::vector<int> off;
    std::vector<double> d;
    upwind(t.p, off, d);
    for (int k = 0; k < nx; ++k) {
      const double th = 2.0 * kPi * k / nx;
      cd z = 0.0;
      for (size_t j = 0; j < off.size(); ++j) z += d[j] * std::exp(cd(0.0, off[j] * th));
      lam[k] = stability(t, -cfl * z);
    }
  }
  Taps f;
  erk_taps(t, cfl, nx, f);
  int nnz_prev = (int)f.off.size();
  long long n = nt;
  for (int l = 1; l < levels; ++l) {
    std::vector<cd> col(nx);
    for (int k = 0; k < nx; ++k) col[k] = ipow(lam[k], m);
    dft(col, true);
    std::vector<double> rcol(nx);
    for (int k = 0; k < nx; ++k) rcol[k] = col[k].real();
    const int w0 = std::max(nnz_prev, cyclic_span(threshold(rcol, 0.02), nx));
    const int w1 = std::max(w0, std::min(max_width, nx));
    // bounds below kBoundFloor are at the rounding level of the fit: such a
    // width meets any target; without one, the narrowest width within
    // kBoundTie of the smallest bound
    constexpr double kBoundFloor = 1e-10, kBoundTie = 1e-3;
    const double T = std::max(target, kBoundFloor);
    std::vector<Taps> cand;
    std::vector<std::vector<cd>> cand_mu;
    std::vector<double> cand_b;
    int chosen = -1;
    for (int W = w0; W <= w1 && chosen < 0; ++W) {
      Taps tp;
      tp.off = best_window(rcol, W);
      max_imag = std::max(max_imag, lsq_psi(lam, m, tp.off, tp.w));
      std::vector<cd> mu;
      taps_eigs(tp, nx, mu);
      const double b = two_level_bound_max(lam, mu, m, n);
      cand.push_back(tp);
      cand_mu.push_back(std::move(mu));
      cand_b.push_back(b);
      if (b <= T) chosen = (int)cand.size() - 1;
    }
    if (chosen < 0) {
      if (cand.empty()) return MGRIT_EINVAL;
      const double bmin = *std::min_element(cand_b.begin(), cand_b.end());
      for (size_t i = 0; i < cand_b.size() && chosen < 0; ++i)
        if (cand_b[i] <= (1.0 + kBoundTie) * bmin) chosen = (int)i;
    }
    Taps pick = cand[chosen];
    std::vector<cd> pick_mu;
    pick_mu.swap(cand_mu[chosen]);
    const double pick_b = cand_b[chosen];
    nnz_prev = (int)pick.off.size();
    lam.swap(pick_mu);
    out.push_back(pick);
    bounds.push_back(pick_b);
    n /= m;
  }
  return max_imag > 1e-8 ? MGRIT_EIMAG : MGRIT_OK;
}

void tap_window(const Taps& t, int nx, int& omin, int& W, std::vector<double>& dense) {
  std::map<int, double> f;
  for (size_t q = 0; q < t.off.size(); ++q) f[((t.off[q] % nx) + nx) % nx] += t.w[q];
  std::vector<int> s;
  for (auto& a : f) s.push_back(a.first);
  if (s.empty()) {
    omin = 0;
    W = 1;
    dense.assign(1, 0.0);
    return;
  }
  // the window starts right after the largest cyclic gap
  int best_gap = s.front() + nx - s.back(), start = s.front();
  for (size_t i = 1; i < s.size(); ++i)
    if (s[i] - s[i - 1] > best_gap) {
      best_gap = s[i] - s[i - 1];
      start = s[i];
    }
  W = (s.size() == 1) ? 1 : nx - best_gap + 1;
  omin = start;
  dense.assign(W, 0.0);
  for (auto& a : f) dense[((a.first - omin) % nx + nx) % nx] += a.second;
}

// ---------------------------------------------------------------------------
// SDIRK stage matrix M = I - gamma dt L as cyclic recurrences
// ---------------------------------------------------------------------------
using ld = long double;
using cld = std::complex<long double>;

// Roots of sum_q p[q] s^q (degree D = p.size()-1) in extended precision:
// Durand-Kerner iterations, then Newton steps on each root.
static std::vector<cld> poly_roots(const std::vector<ld>& p) {
  const int D = (int)p.size() - 1;
  std::vector<cld> a(D + 1);
  for (int q = 0; q <= D; ++q) a[q] = p[q] / p[D];
  auto ev = [&](cld z) {
    cld r = a[D];
    for (int q = D - 1; q >= 0; --q) r = r * z + a[q];
    return r;
  };
  auto dev = [&](cld z) {
    cld r = (ld)D * a[D];
    for (int q = D - 1; q >= 1; --q) r = r * z + (ld)q * a[q];
    return r;
  };
  std::vector<cld> z(D);
  const cld seed(0.4L, 0.9L);
  for (int i = 0; i < D; ++i) z[i] = std::pow(seed, i) * (1.0L + std::abs(a[0]));
  for (int it = 0; it < 2000; ++it) {
    ld delta = 0.0L;
    for (int i = 0; i < D; ++i) {
      cld den = 1.0L;
      for (int j = 0; j < D; ++j)
        if (j != i) den *= (z[i] - z[j]);
      const cld dz = ev(z[i]) / den;
      z[i] -= dz;
      delta = std::max(delta, std::abs(dz));
    }
    if (delta < 1e-19L) break;
  }
  for (int i = 0; i < D; ++i)
    for (int it = 0; it < 3; ++it) {
      const cld d = dev(z[i]);
      if (std::abs(d) > 0) z[i] -= ev(z[i]) / d;
    }
  return z;
}

static void mat2_mul(const ld* a, const ld* b, ld* c) {
  ld r[4] = {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3],
             a[2] * b[0] + a[3] * b[2], a[2] * b[1] + a[3] * b[3]};
  for (int i = 0; i < 4; ++i) c[i] = r[i];
}

static void mat2_pow(const ld* a, long long e, ld* out) {
  ld r[4] = {1, 0, 0, 1}, b[4] = {a[0], a[1], a[2], a[3]};
  while (e > 0) {
    if (e & 1) mat2_mul(r, b, r);
    mat2_mul(b, b, b);
    e >>= 1;
  }
  for (int i = 0; i < 4; ++i) out[i] = r[i];
}

// The stage matrix M = I - gamma dt L = K prod_f (1 - a1_f X - a2_f X^2)
// (X the shift S or S^{-1}) is applied as M^{-1} = scale prod_f (factor
// f)^{-1}.  Roots, factors and the scan constants are computed in extended
// precision and rounded to FP64 once.  On the constant mode (theta = 0) the
// exact M is 1 (the upwind weights sum to zero), and any error of the
// rounded M^{-1} there is repeated every stage of every step: the mean
// drifts n_t-fold.  So the FP64 factor coefficients are taken within a few
// units in the last place of their values such that scale, the FP64 value
// nearest to prod_f (1 - a1_f - a2_f), reproduces that product most
// closely.
bool sdirk_setup(const Tableau& t, double cfl, int K, int NL, SdirkDev& out,
                 std::string& err) {
  out = SdirkDev();
  if (!t.implicit) {
    err = "not an SDIRK scheme";
    return false;
  }
  const double g = t.A[0][0];
  for (int i = 1; i < t.s; ++i)
    if (std::fabs(t.A[i][i] - g) > 1e-15) {
      err = "tableau is not singly diagonal";
      return false;
    }
  TableauOf<ld> tl;
  if (!tableau_of(t.p + 10, tl)) {
    err = "unknown SDIRK scheme";
    return false;
  }
  const ld gl = tl.A[0][0];
  // (M u)_i = sum_j coef_j u_{i+j};  M = I + gamma c D.
  std::map<int, ld> coef;
  for (const UpwindTerm& u : upwind_terms(t.p))
    coef[u.off] += gl * (ld)cfl * ((ld)u.num / (ld)u.den);
  coef[0] += 1.0L;
  const int jmin = coef.begin()->first, jmax = coef.rbegin()->first;
  const int D = jmax - jmin;
  // S^{jmax} M = P(S), P(s) = sum_j coef_j s^{jmax - j}, S u_i = u_{i-1}
  std::vector<ld> p(D + 1, 0.0L);
  for (auto& c : coef) p[jmax - c.first] = c.second;
  std::vector<cld> r = poly_roots(p);
  std::vector<cld> outside, inside;
  for (auto& z : r) {
    if (std::fabs(std::abs(z) - 1.0L) < 1e-10L) {
      err = "stage matrix has a root on the unit circle";
      return false;
    }
    (std::abs(z) > 1.0L ? outside : inside).push_back(z);
  }
  if ((int)inside.size() != jmax) {
    err = "unexpected root split of the stage matrix";
    return false;
  }
  // factors of order <= 2 with real coefficients, in extended precision
  struct Fac {
    int dir;
    ld a1, a2;
  };
  auto make_factors = [&](std::vector<cld> roots, int dir) {
    std::vector<Fac> fs;
    std::vector<bool> used(roots.size(), false);
    std::vector<ld> reals;
    for (size_t i = 0; i < roots.size(); ++i) {
      if (used[i]) continue;
      if (std::fabs(roots[i].imag()) > 1e-12L * std::abs(roots[i])) {
        size_t best = i;
        ld bd = 1e300L;
        for (size_t j = 0; j < roots.size(); ++j)
          if (j != i && !used[j]) {
            const ld dd = std::abs(roots[j] - std::conj(roots[i]));
            if (dd < bd) {
              bd = dd;
              best = j;
            }
          }
        used[i] = used[best] = true;
        const cld q1 = dir > 0 ? 1.0L / roots[i] : roots[i];
        const cld q2 = dir > 0 ? 1.0L / roots[best] : roots[best];
        fs.push_back({dir, (q1 + q2).real(), -(q1 * q2).real()});
      } else {
        used[i] = true;
        reals.push_back(roots[i].real());
      }
    }
    for (size_t i = 0; i < reals.size(); i += 2) {
      const ld q1 = dir > 0 ? 1.0L / reals[i] : reals[i];
      if (i + 1 < reals.size()) {
        const ld q2 = dir > 0 ? 1.0L / reals[i + 1] : reals[i + 1];
        fs.push_back({dir, q1 + q2, -q1 * q2});
      } else {
        fs.push_back({dir, q1, 0.0L});
      }
    }
    return fs;
  };
  std::vector<Fac> fx = make_factors(outside, +1);
  {
    std::vector<Fac> fb = make_factors(inside, -1);
    fx.insert(fx.end(), fb.begin(), fb.end());
  }
  const int nf = (int)fx.size();
  if (nf > MAX_FACTORS) {
    err = "too many recurrence factors";
    return false;
  }
  // FP64 coefficients: nearest values, then up to three non-zero ones (those
  // with the finest spacing) moved by at most kReach units in the last place
  // where that brings scale * prod_f (factor f)^{-1}, with scale the FP64
  // value nearest to prod_f (1 - a1_f - a2_f), closest to the exact M^{-1}
  // on the constant mode and a few long waves (theta <= 0.05)
  std::vector<double> c64(2 * nf);
  for (int q = 0; q < nf; ++q) {
    c64[2 * q] = (double)fx[q].a1;
    c64[2 * q + 1] = (double)fx[q].a2;
  }
  auto prod_at_one = [&](const std::vector<double>& c) {
    ld pr = 1.0L;
    for (int q = 0; q < nf; ++q) pr *= 1.0L - (ld)c[2 * q] - (ld)c[2 * q + 1];
    return pr;
  };
  const ld kTheta[4] = {0.0L, 0.0125L, 0.025L, 0.05L};
  cld Mex[4];
  for (int k = 0; k < 4; ++k) {
    cld m = 0.0L;
    for (auto& c : coef) m += c.second * std::exp(cld(0.0L, (ld)c.first * kTheta[k]));
    Mex[k] = m;  // symbol of M: (M e)_i = sum_j coef_j e_{i+j}
  }
  auto mismatch = [&](const std::vector<double>& c) {
    const ld sc = (ld)(double)prod_at_one(c);
    ld worst = 0.0L;
    for (int k = 0; k < 4; ++k) {
      cld den = 1.0L;
      for (int q = 0; q < nf; ++q) {
        // S e_i = e_{i-1}: X = e^{-i theta} forward, e^{+i theta} backward
        const cld X = std::exp(cld(0.0L, fx[q].dir > 0 ? -kTheta[k] : kTheta[k]));
        den *= 1.0L - (ld)c[2 * q] * X - (ld)c[2 * q + 1] * X * X;
      }
      worst = std::max(worst, std::abs(sc / den * Mex[k] - 1.0L));
    }
    return worst;
  };
  {
    std::vector<int> idx;
    for (int i = 0; i < 2 * nf; ++i)
      if (c64[i] != 0.0) idx.push_back(i);
    std::sort(idx.begin(), idx.end(),
              [&](int x, int y) { return std::fabs(c64[x]) < std::fabs(c64[y]); });
    if (idx.size() > 3) idx.resize(3);
    constexpr int kReach = 6;
    auto shifted = [](double v, int k) {
      for (; k > 0; --k) v = std::nextafter(v, HUGE_VAL);
      for (; k < 0; ++k) v = std::nextafter(v, -HUGE_VAL);
      return v;
    };
    int r[3] = {0, 0, 0};
    for (size_t i = 0; i < idx.size(); ++i) r[i] = kReach;
    std::vector<double> best = c64;
    ld bm = mismatch(c64);
    for (int k0 = -r[0]; k0 <= r[0]; ++k0)
      for (int k1 = -r[1]; k1 <= r[1]; ++k1)
        for (int k2 = -r[2]; k2 <= r[2]; ++k2) {
          std::vector<double> c = c64;
          const int ks[3] = {k0, k1, k2};
          for (size_t i = 0; i < idx.size(); ++i) c[idx[i]] = shifted(c64[idx[i]], ks[i]);
          const ld mm = mismatch(c);
          if (mm < bm) {
            bm = mm;
            best = c;
          }
        }
    c64 = best;
  }
  // check: K * prod_f (1 - a1 X - a2 X^2) (X = S or S^{-1}) reproduces M
  const ld Kc = 1.0L / prod_at_one(c64);
  {
    std::map<int, ld> prod;
    prod[0] = Kc;
    for (int q = 0; q < nf; ++q) {
      std::map<int, ld> nxt;
      // factor as Laurent polynomial in S: dir +1 -> powers 0, 1, 2 of S
      // (first-column offsets 0, 1, 2); dir -1 -> offsets 0, -1, -2
      const int s1 = fx[q].dir > 0 ? 1 : -1;
      for (auto& a : prod) {
        nxt[a.first] += a.second;
        nxt[a.first + s1] += -(ld)c64[2 * q] * a.second;
        nxt[a.first + 2 * s1] += -(ld)c64[2 * q + 1] * a.second;
      }
      prod.swap(nxt);
    }
    ld mx = 0.0L;
    for (auto& c : coef) mx = std::max(mx, std::fabs(c.second));
    std::map<int, ld> want;  // first-column offsets of M: o = -j
    for (auto& c : coef) want[-c.first] = c.second;
    for (auto& a : prod) {
      const ld w = want.count(a.first) ? want[a.first] : 0.0L;
      if (std::fabs(a.second - w) > 1e-12L * mx) {
        err = "stage-matrix factorization check failed";
        return false;
      }
    }
  }
  out.s = t.s;
  out.nf = nf;
  out.K = K;
  out.NL = NL;
  for (int i = 0; i < t.s; ++i) {
    for (int j = 0; j < t.s; ++j) out.A[i][j] = t.A[i][j];
    out.b[i] = t.b[i];
  }
  out.inv_gamma = (double)(1.0L / gl);
  out.scale = (double)prod_at_one(c64);
  for (int q = 0; q < nf; ++q) {
    RecDev f = {};
    f.dir = fx[q].dir;
    f.a1 = c64[2 * q];
    f.a2 = c64[2 * q + 1];
    const ld C[4] = {(ld)f.a1, (ld)f.a2, 1.0L, 0.0L};
    ld H[4];
    mat2_pow(C, K, H);
    for (int dd = 0; dd < 11; ++dd) {
      ld Hd[4];
      mat2_pow(H, 1LL << dd, Hd);
      for (int i = 0; i < 4; ++i) f.Hp[dd][i] = (double)Hd[i];
    }
    ld HN[4];
    mat2_pow(H, NL, HN);
    const ld a = 1.0L - HN[0], b = -HN[1], c = -HN[2], e = 1.0L - HN[3];
    const ld det = a * e - b * c;
    if (!(std::fabs(det) > 1e-300L)) {
      err = "singular cyclic closure";
      return false;
    }
    f.Cinv[0] = (double)(e / det);
    f.Cinv[1] = (double)(-b / det);
    f.Cinv[2] = (double)(-c / det);
    f.Cinv[3] = (double)(a / det);
    out.f[q] = f;
  }
  return true;
}

// ---------------------------------------------------------------------------
// SDIRK stage matrix in partial fractions (SdirkPfDev)
// ---------------------------------------------------------------------------
// With z the symbol of the shift S (z = e^{-i theta} on Fourier mode theta),
// M(z) = sum_j coef_j z^{-j} and z^{jmax} M(z) = P(z).  Every simple root rho
// of P gives one term of 1/M: outside the unit circle a forward recurrence
// (1 - q z)^{-1}, q = 1/rho, with residue A = -q / M'(rho); inside a
// backward one (1 - rho z^{-1})^{-1}, q = rho, with A = (1/rho) / M'(rho);
// c0 = 1/M(infinity) - sum of the backward residues.  Computed in extended
// precision; the FP64 constants are the nearest ones, with c0 and the term
// coefficient of finest spacing moved by up to kReach units in the last
// place where that reproduces M^{-1} on the constant mode and long waves
// (theta <= 0.04) more closely (each rounding error there is repeated in
// every stage of every step).
bool sdirk_setup_pf(const Tableau& t, double cfl, int K, int NL, SdirkPfDev& out,
                    std::string& err) {
  out = SdirkPfDev();
  if (!t.implicit) {
    err = "not an SDIRK scheme";
    return false;
  }
  for (int i = 1; i < t.s; ++i)
    if (std::fabs(t.A[i][i] - t.A[0][0]) > 1e-15) {
      err = "tableau is not singly diagonal";
      return false;
    }
  TableauOf<ld> tl;
  if (!tableau_of(t.p + 10, tl)) {
    err = "unknown SDIRK scheme";
    return false;
  }
  const ld gl = tl.A[0][0];
  std::map<int, ld> coef;
  for (const UpwindTerm& u : upwind_terms(t.p))
    coef[u.off] += gl * (ld)cfl * ((ld)u.num / (ld)u.den);
  coef[0] += 1.0L;
  const int jmin = coef.begin()->first, jmax = coef.rbegin()->first;
  const int D = jmax - jmin;
  std::vector<ld> p(D + 1, 0.0L);
  for (auto& c : coef) p[jmax - c.first] = c.second;
  std::vector<cld> roots = poly_roots(p);
  auto Mof = [&](cld z) {
    cld v = 0.0L;
    for (auto& c : coef) v += c.second * std::pow(z, -c.first);
    return v;
  };
  auto dMof = [&](cld z) {
    cld v = 0.0L;
    for (auto& c : coef) v += -(ld)c.first * c.second * std::pow(z, -c.first - 1);
    return v;
  };
  struct Term {
    int dir;
    cld q, a;
    bool cx;
  };
  std::vector<Term> real, cplx;
  for (const cld& rho : roots) {
    const ld mag = std::abs(rho);
    if (std::fabs(mag - 1.0L) < 1e-10L) {
      err = "stage matrix has a root on the unit circle";
      return false;
    }
    const bool is_real = std::fabs(rho.imag()) <= 1e-12L * mag;
    if (!is_real && rho.imag() < 0) continue;  // its conjugate carries the pair
    const cld r = is_real ? cld(rho.real(), 0.0L) : rho;
    const cld dm = dMof(r);
    Term tm;
    if (mag > 1.0L) {
      tm.dir = +1;
      tm.q = 1.0L / r;
      tm.a = -tm.q / dm;
    } else {
      tm.dir = -1;
      tm.q = r;
      tm.a = (1.0L / r) / dm;
    }
    tm.cx = !is_real;
    if (tm.cx) cplx.push_back(tm);
    else {
      tm.q = cld(tm.q.real(), 0.0L);
      tm.a = cld(tm.a.real(), 0.0L);
      real.push_back(tm);
    }
  }
  if ((int)(real.size() + 2 * cplx.size()) != D) {
    err = "stage matrix roots are not simple";
    return false;
  }
  if (real.size() + cplx.size() > (size_t)MAX_PF_TERMS) {
    err = "too many partial-fraction terms";
    return false;
  }
  const ld m_inf = jmin < 0 ? 0.0L : 1.0L / coef[0];  // 1/M at z -> infinity
  ld c0 = m_inf;
  for (const Term& tm : real)
    if (tm.dir < 0) c0 -= tm.a.real();
  for (const Term& tm : cplx)
    if (tm.dir < 0) c0 -= 2.0L * tm.a.real();
  // order: forward real terms, backward real terms, complex terms (which
  // the kernels run forward)
  std::stable_sort(real.begin(), real.end(),
                   [](const Term& x, const Term& y) { return x.dir > y.dir; });
  for (const Term& tm : cplx)
    if (tm.dir < 0) {
      err = "complex root inside the unit circle";
      return false;
    }
  int nb = 0;
  for (const Term& tm : real) nb += tm.dir < 0;
  std::vector<Term> terms = real;
  terms.insert(terms.end(), cplx.begin(), cplx.end());
  // the decomposition and its conditioning on the unit circle
  auto sum_terms = [&](const std::vector<Term>& ts, ld c, cld z, ld* absum) {
    cld v = c;
    ld sa = std::fabs(c);
    for (const Term& tm : ts) {
      const cld X = tm.dir > 0 ? z : 1.0L / z;
      const cld w = tm.a / (1.0L - tm.q * X);
      if (tm.cx) {
        const cld wc = std::conj(tm.a) / (1.0L - std::conj(tm.q) * X);
        v += w + wc;
        sa += std::abs(w) + std::abs(wc);
      } else {
        v += w;
        sa += std::abs(w);
      }
    }
    if (absum) *absum = sa;
    return v;
  };
  const ld kPi2 = 6.283185307179586476925286766559L;
  for (int k = 0; k < 64; ++k) {
    const cld z = std::exp(cld(0.0L, -kPi2 * k / 64));
    const cld f = 1.0L / Mof(z);
    ld sa = 0.0L;
    const cld v = sum_terms(terms, c0, z, &sa);
    if (std::abs(v - f) > 1e-14L * std::abs(f)) {
      err = "partial-fraction check failed";
      return false;
    }
    if (sa > 64.0L * std::abs(f)) {
      err = "partial-fraction terms cancel (nearly repeated roots)";
      return false;
    }
  }
  // FP64 constants, searched around the nearest values
  const int nt = (int)terms.size();
  std::vector<double> qd(2 * nt), ad(2 * nt);
  for (int i = 0; i < nt; ++i) {
    qd[2 * i] = (double)terms[i].q.real();
    qd[2 * i + 1] = (double)terms[i].q.imag();
    ad[2 * i] = (double)terms[i].a.real();
    ad[2 * i + 1] = (double)terms[i].a.imag();
  }
  const ld kTheta[4] = {0.0L, 0.01L, 0.02L, 0.04L};
  auto mismatch = [&](double c0d, const std::vector<double>& a) {
    std::vector<Term> ts = terms;
    for (int i = 0; i < nt; ++i) {
      ts[i].q = cld((ld)qd[2 * i], (ld)qd[2 * i + 1]);
      ts[i].a = cld((ld)a[2 * i], (ld)a[2 * i + 1]);
    }
    ld worst = 0.0L;
    for (ld th : kTheta) {
      const cld z = std::exp(cld(0.0L, -th));
      worst = std::max(worst, std::abs(sum_terms(ts, (ld)c0d, z, nullptr) * Mof(z) - 1.0L));
    }
    return worst;
  };
  constexpr int kReach = 12;
  auto shifted = [](double v, int k) {
    for (; k > 0; --k) v = std::nextafter(v, HUGE_VAL);
    for (; k < 0; ++k) v = std::nextafter(v, -HUGE_VAL);
    return v;
  };
  int fine = -1;  // the non-zero coefficient component of finest spacing
  for (int i = 0; i < 2 * nt; ++i)
    if (ad[i] != 0.0 && (fine < 0 || std::fabs(ad[i]) < std::fabs(ad[fine]))) fine = i;
  double c0d = (double)c0;
  {
    double best_c = c0d;
    std::vector<double> best_a = ad;
    ld bm = mismatch(c0d, ad);
    const double c0n = c0d;
    for (int k0 = -kReach; k0 <= kReach; ++k0)
      for (int k1 = (fine < 0 ? 0 : -kReach); k1 <= (fine < 0 ? 0 : kReach); ++k1) {
        std::vector<double> a = ad;
        if (fine >= 0) a[fine] = shifted(ad[fine], k1);
        const double c = c0n == 0.0 && k0 == 0 ? 0.0 : shifted(c0n, k0);
        const ld mm = mismatch(c, a);
        if (mm < bm) {
          bm = mm;
          best_c = c;
          best_a = a;
        }
      }
    c0d = best_c;
    ad = best_a;
  }
  out.s = t.s;
  out.nr = (int)real.size();
  out.nb = nb;
  out.nc = (int)cplx.size();
  out.K = K;
  out.NL = NL;
  for (int i = 0; i < t.s; ++i)
    for (int j = 0; j < t.s; ++j) out.A[i][j] = t.A[i][j];
  out.inv_gamma = (double)(1.0L / gl);
  out.c0 = c0d;
  for (int i = 0; i < nt; ++i) {
    PfTermDev& f = out.t[i];
    f.dir = terms[i].dir;
    f.q[0] = qd[2 * i];
    f.q[1] = qd[2 * i + 1];
    f.a[0] = ad[2 * i];
    f.a[1] = ad[2 * i + 1];
    // chunk factor Q = q^K and its powers, from the FP64 q, in extended
    // precision
    const cld q((ld)f.q[0], (ld)f.q[1]);
    cld Q = 1.0L;
    for (int k = 0; k < K; ++k) Q *= q;
    cld pw = Q;
    for (int d = 0; d < 11; ++d) {
      f.Qp[d][0] = (double)pw.real();
      f.Qp[d][1] = (double)pw.imag();
      pw *= pw;
    }
    cld QN = 1.0L;
    for (int l = 0; l < NL; ++l) QN *= Q;
    const cld cl = 1.0L / (1.0L - QN);
    f.close[0] = (double)cl.real();
    f.close[1] = (double)cl.imag();
  }
  return true;
}

}  // namespace mgr
