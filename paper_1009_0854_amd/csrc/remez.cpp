// mact_fit: FP64 Remez exchange for minimax polynomials and rationals
// (Sec. 3.1: the minimax criterion and the Remez exchange algorithm).
//
// The approximant p/q is solved in the Chebyshev basis of s = (2x - a - b)/(b - a)
// and returned in monomial form in x.  Each iteration
//   1. levels the error on the current reference x_0 < ... < x_{N-1}
//      (N = n + m + 2): p(x_i) - f(x_i) q(x_i) = (-1)^i E q(x_i).  The E q term
//      is linearised with the previous denominator and the linear system is
//      solved again until E settles (for m = 0 one solve is exact);
//   2. checks that q keeps one sign on [a, b] (no pole);
//   3. samples the error densely, keeps the largest point of every run of
//      equal sign, and refines each by golden-section search;
//   4. exchanges: the alternating run of N points that holds the largest error;
//   5. stops when max|e| and the smallest levelled error agree to 1e-8.
// A reference that yields a pole is replaced by the alternation set of the
// next lower denominator degree with one point inserted (continuation).
//
// mact_fit_weighted: the same with a positive weight w, levelling
// w (p/q - f): the levelled equations carry (-1)^i E q(x_i) / w(x_i), and the
// extrema, the exchange and the reported eps are those of the weighted error.
// w is given as samples at equally spaced points, linear in between.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <vector>

#include "common.h"

namespace mact {
namespace {

double eval_fn(int fn, double x) {
  switch (fn) {
    case MACT_FN_CBRT: return std::cbrt(x);
    case MACT_FN_ATAN_SQRT3: return std::atan(std::sqrt(3.0) * x);
    case MACT_FN_ASIN2: return 2.0 * std::asin(x / std::sqrt(2.0));
    case MACT_FN_ACOS: return std::acos(x);
    case MACT_FN_ATAN: return std::atan(x);
    case MACT_FN_ATANC: return 0.5 * kPi - std::atan(x);
    case MACT_FN_SIN: return std::sin(x);
    case MACT_FN_COS: return std::cos(x);
    case MACT_FN_ENC709: return 1.099 * std::pow(x, 0.45) - 0.099;
    case MACT_FN_DEC709: return std::pow((x + 0.099) / 1.099, 1.0 / 0.45);
  }
  return NAN;
}

bool domain_ok(int fn, double lo, double hi) {
  switch (fn) {
    case MACT_FN_CBRT: return lo >= 0.0;
    case MACT_FN_ASIN2: return lo >= 0.0 && hi <= std::sqrt(2.0);
    case MACT_FN_ACOS: return lo >= -1.0 && hi <= 1.0;
    case MACT_FN_ENC709: return lo > 0.0;
    case MACT_FN_DEC709: return lo > -0.099;
    default: return true;
  }
}

// Clenshaw evaluation of sum_k c[k] T_k(s).
double cheb(const std::vector<double>& c, double s) {
  double b1 = 0.0, b2 = 0.0;
  for (int k = (int)c.size() - 1; k >= 1; --k) {
    double t = 2.0 * s * b1 - b2 + c[k];
    b2 = b1;
    b1 = t;
  }
  return s * b1 - b2 + c[0];
}

// Dense solve with partial pivoting; A is row-major N x N.
bool solve(std::vector<double> A, std::vector<double>& b, int N) {
  for (int col = 0; col < N; ++col) {
    int piv = col;
    for (int r = col + 1; r < N; ++r)
      if (std::fabs(A[r * N + col]) > std::fabs(A[piv * N + col])) piv = r;
    if (A[piv * N + col] == 0.0 || !std::isfinite(A[piv * N + col])) return false;
    if (piv != col) {
      for (int k = 0; k < N; ++k) std::swap(A[col * N + k], A[piv * N + k]);
      std::swap(b[col], b[piv]);
    }
    for (int r = col + 1; r < N; ++r) {
      double f = A[r * N + col] / A[col * N + col];
      if (f == 0.0) continue;
      for (int k = col; k < N; ++k) A[r * N + k] -= f * A[col * N + k];
      b[r] -= f * b[col];
    }
  }
  for (int r = N - 1; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < N; ++k) s -= A[r * N + k] * b[k];
    b[r] = s / A[r * N + r];
    if (!std::isfinite(b[r])) return false;
  }
  return true;
}

struct Problem {
  int fn, n, m;
  double a, b;
  // weight samples at nw equally spaced points of [a, b], linear in between; none = 1
  const double* w = nullptr;
  int nw = 0;
  double to_s(double x) const { return (2.0 * x - a - b) / (b - a); }
  double f(double x) const { return eval_fn(fn, x); }
  double weight(double x) const {
    if (!w) return 1.0;
    double u = (x - a) / (b - a) * (nw - 1);
    if (!(u > 0.0)) return w[0];
    if (u >= nw - 1) return w[nw - 1];
    int i = (int)u;
    if (i > nw - 2) i = nw - 2;
    double r = u - i;
    return w[i] + r * (w[i + 1] - w[i]);
  }
};

struct Approx {
  std::vector<double> cp, cq;  // Chebyshev coefficients; cq[0] = 1
  double E = 0.0;
  double value(const Problem& pr, double x) const {
    double s = pr.to_s(x);
    return cheb(cp, s) / cheb(cq, s);
  }
  // the weighted error w (p/q - f) whose maximum the fit levels
  double err(const Problem& pr, double x) const { return pr.weight(x) * (value(pr, x) - pr.f(x)); }
};

void cheb_row(double s, int deg, double* out) {
  out[0] = 1.0;
  if (deg >= 1) out[1] = s;
  for (int k = 2; k <= deg; ++k) out[k] = 2.0 * s * out[k - 1] - out[k - 2];
}

bool q_has_no_root(const Problem& pr, const Approx& ap) {
  if (pr.m == 0) return true;
  const int G = 2048;
  double first = 0.0;
  for (int i = 0; i <= G; ++i) {
    double s = -1.0 + 2.0 * i / G;
    double q = cheb(ap.cq, s);
    if (!std::isfinite(q) || q == 0.0) return false;
    if (i == 0) first = q;
    else if ((q > 0) != (first > 0)) return false;
  }
  return true;
}

// Step 1: levelled solution on the reference.
bool level(const Problem& pr, const std::vector<double>& ref, Approx& ap) {
  const int n = pr.n, m = pr.m, N = n + m + 2;
  std::vector<double> s(N), fi(N), sig(N), qprev(N, 1.0);
  for (int i = 0; i < N; ++i) {
    s[i] = pr.to_s(ref[i]);
    fi[i] = pr.f(ref[i]);
    sig[i] = (i % 2 == 0) ? 1.0 : -1.0;
  }
  std::vector<double> Tn(n + 1), Tm(m + 1);
  double Eold = NAN;
  const int passes = (m == 0) ? 1 : 60;
  for (int pass = 0; pass < passes; ++pass) {
    // unknowns: p_0..p_n, q_1..q_m, E   (q_0 = 1)
    std::vector<double> A(N * N, 0.0), rhs(N);
    for (int i = 0; i < N; ++i) {
      cheb_row(s[i], n, Tn.data());
      for (int k = 0; k <= n; ++k) A[i * N + k] = Tn[k];
      if (m > 0) {
        cheb_row(s[i], m, Tm.data());
        for (int j = 1; j <= m; ++j) A[i * N + n + j] = -fi[i] * Tm[j];
      }
      A[i * N + N - 1] = -sig[i] * qprev[i] / pr.weight(ref[i]);
      rhs[i] = fi[i];
    }
    if (!solve(A, rhs, N)) return false;
    ap.cp.assign(rhs.begin(), rhs.begin() + n + 1);
    ap.cq.assign(m + 1, 0.0);
    ap.cq[0] = 1.0;
    for (int j = 1; j <= m; ++j) ap.cq[j] = rhs[n + j];
    ap.E = rhs[N - 1];
    if (m == 0) break;
    for (int i = 0; i < N; ++i) qprev[i] = cheb(ap.cq, s[i]);
    if (std::isfinite(Eold) && std::fabs(ap.E - Eold) <= 1e-14 * std::fabs(ap.E) + 1e-300) break;
    Eold = ap.E;
  }
  return q_has_no_root(pr, ap);
}

// Golden-section maximisation of sgn * e on [lo, hi].
double refine(const Problem& pr, const Approx& ap, double lo, double hi, double sgn, double* xbest) {
  const double g = 0.5 * (std::sqrt(5.0) - 1.0);
  double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo);
  double f1 = sgn * ap.err(pr, x1), f2 = sgn * ap.err(pr, x2);
  for (int it = 0; it < 200 && (hi - lo) > 1e-16 * std::max(1.0, std::fabs(hi)); ++it) {
    if (f1 < f2) {
      lo = x1; x1 = x2; f1 = f2;
      x2 = lo + g * (hi - lo); f2 = sgn * ap.err(pr, x2);
    } else {
      hi = x2; x2 = x1; f2 = f1;
      x1 = hi - g * (hi - lo); f1 = sgn * ap.err(pr, x1);
    }
  }
  if (f1 >= f2) { *xbest = x1; return sgn * f1; }
  *xbest = x2;
  return sgn * f2;
}

// Steps 3 and 4.  Returns max |e| and fills the next reference (empty if the
// error does not alternate often enough).
double extrema_exchange(const Problem& pr, const Approx& ap, const std::vector<double>& ref,
                        std::vector<double>& next) {
  const int N = pr.n + pr.m + 2;
  std::vector<double> xs;
  const int G = 8192;
  xs.reserve(G + 64 * N);
  for (int i = 0; i <= G; ++i) xs.push_back(0.5 * (pr.a + pr.b) - 0.5 * (pr.b - pr.a) * std::cos(kPi * i / G));
  for (size_t i = 0; i + 1 < ref.size(); ++i)
    for (int k = 1; k <= 48; ++k) xs.push_back(ref[i] + (ref[i + 1] - ref[i]) * k / 49.0);
  for (double& x : xs) x = std::min(std::max(x, pr.a), pr.b);
  std::sort(xs.begin(), xs.end());
  xs.erase(std::unique(xs.begin(), xs.end()), xs.end());
  const int M = (int)xs.size();
  std::vector<double> es(M);
  for (int i = 0; i < M; ++i) es[i] = ap.err(pr, xs[i]);
  // one candidate (grid index) per run of equal sign
  std::vector<int> cand;
  for (int i = 0; i < M; ++i) {
    if (es[i] == 0.0) continue;
    if (!cand.empty() && (es[cand.back()] > 0) == (es[i] > 0)) {
      if (std::fabs(es[i]) > std::fabs(es[cand.back()])) cand.back() = i;
    } else {
      cand.push_back(i);
    }
  }
  std::vector<double> px, pe;
  double emax = 0.0;
  for (int i : cand) {
    double x = xs[i], e = es[i];
    if (i > 0 && i < M - 1) {
      double sgn = e > 0 ? 1.0 : -1.0, xr;
      double er = refine(pr, ap, xs[i - 1], xs[i + 1], sgn, &xr);
      if (std::fabs(er) > std::fabs(e)) { x = xr; e = er; }
    }
    px.push_back(x);
    pe.push_back(e);
    emax = std::max(emax, std::fabs(e));
  }
  next.clear();
  if ((int)px.size() < N) return emax;
  int lo = 0, hi = (int)px.size() - 1;  // cut from the smaller end, keep the global max
  int gmax = 0;
  for (int i = 0; i < (int)pe.size(); ++i)
    if (std::fabs(pe[i]) > std::fabs(pe[gmax])) gmax = i;
  while (hi - lo + 1 > N) {
    bool drop_lo = std::fabs(pe[lo]) <= std::fabs(pe[hi]);
    if (lo == gmax) drop_lo = false;
    if (hi == gmax) drop_lo = true;
    if (drop_lo) ++lo; else --hi;
  }
  next.assign(px.begin() + lo, px.begin() + hi + 1);
  return emax;
}

// Chebyshev series in s -> monomial coefficients in x.
std::vector<double> to_monomial(const std::vector<double>& c, double a, double b) {
  const int d = (int)c.size() - 1;
  // monomial in s of each T_k
  std::vector<std::vector<double>> T(d + 1, std::vector<double>(d + 1, 0.0));
  T[0][0] = 1.0;
  if (d >= 1) T[1][1] = 1.0;
  for (int k = 2; k <= d; ++k)
    for (int j = 0; j <= d; ++j) T[k][j] = (j > 0 ? 2.0 * T[k - 1][j - 1] : 0.0) - T[k - 2][j];
  std::vector<double> ms(d + 1, 0.0);
  for (int k = 0; k <= d; ++k)
    for (int j = 0; j <= d; ++j) ms[j] += c[k] * T[k][j];
  // substitute s = alpha x + beta (Horner on polynomials)
  const double alpha = 2.0 / (b - a), beta = -(a + b) / (b - a);
  std::vector<double> out(d + 1, 0.0);
  out[0] = ms[d];
  for (int k = d - 1; k >= 0; --k) {
    std::vector<double> nxt(d + 1, 0.0);
    for (int j = 0; j < d; ++j) {
      nxt[j + 1] += out[j] * alpha;
      nxt[j] += out[j] * beta;
    }
    nxt[0] += ms[k];
    out = nxt;
  }
  return out;
}

double horner(const double* c, int deg, double x) {
  double acc = c[deg];
  for (int k = deg - 1; k >= 0; --k) acc = acc * x + c[k];
  return acc;
}

// max |w (p/q - f)| of the monomial form on a dense grid, refined near the top samples.
double monomial_eps(const Problem& pr, const mact_approx& o) {
  auto e = [&](double x) { return std::fabs(pr.weight(x) * (horner(o.p, o.n, x) / horner(o.q, o.m, x) - pr.f(x))); };
  const int G = 1 << 16;
  double best = 0.0;
  std::vector<std::pair<double, int>> top;
  std::vector<double> xs(G + 1);
  for (int i = 0; i <= G; ++i) {
    xs[i] = std::min(std::max(0.5 * (pr.a + pr.b) - 0.5 * (pr.b - pr.a) * std::cos(kPi * i / G), pr.a), pr.b);
    double v = e(xs[i]);
    best = std::max(best, v);
    top.push_back({v, i});
  }
  std::partial_sort(top.begin(), top.begin() + 16, top.end(), [](auto& l, auto& r) { return l.first > r.first; });
  for (int t = 0; t < 16; ++t) {
    int i = top[t].second;
    double lo = xs[std::max(i - 1, 0)], hi = xs[std::min(i + 1, G)];
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo), f1 = e(x1), f2 = e(x2);
    for (int it = 0; it < 120 && hi - lo > 1e-17; ++it) {
      if (f1 < f2) { lo = x1; x1 = x2; f1 = f2; x2 = lo + g * (hi - lo); f2 = e(x2); }
      else { hi = x2; x2 = x1; f2 = f1; x1 = hi - g * (hi - lo); f1 = e(x1); }
    }
    best = std::max(best, std::max(f1, f2));
  }
  return best;
}

struct Result {
  Approx ap;
  std::vector<double> alt;
  double eps = INFINITY;
  int iters = 0;
  bool converged = false;
  bool ok = false;
};

Result run(const Problem& pr, std::vector<double> ref, int max_iter) {
  Result best;
  const int N = pr.n + pr.m + 2;
  for (int it = 1; it <= max_iter; ++it) {
    Approx ap;
    if (!level(pr, ref, ap)) break;
    std::vector<double> next;
    double emax = extrema_exchange(pr, ap, ref, next);
    if (emax < best.eps) {
      best.ap = ap;
      best.eps = emax;
      best.alt = next.empty() ? ref : next;
      best.iters = it;
      best.ok = true;
    }
    if ((int)next.size() != N) break;
    double emin = INFINITY;
    for (double x : next) emin = std::min(emin, std::fabs(ap.err(pr, x)));
    ref = next;
    if (emax - emin <= 1e-8 * emax) {
      best.ap = ap;
      best.eps = emax;
      best.alt = next;
      best.iters = it;
      best.converged = true;
      best.ok = true;
      break;
    }
  }
  return best;
}

std::vector<double> cheb_reference(const Problem& pr) {
  const int N = pr.n + pr.m + 2;
  std::vector<double> r(N);
  for (int i = 0; i < N; ++i) r[i] = 0.5 * (pr.a + pr.b) - 0.5 * (pr.b - pr.a) * std::cos(kPi * i / (N - 1));
  return r;
}

Result fit_problem(const Problem& pr, int max_iter, int depth) {
  Result r = run(pr, cheb_reference(pr), max_iter);
  if ((r.ok && r.converged) || depth > 8 || pr.m == 0) return r;
  // continuation from the next lower denominator degree
  Problem lower = pr;
  lower.m -= 1;
  lower.n += 0;
  Result lr = fit_problem(lower, max_iter, depth + 1);
  if (!lr.ok || (int)lr.alt.size() != pr.n + pr.m + 1) return r.ok ? r : lr;
  std::vector<double> ref = lr.alt;
  size_t gap = 0;
  for (size_t i = 1; i + 1 < ref.size(); ++i)
    if (ref[i + 1] - ref[i] > ref[gap + 1] - ref[gap]) gap = i;
  ref.insert(ref.begin() + gap + 1, 0.5 * (ref[gap] + ref[gap + 1]));
  Result c = run(pr, ref, max_iter);
  if (c.ok && (!r.ok || c.converged || c.eps < r.eps)) return c;
  return r;
}

}  // namespace
}  // namespace mact

using namespace mact;

namespace {
mact_status fit_impl(int32_t fn, int32_t n, int32_t m, double lo, double hi, const double* w, int32_t nw,
                     int32_t max_iter, mact_approx* out) {
  if (!out) return fail(MACT_E_INVALID, "mact_fit: out is NULL");
  if (fn < 0 || fn >= MACT_FN_COUNT) return fail(MACT_E_INVALID, "mact_fit: unknown function %d", fn);
  if (n < 0 || n > MACT_MAX_DEGREE || m < 0 || m > MACT_MAX_DEGREE)
    return fail(MACT_E_INVALID, "mact_fit: degrees (%d, %d) outside 0..%d", n, m, MACT_MAX_DEGREE);
  if (n + m + 2 > 18) return fail(MACT_E_INVALID, "mact_fit: n + m + 2 = %d exceeds 18", n + m + 2);
  if (!(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi))
    return fail(MACT_E_INVALID, "mact_fit: interval [%g, %g] is empty or not finite", lo, hi);
  if (!domain_ok(fn, lo, hi)) return fail(MACT_E_INVALID, "mact_fit: [%g, %g] leaves the domain of function %d", lo, hi, fn);
  if (max_iter < 1) return fail(MACT_E_INVALID, "mact_fit: max_iter %d < 1", max_iter);

  Problem pr{fn, n, m, lo, hi, w, nw};
  Result r = fit_problem(pr, max_iter, 0);
  std::memset(out, 0, sizeof *out);
  out->fn = fn;
  out->n = n;
  out->m = m;
  out->lo = lo;
  out->hi = hi;
  if (!r.ok) return fail(MACT_E_NOCONV, "mact_fit: no pole-free levelled solution for (%d, %d)", n, m);
  std::vector<double> p = to_monomial(r.ap.cp, lo, hi);
  std::vector<double> q = to_monomial(r.ap.cq, lo, hi);
  const double q0 = q[0];
  for (int k = 0; k <= n; ++k) out->p[k] = p[k] / q0;
  for (int k = 0; k <= m; ++k) out->q[k] = q[k] / q0;
  out->q[0] = 1.0;
  out->iters = r.iters;
  out->converged = r.converged ? 1 : 0;
  out->n_alt = (int32_t)std::min<size_t>(r.alt.size(), 18);
  for (int i = 0; i < out->n_alt; ++i) out->alt[i] = r.alt[i];
  out->eps = monomial_eps(pr, *out);
  if (!r.converged) return fail(MACT_E_NOCONV, "mact_fit: (%d, %d) not levelled after %d iterations (eps %.3e)", n, m, r.iters, out->eps);
  return MACT_OK;
}

}  // namespace

extern "C" mact_status mact_fit_ex(int32_t fn, int32_t n, int32_t m, double lo, double hi, int32_t max_iter,
                                   mact_approx* out) {
  clear_error();
  return fit_impl(fn, n, m, lo, hi, nullptr, 0, max_iter, out);
}

extern "C" mact_status mact_fit(int32_t fn, int32_t n, int32_t m, double lo, double hi, mact_approx* out) {
  return mact_fit_ex(fn, n, m, lo, hi, 100, out);
}

extern "C" mact_status mact_fit_weighted(int32_t fn, int32_t n, int32_t m, double lo, double hi,
                                         const double* weight, int32_t n_weight, int32_t max_iter,
                                         mact_approx* out) {
  clear_error();
  if (!weight) return fail(MACT_E_INVALID, "mact_fit_weighted: weight is NULL");
  if (n_weight < 2 || n_weight > MACT_MAX_WEIGHT_SAMPLES)
    return fail(MACT_E_INVALID, "mact_fit_weighted: n_weight %d outside 2..%d", n_weight, MACT_MAX_WEIGHT_SAMPLES);
  for (int i = 0; i < n_weight; ++i)
    if (!(weight[i] > 0.0) || !std::isfinite(weight[i]))
      return fail(MACT_E_INVALID, "mact_fit_weighted: weight[%d] = %g is not positive and finite", i, weight[i]);
  return fit_impl(fn, n, m, lo, hi, weight, n_weight, max_iter, out);
}
