// Host-side parts of libmact that touch no GPU: status strings and the
// thread-local error, the coefficient tables printed in the paper, the
// library's default approximations, parameter validation, and the FP64 exact
// transforms used to pack LUTs.
#include <cmath>
#include <cstring>
#include <mutex>

#include "common.h"

namespace mact {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = 0; }

// ---------------------------------------------------------------- exact transforms

double inverse_gamma(double k, int gamma) {
  if (gamma == MACT_GAMMA_BT709)  // Sec. 3.2.1
    return k < 0.081 ? k / 4.5 : std::pow((k + 0.099) / 1.099, 1.0 / 0.45);
  if (gamma == MACT_GAMMA_SRGB) return k <= 0.04045 ? k / 12.92 : std::pow((k + 0.055) / 1.055, 2.4);
  return k;
}

static double lab_f(double t) { return t > kLabT0 ? std::cbrt(t) : kLabK * t + kLabC; }

void exact_lab(const double rgb[3], int gamma, double out[3]) {
  double lin[3], f[3];
  for (int c = 0; c < 3; ++c) lin[c] = inverse_gamma(rgb[c], gamma);
  for (int r = 0; r < 3; ++r) {
    double xyz = kM[r][0] * lin[0] + kM[r][1] * lin[1] + kM[r][2] * lin[2];
    f[r] = lab_f(xyz / kWhite[r]);
  }
  out[0] = 116.0 * f[1] - 16.0;
  out[1] = 500.0 * (f[0] - f[1]);
  out[2] = 200.0 * (f[1] - f[2]);
}

void exact_hsi(const double rgb[3], double out[3]) {
  // Kender's form with the exact arctan (Sec. 3.3.1); H = 0 where undefined
  const double R = rgb[0], G = rgb[1], B = rgb[2];
  const double s3 = std::sqrt(3.0);
  double H = 0.0;
  if (R > B && G > B) H = kPi / 3.0 + std::atan(s3 * (G - R) / ((G - B) + (R - B)));
  else if (G > R) H = kPi + std::atan(s3 * (B - G) / ((B - R) + (G - R)));
  else if (B > G) H = 5.0 * kPi / 3.0 + std::atan(s3 * (R - B) / ((R - G) + (B - G)));
  const double sum = R + G + B;
  const double mn = std::fmin(R, std::fmin(G, B));
  out[0] = H;
  out[1] = sum > 0 ? 1.0 - 3.0 * mn / sum : 0.0;
  out[2] = sum / 3.0;
}

void exact_sct(const double rgb[3], double out[3]) {
  const double R = rgb[0], G = rgb[1], B = rgb[2];
  const double L = std::sqrt(R * R + G * G + B * B);
  out[0] = L;
  out[1] = L > 0 ? std::acos(std::fmin(1.0, B / L)) : 0.0;
  out[2] = std::atan2(G, R);
}

void exact_luv(const double rgb[3], int gamma, double out[3]) {
  // CIE 1976 L*u*v* with the CIELAB L* (the extension named in Sec. 4)
  double lin[3], xyz[3];
  for (int c = 0; c < 3; ++c) lin[c] = inverse_gamma(rgb[c], gamma);
  for (int r = 0; r < 3; ++r) xyz[r] = kM[r][0] * lin[0] + kM[r][1] * lin[1] + kM[r][2] * lin[2];
  const double fy = xyz[1] > kLabT0 ? std::cbrt(xyz[1]) : kLabK * xyz[1] + kLabC;
  const double L = 116.0 * fy - 16.0;
  const double d = xyz[0] + 15.0 * xyz[1] + 3.0 * xyz[2];
  const double dn = kWhite[0] + 15.0 * kWhite[1] + 3.0 * kWhite[2];
  out[0] = L;
  out[1] = d > 0.0 ? 13.0 * L * (4.0 * xyz[0] / d - 4.0 * kWhite[0] / dn) : 0.0;
  out[2] = d > 0.0 ? 13.0 * L * (9.0 * xyz[1] / d - 9.0 * kWhite[1] / dn) : 0.0;
}

// ---------------------------------------------------------------- validation

mact_status check_approx(const mact_approx& a, bool rational_ok, const char* what) {
  if (a.n < 0 || a.n > MACT_MAX_DEGREE || a.m < 0 || a.m > MACT_MAX_DEGREE)
    return fail(MACT_E_INVALID, "%s: degrees (%d, %d) outside 0..%d", what, a.n, a.m, MACT_MAX_DEGREE);
  if (a.m > 0 && !rational_ok) return fail(MACT_E_UNSUPPORTED, "%s: rational approximation not supported here", what);
  for (int k = 0; k <= a.n; ++k)
    if (!std::isfinite(a.p[k])) return fail(MACT_E_INVALID, "%s: p[%d] is not finite", what, k);
  for (int k = 0; k <= a.m; ++k)
    if (!std::isfinite(a.q[k])) return fail(MACT_E_INVALID, "%s: q[%d] is not finite", what, k);
  return MACT_OK;
}

mact_status check_params(const mact_params* p) {
  if (!p) return fail(MACT_E_INVALID, "params is NULL");
  if (p->xform < MACT_LAB || p->xform > MACT_LUV) return fail(MACT_E_INVALID, "unknown transform %d", p->xform);
  if (p->out_mode != 0 && p->out_mode != 1) return fail(MACT_E_INVALID, "out_mode %d not 0 or 1", p->out_mode);
  if (p->out_mode == 1 && p->xform != MACT_LAB) return fail(MACT_E_INVALID, "out_mode 1 is for MACT_LAB only");
  const int nf = p->xform == MACT_SCT ? 4 : 1;
  static const char* names[4][4] = {{"cbrt"}, {"atan_sqrt3"}, {"asin2", "acos", "atan", "atanc"}, {"cbrt"}};
  for (int i = 0; i < nf; ++i) {
    mact_status s = check_approx(p->f[i], uses_gamma(p->xform), names[p->xform][i]);
    if (s != MACT_OK) return s;
  }
  if (uses_gamma(p->xform) && p->f[1].fn == MACT_FN_DEC709) {
    mact_status s = check_approx(p->f[1], false, "dec709");
    if (s != MACT_OK) return s;
  }
  return MACT_OK;
}

// ---------------------------------------------------------------- printed tables

namespace {
struct Row {
  int fn, n, m;
  double eps, lo, hi;
  double p[6], q[6];
};
constexpr double k254_256 = 254.0 / 256.0;
const double kInvSqrt2 = 0.70710678118654752440;

const Row kRows[] = {
    // Table 1: cube root, polynomials on [0, 1]
    {MACT_FN_CBRT, 2, 0, 1.271154e-01, 0, 1, {1.268979e-01, 2.393873, -1.647669}, {1}},
    {MACT_FN_CBRT, 3, 0, 9.787829e-02, 0, 1, {9.787826e-02, 4.057495, -7.388864, 4.331370}, {1}},
    {MACT_FN_CBRT, 4, 0, 8.111150e-02, 0, 1, {8.111133e-02, 5.926004, -2.017165e+01, 2.833070e+01, -1.324728e+01}, {1}},
    {MACT_FN_CBRT, 5, 0, 7.002956e-02, 0, 1, {7.002910e-02, 7.961214, -4.329352e+01, 1.063182e+02, -1.135685e+02, 4.358268e+01}, {1}},
    // Table 2: cube root, rationals on [0.008856, 1]
    {MACT_FN_CBRT, 2, 2, 2.060996e-03, kLabT0, 1, {6.309655e-03, 5.785782e-01, 1.591005}, {4.482646e-02, 1.175862, 9.596879e-01}},
    {MACT_FN_CBRT, 2, 3, 7.210231e-04, kLabT0, 1, {2.500705e-03, 3.447113e-01, 1.942708}, {1.978701e-02, 8.542797e-01, 1.664540, -2.503267e-01}},
    {MACT_FN_CBRT, 3, 2, 5.931593e-04, kLabT0, 1, {1.776519e-03, 2.632323e-01, 1.751297, 3.836709e-01}, {1.432256e-02, 6.779998e-01, 1.706260}},
    {MACT_FN_CBRT, 2, 4, 3.107735e-04, kLabT0, 1, {1.317899e-03, 2.390113e-01, 2.099395}, {1.124254e-02, 6.726679e-01, 2.184656, -7.511150e-01, 2.229717e-01}},
    {MACT_FN_CBRT, 3, 3, 1.858694e-04, kLabT0, 1, {4.370889e-04, 9.526952e-02, 1.252009, 1.302733}, {3.912364e-03, 2.954084e-01, 1.717143, 6.343408e-01}},
    {MACT_FN_CBRT, 4, 2, 2.334688e-04, kLabT0, 1, {7.589302e-04, 1.519784e-01, 1.663584, 8.368075e-01, -1.657269e-01}, {6.644723e-03, 4.506424e-01, 2.030622}},
    {MACT_FN_CBRT, 3, 4, 8.539863e-05, kLabT0, 1, {1.683667e-04, 4.667675e-02, 9.106812e-01, 1.810577}, {1.610864e-03, 1.617974e-01, 1.494070, 1.218468, -1.079451e-01}},
    {MACT_FN_CBRT, 4, 3, 8.052920e-05, kLabT0, 1, {1.349673e-04, 3.832079e-02, 7.870174e-01, 1.799062, 2.071170e-01}, {1.299250e-03, 1.345420e-01, 1.330358, 1.365369}},
    {MACT_FN_CBRT, 4, 4, 3.856930e-05, kLabT0, 1, {3.927283e-05, 1.392318e-02, 4.114739e-01, 1.734853, 8.679223e-01}, {4.022100e-04, 5.414536e-02, 8.221526e-01, 1.800167, 3.513617e-01}},
    // Table 3: arctan(sqrt 3 x) on [0, 254/256]; n = 2 with a2 negative (sign lost in print)
    {MACT_FN_ATAN_SQRT3, 2, 0, 6.907910e-03, 0, k254_256, {5.959793e-03, 1.782975, -7.497879e-01}, {1}},
    {MACT_FN_ATAN_SQRT3, 3, 0, 3.654156e-03, 0, k254_256, {-3.654076e-03, 1.884080, -9.805583e-01, 1.430580e-01}, {1}},
    {MACT_FN_ATAN_SQRT3, 4, 0, 1.286371e-03, 0, k254_256, {-1.286369e-03, 1.796716, -4.958969e-01, -6.927404e-01, 4.421541e-01}, {1}},
    {MACT_FN_ATAN_SQRT3, 5, 0, 1.801311e-04, 0, k254_256, {-1.801283e-04, 1.739333, -2.039848e-02, -2.065512, 2.052837, -6.591729e-01}, {1}},
    // Table 4: 2 arcsin(y / sqrt 2) on [0, 1/sqrt 2]
    {MACT_FN_ASIN2, 4, 0, 2.097814e-05, 0, kInvSqrt2, {2.097797e-05, 1.412840, 1.429881e-02, 6.704361e-02, 6.909677e-02}, {1}},
    {MACT_FN_ASIN2, 5, 0, 2.370540e-06, 0, kInvSqrt2, {-2.370048e-06, 1.414434, -3.300037e-03, 1.354670e-01, -3.994259e-02, 6.099502e-02}, {1}},
    // Table 5: arccos on [0, 0.5]
    {MACT_FN_ACOS, 4, 0, 1.048949e-05, 0, 0.5, {1.570786, -9.990285e-01, -1.429899e-02, -9.481335e-02, -1.381942e-01}, {1}},
    {MACT_FN_ACOS, 5, 0, 1.186403e-06, 0, 0.5, {1.570798, -1.000156, 3.299810e-03, -1.915780e-01, 7.988231e-02, -1.725177e-01}, {1}},
    // Table 6: arctan on [0, 254/255]
    {MACT_FN_ATAN, 4, 0, 1.036515e-04, 0, 254.0 / 255.0, {-1.036508e-04, 1.003740, -1.773538e-02, -3.390563e-01, 1.386796e-01}, {1}},
    {MACT_FN_ATAN, 5, 0, 2.073939e-05, 0, 254.0 / 255.0, {2.073866e-05, 9.982666e-01, 2.352573e-02, -4.506862e-01, 2.635050e-01, -4.920822e-02}, {1}},
    // Table 7: pi/2 - arctan(t) on [1/255, 1]
    {MACT_FN_ATANC, 4, 0, 1.051643e-04, 1.0 / 255.0, 1, {1.570917, -1.004004, 1.885694e-02, 3.373159e-01, -1.377930e-01}, {1}},
    {MACT_FN_ATANC, 5, 0, 2.012104e-05, 1.0 / 255.0, 1, {1.570769, -9.981253e-01, -2.440212e-02, 4.528921e-01, -2.659181e-01, 5.016228e-02}, {1}},
};

struct Default {
  int fn, n, m;
  double lo, hi;
};
const Default kDefaults[MACT_FN_COUNT] = {
    {MACT_FN_CBRT, 4, 4, kLabT0, 1.0},     {MACT_FN_ATAN_SQRT3, 5, 0, 0.0, 1.0},
    {MACT_FN_ASIN2, 5, 0, 0.0, kInvSqrt2}, {MACT_FN_ACOS, 5, 0, 0.0, 0.5},
    {MACT_FN_ATAN, 5, 0, 0.0, 1.0},        {MACT_FN_ATANC, 5, 0, 0.0, 1.0},
    {MACT_FN_SIN, 7, 0, 0.0, kPi / 2},     {MACT_FN_COS, 7, 0, 0.0, kPi / 2},
    {MACT_FN_ENC709, 4, 4, 0.018, 1.0},    {MACT_FN_DEC709, 7, 0, 0.081, 1.0},
};

std::once_flag g_default_once[MACT_FN_COUNT];
mact_approx g_default[MACT_FN_COUNT];
mact_status g_default_status[MACT_FN_COUNT];
}  // namespace

}  // namespace mact

using namespace mact;

extern "C" const char* mact_status_str(mact_status s) {
  switch (s) {
    case MACT_OK: return "ok";
    case MACT_E_INVALID: return "invalid argument";
    case MACT_E_NOCONV: return "fit did not converge";
    case MACT_E_DEVICE: return "HIP runtime error";
    case MACT_E_NOMEM: return "out of memory";
    case MACT_E_UNSUPPORTED: return "unsupported combination";
    case MACT_E_BUSY: return "busy";
    case MACT_E_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

extern "C" const char* mact_last_error(void) { return g_err; }

extern "C" const char* mact_version(void) { return "libmact 0.1 (gfx950)"; }

extern "C" mact_status mact_paper_approx(int32_t fn, int32_t n, int32_t m, mact_approx* out) {
  clear_error();
  if (!out) return fail(MACT_E_INVALID, "mact_paper_approx: out is NULL");
  for (const Row& r : kRows) {
    if (r.fn == fn && r.n == n && r.m == m) {
      std::memset(out, 0, sizeof *out);
      out->fn = fn;
      out->n = n;
      out->m = m;
      out->lo = r.lo;
      out->hi = r.hi;
      out->eps = r.eps;
      for (int k = 0; k <= n; ++k) out->p[k] = r.p[k];
      for (int k = 0; k <= m; ++k) out->q[k] = r.q[k];
      out->converged = 1;
      return MACT_OK;
    }
  }
  return fail(MACT_E_INVALID, "mact_paper_approx: the paper prints no row fn=%d n=%d m=%d", fn, n, m);
}

extern "C" mact_status mact_default_approx(int32_t fn, mact_approx* out) {
  clear_error();
  if (!out) return fail(MACT_E_INVALID, "mact_default_approx: out is NULL");
  if (fn < 0 || fn >= MACT_FN_COUNT) return fail(MACT_E_INVALID, "mact_default_approx: unknown function %d", fn);
  std::call_once(g_default_once[fn], [fn] {
    const Default& d = kDefaults[fn];
    g_default_status[fn] = mact_fit(d.fn, d.n, d.m, d.lo, d.hi, &g_default[fn]);
  });
  *out = g_default[fn];
  if (g_default_status[fn] != MACT_OK)
    return fail(g_default_status[fn], "mact_default_approx: default fit of function %d failed", fn);
  return MACT_OK;
}

extern "C" mact_status mact_params_default(int32_t xform, mact_params* p) {
  clear_error();
  if (!p) return fail(MACT_E_INVALID, "mact_params_default: p is NULL");
  if (xform < MACT_LAB || xform > MACT_LUV) return fail(MACT_E_INVALID, "unknown transform %d", xform);
  std::memset(p, 0, sizeof *p);
  p->xform = xform;
  static const int fns[4][4] = {{MACT_FN_CBRT}, {MACT_FN_ATAN_SQRT3}, {MACT_FN_ASIN2, MACT_FN_ACOS, MACT_FN_ATAN, MACT_FN_ATANC},
                                {MACT_FN_CBRT}};
  const int nf = xform == MACT_SCT ? 4 : 1;
  for (int i = 0; i < nf; ++i) {
    mact_status s = mact_default_approx(fns[xform][i], &p->f[i]);
    if (s != MACT_OK) return s;
  }
  return MACT_OK;
}
