/* Scalar FP64 oracle in plain C (test infrastructure only: the tests and the
 * benchmark's CPU baseline load it; the library never does).
 *
 * The same definitions as the numpy oracle, one pixel at a time, in double:
 *   - the exact RGB -> CIELAB transform of Sec. 3.2.1 (BT.709 inverse gamma,
 *     the BT.709 RGB -> XYZ matrix, the D65 white, f(t) = cube root above
 *     0.008856 and 7.787 t + 16/116 at or below it, then L*, a*, b*);
 *   - the MACT evaluation of Sec. 3.2.2: the same steps with the cube root
 *     replaced by a rational p(t)/q(t) given by its coefficients (Horner);
 *   - the packed N^3 CIELAB LUT of Sec. 3.5.3 (node (i, j, k) = the exact
 *     transform of (i, j, k)/(N - 1)) and its tetrahedral interpolation:
 *     the fractions in decreasing order f1 >= f2 >= f3 (ties R before G
 *     before B), the walk from corner 000 along the axes in that order, with
 *     weights 1 - f1, f1 - f2, f2 - f3, f3.
 * Every entry point takes a range of 8-bit RGB pixels (v enters as v/255) so
 * that a caller can spread a batch over threads.  Build:
 *   gcc -O2 -shared -fPIC -o liboracle_c.so cbase.c -lm   (no -ffast-math)
 */
#include <math.h>
#include <stdint.h>

/* ITU-R BT.709 primaries, linear RGB -> CIEXYZ (Sec. 3.2.1). */
static const double kM[3][3] = {{0.412391, 0.357584, 0.180481},
                                {0.212639, 0.715169, 0.072192},
                                {0.019331, 0.119195, 0.950532}};
/* D65 reference white (Sec. 3.2.1). */
static const double kW[3] = {0.950456, 1.0, 1.089058};

/* BT.709 inverse gamma: k/4.5 below 0.081, else ((k + 0.099)/1.099)^(1/0.45). */
static double decode709(double k) { return k < 0.081 ? k / 4.5 : pow((k + 0.099) / 1.099, 1.0 / 0.45); }

static double f_exact(double t) { return t > 0.008856 ? cbrt(t) : 7.787 * t + 16.0 / 116.0; }

static double horner(const double* c, int32_t n, double x) {
  double a = c[n];
  for (int32_t k = n - 1; k >= 0; --k) a = a * x + c[k];
  return a;
}

/* t = (X/X0, Y/Y0, Z/Z0) of one encoded pixel. */
static void lab_t(double r, double g, double b, double t[3]) {
  const double lin[3] = {decode709(r), decode709(g), decode709(b)};
  for (int c = 0; c < 3; ++c) t[c] = (kM[c][0] * lin[0] + kM[c][1] * lin[1] + kM[c][2] * lin[2]) / kW[c];
}

static void lab_from_f(const double f[3], double* out) {
  out[0] = 116.0 * f[1] - 16.0;
  out[1] = 500.0 * (f[0] - f[1]);
  out[2] = 200.0 * (f[1] - f[2]);
}

static void lab_exact(double r, double g, double b, double* out) {
  double t[3], f[3];
  lab_t(r, g, b, t);
  for (int c = 0; c < 3; ++c) f[c] = f_exact(t[c]);
  lab_from_f(f, out);
}

/* Pixels [begin, end) of `rgb` (packed 8-bit R, G, B) -> exact L*a*b* in out[3 i ..]. */
void oc_lab_exact_u8(const uint8_t* rgb, int64_t begin, int64_t end, double* out) {
  for (int64_t i = begin; i < end; ++i)
    lab_exact(rgb[3 * i] / 255.0, rgb[3 * i + 1] / 255.0, rgb[3 * i + 2] / 255.0, out + 3 * i);
}

/* The same with f = p/q (degrees np, nq) above 0.008856: the MACT transform. */
void oc_lab_mact_u8(const uint8_t* rgb, int64_t begin, int64_t end, const double* p, int32_t np, const double* q,
                    int32_t nq, double* out) {
  for (int64_t i = begin; i < end; ++i) {
    double t[3], f[3];
    lab_t(rgb[3 * i] / 255.0, rgb[3 * i + 1] / 255.0, rgb[3 * i + 2] / 255.0, t);
    for (int c = 0; c < 3; ++c)
      f[c] = t[c] > 0.008856 ? horner(p, np, t[c]) / horner(q, nq, t[c]) : 7.787 * t[c] + 16.0 / 116.0;
    lab_from_f(f, out + 3 * i);
  }
}

/* Packed CIELAB LUT: node (i, j, k) at ((i N + j) N + k) * 3, the exact transform of (i, j, k)/(N - 1). */
void oc_lut_build_lab(int32_t N, double* lut) {
  for (int32_t i = 0; i < N; ++i)
    for (int32_t j = 0; j < N; ++j)
      for (int32_t k = 0; k < N; ++k)
        lab_exact((double)i / (N - 1), (double)j / (N - 1), (double)k / (N - 1), lut + 3 * (((int64_t)i * N + j) * N + k));
}

/* Cell and fraction of an 8-bit value: pos = v (N - 1)/255, cell min(floor(pos), N - 2). */
static void locate_u8(int32_t v, int32_t N, int32_t* i, double* f) {
  const int32_t num = v * (N - 1);
  *i = num / 255 < N - 2 ? num / 255 : N - 2;
  *f = (num - 255 * *i) / 255.0;
}

/* Tetrahedral interpolation of pixels [begin, end) in the packed LUT of size N. */
void oc_lut_tetra_u8(const double* lut, int32_t N, const uint8_t* rgb, int64_t begin, int64_t end, double* out) {
  const int64_t sR = (int64_t)N * N * 3, sG = (int64_t)N * 3, sB = 3;
  for (int64_t p = begin; p < end; ++p) {
    int32_t i[3];
    double f[3];
    for (int c = 0; c < 3; ++c) locate_u8(rgb[3 * p + c], N, &i[c], &f[c]);
    /* axes in decreasing order of their fractions, ties R before G before B */
    int a[3] = {0, 1, 2};
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 2 - x; ++y)
        if (f[a[y + 1]] > f[a[y]]) {
          const int s = a[y];
          a[y] = a[y + 1];
          a[y + 1] = s;
        }
    const int64_t step[3] = {sR, sG, sB};
    const double w[4] = {1.0 - f[a[0]], f[a[0]] - f[a[1]], f[a[1]] - f[a[2]], f[a[2]]};
    int64_t at = i[0] * sR + i[1] * sG + i[2] * sB;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < 4; ++s) {
      if (s > 0) at += step[a[s - 1]];
      for (int c = 0; c < 3; ++c) acc[c] += w[s] * lut[at + c];
    }
    out[3 * p] = acc[0];
    out[3 * p + 1] = acc[1];
    out[3 * p + 2] = acc[2];
  }
}
