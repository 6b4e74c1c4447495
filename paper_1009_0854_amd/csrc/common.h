// Internal helpers shared by the host sources of libmact: error reporting and
// the paper's colour constants in double precision.
#pragma once

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/mact.h"

namespace mact {

// Thread-local detail of the last failure; mact_last_error() returns it.
void set_error(const char* fmt, ...);
void clear_error();

inline mact_status fail(mact_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_error("%s", buf);
  return s;
}

// ITU-R BT.709 linear RGB -> CIEXYZ (Sec. 3.2.1) and the D65 white.
constexpr double kM[3][3] = {{0.412391, 0.357584, 0.180481},
                             {0.212639, 0.715169, 0.072192},
                             {0.019331, 0.119195, 0.950532}};
constexpr double kWhite[3] = {0.950456, 1.0, 1.089058};
constexpr double kLabT0 = 0.008856;  // breakpoint of the CIELAB nonlinearity
constexpr double kLabK = 7.787;      // slope of its linear segment
constexpr double kLabC = 16.0 / 116.0;
constexpr double kPi = 3.14159265358979323846;

// Transforms whose input goes through the transfer function (LAB, LUV).
inline bool uses_gamma(int xform) { return xform == MACT_LAB || xform == MACT_LUV; }

// Host FP64 exact transforms (used to pack LUTs).  rgb in [0, 1].
double inverse_gamma(double k, int gamma);
void exact_lab(const double rgb[3], int gamma, double out[3]);
void exact_hsi(const double rgb[3], double out[3]);
void exact_sct(const double rgb[3], double out[3]);
void exact_luv(const double rgb[3], int gamma, double out[3]);

// Validation shared by the entry points.
mact_status check_approx(const mact_approx& a, bool rational_ok, const char* what);
mact_status check_params(const mact_params* p);

}  // namespace mact
