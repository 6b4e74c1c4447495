// Per-pixel MACT arithmetic and pixel addressing, shared by every kernel of
// libmact (plain, batched, served).  One definition of the arithmetic is what
// makes the three forms bitwise identical: every multiply-add that matters is
// an explicit fmaf and the sources are compiled with -ffp-contract=off.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mact {

// ---------------------------------------------------------------- constants

// diag(1/white) * M, rounded once from the double values (Sec. 3.2.1).
#define MW(r, c) static_cast<float>(kM[r][c] / kWhite[r])
constexpr float kMw00 = MW(0, 0), kMw01 = MW(0, 1), kMw02 = MW(0, 2);
constexpr float kMw10 = MW(1, 0), kMw11 = MW(1, 1), kMw12 = MW(1, 2);
constexpr float kMw20 = MW(2, 0), kMw21 = MW(2, 1), kMw22 = MW(2, 2);
#undef MW
constexpr float kT0f = static_cast<float>(kLabT0);
constexpr float kLabKf = static_cast<float>(kLabK);
constexpr float kLabCf = static_cast<float>(kLabC);
constexpr float kPi3f = static_cast<float>(kPi / 3.0);
constexpr float kPif = static_cast<float>(kPi);
constexpr float k5Pi3f = static_cast<float>(5.0 * kPi / 3.0);
constexpr float kPi2f = static_cast<float>(kPi / 2.0);
constexpr float kTwoPif = static_cast<float>(2.0 * kPi);
constexpr float kInv255 = static_cast<float>(1.0 / 255.0);
constexpr float kInv765 = static_cast<float>(1.0 / 765.0);
constexpr float kInv3 = static_cast<float>(1.0 / 3.0);
constexpr float kInv65535 = static_cast<float>(1.0 / 65535.0);
constexpr float kInv196605 = static_cast<float>(1.0 / 196605.0);  // 1 / (3 * 65535)
// BT.709 matrix rows (linear RGB -> XYZ) and the white's u', v' for CIELUV.
#define MF(r, c) static_cast<float>(kM[r][c])
constexpr float kM00 = MF(0, 0), kM01 = MF(0, 1), kM02 = MF(0, 2);
constexpr float kM10 = MF(1, 0), kM11 = MF(1, 1), kM12 = MF(1, 2);
constexpr float kM20 = MF(2, 0), kM21 = MF(2, 1), kM22 = MF(2, 2);
#undef MF
constexpr double kDn = kWhite[0] + 15.0 * kWhite[1] + 3.0 * kWhite[2];
constexpr float kUn = static_cast<float>(4.0 * kWhite[0] / kDn);
constexpr float kVn = static_cast<float>(9.0 * kWhite[1] / kDn);

// ---------------------------------------------------------------- parameters

// Coefficients of one transform, float32, zero-padded to degree 7.  Horner's
// rule over zero leading coefficients is exact, so evaluating at a padded
// degree gives the same bits as at the true degree.
struct KCoef {
  float p[4][8];  // numerators of f[0..3]; LAB with `decode`: p[1] is the BT.709 decoding polynomial
  float q[8];     // denominator of f[0] (LAB); {1, 0, ...} otherwise
  int32_t xform, out_mode;
  int32_t decode;  // LAB: float inputs decode BT.709 with the polynomial p[1] (degree <= 7)
  float lab_c;     // 16/116, the linear segment's offset (CIELAB, CIELUV), as a value pin_lead can place
};

// n / d for 32-bit n and a fixed d >= 1: q = (umulhi(n, m) + n) >> s with the
// round-up multiplier m = floor(2^32 (2^s - d) / d) + 1, 2^s >= d (exact for
// every 32-bit n; the sum is formed in 64 bits).
struct FastDiv {
  uint32_t d, m, s;
  __device__ __forceinline__ uint32_t div(uint32_t n) const {
    return (uint32_t)(((uint64_t)__umulhi(n, m) + n) >> s);
  }
};

// One image as the kernels see it.  Pixel index p in [0, N H W) of one launch
// is 32-bit; the host splits larger launches.
struct KImage {
  void* ptr;
  int32_t dtype, layout;
  int64_t rs, ps, bs;  // row, plane, batch strides in elements (resolved)
  uint32_t W, HW;      // width, pixels per image
  uint32_t packed;     // HWC: element (p, c) at 3 p + c;  CHW: batch and planes packed
  FastDiv div_w, div_hw;
};

// ---------------------------------------------------------------- polynomial

// Moves the leading coefficient of every polynomial, and the linear segment's
// offset, into vector registers once per kernel.  A vector instruction may read
// one scalar register or literal, so the first Horner step,
// fma(c[DEG], x, c[DEG-1]), and the segment fma(7.787, t, 16/116) would
// otherwise each need a copy at every evaluation.  Values are unchanged.
template <int DEG>
__device__ __forceinline__ void pin_lead(KCoef& k) {
#pragma unroll
  for (int i = 0; i < 4; ++i) asm volatile("" : "+v"(k.p[i][DEG]));
  asm volatile("" : "+v"(k.q[DEG]));
  asm volatile("" : "+v"(k.lab_c));
}

template <int DEG>
__device__ __forceinline__ float horner(const float* c, float x) {
  float acc = c[DEG];
#pragma unroll
  for (int k = DEG - 1; k >= 0; --k) acc = __builtin_fmaf(acc, x, c[k]);
  return acc;
}

// a / b through the hardware reciprocal (about one ulp) and one multiply.
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Square root through the hardware instruction (about one ulp; the correctly
// rounded library form costs about 16 instructions).  SMALL: the argument may
// lie below 2^-96 (tiny float32 inputs), where it is scaled by 2^64 first and
// the root by 2^-32, both exact; above 2^-96 both forms give the same bits.
template <bool SMALL>
__device__ __forceinline__ float fsqrt(float x) {
  if (!SMALL) return __builtin_amdgcn_sqrtf(x);
  const bool tiny = x < 0x1p-96f;
  const float r = __builtin_amdgcn_sqrtf(tiny ? x * 0x1p64f : x);
  return tiny ? r * 0x1p-32f : r;
}

// ---------------------------------------------------------------- transforms

// Linear RGB -> the three approximated nonlinearity values (Sec. 3.2).
template <int DEG>
__device__ __forceinline__ void lab_f3(const KCoef& k, float lr, float lg, float lb, float f[3]) {
  const float t[3] = {
      __builtin_fmaf(kMw00, lr, __builtin_fmaf(kMw01, lg, kMw02 * lb)),
      __builtin_fmaf(kMw10, lr, __builtin_fmaf(kMw11, lg, kMw12 * lb)),
      __builtin_fmaf(kMw20, lr, __builtin_fmaf(kMw21, lg, kMw22 * lb)),
  };
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (t[c] > kT0f)
      f[c] = fdiv(horner<DEG>(k.p[0], t[c]), horner<DEG>(k.q, t[c]));
    else
      f[c] = __builtin_fmaf(kLabKf, t[c], k.lab_c);
  }
}

template <int DEG>
__device__ __forceinline__ void lab_px(const KCoef& k, float lr, float lg, float lb, float o[3]) {
  float f[3];
  lab_f3<DEG>(k, lr, lg, lb, f);
  if (k.out_mode == 1) {
    o[0] = f[0];
    o[1] = f[1];
    o[2] = f[2];
    return;
  }
  o[0] = __builtin_fmaf(116.0f, f[1], -16.0f);
  o[1] = 500.0f * (f[0] - f[1]);
  o[2] = 200.0f * (f[1] - f[2]);
}

// CIE 1976 L*u*v* (the extension named in Sec. 4): L* from the same
// approximated nonlinearity as CIELAB's (Y / Yn with Yn = 1), u' = 4X / D,
// v' = 9Y / D with D = X + 15Y + 3Z through one reciprocal; black (D = 0)
// gives u* = v* = 0.
template <int DEG>
__device__ __forceinline__ void luv_px(const KCoef& k, float lr, float lg, float lb, float o[3]) {
  const float X = __builtin_fmaf(kM00, lr, __builtin_fmaf(kM01, lg, kM02 * lb));
  const float Y = __builtin_fmaf(kM10, lr, __builtin_fmaf(kM11, lg, kM12 * lb));
  const float Z = __builtin_fmaf(kM20, lr, __builtin_fmaf(kM21, lg, kM22 * lb));
  const float fy = Y > kT0f ? fdiv(horner<DEG>(k.p[0], Y), horner<DEG>(k.q, Y)) : __builtin_fmaf(kLabKf, Y, k.lab_c);
  const float L = __builtin_fmaf(116.0f, fy, -16.0f);
  const float D = __builtin_fmaf(15.0f, Y, __builtin_fmaf(3.0f, Z, X));
  if (!(D > 0.0f)) {
    o[0] = L; o[1] = 0.0f; o[2] = 0.0f;
    return;
  }
  const float rD = __builtin_amdgcn_rcpf(D);
  const float L13 = 13.0f * L;
  o[0] = L;
  o[1] = L13 * __builtin_fmaf(4.0f * X, rD, -kUn);
  o[2] = L13 * __builtin_fmaf(9.0f * Y, rD, -kVn);
}

// HSI by Kender's branches with the arctan(sqrt 3 x) polynomial (Sec. 3.3).
// R, G, B on any common scale; `iscale` maps (R+G+B) to I.
template <int DEG>
__device__ __forceinline__ void hsi_px(const KCoef& k, float R, float G, float B, float iscale, float o[3]) {
  float num, den, base;
  bool act = true;
  if (R > B && G > B) {
    num = G - R; den = (G - B) + (R - B); base = kPi3f;
  } else if (G > R) {
    num = B - G; den = (B - R) + (G - R); base = kPif;
  } else if (B > G) {
    num = R - B; den = (R - G) + (B - G); base = k5Pi3f;
  } else {
    num = 0.0f; den = 1.0f; base = 0.0f; act = false;
  }
  float H = 0.0f;
  if (act) {
    const float x = fdiv(num, den);
    const float v = horner<DEG>(k.p[0], __builtin_fabsf(x));
    H = base + (x < 0.0f ? -v : v);
  }
  const float sum = (R + G) + B;
  const float mn = __builtin_fminf(R, __builtin_fminf(G, B));
  o[0] = H;
  o[1] = sum > 0.0f ? 1.0f - fdiv(3.0f * mn, sum) : 0.0f;
  o[2] = sum * iscale;
}

// SCT with the arcsin/arccos/arctan polynomials (Sec. 3.4).  R, G, B on any
// common scale; `lscale` maps the norm to L on the [0, 1] input scale.  SMALL
// = false where neither square-root argument can fall below 2^-96: 8- and
// 16-bit codes on their integer scales, float16 values.
template <int DEG, bool SMALL = true>
__device__ __forceinline__ void sct_px(const KCoef& k, float R, float G, float B, float lscale, float o[3]) {
  const float rg2 = __builtin_fmaf(R, R, G * G);
  const float L2 = __builtin_fmaf(B, B, rg2);
  if (!(L2 > 0.0f)) {
    o[0] = 0.0f; o[1] = 0.0f; o[2] = 0.0f;
    return;
  }
  const float L = fsqrt<SMALL>(L2);
  float A;
  if (3.0f * (B * B) >= rg2) {  // B/L >= 0.5: arccos(B/L) = 2 arcsin(sqrt(1 - B/L) / sqrt 2)
    const float y = fsqrt<SMALL>(fdiv(rg2, L * (L + B)));
    A = horner<DEG>(k.p[0], y);
  } else {
    A = horner<DEG>(k.p[1], fdiv(B, L));
  }
  float Bang;
  if (G < R) Bang = horner<DEG>(k.p[2], fdiv(G, R));
  else if (R > 0.0f) Bang = horner<DEG>(k.p[3], fdiv(R, G));
  else if (G > 0.0f) Bang = kPi2f;
  else Bang = 0.0f;
  o[0] = L * lscale;
  o[1] = A;
  o[2] = Bang;
}

// ---------------------------------------------------------------- inputs

__device__ __forceinline__ float clamp01(float v) { return __builtin_fminf(__builtin_fmaxf(v, 0.0f), 1.0f); }

// Inverse transfer function of a float input already clamped to [0, 1].  BT.709
// above 0.081: the exact power, or (k.decode) its minimax polynomial p[1].
__device__ __forceinline__ float lin_float(const KCoef& k, float v, int gamma) {
  if (gamma == MACT_GAMMA_BT709) {
    if (v < 0.081f) return v / 4.5f;
    return k.decode ? horner<7>(k.p[1], v) : __builtin_powf((v + 0.099f) / 1.099f, 1.0f / 0.45f);
  }
  if (gamma == MACT_GAMMA_SRGB) return v <= 0.04045f ? v / 12.92f : __builtin_powf((v + 0.055f) / 1.055f, 2.4f);
  return v;
}

// Offset (elements) of channel c of pixel p in an image.
__device__ __forceinline__ int64_t elem_off(const KImage& im, uint32_t p, int c) {
  if (im.packed) {
    if (im.layout == MACT_HWC) return 3 * (int64_t)p + c;
    const uint32_t n = im.div_hw.div(p);
    return (int64_t)n * im.bs + (int64_t)c * im.ps + (p - n * im.HW);
  }
  const uint32_t n = im.div_hw.div(p);
  const uint32_t r = p - n * im.HW;
  const uint32_t y = im.div_w.div(r);
  const uint32_t x = r - y * im.W;
  if (im.layout == MACT_HWC) return (int64_t)n * im.bs + (int64_t)y * im.rs + 3 * (int64_t)x + c;
  return (int64_t)n * im.bs + (int64_t)c * im.ps + (int64_t)y * im.rs + x;
}

// Raw pixel: 8- and 16-bit codes as integer-valued floats (exact), float
// inputs clamped to [0, 1].
__device__ __forceinline__ void load_px(const KImage& im, uint32_t p, float v[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t o = elem_off(im, p, c);
    if (im.dtype == MACT_U8) v[c] = (float)static_cast<const uint8_t*>(im.ptr)[o];
    else if (im.dtype == MACT_U16) v[c] = (float)static_cast<const uint16_t*>(im.ptr)[o];
    else if (im.dtype == MACT_F16) v[c] = clamp01(__half2float(static_cast<const __half*>(im.ptr)[o]));
    else v[c] = clamp01(static_cast<const float*>(im.ptr)[o]);
  }
}

// float32 -> float16 of the float32 value, rounded to nearest even.  The
// empty asm pins x as a float32 register value: without it the compiler may
// fuse the conversion with the fma that produced x into one mixed-precision
// instruction, which rounds the exact product-sum once, straight to float16,
// and can differ in the last bit.
__device__ __forceinline__ __half f2h_rn(float x) {
  asm volatile("" : "+v"(x));
  return __float2half_rn(x);
}

// Two float32 values -> two float16, each rounded to nearest even (the bits of
// f2h_rn), packed in one word with `a` in the low half: one packed conversion.
__device__ __forceinline__ uint32_t pack2_h_rn(float a, float b) {
  asm volatile("" : "+v"(a));
  asm volatile("" : "+v"(b));
  const __half2 h = __floats2half2_rn(a, b);
  return __builtin_bit_cast(uint32_t, h);
}

__device__ __forceinline__ void store_px(const KImage& im, uint32_t p, const float o3[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t o = elem_off(im, p, c);
    if (im.dtype == MACT_F16) static_cast<__half*>(im.ptr)[o] = f2h_rn(o3[c]);
    else static_cast<float*>(im.ptr)[o] = o3[c];
  }
}

// One pixel of any transform from its raw value (as load_px returns it) of
// element type `dtype`.  `gtab` is the 256-entry inverse gamma of the image's
// transfer function (8-bit inputs); 16-bit codes are normalised to [0, 1] and
// decoded like float inputs.  HSI and SCT are scale-free and take the codes.
template <int DEG>
__device__ __forceinline__ void eval_px(const KCoef& k, int dtype, int gamma, const float* gtab, const float v[3],
                                        float o[3]) {
  if (k.xform == MACT_LAB || k.xform == MACT_LUV) {
    float l[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      l[c] = dtype == MACT_U8 ? gtab[(int)v[c]] : lin_float(k, dtype == MACT_U16 ? v[c] * kInv65535 : v[c], gamma);
    if (k.xform == MACT_LAB) lab_px<DEG>(k, l[0], l[1], l[2], o);
    else luv_px<DEG>(k, l[0], l[1], l[2], o);
  } else if (k.xform == MACT_HSI) {
    hsi_px<DEG>(k, v[0], v[1], v[2], dtype == MACT_U8 ? kInv765 : dtype == MACT_U16 ? kInv196605 : kInv3, o);
  } else {
    sct_px<DEG>(k, v[0], v[1], v[2], dtype == MACT_U8 ? kInv255 : dtype == MACT_U16 ? kInv65535 : 1.0f, o);
  }
}

// eval_px with the element type and the transform fixed at compile time: the
// same arithmetic, so the same bits.
template <int IN, int XF, int DEG>
__device__ __forceinline__ void px1(const KCoef& k, int gamma, const float* gtab, const float v[3], float o[3]) {
  if (XF == MACT_LAB || XF == MACT_LUV) {
    float l[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      l[c] = IN == MACT_U8 ? gtab[(int)v[c]] : lin_float(k, IN == MACT_U16 ? v[c] * kInv65535 : v[c], gamma);
    if (XF == MACT_LAB) lab_px<DEG>(k, l[0], l[1], l[2], o);
    else luv_px<DEG>(k, l[0], l[1], l[2], o);
  } else if (XF == MACT_HSI) {
    hsi_px<DEG>(k, v[0], v[1], v[2], IN == MACT_U8 ? kInv765 : IN == MACT_U16 ? kInv196605 : kInv3, o);
  } else {
    sct_px<DEG, IN == MACT_F32>(k, v[0], v[1], v[2], IN == MACT_U8 ? kInv255 : IN == MACT_U16 ? kInv65535 : 1.0f, o);
  }
}

// ---------------------------------------------------------------- 4-pixel groups

// Byte i (0..11) of 12 bytes held as one 12-byte word.
__device__ __forceinline__ uint32_t byte_of(uint3 w, int i) {
  const uint32_t word = i < 4 ? w.x : (i < 8 ? w.y : w.z);
  return (word >> (8 * (i & 3))) & 0xffu;
}

// Half i (0..11) of 24 bytes held as two 12-byte words.
__device__ __forceinline__ float half_of(uint3 a, uint3 b, int i) {
  const uint3 w = i < 6 ? a : b;
  const int j = i < 6 ? i : i - 6;
  const uint32_t word = j < 2 ? w.x : (j < 4 ? w.y : w.z);
  const uint16_t bits = (uint16_t)(word >> (16 * (j & 1)));
  return clamp01(__half2float(__ushort_as_half(bits)));
}

template <int XF, int DEG>
__device__ __forceinline__ void px4_u8(const KCoef& k, const float* gtab, uint3 w, float o[12]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t r = byte_of(w, 3 * j), g = byte_of(w, 3 * j + 1), b = byte_of(w, 3 * j + 2);
    if (XF == MACT_LAB) lab_px<DEG>(k, gtab[r], gtab[g], gtab[b], o + 3 * j);
    else if (XF == MACT_LUV) luv_px<DEG>(k, gtab[r], gtab[g], gtab[b], o + 3 * j);
    else if (XF == MACT_HSI) hsi_px<DEG>(k, (float)r, (float)g, (float)b, kInv765, o + 3 * j);
    else sct_px<DEG, false>(k, (float)r, (float)g, (float)b, kInv255, o + 3 * j);
  }
}

// Code i (0..11) of 24 bytes held as two 12-byte words (16-bit input), as a float.
__device__ __forceinline__ float code16_of(uint3 a, uint3 b, int i) {
  const uint3 w = i < 6 ? a : b;
  const int j = i < 6 ? i : i - 6;
  const uint32_t word = j < 2 ? w.x : (j < 4 ? w.y : w.z);
  return (float)((word >> (16 * (j & 1))) & 0xffffu);
}

// The same 4 pixels from 16-bit codes: eval_px's arithmetic for MACT_U16.
template <int XF, int DEG>
__device__ __forceinline__ void px4_u16(const KCoef& k, int gamma, uint3 wa, uint3 wb, float o[12]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float r = code16_of(wa, wb, 3 * j), g = code16_of(wa, wb, 3 * j + 1), b = code16_of(wa, wb, 3 * j + 2);
    if (XF == MACT_LAB || XF == MACT_LUV) {
      const float lr = lin_float(k, r * kInv65535, gamma), lg = lin_float(k, g * kInv65535, gamma),
                  lb = lin_float(k, b * kInv65535, gamma);
      if (XF == MACT_LAB) lab_px<DEG>(k, lr, lg, lb, o + 3 * j);
      else luv_px<DEG>(k, lr, lg, lb, o + 3 * j);
    } else if (XF == MACT_HSI) {
      hsi_px<DEG>(k, r, g, b, kInv196605, o + 3 * j);
    } else {
      sct_px<DEG, false>(k, r, g, b, kInv65535, o + 3 * j);
    }
  }
}

// The same 4 pixels from float16 input: eval_px's arithmetic for float inputs.
template <int XF, int DEG>
__device__ __forceinline__ void px4_f16(const KCoef& k, int gamma, uint3 wa, uint3 wb, float o[12]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float r = half_of(wa, wb, 3 * j), g = half_of(wa, wb, 3 * j + 1), b = half_of(wa, wb, 3 * j + 2);
    if (XF == MACT_LAB) lab_px<DEG>(k, lin_float(k, r, gamma), lin_float(k, g, gamma), lin_float(k, b, gamma), o + 3 * j);
    else if (XF == MACT_LUV) luv_px<DEG>(k, lin_float(k, r, gamma), lin_float(k, g, gamma), lin_float(k, b, gamma), o + 3 * j);
    else if (XF == MACT_HSI) hsi_px<DEG>(k, r, g, b, kInv3, o + 3 * j);
    else sct_px<DEG, false>(k, r, g, b, 1.0f, o + 3 * j);
  }
}

}  // namespace mact
