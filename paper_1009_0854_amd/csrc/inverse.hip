// Inverse transforms (CIELAB, HSI, SCT, CIELUV -> RGB) with minimax
// approximations, and on-device error statistics of the forward transforms.
//
// Inverses: the definitions of Sec. 3.2.1 and 3.3.1 solved for R, G, B, the
// SCT inverse of Sec. 3.4.1, and the CIE 1976 L*u*v* definition (the extension
// named in Sec. 4) solved for X, Y, Z, with the elementary functions replaced by
// minimax approximations in the paper's manner: the BT.709 encoding power
// 1.099 L^0.45 - 0.099 by a rational on [0.018, 1] (the cube of the CIELAB and
// CIELUV inverses is exact), cosine by a polynomial on [0, 2 pi/3] (HSI), sine and
// cosine by polynomials on [0, pi/2] (SCT).  float32, explicit fmas; packed
// float32 HWC goes through LDS-staged coalesced chunks, packed CHW (float32,
// float16) 4 pixels per lane by planes, everything else one pixel per lane.
//
// Error statistics: every pixel of an RGB image goes through the forward MACT
// transform (the same per-pixel code as mact_transform, float32) and through
// the exact transform in float64; the paper's metric of the pair (Delta E*ab,
// D_HSI, or the SCT measure: both triples back to RGB, then to CIELAB, then
// Delta E*ab; Delta E*uv for CIELUV) is reduced to its mean and maximum, with
// the largest per-channel differences, in one pass.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "launch.h"
#include "planes.h"

namespace mact {

#include "gamma_table.inc"

namespace {

// M^-1 diag(white): t (= XYZ / white) -> linear RGB (CIELAB), or M^-1 alone:
// XYZ -> linear RGB (CIELUV); rounded once from double.
struct InvMat {
  float m[3][3];
};

InvMat make_inv_mat(bool fold_white) {
  // 3x3 inverse by cofactors, in double
  const double (*a)[3] = kM;
  const double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                     a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                     a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  double inv[3][3];
  inv[0][0] = (a[1][1] * a[2][2] - a[1][2] * a[2][1]) / det;
  inv[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) / det;
  inv[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) / det;
  inv[1][0] = (a[1][2] * a[2][0] - a[1][0] * a[2][2]) / det;
  inv[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) / det;
  inv[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) / det;
  inv[2][0] = (a[1][0] * a[2][1] - a[1][1] * a[2][0]) / det;
  inv[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) / det;
  inv[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) / det;
  InvMat r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[i][j] = (float)(fold_white ? inv[i][j] * kWhite[j] : inv[i][j]);
  return r;
}

constexpr float kEnc0 = 0.018f;  // BT.709 encoding breakpoint (0.081 / 4.5)
constexpr float kTwoPi3f = static_cast<float>(2.0 * kPi / 3.0);

// Raw float element (no clamping): inverse inputs are L*a*b*, HSI or SCT values.
__device__ __forceinline__ void load_raw(const KImage& im, uint32_t p, float v[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t o = elem_off(im, p, c);
    if (im.dtype == MACT_F16) v[c] = __half2float(static_cast<const __half*>(im.ptr)[o]);
    else v[c] = static_cast<const float*>(im.ptr)[o];
  }
}

template <int DEG>
__device__ __forceinline__ void lab_inv_px(const KCoef& k, const InvMat& mi, int gamma, const float v[3], float o[3]) {
  const float fy = (v[0] + 16.0f) * (1.0f / 116.0f);
  const float f[3] = {__builtin_fmaf(v[1], 1.0f / 500.0f, fy), fy, __builtin_fmaf(v[2], -1.0f / 200.0f, fy)};
  float t[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float cube = f[c] * f[c] * f[c];
    t[c] = cube > kT0f ? cube : (f[c] - kLabCf) * (1.0f / kLabKf);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float lin = clamp01(__builtin_fmaf(mi.m[c][0], t[0], __builtin_fmaf(mi.m[c][1], t[1], mi.m[c][2] * t[2])));
    if (gamma == MACT_GAMMA_NONE) o[c] = lin;
    else o[c] = lin >= kEnc0 ? fdiv(horner<DEG>(k.p[0], lin), horner<DEG>(k.q, lin)) : 4.5f * lin;
  }
}

// CIE 1976 L*u*v* -> R'G'B'.  Y from L* as in CIELAB (Y/Yn = t, Yn = 1); u', v'
// from u*, v* through one reciprocal of 13 L*; X = 9 u' q and Z = (12 - 3u' - 20v') q
// with q = Y / (4 v').  L* <= 0 is black.  Values off the image of the forward
// transform (v' <= 0) give unspecified results.
template <int DEG>
__device__ __forceinline__ void luv_inv_px(const KCoef& k, const InvMat& mi, int gamma, const float v[3], float o[3]) {
  float X = 0.0f, Y = 0.0f, Z = 0.0f;
  if (v[0] > 0.0f) {
    const float fy = (v[0] + 16.0f) * (1.0f / 116.0f);
    const float cube = fy * fy * fy;
    Y = cube > kT0f ? cube : (fy - kLabCf) * (1.0f / kLabKf);
    const float r13 = fdiv(1.0f, 13.0f * v[0]);
    const float up = __builtin_fmaf(v[1], r13, kUn);
    const float vp = __builtin_fmaf(v[2], r13, kVn);
    const float q = fdiv(Y, 4.0f * vp);
    X = 9.0f * up * q;
    Z = __builtin_fmaf(-3.0f, up, __builtin_fmaf(-20.0f, vp, 12.0f)) * q;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float lin = clamp01(__builtin_fmaf(mi.m[c][0], X, __builtin_fmaf(mi.m[c][1], Y, mi.m[c][2] * Z)));
    if (gamma == MACT_GAMMA_NONE) o[c] = lin;
    else o[c] = lin >= kEnc0 ? fdiv(horner<DEG>(k.p[0], lin), horner<DEG>(k.q, lin)) : 4.5f * lin;
  }
}

template <int DEG>
__device__ __forceinline__ void hsi_inv_px(const KCoef& k, const float v[3], float o[3]) {
  float H = v[0];
  if (H < 0.0f || H >= kTwoPif) H -= kTwoPif * floorf(H * (1.0f / kTwoPif));
  const float S = v[1], I = v[2];
  const int sector = H < kTwoPi3f ? 0 : (H < 2.0f * kTwoPi3f ? 1 : 2);
  const float h = H - (float)sector * kTwoPi3f;
  const float ratio = fdiv(horner<DEG>(k.p[0], h), horner<DEG>(k.p[0], __builtin_fabsf(kPi3f - h)));
  const float behind = I * (1.0f - S);
  const float start = I * __builtin_fmaf(S, ratio, 1.0f);
  const float third = 3.0f * I - (behind + start);
  if (sector == 0) { o[0] = start; o[1] = third; o[2] = behind; }
  else if (sector == 1) { o[0] = behind; o[1] = start; o[2] = third; }
  else { o[0] = third; o[1] = behind; o[2] = start; }
}

template <int DEG>
__device__ __forceinline__ void sct_inv_px(const KCoef& k, const float v[3], float o[3]) {
  const float L = v[0];
  const float sa = horner<DEG>(k.p[0], v[1]), ca = horner<DEG>(k.p[1], v[1]);
  const float sb = horner<DEG>(k.p[0], v[2]), cb = horner<DEG>(k.p[1], v[2]);
  const float ls = L * sa;
  o[0] = ls * cb;
  o[1] = ls * sb;
  o[2] = L * ca;
}

template <int DEG>
__global__ __launch_bounds__(256) void k_inverse(KImage src, KImage dst, uint32_t n_px, KCoef k, InvMat mi,
                                                 int gamma) {
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t p = blockIdx.x * 256u + threadIdx.x; p < n_px; p += stride) {
    float v[3], o[3];
    load_raw(src, p, v);
    if (k.xform == MACT_LAB) lab_inv_px<DEG>(k, mi, gamma, v, o);
    else if (k.xform == MACT_LUV) luv_inv_px<DEG>(k, mi, gamma, v, o);
    else if (k.xform == MACT_HSI) hsi_inv_px<DEG>(k, v, o);
    else sct_inv_px<DEG>(k, v, o);
    store_px(dst, p, o);
  }
}

// Packed float32 HWC in, packed float32 or float16 (OUT) HWC out, 16-byte
// aligned: each wave takes 256-pixel chunks (3 KB in; 3 KB or 1.5 KB out).
// The chunk comes in as three 1 KB coalesced loads into the wave's LDS slice,
// each lane reads its 4 pixels (48 bytes) from there, computes them, writes
// them back to the slice (float16 rounded to nearest even), and the chunk
// leaves as three coalesced stores of 1 KB (512 B for float16).  The same
// per-pixel code as k_inverse.
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

template <int DEG, int XF, int OUT>
__global__ __launch_bounds__(256) void k_inverse4(const f4* __restrict__ in, void* __restrict__ out, uint32_t n_px,
                                                  KCoef k, InvMat mi, int gamma) {
  __shared__ f4 s_buf[4][192];
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  f4* s = s_buf[wv];
  const uint32_t n_chunks = n_px >> 8;
  for (uint32_t c = blockIdx.x * 4u + wv; c < n_chunks; c += gridDim.x * 4u) {
    const f4* src = in + (size_t)c * 192;
    const f4 a0 = src[lane], a1 = src[64 + lane], a2 = src[128 + lane];
    s[lane] = a0;
    s[64 + lane] = a1;
    s[128 + lane] = a2;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the chunk is in LDS
    __builtin_amdgcn_wave_barrier();
    const f4 b0 = s[3 * lane], b1 = s[3 * lane + 1], b2 = s[3 * lane + 2];
    const float v[12] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w, b2.x, b2.y, b2.z, b2.w};
    float o[12];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (XF == MACT_LAB) lab_inv_px<DEG>(k, mi, gamma, v + 3 * j, o + 3 * j);
      else if (XF == MACT_LUV) luv_inv_px<DEG>(k, mi, gamma, v + 3 * j, o + 3 * j);
      else if (XF == MACT_HSI) hsi_inv_px<DEG>(k, v + 3 * j, o + 3 * j);
      else sct_inv_px<DEG>(k, v + 3 * j, o + 3 * j);
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);  // every lane's reads are done before the slice is rewritten
    __builtin_amdgcn_wave_barrier();
    if (OUT == MACT_F32) {
      s[3 * lane] = f4{o[0], o[1], o[2], o[3]};
      s[3 * lane + 1] = f4{o[4], o[5], o[6], o[7]};
      s[3 * lane + 2] = f4{o[8], o[9], o[10], o[11]};
    } else {
      f2* s2 = reinterpret_cast<f2*>(s);  // 12 halves per lane: three 8-byte words
#pragma unroll
      for (int t = 0; t < 3; ++t)
        s2[3 * lane + t] = f2{__uint_as_float(pack2_h_rn(o[4 * t], o[4 * t + 1])),
                              __uint_as_float(pack2_h_rn(o[4 * t + 2], o[4 * t + 3]))};
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    if (OUT == MACT_F32) {
      f4* dst = static_cast<f4*>(out) + (size_t)c * 192;
#pragma unroll
      for (int q = 0; q < 3; ++q) __builtin_nontemporal_store(s[q * 64 + lane], dst + q * 64 + lane);
    } else {
      f2* dst = static_cast<f2*>(out) + (size_t)c * 192;
      const f2* s2 = reinterpret_cast<const f2*>(s);
#pragma unroll
      for (int q = 0; q < 3; ++q) __builtin_nontemporal_store(s2[q * 64 + lane], dst + q * 64 + lane);
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
  }
  // the last n_px % 256 pixels, one per thread of block 0
  const uint32_t tail0 = n_chunks << 8;
  if (blockIdx.x == 0 && threadIdx.x < n_px - tail0) {
    const float* fi = reinterpret_cast<const float*>(in);
    const size_t p = tail0 + threadIdx.x;
    const float v[3] = {fi[3 * p], fi[3 * p + 1], fi[3 * p + 2]};
    float o[3];
    if (XF == MACT_LAB) lab_inv_px<DEG>(k, mi, gamma, v, o);
    else if (XF == MACT_LUV) luv_inv_px<DEG>(k, mi, gamma, v, o);
    else if (XF == MACT_HSI) hsi_inv_px<DEG>(k, v, o);
    else sct_inv_px<DEG>(k, v, o);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (OUT == MACT_F32) static_cast<float*>(out)[3 * p + c] = o[c];
      else static_cast<__half*>(out)[3 * p + c] = f2h_rn(o[c]);
    }
  }
}

// Packed CHW (float32 or float16) -> packed float32 or float16 (OUT) CHW, W H
// a multiple of 4 (network outputs): 4 pixels per lane, one 16- or 8-byte load
// and one 16- or 8-byte store per plane, each contiguous across the wave.  The
// same per-pixel code.
template <int IN, int DEG, int XF, int OUT>
__global__ __launch_bounds__(256) void k_inverse_chw4(const void* __restrict__ in, void* __restrict__ out,
                                                      uint32_t n_px, uint32_t hw, FastDiv div_hw4, KCoef k, InvMat mi,
                                                      int gamma) {
  const uint32_t n4 = n_px >> 2, hw4 = hw >> 2;
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t g4 = blockIdx.x * 256u + threadIdx.x; g4 < n4; g4 += stride) {
    const uint32_t n = div_hw4.div(g4);
    const size_t base = (size_t)n * 3 * hw + 4 * (size_t)(g4 - n * hw4);
    float v[4][3];
    load_planes4<IN, true>(in, base, hw, v);
    float o[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (XF == MACT_LAB) lab_inv_px<DEG>(k, mi, gamma, v[j], o[j]);
      else if (XF == MACT_LUV) luv_inv_px<DEG>(k, mi, gamma, v[j], o[j]);
      else if (XF == MACT_HSI) hsi_inv_px<DEG>(k, v[j], o[j]);
      else sct_inv_px<DEG>(k, v[j], o[j]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (OUT == MACT_F32)
        __builtin_nontemporal_store(f4{o[0][c], o[1][c], o[2][c], o[3][c]},
                                    reinterpret_cast<f4*>(static_cast<float*>(out) + base + (size_t)c * hw));
      else
        __builtin_nontemporal_store(f2{__uint_as_float(pack2_h_rn(o[0][c], o[1][c])),
                                       __uint_as_float(pack2_h_rn(o[2][c], o[3][c]))},
                                    reinterpret_cast<f2*>(static_cast<__half*>(out) + base + (size_t)c * hw));
    }
  }
}

template <int IN, int DEG, int OUT>
void launch_inverse_chw4(int xform, const void* in, void* out, uint32_t n_px, uint32_t hw, const KCoef& k,
                         const InvMat& mi, int gamma, hipStream_t st) {
  const dim3 grid(std::max<uint32_t>(1, (n_px / 4 + 255) / 256)), blk(256);
  const FastDiv d = make_fastdiv(hw / 4);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_inverse_chw4<IN, DEG, MACT_LAB, OUT>), grid, blk, 0, st, in, out, n_px, hw, d, k, mi, gamma);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_inverse_chw4<IN, DEG, MACT_LUV, OUT>), grid, blk, 0, st, in, out, n_px, hw, d, k, mi, gamma);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_inverse_chw4<IN, DEG, MACT_HSI, OUT>), grid, blk, 0, st, in, out, n_px, hw, d, k, mi, gamma);
  else hipLaunchKernelGGL((k_inverse_chw4<IN, DEG, MACT_SCT, OUT>), grid, blk, 0, st, in, out, n_px, hw, d, k, mi, gamma);
}

template <int IN>
void launch_inverse_chw4_io(int xform, int out_dtype, int deg, const void* in, void* out, uint32_t n_px, uint32_t hw,
                            const KCoef& k, const InvMat& mi, int gamma, hipStream_t st) {
  if (out_dtype == MACT_F32) {
    if (deg == 5) launch_inverse_chw4<IN, 5, MACT_F32>(xform, in, out, n_px, hw, k, mi, gamma, st);
    else launch_inverse_chw4<IN, 7, MACT_F32>(xform, in, out, n_px, hw, k, mi, gamma, st);
  } else {
    if (deg == 5) launch_inverse_chw4<IN, 5, MACT_F16>(xform, in, out, n_px, hw, k, mi, gamma, st);
    else launch_inverse_chw4<IN, 7, MACT_F16>(xform, in, out, n_px, hw, k, mi, gamma, st);
  }
}

template <int DEG, int OUT>
void launch_inverse4(int xform, const void* in, void* out, uint32_t n_px, const KCoef& k, const InvMat& mi, int gamma,
                     unsigned grid, hipStream_t st) {
  const f4* i4 = static_cast<const f4*>(in);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_inverse4<DEG, MACT_LAB, OUT>), dim3(grid), dim3(256), 0, st, i4, out, n_px, k, mi, gamma);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_inverse4<DEG, MACT_LUV, OUT>), dim3(grid), dim3(256), 0, st, i4, out, n_px, k, mi, gamma);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_inverse4<DEG, MACT_HSI, OUT>), dim3(grid), dim3(256), 0, st, i4, out, n_px, k, mi, gamma);
  else hipLaunchKernelGGL((k_inverse4<DEG, MACT_SCT, OUT>), dim3(grid), dim3(256), 0, st, i4, out, n_px, k, mi, gamma);
}

// ---------------------------------------------------------------- exact, float64

__device__ __forceinline__ double dev_inverse_gamma(double k, int gamma) {
  if (gamma == MACT_GAMMA_BT709) return k < 0.081 ? k / 4.5 : pow((k + 0.099) / 1.099, 1.0 / 0.45);
  if (gamma == MACT_GAMMA_SRGB) return k <= 0.04045 ? k / 12.92 : pow((k + 0.055) / 1.055, 2.4);
  return k;
}

__device__ __forceinline__ void dev_lab_lin(const double lin[3], double out[3]) {
  double f[3];
  for (int r = 0; r < 3; ++r) {
    const double t = (kM[r][0] * lin[0] + kM[r][1] * lin[1] + kM[r][2] * lin[2]) / kWhite[r];
    f[r] = t > kLabT0 ? cbrt(t) : kLabK * t + kLabC;
  }
  out[0] = 116.0 * f[1] - 16.0;
  out[1] = 500.0 * (f[0] - f[1]);
  out[2] = 200.0 * (f[1] - f[2]);
}

__device__ __forceinline__ void dev_lab(const double rgb[3], int gamma, double out[3]) {
  double lin[3];
  for (int c = 0; c < 3; ++c) lin[c] = dev_inverse_gamma(rgb[c], gamma);
  dev_lab_lin(lin, out);
}

__device__ __forceinline__ void dev_luv_lin(const double lin[3], double out[3]) {
  double xyz[3];
  for (int r = 0; r < 3; ++r) xyz[r] = kM[r][0] * lin[0] + kM[r][1] * lin[1] + kM[r][2] * lin[2];
  const double fy = xyz[1] > kLabT0 ? cbrt(xyz[1]) : kLabK * xyz[1] + kLabC;
  const double L = 116.0 * fy - 16.0;
  const double d = xyz[0] + 15.0 * xyz[1] + 3.0 * xyz[2];
  const double dn = kWhite[0] + 15.0 * kWhite[1] + 3.0 * kWhite[2];
  out[0] = L;
  out[1] = d > 0.0 ? 13.0 * L * (4.0 * xyz[0] / d - 4.0 * kWhite[0] / dn) : 0.0;
  out[2] = d > 0.0 ? 13.0 * L * (9.0 * xyz[1] / d - 9.0 * kWhite[1] / dn) : 0.0;
}

__device__ __forceinline__ void dev_luv(const double rgb[3], int gamma, double out[3]) {
  double lin[3];
  for (int c = 0; c < 3; ++c) lin[c] = dev_inverse_gamma(rgb[c], gamma);
  dev_luv_lin(lin, out);
}

__device__ __forceinline__ void dev_hsi(const double rgb[3], double out[3]) {
  // Kender's form with the exact arctan (Sec. 3.3.1); H = 0 where undefined
  const double R = rgb[0], G = rgb[1], B = rgb[2];
  double H = 0.0;
  if (R > B && G > B) H = kPi / 3.0 + atan(sqrt(3.0) * (G - R) / ((G - B) + (R - B)));
  else if (G > R) H = kPi + atan(sqrt(3.0) * (B - G) / ((B - R) + (G - R)));
  else if (B > G) H = 5.0 * kPi / 3.0 + atan(sqrt(3.0) * (R - B) / ((R - G) + (B - G)));
  const double s = R + G + B;
  out[0] = H;
  out[1] = s > 0.0 ? 1.0 - 3.0 * fmin(R, fmin(G, B)) / s : 0.0;
  out[2] = s / 3.0;
}

__device__ __forceinline__ void dev_sct(const double rgb[3], double out[3]) {
  const double R = rgb[0], G = rgb[1], B = rgb[2];
  const double L = sqrt(R * R + G * G + B * B);
  out[0] = L;
  out[1] = L > 0.0 ? acos(fmin(1.0, B / L)) : 0.0;
  out[2] = atan2(G, R);
}

__device__ __forceinline__ void dev_sct_to_rgb(const double s[3], double rgb[3]) {
  const double sa = sin(s[1]);
  rgb[0] = s[0] * sa * cos(s[2]);
  rgb[1] = s[0] * sa * sin(s[2]);
  rgb[2] = s[0] * cos(s[1]);
}

__device__ __forceinline__ double dev_delta_e(const double a[3], const double b[3]) {
  const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
  return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

// |a - b| wrapped to [0, pi]
__device__ __forceinline__ double dev_angle_diff(double a, double b) {
  double d = fmod(fabs(a - b), 2.0 * kPi);
  return fmin(d, 2.0 * kPi - d);
}

// Accumulators: [0] sum of the metric, [1] its max, [2..4] per-channel max |difference|.
// Maxima of non-negative doubles are kept as their bit patterns, which order like integers.
struct ErrAcc {
  double sum;
  unsigned long long max_bits[4];
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <int DEG>
__global__ __launch_bounds__(256) void k_error(KImage src, uint32_t n_px, KCoef k, int gamma, ErrAcc* acc) {
  __shared__ float gtab[256];
  __shared__ double s_red[4][5];
  gtab[threadIdx.x] = k_gamma_table[gamma][threadIdx.x];
  __syncthreads();
  const double scale = src.dtype == MACT_U8 ? 1.0 / 255.0 : src.dtype == MACT_U16 ? 1.0 / 65535.0 : 1.0;
  double sum = 0.0, mx[4] = {0.0, 0.0, 0.0, 0.0};
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t p = blockIdx.x * 256u + threadIdx.x; p < n_px; p += stride) {
    float v[3], o[3];
    load_px(src, p, v);
    eval_px<DEG>(k, src.dtype, gamma, gtab, v, o);
    const double rgb[3] = {v[0] * scale, v[1] * scale, v[2] * scale};  // raw values, [0, 1] scale
    const double m[3] = {o[0], o[1], o[2]};
    double ex[3], e, d[3];
    if (k.xform == MACT_LAB || k.xform == MACT_LUV) {
      if (src.dtype == MACT_U8) {
        // 8-bit codes: the decoded values from the double-precision table (no pow per pixel)
        const double lin[3] = {k_gamma_table64[gamma][(int)v[0]], k_gamma_table64[gamma][(int)v[1]],
                               k_gamma_table64[gamma][(int)v[2]]};
        if (k.xform == MACT_LAB) dev_lab_lin(lin, ex);
        else dev_luv_lin(lin, ex);
      } else if (k.xform == MACT_LAB) {
        dev_lab(rgb, gamma, ex);
      } else {
        dev_luv(rgb, gamma, ex);
      }
      e = dev_delta_e(m, ex);
      for (int c = 0; c < 3; ++c) d[c] = fabs(m[c] - ex[c]);
    } else if (k.xform == MACT_HSI) {
      dev_hsi(rgb, ex);
      const double th = dev_angle_diff(m[0], ex[0]);
      const double dv = m[2] - ex[2];
      e = sqrt(fmax(m[1] * m[1] + ex[1] * ex[1] - 2.0 * m[1] * ex[1] * cos(th) + dv * dv, 0.0));
      d[0] = th;
      d[1] = fabs(m[1] - ex[1]);
      d[2] = fabs(dv);
    } else {
      dev_sct(rgb, ex);
      double ra[3], la[3], lb[3];
      dev_sct_to_rgb(m, ra);
      dev_lab(ra, MACT_GAMMA_BT709, la);
      if (src.dtype == MACT_U8) {
        // the exact triple inverts to the input itself: its L*a*b* from the decoding table
        const double lin[3] = {k_gamma_table64[MACT_GAMMA_BT709][(int)v[0]],
                               k_gamma_table64[MACT_GAMMA_BT709][(int)v[1]],
                               k_gamma_table64[MACT_GAMMA_BT709][(int)v[2]]};
        dev_lab_lin(lin, lb);
      } else {
        double rb[3];
        dev_sct_to_rgb(ex, rb);
        dev_lab(rb, MACT_GAMMA_BT709, lb);
      }
      e = dev_delta_e(la, lb);
      for (int c = 0; c < 3; ++c) d[c] = fabs(m[c] - ex[c]);
    }
    sum += e;
    mx[0] = fmax(mx[0], e);
    for (int c = 0; c < 3; ++c) mx[c + 1] = fmax(mx[c + 1], d[c]);
  }
  sum = wave_sum(sum);
  for (int c = 0; c < 4; ++c) mx[c] = wave_max(mx[c]);
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  if (lane == 0) {
    s_red[wv][0] = sum;
    for (int c = 0; c < 4; ++c) s_red[wv][c + 1] = mx[c];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bs = 0.0, bm[4] = {0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < 4; ++w) {
      bs += s_red[w][0];
      for (int c = 0; c < 4; ++c) bm[c] = fmax(bm[c], s_red[w][c + 1]);
    }
    atomicAdd(&acc->sum, bs);
    for (int c = 0; c < 4; ++c) atomicMax(&acc->max_bits[c], (unsigned long long)__double_as_longlong(bm[c]));
  }
}

unsigned grid_256(uint64_t work, int per_cu) {
  const uint64_t need = (work + 255) / 256;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(need, (uint64_t)device_cus() * per_cu));
}

// Cached default inverse approximations (made once per process).
struct InvDefaults {
  mact_approx enc, cos_h, sin_s, cos_s;
  mact_status st = MACT_OK;
};

const InvDefaults& inv_defaults() {
  static InvDefaults d;
  static std::once_flag once;
  std::call_once(once, [] {
    mact_status s = mact_fit(MACT_FN_ENC709, 4, 4, 0.018, 1.0, &d.enc);
    if (s == MACT_OK) s = mact_fit(MACT_FN_COS, 7, 0, 0.0, 2.0 * kPi / 3.0, &d.cos_h);
    if (s == MACT_OK) s = mact_default_approx(MACT_FN_SIN, &d.sin_s);
    if (s == MACT_OK) s = mact_default_approx(MACT_FN_COS, &d.cos_s);
    d.st = s;
  });
  return d;
}

// Validation of inverse parameters; the KCoef packing of pack_coef does not
// apply (the inverse uses f[0] and f[1] in its own way), so they are packed here.
mact_status pack_inverse(const mact_params* p, int gamma, KCoef* k, int* deg) {
  if (!p) return fail(MACT_E_INVALID, "mact_inverse: params is NULL");
  if (p->xform < MACT_LAB || p->xform > MACT_LUV) return fail(MACT_E_INVALID, "mact_inverse: xform %d", p->xform);
  if (p->out_mode != 0) return fail(MACT_E_INVALID, "mact_inverse: out_mode must be 0");
  std::memset(k, 0, sizeof *k);
  k->xform = p->xform;
  k->q[0] = 1.0f;
  int d = 0;
  const int nf = p->xform == MACT_SCT ? 2 : 1;
  const bool encodes = p->xform == MACT_LAB || p->xform == MACT_LUV;
  const bool need = !(encodes && gamma == MACT_GAMMA_NONE);
  for (int i = 0; i < nf && need; ++i) {
    const mact_approx& a = p->f[i];
    mact_status s = check_approx(a, encodes, "mact_inverse");
    if (s != MACT_OK) return s;
    const int want = encodes ? MACT_FN_ENC709 : p->xform == MACT_HSI ? MACT_FN_COS
                                                                     : (i == 0 ? MACT_FN_SIN : MACT_FN_COS);
    if (a.fn != want) return fail(MACT_E_INVALID, "mact_inverse: f[%d] approximates function %d, expected %d", i, a.fn, want);
    for (int j = 0; j <= a.n; ++j) k->p[i][j] = (float)a.p[j];
    d = std::max(d, a.n);
    if (a.m > 0) {
      for (int j = 0; j <= a.m; ++j) k->q[j] = (float)a.q[j];
      d = std::max(d, a.m);
    }
  }
  *deg = d <= 5 ? 5 : 7;
  return MACT_OK;
}

}  // namespace
}  // namespace mact

using namespace mact;

extern "C" mact_status mact_inverse_params_default(int32_t xform, mact_params* p) {
  clear_error();
  if (!p) return fail(MACT_E_INVALID, "mact_inverse_params_default: NULL");
  if (xform < MACT_LAB || xform > MACT_LUV) return fail(MACT_E_INVALID, "mact_inverse_params_default: xform %d", xform);
  const InvDefaults& d = inv_defaults();
  if (d.st != MACT_OK) return fail(d.st, "mact_inverse_params_default: fitting the default approximations failed");
  std::memset(p, 0, sizeof *p);
  p->xform = xform;
  if (xform == MACT_LAB || xform == MACT_LUV) p->f[0] = d.enc;
  else if (xform == MACT_HSI) p->f[0] = d.cos_h;
  else {
    p->f[0] = d.sin_s;
    p->f[1] = d.cos_s;
  }
  return MACT_OK;
}

extern "C" mact_status mact_inverse(const mact_params* params, const mact_image* in, const mact_image* out,
                                    void* hip_stream) {
  clear_error();
  HostImage hi, ho;
  mact_status s;
  if ((s = resolve_image(in, false, "mact_inverse: in", &hi)) != MACT_OK) return s;
  if ((s = resolve_image(out, true, "mact_inverse: out", &ho)) != MACT_OK) return s;
  if ((s = check_same_shape(hi, ho, "mact_inverse: out")) != MACT_OK) return s;
  if (hi.dtype == MACT_U8 || hi.dtype == MACT_U16)
    return fail(MACT_E_UNSUPPORTED, "mact_inverse: in must be MACT_F32 or MACT_F16");
  if (!params) return fail(MACT_E_INVALID, "mact_inverse: params is NULL");
  int gamma = MACT_GAMMA_NONE;
  if (params->xform == MACT_LAB || params->xform == MACT_LUV) {
    gamma = ho.gamma;
    if (gamma == MACT_GAMMA_SRGB) return fail(MACT_E_UNSUPPORTED, "mact_inverse: sRGB encoding has no default approximation");
  }
  KCoef k;
  int deg = 5;
  if ((s = pack_inverse(params, gamma, &k, &deg)) != MACT_OK) return s;
  static const InvMat mi_lab = make_inv_mat(true), mi_luv = make_inv_mat(false);
  const InvMat& mi = params->xform == MACT_LUV ? mi_luv : mi_lab;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int64_t per = images_per_stream_launch(hi, ho);
  // float32 or float16 out for both 4-pixel paths
  const bool fast = hi.dtype == MACT_F32 && hi.layout == MACT_HWC && ho.layout == MACT_HWC && hi.packed && ho.packed;
  const bool chw4 = (hi.dtype == MACT_F32 || hi.dtype == MACT_F16) && hi.layout == MACT_CHW &&
                    ho.layout == MACT_CHW && hi.packed && ho.packed && (hi.W * hi.H) % 4 == 0;
  for (int64_t n0 = 0; n0 < hi.N; n0 += per) {
    const int64_t cnt = std::min(per, hi.N - n0);
    const uint32_t n_px = (uint32_t)(cnt * hi.W * hi.H);
    const KImage ks = kimage(hi, n0, cnt), kd = kimage(ho, n0, cnt);
    if (fast && (uintptr_t)ks.ptr % 16 == 0 && (uintptr_t)kd.ptr % 16 == 0) {
      // one 256-pixel chunk per wave, 4 waves per workgroup, the grid covering the image once;
      // at least one workgroup for the tail
      const unsigned grid = (unsigned)std::max<uint64_t>(1, ((uint64_t)(n_px >> 8) + 3) / 4);
      if (ho.dtype == MACT_F32) {
        if (deg == 5) launch_inverse4<5, MACT_F32>(params->xform, ks.ptr, kd.ptr, n_px, k, mi, gamma, grid, st);
        else launch_inverse4<7, MACT_F32>(params->xform, ks.ptr, kd.ptr, n_px, k, mi, gamma, grid, st);
      } else {
        if (deg == 5) launch_inverse4<5, MACT_F16>(params->xform, ks.ptr, kd.ptr, n_px, k, mi, gamma, grid, st);
        else launch_inverse4<7, MACT_F16>(params->xform, ks.ptr, kd.ptr, n_px, k, mi, gamma, grid, st);
      }
    } else if (chw4 && (uintptr_t)ks.ptr % (4 * hi.esize) == 0 && (uintptr_t)kd.ptr % 16 == 0) {
      const uint32_t hw = (uint32_t)(hi.W * hi.H);
      if (hi.dtype == MACT_F32) launch_inverse_chw4_io<MACT_F32>(params->xform, ho.dtype, deg, ks.ptr, kd.ptr, n_px, hw, k, mi, gamma, st);
      else launch_inverse_chw4_io<MACT_F16>(params->xform, ho.dtype, deg, ks.ptr, kd.ptr, n_px, hw, k, mi, gamma, st);
    } else {
      const dim3 grid(std::max<uint32_t>(1, (n_px + 255) / 256)), blk(256);
      if (deg == 5) hipLaunchKernelGGL(k_inverse<5>, grid, blk, 0, st, ks, kd, n_px, k, mi, gamma);
      else hipLaunchKernelGGL(k_inverse<7>, grid, blk, 0, st, ks, kd, n_px, k, mi, gamma);
    }
    if ((s = hip_check(hipGetLastError(), "mact_inverse: launch")) != MACT_OK) return s;
  }
  return MACT_OK;
}

namespace mact {
namespace {

__global__ void k_clear_acc(ErrAcc* acc) {
  acc->sum = 0.0;
  for (int c = 0; c < 4; ++c) acc->max_bits[c] = 0ull;
}

// Both forms of the error statistics: validate, clear the accumulator `d_acc`
// (a fill kernel, not a memset), launch k_error over the image in equal
// launches, copy the record back, wait for the stream and fill *out.
mact_status error_stats_with(const mact_params* params, const mact_image* in, mact_error* out, void* hip_stream,
                             ErrAcc* (*get_acc)(mact_status*), void (*put_acc)(ErrAcc*), const char* what) {
  if (!out) return fail(MACT_E_INVALID, "%s: out is NULL", what);
  std::memset(out, 0, sizeof *out);
  mact_status s = check_params(params);
  if (s != MACT_OK) return s;
  if (params->out_mode != 0) return fail(MACT_E_INVALID, "%s: out_mode must be 0", what);
  HostImage hi;
  if ((s = resolve_image(in, false, what, &hi)) != MACT_OK) return s;
  KCoef k;
  const int deg = pack_coef(*params, &k);
  const int gamma = uses_gamma(params->xform) ? hi.gamma : MACT_GAMMA_NONE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  ErrAcc* d_acc = get_acc(&s);
  if (!d_acc) return s;
  hipLaunchKernelGGL(k_clear_acc, dim3(1), dim3(1), 0, st, d_acc);
  s = hip_check(hipGetLastError(), "error statistics: clear");
  const int64_t per = images_per_launch(hi);
  for (int64_t n0 = 0; n0 < hi.N && s == MACT_OK; n0 += per) {
    const int64_t cnt = std::min(per, hi.N - n0);
    const uint32_t n_px = (uint32_t)(cnt * hi.W * hi.H);
    const KImage ks = kimage(hi, n0, cnt);
    const dim3 grid(grid_256(n_px, 16)), blk(256);
    if (deg == 5) hipLaunchKernelGGL(k_error<5>, grid, blk, 0, st, ks, n_px, k, gamma, d_acc);
    else hipLaunchKernelGGL(k_error<7>, grid, blk, 0, st, ks, n_px, k, gamma, d_acc);
    s = hip_check(hipGetLastError(), "error statistics: launch");
  }
  ErrAcc h;
  std::memset(&h, 0, sizeof h);
  if (s == MACT_OK) s = hip_check(hipMemcpyAsync(&h, d_acc, sizeof h, hipMemcpyDeviceToHost, st), "error statistics: copy");
  if (s == MACT_OK) s = hip_check(hipStreamSynchronize(st), "error statistics: synchronise");
  put_acc(d_acc);
  if (s != MACT_OK) return s;
  const int64_t count = hi.N * hi.W * hi.H;
  double mx[4];
  for (int c = 0; c < 4; ++c) std::memcpy(&mx[c], &h.max_bits[c], sizeof(double));
  out->count = count;
  out->mean = h.sum / (double)count;
  out->max = mx[0];
  for (int c = 0; c < 3; ++c) out->max_abs[c] = mx[c + 1];
  return MACT_OK;
}

ErrAcc* alloc_acc(mact_status* s) {
  ErrAcc* d = nullptr;
  if (hipMalloc(&d, sizeof(ErrAcc)) != hipSuccess) {
    *s = fail(MACT_E_NOMEM, "mact_error_stats: device allocation");
    return nullptr;
  }
  return d;
}

void free_acc(ErrAcc* d) { (void)hipFree(d); }

}  // namespace
}  // namespace mact

extern "C" mact_status mact_error_stats(const mact_params* params, const mact_image* in, mact_error* out,
                                        void* hip_stream) {
  clear_error();
  return error_stats_with(params, in, out, hip_stream, alloc_acc, free_acc, "mact_error_stats");
}

// ---------------------------------------------------------------- the allocation-free form
//
// The accumulator of mact_error_stats_noalloc lives in `scratch`, a file-scope
// device array: each GPU the library runs on holds its own copy, at its own
// address, until the process ends.  In host code the array's name stands for
// no device address, so host code never passes it to a kernel or a copy; it
// uses the address hipGetSymbolAddress returns for the current GPU, looked up
// once per GPU.  Every call on one GPU uses the same record (cleared by the
// call before use), so calls that overlap on one GPU race.

static constexpr size_t kScratchBytes = 256;
static_assert(sizeof(mact::ErrAcc) <= kScratchBytes, "the accumulator record must fit the scratch array");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices];

mact::ErrAcc* scratch_acc(mact_status* s) {
  int dev = -1;
  if ((*s = mact::hip_check(hipGetDevice(&dev), "mact_error_stats_noalloc: current device")) != MACT_OK) return nullptr;
  if (dev < 0 || dev >= kMaxScratchDevices) {
    *s = mact::fail(MACT_E_UNSUPPORTED, "mact_error_stats_noalloc: device %d beyond the %d the library serves", dev,
                    kMaxScratchDevices);
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if ((*s = mact::hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)),
                              "mact_error_stats_noalloc: scratch address")) != MACT_OK)
      return nullptr;
    if (!ptr) {
      *s = mact::fail(MACT_E_DEVICE, "mact_error_stats_noalloc: no scratch address on device %d", dev);
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return static_cast<mact::ErrAcc*>(g_scratch_ptr[dev]);
}

void keep_acc(mact::ErrAcc*) {}

}  // namespace

extern "C" mact_status mact_error_stats_noalloc(const mact_params* params, const mact_image* in, mact_error* out,
                                                void* hip_stream) {
  clear_error();
  return error_stats_with(params, in, out, hip_stream, scratch_acc, keep_acc, "mact_error_stats_noalloc");
}
