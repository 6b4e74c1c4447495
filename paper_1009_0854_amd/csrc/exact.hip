// The exact transforms in float32 with the device's elementary functions: the
// baseline that MACT replaces.  The paper measures MACT's gain over the exact
// transforms evaluated with the C library's functions (Sec. 3.5, Table 11);
// this is the same comparison on the GPU.
//
// Per pixel, with the arithmetic MACT keeps unchanged (the 8-bit inverse-gamma
// table, the matrix, the linear segment, the Kender branches, the L*a*b*
// assembly) and the approximated functions replaced by the library's:
//   CIELAB, CIELUV: cbrtf above t = 0.008856 (Sec. 3.2.1);
//   HSI: atanf(sqrt(3) x) in Kender's form (Sec. 3.3.1);
//   SCT: sqrtf for L; angle A = arccos(B/L), taken as 2 asinf(sqrt((1 - B/L)/2))
//        where B/L >= 0.5 (the same identity MACT's split uses, which keeps the
//        float32 error small near the blue axis) and acosf(B/L) below; angle B =
//        atan2f(G, R) (Sec. 3.4.1).
// Packed 8-bit HWC in, packed float32 or float16 HWC out, with the hot
// kernel's loads and LDS-transposed stores.
#include <algorithm>
#include <cmath>

#include "launch.h"
#include "stream.h"

namespace mact {

#include "gamma_table.inc"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr float kSqrt3f = 1.7320508075688772f;

__device__ __forceinline__ float lab_f_exact(float t) { return t > kT0f ? cbrtf(t) : __builtin_fmaf(kLabKf, t, kLabCf); }

template <int XF>
__device__ __forceinline__ void exact_px(const float* gtab, uint32_t r8, uint32_t g8, uint32_t b8, float o[3]) {
  if (XF == MACT_LAB) {
    const float lr = gtab[r8], lg = gtab[g8], lb = gtab[b8];
    const float fx = lab_f_exact(__builtin_fmaf(kMw00, lr, __builtin_fmaf(kMw01, lg, kMw02 * lb)));
    const float fy = lab_f_exact(__builtin_fmaf(kMw10, lr, __builtin_fmaf(kMw11, lg, kMw12 * lb)));
    const float fz = lab_f_exact(__builtin_fmaf(kMw20, lr, __builtin_fmaf(kMw21, lg, kMw22 * lb)));
    o[0] = __builtin_fmaf(116.0f, fy, -16.0f);
    o[1] = 500.0f * (fx - fy);
    o[2] = 200.0f * (fy - fz);
  } else if (XF == MACT_LUV) {
    const float lr = gtab[r8], lg = gtab[g8], lb = gtab[b8];
    const float X = __builtin_fmaf(kM00, lr, __builtin_fmaf(kM01, lg, kM02 * lb));
    const float Y = __builtin_fmaf(kM10, lr, __builtin_fmaf(kM11, lg, kM12 * lb));
    const float Z = __builtin_fmaf(kM20, lr, __builtin_fmaf(kM21, lg, kM22 * lb));
    const float L = __builtin_fmaf(116.0f, lab_f_exact(Y), -16.0f);
    const float D = __builtin_fmaf(15.0f, Y, __builtin_fmaf(3.0f, Z, X));
    o[0] = L;
    if (!(D > 0.0f)) {
      o[1] = 0.0f;
      o[2] = 0.0f;
      return;
    }
    const float L13 = 13.0f * L;
    o[1] = L13 * (4.0f * X / D - kUn);
    o[2] = L13 * (9.0f * Y / D - kVn);
  } else if (XF == MACT_HSI) {
    const float R = (float)r8, G = (float)g8, B = (float)b8;
    float H = 0.0f;
    if (R > B && G > B) H = kPi3f + atanf(kSqrt3f * (G - R) / ((G - B) + (R - B)));
    else if (G > R) H = kPif + atanf(kSqrt3f * (B - G) / ((B - R) + (G - R)));
    else if (B > G) H = k5Pi3f + atanf(kSqrt3f * (R - B) / ((R - G) + (B - G)));
    const float sum = (R + G) + B;
    o[0] = H;
    o[1] = sum > 0.0f ? 1.0f - 3.0f * fminf(R, fminf(G, B)) / sum : 0.0f;
    o[2] = sum * kInv765;
  } else {
    const float R = (float)r8, G = (float)g8, B = (float)b8;
    const float rg2 = __builtin_fmaf(R, R, G * G);
    const float L2 = __builtin_fmaf(B, B, rg2);
    if (!(L2 > 0.0f)) {
      o[0] = 0.0f; o[1] = 0.0f; o[2] = 0.0f;
      return;
    }
    const float L = sqrtf(L2);
    o[0] = L * kInv255;
    o[1] = 3.0f * (B * B) >= rg2 ? 2.0f * asinf(sqrtf(rg2 / (2.0f * L * (L + B)))) : acosf(B / L);
    o[2] = atan2f(G, R);
  }
}

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kCpw = 2;  // chunks of 256 pixels per wave

template <int OUT, int XF>
__global__ __launch_bounds__(kBlock) void k_exact4(const uint8_t* __restrict__ in, void* __restrict__ out, uint32_t n_px,
                                                   int gamma) {
  constexpr uint32_t F4PC = OUT == MACT_F32 ? 192 : 96;  // 16-byte output words per chunk
  __shared__ f4 s_out[kWaves][kCpw * F4PC];
  __shared__ float gtab[256];
  for (uint32_t i = threadIdx.x; i < 256u; i += kBlock) gtab[i] = k_gamma_table[gamma][i];
  __syncthreads();
  const uint32_t n_chunks = n_px >> 8;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t c0 = (blockIdx.x * kWaves + wv) * kCpw;
  if (c0 < n_chunks) {
    uint3 w[kCpw];
#pragma unroll
    for (int j = 0; j < kCpw; ++j)
      if (c0 + j < n_chunks) w[j] = reinterpret_cast<const uint3*>(in)[(size_t)(c0 + j) * 64 + lane];
#pragma unroll
    for (int j = 0; j < kCpw; ++j) {
      if (c0 + j >= n_chunks) break;
      float o[12];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        exact_px<XF>(gtab, byte_of(w[j], 3 * i), byte_of(w[j], 3 * i + 1), byte_of(w[j], 3 * i + 2), o + 3 * i);
      if (OUT == MACT_F32) {
        s_out[wv][j * 192 + 3 * lane] = f4{o[0], o[1], o[2], o[3]};
        s_out[wv][j * 192 + 3 * lane + 1] = f4{o[4], o[5], o[6], o[7]};
        s_out[wv][j * 192 + 3 * lane + 2] = f4{o[8], o[9], o[10], o[11]};
      } else {
        f2* s2 = reinterpret_cast<f2*>(&s_out[wv][0]);  // chunk j's halves start at 8-byte word 192 j
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const uint32_t lo = pack2_h_rn(o[4 * t], o[4 * t + 1]);
          const uint32_t hi = pack2_h_rn(o[4 * t + 2], o[4 * t + 3]);
          s2[j * 192 + 3 * lane + t] = f2{__uint_as_float(lo), __uint_as_float(hi)};
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): every lane's LDS writes have landed
    __builtin_amdgcn_wave_barrier();
    const uint32_t n_valid = min((uint32_t)kCpw, n_chunks - c0) * F4PC;
    const StreamBuf dst = wave_stream_buf(reinterpret_cast<f4*>(out) + (size_t)c0 * F4PC, n_valid * 16u);
#pragma unroll
    for (int q = 0; q < (int)(kCpw * F4PC / 64); ++q) {
      const uint32_t e = q * 64 + lane;
      if (e < n_valid) stream_store(dst, e * 16u, s_out[wv][e]);
    }
  }
  // the last n_px % 256 pixels, one per lane of block 0
  const uint32_t tail0 = n_chunks << 8;
  if (blockIdx.x == 0 && threadIdx.x < n_px - tail0) {
    const size_t p = tail0 + threadIdx.x;
    float o[3];
    exact_px<XF>(gtab, in[3 * p], in[3 * p + 1], in[3 * p + 2], o);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (OUT == MACT_F32) static_cast<float*>(out)[3 * p + c] = o[c];
      else static_cast<__half*>(out)[3 * p + c] = f2h_rn(o[c]);
    }
  }
}

template <int OUT>
void launch_exact(int xform, const uint8_t* in, void* out, uint32_t n_px, int gamma, hipStream_t st) {
  const uint32_t per_block = kWaves * kCpw;
  const dim3 grid(std::max<uint32_t>(1, ((n_px >> 8) + per_block - 1) / per_block)), blk(kBlock);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_exact4<OUT, MACT_LAB>), grid, blk, 0, st, in, out, n_px, gamma);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_exact4<OUT, MACT_HSI>), grid, blk, 0, st, in, out, n_px, gamma);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_exact4<OUT, MACT_LUV>), grid, blk, 0, st, in, out, n_px, gamma);
  else hipLaunchKernelGGL((k_exact4<OUT, MACT_SCT>), grid, blk, 0, st, in, out, n_px, gamma);
}

}  // namespace
}  // namespace mact

using namespace mact;

extern "C" mact_status mact_transform_exact(int32_t xform, const mact_image* in, const mact_image* out,
                                            void* hip_stream) {
  clear_error();
  if (xform < MACT_LAB || xform > MACT_LUV) return fail(MACT_E_INVALID, "mact_transform_exact: xform %d", xform);
  HostImage hi, ho;
  mact_status s;
  if ((s = resolve_image(in, false, "mact_transform_exact: in", &hi)) != MACT_OK) return s;
  if ((s = resolve_image(out, true, "mact_transform_exact: out", &ho)) != MACT_OK) return s;
  if ((s = check_same_shape(hi, ho, "mact_transform_exact: out")) != MACT_OK) return s;
  if (hi.dtype != MACT_U8 || hi.layout != MACT_HWC || !hi.packed || ho.layout != MACT_HWC || !ho.packed)
    return fail(MACT_E_UNSUPPORTED, "mact_transform_exact: packed 8-bit HWC in and packed HWC out only");
  const int gamma = uses_gamma(xform) ? hi.gamma : MACT_GAMMA_NONE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int64_t per = images_per_stream_launch(hi, ho);
  for (int64_t n0 = 0; n0 < hi.N; n0 += per) {
    const int64_t cnt = std::min(per, hi.N - n0);
    const uint32_t n_px = (uint32_t)(cnt * hi.W * hi.H);
    const uint8_t* ip = static_cast<const uint8_t*>(hi.data) + (size_t)(n0 * hi.bs);
    char* op = static_cast<char*>(ho.data) + (size_t)(n0 * ho.bs) * ho.esize;
    if ((uintptr_t)ip % 4 || (uintptr_t)op % 16)
      return fail(MACT_E_UNSUPPORTED, "mact_transform_exact: input must be 4-byte and output 16-byte aligned");
    if (ho.dtype == MACT_F32) launch_exact<MACT_F32>(xform, ip, op, n_px, gamma, st);
    else launch_exact<MACT_F16>(xform, ip, op, n_px, gamma, st);
    if ((s = hip_check(hipGetLastError(), "mact_transform_exact: launch")) != MACT_OK) return s;
  }
  return MACT_OK;
}
