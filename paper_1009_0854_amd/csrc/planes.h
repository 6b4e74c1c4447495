// Loads of 4 consecutive pixels from packed CHW planes, shared by the plane
// kernels (forward, layout-converting and inverse).
#pragma once

#include "pixel.h"

namespace mact {

typedef float planes_f4 __attribute__((ext_vector_type(4)));

// The 4 pixels at element `base` of plane 0 of a packed CHW image whose planes
// lie hw elements apart: one 16-, 8- or 4-byte load per plane (float32,
// float16 / 16-bit, 8-bit), contiguous across the wave.  v[j][c] is channel c
// of pixel j as load_px returns it: float values clamped to [0, 1], integer
// codes as they are.  RAW: float values unclamped (the inverse transforms'
// inputs are colour-space values, not RGB).  `base` must be a multiple of 4.
template <int IN, bool RAW = false>
__device__ __forceinline__ void load_planes4(const void* in, size_t base, uint32_t hw, float v[4][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const size_t o = base + (size_t)c * hw;
    if (IN == MACT_F32) {
      const planes_f4 x = *reinterpret_cast<const planes_f4*>(static_cast<const float*>(in) + o);
      const float e[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j][c] = RAW ? e[j] : clamp01(e[j]);
    } else if (IN == MACT_F16) {
      const uint2 x = *reinterpret_cast<const uint2*>(static_cast<const __half*>(in) + o);
      const uint32_t w[2] = {x.x, x.y};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float h = __half2float(__ushort_as_half((uint16_t)(w[j >> 1] >> (16 * (j & 1)))));
        v[j][c] = RAW ? h : clamp01(h);
      }
    } else if (IN == MACT_U16) {
      const uint2 x = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(in) + o);
      const uint32_t w[2] = {x.x, x.y};
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j][c] = (float)((w[j >> 1] >> (16 * (j & 1))) & 0xffffu);
    } else {
      const uint32_t x = *reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(in) + o);
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j][c] = (float)((x >> (8 * j)) & 0xffu);
    }
  }
}

}  // namespace mact
