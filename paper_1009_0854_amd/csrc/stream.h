// Streaming stores: results that nothing in the launch reads again.
//
// They leave with two cache-policy bits set: NT (non-temporal: the L2 is not
// to keep the lines) and SC1 (device scope: the L2 writes the data through
// rather than holding it dirty until the writeback at the end of the kernel).
// The builtin non-temporal store sets NT alone.
//
// Which is faster depends on the kernel; measured on MI355X in one process,
// NT + SC1 against NT alone over the 64 x 1080p batch:
//   8- and 16-bit inputs through the 4-pixel transforms (packed HWC, row
//   views, CHW -> HWC), the exact baseline, the 16-byte copy: +1 to +3%;
//   float32 inputs (the inverses, float32 HWC), the arithmetic-free widening
//   kernel: -2%; the LUTs gathered from the L2: -4%; the CHW plane kernels,
//   the backward pass, the LUTs in LDS: within +-0.4%.
// Only the first group uses these stores; the others keep the builtin.
//
// The compiler exposes the cache-policy operand on the buffer instructions,
// so the stores are raw buffer stores through a resource over [base, base +
// bytes); the hardware drops a store past `bytes`.  base and bytes must be
// the same in every lane (the resource lives in scalar registers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mact {

typedef float stream_f4 __attribute__((ext_vector_type(4)));
typedef float stream_f2 __attribute__((ext_vector_type(2)));
typedef unsigned stream_u4 __attribute__((ext_vector_type(4)));
typedef unsigned stream_u2 __attribute__((ext_vector_type(2)));

constexpr int kStreamPolicy = 2 | 16;          // NT | SC1 in the buffer instructions' cache-policy operand
constexpr int kRawBufferWord3 = 0x00020000;    // resource word 3: 32-bit data format, no swizzle, no index

typedef __amdgpu_buffer_rsrc_t StreamBuf;

// A resource over [base, base + bytes), base and bytes uniform (kernel arguments
// and values computed from them and blockIdx).
__device__ __forceinline__ StreamBuf stream_buf(void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, kRawBufferWord3);
}

// The same for a wave's own output run, whose base the lanes compute from their
// thread index (equal in every lane by construction): taken from the first
// active lane.
__device__ __forceinline__ StreamBuf wave_stream_buf(void* base, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return stream_buf(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), __builtin_amdgcn_readfirstlane(bytes));
}

// One 16- or 8-byte store at byte offset `off` of the resource.
__device__ __forceinline__ void stream_store(StreamBuf b, uint32_t off, stream_f4 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(stream_u4, v), b, (int)off, 0, kStreamPolicy);
}
__device__ __forceinline__ void stream_store(StreamBuf b, uint32_t off, stream_f2 v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(stream_u2, v), b, (int)off, 0, kStreamPolicy);
}

}  // namespace mact
