// Per-pixel MACT transforms (Sec. 3.2-3.4) for the shapes the 4-pixel kernels
// of xform.hip do not take: inputs of HWC rows whose width is not a multiple
// of 4 or whose strides are not whole 4-pixel groups (crops, pitched rows), CHW
// planes of W H not a multiple of 4, misaligned input pointers, into packed
// float32 or float16 HWC or CHW; and any input into float32 or float16 output
// views that are not packed (a crop of a larger canvas, padded rows or planes).
// The catch-all k_generic reads the element type, the transform and the output
// type at run time and computes every address from the descriptors; here those
// are template parameters, and packed HWC output leaves the way the hot
// kernel's does.
//
// A wave takes 256 consecutive pixels of the launch (image after image); lane
// l takes pixels l, l + 64, l + 128 and l + 192, so that the 64 lanes of one
// load read neighbouring pixels.  The input's layout and strides come from its
// descriptor (branches uniform over the launch).  HWC output goes through the
// wave's LDS slice and leaves as 16-byte (float16: 8-byte) stores, each
// instruction 1 KB (512 B) of contiguous output; CHW output goes through the
// slice as well and leaves as aligned 4-element groups of each plane's run.
// Output views leave from the lanes: a pixel's three values as one 12-byte
// store (float16: three 2-byte stores), contiguous across the wave along a
// row, or one store per plane for CHW.
// The per-pixel code is pixel.h's, so the results are the other kernels' bits.
#include <algorithm>

#include "launch.h"

namespace mact {

#include "gamma_table.inc"

typedef float g_f4 __attribute__((ext_vector_type(4)));
typedef float g_f2 __attribute__((ext_vector_type(2)));
typedef float g_f3 __attribute__((ext_vector_type(3))) __attribute__((aligned(4)));  // 12 bytes, 4-aligned

// Pixel p of `im` as load_px returns it (codes as integer-valued floats, float
// inputs clamped to [0, 1]), its element type fixed at compile time.
template <int IN>
__device__ __forceinline__ void load_px_t(const KImage& im, uint32_t p, float v[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t o = elem_off(im, p, c);
    if (IN == MACT_U8) v[c] = (float)static_cast<const uint8_t*>(im.ptr)[o];
    else if (IN == MACT_U16) v[c] = (float)static_cast<const uint16_t*>(im.ptr)[o];
    else if (IN == MACT_F16) v[c] = clamp01(__half2float(static_cast<const __half*>(im.ptr)[o]));
    else v[c] = clamp01(static_cast<const float*>(im.ptr)[o]);
  }
}

// Stages `bytes` bytes starting at `src` (any alignment) in LDS at `dst`, one
// dword per lane and step (MAXQ steps at most); returns sh, the byte at src + i
// then sitting at byte sh + i of dst.  Only whole aligned dwords are loaded,
// each holding at least one byte of the run; an aligned dword never straddles a
// page, so no load leaves the pages the run lies in.
template <int MAXQ>
__device__ __forceinline__ uint32_t stage_run(const void* src, uint32_t bytes, uint32_t* dst, uint32_t lane) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(src);
  const uint32_t sh = (uint32_t)(a & 3u);
  const uint32_t* d = reinterpret_cast<const uint32_t*>(a - sh);
  const uint32_t n = (sh + bytes + 3u) >> 2;
  uint32_t w[MAXQ];
#pragma unroll
  for (int q = 0; q < MAXQ; ++q)
    if (lane + 64u * q < n) w[q] = d[lane + 64u * q];
#pragma unroll
  for (int q = 0; q < MAXQ; ++q)
    if (lane + 64u * q < n) dst[lane + 64u * q] = w[q];
  return sh;
}

// Pixel r of one image whose first element is `base` (the image's place in
// `im`), as load_px_t returns it.  A chunk inside one image takes its base
// once, uniform over the wave, so a lane's address is its pixel's offset in
// the image: one division by the row width for row-strided inputs, none for
// packed ones, where load_px_t divides by the image size and multiplies out
// the strides for every pixel.
template <int IN>
__device__ __forceinline__ void load_in_image(const KImage& im, const void* base, uint32_t r, float v[3]) {
  int64_t o, step;
  if (im.packed) {
    o = im.layout == MACT_HWC ? 3 * (int64_t)r : (int64_t)r;
  } else {
    const uint32_t y = im.div_w.div(r), x = r - y * im.W;
    o = (int64_t)y * im.rs + (im.layout == MACT_HWC ? 3 * (int64_t)x : (int64_t)x);
  }
  step = im.layout == MACT_HWC ? 1 : im.ps;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t e = o + c * step;
    if (IN == MACT_U8) v[c] = (float)static_cast<const uint8_t*>(base)[e];
    else if (IN == MACT_U16) v[c] = (float)static_cast<const uint16_t*>(base)[e];
    else if (IN == MACT_F16) v[c] = clamp01(__half2float(static_cast<const __half*>(base)[e]));
    else v[c] = clamp01(static_cast<const float*>(base)[e]);
  }
}

// Element e of packed output, float16 rounded to nearest even (channel c of
// pixel p, pixel r of image n: HWC e = 3 p + c, CHW e = (3 n + c) hw + r).
template <int OUT>
__device__ __forceinline__ void put(void* out, size_t e, float x) {
  if (OUT == MACT_F32) static_cast<float*>(out)[e] = x;
  else static_cast<__half*>(out)[e] = f2h_rn(x);
}

// Pixel r of one image of the output view `im`, whose first element is `base`:
// its three values, non-temporal.  HWC float32 as one 12-byte store.
template <int OUT>
__device__ __forceinline__ void put_in_image(const KImage& im, void* base, uint32_t r, const float v[3]) {
  int64_t o;
  if (im.packed) {
    o = im.layout == MACT_HWC ? 3 * (int64_t)r : (int64_t)r;
  } else {
    const uint32_t y = im.div_w.div(r), x = r - y * im.W;
    o = (int64_t)y * im.rs + (im.layout == MACT_HWC ? 3 * (int64_t)x : (int64_t)x);
  }
  if (OUT == MACT_F32 && im.layout == MACT_HWC) {
    __builtin_nontemporal_store(g_f3{v[0], v[1], v[2]}, reinterpret_cast<g_f3*>(static_cast<float*>(base) + o));
    return;
  }
  const int64_t step = im.layout == MACT_HWC ? 1 : im.ps;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (OUT == MACT_F32)
      __builtin_nontemporal_store(v[c], static_cast<float*>(base) + o + c * step);
    else
      __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, f2h_rn(v[c])), static_cast<uint16_t*>(base) + o + c * step);
  }
}

// A wave's three plane runs of 256 outputs (pixel lane + 64 j of o[j]), run
// ch starting at run[ch], any element alignment.  In the slice, value k of
// run ch sits at 260 ch + sh + k (sh: the run's start in elements past a
// 16-byte, float16 8-byte, boundary), so that the run's 4-element groups,
// aligned in the output, are aligned in LDS too.  A run covers groups 0..63
// whole when sh = 0, else groups 1..63 whole and sh elements of a 65th: lane
// l stores group l with one 16-byte (8-byte) store, except lane 0 when sh !=
// 0, which then stores the run's first 4 - sh and last sh elements one by
// one, also non-temporal.  (Those element stores issued first, as plain
// stores, cost the packed CHW path 25%; the groups taken in a loop of one or
// two passes, both branches in each, 7%.)
template <int OUT>
__device__ __forceinline__ void store_plane_runs(g_f4* slice, uint32_t lane, const float o[4][3], void* const run[3]) {
  constexpr uintptr_t ES = OUT == MACT_F32 ? 4 : 2;
  uint32_t sh[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) sh[ch] = (uint32_t)((reinterpret_cast<uintptr_t>(run[ch]) / ES) & 3u);
  __builtin_amdgcn_s_waitcnt(0xc07f);  // whatever the slice held before has been read
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const uint32_t i = 260u * ch + sh[ch] + lane + 64u * j;
      if (OUT == MACT_F32) reinterpret_cast<float*>(slice)[i] = o[j][ch];
      else reinterpret_cast<__half*>(slice)[i] = f2h_rn(o[j][ch]);
    }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    const uint32_t lo = 260u * ch;  // group 0 in the slice
    if (OUT == MACT_F32) {
      float* a0 = static_cast<float*>(run[ch]) - sh[ch];  // group 0 in the output
      const float* sl = reinterpret_cast<const float*>(slice) + lo;
      if (lane != 0 || sh[ch] == 0)
        __builtin_nontemporal_store(*reinterpret_cast<const g_f4*>(sl + 4 * lane), reinterpret_cast<g_f4*>(a0 + 4 * lane));
      __builtin_amdgcn_sched_barrier(0);
      if (lane == 0 && sh[ch] != 0) {
#pragma unroll
        for (uint32_t t = 0; t < 4u; ++t) {
          const uint32_t i = t >= sh[ch] ? t : 256u + t;  // the head's elements of group 0, the tail's of group 64
          __builtin_nontemporal_store(sl[i], a0 + i);
        }
      }
    } else {
      __half* a0 = static_cast<__half*>(run[ch]) - sh[ch];
      const __half* sl = reinterpret_cast<const __half*>(slice) + lo;
      if (lane != 0 || sh[ch] == 0)
        __builtin_nontemporal_store(*reinterpret_cast<const g_f2*>(sl + 4 * lane), reinterpret_cast<g_f2*>(a0 + 4 * lane));
      __builtin_amdgcn_sched_barrier(0);
      if (lane == 0 && sh[ch] != 0) {
#pragma unroll
        for (uint32_t t = 0; t < 4u; ++t) {
          const uint32_t i = t >= sh[ch] ? t : 256u + t;
          __builtin_nontemporal_store(reinterpret_cast<const uint16_t*>(sl)[i], reinterpret_cast<uint16_t*>(a0) + i);
        }
      }
    }
  }
}

// A wave's 256 pixels (pixel lane + 64 j of o[j]) as one run of 768 values
// starting at `run` (any element alignment), HWC order.  In the slice, value
// k sits at sh + k (sh: the run's start in elements past a 16-byte, float16
// 8-byte, boundary), so that the run's aligned 4-value groups are aligned in
// LDS too: lanes store groups 0..191 whole (1..191 when sh != 0) with 16-byte
// (8-byte) stores, then lane 0 the run's first 4 - sh and last sh values one
// by one (store_plane_runs' scheme).
template <int OUT>
__device__ __forceinline__ void store_row_run(g_f4* slice, uint32_t lane, const float o[4][3], void* run) {
  constexpr uintptr_t ES = OUT == MACT_F32 ? 4 : 2;
  const uint32_t sh = (uint32_t)((reinterpret_cast<uintptr_t>(run) / ES) & 3u);
  __builtin_amdgcn_s_waitcnt(0xc07f);  // whatever the slice held before has been read
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const uint32_t i = sh + 3u * (lane + 64u * j) + ch;
      if (OUT == MACT_F32) reinterpret_cast<float*>(slice)[i] = o[j][ch];
      else reinterpret_cast<__half*>(slice)[i] = f2h_rn(o[j][ch]);
    }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  if (OUT == MACT_F32) {
    float* a0 = static_cast<float*>(run) - sh;
    const float* sf = reinterpret_cast<const float*>(slice);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const uint32_t g = 64u * q + lane;
      if (g != 0u || sh == 0u)
        __builtin_nontemporal_store(*reinterpret_cast<const g_f4*>(sf + 4u * g), reinterpret_cast<g_f4*>(a0 + 4u * g));
    }
    __builtin_amdgcn_sched_barrier(0);
    if (lane == 0 && sh != 0) {
#pragma unroll
      for (uint32_t t = 0; t < 4u; ++t) {
        const uint32_t i = t >= sh ? t : 768u + t;
        __builtin_nontemporal_store(sf[i], a0 + i);
      }
    }
  } else {
    __half* a0 = static_cast<__half*>(run) - sh;
    const __half* sf = reinterpret_cast<const __half*>(slice);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const uint32_t g = 64u * q + lane;
      if (g != 0u || sh == 0u)
        __builtin_nontemporal_store(*reinterpret_cast<const g_f2*>(sf + 4u * g), reinterpret_cast<g_f2*>(a0 + 4u * g));
    }
    __builtin_amdgcn_sched_barrier(0);
    if (lane == 0 && sh != 0) {
#pragma unroll
      for (uint32_t t = 0; t < 4u; ++t) {
        const uint32_t i = t >= sh ? t : 768u + t;
        __builtin_nontemporal_store(reinterpret_cast<const uint16_t*>(sf)[i], reinterpret_cast<uint16_t*>(a0) + i);
      }
    }
  }
}

// OM: kGatherHWC and kGatherCHW write packed output at `out`; kGatherAny writes
// the output view `dst` (float32 or float16, any layout and strides).
template <int IN, int OUT, int XF, int DEG, int OM>
__global__ __launch_bounds__(256) void k_gather(KImage src, void* __restrict__ out, uint32_t n_px, uint32_t hw,
                                                FastDiv div_hw, KCoef k, int gamma, KImage dst) {
  constexpr bool OCHW = OM == kGatherCHW;
  __shared__ float gtab[256];
  // per wave: 256 pixels of float32 HWC (3 KB; float16 1.5 KB), or 3 planes of 260 elements (CHW)
  // (output views: the chunk's packed HWC input, up to 1.5 KB, then its run of one HWC row, 3 KB,
  // or its three plane runs)
  __shared__ g_f4 s_out[4][OM == kGatherHWC ? 192 : 195];
  if (IN == MACT_U8 && (XF == MACT_LAB || XF == MACT_LUV)) {
    gtab[threadIdx.x] = k_gamma_table[gamma][threadIdx.x];
    __syncthreads();
  }
  pin_lead<DEG>(k);
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t n_chunks = n_px >> 8;
  const uint32_t c = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + wv);
  if (c < n_chunks) {
    const uint32_t p0 = 256u * c, n0 = div_hw.div(p0);
    const bool one = div_hw.div(p0 + 255u) == n0;  // the chunk inside one image
    const uint32_t r0 = p0 - n0 * hw;              // its first pixel in that image
    float o[4][3];
    constexpr int ES = IN == MACT_U8 ? 1 : IN == MACT_F32 ? 4 : 2;
    if (OM == kGatherAny && IN != MACT_F32 && src.packed && src.layout == MACT_HWC &&
        (reinterpret_cast<uintptr_t>(src.ptr) & 3u) == 0) {
      // packed 8- or 16-bit HWC input into an output view: the chunk's 768 or 1536 bytes come in
      // as 12-byte words, lane-contiguous, through the wave's slice
      constexpr int WPC = IN == MACT_U8 ? 1 : 2;
      const uint3* w = reinterpret_cast<const uint3*>(src.ptr) + (size_t)c * 64u * WPC;
      uint3* s3 = reinterpret_cast<uint3*>(s_out[wv]);
#pragma unroll
      for (int q = 0; q < WPC; ++q) s3[q * 64 + lane] = w[q * 64 + lane];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the chunk is in LDS
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t e = 3u * (lane + 64u * j);
        float v[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          if (IN == MACT_U8) v[ch] = (float)reinterpret_cast<const uint8_t*>(s3)[e + ch];
          else if (IN == MACT_U16) v[ch] = (float)reinterpret_cast<const uint16_t*>(s3)[e + ch];
          else v[ch] = clamp01(__half2float(reinterpret_cast<const __half*>(s3)[e + ch]));
        }
        px1<IN, XF, DEG>(k, gamma, gtab, v, o[j]);
      }
    } else {
      // 8- and 16-bit inputs whose chunk is one contiguous run (HWC: packed, or inside one row;
      // CHW: each plane, packed or inside one row): the runs come in through the wave's slice as
      // lane-contiguous dwords (element loads of 1 or 2 bytes would issue 3 loads a pixel)
      uint32_t y0s = 0, x0s = r0;
      if (IN != MACT_F32 && one && !src.packed) {
        y0s = src.div_w.div(r0);
        x0s = r0 - y0s * src.W;
      }
      // (16-bit inputs: element-aligned, so that the staged halfwords are aligned in LDS)
      const bool runs = IN != MACT_F32 && one && (src.packed || x0s + 256u <= src.W) &&
                        (IN == MACT_U8 || (reinterpret_cast<uintptr_t>(src.ptr) & 1u) == 0);
      if (runs) {
        const char* ib = static_cast<const char*>(src.ptr) + (int64_t)n0 * src.bs * ES;
        const int64_t off = src.packed ? (int64_t)r0 : (int64_t)y0s * src.rs + (src.layout == MACT_HWC ? 3 : 1) * (int64_t)x0s;
        uint32_t* sd = reinterpret_cast<uint32_t*>(s_out[wv]);
        uint32_t sh[3];
        constexpr uint32_t PLANE = (256u * ES + 4u) / 4u;  // dwords per staged plane run
        if (src.layout == MACT_HWC) {
          sh[0] = stage_run<IN == MACT_U8 ? 4 : 7>(ib + (src.packed ? 3 * off : off) * ES, 768u * ES, sd, lane);
        } else {
#pragma unroll
          for (int ch = 0; ch < 3; ++ch)
            sh[ch] = stage_run<IN == MACT_U8 ? 2 : 3>(ib + (off + ch * src.ps) * ES, 256u * ES, sd + PLANE * ch, lane);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the runs are in LDS
        __builtin_amdgcn_wave_barrier();
        const uint8_t* sb = reinterpret_cast<const uint8_t*>(sd);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t px = lane + 64u * j;
          float v[3];
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            const uint32_t b = src.layout == MACT_HWC ? sh[0] + (3u * px + ch) * ES : 4u * PLANE * ch + sh[ch] + px * ES;
            if (IN == MACT_U8) v[ch] = (float)sb[b];
            else if (IN == MACT_U16) v[ch] = (float)*reinterpret_cast<const uint16_t*>(sb + b);
            else v[ch] = clamp01(__half2float(*reinterpret_cast<const __half*>(sb + b)));
          }
          px1<IN, XF, DEG>(k, gamma, gtab, v, o[j]);
        }
        // every lane has read its bytes before any output is staged in the slice
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
      } else if (one) {
        const void* base = static_cast<const char*>(src.ptr) + (int64_t)n0 * src.bs * ES;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float v[3];
          load_in_image<IN>(src, base, r0 + lane + 64u * j, v);
          px1<IN, XF, DEG>(k, gamma, gtab, v, o[j]);
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float v[3];
          load_px_t<IN>(src, p0 + lane + 64u * j, v);
          px1<IN, XF, DEG>(k, gamma, gtab, v, o[j]);
        }
      }
    }
    if (OM == kGatherAny) {
      if (one) {
        constexpr int OES = OUT == MACT_F32 ? 4 : 2;
        void* ob = static_cast<char*>(dst.ptr) + (int64_t)n0 * dst.bs * OES;
        const uint32_t y0 = dst.packed ? 0u : dst.div_w.div(r0), x0 = r0 - y0 * dst.W;
        if (dst.layout == MACT_HWC && !dst.packed && x0 + 256u <= dst.W) {
          // the chunk inside one row of an HWC view: its 768 values are one run
          store_row_run<OUT>(s_out[wv], lane, o, static_cast<char*>(ob) + ((int64_t)y0 * dst.rs + 3 * (int64_t)x0) * OES);
        } else if (dst.layout == MACT_CHW && (dst.packed || x0 + 256u <= dst.W)) {
          // the chunk inside one row of a CHW view (or a packed one): each plane's 256 outputs
          // are one run, stored as the packed CHW path stores them
          const int64_t off = dst.packed ? (int64_t)r0 : (int64_t)y0 * dst.rs + x0;
          void* run[3];
#pragma unroll
          for (int ch = 0; ch < 3; ++ch)
            run[ch] = static_cast<char*>(ob) + (off + ch * dst.ps) * OES;
          store_plane_runs<OUT>(s_out[wv], lane, o, run);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) put_in_image<OUT>(dst, ob, r0 + lane + 64u * j, o[j]);
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) put<OUT>(dst.ptr, elem_off(dst, p0 + lane + 64u * j, ch), o[j][ch]);
      }
    } else if (OCHW && one) {
      // the chunk inside one image: each plane's 256 outputs are one run
      const size_t e0 = (size_t)3 * n0 * hw + r0;
      void* run[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const size_t e = e0 + (size_t)ch * hw;
        run[ch] = OUT == MACT_F32 ? (void*)(static_cast<float*>(out) + e) : (void*)(static_cast<__half*>(out) + e);
      }
      store_plane_runs<OUT>(s_out[wv], lane, o, run);
    } else if (OCHW) {
      // the chunk spans two images or more: element by element
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t p = p0 + lane + 64u * j, n = div_hw.div(p);
        const size_t e = (size_t)3 * n * hw + (p - n * hw);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) put<OUT>(out, e + (size_t)ch * hw, o[j][ch]);
      }
    } else {
      // the chunk as packed HWC in the wave's slice, then 3 stores per lane
      if (OUT == MACT_F32) {
        float* sf = reinterpret_cast<float*>(s_out[wv]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) sf[3 * (lane + 64 * j) + ch] = o[j][ch];
      } else {
        __half* sh = reinterpret_cast<__half*>(s_out[wv]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) sh[3 * (lane + 64 * j) + ch] = f2h_rn(o[j][ch]);
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): every lane's LDS writes have landed
      __builtin_amdgcn_wave_barrier();
      if (OUT == MACT_F32) {
        g_f4* d = static_cast<g_f4*>(out) + (size_t)c * 192;
#pragma unroll
        for (int q = 0; q < 3; ++q) __builtin_nontemporal_store(s_out[wv][q * 64 + lane], d + q * 64 + lane);
      } else {
        const g_f2* s2 = reinterpret_cast<const g_f2*>(s_out[wv]);
        g_f2* d = static_cast<g_f2*>(out) + (size_t)c * 192;
#pragma unroll
        for (int q = 0; q < 3; ++q) __builtin_nontemporal_store(s2[q * 64 + lane], d + q * 64 + lane);
      }
    }
  }
  // the last n_px % 256 pixels, one per thread of block 0
  const uint32_t tail0 = n_chunks << 8;
  if (blockIdx.x == 0 && threadIdx.x < n_px - tail0) {
    const uint32_t p = tail0 + threadIdx.x;
    float v[3], r[3];
    load_px_t<IN>(src, p, v);
    px1<IN, XF, DEG>(k, gamma, gtab, v, r);
    if (OM == kGatherAny) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) put<OUT>(dst.ptr, elem_off(dst, p, ch), r[ch]);
    } else {
      const uint32_t n = OCHW ? div_hw.div(p) : 0u;
      const size_t e = OCHW ? (size_t)3 * n * hw + (p - n * hw) : (size_t)3 * p;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) put<OUT>(out, e + (OCHW ? (size_t)ch * hw : (size_t)ch), r[ch]);
    }
  }
}

template <int IN, int OUT, int DEG, int OM>
static void launch_gather_xf(int xform, const KImage& src, const KImage& dst, void* out, uint32_t n_px, uint32_t hw,
                             const KCoef& k, int gamma, hipStream_t st) {
  const uint32_t blocks = std::max<uint32_t>(1, ((n_px >> 8) + 3) / 4);
  const FastDiv d = make_fastdiv(hw);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_gather<IN, OUT, MACT_LAB, DEG, OM>), dim3(blocks), dim3(256), 0, st, src, out, n_px, hw, d, k, gamma, dst);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_gather<IN, OUT, MACT_HSI, DEG, OM>), dim3(blocks), dim3(256), 0, st, src, out, n_px, hw, d, k, gamma, dst);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_gather<IN, OUT, MACT_LUV, DEG, OM>), dim3(blocks), dim3(256), 0, st, src, out, n_px, hw, d, k, gamma, dst);
  else hipLaunchKernelGGL((k_gather<IN, OUT, MACT_SCT, DEG, OM>), dim3(blocks), dim3(256), 0, st, src, out, n_px, hw, d, k, gamma, dst);
}

// The polynomials at their own degree (up to 4, 5, or up to 7), as the 4-pixel
// kernels evaluate them: a zero leading coefficient leaves Horner's sums unchanged.
template <int IN, int OUT, int OM>
static void launch_gather_deg(int xform, int deg, const KImage& src, const KImage& dst, void* out, uint32_t n_px,
                              uint32_t hw, const KCoef& k, int gamma, hipStream_t st) {
  if (deg <= 4) launch_gather_xf<IN, OUT, 4, OM>(xform, src, dst, out, n_px, hw, k, gamma, st);
  else if (deg == 5) launch_gather_xf<IN, OUT, 5, OM>(xform, src, dst, out, n_px, hw, k, gamma, st);
  else launch_gather_xf<IN, OUT, 7, OM>(xform, src, dst, out, n_px, hw, k, gamma, st);
}

template <int IN, int OUT>
static void launch_gather_om(int xform, int out_mode, int deg, const KImage& src, const KImage& dst, void* out,
                             uint32_t n_px, uint32_t hw, const KCoef& k, int gamma, hipStream_t st) {
  if (out_mode == kGatherHWC) launch_gather_deg<IN, OUT, kGatherHWC>(xform, deg, src, dst, out, n_px, hw, k, gamma, st);
  else if (out_mode == kGatherCHW) launch_gather_deg<IN, OUT, kGatherCHW>(xform, deg, src, dst, out, n_px, hw, k, gamma, st);
  else launch_gather_deg<IN, OUT, kGatherAny>(xform, deg, src, dst, out, n_px, hw, k, gamma, st);
}

template <int IN>
static void launch_gather_in(int xform, int out_dtype, int out_mode, int deg, const KImage& src, const KImage& dst,
                             void* out, uint32_t n_px, uint32_t hw, const KCoef& k, int gamma, hipStream_t st) {
  if (out_dtype == MACT_F32) launch_gather_om<IN, MACT_F32>(xform, out_mode, deg, src, dst, out, n_px, hw, k, gamma, st);
  else launch_gather_om<IN, MACT_F16>(xform, out_mode, deg, src, dst, out, n_px, hw, k, gamma, st);
}

void launch_gather(int in_dtype, int xform, int out_dtype, int out_mode, int deg, const KImage& src, const KImage& dst,
                   void* out, uint32_t n_px, uint32_t hw, const KCoef& k, int gamma, hipStream_t st) {
  if (in_dtype == MACT_U8) launch_gather_in<MACT_U8>(xform, out_dtype, out_mode, deg, src, dst, out, n_px, hw, k, gamma, st);
  else if (in_dtype == MACT_U16) launch_gather_in<MACT_U16>(xform, out_dtype, out_mode, deg, src, dst, out, n_px, hw, k, gamma, st);
  else if (in_dtype == MACT_F16) launch_gather_in<MACT_F16>(xform, out_dtype, out_mode, deg, src, dst, out, n_px, hw, k, gamma, st);
  else launch_gather_in<MACT_F32>(xform, out_dtype, out_mode, deg, src, dst, out, n_px, hw, k, gamma, st);
}

}  // namespace mact
