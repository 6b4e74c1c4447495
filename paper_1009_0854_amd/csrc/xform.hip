// Plain per-pixel MACT transforms (Sec. 3.2-3.4), the backward pass of the
// CIELAB transform, and the reference streaming kernels.
//
// The kernels:
//  * k_hwc4: the hot path, packed 8-bit, 16-bit or float16 HWC in and packed
//    float32 or float16 HWC out, staged through LDS so that every global
//    store is a contiguous run of 1 KB per wave (details at the kernel).
//  * k_hwc4f: k_hwc4 for packed float32 HWC input, staged through LDS both ways.
//  * k_rows4: row-strided HWC views (crops, pitched rows), k_hwc4's pattern
//    per 256-pixel run of a row.
//  * k_chw_rows4: row-strided CHW views (crops of the planes, gaps between
//    images) -> packed HWC or CHW, one load per plane and lane.
//  * k_chw4: packed CHW of any input type, 4 pixels per lane, vector access
//    per plane.
//  * k_hwc_chw4: packed HWC of any input type -> packed CHW, 4 pixels per
//    lane, no LDS.
//  * k_chw_hwc4: packed CHW of any input type -> packed HWC through the
//    wave's LDS slice.
//  * k_gather (gather.hip): any other input into packed HWC or CHW output.
//  * k_generic: any element type, layout and stride, one pixel per lane step.
// Every kernel but k_generic writes float32 or float16 by template; k_generic
// writes either at run time.
// All call the same per-pixel functions (pixel.h), so they give identical bits.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "launch.h"
#include "planes.h"
#include "stream.h"

namespace mact {

#include "gamma_table.inc"

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- host helpers

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t l = 0;
  while (l < 32 && (1ull << l) < d) ++l;
  f.s = l;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  return f;
}

static size_t elem_size(int dtype) { return dtype == MACT_U8 ? 1 : (dtype == MACT_F16 || dtype == MACT_U16) ? 2 : 4; }

mact_status resolve_image(const mact_image* im, bool is_output, const char* what, HostImage* out) {
  if (!im) return fail(MACT_E_INVALID, "%s: image is NULL", what);
  if (!im->data) return fail(MACT_E_INVALID, "%s: data is NULL", what);
  if (im->dtype < MACT_U8 || im->dtype > MACT_U16) return fail(MACT_E_INVALID, "%s: unknown dtype %d", what, im->dtype);
  if (is_output && (im->dtype == MACT_U8 || im->dtype == MACT_U16))
    return fail(MACT_E_UNSUPPORTED, "%s: integer output is not supported", what);
  if (im->layout != MACT_HWC && im->layout != MACT_CHW) return fail(MACT_E_INVALID, "%s: unknown layout %d", what, im->layout);
  if (im->width <= 0 || im->height <= 0) return fail(MACT_E_INVALID, "%s: size %lld x %lld", what, (long long)im->width, (long long)im->height);
  if (im->batch < 0) return fail(MACT_E_INVALID, "%s: batch %lld < 0", what, (long long)im->batch);
  if (im->gamma < MACT_GAMMA_BT709 || im->gamma > MACT_GAMMA_NONE) return fail(MACT_E_INVALID, "%s: unknown gamma %d", what, im->gamma);
  HostImage h;
  h.data = im->data;
  h.dtype = im->dtype;
  h.layout = im->layout;
  h.gamma = im->gamma;
  h.W = im->width;
  h.H = im->height;
  h.N = im->batch > 1 ? im->batch : 1;
  h.esize = elem_size(im->dtype);
  if ((uint64_t)h.W * (uint64_t)h.H >= (1ull << 31)) return fail(MACT_E_UNSUPPORTED, "%s: image of 2^31 pixels or more", what);
  if (h.layout == MACT_HWC) {
    h.rs = im->row_stride ? im->row_stride : 3 * h.W;
    if (h.rs < 3 * h.W) return fail(MACT_E_INVALID, "%s: row_stride %lld < 3 W", what, (long long)h.rs);
    h.ps = 1;
    h.bs = im->batch_stride ? im->batch_stride : h.H * h.rs;
    if (h.N > 1 && h.bs < h.H * h.rs) return fail(MACT_E_INVALID, "%s: batch_stride too small", what);
    h.packed = h.rs == 3 * h.W && (h.N == 1 || h.bs == h.H * h.rs);
  } else {
    h.rs = im->row_stride ? im->row_stride : h.W;
    if (h.rs < h.W) return fail(MACT_E_INVALID, "%s: row_stride %lld < W", what, (long long)h.rs);
    h.ps = im->plane_stride ? im->plane_stride : h.H * h.rs;
    if (h.ps < h.H * h.rs) return fail(MACT_E_INVALID, "%s: plane_stride too small", what);
    h.bs = im->batch_stride ? im->batch_stride : 3 * h.ps;
    if (h.N > 1 && h.bs < 3 * h.ps) return fail(MACT_E_INVALID, "%s: batch_stride too small", what);
    h.packed = h.rs == h.W && h.ps == h.H * h.W && (h.N == 1 || h.bs == 3 * h.ps);
  }
  if (h.rs < 0 || h.ps < 0 || h.bs < 0) return fail(MACT_E_INVALID, "%s: negative stride", what);
  *out = h;
  return MACT_OK;
}

mact_status check_same_shape(const HostImage& a, const HostImage& b, const char* what) {
  if (a.W != b.W || a.H != b.H || a.N != b.N)
    return fail(MACT_E_INVALID, "%s: shape %lldx%lldx%lld does not match %lldx%lldx%lld", what, (long long)b.N,
                (long long)b.H, (long long)b.W, (long long)a.N, (long long)a.H, (long long)a.W);
  return MACT_OK;
}

KImage kimage(const HostImage& h, int64_t n0, int64_t count) {
  KImage k;
  k.ptr = static_cast<char*>(h.data) + (size_t)(n0 * h.bs) * h.esize;
  k.dtype = h.dtype;
  k.layout = h.layout;
  k.rs = h.rs;
  k.ps = h.ps;
  k.bs = h.bs;
  k.W = (uint32_t)h.W;
  k.HW = (uint32_t)(h.W * h.H);
  k.packed = h.packed ? 1u : 0u;
  k.div_w = make_fastdiv(k.W);
  k.div_hw = make_fastdiv(k.HW);
  (void)count;
  return k;
}

int64_t images_per_launch(const HostImage& h) {
  const int64_t hw = h.W * h.H;
  return std::max<int64_t>(1, ((1ll << 31) - 1) / hw);
}

int64_t images_per_stream_launch(const HostImage& in, const HostImage& out) {
  const int64_t most = images_per_launch(in);
  if (out.dtype != MACT_F32) return most;
  const int64_t hw = in.W * in.H;
  const int64_t launches = (in.N * hw + (1ll << 26) - 1) >> 26;
  int64_t per = std::max<int64_t>(1, std::min<int64_t>(most, (in.N + launches - 1) / launches));
  // every launch after the first starts per images further on: keep that offset a multiple of
  // the coalesced kernels' alignment (input: 4 bytes, 16 for float32 HWC, 4 elements of a CHW
  // plane; output: 16 bytes), rounding the count up, or a launch would fall back to the
  // one-pixel kernel
  const int64_t need_in = in.layout == MACT_CHW ? 4 * (int64_t)in.esize : in.dtype == MACT_F32 ? 16 : 4;
  const int64_t in_bytes = in.bs * (int64_t)in.esize, out_bytes = out.bs * (int64_t)out.esize;
  for (int64_t q = 1; q <= 16; q *= 2) {
    if ((q * in_bytes) % need_in == 0 && (q * out_bytes) % 16 == 0) {
      const int64_t up = (per + q - 1) / q * q;
      if (up <= most) per = up;
      break;
    }
  }
  return per;
}

int pack_coef(const mact_params& p, KCoef* k, int* exact) {
  std::memset(k, 0, sizeof *k);
  k->xform = p.xform;
  k->out_mode = p.out_mode;
  k->lab_c = kLabCf;
  const int nf = p.xform == MACT_SCT ? 4 : 1;
  int deg = 0;
  for (int i = 0; i < nf; ++i) {
    for (int j = 0; j <= p.f[i].n; ++j) k->p[i][j] = (float)p.f[i].p[j];
    deg = std::max(deg, p.f[i].n);
  }
  if (uses_gamma(p.xform) && p.f[0].m > 0) {
    for (int j = 0; j <= p.f[0].m; ++j) k->q[j] = (float)p.f[0].q[j];
    deg = std::max(deg, p.f[0].m);
  } else {
    k->q[0] = 1.0f;
  }
  if (uses_gamma(p.xform) && p.f[1].fn == MACT_FN_DEC709) {
    // the decoding polynomial has its own fixed evaluation degree (7): it does not raise `deg`
    for (int j = 0; j <= p.f[1].n; ++j) k->p[1][j] = (float)p.f[1].p[j];
    k->decode = 1;
  }
  if (exact) *exact = deg;
  return deg <= 5 ? 5 : 7;
}

int current_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

int device_cus() {
  static std::mutex mu;
  static int cache[64] = {0};
  const int d = current_device();
  std::lock_guard<std::mutex> g(mu);
  if (d >= 0 && d < 64 && cache[d]) return cache[d];
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess || cus <= 0) cus = 256;
  if (d >= 0 && d < 64) cache[d] = cus;
  return cus;
}

// One work item per thread: the grid covers the work once.  Streaming kernels
// run 4-26% faster this way than with a few resident workgroups per CU
// striding over the work.
static unsigned full_grid(uint64_t work_items, int block) {
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((work_items + block - 1) / block, 0x7fffffffu));
}

// ---------------------------------------------------------------- kernels

// Packed HWC (8-bit or float16) -> packed HWC float32 (or float16): the hot
// path.
//
// A wave owns chunks of 256 pixels (768 input bytes for 8-bit input, 1536
// for float16; 3 KB of float32 output, 1.5 KB of float16).  Each lane loads
// its 4 pixels (one 12-byte load, or two for float16) -- the wave's loads
// cover one contiguous run -- and computes them.  The 48 bytes of results
// (24 for float16, rounded to nearest even) go to the wave's slice of LDS,
// and the wave then writes its chunks back as 16-byte stores in which lane l
// writes bytes 16 l .. 16 l + 15 of each KB: every store instruction covers
// 1 KB of contiguous output.  Writing the results straight from the lane (a
// 48-byte stride across the wave) runs at about a third of this bandwidth.
// Each wave handles hot_cpw(IN, OUT, XF) chunks and the grid covers the image
// once (no grid-stride loop).  Two chunks per wave keep two loads in flight per
// lane.  CIELUV from 8-bit input to float32 takes one: its single rational and
// reciprocal form one long dependent chain per pixel, and with a 12 KB
// transpose buffer per workgroup the CU holds 8 workgroups instead of 6 (12%
// faster measured; the same change made CIELAB 3% and the float16-input forms
// 30% slower).  Requires `in` 4-byte and `out` 16-byte aligned; blockDim.x ==
// kHotBlock.
constexpr int kHotBlock = 256;
constexpr int kChunksPerWave = 2;
constexpr int kHotWaves = kHotBlock / 64;
constexpr int hot_cpw(int in, int out, int xf) {
  return (xf == MACT_LUV && in == MACT_U8 && out == MACT_F32) ? 1 : kChunksPerWave;
}

template <int IN, int OUT, int DEG, int XF>
__global__ __launch_bounds__(kHotBlock) void k_hwc4(const void* __restrict__ in, void* __restrict__ out,
                                                     uint32_t n_px, KCoef k, int gamma) {
  constexpr int WPC = IN == MACT_U8 ? 1 : 2;      // 12-byte words per lane per chunk (16-bit inputs: 2)
  constexpr uint32_t F4PC = OUT == MACT_F32 ? 192 : 96;  // 16-byte output words per chunk
  constexpr int CPW = hot_cpw(IN, OUT, XF);
  __shared__ f4 s_out[kHotWaves][CPW * F4PC];
  __shared__ float gtab[256];
  if (IN == MACT_U8 && (XF == MACT_LAB || XF == MACT_LUV)) {
    for (uint32_t i = threadIdx.x; i < 256u; i += kHotBlock) gtab[i] = k_gamma_table[gamma][i];
    __syncthreads();
  }
  pin_lead<DEG>(k);
  const uint3* win = reinterpret_cast<const uint3*>(in);
  const uint32_t n_chunks = n_px >> 8;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t c0 = (blockIdx.x * kHotWaves + wv) * CPW;
  if (c0 < n_chunks) {
    uint3 w[CPW][WPC];
#pragma unroll
    for (int j = 0; j < CPW; ++j)
      if (c0 + j < n_chunks)
#pragma unroll
        for (int q = 0; q < WPC; ++q) w[j][q] = win[((size_t)(c0 + j) * 64 + lane) * WPC + q];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      if (c0 + j >= n_chunks) break;
      float o[12];
      if (IN == MACT_U8) px4_u8<XF, DEG>(k, gtab, w[j][0], o);
      else if (IN == MACT_U16) px4_u16<XF, DEG>(k, gamma, w[j][0], w[j][WPC - 1], o);
      else px4_f16<XF, DEG>(k, gamma, w[j][0], w[j][WPC - 1], o);
      if (OUT == MACT_F32) {
        s_out[wv][j * 192 + 3 * lane] = f4{o[0], o[1], o[2], o[3]};
        s_out[wv][j * 192 + 3 * lane + 1] = f4{o[4], o[5], o[6], o[7]};
        s_out[wv][j * 192 + 3 * lane + 2] = f4{o[8], o[9], o[10], o[11]};
      } else {
        // 12 halves = three 8-byte words; chunk j starts at 8-byte word 192 j
        f2* s2 = reinterpret_cast<f2*>(&s_out[wv][0]);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const uint32_t lo = pack2_h_rn(o[4 * t], o[4 * t + 1]);
          const uint32_t hi = pack2_h_rn(o[4 * t + 2], o[4 * t + 3]);
          s2[j * 192 + 3 * lane + t] = f2{__uint_as_float(lo), __uint_as_float(hi)};
        }
      }
    }
    // the LDS writes of every lane must land before any lane reads them back
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    const uint32_t n_valid = min((uint32_t)CPW, n_chunks - c0) * F4PC;
    const StreamBuf dst = wave_stream_buf(reinterpret_cast<f4*>(out) + (size_t)c0 * F4PC, n_valid * 16u);
    static_assert((CPW * F4PC) % 64 == 0, "whole 1 KB stores per wave");
#pragma unroll
    for (int q = 0; q < (int)(CPW * F4PC / 64); ++q) {
      const uint32_t e = q * 64 + lane;
      if (e < n_valid) stream_store(dst, e * 16u, s_out[wv][e]);
    }
  }
  // the last n_px % 256 pixels, one per lane of block 0
  const uint32_t tail0 = n_chunks << 8;
  if (blockIdx.x == 0 && threadIdx.x < n_px - tail0) {
    const size_t p = tail0 + threadIdx.x;
    float o[3];
    if (IN == MACT_U8) {
      const uint8_t* b8 = static_cast<const uint8_t*>(in);
      const uint32_t r = b8[3 * p], g = b8[3 * p + 1], b = b8[3 * p + 2];
      if (XF == MACT_LAB) lab_px<DEG>(k, gtab[r], gtab[g], gtab[b], o);
      else if (XF == MACT_LUV) luv_px<DEG>(k, gtab[r], gtab[g], gtab[b], o);
      else if (XF == MACT_HSI) hsi_px<DEG>(k, (float)r, (float)g, (float)b, kInv765, o);
      else sct_px<DEG, false>(k, (float)r, (float)g, (float)b, kInv255, o);
    } else if (IN == MACT_U16) {
      const uint16_t* c16 = static_cast<const uint16_t*>(in);
      const float r = (float)c16[3 * p], g = (float)c16[3 * p + 1], b = (float)c16[3 * p + 2];
      if (XF == MACT_LAB || XF == MACT_LUV) {
        const float lr = lin_float(k, r * kInv65535, gamma), lg = lin_float(k, g * kInv65535, gamma),
                    lb = lin_float(k, b * kInv65535, gamma);
        if (XF == MACT_LAB) lab_px<DEG>(k, lr, lg, lb, o);
        else luv_px<DEG>(k, lr, lg, lb, o);
      } else if (XF == MACT_HSI) {
        hsi_px<DEG>(k, r, g, b, kInv196605, o);
      } else {
        sct_px<DEG, false>(k, r, g, b, kInv65535, o);
      }
    } else {
      const __half* h = static_cast<const __half*>(in);
      const float r = clamp01(__half2float(h[3 * p])), g = clamp01(__half2float(h[3 * p + 1])),
                  b = clamp01(__half2float(h[3 * p + 2]));
      if (XF == MACT_LAB) lab_px<DEG>(k, lin_float(k, r, gamma), lin_float(k, g, gamma), lin_float(k, b, gamma), o);
      else if (XF == MACT_LUV) luv_px<DEG>(k, lin_float(k, r, gamma), lin_float(k, g, gamma), lin_float(k, b, gamma), o);
      else if (XF == MACT_HSI) hsi_px<DEG>(k, r, g, b, kInv3, o);
      else sct_px<DEG, false>(k, r, g, b, 1.0f, o);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (OUT == MACT_F32) static_cast<float*>(out)[3 * p + c] = o[c];
      else static_cast<__half*>(out)[3 * p + c] = f2h_rn(o[c]);
    }
  }
}

// Packed float32 HWC -> packed float32 / float16 HWC: k_hwc4 for 12-byte
// pixels.  A chunk's 3 KB of input come in as three coalesced 1 KB loads into
// the wave's LDS slice; each lane reads its 4 pixels (48 bytes) back from
// there, and the results leave through the same slice as in k_hwc4.  One chunk
// per wave: a 12 KB buffer per workgroup, 8 workgroups per CU (two chunks per
// wave measured 5.5 TB/s, the one-chunk inverse kernel of the same pattern
// 5.8).  Requires `in` and `out` 16-byte aligned; blockDim.x == kHotBlock.
constexpr int kF32Cpw = 1;

template <int OUT, int DEG, int XF>
__global__ __launch_bounds__(kHotBlock) void k_hwc4f(const f4* __restrict__ in, void* __restrict__ out,
                                                      uint32_t n_px, KCoef k, int gamma) {
  constexpr uint32_t F4PC = OUT == MACT_F32 ? 192 : 96;  // 16-byte output words per chunk
  constexpr int CPW = kF32Cpw;
  __shared__ f4 s_buf[kHotWaves][CPW * 192];
  pin_lead<DEG>(k);
  const uint32_t n_chunks = n_px >> 8;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t c0 = (blockIdx.x * kHotWaves + wv) * CPW;
  if (c0 < n_chunks) {
    const uint32_t nc = min((uint32_t)CPW, n_chunks - c0);
    f4 a[CPW][3];
#pragma unroll
    for (int j = 0; j < CPW; ++j)
      if ((uint32_t)j < nc)
#pragma unroll
        for (int q = 0; q < 3; ++q) a[j][q] = in[(size_t)(c0 + j) * 192 + q * 64 + lane];
#pragma unroll
    for (int j = 0; j < CPW; ++j)
      if ((uint32_t)j < nc)
#pragma unroll
        for (int q = 0; q < 3; ++q) s_buf[wv][j * 192 + q * 64 + lane] = a[j][q];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the chunks are in LDS
    __builtin_amdgcn_wave_barrier();
    float v[CPW][12];
#pragma unroll
    for (int j = 0; j < CPW; ++j)
      if ((uint32_t)j < nc) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const f4 b = s_buf[wv][j * 192 + 3 * lane + t];
          v[j][4 * t] = b.x; v[j][4 * t + 1] = b.y; v[j][4 * t + 2] = b.z; v[j][4 * t + 3] = b.w;
        }
      }
    __builtin_amdgcn_s_waitcnt(0xc07f);  // every lane's reads are done before the slice is rewritten
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      if ((uint32_t)j >= nc) break;
      float o[12];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float raw[3] = {clamp01(v[j][3 * i]), clamp01(v[j][3 * i + 1]), clamp01(v[j][3 * i + 2])};
        px1<MACT_F32, XF, DEG>(k, gamma, nullptr, raw, o + 3 * i);
      }
      if (OUT == MACT_F32) {
        s_buf[wv][j * 192 + 3 * lane] = f4{o[0], o[1], o[2], o[3]};
        s_buf[wv][j * 192 + 3 * lane + 1] = f4{o[4], o[5], o[6], o[7]};
        s_buf[wv][j * 192 + 3 * lane + 2] = f4{o[8], o[9], o[10], o[11]};
      } else {
        f2* s2 = reinterpret_cast<f2*>(&s_buf[wv][0]);  // chunk j's halves start at 8-byte word 192 j
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const uint32_t lo = pack2_h_rn(o[4 * t], o[4 * t + 1]);
          const uint32_t hi = pack2_h_rn(o[4 * t + 2], o[4 * t + 3]);
          s2[j * 192 + 3 * lane + t] = f2{__uint_as_float(lo), __uint_as_float(hi)};
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    const uint32_t n_valid = nc * F4PC;
    f4* dst = reinterpret_cast<f4*>(out) + (size_t)c0 * F4PC;
#pragma unroll
    for (int q = 0; q < (int)((CPW * F4PC + 63) / 64); ++q) {
      const uint32_t e = q * 64 + lane;
      if (e < n_valid) __builtin_nontemporal_store(s_buf[wv][e], dst + e);
    }
  }
  // the last n_px % 256 pixels, one per lane of block 0
  const uint32_t tail0 = n_chunks << 8;
  if (blockIdx.x == 0 && threadIdx.x < n_px - tail0) {
    const size_t p = tail0 + threadIdx.x;
    const float* fi = reinterpret_cast<const float*>(in);
    const float raw[3] = {clamp01(fi[3 * p]), clamp01(fi[3 * p + 1]), clamp01(fi[3 * p + 2])};
    float o[3];
    px1<MACT_F32, XF, DEG>(k, gamma, nullptr, raw, o);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (OUT == MACT_F32) static_cast<float*>(out)[3 * p + c] = o[c];
      else static_cast<__half*>(out)[3 * p + c] = f2h_rn(o[c]);
    }
  }
}

// Helpers of the kernels below whose output is float32 or float16 (OUT).
//
// stage4: a lane's 4 results (12 values, pixel by pixel) into its wave's LDS
// slice, at 16-byte word 3 lane (float32) or 8-byte word 3 lane (float16,
// rounded to nearest even).
template <int OUT>
__device__ __forceinline__ void stage4(f4* slice, uint32_t lane, const float o[12]) {
  if (OUT == MACT_F32) {
    slice[3 * lane] = f4{o[0], o[1], o[2], o[3]};
    slice[3 * lane + 1] = f4{o[4], o[5], o[6], o[7]};
    slice[3 * lane + 2] = f4{o[8], o[9], o[10], o[11]};
  } else {
    f2* s2 = reinterpret_cast<f2*>(slice);
#pragma unroll
    for (int t = 0; t < 3; ++t)
      s2[3 * lane + t] = f2{__uint_as_float(pack2_h_rn(o[4 * t], o[4 * t + 1])),
                            __uint_as_float(pack2_h_rn(o[4 * t + 2], o[4 * t + 3]))};
  }
}

// store_staged: once every lane has staged, the wave's cnt pixels (a multiple
// of 4, at most 256) from its slice to packed HWC output at dst.  float32
// leaves as 16-byte stores (each instruction 1 KB of contiguous output, dst
// 16-byte aligned), float16 as 8-byte stores (512 B per instruction; dst need
// only be 8-byte aligned, which any run of a multiple of 4 pixels keeps).
template <int OUT, int HALVES = 1>
__device__ __forceinline__ void store_staged(const f4* slice, void* dst, uint32_t cnt, uint32_t lane) {
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): every lane's LDS writes have landed
  __builtin_amdgcn_wave_barrier();
  const uint32_t n_valid = cnt / 4u * 3u;  // 16-byte (float32) or 8-byte (float16) words
  constexpr uint32_t WB = OUT == MACT_F32 ? 16 : 8;
  const StreamBuf b = wave_stream_buf(dst, n_valid * WB);
#pragma unroll
  for (int q = 0; q < 3 * HALVES; ++q) {
    const uint32_t e = q * 64 + lane;
    if (e < n_valid) {
      if (OUT == MACT_F32) stream_store(b, e * WB, slice[e]);
      else stream_store(b, e * WB, reinterpret_cast<const f2*>(slice)[e]);
    }
  }
}

// store_plane4: a lane's 4 results of one output plane to packed CHW output at
// element offset e (a multiple of 4): one 16-byte (float32) or 8-byte (float16)
// store, contiguous across the wave.
template <int OUT>
__device__ __forceinline__ void store_plane4(void* out, size_t e, float a, float b, float c, float d) {
  if (OUT == MACT_F32)
    __builtin_nontemporal_store(f4{a, b, c, d}, reinterpret_cast<f4*>(static_cast<float*>(out) + e));
  else
    __builtin_nontemporal_store(f2{__uint_as_float(pack2_h_rn(a, b)), __uint_as_float(pack2_h_rn(c, d))},
                                reinterpret_cast<f2*>(static_cast<__half*>(out) + e));
}

// Row-strided HWC (a view whose rows or images are not adjacent: a crop, a
// pitched allocation) -> packed float32 or float16 HWC, W a multiple of 4.
// Every row is cut into segments of kRowHalves 256-pixel chunks, the last one
// partial, one segment per wave; each chunk takes k_hwc4's 12-byte loads
// (lanes past the row's end idle; float32 pixels: three 16-byte loads per
// lane), both chunks' loads issued first, then its per-pixel code and its
// LDS-transposed stores.  Requires the input pointer and both strides (in
// bytes) to be multiples of 4 (16 for float32) and `out` 16-byte aligned.
constexpr int kRowHalves = 2;
struct RowGeom {
  uint32_t W, cpr, H;      // pixels per row, chunks per row, rows per image
  FastDiv div_cpr, div_h;  // chunk -> row, row -> image
  uint64_t rs_b, bs_b;     // input row and image strides in bytes
};

template <int IN, int OUT, int DEG, int XF>
__global__ __launch_bounds__(kHotBlock) void k_rows4(const uint8_t* __restrict__ in, void* __restrict__ out,
                                                     uint32_t n_chunks, RowGeom g, KCoef k, int gamma) {
  constexpr int WPC = IN == MACT_U8 ? 1 : IN == MACT_F32 ? 4 : 2;  // 12-byte words per lane
  constexpr uint32_t OSZ = OUT == MACT_F32 ? 4 : 2;
  constexpr uint32_t SLICE = 3 * OSZ * 16;                         // one half's output in 16-byte words
  __shared__ f4 s_out[kHotWaves][kRowHalves * SLICE];
  __shared__ float gtab[256];
  if (IN == MACT_U8 && (XF == MACT_LAB || XF == MACT_LUV)) {
    for (uint32_t i = threadIdx.x; i < 256u; i += kHotBlock) gtab[i] = k_gamma_table[gamma][i];
    __syncthreads();
  }
  pin_lead<DEG>(k);
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t c = blockIdx.x * kHotWaves + wv;
  if (c >= n_chunks) return;  // no block-wide barrier follows
  const uint32_t r = g.div_cpr.div(c), j = c - r * g.cpr;
  const uint32_t n = g.div_h.div(r), y = r - n * g.H;
  const uint32_t px0 = j * (256u * kRowHalves), cnt = min(256u * kRowHalves, g.W - px0);  // cnt: a multiple of 4
  const uint8_t* row = in + n * g.bs_b + y * g.rs_b + (uint64_t)px0 * 3u * (IN == MACT_U8 ? 1u : IN == MACT_F32 ? 4u : 2u);
  // both halves' loads first, then each half's pixels
  uint3 w[kRowHalves][WPC];
  f4 wf[kRowHalves][3];
#pragma unroll
  for (int h = 0; h < kRowHalves; ++h) {
    if (256u * h + 4u * lane < cnt) {
      if (IN == MACT_F32) {
        const f4* rf = reinterpret_cast<const f4*>(row) + 192u * h + 3u * lane;  // 48 bytes per lane, 16-byte aligned
#pragma unroll
        for (int t = 0; t < 3; ++t) wf[h][t] = rf[t];
      } else {
        const uint3* rw = reinterpret_cast<const uint3*>(row) + (64u * h + lane) * WPC;
#pragma unroll
        for (int q = 0; q < WPC; ++q) w[h][q] = rw[q];
      }
    }
  }
#pragma unroll
  for (int h = 0; h < kRowHalves; ++h) {
    float o[12];
    if (256u * h + 4u * lane < cnt) {
      if (IN == MACT_F32) {
        float v[12];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          v[4 * t] = clamp01(wf[h][t].x); v[4 * t + 1] = clamp01(wf[h][t].y);
          v[4 * t + 2] = clamp01(wf[h][t].z); v[4 * t + 3] = clamp01(wf[h][t].w);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) px1<MACT_F32, XF, DEG>(k, gamma, gtab, v + 3 * q, o + 3 * q);
      } else if (IN == MACT_U8) {
        px4_u8<XF, DEG>(k, gtab, w[h][0], o);
      } else if (IN == MACT_U16) {
        px4_u16<XF, DEG>(k, gamma, w[h][0], w[h][WPC - 1], o);
      } else {
        px4_f16<XF, DEG>(k, gamma, w[h][0], w[h][WPC - 1], o);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 12; ++q) o[q] = 0.0f;
    }
    stage4<OUT>(s_out[wv] + SLICE * h, lane, o);
  }
  store_staged<OUT, kRowHalves>(s_out[wv], static_cast<char*>(out) + ((uint64_t)r * g.W + px0) * 3u * OSZ, cnt, lane);
}

// Blocks of k_hwc4 for n_px pixels: every full chunk covered once, and at
// least one block for the tail.
static unsigned hot_grid(uint32_t n_px, int cpw = kChunksPerWave) {
  const uint32_t per_block = kHotWaves * cpw;
  return std::max<unsigned>(1, ((n_px >> 8) + per_block - 1) / per_block);
}

// Packed CHW (float32, float16, 16-bit or 8-bit) -> packed float32 or float16
// CHW, 4 pixels per lane: one 16-, 8- or 4-byte load per plane and one 16- or
// 8-byte store per plane, each contiguous across the wave.  Requires W H % 4
// == 0 and the input pointer aligned to 4 elements.
template <int IN, int OUT, int DEG, int XF>
__global__ __launch_bounds__(256) void k_chw4(const void* __restrict__ in, void* __restrict__ out, uint32_t n_px,
                                               uint32_t hw, FastDiv div_hw4, KCoef k, int gamma) {
  __shared__ float gtab[256];
  if (IN == MACT_U8 && (XF == MACT_LAB || XF == MACT_LUV)) {
    for (uint32_t i = threadIdx.x; i < 256u; i += 256u) gtab[i] = k_gamma_table[gamma][i];
    __syncthreads();
  }
  pin_lead<DEG>(k);
  const uint32_t n4 = n_px >> 2, hw4 = hw >> 2;
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t g4 = blockIdx.x * 256u + threadIdx.x; g4 < n4; g4 += stride) {
    const uint32_t n = div_hw4.div(g4);
    const size_t base = (size_t)n * 3 * hw + 4 * (size_t)(g4 - n * hw4);  // element offset of plane 0
    float v[4][3];  // raw values, as load_px returns them
    load_planes4<IN>(in, base, hw, v);
    float o[3][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float r[3];
      px1<IN, XF, DEG>(k, gamma, gtab, v[j], r);
      o[0][j] = r[0]; o[1][j] = r[1]; o[2][j] = r[2];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) store_plane4<OUT>(out, base + (size_t)c * hw, o[c][0], o[c][1], o[c][2], o[c][3]);
  }
}

// Packed HWC (8-bit, 16-bit, float16 or float32) -> packed float32 or float16
// CHW, 4 pixels per lane with W H a multiple of 4: the lane loads its 4 pixels
// as one 12-byte load (two for 16-bit types, three 16-byte loads for float32;
// the wave's loads cover one contiguous run), and writes each output plane's 4
// values as one 16- or 8-byte store, contiguous across the wave.  No LDS.
// Requires `in` aligned to 4 bytes (16 for float32) and `out` to 16.
template <int IN, int OUT, int DEG, int XF>
__global__ __launch_bounds__(256) void k_hwc_chw4(const void* __restrict__ in, void* __restrict__ out,
                                                  uint32_t n_px, uint32_t hw, FastDiv div_hw4, KCoef k, int gamma) {
  __shared__ float gtab[256];
  if (IN == MACT_U8 && (XF == MACT_LAB || XF == MACT_LUV)) {
    for (uint32_t i = threadIdx.x; i < 256u; i += 256u) gtab[i] = k_gamma_table[gamma][i];
    __syncthreads();
  }
  pin_lead<DEG>(k);
  const uint32_t n4 = n_px >> 2, hw4 = hw >> 2;
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t g4 = blockIdx.x * 256u + threadIdx.x; g4 < n4; g4 += stride) {
    float v[12];  // raw values of the 4 pixels, as load_px returns them
    if (IN == MACT_U8) {
      const uint3 w = reinterpret_cast<const uint3*>(in)[g4];
#pragma unroll
      for (int i = 0; i < 12; ++i) v[i] = (float)byte_of(w, i);
    } else if (IN == MACT_U16) {
      const uint3 wa = reinterpret_cast<const uint3*>(in)[2 * (size_t)g4];
      const uint3 wb = reinterpret_cast<const uint3*>(in)[2 * (size_t)g4 + 1];
#pragma unroll
      for (int i = 0; i < 12; ++i) v[i] = code16_of(wa, wb, i);
    } else if (IN == MACT_F16) {
      const uint3 wa = reinterpret_cast<const uint3*>(in)[2 * (size_t)g4];
      const uint3 wb = reinterpret_cast<const uint3*>(in)[2 * (size_t)g4 + 1];
#pragma unroll
      for (int i = 0; i < 12; ++i) v[i] = half_of(wa, wb, i);
    } else {
      const f4* f = reinterpret_cast<const f4*>(in) + 3 * (size_t)g4;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const f4 b = f[t];
        v[4 * t] = clamp01(b.x); v[4 * t + 1] = clamp01(b.y); v[4 * t + 2] = clamp01(b.z); v[4 * t + 3] = clamp01(b.w);
      }
    }
    float o[3][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float r[3];
      px1<IN, XF, DEG>(k, gamma, gtab, v + 3 * j, r);
      o[0][j] = r[0]; o[1][j] = r[1]; o[2][j] = r[2];
    }
    const uint32_t n = div_hw4.div(g4);
    const size_t base = (size_t)n * 3 * hw + 4 * (size_t)(g4 - n * hw4);
#pragma unroll
    for (int c = 0; c < 3; ++c) store_plane4<OUT>(out, base + (size_t)c * hw, o[c][0], o[c][1], o[c][2], o[c][3]);
  }
}

// Packed CHW (8-bit, 16-bit, float16 or float32) -> packed float32 or float16
// HWC, W H a multiple of 4: one 256-pixel chunk of the batch per wave (the last
// one partial).  Each lane loads its 4 pixels from each plane (one 4-, 8- or
// 16-byte load per plane, contiguous across the wave), computes them, and the
// results leave through the wave's LDS slice as in k_rows4.
template <int IN, int OUT, int DEG, int XF>
__global__ __launch_bounds__(kHotBlock) void k_chw_hwc4(const void* __restrict__ in, void* __restrict__ out,
                                                        uint32_t n_px, uint32_t hw, FastDiv div_hw4, KCoef k,
                                                        int gamma) {
  constexpr uint32_t OSZ = OUT == MACT_F32 ? 4 : 2;
  __shared__ f4 s_out[kHotWaves][3 * OSZ * 16];
  __shared__ float gtab[256];
  if (IN == MACT_U8 && (XF == MACT_LAB || XF == MACT_LUV)) {
    for (uint32_t i = threadIdx.x; i < 256u; i += kHotBlock) gtab[i] = k_gamma_table[gamma][i];
    __syncthreads();
  }
  pin_lead<DEG>(k);
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t c = blockIdx.x * kHotWaves + wv, n_chunks = (n_px + 255u) >> 8;
  if (c >= n_chunks) return;  // no block-wide barrier follows
  const uint32_t cnt = min(256u, n_px - c * 256u);  // a multiple of 4
  const uint32_t g4 = c * 64u + lane, hw4 = hw >> 2;
  float o[12];
  if (4u * lane < cnt) {
    const uint32_t n = div_hw4.div(g4);
    const size_t base = (size_t)n * 3 * hw + 4 * (size_t)(g4 - n * hw4);  // element offset in plane 0
    float v[4][3];
    load_planes4<IN>(in, base, hw, v);
#pragma unroll
    for (int j = 0; j < 4; ++j) px1<IN, XF, DEG>(k, gamma, gtab, v[j], o + 3 * j);
  } else {
#pragma unroll
    for (int q = 0; q < 12; ++q) o[q] = 0.0f;
  }
  stage4<OUT>(s_out[wv], lane, o);
  store_staged<OUT>(s_out[wv], static_cast<char*>(out) + (size_t)c * 768u * OSZ, cnt, lane);
}

// Row-strided CHW (a crop of the planes, a batch with gaps between images)
// -> packed float32 or float16, HWC (OCHW false) or CHW.  W a multiple of 4;
// the input pointer and the row, plane and image strides multiples of 4
// elements, the plane stride below 2^32.  Every row is cut into 256-pixel runs,
// one per wave, 4 pixels per lane: one 4-, 8- or 16-byte load per plane.  HWC
// output leaves through the wave's LDS slice as in k_rows4, CHW output as one
// store per plane and lane.
struct ChwRows {
  uint32_t W, cpr, H;      // pixels per row, runs per row, rows per image
  FastDiv div_cpr, div_h;  // run -> row, row -> image
  uint64_t rs, bs;         // input row and image strides, elements
  uint32_t ps;             // input plane stride, elements
};

template <int IN, int OUT, int DEG, int XF, bool OCHW>
__global__ __launch_bounds__(kHotBlock) void k_chw_rows4(const void* __restrict__ in, void* __restrict__ out,
                                                         uint32_t n_chunks, ChwRows g, KCoef k, int gamma) {
  constexpr uint32_t OSZ = OUT == MACT_F32 ? 4 : 2;
  __shared__ f4 s_out[kHotWaves][OCHW ? 1 : 3 * OSZ * 16];
  __shared__ float gtab[256];
  if (IN == MACT_U8 && (XF == MACT_LAB || XF == MACT_LUV)) {
    for (uint32_t i = threadIdx.x; i < 256u; i += kHotBlock) gtab[i] = k_gamma_table[gamma][i];
    __syncthreads();
  }
  pin_lead<DEG>(k);
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t c = blockIdx.x * kHotWaves + wv;
  if (c >= n_chunks) return;  // no block-wide barrier follows
  const uint32_t r = g.div_cpr.div(c), j = c - r * g.cpr;
  const uint32_t n = g.div_h.div(r), y = r - n * g.H;
  const uint32_t px0 = j * 256u, cnt = min(256u, g.W - px0);  // cnt: a multiple of 4
  const bool live = 4u * lane < cnt;
  float o[12];
  if (live) {
    float v[4][3];
    load_planes4<IN>(in, (size_t)n * g.bs + (size_t)y * g.rs + px0 + 4u * lane, g.ps, v);
#pragma unroll
    for (int q = 0; q < 4; ++q) px1<IN, XF, DEG>(k, gamma, gtab, v[q], o + 3 * q);
  } else {
#pragma unroll
    for (int q = 0; q < 12; ++q) o[q] = 0.0f;
  }
  if (OCHW) {
    if (live) {
      const size_t hw = (size_t)g.W * g.H;
      const size_t e = (size_t)n * 3 * hw + (size_t)y * g.W + px0 + 4u * lane;  // element offset in plane 0
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) store_plane4<OUT>(out, e + ch * hw, o[ch], o[3 + ch], o[6 + ch], o[9 + ch]);
    }
  } else {
    stage4<OUT>(s_out[wv], lane, o);
    store_staged<OUT>(s_out[wv], static_cast<char*>(out) + ((uint64_t)r * g.W + px0) * 3u * OSZ, cnt, lane);
  }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_generic(KImage src, KImage dst, uint32_t n_px, KCoef k, int gamma) {
  __shared__ float gtab[256];
  gtab[threadIdx.x] = k_gamma_table[gamma][threadIdx.x];
  __syncthreads();
  pin_lead<DEG>(k);
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t p = blockIdx.x * 256u + threadIdx.x; p < n_px; p += stride) {
    float v[3], o[3];
    load_px(src, p, v);
    eval_px<DEG>(k, src.dtype, gamma, gtab, v, o);
    store_px(dst, p, o);
  }
}

struct KGrad {
  float dp[8], dq[8];  // derivative coefficients of the float32 p and q
};

// dx of one pixel: (diag(1/white) M)^T (f~'(t) * (J^T g)), zero outside [0, 1].
template <int DEG>
__device__ __forceinline__ void lab_bwd_px(const KCoef& k, const KGrad& kg, const float raw[3], const float g[3],
                                           float dx[3]) {
  float x[3];
  bool in[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    in[c] = raw[c] >= 0.0f && raw[c] <= 1.0f;
    x[c] = clamp01(raw[c]);
  }
  const float t[3] = {
      __builtin_fmaf(kMw00, x[0], __builtin_fmaf(kMw01, x[1], kMw02 * x[2])),
      __builtin_fmaf(kMw10, x[0], __builtin_fmaf(kMw11, x[1], kMw12 * x[2])),
      __builtin_fmaf(kMw20, x[0], __builtin_fmaf(kMw21, x[1], kMw22 * x[2])),
  };
  const float gf[3] = {500.0f * g[1], __builtin_fmaf(116.0f, g[0], __builtin_fmaf(-500.0f, g[1], 200.0f * g[2])),
                       -200.0f * g[2]};
  float gt[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float d = kLabKf;
    if (t[c] > kT0f) {
      const float pv = horner<DEG>(k.p[0], t[c]), qv = horner<DEG>(k.q, t[c]);
      const float dpv = horner<DEG>(kg.dp, t[c]), dqv = horner<DEG>(kg.dq, t[c]);
      d = fdiv(__builtin_fmaf(dpv, qv, -(pv * dqv)), qv * qv);
    }
    gt[c] = gf[c] * d;
  }
  const float r[3] = {
      __builtin_fmaf(kMw00, gt[0], __builtin_fmaf(kMw10, gt[1], kMw20 * gt[2])),
      __builtin_fmaf(kMw01, gt[0], __builtin_fmaf(kMw11, gt[1], kMw21 * gt[2])),
      __builtin_fmaf(kMw02, gt[0], __builtin_fmaf(kMw12, gt[1], kMw22 * gt[2])),
  };
#pragma unroll
  for (int c = 0; c < 3; ++c) dx[c] = in[c] ? r[c] : 0.0f;
}

template <int DEG>
__global__ __launch_bounds__(256) void k_lab_backward(KImage xs, KImage gs, KImage ds, uint32_t n_px, KCoef k,
                                                      KGrad kg) {
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t p = blockIdx.x * 256u + threadIdx.x; p < n_px; p += stride) {
    float raw[3], g[3], dx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      raw[c] = static_cast<const float*>(xs.ptr)[elem_off(xs, p, c)];
      g[c] = static_cast<const float*>(gs.ptr)[elem_off(gs, p, c)];
    }
    lab_bwd_px<DEG>(k, kg, raw, g, dx);
#pragma unroll
    for (int c = 0; c < 3; ++c) static_cast<float*>(ds.ptr)[elem_off(ds, p, c)] = dx[c];
  }
}

// The same on packed CHW tensors, 4 pixels per lane with 16-byte accesses per plane.
template <int DEG>
__global__ __launch_bounds__(256) void k_lab_backward_chw4(const float* __restrict__ xs, const float* __restrict__ gs,
                                                           float* __restrict__ ds, uint32_t n_px, uint32_t hw,
                                                           FastDiv div_hw4, KCoef k, KGrad kg) {
  const uint32_t n4 = n_px >> 2, hw4 = hw >> 2;
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t g4 = blockIdx.x * 256u + threadIdx.x; g4 < n4; g4 += stride) {
    const uint32_t n = div_hw4.div(g4);
    const size_t base = (size_t)n * 3 * hw + 4 * (size_t)(g4 - n * hw4);
    f4 x[3], g[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c] = *reinterpret_cast<const f4*>(xs + base + (size_t)c * hw);
      g[c] = *reinterpret_cast<const f4*>(gs + base + (size_t)c * hw);
    }
    float o[3][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float raw[3] = {x[0][j], x[1][j], x[2][j]}, gg[3] = {g[0][j], g[1][j], g[2][j]};
      float dx[3];
      lab_bwd_px<DEG>(k, kg, raw, gg, dx);
      o[0][j] = dx[0]; o[1][j] = dx[1]; o[2][j] = dx[2];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
      __builtin_nontemporal_store(f4{o[c][0], o[c][1], o[c][2], o[c][3]}, reinterpret_cast<f4*>(ds + base + (size_t)c * hw));
  }
}

// Widen packed bytes to floats with the access pattern of k_hwc4<U8> (no arithmetic).
__global__ __launch_bounds__(kHotBlock) void k_stream_u8_f32(const uint8_t* __restrict__ in, float* __restrict__ out,
                                                             uint32_t n_px) {
  __shared__ f4 s_out[kHotWaves][kChunksPerWave * 192];
  const uint32_t n_chunks = n_px >> 8;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t c0 = (blockIdx.x * kHotWaves + wv) * kChunksPerWave;
  if (c0 < n_chunks) {
    uint3 w[kChunksPerWave];
#pragma unroll
    for (int j = 0; j < kChunksPerWave; ++j)
      if (c0 + j < n_chunks) w[j] = reinterpret_cast<const uint3*>(in)[(size_t)(c0 + j) * 64 + lane];
#pragma unroll
    for (int j = 0; j < kChunksPerWave; ++j) {
      if (c0 + j >= n_chunks) break;
      float o[12];
#pragma unroll
      for (int q = 0; q < 12; ++q) o[q] = (float)byte_of(w[j], q);
      s_out[wv][j * 192 + 3 * lane] = f4{o[0], o[1], o[2], o[3]};
      s_out[wv][j * 192 + 3 * lane + 1] = f4{o[4], o[5], o[6], o[7]};
      s_out[wv][j * 192 + 3 * lane + 2] = f4{o[8], o[9], o[10], o[11]};
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    const uint32_t n_valid = min((uint32_t)kChunksPerWave, n_chunks - c0) * 192u;
    f4* dst = reinterpret_cast<f4*>(out) + (size_t)c0 * 192;
#pragma unroll
    for (int q = 0; q < 3 * kChunksPerWave; ++q) {
      const uint32_t e = q * 64 + lane;
      if (e < n_valid) __builtin_nontemporal_store(s_out[wv][e], dst + e);
    }
  }
  const uint32_t tail0 = n_chunks << 8;
  if (blockIdx.x == 0)
    for (uint32_t e = threadIdx.x; e < 3 * (n_px - tail0); e += kHotBlock)
      out[3 * (size_t)tail0 + e] = (float)in[3 * (size_t)tail0 + e];
}

// A 16-byte copy, each wave one run of 64 words, with the streaming stores of
// the transform kernels.
__global__ __launch_bounds__(256) void k_copy16(const f4* __restrict__ in, f4* __restrict__ out, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  const uint32_t lane = threadIdx.x & 63u;
  for (uint64_t w0 = blockIdx.x * 256ull + (threadIdx.x & ~63u); w0 < n; w0 += stride) {
    const StreamBuf b = wave_stream_buf(out + w0, (uint32_t)std::min<uint64_t>(64, n - w0) * 16u);
    if (w0 + lane < n) stream_store(b, lane * 16u, in[w0 + lane]);
  }
}

// ---------------------------------------------------------------- dispatch

template <int IN, int OUT, int DEG>
static void launch_hwc4(int xform, const void* in, void* out, uint32_t n_px, const KCoef& k, int gamma,
                        hipStream_t st) {
  const dim3 grid(hot_grid(n_px, hot_cpw(IN, OUT, xform))), blk(kHotBlock);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_hwc4<IN, OUT, DEG, MACT_LAB>), grid, blk, 0, st, in, out, n_px, k, gamma);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_hwc4<IN, OUT, DEG, MACT_HSI>), grid, blk, 0, st, in, out, n_px, k, gamma);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_hwc4<IN, OUT, DEG, MACT_LUV>), grid, blk, 0, st, in, out, n_px, k, gamma);
  else hipLaunchKernelGGL((k_hwc4<IN, OUT, DEG, MACT_SCT>), grid, blk, 0, st, in, out, n_px, k, gamma);
}

// deg: the highest degree in use; the instance evaluates Horner from degree 4,
// 5 or 7 (zero leading coefficients leave every bit unchanged).
template <int IN>
static void launch_hwc4_io(int xform, int out_dtype, int deg, const void* in, void* out, uint32_t n_px,
                           const KCoef& k, int gamma, hipStream_t st) {
  if (out_dtype == MACT_F32) {
    if (deg <= 4) launch_hwc4<IN, MACT_F32, 4>(xform, in, out, n_px, k, gamma, st);
    else if (deg == 5) launch_hwc4<IN, MACT_F32, 5>(xform, in, out, n_px, k, gamma, st);
    else launch_hwc4<IN, MACT_F32, 7>(xform, in, out, n_px, k, gamma, st);
  } else {
    if (deg <= 4) launch_hwc4<IN, MACT_F16, 4>(xform, in, out, n_px, k, gamma, st);
    else if (deg == 5) launch_hwc4<IN, MACT_F16, 5>(xform, in, out, n_px, k, gamma, st);
    else launch_hwc4<IN, MACT_F16, 7>(xform, in, out, n_px, k, gamma, st);
  }
}

template <int OUT, int DEG>
static void launch_hwc4f_deg(int xform, const void* in, void* out, uint32_t n_px, const KCoef& k, int gamma,
                             hipStream_t st) {
  const dim3 grid(hot_grid(n_px, kF32Cpw)), blk(kHotBlock);
  const f4* i4 = static_cast<const f4*>(in);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_hwc4f<OUT, DEG, MACT_LAB>), grid, blk, 0, st, i4, out, n_px, k, gamma);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_hwc4f<OUT, DEG, MACT_HSI>), grid, blk, 0, st, i4, out, n_px, k, gamma);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_hwc4f<OUT, DEG, MACT_LUV>), grid, blk, 0, st, i4, out, n_px, k, gamma);
  else hipLaunchKernelGGL((k_hwc4f<OUT, DEG, MACT_SCT>), grid, blk, 0, st, i4, out, n_px, k, gamma);
}

static void launch_hwc4f(int xform, int out_dtype, int deg, const void* in, void* out, uint32_t n_px, const KCoef& k,
                         int gamma, hipStream_t st) {
  if (out_dtype == MACT_F32) {
    if (deg <= 4) launch_hwc4f_deg<MACT_F32, 4>(xform, in, out, n_px, k, gamma, st);
    else if (deg == 5) launch_hwc4f_deg<MACT_F32, 5>(xform, in, out, n_px, k, gamma, st);
    else launch_hwc4f_deg<MACT_F32, 7>(xform, in, out, n_px, k, gamma, st);
  } else {
    if (deg <= 4) launch_hwc4f_deg<MACT_F16, 4>(xform, in, out, n_px, k, gamma, st);
    else if (deg == 5) launch_hwc4f_deg<MACT_F16, 5>(xform, in, out, n_px, k, gamma, st);
    else launch_hwc4f_deg<MACT_F16, 7>(xform, in, out, n_px, k, gamma, st);
  }
}

// The layout kernels below, instanced over output type and degree: OUT is
// float32 or float16; DEG as for k_hwc4 (k_rows4) or 5 / 7 (the others).
template <int IN, int OUT, int DEG>
static void launch_rows4(int xform, const void* in, void* out, uint32_t n_chunks, const RowGeom& g, const KCoef& k,
                         int gamma, hipStream_t st) {
  const dim3 grid(std::max<uint32_t>(1, (n_chunks + kHotWaves - 1) / kHotWaves)), blk(kHotBlock);
  const uint8_t* i8 = static_cast<const uint8_t*>(in);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_rows4<IN, OUT, DEG, MACT_LAB>), grid, blk, 0, st, i8, out, n_chunks, g, k, gamma);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_rows4<IN, OUT, DEG, MACT_HSI>), grid, blk, 0, st, i8, out, n_chunks, g, k, gamma);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_rows4<IN, OUT, DEG, MACT_LUV>), grid, blk, 0, st, i8, out, n_chunks, g, k, gamma);
  else hipLaunchKernelGGL((k_rows4<IN, OUT, DEG, MACT_SCT>), grid, blk, 0, st, i8, out, n_chunks, g, k, gamma);
}

template <int IN, int OUT>
static void launch_rows4_deg(int xform, int deg, const void* in, void* out, uint32_t n_chunks, const RowGeom& g,
                             const KCoef& k, int gamma, hipStream_t st) {
  if (deg <= 4) launch_rows4<IN, OUT, 4>(xform, in, out, n_chunks, g, k, gamma, st);
  else if (deg == 5) launch_rows4<IN, OUT, 5>(xform, in, out, n_chunks, g, k, gamma, st);
  else launch_rows4<IN, OUT, 7>(xform, in, out, n_chunks, g, k, gamma, st);
}

template <int IN>
static void launch_rows4_io(int xform, int out_dtype, int deg, const void* in, void* out, uint32_t n_chunks,
                            const RowGeom& g, const KCoef& k, int gamma, hipStream_t st) {
  if (out_dtype == MACT_F32) launch_rows4_deg<IN, MACT_F32>(xform, deg, in, out, n_chunks, g, k, gamma, st);
  else launch_rows4_deg<IN, MACT_F16>(xform, deg, in, out, n_chunks, g, k, gamma, st);
}

template <int IN, int OUT, int DEG>
static void launch_hwc_chw4(int xform, const void* in, void* out, uint32_t n_px, uint32_t hw, const KCoef& k,
                            int gamma, hipStream_t st) {
  const dim3 grid(full_grid(n_px / 4, 256)), blk(256);
  const FastDiv d = make_fastdiv(hw / 4);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_hwc_chw4<IN, OUT, DEG, MACT_LAB>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_hwc_chw4<IN, OUT, DEG, MACT_HSI>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_hwc_chw4<IN, OUT, DEG, MACT_LUV>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
  else hipLaunchKernelGGL((k_hwc_chw4<IN, OUT, DEG, MACT_SCT>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
}

template <int IN, int OUT, int DEG>
static void launch_chw_hwc4(int xform, const void* in, void* out, uint32_t n_px, uint32_t hw, const KCoef& k,
                            int gamma, hipStream_t st) {
  const dim3 grid(std::max<uint32_t>(1, (((n_px + 255u) >> 8) + kHotWaves - 1) / kHotWaves)), blk(kHotBlock);
  const FastDiv d = make_fastdiv(hw / 4);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_chw_hwc4<IN, OUT, DEG, MACT_LAB>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_chw_hwc4<IN, OUT, DEG, MACT_HSI>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_chw_hwc4<IN, OUT, DEG, MACT_LUV>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
  else hipLaunchKernelGGL((k_chw_hwc4<IN, OUT, DEG, MACT_SCT>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
}

template <int IN, int OUT, int DEG>
static void launch_chw4(int xform, const void* in, void* out, uint32_t n_px, uint32_t hw, const KCoef& k, int gamma,
                        hipStream_t st) {
  const dim3 grid(full_grid(n_px / 4, 256)), blk(256);
  const FastDiv d = make_fastdiv(hw / 4);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_chw4<IN, OUT, DEG, MACT_LAB>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_chw4<IN, OUT, DEG, MACT_HSI>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_chw4<IN, OUT, DEG, MACT_LUV>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
  else hipLaunchKernelGGL((k_chw4<IN, OUT, DEG, MACT_SCT>), grid, blk, 0, st, in, out, n_px, hw, d, k, gamma);
}

// The three plane kernels, by kind (0: CHW -> CHW, 1: HWC -> CHW, 2: CHW ->
// HWC), input type, output type and degree (5 or 7).
template <int KIND, int IN, int OUT, int DEG>
static void launch_planes(int xform, const void* in, void* out, uint32_t n_px, uint32_t hw, const KCoef& k, int gamma,
                          hipStream_t st) {
  if (KIND == 0) launch_chw4<IN, OUT, DEG>(xform, in, out, n_px, hw, k, gamma, st);
  else if (KIND == 1) launch_hwc_chw4<IN, OUT, DEG>(xform, in, out, n_px, hw, k, gamma, st);
  else launch_chw_hwc4<IN, OUT, DEG>(xform, in, out, n_px, hw, k, gamma, st);
}

template <int KIND, int IN>
static void launch_planes_io(int xform, int out_dtype, int deg, const void* in, void* out, uint32_t n_px, uint32_t hw,
                             const KCoef& k, int gamma, hipStream_t st) {
  if (out_dtype == MACT_F32) {
    if (deg <= 4) launch_planes<KIND, IN, MACT_F32, 4>(xform, in, out, n_px, hw, k, gamma, st);
    else if (deg == 5) launch_planes<KIND, IN, MACT_F32, 5>(xform, in, out, n_px, hw, k, gamma, st);
    else launch_planes<KIND, IN, MACT_F32, 7>(xform, in, out, n_px, hw, k, gamma, st);
  } else {
    if (deg <= 4) launch_planes<KIND, IN, MACT_F16, 4>(xform, in, out, n_px, hw, k, gamma, st);
    else if (deg == 5) launch_planes<KIND, IN, MACT_F16, 5>(xform, in, out, n_px, hw, k, gamma, st);
    else launch_planes<KIND, IN, MACT_F16, 7>(xform, in, out, n_px, hw, k, gamma, st);
  }
}

template <int KIND>
static void launch_planes_any(int in_dtype, int xform, int out_dtype, int deg, const void* in, void* out,
                              uint32_t n_px, uint32_t hw, const KCoef& k, int gamma, hipStream_t st) {
  if (in_dtype == MACT_U8) launch_planes_io<KIND, MACT_U8>(xform, out_dtype, deg, in, out, n_px, hw, k, gamma, st);
  else if (in_dtype == MACT_U16) launch_planes_io<KIND, MACT_U16>(xform, out_dtype, deg, in, out, n_px, hw, k, gamma, st);
  else if (in_dtype == MACT_F16) launch_planes_io<KIND, MACT_F16>(xform, out_dtype, deg, in, out, n_px, hw, k, gamma, st);
  else launch_planes_io<KIND, MACT_F32>(xform, out_dtype, deg, in, out, n_px, hw, k, gamma, st);
}

template <int IN, int OUT, int DEG, bool OCHW>
static void launch_chw_rows4(int xform, const void* in, void* out, uint32_t n_chunks, const ChwRows& g, const KCoef& k,
                             int gamma, hipStream_t st) {
  const dim3 grid(std::max<uint32_t>(1, (n_chunks + kHotWaves - 1) / kHotWaves)), blk(kHotBlock);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_chw_rows4<IN, OUT, DEG, MACT_LAB, OCHW>), grid, blk, 0, st, in, out, n_chunks, g, k, gamma);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_chw_rows4<IN, OUT, DEG, MACT_HSI, OCHW>), grid, blk, 0, st, in, out, n_chunks, g, k, gamma);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_chw_rows4<IN, OUT, DEG, MACT_LUV, OCHW>), grid, blk, 0, st, in, out, n_chunks, g, k, gamma);
  else hipLaunchKernelGGL((k_chw_rows4<IN, OUT, DEG, MACT_SCT, OCHW>), grid, blk, 0, st, in, out, n_chunks, g, k, gamma);
}

template <int IN, bool OCHW>
static void launch_chw_rows4_io(int xform, int out_dtype, int deg, const void* in, void* out, uint32_t n_chunks,
                                const ChwRows& g, const KCoef& k, int gamma, hipStream_t st) {
  if (out_dtype == MACT_F32) {
    if (deg <= 4) launch_chw_rows4<IN, MACT_F32, 4, OCHW>(xform, in, out, n_chunks, g, k, gamma, st);
    else if (deg == 5) launch_chw_rows4<IN, MACT_F32, 5, OCHW>(xform, in, out, n_chunks, g, k, gamma, st);
    else launch_chw_rows4<IN, MACT_F32, 7, OCHW>(xform, in, out, n_chunks, g, k, gamma, st);
  } else {
    if (deg <= 4) launch_chw_rows4<IN, MACT_F16, 4, OCHW>(xform, in, out, n_chunks, g, k, gamma, st);
    else if (deg == 5) launch_chw_rows4<IN, MACT_F16, 5, OCHW>(xform, in, out, n_chunks, g, k, gamma, st);
    else launch_chw_rows4<IN, MACT_F16, 7, OCHW>(xform, in, out, n_chunks, g, k, gamma, st);
  }
}

template <bool OCHW>
static void launch_chw_rows4_any(int in_dtype, int xform, int out_dtype, int deg, const void* in, void* out,
                                 uint32_t n_chunks, const ChwRows& g, const KCoef& k, int gamma, hipStream_t st) {
  if (in_dtype == MACT_U8) launch_chw_rows4_io<MACT_U8, OCHW>(xform, out_dtype, deg, in, out, n_chunks, g, k, gamma, st);
  else if (in_dtype == MACT_U16) launch_chw_rows4_io<MACT_U16, OCHW>(xform, out_dtype, deg, in, out, n_chunks, g, k, gamma, st);
  else if (in_dtype == MACT_F16) launch_chw_rows4_io<MACT_F16, OCHW>(xform, out_dtype, deg, in, out, n_chunks, g, k, gamma, st);
  else launch_chw_rows4_io<MACT_F32, OCHW>(xform, out_dtype, deg, in, out, n_chunks, g, k, gamma, st);
}

static bool aligned(const void* p, size_t a) { return (uintptr_t)p % a == 0; }

}  // namespace mact

using namespace mact;

extern "C" mact_status mact_transform(const mact_params* params, const mact_image* in, const mact_image* out,
                                      void* hip_stream) {
  clear_error();
  mact_status s = check_params(params);
  if (s != MACT_OK) return s;
  HostImage hi, ho;
  if ((s = resolve_image(in, false, "mact_transform: in", &hi)) != MACT_OK) return s;
  if ((s = resolve_image(out, true, "mact_transform: out", &ho)) != MACT_OK) return s;
  if ((s = check_same_shape(hi, ho, "mact_transform: out")) != MACT_OK) return s;
  KCoef k;
  int exact_deg = 7;
  const int deg = pack_coef(*params, &k, &exact_deg);
  const int gamma = uses_gamma(params->xform) ? hi.gamma : MACT_GAMMA_NONE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // fast shapes, each to float32 or float16: packed HWC of any input type -> packed HWC or (W H a
  // multiple of 4) packed CHW, row-strided HWC -> packed HWC and row-strided CHW -> packed HWC or
  // CHW (rows of a multiple of 4 pixels), packed CHW of any input type -> packed CHW or HWC (W H a
  // multiple of 4); any other input into packed output, and any input into an output view that
  // is not packed, takes k_gather (gather.hip); outputs not aligned to their element take k_generic
  const bool f_out = ho.dtype == MACT_F32 || ho.dtype == MACT_F16;
  const bool hwc4 = (hi.dtype == MACT_U8 || hi.dtype == MACT_F16 || hi.dtype == MACT_U16) && hi.layout == MACT_HWC &&
                    hi.packed && f_out && ho.layout == MACT_HWC && ho.packed;
  const bool hwc4f = hi.dtype == MACT_F32 && hi.layout == MACT_HWC && hi.packed && f_out && ho.layout == MACT_HWC &&
                     ho.packed;
  const bool planes4 = hi.packed && ho.packed && f_out && (hi.W * hi.H) % 4 == 0 &&
                       (hi.layout == MACT_CHW || ho.layout == MACT_CHW);
  const int64_t rows_align = hi.dtype == MACT_F32 ? 16 : 4;  // row starts: a 12-byte load, or 16-byte loads
  const bool rows4 = hi.layout == MACT_HWC && !hi.packed && f_out && ho.layout == MACT_HWC && ho.packed &&
                     hi.W % 4 == 0 && (hi.rs * (int64_t)hi.esize) % rows_align == 0 &&
                     (hi.bs * (int64_t)hi.esize) % rows_align == 0;
  // row-strided CHW -> packed HWC or CHW: rows of a multiple of 4 pixels, strides of whole 4-element groups
  const bool chw_rows4 = hi.layout == MACT_CHW && !hi.packed && f_out && ho.packed && hi.W % 4 == 0 &&
                         hi.rs % 4 == 0 && hi.ps % 4 == 0 && hi.bs % 4 == 0 && hi.ps < ((int64_t)1 << 32);
  const int64_t per = images_per_stream_launch(hi, ho);
  for (int64_t n0 = 0; n0 < hi.N; n0 += per) {
    const int64_t cnt = std::min(per, hi.N - n0);
    const uint32_t n_px = (uint32_t)(cnt * hi.W * hi.H);
    const void* ip = static_cast<const char*>(hi.data) + (size_t)(n0 * hi.bs) * hi.esize;
    void* op = static_cast<char*>(ho.data) + (size_t)(n0 * ho.bs) * ho.esize;
    // input alignment of the plane kernels: 4 elements of a CHW plane, a 12-byte load of HWC
    // pixels (16 bytes for float32)
    const size_t planes_align = hi.layout == MACT_CHW ? 4 * hi.esize : hi.dtype == MACT_F32 ? 16 : 4;
    if (hwc4 && aligned(ip, 4) && aligned(op, 16)) {
      if (hi.dtype == MACT_U8) launch_hwc4_io<MACT_U8>(params->xform, ho.dtype, exact_deg, ip, op, n_px, k, gamma, st);
      else if (hi.dtype == MACT_U16) launch_hwc4_io<MACT_U16>(params->xform, ho.dtype, exact_deg, ip, op, n_px, k, gamma, st);
      else launch_hwc4_io<MACT_F16>(params->xform, ho.dtype, exact_deg, ip, op, n_px, k, gamma, st);
    } else if (hwc4f && aligned(ip, 16) && aligned(op, 16)) {
      launch_hwc4f(params->xform, ho.dtype, exact_deg, ip, op, n_px, k, gamma, st);
    } else if (planes4 && aligned(ip, planes_align) && aligned(op, 16)) {
      const uint32_t hw = (uint32_t)(hi.W * hi.H);
      if (hi.layout == MACT_CHW && ho.layout == MACT_CHW)
        launch_planes_any<0>(hi.dtype, params->xform, ho.dtype, exact_deg, ip, op, n_px, hw, k, gamma, st);
      else if (ho.layout == MACT_CHW)
        launch_planes_any<1>(hi.dtype, params->xform, ho.dtype, exact_deg, ip, op, n_px, hw, k, gamma, st);
      else
        launch_planes_any<2>(hi.dtype, params->xform, ho.dtype, exact_deg, ip, op, n_px, hw, k, gamma, st);
    } else if (rows4 && aligned(ip, (size_t)rows_align) && aligned(op, 16)) {
      RowGeom g;
      g.W = (uint32_t)hi.W;
      g.H = (uint32_t)hi.H;
      g.cpr = (g.W + 256u * kRowHalves - 1u) / (256u * kRowHalves);
      g.div_cpr = make_fastdiv(g.cpr);
      g.div_h = make_fastdiv(g.H);
      g.rs_b = (uint64_t)hi.rs * hi.esize;
      g.bs_b = (uint64_t)hi.bs * hi.esize;
      const uint32_t n_chunks = (uint32_t)(cnt * hi.H) * g.cpr;
      if (hi.dtype == MACT_U8) launch_rows4_io<MACT_U8>(params->xform, ho.dtype, exact_deg, ip, op, n_chunks, g, k, gamma, st);
      else if (hi.dtype == MACT_U16) launch_rows4_io<MACT_U16>(params->xform, ho.dtype, exact_deg, ip, op, n_chunks, g, k, gamma, st);
      else if (hi.dtype == MACT_F16) launch_rows4_io<MACT_F16>(params->xform, ho.dtype, exact_deg, ip, op, n_chunks, g, k, gamma, st);
      else launch_rows4_io<MACT_F32>(params->xform, ho.dtype, exact_deg, ip, op, n_chunks, g, k, gamma, st);
    } else if (chw_rows4 && aligned(ip, 4 * hi.esize) && aligned(op, 16)) {
      ChwRows g;
      g.W = (uint32_t)hi.W;
      g.H = (uint32_t)hi.H;
      g.cpr = (g.W + 255u) / 256u;
      g.div_cpr = make_fastdiv(g.cpr);
      g.div_h = make_fastdiv(g.H);
      g.rs = (uint64_t)hi.rs;
      g.bs = (uint64_t)hi.bs;
      g.ps = (uint32_t)hi.ps;
      const uint32_t n_chunks = (uint32_t)(cnt * hi.H) * g.cpr;
      if (ho.layout == MACT_CHW)
        launch_chw_rows4_any<true>(hi.dtype, params->xform, ho.dtype, exact_deg, ip, op, n_chunks, g, k, gamma, st);
      else
        launch_chw_rows4_any<false>(hi.dtype, params->xform, ho.dtype, exact_deg, ip, op, n_chunks, g, k, gamma, st);
    } else if (ho.packed && f_out && aligned(op, 16)) {
      launch_gather(hi.dtype, params->xform, ho.dtype, ho.layout == MACT_CHW ? kGatherCHW : kGatherHWC, exact_deg,
                    kimage(hi, n0, cnt), KImage{}, op, n_px, (uint32_t)(hi.W * hi.H), k, gamma, st);
    } else if (f_out && aligned(op, (size_t)ho.esize)) {
      launch_gather(hi.dtype, params->xform, ho.dtype, kGatherAny, exact_deg, kimage(hi, n0, cnt), kimage(ho, n0, cnt),
                    op, n_px, (uint32_t)(hi.W * hi.H), k, gamma, st);
    } else {
      const KImage ks = kimage(hi, n0, cnt), kd = kimage(ho, n0, cnt);
      const unsigned grid = full_grid(n_px, 256);
      if (deg == 5) hipLaunchKernelGGL(k_generic<5>, dim3(grid), dim3(256), 0, st, ks, kd, n_px, k, gamma);
      else hipLaunchKernelGGL(k_generic<7>, dim3(grid), dim3(256), 0, st, ks, kd, n_px, k, gamma);
    }
    if ((s = hip_check(hipGetLastError(), "mact_transform: launch")) != MACT_OK) return s;
  }
  return MACT_OK;
}

extern "C" mact_status mact_transform_backward(const mact_params* params, const mact_image* x,
                                               const mact_image* grad_out, const mact_image* grad_in,
                                               void* hip_stream) {
  clear_error();
  mact_status s = check_params(params);
  if (s != MACT_OK) return s;
  if (params->xform != MACT_LAB) return fail(MACT_E_UNSUPPORTED, "mact_transform_backward: only MACT_LAB");
  if (params->out_mode != 0) return fail(MACT_E_INVALID, "mact_transform_backward: out_mode must be 0");
  HostImage hx, hg, hd;
  if ((s = resolve_image(x, false, "mact_transform_backward: x", &hx)) != MACT_OK) return s;
  if ((s = resolve_image(grad_out, false, "mact_transform_backward: grad_out", &hg)) != MACT_OK) return s;
  if ((s = resolve_image(grad_in, true, "mact_transform_backward: grad_in", &hd)) != MACT_OK) return s;
  if (hx.dtype != MACT_F32 || hg.dtype != MACT_F32 || hd.dtype != MACT_F32)
    return fail(MACT_E_UNSUPPORTED, "mact_transform_backward: x, grad_out and grad_in must be MACT_F32");
  if (hx.gamma != MACT_GAMMA_NONE) return fail(MACT_E_UNSUPPORTED, "mact_transform_backward: x must be linear (MACT_GAMMA_NONE)");
  if ((s = check_same_shape(hx, hg, "mact_transform_backward: grad_out")) != MACT_OK) return s;
  if ((s = check_same_shape(hx, hd, "mact_transform_backward: grad_in")) != MACT_OK) return s;
  KCoef k;
  int exact_deg = 7;
  const int deg = pack_coef(*params, &k, &exact_deg);
  KGrad kg;
  std::memset(&kg, 0, sizeof kg);
  for (int j = 1; j <= 7; ++j) {
    kg.dp[j - 1] = (float)(j * (double)k.p[0][j]);
    kg.dq[j - 1] = (float)(j * (double)k.q[j]);
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const bool chw4 = hx.layout == MACT_CHW && hg.layout == MACT_CHW && hd.layout == MACT_CHW && hx.packed && hg.packed &&
                    hd.packed && (hx.W * hx.H) % 4 == 0;
  const int64_t per = images_per_launch(hx);
  for (int64_t n0 = 0; n0 < hx.N; n0 += per) {
    const int64_t cnt = std::min(per, hx.N - n0);
    const uint32_t n_px = (uint32_t)(cnt * hx.W * hx.H);
    const float* xp = static_cast<const float*>(hx.data) + (size_t)(n0 * hx.bs);
    const float* gp = static_cast<const float*>(hg.data) + (size_t)(n0 * hg.bs);
    float* dp = static_cast<float*>(hd.data) + (size_t)(n0 * hd.bs);
    const uint32_t hw = (uint32_t)(hx.W * hx.H);
    if (chw4 && aligned(xp, 16) && aligned(gp, 16) && aligned(dp, 16)) {
      const dim3 grid(full_grid(n_px / 4, 256));
      const FastDiv d = make_fastdiv(hw / 4);
      if (exact_deg <= 4) hipLaunchKernelGGL(k_lab_backward_chw4<4>, grid, dim3(256), 0, st, xp, gp, dp, n_px, hw, d, k, kg);
      else if (deg == 5) hipLaunchKernelGGL(k_lab_backward_chw4<5>, grid, dim3(256), 0, st, xp, gp, dp, n_px, hw, d, k, kg);
      else hipLaunchKernelGGL(k_lab_backward_chw4<7>, grid, dim3(256), 0, st, xp, gp, dp, n_px, hw, d, k, kg);
    } else {
      const KImage kx = kimage(hx, n0, cnt), kgo = kimage(hg, n0, cnt), kd = kimage(hd, n0, cnt);
      const unsigned grid = full_grid(n_px, 256);
      if (deg == 5) hipLaunchKernelGGL(k_lab_backward<5>, dim3(grid), dim3(256), 0, st, kx, kgo, kd, n_px, k, kg);
      else hipLaunchKernelGGL(k_lab_backward<7>, dim3(grid), dim3(256), 0, st, kx, kgo, kd, n_px, k, kg);
    }
    if ((s = hip_check(hipGetLastError(), "mact_transform_backward: launch")) != MACT_OK) return s;
  }
  return MACT_OK;
}

extern "C" mact_status mact_stream_u8_to_f32(const void* src, void* dst, int64_t n_px, void* hip_stream) {
  clear_error();
  if (!src || !dst) return fail(MACT_E_INVALID, "mact_stream_u8_to_f32: NULL pointer");
  if (n_px <= 0 || n_px >= (1ll << 31)) return fail(MACT_E_INVALID, "mact_stream_u8_to_f32: n_px %lld", (long long)n_px);
  if ((uintptr_t)src % 4 || (uintptr_t)dst % 16) return fail(MACT_E_INVALID, "mact_stream_u8_to_f32: misaligned buffers");
  hipLaunchKernelGGL(k_stream_u8_f32, dim3(hot_grid((uint32_t)n_px)), dim3(kHotBlock), 0, static_cast<hipStream_t>(hip_stream),
                     static_cast<const uint8_t*>(src), static_cast<float*>(dst), (uint32_t)n_px);
  return hip_check(hipGetLastError(), "mact_stream_u8_to_f32: launch");
}

extern "C" mact_status mact_copy(const void* src, void* dst, int64_t bytes, void* hip_stream) {
  clear_error();
  if (!src || !dst) return fail(MACT_E_INVALID, "mact_copy: NULL pointer");
  if (bytes <= 0 || bytes % 16) return fail(MACT_E_INVALID, "mact_copy: bytes %lld not a positive multiple of 16", (long long)bytes);
  if ((uintptr_t)src % 16 || (uintptr_t)dst % 16) return fail(MACT_E_INVALID, "mact_copy: misaligned buffers");
  const uint64_t n = (uint64_t)bytes / 16;
  const unsigned grid = full_grid(n, 256);
  hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     static_cast<const f4*>(src), static_cast<f4*>(dst), n);
  return hip_check(hipGetLastError(), "mact_copy: launch");
}
