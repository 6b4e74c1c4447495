// 3-D LUT packing and interpolation (Sec. 3.5.3): the comparison path.
//
// Packing runs on the host in FP64 (the exact transform at every node) and
// uploads float32 nodes.  A node is one float4 (LAB: L*, a*, b*, 0; HSI:
// cos H, sin H, S, I; SCT: cos A, sin A, cos B, sin B): angular channels are
// stored as unit vectors so that circular interpolation needs no
// trigonometry per corner.  SCT's fifth value, L, lives in a plane of one
// float per node after the N^3 float4 (20 bytes a node, with no padding).
//
// Interpolation: when the packed grid fits the workgroup's LDS beside the
// store buffers (17^3: 78.6 KB, SCT 98.3 KB) one or two workgroups per CU
// stage it once, with G and R strides padded against bank conflicts
// (lds_strides), and stride over the image; every corner gather is then an LDS
// read.  Larger grids (33^3 x 16 B = 575 KB) are gathered from global memory
// through the L2 by a grid that covers the image once, neighbouring lanes on
// neighbouring pixels, and trilinear (every method on cell-major grids) with
// two lanes per pixel, which halves the cache lines a gather touches.  Packed
// 8-bit HWC -> float32 HWC takes k_lut4 (the transform's 12-byte loads and
// LDS-transposed 1 KB stores); other shapes take k_lut, one pixel per lane.
// Each method is a weighted sum of its 8, 6, 5 or 4 corners, summed in two
// chains (even and odd corner ids) on every path, so all paths and forms give
// the same bits.
//
// Cell-major form: (N-1)^3 cells, each holding its 8 corner nodes in one
// contiguous run (128 bytes; for SCT followed, after all cells, by the
// cells' 8 L values, 32 bytes a cell), so that one pixel's corners are one
// cache line instead of four lines N and N^2 nodes apart: the form that only
// reorders memory, beside the paper's caching records (kCache below), which
// store edge differences to save arithmetic.  Corner ids (dR dG dB as bits 2,
// 1, 0) stand in for the node strides, so both forms sum the same values in
// the same order and give the same bits.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "launch.h"

namespace mact {

typedef float f4 __attribute__((ext_vector_type(4)));

// float4 units of a LUT of `entries` nodes (packed: N^3; cell-major: 8 per
// cell): one per node, and for SCT the L plane, one float per node, after them.
static size_t lut_f4s(int xform, size_t entries) { return entries + (xform == MACT_SCT ? (entries + 3) / 4 : 0); }

// Bytes of the caching form: (N-1)^3 records of 13 entries of C floats
// (3, 4 or 5 components), rounded up to 16 bytes.
static size_t lut_cache_size(int xform, size_t n) {
  const size_t c = xform == MACT_SCT ? 5 : xform == MACT_HSI ? 4 : 3;
  const size_t m = n - 1;
  return (m * m * m * 13 * c * sizeof(float) + 15) / 16 * 16;
}

// ---------------------------------------------------------------- device

// atan2(y, x) for the angular channels' resultants, with atan2's quadrants and
// signed zeros.  The ratio t = min / max of |x|, |y| (a reciprocal and one
// Newton correction) folds the angle into [0, pi/4]; there atan t =
// t + t^3 Q(t^2), Q of degree 7 fitted for relative error on [0, 1]
// (1.7e-8; 1.1 ulp in float32 over [0, 1]); pi/2 - and pi - unfold it with
// two-part constants.  About 25 instructions, against about 45 for the
// library's atan2f, which the HSI and SCT LUT kernels spend most of their
// arithmetic on.  Arguments below 2^-64 are scaled first, since the
// reciprocal of a denormal overflows.
__device__ __forceinline__ float lut_atan2(float y, float x) {
  // |x|, |y| <= 1 here; scaled by 2^64 (exactly) so that no denormal reaches the reciprocal, and
  // max >= 2^-100 so that (0, 0) gives t = 0
  const float ax = fabsf(x) * 0x1p64f, ay = fabsf(y) * 0x1p64f;
  const float mx = fmaxf(fmaxf(ax, ay), 0x1p-100f), mn = fminf(ax, ay);
  const float r = __builtin_amdgcn_rcpf(mx);
  float t = mn * r;
  t = __builtin_fmaf(__builtin_fmaf(-mx, t, mn), r, t);
  const float s = t * t;
  float q = 0x1.7ed22cp-9f;
  q = __builtin_fmaf(q, s, -0x1.0c2c1p-6f);
  q = __builtin_fmaf(q, s, 0x1.61fdd8p-5f);
  q = __builtin_fmaf(q, s, -0x1.3556b4p-4f);
  q = __builtin_fmaf(q, s, 0x1.b4e12ap-4f);
  q = __builtin_fmaf(q, s, -0x1.230adcp-3f);
  q = __builtin_fmaf(q, s, 0x1.9978f4p-3f);
  q = __builtin_fmaf(q, s, -0x1.5554dcp-2f);
  float a = __builtin_fmaf(t * s, q, t);
  constexpr float kPi2Lo = static_cast<float>(kPi / 2.0 - static_cast<double>(kPi2f));
  constexpr float kPiLo = static_cast<float>(kPi - static_cast<double>(kPif));
  if (ay > ax) a = (kPi2f - a) + kPi2Lo;  // exact difference: a lies in [pi/4, pi/2]
  if (__builtin_signbit(x)) a = (kPif - a) + kPiLo;
  return __builtin_copysignf(a, y);
}

// Extraction: cell and fraction per channel.
__device__ __forceinline__ void locate_u8(uint32_t v, uint32_t N, uint32_t& i, float& f) {
  const uint32_t num = v * (N - 1);
  i = min(num / 255u, N - 2);
  f = (float)(num - 255u * i) * kInv255;
}

__device__ __forceinline__ void locate_f(float x, uint32_t N, uint32_t& i, float& f) {
  const float pos = x * (float)(N - 1);
  i = min((uint32_t)pos, N - 2);  // x >= 0 after clamping
  f = pos - (float)i;
}

// Corner weights of each method, as (offset, weight) pairs; K = 8, 6, 5, 4.
template <int METHOD>
struct Corners;

template <>
struct Corners<MACT_TRILINEAR> {
  static constexpr int K = 8;
  __device__ __forceinline__ static void get(float fr, float fg, float fb, uint32_t sR, uint32_t sG, uint32_t off[8],
                                             float w[8]) {
    const float r0 = 1.0f - fr, g0 = 1.0f - fg, b0 = 1.0f - fb;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int dr = c >> 2, dg = (c >> 1) & 1, db = c & 1;
      off[c] = dr * sR + dg * sG + db;
      w[c] = (dr ? fr : r0) * (dg ? fg : g0) * (db ? fb : b0);
    }
  }
};

template <>
struct Corners<MACT_TETRAHEDRAL> {
  static constexpr int K = 4;
  __device__ __forceinline__ static void get(float fr, float fg, float fb, uint32_t sR, uint32_t sG, uint32_t off[4],
                                             float w[4]) {
    // decreasing order of the fractions, ties R before G before B, without branches: the largest,
    // median and smallest values, the stride of the largest axis (s1) and of the smallest (s3)
    const bool rg = fr >= fg, rb = fr >= fb, gb = fg >= fb;
    const float f1 = fmaxf(fmaxf(fr, fg), fb), f3 = fminf(fminf(fr, fg), fb);
    const float f2 = __builtin_amdgcn_fmed3f(fr, fg, fb);
    const uint32_t s1 = rg ? (rb ? sR : 1u) : (gb ? sG : 1u);
    const uint32_t s3 = rg ? (gb ? 1u : sG) : (rb ? 1u : sR);
    off[0] = 0; w[0] = 1.0f - f1;
    off[1] = s1; w[1] = f1 - f2;
    off[2] = sR + sG + 1u - s3; w[2] = f2 - f3;
    off[3] = sR + sG + 1; w[3] = f3;
  }
};

// The tetrahedral corners by branches on the fraction order: the same corners
// and weights as Corners<MACT_TETRAHEDRAL>.  Where one lane takes one pixel
// and neighbouring lanes take neighbouring pixels (the L2 path), the branches
// are mostly uniform over a wave, and this form measured faster there (CIELAB
// 33^3: 153 vs 139-146 Gpx/s); elsewhere the branch-free form is (17^3 in LDS,
// HSI and SCT: +8-11%).
__device__ __forceinline__ void tet_corners_branch(float fr, float fg, float fb, uint32_t sR, uint32_t sG,
                                                   uint32_t off[4], float w[4]) {
  float f1, f2, f3;
  uint32_t s1, s2;
  if (fr >= fg) {
    if (fg >= fb) { f1 = fr; f2 = fg; f3 = fb; s1 = sR; s2 = sG; }
    else if (fr >= fb) { f1 = fr; f2 = fb; f3 = fg; s1 = sR; s2 = 1; }
    else { f1 = fb; f2 = fr; f3 = fg; s1 = 1; s2 = sR; }
  } else {
    if (fr >= fb) { f1 = fg; f2 = fr; f3 = fb; s1 = sG; s2 = sR; }
    else if (fg >= fb) { f1 = fg; f2 = fb; f3 = fr; s1 = sG; s2 = 1; }
    else { f1 = fb; f2 = fg; f3 = fr; s1 = 1; s2 = sG; }
  }
  off[0] = 0; w[0] = 1.0f - f1;
  off[1] = s1; w[1] = f1 - f2;
  off[2] = s1 + s2; w[2] = f2 - f3;
  off[3] = sR + sG + 1; w[3] = f3;
}

template <>
struct Corners<MACT_PRISM> {
  static constexpr int K = 6;
  __device__ __forceinline__ static void get(float fr, float fg, float fb, uint32_t sR, uint32_t sG, uint32_t off[6],
                                             float w[6]) {
    // linear along R; triangle of the (G, B) face chosen by f_G >= f_B
    uint32_t t1;
    float w0, w1, w2;
    if (fg >= fb) { t1 = sG; w0 = 1.0f - fg; w1 = fg - fb; w2 = fb; }
    else { t1 = 1; w0 = 1.0f - fb; w1 = fb - fg; w2 = fg; }
    const float r0 = 1.0f - fr;
    off[0] = 0; w[0] = r0 * w0;
    off[1] = t1; w[1] = r0 * w1;
    off[2] = sG + 1; w[2] = r0 * w2;
    off[3] = sR; w[3] = fr * w0;
    off[4] = sR + t1; w[4] = fr * w1;
    off[5] = sR + sG + 1; w[5] = fr * w2;
  }
};

template <>
struct Corners<MACT_PYRAMIDAL> {
  static constexpr int K = 5;
  __device__ __forceinline__ static void get(float fr, float fg, float fb, uint32_t sR, uint32_t sG, uint32_t off[5],
                                             float w[5]) {
    // smallest fraction s (ties R before G before B); u, v the other two in R, G, B order
    float fs, fu, fv;
    uint32_t ss, su, sv;
    if (fr <= fg && fr <= fb) { fs = fr; fu = fg; fv = fb; ss = sR; su = sG; sv = 1; }
    else if (fg <= fb) { fs = fg; fu = fr; fv = fb; ss = sG; su = sR; sv = 1; }
    else { fs = fb; fu = fr; fv = fg; ss = 1; su = sR; sv = sG; }
    const float uv = fu * fv;
    // c000 + (c111 - c0uv) fs + (c0u0 - c000) fu + (c00v - c000) fv + (c0uv - c00v - c0u0 + c000) fu fv
    off[0] = 0; w[0] = ((1.0f - fu) - fv) + uv;
    off[1] = ss + su + sv; w[1] = fs;
    off[2] = su + sv; w[2] = uv - fs;
    off[3] = su; w[3] = fu - uv;
    off[4] = sv; w[4] = fv - uv;
  }
};

// Layout of a LUT buffer: packed nodes, cell-major corners, or the caching
// form's difference records.
enum { kPacked = 0, kCells = 1, kCache = 2 };

// Components of a caching-form entry: LAB, LUV: the three channels; HSI:
// cos H, sin H, S, I; SCT: L, cos A, sin A, cos B, sin B.
template <int XF>
struct CacheC {
  static constexpr int C = XF == MACT_SCT ? 5 : XF == MACT_HSI ? 4 : 3;
};

// Entries of a caching record: 0 the node value c000, then the differences
// along the cell's 12 edges: 1 + 2g + b the R edge at (g, b), 5 + 2r + b the G
// edge at (r, b), 9 + 2r + g the B edge at (r, g).
__device__ __forceinline__ constexpr int edge_r(int g, int b) { return 1 + 2 * g + b; }
__device__ __forceinline__ constexpr int edge_g(int r, int b) { return 5 + 2 * r + b; }
__device__ __forceinline__ constexpr int edge_b(int r, int g) { return 9 + 2 * r + g; }

// Caching form (Sec. 3.5.3): the record of the pixel's cell, entry 0 plus the
// method's edge differences, each times its weight: every corner of the
// method's corner sum written as c000 plus the edges of a path to it, so no
// corner subtraction is left per pixel.
template <int METHOD, int XF>
__device__ __forceinline__ void lut_px_cache(const float* __restrict__ cache, uint32_t N, const uint32_t i[3],
                                             const float f[3], float o[3]) {
  constexpr int C = CacheC<XF>::C;
  const float* __restrict__ r = cache + (size_t)(((i[0] * (N - 1) + i[1]) * (N - 1) + i[2])) * (13 * C);
  float acc[C];
#pragma unroll
  for (int k = 0; k < C; ++k) acc[k] = r[k];
  auto add = [&](int e, float w) {
#pragma unroll
    for (int k = 0; k < C; ++k) acc[k] = __builtin_fmaf(w, r[e * C + k], acc[k]);
  };
  const float fr = f[0], fg = f[1], fb = f[2];
  if (METHOD == MACT_TRILINEAR) {
    const float gb = fg * fb, g0 = fg - gb, rg = fr * fg;
    add(edge_b(0, 0), fb);
    add(edge_g(0, 0), g0);
    add(edge_g(0, 1), gb);
    add(edge_r(0, 0), (fr - rg) * (1.0f - fb));
    add(edge_r(0, 1), (fr - rg) * fb);
    add(edge_r(1, 0), rg * (1.0f - fb));
    add(edge_r(1, 1), rg * fb);
  } else if (METHOD == MACT_PRISM) {
    // linear along R; the (G, B) triangle chosen by f_G >= f_B, its two edges blended along R
    // (the triangle's edges and weights are selected, not branched on, so that a wave whose pixels
    // fall in both triangles issues each load once)
    const float r0 = 1.0f - fr;
    const bool gb = fg >= fb;
    const float wu = gb ? fg : fb, wv = gb ? fb : fg;
    add(edge_r(0, 0), fr);
    add(gb ? edge_g(0, 0) : edge_b(0, 0), wu * r0);
    add(gb ? edge_g(1, 0) : edge_b(1, 0), wu * fr);
    add(gb ? edge_b(0, 1) : edge_g(0, 1), wv * r0);
    add(gb ? edge_b(1, 1) : edge_g(1, 1), wv * fr);
  } else if (METHOD == MACT_TETRAHEDRAL) {
    // the path from c000 along the axes in decreasing order of the fractions (ties R, G, B):
    // each step's edge sits where the earlier steps have moved to
    // (selected, not branched on: rg, gb, rb are the three comparisons; with R >= G the first axis
    // is R unless B beats R, the last B unless G is the smallest; with G > R, mirrored)
    const bool rg = fr >= fg, gb = fg >= fb, rb = fr >= fb;
    const int e1 = rg ? (rb ? edge_r(0, 0) : edge_b(0, 0)) : (gb ? edge_g(0, 0) : edge_b(0, 0));
    const float w1 = rg ? (rb ? fr : fb) : (gb ? fg : fb);
    const int e2 = rg ? (gb ? edge_g(1, 0) : rb ? edge_b(1, 0) : edge_r(0, 1))
                      : (rb ? edge_r(1, 0) : gb ? edge_b(0, 1) : edge_g(0, 1));
    const float w2 = rg ? (gb ? fg : rb ? fb : fr) : (rb ? fr : gb ? fb : fg);
    const int e3 = rg ? (gb ? edge_b(1, 1) : edge_g(1, 1)) : (rb ? edge_b(1, 1) : edge_r(1, 1));
    const float w3 = rg ? (gb ? fb : fg) : (rb ? fb : fr);
    add(e1, w1);
    add(e2, w2);
    add(e3, w3);
  } else {
    // pyramidal: s the axis of the smallest fraction (ties R, G, B), u, v the other two in order:
    // c000 + f_s (s edge at u = v = 1) + f_u (1 - f_v) (u edge at s = v = 0) + f_v (v edge at
    // s = u = 0) + f_u f_v (u edge at s = 0, v = 1)
    // (selected, not branched on)
    const bool sr = fr <= fg && fr <= fb, sg = !sr && fg <= fb;
    const int es = sr ? edge_r(1, 1) : sg ? edge_g(1, 1) : edge_b(1, 1);
    const int eu0 = sr ? edge_g(0, 0) : edge_r(0, 0);
    const int ev = sr || sg ? edge_b(0, 0) : edge_g(0, 0);
    const int eu1 = sr ? edge_g(0, 1) : sg ? edge_r(0, 1) : edge_r(1, 0);
    const float fs = sr ? fr : sg ? fg : fb, fu = sr ? fg : fr, fv = sr || sg ? fb : fg;
    const float uv = fu * fv;
    add(es, fs);
    add(eu0, fu - uv);
    add(ev, fv);
    add(eu1, uv);
  }
  if (XF == MACT_LAB || XF == MACT_LUV) {
    o[0] = acc[0]; o[1] = acc[1]; o[2] = acc[2];
  } else if (XF == MACT_HSI) {
    float h = lut_atan2(acc[1], acc[0]);
    if (h < 0.0f) h += kTwoPif;
    o[0] = h; o[1] = acc[2]; o[2] = acc[C - 1];
  } else {
    o[0] = acc[0];
    o[1] = lut_atan2(acc[2], acc[1]);
    o[2] = lut_atan2(acc[C - 1], acc[3]);
  }
}

// fma of a float4 by a scalar weight: w v + a, channel by channel.
__device__ __forceinline__ f4 fma4(float w, f4 v, f4 a) {
  return f4{__builtin_fmaf(w, v.x, a.x), __builtin_fmaf(w, v.y, a.y), __builtin_fmaf(w, v.z, a.z),
            __builtin_fmaf(w, v.w, a.w)};
}

// The outputs from the weighted sums: linear channels as they are, angles
// from their (cos, sin) resultants.
template <int XF>
__device__ __forceinline__ void lut_out(f4 a0, float a1, float o[3]) {
  if (XF == MACT_LAB || XF == MACT_LUV) {
    o[0] = a0.x; o[1] = a0.y; o[2] = a0.z;
  } else if (XF == MACT_HSI) {
    float h = lut_atan2(a0.y, a0.x);
    if (h < 0.0f) h += kTwoPif;
    o[0] = h; o[1] = a0.z; o[2] = a0.w;
  } else {
    o[0] = a1;
    o[1] = lut_atan2(a0.y, a0.x);
    o[2] = lut_atan2(a0.w, a0.z);
  }
}

// One pixel: the method's weighted corner sum at cell i, fractions f.  FORM
// kCells: `nodes` is the cell-major form; kCache: the caching records.
// `lp`: SCT's L plane (one float per entry of `nodes`); unused otherwise.
template <int METHOD, int XF, int FORM, bool BRANCH = false>
__device__ __forceinline__ void lut_px(const f4* __restrict__ nodes, const float* __restrict__ lp, uint32_t N,
                                       uint32_t sR, uint32_t sG, const uint32_t i[3], const float f[3], float o[3]) {
  if (FORM == kCache) {
    lut_px_cache<METHOD, XF>(reinterpret_cast<const float*>(nodes), N, i, f, o);
    return;
  }
  constexpr bool CELL = FORM == kCells;
  // packed: node (i, j, k) at i sR + j sG + k (N^2, N; more where the grid is staged with padding)
  const uint32_t base = CELL ? ((i[0] * (N - 1) + i[1]) * (N - 1) + i[2]) * 8u : i[0] * sR + i[1] * sG + i[2];
  if (CELL) {
    sR = 4u;
    sG = 2u;
  }
  uint32_t off[8];
  float w[8];
  if constexpr (METHOD == MACT_TETRAHEDRAL && BRANCH)
    tet_corners_branch(f[0], f[1], f[2], sR, sG, off, w);
  else
    Corners<METHOD>::get(f[0], f[1], f[2], sR, sG, off, w);
  // The corners in two chains, even and odd corner ids (each a product, then fused multiply-adds
  // in id order), added last; for trilinear (c = 4 dR + 2 dG + dB) the chains are dB = 0 and 1.
  // SCT's L: the same chains, except trilinear's, which are dR = 0 and 1 (corners 0..3 and 4..7).
  // The two-lane kernels below sum in this order, so every path gives the same bits.
  constexpr int K = Corners<METHOD>::K;
  f4 ch[2];
  float cu[2] = {0.0f, 0.0f};
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    ch[b] = w[b] * nodes[base + off[b]];
#pragma unroll
    for (int c = b + 2; c < K; c += 2) ch[b] = fma4(w[c], nodes[base + off[c]], ch[b]);
  }
#pragma unroll
  for (int b = 0; b < 2 && XF == MACT_SCT; ++b) {
    const int c0 = METHOD == MACT_TRILINEAR ? 4 * b : b, dc = METHOD == MACT_TRILINEAR ? 1 : 2;
    cu[b] = w[c0] * lp[base + off[c0]];
#pragma unroll
    for (int c = c0 + dc; c < (METHOD == MACT_TRILINEAR ? c0 + 4 : K); c += dc)
      cu[b] = __builtin_fmaf(w[c], lp[base + off[c]], cu[b]);
  }
  const f4 a0 = ch[0] + ch[1];
  const float a1 = cu[0] + cu[1];
  lut_out<XF>(a0, a1, o);
}

// Two floats at a 4-byte aligned address (global memory takes unaligned
// multi-dword loads).
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));

// The value of lane l ^ 1: a DPP quad permutation (1, 0, 3, 2), no LDS access.
__device__ __forceinline__ float swap1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// The order in which a wave takes its chunk's 256 pixels from the L2: ord[q] is
// the pixel at position q, the pixels grouped by the cache line of their
// cell's first node (key: R and G cells mod 8, B cell / 8 mod 4; a counting
// sort through 256 counters in `bins`).  The vector L1 looks up the lines of
// each group of 4 neighbouring lanes: lanes on pixels of one cell share them,
// and neighbouring pixels of a noisy image often sit in different cells.
// CELLB (the caching records, 156 to 260 bytes each, so that neighbouring B
// cells share no line): B cell mod 4 in place of B cell / 8, grouping the
// pixels of one cell.
template <bool CELLB = false>
__device__ __forceinline__ void chunk_order(const uint8_t* s8, uint32_t N, uint32_t lane, uint32_t* bins,
                                            uint8_t* ord) {
#pragma unroll
  for (int j = 0; j < 4; ++j) bins[lane + 64 * j] = 0u;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  uint32_t key[4], rank[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t P = lane + 64u * j;
    const uint32_t i0 = min(s8[3 * P] * (N - 1) / 255u, N - 2), i1 = min(s8[3 * P + 1] * (N - 1) / 255u, N - 2),
                   i2 = min(s8[3 * P + 2] * (N - 1) / 255u, N - 2);
    key[j] = ((i0 & 7u) << 5) | ((i1 & 7u) << 2) | (CELLB ? (i2 & 3u) : ((i2 >> 3) & 3u));
    rank[j] = atomicAdd(&bins[key[j]], 1u);
  }
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
  // exclusive scan of the counters: 4 per lane, then across the wave
  const uint4 cnt = reinterpret_cast<const uint4*>(bins)[lane];
  const uint32_t tot = cnt.x + cnt.y + cnt.z + cnt.w;
  uint32_t x = tot;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  const uint32_t e = x - tot;
  reinterpret_cast<uint4*>(bins)[lane] = uint4{e, e + cnt.x, e + cnt.x + cnt.y, e + cnt.x + cnt.y + cnt.z};
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < 4; ++j) ord[bins[key[j]] + rank[j]] = (uint8_t)(lane + 64u * j);
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
}

// Trilinear interpolation of a 256-pixel chunk with 2 lanes per pixel (grids
// read through the L2).  In each of 8 rounds the lane pair h takes the pixel
// at position 32 r + h of the chunk's order `ord` (chunk_order); lane bit 0 is
// dB, and each lane gathers its 4 corners (dR dG = 00,
// 01, 10, 11 at that dB).  The two lanes' corners of one (dR, dG) are
// neighbours along B, one 32-byte run (the cell-major form: one 128-byte run
// per pixel), so an instruction touches about 32 lines instead of 64 and the
// vector L1, whose accesses bound these kernels, does about half the work.
// Each lane sums its corners as a product at dR dG = 00 and fused multiply-adds
// at 01, 10, 11; the pair adds its two sums: lut_px's order, so the results
// are lut_px's bits.  The sum of round r ends in lane 2 h + (r mod 2), slot
// r / 2, with its pixel's index in pix.  s8: the chunk's 768 input bytes.
template <int XF, int FORM>
__device__ __forceinline__ void tri_pairs(const f4* __restrict__ nodes, const float* __restrict__ lp, uint32_t N,
                                          const uint8_t* s8, const uint8_t* ord, uint32_t lane, f4 acc[4],
                                          float acc1[4], uint32_t pix[4]) {
  constexpr bool CELL = FORM == kCells;
  const uint32_t db = lane & 1u, h = lane >> 1;
  const uint32_t sR = CELL ? 4u : N * N, sG = CELL ? 2u : N;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t P = ord[32u * r + h];
    uint32_t i0, i1, i2;
    float f0, f1, f2;
    locate_u8(s8[3 * P], N, i0, f0);
    locate_u8(s8[3 * P + 1], N, i1, f1);
    locate_u8(s8[3 * P + 2], N, i2, f2);
    const float r0 = 1.0f - f0, g0 = 1.0f - f1, wb = db ? f2 : 1.0f - f2;
    const uint32_t base = (CELL ? ((i0 * (N - 1) + i1) * (N - 1) + i2) * 8u : (i0 * N + i1) * N + i2) + db;
    uint32_t n[4];
    float w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {  // q = 2 dR + dG
      n[q] = base + (q >> 1) * sR + (q & 1) * sG;
      w[q] = ((q >> 1) ? f0 : r0) * ((q & 1) ? f1 : g0) * wb;
    }
    f4 a = fma4(w[3], nodes[n[3]], fma4(w[2], nodes[n[2]], fma4(w[1], nodes[n[1]], w[0] * nodes[n[0]])));
    float b = 0.0f;
    if (XF == MACT_SCT) {
      // SCT's L: this lane sums the corners with dR = its lane bit, c = 4 dR .. 4 dR + 3, whose L
      // values are two neighbouring pairs along B (the cell-major form: one 16-byte run)
      const uint32_t c0 = base - db + (CELL ? 4u * db : db * sR);
      float4 v;
      if (CELL) {
        v = *reinterpret_cast<const float4*>(lp + c0);
      } else {
        const f2u lo = *reinterpret_cast<const f2u*>(lp + c0), hi = *reinterpret_cast<const f2u*>(lp + c0 + sG);
        v = float4{lo.x, lo.y, hi.x, hi.y};
      }
      const float wr = db ? f0 : r0, wg0 = wr * g0, wg1 = wr * f1, b0 = 1.0f - f2;
      b = __builtin_fmaf(wg1 * f2, v.w, __builtin_fmaf(wg1 * b0, v.z, __builtin_fmaf(wg0 * f2, v.y, wg0 * b0 * v.x)));
    }
    // plus the partner's sum (a float sum does not depend on the order of its two terms)
    a = a + f4{swap1(a.x), swap1(a.y), swap1(a.z), swap1(a.w)};
    if (XF == MACT_SCT) b = b + swap1(b);
    if (db == (uint32_t)(r & 1)) {
      acc[r >> 1] = a;
      acc1[r >> 1] = b;
      pix[r >> 1] = P;
    }
    // one round's gathers in flight at a time: more fit in registers only at a lower occupancy,
    // and measured slower (cell-major CIELAB and HSI 33^3: 16-18%)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Prism, pyramidal and tetrahedral on the cell-major form with 2 lanes per
// pixel: all of a pixel's corners lie in its cell's 128-byte run, so the lane
// pair of a pixel (position 32 r + h of `ord` in round r of 8, as in
// tri_pairs) touches one line per instruction.  Both lanes take the method's corners and weights; lane bit 0
// picks the even or the odd corner ids, and each lane sums its chain (a
// product, then fused multiply-adds in id order, SCT's L alike); the pair adds
// the two sums.  lut_px's order, so the results are lut_px's bits.
template <int METHOD, int XF, bool SORTED>
__device__ __forceinline__ void cell_pairs(const f4* __restrict__ nodes, const float* __restrict__ lp, uint32_t N,
                                           const uint8_t* s8, const uint8_t* ord, uint32_t lane, f4 acc[4],
                                           float acc1[4], uint32_t pix[4]) {
  constexpr int K = Corners<METHOD>::K;
  const uint32_t db = lane & 1u, h = lane >> 1;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t P = SORTED ? ord[32u * r + h] : 32u * r + h;
    uint32_t i0, i1, i2;
    float f0, f1, f2;
    locate_u8(s8[3 * P], N, i0, f0);
    locate_u8(s8[3 * P + 1], N, i1, f1);
    locate_u8(s8[3 * P + 2], N, i2, f2);
    uint32_t off[8];
    float w[8];
    Corners<METHOD>::get(f0, f1, f2, 4u, 2u, off, w);
    const uint32_t base = ((i0 * (N - 1) + i1) * (N - 1) + i2) * 8u;
    f4 a = {0.0f, 0.0f, 0.0f, 0.0f};
    float b = 0.0f;
#pragma unroll
    for (int j = 0; 2 * j < K; ++j) {
      // corner 2 j + db; with K odd the odd lane has none at the last step
      const bool has = 2 * j + 1 < K || db == 0;
      const uint32_t n = base + (db ? off[2 * j + 1 < K ? 2 * j + 1 : 2 * j] : off[2 * j]);
      const float wc = db ? w[2 * j + 1 < K ? 2 * j + 1 : 2 * j] : w[2 * j];
      if (has) {
        const f4 v = nodes[n];
        a = j == 0 ? wc * v : fma4(wc, v, a);
        if (XF == MACT_SCT) b = j == 0 ? wc * lp[n] : __builtin_fmaf(wc, lp[n], b);
      }
    }
    // plus the partner's sum (a float sum does not depend on the order of its two terms)
    a = a + f4{swap1(a.x), swap1(a.y), swap1(a.z), swap1(a.w)};
    if (XF == MACT_SCT) b = b + swap1(b);
    if (db == (uint32_t)(r & 1)) {
      acc[r >> 1] = a;
      acc1[r >> 1] = b;
      pix[r >> 1] = P;
    }
    // one round's gathers in flight at a time, as in tri_pairs
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int METHOD, int XF, int FORM, bool BRANCH = false>
__device__ __forceinline__ void lut_px_u8(const f4* __restrict__ nodes, const float* __restrict__ lp, uint32_t N,
                                          uint32_t sR, uint32_t sG, uint32_t r, uint32_t g, uint32_t b, float o[3]) {
  uint32_t i[3];
  float f[3];
  locate_u8(r, N, i[0], f[0]);
  locate_u8(g, N, i[1], f[1]);
  locate_u8(b, N, i[2], f[2]);
  lut_px<METHOD, XF, FORM, BRANCH>(nodes, lp, N, sR, sG, i, f, o);
}

// Node entries of a LUT of size N (packed N^3, cell-major 8 (N-1)^3), after
// which SCT's L plane starts; and the float4 units of the whole buffer
// (caching: (N-1)^3 records of 13 C floats, rounded up to a float4).
template <int FORM>
__device__ __forceinline__ uint32_t lut_entries(uint32_t N) {
  return FORM == kCells ? 8u * (N - 1) * (N - 1) * (N - 1) : N * N * N;
}

template <int XF, int FORM>
__device__ __forceinline__ uint32_t lut_f4_units(uint32_t N) {
  if (FORM == kCache) return ((N - 1) * (N - 1) * (N - 1) * 13u * CacheC<XF>::C + 3u) / 4u;
  const uint32_t e = lut_entries<FORM>(N);
  return XF == MACT_SCT ? e + (e + 3) / 4 : e;
}

// Any element type, layout and stride: one pixel per lane step.  LDS: the
// buffer (any form) staged in LDS.
template <int METHOD, int XF, bool LDS, int FORM>
__global__ __launch_bounds__(1024) void k_lut(const f4* __restrict__ lut, uint32_t N, KImage src, KImage dst,
                                              uint32_t n_px) {
  extern __shared__ f4 s_lut[];
  const f4* nodes = lut;
  if (LDS) {
    const uint32_t n_f4 = lut_f4_units<XF, FORM>(N);
    for (uint32_t i = threadIdx.x; i < n_f4; i += blockDim.x) s_lut[i] = lut[i];
    __syncthreads();
    nodes = s_lut;
  }
  const float* lp = reinterpret_cast<const float*>(nodes + lut_entries<FORM>(N));
  const bool u8 = src.dtype == MACT_U8;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n_px; p += stride) {
    float v[3], o[3];
    load_px(src, p, v);
    uint32_t i[3];
    float f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (u8) locate_u8((uint32_t)v[c], N, i[c], f[c]);
      else locate_f(src.dtype == MACT_U16 ? v[c] * kInv65535 : v[c], N, i[c], f[c]);
    }
    lut_px<METHOD, XF, FORM>(nodes, lp, N, N * N, N, i, f, o);
    store_px(dst, p, o);
  }
}

// Packed 8-bit HWC -> packed float32 HWC.  Each wave takes 256-pixel chunks
// (grid-stride, since a staged LUT is worth keeping); each lane reads 12
// bytes (4 pixels) of the chunk, so the wave's load is one contiguous run.
// SPREAD = false: lane l interpolates its own pixels 4 l .. 4 l + 3.
// SPREAD = true: the chunk's bytes go through the wave's LDS slice and lane l
// interpolates pixels l, l + 64, l + 128, l + 192, so the 64 lanes of one
// corner gather are 64 consecutive pixels, whose corners on smooth images
// often share cache lines; there trilinear, and every method on a cell-major
// grid above 256 KB, take two lanes per pixel (tri_pairs, cell_pairs).
// Either way the results leave through the wave's LDS slice as 1 KB
// contiguous stores.  LDS holds the LUT (when LDS; packed grids with the node
// strides sR, sG, else N^2, N) followed by 3 KB per wave.
template <int METHOD, int XF, bool LDS, int FORM, bool SPREAD>
__global__ __launch_bounds__(1024) void k_lut4(const f4* __restrict__ lut, uint32_t N, uint32_t sR, uint32_t sG,
                                               const uint8_t* __restrict__ in, float* __restrict__ out, uint32_t n_px) {
  static_assert(!(LDS && SPREAD), "the consecutive-lane form gathers from global memory (its loads may be unaligned)");
  extern __shared__ f4 smem[];
  const uint32_t n_ent = lut_entries<FORM>(N);
  const uint32_t n_f4 = lut_f4_units<XF, FORM>(N);
  const f4* nodes = lut;
  const float* lp = reinterpret_cast<const float*>(lut + n_ent);
  f4* tbuf = smem;
  if (LDS) {
    if (FORM == kPacked && (sR != N * N || sG != N)) {
      // staged with padded strides: node (i, j, k) to i sR + j sG + k, the L plane (SCT) alike
      // after N sR entries
      const uint32_t nn = N * N, e = N * sR;
      float* ld = reinterpret_cast<float*>(smem + e);
      for (uint32_t t = threadIdx.x; t < n_ent; t += blockDim.x) {
        const uint32_t r = t / nn, g = (t - r * nn) / N, d = r * sR + g * sG + (t - r * nn - g * N);
        smem[d] = lut[t];
        if (XF == MACT_SCT) ld[d] = lp[t];
      }
      tbuf = smem + e + (XF == MACT_SCT ? (e + 3) / 4 : 0);
      lp = ld;
    } else {
      for (uint32_t i = threadIdx.x; i < n_f4; i += blockDim.x) smem[i] = lut[i];
      tbuf = smem + n_f4;
      lp = reinterpret_cast<const float*>(smem + n_ent);
    }
    __syncthreads();
    nodes = smem;
  }
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  f4* s = tbuf + wv * 192;
  const uint32_t n_chunks = n_px >> 8;
  for (uint32_t c = blockIdx.x * nw + wv; c < n_chunks; c += gridDim.x * nw) {
    const uint3 w = reinterpret_cast<const uint3*>(in)[(size_t)c * 64 + lane];
    if (!SPREAD) {
      float o[12];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        lut_px_u8<METHOD, XF, FORM>(nodes, lp, N, sR, sG, byte_of(w, 3 * j), byte_of(w, 3 * j + 1),
                                    byte_of(w, 3 * j + 2), o + 3 * j);
        // SCT's trilinear sums: two pixels' gathers in flight at most, or the corners outgrow the registers
        if (METHOD == MACT_TRILINEAR && XF == MACT_SCT && (j & 1)) __builtin_amdgcn_sched_barrier(0);
      }
      __builtin_amdgcn_wave_barrier();
      s[3 * lane] = f4{o[0], o[1], o[2], o[3]};
      s[3 * lane + 1] = f4{o[4], o[5], o[6], o[7]};
      s[3 * lane + 2] = f4{o[8], o[9], o[10], o[11]};
    } else {
      // the chunk's 768 input bytes at the start of the wave's slice (bytes 0..767 of 3 KB)
      uint32_t* s32 = reinterpret_cast<uint32_t*>(s);
      const uint8_t* s8 = reinterpret_cast<const uint8_t*>(s);
      float* sf = reinterpret_cast<float*>(s);
      __builtin_amdgcn_wave_barrier();
      s32[3 * lane] = w.x;
      s32[3 * lane + 1] = w.y;
      s32[3 * lane + 2] = w.z;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the bytes have landed
      __builtin_amdgcn_wave_barrier();
      // the pixels grouped by cache line (after the wave slices: 256 counters and the order per
      // wave), except for prism and pyramidal on cell-major grids, whose kernels are bound by their
      // arithmetic, which the ordering adds to (17^3, 33^3: -12 to -23%)
      constexpr bool SORT = !(FORM == kCells && (METHOD == MACT_PRISM || METHOD == MACT_PYRAMIDAL));
      uint32_t* bins = reinterpret_cast<uint32_t*>(tbuf + nw * 192) + wv * 320;
      uint8_t* ord = reinterpret_cast<uint8_t*>(bins + 256);
      if (SORT) chunk_order<FORM == kCache>(s8, N, lane, bins, ord);
      // two lanes per pixel: trilinear on the packed and cell-major grids; the other methods on
      // cell-major grids of more than 256 KB (17^3 and up: +2 to +38%; on 9^3, 64 KB, pyramidal
      // lost 19% and the others nothing)
      if ((METHOD == MACT_TRILINEAR && FORM != kCache) || (FORM == kCells && (N - 1) * (N - 1) * (N - 1) > 2048u)) {
        f4 acc[4];
        float acc1[4];
        uint32_t pix[4];
        if (METHOD == MACT_TRILINEAR)
          tri_pairs<XF, FORM>(nodes, lp, N, s8, ord, lane, acc, acc1, pix);
        else
          cell_pairs<METHOD, XF, SORT>(nodes, lp, N, s8, ord, lane, acc, acc1, pix);
        __builtin_amdgcn_s_waitcnt(0xc07f);  // every lane has read its bytes before the slice is reused
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          float o[3];
          lut_out<XF>(acc[m], acc1[m], o);
          const uint32_t p = pix[m];
          sf[3 * p] = o[0];
          sf[3 * p + 1] = o[1];
          sf[3 * p + 2] = o[2];
        }
      } else {
        uint32_t rgb[4][3], pix[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          pix[j] = SORT ? ord[lane + 64 * j] : lane + 64u * j;
#pragma unroll
          for (int q = 0; q < 3; ++q) rgb[j][q] = s8[3 * pix[j] + q];
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);  // every lane has read its bytes before the slice is reused
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float o[3];
          lut_px_u8<METHOD, XF, FORM, true>(nodes, lp, N, sR, sG, rgb[j][0], rgb[j][1], rgb[j][2], o);
          const uint32_t p = pix[j];
          sf[3 * p] = o[0];
          sf[3 * p + 1] = o[1];
          sf[3 * p + 2] = o[2];
          // one pixel's gathers in flight at a time: hoisting the next pixels' gathers costs
          // occupancy and measured slower (the caching form's trilinear, 33^3: 59-92 vs 102 Gpx/s).
          // The caching form's tetrahedral, 4 entries a pixel, takes two pixels at a time, except
          // for SCT's 20-byte entries (CIELAB 33^3 104 -> 109 Gpx/s, HSI 17^3 166 -> 181; SCT -3%)
          constexpr bool kTwo = FORM == kCache && METHOD == MACT_TETRAHEDRAL && XF != MACT_SCT;
          if (!kTwo || (j & 1)) __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): every lane's LDS writes have landed
    __builtin_amdgcn_wave_barrier();
    f4* d = reinterpret_cast<f4*>(out) + (size_t)c * 192;
#pragma unroll
    for (int q = 0; q < 3; ++q) __builtin_nontemporal_store(s[q * 64 + lane], d + q * 64 + lane);
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
  }
  const uint32_t tail0 = n_chunks << 8;
  if (blockIdx.x == 0)
    for (uint32_t p = tail0 + threadIdx.x; p < n_px; p += blockDim.x) {
      float o[3];
      lut_px_u8<METHOD, XF, FORM>(nodes, lp, N, sR, sG, in[3 * (size_t)p], in[3 * (size_t)p + 1], in[3 * (size_t)p + 2],
                                  o);
      out[3 * (size_t)p] = o[0];
      out[3 * (size_t)p + 1] = o[1];
      out[3 * (size_t)p + 2] = o[2];
    }
}

// Cell-major form from the packed grid: entry t = cell 8 + c is corner c of
// cell (i, j, k), the packed node (i + dR, j + dG, k + dB); with `lplanes`, the
// node's L (SCT) goes to the cells' L plane as well.  A plain copy.
__global__ __launch_bounds__(256) void k_lut_cells(const f4* __restrict__ nodes, uint32_t N, bool lplanes,
                                                   f4* __restrict__ cells, uint32_t n_ent) {
  const uint32_t M = N - 1;
  const float* lsrc = reinterpret_cast<const float*>(nodes + N * N * N);
  float* ldst = reinterpret_cast<float*>(cells + n_ent);
  for (uint32_t t = blockIdx.x * 256u + threadIdx.x; t < n_ent; t += gridDim.x * 256u) {
    const uint32_t c = t & 7u, cell = t >> 3;
    const uint32_t k = cell % M, j = (cell / M) % M, i = cell / (M * M);
    const uint32_t node = ((i + (c >> 2)) * N + (j + ((c >> 1) & 1u))) * N + (k + (c & 1u));
    cells[t] = nodes[node];
    if (lplanes) ldst[t] = lsrc[node];
  }
}

// ---------------------------------------------------------------- host

int max_lds_bytes() {
  static std::mutex mu;
  static int cache[64] = {0};
  const int d = current_device();
  std::lock_guard<std::mutex> g(mu);
  if (d >= 0 && d < 64 && cache[d]) return cache[d];
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, d) != hipSuccess || v <= 0) v = 65536;
  if (d >= 0 && d < 64) cache[d] = v;
  return v;
}

template <typename K>
static hipError_t allow_lds(K k, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Node strides of a packed grid staged in LDS.  A float4 node covers 4 of the
// LDS's 4-byte banks, so node n sits in bank group n mod 16, and the lanes of
// one gather mostly hold nodes of a small neighbourhood (neighbouring pixels).
// Unpadded, the strides N and N^2 are both 1 mod 16 at 17^3: steps along R, G
// and B land on the same group, and the lanes' gathers collide.  G rows are
// padded to a stride of 3 mod 16 and R planes to 9 mod 16, which spreads a
// 3 x 3 x 3 neighbourhood over the groups (a simulation of the batch's pixel
// spread: at most 1.3 nodes per group per 16 lanes against 3.0), where the
// grid still fits `room` bytes; `bytes` becomes the staged size.
static void lds_strides(int xform, uint32_t N, size_t room, uint32_t& sR, uint32_t& sG, size_t& bytes) {
  uint32_t g = N;
  while (g % 16 != 3) ++g;
  uint32_t r = N * g;
  while (r % 16 != 9) ++r;
  const size_t e = (size_t)N * r;
  const size_t b = lut_f4s(xform, e) * sizeof(f4);
  if (b > room) return;
  sR = r;
  sG = g;
  bytes = b;
}

// Launch shapes.  LDS-staged grid: 1024-thread workgroups, one or two per CU
// (as many copies of the grid as the CU's LDS holds), grid-stride.  Grid
// gathered through the L2 (and every cell-major grid): 256-thread
// workgroups, eight per CU.
template <int METHOD, int XF, int FORM>
static hipError_t launch_lut(const f4* lut, uint32_t N, const HostImage& hi, const HostImage& ho, int64_t n0,
                             int64_t cnt, uint32_t n_px, hipStream_t st) {
  constexpr bool CELL = FORM == kCells;  // cell-major grids are always read through the L2
  const size_t bytes = FORM == kCache ? lut_cache_size(XF, N) : lut_f4s(XF, (size_t)N * N * N) * sizeof(f4);
  const size_t lds_max = (size_t)max_lds_bytes();
  const void* ip = static_cast<const char*>(hi.data) + (size_t)(n0 * hi.bs) * hi.esize;
  float* op = static_cast<float*>(ho.data) + (size_t)(n0 * ho.bs);
  const bool fast = hi.dtype == MACT_U8 && hi.layout == MACT_HWC && hi.packed && ho.dtype == MACT_F32 &&
                    ho.layout == MACT_HWC && ho.packed && (uintptr_t)ip % 4 == 0 && (uintptr_t)op % 16 == 0;
  const size_t t_lds = 16 * 192 * sizeof(f4);  // k_lut4 with 1024 threads: 16 waves x 3 KB
  // a grid that fits LDS alone but not beside k_lut4's transpose buffers is still worth
  // staging: k_lut below
  if (fast && (CELL || bytes + t_lds <= lds_max || bytes > lds_max)) {
    const bool lds = !CELL && bytes + t_lds <= lds_max;
    const unsigned block = lds ? 1024 : 256;
    uint32_t sR = N * N, sG = N;
    size_t staged = bytes;
    if (lds && FORM == kPacked) lds_strides(XF, N, lds_max - t_lds, sR, sG, staged);
    // per wave: the 3 KB slice, and for gathers through the L2 the chunk's counters and order (1280 B)
    const size_t shm = (lds ? staged : 0) + (size_t)(block / 64) * (192 * sizeof(f4) + (lds ? 0 : 1280));
    const uint64_t chunks = std::max<uint64_t>(1, n_px >> 8);
    // a staged grid is worth keeping: one or two resident workgroups per CU stride over the image;
    // gathers from global memory: the grid covers the image once, one chunk per wave
    // (tetrahedral: one, which measured +8% for CIELAB 9^3, where two fit, and the same elsewhere)
    const uint64_t per_cu =
        METHOD == MACT_TETRAHEDRAL ? 1 : std::max<uint64_t>(1, std::min<uint64_t>(2, lds_max / shm));
    const uint64_t need = (chunks + block / 64 - 1) / (block / 64);
    const unsigned grid = (unsigned)std::max<uint64_t>(1, lds ? std::min<uint64_t>(need, (uint64_t)device_cus() * per_cu)
                                                              : std::min<uint64_t>(need, 0x7fffffffu));
    const uint8_t* in8 = static_cast<const uint8_t*>(ip);
    // lanes on consecutive pixels pay off for gathers through the L1 (33^3: +13-16%, SCT +44%
    // on smooth images) but not for LDS-staged grids (-0 to -6%)
    if (lds) {
      auto k = k_lut4<METHOD, XF, true, FORM, false>;
      hipError_t e = allow_lds(k, shm);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(grid), dim3(block), shm, st, lut, N, sR, sG, in8, op, n_px);
    } else {
      auto k = k_lut4<METHOD, XF, false, FORM, true>;
      hipLaunchKernelGGL(k, dim3(grid), dim3(block), shm, st, lut, N, sR, sG, in8, op, n_px);
    }
    return hipGetLastError();
  }
  const KImage s = kimage(hi, n0, cnt), d = kimage(ho, n0, cnt);
  const bool lds = !CELL && bytes <= lds_max;
  const unsigned block = lds ? 1024 : 256;
  const uint64_t need = (n_px + block - 1) / block;
  // a staged grid: one or two resident workgroups per CU stride over the image; otherwise the grid
  // covers the image once
  const uint64_t per_cu = std::max<uint64_t>(1, std::min<uint64_t>(2, lds_max / std::max<size_t>(bytes, 1)));
  const unsigned grid = (unsigned)std::max<uint64_t>(1, lds ? std::min<uint64_t>(need, (uint64_t)device_cus() * per_cu)
                                                            : std::min<uint64_t>(need, 0x7fffffffu));
  if (lds) {
    auto k = k_lut<METHOD, XF, true, FORM>;
    hipError_t e = allow_lds(k, bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), bytes, st, lut, N, s, d, n_px);
  } else {
    hipLaunchKernelGGL((k_lut<METHOD, XF, false, FORM>), dim3(grid), dim3(block), 0, st, lut, N, s, d, n_px);
  }
  return hipGetLastError();
}

template <int XF, int FORM>
static hipError_t launch_lut_m(int method, const f4* lut, uint32_t N, const HostImage& hi, const HostImage& ho,
                               int64_t n0, int64_t cnt, uint32_t n_px, hipStream_t st) {
  switch (method) {
    case MACT_TRILINEAR: return launch_lut<MACT_TRILINEAR, XF, FORM>(lut, N, hi, ho, n0, cnt, n_px, st);
    case MACT_PRISM: return launch_lut<MACT_PRISM, XF, FORM>(lut, N, hi, ho, n0, cnt, n_px, st);
    case MACT_PYRAMIDAL: return launch_lut<MACT_PYRAMIDAL, XF, FORM>(lut, N, hi, ho, n0, cnt, n_px, st);
    default: return launch_lut<MACT_TETRAHEDRAL, XF, FORM>(lut, N, hi, ho, n0, cnt, n_px, st);
  }
}

// lut_interp and lut_cells_interp: validation, then one launch per run of
// images of fewer than 2^31 pixels.
template <int FORM>
static mact_status interp_common(const char* what, const float* dev_lut, int32_t n, int32_t xform, int32_t method,
                                 const mact_image* in, const mact_image* out, void* hip_stream) {
  if (!dev_lut) return fail(MACT_E_INVALID, "%s: LUT pointer is NULL", what);
  if (xform < MACT_LAB || xform > MACT_LUV || n < 2 || n > 256)
    return fail(MACT_E_INVALID, "%s: transform %d / size %d invalid", what, xform, n);
  if (method < MACT_TRILINEAR || method > MACT_TETRAHEDRAL) return fail(MACT_E_INVALID, "%s: method %d", what, method);
  if ((uintptr_t)dev_lut % 16) return fail(MACT_E_INVALID, "%s: LUT not 16-byte aligned", what);
  HostImage hi, ho;
  mact_status s;
  char nm[64];
  std::snprintf(nm, sizeof nm, "%s: in", what);
  if ((s = resolve_image(in, false, nm, &hi)) != MACT_OK) return s;
  std::snprintf(nm, sizeof nm, "%s: out", what);
  if ((s = resolve_image(out, true, nm, &ho)) != MACT_OK) return s;
  if ((s = check_same_shape(hi, ho, nm)) != MACT_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const f4* lut = reinterpret_cast<const f4*>(dev_lut);
  const int64_t per = images_per_stream_launch(hi, ho);
  for (int64_t n0 = 0; n0 < hi.N; n0 += per) {
    const int64_t cnt = std::min(per, hi.N - n0);
    const uint32_t n_px = (uint32_t)(cnt * hi.W * hi.H);
    hipError_t e;
    if (xform == MACT_LAB) e = launch_lut_m<MACT_LAB, FORM>(method, lut, n, hi, ho, n0, cnt, n_px, st);
    else if (xform == MACT_HSI) e = launch_lut_m<MACT_HSI, FORM>(method, lut, n, hi, ho, n0, cnt, n_px, st);
    else if (xform == MACT_LUV) e = launch_lut_m<MACT_LUV, FORM>(method, lut, n, hi, ho, n0, cnt, n_px, st);
    else e = launch_lut_m<MACT_SCT, FORM>(method, lut, n, hi, ho, n0, cnt, n_px, st);
    std::snprintf(nm, sizeof nm, "%s: launch", what);
    if ((s = hip_check(e, nm)) != MACT_OK) return s;
  }
  return MACT_OK;
}

}  // namespace mact

using namespace mact;

extern "C" size_t lut_bytes(int32_t xform, int32_t n) {
  if (xform < MACT_LAB || xform > MACT_LUV || n < 2 || n > 256) return 0;
  return lut_f4s(xform, (size_t)n * n * n) * sizeof(f4);
}

extern "C" mact_status lut_build(int32_t xform, int32_t n, int32_t gamma, float* dev_lut, size_t bytes,
                                 void* hip_stream) {
  clear_error();
  const size_t need = lut_bytes(xform, n);
  if (need == 0) return fail(MACT_E_INVALID, "lut_build: transform %d / size %d invalid (n in 2..256)", xform, n);
  if (!dev_lut) return fail(MACT_E_INVALID, "lut_build: dev_lut is NULL");
  if (bytes < need) return fail(MACT_E_INVALID, "lut_build: %zu bytes < %zu needed", bytes, need);
  if (gamma < MACT_GAMMA_BT709 || gamma > MACT_GAMMA_NONE) return fail(MACT_E_INVALID, "lut_build: gamma %d", gamma);
  const size_t n3 = (size_t)n * n * n;
  std::vector<float> host(need / sizeof(float), 0.0f);
  float* lplane = host.data() + 4 * n3;  // SCT's L, one float per node
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        const double rgb[3] = {(double)i / (n - 1), (double)j / (n - 1), (double)k / (n - 1)};
        double o[3];
        const size_t node = (size_t)(i * n + j) * n + k;
        float* dst = &host[node * 4];
        if (xform == MACT_LAB) {
          exact_lab(rgb, gamma, o);
          dst[0] = (float)o[0]; dst[1] = (float)o[1]; dst[2] = (float)o[2];
        } else if (xform == MACT_LUV) {
          exact_luv(rgb, gamma, o);
          dst[0] = (float)o[0]; dst[1] = (float)o[1]; dst[2] = (float)o[2];
        } else if (xform == MACT_HSI) {
          exact_hsi(rgb, o);
          dst[0] = (float)std::cos(o[0]); dst[1] = (float)std::sin(o[0]); dst[2] = (float)o[1]; dst[3] = (float)o[2];
        } else {
          exact_sct(rgb, o);
          dst[0] = (float)std::cos(o[1]); dst[1] = (float)std::sin(o[1]);
          dst[2] = (float)std::cos(o[2]); dst[3] = (float)std::sin(o[2]);
          lplane[node] = (float)o[0];
        }
      }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  mact_status s = hip_check(hipMemcpyAsync(dev_lut, host.data(), need, hipMemcpyHostToDevice, st), "lut_build: copy");
  if (s != MACT_OK) return s;
  return hip_check(hipStreamSynchronize(st), "lut_build: synchronise");
}

extern "C" mact_status lut_interp(const float* dev_lut, int32_t n, int32_t xform, int32_t method, const mact_image* in,
                                  const mact_image* out, void* hip_stream) {
  clear_error();
  return interp_common<kPacked>("lut_interp", dev_lut, n, xform, method, in, out, hip_stream);
}

extern "C" size_t lut_cells_bytes(int32_t xform, int32_t n) {
  if (xform < MACT_LAB || xform > MACT_LUV || n < 2 || n > 256) return 0;
  const size_t m = (size_t)(n - 1);
  return lut_f4s(xform, m * m * m * 8) * sizeof(f4);
}

extern "C" mact_status lut_cells_build(const float* dev_lut, int32_t n, int32_t xform, float* dev_cells, size_t bytes,
                                       void* hip_stream) {
  clear_error();
  const size_t need = lut_cells_bytes(xform, n);
  if (need == 0) return fail(MACT_E_INVALID, "lut_cells_build: transform %d / size %d invalid (n in 2..256)", xform, n);
  if (!dev_lut || !dev_cells) return fail(MACT_E_INVALID, "lut_cells_build: NULL LUT pointer");
  if ((uintptr_t)dev_lut % 16 || (uintptr_t)dev_cells % 16)
    return fail(MACT_E_INVALID, "lut_cells_build: LUT pointers must be 16-byte aligned");
  if (bytes < need) return fail(MACT_E_INVALID, "lut_cells_build: %zu bytes < %zu needed", bytes, need);
  const size_t m = (size_t)(n - 1);
  const uint32_t n_ent = (uint32_t)(m * m * m * 8);
  const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n_ent + 255) / 256, (uint64_t)device_cus() * 8));
  hipLaunchKernelGGL(k_lut_cells, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     reinterpret_cast<const f4*>(dev_lut), (uint32_t)n, xform == MACT_SCT, reinterpret_cast<f4*>(dev_cells),
                     n_ent);
  return hip_check(hipGetLastError(), "lut_cells_build: launch");
}

extern "C" mact_status lut_cells_interp(const float* dev_cells, int32_t n, int32_t xform, int32_t method,
                                        const mact_image* in, const mact_image* out, void* hip_stream) {
  clear_error();
  return interp_common<kCells>("lut_cells_interp", dev_cells, n, xform, method, in, out, hip_stream);
}

extern "C" size_t lut_cache_bytes(int32_t xform, int32_t n) {
  if (xform < MACT_LAB || xform > MACT_LUV || n < 2 || n > 256) return 0;
  return lut_cache_size(xform, (size_t)n);
}

extern "C" mact_status lut_cache_build(int32_t xform, int32_t n, int32_t gamma, float* dev_cache, size_t bytes,
                                       void* hip_stream) {
  clear_error();
  const size_t need = lut_cache_bytes(xform, n);
  if (need == 0) return fail(MACT_E_INVALID, "lut_cache_build: transform %d / size %d invalid (n in 2..256)", xform, n);
  if (!dev_cache) return fail(MACT_E_INVALID, "lut_cache_build: dev_cache is NULL");
  if ((uintptr_t)dev_cache % 16) return fail(MACT_E_INVALID, "lut_cache_build: dev_cache not 16-byte aligned");
  if (bytes < need) return fail(MACT_E_INVALID, "lut_cache_build: %zu bytes < %zu needed", bytes, need);
  if (gamma < MACT_GAMMA_BT709 || gamma > MACT_GAMMA_NONE) return fail(MACT_E_INVALID, "lut_cache_build: gamma %d", gamma);
  // the components of every node in FP64: linear channels as they are, angles as (cos, sin)
  const int C = xform == MACT_SCT ? 5 : xform == MACT_HSI ? 4 : 3;
  const size_t n3 = (size_t)n * n * n;
  std::vector<double> comp(n3 * C);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        const double rgb[3] = {(double)i / (n - 1), (double)j / (n - 1), (double)k / (n - 1)};
        double o[3];
        double* c = &comp[((size_t)(i * n + j) * n + k) * C];
        if (xform == MACT_LAB || xform == MACT_LUV) {
          if (xform == MACT_LAB) exact_lab(rgb, gamma, o);
          else exact_luv(rgb, gamma, o);
          c[0] = o[0]; c[1] = o[1]; c[2] = o[2];
        } else if (xform == MACT_HSI) {
          exact_hsi(rgb, o);
          c[0] = std::cos(o[0]); c[1] = std::sin(o[0]); c[2] = o[1]; c[3] = o[2];
        } else {
          exact_sct(rgb, o);
          c[0] = o[0];
          c[1] = std::cos(o[1]); c[2] = std::sin(o[1]);
          c[3] = std::cos(o[2]); c[4] = std::sin(o[2]);
        }
      }
  // record of cell (i, j, k): the node value and the 12 edge differences, in FP64, rounded once
  const int m = n - 1;
  std::vector<float> host(need / sizeof(float), 0.0f);
  auto node = [&](int i, int j, int k) { return &comp[((size_t)(i * n + j) * n + k) * C]; };
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      for (int k = 0; k < m; ++k) {
        float* r = &host[((size_t)(i * m + j) * m + k) * 13 * C];
        const double* c0 = node(i, j, k);
        for (int q = 0; q < C; ++q) r[q] = (float)c0[q];
        for (int u = 0; u < 2; ++u)
          for (int v = 0; v < 2; ++v) {
            const double *r0 = node(i, j + u, k + v), *r1 = node(i + 1, j + u, k + v);  // R edge at (g, b) = (u, v)
            const double *g0 = node(i + u, j, k + v), *g1 = node(i + u, j + 1, k + v);  // G edge at (r, b) = (u, v)
            const double *b0 = node(i + u, j + v, k), *b1 = node(i + u, j + v, k + 1);  // B edge at (r, g) = (u, v)
            for (int q = 0; q < C; ++q) {
              r[(1 + 2 * u + v) * C + q] = (float)(r1[q] - r0[q]);
              r[(5 + 2 * u + v) * C + q] = (float)(g1[q] - g0[q]);
              r[(9 + 2 * u + v) * C + q] = (float)(b1[q] - b0[q]);
            }
          }
      }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  mact_status s = hip_check(hipMemcpyAsync(dev_cache, host.data(), need, hipMemcpyHostToDevice, st),
                            "lut_cache_build: copy");
  if (s != MACT_OK) return s;
  return hip_check(hipStreamSynchronize(st), "lut_cache_build: synchronise");
}

extern "C" mact_status lut_cache_interp(const float* dev_cache, int32_t n, int32_t xform, int32_t method,
                                        const mact_image* in, const mact_image* out, void* hip_stream) {
  clear_error();
  return interp_common<kCache>("lut_cache_interp", dev_cache, n, xform, method, in, out, hip_stream);
}
