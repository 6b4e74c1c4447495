// Batched form: one graph over many images of uneven sizes, mixed element
// types, layouts and transforms.
//
// A plan groups its images into classes (below, k_batch_cls): the images with
// packed 8-bit, 16-bit or float16 HWC input and packed float32 HWC output, per
// transform, coefficient set and transfer function, each class run by a
// kernel specialised like the plain hot kernel; everything else by k_batch.
// The served form's small batches use k_batch alone.
//
// Every image is cut into tiles of `tile` pixels; tile t belongs to the image
// i with tile_start[i] <= t < tile_start[i+1].  The grid either covers the
// tile list once (one workgroup per tile) or, sized to the GPU, walks it (tile
// t, t + gridDim.x, ...), so that the workgroups in flight work on
// neighbouring tiles (one contiguous run of tiles per workgroup measured 7%
// slower).  Each workgroup finds its tile's image in the plan's per-tile map
// (or, for the served form's small batches, by a wave-uniform binary search
// over tile_start), then transforms the tile's pixels with the same per-pixel
// functions as the plain kernels -- packed 8-bit, 16-bit and float16 HWC ->
// float32 HWC tiles through the 4-pixel LDS-transposed path, everything else
// one pixel per lane -- so outputs are bitwise equal to mact_transform's.  The
// plan captures the launch in a HIP graph.  The launch shape (block, tile,
// vector path, waves per CU or one workgroup per tile) comes from an
// autotuner that times candidates on the actual batch and caches the winner
// per GPU and shape class (optionally in a JSON file named by
// MACT_AUTOTUNE_CACHE).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "launch.h"
#include "stream.h"

namespace mact {

#include "gamma_table.inc"

typedef float f4 __attribute__((ext_vector_type(4)));

template <int DEG, int VEC>
__global__ __launch_bounds__(1024) void k_batch(const BDesc* __restrict__ descs, const KCoef* __restrict__ coefs,
                                                const uint32_t* __restrict__ tile_start,
                                                const uint32_t* __restrict__ tile_img, int32_t count,
                                                uint32_t tile0, uint32_t total_tiles, uint32_t tile) {
  __shared__ float gtab[3][256];
  extern __shared__ f4 s_out[];  // VEC == 4: 192 float4 per wave
  for (uint32_t i = threadIdx.x; i < 768u; i += blockDim.x) gtab[i >> 8][i & 255u] = k_gamma_table[i >> 8][i & 255u];
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (uint32_t t = tile0 + blockIdx.x; t < total_tiles; t += gridDim.x) {
    int32_t lo = 0;
    if (tile_img) {
      lo = (int32_t)tile_img[t];
    } else {
      int32_t hi = count - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= t) lo = mid;
        else hi = mid - 1;
      }
    }
    const BDesc& d = descs[lo];
    const KCoef& k = coefs[d.coef];
    const uint32_t p0 = (t - tile_start[lo]) * tile;
    const uint32_t p1 = min(p0 + tile, d.n_px);
    const float* g = gtab[d.gamma];
    uint32_t pstart = p0;
    if (VEC == 4 && d.fast) {
      // full 256-pixel chunks of the tile, one per wave at a time (p0 is a multiple of 256)
      const uint32_t nchunk = (p1 - p0) >> 8;
      f4* s = s_out + wv * 192;
      for (uint32_t c = wv; c < nchunk; c += nw) {
        const uint32_t cp = p0 + (c << 8);
        const uint3* win = reinterpret_cast<const uint3*>(d.src.ptr);
        float o[12];
        if (d.fast == 1) {  // 8-bit: 12 bytes (4 pixels) per lane
          const uint3 w = win[(cp >> 2) + lane];
          if (k.xform == MACT_LAB) px4_u8<MACT_LAB, DEG>(k, g, w, o);
          else if (k.xform == MACT_LUV) px4_u8<MACT_LUV, DEG>(k, g, w, o);
          else if (k.xform == MACT_HSI) px4_u8<MACT_HSI, DEG>(k, g, w, o);
          else px4_u8<MACT_SCT, DEG>(k, g, w, o);
        } else if (d.fast == 2) {  // float16: 24 bytes per lane
          const uint3 wa = win[(cp >> 1) + 2 * lane], wb = win[(cp >> 1) + 2 * lane + 1];
          if (k.xform == MACT_LAB) px4_f16<MACT_LAB, DEG>(k, d.gamma, wa, wb, o);
          else if (k.xform == MACT_LUV) px4_f16<MACT_LUV, DEG>(k, d.gamma, wa, wb, o);
          else if (k.xform == MACT_HSI) px4_f16<MACT_HSI, DEG>(k, d.gamma, wa, wb, o);
          else px4_f16<MACT_SCT, DEG>(k, d.gamma, wa, wb, o);
        } else {  // 16-bit codes: 24 bytes per lane
          const uint3 wa = win[(cp >> 1) + 2 * lane], wb = win[(cp >> 1) + 2 * lane + 1];
          if (k.xform == MACT_LAB) px4_u16<MACT_LAB, DEG>(k, d.gamma, wa, wb, o);
          else if (k.xform == MACT_LUV) px4_u16<MACT_LUV, DEG>(k, d.gamma, wa, wb, o);
          else if (k.xform == MACT_HSI) px4_u16<MACT_HSI, DEG>(k, d.gamma, wa, wb, o);
          else px4_u16<MACT_SCT, DEG>(k, d.gamma, wa, wb, o);
        }
        __builtin_amdgcn_wave_barrier();
        s[3 * lane] = f4{o[0], o[1], o[2], o[3]};
        s[3 * lane + 1] = f4{o[4], o[5], o[6], o[7]};
        s[3 * lane + 2] = f4{o[8], o[9], o[10], o[11]};
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): every lane's LDS writes have landed
        __builtin_amdgcn_wave_barrier();
        const StreamBuf dst = wave_stream_buf(reinterpret_cast<f4*>(d.dst.ptr) + (size_t)(cp >> 2) * 3, 3072u);
#pragma unroll
        for (int q = 0; q < 3; ++q) stream_store(dst, (q * 64 + lane) * 16u, s[q * 64 + lane]);
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
      }
      pstart = p0 + (nchunk << 8);
    }
    for (uint32_t p = pstart + threadIdx.x; p < p1; p += blockDim.x) {
      float v[3], o[3];
      load_px(d.src, p, v);
      eval_px<DEG>(k, d.src.dtype, d.gamma, g, v, o);
      store_px(d.dst, p, o);
    }
  }
}

// Class kernels.  A plan sorts its images into classes of one element type
// (packed 8-bit, float16 or 16-bit HWC in, packed float32 HWC out, aligned),
// one transform, one coefficient set and one transfer function, and runs each
// class's tiles with a kernel specialised for it in the plain hot kernel's
// shape: the coefficients are kernel arguments with their leading terms held
// in registers, one decoding table, 256-thread workgroups, two 256-pixel
// chunks per wave (one for 8-bit CIELUV) whose loads are issued first, and the
// wave's results through its LDS slice as 1 KB streaming stores.  k_batch,
// which branches per tile on the transform and element type and evaluates the
// padded degree, measured 25% below the plain kernel on a uniform 64 x 1080p
// batch (4.7-5.0 against 6.4 TB/s): the arithmetic, not the memory, bounds it.
// The tile walk is k_batch's: tile t of [t0, t1) belongs to image tile_img[t];
// a tile is a multiple of 256 pixels and the image's last n_px % 256 pixels go
// one per thread in the tile that holds them.
template <int IN, int DEG, int XF>
__global__ __launch_bounds__(256) void k_batch_cls(const BDesc* __restrict__ descs,
                                                   const uint32_t* __restrict__ tile_start,
                                                   const uint32_t* __restrict__ tile_img, uint32_t t0, uint32_t t1,
                                                   uint32_t tile, KCoef k, int gamma) {
  constexpr int WPC = IN == MACT_U8 ? 1 : 2;                         // 12-byte words per lane per chunk
  constexpr int CPW = (XF == MACT_LUV && IN == MACT_U8) ? 1 : 2;     // chunks per wave, as the plain kernel
  __shared__ f4 s_out[4][CPW * 192];
  __shared__ float gtab[256];
  if (IN == MACT_U8 && (XF == MACT_LAB || XF == MACT_LUV)) {
    gtab[threadIdx.x] = k_gamma_table[gamma][threadIdx.x];
    __syncthreads();
  }
  pin_lead<DEG>(k);
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  for (uint32_t t = t0 + blockIdx.x; t < t1; t += gridDim.x) {
    const uint32_t img = tile_img[t];
    const BDesc& d = descs[img];
    const uint32_t n_px = d.n_px;
    const uint32_t p0 = (t - tile_start[img]) * tile;
    const uint32_t p1 = min(p0 + tile, n_px);
    const uint32_t cend = p1 >> 8;  // full chunks only
    const uint3* win = reinterpret_cast<const uint3*>(d.src.ptr);
    f4* out4 = reinterpret_cast<f4*>(d.dst.ptr);
    for (uint32_t c0 = (p0 >> 8) + wv * CPW; c0 < cend; c0 += 4 * CPW) {
      uint3 w[CPW][WPC];
#pragma unroll
      for (int j = 0; j < CPW; ++j)
        if (c0 + j < cend)
#pragma unroll
          for (int q = 0; q < WPC; ++q) w[j][q] = win[((size_t)(c0 + j) * 64 + lane) * WPC + q];
#pragma unroll
      for (int j = 0; j < CPW; ++j) {
        if (c0 + j >= cend) break;
        float o[12];
        if (IN == MACT_U8) px4_u8<XF, DEG>(k, gtab, w[j][0], o);
        else if (IN == MACT_U16) px4_u16<XF, DEG>(k, gamma, w[j][0], w[j][WPC - 1], o);
        else px4_f16<XF, DEG>(k, gamma, w[j][0], w[j][WPC - 1], o);
        s_out[wv][j * 192 + 3 * lane] = f4{o[0], o[1], o[2], o[3]};
        s_out[wv][j * 192 + 3 * lane + 1] = f4{o[4], o[5], o[6], o[7]};
        s_out[wv][j * 192 + 3 * lane + 2] = f4{o[8], o[9], o[10], o[11]};
      }
      // the LDS writes of every lane must land before any lane reads them back
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
      __builtin_amdgcn_wave_barrier();
      const uint32_t n_valid = min((uint32_t)CPW, cend - c0) * 192u;
      const StreamBuf dst = wave_stream_buf(out4 + (size_t)c0 * 192, n_valid * 16u);
#pragma unroll
      for (int q = 0; q < CPW * 3; ++q) {
        const uint32_t e = q * 64 + lane;
        if (e < n_valid) stream_store(dst, e * 16u, s_out[wv][e]);
      }
      // every lane has read the slice before the next chunks overwrite it
      __builtin_amdgcn_s_waitcnt(0xc07f);
      __builtin_amdgcn_wave_barrier();
    }
    if (p1 == n_px)
      for (uint32_t p = (cend << 8) + threadIdx.x; p < n_px; p += 256u) {
        float v[3], o[3];
        load_px(d.src, p, v);
        px1<IN, XF, DEG>(k, gamma, gtab, v, o);
        store_px(d.dst, p, o);
      }
  }
}

// ---------------------------------------------------------------- host helpers

mact_status make_batch_descs(const mact_params& p, const mact_image* in, const mact_image* out, int32_t coef,
                             std::vector<BDesc>* descs, int* deg, const char* what) {
  mact_status s = check_params(&p);
  if (s != MACT_OK) return s;
  HostImage hi, ho;
  if ((s = resolve_image(in, false, what, &hi)) != MACT_OK) return s;
  if ((s = resolve_image(out, true, what, &ho)) != MACT_OK) return s;
  if ((s = check_same_shape(hi, ho, what)) != MACT_OK) return s;
  KCoef k;
  *deg = pack_coef(p, &k);
  const int gamma = uses_gamma(p.xform) ? hi.gamma : MACT_GAMMA_NONE;
  // packed 8-bit (1), float16 (2) or 16-bit (3) HWC in, packed float32 HWC out: the 4-pixel LDS path
  const bool hwc4 = (hi.dtype == MACT_U8 || hi.dtype == MACT_F16 || hi.dtype == MACT_U16) && hi.layout == MACT_HWC &&
                    hi.packed &&
                    ho.dtype == MACT_F32 && ho.layout == MACT_HWC && ho.packed;
  const int64_t per = images_per_launch(hi);
  for (int64_t n0 = 0; n0 < hi.N; n0 += per) {
    const int64_t cnt = std::min(per, hi.N - n0);
    BDesc d;
    std::memset(&d, 0, sizeof d);
    d.src = kimage(hi, n0, cnt);
    d.dst = kimage(ho, n0, cnt);
    d.n_px = (uint32_t)(cnt * hi.W * hi.H);
    d.coef = coef;
    d.gamma = gamma;
    const bool al = (uintptr_t)d.src.ptr % 4 == 0 && (uintptr_t)d.dst.ptr % 16 == 0;
    d.fast = (hwc4 && al) ? (hi.dtype == MACT_U8 ? 1 : hi.dtype == MACT_F16 ? 2 : 3) : 0;
    descs->push_back(d);
  }
  return MACT_OK;
}

uint32_t build_tiles(const std::vector<BDesc>& descs, uint32_t tile, std::vector<uint32_t>* tile_start) {
  tile_start->assign(descs.size() + 1, 0);
  uint64_t t = 0;
  for (size_t i = 0; i < descs.size(); ++i) {
    (*tile_start)[i] = (uint32_t)t;
    t += (descs[i].n_px + tile - 1) / tile;
  }
  (*tile_start)[descs.size()] = (uint32_t)t;
  return (uint32_t)t;
}

unsigned batch_grid(const mact_tune& tune, uint32_t total_tiles) {
  // waves_per_cu 0: the grid covers the tile list once (streaming launches run faster this way
  // than a few resident workgroups per CU walking the list)
  if (tune.waves_per_cu == 0) return std::max<uint32_t>(1, std::min<uint32_t>(total_tiles, 0x7fffffffu));
  const uint64_t per_cu = std::max<uint64_t>(1, (uint64_t)tune.waves_per_cu * 64 / tune.block);
  const uint64_t cap = (uint64_t)device_cus() * per_cu;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(total_tiles, cap));
}

// The tile list runs as equal launches of at most 2^26 pixels of tiles each
// (one launch for small batches): streaming launches of that size run faster
// than one launch over a whole large batch.
hipError_t launch_batch_kernel(const BDesc* d_descs, const KCoef* d_coefs, const uint32_t* d_tiles, int32_t count,
                               uint32_t total_tiles, const mact_tune& tune, int deg, hipStream_t st,
                               const uint32_t* d_tile_img) {
  return launch_batch_kernel_range(d_descs, d_coefs, d_tiles, count, 0, total_tiles, tune, deg, st, d_tile_img);
}

hipError_t launch_batch_kernel_range(const BDesc* d_descs, const KCoef* d_coefs, const uint32_t* d_tiles, int32_t count,
                                     uint32_t first, uint32_t end, const mact_tune& tune, int deg, hipStream_t st,
                                     const uint32_t* d_tile_img) {
  if (end <= first) return hipSuccess;
  const size_t shm = tune.vec == 4 ? (size_t)(tune.block / 64) * 192 * sizeof(f4) : 0;
  const uint32_t tile = (uint32_t)tune.tile;
  const uint64_t n_tiles = end - first;
  const uint64_t launches = tune.one_launch ? 1 : std::max<uint64_t>(1, (n_tiles * tile + (1ull << 26) - 1) >> 26);
  const uint32_t per = (uint32_t)((n_tiles + launches - 1) / launches);
  const dim3 b(tune.block);
  for (uint32_t t0 = first; t0 < end; t0 += per) {
    const uint32_t t1 = std::min(end, t0 + per);
    const dim3 g(batch_grid(tune, t1 - t0));
    if (deg == 5) {
      if (tune.vec == 4) hipLaunchKernelGGL((k_batch<5, 4>), g, b, shm, st, d_descs, d_coefs, d_tiles, d_tile_img, count, t0, t1, tile);
      else hipLaunchKernelGGL((k_batch<5, 1>), g, b, shm, st, d_descs, d_coefs, d_tiles, d_tile_img, count, t0, t1, tile);
    } else {
      if (tune.vec == 4) hipLaunchKernelGGL((k_batch<7, 4>), g, b, shm, st, d_descs, d_coefs, d_tiles, d_tile_img, count, t0, t1, tile);
      else hipLaunchKernelGGL((k_batch<7, 1>), g, b, shm, st, d_descs, d_coefs, d_tiles, d_tile_img, count, t0, t1, tile);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static mact_status check_tune(const mact_tune& t) {
  if (t.block < 64 || t.block > 1024 || t.block % 64)
    return fail(MACT_E_INVALID, "mact_tune: block %d not a multiple of 64 in 64..1024", t.block);
  if (t.tile < 256 || t.tile % 256 || t.tile < t.block)
    return fail(MACT_E_INVALID, "mact_tune: tile %d must be a multiple of 256 and >= block", t.tile);
  if (t.vec != 1 && t.vec != 4) return fail(MACT_E_INVALID, "mact_tune: vec %d not 1 or 4", t.vec);
  if (t.waves_per_cu < 0 || t.waves_per_cu > 64) return fail(MACT_E_INVALID, "mact_tune: waves_per_cu %d", t.waves_per_cu);
  if (t.one_launch != 0 && t.one_launch != 1) return fail(MACT_E_INVALID, "mact_tune: one_launch %d not 0 or 1", t.one_launch);
  return MACT_OK;
}

// ---------------------------------------------------------------- autotune cache

namespace {
std::mutex g_tune_mu;
std::map<std::string, mact_tune> g_tune_cache;
bool g_tune_file_loaded = false;

const char* cache_path() {
  const char* p = std::getenv("MACT_AUTOTUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// File format: one JSON object, "key": [block, tile, vec, waves_per_cu, one_launch] entries (an entry
// of the first four alone reads as one_launch 0).
void load_cache_file_locked() {
  if (g_tune_file_loaded) return;
  g_tune_file_loaded = true;
  const char* path = cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "rb");
  if (!f) return;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  std::fclose(f);
  size_t pos = 0;
  while ((pos = s.find('"', pos)) != std::string::npos) {
    const size_t end = s.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = s.substr(pos + 1, end - pos - 1);
    const size_t lb = s.find('[', end), rb = s.find(']', end);
    if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
    mact_tune t{};
    const int got = std::sscanf(s.c_str() + lb + 1, "%d , %d , %d , %d , %d", &t.block, &t.tile, &t.vec,
                                &t.waves_per_cu, &t.one_launch);
    if (got == 4) t.one_launch = 0;
    if ((got == 4 || got == 5) && check_tune(t) == MACT_OK) g_tune_cache[key] = t;
    pos = rb + 1;
  }
  clear_error();
}

void save_cache_file_locked() {
  const char* path = cache_path();
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : g_tune_cache) {
    std::fprintf(f, "  \"%s\": [%d, %d, %d, %d, %d]%s\n", kv.first.c_str(), kv.second.block, kv.second.tile,
                 kv.second.vec, kv.second.waves_per_cu, kv.second.one_launch, ++i == g_tune_cache.size() ? "" : ",");
  }
  std::fprintf(f, "}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

int log2_bucket(uint64_t v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

std::string shape_key(const std::vector<BDesc>& descs, int deg) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, current_device()) == hipSuccess) arch = prop.gcnArchName;
  uint64_t px = 0, fast_px = 0;
  for (const BDesc& d : descs) {
    px += d.n_px;
    if (d.fast) fast_px += d.n_px;
  }
  const int fast_frac = px ? (int)(4 * fast_px / px) : 0;  // quarters of pixels on the 4-pixel path
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s|cu%d|px2^%d|n2^%d|fast%d/4|deg%d", arch.c_str(), device_cus(), log2_bucket(px),
                log2_bucket(descs.size()), fast_frac, deg);
  return buf;
}
}  // namespace

}  // namespace mact

using namespace mact;

// A run of descriptors [d0, d1) of one class, and its tiles [t0, t1) under
// the plan's current tile size.  kind 0: descriptors for k_batch (any layout
// and type); 1, 2, 3: packed 8-bit, float16, 16-bit HWC in, packed float32
// HWC out, aligned, one coefficient set and transfer function: k_batch_cls.
struct BatchClass {
  int kind = 0, xform = 0, deg = 5, gamma = 0;
  KCoef k{};
  size_t d0 = 0, d1 = 0;
  uint32_t t0 = 0, t1 = 0;
};

struct mact_batch_plan {
  int device = 0;
  int32_t count = 0;  // descriptors
  int deg = 5;
  std::vector<BatchClass> classes;
  mact_tune tune{};
  uint32_t total_tiles = 0;
  BDesc* d_descs = nullptr;
  KCoef* d_coefs = nullptr;
  uint32_t* d_tiles = nullptr;
  uint32_t* d_tile_img = nullptr;  // image of every tile
  size_t tile_img_cap = 0;         // entries allocated
  size_t tiles_cap = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<BDesc> descs;
};

static void plan_free(mact_batch_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->d_descs) (void)hipFree(p->d_descs);
  if (p->d_coefs) (void)hipFree(p->d_coefs);
  if (p->d_tiles) (void)hipFree(p->d_tiles);
  if (p->d_tile_img) (void)hipFree(p->d_tile_img);
  delete p;
}

// Upload the tile list for plan->tune.tile (synchronous on the capture stream).
// Tile list for the current tile size: first tile of every image, and the
// image of every tile (so the kernel needs no search).
static mact_status plan_set_tiles(mact_batch_plan* p) {
  std::vector<uint32_t> ts;
  p->total_tiles = build_tiles(p->descs, (uint32_t)p->tune.tile, &ts);
  for (BatchClass& c : p->classes) {
    c.t0 = ts[c.d0];
    c.t1 = ts[c.d1];
  }
  std::vector<uint32_t> img(p->total_tiles);
  for (size_t i = 0; i + 1 < ts.size(); ++i)
    for (uint32_t t = ts[i]; t < ts[i + 1]; ++t) img[t] = (uint32_t)i;
  if (img.size() > p->tile_img_cap) {
    if (p->d_tile_img) (void)hipFree(p->d_tile_img);
    p->d_tile_img = nullptr;
    p->tile_img_cap = 0;
    if (hipMalloc(&p->d_tile_img, img.size() * sizeof(uint32_t)) != hipSuccess)
      return fail(MACT_E_NOMEM, "mact_batch_plan: tile map of %zu entries", img.size());
    p->tile_img_cap = img.size();
  }
  const size_t bytes = ts.size() * sizeof(uint32_t);
  mact_status s = hip_check(hipMemcpyAsync(p->d_tiles, ts.data(), bytes, hipMemcpyHostToDevice, p->cap_stream),
                            "mact_batch_plan: tile upload");
  if (s == MACT_OK && !img.empty())
    s = hip_check(hipMemcpyAsync(p->d_tile_img, img.data(), img.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                                 p->cap_stream),
                  "mact_batch_plan: tile upload");
  if (s != MACT_OK) return s;
  return hip_check(hipStreamSynchronize(p->cap_stream), "mact_batch_plan: tile upload");
}

template <int IN, int DEG>
static void launch_cls_xf(int xform, dim3 g, hipStream_t st, const BDesc* d, const uint32_t* ts, const uint32_t* ti,
                          uint32_t t0, uint32_t t1, uint32_t tile, const KCoef& k, int gamma) {
  const dim3 b(256);
  if (xform == MACT_LAB) hipLaunchKernelGGL((k_batch_cls<IN, DEG, MACT_LAB>), g, b, 0, st, d, ts, ti, t0, t1, tile, k, gamma);
  else if (xform == MACT_HSI) hipLaunchKernelGGL((k_batch_cls<IN, DEG, MACT_HSI>), g, b, 0, st, d, ts, ti, t0, t1, tile, k, gamma);
  else if (xform == MACT_LUV) hipLaunchKernelGGL((k_batch_cls<IN, DEG, MACT_LUV>), g, b, 0, st, d, ts, ti, t0, t1, tile, k, gamma);
  else hipLaunchKernelGGL((k_batch_cls<IN, DEG, MACT_SCT>), g, b, 0, st, d, ts, ti, t0, t1, tile, k, gamma);
}

template <int IN>
static void launch_cls_deg(const BatchClass& c, dim3 g, hipStream_t st, const BDesc* d, const uint32_t* ts,
                           const uint32_t* ti, uint32_t t0, uint32_t t1, uint32_t tile) {
  if (c.deg <= 4) launch_cls_xf<IN, 4>(c.xform, g, st, d, ts, ti, t0, t1, tile, c.k, c.gamma);
  else if (c.deg == 5) launch_cls_xf<IN, 5>(c.xform, g, st, d, ts, ti, t0, t1, tile, c.k, c.gamma);
  else launch_cls_xf<IN, 7>(c.xform, g, st, d, ts, ti, t0, t1, tile, c.k, c.gamma);
}

// Every class of the plan in turn: the vector path's classes through
// k_batch_cls (a persistent grid of waves_per_cu 256-thread workgroups per CU,
// or one workgroup per tile), the rest through k_batch; each class as equal
// launches of at most 2^26 pixels of tiles, or (one_launch) as one.
static hipError_t plan_launch_all(mact_batch_plan* p, hipStream_t st) {
  const mact_tune& tn = p->tune;
  const uint32_t tile = (uint32_t)tn.tile;
  for (const BatchClass& c : p->classes) {
    if (c.t1 <= c.t0) continue;
    if (c.kind == 0 || tn.vec != 4) {
      mact_tune t1 = tn;
      hipError_t e = launch_batch_kernel_range(p->d_descs, p->d_coefs, p->d_tiles, p->count, c.t0, c.t1, t1, p->deg, st,
                                               p->d_tile_img);
      if (e != hipSuccess) return e;
      continue;
    }
    const uint64_t n_tiles = c.t1 - c.t0;
    const uint64_t launches = tn.one_launch ? 1 : std::max<uint64_t>(1, (n_tiles * tile + (1ull << 26) - 1) >> 26);
    const uint32_t per = (uint32_t)((n_tiles + launches - 1) / launches);
    for (uint32_t a = c.t0; a < c.t1; a += per) {
      const uint32_t b = std::min(c.t1, a + per);
      uint64_t grid = b - a;
      if (tn.waves_per_cu > 0)
        grid = std::min<uint64_t>(grid, (uint64_t)device_cus() * std::max(1, tn.waves_per_cu / 4));
      const dim3 g((unsigned)std::max<uint64_t>(1, grid));
      if (c.kind == 1) launch_cls_deg<MACT_U8>(c, g, st, p->d_descs, p->d_tiles, p->d_tile_img, a, b, tile);
      else if (c.kind == 2) launch_cls_deg<MACT_F16>(c, g, st, p->d_descs, p->d_tiles, p->d_tile_img, a, b, tile);
      else launch_cls_deg<MACT_U16>(c, g, st, p->d_descs, p->d_tiles, p->d_tile_img, a, b, tile);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

static mact_status plan_time(mact_batch_plan* p, int reps, float* ms) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return fail(MACT_E_DEVICE, "mact_batch_plan: event");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(MACT_E_DEVICE, "mact_batch_plan: event");
  }
  mact_status s = MACT_OK;
  float best = INFINITY;
  for (int r = 0; r < reps && s == MACT_OK; ++r) {
    (void)hipEventRecord(a, p->cap_stream);
    s = hip_check(plan_launch_all(p, p->cap_stream), "mact_batch_plan: autotune launch");
    (void)hipEventRecord(b, p->cap_stream);
    if (s == MACT_OK) s = hip_check(hipEventSynchronize(b), "mact_batch_plan: autotune");
    float t = 0.0f;
    if (s == MACT_OK && hipEventElapsedTime(&t, a, b) == hipSuccess) best = std::min(best, t);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = best;
  return s;
}

static mact_status plan_autotune(mact_batch_plan* p) {
  const std::string key = shape_key(p->descs, p->deg);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    load_cache_file_locked();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      p->tune = it->second;
      return plan_set_tiles(p);
    }
  }
  static const int blocks[] = {256, 512, 1024};
  static const int tiles[] = {8192, 32768, 131072};
  static const int vecs[] = {4, 1};
  static const int waves[] = {16, 32, 0};
  // every candidate timed 3 times (best of), then the 4 fastest 8 times more
  std::vector<mact_tune> cands;
  for (int v : vecs)
    for (int b : blocks)
      for (int t : tiles)
        for (int w : waves) {
          cands.push_back(mact_tune{b, t, v, w, 0});
          // a persistent grid also as one launch over the whole tile list
          if (w > 0) cands.push_back(mact_tune{b, t, v, w, 1});
        }
  // one workgroup per small tile: one or two 256-pixel chunks per wave, the plain kernel's shape
  for (int b : {256, 512})
    for (int t : {2048, 4096}) cands.push_back(mact_tune{b, t, 4, 0, 0});
  std::vector<std::pair<float, mact_tune>> timed;
  for (const mact_tune& c : cands) {
    p->tune = c;
    mact_status s = plan_set_tiles(p);
    if (s != MACT_OK) return s;
    float ms = INFINITY;
    if ((s = plan_time(p, 3, &ms)) != MACT_OK) return s;
    timed.emplace_back(ms, p->tune);
  }
  std::stable_sort(timed.begin(), timed.end(),
                   [](const std::pair<float, mact_tune>& a, const std::pair<float, mact_tune>& b) { return a.first < b.first; });
  mact_tune best = timed.front().second;
  float best_ms = INFINITY;
  for (size_t i = 0; i < std::min<size_t>(4, timed.size()); ++i) {
    p->tune = timed[i].second;
    mact_status s = plan_set_tiles(p);
    if (s != MACT_OK) return s;
    float ms = INFINITY;
    if ((s = plan_time(p, 8, &ms)) != MACT_OK) return s;
    if (ms < best_ms) {
      best_ms = ms;
      best = p->tune;
    }
  }
  p->tune = best;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = best;
    save_cache_file_locked();
  }
  return plan_set_tiles(p);
}

static mact_status plan_capture(mact_batch_plan* p) {
  if (p->exec) {
    (void)hipGraphExecDestroy(p->exec);
    p->exec = nullptr;
  }
  if (p->graph) {
    (void)hipGraphDestroy(p->graph);
    p->graph = nullptr;
  }
  mact_status s = hip_check(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal),
                            "mact_batch_plan: begin capture");
  if (s != MACT_OK) return s;
  hipError_t le = plan_launch_all(p, p->cap_stream);
  hipError_t ce = hipStreamEndCapture(p->cap_stream, &p->graph);
  if ((s = hip_check(le, "mact_batch_plan: captured launch")) != MACT_OK) return s;
  if ((s = hip_check(ce, "mact_batch_plan: end capture")) != MACT_OK) return s;
  return hip_check(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "mact_batch_plan: instantiate");
}

extern "C" mact_status mact_batch_plan_create(const mact_params* params, const mact_image* in, const mact_image* out,
                                              int32_t count, const mact_tune* tune, void* hip_stream,
                                              mact_batch_plan** plan) {
  clear_error();
  if (!plan) return fail(MACT_E_INVALID, "mact_batch_plan_create: plan is NULL");
  *plan = nullptr;
  if (count <= 0) return fail(MACT_E_INVALID, "mact_batch_plan_create: count %d <= 0", count);
  if (!params || !in || !out) return fail(MACT_E_INVALID, "mact_batch_plan_create: NULL array");
  if (tune) {
    mact_status s = check_tune(*tune);
    if (s != MACT_OK) return s;
  }
  mact_batch_plan* p = new (std::nothrow) mact_batch_plan();
  if (!p) return fail(MACT_E_NOMEM, "mact_batch_plan_create: host allocation");
  p->device = current_device();
  // coefficient table with duplicates folded, with each set's own degree
  std::vector<KCoef> coefs;
  std::vector<int> coef_deg;
  for (int32_t i = 0; i < count; ++i) {
    KCoef k;
    mact_status s = check_params(&params[i]);
    if (s != MACT_OK) {
      plan_free(p);
      return fail(s, "mact_batch_plan_create: image %d: %s", i, mact_last_error());
    }
    int exact = 0;
    pack_coef(params[i], &k, &exact);
    int32_t idx = -1;
    for (size_t j = 0; j < coefs.size(); ++j)
      if (std::memcmp(&coefs[j], &k, sizeof k) == 0) idx = (int32_t)j;
    if (idx < 0) {
      idx = (int32_t)coefs.size();
      coefs.push_back(k);
      coef_deg.push_back(exact);
    }
    int deg = 5;
    char what[64];
    std::snprintf(what, sizeof what, "mact_batch_plan_create: image %d", i);
    if ((s = make_batch_descs(params[i], &in[i], &out[i], idx, &p->descs, &deg, what)) != MACT_OK) {
      plan_free(p);
      return s;
    }
    p->deg = std::max(p->deg, deg);
  }
  // classes: descriptors of the vector path grouped by (element type, coefficient set, transfer
  // function), in order of first appearance, then every other descriptor
  {
    std::vector<BDesc> sorted;
    sorted.reserve(p->descs.size());
    std::vector<bool> used(p->descs.size(), false);
    for (size_t i = 0; i < p->descs.size(); ++i) {
      const BDesc& d = p->descs[i];
      if (used[i] || d.fast == 0) continue;
      BatchClass c;
      c.kind = d.fast;
      c.k = coefs[d.coef];
      c.xform = c.k.xform;
      c.deg = coef_deg[d.coef];
      c.gamma = d.gamma;
      c.d0 = sorted.size();
      for (size_t j = i; j < p->descs.size(); ++j) {
        const BDesc& e = p->descs[j];
        if (!used[j] && e.fast == d.fast && e.coef == d.coef && e.gamma == d.gamma) {
          used[j] = true;
          sorted.push_back(e);
        }
      }
      c.d1 = sorted.size();
      p->classes.push_back(c);
    }
    BatchClass rest;
    rest.d0 = sorted.size();
    for (size_t i = 0; i < p->descs.size(); ++i)
      if (!used[i]) sorted.push_back(p->descs[i]);
    rest.d1 = sorted.size();
    if (rest.d1 > rest.d0) p->classes.push_back(rest);
    p->descs.swap(sorted);
  }
  p->count = (int32_t)p->descs.size();
  hipStream_t user = static_cast<hipStream_t>(hip_stream);
  mact_status s = MACT_OK;
  const size_t tiles_bytes = (p->descs.size() + 1) * sizeof(uint32_t);
  if (hipMalloc(&p->d_descs, p->descs.size() * sizeof(BDesc)) != hipSuccess ||
      hipMalloc(&p->d_coefs, coefs.size() * sizeof(KCoef)) != hipSuccess ||
      hipMalloc(&p->d_tiles, tiles_bytes) != hipSuccess) {
    plan_free(p);
    return fail(MACT_E_NOMEM, "mact_batch_plan_create: device allocation");
  }
  if (s == MACT_OK) s = hip_check(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "mact_batch_plan_create: stream");
  if (s == MACT_OK)
    s = hip_check(hipMemcpyAsync(p->d_descs, p->descs.data(), p->descs.size() * sizeof(BDesc), hipMemcpyHostToDevice,
                                 p->cap_stream), "mact_batch_plan_create: upload");
  if (s == MACT_OK)
    s = hip_check(hipMemcpyAsync(p->d_coefs, coefs.data(), coefs.size() * sizeof(KCoef), hipMemcpyHostToDevice,
                                 p->cap_stream), "mact_batch_plan_create: upload");
  // inputs written on the caller's stream must be complete before the autotuner runs
  if (s == MACT_OK) s = hip_check(hipStreamSynchronize(user), "mact_batch_plan_create: caller stream");
  if (s == MACT_OK) {
    if (tune) {
      p->tune = *tune;
      s = plan_set_tiles(p);
    } else {
      s = plan_autotune(p);
    }
  }
  if (s == MACT_OK) s = plan_capture(p);
  if (s != MACT_OK) {
    plan_free(p);
    return s;
  }
  *plan = p;
  return MACT_OK;
}

extern "C" mact_status mact_batch_plan_launch(mact_batch_plan* p, int32_t use_graph, void* hip_stream) {
  clear_error();
  if (!p) return fail(MACT_E_INVALID, "mact_batch_plan_launch: plan is NULL");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (use_graph) return hip_check(hipGraphLaunch(p->exec, st), "mact_batch_plan_launch: graph launch");
  return hip_check(plan_launch_all(p, st), "mact_batch_plan_launch: launch");
}

extern "C" mact_status mact_batch_plan_tune(const mact_batch_plan* p, mact_tune* tune) {
  clear_error();
  if (!p || !tune) return fail(MACT_E_INVALID, "mact_batch_plan_tune: NULL argument");
  *tune = p->tune;
  return MACT_OK;
}

extern "C" mact_status mact_batch_plan_destroy(mact_batch_plan* p) {
  clear_error();
  plan_free(p);
  return MACT_OK;
}

extern "C" mact_status mact_batch_run(const mact_params* params, const mact_image* in, const mact_image* out,
                                      int32_t count, const mact_tune* tune, void* hip_stream) {
  mact_batch_plan* p = nullptr;
  mact_status s = mact_batch_plan_create(params, in, out, count, tune, hip_stream, &p);
  if (s != MACT_OK) return s;
  s = mact_batch_plan_launch(p, 1, hip_stream);
  if (s == MACT_OK) s = hip_check(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)), "mact_batch_run: synchronise");
  plan_free(p);
  return s;
}
