// Host-side helpers for launching libmact kernels: image descriptor
// resolution and validation, coefficient packing, device properties.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "pixel.h"

namespace mact {

// A validated caller image with every stride resolved.
struct HostImage {
  void* data = nullptr;
  int dtype = 0, layout = 0, gamma = 0;
  int64_t W = 0, H = 0, N = 1;
  int64_t rs = 0, ps = 0, bs = 0;
  bool packed = false;
  size_t esize = 1;
};

FastDiv make_fastdiv(uint32_t d);

// Validates *im (input images accept U8/F16/F32, outputs F16/F32).
mact_status resolve_image(const mact_image* im, bool is_output, const char* what, HostImage* out);
// Same width, height and batch.
mact_status check_same_shape(const HostImage& a, const HostImage& b, const char* what);
// Kernel view of images [n0, n0 + count) of a resolved image.
KImage kimage(const HostImage& h, int64_t n0, int64_t count);
// Images per launch so that a launch covers fewer than 2^31 pixels.
int64_t images_per_launch(const HostImage& h);
// Images per launch of the streaming kernels with float32 output: the batch
// split into equal launches of at most 2^26 pixels (at least one image each).
// Measured in one process against whole-batch launches: CIELAB 64 x 1080p in
// two launches +1.3%, 32 x 4K in four +2.7%, the float32-input forms and the
// inverses +1 to +1.6%.  float16 outputs, whose kernels are bound by the VALU,
// lost 1.5% to the extra launch and keep images_per_launch.  The count is
// rounded up so that every launch starts where the coalesced kernels'
// alignment holds (images with an odd pixel count would otherwise send every
// launch after the first to the one-pixel kernel).
int64_t images_per_stream_launch(const HostImage& in, const HostImage& out);

// Coefficients rounded to float32 and zero padded; returns the padded degree
// (5 or 7) the kernels are instantiated for, and the highest degree actually
// used in *exact (the hot kernel also has a degree-4 instance).
int pack_coef(const mact_params& p, KCoef* k, int* exact = nullptr);

// One image of a batched launch (device-side descriptor).
struct BDesc {
  KImage src, dst;
  uint32_t n_px;  // pixels (N H W) of this descriptor, < 2^31
  int32_t coef;   // index into the coefficient table
  int32_t gamma;  // inverse-gamma row for 8-bit LAB inputs
  int32_t fast;   // packed HWC in (1: 8-bit, 2: float16, 3: 16-bit), packed float32 HWC out, aligned: 4-pixel path
};

// Host preparation of one batch entry: validates (params, in, out) and appends
// its descriptors (several if the image holds 2^31 pixels or more) to `descs`;
// the coefficient index is set to `coef`.  *deg receives the padded degree.
mact_status make_batch_descs(const mact_params& p, const mact_image* in, const mact_image* out, int32_t coef,
                             std::vector<BDesc>* descs, int* deg, const char* what);
// Launch of the persistent batched kernel.  d_tile_img (optional): the image
// of every tile; without it each workgroup finds its tile's image by binary
// search over d_tiles.
hipError_t launch_batch_kernel(const BDesc* d_descs, const KCoef* d_coefs, const uint32_t* d_tiles, int32_t count,
                               uint32_t total_tiles, const mact_tune& tune, int deg, hipStream_t st,
                               const uint32_t* d_tile_img = nullptr);
// The same over tiles [first, end) of the list only.
hipError_t launch_batch_kernel_range(const BDesc* d_descs, const KCoef* d_coefs, const uint32_t* d_tiles, int32_t count,
                                     uint32_t first, uint32_t end, const mact_tune& tune, int deg, hipStream_t st,
                                     const uint32_t* d_tile_img);
// Grid of the batched kernel for a tune and a tile count.
unsigned batch_grid(const mact_tune& tune, uint32_t total_tiles);
// Tile list: tile_start[i] = first tile of descriptor i; returns the total.
uint32_t build_tiles(const std::vector<BDesc>& descs, uint32_t tile, std::vector<uint32_t>* tile_start);

// Any input image (element type in_dtype; layout and strides in `src`) -> float32
// or float16 (out_dtype) output of n_px pixels of hw per image: packed HWC
// (kGatherHWC) or CHW (kGatherCHW) at `out`, 16-byte aligned: the shapes the
// 4-pixel kernels do not take; or (kGatherAny) the output view `dst`, any
// layout and strides, its elements naturally aligned (`out` unused).
// deg: the highest degree among the approximations (evaluated at 4, 5 or 7).
enum { kGatherHWC = 0, kGatherCHW = 1, kGatherAny = 2 };
void launch_gather(int in_dtype, int xform, int out_dtype, int out_mode, int deg, const KImage& src, const KImage& dst,
                   void* out, uint32_t n_px, uint32_t hw, const KCoef& k, int gamma, hipStream_t st);

// Compute units of the current device (cached per device).
int device_cus();
int current_device();

inline mact_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return MACT_OK;
  return fail(MACT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace mact
