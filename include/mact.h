/*
 * mact.h -- C ABI of libmact, the MACT hot path for AMD Instinct MI355X (gfx950).
 *
 * MACT (Celebi, Kingravi & Celiker, "Fast Color Space Transformations Using
 * Minimax Approximations") evaluates per-pixel RGB->CIELAB (Sec. 3.2), RGB->HSI
 * (Sec. 3.3) and RGB->SCT (Sec. 3.4) with the costly elementary functions -- the
 * cube root, and the arctan / arcsin / arccos terms -- replaced by minimax
 * polynomials or rationals computed with the Remez exchange algorithm (Sec. 3.1).
 * The 3-D LUT interpolators the paper compares with (trilinear, prism, pyramidal,
 * tetrahedral; Sec. 3.5.3) are provided beside it.
 *
 * Conventions for every entry point:
 *  - Return value: MACT_OK (0) or a negative mact_status.  Nothing throws,
 *    aborts or prints.  mact_last_error() gives a thread-local detail string.
 *  - Device calls are asynchronous on the hip stream passed as `void*`
 *    (hipStream_t; NULL = the default stream of the current device) and run on
 *    the current HIP device.  Arguments are validated before anything is
 *    launched; an invalid call launches nothing.
 *  - Ownership: the library never allocates, frees or retains caller buffers.
 *    Parameter structs are copied at call time and may be freed on return.
 *  - Reentrant: calls may come from several host threads.  Calls that write the
 *    same output buffer, or that share a batch plan, must not overlap.
 *  - Pixels: R, G, B on the normalised scale [0, 1].  8-bit values v enter as
 *    v/255.  Float inputs outside [0, 1] are clamped to it (the approximations
 *    are fitted on the image of [0, 1] only); NaN inputs give unspecified values.
 */
#ifndef MACT_H
#define MACT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */

typedef int32_t mact_status;
enum {
  MACT_OK = 0,
  MACT_E_INVALID = -1,     /* an argument is out of range, NULL or inconsistent */
  MACT_E_NOCONV = -2,      /* mact_fit did not converge; *out holds the best iterate */
  MACT_E_DEVICE = -3,      /* a HIP runtime call failed (detail in mact_last_error) */
  MACT_E_NOMEM = -4,       /* a library-owned allocation failed */
  MACT_E_UNSUPPORTED = -5, /* a valid but unimplemented combination */
  MACT_E_BUSY = -6,        /* serving: the request cannot be admitted yet */
  MACT_E_CANCELLED = -7    /* serving: the request was withdrawn before admission */
};

/* Static description of a status code. */
const char* mact_status_str(mact_status s);
/* Detail of the last failing call on this thread ("" if none).  Valid until
   the next library call on the same thread. */
const char* mact_last_error(void);
/* Library version string. */
const char* mact_version(void);

/* ------------------------------------------------- minimax approximations */

/* Functions the paper approximates (Sec. 3.2.2, 3.3.2, 3.4.2, 3.4.3), and the
   ones the inverse transforms approximate in the same way. */
enum {
  MACT_FN_CBRT = 0,       /* t^(1/3): the CIELAB nonlinearity above 0.008856 */
  MACT_FN_ATAN_SQRT3 = 1, /* arctan(sqrt(3) x): Kender's hue, odd extension */
  MACT_FN_ASIN2 = 2,      /* 2 arcsin(y / sqrt 2) = arccos(1 - y^2): SCT angle A, B/L >= 0.5 */
  MACT_FN_ACOS = 3,       /* arccos(x): SCT angle A, B/L < 0.5 */
  MACT_FN_ATAN = 4,       /* arctan(x): SCT angle B for G < R (f of the split) */
  MACT_FN_ATANC = 5,      /* pi/2 - arctan(t): SCT angle B for R <= G (g of the split) */
  MACT_FN_SIN = 6,        /* sin(x): SCT -> RGB */
  MACT_FN_COS = 7,        /* cos(x): SCT -> RGB and HSI -> RGB */
  MACT_FN_ENC709 = 8,     /* 1.099 x^0.45 - 0.099: BT.709 encoding above 0.018, CIELAB -> R'G'B' */
  MACT_FN_DEC709 = 9,     /* ((x + 0.099) / 1.099)^(1/0.45): BT.709 decoding above 0.081, float inputs */
  MACT_FN_COUNT = 10
};

#define MACT_MAX_DEGREE 7
#define MACT_MAX_WEIGHT_SAMPLES 65536

/* A minimax approximation p/q on [lo, hi] (Sec. 3.1).  Monomial coefficients,
   lowest degree first, q[0] = 1 for fits made here (printed tables keep the
   paper's scaling).  m = 0: polynomial (q = 1). */
typedef struct mact_approx {
  int32_t fn;        /* MACT_FN_* */
  int32_t n, m;      /* degrees of p and q, 0..MACT_MAX_DEGREE */
  int32_t iters;     /* Remez iterations used (0 for tabulated sets) */
  double lo, hi;     /* fit interval */
  double p[8];       /* numerator coefficients (entries > n are 0) */
  double q[8];       /* denominator coefficients (entries > m are 0) */
  double eps;        /* max |f - p/q| on [lo, hi] (max |w (f - p/q)| for a weighted fit) */
  double alt[18];    /* final alternation points (n + m + 2 of them) */
  int32_t n_alt;
  int32_t converged; /* 1 if the levelled error met the tolerance */
} mact_approx;

/* Remez exchange fit of function `fn` by p/q with deg p = n, deg q = m on
   [lo, hi] (Sec. 3.1; the paper names the algorithm and cites its details).
   Host only, FP64.  Errors: MACT_E_INVALID for NULL out, degrees outside
   0..7, n + m + 2 > 18, lo >= hi, or an interval outside the function's
   domain; MACT_E_NOCONV when the levelled error does not reach the tolerance
   in `max_iter` iterations (out holds the best iterate and its eps). */
mact_status mact_fit(int32_t fn, int32_t n, int32_t m, double lo, double hi, mact_approx* out);
mact_status mact_fit_ex(int32_t fn, int32_t n, int32_t m, double lo, double hi, int32_t max_iter,
                        mact_approx* out);

/* Weighted Chebyshev fit: p/q minimising max |w(x) (f(x) - p(x)/q(x))| on
   [lo, hi], the criterion of Sec. 3.1 under a positive weight (w = 1 is
   mact_fit).  `weight` holds n_weight samples of w at the equally spaced points
   lo + i (hi - lo) / (n_weight - 1), i = 0..n_weight-1 (host memory, read
   during the call only); w is linear between samples.  A weight small near one
   end of the interval lets the error grow there and shrink elsewhere: for the
   CIELAB cube root, damping the dark end trades the largest Delta E*ab over the
   RGB cube for a smaller mean.  out->eps is the weighted maximum.  Errors: as
   mact_fit_ex, and MACT_E_INVALID for a NULL weight, n_weight outside
   2..MACT_MAX_WEIGHT_SAMPLES, or a sample that is not positive and finite. */
mact_status mact_fit_weighted(int32_t fn, int32_t n, int32_t m, double lo, double hi, const double* weight,
                              int32_t n_weight, int32_t max_iter, mact_approx* out);

/* The library's default approximation of `fn` (its own Remez fits, made once
   per process and cached): cube root (4,4) rational on [0.008856, 1] (Table 2's
   degree); arctan(sqrt 3 x) degree 5 on [0, 1]; 2 arcsin(y/sqrt 2) degree 5 on
   [0, 1/sqrt 2]; arccos degree 5 on [0, 0.5]; arctan and pi/2 - arctan degree 5
   on [0, 1] (the full range of G/R and R/G for float inputs); sine and cosine
   degree 7 on [0, pi/2]; the BT.709 encoding (4,4) rational on [0.018, 1]; the
   BT.709 decoding degree 7 on [0.081, 1]. */
mact_status mact_default_approx(int32_t fn, mact_approx* out);

/* The coefficients printed in the paper: Table 1 (fn CBRT, m = 0, n = 2..5),
   Table 2 (CBRT, n, m in 2..4), Table 3 (ATAN_SQRT3, n = 2..5; the n = 2 row
   with a2 = -0.7497879, the printed + sign being lost), Tables 4-7 (ASIN2,
   ACOS, ATAN, ATANC, n = 4, 5).  eps is the printed eps^A_max.
   MACT_E_INVALID if the paper has no such row. */
mact_status mact_paper_approx(int32_t fn, int32_t n, int32_t m, mact_approx* out);

/* ------------------------------------------------------------ images */

enum { MACT_LAB = 0, MACT_HSI = 1, MACT_SCT = 2, MACT_LUV = 3 };   /* transforms; CIELUV is the extension named in Sec. 4 */
enum { MACT_U8 = 0, MACT_F16 = 1, MACT_F32 = 2, MACT_U16 = 3 };  /* element types; U16 codes are full-range (v / 65535) */
enum { MACT_HWC = 0, MACT_CHW = 1 };                 /* layouts */
enum {                                              /* input transfer function (LAB) */
  MACT_GAMMA_BT709 = 0, /* Sec. 3.2.1's inverse gamma (ITU-R BT.709); default */
  MACT_GAMMA_SRGB = 1,  /* IEC 61966-2-1 curve */
  MACT_GAMMA_NONE = 2   /* the input is linear RGB */
};

/* A device image or a batch of equally shaped images.  Element (n, y, x, c) is at
     HWC: data + (n*batch_stride + y*row_stride + 3*x + c) * elem_size
     CHW: data + (n*batch_stride + c*plane_stride + y*row_stride + x) * elem_size
   Strides are in elements; 0 selects the packed value (HWC row_stride = 3 W;
   CHW row_stride = W, plane_stride = H row_stride; batch_stride = H row_stride
   (HWC) or 3 plane_stride (CHW)).  `gamma` applies to LAB and LUV inputs only. */
typedef struct mact_image {
  void* data;
  int32_t dtype, layout;
  int64_t width, height;
  int64_t row_stride, plane_stride;
  int64_t batch, batch_stride; /* batch 0 or 1: a single image */
  int32_t gamma;
  int32_t reserved;
} mact_image;

/* Which approximations a transform uses:
     LAB: f[0] = cube root (polynomial or rational); optionally f[1] = the
          BT.709 decoding (fn MACT_FN_DEC709, a polynomial of degree <= 7),
          which then replaces the exact power for float inputs with gamma
          MACT_GAMMA_BT709 (8-bit inputs use their exact 256-entry table);
          f[1] with any other fn is ignored;
     HSI: f[0] = arctan(sqrt 3 x) (polynomial);
     SCT: f[0] = 2 arcsin(y/sqrt 2), f[1] = arccos, f[2] = arctan, f[3] = pi/2 - arctan
          (polynomials);
     LUV: as LAB (f[0] = cube root, optional f[1] = the BT.709 decoding).
   out_mode 0: transform values.  out_mode 1 (LAB only): the three values of
   the approximated nonlinearity f~(X/X0), f~(Y/Y0), f~(Z/Z0) instead of L*a*b*. */
typedef struct mact_params {
  int32_t xform;
  int32_t out_mode;
  mact_approx f[4];
} mact_params;

/* Fill *p with transform `xform` and the default approximations. */
mact_status mact_params_default(int32_t xform, mact_params* p);

/* ------------------------------------------------------------ transforms */

/* Per-pixel MACT transform of `in` into `out` (Sec. 3.2-3.4):
     LAB: inverse gamma (8-bit inputs through a 256-entry table of the exact
          values), BT.709 RGB->XYZ, D65 white, f~ = p/q above t = 0.008856 and
          the exact linear segment at or below it; L* = 116 fy - 16,
          a* = 500 (fx - fy), b* = 200 (fy - fz).
     HSI: Kender's branch form; H = base + P(x) for x >= 0, base - P(-x) for
          x < 0 (arctan's odd symmetry); H = 0 on the red ray and the gray
          axis; S = 1 - 3 min / (R+G+B) (0 for black); I = (R+G+B)/3.
          H in [0, 2 pi] radians; S, I in [0, 1].
     SCT: L = |RGB|; angle A = P_asin2(sqrt(1 - B/L)) if 3 B^2 >= R^2 + G^2
          (B/L >= 0.5), else P_acos(B/L); angle B = P_atan(G/R) if G < R,
          P_atanc(R/G) if 0 < R <= G, pi/2 if R = 0 < G, 0 if R = G = 0;
          black gives (0, 0, 0).  Radians.
     LUV: CIE 1976 L*u*v* (Sec. 4 names it as the next transform): linear RGB
          as for LAB, X, Y, Z by the BT.709 matrix, L* = 116 f~(Y) - 16 with
          CIELAB's approximated nonlinearity (Y / Yn, Yn = 1), u' = 4X / D,
          v' = 9Y / D with D = X + 15Y + 3Z, u* = 13 L* (u' - u'n),
          v* = 13 L* (v' - v'n) with the D65 white's u'n, v'n; D = 0 (black)
          gives u* = v* = 0.
   in: MACT_U8 / MACT_U16 / MACT_F16 / MACT_F32, HWC or CHW, any strides.  out:
   MACT_F32 or MACT_F16, HWC or CHW, same width, height and batch as `in`.
   Evaluation is float32 with explicit fused multiply-adds; the result does not
   depend on the layout or the launch configuration, so every form (plain,
   batched, served) gives identical bits.  Coalesced kernels, each to float32
   or float16 output, serve packed HWC in to packed HWC out; packed HWC or CHW
   in to packed CHW or HWC out (W H a multiple of 4); row-strided HWC views to
   packed HWC (rows of a multiple of 4 pixels, strides in whole 4-byte words,
   16-byte for float32); and row-strided CHW views (crops of the planes, gaps
   between images) to packed HWC or CHW (rows of a multiple of 4 pixels,
   strides in whole 4-element groups).  Other combinations (odd widths, other
   strides, strided outputs) run one pixel per lane at a fraction of the
   bandwidth.  With float32 output, a batch of more than 2^26 pixels runs as
   several launches of whole images, in order on `hip_stream` (equal groups of
   at most 2^26 pixels, or one image each if images are larger); a graph
   captured from the call holds them all.
   Errors: MACT_E_INVALID (NULL pointers, sizes <= 0, strides too small,
   mismatched shapes, gamma set for HSI/SCT, out_mode 1 for HSI/SCT, degrees
   outside 0..7); MACT_E_UNSUPPORTED (rational approximations for HSI/SCT,
   U8 output); MACT_E_DEVICE (launch failure). */
mact_status mact_transform(const mact_params* params, const mact_image* in, const mact_image* out,
                           void* hip_stream);

/* The exact transform of `xform` in float32 with the device's elementary
   functions -- the baseline MACT replaces, for measuring its gain as the paper
   does against the C library's functions (Sec. 3.5, Table 11).  Everything but
   the approximated functions is MACT's own arithmetic: the 8-bit inverse-gamma
   table, the matrix, the linear segment, Kender's branches.  LAB / LUV use
   cbrtf; HSI atanf(sqrt 3 x); SCT sqrtf, arccos(B/L) as 2 asinf(sqrt((1 - B/L)
   / 2)) where B/L >= 0.5 and acosf(B/L) below, and atan2f(G, R).  in: packed
   8-bit HWC, 4-byte aligned; out: packed float32 or float16 HWC, 16-byte
   aligned.  Errors: as mact_transform; MACT_E_UNSUPPORTED for other element
   types, layouts or alignments. */
mact_status mact_transform_exact(int32_t xform, const mact_image* in, const mact_image* out, void* hip_stream);

/* Vector-Jacobian product of the LAB transform (chain rule through the
   definition of Sec. 3.2 with f~ in place of the cube root; the paper does not
   differentiate the transform):
     g_f = (500 g_a, 116 g_L - 500 g_a + 200 g_b, -200 g_b),
     g_t = g_f * f~'(t)   (f~' = (p' q - p q') / q^2 above 0.008856, 7.787 below),
     dx  = (diag(1/white) M)^T g_t, zeroed for inputs outside [0, 1].
   x: MACT_F32 linear RGB (gamma MACT_GAMMA_NONE); grad_out and grad_in: MACT_F32
   with the same geometry as x (any layouts).  params->xform must be MACT_LAB.
   Errors as mact_transform; MACT_E_UNSUPPORTED for non-F32 or gamma != NONE. */
mact_status mact_transform_backward(const mact_params* params, const mact_image* x,
                                    const mact_image* grad_out, const mact_image* grad_in,
                                    void* hip_stream);

/* ------------------------------------------------------------ inverses, error statistics */

/* Fill *p with the default approximations of the inverse of `xform`:
     LAB, LUV: f[0] = the BT.709 encoding power, (4,4) rational on [0.018, 1];
     HSI: f[0] = cosine, degree 7 on [0, 2 pi/3];
     SCT: f[0] = sine, f[1] = cosine, degree 7 on [0, pi/2]. */
mact_status mact_inverse_params_default(int32_t xform, mact_params* p);

/* Inverse MACT transform of `in` (L*a*b*, HSI, SCT or L*u*v* triples) into `out`
   (R'G'B' on the [0, 1] scale):
     LAB: fy = (L* + 16)/116, fx = fy + a* / 500, fz = fy - b* / 200; t = f^3 where
          that exceeds 0.008856, else (f - 16/116)/7.787 (Sec. 3.2.1 solved for
          t); linear RGB = M^-1 (t * white), clamped to [0, 1]; then, for an
          `out` with gamma MACT_GAMMA_BT709, 4.5 L below 0.018 and f[0](L) at or
          above (the encoding that inverts Sec. 3.2.1's inverse gamma); with
          MACT_GAMMA_NONE the linear values.
     HSI: by sectors of 2 pi/3 (H taken modulo 2 pi): in the sector starting
          at h0, with h = H - h0, the channel behind the sector is I (1 - S), the
          one at its start I (1 + S c(h) / c(|pi/3 - h|)) with c = f[0] ~ cos,
          and the third 3 I - (the other two) (Sec. 3.3.1 solved for R, G, B).
     SCT: R = L s(A) c(B), G = L s(A) s(B), B = L c(A) with s = f[0] ~ sin and
          c = f[1] ~ cos (Sec. 3.4.1's inverse); A, B in [0, pi/2], the range
          the forward transform gives for non-negative RGB.
     LUV: Y from L* as for LAB; u' = u* / (13 L*) + u'n, v' = v* / (13 L*) + v'n;
          X = 9 u' Y / (4 v'), Z = (12 - 3 u' - 20 v') Y / (4 v') (the CIE 1976
          definition solved for X, Y, Z); L* <= 0 gives black; then M^-1 XYZ,
          the clamp and the encoding as for LAB.  Triples off the image of the
          forward transform (v' <= 0) give unspecified values.
   in: MACT_F32 or MACT_F16, any layout; out: MACT_F32 or MACT_F16, any layout,
   same geometry.  float32 arithmetic; float16 outputs are the float32 results
   rounded to nearest even.  Coalesced kernels serve packed float32 HWC in to
   packed HWC out and packed CHW in to packed CHW out (W H a multiple of 4);
   other combinations run one pixel per lane.  Large float32-output batches
   run as several launches, as for mact_transform.  Errors: MACT_E_INVALID (NULL, shapes,
   approximations of the wrong function or degree); MACT_E_UNSUPPORTED (8-bit
   in, sRGB encoding); MACT_E_DEVICE. */
mact_status mact_inverse(const mact_params* params, const mact_image* in, const mact_image* out,
                         void* hip_stream);

/* Accuracy of a forward transform over an image, computed on the device. */
typedef struct mact_error {
  int64_t count;       /* pixels */
  double mean, max;    /* of the metric: Delta E*ab (LAB, Sec. 3.2.1), Delta E*uv (LUV), D_HSI (HSI, Sec. 3.3.1),
                          or the SCT measure of Sec. 3.4.1 (both triples back to RGB, no
                          clipping, then CIELAB with BT.709, then Delta E*ab) */
  double max_abs[3];   /* largest |MACT - exact| per channel (HSI hue wrapped to [0, pi]) */
} mact_error;

/* Every pixel of `in` (an RGB image as mact_transform takes it) through the
   MACT transform of `params` (float32, the same arithmetic as mact_transform)
   and through the exact transform (float64 on the device: the definitions of
   Sec. 3.2.1, 3.3.1, 3.4.1 with the library's cube root, arctangent and
   arccosine); the metric per pixel, reduced to mean and max.  Enqueues on
   `hip_stream`, waits for it, and fills *out.  The library allocates and frees
   40 bytes of device memory per call.  Errors as mact_transform; MACT_E_NOMEM. */
mact_status mact_error_stats(const mact_params* params, const mact_image* in, mact_error* out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   statistics as mact_error_stats, with the same kernels, arguments, results
   and errors, but no hipMalloc, hipFree or other allocating call.  The
   accumulator (one 40-byte record) lives in a fixed 256-byte device array that
   each GPU the library runs on holds until the process ends; its address is
   looked up once per GPU, on the first call with that GPU current.  The record
   does not grow with the input, so no image size is refused on its account.
   Every call on one GPU shares that record and clears it first: calls that
   overlap on one GPU (other threads, other streams) race and must be
   serialised by the caller.  Enqueues on `hip_stream` and waits for it, as
   mact_error_stats does.  MACT_E_UNSUPPORTED for a device index of 64 or
   more; MACT_E_DEVICE if the array's address cannot be obtained. */
mact_status mact_error_stats_noalloc(const mact_params* params, const mact_image* in, mact_error* out,
                                     void* hip_stream);

/* ------------------------------------------------------------ 3-D LUTs */

enum { MACT_TRILINEAR = 0, MACT_PRISM = 1, MACT_PYRAMIDAL = 2, MACT_TETRAHEDRAL = 3 };

/* Bytes of a packed N x N x N LUT for `xform`: N^3 nodes of 4 floats (LAB:
   L*, a*, b*, 0; LUV: L*, u*, v*, 0; HSI: cos H, sin H, S, I; SCT: cos A,
   sin A, cos B, sin B); for SCT the N^3 nodes are followed by a plane of N^3
   floats holding L, padded to a multiple of 16 bytes (20 bytes a node).  Node
   (i, j, k) at index (i N + j) N + k holds the exact transform of the input
   (i, j, k)/(N - 1) (Sec. 3.5.3's packing).  Returns 0 for invalid arguments. */
size_t lut_bytes(int32_t xform, int32_t n);

/* Packing (Sec. 3.5.3): evaluates the exact transform in FP64 on the host at
   every node, rounds to float32 and copies the packed LUT to the device buffer
   `dev_lut` (caller-owned, >= lut_bytes bytes) on `hip_stream`.  Returns after
   the copy has completed.  n in 2..256.  gamma applies to LAB and LUV. */
mact_status lut_build(int32_t xform, int32_t n, int32_t gamma, float* dev_lut, size_t bytes,
                      void* hip_stream);

/* Extraction + 3-D interpolation (Sec. 3.5.3) of every pixel of `in` in the
   LUT: cell i = min(floor(x (N-1)), N-2) and fraction per channel (exact
   integer arithmetic for 8-bit inputs), then
     TRILINEAR   tensor-product weights on 8 corners;
     PRISM       linear along R, triangle (0,0),(1,0),(1,1) of the (G,B) face if
                 f_G >= f_B else (0,0),(0,1),(1,1): 6 corners;
     PYRAMIDAL   apex corner 111, base the cell face through 000 normal to the
                 axis of the smallest fraction, in Kang's polynomial form: 5 corners;
     TETRAHEDRAL fractions sorted f1 >= f2 >= f3, path 000 -> 111 along the
                 axes in that order, weights 1-f1, f1-f2, f2-f3, f3: 4 corners.
   Angular channels (H; angles A and B) are interpolated as circular data: the
   angle of the weighted sum of the nodes' unit vectors, within 2 float32 ulp of
   atan2 (H in [0, 2 pi), SCT angles in (-pi, pi]).  Grids whose bytes fit the workgroup's LDS are staged
   there; larger ones are read through the L2.  in/out as mact_transform.
   Errors: MACT_E_INVALID (NULL, n outside 2..256, bad method, shapes). */
mact_status lut_interp(const float* dev_lut, int32_t n, int32_t xform, int32_t method,
                       const mact_image* in, const mact_image* out, void* hip_stream);

/* Cell-major form of an N^3 LUT, the counterpart of the caching LUTs of
   Sec. 3.5.3 (which store neighbour information in every node to save
   per-pixel work): (N-1)^3 cells, cell (i, j, k) at index (i (N-1) + j) (N-1)
   + k, each holding its 8 corner nodes in the order dR dG dB = 000, 001, 010,
   011, 100, 101, 110, 111, nodes as in lut_bytes (for SCT the 8 (N-1)^3 nodes
   are followed by their L values, one float each, in the same order).  One
   pixel's corners are then one contiguous 128-byte run (and 32 bytes of L for
   SCT) rather than four runs N and N^2 nodes apart.  Returns the bytes, 0 for
   invalid arguments. */
size_t lut_cells_bytes(int32_t xform, int32_t n);

/* Fills `dev_cells` (caller-owned device buffer, >= lut_cells_bytes bytes,
   16-byte aligned) with the cell-major form of the packed LUT `dev_lut` (as
   lut_build writes it, on the device, 16-byte aligned); node values are copied
   bit for bit.  Asynchronous on `hip_stream`.
   Errors: MACT_E_INVALID (NULL, misaligned, n outside 2..256, short buffer). */
mact_status lut_cells_build(const float* dev_lut, int32_t n, int32_t xform, float* dev_cells, size_t bytes,
                            void* hip_stream);

/* lut_interp on the cell-major form: the same extraction, methods, weights and
   summation order, hence bitwise the same outputs; the cells are always read
   through the L2 (they are 8x the packed grid's bytes).  Arguments and errors
   as lut_interp. */
mact_status lut_cells_interp(const float* dev_cells, int32_t n, int32_t xform, int32_t method,
                             const mact_image* in, const mact_image* out, void* hip_stream);

/* The caching LUT of Sec. 3.5.3: the paper's second version of every method,
   which precomputes the differences between neighbouring lattice points and
   stores them with each node.  (N-1)^3 records, record (i, j, k) at index
   (i (N-1) + j) (N-1) + k for the node (i, j, k) as the 000 corner of its cell,
   each of 13 entries of C floats: entry 0 the node value c000; entries 1-4 the
   R edges c(1,g,b) - c(0,g,b) for (g, b) = 00, 01, 10, 11; 5-8 the G edges
   c(r,1,b) - c(r,0,b) for (r, b) = 00, 01, 10, 11; 9-12 the B edges
   c(r,g,1) - c(r,g,0) for (r, g) = 00, 01, 10, 11.  C = 3 (LAB: L*, a*, b*;
   LUV: L*, u*, v*), 4 (HSI: cos H, sin H, S, I) or 5 (SCT: L, cos A, sin A,
   cos B, sin B).  Returns the bytes (rounded up to 16), 0 for invalid
   arguments. */
size_t lut_cache_bytes(int32_t xform, int32_t n);

/* Builds the caching form on the host: the exact transform at every node in
   FP64 (as lut_build), the differences in FP64, each value rounded once to
   float32; copies it to `dev_cache` (caller-owned device buffer, >=
   lut_cache_bytes bytes, 16-byte aligned) on `hip_stream` and returns after
   the copy has completed.  n in 2..256; gamma applies to LAB and LUV.
   Errors: MACT_E_INVALID (NULL, misaligned, n, gamma, short buffer);
   MACT_E_DEVICE. */
mact_status lut_cache_build(int32_t xform, int32_t n, int32_t gamma, float* dev_cache, size_t bytes,
                            void* hip_stream);

/* Interpolation with the caching form: the same extraction as lut_interp, then
   the pixel's record: entry 0 plus each of the method's edge differences times
   its weight (trilinear 7, prism 5, pyramidal 4, tetrahedral 3 terms; the
   corner weights of lut_interp regrouped along paths from c000, so the result
   equals lut_interp's up to float32 rounding, not bitwise).  Records that fit
   the LDS beside the store buffers (9^3 LAB, HSI) are staged there; the rest
   are read through the L2.  Arguments and errors as lut_interp. */
mact_status lut_cache_interp(const float* dev_cache, int32_t n, int32_t xform, int32_t method,
                             const mact_image* in, const mact_image* out, void* hip_stream);

/* ------------------------------------------------------------ batched form */

/* Launch shape picked by the autotuner (or given by the caller). */
typedef struct mact_tune {
  int32_t block;      /* threads per workgroup of the general batched kernel: 64, 128, 256, 512, 1024
                         (the class kernels of the vector path use 256) */
  int32_t tile;       /* pixels per work tile: multiple of 256 and of the block, >= block */
  int32_t vec;        /* 4: packed 8-bit, 16-bit and float16 HWC images with packed float32 HWC
                         output run through the class kernels, 4 pixels per lane; 1: every image
                         through the general kernel, one pixel per lane */
  int32_t waves_per_cu; /* 1..64: persistent grid = CUs x this / (block / 64) workgroups, capped
                           by the tile count; 0: one workgroup per tile */
  int32_t one_launch; /* 1: each class's tiles in one launch; 0: equal launches of at most
                         2^26 pixels of tiles each (a large batch becomes several kernel nodes
                         of one graph: streaming launches of that size measured faster) */
} mact_tune;

typedef struct mact_batch_plan mact_batch_plan;

/* A batched transform of `count` images of any sizes, element types, layouts
   and transforms (image i uses params[i], in[i], out[i]) captured in one HIP
   graph.  The images are cut into tiles of `tile` pixels and grouped into
   classes: images of one element type (packed 8-bit, float16 or 16-bit HWC in,
   packed float32 HWC out), one transform, one coefficient set and one transfer
   function form a class run by a kernel specialised for it (the plain hot
   kernel's shape); every other image goes through a general kernel.  Either a
   persistent grid sized to the GPU walks a class's tiles (waves_per_cu > 0)
   or one workgroup takes each tile (waves_per_cu = 0), in one launch per class
   (one_launch = 1) or in equal launches of at most 2^26 pixels.  The
   autotuner chooses among all of these by time on the batch itself; on MI355X
   it picks one workgroup per 2048-pixel tile, which measured faster than a
   persistent grid (a persistent grid walking a streaming workload holds fewer
   bytes in flight).  The per-pixel arithmetic is that of mact_transform, so
   every output is bitwise equal to the plain call's.  The
   plan copies the descriptors to device memory (library-owned), picks the
   launch shape with the autotuner when `tune` is NULL (timings on `hip_stream`,
   cached per GPU and shape class; a JSON cache file is read and written when the
   MACT_AUTOTUNE_CACHE environment variable names one), and captures the launch
   in a HIP graph.  The image buffers must stay valid while the plan is used.
   Errors: as mact_transform for any image; MACT_E_NOMEM; MACT_E_DEVICE. */
mact_status mact_batch_plan_create(const mact_params* params, const mact_image* in, const mact_image* out,
                                   int32_t count, const mact_tune* tune, void* hip_stream,
                                   mact_batch_plan** plan);
/* Replays the captured graph on `hip_stream` (use_graph = 1) or launches the
   persistent kernel directly (use_graph = 0). */
mact_status mact_batch_plan_launch(mact_batch_plan* plan, int32_t use_graph, void* hip_stream);
/* The launch shape the plan uses. */
mact_status mact_batch_plan_tune(const mact_batch_plan* plan, mact_tune* tune);
/* Waits for nothing: the caller synchronises its stream before destroying. */
mact_status mact_batch_plan_destroy(mact_batch_plan* plan);
/* Create + launch (graph) + stream synchronise + destroy. */
mact_status mact_batch_run(const mact_params* params, const mact_image* in, const mact_image* out,
                           int32_t count, const mact_tune* tune, void* hip_stream);

/* ------------------------------------------------------------ serving */

/* A continuous-batching engine on the current device.  Requests carry host
   (pinned) input and output buffers.  A scheduler thread admits a request, in
   arrival order, when its device bytes fit in the engine's arena (a first-fit
   free list over one allocation, 256-byte granules), copies it in on a copy
   stream, and groups every request whose input has arrived into one persistent
   batched launch on the next free of `compute_streams` streams; batches overlap
   on the device, and requests that arrive while batches are in flight join the
   next one.  Outputs go back on one device-to-host stream, smallest first
   within a batch, and each request completes when its own output has landed.
   Coefficients stay resident in the engine.  The scheduler makes every HIP call
   after creation, without holding the locks that submit / poll / wait take, so
   those never wait on device work.

   mact_server_create allocates the arena and per-stream buffers, clears the
   arena once and runs one small request through every stream (so that first-use
   costs fall on creation, not on the first requests), then starts the
   scheduler.  Errors: MACT_E_INVALID (config out of range), MACT_E_NOMEM,
   MACT_E_DEVICE. */
typedef struct mact_server_config {
  size_t arena_bytes;      /* device memory for request inputs and outputs */
  int32_t max_batch;       /* most requests in one launch */
  int32_t compute_streams; /* concurrent batches in flight (1..8) */
  int32_t max_queue;       /* submitted but not admitted requests before MACT_E_BUSY */
  int32_t fail_request;    /* fault injection for tests of the error path: the request with this id is
                              rejected when its batch is built, as if its descriptors were invalid,
                              and completes with MACT_E_INVALID; 0 in normal use */
  mact_params params[4];   /* per transform: LAB, HSI, SCT, LUV */
} mact_server_config;

typedef struct mact_request {
  const void* host_in;     /* pinned host pixels, packed HWC */
  void* host_out;          /* pinned host output, packed HWC */
  int32_t in_dtype;        /* MACT_U8, MACT_U16, MACT_F16 or MACT_F32 */
  int32_t out_dtype;       /* MACT_F32 or MACT_F16 */
  int32_t xform;           /* MACT_LAB / MACT_HSI / MACT_SCT / MACT_LUV */
  int32_t gamma;           /* LAB / LUV input transfer function */
  int64_t width, height;
} mact_request;

typedef struct mact_server_stats {
  int64_t submitted, completed, rejected, batches;
  double p50_ms, p99_ms, mean_ms; /* submit -> output copied back, completed requests */
  double mean_batch;              /* requests per launch */
  double device_busy_ms;          /* sum of batch kernel times */
  int64_t failed;                 /* requests completed with an error status */
  int64_t cancelled;              /* requests withdrawn before admission (mact_server_cancel) */
} mact_server_stats;

typedef struct mact_server mact_server;

mact_status mact_server_create(const mact_server_config* cfg, mact_server** srv);
/* Queue a request; *id receives its handle.  MACT_E_BUSY if max_queue requests
   are already waiting (nothing is queued); MACT_E_INVALID if it could never fit
   the arena or its fields are out of range. */
mact_status mact_server_submit(mact_server* srv, const mact_request* req, int64_t* id);
/* *done = 1 once request `id` has completed.  A request completes either with
   its host_out written (MACT_OK) or with an error: its descriptors were
   rejected, or a copy, the launch or an event of its batch reported a HIP
   error.  For a request completed with an error, poll sets *done = 1 and
   returns that status (the detail in mact_last_error); host_out is then
   unspecified. */
mact_status mact_server_poll(mact_server* srv, int64_t id, int32_t* done);
/* Block until request `id` completes or timeout_ms passes (MACT_E_BUSY).
   Returns the request's status: MACT_OK, or the error it completed with
   (MACT_E_INVALID, MACT_E_DEVICE, MACT_E_CANCELLED) as poll reports it. */
mact_status mact_server_wait(mact_server* srv, int64_t id, int32_t timeout_ms);
/* Withdraws request `id` if it is still waiting for admission (no device
   memory, copy or launch has been given to it yet): it completes at once with
   MACT_E_CANCELLED, which poll and wait then report, and the engine never
   touches its host buffers again; the call returns MACT_OK.  A request already
   admitted (its copies or batch may be in flight, or it has completed) runs to
   completion and the call returns MACT_E_BUSY; MACT_E_INVALID for an unknown
   id. */
mact_status mact_server_cancel(mact_server* srv, int64_t id);
/* Latency of a completed request in milliseconds (submit -> output on host);
   the request's error status if it completed with one. */
mact_status mact_server_latency(mact_server* srv, int64_t id, double* ms);
mact_status mact_server_stats_get(mact_server* srv, mact_server_stats* st);
/* Drains every queued request, stops the scheduler, frees the arena. */
mact_status mact_server_destroy(mact_server* srv);

/* ------------------------------------------------------------ reference kernels */

/* The byte pattern of the packed 8-bit -> float32 transform with no
   arithmetic: reads n_px * 3 bytes from src and writes n_px * 12 bytes to dst
   (the bytes widened to floats).  It measures the practical HBM ceiling of the
   hot path's access pattern. */
mact_status mact_stream_u8_to_f32(const void* src, void* dst, int64_t n_px, void* hip_stream);
/* Plain 16-byte-vector copy of `bytes` (a multiple of 16). */
mact_status mact_copy(const void* src, void* dst, int64_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* MACT_H */
