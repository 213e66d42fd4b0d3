/*
 * hcg.h -- C ABI of the MI355X (gfx950) convolutional gridding library.
 *
 * Gridding resamples N non-uniform sky samples (lon_n, lat_n, spectrum s_n)
 * onto a regular lon/lat grid.  Every output cell g takes the kernel-weighted
 * mean of the samples within the support radius R (HCGrid, Wang et al. 2020,
 * Eq. (1) of Section 2.1):
 *
 *     V[c][g] = sum_n w(g,n) s_n[c] / W_g,      W_g = sum_n w(g,n),
 *     w(g,n)  = exp(-d(g,n)^2 / (2 sigma^2))   if d(g,n) <= R, else 0,
 *
 * with d the great-circle distance, sigma = FWHM / (2 sqrt(2 ln 2)) and the
 * Gaussian kernel of Section 3.6 (iii).  A cell with no sample inside R has
 * W = 0 and V = NaN.
 *
 * The work is split in two calls, following the gridding module of Section 3
 * (pre-ordering, then gather-side convolution), both done on the GPU:
 *   hcg_plan  -- geometry only: HEALPix ring-scheme pixel of every sample
 *                (Section 3.2), a stable sort of (pixel, sample index)
 *                (Section 3.3 step I), the ring lookup table (step III) and,
 *                for every tile of output cells, the sample ranges that can
 *                lie within R (the search of Section 3.4, steps i-iv).
 *   hcg_grid  -- data: weights and the channel accumulation of Eq. (1) for
 *                any number of channels, normalised, written as a cube.
 * A plan is immutable after hcg_plan returns and may be reused for any number
 * of hcg_grid calls (different spectra, channel slabs or precisions).
 *
 * Conventions for every entry point:
 *   - Angles are degrees.  Grid cell (ix, iy) is centred at
 *       lon0 + (ix - (nx-1)/2) dlon,   lat0 + (iy - (ny-1)/2) dlat.
 *   - "device" pointers are HIP device memory of the current device; the
 *     library never takes ownership of caller memory.
 *   - hip_stream is a hipStream_t (NULL = the null stream).
 *   - Every call returns a status; on any status other than HCG_OK,
 *     hcg_last_error() returns a message for the calling thread.  No C++
 *     exception crosses this interface.
 *   - The library runs on gfx950 only; it fails with HCG_E_UNSUPPORTED on
 *     any other device.
 */
#ifndef HCG_H
#define HCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hcg_plan_s* hcg_plan_t;

typedef enum {
  HCG_OK = 0,
  HCG_E_ARG = 1,          /* invalid argument (NULL, out of range, non-finite) */
  HCG_E_NOMEM = 2,        /* device memory allocation failed */
  HCG_E_DEVICE = 3,       /* a HIP call or kernel launch failed */
  HCG_E_UNSUPPORTED = 4,  /* valid request this build or device cannot serve */
  HCG_E_STATE = 5         /* handle is not a live plan */
} hcg_status;

/* Storage type of the spectra passed to hcg_grid.  Every form accumulates in
 * FP32 on the matrix cores; the weights are rounded to the operand type of
 * the form (the spectra's), and V is normalised by the sum of the weights as
 * rounded, so a constant input still maps to the same constant.
 *   HCG_F32             float32 [n][C]; FP32 weights.
 *   HCG_BF16            bfloat16 [n][C]; BF16 weights.
 *   HCG_BF16_SPLIT      two bfloat16 planes [2][n][C]: hi = bf16(x) then
 *                       lo = bf16(x - hi); weights split the same way; three
 *                       products per pair (hi.hi + hi.lo + lo.hi).
 *   HCG_F16_SCALED      float16 [n][C] holding x / scale[c]; FP16 weights;
 *                       V is multiplied back by scale[c].
 *   HCG_FP8E4M3_SCALED  OCP FP8 E4M3 [n][C] holding x / scale[c]; FP8 E4M3
 *                       weights (of 256 w, inside E4M3's normal range); V
 *                       is multiplied back by scale[c].
 *   HCG_FP8E4M3_SPLIT   two FP8 E4M3 planes [2][n][C] with one scale per
 *                       channel: hi = e4m3(x / scale[c]) then lo =
 *                       e4m3(x / scale[c] - hi); weights split the same way;
 *                       three products per pair (hi.hi + hi.lo + lo.hi).
 * hcg_quantize produces these encodings (with power-of-two scales) from
 * float32 spectra. */
typedef enum {
  HCG_F32 = 0,
  HCG_BF16 = 1,
  HCG_BF16_SPLIT = 2,
  HCG_F16_SCALED = 3,
  HCG_FP8E4M3_SCALED = 4,
  HCG_FP8E4M3_SPLIT = 5
} hcg_dtype;

/* Linear lon/lat target grid (degrees).  nx, ny >= 1; dlon, dlat finite and
 * non-zero; every cell latitude within [-90, 90]. */
typedef struct {
  int32_t nx, ny;
  double lon0_deg, lat0_deg;
  double dlon_deg, dlat_deg;
} hcg_grid_desc;

/* Tuning options; a zero field means "choose automatically".
 *   nside     HEALPix resolution (power of two, 1 .. 16384).  Auto: the
 *             smallest nside whose mean pixel size is <= sigma/2 (the
 *             hpx_max_resolution ~ sigma_kernel/2 rule of Section 3.6 (iii)).
 *   tile_x/y  output-cell tile; only 8 x 8 (or 0) is accepted.
 *   coarsen, chan_tile, flags: reserved, must be 0. */
typedef struct {
  int32_t nside;
  int32_t tile_x, tile_y;
  int32_t coarsen;
  int32_t chan_tile;
  uint32_t flags;
} hcg_opts;

/*
 * hcg_plan -- build the search geometry for N samples and one target grid.
 *
 *   out          receives the plan handle; set to NULL on failure.
 *   lon_deg,     device, float64 [n]: sample coordinates (any longitude;
 *   lat_deg      latitude within [-90, 90]; all finite).  Read only during
 *                the call; the plan keeps its own sorted copies.
 *   n            number of samples, >= 1 and < 2^31.
 *   grid         host pointer to the target grid.
 *   fwhm_deg     kernel FWHM (> 0, finite).
 *   support_deg  support radius R (>= 0, finite, < 90); Section 3.6 (iii)
 *                recommends 3 to 5 sigma.
 *   opts         host pointer or NULL (all automatic).
 *
 * Synchronous with respect to hip_stream: returns after the plan is built
 * (it reads back a few bytes once).  Errors: HCG_E_ARG for a NULL pointer,
 * n out of range, bad grid, fwhm <= 0, support < 0, nside not a power of two
 * in 1..16384, or any non-finite / out-of-range sample coordinate (checked
 * on the device); HCG_E_NOMEM; HCG_E_DEVICE; HCG_E_UNSUPPORTED for options
 * this build does not serve.  Nothing leaks on failure.
 */
hcg_status hcg_plan(hcg_plan_t* out, const double* lon_deg, const double* lat_deg, int64_t n,
                    const hcg_grid_desc* grid, double fwhm_deg, double support_deg,
                    const hcg_opts* opts, void* hip_stream);

/* Kernel shapes w(g, n) for a pair at great-circle distance d <= R
 * (Section 3.6 (iii): the Gaussian is the default; the sinc is the optimal
 * kernel of infinite length, used here with a Gaussian taper):
 *   HCG_KERNEL_GAUSS           exp(-d^2 / (2 sigma^2)), sigma from fwhm_deg.
 *   HCG_KERNEL_ELLIPTIC_GAUSS  exp(-d^2/2 [cos^2(b - pa) / sa^2 + sin^2(b - pa) / sb^2]),
 *                              b the bearing of the sample seen from the cell
 *                              (east of north), sa and sb the sigmas of the
 *                              major (fwhm_deg) and minor (fwhm_minor_deg)
 *                              axes, pa = pa_deg the position angle of the
 *                              major axis; 1 at d = 0.  At a pole the bearing
 *                              is taken in the frame of longitude 0.
 *   HCG_KERNEL_TAPERED_SINC    sinc(d / b) exp(-(d / a)^2), sinc(x) = sin(pi x) /
 *                              (pi x), b = sinc_deg, a = taper_deg.  Weights
 *                              can be negative; V is NaN where W = 0.
 * Unused fields are ignored.  The automatic nside follows the sigma/2 rule
 * with sigma of the Gaussian, of the minor axis, or half the smaller of a
 * and b. */
typedef enum {
  HCG_KERNEL_GAUSS = 0,
  HCG_KERNEL_ELLIPTIC_GAUSS = 1,
  HCG_KERNEL_TAPERED_SINC = 2
} hcg_kernel_type;

typedef struct {
  int32_t type;          /* hcg_kernel_type */
  double fwhm_deg;       /* Gaussian FWHM; elliptical: major axis */
  double fwhm_minor_deg; /* elliptical: minor axis */
  double pa_deg;         /* elliptical: position angle of the major axis */
  double sinc_deg;       /* tapered sinc: b, the first zero */
  double taper_deg;      /* tapered sinc: a, the Gaussian taper width */
} hcg_kernel;

/* Target cells given by their centres: the pixel centres of a projected
 * (WCS) map, which the paper grids onto (Section 2.1).  lon_deg / lat_deg
 * are device float64 [ny][nx]; a centre that is not finite (or |lat| > 90)
 * is a cell that no sample reaches (W = 0, V = NaN).  hcg_wcs_centres
 * computes them for the CAR, SFL, SIN and TAN projections. */
typedef struct {
  int32_t nx, ny;
  const double* lon_deg;
  const double* lat_deg;
} hcg_cell_centres;

/* A projected map: FITS world coordinates with a diagonal CDELT (Calabretta
 * & Greisen 2002, the reference the paper gives for its WCS-space gridding,
 * Section 2.1).  Pixel (ix, iy) of the [ny][nx] map is FITS pixel
 * (ix + 1, iy + 1).  lonpole: LONPOLE in degrees when lonpole_set, else its
 * default (0 when CRVAL2 >= theta_0, else 180; theta_0 = 0 for CAR and SFL,
 * 90 for SIN and TAN); latpole: LATPOLE in degrees (FITS default 90), which
 * picks between the two celestial poles a cylindrical map can have. */
typedef enum {
  HCG_PROJ_CAR = 0, /* plate carree */
  HCG_PROJ_SFL = 1, /* Sanson-Flamsteed */
  HCG_PROJ_SIN = 2, /* orthographic (no xi / eta terms) */
  HCG_PROJ_TAN = 3  /* gnomonic */
} hcg_projection;

typedef struct {
  int32_t proj;         /* hcg_projection */
  int32_t nx, ny;
  int32_t lonpole_set;
  double crpix1, crpix2; /* reference pixel (1-based) */
  double cdelt1, cdelt2; /* degrees per pixel, non-zero */
  double crval1, crval2; /* world coordinates of the reference pixel */
  double lonpole, latpole;
} hcg_wcs;

/*
 * hcg_wcs_centres -- world coordinates (lon, lat in degrees, lon in
 * [0, 360)) of every pixel centre of a projected map, into device float64
 * lon_deg / lat_deg [ny][nx]: pixel -> intermediate world coordinates ->
 * native spherical coordinates (the projection's inverse) -> celestial
 * coordinates (Paper II eq. (2), with the celestial pole from eqs. (8) to
 * (10)).  Pixels outside the projection's domain (SIN beyond its disc) get
 * NaN.  The result feeds hcg_plan_ex as hcg_cell_centres.  Asynchronous on
 * hip_stream.  Errors: HCG_E_ARG (NULL pointer, bad sizes, zero CDELT,
 * non-finite parameters, |CRVAL2| > 90, a LONPOLE that reaches no celestial
 * pole), HCG_E_UNSUPPORTED (projection), HCG_E_DEVICE.
 */
hcg_status hcg_wcs_centres(const hcg_wcs* wcs, double* lon_deg, double* lat_deg,
                           void* hip_stream);

/*
 * hcg_plan_ex -- hcg_plan for any kernel shape and for a target given
 * either as a linear grid (grid, centres = NULL) or by cell centres (grid =
 * NULL).  With centres, the candidate search of each 8 x 8 tile starts from
 * the smallest cap (about the normalised mean of its cells) that holds them,
 * widened by R; the result is the same Eq. (1).  The centre arrays are read
 * during the call only.  Errors as hcg_plan, plus HCG_E_ARG for both or
 * neither of grid and centres, bad centre dimensions or kernel parameters,
 * and HCG_E_UNSUPPORTED for an unknown kernel type or tiles whose cells
 * spread over more rings than the range table holds.
 */
hcg_status hcg_plan_ex(hcg_plan_t* out, const double* lon_deg, const double* lat_deg, int64_t n,
                       const hcg_grid_desc* grid, const hcg_cell_centres* centres,
                       const hcg_kernel* kernel, double support_deg, const hcg_opts* opts,
                       void* hip_stream);

/*
 * hcg_grid -- Eq. (1) for every cell and channel of the plan's grid.
 *
 *   spectra     device [n][nchan] in the sample order given to hcg_plan,
 *               channel-fastest, in the storage type of dtype (two planes
 *               for the split dtypes).  Any element alignment is accepted;
 *               rows read several elements at a time (nchan a multiple of
 *               4, spectra aligned to 4 elements; for BF16, FP16 x scale
 *               and FP8 x scale a multiple of 8 and 8 elements as well) are
 *               gridded faster.
 *               Values should be finite: with
 *               nchan <= 8 (FP32) a non-finite value reaches exactly the
 *               cells within R of its sample, but the matrix-core forms
 *               multiply zero weights too (0 x NaN = NaN), so it can reach
 *               any cell of an 8 x 8 tile that lists the sample as a
 *               candidate (within about R + the tile's diagonal + one
 *               HEALPix pixel).  Data with flagged (NaN) values go through
 *               hcg_grid_masked, which leaves them out channel by channel.
 *   nchan       >= 1.
 *   chan_scale  device float [nchan] for the scaled dtypes (the scales the
 *               encoding used); NULL for the others.
 *   cube        device float32 [nchan][ny][nx], caller-allocated: the
 *               normalised map V (NaN where W = 0).
 *   weights     device float32 [ny][nx] or NULL: the weight map W (FP64 sum
 *               of the unrounded weights, stored as float32).
 *
 * Asynchronous on hip_stream: returns once the work is queued; device faults
 * surface at the caller's next synchronisation.  The plan is read only, so
 * calls on different streams may overlap.  Errors: HCG_E_ARG (NULL spectra
 * or cube, nchan < 1, chan_scale missing for a scaled dtype or given for
 * another), HCG_E_UNSUPPORTED (unknown dtype), HCG_E_STATE (not a live
 * plan), HCG_E_DEVICE (launch failure).
 */
hcg_status hcg_grid(hcg_plan_t plan, const void* spectra, int64_t nchan, hcg_dtype dtype,
                    const float* chan_scale, float* cube, float* weights, void* hip_stream);

/*
 * hcg_grid_noalloc -- hcg_grid for callers that cannot allocate device
 * memory during the call: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, kernels, results and
 * errors as hcg_grid; it calls no hipMalloc, hipFree or allocating library
 * routine.  Where hcg_grid takes stream-ordered memory for partial sums (the
 * FP32 form with nchan <= 8 on maps of fewer than 1024 8 x 8 tiles), this call
 * uses a static device array of HCG_NOALLOC_SCRATCH_BYTES per device, held by
 * each device the library runs on until the process ends (every such map
 * fits: it needs at most about 14 MB); a map that would need more is refused
 * with HCG_E_UNSUPPORTED.  The partial sums are written whole before they are
 * read, so nothing carries over from an earlier call.  All calls on one
 * device share that array: calls of hcg_grid_noalloc that overlap on one
 * device (on different streams, or from different host threads without
 * ordering) race and give wrong maps; calls on one stream are ordered and
 * safe.  The first call on a device looks up the array's device address
 * once (hipGetSymbolAddress, with that device current).
 */
#define HCG_NOALLOC_SCRATCH_BYTES (16u << 20)
hcg_status hcg_grid_noalloc(hcg_plan_t plan, const void* spectra, int64_t nchan,
                            hcg_dtype dtype, const float* chan_scale, float* cube,
                            float* weights, void* hip_stream);

/*
 * hcg_grid_masked -- Eq. (1) with per-channel flags, for data whose flagged
 * values (RFI, Section 4) are non-finite: a NaN or infinite s_n[c] leaves
 * sample n out of channel c, from the numerator and from that channel's
 * weight sum alike, so every channel has its own W.
 *   spectra       device float32 [n][nchan] (input sample order).
 *   cube          device float32 [nchan][ny][nx]: V[c] = U[c] / W[c], NaN
 *                 where W[c] = 0.
 *   chan_weights  device float32 [nchan][ny][nx] or NULL: W[c] (FP64 sums
 *                 for nchan <= 8, FP32 matrix-core sums otherwise).
 * FP32 only.  Asynchronous on hip_stream.  Errors: HCG_E_ARG (NULL spectra
 * or cube, nchan < 1), HCG_E_STATE, HCG_E_DEVICE.
 */
hcg_status hcg_grid_masked(hcg_plan_t plan, const float* spectra, int64_t nchan, float* cube,
                           float* chan_weights, void* hip_stream);

/*
 * hcg_quantize -- encode float32 spectra for a low-precision form of
 * hcg_grid (the per-channel scaling of the precision forms).
 *
 *   in          device float [n][nchan].
 *   dtype       HCG_BF16, HCG_BF16_SPLIT, HCG_F16_SCALED, HCG_FP8E4M3_SCALED
 *               or HCG_FP8E4M3_SPLIT.
 *   out         device buffer: 2 n nchan bytes (BF16, F16, FP8 split: hi
 *               plane then lo plane), 4 n nchan bytes (BF16 split: hi plane
 *               then lo plane), n nchan bytes (FP8).
 *   chan_scale  device float [nchan], written for the scaled forms:
 *               scale[c] = 2^ceil(log2(max_n |x[n][c]| / top)) with top =
 *               2^14 (FP16) or 448 (the largest E4M3 value); 1 for an
 *               all-zero channel.  NULL for the unscaled forms.
 * Every element is rounded to nearest even (the scales keep every x / scale
 * within the E4M3 range, +-448).
 * Asynchronous on hip_stream.  Errors: HCG_E_ARG (shape, NULL pointer,
 * dtype not a low-precision form, missing chan_scale), HCG_E_DEVICE.
 */
hcg_status hcg_quantize(const float* in, int64_t n, int64_t nchan, hcg_dtype dtype, void* out,
                        float* chan_scale, void* hip_stream);

/*
 * Plan-ordered spectra.  The gather reads each candidate sample's spectrum
 * through the plan's permutation; a low-precision encoding can instead be
 * written once in the plan's sorted order, as the paper's pre-ordering
 * (Section 3.3, step I) reorders the raw samples, data and coordinates, by
 * pixel.  Layout of one plane, with Cp = nchan rounded up to a multiple of
 * 16: element (sorted position p, channel c) at ((p / 8) Cp + c) 8 + p % 8,
 * for p < 8 ceil(n / 8) and c < Cp (positions >= n and channels >= nchan
 * hold zero); the split forms store the hi plane, then the lo plane.  Eight
 * consecutive sorted samples of one channel are then one 16-byte (16-bit
 * forms) or 8-byte (FP8) operand of the matrix-core step, and 16 channels
 * of a group one aligned 256- or 128-byte block.
 *
 * hcg_packed_bytes -- bytes of the plan-ordered encoding of nchan channels in
 *   dtype (a low-precision form): planes x 8 ceil(n / 8) x Cp x element
 *   size.  Errors: HCG_E_ARG (NULL, nchan < 1, dtype HCG_F32 or unknown),
 *   HCG_E_STATE.
 *
 * hcg_quantize_packed -- encode float32 spectra for a low-precision form, in
 *   the plan's sorted order.
 *   in          device float [n][nchan] in the sample order given to
 *               hcg_plan (n = the plan's sample count).
 *   out         device buffer of hcg_packed_bytes bytes, 16-byte aligned
 *               (8-byte for the FP8 forms).
 *   chan_scale  as for hcg_quantize (same scales, same element codes).
 *   Asynchronous on hip_stream.  Errors: HCG_E_ARG (NULL pointer, nchan < 1,
 *   dtype not a low-precision form, chan_scale missing or given wrongly,
 *   misaligned out), HCG_E_STATE, HCG_E_DEVICE.
 *
 * hcg_grid_packed -- hcg_grid on plan-ordered spectra of the same plan
 *   (from hcg_quantize_packed or written in the same layout); the result is
 *   the one hcg_grid gives for the input-order encoding, up to the order of
 *   the FP32 accumulation.  Arguments and errors as for hcg_grid; dtype must
 *   be a low-precision form and packed suitably aligned (HCG_E_ARG).
 */
hcg_status hcg_packed_bytes(hcg_plan_t plan, int64_t nchan, hcg_dtype dtype, int64_t* bytes);
hcg_status hcg_quantize_packed(hcg_plan_t plan, const float* in, int64_t nchan, hcg_dtype dtype,
                               void* out, float* chan_scale, void* hip_stream);
hcg_status hcg_grid_packed(hcg_plan_t plan, const void* packed, int64_t nchan, hcg_dtype dtype,
                           const float* chan_scale, float* cube, float* weights,
                           void* hip_stream);

/*
 * hcg_grid_host -- hcg_grid for spectra and a cube held in host memory,
 * streamed through the device in channel slabs: the overlap of host-device
 * copies with the gridding on separate streams that Section 5 names as
 * future work, so that a cube larger than device memory can be made with one
 * plan.  Every storage form of hcg_grid can be streamed; the 16- and 8-bit
 * forms move half or a quarter of the FP32 bytes over the host link.
 *
 *   spectra_host  host memory in the sample order given to hcg_plan,
 *                 channel-fastest, in the storage of dtype as hcg_grid takes
 *                 it: [n][nchan] elements of the form, or [2][n][nchan] (the
 *                 high plane, then the low plane) for the split forms.
 *   nchan         >= 1.
 *   dtype         any hcg_dtype.
 *   chan_scale    host float [nchan] for the scaled forms (the scales the
 *                 encoding used, as hcg_quantize writes them); NULL for the
 *                 others.
 *   slab_chan     channels per slab; 0 picks 512, or fewer (a multiple of
 *                 8) where the slab buffers below would take more than a
 *                 quarter of the free device memory.  The last slab may be
 *                 shorter.
 *   cube_host     host float [nchan][ny][nx]: V as hcg_grid writes it.
 *   weights_host  host float [ny][nx] or NULL: W as hcg_grid writes it.
 *
 * Slab s + 1 is copied in on a stream of the library's while slab s is
 * gridded on hip_stream and slab s - 1 is copied out on a third stream, each
 * through two device buffers of slab_chan channels (2 slab_chan (b n + 4 nx
 * ny) bytes of device memory, b the bytes per sample and channel of the
 * form, all planes, plus 4 nx ny for W and 4 nchan for the scales, allocated
 * per call and freed on return).  Each slab is gridded by hcg_grid on the
 * slab's channels (and their scales), so the cube equals, bit for bit, what
 * hcg_grid gives for those channels on the device.  The copies overlap the
 * gridding only for page-locked host memory (hipHostMalloc); pageable memory
 * gives the same result, slower.  Synchronous: returns after the last slab
 * has reached cube_host (the work queued earlier on hip_stream runs first).
 * Errors: HCG_E_ARG (NULL pointer, nchan < 1, slab_chan < 0, a device
 * pointer given for host memory, chan_scale missing for a scaled dtype or
 * given for another), HCG_E_UNSUPPORTED (unknown dtype), HCG_E_STATE (not a
 * live plan), HCG_E_NOMEM (the slab buffers do not fit), HCG_E_DEVICE (a
 * copy or launch failed; the streams are drained before the call returns).
 */
hcg_status hcg_grid_host(hcg_plan_t plan, const void* spectra_host, int64_t nchan,
                         hcg_dtype dtype, const float* chan_scale, int64_t slab_chan,
                         float* cube_host, float* weights_host, void* hip_stream);

/*
 * hcg_grid_rowthreads -- the paper's GPU gather scheme on one channel, the
 * baseline that hcg_grid is measured against: one thread per gamma
 * consecutive cells of a latitude row (Section 3.5 I, thread organisation
 * and coarsening), each thread searching its own candidates through the
 * plan's ring table and sorted keys (Section 3.4, steps i-v) and summing in
 * FP64 registers.
 *
 *   spectra  device float [n], one value per sample, in the sample order
 *            given to hcg_plan.
 *   gamma    cells per thread, 1 .. 4 (the coarsening factor).
 *   block    threads per block, a multiple of 64 in 64 .. 512.
 *   map      device float [ny][nx]: V of Eq. (1), NaN where W = 0.
 *   weights  device float [ny][nx] or NULL: W.
 *
 * The result equals that of hcg_grid with nchan = 1 up to the order of the
 * FP64 sums.  Asynchronous on hip_stream.  Errors: HCG_E_ARG (NULL spectra
 * or map, gamma or block out of range), HCG_E_STATE (not a live plan),
 * HCG_E_DEVICE (launch failure).
 */
hcg_status hcg_grid_rowthreads(hcg_plan_t plan, const float* spectra, int gamma, int block,
                               float* map, float* weights, void* hip_stream);

/* hcg_destroy -- wait for the device, then free the plan.  NULL is a no-op
 * (HCG_OK); a handle that is not a live plan gives HCG_E_STATE.  A plan's
 * arrays, and the scratch of hcg_plan and hcg_grid, come from a stream-ordered
 * memory pool of the library's own (one per device, alive until the process
 * ends); freed memory up to 2 GiB per device stays in it for the next plan
 * instead of going back to the driver. */
hcg_status hcg_destroy(hcg_plan_t plan);

/* Message for the last non-OK status returned to the calling thread. */
const char* hcg_last_error(void);

/* ------------------------------------------------------------------------ */
/* Inspection of a plan and its intermediate arrays, for tests and tooling.  */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t n;              /* samples */
  int32_t nside;          /* HEALPix resolution used */
  int32_t key_bits;       /* significant bits of (pixel - pix_base) */
  uint32_t pix_base;      /* smallest pixel index of any sample */
  uint32_t pix_max;       /* largest pixel index of any sample */
  int32_t ring_first;     /* ring of pix_base (rings are 1 .. 4 nside - 1) */
  int32_t ring_last;      /* ring of pix_max */
  int32_t tile_x, tile_y; /* output-cell tile */
  int32_t ntiles_x, ntiles_y;
  int32_t max_ranges;     /* candidate-range slots per tile */
  int32_t sort_passes;    /* radix passes (8-bit digits) */
  double sigma_rad, support_rad;
} hcg_plan_info;

hcg_status hcg_get_plan_info(hcg_plan_t plan, hcg_plan_info* info);

/* Arrays hcg_export copies out of a plan (device to caller device memory):
 *   HCG_ARR_KEYS     uint32 [n]   sorted keys (pixel - pix_base), non-descending
 *   HCG_ARR_PERM     uint32 [n]   input index of each sorted sample (stable)
 *   HCG_ARR_RING_CSR uint32 [ring_last - ring_first + 2]  start of every ring
 *                    in the sorted order, then the end sentinel n
 *   HCG_ARR_TILE_NRANGES uint32 [ntiles]  ranges used by each tile
 *                    (tile t = ty * ntiles_x + tx)
 *   HCG_ARR_TILE_RANGES  uint32 [ntiles][max_ranges][2]  half-open [a, b)
 *                    ranges of sorted positions that may lie within R of a
 *                    cell of the tile (every such sample is covered) */
typedef enum {
  HCG_ARR_KEYS = 0,
  HCG_ARR_PERM = 1,
  HCG_ARR_RING_CSR = 2,
  HCG_ARR_TILE_NRANGES = 3,
  HCG_ARR_TILE_RANGES = 4
} hcg_array;

/* Copies array `which` into device memory dst of `bytes` bytes (must equal
 * the array size).  Asynchronous on hip_stream. */
hcg_status hcg_export(hcg_plan_t plan, hcg_array which, void* dst, int64_t bytes,
                      void* hip_stream);

/* Size in bytes of array `which` of a plan. */
hcg_status hcg_export_size(hcg_plan_t plan, hcg_array which, int64_t* bytes);

typedef struct {
  int64_t pairs;       /* (cell, sample) pairs with d <= R: the nonzeros of Eq. (1) */
  int64_t candidates;  /* sum over tiles of the candidate samples searched */
  int64_t cells;       /* nx * ny */
} hcg_plan_stats;

/* Counts the exact pair work of a plan (runs a counting kernel, then
 * synchronises hip_stream). */
hcg_status hcg_get_plan_stats(hcg_plan_t plan, hcg_plan_stats* stats, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Single steps of the plan, callable on their own (same kernels).           */
/* ------------------------------------------------------------------------ */

/* HEALPix ring-scheme pixel of every sample (Section 3.2): device float64
 * lon_deg/lat_deg [n] -> device uint32 pix [n].  nside a power of two in
 * 1..16384.  Inputs with a non-finite coordinate or |lat| > 90 get pixel
 * 0xFFFFFFFF and make the call return HCG_E_ARG (after the kernel, so the
 * call synchronises hip_stream).  n >= 0. */
hcg_status hcg_ang2pix(const double* lon_deg, const double* lat_deg, int64_t n, int32_t nside,
                       uint32_t* pix, void* hip_stream);

/* Stable LSD radix sort of uint32 keys, sorting only the low key_bits bits
 * (1..32; higher bits must be zero): device keys_in [n] -> device keys_out
 * [n] (non-descending) and perm_out [n] (input index of each output element;
 * equal keys keep input order, Section 3.3 step I).  keys_in is not
 * modified.  Synchronous with respect to hip_stream.  0 <= n < 2^31. */
hcg_status hcg_sort_keys(const uint32_t* keys_in, int64_t n, int32_t key_bits, uint32_t* keys_out,
                         uint32_t* perm_out, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Batches: many independent maps of uneven size in one persistent launch.  */
/* ------------------------------------------------------------------------ */

typedef struct hcg_batch_s* hcg_batch_t;

/* One field of a batch: the arguments of hcg_plan. */
typedef struct {
  const double* lon_deg; /* device float64 [n] */
  const double* lat_deg; /* device float64 [n] */
  int64_t n;
  hcg_grid_desc grid;
  double fwhm_deg;
  double support_deg;
} hcg_field_desc;

/* The data of one field for hcg_grid_batch: the spectra in any storage form
 * of hcg_grid (input sample order; the split dtypes hold the hi plane, then
 * the lo plane), with the channel scales of the scaled forms. */
typedef struct {
  const void* spectra;     /* device, dtype storage [n][nchan] ([2][n][nchan] split) */
  int64_t nchan;           /* >= 1 */
  int32_t dtype;           /* hcg_dtype */
  const float* chan_scale; /* device float [nchan] for the scaled dtypes, else NULL */
  float* cube;             /* device float32 [nchan][ny][nx] */
  float* weights;          /* device float32 [ny][nx] or NULL */
} hcg_field_data;

/* hcg_opts.flags of hcg_plan_batch: fix the launch strategy of
 * hcg_grid_batch (at most one; neither = autotuned). */
#define HCG_BATCH_PERSISTENT 1u /* persistent kernels popping work items */
#define HCG_BATCH_ITEMS 2u      /* one workgroup per work item */

/*
 * hcg_plan_batch -- one plan per field (the steps of hcg_plan for each).
 *   fields  host array [nfields] (pointers inside are device pointers).
 *   opts    host pointer or NULL.  opts->chan_tile selects the channel slab
 *           of the matrix-core work items: 0 = autotune on the first
 *           hcg_grid_batch call, 256 or 512 = fixed (items ordered by cost);
 *           opts->flags may fix the launch strategy (HCG_BATCH_PERSISTENT
 *           or HCG_BATCH_ITEMS); nside and tile fields apply to every field
 *           as in hcg_plan.
 * The plans are built step by step for all fields at once, on up to eight
 * streams of the library (kept for later calls) that first wait for
 * hip_stream, with one host synchronisation per build step.
 * Synchronous.  Errors as hcg_plan, with the failing field named in the
 * message (HCG_E_UNSUPPORTED for other flags); nothing leaks on failure.
 */
hcg_status hcg_plan_batch(hcg_batch_t* out, int32_t nfields, const hcg_field_desc* fields,
                          const hcg_opts* opts, void* hip_stream);

/*
 * hcg_grid_batch -- Eq. (1) for every field of the batch in one graph launch.
 *   data  host array [nfields] in the order given to hcg_plan_batch; fields
 *         may use different storage forms.
 * Every (field, tile, channel slab) is a work item.  Items are grouped by
 * kernel class (the few-channel FP32 gather, and the matrix-core gather of
 * each storage form, for rows read four elements or one at a time; a
 * BF16, FP16 x scale or FP8 x scale class takes 512-channel slabs at narrow
 * support only if every field's rows can be read eight at a time: nchan a
 * multiple of 8, spectra aligned to 8 elements); per
 * class, either a persistent kernel of two workgroups per CU pops the items
 * from per-XCD counters, or one launch runs one workgroup per item (the
 * fields' items in turn, each field's tiles dealt to the XCDs in contiguous
 * eighths).  The first call may run the batch several times to autotune the
 * channel slab, the field order (largest cost first, or as given) and the
 * launch strategy (same results every time); it then captures the classes'
 * launches in one hipGraph that later calls replay.  Pointers,
 * forms and channel counts may change between calls (the device tables are
 * rewritten before the replay, and the graph captured again when the
 * classes change; the rewrite waits for the previous launch, on whichever
 * stream it ran).  Asynchronous on hip_stream after the first call (which
 * synchronises).  Errors: HCG_E_ARG (NULL pointers, nchan < 1, chan_scale
 * missing for a scaled dtype or given for another), HCG_E_UNSUPPORTED
 * (unknown dtype), HCG_E_STATE (not a live batch), HCG_E_NOMEM,
 * HCG_E_DEVICE.  Calls on one batch must not overlap on the host (one thread
 * at a time); the outputs of successive calls are written in call order.
 */
hcg_status hcg_grid_batch(hcg_batch_t batch, const hcg_field_data* data, void* hip_stream);

/* Waits for the device, then frees the batch and its plans.  NULL is a
 * no-op; a handle that is not a live batch gives HCG_E_STATE. */
hcg_status hcg_destroy_batch(hcg_batch_t batch);

typedef struct {
  int32_t nfields;
  int32_t chan_slab;         /* channels per work item for C > 8 (256 or 512) */
  int32_t cost_order;        /* 1: items by decreasing cost; 0: by field, tile */
  int32_t tuned;             /* 1 once the configuration is fixed */
  int32_t graph_captured;    /* 1 once the launch is captured */
  int32_t persistent_blocks; /* 256-thread workgroups of the persistent kernels (the
                                C <= 8 class runs eight 64-thread ones for each) */
  int64_t items;             /* work items of the last build */
  double tune_ms[8];         /* autotuner timings, persistent then work-item
                                launch, each (256, cost), (512, cost),
                                (256, natural), (512, natural); 0 if skipped */
  int32_t launch;            /* 0: persistent kernels; 1: one workgroup per item */
  int32_t reserved;
} hcg_batch_info;

hcg_status hcg_get_batch_info(hcg_batch_t batch, hcg_batch_info* info);

/*
 * hcg_batch_get_plan -- the plan of field `field` of a batch (built by
 * hcg_plan_batch with every build step shared by all fields), for
 * inspection: hcg_get_plan_info, hcg_export, hcg_get_plan_stats and hcg_grid
 * accept it.  Borrowed: valid until hcg_destroy_batch, and hcg_destroy
 * refuses it (HCG_E_STATE).  Errors: HCG_E_ARG (NULL pointer, field out of
 * range), HCG_E_STATE (not a live batch).
 */
hcg_status hcg_batch_get_plan(hcg_batch_t batch, int32_t field, hcg_plan_t* out);

#ifdef __cplusplus
}
#endif

#endif /* HCG_H */
