// Encoders for the low-precision storage forms of hcg_grid: float32 spectra
// [n][C] -> BF16, BF16 hi + lo planes, FP16, OCP FP8 E4M3 or E4M3 hi + lo
// planes with one power-of-two scale per channel (so that scaling and
// unscaling are exact).
#include <cmath>

#include "hcg_internal.h"

namespace hcg {

// Per-channel max |x| as float bits (ordered like the values for x >= 0).
// Block (256 threads) = 256 channels x a slice of rows.
__global__ void __launch_bounds__(256) k_chan_absmax(const float* __restrict__ in, int64_t n,
                                                     int64_t C, int64_t rows_per_block,
                                                     uint32_t* __restrict__ amax) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= C) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_block;
  const int64_t r1 = min(n, r0 + rows_per_block);
  float m = 0.f;
  for (int64_t r = r0; r < r1; ++r) m = fmaxf(m, fabsf(in[r * C + c]));
  atomicMax(&amax[c], __float_as_uint(m));
}

// scale = 2^ceil(log2(max|x| / top)); 1 for an all-zero or non-finite channel
__global__ void k_chan_scale(float* __restrict__ scale, int64_t C, float top) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const float m = scale[c];  // holds max |x| written by k_chan_absmax
  float s = 1.f;
  if (m > 0.f && isfinite(m)) {
    int e;
    const float f = frexpf(m / top, &e);  // m / top = f 2^e, f in [0.5, 1)
    s = ldexpf(1.f, (f > 0.5f) ? e : e - 1);
  }
  scale[c] = s;
}

template <int kDtype>
__global__ void __launch_bounds__(256) k_encode(const float* __restrict__ in, int64_t total,
                                                int64_t C, const float* __restrict__ scale,
                                                void* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float x = in[i];
    if (kDtype == HCG_BF16) {
      ((uint16_t*)out)[i] = (uint16_t)f32_to_bf16(x);
    } else if (kDtype == HCG_BF16_SPLIT) {
      const uint32_t hi = f32_to_bf16(x);
      ((uint16_t*)out)[i] = (uint16_t)hi;
      ((uint16_t*)out)[total + i] = (uint16_t)f32_to_bf16(x - bf16_to_f32(hi));
    } else if (kDtype == HCG_F16_SCALED) {
      ((uint16_t*)out)[i] = (uint16_t)f32_to_f16(x / scale[i % C]);
    } else if (kDtype == HCG_FP8E4M3_SPLIT) {
      const float y = x / scale[i % C];
      const uint32_t hi = f32_to_e4m3(y);
      ((uint8_t*)out)[i] = (uint8_t)hi;
      ((uint8_t*)out)[total + i] = (uint8_t)f32_to_e4m3(y - e4m3_to_f32(hi));
    } else {
      ((uint8_t*)out)[i] = (uint8_t)f32_to_e4m3(x / scale[i % C]);
    }
  }
}

}  // namespace hcg

using namespace hcg;

extern "C" hcg_status hcg_quantize(const float* in, int64_t n, int64_t nchan, hcg_dtype dtype,
                                   void* out, float* chan_scale, void* hip_stream) {
  if (n < 0 || nchan < 1) return fail(HCG_E_ARG, "hcg_quantize: bad shape");
  if (n > 0 && (!in || !out)) return fail(HCG_E_ARG, "hcg_quantize: NULL pointer");
  const bool scaled = (dtype == HCG_F16_SCALED || dtype == HCG_FP8E4M3_SCALED ||
                       dtype == HCG_FP8E4M3_SPLIT);
  if (dtype != HCG_BF16 && dtype != HCG_BF16_SPLIT && !scaled)
    return fail(HCG_E_ARG, "hcg_quantize: dtype %d is not a low-precision form", (int)dtype);
  if (scaled && !chan_scale) return fail(HCG_E_ARG, "hcg_quantize: chan_scale is required");
  hcg_status st = check_device_arch();
  if (st != HCG_OK) return st;
  hipStream_t stream = (hipStream_t)hip_stream;
  if (scaled) {
    HCG_HIP(hipMemsetAsync(chan_scale, 0, sizeof(float) * nchan, stream));
    if (n > 0) {
      const int64_t rows_per_block = std::max<int64_t>(64, (n + 255) / 256);
      const dim3 grid((unsigned)((nchan + 255) / 256),
                      (unsigned)((n + rows_per_block - 1) / rows_per_block));
      k_chan_absmax<<<grid, 256, 0, stream>>>(in, n, nchan, rows_per_block,
                                              (uint32_t*)chan_scale);
      HCG_LAUNCH_CHECK("k_chan_absmax");
    }
    const float top = (dtype == HCG_F16_SCALED) ? 16384.f : 448.f;
    k_chan_scale<<<(unsigned)((nchan + 255) / 256), 256, 0, stream>>>(chan_scale, nchan, top);
    HCG_LAUNCH_CHECK("k_chan_scale");
  }
  const int64_t total = n * nchan;
  if (total == 0) return HCG_OK;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  switch (dtype) {
    case HCG_BF16:
      k_encode<HCG_BF16><<<blocks, 256, 0, stream>>>(in, total, nchan, chan_scale, out);
      break;
    case HCG_BF16_SPLIT:
      k_encode<HCG_BF16_SPLIT><<<blocks, 256, 0, stream>>>(in, total, nchan, chan_scale, out);
      break;
    case HCG_F16_SCALED:
      k_encode<HCG_F16_SCALED><<<blocks, 256, 0, stream>>>(in, total, nchan, chan_scale, out);
      break;
    case HCG_FP8E4M3_SPLIT:
      k_encode<HCG_FP8E4M3_SPLIT><<<blocks, 256, 0, stream>>>(in, total, nchan, chan_scale, out);
      break;
    default:
      k_encode<HCG_FP8E4M3_SCALED><<<blocks, 256, 0, stream>>>(in, total, nchan, chan_scale, out);
      break;
  }
  HCG_LAUNCH_CHECK("k_encode");
  return HCG_OK;
}
