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

// The same for rows that can be read four channels at a time (C % 4 == 0,
// 16-byte aligned): block = 64 four-channel groups x 4 interleaved row lanes,
// partial maxima combined in LDS, one atomic per channel and block.
__global__ void __launch_bounds__(256) k_chan_absmax4(const float* __restrict__ in, int64_t n,
                                                      int64_t C, int64_t rows_per_block,
                                                      uint32_t* __restrict__ amax) {
  __shared__ float4 s_m[4][64];
  const int quad = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int64_t c4 = (int64_t)blockIdx.x * 64 + quad;  // index of a 4-channel group
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_block;
  const int64_t r1 = min(n, r0 + rows_per_block);
  float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
  if (4 * c4 < C) {
    const float4* src = (const float4*)in + c4;
    const int64_t stride = C / 4;
#pragma unroll 4
    for (int64_t r = r0 + rl; r < r1; r += 4) {
      const float4 v = src[r * stride];
      m.x = fmaxf(m.x, fabsf(v.x));
      m.y = fmaxf(m.y, fabsf(v.y));
      m.z = fmaxf(m.z, fabsf(v.z));
      m.w = fmaxf(m.w, fabsf(v.w));
    }
  }
  s_m[rl][quad] = m;
  __syncthreads();
  if (rl == 0 && 4 * c4 < C) {
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      const float4 o = s_m[k][quad];
      m.x = fmaxf(m.x, o.x);
      m.y = fmaxf(m.y, o.y);
      m.z = fmaxf(m.z, o.z);
      m.w = fmaxf(m.w, o.w);
    }
    atomicMax(&amax[4 * c4 + 0], __float_as_uint(m.x));
    atomicMax(&amax[4 * c4 + 1], __float_as_uint(m.y));
    atomicMax(&amax[4 * c4 + 2], __float_as_uint(m.z));
    atomicMax(&amax[4 * c4 + 3], __float_as_uint(m.w));
  }
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

// One block per row at a time (grid-stride over rows), threads over channels.
template <int kDtype>
__global__ void __launch_bounds__(256) k_encode(const float* __restrict__ in, int64_t n,
                                                int64_t C, const float* __restrict__ scale,
                                                void* __restrict__ out) {
  const int64_t total = n * C;
  for (int64_t row = blockIdx.x; row < n; row += gridDim.x)
  for (int64_t c = threadIdx.x; c < C; c += blockDim.x) {
    const int64_t i = row * C + c;
    const float x = in[i];
    if (kDtype == HCG_BF16) {
      ((uint16_t*)out)[i] = (uint16_t)f32_to_bf16(x);
    } else if (kDtype == HCG_BF16_SPLIT) {
      const uint32_t hi = f32_to_bf16(x);
      ((uint16_t*)out)[i] = (uint16_t)hi;
      ((uint16_t*)out)[total + i] = (uint16_t)f32_to_bf16(x - bf16_to_f32(hi));
    } else if (kDtype == HCG_F16_SCALED) {
      ((uint16_t*)out)[i] = (uint16_t)f32_to_f16(x / scale[c]);
    } else if (kDtype == HCG_FP8E4M3_SPLIT) {
      const float y = x / scale[c];
      const uint32_t hi = f32_to_e4m3_cvt(y);
      ((uint8_t*)out)[i] = (uint8_t)hi;
      ((uint8_t*)out)[total + i] = (uint8_t)f32_to_e4m3_cvt(y - e4m3_cvt_to_f32(hi));
    } else {
      ((uint8_t*)out)[i] = (uint8_t)f32_to_e4m3_cvt(x / scale[c]);
    }
  }
}

// The same for rows that can be read four channels at a time (C % 4 == 0,
// input 16-byte and output 8-byte aligned): one thread per 4 consecutive
// elements, one 16-byte load and one 8-byte (16-bit forms) or 4-byte (FP8)
// store per plane.  Element for element the arithmetic of k_encode.
template <int kDtype>
__global__ void __launch_bounds__(256) k_encode4(const float* __restrict__ in, int64_t n,
                                                 int64_t C, const float* __restrict__ scale,
                                                 void* __restrict__ out) {
  constexpr bool k8 = (kDtype == HCG_FP8E4M3_SCALED || kDtype == HCG_FP8E4M3_SPLIT);
  constexpr bool kSplit = (kDtype == HCG_BF16_SPLIT || kDtype == HCG_FP8E4M3_SPLIT);
  constexpr bool kScaled = (kDtype == HCG_F16_SCALED || k8);
  const int64_t total = n * C;
  const int64_t quads = total / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < quads; k += stride) {
    const float4 v = ((const float4*)in)[k];
    const float xv[4] = {v.x, v.y, v.z, v.w};
    const int64_t c0 = (4 * k) % C;  // a quad lies inside one row
    uint32_t h[4], l[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float x = kScaled ? xv[j] / scale[c0 + j] : xv[j];
      l[j] = 0u;
      if (kDtype == HCG_BF16) {
        h[j] = f32_to_bf16(x);
      } else if (kDtype == HCG_BF16_SPLIT) {
        h[j] = f32_to_bf16(x);
        l[j] = f32_to_bf16(x - bf16_to_f32(h[j]));
      } else if (kDtype == HCG_F16_SCALED) {
        h[j] = f32_to_f16(x);
      } else {
        h[j] = f32_to_e4m3_cvt(x);
        if (kSplit) l[j] = f32_to_e4m3_cvt(x - e4m3_cvt_to_f32(h[j]));
      }
    }
    if (k8) {
      ((uint32_t*)out)[k] = h[0] | (h[1] << 8) | (h[2] << 16) | (h[3] << 24);
      if (kSplit)
        ((uint32_t*)((uint8_t*)out + total))[k] = l[0] | (l[1] << 8) | (l[2] << 16) | (l[3] << 24);
    } else {
      ((uint2*)out)[k] = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
      if (kSplit)
        ((uint2*)((uint16_t*)out + total))[k] = make_uint2(l[0] | (l[1] << 16), l[2] | (l[3] << 16));
    }
  }
}

// One element in the storage code of a form (x already divided by its scale
// for the scaled forms); lo: the code of the remainder for the split forms.
template <int kDtype>
__device__ __forceinline__ uint32_t encode_elem(float x, uint32_t* lo) {
  if (kDtype == HCG_BF16) return f32_to_bf16(x);
  if (kDtype == HCG_BF16_SPLIT) {
    const uint32_t hi = f32_to_bf16(x);
    *lo = f32_to_bf16(x - bf16_to_f32(hi));
    return hi;
  }
  if (kDtype == HCG_F16_SCALED) return f32_to_f16(x);
  const uint32_t hi = f32_to_e4m3_cvt(x);
  if (kDtype == HCG_FP8E4M3_SPLIT) *lo = f32_to_e4m3_cvt(x - e4m3_cvt_to_f32(hi));
  return hi;
}

// Plan-ordered encoding: element (sorted position p, channel c) of a plane
// sits at ((p / 8) Cp + c) 8 + p % 8 with Cp = C rounded up to 16, so the 8
// sorted samples of a group are contiguous for each channel; positions
// p >= n and channels c >= C (the padding) hold zero.  One thread per
// (group, channel): 8 row reads through the plan's permutation, one 16-byte
// (16-bit forms) or 8-byte (FP8) store per plane.
template <int kDtype>
__global__ void __launch_bounds__(256) k_encode_packed(const float* __restrict__ in, int64_t n,
                                                       int64_t C, const uint32_t* __restrict__ perm,
                                                       const float* __restrict__ scale,
                                                       void* __restrict__ out, int64_t plane) {
  constexpr bool k8 = (kDtype == HCG_FP8E4M3_SCALED || kDtype == HCG_FP8E4M3_SPLIT);
  constexpr bool kSplit = (kDtype == HCG_BF16_SPLIT || kDtype == HCG_FP8E4M3_SPLIT);
  constexpr bool kScaled = (kDtype == HCG_F16_SCALED || k8);
  const int64_t groups = (n + 7) / 8;
  const int64_t Cp = (C + 15) & ~int64_t(15);
  for (int64_t grp = blockIdx.x; grp < groups; grp += gridDim.x)
  for (int64_t c = threadIdx.x; c < Cp; c += blockDim.x) {
    const int64_t i = grp * Cp + c;
    const float sc = (kScaled && c < C) ? scale[c] : 1.f;
    uint32_t hw[4] = {0u, 0u, 0u, 0u}, lw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t pos = grp * 8 + t;
      if (pos >= n || c >= C) break;
      const float x = in[(int64_t)perm[pos] * C + c];
      uint32_t l = 0u;
      const uint32_t h = encode_elem<kDtype>(kScaled ? x / sc : x, &l);
      if (k8) {
        hw[t >> 2] |= h << (8 * (t & 3));
        lw[t >> 2] |= l << (8 * (t & 3));
      } else {
        hw[t >> 1] |= h << (16 * (t & 1));
        lw[t >> 1] |= l << (16 * (t & 1));
      }
    }
    if (k8) {
      ((uint2*)out)[i] = make_uint2(hw[0], hw[1]);
      if (kSplit) ((uint2*)((uint8_t*)out + plane))[i] = make_uint2(lw[0], lw[1]);
    } else {
      ((uint4*)out)[i] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
      if (kSplit) ((uint4*)((uint16_t*)out + plane))[i] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
  }
}

// The same encoding for rows that can be read four channels at a time
// (C % 4 == 0, 16-byte aligned): one thread per (group of 8 sorted samples,
// 4 channels), whose 8 row reads are 16-byte loads all in flight at once and
// whose 4 (or 8, split) stores are contiguous.  Element for element the same
// arithmetic as k_encode_packed, so the same bytes.
template <int kDtype>
__global__ void __launch_bounds__(256) k_encode_packed4(const float* __restrict__ in, int64_t n,
                                                        int64_t C, const uint32_t* __restrict__ perm,
                                                        const float* __restrict__ scale,
                                                        void* __restrict__ out, int64_t plane) {
  constexpr bool k8 = (kDtype == HCG_FP8E4M3_SCALED || kDtype == HCG_FP8E4M3_SPLIT);
  constexpr bool kSplit = (kDtype == HCG_BF16_SPLIT || kDtype == HCG_FP8E4M3_SPLIT);
  constexpr bool kScaled = (kDtype == HCG_F16_SCALED || k8);
  const int64_t groups = (n + 7) / 8;
  const int64_t Cp = (C + 15) & ~int64_t(15);
  const int64_t qpg = Cp / 4;  // 4-channel quads per group, padding included
  const int64_t total = groups * qpg;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const int64_t grp = idx / qpg;
    const int64_t q = idx - grp * qpg;
    const int64_t c0 = 4 * q;
    uint32_t hw[4][4], lw[4][4];  // [channel of the quad][word]
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < 4; ++k) hw[j][k] = lw[j][k] = 0u;
    if (c0 < C) {  // C % 4 == 0: the whole quad is inside the row
      float sc[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) sc[j] = kScaled ? scale[c0 + j] : 1.f;
      float4 x[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int64_t pos = grp * 8 + t;
        x[t] = (pos < n) ? ((const float4*)(in + (int64_t)perm[pos] * C))[q]
                         : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (grp * 8 + t >= n) break;
        const float xv[4] = {x[t].x, x[t].y, x[t].z, x[t].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          uint32_t l = 0u;
          const uint32_t h = encode_elem<kDtype>(kScaled ? xv[j] / sc[j] : xv[j], &l);
          if (k8) {
            hw[j][t >> 2] |= h << (8 * (t & 3));
            lw[j][t >> 2] |= l << (8 * (t & 3));
          } else {
            hw[j][t >> 1] |= h << (16 * (t & 1));
            lw[j][t >> 1] |= l << (16 * (t & 1));
          }
        }
      }
    }
    const int64_t i = grp * Cp + c0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (k8) {
        ((uint2*)out)[i + j] = make_uint2(hw[j][0], hw[j][1]);
        if (kSplit) ((uint2*)((uint8_t*)out + plane))[i + j] = make_uint2(lw[j][0], lw[j][1]);
      } else {
        ((uint4*)out)[i + j] = make_uint4(hw[j][0], hw[j][1], hw[j][2], hw[j][3]);
        if (kSplit)
          ((uint4*)((uint16_t*)out + plane))[i + j] = make_uint4(lw[j][0], lw[j][1], lw[j][2], lw[j][3]);
      }
    }
  }
}

// Per-channel power-of-two scales of the scaled forms into chan_scale.
static hcg_status channel_scales(const float* in, int64_t n, int64_t nchan, hcg_dtype dtype,
                                 float* chan_scale, hipStream_t stream) {
  HCG_HIP(hipMemsetAsync(chan_scale, 0, sizeof(float) * nchan, stream));
  if (n > 0 && nchan % 4 == 0 && (uintptr_t)in % 16 == 0) {
    // about 16 waves' worth of rows per block and a few blocks per CU
    const int64_t rows_per_block = std::max<int64_t>(256, (n + 2047) / 2048);
    const dim3 grid((unsigned)((nchan / 4 + 63) / 64),
                    (unsigned)((n + rows_per_block - 1) / rows_per_block));
    k_chan_absmax4<<<grid, 256, 0, stream>>>(in, n, nchan, rows_per_block,
                                              (uint32_t*)chan_scale);
    HCG_LAUNCH_CHECK("k_chan_absmax4");
  } else if (n > 0) {
    const int64_t rows_per_block = std::max<int64_t>(64, (n + 255) / 256);
    const dim3 grid((unsigned)((nchan + 255) / 256),
                    (unsigned)((n + rows_per_block - 1) / rows_per_block));
    k_chan_absmax<<<grid, 256, 0, stream>>>(in, n, nchan, rows_per_block, (uint32_t*)chan_scale);
    HCG_LAUNCH_CHECK("k_chan_absmax");
  }
  const float top = (dtype == HCG_F16_SCALED) ? 16384.f : 448.f;
  k_chan_scale<<<(unsigned)((nchan + 255) / 256), 256, 0, stream>>>(chan_scale, nchan, top);
  HCG_LAUNCH_CHECK("k_chan_scale");
  return HCG_OK;
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
    st = channel_scales(in, n, nchan, dtype, chan_scale, stream);
    if (st != HCG_OK) return st;
  }
  if (n == 0) return HCG_OK;
  const unsigned blocks = (unsigned)std::min<int64_t>(n, 1 << 18);
  // rows read four channels at a time where the layout allows it
  const bool quads = nchan % 4 == 0 && (uintptr_t)in % 16 == 0 && (uintptr_t)out % 8 == 0;
  const unsigned blocks4 = (unsigned)std::min<int64_t>((n * nchan / 4 + 255) / 256, int64_t(1) << 22);
#define HCG_ENC(D)                                                                 \
  if (quads)                                                                       \
    k_encode4<D><<<blocks4, 256, 0, stream>>>(in, n, nchan, chan_scale, out);      \
  else                                                                             \
    k_encode<D><<<blocks, 256, 0, stream>>>(in, n, nchan, chan_scale, out)
  switch (dtype) {
    case HCG_BF16: HCG_ENC(HCG_BF16); break;
    case HCG_BF16_SPLIT: HCG_ENC(HCG_BF16_SPLIT); break;
    case HCG_F16_SCALED: HCG_ENC(HCG_F16_SCALED); break;
    case HCG_FP8E4M3_SPLIT: HCG_ENC(HCG_FP8E4M3_SPLIT); break;
    default: HCG_ENC(HCG_FP8E4M3_SCALED); break;
  }
#undef HCG_ENC
  HCG_LAUNCH_CHECK("k_encode");
  return HCG_OK;
}

extern "C" hcg_status hcg_quantize_packed(hcg_plan_t plan, const float* in, int64_t nchan,
                                          hcg_dtype dtype, void* out, float* chan_scale,
                                          void* hip_stream) {
  if (!plan) return fail(HCG_E_ARG, "hcg_quantize_packed: plan is NULL");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_quantize_packed: not a live plan");
  if (nchan < 1) return fail(HCG_E_ARG, "hcg_quantize_packed: nchan must be >= 1");
  if (!in || !out) return fail(HCG_E_ARG, "hcg_quantize_packed: NULL pointer");
  const bool scaled = (dtype == HCG_F16_SCALED || dtype == HCG_FP8E4M3_SCALED ||
                       dtype == HCG_FP8E4M3_SPLIT);
  if (dtype != HCG_BF16 && dtype != HCG_BF16_SPLIT && !scaled)
    return fail(HCG_E_ARG, "hcg_quantize_packed: dtype %d is not a low-precision form", (int)dtype);
  if (scaled && !chan_scale) return fail(HCG_E_ARG, "hcg_quantize_packed: chan_scale is required");
  if (!scaled && chan_scale) return fail(HCG_E_ARG, "hcg_quantize_packed: chan_scale must be NULL");
  const bool k8 = (dtype == HCG_FP8E4M3_SCALED || dtype == HCG_FP8E4M3_SPLIT);
  if ((uintptr_t)out % (k8 ? 8 : 16) != 0)
    return fail(HCG_E_ARG, "hcg_quantize_packed: out must be %d-byte aligned", k8 ? 8 : 16);
  const hcg_plan_s* p = plan;
  hipStream_t stream = (hipStream_t)hip_stream;
  const int64_t n = p->n;
  if (scaled) {
    hcg_status st = channel_scales(in, n, nchan, dtype, chan_scale, stream);
    if (st != HCG_OK) return st;
  }
  const int64_t cp = (nchan + 15) & ~int64_t(15);
  const int64_t plane = (n + 7) / 8 * 8 * cp;  // elements per plane
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 7) / 8, 1 << 18);
  // rows read four channels at a time where they allow it
  const bool quads = nchan % 4 == 0 && (uintptr_t)in % 16 == 0;
  const unsigned blocks4 =
      (unsigned)std::min<int64_t>(((n + 7) / 8 * (cp / 4) + 255) / 256, int64_t(1) << 22);
#define HCG_PACK(D)                                                                           \
  if (quads)                                                                                  \
    k_encode_packed4<D><<<blocks4, 256, 0, stream>>>(in, n, nchan, p->perm, chan_scale, out, \
                                                      plane);                                \
  else                                                                                        \
    k_encode_packed<D><<<blocks, 256, 0, stream>>>(in, n, nchan, p->perm, chan_scale, out,   \
                                                    plane)
  switch (dtype) {
    case HCG_BF16: HCG_PACK(HCG_BF16); break;
    case HCG_BF16_SPLIT: HCG_PACK(HCG_BF16_SPLIT); break;
    case HCG_F16_SCALED: HCG_PACK(HCG_F16_SCALED); break;
    case HCG_FP8E4M3_SCALED: HCG_PACK(HCG_FP8E4M3_SCALED); break;
    default: HCG_PACK(HCG_FP8E4M3_SPLIT); break;
  }
#undef HCG_PACK
  HCG_LAUNCH_CHECK("k_encode_packed");
  return HCG_OK;
}
