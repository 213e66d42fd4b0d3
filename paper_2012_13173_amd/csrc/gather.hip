// Data stage of the gridding library: Eq. (1) of HCGrid (Section 2.1) for
// every output cell and channel, gather-side (Section 2.2: each cell pulls
// the samples within its support, so no two workgroups write the same cell).
//
// Work decomposition: one workgroup per 8 x 8 tile of output cells (and per
// 256- or 512-channel slab for many channels).  The tile's candidate samples
// come from the plan's sorted-sample ranges and are staged in blocks of 64,
// one block ahead:
//   1. weights: FP64 great-circle distance of every (cell, candidate) pair
//      of the block that a coarse per-cell-block test cannot rule out (from
//      the chord of the unit vectors), exact support test, Gaussian weight
//      (exponent in FP64; exp2 in FP32 for the matrix-core forms, in FP64 for
//      the few-channel path), rounded to the operand type of the form; FP64
//      sums of the weights per cell;
//   2. accumulation: for many channels the block is a dense contraction
//      U[cells x channels] += Wt[cells x 64] . S[64 x channels] done on the
//      matrix cores with FP32 accumulation -- FP32 operands
//      (v_mfma_f32_16x16x4_f32) or BF16 / FP16 / FP8 operands (16x16x32),
//      skipping every 16-cell x k-step sub-block whose weights are all zero;
//      the spectra are read in the caller's sample order through the plan's
//      permutation, or (low-precision forms) from an encoding in the plan's
//      sorted order whose groups of 8 samples are ready-made B operands;
//      for a few FP32 channels each lane owns one cell and accumulates in
//      FP64;
//   3. epilogue: V = U / W~ (W~ the sum of the weights actually multiplied,
//      times the channel scale for the scaled forms), NaN where no sample is
//      within the support; W map = FP64 sum of the unrounded weights.
#include <cmath>
#include <mutex>
#include <vector>

#include "gather_tile.h"

namespace hcg {

template <int kForm, int kQW, bool kVec, bool kPacked, bool kWide, bool kGen = false,
          bool kMask = false>
__global__ void __launch_bounds__(256, 2) k_gather_mfma(const GatherArgs a) {
  __shared__ GatherSmem sm;
  // XCD-aware order: the hardware deals consecutive workgroups to the eight
  // XCDs in turn; give each XCD a contiguous run of tiles so that tiles that
  // share candidate rows run together behind the same L2.
  const int per_slab = a.tiles_per_xcd * 8;
  const int slab = blockIdx.x / per_slab;
  const int local = blockIdx.x - slab * per_slab;
  const int tile = (local & 7) * a.tiles_per_xcd + (local >> 3);
  if (tile >= a.ntiles) return;
  gather_tile<kForm, kQW, kVec, kPacked, kWide, true, kGen, kMask>(a, tile, slab, sm);
}

// ---------------------------------------------------------------------------
// Few channels (C <= 8) and pair counting: one lane per cell of the 8 x 8
// tile, candidates staged 64 at a time, weights summed in FP64.
// A map of few tiles gives too few waves to hide the latency of the
// candidate loads, so the candidates of a tile can be split over nsplit
// workgroups (blockIdx.y takes every nsplit-th staged block of 64); each
// then writes its FP64 partial sums to part[split][kSlots][tile * 64 + lane]
// (the channel sums, then W, or with flags the channel weight sums) and
// k_cells_finish adds them in split order.  nsplit = 1 writes the map
// directly.  kMask: a non-finite value is a flag, left out of its channel's
// sums (numerator and weights); the per-channel weights go to wcube.
// kGen: a kernel shape other than the circular Gaussian (FP64 weights
// through pair_weight_gen); the Gaussian kernels do not carry that path.
// ---------------------------------------------------------------------------
template <int kCM, bool kMask>
struct CellSlots {
  static constexpr int kW = kMask ? kCM : 1;  // weight sums per cell
  static constexpr int kN = kCM + kW;         // partial sums per cell
};

template <int kCM, bool kCount, bool kMask = false, bool kGen = false>
__global__ void __launch_bounds__(64) k_gather_cells(
    const double4* __restrict__ cells, const double4* __restrict__ xyz,
    const uint32_t* __restrict__ perm, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ nranges, int maxr, const float* __restrict__ spectra, int C,
    GridGeom g, int ntx, double c2R, KernelParams kp, float* __restrict__ cube,
    float* __restrict__ wmap, float* __restrict__ wcube,
    unsigned long long* __restrict__ pair_count, int nsplit, double* __restrict__ part) {
  constexpr int kM = kCM > 0 ? kCM : 1;
  constexpr int kW = CellSlots<kM, kMask>::kW;
  // LDS of cells_lds_bytes(kM, maxr): staged vectors and values, then the
  // tile's ranges sized to the plan's largest range count (not to
  // kMaxRangesLimit), so that many one-wave workgroups fit on a CU
  extern __shared__ __align__(16) unsigned char s_dyn[];
  double4* s_xyz = (double4*)s_dyn;                   // [kKB]
  float (*s_spec)[kM] = (float (*)[kM])(s_xyz + kKB);  // [kKB][kM]
  uint2* s_rng = (uint2*)(s_spec + kKB);              // [maxr]
  uint32_t* s_pre = (uint32_t*)(s_rng + maxr);        // [maxr + 1]

  const int tile = blockIdx.x;
  const int lane = threadIdx.x;
  const int tx = tile % ntx, ty = tile / ntx;
  const int ix = tx * kTileX + (lane & 7), iy = ty * kTileY + (lane >> 3);
  const CellVec cell = cell_at(cells, g, ix, iy);
  const CellFrame frame = (kGen && kp.type == kElliptic) ? cell_frame(cell)
                                                         : CellFrame{0.0, 0.0, 0.0, 0.0, 0.0};
  const uint32_t total = stage_ranges(ranges + (int64_t)tile * maxr, nranges[tile], s_rng, s_pre);

  double accv[kM];
  double wsum[kW];
#pragma unroll
  for (int c = 0; c < kM; ++c) accv[c] = 0.0;
#pragma unroll
  for (int c = 0; c < kW; ++c) wsum[c] = 0.0;
  unsigned long long npair = 0;
  uint32_t cur = 0;
  const uint32_t step = (uint32_t)nsplit * kKB;
  for (uint32_t q0 = blockIdx.y * (uint32_t)kKB; q0 < total; q0 += step) {
    const uint32_t q = q0 + lane;
    if (q < total) {
      const uint32_t pos = cand_pos(q, s_rng, s_pre, &cur);
      s_xyz[lane] = xyz[pos];
      if (!kCount) {
        const int64_t row = perm[pos];
#pragma unroll
        for (int c = 0; c < kM; ++c) s_spec[lane][c] = (c < C) ? spectra[row * C + c] : 0.f;
      }
    } else {
      const double nan = __builtin_nan("");
      s_xyz[lane] = make_double4(nan, nan, nan, nan);
    }
    __syncthreads();
    const int kmax = (int)min<uint32_t>(kKB, total - q0);
    for (int k = 0; k < kmax; ++k) {
      const double4 v = s_xyz[k];
      const double c2 = chord2(cell, v);
      if (c2 <= c2R) {
        if (kCount) {
          ++npair;
        } else {
          const double w = kGen ? pair_weight_gen(kp, c2, v, cell, frame)
                                : pair_weight64(c2, kp.wscale);
          if constexpr (kMask) {
#pragma unroll
            for (int c = 0; c < kM; ++c) {
              const float x = s_spec[k][c];
              if ((__float_as_uint(x) & 0x7F800000u) != 0x7F800000u) {
                accv[c] += w * (double)x;
                wsum[c] += w;
              }
            }
          } else {
            wsum[0] += w;
#pragma unroll
            for (int c = 0; c < kM; ++c) accv[c] += w * (double)s_spec[k][c];
          }
        }
      }
    }
    __syncthreads();
  }
  if (kCount) {
    for (int off = 32; off > 0; off >>= 1) npair += __shfl_xor(npair, off);
    if (lane == 0) atomicAdd(pair_count, npair);
    return;
  }
  if (nsplit > 1) {
    const int64_t slots = (int64_t)gridDim.x * kTileCells;
    double* out = part + (int64_t)blockIdx.y * (kM + kW) * slots + (int64_t)tile * kTileCells + lane;
#pragma unroll
    for (int c = 0; c < kM; ++c) out[c * slots] = accv[c];
#pragma unroll
    for (int c = 0; c < kW; ++c) out[(kM + c) * slots] = wsum[c];
    return;
  }
  if (ix >= g.nx || iy >= g.ny) return;
  const int64_t G = (int64_t)g.nx * g.ny;
  const int64_t cellidx = (int64_t)iy * g.nx + ix;
  if (!kMask && wmap) wmap[cellidx] = (float)wsum[0];
#pragma unroll
  for (int c = 0; c < kM; ++c) {
    if (c >= C) continue;
    const double wc = wsum[kMask ? c : 0];
    cube[c * G + cellidx] = (wc != 0.0) ? (float)(accv[c] / wc) : __builtin_nanf("");
    if (kMask && wcube) wcube[c * G + cellidx] = (float)wc;
  }
}

// Sum of the nsplit partial sums of every cell, in split order; V and W.
template <int kCM, bool kMask = false>
__global__ void __launch_bounds__(256) k_cells_finish(const double* __restrict__ part, int nsplit,
                                                       int ntiles, int C, GridGeom g, int ntx,
                                                       float* __restrict__ cube,
                                                       float* __restrict__ wmap,
                                                       float* __restrict__ wcube) {
  constexpr int kW = CellSlots<kCM, kMask>::kW;
  const int64_t slots = (int64_t)ntiles * kTileCells;
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= slots) return;
  const int tile = (int)(slot / kTileCells), lane = (int)(slot % kTileCells);
  const int ix = (tile % ntx) * kTileX + (lane & 7), iy = (tile / ntx) * kTileY + (lane >> 3);
  if (ix >= g.nx || iy >= g.ny) return;
  double accv[kCM], wsum[kW];
#pragma unroll
  for (int c = 0; c < kCM; ++c) accv[c] = 0.0;
#pragma unroll
  for (int c = 0; c < kW; ++c) wsum[c] = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) {
    const double* in = part + (int64_t)sp * (kCM + kW) * slots + slot;
#pragma unroll
    for (int c = 0; c < kCM; ++c) accv[c] += in[c * slots];
#pragma unroll
    for (int c = 0; c < kW; ++c) wsum[c] += in[(kCM + c) * slots];
  }
  const int64_t G = (int64_t)g.nx * g.ny;
  const int64_t cellidx = (int64_t)iy * g.nx + ix;
  if (!kMask && wmap) wmap[cellidx] = (float)wsum[0];
#pragma unroll
  for (int c = 0; c < kCM; ++c) {
    if (c >= C) continue;
    const double wc = wsum[kMask ? c : 0];
    cube[c * G + cellidx] = (wc != 0.0) ? (float)(accv[c] / wc) : __builtin_nanf("");
    if (kMask && wcube) wcube[c * G + cellidx] = (float)wc;
  }
}

// A map of fewer than kCellsSplitBelow tiles is spread over about
// kCellsTargetGroups workgroups (eight per CU); from about 2000 tiles on, a
// split of two measured slower than none (the partial sums cost more than
// the extra waves gain).
constexpr int kCellsSplitBelow = 1024;
constexpr int kCellsTargetGroups = 2048;
constexpr int kCellsMaxSplit = 64;

// Split of a map's candidate lists and the bytes of FP64 partial sums it
// needs (0 when the gather writes the map directly).
static int cells_split(unsigned ntiles) {
  return (ntiles >= (unsigned)kCellsSplitBelow)
             ? 1
             : (int)std::min<int64_t>(kCellsMaxSplit, (kCellsTargetGroups + ntiles - 1) / ntiles);
}
// Dynamic LDS of k_gather_cells for km staged values per candidate.
static size_t cells_lds_bytes(int km, int maxr) {
  return sizeof(double4) * kKB + sizeof(float) * kKB * km + sizeof(uint2) * maxr +
         sizeof(uint32_t) * (maxr + 1);
}

static size_t cells_part_bytes(int nsplit, int cm, bool mask, unsigned ntiles) {
  if (nsplit <= 1) return 0;
  const int slots = cm + (mask ? cm : 1);
  return sizeof(double) * (size_t)nsplit * slots * ntiles * kTileCells;
}

// part: caller-provided scratch of cells_part_bytes(...) bytes, or NULL to
// allocate it stream-ordered here (one workgroup per tile if that fails).
static hcg_status launch_cells(const hcg_plan_s* p, const float* spec, int C, float* cube,
                               float* wmap, float* wcube, bool mask, double* part,
                               hipStream_t stream) {
  const double c2R = support_chord2(p);
  const unsigned ntiles = (unsigned)(p->ntx * p->nty);
  const int cm = (C == 1) ? 1 : (C == 2) ? 2 : (C <= 4) ? 4 : 8;
  int nsplit = cells_split(ntiles);
  bool owned = false;
  if (nsplit > 1 && !part) {
    const size_t bytes = cells_part_bytes(nsplit, cm, mask, ntiles);
    hipMemPool_t pool = plan_pool();
    if ((pool ? hipMallocFromPoolAsync((void**)&part, bytes, pool, stream)
              : hipMallocAsync((void**)&part, bytes, stream)) != hipSuccess) {
      (void)hipGetLastError();  // no room for the partial sums: one workgroup per tile
      part = nullptr;
      nsplit = 1;
    } else {
      owned = true;
    }
  }
  const dim3 grid(ntiles, (unsigned)nsplit);
  const unsigned fin_blocks = (unsigned)((ntiles * (int64_t)kTileCells + 255) / 256);
  // the circular Gaussian and the other kernel shapes are separate kernels,
  // so the common case carries no general weight path in its registers
  const bool gen = p->kern.type != kGauss;
#define HCG_CELLS(CM, MASK, GEN)                                                               \
  do {                                                                                         \
    k_gather_cells<CM, false, MASK, GEN><<<grid, 64, cells_lds_bytes(CM, p->maxr), stream>>>(  \
        p->cells, p->xyz, p->perm, p->ranges, p->nranges, p->maxr, spec, C, p->grid, p->ntx,   \
        c2R, p->kern, cube, wmap, wcube, nullptr, nsplit, part);                               \
    if (nsplit > 1)                                                                            \
      k_cells_finish<CM, MASK><<<fin_blocks, 256, 0, stream>>>(part, nsplit, (int)ntiles, C,   \
                                                               p->grid, p->ntx, cube, wmap,    \
                                                               wcube);                         \
  } while (0)
#define HCG_CELLS_CM(MASK, GEN)               \
  do {                                        \
    if (cm == 1) HCG_CELLS(1, MASK, GEN);      \
    else if (cm == 2) HCG_CELLS(2, MASK, GEN); \
    else if (cm == 4) HCG_CELLS(4, MASK, GEN); \
    else HCG_CELLS(8, MASK, GEN);              \
  } while (0)
  if (mask) {
    if (gen) HCG_CELLS_CM(true, true);
    else HCG_CELLS_CM(true, false);
  } else {
    if (gen) HCG_CELLS_CM(false, true);
    else HCG_CELLS_CM(false, false);
  }
#undef HCG_CELLS_CM
#undef HCG_CELLS
  const hipError_t le = hipGetLastError();
  if (owned) (void)hipFreeAsync(part, stream);
  if (le != hipSuccess)
    return fail(HCG_E_DEVICE, "launch of k_gather_cells failed: %s", hipGetErrorString(le));
  return HCG_OK;
}

// Below this many 512-channel workgroups (two per CU on 256 CUs, twice
// over) a gather takes 256-channel slabs.
constexpr int64_t kFewGroups = 1024;

template <int kForm, bool kPacked = false, bool kMask = false>
static hcg_status launch_mfma(const hcg_plan_s* p, const void* spec, const void* spec_lo,
                              const float* scale, int64_t C, float* cube, float* wmap,
                              hipStream_t stream, float* wcube = nullptr) {
  static_assert(!(kPacked && kForm == kF32), "plan-ordered spectra are a low-precision input");
  GatherArgs a;
  memset(&a, 0, sizeof(a));
  a.cells = p->cells;
  a.kern = p->kern;
  a.wcube = wcube;
  a.xyz = p->xyz;
  a.sentinel = (uint32_t)p->n;
  a.perm = p->perm;
  a.ranges = p->ranges;
  a.nranges = p->nranges;
  a.maxr = p->maxr;
  a.spec = spec;
  a.spec_lo = spec_lo;
  a.scale = scale;
  a.C = C;
  a.g = p->grid;
  a.ntx = p->ntx;
  a.ntiles = p->ntx * p->nty;
  a.tiles_per_xcd = (a.ntiles + 7) / 8;
  a.c2R = support_chord2(p);
  a.cube = cube;
  a.wmap = wmap;
  const size_t esz = (kForm == kF32) ? 4 : is_fp8(kForm) ? 1 : 2;
  // plan-ordered spectra are read 8 samples of a channel at a time
  const bool vec = kPacked || ((C % 4 == 0) && ((uintptr_t)spec % (4 * esz) == 0) &&
                               (!spec_lo || (uintptr_t)spec_lo % (4 * esz) == 0));
  if (kPacked && ((uintptr_t)spec % (8 * esz) != 0 || (uintptr_t)spec_lo % (8 * esz) != 0))
    return fail(HCG_E_ARG, "hcg_grid_packed: spectra must be %zu-byte aligned", 8 * esz);
  a.vec = vec ? 1 : 0;
  // 512-channel slabs (weights computed once per 512 channels) where the
  // registers allow it, else 256; a map of few tiles takes 256-channel slabs
  // too, for twice the workgroups (512-channel slabs would leave CUs idle)
  const int64_t groups512 = (int64_t)a.ntiles * ((C + 511) / 512);
  // the other kernel shapes and the flagged form keep to 256-channel slabs
  // (registers for the cell frame, or for the weight-sum accumulators)
  const bool gen = p->kern.type != kGauss;
  // supports below 0.57 deg (squared chord < 1e-4) take the kernels with the
  // short distance series
  const bool wide = !(a.c2R < kNarrowChord2);
  // the narrow-support 512-channel kernels of BF16, FP16 x scale and FP8 x
  // scale in input order read a row's channels eight at a time
  const bool rows8 = kPacked || wide || !(kForm == kBF16 || kForm == kF16S || kForm == kFP8S) ||
                     (C % 8 == 0 && (uintptr_t)spec % (8 * esz) == 0);
  const int qw = (C > 256 && vec && rows8 && kForm != kBF16Split && !gen && !kMask &&
                  groups512 >= kFewGroups) ? 2 : 1;
  const int64_t slab_ch = 256 * qw;
  const int64_t slabs = (C + slab_ch - 1) / slab_ch;
  const int64_t blocks = slabs * a.tiles_per_xcd * 8;
  if (blocks > INT32_MAX) return fail(HCG_E_UNSUPPORTED, "hcg_grid: too many channels");
  const dim3 grid((unsigned)blocks), block(256);
#define HCG_MFMA(QW, VEC)                                                                \
  do {                                                                                   \
    if (wide) k_gather_mfma<kForm, QW, VEC, kPacked, true><<<grid, block, 0, stream>>>(a); \
    else k_gather_mfma<kForm, QW, VEC, kPacked, false><<<grid, block, 0, stream>>>(a);    \
  } while (0)
  if (gen || kMask) {
    // one instance per form and row access: the general distance series,
    // 256-channel slabs
    if constexpr (kPacked) {
      k_gather_mfma<kForm, 1, true, true, true, true, false><<<grid, block, 0, stream>>>(a);
    } else if constexpr (kMask) {
      if (vec) {
        if (gen) k_gather_mfma<kForm, 1, true, false, true, true, true><<<grid, block, 0, stream>>>(a);
        else k_gather_mfma<kForm, 1, true, false, true, false, true><<<grid, block, 0, stream>>>(a);
      } else {
        if (gen) k_gather_mfma<kForm, 1, false, false, true, true, true><<<grid, block, 0, stream>>>(a);
        else k_gather_mfma<kForm, 1, false, false, true, false, true><<<grid, block, 0, stream>>>(a);
      }
    } else {
      if (vec) k_gather_mfma<kForm, 1, true, false, true, true, false><<<grid, block, 0, stream>>>(a);
      else k_gather_mfma<kForm, 1, false, false, true, true, false><<<grid, block, 0, stream>>>(a);
    }
    HCG_LAUNCH_CHECK("k_gather_mfma");
    return HCG_OK;
  }
  if constexpr (kForm != kBF16Split) {
    if (qw == 2) {
      HCG_MFMA(2, true);
      HCG_LAUNCH_CHECK("k_gather_mfma");
      return HCG_OK;
    }
  }
  if constexpr (kPacked) {
    HCG_MFMA(1, true);
  } else {
    if (vec) HCG_MFMA(1, true);
    else HCG_MFMA(1, false);
  }
#undef HCG_MFMA
  HCG_LAUNCH_CHECK("k_gather_mfma");
  return HCG_OK;
}

}  // namespace hcg

using namespace hcg;

namespace hcg {

// Scratch of the entry point that allocates nothing: the FP64 partial sums of
// the few-channel gather's split candidate lists live in this array, one copy
// per device for the life of the process.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it passes the device address that hipGetSymbolAddress returns on
// each device, looked up once per device with that device current.
constexpr size_t kNoAllocScratchBytes = HCG_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxScratchDevices] = {};

// Device address of the current device's scratch array.
static hcg_status scratch_address(void** out, const char* where) {
  int dev = -1;
  const hipError_t ge = hipGetDevice(&dev);
  if (ge != hipSuccess) return fail(HCG_E_DEVICE, "%s: hipGetDevice failed: %s", where, hipGetErrorString(ge));
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(HCG_E_UNSUPPORTED, "%s: device %d is beyond the %d devices served", where, dev,
                kMaxScratchDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(HCG_E_DEVICE, "%s: hipGetSymbolAddress of the scratch array failed: %s", where,
                  hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return HCG_OK;
}

// hcg_grid and hcg_grid_noalloc: the same kernels; with noalloc the
// few-channel gather's partial sums go to the static scratch array instead of
// stream-ordered memory.
static hcg_status grid_dispatch(const char* where, hcg_plan_t plan, const void* spectra,
                                int64_t nchan, hcg_dtype dtype, const float* chan_scale,
                                float* cube, float* weights, void* hip_stream, bool noalloc) {
  if (!plan) return fail(HCG_E_ARG, "%s: plan is NULL", where);
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "%s: not a live plan", where);
  if (!spectra || !cube) return fail(HCG_E_ARG, "%s: spectra and cube must not be NULL", where);
  if (nchan < 1) return fail(HCG_E_ARG, "%s: nchan must be >= 1", where);
  const bool scaled = (dtype == HCG_F16_SCALED || dtype == HCG_FP8E4M3_SCALED ||
                       dtype == HCG_FP8E4M3_SPLIT);
  if (dtype < HCG_F32 || dtype > HCG_FP8E4M3_SPLIT)
    return fail(HCG_E_UNSUPPORTED, "%s: unknown dtype %d", where, (int)dtype);
  if (scaled && !chan_scale) return fail(HCG_E_ARG, "%s: chan_scale is required for this dtype", where);
  if (!scaled && chan_scale) return fail(HCG_E_ARG, "%s: chan_scale must be NULL for this dtype", where);
  const hcg_plan_s* p = plan;
  hipStream_t stream = (hipStream_t)hip_stream;
  switch (dtype) {
    case HCG_F32:
      if (nchan <= 8) {
        double* part = nullptr;
        if (noalloc) {
          const unsigned ntiles = (unsigned)(p->ntx * p->nty);
          const int cm = (nchan == 1) ? 1 : (nchan == 2) ? 2 : (nchan <= 4) ? 4 : 8;
          const size_t need = cells_part_bytes(cells_split(ntiles), cm, false, ntiles);
          if (need > kNoAllocScratchBytes)
            return fail(HCG_E_UNSUPPORTED,
                        "%s: the partial sums of this map need %zu bytes of scratch, more than "
                        "the %zu the library holds", where, need, kNoAllocScratchBytes);
          if (need > 0) {
            void* s = nullptr;
            const hcg_status st = scratch_address(&s, where);
            if (st != HCG_OK) return st;
            part = (double*)s;
          }
        }
        return launch_cells(p, (const float*)spectra, (int)nchan, cube, weights, nullptr, false,
                            part, stream);
      }
      return launch_mfma<kF32>(p, spectra, nullptr, nullptr, nchan, cube, weights, stream);
    case HCG_BF16:
      return launch_mfma<kBF16>(p, spectra, nullptr, nullptr, nchan, cube, weights, stream);
    case HCG_BF16_SPLIT:
      return launch_mfma<kBF16Split>(p, spectra,
                                     (const char*)spectra + (size_t)2 * p->n * nchan, nullptr,
                                     nchan, cube, weights, stream);
    case HCG_F16_SCALED:
      return launch_mfma<kF16S>(p, spectra, nullptr, chan_scale, nchan, cube, weights, stream);
    case HCG_FP8E4M3_SCALED:
      return launch_mfma<kFP8S>(p, spectra, nullptr, chan_scale, nchan, cube, weights, stream);
    case HCG_FP8E4M3_SPLIT:
      return launch_mfma<kFP8Split>(p, spectra, (const char*)spectra + (size_t)p->n * nchan,
                                    chan_scale, nchan, cube, weights, stream);
  }
  return fail(HCG_E_UNSUPPORTED, "%s: dtype %d", where, (int)dtype);
}

}  // namespace hcg

extern "C" hcg_status hcg_grid(hcg_plan_t plan, const void* spectra, int64_t nchan,
                               hcg_dtype dtype, const float* chan_scale, float* cube,
                               float* weights, void* hip_stream) {
  return grid_dispatch("hcg_grid", plan, spectra, nchan, dtype, chan_scale, cube, weights,
                       hip_stream, false);
}

extern "C" hcg_status hcg_grid_noalloc(hcg_plan_t plan, const void* spectra, int64_t nchan,
                                       hcg_dtype dtype, const float* chan_scale, float* cube,
                                       float* weights, void* hip_stream) {
  return grid_dispatch("hcg_grid_noalloc", plan, spectra, nchan, dtype, chan_scale, cube,
                       weights, hip_stream, true);
}

extern "C" hcg_status hcg_grid_masked(hcg_plan_t plan, const float* spectra, int64_t nchan,
                                      float* cube, float* chan_weights, void* hip_stream) {
  if (!plan) return fail(HCG_E_ARG, "hcg_grid_masked: plan is NULL");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_grid_masked: not a live plan");
  if (!spectra || !cube) return fail(HCG_E_ARG, "hcg_grid_masked: spectra and cube must not be NULL");
  if (nchan < 1) return fail(HCG_E_ARG, "hcg_grid_masked: nchan must be >= 1");
  const hcg_plan_s* p = plan;
  hipStream_t stream = (hipStream_t)hip_stream;
  if (nchan <= 8)
    return launch_cells(p, spectra, (int)nchan, cube, nullptr, chan_weights, true, nullptr,
                        stream);
  return launch_mfma<kF32, false, true>(p, spectra, nullptr, nullptr, nchan, cube, nullptr,
                                        stream, chan_weights);
}

extern "C" hcg_status hcg_packed_bytes(hcg_plan_t plan, int64_t nchan, hcg_dtype dtype,
                                       int64_t* bytes) {
  if (!plan || !bytes) return fail(HCG_E_ARG, "hcg_packed_bytes: NULL pointer");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_packed_bytes: not a live plan");
  if (nchan < 1) return fail(HCG_E_ARG, "hcg_packed_bytes: nchan must be >= 1");
  int64_t esz = 0, planes = 1;
  switch (dtype) {
    case HCG_BF16: case HCG_F16_SCALED: esz = 2; break;
    case HCG_BF16_SPLIT: esz = 2; planes = 2; break;
    case HCG_FP8E4M3_SCALED: esz = 1; break;
    case HCG_FP8E4M3_SPLIT: esz = 1; planes = 2; break;
    default: return fail(HCG_E_ARG, "hcg_packed_bytes: dtype %d is not a low-precision form", (int)dtype);
  }
  const int64_t groups = (plan->n + 7) / 8;
  *bytes = planes * groups * 8 * ((nchan + 15) & ~int64_t(15)) * esz;
  return HCG_OK;
}

extern "C" hcg_status hcg_grid_packed(hcg_plan_t plan, const void* packed, int64_t nchan,
                                      hcg_dtype dtype, const float* chan_scale, float* cube,
                                      float* weights, void* hip_stream) {
  if (!plan) return fail(HCG_E_ARG, "hcg_grid_packed: plan is NULL");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_grid_packed: not a live plan");
  if (!packed || !cube) return fail(HCG_E_ARG, "hcg_grid_packed: spectra and cube must not be NULL");
  if (nchan < 1) return fail(HCG_E_ARG, "hcg_grid_packed: nchan must be >= 1");
  const bool scaled = (dtype == HCG_F16_SCALED || dtype == HCG_FP8E4M3_SCALED ||
                       dtype == HCG_FP8E4M3_SPLIT);
  if (dtype < HCG_BF16 || dtype > HCG_FP8E4M3_SPLIT)
    return fail(HCG_E_ARG, "hcg_grid_packed: dtype %d is not a low-precision form", (int)dtype);
  if (scaled && !chan_scale) return fail(HCG_E_ARG, "hcg_grid_packed: chan_scale is required for this dtype");
  if (!scaled && chan_scale) return fail(HCG_E_ARG, "hcg_grid_packed: chan_scale must be NULL for this dtype");
  const hcg_plan_s* p = plan;
  hipStream_t stream = (hipStream_t)hip_stream;
  // elements per plane: 8 ceil(n / 8) sorted positions x nchan rounded up to 16
  const size_t plane = (size_t)((p->n + 7) / 8) * 8 * (size_t)((nchan + 15) & ~int64_t(15));
  const char* sp = (const char*)packed;
  switch (dtype) {
    case HCG_BF16:
      return launch_mfma<kBF16, true>(p, sp, sp, nullptr, nchan, cube, weights, stream);
    case HCG_BF16_SPLIT:
      return launch_mfma<kBF16Split, true>(p, sp, sp + 2 * plane, nullptr, nchan, cube, weights,
                                           stream);
    case HCG_F16_SCALED:
      return launch_mfma<kF16S, true>(p, sp, sp, chan_scale, nchan, cube, weights, stream);
    case HCG_FP8E4M3_SCALED:
      return launch_mfma<kFP8S, true>(p, sp, sp, chan_scale, nchan, cube, weights, stream);
    case HCG_FP8E4M3_SPLIT:
      return launch_mfma<kFP8Split, true>(p, sp, sp + plane, chan_scale, nchan, cube, weights,
                                          stream);
    default:
      break;
  }
  return fail(HCG_E_ARG, "hcg_grid_packed: dtype %d", (int)dtype);
}

extern "C" hcg_status hcg_get_plan_stats(hcg_plan_t plan, hcg_plan_stats* stats,
                                         void* hip_stream) {
  if (!plan || !stats) return fail(HCG_E_ARG, "hcg_get_plan_stats: NULL pointer");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_get_plan_stats: not a live plan");
  const hcg_plan_s* p = plan;
  hipStream_t stream = (hipStream_t)hip_stream;
  const unsigned ntiles = (unsigned)(p->ntx * p->nty);
  unsigned long long* dcount = nullptr;
  HCG_HIP(hipMalloc(&dcount, sizeof(unsigned long long)));
  struct Free {
    void* q;
    ~Free() { (void)hipFree(q); }
  } fr{dcount};
  HCG_HIP(hipMemsetAsync(dcount, 0, sizeof(unsigned long long), stream));
  k_gather_cells<0, true><<<ntiles, 64, cells_lds_bytes(1, p->maxr), stream>>>(
      p->cells, p->xyz, p->perm, p->ranges, p->nranges, p->maxr, nullptr, 0, p->grid, p->ntx,
      support_chord2(p), p->kern, nullptr, nullptr, nullptr, dcount, 1, nullptr);
  HCG_LAUNCH_CHECK("k_gather_cells<count>");
  unsigned long long pairs = 0;
  HCG_HIP(hipMemcpyAsync(&pairs, dcount, sizeof(pairs), hipMemcpyDeviceToHost, stream));
  std::vector<uint32_t> nc(ntiles);
  HCG_HIP(hipMemcpyAsync(nc.data(), p->ncand, sizeof(uint32_t) * ntiles, hipMemcpyDeviceToHost,
                         stream));
  HCG_HIP(hipStreamSynchronize(stream));
  int64_t cand = 0;
  for (uint32_t v : nc) cand += v;
  stats->pairs = (int64_t)pairs;
  stats->candidates = cand;
  stats->cells = (int64_t)p->grid.nx * p->grid.ny;
  return HCG_OK;
}
