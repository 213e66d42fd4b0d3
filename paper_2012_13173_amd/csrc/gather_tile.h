// Device code of the gather shared by the per-plan kernels (gather.hip) and
// the persistent batch kernels (batch.hip): candidate staging, the weights
// of Eq. (1) and the matrix-core contraction of one (tile, channel slab), and
// the one-lane-per-cell accumulation of a tile for few channels.
#pragma once

#include "hcg_internal.h"
#include "sphere.h"

namespace hcg {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kKB = 64;             // candidates staged per block

// FP32 weight of a pair inside the support: the exponent -d^2 log2(e) /
// (2 sigma^2) is formed in FP64 and evaluated with the hardware base-2
// exponential (v_exp_f32; the exponent lies in [-6.5, 0] for a 3 sigma
// support and [-18, 0] for 5 sigma, so no result is subnormal).
template <bool kWide>
__device__ __forceinline__ float pair_weight(double c2, double wscale) {
  return __builtin_amdgcn_exp2f((float)(dist2_from_chord2<kWide>(c2) * wscale));
}

// bit q (q < 8) of the result: any of bits 4q .. 4q + 3 of x
__device__ __forceinline__ uint32_t any_of_nibbles(uint32_t x) {
  x |= x >> 1;
  x |= x >> 2;
  x &= 0x11111111u;
  x = (x | (x >> 3)) & 0x03030303u;
  x = (x | (x >> 6)) & 0x000F000Fu;
  return (x | (x >> 12)) & 0xFFu;
}
// bit q (q < 4) of the result: any of bits 8q .. 8q + 7 of x
__device__ __forceinline__ uint32_t any_of_bytes(uint32_t x) {
  x |= x >> 1;
  x |= x >> 2;
  x |= x >> 4;
  x &= 0x01010101u;
  x = (x | (x >> 7)) & 0x00030003u;
  return (x | (x >> 14)) & 0xFu;
}

// Centres and coarse thresholds of the four 4 x 4 cell blocks of tile (tx,
// ty); called by threads 0..63 (block t / 16, cell t % 16).  The centre is
// the normalised mean of the block's cells inside the grid; a candidate can
// only be within R of a cell of the block if it is within R + h of the
// centre (h: the largest centre-to-cell distance; triangle inequality), so
// the threshold is the squared chord of R + h, with slack for rounding.  A
// block without cells gets threshold -1 (never marked).
__device__ inline void block_centres(const GatherArgs& a, int tx, int ty, int t, double4* ctr) {
  const GridGeom& g = a.g;
  const int cb = t >> 4, i = t & 15;
  const int x = tx * kTileX + (cb & 1) * 4 + (i & 3), y = ty * kTileY + (cb >> 1) * 4 + (i >> 2);
  const bool in_grid = x < g.nx && y < g.ny;
  const CellVec v = cell_at(a.cells, g, x, y);
  const bool valid = in_grid && v.x == v.x;  // a cell without a centre is left out
  double sx = valid ? v.x : 0.0, sy = valid ? v.y : 0.0, sz = valid ? v.z : 0.0;
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    sx += __shfl_xor(sx, o);
    sy += __shfl_xor(sy, o);
    sz += __shfl_xor(sz, o);
  }
  const double nrm = sqrt(sx * sx + sy * sy + sz * sz);
  const CellVec c{sx / nrm, sy / nrm, sz / nrm};
  double hc2 = valid ? chord2(c, make_double4(v.x, v.y, v.z, 0.0)) : 0.0;
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) hc2 = fmax(hc2, __shfl_xor(hc2, o));
  const double R = 2.0 * asin(fmin(0.5 * sqrt(a.c2R), 1.0));
  const double h = 2.0 * asin(fmin(0.5 * sqrt(hc2), 1.0));
  const double sh = sin(0.5 * fmin(R + h, kPi));
  double thr = 4.0 * sh * sh * (1.0 + 1e-9) + 1e-15;
  if (!(nrm > 0.0)) thr = -1.0;
  if (i == 0) ctr[cb] = make_double4(c.x, c.y, c.z, thr);
}

// Inclusive scans across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_scan_add(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  return x;
}
__device__ __forceinline__ uint32_t wave_scan_max(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= d) x = max(x, y);
  }
  return x;
}

// Loads the tile's candidate ranges into LDS with exclusive prefix sums;
// returns the total candidate count.  blockDim.x (>= 64) threads take part;
// with widening or rotation the first wave computes the prefix sums, 64
// ranges at a time (and s_pre needs kMaxRangesLimit + 1 entries); plain
// ranges need s_rng[nr] and s_pre[nr + 1] only.
// With npad > 0 (the sample count rounded up to a multiple of 8) every range
// is widened to whole groups of 8 sorted positions, capped at npad, and cut
// where it would overlap the previous one (the plan's ranges are disjoint
// and increasing), so that every aligned group of 8 candidates is one group
// of the plan-ordered spectra.  Samples added this way lie outside the
// plan's ranges, hence beyond R of every cell of the tile: weight 0.  The
// cut is where the previous widened range ends: the running maximum of
// max(lo rounded down, hi rounded up and capped) over the ranges before.
//
// With kPhase every range [lo, hi) is read from its phase point on: the
// first multiple w of M = (hi - lo) rounded up to kPhaseQuantum at or after
// lo, i.e. as [w, hi) followed by [lo, w).  Tiles side by side on a row of
// the map reach each ring over ranges of about the same length, shifted
// along the ring; unrotated, a tile meets a sample shared with its eastern
// neighbour about one tile width of candidates after that neighbour did,
// and the rows read by the other tiles of the XCD in that interval evict it
// from L2.  Rotated to a common phase, both meet the shared samples at about
// the same place in their lists.  The set of candidates is unchanged; the
// order only decides which of them share a matrix-core step.  A tile's
// ranges then take up to twice their number of entries, so a tile of more
// than kMaxRangesLimit / 2 ranges (a ring split at longitude 0 gives two)
// keeps the plan's order.
constexpr uint32_t kPhaseQuantum = 128;
template <bool kPhase = false>
__device__ inline uint32_t stage_ranges(const uint2* __restrict__ ranges, uint32_t nr, uint2* s_rng,
                                        uint32_t* s_pre, uint32_t npad = 0) {
  const int nt = blockDim.x;
  // rotated: the plan's ranges go to the upper half and the staged ones are
  // written from the start; a chunk of 64 reads its entries before it
  // writes, and chunk j writes below 128 j + 128 <= kMaxRangesLimit / 2 +
  // 64 (j + 1), where the next chunk's entries begin (j <= 7)
  const bool rotate = kPhase && nr <= (uint32_t)kMaxRangesLimit / 2;
  const uint32_t kIn = rotate ? kMaxRangesLimit / 2 : 0;
  for (uint32_t r = threadIdx.x; r < nr; r += nt) s_rng[kIn + r] = ranges[r];
  __syncthreads();
  if (!kPhase && npad == 0) {
    // plain ranges: one thread's loop, whose loads do not wait on the
    // running sum (faster than the wave scans, whose shuffles each wait
    // on LDS, for the few-channel gathers that stage ranges per workgroup
    // of a split tile)
    if (threadIdx.x == 0) {
      uint32_t acc = 0;
      for (uint32_t r = 0; r < nr; ++r) {
        s_pre[r] = acc;
        acc += s_rng[r].y - s_rng[r].x;
      }
      s_pre[nr] = acc;
    }
  } else if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    uint32_t end = 0, acc = 0, o = 0;  // carried from chunk to chunk
    for (uint32_t base = 0; base < nr; base += 64) {
      const uint32_t r = base + l;
      const bool live = r < nr;
      uint2 v = live ? s_rng[kIn + r] : make_uint2(0u, 0u);
      if (npad) {
        const uint32_t lo8 = v.x & ~7u;
        const uint32_t hi8 = min((v.y + 7u) & ~7u, npad);
        const uint32_t run = wave_scan_max(live ? max(lo8, hi8) : 0u, l);
        uint32_t prev = __shfl_up(run, 1);
        prev = max(l == 0 ? 0u : prev, end);
        const uint32_t lo = max(lo8, prev);
        v = live ? make_uint2(lo, max(lo, hi8)) : make_uint2(0u, 0u);
        end = max(end, (uint32_t)__shfl(run, 63));
      }
      uint32_t w = 0u;
      bool split = false;
      if (rotate && v.y > v.x) {
        const uint64_t M = (uint64_t)(v.y - v.x + kPhaseQuantum - 1) / kPhaseQuantum * kPhaseQuantum;
        const uint64_t wq = ((uint64_t)v.x + M - 1) / M * M;
        split = wq > v.x && wq < v.y;
        w = (uint32_t)wq;
      }
      const uint32_t len = v.y - v.x;
      const uint32_t cnt = live ? (split ? 2u : 1u) : 0u;
      const uint32_t cnt_in = wave_scan_add(cnt, l);
      const uint32_t len_in = wave_scan_add(len, l);
      const uint32_t at = o + cnt_in - cnt;
      const uint32_t pre = acc + len_in - len;
      if (live) {
        if (split) {
          s_rng[at] = make_uint2(w, v.y);
          s_pre[at] = pre;
          s_rng[at + 1] = make_uint2(v.x, w);
          s_pre[at + 1] = pre + (v.y - w);
        } else {
          s_rng[at] = v;
          s_pre[at] = pre;
        }
      }
      o += (uint32_t)__shfl(cnt_in, 63);
      acc += (uint32_t)__shfl(len_in, 63);
    }
    if (l == 0) {
      s_pre[o] = acc;
      s_pre[kMaxRangesLimit] = acc;
    }
  }
  __syncthreads();
  return (!kPhase && npad == 0) ? s_pre[nr] : s_pre[kMaxRangesLimit];
}

// Sorted position of candidate q; *cur is a monotone cursor over ranges.
__device__ __forceinline__ uint32_t cand_pos(uint32_t q, const uint2* s_rng, const uint32_t* s_pre,
                                             uint32_t* cur) {
  uint32_t r = *cur;
  while (q >= s_pre[r + 1]) ++r;
  *cur = r;
  return s_rng[r].x + (q - s_pre[r]);
}

// ---------------------------------------------------------------------------
// Storage forms of the spectra and of the weights on the matrix cores.
// ---------------------------------------------------------------------------
enum Form : int { kF32 = 0, kBF16 = 1, kBF16Split = 2, kF16S = 3, kFP8S = 4, kFP8Split = 5 };

constexpr bool is_fp8(int f) { return f == kFP8S || f == kFP8Split; }
constexpr bool is_split(int f) { return f == kBF16Split || f == kFP8Split; }

// The FP8 forms encode 256 w: the weights (0.011 .. 1 at a 3 sigma support)
// then sit in E4M3's normal range, where the relative rounding step is 2^-3
// everywhere.  The factor is a power of two and cancels in U / W~.
constexpr float kW8Scale = 256.f;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// Many channels: matrix-core contraction per staged block of 64 candidates.
//
// Workgroup = 4 waves, tile = 8 x 8 cells = four 4 x 4 cell blocks (MFMA M =
// 16 cells), channel slab = 4 waves x 64 QW channels.  Per block:
//  - weights: wave w computes the FP64 weights of cell block w for the 64
//    candidates (one cell per lane), rounds them to the operand type and
//    writes them to LDS in the A-operand layout; one bit per (cell block,
//    k-step) marks a non-zero sub-block;
//  - contraction: wave w streams its channels of the block's candidate rows
//    from HBM into B operands and issues the MFMAs of the non-zero
//    sub-blocks for all four cell blocks.
// Operand layouts (lane l, i = l % 16, g = l / 16):
//   FP32  v_mfma_f32_16x16x4_f32: A = w(cell i, cand 4s + g), B = spectrum of
//         cand 4s + g at channel 4i + q (MFMA q of a 64-channel group);
//   16-bit / FP8 16x16x32: A = w(cell i, cands 32s + 8g .. +7) packed, B = the
//         same 8 candidates at channel 4i + q, repacked from 8-byte (16-bit)
//         or 4-byte (FP8) row loads.
// Output D[i][j]: lane l, register r holds cell 4 (l/16) + r of the block and
// channel 4 (l % 16) + q of the group.
// ---------------------------------------------------------------------------

template <int kForm>
struct FormTraits;
template <>
struct FormTraits<kF32> { static constexpr int kK = 4; };
template <>
struct FormTraits<kBF16> { static constexpr int kK = 32; };
template <>
struct FormTraits<kBF16Split> { static constexpr int kK = 32; };
template <>
struct FormTraits<kF16S> { static constexpr int kK = 32; };
template <>
struct FormTraits<kFP8S> { static constexpr int kK = 32; };
template <>
struct FormTraits<kFP8Split> { static constexpr int kK = 32; };

// E4M3 codes of the weights (256 w <= 256, and its remainder) go through the
// conversion instructions (f32_to_e4m3_cvt), one instruction each.
template <int kForm>
__device__ __forceinline__ uint32_t enc_w(float w) {
  if (kForm == kF16S) return f32_to_f16(w);
  if (is_fp8(kForm)) return f32_to_e4m3_cvt(w * kW8Scale);
  return f32_to_bf16(w);
}
template <int kForm>
__device__ __forceinline__ float dec_w(uint32_t c) {
  if (kForm == kF16S) return f16_to_f32(c);
  if (is_fp8(kForm)) return e4m3_cvt_to_f32(c);  // in units of 1 / kW8Scale
  return bf16_to_f32(c);
}

// the 16-bit element q (0..3) of an 8-byte load
__device__ __forceinline__ uint32_t elem16(uint2 d, int q) {
  const uint32_t w = (q < 2) ? d.x : d.y;
  return (q & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// LDS slot of staged candidate k: one double4 of padding after every 8, so
// that the four 16-lane groups of a wave reading candidates 8 apart (the
// 16-bit and FP8 weights: lane l takes the 8 candidates of group l / 16)
// meet different banks instead of the same ones 256 bytes apart.
__device__ __forceinline__ int xyz_slot(int k) { return k + (k >> 3); }

// LDS of one workgroup of the gather (shared by the per-plan kernel and the
// persistent batch kernel).
struct GatherSmem {
  uint2 rng[kMaxRangesLimit];
  uint32_t pre[kMaxRangesLimit + 1];
  double4 xyz[3][kKB + kKB / 8];  // staged unit vectors, three blocks in flight (xyz_slot)
  double4 ctr[4];       // cell-block centres and coarse thresholds
  uint32_t row[3][kKB];
  uint4 Araw[2][1024];  // weights in the A-operand layout, two blocks in flight
  uint32_t nz[2][4];
  double Wt[kTileCells];
};

// B operand of one 16-channel MFMA tile from the plan-ordered spectra: 8
// sorted samples of one channel (16 bytes for the 16-bit forms, 8 for FP8).
template <int kForm>
struct PackedB {
  using T = uint4;
};
template <>
struct PackedB<kFP8S> {
  using T = uint2;
};
template <>
struct PackedB<kFP8Split> {
  using T = uint2;
};

// One (tile, channel slab) of the contraction; all 256 threads take part.
// kPacked: the spectra are plan-ordered, [ceil(n/8)][C][8] elements per plane
// (hcg_quantize_packed), so a lane's B operand (8 consecutive sorted samples
// of one channel) is one load and the loads of a block are issued before its
// weights are computed.
// kGen: a kernel shape other than the circular Gaussian (FP64 weights through
// pair_weight_gen).  kMask (FP32, input order): a non-finite spectrum value is
// a flag -- it is replaced by 0 in the product and its sample is left out of
// that channel's weight sum, accumulated by a second contraction with the
// 0/1 flags as the B operand.
template <int kForm, int kQW, bool kVec, bool kPacked, bool kWide, bool kAhead = true,
          bool kGen = false, bool kMask = false>
__device__ __forceinline__ void gather_tile(const GatherArgs& a, int tile, int slab,
                                            GatherSmem& sm) {
  static_assert(!kMask || (kForm == kF32 && !kPacked), "flags are an FP32 input-order form");
  constexpr int kK = FormTraits<kForm>::kK;
  constexpr int kNS = kKB / kK;  // k-steps per staged block
  uint2* s_rng = sm.rng;
  uint32_t* s_pre = sm.pre;
  double* s_Wt = sm.Wt;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
  const int tx = tile % a.ntx, ty = tile / a.ntx;
  const GridGeom& g = a.g;
  const int64_t C = a.C;
  const int64_t G = (int64_t)g.nx * g.ny;

  const int ci = lane & 15;
  const int my_x = tx * kTileX + (wave & 1) * 4 + (ci & 3);
  const int my_y = ty * kTileY + (wave >> 1) * 4 + (ci >> 2);
  const CellVec cell = cell_at(a.cells, g, my_x, my_y);
  const CellFrame frame = kGen ? cell_frame(cell) : CellFrame{0.0, 0.0, 0.0, 0.0, 0.0};
  // weight of this lane's cell and a staged candidate inside the support
  auto weight = [&](double c2, const double4& v) -> float {
    if constexpr (kGen) return (float)pair_weight_gen(a.kern, c2, v, cell, frame);
    else return pair_weight<kWide>(c2, a.kern.wscale);
  };

  const uint32_t total =
      stage_ranges<true>(a.ranges + (int64_t)tile * a.maxr, a.nranges[tile], s_rng, s_pre,
                         kPacked ? (a.sentinel + 7u) & ~7u : 0u);
  if (tid < 64) block_centres(a, tx, ty, tid, sm.ctr);

  floatx4 acc[4][4 * kQW];
  floatx4 accw[kMask ? 4 : 1][kMask ? 4 * kQW : 1];  // flagged form: channel weight sums
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int q = 0; q < 4 * kQW; ++q) {
      acc[cb][q] = floatx4{0.f, 0.f, 0.f, 0.f};
      if constexpr (kMask) accw[cb][q] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  double wsum = 0.0;   // FP64 sum of the unrounded weights (this lane's share)
  double wtsum = 0.0;  // FP64 sum of the weights as used in the products
  uint32_t cur = 0;
  const int64_t c_w = (int64_t)slab * (256 * kQW) + wave * (64 * kQW);
  const int64_t my_ch = c_w + 4 * (lane & 15);  // + 64 h + q
  // FP32: 64-channel groups of this wave that hold a channel < C (uniform);
  // the others issue no products (a wave past the last channel still
  // computes its cell block's weights for the others)
  const int hlive = (int)min<int64_t>(kQW, max<int64_t>(0, (C - c_w + 63) / 64));

  // Weights in the A-operand layout, one buffer per block in flight.
  auto sA32 = [&](int ab) { return (float*)sm.Araw[ab]; };   // [4][16][64]
  auto sA16 = [&](int ab) { return sm.Araw[ab]; };           // [4][kNS][64] (+ lo plane after)
  auto sA8 = [&](int ab) { return (uint2*)sm.Araw[ab]; };    // [4][kNS][64] (+ lo plane after)

  // Blocks of 64 candidates go through a three-stage pipeline with one
  // barrier per block: while block b's rows are read and multiplied, each
  // wave computes its cell block's weights of block b + 1 (from the unit
  // vectors staged one block earlier), and wave 0 stages block b + 2, whose
  // unit vectors and rows (or groups) it loaded into registers during the
  // previous block (kAhead; without it, where registers are short, it loads
  // them when it stages them).  LDS holds three staging buffers and two
  // weight buffers.
  double nx = 0.0, ny = 0.0, nz = 0.0;
  uint32_t nrow = 0u;
  // Padding past the last candidate has weight 0 (a NaN position) and the
  // row or group of the last candidate, which shares the matrix-core step
  // with every padding candidate that is ever multiplied: a non-finite
  // spectrum value then reaches no cell through padding (0 x NaN) that it
  // would not reach through its own candidate.
  uint32_t pad_row = 0u;
  if (total > 0u) {
    uint32_t c0 = 0u;
    const uint32_t last = cand_pos(total - 1u, s_rng, s_pre, &c0);
    pad_row = kPacked ? last >> 3 : a.perm[last];
  }
  pad_row = __builtin_amdgcn_readfirstlane(pad_row);
  auto fetch = [&](uint32_t qb) {
    if (wave == 0) {
      const uint32_t q = qb + tid;
      if (q < total) {
        const uint32_t pos = cand_pos(q, s_rng, s_pre, &cur);
        const double4 v = a.xyz[pos];
        nx = v.x;
        ny = v.y;
        nz = v.z;
        nrow = kPacked ? pos >> 3 : a.perm[pos];  // group of 8 sorted samples, or row
      } else {
        nx = ny = nz = __builtin_nan("");
        nrow = pad_row;
      }
    }
  };
  auto stage = [&](int buf) {
    if (wave == 0) {
      sm.xyz[buf][xyz_slot(tid)] = make_double4(nx, ny, nz, 0.0);
      if (!kPacked) sm.row[buf][tid] = nrow;
      else if ((tid & 7) == 0) sm.row[buf][tid >> 3] = nrow;
    }
  };

  // ---- weights of cell block `wave` for the block staged in `buf`, into
  // weight buffer `ab`.  A coarse test against the block's centre (lane l:
  // candidate l) marks the fragments (k-steps) that can hold a pair within
  // R; only those are evaluated exactly.  Unmarked fragments are never
  // multiplied.
  auto weights = [&](int buf, int ab) {
    const double4* s_xyz = sm.xyz[buf];
    uint32_t nzbits = 0;
    const double4 c = sm.ctr[wave];
    const double c2c = chord2(CellVec{c.x, c.y, c.z}, s_xyz[xyz_slot(lane)]);
    const uint64_t bm = __ballot(c2c <= c.w);
    const uint32_t lo = (uint32_t)bm, hi = (uint32_t)(bm >> 32);
    if (kForm == kF32) {
      float* A = sA32(ab);
      uint32_t pm = any_of_nibbles(lo) | (any_of_nibbles(hi) << 8);
      while (pm) {
        const int ks = __builtin_ctz(pm);
        pm &= pm - 1u;
        const double4 sv = s_xyz[xyz_slot(4 * ks + (lane >> 4))];
        const double c2 = chord2(cell, sv);
        float wf = 0.f;
        if (c2 <= a.c2R) wf = weight(c2, sv);
        wsum += (double)wf;
        A[(wave * kNS + ks) * 64 + lane] = wf;
        if (__ballot(wf != 0.f)) nzbits |= 1u << ks;
      }
    } else {
      uint4* A16 = sA16(ab);
      uint2* A8 = sA8(ab);
      // bit 4 s + j: 8-candidate group j of k-step s
      const uint32_t gm = any_of_bytes(lo) | (any_of_bytes(hi) << 4);
      uint32_t pm = ((gm & 15u) ? 1u : 0u) | ((gm >> 4) ? 2u : 0u);
      const int grp = lane >> 4;
      while (pm) {
        const int ks = __builtin_ctz(pm);
        pm &= pm - 1u;
        // codes packed as they are made: 16-bit forms two per word, FP8 four
        uint32_t hw[4] = {0u, 0u, 0u, 0u}, lw[4] = {0u, 0u, 0u, 0u};
        if ((gm >> (4 * ks + grp)) & 1u) {
          const int k0 = kK * ks + 8 * grp;
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const double4 sv = s_xyz[xyz_slot(k0 + t)];
            const double c2 = chord2(cell, sv);
            uint32_t h = 0u, l = 0u;
            if (c2 <= a.c2R) {
              const float wf = weight(c2, sv);
              h = enc_w<kForm>(wf);
              double eff = (double)dec_w<kForm>(h);
              if (kForm == kBF16Split) {
                l = f32_to_bf16(wf - dec_w<kForm>(h));
                eff += (double)bf16_to_f32(l);
              } else if (kForm == kFP8Split) {
                l = f32_to_e4m3_cvt(wf * kW8Scale - dec_w<kForm>(h));
                eff += (double)e4m3_cvt_to_f32(l);
              }
              wsum += (double)wf;
              wtsum += eff;
            }
            if (is_fp8(kForm)) {
              hw[t >> 2] |= h << (8 * (t & 3));
              if (kForm == kFP8Split) lw[t >> 2] |= l << (8 * (t & 3));
            } else {
              hw[t >> 1] |= h << (16 * (t & 1));
              if (kForm == kBF16Split) lw[t >> 1] |= l << (16 * (t & 1));
            }
          }
        }
        uint32_t any;
        const int slot = (wave * kNS + ks) * 64 + lane;
        const int slot_lo = 4 * kNS * 64 + slot;
        if (is_fp8(kForm)) {
          A8[slot] = make_uint2(hw[0], hw[1]);
          any = hw[0] | hw[1];
          if (kForm == kFP8Split) {
            A8[slot_lo] = make_uint2(lw[0], lw[1]);
            any |= lw[0] | lw[1];
          }
        } else {
          A16[slot] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
          any = hw[0] | hw[1] | hw[2] | hw[3];
          if (kForm == kBF16Split) {
            A16[slot_lo] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
            any |= lw[0] | lw[1] | lw[2] | lw[3];
          }
        }
        if (__ballot(any != 0u)) nzbits |= 1u << ks;
      }
    }
    if (lane == 0) sm.nz[ab][wave] = nzbits;
  };

  // ---- pipeline prologue: blocks 0 and 1 staged, block 2 in flight, the
  // weights of block 0 computed
  const uint32_t nblk = (total + kKB - 1) / kKB;
  if (nblk > 0) {
    fetch(0);
    stage(0);
  }
  if (nblk > 1) {
    fetch(kKB);
    stage(1);
  }
  if (kAhead && nblk > 2) fetch(2 * kKB);
  __syncthreads();
  if (nblk > 0) weights(0, 0);
  __syncthreads();

  // B operands: a block's first loads are issued at its top, so that they
  // are in flight while the next block's weights are computed.  (Carrying
  // them across the barrier, issued once the previous block's products had
  // read their registers, measured slower: the registers then stay live
  // through the weights.)
  using BT = typename PackedB<kForm>::T;
  constexpr int kNJ = kPacked ? 4 * kQW : 1;
  constexpr int kNSP = kPacked ? kNS : 1;
  // plan-ordered: the k-steps loaded at the block's top -- all of them,
  // except in the wide-support kernels of 512-channel slabs, whose
  // registers take only the first (the others are loaded once the previous
  // k-step's products are issued)
  constexpr int kEarly = (kQW == 1 || kForm == kFP8S || !kWide) ? kNSP : 1;
  BT bq[kNSP][kNJ];
  BT bql[kNSP][kNJ];
  // Plan-ordered planes hold Cp = C rounded up to 16 channels, so a
  // 16-channel tile is read whole; a tile past Cp reads the last tile
  // instead (a uniform clamp: its products only reach channels >= C, which
  // are not stored).
  auto load_b = [&](const uint32_t* rows, int ks) {
    const int64_t Cp = (C + 15) & ~int64_t(15);
    const int64_t at = (int64_t)rows[4 * ks + (lane >> 4)] * Cp + (lane & 15);
    const BT* hi = (const BT*)a.spec + at;
    const BT* lo = (const BT*)a.spec_lo + at;
#pragma unroll
    for (int j = 0; j < kNJ; ++j) {
      const int64_t cj = min<int64_t>(c_w + 16 * j, Cp - 16);
      bq[ks][j] = hi[cj];
      if (is_split(kForm)) bql[ks][j] = lo[cj];
    }
  };
  // input-order 16-bit and FP8 spectra: the first k-step's raw row pieces
  // are loaded at the block's top as well (repacked where they are used)
  constexpr bool kEarlyRaw = !kPacked && kVec && (kForm == kBF16 || kForm == kF16S ||
                                                  kForm == kFP8S);
  // input-order FP8 hi+lo: both planes' pieces one k-step ahead (not in the
  // general-shape kernels, whose registers would spill)
  constexpr bool kSplitAhead = !kPacked && kVec && kForm == kFP8Split && !kGen && (!kWide || kQW == 1);
  // the later k-steps' pieces too, one k-step ahead -- except in the
  // wide-support kernels of 512-channel slabs, whose registers would spill
  constexpr bool kRawAhead = (kEarlyRaw && (!kWide || kQW == 1)) || kSplitAhead;
  uint2 e16[(kEarlyRaw && !is_fp8(kForm)) ? kQW : 1][8];
  uint32_t e8[((kEarlyRaw && is_fp8(kForm)) || kSplitAhead) ? kQW : 1][8];
  uint32_t e8l[kSplitAhead ? kQW : 1][8];
  auto load_raw_h = [&](const uint32_t* rows, int ks, int h) {
    {
      const int64_t ch = my_ch + 64 * h;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int64_t row = rows[kK * ks + 8 * (lane >> 4) + t];
        if constexpr (is_fp8(kForm)) {
          // 4-byte pieces: unconditional (clamped) loads measured faster
          const bool ok = ch + 3 < C;
          e8[h][t] = *(const uint32_t*)((const uint8_t*)a.spec + row * C + (ok ? ch : 0));
          if constexpr (kSplitAhead)
            e8l[h][t] = *(const uint32_t*)((const uint8_t*)a.spec_lo + row * C + (ok ? ch : 0));
        } else {
          if constexpr (kRawAhead) {
            e16[h][t] = *(const uint2*)((const uint16_t*)a.spec + row * C + ((ch + 3 < C) ? ch : 0));
          } else {
            const uint16_t* src = (const uint16_t*)a.spec + row * C + ch;
            e16[h][t] = (ch + 3 < C) ? *(const uint2*)src : make_uint2(0u, 0u);
          }
        }
      }
    }
  };
  auto load_raw = [&](const uint32_t* rows) {
#pragma unroll
    for (int h = 0; h < kQW; ++h) load_raw_h(rows, 0, h);
  };
  // BF16 and FP16 x scale in 512-channel slabs (narrow support): a lane's
  // eight consecutive channels of a row in one 16-byte load, so that a
  // k-step takes eight loads per lane instead of sixteen.  The launchers
  // take these kernels only for rows that can be read eight elements at a
  // time (C a multiple of 8, spectra aligned to 8 elements); with C % 8 == 0
  // a lane's eight channels are all in the row or all past it.
  constexpr bool kW16 = kRawAhead && kQW == 2 && !is_fp8(kForm);
  // FP8 x scale the same way, eight channels in one 8-byte load (FP8 x scale
  // 20.3 -> 18.4 ms on the drift scan, same results bit for bit)
  constexpr bool kW8 = kRawAhead && kQW == 2 && kForm == kFP8S;
  const int64_t my_ch8 = c_w + 8 * (lane & 15);
  uint4 w16[kW16 ? 8 : 1];
  uint2 w8[kW8 ? 8 : 1];
  auto load_w8 = [&](const uint32_t* rows, int ks, int t) {
    const bool ok = my_ch8 < C;
    const int64_t row = rows[kK * ks + 8 * (lane >> 4) + t];
    w8[t] = *(const uint2*)((const uint8_t*)a.spec + row * C + (ok ? my_ch8 : 0));
  };
  // The loads of the kernels that load a k-step ahead are unconditional and
  // keep what they read: a select of zero for the lanes past the last
  // channel made the compiler branch around the load, and after such a
  // branch it waits for every outstanding load, the next k-step's included
  // (BF16 and FP16 x scale 23.8 -> 21.2 ms on the drift scan).  Such a lane
  // reads its row's first channels instead; their products only reach
  // accumulators of channels >= C, which are never stored.
  auto load_w = [&](const uint32_t* rows, int ks, int t) {
    const bool ok = my_ch8 < C;
    const int64_t row = rows[kK * ks + 8 * (lane >> 4) + t];
    w16[t] = *(const uint4*)((const uint16_t*)a.spec + row * C + (ok ? my_ch8 : 0));
  };
  // FP32: a ring of kDepth k-steps' rows in flight.  The row loads are
  // issued unconditionally (an index past the last channel is clamped into
  // the row; rows read one element at a time replace the value after the
  // load, rows read four at a time keep it): a load under a divergent
  // branch makes the compiler wait for every outstanding load before its
  // value is used, which serialised the ring (66.3 -> 60.5 ms on the
  // 9.12M x 1024 drift scan with this and the A operands read a k-step ahead).
  constexpr int kDepth = kWide ? 4 : 6;
  floatx4 bb[kForm == kF32 ? kDepth : 1][kQW];
  auto load = [&](const uint32_t* rows, int ks, floatx4* dst) {
    const float* spec = (const float*)a.spec;
    const int64_t row = rows[4 * ks + (lane >> 4)];
#pragma unroll
    for (int h = 0; h < kQW; ++h) {
      const int64_t ch = my_ch + 64 * h;
      const float* rp = spec + row * C;
      if (kVec) {
        const bool ok = ch + 3 < C;
        // a lane past the last channel keeps what it reads (the row's first
        // channels): those products only reach accumulators that are never
        // stored, and the select that zeroed them cost 60.3 -> 58.9 ms on
        // the drift scan
        dst[h] = *(const floatx4*)(rp + (ok ? ch : 0));
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = ch + e < C;
          const float v = rp[ok ? ch + e : 0];
          dst[h][e] = ok ? v : 0.f;
        }
      }
    }
  };

  for (uint32_t b = 0; b < nblk; ++b) {
    const int sb = (int)(b % 3u), ab = (int)(b & 1u);
    const uint32_t* s_row = sm.row[sb];                 // rows (or groups) of block b
    const bool more = b + 1 < nblk;
    if constexpr (kPacked) {
#pragma unroll
      for (int ks = 0; ks < kEarly; ++ks) load_b(s_row, ks);
    }
    if constexpr (kW16) {
#pragma unroll
      for (int t = 0; t < 8; ++t) load_w(s_row, 0, t);
    } else if constexpr (kW8) {
#pragma unroll
      for (int t = 0; t < 8; ++t) load_w8(s_row, 0, t);
    } else if constexpr (kEarlyRaw || kSplitAhead) {
      load_raw(s_row);
    }
    if constexpr (kForm == kF32) {
#pragma unroll
      for (int d = 0; d < kDepth; ++d) load(s_row, d, bb[d]);
    }

    // the next block's weights, while this block's loads are in flight
    if (more) weights((int)((b + 1u) % 3u), ab ^ 1);

    // ---- contraction over block b
    const uint32_t nzc[4] = {sm.nz[ab][0], sm.nz[ab][1], sm.nz[ab][2], sm.nz[ab][3]};
    if constexpr (kForm == kF32) {
      const float* A = sA32(ab);
      // the four cell blocks' A values of a k-step are read together, one
      // k-step ahead, so that no product waits on an LDS read
      float avn[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) avn[cb] = A[cb * kNS * 64 + lane];
#pragma unroll
      for (int ks = 0; ks < kNS; ++ks) {
        float avk[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) avk[cb] = avn[cb];
        if (ks + 1 < kNS) {
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) avn[cb] = A[(cb * kNS + ks + 1) * 64 + lane];
        }
        floatx4 cb_b[kQW];
        floatx4 cb_m[kMask ? kQW : 1];
#pragma unroll
        for (int h = 0; h < kQW; ++h) {
          cb_b[h] = bb[ks % kDepth][h];
          if constexpr (kMask) {
            // flags: a non-finite value becomes 0 in the product and 0 in
            // the channel's weight operand
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const bool fin = (__float_as_uint(cb_b[h][e]) & 0x7F800000u) != 0x7F800000u;
              cb_m[h][e] = fin ? 1.f : 0.f;
              cb_b[h][e] = fin ? cb_b[h][e] : 0.f;
            }
          }
        }
        if (ks + kDepth < kNS) load(s_row, ks + kDepth, bb[ks % kDepth]);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          if ((nzc[cb] >> ks) & 1u) {
            const float av = avk[cb];
#pragma unroll
            for (int h = 0; h < kQW; ++h) {
              if (h >= hlive) continue;
              acc[cb][4 * h + 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, cb_b[h].x, acc[cb][4 * h + 0], 0, 0, 0);
              acc[cb][4 * h + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, cb_b[h].y, acc[cb][4 * h + 1], 0, 0, 0);
              acc[cb][4 * h + 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, cb_b[h].z, acc[cb][4 * h + 2], 0, 0, 0);
              acc[cb][4 * h + 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, cb_b[h].w, acc[cb][4 * h + 3], 0, 0, 0);
              if constexpr (kMask) {
                accw[cb][4 * h + 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, cb_m[h].x, accw[cb][4 * h + 0], 0, 0, 0);
                accw[cb][4 * h + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, cb_m[h].y, accw[cb][4 * h + 1], 0, 0, 0);
                accw[cb][4 * h + 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, cb_m[h].z, accw[cb][4 * h + 2], 0, 0, 0);
                accw[cb][4 * h + 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, cb_m[h].w, accw[cb][4 * h + 3], 0, 0, 0);
              }
            }
          }
        }
      }
    } else if constexpr (kPacked) {
      const uint4* A16 = sA16(ab);
      const uint2* A8 = sA8(ab);
#pragma unroll
      for (int ks = 0; ks < kNS; ++ks) {
        // the k-steps not loaded early are loaded once the previous k-step's
        // products are issued (registers); the scheduler may not merge them
        __builtin_amdgcn_sched_barrier(0);
        if (ks >= kEarly) load_b(s_row, ks);
        // the four cell blocks' A operands of the k-step, read together
        uint4 a16[is_fp8(kForm) ? 1 : 4];
        uint2 a8[is_fp8(kForm) ? 4 : 1];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          if constexpr (is_fp8(kForm)) a8[cb] = A8[(cb * kNS + ks) * 64 + lane];
          else a16[cb] = A16[(cb * kNS + ks) * 64 + lane];
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          if (!((nzc[cb] >> ks) & 1u)) continue;
          if constexpr (is_fp8(kForm)) {
            const uint2 av = a8[cb];
            const long Aop = (long)(((uint64_t)av.y << 32) | av.x);
            long Al = 0;
            if (kForm == kFP8Split) {
              const uint2 al = A8[(4 * kNS + cb * kNS + ks) * 64 + lane];
              Al = (long)(((uint64_t)al.y << 32) | al.x);
            }
#pragma unroll
            for (int j = 0; j < kNJ; ++j) {
              floatx4& c = acc[cb][j];
              const long B = (long)(((uint64_t)bq[ks][j].y << 32) | bq[ks][j].x);
              c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(Aop, B, c, 0, 0, 0);
              if (kForm == kFP8Split) {
                const long Bl = (long)(((uint64_t)bql[ks][j].y << 32) | bql[ks][j].x);
                c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(Aop, Bl, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(Al, B, c, 0, 0, 0);
              }
            }
          } else {
            const uint4 av = a16[is_fp8(kForm) ? 0 : cb];
            uint4 al = make_uint4(0u, 0u, 0u, 0u);
            if (kForm == kBF16Split) al = A16[(4 * kNS + cb * kNS + ks) * 64 + lane];
#pragma unroll
            for (int j = 0; j < kNJ; ++j) {
              floatx4& c = acc[cb][j];
              if (kForm == kF16S) {
                c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(halfx8, av),
                                                          __builtin_bit_cast(halfx8, bq[ks][j]),
                                                          c, 0, 0, 0);
              } else {
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                           __builtin_bit_cast(bf16x8, bq[ks][j]),
                                                           c, 0, 0, 0);
                if (kForm == kBF16Split) {
                  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                             __builtin_bit_cast(bf16x8, bql[ks][j]),
                                                             c, 0, 0, 0);
                  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al),
                                                             __builtin_bit_cast(bf16x8, bq[ks][j]),
                                                             c, 0, 0, 0);
                }
              }
            }
          }
        }
      }
    } else if constexpr (kW16) {
      // the eight rows' pieces are transposed into the B operands of the
      // eight channels two rows at a time, and those two rows' pieces of the
      // next k-step loaded into the freed registers (all unconditional); the
      // products of the k-step follow.  (Drift scan, 9.12M x 1024: FP16 x
      // scale 29.6 -> 22.9 ms, BF16 30.0 -> 23.5 ms, same results bit for
      // bit; loading all eight rows after the transposition spilled
      // registers, and loading them at the k-step was slower.)
      const uint4* A16 = sA16(ab);
      const uint32_t any = nzc[0] | nzc[1] | nzc[2] | nzc[3];
#pragma unroll
      for (int ks = 0; ks < kNS; ++ks) {
        const bool act = (any >> ks) & 1u;
        uint32_t fb[8][4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const uint4 d0 = w16[2 * m], d1 = w16[2 * m + 1];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const uint2 h0 = q < 4 ? make_uint2(d0.x, d0.y) : make_uint2(d0.z, d0.w);
            const uint2 h1 = q < 4 ? make_uint2(d1.x, d1.y) : make_uint2(d1.z, d1.w);
            fb[q][m] = elem16(h0, q & 3) | (elem16(h1, q & 3) << 16);
          }
          if (ks + 1 < kNS) {
            load_w(s_row, ks + 1, 2 * m);
            load_w(s_row, ks + 1, 2 * m + 1);
          }
        }
        if (!act) continue;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          if (!((nzc[cb] >> ks) & 1u)) continue;
          const uint4 av = A16[(cb * kNS + ks) * 64 + lane];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            floatx4& c = acc[cb][q];
            const uint4 bv = make_uint4(fb[q][0], fb[q][1], fb[q][2], fb[q][3]);
            if constexpr (kForm == kF16S)
              c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(halfx8, av),
                                                        __builtin_bit_cast(halfx8, bv), c, 0, 0, 0);
            else
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                         __builtin_bit_cast(bf16x8, bv), c, 0, 0, 0);
          }
        }
      }
    } else if constexpr (kW8) {
      const uint2* A8 = sA8(ab);
      const uint32_t any = nzc[0] | nzc[1] | nzc[2] | nzc[3];
#pragma unroll
      for (int ks = 0; ks < kNS; ++ks) {
        const bool act = (any >> ks) & 1u;
        uint32_t fb[8][2];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int sh = 8 * (q & 3);
          uint32_t v0 = 0u, v1 = 0u;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            v0 |= (((q < 4 ? w8[t].x : w8[t].y) >> sh) & 0xFFu) << (8 * t);
            v1 |= (((q < 4 ? w8[4 + t].x : w8[4 + t].y) >> sh) & 0xFFu) << (8 * t);
          }
          fb[q][0] = v0;
          fb[q][1] = v1;
        }
        if (ks + 1 < kNS) {
#pragma unroll
          for (int t = 0; t < 8; ++t) load_w8(s_row, ks + 1, t);
        }
        if (!act) continue;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          if (!((nzc[cb] >> ks) & 1u)) continue;
          const uint2 av = A8[(cb * kNS + ks) * 64 + lane];
          const long Aop = (long)(((uint64_t)av.y << 32) | av.x);
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const long B = (long)(((uint64_t)fb[q][1] << 32) | fb[q][0]);
            acc[cb][q] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(Aop, B, acc[cb][q], 0, 0, 0);
          }
        }
      }
    } else if constexpr (kRawAhead) {
      // input-order rows read four channels at a time (the 256-channel
      // BF16, FP16 x scale and FP8 x scale kernels, and FP8 hi+lo): the raw
      // row pieces of k-step ks + 1 are loaded into the registers that held
      // those of k-step ks once these are repacked into B operands, so that
      // a k-step's loads are in flight while the previous k-step's products
      // are issued (k-step 0's are loaded at the block's top).  The loads are
      // unconditional: a load under a branch makes the compiler wait for all
      // outstanding loads.  (Drift scan, 9.12M x 1024: FP8 hi+lo 33.7 -> 32.4
      // ms, and FP8 x scale 22.2 -> 20.4 ms before its 512-channel kernel
      // read eight channels per lane; same results bit for bit.)
      const uint4* A16 = sA16(ab);
      const uint2* A8 = sA8(ab);
      const uint32_t any = nzc[0] | nzc[1] | nzc[2] | nzc[3];
#pragma unroll
      for (int ks = 0; ks < kNS; ++ks) {
        const bool act = (any >> ks) & 1u;
#pragma unroll
        for (int h = 0; h < kQW; ++h) {
          uint32_t fb[4][4];
          uint32_t fbl[kSplitAhead ? 4 : 1][2];
          if constexpr (is_fp8(kForm)) {
            const uint32_t* d = e8[h];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              fb[q][0] = ((d[0] >> (8 * q)) & 0xFFu) | (((d[1] >> (8 * q)) & 0xFFu) << 8) |
                         (((d[2] >> (8 * q)) & 0xFFu) << 16) | (((d[3] >> (8 * q)) & 0xFFu) << 24);
              fb[q][1] = ((d[4] >> (8 * q)) & 0xFFu) | (((d[5] >> (8 * q)) & 0xFFu) << 8) |
                         (((d[6] >> (8 * q)) & 0xFFu) << 16) | (((d[7] >> (8 * q)) & 0xFFu) << 24);
            }
            if constexpr (kSplitAhead) {
              const uint32_t* dl = e8l[h];
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                fbl[q][0] = ((dl[0] >> (8 * q)) & 0xFFu) | (((dl[1] >> (8 * q)) & 0xFFu) << 8) |
                            (((dl[2] >> (8 * q)) & 0xFFu) << 16) | (((dl[3] >> (8 * q)) & 0xFFu) << 24);
                fbl[q][1] = ((dl[4] >> (8 * q)) & 0xFFu) | (((dl[5] >> (8 * q)) & 0xFFu) << 8) |
                            (((dl[6] >> (8 * q)) & 0xFFu) << 16) | (((dl[7] >> (8 * q)) & 0xFFu) << 24);
              }
            }
          } else {
            const uint2* d = e16[kEarlyRaw ? h : 0];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int m = 0; m < 4; ++m)
                fb[q][m] = elem16(d[2 * m], q) | (elem16(d[2 * m + 1], q) << 16);
          }
          if (ks + 1 < kNS) load_raw_h(s_row, ks + 1, h);
          if (!act) continue;
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            if (!((nzc[cb] >> ks) & 1u)) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              floatx4& c = acc[cb][4 * h + q];
              if constexpr (is_fp8(kForm)) {
                const uint2 av = A8[(cb * kNS + ks) * 64 + lane];
                const long Aop = (long)(((uint64_t)av.y << 32) | av.x);
                const long B = (long)(((uint64_t)fb[q][1] << 32) | fb[q][0]);
                c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(Aop, B, c, 0, 0, 0);
                if constexpr (kSplitAhead) {
                  // W_hi S_lo + W_lo S_hi (the W_lo S_lo term is below the budget)
                  const uint2 al = A8[(4 * kNS + cb * kNS + ks) * 64 + lane];
                  const long Al = (long)(((uint64_t)al.y << 32) | al.x);
                  const long Bl = (long)(((uint64_t)fbl[q][1] << 32) | fbl[q][0]);
                  c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(Aop, Bl, c, 0, 0, 0);
                  c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(Al, B, c, 0, 0, 0);
                }
              } else {
                const uint4 av = A16[(cb * kNS + ks) * 64 + lane];
                const uint4 bv = make_uint4(fb[q][0], fb[q][1], fb[q][2], fb[q][3]);
                if constexpr (kForm == kF16S)
                  c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(halfx8, av),
                                                            __builtin_bit_cast(halfx8, bv), c, 0, 0, 0);
                else
                  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                             __builtin_bit_cast(bf16x8, bv), c, 0, 0, 0);
              }
            }
          }
        }
      }
    } else {
      const uint4* A16 = sA16(ab);
      const uint2* A8 = sA8(ab);
#pragma unroll
      for (int ks = 0; ks < kNS; ++ks) {
        const uint32_t any = nzc[0] | nzc[1] | nzc[2] | nzc[3];
        if (!((any >> ks) & 1u)) continue;
        // one 64-channel group at a time: B fragments of 8 candidates (rows)
        // x 4 channels, then the MFMAs of every non-zero cell block
#pragma unroll
        for (int h = 0; h < kQW; ++h) {
          const int64_t ch = my_ch + 64 * h;
          uint32_t fb[4][4];   // [q][dword] (16-bit) or [q][0..1] (FP8)
          uint32_t fbl[4][4];  // low plane (split form)
          if (is_fp8(kForm)) {
#pragma unroll
            for (int plane = 0; plane < (kForm == kFP8Split ? 2 : 1); ++plane) {
              const uint8_t* spec = (const uint8_t*)(plane ? a.spec_lo : a.spec);
              uint32_t d[8];
#pragma unroll
              for (int t = 0; t < 8; ++t) {
                const int64_t row = s_row[kK * ks + 8 * (lane >> 4) + t];
                const uint8_t* rp = spec + row * C;
                if (kEarlyRaw && ks == 0) {
                  d[t] = e8[kEarlyRaw ? h : 0][t];
                } else if (kVec) {
                  const bool ok = ch + 3 < C;
                  const uint32_t v = *(const uint32_t*)(rp + (ok ? ch : 0));
                  d[t] = ok ? v : 0u;
                } else {
                  d[t] = 0u;
#pragma unroll
                  for (int e = 0; e < 4; ++e) {
                    const bool ok = ch + e < C;
                    const uint32_t v = rp[ok ? ch + e : 0];
                    d[t] |= (ok ? v : 0u) << (8 * e);
                  }
                }
              }
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const uint32_t v0 = ((d[0] >> (8 * q)) & 0xFFu) | (((d[1] >> (8 * q)) & 0xFFu) << 8) |
                                    (((d[2] >> (8 * q)) & 0xFFu) << 16) |
                                    (((d[3] >> (8 * q)) & 0xFFu) << 24);
                const uint32_t v1 = ((d[4] >> (8 * q)) & 0xFFu) | (((d[5] >> (8 * q)) & 0xFFu) << 8) |
                                    (((d[6] >> (8 * q)) & 0xFFu) << 16) |
                                    (((d[7] >> (8 * q)) & 0xFFu) << 24);
                if (plane) {
                  fbl[q][0] = v0;
                  fbl[q][1] = v1;
                } else {
                  fb[q][0] = v0;
                  fb[q][1] = v1;
                }
              }
            }
          } else {
#pragma unroll
            for (int plane = 0; plane < (kForm == kBF16Split ? 2 : 1); ++plane) {
              const uint16_t* spec = (const uint16_t*)(plane ? a.spec_lo : a.spec);
              uint2 d[8];
#pragma unroll
              for (int t = 0; t < 8; ++t) {
                const int64_t row = s_row[kK * ks + 8 * (lane >> 4) + t];
                const uint16_t* rp = spec + row * C;
                if (kEarlyRaw && ks == 0 && plane == 0) {
                  d[t] = e16[kEarlyRaw ? h : 0][t];
                } else if (kVec && kQW == 1) {
                  // unconditional, keeping what a lane past the last channel
                  // reads (those products are never stored): without the
                  // branch around each load the BF16 hi+lo gather took 43.2
                  // instead of 48.1 ms on the drift scan; the wide-support
                  // 512-channel kernels that come here would spill
                  d[t] = *(const uint2*)(rp + ((ch + 3 < C) ? ch : 0));
                } else if (kVec) {
                  d[t] = (ch + 3 < C) ? *(const uint2*)(rp + ch) : make_uint2(0u, 0u);
                } else {
                  uint32_t e[4];
#pragma unroll
                  for (int k = 0; k < 4; ++k) {
                    const bool ok = ch + k < C;
                    const uint32_t v = rp[ok ? ch + k : 0];
                    e[k] = ok ? v : 0u;
                  }
                  d[t] = make_uint2(e[0] | (e[1] << 16), e[2] | (e[3] << 16));
                }
              }
#pragma unroll
              for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                  const uint32_t v = elem16(d[2 * m], q) | (elem16(d[2 * m + 1], q) << 16);
                  if (plane) fbl[q][m] = v; else fb[q][m] = v;
                }
            }
          }
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            if (!((nzc[cb] >> ks) & 1u)) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              floatx4& c = acc[cb][4 * h + q];
              if (is_fp8(kForm)) {
                const uint2 av = A8[(cb * kNS + ks) * 64 + lane];
                const long Aop = (long)(((uint64_t)av.y << 32) | av.x);
                const long B = (long)(((uint64_t)fb[q][1] << 32) | fb[q][0]);
                c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(Aop, B, c, 0, 0, 0);
                if (kForm == kFP8Split) {
                  // W_hi S_lo + W_lo S_hi (the W_lo S_lo term is below the budget)
                  const uint2 al = A8[(4 * kNS + cb * kNS + ks) * 64 + lane];
                  const long Al = (long)(((uint64_t)al.y << 32) | al.x);
                  const long Bl = (long)(((uint64_t)fbl[q][1] << 32) | fbl[q][0]);
                  c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(Aop, Bl, c, 0, 0, 0);
                  c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(Al, B, c, 0, 0, 0);
                }
              } else {
                const uint4 av = A16[(cb * kNS + ks) * 64 + lane];
                const uint4 bv = make_uint4(fb[q][0], fb[q][1], fb[q][2], fb[q][3]);
                if (kForm == kF16S) {
                  c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(halfx8, av),
                                                            __builtin_bit_cast(halfx8, bv), c, 0, 0, 0);
                } else {
                  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                             __builtin_bit_cast(bf16x8, bv), c, 0, 0, 0);
                  if (kForm == kBF16Split) {
                    const uint4 al = A16[(4 * kNS + cb * kNS + ks) * 64 + lane];
                    const uint4 bl = make_uint4(fbl[q][0], fbl[q][1], fbl[q][2], fbl[q][3]);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                               __builtin_bit_cast(bf16x8, bl), c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al),
                                                               __builtin_bit_cast(bf16x8, bv), c, 0, 0, 0);
                  }
                }
              }
            }
          }
        }
      }
    }

    // wave 0 stages block b + 2 (loaded during the previous block) and
    // starts the loads of block b + 3
    if (b + 2 < nblk) {
      if (!kAhead) fetch((b + 2u) * kKB);
      stage((int)((b + 2u) % 3u));
      if (kAhead && b + 3 < nblk) fetch((b + 3u) * kKB);
    }
    __syncthreads();
  }

  // weight sums of cell block `wave`: reduce the four lanes sharing a cell
  if (kForm == kF32) wtsum = wsum;  // the FP32 form multiplies the weights as they are
  wsum += __shfl_xor(wsum, 16);
  wsum += __shfl_xor(wsum, 32);
  wtsum += __shfl_xor(wtsum, 16);
  wtsum += __shfl_xor(wtsum, 32);
  if (lane < 16) {
    s_Wt[wave * 16 + lane] = wtsum;
    if (!kMask && a.wmap && slab == 0 && my_x < g.nx && my_y < g.ny)
      a.wmap[(int64_t)my_y * g.nx + my_x] = (float)wsum;
  }
  __syncthreads();

  // A lane's four cells r = 0..3 of a cell block are consecutive in x: one
  // 16-byte store per channel where rows and the cube allow it (a 4-byte
  // store costs a whole 32-byte write in HBM), else one store per cell.
  const float qnan = __builtin_nanf("");
  const bool st4 = (g.nx % 4 == 0) && (((uintptr_t)a.cube & 15u) == 0);
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int y = ty * kTileY + (cb >> 1) * 4 + (lane >> 4);
    const int x0 = tx * kTileX + (cb & 1) * 4;
    if (y >= g.ny || x0 >= g.nx) continue;
    float inv[4];
    bool has[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double wt = s_Wt[cb * 16 + 4 * (lane >> 4) + r];
      has[r] = wt != 0.0;
      inv[r] = has[r] ? (float)(1.0 / wt) : 0.f;
    }
    const int64_t row0 = (int64_t)y * g.nx + x0;
    const bool full = st4 && x0 + 3 < g.nx;
#pragma unroll
    for (int h = 0; h < kQW; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // accumulator 4 h + q: channel 4 (lane % 16) + 64 h + q, or for the
        // plan-ordered spectra lane % 16 + 16 (4 h + q), or for eight
        // channels per lane 8 (lane % 16) + 4 h + q
        const int64_t ch = kPacked ? c_w + 16 * (4 * h + q) + (lane & 15)
                           : (kW16 || kW8) ? my_ch8 + 4 * h + q
                                   : my_ch + 64 * h + q;
        if (ch >= C) continue;
        const float sc = (kForm == kF16S || is_fp8(kForm)) ? a.scale[ch] : 1.f;
        float v[4], wc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if constexpr (kMask) {
            // the channel's own weight sum (FP32 accumulation of FP32 weights)
            wc[r] = accw[cb][4 * h + q][r];
            v[r] = (wc[r] != 0.f) ? acc[cb][4 * h + q][r] / wc[r] : qnan;
          } else {
            float t = acc[cb][4 * h + q][r] * inv[r];
            if (kForm == kF16S || is_fp8(kForm)) t *= sc;
            v[r] = has[r] ? t : qnan;
          }
        }
        float* dst = a.cube + ch * G + row0;
        float* wdst = kMask ? a.wcube + ch * G + row0 : nullptr;
        if (full) {
          *(floatx4*)dst = floatx4{v[0], v[1], v[2], v[3]};
          if (kMask && wdst) *(floatx4*)wdst = floatx4{wc[0], wc[1], wc[2], wc[3]};
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (x0 + r < g.nx) {
              dst[r] = v[r];
              if (kMask && wdst) wdst[r] = wc[r];
            }
        }
      }
  }
}

// LDS of the few-channel gather in a batch (one wave per workgroup), carved
// from dynamic LDS of cells_batch_lds_bytes(maxr) bytes with maxr the largest
// range count of the batch's plans: small, so that many tiles are in flight
// on a CU -- most tiles of a sparse field hold a few candidates, and their
// time is the latency of the range, vector and value loads.
struct CellsLds {
  double4* xyz;       // [kKB]
  float (*spec)[8];   // [kKB][8]
  uint2* rng;         // [maxr]
  uint32_t* pre;      // [maxr + 1]
};
__host__ __device__ constexpr size_t cells_batch_lds_bytes(int maxr) {
  return sizeof(double4) * kKB + sizeof(float) * kKB * 8 + sizeof(uint2) * (size_t)maxr +
         sizeof(uint32_t) * ((size_t)maxr + 1);
}
__device__ inline CellsLds cells_lds(unsigned char* base, int maxr) {
  CellsLds L;
  L.xyz = (double4*)base;
  L.spec = (float (*)[8])(L.xyz + kKB);
  L.rng = (uint2*)(L.spec + kKB);
  L.pre = (uint32_t*)(L.rng + maxr);
  return L;
}

// Few channels (C <= kCM <= 8) for a 64-thread workgroup: one lane per cell
// of the 8 x 8 tile, candidates staged 64 at a time, weights and sums in
// FP64 (the per-plan k_gather_cells without the split of the candidates).
template <int kCM>
__device__ inline void gather_cells_tile_wave(const GatherArgs& a, int tile, const CellsLds& sm) {
  const int lane = threadIdx.x;
  const int tx = tile % a.ntx, ty = tile / a.ntx;
  const GridGeom& g = a.g;
  const int ix = tx * kTileX + (lane & 7), iy = ty * kTileY + (lane >> 3);
  const CellVec cell = cell_at(a.cells, g, ix, iy);
  const uint32_t total =
      stage_ranges(a.ranges + (int64_t)tile * a.maxr, a.nranges[tile], sm.rng, sm.pre);
  const int C = (int)a.C;
  const float* spec = (const float*)a.spec;
  double acc[kCM];
#pragma unroll
  for (int c = 0; c < kCM; ++c) acc[c] = 0.0;
  double wsum = 0.0;
  uint32_t cur = 0;
  for (uint32_t q0 = 0; q0 < total; q0 += kKB) {
    const uint32_t q = q0 + lane;
    if (q < total) {
      const uint32_t pos = cand_pos(q, sm.rng, sm.pre, &cur);
      sm.xyz[lane] = a.xyz[pos];
      const int64_t row = a.perm[pos];
#pragma unroll
      for (int c = 0; c < kCM; ++c) sm.spec[lane][c] = (c < C) ? spec[row * C + c] : 0.f;
    }
    __syncthreads();
    const int kmax = (int)min<uint32_t>(kKB, total - q0);
    for (int k = 0; k < kmax; ++k) {
      const double c2 = chord2(cell, sm.xyz[k]);
      if (c2 <= a.c2R) {
        const double w = pair_weight64(c2, a.kern.wscale);
        wsum += w;
#pragma unroll
        for (int c = 0; c < kCM; ++c) acc[c] += w * (double)sm.spec[k][c];
      }
    }
    __syncthreads();
  }
  if (ix >= g.nx || iy >= g.ny) return;
  const int64_t G = (int64_t)g.nx * g.ny;
  const int64_t cellidx = (int64_t)iy * g.nx + ix;
  if (a.wmap) a.wmap[cellidx] = (float)wsum;
#pragma unroll
  for (int c = 0; c < kCM; ++c)
    if (c < C) a.cube[c * G + cellidx] = (wsum != 0.0) ? (float)(acc[c] / wsum) : __builtin_nanf("");
}

// The few-channel gather of one tile, by channel count.
__device__ inline void gather_cells_tile(const GatherArgs& a, int tile, const CellsLds& sm) {
  if (a.C == 1) gather_cells_tile_wave<1>(a, tile, sm);
  else gather_cells_tile_wave<8>(a, tile, sm);
}

}  // namespace hcg
