// Data stage of the gridding library: Eq. (1) of HCGrid (Section 2.1) for
// every output cell and channel, gather-side (Section 2.2: each cell pulls
// the samples within its support, so no two workgroups write the same cell).
//
// Work decomposition: one workgroup (8 waves) per 16 x 16 tile of output
// cells and 256-channel slab.  The tile's candidate samples come from the
// plan's sorted-sample ranges and are staged in blocks of 64:
//   1. weights: FP64 chord distance between unit vectors of cell and sample,
//      exact support test (chord <= 2 sin(R/2), i.e. d <= R), FP64 exponent
//      of the Gaussian, evaluated with exp2f, rounded to the operand type of
//      the form; FP64 sums of the weights per cell;
//   2. accumulation: the block is a dense contraction
//      U[cells x channels] += Wt[cells x 64] . S[64 x channels] on the matrix
//      cores with FP32 accumulation -- FP32 operands (v_mfma_f32_16x16x4_f32)
//      or BF16 / FP16 / FP8 operands (16x16x32) -- skipping every 16-cell x
//      k-step sub-block whose weights are all zero; for a few FP32 channels
//      each thread owns one cell and accumulates in FP64;
//   3. epilogue: V = U / W~ (W~ the sum of the weights actually multiplied),
//      times the channel scale for the scaled forms, NaN where no sample is
//      within the support; the W map is the FP64 sum of the weights.
#include <cmath>
#include <vector>

#include "hcg_internal.h"

namespace hcg {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

constexpr int kKB = 64;          // candidates staged per block
constexpr int kCB = 16;          // 4 x 4 cell blocks per 16 x 16 tile
constexpr int kWGThreads = 512;  // 8 waves
constexpr int kSlab = 256;       // channels per workgroup (4 groups of 64)

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
struct CellVec {
  double x, y, z;
};

// Unit vector of cell (ix, iy); NaN outside the grid (never within R).
__device__ __forceinline__ CellVec cell_vec(const GridGeom& g, int ix, int iy) {
  CellVec c;
  if (ix >= g.nx || iy >= g.ny || ix < 0 || iy < 0) {
    c.x = c.y = c.z = __builtin_nan("");
    return c;
  }
  double sb, cb, sl, cl;
  sincos(cell_lat_deg(g, iy) * kDeg2Rad, &sb, &cb);
  sincos(cell_lon_deg(g, ix) * kDeg2Rad, &sl, &cl);
  c.x = cb * cl;
  c.y = cb * sl;
  c.z = sb;
  return c;
}

// Squared chord |u - v|^2 = 4 sin^2(d/2) between a cell and a sample.
__device__ __forceinline__ double chord2(const CellVec& c, const double4& v) {
  const double dx = v.x - c.x, dy = v.y - c.y, dz = v.z - c.z;
  return dx * dx + dy * dy + dz * dz;
}
__device__ __forceinline__ double chord2(const CellVec& c, const double2& xy, double z) {
  const double dx = xy.x - c.x, dy = xy.y - c.y, dz = z - c.z;
  return dx * dx + dy * dy + dz * dz;
}


// Weight of a pair inside the support.  d^2 = 4 asin^2(chord / 2)
// = 2 sum_n c2^n / (n^2 binom(2n, n)) = c2 (1 + c2/12 + c2^2/90 + c2^3/560
// + c2^4/3150 + c2^5/16632 + ...): for c2 < 1e-2 (d < 5.7 deg) six terms
// leave a relative error below 2e-17.  Wider supports (kWide) take the
// arcsine beyond that.  The exponent -d^2 log2(e) / (2 sigma^2) is formed
// in FP64 and evaluated with exp2f.
constexpr double kSeriesMax = 1e-2;

template <bool kWide>
__device__ __forceinline__ float pair_weight(double c2, double wscale) {
  double d2;
  if (!kWide || c2 < kSeriesMax) {
    d2 = c2 * (1.0 + c2 * (1.0 / 12.0 + c2 * (1.0 / 90.0 + c2 * (1.0 / 560.0 +
              c2 * (1.0 / 3150.0 + c2 * (1.0 / 16632.0))))));
  } else {
    const double d = 2.0 * asin(fmin(0.5 * sqrt(c2), 1.0));
    d2 = d * d;
  }
  return exp2f((float)(d2 * wscale));
}

// Loads the tile's candidate ranges into LDS with exclusive prefix sums;
// returns the total candidate count.  All threads of the block take part.
__device__ uint32_t stage_ranges(const uint2* __restrict__ ranges, uint32_t nr, uint2* s_rng,
                                 uint32_t* s_pre) {
  const int nt = blockDim.x;
  for (uint32_t r = threadIdx.x; r < nr; r += nt) s_rng[r] = ranges[r];
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t r = 0; r < nr; ++r) {
      s_pre[r] = acc;
      acc += s_rng[r].y - s_rng[r].x;
    }
    s_pre[nr] = acc;
  }
  __syncthreads();
  return s_pre[nr];
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
enum Form : int { kF32 = 0, kBF16 = 1, kBF16Split = 2, kF16S = 3, kFP8S = 4 };

template <int kForm>
struct FormTraits {
  static constexpr int kK = (kForm == kF32) ? 4 : 32;  // candidates per MFMA k-step
};

template <int kForm>
__device__ __forceinline__ uint32_t enc_w(float w) {
  if (kForm == kF16S) return f32_to_f16(w);
  if (kForm == kFP8S) return f32_to_e4m3(w);
  return f32_to_bf16(w);
}
template <int kForm>
__device__ __forceinline__ float dec_w(uint32_t c) {
  if (kForm == kF16S) return f16_to_f32(c);
  if (kForm == kFP8S) return e4m3_to_f32(c);
  return bf16_to_f32(c);
}

// the 16-bit element q (0..3) of an 8-byte load
__device__ __forceinline__ uint32_t elem16(uint2 d, int q) {
  const uint32_t w = (q < 2) ? d.x : d.y;
  return (q & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// LDS of one workgroup (shared by the per-plan kernels and the batch kernel).
// Staged candidate blocks are double-buffered (coordinates, A fragments) or
// triple-buffered (rows, read by the spectrum loads one block ahead).
struct GatherSmem {
  uint2 rng[kMaxRangesLimit];
  uint32_t pre[kMaxRangesLimit + 1];
  double2 xy[2][kKB];    // staged coordinates: x, y
  double2 zw[2][kKB];    // z, 0
  double4 ctr[kCB];      // cell-block centre (unit vector), coarse squared chord
  uint32_t row[3][kKB];
  uint32_t nzm[2][kCB];  // non-zero k-steps of each cell block
  // A fragments, per buffer: FP32 [16 cb][16 k-steps][64 lanes] float;
  // BF16 / FP16 [16 cb][2 k-steps][64] uint4 (+ the low plane of the split
  // form behind it); FP8 [16][2][64] uint2.  Also the staging area of the
  // few-channel path.
  uint4 A[2][kCB * 16 * 64 / 4];
  double Wt[kTileCells];
};
static_assert(sizeof(GatherSmem::A) >= 2 * 2 * 256 * sizeof(double4),
              "the few-channel path stages two parts of 16 KB in A");
static_assert(sizeof(GatherSmem) <= 160 * 1024, "LDS of one workgroup");

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

// ---------------------------------------------------------------------------
// Many channels: one (16 x 16 tile, 256-channel slab) on the matrix cores.
//
// The tile's 256 cells form sixteen 4 x 4 cell blocks (cb); a staged block of
// 64 candidates forms k-steps of 4 (FP32) or 32 (BF16 / FP16 / FP8)
// candidates.  An A fragment is one (cb, k-step): lane l of it holds cell
// l % 16 and candidate l / 16 (FP32) or candidates 8 (l / 16) .. +7.
//
// Weights: wave w owns cell blocks 2w and 2w + 1.  A coarse test first marks
// the fragments that can hold a pair within R: a candidate can only be within
// R of some cell of a block if it is within R + h of the block's centre (h:
// the block's largest centre-to-cell distance; triangle inequality).  Only
// those fragments are evaluated exactly (FP64 chord, exact support test,
// weight), lane by lane straight into the A layout; a fragment found all zero
// is dropped.  The fragment lists are wave-uniform.
// Contraction: wave w covers cell blocks 8 (w % 2) .. +7 and the 64 channels
// 64 (w / 2) .. +63 of the slab; lane l streams channels 4 (l % 16) .. +3
// (column j of MFMA q is channel 4 j + q of the group), skipping the
// fragments that are not marked.
// Output D[i][j]: lane l, register r holds cell 4 (l / 16) + r of the block.
//
// Software pipeline over the blocks, one barrier per block: while a wave runs
// the products of block b it evaluates its fragments of block b + 1 between
// the matrix instructions, and its spectrum loads run ahead across the block
// boundary; coordinates and rows of block b + 2 are staged meanwhile.
// ---------------------------------------------------------------------------
// kVec: 1 = rows read 4 elements at a time, 0 = one at a time, 2 = as a.vec
// says (FP32 only).  kWide: the support reaches c2 >= kSeriesMax.
template <int kForm, int kVec, bool kWide>
__device__ __forceinline__ void gather_tile(const GatherArgs& a, int tile, int slab,
                                            GatherSmem& sm) {
  constexpr int kK = FormTraits<kForm>::kK;
  constexpr int kNS = kKB / kK;  // k-steps per staged block
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tx = tile % a.ntx, ty = tile / a.ntx;
  const GridGeom& g = a.g;
  const int64_t C = a.C;
  const int64_t G = (int64_t)g.nx * g.ny;

  // weight role: cell blocks cbA = 2 wave, cbB = cbA + 1; lane l: cell l % 16
  const int li = lane & 15;
  const int cbA = 2 * wave, cbB = cbA + 1;
  auto cell_x = [&](int cb) { return tx * kTileX + (cb & 3) * 4 + (li & 3); };
  auto cell_y = [&](int cb) { return ty * kTileY + (cb >> 2) * 4 + (li >> 2); };
  const CellVec cellA = cell_vec(g, cell_x(cbA), cell_y(cbA));
  const CellVec cellB = cell_vec(g, cell_x(cbB), cell_y(cbB));
  // contraction role
  const int cg = wave & 1;
  const int64_t my_ch = (int64_t)slab * kSlab + (wave >> 1) * 64 + 4 * (lane & 15);
  const bool ch_ok = my_ch + 3 < C;  // the vector loads (C % 4 == 0 there)

  const uint32_t total =
      stage_ranges(a.ranges + (int64_t)tile * a.maxr, a.nranges[tile], sm.rng, sm.pre);
  const uint32_t nb = (total + kKB - 1) / kKB;

  floatx4 acc[8][4];
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[c][q] = floatx4{0.f, 0.f, 0.f, 0.f};
  // FP64 sums of the weights of this lane's cell in cbA / cbB (its share of
  // the candidates), as evaluated and as multiplied (rounded forms)
  double wsA = 0.0, wsB = 0.0, wtA = 0.0, wtB = 0.0;
  uint32_t cur = 0;

  // Coordinates and rows of block blk, read by wave 0 into registers
  // (stage_load: unconditional loads; past the last candidate the plan's
  // sentinel entry, NaN vector and row 0) and written to LDS after the
  // block's products (stage_store), so that the wait for them does not drain
  // the spectrum loads in flight.
  const bool stager = wave == 0;
  double4 st_v = make_double4(0.0, 0.0, 0.0, 0.0);
  uint32_t st_r = 0u;
  auto stage_load = [&](uint32_t blk) {
    if (stager) {
      const uint32_t q = blk * kKB + lane;
      const uint32_t pos = (q < total) ? cand_pos(q, sm.rng, sm.pre, &cur) : a.sentinel;
      st_v = a.xyz[pos];
      st_r = a.perm[pos];
    }
  };
  auto stage_store = [&](uint32_t blk, int rbuf) {
    if (stager) {
      sm.xy[blk & 1][lane] = make_double2(st_v.x, st_v.y);
      sm.zw[blk & 1][lane] = make_double2(st_v.z, st_v.w);
      sm.row[rbuf][lane] = st_r;
    }
  };

  // Cell-block centres and coarse thresholds (threads 0..255: block t / 16,
  // cell t % 16).  Cells outside the grid do not count; a block without
  // cells gets threshold -1 (never marked).
  if (tid < kTileCells) {
    const int cb = tid >> 4, i = tid & 15;
    const int x = tx * kTileX + (cb & 3) * 4 + (i & 3), y = ty * kTileY + (cb >> 2) * 4 + (i >> 2);
    const bool valid = x < g.nx && y < g.ny;
    const CellVec v = cell_vec(g, x, y);
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
    const double ang = R + h;
    const double sh = sin(0.5 * fmin(ang, kPi));
    double thr = 4.0 * sh * sh * (1.0 + 1e-9) + 1e-15;  // slack for rounding
    if (!(nrm > 0.0)) thr = -1.0;
    if (i == 0) sm.ctr[cb] = make_double4(c.x, c.y, c.z, thr);
  }

  // Coarse marks of the wave's two blocks for the candidates in buffer buf.
  // Lane l tests candidates l % 32 and l % 32 + 32 against block cbA (l < 32)
  // or cbB.  F32: bit s of m = k-step s; other forms: bit s of m = k-step s,
  // bit 4 s + j of gm = its 8-candidate group j.
  auto coarse = [&](int buf, uint32_t& mA, uint32_t& mB, uint32_t& gA, uint32_t& gB) {
    const double4 c = sm.ctr[cbA + (lane >> 5)];
    const CellVec cc{c.x, c.y, c.z};
    const int j = lane & 31;
    const double c2a = chord2(cc, sm.xy[buf][j], sm.zw[buf][j].x);
    const double c2b = chord2(cc, sm.xy[buf][j + 32], sm.zw[buf][j + 32].x);
    const uint64_t b1 = __ballot(c2a <= c.w), b2 = __ballot(c2b <= c.w);
    const uint32_t a1 = (uint32_t)b1, a2 = (uint32_t)b2;
    const uint32_t h1 = (uint32_t)(b1 >> 32), h2 = (uint32_t)(b2 >> 32);
    if constexpr (kForm == kF32) {
      mA = any_of_nibbles(a1) | (any_of_nibbles(a2) << 8);
      mB = any_of_nibbles(h1) | (any_of_nibbles(h2) << 8);
      gA = gB = 0u;
    } else {
      gA = any_of_bytes(a1) | (any_of_bytes(a2) << 4);
      gB = any_of_bytes(h1) | (any_of_bytes(h2) << 4);
      mA = ((gA & 15u) ? 1u : 0u) | ((gA >> 4) ? 2u : 0u);
      mB = ((gB & 15u) ? 1u : 0u) | ((gB >> 4) ? 2u : 0u);
    }
  };

  // Exact weights of fragment (cb, ks) of the block in buffer buf; returns
  // whether any weight is non-zero.
  auto frag = [&](int buf, int cb, int ks, const CellVec& cv, uint32_t gm, double& ws,
                  double& wt) -> bool {
    if constexpr (kForm == kF32) {
      const int k = 4 * ks + (lane >> 4);
      const double c2 = chord2(cv, sm.xy[buf][k], sm.zw[buf][k].x);
      float wf = 0.f;
      if (c2 <= a.c2R) wf = pair_weight<kWide>(c2, a.wscale);
      ws += (double)wf;
      ((float*)sm.A[buf])[(cb * 16 + ks) * 64 + lane] = wf;
      return __ballot(wf != 0.f) != 0ull;
    } else {
      const int grp = lane >> 4;
      uint32_t hi[8], lo[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) hi[t] = lo[t] = 0u;
      if ((gm >> (4 * ks + grp)) & 1u) {
        const int k0 = 32 * ks + 8 * grp;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const double c2 = chord2(cv, sm.xy[buf][k0 + t], sm.zw[buf][k0 + t].x);
          if (c2 <= a.c2R) {
            const float wf = pair_weight<kWide>(c2, a.wscale);
            hi[t] = enc_w<kForm>(wf);
            double eff = (double)dec_w<kForm>(hi[t]);
            if (kForm == kBF16Split) {
              lo[t] = f32_to_bf16(wf - dec_w<kForm>(hi[t]));
              eff += (double)bf16_to_f32(lo[t]);
            }
            ws += (double)wf;
            wt += eff;
          }
        }
      }
      const int slot = (cb * 2 + ks) * 64 + lane;
      uint32_t any;
      if (kForm == kFP8S) {
        const uint2 v = make_uint2(hi[0] | (hi[1] << 8) | (hi[2] << 16) | (hi[3] << 24),
                                   hi[4] | (hi[5] << 8) | (hi[6] << 16) | (hi[7] << 24));
        ((uint2*)sm.A[buf])[slot] = v;
        any = v.x | v.y;
      } else {
        const uint4 v = make_uint4(hi[0] | (hi[1] << 16), hi[2] | (hi[3] << 16),
                                   hi[4] | (hi[5] << 16), hi[6] | (hi[7] << 16));
        sm.A[buf][slot] = v;
        any = v.x | v.y | v.z | v.w;
        if (kForm == kBF16Split) {
          const uint4 u = make_uint4(lo[0] | (lo[1] << 16), lo[2] | (lo[3] << 16),
                                     lo[4] | (lo[5] << 16), lo[6] | (lo[7] << 16));
          sm.A[buf][kCB * 2 * 64 + slot] = u;
          any |= u.x | u.y | u.z | u.w;
        }
      }
      return __ballot(any != 0u) != 0ull;
    }
  };

  // The wave's fragment lists of the block being weighted, one bit per
  // (block, k-step): bit ks for cbA, bit kNS + ks for cbB; pending (pm) and
  // kept (rm: marked and not found all zero).  Wave-uniform.
  uint32_t pm = 0u, rm = 0u, gA = 0u, gB = 0u;
  auto start_block = [&](int buf) {
    uint32_t mA, mB;
    coarse(buf, mA, mB, gA, gB);
    pm = rm = mA | (mB << kNS);
  };
  auto one_frag = [&](int buf) {
    if (pm) {
      const int bit = __builtin_ctz(pm);
      pm &= pm - 1u;
      const bool isB = bit >= kNS;
      const int ks = isB ? bit - kNS : bit;
      double dws = 0.0, dwt = 0.0;
      const bool nz = isB ? frag(buf, cbB, ks, cellB, gB, dws, dwt)
                          : frag(buf, cbA, ks, cellA, gA, dws, dwt);
      if (!nz) rm &= ~(1u << bit);
      if (isB) {
        wsB += dws;
        wtB += dwt;
      } else {
        wsA += dws;
        wtA += dwt;
      }
    }
  };
  auto finish_block = [&](int buf) {
    while (pm) one_frag(buf);
    if (lane == 0) {
      sm.nzm[buf][cbA] = rm & ((1u << kNS) - 1u);
      sm.nzm[buf][cbB] = rm >> kNS;
    }
  };

  // prologue: centres, blocks 0 and 1 staged, weights of block 0
  if (nb > 0) {
    stage_load(0);
    stage_store(0, 0);
    stage_load(1);
    stage_store(1, 1);
  }
  __syncthreads();
  if (nb > 0) {
    start_block(0);
    finish_block(0);
  }
  __syncthreads();

  if constexpr (kForm == kF32) {
    const float* spec = (const float*)a.spec;
    constexpr int kDepth = 4;
    static_assert(kNS % kDepth == 0, "the load window must divide the k-steps");
    // Every load is issued unconditionally, so that the waits for them can
    // be counted exactly.  A channel past C reads a clamped address instead;
    // its value only reaches MFMA columns that are never stored (column j of
    // the product depends on column j of B alone).
    auto load = [&](int rbuf, int ks) -> floatx4 {
      const int64_t row = sm.row[rbuf][4 * ks + (lane >> 4)];
      const float* src = spec + row * C;
      floatx4 v;
      if (kVec == 1 || (kVec == 2 && (a.vec & 1))) {
        v = *(const floatx4*)(src + (ch_ok ? my_ch : 0));
      } else {
        v.x = src[min(my_ch + 0, C - 1)];
        v.y = src[min(my_ch + 1, C - 1)];
        v.z = src[min(my_ch + 2, C - 1)];
        v.w = src[min(my_ch + 3, C - 1)];
      }
      return v;
    };
    floatx4 bw[kDepth];
    if (nb > 0) {
#pragma unroll
      for (int d = 0; d < kDepth; ++d) bw[d] = load(0, d);
    }
    int rb = 0;  // row buffer of block b (b mod 3)
    for (uint32_t b = 0; b < nb; ++b) {
      const int cb_ = b & 1, nx_ = cb_ ^ 1;
      const int rn = (rb == 2) ? 0 : rb + 1, rn2 = (rn == 2) ? 0 : rn + 1;
      stage_load(b + 2);
      start_block(nx_);  // block b + 1 (an empty block after the last one)
      uint32_t nzc[8];   // wave-uniform: kept in scalar registers
#pragma unroll
      for (int c = 0; c < 8; ++c) nzc[c] = __builtin_amdgcn_readfirstlane(sm.nzm[cb_][8 * cg + c]);
      const float* sA = (const float*)sm.A[cb_] + (8 * cg * 16) * 64 + lane;
      // the k-steps in quads of kDepth (a runtime loop: the code of the
      // whole block would not fit the instruction cache)
#pragma unroll 1
      for (int qd = 0; qd < kNS / kDepth; ++qd) {
        // the window runs on into block b + 1 (empty past the last block)
        const bool last = qd + 1 == kNS / kDepth;
        const int lrb = last ? rn : rb;
        const int lks = last ? 0 : kDepth * (qd + 1);
#pragma unroll
        for (int j = 0; j < kDepth; ++j) {
          const int ks = kDepth * qd + j;
          const floatx4 bv = bw[j];
          bw[j] = load(lrb, lks + j);
          one_frag(nx_);
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            if ((nzc[c] >> ks) & 1u) {
              const float av = sA[(c * 16 + ks) * 64];
              acc[c][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv.x, acc[c][0], 0, 0, 0);
              acc[c][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv.y, acc[c][1], 0, 0, 0);
              acc[c][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv.z, acc[c][2], 0, 0, 0);
              acc[c][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv.w, acc[c][3], 0, 0, 0);
            }
          }
          // keep each k-step's loads, weights and products together (register
          // pressure: the scheduler would otherwise hoist the next k-steps')
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      finish_block(nx_);
      stage_store(b + 2, rn2);
      rb = rn;
      __syncthreads();
    }
  } else {
    // B fragments of one k-step: 8 candidate rows x 4 channels per lane
    constexpr bool kSplit = (kForm == kBF16Split);
    // k-steps loaded ahead (0: at use; the split and element-wise forms
    // have no registers to spare for a window)
    constexpr int kDepth = (kForm == kFP8S) ? 2 : (kSplit || kVec != 1) ? 0 : 1;
    struct Frag {
      uint32_t x[8], y[8];    // FP8: x only (4 bytes per row); 16-bit: 8 bytes per row
      uint32_t lx[8], ly[8];  // low plane of the split form
    };
    auto load = [&](int rbuf, int ks, Frag& f) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int64_t row = sm.row[rbuf][kK * ks + 8 * (lane >> 4) + t];
        // unconditional loads, clamped past C (as in the FP32 path)
        if (kForm == kFP8S) {
          const uint8_t* src = (const uint8_t*)a.spec + row * C;
          if (kVec == 1) {
            f.x[t] = *(const uint32_t*)(src + (ch_ok ? my_ch : 0));
          } else {
            uint32_t v = 0u;
#pragma unroll
            for (int e = 0; e < 4; ++e) v |= (uint32_t)src[min(my_ch + e, C - 1)] << (8 * e);
            f.x[t] = v;
          }
        } else {
#pragma unroll
          for (int plane = 0; plane < (kSplit ? 2 : 1); ++plane) {
            const uint16_t* src = (const uint16_t*)(plane ? a.spec_lo : a.spec) + row * C;
            uint2 d;
            if (kVec == 1) {
              d = *(const uint2*)(src + (ch_ok ? my_ch : 0));
            } else {
              uint32_t e[4];
#pragma unroll
              for (int j = 0; j < 4; ++j) e[j] = src[min(my_ch + j, C - 1)];
              d = make_uint2(e[0] | (e[1] << 16), e[2] | (e[3] << 16));
            }
            if (plane) { f.lx[t] = d.x; f.ly[t] = d.y; }
            else { f.x[t] = d.x; f.y[t] = d.y; }
          }
        }
      }
    };
    Frag bw[kDepth > 0 ? kDepth : 1];
    if (nb > 0) {
#pragma unroll
      for (int d = 0; d < kDepth; ++d) load(0, d, bw[d]);
    }
    int rb = 0;
    for (uint32_t b = 0; b < nb; ++b) {
      const int cb_ = b & 1, nx_ = cb_ ^ 1;
      const int rn = (rb == 2) ? 0 : rb + 1, rn2 = (rn == 2) ? 0 : rn + 1;
      stage_load(b + 2);
      start_block(nx_);
      uint32_t nzc[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) nzc[c] = __builtin_amdgcn_readfirstlane(sm.nzm[cb_][8 * cg + c]);
#pragma unroll
      for (int ks = 0; ks < kNS; ++ks) {
        Frag f;
        if constexpr (kDepth == 0) {
          load(rb, ks, f);
        } else {
          f = bw[ks % kDepth];
          if (ks + kDepth < kNS) load(rb, ks + kDepth, bw[ks % kDepth]);
          else load(rn, ks + kDepth - kNS, bw[ks % kDepth]);
        }
        one_frag(nx_);
        uint32_t any = 0;
#pragma unroll
        for (int c = 0; c < 8; ++c) any |= nzc[c];
        if (!((any >> ks) & 1u)) continue;
        // repack: the 8 rows of channel q into the B operand of MFMA q
        uint32_t fb[4][4], fbl[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (kForm == kFP8S) {
            fb[q][0] = ((f.x[0] >> (8 * q)) & 0xFFu) | (((f.x[1] >> (8 * q)) & 0xFFu) << 8) |
                       (((f.x[2] >> (8 * q)) & 0xFFu) << 16) | (((f.x[3] >> (8 * q)) & 0xFFu) << 24);
            fb[q][1] = ((f.x[4] >> (8 * q)) & 0xFFu) | (((f.x[5] >> (8 * q)) & 0xFFu) << 8) |
                       (((f.x[6] >> (8 * q)) & 0xFFu) << 16) | (((f.x[7] >> (8 * q)) & 0xFFu) << 24);
          } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              fb[q][m] = elem16(make_uint2(f.x[2 * m], f.y[2 * m]), q) |
                         (elem16(make_uint2(f.x[2 * m + 1], f.y[2 * m + 1]), q) << 16);
              if (kSplit)
                fbl[q][m] = elem16(make_uint2(f.lx[2 * m], f.ly[2 * m]), q) |
                            (elem16(make_uint2(f.lx[2 * m + 1], f.ly[2 * m + 1]), q) << 16);
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          if (!((nzc[c] >> ks) & 1u)) continue;
          const int slot = ((8 * cg + c) * 2 + ks) * 64 + lane;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            floatx4& acq = acc[c][q];
            if (kForm == kFP8S) {
              const uint2 av = ((const uint2*)sm.A[cb_])[slot];
              const long A = (long)(((uint64_t)av.y << 32) | av.x);
              const long B = (long)(((uint64_t)fb[q][1] << 32) | fb[q][0]);
              acq = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(A, B, acq, 0, 0, 0);
            } else {
              const uint4 av = sm.A[cb_][slot];
              const uint4 bv = make_uint4(fb[q][0], fb[q][1], fb[q][2], fb[q][3]);
              if (kForm == kF16S) {
                acq = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(halfx8, av),
                                                            __builtin_bit_cast(halfx8, bv), acq, 0, 0, 0);
              } else {
                acq = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                             __builtin_bit_cast(bf16x8, bv), acq, 0, 0, 0);
                if (kSplit) {
                  const uint4 al = sm.A[cb_][kCB * 2 * 64 + slot];
                  const uint4 bl = make_uint4(fbl[q][0], fbl[q][1], fbl[q][2], fbl[q][3]);
                  acq = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                               __builtin_bit_cast(bf16x8, bl), acq, 0, 0, 0);
                  acq = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al),
                                                               __builtin_bit_cast(bf16x8, bv), acq, 0, 0, 0);
                }
              }
            }
          }
        }
      }
      finish_block(nx_);
      stage_store(b + 2, rn2);
      rb = rn;
      __syncthreads();
    }
  }

  // weight sums of each cell: add the four candidate subsets (lanes l,
  // l + 16, l + 32, l + 48)
  if (kForm == kF32) {
    wtA = wsA;
    wtB = wsB;
  }
#pragma unroll
  for (int o = 16; o < 64; o <<= 1) {
    wsA += __shfl_xor(wsA, o);
    wsB += __shfl_xor(wsB, o);
    wtA += __shfl_xor(wtA, o);
    wtB += __shfl_xor(wtB, o);
  }
  if (lane < 16) {
    sm.Wt[cbA * 16 + li] = wtA;
    sm.Wt[cbB * 16 + li] = wtB;
    if (a.wmap && slab == 0) {
      const int xa = cell_x(cbA), ya = cell_y(cbA), xb = cell_x(cbB), yb = cell_y(cbB);
      if (xa < g.nx && ya < g.ny) a.wmap[(int64_t)ya * g.nx + xa] = (float)wsA;
      if (xb < g.nx && yb < g.ny) a.wmap[(int64_t)yb * g.nx + xb] = (float)wsB;
    }
  }
  __syncthreads();

  // V = U / W~ (x the channel scale), NaN where no pair is within R.  The four
  // cells r = 0..3 of a lane are consecutive in x: one 16-byte store per
  // channel where the rows allow it (bit 1 of a.vec), else one per cell.
  const float qnan = __builtin_nanf("");
  const bool vst = (a.vec & 2) != 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int cb = 8 * cg + c;
    const int y = ty * kTileY + (cb >> 2) * 4 + (lane >> 4);
    const int x0 = tx * kTileX + (cb & 3) * 4;
    if (y >= g.ny || x0 >= g.nx) continue;
    float inv[4];
    bool has[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double wt = sm.Wt[cb * 16 + 4 * (lane >> 4) + r];
      has[r] = wt > 0.0;
      inv[r] = has[r] ? (float)(1.0 / wt) : 0.f;
    }
    float* row = a.cube + (int64_t)y * g.nx + x0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t ch = my_ch + q;
      if (ch >= C) continue;
      const float sc = (kForm == kF16S || kForm == kFP8S) ? a.scale[ch] : 1.f;
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = has[r] ? acc[c][q][r] * inv[r] * sc : qnan;
      float* dst = row + ch * G;
      if (vst && x0 + 3 < g.nx) {
        *(floatx4*)dst = floatx4{v[0], v[1], v[2], v[3]};
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (x0 + r < g.nx) dst[r] = v[r];
      }
    }
  }
}

template <int kForm, int kVec, bool kWide>
__global__ void __launch_bounds__(kWGThreads, 1) k_gather_mfma(const GatherArgs a) {
  __shared__ GatherSmem sm;
  // XCD-aware order: the hardware deals consecutive workgroups to the eight
  // XCDs in turn; give each XCD a contiguous run of tiles so that tiles that
  // share candidate rows run together behind the same L2.
  const int per_slab = a.tiles_per_xcd * 8;
  const int slab = blockIdx.x / per_slab;
  const int local = blockIdx.x - slab * per_slab;
  const int tile = (local & 7) * a.tiles_per_xcd + (local >> 3);
  if (tile >= a.ntiles) return;
  gather_tile<kForm, kVec, kWide>(a, tile, slab, sm);
}

// ---------------------------------------------------------------------------
// Few channels (C <= 8, FP32) and pair counting: one thread per cell of the
// 16 x 16 tile (256 threads); with a 512-thread workgroup the two halves take
// alternate blocks of 256 candidates and their FP64 sums are added.
// ---------------------------------------------------------------------------
// stage: nparts x 16 KB of LDS (candidate vectors, then their spectra);
// with two parts also the 18 KB of the final reduction.
template <bool kCount>
__device__ void cells_tile(const GatherArgs& a, int tile, uint2* s_rng, uint32_t* s_pre,
                           double4* stage, unsigned long long* pair_count) {
  constexpr int kBlk = 256;
  const int tid = threadIdx.x;
  const int part = tid >> 8, nparts = blockDim.x >> 8;
  const int ci = tid & 255;
  const int tx = tile % a.ntx, ty = tile / a.ntx;
  const GridGeom& g = a.g;
  const int ix = tx * kTileX + (ci & 15), iy = ty * kTileY + (ci >> 4);
  const CellVec cell = cell_vec(g, ix, iy);
  const uint32_t total =
      stage_ranges(a.ranges + (int64_t)tile * a.maxr, a.nranges[tile], s_rng, s_pre);
  const int C = (int)a.C;
  const float* spec = (const float*)a.spec;
  double4* sx = stage + part * kBlk;                                   // [nparts][256] double4
  float* sspec = (float*)(stage + nparts * kBlk) + part * kBlk * 8;    // [nparts][256][8] float
  double acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = 0.0;
  double wsum = 0.0;
  unsigned long long npair = 0;
  uint32_t cur = 0;
  const uint32_t nblk = (total + kBlk - 1) / kBlk;
  for (uint32_t b0 = 0; b0 < nblk; b0 += nparts) {
    const uint32_t blk = b0 + part;
    const uint32_t q = blk * kBlk + ci;
    if (blk < nblk && q < total) {
      const uint32_t pos = cand_pos(q, s_rng, s_pre, &cur);
      sx[ci] = a.xyz[pos];
      if (!kCount) {
        const int64_t row = a.perm[pos];
#pragma unroll
        for (int c = 0; c < 8; ++c) sspec[ci * 8 + c] = (c < C) ? spec[row * C + c] : 0.f;
      }
    } else {
      const double nan = __builtin_nan("");
      sx[ci] = make_double4(nan, nan, nan, nan);
    }
    __syncthreads();
    if (blk < nblk) {
      const int kmax = (int)min<uint32_t>(kBlk, total - blk * kBlk);
      for (int k = 0; k < kmax; ++k) {
        const double c2 = chord2(cell, sx[k]);
        if (c2 <= a.c2R) {
          if (kCount) {
            ++npair;
          } else {
            const double w = (double)pair_weight<true>(c2, a.wscale);
            wsum += w;
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[c] += w * (double)sspec[k * 8 + c];
          }
        }
      }
    }
    __syncthreads();
  }
  if (kCount) {
    for (int off = 32; off > 0; off >>= 1) npair += __shfl_xor(npair, off);
    if ((tid & 63) == 0 && npair) atomicAdd(pair_count, npair);
    return;
  }
  if (nparts > 1) {
    double* red = (double*)stage;  // [9][256]
    if (part == 1) {
#pragma unroll
      for (int c = 0; c < 8; ++c) red[c * 256 + ci] = acc[c];
      red[8 * 256 + ci] = wsum;
    }
    __syncthreads();
    if (part == 0) {
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] += red[c * 256 + ci];
      wsum += red[8 * 256 + ci];
    }
  }
  if (part != 0 || ix >= g.nx || iy >= g.ny) return;
  const int64_t G = (int64_t)g.nx * g.ny;
  const int64_t cellidx = (int64_t)iy * g.nx + ix;
  if (a.wmap) a.wmap[cellidx] = (float)wsum;
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (c < C) a.cube[c * G + cellidx] = (wsum > 0.0) ? (float)(acc[c] / wsum) : __builtin_nanf("");
}

struct CellsSmem {
  uint2 rng[kMaxRangesLimit];
  uint32_t pre[kMaxRangesLimit + 1];
  double4 stage[2 * 256];
};

template <bool kCount>
__global__ void __launch_bounds__(256) k_gather_cells(const GatherArgs a,
                                                      unsigned long long* __restrict__ pair_count) {
  __shared__ CellsSmem sm;
  cells_tile<kCount>(a, (int)blockIdx.x, sm.rng, sm.pre, sm.stage, pair_count);
}

// ---------------------------------------------------------------------------
// Batch kernel (FP32 spectra, rows read 4 elements at a time, supports below
// the series bound).  The item space concatenates the fields' (slab, tile)
// grids in the host's field order; workgroup b takes one item.  With the XCD
// split, the hardware's round-robin of workgroups over the eight XCDs is
// undone: XCD x (workgroups b with b % 8 == x) takes the contiguous x-th
// eighth of the item space, so that neighbouring tiles of one field, which
// share candidate rows, run behind the same L2.  The dispatcher hands out
// workgroups as CUs free up, which balances fields of unequal cost.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kWGThreads, 1) k_gather_batch(const GatherArgs* __restrict__ fields,
                                                                const BatchSeg* __restrict__ segs,
                                                                uint32_t nseg, uint32_t nitems,
                                                                int xcd_split) {
  __shared__ GatherSmem sm;
  const uint32_t per_xcd = (nitems + kBatchXcds - 1) / kBatchXcds;
  const uint32_t it = xcd_split ? (blockIdx.x % kBatchXcds) * per_xcd + blockIdx.x / kBatchXcds
                                : blockIdx.x;
  if (it >= nitems) return;
  // the last segment whose base is <= it (values made wave-uniform: scalar
  // registers, not vector ones)
  uint32_t lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (__builtin_amdgcn_readfirstlane(segs[mid].base) <= it) lo = mid; else hi = mid - 1;
  }
  const uint32_t base = __builtin_amdgcn_readfirstlane(segs[lo].base);
  const uint32_t ntiles = __builtin_amdgcn_readfirstlane(segs[lo].ntiles);
  const uint32_t field = __builtin_amdgcn_readfirstlane(segs[lo].field);
  const uint32_t local = it - base;
  const uint32_t slab = local / ntiles;
  const uint32_t tile = local - slab * ntiles;
  GatherArgs a;
  {
    static_assert(sizeof(GatherArgs) % 4 == 0, "copied word by word");
    const uint32_t* src = (const uint32_t*)(fields + field);
    uint32_t* dst = (uint32_t*)&a;
#pragma unroll
    for (int w = 0; w < (int)(sizeof(GatherArgs) / 4); ++w)
      dst[w] = __builtin_amdgcn_readfirstlane(src[w]);
  }
  gather_tile<kF32, 1, false>(a, (int)tile, (int)slab, sm);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static bool g_vec_rows(int nx, const float* cube) {
  return nx % 4 == 0 && (uintptr_t)cube % 16 == 0;
}

static GatherArgs base_args(const hcg_plan_s* p, int64_t C, float* cube, float* wmap) {
  GatherArgs a;
  memset(&a, 0, sizeof(a));  // padding bytes too: the batch compares tables bytewise
  a.xyz = p->xyz;
  a.perm = p->perm;
  a.ranges = p->ranges;
  a.nranges = p->nranges;
  a.maxr = p->maxr;
  a.sentinel = (uint32_t)p->n;
  a.C = C;
  a.g = p->grid;
  a.ntx = p->ntx;
  a.ntiles = p->ntx * p->nty;
  a.tiles_per_xcd = (a.ntiles + 7) / 8;
  const double s = std::sin(0.5 * p->support_rad);
  a.c2R = 4.0 * s * s;
  a.wscale = -1.4426950408889634 / (2.0 * p->sigma_rad * p->sigma_rad);  // -log2(e) / 2 sigma^2
  a.cube = cube;
  a.wmap = wmap;
  // bit 1: every 4-cell group of a cube row starts 16-byte aligned
  if (g_vec_rows(p->grid.nx, cube)) a.vec |= 2;
  return a;
}

GatherArgs make_f32_args(const hcg_plan_s* p, const float* spec, int64_t C, float* cube,
                         float* wmap) {
  GatherArgs a = base_args(p, C, cube, wmap);
  a.spec = spec;
  if (C % 4 == 0 && (uintptr_t)spec % 16 == 0) a.vec |= 1;
  return a;
}

bool batch_takes(const GatherArgs& a) { return a.C > 8 && (a.vec & 1) && a.c2R < kSeriesMax; }

hcg_status launch_f32(const GatherArgs& a, hipStream_t stream) {
  if (a.C <= 8) {
    k_gather_cells<false><<<(unsigned)a.ntiles, 256, 0, stream>>>(a, nullptr);
    HCG_LAUNCH_CHECK("k_gather_cells");
    return HCG_OK;
  }
  const int64_t slabs = (a.C + kSlab - 1) / kSlab;
  const int64_t blocks = slabs * a.tiles_per_xcd * 8;
  if (blocks > INT32_MAX) return fail(HCG_E_UNSUPPORTED, "hcg_grid: too many channels");
  const bool wide = a.c2R >= kSeriesMax;
  if ((a.vec & 1) && !wide) k_gather_mfma<kF32, 1, false><<<(unsigned)blocks, kWGThreads, 0, stream>>>(a);
  else if (a.vec & 1) k_gather_mfma<kF32, 1, true><<<(unsigned)blocks, kWGThreads, 0, stream>>>(a);
  else if (!wide) k_gather_mfma<kF32, 0, false><<<(unsigned)blocks, kWGThreads, 0, stream>>>(a);
  else k_gather_mfma<kF32, 0, true><<<(unsigned)blocks, kWGThreads, 0, stream>>>(a);
  HCG_LAUNCH_CHECK("k_gather_mfma");
  return HCG_OK;
}

hcg_status launch_batch(const GatherArgs* fields, const BatchSeg* segs, uint32_t nseg,
                        uint32_t nitems, int xcd_split, hipStream_t stream) {
  if (nitems == 0) return HCG_OK;
  const uint32_t per_xcd = (nitems + kBatchXcds - 1) / kBatchXcds;
  const uint32_t blocks = xcd_split ? per_xcd * kBatchXcds : nitems;
  k_gather_batch<<<blocks, kWGThreads, 0, stream>>>(fields, segs, nseg, nitems, xcd_split);
  HCG_LAUNCH_CHECK("k_gather_batch");
  return HCG_OK;
}

template <int kForm>
static hcg_status launch_mfma(const hcg_plan_s* p, const void* spec, const void* spec_lo,
                              const float* scale, int64_t C, float* cube, float* wmap,
                              hipStream_t stream) {
  GatherArgs a = base_args(p, C, cube, wmap);
  a.spec = spec;
  a.spec_lo = spec_lo;
  a.scale = scale;
  const size_t esz = (kForm == kF32) ? 4 : (kForm == kFP8S) ? 1 : 2;
  const bool vec = (C % 4 == 0) && ((uintptr_t)spec % (4 * esz) == 0) &&
                   (!spec_lo || (uintptr_t)spec_lo % (4 * esz) == 0);
  if (vec) a.vec |= 1;
  const int64_t slabs = (C + kSlab - 1) / kSlab;
  const int64_t blocks = slabs * a.tiles_per_xcd * 8;
  if (blocks > INT32_MAX) return fail(HCG_E_UNSUPPORTED, "hcg_grid: too many channels");
  const bool wide = a.c2R >= kSeriesMax;
  if (vec && !wide) k_gather_mfma<kForm, 1, false><<<(unsigned)blocks, kWGThreads, 0, stream>>>(a);
  else if (vec) k_gather_mfma<kForm, 1, true><<<(unsigned)blocks, kWGThreads, 0, stream>>>(a);
  else if (!wide) k_gather_mfma<kForm, 0, false><<<(unsigned)blocks, kWGThreads, 0, stream>>>(a);
  else k_gather_mfma<kForm, 0, true><<<(unsigned)blocks, kWGThreads, 0, stream>>>(a);
  HCG_LAUNCH_CHECK("k_gather_mfma");
  return HCG_OK;
}

}  // namespace hcg

using namespace hcg;

extern "C" hcg_status hcg_grid(hcg_plan_t plan, const void* spectra, int64_t nchan,
                               hcg_dtype dtype, const float* chan_scale, float* cube,
                               float* weights, void* hip_stream) {
  if (!plan) return fail(HCG_E_ARG, "hcg_grid: plan is NULL");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_grid: not a live plan");
  if (!spectra || !cube) return fail(HCG_E_ARG, "hcg_grid: spectra and cube must not be NULL");
  if (nchan < 1) return fail(HCG_E_ARG, "hcg_grid: nchan must be >= 1");
  const bool scaled = (dtype == HCG_F16_SCALED || dtype == HCG_FP8E4M3_SCALED);
  if (dtype < HCG_F32 || dtype > HCG_FP8E4M3_SCALED)
    return fail(HCG_E_UNSUPPORTED, "hcg_grid: unknown dtype %d", (int)dtype);
  if (scaled && !chan_scale) return fail(HCG_E_ARG, "hcg_grid: chan_scale is required for this dtype");
  if (!scaled && chan_scale) return fail(HCG_E_ARG, "hcg_grid: chan_scale must be NULL for this dtype");
  const hcg_plan_s* p = plan;
  hipStream_t stream = (hipStream_t)hip_stream;
  switch (dtype) {
    case HCG_F32:
      return launch_f32(make_f32_args(p, (const float*)spectra, nchan, cube, weights), stream);
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
  }
  return fail(HCG_E_UNSUPPORTED, "hcg_grid: dtype %d", (int)dtype);
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
  const GatherArgs a = base_args(p, 1, nullptr, nullptr);
  k_gather_cells<true><<<ntiles, 256, 0, stream>>>(a, dcount);
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
