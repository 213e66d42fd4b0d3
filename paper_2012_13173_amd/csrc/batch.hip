// Batches of independent maps in one graph-captured launch of persistent
// kernels.
//
// hcg_plan_batch builds one plan per field (same device steps as hcg_plan).
// hcg_grid_batch makes every (field, tile, channel slab) a work item.  Items
// are grouped by kernel class -- the few-channel FP32 gather, and the
// matrix-core gather of each storage form -- and each class has one
// persistent kernel that runs all of its fields: the fields' item ranges are
// concatenated in a chosen field order (by estimated cost, candidates x
// channels, largest first, or as given) and the kernel decodes an item index
// through a small per-field segment table.  Its workgroups pop items from
// per-XCD counters over contiguous eighths of the class's item space and
// steal from the other eighths at the end.  The counter resets and the
// class launches are captured once in a hipGraph and replayed; the argument
// and segment tables live in device memory and are rewritten before a replay
// when pointers, forms or channel counts change.  On the first call an
// autotuner times the channel slab (256 or 512 channels) and the field order
// and keeps the fastest; the choice can be cached on disk
// (HCG_TUNE_CACHE=<file>).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "forms.h"
#include "gather_tile.h"

namespace hcg {

// Kernel classes of the batch: the matrix-core gather of each storage form
// for rows read four channels at a time (the hcg_dtype values), the
// few-channel FP32 gather, and the matrix-core gather of each form for rows
// read one element at a time (hcg_dtype + kClsScalarRows).  Each class's
// persistent kernel compiles one gather path, which keeps it in the
// registers of two workgroups per CU.
constexpr int kClsCells = 6;
constexpr int kClsScalarRows = 7;
constexpr int kClasses = 13;

// ctl: [0..7] next item of each XCD's segment, [8] item count, [9] segment
// count.  The item space of a class is cut into eight contiguous segments,
// one per XCD (the hardware deals workgroups to the XCDs in turn, so
// workgroup b starts on XCD b % 8); a workgroup pops items from its own
// XCD's segment -- neighbouring tiles of one field, sharing candidate rows in
// that XCD's L2 -- and, once it is empty, from the others.
__device__ __forceinline__ uint32_t batch_seg_begin(uint32_t total, int x) {
  return (uint32_t)(((uint64_t)total * (uint32_t)x) / kBatchXcds);
}

__global__ void k_batch_reset(uint32_t* __restrict__ ctl) {
  const uint32_t total = ctl[8];
  for (int x = 0; x < kBatchXcds; ++x) ctl[x] = batch_seg_begin(total, x);
}

// The next item of a persistent workgroup: thread 0 pops one from its
// XCD's segment, then from the others once it is empty (*k counts the
// segments it has found empty); 0xFFFFFFFF when every segment is empty.
// Called by every thread of the workgroup.
__device__ inline uint32_t batch_next_item(uint32_t* __restrict__ ctl, uint32_t total, int home,
                                           int* k, uint32_t* s_item) {
  if (threadIdx.x == 0) {
    uint32_t it = 0xFFFFFFFFu;
    while (*k < kBatchXcds) {
      const int x = (home + *k) % kBatchXcds;
      const uint32_t i = atomicAdd(&ctl[x], 1u);
      if (i < batch_seg_begin(total, x + 1)) { it = i; break; }
      ++*k;
    }
    *s_item = it;
  }
  __syncthreads();
  const uint32_t it = __builtin_amdgcn_readfirstlane(*s_item);
  __syncthreads();
  return it;
}

// The segment of item it: the last one whose base is <= it.
__device__ inline BatchSeg batch_seg_of(const BatchSeg* __restrict__ segs, uint32_t nseg,
                                        uint32_t it) {
  uint32_t lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (segs[mid].base <= it) lo = mid; else hi = mid - 1;
  }
  return segs[lo];
}

// The few-channel class (FP32, C <= 8): one wave per tile, on dynamic LDS of
// cells_batch_lds_bytes(maxr) with maxr the largest range count of the
// batch's plans, in kernels of their own (bounded at 64 threads, not by the
// matrix-core classes' 256-thread, two-per-CU bounds, so that they keep few
// registers): many tiles in flight on a CU.  Items are tiles.
//
// One workgroup per item:
__global__ void __launch_bounds__(64) k_cells_items(const GatherArgs* __restrict__ fields,
                                                    const BatchSeg* __restrict__ segs,
                                                    uint32_t nseg, int maxr) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  const uint32_t it = blockIdx.x;
  const BatchSeg sg = batch_seg_of(segs, nseg, it);
  gather_cells_tile(fields[sg.field], (int)(it - sg.base), cells_lds(s_dyn, maxr));
}

// Persistent workgroups (sixteen per CU) popping items:
__global__ void __launch_bounds__(64) k_cells_batch(const GatherArgs* __restrict__ fields,
                                                    const BatchSeg* __restrict__ segs,
                                                    uint32_t* __restrict__ ctl, int maxr) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  __shared__ uint32_t s_item;
  const CellsLds L = cells_lds(s_dyn, maxr);
  const uint32_t total = ctl[8];
  const uint32_t nseg = ctl[9];
  const int home = (int)(blockIdx.x % kBatchXcds);
  int k = 0;
  for (;;) {
    const uint32_t it = batch_next_item(ctl, total, home, &k, &s_item);
    if (it == 0xFFFFFFFFu) break;
    const BatchSeg sg = batch_seg_of(segs, nseg, it);
    gather_cells_tile(fields[sg.field], (int)(it - sg.base), L);
    __syncthreads();
  }
}

template <int kCls, int kQW, bool kWide>
__global__ void __launch_bounds__(256, 2) k_gather_batch(const GatherArgs* __restrict__ fields,
                                                         const BatchSeg* __restrict__ segs,
                                                         uint32_t* __restrict__ ctl) {
  static_assert(kCls != kClsCells, "the few-channel class has kernels of its own");
  __shared__ GatherSmem sm;
  __shared__ uint32_t s_item;
  const uint32_t total = ctl[8];
  const uint32_t nseg = ctl[9];
  const int home = (int)(blockIdx.x % kBatchXcds);
  int k = 0;  // segments visited so far (thread 0 only)
  for (;;) {
    const uint32_t it = batch_next_item(ctl, total, home, &k, &s_item);
    if (it == 0xFFFFFFFFu) break;
    const BatchSeg sg = batch_seg_of(segs, nseg, it);
    const uint32_t local = it - sg.base;
    const uint32_t slab = local / sg.ntiles;
    const uint32_t tile = local - slab * sg.ntiles;
    const GatherArgs& a = fields[sg.field];  // read on demand (scalar loads)
    if constexpr (kCls >= kClsScalarRows) {  // 256-channel slabs
      gather_tile<kCls - kClsScalarRows, 1, false, false, kWide, false>(a, (int)tile, (int)slab, sm);
    } else if constexpr (kCls == kBF16Split) {  // 256-channel slabs only (registers)
      gather_tile<kBF16Split, 1, true, false, kWide, true>(a, (int)tile, (int)slab, sm);
    } else {
      gather_tile<kCls, kQW, true, false, kWide, true>(a, (int)tile, (int)slab, sm);
    }
    __syncthreads();
  }
}

// The work-item launch of a class: one workgroup per item, no counters.  A
// field's items are its slabs x (tiles rounded up to whole eighths), decoded
// as in the per-plan gather: consecutive workgroups go to the eight XCDs in
// turn and XCD x takes the x-th eighth of the field's tiles, so the tiles an
// XCD runs together are neighbours.  The hardware dispatcher starts the
// next field's workgroups as the previous field's finish, which fills the
// tail of each field with work.  Compiled without the persistent loop, the
// 512-channel kernels keep their registers.
template <int kCls, int kQW, bool kWide>
__global__ void __launch_bounds__(256, 2) k_gather_items(const GatherArgs* __restrict__ fields,
                                                         const BatchSeg* __restrict__ segs,
                                                         uint32_t nseg) {
  static_assert(kCls != kClsCells, "the few-channel class has kernels of its own");
  __shared__ GatherSmem sm;
  const uint32_t it = blockIdx.x;
  const BatchSeg sg = batch_seg_of(segs, nseg, it);
  const uint32_t local = it - sg.base;
  const GatherArgs& a = fields[sg.field];
  const uint32_t per_slab = (uint32_t)a.tiles_per_xcd * 8u;
  const uint32_t slab = local / per_slab;
  const uint32_t loc = local - slab * per_slab;
  const uint32_t tile = (loc & 7u) * (uint32_t)a.tiles_per_xcd + (loc >> 3);
  if (tile >= (uint32_t)a.ntiles) return;
  if constexpr (kCls >= kClsScalarRows) {
    gather_tile<kCls - kClsScalarRows, 1, false, false, kWide, false>(a, (int)tile, (int)slab, sm);
  } else if constexpr (kCls == kBF16Split) {
    gather_tile<kBF16Split, 1, true, false, kWide, true>(a, (int)tile, (int)slab, sm);
  } else {
    gather_tile<kCls, kQW, true, false, kWide, true>(a, (int)tile, (int)slab, sm);
  }
}

// Launch strategies of hcg_grid_batch.
constexpr int kLaunchPersistent = 0;
constexpr int kLaunchItems = 1;

namespace {

// Launch geometry of one class: the persistent kernel (nblocks workgroups,
// after its counter reset) or the work-item kernel (one workgroup per item).
struct ClassLaunch {
  int strategy;
  int nblocks;
  uint32_t nitems, nseg;
  int cells_maxr;  // largest range count of the batch's plans (few-channel LDS)
};

template <int kCls, int kQW, bool kWide>
void launch_one(const ClassLaunch& l, const GatherArgs* fields, const BatchSeg* segs,
                uint32_t* ctl, hipStream_t stream) {
  if (l.strategy == kLaunchItems)
    k_gather_items<kCls, kQW, kWide><<<l.nitems, 256, 0, stream>>>(fields, segs, l.nseg);
  else
    k_gather_batch<kCls, kQW, kWide><<<l.nblocks, 256, 0, stream>>>(fields, segs, ctl);
}

template <int kCls>
void launch_cls(int qw, bool wide, const GatherArgs* fields, const BatchSeg* segs, uint32_t* ctl,
                const ClassLaunch& l, hipStream_t stream) {
  // classes with 256-channel slabs only have no 512-channel kernels
  constexpr bool kSlab512 = kCls < kClsCells && kCls != kBF16Split;
  if constexpr (kSlab512) {
    if (qw == 2) {
      if (wide) launch_one<kCls, 2, true>(l, fields, segs, ctl, stream);
      else launch_one<kCls, 2, false>(l, fields, segs, ctl, stream);
      return;
    }
  }
  if (wide) launch_one<kCls, 1, true>(l, fields, segs, ctl, stream);
  else launch_one<kCls, 1, false>(l, fields, segs, ctl, stream);
}

hcg_status launch_class(int cls, int qw, bool wide, const GatherArgs* fields,
                        const BatchSeg* segs, uint32_t* ctl, const ClassLaunch& l,
                        hipStream_t stream) {
  if (l.strategy == kLaunchPersistent) {
    k_batch_reset<<<1, 1, 0, stream>>>(ctl);
    HCG_LAUNCH_CHECK("k_batch_reset");
  }
  switch (cls) {
    case kClsCells: {
      // one-wave workgroups; the persistent grid eight per 256-thread one
      const size_t lds = cells_batch_lds_bytes(l.cells_maxr);
      if (l.strategy == kLaunchItems)
        k_cells_items<<<l.nitems, 64, lds, stream>>>(fields, segs, l.nseg, l.cells_maxr);
      else
        k_cells_batch<<<l.nblocks * 8, 64, lds, stream>>>(fields, segs, ctl, l.cells_maxr);
      break;
    }
    case kBF16Split: launch_cls<kBF16Split>(1, wide, fields, segs, ctl, l, stream); break;
    case kF32: launch_cls<kF32>(qw, wide, fields, segs, ctl, l, stream); break;
    case kBF16: launch_cls<kBF16>(qw, wide, fields, segs, ctl, l, stream); break;
    case kF16S: launch_cls<kF16S>(qw, wide, fields, segs, ctl, l, stream); break;
    case kFP8S: launch_cls<kFP8S>(qw, wide, fields, segs, ctl, l, stream); break;
    case kFP8Split: launch_cls<kFP8Split>(qw, wide, fields, segs, ctl, l, stream); break;
    case kClsScalarRows + kF32: launch_cls<kClsScalarRows + kF32>(1, wide, fields, segs, ctl, l, stream); break;
    case kClsScalarRows + kBF16: launch_cls<kClsScalarRows + kBF16>(1, wide, fields, segs, ctl, l, stream); break;
    case kClsScalarRows + kBF16Split: launch_cls<kClsScalarRows + kBF16Split>(1, wide, fields, segs, ctl, l, stream); break;
    case kClsScalarRows + kF16S: launch_cls<kClsScalarRows + kF16S>(1, wide, fields, segs, ctl, l, stream); break;
    case kClsScalarRows + kFP8S: launch_cls<kClsScalarRows + kFP8S>(1, wide, fields, segs, ctl, l, stream); break;
    default: launch_cls<kClsScalarRows + kFP8Split>(1, wide, fields, segs, ctl, l, stream); break;
  }
  HCG_LAUNCH_CHECK("k_gather_batch");
  return HCG_OK;
}

// Kernel class of a field's data (vec: rows read four elements at a time).
int field_class(const hcg_field_data& d, bool vec) {
  if (d.dtype == HCG_F32 && d.nchan <= 8) return kClsCells;
  return vec ? (int)d.dtype : kClsScalarRows + (int)d.dtype;
}

// Gather arguments of one field: the plan's arrays, the spectra in the form's
// storage (the low plane of a split form follows the high plane), the
// channel scales, the outputs.
GatherArgs make_field_args(const hcg_plan_s* p, const hcg_field_data& d) {
  GatherArgs a;
  memset(&a, 0, sizeof(a));  // padding bytes too: the tables are compared bytewise
  a.cells = p->cells;
  a.kern = p->kern;
  a.xyz = p->xyz;
  a.sentinel = (uint32_t)p->n;
  a.perm = p->perm;
  a.ranges = p->ranges;
  a.nranges = p->nranges;
  a.maxr = p->maxr;
  a.spec = d.spectra;
  const size_t esz = form_elem(d.dtype);
  a.spec_lo = form_split(d.dtype) ? (const char*)d.spectra + esz * (size_t)p->n * d.nchan : nullptr;
  a.scale = d.chan_scale;
  a.C = d.nchan;
  a.g = p->grid;
  a.ntx = p->ntx;
  a.ntiles = p->ntx * p->nty;
  a.tiles_per_xcd = (a.ntiles + 7) / 8;
  // 1: rows read four elements at a time; 2: eight too (rows aligned to 8
  // elements), which the narrow-support 512-channel BF16, FP16 x scale and
  // FP8 x scale kernels need
  const bool rows4 = d.nchan % 4 == 0 && (uintptr_t)d.spectra % (4 * esz) == 0 &&
                     (!a.spec_lo || (uintptr_t)a.spec_lo % (4 * esz) == 0);
  const bool rows8 = rows4 && !a.spec_lo && d.nchan % 8 == 0 &&
                     (uintptr_t)d.spectra % (8 * esz) == 0;
  a.vec = rows8 ? 2 : rows4 ? 1 : 0;
  a.c2R = support_chord2(p);
  a.cube = d.cube;
  a.wmap = d.weights;
  return a;
}

constexpr uint64_t kBatchMagic = 0x48434742'41544332ull;  // "HCGBATC2"

}  // namespace
}  // namespace hcg

using namespace hcg;

struct hcg_batch_s {
  uint64_t magic = kBatchMagic;
  int device = 0;
  int nblocks = 0;
  std::vector<hcg_plan_t> plans;
  void* arena = nullptr;  // the plans' arrays (plan_build_fields)
  std::vector<std::vector<uint32_t>> ncand;  // per field, per tile
  hcg_opts opts{};
  GatherArgs* d_fields = nullptr;  // [nfields]
  BatchSeg* d_segs = nullptr;      // [kClasses][nfields]
  uint32_t* d_ctl = nullptr;       // [kClasses][kBatchCtl]
  std::vector<GatherArgs> h_fields;
  std::vector<int64_t> built_C;
  std::vector<int> built_vec, built_cls;
  int built_qw = 0, built_order = -1, built_strategy = -1;
  uint32_t nitems[kClasses] = {};
  uint32_t nseg[kClasses] = {};
  bool wide[kClasses] = {};
  int cls_qw[kClasses] = {};  // slab width / 256 of each class
  int qw = 0, cost_order = 1, strategy = kLaunchPersistent;
  int cells_maxr = 0;  // largest range count of the plans
  bool tuned = false;
  double tune_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_qw = 0;
  // recorded after every launch: the next call's table updates wait for it,
  // so a call on another stream cannot rewrite tables a launch still reads
  hipEvent_t done = nullptr;
  bool launched = false;
};

namespace {

std::mutex g_batch_mu;
std::vector<const hcg_batch_s*> g_batches;

bool batch_is_live(const hcg_batch_s* b) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  return b && std::find(g_batches.begin(), g_batches.end(), b) != g_batches.end() &&
         b->magic == kBatchMagic;
}

void free_batch(hcg_batch_s* b) {
  if (b->done) (void)hipEventDestroy(b->done);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->d_fields) (void)hipFree(b->d_fields);
  if (b->d_segs) (void)hipFree(b->d_segs);
  if (b->d_ctl) (void)hipFree(b->d_ctl);
  for (hcg_plan_t p : b->plans) {
    if (!p) continue;
    p->batch_owned = 0;
    (void)hcg_destroy(p);
  }
  if (b->arena) (void)hipFree(b->arena);
  b->magic = 0;
  delete b;
}

// Item segments of every class for slab width 256 * qw (256 for the BF16
// hi+lo form, for fields whose rows cannot be read four elements at a time,
// and for a narrow-support BF16, FP16 x scale or FP8 x scale class with a
// field whose rows cannot be read eight at a time; one item per tile for the
// few-channel class).  The work-item launch
// gives a field slabs x (tiles rounded up to whole eighths) items.
hcg_status build_items(hcg_batch_s* b, const hcg_field_data* data, int qw, int cost_order,
                       int strategy, hipStream_t stream) {
  const size_t nf = b->plans.size();
  bool cwide[kClasses] = {}, all8[kClasses];
  for (int c = 0; c < kClasses; ++c) all8[c] = true;
  for (size_t f = 0; f < nf; ++f) {
    const int c = b->built_cls[f];
    cwide[c] = cwide[c] || !(b->h_fields[f].c2R < kNarrowChord2);
    all8[c] = all8[c] && b->built_vec[f] == 2;
  }
  for (int c = 0; c < kClasses; ++c)
    b->cls_qw[c] = (c >= kClsCells || c == kBF16Split) ? 1
                   : ((c == kBF16 || c == kF16S || c == kFP8S) && !cwide[c] && !all8[c]) ? 1
                                                                            : qw;
  std::vector<double> cost(nf);
  std::vector<BatchSeg> seg(nf);
  for (size_t f = 0; f < nf; ++f) {
    const int64_t C = data[f].nchan;
    const int cls = b->built_cls[f];
    const bool cells = cls == kClsCells;
    const int64_t width = cells ? C : 256 * b->cls_qw[cls];
    const int64_t slabs = cells ? 1 : (C + width - 1) / width;
    const std::vector<uint32_t>& nc = b->ncand[f];
    double cand = 0.0;
    for (uint32_t v : nc) cand += v;
    // candidates x channels, plus the output writes
    cost[f] = cand * (cells ? 8.0 : (double)std::max<int64_t>(C, 64)) +
              64.0 * (double)nc.size() * (double)C;
    seg[f] = BatchSeg{0u, (uint32_t)nc.size(), (uint32_t)slabs, (uint32_t)f};
  }
  std::vector<size_t> order(nf);
  for (size_t f = 0; f < nf; ++f) order[f] = f;
  if (cost_order)
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return cost[x] > cost[y]; });
  std::vector<BatchSeg> host((size_t)kClasses * nf);
  std::vector<uint32_t> ctl((size_t)kClasses * kBatchCtl, 0u);
  for (int c = 0; c < kClasses; ++c) {
    uint64_t base = 0;
    uint32_t nseg = 0;
    bool wide = false;
    for (size_t k = 0; k < nf; ++k) {
      const size_t f = order[k];
      if (b->built_cls[f] != c) continue;
      BatchSeg sg = seg[f];
      sg.base = (uint32_t)base;
      host[(size_t)c * nf + nseg++] = sg;
      const uint64_t span = (strategy == kLaunchItems && c != kClsCells)
                                ? (uint64_t)b->h_fields[f].tiles_per_xcd * 8u
                                : (uint64_t)sg.ntiles;
      base += span * sg.slabs;
      if (base >= 0x7FFFFFF0ull) return fail(HCG_E_UNSUPPORTED, "hcg_grid_batch: too many items");
      wide = wide || !(b->h_fields[f].c2R < kNarrowChord2);
    }
    b->nitems[c] = (uint32_t)base;
    b->nseg[c] = nseg;
    b->wide[c] = wide;
    ctl[(size_t)c * kBatchCtl + 8] = (uint32_t)base;
    ctl[(size_t)c * kBatchCtl + 9] = nseg;
  }
  HCG_HIP(hipMemcpyAsync(b->d_segs, host.data(), sizeof(BatchSeg) * host.size(),
                         hipMemcpyHostToDevice, stream));
  HCG_HIP(hipMemcpyAsync(b->d_ctl, ctl.data(), sizeof(uint32_t) * ctl.size(),
                         hipMemcpyHostToDevice, stream));
  HCG_HIP(hipStreamSynchronize(stream));  // the host arrays above go out of scope
  b->built_qw = qw;
  b->built_order = cost_order;
  b->built_strategy = strategy;
  return HCG_OK;
}

// One persistent launch (after its counter reset) per class that has items.
hcg_status launch_direct(hcg_batch_s* b, hipStream_t stream) {
  const size_t nf = b->plans.size();
  for (int c = 0; c < kClasses; ++c) {
    if (!b->nitems[c]) continue;
    const ClassLaunch l{b->strategy, b->nblocks, b->nitems[c], b->nseg[c], b->cells_maxr};
    const hcg_status st = launch_class(c, b->cls_qw[c], b->wide[c], b->d_fields,
                                       b->d_segs + (size_t)c * nf,
                                       b->d_ctl + (size_t)c * kBatchCtl, l, stream);
    if (st != HCG_OK) return st;
  }
  return HCG_OK;
}

std::string batch_signature(const hcg_batch_s* b, const hcg_field_data* data) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](double v) {
    unsigned char bytes[8];
    memcpy(bytes, &v, 8);
    for (unsigned char c : bytes) { h ^= c; h *= 1099511628211ull; }
  };
  for (size_t f = 0; f < b->plans.size(); ++f) {
    const hcg_plan_s* p = b->plans[f];
    mix((double)p->n);
    mix((double)p->grid.nx);
    mix((double)p->grid.ny);
    mix(p->sigma_rad);
    mix(p->support_rad);
    mix((double)data[f].nchan);
    mix((double)data[f].dtype);
  }
  char buf[32];
  snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  return buf;
}

// Tune cache lines: "<signature> <qw> <cost order> <launch strategy>"; lines
// of another shape are skipped, the last matching line wins.
bool tune_cache_lookup(const std::string& sig, int* qw, int* order, int* strategy) {
  const char* path = getenv("HCG_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[256], s[64];
  int q, o, l;
  bool found = false;
  while (fgets(line, sizeof(line), f))
    if (sscanf(line, "%63s %d %d %d", s, &q, &o, &l) == 4 && sig == s && (q == 1 || q == 2) &&
        (o == 0 || o == 1) && (l == kLaunchPersistent || l == kLaunchItems)) {
      *qw = q;
      *order = o;
      *strategy = l;
      found = true;
    }
  fclose(f);
  return found;
}

void tune_cache_store(const std::string& sig, int qw, int order, int strategy) {
  const char* path = getenv("HCG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d %d\n", sig.c_str(), qw, order, strategy);
  fclose(f);
}

}  // namespace

extern "C" hcg_status hcg_plan_batch(hcg_batch_t* out, int32_t nfields,
                                     const hcg_field_desc* fields, const hcg_opts* opts,
                                     void* hip_stream) {
  if (!out) return fail(HCG_E_ARG, "hcg_plan_batch: out is NULL");
  *out = nullptr;
  if (nfields < 1 || !fields) return fail(HCG_E_ARG, "hcg_plan_batch: need at least one field");
  hcg_opts o{};
  if (opts) o = *opts;
  if (o.chan_tile != 0 && o.chan_tile != 256 && o.chan_tile != 512)
    return fail(HCG_E_UNSUPPORTED, "hcg_plan_batch: chan_tile must be 0, 256 or 512");
  if (o.coarsen) return fail(HCG_E_UNSUPPORTED, "hcg_plan_batch: coarsen must be 0");
  if (o.flags & ~(uint32_t)(HCG_BATCH_PERSISTENT | HCG_BATCH_ITEMS) ||
      (o.flags & HCG_BATCH_PERSISTENT && o.flags & HCG_BATCH_ITEMS))
    return fail(HCG_E_UNSUPPORTED, "hcg_plan_batch: flags may hold one of HCG_BATCH_PERSISTENT "
                "and HCG_BATCH_ITEMS only");
  hcg_status st = check_device_arch();
  if (st != HCG_OK) return st;
  hipStream_t stream = (hipStream_t)hip_stream;
  auto* b = new hcg_batch_s();
  b->opts = o;
  hcg_opts po = o;  // the per-field plans take nside and tile only
  po.chan_tile = 0;
  po.flags = 0;
  int cus = 0;
  if (hipGetDevice(&b->device) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
    free_batch(b);
    return fail(HCG_E_DEVICE, "hcg_plan_batch: device query failed");
  }
  // The plans are built together (plan_build_fields): each build step runs
  // for every field in one launch on the caller's stream, with one host read
  // after the pixels and one at the end; the plans' arrays share one
  // allocation that the batch owns.
  b->plans.assign(nfields, nullptr);
  int32_t failed = -1;
  st = plan_build_fields(nfields, fields, &po, stream, b->plans.data(), &b->arena, &b->ncand,
                         &failed);
  if (st != HCG_OK) {
    const std::string msg = hcg_last_error();
    free_batch(b);
    if (failed >= 0) return fail(st, "hcg_plan_batch: field %d: %s", failed, msg.c_str());
    return fail(st, "hcg_plan_batch: %s", msg.c_str());
  }
  b->nblocks = 2 * cus;  // two 256-thread workgroups per CU
  for (hcg_plan_t pl : b->plans) b->cells_maxr = std::max(b->cells_maxr, pl->maxr);
  if (hipMalloc(&b->d_fields, sizeof(GatherArgs) * nfields) != hipSuccess ||
      hipMalloc(&b->d_segs, sizeof(BatchSeg) * nfields * kClasses) != hipSuccess ||
      hipMalloc(&b->d_ctl, sizeof(uint32_t) * kBatchCtl * kClasses) != hipSuccess ||
      hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    free_batch(b);
    return fail(HCG_E_NOMEM, "hcg_plan_batch: cannot allocate the batch tables");
  }
  b->h_fields.resize(nfields);
  memset(b->h_fields.data(), 0, sizeof(GatherArgs) * nfields);
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    g_batches.push_back(b);
  }
  *out = b;
  return HCG_OK;
}

extern "C" hcg_status hcg_grid_batch(hcg_batch_t batch, const hcg_field_data* data,
                                     void* hip_stream) {
  if (!batch || !data) return fail(HCG_E_ARG, "hcg_grid_batch: NULL pointer");
  if (!batch_is_live(batch)) return fail(HCG_E_STATE, "hcg_grid_batch: not a live batch");
  hcg_batch_s* b = batch;
  hipStream_t stream = (hipStream_t)hip_stream;
  const size_t nf = b->plans.size();
  for (size_t f = 0; f < nf; ++f) {
    const hcg_field_data& d = data[f];
    if (!d.spectra || !d.cube) return fail(HCG_E_ARG, "hcg_grid_batch: field %zu: NULL spectra or cube", f);
    if (d.nchan < 1) return fail(HCG_E_ARG, "hcg_grid_batch: field %zu: nchan must be >= 1", f);
    if (d.dtype < HCG_F32 || d.dtype > HCG_FP8E4M3_SPLIT)
      return fail(HCG_E_UNSUPPORTED, "hcg_grid_batch: field %zu: unknown dtype %d", f, (int)d.dtype);
    if (form_scaled(d.dtype) != (d.chan_scale != nullptr))
      return fail(HCG_E_ARG, "hcg_grid_batch: field %zu: chan_scale is required for the scaled "
                  "dtypes and must be NULL for the others", f);
  }
  // the tables below are rewritten on this stream: wait for the last launch,
  // whichever stream it ran on
  if (b->launched) HCG_HIP(hipStreamWaitEvent(stream, b->done, 0));
  // argument table
  bool layout_changed = b->built_C.size() != nf;
  std::vector<GatherArgs> fresh(nf);
  std::vector<int> vecs(nf), clss(nf);
  for (size_t f = 0; f < nf; ++f) {
    const hcg_field_data& d = data[f];
    fresh[f] = make_field_args(b->plans[f], d);
    vecs[f] = fresh[f].vec;
    clss[f] = field_class(d, vecs[f] != 0);
    if (!layout_changed && (b->built_C[f] != d.nchan || b->built_vec[f] != vecs[f] ||
                            b->built_cls[f] != clss[f]))
      layout_changed = true;
  }
  if (memcmp(fresh.data(), b->h_fields.data(), sizeof(GatherArgs) * nf) != 0) {
    b->h_fields = fresh;
    HCG_HIP(hipMemcpyAsync(b->d_fields, b->h_fields.data(), sizeof(GatherArgs) * nf,
                           hipMemcpyHostToDevice, stream));
  }
  if (layout_changed) {
    b->built_C.resize(nf);
    b->built_vec = vecs;
    b->built_cls = clss;
    for (size_t f = 0; f < nf; ++f) b->built_C[f] = data[f].nchan;
    b->built_qw = 0;  // force a rebuild
  }
  hcg_status st;
  if (!b->tuned) {
    // the configurations the options leave open: slab width x field order x
    // launch strategy, each timed once on this batch
    const int fixed_strategy = (b->opts.flags & HCG_BATCH_PERSISTENT) ? kLaunchPersistent
                               : (b->opts.flags & HCG_BATCH_ITEMS)    ? kLaunchItems
                                                                      : -1;
    int cfg[8][3], ncfg = 0;
    for (int l = 0; l < 2; ++l)
      for (int o = 1; o >= 0; --o)
        for (int q = 1; q <= 2; ++q) {
          if (fixed_strategy >= 0 && l != fixed_strategy) continue;
          if (b->opts.chan_tile && (q != b->opts.chan_tile / 256 || o != 1)) continue;
          cfg[ncfg][0] = q;
          cfg[ncfg][1] = o;
          cfg[ncfg][2] = l;
          ++ncfg;
        }
    const std::string sig = batch_signature(b, data);
    int q = cfg[0][0], o = cfg[0][1], l = cfg[0][2];
    if (ncfg > 1 && !tune_cache_lookup(sig, &q, &o, &l)) {
      double best = 1e300;
      hipEvent_t e0, e1;
      HCG_HIP(hipEventCreate(&e0));
      HCG_HIP(hipEventCreate(&e1));
      for (int k = 0; k < ncfg; ++k) {
        st = build_items(b, data, cfg[k][0], cfg[k][1], cfg[k][2], stream);
        if (st != HCG_OK) return st;
        b->qw = cfg[k][0];
        b->strategy = cfg[k][2];
        HCG_HIP(hipEventRecord(e0, stream));
        st = launch_direct(b, stream);
        if (st != HCG_OK) return st;
        HCG_HIP(hipEventRecord(e1, stream));
        HCG_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        HCG_HIP(hipEventElapsedTime(&ms, e0, e1));
        // slot: strategy * 4 + (order ? 0 : 2) + (qw - 1)
        b->tune_ms[cfg[k][2] * 4 + (cfg[k][1] ? 0 : 2) + (cfg[k][0] - 1)] = ms;
        if (ms < best) { best = ms; q = cfg[k][0]; o = cfg[k][1]; l = cfg[k][2]; }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      tune_cache_store(sig, q, o, l);
    }
    b->qw = q;
    b->cost_order = o;
    b->strategy = l;
    b->tuned = true;
  }
  const bool rebuilt = b->built_qw != b->qw || b->built_order != b->cost_order ||
                       b->built_strategy != b->strategy;
  if (rebuilt) {
    st = build_items(b, data, b->qw, b->cost_order, b->strategy, stream);
    if (st != HCG_OK) return st;
  }
  // the graph holds one launch per class with items: capture again when the
  // set of classes, their narrow/wide kernels or the slab width changed
  if (!b->exec || b->graph_qw != b->qw || rebuilt) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    if (!b->cap_stream) HCG_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HCG_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    st = launch_direct(b, b->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->cap_stream, &g);
    if (st != HCG_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (ec != hipSuccess) return fail(HCG_E_DEVICE, "hcg_grid_batch: graph capture failed: %s", hipGetErrorString(ec));
    b->graph = g;
    HCG_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_qw = b->qw;
  }
  HCG_HIP(hipGraphLaunch(b->exec, stream));
  HCG_HIP(hipEventRecord(b->done, stream));
  b->launched = true;
  return HCG_OK;
}

extern "C" hcg_status hcg_destroy_batch(hcg_batch_t batch) {
  if (!batch) return HCG_OK;
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto it = std::find(g_batches.begin(), g_batches.end(), batch);
    if (it == g_batches.end() || batch->magic != kBatchMagic)
      return fail(HCG_E_STATE, "hcg_destroy_batch: not a live batch");
    g_batches.erase(it);
  }
  const hipError_t e = hipDeviceSynchronize();
  free_batch(batch);
  if (e != hipSuccess) return fail(HCG_E_DEVICE, "hcg_destroy_batch: %s", hipGetErrorString(e));
  return HCG_OK;
}

extern "C" hcg_status hcg_get_batch_info(hcg_batch_t batch, hcg_batch_info* info) {
  if (!batch || !info) return fail(HCG_E_ARG, "hcg_get_batch_info: NULL pointer");
  if (!batch_is_live(batch)) return fail(HCG_E_STATE, "hcg_get_batch_info: not a live batch");
  info->nfields = (int32_t)batch->plans.size();
  info->chan_slab = 256 * batch->qw;
  info->cost_order = batch->cost_order;
  info->tuned = batch->tuned ? 1 : 0;
  info->graph_captured = batch->exec ? 1 : 0;
  int64_t items = 0;
  for (int c = 0; c < kClasses; ++c) items += batch->nitems[c];
  info->items = items;
  info->persistent_blocks = batch->nblocks;
  info->launch = batch->strategy;
  for (int k = 0; k < 8; ++k) info->tune_ms[k] = batch->tune_ms[k];
  return HCG_OK;
}

extern "C" hcg_status hcg_batch_get_plan(hcg_batch_t batch, int32_t field, hcg_plan_t* out) {
  if (!batch || !out) return fail(HCG_E_ARG, "hcg_batch_get_plan: NULL pointer");
  *out = nullptr;
  if (!batch_is_live(batch)) return fail(HCG_E_STATE, "hcg_batch_get_plan: not a live batch");
  if (field < 0 || field >= (int32_t)batch->plans.size())
    return fail(HCG_E_ARG, "hcg_batch_get_plan: field %d out of range", field);
  *out = batch->plans[field];
  return HCG_OK;
}
