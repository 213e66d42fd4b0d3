// Batches of independent maps in one persistent launch.
//
// hcg_plan_batch builds one plan per field (same device steps as hcg_plan).
// hcg_grid_batch makes every (field, tile, channel slab) a work item: the
// fields' item ranges are concatenated in a chosen field order (by estimated
// cost, candidates x channels, largest first, or as given) and the kernel
// decodes an item index through a small per-field segment table.  One launch
// of a persistent kernel runs them all; its workgroups pop items from per-XCD
// counters over contiguous eighths of the item space and steal from the
// other eighths at the end.  The counter reset and the launch are captured
// once in a hipGraph and replayed; the argument and segment tables live in
// device memory and are rewritten before a replay when pointers or channel
// counts change.  On the first call an autotuner times the channel slab (256
// or 512 channels) and the field order and keeps the fastest; the choice can
// be cached on disk (HCG_TUNE_CACHE=<file>).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hcg_internal.h"

using namespace hcg;

namespace {
constexpr uint64_t kBatchMagic = 0x48434742'41544331ull;  // "HCGBATC1"
}

struct hcg_batch_s {
  uint64_t magic = kBatchMagic;
  int device = 0;
  int nblocks = 0;
  std::vector<hcg_plan_t> plans;
  std::vector<std::vector<uint32_t>> ncand;  // per field, per tile
  hcg_opts opts{};
  GatherArgs* d_fields = nullptr;  // [nfields]
  BatchSeg* d_segs = nullptr;  // [nfields]
  uint32_t* d_ctl = nullptr;   // kBatchCtl words
  std::vector<GatherArgs> h_fields;
  std::vector<int64_t> built_C;
  std::vector<int> built_vec;
  int built_qw = 0, built_order = -1;
  uint32_t nitems = 0;
  int qw = 0, cost_order = 1;
  bool tuned = false;
  double tune_ms[4] = {0, 0, 0, 0};
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
  for (hcg_plan_t p : b->plans) (void)hcg_destroy(p);
  b->magic = 0;
  delete b;
}

// Item segments for slab width 256 * qw (256 for fields whose rows cannot be
// read four elements at a time; one item per tile for C <= 8).
hcg_status build_items(hcg_batch_s* b, const hcg_field_data* data, int qw, int cost_order,
                       hipStream_t stream) {
  const size_t nf = b->plans.size();
  std::vector<double> cost(nf);
  std::vector<BatchSeg> seg(nf);
  for (size_t f = 0; f < nf; ++f) {
    const int64_t C = data[f].nchan;
    const int64_t width = (C <= 8) ? C : (b->built_vec[f] ? 256 * qw : 256);
    const int64_t slabs = (C <= 8) ? 1 : (C + width - 1) / width;
    const std::vector<uint32_t>& nc = b->ncand[f];
    double cand = 0.0;
    for (uint32_t v : nc) cand += v;
    // candidates x channels, plus the output writes
    cost[f] = cand * (C <= 8 ? 8.0 : (double)std::max<int64_t>(C, 64)) +
              64.0 * (double)nc.size() * (double)C;
    seg[f] = BatchSeg{0u, (uint32_t)nc.size(), (uint32_t)slabs, (uint32_t)f};
  }
  std::vector<size_t> order(nf);
  for (size_t f = 0; f < nf; ++f) order[f] = f;
  if (cost_order)
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return cost[x] > cost[y]; });
  std::vector<BatchSeg> host(nf);
  uint64_t base = 0;
  for (size_t k = 0; k < nf; ++k) {
    host[k] = seg[order[k]];
    host[k].base = (uint32_t)base;
    base += (uint64_t)host[k].ntiles * host[k].slabs;
    if (base >= 0xFFFFFFF0ull) return fail(HCG_E_UNSUPPORTED, "hcg_grid_batch: too many items");
  }
  b->nitems = (uint32_t)base;
  HCG_HIP(hipMemcpyAsync(b->d_segs, host.data(), sizeof(BatchSeg) * nf, hipMemcpyHostToDevice,
                         stream));
  uint32_t ctl[kBatchCtl] = {0};
  ctl[8] = b->nitems;
  ctl[9] = (uint32_t)nf;
  HCG_HIP(hipMemcpyAsync(b->d_ctl, ctl, sizeof(ctl), hipMemcpyHostToDevice, stream));
  HCG_HIP(hipStreamSynchronize(stream));  // the host arrays above go out of scope
  b->built_qw = qw;
  b->built_order = cost_order;
  return HCG_OK;
}

hcg_status launch_direct(hcg_batch_s* b, hipStream_t stream) {
  hcg_status st = launch_batch_reset(b->d_ctl, stream);
  if (st != HCG_OK) return st;
  bool wide = false;
  for (const GatherArgs& f : b->h_fields) wide = wide || !(f.c2R < kNarrowChord2);
  return launch_batch(b->qw, wide, b->d_fields, b->d_segs, b->d_ctl, b->nblocks, stream);
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
  }
  char buf[32];
  snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  return buf;
}

bool tune_cache_lookup(const std::string& sig, int* qw, int* order) {
  const char* path = getenv("HCG_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char s[64];
  int q, o;
  bool found = false;
  while (fscanf(f, "%63s %d %d", s, &q, &o) == 3)
    if (sig == s && (q == 1 || q == 2) && (o == 0 || o == 1)) { *qw = q; *order = o; found = true; }
  fclose(f);
  return found;
}

void tune_cache_store(const std::string& sig, int qw, int order) {
  const char* path = getenv("HCG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d\n", sig.c_str(), qw, order);
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
  if (o.coarsen || o.flags) return fail(HCG_E_UNSUPPORTED, "hcg_plan_batch: coarsen and flags must be 0");
  hcg_status st = check_device_arch();
  if (st != HCG_OK) return st;
  hipStream_t stream = (hipStream_t)hip_stream;
  auto* b = new hcg_batch_s();
  b->opts = o;
  hcg_opts po = o;
  po.chan_tile = 0;
  for (int32_t f = 0; f < nfields; ++f) {
    const hcg_field_desc& d = fields[f];
    hcg_plan_t p = nullptr;
    st = hcg_plan(&p, d.lon_deg, d.lat_deg, d.n, &d.grid, d.fwhm_deg, d.support_deg, &po,
                  hip_stream);
    if (st != HCG_OK) {
      std::string msg = hcg_last_error();
      free_batch(b);
      return fail(st, "hcg_plan_batch: field %d: %s", f, msg.c_str());
    }
    b->plans.push_back(p);
    const size_t nt = (size_t)p->ntx * p->nty;
    b->ncand.emplace_back(nt);
    if (hipMemcpyAsync(b->ncand.back().data(), p->ncand, sizeof(uint32_t) * nt,
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
      free_batch(b);
      return fail(HCG_E_DEVICE, "hcg_plan_batch: reading candidate counts failed");
    }
  }
  int cus = 0;
  if (hipGetDevice(&b->device) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
    free_batch(b);
    return fail(HCG_E_DEVICE, "hcg_plan_batch: device query failed");
  }
  b->nblocks = 2 * cus;  // two 256-thread workgroups per CU
  if (hipMalloc(&b->d_fields, sizeof(GatherArgs) * nfields) != hipSuccess ||
      hipMalloc(&b->d_segs, sizeof(BatchSeg) * nfields) != hipSuccess ||
      hipMalloc(&b->d_ctl, sizeof(uint32_t) * kBatchCtl) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess ||
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
  // the tables below are rewritten on this stream: wait for the last launch,
  // whichever stream it ran on
  if (b->launched) HCG_HIP(hipStreamWaitEvent(stream, b->done, 0));
  // argument table
  bool layout_changed = b->built_C.size() != nf;
  std::vector<GatherArgs> fresh(nf);
  std::vector<int> vecs(nf);
  for (size_t f = 0; f < nf; ++f) {
    const hcg_field_data& d = data[f];
    if (!d.spectra || !d.cube) return fail(HCG_E_ARG, "hcg_grid_batch: field %zu: NULL spectra or cube", f);
    if (d.nchan < 1) return fail(HCG_E_ARG, "hcg_grid_batch: field %zu: nchan must be >= 1", f);
    fresh[f] = make_f32_args(b->plans[f], d.spectra, d.nchan, d.cube, d.weights);
    vecs[f] = (d.nchan % 4 == 0 && (uintptr_t)d.spectra % 16 == 0) ? 1 : 0;
    if (!layout_changed && (b->built_C[f] != d.nchan || b->built_vec[f] != vecs[f]))
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
    for (size_t f = 0; f < nf; ++f) b->built_C[f] = data[f].nchan;
    b->built_qw = 0;  // force a rebuild
  }
  hcg_status st;
  if (!b->tuned) {
    if (b->opts.chan_tile) {
      b->qw = b->opts.chan_tile / 256;
      b->cost_order = 1;
    } else {
      const std::string sig = batch_signature(b, data);
      int q = 0, o = 0;
      if (tune_cache_lookup(sig, &q, &o)) {
        b->qw = q;
        b->cost_order = o;
      } else {
        const int cfg[4][2] = {{1, 1}, {2, 1}, {1, 0}, {2, 0}};
        double best = 1e300;
        hipEvent_t e0, e1;
        HCG_HIP(hipEventCreate(&e0));
        HCG_HIP(hipEventCreate(&e1));
        for (int k = 0; k < 4; ++k) {
          st = build_items(b, data, cfg[k][0], cfg[k][1], stream);
          if (st != HCG_OK) return st;
          b->qw = cfg[k][0];
          HCG_HIP(hipEventRecord(e0, stream));
          st = launch_direct(b, stream);
          if (st != HCG_OK) return st;
          HCG_HIP(hipEventRecord(e1, stream));
          HCG_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          HCG_HIP(hipEventElapsedTime(&ms, e0, e1));
          b->tune_ms[k] = ms;
          if (ms < best) { best = ms; q = cfg[k][0]; o = cfg[k][1]; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->qw = q;
        b->cost_order = o;
        tune_cache_store(sig, q, o);
      }
    }
    b->tuned = true;
  }
  if (b->built_qw != b->qw || b->built_order != b->cost_order) {
    st = build_items(b, data, b->qw, b->cost_order, stream);
    if (st != HCG_OK) return st;
  }
  if (!b->exec || b->graph_qw != b->qw) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
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
  info->items = batch->nitems;
  info->persistent_blocks = batch->nblocks;
  for (int k = 0; k < 4; ++k) info->tune_ms[k] = batch->tune_ms[k];
  return HCG_OK;
}
