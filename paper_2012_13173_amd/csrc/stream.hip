// Out-of-core gridding: spectra and cube in host memory, streamed through the
// device one channel slab at a time (the CUDA-streams overlap of copy and
// compute that Section 5 names as future work, for cubes larger than HBM).
//
// One plan serves every slab.  Three streams overlap the three stages of
// consecutive slabs: the host-to-device copy of slab s + 1, the gather of
// slab s and the device-to-host copy of slab s - 1.  Two device buffers per
// stage (double buffering) and events order them:
//   in[s]   waits until the gather of slab s - 2 has read its buffer;
//   grid[s] waits for in[s] and for the copy-out of slab s - 2;
//   out[s]  waits for grid[s].
// A slab of spectra is a strided host region per storage plane (n rows of
// slab channels, row pitch nchan elements) that becomes a dense
// [planes][n][slab] device buffer, which is what hcg_grid takes; every form
// of hcg_grid streams this way, so spectra stored in a 16- or 8-bit form
// cross the host link in half or a quarter of the FP32 bytes.
//
// Page-locked host memory is copied by the DMA engines directly (one 2-D copy
// per slab in, one copy per slab out).  Pageable memory goes through rings
// of page-locked chunks that the library owns: host threads pack row blocks
// of a slab into a chunk that is then copied in, and unpack the chunks that
// the cube slab is copied out through.  A chunk is refilled only after the
// copy that last used it has completed.
#include <sched.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <stdexcept>
#include <thread>
#include <vector>

#include "forms.h"
#include "hcg_internal.h"

using namespace hcg;

namespace {

// Runs fn(lo, hi) over [0, count) split into one contiguous part per thread;
// the calling thread takes part 0.
class HostPool {
 public:
  explicit HostPool(int nthreads) : n_(std::max(1, nthreads)) {
    for (int i = 1; i < n_; ++i) {
      try {
        th_.emplace_back([this, i] { worker(i); });
      } catch (...) {  // fewer threads than asked: the parts are cut for those started
        n_ = i;
        break;
      }
    }
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> g(m_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  void run(int64_t count, const std::function<void(int64_t, int64_t)>& fn) {
    if (n_ == 1 || count < 2 * n_) {
      fn(0, count);
      return;
    }
    {
      std::lock_guard<std::mutex> g(m_);
      fn_ = &fn;
      count_ = count;
      pending_ = n_ - 1;
      ++gen_;
    }
    cv_.notify_all();
    part(0, fn, count);
    std::unique_lock<std::mutex> g(m_);
    done_.wait(g, [this] { return pending_ == 0; });
    fn_ = nullptr;
  }

 private:
  void part(int i, const std::function<void(int64_t, int64_t)>& fn, int64_t count) {
    const int64_t lo = count * i / n_, hi = count * (i + 1) / n_;
    if (hi > lo) fn(lo, hi);
  }
  void worker(int i) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int64_t, int64_t)>* fn;
      int64_t count;
      {
        std::unique_lock<std::mutex> g(m_);
        cv_.wait(g, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        fn = fn_;
        count = count_;
      }
      part(i, *fn, count);
      {
        std::lock_guard<std::mutex> g(m_);
        if (--pending_ == 0) done_.notify_one();
      }
    }
  }
  int n_;
  std::vector<std::thread> th_;
  std::mutex m_;
  std::condition_variable cv_, done_;
  const std::function<void(int64_t, int64_t)>* fn_ = nullptr;
  int64_t count_ = 0;
  uint64_t gen_ = 0;
  int pending_ = 0;
  bool stop_ = false;
};

int host_threads() {
  cpu_set_t set;
  int n = 8;
  if (sched_getaffinity(0, sizeof(set), &set) == 0) n = CPU_COUNT(&set);
  return std::max(1, std::min(n, 16));
}

// Page-locked staging chunks with the event of the copy that last used each
// and, for the copy-out ring, where its bytes go once that copy is done.
struct Ring {
  static constexpr int kMax = 4;
  int k = 0, next = 0;
  size_t bytes = 0;
  void* buf[kMax] = {};
  hipEvent_t ev[kMax] = {};
  bool busy[kMax] = {};
  char* dst[kMax] = {};
  size_t len[kMax] = {};
};

struct StreamRes {
  hipStream_t s_in = nullptr, s_out = nullptr, s_grid = nullptr;
  bool s_grid_set = false;
  hipEvent_t ev_in[2] = {}, ev_grid[2] = {}, ev_out[2] = {};
  void* dspec[2] = {};
  void* dcube[2] = {};
  float* dw = nullptr;
  float* dscale = nullptr;
  Ring rin, rout;
  ~StreamRes() {
    // no copy or gather may still use the buffers when they go (an error
    // can end the call with work queued)
    if (s_in) (void)hipStreamSynchronize(s_in);
    if (s_grid_set) (void)hipStreamSynchronize(s_grid);
    if (s_out) (void)hipStreamSynchronize(s_out);
    for (Ring* r : {&rin, &rout})
      for (int i = 0; i < r->k; ++i) {
        if (r->ev[i]) (void)hipEventDestroy(r->ev[i]);
        if (r->buf[i]) (void)hipHostFree(r->buf[i]);
      }
    for (int b = 0; b < 2; ++b) {
      if (ev_in[b]) (void)hipEventDestroy(ev_in[b]);
      if (ev_grid[b]) (void)hipEventDestroy(ev_grid[b]);
      if (ev_out[b]) (void)hipEventDestroy(ev_out[b]);
      if (dspec[b]) (void)hipFree(dspec[b]);
      if (dcube[b]) (void)hipFree(dcube[b]);
    }
    if (dw) (void)hipFree(dw);
    if (dscale) (void)hipFree(dscale);
    if (s_in) (void)hipStreamDestroy(s_in);
    if (s_out) (void)hipStreamDestroy(s_out);
  }
};

hcg_status ring_init(Ring& r, int k, size_t bytes) {
  r.k = k;
  r.bytes = bytes;
  for (int i = 0; i < k; ++i) {
    if (hipHostMalloc(&r.buf[i], bytes, hipHostMallocDefault) != hipSuccess) {
      r.buf[i] = nullptr;
      (void)hipGetLastError();
      return fail(HCG_E_NOMEM, "hcg_grid_host: cannot allocate %zu page-locked bytes", bytes);
    }
    HCG_HIP(hipEventCreateWithFlags(&r.ev[i], hipEventDisableTiming));
  }
  return HCG_OK;
}

// Next chunk of the ring, once the copy that last used it has completed (and
// its bytes, for the copy-out ring, have been moved to their destination).
hcg_status ring_acquire(Ring& r, HostPool& pool, int* idx) {
  const int i = r.next;
  r.next = (r.next + 1) % r.k;
  if (r.busy[i]) {
    HCG_HIP(hipEventSynchronize(r.ev[i]));
    if (r.dst[i]) {
      char* d = r.dst[i];
      const char* s = (const char*)r.buf[i];
      pool.run((int64_t)r.len[i], [&](int64_t lo, int64_t hi) { memcpy(d + lo, s + lo, hi - lo); });
      r.dst[i] = nullptr;
    }
    r.busy[i] = false;
  }
  *idx = i;
  return HCG_OK;
}

hcg_status ring_drain(Ring& r, HostPool& pool) {
  for (int j = 0; j < r.k; ++j) {
    int i;
    hcg_status st = ring_acquire(r, pool, &i);
    if (st != HCG_OK) return st;
  }
  return HCG_OK;
}

bool page_locked(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeHost;
}

bool device_memory(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

constexpr size_t kChunkBytes = size_t(64) << 20;

}  // namespace

static hcg_status grid_host(hcg_plan_t plan, const void* spectra_host, int64_t nchan,
                            hcg_dtype dtype, const float* chan_scale, int64_t slab_chan,
                            float* cube_host, float* weights_host, void* hip_stream) {
  if (!plan) return fail(HCG_E_ARG, "hcg_grid_host: plan is NULL");
  if (!plan_is_live(plan)) return fail(HCG_E_STATE, "hcg_grid_host: not a live plan");
  if (!spectra_host || !cube_host) return fail(HCG_E_ARG, "hcg_grid_host: NULL pointer");
  if (nchan < 1) return fail(HCG_E_ARG, "hcg_grid_host: nchan must be >= 1");
  if (slab_chan < 0) return fail(HCG_E_ARG, "hcg_grid_host: slab_chan must be >= 0");
  if ((int)dtype < HCG_F32 || (int)dtype > HCG_FP8E4M3_SPLIT)
    return fail(HCG_E_UNSUPPORTED, "hcg_grid_host: unknown dtype %d", (int)dtype);
  const bool scaled = form_scaled(dtype);
  if (scaled && !chan_scale)
    return fail(HCG_E_ARG, "hcg_grid_host: chan_scale is required for this dtype");
  if (!scaled && chan_scale)
    return fail(HCG_E_ARG, "hcg_grid_host: chan_scale must be NULL for this dtype");
  if (device_memory(spectra_host) || device_memory(cube_host) ||
      (weights_host && device_memory(weights_host)) || (chan_scale && device_memory(chan_scale)))
    return fail(HCG_E_ARG, "hcg_grid_host: a device pointer was given for host memory");
  const hcg_plan_s* p = plan;
  const int64_t n = p->n;
  const int64_t G = (int64_t)p->grid.nx * p->grid.ny;
  const size_t esz = form_elem(dtype);
  const int planes = form_split(dtype) ? 2 : 1;
  // default slab: 512 channels, or fewer so that the double buffers of
  // spectra (all planes) and cube take at most a quarter of the free device
  // memory, rounded down to a multiple of 8 channels (wide rows copy at the
  // link's rate; rows of a few dozen bytes copy at a fraction of it)
  int64_t cs = slab_chan ? slab_chan : 512;
  if (!slab_chan) {
    size_t free_b = 0, total_b = 0;
    HCG_HIP(hipMemGetInfo(&free_b, &total_b));
    const int64_t per_chan = 2 * ((int64_t)esz * planes * n + 4 * G);
    int64_t cap = std::max<int64_t>(1, (int64_t)(free_b / 4) / std::max<int64_t>(per_chan, 1));
    if (cap >= 8) cap -= cap % 8;
    cs = std::min(cs, cap);
  }
  cs = std::min(cs, nchan);
  const int64_t nslab = (nchan + cs - 1) / cs;
  hipStream_t s_grid = (hipStream_t)hip_stream;
  const bool in_direct = page_locked(spectra_host);
  const bool out_direct = page_locked(cube_host) && (!weights_host || page_locked(weights_host));

  StreamRes r;
  r.s_grid = s_grid;
  r.s_grid_set = true;
  HCG_HIP(hipStreamCreateWithFlags(&r.s_in, hipStreamNonBlocking));
  HCG_HIP(hipStreamCreateWithFlags(&r.s_out, hipStreamNonBlocking));
  for (int b = 0; b < 2; ++b) {
    HCG_HIP(hipEventCreateWithFlags(&r.ev_in[b], hipEventDisableTiming));
    HCG_HIP(hipEventCreateWithFlags(&r.ev_grid[b], hipEventDisableTiming));
    HCG_HIP(hipEventCreateWithFlags(&r.ev_out[b], hipEventDisableTiming));
    if (hipMalloc(&r.dspec[b], esz * planes * n * cs) != hipSuccess ||
        hipMalloc(&r.dcube[b], sizeof(float) * G * cs) != hipSuccess) {
      (void)hipGetLastError();
      return fail(HCG_E_NOMEM, "hcg_grid_host: cannot allocate two slabs of %lld channels",
                  (long long)cs);
    }
  }
  if (weights_host && hipMalloc(&r.dw, sizeof(float) * G) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HCG_E_NOMEM, "hcg_grid_host: cannot allocate the weight map");
  }
  if (scaled && hipMalloc((void**)&r.dscale, sizeof(float) * nchan) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HCG_E_NOMEM, "hcg_grid_host: cannot allocate the channel scales");
  }
  // rows per copy-in chunk (at least one row of a slab, of one plane)
  const size_t row_bytes = esz * (size_t)cs;
  const int64_t chunk_rows = (int64_t)std::max<size_t>(1, kChunkBytes / row_bytes);
  hcg_status st = HCG_OK;
  if (!in_direct) st = ring_init(r.rin, 4, (size_t)chunk_rows * row_bytes);
  if (st == HCG_OK && !out_direct) st = ring_init(r.rout, 2, kChunkBytes);
  if (st != HCG_OK) return st;
  HostPool pool((in_direct && out_direct) ? 1 : host_threads());

  // the caller's earlier work on its stream comes first
  HCG_HIP(hipEventRecord(r.ev_grid[1], s_grid));
  HCG_HIP(hipStreamWaitEvent(r.s_in, r.ev_grid[1], 0));
  // all the scales go in once, ahead of the first slab (its event orders
  // them before every gather)
  if (scaled)
    HCG_HIP(hipMemcpyAsync(r.dscale, chan_scale, sizeof(float) * nchan, hipMemcpyHostToDevice,
                           r.s_in));

  auto copy_in = [&](int64_t s) -> hcg_status {
    const int b = (int)(s & 1);
    const int64_t c0 = s * cs, cn = std::min(cs, nchan - c0);
    // the buffer was last read by the gather of slab s - 2
    if (s >= 2) HCG_HIP(hipStreamWaitEvent(r.s_in, r.ev_grid[b], 0));
    // plane pl of the slab: n rows of cn elements at row pitch nchan, into
    // the dense [n][cn] plane pl of the device buffer
    const size_t pitch = esz * (size_t)nchan, width = esz * (size_t)cn;
    for (int pl = 0; pl < planes; ++pl) {
      const char* src = (const char*)spectra_host + esz * ((size_t)pl * n * nchan + c0);
      char* dst = (char*)r.dspec[b] + (size_t)pl * n * width;
      if (in_direct) {
        HCG_HIP(hipMemcpy2DAsync(dst, width, src, pitch, width, n, hipMemcpyHostToDevice,
                                 r.s_in));
        continue;
      }
      const int64_t rows = std::max<int64_t>(1, (int64_t)(r.rin.bytes / width));
      for (int64_t r0 = 0; r0 < n; r0 += rows) {
        const int64_t nr = std::min(rows, n - r0);
        int i;
        hcg_status e = ring_acquire(r.rin, pool, &i);
        if (e != HCG_OK) return e;
        char* stage = (char*)r.rin.buf[i];
        if (cn == nchan) {
          const char* from = src + r0 * pitch;
          pool.run(nr * (int64_t)width, [&](int64_t lo, int64_t hi) {
            memcpy(stage + lo, from + lo, hi - lo);
          });
        } else {
          pool.run(nr, [&](int64_t lo, int64_t hi) {
            for (int64_t q = lo; q < hi; ++q)
              memcpy(stage + q * width, src + (r0 + q) * pitch, width);
          });
        }
        HCG_HIP(hipMemcpyAsync(dst + r0 * width, stage, nr * width, hipMemcpyHostToDevice,
                               r.s_in));
        HCG_HIP(hipEventRecord(r.rin.ev[i], r.s_in));
        r.rin.busy[i] = true;
      }
    }
    HCG_HIP(hipEventRecord(r.ev_in[b], r.s_in));
    return HCG_OK;
  };

  auto out_bytes = [&](char* dst, const char* src, size_t bytes) -> hcg_status {
    if (out_direct) {
      HCG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, r.s_out));
      return HCG_OK;
    }
    for (size_t o = 0; o < bytes; o += r.rout.bytes) {
      const size_t len = std::min(r.rout.bytes, bytes - o);
      int i;
      hcg_status e = ring_acquire(r.rout, pool, &i);
      if (e != HCG_OK) return e;
      HCG_HIP(hipMemcpyAsync(r.rout.buf[i], src + o, len, hipMemcpyDeviceToHost, r.s_out));
      HCG_HIP(hipEventRecord(r.rout.ev[i], r.s_out));
      r.rout.busy[i] = true;
      r.rout.dst[i] = dst + o;
      r.rout.len[i] = len;
    }
    return HCG_OK;
  };

  auto copy_out = [&](int64_t s) -> hcg_status {
    const int b = (int)(s & 1);
    const int64_t c0 = s * cs, cn = std::min(cs, nchan - c0);
    HCG_HIP(hipStreamWaitEvent(r.s_out, r.ev_grid[b], 0));
    // the cube slab is contiguous in [C][ny][nx]
    hcg_status e = out_bytes((char*)(cube_host + c0 * G), (const char*)r.dcube[b],
                             sizeof(float) * cn * G);
    if (e == HCG_OK && s == 0 && weights_host)
      e = out_bytes((char*)weights_host, (const char*)r.dw, sizeof(float) * G);
    if (e != HCG_OK) return e;
    HCG_HIP(hipEventRecord(r.ev_out[b], r.s_out));
    return HCG_OK;
  };

  // slab s is copied in and gridded, then slab s - 1 copied out: the host
  // packs slab s while the gather of slab s - 1 runs
  for (int64_t s = 0; s <= nslab && st == HCG_OK; ++s) {
    if (s < nslab) {
      const int b = (int)(s & 1);
      const int64_t cn = std::min(cs, nchan - s * cs);
      st = copy_in(s);
      if (st != HCG_OK) break;
      HCG_HIP(hipStreamWaitEvent(s_grid, r.ev_in[b], 0));
      if (s >= 2) HCG_HIP(hipStreamWaitEvent(s_grid, r.ev_out[b], 0));
      st = hcg_grid(plan, r.dspec[b], cn, dtype, scaled ? r.dscale + s * cs : nullptr,
                    (float*)r.dcube[b], s == 0 ? r.dw : nullptr, s_grid);
      if (st != HCG_OK) break;
      HCG_HIP(hipEventRecord(r.ev_grid[b], s_grid));
    }
    if (s >= 1) st = copy_out(s - 1);
  }
  // drain every stage before the buffers are freed (also after an error)
  const hipError_t e1 = hipStreamSynchronize(r.s_in);
  const hipError_t e2 = hipStreamSynchronize(s_grid);
  const hipError_t e3 = hipStreamSynchronize(r.s_out);
  if (st != HCG_OK) return st;
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
    return fail(HCG_E_DEVICE, "hcg_grid_host: %s",
                hipGetErrorString(e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3));
  if (!out_direct) return ring_drain(r.rout, pool);
  return HCG_OK;
}

// No C++ exception crosses the C ABI: thread creation and the pool's job
// objects can throw; the streams are drained by the resources' destructors
// before the status is returned.
extern "C" hcg_status hcg_grid_host(hcg_plan_t plan, const void* spectra_host, int64_t nchan,
                                    hcg_dtype dtype, const float* chan_scale, int64_t slab_chan,
                                    float* cube_host, float* weights_host, void* hip_stream) {
  try {
    return grid_host(plan, spectra_host, nchan, dtype, chan_scale, slab_chan, cube_host,
                     weights_host, hip_stream);
  } catch (const std::bad_alloc&) {
    return fail(HCG_E_NOMEM, "hcg_grid_host: out of host memory");
  } catch (const std::exception& e) {
    return fail(HCG_E_DEVICE, "hcg_grid_host: %s", e.what());
  }
}
