// Continuous-batching server for CoNet-Rx slot requests.
//
// Requests (one TTI each, any PRB allocation, 2..N_rx antennas, any modulation up to the
// model's head width) are queued by conet_serve_submit. Each lane (a HIP stream with its
// own buffers) has a thread that forms a ragged batch whenever the lane is free: it takes
// queued requests in arrival order while their REs fit the lane's buffers (admission by
// memory; a request never waits for a batch to fill), and enqueues H2D copies -> ragged
// forward -> D2H copies on the lane's stream. Lanes run on separate streams, so a batch
// formed while others are on the GPU overlaps with them on the device. The same thread
// then waits for its batch, moves the LLRs to the callers' buffers where the copy engines
// could not, and releases the waiters.
//
// A request may carry the received grid instead of the features: the grid (8 bytes per RE
// and antenna instead of 16) is copied, and the lane forms the features on the GPU
// (conet_featurise) before the forward. Inputs in page-locked caller memory that need no
// reshaping (grids, and features with all C_in channels) are copied by DMA straight from
// the caller's buffer; the rest are first packed into the lane's pinned staging buffer
// (zero-padding missing antennas). On the way out, a request whose modulation uses fewer
// bits than the head's width has its LLR channels packed on the GPU, and the LLRs go by
// DMA to the caller's buffer when it is page-locked, else to pinned staging followed by a
// host copy. Host copies are on the critical path of every request that needs them; a
// small pool of helper threads splits each over the batch.
//
// Every slot is computed in tiles that never cross slot boundaries and each kernel's
// arithmetic per RE does not depend on the other slots, so a request's LLRs are
// identical whether it runs alone or inside any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "conet.h"
#include "conet_model.h"

namespace conet {

using clk = std::chrono::steady_clock;

constexpr int SERVE_COPY_HELPERS = 3;  // host copies run on the calling thread + 3 helpers

// LLR channels 0..mq-1 of each of n REs whose LLRs are m apart, written back to back
// (a request whose modulation uses fewer bits than the head's width).
__global__ void __launch_bounds__(256) compact_llr_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                          int64_t n, int m, int mq) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * mq) return;
  const int64_t r = i / mq;
  dst[i] = src[r * m + (i - r * mq)];
}

// Whether [p, p + bytes) lies in one page-locked host allocation (hipHostMalloc), which the
// copy engines read and write directly. A pageable pointer makes the query fail on some
// runtimes; that error is taken back so that it is not reported by a later call.
static bool host_pinned(const void* p, size_t bytes) {
  const char* q = static_cast<const char*>(p);
  hipPointerAttribute_t a0{}, a1{};
  hipError_t e0 = hipPointerGetAttributes(&a0, q);
  hipError_t e1 = e0 == hipSuccess ? hipPointerGetAttributes(&a1, q + bytes - 1) : e0;
  if (e0 != hipSuccess || e1 != hipSuccess) (void)hipGetLastError();
  return e0 == hipSuccess && e1 == hipSuccess && a0.type == hipMemoryTypeHost && a1.type == hipMemoryTypeHost &&
         static_cast<const char*>(a1.devicePointer) - static_cast<const char*>(a0.devicePointer) == (ptrdiff_t)(bytes - 1);
}

// One DMA copy; consecutive pieces that continue each other on both sides merge.
struct CopyRun {
  void* dst;
  const void* src;
  size_t bytes;
};
static void add_copy(std::vector<CopyRun>& v, void* dst, const void* src, size_t bytes) {
  if (!v.empty() && static_cast<char*>(v.back().dst) + v.back().bytes == dst &&
      static_cast<const char*>(v.back().src) + v.back().bytes == src) {
    v.back().bytes += bytes;
    return;
  }
  v.push_back({dst, src, bytes});
}

// Fixed helper threads for the batch's host copies: run(fn) calls fn(part, parts) for
// part 0 on the calling thread and parts 1.. on the helpers, and returns when all are
// done. One job at a time (callers from different threads take turns).
class CopyPool {
 public:
  explicit CopyPool(int helpers) {
    for (int i = 0; i < helpers; ++i) th_.emplace_back([this, i] { loop(i + 1); });
  }
  ~CopyPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  int parts() const { return (int)th_.size() + 1; }
  void run(const std::function<void(int, int)>& fn) {
    std::lock_guard<std::mutex> job(job_mu_);
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &fn;
      pending_ = (int)th_.size();
      ++gen_;
    }
    cv_.notify_all();
    fn(0, parts());
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return pending_ == 0; });
    job_ = nullptr;
  }

 private:
  void loop(int part) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int, int)>* f;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        f = job_;
      }
      (*f)(part, parts());
      std::lock_guard<std::mutex> lk(mu_);
      if (--pending_ == 0) cv_done_.notify_one();
    }
  }
  std::vector<std::thread> th_;
  std::mutex mu_, job_mu_;
  std::condition_variable cv_, cv_done_;
  const std::function<void(int, int)>* job_ = nullptr;
  int pending_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

struct Pending {
  conet_request req;
  uint64_t ticket;
  clk::time_point t_submit;
  int64_t n_re;
  // the input is copied by DMA from the caller's buffer (page-locked, and a grid or features
  // with all C_in channels); the LLRs are copied by DMA to the caller's buffer (page-locked)
  bool x_direct = false, llr_direct = false;
};

struct Done {
  bool done = false;
  conet_status status = CONET_OK;
  double latency_us = 0;
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;         // end of the batch (after the D2H copy)
  hipEvent_t ev_h2d = nullptr, ev_fwd = nullptr, ev_d2h = nullptr;  // starts of the three steps
  uint8_t* dev = nullptr;          // arena + x + llr
  Arena arena;
  float* x_dev = nullptr;          // [max_res][C_in]
  float* llr_dev = nullptr;        // [max_res][m]
  float* llr_c = nullptr;          // LLRs of requests with fewer than m bits, packed at c_off
  float* x_pin = nullptr;          // pinned staging
  float* y_dev = nullptr;          // received grids of the batch's grid requests, packed
  float* y_pin = nullptr;
  std::vector<int64_t> y_off;      // per request of the batch: offset (floats) of its grid in y_pin, or -1
  std::vector<int64_t> c_off;      // per request: offset (floats) of its mq-wide LLRs in llr_c and llr_pin
  std::vector<CopyRun> h2d, d2h;   // the batch's DMA copies
  float* llr_pin = nullptr;
  TileDesc* tiles_pin = nullptr;   // pinned staging of the batch's tile list
  std::vector<Pending> batch;      // requests of the batch in flight
  std::vector<int32_t> F;          // widths of the batch's slots
  clk::time_point t_formed, t_enqueued;  // batch taken from the queue; all its GPU work enqueued
  bool busy = false;               // a batch is assigned to the lane
  bool launched = false;           // ... and its completion event is recorded
  std::thread worker;              // forms, enqueues, waits for and delivers the lane's batches
};

}  // namespace conet

struct conet_server {
  conet_model* M = nullptr;
  int device = 0;
  int64_t lane_res = 0;
  size_t max_queue = 0;
  std::vector<conet::Lane> lanes;
  std::mutex mu;
  std::condition_variable cv_sched;   // the queue grew, or batches may be formed again
  std::condition_variable cv_done;    // a request completed
  std::deque<conet::Pending> queue;
  conet::CopyPool* pool = nullptr;    // helpers for packing and scattering
  std::unordered_map<uint64_t, conet::Done> results;
  uint64_t next_ticket = 1;
  bool stop = false;
  bool paused = false;                // no new batches are formed while set
  // statistics
  std::vector<double> lat_us;
  uint64_t completed = 0, rejected = 0, batches = 0, batched_requests = 0, direct_inputs = 0, direct_outputs = 0;
  int64_t res_done = 0;
  double sum_queue_us = 0, sum_prep_us = 0, sum_device_us = 0, sum_scatter_us = 0;
  double sum_h2d_us = 0, sum_fwd_us = 0, sum_d2h_us = 0;
  double slowest_us = 0, slowest_phase_us[4] = {0, 0, 0, 0};  // the slowest request: queue, prep, device, scatter
  bool have_first = false;
  conet::clk::time_point t_first, t_last;
  conet_status async_error = CONET_OK;
};

namespace conet {

static void launch_batch(conet_server* S, int li, std::unique_lock<std::mutex>& lk);

// One thread per lane: when the lane is free, take a batch from the head of the queue, enqueue
// its work, wait for it and deliver the LLRs. Lanes form their batches independently, so a
// batch whose host work is held up (a thread not scheduled for a while) delays only its lane.
static void lane_loop(conet_server* S, int li) {
  Lane& ln = S->lanes[li];
  (void)hipSetDevice(S->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_sched.wait(lk, [&] { return S->stop || (!S->paused && !S->queue.empty()); });
      if (S->stop) return;
      launch_batch(S, li, lk);  // unlocks while packing and enqueueing; returns with the lock held
      if (!ln.launched) continue;  // the batch failed (its requests are completed with the error)
    }
    hipError_t e = hipEventSynchronize(ln.ev);
    const auto t_done_gpu = clk::now();
    float ms_h2d = 0.f, ms_fwd = 0.f, ms_d2h = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_h2d, ln.ev_h2d, ln.ev_fwd);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_fwd, ln.ev_fwd, ln.ev_d2h);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_d2h, ln.ev_d2h, ln.ev);
    auto us = [](clk::time_point a, clk::time_point b) { return std::chrono::duration<double, std::micro>(b - a).count(); };
    // LLRs that went to pinned staging: request q's n_re * mq floats sit at c_off[q]. Each
    // part copies its share [r0, r1) of those floats, counted over the batch's requests.
    if (e == hipSuccess) {
      int64_t total = 0;
      for (auto& p : ln.batch)
        if (!p.llr_direct) total += p.n_re * p.req.bits_per_symbol;
      if (total > 0)
        S->pool->run([&](int part, int parts) {
          const int64_t r0 = total * part / parts, r1 = total * (part + 1) / parts;
          int64_t off = 0;
          for (size_t q = 0; q < ln.batch.size(); ++q) {
            const Pending& p = ln.batch[q];
            if (p.llr_direct) continue;
            const int64_t n = p.n_re * p.req.bits_per_symbol;
            const int64_t a = std::max(r0, off), b = std::min(r1, off + n);
            if (a < b) memcpy(p.req.llr_host + (a - off), ln.llr_pin + ln.c_off[q] + (a - off), sizeof(float) * (b - a));
            off += n;
          }
        });
    }
    const auto t_done = clk::now();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (auto& p : ln.batch) {
        Done& d = S->results[p.ticket];
        d.done = true;
        d.status = e == hipSuccess ? CONET_OK : CONET_EDEVICE;
        d.latency_us = std::chrono::duration<double, std::micro>(t_done - p.t_submit).count();
        if (e == hipSuccess) {
          S->lat_us.push_back(d.latency_us);
          ++S->completed;
          S->direct_inputs += p.x_direct;
          S->direct_outputs += p.llr_direct;
          S->res_done += p.n_re;
          const double ph[4] = {us(p.t_submit, ln.t_formed), us(ln.t_formed, ln.t_enqueued),
                                us(ln.t_enqueued, t_done_gpu), us(t_done_gpu, t_done)};
          S->sum_queue_us += ph[0];
          S->sum_prep_us += ph[1];
          S->sum_device_us += ph[2];
          S->sum_scatter_us += ph[3];
          if (d.latency_us > S->slowest_us) {
            S->slowest_us = d.latency_us;
            for (int i = 0; i < 4; ++i) S->slowest_phase_us[i] = ph[i];
          }
          S->sum_h2d_us += 1e3 * ms_h2d;
          S->sum_fwd_us += 1e3 * ms_fwd;
          S->sum_d2h_us += 1e3 * ms_d2h;
        }
      }
      if (e != hipSuccess) S->async_error = CONET_EDEVICE;
      S->t_last = t_done;
      ln.batch.clear();
      ln.launched = false;
      ln.busy = false;
    }
    S->cv_done.notify_all();
  }
}

// Form and launch one batch on lane `li` from the head of the queue (called with the lock held).
static void launch_batch(conet_server* S, int li, std::unique_lock<std::mutex>& lk) {
  Lane& ln = S->lanes[li];
  const conet_config& c = S->M->cfg;
  ln.batch.clear();
  ln.F.clear();
  int64_t res = 0;
  while (!S->queue.empty() && res + S->queue.front().n_re <= S->lane_res) {
    res += S->queue.front().n_re;
    ln.batch.push_back(S->queue.front());
    S->queue.pop_front();
  }
  if (ln.batch.empty()) return;
  ln.t_formed = clk::now();
  ln.busy = true;
  ++S->batches;
  S->batched_requests += ln.batch.size();
  lk.unlock();
  // Inputs: a grid goes to its packed place in y (featurised below), features to their REs'
  // rows of x. A page-locked caller buffer that needs no reshaping is the DMA source itself;
  // the others are packed into pinned staging first, each part of the pool copying its share
  // [r0, r1) of the batch's REs (zero-padding antennas beyond the request's).
  const int Ci = c.in_channels, m = c.bits_per_symbol, T = ln.batch[0].req.T;
  const size_t nb = ln.batch.size();
  int64_t y_total = 0;
  bool any_pack = false;
  ln.y_off.clear();
  for (auto& p : ln.batch) {
    ln.F.push_back(12 * p.req.n_prb);
    const bool grid = p.req.input == CONET_INPUT_GRID;
    ln.y_off.push_back(grid ? y_total : -1);
    if (grid) y_total += p.n_re * 2 * p.req.n_rx;
    any_pack |= !p.x_direct;
  }
  if (any_pack)
    S->pool->run([&](int part, int parts) {
      const int64_t r0 = res * part / parts, r1 = res * (part + 1) / parts;
      int64_t off = 0;
      for (size_t q = 0; q < nb; ++q) {
        const Pending& p = ln.batch[q];
        const int64_t a = std::max(r0, off), b = std::min(r1, off + p.n_re);
        off += p.n_re;
        if (a >= b || p.x_direct) continue;
        const int64_t o = off - p.n_re;
        if (ln.y_off[q] >= 0) {
          const int yc = 2 * p.req.n_rx;
          memcpy(ln.y_pin + ln.y_off[q] + (a - o) * yc, p.req.x_host + (a - o) * yc, sizeof(float) * (b - a) * yc);
          continue;
        }
        const int ci = 4 * p.req.n_rx;
        float* dst = ln.x_pin + a * Ci;
        const float* src = p.req.x_host + (a - o) * ci;
        if (ci == Ci) {
          memcpy(dst, src, sizeof(float) * (b - a) * Ci);
        } else {
          for (int64_t r = 0; r < b - a; ++r) {
            memcpy(dst + r * Ci, src + r * ci, sizeof(float) * ci);
            memset(dst + r * Ci + ci, 0, sizeof(float) * (Ci - ci));
          }
        }
      }
    });
  ln.h2d.clear();
  {
    int64_t off = 0;
    for (size_t q = 0; q < nb; ++q) {
      const Pending& p = ln.batch[q];
      const bool direct = p.x_direct;
      if (ln.y_off[q] >= 0)
        add_copy(ln.h2d, ln.y_dev + ln.y_off[q], direct ? p.req.x_host : ln.y_pin + ln.y_off[q],
                 sizeof(float) * p.n_re * 2 * p.req.n_rx);
      else
        add_copy(ln.h2d, ln.x_dev + off * Ci, direct ? p.req.x_host : ln.x_pin + off * Ci, sizeof(float) * p.n_re * Ci);
      off += p.n_re;
    }
  }
  hipError_t e = hipEventRecord(ln.ev_h2d, ln.stream);
  for (const CopyRun& r : ln.h2d)
    if (e == hipSuccess) e = hipMemcpyAsync(r.dst, r.src, r.bytes, hipMemcpyHostToDevice, ln.stream);
  if (e == hipSuccess) e = hipEventRecord(ln.ev_fwd, ln.stream);
  conet_status st = e == hipSuccess ? CONET_OK : hip_fail(e, "serving H2D");
  {  // features of the grid requests, written where the forward reads them
    int64_t off = 0;
    for (size_t q = 0; q < nb && st == CONET_OK; ++q) {
      const Pending& p = ln.batch[q];
      if (ln.y_off[q] >= 0)
        st = conet_featurise(ln.y_dev + ln.y_off[q], 1, T, 12 * p.req.n_prb, p.req.n_rx, Ci, ln.x_dev + off * Ci,
                             ln.stream);
      off += p.n_re;
    }
  }
  if (st == CONET_OK) {
    Geometry geo;
    geo.uniform = false;
    geo.T = T;
    geo.n_slots = (int)ln.F.size();
    geo.F_host = ln.F.data();
    geo.tiles_pin = ln.tiles_pin;
    geo.tiles_pin_cap = ln.arena.max_tiles;
    st = run_forward(S->M, ln.arena, ln.x_dev, geo, ln.llr_dev, ln.stream, nullptr);
  }
  // Outputs: request q's LLRs, mq = its bits per symbol of the head's m per RE, packed on
  // the GPU when mq < m, then copied to its buffer (page-locked) or to pinned staging at
  // the same packed offset c_off[q].
  if (st == CONET_OK) {
    ln.c_off.clear();
    ln.d2h.clear();
    int64_t off = 0, coff = 0;
    for (size_t q = 0; q < nb && e == hipSuccess; ++q) {
      const Pending& p = ln.batch[q];
      const int mq = p.req.bits_per_symbol;
      const float* src = ln.llr_dev + off * m;
      if (mq != m) {
        const int64_t n = p.n_re * mq;
        hipLaunchKernelGGL(compact_llr_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ln.stream, src,
                           ln.llr_c + coff, p.n_re, m, mq);
        e = hipGetLastError();
        src = ln.llr_c + coff;
      }
      add_copy(ln.d2h, p.llr_direct ? p.req.llr_host : ln.llr_pin + coff, src, sizeof(float) * p.n_re * mq);
      ln.c_off.push_back(coff);
      off += p.n_re;
      coff += p.n_re * mq;
    }
    if (e == hipSuccess) e = hipEventRecord(ln.ev_d2h, ln.stream);
    for (const CopyRun& r : ln.d2h)
      if (e == hipSuccess) e = hipMemcpyAsync(r.dst, r.src, r.bytes, hipMemcpyDeviceToHost, ln.stream);
    if (e == hipSuccess) e = hipEventRecord(ln.ev, ln.stream);
    if (e != hipSuccess) st = hip_fail(e, "serving D2H");
  }
  ln.t_enqueued = clk::now();
  if (st != CONET_OK) {
    // Part of the batch may already be enqueued (copies out of callers' page-locked inputs or
    // the lane's pinned staging, copies into callers' LLR buffers). Drain the stream before the
    // requests complete and the staging is reused; the batch fails whatever this returns.
    (void)hipStreamSynchronize(ln.stream);
  }
  lk.lock();
  if (st != CONET_OK) {  // fail the whole batch; the lane stays usable
    for (auto& p : ln.batch) {
      Done& d = S->results[p.ticket];
      d.done = true;
      d.status = st;
    }
    ln.batch.clear();
    ln.busy = false;
    S->cv_done.notify_all();
    return;
  }
  ln.launched = true;
}

// grid staging: at most C_in / 4 antennas of (Re, Im) per RE
static size_t grid_floats(const conet_config& c, int64_t res) { return (size_t)res * (c.in_channels / 4) * 2; }

static size_t lane_bytes(const conet_config& c, int64_t res) {
  auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return a256(arena_bytes(c, res)) + a256(sizeof(float) * res * c.in_channels) +
         2 * a256(sizeof(float) * res * c.bits_per_symbol) + a256(sizeof(float) * grid_floats(c, res));
}

}  // namespace conet

using namespace conet;

extern "C" {

conet_status conet_serve_create(conet_model* M, size_t mem_budget_bytes, int32_t n_streams, int32_t max_batch_res,
                                 int32_t max_queue, conet_server** out) {
  if (!M || !out) return fail(CONET_EINVAL, "null argument");
  *out = nullptr;
  if (n_streams < 1 || n_streams > 16) return fail(CONET_EINVAL, "n_streams must be 1..16");
  if (max_batch_res < 1 || max_queue < 1) return fail(CONET_EINVAL, "max_batch_res and max_queue must be positive");
  const conet_config& c = M->cfg;
  if (c.dtype == DT_FP8 && !M->scales_set) return fail(CONET_ESTATE, "FP8 model needs activation scales");
  if (c.train && c.norm == CONET_NORM_BN)  // batch statistics would couple the requests of a batch
    return fail(CONET_EINVAL, "a BatchNorm model in training normalises by batch statistics: serve a model created "
                              "from its weights with train = 0");
  // admission by memory: every lane holds buffers for lane_res REs within the budget
  int64_t lane_res = max_batch_res;
  while (lane_res > 1 && (size_t)n_streams * lane_bytes(c, lane_res) > mem_budget_bytes) lane_res /= 2;
  if ((size_t)n_streams * lane_bytes(c, lane_res) > mem_budget_bytes)
    return fail(CONET_ENOMEM, "memory budget %zu bytes cannot hold %d lanes", mem_budget_bytes, n_streams);
  conet_server* S = new (std::nothrow) conet_server();
  if (!S) return fail(CONET_ENOMEM, "host allocation failed");
  S->M = M;
  S->device = M->device;
  S->lane_res = lane_res;
  S->max_queue = (size_t)max_queue;
  S->lanes.resize(n_streams);
  hipError_t e = hipSetDevice(M->device);
  for (auto& ln : S->lanes) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&ln.ev);
    if (e == hipSuccess) e = hipEventCreate(&ln.ev_h2d);
    if (e == hipSuccess) e = hipEventCreate(&ln.ev_fwd);
    if (e == hipSuccess) e = hipEventCreate(&ln.ev_d2h);
    if (e == hipSuccess) e = hipMalloc(&ln.dev, lane_bytes(c, lane_res));
    if (e == hipSuccess) e = hipHostMalloc(&ln.x_pin, sizeof(float) * lane_res * c.in_channels, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&ln.llr_pin, sizeof(float) * lane_res * c.bits_per_symbol, hipHostMallocDefault);
    if (e != hipSuccess) break;
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    arena_carve(c, lane_res, ln.dev, ln.arena);
    e = hipHostMalloc(&ln.tiles_pin, sizeof(TileDesc) * ln.arena.max_tiles, hipHostMallocDefault);
    if (e != hipSuccess) break;
    ln.x_dev = reinterpret_cast<float*>(ln.dev + a256(arena_bytes(c, lane_res)));
    ln.llr_dev = reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(ln.x_dev) + a256(sizeof(float) * lane_res * c.in_channels));
    ln.llr_c = reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(ln.llr_dev) + a256(sizeof(float) * lane_res * c.bits_per_symbol));
    ln.y_dev = reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(ln.llr_c) + a256(sizeof(float) * lane_res * c.bits_per_symbol));
    e = hipHostMalloc(&ln.y_pin, sizeof(float) * grid_floats(c, lane_res), hipHostMallocDefault);
    if (e != hipSuccess) break;
  }
  if (e != hipSuccess) {
    conet_status st = hip_fail(e, "serving lane set-up");
    for (auto& ln : S->lanes) {
      if (ln.stream) (void)hipStreamDestroy(ln.stream);
      for (hipEvent_t v : {ln.ev, ln.ev_h2d, ln.ev_fwd, ln.ev_d2h})
        if (v) (void)hipEventDestroy(v);
      if (ln.dev) (void)hipFree(ln.dev);
      if (ln.x_pin) (void)hipHostFree(ln.x_pin);
      if (ln.llr_pin) (void)hipHostFree(ln.llr_pin);
      if (ln.tiles_pin) (void)hipHostFree(ln.tiles_pin);
      if (ln.y_pin) (void)hipHostFree(ln.y_pin);
    }
    delete S;
    return st;
  }
  S->pool = new CopyPool(SERVE_COPY_HELPERS);
  for (int i = 0; i < n_streams; ++i) S->lanes[i].worker = std::thread(lane_loop, S, i);
  *out = S;
  return CONET_OK;
}

conet_status conet_serve_submit(conet_server* S, const conet_request* r, uint64_t* ticket) {
  if (!S || !r || !ticket) return fail(CONET_EINVAL, "null argument");
  const conet_config& c = S->M->cfg;
  if (!r->x_host || !r->llr_host) return fail(CONET_EINVAL, "null request buffer");
  if (r->T < 1 || r->T > TMAX || r->n_prb < 1 || r->n_rx < 1 || 4 * r->n_rx > c.in_channels ||
      r->bits_per_symbol < 1 || r->bits_per_symbol > c.bits_per_symbol)
    return fail(CONET_ESHAPE, "request does not fit the model (T=%d n_prb=%d n_rx=%d m=%d)", r->T, r->n_prb, r->n_rx,
                r->bits_per_symbol);
  if (r->input != CONET_INPUT_FEATURES && r->input != CONET_INPUT_GRID)
    return fail(CONET_EINVAL, "input must be CONET_INPUT_FEATURES or CONET_INPUT_GRID");
  if (r->input == CONET_INPUT_GRID && r->T < 12)
    return fail(CONET_ESHAPE, "a grid request needs T >= 12 (pilots on symbols 2 and 11)");
  const int64_t n_re = (int64_t)r->T * 12 * r->n_prb;
  const size_t in_floats = (size_t)n_re * (r->input == CONET_INPUT_GRID ? 2 : 4) * r->n_rx;
  const bool x_direct = (r->input == CONET_INPUT_GRID || 4 * r->n_rx == c.in_channels) &&
                        host_pinned(r->x_host, sizeof(float) * in_floats);
  const bool llr_direct = host_pinned(r->llr_host, sizeof(float) * n_re * r->bits_per_symbol);
  std::lock_guard<std::mutex> lk(S->mu);
  if (n_re > S->lane_res) {
    ++S->rejected;
    return fail(CONET_ESHAPE, "request of %lld REs exceeds a lane's %lld", (long long)n_re, (long long)S->lane_res);
  }
  if (S->queue.size() >= S->max_queue) {
    ++S->rejected;
    return fail(CONET_EBUSY, "queue full (%zu requests)", S->max_queue);
  }
  if (!S->queue.empty() && S->queue.front().req.T != r->T)
    return fail(CONET_ESHAPE, "all queued requests must share T");
  Pending p;
  p.req = *r;
  p.ticket = S->next_ticket++;
  p.t_submit = clk::now();
  p.n_re = n_re;
  p.x_direct = x_direct;
  p.llr_direct = llr_direct;
  if (!S->have_first) { S->have_first = true; S->t_first = p.t_submit; }
  S->results[p.ticket] = Done();
  S->queue.push_back(p);
  *ticket = p.ticket;
  S->cv_sched.notify_one();
  return CONET_OK;
}

conet_status conet_serve_wait(conet_server* S, uint64_t ticket, int64_t timeout_us, double* latency_us) {
  if (!S) return fail(CONET_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->results.find(ticket);
  if (it == S->results.end()) return fail(CONET_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  auto ready = [&] { return S->results[ticket].done; };
  if (timeout_us < 0) {
    S->cv_done.wait(lk, ready);
  } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return fail(CONET_ETIMEOUT, "ticket %llu not done after %lld us", (unsigned long long)ticket, (long long)timeout_us);
  }
  Done d = S->results[ticket];
  S->results.erase(ticket);
  if (latency_us) *latency_us = d.latency_us;
  if (d.status != CONET_OK) return fail(d.status, "request %llu failed on the device", (unsigned long long)ticket);
  return CONET_OK;
}

conet_status conet_serve_get_stats(conet_server* S, conet_serve_stats* st) {
  if (!S || !st) return fail(CONET_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  std::vector<double> v = S->lat_us;
  memset(st, 0, sizeof(*st));
  st->completed = S->completed;
  st->rejected = S->rejected;
  st->batches = S->batches;
  st->mean_batch_requests = S->batches ? (double)S->batched_requests / S->batches : 0.0;
  st->lane_res = S->lane_res;
  st->direct_inputs = S->direct_inputs;
  st->direct_outputs = S->direct_outputs;
  st->slowest_queue_us = S->slowest_phase_us[0];
  st->slowest_prep_us = S->slowest_phase_us[1];
  st->slowest_device_us = S->slowest_phase_us[2];
  st->slowest_scatter_us = S->slowest_phase_us[3];
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto q = [&](double f) { return v[std::min(v.size() - 1, (size_t)(f * (v.size() - 1) + 0.5))]; };
    st->p50_us = q(0.50);
    st->p99_us = q(0.99);
    st->max_us = v.back();
    double s = 0;
    for (double x : v) s += x;
    st->mean_us = s / v.size();
    const double span = std::chrono::duration<double>(S->t_last - S->t_first).count();
    st->res_per_s = span > 0 ? S->res_done / span : 0.0;
    const double n = (double)S->completed;
    st->mean_queue_us = S->sum_queue_us / n;
    st->mean_prep_us = S->sum_prep_us / n;
    st->mean_device_us = S->sum_device_us / n;
    st->mean_scatter_us = S->sum_scatter_us / n;
    st->mean_h2d_us = S->sum_h2d_us / n;
    st->mean_forward_us = S->sum_fwd_us / n;
    st->mean_d2h_us = S->sum_d2h_us / n;
  }
  return S->async_error;
}

conet_status conet_serve_reset_stats(conet_server* S) {
  if (!S) return fail(CONET_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  S->lat_us.clear();
  S->completed = S->rejected = S->batches = S->batched_requests = 0;
  S->direct_inputs = S->direct_outputs = 0;
  S->slowest_us = 0;
  for (double& v : S->slowest_phase_us) v = 0;
  S->res_done = 0;
  S->sum_queue_us = S->sum_prep_us = S->sum_device_us = S->sum_scatter_us = 0;
  S->sum_h2d_us = S->sum_fwd_us = S->sum_d2h_us = 0;
  S->have_first = false;
  return CONET_OK;
}

conet_status conet_serve_pause(conet_server* S, int32_t paused) {
  if (!S) return fail(CONET_EINVAL, "null server");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->paused = paused != 0;
  }
  S->cv_sched.notify_all();
  return CONET_OK;
}

conet_status conet_serve_destroy(conet_server* S) {
  if (!S) return fail(CONET_EINVAL, "null server");
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->paused = false;
    S->cv_sched.notify_all();
    // let queued and in-flight batches finish
    S->cv_done.wait(lk, [&] {
      if (!S->queue.empty()) return false;
      for (auto& ln : S->lanes) if (ln.busy) return false;
      return true;
    });
    S->stop = true;
  }
  S->cv_sched.notify_all();
  for (auto& ln : S->lanes) if (ln.worker.joinable()) ln.worker.join();
  for (auto& ln : S->lanes) {
    (void)hipStreamSynchronize(ln.stream);
    (void)hipStreamDestroy(ln.stream);
    for (hipEvent_t v : {ln.ev, ln.ev_h2d, ln.ev_fwd, ln.ev_d2h}) (void)hipEventDestroy(v);
    (void)hipFree(ln.dev);
    (void)hipHostFree(ln.x_pin);
    (void)hipHostFree(ln.llr_pin);
    (void)hipHostFree(ln.tiles_pin);
    (void)hipHostFree(ln.y_pin);
  }
  delete S->pool;
  delete S;
  return CONET_OK;
}

}  // extern "C"
