// Serving: many resident filter instances, frames batched across instances.
//
// Admission: instance workspaces are carved out of the caller's device arena
// (the HBM budget) with a first-fit allocator; an instance that does not fit
// is refused with LETKF_ENOMEM and can be admitted once others are removed.
//
// Continuous batching: submit_frame copies the slopes into the instance's
// queue and returns.  Instances fall into classes (equal padded ensemble size
// and storage precision); a batch holds the oldest pending frame of several
// instances of one class (at most max_batch), and every domain of every
// instance in it is one work item of the same analysis launch.  Each of the
// kSlots staging slots has its own stream, so batches of different classes
// (or of other instances of the same class) run on the GPU at the same time
// and a light instance never waits behind a heavy one.  A batch is
//   upload {header, slopes} -> slope synthesis -> domain analysis ->
//   merge + forecast -> download of the prediction means
// on its slot's stream.  An instance has at most one frame in flight, which
// keeps its frames in order across streams.
//
// Launch policy (scheduler thread): a class with ready frames is launched
// when every idle instance of the class has a frame (nothing to wait for), or
// when its oldest ready frame has waited window_us for the others; among
// launchable classes the one with the oldest frame goes first.  One
// completion thread per slot waits for its batch, copies the means to the
// callers' buffers and fires the callbacks (which may submit again).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

using namespace letkf;

namespace {

constexpr int kMaxInstances = 64;
constexpr int kSlots = 8;                 // staging slots = concurrent batches (one stream each)
constexpr size_t kStageDoubles = 1 << 18; // slopes per slot and means per slot (each 2 MiB)
constexpr size_t kQueueCap = 64;          // pending frames per instance

using Clock = std::chrono::steady_clock;

struct Frame {
  uint64_t id;
  double* pred_out;
  letkf_done_fn cb;
  void* user;
  std::vector<double> y;       // host slopes (copied at submit), or empty when ydev is set
  const double* ydev;          // caller's device slopes
  Clock::time_point t_enq{};   // submission time (batching window)
};

struct Batch {
  int slot;
  int cls = 0;                 // the class of every instance in the batch
  int grid_cap = 0;            // upper bound on the analysis workgroups (0 = none)
  bool pistons = false;        // some instance of the batch removes differential pistons
  std::vector<std::pair<letkf_handle*, Frame>> frames;
  std::vector<int32_t> out_off;
};

// A replayable launch sequence: class, analysis grid, pistons, and the
// power-of-two buckets of slope rows, domain items and actuator rows that
// size the other grids (their kernels loop over the batch's actual work).
struct GraphKey {
  int cls, grid, pistons, rows_s, items, rows_a;
  bool operator<(const GraphKey& o) const {
    return std::tie(cls, grid, pistons, rows_s, items, rows_a) <
           std::tie(o.cls, o.grid, o.pistons, o.rows_s, o.items, o.rows_a);
  }
};
constexpr size_t kMaxGraphsPerSlot = 32;

int pow2ceil(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}

}  // namespace

struct letkf_server {
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int device = 0;
  int max_batch = kMaxBatch;
  int num_cu = 256;
  int64_t window_us = 100;        // longest wait of a ready frame for the rest of its class
  uint32_t flags = 0;
  int bpc[kNumClasses] = {};       // analysis workgroups of each class one CU holds
  int cls_grid[kNumClasses] = {};  // analysis grid per class (letkf_server_autotune; 0 = bpc x CUs)
  hipStream_t capture = nullptr;   // graph capture (scheduler thread only)
  std::map<GraphKey, hipGraphExec_t> graphs[kSlots];
  hipStream_t stream[kSlots] = {};  // one per staging slot
  hipStream_t upload = nullptr;   // admissions, state access of idle instances
  // arena: [table][hdr x kSlots][y x kSlots][means x kSlots][instance region]
  size_t table_off = 0, hdr_off = 0, y_off = 0, out_off = 0, region_off = 0;
  std::map<size_t, size_t> free_list;  // offset -> bytes (instance region)
  // pinned staging
  BatchHdr* h_hdr[kSlots] = {};
  double* h_y[kSlots] = {};
  double* h_out[kSlots] = {};
  hipEvent_t done_ev[kSlots] = {};
  bool slot_busy[kSlots] = {};     // launched or being launched
  bool slot_has[kSlots] = {};      // slot_batch[k] is waiting for its completion thread
  int slot_cls[kSlots] = {};       // class of the batch last launched on slot k
  Batch slot_batch[kSlots];

  std::mutex mu;
  std::condition_variable cv_work;   // scheduler: new frames / stop
  std::condition_variable cv_slot;   // scheduler: a slot freed
  std::condition_variable cv_done;   // completion thread: new batch; drain: progress
  std::vector<letkf_handle*> inst;   // by table slot (nullptr = free)
  std::map<letkf_handle*, std::deque<Frame>> queues;
  std::map<letkf_handle*, int> in_flight;
  int inflight = 0;                 // batches launched and not yet completed
  int rr = 0;
  bool stop = false;
  // letkf_server_autotune is timing launches on slot 0 (without holding mu):
  // the scheduler launches nothing, submissions queue, and calls that change
  // the instances or read their state return LETKF_EAGAIN
  bool tuning = false;
  uint64_t frames_done = 0, batches = 0, batched_frames = 0, pending = 0;
  std::thread sched, compl_thr[kSlots];

  InstDesc* table() { return (InstDesc*)(arena + table_off); }
  BatchHdr* dhdr(int s) { return (BatchHdr*)(arena + hdr_off) + s; }
  double* dy(int s) { return (double*)(arena + y_off) + (size_t)s * kStageDoubles; }
  double* dout(int s) { return (double*)(arena + out_off) + (size_t)s * 2 * kStageDoubles; }

  void scheduler_loop();
  void completion_loop(int k);
  int launch_batch(Batch& b);
  int graph_for(int slot, const GraphKey& k, hipGraphExec_t* out);
  void drop_graphs();
  // Most analysis workgroups of class c per launch while batches can overlap
  // (more admitted instances than one batch takes, or several classes): a
  // class that fits two or more workgroups on a CU leaves one slot per CU free,
  // so that the slope and merge kernels of the batches beside it start at once
  // instead of waiting for the analysis to drain (measured with 4 BF16 84x84
  // instances in batches of 2: grid 512 against 750 gave +9 % frames/s and a
  // p99 of 0.86 ms against 1.23 ms).  0: no cap.  Caller holds mu.
  int overlap_cap(int c) const {
    if (bpc[c] < 2) return 0;
    int n = 0, cls0 = -1;
    bool classes = false;
    for (letkf_handle* h : inst) {
      if (!h) continue;
      ++n;
      if (cls0 < 0) cls0 = h->cls;
      else if (h->cls != cls0) classes = true;
    }
    return (n > max_batch || classes) ? (bpc[c] - 1) * num_cu : 0;
  }
  // nothing queued, being launched or in flight (caller holds mu)
  bool idle() const {
    if (pending > 0 || inflight > 0) return false;
    for (bool b : slot_busy)
      if (b) return false;
    return true;
  }
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

void letkf_server::drop_graphs() {
  for (auto& cache : graphs) {
    for (auto& kv : cache) (void)hipGraphExecDestroy(kv.second);
    cache.clear();
  }
}

// The kernels of a batch on slot `slot` captured once per key (their
// arguments are the slot's device header and the instance table, whose
// contents change from batch to batch, not their addresses).
int letkf_server::graph_for(int slot, const GraphKey& k, hipGraphExec_t* out) {
  auto& cache = graphs[slot];
  auto it = cache.find(k);
  if (it != cache.end()) { *out = it->second; return LETKF_OK; }
  if (cache.size() >= kMaxGraphsPerSlot) {
    for (auto& kv : cache) (void)hipGraphExecDestroy(kv.second);
    cache.clear();
  }
  hipGraph_t g = nullptr;
  LETKF_HIP(hipStreamBeginCapture(capture, hipStreamCaptureModeThreadLocal));
  launch_slopes(k.cls, k.rows_s, table(), dhdr(slot), capture);
  launch_analysis(k.cls, k.grid, table(), dhdr(slot), capture);
  if (k.pistons) launch_pistons(k.cls, k.items, table(), dhdr(slot), capture);
  launch_rows(k.cls, 2, k.rows_a, table(), dhdr(slot), capture);
  const hipError_t le = hipGetLastError();
  const hipError_t ee = hipStreamEndCapture(capture, &g);
  if (le != hipSuccess || ee != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return fail(LETKF_EDEVICE, "stream capture of a batch failed");
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return fail(LETKF_EDEVICE, "hipGraphInstantiate");
  cache[k] = ex;
  *out = ex;
  return LETKF_OK;
}

int letkf_server::launch_batch(Batch& b) {
  const int s = b.slot, c = b.cls;
  BatchHdr& H = *h_hdr[s];
  std::memset(&H, 0, sizeof(H));
  H.amean = dout(s);
  H.pmean = dout(s) + kStageDoubles;
  H.check_y = 1;  // device slopes are checked by the slope kernel (bad[] uploaded as zeros)
  size_t ytot = 0, otot = 0;
  ClassBatch& cb = H.cls[c];
  for (size_t e = 0; e < b.frames.size(); ++e) {
    letkf_handle* h = b.frames[e].first;
    const Frame& f = b.frames[e].second;
    if (h->cls != c) return fail(LETKF_ESTATE, "batch mixes classes");
    H.out_off[e] = (int32_t)otot;
    if (f.ydev) {
      H.yptr[e] = f.ydev;
    } else {
      H.yptr[e] = dy(s) + ytot;
      std::memcpy(h_y[s] + ytot, f.y.data(), sizeof(double) * h->P.p());
      ytot += h->P.p();
    }
    b.out_off.push_back((int32_t)otot);
    otot += h->P.n_act;
    const int k = cb.n++;
    cb.inst[k] = h->slot;
    cb.ent[k] = (int32_t)e;
    cb.act_off[k + 1] = cb.act_off[k] + h->P.n_act;
    cb.slope_off[k + 1] = cb.slope_off[k] + h->P.p();
    cb.dom_off[k + 1] = cb.dom_off[k] + h->P.n_dom;
  }
  const int rows_s = cb.slope_off[cb.n], rows_a = cb.act_off[cb.n], items = cb.dom_off[cb.n];
  int grid = std::min(items, cls_grid[c] ? cls_grid[c] : bpc[c] * num_cu);
  if (b.grid_cap) grid = std::min(grid, b.grid_cap);
  if (const int cap = overlap_cap(c)) grid = std::min(grid, cap);
  hipStream_t st = stream[s];
  LETKF_HIP(hipMemcpyAsync(dhdr(s), &H, sizeof(H), hipMemcpyHostToDevice, st));
  if (ytot) LETKF_HIP(hipMemcpyAsync(dy(s), h_y[s], ytot * sizeof(double), hipMemcpyHostToDevice, st));
  if (flags & LETKF_SERVER_GRAPHS) {
    const GraphKey key{c, grid, b.pistons ? 1 : 0, pow2ceil(rows_s), pow2ceil(items), pow2ceil(rows_a)};
    hipGraphExec_t ex = nullptr;
    int rc = graph_for(s, key, &ex);
    if (rc) return rc;
    LETKF_HIP(hipGraphLaunch(ex, st));
  } else {
    launch_slopes(c, rows_s, table(), dhdr(s), st);
    launch_analysis(c, grid, table(), dhdr(s), st);
    if (b.pistons) launch_pistons(c, items, table(), dhdr(s), st);
    launch_rows(c, 2, rows_a, table(), dhdr(s), st);
    LETKF_HIP(hipGetLastError());
  }
  LETKF_HIP(hipMemcpyAsync(h_out[s], dout(s) + kStageDoubles, otot * sizeof(double), hipMemcpyDeviceToHost, st));
  // which entries the slope kernel refused (non-finite slopes), into the pinned
  // header, which stays untouched until this slot's completion thread is done
  LETKF_HIP(hipMemcpyAsync(H.bad, dhdr(s)->bad, sizeof(int32_t) * b.frames.size(), hipMemcpyDeviceToHost, st));
  LETKF_HIP(hipEventRecord(done_ev[s], st));
  return LETKF_OK;
}

void letkf_server::scheduler_loop() {
  (void)hipSetDevice(device);  // a failure shows up as an error status of the first batch
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] { return (stop || pending > 0) && !tuning; });
    if (stop && pending == 0) return;
    int s = -1;
    for (int k = 0; k < kSlots; ++k)
      if (!slot_busy[k]) { s = k; break; }
    if (s < 0) {
      cv_slot.wait(lk);
      continue;
    }
    // pick the class to launch
    const auto now = Clock::now();
    const auto window = std::chrono::microseconds(window_us);
    int best = -1;
    Clock::time_point best_t{}, deadline = Clock::time_point::max();
    for (int c = 0; c < kNumClasses; ++c) {
      bool any_ready = false, idle_empty = false;
      Clock::time_point oldest = Clock::time_point::max();
      for (letkf_handle* h : inst) {
        if (!h || h->cls != c || in_flight[h] > 0) continue;
        auto& q = queues[h];
        if (q.empty()) {
          idle_empty = true;
        } else {
          any_ready = true;
          oldest = std::min(oldest, q.front().t_enq);
        }
      }
      if (!any_ready) continue;
      if (stop || !idle_empty || now - oldest >= window) {
        if (best < 0 || oldest < best_t) { best = c; best_t = oldest; }
      } else {
        deadline = std::min(deadline, oldest + window);
      }
    }
    if (best < 0) {
      // frames of in-flight instances wait for a completion; others for their window
      if (deadline == Clock::time_point::max()) cv_work.wait(lk);
      else cv_work.wait_until(lk, deadline);
      continue;
    }
    // The slots' streams share the process's hardware queues in turn (slot k
    // and slot k + kSlots / 2 on one queue, as created), and a queue runs its
    // kernels in order: a batch behind a long one on the same queue waits for
    // it.  Prefer a slot whose queue partner is idle, then one whose partner
    // runs the same class.
    {
      int pick = -1;
      for (int pass = 0; pass < 3 && pick < 0; ++pass)
        for (int k = 0; k < kSlots && pick < 0; ++k) {
          if (slot_busy[k]) continue;
          const int mate = (k + kSlots / 2) % kSlots;
          if (pass == 0 && !slot_busy[mate]) pick = k;
          if (pass == 1 && slot_cls[mate] == best) pick = k;
          if (pass == 2) pick = k;
        }
      s = pick;
    }
    // one frame per ready instance of the class, round robin from rr
    Batch b;
    b.slot = s;
    b.cls = best;
    // m = 128 workgroups fill a CU each (LDS); while instances of other classes
    // are resident, such a batch keeps a quarter of the CUs free for them
    if (best % 4 == 3)
      for (letkf_handle* h : inst)
        if (h && h->cls != best) { b.grid_cap = num_cu * 3 / 4; break; }
    size_t ytot = 0, otot = 0;
    const int n = (int)inst.size();
    for (int t = 0; t < n && (int)b.frames.size() < max_batch; ++t) {
      letkf_handle* h = inst[(rr + t) % n];
      if (!h || h->cls != best || in_flight[h] > 0) continue;
      auto& q = queues[h];
      if (q.empty()) continue;
      if (ytot + h->P.p() > kStageDoubles || otot + h->P.n_act > kStageDoubles) break;
      ytot += h->P.p();
      otot += h->P.n_act;
      b.pistons |= (h->P.flags & LETKF_FLAG_PISTONS) != 0;
      b.frames.emplace_back(h, std::move(q.front()));
      q.pop_front();
      in_flight[h]++;
      --pending;
    }
    rr = (rr + 1) % std::max(n, 1);
    if (b.frames.empty()) continue;
    slot_busy[s] = true;
    slot_cls[s] = best;
    lk.unlock();
    int rc = launch_batch(b);
    lk.lock();
    if (rc) {
      // report the failure through the callbacks of every frame of the batch
      lk.unlock();
      for (auto& [h, f] : b.frames)
        if (f.cb) f.cb(f.user, f.id, rc);
      lk.lock();
      for (auto& [h, f] : b.frames) in_flight[h]--;
      slot_busy[s] = false;
      cv_done.notify_all();
      cv_work.notify_all();
      continue;
    }
    ++batches;
    ++inflight;
    batched_frames += b.frames.size();
    slot_batch[s] = std::move(b);
    slot_has[s] = true;
    cv_done.notify_all();
  }
}

void letkf_server::completion_loop(int k) {
  (void)hipSetDevice(device);  // a failure shows up as an error status of the first batch
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_done.wait(lk, [&] { return stop || slot_has[k]; });
    if (!slot_has[k]) {
      if (stop) return;
      continue;
    }
    Batch b = std::move(slot_batch[k]);
    slot_has[k] = false;
    lk.unlock();
    const hipError_t e = hipEventSynchronize(done_ev[k]);
    const int status = e == hipSuccess ? LETKF_OK : LETKF_EDEVICE;
    // per frame: a frame whose slopes were not finite was refused on the
    // device (its instance's state is unchanged) and reports LETKF_ENUMERIC
    std::vector<int> st(b.frames.size(), status);
    for (size_t i = 0; i < b.frames.size(); ++i) {
      auto& [h, f] = b.frames[i];
      if (status == LETKF_OK && h_hdr[k]->bad[i]) st[i] = LETKF_ENUMERIC;
      if (st[i] == LETKF_OK && f.pred_out)
        std::memcpy(f.pred_out, h_out[k] + b.out_off[i], sizeof(double) * h->P.n_act);
    }
    // callbacks first, then the instances are released: the frames that the
    // callbacks of one batch submit are all queued when the scheduler looks
    // at them again, so closed loops keep full batches
    for (size_t i = 0; i < b.frames.size(); ++i) {
      auto& [h, f] = b.frames[i];
      if (f.cb) f.cb(f.user, f.id, st[i]);
    }
    lk.lock();
    for (auto& [h, f] : b.frames) in_flight[h]--;
    frames_done += b.frames.size();
    --inflight;
    slot_busy[k] = false;
    cv_slot.notify_all();
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

int letkf::server_idle_stream(letkf_handle* h, hipStream_t* stream) {
  letkf_server* s = h->server;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->tuning) return fail(LETKF_EAGAIN, "server autotuning in progress");
    if (!s->queues[h].empty() || s->in_flight[h] > 0) return fail(LETKF_EAGAIN, "instance has frames in flight");
  }
  // the instance's last batch has completed (its completion thread released
  // it), so the admission stream can touch its workspace
  LETKF_HIP(hipStreamSynchronize(s->upload));
  *stream = s->upload;
  return LETKF_OK;
}

extern "C" {

static size_t reserved_layout(size_t* table_off, size_t* hdr_off, size_t* y_off, size_t* out_off) {
  size_t off = 0;
  *table_off = off; off = align256(off + sizeof(InstDesc) * kMaxInstances);
  *hdr_off = off; off = align256(off + sizeof(BatchHdr) * kSlots);
  *y_off = off; off = align256(off + sizeof(double) * kStageDoubles * kSlots);
  *out_off = off; off = align256(off + 2 * sizeof(double) * kStageDoubles * kSlots);
  return off;
}

size_t letkf_server_reserved_bytes(void) {
  size_t a, b, c, d;
  return reserved_layout(&a, &b, &c, &d);
}

int letkf_server_create(void* arena, size_t arena_bytes, int32_t max_batch, uint32_t flags, letkf_server** out) {
  if (!out) return fail(LETKF_EINVAL, "null out");
  *out = nullptr;
  if (!arena || ((uintptr_t)arena & 255)) return fail(LETKF_EINVAL, "arena must be non-null and 256-byte aligned");
  if (max_batch < 1 || max_batch > kMaxBatch) return fail(LETKF_EINVAL, "max_batch must be in [1, 64]");
  if (flags & ~LETKF_SERVER_GRAPHS) return fail(LETKF_EINVAL, "unknown flags");
  auto* s = new letkf_server();
  s->flags = flags;
  s->arena = (char*)arena;
  s->arena_bytes = arena_bytes;
  s->max_batch = max_batch;
  const size_t off = reserved_layout(&s->table_off, &s->hdr_off, &s->y_off, &s->out_off);
  s->region_off = off;
  if (arena_bytes < off + 256) { delete s; return fail(LETKF_ENOMEM, "arena smaller than the server's own tables"); }
  s->free_list[off] = arena_bytes - off;
  s->inst.assign(kMaxInstances, nullptr);
  int rc = LETKF_OK;
  if (hipGetDevice(&s->device) != hipSuccess) rc = fail(LETKF_EDEVICE, "hipGetDevice");
  if (!rc && hipDeviceGetAttribute(&s->num_cu, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess)
    rc = fail(LETKF_EDEVICE, "hipDeviceGetAttribute");
  for (int k = 0; k < kSlots && !rc; ++k)
    if (hipStreamCreateWithFlags(&s->stream[k], hipStreamNonBlocking) != hipSuccess) rc = fail(LETKF_EDEVICE, "stream");
  if (!rc && hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking) != hipSuccess) rc = fail(LETKF_EDEVICE, "stream");
  if (!rc && hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking) != hipSuccess) rc = fail(LETKF_EDEVICE, "stream");
  for (int c = 0; c < kNumClasses && !rc; ++c) s->bpc[c] = analysis_blocks_per_cu(c);
  for (int k = 0; k < kSlots && !rc; ++k) {
    if (hipHostMalloc((void**)&s->h_hdr[k], sizeof(BatchHdr)) != hipSuccess ||
        hipHostMalloc((void**)&s->h_y[k], sizeof(double) * kStageDoubles) != hipSuccess ||
        hipHostMalloc((void**)&s->h_out[k], sizeof(double) * kStageDoubles) != hipSuccess ||
        hipEventCreateWithFlags(&s->done_ev[k], hipEventDisableTiming) != hipSuccess)
      rc = fail(LETKF_EDEVICE, "pinned staging / events");
  }
  if (rc) { letkf_server_destroy(s); return rc; }
  s->sched = std::thread([s] { s->scheduler_loop(); });
  for (int k = 0; k < kSlots; ++k) s->compl_thr[k] = std::thread([s, k] { s->completion_loop(k); });
  *out = s;
  return LETKF_OK;
}

// Whether a validated problem can be served: ensembles of at most 128
// members, and slopes and means that fit one batch's staging slot (a batch
// stages every frame's p slopes and n_act means in slots of kStageDoubles
// values; a larger instance could never be batched).
static int server_admissible(const Problem& P) {
  if (P.m > 128) return fail(LETKF_EINVAL, "m > 128 runs on the plain path only");
  if ((size_t)P.p() > kStageDoubles || (size_t)P.n_act > kStageDoubles)
    return fail(LETKF_EINVAL, "instance too large for the server's staging slots: p and n_act must be <= " +
                                  std::to_string(kStageDoubles));
  return LETKF_OK;
}

int letkf_server_add(letkf_server* s, const letkf_dims* dims, const letkf_model* model,
                     const letkf_domain_map* map, int precision, uint32_t flags, const double* X0,
                     letkf_handle** out) {
  if (!out) return fail(LETKF_EINVAL, "null out");
  *out = nullptr;
  auto* h = new letkf_handle();
  // the arguments are checked before the server is used
  int rc = validate(dims, model, map, precision, flags, h->P);
  if (!rc) rc = server_admissible(h->P);
  if (!rc && !s) rc = fail(LETKF_EINVAL, "null server");
  if (rc) { delete h; return rc; }
  if (!X0) { delete h; return fail(LETKF_EINVAL, "null X0"); }
  for (size_t i = 0; i < 2 * (size_t)h->P.n_act * h->P.m; ++i)
    if (!std::isfinite(X0[i])) { delete h; return fail(LETKF_ENUMERIC, "non-finite X0"); }
  h->L = make_layout(h->P);
  h->mpad = padded_members(h->P.m);
  h->cls = h->P.cls();
  h->device = s->device;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->tuning) { delete h; return fail(LETKF_EAGAIN, "server autotuning in progress"); }
    int slot = -1;
    for (int k = 0; k < kMaxInstances; ++k)
      if (!s->inst[k]) { slot = k; break; }
    if (slot < 0) { delete h; return fail(LETKF_ENOMEM, "server holds the maximum number of instances"); }
    size_t off = 0;
    for (auto it = s->free_list.begin(); it != s->free_list.end(); ++it) {
      if (it->second >= h->L.total) {
        off = it->first;
        const size_t rest = it->second - h->L.total;
        s->free_list.erase(it);
        if (rest) s->free_list[off + h->L.total] = rest;
        break;
      }
    }
    if (!off) {
      const size_t need = h->L.total;
      delete h;
      return fail(LETKF_ENOMEM, "HBM budget exhausted: instance needs " + std::to_string(need) + " bytes");
    }
    h->arena_off = off;
    h->ws = s->arena + off;
    h->slot = slot;
    h->server = s;
    s->inst[slot] = h;  // reserved; invisible to the scheduler until its queue exists
  }
  if (hipSetDevice(s->device) != hipSuccess) rc = fail(LETKF_EDEVICE, "hipSetDevice");
  if (!rc) rc = upload_instance(h->P, h->L, h->ws, X0, s->upload, h->desc);
  if (!rc && hipMemcpyAsync(s->table() + h->slot, &h->desc, sizeof(InstDesc), hipMemcpyHostToDevice, s->upload) != hipSuccess)
    rc = fail(LETKF_EDEVICE, "table upload");
  if (!rc && hipStreamSynchronize(s->upload) != hipSuccess) rc = fail(LETKF_EDEVICE, "upload sync");
  if (!rc && hipHostMalloc((void**)&h->h_out, sizeof(double) * h->P.n_act) != hipSuccess) rc = fail(LETKF_EDEVICE, "pinned");
  std::lock_guard<std::mutex> lk(s->mu);
  if (rc) {
    s->inst[h->slot] = nullptr;
    s->free_list[h->arena_off] = h->L.total;
    if (h->h_out) (void)hipHostFree(h->h_out);
    delete h;
    return rc;
  }
  s->queues[h];
  s->in_flight[h] = 0;
  *out = h;
  return LETKF_OK;
}

int letkf_server_remove(letkf_server* s, letkf_handle* h) {
  if (!s || !h || h->server != s) return fail(LETKF_EINVAL, "handle does not belong to this server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->tuning) return fail(LETKF_EAGAIN, "server autotuning in progress");
  if (!s->queues[h].empty() || s->in_flight[h] > 0) return fail(LETKF_EAGAIN, "instance still has frames in flight");
  s->queues.erase(h);
  s->in_flight.erase(h);
  s->inst[h->slot] = nullptr;
  // return the range and coalesce with neighbours
  auto it = s->free_list.emplace(h->arena_off, h->L.total).first;
  if (it != s->free_list.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      s->free_list.erase(it);
      it = prev;
    }
  }
  auto next = std::next(it);
  if (next != s->free_list.end() && it->first + it->second == next->first) {
    it->second += next->second;
    s->free_list.erase(next);
  }
  if (h->h_out) (void)hipHostFree(h->h_out);
  delete h;
  return LETKF_OK;
}

static int enqueue(letkf_handle* h, Frame&& f) {
  letkf_server* s = h->server;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(LETKF_ESTATE, "server is stopping");
  auto& q = s->queues[h];
  if (q.size() >= kQueueCap) return fail(LETKF_EAGAIN, "instance queue full");
  f.t_enq = Clock::now();
  q.push_back(std::move(f));
  s->pending++;
  s->cv_work.notify_one();
  return LETKF_OK;
}

int letkf_submit_frame(letkf_handle* h, const double* y, uint64_t frame_id, double* pred_out, letkf_done_fn cb,
                       void* user) {
  if (!h || !h->server) return fail(LETKF_EINVAL, "handle is not a server instance");
  if (!y) return fail(LETKF_EINVAL, "null y");
  const int p = h->P.p();
  for (int i = 0; i < p; ++i)
    if (!std::isfinite(y[i])) return fail(LETKF_ENUMERIC, "non-finite slopes");
  return enqueue(h, Frame{frame_id, pred_out, cb, user, std::vector<double>(y, y + p), nullptr});
}

int letkf_submit_frame_device(letkf_handle* h, const double* y_dev, uint64_t frame_id, double* pred_out,
                              letkf_done_fn cb, void* user) {
  if (!h || !h->server) return fail(LETKF_EINVAL, "handle is not a server instance");
  if (!y_dev) return fail(LETKF_EINVAL, "null y");
  return enqueue(h, Frame{frame_id, pred_out, cb, user, std::vector<double>(), y_dev});
}

int letkf_server_drain(letkf_server* s) {
  if (!s) return fail(LETKF_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] {
    if (s->pending || s->inflight) return false;
    for (auto& [h, n] : s->in_flight)
      if (n) return false;
    return true;
  });
  return LETKF_OK;
}

int letkf_server_set_window(letkf_server* s, uint32_t window_us) {
  if (!s) return fail(LETKF_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  s->window_us = window_us;
  return LETKF_OK;
}

int letkf_server_stats(letkf_server* s, uint64_t* frames, uint64_t* batches, uint64_t* batched_frames) {
  if (!s) return fail(LETKF_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (frames) *frames = s->frames_done;
  if (batches) *batches = s->batches;
  if (batched_frames) *batched_frames = s->batched_frames;
  return LETKF_OK;
}

int letkf_server_autotune(letkf_server* s, int32_t reps, letkf_tuning* out) {
  if (!s) return fail(LETKF_EINVAL, "null server");
  std::vector<letkf_handle*> all;
  int caps[kBigClass] = {};
  {
    // The tuning launches run without the lock, so that submitters are not held
    // up for the seconds it takes; meanwhile the scheduler launches nothing
    // (slot 0, its stream and staging are free: the server is idle) and the
    // instance set cannot change.
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->tuning) return fail(LETKF_EAGAIN, "server autotuning in progress");
    if (!s->idle()) return fail(LETKF_EAGAIN, "server has frames queued, being launched or in flight");
    s->tuning = true;
    for (letkf_handle* h : s->inst)
      if (h) all.push_back(h);
    for (int c = 0; c < kBigClass; ++c) caps[c] = s->overlap_cap(c);
  }
  const int slot = 0;
  hipStream_t st = s->stream[slot];
  int rc = LETKF_OK;
  int grids[kBigClass] = {};
  for (int c = 0; c < kBigClass && !rc; ++c) {  // the tunable classes (no m > 128 instance is admitted)
    if (out) out[c] = letkf_tuning{};
    BatchHdr& H = *s->h_hdr[slot];
    std::memset(&H, 0, sizeof(H));
    H.amean = s->dout(slot);
    H.pmean = s->dout(slot) + kStageDoubles;
    ClassBatch& cb = H.cls[c];
    std::vector<letkf_handle*> insts;
    size_t ytot = 0, otot = 0;
    for (letkf_handle* h : all) {
      if (h->cls != c || cb.n >= s->max_batch) continue;
      if (ytot + h->P.p() > kStageDoubles || otot + h->P.n_act > kStageDoubles) break;
      const int k = cb.n++;
      H.yptr[k] = s->dy(slot) + ytot;  // zero slopes: the solve's cost does not depend on them
      H.out_off[k] = (int32_t)otot;
      ytot += h->P.p();
      otot += h->P.n_act;
      cb.inst[k] = h->slot;
      cb.ent[k] = k;
      cb.act_off[k + 1] = cb.act_off[k] + h->P.n_act;
      cb.slope_off[k + 1] = cb.slope_off[k] + h->P.p();
      cb.dom_off[k + 1] = cb.dom_off[k] + h->P.n_dom;
      insts.push_back(h);
    }
    if (insts.empty()) continue;
    if (hipMemsetAsync(s->dy(slot), 0, ytot * sizeof(double), st) != hipSuccess ||
        hipMemcpyAsync(s->dhdr(slot), &H, sizeof(H), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {  // H is reused for the next class
      rc = fail(LETKF_EDEVICE, "autotune staging");
      break;
    }
    rc = tune_class(c, s->table(), s->dhdr(slot), cb.slope_off[cb.n], cb.dom_off[cb.n], insts, s->num_cu, reps, false,
                    caps[c], st, out ? &out[c] : nullptr, &grids[c]);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!rc) {
      for (int c = 0; c < kBigClass; ++c)
        if (grids[c]) s->cls_grid[c] = grids[c];
      s->drop_graphs();  // captured with the old grids
    }
    s->tuning = false;
  }
  s->cv_work.notify_all();
  return rc;
}

int letkf_server_set_tuning(letkf_server* s, int32_t cls, const letkf_tuning* t) {
  if (!s) return fail(LETKF_EINVAL, "null server");
  if (cls < 0 || cls >= kBigClass) return fail(LETKF_EINVAL, "class must be in [0, " + std::to_string(kBigClass) + ")");
  if (!t || t->grid < 1 || t->grid > 65535 || t->order < LETKF_ORDER_MAP || t->order > LETKF_ORDER_XCD)
    return fail(LETKF_EINVAL, "tuning: grid must be in [1, 65535] and order one of LETKF_ORDER_*");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->tuning) return fail(LETKF_EAGAIN, "server autotuning in progress");
  if (!s->idle()) return fail(LETKF_EAGAIN, "server has frames queued, being launched or in flight");
  for (letkf_handle* h : s->inst)
    if (h && h->cls == cls) {
      int rc = upload_order(h, t->order, s->upload);
      if (rc) return rc;
    }
  s->cls_grid[cls] = t->grid;
  s->drop_graphs();
  return LETKF_OK;
}

int letkf_server_destroy(letkf_server* s) {
  if (!s) return LETKF_OK;
  if (s->sched.joinable()) {
    letkf_server_drain(s);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    s->cv_slot.notify_all();
    s->sched.join();
    for (auto& t : s->compl_thr) t.join();
  }
  for (letkf_handle* h : s->inst)
    if (h) {
      if (h->h_out) (void)hipHostFree(h->h_out);
      delete h;
    }
  for (int k = 0; k < kSlots; ++k) {
    if (s->h_hdr[k]) (void)hipHostFree(s->h_hdr[k]);
    if (s->h_y[k]) (void)hipHostFree(s->h_y[k]);
    if (s->h_out[k]) (void)hipHostFree(s->h_out[k]);
    if (s->done_ev[k]) (void)hipEventDestroy(s->done_ev[k]);
  }
  s->drop_graphs();
  for (auto& st : s->stream)
    if (st) (void)hipStreamDestroy(st);
  if (s->upload) (void)hipStreamDestroy(s->upload);
  if (s->capture) (void)hipStreamDestroy(s->capture);
  delete s;
  return LETKF_OK;
}

}  // extern "C"
