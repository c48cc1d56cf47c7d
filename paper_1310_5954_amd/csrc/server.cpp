// Serving: many resident filter instances, frames batched across instances.
//
// Admission: instance workspaces are carved out of the caller's device arena
// (the HBM budget) with a first-fit allocator; an instance that does not fit
// is refused with LETKF_ENOMEM and can be admitted once others are removed.
//
// Continuous batching: submit_frame copies the slopes into the instance's
// queue and returns.  A scheduler thread repeatedly takes the oldest pending
// frame of every instance that has one (one frame per instance per batch,
// at most max_batch) and enqueues one launch sequence for the whole batch on
// the server stream: upload {header, slopes} -> slope synthesis per class ->
// domain analysis per class -> merge + forecast per class -> download of the
// prediction means.  Classes group instances of equal padded ensemble size
// and storage precision; every domain of every instance of a class is one
// work item of the same analysis launch.  While a batch runs, the next one is
// prepared in another staging slot; frames that arrive meanwhile join it.
// A completion thread waits for each batch, copies the means to the callers'
// buffers and fires the callbacks.  Frames of one instance stay in order
// because batches execute in stream order.
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
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

using namespace letkf;

namespace {

constexpr int kMaxInstances = 64;
constexpr int kSlots = 3;                 // staging slots (batches in flight + in preparation)
constexpr size_t kStageDoubles = 1 << 18; // slopes per slot and means per slot (each 2 MiB)
constexpr size_t kQueueCap = 64;          // pending frames per instance

struct Frame {
  uint64_t id;
  double* pred_out;
  letkf_done_fn cb;
  void* user;
  std::vector<double> y;       // host slopes (copied at submit), or empty when ydev is set
  const double* ydev;          // caller's device slopes
};

struct Batch {
  int slot;
  std::vector<std::pair<letkf_handle*, Frame>> frames;
  std::vector<int32_t> out_off;
};

}  // namespace

struct letkf_server {
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int device = 0;
  int max_batch = kMaxBatch;
  int64_t window_us = 100;        // idle-GPU wait for the other instances' frames
  hipStream_t stream = nullptr;   // batches
  hipStream_t upload = nullptr;   // admissions
  // arena: [table][hdr x kSlots][y x kSlots][means x kSlots][instance region]
  size_t table_off = 0, hdr_off = 0, y_off = 0, out_off = 0, region_off = 0;
  std::map<size_t, size_t> free_list;  // offset -> bytes (instance region)
  // pinned staging
  BatchHdr* h_hdr[kSlots] = {};
  double* h_y[kSlots] = {};
  double* h_out[kSlots] = {};
  hipEvent_t done_ev[kSlots] = {};
  bool slot_busy[kSlots] = {};

  std::mutex mu;
  std::condition_variable cv_work;   // scheduler: new frames / stop
  std::condition_variable cv_slot;   // scheduler: a slot freed
  std::condition_variable cv_done;   // completion thread: new batch; drain: progress
  std::vector<letkf_handle*> inst;   // by table slot (nullptr = free)
  std::map<letkf_handle*, std::deque<Frame>> queues;
  std::map<letkf_handle*, int> in_flight;
  std::deque<Batch> running;        // launched, not yet taken by the completion thread
  int inflight = 0;                 // launched and not yet completed
  int rr = 0;
  bool stop = false;
  uint64_t frames_done = 0, batches = 0, batched_frames = 0, pending = 0;
  std::thread sched, compl_thr;

  InstDesc* table() { return (InstDesc*)(arena + table_off); }
  BatchHdr* dhdr(int s) { return (BatchHdr*)(arena + hdr_off) + s; }
  double* dy(int s) { return (double*)(arena + y_off) + (size_t)s * kStageDoubles; }
  double* dout(int s) { return (double*)(arena + out_off) + (size_t)s * 2 * kStageDoubles; }

  void scheduler_loop();
  void completion_loop();
  int launch_batch(Batch& b);
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int letkf_server::launch_batch(Batch& b) {
  const int s = b.slot;
  BatchHdr& H = *h_hdr[s];
  std::memset(&H, 0, sizeof(H));
  H.amean = dout(s);
  H.pmean = dout(s) + kStageDoubles;
  size_t ytot = 0, otot = 0;
  int rows_slopes[kNumClasses] = {}, rows_act[kNumClasses] = {}, items[kNumClasses] = {};
  for (size_t e = 0; e < b.frames.size(); ++e) {
    letkf_handle* h = b.frames[e].first;
    const Frame& f = b.frames[e].second;
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
    ClassBatch& cb = H.cls[h->cls];
    const int k = cb.n++;
    cb.inst[k] = h->slot;
    cb.ent[k] = (int32_t)e;
    cb.act_off[k + 1] = cb.act_off[k] + h->P.n_act;
    cb.slope_off[k + 1] = cb.slope_off[k] + h->P.p();
    cb.dom_off[k + 1] = cb.dom_off[k] + h->P.n_dom;
    rows_slopes[h->cls] = cb.slope_off[k + 1];
    rows_act[h->cls] = cb.act_off[k + 1];
    items[h->cls] = cb.dom_off[k + 1];
  }
  LETKF_HIP(hipMemcpyAsync(dhdr(s), &H, sizeof(H), hipMemcpyHostToDevice, stream));
  if (ytot) LETKF_HIP(hipMemcpyAsync(dy(s), h_y[s], ytot * sizeof(double), hipMemcpyHostToDevice, stream));
  for (int c = 0; c < kNumClasses; ++c)
    if (H.cls[c].n) launch_slopes(c, rows_slopes[c], table(), dhdr(s), stream);
  for (int c = 0; c < kNumClasses; ++c)
    if (H.cls[c].n) launch_analysis(c, items[c], table(), dhdr(s), stream);
  for (int c = 0; c < kNumClasses; ++c)
    if (H.cls[c].n) launch_rows(c, 2, rows_act[c], table(), dhdr(s), stream);
  LETKF_HIP(hipGetLastError());
  LETKF_HIP(hipMemcpyAsync(h_out[s], dout(s) + kStageDoubles, otot * sizeof(double), hipMemcpyDeviceToHost,
                           stream));
  LETKF_HIP(hipEventRecord(done_ev[s], stream));
  return LETKF_OK;
}

void letkf_server::scheduler_loop() {
  (void)hipSetDevice(device);  // a failure shows up as an error status of the first batch
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] { return stop || pending > 0; });
    if (stop && pending == 0) return;
    // Adaptive batching: while a batch runs, a partial batch would only queue
    // behind it, so wait until every instance has a frame or the GPU drains;
    // on an idle GPU wait at most window_us for the missing instances.
    auto all_ready = [&] {
      for (auto& kv : queues)
        if (kv.second.empty()) return false;
      return true;
    };
    if (!stop && !all_ready()) {
      if (inflight > 0) cv_work.wait(lk, [&] { return stop || all_ready() || inflight == 0; });
      if (!stop && !all_ready() && window_us > 0)
        cv_work.wait_for(lk, std::chrono::microseconds(window_us), [&] { return stop || all_ready(); });
    }
    int s = -1;
    cv_slot.wait(lk, [&] {
      for (int k = 0; k < kSlots; ++k)
        if (!slot_busy[k]) { s = k; return true; }
      return false;
    });
    // one frame per instance with pending work, round robin from rr
    Batch b;
    b.slot = s;
    size_t ytot = 0, otot = 0;
    const int n = (int)inst.size();
    for (int t = 0; t < n && (int)b.frames.size() < max_batch; ++t) {
      letkf_handle* h = inst[(rr + t) % n];
      if (!h) continue;
      auto& q = queues[h];
      if (q.empty()) continue;
      if (ytot + h->P.p() > kStageDoubles || otot + h->P.n_act > kStageDoubles) break;
      ytot += h->P.p();
      otot += h->P.n_act;
      b.frames.emplace_back(h, std::move(q.front()));
      q.pop_front();
      in_flight[h]++;
      --pending;
    }
    rr = (rr + 1) % std::max(n, 1);
    if (b.frames.empty()) continue;
    slot_busy[s] = true;
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
      continue;
    }
    ++batches;
    ++inflight;
    batched_frames += b.frames.size();
    running.push_back(std::move(b));
    cv_done.notify_all();
  }
}

void letkf_server::completion_loop() {
  (void)hipSetDevice(device);  // a failure shows up as an error status of the first batch
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_done.wait(lk, [&] { return stop || !running.empty(); });
    if (running.empty()) {
      if (stop) return;
      continue;
    }
    Batch b = std::move(running.front());
    running.pop_front();
    lk.unlock();
    const hipError_t e = hipEventSynchronize(done_ev[b.slot]);
    const int status = e == hipSuccess ? LETKF_OK : LETKF_EDEVICE;
    for (size_t k = 0; k < b.frames.size(); ++k) {
      auto& [h, f] = b.frames[k];
      if (status == LETKF_OK && f.pred_out)
        std::memcpy(f.pred_out, h_out[b.slot] + b.out_off[k], sizeof(double) * h->P.n_act);
      if (f.cb) f.cb(f.user, f.id, status);
    }
    lk.lock();
    for (auto& [h, f] : b.frames) in_flight[h]--;
    frames_done += b.frames.size();
    --inflight;
    slot_busy[b.slot] = false;
    cv_slot.notify_all();
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

int letkf::server_idle_stream(letkf_handle* h, hipStream_t* stream) {
  letkf_server* s = h->server;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->queues[h].empty() || s->in_flight[h] > 0) return fail(LETKF_EAGAIN, "instance has frames in flight");
  }
  LETKF_HIP(hipStreamSynchronize(s->stream));
  *stream = s->stream;
  return LETKF_OK;
}

extern "C" {

int letkf_server_create(void* arena, size_t arena_bytes, int32_t max_batch, uint32_t flags, letkf_server** out) {
  if (!out) return fail(LETKF_EINVAL, "null out");
  *out = nullptr;
  if (!arena || ((uintptr_t)arena & 255)) return fail(LETKF_EINVAL, "arena must be non-null and 256-byte aligned");
  if (max_batch < 1 || max_batch > kMaxBatch) return fail(LETKF_EINVAL, "max_batch must be in [1, 64]");
  if (flags) return fail(LETKF_EINVAL, "unknown flags");
  auto* s = new letkf_server();
  s->arena = (char*)arena;
  s->arena_bytes = arena_bytes;
  s->max_batch = max_batch;
  size_t off = 0;
  s->table_off = off; off = align256(off + sizeof(InstDesc) * kMaxInstances);
  s->hdr_off = off; off = align256(off + sizeof(BatchHdr) * kSlots);
  s->y_off = off; off = align256(off + sizeof(double) * kStageDoubles * kSlots);
  s->out_off = off; off = align256(off + 2 * sizeof(double) * kStageDoubles * kSlots);
  s->region_off = off;
  if (arena_bytes < off + 256) { delete s; return fail(LETKF_ENOMEM, "arena smaller than the server's own tables"); }
  s->free_list[off] = arena_bytes - off;
  s->inst.assign(kMaxInstances, nullptr);
  int rc = LETKF_OK;
  if (hipGetDevice(&s->device) != hipSuccess) rc = fail(LETKF_EDEVICE, "hipGetDevice");
  if (!rc && hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) rc = fail(LETKF_EDEVICE, "stream");
  if (!rc && hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking) != hipSuccess) rc = fail(LETKF_EDEVICE, "stream");
  for (int k = 0; k < kSlots && !rc; ++k) {
    if (hipHostMalloc((void**)&s->h_hdr[k], sizeof(BatchHdr)) != hipSuccess ||
        hipHostMalloc((void**)&s->h_y[k], sizeof(double) * kStageDoubles) != hipSuccess ||
        hipHostMalloc((void**)&s->h_out[k], sizeof(double) * kStageDoubles) != hipSuccess ||
        hipEventCreateWithFlags(&s->done_ev[k], hipEventDisableTiming) != hipSuccess)
      rc = fail(LETKF_EDEVICE, "pinned staging / events");
  }
  if (rc) { letkf_server_destroy(s); return rc; }
  s->sched = std::thread([s] { s->scheduler_loop(); });
  s->compl_thr = std::thread([s] { s->completion_loop(); });
  *out = s;
  return LETKF_OK;
}

int letkf_server_add(letkf_server* s, const letkf_dims* dims, const letkf_model* model,
                     const letkf_domain_map* map, int precision, uint32_t flags, const double* X0,
                     letkf_handle** out) {
  if (!s || !out) return fail(LETKF_EINVAL, "null server/out");
  *out = nullptr;
  auto* h = new letkf_handle();
  int rc = validate(dims, model, map, precision, flags, h->P);
  if (rc) { delete h; return rc; }
  if (!X0) { delete h; return fail(LETKF_EINVAL, "null X0"); }
  for (size_t i = 0; i < 2 * (size_t)h->P.n_act * h->P.m; ++i)
    if (!std::isfinite(X0[i])) { delete h; return fail(LETKF_ENUMERIC, "non-finite X0"); }
  h->L = make_layout(h->P);
  h->mpad = padded_members(h->P.m);
  h->cls = class_of(h->mpad, h->P.prec);
  h->device = s->device;
  {
    std::lock_guard<std::mutex> lk(s->mu);
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
    if (s->pending || !s->running.empty()) return false;
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
    s->compl_thr.join();
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
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->upload) (void)hipStreamDestroy(s->upload);
  delete s;
  return LETKF_OK;
}

}  // extern "C"
