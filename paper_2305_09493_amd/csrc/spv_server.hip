// Continuous-batching validation server (host runtime around the kernels).
//
// Requests (host word buffers, one SPIR-V module each) carry an arrival time.
// A worker thread admits arrived requests into "slots": each slot owns a
// stream, pinned host staging, and device buffers sized from the device
// memory budget.  Whenever a slot is free, every request that has arrived and
// fits (module count and words) joins the next batch: its words are staged,
// copied to the device, validated as one CSR batch (one spv_validate call,
// or a replay of a HIP graph captured for the batch's padded size bucket),
// and its 16-byte results come back; several slots are in flight at once, so
// copies and kernels of different batches overlap.  Latency of a request is
// completion time minus arrival time.  With max_batch_modules = 1 the same
// machinery is the one-module-per-launch baseline.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_set>
#include <utility>
#include <vector>

#include "spv_admission.h"
#include "spv_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  int64_t id;
  const uint32_t* words;
  int64_t n;
  int64_t t_arr_ns;  // relative to the server start
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint32_t* d_words = nullptr;
  int64_t* d_mod_off = nullptr;
  spv_result* d_res = nullptr;
  uint32_t* d_idx_off = nullptr;
  uint16_t* d_idx_op = nullptr;
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t* h_words = nullptr;
  int64_t* h_mod_off = nullptr;
  spv_result* h_res = nullptr;
  int64_t cap_words = 0, cap_modules = 0;
  bool busy = false;
  std::vector<Req> batch;
  std::map<std::pair<int64_t, int64_t>, hipGraphExec_t> graphs;
};

}  // namespace

struct spv_server {
  spv_ctx* ctx = nullptr;
  int device = 0;
  std::vector<Slot> slots;
  int64_t max_batch = 0;
  bool use_graphs = false;
  std::mutex mu;
  std::deque<Req> incoming;  // submitted, sorted by arrival within each submit call
  std::unordered_set<int64_t> cancel;  // ids to cancel if not yet admitted to a batch
  std::vector<spv_completion> completed;
  std::thread worker;
  std::atomic<bool> stop{false};
  std::atomic<bool> started{false};
  Clock::time_point t0;
  std::atomic<int64_t> in_flight{0};
  int64_t n_batches = 0, n_modules = 0, n_words = 0, max_seen_batch = 0;
  hipError_t err = hipSuccess;
};

namespace {

int64_t now_ns(const spv_server* s) {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - s->t0).count();
}

using spv::bucket_up;

// Launch (or replay) the validation of the slot's staged batch.
hipError_t launch_batch(spv_server* S, Slot& sl, int64_t M, int64_t W) {
  int64_t Mp = M, Wp = W;
  if (S->use_graphs) {
    Wp = bucket_up(W + 1);  // the padding words form one extra module
    Mp = bucket_up(M + 1);
    if (Wp > sl.cap_words) Wp = sl.cap_words;
    if (Mp > sl.cap_modules) Mp = sl.cap_modules;
    // padded layout: modules M..Mp-1 are empty except the first, which owns
    // the padding words [W, Wp)
    for (int64_t m = M + 1; m <= Mp; ++m) sl.h_mod_off[m] = Wp;
    memset(sl.h_words + W, 0, size_t(Wp - W) * 4);
  }
  hipError_t e = hipMemcpyAsync(sl.d_words, sl.h_words, size_t(Wp) * 4, hipMemcpyHostToDevice, sl.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.d_mod_off, sl.h_mod_off, size_t(Mp + 1) * 8, hipMemcpyHostToDevice, sl.stream);
  if (e != hipSuccess) return e;
  if (!S->use_graphs) {
    int r = spv_validate(S->ctx, sl.d_words, sl.d_mod_off, Mp, Wp, sl.d_idx_off, sl.d_idx_op, Wp, sl.d_res, 0,
                         sl.d_ws, sl.ws_bytes, sl.stream);
    if (r != SPV_SUCCESS) return hipErrorLaunchFailure;
  } else {
    auto key = std::make_pair(Mp, Wp);
    auto it = sl.graphs.find(key);
    if (it == sl.graphs.end()) {
      hipGraph_t g = nullptr;
      e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return e;
      int r = spv_validate(S->ctx, sl.d_words, sl.d_mod_off, Mp, Wp, sl.d_idx_off, sl.d_idx_op, Wp, sl.d_res, 0,
                           sl.d_ws, sl.ws_bytes, sl.stream);
      e = hipStreamEndCapture(sl.stream, &g);  // (ends the capture on every path)
      if (r != SPV_SUCCESS || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e != hipSuccess ? e : hipErrorLaunchFailure;
      }
      hipGraphExec_t ge;
      e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return e;
      it = sl.graphs.emplace(key, ge).first;
    }
    e = hipGraphLaunch(it->second, sl.stream);
    if (e != hipSuccess) return e;
  }
  e = hipMemcpyAsync(sl.h_res, sl.d_res, size_t(M) * sizeof(spv_result), hipMemcpyDeviceToHost, sl.stream);
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  return e;
}

// Complete every request of the slot's batch (status 0: with the results the
// batch copied back) and free the slot.
void finish_batch(spv_server* S, Slot& sl, int status) {
  const int64_t t_done = now_ns(S);
  std::lock_guard<std::mutex> lk(S->mu);
  spv::complete_batch(
      int64_t(sl.batch.size()), [&](int64_t i) -> const Req& { return sl.batch[size_t(i)]; },
      status == 0 ? sl.h_res : nullptr, status, t_done, S->completed);
  S->in_flight -= int64_t(sl.batch.size());
  sl.batch.clear();
  sl.busy = false;
}

void worker_main(spv_server* S) {
  (void)hipSetDevice(S->device);
  std::deque<Req> ready;      // arrived, waiting for a slot (FIFO)
  std::deque<Req> waiting;    // submitted, not yet arrived
  std::vector<uint8_t> action;  // admission decisions for the front of `ready`
  for (;;) {
    std::unordered_set<int64_t> to_cancel;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      while (!S->incoming.empty()) {
        waiting.push_back(S->incoming.front());
        S->incoming.pop_front();
      }
      to_cancel.swap(S->cancel);
    }
    if (!to_cancel.empty()) {
      // cancelled requests not yet in a batch complete at once; ids not
      // queued any more (admitted or done) are ignored
      const int64_t t = now_ns(S);
      std::vector<spv_completion> done;
      for (std::deque<Req>* q : {&waiting, &ready}) {
        std::deque<Req> keep;
        for (const Req& r : *q) {
          if (to_cancel.count(r.id)) {
            spv_completion c;
            memset(&c, 0, sizeof(c));
            c.id = r.id;
            c.status = SPV_ERR_CANCELED;
            c.t_arrival_ns = r.t_arr_ns;
            c.t_done_ns = t;
            done.push_back(c);
          } else {
            keep.push_back(r);
          }
        }
        q->swap(keep);
      }
      if (!done.empty()) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->completed.insert(S->completed.end(), done.begin(), done.end());
        S->in_flight -= int64_t(done.size());
      }
    }
    const int64_t now = now_ns(S);
    // arrivals (requests are submitted in arrival order)
    while (!waiting.empty() && waiting.front().t_arr_ns <= now) {
      ready.push_back(waiting.front());
      waiting.pop_front();
    }
    bool did = false;
    // completions
    for (Slot& sl : S->slots) {
      if (!sl.busy) continue;
      hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) S->err = q;
      finish_batch(S, sl, q == hipSuccess ? 0 : SPV_ERR_HIP);
      did = true;
    }
    // admission: fill every free slot with arrived requests that fit
    for (Slot& sl : S->slots) {
      if (sl.busy || ready.empty()) continue;
      int64_t W = 0, M = 0;
      sl.h_mod_off[0] = 0;
      const int64_t n_look = int64_t(ready.size()) < S->max_batch + 64 ? int64_t(ready.size()) : S->max_batch + 64;
      action.resize(size_t(n_look));
      const int64_t n_ex = spv::admit_batch(
          n_look, [&](int64_t i) { return ready[size_t(i)].n; }, S->max_batch, sl.cap_modules, sl.cap_words,
          action.data());
      for (int64_t i = 0; i < n_ex; ++i) {
        const Req& r = ready.front();
        if (action[size_t(i)] == spv::kAdmitReject) {
          // larger than a slot: rejected
          std::lock_guard<std::mutex> lk(S->mu);
          spv_completion c;
          memset(&c, 0, sizeof(c));
          c.id = r.id;
          c.status = SPV_ERR_CAPACITY;
          c.t_arrival_ns = r.t_arr_ns;
          c.t_done_ns = now_ns(S);
          S->completed.push_back(c);
          S->in_flight -= 1;
        } else {
          memcpy(sl.h_words + W, r.words, size_t(r.n) * 4);
          W += r.n;
          sl.batch.push_back(r);
          sl.h_mod_off[++M] = W;
        }
        ready.pop_front();
      }
      if (M == 0) continue;
      hipError_t e = launch_batch(S, sl, M, W);
      if (e != hipSuccess) {
        // nothing of this batch will complete on the GPU: its requests end
        // now with SPV_ERR_HIP and the slot stays free
        S->err = e;
        finish_batch(S, sl, SPV_ERR_HIP);
      } else {
        sl.busy = true;
      }
      S->n_batches += 1;
      S->n_modules += M;
      S->n_words += W;
      S->max_seen_batch = std::max(S->max_seen_batch, M);
      did = true;
    }
    if (S->stop.load() && waiting.empty() && ready.empty()) {
      bool any = false;
      for (Slot& sl : S->slots) any |= sl.busy;
      if (!any) {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->incoming.empty()) break;
      }
    }
    if (!did) std::this_thread::yield();
  }
}

void free_slot(Slot& sl) {
  for (auto& kv : sl.graphs) (void)hipGraphExecDestroy(kv.second);
  sl.graphs.clear();
  if (sl.done) (void)hipEventDestroy(sl.done);
  if (sl.stream) (void)hipStreamDestroy(sl.stream);
  (void)hipFree(sl.d_words);
  (void)hipFree(sl.d_mod_off);
  (void)hipFree(sl.d_res);
  (void)hipFree(sl.d_idx_off);
  (void)hipFree(sl.d_idx_op);
  (void)hipFree(sl.d_ws);
  (void)hipHostFree(sl.h_words);
  (void)hipHostFree(sl.h_mod_off);
  (void)hipHostFree(sl.h_res);
}

}  // namespace

extern "C" {

int spv_server_create(spv_server** out, spv_ctx* ctx, int hip_device, size_t device_budget_bytes, int n_slots,
                      int64_t max_batch_modules, int64_t slot_max_modules, int use_graphs) {
  if (!out || !ctx || n_slots < 1 || n_slots > 16 || max_batch_modules < 1 || slot_max_modules < 2)
    return SPV_ERR_INVALID_ARG;
  *out = nullptr;
  if (hipSetDevice(hip_device) != hipSuccess) return SPV_ERR_HIP;
  spv_server* S = new spv_server;
  S->ctx = ctx;
  S->device = hip_device;
  S->max_batch = max_batch_modules;
  S->use_graphs = use_graphs != 0;
  // device bytes per slot word: words 4 + index 6 + workspace ~8; per module
  // mod_off 8 + results 16 + workspace state
  const size_t per_slot = device_budget_bytes / size_t(n_slots);
  const int64_t cap_modules = slot_max_modules;
  size_t ws_mod = 0;
  spv_workspace_size(ctx, cap_modules, 0, &ws_mod);
  const size_t fixed = size_t(cap_modules + 1) * (8 + 16) + ws_mod + (1 << 20);
  if (per_slot <= fixed) {
    delete S;
    return SPV_ERR_CAPACITY;
  }
  int64_t cap_words = int64_t((per_slot - fixed) / 19);  // 4 + 4 + 2 + 8 (+1 slack) bytes per word
  if (cap_words > (int64_t(1) << 26)) cap_words = int64_t(1) << 26;  // bounds the pinned staging too
  cap_words &= ~int64_t(4095);
  S->slots.resize(size_t(n_slots));
  int rc = SPV_SUCCESS;
  for (Slot& sl : S->slots) {
    sl.cap_words = cap_words;
    sl.cap_modules = cap_modules;
    spv_workspace_size(ctx, cap_modules, cap_words, &sl.ws_bytes);
    hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&sl.d_words, size_t(cap_words) * 4);
    if (e == hipSuccess) e = hipMalloc(&sl.d_mod_off, size_t(cap_modules + 1) * 8);
    if (e == hipSuccess) e = hipMalloc(&sl.d_res, size_t(cap_modules) * sizeof(spv_result));
    if (e == hipSuccess) e = hipMalloc(&sl.d_idx_off, size_t(cap_words) * 4);
    if (e == hipSuccess) e = hipMalloc(&sl.d_idx_op, size_t(cap_words) * 2);
    if (e == hipSuccess) e = hipMalloc(&sl.d_ws, sl.ws_bytes);
    if (e == hipSuccess) e = hipHostMalloc(&sl.h_words, size_t(cap_words) * 4, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&sl.h_mod_off, size_t(cap_modules + 1) * 8, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&sl.h_res, size_t(cap_modules) * sizeof(spv_result), hipHostMallocDefault);
    if (e != hipSuccess) {
      rc = SPV_ERR_HIP;
      break;
    }
  }
  if (rc != SPV_SUCCESS) {
    for (Slot& sl : S->slots) free_slot(sl);
    delete S;
    return rc;
  }
  S->t0 = Clock::now();
  *out = S;
  return SPV_SUCCESS;
}

int spv_server_start(spv_server* S) {
  if (!S || S->started.load()) return SPV_ERR_INVALID_ARG;
  S->t0 = Clock::now();
  S->started = true;
  S->worker = std::thread(worker_main, S);
  return SPV_SUCCESS;
}

int spv_server_submit(spv_server* S, int64_t n, const int64_t* ids, const uint32_t* const* words,
                      const int64_t* n_words, const int64_t* t_arrival_ns) {
  if (!S || n < 0 || (n > 0 && (!ids || !words || !n_words))) return SPV_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  const int64_t now = now_ns(S);
  for (int64_t i = 0; i < n; ++i) {
    Req r;
    r.id = ids[i];
    r.words = words[i];
    r.n = n_words[i];
    r.t_arr_ns = (t_arrival_ns && t_arrival_ns[i] >= 0) ? t_arrival_ns[i] : now;
    S->incoming.push_back(r);
  }
  S->in_flight += n;
  return SPV_SUCCESS;
}

int spv_server_cancel(spv_server* S, int64_t n, const int64_t* ids) {
  if (!S || n < 0 || (n > 0 && !ids)) return SPV_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  for (int64_t i = 0; i < n; ++i) S->cancel.insert(ids[i]);
  return SPV_SUCCESS;
}

int spv_server_poll(spv_server* S, spv_completion* out, int64_t max_out, int64_t* n_out, int64_t* pending) {
  if (!S || !n_out || max_out < 0 || (max_out > 0 && !out)) return SPV_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  int64_t k = std::min<int64_t>(max_out, int64_t(S->completed.size()));
  for (int64_t i = 0; i < k; ++i) out[i] = S->completed[size_t(i)];
  S->completed.erase(S->completed.begin(), S->completed.begin() + k);
  *n_out = k;
  if (pending) *pending = S->in_flight.load();
  return S->err == hipSuccess ? SPV_SUCCESS : SPV_ERR_HIP;
}

int spv_server_stats(spv_server* S, int64_t* n_batches, int64_t* n_modules, int64_t* n_words, int64_t* max_batch,
                     int64_t* slot_capacity_words) {
  if (!S) return SPV_ERR_INVALID_ARG;
  if (n_batches) *n_batches = S->n_batches;
  if (n_modules) *n_modules = S->n_modules;
  if (n_words) *n_words = S->n_words;
  if (max_batch) *max_batch = S->max_seen_batch;
  if (slot_capacity_words) *slot_capacity_words = S->slots.empty() ? 0 : S->slots[0].cap_words;
  return SPV_SUCCESS;
}

int spv_server_destroy(spv_server* S) {
  if (!S) return SPV_ERR_INVALID_ARG;
  S->stop = true;
  if (S->worker.joinable()) S->worker.join();
  for (Slot& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    free_slot(sl);
  }
  delete S;
  return SPV_SUCCESS;
}

}  // extern "C"
