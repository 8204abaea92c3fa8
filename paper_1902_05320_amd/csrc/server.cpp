// Continuous-batching hash server.
//
// Requests (a variant and a list of (offset, length) slices of a
// device-resident byte pool) are queued by any host thread.  One worker
// thread forms steps: it admits queued requests in arrival order while the
// step has message slots and byte budget left (a request never straddles
// steps; one larger than a step is rejected at submit), writes the step's
// descriptors into pinned host buffers and replays the step slot's graph on
// the slot's stream.  The graph, captured when the server is created, holds
// the uploads of the descriptors and of the message count, both passes of
// the mixed-variant persistent form (which read the count from device
// memory, so one capture serves every step size) and the digest download;
// the copy sizes are set to the step's message count before each replay.
// Up to `steps_in_flight` steps are in flight at once, so requests that
// arrive while others are on the GPU are admitted into the next step as
// soon as a step slot frees up, and their work overlaps the running steps on
// the device.  When a step's event has completed the worker copies each
// request's digests out and marks it done.
//
// The executor is pluggable: the default one does the above with HIP (or,
// with KB_SERVER_EAGER, as separate copies and a keccak_batch_mixed call); a
// caller-supplied callback replaces upload/launch/download (used to test the
// admission and completion logic without a GPU).
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "kb_internal.h"
#include "kbatch.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id;
  int variant;
  std::vector<uint64_t> offs, lens;
  uint64_t bytes = 0;  // sum of the lengths
  Clock::time_point t_submit;
  Clock::time_point t_done;
  std::vector<uint8_t> digests;  // n * 64
  int status = KB_OK;
};

struct StepSlot {
  // host side (pinned for the HIP executor, plain for a callback executor)
  uint64_t* h_offs = nullptr;
  uint64_t* h_lens = nullptr;
  uint8_t* h_vars = nullptr;
  uint8_t* h_out = nullptr;
  // device side (HIP executor)
  uint64_t* d_offs = nullptr;
  uint64_t* d_lens = nullptr;
  uint8_t* d_vars = nullptr;
  uint8_t* d_out = nullptr;
  uint32_t* h_count = nullptr;  // pinned: the step's message count
  uint32_t* d_count = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  // the step graph: count and descriptor uploads -> the batch -> download
  kb_graph* batch = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t n_count = nullptr, n_offs = nullptr, n_lens = nullptr, n_vars = nullptr,
                 n_batch = nullptr, n_out = nullptr;
  bool busy = false;
  uint64_t n = 0;
  std::vector<Request*> reqs;
  Clock::time_point t_launch;
};

}  // namespace

struct kb_server {
  kb_server_config cfg{};
  int device = 0;
  std::vector<StepSlot> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> pending;
  std::map<uint64_t, Request*> done;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  std::string error;
  // statistics
  uint64_t steps = 0, msgs = 0, bytes = 0, completed = 0, rejected = 0, max_step_msgs_seen = 0;
  double busy_s = 0.0;
  Clock::time_point t_first_launch{}, t_last_done{};
  bool any_launch = false;
};

namespace {

thread_local std::string g_srv_err;

int srv_fail(int code, const char* msg) {
  g_srv_err = msg;
  return code;
}

bool hip_ok(hipError_t e, kb_server* s, const char* what) {
  if (e == hipSuccess) return true;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error.empty()) s->error = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

// Launch one step on its slot (HIP executor or callback).
bool launch_step(kb_server* s, StepSlot& st) {
  const uint64_t n = st.n;
  if (s->cfg.executor) {
    const int rc = s->cfg.executor(s->cfg.executor_user, st.h_vars, st.h_offs, st.h_lens, n, st.h_out);
    if (rc != KB_OK) {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->error.empty()) s->error = "executor callback failed";
      return false;
    }
    return true;
  }
  if (st.exec) {
    *st.h_count = static_cast<uint32_t>(n);
    return hip_ok(hipGraphExecMemcpyNodeSetParams1D(st.exec, st.n_offs, st.d_offs, st.h_offs, n * 8,
                                                    hipMemcpyHostToDevice), s, "step offsets size") &&
           hip_ok(hipGraphExecMemcpyNodeSetParams1D(st.exec, st.n_lens, st.d_lens, st.h_lens, n * 8,
                                                    hipMemcpyHostToDevice), s, "step lengths size") &&
           hip_ok(hipGraphExecMemcpyNodeSetParams1D(st.exec, st.n_vars, st.d_vars, st.h_vars, n,
                                                    hipMemcpyHostToDevice), s, "step variants size") &&
           hip_ok(hipGraphExecMemcpyNodeSetParams1D(st.exec, st.n_out, st.h_out, st.d_out, n * 64,
                                                    hipMemcpyDeviceToHost), s, "step digests size") &&
           hip_ok(hipGraphLaunch(st.exec, st.stream), s, "step graph launch") &&
           hip_ok(hipEventRecord(st.done, st.stream), s, "record event");
  }
  if (!hip_ok(hipMemcpyAsync(st.d_offs, st.h_offs, n * 8, hipMemcpyHostToDevice, st.stream), s, "upload offsets") ||
      !hip_ok(hipMemcpyAsync(st.d_lens, st.h_lens, n * 8, hipMemcpyHostToDevice, st.stream), s, "upload lengths") ||
      !hip_ok(hipMemcpyAsync(st.d_vars, st.h_vars, n, hipMemcpyHostToDevice, st.stream), s, "upload variants"))
    return false;
  const int rc = keccak_batch_mixed(st.d_vars, s->cfg.d_pool, st.d_offs, st.d_lens, n, st.d_out,
                                    st.stream);
  if (rc != KB_OK) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error.empty()) s->error = std::string("keccak_batch_mixed: ") + keccak_last_error();
    return false;
  }
  return hip_ok(hipMemcpyAsync(st.h_out, st.d_out, n * 64, hipMemcpyDeviceToHost, st.stream), s,
                "download digests") &&
         hip_ok(hipEventRecord(st.done, st.stream), s, "record event");
}

bool step_finished(kb_server* s, StepSlot& st) {
  if (s->cfg.executor) return true;  // the callback ran synchronously
  const hipError_t e = hipEventQuery(st.done);
  if (e == hipErrorNotReady) return false;
  hip_ok(e, s, "step event");
  return true;
}

void complete_step(kb_server* s, StepSlot& st) {
  const auto now = Clock::now();
  uint64_t pos = 0;
  for (Request* r : st.reqs) {
    const uint64_t k = r->offs.size();
    r->digests.assign(st.h_out + pos * 64, st.h_out + (pos + k) * 64);
    r->t_done = now;
    pos += k;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  for (Request* r : st.reqs) s->done[r->id] = r;
  s->completed += st.reqs.size();
  s->busy_s += std::chrono::duration<double>(now - st.t_launch).count();
  s->t_last_done = now;
  st.reqs.clear();
  st.busy = false;
  st.n = 0;
  s->cv.notify_all();
}

void worker_main(kb_server* s) {
  if (!s->cfg.executor) (void)hipSetDevice(s->device);
  for (;;) {
    // retire finished steps
    bool any_busy = false;
    for (StepSlot& st : s->slots) {
      if (st.busy && step_finished(s, st)) complete_step(s, st);
      any_busy = any_busy || st.busy;
    }
    StepSlot* free_slot = nullptr;
    for (StepSlot& st : s->slots)
      if (!st.busy) {
        free_slot = &st;
        break;
      }
    std::vector<Request*> batch;
    uint64_t n = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop && s->pending.empty() && !any_busy) return;
      if (free_slot) {
        // admit in arrival order while the step has message slots and
        // byte budget left
        uint64_t bytes = 0;
        while (!s->pending.empty()) {
          Request* r = s->pending.front();
          if (n + r->offs.size() > s->cfg.max_step_msgs) break;
          if (s->cfg.max_step_bytes && bytes + r->bytes > s->cfg.max_step_bytes) break;
          n += r->offs.size();
          bytes += r->bytes;
          batch.push_back(r);
          s->pending.pop_front();
        }
      }
      if (batch.empty()) {
        // nothing to launch: wait for a submission, or poll in-flight steps
        if (any_busy)
          s->cv.wait_for(lk, std::chrono::microseconds(50));
        else if (!s->stop)
          s->cv.wait_for(lk, std::chrono::milliseconds(5), [s] { return s->stop || !s->pending.empty(); });
        continue;
      }
    }
    StepSlot& st = *free_slot;
    uint64_t pos = 0;
    for (Request* r : batch) {
      const uint64_t k = r->offs.size();
      std::memcpy(st.h_offs + pos, r->offs.data(), k * 8);
      std::memcpy(st.h_lens + pos, r->lens.data(), k * 8);
      std::memset(st.h_vars + pos, r->variant, k);
      pos += k;
    }
    st.n = n;
    st.reqs = std::move(batch);
    st.busy = true;
    st.t_launch = Clock::now();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (!s->any_launch) {
        s->t_first_launch = st.t_launch;
        s->any_launch = true;
      }
      ++s->steps;
      s->msgs += n;
      for (Request* r : st.reqs) s->bytes += r->bytes;
      if (n > s->max_step_msgs_seen) s->max_step_msgs_seen = n;
    }
    if (!launch_step(s, st)) {
      for (Request* r : st.reqs) r->status = KB_EHIP;
      complete_step(s, st);
    }
  }
}

// Build a slot's step graph: the count and descriptor uploads, then the
// batch captured over the slot's buffers (count read on the device), then the
// digest download.  The copy sizes are placeholders, set before each replay.
// The nodes form one chain: with the four uploads as independent branches,
// the steps of different slots no longer overlapped on the device (each took
// about twice as long as the same step run eagerly, measured), as if the
// runtime ran the branches on streams shared by every graph.
bool build_step_graph(kb_server* s, StepSlot& st) {
  const uint64_t m = s->cfg.max_step_msgs;
  if (keccak_graph_create_counted(-1, st.d_vars, s->cfg.d_pool, st.d_offs, st.d_lens, st.d_count, m,
                                  st.d_out, st.stream, &st.batch) != KB_OK)
    return false;
  if (hipGraphCreate(&st.graph, 0) != hipSuccess) return false;
  if (hipGraphAddMemcpyNode1D(&st.n_count, st.graph, nullptr, 0, st.d_count, st.h_count, 4,
                              hipMemcpyHostToDevice) != hipSuccess ||
      hipGraphAddMemcpyNode1D(&st.n_offs, st.graph, &st.n_count, 1, st.d_offs, st.h_offs, 8,
                              hipMemcpyHostToDevice) != hipSuccess ||
      hipGraphAddMemcpyNode1D(&st.n_lens, st.graph, &st.n_offs, 1, st.d_lens, st.h_lens, 8,
                              hipMemcpyHostToDevice) != hipSuccess ||
      hipGraphAddMemcpyNode1D(&st.n_vars, st.graph, &st.n_lens, 1, st.d_vars, st.h_vars, 1,
                              hipMemcpyHostToDevice) != hipSuccess)
    return false;
  if (hipGraphAddChildGraphNode(&st.n_batch, st.graph, &st.n_vars, 1, kb::native_graph(st.batch)) !=
          hipSuccess ||
      hipGraphAddMemcpyNode1D(&st.n_out, st.graph, &st.n_batch, 1, st.h_out, st.d_out, 64,
                              hipMemcpyDeviceToHost) != hipSuccess)
    return false;
  return hipGraphInstantiate(&st.exec, st.graph, nullptr, nullptr, 0) == hipSuccess;
}

void free_slots(kb_server* s) {
  for (StepSlot& st : s->slots) {
    if (s->cfg.executor) {
      delete[] st.h_offs;
      delete[] st.h_lens;
      delete[] st.h_vars;
      delete[] st.h_out;
    } else {
      if (st.h_offs) (void)hipHostFree(st.h_offs);
      if (st.h_lens) (void)hipHostFree(st.h_lens);
      if (st.h_vars) (void)hipHostFree(st.h_vars);
      if (st.h_out) (void)hipHostFree(st.h_out);
      if (st.d_offs) (void)hipFree(st.d_offs);
      if (st.d_lens) (void)hipFree(st.d_lens);
      if (st.d_vars) (void)hipFree(st.d_vars);
      if (st.d_out) (void)hipFree(st.d_out);
      if (st.h_count) (void)hipHostFree(st.h_count);
      if (st.d_count) (void)hipFree(st.d_count);
      if (st.exec) (void)hipGraphExecDestroy(st.exec);
      if (st.graph) (void)hipGraphDestroy(st.graph);
      if (st.batch) (void)keccak_graph_destroy(st.batch);
      if (st.done) (void)hipEventDestroy(st.done);
      if (st.stream) (void)hipStreamDestroy(st.stream);
    }
  }
  s->slots.clear();
}

}  // namespace

extern "C" {

int keccak_server_create(const kb_server_config* cfg, kb_server** out) {
  g_srv_err.clear();
  if (!cfg || !out) return srv_fail(KB_EINVAL, "NULL argument");
  if (cfg->max_step_msgs == 0 || cfg->max_step_msgs >= 0xFFFFFFFFull)
    return srv_fail(KB_EINVAL, "max_step_msgs must be in [1, 2^32)");
  if (cfg->steps_in_flight < 1 || cfg->steps_in_flight > 8)
    return srv_fail(KB_EINVAL, "steps_in_flight must be 1..8");
  if (cfg->flags & ~static_cast<uint32_t>(KB_SERVER_EAGER)) return srv_fail(KB_EINVAL, "unknown flags");
  if (!cfg->executor && !cfg->d_pool && cfg->pool_bytes)
    return srv_fail(KB_EINVAL, "d_pool is NULL");
  kb_server* s = new kb_server();
  s->cfg = *cfg;
  const uint64_t m = cfg->max_step_msgs;
  s->slots.resize(cfg->steps_in_flight);
  bool ok = true;
  if (!cfg->executor) {
    ok = hipGetDevice(&s->device) == hipSuccess;
    for (StepSlot& st : s->slots) {
      if (!ok) break;
      ok = hipHostMalloc(reinterpret_cast<void**>(&st.h_offs), m * 8, 0) == hipSuccess &&
           hipHostMalloc(reinterpret_cast<void**>(&st.h_lens), m * 8, 0) == hipSuccess &&
           hipHostMalloc(reinterpret_cast<void**>(&st.h_vars), m, 0) == hipSuccess &&
           hipHostMalloc(reinterpret_cast<void**>(&st.h_out), m * 64, 0) == hipSuccess &&
           hipMalloc(reinterpret_cast<void**>(&st.d_offs), m * 8) == hipSuccess &&
           hipMalloc(reinterpret_cast<void**>(&st.d_lens), m * 8) == hipSuccess &&
           hipMalloc(reinterpret_cast<void**>(&st.d_vars), m) == hipSuccess &&
           hipMalloc(reinterpret_cast<void**>(&st.d_out), m * 64) == hipSuccess &&
           hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&st.done, hipEventDisableTiming) == hipSuccess;
      if (ok && (cfg->flags & KB_SERVER_EAGER)) ok = keccak_reserve(m, 0, st.stream) == KB_OK;
      if (ok && !(cfg->flags & KB_SERVER_EAGER))
        ok = hipHostMalloc(reinterpret_cast<void**>(&st.h_count), 4, 0) == hipSuccess &&
             hipMalloc(reinterpret_cast<void**>(&st.d_count), 4) == hipSuccess &&
             build_step_graph(s, st);
    }
  } else {
    for (StepSlot& st : s->slots) {
      st.h_offs = new uint64_t[m];
      st.h_lens = new uint64_t[m];
      st.h_vars = new uint8_t[m];
      st.h_out = new uint8_t[m * 64];
    }
  }
  if (!ok) {
    (void)hipGetLastError();
    free_slots(s);
    delete s;
    return srv_fail(KB_ENOMEM, "could not allocate the server's step buffers");
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return KB_OK;
}

int keccak_server_submit(kb_server* s, int variant, const uint64_t* h_offsets,
                     const uint64_t* h_lengths, uint64_t n, uint64_t* request_id) {
  g_srv_err.clear();
  if (!s || !request_id || (n && (!h_offsets || !h_lengths))) return srv_fail(KB_EINVAL, "NULL argument");
  if (variant < 0 || variant > 3) return srv_fail(KB_EINVAL, "variant out of range");
  if (n == 0) return srv_fail(KB_EINVAL, "a request needs at least one message");
  if (n > s->cfg.max_step_msgs) {
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->rejected;
    return srv_fail(KB_ENOMEM, "request has more messages than a step holds");
  }
  uint64_t bytes = 0;
  for (uint64_t i = 0; i < n; ++i) {
    if (h_offsets[i] > s->cfg.pool_bytes || h_lengths[i] > s->cfg.pool_bytes - h_offsets[i])
      return srv_fail(KB_EINVAL, "a message lies outside the pool");
    bytes += h_lengths[i];
  }
  if (s->cfg.max_step_bytes && bytes > s->cfg.max_step_bytes) {
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->rejected;
    return srv_fail(KB_ENOMEM, "request has more message bytes than a step holds");
  }
  Request* r = new Request();
  r->variant = variant;
  r->bytes = bytes;
  r->offs.assign(h_offsets, h_offsets + n);
  r->lens.assign(h_lengths, h_lengths + n);
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete r;
      return srv_fail(KB_EINVAL, "server is shutting down");
    }
    r->id = s->next_id++;
    *request_id = r->id;
    s->pending.push_back(r);
  }
  s->cv.notify_all();
  return KB_OK;
}

int keccak_server_poll(kb_server* s, uint64_t* ids, uint64_t max_ids, uint64_t* count, int wait_ms) {
  g_srv_err.clear();
  if (!s || !count || (max_ids && !ids)) return srv_fail(KB_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ms > 0)
    s->cv.wait_for(lk, std::chrono::milliseconds(wait_ms), [s] { return !s->done.empty(); });
  uint64_t c = 0;
  for (auto& kv : s->done) {
    if (c == max_ids) break;
    ids[c++] = kv.first;
  }
  *count = c;
  return s->error.empty() ? KB_OK : srv_fail(KB_EHIP, s->error.c_str());
}

int keccak_server_result(kb_server* s, uint64_t id, uint8_t* h_out, uint64_t out_bytes,
                     double* latency_ms) {
  g_srv_err.clear();
  if (!s) return srv_fail(KB_EINVAL, "NULL server");
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->done.find(id);
    if (it == s->done.end()) return srv_fail(KB_EINVAL, "request is unknown or not finished");
    r = it->second;
    if (h_out && out_bytes < r->digests.size()) return srv_fail(KB_EINVAL, "output buffer too small");
    s->done.erase(it);
  }
  const int status = r->status;
  if (h_out) std::memcpy(h_out, r->digests.data(), r->digests.size());
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  delete r;
  return status == KB_OK ? KB_OK : srv_fail(status, "the step holding this request failed");
}

int keccak_server_stats(kb_server* s, kb_server_stats* out) {
  g_srv_err.clear();
  if (!s || !out) return srv_fail(KB_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out->steps = s->steps;
  out->messages = s->msgs;
  out->bytes = s->bytes;
  out->completed = s->completed;
  out->rejected = s->rejected;
  out->pending = s->pending.size();
  out->max_step_msgs_seen = s->max_step_msgs_seen;
  out->step_busy_s = s->busy_s;
  out->span_s = s->any_launch ? std::chrono::duration<double>(s->t_last_done - s->t_first_launch).count() : 0.0;
  return KB_OK;
}

int keccak_server_destroy(kb_server* s) {
  g_srv_err.clear();
  if (!s) return KB_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->done) delete kv.second;
  for (Request* r : s->pending) delete r;
  free_slots(s);
  delete s;
  return KB_OK;
}

const char* keccak_server_last_error(void) { return g_srv_err.c_str(); }

}  // extern "C"
