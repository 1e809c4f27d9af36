// Serving form: single requests (query, k, nprobe) arrive one by one and are
// answered from device batches (continuous batching).  A worker thread keeps
// up to `lanes` batches in flight, each on its own stream with its own
// workspace, so the work of a batch admitted while others run overlaps with
// theirs on the device.  Admission takes the pending requests in arrival
// order into a new batch while a lane is free, the requests in flight stay
// within max_slots and the workspace bytes of all batches in flight (each
// request counted at its bbc_query_bytes) stay within the memory budget; a
// finished batch frees its slots and bytes for the next.  Every request's
// result is the one a search of it alone returns: the query path treats the
// queries of a batch independently.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "kernels.h"

namespace {

using Clock = std::chrono::steady_clock;

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t ticket = 0;
  std::vector<float> q;
  int32_t k = 0, nprobe = 0;
  int64_t bytes = 0;
  int64_t t_submit = 0;
};

struct Res {
  std::vector<int64_t> ids;
  std::vector<float> dists;
  bbc_request_info info{};
  std::string err;
};

// One batch in flight: stream, completion event, workspace and I/O buffers
// (device and pinned host), grown on demand and kept for the server's life.
struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char* ws = nullptr;
  size_t ws_cap = 0;
  float* dq = nullptr;
  int32_t* dcnt = nullptr;
  float* hq = nullptr;
  int32_t* hcnt = nullptr;
  int64_t* hwork = nullptr;  // [2][nq] codes scanned, exact distances computed
  size_t cap_q = 0;
  int64_t* dids = nullptr;
  float* ddist = nullptr;
  int64_t* hids = nullptr;
  float* hdist = nullptr;
  size_t cap_out = 0;

  bool busy = false;
  std::vector<Req> batch;
  std::vector<int32_t> k, nprobe;
  std::vector<int64_t> off;
  int64_t bytes = 0;

  void release() {
    if (stream) { hipStreamSynchronize(stream); hipStreamDestroy(stream); }
    if (done) hipEventDestroy(done);
    hipFree(ws); hipFree(dq); hipFree(dcnt); hipFree(dids); hipFree(ddist);
    hipHostFree(hq); hipHostFree(hcnt); hipHostFree(hwork); hipHostFree(hids); hipHostFree(hdist);
    stream = nullptr; done = nullptr;
  }

  int32_t grow(size_t nq, size_t nout, size_t wsb, int d) {
    if (wsb > ws_cap) {
      const size_t c = std::max(wsb, ws_cap + ws_cap / 2);
      hipFree(ws);
      ws = nullptr;
      ws_cap = 0;
      if (hipMalloc(reinterpret_cast<void**>(&ws), c) != hipSuccess) { ws = nullptr; return BBC_ENOMEM; }
      ws_cap = c;
    }
    if (nq > cap_q) {
      const size_t c = std::max<size_t>(nq, 2 * cap_q);
      hipFree(dq); hipFree(dcnt); hipHostFree(hq); hipHostFree(hcnt); hipHostFree(hwork);
      dq = nullptr; dcnt = nullptr; hq = nullptr; hcnt = nullptr; hwork = nullptr;
      cap_q = 0;
      if (hipMalloc(reinterpret_cast<void**>(&dq), sizeof(float) * c * d) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&dcnt), sizeof(int32_t) * c) != hipSuccess ||
          hipHostMalloc(reinterpret_cast<void**>(&hq), sizeof(float) * c * d) != hipSuccess ||
          hipHostMalloc(reinterpret_cast<void**>(&hcnt), sizeof(int32_t) * c) != hipSuccess ||
          hipHostMalloc(reinterpret_cast<void**>(&hwork), sizeof(int64_t) * 2 * c) != hipSuccess)
        return BBC_ENOMEM;
      cap_q = c;
    }
    if (nout > cap_out) {
      const size_t c = std::max(nout, cap_out + cap_out / 2);
      hipFree(dids); hipFree(ddist); hipHostFree(hids); hipHostFree(hdist);
      dids = nullptr; ddist = nullptr; hids = nullptr; hdist = nullptr;
      cap_out = 0;
      if (hipMalloc(reinterpret_cast<void**>(&dids), sizeof(int64_t) * c) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&ddist), sizeof(float) * c) != hipSuccess ||
          hipHostMalloc(reinterpret_cast<void**>(&hids), sizeof(int64_t) * c) != hipSuccess ||
          hipHostMalloc(reinterpret_cast<void**>(&hdist), sizeof(float) * c) != hipSuccess)
        return BBC_ENOMEM;
      cap_out = c;
    }
    return BBC_OK;
  }
};

}  // namespace

struct bbc_server {
  bbc_index* ix = nullptr;
  bbc_search_params prm{};
  int64_t budget = 0;
  int32_t max_slots = 0;
  int32_t d = 0;
  int device = 0;
  std::vector<Lane> lanes;

  // shared with the submitting threads (under mu)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::deque<Req> pending;
  std::unordered_set<uint64_t> outstanding;  // submitted, not yet filed
  std::unordered_map<uint64_t, Res> done;
  uint64_t next_ticket = 1;
  int64_t n_batches = 0, n_requests = 0, max_batch = 0, max_inflight = 0;
  std::thread worker;

  // worker thread only
  int64_t inflight_bytes = 0;
  int64_t inflight_reqs = 0;

  // Enqueue a lane's batch: query upload, search, result download, event.
  int32_t launch(Lane& L) {
    const size_t nq = L.batch.size();
    L.k.resize(nq);
    L.nprobe.resize(nq);
    L.off.assign(nq + 1, 0);
    for (size_t i = 0; i < nq; ++i) {
      L.k[i] = L.batch[i].k;
      L.nprobe[i] = L.batch[i].nprobe;
      L.off[i + 1] = L.off[i] + L.batch[i].k;
    }
    bbc_search_params p = prm;
    p.device_io = 1;
    p.stream = L.stream;
    size_t wsb = 0;
    int32_t rc = bbc::search_in_workspace(ix, nullptr, (int64_t)nq, L.k.data(), L.nprobe.data(), &p, L.off.data(),
                                          nullptr, nullptr, nullptr, nullptr, &wsb);
    if (rc) return rc;
    rc = L.grow(nq, (size_t)L.off[nq], wsb, d);
    if (rc) return bbc::set_error(rc, "server buffer allocation failed");
    for (size_t i = 0; i < nq; ++i) std::memcpy(L.hq + i * d, L.batch[i].q.data(), sizeof(float) * d);
    if (hipMemcpyAsync(L.dq, L.hq, sizeof(float) * nq * d, hipMemcpyHostToDevice, L.stream) != hipSuccess)
      return bbc::set_error(BBC_EDEVICE, "query upload failed");
    rc = bbc::search_in_workspace(ix, L.dq, (int64_t)nq, L.k.data(), L.nprobe.data(), &p, L.off.data(), L.dids,
                                  L.ddist, L.dcnt, L.ws, &wsb, L.hwork);
    if (rc) return rc;
    const int64_t nout = L.off[nq];
    if (hipMemcpyAsync(L.hids, L.dids, sizeof(int64_t) * nout, hipMemcpyDeviceToHost, L.stream) != hipSuccess ||
        hipMemcpyAsync(L.hdist, L.ddist, sizeof(float) * nout, hipMemcpyDeviceToHost, L.stream) != hipSuccess ||
        hipMemcpyAsync(L.hcnt, L.dcnt, sizeof(int32_t) * nq, hipMemcpyDeviceToHost, L.stream) != hipSuccess ||
        hipEventRecord(L.done, L.stream) != hipSuccess)
      return bbc::set_error(BBC_EDEVICE, "result download failed");
    return BBC_OK;
  }

  // File a lane's results (or its failure) under the tickets; frees the lane.
  void finish(Lane& L, int32_t status, const char* err) {
    const int64_t t = now_ns();
    {
      std::lock_guard<std::mutex> lk(mu);
      const size_t nq = L.batch.size();
      for (size_t i = 0; i < nq; ++i) {
        Res r;
        r.info.status = status;
        r.info.latency_ns = t - L.batch[i].t_submit;
        r.info.batch_size = (int64_t)nq;
        if (status == BBC_OK) {
          r.ids.assign(L.hids + L.off[i], L.hids + L.off[i + 1]);
          r.dists.assign(L.hdist + L.off[i], L.hdist + L.off[i + 1]);
          r.info.count = L.hcnt[i];
          r.info.n_scanned = L.hwork[i];
          r.info.n_reranked = L.hwork[nq + i];
        } else {
          r.err = err ? err : "";
        }
        outstanding.erase(L.batch[i].ticket);
        done[L.batch[i].ticket] = std::move(r);
      }
      n_batches += 1;
      n_requests += (int64_t)L.batch.size();
    }
    inflight_bytes -= L.bytes;
    inflight_reqs -= (int64_t)L.batch.size();
    L.batch.clear();
    L.busy = false;
    cv_done.notify_all();
  }

  // Files the finished lanes; returns whether a lane is still busy.
  bool harvest() {
    bool any = false;
    for (Lane& L : lanes) {
      if (!L.busy) continue;
      const hipError_t e = hipEventQuery(L.done);
      if (e == hipSuccess) {
        finish(L, BBC_OK, nullptr);
      } else if (e != hipErrorNotReady) {
        finish(L, BBC_EDEVICE, "batch failed on the device");
      } else {
        any = true;
      }
    }
    return any;
  }

  void run() {
    hipSetDevice(device);
    while (true) {
      const bool busy = harvest();
      Lane* free_lane = nullptr;
      for (Lane& L : lanes)
        if (!L.busy) { free_lane = &L; break; }
      if (free_lane) {
        Lane& L = *free_lane;
        std::unique_lock<std::mutex> lk(mu);
        if (pending.empty() && !busy) {
          cv_work.wait(lk, [&] { return stop || !pending.empty(); });
          if (pending.empty()) break;  // stopping, nothing left to answer
        }
        // admission: arrival order, slots and bytes in flight (nothing in
        // flight always admits the head: it fits the budget by itself)
        int64_t bytes = 0;
        L.batch.clear();
        while (!pending.empty() && inflight_reqs + (int64_t)L.batch.size() < max_slots &&
               inflight_bytes + bytes + pending.front().bytes <= budget) {
          bytes += pending.front().bytes;
          L.batch.push_back(std::move(pending.front()));
          pending.pop_front();
        }
        if (!L.batch.empty()) {
          L.bytes = bytes;
          inflight_bytes += bytes;
          inflight_reqs += (int64_t)L.batch.size();
          L.busy = true;
          max_batch = std::max(max_batch, (int64_t)L.batch.size());
          max_inflight = std::max(max_inflight, inflight_reqs);
          lk.unlock();
          const int32_t rc = launch(L);
          if (rc != BBC_OK) {
            const std::string msg = bbc_last_error();
            hipStreamSynchronize(L.stream);  // whatever part was enqueued
            finish(L, rc, msg.c_str());
          }
          continue;
        }
      }
      if (!busy) continue;
      // batches in flight and nothing admissible now: wait briefly for a
      // submission, then look at the lanes again
      std::unique_lock<std::mutex> lk(mu);
      const size_t seen = pending.size();
      cv_work.wait_for(lk, std::chrono::microseconds(50), [&] { return pending.size() != seen; });
    }
  }
};

namespace {

// Under s->mu.  True if the ticket's result was filed (and is now handed out).
bool take_result(bbc_server* s, uint64_t ticket, int64_t* ids, float* dists, bbc_request_info* info,
                 int32_t* status) {
  auto it = s->done.find(ticket);
  if (it == s->done.end()) return false;
  const Res& r = it->second;
  *status = r.info.status;
  if (info) *info = r.info;
  if (r.info.status == BBC_OK) {
    if (ids) std::memcpy(ids, r.ids.data(), sizeof(int64_t) * r.ids.size());
    if (dists) std::memcpy(dists, r.dists.data(), sizeof(float) * r.dists.size());
  } else {
    bbc::set_error(r.info.status, r.err);
  }
  s->done.erase(it);
  return true;
}

}  // namespace

extern "C" {

int32_t bbc_server_create(bbc_index* ix, const bbc_search_params* params, int64_t mem_budget_bytes,
                          int32_t max_slots, int32_t lanes, bbc_server** out) {
  if (!out) return bbc::set_error(BBC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ix || !params) return bbc::set_error(BBC_EINVAL, "NULL argument");
  if (mem_budget_bytes < 1 || max_slots < 1) return bbc::set_error(BBC_EINVAL, "budget and slots must be >= 1");
  if (lanes < 0 || lanes > 8) return bbc::set_error(BBC_EINVAL, "lanes must be in [0, 8]");
  if (!(params->ncand_ratio >= 1.0)) return bbc::set_error(BBC_EINVAL, "ncand_ratio must be >= 1");
  int32_t d = 0;
  const int32_t rc = bbc_index_info(ix, nullptr, &d, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (rc) return rc;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return bbc::set_error(BBC_EDEVICE, "hipGetDevice failed");
  bbc_server* s = new bbc_server();
  s->ix = ix;
  s->prm = *params;
  s->budget = mem_budget_bytes;
  s->max_slots = max_slots;
  s->d = d;
  s->device = dev;
  s->lanes.resize(lanes ? lanes : 2);
  for (Lane& L : s->lanes) {
    if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
      for (Lane& M : s->lanes) M.release();
      delete s;
      return bbc::set_error(BBC_EDEVICE, "stream or event creation failed");
    }
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return BBC_OK;
}

int32_t bbc_server_submit(bbc_server* s, const float* q, int32_t k, int32_t nprobe, uint64_t* ticket) {
  if (!s || !q || !ticket) return bbc::set_error(BBC_EINVAL, "NULL argument");
  const int64_t bytes = bbc_query_bytes(s->ix, k, nprobe, &s->prm);
  if (bytes < 0) return (int32_t)bytes;
  if (bytes > s->budget) return bbc::set_error(BBC_ENOMEM, "request exceeds the server's memory budget");
  for (int32_t e = 0; e < s->d; ++e)
    if (!std::isfinite(q[e])) return bbc::set_error(BBC_EINVAL, "non-finite query value");
  Req r;
  r.q.assign(q, q + s->d);
  r.k = k;
  r.nprobe = nprobe;
  r.bytes = bytes;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return bbc::set_error(BBC_EINVAL, "server is stopping");
    r.t_submit = now_ns();
    r.ticket = s->next_ticket++;
    *ticket = r.ticket;
    s->outstanding.insert(r.ticket);
    s->pending.push_back(std::move(r));
  }
  s->cv_work.notify_one();
  return BBC_OK;
}

int32_t bbc_server_poll(bbc_server* s, uint64_t ticket, int64_t* ids, float* dists, bbc_request_info* info) {
  if (!s) return bbc::set_error(BBC_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t status = BBC_OK;
  if (take_result(s, ticket, ids, dists, info, &status)) return status;
  if (s->outstanding.count(ticket)) return BBC_EBUSY;
  return bbc::set_error(BBC_EINVAL, "unknown or already collected ticket");
}

int32_t bbc_server_wait(bbc_server* s, uint64_t ticket, int32_t timeout_ms, int64_t* ids, float* dists,
                        bbc_request_info* info) {
  if (!s) return bbc::set_error(BBC_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  const auto until = Clock::now() + std::chrono::milliseconds(std::max(0, timeout_ms));
  int32_t status = BBC_OK;
  while (!take_result(s, ticket, ids, dists, info, &status)) {
    if (!s->outstanding.count(ticket)) return bbc::set_error(BBC_EINVAL, "unknown or already collected ticket");
    if (s->cv_done.wait_until(lk, until) == std::cv_status::timeout) {
      if (take_result(s, ticket, ids, dists, info, &status)) return status;
      return BBC_EBUSY;
    }
  }
  return status;
}

int32_t bbc_server_stats(bbc_server* s, int64_t* batches, int64_t* requests, int64_t* max_batch,
                         int64_t* max_inflight, int64_t* pending) {
  if (!s) return bbc::set_error(BBC_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (batches) *batches = s->n_batches;
  if (requests) *requests = s->n_requests;
  if (max_batch) *max_batch = s->max_batch;
  if (max_inflight) *max_inflight = s->max_inflight;
  if (pending) *pending = (int64_t)s->pending.size();
  return BBC_OK;
}

void bbc_server_destroy(bbc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  hipSetDevice(s->device);
  for (Lane& L : s->lanes) L.release();
  delete s;
}

}  // extern "C"
