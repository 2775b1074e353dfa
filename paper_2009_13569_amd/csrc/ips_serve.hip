// Serving scheduler over the batched sort (ips_sort_batch): replays an
// arrival trace of sort requests whose data is already in device memory,
// admits waiting requests by an HBM budget and sorts each round's admitted
// requests in one batched call per element type and algorithm.  Host code
// only; every sort runs in the library's kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <deque>
#include <thread>
#include <vector>

#include "../../include/ips.h"

extern "C" __attribute__((visibility("hidden"))) size_t ips_internal_ws_bound(uint64_t n, uint64_t nseg, int type, int algo,
                                        const ips_params* params);

namespace {

uint32_t elem_size(int t) {
  switch (t) {
    case IPS_U32: return 4;
    case IPS_U64: return 8;
    case IPS_F64: return 8;
    case IPS_PAIR_U64_U64: return 16;
    case IPS_REC100: return 100;
    default: return 0;
  }
}

using Clock = std::chrono::steady_clock;

double since(Clock::time_point t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

void wait_until(Clock::time_point t0, double t) {
  for (;;) {
    const double left = t - since(t0);
    if (left <= 0) return;
    if (left > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(left - 1e-4));
  }
}

// (type, algo) group of one round: element sum and request count.
struct Group {
  int type, algo;
  uint64_t elems, count;
  std::vector<uint32_t> reqs;
};

int error_detail(ips_ctx* ctx, int rc) {
  if (rc == IPS_E_DEVICE) return ips_last_device_error(ctx);
  if (rc == IPS_E_HIP) return ips_last_hip_error(ctx);
  return 0;
}

int sort_one(ips_ctx* ctx, ips_request& q, void* ws, size_t ws_bytes, const ips_params* params,
             void* stream) {
  if (q.elem_type == IPS_PAIR_U64_U64 || q.elem_type == IPS_REC100)
    return ips_sort_pairs(ctx, q.d_data, q.n, q.elem_type, q.algo, ws, ws_bytes, params, stream);
  return ips_sort_keys(ctx, q.d_data, q.n, q.elem_type, q.algo, ws, ws_bytes, params, stream);
}

}  // namespace

extern "C" {

int ips_serve_workspace_bytes(const ips_request* reqs, uint32_t nreq, const ips_serve_config* cfg,
                              const ips_params* params, size_t* out_bytes) {
  if (!out_bytes || !cfg || (nreq && !reqs)) return IPS_E_INVALID_ARG;
  *out_bytes = 0;
  for (uint32_t i = 0; i < nreq; ++i) {
    const uint32_t D = elem_size(reqs[i].elem_type);
    if (!D) return IPS_E_INVALID_ARG;
    if (reqs[i].algo == IPS_RADIX && reqs[i].elem_type == IPS_REC100) return IPS_E_UNSUPPORTED;
    // A batch of this type holds at most budget / D elements.
    const uint64_t nmax = std::max<uint64_t>(reqs[i].n, cfg->hbm_budget / D);
    const size_t b = ips_internal_ws_bound(nmax, nreq, reqs[i].elem_type, reqs[i].algo, params);
    *out_bytes = std::max(*out_bytes, b);
  }
  return IPS_OK;
}

int ips_serve_trace(ips_ctx* ctx, ips_request* reqs, uint32_t nreq, const ips_serve_config* cfg,
                    void* d_ws, size_t ws_bytes, const ips_params* params, void* stream) {
  if (!ctx || !cfg || (nreq && !reqs)) return IPS_E_INVALID_ARG;
  if (cfg->policy != IPS_SERVE_BATCH && cfg->policy != IPS_SERVE_FIFO) return IPS_E_INVALID_ARG;
  if (params && (params->flags & IPS_FLAG_LEVEL1_ONLY)) return IPS_E_INVALID_ARG;
  for (uint32_t i = 0; i < nreq; ++i) {
    if (!elem_size(reqs[i].elem_type)) return IPS_E_INVALID_ARG;
    if (reqs[i].algo != IPS_SAMPLESORT && reqs[i].algo != IPS_RADIX) return IPS_E_INVALID_ARG;
    if (!(reqs[i].arrival_s >= 0)) return IPS_E_INVALID_ARG;
    reqs[i].start_s = reqs[i].done_s = -1.0;
    reqs[i].status = 1;   // pending
    reqs[i].batch = 0xFFFFFFFFu;
    reqs[i].detail = 0;
  }
  std::vector<uint32_t> order(nreq);
  for (uint32_t i = 0; i < nreq; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
  const Clock::time_point t0 = Clock::now();
  std::deque<uint32_t> waiting;
  uint32_t next = 0, done = 0, batch = 0;
  int first_error = IPS_OK;
  while (done < nreq) {
    const double t = since(t0);
    while (next < nreq && reqs[order[next]].arrival_s <= t) waiting.push_back(order[next++]);
    if (waiting.empty()) {
      wait_until(t0, reqs[order[next]].arrival_s);
      continue;
    }
    if (cfg->policy == IPS_SERVE_FIFO) {
      ips_request& q = reqs[waiting.front()];
      waiting.pop_front();
      q.start_s = since(t0);
      q.status = sort_one(ctx, q, d_ws, ws_bytes, params, stream);
      q.done_s = since(t0);
      q.detail = error_detail(ctx, q.status);
      q.batch = batch++;
      if (q.status != IPS_OK && first_error == IPS_OK) first_error = q.status;
      ++done;
      continue;
    }
    // Admission in arrival order while the round's data plus the largest
    // workspace of its groups stays within the budget (no overtaking, so
    // a large request is not starved by later small ones).
    std::vector<Group> groups;
    uint64_t data_bytes = 0;
    size_t ws_need = 0;
    uint32_t admitted = 0;
    while (!waiting.empty()) {
      const uint32_t id = waiting.front();
      ips_request& q = reqs[id];
      const uint64_t bytes = q.n * (uint64_t)elem_size(q.elem_type);
      const size_t alone = ips_internal_ws_bound(q.n, 1, q.elem_type, q.algo, params);
      if (bytes + alone > cfg->hbm_budget || alone > ws_bytes) {   // can never be admitted
        waiting.pop_front();
        q.status = IPS_E_WORKSPACE;
        q.start_s = q.done_s = since(t0);
        if (first_error == IPS_OK) first_error = IPS_E_WORKSPACE;
        ++done;
        continue;
      }
      if (cfg->max_batch && admitted >= cfg->max_batch) break;
      Group* g = nullptr;
      for (Group& x : groups)
        if (x.type == q.elem_type && x.algo == q.algo) g = &x;
      const uint64_t ge = (g ? g->elems : 0) + q.n, gc = (g ? g->count : 0) + 1;
      const size_t gws = ips_internal_ws_bound(ge, gc, q.elem_type, q.algo, params);
      const size_t ws_new = std::max(ws_need, gws);
      if (admitted && (data_bytes + bytes + ws_new > cfg->hbm_budget || ws_new > ws_bytes)) break;
      if (!g) {
        groups.push_back(Group{q.elem_type, q.algo, 0, 0, {}});
        g = &groups.back();
      }
      g->elems = ge;
      g->count = gc;
      g->reqs.push_back(id);
      data_bytes += bytes;
      ws_need = ws_new;
      ++admitted;
      waiting.pop_front();
    }
    for (Group& g : groups) {
      std::vector<void*> ptrs;
      std::vector<uint64_t> ns;
      for (uint32_t id : g.reqs) { ptrs.push_back(reqs[id].d_data); ns.push_back(reqs[id].n); }
      const double ts = since(t0);
      const int rc = ips_sort_batch(ctx, ptrs.data(), ns.data(), (uint32_t)ptrs.size(), g.type, g.algo,
                                    d_ws, ws_bytes, params, stream);
      const double te = since(t0);
      const int det = error_detail(ctx, rc);
      for (uint32_t id : g.reqs) {
        reqs[id].detail = det;
        reqs[id].start_s = ts;
        reqs[id].done_s = te;
        reqs[id].status = rc;
        reqs[id].batch = batch;
      }
      if (rc != IPS_OK && first_error == IPS_OK) first_error = rc;
      done += (uint32_t)g.reqs.size();
      ++batch;
    }
  }
  return first_error;
}

}  // extern "C"
