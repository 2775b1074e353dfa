// Serving: replays an arrival trace of sort requests whose data is already
// in device memory.  IPS_SERVE_BATCH runs the continuous-batching engine of
// the host orchestrator (requests admitted into running per-type task
// queues as they arrive); IPS_SERVE_FIFO sorts one request per call in
// arrival order, the comparison baseline.  Host code only; every sort runs
// in the library's kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/ips.h"

extern "C" __attribute__((visibility("hidden"))) size_t ips_internal_ws_bound(uint64_t n, uint64_t nseg, int type, int algo,
                                        const ips_params* params);
extern "C" __attribute__((visibility("hidden"))) int ips_internal_serve_continuous(
    ips_ctx* ctx, ips_request* reqs, uint32_t nreq, const ips_serve_config* cfg, void* d_ws, size_t ws_bytes,
    const ips_params* params);
extern "C" __attribute__((visibility("hidden"))) int ips_internal_serve_ws(const ips_request* reqs, uint32_t nreq,
                                                                           uint64_t budget, const ips_params* params,
                                                                           size_t* out);

namespace {

uint32_t elem_size(int t) {
  switch (t) {
    case IPS_U32: return 4;
    case IPS_U64: return 8;
    case IPS_F64: return 8;
    case IPS_PAIR_U64_U64: return 16;
    case IPS_REC100: return 100;
    case IPS_QUARTET: return 32;
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

int error_detail(ips_ctx* ctx, int rc) {
  if (rc == IPS_E_DEVICE) return ips_last_device_error(ctx);
  if (rc == IPS_E_HIP) return ips_last_hip_error(ctx);
  return 0;
}

int sort_one(ips_ctx* ctx, ips_request& q, void* ws, size_t ws_bytes, const ips_params* params,
             void* stream) {
  if (q.elem_type == IPS_PAIR_U64_U64 || q.elem_type == IPS_REC100 || q.elem_type == IPS_QUARTET)
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
    if (reqs[i].algo != IPS_SAMPLESORT && reqs[i].algo != IPS_RADIX) return IPS_E_INVALID_ARG;
    if (reqs[i].algo == IPS_RADIX && (reqs[i].elem_type == IPS_REC100 || reqs[i].elem_type == IPS_QUARTET)) return IPS_E_UNSUPPORTED;
    // one call per request: the largest request alone
    *out_bytes = std::max(*out_bytes, ips_internal_ws_bound(reqs[i].n, 1, reqs[i].elem_type, reqs[i].algo, params));
  }
  // continuous batching: every lane's slice
  size_t lanes = 0;
  if (int e = ips_internal_serve_ws(reqs, nreq, cfg->hbm_budget, params, &lanes)) return e;
  *out_bytes = std::max(*out_bytes, lanes);
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
  if (cfg->policy == IPS_SERVE_BATCH) {
    for (uint32_t i = 0; i < nreq; ++i)
      if (reqs[i].algo == IPS_RADIX && (reqs[i].elem_type == IPS_REC100 || reqs[i].elem_type == IPS_QUARTET)) return IPS_E_UNSUPPORTED;
    return ips_internal_serve_continuous(ctx, reqs, nreq, cfg, d_ws, ws_bytes, params);
  }
  // One call per request, in arrival order (the comparison baseline).
  std::vector<uint32_t> order(nreq);
  for (uint32_t i = 0; i < nreq; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
  const Clock::time_point t0 = Clock::now();
  uint32_t next = 0, batch = 0;
  int first_error = IPS_OK;
  while (next < nreq) {
    ips_request& q = reqs[order[next++]];
    wait_until(t0, q.arrival_s);
    q.start_s = since(t0);
    q.status = sort_one(ctx, q, d_ws, ws_bytes, params, stream);
    q.done_s = since(t0);
    q.detail = error_detail(ctx, q.status);
    q.batch = batch++;
    if (q.status != IPS_OK && first_error == IPS_OK) first_error = q.status;
  }
  return first_error;
}

}  // extern "C"
