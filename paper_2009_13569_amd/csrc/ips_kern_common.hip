// Kernels that do not depend on the element type.
#define IPS_COMMON_KERNELS 1
#include "ips_kernels.hpp"
#include "ips_launch.hpp"
#include "ips_oop.hpp"
#include "ips_fused.hpp"

namespace ips {

hipError_t launch_boundaries(const BatchArgs& a, uint32_t nt, uint32_t max_nb, uint32_t cmax,
                             hipStream_t st) {
  if (!nt) return hipSuccess;
  const uint32_t gpt = (max_nb + 7) / 8;
  hipLaunchKernelGGL(k_bucket_sums, dim3(nt * gpt), dim3(512), 0, st, a, gpt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_boundaries, dim3(nt), dim3(512), 0, st, a, cmax);
  return hipGetLastError();
}

hipError_t launch_fill32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st) {
  if (!n) return hipSuccess;
  uint32_t g = (uint32_t)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_fill32, dim3(g), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_children(const BatchArgs& a, const ChildArgs& c, uint32_t nt, hipStream_t st) {
  if (!nt) return hipSuccess;
  const uint32_t grid = nt < CHILD_WGS ? nt : CHILD_WGS;
  hipLaunchKernelGGL(k_children, dim3(grid), dim3(256), 0, st, a, c, nt);
  return hipGetLastError();
}

hipError_t launch_plan_pop(const BatchArgs& a, const PlanCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_plan_pop, dim3(1), dim3(PLAN_THREADS), 0, st, a, c);
  return hipGetLastError();
}

hipError_t launch_plan_geom(const BatchArgs& a, const PlanCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_plan_geom, dim3(1), dim3(PLAN_THREADS), 0, st, a, c);
  return hipGetLastError();
}

hipError_t launch_lds_decide(uint32_t* ctrl, uint32_t min_tasks, uint32_t step_cap, hipStream_t st) {
  hipLaunchKernelGGL(k_lds_decide, dim3(1), dim3(64), 0, st, ctrl, min_tasks, step_cap);
  return hipGetLastError();
}

hipError_t launch_lds_reset(uint32_t* ctrl, hipStream_t st) {
  hipLaunchKernelGGL(k_lds_reset, dim3(1), dim3(64), 0, st, ctrl);
  return hipGetLastError();
}

hipError_t launch_fill32_cnt(uint32_t* p, const uint32_t* count, uint32_t max_n, uint32_t v, hipStream_t st) {
  if (!max_n) return hipSuccess;
  uint32_t g = (max_n + 255) / 256 < 4096 ? (max_n + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_fill32_cnt, dim3(g), dim3(256), 0, st, p, count, v);
  return hipGetLastError();
}

hipError_t launch_oop_scan(const OopArgs& a, uint32_t nt, hipStream_t st) {
  if (!nt) return hipSuccess;
  hipLaunchKernelGGL(k_oop_scan, dim3(nt), dim3(MAX_NB), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fscan(const BatchArgs& a, uint32_t nt, hipStream_t st) {
  if (!nt) return hipSuccess;
  hipLaunchKernelGGL(k_fscan, dim3(nt), dim3(MAX_K), 0, st, a, nt);
  return hipGetLastError();
}

hipError_t launch_oop_children(const OopArgs& a, uint32_t nt, uint32_t* ctrl, CTask* next, uint32_t next_cap,
                               LTask* lds, LTask* copy, uint32_t list_cap, uint32_t cap, uint32_t to_second,
                               hipStream_t st) {
  if (!nt) return hipSuccess;
  hipLaunchKernelGGL(k_oop_children, dim3(nt), dim3(256), 0, st, a, ctrl, next, next_cap, lds, copy, list_cap,
                     cap, to_second);
  return hipGetLastError();
}

}  // namespace ips
