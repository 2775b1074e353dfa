// Per-element-type kernel launchers (one table per type, defined in the
// per-type translation units).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ips_common.hpp"

namespace ips {

struct OopArgs;

struct Launchers {
  int code;
  uint32_t dw;            // dwords per element
  uint32_t key_slot;      // bytes of a key in StepRec slots actually used
  bool keys_only, radix_ok;
  uint32_t lds_cap;       // LDS-tier capacity (elements)
  uint32_t lds_caps[3];   // capacities of the three LDS-tier variants (ascending)
  uint32_t buf_bytes;     // LDS of the classification's buffer blocks
  hipError_t (*sample)(const BatchArgs&, uint32_t ntask, uint64_t seed, hipStream_t);
  hipError_t (*classify)(const BatchArgs&, uint32_t nwg, uint32_t dyn_lds, bool gbuf, hipStream_t);
  hipError_t (*permute)(const BatchArgs&, uint32_t nwg, uint32_t threads, hipStream_t);
  hipError_t (*cleanup_a)(const BatchArgs&, uint32_t ntask, hipStream_t);
  hipError_t (*cleanup_b)(const BatchArgs&, uint32_t nwg, uint32_t max_w, hipStream_t);
  hipError_t (*lds_sort)(const LTask*, uint32_t nt, uint32_t* data, uint32_t variant, uint32_t* ctrl,
                         const uint32_t* cnt, uint32_t cnt_cap, hipStream_t);
  hipError_t (*sorted_sample)(const uint32_t* data, uint64_t n, uint32_t* ctrl, hipStream_t);
  hipError_t (*sorted_check)(const uint32_t* data, uint64_t n, uint32_t* ctrl, hipStream_t);
  hipError_t (*reverse)(uint32_t* data, uint64_t n, hipStream_t);
  hipError_t (*minmax)(const uint32_t* data, uint64_t n, uint32_t* ctrl, hipStream_t);
  hipError_t (*seg_minmax)(const SegItem* items, uint32_t nitems, const uint32_t* data,
                           uint64_t* smin, uint64_t* smax, hipStream_t);
  hipError_t (*seg_order)(const SegItem* items, uint32_t nitems, const uint32_t* data,
                          uint32_t* flags, hipStream_t);
  hipError_t (*seg_reverse)(const RevItem* items, uint32_t nitems, uint32_t* data, hipStream_t);
  // out-of-place partitioning step (ablation)
  hipError_t (*oop_classify)(const OopArgs&, uint32_t nwg, hipStream_t);
  hipError_t (*oop_distribute)(const OopArgs&, uint32_t nwg, hipStream_t);
  hipError_t (*copy_ranges)(const LTask* list, uint32_t count, const uint32_t* from, uint32_t* to, hipStream_t);
  // radix step with classification fused into the permutation (null for
  // types without a radix key)
  hipError_t (*fhist)(const BatchArgs&, uint32_t nwg, hipStream_t);
  hipError_t (*fused)(const BatchArgs&, uint32_t nwg, uint32_t dyn_lds, hipStream_t);
};

const Launchers* launchers_u32();
const Launchers* launchers_u64();
const Launchers* launchers_f64();
const Launchers* launchers_pair();
const Launchers* launchers_rec100();
const Launchers* launchers_quartet();

hipError_t launch_boundaries(const BatchArgs&, uint32_t ntask, uint32_t max_nb, uint32_t cmax,
                             hipStream_t);
hipError_t launch_fill32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t);
hipError_t launch_lds_decide(uint32_t* ctrl, uint32_t min_tasks, uint32_t step_cap, hipStream_t);
hipError_t launch_lds_reset(uint32_t* ctrl, hipStream_t);
hipError_t launch_children(const BatchArgs&, const ChildArgs&, uint32_t ntask, hipStream_t);
hipError_t launch_plan_pop(const BatchArgs&, const PlanCfg&, hipStream_t);
hipError_t launch_plan_geom(const BatchArgs&, const PlanCfg&, hipStream_t);
hipError_t launch_fill32_cnt(uint32_t* p, const uint32_t* count, uint32_t max_n, uint32_t v, hipStream_t);
hipError_t launch_oop_scan(const OopArgs&, uint32_t ntask, hipStream_t);
hipError_t launch_fscan(const BatchArgs&, uint32_t ntask, hipStream_t);
hipError_t launch_oop_children(const OopArgs&, uint32_t ntask, uint32_t* ctrl, CTask* next, uint32_t next_cap,
                               LTask* lds, LTask* copy, uint32_t list_cap, uint32_t cap, uint32_t to_second,
                               hipStream_t);

}  // namespace ips
