// Launcher table for one element type.  Included once per type by the
// ips_kern_<type>.hip translation units.
#pragma once
#include "ips_kernels.hpp"
#include "ips_launch.hpp"
#include "ips_lds_tier.hpp"
#include "ips_oop.hpp"
#include "ips_fused.hpp"

#include <type_traits>

namespace ips {

// LDS-tier shapes per type: (threads, keys per thread) of three variants of
// increasing capacity (a task runs on the smallest variant that holds it),
// and NET: bins hold about NET/4 keys and are sorted in registers up to
// NET/2 keys.  Keys with indices (Pair) take the smaller networks: with
// NET = 32 their (key, index) networks spilled registers and the tier ran
// a third slower (2.5 against 1.9 ms for 2^27 Pairs), while 8-byte keys
// alone ran it twice as long with NET = 16; 4-byte keys fit networks of 32
// keys per lane without spills (1.25 -> 1.22 ms for 2^28 u32).
template <class T> struct LdsShape;
template <> struct LdsShape<TU32> {
  static constexpr uint32_t N0 = 256, E0 = 16, N1 = 512, E1 = 16, N2 = 1024, E2 = 16, NET = 64;
};
template <> struct LdsShape<TU64> {
  static constexpr uint32_t N0 = 256, E0 = 16, N1 = 512, E1 = 16, N2 = 1024, E2 = 16, NET = 32;
};
template <> struct LdsShape<TF64> {
  static constexpr uint32_t N0 = 256, E0 = 16, N1 = 512, E1 = 16, N2 = 1024, E2 = 16, NET = 32;
};
template <> struct LdsShape<TPair> {
  static constexpr uint32_t N0 = 256, E0 = 8, N1 = 512, E1 = 8, N2 = 1024, E2 = 8, NET = 16;
};
template <> struct LdsShape<TRec100> {
  static constexpr uint32_t N0 = 256, E0 = 4, N1 = 256, E1 = 4, N2 = 256, E2 = 4, NET = 16;
};
// The Quartet's tier is the bitonic kernel (capacities 512, 1024, 2048).
template <> struct LdsShape<TQuartet> {
  static constexpr uint32_t N0 = 256, E0 = 2, N1 = 256, E1 = 4, N2 = 256, E2 = 8, NET = 32;
};

template <class T>
struct LaunchImpl {
  using SH = LdsShape<T>;
  static constexpr uint32_t CAP0 = SH::N0 * SH::E0, CAP1 = SH::N1 * SH::E1, CAP2 = SH::N2 * SH::E2;

  static hipError_t sample_(const BatchArgs& a, uint32_t nt, uint64_t seed, hipStream_t st) {
    if (!nt) return hipSuccess;
    hipLaunchKernelGGL((k_sample<T>), dim3(nt), dim3(SMP_THREADS), 0, st, a, seed);
    return hipGetLastError();
  }
  static hipError_t classify(const BatchArgs& a, uint32_t nwg, uint32_t dyn, bool gbuf, hipStream_t st) {
    if (!nwg) return hipSuccess;
    static bool attr_done = false;
    if (!attr_done) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_classify<T, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(T::BUF_BYTES + MAX_NB * BUF_PAD_DW * 4));
      attr_done = true;
    }
    if (gbuf)
      hipLaunchKernelGGL((k_classify<T, true>), dim3(nwg), dim3(CLS_THREADS), 0, st, a);
    else
      hipLaunchKernelGGL((k_classify<T, false>), dim3(nwg), dim3(CLS_THREADS), dyn, st, a);
    return hipGetLastError();
  }
  // Workgroups of 128, 256 or 512 threads (the tuning table picks one).
  static hipError_t permute(const BatchArgs& a, uint32_t nwg, uint32_t threads, hipStream_t st) {
    if (!nwg) return hipSuccess;
    if (threads == 128) hipLaunchKernelGGL((k_permute<T, 128>), dim3(nwg), dim3(128), 0, st, a);
    else if (threads == 512) hipLaunchKernelGGL((k_permute<T, 512>), dim3(nwg), dim3(512), 0, st, a);
    else if (threads == 256) hipLaunchKernelGGL((k_permute<T, 256>), dim3(nwg), dim3(256), 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  static hipError_t cleanup_a(const BatchArgs& a, uint32_t nt, hipStream_t st) {
    if (!nt) return hipSuccess;
    hipLaunchKernelGGL((k_cleanup_a<T>), dim3(nt), dim3(CLN_THREADS), 0, st, a);
    return hipGetLastError();
  }
  static hipError_t cleanup_b(const BatchArgs& a, uint32_t nwg, uint32_t max_w, hipStream_t st) {
    if (!nwg) return hipSuccess;
    const size_t dyn = (size_t)(max_w + 3) * sizeof(uint64_t);
    hipLaunchKernelGGL((k_cleanup_b<T>), dim3(nwg), dim3(CLN_THREADS), dyn, st, a, max_w);
    return hipGetLastError();
  }
  template <uint32_t N, uint32_t E>
  static hipError_t lds_launch(const LTask* lt, uint32_t nt, uint32_t* data, uint32_t* ctrl,
                               const uint32_t* cnt, uint32_t cnt_cap, uint32_t* pop, hipStream_t st) {
    if constexpr (std::is_same_v<T, TQuartet>) {
      constexpr uint32_t C = N * E;
      static bool qattr = false;
      static uint32_t qres = 0;
      const size_t dyn = lds_bitonic_bytes<T, C>();
      if (!qattr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lds_bitonic<T, C>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
        int per_cu = 0, cus = 0, dev = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_lds_bitonic<T, C>),
                                                         256, dyn) == hipSuccess &&
            per_cu > 0 && cus > 0)
          qres = (uint32_t)(per_cu * cus);
        qattr = true;
      }
      if (cnt && qres && nt > qres) nt = qres;
      hipLaunchKernelGGL((k_lds_bitonic<T, C>), dim3(nt), dim3(256), dyn, st, lt, data, ctrl, cnt, cnt_cap, pop);
      return hipGetLastError();
    } else {
    static bool attr_done = false;
    static uint32_t resident = 0;   // workgroups of this kernel the device holds at once
    const size_t dyn = LdsTier<T, N, E, SH::NET>::lds_bytes();
    if (!attr_done) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lds_tier<T, N, E, SH::NET>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
      int per_cu = 0, cus = 0, dev = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(
                                                           &k_lds_tier<T, N, E, SH::NET>), (int)N, dyn) ==
              hipSuccess &&
          per_cu > 0 && cus > 0)
        resident = (uint32_t)(per_cu * cus);
      attr_done = true;
    }
    // Claiming workgroups (device count): more than the resident ones only
    // add empty launches.
    if (cnt && resident && nt > resident) nt = resident;
    hipLaunchKernelGGL((k_lds_tier<T, N, E, SH::NET>), dim3(nt), dim3(N), dyn, st, lt, data, ctrl, cnt,
                       cnt_cap, pop);
    return hipGetLastError();
    }
  }
  // nt workgroups; with `cnt` (a device count) they claim the list's tasks
  // through the variant's counter ctrl[CTRL_LDSPOP + variant] (zero at launch).
  static hipError_t lds_sort(const LTask* lt, uint32_t nt, uint32_t* data, uint32_t variant, uint32_t* ctrl,
                             const uint32_t* cnt, uint32_t cnt_cap, hipStream_t st) {
    if (!nt) return hipSuccess;
    if (variant == LDS_INSERTION) {   // the paper's insertion-sort base case, one task per thread
      uint32_t g = (nt + 255) / 256;
      if (g > 2048) g = 2048;
      hipLaunchKernelGGL((k_insertion<T>), dim3(g), dim3(256), 0, st, lt, nt, data, ctrl, cnt, cnt_cap);
      return hipGetLastError();
    }
    if (variant > 2) return hipErrorInvalidValue;
    uint32_t* pop = cnt ? ctrl + CTRL_LDSPOP + variant : nullptr;
    if (variant == 2) return lds_launch<SH::N2, SH::E2>(lt, nt, data, ctrl, cnt, cnt_cap, pop, st);
    if (variant == 1) return lds_launch<SH::N1, SH::E1>(lt, nt, data, ctrl, cnt, cnt_cap, pop, st);
    return lds_launch<SH::N0, SH::E0>(lt, nt, data, ctrl, cnt, cnt_cap, pop, st);
  }
  static hipError_t sorted_sample(const uint32_t* data, uint64_t n, uint32_t* ctrl, hipStream_t st) {
    hipLaunchKernelGGL((k_sorted_sample<T>), dim3(64), dim3(1024), 0, st, data, n, ctrl);
    return hipGetLastError();
  }
  static hipError_t sorted_check(const uint32_t* data, uint64_t n, uint32_t* ctrl, hipStream_t st) {
    uint64_t chunks = (n + 4095) / 4096;
    uint32_t g = (uint32_t)(chunks < 2048 ? (chunks ? chunks : 1) : 2048);
    hipLaunchKernelGGL((k_sorted_check<T>), dim3(g), dim3(256), 0, st, data, n, ctrl);
    return hipGetLastError();
  }
  static hipError_t reverse(uint32_t* data, uint64_t n, hipStream_t st) {
    uint64_t half = n / 2;
    uint32_t g = (uint32_t)((half + 255) / 256 < 4096 ? (half + 255) / 256 : 4096);
    if (!g) return hipSuccess;
    hipLaunchKernelGGL((k_reverse<T::DW>), dim3(g), dim3(256), 0, st, data, n);
    return hipGetLastError();
  }
  static hipError_t minmax(const uint32_t* data, uint64_t n, uint32_t* ctrl, hipStream_t st) {
    if constexpr (T::RADIX_OK) {
      uint32_t g = (uint32_t)((n + 2047) / 2048 < 2048 ? (n + 2047) / 2048 : 2048);   // 2048 elements per round
      if (!g) g = 1;
      hipLaunchKernelGGL((k_minmax<T>), dim3(g), dim3(256), 0, st, data, n, ctrl);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  static hipError_t seg_minmax(const SegItem* items, uint32_t nitems, const uint32_t* data,
                               uint64_t* smin, uint64_t* smax, hipStream_t st) {
    if constexpr (T::RADIX_OK) {
      if (!nitems) return hipSuccess;
      hipLaunchKernelGGL((k_seg_minmax<T>), dim3(nitems), dim3(256), 0, st, items, data, smin, smax);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  static hipError_t seg_order(const SegItem* items, uint32_t nitems, const uint32_t* data,
                              uint32_t* flags, hipStream_t st) {
    if (!nitems) return hipSuccess;
    hipLaunchKernelGGL((k_seg_order<T>), dim3(nitems), dim3(256), 0, st, items, data, flags);
    return hipGetLastError();
  }
  static hipError_t seg_reverse(const RevItem* items, uint32_t nitems, uint32_t* data, hipStream_t st) {
    if (!nitems) return hipSuccess;
    hipLaunchKernelGGL((k_seg_reverse<T::DW>), dim3(nitems), dim3(256), 0, st, items, data);
    return hipGetLastError();
  }
  static hipError_t oop_classify(const OopArgs& a, uint32_t nwg, hipStream_t st) {
    if (!nwg) return hipSuccess;
    hipLaunchKernelGGL((k_oop_classify<T>), dim3(nwg), dim3(OOP_THREADS), 0, st, a);
    return hipGetLastError();
  }
  static hipError_t oop_distribute(const OopArgs& a, uint32_t nwg, hipStream_t st) {
    if (!nwg) return hipSuccess;
    hipLaunchKernelGGL((k_oop_distribute<T>), dim3(nwg), dim3(OOP_THREADS), 0, st, a);
    return hipGetLastError();
  }
  static hipError_t copy_ranges(const LTask* list, uint32_t count, const uint32_t* from, uint32_t* to,
                                hipStream_t st) {
    if (!count) return hipSuccess;
    hipLaunchKernelGGL((k_copy_ranges<T::DW>), dim3(count), dim3(256), 0, st, list, from, to);
    return hipGetLastError();
  }
  static hipError_t fhist(const BatchArgs& a, uint32_t nwg, hipStream_t st) {
    if constexpr (T::RADIX_OK) {
      if (!nwg) return hipSuccess;
      hipLaunchKernelGGL((k_fhist<T>), dim3(nwg), dim3(CLS_THREADS), 0, st, a);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  static hipError_t fused(const BatchArgs& a, uint32_t nwg, uint32_t dyn, hipStream_t st) {
    if constexpr (T::RADIX_OK) {
      static bool attr_done = false;
      if (!attr_done) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(FUSED_BUF_BYTES + MAX_K * BUF_PAD_DW * 4));
        attr_done = true;
      }
      if (!nwg) return hipSuccess;
      hipLaunchKernelGGL((k_fused<T>), dim3(nwg), dim3(FUSED_THREADS), dyn, st, a);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  static const Launchers* table() {
    static const Launchers t = {
        T::CODE, (uint32_t)T::DW, (uint32_t)sizeof(typename T::Key), T::KEYS_ONLY, T::RADIX_OK,
        CAP2, {CAP0, CAP1, CAP2}, T::BUF_BYTES, &sample_, &classify, &permute, &cleanup_a, &cleanup_b, &lds_sort,
        &sorted_sample, &sorted_check, &reverse, &minmax, &seg_minmax, &seg_order, &seg_reverse,
        &oop_classify, &oop_distribute, &copy_ranges, &fhist, &fused};
    return &t;
  }
};

}  // namespace ips
