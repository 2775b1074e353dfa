// Out-of-place partitioning step of super scalar samplesort (the algorithm
// of Sanders and Winkel that arXiv 2009.13569 re-implements on its own
// framework, Section 7 "Implementation Details", and whose I/O volume its
// appendix compares with the in-place step).  It is built here as an
// ablation of the in-place step on the same GPU, with the same sampling,
// decision tree, start table and base case:
//  - classification: every element is classified once; its bucket goes to
//    an oracle array (one byte per element, two with more than 256
//    buckets) and each workgroup counts the sizes of the buckets of its
//    stripe;
//  - a prefix sum over (bucket, stripe) gives every stripe's first position
//    in every bucket;
//  - distribution: every element and its oracle entry are read again and
//    the element is written to its bucket's range of the other array.
// A level therefore reads the elements twice, writes them once and writes
// and reads the oracle once: 3 D + 2 o bytes per element (o = oracle entry
// bytes), against 4 D for the in-place step.
#pragma once
#include "ips_kernels.hpp"

namespace ips {

constexpr uint32_t OOP_THREADS = 512;
constexpr int OOP_EPT = 4;   // elements per thread in flight

struct OopArgs {
  const uint32_t* src;        // elements of the level (dwords)
  uint32_t* dst;              // the other array
  uint8_t* oracle;            // bucket of every element of the level (o bytes each)
  const PTask* tasks;         // l, n, W, wg_base, nb, K, logK, eq, bucket_base
  const StepRec* recs;
  const uint32_t* wg_task;    // workgroup -> task
  uint32_t* cnt;              // [WG][nbs] bucket sizes, then first destinations
  uint64_t* b_start;          // [bucket_base + j], j = 0..nb: bucket starts (task-relative)
  uint32_t nbs;
};

__device__ __forceinline__ void oop_stripe(const PTask& tk, uint32_t s, uint64_t* lo, uint64_t* hi) {
  *lo = tk.n * s / tk.W;
  *hi = tk.n * (s + 1) / tk.W;
}

// Classification: bucket of every element of the stripe into the oracle,
// bucket sizes into cnt[wg].
template <class T>
__global__ void __launch_bounds__(OOP_THREADS) k_oop_classify(OopArgs a) {
  using Key = typename T::Key;
  constexpr int DW = T::DW;
  __shared__ Key s_ts[2 * MAX_K];
  __shared__ uint16_t s_start[1u << START_BITS];
  __shared__ uint32_t s_cnt[MAX_NB];
  const uint32_t tid = threadIdx.x, wg = blockIdx.x;
  const uint32_t tix = a.wg_task[wg];
  const PTask& tk = a.tasks[tix];
  const StepRec* rec = a.recs + tix;
  for (uint32_t i = tid; i < tk.K; i += OOP_THREADS) {
    s_ts[i] = T::from_slot(rec->tree[i]);
    s_ts[MAX_K + i] = T::from_slot(rec->spl[i]);
  }
  for (uint32_t i = tid; i < (1u << START_BITS); i += OOP_THREADS) s_start[i] = rec->tstart[i];
  for (uint32_t j = tid; j < tk.nb; j += OOP_THREADS) s_cnt[j] = 0;
  StartTable stab;
  stab.start = s_start;
  stab.base = rec->tbase;
  stab.shift = rec->tshift;
  __syncthreads();
  uint64_t lo, hi;
  oop_stripe(tk, wg - tk.wg_base, &lo, &hi);
  const uint32_t* gs = a.src + tk.l * DW;
  const bool wide = tk.nb > 256;
  for (uint64_t base = lo; base < hi; base += (uint64_t)OOP_THREADS * OOP_EPT) {
    Key key[OOP_EPT];
    uint32_t bk[OOP_EPT];
#pragma unroll
    for (int i = 0; i < OOP_EPT; ++i) {
      const uint64_t x = base + (uint64_t)i * OOP_THREADS + tid;
      uint32_t w[DW];
      if (x < hi) ld_elem<DW>(gs + x * DW, w);
      else
#pragma unroll
        for (int d = 0; d < DW; ++d) w[d] = 0;
      key[i] = key_of<T>(w);
    }
    tree_buckets<T, OOP_EPT>(key, s_ts, tk.logK, tk.eq, stab, bk);
#pragma unroll
    for (int i = 0; i < OOP_EPT; ++i) {
      const uint64_t x = base + (uint64_t)i * OOP_THREADS + tid;
      if (x < hi) {
        atomicAdd(&s_cnt[bk[i]], 1u);
        if (wide) reinterpret_cast<uint16_t*>(a.oracle)[tk.l + x] = (uint16_t)bk[i];
        else a.oracle[tk.l + x] = (uint8_t)bk[i];
      }
    }
  }
  __syncthreads();
  for (uint32_t j = tid; j < tk.nb; j += OOP_THREADS) a.cnt[(uint64_t)wg * a.nbs + j] = s_cnt[j];
}

#ifdef IPS_COMMON_KERNELS
// Prefix sums of one task (one workgroup, one thread per bucket): bucket
// starts, and every stripe's first position in every bucket.
__global__ void __launch_bounds__(MAX_NB) k_oop_scan(OopArgs a) {
  __shared__ uint64_t s_w[MAX_NB / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const PTask& tk = a.tasks[blockIdx.x];
  const uint32_t nb = tk.nb, W = tk.W;
  uint64_t tot = 0;
  if (tid < nb)
    for (uint32_t s = 0; s < W; ++s) tot += a.cnt[(uint64_t)(tk.wg_base + s) * a.nbs + tid];
  uint64_t inc = tot;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = (uint64_t)__shfl_up((long long)inc, o, 64);
    if ((int)lane >= o) inc += y;
  }
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  uint64_t base = 0;
  for (uint32_t w = 0; w < wave; ++w) base += s_w[w];
  const uint64_t start = base + inc - tot;
  if (tid < nb) {
    a.b_start[tk.bucket_base + tid] = start;
    uint64_t p = start;
    for (uint32_t s = 0; s < W; ++s) {
      uint32_t* c = &a.cnt[(uint64_t)(tk.wg_base + s) * a.nbs + tid];
      const uint32_t v = *c;
      *c = (uint32_t)p;   // task-relative positions fit 32 bits (tasks stay below 2^32 elements)
      p += v;
    }
  }
  if (tid == 0) a.b_start[tk.bucket_base + nb] = tk.n;
}

#endif  // IPS_COMMON_KERNELS

// Distribution: every element to the next free position of its bucket in
// the other array (positions within a bucket in arrival order).
template <class T>
__global__ void __launch_bounds__(OOP_THREADS) k_oop_distribute(OopArgs a) {
  constexpr int DW = T::DW;
  __shared__ uint32_t s_off[MAX_NB];
  const uint32_t tid = threadIdx.x, wg = blockIdx.x;
  const PTask& tk = a.tasks[a.wg_task[wg]];
  for (uint32_t j = tid; j < tk.nb; j += OOP_THREADS) s_off[j] = a.cnt[(uint64_t)wg * a.nbs + j];
  __syncthreads();
  uint64_t lo, hi;
  oop_stripe(tk, wg - tk.wg_base, &lo, &hi);
  const uint32_t* gs = a.src + tk.l * DW;
  uint32_t* gd = a.dst + tk.l * DW;
  const bool wide = tk.nb > 256;
  for (uint64_t base = lo; base < hi; base += (uint64_t)OOP_THREADS * OOP_EPT) {
    uint32_t w[OOP_EPT][DW];
    uint32_t bk[OOP_EPT];
#pragma unroll
    for (int i = 0; i < OOP_EPT; ++i) {
      const uint64_t x = base + (uint64_t)i * OOP_THREADS + tid;
      bk[i] = 0;
      if (x < hi) {
        ld_elem<DW>(gs + x * DW, w[i]);
        bk[i] = wide ? reinterpret_cast<const uint16_t*>(a.oracle)[tk.l + x] : a.oracle[tk.l + x];
      }
    }
#pragma unroll
    for (int i = 0; i < OOP_EPT; ++i) {
      const uint64_t x = base + (uint64_t)i * OOP_THREADS + tid;
      if (x < hi) {
        const uint32_t pos = atomicAdd(&s_off[bk[i]], 1u);
        st_elem<DW>(gd + (uint64_t)pos * DW, w[i]);
      }
    }
  }
}

#ifdef IPS_COMMON_KERNELS
// Children of the tasks of one out-of-place step (one workgroup per task,
// one thread per bucket): final buckets (at most one element, or an
// equality bucket), LDS-tier buckets (at most `cap` elements) and
// next-level tasks, the next level's tasks with equality buckets forced on
// when a bucket holds the whole task.  When the step wrote into the second
// array, every bucket that stays there (final or LDS tier) is also listed
// for the copy back.  Counters: ctrl[CTRL_NNEXT] next tasks,
// ctrl[CTRL_NLDS] LDS-tier tasks, ctrl[CTRL_NLDS + 1] copies.
__global__ void __launch_bounds__(256) k_oop_children(OopArgs a, uint32_t* ctrl, CTask* next, uint32_t next_cap,
                                                      LTask* lds, LTask* copy, uint32_t list_cap, uint32_t cap,
                                                      uint32_t to_second) {
  const PTask& tk = a.tasks[blockIdx.x];
  for (uint32_t j = threadIdx.x; j < tk.nb; j += 256) {
    const uint64_t s0 = a.b_start[tk.bucket_base + j];
    const uint64_t sz = a.b_start[tk.bucket_base + j + 1] - s0;
    if (!sz) continue;
    const bool eqb = tk.eq && (j & 1u) && j != 2 * tk.K - 1;
    if (sz > cap && !eqb) {
      const uint32_t q = atomicAdd(&ctrl[CTRL_NNEXT], 1u);
      if (q < next_cap) {
        CTask t;
        t.l = tk.l + s0; t.n = sz; t.level = tk.level + 1; t.tflags = sz == tk.n ? TF_EQ_ON : 0u;
        t.shift = 0; t.width = 0;
        next[q] = t;
      } else {
        dev_error(ctrl, DE_QUEUE, blockIdx.x, q);
      }
      continue;
    }
    LTask t;
    t.l = tk.l + s0; t.n = (uint32_t)sz; t.req = 0;
    if (sz >= 2 && !eqb) {
      const uint32_t q = atomicAdd(&ctrl[CTRL_NLDS], 1u);
      if (q < list_cap) lds[q] = t;
      else dev_error(ctrl, DE_CLN_RANGE, blockIdx.x, q);
    }
    if (to_second) {
      const uint32_t q = atomicAdd(&ctrl[CTRL_NLDS + 1], 1u);
      if (q < list_cap) copy[q] = t;
      else dev_error(ctrl, DE_CLN_RANGE, blockIdx.x, q);
    }
  }
}

#endif  // IPS_COMMON_KERNELS

// Copies the listed ranges (element units) from `from` to `to`: one
// workgroup per range.
template <int DW>
__global__ void __launch_bounds__(256) k_copy_ranges(const LTask* list, const uint32_t* from, uint32_t* to) {
  const LTask t = list[blockIdx.x];
  const uint64_t n = (uint64_t)t.n * DW;
  const uint32_t* s = from + t.l * DW;
  uint32_t* d = to + t.l * DW;
  for (uint64_t i = threadIdx.x; i < n; i += 256) d[i] = s[i];
}

}  // namespace ips
