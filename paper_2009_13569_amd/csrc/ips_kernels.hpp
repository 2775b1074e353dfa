// gfx950 kernels of the in-place partitioning step of IPS4o / IPS2Ra
// (arXiv 2009.13569, Section 4.1) and the LDS-resident base case.
//
// One partitioning step on a batch of tasks runs as:
//   k_sample      sampling, splitter selection, decision tree   (Sec. 4.1)
//   k_classify    classification into per-bucket buffer blocks; full blocks
//                 are flushed to the front of the workgroup's stripe
//   k_boundaries  bucket sizes, delimiters, read/write pointer pieces
//   k_permute     block permutation with atomic read/write pointers
//   k_cleanup_a/b cleanup of bucket heads/tails (Section 4.1 "Cleanup")
// Tasks small enough for one workgroup's LDS are sorted by k_lds_tier
// (ips_lds_tier.hpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ips_common.hpp"
#include "ips_traits.hpp"

namespace ips {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ uint64_t at_load64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t at_add64(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t at_load32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void at_store32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Serving: the request that holds element l of the data (the last entry of
// the ascending table of the requests' first elements that is <= l), and
// the per-request counters of elements in their final place.
__device__ __forceinline__ uint32_t seg_find(const uint32_t* ctrl, uint32_t nseg, uint64_t l) {
  const uint64_t* lo = reinterpret_cast<const uint64_t*>((uint64_t)ctrl[CTRL_SEGLO] |
                                                         ((uint64_t)ctrl[CTRL_SEGLO + 1] << 32));
  uint32_t a = 0, b = nseg;
  while (b - a > 1) {
    const uint32_t m = (a + b) >> 1;
    if (lo[m] <= l) a = m; else b = m;
  }
  return a;
}
__device__ __forceinline__ unsigned long long* seg_done_ptr(const uint32_t* ctrl) {
  return reinterpret_cast<unsigned long long*>((uint64_t)ctrl[CTRL_SEGDONE] |
                                               ((uint64_t)ctrl[CTRL_SEGDONE + 1] << 32));
}


__device__ __forceinline__ void dev_error(uint32_t* ctrl, uint32_t code, uint32_t x,
                                          uint32_t y) {
  if (atomicCAS(&ctrl[CTRL_ERR], 0u, code) == 0u) {
    ctrl[CTRL_ERR_A] = x;
    ctrl[CTRL_ERR_B] = y;
  }
}

// SplitMix64 (Steele, Lea, Flood 2014): output j of the generator seeded
// with s is mix(s + (j+1) * gamma).
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t sm64_at(uint64_t s, uint64_t j) {
  return sm64_mix(s + (j + 1) * 0x9E3779B97F4A7C15ull);
}

__device__ __forceinline__ uint32_t ilog2_u64(uint64_t x) { return 63u - __clzll(x); }

// 64-bit shifts by a run-time amount, built from 32-bit operations
// (v_alignbit_b32 funnel shifts and word selects).  A 64-bit VALU shift
// (v_lshrrev_b64 and its kin) whose amount sits in the last VGPR of an
// allocation granule has been seen to take its amount from the register
// after it, outside the wave's allocation, so the kernels avoid that
// instruction for run-time amounts; the build rejects code that has it.
// Amounts are below 64 unless stated.
__device__ __forceinline__ uint32_t lo32_shr(uint64_t x, uint32_t s) {   // low word of x >> s
  const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  const bool up = s >= 32;
  return __builtin_amdgcn_alignbit(up ? 0u : hi, up ? hi : lo, s & 31);
}
__device__ __forceinline__ uint32_t lo32_shr(unsigned __int128 x, uint32_t s) {   // s < 128
  const uint32_t w0 = (uint32_t)x, w1 = (uint32_t)(x >> 32), w2 = (uint32_t)(x >> 64),
                 w3 = (uint32_t)(x >> 96), q = s >> 5;
  const uint32_t a = q == 0 ? w0 : (q == 1 ? w1 : (q == 2 ? w2 : w3));
  const uint32_t b = q == 0 ? w1 : (q == 1 ? w2 : (q == 2 ? w3 : 0u));
  return __builtin_amdgcn_alignbit(b, a, s & 31);
}
__device__ __forceinline__ uint64_t shr64(uint64_t x, uint32_t s) {
  const uint32_t hi = (uint32_t)(x >> 32);
  const uint32_t rhi = s >= 32 ? 0u : (hi >> (s & 31));
  return ((uint64_t)rhi << 32) | lo32_shr(x, s);
}
__device__ __forceinline__ uint64_t shl64(uint64_t x, uint32_t s) {
  const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32), r = s & 31;
  const bool up = s >= 32;
  const uint32_t a = up ? lo : hi, b = up ? 0u : lo;
  const uint32_t rhi = r ? __builtin_amdgcn_alignbit(a, b, 32 - r) : a;
  const uint32_t rlo = up ? 0u : (lo << r);
  return ((uint64_t)rhi << 32) | rlo;
}
// A shift amount that is the same in every lane, moved to a scalar register:
// 64-bit shifts by an SGPR amount are not affected by the hazard above and
// take one instruction.
__device__ __forceinline__ uint32_t uniform_amount(uint32_t s) { return __builtin_amdgcn_readfirstlane(s); }
__device__ __forceinline__ uint64_t bit64(uint32_t q) {   // 1 << q
  const uint32_t b = 1u << (q & 31);
  return q >= 32 ? ((uint64_t)b << 32) : (uint64_t)b;
}
__device__ __forceinline__ uint64_t low_mask64(uint32_t n) {   // n low bits set, n <= 64
  return n >= 64 ? ~0ull : bit64(n) - 1;
}
__device__ __forceinline__ uint32_t low_mask32(uint32_t n) {   // n low bits set, any n
  return n >= 32 ? ~0u : (1u << n) - 1;
}
__device__ __forceinline__ uint32_t bit_of(uint64_t x, uint32_t q) {   // bit q of x
  return ((q >= 32 ? (uint32_t)(x >> 32) : (uint32_t)x) >> (q & 31)) & 1u;
}

// Oversampling factor floor(0.2 log2 n), at least 1 (Section 6).
__device__ __forceinline__ uint32_t step_alpha(uint64_t n) {
  uint32_t a = ilog2_u64(n > 0 ? n : 1) / 5;
  return a ? a : 1;
}

__device__ __forceinline__ uint64_t step_task_seed(uint64_t seed, uint64_t l, uint32_t level) {
  return sm64_mix((seed ^ (l * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)level << 56)) +
                  0x9E3779B97F4A7C15ull);
}

template <int DW>
__device__ __forceinline__ void ld_elem(const uint32_t* p, uint32_t (&w)[DW]) {
  if constexpr (DW == 2) {
    uint2 v = *reinterpret_cast<const uint2*>(p);
    w[0] = v.x; w[1] = v.y;
  } else if constexpr (DW == 4) {
    uint2 v0 = *reinterpret_cast<const uint2*>(p);
    uint2 v1 = *reinterpret_cast<const uint2*>(p + 2);
    w[0] = v0.x; w[1] = v0.y; w[2] = v1.x; w[3] = v1.y;
  } else {
#pragma unroll
    for (int i = 0; i < DW; ++i) w[i] = p[i];
  }
}
template <int DW>
__device__ __forceinline__ void st_elem(uint32_t* p, const uint32_t (&w)[DW]) {
  if constexpr (DW == 2) {
    *reinterpret_cast<uint2*>(p) = make_uint2(w[0], w[1]);
  } else if constexpr (DW == 4) {
    *reinterpret_cast<uint2*>(p) = make_uint2(w[0], w[1]);
    *reinterpret_cast<uint2*>(p + 2) = make_uint2(w[2], w[3]);
  } else {
#pragma unroll
    for (int i = 0; i < DW; ++i) p[i] = w[i];
  }
}

// Division by the block size: a shift when it is a power of two (the
// branch is uniform across the workgroup).
// Placement pieces per bucket aimed for: few enough that a 64-bit mask
// can record which of them are full, enough to spread pointer contention.

// Number of lanes below this one whose bit is set in the wavefront mask m.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

struct BlockDiv {
  uint32_t b, sh;
  bool pow2;
  __device__ __forceinline__ explicit BlockDiv(uint32_t bb)
      : b(bb), sh((uint32_t)__builtin_ctz(bb)), pow2((bb & (bb - 1)) == 0) {}
  __device__ __forceinline__ uint32_t div(uint32_t x) const { return pow2 ? (x >> sh) : (x / b); }
};

template <class T>
__device__ __forceinline__ typename T::Key key_of(const uint32_t (&w)[T::DW]) {
  return T::key_w(w);
}

// Branchless decision tree (Definitions and Preliminaries, Algorithm 1):
// from node 1, i <- 2i + [tree_i < e] for log2 K levels; the leaf gives the
// bucket i with s_{i-1} < e <= s_i.  With equality buckets the bucket
// becomes 2i + 1 - [e < s_i], using s_{K-1} = s_{K-2}.
template <class Key>
__device__ __forceinline__ uint32_t tree_bucket(const Key* __restrict__ tree,
                                                const Key* __restrict__ spl,
                                                uint32_t logK, uint32_t eq, const Key& e) {
  uint32_t i = 1;
  for (uint32_t l = 0; l < logK; ++l) i = 2 * i + (kless(tree[i], e) ? 1u : 0u);
  i -= (1u << logK);
  if (eq) i = 2 * i + (kless(e, spl[i]) ? 0u : 1u);
  return i;
}

template <class T>
__device__ __forceinline__ uint32_t bucket_of(const typename T::Key& k, const typename T::Key* tree,
                                              const typename T::Key* spl, uint32_t logK,
                                              uint32_t eq, bool radix, uint32_t shift,
                                              uint32_t rmask) {
  if constexpr (T::RADIX_OK) {
    if (radix) return (uint32_t)(T::rkey(k) >> uniform_amount(shift)) & rmask;   // shift is the task's
  }
  return tree_bucket(tree, spl, logK, eq, k);
}

// Start-node table (the lookup table of start nodes addressed by the most
// significant key bits suggested in the paper's Section 8).  Entry p covers
// the keys whose image lies in prefix range p.  When those keys fall into at
// most START_SPAN consecutive buckets the entry holds the first of them and
// how many follow, and a key's bucket is found by comparing it with the
// splitters in between (usually none or one); otherwise it holds the deepest
// tree node whose subtree receives all of them, and the descent starts there.
struct StartTable {
  const uint16_t* start;
  uint64_t base;
  uint32_t shift;
  __device__ __forceinline__ uint32_t index(uint64_t x) const {
    if (x < base) return 0;
    const uint64_t q = (x - base) >> uniform_amount(shift);   // one table per workgroup
    return q >= (1u << START_BITS) ? (1u << START_BITS) - 1 : (uint32_t)q;
  }
};

// --------------------------------------------------------------- sampling

// Bitonic sort of n2 (power of two) keys in LDS by all threads of the block.
template <class Key>
__device__ void lds_bitonic_keys(Key* a, uint32_t n2) {
  for (uint32_t k = 2; k <= n2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < n2 / 2; i += blockDim.x) {
        uint32_t lo = (i / j) * 2 * j + (i % j), hi = lo + j;
        bool up = (lo & k) == 0;
        Key x = a[lo], y = a[hi];
        if (kless(y, x) == up) { a[lo] = y; a[hi] = x; }
      }
      __syncthreads();
    }
  }
}

// Sampling phase (Section 4.1) of every task of the batch (k' chosen by the
// host, see ips_host.hip): alpha k' samples
// drawn with replacement at positions l + floor(n x_j / 2^64), sorted;
// k'-1 equidistant splitters (the i-th at sorted position (i+1) alpha - 1);
// duplicates removed; equality buckets iff a duplicate was removed; K the
// next power of two >= u+1 with the splitters padded by the largest; tree
// in breadth-first order.
template <class T>
__global__ void __launch_bounds__(SMP_THREADS)
k_sample(BatchArgs a, uint64_t seed) {
  using Key = typename T::Key;
  constexpr int DW = T::DW;
  __shared__ Key s_smp[MAX_SAMPLE];
  __shared__ Key s_spl[MAX_K];
  __shared__ uint32_t s_u;
  const uint32_t tix = blockIdx.x;
  if (a.devplan && tix >= a.ctrl[CTRL_T]) return;
  const PTask& tk = a.tasks[tix];
  const uint64_t n = tk.n, l = tk.l;
  StepRec* rec = a.recs + tix;
  const uint32_t kp = tk.kp;
  // Oversampling: at least DEEP_ALPHA per bucket (the sample of a task
  // costs next to nothing on the GPU, and even bucket sizes keep the next
  // level's buckets inside the LDS tier's capacity); the paper's alpha at a
  // root that asks for it.
  uint32_t alpha = step_alpha(n);
  const bool deep = tk.level > 0 || (tk.tflags & TF_ROOT_ALPHA);
  if (deep && alpha < DEEP_ALPHA && DEEP_ALPHA * kp <= MAX_SAMPLE) alpha = DEEP_ALPHA;
  const uint32_t m = alpha * kp;
  uint32_t P = 1;
  while (P < m) P <<= 1;
  if (P > MAX_SAMPLE) {
    if (threadIdx.x == 0) dev_error(a.ctrl, DE_SAMPLE, tix, m);
    return;
  }
  const uint64_t ts = step_task_seed(seed, l, tk.level);
  const uint32_t* gd = a.data + l * DW;
  for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) {
    if (j < m) {
      uint64_t pos = __umul64hi(sm64_at(ts, j), n);
      uint32_t w[DW];
      ld_elem<DW>(gd + pos * DW, w);
      s_smp[j] = key_of<T>(w);
    } else {
      s_smp[j] = T::kmax();
    }
  }
  __syncthreads();
  lds_bitonic_keys(s_smp, P);
  // Splitter i (i < kp - 1) is sample (i + 1) alpha - 1; a splitter equal to
  // the one before it is dropped (the sample is sorted, so equal splitters
  // are adjacent).  Thread i keeps or drops splitter i; the kept ones are
  // packed in order by a ballot prefix count.
  {
    static_assert(MAX_K <= SMP_THREADS, "one splitter per thread");
    __shared__ uint32_t s_wkeep[SMP_THREADS / 64];
    const uint32_t i = threadIdx.x, lane = i & 63, wave = i >> 6;
    bool keep = false;
    Key sp = s_smp[0];
    if (i + 1 < kp) {
      sp = s_smp[(i + 1) * alpha - 1];
      keep = i == 0 || !keq(sp, s_smp[i * alpha - 1]);
    }
    const uint64_t bm = __ballot(keep);
    if (lane == 0) s_wkeep[wave] = (uint32_t)__popcll(bm);
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (uint32_t w = 0; w < SMP_THREADS / 64; ++w) {
      const uint32_t c = s_wkeep[w];
      before += w < wave ? c : 0u;
      total += c;
    }
    if (keep) s_spl[before + lanes_below(bm)] = sp;
    if (i == 0) s_u = total;
  }
  __syncthreads();
  const uint32_t u = s_u;
  uint32_t eq = (u < kp - 1) ? 1u : 0u;
  if (tk.tflags & TF_EQ_ON) eq = 1;
  if (tk.tflags & TF_EQ_OFF) eq = 0;
  uint32_t K = 1, logK = 0;
  while (K < u + 1) { K <<= 1; ++logK; }
  for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) {
    Key v = s_spl[i < u ? i : u - 1];
    T::to_slot(v, rec->spl[i]);
  }
  for (uint32_t i = threadIdx.x; i < MAX_K; i += blockDim.x) {
    if (i >= 1 && i < K) {
      uint32_t d = 31u - __clz(i);
      uint32_t p = i - (1u << d);
      uint32_t idx = ((2 * p + 1) << (logK - d - 1)) - 1;
      Key v = s_spl[idx < u ? idx : u - 1];
      T::to_slot(v, rec->tree[i]);
    }
  }
  // Start-node table over the splitters' key range [s_0, s_{u-1}].
  const uint64_t base = T::img(s_spl[0]);
  const uint64_t top = T::img(s_spl[u - 1]);
  const uint64_t span = top - base;
  uint32_t tsh = 0;
  {
    const uint32_t len = span ? 64u - (uint32_t)__clzll(span) : 0u;   // smallest tsh with span >> tsh < 2^START_BITS
    tsh = len > START_BITS ? len - START_BITS : 0u;
  }
  __syncthreads();
  __shared__ Key s_tree[MAX_K];
  for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) {
    if (i >= 1) {
      uint32_t d = 31u - __clz(i);
      uint32_t p = i - (1u << d);
      uint32_t idx = ((2 * p + 1) << (logK - d - 1)) - 1;
      s_tree[i] = s_spl[idx < u ? idx : u - 1];
    }
  }
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < (1u << START_BITS); p += blockDim.x) {
    const uint64_t lo = p == 0 ? 0 : base + shl64(p, tsh);
    uint64_t hi;
    if (p == (1u << START_BITS) - 1) {
      hi = T::IMG_MAX;
    } else {
      const uint64_t nx = base + shl64(p + 1, tsh);
      hi = (nx < base) ? T::IMG_MAX : nx - 1;   // saturate on wrap
      if (hi > T::IMG_MAX) hi = T::IMG_MAX;
    }
    const Key klo = T::lo_of(lo), khi = T::hi_of(hi);
    uint32_t bl = 1, bh = 1;   // buckets of the range's lowest and highest key
    while (bl < K) bl = 2 * bl + (kless(s_tree[bl], klo) ? 1u : 0u);
    while (bh < K) bh = 2 * bh + (kless(s_tree[bh], khi) ? 1u : 0u);
    bl -= K; bh -= K;
    uint32_t v;
    if (bh - bl < START_SPAN) {
      v = START_DIRECT | ((bh - bl) << 9) | bl;
    } else {
      v = 1;
      while (v < K) {
        if (kless(s_tree[v], klo)) v = 2 * v + 1;          // every key goes right
        else if (!kless(s_tree[v], khi)) v = 2 * v;       // every key goes left
        else break;
      }
    }
    rec->tstart[p] = (uint16_t)v;
  }
  if (threadIdx.x == 0) {
    rec->K = K; rec->logK = logK; rec->eq = eq; rec->nb = eq ? 2 * K : K;
    rec->u = u; rec->alpha = alpha; rec->kp = kp; rec->m = m;
    rec->shift = 0; rec->width = 0; rec->radix = 0;
    rec->tbase = base;
    rec->tshift = tsh;
  }
}

// --------------------------------------------------------- classification

// s_waitcnt immediate that waits for every outstanding vector memory
// operation of the wave (vmcnt(0); LDS and export counts unrestricted).
constexpr int WAITCNT_VM0 = 0x0F70;

// Buckets of the EPT elements a thread holds, all stepping together.  Each
// element starts from its start-table entry: a tree node to descend from,
// or a first bucket and a number of splitters to compare with in order
// (the bucket grows while the splitter is below the key).  Every step reads
// one tree node or splitter for each element not yet done (a branch-free
// step), so the LDS reads of all elements are in flight at once; the steps
// end when no element of the wavefront has one left.  State per element:
// the node (leaves K + bucket) in bits 0-15, splitters left in bits 16-31.
template <class T, int EPT>
__device__ __forceinline__ void tree_buckets(const typename T::Key (&key)[EPT],
                                             const typename T::Key* __restrict__ ts,
                                             uint32_t logK, uint32_t eq, const StartTable& st,
                                             uint32_t (&bk)[EPT]) {
  using Key = typename T::Key;
  const uint32_t K = 1u << logK;
  uint32_t w[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const uint32_t v = st.start[st.index(T::img(key[i]))];
    w[i] = (v & START_DIRECT) ? ((K + (v & 0x1FFu)) | (((v >> 9) & 7u) << 16)) : v;
  }
  for (uint32_t l = 0; l < logK + START_SPAN; ++l) {
    bool act = false;
#pragma unroll
    for (int i = 0; i < EPT; ++i) act = act || (w[i] & 0xFFFFu) < K || (w[i] >> 16) != 0;
    if (!__any(act)) break;
    // All reads first: tree node, else splitter node - K (read but unused
    // once the element is done).
    Key t[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t node = w[i] & 0xFFFFu;
      t[i] = ts[node < K ? node : node - K + MAX_K];
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t node = w[i] & 0xFFFFu, r = w[i] >> 16;
      const uint32_t g = kless(t[i], key[i]) ? 1u : 0u;
      const uint32_t wt = 2 * node + g;                        // descend
      const uint32_t wc = (node + g) | ((g * (r - 1)) << 16);  // next splitter, or stop
      const uint32_t mt = 0u - (uint32_t)(node < K);
      const uint32_t mc = 0u - (uint32_t)(node >= K && r != 0);
      w[i] = (wt & mt) | (wc & mc) | (w[i] & ~(mt | mc));
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) bk[i] = (w[i] & 0xFFFFu) - K;
  if (eq) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const Key sp = ts[MAX_K + bk[i]];
      bk[i] = 2 * bk[i] + (kless(key[i], sp) ? 0u : 1u);
    }
  }
}

// Classification phase (Section 4.1): the workgroup scans its stripe of
// blocks tile by tile, classifies each element, and appends it to the
// buffer block of its bucket.  A full buffer block is written back to the
// stripe at the front (the write position never passes the read position);
// blocks that a single tile fills completely are written directly.  At the
// end the partial buffers are saved in the stripe's slot and the per-bucket
// counts are published.
//
// LDS buffers are laid out with a stride of b*DW + BUF_PAD dwords per bucket
// so that lanes appending at the same offset of different buckets fall into
// different banks.  Each bucket's tile state is an 8-byte word (blocks full
// before the tile, after it) that every element reads, beside its block base
// that only elements stored straight to the stripe read; 8-byte words of
// random buckets spread over twice as many banks as 16-byte ones.
constexpr uint32_t BUF_PAD = BUF_PAD_DW;

// Copies the listed buffer blocks (bucket s_cj[q] for q < ncp, to stripe
// block s_cpos[q]), unit u of the flattened list going to lane u mod NT;
// CP_UNROLL units per lane are loaded before any is stored.  A block that
// would land at or beyond the read position is reported and not written.
constexpr int CP_UNROLL = 4;
template <class U, int UW>
__device__ __forceinline__ void copy_units(uint32_t ncp, uint32_t upb, const BlockDiv& ud,
                                           const uint16_t* s_cj, const uint32_t* s_cpos,
                                           const uint32_t* buf, uint32_t bstride, uint32_t* gs,
                                           uint32_t b, uint32_t DW, uint32_t consumed, uint32_t* ctrl,
                                           uint32_t wg) {
  const uint32_t tot = ncp * upb;
  for (uint32_t u0 = threadIdx.x; u0 < tot; u0 += CLS_THREADS * CP_UNROLL) {
    U v[CP_UNROLL];
    uint64_t off[CP_UNROLL];
    bool ok[CP_UNROLL];
#pragma unroll
    for (int r = 0; r < CP_UNROLL; ++r) {
      const uint32_t u = u0 + (uint32_t)r * CLS_THREADS;
      ok[r] = false;
      if (u < tot) {
        const uint32_t q = ud.div(u), x = u - q * upb;
        const uint32_t j = s_cj[q];
        const uint32_t pos = s_cpos[q] * b;
        if (pos + b > consumed) {
          if (x == 0) dev_error(ctrl, DE_CLS_INPLACE, wg, pos);
        } else {
          v[r] = reinterpret_cast<const U*>(buf + j * bstride)[x];
          off[r] = (uint64_t)pos * DW + x * UW;
          ok[r] = true;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < CP_UNROLL; ++r)
      if (ok[r]) *reinterpret_cast<U*>(gs + off[r]) = v[r];
  }
}

template <class T, bool GBUF>
__global__ void __launch_bounds__(CLS_THREADS)
k_classify(BatchArgs a) {
  using Key = typename T::Key;
  constexpr int DW = T::DW;
  constexpr int EPT = T::EPT;
  constexpr uint32_t NT = CLS_THREADS;
  constexpr uint32_t TILE = NT * EPT;
  __shared__ Key s_ts[2 * MAX_K];         // tree nodes [0, K), splitters from MAX_K
  __shared__ uint32_t s_cnt[MAX_NB];
  __shared__ uint2 s_fn[MAX_NB];          // {blocks full before the tile, after it}
  __shared__ uint32_t s_base[MAX_NB];     // block j of the bucket goes to stripe block base + j
  constexpr uint32_t NMM = T::RADIX_OK ? MAX_K : 1;   // radix key ranges per bucket
  __shared__ uint64_t s_mn[NMM], s_mx[NMM];
  __shared__ uint16_t s_start[1u << START_BITS];
  __shared__ uint16_t s_cj[MAX_NB];       // buckets whose LDS buffer block fills in this tile
  __shared__ uint32_t s_cpos[MAX_NB];     // and the stripe block it goes to
  __shared__ uint32_t s_wpos, s_ncopy;
  extern __shared__ __align__(16) uint32_t s_buf[];
  static_assert(MAX_NB <= CLS_THREADS, "one bucket per thread in the block-state pass");

  const uint32_t tid = threadIdx.x;
  const uint32_t wg = blockIdx.x;
  if (a.devplan && wg >= a.ctrl[CTRL_NWG]) return;
  const uint32_t tix = a.cls_task[wg];
  const PTask& tk = a.tasks[tix];
  const uint64_t tn = tk.n;
  const uint32_t b = tk.b, nb = tk.nb, NB = tk.NB, W = tk.W;
  const BlockDiv bd(b);
  const uint32_t s = wg - tk.wg_base;
  const bool radix = (tk.tflags & TF_RADIX) != 0;
  const uint32_t logK = tk.logK, eq = tk.eq, shift = tk.shift;
  const uint32_t rmask = low_mask32(tk.width);
  const StepRec* rec = a.recs + tix;
  if (!radix) {
    for (uint32_t i = tid; i < tk.K; i += NT) {
      s_ts[i] = T::from_slot(rec->tree[i]);
      s_ts[MAX_K + i] = T::from_slot(rec->spl[i]);
    }
    for (uint32_t i = tid; i < (1u << START_BITS); i += NT) s_start[i] = rec->tstart[i];
  }
  StartTable stab;
  stab.start = s_start;
  stab.base = radix ? 0 : rec->tbase;
  stab.shift = radix ? 0 : rec->tshift;
  for (uint32_t j = tid; j < nb; j += NT) { s_cnt[j] = 0; s_fn[j] = make_uint2(0, 0); s_base[j] = 0; }
  for (uint32_t j = tid; j < NMM; j += NT) { s_mn[j] = ~0ull; s_mx[j] = 0; }
  if (tid == 0) { s_wpos = 0; s_ncopy = 0; }
  // buffer of bucket j at buf + j * bstride (dwords)
  const uint32_t bdw = b * DW;
  const uint32_t bstride = GBUF ? bdw : bdw + BUF_PAD;
  uint32_t* buf = GBUF ? reinterpret_cast<uint32_t*>(a.slots + tk.slot_off + (uint64_t)s * tk.slot_bytes)
                       : s_buf;
  __syncthreads();

  const uint32_t blo = (uint32_t)(((uint64_t)s * NB) / W);
  const uint32_t bhi = (uint32_t)(((uint64_t)(s + 1) * NB) / W);
  const uint64_t elo = (uint64_t)blo * b;
  const uint64_t ehi = ((uint64_t)bhi * b < tn) ? (uint64_t)bhi * b : tn;
  const uint32_t slen = (uint32_t)(ehi - elo);        // stripe length (elements)
  uint32_t* gs = a.data + (tk.l + elo) * DW;          // stripe base
  const bool pair_units = (bdw & 1) == 0 && (reinterpret_cast<uintptr_t>(gs) & 7) == 0;
  const BlockDiv ud(pair_units ? bdw / 2 : bdw);

  uint32_t cur[EPT][DW];
  uint32_t nxt[EPT][DW];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const uint32_t idx = (uint32_t)i * NT + tid;
    if (idx < slen) ld_elem<DW>(gs + (uint64_t)idx * DW, cur[i]);
  }
  // Loads issued before the loop are complete when it starts, so that no
  // wait inside the loop is tied to them (the wave's one memory counter also
  // counts the block stores of the previous tile).
  __builtin_amdgcn_s_waitcnt(WAITCNT_VM0);
  for (uint32_t ts = 0; ts < slen; ts += TILE) {
    const bool full = ts + TILE <= slen;
    uint32_t bk[EPT], sl[EPT];
    Key key[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) key[i] = key_of<T>(cur[i]);
    bool radix_done = false;
    if constexpr (T::RADIX_OK) {
      if (radix) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
          bk[i] = (uint32_t)(T::rkey(key[i]) >> uniform_amount(shift)) & rmask;
          if (full || ts + (uint32_t)i * NT + tid < slen) {
            atomicMin((unsigned long long*)&s_mn[bk[i]], (unsigned long long)T::rkey(key[i]));
            atomicMax((unsigned long long*)&s_mx[bk[i]], (unsigned long long)T::rkey(key[i]));
          }
        }
        radix_done = true;
      }
    }
    if (!radix_done) tree_buckets<T, EPT>(key, s_ts, logK, eq, stab, bk);
    if (full) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) sl[i] = atomicAdd(&s_cnt[bk[i]], 1u);
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        sl[i] = 0;
        if (ts + (uint32_t)i * NT + tid < slen) sl[i] = atomicAdd(&s_cnt[bk[i]], 1u);
      }
    }
    // Prefetch the next tile; it is never written while this tile is processed.
    const uint32_t tn2 = ts + TILE;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t idx = tn2 + (uint32_t)i * NT + tid;
      if (idx < slen) ld_elem<DW>(gs + (uint64_t)idx * DW, nxt[i]);
    }
    __syncthreads();
    // Block state of each bucket (thread j): blocks full before and after
    // the tile, and where its new full blocks go.  The new blocks of a
    // wavefront's buckets are numbered by a prefix sum over the wavefront
    // and placed after the blocks already written (one counter update per
    // wavefront); buckets whose buffer block fills are listed for the copy.
    if ((tid & ~63u) < nb) {
      const uint32_t lane = tid & 63;
      const bool valid = tid < nb;
      const uint32_t fo = valid ? s_fn[tid].y : 0u;          // blocks full before this tile
      const uint32_t nf = valid ? bd.div(s_cnt[tid]) : 0u;
      const uint32_t d = nf - fo;
      uint32_t inc = d;
#pragma unroll
      for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)inc, off);
        if (lane >= off) inc += t;
      }
      const uint64_t cm = __ballot(d != 0);
      uint32_t wb = 0, cb = 0;
      if (lane == 63) {
        wb = atomicAdd(&s_wpos, inc);
        cb = atomicAdd(&s_ncopy, (uint32_t)__popcll(cm));
      }
      wb = (uint32_t)__builtin_amdgcn_readlane((int)wb, 63);
      cb = (uint32_t)__builtin_amdgcn_readlane((int)cb, 63);
      if (valid) {
        s_fn[tid] = make_uint2(fo, nf);
        s_base[tid] = wb + inc - d - fo;
        if (d) {
          const uint32_t r = lanes_below(cm);
          s_cj[cb + r] = (uint16_t)tid;
          s_cpos[cb + r] = wb + inc - d;
        }
      }
    }
    __syncthreads();
    const uint32_t consumed = (ts + TILE < slen) ? ts + TILE : slen;
    // Per-bucket tile states of the elements, read together (kept in
    // registers when there are at most 8 elements per thread).
    constexpr int NST = EPT <= 12 ? EPT : 1;
    uint2 stv[NST];
    if constexpr (EPT <= 12) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) stv[i] = s_fn[bk[i]];
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t idx = ts + (uint32_t)i * NT + tid;
      if (full || idx < slen) {
        const uint2 st = (EPT <= 12) ? stv[i < NST ? i : 0] : s_fn[bk[i]];
        const uint32_t blk = bd.div(sl[i]), o = sl[i] - blk * b;
        if (blk == st.x) {
          st_elem<DW>(buf + bk[i] * bstride + o * DW, cur[i]);
        } else if (blk < st.y) {
          const uint32_t pos = (s_base[bk[i]] + blk) * b + o;
          if (pos >= consumed) dev_error(a.ctrl, DE_CLS_INPLACE, wg, pos);
          else st_elem<DW>(gs + (uint64_t)pos * DW, cur[i]);
        }
      }
    }
    __syncthreads();
    // The next tile's loads (issued two barriers ago) are waited for here,
    // before this tile's block stores, so that using them later does not
    // wait for the stores.
    __builtin_amdgcn_s_waitcnt(WAITCNT_VM0);
    // Copy of the buffer blocks that filled (listed in s_cj) to their
    // places in the stripe, spread over all lanes in 8-byte units (dwords
    // when a block is not made of whole 8-byte units).
    {
      const uint32_t ncp = s_ncopy;
      if (pair_units) copy_units<uint2, 2>(ncp, bdw / 2, ud, s_cj, s_cpos, buf, bstride, gs, b, DW, consumed, a.ctrl, wg);
      else copy_units<uint32_t, 1>(ncp, bdw, ud, s_cj, s_cpos, buf, bstride, gs, b, DW, consumed, a.ctrl, wg);
    }
    __syncthreads();
    if (tid == 0) s_ncopy = 0;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t idx = ts + (uint32_t)i * NT + tid;
      if (full || idx < slen) {
        const uint2 st = (EPT <= 12) ? stv[i < NST ? i : 0] : s_fn[bk[i]];
        const uint32_t blk = bd.div(sl[i]), o = sl[i] - blk * b;
        if (blk == st.y && blk > st.x) st_elem<DW>(buf + bk[i] * bstride + o * DW, cur[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i)
#pragma unroll
      for (int d = 0; d < DW; ++d) cur[i][d] = nxt[i][d];
  }
  __syncthreads();
  for (uint32_t j = tid; j < nb; j += NT) {
    const uint32_t nfull = s_fn[j].y;
    a.wg_nfull[(uint64_t)wg * a.nbs + j] = nfull;
    a.wg_left[(uint64_t)wg * a.nbs + j] = s_cnt[j] - nfull * b;
    if (radix && j < MAX_K) {
      a.wg_min[(uint64_t)wg * a.nbs + j] = s_mn[j];
      a.wg_max[(uint64_t)wg * a.nbs + j] = s_mx[j];
    }
  }
  if (tid == 0) a.wg_F[wg] = s_wpos;
  if (!GBUF) {
    uint32_t* slot = reinterpret_cast<uint32_t*>(a.slots + tk.slot_off + (uint64_t)s * tk.slot_bytes);
    const uint32_t wave = tid >> 6, lane = tid & 63;
    for (uint32_t j = wave; j < nb; j += NT / 64) {
      const uint32_t fill = (s_cnt[j] - s_fn[j].y * b) * DW;
      const uint32_t* src = buf + j * bstride;
      uint32_t* dst = slot + (uint64_t)j * bdw;
      for (uint32_t x = lane; x < fill; x += 64) dst[x] = src[x];
    }
  }
}

// -------------------------------------------------------------- boundaries

__device__ __forceinline__ uint32_t stripe_of(uint32_t p, uint32_t W, uint32_t NB) {
  return (uint32_t)((((uint64_t)p + 1) * W - 1) / NB);
}
__device__ __forceinline__ uint32_t stripe_begin(uint32_t s, uint32_t W, uint32_t NB) {
  return (uint32_t)(((uint64_t)s * NB) / W);
}

// Walks the pieces of bucket range [d, dend): split at stripe ends, at the
// end e of the bucket's own blocks, and every cmax blocks.  A piece is a
// placement piece if it lies before e; pieces after e only hold blocks of
// other buckets that must be read out.  Inside one stripe the full blocks
// are a prefix, so each piece is "unprocessed blocks, then empty blocks",
// the invariant of the block permutation (Section 4.1).
template <class F>
__device__ void for_each_piece(uint32_t d, uint32_t dend, uint32_t e, uint32_t cmax, uint32_t W,
                               uint32_t NB, const uint32_t* stripeF, F&& f) {
  uint32_t cur = d;
  while (cur < dend) {
    const uint32_t s = stripe_of(cur, W, NB);
    const uint32_t snext = stripe_begin(s + 1, W, NB);
    const uint32_t fend = stripe_begin(s, W, NB) + stripeF[s];
    uint32_t end = dend < snext ? dend : snext;
    if (cur + cmax < end) end = cur + cmax;
    if (cur < e && end > e) end = e;
    const uint32_t uend = fend < end ? fend : end;
    const int32_t rinit = (uend > cur) ? (int32_t)uend - 1 : (int32_t)cur - 1;
    const bool place = end <= e;
    if (place || uend > cur) f(cur, end, rinit, place);
    cur = end;
  }
}

#ifdef IPS_COMMON_KERNELS
// Bucket totals over the stripes: one wavefront per bucket, lanes over the
// stripes.  Sizes go to b_start (turned into starts by k_boundaries),
// full-block counts to b_count, radix key ranges to b_min / b_max.
__global__ void __launch_bounds__(512) k_bucket_sums(BatchArgs a, uint32_t groups_per_task) {
  const uint32_t tix = blockIdx.x / groups_per_task;
  if (a.devplan && tix >= a.ctrl[CTRL_T]) return;
  const PTask& tk = a.tasks[tix];
  const uint32_t j = (blockIdx.x % groups_per_task) * 8 + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63;
  if (j >= tk.nb) return;
  const uint32_t W = tk.W, wg0 = tk.wg_base, bb = tk.bucket_base;
  const bool radix = (tk.tflags & TF_RADIX) != 0;
  uint64_t full = 0, left = 0, mn = ~0ull, mx = 0;
  for (uint32_t s = lane; s < W; s += 64) {
    const uint64_t o = (uint64_t)(wg0 + s) * a.nbs + j;
    full += a.wg_nfull[o];
    left += a.wg_left[o];
    if (radix) {
      const uint64_t om = (uint64_t)(wg0 + s) * a.nbs + j;
      const uint64_t x = a.wg_min[om], y = a.wg_max[om];
      mn = x < mn ? x : mn;
      mx = y > mx ? y : mx;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    full += (uint64_t)__shfl_xor((long long)full, o, 64);
    left += (uint64_t)__shfl_xor((long long)left, o, 64);
    if (radix) {
      const uint64_t x = (uint64_t)__shfl_xor((long long)mn, o, 64);
      const uint64_t y = (uint64_t)__shfl_xor((long long)mx, o, 64);
      mn = x < mn ? x : mn;
      mx = y > mx ? y : mx;
    }
  }
  if (lane == 0) {
    a.b_start[bb + j] = full * tk.b + left;
    a.b_count[bb + j] = (uint32_t)full;
    if (radix) { a.b_min[bb + j] = mn; a.b_max[bb + j] = mx; }
  }
}

// Bucket boundaries (Section 4.1): exclusive prefix sum of the bucket
// sizes, delimiters rounded up to blocks, and the pieces with their packed
// (write, read) pointers.
__global__ void __launch_bounds__(512) k_boundaries(BatchArgs a, uint32_t cmax) {
  constexpr uint32_t NT = 512;
  __shared__ uint64_t s_start[MAX_NB + 1];
  __shared__ uint32_t s_cntb[MAX_NB];
  __shared__ uint32_t s_np[MAX_NB + 1], s_up[MAX_NB + 1];
  __shared__ uint64_t s_wsum[NT / 64];
  __shared__ uint32_t s_w32[2][NT / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t tix = blockIdx.x;
  if (a.devplan && tix >= a.ctrl[CTRL_T]) return;
  const PTask& tk = a.tasks[tix];
  const uint32_t nb = tk.nb, b = tk.b, NB = tk.NB, W = tk.W, wg0 = tk.wg_base;
  const uint32_t bb = tk.bucket_base;
  const uint32_t* stripeF = a.wg_F + wg0;
  // sizes -> exclusive prefix (nb <= 512 = one bucket per thread)
  uint64_t sz = tid < nb ? a.b_start[bb + tid] : 0;
  if (tid < nb) s_cntb[tid] = a.b_count[bb + tid];
  uint64_t inc = sz;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = (uint64_t)__shfl_up((long long)inc, o, 64);
    if ((int)lane >= o) inc += y;
  }
  if (lane == 63) s_wsum[wave] = inc;
  __syncthreads();
  uint64_t base = 0, total = 0;
  for (uint32_t w = 0; w < NT / 64; ++w) {
    if (w < wave) base += s_wsum[w];
    total += s_wsum[w];
  }
  if (tid < nb) s_start[tid] = base + inc - sz;
  if (tid == 0) s_start[nb] = total;
  __syncthreads();
  // pieces per bucket, then their prefix sums
  uint32_t np = 0, up = 0;
  if (tid < nb) {
    const uint64_t st = s_start[tid];
    const uint32_t d = (uint32_t)((st + b - 1) / b);
    const uint32_t dend = (tid + 1 < nb) ? (uint32_t)((s_start[tid + 1] + b - 1) / b) : NB;
    const uint32_t e = d + s_cntb[tid];
    const uint32_t cm = max(cmax, (s_cntb[tid] + MAX_PLACE_PIECES - 1) / MAX_PLACE_PIECES);
    for_each_piece(d, dend, e, cm, W, NB, stripeF,
                   [&](uint32_t c0, uint32_t, int32_t ri, bool) {
                     ++np;
                     up += (uint32_t)(ri - (int32_t)c0 + 1);
                   });
    a.b_start[bb + tid] = st;
    a.b_d[bb + tid] = d;
  }
  uint32_t ip = np, iu = up;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y0 = (uint32_t)__shfl_up((int)ip, o, 64);
    const uint32_t y1 = (uint32_t)__shfl_up((int)iu, o, 64);
    if ((int)lane >= o) { ip += y0; iu += y1; }
  }
  if (lane == 63) { s_w32[0][wave] = ip; s_w32[1][wave] = iu; }
  __syncthreads();
  uint32_t bp = 0, bu = 0, tp = 0, tu = 0;
  for (uint32_t w = 0; w < NT / 64; ++w) {
    if (w < wave) { bp += s_w32[0][w]; bu += s_w32[1][w]; }
    tp += s_w32[0][w];
    tu += s_w32[1][w];
  }
  if (tid < nb) { s_np[tid] = bp + ip - np; s_up[tid] = bu + iu - up; }
  if (tid == 0) {
    s_np[nb] = tp;
    s_up[nb] = tu;
    a.b_start[bb + nb] = total;
    a.t_npieces[tix] = tp;
    a.t_unproc[tix] = tu;
    if (tp > tk.piece_cap) dev_error(a.ctrl, DE_PIECES, tix, tp);
    if (total != tk.n) dev_error(a.ctrl, DE_CLEANUP_COUNT, tix, 0xFFFFFFFFu);
  }
  __syncthreads();
  if (s_np[nb] > tk.piece_cap) return;
  const uint32_t pb = tk.piece_base;
  if (tid < nb) {
    const uint32_t j = tid;
    const uint64_t st = s_start[j];
    const uint32_t d = (uint32_t)((st + b - 1) / b);
    const uint32_t dend = (j + 1 < nb) ? (uint32_t)((s_start[j + 1] + b - 1) / b) : NB;
    const uint32_t e = d + s_cntb[j];
    const uint32_t cm = max(cmax, (s_cntb[j] + MAX_PLACE_PIECES - 1) / MAX_PLACE_PIECES);
    uint32_t p = pb + s_np[j];
    uint32_t cu = s_up[j];
    uint32_t plb = p, ple = p;
    for_each_piece(d, dend, e, cm, W, NB, stripeF,
                   [&](uint32_t c0, uint32_t c1, int32_t ri, bool place) {
                     a.p_a[p] = c0;
                     a.p_c[p] = place ? c1 : c0;
                     a.p_rinit[p] = ri;
                     a.p_cum[p] = cu;
                     a.p_fcnt[p] = 0;
                     a.p_word[(uint64_t)p * PWORD_STRIDE] = ((uint64_t)c0 << 32) | (uint64_t)((uint32_t)ri + PTR_BIAS);
                     a.p_word[(uint64_t)p * PWORD_STRIDE + 1] = 0;
                     cu += (uint32_t)(ri - (int32_t)c0 + 1);
                     ++p;
                     if (place) ple = p;
                   });
    a.b_plb[bb + j] = plb;
    a.b_ple[bb + j] = ple;
    a.b_full[bb + j] = 0;
  }
}

#endif  // IPS_COMMON_KERNELS

// ------------------------------------------------------------ permutation

__device__ __forceinline__ uint32_t shfl32(uint32_t v, uint32_t lane) {
  return (uint32_t)__shfl((int)v, (int)lane, 64);
}


template <class T>
__device__ __forceinline__ uint32_t block_bucket(const uint32_t (&dat)[PERM_RD], uint32_t lbase, uint32_t glanes,
                                                 const typename T::Key* tree,
                                                 const typename T::Key* spl, uint32_t logK,
                                                 uint32_t eq, bool radix, uint32_t shift,
                                                 uint32_t rmask) {
  // dword x of the block is register x / glanes of lane lbase + x % glanes
  // (glanes >= 4, so the first element's KDW <= 6 key dwords are in
  // registers 0 and 1)
  static_assert(T::KDW <= 8, "key dwords beyond the first two registers of a group");
  uint32_t w[T::KDW];
#pragma unroll
  for (int x = 0; x < T::KDW; ++x) {
    if constexpr (T::KDW <= 4) {
      w[x] = shfl32(dat[0], lbase + x);
    } else {
      const uint32_t q = (uint32_t)x >= glanes, l = q ? (uint32_t)x - glanes : (uint32_t)x;
      w[x] = shfl32(q ? dat[1] : dat[0], lbase + l);
    }
  }
  return bucket_of<T>(T::key_w(w), tree, spl, logK, eq, radix, shift, rmask);
}

// Waits until every load into `v` has returned (an opaque use of each
// register), so that a later store or flag cannot overtake them.
__device__ __forceinline__ void wait_regs(const uint32_t (&v)[PERM_RD]) {
#pragma unroll
  for (int r = 0; r < PERM_RD; ++r) asm volatile("" ::"v"(v[r]) : "memory");
}

// Block permutation (Section 4.1).  A group of `glanes` lanes plays the
// role of one thread of the paper: it holds one block in registers (its
// swap buffer).  Each bucket's final block range is split into pieces, each
// with a packed (w, r) pointer word: blocks [a, w) are correct, [w, r]
// unprocessed, the rest empty.  A group claims an unprocessed block by
// decrementing r of a piece of its assigned source range, classifies its
// first element, and reserves the next slot w of a piece of the destination
// bucket: an unprocessed block there is swapped out (or skipped if it is
// already correct), an empty slot is written.  A slot that another group
// may still be reading (w > r but w <= the piece's initial r) is written
// only after every read of a block claimed from that piece has finished:
// the paper's reader counter of a bucket, kept per piece in the word next
// to the pointer word.  Its low half counts finished reads; its high half
// is set, by whichever operation takes the piece's last unprocessed block
// (a claim with r = w or a swap with w = r), to 1 + the first block that
// claims took (claims take blocks from the initial r downward, so blocks
// [first, r_init] are exactly the claimed ones, and no later claim can
// succeed).  A waiting writer proceeds once the count reaches
// r_init - first + 1, so the reader state is one word per piece,
// O(k + stripes) per task, not one flag per block.
//
// Every iteration first issues the pointer operations of all groups of the
// wavefront together, then all block loads together, so that one iteration
// costs about one atomic and one load latency whatever mix of states the
// groups are in.
// Elements of up to four dwords: at least seven wavefronts per SIMD (the
// second bound; at most 72 VGPRs), so that as many block chains as
// possible are in flight.
template <class T, uint32_t NT>
__global__ void __launch_bounds__(NT, (T::DW <= 4 ? 7 : 1))
k_permute(BatchArgs a) {
  using Key = typename T::Key;
  __shared__ Key s_tree[MAX_K];
  __shared__ Key s_spl[MAX_K];
  __shared__ uint32_t s_plb[MAX_NB];   // placement pieces of each bucket
  __shared__ uint32_t s_npl[MAX_NB];
  __shared__ uint64_t s_full[MAX_NB];  // the workgroup's view of each bucket's full-piece mask
  if (a.devplan && blockIdx.x >= a.ctrl[CTRL_NPWG]) return;
  const uint32_t tix = a.perm_task[blockIdx.x];
  const PTask& tk = a.tasks[tix];
  const bool radix = (tk.tflags & TF_RADIX) != 0;
  const uint32_t logK = tk.logK, eq = tk.eq, shift = tk.shift;
  const uint32_t rmask = low_mask32(tk.width);
  if (!radix) {
    const StepRec* rec = a.recs + tix;
    for (uint32_t i = threadIdx.x; i < tk.K; i += NT) {
      s_tree[i] = T::from_slot(rec->tree[i]);
      s_spl[i] = T::from_slot(rec->spl[i]);
    }
  }
  for (uint32_t j = threadIdx.x; j < tk.nb; j += NT) {
    const uint32_t lo = a.b_plb[tk.bucket_base + j] - tk.piece_base;
    s_plb[j] = lo;
    s_npl[j] = a.b_ple[tk.bucket_base + j] - tk.piece_base - lo;
    s_full[j] = a.b_full[tk.bucket_base + j];
  }
  __syncthreads();
  const uint32_t GL = tk.glanes;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t gl = lane & (GL - 1);
  const uint32_t lbase = lane - gl;
  const uint32_t gid = (blockIdx.x - tk.pwg_base) * (NT / GL) + threadIdx.x / GL;
  const uint32_t b = tk.b, NB = tk.NB;
  const uint32_t BDW = b * T::DW;
  uint32_t* gd = a.data + tk.l * T::DW;
  const uint32_t pb = tk.piece_base;
  const uint32_t np = a.t_npieces[tix];
  const uint32_t U = a.t_unproc[tix];
  uint64_t* word = a.p_word + (uint64_t)pb * PWORD_STRIDE;
  const uint32_t* pa = a.p_a + pb;
  const uint32_t* pc = a.p_c + pb;
  const int32_t* pr = a.p_rinit + pb;
  const uint32_t* pcum = a.p_cum + pb;
  const uint32_t bb = tk.bucket_base;
  const bool partial = (tk.n % b) != 0;
  uint32_t* ovf = a.ovf + (uint64_t)tix * (MAX_BLOCK_BYTES / 4);
  if (BDW > PERM_RD * GL) {
    if (threadIdx.x == 0) dev_error(a.ctrl, DE_BLOCK, tix, BDW);
    return;
  }
#ifdef IPS_PERM_STATS
  uint32_t st_claim_ok = 0, st_claim_fail = 0, st_swap = 0, st_skip = 0, st_empty = 0,
           st_wait = 0, st_full = 0, st_waitit = 0, st_loop = 0;
#define PSTAT(x) (++(x))
#else
#define PSTAT(x) ((void)0)
#endif
  enum : uint32_t { CLAIM = 0, PLACE = 1, WAIT = 2, DONE = 3 };
  constexpr uint32_t NONE = 0xFFFFFFFFu;
  uint32_t mode = (gid < tk.ngrp && U > 0) ? CLAIM : DONE;
  uint32_t src = 0, src_end = 0;
  if (mode == CLAIM) {
    const uint64_t ulo = (uint64_t)gid * U / tk.ngrp;
    const uint64_t uhi = (uint64_t)(gid + 1) * U / tk.ngrp;
    if (ulo == uhi) {
      mode = DONE;
    } else {
      uint32_t lo = 0, hi = np;            // first p with cum + unproc > ulo
      while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        const uint64_t ce = (uint64_t)pcum[mid] + (uint32_t)(pr[mid] - (int32_t)pa[mid] + 1);
        if (ce > ulo) hi = mid; else lo = mid + 1;
      }
      src = lo;
      lo = src; hi = np;                   // first p with cum >= uhi
      while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        if ((uint64_t)pcum[mid] >= uhi) hi = mid; else lo = mid + 1;
      }
      src_end = lo;
    }
  }
  uint32_t dat[PERM_RD], tmp[PERM_RD];
#pragma unroll
  for (int q = 0; q < PERM_RD; ++q) { dat[q] = 0; tmp[q] = 0; }
  uint32_t dest = 0, probe = 0, wpos = 0, spin = 0, fails = 0, cur_q = 0;
  bool use_mask = false;
  // The first choice of a placement piece reads the workgroup's LDS copy of
  // the full-piece mask when the task has few groups per piece: with many
  // (a root step of the whole array) other workgroups fill pieces faster
  // than a copy taken at the workgroup's start can follow.
  const bool lds_mask = tk.ngrp <= 4u * np;

  auto store_block = [&](uint32_t* dst) {
#pragma unroll
    for (int q = 0; q < PERM_RD; ++q) {
      const uint32_t x = gl + GL * q;
      if (x < BDW) dst[x] = dat[q];
    }
  };

  while (true) {
    if (__all(mode == DONE)) break;
    PSTAT(st_loop);
    // 1. Pointer operations of every group (leader lanes).
    uint32_t r0 = NONE, r1 = 0, r2 = 0;   // CLAIM: r0 = P, r1 = 1 if P = w; PLACE: r0 = w (NONE: piece full), r1 = r,
                                          // r2 = the piece's initial r; WAIT: r0 = 1 once the slot's reads are done
    if (gl == 0) {
      if (mode == CLAIM) {
        // Decrementing r of an exhausted piece is harmless (r only moves
        // further below w), so each attempt is one read-modify-write.
        while (src < src_end) {
          const uint64_t wv = at_add64(&word[src * PWORD_STRIDE], ~0ull);
          const int32_t w = (int32_t)(wv >> 32), r = (int32_t)((uint32_t)wv - PTR_BIAS);
          if (r >= w) {
            r0 = (uint32_t)r;
            r1 = r == w;   // the piece's last unprocessed block: blocks [w, r_init] were claimed
            PSTAT(st_claim_ok);
            break;
          }
          PSTAT(st_claim_fail);
          ++src;
        }
      } else if (mode == PLACE) {
        // A placement piece of the bucket with room.  The bucket's mask has
        // one bit per chunk of cs consecutive pieces (cs = 1 for up to 64
        // pieces); a bit is set once every piece of its chunk is full.  The
        // first choice is a random piece of a random chunk not known to be
        // full (the mask only gains bits, so a stale copy only costs a
        // miss).  With cs = 1 and few groups per piece that copy is the
        // workgroup's own in LDS, which keeps the pointer update off a
        // global load's latency; otherwise it is the mask read through the
        // cache, which stays fresher.  After a miss the mask is read
        // coherently (and merged into the LDS copy): with cs = 1 a random
        // non-full piece is taken again; with cs > 1 the search moves on
        // linearly from the missed piece, skipping full chunks, so it
        // visits every piece with room.
        const uint32_t plb = s_plb[dest], npl = s_npl[dest];
        uint64_t* fm = a.b_full + bb + dest;
        const uint32_t cs = (npl + 63) >> 6;
        const uint32_t nch = cs ? (npl + cs - 1) / cs : 0;
        const uint64_t m = low_mask64(nch);
        if (npl) {
          uint64_t seen;
          if (use_mask) {
            seen = at_load64(fm);
            if (cs == 1 && lds_mask) atomicOr((unsigned long long*)&s_full[dest], (unsigned long long)seen);
          } else {
            seen = (cs == 1 && lds_mask) ? s_full[dest] : *fm;
          }
          const uint64_t fr = ~seen & m;
          if (cs == 1 || !use_mask) {
            uint32_t ch = probe % nch;
            if (fr) {
              uint32_t kth = probe % (uint32_t)(__popc((uint32_t)fr) + __popc((uint32_t)(fr >> 32)));
              uint64_t x = fr;
              for (; kth > 0; --kth) x &= x - 1;
              ch = (uint32_t)__ffsll((long long)x) - 1;
            }
            const uint32_t c0 = ch * cs, clen = min(cs, npl - c0);
            cur_q = c0 + (cs == 1 ? 0u : (probe >> 7) % clen);
          } else {
            cur_q = cur_q + 1 < npl ? cur_q + 1 : 0;
            const uint32_t ch = cur_q / cs;
            if (bit_of(seen, ch) && fr) {
              const uint64_t up = fr & ~low_mask64(ch);
              const uint32_t nc = (uint32_t)__ffsll((long long)(up ? up : fr)) - 1;
              cur_q = nc * cs;
            }
          }
          const uint32_t q = cur_q;
          const uint32_t sr = plb + q;
          // piece metadata loads are issued before the pointer update so that
          // their latencies overlap
          const uint32_t cap = pc[sr];
          const int32_t rin = pr[sr];
          const uint64_t wv = at_add64(&word[sr * PWORD_STRIDE], 1ull << 32);
          const uint32_t w = (uint32_t)(wv >> 32);
          r2 = (uint32_t)rin;
          if (w < cap) {
            r0 = w;
            r1 = (uint32_t)((int32_t)((uint32_t)wv - PTR_BIAS));
            if (r0 == r1)   // this swap takes the last unprocessed block: [w + 1, r_init] were claimed
              (void)at_add64(&word[sr * PWORD_STRIDE + 1], (uint64_t)(w + 2) << 32);
            if (w + 1 == cap) {            // this placement filled the piece
              if (cs == 1) {
                atomicOr((unsigned long long*)fm, bit64(q));
                atomicOr((unsigned long long*)&s_full[dest], (unsigned long long)bit64(q));
              } else {
                const uint32_t c0 = (q / cs) * cs, clen = min(cs, npl - c0);
                if (atomicAdd(&a.p_fcnt[pb + plb + c0], 1u) + 1 == clen)
                  atomicOr((unsigned long long*)fm, bit64(q / cs));
              }
            }
          } else {
            if (cs == 1) {
              atomicOr((unsigned long long*)fm, bit64(q));
              atomicOr((unsigned long long*)&s_full[dest], (unsigned long long)bit64(q));
            }
            PSTAT(st_full);
          }
        }
      } else if (mode == WAIT) {
        // the waited slot lies in placement piece cur_q of the held block's bucket
        const uint32_t sr = s_plb[dest] + cur_q;
        const uint64_t v = at_load64(&word[sr * PWORD_STRIDE + 1]);
        const uint32_t first1 = (uint32_t)(v >> 32), done = (uint32_t)v;   // 1 + first claimed block
        r0 = (first1 != 0 && (uint64_t)done + first1 >= (uint64_t)(uint32_t)pr[sr] + 2) ? 1u : 0u;
      }
    }
    r0 = shfl32(r0, lbase);
    r1 = shfl32(r1, lbase);
    r2 = shfl32(r2, lbase);
    // 2. Transitions that need no data, and the block loads.
    uint32_t ld = NONE;
    if (mode == CLAIM) {
      if (r0 == NONE) {
        mode = DONE;
      } else if (r0 >= NB || (r0 == NB - 1 && partial)) {
        if (gl == 0) dev_error(a.ctrl, DE_PERM_RANGE, tix, r0);
        mode = DONE;
      } else {
        ld = r0;
      }
    } else if (mode == PLACE) {
      if (r0 == NONE) {
        use_mask = true;
        probe = probe * 0x9E3779B1u + 0x7F4A7C15u;
        // A held block always has a slot left in its bucket (a bucket
        // receives exactly as many blocks as its placement pieces hold), so
        // the search ends; the bound only stops a broken invariant.
        if (++fails > 4 * s_npl[dest] + 4096) {
          if (gl == 0) dev_error(a.ctrl, DE_PLACE, tix, dest);
          mode = DONE;
        }
      } else if (r0 >= NB || ((int32_t)r0 <= (int32_t)r1 && r0 == NB - 1 && partial)) {
        if (gl == 0) dev_error(a.ctrl, DE_PERM_RANGE, tix, r0);
        mode = DONE;
      } else if ((int32_t)r0 <= (int32_t)r1) {
        ld = r0;                                   // unprocessed: swap candidate
      } else if ((int32_t)r0 <= (int32_t)r2) {
        wpos = r0;                                 // maybe still being read by another group
        spin = 0;
        mode = WAIT;
        PSTAT(st_wait);
      } else {
        store_block((r0 == NB - 1 && partial) ? ovf : gd + (uint64_t)r0 * BDW);
        mode = CLAIM;
        PSTAT(st_empty);
      }
    } else if (mode == WAIT) {
      PSTAT(st_waitit);
      if (r0) {
        store_block(gd + (uint64_t)wpos * BDW);
        mode = CLAIM;
      } else if (++spin > (1u << 22)) {
        if (gl == 0) dev_error(a.ctrl, DE_WAIT, tix, wpos);
        mode = DONE;
      }
    }
    if (ld != NONE) {
      const uint32_t* sp = gd + (uint64_t)ld * BDW;
#pragma unroll
      for (int q = 0; q < PERM_RD; ++q) {
        const uint32_t x = gl + GL * q;
        if (x < BDW) tmp[q] = sp[x];
      }
      wait_regs(tmp);
      if (mode == CLAIM) {
        // This read has finished; a claim that took the piece's last
        // unprocessed block also publishes 1 + the first claimed block (its
        // own), which waiting writers need together with this read anyway.
        if (gl == 0) (void)at_add64(&word[src * PWORD_STRIDE + 1], 1ull + (r1 ? (uint64_t)(ld + 1) << 32 : 0ull));
#pragma unroll
        for (int q = 0; q < PERM_RD; ++q) dat[q] = tmp[q];
        dest = block_bucket<T>(dat, lbase, GL, s_tree, s_spl, logK, eq, radix, shift, rmask);
        probe = gid * 0x9E3779B1u + dest * 0x85EBCA6Bu;
        use_mask = false;
        fails = 0;
        mode = PLACE;
      } else {
        const uint32_t d2 = block_bucket<T>(tmp, lbase, GL, s_tree, s_spl, logK, eq, radix, shift, rmask);
        if (d2 == dest) {
          PSTAT(st_skip);                          // already in its bucket
        } else {
          PSTAT(st_swap);
          uint32_t* wp = gd + (uint64_t)ld * BDW;
#pragma unroll
          for (int q = 0; q < PERM_RD; ++q) {
            const uint32_t x = gl + GL * q;
            if (x < BDW) wp[x] = dat[q];
            dat[q] = tmp[q];
          }
          dest = d2;
          probe = gid * 0x9E3779B1u + dest * 0x85EBCA6Bu;
          use_mask = false;
          fails = 0;
        }
      }
    }
    if (mode == WAIT) __builtin_amdgcn_s_sleep(1);
  }
#ifdef IPS_PERM_STATS
  if (gl == 0) {
    // root step at control words 32..49, deeper steps at 84..101
    unsigned long long* c = reinterpret_cast<unsigned long long*>(a.ctrl + (tk.level ? 84 : 32));
    atomicAdd(&c[0], (unsigned long long)st_claim_ok);
    atomicAdd(&c[1], (unsigned long long)st_claim_fail);
    atomicAdd(&c[2], (unsigned long long)st_swap);
    atomicAdd(&c[3], (unsigned long long)st_skip);
    atomicAdd(&c[4], (unsigned long long)st_empty);
    atomicAdd(&c[5], (unsigned long long)st_wait);
    atomicAdd(&c[6], (unsigned long long)st_full);
    atomicAdd(&c[7], (unsigned long long)st_waitit);
    if (lane == 0) atomicAdd(&c[8], (unsigned long long)st_loop);
  }
#endif
#undef PSTAT
}

// ----------------------------------------------------------------- cleanup

struct BucketGeo {
  uint64_t start, end, F;   // F: end of the bucket's blocks inside the array
  uint32_t d, count;
  bool ovf;                 // the bucket's last block sits in the overflow block
};

__device__ __forceinline__ BucketGeo bucket_geo(const BatchArgs& a, const PTask& tk, uint32_t j) {
  BucketGeo g;
  const uint32_t bb = tk.bucket_base;
  g.start = a.b_start[bb + j];
  g.end = a.b_start[bb + j + 1];
  g.d = a.b_d[bb + j];
  g.count = a.b_count[bb + j];
  const uint32_t e = g.d + g.count;
  g.ovf = g.count > 0 && e == tk.NB && (tk.n % tk.b) != 0;
  g.F = (uint64_t)(g.ovf ? e - 1 : e) * tk.b;
  return g;
}

// Cleanup, first part: the last block of a bucket may reach into the head of
// the next bucket; those elements are saved before any head is rewritten.
template <class T>
__global__ void __launch_bounds__(CLN_THREADS) k_cleanup_a(BatchArgs a) {
  constexpr int DW = T::DW;
  const uint32_t tix = blockIdx.x;
  if (a.devplan && tix >= a.ctrl[CTRL_T]) return;
  const PTask& tk = a.tasks[tix];
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t* gd = a.data + tk.l * DW;
  uint32_t* spill = reinterpret_cast<uint32_t*>(a.spill + tk.spill_off);
  for (uint32_t j = wave; j < tk.nb; j += CLN_THREADS / 64) {
    const BucketGeo g = bucket_geo(a, tk, j);
    if (g.count > 0 && !g.ovf && g.F > g.end) {
      const uint64_t len = (g.F - g.end) * DW;
      if (g.F - g.end >= tk.b || g.F > (uint64_t)tk.NB * tk.b) {
        if (lane == 0) dev_error(a.ctrl, DE_CLN_RANGE, tix, j);
        continue;
      }
      const uint32_t* src = gd + g.end * DW;
      uint32_t* dst = spill + (uint64_t)j * tk.b * DW;
      for (uint64_t x = lane; x < len; x += 64) dst[x] = src[x];
    }
  }
}

// Cleanup, second part (Section 4.1 "Cleanup"): the elements of bucket j
// that are not yet inside [start_j, end_j) - the saved spill, the overflow
// block, and the partial buffer blocks of every stripe - fill the bucket's
// free positions: its head [start_j, d_j b) and its tail after its blocks.
template <class T>
__device__ void cleanup_b_item(const BatchArgs& a, uint32_t item, uint32_t part, uint32_t parts,
                               uint32_t max_w, uint64_t* s_off) {
  constexpr int DW = T::DW;
  const uint32_t m = a.cln_map[item];
  const uint32_t tix = m >> 10, j = m & 1023u;
  const PTask& tk = a.tasks[tix];
  const BucketGeo g = bucket_geo(a, tk, j);
  const uint32_t b = tk.b, W = tk.W;
  if (W > max_w) {
    if (threadIdx.x == 0) dev_error(a.ctrl, DE_CLN_RANGE, tix, W);
    return;
  }
  const uint64_t hend = ((uint64_t)g.d * b < g.end) ? (uint64_t)g.d * b : g.end;
  const uint64_t hlen = hend - g.start;
  const uint64_t tlen = (g.F < g.end) ? g.end - g.F : 0;
  const uint64_t sp = (g.count > 0 && !g.ovf && g.F > g.end) ? g.F - g.end : 0;
  {
    // s_off[0..2]: spill and overflow; s_off[3 + s]: end of stripe s's
    // leftovers (block-wide scan over the stripes)
    __shared__ uint64_t s_ws[CLN_THREADS / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t per = (W + CLN_THREADS - 1) / CLN_THREADS;
    const uint32_t s0 = tid * per;
    uint64_t loc = 0;
    for (uint32_t i = 0; i < per; ++i)
      if (s0 + i < W) loc += a.wg_left[(uint64_t)(tk.wg_base + s0 + i) * a.nbs + j];
    uint64_t inc = loc;
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t y = (uint64_t)__shfl_up((long long)inc, o, 64);
      if ((int)lane >= o) inc += y;
    }
    if (lane == 63) s_ws[wave] = inc;
    __syncthreads();
    const uint64_t head = sp + (g.ovf ? b : 0);
    uint64_t acc = head + inc - loc;
    for (uint32_t w = 0; w < wave; ++w) acc += s_ws[w];
    for (uint32_t i = 0; i < per; ++i) {
      if (s0 + i < W) {
        acc += a.wg_left[(uint64_t)(tk.wg_base + s0 + i) * a.nbs + j];
        s_off[3 + s0 + i] = acc;
      }
    }
    if (tid == 0) { s_off[0] = 0; s_off[1] = sp; s_off[2] = head; }
    __syncthreads();
  }
  const uint64_t total = s_off[2 + W];
  if (total != hlen + tlen) {
    if (threadIdx.x == 0) dev_error(a.ctrl, DE_CLEANUP_COUNT, tix, j);
    return;
  }
  uint32_t* gd = a.data + tk.l * DW;
  const uint32_t* spill = reinterpret_cast<const uint32_t*>(a.spill + tk.spill_off) + (uint64_t)j * b * DW;
  const uint32_t* ovf = a.ovf + (uint64_t)tix * (MAX_BLOCK_BYTES / 4);
  const uint8_t* slot0 = a.slots + tk.slot_off;
  for (uint64_t e = (uint64_t)part * CLN_THREADS + threadIdx.x; e < total; e += (uint64_t)parts * CLN_THREADS) {
    uint32_t lo = 0, hi = W + 2;     // segment: largest i with s_off[i] <= e
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) / 2;
      if (s_off[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const uint64_t k = e - s_off[lo];
    const uint32_t* src;
    if (lo == 0) src = spill + k * DW;
    else if (lo == 1) src = ovf + k * DW;
    else src = reinterpret_cast<const uint32_t*>(slot0 + (uint64_t)(lo - 2) * tk.slot_bytes) +
               ((uint64_t)j * b + k) * DW;
    const uint64_t dst = (e < hlen) ? g.start + e : g.F + (e - hlen);
    if (dst < g.start || dst >= g.end) {
      dev_error(a.ctrl, DE_CLN_RANGE, tix, j);
      continue;
    }
    uint32_t w[DW];
    ld_elem<DW>(src, w);
    st_elem<DW>(gd + dst * DW, w);
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same cleanup of one bucket item by one wavefront, for a task of at
// most CLN_WAVE_W stripes: lane s scans stripe s's leftovers (a lane-shuffle
// prefix sum), the offsets go to this wavefront's s_offw, and the lanes copy
// the elements.
constexpr uint32_t CLN_WAVE_W = 61;
template <class T>
__device__ void cleanup_b_item_wave(const BatchArgs& a, uint32_t item, uint64_t* s_offw) {
  constexpr int DW = T::DW;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t m = a.cln_map[item];
  const uint32_t tix = m >> 10, j = m & 1023u;
  const PTask& tk = a.tasks[tix];
  const BucketGeo g = bucket_geo(a, tk, j);
  const uint32_t b = tk.b, W = tk.W;
  const uint64_t hend = ((uint64_t)g.d * b < g.end) ? (uint64_t)g.d * b : g.end;
  const uint64_t hlen = hend - g.start;
  const uint64_t tlen = (g.F < g.end) ? g.end - g.F : 0;
  const uint64_t sp = (g.count > 0 && !g.ovf && g.F > g.end) ? g.F - g.end : 0;
  const uint64_t head = sp + (g.ovf ? b : 0);
  const uint64_t loc = lane < W ? a.wg_left[(uint64_t)(tk.wg_base + lane) * a.nbs + j] : 0;
  uint64_t inc = loc;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = (uint64_t)__shfl_up((long long)inc, o, 64);
    if ((int)lane >= o) inc += y;
  }
  if (lane < W) s_offw[3 + lane] = head + inc;
  if (lane == 0) { s_offw[0] = 0; s_offw[1] = sp; s_offw[2] = head; }
  wave_sync();
  const uint64_t total = s_offw[2 + W];
  if (total != hlen + tlen) {
    if (lane == 0) dev_error(a.ctrl, DE_CLEANUP_COUNT, tix, j);
    wave_sync();
    return;
  }
  uint32_t* gd = a.data + tk.l * DW;
  const uint32_t* spill = reinterpret_cast<const uint32_t*>(a.spill + tk.spill_off) + (uint64_t)j * b * DW;
  const uint32_t* ovf = a.ovf + (uint64_t)tix * (MAX_BLOCK_BYTES / 4);
  const uint8_t* slot0 = a.slots + tk.slot_off;
  for (uint64_t e = lane; e < total; e += 64) {
    uint32_t lo = 0, hi = W + 2;     // segment: largest i with s_offw[i] <= e
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) / 2;
      if (s_offw[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const uint64_t k = e - s_offw[lo];
    const uint32_t* src;
    if (lo == 0) src = spill + k * DW;
    else if (lo == 1) src = ovf + k * DW;
    else src = reinterpret_cast<const uint32_t*>(slot0 + (uint64_t)(lo - 2) * tk.slot_bytes) +
               ((uint64_t)j * b + k) * DW;
    const uint64_t dst = (e < hlen) ? g.start + e : g.F + (e - hlen);
    if (dst < g.start || dst >= g.end) {
      dev_error(a.ctrl, DE_CLN_RANGE, tix, j);
      continue;
    }
    uint32_t w[DW];
    ld_elem<DW>(src, w);
    st_elem<DW>(gd + dst * DW, w);
  }
  wave_sync();   // s_offw is read before the next item writes it
}

// One workgroup per bucket item (task, bucket); with device-planned counts
// the grid loops over the step's items.  When the grid has several
// workgroups per item (few large buckets), each item is split into up to
// CLN_PARTS parts: every part computes the bucket's leftover offsets and
// copies every parts-th run of CLN_THREADS elements.  Otherwise a workgroup
// takes its items four at a time, one per wavefront when all four tasks
// have at most CLN_WAVE_W stripes (small tasks of a deep level), else one
// after the other with the whole workgroup.
constexpr uint32_t CLN_PARTS = 16;
template <class T>
__global__ void __launch_bounds__(CLN_THREADS) k_cleanup_b(BatchArgs a, uint32_t max_w) {
  extern __shared__ uint64_t s_off[];   // max_w + 3 entries
  constexpr uint32_t NWV = CLN_THREADS / 64;
  __shared__ uint64_t s_offw[NWV][CLN_WAVE_W + 3];
  const uint32_t count = a.devplan ? a.ctrl[CTRL_NCLN] : gridDim.x;
  uint32_t parts = count ? gridDim.x / count : 1u;
  parts = parts < 1u ? 1u : (parts > CLN_PARTS ? CLN_PARTS : parts);
  if (parts > 1) {
    for (uint32_t x = blockIdx.x; x < count * parts; x += gridDim.x) {
      cleanup_b_item<T>(a, x / parts, x % parts, parts, max_w, s_off);
      __syncthreads();
    }
    return;
  }
  const uint32_t wave = threadIdx.x >> 6;
  for (uint32_t x0 = blockIdx.x * NWV; x0 < count; x0 += gridDim.x * NWV) {
    const uint32_t item = x0 + wave;
    bool small = true;
    if (item < count) small = a.tasks[a.cln_map[item] >> 10].W <= CLN_WAVE_W;
    if (__syncthreads_and(small ? 1 : 0)) {
      if (item < count) cleanup_b_item_wave<T>(a, item, s_offw[wave]);
    } else {
      for (uint32_t q = 0; q < NWV && x0 + q < count; ++q) {
        cleanup_b_item<T>(a, x0 + q, 0, 1, max_w, s_off);
        __syncthreads();
      }
    }
  }
}

// -------------------------------------------------- sorted check, radix root

// Sorted / reverse-sorted detection (Section 6): records whether any
// adjacent pair descends or ascends; workgroups stop early once both have
// been seen.
template <class T>
__global__ void __launch_bounds__(256) k_sorted_check(const uint32_t* data, uint64_t n, uint32_t* ctrl) {
  using Key = typename T::Key;
  constexpr int DW = T::DW;
  constexpr uint64_t CH = 256 * 16;
  __shared__ uint32_t s_f[2];
  for (uint64_t c0 = (uint64_t)blockIdx.x * CH; c0 + 1 < n; c0 += (uint64_t)gridDim.x * CH) {
    if (threadIdx.x == 0) { s_f[0] = at_load32(&ctrl[CTRL_DESC]); s_f[1] = at_load32(&ctrl[CTRL_ASC]); }
    __syncthreads();
    const bool stop = s_f[0] && s_f[1];
    const bool had_desc = s_f[0] != 0, had_asc = s_f[1] != 0;
    __syncthreads();
    if (stop) return;
    uint32_t desc = 0, asc = 0;
    for (uint32_t q = 0; q < 16; ++q) {
      const uint64_t i = c0 + (uint64_t)q * 256 + threadIdx.x;
      if (i + 1 < n) {
        uint32_t w0[DW], w1[DW];
        ld_elem<DW>(data + i * DW, w0);
        ld_elem<DW>(data + (i + 1) * DW, w1);
        const Key x = key_of<T>(w0), y = key_of<T>(w1);
        desc |= kless(y, x) ? 1u : 0u;
        asc |= kless(x, y) ? 1u : 0u;
      }
    }
    // a flag already seen set needs no atomic (a sorted input would otherwise
    // send one atomic per wavefront and chunk to the same word)
    if (!had_desc && __any(desc) && (threadIdx.x & 63) == 0) atomicOr(&ctrl[CTRL_DESC], 1u);
    if (!had_asc && __any(asc) && (threadIdx.x & 63) == 0) atomicOr(&ctrl[CTRL_ASC], 1u);
  }
}

// Cheap first look at sortedness: 65536 adjacent pairs spread evenly over
// the array.  If it already finds an ascent and a descent, the input is
// neither sorted nor reverse sorted and the full scan is skipped.
template <class T>
__global__ void __launch_bounds__(1024) k_sorted_sample(const uint32_t* data, uint64_t n, uint32_t* ctrl) {
  using Key = typename T::Key;
  constexpr int DW = T::DW;
  constexpr uint64_t PAIRS = 65536;
  uint32_t desc = 0, asc = 0;
  for (uint64_t j = (uint64_t)blockIdx.x * 1024 + threadIdx.x; j < PAIRS; j += (uint64_t)gridDim.x * 1024) {
    const uint64_t i = (uint64_t)(((unsigned __int128)j * (n - 1)) / PAIRS);
    if (i + 1 < n) {
      uint32_t w0[DW], w1[DW];
      ld_elem<DW>(data + i * DW, w0);
      ld_elem<DW>(data + (i + 1) * DW, w1);
      const Key x = key_of<T>(w0), y = key_of<T>(w1);
      desc |= kless(y, x) ? 1u : 0u;
      asc |= kless(x, y) ? 1u : 0u;
    }
  }
  if (__any(desc) && (threadIdx.x & 63) == 0) atomicOr(&ctrl[CTRL_DESC], 1u);
  if (__any(asc) && (threadIdx.x & 63) == 0) atomicOr(&ctrl[CTRL_ASC], 1u);
}

template <int DW>
__global__ void __launch_bounds__(256) k_reverse(uint32_t* data, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n / 2; i += (uint64_t)gridDim.x * 256) {
    uint32_t x[DW], y[DW];
    ld_elem<DW>(data + i * DW, x);
    ld_elem<DW>(data + (n - 1 - i) * DW, y);
    st_elem<DW>(data + i * DW, y);
    st_elem<DW>(data + (n - 1 - i) * DW, x);
  }
}

// Minimum and maximum radix key of the whole input (significant-bit
// detection of the radix variant).
template <class T>
__global__ void __launch_bounds__(256) k_minmax(const uint32_t* data, uint64_t n, uint32_t* ctrl) {
  constexpr int DW = T::DW;
  constexpr int U = 8;   // loads in flight per lane
  // A workgroup reads U * 256 consecutive elements per round (contiguous
  // chunks, as a streaming copy does), then moves on by the grid's span.
  const uint64_t stride = (uint64_t)gridDim.x * 256 * U;
  uint64_t mn = ~0ull, mx = 0;
  for (uint64_t i0 = (uint64_t)blockIdx.x * 256 * U + threadIdx.x; i0 < n; i0 += stride) {
    uint32_t w[U][DW];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = i0 + (uint64_t)u * 256;
      if (i < n) ld_elem<DW>(data + i * DW, w[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + (uint64_t)u * 256 < n) {
        const uint64_t k = T::rkey(key_of<T>(w[u]));
        mn = k < mn ? k : mn;
        mx = k > mx ? k : mx;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t a = (uint64_t)__shfl_xor((long long)mn, o, 64);
    const uint64_t b = (uint64_t)__shfl_xor((long long)mx, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if ((threadIdx.x & 63) == 0) {
    uint64_t* mm = reinterpret_cast<uint64_t*>(ctrl + CTRL_MINMAX);
    atomicMin((unsigned long long*)&mm[0], (unsigned long long)mn);
    atomicMax((unsigned long long*)&mm[1], (unsigned long long)mx);
  }
}

// Per-segment order check of a batched call (the sorted-input detection of
// Section 6 applied to every segment): flags[2 seg] is set on a descent,
// flags[2 seg + 1] on an ascent.  A chunk compares each element with its
// predecessor unless the element starts the segment, 2048 pairs per round;
// it stops after the first round in which the workgroup has seen both a
// descent and an ascent, since the segment can then be neither sorted nor
// reverse sorted whatever the rest holds (random input stops after one
// round, nearly sorted input after a few; only sorted runs read the whole
// chunk).
template <class T>
__global__ void __launch_bounds__(256) k_seg_order(const SegItem* items, const uint32_t* data,
                                                   uint32_t* flags) {
  using Key = typename T::Key;
  constexpr int DW = T::DW;
  constexpr uint32_t U = 8;
  const SegItem it = items[blockIdx.x];
  uint32_t desc = 0, asc = 0;
  const uint32_t q0 = it.first ? 1u : 0u;
  for (uint32_t base = q0; base < it.n; base += 256 * U) {
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      const uint32_t q = base + u * 256 + threadIdx.x;
      if (q < it.n) {
        uint32_t w0[DW], w1[DW];
        ld_elem<DW>(data + (it.l + q - 1) * DW, w0);
        ld_elem<DW>(data + (it.l + q) * DW, w1);
        const Key x = key_of<T>(w0), y = key_of<T>(w1);
        desc |= kless(y, x) ? 1u : 0u;
        asc |= kless(x, y) ? 1u : 0u;
      }
    }
    // (both votes return the same value to every thread)
    if (__syncthreads_or((int)desc) && __syncthreads_or((int)asc)) break;
  }
  if (__any(desc) && (threadIdx.x & 63) == 0) atomicOr(&flags[2 * it.seg], 1u);
  if (__any(asc) && (threadIdx.x & 63) == 0) atomicOr(&flags[2 * it.seg + 1], 1u);
}

// In-place reversal of reverse-sorted segments, one workgroup per chunk.
template <int DW>
__global__ void __launch_bounds__(256) k_seg_reverse(const RevItem* items, uint32_t* data) {
  const RevItem it = items[blockIdx.x];
  for (uint32_t q = threadIdx.x; q < it.cn; q += 256) {
    const uint64_t i = it.c0 + q, j = it.len - 1 - i;
    uint32_t x[DW], y[DW];
    ld_elem<DW>(data + (it.l + i) * DW, x);
    ld_elem<DW>(data + (it.l + j) * DW, y);
    st_elem<DW>(data + (it.l + i) * DW, y);
    st_elem<DW>(data + (it.l + j) * DW, x);
  }
}

// Per-segment key range of a batched radix call: one workgroup per chunk,
// combined with 64-bit atomics into smin[seg] / smax[seg] (which start at
// all ones / zero).  The root digit of each segment is taken below the
// highest bit in which its smallest and largest keys differ (Section 6).
template <class T>
__global__ void __launch_bounds__(256) k_seg_minmax(const SegItem* items, const uint32_t* data,
                                                    uint64_t* smin, uint64_t* smax) {
  constexpr int DW = T::DW;
  const SegItem it = items[blockIdx.x];
  uint64_t mn = ~0ull, mx = 0;
  for (uint32_t i = threadIdx.x; i < it.n; i += 256) {
    uint32_t w[DW];
    ld_elem<DW>(data + (it.l + i) * DW, w);
    const uint64_t k = T::rkey(key_of<T>(w));
    mn = k < mn ? k : mn;
    mx = k > mx ? k : mx;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t a = (uint64_t)__shfl_xor((long long)mn, o, 64);
    const uint64_t b = (uint64_t)__shfl_xor((long long)mx, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin((unsigned long long*)&smin[it.seg], (unsigned long long)mn);
    atomicMax((unsigned long long*)&smax[it.seg], (unsigned long long)mx);
  }
}

#ifdef IPS_COMMON_KERNELS
// Children of every task of a batch (Section 4.2).  A bucket of at most one
// element, an equality bucket, or (radix) a bucket whose keys are all equal
// is final; a bucket of at most caps[2] elements becomes an LDS-tier task of
// the smallest variant that holds it; any other bucket becomes a next-level
// task (with equality buckets forced on when it holds the whole parent, and
// for radix with the digit below the highest bit in which its keys differ).
struct Child {
  uint32_t dest;            // 0..2: LDS-tier variant, 3: next level, 4: final
  uint32_t tflags, shift, width;
  uint64_t s0, sz;
};

__device__ __forceinline__ Child child_of(const BatchArgs& a, const ChildArgs& c, const PTask& tk, uint32_t j) {
  Child ch;
  ch.dest = 4; ch.tflags = 0; ch.shift = 0; ch.width = 0;
  const bool radix = (tk.tflags & TF_RADIX) != 0;
  const uint32_t bb = tk.bucket_base;
  ch.s0 = a.b_start[bb + j];
  ch.sz = a.b_start[bb + j + 1] - ch.s0;
  if (ch.sz <= 1) return ch;
  if (!radix && tk.eq && (j & 1u) && j != 2 * tk.K - 1) return ch;   // equality bucket
  if (radix) {
    const uint64_t mn = a.b_min[bb + j], mx = a.b_max[bb + j];
    if (mn == mx) return ch;
    const uint32_t h = 63u - (uint32_t)__clzll(mn ^ mx);
    ch.shift = h >= 7 ? h - 7 : 0;
    ch.width = h - ch.shift + 1;
  } else if (ch.sz == tk.n) {
    ch.tflags = TF_EQ_ON;   // no progress without equality buckets
  }
  if (c.ins_parent) {   // the paper's base-case rule: size <= 2 n0, or the parent <= k n0
    ch.dest = (ch.sz <= c.caps[0] || tk.n <= c.ins_parent) ? 0u : 3u;
    return ch;
  }
  ch.dest = ch.sz <= c.caps[2] ? (ch.sz <= c.caps[0] ? 0u : (ch.sz <= c.caps[1] ? 1u : 2u)) : 3u;
  return ch;
}

// Workgroups take the tasks by stride, threads the buckets.  A first pass
// counts each workgroup's children per destination in LDS, one atomic per
// destination reserves the workgroup's positions in the lists (or the task
// queue), and a second pass writes the entries: the shared counters see one
// atomic per workgroup instead of one per child.  `ntask` is the number of
// tasks (device-planned steps read it from the control block).
__global__ void __launch_bounds__(256) k_children(BatchArgs a, ChildArgs c, uint32_t ntask) {
  const uint32_t T = a.devplan ? a.ctrl[CTRL_T] : ntask;
  const uint32_t nseg = a.ctrl[CTRL_NSEG];
  __shared__ uint32_t s_n[4], s_base[4], s_pos[4];
  __shared__ unsigned long long s_el[3];
  const uint32_t tid = threadIdx.x;
  if (tid < 4) { s_n[tid] = 0; s_pos[tid] = 0; }
  if (tid < 3) s_el[tid] = 0;
  __syncthreads();
  for (uint32_t ti = blockIdx.x; ti < T; ti += gridDim.x) {
    const PTask& tk = a.tasks[ti];
    for (uint32_t j = tid; j < tk.nb; j += 256) {
      const Child ch = child_of(a, c, tk, j);
      if (ch.dest < 4) atomicAdd(&s_n[ch.dest], 1u);
      if (ch.dest < 3) atomicAdd(&s_el[ch.dest], (unsigned long long)ch.sz);
      if (ch.dest == 4 && ch.sz && nseg)   // serving: a final bucket's elements are done
        atomicAdd(&seg_done_ptr(a.ctrl)[seg_find(a.ctrl, nseg, tk.l + ch.s0)], (unsigned long long)ch.sz);
    }
  }
  __syncthreads();
  if (tid < 4 && s_n[tid]) {
    uint32_t* ctr = tid < 3 ? a.ctrl + CTRL_NLDS + tid : (a.devplan ? a.ctrl + CTRL_QTAIL : a.ctrl + CTRL_NNEXT);
    s_base[tid] = atomicAdd(ctr, s_n[tid]);
  }
  if (tid < 3 && s_el[tid]) {
    unsigned long long* ldsel = reinterpret_cast<unsigned long long*>(a.ctrl + CTRL_LDSEL);
    atomicAdd(&ldsel[tid], s_el[tid]);
    atomicAdd((unsigned long long*)(a.ctrl + CTRL_LDSELT), s_el[tid]);
    if (a.devplan && a.step < MAX_STEPS_RECORDED)
      atomicAdd((unsigned long long*)&a.step_el[a.step * 4 + 1 + tid], s_el[tid]);
  }
  if (tid == 0 && s_n[0] + s_n[1] + s_n[2]) atomicAdd(&a.ctrl[CTRL_LDSTASKS], s_n[0] + s_n[1] + s_n[2]);
  __syncthreads();
  for (uint32_t ti = blockIdx.x; ti < T; ti += gridDim.x) {
    const PTask& tk = a.tasks[ti];
    for (uint32_t j = tid; j < tk.nb; j += 256) {
      const Child ch = child_of(a, c, tk, j);
      if (ch.dest >= 4) continue;
      const uint32_t q = s_base[ch.dest] + atomicAdd(&s_pos[ch.dest], 1u);
      if (ch.dest < 3) {
        if (q < c.lt_cap) {
          LTask t;
          t.l = tk.l + ch.s0;
          t.n = (uint32_t)ch.sz;
          t.req = nseg ? seg_find(a.ctrl, nseg, t.l) : 0u;   // serving: the task's request
          c.lt[ch.dest][q] = t;
        } else {
          dev_error(a.ctrl, DE_CLN_RANGE, ti, q);
        }
      } else {
        CTask t;
        t.l = tk.l + ch.s0;
        t.n = ch.sz;
        t.level = tk.level + 1;
        t.tflags = ch.tflags;
        t.shift = ch.shift;
        t.width = ch.width;
        if (a.devplan) {           // onto the task queue
          if (q - a.ctrl[CTRL_QHEAD] < a.qcap) a.queue[q % a.qcap] = t;
          else dev_error(a.ctrl, DE_QUEUE, ti, q);
        } else {
          if (q < c.next_cap) c.next[q] = t;
          else dev_error(a.ctrl, DE_CLN_RANGE, ti, q);
        }
      }
    }
  }
}

// ------------------------------------------- device-planned execution
//
// The host plans a batch from bucket sizes it reads back; here the same
// rules run on the device, so that a sequence of steps needs no host
// round trip: k_plan_pop takes the next tasks from the queue while the
// workspace budgets hold, the sampling phase runs, k_plan_geom lays out
// blocks, stripes, buffer slots, pieces and permutation groups, and every
// later kernel of the step reads its workgroup count from the control block.

// Buckets k' of a task (Section 4.2): the paper's adaptive rule when n0 is
// given, otherwise the smallest power of two that makes the mean bucket at
// most a quarter of the LDS-tier capacity.
__device__ uint32_t dev_kprime(const PlanCfg& c, uint64_t n, uint32_t level) {
  const uint32_t k = level ? c.k : c.k_root;
  if (c.n0) {
    const uint64_t kn0 = (uint64_t)k * c.n0, kkn0 = kn0 * k;
    uint64_t r = k;
    if (n > kn0 && n < kkn0) {
      uint32_t q = 1;
      while (shl64(c.n0, 2 * q - 1) < n) ++q;
      r = bit64(q);
    } else if (n > c.n0 && n <= kn0) {
      uint32_t q = 0;
      while (shl64(c.n0, q) < n) ++q;
      r = bit64(q);
    }
    return (uint32_t)(r < 2 ? 2 : (r > k ? k : r));
  }
  uint64_t r = 2;
  while (r < k && r * (c.cap / 4) < n) r *= 2;
  return (uint32_t)r;
}

// Block elements of a step with nb buckets (one LDS buffer block per bucket
// unless the buffers are global).
__device__ uint32_t dev_block_elems(const PlanCfg& c, uint32_t nb) {
  const uint32_t bmax = MAX_BLOCK_BYTES / c.D ? MAX_BLOCK_BYTES / c.D : 1;
  if (c.gbuf) {
    const uint32_t b = c.b_req ? c.b_req : 1;
    return b < bmax ? b : bmax;
  }
  uint32_t b = c.buf_bytes / (nb * c.D);
  if (!b) b = 1;
  if (b > bmax) b = bmax;
  if (c.b_req && c.b_req < b) b = c.b_req;
  return b;
}

// Inclusive prefix sum of one value per thread over a block of NT threads.
template <uint32_t NT>
__device__ uint64_t block_incl_scan64(uint64_t v, uint64_t* s_w, uint64_t* total) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = (uint64_t)__shfl_up((long long)inc, o, 64);
    if ((int)lane >= o) inc += y;
  }
  __syncthreads();
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  uint64_t base = 0, tot = 0;
  for (uint32_t w = 0; w < NT / 64; ++w) {
    if (w < wave) base += s_w[w];
    tot += s_w[w];
  }
  *total = tot;
  return base + inc;
}

constexpr uint32_t PLAN_THREADS = 512;   // >= tasks per batch

// Takes the next tasks from the queue, in order, while the batch's resource
// needs (estimated for the stripe length of all candidates) fit the
// workspace budgets; at least one task when the queue is not empty.
__global__ void __launch_bounds__(PLAN_THREADS) k_plan_pop(BatchArgs a, PlanCfg c) {
  __shared__ uint64_t s_w[PLAN_THREADS / 64];
  __shared__ uint32_t s_take;
  const uint32_t t = threadIdx.x;
  const uint32_t head = a.ctrl[CTRL_QHEAD], tail = a.ctrl[CTRL_QTAIL];
  // after any consistency error nothing more is taken (the host reports it)
  const uint32_t avail = a.ctrl[CTRL_ERR] ? 0u : tail - head;
  const uint32_t cand = avail < c.TB ? avail : c.TB;
  CTask q;
  q.l = 0; q.n = 0; q.level = 0; q.tflags = 0; q.shift = 0; q.width = 0;
  if (t < cand) q = a.queue[(head + t) % a.qcap];
  uint64_t tot_n = 0;
  (void)block_incl_scan64<PLAN_THREADS>(t < cand ? q.n : 0, s_w, &tot_n);
  uint64_t S = tot_n / c.wg_target ? tot_n / c.wg_target : 1;
  // Stripes long enough that all candidates fit the workgroup budget (each
  // task adds at most one rounding workgroup): with a budget below the
  // stripe target, a stripe length taken from the candidates alone would
  // let every step take only part of the queue, and the next step (fewer
  // candidates, shorter stripes) again only part of the rest.
  if (c.WB > cand) {
    const uint64_t room = c.WB - cand, Sw = (tot_n + room - 1) / room;
    if (Sw > S) S = Sw;
  }
  // resource needs of the task (upper bounds, as the host estimates them)
  uint64_t nw = 0, nslot = 0, nspill = 0, npieces = 0;
  if (t < cand) {
    const uint64_t wub = (q.n + S - 1) / S;
    nw = wub < c.wg_target ? wub : c.wg_target;
    if (nw > c.WB) nw = c.WB;
    const uint64_t s2 = q.n * c.D / 4 + nw * 256;
    nslot = nw * c.slot_max;
    if (nslot > (s2 > c.slot_max ? s2 : c.slot_max)) nslot = s2 > c.slot_max ? s2 : c.slot_max;
    nspill = c.slot_max;
    const uint32_t nbt = c.radix ? MAX_K : 2 * dev_kprime(c, q.n, q.level);   // buckets at most
    const uint32_t bmin = dev_block_elems(c, nbt);
    npieces = 2ull * nbt + 3 + nw + (q.n / bmin + 1) / c.cmax + 1;
  }
  uint64_t tw, tsl, tsp, tpc;
  const uint64_t pw = block_incl_scan64<PLAN_THREADS>(nw, s_w, &tw);
  const uint64_t psl = block_incl_scan64<PLAN_THREADS>(nslot, s_w, &tsl);
  const uint64_t psp = block_incl_scan64<PLAN_THREADS>(nspill, s_w, &tsp);
  const uint64_t ppc = block_incl_scan64<PLAN_THREADS>(npieces, s_w, &tpc);
  if (t == 0) s_take = cand;
  __syncthreads();
  const bool fits = pw <= c.WB && psl <= c.SB && psp <= c.SPB && ppc <= c.PB;
  if (t < cand && t > 0 && !fits) atomicMin(&s_take, t);
  __syncthreads();
  const uint32_t T = s_take;
  if (t < T) {
    PTask& p = const_cast<PTask*>(a.tasks)[t];
    p.l = q.l;
    p.n = q.n;
    p.level = q.level;
    p.tflags = q.tflags | (c.radix ? TF_RADIX : 0u);
    p.shift = q.shift;
    p.width = q.width;
    p.kp = c.radix ? 0u : dev_kprime(c, q.n, q.level);
  }
  // statistics
  uint64_t tn = 0, mx = t < T ? q.n : 0;
  (void)block_incl_scan64<PLAN_THREADS>(t < T ? q.n : 0, s_w, &tn);
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t y = (uint64_t)__shfl_xor((long long)mx, o, 64);
    mx = y > mx ? y : mx;
  }
  if ((t & 63) == 0 && mx) atomicMax((unsigned long long*)(a.ctrl + CTRL_MAXSTEP), (unsigned long long)mx);
  if (t < T) atomicMax(&a.ctrl[CTRL_LEVELS], q.level + 1);
  if (t == 0) {
    if (a.step < MAX_STEPS_RECORDED) a.step_el[a.step * 4] = tn;
    a.ctrl[CTRL_T] = T;
    a.ctrl[CTRL_QHEAD] = head + T;
    *reinterpret_cast<uint64_t*>(a.ctrl + CTRL_SPOP) = S;
    a.ctrl[CTRL_STEPS] += T;
    a.ctrl[CTRL_BATCHES] += T ? 1u : 0u;
    *reinterpret_cast<uint64_t*>(a.ctrl + CTRL_PARTEL) += tn;
  }
}

// Geometry of the step's tasks after sampling: blocks, stripes (about one
// WG_TARGET-th of the batch each, fewer while the budgets are exceeded),
// buffer slots, spill areas, pieces, permutation groups and the
// workgroup-to-task maps of the later kernels.
__global__ void __launch_bounds__(PLAN_THREADS) k_plan_geom(BatchArgs a, PlanCfg c) {
  __shared__ uint64_t s_w[PLAN_THREADS / 64];
  __shared__ uint32_t s_ok;
  const uint32_t t = threadIdx.x;
  const uint32_t T = a.ctrl[CTRL_T];
  if (T == 0) {
    if (t == 0) {
      a.ctrl[CTRL_NWG] = 0; a.ctrl[CTRL_NPWG] = 0; a.ctrl[CTRL_NCLN] = 0;
      a.ctrl[CTRL_MAXW] = 0;
    }
    return;
  }
  const bool act = t < T;
  PTask p;
  if (act) p = a.tasks[t];
  uint32_t K = 0, logK = 0, eq = 0, nb = 0;
  if (act) {
    if (c.radix) {
      K = 1u << p.width; logK = p.width; eq = 0; nb = K;
    } else {
      const StepRec* rec = a.recs + t;
      K = rec->K; logK = rec->logK; eq = rec->eq; nb = rec->nb;
    }
  }
  const uint32_t b = act ? dev_block_elems(c, nb) : 1;
  // ceil(n / b); a power of two b divides by a shift built from 32-bit operations
  const uint32_t NB = !act ? 0u
                           : ((b & (b - 1)) == 0 ? (uint32_t)shr64(p.n + b - 1, (uint32_t)__builtin_ctz(b))
                                                 : (uint32_t)((p.n + b - 1) / b));
  const uint64_t slot_bytes = act ? (((uint64_t)nb * b * c.D + 255) & ~255ull) : 0;
  uint64_t tot_n = 0;
  (void)block_incl_scan64<PLAN_THREADS>(act ? p.n : 0, s_w, &tot_n);
  const uint64_t S_pop = *reinterpret_cast<const uint64_t*>(a.ctrl + CTRL_SPOP);
  uint64_t S = tot_n / c.wg_target ? tot_n / c.wg_target : 1;
  uint32_t W = 0;
  for (;;) {
    if (act) {
      uint64_t w = (p.n + S / 2) / S;
      if (!w) w = 1;
      const uint64_t wcap = p.n / (4ull * nb * b);
      if (w > (wcap ? wcap : 1)) w = wcap ? wcap : 1;
      if (w > NB) w = NB;
      if (w > c.wg_target) w = c.wg_target;
      if (w > c.WB) w = c.WB;
      W = (uint32_t)w;
    }
    uint64_t sw, ss;
    (void)block_incl_scan64<PLAN_THREADS>(act ? W : 0, s_w, &sw);
    (void)block_incl_scan64<PLAN_THREADS>(act ? (uint64_t)W * slot_bytes : 0, s_w, &ss);
    if ((sw <= c.WB && ss <= c.SB) || S >= S_pop) break;
    S *= 2;
  }
  if (S > S_pop) S = S_pop;   // (the loop ends there at the latest)
  uint64_t blocks_sum = 0;
  (void)block_incl_scan64<PLAN_THREADS>(act ? NB : 0, s_w, &blocks_sum);
  uint32_t gl = 4;
  while (gl * PERM_RD < b * c.DW) gl *= 2;
  uint64_t ng = act ? (uint64_t)c.groups * NB / (blocks_sum ? blocks_sum : 1) : 0;
  if (act) {
    if (ng > NB / 4) ng = NB / 4;
    if (!ng) ng = 1;
  }
  const uint32_t gpw = c.perm_threads / gl;
  const uint32_t nwg = act ? ((uint32_t)ng + gpw - 1) / gpw : 0;   // ng <= NB / 4 fits 32 bits
  const uint32_t piece_cap = act ? 2 * nb + 2 + W + NB / c.cmax + 1 : 0;
  uint64_t t_wg, t_slot, t_spill, t_piece, t_bucket, t_pwg, t_cln;
  // Classification workgroups: the tasks whose stripes are longer than S
  // take the first indices (workgroups start roughly in index order, so the
  // longest start first and the shorter ones fill the end of the launch).
  const bool lng = act && (uint64_t)W * S < p.n;
  uint64_t t_wl, t_ws;
  const uint64_t e_wl = block_incl_scan64<PLAN_THREADS>(lng ? W : 0, s_w, &t_wl) - (lng ? W : 0);
  const uint64_t e_ws = block_incl_scan64<PLAN_THREADS>((act && !lng) ? W : 0, s_w, &t_ws) -
                        ((act && !lng) ? W : 0);
  const uint64_t e_wg = lng ? e_wl : t_wl + e_ws;
  t_wg = t_wl + t_ws;
  const uint64_t e_slot = block_incl_scan64<PLAN_THREADS>(act ? W * slot_bytes : 0, s_w, &t_slot) -
                          (act ? W * slot_bytes : 0);
  const uint64_t e_spill = block_incl_scan64<PLAN_THREADS>(slot_bytes, s_w, &t_spill) - slot_bytes;
  const uint64_t e_piece = block_incl_scan64<PLAN_THREADS>(piece_cap, s_w, &t_piece) - piece_cap;
  const uint64_t e_bucket = block_incl_scan64<PLAN_THREADS>(act ? nb + 1 : 0, s_w, &t_bucket) - (act ? nb + 1 : 0);
  const uint64_t e_pwg = block_incl_scan64<PLAN_THREADS>(nwg, s_w, &t_pwg) - nwg;
  const uint64_t e_cln = block_incl_scan64<PLAN_THREADS>(act ? nb : 0, s_w, &t_cln) - (act ? nb : 0);
  uint32_t maxw = W;
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t y = (uint32_t)__shfl_xor((int)maxw, o, 64);
    maxw = y > maxw ? y : maxw;
  }
  if (t == 0) s_ok = 1;
  __syncthreads();
  if (t == 0 && (t_wg > c.WB || t_pwg > c.PWB || t_slot > c.SB || t_spill > c.SPB ||
                 t_piece > c.PB || t_bucket > c.NBE || t_cln > c.CLNB)) {
    s_ok = 0;
    dev_error(a.ctrl, DE_PLAN, (uint32_t)T, (uint32_t)t_wg);
  }
  if ((t & 63) == 0) atomicMax(&a.ctrl[CTRL_MAXW], maxw);
  __syncthreads();
  if (!s_ok) {
    if (t == 0) {
      a.ctrl[CTRL_T] = 0; a.ctrl[CTRL_NWG] = 0; a.ctrl[CTRL_NPWG] = 0; a.ctrl[CTRL_NCLN] = 0;
    }
    return;
  }
  if (act) {
    PTask& q = const_cast<PTask*>(a.tasks)[t];
    q.nb = nb; q.K = K; q.logK = logK; q.eq = eq;
    q.b = b; q.NB = NB; q.W = W; q.wg_base = (uint32_t)e_wg;
    q.slot_bytes = (uint32_t)slot_bytes; q.slot_off = e_slot;
    q.spill_off = e_spill;
    q.piece_base = (uint32_t)e_piece; q.piece_cap = piece_cap;
    q.bucket_base = (uint32_t)e_bucket;
    q.glanes = gl; q.ngrp = (uint32_t)ng; q.pwg_base = (uint32_t)e_pwg;
  }
  // Workgroup-to-task maps of the later kernels, one wavefront per task (a
  // task may own tens of thousands of entries, a step up to PLAN_THREADS tasks).
  __shared__ uint32_t s_mb[3][PLAN_THREADS], s_mc[3][PLAN_THREADS];
  s_mb[0][t] = (uint32_t)e_wg;  s_mc[0][t] = act ? W : 0;
  s_mb[1][t] = (uint32_t)e_pwg; s_mc[1][t] = act ? nwg : 0;
  s_mb[2][t] = (uint32_t)e_cln; s_mc[2][t] = act ? nb : 0;
  __syncthreads();
  {
    uint32_t* cls = const_cast<uint32_t*>(a.cls_task);
    uint32_t* perm = const_cast<uint32_t*>(a.perm_task);
    uint32_t* cln = const_cast<uint32_t*>(a.cln_map);
    const uint32_t lane = t & 63;
    for (uint32_t i = t >> 6; i < T; i += PLAN_THREADS / 64) {
      for (uint32_t x = lane; x < s_mc[0][i]; x += 64) cls[s_mb[0][i] + x] = i;
      for (uint32_t x = lane; x < s_mc[1][i]; x += 64) perm[s_mb[1][i] + x] = i;
      for (uint32_t x = lane; x < s_mc[2][i]; x += 64) cln[s_mb[2][i] + x] = (i << 10) | x;
    }
  }
  if (t == 0) {
    a.ctrl[CTRL_NWG] = (uint32_t)t_wg;
    a.ctrl[CTRL_NPWG] = (uint32_t)t_pwg;
    a.ctrl[CTRL_NCLN] = (uint32_t)t_cln;
  }
}

// Device-planned steps defer the LDS tier: the children of several steps
// collect in the lists (2 * step_cap entries per variant) and are sorted in
// one pass, which keeps the tier's launches large.  After a step's children
// the lists run when they hold at least `min_tasks` tasks, when a list could
// overflow during the next step (more than step_cap entries), or when the
// task queue is empty (nothing further will be added); ctrl[CTRL_LDSRUN]
// tells the step's LDS-tier launches and k_lds_reset.
__global__ void k_lds_decide(uint32_t* ctrl, uint32_t min_tasks, uint32_t step_cap) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t n0 = ctrl[CTRL_NLDS], n1 = ctrl[CTRL_NLDS + 1], n2 = ctrl[CTRL_NLDS + 2];
  const uint32_t pending = n0 + n1 + n2;
  const bool full = n0 > step_cap || n1 > step_cap || n2 > step_cap;
  const bool last = ctrl[CTRL_QHEAD] == ctrl[CTRL_QTAIL];
  ctrl[CTRL_LDSRUN] = (pending && (pending >= min_tasks || full || last)) ? 1u : 0u;
}

// After the LDS-tier launches of a step: empty the lists if they ran.
__global__ void k_lds_reset(uint32_t* ctrl) {
  const uint32_t t = threadIdx.x;
  if (!ctrl[CTRL_LDSRUN]) return;
  __syncthreads();   // every lane has read the flag
  if (t < 3) { ctrl[CTRL_NLDS + t] = 0; ctrl[CTRL_LDSPOP + t] = 0; }
  if (t < 6) ctrl[CTRL_LDSEL + t] = 0;
  __syncthreads();
  if (t == 0) ctrl[CTRL_LDSRUN] = 0;
}

// Fills p[0, *count) with v.
__global__ void __launch_bounds__(256) k_fill32_cnt(uint32_t* p, const uint32_t* count, uint32_t v) {
  const uint32_t n = *count;
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = v;
}

__global__ void __launch_bounds__(256) k_fill32(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) p[i] = v;
}
#endif  // IPS_COMMON_KERNELS

}  // namespace ips
