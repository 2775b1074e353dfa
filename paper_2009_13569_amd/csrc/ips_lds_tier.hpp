// LDS tier: a task small enough for one workgroup is loaded once, sorted
// inside LDS and registers, and stored once (the base case of the
// recursion; Section 6 of arXiv 2009.13569 uses insertion sort for IPS4o and
// a radix sort for IPS2Ra).  Here the base case is itself one distribution
// pass plus tiny sorts:
//   1. keys go to registers; the task's minimum and maximum are reduced;
//   2. each key gets the bin (key - min) >> shift, where shift leaves about
//      NET/4 keys per bin (equal-width bins over the key range);
//   3. bin counts by LDS atomics, an exclusive scan, a scatter into LDS;
//   4. each thread sorts one bin of at most NET/2 keys with a register
//      bitonic network of size NET/4 or NET/2, the smaller one that holds it
//      (bins are grouped by that size, one pass per size); in the same phase
//      each bin of NET/2 .. WAVE_NET keys is sorted by one wavefront with a
//      bitonic network in registers across its lanes (one or two keys per
//      lane, partners read by lane shuffles), or, when the bin spans at most
//      64 possible key values, by a counting sort over those values (ranks
//      from ballots; duplicate-heavy inputs make such bins); a bin whose keys
//      are all equal needs nothing;
//   5. a bin above WAVE_NET keys is binned again by the whole workgroup over
//      its own key range (bins that collect many keys are the ones skewed or
//      duplicate-heavy inputs produce): its sub-bins of at most NET/2 keys
//      are sorted in registers at once, larger ones are queued again; every
//      round splits a bin (its minimum and maximum land in different
//      sub-bins) and a sub-bin of one value is final;
//   6. only if a list overflows does the whole task fall back to a
//      block-wide bitonic network in LDS;
//   7. one coalesced store (records of up to four dwords are gathered from
//      their input positions in HBM, wider ones from their LDS copy).
#pragma once
#include "ips_kernels.hpp"

namespace ips {

constexpr uint32_t WAVE_NET = 128;    // largest bin sorted by one wavefront's network
constexpr uint32_t WAVE_CNT = 512;    // largest bin sorted by one wavefront's counting sort (keys only;
                                      // half that with indices, for registers)
constexpr uint32_t FATCAP = 128;      // bins waiting to be binned again (each > WAVE_NET keys)
constexpr uint32_t FAT_ROUNDS = 1024; // re-binning rounds per task before the fallback

// Order-preserving unsigned image of a key for binning.
__device__ __forceinline__ uint64_t bin_image(uint32_t k) { return k; }
__device__ __forceinline__ uint64_t bin_image(uint64_t k) { return k; }
__device__ __forceinline__ unsigned __int128 bin_image(const K80& k) {
  return ((unsigned __int128)k.hi << 16) | (unsigned __int128)k.lo;
}
__device__ __forceinline__ uint64_t shfl_xor_img(uint64_t v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ unsigned __int128 shfl_xor_img(unsigned __int128 v, int m) {
  const uint64_t lo = shfl_xor_img((uint64_t)v, m), hi = shfl_xor_img((uint64_t)(v >> 64), m);
  return ((unsigned __int128)hi << 64) | lo;
}

// Exclusive prefix sum of cnt[0, nb) into off[0, nb] by the whole block.
template <uint32_t NT>
__device__ void block_excl_scan(const uint32_t* cnt, uint32_t* off, uint32_t nb, uint32_t* s_wsum) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t per = (nb + NT - 1) / NT;
  const uint32_t b0 = tid * per;
  uint32_t loc = 0;
  for (uint32_t i = 0; i < per; ++i)
    if (b0 + i < nb) loc += cnt[b0 + i];
  uint32_t inc = loc;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)inc, o, 64);
    if ((int)lane >= o) inc += y;
  }
  if (lane == 63) s_wsum[wave] = inc;
  __syncthreads();
  uint32_t wbase = 0;
  for (uint32_t w = 0; w < wave; ++w) wbase += s_wsum[w];
  uint32_t acc = wbase + inc - loc;
  for (uint32_t i = 0; i < per; ++i) {
    if (b0 + i < nb) { off[b0 + i] = acc; acc += cnt[b0 + i]; }
  }
  if (tid == NT - 1) {
    uint32_t tot = 0;
    for (uint32_t w = 0; w < NT / 64; ++w) tot += s_wsum[w];
    off[nb] = tot;
  }
  __syncthreads();
}

__device__ __forceinline__ uint32_t bitlen(uint64_t x) { return x ? 64u - __clzll(x) : 0u; }
__device__ __forceinline__ uint32_t bitlen(unsigned __int128 x) {
  const uint64_t hi = (uint64_t)(x >> 64);
  return hi ? 128u - __clzll(hi) : bitlen((uint64_t)x);
}

template <class Key, bool IDX>
__device__ __forceinline__ void ce_up(Key& a, Key& b, uint32_t& ia, uint32_t& ib) {
  const bool sw = kless(b, a) || (IDX && keq(a, b) && ib < ia);
  const Key ta = a, tb = b;
  a = ksel(sw, tb, ta);
  b = ksel(sw, ta, tb);
  if (IDX) {
    const uint32_t ua = ia, ub = ib;
    ia = sw ? ub : ua;
    ib = sw ? ua : ub;
  }
}

// One stage of the all-ascending bitonic network on N register keys: the
// first step of each merge of size K compares i with i ^ (K - 1), the later
// steps (half size J) compare i with i ^ J.  Template parameters keep every
// register index a compile-time constant.
template <uint32_t N, uint32_t K, uint32_t J, class Key, bool IDX>
__device__ __forceinline__ void net_stage(Key (&v)[N], uint32_t (&ix)[N]) {
#pragma unroll
  for (uint32_t i = 0; i < N; ++i) {
    const uint32_t p = (J == K / 2) ? (i ^ (K - 1)) : (i ^ J);
    if (p > i) ce_up<Key, IDX>(v[i], v[p], ix[i], ix[p]);
  }
}

template <uint32_t N, uint32_t K, uint32_t J, class Key, bool IDX>
__device__ __forceinline__ void net_merge(Key (&v)[N], uint32_t (&ix)[N]) {
  net_stage<N, K, J, Key, IDX>(v, ix);
  if constexpr (J > 1) net_merge<N, K, J / 2, Key, IDX>(v, ix);
}

template <uint32_t N, uint32_t K, class Key, bool IDX>
__device__ __forceinline__ void net_sort(Key (&v)[N], uint32_t (&ix)[N]) {
  net_merge<N, K, K / 2, Key, IDX>(v, ix);
  if constexpr (K < N) net_sort<N, 2 * K, Key, IDX>(v, ix);
}

// Sorts N register keys ascending; padding with the largest key at the end
// stays in place because every comparator puts the minimum at the lower index.
template <uint32_t N, class Key, bool IDX>
__device__ __forceinline__ void reg_network(Key (&v)[N], uint32_t (&ix)[N]) {
  net_sort<N, 2, Key, IDX>(v, ix);
}

// A key from lane `src` of the wavefront (every dword of it).
template <class Key>
__device__ __forceinline__ Key shfl_key(const Key& k, uint32_t src) {
  constexpr int KW = (int)(sizeof(Key) / 4);
  uint32_t w[KW];
  __builtin_memcpy(w, &k, sizeof(Key));
#pragma unroll
  for (int d = 0; d < KW; ++d) w[d] = (uint32_t)__shfl((int)w[d], (int)src, 64);
  Key r;
  __builtin_memcpy(&r, w, sizeof(Key));
  return r;
}

// One wavefront sorts keys[0, s) (s <= 64 R) and their indices in
// registers, R keys per lane (element i = lane * R + r), with the same
// all-ascending network over the next power of two, padded with the largest
// key.  A comparator whose partner i ^ m lies in another lane reads the
// partner through a lane shuffle; the lower index keeps the smaller of the
// two (key, index) pairs, the upper one the larger, so both sides of a
// comparator agree.
template <class T, bool IDX, uint32_t R>
__device__ void wave_reg_network(typename T::Key* keys, uint16_t* idx, uint32_t s) {
  using Key = typename T::Key;
  static_assert(R == 1 || R == 2, "one or two keys per lane");
  const uint32_t lane = threadIdx.x & 63;
  uint32_t P = 2;
  while (P < s) P <<= 1;
  Key v[R];
  uint32_t ix[R];
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t i = lane * R + r;
    v[r] = i < s ? keys[i] : T::kmax();
    ix[r] = i < s ? (IDX ? (uint32_t)idx[i] : 0u) : 0xFFFFFFFFu;
  }
  for (uint32_t K = 2; K <= P; K <<= 1) {
    for (uint32_t J = K >> 1; J > 0; J >>= 1) {
      const uint32_t m = (J == (K >> 1)) ? K - 1 : J;   // partner i ^ m
      Key nv[R];
      uint32_t nix[R];
#pragma unroll
      for (uint32_t r = 0; r < R; ++r) {
        const uint32_t i = lane * R + r;
        const uint32_t pr = r ^ (m & (R - 1));            // partner's register
        const Key own = ksel(pr == 0, v[0], v[R - 1]);
        const uint32_t oix = (pr == 0) ? ix[0] : ix[R - 1];
        Key pv = own;
        uint32_t pix = oix;
        if (m >= R) {                                       // partner in lane lane ^ (m / R)
          const uint32_t pl = lane ^ (m / R);
          pv = shfl_key(own, pl);
          if (IDX) pix = (uint32_t)__shfl((int)oix, (int)pl, 64);
        }
        const bool pless = kless(pv, v[r]) || (IDX && keq(pv, v[r]) && pix < ix[r]);
        const bool mless = kless(v[r], pv) || (IDX && keq(v[r], pv) && ix[r] < pix);
        const bool take = (i & J) == 0 ? pless : mless;
        nv[r] = ksel(take, pv, v[r]);
        nix[r] = take ? pix : ix[r];
      }
#pragma unroll
      for (uint32_t r = 0; r < R; ++r) { v[r] = nv[r]; ix[r] = nix[r]; }
    }
  }
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t i = lane * R + r;
    if (i < s) {
      keys[i] = v[r];
      if (IDX) idx[i] = (uint16_t)ix[r];
    }
  }
}

// Counting-sort information of a binning with shift ush from image mn: a
// bin spans at most 2^ush consecutive images, so for ush <= 6 a key's rank
// inside its bin is (image - mn) mod 2^ush, and only mn mod 64 is needed.
// Bits 0-2: ush + 1 (0: no counting sort), bits 3-8: mn mod 64.
template <class Img>
__device__ __forceinline__ uint32_t count_info(uint32_t ush, Img mn) {
  return ush <= 6 ? ((ush + 1) | (((uint32_t)mn & 63u) << 3)) : 0u;
}

// One wavefront sorts keys[0, s) (s <= 64 R, R per lane) whose images lie
// in a window of 2^ush <= 64 consecutive values starting at an image equal
// to mnl modulo 64: each key's value index d = (image - mnl) mod 2^ush, and
// for each value in turn the lanes holding it take the next places, ranked
// by ballots.  Equal keys end up in an arbitrary order.
template <class T, bool IDX, uint32_t R>
__device__ void wave_count_sort(typename T::Key* keys, uint16_t* idx, uint32_t s, uint32_t ush,
                                uint32_t mnl) {
  using Key = typename T::Key;
  using Img = decltype(bin_image(Key()));
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t nv = 1u << ush, mask = nv - 1;
  Key v[R];
  uint32_t ix[R], d[R], pos[R];
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t i = lane * R + r;
    d[r] = nv;            // no key
    pos[r] = 0;
    ix[r] = 0;
    if (i < s) {
      v[r] = keys[i];
      if (IDX) ix[r] = idx[i];
      d[r] = (uint32_t)(bin_image(v[r]) - (Img)mnl) & mask;
    }
  }
  uint32_t base = 0;
  for (uint32_t val = 0; val < nv && base < s; ++val) {
    uint32_t below = 0;
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
      const uint64_t m = __ballot(d[r] == val);
      if (d[r] == val) pos[r] = base + below + lanes_below(m);
      below += (uint32_t)__popcll(m);
    }
    base += below;
  }
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    if (lane * R + r < s) {
      keys[pos[r]] = v[r];
      if (IDX) idx[pos[r]] = (uint16_t)ix[r];
    }
  }
}

// Whole-task fallback: block-wide all-ascending network over keys[0, s).
template <class Key, bool IDX>
__device__ void block_network(Key* keys, uint16_t* idx, uint32_t s) {
  uint32_t P = 1;
  while (P < s) P <<= 1;
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
        const uint32_t p = (j == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j);
        if (p > i && p < s) {
          Key a = keys[i], b = keys[p];
          uint32_t ia = IDX ? idx[i] : 0, ib = IDX ? idx[p] : 0;
          const bool sw = kless(b, a) || (IDX && keq(a, b) && ib < ia);
          if (sw) {
            keys[i] = b; keys[p] = a;
            if (IDX) { idx[i] = (uint16_t)ib; idx[p] = (uint16_t)ia; }
          }
        }
      }
      __syncthreads();
    }
  }
}

// Sorts the s <= N keys keys[o, o + s) (and their indices) with a register
// network of size N, padding with the largest key.
template <class T, bool IDX, uint32_t N>
__device__ __forceinline__ void sort_bin(typename T::Key* keys, uint16_t* idxb, uint32_t o, uint32_t s) {
  typename T::Key v[N];
  uint32_t ix[N];
#pragma unroll
  for (uint32_t i = 0; i < N; ++i) {
    v[i] = (i < s) ? keys[o + i] : T::kmax();
    ix[i] = (i < s) ? (IDX ? (uint32_t)idxb[o + i] : 0u) : 0xFFFFFFFFu;
  }
  reg_network<N, typename T::Key, IDX>(v, ix);
#pragma unroll
  for (uint32_t i = 0; i < N; ++i) {
    if (i < s) {
      keys[o + i] = v[i];
      if constexpr (IDX) idxb[o + i] = (uint16_t)ix[i];
    }
  }
}

template <class T, uint32_t NT, uint32_t E, uint32_t NET>
struct LdsTier {
  using Key = typename T::Key;
  static constexpr uint32_t CAP = NT * E;
  static constexpr uint32_t MEAN = NET / 4;   // target keys per bin
  static constexpr uint32_t MAXBINS = (CAP / MEAN < 2048) ? CAP / MEAN : 2048;
  static constexpr bool IDX = !T::KEYS_ONLY;
  // Records of up to four dwords (Pair) are not staged: the keys come from
  // HBM like keys alone, (key, index) pairs are sorted, and the store
  // gathers each record from its input position (every gather of the task
  // returns before its first store), which leaves twice the capacity of a
  // staged record in LDS.  Wider records are staged in LDS and gathered
  // from there.
  static constexpr bool GATHER = IDX && T::DW <= 4;
  static constexpr bool STAGE = IDX && !GATHER;
  // dynamic LDS: keys[CAP] | idx[CAP] (records) | stage[CAP * DW] (staged records)
  static constexpr size_t lds_bytes() {
    return (size_t)CAP * sizeof(Key) + (IDX ? (size_t)CAP * 2 : 0) + (STAGE ? (size_t)CAP * T::DW * 4 : 0);
  }
};

// Sorts LDS-tier task number `ti` of the list.
// `pf`: thread 0 loads descriptor lt[nxt] of the workgroup's next task into
// *s_t (free once every thread has read the current one), the load issued
// before this task's key loads and stored after them.
template <class T, uint32_t NT, uint32_t E, uint32_t NET>
__device__ void lds_tier_task(const LTask t, uint32_t ti, uint32_t* data, uint32_t* ctrl, uint32_t tid,
                              const LTask* lt, uint32_t nxt, bool pf, LTask* s_t) {
  using LT = LdsTier<T, NT, E, NET>;
  using Key = typename T::Key;
  using Img = decltype(bin_image(Key()));
  constexpr int DW = T::DW;
  constexpr uint32_t CAP = LT::CAP, MAXBINS = LT::MAXBINS;
  constexpr bool IDX = LT::IDX, GATHER = LT::GATHER, STAGE = LT::STAGE;
  extern __shared__ __align__(16) uint8_t s_raw[];
  __shared__ uint32_t s_cnt[MAXBINS];
  __shared__ uint32_t s_off[MAXBINS + 1];
  __shared__ Img s_min[NT / 64], s_max[NT / 64];
  __shared__ uint16_t s_list[MAXBINS];       // bins grouped by size class
  __shared__ uint32_t s_ccnt[2];
  constexpr uint32_t MIDCAP = MAXBINS / 2;   // > CAP / (NET/2 + 1): never overflows
  __shared__ uint32_t s_mid[MIDCAP];         // (offset << 16) | size, for the wavefronts
  __shared__ uint16_t s_midc[MIDCAP];        // and its counting-sort information
  __shared__ uint32_t s_fat_o[FATCAP], s_fat_s[FATCAP];
  __shared__ uint32_t s_wsum[NT / 64];
  __shared__ uint32_t s_nmid, s_mdone, s_fat_head, s_fat_tail, s_fallback;

  Key* keys = reinterpret_cast<Key*>(s_raw);
  uint16_t* idxb = reinterpret_cast<uint16_t*>(keys + CAP);
  uint32_t* stage = reinterpret_cast<uint32_t*>(idxb + CAP);
  const uint32_t n = t.n, lane = tid & 63, wave = tid >> 6;
  const bool pf0 = pf && tid == 0;
#ifdef IPS_LDS_STATS
  // cycles of the task's phases seen by thread 0, added to control words
  // 32.. (load, min/max, binning, bin sorts, re-binning, store, tasks)
  uint64_t lt0 = __builtin_readcyclecounter();
  auto LSTAT = [&](int i) {
    if (tid == 0) {
      const uint64_t t1 = __builtin_readcyclecounter();
      atomicAdd(reinterpret_cast<unsigned long long*>(ctrl + 32) + i, (unsigned long long)(t1 - lt0));
      lt0 = t1;
    }
  };
#else
  auto LSTAT = [](int) {};
#endif
  if (n > CAP || n < 2) {
    if (tid == 0 && n > CAP) dev_error(ctrl, DE_LDST, ti, n);
    if (pf0) *s_t = lt[nxt];
    return;
  }
  uint32_t* gd = data + t.l * DW;
  LTask nt = t;
  if (pf0) nt = lt[nxt];
  if (tid == 0) { s_nmid = 0; s_mdone = 0; s_fat_head = 0; s_fat_tail = 0; s_fallback = 0; }
  if constexpr (STAGE) {   // wide records: staged in LDS, gathered at the store
    // SU dwords per lane are loaded before any is stored, so their loads overlap
    constexpr uint32_t SU = 8;
    const uint32_t tot = n * DW;
    for (uint32_t x0 = tid; x0 < tot; x0 += NT * SU) {
      uint32_t v[SU];
#pragma unroll
      for (uint32_t u = 0; u < SU; ++u) {
        const uint32_t x = x0 + u * NT;
        v[u] = x < tot ? gd[x] : 0u;
      }
#pragma unroll
      for (uint32_t u = 0; u < SU; ++u) {
        const uint32_t x = x0 + u * NT;
        if (x < tot) stage[x] = v[u];
      }
    }
  }

  // A bin of more than NET/2 keys at [o, o + sz): listed for a wavefront up
  // to WAVE_NET keys (WAVE_CNT keys when it spans at most 64 values),
  // otherwise queued for another binning round.  A list entry is
  // o << 16 | sz, beside cinfo, the counting-sort information of the
  // binning that made the bin (see count_info).
  auto push_big = [&](uint32_t o, uint32_t sz, uint32_t cinfo) {
    if (sz <= WAVE_NET || (cinfo && sz <= (IDX ? WAVE_CNT / 2 : WAVE_CNT))) {
      const uint32_t slot = atomicAdd(&s_nmid, 1u);
      if (slot < MIDCAP) { s_mid[slot] = (o << 16) | sz; s_midc[slot] = (uint16_t)cinfo; }
      else s_fallback = 1;
    } else {
      const uint32_t slot = atomicAdd(&s_fat_tail, 1u);
      if (slot - s_fat_head < FATCAP) {
        s_fat_o[slot % FATCAP] = o;
        s_fat_s[slot % FATCAP] = sz;
      } else {
        s_fallback = 1;
      }
    }
  };

  // Bins sorted by size class: up to NET/4 and up to NET/2 keys are sorted
  // in registers by one thread each with a network of that size (each class
  // in its own pass, so that a wavefront runs one network size); larger bins
  // go to the wavefront list or the queue of re-binning rounds.  Bin b of
  // nbins lies at o + s_off[b] and holds s_cnt[b] keys.
  // The list of each class is built without per-bin atomics: a bin's place
  // is its rank among the wavefront's bins of that class (ballots) after the
  // wavefront's base (one counter update per wavefront and class).
  auto sort_bins = [&](uint32_t o, uint32_t nbins, uint32_t cinfo) {
    constexpr uint32_t BPT = (MAXBINS + NT - 1) / NT;   // bins per thread
    uint32_t cls_of[BPT], rk[BPT];
    if (tid < 2) s_ccnt[tid] = 0;
    __syncthreads();
    uint32_t run0 = 0, run1 = 0;
#pragma unroll
    for (uint32_t q = 0; q < BPT; ++q) {
      const uint32_t b = q * NT + tid;
      cls_of[q] = 4;
      if (b < nbins) {
        const uint32_t sz = s_cnt[b];
        if (sz > 1) {
          cls_of[q] = sz <= NET / 4 ? 0u : (sz <= NET / 2 ? 1u : 3u);
          if (cls_of[q] == 3) push_big(o + s_off[b], sz, cinfo);
        }
      }
      const uint64_t m0 = __ballot(cls_of[q] == 0), m1 = __ballot(cls_of[q] == 1);
      rk[q] = cls_of[q] == 0 ? run0 + lanes_below(m0) : run1 + lanes_below(m1);
      run0 += (uint32_t)__popcll(m0);
      run1 += (uint32_t)__popcll(m1);
    }
    uint32_t wb0 = 0, wb1 = 0;
    if (lane == 0) {
      wb0 = atomicAdd(&s_ccnt[0], run0);
      wb1 = atomicAdd(&s_ccnt[1], run1);
    }
    wb0 = (uint32_t)__builtin_amdgcn_readlane((int)wb0, 0);
    wb1 = (uint32_t)__builtin_amdgcn_readlane((int)wb1, 0);
    __syncthreads();
    const uint32_t n0 = s_ccnt[0], n1 = s_ccnt[1];
#pragma unroll
    for (uint32_t q = 0; q < BPT; ++q) {
      const uint32_t c = cls_of[q];
      if (c == 0) s_list[wb0 + rk[q]] = (uint16_t)(q * NT + tid);
      else if (c == 1) s_list[n0 + wb1 + rk[q]] = (uint16_t)(q * NT + tid);
    }
    __syncthreads();
    for (uint32_t q = tid; q < n0; q += NT) {
      const uint32_t b = s_list[q];
      sort_bin<T, IDX, NET / 4>(keys, idxb, o + s_off[b], s_cnt[b]);
    }
    for (uint32_t q = tid; q < n1; q += NT) {
      const uint32_t b = s_list[n0 + q];
      sort_bin<T, IDX, NET / 2>(keys, idxb, o + s_off[b], s_cnt[b]);
    }
    // The bins of NET/2 .. WAVE_NET keys listed since the last call, one per
    // wavefront, from the last wavefront down (the class passes give the
    // first threads the most bins); a bin of one value needs nothing.
    const uint32_t m0 = s_mdone, m1 = s_nmid < MIDCAP ? s_nmid : MIDCAP;
    if (!s_fallback) {
      for (uint32_t q = m0 + (NT / 64 - 1 - wave); q < m1; q += NT / 64) {
        const uint32_t ent = s_mid[q], mo = ent >> 16, ms = ent & 0xFFFFu;
        const uint32_t ci = s_midc[q], cu = ci & 7u, cm = (ci >> 3) & 63u;
        bool same = true;
        for (uint32_t i = lane; i < ms; i += 64) same = same && keq(keys[mo + i], keys[mo]);
        if (__all(same)) continue;
        if (cu) {   // at most 64 possible values: counting sort by value
          if (ms <= 64) wave_count_sort<T, IDX, 1>(keys + mo, idxb + mo, ms, cu - 1, cm);
          else if (ms <= 128) wave_count_sort<T, IDX, 2>(keys + mo, idxb + mo, ms, cu - 1, cm);
          else if (IDX || ms <= 256) wave_count_sort<T, IDX, 4>(keys + mo, idxb + mo, ms, cu - 1, cm);
          else wave_count_sort<T, IDX, IDX ? 4 : 8>(keys + mo, idxb + mo, ms, cu - 1, cm);
        } else if (ms <= 64) {
          wave_reg_network<T, IDX, 1>(keys + mo, idxb + mo, ms);
        } else {
          wave_reg_network<T, IDX, 2>(keys + mo, idxb + mo, ms);
        }
      }
    }
    __syncthreads();
    if (tid == 0) s_mdone = m1;
  };

  // 1. Load keys into registers (staged records: from their LDS stage).
  Key k[E];
  if constexpr (STAGE) {
    __syncthreads();
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t i = e * NT + tid;
      if (i < n) {
        const uint32_t* r = stage + i * DW;
        k[e] = T::key_w(r);
      }
    }
  } else {
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t i = e * NT + tid;
      if (i < n) {
        uint32_t w[DW];
        if constexpr (GATHER) {   // the key dwords only
          static_assert(T::KDW == 2, "gathered records have two key dwords");
          const uint2 v = *reinterpret_cast<const uint2*>(gd + (uint64_t)i * DW);
          w[0] = v.x;
          w[1] = v.y;
          k[e] = T::key_w(w);
        } else {
          ld_elem<DW>(gd + (uint64_t)i * DW, w);
          k[e] = key_of<T>(w);
        }
      }
    }
  }
  Img mn = ~(Img)0, mx = 0;
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    if (e * NT + tid < n) {
      const Img b = bin_image(k[e]);
      mn = b < mn ? b : mn;
      mx = b > mx ? b : mx;
    }
  }
  for (int sh = 32; sh > 0; sh >>= 1) {
    const Img a2 = shfl_xor_img(mn, sh), b2 = shfl_xor_img(mx, sh);
    mn = a2 < mn ? a2 : mn;
    mx = b2 > mx ? b2 : mx;
  }
  LSTAT(0);
  if (lane == 0) { s_min[wave] = mn; s_max[wave] = mx; }
  if (pf0) *s_t = nt;
  for (uint32_t j = tid; j < MAXBINS; j += NT) s_cnt[j] = 0;
  __syncthreads();
  LSTAT(1);
  mn = s_min[0];
  mx = s_max[0];
  for (uint32_t w = 1; w < NT / 64; ++w) {
    mn = s_min[w] < mn ? s_min[w] : mn;
    mx = s_max[w] > mx ? s_max[w] : mx;
  }
  if (mn == mx) return;   // all keys equal: already sorted

  // 2./3. Bins of about MEAN keys over [mn, mx], counts, scan, scatter.
  {
    uint32_t lb = 1;
    while ((1u << lb) < MAXBINS && (1u << lb) * LT::MEAN < n) ++lb;
    const uint32_t span = bitlen((Img)(mx - mn));
    const uint32_t nbins = 1u << lb;
    const uint32_t ush = uniform_amount(span > lb ? span - lb : 0);   // the same in every lane
    uint32_t bin[E], rk[E];
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      if (e * NT + tid < n) {
        bin[e] = (uint32_t)((Img)(bin_image(k[e]) - mn) >> ush);
        rk[e] = atomicAdd(&s_cnt[bin[e]], 1u);
      }
    }
    __syncthreads();
    block_excl_scan<NT>(s_cnt, s_off, nbins, s_wsum);
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t i = e * NT + tid;
      if (i < n) {
        const uint32_t q = s_off[bin[e]] + rk[e];
        keys[q] = k[e];
        if constexpr (IDX) idxb[q] = (uint16_t)i;
      }
    }
    __syncthreads();
    LSTAT(2);
    // 4. Bins by size class.
    sort_bins(0, nbins, count_info(ush, mn));
    LSTAT(3);
  }

  // 5. Re-binning rounds, one queued bin [o, o + s) at a time by the whole
  // workgroup: the keys (and indices) are copied, counted by sub-bin, and
  // scattered back from the copy through per-sub-bin cursors.  The copy is
  // the task's own range in HBM, which is free until the store, one key per
  // thread at a time; with gathered records that range still holds the
  // input, so the copy is in registers (at most E keys per thread).
  constexpr uint32_t KW = (uint32_t)(sizeof(Key) / 4);        // key dwords
  constexpr uint32_t SW = KW + (IDX ? 1u : 0u);               // copy dwords per element
  static_assert(SW <= (uint32_t)DW, "the copy of an element fits the element");
  constexpr uint32_t RE = GATHER ? E : 1;                     // register copy per thread
  for (uint32_t round = 0;; ++round) {
    const uint32_t head = s_fat_head, tail = s_fat_tail;
    if (head == tail || s_fallback) break;
    if (round >= FAT_ROUNDS) {
      __syncthreads();
      if (tid == 0) s_fallback = 1;
      __syncthreads();
      break;
    }
    const uint32_t o = s_fat_o[head % FATCAP], s = s_fat_s[head % FATCAP];
    Img mn2 = ~(Img)0, mx2 = 0;
    Key rx[RE];
    uint32_t ri[RE];
    if constexpr (GATHER) {
#pragma unroll
      for (uint32_t e = 0; e < RE; ++e) {
        const uint32_t i = e * NT + tid;
        rx[e] = Key();
        ri[e] = 0;
        if (i < s) {
          rx[e] = keys[o + i];
          ri[e] = idxb[o + i];
          const Img b = bin_image(rx[e]);
          mn2 = b < mn2 ? b : mn2;
          mx2 = b > mx2 ? b : mx2;
        }
      }
    } else {
      for (uint32_t i = tid; i < s; i += NT) {
        const Key x = keys[o + i];
        const Img b = bin_image(x);
        mn2 = b < mn2 ? b : mn2;
        mx2 = b > mx2 ? b : mx2;
        uint32_t* dst = gd + (uint64_t)(o + i) * DW;
        const uint32_t* xw = reinterpret_cast<const uint32_t*>(&x);
#pragma unroll
        for (uint32_t d = 0; d < KW; ++d) dst[d] = xw[d];
        if constexpr (IDX) dst[KW] = idxb[o + i];
      }
    }
    for (int sh = 32; sh > 0; sh >>= 1) {
      const Img a2 = shfl_xor_img(mn2, sh), b2 = shfl_xor_img(mx2, sh);
      mn2 = a2 < mn2 ? a2 : mn2;
      mx2 = b2 > mx2 ? b2 : mx2;
    }
    __syncthreads();   // every lane has read head and the entry
    if (lane == 0) { s_min[wave] = mn2; s_max[wave] = mx2; }
    if (tid == 0) s_fat_head = head + 1;
    for (uint32_t j = tid; j < MAXBINS; j += NT) s_cnt[j] = 0;
    __syncthreads();
    mn2 = s_min[0];
    mx2 = s_max[0];
    for (uint32_t w = 1; w < NT / 64; ++w) {
      mn2 = s_min[w] < mn2 ? s_min[w] : mn2;
      mx2 = s_max[w] > mx2 ? s_max[w] : mx2;
    }
    if (mn2 == mx2) continue;   // one value: final (the next round reads the list after the barrier above)
    uint32_t lb2 = 1;
    while ((1u << lb2) < MAXBINS && (1u << lb2) * LT::MEAN < s) ++lb2;
    const uint32_t span2 = bitlen((Img)(mx2 - mn2));
    const uint32_t nsub = 1u << lb2;
    const uint32_t ush2 = uniform_amount(span2 > lb2 ? span2 - lb2 : 0);
    for (uint32_t i = tid; i < s; i += NT)
      atomicAdd(&s_cnt[(uint32_t)((Img)(bin_image(keys[o + i]) - mn2) >> ush2)], 1u);
    __syncthreads();
    block_excl_scan<NT>(s_cnt, s_off, nsub, s_wsum);
    for (uint32_t j = tid; j < nsub; j += NT) s_cnt[j] = s_off[j];   // cursors
    __syncthreads();
    if constexpr (GATHER) {
#pragma unroll
      for (uint32_t e = 0; e < RE; ++e) {
        if (e * NT + tid < s) {
          const uint32_t p = o + atomicAdd(&s_cnt[(uint32_t)((Img)(bin_image(rx[e]) - mn2) >> ush2)], 1u);
          keys[p] = rx[e];
          idxb[p] = (uint16_t)ri[e];
        }
      }
    } else {
      for (uint32_t i = tid; i < s; i += NT) {
        const uint32_t* src = gd + (uint64_t)(o + i) * DW;
        Key x;
        uint32_t* xw = reinterpret_cast<uint32_t*>(&x);
#pragma unroll
        for (uint32_t d = 0; d < KW; ++d) xw[d] = src[d];
        const uint32_t p = o + atomicAdd(&s_cnt[(uint32_t)((Img)(bin_image(x) - mn2) >> ush2)], 1u);
        keys[p] = x;
        if constexpr (IDX) idxb[p] = (uint16_t)src[KW];
      }
    }
    __syncthreads();
    for (uint32_t j = tid; j < nsub; j += NT) s_cnt[j] = s_off[j + 1] - s_off[j];   // sizes
    __syncthreads();
    sort_bins(o, nsub, count_info(ush2, mn2));
  }

  // 6. (Bins of NET/2 .. WAVE_NET keys were sorted with their size classes.)
  // A list overflow leaves the whole task to the block-wide network.
  __syncthreads();
  if (s_fallback) block_network<Key, IDX>(keys, idxb, n);
  __syncthreads();
  LSTAT(4);

  // 7. Store.
  if constexpr (GATHER) {
    // Each thread gathers the records of its output positions from their
    // input positions in HBM; every gather of the workgroup has returned (an
    // opaque use of each loaded register) before the barrier that precedes
    // the first store.
    uint32_t v[E][DW];
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t i = e * NT + tid;
#pragma unroll
      for (int d = 0; d < DW; ++d) v[e][d] = 0;
      if (i < n) ld_elem<DW>(gd + (uint64_t)idxb[i] * DW, v[e]);
    }
#pragma unroll
    for (uint32_t e = 0; e < E; ++e)
#pragma unroll
      for (int d = 0; d < DW; ++d) asm volatile("" ::"v"(v[e][d]) : "memory");
    __syncthreads();
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t i = e * NT + tid;
      if (i < n) st_elem<DW>(gd + (uint64_t)i * DW, v[e]);
    }
  } else if constexpr (IDX) {
    constexpr uint32_t SU = 8;
    const uint32_t tot = n * DW;
    for (uint32_t x0 = tid; x0 < tot; x0 += NT * SU) {
      uint32_t v[SU];
#pragma unroll
      for (uint32_t u = 0; u < SU; ++u) {
        const uint32_t x = x0 + u * NT;
        if (x < tot) {
          const uint32_t i = x / DW, d = x - i * DW;
          v[u] = stage[(uint32_t)idxb[i] * DW + d];
        }
      }
#pragma unroll
      for (uint32_t u = 0; u < SU; ++u) {
        const uint32_t x = x0 + u * NT;
        if (x < tot) gd[x] = v[u];
      }
    }
  } else {
    for (uint32_t i = tid; i < n; i += NT) {
      uint32_t w[DW];
      T::from_key(keys[i], w);
      st_elem<DW>(gd + (uint64_t)i * DW, w);
    }
  }
  LSTAT(5);
#ifdef IPS_LDS_STATS
  if (tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(ctrl + 32) + 6, 1ull);
#endif
}

// One workgroup per task of the list (cnt == nullptr: the grid is the
// list).  With a device count `cnt` (at most cnt_cap) the workgroups claim
// tasks from the counter `pop` (zero at launch) until the list is used up,
// so that long and short tasks balance as with one workgroup per task.
// Claims run one task ahead: while a task is sorted, the next one is
// already claimed and its descriptor is loading (issued before the task's
// key loads, so it waits with them), and the claim after it is in flight.
template <class T, uint32_t NT, uint32_t E, uint32_t NET>
__global__ void __launch_bounds__(NT, (NT <= 512 ? 4 : 1))
k_lds_tier(const LTask* lt, uint32_t* data, uint32_t* ctrl, const uint32_t* cnt, uint32_t cnt_cap,
           uint32_t* pop) {
  __shared__ uint32_t s_next, s_after;
  __shared__ LTask s_t;
  uint32_t count, ti;
  // Serving: a finished task adds its elements to its request's counter
  // (the table is read here, before any store, so that no wait at a task's
  // end is tied to its stores).
  const uint32_t nseg = ctrl[CTRL_NSEG];
  unsigned long long* const seg_done = nseg ? seg_done_ptr(ctrl) : nullptr;
  if (cnt) {
    if (!ctrl[CTRL_LDSRUN]) return;          // device-planned step that defers the lists
    count = *cnt < cnt_cap ? *cnt : cnt_cap;   // a list never holds more than cnt_cap
    if (threadIdx.x == 0) {
      const uint32_t c0 = atomicAdd(pop, 1u);
      s_after = atomicAdd(pop, 1u);
      s_next = c0;
      if (c0 < count) s_t = lt[c0];
    }
  } else {
    ti = blockIdx.x;
    count = ti + 1;
    if (threadIdx.x == 0) { s_next = ti; s_t = lt[ti]; }
  }
  __syncthreads();
  ti = s_next;
  while (ti < count) {
    const LTask t = s_t;
    __syncthreads();   // every thread has read s_next and s_t
    // The thread index is made opaque on every pass so that the compiler
    // recomputes the many addresses derived from it inside the loop instead
    // of keeping them all live across it (which costs registers).
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t nxt = count, after = count;   // the grid's own task only, without a device count
    if (cnt && tid == 0) {
      nxt = s_after;                       // claimed during the previous task
      after = atomicAdd(pop, 1u);
    }
    lds_tier_task<T, NT, E, NET>(t, ti, data, ctrl, tid, lt, nxt, cnt && nxt < count, &s_t);
    if (tid == 0) {
      s_next = nxt;
      s_after = after;
      if (seg_done) atomicAdd(&seg_done[t.req], (unsigned long long)t.n);   // serving: elements final
    }
    __syncthreads();
    ti = s_next;
  }
}

// LDS tier of the Quartet, whose 192-bit keys the binning above has no
// image for: (key, index) pairs of the task, padded to a power of two, are
// sorted by a bitonic network in LDS, and the records are gathered from the
// task's region in key order into registers and stored back over it.  LDS
// holds the pairs only (26 bytes per element), not the records, so that up
// to seven 512-element tasks run on a CU at once.  Same calling convention
// as k_lds_tier (a list, or claims from a device count).
template <class T, uint32_t CAP>
__global__ void __launch_bounds__(256)
k_lds_bitonic(const LTask* lt, uint32_t* data, uint32_t* ctrl, const uint32_t* cnt, uint32_t cnt_cap,
              uint32_t* pop) {
  using Key = typename T::Key;
  constexpr uint32_t NT = 256;
  constexpr int DW = T::DW;
  static_assert(DW % 2 == 0 && CAP % NT == 0, "records move as aligned 8-byte words, CAP / NT per thread");
  extern __shared__ __align__(16) uint8_t s_raw[];
  Key* keys = reinterpret_cast<Key*>(s_raw);
  uint16_t* idx = reinterpret_cast<uint16_t*>(keys + CAP);
  __shared__ uint32_t s_next;
  __shared__ LTask s_t;
  uint32_t count;
  if (cnt) {
    if (!ctrl[CTRL_LDSRUN]) return;
    count = *cnt < cnt_cap ? *cnt : cnt_cap;
  } else {
    count = gridDim.x;   // one workgroup per task of the list
  }
  const uint32_t tid = threadIdx.x;
  const uint32_t nseg = ctrl[CTRL_NSEG];
  unsigned long long* const seg_done = nseg ? seg_done_ptr(ctrl) : nullptr;
  for (uint32_t it = 0;; ++it) {
    if (tid == 0) {
      const uint32_t nx = cnt ? atomicAdd(pop, 1u) : (it == 0 ? blockIdx.x : count);
      s_next = nx;
      if (nx < count) s_t = lt[nx];
    }
    __syncthreads();
    const uint32_t ti = s_next;
    if (ti >= count) break;
    const LTask t = s_t;
    const uint32_t n = t.n;
    if (n > CAP) {
      if (tid == 0) dev_error(ctrl, DE_LDST, ti, n);
    } else if (n >= 2) {
      // Keys come straight from the records (the task's region is read again
      // for the gather below, from the caches); only (key, index) pairs live
      // in LDS, so that more tasks fit on a CU at once.
      const uint32_t* const gd = data + t.l * DW;
      uint32_t P = 1;
      while (P < n) P <<= 1;
#pragma unroll
      for (uint32_t r = 0; r < CAP / NT; ++r) {
        const uint32_t i = r * NT + tid;
        if (i < P) {
          keys[i] = i < n ? T::key_w(gd + (uint64_t)i * DW) : T::kmax();
          idx[i] = (uint16_t)(i < n ? i : 0xFFFFu);
        }
      }
      __syncthreads();
      for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
          for (uint32_t i = tid; i < P / 2; i += NT) {
            const uint32_t lo = (i / j) * 2 * j + (i % j), hi = lo + j;
            const bool up = (lo & k) == 0;
            const Key x = keys[lo], y = keys[hi];
            const uint16_t ix = idx[lo], iy = idx[hi];
            // (key, index) order: padding (index 0xFFFF) sorts last among equal keys
            const bool gt = kless(y, x) || (keq(x, y) && iy < ix);
            if (gt == up) { keys[lo] = y; keys[hi] = x; idx[lo] = iy; idx[hi] = ix; }
          }
          __syncthreads();
        }
      }
      // Gather: every record of the task is read into registers in key order,
      // each value used before the barrier (so every load has returned), and
      // only then are the records stored over the task's region.
      // Each thread moves 8-byte words x = u * NT + tid of the output, word
      // x % (DW / 2) of the record that sorts to position x / (DW / 2).
      constexpr uint32_t RW = CAP / NT * (DW / 2);
      const uint32_t m = n * (DW / 2);
      const uint2* const src = reinterpret_cast<const uint2*>(gd);
      uint2 v[RW];
#pragma unroll
      for (uint32_t u = 0; u < RW; ++u) {
        const uint32_t x = u * NT + tid;
        if (x < m) {
          const uint32_t i = x / (DW / 2), w = x - i * (DW / 2);
          v[u] = src[(uint64_t)idx[i] * (DW / 2) + w];
        }
      }
#pragma unroll
      for (uint32_t u = 0; u < RW; ++u)
        if (u * NT + tid < m) asm volatile("" ::"v"(v[u].x), "v"(v[u].y));
      __syncthreads();
      uint2* const g2 = reinterpret_cast<uint2*>(data + t.l * DW);
#pragma unroll
      for (uint32_t u = 0; u < RW; ++u) {
        const uint32_t x = u * NT + tid;
        if (x < m) g2[x] = v[u];
      }
    }
    if (tid == 0 && seg_done) atomicAdd(&seg_done[t.req], (unsigned long long)t.n);   // serving
    __syncthreads();   // LDS reused by the next task; s_next read by every thread
  }
}

// The paper's base case (Section 4.2): insertion sort of one small task
// per thread, in place in global memory (the elements of a task of a few
// dozen elements stay in the caches).  Used with IPS_FLAG_INSERTION_BASE,
// where a bucket of at most 2 n0 elements, or any bucket of a task of at
// most k n0 elements, is a base case.  Same calling convention as
// k_lds_tier (a list of nt tasks, or a device count).
template <class T>
__global__ void __launch_bounds__(256)
k_insertion(const LTask* lt, uint32_t nt, uint32_t* data, uint32_t* ctrl, const uint32_t* cnt, uint32_t cnt_cap) {
  constexpr int DW = T::DW;
  if (cnt && !ctrl[CTRL_LDSRUN]) return;
  const uint32_t count = cnt ? (*cnt < cnt_cap ? *cnt : cnt_cap) : nt;
  const uint32_t nseg = ctrl[CTRL_NSEG];
  unsigned long long* const seg_done = nseg ? seg_done_ptr(ctrl) : nullptr;
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < count; i += gridDim.x * 256) {
    const LTask t = lt[i];
    uint32_t* g = data + t.l * DW;
    for (uint32_t x = 1; x < t.n; ++x) {
      uint32_t e[DW];
      ld_elem<DW>(g + (uint64_t)x * DW, e);
      const typename T::Key k = T::key_w(e);
      uint32_t y = x;
      while (y > 0) {
        uint32_t p[DW];
        ld_elem<DW>(g + (uint64_t)(y - 1) * DW, p);
        if (!kless(k, T::key_w(p))) break;
        st_elem<DW>(g + (uint64_t)y * DW, p);
        --y;
      }
      st_elem<DW>(g + (uint64_t)y * DW, e);
    }
    if (seg_done) atomicAdd(&seg_done[t.req], (unsigned long long)t.n);   // serving
  }
}

template <class T, uint32_t CAP>
constexpr size_t lds_bitonic_bytes() {
  return (size_t)CAP * sizeof(typename T::Key) + (size_t)CAP * 2;
}

}  // namespace ips
