// Radix partitioning step with classification fused into the block
// permutation, from exact bucket sizes (the memory-volume idea of the
// paper's future work, Section 8: determine exact bucket sizes first, as
// radix sorts and the original super scalar samplesort do, then integrate
// the classification and permutation phases, still moving blocks between
// local buffer blocks and the array).
//
// A step of one task runs three kernels:
//  - k_fhist: every workgroup counts the digits of its stripe and adds the
//    counts to the task's bucket counters (read D bytes per element);
//  - k_fscan: bucket starts s_j from the counts, and per bucket a packed
//    pointer word (w, r) with w = s_j and r = s_{j+1}: [s_j, w) holds
//    bucket j's elements, [w, r) unread input, [r, s_{j+1}) input that a
//    workgroup has claimed (read out, or being read);
//  - k_fused: every workgroup holds one LDS buffer block per bucket (as in
//    classification).  It classifies a tile of elements into the buffers;
//    for every block a tile completes it reserves the next b positions of
//    the bucket (w += b, one atomic per bucket and tile), reads the input
//    still unread in them and then writes the block there.  What it read is
//    its next tile; when a tile would be short it claims unread input from
//    the top of a bucket's range (r -= c).  Reserved positions that were
//    claimed earlier are written only after every claimed read of the
//    bucket has finished (the paper's reader counter, per bucket: a count
//    of finished claimed elements, and the position where claims stopped,
//    published by the operation that took the bucket's last unread
//    element).  When no unread input is left anywhere in the task, the
//    workgroup writes its partial buffer blocks to positions reserved the
//    same way (w += count): exact sizes leave no cleanup.
// Every element is read once from its input position and written once to
// its final position: 3 D bytes per element and level (histogram read,
// one read and one write), against 4 D for classification followed by the
// block permutation.  Swap reads that do not fit the next tile are kept in
// the workgroup's buffer slot in the workspace until a later tile takes
// them (at most one buffer block per bucket at any time).
#pragma once
#include "ips_kernels.hpp"

namespace ips {

constexpr uint32_t FUSED_CLAIMS = 8;                 // buckets claimed from in parallel
constexpr uint32_t FUSED_CLAIMS_MAX = 64;            // claims per tile at most
constexpr uint32_t FUSED_SEGS = MAX_K + 1 + FUSED_CLAIMS_MAX;
constexpr uint32_t FUSED_DEFER = 0x80000000u;        // segment source: the workgroup's deferral stack

// Elements per thread of a fused tile: larger tiles than classification's
// (one reservation atomic per bucket and tile, fewer barriers per element),
// as far as the registers of four waves per SIMD allow.
template <class T> struct FusedEpt { static constexpr int value = T::DW == 1 ? 14 : (T::DW == 2 ? 10 : 5); };

// Positions of a bucket's reader word: low half the claimed elements whose
// reads have finished, high half 1 + the position where claims stopped (0
// while unread input is left).
__device__ __forceinline__ bool fused_reads_done(uint64_t v, uint32_t end) {
  const uint32_t x1 = (uint32_t)(v >> 32), done = (uint32_t)v;
  return x1 != 0 && done == end - (x1 - 1);
}

// Digit histogram of each stripe, added to the task's counters.  Per-wave
// sub-histograms keep contention of skewed digits inside a wavefront.
template <class T>
__global__ void __launch_bounds__(CLS_THREADS) k_fhist(BatchArgs a) {
  constexpr int DW = T::DW;
  constexpr int EPT = T::EPT;
  constexpr uint32_t NT = CLS_THREADS, NWV = NT / 64;
  __shared__ uint32_t s_h[NWV][MAX_K];
  const uint32_t wg = blockIdx.x, tid = threadIdx.x;
  if (a.devplan && wg >= a.ctrl[CTRL_NWG]) return;
  const uint32_t tix = a.cls_task[wg];
  const PTask& tk = a.tasks[tix];
  const uint32_t s = wg - tk.wg_base, W = tk.W, nb = tk.nb;
  for (uint32_t i = tid; i < NWV * MAX_K; i += NT) (&s_h[0][0])[i] = 0;
  __syncthreads();
  const uint64_t lo = tk.n * s / W, hi = tk.n * (s + 1) / W;
  const uint32_t len = (uint32_t)(hi - lo);
  const uint32_t* g = a.data + (tk.l + lo) * DW;
  const uint32_t shift = uniform_amount(tk.shift), rmask = low_mask32(tk.width);
  uint32_t* h = s_h[tid >> 6];
  for (uint32_t base = 0; base < len; base += NT * EPT) {
    uint32_t v[EPT][DW];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t m = base + (uint32_t)i * NT + tid;
      if (m < len) ld_elem<DW>(g + (uint64_t)m * DW, v[i]);
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t m = base + (uint32_t)i * NT + tid;
      if (m < len) atomicAdd(&h[(uint32_t)(T::rkey(key_of<T>(v[i])) >> shift) & rmask], 1u);
    }
  }
  __syncthreads();
  for (uint32_t j = tid; j < nb; j += NT) {
    uint32_t c = 0;
#pragma unroll
    for (uint32_t w = 0; w < NWV; ++w) c += s_h[w][j];
    if (c) atomicAdd(&a.b_count[tk.bucket_base + j], c);
  }
}

#ifdef IPS_COMMON_KERNELS
// Bucket starts of every task from its counters (which it zeroes for the
// next step), the pointer and reader words, and the key-range accumulators.
__global__ void __launch_bounds__(MAX_K) k_fscan(BatchArgs a, uint32_t ntask) {
  __shared__ uint32_t s_w[MAX_K / 64];
  const uint32_t ti = blockIdx.x, j = threadIdx.x;
  if (ti >= (a.devplan ? a.ctrl[CTRL_T] : ntask)) return;
  const PTask& tk = a.tasks[ti];
  const uint32_t nb = tk.nb, bb = tk.bucket_base;
  const uint32_t c = j < nb ? a.b_count[bb + j] : 0u;
  if (j < nb) a.b_count[bb + j] = 0;
  // exclusive prefix sum over the (at most 256) buckets
  const uint32_t lane = j & 63, wv = j >> 6;
  uint32_t inc = c;
#pragma unroll
  for (uint32_t off = 1; off < 64; off <<= 1) {
    const uint32_t t = (uint32_t)__shfl_up((int)inc, off);
    if (lane >= off) inc += t;
  }
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  uint32_t before = 0;
  for (uint32_t w = 0; w < wv; ++w) before += s_w[w];
  const uint32_t st = before + inc - c;
  if (j < nb) {
    a.b_start[bb + j] = st;
    uint64_t* pw = a.p_word + (uint64_t)(tk.piece_base + j) * PWORD_STRIDE;
    pw[0] = ((uint64_t)st << 32) | (uint64_t)(st + c + PTR_BIAS);
    pw[1] = 0;
    a.b_min[bb + j] = ~0ull;
    a.b_max[bb + j] = 0;
    if (j == nb - 1) {
      a.b_start[bb + nb] = st + c;
      if ((uint64_t)st + c != tk.n) dev_error(a.ctrl, DE_CLEANUP_COUNT, ti, st + c);
    }
  }
}
#endif  // IPS_COMMON_KERNELS

// At least four wavefronts per SIMD (the second bound): two workgroups per CU.
template <class T>
__global__ void __launch_bounds__(FUSED_THREADS, 4) k_fused(BatchArgs a) {
  constexpr int DW = T::DW;
  constexpr int EPT = FusedEpt<T>::value;   // elements per thread and tile
  constexpr uint32_t NT = FUSED_THREADS;
  constexpr uint32_t TILE = NT * EPT;
  __shared__ uint32_t s_cnt[MAX_K];       // elements of bucket j taken so far
  __shared__ uint2 s_fn[MAX_K];           // {blocks complete before the tile, after it}
  __shared__ uint32_t s_res[MAX_K];       // first position reserved for the tile's complete blocks
  __shared__ uint32_t s_end[MAX_K];       // end of bucket j (task-relative)
  __shared__ uint64_t s_mn[MAX_K], s_mx[MAX_K];
  __shared__ uint16_t s_cj[MAX_K];        // buckets whose LDS buffer block completes in the tile
  __shared__ uint32_t s_cpos[MAX_K];      // and the position it goes to
  __shared__ uint16_t s_wait[MAX_K];      // buckets whose reserved positions include claimed ones
  __shared__ uint32_t s_segend[FUSED_SEGS];   // inclusive end (material index) of segment q
  __shared__ uint32_t s_segsrc[FUSED_SEGS];   // its source (task-relative position, or FUSED_DEFER | stack index)
  __shared__ uint64_t s_segctr;           // (segments << 32) | elements appended by the reservation pass
  __shared__ uint32_t s_ncopy, s_nwait, s_nseg, s_M, s_push, s_pushbase, s_dtop, s_cursor, s_ncl;
  __shared__ uint16_t s_clj[FUSED_CLAIMS_MAX];
  __shared__ uint32_t s_cll[FUSED_CLAIMS_MAX];
  extern __shared__ __align__(16) uint32_t s_buf[];

  const uint32_t tid = threadIdx.x, wg = blockIdx.x;
  if (a.devplan && wg >= a.ctrl[CTRL_NWG]) return;
  const uint32_t tix = a.cls_task[wg];
  const PTask& tk = a.tasks[tix];
  const uint32_t b = tk.b, nb = tk.nb, W = tk.W;
  const uint32_t s = wg - tk.wg_base;
  const BlockDiv bd(b);
  const uint32_t shift = uniform_amount(tk.shift), rmask = low_mask32(tk.width);
  uint32_t* gd = a.data + tk.l * DW;
  uint64_t* word = a.p_word + (uint64_t)tk.piece_base * PWORD_STRIDE;
  uint32_t* defer = reinterpret_cast<uint32_t*>(a.slots + tk.slot_off + (uint64_t)s * tk.slot_bytes);
  const uint32_t dcap = tk.slot_bytes / (DW * 4);
  const uint32_t bdw = b * DW, bstride = bdw + BUF_PAD_DW;
  uint32_t* buf = s_buf;
  for (uint32_t j = tid; j < nb; j += NT) {
    s_cnt[j] = 0;
    s_fn[j] = make_uint2(0, 0);
    s_end[j] = (uint32_t)a.b_start[tk.bucket_base + j + 1];
    s_mn[j] = ~0ull;
    s_mx[j] = 0;
  }
  if (tid == 0) {
    s_dtop = 0;
    s_cursor = 0;
    s_M = 0;
  }
  __syncthreads();
  const uint32_t cstart = (uint32_t)(((uint64_t)s * nb) / (W ? W : 1));   // first bucket this workgroup claims from

  uint32_t cur[EPT][DW], nxt[EPT][DW];
  uint32_t M = 0;   // elements in cur (a prefix of the material index space)
#ifdef IPS_FUSED_STATS
  // phase cycles seen by thread 0: classify, reserve, serial, load, waits, store; tiles, claims
  uint64_t fst[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  uint64_t ft = __builtin_readcyclecounter();
#define FSTAT(i)                                           \
  do {                                                     \
    if (tid == 0) {                                        \
      const uint64_t t1_ = __builtin_readcyclecounter();   \
      fst[i] += t1_ - ft;                                  \
      ft = t1_;                                            \
    }                                                      \
  } while (0)
#else
#define FSTAT(i) ((void)0)
#endif
  for (;;) {
    // 1. Classify the tile and take buffer positions.
    uint32_t bk[EPT], sl[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t m = (uint32_t)i * NT + tid;
      bk[i] = 0;
      sl[i] = 0;
      if (m < M) {
        const uint64_t rk = T::rkey(key_of<T>(cur[i]));
        bk[i] = (uint32_t)(rk >> shift) & rmask;
        sl[i] = atomicAdd(&s_cnt[bk[i]], 1u);
        atomicMin((unsigned long long*)&s_mn[bk[i]], (unsigned long long)rk);
        atomicMax((unsigned long long*)&s_mx[bk[i]], (unsigned long long)rk);
      }
    }
    if (tid == 0) { s_segctr = 0; s_ncopy = 0; s_nwait = 0; }
    __syncthreads();
    FSTAT(0);
    // 2. Reservations: per bucket one atomic for the blocks the tile
    // completes; the unread input in them becomes material segments.
    if ((tid & ~63u) < nb) {
      const uint32_t lane = tid & 63;
      const bool valid = tid < nb;
      const uint32_t fo = valid ? s_fn[tid].y : 0u;
      const uint32_t nf = valid ? bd.div(s_cnt[tid]) : 0u;
      const uint32_t d = nf - fo, len = d * b;
      uint32_t pos = 0, u = 0;
      bool hole = false;
      if (d) {
        const uint64_t old = at_add64(&word[tid * PWORD_STRIDE], (uint64_t)len << 32);
        pos = (uint32_t)(old >> 32);
        const int32_t r = (int32_t)((uint32_t)old - PTR_BIAS);
        if ((int32_t)pos < r) {
          u = (uint32_t)r - pos < len ? (uint32_t)r - pos : len;
          if ((uint32_t)r - pos <= len)   // this reservation took the bucket's last unread element
            (void)at_add64(&word[tid * PWORD_STRIDE + 1], (uint64_t)((uint32_t)r + 1) << 32);
        }
        hole = u < len;
        if ((uint64_t)pos + len > s_end[tid]) dev_error(a.ctrl, DE_PERM_RANGE, tix, pos);
      }
      // append the wave's segments (unread parts) in one LDS atomic
      uint32_t inc = u, incs = u ? 1u : 0u;
#pragma unroll
      for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t t0 = (uint32_t)__shfl_up((int)inc, off);
        const uint32_t t1 = (uint32_t)__shfl_up((int)incs, off);
        if (lane >= off) { inc += t0; incs += t1; }
      }
      uint64_t base = 0;
      if (lane == 63 && (inc || incs)) base = atomicAdd((unsigned long long*)&s_segctr, ((uint64_t)incs << 32) | inc);
      base = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(base >> 32), 63) << 32) |
             (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)base, 63);
      if (u) {
        const uint32_t q = (uint32_t)(base >> 32) + incs - 1;
        s_segend[q] = (uint32_t)base + inc;
        s_segsrc[q] = pos;
      }
      if (valid) {
        s_fn[tid] = make_uint2(fo, nf);
        s_res[tid] = pos;
        if (d && (uint64_t)pos + len <= s_end[tid]) {
          const uint32_t c = atomicAdd(&s_ncopy, 1u);
          s_cj[c] = (uint16_t)tid;
          s_cpos[c] = pos;
        }
        if (hole) s_wait[atomicAdd(&s_nwait, 1u)] = (uint16_t)tid;
      }
    }
    __syncthreads();
    FSTAT(1);
    // 3. The next tile: swap reads first; beyond a tile they go to the
    // deferral stack; a short tile takes deferred elements, then claims
    // (wavefront 0: rounds of claims from up to FUSED_CLAIMS buckets at
    // once, until the tile is full or every bucket's unread input is gone).
    if (tid < 64) {
      const uint32_t lane = tid;
      const uint64_t sc = s_segctr;
      uint32_t nseg = (uint32_t)(sc >> 32), Mn = (uint32_t)sc, push = 0, ncl = 0;
      uint32_t dtop = s_dtop;
      const uint32_t pushbase = dtop;
      if (Mn > TILE) {
        push = Mn - TILE;
        if (dtop + push > dcap) {   // cannot happen (at most one buffer block per bucket is deferred)
          if (lane == 0) dev_error(a.ctrl, DE_PIECES, tix, dtop + push);
          push = 0;
        }
        dtop += push;
        Mn = TILE;
      } else {
        if (dtop && Mn < TILE) {
          const uint32_t pop = dtop < TILE - Mn ? dtop : TILE - Mn;
          dtop -= pop;
          Mn += pop;
          if (lane == 0) {
            s_segend[nseg] = Mn;
            s_segsrc[nseg] = FUSED_DEFER | dtop;
          }
          ++nseg;
        }
        uint32_t cursor = s_cursor;
        while (Mn < TILE && cursor < nb && ncl + FUSED_CLAIMS <= FUSED_CLAIMS_MAX) {
          const uint32_t need = TILE - Mn;
          const uint32_t nl = nb - cursor < FUSED_CLAIMS ? nb - cursor : FUSED_CLAIMS;
          const uint32_t share = lane < nl ? need / nl + (lane < need % nl ? 1u : 0u) : 0u;
          uint32_t got = 0, src = 0, j = 0;
          bool ex = false;
          if (lane < nl) {
            j = cstart + cursor + lane;
            if (j >= nb) j -= nb;
            uint64_t* pw = &word[j * PWORD_STRIDE];
            if (at_load64(pw + 1) >> 32) {
              ex = true;                         // no unread input left
            } else if (share) {
              const uint64_t old = at_add64(pw, 0ull - (uint64_t)share);
              const uint32_t w = (uint32_t)(old >> 32);
              const int32_t r = (int32_t)((uint32_t)old - PTR_BIAS);
              if (r > (int32_t)w) {
                const uint32_t avail = (uint32_t)r - w;
                got = avail < share ? avail : share;
                src = (uint32_t)r - got;
                if (avail <= share) {            // the claim took the last unread element: claims stop at w
                  (void)at_add64(pw + 1, (uint64_t)(w + 1) << 32);
                  ex = true;
                }
              } else {
                ex = true;
              }
            }
          }
          // lane-ordered segments of this round
          uint32_t inc = got, incs = got ? 1u : 0u;
#pragma unroll
          for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint32_t t0 = (uint32_t)__shfl_up((int)inc, off);
            const uint32_t t1 = (uint32_t)__shfl_up((int)incs, off);
            if (lane >= off) { inc += t0; incs += t1; }
          }
          if (got) {
            s_segend[nseg + incs - 1] = Mn + inc;
            s_segsrc[nseg + incs - 1] = src;
            s_clj[ncl + incs - 1] = (uint16_t)j;
            s_cll[ncl + incs - 1] = got;
          }
          const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
          const uint32_t cnt = (uint32_t)__builtin_amdgcn_readlane((int)incs, 63);
          Mn += tot;
          nseg += cnt;
          ncl += cnt;
          // the cursor moves past the leading buckets found without unread input
          const uint64_t exm = __ballot(ex) | ~low_mask64(nl);
          cursor += exm == ~0ull ? nl : (uint32_t)__builtin_ctzll(~exm);
        }
        if (lane == 0) s_cursor = cursor;
      }
      if (lane == 0) {
        s_dtop = dtop;
        s_pushbase = pushbase;
        s_nseg = nseg;
        s_M = Mn;
        s_push = push;
        s_ncl = ncl;
#ifdef IPS_FUSED_STATS
        fst[6] += 1;
        fst[7] += ncl;
#endif
      }
    }
    __syncthreads();
    FSTAT(2);
    const uint32_t Mn = s_M, nseg = s_nseg, push = s_push;
    auto src_of = [&](uint32_t m) -> const uint32_t* {
      uint32_t lo = 0, hi = nseg;   // first segment whose end exceeds m
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_segend[mid] > m) hi = mid; else lo = mid + 1;
      }
      const uint32_t off = m - (lo ? s_segend[lo - 1] : 0u);
      const uint32_t sr = s_segsrc[lo];
      return (sr & FUSED_DEFER) ? defer + (uint64_t)((sr & ~FUSED_DEFER) + off) * DW
                                : gd + (uint64_t)(sr + off) * DW;
    };
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t m = (uint32_t)i * NT + tid;
      if (m < Mn) ld_elem<DW>(src_of(m), nxt[i]);
    }
    if (push) {
      const uint32_t pb = s_pushbase;
      for (uint32_t m = tid; m < push; m += NT) {
        uint32_t v[DW];
        ld_elem<DW>(src_of(TILE + m), v);
        st_elem<DW>(defer + (uint64_t)(pb + m) * DW, v);
      }
    }
    // Every read of the reserved positions has returned before any of them
    // is written.
    __builtin_amdgcn_s_waitcnt(WAITCNT_VM0);
    __syncthreads();
    FSTAT(3);
    // 4. Claimed reads finished; then wait until every claimed read of the
    // buckets whose reserved positions were claimed earlier has finished.
    if (tid < s_ncl) (void)at_add64(&word[s_clj[tid] * PWORD_STRIDE + 1], (uint64_t)s_cll[tid]);
    __syncthreads();
    for (uint32_t q = tid; q < s_nwait; q += NT) {
      const uint32_t j = s_wait[q];
      uint32_t spin = 0;
      while (!fused_reads_done(at_load64(&word[j * PWORD_STRIDE + 1]), s_end[j])) {
        __builtin_amdgcn_s_sleep(2);
        if (++spin > (1u << 22)) { dev_error(a.ctrl, DE_WAIT, tix, j); break; }
      }
    }
    __syncthreads();
    FSTAT(4);
    // 5. Writes, as in classification: elements of the buffer block that
    // completes go to the LDS buffer, whole blocks of the tile straight to
    // their reserved positions, then the completed buffer blocks are
    // copied, then elements past them start the next buffer blocks.
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t m = (uint32_t)i * NT + tid;
      if (m < M) {
        const uint2 st = s_fn[bk[i]];
        const uint32_t blk = bd.div(sl[i]), o = sl[i] - blk * b;
        if (blk == st.x) {
          st_elem<DW>(buf + bk[i] * bstride + o * DW, cur[i]);
        } else if (blk < st.y) {
          const uint64_t pos = (uint64_t)s_res[bk[i]] + (uint64_t)(blk - st.x) * b + o;
          if (pos < s_end[bk[i]]) st_elem<DW>(gd + pos * DW, cur[i]);
        }
      }
    }
    __syncthreads();
    {
      const uint32_t ncp = s_ncopy, wave = tid >> 6, lane = tid & 63;
      for (uint32_t q = wave; q < ncp; q += NT / 64) {
        const uint32_t* src = buf + s_cj[q] * bstride;
        uint32_t* dst = gd + (uint64_t)s_cpos[q] * DW;
        if constexpr (DW % 2 == 0) {   // 8-byte units (elements of even dwords are 8-byte aligned)
          for (uint32_t x = lane; x < bdw / 2; x += 64)
            *reinterpret_cast<uint2*>(dst + 2 * x) = *reinterpret_cast<const uint2*>(src + 2 * x);
        } else {
          for (uint32_t x = lane; x < bdw; x += 64) dst[x] = src[x];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t m = (uint32_t)i * NT + tid;
      if (m < M) {
        const uint2 st = s_fn[bk[i]];
        const uint32_t blk = bd.div(sl[i]), o = sl[i] - blk * b;
        if (blk == st.y && blk > st.x) st_elem<DW>(buf + bk[i] * bstride + o * DW, cur[i]);
      }
    }
    // the next tile
#pragma unroll
    for (int i = 0; i < EPT; ++i)
#pragma unroll
      for (int d = 0; d < DW; ++d) cur[i][d] = nxt[i][d];
    M = Mn;
    __syncthreads();
    FSTAT(5);
    if (M == 0) break;   // no unread input left in the task and nothing deferred
  }
#ifdef IPS_FUSED_STATS
  if (tid == 0) {
    // root step at control words 32..47, deeper steps at 48..63
    unsigned long long* c = reinterpret_cast<unsigned long long*>(a.ctrl + (tk.level ? 48 : 32));
    for (int i = 0; i < 8; ++i) atomicAdd(&c[i], (unsigned long long)fst[i]);
  }
#endif
#undef FSTAT
  // Partial buffer blocks: no unread input is left, so the reserved
  // positions were all claimed; they are written once those reads are done.
  const uint32_t wave = tid >> 6, lane = tid & 63;
  for (uint32_t j = wave; j < nb; j += NT / 64) {
    const uint32_t left = s_cnt[j] - s_fn[j].y * b;
    if (!left) continue;
    uint32_t pos = 0;
    if (lane == 0) {
      pos = (uint32_t)(at_add64(&word[j * PWORD_STRIDE], (uint64_t)left << 32) >> 32);
      if ((uint64_t)pos + left > s_end[j]) {
        dev_error(a.ctrl, DE_CLEANUP_COUNT, tix, pos);
        pos = 0xFFFFFFFFu;
      } else {
        uint32_t spin = 0;
        while (!fused_reads_done(at_load64(&word[j * PWORD_STRIDE + 1]), s_end[j])) {
          __builtin_amdgcn_s_sleep(2);
          if (++spin > (1u << 22)) { dev_error(a.ctrl, DE_WAIT, tix, j); break; }
        }
      }
    }
    pos = (uint32_t)__builtin_amdgcn_readfirstlane((int)pos);
    if (pos == 0xFFFFFFFFu) continue;
    const uint32_t* src = buf + j * bstride;
    uint32_t* dst = gd + (uint64_t)pos * DW;
    for (uint32_t x = lane; x < left * DW; x += 64) dst[x] = src[x];
  }
  for (uint32_t j = tid; j < nb; j += NT) {
    if (s_cnt[j]) {
      atomicMin((unsigned long long*)&a.b_min[tk.bucket_base + j], (unsigned long long)s_mn[j]);
      atomicMax((unsigned long long*)&a.b_max[tk.bucket_base + j], (unsigned long long)s_mx[j]);
    }
  }
}

}  // namespace ips
