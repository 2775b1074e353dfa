/* Test infrastructure only (see oracle.h).  Plain single-threaded C.
 *
 * Paper references are to arXiv 2009.13569: "Definitions and
 * Preliminaries" (problem statement, super scalar samplesort, branchless
 * decision tree with equality buckets, Algorithm 1), Section 4.1 (partitioning step, "Sampling"),
 * Section 4.2 "Task Scheduling" (adaptive k), Section 6 "Implementation
 * Details" (parameters, IPS2Ra) and Section 7 (data types, comparators
 * Algorithms 3-4).
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

size_t oracle_elem_bytes(int type) {
  switch (type) {
    case 1: return 4;
    case 2: return 8;
    case 3: return 8;
    case 4: return 16;
    case 5: return 100;
    case 6: return 32;
    default: return 0;
  }
}

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): state advances by the golden
 * gamma, output is the variant-13 style mix of the new state. */
uint64_t oracle_splitmix64_next(uint64_t* state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t oracle_mulhi64(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

static uint64_t rd64(const void* p) { uint64_t v; memcpy(&v, p, 8); return v; }
static uint32_t rd32(const void* p) { uint32_t v; memcpy(&v, p, 4); return v; }

/* IEEE 754 totalOrder on binary64, written from its definition: negative
 * numbers (sign bit set) precede positive ones; among positives a larger
 * encoding is a larger value; among negatives a larger encoding is a smaller
 * value.  -0 precedes +0. */
static int f64_total_less(uint64_t a, uint64_t b) {
  int sa = (int)(a >> 63), sb = (int)(b >> 63);
  if (sa != sb) return sa > sb;
  if (!sa) return a < b;
  return a > b;
}

/* Strict key order of the element types.  Pair compares only its key
 * (value is payload, Section 7); rec100 compares the first ten bytes
 * lexicographically as unsigned bytes (Algorithm 4 read with unsigned
 * char, the memcmp order); Quartet compares its three 64-bit key words
 * a, b, c (bytes 0, 8, 16) lexicographically, the fourth word being
 * payload (Algorithm 3). */
int oracle_key_less(int type, const void* a, const void* b) {
  switch (type) {
    case 1: return rd32(a) < rd32(b);
    case 2: return rd64(a) < rd64(b);
    case 3: return f64_total_less(rd64(a), rd64(b));
    case 4: return rd64(a) < rd64(b);
    case 5: {
      const unsigned char* x = (const unsigned char*)a;
      const unsigned char* y = (const unsigned char*)b;
      for (int i = 0; i < 10; ++i)
        if (x[i] != y[i]) return x[i] < y[i];
      return 0;
    }
    case 6: {
      const unsigned char* x = (const unsigned char*)a;
      const unsigned char* y = (const unsigned char*)b;
      for (int w = 0; w < 3; ++w) {
        const uint64_t u = rd64(x + 8 * w), v = rd64(y + 8 * w);
        if (u != v) return u < v;
      }
      return 0;
    }
    default: return 0;
  }
}

static int key_equal(int type, const void* a, const void* b) {
  return !oracle_key_less(type, a, b) && !oracle_key_less(type, b, a);
}

/* Plain sort: insertion sort on runs of 16, then bottom-up stable merging
 * with one n-element temporary.  The result is the input rearranged so that
 * keys are non-decreasing (problem statement, Section 2). */
int oracle_sort(void* data, uint64_t n, int type) {
  size_t D = oracle_elem_bytes(type);
  if (!D) return -1;
  if (n < 2) return 0;
  unsigned char* a = (unsigned char*)data;
  unsigned char* tmp = (unsigned char*)malloc((size_t)n * D);
  unsigned char* e = (unsigned char*)malloc(D);
  if (!tmp || !e) { free(tmp); free(e); return -2; }
  const uint64_t RUN = 16;
  for (uint64_t s = 0; s < n; s += RUN) {
    uint64_t t = s + RUN < n ? s + RUN : n;
    for (uint64_t i = s + 1; i < t; ++i) {
      memcpy(e, a + i * D, D);
      uint64_t j = i;
      while (j > s && oracle_key_less(type, e, a + (j - 1) * D)) {
        memcpy(a + j * D, a + (j - 1) * D, D);
        --j;
      }
      memcpy(a + j * D, e, D);
    }
  }
  unsigned char* src = a;
  unsigned char* dst = tmp;
  for (uint64_t w = RUN; w < n; w *= 2) {
    for (uint64_t lo = 0; lo < n; lo += 2 * w) {
      uint64_t mid = lo + w < n ? lo + w : n;
      uint64_t hi = lo + 2 * w < n ? lo + 2 * w : n;
      uint64_t i = lo, j = mid, o = lo;
      while (i < mid && j < hi) {
        if (oracle_key_less(type, src + j * D, src + i * D)) {
          memcpy(dst + o * D, src + j * D, D); ++j;
        } else {
          memcpy(dst + o * D, src + i * D, D); ++i;
        }
        ++o;
      }
      if (i < mid) memcpy(dst + o * D, src + i * D, (size_t)(mid - i) * D), o += mid - i;
      if (j < hi) memcpy(dst + o * D, src + j * D, (size_t)(hi - j) * D);
    }
    unsigned char* t = src; src = dst; dst = t;
  }
  if (src != a) memcpy(a, src, (size_t)n * D);
  free(tmp);
  free(e);
  return 0;
}

static uint32_t floor_log2_u64(uint64_t x) {
  uint32_t r = 0;
  while (x >>= 1) ++r;
  return r;
}

/* Oversampling factor alpha = 0.2 log2 n (Section 6), floored and at least
 * one.  floor(log2(n)/5) equals floor(floor(log2 n)/5), so the integer form
 * is exact. */
uint32_t oracle_alpha(uint64_t n) {
  uint32_t a = floor_log2_u64(n ? n : 1) / 5;
  return a ? a : 1;
}

/* Adaptive number of buckets (Section 4.2): for k n0 < n < k^2 n0 use
 * 2^ceil((log2(n/n0)+1)/2); for n0 < n <= k n0 use 2^ceil(log2(n/n0));
 * otherwise k.  Evaluated exactly with integers: the smallest c with
 * n0 * 2^(2c-1) >= n, resp. n0 * 2^c >= n.  Clamped to [2, k]. */
uint32_t oracle_adaptive_k(uint64_t n, uint32_t k, uint32_t n0) {
  unsigned __int128 kn0 = (unsigned __int128)k * n0;
  unsigned __int128 kkn0 = kn0 * k;
  uint32_t c = 0;
  uint64_t r = k;
  if ((unsigned __int128)n > kn0 && (unsigned __int128)n < kkn0) {
    c = 0;
    while (((unsigned __int128)n0 << (2 * c > 0 ? 2 * c - 1 : 0)) < n || 2 * c < 1) ++c;
    r = 1ull << c;
  } else if (n > n0 && (unsigned __int128)n <= kn0) {
    c = 0;
    while (((unsigned __int128)n0 << c) < n) ++c;
    r = 1ull << c;
  }
  if (r > k) r = k;
  if (r < 2) r = 2;
  return (uint32_t)r;
}

/* Seed of the sampling stream of the task starting at element l on
 * recursion level `level`: the first SplitMix64 output for state
 * seed ^ (l * gamma) ^ (level << 56). */
uint64_t oracle_task_seed(uint64_t seed, uint64_t l, uint32_t level) {
  uint64_t st = seed ^ (l * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)level << 56);
  return oracle_splitmix64_next(&st);
}

/* Sampling phase of one partitioning step (Section 4.1) on the task
 * data[l, l+n):
 *   alpha = oracle_alpha(n), k' = oracle_adaptive_k(n, k, n0), m = alpha k';
 *   sample j (0 <= j < m) is the element at l + floor(n * x_j / 2^64) where
 *   x_j is output j of SplitMix64 seeded with oracle_task_seed (sampling
 *   with replacement; samples are copied, not swapped);
 *   the sample is sorted and k'-1 splitters are taken equidistantly, the
 *   i-th at sorted position (i+1) alpha - 1;
 *   duplicate splitters are removed (u distinct remain), equality buckets
 *   are enabled iff a duplicate was removed (eq_mode: -1 auto, 0 off, 1 on);
 *   the splitter array is padded with the largest splitter to K-1 entries,
 *   K = the smallest power of two >= u+1, and entry K-1 duplicates K-2
 *   (Definitions and Preliminaries).
 * info[0..6] = {alpha, k', m, u, K, eq, number of buckets}.  splitters_out
 * receives K elements; sample_out (optional) the m sorted samples. */
int oracle_sample_step(const void* data, uint64_t l, uint64_t n, int type,
                       uint32_t k, uint32_t n0, uint64_t seed, uint32_t level,
                       int eq_mode, uint32_t* info, void* splitters_out,
                       void* sample_out) {
  size_t D = oracle_elem_bytes(type);
  if (!D || n == 0 || k < 2) return -1;
  const unsigned char* a = (const unsigned char*)data;
  uint32_t alpha = oracle_alpha(n);
  uint32_t kp = oracle_adaptive_k(n, k, n0);
  uint32_t m = alpha * kp;
  unsigned char* smp = (unsigned char*)malloc((size_t)m * D);
  unsigned char* spl = (unsigned char*)malloc((size_t)kp * D);
  if (!smp || !spl) { free(smp); free(spl); return -2; }
  uint64_t st = oracle_task_seed(seed, l, level);
  for (uint32_t j = 0; j < m; ++j) {
    uint64_t x = oracle_splitmix64_next(&st);
    uint64_t pos = l + oracle_mulhi64(x, n);
    memcpy(smp + (size_t)j * D, a + pos * D, D);
  }
  oracle_sort(smp, m, type);
  if (sample_out) memcpy(sample_out, smp, (size_t)m * D);
  uint32_t u = 0;
  for (uint32_t i = 0; i + 1 < kp; ++i) {
    const unsigned char* s = smp + ((size_t)(i + 1) * alpha - 1) * D;
    if (u > 0 && key_equal(type, s, spl + (size_t)(u - 1) * D)) continue;
    memcpy(spl + (size_t)u * D, s, D);
    ++u;
  }
  int eq = (u < kp - 1);
  if (eq_mode == 0) eq = 0;
  if (eq_mode == 1) eq = 1;
  uint32_t K = 1;
  while (K < u + 1) K *= 2;
  unsigned char* out = (unsigned char*)splitters_out;
  for (uint32_t i = 0; i < K; ++i) {
    uint32_t src = i < u ? i : u - 1;
    memcpy(out + (size_t)i * D, spl + (size_t)src * D, D);
  }
  info[0] = alpha; info[1] = kp; info[2] = m; info[3] = u; info[4] = K;
  info[5] = (uint32_t)eq; info[6] = eq ? 2 * K : K;
  free(smp);
  free(spl);
  return 0;
}

/* Bucket of element e (Definitions and Preliminaries): i is the number of
 * splitters s_0..s_{K-2} strictly smaller than e, so s_{i-1} < e <= s_i.
 * Without equality buckets the bucket is i.  With them, an element equal to
 * s_i (i < K-1) goes to bucket 2i+1, any other to 2i, and e above every
 * splitter (i = K-1) to 2K-1 because s_{K-1} is taken equal to s_{K-2}. */
uint32_t oracle_classify(int type, const void* e, const void* splitters,
                         uint32_t K, int eq) {
  size_t D = oracle_elem_bytes(type);
  const unsigned char* s = (const unsigned char*)splitters;
  uint32_t i = 0;
  for (uint32_t j = 0; j + 1 < K; ++j)
    if (oracle_key_less(type, s + (size_t)j * D, e)) ++i;
  if (!eq) return i;
  if (i == K - 1) return 2 * K - 1;
  return key_equal(type, e, s + (size_t)i * D) ? 2 * i + 1 : 2 * i;
}

int oracle_histogram(const void* data, uint64_t n, int type,
                     const void* splitters, uint32_t K, int eq,
                     uint64_t* counts) {
  size_t D = oracle_elem_bytes(type);
  if (!D) return -1;
  uint32_t nb = eq ? 2 * K : K;
  memset(counts, 0, sizeof(uint64_t) * nb);
  const unsigned char* a = (const unsigned char*)data;
  for (uint64_t i = 0; i < n; ++i)
    counts[oracle_classify(type, a + i * D, splitters, K, eq)]++;
  return 0;
}

/* Unsigned integer key used by the radix variant (Section 6: IPS2Ra takes
 * unsigned integer keys).  Doubles use the order-preserving bit map of
 * totalOrder: flip all bits of negatives, set the sign bit of positives. */
static uint64_t radix_key(int type, const void* e) {
  switch (type) {
    case 1: return rd32(e);
    case 2: return rd64(e);
    case 3: { uint64_t b = rd64(e); return (b >> 63) ? ~b : (b | (1ull << 63)); }
    case 4: return rd64(e);
    default: return 0;
  }
}

/* Digit of the radix variant on one task: the task's minimum and maximum
 * key are scanned, h is the highest bit in which they differ (significant
 * bit detection, Section 7.2), and the digit is bits [max(0,h-7), h].
 * info = {shift, width, all_equal}. */
int oracle_radix_digit_info(const void* data, uint64_t n, int type,
                            uint32_t* info) {
  size_t D = oracle_elem_bytes(type);
  if (!D || type == 5 || n == 0) return -1;
  const unsigned char* a = (const unsigned char*)data;
  uint64_t mn = radix_key(type, a), mx = mn;
  for (uint64_t i = 1; i < n; ++i) {
    uint64_t k = radix_key(type, a + i * D);
    if (k < mn) mn = k;
    if (k > mx) mx = k;
  }
  if (mn == mx) { info[0] = 0; info[1] = 0; info[2] = 1; return 0; }
  uint32_t h = floor_log2_u64(mn ^ mx);
  uint32_t shift = h >= 7 ? h - 7 : 0;
  info[0] = shift;
  info[1] = h - shift + 1;
  info[2] = 0;
  return 0;
}

int oracle_radix_histogram(const void* data, uint64_t n, int type,
                           uint32_t shift, uint32_t width, uint64_t* counts) {
  size_t D = oracle_elem_bytes(type);
  if (!D || width == 0 || width > 16) return -1;
  memset(counts, 0, sizeof(uint64_t) << width);
  const unsigned char* a = (const unsigned char*)data;
  uint64_t mask = (1ull << width) - 1;
  for (uint64_t i = 0; i < n; ++i)
    counts[(radix_key(type, a + i * D) >> shift) & mask]++;
  return 0;
}

/* Partition property after a partitioning step: every element of
 * data[bucket_start[j], bucket_start[j+1]) is classified into bucket j.
 * Returns 0 if it holds, 1 otherwise with the first offending index. */
int oracle_check_partition(const void* data, uint64_t n, int type,
                           const void* splitters, uint32_t K, int eq,
                           const uint64_t* bucket_start, uint64_t* bad_index) {
  size_t D = oracle_elem_bytes(type);
  uint32_t nb = eq ? 2 * K : K;
  const unsigned char* a = (const unsigned char*)data;
  if (bucket_start[0] != 0 || bucket_start[nb] != n) { *bad_index = n; return 1; }
  for (uint32_t j = 0; j < nb; ++j) {
    for (uint64_t i = bucket_start[j]; i < bucket_start[j + 1]; ++i) {
      if (oracle_classify(type, a + i * D, splitters, K, eq) != j) {
        *bad_index = i;
        return 1;
      }
    }
  }
  return 0;
}

/* Number of elements with key < v (or <= v): the rank window of v, used to
 * check single output positions of very large sorts one by one. */
uint64_t oracle_count_less(const void* data, uint64_t n, int type, const void* v,
                           int or_equal) {
  size_t D = oracle_elem_bytes(type);
  const unsigned char* a = (const unsigned char*)data;
  uint64_t c = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const unsigned char* e = a + i * D;
    if (oracle_key_less(type, e, v) || (or_equal && !oracle_key_less(type, v, e))) ++c;
  }
  return c;
}
