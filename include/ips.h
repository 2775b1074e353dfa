/* ips.h - C ABI of an MI355X (gfx950) in-place parallel samplesort and
 * radix sort.
 *
 * The operation is the sorting problem stated in Section 2 ("Definitions
 * and Preliminaries") of Axtmann, Witt, Ferizovic, Sanders, "Engineering
 * In-place (Shared-memory) Sorting Algorithms" (arXiv 2009.13569): the n
 * elements of an array are rearranged in that same array so that their
 * keys are non-decreasing.  The method is the paper's recursive in-place
 * partitioning step (Section 4.1: sampling with a branchless decision tree,
 * classification through buffer blocks, block permutation with per-bucket
 * read/write pointers, cleanup; equality buckets for duplicate keys) and,
 * for IPS_RADIX, the radix variant IPS2Ra of Section 6 that replaces the
 * decision tree by an 8-bit digit of unsigned integer keys.
 *
 * Conventions for every entry point:
 *  - Device pointers refer to memory of the device the context was created
 *    on.  The caller owns all of it.  The library never allocates or frees
 *    device memory while sorting; extra memory comes from the caller's
 *    workspace, sized by ips_workspace_bytes.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on it.  The partitioning steps are planned on the
 *    device from a task queue in the workspace; the host enqueues rounds of
 *    steps and synchronizes with the stream between rounds to read the
 *    queue's head and tail (and once after the sorted-input check), so the
 *    sort entry points return only when the data is sorted.  With
 *    IPS_FLAG_HOST_PLAN the host instead plans every batch of a recursion
 *    level from read-back bucket sizes.
 *  - After IPS_E_DEVICE the contents of the array are unspecified (a kernel
 *    stopped part-way through moving blocks); after any other error code
 *    the array is unchanged unless the error came from a HIP call made
 *    after the first kernel launch.
 *  - Return values are IPS_OK (0) or a negative IPS_E_* code; arguments are
 *    validated before any HIP call.  ips_status_string names every code.
 *  - The sort is unstable: records with equal keys may end in any order.
 *  - One context must not be used by two host threads at once.
 */
#ifndef IPS_H
#define IPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IPS_ABI_VERSION 2

/* Status codes. */
#define IPS_OK 0
#define IPS_E_INVALID_ARG (-1)     /* null pointer with n > 0, bad enum, bad params */
#define IPS_E_UNSUPPORTED (-2)     /* e.g. IPS_RADIX on 100-byte records */
#define IPS_E_WORKSPACE (-3)       /* workspace smaller than ips_workspace_bytes */
#define IPS_E_MISALIGNED (-4)      /* data not naturally aligned (4 B for u32 and
                                      100-byte records, 8 B otherwise), or the
                                      workspace not 256-byte aligned */
#define IPS_E_TOO_LARGE (-5)       /* n beyond what the block pointers can index */
#define IPS_E_HIP (-6)             /* a HIP runtime call failed; see ips_last_hip_error */
#define IPS_E_DEVICE (-7)          /* a kernel reported an internal consistency error;
                                      see ips_last_device_error */
#define IPS_E_NO_DEVICE (-8)       /* no usable gfx950 device */
#define IPS_E_SCRATCH (-9)         /* ips_sort_keys_noalloc: the call needs more than
                                      the static scratch (or pinned staging) holds */

/* Element types.  Keys: u32, u64, f64 (ordered by IEEE 754 totalOrder, so
 * -0.0 < +0.0 and NaNs sort to the ends by sign).  Records (Section 7 of the
 * paper): IPS_PAIR_U64_U64 is 16 bytes, a u64 key at byte 0 and a u64 value
 * at byte 8; IPS_REC100 is 100 bytes whose key is bytes 0..9 compared
 * lexicographically as unsigned bytes (memcmp order, Algorithm 4);
 * IPS_QUARTET is 32 bytes, three u64 key words a, b, c at bytes 0, 8, 16
 * compared lexicographically (Algorithm 3) and a u64 value at byte 24. */
typedef enum { IPS_U32 = 1, IPS_U64 = 2, IPS_F64 = 3 } ips_key_type;
typedef enum { IPS_PAIR_U64_U64 = 4, IPS_REC100 = 5, IPS_QUARTET = 6 } ips_rec_type;

/* IPS_SAMPLESORT: IPS4o.  IPS_RADIX: IPS2Ra (unsigned integer keys; the
 * f64 key is mapped to its order-preserving unsigned image; not available
 * for IPS_REC100 and IPS_QUARTET). */
typedef enum { IPS_SAMPLESORT = 0, IPS_RADIX = 1 } ips_algo;

/* Flags of ips_params. */
#define IPS_FLAG_NO_SORTED_CHECK 0x1u  /* skip the sorted / reverse-sorted detection
                                          (Section 6) */
#define IPS_FLAG_EQ_ON 0x2u           /* force equality buckets on every step */
#define IPS_FLAG_EQ_OFF 0x4u          /* no equality buckets on the root step (later
                                          steps still enable them when a step would
                                          otherwise make no progress) */
#define IPS_FLAG_LEVEL1_ONLY 0x8u     /* stop after the root partitioning step: the
                                          array is then partitioned, not sorted; see
                                          ips_get_root_info */
#define IPS_FLAG_PROFILE 0x20u        /* time every kernel launch with HIP events on
                                          `stream`; see ips_get_profile */
#define IPS_FLAG_GRAPH 0x40u          /* capture a round of device-planned steps as a HIP
                                          graph once per call and replay it until the task
                                          queue is empty; `stream` must be a created stream
                                          (not the null stream) that is not capturing;
                                          IPS_FLAG_PROFILE is ignored */
#define IPS_FLAG_HOST_PLAN 0x80u      /* plan every batch on the host from read-back bucket
                                          sizes instead of on the device */
#define IPS_FLAG_GLOBAL_BUFFERS 0x10u /* keep the classification buffer blocks in the
                                          workspace instead of LDS, so that block_bytes
                                          may exceed the LDS budget (e.g. 2 KiB blocks
                                          with 256 buckets) */
#define IPS_FLAG_FUSED 0x100u         /* IPS_RADIX only: run every partitioning step
                                          with exact bucket sizes and classification
                                          fused into the block permutation (Section 8,
                                          future work): a digit histogram pass, then
                                          one pass that reads every element once and
                                          writes it once to its final position.
                                          IPS_E_UNSUPPORTED with IPS_SAMPLESORT,
                                          IPS_FLAG_HOST_PLAN, IPS_FLAG_LEVEL1_ONLY or
                                          IPS_FLAG_GLOBAL_BUFFERS; IPS_E_TOO_LARGE for
                                          n >= 2^31 - 2^16 elements */
#define IPS_FLAG_PAPER_ROOT_ALPHA 0x400u /* the root step samples the paper's
                                          alpha = max(1, floor(0.2 log2 n)) elements per
                                          bucket (Section 6).  By default every step,
                                          the root included, samples at least 16 per
                                          bucket when 16 k' elements fit the 4096-key
                                          sample: more even root buckets, so that no
                                          level-1 bucket exceeds the LDS tier at
                                          2^28 u64 (the sorted result is the same) */
#define IPS_FLAG_INSERTION_BASE 0x200u /* IPS_SAMPLESORT with n0 > 0: the paper's base
                                          case (Section 4.2): a bucket of at most 2 n0
                                          elements, or any bucket of a task of at most
                                          k n0 elements, is sorted by insertion sort
                                          (one thread per bucket) instead of the LDS
                                          tier; larger ones are partitioned again.
                                          The number of tasks grows as n / n0, and the
                                          workspace with it.  IPS_E_INVALID_ARG when
                                          n0 = 0, IPS_E_UNSUPPORTED with IPS_RADIX */

/* Tuning and test parameters.  A zero field selects the default.
 *  k            maximum number of buckets per step (power of two, 2..256;
 *               default 256, Section 6)
 *  block_bytes  requested block size in bytes; the block holds
 *               max(1, block_bytes / element size) elements.  Default: the
 *               largest block for which one buffer block per bucket fits the
 *               LDS budget.  Larger requests need IPS_FLAG_GLOBAL_BUFFERS.
 *  n0           base-case size of the paper's adaptive-k rule (Section 4.2;
 *               the paper uses 16).  0 (default): the number of buckets of a
 *               step is the smallest power of two (at most k) that makes the
 *               mean bucket at most a quarter of the LDS-tier capacity.
 *  lds_task_max tasks with at most this many elements are sorted inside one
 *               workgroup's LDS (default: per type, 1..16384); 1 forces every
 *               task of two or more elements through a partitioning step
 *  piece_blocks maximum blocks per pointer piece of the block permutation
 *               (default 1024)
 *  seed         seed of the sampling stream (default 0)
 *  perm_groups  target number of block-permutation groups (swap buffers) per
 *               batch (default 131072)
 *  perm_wg      workgroup size of the block permutation: 128, 256 or 512
 *               threads (default 256)
 *  k_root       maximum number of buckets of a root step (level 0; power of
 *               two, 2..256; default k): fewer, larger buckets at the root
 *               give larger blocks and fewer pointer operations there when
 *               the next level still fits its buckets in the LDS tier
 *  profile_mask with IPS_FLAG_PROFILE: bit (1 << IPS_PH_x) selects the phases
 *               whose launches are timed (0 = all phases).  Every timed
 *               launch adds two event records to the stream.
 */
typedef struct {
  uint32_t k;
  uint32_t block_bytes;
  uint32_t n0;
  uint32_t lds_task_max;
  uint32_t piece_blocks;
  uint32_t flags;
  uint64_t seed;
  uint32_t perm_groups;
  uint32_t profile_mask;
  uint32_t perm_wg;
  uint32_t k_root;
} ips_params;

typedef struct ips_ctx ips_ctx;

/* Create a context on HIP device `device` (the "sorter object" of
 * Section 7.6: it keeps host-side state and pinned staging buffers between
 * calls; it holds no device memory).  Creation allocates 8 MiB of pinned
 * host staging (grown later by calls that need more, except the
 * allocation-free entry point) and, for the first context on a device,
 * takes that device's address of the static scratch of
 * ips_sort_keys_noalloc (the current device is restored afterwards).
 * Errors: IPS_E_INVALID_ARG for a null `out`, IPS_E_NO_DEVICE, IPS_E_HIP. */
int ips_ctx_create(ips_ctx** out, int device);

/* Destroy a context (NULL is accepted). */
int ips_ctx_destroy(ips_ctx* ctx);

/* Workspace bytes needed to sort n elements of `elem_type` (1..6) with
 * `algo` and `params` (nullable).  Pure host computation, no HIP call.
 * The size is O(k * b * element size) per workgroup of the largest step
 * plus O(k) words per task of that step (Section 5.1), and two terms that
 * grow with n by well under 0.1% of the data (the task queue and the
 * permutation's pointer pieces).  Errors: IPS_E_INVALID_ARG, IPS_E_UNSUPPORTED,
 * IPS_E_TOO_LARGE. */
int ips_workspace_bytes(uint64_t n, int elem_type, int algo,
                        const ips_params* params, size_t* out_bytes);

/* Sort n keys in place at device pointer d_keys.  d_ws: device workspace of
 * ws_bytes >= ips_workspace_bytes(...) bytes, 256-byte aligned; its
 * contents need no initialization and are garbage afterwards.  n in {0, 1}
 * is a successful no-op. */
int ips_sort_keys(ips_ctx* ctx, void* d_keys, uint64_t n, int key_type,
                  int algo, void* d_ws, size_t ws_bytes,
                  const ips_params* params, void* stream);

/* Allocation-free variant of ips_sort_keys, for callers that cannot
 * allocate memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same sort, same kernels and the same
 * arguments except the workspace: the scratch is a static device array of
 * 64 MiB inside the library (one copy per GPU, held until the process ends;
 * its address is taken when the first context on a GPU is created), and
 * the pinned host staging is the buffer the context allocated when it was
 * created.  The call allocates no device or pinned host memory and creates
 * no events or graphs.
 *  - Limit: calls whose workspace (ips_workspace_bytes with the same
 *    arguments) exceeds 64 MiB are rejected with IPS_E_SCRATCH before any
 *    HIP call.  With the default parameters that admits up to 2^23 u64 or
 *    f64 keys and 2^24 u32 keys.
 *  - IPS_FLAG_PROFILE and IPS_FLAG_GRAPH are rejected (IPS_E_INVALID_ARG):
 *    both would create HIP objects.
 *  - Every call on one GPU shares that GPU's scratch, which keeps the last
 *    call's contents (the sort initialises what it needs).  Calls that
 *    overlap in time on one GPU (other threads, other streams, other
 *    contexts) race on it and must be serialized by the caller.
 *  - Like ips_sort_keys, the call synchronizes with `stream` between
 *    rounds of steps and returns when the keys are sorted.
 * Errors: as ips_sort_keys, plus IPS_E_SCRATCH. */
int ips_sort_keys_noalloc(ips_ctx* ctx, void* d_keys, uint64_t n, int key_type, int algo,
                          const ips_params* params, void* stream);

/* Out-of-place ablation: the partitioning step of super scalar samplesort
 * (Sanders and Winkel), which the paper re-implements on its framework
 * (Section 7) and compares with its in-place step by I/O volume (appendix,
 * "Comparing the I/O Volume"), run with the same sampling, decision tree,
 * start table and LDS-tier base case as ips_sort_keys/ips_sort_pairs with
 * IPS_SAMPLESORT.  Each level classifies every element into an oracle
 * array (one byte per element, two when a step has more than 256 buckets),
 * sums the bucket sizes, and distributes the elements into the other of
 * two arrays; a level moves 3 D + 2 o bytes per element instead of 4 D.
 * The sorted result ends in d_data.  It needs a second device buffer d_tmp
 * of tmp_bytes (the element array plus the oracle, 256-byte aligned, owned
 * by the caller, contents garbage afterwards) besides the workspace; both
 * sizes come from ips_oop_workspace_bytes.  elem_type is any of 1..6; no
 * sorted-input detection; IPS_FLAG_LEVEL1_ONLY, IPS_FLAG_GRAPH,
 * IPS_FLAG_HOST_PLAN and IPS_FLAG_GLOBAL_BUFFERS are rejected.  n must be
 * below 2^32.  Errors: as ips_sort_keys; IPS_E_WORKSPACE also for a short
 * d_tmp. */
int ips_oop_workspace_bytes(uint64_t n, int elem_type, const ips_params* params, size_t* ws_bytes,
                            size_t* tmp_bytes);
int ips_sort_oop(ips_ctx* ctx, void* d_data, uint64_t n, int elem_type, void* d_tmp, size_t tmp_bytes,
                 void* d_ws, size_t ws_bytes, const ips_params* params, void* stream);

/* Sort n records in place at device pointer d_recs (array of structures).
 * Records move as whole records; only the key is compared. */
int ips_sort_pairs(ips_ctx* ctx, void* d_recs, uint64_t n, int rec_type,
                   int algo, void* d_ws, size_t ws_bytes,
                   const ips_params* params, void* stream);

/* A segment of a batched call: elements [offset, offset + n) of the data
 * array (element units). */
typedef struct {
  uint64_t offset, n;
} ips_segment;

/* Workspace bytes of ips_sort_segments over a data array of n_total
 * elements with the given segments (host array of nseg entries).  Pure host
 * computation.  Errors: as ips_workspace_bytes, and IPS_E_INVALID_ARG for a
 * segment outside [0, n_total) or two overlapping segments. */
int ips_segments_workspace_bytes(uint64_t n_total, const ips_segment* segs,
                                 uint32_t nseg, int elem_type, int algo,
                                 const ips_params* params, size_t* out_bytes);

/* Sort each of nseg segments of one device array independently, in place,
 * in one call (batched sorting of many arrays; the paper's problem of
 * Section 2 applied to every segment).  d_data holds n_total elements of
 * elem_type (1..6, keys or records); segs is a HOST array of nseg
 * non-overlapping segments (read during the call only); elements outside
 * every segment are left unchanged.  All segments' partitioning steps of one
 * recursion level run in shared launches (Section 4.2 breadth first);
 * segments no larger than the LDS tier are sorted in one launch.  Segments
 * larger than the LDS tier first get the sorted / reverse-sorted detection
 * of Section 6 (one batched scan; unless IPS_FLAG_NO_SORTED_CHECK): sorted
 * ones are left as they are, reverse-sorted ones are reversed in place.
 * IPS_FLAG_LEVEL1_ONLY is rejected.
 * The workspace must hold ips_segments_workspace_bytes(...) bytes.  Errors:
 * as ips_sort_keys, plus IPS_E_INVALID_ARG for bad segments. */
int ips_sort_segments(ips_ctx* ctx, void* d_data, uint64_t n_total,
                      int elem_type, int algo, const ips_segment* segs,
                      uint32_t nseg, void* d_ws, size_t ws_bytes,
                      const ips_params* params, void* stream);

/* Workspace bytes of ips_sort_batch for the given requests (device
 * pointers d_ptrs[i] of ns[i] elements each).  Pure host computation. */
int ips_batch_workspace_bytes(void* const* d_ptrs, const uint64_t* ns,
                              uint32_t count, int elem_type, int algo,
                              const ips_params* params, size_t* out_bytes);

/* Sort `count` arrays in separate device buffers (d_ptrs[i], ns[i]
 * elements of elem_type each, non-overlapping; HOST arrays read during the
 * call) in place, as ips_sort_segments does for segments of one array:
 * arrays whose addresses are congruent modulo the element size become
 * segments of one batched call (one call for 4/8/16-byte elements in
 * 256-byte aligned buffers).  Errors: as ips_sort_segments, plus
 * IPS_E_MISALIGNED for a misaligned pointer. */
int ips_sort_batch(ips_ctx* ctx, void* const* d_ptrs, const uint64_t* ns,
                   uint32_t count, int elem_type, int algo, void* d_ws,
                   size_t ws_bytes, const ips_params* params, void* stream);

/* Serving: replay of an arrival trace of sort requests (no paper passage;
 * built on the batched sort).  A request's data is in device memory at
 * d_data when it arrives; arrival_s is its arrival time in seconds after
 * the replay starts.  The scheduler admits waiting requests in arrival
 * order while the admitted data plus the workspace of the round's largest
 * batch stays within hbm_budget bytes (and the workspace within ws_bytes),
 * then sorts the round's requests with one ips_sort_batch call per (type,
 * algorithm) and starts the next round with everything that arrived
 * meanwhile (continuous batching at round granularity).  Policy
 * IPS_SERVE_FIFO instead sorts one request per call in arrival order (the
 * comparison baseline).  Outputs per request: start_s and done_s (seconds
 * after the replay start when its call was issued and returned), status
 * (IPS_OK, IPS_E_WORKSPACE when the request alone exceeds the budget or
 * the workspace, or the call's error) and the index of its batch. */
#define IPS_SERVE_BATCH 0u
#define IPS_SERVE_FIFO 1u
typedef struct {
  void* d_data;
  uint64_t n;
  int32_t elem_type, algo;
  double arrival_s;
  double start_s, done_s;   /* out */
  int32_t status;           /* out */
  uint32_t batch;           /* out */
  int32_t detail;           /* out: on IPS_E_DEVICE / IPS_E_HIP, ips_last_device_error /
                               ips_last_hip_error right after the failing call */
  int32_t pad;
} ips_request;

typedef struct {
  uint64_t hbm_budget;   /* bytes of request data plus workspace in flight */
  uint32_t policy;       /* IPS_SERVE_BATCH or IPS_SERVE_FIFO */
  uint32_t max_batch;    /* requests per round at most (0: no limit) */
} ips_serve_config;

/* Workspace bytes that any round of ips_serve_trace over these requests
 * can need under cfg->hbm_budget.  Pure host computation. */
int ips_serve_workspace_bytes(const ips_request* reqs, uint32_t nreq,
                              const ips_serve_config* cfg,
                              const ips_params* params, size_t* out_bytes);

/* Replays the trace (blocking; returns when every request is finished).
 * Returns IPS_OK, or the first error any request got (the others are
 * still served). */
int ips_serve_trace(ips_ctx* ctx, ips_request* reqs, uint32_t nreq,
                    const ips_serve_config* cfg, void* d_ws, size_t ws_bytes,
                    const ips_params* params, void* stream);

/* Description of the root partitioning step of the last sort on `ctx`
 * (Section 4.1).  For IPS_SAMPLESORT: alpha, k_prime (adaptive k), m (sample
 * size), u (distinct splitters), K (power of two >= u+1), eq (equality
 * buckets), nb (buckets: K, or 2K with equality buckets), splitters[0..K-1]
 * stored as keys (u32 keys widened to u64; f64 as the raw double bits; the
 * 100-byte record key as bytes 0..9 in the first ten bytes of the 16-byte
 * slot; the Quartet's first two key words a, b, its third word c not
 * reported).  For IPS_RADIX: radix_shift and radix_width of the root digit.
 * bucket_start[0..nb] are the bucket boundaries (elements) after the step.
 * valid is 0 when the last sort had no root partitioning step (n small,
 * sorted input). */
typedef struct {
  uint32_t valid, algo, alpha, k_prime, m, u, K, eq, nb;
  uint32_t radix_shift, radix_width, block_elems, stripes, pad;
  uint64_t n;
  uint8_t splitters[256][16];
  uint64_t bucket_start[513];
} ips_root_info;

int ips_get_root_info(ips_ctx* ctx, ips_root_info* out);

/* Counters of the last sort: partitioning levels, steps, elements moved
 * through partitioning steps and through the LDS tier, whether the input
 * was detected as sorted (1) or reverse sorted (2). */
typedef struct {
  uint32_t levels, steps, batches, lds_tasks;
  uint32_t detected, pad0;
  uint64_t partitioned_elems, lds_elems;
  uint64_t max_step_elems;
} ips_stats;

int ips_get_stats(ips_ctx* ctx, ips_stats* out);

/* Per-kernel timing of the last sort made with IPS_FLAG_PROFILE.  Row L <
 * IPS_MAX_LEVELS covers the partitioning steps of recursion level L and the
 * LDS-tier sorts of the buckets they produced; row IPS_MAX_LEVELS covers
 * work outside the levels (sorted check, radix min/max, an LDS-only root).
 * Columns are the IPS_PH_* kernels: ms is the summed launch duration,
 * elems the elements of the tasks those launches covered, launches the
 * number of launches. */
#define IPS_MAX_LEVELS 16
#define IPS_PHASES 13
enum {
  IPS_PH_SORTED_CHECK = 0, IPS_PH_MINMAX = 1, IPS_PH_SAMPLE = 2, IPS_PH_CLASSIFY = 3,
  IPS_PH_BOUNDARIES = 4, IPS_PH_FLAGS = 5, IPS_PH_PERMUTE = 6, IPS_PH_CLEANUP_A = 7,
  IPS_PH_CLEANUP_B = 8, IPS_PH_LDS_SORT = 9, IPS_PH_REVERSE = 10,
  IPS_PH_HISTOGRAM = 11,   /* IPS_FLAG_FUSED: digit histogram of a step */
  IPS_PH_FUSED = 12        /* IPS_FLAG_FUSED: classification fused with the permutation */
};
typedef struct {
  uint32_t levels, pad;
  double ms[IPS_MAX_LEVELS + 1][IPS_PHASES];
  uint64_t elems[IPS_MAX_LEVELS + 1][IPS_PHASES];
  uint32_t launches[IPS_MAX_LEVELS + 1][IPS_PHASES];
} ips_profile;

int ips_get_profile(ips_ctx* ctx, ips_profile* out);

/* Autotuned parameters.  The paper tunes k, the block size and the base
 * case per machine (Section 6) and notes that the best values depend on the
 * input size; an entry of this table holds measured best values for one
 * element type and algorithm over a range of size classes (floor(log2 n)
 * of the elements of one call, all segments or arrays of a batched call
 * together), separately for single-array calls (batched = 0) and batched
 * calls (batched = 1).  The table is written by the tuning script of the
 * Python package from timings on the GPU; the library stores none.
 * A zero field means "no tuned value" (the default applies). */
typedef struct {
  int32_t elem_type;      /* IPS_U32 .. IPS_QUARTET */
  int32_t algo;           /* IPS_SAMPLESORT or IPS_RADIX */
  uint32_t log2n_min;     /* size classes [log2n_min, log2n_max] */
  uint32_t log2n_max;
  uint32_t batched;       /* 0: ips_sort_keys/pairs, 1: segments or batch calls */
  uint32_t k;             /* as in ips_params */
  uint32_t block_bytes;
  uint32_t n0;
  uint32_t lds_task_max;  /* selects which of the LDS tier's workgroup shapes run */
  uint32_t piece_blocks;
  uint32_t perm_groups;
  uint32_t perm_wg;       /* workgroup size of the block permutation */
  uint32_t k_root;        /* buckets of a root step at most */
} ips_tune_entry;

/* Parameters for one call from a tuning table: *out = *base (zeroed when
 * base is NULL), then every field of *out that is zero and tunable (k,
 * block_bytes, n0, lds_task_max, piece_blocks, perm_groups, perm_wg, k_root) takes the value
 * of the first entry of table[0, count) that matches elem_type, algo,
 * batched and floor(log2 n) (n >= 1).  Fields the caller set are kept; flags,
 * seed and profile_mask are never changed.  Pass the same *out to the
 * workspace query and to the sort.  Pure host computation.  Returns 1 when
 * an entry matched, 0 when none did (then *out = *base), or
 * IPS_E_INVALID_ARG for a null `out`, a null table with count > 0, or an
 * entry whose log2n_min exceeds log2n_max. */
int ips_tuned_params(const ips_tune_entry* table, uint32_t count, uint64_t n, int elem_type, int algo,
                     int batched, const ips_params* base, ips_params* out);

/* Last HIP error code seen by the context (hipError_t as int) and the
 * last kernel-reported consistency error (0 = none; bits 0-7 the error
 * code, bits 8-19 and 20-31 the low bits of its two arguments). */
int ips_last_hip_error(ips_ctx* ctx);
int ips_last_device_error(ips_ctx* ctx);

const char* ips_status_string(int status);
int ips_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* IPS_H */
