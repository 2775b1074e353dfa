// Host side of the C ABI (include/ips.h): argument validation, workspace
// planning, and the level-by-level orchestration of partitioning steps
// (arXiv 2009.13569, Sections 4.1-4.2 and 6) on one MI355X.
//
// The recursion is breadth first.  All partitioning tasks of one recursion
// level are grouped into batches; one batch runs each phase of the
// partitioning step as one kernel launch over all of its tasks.  Bucket
// sizes come back to the host after each batch, which turns large buckets
// into next-level tasks and launches the LDS-tier sort for small ones.
// Equality buckets are final (Section 4.1, "Sampling").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <deque>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/ips.h"
#include "ips_common.hpp"
#include "ips_launch.hpp"
#include "ips_oop.hpp"

using namespace ips;

namespace {

constexpr uint32_t WG_TARGET = 1024;      // classification workgroups per level (4 per CU)
constexpr uint32_t GRP_TARGET = 131072;   // default permutation groups per batch
constexpr uint32_t TB_MAX = 512;          // tasks per batch
constexpr uint32_t WB_MAX = 2048;         // classification workgroups per batch

struct Cfg {
  const Launchers* L;
  int type;
  uint32_t D, DW;
  bool radix, gbuf;
  uint32_t k, n0, cap, cmax, flags;
  uint32_t k_root;  // buckets of a root step at most (level 0; k for deeper levels)
  uint64_t seed;
  uint32_t b_req;   // requested block elements (0 = automatic)
  uint32_t groups;  // permutation groups per batch
  uint32_t perm_threads;   // workgroup size of the block permutation
  uint32_t buf_bytes;      // LDS of the classification's buffer blocks
  bool fused;              // radix steps with classification fused into the permutation
  bool insertion;          // the paper's base case: insertion sort of buckets of <= 2 n0 elements
};

// Largest task of the fused radix step: its pointer words hold element
// positions in 31 bits.
constexpr uint64_t FUSED_MAX_N = (1ull << 31) - (1ull << 16);

uint32_t elem_bytes(int t) {
  switch (t) {
    case 1: return 4;
    case 2: return 8;
    case 3: return 8;
    case 4: return 16;
    case 5: return 100;
    case 6: return 32;
    default: return 0;
  }
}

const Launchers* launchers_for(int t) {
  switch (t) {
    case 1: return launchers_u32();
    case 2: return launchers_u64();
    case 3: return launchers_f64();
    case 4: return launchers_pair();
    case 5: return launchers_rec100();
    case 6: return launchers_quartet();
    default: return nullptr;
  }
}

uint32_t default_cap(int t) {
  const Launchers* L = launchers_for(t);
  return L ? L->lds_cap : 0;
}

// Paper's block size max(1, 2^floor(11 - log2 D)) elements (Section 6).
uint32_t paper_block(uint32_t D) {
  uint32_t b = 1;
  while ((uint64_t)b * 2 * D <= 2048) b *= 2;
  return b;
}

int make_cfg(uint64_t n, int type, int algo, const ips_params* p, Cfg* c) {
  (void)n;
  const uint32_t D = elem_bytes(type);
  if (!D) return IPS_E_INVALID_ARG;
  if (algo != IPS_SAMPLESORT && algo != IPS_RADIX) return IPS_E_INVALID_ARG;
  if (algo == IPS_RADIX && (type == 5 || type == 6)) return IPS_E_UNSUPPORTED;
  ips_params z;
  std::memset(&z, 0, sizeof(z));
  if (!p) p = &z;
  c->type = type;
  c->D = D;
  c->DW = D / 4;
  c->radix = algo == IPS_RADIX;
  c->flags = p->flags;
  c->gbuf = (p->flags & IPS_FLAG_GLOBAL_BUFFERS) != 0;
  c->k = p->k ? p->k : MAX_K;
  if (c->k < 2 || c->k > MAX_K || (c->k & (c->k - 1))) return IPS_E_INVALID_ARG;
  const uint32_t dcap = default_cap(type);
  c->cap = p->lds_task_max ? p->lds_task_max : dcap;
  if (c->cap > dcap) return IPS_E_INVALID_ARG;
  c->n0 = p->n0;   // 0: buckets sized for the LDS tier (see task_kprime)
  c->cmax = p->piece_blocks ? p->piece_blocks : 1024;
  c->groups = p->perm_groups ? p->perm_groups : GRP_TARGET;
  if (c->groups > (1u << 20)) return IPS_E_INVALID_ARG;
  c->perm_threads = p->perm_wg ? p->perm_wg : PERM_THREADS;
  c->buf_bytes = launchers_for(type)->buf_bytes;
  if (c->perm_threads != 128 && c->perm_threads != 256 && c->perm_threads != 512) return IPS_E_INVALID_ARG;
  c->k_root = p->k_root ? p->k_root : c->k;
  if (c->k_root < 2 || c->k_root > MAX_K || (c->k_root & (c->k_root - 1))) return IPS_E_INVALID_ARG;
  c->seed = p->seed;
  c->b_req = 0;
  if (p->block_bytes) {
    c->b_req = std::max<uint32_t>(1, p->block_bytes / D);
    if ((uint64_t)c->b_req * D > MAX_BLOCK_BYTES) return IPS_E_INVALID_ARG;
  } else if (c->gbuf) {
    c->b_req = paper_block(D);
  }
  if ((p->flags & IPS_FLAG_EQ_ON) && (p->flags & IPS_FLAG_EQ_OFF)) return IPS_E_INVALID_ARG;
  if (p->flags & ~0x7FFu) return IPS_E_INVALID_ARG;
  c->insertion = (p->flags & IPS_FLAG_INSERTION_BASE) != 0;
  if (c->insertion) {
    if (c->radix) return IPS_E_UNSUPPORTED;
    if (!c->n0) return IPS_E_INVALID_ARG;
    c->cap = std::min<uint32_t>(dcap, 2 * c->n0);   // a task of at most 2 n0 elements is a base case
  }
  c->fused = (p->flags & IPS_FLAG_FUSED) != 0;
  if (c->fused) {
    if (!c->radix || !launchers_for(type)->fhist) return IPS_E_UNSUPPORTED;
    if (c->gbuf || (p->flags & (IPS_FLAG_HOST_PLAN | IPS_FLAG_LEVEL1_ONLY))) return IPS_E_UNSUPPORTED;
    if (n > FUSED_MAX_N) return IPS_E_TOO_LARGE;
    c->buf_bytes = FUSED_BUF_BYTES;   // two workgroups of the fused kernel share a CU's LDS
  }
  if (p->profile_mask >> IPS_PHASES) return IPS_E_INVALID_ARG;
  c->L = nullptr;
  return IPS_OK;
}

// Adaptive number of buckets of the paper (Section 4.2): for
// k n0 < n < k^2 n0 the smallest power of two 2^c with 2c >= log2(n/n0)+1,
// for n0 < n <= k n0 the smallest 2^c >= n/n0, otherwise k; in [2, k].
uint32_t paper_kprime(uint64_t n, uint32_t k, uint32_t n0) {
  const unsigned __int128 kn0 = (unsigned __int128)k * n0, kkn0 = kn0 * k;
  uint64_t r = k;
  if ((unsigned __int128)n > kn0 && (unsigned __int128)n < kkn0) {
    uint32_t c = 1;
    while (((unsigned __int128)n0 << (2 * c - 1)) < n) ++c;
    r = 1ull << c;
  } else if (n > n0 && (unsigned __int128)n <= kn0) {
    uint32_t c = 0;
    while (((unsigned __int128)n0 << c) < n) ++c;
    r = 1ull << c;
  }
  return (uint32_t)std::min<uint64_t>(k, std::max<uint64_t>(2, r));
}

// k' of a task.  With an explicit n0 the paper's rule.  By default the base
// case is the LDS tier of capacity cap instead of insertion sort on n0
// elements, so k' is the smallest power of two that makes the mean bucket at
// most cap / 4 (a bucket then exceeds the tier only with negligible
// probability), capped at k.
uint32_t task_kprime(const Cfg& c, uint64_t n, uint32_t level) {
  const uint32_t k = level ? c.k : c.k_root;
  if (c.n0) return paper_kprime(n, k, c.n0);
  uint64_t r = 2;
  while (r < k && r * (c.cap / 4) < n) r *= 2;
  return (uint32_t)r;
}

// Block elements of a step with nb buckets: in LDS mode one buffer block per
// bucket must fit the LDS budget; a block never exceeds MAX_BLOCK_BYTES.
uint32_t block_elems(const Cfg& c, uint32_t nb) {
  const uint32_t bmax = std::max<uint32_t>(1, MAX_BLOCK_BYTES / c.D);
  if (c.gbuf) return std::min(bmax, std::max<uint32_t>(1, c.b_req));
  // LDS holds nb buffers of b elements (plus BUF_PAD_DW dwords of padding each)
  uint32_t b = std::max<uint32_t>(1, c.buf_bytes / (nb * c.D));
  b = std::min(b, bmax);
  if (c.b_req) b = std::min(b, c.b_req);
  return b;
}

uint32_t max_nb(const Cfg& c) { return c.radix ? MAX_K : 2 * c.k; }

// Buckets of any step of a sort of at most n elements: radix steps have at
// most 2^8; a samplesort task of n' elements has at most 2 k'(n') (equality
// buckets double K <= k'), and the default k' rule grows with n' (the
// paper's rule does not, so it is bounded by k).
uint32_t plan_nb(const Cfg& c, uint64_t n) {
  if (c.radix) return MAX_K;
  if (c.n0) return 2 * std::max(c.k, c.k_root);
  return 2 * std::max(task_kprime(c, n, 0), task_kprime(c, n, 1));
}

struct Layout {
  uint32_t TB, WB, PWB, LTB, NBE;   // tasks, cls WGs, perm WGs, LDS tasks, bucket entries
  uint32_t NXB;                     // next-level tasks one batch can produce
  uint32_t QCAP;                    // task queue of the device-planned execution
  uint32_t NBS;                     // buckets per step at most (row length of per-WG arrays)
  uint64_t SB, SPB, PB;             // slot bytes, spill bytes, pieces
  uint64_t slot_max;
  size_t off[40];
  size_t total;
};

enum Region {
  R_CTRL, R_TASKS, R_RECS, R_CLS, R_PERM, R_CLN, R_NFULL, R_LEFT, R_F, R_WMIN, R_WMAX, R_SLOTS,
  R_SPILL, R_OVF, R_BSTART, R_BCOUNT, R_BD, R_BPLB, R_BPLE, R_BMIN, R_BMAX, R_PWORD,
  R_PA, R_PC, R_PR, R_PCUM, R_TNP, R_TUP, R_LT, R_BFULL, R_PFCNT, R_LTC, R_NEXT, R_QUEUE, R_STEPEL, R_COUNT
};

// Workspace plan of a sort of n elements (Section 5.1: O(k b) extra memory
// per thread; here per workgroup).  Every region is either per task (O(k)
// words: step records, bucket tables, pieces, one overflow block and one
// spill area of one buffer block per bucket), per workgroup (O(k) counters
// and, for the stripes' buffer blocks saved after classification, one
// buffer block per bucket = the LDS budget), or bounded by the number of
// tasks and workgroups of one step.  The step's task and workgroup budgets
// (TB <= 512 tasks, WB <= 2048 workgroups) are constants, so for large n the
// workspace no longer grows with n; for small n the budgets shrink with the
// data (a single task never needs more slots than a quarter of its data
// plus one buffer block per bucket).
void plan(uint64_t n, const Cfg& c, Layout* L) {
  const uint32_t nbm = plan_nb(c, n);
  const uint32_t bmin = block_elems(c, nbm);
  uint64_t slot_max = 0;
  for (uint32_t nb = 2; nb <= nbm; nb *= 2)
    slot_max = std::max<uint64_t>(slot_max, ((uint64_t)nb * block_elems(c, nb) * c.D + 255) & ~255ull);
  // Tasks of one step: every queued partitioning task holds more than cap
  // elements, so at most n / (cap + 1) of them exist at once.
  const uint64_t tasks_ub = std::max<uint64_t>(1, n / ((uint64_t)c.cap + 1));
  L->TB = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(TB_MAX, tasks_ub),
                                       std::max<uint64_t>(16, n * c.D / (256 * 1024)));
  L->WB = (uint32_t)std::min<uint64_t>(std::min<uint32_t>(WB_MAX, WG_TARGET + L->TB),
                                       L->TB + n * c.D / 65536 + 16);
  L->NBS = nbm;
  L->slot_max = slot_max;
  // Buffer slots: one buffer block per bucket per stripe, and any single task
  // fits (a task has at most n D / (4 nb b) stripes, so its slots need at
  // most max(one slot, n D / 4 + 256 per stripe of rounding)).
  const uint64_t data_budget = std::max<uint64_t>(slot_max, n * c.D / 4 + (uint64_t)L->WB * 256);
  L->SB = std::min<uint64_t>((uint64_t)L->WB * slot_max, data_budget);
  L->SPB = std::min<uint64_t>((uint64_t)L->TB * slot_max, data_budget);
  // Pieces: a task with nb buckets has at most 2 nb + 3 + W + NB / cmax of
  // them.  Under the default k' rule k' is below 8 n' / cap (or 2), so a
  // samplesort batch needs at most 32 n / cap + 13 per task besides the
  // stripe and chunk terms (radix steps always have up to 256 buckets).
  uint64_t pb_buckets = (uint64_t)L->TB * (2 * nbm + 3);
  if (!c.n0 && !c.radix) pb_buckets = std::min<uint64_t>(pb_buckets, 32 * n / c.cap + 13ull * L->TB);
  // Chunk pieces: a bucket's range is cut every max(cmax, its blocks / 32)
  // blocks, so at most 64 times per bucket (its range exceeds its own full
  // blocks by at most one block per stripe), and never more than the blocks
  // of the step divided by cmax.
  L->PB = pb_buckets + L->WB + std::min<uint64_t>(n / bmin / c.cmax + L->TB, 64ull * nbm * L->TB) + 16;
  // Permutation workgroups: a task of NB blocks gets at most NB / 4 groups
  // (or one) of max(4, b DW / 4) lanes at most; a workgroup of NT threads
  // holds NT / lanes groups, so one step needs at most
  // min(groups * 64 / NT, n / (NT bmin) + n DW / (16 NT)) workgroups plus two
  // per task.
  const uint64_t NT = c.perm_threads;
  const uint64_t pw_data = n / (NT * bmin) + n * c.DW / (16 * NT) + 1;
  L->PWB = (uint32_t)(std::min<uint64_t>(c.groups * 64 / NT, pw_data) + 2ull * L->TB + 16);
  // Buckets of one step: at most 2k' (equality buckets) per task; under the
  // default k' rule k' < 8 n' / cap (or 2), and the tasks of a step are
  // disjoint, so a step has fewer than 16 n / cap + 4 TB of them.  These
  // bound the bucket tables, the cleanup items and the LDS-tier children.
  uint64_t nbe = (uint64_t)L->TB * nbm;
  if (!c.n0 && !c.radix) nbe = std::min<uint64_t>(nbe, 16 * n / c.cap + 4ull * L->TB);
  L->NBE = (uint32_t)(nbe + L->TB);
  L->LTB = (uint32_t)nbe + 1;
  size_t sz[R_COUNT];
  sz[R_CTRL] = CTRL_WORDS * 4;
  sz[R_TASKS] = (size_t)L->TB * sizeof(PTask);
  sz[R_RECS] = c.radix ? 0 : (size_t)L->TB * sizeof(StepRec);   // radix steps take no sample
  sz[R_CLS] = (size_t)L->WB * 4;
  sz[R_PERM] = (size_t)L->PWB * 4;
  sz[R_CLN] = (size_t)L->NBE * 4;
  sz[R_NFULL] = (size_t)L->WB * nbm * 4;
  sz[R_LEFT] = (size_t)L->WB * nbm * 4;
  sz[R_F] = (size_t)L->WB * 4;
  sz[R_WMIN] = c.radix ? (size_t)L->WB * nbm * 8 : 0;
  sz[R_WMAX] = sz[R_WMIN];
  sz[R_SLOTS] = L->SB;
  sz[R_SPILL] = L->SPB;
  sz[R_OVF] = (size_t)L->TB * MAX_BLOCK_BYTES;
  sz[R_BSTART] = (size_t)L->NBE * 8;
  sz[R_BCOUNT] = (size_t)L->NBE * 4;
  sz[R_BD] = (size_t)L->NBE * 4;
  sz[R_BPLB] = (size_t)L->NBE * 4;
  sz[R_BPLE] = (size_t)L->NBE * 4;
  sz[R_BMIN] = c.radix ? (size_t)L->NBE * 8 : 0;
  sz[R_BMAX] = sz[R_BMIN];
  sz[R_PWORD] = L->PB * 8 * PWORD_STRIDE;
  sz[R_PA] = L->PB * 4;
  sz[R_PC] = L->PB * 4;
  sz[R_PR] = L->PB * 4;
  sz[R_PCUM] = L->PB * 4;
  sz[R_PFCNT] = L->PB * 4;
  // children for the LDS tier, per variant: two steps' worth (device-planned
  // steps let the lists fill over several steps)
  sz[R_LTC] = 3 * 2 * (size_t)L->LTB * sizeof(LTask);
  L->NXB = (uint32_t)std::min<uint64_t>((uint64_t)L->TB * nbm, tasks_ub + L->TB);
  sz[R_NEXT] = (size_t)L->NXB * sizeof(CTask);
  L->QCAP = (uint32_t)std::min<uint64_t>(tasks_ub + L->TB, 0xFFFFFFF0ull);
  sz[R_QUEUE] = (size_t)L->QCAP * sizeof(CTask);
  sz[R_STEPEL] = (size_t)MAX_STEPS_RECORDED * 4 * 8;
  sz[R_TNP] = (size_t)L->TB * 4;
  sz[R_TUP] = (size_t)L->TB * 4;
  sz[R_LT] = (size_t)L->LTB * sizeof(LTask);
  sz[R_BFULL] = (size_t)L->NBE * 8;
  size_t off = 0;
  for (int r = 0; r < R_COUNT; ++r) {
    L->off[r] = off;
    off += (sz[r] + 255) & ~(size_t)255;
  }
  L->total = off;
}

struct HTask {
  uint64_t l, n;
  uint32_t level, tflags, shift, width;
};

}  // namespace

// Scratch of ips_sort_keys_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes `scratch`
// itself to a kernel (in host code the name is only a stand-in); its device
// address on each GPU is taken once with hipGetSymbolAddress when the first
// context on that GPU is created, and that address is used everywhere.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Pinned staging every context allocates when it is created: enough for the
// largest plan of any call whose workspace fits the static scratch (at most
// TB_MAX tasks, WB_MAX classification workgroups, 2^18 + 2 TB_MAX + 16
// permutation workgroups and TB_MAX * MAX_NB LDS-tier tasks), so that the
// allocation-free entry point never needs a larger buffer.
constexpr size_t PIN_PREALLOC_BYTES = (size_t)8 << 20;

struct ips_ctx {
  int device = 0;
  bool noalloc = false;      // inside ips_sort_keys_noalloc: never allocate
  void* scratch = nullptr;   // this device's address of `scratch`
  int last_hip = 0;
  int last_dev = 0;
  ips_root_info root;
  ips_stats stats;
  ips_profile prof;
  uint8_t* pin = nullptr;   // pinned staging
  size_t pin_bytes = 0;
  // Launch timing (IPS_FLAG_PROFILE): event pairs resolved at sync points.
  std::vector<hipEvent_t> ev_pool;
  // src >= 0: elems are read from the device's per-step record src of step row
  struct Pending { hipEvent_t a, b; uint32_t row, ph; uint64_t elems; int src; };
  std::vector<Pending> pending;
  bool profiling = false;
  uint32_t profile_mask = 0;   // phases timed (0: all)
};

namespace {

hipEvent_t take_event(ips_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Collects the durations of finished launches into ctx->prof.
void resolve_profile(ips_ctx* ctx) {
  for (const auto& p : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->prof.ms[p.row][p.ph] += ms;
      ctx->prof.elems[p.row][p.ph] += p.elems;
      ctx->prof.launches[p.row][p.ph] += 1;
    }
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.clear();
}

// Brackets one launch with events when profiling.
template <class F>
hipError_t timed(ips_ctx* ctx, hipStream_t st, uint32_t row, uint32_t ph, uint64_t elems, F&& launch,
                 int src = -1) {
  if (!ctx->profiling || (ctx->profile_mask && !((ctx->profile_mask >> ph) & 1u))) return launch();
  hipEvent_t a = take_event(ctx), b = take_event(ctx);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, st);
  if (e != hipSuccess) return e;
  if (row > IPS_MAX_LEVELS) row = IPS_MAX_LEVELS;
  ctx->pending.push_back({a, b, row, ph, elems, src});
  return hipSuccess;
}

#define HIPCHK(ctx, expr)                        \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) {                      \
      (ctx)->last_hip = (int)e_;                 \
      return IPS_E_HIP;                          \
    }                                            \
  } while (0)

int ensure_pinned(ips_ctx* ctx, size_t bytes) {
  if (ctx->pin_bytes >= bytes) return IPS_OK;
  if (ctx->noalloc) return IPS_E_SCRATCH;
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  ctx->pin = nullptr;
  ctx->pin_bytes = 0;
  size_t want = std::max<size_t>(bytes, 1 << 20);
  HIPCHK(ctx, hipHostMalloc(reinterpret_cast<void**>(&ctx->pin), want, hipHostMallocDefault));
  ctx->pin_bytes = want;
  return IPS_OK;
}

struct Run {
  ips_ctx* ctx;
  Cfg c;
  Layout L;
  uint8_t* ws;
  uint32_t* data;
  uint64_t n;
  hipStream_t st;
  BatchArgs a;
  // pinned staging areas
  PTask* h_tasks;
  uint32_t* h_maps;   // cls | perm | cln
  LTask* h_lt;
  uint8_t* h_rb;      // readback
  size_t rb_bytes;
  uint32_t* h_ctrl;
  uint32_t lds_min = LDS_DEFER_TASKS;   // device-planned steps: LDS-tier lists run from this many tasks
};

template <class P>
P* wsp(Run& r, Region reg) { return reinterpret_cast<P*>(r.ws + r.L.off[reg]); }

int check_dev_error(Run& r) {
  uint32_t err = r.h_ctrl[CTRL_ERR];
  if (err) {
    r.ctx->last_dev = (int)((err & 0xFFu) | ((r.h_ctrl[CTRL_ERR_A] & 0xFFFu) << 8) |
                            ((r.h_ctrl[CTRL_ERR_B] & 0xFFFu) << 20));
    return IPS_E_DEVICE;
  }
  return IPS_OK;
}

int read_ctrl(Run& r) {
  HIPCHK(r.ctx, hipMemcpyAsync(r.h_ctrl, r.a.ctrl, CTRL_WORDS * 4, hipMemcpyDeviceToHost, r.st));
  HIPCHK(r.ctx, hipStreamSynchronize(r.st));
  resolve_profile(r.ctx);
  return check_dev_error(r);
}

// Sorts the given small tasks in the LDS tier: each task runs on the
// smallest of the three workgroup variants that holds it; all parts share
// one upload.
int launch_lds_tasks(Run& r, const std::vector<LTask>& lt_in, uint32_t row) {
  const uint32_t* caps = r.c.L->lds_caps;
  std::vector<LTask> lt;
  lt.reserve(lt_in.size());
  size_t bound[4] = {0, 0, 0, 0};
  if (r.c.insertion) {   // one list, sorted by insertion sort
    lt = lt_in;
    bound[1] = bound[2] = bound[3] = lt.size();
  } else {
    for (uint32_t v = 0; v < 3; ++v) {
      const uint32_t lo = v ? caps[v - 1] : 0;
      if (v && caps[v] == caps[v - 1]) { bound[v + 1] = lt.size(); continue; }
      for (const LTask& t : lt_in)
        if (t.n > lo && t.n <= caps[v]) lt.push_back(t);
      bound[v + 1] = lt.size();
    }
  }
  size_t done = 0;
  while (done < lt.size()) {
    const size_t cnt = std::min<size_t>(lt.size() - done, r.L.LTB);
    std::memcpy(r.h_lt, lt.data() + done, cnt * sizeof(LTask));
    LTask* d_lt = wsp<LTask>(r, R_LT);
    HIPCHK(r.ctx, hipMemcpyAsync(d_lt, r.h_lt, cnt * sizeof(LTask), hipMemcpyHostToDevice, r.st));
    for (uint32_t v = 0; v < 3; ++v) {
      const size_t p0 = std::max(done, bound[v]);
      const size_t p1 = std::min(done + cnt, bound[v + 1]);
      if (p1 <= p0) continue;
      uint64_t el = 0;
      for (size_t q = p0; q < p1; ++q) el += lt[q].n;
      HIPCHK(r.ctx, timed(r.ctx, r.st, row, IPS_PH_LDS_SORT, el, [&] {
               return r.c.L->lds_sort(d_lt + (p0 - done), (uint32_t)(p1 - p0), r.data,
                                      r.c.insertion ? LDS_INSERTION : v, r.a.ctrl, nullptr, 0, r.st);
             }));
    }
    done += cnt;
    r.ctx->stats.lds_tasks += (uint32_t)cnt;
    if (done < lt.size()) {   // the staging buffer is reused: wait for the copy
      HIPCHK(r.ctx, hipStreamSynchronize(r.st));
      resolve_profile(r.ctx);
    }
  }
  return IPS_OK;
}

// Launches the LDS tier on the per-variant task lists the children kernel
// wrote on the device (counts read back by the host).
hipError_t launch_lds_lists(Run& r, const ChildArgs& ca, const uint32_t (&cnt)[3], const uint64_t (&el)[3],
                            uint32_t row) {
  for (uint32_t v = 0; v < 3; ++v) {
    if (!cnt[v]) continue;
    if (v && (r.c.insertion || r.c.L->lds_caps[v] == r.c.L->lds_caps[v - 1])) return hipErrorInvalidValue;
    hipError_t e = timed(r.ctx, r.st, row, IPS_PH_LDS_SORT, el[v], [&] {
      return r.c.L->lds_sort(ca.lt[v], cnt[v], r.data, r.c.insertion ? LDS_INSERTION : v, r.a.ctrl, nullptr, 0,
                             r.st);
    });
    if (e != hipSuccess) return e;
    r.ctx->stats.lds_tasks += cnt[v];
  }
  return hipSuccess;
}

// Upper bounds of one task's resources before its step is sampled.
struct Need {
  uint64_t wg, slot, spill, pieces;
};

Need task_need(const Run& r, const HTask& t, uint64_t level_elems) {
  Need nd;
  const uint64_t S = std::max<uint64_t>(1, level_elems / WG_TARGET);
  const uint64_t wub = (t.n + S - 1) / S;
  nd.wg = std::min<uint64_t>(std::min<uint64_t>(wub, WG_TARGET), r.L.WB);
  nd.slot = std::min<uint64_t>(nd.wg * r.L.slot_max,
                               std::max<uint64_t>(r.L.slot_max, t.n * r.c.D / 4 + nd.wg * 256));
  nd.spill = r.L.slot_max;
  const uint32_t nbt = r.c.radix ? MAX_K : 2 * task_kprime(r.c, t.n, t.level);   // buckets at most
  const uint32_t bmin = block_elems(r.c, nbt);
  nd.pieces = 2ull * nbt + 3 + nd.wg + (t.n / bmin + 1) / r.c.cmax + 1;
  return nd;
}

int run_batch(Run& r, const std::vector<HTask>& bt, uint64_t level_elems, std::vector<HTask>& next,
              bool root_level) {
  ips_ctx* ctx = r.ctx;
  const Cfg& c = r.c;
  const uint32_t T = (uint32_t)bt.size();
  // 1. Tasks and, for samplesort, the sampling phase.
  for (uint32_t t = 0; t < T; ++t) {
    PTask& p = r.h_tasks[t];
    std::memset(&p, 0, sizeof(p));
    p.l = bt[t].l;
    p.n = bt[t].n;
    p.level = bt[t].level;
    p.tflags = bt[t].tflags | (c.radix ? TF_RADIX : 0u);
    p.shift = bt[t].shift;
    p.width = bt[t].width;
    p.kp = task_kprime(c, bt[t].n, bt[t].level);
  }
  PTask* d_tasks = wsp<PTask>(r, R_TASKS);
  StepRec* d_recs = wsp<StepRec>(r, R_RECS);
  struct Hdr { uint32_t K, logK, eq, nb, u, alpha, kp, m; };
  std::vector<Hdr> hdr(T);
  if (!c.radix) {
    HIPCHK(ctx, hipMemcpyAsync(d_tasks, r.h_tasks, T * sizeof(PTask), hipMemcpyHostToDevice, r.st));
    uint64_t el = 0;
    for (const HTask& t : bt) el += t.n;
    HIPCHK(ctx, timed(ctx, r.st, bt[0].level, IPS_PH_SAMPLE, el,
                      [&] { return c.L->sample(r.a, T, c.seed, r.st); }));
    HIPCHK(ctx, hipMemcpy2DAsync(r.h_rb, sizeof(Hdr), d_recs, sizeof(StepRec), sizeof(Hdr), T,
                                 hipMemcpyDeviceToHost, r.st));
    HIPCHK(ctx, hipMemcpyAsync(r.h_ctrl, r.a.ctrl, CTRL_WORDS * 4, hipMemcpyDeviceToHost, r.st));
    HIPCHK(ctx, hipStreamSynchronize(r.st));
    resolve_profile(ctx);
    if (int e = check_dev_error(r)) return e;
    std::memcpy(hdr.data(), r.h_rb, T * sizeof(Hdr));
  } else {
    for (uint32_t t = 0; t < T; ++t) {
      Hdr& h = hdr[t];
      std::memset(&h, 0, sizeof(h));
      h.K = 1u << bt[t].width;
      h.logK = bt[t].width;
      h.nb = h.K;
    }
  }
  // 2. Geometry of every task.
  uint64_t nb_sum = 0, blocks_sum = 0;
  std::vector<uint32_t> bvec(T), NBv(T), nbv(T);
  for (uint32_t t = 0; t < T; ++t) {
    nbv[t] = hdr[t].nb;
    bvec[t] = block_elems(c, nbv[t]);
    NBv[t] = (uint32_t)((bt[t].n + bvec[t] - 1) / bvec[t]);
    nb_sum += nbv[t];
    blocks_sum += NBv[t];
  }
  uint32_t wg = 0, pwg = 0, maxW = 1, cln = 0;
  uint64_t slot_off = 0, spill_off = 0;
  uint32_t piece = 0, bucket = 0;
  uint32_t* h_cls = r.h_maps;
  uint32_t* h_perm = h_cls + r.L.WB;
  uint32_t* h_cln = h_perm + r.L.PWB;
  size_t max_dyn = 0;
  uint32_t max_nb_batch = 1;
  for (uint32_t t = 0; t < T; ++t) max_nb_batch = std::max(max_nb_batch, nbv[t]);
  // Stripe length S: the batch's elements spread over WG_TARGET workgroups
  // (the largest stripe bounds the phase), doubled while the stripes would
  // exceed the batch's workgroup or buffer-slot budget.  At the level's
  // stripe length (which the batch was packed for) both budgets hold.
  uint64_t batch_elems = 0;
  for (uint32_t t = 0; t < T; ++t) batch_elems += bt[t].n;
  const uint64_t S_level = std::max<uint64_t>(1, level_elems / WG_TARGET);
  uint64_t S = std::max<uint64_t>(1, batch_elems / WG_TARGET);
  for (; S < S_level; S *= 2) {
    uint64_t wsum = 0, ssum = 0;
    for (uint32_t t = 0; t < T; ++t) {
      uint64_t W = std::max<uint64_t>(1, (bt[t].n + S / 2) / S);
      W = std::min<uint64_t>(W, std::max<uint64_t>(1, bt[t].n / (4ull * nbv[t] * bvec[t])));
      W = std::min<uint64_t>(W, NBv[t]);
      W = std::min<uint64_t>(W, WG_TARGET);
      wsum += W;
      ssum += W * (((uint64_t)nbv[t] * bvec[t] * c.D + 255) & ~255ull);
    }
    if (wsum <= r.L.WB && ssum <= r.L.SB) break;
  }
  S = std::min(S, S_level);
  for (uint32_t t = 0; t < T; ++t) {
    PTask& p = r.h_tasks[t];
    const uint32_t b = bvec[t], nb = nbv[t], NB = NBv[t];
    p.nb = nb;
    p.K = hdr[t].K;
    p.logK = hdr[t].logK;
    p.eq = hdr[t].eq;
    p.b = b;
    p.NB = NB;
    // About n / S stripes (rounded to the nearest count, so that a batch of
    // equal tasks fills whole rounds of workgroups), but at least four
    // buffer capacities long.
    uint64_t W = std::max<uint64_t>(1, (p.n + S / 2) / S);
    W = std::min<uint64_t>(W, std::max<uint64_t>(1, p.n / (4ull * nb * b)));
    W = std::min<uint64_t>(W, NB);
    W = std::min<uint64_t>(W, WG_TARGET);
    W = std::min<uint64_t>(W, r.L.WB);
    p.W = (uint32_t)W;
    p.wg_base = wg;
    for (uint32_t s = 0; s < p.W; ++s) h_cls[wg + s] = t;
    wg += p.W;
    maxW = std::max(maxW, p.W);
    p.slot_bytes = (uint32_t)(((uint64_t)nb * b * c.D + 255) & ~255ull);
    p.slot_off = slot_off;
    slot_off += (uint64_t)p.W * p.slot_bytes;
    p.spill_off = spill_off;
    spill_off += p.slot_bytes;
    p.piece_base = piece;
    p.piece_cap = 2 * nb + 2 + p.W + NB / c.cmax + 1;   // chunks are never smaller than cmax
    piece += p.piece_cap;
    p.bucket_base = bucket;
    bucket += nb + 1;
    const uint32_t bdw = b * c.DW;
    uint32_t gl = 4;
    while (gl * PERM_RD < bdw) gl *= 2;   // each lane holds up to PERM_RD dwords of the block
    p.glanes = gl;
    uint64_t ng = std::max<uint64_t>(1, std::min<uint64_t>(NB / 4, (uint64_t)c.groups * NB / std::max<uint64_t>(1, blocks_sum)));
    p.ngrp = (uint32_t)ng;
    const uint32_t gpw = c.perm_threads / gl;
    const uint32_t nwg = (uint32_t)((ng + gpw - 1) / gpw);
    p.pwg_base = pwg;
    for (uint32_t x = 0; x < nwg; ++x) h_perm[pwg + x] = t;
    pwg += nwg;
    for (uint32_t j = 0; j < nb; ++j) h_cln[cln++] = (t << 10) | j;
    if (!c.gbuf) max_dyn = std::max<size_t>(max_dyn, (size_t)nb * (b * c.DW + BUF_PAD_DW) * 4);
  }
  if (wg > r.L.WB || pwg > r.L.PWB || slot_off > r.L.SB || spill_off > r.L.SPB || max_nb_batch > r.L.NBS ||
      piece > r.L.PB || bucket > r.L.NBE || cln > r.L.NBE) {
    ctx->last_dev = 0x100;
    return IPS_E_DEVICE;
  }
  // 3. Upload and run the phases.
  HIPCHK(ctx, hipMemcpyAsync(d_tasks, r.h_tasks, T * sizeof(PTask), hipMemcpyHostToDevice, r.st));
  HIPCHK(ctx, hipMemcpyAsync(wsp<uint32_t>(r, R_CLS), h_cls, wg * 4, hipMemcpyHostToDevice, r.st));
  HIPCHK(ctx, hipMemcpyAsync(wsp<uint32_t>(r, R_PERM), h_perm, pwg * 4, hipMemcpyHostToDevice, r.st));
  HIPCHK(ctx, hipMemcpyAsync(wsp<uint32_t>(r, R_CLN), h_cln, cln * 4, hipMemcpyHostToDevice, r.st));
  uint64_t bel = 0;
  for (const HTask& t : bt) bel += t.n;
  const uint32_t row = bt[0].level;
  HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_CLASSIFY, bel,
                    [&] { return c.L->classify(r.a, wg, (uint32_t)max_dyn, c.gbuf, r.st); }));
  HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_BOUNDARIES, bel,
                    [&] { return launch_boundaries(r.a, T, max_nb_batch, c.cmax, r.st); }));
  HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_PERMUTE, bel,
                    [&] { return c.L->permute(r.a, pwg, c.perm_threads, r.st); }));
  HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_CLEANUP_A, bel, [&] { return c.L->cleanup_a(r.a, T, r.st); }));
  HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_CLEANUP_B, bel,
                    [&] { return c.L->cleanup_b(r.a, cln, maxW, r.st); }));
  // 4. Children on the device: LDS-tier task lists and next-level tasks.
  const bool want_root = root_level && T == 1;
  const bool level1 = (c.flags & IPS_FLAG_LEVEL1_ONLY) != 0;
  ChildArgs ca;
  LTask* d_ltc = wsp<LTask>(r, R_LTC);
  for (uint32_t v = 0; v < 3; ++v) {
    ca.lt[v] = d_ltc + (size_t)v * r.L.LTB;
    ca.caps[v] = std::min(c.cap, c.L->lds_caps[v]);
  }
  ca.next = wsp<CTask>(r, R_NEXT);
  ca.lt_cap = r.L.LTB;
  ca.next_cap = r.L.NXB;
  ca.ins_parent = c.insertion ? (uint64_t)c.k * c.n0 : 0;
  CTask* h_next = reinterpret_cast<CTask*>(r.h_rb);
  const uint32_t next_pre = (uint32_t)std::min<size_t>(r.L.NXB, (r.rb_bytes / 2) / sizeof(CTask));
  uint64_t* h_root = reinterpret_cast<uint64_t*>(r.h_rb + r.rb_bytes / 2);
  if (!level1) {
    HIPCHK(ctx, launch_fill32(r.a.ctrl + CTRL_NLDS, 13, 0u, r.st));
    HIPCHK(ctx, launch_children(r.a, ca, T, r.st));
    HIPCHK(ctx, hipMemcpyAsync(h_next, ca.next, (size_t)next_pre * sizeof(CTask), hipMemcpyDeviceToHost, r.st));
  }
  if (want_root) {
    const PTask& p = r.h_tasks[0];
    if ((size_t)(p.nb + 1) * 8 > r.rb_bytes / 2) { ctx->last_dev = 0x101; return IPS_E_DEVICE; }
    HIPCHK(ctx, hipMemcpyAsync(h_root, r.a.b_start + p.bucket_base, (size_t)(p.nb + 1) * 8,
                               hipMemcpyDeviceToHost, r.st));
  }
  if (int e = read_ctrl(r)) return e;
  ctx->stats.steps += T;
  ctx->stats.batches += 1;
  // Root-step description for ips_get_root_info.
  if (want_root) {
    ips_root_info& ri = ctx->root;
    const PTask& p = r.h_tasks[0];
    ri.valid = 1;
    ri.algo = c.radix ? 1 : 0;
    ri.alpha = hdr[0].alpha;
    ri.k_prime = hdr[0].kp;
    ri.m = hdr[0].m;
    ri.u = hdr[0].u;
    ri.K = p.K;
    ri.eq = p.eq;
    ri.nb = p.nb;
    ri.radix_shift = p.shift;
    ri.radix_width = p.width;
    ri.block_elems = p.b;
    ri.stripes = p.W;
    ri.n = p.n;
    for (uint32_t j2 = 0; j2 <= p.nb && j2 < 513; ++j2) ri.bucket_start[j2] = h_root[j2];
    if (!c.radix) {
      std::vector<uint64_t> spl((size_t)p.K * 3);
      HIPCHK(ctx, hipMemcpy(spl.data(), &d_recs[0].spl[0][0], spl.size() * 8, hipMemcpyDeviceToHost));
      for (uint32_t q = 0; q < p.K && q < 256; ++q) {
        uint64_t k0 = spl[3 * q], k1 = spl[3 * q + 1];
        if (c.type == 3) k0 = (k0 >> 63) ? (k0 & ~(1ull << 63)) : ~k0;   // ordered image -> bits
        if (c.type == 5) {
          uint8_t* d = ri.splitters[q];
          for (int x = 0; x < 8; ++x) d[x] = (uint8_t)(k0 >> (56 - 8 * x));
          d[8] = (uint8_t)(k1 >> 8);
          d[9] = (uint8_t)k1;
        } else if (c.type == 6) {   // the Quartet's first two key words (a, b)
          std::memcpy(ri.splitters[q], &k0, 8);
          std::memcpy(ri.splitters[q] + 8, &k1, 8);
        } else {
          std::memcpy(ri.splitters[q], &k0, 8);
        }
      }
    }
  }
  if (level1) return IPS_OK;
  for (uint32_t t = 0; t < T; ++t) {
    ctx->stats.partitioned_elems += r.h_tasks[t].n;
    ctx->stats.max_step_elems = std::max<uint64_t>(ctx->stats.max_step_elems, r.h_tasks[t].n);
  }
  // 5. Next-level tasks (read back beyond the first part if there are many),
  // in a fixed order, and the LDS tier on the device lists.
  const uint32_t nnext = r.h_ctrl[CTRL_NNEXT];
  const uint32_t nlds[3] = {r.h_ctrl[CTRL_NLDS], r.h_ctrl[CTRL_NLDS + 1], r.h_ctrl[CTRL_NLDS + 2]};
  uint64_t lel[3];
  for (uint32_t v = 0; v < 3; ++v) {
    lel[v] = (uint64_t)r.h_ctrl[CTRL_LDSEL + 2 * v] | ((uint64_t)r.h_ctrl[CTRL_LDSEL + 2 * v + 1] << 32);
    ctx->stats.lds_elems += lel[v];
  }
  if (nnext > r.L.NXB || nlds[0] > r.L.LTB || nlds[1] > r.L.LTB || nlds[2] > r.L.LTB) {
    ctx->last_dev = 0x102;
    return IPS_E_DEVICE;
  }
  HIPCHK(ctx, launch_lds_lists(r, ca, nlds, lel, bt[0].level));
  std::vector<CTask> ch(nnext);
  const uint32_t first = std::min(nnext, next_pre);
  if (first) std::memcpy(ch.data(), h_next, (size_t)first * sizeof(CTask));
  for (uint32_t done = first; done < nnext;) {
    const uint32_t cnt = std::min(nnext - done, next_pre);
    HIPCHK(ctx, hipMemcpyAsync(h_next, ca.next + done, (size_t)cnt * sizeof(CTask), hipMemcpyDeviceToHost, r.st));
    HIPCHK(ctx, hipStreamSynchronize(r.st));
    std::memcpy(ch.data() + done, h_next, (size_t)cnt * sizeof(CTask));
    done += cnt;
  }
  std::sort(ch.begin(), ch.end(), [](const CTask& x, const CTask& y) { return x.l < y.l; });
  for (const CTask& q : ch) {
    HTask h;
    h.l = q.l;
    h.n = q.n;
    h.level = q.level;
    h.tflags = q.tflags;
    h.shift = q.shift;
    h.width = q.width;
    next.push_back(h);
  }
  return IPS_OK;
}

// Extra areas of a segmented call, in the workspace and in pinned host
// memory alike: chunk descriptors of the partitioned segments, their order
// flags, their radix key ranges and the reversal chunks.
struct SegAreas {
  uint64_t items_ub, rev_ub;
  size_t o_items, o_flags, o_min, o_max, o_rev, total;
};

SegAreas seg_areas(const Cfg& c, uint64_t n, uint64_t nseg) {
  SegAreas s;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  s.items_ub = n / SEG_CHUNK + nseg;
  s.rev_ub = n / (2 * SEG_CHUNK) + nseg;
  s.o_items = 0;
  s.o_flags = al(s.items_ub * sizeof(SegItem));
  s.o_min = s.o_flags + al(nseg * 8);
  s.o_max = s.o_min + (c.radix ? al(nseg * 8) : 0);
  s.o_rev = s.o_max + (c.radix ? al(nseg * 8) : 0);
  s.total = s.o_rev + al(s.rev_ub * sizeof(RevItem));
  return s;
}

size_t seg_extra_bytes(const Cfg& c, uint64_t n_total, uint64_t nseg) {
  return nseg ? seg_areas(c, n_total, nseg).total : 0;
}

// Validation, workspace plan, pinned staging and device views shared by
// every sort entry point.  n is the length of the data array, n_plan the
// number of elements to be sorted (the workspace is planned for n_plan).
// `extra_pin` bytes of pinned memory are reserved after the common staging
// areas (returned in *extra).
int setup_run(ips_ctx* ctx, Run& r, void* d, uint64_t n, uint64_t n_plan, int type, int algo,
              void* ws, size_t ws_bytes, size_t ws_extra, const ips_params* params, void* stream,
              size_t extra_pin, uint8_t** extra) {
  if (!ctx) return IPS_E_INVALID_ARG;
  std::memset(&r.a, 0, sizeof(r.a));
  int rc = make_cfg(n, type, algo, params, &r.c);
  if (rc) return rc;
  if (n > 0 && !d) return IPS_E_INVALID_ARG;
  const uint32_t align = (type == 1 || type == 5) ? 4 : 8;
  if (reinterpret_cast<uintptr_t>(d) % align) return IPS_E_MISALIGNED;
  if (n >= (1ull << 31) * (uint64_t)block_elems(r.c, max_nb(r.c))) return IPS_E_TOO_LARGE;
  std::memset(&ctx->root, 0, sizeof(ctx->root));
  std::memset(&ctx->stats, 0, sizeof(ctx->stats));
  std::memset(&ctx->prof, 0, sizeof(ctx->prof));
  for (const auto& p : ctx->pending) { ctx->ev_pool.push_back(p.a); ctx->ev_pool.push_back(p.b); }
  ctx->pending.clear();
  ctx->profiling = (r.c.flags & IPS_FLAG_PROFILE) != 0;
  ctx->profile_mask = params ? params->profile_mask : 0u;
  ctx->last_dev = 0;
  r.ctx = ctx;
  r.n = n;
  if (n < 2 || n_plan < 2) return IPS_OK;
  plan(n_plan, r.c, &r.L);
  if (!ws) return IPS_E_INVALID_ARG;
  if (ws_bytes < r.L.total + ws_extra) return IPS_E_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(ws) % 256) return IPS_E_MISALIGNED;
  r.c.L = launchers_for(type);
  r.ws = static_cast<uint8_t*>(ws);
  r.data = static_cast<uint32_t*>(d);
  r.st = static_cast<hipStream_t>(stream);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  // Pinned staging: tasks | maps | LDS tasks | readback | ctrl | extra.
  const size_t b_tasks = (size_t)r.L.TB * sizeof(PTask);
  const size_t b_maps = ((size_t)r.L.WB + r.L.PWB + (size_t)r.L.NBE) * 4;
  const size_t b_lt = (size_t)r.L.LTB * sizeof(LTask);
  // readback: sampling headers, or next-level tasks (first half) and the
  // root step's bucket starts (second half)
  const size_t b_rb = std::max<size_t>((size_t)r.L.TB * 64, 2 * 4096 * sizeof(CTask)) + 8192;
  const size_t b_ctrl = CTRL_WORDS * 4;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  if (int e = ensure_pinned(ctx, al(b_tasks) + al(b_maps) + al(b_lt) + al(b_rb) + al(b_ctrl) + al(extra_pin)))
    return e;
  uint8_t* pp = ctx->pin;
  r.h_tasks = reinterpret_cast<PTask*>(pp); pp += al(b_tasks);
  r.h_maps = reinterpret_cast<uint32_t*>(pp); pp += al(b_maps);
  r.h_lt = reinterpret_cast<LTask*>(pp); pp += al(b_lt);
  r.h_rb = pp; r.rb_bytes = b_rb; pp += al(b_rb);
  r.h_ctrl = reinterpret_cast<uint32_t*>(pp); pp += al(b_ctrl);
  if (extra) *extra = pp;
  // Device views of the workspace.
  BatchArgs& a = r.a;
  a.data = r.data;
  a.ctrl = wsp<uint32_t>(r, R_CTRL);
  a.tasks = wsp<PTask>(r, R_TASKS);
  a.recs = wsp<StepRec>(r, R_RECS);
  a.cls_task = wsp<uint32_t>(r, R_CLS);
  a.perm_task = wsp<uint32_t>(r, R_PERM);
  a.cln_map = wsp<uint32_t>(r, R_CLN);
  a.wg_nfull = wsp<uint32_t>(r, R_NFULL);
  a.wg_left = wsp<uint32_t>(r, R_LEFT);
  a.wg_F = wsp<uint32_t>(r, R_F);
  a.wg_min = wsp<uint64_t>(r, R_WMIN);
  a.wg_max = wsp<uint64_t>(r, R_WMAX);
  a.slots = wsp<uint8_t>(r, R_SLOTS);
  a.spill = wsp<uint8_t>(r, R_SPILL);
  a.ovf = wsp<uint32_t>(r, R_OVF);
  a.nbs = r.L.NBS;
  a.b_start = wsp<uint64_t>(r, R_BSTART);
  a.b_count = wsp<uint32_t>(r, R_BCOUNT);
  a.b_d = wsp<uint32_t>(r, R_BD);
  a.b_plb = wsp<uint32_t>(r, R_BPLB);
  a.b_ple = wsp<uint32_t>(r, R_BPLE);
  a.b_min = wsp<uint64_t>(r, R_BMIN);
  a.b_max = wsp<uint64_t>(r, R_BMAX);
  a.b_full = wsp<uint64_t>(r, R_BFULL);
  a.p_word = wsp<uint64_t>(r, R_PWORD);
  a.p_a = wsp<uint32_t>(r, R_PA);
  a.p_c = wsp<uint32_t>(r, R_PC);
  a.p_rinit = wsp<int32_t>(r, R_PR);
  a.p_cum = wsp<uint32_t>(r, R_PCUM);
  a.p_fcnt = wsp<uint32_t>(r, R_PFCNT);
  a.t_npieces = wsp<uint32_t>(r, R_TNP);
  a.t_unproc = wsp<uint32_t>(r, R_TUP);
  a.gbuf = r.c.gbuf ? 1 : 0;
  a.queue = wsp<CTask>(r, R_QUEUE);
  a.qcap = r.L.QCAP;
  a.devplan = 0;
  a.step = 0;
  a.step_el = wsp<uint64_t>(r, R_STEPEL);
  // Control block: errors and flags cleared; min = all ones, max = 0.
  HIPCHK(ctx, launch_fill32(a.ctrl, CTRL_WORDS, 0u, r.st));
  // Fused radix steps add their histograms to the bucket counters (each
  // step zeroes the counters it used).
  if (r.c.fused) HIPCHK(ctx, launch_fill32(a.b_count, r.L.NBE, 0u, r.st));
  HIPCHK(ctx, launch_fill32(a.ctrl + CTRL_MINMAX, 2, 0xFFFFFFFFu, r.st));
  return IPS_OK;
}

// Root task of a partitioned range, with the radix digit below the highest
// bit in which its smallest and largest keys differ.  Returns false when
// all keys are equal (radix: nothing to do).
bool make_root(const Cfg& c, uint64_t l, uint64_t n, uint64_t mn, uint64_t mx, HTask* t) {
  t->l = l;
  t->n = n;
  t->level = 0;
  t->tflags = 0;
  t->shift = 0;
  t->width = 0;
  if (c.flags & IPS_FLAG_EQ_ON) t->tflags |= TF_EQ_ON;
  if (c.flags & IPS_FLAG_EQ_OFF) t->tflags |= TF_EQ_OFF;
  if (!(c.flags & IPS_FLAG_PAPER_ROOT_ALPHA)) t->tflags |= TF_ROOT_ALPHA;
  if (c.radix) {
    if (mn == mx) return false;
    const uint32_t h = 63u - (uint32_t)__builtin_clzll(mn ^ mx);
    t->shift = h >= 7 ? h - 7 : 0;
    t->width = h - t->shift + 1;
  }
  return true;
}

// Breadth-first recursion (Section 4.2) from the given partitioning roots
// and LDS-tier roots: every level's tasks run in as few batches as the
// workspace allows.
int level_loop(Run& r, std::vector<HTask> cur, const std::vector<LTask>& lds_roots, bool record_root) {
  ips_ctx* ctx = r.ctx;
  if (!lds_roots.empty()) {
    for (const LTask& t : lds_roots) ctx->stats.lds_elems += t.n;
    if (int e = launch_lds_tasks(r, lds_roots, record_root ? IPS_MAX_LEVELS : 0)) return e;
  }
  std::vector<HTask> next;
  uint32_t level = 0;
  while (!cur.empty()) {
    uint64_t level_elems = 0;
    for (const HTask& t : cur) level_elems += t.n;
    next.clear();
    size_t i = 0;
    while (i < cur.size()) {
      std::vector<HTask> bt;
      Need tot{0, 0, 0, 0};
      while (i < cur.size() && bt.size() < r.L.TB) {
        Need nd = task_need(r, cur[i], level_elems);
        if (!bt.empty() && (tot.wg + nd.wg > r.L.WB || tot.slot + nd.slot > r.L.SB ||
                            tot.spill + nd.spill > r.L.SPB || tot.pieces + nd.pieces > r.L.PB))
          break;
        tot.wg += nd.wg; tot.slot += nd.slot; tot.spill += nd.spill;
        tot.pieces += nd.pieces;
        bt.push_back(cur[i++]);
      }
      if (int e = run_batch(r, bt, level_elems, next, record_root && level == 0)) return e;
      if (r.c.flags & IPS_FLAG_LEVEL1_ONLY) return IPS_OK;
    }
    ctx->stats.levels = ++level;
    ctx->prof.levels = std::min<uint32_t>(level, IPS_MAX_LEVELS);
    std::swap(cur, next);
  }
  return read_ctrl(r);
}

// Device-planned execution (the same steps as level_loop, planned on the
// device): the roots go into a task queue in the workspace; each step takes
// the next batch from the queue, partitions it, pushes its large buckets
// back onto the queue and sorts its small ones in the LDS tier.  The host
// enqueues several steps at a time and only reads the queue state between
// rounds of steps; with IPS_FLAG_GRAPH a round is captured once as a HIP
// graph and replayed.
int enqueue_step(Run& r, const PlanCfg& pc, const ChildArgs& ca, uint32_t step) {
  ips_ctx* ctx = r.ctx;
  const Cfg& c = r.c;
  BatchArgs a = r.a;
  a.devplan = 1;
  a.step = step;
  const uint32_t row = std::min<uint32_t>(step, IPS_MAX_LEVELS - 1);
  const uint32_t nbm = r.L.NBS;
  HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_SAMPLE, 0, [&] {
           hipError_t e = launch_plan_pop(a, pc, r.st);
           if (e != hipSuccess || c.radix) return e;
           return c.L->sample(a, r.L.TB, c.seed, r.st);
         }, 0));
  HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_FLAGS, 0, [&] { return launch_plan_geom(a, pc, r.st); }, 0));
  const size_t dyn = c.gbuf ? 0 : (size_t)c.buf_bytes + (size_t)MAX_NB * BUF_PAD_DW * 4;
  if (c.fused) {
    // exact bucket sizes, then classification fused with the permutation
    HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_HISTOGRAM, 0, [&] { return c.L->fhist(a, r.L.WB, r.st); }, 0));
    HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_BOUNDARIES, 0, [&] { return launch_fscan(a, r.L.TB, r.st); }, 0));
    const size_t fdyn = (size_t)c.buf_bytes + (size_t)MAX_K * BUF_PAD_DW * 4;
    HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_FUSED, 0,
                      [&] { return c.L->fused(a, r.L.WB, (uint32_t)fdyn, r.st); }, 0));
  } else {
    HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_CLASSIFY, 0,
                      [&] { return c.L->classify(a, r.L.WB, (uint32_t)dyn, c.gbuf, r.st); }, 0));
    HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_BOUNDARIES, 0,
                      [&] { return launch_boundaries(a, r.L.TB, nbm, c.cmax, r.st); }, 0));
    HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_PERMUTE, 0,
                      [&] { return c.L->permute(a, r.L.PWB, c.perm_threads, r.st); }, 0));
    HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_CLEANUP_A, 0, [&] { return c.L->cleanup_a(a, r.L.TB, r.st); }, 0));
    const uint32_t cln_grid = (uint32_t)std::min<uint64_t>((uint64_t)r.L.TB * nbm, 16384);
    HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_CLEANUP_B, 0,
                      [&] { return c.L->cleanup_b(a, cln_grid, r.L.WB, r.st); }, 0));
  }
  HIPCHK(ctx, launch_children(a, ca, r.L.TB, r.st));
  HIPCHK(ctx, launch_lds_decide(a.ctrl, r.lds_min, r.L.LTB, r.st));
  for (uint32_t v = 0; v < 3; ++v) {
    if (v && (c.insertion || c.L->lds_caps[v] == c.L->lds_caps[v - 1])) continue;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(ca.lt_cap, c.insertion ? (uint64_t)ca.lt_cap : 2048);
    HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_LDS_SORT, 0, [&] {
             return c.L->lds_sort(ca.lt[v], grid, r.data, c.insertion ? LDS_INSERTION : v, a.ctrl,
                                  a.ctrl + CTRL_NLDS + v, ca.lt_cap, r.st);
           }, 1 + (int)v));
  }
  HIPCHK(ctx, launch_lds_reset(a.ctrl, r.st));
  return IPS_OK;
}

// Budgets of the device planner and the children lists of device-planned
// steps (lists of two steps' capacity).
void plan_cfg(const Run& r, PlanCfg* pcp, ChildArgs* cap) {
  const Cfg& c = r.c;
  PlanCfg& pc = *pcp;
  pc.SB = r.L.SB; pc.SPB = r.L.SPB; pc.PB = r.L.PB; pc.slot_max = r.L.slot_max;
  pc.TB = r.L.TB; pc.WB = r.L.WB; pc.PWB = r.L.PWB; pc.NBE = r.L.NBE; pc.QCAP = r.L.QCAP;
  pc.CLNB = r.L.NBE;
  pc.D = c.D; pc.DW = c.DW; pc.k = c.k; pc.k_root = c.k_root; pc.n0 = c.n0; pc.cap = c.cap; pc.cmax = c.cmax;
  pc.groups = c.groups; pc.b_req = c.b_req; pc.gbuf = c.gbuf ? 1 : 0; pc.radix = c.radix ? 1 : 0;
  pc.tflags0 = 0; pc.wg_target = WG_TARGET; pc.perm_threads = c.perm_threads; pc.buf_bytes = c.buf_bytes;
  ChildArgs& ca = *cap;
  LTask* d_ltc = reinterpret_cast<LTask*>(r.ws + r.L.off[R_LTC]);
  for (uint32_t v = 0; v < 3; ++v) {
    ca.lt[v] = d_ltc + (size_t)v * 2 * r.L.LTB;
    ca.caps[v] = std::min(c.cap, c.L->lds_caps[v]);
  }
  ca.next = reinterpret_cast<CTask*>(r.ws + r.L.off[R_NEXT]);
  ca.lt_cap = 2 * r.L.LTB;
  ca.next_cap = r.L.NXB;
  ca.ins_parent = c.insertion ? (uint64_t)c.k * c.n0 : 0;
}

int device_loop(Run& r, const std::vector<HTask>& roots, const std::vector<LTask>& lds_roots) {
  ips_ctx* ctx = r.ctx;
  const Cfg& c = r.c;
  if (!lds_roots.empty()) {
    for (const LTask& t : lds_roots) ctx->stats.lds_elems += t.n;
    if (int e = launch_lds_tasks(r, lds_roots, 0)) return e;
  }
  if (roots.empty()) return read_ctrl(r);
  if (roots.size() > r.L.QCAP) { ctx->last_dev = 0x103; return IPS_E_DEVICE; }
  // Roots onto the queue (through the readback staging area, in chunks).
  CTask* h = reinterpret_cast<CTask*>(r.h_rb);
  const size_t chunk = r.rb_bytes / sizeof(CTask);
  for (size_t done = 0; done < roots.size();) {
    const size_t cnt = std::min(chunk, roots.size() - done);
    for (size_t i = 0; i < cnt; ++i) {
      const HTask& t = roots[done + i];
      h[i].l = t.l; h[i].n = t.n; h[i].level = t.level; h[i].tflags = t.tflags;
      h[i].shift = t.shift; h[i].width = t.width;
    }
    HIPCHK(ctx, hipMemcpyAsync(r.a.queue + done, h, cnt * sizeof(CTask), hipMemcpyHostToDevice, r.st));
    HIPCHK(ctx, hipStreamSynchronize(r.st));
    done += cnt;
  }
  HIPCHK(ctx, launch_fill32(r.a.ctrl + CTRL_QHEAD, 1, 0u, r.st));
  HIPCHK(ctx, launch_fill32(r.a.ctrl + CTRL_QTAIL, 1, (uint32_t)roots.size(), r.st));
  HIPCHK(ctx, launch_fill32(reinterpret_cast<uint32_t*>(r.a.step_el), MAX_STEPS_RECORDED * 8, 0u, r.st));
  PlanCfg pc;
  ChildArgs ca;
  plan_cfg(r, &pc, &ca);
  HIPCHK(ctx, launch_fill32(r.a.ctrl + CTRL_NLDS, 14, 0u, r.st));   // lists empty, no run pending
  const bool graph = (c.flags & IPS_FLAG_GRAPH) != 0;
  if (graph) ctx->profiling = false;   // no event records inside a captured graph
  uint64_t* h_sel = reinterpret_cast<uint64_t*>(r.h_rb);
  // Rounds of steps between readbacks: one step first (a small sort is done
  // after its root step, and steps beyond the work cost their launches),
  // then doubling to 32; a captured graph holds 4 steps.
  uint32_t step = 0, round_steps = graph ? 4u : 1u;
  hipGraphExec_t exec = nullptr;
  int rc = IPS_OK;
  for (uint32_t round = 0;; ++round) {
    if (graph) {
      if (!exec) {   // one round of steps, captured once and replayed
        hipGraph_t g = nullptr;
        HIPCHK(ctx, hipStreamBeginCapture(r.st, hipStreamCaptureModeThreadLocal));
        int e = IPS_OK;
        for (uint32_t s = 0; s < round_steps && e == IPS_OK; ++s) e = enqueue_step(r, pc, ca, MAX_STEPS_RECORDED);
        hipError_t ce = hipStreamEndCapture(r.st, &g);
        if (e != IPS_OK) { if (g) (void)hipGraphDestroy(g); return e; }
        if (ce != hipSuccess) { ctx->last_hip = (int)ce; return IPS_E_HIP; }
        hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) { ctx->last_hip = (int)ie; return IPS_E_HIP; }
      }
      hipError_t le = hipGraphLaunch(exec, r.st);
      if (le != hipSuccess) { ctx->last_hip = (int)le; rc = IPS_E_HIP; break; }
      step += round_steps;
    } else {
      for (uint32_t s = 0; s < round_steps; ++s, ++step)
        if (int e = enqueue_step(r, pc, ca, step)) return e;
    }
    hipError_t e1 = hipMemcpyAsync(r.h_ctrl, r.a.ctrl, CTRL_WORDS * 4, hipMemcpyDeviceToHost, r.st);
    hipError_t e2 = hipMemcpyAsync(h_sel, r.a.step_el, MAX_STEPS_RECORDED * 32, hipMemcpyDeviceToHost, r.st);
    hipError_t e3 = hipStreamSynchronize(r.st);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
      ctx->last_hip = (int)(e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3);
      rc = IPS_E_HIP;
      break;
    }
    for (auto& pe : ctx->pending)
      if (pe.src >= 0 && pe.row < MAX_STEPS_RECORDED) pe.elems = h_sel[pe.row * 4 + pe.src];
    resolve_profile(ctx);
    if ((rc = check_dev_error(r)) != IPS_OK) break;
    if (r.h_ctrl[CTRL_QHEAD] == r.h_ctrl[CTRL_QTAIL]) break;
    if (!graph) round_steps = std::min<uint32_t>(round_steps * 2, 32);
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (rc != IPS_OK) return rc;
  ips_stats& st = ctx->stats;
  auto u64at = [&](uint32_t w) { return (uint64_t)r.h_ctrl[w] | ((uint64_t)r.h_ctrl[w + 1] << 32); };
  st.steps += r.h_ctrl[CTRL_STEPS];
  st.batches += r.h_ctrl[CTRL_BATCHES];
  st.levels = std::max<uint32_t>(st.levels, r.h_ctrl[CTRL_LEVELS]);
  st.lds_tasks += r.h_ctrl[CTRL_LDSTASKS];
  st.partitioned_elems += u64at(CTRL_PARTEL);
  st.lds_elems += u64at(CTRL_LDSELT);
  st.max_step_elems = std::max<uint64_t>(st.max_step_elems, u64at(CTRL_MAXSTEP));
  ctx->prof.levels = std::min<uint32_t>(std::min<uint32_t>(step, IPS_MAX_LEVELS), st.levels);
  return IPS_OK;
}

int sort_impl(ips_ctx* ctx, void* d, uint64_t n, int type, int algo, void* ws, size_t ws_bytes,
              const ips_params* params, void* stream) {
  Run r;
  int rc = setup_run(ctx, r, d, n, n, type, algo, ws, ws_bytes, 0, params, stream, 0, nullptr);
  if (rc || n < 2) return rc;
  BatchArgs& a = r.a;
  // Sorted and reverse-sorted inputs (Section 6).
  if (!(r.c.flags & (IPS_FLAG_NO_SORTED_CHECK | IPS_FLAG_LEVEL1_ONLY))) {
    HIPCHK(ctx, timed(ctx, r.st, IPS_MAX_LEVELS, IPS_PH_SORTED_CHECK, n,
                      [&] { return r.c.L->sorted_sample(r.data, n, a.ctrl, r.st); }));
    if (int e = read_ctrl(r)) return e;
    if (!r.h_ctrl[CTRL_DESC] || !r.h_ctrl[CTRL_ASC]) {   // inconclusive: scan everything
      HIPCHK(ctx, timed(ctx, r.st, IPS_MAX_LEVELS, IPS_PH_SORTED_CHECK, n,
                        [&] { return r.c.L->sorted_check(r.data, n, a.ctrl, r.st); }));
      if (int e = read_ctrl(r)) return e;
    }
    if (!r.h_ctrl[CTRL_DESC]) { ctx->stats.detected = 1; return IPS_OK; }
    if (!r.h_ctrl[CTRL_ASC]) {
      ctx->stats.detected = 2;
      HIPCHK(ctx, timed(ctx, r.st, IPS_MAX_LEVELS, IPS_PH_REVERSE, n,
                        [&] { return r.c.L->reverse(r.data, n, r.st); }));
      return read_ctrl(r);
    }
  }
  uint64_t mn = 0, mx = 0;
  if (r.c.radix) {
    HIPCHK(ctx, timed(ctx, r.st, IPS_MAX_LEVELS, IPS_PH_MINMAX, n,
                      [&] { return r.c.L->minmax(r.data, n, a.ctrl, r.st); }));
    if (int e = read_ctrl(r)) return e;
    mn = (uint64_t)r.h_ctrl[CTRL_MINMAX] | ((uint64_t)r.h_ctrl[CTRL_MINMAX + 1] << 32);
    mx = (uint64_t)r.h_ctrl[CTRL_MINMAX + 2] | ((uint64_t)r.h_ctrl[CTRL_MINMAX + 3] << 32);
  }
  HTask root;
  if (!make_root(r.c, 0, n, mn, mx, &root)) return IPS_OK;
  if (n <= r.c.cap && !(r.c.flags & IPS_FLAG_LEVEL1_ONLY)) {
    std::vector<LTask> lt(1);
    lt[0].l = 0;
    lt[0].n = (uint32_t)n;
    lt[0].req = 0;
    return level_loop(r, {}, lt, true);
  }
  if (r.c.flags & (IPS_FLAG_LEVEL1_ONLY | IPS_FLAG_HOST_PLAN))
    return level_loop(r, std::vector<HTask>(1, root), {}, true);
  return device_loop(r, std::vector<HTask>(1, root), {});
}

// Checks a segment list against the data length: every segment inside
// [0, n_total) and no two overlapping.  Returns the sum of the lengths.
int check_segments(const ips_segment* segs, uint32_t nseg, uint64_t n_total, uint64_t* sum) {
  *sum = 0;
  if (nseg && !segs) return IPS_E_INVALID_ARG;
  std::vector<uint32_t> ord(nseg);
  for (uint32_t i = 0; i < nseg; ++i) {
    if (segs[i].offset > n_total || segs[i].n > n_total - segs[i].offset) return IPS_E_INVALID_ARG;
    ord[i] = i;
    *sum += segs[i].n;
  }
  std::sort(ord.begin(), ord.end(),
            [&](uint32_t x, uint32_t y) { return segs[x].offset < segs[y].offset; });
  for (uint32_t i = 1; i < nseg; ++i) {
    const ips_segment& p = segs[ord[i - 1]];
    if (p.n && segs[ord[i]].n && p.offset + p.n > segs[ord[i]].offset) return IPS_E_INVALID_ARG;
  }
  return IPS_OK;
}

// Workspace of a segmented call: planned for the sum of the segment
// lengths, plus the radix key-range area of the partitioned segments.
int segments_ws(uint64_t sum, const ips_segment* segs, uint32_t nseg, int type, int algo,
                const ips_params* params, size_t* out) {
  *out = 0;
  Cfg c;
  if (int e = make_cfg(sum, type, algo, params, &c)) return e;
  if (sum >= (1ull << 31) * (uint64_t)block_elems(c, max_nb(c))) return IPS_E_TOO_LARGE;
  if (sum < 2) return IPS_OK;
  Layout L;
  plan(sum, c, &L);
  uint64_t big = 0, big_elems = 0;
  for (uint32_t i = 0; i < nseg; ++i)
    if (segs[i].n > c.cap) { ++big; big_elems += segs[i].n; }
  *out = L.total + seg_extra_bytes(c, big_elems, big);
  return IPS_OK;
}

// Sorts the (validated, non-overlapping) segments of the array at d.
int segments_impl(ips_ctx* ctx, void* d, uint64_t n_total, int type, int algo,
                  const ips_segment* segs, uint32_t nseg, void* ws, size_t ws_bytes,
                  const ips_params* params, void* stream) {
  if (!ctx) return IPS_E_INVALID_ARG;
  if (params && (params->flags & IPS_FLAG_LEVEL1_ONLY)) return IPS_E_INVALID_ARG;
  uint64_t sum = 0;
  if (int e = check_segments(segs, nseg, n_total, &sum)) return e;
  Cfg c0;
  if (int e = make_cfg(sum, type, algo, params, &c0)) return e;
  // Segments that are partitioned (larger than the LDS tier).
  std::vector<uint32_t> big;
  uint64_t big_elems = 0;
  for (uint32_t i = 0; i < nseg; ++i)
    if (segs[i].n > c0.cap) { big.push_back(i); big_elems += segs[i].n; }
  const SegAreas sa = seg_areas(c0, big_elems, big.size());
  const size_t extra = seg_extra_bytes(c0, big_elems, big.size());
  Run r;
  uint8_t* hx = nullptr;
  int rc = setup_run(ctx, r, d, n_total, sum, type, algo, ws, ws_bytes, extra, params, stream,
                     big.empty() ? 0 : sa.total, &hx);
  if (rc || n_total < 2 || sum < 2) return rc;
  std::vector<HTask> roots;
  std::vector<LTask> lt;
  for (uint32_t i = 0; i < nseg; ++i) {
    if (segs[i].n < 2 || segs[i].n > r.c.cap) continue;
    LTask q;
    q.l = segs[i].offset;
    q.n = (uint32_t)segs[i].n;
    q.req = 0;
    lt.push_back(q);
  }
  const bool check = !(r.c.flags & IPS_FLAG_NO_SORTED_CHECK);
  std::vector<uint64_t> mn(big.size(), 0), mx(big.size(), 1);
  std::vector<char> finished(big.size(), 0);
  const uint32_t nbig = (uint32_t)big.size();
  if (nbig && (check || r.c.radix)) {
    // Order flags and key ranges of the partitioned segments.
    uint8_t* wx = r.ws + r.L.total;
    SegItem* h_items = reinterpret_cast<SegItem*>(hx + sa.o_items);
    uint32_t* h_flags = reinterpret_cast<uint32_t*>(hx + sa.o_flags);
    uint64_t* h_min = reinterpret_cast<uint64_t*>(hx + sa.o_min);
    uint64_t* h_max = reinterpret_cast<uint64_t*>(hx + sa.o_max);
    SegItem* d_items = reinterpret_cast<SegItem*>(wx + sa.o_items);
    uint32_t* d_flags = reinterpret_cast<uint32_t*>(wx + sa.o_flags);
    uint64_t* d_min = reinterpret_cast<uint64_t*>(wx + sa.o_min);
    uint64_t* d_max = reinterpret_cast<uint64_t*>(wx + sa.o_max);
    uint64_t ni = 0;
    for (uint32_t q = 0; q < nbig; ++q) {
      const ips_segment& sg = segs[big[q]];
      for (uint64_t o = 0; o < sg.n; o += SEG_CHUNK) {
        SegItem it;
        it.l = sg.offset + o;
        it.n = (uint32_t)std::min<uint64_t>(SEG_CHUNK, sg.n - o);
        it.seg = q;
        it.first = o == 0 ? 1u : 0u;
        it.pad = 0;
        h_items[ni++] = it;
      }
    }
    HIPCHK(ctx, hipMemcpyAsync(d_items, h_items, ni * sizeof(SegItem), hipMemcpyHostToDevice, r.st));
    if (check) {
      HIPCHK(ctx, launch_fill32(d_flags, 2 * nbig, 0u, r.st));
      HIPCHK(ctx, timed(ctx, r.st, IPS_MAX_LEVELS, IPS_PH_SORTED_CHECK, big_elems, [&] {
               return r.c.L->seg_order(d_items, (uint32_t)ni, r.data, d_flags, r.st);
             }));
      HIPCHK(ctx, hipMemcpyAsync(h_flags, d_flags, 2 * nbig * 4, hipMemcpyDeviceToHost, r.st));
    }
    if (r.c.radix) {
      HIPCHK(ctx, launch_fill32(reinterpret_cast<uint32_t*>(d_min), 2 * nbig, 0xFFFFFFFFu, r.st));
      HIPCHK(ctx, launch_fill32(reinterpret_cast<uint32_t*>(d_max), 2 * nbig, 0u, r.st));
      HIPCHK(ctx, timed(ctx, r.st, IPS_MAX_LEVELS, IPS_PH_MINMAX, big_elems, [&] {
               return r.c.L->seg_minmax(d_items, (uint32_t)ni, r.data, d_min, d_max, r.st);
             }));
      HIPCHK(ctx, hipMemcpyAsync(h_min, d_min, nbig * 8, hipMemcpyDeviceToHost, r.st));
      HIPCHK(ctx, hipMemcpyAsync(h_max, d_max, nbig * 8, hipMemcpyDeviceToHost, r.st));
    }
    if (int e = read_ctrl(r)) return e;
    if (r.c.radix)
      for (uint32_t q = 0; q < nbig; ++q) { mn[q] = h_min[q]; mx[q] = h_max[q]; }
    if (check) {
      // Sorted segments are done; reverse-sorted ones are reversed in place.
      RevItem* h_rev = reinterpret_cast<RevItem*>(hx + sa.o_rev);
      RevItem* d_rev = reinterpret_cast<RevItem*>(wx + sa.o_rev);
      uint64_t nr = 0;
      for (uint32_t q = 0; q < nbig; ++q) {
        if (!h_flags[2 * q]) { finished[q] = 1; continue; }
        if (h_flags[2 * q + 1]) continue;
        finished[q] = 1;
        const ips_segment& sg = segs[big[q]];
        for (uint64_t o = 0; o < sg.n / 2; o += SEG_CHUNK) {
          RevItem it;
          it.l = sg.offset;
          it.len = sg.n;
          it.c0 = o;
          it.cn = (uint32_t)std::min<uint64_t>(SEG_CHUNK, sg.n / 2 - o);
          it.pad = 0;
          h_rev[nr++] = it;
        }
      }
      if (nr) {
        HIPCHK(ctx, hipMemcpyAsync(d_rev, h_rev, nr * sizeof(RevItem), hipMemcpyHostToDevice, r.st));
        HIPCHK(ctx, timed(ctx, r.st, IPS_MAX_LEVELS, IPS_PH_REVERSE, big_elems, [&] {
                 return r.c.L->seg_reverse(d_rev, (uint32_t)nr, r.data, r.st);
               }));
      }
    }
  }
  for (uint32_t q = 0; q < nbig; ++q) {
    HTask t;
    if (finished[q]) continue;
    if (make_root(r.c, segs[big[q]].offset, segs[big[q]].n, mn[q], mx[q], &t)) roots.push_back(t);
  }
  if (r.c.flags & IPS_FLAG_HOST_PLAN) return level_loop(r, roots, lt, false);
  return device_loop(r, roots, lt);
}

// Requests in separate device buffers: those whose addresses are congruent
// modulo the element size share a base pointer and become segments of one
// call.  Each group's workspace is planned separately; the largest is
// returned.
struct PtrGroup {
  uintptr_t base;
  uint64_t span;
  std::vector<ips_segment> segs;
};

int group_batch(void* const* ptrs, const uint64_t* ns, uint32_t count, int type,
                std::vector<PtrGroup>* groups) {
  groups->clear();
  if (count && (!ptrs || !ns)) return IPS_E_INVALID_ARG;
  const uint32_t D = elem_bytes(type);
  if (!D) return IPS_E_INVALID_ARG;
  const uint32_t align = (type == 1 || type == 5) ? 4 : 8;
  std::vector<uint32_t> ord;
  for (uint32_t i = 0; i < count; ++i) {
    if (ns[i] == 0) continue;
    if (!ptrs[i]) return IPS_E_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(ptrs[i]) % align) return IPS_E_MISALIGNED;
    if (ns[i] > (~(uintptr_t)0 - reinterpret_cast<uintptr_t>(ptrs[i])) / D) return IPS_E_INVALID_ARG;
    ord.push_back(i);
  }
  // No two buffers may overlap (byte ranges, over all groups).
  std::sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) {
    return reinterpret_cast<uintptr_t>(ptrs[x]) < reinterpret_cast<uintptr_t>(ptrs[y]);
  });
  for (uint32_t q = 1; q < ord.size(); ++q) {
    const uintptr_t e = reinterpret_cast<uintptr_t>(ptrs[ord[q - 1]]) + ns[ord[q - 1]] * D;
    if (e > reinterpret_cast<uintptr_t>(ptrs[ord[q]])) return IPS_E_INVALID_ARG;
  }
  std::stable_sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) {
    return reinterpret_cast<uintptr_t>(ptrs[x]) % D < reinterpret_cast<uintptr_t>(ptrs[y]) % D;
  });
  for (uint32_t q = 0; q < ord.size(); ++q) {
    const uintptr_t p = reinterpret_cast<uintptr_t>(ptrs[ord[q]]);
    if (groups->empty() || groups->back().base % D != p % D) {
      PtrGroup g;
      g.base = p;
      g.span = 0;
      groups->push_back(g);
    }
    PtrGroup& g = groups->back();
    ips_segment sg;
    sg.offset = (p - g.base) / D;
    sg.n = ns[ord[q]];
    g.segs.push_back(sg);
    g.span = sg.offset + sg.n;
  }
  return IPS_OK;
}

int batch_ws(void* const* ptrs, const uint64_t* ns, uint32_t count, int type, int algo,
             const ips_params* params, size_t* out) {
  *out = 0;
  std::vector<PtrGroup> groups;
  if (int e = group_batch(ptrs, ns, count, type, &groups)) return e;
  Cfg c;
  if (int e = make_cfg(0, type, algo, params, &c)) return e;
  for (const PtrGroup& g : groups) {
    uint64_t sum = 0;
    for (const ips_segment& sg : g.segs) sum += sg.n;
    size_t b = 0;
    if (int e = segments_ws(sum, g.segs.data(), (uint32_t)g.segs.size(), type, algo, params, &b)) return e;
    *out = std::max(*out, b);
  }
  return IPS_OK;
}

int batch_impl(ips_ctx* ctx, void* const* ptrs, const uint64_t* ns, uint32_t count, int type,
               int algo, void* ws, size_t ws_bytes, const ips_params* params, void* stream) {
  if (!ctx) return IPS_E_INVALID_ARG;
  std::vector<PtrGroup> groups;
  if (int e = group_batch(ptrs, ns, count, type, &groups)) return e;
  Cfg c;
  if (int e = make_cfg(0, type, algo, params, &c)) return e;
  for (const PtrGroup& g : groups) {
    if (int e = segments_impl(ctx, reinterpret_cast<void*>(g.base), g.span, type, algo, g.segs.data(),
                              (uint32_t)g.segs.size(), ws, ws_bytes, params, stream))
      return e;
  }
  return IPS_OK;
}

// ------------------------------------------------- out-of-place ablation
//
// Super scalar samplesort's out-of-place partitioning step (the algorithm the
// paper re-implements on its framework, Section 7, and compares by I/O
// volume in its appendix) on the same GPU, with the same sampling, decision
// tree, start table and LDS-tier base case as the in-place step, as an
// ablation of the paper's in-place design.  Levels alternate between the
// input and a second array of the caller; buckets that end in the second
// array (final ones and LDS-tier tasks of a level that wrote there) are
// copied back before the LDS tier sorts them in the input, which is where
// super scalar samplesort copies back after an odd number of levels.

uint64_t oop_tmp_bytes(uint64_t n, uint32_t D) {
  return ((n * D + 255) & ~255ull) + ((2 * n + 255) & ~255ull);
}

// Reads `count` entries of a device list through a pinned staging area of
// `cap` entries (the stream is synchronized for every chunk).
template <class E>
int read_list(Run& r, const E* d_list, uint32_t count, E* staging, size_t cap, std::vector<E>* out) {
  for (uint32_t done = 0; done < count;) {
    const uint32_t cnt = (uint32_t)std::min<size_t>(count - done, cap);
    HIPCHK(r.ctx, hipMemcpyAsync(staging, d_list + done, (size_t)cnt * sizeof(E), hipMemcpyDeviceToHost, r.st));
    HIPCHK(r.ctx, hipStreamSynchronize(r.st));
    out->insert(out->end(), staging, staging + cnt);
    done += cnt;
  }
  return IPS_OK;
}

int oop_impl(ips_ctx* ctx, void* d, uint64_t n, int type, void* tmp, size_t tmp_bytes, void* ws, size_t ws_bytes,
             const ips_params* params, void* stream) {
  ips_params p;
  if (params) p = *params;
  else std::memset(&p, 0, sizeof(p));
  if (p.flags & (IPS_FLAG_LEVEL1_ONLY | IPS_FLAG_GRAPH | IPS_FLAG_HOST_PLAN | IPS_FLAG_GLOBAL_BUFFERS |
                 IPS_FLAG_FUSED | IPS_FLAG_INSERTION_BASE))
    return IPS_E_INVALID_ARG;
  if (n >= (1ull << 32)) return IPS_E_TOO_LARGE;
  Run r;
  int rc = setup_run(ctx, r, d, n, n, type, IPS_SAMPLESORT, ws, ws_bytes, 0, &p, stream, 0, nullptr);
  if (rc || n < 2) return rc;
  const Cfg& c = r.c;
  if (!tmp || tmp_bytes < oop_tmp_bytes(n, c.D)) return IPS_E_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(tmp) % 256) return IPS_E_MISALIGNED;
  if (n <= c.cap) {
    std::vector<LTask> lt(1);
    lt[0].l = 0; lt[0].n = (uint32_t)n; lt[0].req = 0;
    return level_loop(r, {}, lt, true);
  }
  uint32_t* A = r.data;
  uint32_t* B = static_cast<uint32_t*>(tmp);
  OopArgs o;
  o.oracle = static_cast<uint8_t*>(tmp) + ((n * c.D + 255) & ~255ull);
  o.tasks = r.a.tasks;
  o.recs = r.a.recs;
  o.wg_task = r.a.cls_task;
  o.cnt = r.a.wg_nfull;
  o.b_start = r.a.b_start;
  o.nbs = r.L.NBS;
  LTask* d_lds = wsp<LTask>(r, R_LTC);
  LTask* d_copy = d_lds + r.L.LTB;
  CTask* d_next = wsp<CTask>(r, R_NEXT);
  struct Hdr { uint32_t K, logK, eq, nb, u, alpha, kp, m; };
  std::vector<HTask> cur(1);
  cur[0].l = 0; cur[0].n = n; cur[0].level = 0; cur[0].shift = 0; cur[0].width = 0;
  cur[0].tflags = (c.flags & IPS_FLAG_EQ_ON) ? TF_EQ_ON : (c.flags & IPS_FLAG_EQ_OFF) ? TF_EQ_OFF : 0u;
  if (!(c.flags & IPS_FLAG_PAPER_ROOT_ALPHA)) cur[0].tflags |= TF_ROOT_ALPHA;
  uint32_t level = 0;
  while (!cur.empty()) {
    const bool to_b = (level % 2) == 0;
    uint32_t* src = to_b ? A : B;
    uint32_t* dst = to_b ? B : A;
    uint64_t level_elems = 0;
    for (const HTask& t : cur) level_elems += t.n;
    const uint64_t S = std::max<uint64_t>(16384, level_elems / WG_TARGET);   // stripe length
    std::vector<HTask> next;
    std::vector<LTask> lds, copy;
    const uint32_t row = std::min<uint32_t>(level, IPS_MAX_LEVELS - 1);
    for (size_t i = 0; i < cur.size();) {
      // a batch: as many tasks as the task, workgroup and bucket budgets hold
      uint32_t T = 0, wsum = 0, nbsum = 0;
      while (i + T < cur.size() && T < r.L.TB) {
        const HTask& t = cur[i + T];
        const uint32_t w = (uint32_t)std::min<uint64_t>(WG_TARGET, (t.n + S - 1) / S);
        const uint32_t nbt = 2 * task_kprime(c, t.n, t.level) + 1;
        if (T && (wsum + w > r.L.WB || nbsum + nbt > r.L.NBE)) break;
        wsum += w;
        nbsum += nbt;
        ++T;
      }
      for (uint32_t t = 0; t < T; ++t) {
        PTask& q = r.h_tasks[t];
        std::memset(&q, 0, sizeof(q));
        q.l = cur[i + t].l;
        q.n = cur[i + t].n;
        q.level = cur[i + t].level;
        q.tflags = cur[i + t].tflags;
        q.kp = task_kprime(c, q.n, q.level);
      }
      BatchArgs a = r.a;
      a.data = src;
      HIPCHK(ctx, hipMemcpyAsync(wsp<PTask>(r, R_TASKS), r.h_tasks, T * sizeof(PTask), hipMemcpyHostToDevice, r.st));
      HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_SAMPLE, 0, [&] { return c.L->sample(a, T, c.seed, r.st); }));
      HIPCHK(ctx, hipMemcpy2DAsync(r.h_rb, sizeof(Hdr), r.a.recs, sizeof(StepRec), sizeof(Hdr), T,
                                   hipMemcpyDeviceToHost, r.st));
      if (int e = read_ctrl(r)) return e;
      const Hdr* hdr = reinterpret_cast<const Hdr*>(r.h_rb);
      uint32_t wg = 0, bucket = 0;
      uint64_t bel = 0;
      uint32_t* h_cls = r.h_maps;
      for (uint32_t t = 0; t < T; ++t) {
        PTask& q = r.h_tasks[t];
        q.K = hdr[t].K; q.logK = hdr[t].logK; q.eq = hdr[t].eq; q.nb = hdr[t].nb;
        if (q.nb > r.L.NBS) { ctx->last_dev = 0x105; return IPS_E_DEVICE; }
        q.W = (uint32_t)std::min<uint64_t>(WG_TARGET, (q.n + S - 1) / S);
        q.wg_base = wg;
        for (uint32_t x = 0; x < q.W; ++x) h_cls[wg + x] = t;
        wg += q.W;
        q.bucket_base = bucket;
        bucket += q.nb + 1;
        bel += q.n;
      }
      if (wg > r.L.WB || bucket > r.L.NBE) { ctx->last_dev = 0x106; return IPS_E_DEVICE; }
      HIPCHK(ctx, hipMemcpyAsync(wsp<PTask>(r, R_TASKS), r.h_tasks, T * sizeof(PTask), hipMemcpyHostToDevice, r.st));
      HIPCHK(ctx, hipMemcpyAsync(const_cast<uint32_t*>(r.a.cls_task), h_cls, wg * 4, hipMemcpyHostToDevice, r.st));
      o.src = src;
      o.dst = dst;
      HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_CLASSIFY, bel, [&] { return c.L->oop_classify(o, wg, r.st); }));
      HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_BOUNDARIES, bel, [&] { return launch_oop_scan(o, T, r.st); }));
      HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_PERMUTE, bel, [&] { return c.L->oop_distribute(o, wg, r.st); }));
      HIPCHK(ctx, launch_fill32(r.a.ctrl + CTRL_NLDS, 4, 0u, r.st));
      HIPCHK(ctx, launch_oop_children(o, T, r.a.ctrl, d_next, r.L.NXB, d_lds, d_copy, r.L.LTB, c.cap,
                                      to_b ? 1u : 0u, r.st));
      if (int e = read_ctrl(r)) return e;
      const uint32_t nnext = r.h_ctrl[CTRL_NNEXT], nlds = r.h_ctrl[CTRL_NLDS], ncopy = r.h_ctrl[CTRL_NLDS + 1];
      if (nnext > r.L.NXB || nlds > r.L.LTB || ncopy > r.L.LTB) { ctx->last_dev = 0x107; return IPS_E_DEVICE; }
      std::vector<CTask> ch;
      if (int e = read_list(r, d_next, nnext, reinterpret_cast<CTask*>(r.h_rb), r.rb_bytes / sizeof(CTask), &ch))
        return e;
      for (const CTask& q : ch) {
        HTask h;
        h.l = q.l; h.n = q.n; h.level = q.level; h.tflags = q.tflags; h.shift = 0; h.width = 0;
        next.push_back(h);
      }
      if (int e = read_list(r, d_lds, nlds, r.h_lt, r.L.LTB, &lds)) return e;
      if (int e = read_list(r, d_copy, ncopy, r.h_lt, r.L.LTB, &copy)) return e;
      ctx->stats.steps += T;
      ctx->stats.batches += 1;
      ctx->stats.partitioned_elems += bel;
      i += T;
    }
    // buckets that stay in the second array come back first
    uint64_t cel = 0;
    for (const LTask& t : copy) cel += t.n;
    for (size_t done = 0; done < copy.size();) {
      const size_t cnt = std::min<size_t>(copy.size() - done, r.L.LTB);
      std::memcpy(r.h_lt, copy.data() + done, cnt * sizeof(LTask));
      LTask* d_lt = wsp<LTask>(r, R_LT);
      HIPCHK(ctx, hipMemcpyAsync(d_lt, r.h_lt, cnt * sizeof(LTask), hipMemcpyHostToDevice, r.st));
      HIPCHK(ctx, timed(ctx, r.st, row, IPS_PH_CLEANUP_B, cel,
                        [&] { return c.L->copy_ranges(d_lt, (uint32_t)cnt, B, A, r.st); }));
      HIPCHK(ctx, hipStreamSynchronize(r.st));   // the staging is reused
      done += cnt;
    }
    for (const LTask& t : lds) ctx->stats.lds_elems += t.n;
    if (!lds.empty())
      if (int e = launch_lds_tasks(r, lds, row)) return e;
    std::sort(next.begin(), next.end(), [](const HTask& x, const HTask& y) { return x.l < y.l; });
    cur.swap(next);
    ctx->stats.levels = ++level;
    ctx->prof.levels = std::min<uint32_t>(level, IPS_MAX_LEVELS);
  }
  return read_ctrl(r);
}

// ------------------------------------------------------------------ serving
//
// Continuous batching (no paper passage; the closest analogue is the reuse
// of a preallocated sorter object, Section 7.6).  Requests are grouped into
// lanes by element type and algorithm; each lane owns a slice of the
// workspace planned for its share of the HBM budget, its own stream and its
// own pinned staging, and runs device-planned steps over one task queue.
// Between two rounds of a lane (a round is a few steps followed by an
// asynchronous read-back of the control block and of the per-request
// counters), arrived requests are admitted in arrival order while the lane's
// elements in flight stay within its plan and all request data plus the
// lanes' workspaces stays within the budget: requests larger than the LDS
// tier become root tasks at the tail of the running queue, smaller ones are
// sorted by the LDS tier at the start of the next round.  The kernels add
// the elements of every final bucket and every finished LDS-tier task to the
// counter of the request they belong to, so a request completes at the first
// read-back that shows all its elements final.  Lanes run on separate
// streams, so the work of requests of different types overlaps on the GPU,
// and requests of one type share the launches of every step.

struct SLane {
  int type = 0, algo = 0;
  uint32_t D = 0;
  ips_ctx* lctx = nullptr;
  Run r;
  PlanCfg pc;
  ChildArgs ca;
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  uintptr_t base = 0;
  uint64_t span = 0, n_plan = 0, inflight = 0;
  size_t ws_off = 0, ws_bytes = 0;
  std::vector<uint32_t> reqs;      // requests of the lane, by address (request table order)
  std::vector<uint32_t> seg_of;    // request id -> table index (indexed by position in reqs)
  uint64_t* d_seglo = nullptr;
  uint64_t* d_done = nullptr;
  uint64_t* h_done = nullptr;
  uint64_t* h_seglo = nullptr;
  uint32_t* h_words = nullptr;     // staging of control words
  SegItem* h_items = nullptr;
  SegItem* d_items = nullptr;
  uint64_t *d_mn = nullptr, *d_mx = nullptr, *h_mn = nullptr, *h_mx = nullptr;
  uint64_t items_cap = 0;
  std::deque<uint32_t> waiting;
  std::vector<uint32_t> active;
  std::vector<LTask> lt_new;
  std::vector<CTask> roots_new;
  uint32_t qhead = 0, qtail = 0, rounds = 0;
  bool busy = false, ready = false;
  int err = IPS_OK;
};

// Steps per round of a lane (arrivals are admitted between rounds).  A
// round whose task queue is empty runs no step (only the LDS-tier sorts of
// newly admitted small requests).
constexpr uint32_t SERVE_STEPS = 1;

struct LaneExtra {
  size_t o_seglo, o_done, o_items, o_mn, o_mx, total;
};

LaneExtra lane_extra(uint64_t nseg, uint64_t items) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  LaneExtra e;
  e.o_seglo = 0;
  e.o_done = al(nseg * 8);
  e.o_items = e.o_done + al(nseg * 8);
  e.o_mn = e.o_items + al(items * sizeof(SegItem));
  e.o_mx = e.o_mn + al(nseg * 8);
  e.total = e.o_mx + al(nseg * 8);
  return e;
}

// Scan chunks of the radix roots admitted at once: every root holds more
// than cap elements, and all of them together at most n_plan.
uint64_t lane_items(uint64_t n_plan, uint32_t cap) { return n_plan / SEG_CHUNK + n_plan / ((uint64_t)cap + 1) + 2; }

// Elements a lane holds in flight at most: its share of half the budget.
uint64_t lane_plan_elems(uint64_t budget, uint32_t lanes, uint32_t D) {
  return std::max<uint64_t>(2, budget / (2ull * std::max<uint32_t>(1, lanes) * D));
}

size_t lane_ws_bytes(int type, int algo, uint64_t n_plan, uint64_t nseg, const ips_params* params, int* rc) {
  Cfg c;
  *rc = make_cfg(n_plan, type, algo, params, &c);
  if (*rc) return 0;
  Layout L;
  plan(n_plan, c, &L);
  return ((L.total + lane_extra(nseg, lane_items(n_plan, c.cap)).total) + 255) & ~(size_t)255;
}

void lane_fail(SLane& L, ips_request* reqs, int rc, double now, uint32_t* done_cnt) {
  for (uint32_t id : L.active) {
    reqs[id].status = rc;
    reqs[id].done_s = now;
    reqs[id].detail = rc == IPS_E_DEVICE ? L.lctx->last_dev : rc == IPS_E_HIP ? L.lctx->last_hip : 0;
    ++*done_cnt;
  }
  L.active.clear();
  L.inflight = 0;
  L.err = rc;
}

// Sets up a lane: context, stream, event, workspace slice, request table.
int lane_init(SLane& L, ips_ctx* ctx, ips_request* reqs, uint8_t* ws, const ips_params* params) {
  L.lctx = new (std::nothrow) ips_ctx();
  if (!L.lctx) return IPS_E_INVALID_ARG;
  L.lctx->device = ctx->device;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking));
  HIPCHK(ctx, hipEventCreateWithFlags(&L.ev, hipEventDisableTiming));
  const uint64_t nseg = L.reqs.size();
  Cfg c0;
  if (int e = make_cfg(L.n_plan, L.type, L.algo, params, &c0)) return e;
  const uint64_t items = lane_items(L.n_plan, c0.cap);
  L.items_cap = items;
  const LaneExtra ex = lane_extra(nseg, items);
  ips_params p;
  if (params) p = *params;
  else std::memset(&p, 0, sizeof(p));
  p.flags = (p.flags | IPS_FLAG_NO_SORTED_CHECK) & ~(uint32_t)(IPS_FLAG_PROFILE | IPS_FLAG_GRAPH | IPS_FLAG_HOST_PLAN);
  const size_t pin_extra = ex.total + 256;
  uint8_t* hx = nullptr;
  int rc = setup_run(L.lctx, L.r, reinterpret_cast<void*>(L.base), L.span, L.n_plan, L.type, L.algo,
                     ws + L.ws_off, L.ws_bytes, ex.total, &p, L.st, pin_extra, &hx);
  if (rc) return rc;
  if (!hx) return IPS_E_INVALID_ARG;
  Run& r = L.r;
  r.lds_min = 1;   // every step sorts the LDS-tier children it produced (latency)
  uint8_t* wx = r.ws + r.L.total;
  L.d_seglo = reinterpret_cast<uint64_t*>(wx + ex.o_seglo);
  L.d_done = reinterpret_cast<uint64_t*>(wx + ex.o_done);
  L.d_items = reinterpret_cast<SegItem*>(wx + ex.o_items);
  L.d_mn = reinterpret_cast<uint64_t*>(wx + ex.o_mn);
  L.d_mx = reinterpret_cast<uint64_t*>(wx + ex.o_mx);
  L.h_seglo = reinterpret_cast<uint64_t*>(hx + ex.o_seglo);
  L.h_done = reinterpret_cast<uint64_t*>(hx + ex.o_done);
  L.h_items = reinterpret_cast<SegItem*>(hx + ex.o_items);
  L.h_mn = reinterpret_cast<uint64_t*>(hx + ex.o_mn);
  L.h_mx = reinterpret_cast<uint64_t*>(hx + ex.o_mx);
  L.h_words = reinterpret_cast<uint32_t*>(hx + ex.total);
  for (uint64_t i = 0; i < nseg; ++i)
    L.h_seglo[i] = (reinterpret_cast<uintptr_t>(reqs[L.reqs[i]].d_data) - L.base) / L.D;
  HIPCHK(L.lctx, hipMemcpyAsync(L.d_seglo, L.h_seglo, nseg * 8, hipMemcpyHostToDevice, L.st));
  HIPCHK(L.lctx, launch_fill32(reinterpret_cast<uint32_t*>(L.d_done), 2 * nseg, 0u, L.st));
  const uint64_t lo = reinterpret_cast<uintptr_t>(L.d_seglo), dn = reinterpret_cast<uintptr_t>(L.d_done);
  L.h_words[0] = (uint32_t)lo; L.h_words[1] = (uint32_t)(lo >> 32);
  L.h_words[2] = (uint32_t)dn; L.h_words[3] = (uint32_t)(dn >> 32);
  L.h_words[4] = (uint32_t)nseg;
  HIPCHK(L.lctx, hipMemcpyAsync(r.a.ctrl + CTRL_SEGLO, L.h_words, 5 * 4, hipMemcpyHostToDevice, L.st));
  HIPCHK(L.lctx, launch_fill32(r.a.ctrl + CTRL_QHEAD, 2, 0u, L.st));
  HIPCHK(L.lctx, launch_fill32(reinterpret_cast<uint32_t*>(r.a.step_el), MAX_STEPS_RECORDED * 8, 0u, L.st));
  HIPCHK(L.lctx, launch_fill32(r.a.ctrl + CTRL_NLDS, 14, 0u, L.st));
  plan_cfg(r, &L.pc, &L.ca);
  HIPCHK(L.lctx, hipStreamSynchronize(L.st));   // the staging of the table is reused below
  L.ready = true;
  return IPS_OK;
}

// Admission of one request into an idle lane (returns false when it must
// wait).  Radix roots need their key range first: collected here and
// resolved by lane_resolve_radix.
bool lane_admit(SLane& L, ips_request& q, uint32_t id, std::vector<uint32_t>& radix_new) {
  if (L.inflight + q.n > L.n_plan) return false;
  L.inflight += q.n;
  const uint64_t l = (reinterpret_cast<uintptr_t>(q.d_data) - L.base) / L.D;
  L.active.push_back(id);
  if (q.n <= L.r.c.cap) {
    LTask t;
    t.l = l;
    t.n = (uint32_t)q.n;
    t.req = L.seg_of[id];   // the request's entry in the lane's table
    L.lt_new.push_back(t);
  } else if (L.r.c.radix) {
    radix_new.push_back(id);
  } else {
    CTask t;
    t.l = l; t.n = q.n; t.level = 0; t.shift = 0; t.width = 0;
    t.tflags = (L.r.c.flags & IPS_FLAG_PAPER_ROOT_ALPHA) ? 0u : TF_ROOT_ALPHA;
    L.roots_new.push_back(t);
  }
  return true;
}

// Key ranges of newly admitted radix requests (one batched scan, waited
// for: the lane is idle), then their root tasks.  Requests whose keys are
// all equal are finished at once.
int lane_resolve_radix(SLane& L, ips_request* reqs, const std::vector<uint32_t>& ids, double now,
                       uint32_t* done_cnt) {
  if (ids.empty()) return IPS_OK;
  Run& r = L.r;
  uint64_t ni = 0;
  for (uint32_t q = 0; q < ids.size(); ++q) {
    const ips_request& rq = reqs[ids[q]];
    const uint64_t l = (reinterpret_cast<uintptr_t>(rq.d_data) - L.base) / L.D;
    for (uint64_t o = 0; o < rq.n; o += SEG_CHUNK) {
      if (ni >= L.items_cap) return IPS_E_INVALID_ARG;
      SegItem it;
      it.l = l + o;
      it.n = (uint32_t)std::min<uint64_t>(SEG_CHUNK, rq.n - o);
      it.seg = q;
      it.first = o == 0;
      it.pad = 0;
      L.h_items[ni++] = it;
    }
  }
  const uint32_t m = (uint32_t)ids.size();
  HIPCHK(L.lctx, hipMemcpyAsync(L.d_items, L.h_items, ni * sizeof(SegItem), hipMemcpyHostToDevice, L.st));
  HIPCHK(L.lctx, launch_fill32(reinterpret_cast<uint32_t*>(L.d_mn), 2 * m, 0xFFFFFFFFu, L.st));
  HIPCHK(L.lctx, launch_fill32(reinterpret_cast<uint32_t*>(L.d_mx), 2 * m, 0u, L.st));
  HIPCHK(L.lctx, r.c.L->seg_minmax(L.d_items, (uint32_t)ni, r.data, L.d_mn, L.d_mx, L.st));
  HIPCHK(L.lctx, hipMemcpyAsync(L.h_mn, L.d_mn, m * 8, hipMemcpyDeviceToHost, L.st));
  HIPCHK(L.lctx, hipMemcpyAsync(L.h_mx, L.d_mx, m * 8, hipMemcpyDeviceToHost, L.st));
  HIPCHK(L.lctx, hipStreamSynchronize(L.st));
  for (uint32_t q = 0; q < m; ++q) {
    ips_request& rq = reqs[ids[q]];
    HTask h;
    const uint64_t l = (reinterpret_cast<uintptr_t>(rq.d_data) - L.base) / L.D;
    if (!make_root(r.c, l, rq.n, L.h_mn[q], L.h_mx[q], &h)) {   // all keys equal: sorted
      rq.status = IPS_OK;
      rq.done_s = now;
      L.inflight -= rq.n;
      L.active.erase(std::find(L.active.begin(), L.active.end(), ids[q]));
      ++*done_cnt;
      continue;
    }
    CTask t;
    t.l = h.l; t.n = h.n; t.level = 0; t.tflags = h.tflags; t.shift = h.shift; t.width = h.width;
    L.roots_new.push_back(t);
  }
  return IPS_OK;
}

// One round of an idle lane: the new small requests through the LDS tier,
// the new roots onto the queue, SERVE_STEPS device-planned steps, and the
// asynchronous read-back of the control block and the request counters.
int lane_launch(SLane& L, uint32_t steps) {
  Run& r = L.r;
  if (!L.lt_new.empty()) {
    if (int e = launch_lds_tasks(r, L.lt_new, 0)) return e;
    L.lt_new.clear();
  }
  if (!L.roots_new.empty()) {
    if ((uint64_t)(L.qtail - L.qhead) + L.roots_new.size() > r.L.QCAP) return IPS_E_DEVICE;
    CTask* h = reinterpret_cast<CTask*>(r.h_rb);
    const size_t chunk = r.rb_bytes / sizeof(CTask);
    size_t done = 0;
    while (done < L.roots_new.size()) {
      const size_t cnt = std::min(chunk, L.roots_new.size() - done);
      std::memcpy(h, L.roots_new.data() + done, cnt * sizeof(CTask));
      // ring positions qtail .. qtail + cnt - 1 (modulo the capacity): at most two copies
      const uint32_t p0 = L.qtail % r.L.QCAP;
      const size_t first = std::min<size_t>(cnt, r.L.QCAP - p0);
      HIPCHK(L.lctx, hipMemcpyAsync(r.a.queue + p0, h, first * sizeof(CTask), hipMemcpyHostToDevice, L.st));
      if (first < cnt)
        HIPCHK(L.lctx, hipMemcpyAsync(r.a.queue, h + first, (cnt - first) * sizeof(CTask), hipMemcpyHostToDevice,
                                      L.st));
      L.qtail += (uint32_t)cnt;
      done += cnt;
      if (done < L.roots_new.size()) HIPCHK(L.lctx, hipStreamSynchronize(L.st));   // staging reused
    }
    L.roots_new.clear();
    HIPCHK(L.lctx, launch_fill32(r.a.ctrl + CTRL_QTAIL, 1, L.qtail, L.st));
  }
  if (L.qhead == L.qtail) steps = 0;   // nothing queued (the host's view is exact between rounds)
  for (uint32_t s = 0; s < steps; ++s)
    if (int e = enqueue_step(r, L.pc, L.ca, MAX_STEPS_RECORDED)) return e;
  HIPCHK(L.lctx, hipMemcpyAsync(r.h_ctrl, r.a.ctrl, CTRL_WORDS * 4, hipMemcpyDeviceToHost, L.st));
  HIPCHK(L.lctx, hipMemcpyAsync(L.h_done, L.d_done, L.reqs.size() * 8, hipMemcpyDeviceToHost, L.st));
  HIPCHK(L.lctx, hipEventRecord(L.ev, L.st));
  L.busy = true;
  ++L.rounds;
  return IPS_OK;
}

// Checks a busy lane; after its round finished, completes the requests whose
// elements are all final.  Returns an error code of the round, if any.
int lane_poll(SLane& L, ips_request* reqs, double now, uint64_t* data_bytes, uint32_t* done_cnt) {
  if (!L.busy) return IPS_OK;
  const hipError_t q = hipEventQuery(L.ev);
  if (q == hipErrorNotReady) return IPS_OK;
  L.busy = false;
  if (q != hipSuccess) { L.lctx->last_hip = (int)q; return IPS_E_HIP; }
  if (int e = check_dev_error(L.r)) return e;
  L.qhead = L.r.h_ctrl[CTRL_QHEAD];
  L.qtail = L.r.h_ctrl[CTRL_QTAIL];
  std::vector<uint32_t> still;
  for (uint32_t id : L.active) {
    const uint32_t pos = L.seg_of[id];
    if (L.h_done[pos] >= reqs[id].n) {
      reqs[id].status = IPS_OK;
      reqs[id].done_s = now;
      L.inflight -= reqs[id].n;
      *data_bytes -= reqs[id].n * (uint64_t)L.D;
      ++*done_cnt;
    } else {
      still.push_back(id);
    }
  }
  L.active.swap(still);
  // An empty queue runs every pending LDS-tier task within the round, so
  // work left over then is a broken invariant, not a reason to spin.
  if (!L.active.empty() && L.qhead == L.qtail && L.lt_new.empty() && L.roots_new.empty()) {
    L.lctx->last_dev = 0x104;
    return IPS_E_DEVICE;
  }
  return IPS_OK;
}

using SClock = std::chrono::steady_clock;
double s_since(SClock::time_point t0) { return std::chrono::duration<double>(SClock::now() - t0).count(); }

int serve_lanes_plan(const ips_request* reqs, uint32_t nreq, uint64_t budget, const ips_params* params,
                     std::vector<SLane>* lanes_out, size_t* total_ws) {
  std::vector<SLane>& lanes = *lanes_out;
  lanes.clear();
  *total_ws = 0;
  std::vector<std::pair<int, int>> keys;
  for (uint32_t i = 0; i < nreq; ++i) {
    const std::pair<int, int> k(reqs[i].elem_type, reqs[i].algo);
    if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
  }
  lanes.resize(keys.size());
  for (size_t g = 0; g < keys.size(); ++g) {
    SLane& L = lanes[g];
    L.type = keys[g].first;
    L.algo = keys[g].second;
    L.D = elem_bytes(L.type);
    if (!L.D) return IPS_E_INVALID_ARG;
    L.n_plan = lane_plan_elems(budget, (uint32_t)keys.size(), L.D);
    uintptr_t lo = ~(uintptr_t)0, hi = 0;
    for (uint32_t i = 0; i < nreq; ++i) {
      if (reqs[i].elem_type != L.type || reqs[i].algo != L.algo || reqs[i].n < 2) continue;
      const uintptr_t p = reinterpret_cast<uintptr_t>(reqs[i].d_data);
      lo = std::min(lo, p);
      hi = std::max<uintptr_t>(hi, p + reqs[i].n * L.D);
      L.reqs.push_back(i);
    }
    if (L.reqs.empty()) { L.base = 0; L.span = 0; continue; }
    L.base = lo;
    L.span = (hi - lo + L.D - 1) / L.D;
    std::sort(L.reqs.begin(), L.reqs.end(), [&](uint32_t a, uint32_t b) { return reqs[a].d_data < reqs[b].d_data; });
    int rc = IPS_OK;
    L.ws_off = *total_ws;
    L.ws_bytes = lane_ws_bytes(L.type, L.algo, L.n_plan, L.reqs.size(), params, &rc);
    if (rc) return rc;
    *total_ws += L.ws_bytes;
  }
  return IPS_OK;
}

int serve_continuous(ips_ctx* ctx, ips_request* reqs, uint32_t nreq, const ips_serve_config* cfg, void* d_ws,
                     size_t ws_bytes, const ips_params* params) {
  std::vector<SLane> lanes;
  size_t total_ws = 0;
  if (int e = serve_lanes_plan(reqs, nreq, cfg->hbm_budget, params, &lanes, &total_ws)) return e;
  if (total_ws > ws_bytes) return IPS_E_WORKSPACE;
  if (nreq && !d_ws) return IPS_E_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return IPS_E_MISALIGNED;
  std::vector<int32_t> lane_of(nreq, -1);
  for (size_t g = 0; g < lanes.size(); ++g) {
    SLane& L = lanes[g];
    L.seg_of.assign(nreq, 0);
    for (uint32_t pos = 0; pos < L.reqs.size(); ++pos) {
      L.seg_of[L.reqs[pos]] = pos;
      lane_of[L.reqs[pos]] = (int32_t)g;
    }
  }
  int first_error = IPS_OK;
  int rc = IPS_OK;
  std::vector<uint32_t> order(nreq);
  for (uint32_t i = 0; i < nreq; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
  uint32_t next = 0, done = 0, round_id = 0;
  uint64_t data_bytes = 0;
  const SClock::time_point t0 = SClock::now();
  while (rc == IPS_OK && done < nreq) {
    double now = s_since(t0);
    // arrivals go to their lane's queue (empty requests finish at once)
    while (next < nreq && reqs[order[next]].arrival_s <= now) {
      const uint32_t id = order[next++];
      ips_request& q = reqs[id];
      const int g = lane_of[id];
      if (q.n < 2 || g < 0) {
        q.start_s = q.done_s = now;
        q.status = IPS_OK;
        ++done;
        continue;
      }
      SLane& L = lanes[(size_t)g];
      if (q.n > L.n_plan || (reinterpret_cast<uintptr_t>(q.d_data) - L.base) % L.D) {
        q.start_s = q.done_s = now;
        q.status = q.n > L.n_plan ? IPS_E_WORKSPACE : IPS_E_MISALIGNED;
        if (first_error == IPS_OK) first_error = q.status;
        ++done;
        continue;
      }
      if (L.err) {
        q.start_s = q.done_s = now;
        q.status = L.err;
        ++done;
        continue;
      }
      L.waiting.push_back(id);
    }
    bool any_busy = false;
    for (SLane& L : lanes) {
      if (!L.ready) {   // a lane is set up when its first request can be admitted
        if (L.waiting.empty() || L.err) continue;
        const int e = lane_init(L, ctx, reqs, static_cast<uint8_t*>(d_ws), params);
        if (e) {
          L.err = e;
          if (first_error == IPS_OK) first_error = e;
          for (uint32_t id : L.waiting) { reqs[id].status = e; reqs[id].start_s = reqs[id].done_s = now; ++done; }
          L.waiting.clear();
          continue;
        }
      }
      const int e = lane_poll(L, reqs, now, &data_bytes, &done);
      if (e) {
        data_bytes -= L.inflight * L.D;
        lane_fail(L, reqs, e, now, &done);
        if (first_error == IPS_OK) first_error = e;
        for (uint32_t id : L.waiting) { reqs[id].status = e; reqs[id].start_s = reqs[id].done_s = now; ++done; }
        L.waiting.clear();
        continue;
      }
      if (L.busy) { any_busy = true; continue; }
      // admission in arrival order while the lane's plan and the budget hold
      now = s_since(t0);
      std::vector<uint32_t> radix_new;
      uint32_t admitted = 0;
      while (!L.waiting.empty() && !(cfg->max_batch && admitted >= cfg->max_batch)) {
        ips_request& q = reqs[L.waiting.front()];
        const uint64_t bytes = q.n * (uint64_t)L.D;
        if (data_bytes + bytes + total_ws > cfg->hbm_budget && !L.active.empty()) break;
        if (!lane_admit(L, q, L.waiting.front(), radix_new)) break;
        q.start_s = now;
        q.batch = round_id;
        data_bytes += bytes;
        L.waiting.pop_front();
        ++admitted;
      }
      int e2 = lane_resolve_radix(L, reqs, radix_new, now, &done);
      if (!e2 && !L.active.empty()) {
        e2 = lane_launch(L, SERVE_STEPS);
        ++round_id;
        any_busy = any_busy || L.busy;
      }
      if (e2) {
        data_bytes -= L.inflight * L.D;
        lane_fail(L, reqs, e2, now, &done);
        if (first_error == IPS_OK) first_error = e2;
      }
    }
    if (!any_busy && done < nreq) {
      // idle: sleep until the next arrival
      if (next < nreq) {
        const double left = reqs[order[next]].arrival_s - s_since(t0);
        if (left > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(left - 1e-4));
      }
    } else if (any_busy) {
      // poll the lanes' events again at once (a timed sleep lasts tens of
      // microseconds on a Linux host, longer than a small request's round)
      std::this_thread::yield();
    }
  }
  for (SLane& L : lanes) {
    if (L.st) {
      (void)hipStreamSynchronize(L.st);
      (void)hipStreamDestroy(L.st);
    }
    if (L.ev) (void)hipEventDestroy(L.ev);
    if (L.lctx) {
      for (hipEvent_t e : L.lctx->ev_pool) (void)hipEventDestroy(e);
      if (L.lctx->pin) (void)hipHostFree(L.lctx->pin);
      delete L.lctx;
    }
  }
  if (rc) return rc;
  return first_error;
}

}  // namespace

extern "C" {

int ips_tuned_params(const ips_tune_entry* table, uint32_t count, uint64_t n, int elem_type, int algo,
                     int batched, const ips_params* base, ips_params* out) {
  if (!out || (!table && count)) return IPS_E_INVALID_ARG;
  for (uint32_t i = 0; i < count; ++i)
    if (table[i].log2n_min > table[i].log2n_max) return IPS_E_INVALID_ARG;
  ips_params p;
  if (base) p = *base;
  else std::memset(&p, 0, sizeof(p));
  *out = p;
  if (n < 1) return 0;
  const uint32_t cls = 63u - (uint32_t)__builtin_clzll(n);
  for (uint32_t i = 0; i < count; ++i) {
    const ips_tune_entry& e = table[i];
    if (e.elem_type != elem_type || e.algo != algo || e.batched != (batched ? 1u : 0u) ||
        cls < e.log2n_min || cls > e.log2n_max)
      continue;
    if (!p.k) p.k = e.k;
    if (!p.block_bytes) p.block_bytes = e.block_bytes;
    if (!p.n0) p.n0 = e.n0;
    if (!p.lds_task_max) p.lds_task_max = e.lds_task_max;
    if (!p.piece_blocks) p.piece_blocks = e.piece_blocks;
    if (!p.perm_groups) p.perm_groups = e.perm_groups;
    if (!p.perm_wg) p.perm_wg = e.perm_wg;
    if (!p.k_root) p.k_root = e.k_root;
    *out = p;
    return 1;
  }
  return 0;
}

int ips_abi_version(void) { return IPS_ABI_VERSION; }

const char* ips_status_string(int s) {
  switch (s) {
    case IPS_OK: return "IPS_OK";
    case IPS_E_INVALID_ARG: return "IPS_E_INVALID_ARG: invalid argument";
    case IPS_E_UNSUPPORTED: return "IPS_E_UNSUPPORTED: unsupported type/algorithm combination";
    case IPS_E_WORKSPACE: return "IPS_E_WORKSPACE: workspace too small";
    case IPS_E_MISALIGNED: return "IPS_E_MISALIGNED: pointer not aligned";
    case IPS_E_TOO_LARGE: return "IPS_E_TOO_LARGE: too many elements";
    case IPS_E_HIP: return "IPS_E_HIP: HIP runtime error";
    case IPS_E_DEVICE: return "IPS_E_DEVICE: kernel consistency error";
    case IPS_E_NO_DEVICE: return "IPS_E_NO_DEVICE: no usable device";
    case IPS_E_SCRATCH:
      return "IPS_E_SCRATCH: the call needs more than the 64 MiB static scratch (or the context's pinned "
             "staging) of the allocation-free entry point";
    default: return "unknown status";
  }
}

int ips_ctx_create(ips_ctx** out, int device) {
  if (!out) return IPS_E_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return IPS_E_NO_DEVICE;
  ips_ctx* c = new (std::nothrow) ips_ctx();
  if (!c) return IPS_E_INVALID_ARG;
  c->device = device;
  std::memset(&c->root, 0, sizeof(c->root));
  std::memset(&c->stats, 0, sizeof(c->stats));
  if (device >= MAX_DEVICES) { delete c; return IPS_E_NO_DEVICE; }
  {
    // Once per device, with that device current: the device address of the
    // allocation-free entry point's scratch array.
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
      int prev = 0;
      hipError_t e = hipGetDevice(&prev);
      if (e == hipSuccess) e = hipSetDevice(device);
      void* ptr = nullptr;
      if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      const hipError_t e2 = hipSetDevice(prev);
      if (e == hipSuccess && e2 != hipSuccess) e = e2;
      if (e != hipSuccess || !ptr) {
        delete c;
        return IPS_E_HIP;
      }
      g_scratch_ptr[device] = ptr;
    }
    c->scratch = g_scratch_ptr[device];
  }
  if (int e = ensure_pinned(c, PIN_PREALLOC_BYTES)) {
    delete c;
    return e;
  }
  *out = c;
  return IPS_OK;
}

int ips_ctx_destroy(ips_ctx* ctx) {
  if (!ctx) return IPS_OK;
  for (const auto& p : ctx->pending) { ctx->ev_pool.push_back(p.a); ctx->ev_pool.push_back(p.b); }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  delete ctx;
  return IPS_OK;
}

int ips_workspace_bytes(uint64_t n, int elem_type, int algo, const ips_params* params,
                        size_t* out_bytes) {
  if (!out_bytes) return IPS_E_INVALID_ARG;
  *out_bytes = 0;
  Cfg c;
  int rc = make_cfg(n, elem_type, algo, params, &c);
  if (rc) return rc;
  if (n >= (1ull << 31) * (uint64_t)block_elems(c, max_nb(c))) return IPS_E_TOO_LARGE;
  if (n < 2) return IPS_OK;
  Layout L;
  plan(n, c, &L);
  *out_bytes = L.total;
  return IPS_OK;
}

int ips_sort_keys(ips_ctx* ctx, void* d_keys, uint64_t n, int key_type, int algo, void* d_ws,
                  size_t ws_bytes, const ips_params* params, void* stream) {
  if (key_type != IPS_U32 && key_type != IPS_U64 && key_type != IPS_F64) return IPS_E_INVALID_ARG;
  return sort_impl(ctx, d_keys, n, key_type, algo, d_ws, ws_bytes, params, stream);
}

int ips_sort_keys_noalloc(ips_ctx* ctx, void* d_keys, uint64_t n, int key_type, int algo,
                          const ips_params* params, void* stream) {
  if (!ctx) return IPS_E_INVALID_ARG;
  if (key_type != IPS_U32 && key_type != IPS_U64 && key_type != IPS_F64) return IPS_E_INVALID_ARG;
  if (params && (params->flags & (IPS_FLAG_PROFILE | IPS_FLAG_GRAPH))) return IPS_E_INVALID_ARG;
  Cfg c;
  if (int e = make_cfg(n, key_type, algo, params, &c)) return e;
  if (n >= (1ull << 31) * (uint64_t)block_elems(c, max_nb(c))) return IPS_E_TOO_LARGE;
  if (n >= 2) {
    Layout L;
    plan(n, c, &L);
    if (L.total > NOALLOC_SCRATCH_BYTES) return IPS_E_SCRATCH;
  }
  if (!ctx->scratch) return IPS_E_HIP;
  ctx->noalloc = true;
  const int rc = sort_impl(ctx, d_keys, n, key_type, algo, ctx->scratch, NOALLOC_SCRATCH_BYTES, params, stream);
  ctx->noalloc = false;
  return rc;
}

int ips_oop_workspace_bytes(uint64_t n, int elem_type, const ips_params* params, size_t* ws_bytes,
                            size_t* tmp_bytes) {
  if (!ws_bytes || !tmp_bytes) return IPS_E_INVALID_ARG;
  *ws_bytes = 0;
  *tmp_bytes = 0;
  if (n >= (1ull << 32)) return IPS_E_TOO_LARGE;
  if (int e = ips_workspace_bytes(n, elem_type, IPS_SAMPLESORT, params, ws_bytes)) return e;
  if (n >= 2) *tmp_bytes = oop_tmp_bytes(n, elem_bytes(elem_type));
  return IPS_OK;
}

int ips_sort_oop(ips_ctx* ctx, void* d_data, uint64_t n, int elem_type, void* d_tmp, size_t tmp_bytes,
                 void* d_ws, size_t ws_bytes, const ips_params* params, void* stream) {
  if (!ctx) return IPS_E_INVALID_ARG;
  if (!elem_bytes(elem_type)) return IPS_E_INVALID_ARG;
  return oop_impl(ctx, d_data, n, elem_type, d_tmp, tmp_bytes, d_ws, ws_bytes, params, stream);
}

int ips_sort_pairs(ips_ctx* ctx, void* d_recs, uint64_t n, int rec_type, int algo, void* d_ws,
                   size_t ws_bytes, const ips_params* params, void* stream) {
  if (rec_type != IPS_PAIR_U64_U64 && rec_type != IPS_REC100 && rec_type != IPS_QUARTET) return IPS_E_INVALID_ARG;
  return sort_impl(ctx, d_recs, n, rec_type, algo, d_ws, ws_bytes, params, stream);
}

int ips_segments_workspace_bytes(uint64_t n_total, const ips_segment* segs, uint32_t nseg,
                                 int elem_type, int algo, const ips_params* params,
                                 size_t* out_bytes) {
  if (!out_bytes) return IPS_E_INVALID_ARG;
  *out_bytes = 0;
  uint64_t sum = 0;
  if (int e = check_segments(segs, nseg, n_total, &sum)) return e;
  return segments_ws(sum, segs, nseg, elem_type, algo, params, out_bytes);
}

int ips_batch_workspace_bytes(void* const* d_ptrs, const uint64_t* ns, uint32_t count,
                              int elem_type, int algo, const ips_params* params,
                              size_t* out_bytes) {
  if (!out_bytes) return IPS_E_INVALID_ARG;
  return batch_ws(d_ptrs, ns, count, elem_type, algo, params, out_bytes);
}

// Upper bound of the workspace of any batch of nseg segments holding n
// elements in total (used by the serving scheduler for admission).
__attribute__((visibility("hidden")))
size_t ips_internal_ws_bound(uint64_t n, uint64_t nseg, int type, int algo, const ips_params* params) {
  Cfg c;
  if (make_cfg(n, type, algo, params, &c) != IPS_OK || n < 2) return 0;
  Layout L;
  plan(n, c, &L);
  return L.total + seg_extra_bytes(c, n, nseg);
}

// Continuous-batching replay of a trace and its workspace (ips_serve.hip).
__attribute__((visibility("hidden")))
int ips_internal_serve_continuous(ips_ctx* ctx, ips_request* reqs, uint32_t nreq, const ips_serve_config* cfg,
                                  void* d_ws, size_t ws_bytes, const ips_params* params) {
  if (!ctx) return IPS_E_INVALID_ARG;
  return serve_continuous(ctx, reqs, nreq, cfg, d_ws, ws_bytes, params);
}

__attribute__((visibility("hidden")))
int ips_internal_serve_ws(const ips_request* reqs, uint32_t nreq, uint64_t budget, const ips_params* params,
                          size_t* out) {
  std::vector<SLane> lanes;
  return serve_lanes_plan(reqs, nreq, budget, params, &lanes, out);
}

int ips_sort_batch(ips_ctx* ctx, void* const* d_ptrs, const uint64_t* ns, uint32_t count,
                   int elem_type, int algo, void* d_ws, size_t ws_bytes, const ips_params* params,
                   void* stream) {
  return batch_impl(ctx, d_ptrs, ns, count, elem_type, algo, d_ws, ws_bytes, params, stream);
}

int ips_sort_segments(ips_ctx* ctx, void* d_data, uint64_t n_total, int elem_type, int algo,
                      const ips_segment* segs, uint32_t nseg, void* d_ws, size_t ws_bytes,
                      const ips_params* params, void* stream) {
  return segments_impl(ctx, d_data, n_total, elem_type, algo, segs, nseg, d_ws, ws_bytes, params,
                       stream);
}

int ips_get_root_info(ips_ctx* ctx, ips_root_info* out) {
  if (!ctx || !out) return IPS_E_INVALID_ARG;
  *out = ctx->root;
  return IPS_OK;
}

int ips_get_stats(ips_ctx* ctx, ips_stats* out) {
  if (!ctx || !out) return IPS_E_INVALID_ARG;
  *out = ctx->stats;
  return IPS_OK;
}

int ips_get_profile(ips_ctx* ctx, ips_profile* out) {
  if (!ctx || !out) return IPS_E_INVALID_ARG;
  *out = ctx->prof;
  return IPS_OK;
}

int ips_last_hip_error(ips_ctx* ctx) { return ctx ? ctx->last_hip : 0; }
int ips_last_device_error(ips_ctx* ctx) { return ctx ? ctx->last_dev : 0; }

}  // extern "C"
