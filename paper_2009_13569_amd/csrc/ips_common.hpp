// Definitions shared by the host orchestrator and the gfx950 kernels of the
// in-place samplesort (IPS4o) / radix sort (IPS2Ra) hot path of
// arXiv 2009.13569.
#pragma once
#include <stdint.h>

namespace ips {

// Limits.  MAX_K is the largest number of buckets of a step without
// equality buckets (k <= 256, Section 6); with equality buckets a step has
// 2K buckets (Definitions and Preliminaries), so at most MAX_NB.
constexpr uint32_t MAX_K = 256;
constexpr uint32_t MAX_NB = 512;
constexpr uint32_t MAX_BLOCK_BYTES = 2048;   // 64 lanes x 8 dwords
constexpr uint32_t BUF_LDS_BYTES = 128u * 1024u;   // buffer blocks in LDS (before padding)
constexpr uint32_t BUF_PAD_DW = 2;                 // padding dwords per LDS buffer block
// Block permutation tuning: dwords of the held block per lane, spacing of
// the pieces' pointer words (in 8-byte words), and the number of placement
// pieces a bucket's block range is cut into at most (besides stripe ends).
#ifndef IPS_PERM_RD
#define IPS_PERM_RD 8
#endif
#ifndef IPS_PWORD_STRIDE
#define IPS_PWORD_STRIDE 4    // pointer words 32 bytes apart
#endif
#ifndef IPS_MAX_PLACE_PIECES
#define IPS_MAX_PLACE_PIECES 32
#endif
constexpr int PERM_RD = IPS_PERM_RD;
constexpr uint32_t PWORD_STRIDE = IPS_PWORD_STRIDE;
constexpr uint32_t MAX_PLACE_PIECES = IPS_MAX_PLACE_PIECES;
constexpr uint32_t CLS_THREADS = 1024;
constexpr uint32_t PERM_THREADS = 256;   // default workgroup size of the block permutation
constexpr uint32_t SMP_THREADS = 1024;
constexpr uint32_t CLN_THREADS = 256;
constexpr uint32_t LDST_THREADS = 512;
constexpr uint32_t MAX_SAMPLE = 4096;        // padded sample of one step
constexpr uint32_t DEEP_ALPHA = 16;          // least oversampling below the root
constexpr uint32_t PTR_BIAS = 0x80000000u;   // bias of the read pointer half
constexpr uint32_t LDS_INSERTION = 3;   // base-case "variant" that sorts list 0 by insertion sort
constexpr uint32_t FUSED_THREADS = 512;             // fused radix step: two workgroups per CU
constexpr uint32_t FUSED_BUF_BYTES = 64u * 1024u;   // and the LDS buffer blocks of one of them

// Control block at the start of the workspace.
enum CtrlSlot : uint32_t {
  CTRL_ERR = 0,        // first consistency error code (0 = none)
  CTRL_ERR_A = 1,
  CTRL_ERR_B = 2,
  CTRL_DESC = 4,       // sorted check: a descent was found
  CTRL_ASC = 5,        // sorted check: an ascent was found
  CTRL_MINMAX = 8,     // two u64: min and max radix key (dword index 8..11)
  CTRL_NLDS = 12,      // children of a batch: LDS-tier tasks per variant (12..14)
  CTRL_NNEXT = 15,     // children of a batch: next-level tasks
  CTRL_LDSEL = 16,     // children of a batch: u64 elements per LDS-tier variant (16..21)
  CTRL_LDSPOP = 22,    // LDS-tier tasks claimed per variant (22..24), zeroed with NLDS..LDSEL
  CTRL_LDSRUN = 25,    // device-planned step: 1 when this step's LDS-tier launches sort the lists
  // serving: per-request completion counters (all zero: off)
  CTRL_SEGLO = 26,     // u64 device address of the requests' first elements, ascending (26..27)
  CTRL_SEGDONE = 28,   // u64 device address of the per-request counters of finished elements (28..29)
  CTRL_NSEG = 30,      // number of requests in the table
  // device-planned execution (queue of tasks, per-step counts, statistics)
  CTRL_QHEAD = 64,     // next task to take from the queue
  CTRL_QTAIL = 65,     // end of the queued tasks
  CTRL_T = 66,         // tasks of the current step
  CTRL_NWG = 67,       // classification workgroups of the step
  CTRL_NPWG = 68,      // permutation workgroups of the step
  CTRL_NCLN = 69,      // buckets of the step (cleanup items)
  CTRL_RSV70 = 70,     // unused
  CTRL_MAXW = 71,      // largest stripe count of the step
  CTRL_SPOP = 72,      // stripe length the step's tasks were chosen for (u64: 72..73)
  CTRL_STEPS = 74,     // statistics: partitioning steps (tasks)
  CTRL_BATCHES = 75,   // statistics: steps with tasks
  CTRL_LEVELS = 76,    // statistics: deepest level + 1
  CTRL_LDSTASKS = 77,  // statistics: LDS-tier tasks
  CTRL_PARTEL = 78,    // statistics: u64 elements partitioned (78..79)
  CTRL_LDSELT = 80,    // statistics: u64 elements sorted in the LDS tier (80..81)
  CTRL_MAXSTEP = 82,   // statistics: u64 largest task (82..83)
  CTRL_WORDS = 128
};

// Device error codes.
enum DevErr : uint32_t {
  DE_NONE = 0,
  DE_CLS_INPLACE = 1,     // classification write past the consumed region
  DE_PIECES = 2,          // more pointer pieces than planned
  DE_PLACE = 3,           // no free slot found for a block
  DE_WAIT = 4,            // a slot's reader never finished
  DE_CLEANUP_COUNT = 5,   // elements to place != free positions
  DE_SAMPLE = 6,          // sample too large
  DE_PERM_RANGE = 7,      // block position outside the task
  DE_CLN_RANGE = 8,
  DE_LDST = 9,            // task too large for the LDS tier
  DE_BLOCK = 10,          // block larger than the group can hold
  DE_PLAN = 11,           // a step's geometry exceeds the workspace budgets
  DE_QUEUE = 12,          // task queue overflow
};

// Result of the sampling phase of one step (Section 4.1) or the digit of a
// radix step.  Keys live in 24-byte slots so that every key type fits.
constexpr uint32_t CHILD_WGS = 1024;   // workgroups of the children kernel (at most)
constexpr uint32_t LDS_DEFER_TASKS = 16384;   // device-planned steps: LDS-tier lists run from this many tasks
constexpr uint32_t START_BITS = 12;   // start-node table: 2^12 entries
// A start-table entry either names the tree node to descend from, or (with
// START_DIRECT set) the first bucket of its key range in bits 0-8 and the
// number of further buckets the range reaches (at most START_SPAN - 1) in
// bits 9-11: the bucket is then found by comparing with those splitters.
constexpr uint32_t START_DIRECT = 0x8000u;
constexpr uint32_t START_SPAN = 8;
struct StepRec {
  uint32_t K, logK, eq, nb, u, alpha, kp, m;
  uint32_t shift, width, radix, tshift;
  uint64_t tbase;            // start-node table: key image of s_0 and shift
  uint64_t tree[MAX_K][3];   // tree[1..K-1], breadth-first order
  uint64_t spl[MAX_K][3];    // sorted splitters s_0..s_{K-1}, s_{K-1} = s_{K-2}
  uint16_t tstart[1u << START_BITS];   // start-table entries (tree node or first bucket and span), by key prefix
};

// One partitioning task of a batch (a subarray A[l, l+n) of the input).
struct PTask {
  uint64_t l, n;             // element offset and size
  uint64_t slot_off;         // byte offset of stripe 0's buffer slot (slots contiguous)
  uint64_t spill_off;        // byte offset of the per-bucket spill area
  uint32_t level, tflags;    // recursion depth; TF_* bits
  uint32_t b, NB, W, wg_base;        // block elements, blocks, stripes, first WG
  uint32_t nb, K, logK, eq;          // buckets of the step
  uint32_t slot_bytes;               // bytes of one stripe's buffer slot
  uint32_t piece_base, piece_cap;    // pointer pieces of the permutation
  uint32_t ngrp, pwg_base, glanes;   // permutation groups
  uint32_t bucket_base;              // first entry in the batch bucket tables
  uint32_t shift, width;             // radix digit
  uint32_t kp;                       // number of buckets k' asked of the sampling phase
  uint32_t pad1;
};

enum TaskFlags : uint32_t { TF_EQ_ON = 1u, TF_EQ_OFF = 2u, TF_RADIX = 4u, TF_ROOT_ALPHA = 8u };

// A task of the LDS tier: sorted entirely inside one workgroup's LDS.
struct LTask {
  uint64_t l;
  uint32_t n;
  uint32_t req;   // serving: index of the task's request in the request table (else 0)
};

// A chunk of one segment of a batched call (ips_sort_segments): elements
// [l, l + n) of the data, belonging to segment `seg`.
struct SegItem {
  uint64_t l;
  uint32_t n, seg;
  uint32_t first, pad;   // first: the chunk starts its segment
};
// A chunk of the in-place reversal of a segment [l, l + len): the pairs
// (i, len - 1 - i) for i in [c0, c0 + cn).
struct RevItem {
  uint64_t l, len, c0;
  uint32_t cn, pad;
};
constexpr uint32_t SEG_CHUNK = 65536;   // elements per chunk

// A next-level partitioning task produced on the device.
struct CTask {
  uint64_t l, n;
  uint32_t level, tflags, shift, width;
};

// Where the children of a batch go: LDS-tier tasks by variant (the smallest
// variant that holds the task), larger ones to the next level.
struct ChildArgs {
  LTask* lt[3];
  CTask* next;
  uint32_t caps[3];
  uint32_t lt_cap, next_cap;
  uint64_t ins_parent;   // insertion-sort base case: every bucket of a task of at most k n0 elements (0: off)
};

// Workspace budgets and parameters of the device-planned execution (the
// same rules the host applies when it plans a batch).
struct PlanCfg {
  uint64_t SB, SPB, PB, slot_max;
  uint32_t TB, WB, PWB, NBE, QCAP, CLNB;
  uint32_t D, DW, k, n0, cap, cmax, groups, b_req, gbuf, radix, tflags0, wg_target, perm_threads, buf_bytes;
  uint32_t k_root;
};

// Arguments shared by the kernels of one batch.
struct BatchArgs {
  uint32_t* data;             // the array (as dwords)
  uint32_t* ctrl;             // control block
  const PTask* tasks;
  StepRec* recs;
  const uint32_t* cls_task;   // classification WG -> task
  const uint32_t* perm_task;  // permutation WG -> task
  const uint32_t* cln_map;    // cleanup WG -> (task << 10) | bucket
  uint32_t* wg_nfull;         // [WG][nbs] full blocks flushed per bucket
  uint32_t* wg_left;          // [WG][nbs] elements left in the buffer
  uint32_t* wg_F;             // [WG] full blocks at the stripe front
  uint64_t* wg_min;           // [WG][nbs] radix: min key per bucket
  uint64_t* wg_max;
  uint32_t nbs;               // row length of the per-workgroup bucket arrays (>= any task's nb)
  uint8_t* slots;             // stripe buffer slots
  uint8_t* spill;             // spill areas
  uint32_t* ovf;              // [task][MAX_BLOCK_BYTES/4] overflow blocks
  uint64_t* b_start;          // [bucket_base + j], j = 0..nb (task-relative)
  uint32_t* b_count;          // blocks of bucket j
  uint32_t* b_d;              // first block of bucket j
  uint32_t* b_plb;            // placement pieces [plb, ple) of bucket j
  uint32_t* b_ple;
  uint64_t* b_min;            // radix: min/max key of bucket j
  uint64_t* b_max;
  uint64_t* b_full;           // bit i: placement piece plb + i of bucket j is full
  uint64_t* p_word;           // pieces, PWORD_STRIDE words each: [0] packed (w << 32) | (r + PTR_BIAS);
                              // [1] reader state: low half the claimed blocks whose reads have
                              // finished, high half 1 + the first claimed block once no
                              // more claims can succeed (0 before)
  uint32_t* p_a;              // first block of the piece
  uint32_t* p_c;              // end block (exclusive) of the piece
  int32_t* p_rinit;           // last unprocessed block at the start (a-1: none)
  uint32_t* p_cum;            // unprocessed blocks of the earlier pieces
  uint32_t* p_fcnt;           // full pieces of the mask chunk starting at this piece
  uint32_t* t_npieces;        // [task] number of pieces
  uint32_t* t_unproc;         // [task] unprocessed blocks in total
  uint32_t gbuf;              // buffer blocks in the slots instead of LDS
  uint32_t ntasks;
  CTask* queue;               // device-planned execution: task ring buffer
  uint32_t qcap;              // its capacity
  uint32_t devplan;           // 1: counts of the step come from the control block
  uint32_t step;              // device-planned execution: step number of the launch
  uint64_t* step_el;          // [step][0]: elements partitioned, [1 + v]: LDS-tier variant v
};
constexpr uint32_t MAX_STEPS_RECORDED = 64;

}  // namespace ips
