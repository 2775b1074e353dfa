/* Test infrastructure only: a plain, single-threaded CPU oracle for the
 * in-place samplesort / radix-sort hot path of Axtmann, Witt, Ferizovic and
 * Sanders, "Engineering In-place (Shared-memory) Sorting Algorithms"
 * (arXiv 2009.13569).  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the product path
 * never does.  It shares no code with the GPU library.
 *
 * Element types (codes shared by value only, not by header):
 *   1 u32, 2 u64, 3 f64 (IEEE-754 totalOrder), 4 pair (u64 key at byte 0,
 *   u64 value at byte 8), 5 rec100 (100-byte record, key = bytes 0..9
 *   compared as unsigned bytes), 6 quartet (32 bytes: u64 key words a, b,
 *   c at bytes 0, 8, 16 compared lexicographically, u64 value at byte 24).
 */
#ifndef IPS_ORACLE_H
#define IPS_ORACLE_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

size_t   oracle_elem_bytes(int type);
uint64_t oracle_splitmix64_next(uint64_t* state);
uint64_t oracle_mulhi64(uint64_t a, uint64_t b);
int      oracle_key_less(int type, const void* a, const void* b);
int      oracle_sort(void* data, uint64_t n, int type);
uint32_t oracle_alpha(uint64_t n);
uint32_t oracle_adaptive_k(uint64_t n, uint32_t k, uint32_t n0);
uint64_t oracle_task_seed(uint64_t seed, uint64_t l, uint32_t level);
int      oracle_sample_step(const void* data, uint64_t l, uint64_t n, int type,
                            uint32_t k, uint32_t n0, uint64_t seed, uint32_t level,
                            int eq_mode, uint32_t* info, void* splitters_out,
                            void* sample_out);
uint32_t oracle_classify(int type, const void* e, const void* splitters,
                         uint32_t K, int eq);
int      oracle_histogram(const void* data, uint64_t n, int type,
                          const void* splitters, uint32_t K, int eq,
                          uint64_t* counts);
int      oracle_radix_digit_info(const void* data, uint64_t n, int type,
                                 uint32_t* info);
int      oracle_radix_histogram(const void* data, uint64_t n, int type,
                                uint32_t shift, uint32_t width, uint64_t* counts);
int      oracle_check_partition(const void* data, uint64_t n, int type,
                                const void* splitters, uint32_t K, int eq,
                                const uint64_t* bucket_start, uint64_t* bad_index);
uint64_t oracle_count_less(const void* data, uint64_t n, int type, const void* v,
                           int or_equal);
#ifdef __cplusplus
}
#endif
#endif
