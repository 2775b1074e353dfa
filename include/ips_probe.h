/* Memory-system probes of the GPU the library sorts on.
 *
 * Not part of sorting.  The sort's kernels are measured against the HBM
 * peak; these probes measure what plain access patterns reach on the same
 * device, so that a kernel's fraction of the peak can be read beside the
 * fraction a kernel of the same shape without any sorting work reaches:
 *  - IPS_PROBE_COPY: read `src`, write `dst`, 16-byte accesses, streaming
 *    (the pattern of classification and of the LDS tier, without their
 *    on-chip work);
 *  - IPS_PROBE_READ / IPS_PROBE_WRITE: one direction only;
 *  - IPS_PROBE_BLOCKS: copy blocks of `block_bytes` from pseudo-random
 *    source blocks to pseudo-random destination blocks (every block of
 *    `src` read once, every block of `dst` written once; the block
 *    permutation's data movement without its pointer chain);
 *  - IPS_PROBE_CHAIN: `groups` groups of 16 lanes, each repeating
 *    (a returning 64-bit atomic add on a pseudo-random word of `table`) ->
 *    (load of one block of `block_bytes` at an address derived from the
 *    atomic's result) -> (store of the block to another derived address):
 *    the dependent chain one group of the block permutation runs per block
 *    (Section 4.1, block permutation), without its bookkeeping.
 *
 * Arguments: `src` and `dst` are device buffers of `bytes` bytes (16-byte
 * aligned, `bytes` a multiple of 16; IPS_PROBE_READ does not write `dst`
 * beyond its first 4 bytes and IPS_PROBE_WRITE does not read `src`, but
 * both must be valid); for IPS_PROBE_BLOCKS and IPS_PROBE_CHAIN,
 * `block_bytes` is 256, 512, 1024 or 2048 and bytes / block_bytes is a
 * power of two; IPS_PROBE_CHAIN also needs `table`, a device array of
 * `table_words` (a power of two) 64-bit words that it increments, and
 * `groups` >= 1 (bytes / (groups * block_bytes) blocks per group, at least
 * one); other modes ignore `block_bytes`, `table`, `table_words` and
 * `groups`.  The contents of `dst` afterwards are the probe's, not a
 * result.  The probe launches once untimed, then `reps` (>= 1) times
 * between two HIP events on `stream` (null: the null stream) and returns
 * the mean milliseconds per launch in *ms_per_rep; the call blocks until
 * the second event has completed.  Bytes moved per launch: 2 * bytes for
 * COPY and BLOCKS (read and written), `bytes` for READ and WRITE, and
 * 2 * groups * block_bytes * floor(bytes / (groups * block_bytes)) for
 * CHAIN.
 *
 * Errors: IPS_E_INVALID_ARG (before any HIP call) for a bad mode, null or
 * misaligned buffers, sizes that break the rules above, reps = 0 or a null
 * `ms_per_rep`; IPS_E_HIP when a HIP call fails. */
#ifndef IPS_PROBE_H
#define IPS_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IPS_PROBE_COPY 0
#define IPS_PROBE_READ 1
#define IPS_PROBE_WRITE 2
#define IPS_PROBE_BLOCKS 3
#define IPS_PROBE_CHAIN 4

int ips_probe_memory(int mode, const void* src, void* dst, uint64_t bytes, uint32_t block_bytes,
                     uint64_t* table, uint32_t table_words, uint32_t groups, uint32_t reps, void* stream,
                     float* ms_per_rep);

#ifdef __cplusplus
}
#endif

#endif /* IPS_PROBE_H */
