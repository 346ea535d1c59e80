/*
 * libspd_ceilings: microbenchmarks of the MI355X ceilings behind the scan's design (not part of
 * the detection path).  Each call launches one kernel on `stream` (a hipStream_t as void*) and
 * returns 0, -1 for a bad argument (nothing launched) or -3 for a launch error.  Buffers are device
 * memory owned by the caller; every access is masked into the stated size.
 *
 *  - spd_ceil_stream_read: reads `bytes` (a multiple of 16, 16-byte aligned) with non-temporal
 *    16-byte loads; `sink` receives a word only on a practically impossible checksum.
 *  - spd_ceil_atomic_or: n_ops device-scope relaxed atomicOr on uniformly random words of a table
 *    of `words` 32-bit words (a power of two), the direct scan's update.
 *  - spd_ceil_store16: n_ops plain 16-bit stores to uniformly random entries of a table of `elems`
 *    entries (a power of two), the sliding scan's stamp update.
 *  - spd_ceil_lds_atomic_or: `blocks` workgroups of spd_ceil_block() threads, each thread n_iter
 *    LDS atomicOr on random words of a 128 KiB bitmap, the binned scan's apply phase.
 */
#ifndef SPD_CEILINGS_H
#define SPD_CEILINGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int spd_ceil_stream_read(const void *p, uint64_t bytes, uint32_t *sink, void *stream);
int spd_ceil_atomic_or(uint32_t *table, uint64_t words, uint64_t n_ops, uint64_t seed, void *stream);
int spd_ceil_store16(uint16_t *table, uint64_t elems, uint64_t n_ops, uint64_t seed, void *stream);
int spd_ceil_lds_atomic_or(uint32_t blocks, uint32_t n_iter, uint32_t *sink, void *stream);
uint32_t spd_ceil_block(void);

#ifdef __cplusplus
}
#endif

#endif /* SPD_CEILINGS_H */
