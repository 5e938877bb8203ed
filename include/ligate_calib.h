/*
 * Peak-calibration kernels of libligate: measurement helpers that give the roofline figures the
 * screen is compared with.  They compute nothing of the docking method.
 *
 * Conventions as in ligate_dock.h: caller-owned device memory, asynchronous on `stream`, return
 * DOCK_OK or a negative DOCK_ERR_* code (detail in dock_last_error()).
 */
#ifndef LIGATE_CALIB_H
#define LIGATE_CALIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Vector FP32 FMA throughput: `blocks` blocks of 256 threads, each thread running `iters`
 * iterations of 16 independent non-packed FMA chains (32 FLOP per chain step), i.e.
 * blocks * 256 * iters * 16 * 2 FLOP.  d_out [blocks * 256] receives each thread's chain sum so
 * the work cannot be removed.  1 <= blocks <= 2^20, 1 <= iters <= 2^24.
 */
int calib_fma_f32(int32_t blocks, int32_t iters, float *d_out, void *stream);

/*
 * Cache-resident read bandwidth: each of `blocks` blocks of 256 threads reads all `bytes` bytes at
 * d_buf (16-byte aligned; bytes a positive multiple of 16384) `reps` times with 16-byte loads,
 * every wavefront step covering a contiguous 1 KiB, blocks starting at different offsets.  A
 * buffer larger than the L1 caches and smaller than one L2 is then served by the L2 caches.
 * Bytes read = blocks * reps * bytes.  d_out [blocks * 256] receives per-thread sums.
 * 1 <= blocks <= 2^20, 1 <= reps <= 2^20.
 */
int calib_cache_read(const void *d_buf, size_t bytes, int32_t reps, int32_t blocks, float *d_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif
