/* Measurement probes that verify, on the GPU at hand, the peaks the roofline figures are
 * quoted against.  They are not part of the counting path.  Device pointers; the caller
 * owns every buffer; return 0 on success, 1 invalid argument, 3 buffer too small, 4 HIP
 * error.  Both synchronise the stream. */
#pragma once
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* LDS read bandwidth: blocks_per_cu (1 or 2) blocks of 1024 lanes per CU read 16-byte
 * vectors of a 64 KiB LDS buffer at conflict-free addresses 20000 times each;
 * *bytes_per_s = bytes read / elapsed.  scratch: device uint32 of at least
 * blocks * 1024 words (one result per lane, keeps the loads live). */
int arb_probe_lds_read(uint32_t *scratch, int64_t scratch_words, int blocks_per_cu, double *bytes_per_s,
                       void *stream);

/* Device-memory copy bandwidth: dst = src (bytes, a multiple of 16) reps times after one
 * warm-up copy; *bytes_per_s = 2 * bytes * reps / elapsed (read plus write). */
int arb_probe_copy(const void *src, void *dst, int64_t bytes, int reps, double *bytes_per_s, void *stream);

#ifdef __cplusplus
}
#endif
