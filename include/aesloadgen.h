/*
 * aesloadgen.h -- C ABI of libaesloadgen.so: open-loop load generation for
 * the serving engine of libaesctr.so (test and benchmark tooling).
 *
 * The paper measures latency under load with open-loop Poisson arrivals and
 * reports median and tail latency (Sec. 6, "Latency under offered load").
 * These calls replay a given arrival schedule against either
 *   - the engine (aes_submit_at with the scheduled arrival time, so time a
 *     request waits because the generator fell behind is still counted), or
 *   - the synchronous per-request path: one aes_ctr_crypt followed by a
 *     stream synchronisation at a time, as a server that blocks on its
 *     offload would, with each request's latency counted from its scheduled
 *     arrival.
 * Latency = completion observed - scheduled arrival, in microseconds.
 */
#ifndef AESLOADGEN_H
#define AESLOADGEN_H

#include <stddef.h>
#include <stdint.h>

#include "aesctr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double wall_s;          /* first scheduled arrival -> last completion */
    double achieved_rps;    /* completed requests / wall_s */
    double gbps;            /* payload bytes / wall_s / 1e9 */
    double max_lag_us;      /* worst lateness of a submission vs its schedule */
    double p50_us, p99_us, p999_us, max_us;
    uint64_t completed, errors;
} aes_load_result_t;

/* Replay arrivals against an engine.  pool: request descriptors reused in
 * round-robin order (i mod npool); arrival_s: n non-decreasing offsets in
 * seconds from the start.  Up to four submitting threads share the schedule
 * (arrival i goes to thread i mod T), each spinning until its request's
 * arrival time; a collector thread retires tickets.  Blocks until every
 * request completed.  The engine's statistics are reset at the start.
 * Errors: AES_EINVAL (null pointers, npool == 0), or the first error a
 * submission returned (the run stops submitting at that point). */
int aes_load_engine(aes_engine_t *e, const aes_ctr_desc_t *pool, size_t npool, const double *arrival_s,
                    size_t n, aes_load_result_t *out);

/* The same schedule through the synchronous per-request path on `stream`
 * (device buffers).  Errors: AES_EINVAL, or an aes_ctr_crypt error. */
int aes_load_sync(const aes_ctr_desc_t *pool, size_t npool, const double *arrival_s, size_t n,
                  void *stream, aes_load_result_t *out);

/* The synchronous per-request path for host-resident payloads: the pool's
 * in/out are pinned host memory (hipHostMalloc); each request is copied to
 * the device buffer dev_buf (dev_bytes long, at least the largest request),
 * encrypted there in place, copied back to its out buffer and synchronised,
 * one at a time, on `stream`.  Errors: AES_EINVAL (null pointers, a request
 * longer than dev_bytes), AES_EDEVICE (a failed copy), or an aes_ctr_crypt
 * error. */
int aes_load_sync_host(const aes_ctr_desc_t *pool, size_t npool, const double *arrival_s, size_t n,
                       void *dev_buf, size_t dev_bytes, void *stream, aes_load_result_t *out);

#ifdef __cplusplus
}
#endif
#endif /* AESLOADGEN_H */
