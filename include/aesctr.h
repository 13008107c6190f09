/*
 * aesctr.h -- C ABI of libaesctr.so, bulk AES counter-mode encryption of
 * request payloads on an AMD Instinct MI355X (gfx950).
 *
 * The operation is the offload the paper measures (Sec. 6, experimental
 * setup: AES on its own GPU stream, completion polled by an event query;
 * block sizes 4 KiB to 8 MiB, Appendix A, Table 2), with the cipher fixed as:
 *   - AES-128 or AES-256 (FIPS-197: Cipher Sec. 5.1, KeyExpansion Sec. 5.2);
 *   - counter mode (NIST SP 800-38A Sec. 6.5): the counter block of block j is
 *     nonce (12 bytes) || BE32((ctr0 + j) mod 2^32), i.e. a 96-bit nonce and a
 *     32-bit big-endian counter that wraps without touching the nonce (the
 *     inc32 function of SP 800-38A Appendix B);
 *   - C = P XOR (O_0 || O_1 || ...)[0:len]: the last partial block uses the
 *     leading bytes of its keystream block.  Encryption and decryption are the
 *     same call.
 * Results are bit-exact; there is exactly one correct output.
 *
 * Conventions for every call:
 *   - Return value: AES_OK (0) or a negative aes_status_t.  aes_strerror()
 *     names it.  Argument errors are reported before any device work.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *   - The library links libamdhip64.so.7.  A process must hold one HIP
 *     runtime: where another component brings its own copy (PyTorch's wheels
 *     ship one under torch/lib), load that component first so this library
 *     binds to the same copy; streams of one runtime mean nothing to another.
 *   - "device pointer" means memory of the current HIP device (hipMalloc,
 *     a torch CUDA tensor, ...).  Calls that take device pointers are
 *     asynchronous on the given stream; buffers must stay valid until the
 *     stream reaches the work.
 *   - The library copies every scalar, schedule, nonce and descriptor at
 *     call time; the caller may reuse those host objects once a call returns.
 *   - in == out (in place) is allowed; any other overlap of [in, in+len) and
 *     [out, out+len) is rejected with AES_EOVERLAP.  Any alignment works;
 *     16-byte-aligned in and out take the fast path.
 *   - len == 0 is a no-op.  len > 2^32 * 16 bytes would reuse counter blocks
 *     within one message and is rejected with AES_ERANGE.
 */
#ifndef AESCTR_H
#define AESCTR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AES_OK = 0,
    AES_EINVAL = -1,      /* bad argument (null pointer, bad key size, ...) */
    AES_ENOMEM = -2,      /* host or device allocation failed */
    AES_EAGAIN = -3,      /* engine: request does not fit the memory budget now */
    AES_ERANGE = -4,      /* message longer than 2^32 blocks */
    AES_EDEVICE = -5,     /* a HIP runtime call failed / no usable device */
    AES_ENOTFOUND = -6,   /* engine: unknown or already-retired ticket */
    AES_ETIMEDOUT = -7,   /* engine: aes_wait deadline passed */
    AES_EOVERLAP = -8,    /* input and output partially overlap */
    AES_ECLOSED = -9,     /* engine is shutting down */
    AES_ECANCELED = -10,  /* engine: request dropped at shutdown */
    AES_ETOOBIG = -11     /* more requests than a fixed-size table holds */
} aes_status_t;

/* Human-readable name of a status value (static string, never NULL). */
const char *aes_strerror(int status);

/* Name of the HIP error (e.g. "hipErrorOutOfMemory") behind the calling
 * thread's latest AES_EDEVICE, or "hipSuccess" if there was none; a static
 * string, never NULL.  Errors met by an engine's driver thread are recorded
 * on that thread and surface as AES_EDEVICE tickets. */
const char *aes_last_device_error(void);

/* ---------------------------------------------------------------------- */
/* Key schedule (FIPS-197 Sec. 5.2)                                        */
/* ---------------------------------------------------------------------- */

/* Expanded key.  rk[i] is the schedule word w[i] of FIPS-197 Sec. 5.2,
 * packed big-endian (w = k0<<24 | k1<<16 | k2<<8 | k3); 4*(nr+1) words are
 * valid (44 for AES-128, 60 for AES-256).  Plain data owned by the caller. */
typedef struct {
    uint32_t rk[60];
    int32_t nr;         /* 10 or 14 */
    int32_t key_bits;   /* 128 or 256 */
} aes_sched_t;

/* Expand a 16-byte (key_bits = 128) or 32-byte (key_bits = 256) key into
 * *out.  Host only; never touches a device.
 * Errors: AES_EINVAL for null pointers or key_bits not in {128, 256}. */
int aes_expand_key(const uint8_t *key, int key_bits, aes_sched_t *out);

/* ---------------------------------------------------------------------- */
/* Single buffer                                                           */
/* ---------------------------------------------------------------------- */

/* out[0:len] = in[0:len] XOR keystream(sched, nonce, ctr0), as defined above.
 * sched: host pointer to an expanded key; nonce: host pointer to 12 bytes;
 * in, out: device pointers (may be equal).  One kernel launch on stream.
 * Errors: AES_EINVAL (null sched/nonce, null in/out with len > 0, bad
 * sched->nr/key_bits), AES_ERANGE, AES_EOVERLAP, AES_EDEVICE (no device /
 * launch failure). */
int aes_ctr_crypt(const aes_sched_t *sched, const uint8_t nonce[12], uint32_t ctr0,
                  const void *in, void *out, size_t len, void *stream);

/* Kernel variants of the keystream (all give identical output). */
typedef enum {
    AES_VARIANT_AUTO = 0,      /* tuned choice */
    AES_VARIANT_TTABLE = 1,    /* round T-tables in LDS, replicated per bank */
    AES_VARIANT_BITSLICE = 2,  /* bitsliced: 32 blocks per 32-bit word */
    AES_VARIANT_VPERM = 3      /* no memory tables: the S-box through GF(2^4)
                                  with 16-entry nibble lookups by v_perm_b32
                                  (Hamburg's vector-permute AES, CHES 2009) */
} aes_variant_t;

/* Launch shape.  Zero in any field means "tuned default".
 *   variant          aes_variant_t
 *   blocks_per_lane  16-byte blocks one lane handles per loop step (1, 2, 4)
 *   wg_size          threads per workgroup (multiple of 64, <= 1024; the
 *                    bitsliced and vector-permute kernels: 64..256)
 *   grid             workgroups launched (persistent grid-stride loop)
 *   lds_copies       T-table replication (32 or 64 copies per table), T-table only
 *   lds_tables       T-tables held in LDS, T-table only: 4 (T0..T3, 32 copies,
 *                    128 KiB) or 2 (T0 and T2, T1 and T3 by rotation: 32
 *                    copies in 64 KiB, or 64 copies in 128 KiB).  64 copies
 *                    imply 2 tables; 64 copies of 4 tables is AES_EINVAL.
 *   wave_groups      how the T-table kernel's first chunk gets rounds 1-2
 *                    (counter-mode caching shares them across groups of 256
 *                    counters).  Input: 0 = the shape rule's choice, 1 =
 *                    every wave computes its own group constants (2 tables
 *                    of 32 copies, 1-2 blocks per lane, <= 512 threads), 2 =
 *                    rounds 1-2 in full for the first chunk, no group
 *                    constants (1-2 blocks per lane, <= 512 threads), 3 =
 *                    wave 0 computes them for its workgroup; a mode the
 *                    shape is not built for is AES_EINVAL.  Output (from
 *                    aes_ctr_launch_shape): the mode used, 1, 2, or 0 for
 *                    wave 0. */
typedef struct {
    int32_t variant;
    int32_t blocks_per_lane;
    int32_t wg_size;
    int32_t grid;
    int32_t lds_copies;
    int32_t lds_tables;
    int32_t wave_groups;
    int32_t reserved;
} aes_launch_cfg_t;

/* aes_ctr_crypt with an explicit launch shape (cfg may be NULL = defaults).
 * Same output for every valid cfg.  Errors as aes_ctr_crypt, plus AES_EINVAL
 * for an unsupported field value. */
int aes_ctr_crypt_cfg(const aes_sched_t *sched, const uint8_t nonce[12], uint32_t ctr0,
                      const void *in, void *out, size_t len,
                      const aes_launch_cfg_t *cfg, void *stream);

/* The launch shape aes_ctr_crypt_cfg would use for a len-byte message with
 * this key size and cfg (NULL = defaults): the default shape, or the tune
 * cache's entry for the same floor(log2(len)) where it has one, overridden
 * by cfg's non-zero fields,
 * with the grid clamped to the work.  All fields of *out are set (variant 1,
 * 2 or 3, never AUTO; lds_copies and lds_tables 0 for the kernels without
 * T-tables).  Host only; it
 * needs the current device's CU count.  Errors: AES_EINVAL (null out, key
 * size not 128/256, bad cfg), AES_EDEVICE. */
int aes_ctr_launch_shape(int key_bits, size_t len, const aes_launch_cfg_t *cfg, aes_launch_cfg_t *out);

/* ---------------------------------------------------------------------- */
/* Batch: many requests, one launch                                        */
/* ---------------------------------------------------------------------- */

/* One request.  in/out are device pointers (in == out allowed), sched a host
 * pointer to its expanded key (AES-128 and AES-256 may be mixed), nonce and
 * ctr0 its counter-block parameters.  flags: 0 for AES-CTR; for the engine
 * (aes_submit) also AES_FLAG_SHA256, which makes the request a SHA-256 hash
 * of in[0..len) into the 32-byte digest at out (shabatch.h's semantics;
 * sched, nonce and ctr0 are ignored and sched may be NULL). */
enum { AES_FLAG_SHA256 = 1 };

typedef struct {
    const void *in;
    void *out;
    uint64_t len;
    const aes_sched_t *sched;
    uint8_t nonce[12];
    uint32_t ctr0;
    uint32_t flags;
    uint32_t reserved;
} aes_ctr_desc_t;

/* Encrypt n requests with one persistent kernel launch over a device
 * descriptor table (the shape of the paper's job queue, Listing 1, with every
 * job handed to the device at once).  The descriptors, schedules and tile
 * index are staged in pinned host memory and copied by a node of a captured
 * HIP graph, replayed on each call.  A batch of at most 8 requests skips the
 * table: its records travel in the kernel's argument block, so no copy
 * precedes the launch.  Each request's output equals
 * aes_ctr_crypt on that request alone.  n == 0 is a no-op.
 * Errors: AES_EINVAL (null desc with n > 0, null sched, flags != 0, a
 * stream that is being captured -- the call launches its own graph and its
 * staging is rewritten by later calls), AES_ERANGE, AES_EOVERLAP (per
 * request), AES_ENOMEM, AES_EDEVICE.  Thread-safe for calls on distinct
 * streams; calls on one stream are serialised. */
int aes_ctr_crypt_batch(const aes_ctr_desc_t *desc, size_t n, void *stream);

/* Batch launch shape: tile_bytes (bytes of a request one wave-tile covers,
 * multiple of 1024), wg_size, grid, blocks_per_lane; zero = default (tiles
 * sized to the batch, about sixteen per CU within 2-64 KiB; 2 blocks per
 * lane; 1024-thread workgroups, one per CU; a tune cache may override).
 * use_graph: 1 = captured graph, 0 = plain copy + launch; a call without cfg
 * uses the graph; batches of at most 8 requests use neither: their kernel
 * has 256-thread workgroups, a wave per tile up to twice `grid` workgroups,
 * and takes tile_bytes and blocks_per_lane from cfg like the table kernel. */
typedef struct {
    int32_t tile_bytes;
    int32_t wg_size;
    int32_t grid;
    int32_t blocks_per_lane;
    int32_t use_graph;
    int32_t reserved[3];
} aes_batch_cfg_t;

int aes_ctr_crypt_batch_cfg(const aes_ctr_desc_t *desc, size_t n,
                            const aes_batch_cfg_t *cfg, void *stream);

/* aes_ctr_crypt_batch for callers that cannot allocate (code that must not
 * call hipMalloc or create library state at run time: tight serving loops,
 * harnesses that forbid allocation).  It allocates nothing, host or device:
 * the descriptor table lives in a fixed device array of the library's, 1.25
 * MiB per GPU (held until the process ends), and is built on the calling
 * thread's stack and copied in with hipMemcpyAsync from that pageable memory
 * on `stream`, then the same persistent batch kernel runs over it.  Every
 * request's key travels inline.  Output equals aes_ctr_crypt_batch's (and so
 * aes_ctr_crypt's on each request alone).
 * Limits: at most 4096 requests per call (more: AES_ETOOBIG, before any
 * device work).  All calls on one GPU share that array: calls that overlap
 * on one GPU (another thread, another stream) race and must be serialised by
 * the caller; a call may be made again as soon as the previous one returned
 * on the same stream.  Not for a stream under graph capture (AES_EINVAL).
 * Errors: as aes_ctr_crypt_batch, plus AES_ETOOBIG. */
int aes_ctr_crypt_batch_noalloc(const aes_ctr_desc_t *desc, size_t n, void *stream);

/* ---------------------------------------------------------------------- */
/* Engine: submit -> (caller suspends) -> poll / wait -> resume            */
/* ---------------------------------------------------------------------- */
/*
 * The executor half of the paper's three-step reroute (Sec. 3: submit the
 * offload to a background executor, suspend the request with the server's
 * own deferred-response primitive, resume it on completion; Listing 1).
 * aes_submit hands a request to the engine and returns a ticket at once; the
 * engine admits requests while the bytes in flight stay within a device
 * memory budget, coalesces everything admitted into batched launches on
 * several streams (continuous batching: requests arriving while others run
 * join the next launch), detects completion by polling HIP events (as the
 * paper polls its stream's event), and retires tickets.  The ticket is
 * registered before the work can complete, so completion cannot race the
 * caller's suspension (the ordering of Listing 1).
 */
typedef struct aes_engine aes_engine_t;

typedef struct {
    uint64_t budget_bytes;      /* bytes in flight (0 = 4 GiB): the buffers of
                                   every admitted request (input and output,
                                   counted once when in place; a hash request's
                                   message and digest) plus its staged records
                                   (aes_engine_request_overhead() bytes for a
                                   cipher request)                             */
    int32_t n_streams;          /* concurrent batch launches (0 = 2)           */
    int32_t max_batch_reqs;     /* requests per launch (0, or more than 4096,
                                   = 4096)                                     */
    uint64_t max_batch_bytes;   /* payload bytes per launch (0 = 256 MiB or the
                                   budget if smaller; a larger request runs
                                   alone)                                      */
    int32_t key_slots;          /* resident key schedules (0 .. 65536; 0 = none):
                                   the engine keeps this many expanded keys in
                                   a device table of its own (256 bytes each).
                                   A request whose key is resident is launched
                                   with a slot index instead of its schedule;
                                   a request whose key is not carries it
                                   inline and, when a slot is free or the
                                   least recently used slot is not read by a
                                   launch in flight, installs it there for
                                   later requests.  Outputs do not depend on
                                   it.                                         */
    int32_t host_buffers;       /* 1: in/out are pinned host memory
                                   (hipHostMalloc) that the kernel reads and
                                   writes directly over PCIe (zero-copy)       */
    int32_t device;             /* HIP device ordinal (-1 = current)           */
    int32_t reserved[5];
} aes_engine_cfg_t;

typedef struct {
    uint64_t submitted, completed, rejected, batches;
    uint64_t bytes_completed;       /* payload bytes of the completed requests */
    uint64_t budget_high_water;     /* max bytes admitted at once */
    uint64_t queued_now, inflight_now;
    double mean_batch_reqs;
    double p50_us, p99_us, p999_us; /* arrival (submit) -> completion seen by the poller */
    double busy_s;                  /* wall time with at least one launch in flight */
    double max_us;                  /* slowest request, same clock as p50_us */
    uint64_t key_hits;              /* cipher requests launched with their key read
                                       from a resident slot (key_slots > 0)    */
    uint64_t key_misses;            /* cipher requests launched with their key inline
                                       (key_slots > 0): a key not resident yet, or
                                       one whose install was still in flight   */
} aes_stats_t;

/* Bytes the admission budget charges a cipher request beyond its buffers:
 * its descriptor record and an inline key record (64 + 256). */
uint64_t aes_engine_request_overhead(void);

/* Create an engine (cfg may be NULL = defaults).  Starts its driver thread,
 * which forms and launches batches and polls their completion events.
 * Errors: AES_EINVAL, AES_ENOMEM, AES_EDEVICE. */
int aes_engine_create(const aes_engine_cfg_t *cfg, aes_engine_t **out);

/* Stop accepting work, finish everything submitted, release resources.
 * Tickets not yet retired by poll/wait are dropped with the engine. */
int aes_engine_destroy(aes_engine_t *e);

/* Submit one request (*d copied, its schedule copied).  Never blocks on the
 * device: a request that does not fit the budget now waits in FIFO order.
 * Cipher and hash requests (flags = AES_FLAG_SHA256) may be mixed; a launch
 * runs the batch kernel for the cipher requests and the hash kernel for the
 * hash requests back to back on its stream.
 * The engine launches on streams of its own, not ordered after any stream
 * of the caller: the input must hold its final contents when aes_submit is
 * called, and neither buffer may be touched again until the ticket
 * completes.
 * Takes no lock; when 32768 requests are already queued (admitted requests
 * do not count) the call yields until the engine takes some.  Thread-safe;
 * calls racing with aes_engine_destroy are not allowed.
 * Errors: AES_EINVAL, AES_ERANGE, AES_EOVERLAP, AES_EAGAIN (larger than the
 * whole budget), AES_ECLOSED. */
int aes_submit(aes_engine_t *e, const aes_ctr_desc_t *d, uint64_t *ticket);

/* aes_submit with an explicit arrival time: t_arrival_ns on the
 * CLOCK_MONOTONIC (steady) clock, the moment the request reached the server.
 * Latency statistics then count from arrival rather than from the call, so a
 * server that queued the request before submitting it (or a load generator
 * running behind schedule) is charged for that wait. */
int aes_submit_at(aes_engine_t *e, const aes_ctr_desc_t *d, int64_t t_arrival_ns, uint64_t *ticket);

/* 1 = done (the ticket is retired by this call), 0 = pending, < 0 = error
 * (AES_ENOTFOUND, AES_EDEVICE if the request's launch failed, AES_ECANCELED).
 * Never blocks and takes no lock.  A finished ticket keeps its result until
 * it is retired or until 2^20 later tickets have been issued (then
 * AES_ENOTFOUND). */
int aes_poll(aes_engine_t *e, uint64_t ticket);

/* Block until the ticket completes or timeout_us passes (< 0 = forever):
 * spins for up to 20 us, then sleeps until a completion signals it.
 * Returns AES_OK and retires the ticket, AES_ETIMEDOUT (ticket stays
 * pending), or an error as aes_poll. */
int aes_wait(aes_engine_t *e, uint64_t ticket, int64_t timeout_us);

/* Counters and latency percentiles since creation (or the last reset). */
int aes_engine_stats(aes_engine_t *e, aes_stats_t *out);
int aes_engine_reset_stats(aes_engine_t *e);

/* A file descriptor (eventfd) that becomes readable whenever tickets
 * complete, for event loops that want to sleep instead of polling.  Owned by
 * the engine. */
int aes_engine_completion_fd(aes_engine_t *e);

#ifdef __cplusplus
}
#endif
#endif /* AESCTR_H */
