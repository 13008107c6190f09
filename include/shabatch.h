/*
 * shabatch.h -- C ABI of the batched SHA-256 offload in libaesctr.so.
 *
 * A second pure offload beside AES-CTR: the paper names bulk hashing among
 * the computations that are safe to move off the request path (Sec. 5, the
 * pure-offload class).  One call hashes many independent messages with
 * SHA-256 as FIPS 180-4 defines it (padding Sec. 5.1.1, hash computation
 * Sec. 6.2.2); each digest is the standard 32-byte big-endian value, bit for
 * bit.  SHA-256 is sequential within a message, so the GPU parallelism is
 * across messages: the call pays off for many messages at once.
 *
 * Conventions follow aesctr.h: statuses are aes_status_t (AES_OK = 0,
 * negative on error, aes_strerror() names them; AES_EDEVICE also sets
 * aes_last_device_error()); "stream" is a hipStream_t passed as void*.
 */
#ifndef SHABATCH_H
#define SHABATCH_H

#include <stddef.h>
#include <stdint.h>

#include "aesctr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One message.  in: len bytes of device memory (any alignment; NULL allowed
 * when len == 0).  digest: 32 bytes of device memory that receive the
 * digest; it must not overlap this message's input.  reserved must be 0.
 * The caller owns both buffers; they must stay valid until the stream
 * reaches the call. */
typedef struct {
    const void *in;
    uint64_t len;
    void *digest;
    uint64_t reserved;
} sha256_desc_t;

/* Hash n messages (n == 0 is a no-op).  The descriptor array is copied at
 * call time: the caller may reuse it when the call returns.  Asynchronous on
 * `stream`; the descriptors travel through staging that the library keeps
 * per (device, stream) until the process ends: two pinned host buffers and
 * two device buffers of 4 MiB each, and a side stream for their uploads (an
 * engine's streams hand theirs to the next engine when it is destroyed).
 * Calls with more than 131,072 messages are cut into launches of that many;
 * the call returns once the last launch is queued, which may wait for the
 * launch two before it.  A message may be at most 2^61 - 1
 * bytes (the bit length must fit the 64-bit length field).
 * Errors: AES_EINVAL (null desc with n > 0, null digest, null in with
 * len > 0, reserved != 0, a stream that is being captured -- a captured
 * graph would keep reading staging that later calls rewrite), AES_ERANGE (message too long), AES_EOVERLAP
 * (digest overlaps its input), AES_ENOMEM, AES_EDEVICE.  Thread-safe for
 * calls on distinct streams; calls on one stream are serialised. */
int sha256_batch(const sha256_desc_t *desc, size_t n, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SHABATCH_H */
