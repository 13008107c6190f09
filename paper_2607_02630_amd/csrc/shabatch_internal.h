// shabatch_internal.h -- shared between the batched SHA-256 host code and its
// kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aesctr_internal.h"

namespace aesctr {

// One message as the kernel sees it (device addresses).
struct ShaRecord {
    uint64_t in;
    uint64_t len;
    uint64_t digest;
    uint64_t pad;
};

constexpr uint32_t kMaxShaBatch = 1u << 17;   // records per launch (4 MiB table)

int launch_sha256_batch(const ShaRecord *dev_recs, uint32_t n, int grid, hipStream_t st);

// Validation of one message (AES_OK, AES_EINVAL, AES_ERANGE, AES_EOVERLAP).
int check_sha(const void *in, uint64_t len, const void *digest);

// Orders n records longest first, stages them on the (device, stream)
// context and launches the hash kernel (kMaxShaBatch per launch).
int launch_sha_records(int device, hipStream_t st, const ShaRecord *recs, size_t n, int num_cus);

// Returns stream st's staging context to the device's free list (as
// release_batch_stream does for the cipher batch).
void release_sha_stream(int device, hipStream_t st);

}  // namespace aesctr
