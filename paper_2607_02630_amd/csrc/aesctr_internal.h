// aesctr_internal.h -- shared declarations of the library's host code and
// its kernels.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/aesctr.h"

namespace aesctr {

// Everything one keystream needs, in the layout the kernels use.  A state
// column is a little-endian word whose byte r is row r, so a FIPS-197
// schedule word w (big-endian packed) becomes bswap(w).
struct KeyMaterial {
    uint32_t rk[60];    // round keys as column words, rk[4*round + column]
    uint32_t k1[4];     // round-1 output columns minus their counter term
    uint32_t x0;        // round-0 key of the counter column (column 3)
    int32_t nr;         // 10 or 14
};

// Counter-mode caching (Bernstein and Schwabe, "New AES software speed
// records", 2008): of the four round-0 columns only column 3 (the counter)
// varies between blocks, and after ShiftRows each round-1 output column takes
// exactly one byte of it.  The other three T-table terms of every round-1
// column and its round key are folded into k1 once per request, so round 1
// costs four lookups per block instead of sixteen:
//   x   = bswap(ctr) ^ x0
//   u_c = k1[c] ^ T_(3-c)[byte (3-c) of x]
void make_key_material(const aes_sched_t &s, const uint8_t nonce[12], KeyMaterial *km);

// Resolved launch shape of the single-buffer kernels.
struct Shape {
    int variant;        // AES_VARIANT_TTABLE or AES_VARIANT_BITSLICE
    int bpl;            // 16-byte blocks per lane per loop step
    int wg;             // threads per workgroup
    int grid;           // workgroups
    int copies;         // T-table replication (32 or 64 copies per table)
    int tables;         // T-tables in LDS: 4 (T0..T3) or 2 (T0, T2)
    bool wave_groups;   // each wave computes its first chunk's group constants
};

// Arguments of the single-buffer kernels (passed by value in the kernarg
// segment; the round keys become scalar registers).
struct CtrArgs {
    const uint8_t *in;
    uint8_t *out;
    uint64_t len;       // bytes
    uint32_t ctr0;
    uint32_t x0;
    uint32_t k1[4];
    uint32_t rk[60];
};

// Device facts the launchers need, cached per device.
struct DeviceInfo {
    int ordinal;
    int num_cus;
    int max_lds_per_block;
};
int device_info(DeviceInfo *out);   // AES_OK or AES_EDEVICE

// Device-error bookkeeping for aes_last_device_error(): the HIP error behind
// the calling thread's latest AES_EDEVICE.  note_device_error() keeps e if it
// is an error; device_error() takes (and clears) HIP's pending error, keeps
// it and returns AES_EDEVICE.  Launchers clear HIP's pending error before a
// launch (it may have been left by other code in the process) and read it
// back with launch_status().
void note_device_error(hipError_t e);
int device_error();
int launch_status();

// Argument checks shared by the entry points (AES_OK or an error status).
int check_sched(const aes_sched_t *s);
int check_buffers(const void *in, const void *out, uint64_t len);

// Launchers (return AES_OK or AES_EDEVICE).
int launch_ctr_ttable(const CtrArgs &a, int nr, const Shape &sh, hipStream_t st);
int launch_ctr_bitslice(const CtrArgs &a, int nr, const Shape &sh, hipStream_t st);

// ---- Batched launch -------------------------------------------------------
// Device table = BatchHeader followed by n BatchDesc records.  Requests are cut
// into tiles of tile_blocks 16-byte blocks; tile0 is a request's first tile
// (exclusive prefix sum), so the tile t belongs to the last request whose
// tile0 <= t.  next is the work counter the waves claim tiles from; every
// upload carries it as 0.
constexpr int kMaxBatch = 4096;          // requests per launch (tile0 index in LDS)
constexpr int kMaxBatchGrid = 1 << 20;   // workgroups per batch launch (keeps tile indices in 32 bits)

struct alignas(64) BatchHeader {
    uint32_t n;
    uint32_t total_tiles;
    uint32_t tile_blocks;
    uint32_t next;
    uint32_t pad[12];
};

struct alignas(64) BatchDesc {
    uint64_t in, out, len;
    uint32_t ctr0, x0, nr, aligned;     // aligned: in and out 16-byte aligned
    uint32_t k1[4];
    uint32_t tile0;
    uint32_t pad[5];
    uint32_t rk[60];
};
static_assert(sizeof(BatchHeader) == 64, "header layout");
static_assert(sizeof(BatchDesc) == 320, "descriptor layout");

int launch_ctr_batch(const void *dev_table, int grid, int wg, int bpl, hipStream_t st);

// Small batches (at most kSmallBatch requests) travel in the kernel argument
// block instead of a device table: the same fields as BatchDesc, without its
// 64-byte alignment (kernel arguments are 16-byte aligned).
constexpr uint32_t kSmallBatch = 8;

struct SmallRec {
    uint64_t in, out, len;
    uint32_t ctr0, x0, nr, aligned;
    uint32_t k1[4];
    uint32_t tile0;
    uint32_t rk[60];
};

struct SmallBatchArgs {
    uint32_t n, total_tiles, tile_blocks, pad;
    SmallRec r[kSmallBatch];
};
static_assert(sizeof(SmallBatchArgs) <= 4096, "kernel arguments are limited to 4 KiB");

int launch_ctr_batch_small(const SmallBatchArgs &args, int grid, int wg, int bpl, hipStream_t st);

// Host side of the batch path (batch.cpp).  make_batch_record expands one
// validated request into its device record; launch_records stages up to any
// number of records (kMaxBatch per launch) on the (device, stream) context and
// launches them, through the per-slot captured graph or a plain copy+launch,
// or, with allow_small and at most kSmallBatch records, in the kernel's
// argument block.
int check_desc(const aes_ctr_desc_t &d);
// Tile size for a batch of batch_bytes payload bytes (2-64 KiB, multiple of 2 KiB).
uint64_t batch_tile_bytes(uint64_t batch_bytes, int num_cus);
void make_batch_record(const aes_ctr_desc_t &d, BatchDesc *o);
int launch_records(int device, hipStream_t st, const BatchDesc *recs, size_t n, int tile_bytes, int grid,
                   int bpl, bool use_graph, bool allow_small);
// Completes a staged table (header + n records at buf): assigns each
// record's first tile and fills the header.  Returns the table's bytes, or 0
// if the tile count would overflow 31 bits.
size_t finish_stage(uint8_t *buf, size_t n, uint32_t tile_blocks);

// Returns the staging context of stream st on device to the device's free
// list (the stream is about to be destroyed; its work must have finished or
// be finishing).  A later stream reuses it instead of allocating another.
void release_batch_stream(int device, hipStream_t st);

// Defaults before tuning, per variant and size.
Shape default_shape(int variant, int key_bits, uint64_t len, const DeviceInfo &di);

}  // namespace aesctr
