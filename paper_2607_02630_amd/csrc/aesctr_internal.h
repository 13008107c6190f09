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
    int variant;        // AES_VARIANT_TTABLE, _BITSLICE or _VPERM
    int bpl;            // 16-byte blocks per lane per loop step
    int wg;             // threads per workgroup
    int grid;           // workgroups
    int copies;         // T-table replication (32 or 64 copies per table)
    int tables;         // T-tables in LDS: 4 (T0..T3) or 2 (T0, T2)
    int wave_groups;    // first chunk's rounds 1-2 (T-table kernel): kFirstWave0,
                        // kFirstPerWave or kFirstFull
};

// First-chunk modes of the T-table kernel (Shape::wave_groups, and the
// wave_groups field of aes_launch_cfg_t on output).
enum : int { kFirstWave0 = 0, kFirstPerWave = 1, kFirstFull = 2 };
// Whether a shape is built with first-chunk mode m.
inline bool first_chunk_mode_ok(int m, int copies, int tables, int bpl, int wg)
{
    if (m == kFirstWave0)
        return true;
    if (bpl > 2 || wg > 512)
        return false;
    return m == kFirstFull || (m == kFirstPerWave && copies == 32 && tables == 2);
}

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

// The key material of CtrArgs as a kernel argument of its own, after the
// scalars (which the dispatcher can then preload into SGPRs).
struct CtrKeys {
    uint32_t k1[4];
    uint32_t rk[60];
};

inline CtrKeys ctr_keys(const CtrArgs &a)
{
    CtrKeys k;
    for (int i = 0; i < 4; ++i)
        k.k1[i] = a.k1[i];
    for (int i = 0; i < 60; ++i)
        k.rk[i] = a.rk[i];
    return k;
}

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

// Arguments of the vector-permute kernel (ctr_vperm.hip): the round keys in
// the (i, k) nibble form of its tower field, row words (byte c = column c).
//   x0      rk0's counter column in standard bytes (byte r = row r)
//   rki/rkk index 0: round 1's output rows without their counter terms
//           (the nonce columns' MixColumns terms, rk1 and the {63} fold);
//           index t - 1, t = 2..Nr-1: (round key t ^ {63}), in i and k nibbles
//   rkn     round Nr: (round key ^ {63}) in standard bytes
struct VpArgs {
    const uint8_t *in;
    uint8_t *out;
    uint64_t len;
    uint32_t ctr0;
    uint32_t x0;
    uint32_t rki[13][4], rkk[13][4];
    uint32_t rkn[4];
};
void make_vperm_args(const aes_sched_t &s, const uint8_t nonce[12], uint32_t ctr0, const void *in, void *out,
                     uint64_t len, VpArgs *a);
int launch_ctr_vperm(const VpArgs &a, int nr, const Shape &sh, hipStream_t st);

// ---- Batched launch -------------------------------------------------------
// Device table of one launch:
//   BatchHeader
//   n BatchDesc records (64 B each)
//   n_keys KeyRec records (256 B each) at keys_off: the round keys of the
//     requests whose key travels with the launch ("inline")
//   n_install InstallRec records at install_off: inline keys the launch also
//     writes into slots of a resident key table (a serving engine's, at
//     header.resident), for later launches to read.
// Requests are cut into tiles of tile_blocks 16-byte blocks; tile0 is a
// request's first tile (exclusive prefix sum), so tile t belongs to the last
// request whose tile0 <= t.  next is the work counter the waves claim tiles
// from; every upload carries it as 0.
constexpr int kMaxBatch = 4096;          // requests per launch (tile0 index in LDS)
constexpr int kMaxBatchGrid = 1 << 20;   // workgroups per batch launch (keeps tile indices in 32 bits)
// BatchDesc::key: kKeyResident | slot reads slot `slot` of the resident key
// table; otherwise the value indexes the launch's own KeyRec records.
constexpr uint32_t kKeyResident = 0x80000000u;
constexpr uint32_t kNoInstall = 0xffffffffu;

struct alignas(64) BatchHeader {
    uint32_t n;
    uint32_t total_tiles;
    uint32_t tile_blocks;
    uint32_t next;
    uint32_t n_keys;
    uint32_t n_install;
    uint32_t keys_off;       // byte offsets from the start of the table
    uint32_t install_off;
    uint64_t resident;       // device address of the resident key table, or 0
    uint32_t pad[6];
};

struct alignas(64) BatchDesc {
    uint64_t in, out, len;
    uint32_t ctr0, x0;
    uint32_t k1[4];
    uint32_t tile0;
    uint32_t key;            // kKeyResident | slot, or an inline KeyRec index
    uint16_t nr, aligned;    // aligned: in and out 16-byte aligned
    uint32_t pad;
};

// Round keys of one expanded key as column words (KeyMaterial::rk).
struct KeyRec {
    uint32_t rk[64];
};

struct InstallRec {
    uint32_t key;            // inline KeyRec index
    uint32_t slot;           // resident slot it is written to
};
static_assert(sizeof(BatchHeader) == 64, "header layout");
static_assert(sizeof(BatchDesc) == 64, "descriptor layout");
static_assert(sizeof(KeyRec) == 256, "key record layout");

// Bytes of a launch table with n requests, n_keys inline keys and n_install
// installs, and the offsets of its sections.
constexpr size_t batch_keys_off(size_t n) { return sizeof(BatchHeader) + n * sizeof(BatchDesc); }
constexpr size_t batch_install_off(size_t n, size_t n_keys) { return batch_keys_off(n) + n_keys * sizeof(KeyRec); }
constexpr size_t batch_table_bytes(size_t n, size_t n_keys, size_t n_install)
{
    return batch_install_off(n, n_keys) + n_install * sizeof(InstallRec);
}
constexpr size_t kMaxTableBytes = batch_table_bytes(kMaxBatch, kMaxBatch, kMaxBatch);

int launch_ctr_batch(const void *dev_table, int grid, int wg, int bpl, hipStream_t st);

// Small batches (at most kSmallBatch requests) travel in the kernel argument
// block instead of a device table; each record carries its own round keys
// (used unless it names a resident slot) and the slot it installs them into,
// if any.
constexpr uint32_t kSmallBatch = 8;

struct SmallRec {
    uint64_t in, out, len;
    uint32_t ctr0, x0;
    uint32_t k1[4];
    uint32_t tile0;
    uint32_t key;            // kKeyResident | slot, or anything else = rk below
    uint32_t install;        // slot to write rk into, or kNoInstall
    uint16_t nr, aligned;
    uint32_t rk[60];
};

struct SmallBatchArgs {
    uint32_t n, total_tiles, tile_blocks, pad;
    uint64_t resident;       // resident key table, or 0
    uint64_t pad2;
    SmallRec r[kSmallBatch];
};
static_assert(sizeof(SmallBatchArgs) <= 4096, "kernel arguments are limited to 4 KiB");

// grid: workgroups of the argument-path kernel's own size (256 threads).
int launch_ctr_batch_small(const SmallBatchArgs &args, int grid, int bpl, hipStream_t st);

// One request as the host keeps it before staging: its descriptor (key field
// not yet assigned) and its round keys.
struct RequestRec {
    BatchDesc d;
    KeyRec key;
};

// A launch as the host hands it to the batch path: requests whose key field is
// already assigned, the inline key records they index, the installs, and the
// resident table the launch reads (or 0).
struct LaunchSpec {
    const BatchDesc *descs = nullptr;
    size_t n = 0;
    const KeyRec *keys = nullptr;
    size_t n_keys = 0;
    const InstallRec *installs = nullptr;
    size_t n_install = 0;
    uint64_t resident = 0;
};

// Host side of the batch path (batch.cpp).  make_batch_record expands one
// validated request into its record.  launch_spec stages one launch (at most
// kMaxBatch requests) on the (device, stream) context and launches it through
// the slot's captured graph or a plain copy + launch, or, with allow_small and
// at most kSmallBatch requests, in the kernel's argument block.
int check_desc(const aes_ctr_desc_t &d);
// Tile size for a batch of batch_bytes payload bytes (about 16 tiles per CU,
// 2-64 KiB, multiple of 2 KiB, or the tune cache's constants) and the blocks
// per lane of batch launches (2, or the tune cache's).
uint64_t batch_tile_bytes(uint64_t batch_bytes, int num_cus);
int batch_blocks_per_lane();
void make_batch_record(const aes_ctr_desc_t &d, RequestRec *o);
void make_batch_desc(const aes_ctr_desc_t &d, BatchDesc *o, KeyRec *k);
int launch_spec(int device, hipStream_t st, const LaunchSpec &spec, int tile_bytes, int grid, int bpl,
                bool use_graph, bool allow_small);
// Completes a staged table of n requests at buf (descriptors, keys and
// installs written, n_keys / n_install / resident set in the header):
// assigns each request's first tile and fills the rest of the header.
// Returns the table's bytes, or 0 if the tile count would overflow 31 bits.
size_t finish_stage(uint8_t *buf, size_t n, uint32_t tile_blocks);

// Returns the staging context of stream st on device to the device's free
// list (the stream is about to be destroyed; its work must have finished or
// be finishing).  A later stream reuses it instead of allocating another.
void release_batch_stream(int device, hipStream_t st);

// Defaults before tuning, per variant and size.
Shape default_shape(int variant, int key_bits, uint64_t len, const DeviceInfo &di);

}  // namespace aesctr
