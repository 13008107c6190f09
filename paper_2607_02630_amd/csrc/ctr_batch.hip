// ctr_batch.hip -- one persistent launch over a table of requests (gfx950).
//
// Each workgroup fills the bank-replicated T-tables into LDS once (the same
// round code as the single-buffer kernel, ttable_device.h), copies the
// requests' first-tile indices into LDS, then its waves claim tiles from a
// device counter until the table is exhausted.  A tile is tile_blocks
// consecutive 16-byte blocks of one request; the wave finds the request by a
// binary search over the tile indices in LDS and reads that request's key
// material, pointers and counter parameters with scalar loads (they are the
// same for the whole wave).  Requests of any size, key length (AES-128 and
// AES-256 mixed) and alignment share the launch; dynamic claiming balances
// the log-uniform size mix.
#include <stddef.h>

#include "ttable_device.h"

namespace aesctr {
namespace {

constexpr int kBatchWG = 1024;
constexpr int kBatchLayout = kLayout4x32;
// The argument-path kernel (at most kSmallBatch requests, mostly a tile or
// two per wave) keeps the single-buffer kernel's small-message shape: 256
// threads, two tables x 32 copies (half the fill), rounds 1-2 in full (no
// group-constant chain of scalar loads ahead of the rounds).
constexpr int kSmallWG = 256;
constexpr int kSmallLayout = kLayout2x32;

// Request pointers arrive as integers; these types keep their accesses in the
// global address space (global_load/store rather than flat).
typedef __attribute__((address_space(1))) const u32x4 g_cu32x4;
typedef __attribute__((address_space(1))) u32x4 g_u32x4;
typedef __attribute__((address_space(1))) const uint8_t g_cu8;
typedef __attribute__((address_space(1))) uint8_t g_u8;
// Round keys are read through the constant address space, so they load with
// scalar instructions even though workgroup 0 of the same launch writes
// other slots of the resident table (installs): no launch reads a slot that
// it, or any launch in flight, writes.
typedef __attribute__((address_space(4))) const uint32_t c_u32;

// Blocks [b0, b1) of one request.  The loop trip count is the same for every
// lane (the round-1/2 sharing needs the whole wave), and lane i of each step
// holds block s0 + 64*b + i.  FULL: rounds 1-2 of every block in full
// instead of from the wave's group constants.
template <int NR, int LAYOUT, int BPL, bool ALIGNED, bool FULL>
__device__ __forceinline__ void run_tile(const TTable<LAYOUT> &tt, const CtrArgs &a, uint64_t b0,
                                         uint64_t b1, uint32_t lane)
{
    const uint64_t nfull = a.len >> 4;
    // rotr(rk, 8) of rounds 2..Nr-1 for the two-table fold (the four-table
    // layout reads none).
    uint32_t krot[60];
    if constexpr (LAYOUT != kLayout4x32) {
#pragma unroll
        for (int i = 8; i < 4 * NR; ++i) krot[i] = rotr8(a.rk[i]);
    }
    for (uint64_t s0 = b0; s0 < b1; s0 += 64 * BPL) {
        uint32_t ctr[BPL], ks[BPL][4];
        u32x4 d[BPL];
#pragma unroll
        for (int b = 0; b < BPL; ++b) {
            const uint64_t idx = s0 + 64 * b + lane;
            ctr[b] = a.ctr0 + static_cast<uint32_t>(idx);
            if (idx < b1 && idx < nfull) {
                if constexpr (ALIGNED) {
                    d[b] = __builtin_nontemporal_load((g_cu32x4 *)(uintptr_t)a.in + idx);
                } else {
                    g_cu8 *p = (g_cu8 *)(uintptr_t)a.in + 16 * idx;
                    uint8_t tmp[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) tmp[i] = p[i];
                    __builtin_memcpy(&d[b], tmp, 16);
                }
            }
        }
        if constexpr (FULL) {
            keystream<NR, LAYOUT, BPL>(tt, a, krot, ctr, ks);
        } else {
            const WaveGroups w = wave_groups<BPL>(a, a.ctr0 + static_cast<uint32_t>(s0));
            keystream_wave<NR, LAYOUT, BPL>(tt, a, krot, ctr, w, ks);
        }
#pragma unroll
        for (int b = 0; b < BPL; ++b) {
            const uint64_t idx = s0 + 64 * b + lane;
            if (idx >= b1)
                continue;
            const u32x4 k = u32x4{ks[b][0], ks[b][1], ks[b][2], ks[b][3]};
            if (idx < nfull) {
                if constexpr (ALIGNED) {
                    __builtin_nontemporal_store(d[b] ^ k, (g_u32x4 *)(uintptr_t)a.out + idx);
                } else {
                    const u32x4 v = d[b] ^ k;
                    uint8_t tmp[16];
                    __builtin_memcpy(tmp, &v, 16);
                    g_u8 *p = (g_u8 *)(uintptr_t)a.out + 16 * idx;
#pragma unroll
                    for (int i = 0; i < 16; ++i) p[i] = tmp[i];
                }
            } else if (idx == nfull) {
                // Final partial block: leading bytes of its keystream block.
                const uint32_t tail = static_cast<uint32_t>(a.len & 15);
                g_cu8 *src = (g_cu8 *)(uintptr_t)a.in + 16 * idx;
                g_u8 *dst = (g_u8 *)(uintptr_t)a.out + 16 * idx;
                for (uint32_t i = 0; i < tail; ++i)
                    dst[i] = src[i] ^ static_cast<uint8_t>(k[i >> 2] >> (8 * (i & 3)));
            }
        }
    }
}

// Tile t of request R (a BatchDesc in the device table or a SmallRec in the
// kernel arguments; both wave-uniform, so their fields arrive by scalar
// loads) with round keys rk (wave-uniform, read from the launch's inline keys
// or from a slot of the resident key table): the request's key material and
// pointers, then the tile's blocks.
template <int LAYOUT, int BPL, bool FULL, class Rec>
__device__ __forceinline__ void request_tile(const TTable<LAYOUT> &tt, const Rec &R, const uint32_t (&rk)[60],
                                             uint32_t t, uint32_t tile_blocks, uint32_t lane)
{
    CtrArgs a;
    a.in = reinterpret_cast<const uint8_t *>(R.in);
    a.out = reinterpret_cast<uint8_t *>(R.out);
    a.len = R.len;
    a.ctr0 = R.ctr0;
    a.x0 = R.x0;
#pragma unroll
    for (int c = 0; c < 4; ++c)
        a.k1[c] = R.k1[c];
    const uint32_t nr = R.nr;
    const uint32_t nrk = 4 * (nr + 1);
#pragma unroll
    for (int i = 0; i < 60; ++i)
        a.rk[i] = i < 44 || nrk > 44 ? rk[i] : 0;
    const uint64_t nblocks = (a.len + 15) >> 4;
    const uint64_t b0 = static_cast<uint64_t>(t - R.tile0) * tile_blocks;
    const uint64_t b1 = b0 + tile_blocks < nblocks ? b0 + tile_blocks : nblocks;
    if (R.aligned) {
        if (nr == 10)
            run_tile<10, LAYOUT, BPL, true, FULL>(tt, a, b0, b1, lane);
        else
            run_tile<14, LAYOUT, BPL, true, FULL>(tt, a, b0, b1, lane);
    } else {
        if (nr == 10)
            run_tile<10, LAYOUT, BPL, false, FULL>(tt, a, b0, b1, lane);
        else
            run_tile<14, LAYOUT, BPL, false, FULL>(tt, a, b0, b1, lane);
    }
}

// Writes the round keys of key record `src` (64 words) into slot `slot` of
// the resident table, one word per thread of the workgroup, with vector
// stores.  No wave of this launch reads that slot (its requests read the
// inline copy), and no launch in flight reads it either: the host hands a
// slot out for installing only when nothing references it.
__device__ __forceinline__ void install_key(uint32_t *resident, uint32_t slot, const uint32_t *src, uint32_t word)
{
    resident[64u * slot + word] = src[word];
}

// table: the uploaded header, descriptors, inline keys and installs,
// read-only here (so request fields come in through the scalar cache);
// counter: the header's `next` word.  Besides the outputs the kernel writes
// only that counter and, in workgroup 0, the installs' resident slots.
template <int BPL>
__global__ __launch_bounds__(kBatchWG) void ctr_batch_kernel(const uint8_t *__restrict__ table,
                                                             uint32_t *__restrict__ counter)
{
    __shared__ uint32_t lds[kLdsWords];
    __shared__ uint32_t s_tile0[kMaxBatch];

    const BatchHeader *hdr = reinterpret_cast<const BatchHeader *>(table);
    const BatchDesc *desc = reinterpret_cast<const BatchDesc *>(table + sizeof(BatchHeader));
    const uint32_t n = hdr->n;
    const uint32_t total = hdr->total_tiles;
    const uint32_t tile_blocks = hdr->tile_blocks;
    const uint32_t *keys = reinterpret_cast<const uint32_t *>(table + hdr->keys_off);
    uint32_t *resident = reinterpret_cast<uint32_t *>(hdr->resident);

    uint32_t tv[kFillStores / kBatchWG];
    fill_read<kBatchLayout, kBatchWG>(tv);
    for (uint32_t i = threadIdx.x; i < n; i += kBatchWG)
        s_tile0[i] = desc[i].tile0;
    if (blockIdx.x == 0) {
        const InstallRec *inst = reinterpret_cast<const InstallRec *>(table + hdr->install_off);
        const uint32_t words = 64u * hdr->n_install;
        for (uint32_t i = threadIdx.x; i < words; i += kBatchWG) {
            const InstallRec r = inst[i >> 6];
            install_key(resident, r.slot, keys + 64u * r.key, i & 63u);
        }
    }
    fill_write<kBatchLayout, kBatchWG>(lds, tv);
    __syncthreads();

    const uint32_t lane = threadIdx.x & 63;
    TTable<kBatchLayout> tt{reinterpret_cast<const char *>(lds), 4 * (lane & 31), 4 * (lane & 31) | 0x10000u};

    // Tile claiming.  The launch's W waves first take tiles 0..W-1 statically,
    // spread so that consecutive tiles land on different CUs (wave j of
    // workgroup b takes tile j * grid + b): a batch of at most W tiles needs
    // no atomic at all.  Later tiles are claimed from the header counter
    // (tile = W + counter); a wave issues its next claim when it starts a
    // tile, so the atomic's round trip hides behind the tile's work.
    const uint32_t waves = gridDim.x * (kBatchWG / 64);
    uint32_t t = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * gridDim.x + blockIdx.x;
    while (t < total) {
        uint32_t claim = 0;
        if (lane == 0)
            claim = atomicAdd(counter, 1u);
        // Last request whose first tile is <= t (empty requests share their
        // successor's tile0 and are skipped by taking the last match).
        uint32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (s_tile0[mid] <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint32_t r = __builtin_amdgcn_readfirstlane(lo);
        const BatchDesc &R = desc[r];
        const uint32_t key = R.key;
        uint32_t rk[60];
        if (key & kKeyResident) {
            c_u32 *p = (c_u32 *)(uintptr_t)(resident + 64u * (key & ~kKeyResident));
#pragma unroll
            for (int i = 0; i < 60; ++i) rk[i] = p[i];
        } else {
            const uint32_t *p = keys + 64u * key;
#pragma unroll
            for (int i = 0; i < 60; ++i) rk[i] = p[i];
        }
        request_tile<kBatchLayout, BPL, false>(tt, R, rk, t, tile_blocks, lane);
        t = waves + __builtin_amdgcn_readfirstlane(claim);
    }
}

// A batch of at most kSmallBatch requests whose records travel in the kernel
// argument block: no descriptor upload goes ahead of the launch (a separate
// host-to-device copy adds about 20 us to a small batch's latency).  Tiles
// are assigned statically, wave w taking tiles w, w + W, w + 2W, ... (W
// waves, numbered as in ctr_batch_kernel), so no work counter is needed.
template <int BPL>
__global__ __launch_bounds__(kSmallWG) void ctr_batch_small_kernel(const SmallBatchArgs args)
{
    __shared__ uint32_t lds[layout_lds_words(kSmallLayout)];

    uint32_t tv[kFillStores / kSmallWG];
    fill_read<kSmallLayout, kSmallWG>(tv);
    uint32_t *resident = reinterpret_cast<uint32_t *>(args.resident);
    const uint32_t n = args.n;
    if (blockIdx.x == 0) {
        for (uint32_t j = threadIdx.x; j < 64u * n; j += kSmallWG) {
            const uint32_t i = j >> 6, w = j & 63u;
            if (args.r[i].install != kNoInstall && w < 60u)
                install_key(resident, args.r[i].install, args.r[i].rk, w);
        }
    }
    fill_write<kSmallLayout, kSmallWG>(lds, tv);
    __syncthreads();

    const uint32_t lane = threadIdx.x & 63;
    TTable<kSmallLayout> tt{reinterpret_cast<const char *>(lds), 4 * (lane & 31), 4 * (lane & 31) | 0x10000u};
    const uint32_t waves = gridDim.x * (kSmallWG / 64);
    for (uint32_t t = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * gridDim.x + blockIdx.x;
         t < args.total_tiles; t += waves) {
        // Last request whose first tile is <= t (skips empty requests).
        uint32_t r = 0;
        for (uint32_t i = 1; i < n; ++i)
            if (args.r[i].tile0 <= t)
                r = i;
        const SmallRec &R = args.r[r];
        uint32_t rk[60];
        if (R.key & kKeyResident) {
            c_u32 *p = (c_u32 *)(uintptr_t)(resident + 64u * (R.key & ~kKeyResident));
#pragma unroll
            for (int i = 0; i < 60; ++i) rk[i] = p[i];
        } else {
#pragma unroll
            for (int i = 0; i < 60; ++i) rk[i] = R.rk[i];
        }
        request_tile<kSmallLayout, BPL, true>(tt, R, rk, t, args.tile_blocks, lane);
    }
}

}  // namespace

int launch_ctr_batch(const void *dev_table, int grid, int wg, int bpl, hipStream_t st)
{
    if (wg != kBatchWG || grid <= 0 || grid > kMaxBatchGrid)
        return AES_EINVAL;
    const uint8_t *t = static_cast<const uint8_t *>(dev_table);
    uint32_t *ctr = reinterpret_cast<uint32_t *>(const_cast<uint8_t *>(t) + offsetof(BatchHeader, next));
    (void)hipGetLastError();   // not ours: left by earlier calls
    switch (bpl) {
    case 1: hipLaunchKernelGGL(ctr_batch_kernel<1>, dim3(grid), dim3(kBatchWG), 0, st, t, ctr); break;
    case 2: hipLaunchKernelGGL(ctr_batch_kernel<2>, dim3(grid), dim3(kBatchWG), 0, st, t, ctr); break;
    default: return AES_EINVAL;
    }
    return launch_status();
}

int launch_ctr_batch_small(const SmallBatchArgs &args, int grid, int bpl, hipStream_t st)
{
    if (grid <= 0 || grid > kMaxBatchGrid || args.n > kSmallBatch)
        return AES_EINVAL;
    (void)hipGetLastError();   // not ours: left by earlier calls
    switch (bpl) {
    case 1: hipLaunchKernelGGL(ctr_batch_small_kernel<1>, dim3(grid), dim3(kSmallWG), 0, st, args); break;
    case 2: hipLaunchKernelGGL(ctr_batch_small_kernel<2>, dim3(grid), dim3(kSmallWG), 0, st, args); break;
    default: return AES_EINVAL;
    }
    return launch_status();
}

}  // namespace aesctr
