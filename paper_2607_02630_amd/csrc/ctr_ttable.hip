// ctr_ttable.hip -- AES-CTR keystream + XOR with round T-tables in LDS (gfx950).
//
// One lane encrypts one 16-byte counter block per loop step (BPL of them
// interleaved for latency hiding); a workgroup covers a contiguous chunk of
// wg * BPL blocks, so every global load/store instruction moves 64
// consecutive 16-byte blocks (1 KiB per wave, dwordx4 per lane).  The round
// function and the LDS table layout are in ttable_device.h.
#include "ttable_device.h"

namespace aesctr {
namespace {

template <bool ALIGNED>
__device__ __forceinline__ u32x4 load_block(const u32x4 *src, uint64_t idx)
{
    if constexpr (ALIGNED) {
        return __builtin_nontemporal_load(src + idx);
    } else {
        u32x4 d;
        __builtin_memcpy(&d, reinterpret_cast<const uint8_t *>(src) + 16 * idx, 16);
        return d;
    }
}

template <bool ALIGNED>
__device__ __forceinline__ void store_block(const CtrArgs &a, uint64_t idx, u32x4 v)
{
    if constexpr (ALIGNED) {
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(a.out) + idx);
    } else {
        __builtin_memcpy(a.out + 16 * idx, &v, 16);
    }
}

// Block of lane `lane`, slot b, in the chunk at `start`: wave `wave` owns
// the 64 x BPL consecutive blocks from start + 64 BPL wave, so each load or
// store instruction still covers 1 KiB of contiguous payload.
template <int BPL>
__device__ __forceinline__ uint64_t block_of(uint64_t start, uint32_t wave, uint32_t lane, int b)
{
    return start + 64u * (wave * BPL + b) + lane;
}

template <bool ALIGNED, int BPL>
__device__ __forceinline__ void prefetch(const u32x4 *src, uint64_t start, uint32_t wave, uint32_t lane,
                                         uint64_t nfull, uint64_t last, u32x4 (&d)[BPL])
{
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
        const uint64_t idx = block_of<BPL>(start, wave, lane, b);
        d[b] = load_block<ALIGNED>(src, idx < nfull ? idx : last);
    }
}

// FULL: rounds 1-2 of every block in full (no group constants); otherwise
// round 2 from the wave's group constants w.
template <int NR, int LAYOUT, int BPL, bool ALIGNED, bool FULL = false>
__device__ __forceinline__ void chunk_step(const TTable<LAYOUT> &tt, const CtrArgs &a, const uint32_t *krot,
                                           uint64_t start, uint64_t chunk, uint32_t wave, uint32_t lane,
                                           uint64_t nfull, const WaveGroups &w, const u32x4 (&d)[BPL])
{
    uint32_t ctr[BPL], ks[BPL][4];
#pragma unroll
    for (int b = 0; b < BPL; ++b)
        ctr[b] = a.ctr0 + static_cast<uint32_t>(block_of<BPL>(start, wave, lane, b));
    if constexpr (FULL)
        keystream<NR, LAYOUT, BPL>(tt, a, krot, ctr, ks);
    else
        keystream_wave<NR, LAYOUT, BPL>(tt, a, krot, ctr, w, ks);
    if (start + chunk <= nfull) {
#pragma unroll
        for (int b = 0; b < BPL; ++b)
            store_block<ALIGNED>(a, block_of<BPL>(start, wave, lane, b),
                                 d[b] ^ u32x4{ks[b][0], ks[b][1], ks[b][2], ks[b][3]});
    } else {
#pragma unroll
        for (int b = 0; b < BPL; ++b) {
            const uint64_t idx = block_of<BPL>(start, wave, lane, b);
            if (idx < nfull)
                store_block<ALIGNED>(a, idx, d[b] ^ u32x4{ks[b][0], ks[b][1], ks[b][2], ks[b][3]});
        }
    }
}

// The wave's first counter in the chunk at `start` (wave-uniform).
template <int BPL>
__device__ __forceinline__ uint32_t first_ctr(const CtrArgs &a, uint64_t start, uint32_t wave)
{
    return a.ctr0 + static_cast<uint32_t>(start + 64u * wave * BPL);
}

// How the first chunk gets its rounds 1-2 (FIRST): kFirstWave0 -- wave 0
// computes the group constants of the workgroup's chunk from the LDS tables
// and the waves pick theirs up after a second barrier; kFirstPerWave -- each
// wave computes its own two groups' constants (four lanes per group);
// kFirstFull -- the first chunk runs rounds 1-2 in full (15 more lookups
// per block, no group constants and no second barrier).  Later chunks
// compute theirs on the scalar unit.
//
// The scalars come first in the argument list, apart from the key material,
// so the dispatcher preloads them into SGPRs (the build asks for kernel
// argument preloading) and the first data loads need no argument fetch.
template <int NR, int LAYOUT, int BPL, int WG, bool ALIGNED, int FIRST>
__global__ __launch_bounds__(WG) void ctr_ttable_kernel(const uint8_t *in, uint8_t *out, uint64_t len,
                                                        uint32_t ctr0, uint32_t x0, const CtrKeys keys)
{
    static_assert(FIRST == kFirstWave0 || BPL <= 2, "the other first-chunk modes are built for 1-2 blocks per lane");
    CtrArgs a;
    a.in = in;
    a.out = out;
    a.len = len;
    a.ctr0 = ctr0;
    a.x0 = x0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        a.k1[i] = keys.k1[i];
#pragma unroll
    for (int i = 0; i < 4 * (NR + 1); ++i)
        a.rk[i] = keys.rk[i];
    __shared__ uint32_t lds[layout_lds_words(LAYOUT)];

    const uint64_t nfull = a.len >> 4;
    const uint64_t wg = WG;
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * wg * BPL;
    uint64_t start = static_cast<uint64_t>(blockIdx.x) * wg * BPL;

    // Table reads first, then the first chunk's data, so the LDS writes wait
    // only for the (cached) table reads while the data is still in flight.
    // Out-of-range lanes load a clamped (valid) block and never store it, so
    // no branch separates these loads from the table reads (a branch would
    // make the compiler wait for every load before the LDS writes).  With no
    // whole block at all, the loads read a dummy block instead.
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t chunk = wg * BPL;
    uint32_t tv[kFillStores / WG];
    fill_read<LAYOUT, WG>(tv);
    const uint64_t last = nfull ? nfull - 1 : 0;
    const u32x4 *src = nfull ? reinterpret_cast<const u32x4 *>(a.in) : &g_dummy_block;
    u32x4 d[BPL];
    prefetch<ALIGNED, BPL>(src, start, wave, lane, nfull, last, d);
    fill_write<LAYOUT, WG>(lds, tv);
    __syncthreads();

    const uint32_t k = LAYOUT == kLayout2x64 ? lane : (lane & 31);
    TTable<LAYOUT> tt{reinterpret_cast<const char *>(lds), 4 * k, 4 * k | 0x10000u};

    // Group constants of the first chunk, from the LDS tables (see FIRST).
    WaveGroups w{};
    if constexpr (FIRST == kFirstPerWave) {
        w = wave_groups_lds<LAYOUT, BPL>(tt, a, first_ctr<BPL>(a, start, wave), lane);
    } else if constexpr (FIRST == kFirstWave0) {
        static_assert(WG * BPL <= 4096, "a chunk must span at most kChunkGroups groups");
        __shared__ u32x4 s_groups[kChunkGroups];
        const uint32_t chunk_first = a.ctr0 + static_cast<uint32_t>(start);
        const uint32_t g0 = chunk_first >> 8;
        if (wave == 0) {
            const uint32_t ng = ((chunk_first & 255u) + WG * BPL + 255u) >> 8;
            if (lane < ng) {
                uint32_t G[4];
                group_consts_lds(tt, a, (g0 + lane) & 0xffffffu, G);
                s_groups[lane] = u32x4{G[0], G[1], G[2], G[3]};
            }
        }
        __syncthreads();
        {
            const uint32_t first = first_ctr<BPL>(a, start, wave);
            w.gA = first >> 8;
            const u32x4 ga = s_groups[(w.gA - g0) & 0xffffffu];
            const u32x4 gb = s_groups[(((first + 64u * BPL - 1u) >> 8) - g0) & 0xffffffu];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                w.GA[c] = ga[c];
                w.GB[c] = gb[c];
            }
        }
    }

    // rotr(rk, 8) for the two-table fold; uniform, lives in scalar registers.
    uint32_t krot[60];
    if constexpr (LAYOUT != kLayout4x32) {
#pragma unroll
        for (int i = 0; i < 4 * (NR + 1); ++i) krot[i] = (a.rk[i] >> 8) | (a.rk[i] << 24);
    }

    // The first chunk is peeled off so no loop-header wait delays it; then
    // two chunks per trip with the data buffers swapping roles, so no
    // register copy forces an early wait on the loads in flight.
    u32x4 e[BPL];
    if (start < nfull) {
        prefetch<ALIGNED, BPL>(src, start + step, wave, lane, nfull, last, e);
        chunk_step<NR, LAYOUT, BPL, ALIGNED, FIRST == kFirstFull>(tt, a, krot, start, chunk, wave, lane, nfull, w, d);
        start += step;
        while (start < nfull) {
            prefetch<ALIGNED, BPL>(src, start + step, wave, lane, nfull, last, d);
            w = wave_groups<BPL>(a, first_ctr<BPL>(a, start, wave));
            chunk_step<NR, LAYOUT, BPL, ALIGNED>(tt, a, krot, start, chunk, wave, lane, nfull, w, e);
            start += step;
            if (!(start < nfull))
                break;
            prefetch<ALIGNED, BPL>(src, start + step, wave, lane, nfull, last, e);
            w = wave_groups<BPL>(a, first_ctr<BPL>(a, start, wave));
            chunk_step<NR, LAYOUT, BPL, ALIGNED>(tt, a, krot, start, chunk, wave, lane, nfull, w, d);
            start += step;
        }
    }

    // Final partial block: leading bytes of its keystream block.
    const uint32_t tail = static_cast<uint32_t>(a.len & 15);
    if (tail != 0 && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        uint32_t ctr1[1] = {a.ctr0 + static_cast<uint32_t>(nfull)};
        uint32_t ks[1][4];
        keystream<NR, LAYOUT, 1>(tt, a, krot, ctr1, ks);
        const uint64_t off = 16 * nfull;
        for (uint32_t i = 0; i < tail; ++i)
            a.out[off + i] = a.in[off + i] ^ static_cast<uint8_t>(ks[0][i >> 2] >> (8 * (i & 3)));
    }
}

template <int NR, int LAYOUT, int BPL, int WG, int FIRST>
int launch_g(const CtrArgs &a, const Shape &sh, hipStream_t st)
{
    const bool aligned = ((reinterpret_cast<uintptr_t>(a.in) | reinterpret_cast<uintptr_t>(a.out)) & 15) == 0;
    const CtrKeys keys = ctr_keys(a);
    (void)hipGetLastError();   // not ours: left by earlier calls
    if (aligned)
        hipLaunchKernelGGL((ctr_ttable_kernel<NR, LAYOUT, BPL, WG, true, FIRST>), dim3(sh.grid), dim3(WG), 0, st,
                           a.in, a.out, a.len, a.ctr0, a.x0, keys);
    else
        hipLaunchKernelGGL((ctr_ttable_kernel<NR, LAYOUT, BPL, WG, false, FIRST>), dim3(sh.grid), dim3(WG), 0, st,
                           a.in, a.out, a.len, a.ctr0, a.x0, keys);
    return launch_status();
}

// The per-wave and full first-chunk modes are built only for the shapes that
// can use them (first_chunk_mode_ok): two tables x 32 copies for per-wave
// constants, 1-2 blocks per lane, up to 512 threads.
template <int NR, int LAYOUT, int BPL, int WG>
int launch_w(const CtrArgs &a, const Shape &sh, hipStream_t st)
{
    if constexpr (BPL <= 2 && WG <= 512) {
        if constexpr (LAYOUT == kLayout2x32) {
            if (sh.wave_groups == kFirstPerWave)
                return launch_g<NR, LAYOUT, BPL, WG, kFirstPerWave>(a, sh, st);
        }
        if (sh.wave_groups == kFirstFull)
            return launch_g<NR, LAYOUT, BPL, WG, kFirstFull>(a, sh, st);
    }
    if (sh.wave_groups != kFirstWave0)
        return AES_EINVAL;
    return launch_g<NR, LAYOUT, BPL, WG, kFirstWave0>(a, sh, st);
}

template <int NR, int LAYOUT, int BPL>
int launch_t(const CtrArgs &a, const Shape &sh, hipStream_t st)
{
    switch (sh.wg) {
    case 256: return launch_w<NR, LAYOUT, BPL, 256>(a, sh, st);
    case 512: return launch_w<NR, LAYOUT, BPL, 512>(a, sh, st);
    case 1024: return launch_w<NR, LAYOUT, BPL, 1024>(a, sh, st);
    default: return AES_EINVAL;
    }
}

template <int NR, int LAYOUT>
int launch_b(const CtrArgs &a, const Shape &sh, hipStream_t st)
{
    switch (sh.bpl) {
    case 1: return launch_t<NR, LAYOUT, 1>(a, sh, st);
    case 2: return launch_t<NR, LAYOUT, 2>(a, sh, st);
    case 4: return launch_t<NR, LAYOUT, 4>(a, sh, st);
    default: return AES_EINVAL;
    }
}

}  // namespace

int launch_ctr_ttable(const CtrArgs &a, int nr, const Shape &sh, hipStream_t st)
{
    // The LDS fill splits 8192 stores evenly over the workgroup.
    if ((sh.wg != 256 && sh.wg != 512 && sh.wg != 1024) || sh.grid <= 0)
        return AES_EINVAL;
    // (copies, tables): (32, 4), (64, 2) or (32, 2).
    int layout;
    if (sh.copies == 32 && sh.tables == 4)
        layout = kLayout4x32;
    else if (sh.copies == 64 && sh.tables == 2)
        layout = kLayout2x64;
    else if (sh.copies == 32 && sh.tables == 2)
        layout = kLayout2x32;
    else
        return AES_EINVAL;
    if (nr == 10)
        return layout == kLayout4x32 ? launch_b<10, kLayout4x32>(a, sh, st)
             : layout == kLayout2x64 ? launch_b<10, kLayout2x64>(a, sh, st)
                                     : launch_b<10, kLayout2x32>(a, sh, st);
    if (nr == 14)
        return layout == kLayout4x32 ? launch_b<14, kLayout4x32>(a, sh, st)
             : layout == kLayout2x64 ? launch_b<14, kLayout2x64>(a, sh, st)
                                     : launch_b<14, kLayout2x32>(a, sh, st);
    return AES_EINVAL;
}

}  // namespace aesctr
