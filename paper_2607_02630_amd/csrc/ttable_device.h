// ttable_device.h -- device code of the T-table AES round shared by the
// single-buffer and batched kernels (each translation unit gets its own copy
// of the constant table).
//
// Rounds (FIPS-197 Sec. 5.1) use the T-table form: output column c of a full
// round is T0[s_c.b0] ^ T1[s_(c+1).b1] ^ T2[s_(c+2).b2] ^ T3[s_(c+3).b3] ^ rk,
// i.e. SubBytes + ShiftRows + MixColumns + AddRoundKey in four lookups and
// two 3-input XORs (v_bitop3_b32).  The last round (no MixColumns) picks the
// S-box byte out of T0/T2 entries with v_perm_b32.
//
// Random table indices would serialise on LDS banks, so every lane reads its
// own bank-resident copy.  The entry for index x sits at byte 256*x, and the
// lane's copy at +4*k (k = lane mod the copy count): the address is built by
// one v_perm_b32 that drops the state byte into bits 8..15 next to the lane's
// constant bits.  Three layouts (the kernels' LAYOUT parameter):
//   kLayout4x32: 32 copies of each of T0..T3 (128 KiB): T0|T1 interleaved in
//                [0, 64 KiB) (T1 at +128 B), T2|T3 in [64 KiB, 128 KiB).
//                Lanes l and l+32 share a bank.
//   kLayout2x64: 64 copies of T0 in [0, 64 KiB) and of T2 in [64 KiB,
//                128 KiB); T1 = rotl(T0, 8) and T3 = rotl(T2, 8) are folded
//                into one rotate per column.
//   kLayout2x32: 32 copies of T0 and of T2, interleaved in [0, 64 KiB) (T2 at
//                +128 B), with the same fold: half the table fill of the other
//                two for about 15% more VALU work per block, and two
//                workgroups fit in a CU's LDS, so one's fill and barriers
//                overlap the other's rounds.
#pragma once

#include "aes_tables.h"
#include "aesctr_internal.h"

namespace aesctr {
namespace {


__constant__ Tables c_tables = build_tables();

// All four round tables, T_t[x] = rotl(T0[x], 8t), for the scalar unit (it
// has no rotate): the wave-uniform group constants of rounds 1-2 read them
// with scalar loads.
struct RoundTables {
    uint32_t t[4][256];
};

constexpr RoundTables build_round_tables()
{
    RoundTables r{};
    const Tables b = build_tables();
    for (int t = 0; t < 4; ++t)
        for (int x = 0; x < 256; ++x)
            r.t[t][x] = rotl32(b.t0[x], 8 * t);
    return r;
}

__constant__ RoundTables c_round = build_round_tables();

constexpr int kLdsWords = 32768;   // 128 KiB

enum : int { kLayout4x32 = 0, kLayout2x64 = 1, kLayout2x32 = 2 };

// LDS words a layout occupies.
constexpr int layout_lds_words(int layout) { return layout == kLayout2x32 ? kLdsWords / 2 : kLdsWords; }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Valid global memory for loads issued when a message has no whole block.
__device__ u32x4 g_dummy_block;

__device__ __forceinline__ uint32_t vperm(uint32_t s0, uint32_t s1, uint32_t sel)
{
    return __builtin_amdgcn_perm(s0, s1, sel);
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint32_t rotl8(uint32_t x)
{
    return __builtin_amdgcn_alignbit(x, x, 24);
}

__device__ __forceinline__ uint32_t rotr8(uint32_t x)
{
    return __builtin_amdgcn_alignbit(x, x, 8);
}

// Address of the entry for byte R of v in the table region selected by lb
// (lb = 4*copy | region << 16): bytes [lb.b0, v.bR, lb.b2, 0].
template <int R>
__device__ __forceinline__ uint32_t taddr(uint32_t v, uint32_t lb)
{
    return vperm(v, lb, 0x0c020000u | ((4u + R) << 8));
}

__device__ __forceinline__ uint32_t lds_at(const char *lds, uint32_t byte_addr)
{
    return *reinterpret_cast<const uint32_t *>(lds + byte_addr);
}

// The LDS image is fill_stores(LAYOUT) 16-byte stores: 8192 (128 KiB), or
// 4096 (64 KiB) for kLayout2x32.  Each store is a 4-way broadcast of one
// table entry (a run of four copies).  The entries are read from the constant
// table first (fill_read) so the caller can issue its own global loads before
// the table reads are waited for; fill_write then stores them.
//  * kLayout4x32, kLayout2x64: thread t performs stores w = t + u*WG, one
//    value read per store.
//  * kLayout2x32: two stores per value read, so a value needs one rotate and
//    one set of register copies for both.  The 16 stores of entry i (8 per
//    table) come from threads 8i' + 4h + q (i' = i mod WG/8), which write
//    quads q + 4h and then q + 4(1 - h) of table h's half of the entry: the
//    8 threads of an entry cover all 32 banks in each store instruction.
constexpr int kFillStores = 8192;

constexpr int fill_stores(int layout) { return layout == kLayout2x32 ? kFillStores / 2 : kFillStores; }

template <int LAYOUT, int WG>
__device__ __forceinline__ void fill_read(uint32_t (&tv)[kFillStores / WG])
{
    if constexpr (LAYOUT == kLayout2x32) {
#pragma unroll
        for (int u = 0; u < 2048 / WG; ++u)
            tv[u] = c_tables.t0[(threadIdx.x >> 3) + u * (WG / 8)];
    } else {
#pragma unroll
        for (int u = 0; u < fill_stores(LAYOUT) / WG; ++u)
            tv[u] = c_tables.t0[(threadIdx.x + u * WG) >> 5];
    }
}

template <int LAYOUT, int WG>
__device__ __forceinline__ void fill_write(uint32_t *lds, const uint32_t (&tv)[kFillStores / WG])
{
    if constexpr (LAYOUT == kLayout2x32) {
        const uint32_t t = threadIdx.x, q = t & 3, h = (t >> 2) & 1;
        const uint32_t a0 = (t >> 3) * 256 + h * 128 + q * 16 + h * 64, a1 = a0 ^ 64;
        char *base = reinterpret_cast<char *>(lds);
#pragma unroll
        for (int u = 0; u < 2048 / WG; ++u) {
            const uint32_t val = h ? rotl32(tv[u], 16) : tv[u];
            const u32x4 v4{val, val, val, val};
            *reinterpret_cast<u32x4 *>(base + a0 + u * 32 * WG) = v4;
            *reinterpret_cast<u32x4 *>(base + a1 + u * 32 * WG) = v4;
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < fill_stores(LAYOUT) / WG; ++u) {
        const uint32_t w = threadIdx.x + u * WG;
        uint32_t val, addr;
        if constexpr (LAYOUT == kLayout4x32) {
            const uint32_t i = w >> 5, q = w & 7, t = (w >> 3) & 3;
            val = rotl32(tv[u], 8 * t);
            addr = (t >> 1) * 65536 + i * 256 + (t & 1) * 128 + q * 16;
        } else if constexpr (LAYOUT == kLayout2x64) {
            const uint32_t i = w >> 5, q = w & 15, t2 = (w >> 4) & 1;
            val = t2 ? rotl32(tv[u], 16) : tv[u];
            addr = t2 * 65536 + i * 256 + q * 16;
        } else {
            const uint32_t i = w >> 4, q = w & 7, t2 = (w >> 3) & 1;
            val = t2 ? rotl32(tv[u], 16) : tv[u];
            addr = i * 256 + t2 * 128 + q * 16;
        }
        *reinterpret_cast<u32x4 *>(reinterpret_cast<char *>(lds) + addr) = u32x4{val, val, val, val};
    }
}

// lb0 / lb1: the lane's copy offset 4*k for the first / second 64 KiB
// (lb1 = lb0 | 64 KiB; unused by kLayout2x32).
template <int LAYOUT>
struct TTable {
    const char *lds;
    uint32_t lb0, lb1;

    // T_t[byte R of v] for t = 0..3.
    template <int T, int R>
    __device__ __forceinline__ uint32_t get(uint32_t v) const
    {
        if constexpr (LAYOUT == kLayout4x32) {
            const uint32_t a = taddr<R>(v, (T >= 2) ? lb1 : lb0);
            return lds_at(lds, a + ((T & 1) ? 128u : 0u));
        } else {
            const uint32_t e = raw<(T >= 2) ? 1 : 0, R>(v);
            return (T & 1) ? rotl8(e) : e;
        }
    }

    // Raw entries of the T0 (REGION 0) or T2 (REGION 1) table, without the
    // odd tables' rotation.
    template <int REGION, int R>
    __device__ __forceinline__ uint32_t raw(uint32_t v) const
    {
        if constexpr (LAYOUT == kLayout2x32)
            return lds_at(lds, taddr<R>(v, lb0) + (REGION ? 128u : 0u));
        else
            return lds_at(lds, taddr<R>(v, REGION ? lb1 : lb0));
    }

    // T0[byte of v at bit `pos`] for a lane-varying byte position (every
    // layout keeps T0 entry x at 256*x + lb0).
    __device__ __forceinline__ uint32_t t0_at(uint32_t v, uint32_t pos) const
    {
        return lds_at(lds, (__builtin_amdgcn_ubfe(v, pos, 8) << 8) | lb0);
    }

    // One full round: s -> o with round key words k[0..3]; krot holds
    // rotr(k, 8) for the two-table fold.
    __device__ __forceinline__ void round(const uint32_t s[4], uint32_t o[4],
                                          const uint32_t *k, const uint32_t *krot) const
    {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t s0 = s[c], s1 = s[(c + 1) & 3], s2 = s[(c + 2) & 3], s3 = s[(c + 3) & 3];
            if constexpr (LAYOUT == kLayout4x32) {
                o[c] = xor3(xor3(get<0, 0>(s0), get<1, 1>(s1), get<2, 2>(s2)), get<3, 3>(s3), k[c]);
            } else {
                // T1[b]^T3[d]^k = rotl8(T0[b]^T2[d]^rotr8(k))
                uint32_t odd = rotl8(xor3(raw<0, 1>(s1), raw<1, 3>(s3), krot[c]));
                o[c] = xor3(raw<0, 0>(s0), raw<1, 2>(s2), odd);
            }
        }
    }

    // Last round: S-box bytes only.  Row 0 byte from a T2 entry (S at byte 0),
    // row 1 and row 2 from T0 entries (S at bytes 1, 2), row 3 from T2 (byte 3).
    __device__ __forceinline__ void last_round(const uint32_t s[4], uint32_t o[4],
                                               const uint32_t *k) const
    {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            uint32_t e0 = raw<1, 0>(s[c]);
            uint32_t e1 = raw<0, 1>(s[(c + 1) & 3]);
            uint32_t e2 = raw<0, 2>(s[(c + 2) & 3]);
            uint32_t e3 = raw<1, 3>(s[(c + 3) & 3]);
            uint32_t lo = vperm(e1, e0, 0x0c0c0500u);   // [e0.b0, e1.b1, 0, 0]
            uint32_t hi = vperm(e3, e2, 0x07020c0cu);   // [0, 0, e2.b2, e3.b3]
            o[c] = xor3(lo, hi, k[c]);
        }
    }
};

// Keystreams of N counter blocks, computed round by round across the N
// blocks so their independent lookups interleave.  ctr[i] is already
// ctr0 + j mod 2^32.
template <int NR, int LAYOUT, int N>
__device__ __forceinline__ void keystream(const TTable<LAYOUT> &tt, const CtrArgs &a,
                                          const uint32_t *krot, const uint32_t *ctr, uint32_t (*ks)[4])
{
    uint32_t s[N][4], o[N][4];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        // Rounds 0 and 1 of the counter column; the other terms are in k1.
        const uint32_t x = vperm(ctr[b], ctr[b], 0x00010203u) ^ a.x0;   // big-endian counter
        s[b][0] = a.k1[0] ^ tt.template get<3, 3>(x);
        s[b][1] = a.k1[1] ^ tt.template get<2, 2>(x);
        s[b][2] = a.k1[2] ^ tt.template get<1, 1>(x);
        s[b][3] = a.k1[3] ^ tt.template get<0, 0>(x);
    }
#pragma unroll
    for (int r = 2; r < NR; ++r) {
#pragma unroll
        for (int b = 0; b < N; ++b)
            tt.round(s[b], o[b], &a.rk[4 * r], &krot[4 * r]);
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c) s[b][c] = o[b][c];
    }
#pragma unroll
    for (int b = 0; b < N; ++b)
        tt.last_round(s[b], ks[b], &a.rk[4 * NR]);
}

// ---- Rounds 1-2 shared by a wave ------------------------------------------
//
// Beyond the per-request constant k1, the counter's top three bytes change
// only every 256 blocks.  Within a "group" of counters with equal bits 31..8
// only byte 3 of x = bswap(ctr) ^ x0 varies, so of the round-1 output only
// column 0, s1_0 = k1[0] ^ T3[x.b3], varies; s1_1 = k1[1] ^ T2[x.b2],
// s1_2 = k1[2] ^ T1[x.b1], s1_3 = k1[3] ^ T0[x.b0] are group constants.  After
// ShiftRows every round-2 column takes exactly one byte of s1_0, so
//   s2_c = G_c ^ T_r(c)[byte r(c) of s1_0],  r(c) = (4 - c) mod 4,
// with G_c = rk2_c ^ (the three T-table terms from s1_1..s1_3).  Rounds 1-2
// then cost 5 lookups per block instead of 20.  A wave works on 64 x N
// consecutive counters (N <= 4), which span at most two groups; it computes
// their G once per step on the scalar unit.

// T_t[byte R of v] from the constant round tables; with a wave-uniform v
// this is one s_bfe and one s_load on the scalar unit, off the VALU and LDS
// pipes that the per-block rounds saturate.
template <int T, int R>
__device__ __forceinline__ uint32_t ctab(uint32_t v)
{
    return c_round.t[T][(v >> (8 * R)) & 255u];
}

// Round-2 group constants G_0..G_3 of counter group g (wave-uniform): G_c is
// rk2_c xor the row-R terms T_R[byte R of s1_(c+R mod 4)] from the three
// group-constant columns of round 1.  Bytes 0..2 of x = bswap(ctr) ^ x0 are
// the counter's bits 31..24, 23..16 and 15..8, i.e. bytes 2, 1, 0 of g.
__device__ __forceinline__ void group_consts(const CtrArgs &a, uint32_t g, uint32_t G[4])
{
    const uint32_t s1 = a.k1[1] ^ ctab<2, 0>(g ^ (a.x0 >> 16));   // T2[x.b2]
    const uint32_t s2 = a.k1[2] ^ ctab<1, 1>(g ^ a.x0);            // T1[x.b1]
    const uint32_t s3 = a.k1[3] ^ ctab<0, 2>(g ^ (a.x0 << 16));   // T0[x.b0]
    G[0] = a.rk[8] ^ ctab<1, 1>(s1) ^ ctab<2, 2>(s2) ^ ctab<3, 3>(s3);
    G[1] = a.rk[9] ^ ctab<0, 0>(s1) ^ ctab<1, 1>(s2) ^ ctab<2, 2>(s3);
    G[2] = a.rk[10] ^ ctab<0, 0>(s2) ^ ctab<1, 1>(s3) ^ ctab<3, 3>(s1);
    G[3] = a.rk[11] ^ ctab<0, 0>(s3) ^ ctab<2, 2>(s1) ^ ctab<3, 3>(s2);
}

// The same constants from the LDS tables, for a per-lane group g: the first
// chunk of a launch has every wave of a workgroup start at once, and one
// wave computing all of the workgroup's groups (a lane each) costs less than
// sixteen waves queueing on the CU's one scalar unit.
template <int LAYOUT>
__device__ __forceinline__ void group_consts_lds(const TTable<LAYOUT> &tt, const CtrArgs &a, uint32_t g,
                                                 uint32_t G[4])
{
    const uint32_t s1 = a.k1[1] ^ tt.template get<2, 0>(g ^ (a.x0 >> 16));
    const uint32_t s2 = a.k1[2] ^ tt.template get<1, 1>(g ^ a.x0);
    const uint32_t s3 = a.k1[3] ^ tt.template get<0, 2>(g ^ (a.x0 << 16));
    G[0] = a.rk[8] ^ tt.template get<1, 1>(s1) ^ tt.template get<2, 2>(s2) ^ tt.template get<3, 3>(s3);
    G[1] = a.rk[9] ^ tt.template get<0, 0>(s1) ^ tt.template get<1, 1>(s2) ^ tt.template get<2, 2>(s3);
    G[2] = a.rk[10] ^ tt.template get<0, 0>(s2) ^ tt.template get<1, 1>(s3) ^ tt.template get<3, 3>(s1);
    G[3] = a.rk[11] ^ tt.template get<0, 0>(s3) ^ tt.template get<2, 2>(s1) ^ tt.template get<3, 3>(s2);
}

// Most groups one workgroup chunk of up to 4096 consecutive counters spans.
constexpr int kChunkGroups = 17;

// The group constants one wave needs: its N x 64 counters are first + i
// (lane i mod 64, block i / 64), so they reach at most the next group.
struct WaveGroups {
    uint32_t gA;
    uint32_t GA[4], GB[4];
};

template <int N>
__device__ __forceinline__ WaveGroups wave_groups(const CtrArgs &a, uint32_t first)
{
    static_assert(64 * N <= 256, "a wave's counters must span at most two groups");
    WaveGroups w;
    w.gA = first >> 8;
    const uint32_t gB = (first + 64u * N - 1u) >> 8;
    group_consts(a, w.gA, w.GA);
    if (gB != w.gA) {
        group_consts(a, gB, w.GB);
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) w.GB[c] = w.GA[c];
    }
    return w;
}

// The same constants from the LDS tables, for a wave's first chunk, where
// every wave of the CU starts at once (sixteen waves' scalar group constants
// would queue on the CU's one scalar unit).  Four lanes per group: lane
// 4h + c computes column c of the wave's first (h = 0) or second (h = 1)
// group,
//   G_c = rk2_c ^ T_t1[byte t1 of s1_1] ^ T_t2[byte t2 of s1_2] ^ T_t3[byte t3 of s1_3],
// t_j = (j - c) mod 4 and T_t = rotl(T0, 8t), and v_readlane hands the eight
// words to the whole wave.  Every lane of the wave must be active (lanes 8
// and up compute values nobody reads).
template <int LAYOUT, int N>
__device__ __forceinline__ WaveGroups wave_groups_lds(const TTable<LAYOUT> &tt, const CtrArgs &a, uint32_t first,
                                                      uint32_t lane)
{
    static_assert(64 * N <= 256, "a wave's counters must span at most two groups");
    WaveGroups w;
    w.gA = first >> 8;
    const uint32_t g = (lane & 4) ? (first + 64u * N - 1u) >> 8 : w.gA;
    const uint32_t c = lane & 3;
    const uint32_t s1[3] = {a.k1[1] ^ tt.template get<2, 0>(g ^ (a.x0 >> 16)),
                            a.k1[2] ^ tt.template get<1, 1>(g ^ a.x0),
                            a.k1[3] ^ tt.template get<0, 2>(g ^ (a.x0 << 16))};
    uint32_t G = 0;
#pragma unroll
    for (uint32_t j = 1; j <= 3; ++j) {
        const uint32_t t = (j - c) & 3u;
        const uint32_t e = tt.t0_at(s1[j - 1], 8u * t);
        G ^= __builtin_amdgcn_alignbit(e, e, (32u - 8u * t) & 31u);   // rotl(e, 8t)
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        w.GA[k] = a.rk[8 + k] ^ static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(G), k));
        w.GB[k] = a.rk[8 + k] ^ static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(G), 4 + k));
    }
    return w;
}

// Keystream of N blocks per lane, lane i / block b holding counter
// first + 64 b + i where w = wave_groups<N>(a, first).  Every lane of the
// wave must be active.
template <int NR, int LAYOUT, int N>
__device__ __forceinline__ void keystream_wave(const TTable<LAYOUT> &tt, const CtrArgs &a, const uint32_t *krot,
                                               const uint32_t *ctr, const WaveGroups &w, uint32_t (*ks)[4])
{
    uint32_t s[N][4], o[N][4];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        const bool in_b = (ctr[b] >> 8) != w.gA;
        uint32_t G[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) G[c] = in_b ? w.GB[c] : w.GA[c];
        const uint32_t x = vperm(ctr[b], ctr[b], 0x00010203u) ^ a.x0;
        const uint32_t s10 = a.k1[0] ^ tt.template get<3, 3>(x);
        s[b][0] = G[0] ^ tt.template get<0, 0>(s10);
        s[b][1] = G[1] ^ tt.template get<3, 3>(s10);
        s[b][2] = G[2] ^ tt.template get<2, 2>(s10);
        s[b][3] = G[3] ^ tt.template get<1, 1>(s10);
    }
#pragma unroll
    for (int r = 3; r < NR; ++r) {
#pragma unroll
        for (int b = 0; b < N; ++b)
            tt.round(s[b], o[b], &a.rk[4 * r], &krot[4 * r]);
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c) s[b][c] = o[b][c];
    }
#pragma unroll
    for (int b = 0; b < N; ++b)
        tt.last_round(s[b], ks[b], &a.rk[4 * NR]);
}

}  // namespace
}  // namespace aesctr
