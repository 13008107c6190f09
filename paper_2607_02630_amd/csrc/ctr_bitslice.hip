// ctr_bitslice.hip -- AES-CTR keystream + XOR, bitsliced (gfx950).
//
// Layout.  Four consecutive lanes (a quad) share 32 counter blocks; lane q of
// the quad holds state column q (FIPS-197 Sec. 3.4) of all 32 blocks as 32
// "slice" words: word (r, b) carries bit b of the byte in row r, bit i of the
// word belonging to block chunk + 16*i + quad.  A wave covers 512 blocks,
// so an 8 MiB buffer still spreads over every SIMD.
//
// Round transformations (FIPS-197 Sec. 5.1) on slices:
//   SubBytes    the S-box as a straight-line program of 3-input boolean
//               functions (v_bitop3_b32), generated from the field arithmetic
//               by gen_sbox_circuit.py into sbox_circuit.inc; four per lane;
//   ShiftRows   row r of column q comes from column q + r: a DPP quad_perm
//               read from the neighbouring lane of the quad;
//   MixColumns  inside the lane: with t_r = a_r ^ a_(r+1) and
//               T = a_0^a_1^a_2^a_3 each output byte is xtime(t_r) ^ T ^ a_r;
//   AddRoundKey a round-key bit is the same for all 32 blocks of the lane:
//               a 0 / ~0 mask folded into the MixColumns 3-input XORs.  The
//               masks of every round and column are built once per
//               workgroup into LDS and read back 16 bytes at a time (the
//               kernel is bound by VALU issue; LDS is otherwise idle).
// Counter blocks are built directly in sliced form (no transpose on the way
// in).  Rounds 0 and 1 use the per-request constant k1 shared with the
// T-table kernel: round 1 needs one S-box per lane, on the counter byte that
// lands in its column.  The keystream is transposed back to words in
// registers (byte-granular stages by v_perm_b32, bit-granular ones by shift
// + bitop3 select); lane q then owns word q of each block, so each dword
// load/store instruction of a wave covers 256 consecutive bytes.
#include "aesctr_internal.h"

namespace aesctr {
namespace {

#define bitop3(a, b, c, t) __builtin_amdgcn_bitop3_b32((a), (b), (c), (t))

__device__ __forceinline__ void sbox_bs(uint32_t (&x)[8])
{
#include "sbox_circuit.inc"
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return bitop3(a, b, c, 0x96); }

// 0 or ~0 from bit n of w (n may differ per lane).
__device__ __forceinline__ uint32_t bitmask(uint32_t w, uint32_t n)
{
    return 0u - ((w >> n) & 1u);
}

__device__ __forceinline__ uint32_t sel4(uint32_t q, uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3)
{
    return q == 0 ? v0 : q == 1 ? v1 : q == 2 ? v2 : v3;
}

// Value of v in lane (q + R) mod 4 of this lane's quad.  Every row and bank
// is enabled and a quad permutation reads only lanes of the same quad, so
// every lane is written: the DPP move needs no "old" value (one with
// update_dpp costs a v_mov of the old value per exchange).
template <int R>
__device__ __forceinline__ uint32_t from_quad(uint32_t v)
{
    constexpr int ctrl = ((0 + R) & 3) | (((1 + R) & 3) << 2) | (((2 + R) & 3) << 4) | (((3 + R) & 3) << 6);
    return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), ctrl, 0xF, 0xF, false));
}

// Slices of the 32-bit counters c_i = C + 16*i (i = 0..31), C = this quad's
// counter for i = 0: cs[k] bit i = bit k of c_i.  Bits 0..3 of c_i are those
// of C; bits 4.. are those of D + i with D = C >> 4, d = D mod 32:
//   bits 0..4 of D + i  -> (d + i) mod 32, the pattern of i rotated by d;
//   bits 5..27          -> from H = D - d for i < 32 - d, from H + 32 after.
__device__ __forceinline__ void counter_slices(uint32_t C, uint32_t (&cs)[32])
{
    const uint32_t pat[5] = {0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u, 0xFF00FF00u, 0xFFFF0000u};
#pragma unroll
    for (int k = 0; k < 4; ++k)
        cs[k] = bitmask(C, k);
    const uint32_t D = C >> 4;
    const uint32_t d = D & 31;
    const uint32_t H0 = D - d;
    const uint32_t H1 = H0 + 32;
    const uint32_t M = d ? (0xFFFFFFFFu << (32 - d)) : 0u;   // bits i >= 32 - d
#pragma unroll
    for (int m = 0; m < 5; ++m)
        cs[4 + m] = d ? __builtin_amdgcn_alignbit(pat[m], pat[m], d) : pat[m];
#pragma unroll
    for (int m = 5; m < 28; ++m)
        cs[4 + m] = bitop3(M, bitmask(H1, m), bitmask(H0, m), 0xCA);   // M ? hi : lo
}

// xtime on a sliced byte: bit b of {02}*a.
__device__ __forceinline__ uint32_t xt_bit(const uint32_t (&a)[8], int b)
{
    if (b == 0)
        return a[7];
    if (b == 1 || b == 3 || b == 4)
        return a[b - 1] ^ a[7];
    return a[b - 1];
}

// ShiftRows for this lane's column: row r from lane q + r of the quad.
__device__ __forceinline__ void shift_rows(uint32_t (&st)[4][8])
{
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        st[1][b] = from_quad<1>(st[1][b]);
        st[2][b] = from_quad<2>(st[2][b]);
        st[3][b] = from_quad<3>(st[3][b]);
    }
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Round-key masks (0 or ~0, one per key bit) in LDS.  Entry e, column q:
// e = 0: the counter column's round-0 key byte that lands in column q (row
// 3 - q), bits 0-7; e = 1: k1[q]; e = 2..NR: round key word 4e + q; word 8r
// + b is bit b of row r.  Rows of 36 words (144 bytes), so the 16-byte reads
// of the four columns in one instruction start on different banks.
constexpr int kMaskRow = 36;

template <int NR>
struct MaskTable {
    uint32_t m[NR + 1][4][kMaskRow];
};

// Fills the table: the (column, bit) pairs are spread over the workgroup,
// the entries unrolled so every key word index is uniform.
template <int NR>
__device__ __forceinline__ void fill_masks(const CtrArgs &a, MaskTable<NR> &t)
{
    for (uint32_t p = threadIdx.x; p < 128; p += blockDim.x) {
        const uint32_t q = p >> 5, j = p & 31;
        t.m[0][q][j] = j < 8 ? bitmask(a.x0, 8 * (3 - q) + j) : 0u;
        t.m[1][q][j] = bitmask(sel4(q, a.k1[0], a.k1[1], a.k1[2], a.k1[3]), j);
#pragma unroll
        for (int e = 2; e <= NR; ++e)
            t.m[e][q][j] = bitmask(sel4(q, a.rk[4 * e], a.rk[4 * e + 1], a.rk[4 * e + 2], a.rk[4 * e + 3]), j);
    }
}

// The 32 masks of one entry for this lane's column, in registers.
__device__ __forceinline__ void read_masks(const uint32_t *row, uint32_t (&km)[32])
{
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const u32x4 v = reinterpret_cast<const u32x4 *>(row)[i];
        km[4 * i] = v[0];
        km[4 * i + 1] = v[1];
        km[4 * i + 2] = v[2];
        km[4 * i + 3] = v[3];
    }
}

// MixColumns + AddRoundKey on this lane's column; km = the masks of the
// lane's round-key column (word 8r + b: bit b of row r).
__device__ __forceinline__ void mix_column(uint32_t (&a)[4][8], const uint32_t (&km)[32])
{
    uint32_t t[4][8], tot[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        t[0][b] = a[0][b] ^ a[1][b];
        t[1][b] = a[1][b] ^ a[2][b];
        t[2][b] = a[2][b] ^ a[3][b];
        t[3][b] = xor3(t[0][b], t[1][b], t[2][b]);     // a3 ^ a0
        tot[b] = t[0][b] ^ t[2][b];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint32_t k = km[8 * r + b];
            uint32_t v;
            if (b == 0)
                v = xor3(xor3(t[r][7], tot[0], a[r][0]), k, 0);
            else if (b == 1 || b == 3 || b == 4)
                v = xor3(xor3(t[r][b - 1], t[r][7], tot[b]), a[r][b], k);
            else
                v = xor3(xor3(t[r][b - 1], tot[b], a[r][b]), k, 0);
            a[r][b] = v;
        }
    }
}

// 32x32 bit transpose of w in place: afterwards w[i] bit q = old w[q] bit i.
__device__ __forceinline__ void transpose32(uint32_t (&w)[32])
{
    // j = 16 and 8 move whole bytes: one v_perm_b32 per output word.
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint32_t a = w[q], b = w[q + 16];
        w[q] = __builtin_amdgcn_perm(b, a, 0x05040100u);        // [a0 a1 b0 b1]
        w[q + 16] = __builtin_amdgcn_perm(b, a, 0x07060302u);   // [a2 a3 b2 b3]
    }
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        if (q & 8)
            continue;
        const uint32_t a = w[q], b = w[q + 8];
        w[q] = __builtin_amdgcn_perm(b, a, 0x06020400u);        // [a0 b0 a2 b2]
        w[q + 8] = __builtin_amdgcn_perm(b, a, 0x07030501u);    // [a1 b1 a3 b3]
    }
    const uint32_t masks[3] = {0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int j = 4 >> s;
        const uint32_t m = masks[s];
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            if (q & j)
                continue;
            const uint32_t a = w[q], b = w[q + j];
            w[q] = bitop3(m, a, b << j, 0xCA);          // m ? a : b << j
            w[q + j] = bitop3(m, a >> j, b, 0xCA);      // m ? a >> j : b
        }
    }
}

// Keystream of this lane's column for the quad's 32 blocks, as slices.
// q = column, C = counter of block i = 0.
template <int NR>
__device__ __forceinline__ void keystream_column(const MaskTable<NR> &mt, uint32_t q, uint32_t C,
                                                 uint32_t (&st)[4][8])
{
    // Rounds 0 + 1.  The counter column x = bswap(ctr) ^ x0 has byte r equal
    // to counter byte 12 + r (big-endian) XOR byte r of x0; its byte r lands
    // in column 3 - r through T_r.  This lane's column q takes byte r = 3 - q,
    // i.e. counter bits 8q .. 8q+7.
    {
        uint32_t cs[32];
        counter_slices(C, cs);
        const uint32_t r = 3 - q;
        uint32_t km[32];
        read_masks(mt.m[0][q], km);
        uint32_t y[8];
#pragma unroll
        for (int b = 0; b < 8; ++b)
            y[b] = sel4(q, cs[b], cs[8 + b], cs[16 + b], cs[24 + b]) ^ km[b];
        sbox_bs(y);
        // Row i gets coef[(i - r) mod 4] * S(x_r), coef = {02},{01},{01},{03}.
        read_masks(mt.m[1][q], km);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t ci = (static_cast<uint32_t>(i) - r) & 3;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const uint32_t x2 = xt_bit(y, b);
                const uint32_t v = ci == 0 ? x2 : ci == 3 ? (x2 ^ y[b]) : y[b];
                st[i][b] = v ^ km[8 * i + b];
            }
        }
    }
#pragma unroll
    for (int rnd = 2; rnd < NR; ++rnd) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            sbox_bs(st[r]);
        shift_rows(st);
        uint32_t km[32];
        read_masks(mt.m[rnd][q], km);
        mix_column(st, km);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        sbox_bs(st[r]);
    shift_rows(st);
    uint32_t km[32];
    read_masks(mt.m[NR][q], km);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int b = 0; b < 8; ++b) st[r][b] ^= km[8 * r + b];
}

template <bool ALIGNED>
__device__ __forceinline__ uint32_t load_word(const uint8_t *p)
{
    if constexpr (ALIGNED) {
        return __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(p));
    } else {
        uint32_t v;
        __builtin_memcpy(&v, p, 4);
        return v;
    }
}

template <bool ALIGNED>
__device__ __forceinline__ void store_word(uint8_t *p, uint32_t v)
{
    if constexpr (ALIGNED) {
        __builtin_nontemporal_store(v, reinterpret_cast<uint32_t *>(p));
    } else {
        __builtin_memcpy(p, &v, 4);
    }
}

template <int NR, bool ALIGNED>
__global__ __launch_bounds__(256) void ctr_bitslice_kernel(const CtrArgs a)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t q = lane & 3;
    const uint32_t g = lane >> 2;
    const uint64_t nblocks = (a.len + 15) >> 4;
    const uint64_t nfull = a.len >> 4;
    const uint64_t waves_per_wg = blockDim.x >> 6;
    const uint64_t gw = blockIdx.x * waves_per_wg + (threadIdx.x >> 6);
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * waves_per_wg * 512;
    __shared__ MaskTable<NR> mt;
    fill_masks<NR>(a, mt);
    __syncthreads();

    for (uint64_t base = gw * 512; base < nblocks; base += step) {
        // The mask table never changes, but its reads must stay in the round
        // that uses them: hoisted out of the loop they would hold all 352
        // masks in registers.  A compiler-only barrier (no instruction).
        asm volatile("" ::: "memory");
        // Data words first (block base + 16 i + g, word q); their latency
        // hides behind the rounds.
        uint32_t d[32];
        const bool whole = base + 512 <= nfull;
        if (whole) {
#pragma unroll
            for (int i = 0; i < 32; ++i)
                d[i] = load_word<ALIGNED>(a.in + 16 * (base + 16 * i + g) + 4 * q);
        }
        uint32_t st[4][8];
        keystream_column<NR>(mt, q, a.ctr0 + static_cast<uint32_t>(base + g), st);
        uint32_t w[32];
#pragma unroll
        for (int k = 0; k < 32; ++k)
            w[k] = st[k >> 3][k & 7];
        transpose32(w);      // w[i] = keystream word q of block base + 16 i + g
        if (whole) {
#pragma unroll
            for (int i = 0; i < 32; ++i)
                store_word<ALIGNED>(a.out + 16 * (base + 16 * i + g) + 4 * q, d[i] ^ w[i]);
        } else {
            for (int i = 0; i < 32; ++i) {
                const uint64_t idx = base + 16 * i + g;
                if (idx < nfull) {
                    const uint64_t off = 16 * idx + 4 * q;
                    store_word<ALIGNED>(a.out + off, load_word<ALIGNED>(a.in + off) ^ w[i]);
                } else if (idx == nfull && idx < nblocks) {
                    // Final partial block: leading bytes of its keystream.
                    const uint32_t tail = static_cast<uint32_t>(a.len & 15);
                    for (uint32_t t = 4 * q; t < tail && t < 4 * q + 4; ++t)
                        a.out[16 * idx + t] = a.in[16 * idx + t] ^ static_cast<uint8_t>(w[i] >> (8 * (t & 3)));
                }
            }
        }
    }
}

template <int NR>
int launch_nr(const CtrArgs &a, const Shape &sh, hipStream_t st)
{
    const bool aligned = ((reinterpret_cast<uintptr_t>(a.in) | reinterpret_cast<uintptr_t>(a.out)) & 3) == 0;
    (void)hipGetLastError();   // not ours: left by earlier calls
    if (aligned)
        hipLaunchKernelGGL((ctr_bitslice_kernel<NR, true>), dim3(sh.grid), dim3(sh.wg), 0, st, a);
    else
        hipLaunchKernelGGL((ctr_bitslice_kernel<NR, false>), dim3(sh.grid), dim3(sh.wg), 0, st, a);
    return launch_status();
}

}  // namespace

int launch_ctr_bitslice(const CtrArgs &a, int nr, const Shape &sh, hipStream_t st)
{
    if (sh.wg < 64 || sh.wg > 256 || sh.wg % 64 != 0 || sh.grid <= 0)
        return AES_EINVAL;
    if (nr == 10)
        return launch_nr<10>(a, sh, st);
    if (nr == 14)
        return launch_nr<14>(a, sh, st);
    return AES_EINVAL;
}

}  // namespace aesctr
