// ctr_vperm.hip -- AES-CTR keystream + XOR with no memory lookups: the S-box
// from 16-entry nibble lookups done by the byte permute v_perm_b32 (gfx950).
//
// The approach follows Hamburg, "Accelerating AES with vector permute
// instructions" (CHES 2009): invert in GF(2^8) through its subfield GF(2^4),
// where every nonlinear step is a lookup in a 16-entry table.  The tower, the
// inversion chain and every table are derived in gen_vperm_tables.py, which
// writes vperm_tables.inc; the key facts used here:
//   - a state byte s is held as two nibbles (i, k) of its tower
//     representation, each in its own byte lane as E(n) = (n & 7) | n3 << 7;
//     XOR of encodings is the encoding of the XOR, and 0x40 stands for inf;
//   - a lookup of byte lanes e is perm(W1, W0, e) ^ perm(W3, W2, e ^ 0x80),
//     with the table's complemented entries in W0..W3 (v_perm gives 0xff for
//     a selector of 13 or more, so exactly one permute per lane yields an
//     entry, and inf yields 0);
//   - the inversion chain is ak = a/k, ia = 1/i + ak, ja = 1/(i+k) + ak,
//     io = 1/ia + (i+k), jo = 1/ja + i, and any GF(2)-linear function of
//     s^-1 is F[io] ^ G[jo] for two tables; the round's output tables give
//     the (i, k) nibbles of S(s) - {63} and of 2*(S(s) - {63}), the last
//     round's give standard bytes, and {63} is folded into the round keys.
//
// Layout.  One lane encrypts one 16-byte counter block.  The state is kept by
// rows: word r holds row r of the four columns (byte c = column c), as i- and
// k-nibble words, so ShiftRows is a rotate of each row word and MixColumns is
// a XOR of row words:
//   out_r = 2 S_r ^ 2 S_(r+1) ^ S_(r+1) ^ S_(r+2) ^ S_(r+3) ^ rk_r.
// Round 1 is cached (counter mode): columns 0-2 of the round-0 state are the
// constant nonce xor rk0, and after ShiftRows output column c takes exactly
// one counter byte, the one of row 3 - c.  So one inversion chain on the
// counter column's four bytes (converted to (i, k) form in the kernel, four
// nibble lookups) gives every varying term of round 1, and the host folds the
// rest of each output row, with rk1, into one constant per row.  The
// keystream leaves as standard bytes, transposed back to column words.
#include <string.h>

#include "aes_tables.h"
#include "aesctr_internal.h"

namespace aesctr {
namespace {

#include "vperm_tables.inc"

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kHi = 0x80808080u;

__device__ __forceinline__ uint32_t vperm(uint32_t s0, uint32_t s1, uint32_t sel)
{
    return __builtin_amdgcn_perm(s0, s1, sel);
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Table lookup of the four byte lanes of e (ec = e ^ 0x80808080): the two
// permutes whose XOR is the lookup, left apart so the XOR can merge with the
// next one into a 3-input XOR.
struct Pair {
    uint32_t a, b;
};

template <const uint32_t (&T)[4]>
__device__ __forceinline__ Pair look(uint32_t e, uint32_t ec)
{
    return Pair{vperm(T[1], T[0], e), vperm(T[3], T[2], ec)};
}

// lookup ^ x
__device__ __forceinline__ uint32_t plus(const Pair &p, uint32_t x)
{
    return xor3(p.a, p.b, x);
}

__device__ __forceinline__ uint32_t rotr(uint32_t x, int n)
{
    return n ? __builtin_amdgcn_alignbit(x, x, n) : x;
}

// The inversion chain of one row word: (i, k) nibble words -> (io, jo),
// each also with its top bits flipped (the second permute's selector).
struct Chain {
    uint32_t io, ioc, jo, joc;
};

__device__ __forceinline__ Chain chain(uint32_t I, uint32_t K)
{
    const uint32_t Ic = I ^ kHi, Kc = K ^ kHi;
    const Pair pa = look<kVp_adiv>(K, Kc);
    const uint32_t ak = pa.a ^ pa.b, akc = xor3(pa.a, pa.b, kHi);
    const uint32_t j = I ^ K, jc = xor3(I, K, kHi);
    const Pair pi = look<kVp_inv>(I, Ic);
    const Pair pj = look<kVp_inv>(j, jc);
    const uint32_t ia = plus(pi, ak), iac = plus(pi, akc);
    const uint32_t ja = plus(pj, ak), jac = plus(pj, akc);
    const Pair qi = look<kVp_inv>(ia, iac);
    const Pair qj = look<kVp_inv>(ja, jac);
    Chain c;
    c.io = plus(qi, j);
    c.ioc = plus(qi, jc);
    c.jo = plus(qj, I);
    c.joc = plus(qj, Ic);
    return c;
}

template <const uint32_t (&F)[4], const uint32_t (&G)[4]>
__device__ __forceinline__ uint32_t out_of(const Chain &c)
{
    const Pair f = look<F>(c.io, c.ioc);
    const Pair g = look<G>(c.jo, c.joc);
    return xor3(f.a, f.b, g.a) ^ g.b;
}

// MixColumns coefficient of row rp's byte in output row r: {02} on the
// diagonal, {03} just right of it, {01} elsewhere.
constexpr int mix_coef(int r, int rp) { return rp == r ? 2 : rp == ((r + 1) & 3) ? 3 : 1; }

// Round 1, output row r: byte c holds coefficient mix_coef(r, 3 - c) times
// S'(x_(3-c)), x_j being the counter column's byte of row j.  With S (byte j
// = S'(x_j)), D = 2S and T = S ^ D = 3S: row1_sel picks S or T bytes (from
// v_perm_b32(T, S, .)), 0x0c zeroes the {02} byte, and row1_dsel places D's
// byte there (from v_perm_b32(D, D, .)).
constexpr uint32_t row1_sel(int r)
{
    uint32_t s = 0;
    for (int c = 0; c < 4; ++c) {
        const int rp = 3 - c, k = mix_coef(r, rp);
        s |= static_cast<uint32_t>(k == 1 ? rp : k == 3 ? 4 + rp : 12) << (8 * c);
    }
    return s;
}
constexpr uint32_t row1_dsel(int r)
{
    uint32_t s = 0;
    for (int c = 0; c < 4; ++c) {
        const int rp = 3 - c;
        s |= static_cast<uint32_t>(rp == r ? rp : 12) << (8 * c);
    }
    return s;
}

// AES-256's nibble-form round keys in LDS, read back 16 bytes at a time
// (the same address for every lane).  Held in scalar registers, its 104 words
// spill to vector-register lanes and come back with a v_readlane each (about
// 120 per block); the kernel is bound by VALU issue, and LDS is otherwise
// idle.  AES-128's 72 words stay in scalar registers (about 30 spilled reads
// per block, which measured cheaper than the LDS reads).
template <int NR>
constexpr bool keys_in_lds() { return NR == 14; }

struct VpKeyTable {
    u32x4 k[13][2];     // [t - 1]: (rki, rkk) of round t; [0]: round 1's constant rows
    u32x4 kn;           // rkn
};

// Filled by lane 0 of the workgroup (wave-uniform sources, no per-lane
// indexing of the argument block).
template <int NR>
__device__ __forceinline__ void fill_keys(const VpArgs &a, VpKeyTable &t)
{
    if (keys_in_lds<NR>() && threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NR - 1; ++i) {
            t.k[i][0] = u32x4{a.rki[i][0], a.rki[i][1], a.rki[i][2], a.rki[i][3]};
            t.k[i][1] = u32x4{a.rkk[i][0], a.rkk[i][1], a.rkk[i][2], a.rkk[i][3]};
        }
        t.kn = u32x4{a.rkn[0], a.rkn[1], a.rkn[2], a.rkn[3]};
    }
}

// Round t's key rows (i and k nibbles), t = 1..NR-1 (t = 1: round 1's
// constant rows), and the last round's.
template <int NR>
__device__ __forceinline__ void round_keys(const VpArgs &a, const VpKeyTable &kt, int t, u32x4 &ki, u32x4 &kk)
{
    if constexpr (keys_in_lds<NR>()) {
        ki = kt.k[t - 1][0];
        kk = kt.k[t - 1][1];
    } else {
        ki = u32x4{a.rki[t - 1][0], a.rki[t - 1][1], a.rki[t - 1][2], a.rki[t - 1][3]};
        kk = u32x4{a.rkk[t - 1][0], a.rkk[t - 1][1], a.rkk[t - 1][2], a.rkk[t - 1][3]};
    }
}

template <int NR>
__device__ __forceinline__ u32x4 last_key(const VpArgs &a, const VpKeyTable &kt)
{
    if constexpr (keys_in_lds<NR>())
        return kt.kn;
    else
        return u32x4{a.rkn[0], a.rkn[1], a.rkn[2], a.rkn[3]};
}

// Keystream block of counter value ctr (already ctr0 + j) -> column words.
template <int NR>
__device__ __forceinline__ void keystream_vp(const VpArgs &a, const VpKeyTable &kt, uint32_t ctr,
                                             uint32_t (&ks)[4])
{
    // Round 0 of the counter column: ctr xor rk0 in standard bytes (byte r =
    // row r), converted to (i, k) nibbles.
    const uint32_t X = vperm(ctr, ctr, 0x00010203u) ^ a.x0;
    const uint32_t lo = (X & 0x07070707u) | ((X << 4) & kHi);
    const uint32_t hi = ((X >> 4) & 0x07070707u) | (X & kHi);
    const uint32_t loc = lo ^ kHi, hic = hi ^ kHi;
    const Pair il = look<kVp_cvi_lo>(lo, loc), ih = look<kVp_cvi_hi>(hi, hic);
    const Pair kl = look<kVp_cvk_lo>(lo, loc), kh = look<kVp_cvk_hi>(hi, hic);
    const uint32_t XI = xor3(il.a, il.b, ih.a) ^ ih.b;
    const uint32_t XK = xor3(kl.a, kl.b, kh.a) ^ kh.b;
    // Round 1: one chain for the four counter bytes; the rest of each row is
    // the host's constant (rki[0] / rkk[0]).
    uint32_t I[4], K[4];
    {
        const Chain c = chain(XI, XK);
        const uint32_t SI = out_of<kVp_si_f, kVp_si_g>(c), SK = out_of<kVp_sk_f, kVp_sk_g>(c);
        const uint32_t DI = out_of<kVp_di_f, kVp_di_g>(c), DK = out_of<kVp_dk_f, kVp_dk_g>(c);
        const uint32_t TI = SI ^ DI, TK = SK ^ DK;
        u32x4 ki, kk;
        round_keys<NR>(a, kt, 1, ki, kk);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            I[r] = xor3(vperm(TI, SI, row1_sel(r)), vperm(DI, DI, row1_dsel(r)), ki[r]);
            K[r] = xor3(vperm(TK, SK, row1_sel(r)), vperm(DK, DK, row1_dsel(r)), kk[r]);
        }
    }
#pragma unroll
    for (int t = 2; t < NR; ++t) {
        uint32_t SI[4], SK[4], DI[4], DK[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const Chain c = chain(rotr(I[r], 8 * r), rotr(K[r], 8 * r));
            SI[r] = out_of<kVp_si_f, kVp_si_g>(c);
            SK[r] = out_of<kVp_sk_f, kVp_sk_g>(c);
            DI[r] = out_of<kVp_di_f, kVp_di_g>(c);
            DK[r] = out_of<kVp_dk_f, kVp_dk_g>(c);
        }
        u32x4 ki, kk;
        round_keys<NR>(a, kt, t, ki, kk);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int r1 = (r + 1) & 3, r2 = (r + 2) & 3, r3 = (r + 3) & 3;
            I[r] = xor3(xor3(DI[r], DI[r1], SI[r1]), xor3(SI[r2], SI[r3], ki[r]), 0u);
            K[r] = xor3(xor3(DK[r], DK[r1], SK[r1]), xor3(SK[r2], SK[r3], kk[r]), 0u);
        }
    }
    uint32_t row[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const Chain c = chain(rotr(I[r], 8 * r), rotr(K[r], 8 * r));
        const Pair f = look<kVp_out_f>(c.io, c.ioc);
        const Pair g = look<kVp_out_g>(c.jo, c.joc);
        row[r] = xor3(xor3(f.a, f.b, g.a), g.b, last_key<NR>(a, kt)[r]);
    }
    // Rows -> columns: ks[c] byte r = row[r] byte c.
    const uint32_t t01l = vperm(row[1], row[0], 0x05010400u);   // r0c0 r1c0 r0c1 r1c1
    const uint32_t t01h = vperm(row[1], row[0], 0x07030602u);   // r0c2 r1c2 r0c3 r1c3
    const uint32_t t23l = vperm(row[3], row[2], 0x05010400u);
    const uint32_t t23h = vperm(row[3], row[2], 0x07030602u);
    ks[0] = vperm(t23l, t01l, 0x05040100u);
    ks[1] = vperm(t23l, t01l, 0x07060302u);
    ks[2] = vperm(t23h, t01h, 0x05040100u);
    ks[3] = vperm(t23h, t01h, 0x07060302u);
}

template <int NR, bool ALIGNED>
__global__ __launch_bounds__(256) void ctr_vperm_kernel(const VpArgs a)
{
    const uint64_t nfull = a.len >> 4;
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    __shared__ VpKeyTable kt;
    if constexpr (keys_in_lds<NR>()) {
        fill_keys<NR>(a, kt);
        __syncthreads();
    }
    for (uint64_t idx = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < nfull; idx += step) {
        // The key table never changes, but its reads must stay in their
        // rounds (hoisted out of the loop they would hold every round key in
        // registers).  A compiler-only barrier (no instruction).
        if constexpr (keys_in_lds<NR>())
            asm volatile("" ::: "memory");
        u32x4 d;
        if constexpr (ALIGNED) {
            d = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(a.in) + idx);
        } else {
            __builtin_memcpy(&d, a.in + 16 * idx, 16);
        }
        uint32_t ks[4];
        keystream_vp<NR>(a, kt, a.ctr0 + static_cast<uint32_t>(idx), ks);
        const u32x4 v = d ^ u32x4{ks[0], ks[1], ks[2], ks[3]};
        if constexpr (ALIGNED) {
            __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(a.out) + idx);
        } else {
            __builtin_memcpy(a.out + 16 * idx, &v, 16);
        }
    }
    // Final partial block: leading bytes of its keystream block.
    const uint32_t tail = static_cast<uint32_t>(a.len & 15);
    if (tail != 0 && blockIdx.x == gridDim.x - 1 && threadIdx.x == blockDim.x - 1) {
        uint32_t ks[4];
        keystream_vp<NR>(a, kt, a.ctr0 + static_cast<uint32_t>(nfull), ks);
        const uint64_t off = 16 * nfull;
        for (uint32_t i = 0; i < tail; ++i)
            a.out[off + i] = a.in[off + i] ^ static_cast<uint8_t>(ks[i >> 2] >> (8 * (i & 3)));
    }
}

template <int NR>
int launch_nr(const VpArgs &a, const Shape &sh, hipStream_t st)
{
    const bool aligned = ((reinterpret_cast<uintptr_t>(a.in) | reinterpret_cast<uintptr_t>(a.out)) & 15) == 0;
    (void)hipGetLastError();   // not ours: left by earlier calls
    if (aligned)
        hipLaunchKernelGGL((ctr_vperm_kernel<NR, true>), dim3(sh.grid), dim3(sh.wg), 0, st, a);
    else
        hipLaunchKernelGGL((ctr_vperm_kernel<NR, false>), dim3(sh.grid), dim3(sh.wg), 0, st, a);
    return launch_status();
}

// (i, k) nibble encodings of byte v as a pair of bytes.
inline uint32_t part_i(uint32_t v) { return kVpToParts[v & 255] & 0xffu; }
inline uint32_t part_k(uint32_t v) { return kVpToParts[v & 255] >> 8; }

}  // namespace

void make_vperm_args(const aes_sched_t &s, const uint8_t nonce[12], uint32_t ctr0, const void *in, void *out,
                     uint64_t len, VpArgs *a)
{
    memset(a, 0, sizeof(*a));
    a->in = static_cast<const uint8_t *>(in);
    a->out = static_cast<uint8_t *>(out);
    a->len = len;
    a->ctr0 = ctr0;
    const int nr = s.nr;
    // Byte r of column c of round key t: byte r (from the top) of schedule
    // word 4t + c (FIPS-197 words are big-endian packed).
    auto rk = [&](int t, int c, int r) { return (s.rk[4 * t + c] >> (24 - 8 * r)) & 0xffu; };
    for (int r = 0; r < 4; ++r)
        a->x0 |= rk(0, 3, r) << (8 * r);
    // Round 1's constant part.  Output column c (a word, byte r = row r) is
    // rk1's column c xor the S-box-and-MixColumns terms tr(r', b) of the
    // three constant bytes b = state(r', c + r') (columns 0-2 of nonce xor
    // rk0, r' != 3 - c), xor the MixColumns term of {63} in row 3 - c: the
    // kernel adds that row's counter term from the S - {63} tables.
    uint32_t col[4];
    for (int c = 0; c < 4; ++c) {
        uint32_t w = 0;
        for (int r = 0; r < 4; ++r)
            w |= rk(1, c, r) << (8 * r);
        for (int rp = 0; rp < 4; ++rp) {
            if (rp == 3 - c)
                continue;
            const int cc = (c + rp) & 3;
            w ^= tr(rp, static_cast<uint8_t>(nonce[4 * cc + rp] ^ rk(0, cc, rp)));
        }
        const uint8_t s63 = 0x63, d63 = gf_double(s63);
        const uint32_t t63 = static_cast<uint32_t>(d63) | static_cast<uint32_t>(s63) << 8 |
                             static_cast<uint32_t>(s63) << 16 | static_cast<uint32_t>(d63 ^ s63) << 24;
        col[c] = w ^ rotl32(t63, 8 * (3 - c));
    }
    for (int r = 0; r < 4; ++r) {
        uint32_t wi = 0, wk = 0;
        for (int c = 0; c < 4; ++c) {
            const uint32_t v = (col[c] >> (8 * r)) & 0xffu;
            wi |= part_i(v) << (8 * c);
            wk |= part_k(v) << (8 * c);
        }
        a->rki[0][r] = wi;
        a->rkk[0][r] = wk;
    }
    for (int t = 2; t < nr; ++t)
        for (int r = 0; r < 4; ++r) {
            uint32_t wi = 0, wk = 0;
            for (int c = 0; c < 4; ++c) {
                const uint32_t v = rk(t, c, r) ^ 0x63u;
                wi |= part_i(v) << (8 * c);
                wk |= part_k(v) << (8 * c);
            }
            a->rki[t - 1][r] = wi;
            a->rkk[t - 1][r] = wk;
        }
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            a->rkn[r] |= (rk(nr, c, r) ^ 0x63u) << (8 * c);
}

int launch_ctr_vperm(const VpArgs &a, int nr, const Shape &sh, hipStream_t st)
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
