// sha256_batch.hip -- SHA-256 of many independent messages, one lane each.
//
// FIPS 180-4: padding (Sec. 5.1.1), parsing into 512-bit blocks of sixteen
// big-endian words (Sec. 5.2.1), the message schedule and 64 rounds of the
// hash computation (Sec. 6.2.2) with the functions of Sec. 4.1.2.  The round
// constants (Sec. 4.2.2) and the initial hash value (Sec. 5.3.3) are derived
// at compile time from their definitions.
//
// gfx950 mapping: a lane owns one message and keeps the eight working
// variables and a rolling 16-word schedule in registers; the 64 rounds are
// unrolled so every K_t is an instruction literal.  Rotations are single
// v_alignbit_b32, Ch / Maj / three-way XORs single v_bitop3_b32, and the sums
// v_add3_u32.  The host orders a launch's messages longest first, so lanes of
// a wave run for similar lengths.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shabatch_internal.h"

namespace aesctr {
namespace {

// ---- Constants from their definitions (compile time) --------------------

constexpr bool is_prime(uint32_t n)
{
    if (n < 2)
        return false;
    for (uint32_t d = 2; d * d <= n; ++d)
        if (n % d == 0)
            return false;
    return true;
}

constexpr uint32_t nth_prime(int i)
{
    uint32_t n = 1;
    for (int found = -1; found < i;)
        if (is_prime(++n))
            ++found;
    return n;
}

// floor(x^(1/e)) for e = 2, 3 by bisection over exact 128-bit integers.
constexpr uint64_t int_root(unsigned __int128 x, int e)
{
    uint64_t lo = 0, hi = uint64_t(1) << 40;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        unsigned __int128 p = static_cast<unsigned __int128>(mid) * mid;
        if (e == 3)
            p *= mid;
        if (p <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// First 32 bits of the fractional part of the e-th root of p.
constexpr uint32_t frac_bits(uint32_t p, int e)
{
    return static_cast<uint32_t>(int_root(static_cast<unsigned __int128>(p) << (32 * e), e));
}

struct ShaConsts {
    uint32_t k[64];
    uint32_t h0[8];
};

constexpr ShaConsts make_consts()
{
    ShaConsts c{};
    for (int i = 0; i < 64; ++i)
        c.k[i] = frac_bits(nth_prime(i), 3);
    for (int i = 0; i < 8; ++i)
        c.h0[i] = frac_bits(nth_prime(i), 2);
    return c;
}

constexpr ShaConsts kSha = make_consts();
static_assert(nth_prime(63) == 311, "the 64th prime");

// ---- Round functions -------------------------------------------------------

__device__ __forceinline__ uint32_t rotr(uint32_t x, int n) { return __builtin_amdgcn_alignbit(x, x, n); }

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Ch(x,y,z) = x ? y : z per bit; Maj = majority (bitop3 truth tables indexed
// by x<<2 | y<<1 | z).
__device__ __forceinline__ uint32_t ch(uint32_t x, uint32_t y, uint32_t z)
{
    return __builtin_amdgcn_bitop3_b32(x, y, z, 0xCA);
}

__device__ __forceinline__ uint32_t maj(uint32_t x, uint32_t y, uint32_t z)
{
    return __builtin_amdgcn_bitop3_b32(x, y, z, 0xE8);
}

__device__ __forceinline__ uint32_t bsig0(uint32_t x) { return xor3(rotr(x, 2), rotr(x, 13), rotr(x, 22)); }
__device__ __forceinline__ uint32_t bsig1(uint32_t x) { return xor3(rotr(x, 6), rotr(x, 11), rotr(x, 25)); }
__device__ __forceinline__ uint32_t ssig0(uint32_t x) { return xor3(rotr(x, 7), rotr(x, 18), x >> 3); }
__device__ __forceinline__ uint32_t ssig1(uint32_t x) { return xor3(rotr(x, 17), rotr(x, 19), x >> 10); }

__device__ __forceinline__ uint32_t add3(uint32_t a, uint32_t b, uint32_t c) { return a + b + c; }

__device__ __forceinline__ uint32_t bswap(uint32_t x) { return __builtin_amdgcn_perm(x, x, 0x00010203u); }

// One 512-bit block: w[0..15] are the block's big-endian words.
__device__ __forceinline__ void compress(uint32_t H[8], uint32_t w[16])
{
    uint32_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7];
#pragma unroll
    for (int t = 0; t < 64; ++t) {
        if (t >= 16) {
            // W_t = s1(W_{t-2}) + W_{t-7} + s0(W_{t-15}) + W_{t-16}, rolling in place.
            w[t & 15] = add3(ssig1(w[(t - 2) & 15]), w[(t - 7) & 15], ssig0(w[(t - 15) & 15])) + w[t & 15];
        }
        const uint32_t t1 = add3(h, bsig1(e), ch(e, f, g)) + (kSha.k[t] + w[t & 15]);
        const uint32_t t2 = bsig0(a) + maj(a, b, c);
        h = g;
        g = f;
        f = e;
        e = d + t1;
        d = c;
        c = b;
        b = a;
        a = t1 + t2;
    }
    H[0] += a;
    H[1] += b;
    H[2] += c;
    H[3] += d;
    H[4] += e;
    H[5] += f;
    H[6] += g;
    H[7] += h;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Global-address-space views, so loads and stores are global_* rather than flat_*.
typedef const __attribute__((address_space(1))) u32x4 g_cu32x4;
typedef __attribute__((address_space(1))) u32x4 g_u32x4;
typedef const __attribute__((address_space(1))) uint8_t g_cu8;
typedef __attribute__((address_space(1))) uint8_t g_u8;

// Sixteen big-endian words of a full block at p.
template <bool ALIGNED16>
__device__ __forceinline__ void load_block(g_cu8 *p, uint32_t w[16])
{
    if constexpr (ALIGNED16) {
        g_cu32x4 *q = reinterpret_cast<g_cu32x4 *>(p);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const u32x4 v = __builtin_nontemporal_load(q + i);
            w[4 * i] = bswap(v[0]);
            w[4 * i + 1] = bswap(v[1]);
            w[4 * i + 2] = bswap(v[2]);
            w[4 * i + 3] = bswap(v[3]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            w[i] = uint32_t(p[4 * i]) << 24 | uint32_t(p[4 * i + 1]) << 16 | uint32_t(p[4 * i + 2]) << 8 |
                   uint32_t(p[4 * i + 3]);
    }
}

// The last one or two blocks: the rest (< 64 bytes) of the message, the 0x80
// byte, zeros and the 64-bit big-endian bit length (Sec. 5.1.1).
__device__ __forceinline__ void finish(uint32_t H[8], g_cu8 *p, uint32_t rest, uint64_t len)
{
    uint32_t w[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        uint32_t v = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t pos = 4 * i + j;
            const uint32_t byte = pos < rest ? uint32_t(p[pos]) : pos == rest ? 0x80u : 0u;
            v |= byte << (24 - 8 * j);
        }
        w[i] = v;
    }
    const uint64_t bits = len << 3;
    if (rest < 56) {
        w[14] = static_cast<uint32_t>(bits >> 32);
        w[15] = static_cast<uint32_t>(bits);
        compress(H, w);
    } else {
        compress(H, w);
#pragma unroll
        for (int i = 0; i < 14; ++i) w[i] = 0;
        w[14] = static_cast<uint32_t>(bits >> 32);
        w[15] = static_cast<uint32_t>(bits);
        compress(H, w);
    }
}

__global__ __launch_bounds__(256) void sha256_batch_kernel(const ShaRecord *__restrict__ recs, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const ShaRecord r = recs[i];
        g_cu8 *p = reinterpret_cast<g_cu8 *>(static_cast<uintptr_t>(r.in));
        uint32_t H[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) H[j] = kSha.h0[j];
        const uint64_t full = r.len >> 6;
        uint32_t w[16];
        if ((r.in & 15) == 0) {
            // The next block's loads are in flight while this one compresses.
            if (full > 0) {
                load_block<true>(p, w);
                for (uint64_t blk = 1; blk < full; ++blk) {
                    uint32_t nx[16];
                    load_block<true>(p + 64 * blk, nx);
                    compress(H, w);
#pragma unroll
                    for (int j = 0; j < 16; ++j) w[j] = nx[j];
                }
                compress(H, w);
            }
        } else {
            for (uint64_t blk = 0; blk < full; ++blk) {
                load_block<false>(p + 64 * blk, w);
                compress(H, w);
            }
        }
        finish(H, p + 64 * full, static_cast<uint32_t>(r.len & 63), r.len);
        g_u8 *out = reinterpret_cast<g_u8 *>(static_cast<uintptr_t>(r.digest));
        if ((r.digest & 15) == 0) {
            g_u32x4 *o = reinterpret_cast<g_u32x4 *>(out);
            o[0] = u32x4{bswap(H[0]), bswap(H[1]), bswap(H[2]), bswap(H[3])};
            o[1] = u32x4{bswap(H[4]), bswap(H[5]), bswap(H[6]), bswap(H[7])};
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                out[4 * j] = static_cast<uint8_t>(H[j] >> 24);
                out[4 * j + 1] = static_cast<uint8_t>(H[j] >> 16);
                out[4 * j + 2] = static_cast<uint8_t>(H[j] >> 8);
                out[4 * j + 3] = static_cast<uint8_t>(H[j]);
            }
        }
    }
}

}  // namespace

int launch_sha256_batch(const ShaRecord *dev_recs, uint32_t n, int grid, hipStream_t st)
{
    if (grid <= 0 || n == 0)
        return AES_EINVAL;
    (void)hipGetLastError();   // not ours: left by earlier calls
    hipLaunchKernelGGL(sha256_batch_kernel, dim3(grid), dim3(256), 0, st, dev_recs, n);
    return launch_status();
}

}  // namespace aesctr
