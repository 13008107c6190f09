/*
 * sharef.c -- CPU oracle for SHA-256 (TEST INFRASTRUCTURE ONLY).
 * Written from FIPS 180-4; see sharef.h for the sections followed.
 */
#include "sharef.h"

#include <pthread.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---- Constants from their definitions (Sec. 4.2.2, Sec. 5.3.3) -------- */

void sharef_primes(int n, uint32_t *out)
{
    int found = 0;
    for (uint32_t c = 2; found < n; ++c) {
        int prime = 1;
        for (uint32_t d = 2; d * d <= c; ++d)
            if (c % d == 0) {
                prime = 0;
                break;
            }
        if (prime)
            out[found++] = c;
    }
}

/* Largest y with y^e <= x (e = 2 or 3), by bisection on exact integers. */
static uint64_t iroot(u128 x, int e)
{
    uint64_t lo = 0, hi = (uint64_t)1 << 40;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        u128 p = (u128)mid * mid;
        if (e == 3)
            p *= mid;
        if (p <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

/* floor(root_e(p) * 2^32) mod 2^32: the first 32 bits of the fractional part
 * of the e-th root of p, i.e. the e-th root of p * 2^(32e), truncated. */
static uint32_t frac_root_bits(uint32_t p, int e)
{
    const u128 x = (u128)p << (32 * e);
    return (uint32_t)iroot(x, e);
}

void sharef_k(uint32_t k[64])
{
    uint32_t p[64];
    sharef_primes(64, p);
    for (int i = 0; i < 64; ++i)
        k[i] = frac_root_bits(p[i], 3);
}

void sharef_h0(uint32_t h[8])
{
    uint32_t p[8];
    sharef_primes(8, p);
    for (int i = 0; i < 8; ++i)
        h[i] = frac_root_bits(p[i], 2);
}

/* ---- Functions (Sec. 3.2, 4.1.2) -------------------------------------- */

static uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }
static uint32_t ch(uint32_t x, uint32_t y, uint32_t z) { return (x & y) ^ (~x & z); }
static uint32_t maj(uint32_t x, uint32_t y, uint32_t z) { return (x & y) ^ (x & z) ^ (y & z); }
static uint32_t big_sigma0(uint32_t x) { return rotr(x, 2) ^ rotr(x, 13) ^ rotr(x, 22); }
static uint32_t big_sigma1(uint32_t x) { return rotr(x, 6) ^ rotr(x, 11) ^ rotr(x, 25); }
static uint32_t small_sigma0(uint32_t x) { return rotr(x, 7) ^ rotr(x, 18) ^ (x >> 3); }
static uint32_t small_sigma1(uint32_t x) { return rotr(x, 17) ^ rotr(x, 19) ^ (x >> 10); }

/* ---- Hash computation (Sec. 6.2.2) ------------------------------------ */

static void compress(uint32_t H[8], const uint8_t block[64], const uint32_t K[64])
{
    uint32_t W[64];
    /* 1. message schedule; words are big-endian (Sec. 3.1, 5.2.1) */
    for (int t = 0; t < 16; ++t)
        W[t] = (uint32_t)block[4 * t] << 24 | (uint32_t)block[4 * t + 1] << 16 |
               (uint32_t)block[4 * t + 2] << 8 | (uint32_t)block[4 * t + 3];
    for (int t = 16; t < 64; ++t)
        W[t] = small_sigma1(W[t - 2]) + W[t - 7] + small_sigma0(W[t - 15]) + W[t - 16];
    /* 2. working variables */
    uint32_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7];
    /* 3. 64 rounds */
    for (int t = 0; t < 64; ++t) {
        const uint32_t T1 = h + big_sigma1(e) + ch(e, f, g) + K[t] + W[t];
        const uint32_t T2 = big_sigma0(a) + maj(a, b, c);
        h = g;
        g = f;
        f = e;
        e = d + T1;
        d = c;
        c = b;
        b = a;
        a = T1 + T2;
    }
    /* 4. intermediate hash value */
    H[0] += a;
    H[1] += b;
    H[2] += c;
    H[3] += d;
    H[4] += e;
    H[5] += f;
    H[6] += g;
    H[7] += h;
}

void sharef_sha256(const uint8_t *msg, uint64_t len, uint8_t digest[32])
{
    uint32_t K[64], H[8];
    sharef_k(K);
    sharef_h0(H);
    uint64_t off = 0;
    for (; off + 64 <= len; off += 64)
        compress(H, msg + off, K);
    /* Padding (Sec. 5.1.1): the rest, a 1 bit, zeros, then the length in
     * bits as a 64-bit big-endian integer, to a multiple of 512 bits. */
    uint8_t tail[128];
    memset(tail, 0, sizeof(tail));
    const uint64_t rest = len - off;
    memcpy(tail, msg + off, rest);
    tail[rest] = 0x80;
    const uint64_t tail_len = rest + 1 + 8 <= 64 ? 64 : 128;
    const uint64_t bits = len * 8;
    for (int i = 0; i < 8; ++i)
        tail[tail_len - 1 - i] = (uint8_t)(bits >> (8 * i));
    for (uint64_t o = 0; o < tail_len; o += 64)
        compress(H, tail + o, K);
    for (int i = 0; i < 8; ++i) {
        digest[4 * i] = (uint8_t)(H[i] >> 24);
        digest[4 * i + 1] = (uint8_t)(H[i] >> 16);
        digest[4 * i + 2] = (uint8_t)(H[i] >> 8);
        digest[4 * i + 3] = (uint8_t)H[i];
    }
}

/* ---- Many messages, threaded (timing driver only) --------------------- */

struct job {
    const uint8_t *msgs;
    uint64_t len, first, count;
    uint8_t *out;
};

static void *worker(void *arg)
{
    struct job *j = (struct job *)arg;
    for (uint64_t i = j->first; i < j->first + j->count; ++i)
        sharef_sha256(j->msgs + i * j->len, j->len, j->out + 32 * i);
    return NULL;
}

int sharef_sha256_many(const uint8_t *msgs, uint64_t len, uint64_t n, uint8_t *out, int threads)
{
    if (threads <= 1 || n < 2) {
        struct job j = {msgs, len, 0, n, out};
        worker(&j);
        return 1;
    }
    if ((uint64_t)threads > n)
        threads = (int)n;
    if (threads > 256)
        threads = 256;
    pthread_t tid[256];
    struct job jobs[256];
    const uint64_t per = n / (uint64_t)threads, extra = n % (uint64_t)threads;
    uint64_t first = 0;
    for (int t = 0; t < threads; ++t) {
        const uint64_t count = per + ((uint64_t)t < extra ? 1 : 0);
        jobs[t] = (struct job){msgs, len, first, count, out};
        first += count;
        pthread_create(&tid[t], NULL, worker, &jobs[t]);
    }
    for (int t = 0; t < threads; ++t)
        pthread_join(tid[t], NULL);
    return threads;
}
