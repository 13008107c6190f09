/*
 * aesref.c -- CPU oracle for AES-CTR.  TEST INFRASTRUCTURE ONLY: the tests,
 * the smoke check and the benchmark's CPU-baseline leg load it; the product
 * library never does.
 *
 * Written from the FIPS-197 definitions, in the standard's own order and
 * notation: the state is a 4x4 byte array s[r][c] filled column by column
 * (s[r][c] = in[r + 4c]); each round is SubBytes, ShiftRows, MixColumns
 * (skipped in the last round) and AddRoundKey.  No lookup table is typed in:
 * the S-box is built at first use from the field inverse and the affine map
 * (Sec. 5.1.1).  No compiler intrinsics, no AES-NI (built with -mno-aes).
 *
 * Counter mode follows NIST SP 800-38A Sec. 6.5 with counter blocks
 * nonce(12 bytes) || BE32((ctr0 + j) mod 2^32).
 */
#include "aesref.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ---------------------------------------------------------------------- */
/* FIPS-197 Sec. 4: the field GF(2^8) modulo m(x) = x^8+x^4+x^3+x+1.      */
/* ---------------------------------------------------------------------- */

/* Sec. 4.2.1: multiplication by x is a left shift, reduced by m(x) (the
 * byte {1b}) when the shifted-out bit b7 was set. */
uint8_t aesref_xtime(uint8_t b)
{
    uint8_t shifted = (uint8_t)(b << 1);
    return (b & 0x80) ? (uint8_t)(shifted ^ 0x1b) : shifted;
}

/* Sec. 4.2: product of a and b as the sum (XOR) of b * x^i over the set bits
 * a_i of a, the powers of x obtained by repeated xtime. */
uint8_t aesref_gf_mul(uint8_t a, uint8_t b)
{
    uint8_t acc = 0;
    uint8_t term = b;            /* b * x^i */
    for (int i = 0; i < 8; i++) {
        if (a & (1u << i))
            acc ^= term;
        term = aesref_xtime(term);
    }
    return acc;
}

/* Sec. 4.2: the multiplicative inverse.  The nonzero elements form a group
 * of order 255, so a^-1 = a^254; computed by plain repeated multiplication.
 * The element 0 maps to itself (Sec. 5.1.1). */
uint8_t aesref_gf_inv(uint8_t a)
{
    if (a == 0)
        return 0;
    uint8_t r = 1;
    for (int i = 0; i < 254; i++)
        r = aesref_gf_mul(r, a);
    return r;
}

/* ---------------------------------------------------------------------- */
/* Sec. 5.1.1: the S-box = affine transformation of the field inverse.     */
/* ---------------------------------------------------------------------- */

static uint8_t g_sbox[256];
static uint8_t g_inv_sbox[256];
static pthread_once_t g_tables_once = PTHREAD_ONCE_INIT;

static int bit_of(uint8_t v, int i) { return (v >> (i & 7)) & 1; }

/* b'_i = b_i ^ b_(i+4 mod 8) ^ b_(i+5 mod 8) ^ b_(i+6 mod 8) ^ b_(i+7 mod 8) ^ c_i
 * with c = {63}, applied to b = x^-1. */
static uint8_t sbox_entry(uint8_t x)
{
    const uint8_t c = 0x63;
    uint8_t b = aesref_gf_inv(x);
    uint8_t out = 0;
    for (int i = 0; i < 8; i++) {
        int v = bit_of(b, i) ^ bit_of(b, i + 4) ^ bit_of(b, i + 5) ^ bit_of(b, i + 6) ^
                bit_of(b, i + 7) ^ bit_of(c, i);
        out |= (uint8_t)(v << i);
    }
    return out;
}

static void build_tables(void)
{
    for (int x = 0; x < 256; x++)
        g_sbox[x] = sbox_entry((uint8_t)x);
    /* InvSubBytes (Sec. 5.3.2) uses the inverse permutation. */
    for (int x = 0; x < 256; x++)
        g_inv_sbox[g_sbox[x]] = (uint8_t)x;
}

static void ensure_tables(void) { pthread_once(&g_tables_once, build_tables); }

void aesref_sbox(uint8_t out[256])
{
    ensure_tables();
    memcpy(out, g_sbox, 256);
}

void aesref_inv_sbox(uint8_t out[256])
{
    ensure_tables();
    memcpy(out, g_inv_sbox, 256);
}

/* Sec. 5.2: Rcon[i] = [x^(i-1), {00}, {00}, {00}], the powers of x = {02}. */
uint8_t aesref_rcon(int i)
{
    uint8_t p = 0x01;
    for (int k = 1; k < i; k++)
        p = aesref_xtime(p);
    return p;
}

/* ---------------------------------------------------------------------- */
/* Round transformations (Sec. 5.1.1 - 5.1.4 and 5.3).                     */
/* ---------------------------------------------------------------------- */

typedef uint8_t state_t[4][4];   /* s[r][c] */

static void sub_bytes(state_t s)
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = g_sbox[s[r][c]];
}

static void inv_sub_bytes(state_t s)
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = g_inv_sbox[s[r][c]];
}

/* Sec. 5.1.2: row r is rotated left by shift(r, 4) = r positions:
 * s'[r][c] = s[r][(c + r) mod 4]. */
static void shift_rows(state_t s)
{
    for (int r = 1; r < 4; r++) {
        uint8_t row[4];
        for (int c = 0; c < 4; c++)
            row[c] = s[r][(c + r) % 4];
        for (int c = 0; c < 4; c++)
            s[r][c] = row[c];
    }
}

/* Sec. 5.3.1: the inverse rotates row r right by r: s'[r][(c + r) mod 4] = s[r][c]. */
static void inv_shift_rows(state_t s)
{
    for (int r = 1; r < 4; r++) {
        uint8_t row[4];
        for (int c = 0; c < 4; c++)
            row[(c + r) % 4] = s[r][c];
        for (int c = 0; c < 4; c++)
            s[r][c] = row[c];
    }
}

/* Sec. 5.1.3: a column, as a polynomial over GF(2^8), times
 * a(x) = {03}x^3 + {01}x^2 + {01}x + {02} modulo x^4 + 1.  Written as the
 * matrix product whose row r is the coefficient vector rotated: out_r =
 * sum_k coef[(k - r) mod 4] * in_k with coef = {02},{03},{01},{01}. */
static void poly_mul_column(uint8_t col[4], const uint8_t coef[4])
{
    uint8_t in[4];
    memcpy(in, col, 4);
    for (int r = 0; r < 4; r++) {
        uint8_t acc = 0;
        for (int k = 0; k < 4; k++)
            acc ^= aesref_gf_mul(coef[(k - r + 4) % 4], in[k]);
        col[r] = acc;
    }
}

void aesref_mix_column(uint8_t col[4])
{
    static const uint8_t a[4] = {0x02, 0x03, 0x01, 0x01};
    poly_mul_column(col, a);
}

/* Sec. 5.3.3: a^-1(x) = {0b}x^3 + {0d}x^2 + {09}x + {0e}. */
void aesref_inv_mix_column(uint8_t col[4])
{
    static const uint8_t ainv[4] = {0x0e, 0x0b, 0x0d, 0x09};
    poly_mul_column(col, ainv);
}

static void mix_columns(state_t s)
{
    for (int c = 0; c < 4; c++) {
        uint8_t col[4] = {s[0][c], s[1][c], s[2][c], s[3][c]};
        aesref_mix_column(col);
        for (int r = 0; r < 4; r++)
            s[r][c] = col[r];
    }
}

static void inv_mix_columns(state_t s)
{
    for (int c = 0; c < 4; c++) {
        uint8_t col[4] = {s[0][c], s[1][c], s[2][c], s[3][c]};
        aesref_inv_mix_column(col);
        for (int r = 0; r < 4; r++)
            s[r][c] = col[r];
    }
}

/* Sec. 5.1.4: column c is XORed with the schedule word w[round*Nb + c];
 * byte r of the column takes byte r (most significant first) of the word. */
static void add_round_key(state_t s, const uint32_t *w, int round)
{
    for (int c = 0; c < 4; c++) {
        uint32_t word = w[round * 4 + c];
        for (int r = 0; r < 4; r++)
            s[r][c] ^= (uint8_t)(word >> (24 - 8 * r));
    }
}

/* ---------------------------------------------------------------------- */
/* Sec. 5.2: KeyExpansion.                                                 */
/* ---------------------------------------------------------------------- */

static uint32_t sub_word(uint32_t x)
{
    uint32_t out = 0;
    for (int k = 0; k < 4; k++)
        out |= (uint32_t)g_sbox[(x >> (8 * k)) & 0xff] << (8 * k);
    return out;
}

/* [a0,a1,a2,a3] -> [a1,a2,a3,a0], a0 being the most significant byte. */
static uint32_t rot_word(uint32_t x) { return (x << 8) | (x >> 24); }

int aesref_expand(const uint8_t *key, int key_bits, uint32_t *w)
{
    int nk, nr;
    switch (key_bits) {
    case 128: nk = 4; nr = 10; break;
    case 192: nk = 6; nr = 12; break;
    case 256: nk = 8; nr = 14; break;
    default: return -1;
    }
    if (!key || !w)
        return -1;
    ensure_tables();
    int total = 4 * (nr + 1);           /* Nb * (Nr + 1) with Nb = 4 */
    for (int i = 0; i < nk; i++)
        w[i] = (uint32_t)key[4 * i] << 24 | (uint32_t)key[4 * i + 1] << 16 |
               (uint32_t)key[4 * i + 2] << 8 | (uint32_t)key[4 * i + 3];
    for (int i = nk; i < total; i++) {
        uint32_t temp = w[i - 1];
        if (i % nk == 0)
            temp = sub_word(rot_word(temp)) ^ ((uint32_t)aesref_rcon(i / nk) << 24);
        else if (nk > 6 && i % nk == 4)
            temp = sub_word(temp);
        w[i] = w[i - nk] ^ temp;
    }
    return nr;
}

/* ---------------------------------------------------------------------- */
/* Sec. 5.1 Cipher and Sec. 5.3 InvCipher.                                 */
/* ---------------------------------------------------------------------- */

static void load_state(state_t s, const uint8_t in[16])
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = in[r + 4 * c];
}

static void store_state(const state_t s, uint8_t out[16])
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            out[r + 4 * c] = s[r][c];
}

void aesref_encrypt_block(const uint32_t *w, int nr, const uint8_t in[16], uint8_t out[16])
{
    state_t s;
    ensure_tables();
    load_state(s, in);
    add_round_key(s, w, 0);
    for (int round = 1; round < nr; round++) {
        sub_bytes(s);
        shift_rows(s);
        mix_columns(s);
        add_round_key(s, w, round);
    }
    sub_bytes(s);
    shift_rows(s);
    add_round_key(s, w, nr);
    store_state(s, out);
}

void aesref_decrypt_block(const uint32_t *w, int nr, const uint8_t in[16], uint8_t out[16])
{
    state_t s;
    ensure_tables();
    load_state(s, in);
    add_round_key(s, w, nr);
    for (int round = nr - 1; round >= 1; round--) {
        inv_shift_rows(s);
        inv_sub_bytes(s);
        add_round_key(s, w, round);
        inv_mix_columns(s);
    }
    inv_shift_rows(s);
    inv_sub_bytes(s);
    add_round_key(s, w, 0);
    store_state(s, out);
}

/* ---------------------------------------------------------------------- */
/* SP 800-38A Sec. 6.5: CTR mode.                                          */
/* ---------------------------------------------------------------------- */

void aesref_counter_block(const uint8_t nonce[12], uint32_t ctr0, uint64_t j, uint8_t out[16])
{
    uint32_t ctr = (uint32_t)(ctr0 + (uint32_t)j);   /* mod 2^32 */
    memcpy(out, nonce, 12);
    out[12] = (uint8_t)(ctr >> 24);
    out[13] = (uint8_t)(ctr >> 16);
    out[14] = (uint8_t)(ctr >> 8);
    out[15] = (uint8_t)ctr;
}

/* Blocks [jb, je) of the message: O_j = CIPH_K(T_j); C_j = P_j ^ O_j, the
 * last (possibly partial) block XORed with the leading bytes of O_j. */
static void ctr_range(const uint32_t *w, int nr, const uint8_t nonce[12], uint32_t ctr0,
                      const uint8_t *in, uint8_t *out, uint64_t len, uint64_t jb, uint64_t je)
{
    uint8_t t[16], o[16];
    for (uint64_t j = jb; j < je; j++) {
        aesref_counter_block(nonce, ctr0, j, t);
        aesref_encrypt_block(w, nr, t, o);
        uint64_t off = 16 * j;
        uint64_t n = len - off < 16 ? len - off : 16;
        for (uint64_t b = 0; b < n; b++)
            out[off + b] = in[off + b] ^ o[b];
    }
}

/* More than 2^32 blocks would reuse counter blocks within one message. */
static int ctr_args_ok(const uint8_t *key, const uint8_t *nonce, const uint8_t *in,
                       uint8_t *out, uint64_t len)
{
    if (!key || !nonce)
        return 0;
    if (len > 0 && (!in || !out))
        return 0;
    if (len > ((uint64_t)1 << 32) * 16)
        return 0;
    return 1;
}

int aesref_ctr(const uint8_t *key, int key_bits, const uint8_t nonce[12], uint32_t ctr0,
               const uint8_t *in, uint8_t *out, uint64_t len)
{
    uint32_t w[60];
    if (!ctr_args_ok(key, nonce, in, out, len))
        return -1;
    int nr = aesref_expand(key, key_bits, w);
    if (nr < 0)
        return -1;
    ctr_range(w, nr, nonce, ctr0, in, out, len, 0, (len + 15) / 16);
    return 0;
}

typedef struct {
    const uint32_t *w;
    int nr;
    const uint8_t *nonce;
    uint32_t ctr0;
    const uint8_t *in;
    uint8_t *out;
    uint64_t len, jb, je;
} ctr_job_t;

static void *ctr_worker(void *arg)
{
    ctr_job_t *j = (ctr_job_t *)arg;
    ctr_range(j->w, j->nr, j->nonce, j->ctr0, j->in, j->out, j->len, j->jb, j->je);
    return NULL;
}

int aesref_ctr_mt(const uint8_t *key, int key_bits, const uint8_t nonce[12], uint32_t ctr0,
                  const uint8_t *in, uint8_t *out, uint64_t len, int nthreads)
{
    uint32_t w[60];
    if (!ctr_args_ok(key, nonce, in, out, len))
        return -1;
    int nr = aesref_expand(key, key_bits, w);
    if (nr < 0)
        return -1;
    if (nthreads <= 0) {
        long n = sysconf(_SC_NPROCESSORS_ONLN);
        nthreads = n > 0 ? (int)n : 1;
    }
    uint64_t nblocks = (len + 15) / 16;
    if ((uint64_t)nthreads > nblocks)
        nthreads = nblocks > 0 ? (int)nblocks : 1;
    ctr_job_t *jobs = (ctr_job_t *)calloc((size_t)nthreads, sizeof(ctr_job_t));
    pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return -1;
    }
    for (int t = 0; t < nthreads; t++) {
        jobs[t] = (ctr_job_t){w, nr, nonce, ctr0, in, out, len,
                              nblocks * (uint64_t)t / (uint64_t)nthreads,
                              nblocks * (uint64_t)(t + 1) / (uint64_t)nthreads};
    }
    int started = 0;
    for (int t = 1; t < nthreads; t++) {
        if (pthread_create(&tids[t], NULL, ctr_worker, &jobs[t]) != 0)
            break;
        started = t;
    }
    ctr_worker(&jobs[0]);
    for (int t = 1; t <= started; t++)
        pthread_join(tids[t], NULL);
    /* Any range whose thread failed to start is done here. */
    for (int t = started + 1; t < nthreads; t++)
        ctr_worker(&jobs[t]);
    free(jobs);
    free(tids);
    return nthreads;
}
