/*
 * aesref.h -- CPU oracle for AES-CTR. TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, byte-oriented AES written from the definitions of FIPS-197
 * (the field, the S-box, the round transformations, KeyExpansion, Cipher and
 * InvCipher) with the counter mode of NIST SP 800-38A on top.  It exists to
 * check the GPU library bit for bit; nothing in the product links it.  Only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.
 *
 * Counter block (the reading used throughout): bytes 0..11 are the 96-bit
 * nonce, bytes 12..15 hold a 32-bit counter in big-endian byte order, and the
 * counter for block j is (ctr0 + j) mod 2^32 -- the "inc32" incrementing
 * function of SP 800-38A Appendix B with m = 32; the nonce never changes.
 *
 * Pinned by tests/test_oracle.py (closed forms, exhaustive invariants and an
 * independent AES implementation, OpenSSL's libcrypto, run as a library).
 */
#ifndef AESREF_H
#define AESREF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* --- GF(2^8) with m(x) = x^8 + x^4 + x^3 + x + 1 (FIPS-197 Sec. 4) ------- */
uint8_t aesref_xtime(uint8_t b);                 /* b * {02}, Sec. 4.2.1   */
uint8_t aesref_gf_mul(uint8_t a, uint8_t b);     /* shift-and-xtime product */
uint8_t aesref_gf_inv(uint8_t a);                /* multiplicative inverse; 0 -> 0 */

/* --- S-box (FIPS-197 Sec. 5.1.1), computed, never typed in -------------- */
void aesref_sbox(uint8_t out[256]);
void aesref_inv_sbox(uint8_t out[256]);

/* Rcon[i] = (x^(i-1), 0, 0, 0); returns the leading byte x^(i-1), i >= 1. */
uint8_t aesref_rcon(int i);

/* MixColumns / InvMixColumns on one 4-byte column (Sec. 5.1.3, 5.3.3). */
void aesref_mix_column(uint8_t col[4]);
void aesref_inv_mix_column(uint8_t col[4]);

/* KeyExpansion (Sec. 5.2).  key_bits in {128, 192, 256}.  Writes 4*(Nr+1)
 * words w[i], each packed big-endian from four key-schedule bytes
 * (w = b0<<24 | b1<<16 | b2<<8 | b3).  Returns Nr, or -1 for bad key_bits. */
int aesref_expand(const uint8_t *key, int key_bits, uint32_t *w);

/* Cipher (Sec. 5.1) and InvCipher (Sec. 5.3) on one 16-byte block. */
void aesref_encrypt_block(const uint32_t *w, int nr, const uint8_t in[16], uint8_t out[16]);
void aesref_decrypt_block(const uint32_t *w, int nr, const uint8_t in[16], uint8_t out[16]);

/* Counter block T_j = nonce || BE32((ctr0 + j) mod 2^32). */
void aesref_counter_block(const uint8_t nonce[12], uint32_t ctr0, uint64_t j, uint8_t out[16]);

/* CTR encryption = decryption (SP 800-38A Sec. 6.5).  Output length equals
 * input length; the final partial block uses the leading bytes of its
 * keystream block.  in == out is allowed.  Returns 0, or -1 on bad args. */
int aesref_ctr(const uint8_t *key, int key_bits, const uint8_t nonce[12], uint32_t ctr0,
               const uint8_t *in, uint8_t *out, uint64_t len);

/* Same result, block range split into contiguous per-thread pieces.
 * nthreads <= 0 means one thread per online CPU.  Returns the thread count
 * used, or -1 on bad args.  Only the timing driver uses this. */
int aesref_ctr_mt(const uint8_t *key, int key_bits, const uint8_t nonce[12], uint32_t ctr0,
                  const uint8_t *in, uint8_t *out, uint64_t len, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
