/*
 * sharef.h -- CPU oracle for SHA-256 (TEST INFRASTRUCTURE ONLY).
 *
 * Plain C written from FIPS 180-4: the logical functions (Sec. 4.1.2), the
 * constants (Sec. 4.2.2 and the initial hash value of Sec. 5.3.3, both
 * computed here from their definitions as fractional parts of cube and
 * square roots of the first primes), padding (Sec. 5.1.1), parsing
 * (Sec. 5.2.1) and the hash computation (Sec. 6.2.2).  Only tests/, the
 * smoke check and the benchmark's CPU baseline use it; the product library
 * shares no code with it.
 */
#ifndef SHAREF_H
#define SHAREF_H

#include <stddef.h>
#include <stdint.h>

/* The first n primes (n <= 64). */
void sharef_primes(int n, uint32_t *out);

/* K_0..K_63: first 32 bits of the fractional parts of the cube roots of the
 * first 64 primes (Sec. 4.2.2). */
void sharef_k(uint32_t k[64]);

/* H(0): first 32 bits of the fractional parts of the square roots of the
 * first 8 primes (Sec. 5.3.3). */
void sharef_h0(uint32_t h[8]);

/* Digest of msg[0..len) (Sec. 6.2), 32 bytes. */
void sharef_sha256(const uint8_t *msg, uint64_t len, uint8_t digest[32]);

/* n messages of equal length len, back to back in msgs; digests back to
 * back in out.  threads <= 0: one thread.  Returns the threads used. */
int sharef_sha256_many(const uint8_t *msgs, uint64_t len, uint64_t n, uint8_t *out, int threads);

#endif /* SHAREF_H */
