// aes_tables.h -- compile-time AES tables for the GPU library.
//
// The S-box of FIPS-197 Sec. 5.1.1 is the affine map of the multiplicative
// inverse in GF(2^8) (m(x) = x^8 + x^4 + x^3 + x + 1, Sec. 4.2).  Here the
// inverse comes from discrete logarithms: {03} generates the multiplicative
// group, so with exp[i] = {03}^i and log[exp[i]] = i, a^-1 = exp[255 - log a].
// The affine map is applied in its rotation form
//   s = b ^ rotl(b,1) ^ rotl(b,2) ^ rotl(b,3) ^ rotl(b,4) ^ {63}.
//
// The round T-table folds SubBytes and MixColumns (Sec. 5.1.1, 5.1.3) for one
// state byte.  A column is held as a little-endian 32-bit word whose byte r is
// row r.  MixColumns multiplies by the circulant matrix with first row
// {02} {03} {01} {01}, so a byte in row 0 contributes {02}S to row 0, S to
// rows 1 and 2, and {03}S to row 3:
//   T0[x] = {02}S(x) | S(x) << 8 | S(x) << 16 | {03}S(x) << 24
// and the byte of row r uses Tr[x] = rotl(T0[x], 8r).
#pragma once

#include <stdint.h>

namespace aesctr {

struct Tables {
    uint8_t sbox[256];
    uint32_t t0[256];
};

constexpr uint8_t gf_double(uint8_t b)
{
    return static_cast<uint8_t>((b << 1) ^ ((b & 0x80) ? 0x1b : 0x00));
}

constexpr uint8_t rotl8c(uint8_t b, int n)
{
    return static_cast<uint8_t>((b << n) | (b >> (8 - n)));
}

constexpr Tables build_tables()
{
    Tables t{};
    uint8_t exp_t[256]{};
    uint8_t log_t[256]{};
    uint8_t x = 1;
    for (int i = 0; i < 255; ++i) {
        exp_t[i] = x;
        log_t[x] = static_cast<uint8_t>(i);
        x = static_cast<uint8_t>(x ^ gf_double(x));     // x * {03}
    }
    for (int a = 0; a < 256; ++a) {
        uint8_t inv = a == 0 ? 0 : exp_t[(255 - log_t[a]) % 255];
        uint8_t s = static_cast<uint8_t>(inv ^ rotl8c(inv, 1) ^ rotl8c(inv, 2) ^
                                         rotl8c(inv, 3) ^ rotl8c(inv, 4) ^ 0x63);
        t.sbox[a] = s;
    }
    for (int a = 0; a < 256; ++a) {
        uint8_t s = t.sbox[a];
        uint8_t s2 = gf_double(s);
        uint8_t s3 = static_cast<uint8_t>(s2 ^ s);
        t.t0[a] = static_cast<uint32_t>(s2) | static_cast<uint32_t>(s) << 8 |
                  static_cast<uint32_t>(s) << 16 | static_cast<uint32_t>(s3) << 24;
    }
    return t;
}

inline constexpr Tables kTables = build_tables();

constexpr uint32_t rotl32(uint32_t v, int n)
{
    return n == 0 ? v : (v << n) | (v >> (32 - n));
}

constexpr uint32_t bswap32(uint32_t v)
{
    return (v >> 24) | ((v >> 8) & 0xff00u) | ((v << 8) & 0xff0000u) | (v << 24);
}

// Round table r (0..3) at index x.
constexpr uint32_t tr(int r, uint8_t x) { return rotl32(kTables.t0[x], 8 * r); }

}  // namespace aesctr
