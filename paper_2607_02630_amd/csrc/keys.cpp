// keys.cpp -- host-side key schedule and per-request key material.
#include <string.h>

#include "aes_tables.h"
#include "aesctr_internal.h"

namespace aesctr {

namespace {

uint32_t sub_word(uint32_t w)
{
    return static_cast<uint32_t>(kTables.sbox[w >> 24]) << 24 |
           static_cast<uint32_t>(kTables.sbox[(w >> 16) & 0xff]) << 16 |
           static_cast<uint32_t>(kTables.sbox[(w >> 8) & 0xff]) << 8 |
           static_cast<uint32_t>(kTables.sbox[w & 0xff]);
}

uint32_t le_word(const uint8_t *p)
{
    return static_cast<uint32_t>(p[0]) | static_cast<uint32_t>(p[1]) << 8 |
           static_cast<uint32_t>(p[2]) << 16 | static_cast<uint32_t>(p[3]) << 24;
}

uint8_t byte_of(uint32_t w, int r) { return static_cast<uint8_t>(w >> (8 * r)); }

}  // namespace

void make_key_material(const aes_sched_t &s, const uint8_t nonce[12], KeyMaterial *km)
{
    const int nwords = 4 * (s.nr + 1);
    memset(km, 0, sizeof(*km));
    for (int i = 0; i < nwords; ++i)
        km->rk[i] = bswap32(s.rk[i]);
    km->nr = s.nr;
    // Round-0 state: columns 0..2 are the nonce, column 3 the counter.
    uint32_t st[3];
    for (int c = 0; c < 3; ++c)
        st[c] = le_word(nonce + 4 * c) ^ km->rk[c];
    km->x0 = km->rk[3];
    // Round-1 column c = XOR_r T_r[row r of column (c + r) mod 4] ^ rk1_c; the
    // term whose column is 3 stays on the device.
    for (int c = 0; c < 4; ++c) {
        uint32_t acc = km->rk[4 + c];
        for (int r = 0; r < 4; ++r) {
            int col = (c + r) & 3;
            if (col == 3)
                continue;
            acc ^= tr(r, byte_of(st[col], r));
        }
        km->k1[c] = acc;
    }
}

}  // namespace aesctr

extern "C" int aes_expand_key(const uint8_t *key, int key_bits, aes_sched_t *out)
{
    using namespace aesctr;
    if (!key || !out)
        return AES_EINVAL;
    int nk;
    if (key_bits == 128)
        nk = 4;
    else if (key_bits == 256)
        nk = 8;
    else
        return AES_EINVAL;
    const int nr = nk + 6;
    const int total = 4 * (nr + 1);
    memset(out, 0, sizeof(*out));
    for (int i = 0; i < nk; ++i)
        out->rk[i] = static_cast<uint32_t>(key[4 * i]) << 24 | static_cast<uint32_t>(key[4 * i + 1]) << 16 |
                     static_cast<uint32_t>(key[4 * i + 2]) << 8 | static_cast<uint32_t>(key[4 * i + 3]);
    uint8_t rcon = 0x01;
    for (int i = nk; i < total; ++i) {
        uint32_t t = out->rk[i - 1];
        if (i % nk == 0) {
            t = sub_word((t << 8) | (t >> 24)) ^ (static_cast<uint32_t>(rcon) << 24);
            rcon = gf_double(rcon);
        } else if (nk == 8 && i % nk == 4) {
            t = sub_word(t);
        }
        out->rk[i] = out->rk[i - nk] ^ t;
    }
    out->nr = nr;
    out->key_bits = key_bits;
    return AES_OK;
}
