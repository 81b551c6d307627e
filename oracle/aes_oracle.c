/*
 * aes_oracle.c -- plain, slow, obviously-correct CPU AES.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity oracle for the GPU
 * library.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, tables or headers with
 * the GPU path: every S-box entry is obtained by a GF(2^8) inversion followed
 * by an affine map over GF(2), and every MixColumns is a 4x4 matrix product
 * over GF(2^8) done with the shift-and-add multiply below.  Nothing here is
 * blocked, fused or table-driven beyond the 256-entry S-box itself.
 *
 * Paper: Kepner et al., "Parallel Vectorized Algebraic AES in MATLAB ...",
 * arXiv 1506.08503.  Citations below name the section / appendix.
 *
 * State convention (implied by the ShiftRows index vectors of App. A1/A4):
 * input byte k sits at row k mod 4, column k div 4 of the 4x4 state.
 *
 * Readings where the paper is silent (all in the design notes):
 *  - AES-192/256 key schedule (Nk = 6, 8) follows FIPS-197 sec. 5.2; the paper
 *    only treats 128-bit keys (sec. II).
 *  - CTR mode is not in the paper.  Counter block i is
 *    nonce[0..11] || big-endian 32-bit (ctr0 + i); the caller must keep
 *    ctr0 + nblocks <= 2^32 (no silent wrap).
 *  - The saturating uint8 "+1" in the App. A3 S-box index is read as the
 *    standard S-box lookup (no saturation).
 *
 * Parity pins: every function here is pinned by tests that do not re-type
 * its formula: the paper's printed GF examples, brute-force field
 * identities, S-box / inverse S-box built independently, the paper's
 * ShiftRows index vectors, mix-matrix inverse identity, the FIPS-197 and
 * SP 800-38A example vectors, an independent numpy construction of the
 * paper's vectorized algorithm, and the system OpenSSL command-line tool.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

/* ---------------------------------------------------------------- GF(2^8)
 * Sec. II: a byte is a polynomial over GF(2) whose coefficients are its bits;
 * addition is coefficient-wise, i.e. XOR; products are reduced modulo the AES
 * polynomial x^8 + x^4 + x^3 + x + 1 (0x11B).
 */
#define AES_POLY 0x11Bu

uint8_t oracle_gf_add(uint8_t a, uint8_t b) { return (uint8_t)(a ^ b); }

/* Schoolbook product: for every set bit i of b add a * x^i, where a * x is
 * formed by shifting and, if degree 8 appears, subtracting (XOR) the AES
 * polynomial (sec. II, the reduction modulo 0x11B). */
uint8_t oracle_gf_mul(uint8_t a, uint8_t b)
{
    unsigned acc = 0;
    unsigned term = a;            /* a * x^i, kept reduced */
    for (int i = 0; i < 8; ++i) {
        if (b & (1u << i))
            acc ^= term;
        term <<= 1;
        if (term & 0x100u)
            term ^= AES_POLY;
    }
    return (uint8_t)acc;
}

uint8_t oracle_gf_pow(uint8_t a, unsigned e)
{
    uint8_t result = 1, base = a;
    while (e) {
        if (e & 1u)
            result = oracle_gf_mul(result, base);
        base = oracle_gf_mul(base, base);
        e >>= 1;
    }
    return result;
}

/* Multiplicative inverse: the nonzero elements form a group of order 255,
 * so a^-1 = a^254.  The paper leaves 0 mapped to 0 (App. A2, A5); 0^254 = 0
 * gives exactly that. */
uint8_t oracle_gf_inv(uint8_t a) { return oracle_gf_pow(a, 254u); }

/* --------------------------------------------------------- GF(2) affine map
 * App. A2 / A5: y = A * bits(x) + b over GF(2), where A is the circulant
 * matrix whose first row is given and bits() lists the byte MSB first
 * (dec2bin order).  Circulant: A(i, j) = row[(j - i) mod 8].
 */
static void byte_to_bits_msb_first(uint8_t x, int v[8])
{
    for (int k = 0; k < 8; ++k)
        v[k] = (x >> (7 - k)) & 1;
}

static uint8_t bits_msb_first_to_byte(const int v[8])
{
    uint8_t x = 0;
    for (int k = 0; k < 8; ++k)
        x = (uint8_t)(x | (v[k] << (7 - k)));
    return x;
}

static uint8_t affine_gf2(const int row[8], const int bvec[8], uint8_t x)
{
    int v[8], z[8];
    byte_to_bits_msb_first(x, v);
    for (int i = 0; i < 8; ++i) {
        int s = 0;
        for (int j = 0; j < 8; ++j)
            s ^= row[(j - i + 8) % 8] & v[j];
        z[i] = s ^ bvec[i];
    }
    return bits_msb_first_to_byte(z);
}

/* App. A2: S(x) = A * bits(inv(x)) + b, A = circ[1 1 1 1 1 0 0 0],
 * b = [0 1 1 0 0 0 1 1] (MSB first, i.e. 0x63). */
static const int SBOX_ROW[8] = {1, 1, 1, 1, 1, 0, 0, 0};
static const int SBOX_B[8]   = {0, 1, 1, 0, 0, 0, 1, 1};
/* App. A5: S^-1(y) = inv(A' * bits(y) + b'), A' = circ[0 1 0 1 0 0 1 0],
 * b' = [0 0 0 0 0 1 0 1] (0x05). */
static const int INV_ROW[8]  = {0, 1, 0, 1, 0, 0, 1, 0};
static const int INV_B[8]    = {0, 0, 0, 0, 0, 1, 0, 1};

uint8_t oracle_sbox_entry(uint8_t x)
{
    return affine_gf2(SBOX_ROW, SBOX_B, oracle_gf_inv(x));
}

uint8_t oracle_inv_sbox_entry(uint8_t y)
{
    return oracle_gf_inv(affine_gf2(INV_ROW, INV_B, y));
}

void oracle_sbox(uint8_t out[256])
{
    for (int x = 0; x < 256; ++x)
        out[x] = oracle_sbox_entry((uint8_t)x);
}

void oracle_inv_sbox(uint8_t out[256])
{
    for (int y = 0; y < 256; ++y)
        out[y] = oracle_inv_sbox_entry((uint8_t)y);
}

/* ------------------------------------------------------------ key schedule
 * App. A3 for 128-bit keys: round key r+1 is built from round key r.  Its
 * first word is the last word of key r rotated by one byte, passed through
 * the S-box, plus the round constant x^(r) in its first byte, plus the first
 * word of key r; each following word adds the previous new word to the
 * matching word of key r.
 *
 * Written here in the word-recurrence form that also covers 192- and 256-bit
 * keys (FIPS-197 sec. 5.2; the paper is silent on them):
 *   w[i] = w[i - Nk] + t,  t = SubWord(RotWord(w[i-1])) + Rcon(i / Nk)
 *                             if i mod Nk == 0,
 *                          t = SubWord(w[i-1])  if Nk > 6 and i mod Nk == 4,
 *                          t = w[i-1] otherwise.
 * Words are 4-byte arrays; "+" is GF(2^8) addition bytewise.
 * Returns Nr, or -1 for an unsupported key length.
 */
int oracle_num_rounds(int key_bytes)
{
    if (key_bytes == 16) return 10;
    if (key_bytes == 24) return 12;
    if (key_bytes == 32) return 14;
    return -1;
}

uint8_t oracle_rcon(int j)
{
    /* App. A3: round constant of round j (j >= 1) is x^(j-1) in GF(2^8). */
    return oracle_gf_pow(0x02, (unsigned)(j - 1));
}

int oracle_expand_key(const uint8_t *key, int key_bytes, uint8_t *round_keys)
{
    int nr = oracle_num_rounds(key_bytes);
    if (nr < 0)
        return -1;
    int nk = key_bytes / 4;
    int nwords = 4 * (nr + 1);
    uint8_t sbox[256];
    oracle_sbox(sbox);
    uint8_t w[60][4];
    for (int i = 0; i < nk; ++i)
        for (int b = 0; b < 4; ++b)
            w[i][b] = key[4 * i + b];
    for (int i = nk; i < nwords; ++i) {
        uint8_t t[4];
        memcpy(t, w[i - 1], 4);
        if (i % nk == 0) {
            uint8_t rot[4] = {t[1], t[2], t[3], t[0]};
            for (int b = 0; b < 4; ++b)
                t[b] = sbox[rot[b]];
            t[0] = oracle_gf_add(t[0], oracle_rcon(i / nk));
        } else if (nk > 6 && i % nk == 4) {
            for (int b = 0; b < 4; ++b)
                t[b] = sbox[t[b]];
        }
        for (int b = 0; b < 4; ++b)
            w[i][b] = oracle_gf_add(w[i - nk][b], t[b]);
    }
    for (int i = 0; i < nwords; ++i)
        memcpy(round_keys + 4 * i, w[i], 4);
    return nr;
}

/* ------------------------------------------------------------ round steps
 * The state is st[row][col]; byte k of a block is st[k % 4][k / 4].
 */
typedef uint8_t state_t[4][4];

static void load_state(state_t st, const uint8_t in[16])
{
    for (int k = 0; k < 16; ++k)
        st[k % 4][k / 4] = in[k];
}

static void store_state(uint8_t out[16], state_t st)
{
    for (int k = 0; k < 16; ++k)
        out[k] = st[k % 4][k / 4];
}

/* AddRoundKey (sec. II "add round key"): state + K(r) in GF(2^8). */
static void add_round_key(state_t st, const uint8_t rk[16])
{
    for (int k = 0; k < 16; ++k)
        st[k % 4][k / 4] = oracle_gf_add(st[k % 4][k / 4], rk[k]);
}

/* SubBytes (sec. II "apply s-box"): every byte replaced by its S-box entry. */
static void sub_bytes(state_t st, const uint8_t box[256])
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            st[r][c] = box[st[r][c]];
}

/* ShiftRows (sec. II "shift rows"; index vectors of App. A1): row r of the
 * state is rotated left by r columns. */
static void shift_rows(state_t st)
{
    state_t t;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            t[r][c] = st[r][(c + r) % 4];
    memcpy(st, t, sizeof(state_t));
}

/* Inverse ShiftRows (App. A4): row r rotated right by r columns. */
static void inv_shift_rows(state_t st)
{
    state_t t;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            t[r][(c + r) % 4] = st[r][c];
    memcpy(st, t, sizeof(state_t));
}

/* Multiply every state column by the 4x4 circulant matrix whose first row
 * is given, over GF(2^8): column' = M * column (sec. II "multiply by M";
 * App. A1 uses circ[2 3 1 1], App. A4 uses circ[14 11 13 9]). */
static void mix_columns_with(state_t st, const uint8_t row[4])
{
    uint8_t m[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            m[i][j] = row[(j - i + 4) % 4];
    for (int c = 0; c < 4; ++c) {
        uint8_t col[4];
        for (int i = 0; i < 4; ++i) {
            uint8_t s = 0;
            for (int j = 0; j < 4; ++j)
                s = oracle_gf_add(s, oracle_gf_mul(m[i][j], st[j][c]));
            col[i] = s;
        }
        for (int i = 0; i < 4; ++i)
            st[i][c] = col[i];
    }
}

static const uint8_t MIX_ROW[4]     = {2, 3, 1, 1};
static const uint8_t INV_MIX_ROW[4] = {14, 11, 13, 9};

/* Single-step entry points on one 16-byte block, so the tests can pin each
 * round step on its own (App. A1 / A4 index vectors, mix-matrix inverse). */
void oracle_apply_shift_rows(uint8_t blk[16])
{
    state_t st;
    load_state(st, blk);
    shift_rows(st);
    store_state(blk, st);
}

void oracle_apply_inv_shift_rows(uint8_t blk[16])
{
    state_t st;
    load_state(st, blk);
    inv_shift_rows(st);
    store_state(blk, st);
}

void oracle_apply_mix_columns(uint8_t blk[16])
{
    state_t st;
    load_state(st, blk);
    mix_columns_with(st, MIX_ROW);
    store_state(blk, st);
}

void oracle_apply_inv_mix_columns(uint8_t blk[16])
{
    state_t st;
    load_state(st, blk);
    mix_columns_with(st, INV_MIX_ROW);
    store_state(blk, st);
}

/* ------------------------------------------------------------ block cipher
 * Sec. II / App. A1 without the CBC chaining: add round key 0, then Nr
 * rounds of SubBytes, ShiftRows, MixColumns (skipped in the last round) and
 * AddRoundKey.
 */
static void cipher_block(const uint8_t *rk, int nr, const uint8_t box[256],
                         const uint8_t in[16], uint8_t out[16])
{
    state_t st;
    load_state(st, in);
    add_round_key(st, rk);
    for (int r = 1; r <= nr; ++r) {
        sub_bytes(st, box);
        shift_rows(st);
        if (r < nr)
            mix_columns_with(st, MIX_ROW);
        add_round_key(st, rk + 16 * r);
    }
    store_state(out, st);
}

/* App. A4 without the CBC chaining: for r = Nr down to 1 add round key r,
 * apply the inverse mix matrix (not when r = Nr), inverse ShiftRows and the
 * inverse S-box; finally add round key 0. */
static void inv_cipher_block(const uint8_t *rk, int nr, const uint8_t ibox[256],
                             const uint8_t in[16], uint8_t out[16])
{
    state_t st;
    load_state(st, in);
    for (int r = nr; r >= 1; --r) {
        add_round_key(st, rk + 16 * r);
        if (r < nr)
            mix_columns_with(st, INV_MIX_ROW);
        inv_shift_rows(st);
        sub_bytes(st, ibox);
    }
    add_round_key(st, rk);
    store_state(out, st);
}

int oracle_encrypt_block(const uint8_t *key, int key_bytes,
                         const uint8_t in[16], uint8_t out[16])
{
    uint8_t rk[240], box[256];
    int nr = oracle_expand_key(key, key_bytes, rk);
    if (nr < 0)
        return -1;
    oracle_sbox(box);
    cipher_block(rk, nr, box, in, out);
    return 0;
}

int oracle_decrypt_block(const uint8_t *key, int key_bytes,
                         const uint8_t in[16], uint8_t out[16])
{
    uint8_t rk[240], ibox[256];
    int nr = oracle_expand_key(key, key_bytes, rk);
    if (nr < 0)
        return -1;
    oracle_inv_sbox(ibox);
    inv_cipher_block(rk, nr, ibox, in, out);
    return 0;
}

/* -------------------------------------------------------------------- modes
 * Return codes: 0 ok, -1 bad key length, -2 length not a multiple of 16
 * (ECB / CBC), -3 counter range exceeds 2^32 blocks (CTR).
 */

/* ECB (sec. II): every 16-byte block encrypted on its own. */
int oracle_ecb_encrypt(const uint8_t *key, int key_bytes, const uint8_t *in,
                       uint8_t *out, size_t nbytes)
{
    uint8_t rk[240], box[256];
    int nr = oracle_expand_key(key, key_bytes, rk);
    if (nr < 0)
        return -1;
    if (nbytes % 16)
        return -2;
    oracle_sbox(box);
    for (size_t off = 0; off < nbytes; off += 16)
        cipher_block(rk, nr, box, in + off, out + off);
    return 0;
}

int oracle_ecb_decrypt(const uint8_t *key, int key_bytes, const uint8_t *in,
                       uint8_t *out, size_t nbytes)
{
    uint8_t rk[240], ibox[256];
    int nr = oracle_expand_key(key, key_bytes, rk);
    if (nr < 0)
        return -1;
    if (nbytes % 16)
        return -2;
    oracle_inv_sbox(ibox);
    for (size_t off = 0; off < nbytes; off += 16)
        inv_cipher_block(rk, nr, ibox, in + off, out + off);
    return 0;
}

/* Counter block for block index i: 12 nonce bytes, then ctr0 + i as a
 * big-endian 32-bit integer. */
static void counter_block(const uint8_t nonce[12], uint32_t ctr, uint8_t blk[16])
{
    memcpy(blk, nonce, 12);
    blk[12] = (uint8_t)(ctr >> 24);
    blk[13] = (uint8_t)(ctr >> 16);
    blk[14] = (uint8_t)(ctr >> 8);
    blk[15] = (uint8_t)ctr;
}

/* CTR: out = in + E(counter block i) for every byte of block i; a short last
 * block uses the first (nbytes mod 16) keystream bytes.  The same call
 * decrypts. */
int oracle_ctr_xcrypt(const uint8_t *key, int key_bytes, const uint8_t nonce[12],
                      uint32_t ctr0, const uint8_t *in, uint8_t *out,
                      size_t nbytes)
{
    uint8_t rk[240], box[256];
    int nr = oracle_expand_key(key, key_bytes, rk);
    if (nr < 0)
        return -1;
    uint64_t nblocks = (nbytes + 15) / 16;
    if ((uint64_t)ctr0 + nblocks > (1ull << 32))
        return -3;
    oracle_sbox(box);
    for (uint64_t i = 0; i < nblocks; ++i) {
        uint8_t cb[16], ks[16];
        counter_block(nonce, (uint32_t)(ctr0 + i), cb);
        cipher_block(rk, nr, box, cb, ks);
        size_t off = (size_t)(16 * i);
        size_t len = nbytes - off < 16 ? nbytes - off : 16;
        for (size_t k = 0; k < len; ++k)
            out[off + k] = oracle_gf_add(in[off + k], ks[k]);
    }
    return 0;
}

/* Keystream blocks at arbitrary block indices (CTR allows random access):
 * ks[16*j .. 16*j+15] = E(nonce || BE32(ctr0 + idx[j])).  Used to check a
 * sample of a very large output one block at a time. */
int oracle_ctr_keystream_at(const uint8_t *key, int key_bytes,
                            const uint8_t nonce[12], uint32_t ctr0,
                            const uint64_t *idx, size_t n, uint8_t *ks)
{
    uint8_t rk[240], box[256];
    int nr = oracle_expand_key(key, key_bytes, rk);
    if (nr < 0)
        return -1;
    oracle_sbox(box);
    for (size_t j = 0; j < n; ++j) {
        if ((uint64_t)ctr0 + idx[j] >= (1ull << 32))
            return -3;
        uint8_t cb[16];
        counter_block(nonce, (uint32_t)(ctr0 + idx[j]), cb);
        cipher_block(rk, nr, box, cb, ks + 16 * j);
    }
    return 0;
}

/* CBC, the mode the paper implements (App. A1 / A4): block i is encrypted
 * after adding the previous ciphertext block (the IV for block 0). */
int oracle_cbc_encrypt(const uint8_t *key, int key_bytes, const uint8_t iv[16],
                       const uint8_t *in, uint8_t *out, size_t nbytes)
{
    uint8_t rk[240], box[256];
    int nr = oracle_expand_key(key, key_bytes, rk);
    if (nr < 0)
        return -1;
    if (nbytes % 16)
        return -2;
    oracle_sbox(box);
    uint8_t chain[16];
    memcpy(chain, iv, 16);
    for (size_t off = 0; off < nbytes; off += 16) {
        uint8_t x[16];
        for (int k = 0; k < 16; ++k)
            x[k] = oracle_gf_add(in[off + k], chain[k]);
        cipher_block(rk, nr, box, x, out + off);
        memcpy(chain, out + off, 16);
    }
    return 0;
}

int oracle_cbc_decrypt(const uint8_t *key, int key_bytes, const uint8_t iv[16],
                       const uint8_t *in, uint8_t *out, size_t nbytes)
{
    uint8_t rk[240], ibox[256];
    int nr = oracle_expand_key(key, key_bytes, rk);
    if (nr < 0)
        return -1;
    if (nbytes % 16)
        return -2;
    oracle_inv_sbox(ibox);
    uint8_t chain[16];
    memcpy(chain, iv, 16);
    for (size_t off = 0; off < nbytes; off += 16) {
        uint8_t x[16], c[16];
        memcpy(c, in + off, 16);
        inv_cipher_block(rk, nr, ibox, c, x);
        for (int k = 0; k < 16; ++k)
            out[off + k] = oracle_gf_add(x[k], chain[k]);
        memcpy(chain, c, 16);
    }
    return 0;
}

/* ------------------------------------------------------------------ GCM
 * Galois/Counter Mode, which the paper names as future work (sec. V: it
 * needs a 128-bit Galois field).  Written from NIST SP 800-38D:
 *   H = E(0^128); for a 96-bit IV, J0 = IV || 0^31 || 1;
 *   C = CTR from inc32(J0)  (nonce IV, first counter 2, as oracle_ctr_xcrypt);
 *   S = GHASH_H(A || 0-pad || C || 0-pad || [len(A)]_64 || [len(C)]_64)
 *       with lengths in bits, big-endian;
 *   T = E(J0) xor S.
 * GHASH_H(X_1..X_m): Y_0 = 0, Y_i = (Y_{i-1} xor X_i) * H in GF(2^128).
 * Field element bit order: bit 0 is the most significant bit of byte 0 and is
 * the coefficient of x^0; the field polynomial is x^128 + x^7 + x^2 + x + 1.
 */
/* Product in GF(2^128) (SP 800-38D sec. 6.3, Algorithm 1): for every bit i of
 * X (in the order above) add V when it is set, then V <- V * x, i.e. a shift
 * towards higher coefficients (one bit right in byte order) with the
 * reduction R = 11100001 || 0^120 when x^127 falls out. */
void oracle_gf128_mul(const uint8_t X[16], const uint8_t Y[16], uint8_t out[16])
{
    uint8_t Z[16] = {0}, V[16];
    memcpy(V, Y, 16);
    for (int i = 0; i < 128; ++i) {
        int xi = (X[i / 8] >> (7 - i % 8)) & 1;
        if (xi)
            for (int k = 0; k < 16; ++k)
                Z[k] ^= V[k];
        int lsb = V[15] & 1;
        for (int k = 15; k > 0; --k)
            V[k] = (uint8_t)((V[k] >> 1) | (V[k - 1] << 7));
        V[0] >>= 1;
        if (lsb)
            V[0] ^= 0xE1;
    }
    memcpy(out, Z, 16);
}

/* GHASH over m whole blocks (SP 800-38D Algorithm 2). */
void oracle_ghash(const uint8_t H[16], const uint8_t *X, size_t nblocks, uint8_t Y[16])
{
    uint8_t acc[16] = {0};
    for (size_t i = 0; i < nblocks; ++i) {
        for (int k = 0; k < 16; ++k)
            acc[k] ^= X[16 * i + k];
        oracle_gf128_mul(acc, H, acc);
    }
    memcpy(Y, acc, 16);
}

/* One GHASH step over a byte string zero-padded to whole blocks. */
static void ghash_update(const uint8_t H[16], uint8_t acc[16], const uint8_t *p, size_t n)
{
    for (size_t off = 0; off < n; off += 16) {
        size_t len = n - off < 16 ? n - off : 16;
        for (size_t k = 0; k < len; ++k)
            acc[k] ^= p[off + k];
        oracle_gf128_mul(acc, H, acc);
    }
}

/* Tag of (A, C) under key / 96-bit IV; shared by encryption and decryption. */
static int gcm_tag(const uint8_t *key, int key_bytes, const uint8_t iv[12],
                   const uint8_t *aad, size_t aad_len, const uint8_t *ct, size_t ct_len,
                   uint8_t tag[16])
{
    uint8_t zero[16] = {0}, H[16], J0[16], EJ0[16], acc[16] = {0}, lens[16];
    if (oracle_encrypt_block(key, key_bytes, zero, H))
        return -1;
    memcpy(J0, iv, 12);
    J0[12] = J0[13] = J0[14] = 0;
    J0[15] = 1;
    oracle_encrypt_block(key, key_bytes, J0, EJ0);
    ghash_update(H, acc, aad, aad_len);
    ghash_update(H, acc, ct, ct_len);
    uint64_t abits = (uint64_t)aad_len * 8, cbits = (uint64_t)ct_len * 8;
    for (int k = 0; k < 8; ++k) {
        lens[k] = (uint8_t)(abits >> (56 - 8 * k));
        lens[8 + k] = (uint8_t)(cbits >> (56 - 8 * k));
    }
    ghash_update(H, acc, lens, 16);
    for (int k = 0; k < 16; ++k)
        tag[k] = EJ0[k] ^ acc[k];
    return 0;
}

int oracle_gcm_encrypt(const uint8_t *key, int key_bytes, const uint8_t iv[12],
                       const uint8_t *aad, size_t aad_len, const uint8_t *in, uint8_t *out,
                       size_t nbytes, uint8_t tag[16])
{
    int rc = oracle_ctr_xcrypt(key, key_bytes, iv, 2, in, out, nbytes);
    if (rc)
        return rc;
    return gcm_tag(key, key_bytes, iv, aad, aad_len, out, nbytes, tag);
}

/* Decryption returns the plaintext and the tag computed over the received
 * ciphertext; the caller compares it with the received tag. */
int oracle_gcm_decrypt(const uint8_t *key, int key_bytes, const uint8_t iv[12],
                       const uint8_t *aad, size_t aad_len, const uint8_t *in, uint8_t *out,
                       size_t nbytes, uint8_t tag[16])
{
    int rc = gcm_tag(key, key_bytes, iv, aad, aad_len, in, nbytes, tag);
    if (rc)
        return rc;
    return oracle_ctr_xcrypt(key, key_bytes, iv, 2, in, out, nbytes);
}
