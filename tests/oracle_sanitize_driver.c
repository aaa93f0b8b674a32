/*
 * Drives every entry point of the CPU oracle on seeded random inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers.py).  It checks nothing itself beyond a few
 * consistency relations; the sanitizers check the memory accesses and the
 * integer arithmetic.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_sha256(const uint8_t *msg, size_t len, uint8_t digest[32]);
void oracle_hmac_sha256(const uint8_t *key, size_t klen, const uint8_t *text, size_t tlen,
                        uint8_t out[32]);
int oracle_hkdf_sha256(const uint8_t *salt, size_t slen, const uint8_t *ikm, size_t ilen,
                       const uint8_t *info, size_t infolen, uint8_t *okm, size_t L);
void oracle_derive_keys(const uint8_t *rev, uint32_t n_id, const uint8_t *salt, size_t slen,
                        const uint8_t *info, size_t infolen, uint8_t *keys_out, int nthreads);
void oracle_verify_batch(const uint8_t *keys, uint32_t n_id, const uint8_t *msg,
                         const uint64_t *off, const uint32_t *id, const uint8_t *tag, uint64_t n,
                         uint32_t *bitmask_out, uint64_t *count_out, int nthreads);
void oracle_verify_attest(const uint8_t *keys, uint32_t n_id, const uint8_t *payload,
                          const uint64_t *poff, const uint32_t *id, const uint8_t *att, uint64_t n,
                          uint32_t *bitmask_out, uint64_t *count_out, int nthreads);
void oracle_poh_verify(const uint8_t *start, const uint8_t *end, const uint32_t *steps, uint64_t n,
                       uint32_t *bitmask_out, uint64_t *count_out, int nthreads);
int oracle_merkle_root(const uint8_t *data, const uint64_t *off, uint64_t n, uint8_t root[32]);

static uint64_t rs = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void)
{
    rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17;
    return (uint32_t)(rs >> 11);
}
static uint8_t *rbytes(size_t n)
{
    uint8_t *p = (uint8_t *)malloc(n ? n : 1);
    for (size_t i = 0; i < n; ++i) p[i] = (uint8_t)rnd();
    return p;
}

int main(void)
{
    uint8_t d[32], e[32];
    for (size_t L = 0; L < 300; ++L) {          /* every padding case, exact-size buffers */
        uint8_t *m = rbytes(L);
        oracle_sha256(m, L, d);
        uint8_t *k = rbytes(L % 150);
        oracle_hmac_sha256(k, L % 150, m, L, e);
        free(k);
        free(m);
    }
    uint8_t okm[8160];
    uint8_t *salt = rbytes(200), *ikm = rbytes(32), *info = rbytes(255);
    if (oracle_hkdf_sha256(salt, 200, ikm, 32, info, 255, okm, 8160) != 0) return 1;
    if (oracle_hkdf_sha256(NULL, 0, ikm, 32, info, 0, okm, 32) != 0) return 1;
    if (oracle_hkdf_sha256(salt, 0, ikm, 32, info, 0, okm, 8161) == 0) return 1;

    const uint32_t n_id = 64;
    const uint64_t n = 1000;
    uint8_t *rev = rbytes(32 * n_id), *keys = (uint8_t *)malloc(32 * n_id);
    oracle_derive_keys(rev, n_id, salt, 32, info, 16, keys, 3);
    uint64_t *off = (uint64_t *)malloc(8 * (n + 1));
    off[0] = 0;
    for (uint64_t i = 0; i < n; ++i) off[i + 1] = off[i] + rnd() % 200;
    uint8_t *msg = rbytes(off[n]);
    uint32_t *id = (uint32_t *)malloc(4 * n);
    for (uint64_t i = 0; i < n; ++i) id[i] = rnd() % (n_id + 3);   /* some unregistered */
    uint8_t *tag = rbytes(32 * n), *att = rbytes(72 * n);
    uint32_t *mask = (uint32_t *)malloc(4 * ((n + 31) / 32));
    uint64_t count = 0;
    oracle_verify_batch(keys, n_id, msg, off, id, tag, n, mask, &count, 4);
    oracle_verify_attest(keys, n_id, msg, off, id, att, n, mask, &count, 4);
    off[500] = off[501] + 5;                                         /* decreasing offsets */
    oracle_verify_batch(keys, n_id, msg, off, id, tag, n, mask, &count, 2);
    uint8_t *st = rbytes(32 * n), *en = rbytes(32 * n);
    uint32_t *steps = (uint32_t *)malloc(4 * n);
    for (uint64_t i = 0; i < n; ++i) steps[i] = rnd() % 20;
    oracle_poh_verify(st, en, steps, n, mask, &count, 3);
    oracle_merkle_root(msg, off, 0, d);
    oracle_merkle_root(msg, off, 1, d);
    oracle_merkle_root(msg, off, 499, d);
    printf("ok\n");
    free(salt); free(ikm); free(info); free(rev); free(keys); free(off); free(msg); free(id);
    free(tag); free(att); free(mask); free(st); free(en); free(steps);
    return 0;
}
