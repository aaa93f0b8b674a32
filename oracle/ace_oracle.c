/*
 * ace_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU oracle for the attestation check of
 * the ACE Runtime paper (Alg. 1, Phase 1a AttestCheck; Def. 3.1, equations
 * attestkey and credential).  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library: the SHA-256
 * constants below are not written out but computed from their closed form.
 *
 * Everything follows the plain definitions, in their notation:
 *   - SHA-256: FIPS 180-4 (sec. 4.1.2 functions, 4.2.2 constants, 5.1.1
 *     padding, 5.3.3 initial value, 6.2.2 hash computation).
 *   - HMAC-SHA256: RFC 2104 sec. 2, computed on concatenated byte strings
 *     (no midstates).
 *   - HKDF-SHA256: RFC 5869 sec. 2.2 (extract) and 2.3 (expand).
 *   - Key per identity: Def. 2.1 / equation attestkey, with the roles
 *     IKM = REV, info = the purpose string, salt = the context.
 *   - Verdict per transaction: Alg. 1 Phase 1a -- recompute the HMAC of the
 *     message under the identity's key and compare with the credential;
 *     an identity outside the registry is rejected (Alg. 2, identity
 *     existence check).
 *   - Paper-form attestation: Def. 3.1 (obj_hash, domain, credential) with
 *     Alg. 2's payload binding.
 *   - Hash-chain segments: the consensus section's clock, H_{i+1} =
 *     SHA-256(H_i).
 *   - Merkle roots of the block header (App. C, Table "ACE block header
 *     fields"); the paper fixes no leaf or odd-node rule, so the reading
 *     taken is written at oracle_merkle_root.
 *
 * Pins (none of them this file): hashlib / hmac / the openssl CLI on seeded
 * inputs, exact integer closed forms for the constants, brute force over
 * every padding length, and tamper invariants (Thm. attestation
 * unforgeability).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Constants (FIPS 180-4 sec. 4.2.2 and 5.3.3), computed, not tabled.   */
/* K[t] = first 32 bits of the fractional part of the cube root of the  */
/* t-th prime; H0[i] = same with the square root of the i-th prime.     */
/* floor(frac(cbrt(p)) * 2^32) == floor(cbrt(p * 2^96)) mod 2^32.       */
/* ------------------------------------------------------------------ */
typedef unsigned __int128 u128;

static uint32_t K[64];
static uint32_t H0[8];
static pthread_once_t constants_once = PTHREAD_ONCE_INIT;

static int is_prime(unsigned p)
{
    if (p < 2) return 0;
    for (unsigned d = 2; d * d <= p; ++d)
        if (p % d == 0) return 0;
    return 1;
}

/* largest r with r^k <= x, by bisection on exact 128-bit integers */
static uint64_t iroot(u128 x, int k)
{
    uint64_t lo = 0, hi = (uint64_t)1 << 40; /* x < 2^112 here => root < 2^38 */
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        u128 v = 1;
        for (int i = 0; i < k; ++i) v *= mid;
        if (v <= x) lo = mid; else hi = mid;
    }
    return lo;
}

static void compute_constants(void)
{
    unsigned found = 0;
    for (unsigned p = 2; found < 64; ++p) {
        if (!is_prime(p)) continue;
        K[found] = (uint32_t)iroot((u128)p << 96, 3);
        if (found < 8) H0[found] = (uint32_t)iroot((u128)p << 64, 2);
        ++found;
    }
}

static void ensure_constants(void) { pthread_once(&constants_once, compute_constants); }

void oracle_constants(uint32_t k_out[64], uint32_t iv_out[8])
{
    ensure_constants();
    memcpy(k_out, K, sizeof K);
    memcpy(iv_out, H0, sizeof H0);
}

/* ------------------------------------------------------------------ */
/* SHA-256 logical functions (FIPS 180-4 sec. 4.1.2)                     */
/* ------------------------------------------------------------------ */
static uint32_t ROTR(uint32_t x, unsigned n) { return (x >> n) | (x << (32 - n)); }
static uint32_t SHR(uint32_t x, unsigned n) { return x >> n; }
static uint32_t Ch(uint32_t x, uint32_t y, uint32_t z) { return (x & y) ^ (~x & z); }
static uint32_t Maj(uint32_t x, uint32_t y, uint32_t z) { return (x & y) ^ (x & z) ^ (y & z); }
static uint32_t BSIG0(uint32_t x) { return ROTR(x, 2) ^ ROTR(x, 13) ^ ROTR(x, 22); }
static uint32_t BSIG1(uint32_t x) { return ROTR(x, 6) ^ ROTR(x, 11) ^ ROTR(x, 25); }
static uint32_t SSIG0(uint32_t x) { return ROTR(x, 7) ^ ROTR(x, 18) ^ SHR(x, 3); }
static uint32_t SSIG1(uint32_t x) { return ROTR(x, 17) ^ ROTR(x, 19) ^ SHR(x, 10); }

/* One application of the hash computation of FIPS 180-4 sec. 6.2.2 to a
 * single 512-bit block M (64 bytes, words read big-endian per sec. 3.1).
 * H is updated in place: H <- H + rounds(H, M). */
void oracle_sha256_compress(uint32_t H[8], const uint8_t M[64])
{
    ensure_constants();
    uint32_t W[64];
    for (int t = 0; t < 16; ++t)
        W[t] = ((uint32_t)M[4 * t] << 24) | ((uint32_t)M[4 * t + 1] << 16) |
               ((uint32_t)M[4 * t + 2] << 8) | (uint32_t)M[4 * t + 3];
    for (int t = 16; t < 64; ++t)
        W[t] = SSIG1(W[t - 2]) + W[t - 7] + SSIG0(W[t - 15]) + W[t - 16];

    uint32_t a = H[0], b = H[1], c = H[2], d = H[3];
    uint32_t e = H[4], f = H[5], g = H[6], h = H[7];
    for (int t = 0; t < 64; ++t) {
        uint32_t T1 = h + BSIG1(e) + Ch(e, f, g) + K[t] + W[t];
        uint32_t T2 = BSIG0(a) + Maj(a, b, c);
        h = g; g = f; f = e; e = d + T1;
        d = c; c = b; b = a; a = T1 + T2;
    }
    H[0] += a; H[1] += b; H[2] += c; H[3] += d;
    H[4] += e; H[5] += f; H[6] += g; H[7] += h;
}

void oracle_sha256_iv(uint32_t H[8])
{
    ensure_constants();
    memcpy(H, H0, sizeof H0);
}

/* SHA-256 of a whole message: pad per sec. 5.1.1 (0x80, zeros, 64-bit
 * big-endian bit length), then compress block by block from H(0). */
void oracle_sha256(const uint8_t *msg, size_t len, uint8_t digest[32])
{
    ensure_constants();
    size_t padded = ((len + 9 + 63) / 64) * 64;
    uint8_t *buf = (uint8_t *)calloc(padded, 1);
    if (len) memcpy(buf, msg, len);
    buf[len] = 0x80;
    uint64_t bits = (uint64_t)len * 8u;
    for (int i = 0; i < 8; ++i) buf[padded - 1 - i] = (uint8_t)(bits >> (8 * i));

    uint32_t H[8];
    memcpy(H, H0, sizeof H);
    for (size_t off = 0; off < padded; off += 64) oracle_sha256_compress(H, buf + off);
    free(buf);
    for (int i = 0; i < 8; ++i) {
        digest[4 * i] = (uint8_t)(H[i] >> 24);
        digest[4 * i + 1] = (uint8_t)(H[i] >> 16);
        digest[4 * i + 2] = (uint8_t)(H[i] >> 8);
        digest[4 * i + 3] = (uint8_t)H[i];
    }
}

/* ------------------------------------------------------------------ */
/* HMAC-SHA256, RFC 2104 sec. 2 with B = 64, L = 32:                    */
/*   K0 = K padded with zeros to B (K hashed first when |K| > B)        */
/*   HMAC = H((K0 ^ opad) || H((K0 ^ ipad) || text))                    */
/* computed on the concatenated byte strings.                           */
/* ------------------------------------------------------------------ */
static void hmac_key_block(const uint8_t *key, size_t klen, uint8_t K0[64])
{
    memset(K0, 0, 64);
    if (klen > 64) oracle_sha256(key, klen, K0);
    else if (klen) memcpy(K0, key, klen);
}

void oracle_hmac_sha256(const uint8_t *key, size_t klen, const uint8_t *text, size_t tlen,
                        uint8_t mac[32])
{
    uint8_t K0[64];
    hmac_key_block(key, klen, K0);

    uint8_t *inner = (uint8_t *)malloc(64 + tlen);
    for (int i = 0; i < 64; ++i) inner[i] = K0[i] ^ 0x36;
    if (tlen) memcpy(inner + 64, text, tlen);
    uint8_t ih[32];
    oracle_sha256(inner, 64 + tlen, ih);
    free(inner);

    uint8_t outer[64 + 32];
    for (int i = 0; i < 64; ++i) outer[i] = K0[i] ^ 0x5c;
    memcpy(outer + 64, ih, 32);
    oracle_sha256(outer, sizeof outer, mac);
}

/* The two HMAC midstates of a key: F(H0, K0 ^ ipad) and F(H0, K0 ^ opad),
 * where F is the single-block computation above.  out[0..7] = ipad state,
 * out[8..15] = opad state, as native 32-bit words. */
void oracle_hmac_midstates(const uint8_t *key, size_t klen, uint32_t out[16])
{
    uint8_t K0[64], blk[64];
    hmac_key_block(key, klen, K0);
    for (int i = 0; i < 64; ++i) blk[i] = K0[i] ^ 0x36;
    oracle_sha256_iv(out);
    oracle_sha256_compress(out, blk);
    for (int i = 0; i < 64; ++i) blk[i] = K0[i] ^ 0x5c;
    oracle_sha256_iv(out + 8);
    oracle_sha256_compress(out + 8, blk);
}

/* ------------------------------------------------------------------ */
/* HKDF-SHA256, RFC 5869.                                               */
/*   2.2 Extract: PRK = HMAC(salt, IKM); absent salt = HashLen zeros.   */
/*   2.3 Expand:  T(0) = empty; T(i) = HMAC(PRK, T(i-1) || info || i);  */
/*                OKM = first L octets of T(1) || T(2) || ...           */
/* Returns 0, or -1 when L > 255 * HashLen.                             */
/* ------------------------------------------------------------------ */
int oracle_hkdf_sha256(const uint8_t *salt, size_t slen, const uint8_t *ikm, size_t ilen,
                       const uint8_t *info, size_t infolen, uint8_t *okm, size_t L)
{
    if (L > 255u * 32u) return -1;
    static const uint8_t zeros[32] = {0};
    if (salt == NULL || slen == 0) { salt = zeros; slen = 32; }

    uint8_t prk[32];
    oracle_hmac_sha256(salt, slen, ikm, ilen, prk);

    size_t N = (L + 31) / 32;
    uint8_t T[32];
    size_t tlen = 0, done = 0;
    uint8_t *buf = (uint8_t *)malloc(32 + infolen + 1);
    for (size_t i = 1; i <= N; ++i) {
        size_t pos = 0;
        memcpy(buf + pos, T, tlen); pos += tlen;
        if (infolen) memcpy(buf + pos, info, infolen);
        pos += infolen;
        buf[pos++] = (uint8_t)i;
        oracle_hmac_sha256(prk, 32, buf, pos, T);
        tlen = 32;
        size_t take = (L - done < 32) ? (L - done) : 32;
        memcpy(okm + done, T, take);
        done += take;
    }
    free(buf);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Batched forms, split over threads by static ranges (timing only;     */
/* each item is the plain definition above).                            */
/* ------------------------------------------------------------------ */
typedef struct {
    int kind; /* 0 = derive keys, 1 = verify */
    size_t lo, hi;
    /* derive */
    const uint8_t *rev; const uint8_t *salt; size_t slen; const uint8_t *info; size_t infolen;
    uint8_t *keys_out;
    /* verify */
    const uint8_t *keys; uint32_t n_id;
    const uint8_t *msg; const uint64_t *off; const uint32_t *id; const uint8_t *tag;
    uint32_t *bitmask; uint64_t count;
    /* paper-form attestation */
    const uint8_t *att; /* [n][72]: obj_hash (32) || domain (8) || credential (32) */
    /* hash-chain segments */
    const uint8_t *seg_start, *seg_end; const uint32_t *seg_steps;
} job_t;

/* Full 32-byte compare with no early exit: OR of the XORs of all bytes. */
static int cteq32(const uint8_t *x, const uint8_t *y)
{
    uint8_t d = 0;
    for (int i = 0; i < 32; ++i) d |= (uint8_t)(x[i] ^ y[i]);
    return d == 0;
}

static void *run_job(void *arg)
{
    job_t *j = (job_t *)arg;
    if (j->kind == 0) {
        for (size_t i = j->lo; i < j->hi; ++i)
            oracle_hkdf_sha256(j->salt, j->slen, j->rev + 32 * i, 32, j->info, j->infolen,
                               j->keys_out + 32 * i, 32);
        return NULL;
    }
    uint64_t count = 0;
    if (j->kind == 3) {
        /* Sec. "Verifiable Clock via Proof of History": H_{i+1} = SHA-256(H_i)
         * over the 32 digest bytes; segment i is valid when steps[i] such
         * hashes lead from its start to its end. */
        for (size_t i = j->lo; i < j->hi; ++i) {
            uint8_t h[32], nxt[32];
            memcpy(h, j->seg_start + 32 * i, 32);
            for (uint32_t t = 0; t < j->seg_steps[i]; ++t) {
                oracle_sha256(h, 32, nxt);
                memcpy(h, nxt, 32);
            }
            if (cteq32(h, j->seg_end + 32 * i)) {
                j->bitmask[i / 32] |= (uint32_t)1 << (i % 32);
                ++count;
            }
        }
        j->count = count;
        return NULL;
    }
    for (size_t i = j->lo; i < j->hi; ++i) {
        int valid = 0;
        uint32_t who = j->id[i];
        uint64_t a = j->off[i], b = j->off[i + 1];
        if (j->kind == 2) {
            /* Def. 3.1 / Alg. 2: obj_hash = SHA-256(P) (payload binding) and
             * credential = HMAC(k, obj_hash || domain), identity registered. */
            if (who < j->n_id && a <= b) {
                const uint8_t *A = j->att + 72 * i;
                uint8_t h[32], mac[32];
                oracle_sha256(j->msg + a, (size_t)(b - a), h);
                oracle_hmac_sha256(j->keys + 32 * (size_t)who, 32, A, 40, mac);
                valid = cteq32(h, A) & cteq32(mac, A + 40);
            }
        } else if (who < j->n_id && a <= b) {
            uint8_t mac[32];
            oracle_hmac_sha256(j->keys + 32 * (size_t)who, 32, j->msg + a, (size_t)(b - a), mac);
            valid = cteq32(mac, j->tag + 32 * i);
        }
        if (valid) {
            j->bitmask[i / 32] |= (uint32_t)1 << (i % 32);
            ++count;
        }
    }
    j->count = count;
    return NULL;
}

static void run_split(job_t *tmpl, size_t n, int nthreads, size_t align, uint64_t *count_out)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    job_t jobs[256];
    pthread_t th[256];
    int started[256];
    size_t per = (n + (size_t)nthreads - 1) / (size_t)nthreads;
    per = ((per + align - 1) / align) * align; /* threads own whole bitmask words */
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *tmpl;
        size_t lo = (size_t)t * per;
        jobs[t].lo = lo < n ? lo : n;
        jobs[t].hi = jobs[t].lo + per < n ? jobs[t].lo + per : n;
        jobs[t].count = 0;
        started[t] = 0;
        if (t > 0 && jobs[t].lo < jobs[t].hi)
            started[t] = pthread_create(&th[t], NULL, run_job, &jobs[t]) == 0;
    }
    run_job(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) {
        if (started[t]) pthread_join(th[t], NULL);
        else if (jobs[t].lo < jobs[t].hi) run_job(&jobs[t]); /* thread creation failed */
    }
    uint64_t total = 0;
    for (int t = 0; t < nthreads; ++t) total += jobs[t].count;
    if (count_out) *count_out = total;
}

/* k_j = HKDF(salt, IKM = rev[j], info, 32) for j < n_id (Def. 2.1). */
void oracle_derive_keys(const uint8_t *rev, uint32_t n_id, const uint8_t *salt, size_t slen,
                        const uint8_t *info, size_t infolen, uint8_t *keys_out, int nthreads)
{
    job_t t;
    memset(&t, 0, sizeof t);
    t.kind = 0;
    t.rev = rev; t.salt = salt; t.slen = slen; t.info = info; t.infolen = infolen;
    t.keys_out = keys_out;
    run_split(&t, n_id, nthreads, 1, NULL);
}

/* valid_i = (id_i < n_id) and (off_i <= off_{i+1}) and
 *           CTEQ32(HMAC(k_{id_i}, msg[off_i .. off_{i+1})), tag_i)
 * bitmask: bit i%32 of word i/32, LSB first, unused tail bits 0. */
void oracle_verify_batch(const uint8_t *keys, uint32_t n_id, const uint8_t *msg,
                         const uint64_t *off, const uint32_t *id, const uint8_t *tag, uint64_t n,
                         uint32_t *bitmask_out, uint64_t *count_out, int nthreads)
{
    memset(bitmask_out, 0, sizeof(uint32_t) * (size_t)((n + 31) / 32));
    job_t t;
    memset(&t, 0, sizeof t);
    t.kind = 1;
    t.keys = keys; t.n_id = n_id; t.msg = msg; t.off = off; t.id = id; t.tag = tag;
    t.bitmask = bitmask_out;
    run_split(&t, (size_t)n, nthreads, 32, count_out);
}

/* Paper-form attestation check of Def. 3.1 and Alg. 2 (the "full check"):
 *   valid_i = (id_i < n_id) and (poff_i <= poff_{i+1})
 *             and SHA-256(payload_i) == obj_hash_i
 *             and HMAC-SHA256(k_{id_i}, obj_hash_i || domain_i) == credential_i
 * with att_i = obj_hash (32) || domain (8) || credential (32). */
void oracle_verify_attest(const uint8_t *keys, uint32_t n_id, const uint8_t *payload,
                          const uint64_t *poff, const uint32_t *id, const uint8_t *att, uint64_t n,
                          uint32_t *bitmask_out, uint64_t *count_out, int nthreads)
{
    memset(bitmask_out, 0, sizeof(uint32_t) * (size_t)((n + 31) / 32));
    job_t t;
    memset(&t, 0, sizeof t);
    t.kind = 2;
    t.keys = keys; t.n_id = n_id; t.msg = payload; t.off = poff; t.id = id; t.att = att;
    t.bitmask = bitmask_out;
    run_split(&t, (size_t)n, nthreads, 32, count_out);
}

/* Hash-chain segments: bit i set iff SHA-256 applied steps[i] times to
 * start[i] gives end[i] (32-byte values). */
void oracle_poh_verify(const uint8_t *start, const uint8_t *end, const uint32_t *steps, uint64_t n,
                       uint32_t *bitmask_out, uint64_t *count_out, int nthreads)
{
    memset(bitmask_out, 0, sizeof(uint32_t) * (size_t)((n + 31) / 32));
    job_t t;
    memset(&t, 0, sizeof t);
    t.kind = 3;
    t.seg_start = start; t.seg_end = end; t.seg_steps = steps;
    t.bitmask = bitmask_out;
    run_split(&t, (size_t)n, nthreads, 32, count_out);
}

/* Merkle root of the n leaves data[off[i] .. off[i+1]) (the block header's
 * transaction and attestation roots): leaf node = SHA-256(leaf bytes), parent
 * = SHA-256(left || right); when a level has an odd count its last node moves
 * up unchanged; no leaves gives SHA-256 of the empty string.  A leaf with
 * off[i+1] < off[i] is hashed as the empty string.  Returns 0, or -1 when
 * memory runs out. */
int oracle_merkle_root(const uint8_t *data, const uint64_t *off, uint64_t n, uint8_t root[32])
{
    static const uint8_t none = 0;
    if (n == 0) {
        oracle_sha256(&none, 0, root);
        return 0;
    }
    uint8_t *lvl = (uint8_t *)malloc((size_t)(32 * n));
    if (!lvl) return -1;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t a = off[i], b = off[i + 1];
        oracle_sha256(b >= a ? data + a : &none, b >= a ? (size_t)(b - a) : 0, lvl + 32 * i);
    }
    uint64_t m = n;
    while (m > 1) {
        uint64_t k = 0;
        for (uint64_t i = 0; i + 1 < m; i += 2, ++k) {
            uint8_t pair[64];
            memcpy(pair, lvl + 32 * i, 32);
            memcpy(pair + 32, lvl + 32 * (i + 1), 32);
            oracle_sha256(pair, 64, lvl + 32 * k);
        }
        if (m & 1) {
            memmove(lvl + 32 * k, lvl + 32 * (m - 1), 32);
            ++k;
        }
        m = k;
    }
    memcpy(root, lvl, 32);
    free(lvl);
    return 0;
}
