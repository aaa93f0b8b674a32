/*
 * attest_client.c -- client side of the synthetic workload.
 *
 * Makes the credentials a client would attach to its transactions (the
 * paper's Alg. 2, GenerateAttestation: key by HKDF, credential by HMAC)
 * so that the verifier has something to check.  Every cryptographic step is
 * delegated to the host's OpenSSL (EVP_KDF "HKDF", EVP_MAC "HMAC"); this
 * file contains no hash arithmetic of its own and is used by neither the
 * GPU library nor the CPU oracle.
 */
#include <openssl/core_names.h>
#include <openssl/evp.h>
#include <openssl/kdf.h>
#include <openssl/params.h>
#include <pthread.h>
#include <stdint.h>
#include <string.h>

typedef struct {
    int kind; /* 0 = keys, 1 = tags, 2 = digests, 3 = hash chains */
    uint64_t lo, hi;
    const uint8_t *rev, *salt, *info;
    size_t slen, ilen;
    uint8_t *keys_out;
    const uint8_t *keys;
    const uint8_t *msg;
    const uint64_t *off;
    const uint32_t *key_index;
    uint8_t *tags_out;
    const uint32_t *steps;
    int status;
} job_t;

static void derive_range(job_t *j)
{
    EVP_KDF *kdf = EVP_KDF_fetch(NULL, "HKDF", NULL);
    EVP_KDF_CTX *ctx = kdf ? EVP_KDF_CTX_new(kdf) : NULL;
    if (!ctx) { j->status = -1; EVP_KDF_free(kdf); return; }
    /* digest, salt and info are the same for every identity and set once (the
       digest named in every call was looked up again each time, under a lock
       the threads share); each derivation passes only its key */
    OSSL_PARAM c[4], *q = c;
    *q++ = OSSL_PARAM_construct_utf8_string(OSSL_KDF_PARAM_DIGEST, (char *)"SHA256", 0);
    if (j->slen)
        *q++ = OSSL_PARAM_construct_octet_string(OSSL_KDF_PARAM_SALT, (void *)j->salt, j->slen);
    *q++ = OSSL_PARAM_construct_octet_string(OSSL_KDF_PARAM_INFO, (void *)j->info, j->ilen);
    *q = OSSL_PARAM_construct_end();
    if (EVP_KDF_CTX_set_params(ctx, c) <= 0) j->status = -1;
    for (uint64_t i = j->lo; i < j->hi && !j->status; ++i) {
        OSSL_PARAM p[2];
        p[0] = OSSL_PARAM_construct_octet_string(OSSL_KDF_PARAM_KEY, (void *)(j->rev + 32 * i), 32);
        p[1] = OSSL_PARAM_construct_end();
        if (EVP_KDF_derive(ctx, j->keys_out + 32 * i, 32, p) <= 0) { j->status = -2; break; }
    }
    EVP_KDF_CTX_free(ctx);
    EVP_KDF_free(kdf);
}

static void sign_range(job_t *j)
{
    EVP_MAC *mac = EVP_MAC_fetch(NULL, "HMAC", NULL);
    EVP_MAC_CTX *ctx = mac ? EVP_MAC_CTX_new(mac) : NULL;
    if (!ctx) { j->status = -1; EVP_MAC_free(mac); return; }
    OSSL_PARAM p[2];
    p[0] = OSSL_PARAM_construct_utf8_string(OSSL_MAC_PARAM_DIGEST, (char *)"SHA256", 0);
    p[1] = OSSL_PARAM_construct_end();
    /* the digest is set once: passed to every init, it was looked up again each
       time, under a lock the threads share */
    if (EVP_MAC_CTX_set_params(ctx, p) <= 0) { j->status = -1; EVP_MAC_CTX_free(ctx); EVP_MAC_free(mac); return; }
    for (uint64_t i = j->lo; i < j->hi; ++i) {
        size_t outl = 0;
        const uint8_t *key = j->keys + 32 * (size_t)j->key_index[i];
        const uint8_t *m = j->msg + j->off[i];
        size_t len = (size_t)(j->off[i + 1] - j->off[i]);
        if (EVP_MAC_init(ctx, key, 32, NULL) <= 0 || EVP_MAC_update(ctx, m, len) <= 0 ||
            EVP_MAC_final(ctx, j->tags_out + 32 * i, &outl, 32) <= 0 || outl != 32) {
            j->status = -2;
            break;
        }
    }
    EVP_MAC_CTX_free(ctx);
    EVP_MAC_free(mac);
}

static void digest_range(job_t *j)
{
    for (uint64_t i = j->lo; i < j->hi; ++i) {
        unsigned int outl = 0;
        const uint8_t *m = j->msg + j->off[i];
        size_t len = (size_t)(j->off[i + 1] - j->off[i]);
        if (EVP_Digest(m, len, j->tags_out + 32 * i, &outl, EVP_sha256(), NULL) <= 0 || outl != 32) {
            j->status = -2;
            break;
        }
    }
}

static void chain_range(job_t *j)
{
    EVP_MD *md = EVP_MD_fetch(NULL, "SHA256", NULL);
    EVP_MD_CTX *ctx = md ? EVP_MD_CTX_new() : NULL;
    if (!ctx) { j->status = -1; EVP_MD_free(md); return; }
    for (uint64_t i = j->lo; i < j->hi && !j->status; ++i) {
        uint8_t h[32];
        unsigned int outl = 0;
        memcpy(h, j->msg + 32 * i, 32);
        for (uint32_t t = 0; t < j->steps[i]; ++t) {
            if (EVP_DigestInit_ex(ctx, md, NULL) <= 0 || EVP_DigestUpdate(ctx, h, 32) <= 0 ||
                EVP_DigestFinal_ex(ctx, h, &outl) <= 0 || outl != 32) {
                j->status = -2;
                break;
            }
        }
        memcpy(j->tags_out + 32 * i, h, 32);
    }
    EVP_MD_CTX_free(ctx);
    EVP_MD_free(md);
}

static void *run(void *arg)
{
    job_t *j = (job_t *)arg;
    if (j->kind == 0) derive_range(j);
    else if (j->kind == 1) sign_range(j);
    else if (j->kind == 2) digest_range(j);
    else chain_range(j);
    return NULL;
}

static int split(job_t *tmpl, uint64_t n, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 128) nthreads = 128;
    job_t jobs[128];
    pthread_t th[128];
    int started[128];
    uint64_t per = (n + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *tmpl;
        jobs[t].lo = (uint64_t)t * per < n ? (uint64_t)t * per : n;
        jobs[t].hi = jobs[t].lo + per < n ? jobs[t].lo + per : n;
        jobs[t].status = 0;
        started[t] = (t > 0 && jobs[t].lo < jobs[t].hi) &&
                     pthread_create(&th[t], NULL, run, &jobs[t]) == 0;
    }
    run(&jobs[0]);
    int status = 0;
    for (int t = 1; t < nthreads; ++t) {
        if (started[t]) pthread_join(th[t], NULL);
        else if (jobs[t].lo < jobs[t].hi) run(&jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t)
        if (jobs[t].status) status = jobs[t].status;
    return status;
}

/* keys[j] = HKDF-SHA256(salt, IKM = rev[j], info, 32 bytes) via OpenSSL. */
int client_derive_keys(const uint8_t *rev, uint64_t n_id, const uint8_t *salt, size_t slen,
                       const uint8_t *info, size_t ilen, uint8_t *keys_out, int nthreads)
{
    job_t t;
    memset(&t, 0, sizeof t);
    t.kind = 0;
    t.rev = rev; t.salt = salt; t.slen = slen; t.info = info; t.ilen = ilen;
    t.keys_out = keys_out;
    return split(&t, n_id, nthreads);
}

/* tags[i] = HMAC-SHA256(keys[key_index[i]], msg[off[i] .. off[i+1])) via OpenSSL. */
int client_sign(const uint8_t *keys, const uint8_t *msg, const uint64_t *off,
                const uint32_t *key_index, uint64_t n, uint8_t *tags_out, int nthreads)
{
    job_t t;
    memset(&t, 0, sizeof t);
    t.kind = 1;
    t.keys = keys; t.msg = msg; t.off = off; t.key_index = key_index; t.tags_out = tags_out;
    return split(&t, n, nthreads);
}

/* out[i] = SHA-256(msg[off[i] .. off[i+1])) via OpenSSL. */
int client_digest(const uint8_t *msg, const uint64_t *off, uint64_t n, uint8_t *out, int nthreads)
{
    job_t t;
    memset(&t, 0, sizeof t);
    t.kind = 2;
    t.msg = msg; t.off = off; t.tags_out = out;
    return split(&t, n, nthreads);
}

/* end[i] = SHA-256 applied steps[i] times to start[i] (32-byte values) via OpenSSL. */
int client_hash_chain(const uint8_t *start, const uint32_t *steps, uint64_t n, uint8_t *end,
                      int nthreads)
{
    job_t t;
    memset(&t, 0, sizeof t);
    t.kind = 3;
    t.msg = start; t.steps = steps; t.tags_out = end;
    return split(&t, n, nthreads);
}
