// hkdf_kernels.hip -- key derivation on gfx950: HKDF-SHA256 (RFC 5869) of
// each identity's root entropy under a (salt, info) pair (Def. 2.1; Def. 3.1
// equation attestkey) and the HMAC ipad/opad midstates of the derived key.
//
//   k_derive         one identity per lane, one parameter set.
//   k_derive_multi   one grid row per parameter set (several purpose streams).
//
// Included by ace_kernels.hip after its load and lane helpers.

namespace ace {

// Big-endian word g of the SHA-256 padding of the byte string
// p[0..len) || tail[0..tail_len) whose bit-length field holds `bitlen` and
// whose padded form has `nblocks` blocks (FIPS 180-4 sec. 5.1.1).
__device__ inline uint32_t padded_word(const uint8_t *p, uint32_t len, uint32_t tail,
                                       uint32_t tail_len, uint32_t g, uint32_t nblocks,
                                       uint64_t bitlen)
{
    if (g == 16 * nblocks - 2) return (uint32_t)(bitlen >> 32);
    if (g == 16 * nblocks - 1) return (uint32_t)bitlen;
    const uint32_t total = len + tail_len;
    uint32_t w = 0;
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t pos = 4 * g + k;
        uint32_t byte;
        if (pos < len) byte = p[pos];
        else if (pos < total) byte = (tail >> (8 * (pos - len))) & 0xFFu;
        else byte = pos == total ? 0x80u : 0u;
        w = (w << 8) | byte;
    }
    return w;
}

// Per-workgroup HKDF constants: the salt's HMAC midstates and the padded
// expand input (info || 0x01), built by wave 0 (all lanes compute the same
// values) into LDS.
template <class Params>
__device__ void hkdf_prepare(const Params &hp, HkdfPrep &out)
{
    uint32_t k0[16];
    const uint32_t sl = hp.salt_len;
    if (sl > 64) {
        // RFC 2104: keys longer than the block are hashed first.
        const uint32_t nblk = (sl + 9 + 63) / 64;
        State s = initial_state();
        for (uint32_t blk = 0; blk < nblk; ++blk) {
            uint32_t W[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) W[j] = padded_word(hp.salt, sl, 0, 0, 16 * blk + j, nblk, 8ull * sl);
            compress(s, W);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) k0[j] = s.h[j];
#pragma unroll
        for (int j = 8; j < 16; ++j) k0[j] = 0;
    } else {
        // RFC 5869: an absent salt is HashLen zero bytes, whose key block is
        // the same all-zero K0 as the empty key's.
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            uint32_t w = 0;
            for (uint32_t k = 0; k < 4; ++k) {
                const uint32_t pos = 4 * j + k;
                w = (w << 8) | (pos < sl ? hp.salt[pos] : 0u);
            }
            k0[j] = w;
        }
    }
    for (int pass = 0; pass < 2; ++pass) {
        const uint32_t x = pass ? 0x5c5c5c5cu : 0x36363636u;
        uint32_t W[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) W[j] = k0[j] ^ x;
        State s = initial_state();
        compress(s, W);
        if (lane_id() == 0) {
#pragma unroll
            for (int j = 0; j < 8; ++j) (pass ? out.salt_opad : out.salt_ipad)[j] = s.h[j];
        }
    }
    // Expand input T(1) = HMAC(PRK, info || 0x01): after the 64-byte key
    // block the hashed stream is info || 0x01, bit length (64 + len + 1) * 8.
    // Each of its blocks is stored as K[t] + W[t] for all 64 rounds (FIPS
    // 180-4 sec. 6.2.2 steps 1 and 3 with the message-dependent part done once).
    const uint32_t il = hp.info_len;
    const uint32_t nq = (il + 1 + 9 + 63) / 64;
    if (lane_id() == 0) {
        for (uint32_t q = 0; q < nq; ++q) {
            uint32_t W[16];
#pragma unroll
            for (int j = 0; j < 16; ++j)
                W[j] = padded_word(hp.info, il, 0x01u, 1, 16 * q + j, nq, 8ull * (64 + il + 1));
#pragma unroll
            for (int t = 0; t < 64; ++t) {
                if (t >= 16)
                    W[t & 15] = small_sigma1(W[(t - 2) & 15]) + W[(t - 7) & 15] +
                                small_sigma0(W[(t - 15) & 15]) + W[t & 15];
                out.info_kw[q][t] = W[t & 15] + kRound[t];
            }
        }
        out.info_blocks = nq;
    }
}

// F(s, B) for a block B whose schedule is the same on every lane, given as
// kw[t] = K[t] + W[t]: only the 64 rounds run per lane (about 900 instead of
// 1,384 VALU instructions).  kw lives in LDS; sixteen words are read per
// iteration of the round loop.
__device__ __forceinline__ void compress_kw(State &s, const uint32_t *kw)
{
    uint32_t a = s.h[0], b = s.h[1], c = s.h[2], d = s.h[3];
    uint32_t e = s.h[4], f = s.h[5], g = s.h[6], h = s.h[7];
#pragma nounroll
    for (int q = 0; q < 4; ++q) {
        const RoundConsts16 kq = *reinterpret_cast<const RoundConsts16 *>(kw + 16 * q);
#pragma unroll
        for (int j = 0; j < 16; ++j) round_step(a, b, c, d, e, f, g, h, 0u, kq.k[j]);
    }
    s.h[0] += a; s.h[1] += b; s.h[2] += c; s.h[3] += d;
    s.h[4] += e; s.h[5] += f; s.h[6] += g; s.h[7] += h;
}

// HMAC midstate F(IV, K0 ^ pad) of a 32-byte key held as state words
// (K0 = key || 0^32): words 8..15 of the block are the pad pattern itself.
template <uint32_t PAD>
__device__ __forceinline__ State hmac_midstate(const State &k)
{
    uint32_t W[16];
#pragma unroll
    for (int i = 0; i < 8; ++i) W[i] = k.h[i] ^ PAD;
#pragma unroll
    for (int i = 8; i < 16; ++i) W[i] = PAD;
    State t = initial_state();
    compress_fold(t, W);
    return t;
}

// Both midstates; each pass has its pad as a constant, so its words 8..15
// fold into the schedule.
__device__ __forceinline__ void hmac_midstates(const State &k, State &ipad, State &opad)
{
    ipad = hmac_midstate<0x36363636u>(k);
    opad = hmac_midstate<0x5c5c5c5cu>(k);
}

// F(in, m || 0x80 || 0 || 768): a 32-byte message after a 64-byte key block.
__device__ __forceinline__ void compress_tail32(State &in, const State &m)
{
    uint32_t W[16];
#pragma unroll
    for (int i = 0; i < 8; ++i) W[i] = m.h[i];
    W[8] = 0x80000000u;
#pragma unroll
    for (int i = 9; i < 15; ++i) W[i] = 0u;
    W[15] = 768u;
    compress_fold(in, W);
}

// HKDF-SHA256 (RFC 5869, L = 32) of one 32-byte root entropy rv (big-endian
// words) and the midstates of the resulting key:
//   extract  PRK = HMAC(salt, rv): F(salt_ipad, rv || pad), then F(salt_opad, . || pad)
//   expand   k = HMAC(PRK, info || 0x01): PRK midstates, the info blocks from
//            the PRK ipad state, then F(PRK opad state, . || pad)
//   and the key's own midstates F(IV, k^ipad), F(IV, k^opad).
__device__ __forceinline__ void derive_lane(bool live, const uint32_t (&rv)[8], const HkdfPrep &P,
                                            uint32_t (&key)[8], State &kip, State &kop)
{
    (void)live;  // lanes without an identity compute on zeros; their results are not stored
    State m, x, prk;
#pragma unroll
    for (int i = 0; i < 8; ++i) { m.h[i] = rv[i]; x.h[i] = P.salt_ipad[i]; prk.h[i] = P.salt_opad[i]; }
    compress_tail32(x, m);
    compress_tail32(prk, x);
    State pi, po;
    hmac_midstates(prk, pi, po);
    const uint32_t nq = P.info_blocks;
    for (uint32_t q = 0; q < nq; ++q) compress_kw(pi, P.info_kw[q]);
    compress_tail32(po, pi);  // po = k
#pragma unroll
    for (int i = 0; i < 8; ++i) key[i] = po.h[i];
    hmac_midstates(po, kip, kop);
}

// ------------------------------------------------------------------------------------------
// k_derive: one identity per lane.
// ------------------------------------------------------------------------------------------
// Root entropy of identity j as loaded (little-endian words).
struct RevRaw {
    U4 a, b;
};

__device__ __forceinline__ RevRaw load_rev(const uint8_t *__restrict__ rev, uint32_t j)
{
    const uint32_t *p = reinterpret_cast<const uint32_t *>(rev + 32ull * j);
    return RevRaw{load16(p), load16(p + 4)};
}

// Key and midstates of an identity from its root entropy x (ignored unless
// live); outputs go to row `row` of key_out / mid_out.
__device__ __forceinline__ void derive_store(bool live, const RevRaw &x, uint64_t row,
                                             const HkdfPrep &prep, uint8_t *__restrict__ key_out,
                                             uint32_t *__restrict__ mid_out)
{
    uint32_t rv[8];
    if (live) {
        rv[0] = bswap32(x.a.x); rv[1] = bswap32(x.a.y); rv[2] = bswap32(x.a.z); rv[3] = bswap32(x.a.w);
        rv[4] = bswap32(x.b.x); rv[5] = bswap32(x.b.y); rv[6] = bswap32(x.b.z); rv[7] = bswap32(x.b.w);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) rv[i] = 0;
    }
    uint32_t key[8];
    State kip, kop;
    derive_lane(live, rv, prep, key, kip, kop);
    if (!live) return;
    if (key_out) {
        uint32_t *q = reinterpret_cast<uint32_t *>(key_out + 32ull * row);
#pragma unroll
        for (int i = 0; i < 8; ++i) q[i] = bswap32(key[i]);
    }
    if (mid_out) {
        uint32_t *q = mid_out + 16ull * row;
#pragma unroll
        for (int i = 0; i < 8; ++i) { q[i] = kip.h[i]; q[8 + i] = kop.h[i]; }
    }
}

__global__ void __launch_bounds__(kWG) ACE_WAVES(5) k_derive(const uint8_t *__restrict__ rev, uint32_t n_id,
                                                uint8_t *__restrict__ key_out,
                                                uint32_t *__restrict__ mid_out, HkdfParams hp)
{
    // grid-stride: a grid smaller than n_id / kWG leaves CU slots to kernels
    // running beside it on another stream.  Each lane's next identity is
    // loaded before the current one is derived (the first one before the
    // parameter set is prepared), so with one wave per SIMD the load's
    // latency is not added to every identity.
    const uint64_t stride = (uint64_t)gridDim.x * kWG;
    uint64_t j = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    RevRaw next{};
    if (j < n_id) next = load_rev(rev, (uint32_t)j);
    __shared__ HkdfPrep prep;
    if (threadIdx.x < 64) hkdf_prepare(hp, prep);
    __syncthreads();
    // the first identity's words are waited for here, so that in the loop the
    // compiler waits only for the prefetch and not for the stores after it
    asm volatile("" :: "v"(next.a.x), "v"(next.a.y), "v"(next.a.z), "v"(next.a.w), "v"(next.b.x),
                 "v"(next.b.y), "v"(next.b.z), "v"(next.b.w));
    for (uint64_t base = (uint64_t)blockIdx.x * kWG; base < n_id; base += stride, j += stride) {
        const RevRaw cur = next;
        if (j + stride < n_id) next = load_rev(rev, (uint32_t)(j + stride));
        derive_store(j < n_id, cur, j, prep, key_out, mid_out);
    }
}

// k_derive_multi: grid row y derives every identity's key under parameter set
// first + y (Def. 2.1's purpose streams, per-slot domains); output row
// (first + y) * n_id + j.
__global__ void __launch_bounds__(kWG) ACE_WAVES(5) k_derive_multi(const uint8_t *__restrict__ rev,
                                                      uint32_t n_id, uint8_t *__restrict__ key_out,
                                                      uint32_t *__restrict__ mid_out, MultiHkdf mp)
{
    __shared__ HkdfPrep prep;
    const uint32_t y = blockIdx.y;
    if (threadIdx.x < 64) hkdf_prepare(mp.s[y], prep);
    __syncthreads();
    const uint32_t j = blockIdx.x * kWG + threadIdx.x;
    const bool live = j < n_id;
    RevRaw x{};
    if (live) x = load_rev(rev, j);
    derive_store(live, x, (uint64_t)(mp.first + y) * n_id + j, prep, key_out, mid_out);
}

}  // namespace ace
