// sha256_gfx950.h -- SHA-256 block computation as gfx950 (CDNA4) device code.
//
// One lane owns one hash chain.  The eight working variables and the
// sixteen-word message-schedule window live in VGPRs; round constants are
// scalar operands (SGPRs) of v_add3_u32.  Two forms compute the same block:
// `compress`, fully unrolled with compile-time constants, and
// `compress_looped` (the kernels' default), whose rounds 16..63 run as a
// three-iteration loop fed by one scalar load of sixteen constants per
// iteration, which needs about half the VGPRs.  Per round: 3 v_alignbit_b32 +
// 1 v_bitop3_b32 for each big sigma, 1 v_bitop3_b32 each for Ch and Maj,
// 2 v_add3_u32 for T1, 1 v_add_u32 for e, 1 v_add3_u32 for a; per schedule
// word 2 v_alignbit + 1 v_lshrrev + 1 v_bitop3 per small sigma and
// v_add3 + v_add.  That is 14 x 64 + 10 x 48 + 8 = 1,384 VALU instructions
// per block, the count the throughput accounting uses.
//
// Functions and constants are those of FIPS 180-4 (sec. 4.1.2 and 4.2.2);
// the constant table below is checked against its closed form by the tests.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ace {

// FIPS 180-4 sec. 4.2.2: first 32 bits of the fractional parts of the cube
// roots of the first 64 primes.
static constexpr uint32_t kRound[64] = {
    0x428a2f98u, 0x71374491u, 0xb5c0fbcfu, 0xe9b5dba5u, 0x3956c25bu, 0x59f111f1u, 0x923f82a4u,
    0xab1c5ed5u, 0xd807aa98u, 0x12835b01u, 0x243185beu, 0x550c7dc3u, 0x72be5d74u, 0x80deb1feu,
    0x9bdc06a7u, 0xc19bf174u, 0xe49b69c1u, 0xefbe4786u, 0x0fc19dc6u, 0x240ca1ccu, 0x2de92c6fu,
    0x4a7484aau, 0x5cb0a9dcu, 0x76f988dau, 0x983e5152u, 0xa831c66du, 0xb00327c8u, 0xbf597fc7u,
    0xc6e00bf3u, 0xd5a79147u, 0x06ca6351u, 0x14292967u, 0x27b70a85u, 0x2e1b2138u, 0x4d2c6dfcu,
    0x53380d13u, 0x650a7354u, 0x766a0abbu, 0x81c2c92eu, 0x92722c85u, 0xa2bfe8a1u, 0xa81a664bu,
    0xc24b8b70u, 0xc76c51a3u, 0xd192e819u, 0xd6990624u, 0xf40e3585u, 0x106aa070u, 0x19a4c116u,
    0x1e376c08u, 0x2748774cu, 0x34b0bcb5u, 0x391c0cb3u, 0x4ed8aa4au, 0x5b9cca4fu, 0x682e6ff3u,
    0x748f82eeu, 0x78a5636fu, 0x84c87814u, 0x8cc70208u, 0x90befffau, 0xa4506cebu, 0xbef9a3f7u,
    0xc67178f2u};

// FIPS 180-4 sec. 5.3.3: first 32 bits of the fractional parts of the square
// roots of the first 8 primes.
static constexpr uint32_t kInit[8] = {0x6a09e667u, 0xbb67ae85u, 0x3c6ef372u, 0xa54ff53au,
                                      0x510e527fu, 0x9b05688cu, 0x1f83d9abu, 0x5be0cd19u};

__device__ __forceinline__ uint32_t rotr(uint32_t x, uint32_t n)
{
    return __builtin_amdgcn_alignbit(x, x, n);
}
// v_bitop3_b32 truth tables with operand patterns S0 = 0xF0, S1 = 0xCC, S2 = 0xAA.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t ch(uint32_t e, uint32_t f, uint32_t g)
{
    return __builtin_amdgcn_bitop3_b32(e, f, g, 0xCA);  // e ? f : g
}
__device__ __forceinline__ uint32_t maj(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}
__device__ __forceinline__ uint32_t or_xor(uint32_t acc, uint32_t x, uint32_t y)
{
    return __builtin_amdgcn_bitop3_b32(acc, x, y, 0xF6);  // acc | (x ^ y)
}
__device__ __forceinline__ uint32_t big_sigma0(uint32_t x) { return xor3(rotr(x, 2), rotr(x, 13), rotr(x, 22)); }
__device__ __forceinline__ uint32_t big_sigma1(uint32_t x) { return xor3(rotr(x, 6), rotr(x, 11), rotr(x, 25)); }
__device__ __forceinline__ uint32_t small_sigma0(uint32_t x) { return xor3(rotr(x, 7), rotr(x, 18), x >> 3); }
__device__ __forceinline__ uint32_t small_sigma1(uint32_t x) { return xor3(rotr(x, 17), rotr(x, 19), x >> 10); }

// Byte swap of a 32-bit word (big-endian message words, FIPS 180-4 sec. 3.1).
__device__ __forceinline__ uint32_t bswap32(uint32_t x) { return __builtin_amdgcn_perm(0u, x, 0x00010203u); }

struct State {
    uint32_t h[8];
};

__device__ __forceinline__ State initial_state()
{
    State s;
#pragma unroll
    for (int i = 0; i < 8; ++i) s.h[i] = kInit[i];
    return s;
}

// s <- s + rounds(s, W) for one 16-word block (W is consumed as the schedule
// window and left holding W[48..63]).
__device__ __forceinline__ void compress(State &s, uint32_t (&W)[16])
{
    uint32_t a = s.h[0], b = s.h[1], c = s.h[2], d = s.h[3];
    uint32_t e = s.h[4], f = s.h[5], g = s.h[6], h = s.h[7];
#pragma unroll
    for (int t = 0; t < 64; ++t) {
        uint32_t wt;
        if (t < 16) {
            wt = W[t];
        } else {
            wt = small_sigma1(W[(t - 2) & 15]) + W[(t - 7) & 15] + small_sigma0(W[(t - 15) & 15]) +
                 W[t & 15];
            W[t & 15] = wt;
        }
        const uint32_t t1 = (h + wt + kRound[t]) + (big_sigma1(e) + ch(e, f, g));
        const uint32_t t2 = big_sigma0(a) + maj(a, b, c);
        h = g; g = f; f = e; e = d + t1;
        d = c; c = b; b = a; a = t1 + t2;
    }
    s.h[0] += a; s.h[1] += b; s.h[2] += c; s.h[3] += d;
    s.h[4] += e; s.h[5] += f; s.h[6] += g; s.h[7] += h;
}

// The same block computation with rounds 16..63 as a three-iteration loop of
// sixteen rounds.  Their constants come from one scalar load of sixteen words
// per iteration; the loop boundary keeps the scheduler from interleaving all
// 64 rounds, which roughly halves the VGPRs a lane needs (more waves per SIMD)
// at the same 1,384 VALU instructions per block.
__constant__ __attribute__((aligned(64))) uint32_t kRoundTable[64] = {
    0x428a2f98u, 0x71374491u, 0xb5c0fbcfu, 0xe9b5dba5u, 0x3956c25bu, 0x59f111f1u, 0x923f82a4u,
    0xab1c5ed5u, 0xd807aa98u, 0x12835b01u, 0x243185beu, 0x550c7dc3u, 0x72be5d74u, 0x80deb1feu,
    0x9bdc06a7u, 0xc19bf174u, 0xe49b69c1u, 0xefbe4786u, 0x0fc19dc6u, 0x240ca1ccu, 0x2de92c6fu,
    0x4a7484aau, 0x5cb0a9dcu, 0x76f988dau, 0x983e5152u, 0xa831c66du, 0xb00327c8u, 0xbf597fc7u,
    0xc6e00bf3u, 0xd5a79147u, 0x06ca6351u, 0x14292967u, 0x27b70a85u, 0x2e1b2138u, 0x4d2c6dfcu,
    0x53380d13u, 0x650a7354u, 0x766a0abbu, 0x81c2c92eu, 0x92722c85u, 0xa2bfe8a1u, 0xa81a664bu,
    0xc24b8b70u, 0xc76c51a3u, 0xd192e819u, 0xd6990624u, 0xf40e3585u, 0x106aa070u, 0x19a4c116u,
    0x1e376c08u, 0x2748774cu, 0x34b0bcb5u, 0x391c0cb3u, 0x4ed8aa4au, 0x5b9cca4fu, 0x682e6ff3u,
    0x748f82eeu, 0x78a5636fu, 0x84c87814u, 0x8cc70208u, 0x90befffau, 0xa4506cebu, 0xbef9a3f7u,
    0xc67178f2u};

struct RoundConsts16 {
    uint32_t k[16];
};

__device__ __forceinline__ void round_step(uint32_t &a, uint32_t &b, uint32_t &c, uint32_t &d,
                                           uint32_t &e, uint32_t &f, uint32_t &g, uint32_t &h,
                                           uint32_t wt, uint32_t kt)
{
    const uint32_t t1 = (h + wt + kt) + (big_sigma1(e) + ch(e, f, g));
    const uint32_t t2 = big_sigma0(a) + maj(a, b, c);
    h = g; g = f; f = e; e = d + t1;
    d = c; c = b; b = a; a = t1 + t2;
}

__device__ __forceinline__ void compress_looped(State &s, uint32_t (&W)[16])
{
    uint32_t a = s.h[0], b = s.h[1], c = s.h[2], d = s.h[3];
    uint32_t e = s.h[4], f = s.h[5], g = s.h[6], h = s.h[7];
#pragma unroll
    for (int j = 0; j < 16; ++j) round_step(a, b, c, d, e, f, g, h, W[j], kRound[j]);
#pragma nounroll
    for (int q = 1; q < 4; ++q) {
        const RoundConsts16 kq = *reinterpret_cast<const RoundConsts16 *>(&kRoundTable[16 * q]);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const uint32_t wt = small_sigma1(W[(j - 2) & 15]) + W[(j - 7) & 15] +
                                small_sigma0(W[(j - 15) & 15]) + W[j];
            W[j] = wt;
            round_step(a, b, c, d, e, f, g, h, wt, kq.k[j]);
        }
    }
    s.h[0] += a; s.h[1] += b; s.h[2] += c; s.h[3] += d;
    s.h[4] += e; s.h[5] += f; s.h[6] += g; s.h[7] += h;
}

// The looped form with rounds 16..31 unrolled as well, for blocks whose
// words 8..15 are constants at the call site (an HMAC block over a 32-byte
// digest, a key block's pad bytes): those words then fold into the first
// sixteen schedule words instead of being computed on (zero words drop out
// of the sums, sigma0 of a constant is a constant).
__device__ __forceinline__ void compress_fold(State &s, uint32_t (&W)[16])
{
    uint32_t a = s.h[0], b = s.h[1], c = s.h[2], d = s.h[3];
    uint32_t e = s.h[4], f = s.h[5], g = s.h[6], h = s.h[7];
#pragma unroll
    for (int j = 0; j < 16; ++j) round_step(a, b, c, d, e, f, g, h, W[j], kRound[j]);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t wt = small_sigma1(W[(j - 2) & 15]) + W[(j - 7) & 15] +
                            small_sigma0(W[(j - 15) & 15]) + W[j];
        W[j] = wt;
        round_step(a, b, c, d, e, f, g, h, wt, kRound[16 + j]);
    }
#pragma nounroll
    for (int q = 2; q < 4; ++q) {
        const RoundConsts16 kq = *reinterpret_cast<const RoundConsts16 *>(&kRoundTable[16 * q]);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const uint32_t wt = small_sigma1(W[(j - 2) & 15]) + W[(j - 7) & 15] +
                                small_sigma0(W[(j - 15) & 15]) + W[j];
            W[j] = wt;
            round_step(a, b, c, d, e, f, g, h, wt, kq.k[j]);
        }
    }
    s.h[0] += a; s.h[1] += b; s.h[2] += c; s.h[3] += d;
    s.h[4] += e; s.h[5] += f; s.h[6] += g; s.h[7] += h;
}

#ifndef ACE_COMPRESS_LOOPED
#define ACE_COMPRESS_LOOPED 1
#endif

// The block computation the kernels use.
__device__ __forceinline__ void compress_block(State &s, uint32_t (&W)[16])
{
#if ACE_COMPRESS_LOOPED
    compress_looped(s, W);
#else
    compress(s, W);
#endif
}

}  // namespace ace
