// chain_kernels.hip -- segments of the SHA-256 hash chain the consensus
// section uses as its clock.  Included by ace_api.hip after ace_kernels.hip.

namespace ace {

// ------------------------------------------------------------------------------------------
// Hash-chain segments (the consensus section's clock: H_{i+1} = SHA-256(H_i)
// over the 32 digest bytes).  One segment per lane: steps[i] single-block
// hashes from start[i], compared with end[i].
// ------------------------------------------------------------------------------------------
__global__ void k_poh_zero(unsigned long long *count) { *count = 0; }

__global__ void __launch_bounds__(kWG) ACE_WAVES(8) k_poh_verify(const uint8_t *__restrict__ start,
                                                   const uint8_t *__restrict__ end,
                                                   const uint32_t *__restrict__ steps,
                                                   uint32_t uniform_steps, uint64_t n,
                                                   uint32_t *__restrict__ bitmask,
                                                   unsigned long long *__restrict__ count)
{
    const uint64_t i0 = 64ull * ((uint64_t)blockIdx.x * kWavesPerWG + (threadIdx.x >> 6));
    if (i0 >= n) return;  // whole wave past the end
    const uint64_t i = i0 + lane_id();
    const bool live = i < n;
    State h;
    uint32_t T = 0;
    if (live) {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(start + 32ull * i);
        const U4 a = load16(p), b = load16(p + 4);
        h.h[0] = bswap32(a.x); h.h[1] = bswap32(a.y); h.h[2] = bswap32(a.z); h.h[3] = bswap32(a.w);
        h.h[4] = bswap32(b.x); h.h[5] = bswap32(b.y); h.h[6] = bswap32(b.z); h.h[7] = bswap32(b.w);
        T = steps ? steps[i] : uniform_steps;
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) h.h[k] = 0;
    }
    for (uint32_t t = 0;; ++t) {
        const bool run = live && t < T;
        if (__ballot(run) == 0) break;
        if (run) {
            // the 32-byte value, 0x80, zeros, bit length 256: one block
            uint32_t W[16];
#pragma unroll
            for (int k = 0; k < 8; ++k) W[k] = h.h[k];
            W[8] = 0x80000000u;
#pragma unroll
            for (int k = 9; k < 15; ++k) W[k] = 0u;
            W[15] = 256u;
            State s = initial_state();
            compress_fold(s, W);  // words 8..15 are constants
            h = s;
        }
    }
    bool ok = false;
    if (live) {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(end + 32ull * i);
        const U4 a = load16(p), b = load16(p + 4);
        uint32_t d = 0;
        d = or_xor(d, h.h[0], bswap32(a.x)); d = or_xor(d, h.h[1], bswap32(a.y));
        d = or_xor(d, h.h[2], bswap32(a.z)); d = or_xor(d, h.h[3], bswap32(a.w));
        d = or_xor(d, h.h[4], bswap32(b.x)); d = or_xor(d, h.h[5], bswap32(b.y));
        d = or_xor(d, h.h[6], bswap32(b.z)); d = or_xor(d, h.h[7], bswap32(b.w));
        ok = d == 0;
    }
    const unsigned long long m = __ballot(ok);
    if (lane_id() == 0) {
        bitmask[i0 >> 5] = (uint32_t)m;
        if (i0 + 32 < n) bitmask[(i0 >> 5) + 1] = (uint32_t)(m >> 32);
        const unsigned c = __popcll(m);
        if (c) atomicAdd(count, (unsigned long long)c);
    }
}

}  // namespace ace
