// Measurement aid: the INT32 VALU issue rate of the device, the peak the
// verify kernels' roofline is priced against.  Not a step of the method.
//
// Every lane runs eight independent dependency chains of the three 32-bit
// instructions the SHA-256 block computation is made of (v_alignbit_b32,
// v_bitop3_b32, v_add3_u32), 24 VALU instructions per unrolled step.  The
// result is written only when a kernel argument takes a value the host never
// passes, so the compiler keeps every instruction and nothing is stored.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ace {

constexpr uint32_t kValuOpsPerStep = 24;
constexpr uint32_t kValuStepsPerIter = 8;

__global__ void __launch_bounds__(256) k_valu_rate(uint32_t iters, uint32_t seed, uint32_t *sink)
{
    uint32_t a = threadIdx.x ^ seed, b = a * 3u + 1u, c = a * 5u + 7u, d = a ^ 0x5a5a5a5au;
    uint32_t e = a + 11u, f = b ^ 0x3c3c3c3cu, g = c + 13u, h = d * 9u;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (uint32_t k = 0; k < kValuStepsPerIter; ++k) {
            a = __builtin_amdgcn_alignbit(a, b, 7);
            b = __builtin_amdgcn_alignbit(b, c, 11);
            c = __builtin_amdgcn_alignbit(c, d, 13);
            d = __builtin_amdgcn_alignbit(d, e, 17);
            e = __builtin_amdgcn_alignbit(e, f, 19);
            f = __builtin_amdgcn_alignbit(f, g, 23);
            g = __builtin_amdgcn_alignbit(g, h, 25);
            h = __builtin_amdgcn_alignbit(h, a, 29);
            a = __builtin_amdgcn_bitop3_b32(a, c, e, 0x96);
            b = __builtin_amdgcn_bitop3_b32(b, d, f, 0xCA);
            c = __builtin_amdgcn_bitop3_b32(c, e, g, 0xE8);
            d = __builtin_amdgcn_bitop3_b32(d, f, h, 0x96);
            e = __builtin_amdgcn_bitop3_b32(e, g, a, 0xCA);
            f = __builtin_amdgcn_bitop3_b32(f, h, b, 0xE8);
            g = __builtin_amdgcn_bitop3_b32(g, a, c, 0x96);
            h = __builtin_amdgcn_bitop3_b32(h, b, d, 0xCA);
            a = a + b + h;
            b = b + c + a;
            c = c + d + b;
            d = d + e + c;
            e = e + f + d;
            f = f + g + e;
            g = g + h + f;
            h = h + a + g;
        }
    }
    const uint32_t r = a ^ b ^ c ^ d ^ e ^ f ^ g ^ h;
    if (seed == 0xFFFFFFFFu && r == 0x9E3779B9u) sink[0] = r;
}

}  // namespace ace
