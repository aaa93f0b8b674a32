// ace_kernels.hip -- gfx950 kernels of the attestation check.
//
//   k_zero           clears the per-block counts and the binning control words.
//   k_bin_count      histogram of transactions by inner block count.
//   k_bin_scan       bin start positions, longest messages first.
//   k_bin_scatter    transaction records into bin order.
//   k_verify         Alg. 1 Phase 1a per transaction: inner hash of the message
//                    from the cached ipad midstate, outer hash from the opad
//                    midstate, constant-time compare with the credential,
//                    wave64 ballot of the verdicts (also the paper's
//                    attestation form, Def. 3.1 with Alg. 2's payload binding).
//   k_finalize       bin-order verdicts back to input order.
//   k_count          valid counts from the finished bitmasks.
//   k_plan           device-side plan of a graph replay.
// The key derivation (Def. 2.1) is in hkdf_kernels.hip, the hash-chain
// segments in chain_kernels.hip, the Merkle roots in merkle_kernels.hip.
//
// One transaction per lane.  Message bytes are read straight from HBM as
// aligned dwords and turned into big-endian schedule words with one
// v_perm_b32 each, whose per-lane selector also absorbs the message's byte
// misalignment; the padding (0x80, zeros, bit length) is applied on the fly
// in the last one or two blocks of each message.
#include "ace_internal.h"
#include "sha256_gfx950.h"

namespace ace {

// ------------------------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

// Loads from 4-byte aligned addresses in device memory, issued as global
// (not flat) loads: they then count only against the vector memory counter,
// so waiting for the round constants' scalar loads does not also wait for
// them.
typedef const __attribute__((address_space(1))) uint32_t *gptr;
__device__ __forceinline__ U4 load16(const uint32_t *p)
{
    const gptr g = (gptr)p;
    U4 v;
    v.x = g[0]; v.y = g[1]; v.z = g[2]; v.w = g[3];
    return v;
}
__device__ __forceinline__ uint32_t load32(const uint32_t *p) { return *(gptr)p; }

// Block count and totals of a call: kernel arguments, or the device header
// of a graph replay.
struct Totals {
    uint32_t n_blocks;
    bool inline_one;
    uint64_t tx, tiles, waves;
};

// The same value in every lane, made visible to the compiler as such, so
// that loops bounded by it stay scalar.
__device__ __forceinline__ uint32_t uniform32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    return ((uint64_t)uniform32((uint32_t)(v >> 32)) << 32) | uniform32((uint32_t)v);
}

__device__ __forceinline__ Totals totals(const Batch &bt)
{
    Totals t;
    if (bt.hdr) {
        // one header read by every lane at the same address
        t.n_blocks = uniform32(bt.hdr->n_blocks);
        t.tx = uniform64(bt.hdr->total_tx);
        t.tiles = uniform64(bt.hdr->total_tiles);
        t.waves = uniform64(bt.hdr->total_waves);
        t.inline_one = false;
    } else {
        t.n_blocks = bt.n_blocks;
        t.tx = bt.total_tx;
        t.tiles = bt.total_tiles;
        t.waves = bt.total_waves;
        t.inline_one = bt.n_blocks == 1;
    }
    return t;
}

__device__ __forceinline__ DevBlock get_block(const Batch &bt, const Totals &T, uint32_t b)
{
    if (T.inline_one) return bt.one;
    return bt.table[b];
}

// Last block whose prefix (selected by `field`) is <= x; empty blocks share
// their prefix with the next block, so the last match is the owner.
template <int FIELD>
__device__ __forceinline__ uint32_t find_block(const Batch &bt, const Totals &T, uint64_t x)
{
    if (T.n_blocks == 1) return 0;
    uint32_t lo = 0, hi = T.n_blocks;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        const DevBlock &d = bt.table[mid];
        const uint64_t v = FIELD == 0 ? d.tile0 : d.wave0;
        if (v <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

}  // namespace ace

#include "hkdf_kernels.hip"

namespace ace {

// ------------------------------------------------------------------------------------------
// Verification of one transaction per lane.
// ------------------------------------------------------------------------------------------
struct TxRef {
    const uint8_t *msg;   // message start
    uint64_t L;           // message length
    const uint32_t *mid;  // midstate row (ipad 0..7, opad 8..15), if cached
    const uint8_t *rev;   // root entropy row, if derived per transaction
    const uint8_t *tag;   // credential
    bool overread_ok;     // reading up to kOverread bytes past the message end stays in its block
};

// Bytes of a transaction's check record: its credential (HMAC form), or its
// attestation obj_hash (32) || domain (8) || credential (32) (paper form of
// Def. 3.1, with the payload as the message).
template <bool ATTEST>
constexpr uint32_t check_stride() { return ATTEST ? 72u : 32u; }

// The 17 dwords from dword 16 b of a message's aligned area: the 64 bytes of
// message block b after the alignment shift, plus the next dword.  Either the
// loads stay within kOverread bytes past the message end inside the block's
// message area (overread_ok), or every address is clamped to a dword that
// holds message bytes: nothing outside the caller's buffers is touched, and
// bytes past the message end only feed words the padding overwrites.
__device__ __forceinline__ void load_window(uint32_t (&D)[17], const uint32_t *q, int64_t rb,
                                            bool overread_ok, const uint32_t *A0, uint64_t last,
                                            uint32_t b)
{
    if (overread_ok || rb >= 68) {
        // whole 16-byte loads and dword 16 (with 68 message bytes left every
        // dword holds some)
        const U4 v0 = load16(q), v1 = load16(q + 4), v2 = load16(q + 8), v3 = load16(q + 12);
        D[0] = v0.x; D[1] = v0.y; D[2] = v0.z; D[3] = v0.w;
        D[4] = v1.x; D[5] = v1.y; D[6] = v1.z; D[7] = v1.w;
        D[8] = v2.x; D[9] = v2.y; D[10] = v2.z; D[11] = v2.w;
        D[12] = v3.x; D[13] = v3.y; D[14] = v3.z; D[15] = v3.w;
        D[16] = load32(q + 16);
    } else {
        // the last message before the end of its block's area
#pragma unroll
        for (int k = 0; k < 17; ++k) {
            const uint64_t idx = 16ull * b + k;
            D[k] = load32(A0 + (idx < last ? idx : last));
        }
        // keeps these loads in this branch: merged with the other branch's
        // they became 17 dword loads on the common path
        __asm__ volatile("" ::: "memory");
    }
}

// Where a lane's message blocks come from and how the last one is padded.
struct LaneGeom {
    uint32_t nb;         // message blocks (0 for a dead lane)
    uint32_t sel;        // byte selector of the alignment shift, big-endian
    const uint32_t *A0;  // dword-aligned start of the message area
    uint64_t last;       // last dword index that holds message bytes
    uint32_t len_hi, len_lo;  // bit length in the final block
};

template <bool ATTEST>
__device__ __forceinline__ LaneGeom lane_geom(bool live, const TxRef &t)
{
    LaneGeom g;
    const uint64_t L = t.L;
    g.nb = live ? (uint32_t)((L + 9 + 63) >> 6) : 0u;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(t.msg);
    const uint32_t sh = (uint32_t)addr & 3u;
    g.sel = 0x00010203u + sh * 0x01010101u;  // bytes sh..sh+3 of {hi:lo}, big-endian
    const uint64_t lim = (uint64_t)sh + L;   // dword k holds message bytes iff 4k < lim
    g.last = lim ? ((lim - 1) >> 2) : 0;
    // an empty message without overread room reads its dwords from the check
    // record (bytes the padding overwrites)
    g.A0 = (lim || t.overread_ok) ? reinterpret_cast<const uint32_t *>(addr - sh)
                                  : reinterpret_cast<const uint32_t *>(t.tag);
    // the HMAC inner hash counts the 64-byte key block before the message
    const uint64_t bits = ((ATTEST ? 0 : 64) + L) << 3;
    g.len_hi = (uint32_t)(bits >> 32);
    g.len_lo = (uint32_t)bits;
    return g;
}

// Loads of the windows of N consecutive blocks from q: 16 N + 1 dwords.
template <int N, int K>
__device__ __forceinline__ void load_windows(uint32_t (&D)[16 * K + 1], const uint32_t *q)
{
#pragma unroll
    for (int c = 0; c < 4 * N; ++c) {
        const U4 v = load16(q + 4 * c);
        D[4 * c] = v.x; D[4 * c + 1] = v.y; D[4 * c + 2] = v.z; D[4 * c + 3] = v.w;
    }
    D[16 * N] = load32(q + 16 * N);
}

// Schedule words of the window in slot S (dwords 16 S .. 16 S + 16).
template <int S, int K>
__device__ __forceinline__ void window_words(uint32_t (&W)[16], const uint32_t (&D)[16 * K + 1],
                                             uint32_t sel)
{
#pragma unroll
    for (int j = 0; j < 16; ++j) W[j] = __builtin_amdgcn_perm(D[16 * S + j + 1], D[16 * S + j], sel);
}

// The message blocks of one lane, chained onto S.  The windows of up to K
// consecutive blocks come in one load of 16 K + 1 dwords (K blocks touch
// about 1 + (64 K + 3) / 128 cache lines together instead of about 1.5 each),
// and the following blocks take their windows from the registers holding
// them.  A group of K windows is loaded when K blocks remain, else a pair,
// else one window; a group may read at most 76 bytes past the message end
// (its last block exists, so at least 64 (K - 2) + 56 message bytes are
// left), which the caller allows (overread_ok) or the message covers.  The
// first group is loaded before the block loop, so its loads are in flight
// together with the caller's midstate loads (inside the loop the compiler
// waited for all outstanding loads before issuing a group's).  Lanes of one
// wave share their block count (same bin), so the branches below are uniform
// in the binned kernels.
template <int K>
__device__ __forceinline__ void message_blocks(State &S, bool live, bool overread_ok, const LaneGeom &g,
                                               int64_t L)
{
    static_assert(K >= 2 && K <= 3, "groups of two or three windows");
    // a do-while with the wave's vote at the end: with the vote at the top the
    // state was copied twice per block
    const uint32_t *q = g.A0;  // dword 16 b of the message area, advanced per block
    int64_t rb = L;            // message bytes from this block on
    uint32_t b = 0;
    bool run = live;           // a live lane has at least one block
    uint32_t slot = 0;         // slot of this block's window in D
    uint32_t D[16 * K + 1];
    uint32_t avail = 0;        // windows of this and later blocks already in D
    if (run) {
        // the first group before the loop: its loads go out with the midstate loads
        const uint32_t left = g.nb;
        uint32_t m = 1;
        if (left >= (uint32_t)K && (overread_ok || rb >= 64 * (K - 1) + 68)) m = K;
        else if (left >= 2 && (overread_ok || rb >= 132)) m = 2;
        if (m == (uint32_t)K) load_windows<K, K>(D, q);
        else if (m == 2) load_windows<2, K>(D, q);
        else {
            uint32_t E[17];
            load_window(E, q, rb, overread_ok, g.A0, g.last, 0);
#pragma unroll
            for (int j = 0; j < 17; ++j) D[j] = E[j];
        }
        avail = m;
    }
    if (__ballot(run)) do {
        if (run) {
            uint32_t W[16];
            if (avail == 0) {
                const uint32_t left = g.nb - b;
                uint32_t m = 1;
                if (left >= (uint32_t)K && (overread_ok || rb >= 64 * (K - 1) + 68)) m = K;
                else if (left >= 2 && (overread_ok || rb >= 132)) m = 2;
                if (m == (uint32_t)K) {
                    load_windows<K, K>(D, q);
                } else if (m == 2) {
                    load_windows<2, K>(D, q);
                } else {
                    uint32_t E[17];
                    load_window(E, q, rb, overread_ok, g.A0, g.last, b);
#pragma unroll
                    for (int j = 0; j < 17; ++j) D[j] = E[j];
                }
                avail = m;
                slot = 0;
            }
            if (slot == 0) window_words<0, K>(W, D, g.sel);
            else if (K == 2 || slot == 1) window_words<1, K>(W, D, g.sel);
            else window_words<K - 1, K>(W, D, g.sel);
            ++slot;
            --avail;
            if (rb < 64) {
                // padding: word jf holds byte rb (the 0x80 marker) after its c
                // message bytes; earlier words are message, later ones zero.
                // In the last block the marker is in words 0..13 (or was in the
                // block before: jf < 0) and words 14..15 hold the bit length;
                // in a block before it, the message fills 56..63 bytes, so only
                // words 14..15 change.  (Lanes of a binned wave share their
                // block count, so one of the two branches runs per block.)
                const int32_t r0 = (int32_t)rb;
                const int32_t jf = r0 >> 2;   // negative: the marker was in the previous block
                const uint32_t c8 = ((uint32_t)r0 & 3u) << 3;
                const uint32_t keep = ~(0xFFFFFFFFu >> c8);
                const uint32_t pad = 0x80000000u >> c8;
                if (b + 1 == g.nb) {
#pragma unroll
                    for (int j = 0; j < 14; ++j) {
                        const uint32_t part = (W[j] & keep) | pad;
                        W[j] = j < jf ? W[j] : (j == jf ? part : 0u);
                    }
                    W[14] = g.len_hi;
                    W[15] = g.len_lo;
                } else {
#pragma unroll
                    for (int j = 14; j < 16; ++j) {
                        const uint32_t part = (W[j] & keep) | pad;
                        W[j] = j < jf ? W[j] : (j == jf ? part : 0u);
                    }
                }
            }
            compress_block(S, W);
        }
        ++b; q += 16; rb -= 64;
        run = live && b < g.nb;
    } while (__ballot(run) != 0);
}

// Dwords of a transaction's check record: the credential (HMAC form), or
// obj_hash (8) || domain (2) || credential (8) (paper form of Def. 3.1, with
// the payload as the message).
template <bool ATTEST>
constexpr int check_words() { return ATTEST ? 18 : 8; }

template <bool ATTEST>
__device__ __forceinline__ void load_check(const uint8_t *tag, uint32_t (&C)[check_words<ATTEST>()])
{
    const uint32_t *p = reinterpret_cast<const uint32_t *>(tag);
    const U4 a = load16(p), c = load16(p + 4);
    C[0] = a.x; C[1] = a.y; C[2] = a.z; C[3] = a.w;
    C[4] = c.x; C[5] = c.y; C[6] = c.z; C[7] = c.w;
    if constexpr (ATTEST) {
        const U4 e = load16(p + 8), f = load16(p + 12);
        C[8] = e.x; C[9] = e.y; C[10] = e.z; C[11] = e.w;
        C[12] = f.x; C[13] = f.y; C[14] = f.z; C[15] = f.w;
        C[16] = load32(p + 16); C[17] = load32(p + 17);
    }
}

// After the message blocks: S is the HMAC inner state (HMAC form) or
// SHA-256(P) (paper form).  Paper form: compare S with obj_hash, then the
// HMAC inner block over obj_hash || domain (40 bytes, bit length
// (64 + 40) * 8).  Both: the outer hash F(opad, inner digest || 0x80 || 0 ||
// 768) and the constant-time compare with the credential.
// FOLD: the fixed-form blocks use compress_fold (50 fewer VALU per block, a
// few more registers; kernels at their register limit keep the plain form).
template <bool FOLD>
__device__ __forceinline__ void compress_tail_block(State &s, uint32_t (&W)[16])
{
    if constexpr (FOLD) compress_fold(s, W);
    else compress_block(s, W);
}

template <bool ATTEST, bool FOLD>
__device__ __forceinline__ bool lane_result(bool live, State S, const State &ipad, const State &opad,
                                            const uint32_t (&C)[check_words<ATTEST>()])
{
    uint32_t d = 0;
    if constexpr (ATTEST) {
        uint32_t W[16];
#pragma unroll
        for (int i = 0; i < 10; ++i) W[i] = bswap32(C[i]);
#pragma unroll
        for (int i = 0; i < 8; ++i) d = or_xor(d, S.h[i], W[i]);
        W[10] = 0x80000000u;
#pragma unroll
        for (int i = 11; i < 15; ++i) W[i] = 0u;
        W[15] = (64u + 40u) * 8u;
        State T = ipad;
        compress_tail_block<FOLD>(T, W);
        S = T;
    }
    {
        uint32_t W[16];
#pragma unroll
        for (int i = 0; i < 8; ++i) W[i] = S.h[i];
        W[8] = 0x80000000u;
#pragma unroll
        for (int i = 9; i < 15; ++i) W[i] = 0u;
        W[15] = 768u;
        State T = opad;
        compress_tail_block<FOLD>(T, W);
        S = T;
    }
    constexpr int c0 = ATTEST ? 10 : 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) d = or_xor(d, S.h[i], bswap32(C[c0 + i]));
    return live && d == 0;
}

__device__ __forceinline__ void load_midstates(const uint32_t *mid, uint32_t (&M)[16])
{
    // both halves of the 64-byte row at once: one cache line, fetched once
    const U4 a = load16(mid), b = load16(mid + 4), c = load16(mid + 8), e = load16(mid + 12);
    M[0] = a.x; M[1] = a.y; M[2] = a.z; M[3] = a.w; M[4] = b.x; M[5] = b.y; M[6] = b.z; M[7] = b.w;
    M[8] = c.x; M[9] = c.y; M[10] = c.z; M[11] = c.w; M[12] = e.x; M[13] = e.y; M[14] = e.z; M[15] = e.w;
}

// HMAC form: valid iff HMAC(k, msg) == credential.
// Paper form (ATTEST): the message is the payload P; valid iff SHA-256(P) ==
// obj_hash (payload binding) and HMAC(k, obj_hash || domain) == credential.
template <bool PER_TX_KEYS, bool ATTEST, bool FOLD>
__device__ __forceinline__ bool verify_lane(bool live, const TxRef &t, const HkdfPrep *prep)
{
    State ipad, opad;
#pragma unroll
    for (int i = 0; i < 8; ++i) { ipad.h[i] = 0; opad.h[i] = 0; }
    if constexpr (PER_TX_KEYS) {
        uint32_t rv[8];
        if (live) {
            const uint32_t *p = reinterpret_cast<const uint32_t *>(t.rev);
            const U4 a = load16(p), b = load16(p + 4);
            rv[0] = bswap32(a.x); rv[1] = bswap32(a.y); rv[2] = bswap32(a.z); rv[3] = bswap32(a.w);
            rv[4] = bswap32(b.x); rv[5] = bswap32(b.y); rv[6] = bswap32(b.z); rv[7] = bswap32(b.w);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) rv[i] = 0;
        }
        uint32_t key[8];
        derive_lane(live, rv, *prep, key, ipad, opad);
    } else {
        if (live) {
            uint32_t M[16];
            load_midstates(t.mid, M);
#pragma unroll
            for (int i = 0; i < 8; ++i) { ipad.h[i] = M[i]; opad.h[i] = M[8 + i]; }
        }
    }
    // the message chain starts from the ipad state (HMAC inner hash) or, for
    // the payload digest, from the initial value
    State S = ATTEST ? initial_state() : ipad;
    const LaneGeom g = lane_geom<ATTEST>(live, t);
    // three windows per load where the registers allow it; the per-transaction
    // derivation's state leaves room for two
    message_blocks<PER_TX_KEYS ? 2 : 3>(S, live, t.overread_ok, g, (int64_t)t.L);
    uint32_t C[check_words<ATTEST>()];
#pragma unroll
    for (int i = 0; i < check_words<ATTEST>(); ++i) C[i] = 0;
    if (live) load_check<ATTEST>(t.tag, C);
    return lane_result<ATTEST, FOLD>(live, S, ipad, opad, C);
}

// Loads what one lane needs about transaction i of block d.  Returns whether
// the transaction can be valid at all (registered identity, ordered offsets).
template <bool ATTEST>
__device__ __forceinline__ bool load_tx(const DevBlock &d, uint64_t i, const KeySource &ks, TxRef &t)
{
    const uint64_t a = d.off[i], e = d.off[i + 1];
    const uint32_t who = d.id[i];
    const bool ok = who < ks.n_id && a <= e;
    t.msg = d.msg + a;
    t.L = ok ? e - a : 0;
    t.mid = ks.mid ? ks.mid + 16ull * (ok ? who : 0u) : nullptr;
    t.rev = ks.rev ? ks.rev + 32ull * (ok ? who : 0u) : nullptr;
    t.tag = d.tag + (uint64_t)check_stride<ATTEST>() * i;
    t.overread_ok = ok && e + kOverread <= d.off[d.n];
    return ok;
}

// ------------------------------------------------------------------------------------------
// k_verify, in-order form: wave tile w covers transactions 64w' .. 64w'+63 of
// one block; the ballot is that block's two bitmask words.
// ------------------------------------------------------------------------------------------
template <bool PER_TX_KEYS, bool ATTEST>
__global__ void __launch_bounds__(kWG) ACE_WAVES(4) k_verify_ordered(Batch bt, KeySource ks, HkdfParams hp)
{
    __shared__ HkdfPrep prep;
    if constexpr (PER_TX_KEYS) {
        if (threadIdx.x < 64) hkdf_prepare(hp, prep);
        __syncthreads();
    }
    const Totals T = totals(bt);
    // grid-stride over wave tiles (wave-uniform loop bound)
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint64_t w = (uint64_t)blockIdx.x * kWavesPerWG + wave; w < T.waves;
         w += (uint64_t)gridDim.x * kWavesPerWG) {
        const uint32_t b = find_block<1>(bt, T, w);
        const DevBlock d = get_block(bt, T, b);
        const uint64_t i0 = 64ull * (w - d.wave0);
        const uint64_t i = i0 + lane_id();
        const bool active = i < d.n;
        TxRef t{};
        bool live = false;
        if (active) live = load_tx<ATTEST>(d, i, ks, t);
        const bool valid = verify_lane<PER_TX_KEYS, ATTEST, !ATTEST>(live, t, &prep) && live;
        const unsigned long long m = __ballot(valid);
        if (lane_id() == 0) {
            d.bitmask[i0 >> 5] = (uint32_t)m;
            if (i0 + 32 < d.n) d.bitmask[(i0 >> 5) + 1] = (uint32_t)(m >> 32);
        }
    }
}

// ------------------------------------------------------------------------------------------
// Binning by inner block count.  Three passes over the batch's tiles of kTile
// transactions: k_bin_count writes each tile's bin histogram into the table
// thist[bin][tile]; k_bin_scan turns every bin's row into exclusive prefixes
// over the tiles and stores the bin totals; k_bin_scatter then knows where each
// tile's transactions of each bin go without any global atomic: bins laid out
// longest first, each padded to a multiple of 64, tiles in order within a bin.
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kWG) k_zero(Batch bt, Ctrl *ctrl)
{
    const Totals T = totals(bt);
    const uint32_t t = blockIdx.x * kWG + threadIdx.x;
    for (uint32_t b = t; b < T.n_blocks; b += gridDim.x * kWG) *get_block(bt, T, b).count = 0;
    if (ctrl && blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->total_pos = 0;
        ctrl->work = 0;
    }
}

// A tile's offsets and identities as the binning passes read them: thread t
// holds transactions i0 + t + k kWG, k < kPer.  A workgroup loads its next
// tile into a second TileTx while it bins the current one, so its loads stay
// in flight across the tile's LDS atomics, barriers and stores (one tile at a
// time, the passes' waves spent most of their cycles waiting on loads).
constexpr int kPer = kTile / kWG;

struct TileTx {
    uint64_t a[kPer], e[kPer];
    uint32_t who[kPer];
};

// Every lane loads (past the block's last transaction it reloads that one,
// which the caller then ignores): with loads under a branch the compiler
// waited for all of them, the next tile's included, before using any.
// (Global, not flat, loads: they count only against the vector memory
// counter, so LDS accesses do not wait for them.)
typedef const __attribute__((address_space(1))) uint64_t *gptr64;

__device__ __forceinline__ void load_tile_tx(const DevBlock &d, uint64_t i0, TileTx &x)
{
    const gptr64 off = (gptr64)d.off;
    const gptr id = (gptr)d.id;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const uint64_t i = i0 + threadIdx.x + (uint64_t)k * kWG;
        const uint64_t j = i < d.n ? i : d.n - 1;  // a tile's block holds at least one transaction
        x.a[k] = off[j];
        x.e[k] = off[j + 1];
        x.who[k] = id[j];
    }
}

// Length used for binning: transactions that cannot be valid hash nothing.
__device__ __forceinline__ uint64_t tx_length(uint64_t a, uint64_t e, uint32_t who, uint32_t n_id)
{
    return (a <= e && who < n_id) ? e - a : 0;
}

__global__ void __launch_bounds__(kWG) k_bin_count(Batch bt, uint32_t *__restrict__ thist,
                                                   uint64_t tstride, uint32_t n_id)
{
    __shared__ uint32_t h[kBins];
    // The binning passes run beside the key derivation (the caller's
    // stream and the second one): their waves, mostly waiting on memory,
    // issue first whenever they are ready, and the derivation's waves take
    // the remaining issue slots.
    __builtin_amdgcn_s_setprio(3);
    const Totals T = totals(bt);
    if (blockIdx.x >= T.tiles) return;  // the whole workgroup
    // Two buffers used in turn (the loop body twice, no copies between them):
    // the tile in one is binned while the next tile's loads fill the other.
    TileTx xa, xb;
    DevBlock da = get_block(bt, T, find_block<0>(bt, T, blockIdx.x)), db;
    uint64_t ta = blockIdx.x, tb;
    load_tile_tx(da, (ta - da.tile0) * kTile, xa);
    // bins tile t (block d, loads x) while tile `nt` (the last tile: t again,
    // unused) loads into y; returns whether there was a next tile
    auto step = [&](const TileTx &x, const DevBlock &d, uint64_t t, TileTx &y, DevBlock &dn,
                    uint64_t &nt) -> bool {
        const bool more = t + gridDim.x < T.tiles;  // uniform
        nt = more ? t + gridDim.x : t;
        dn = get_block(bt, T, find_block<0>(bt, T, nt));
        load_tile_tx(dn, (nt - dn.tile0) * kTile, y);
        if (threadIdx.x < kBins) h[threadIdx.x] = 0;
        __syncthreads();
        const uint64_t i0 = (t - d.tile0) * kTile;
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (i0 + threadIdx.x + (uint64_t)k * kWG < d.n)
                atomicAdd(&h[bin_of_length(tx_length(x.a[k], x.e[k], x.who[k], n_id))], 1u);
        __syncthreads();
        if (threadIdx.x < kBins) thist[threadIdx.x * tstride + t] = h[threadIdx.x];
        __syncthreads();
        return more;
    };
    for (;;) {
        if (!step(xa, da, ta, xb, db, tb)) break;
        if (!step(xb, db, tb, xa, da, ta)) break;
    }
}

// One workgroup per bin: the bin's per-tile counts become exclusive prefixes
// (in place), and the bin's total goes to ctrl->bincount.
constexpr int kScanWG = 1024;
__global__ void __launch_bounds__(kScanWG) k_bin_scan(Batch bt, Ctrl *ctrl,
                                                      uint32_t *__restrict__ thist, uint64_t tstride)
{
    __shared__ uint32_t part[kScanWG];
    __builtin_amdgcn_s_setprio(3);  // as in k_bin_count
    const uint32_t bin = blockIdx.x;
    const uint32_t t = threadIdx.x;
    const Totals T = totals(bt);
    uint32_t *row = thist + bin * tstride;
    // thread t owns a contiguous run of tiles
    const uint64_t per = (T.tiles + kScanWG - 1) / kScanWG;
    const uint64_t t0 = per * t < T.tiles ? per * t : T.tiles;
    const uint64_t t1 = t0 + per < T.tiles ? t0 + per : T.tiles;
    uint32_t sum = 0;
    for (uint64_t k = t0; k < t1; ++k) sum += row[k];
    part[t] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < kScanWG; off <<= 1) {  // inclusive scan (Hillis-Steele)
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (uint64_t k = t0; k < t1; ++k) {
        const uint32_t c = row[k];
        row[k] = run;
        run += c;
    }
    if (t == kScanWG - 1) ctrl->bincount[bin] = part[t];
}

// Scatter of the tiles wg, wg + n_wg, ... into bin order (one workgroup),
// the next tile's loads in flight while the current one is placed (two
// buffers used in turn, as in k_bin_count).  `start` holds every bin's
// padded start (longest bins first).
__device__ __forceinline__ void bin_scatter(const Batch &bt, const uint32_t *__restrict__ thist,
                                            uint64_t tstride, const uint32_t *start, uint32_t n_id,
                                            unsigned long long *__restrict__ perm,
                                            TxRec *__restrict__ rec, uint32_t *__restrict__ pos_of,
                                            uint64_t wide_min, uint32_t wg, uint32_t n_wg)
{
    __shared__ uint32_t cnt[kBins];
    __shared__ uint32_t base[kBins];
    const Totals T = totals(bt);
    if (wg >= T.tiles) return;  // the whole workgroup
    // a tile's loads: its transactions, its block, the block's message-area
    // end, and (lanes below kBins) the tile's transactions of each bin in
    // earlier tiles
    struct Tile {
        TileTx x;
        DevBlock d;
        uint32_t b, before;
        uint64_t t, area_end;
    };
    auto load = [&](uint64_t t, Tile &z) {
        z.t = t;
        z.b = find_block<0>(bt, T, t);
        z.d = get_block(bt, T, z.b);
        load_tile_tx(z.d, (t - z.d.tile0) * kTile, z.x);
        z.before = ((gptr)thist)[(threadIdx.x < kBins ? threadIdx.x : 0u) * tstride + t];
        z.area_end = ((gptr64)z.d.off)[z.d.n];
    };
    // places tile z while the next one (the last tile: z's again, unused)
    // loads into y; returns whether there was a next tile
    auto step = [&](const Tile &z, Tile &y) -> bool {
        const bool more = z.t + n_wg < T.tiles;  // uniform
        load(more ? z.t + n_wg : z.t, y);
        if (threadIdx.x < kBins) {
            cnt[threadIdx.x] = 0;
            base[threadIdx.x] = start[threadIdx.x] + z.before;  // the tile's first position in each bin
        }
        __syncthreads();
        const uint64_t i0 = (z.t - z.d.tile0) * kTile;
        uint32_t bins[kPer], rank[kPer];
        TxRec r[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint64_t i = i0 + threadIdx.x + (uint64_t)k * kWG;
            bins[k] = kBins;
            if (i < z.d.n) {
                const uint64_t a = z.x.a[k], e = z.x.e[k];
                const uint32_t who = z.x.who[k];
                const bool ok = a <= e && who < n_id;
                const uint64_t L = ok ? e - a : 0;
                r[k].addr = reinterpret_cast<uint64_t>(z.d.msg + a);
                r[k].len = L >= wide_min ? kRecWide
                                         : (uint32_t)L | (e + kOverread <= z.area_end ? 0u : kRecNearEnd);
                r[k].id = ok ? who : kRecInvalid;
                bins[k] = bin_of_length(L);
                rank[k] = atomicAdd(&cnt[bins[k]], 1u);
            }
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (bins[k] < kBins) {
                const uint64_t i = i0 + threadIdx.x + (uint64_t)k * kWG;
                const uint32_t pos = base[bins[k]] + rank[k];
                perm[pos] = ((unsigned long long)z.b << 40) | i;
                rec[pos] = r[k];
                pos_of[z.d.tx0 + i] = pos;
            }
        }
        __syncthreads();
        return more;
    };
    Tile za, zb;
    load(wg, za);
    for (;;) {
        if (!step(za, zb)) break;
        if (!step(zb, za)) break;
    }
}

__global__ void __launch_bounds__(kWG) k_bin_scatter(Batch bt, Ctrl *ctrl,
                                                     const uint32_t *__restrict__ thist,
                                                     uint64_t tstride, uint32_t n_id,
                                                     unsigned long long *__restrict__ perm,
                                                     TxRec *__restrict__ rec,
                                                     uint32_t *__restrict__ pos_of, uint64_t wide_min)
{
    __builtin_amdgcn_s_setprio(3);  // as in k_bin_count
    // bin layout from the totals: order o = 63 - bin, longest first, each bin
    // padded to a multiple of 64; workgroup 0 publishes it for the verify pass
    __shared__ uint32_t pad[kBins];
    __shared__ uint32_t start[kBins];
    const uint32_t o = threadIdx.x;
    uint32_t c = 0;
    if (o < kBins) {
        c = ctrl->bincount[kBins - 1 - o];
        pad[o] = (c + 63u) & ~63u;
    }
    __syncthreads();
    if (o < kBins) {
        uint32_t at = 0;
        for (uint32_t k = 0; k < o; ++k) at += pad[k];
        start[kBins - 1 - o] = at;
        if (blockIdx.x == 0) {
            ctrl->ostart[o] = at;
            ctrl->ocount[o] = c;
            ctrl->opad[o] = pad[o];
            if (o == kBins - 1) ctrl->total_pos = at + pad[o];
        }
    }
    __syncthreads();
    bin_scatter(bt, thist, tstride, start, n_id, perm, rec, pos_of,
                wide_min < kRecMaxLen ? wide_min : kRecMaxLen, blockIdx.x, gridDim.x);
}

// Most wave tiles a persistent verify wave takes per atomic grab.
constexpr uint32_t kGrab = 8;

// ------------------------------------------------------------------------------------------
// k_verify, binned form: wave tile w covers bin-order positions 64w..64w+63,
// all in one bin; verdicts go to a bin-order bitmap.
// ------------------------------------------------------------------------------------------
// A transaction from its bin-order entry: e = block << 40 | index, r its
// record.  Returns whether it can be valid at all.
template <bool ATTEST>
__device__ __forceinline__ bool binned_tx(const Batch &bt, const Totals &T, const KeySource &ks,
                                          unsigned long long e, const TxRec &r, TxRef &t)
{
    const uint32_t b = (uint32_t)(e >> 40);
    const uint64_t i = e & ((1ull << 40) - 1);
    if (r.len == kRecWide) return load_tx<ATTEST>(get_block(bt, T, b), i, ks, t);  // a wide message
    const bool live = r.id != kRecInvalid;
    const uint32_t who = live ? r.id : 0u;
    t.msg = reinterpret_cast<const uint8_t *>(r.addr);
    t.L = r.len & ~kRecNearEnd;
    t.overread_ok = (r.len & kRecNearEnd) == 0;
    t.mid = ks.mid ? ks.mid + 16ull * who : nullptr;
    t.rev = ks.rev ? ks.rev + 32ull * who : nullptr;
    t.tag = (T.inline_one ? bt.one.tag : bt.table[b].tag) + (uint64_t)check_stride<ATTEST>() * i;
    return live;
}

template <bool PER_TX_KEYS, bool PERSISTENT, bool ATTEST>
__global__ void __launch_bounds__(kWG) ACE_WAVES(4) k_verify_binned(Batch bt, KeySource ks, HkdfParams hp,
                                                       Ctrl *ctrl,
                                                       const unsigned long long *__restrict__ perm,
                                                       const TxRec *__restrict__ rec,
                                                       uint32_t *__restrict__ vperm, GrabCaps caps)
{
    __shared__ HkdfPrep prep;
    __shared__ uint32_t ostart[kBins], ocount[kBins], oend[kBins];
    if constexpr (PER_TX_KEYS) {
        if (threadIdx.x < 64) hkdf_prepare(hp, prep);
    }
    if (threadIdx.x < kBins) {
        ostart[threadIdx.x] = ctrl->ostart[threadIdx.x];
        ocount[threadIdx.x] = ctrl->ocount[threadIdx.x];
        oend[threadIdx.x] = ctrl->ostart[threadIdx.x] + ctrl->opad[threadIdx.x];
    }
    __syncthreads();
    const Totals T = totals(bt);
    const uint32_t total = uniform32(ctrl->total_pos);
    const uint32_t nwaves = total >> 6;
    // persistent: tiles per grab, up to kGrab while every wave still gets
    // about four grabs (small batches take one tile at a time)
    uint32_t grab = nwaves / (gridDim.x * kWavesPerWG * 4u);
    grab = grab < 1u ? 1u : (grab > kGrab ? kGrab : grab);
    const uint32_t lane = lane_id();
    uint32_t w = PERSISTENT ? 0u
                            : blockIdx.x * kWavesPerWG + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t left = 0;  // persistent: wave tiles left of the last grab
    uint32_t o_last = 0;  // persistent: bin order of the wave's last tile (longest bin first)
    for (;;) {
        if constexpr (PERSISTENT) {
            if (left == 0) {
                // the length bucket's cap on tiles per grab (from the launch
                // tuning; 0 = none), by the bin the wave last worked on
                const uint32_t cap = caps.cap[kBins - 1 - o_last];
                const uint32_t g = cap && cap < grab ? cap : grab;
                // Every lane takes part in the atomic (lane 0 adds the grab, the
                // others 0) so no divergent branch precedes the readfirstlane:
                // with the atomic under `if (lane == 0)` the compiler may split
                // this loop per lane and leave lanes 1..63 re-reading a stale
                // tile forever.  Grabs of several tiles keep the counter's
                // same-address atomics few.
                const uint32_t v = atomicAdd(&ctrl->work, lane == 0 ? g : 0u);
                w = __builtin_amdgcn_readfirstlane(v);
                left = g;
            } else {
                ++w;
            }
            --left;
        }
        if (w >= nwaves) break;
        const uint32_t k0 = w << 6;
        // bin of this wave: number of bins that end at or before k0
        const uint32_t o = __popcll(__ballot(oend[lane] <= k0));
        o_last = o;
        const uint32_t k = k0 + lane;
        const bool active = k - ostart[o] < ocount[o];
        TxRef t{};
        bool live = false;
        if (active) live = binned_tx<ATTEST>(bt, T, ks, perm[k], rec[k], t);
        const bool valid = verify_lane<PER_TX_KEYS, ATTEST, !PERSISTENT>(live, t, &prep) && live;
        const unsigned long long m = __ballot(valid);
        if (lane == 0) {
            vperm[2 * w] = (uint32_t)m;
            vperm[2 * w + 1] = (uint32_t)(m >> 32);
        }
        if constexpr (!PERSISTENT) break;
    }
}

// Bin-order verdicts back to input order: one lane per transaction gathers
// its bit through its bin-order position, a wave64 ballot per 64
// transactions gives two bitmask words (k_count then adds up the counts).
__global__ void __launch_bounds__(kWG) k_finalize(Batch bt, const uint32_t *__restrict__ pos_of,
                                                  const uint32_t *__restrict__ vperm)
{
    const uint32_t lane = lane_id();
    const Totals T = totals(bt);
    if (blockIdx.x >= T.tiles) return;  // the whole workgroup
    // tiles g, g + G, ...: the next tile's positions load while the current
    // tile's bits are gathered (two buffers in turn, as in the binning passes;
    // lanes past a block's end reload its last position and drop the bit)
    struct Tile {
        DevBlock d;
        uint64_t t;
        uint32_t p[kPer];
    };
    auto load = [&](uint64_t t, Tile &z) {
        z.t = t;
        z.d = get_block(bt, T, find_block<0>(bt, T, t));
        const uint64_t i0 = (t - z.d.tile0) * kTile;
        const gptr src = (gptr)(pos_of + z.d.tx0);
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint64_t i = i0 + threadIdx.x + (uint64_t)k * kWG;
            z.p[k] = src[i < z.d.n ? i : z.d.n - 1];
        }
    };
    auto step = [&](const Tile &z, Tile &y) -> bool {
        const bool more = z.t + gridDim.x < T.tiles;  // uniform
        load(more ? z.t + gridDim.x : z.t, y);
        const uint64_t i0 = (z.t - z.d.tile0) * kTile;
        uint32_t v[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) v[k] = ((gptr)vperm)[z.p[k] >> 5];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {  // uniform trip count: the ballot sees every lane
            const uint64_t i = i0 + threadIdx.x + (uint64_t)k * kWG;
            const bool bit = i < z.d.n && ((v[k] >> (z.p[k] & 31)) & 1u);
            const unsigned long long m = __ballot(bit);
            const uint64_t base = i - lane;
            if (lane == 0 && base < z.d.n) {
                z.d.bitmask[base >> 5] = (uint32_t)m;
                if (base + 32 < z.d.n) z.d.bitmask[(base >> 5) + 1] = (uint32_t)(m >> 32);
            }
        }
        return more;
    };
    Tile za, zb;
    load(blockIdx.x, za);
    for (;;) {
        if (!step(za, zb)) break;
        if (!step(zb, za)) break;
    }
}

// Valid counts from the finished bitmasks (their unused tail bits are 0):
// workgroup w sums a contiguous run of tiles, one 64-word tile per wave at a
// time, and adds each block's part with one atomic, so a counter sees at most
// gridDim.x atomics.
__global__ void __launch_bounds__(kWG) k_count(Batch bt)
{
    __shared__ unsigned long long part[kWavesPerWG];
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x >> 6;
    const Totals T = totals(bt);
    const uint64_t per = (T.tiles + gridDim.x - 1) / gridDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * per;
    const uint64_t t1 = t0 + per < T.tiles ? t0 + per : T.tiles;
    for (uint64_t t = t0; t < t1;) {
        const DevBlock d = get_block(bt, T, find_block<0>(bt, T, t));
        const uint64_t dt_end = uniform64(d.tile0 + (d.n + kTile - 1) / kTile);
        const uint64_t end = dt_end < t1 ? dt_end : t1;
        const uint64_t words = (d.n + 31) / 32;
        unsigned long long acc = 0;
        for (uint64_t u = t + wave; u < end; u += kWavesPerWG) {
            const uint64_t w = (u - d.tile0) * (kTile / 32) + lane;  // kTile / 32 == 64 words
            if (w < words) acc += __popc(d.bitmask[w]);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
        if (lane == 0) part[wave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long s = 0;
            for (int v = 0; v < kWavesPerWG; ++v) s += part[v];
            if (s) atomicAdd(d.count, s);
        }
        __syncthreads();
        t = end;
    }
}

// Device-side plan of a graph replay: copies the block descriptors the host
// wrote into pinned memory, computes their prefixes in the three index
// spaces (transactions, tiles, wave tiles), publishes the totals, and clears
// the per-block counts and the persistent verify's tile counter.  One
// workgroup.
constexpr int kPlanWG = 1024;
__global__ void __launch_bounds__(kPlanWG) k_plan(const DevBlock *__restrict__ src,
                                                  const uint32_t *__restrict__ src_n,
                                                  uint32_t max_blocks, DevBlock *__restrict__ table,
                                                  BatchHdr *__restrict__ hdr, Ctrl *__restrict__ ctrl)
{
    __shared__ uint64_t sc[3][kPlanWG];
    __shared__ uint64_t carry[3];
    const uint32_t t = threadIdx.x;
    uint32_t n = *src_n;
    if (n > max_blocks) n = max_blocks;
    if (t < 3) carry[t] = 0;
    if (ctrl && t == 0) {
        ctrl->total_pos = 0;
        ctrl->work = 0;
    }
    __syncthreads();
    for (uint32_t base = 0; base < n; base += kPlanWG) {
        const uint32_t b = base + t;
        DevBlock d{};
        uint64_t v[3] = {0, 0, 0};
        if (b < n) {
            d = src[b];
            v[0] = d.n;
            v[1] = (d.n + kTile - 1) / kTile;
            v[2] = (d.n + 63) / 64;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) sc[k][t] = v[k];
        __syncthreads();
        for (uint32_t off = 1; off < kPlanWG; off <<= 1) {  // inclusive scan (Hillis-Steele)
            uint64_t a[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) a[k] = t >= off ? sc[k][t - off] : 0;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 3; ++k) sc[k][t] += a[k];
            __syncthreads();
        }
        if (b < n) {
            d.tx0 = carry[0] + sc[0][t] - v[0];
            d.tile0 = carry[1] + sc[1][t] - v[1];
            d.wave0 = carry[2] + sc[2][t] - v[2];
            table[b] = d;
            *d.count = 0;
        }
        __syncthreads();
        if (t == kPlanWG - 1) {
#pragma unroll
            for (int k = 0; k < 3; ++k) carry[k] += sc[k][t];
        }
        __syncthreads();
    }
    if (t == 0) {
        hdr->n_blocks = n;
        hdr->total_tx = carry[0];
        hdr->total_tiles = carry[1];
        hdr->total_waves = carry[2];
    }
}

// Writes a chunk of block descriptors (passed by value) into the device table.
__global__ void k_put_descs(DevBlock *table, DescChunk c)
{
    const uint32_t t = threadIdx.x;
    if (t < c.count) table[c.first + t] = c.d[t];
}

// Explicit instantiations used by the host entry points.
template __global__ void k_verify_ordered<false, false>(Batch, KeySource, HkdfParams);
template __global__ void k_verify_ordered<true, false>(Batch, KeySource, HkdfParams);
template __global__ void k_verify_ordered<false, true>(Batch, KeySource, HkdfParams);
#define ACE_BINNED(P, Q, R)                                                                     \
    template __global__ void k_verify_binned<P, Q, R>(Batch, KeySource, HkdfParams, Ctrl *,   \
                                                      const unsigned long long *, const TxRec *, \
                                                      uint32_t *, GrabCaps);
ACE_BINNED(false, false, false)
ACE_BINNED(false, true, false)
ACE_BINNED(true, false, false)
ACE_BINNED(true, true, false)
ACE_BINNED(false, false, true)
ACE_BINNED(false, true, true)
#undef ACE_BINNED

}  // namespace ace
