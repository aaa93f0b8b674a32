// merkle_kernels.hip -- Merkle roots of the block header's transaction and
// attestation lists (App. C, block header fields tx_merkle_root and
// attest_merkle_root; a validator recomputes the attestation root, Alg. 4).
//
// Reading (the paper fixes neither): leaf node = SHA-256(leaf bytes); parent
// = SHA-256(left || right); at a level with an odd number of nodes the last
// one moves up unchanged; a tree without leaves has the root SHA-256("").
//
// Layout: node j of level k of a tree whose leaves start at global leaf
// index leaf0 lives in slot leaf0 + j * 2^k of one node array (8 native
// words per slot).  A parent overwrites its left child's slot, so levels are
// reduced in place, and an unpaired last node is already where the next
// level expects it.
//
//   k_merkle_leaves  one leaf per lane: SHA-256 of its bytes into its slot.
//   k_merkle_plan    per level (one workgroup each), exclusive prefix of each
//                    tree's pair count.
//   k_merkle_level   one parent per lane at level k -> k + 1 (two blocks:
//                    the 64 child bytes, then the constant padding block).
//   k_merkle_top     the levels from k0 up, where every tree has at most
//                    kTopNodes nodes: one workgroup per tree, in LDS.
//   k_merkle_out     roots to the callers' 32-byte outputs.

namespace ace {

struct MerkleDesc {
    const uint8_t *data;
    const uint64_t *off;
    uint64_t n;      // leaves
    uint8_t *root;   // 32-byte output
    uint64_t leaf0;  // global index of the first leaf
};

constexpr uint32_t kMerkleChunk = 64;
struct MerkleChunk {
    MerkleDesc d[kMerkleChunk];
    uint32_t first;
    uint32_t count;
};

// The second block of every parent is the padding of a 64-byte message
// (0x80, zeros, bit length 512): its whole message schedule is known at
// compile time, so it is folded into the round constants, kw[t] = K[t] +
// W[t], and the block costs the 64 rounds and the feed-forward only.
constexpr uint32_t c_rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }
struct ScheduleKW {
    uint32_t v[64];
};
constexpr ScheduleKW fold_pad64()
{
    ScheduleKW r{};
    uint32_t w[64] = {};
    w[0] = 0x80000000u;
    w[15] = 512u;
    for (int t = 16; t < 64; ++t) {
        const uint32_t s0 = c_rotr(w[t - 15], 7) ^ c_rotr(w[t - 15], 18) ^ (w[t - 15] >> 3);
        const uint32_t s1 = c_rotr(w[t - 2], 17) ^ c_rotr(w[t - 2], 19) ^ (w[t - 2] >> 10);
        w[t] = s1 + w[t - 7] + s0 + w[t - 16];
    }
    for (int t = 0; t < 64; ++t) r.v[t] = kRound[t] + w[t];
    return r;
}
__constant__ __attribute__((aligned(64))) ScheduleKW kPad64KW = fold_pad64();

__device__ __forceinline__ void compress_pad64(State &s)
{
    uint32_t a = s.h[0], b = s.h[1], c = s.h[2], d = s.h[3];
    uint32_t e = s.h[4], f = s.h[5], g = s.h[6], h = s.h[7];
#pragma nounroll
    for (int q = 0; q < 4; ++q) {
        const RoundConsts16 kq = *reinterpret_cast<const RoundConsts16 *>(&kPad64KW.v[16 * q]);
#pragma unroll
        for (int j = 0; j < 16; ++j) round_step(a, b, c, d, e, f, g, h, 0u, kq.k[j]);
    }
    s.h[0] += a; s.h[1] += b; s.h[2] += c; s.h[3] += d;
    s.h[4] += e; s.h[5] += f; s.h[6] += g; s.h[7] += h;
}

__global__ void k_merkle_put(MerkleDesc *table, MerkleChunk c)
{
    const uint32_t t = threadIdx.x;
    if (t < c.count) table[c.first + t] = c.d[t];
}

// Last i < n with key(i) <= x, for keys that do not decrease (equal keys:
// the last of them).  The lanes of a wave hold consecutive x, so the first
// active lane's x is searched once for the wave (a uniform loop on scalar
// loads); only lanes at or past the next key (a wave across two trees)
// search again, each on its own.
template <class Key>
__device__ __forceinline__ uint32_t last_at_or_below(uint32_t n, uint64_t x, Key key)
{
    const uint64_t x0 = uniform64(x);
    uint32_t lo = 0, hi = n;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (key(mid) <= x0) lo = mid;
        else hi = mid;
    }
    if (lo + 1 < n && key(lo + 1) <= x) {
        uint32_t l = lo + 1, h = n;
        while (h - l > 1) {
            const uint32_t mid = (l + h) >> 1;
            if (key(mid) <= x) l = mid;
            else h = mid;
        }
        return l;
    }
    return lo;
}

// Tree of leaf g: the last tree whose first leaf is <= g (trees with no
// leaves are skipped by taking the last of equal starts).
__device__ __forceinline__ uint32_t merkle_tree_of(const MerkleDesc *__restrict__ table,
                                                   uint32_t n_trees, uint64_t g)
{
    return last_at_or_below(n_trees, g, [&](uint32_t i) { return table[i].leaf0; });
}

// SHA-256 of L bytes at p into S (from the initial value).  With
// overread_ok (the tree's data area extends at least 80 bytes past this
// leaf) whole 16-byte loads are used, whose bytes past the leaf's end feed
// only words the padding overwrites; otherwise every dword address is
// clamped to one that holds leaf bytes (for L == 0 none is read).
__device__ __forceinline__ void sha256_bytes(bool live, const uint8_t *p, uint64_t L, State &S,
                                             bool overread_ok = false)
{
    S = initial_state();
    const uint32_t nb = live ? (uint32_t)((L + 9 + 63) >> 6) : 0u;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(p);
    const uint32_t sh = (uint32_t)addr & 3u;
    const uint32_t sel = 0x00010203u + sh * 0x01010101u;
    const uint64_t lim = (uint64_t)sh + L;
    const uint64_t last = lim ? ((lim - 1) >> 2) : 0;
    const uint32_t *A0 = reinterpret_cast<const uint32_t *>(addr - sh);
    const uint64_t bits = L << 3;
    for (uint32_t b = 0;; ++b) {
        const bool run = live && b < nb;
        if (__ballot(run) == 0) break;
        if (run) {
            uint32_t D[17], W[16];
            if (overread_ok) {
                const uint32_t *q = A0 + 16ull * b;
                const U4 v0 = load16(q), v1 = load16(q + 4), v2 = load16(q + 8), v3 = load16(q + 12);
                D[0] = v0.x; D[1] = v0.y; D[2] = v0.z; D[3] = v0.w;
                D[4] = v1.x; D[5] = v1.y; D[6] = v1.z; D[7] = v1.w;
                D[8] = v2.x; D[9] = v2.y; D[10] = v2.z; D[11] = v2.w;
                D[12] = v3.x; D[13] = v3.y; D[14] = v3.z; D[15] = v3.w;
                D[16] = load32(q + 16);
            } else {
#pragma unroll
                for (int k = 0; k < 17; ++k) {
                    const uint64_t idx = 16ull * b + k;
                    D[k] = lim ? load32(A0 + (idx < last ? idx : last)) : 0u;
                }
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) W[j] = __builtin_amdgcn_perm(D[j + 1], D[j], sel);
            const int64_t rb = (int64_t)L - 64 * (int64_t)b;
            if (rb < 64) {
                const int32_t r0 = (int32_t)rb;
                const int32_t jf = r0 >> 2;
                const uint32_t c8 = ((uint32_t)r0 & 3u) << 3;
                const uint32_t keep = ~(0xFFFFFFFFu >> c8);
                const uint32_t pad = 0x80000000u >> c8;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const uint32_t part = (W[j] & keep) | pad;
                    W[j] = j < jf ? W[j] : (j == jf ? part : 0u);
                }
                if (b + 1 == nb) {
                    W[14] = (uint32_t)(bits >> 32);
                    W[15] = (uint32_t)bits;
                }
            }
            compress_block(S, W);
        }
    }
}

// SHA-256 of a 72-byte leaf at p (4-byte alignment not required): the
// paper form's check record, obj_hash (32) || domain (8) || credential (32),
// the leaf of an attestation root.  Its second block holds 8 record bytes,
// then the 0x80 marker, zeros and the bit length 576: words 2..15 are
// constants there and fold into that block's schedule.  The 19 dwords from
// the aligned start hold the record at any alignment; the last one is read
// only when it holds record bytes.
constexpr uint64_t kRecordLeaf = 72;
__device__ __forceinline__ void sha256_record72(const uint8_t *p, State &S)
{
    const uintptr_t addr = reinterpret_cast<uintptr_t>(p);
    const uint32_t sh = (uint32_t)addr & 3u;
    const uint32_t sel = 0x00010203u + sh * 0x01010101u;
    const uint32_t *A0 = reinterpret_cast<const uint32_t *>(addr - sh);
    uint32_t D[19];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const U4 v = load16(A0 + 4 * c);
        D[4 * c] = v.x; D[4 * c + 1] = v.y; D[4 * c + 2] = v.z; D[4 * c + 3] = v.w;
    }
    D[16] = load32(A0 + 16);
    D[17] = load32(A0 + 17);
    D[18] = load32(A0 + (sh ? 18 : 17));
    uint32_t W[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) W[j] = __builtin_amdgcn_perm(D[j + 1], D[j], sel);
    S = initial_state();
    compress_block(S, W);
    W[0] = __builtin_amdgcn_perm(D[17], D[16], sel);
    W[1] = __builtin_amdgcn_perm(D[18], D[17], sel);
    W[2] = 0x80000000u;
#pragma unroll
    for (int j = 3; j < 15; ++j) W[j] = 0u;
    W[15] = (uint32_t)(kRecordLeaf * 8);
    compress_fold(S, W);
}

__global__ void __launch_bounds__(kWG) k_merkle_leaves(const MerkleDesc *__restrict__ table,
                                                       uint32_t n_trees, uint64_t n_leaves,
                                                       uint32_t *__restrict__ nodes)
{
    const uint64_t g = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    const bool live = g < n_leaves;
    const uint8_t *p = nullptr;
    uint64_t L = 0;
    bool overread_ok = false;
    if (live) {
        const MerkleDesc d = table[merkle_tree_of(table, n_trees, g)];
        const uint64_t i = g - d.leaf0;
        const uint64_t a = d.off[i], e = d.off[i + 1];
        p = d.data + a;
        L = e >= a ? e - a : 0;  // decreasing offsets: the empty leaf
        // 17 dwords from the aligned start of the last block reach at most 76
        // bytes past the leaf's end; the tree's leaves end at off[n]
        overread_ok = e >= a && a + L + 80 <= d.off[d.n];
    }
    State S;
    if (__ballot(live && L != kRecordLeaf) == 0) {
        // every live leaf of the wave is a 72-byte record
        if (live) sha256_record72(p, S);
    } else {
        sha256_bytes(live, p, L, S, overread_ok);
    }
    if (live) {
        uint32_t *q = nodes + 8ull * g;
#pragma unroll
        for (int k = 0; k < 8; ++k) q[k] = S.h[k];
    }
}

// P[k * (n_trees + 1) + b] = pairs at level k of trees before b; the last
// entry of each row is the level's total.  Workgroup k scans level k.
constexpr uint32_t kPlanThreads = 1024;
__global__ void __launch_bounds__(kPlanThreads) k_merkle_plan(const MerkleDesc *__restrict__ table,
                                                              uint32_t n_trees,
                                                              unsigned long long *__restrict__ P)
{
    __shared__ unsigned long long part[kPlanThreads];
    const uint32_t t = threadIdx.x;
    const uint32_t k = blockIdx.x;
    unsigned long long *row = P + (uint64_t)k * (n_trees + 1);
    unsigned long long running = 0;
    for (uint32_t c = 0; c < n_trees; c += kPlanThreads) {
        const uint32_t b = c + t;
        unsigned long long v = 0;
        if (b < n_trees) {
            const uint64_t n = table[b].n;
            const uint64_t m = k >= 63 ? (n ? 1 : 0) : (n + (1ull << k) - 1) >> k;
            v = m >> 1;
        }
        part[t] = v;
        __syncthreads();
        // Hillis-Steele inclusive scan
        for (uint32_t s = 1; s < kPlanThreads; s <<= 1) {
            const unsigned long long add = t >= s ? part[t - s] : 0ull;
            __syncthreads();
            part[t] += add;
            __syncthreads();
        }
        if (b < n_trees) row[b] = running + part[t] - v;
        running += part[kPlanThreads - 1];
        __syncthreads();
    }
    if (t == 0) row[n_trees] = running;
}

__global__ void __launch_bounds__(kWG) k_merkle_level(const MerkleDesc *__restrict__ table,
                                                      uint32_t n_trees, uint32_t k,
                                                      const unsigned long long *__restrict__ Pk,
                                                      uint32_t *__restrict__ nodes)
{
    const uint64_t q = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    const bool live = q < Pk[n_trees];
    uint32_t W[16];
    uint64_t left = 0;
    if (live) {
        // last tree whose prefix is <= q
        const uint32_t lo = last_at_or_below(n_trees, q, [&](uint32_t i) { return Pk[i]; });
        const uint64_t p = q - Pk[lo];
        left = table[lo].leaf0 + ((2 * p) << k);
        const uint64_t right = left + (1ull << k);
        const uint32_t *a = nodes + 8ull * left;
        const uint32_t *b = nodes + 8ull * right;
        const U4 a0 = load16(a), a1 = load16(a + 4), b0 = load16(b), b1 = load16(b + 4);
        W[0] = a0.x; W[1] = a0.y; W[2] = a0.z; W[3] = a0.w;
        W[4] = a1.x; W[5] = a1.y; W[6] = a1.z; W[7] = a1.w;
        W[8] = b0.x; W[9] = b0.y; W[10] = b0.z; W[11] = b0.w;
        W[12] = b1.x; W[13] = b1.y; W[14] = b1.z; W[15] = b1.w;
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) W[j] = 0;
    }
    if (__ballot(live) == 0) return;
    State S = initial_state();
    compress_block(S, W);
    compress_pad64(S);  // the 64-byte message's padding block
    if (live) {
        uint32_t *o = nodes + 8ull * left;
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = S.h[j];
    }
}

// The narrow top of every tree in one launch: workgroup b takes tree b from
// level k0 (at most kTopNodes nodes there) to its root in LDS, one parent per
// lane and level, and writes the root to the tree's first slot.  One launch
// per level up there cost more in launches than in hashing.
constexpr uint32_t kTopWG = 512;
constexpr uint32_t kTopNodes = 2 * kTopWG;
__global__ void __launch_bounds__(kTopWG) k_merkle_top(const MerkleDesc *__restrict__ table, uint32_t k0,
                                                       uint32_t *__restrict__ nodes)
{
    __shared__ uint32_t node[kTopNodes][8];
    const MerkleDesc d = table[blockIdx.x];
    const uint32_t t = threadIdx.x;
    // nodes of the tree at level k0 (the host picks k0 so that m <= kTopNodes)
    uint32_t m = d.n ? (uint32_t)((d.n + (1ull << k0) - 1) >> k0) : 0u;
    if (m <= 1) return;  // the whole workgroup: the root is already in place
    for (uint32_t j = t; j < m; j += kTopWG) {
        const uint32_t *q = nodes + 8ull * (d.leaf0 + ((uint64_t)j << k0));
        const U4 a = load16(q), b = load16(q + 4);
        node[j][0] = a.x; node[j][1] = a.y; node[j][2] = a.z; node[j][3] = a.w;
        node[j][4] = b.x; node[j][5] = b.y; node[j][6] = b.z; node[j][7] = b.w;
    }
    __syncthreads();
    while (m > 1) {  // uniform
        const uint32_t pairs = m >> 1;
        const bool act = t < pairs;
        State S = initial_state();
        if (act) {
            uint32_t W[16];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                W[j] = node[2 * t][j];
                W[8 + j] = node[2 * t + 1][j];
            }
            compress_block(S, W);
            compress_pad64(S);  // the 64-byte message's padding block
        }
        // an unpaired last node moves up unchanged, to index `pairs`
        uint32_t carry[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) carry[j] = node[m - 1][j];
        __syncthreads();
        if (act) {
#pragma unroll
            for (int j = 0; j < 8; ++j) node[t][j] = S.h[j];
        }
        if ((m & 1) && t == 0) {
#pragma unroll
            for (int j = 0; j < 8; ++j) node[pairs][j] = carry[j];
        }
        __syncthreads();
        m = pairs + (m & 1);
    }
    if (t < 8) nodes[8ull * d.leaf0 + t] = node[0][t];
}

__global__ void __launch_bounds__(kWG) k_merkle_out(const MerkleDesc *__restrict__ table,
                                                    uint32_t n_trees,
                                                    const uint32_t *__restrict__ nodes)
{
    const uint32_t b = blockIdx.x * kWG + threadIdx.x;
    const bool live = b < n_trees;
    MerkleDesc d{};
    if (live) d = table[b];
    // SHA-256 of the empty string for a tree without leaves
    State S;
    sha256_bytes(live && d.n == 0, nullptr, 0, S);
    if (!live) return;
    if (d.n) {
        const uint32_t *q = nodes + 8ull * d.leaf0;
#pragma unroll
        for (int j = 0; j < 8; ++j) S.h[j] = q[j];
    }
    uint32_t *o = reinterpret_cast<uint32_t *>(d.root);
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = bswap32(S.h[j]);
}

}  // namespace ace
