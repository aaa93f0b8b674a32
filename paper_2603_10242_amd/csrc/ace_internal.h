// ace_internal.h -- device-side data layout shared by the kernels and the
// host entry points of libace.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ace {

constexpr int kWG = 256;          // threads per workgroup (4 wave64)
constexpr int kWavesPerWG = kWG / 64;
constexpr int kTile = 2048;       // transactions per tile of the binning/finalize passes
constexpr int kBins = 64;         // bins by inner block count nb = ceil((L+9)/64); bin 63 = nb >= 64
constexpr uint32_t kMaxSalt = 1024;
constexpr uint32_t kMaxInfo = 255;
constexpr uint32_t kMaxInfoBlocks = 5;  // ceil((64 + 255 + 1 + 9) / 64) - 1

// One block of transactions as the kernels see it, plus its prefixes in the
// concatenated index spaces of a multi-block call.
struct DevBlock {
    const uint8_t *msg;
    const uint64_t *off;
    const uint32_t *id;
    const uint8_t *tag;
    uint32_t *bitmask;
    unsigned long long *count;
    uint64_t n;      // transactions
    uint64_t tx0;    // first global transaction index
    uint64_t tile0;  // first tile (kTile transactions per tile)
    uint64_t wave0;  // first wave tile of the in-order verify (64 per wave)
};

// Sizes of a call that a captured graph reads from device memory (they
// change from replay to replay while the kernel arguments stay fixed).
struct BatchHdr {
    uint32_t n_blocks;
    uint32_t pad_;
    uint64_t total_tx;
    uint64_t total_tiles;
    uint64_t total_waves;
};

// Blocks of one call: a single block travels inline in the kernel arguments,
// several blocks in a device table.  When `hdr` is set, the block count and
// totals come from it and every block from the table.
struct Batch {
    DevBlock one;
    const DevBlock *table;
    const BatchHdr *hdr;
    uint32_t n_blocks;
    uint64_t total_tx;
    uint64_t total_tiles;
    uint64_t total_waves;
};

// Control words of a bucketed pass (start of the workspace).  The per-tile
// bin counts live beside them in the workspace (see k_bin_count).
struct Ctrl {
    uint32_t bincount[kBins];  // transactions per bin (k_bin_scan)
    uint32_t ostart[kBins];    // bins in order o = 63 - bin (longest first): padded start
    uint32_t ocount[kBins];    // real transactions
    uint32_t opad[kBins];      // count rounded up to a multiple of 64
    uint32_t total_pos;        // sum of opad
    uint32_t work;             // wave-tile counter of the persistent verify
    uint32_t pad_[62];
};

// Persistent verify kernel: most wave tiles per atomic grab while a wave
// works on bin b (0: no cap), a kernel argument set from the launch tuning.
struct GrabCaps {
    uint8_t cap[kBins];
};

// HKDF parameters shared by all identities of a keyset (kernel argument).
struct HkdfParams {
    uint32_t salt_len;
    uint32_t info_len;
    uint8_t salt[kMaxSalt];
    uint8_t info[kMaxInfo + 1];
};

// Several HKDF parameter sets in one launch (one per grid row): short salts
// and infos only, so that the set fits the kernel's argument block.
constexpr uint32_t kMultiStreams = 16;
constexpr uint32_t kMultiSalt = 64;
constexpr uint32_t kMultiInfo = 64;
struct StreamParams {
    uint32_t salt_len;
    uint32_t info_len;
    uint8_t salt[kMultiSalt];
    uint8_t info[kMultiInfo];
};
struct MultiHkdf {
    uint32_t first;  // index of s[0] among the call's streams
    uint32_t count;
    StreamParams s[kMultiStreams];
};

// Derived per-workgroup constants of an HKDF parameter set (built in LDS).
// The expand blocks (info || 0x01 and its padding) are the same for every
// identity, so they are held as their whole schedules with the round
// constants added: info_kw[q][t] = K[t] + W_q[t].
struct HkdfPrep {
    uint32_t salt_ipad[8];
    uint32_t salt_opad[8];
    alignas(16) uint32_t info_kw[kMaxInfoBlocks][64];
    uint32_t info_blocks;
};

// One transaction in bin order, written by the scatter pass so that the
// verify kernel reads contiguous records instead of gathering offsets and
// identities from scattered lines.
constexpr uint32_t kRecWide = 0xFFFFFFFFu;     // len: a wide message, re-read the offsets
constexpr uint64_t kRecMaxLen = 0x7FFFFFFFu;   // messages this long or longer are always wide
constexpr uint32_t kRecNearEnd = 0x80000000u;  // len flag: the block's message area ends within
                                               // kOverread bytes after this message
constexpr uint32_t kRecInvalid = 0xFFFFFFFFu;  // id: the transaction cannot be valid
struct TxRec {
    uint64_t addr;  // address of the first message byte
    uint32_t len;   // message length | kRecNearEnd, or kRecWide
    uint32_t id;    // identity index, or kRecInvalid
};

// Bytes past a message's end that the block loads of its last blocks may
// read: 17 dwords from the aligned start of the last block, whose message
// part is at least L - 64 * (nb - 1) > -9 bytes, give at most 76.
constexpr uint64_t kOverread = 80;

struct KeySource {
    const uint32_t *mid;   // [n_id][16] midstates, or NULL when keys come from rev
    const uint8_t *rev;    // [n_id][32] root entropy (per-transaction derivation)
    uint32_t n_id;
};

// A chunk of block descriptors passed by value to the kernel that writes
// them into the device table (no host staging buffer is needed).
constexpr int kDescChunk = 24;
struct DescChunk {
    DevBlock d[kDescChunk];
    uint32_t first;
    uint32_t count;
};

// Occupancy targets (waves per SIMD) that the hash kernels reach without
// spilling when the block computation is the looped form; the register
// allocator is asked for them explicitly because on its own it trades
// occupancy for scheduling freedom (about 120 VGPRs, 4 waves).
#ifndef ACE_WAVES_HINTS
#define ACE_WAVES_HINTS 1
#endif
#if ACE_WAVES_HINTS
#define ACE_WAVES(n) __attribute__((amdgpu_waves_per_eu(n, n)))
#else
#define ACE_WAVES(n)
#endif

__host__ __device__ inline uint32_t bin_of_length(uint64_t L)
{
    uint64_t nb = (L + 9 + 63) >> 6;
    return (uint32_t)(nb >= (uint64_t)kBins ? kBins : nb) - 1u;
}

}  // namespace ace
