// ace_api.hip -- host entry points of libace.so (declared in include/ace.h).
//
// Argument checking, workspace layout, launch sequences, graph capture and
// stage timing.  Nothing here computes any part of the attestation check:
// every hash runs in the kernels of ace_kernels.hip.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/ace.h"

// The kernels are compiled in this translation unit.
#include "ace_kernels.hip"
#include "valu_rate.hip"
#include "chain_kernels.hip"
#include "merkle_kernels.hip"

using namespace ace;

namespace {

thread_local char g_err[512];

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return ACE_OK;
    return fail(ACE_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int launch_status(const char *what) { return check_hip(hipGetLastError(), what); }

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Workgroups per CU of a key derivation that has the GPU to itself: four
// waves per SIMD, the kernel's lanes striding over the identities, so that
// every wave derives the same number of keys (a million identities in waves of
// one each are 3.2 rounds of the five-wave slots, the last one a fifth full).
constexpr unsigned kDeriveWgsPerCu = 4;

// Compute units of the current device (cached per device).
int cu_count()
{
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (!cache[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        cache[dev] = v;
    }
    return cache[dev];
}

// ------------------------------------------------------------------------------------------
// Tuning (set by the autotuner through ace_set_tuning).
// ------------------------------------------------------------------------------------------
std::mutex g_tune_mu;
ace_tuning g_tune = {
    /* binned_min_tx     */ 1u << 18,
    /* verify_wgs_per_cu */ 8,
    /* aux_wgs_per_cu    */ 8,
    /* auto_persistent   */ 0,
    /* derive_wgs_per_cu */ 4,
    /* wide_min_len      */ kRecMaxLen,
    /* grab_cap          */ {0},
};

ace_tuning tuning()
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    return g_tune;
}

// ------------------------------------------------------------------------------------------
// Stage timing: one set of events per profiled call, reused after a reset.
// ------------------------------------------------------------------------------------------
struct ProfCall {
    hipEvent_t ev[5];  // start, after derive, after binning, after verify, end
};
struct ProfState {
    bool on = false;
    std::vector<ProfCall> calls;
    size_t used = 0;
    ~ProfState()
    {
        for (auto &c : calls)
            for (auto &e : c.ev) (void)hipEventDestroy(e);
    }
};
thread_local ProfState g_prof;

ProfCall *prof_begin(hipStream_t s)
{
    if (!g_prof.on) return nullptr;
    if (g_prof.used == g_prof.calls.size()) {
        ProfCall c;
        for (auto &e : c.ev)
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_prof.calls.push_back(c);
    }
    ProfCall *c = &g_prof.calls[g_prof.used++];
    (void)hipEventRecord(c->ev[0], s);
    return c;
}

inline void prof_mark(ProfCall *c, int k, hipStream_t s)
{
    if (c) (void)hipEventRecord(c->ev[k], s);
}

// ------------------------------------------------------------------------------------------
// Arguments, plan and workspace layout.
// ------------------------------------------------------------------------------------------
int fill_hkdf(HkdfParams &hp, const uint8_t *salt, size_t salt_len, const uint8_t *info,
              size_t info_len)
{
    if (salt_len > kMaxSalt)
        return fail(ACE_ERR_INVALID_ARG, "salt_len %zu exceeds %u", salt_len, kMaxSalt);
    if (info_len > kMaxInfo)
        return fail(ACE_ERR_INVALID_ARG, "info_len %zu exceeds %u", info_len, kMaxInfo);
    if (salt_len && !salt) return fail(ACE_ERR_INVALID_ARG, "h_salt is NULL with salt_len > 0");
    if (info_len && !info) return fail(ACE_ERR_INVALID_ARG, "h_info is NULL with info_len > 0");
    memset(&hp, 0, sizeof hp);
    hp.salt_len = (uint32_t)salt_len;
    hp.info_len = (uint32_t)info_len;
    if (salt_len) memcpy(hp.salt, salt, salt_len);
    if (info_len) memcpy(hp.info, info, info_len);
    return ACE_OK;
}

enum Mode { kOrdered, kBinned };

struct Plan {
    Mode mode;
    bool per_tx;
    bool persistent;
    bool rev;
    bool attest;  // paper-form records (payload binding + credential over obj_hash || domain)
    uint32_t n_blocks;
    uint64_t total_tx;
    uint64_t total_tiles;
    uint64_t total_waves;
    uint64_t max_pos;  // upper bound of bin-order positions
    uint64_t tstride;  // tiles the per-tile bin counts have room for (row length)
    // workspace layout (byte offsets)
    size_t off_ctrl, off_hdr, off_descs, off_mid, off_thist, off_perm, off_rec, off_posof,
        off_vperm, bytes;
};

int check_keyset(const ace_keyset *keys, uint32_t flags, Plan &p)
{
    if (!keys) return fail(ACE_ERR_INVALID_ARG, "keys is NULL");
    const uint32_t known = ACE_ORDERED | ACE_BUCKETED | ACE_PERSISTENT | ACE_PER_TX_KEYS;
    if (flags & ~known) return fail(ACE_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags & ~known);
    if ((flags & ACE_ORDERED) && (flags & ACE_BUCKETED))
        return fail(ACE_ERR_INVALID_ARG, "ACE_ORDERED and ACE_BUCKETED are exclusive");
    if (keys->kind != ACE_KEYS_MIDSTATE && keys->kind != ACE_KEYS_REV)
        return fail(ACE_ERR_INVALID_ARG, "unknown keyset kind %d", keys->kind);
    p.rev = keys->kind == ACE_KEYS_REV;
    p.per_tx = (flags & ACE_PER_TX_KEYS) != 0;
    if (p.per_tx && !p.rev)
        return fail(ACE_ERR_INVALID_ARG, "ACE_PER_TX_KEYS needs a keyset of kind ACE_KEYS_REV");
    if (keys->n_id) {
        if (p.rev) {
            if (!keys->d_rev) return fail(ACE_ERR_INVALID_ARG, "keyset d_rev is NULL");
            if (!aligned(keys->d_rev, 4)) return fail(ACE_ERR_INVALID_ARG, "keyset d_rev not 4-byte aligned");
        } else {
            if (!keys->d_mid) return fail(ACE_ERR_INVALID_ARG, "keyset d_mid is NULL");
            if (!aligned(keys->d_mid, 16)) return fail(ACE_ERR_INVALID_ARG, "keyset d_mid not 16-byte aligned");
        }
    }
    if (p.rev) {
        if (keys->salt_len > kMaxSalt || keys->info_len > kMaxInfo)
            return fail(ACE_ERR_INVALID_ARG, "salt_len or info_len too long");
        if ((keys->salt_len && !keys->h_salt) || (keys->info_len && !keys->h_info))
            return fail(ACE_ERR_INVALID_ARG, "keyset h_salt/h_info is NULL");
    }
    return ACE_OK;
}

int check_blocks(const ace_block *blocks, uint32_t n_blocks, uint64_t &total, uint64_t &tiles,
                 uint64_t &waves)
{
    if (n_blocks && !blocks) return fail(ACE_ERR_INVALID_ARG, "blocks is NULL");
    if (n_blocks >= (1u << 24)) return fail(ACE_ERR_RANGE, "n_blocks %u >= 2^24", n_blocks);
    total = tiles = waves = 0;
    for (uint32_t b = 0; b < n_blocks; ++b) {
        const ace_block &k = blocks[b];
        if (!k.d_count_out) return fail(ACE_ERR_INVALID_ARG, "block %u: d_count_out is NULL", b);
        if (!aligned(k.d_count_out, 8))
            return fail(ACE_ERR_INVALID_ARG, "block %u: d_count_out not 8-byte aligned", b);
        if (k.n_tx) {
            if (!k.d_off || !k.d_id || !k.d_tag || !k.d_bitmask_out || !k.d_msg)
                return fail(ACE_ERR_INVALID_ARG, "block %u: NULL array with n_tx > 0", b);
            if (!aligned(k.d_off, 8) || !aligned(k.d_id, 4) || !aligned(k.d_tag, 4) ||
                !aligned(k.d_bitmask_out, 4))
                return fail(ACE_ERR_INVALID_ARG, "block %u: misaligned array", b);
        }
        if (k.n_tx > ACE_MAX_TX) return fail(ACE_ERR_RANGE, "block %u: n_tx too large", b);
        total += k.n_tx;
        if (total > ACE_MAX_TX) return fail(ACE_ERR_RANGE, "total transactions exceed ACE_MAX_TX");
        tiles += (k.n_tx + kTile - 1) / kTile;
        waves += (k.n_tx + 63) / 64;
    }
    return ACE_OK;
}

// Mode, persistence and workspace layout for n_blocks blocks of `total`
// transactions in all (exact sizes for a call, maxima for a graph).  `tiles`:
// the call's tiles of kTile transactions (a graph bounds them from the maxima).
void layout(const ace_keyset *keys, uint32_t n_blocks, uint64_t total, uint64_t tiles,
            uint32_t flags, bool graph, Plan &p)
{
    const ace_tuning t = tuning();
    p.n_blocks = n_blocks;
    if (flags & ACE_ORDERED) p.mode = kOrdered;
    else if (flags & ACE_BUCKETED) p.mode = kBinned;
    else p.mode = total >= t.binned_min_tx ? kBinned : kOrdered;
    const bool binned = p.mode == kBinned;
    p.persistent = binned && ((flags & ACE_PERSISTENT) ||
                              (!(flags & (ACE_ORDERED | ACE_BUCKETED)) && t.auto_persistent));
    p.max_pos = total + 64ull * kBins;
    p.tstride = graph ? (total + kTile - 1) / kTile + n_blocks : tiles;
    if (p.tstride < 1) p.tstride = 1;
    const bool table = graph || n_blocks > 1;
    size_t o = 0;
    p.off_ctrl = o;  o = align_up(o + sizeof(Ctrl), 256);
    p.off_hdr = o;   o = align_up(o + (graph ? sizeof(BatchHdr) : 0), 256);
    p.off_descs = o; o = align_up(o + (table ? (size_t)n_blocks * sizeof(DevBlock) : 0), 256);
    p.off_mid = o;   o = align_up(o + (p.rev && !p.per_tx ? 64ull * keys->n_id : 0), 256);
    p.off_thist = o; o = align_up(o + (binned ? 4ull * kBins * p.tstride : 0), 256);
    p.off_perm = o;  o = align_up(o + (binned ? 8ull * p.max_pos : 0), 256);
    p.off_rec = o;   o = align_up(o + (binned ? sizeof(TxRec) * p.max_pos : 0), 256);
    p.off_posof = o; o = align_up(o + (binned ? 4ull * total : 0), 256);
    p.off_vperm = o; o = align_up(o + (binned ? 4ull * (p.max_pos / 32 + 2) : 0), 256);
    p.bytes = o;
}

int make_plan(const ace_keyset *keys, const ace_block *blocks, uint32_t n_blocks, uint32_t flags,
              Plan &p, bool attest = false)
{
    int rc = check_keyset(keys, flags, p);
    if (rc) return rc;
    p.attest = attest;
    uint64_t total, tiles, waves;
    if ((rc = check_blocks(blocks, n_blocks, total, tiles, waves))) return rc;
    p.total_tx = total;
    p.total_tiles = tiles;
    p.total_waves = waves;
    layout(keys, n_blocks, total, tiles, flags, false, p);
    return ACE_OK;
}

unsigned grid_for(uint64_t items, uint64_t per_wg, unsigned cap)
{
    uint64_t g = (items + per_wg - 1) / per_wg;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

DevBlock dev_block(const ace_block &k)
{
    DevBlock d;
    memset(&d, 0, sizeof d);
    d.msg = k.d_msg;
    d.off = k.d_off;
    d.id = k.d_id;
    d.tag = k.d_tag;
    d.bitmask = k.d_bitmask_out;
    d.count = reinterpret_cast<unsigned long long *>(k.d_count_out);
    d.n = k.n_tx;
    return d;
}

// A second stream per thread and device on which the key derivation runs
// beside the binning passes: forked from and joined back to the caller's
// stream with events (under graph capture, two branches of the graph).  When
// a thread ends, its contexts go to a process-wide free list that later
// threads take from, so threads that come and go do not add streams; the
// list itself is never destroyed (no HIP calls during process exit).
struct Fork {
    int dev;
    hipStream_t aux;
    hipEvent_t fork, join;
    hipEvent_t mark;  // timing-enabled marker on the caller's stream, see below
};

std::mutex g_fork_mu;
std::vector<Fork> *g_fork_free = new std::vector<Fork>();

struct ForkCache {
    std::vector<Fork> forks;
    ~ForkCache()
    {
        std::lock_guard<std::mutex> lock(g_fork_mu);
        for (const Fork &f : forks) g_fork_free->push_back(f);
    }
};

bool fork_create(int dev, Fork &f)
{
    f = Fork{dev, nullptr, nullptr, nullptr, nullptr};
    bool ok = hipStreamCreateWithFlags(&f.aux, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&f.fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&f.join, hipEventDisableTiming) == hipSuccess &&
              hipEventCreate(&f.mark) == hipSuccess;
    if (!ok) {
        if (f.mark) (void)hipEventDestroy(f.mark);
        if (f.join) (void)hipEventDestroy(f.join);
        if (f.fork) (void)hipEventDestroy(f.fork);
        if (f.aux) (void)hipStreamDestroy(f.aux);
    }
    return ok;
}

Fork *fork_ctx()
{
    thread_local ForkCache cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    for (auto &f : cache.forks)
        if (f.dev == dev) return &f;
    Fork f{};
    bool have = false;
    {
        std::lock_guard<std::mutex> lock(g_fork_mu);
        for (size_t i = 0; i < g_fork_free->size(); ++i) {
            if ((*g_fork_free)[i].dev == dev) {
                f = (*g_fork_free)[i];
                (*g_fork_free)[i] = g_fork_free->back();
                g_fork_free->pop_back();
                have = true;
                break;
            }
        }
    }
    if (!have && !fork_create(dev, f)) return nullptr;
    cache.forks.push_back(f);
    return &cache.forks.back();
}

// Workgroups of the count pass: each adds to a block's count at most once.
constexpr uint64_t kCountWGs = 256;

// Verify-kernel launches for the plan's key source, persistence and record form.
template <bool PT, bool AT>
void launch_ordered_t(unsigned g, hipStream_t s, const Batch &bt, const KeySource &ks,
                      const HkdfParams &hp)
{
    hipLaunchKernelGGL((k_verify_ordered<PT, AT>), dim3(g), dim3(kWG), 0, s, bt, ks, hp);
}

void launch_ordered(const Plan &p, unsigned g, hipStream_t s, const Batch &bt, const KeySource &ks,
                    const HkdfParams &hp)
{
    if (p.attest) {
        if (p.per_tx) launch_ordered_t<true, true>(g, s, bt, ks, hp);
        else launch_ordered_t<false, true>(g, s, bt, ks, hp);
    } else {
        if (p.per_tx) launch_ordered_t<true, false>(g, s, bt, ks, hp);
        else launch_ordered_t<false, false>(g, s, bt, ks, hp);
    }
}

template <bool PT, bool PE, bool AT>
void launch_binned_t(unsigned g, hipStream_t s, const Batch &bt, const KeySource &ks,
                     const HkdfParams &hp, Ctrl *ctrl, const unsigned long long *perm,
                     const TxRec *rec, uint32_t *vperm, const GrabCaps &caps)
{
    hipLaunchKernelGGL((k_verify_binned<PT, PE, AT>), dim3(g), dim3(kWG), 0, s, bt, ks, hp, ctrl,
                       perm, rec, vperm, caps);
}

void launch_binned(const Plan &p, unsigned g, hipStream_t s, const Batch &bt, const KeySource &ks,
                   const HkdfParams &hp, Ctrl *ctrl, const unsigned long long *perm,
                   const TxRec *rec, uint32_t *vperm, const GrabCaps &caps)
{
#define ACE_B(PT, PE, AT) launch_binned_t<PT, PE, AT>(g, s, bt, ks, hp, ctrl, perm, rec, vperm, caps)
    if (p.attest) {
        if (p.per_tx) { if (p.persistent) ACE_B(true, true, true); else ACE_B(true, false, true); }
        else { if (p.persistent) ACE_B(false, true, true); else ACE_B(false, false, true); }
    } else {
        if (p.per_tx) { if (p.persistent) ACE_B(true, true, false); else ACE_B(true, false, false); }
        else { if (p.persistent) ACE_B(false, true, false); else ACE_B(false, false, false); }
    }
#undef ACE_B
}

// The launch sequence after the block table is in place.  `graph` marks a
// capture: sizes then come from the device header and every grid is fixed.
// `fork`: a binned call with keys derived in it may run the derivation on
// the thread's second stream (created on first use); without it the
// derivation runs first on `s`.
int enqueue_stages(const Plan &p, const Batch &bt, const ace_keyset *keys, const HkdfParams &hp,
                   uint8_t *ws, hipStream_t s, ProfCall *prof, bool graph, bool fork = true)
{
    int rc;
    const ace_tuning tn = tuning();
    const unsigned cus = (unsigned)cu_count();
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(ws + p.off_ctrl);
    const bool binned = p.mode == kBinned;

    KeySource ks;
    ks.n_id = keys->n_id;
    ks.mid = nullptr;
    ks.rev = nullptr;
    // keys derived in the call: in the binned form the derivation (VALU-bound)
    // runs on a second stream beside the binning passes (memory-bound), which
    // do not depend on it; the verify kernel waits for both
    Fork *fk = nullptr;
    if (!p.rev) {
        ks.mid = keys->d_mid;
    } else if (p.per_tx) {
        ks.rev = keys->d_rev;
    } else {
        uint32_t *mid = reinterpret_cast<uint32_t *>(ws + p.off_mid);
        if (keys->n_id) {
            unsigned g = std::min<unsigned>((unsigned)((keys->n_id + kWG - 1) / kWG),
                                            kDeriveWgsPerCu * cus);
            hipStream_t ds = s;
            if (fork && binned && (graph || p.total_tx) && (fk = fork_ctx())) {
                if ((rc = check_hip(hipEventRecord(fk->fork, s), "hipEventRecord"))) return rc;
                if ((rc = check_hip(hipStreamWaitEvent(fk->aux, fk->fork, 0), "hipStreamWaitEvent")))
                    return rc;
                ds = fk->aux;
                // leave wave slots to the binning passes on the caller's stream
                if (tn.derive_wgs_per_cu) g = std::min<unsigned>(g, tn.derive_wgs_per_cu * cus);
            }
            hipLaunchKernelGGL(k_derive, dim3(g), dim3(kWG), 0, ds, keys->d_rev, keys->n_id,
                               (uint8_t *)nullptr, mid, hp);
            if ((rc = launch_status("k_derive launch"))) return rc;
            if (fk) {
                if ((rc = check_hip(hipEventRecord(fk->join, fk->aux), "hipEventRecord"))) return rc;
                // A timing-enabled marker on the caller's stream right after the
                // derivation's launch: without it the binning kernels took the
                // CUs first and the derivation ran after them (measured at 16M
                // transactions: 5.2 ms per step without, 4.4 ms with).
                if ((rc = check_hip(hipEventRecord(fk->mark, s), "hipEventRecord"))) return rc;
            }
        }
        ks.mid = mid;
    }
    prof_mark(prof, 1, s);

    if (!graph) {
        hipLaunchKernelGGL(k_zero, dim3(grid_for(p.n_blocks, kWG, 1024)), dim3(kWG), 0, s, bt,
                           binned ? ctrl : (Ctrl *)nullptr);
        if ((rc = launch_status("k_zero launch"))) return rc;
    }

    if (!binned) {
        prof_mark(prof, 2, s);
        if (graph || p.total_tx) {
            const unsigned g = graph ? tn.verify_wgs_per_cu * cus
                                     : grid_for(p.total_waves, kWavesPerWG, 0x7fffffffu);
            launch_ordered(p, g, s, bt, ks, hp);
            if ((rc = launch_status("k_verify_ordered launch"))) return rc;
        }
        prof_mark(prof, 3, s);
        if (graph || p.total_tx) {
            hipLaunchKernelGGL(k_count, dim3(grid_for(graph ? (p.total_tx + kTile - 1) / kTile + p.n_blocks
                                                            : p.total_tiles, 1, kCountWGs)),
                               dim3(kWG), 0, s, bt);
            if ((rc = launch_status("k_count launch"))) return rc;
        }
        prof_mark(prof, 4, s);
        return ACE_OK;
    }
    if (!graph && p.total_tx == 0) {
        for (int k = 2; k <= 4; ++k) prof_mark(prof, k, s);
        return ACE_OK;
    }

    unsigned long long *perm = reinterpret_cast<unsigned long long *>(ws + p.off_perm);
    TxRec *rec = reinterpret_cast<TxRec *>(ws + p.off_rec);
    uint32_t *pos_of = reinterpret_cast<uint32_t *>(ws + p.off_posof);
    uint32_t *vperm = reinterpret_cast<uint32_t *>(ws + p.off_vperm);
    const uint64_t tiles_bound = graph ? (p.total_tx + kTile - 1) / kTile + p.n_blocks : p.total_tiles;
    const unsigned gtiles = grid_for(tiles_bound, 1, tn.aux_wgs_per_cu * cus);

    uint32_t *thist = reinterpret_cast<uint32_t *>(ws + p.off_thist);
    hipLaunchKernelGGL(k_bin_count, dim3(gtiles), dim3(kWG), 0, s, bt, thist, p.tstride, keys->n_id);
    if ((rc = launch_status("k_bin_count launch"))) return rc;
    hipLaunchKernelGGL(k_bin_scan, dim3(kBins), dim3(kScanWG), 0, s, bt, ctrl, thist, p.tstride);
    if ((rc = launch_status("k_bin_scan launch"))) return rc;
    hipLaunchKernelGGL(k_bin_scatter, dim3(gtiles), dim3(kWG), 0, s, bt, ctrl, thist, p.tstride,
                       keys->n_id, perm, rec,
                       pos_of, tn.wide_min_len);
    if ((rc = launch_status("k_bin_scatter launch"))) return rc;
    if (fk && (rc = check_hip(hipStreamWaitEvent(s, fk->join, 0), "hipStreamWaitEvent"))) return rc;
    prof_mark(prof, 2, s);

    {
        const unsigned g = p.persistent ? tn.verify_wgs_per_cu * cus
                                        : grid_for(p.max_pos / 64, kWavesPerWG, 0x7fffffffu);
        GrabCaps caps;
        static_assert(sizeof caps.cap == sizeof tn.grab_cap, "one cap per length bucket");
        memcpy(caps.cap, tn.grab_cap, sizeof caps.cap);
        launch_binned(p, g, s, bt, ks, hp, ctrl, perm, rec, vperm, caps);
    }
    if ((rc = launch_status("k_verify_binned launch"))) return rc;
    prof_mark(prof, 3, s);
    hipLaunchKernelGGL(k_finalize, dim3(gtiles), dim3(kWG), 0, s, bt, pos_of, vperm);
    if ((rc = launch_status("k_finalize launch"))) return rc;
    hipLaunchKernelGGL(k_count, dim3(grid_for(tiles_bound, 1, kCountWGs)), dim3(kWG), 0, s, bt);
    if ((rc = launch_status("k_count launch"))) return rc;
    prof_mark(prof, 4, s);
    return ACE_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Graph object.
// ------------------------------------------------------------------------------------------
struct ace_graph {
    int device;
    Plan plan;
    uint32_t max_blocks;
    uint64_t max_tx;
    struct Slot {
        DevBlock *h_descs;  // pinned, read by k_plan at replay time
        uint32_t *h_n;
        hipGraph_t graph;
        hipGraphExec_t exec;
        hipEvent_t done;
        bool used;
    } slot[2];
    int next;
    hipStream_t capture;
};

namespace {

void graph_free(ace_graph *g)
{
    if (!g) return;
    for (auto &sl : g->slot) {
        if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
        if (sl.graph) (void)hipGraphDestroy(sl.graph);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.h_descs) (void)hipHostFree(sl.h_descs);
    }
    if (g->capture) (void)hipStreamDestroy(g->capture);
    delete g;
}

}  // namespace

extern "C" {

ACE_API const char *ace_last_error(void) { return g_err; }

ACE_API const char *ace_version(void) { return "ace 0.2 gfx950"; }

ACE_API int ace_valu_rate(uint32_t iters, uint32_t wgs_per_cu, uint32_t *d_sink,
                          double *out_lane_instr_per_s, void *stream)
{
    clear_error();
    if (!out_lane_instr_per_s || !d_sink) return fail(ACE_ERR_INVALID_ARG, "NULL output");
    if (!aligned(d_sink, 4)) return fail(ACE_ERR_INVALID_ARG, "d_sink not 4-byte aligned");
    if (iters < 1 || wgs_per_cu < 1 || wgs_per_cu > 64)
        return fail(ACE_ERR_INVALID_ARG, "iters >= 1 and wgs_per_cu in 1..64");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const unsigned g = (unsigned)cu_count() * wgs_per_cu;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int rc = check_hip(hipEventCreate(&ev[0]), "hipEventCreate");
    if (!rc) rc = check_hip(hipEventCreate(&ev[1]), "hipEventCreate");
    if (!rc) rc = check_hip(hipEventRecord(ev[0], s), "hipEventRecord");
    if (!rc) {
        hipLaunchKernelGGL(k_valu_rate, dim3(g), dim3(256), 0, s, iters, 1u, d_sink);
        rc = launch_status("k_valu_rate launch");
    }
    if (!rc) rc = check_hip(hipEventRecord(ev[1], s), "hipEventRecord");
    if (!rc) rc = check_hip(hipEventSynchronize(ev[1]), "hipEventSynchronize");
    float ms = 0.f;
    if (!rc) rc = check_hip(hipEventElapsedTime(&ms, ev[0], ev[1]), "hipEventElapsedTime");
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc) return rc;
    const double lanes = (double)g * 256.0;
    const double instr = (double)iters * kValuStepsPerIter * kValuOpsPerStep;
    *out_lane_instr_per_s = ms > 0.f ? lanes * instr / (ms * 1e-3) : 0.0;
    return ACE_OK;
}

ACE_API int ace_get_tuning(ace_tuning *out)
{
    clear_error();
    if (!out) return fail(ACE_ERR_INVALID_ARG, "out is NULL");
    *out = tuning();
    return ACE_OK;
}

ACE_API int ace_set_tuning(const ace_tuning *t)
{
    clear_error();
    if (!t) return fail(ACE_ERR_INVALID_ARG, "tuning is NULL");
    if (t->verify_wgs_per_cu < 1 || t->verify_wgs_per_cu > 64 || t->aux_wgs_per_cu < 1 ||
        t->aux_wgs_per_cu > 64 || t->derive_wgs_per_cu > 64)
        return fail(ACE_ERR_INVALID_ARG, "workgroups per CU must be in 1..64 (derive: 0..64)");
    if (t->wide_min_len < 1 || t->wide_min_len > kRecMaxLen)
        return fail(ACE_ERR_INVALID_ARG, "wide_min_len must be in 1..2^31 - 1");
    for (int b = 0; b < ACE_LENGTH_BUCKETS; ++b)
        if (t->grab_cap[b] > kGrab)
            return fail(ACE_ERR_INVALID_ARG, "grab_cap[%d] = %u exceeds %u", b, t->grab_cap[b], kGrab);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune = *t;
    return ACE_OK;
}

ACE_API int ace_derive_keys(const uint8_t *d_rev, uint32_t n_id, const uint8_t *h_salt,
                            size_t salt_len, const uint8_t *h_info, size_t info_len,
                            uint8_t *d_key_out, uint32_t *d_mid_out, void *stream)
{
    clear_error();
    if (!d_key_out && !d_mid_out) return fail(ACE_ERR_INVALID_ARG, "d_key_out and d_mid_out are both NULL");
    HkdfParams hp;
    int rc = fill_hkdf(hp, h_salt, salt_len, h_info, info_len);
    if (rc) return rc;
    if (n_id == 0) return ACE_OK;
    if (!d_rev) return fail(ACE_ERR_INVALID_ARG, "d_rev is NULL");
    if (!aligned(d_rev, 4) || (d_key_out && !aligned(d_key_out, 4)) || (d_mid_out && !aligned(d_mid_out, 4)))
        return fail(ACE_ERR_INVALID_ARG, "misaligned device array");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const unsigned grid = std::min<unsigned>((unsigned)((n_id + kWG - 1) / kWG),
                                             kDeriveWgsPerCu * (unsigned)cu_count());
    hipLaunchKernelGGL(k_derive, dim3(grid), dim3(kWG), 0, s, d_rev, n_id, d_key_out, d_mid_out, hp);
    return launch_status("k_derive launch");
}

ACE_API int ace_derive_keys_multi(const uint8_t *d_rev, uint32_t n_id,
                                  const ace_hkdf_stream *h_streams, uint32_t n_streams,
                                  uint8_t *d_key_out, uint32_t *d_mid_out, void *stream)
{
    clear_error();
    if (!d_key_out && !d_mid_out) return fail(ACE_ERR_INVALID_ARG, "d_key_out and d_mid_out are both NULL");
    if (n_streams && !h_streams) return fail(ACE_ERR_INVALID_ARG, "h_streams is NULL");
    for (uint32_t k = 0; k < n_streams; ++k) {
        const ace_hkdf_stream &t = h_streams[k];
        if (t.salt_len > kMultiSalt || t.info_len > kMultiInfo)
            return fail(ACE_ERR_INVALID_ARG, "stream %u: salt_len %zu / info_len %zu exceed %u / %u", k,
                        t.salt_len, t.info_len, kMultiSalt, kMultiInfo);
        if ((t.salt_len && !t.h_salt) || (t.info_len && !t.h_info))
            return fail(ACE_ERR_INVALID_ARG, "stream %u: NULL salt or info with nonzero length", k);
    }
    if (n_id == 0 || n_streams == 0) return ACE_OK;
    if (!d_rev) return fail(ACE_ERR_INVALID_ARG, "d_rev is NULL");
    if (!aligned(d_rev, 4) || (d_key_out && !aligned(d_key_out, 4)) || (d_mid_out && !aligned(d_mid_out, 4)))
        return fail(ACE_ERR_INVALID_ARG, "misaligned device array");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const unsigned gx = (unsigned)((n_id + kWG - 1) / kWG);
    for (uint32_t first = 0; first < n_streams; first += kMultiStreams) {
        MultiHkdf mp;
        memset(&mp, 0, sizeof mp);
        mp.first = first;
        mp.count = std::min<uint32_t>(kMultiStreams, n_streams - first);
        for (uint32_t y = 0; y < mp.count; ++y) {
            const ace_hkdf_stream &t = h_streams[first + y];
            mp.s[y].salt_len = (uint32_t)t.salt_len;
            mp.s[y].info_len = (uint32_t)t.info_len;
            if (t.salt_len) memcpy(mp.s[y].salt, t.h_salt, t.salt_len);
            if (t.info_len) memcpy(mp.s[y].info, t.h_info, t.info_len);
        }
        hipLaunchKernelGGL(k_derive_multi, dim3(gx, mp.count), dim3(kWG), 0, s, d_rev, n_id, d_key_out,
                           d_mid_out, mp);
        int rc = launch_status("k_derive_multi launch");
        if (rc) return rc;
    }
    return ACE_OK;
}

ACE_API int ace_poh_verify(const uint8_t *d_start, const uint8_t *d_end, const uint32_t *d_steps,
                           uint32_t steps, uint64_t n_segments, uint32_t *d_bitmask_out,
                           uint64_t *d_count_out, void *stream)
{
    clear_error();
    if (!d_count_out) return fail(ACE_ERR_INVALID_ARG, "d_count_out is NULL");
    if (!aligned(d_count_out, 8)) return fail(ACE_ERR_INVALID_ARG, "d_count_out not 8-byte aligned");
    if (n_segments > ACE_MAX_TX) return fail(ACE_ERR_RANGE, "n_segments too large");
    if (n_segments) {
        if (!d_start || !d_end || !d_bitmask_out)
            return fail(ACE_ERR_INVALID_ARG, "NULL array with n_segments > 0");
        if (!aligned(d_start, 4) || !aligned(d_end, 4) || !aligned(d_bitmask_out, 4) ||
            (d_steps && !aligned(d_steps, 4)))
            return fail(ACE_ERR_INVALID_ARG, "misaligned device array");
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(d_count_out);
    hipLaunchKernelGGL(k_poh_zero, dim3(1), dim3(1), 0, s, cnt);
    int rc = launch_status("k_poh_zero launch");
    if (rc || !n_segments) return rc;
    const unsigned g = (unsigned)((n_segments + kWG - 1) / kWG);
    hipLaunchKernelGGL(k_poh_verify, dim3(g), dim3(kWG), 0, s, d_start, d_end, d_steps, steps,
                       n_segments, d_bitmask_out, cnt);
    return launch_status("k_poh_verify launch");
}

}  // extern "C"

namespace {

struct MerklePlan {
    uint64_t total;    // leaves of all trees
    uint32_t levels;   // reductions of the largest tree
    size_t off_table, off_nodes, off_prefix, bytes;
};

int merkle_plan(const ace_merkle_tree *trees, uint32_t n_trees, MerklePlan &p)
{
    if (n_trees && !trees) return fail(ACE_ERR_INVALID_ARG, "trees is NULL");
    if (n_trees >= (1u << 24)) return fail(ACE_ERR_RANGE, "n_trees %u >= 2^24", n_trees);
    p.total = 0;
    p.levels = 0;
    for (uint32_t b = 0; b < n_trees; ++b) {
        const ace_merkle_tree &t = trees[b];
        if (!t.d_root_out) return fail(ACE_ERR_INVALID_ARG, "tree %u: d_root_out is NULL", b);
        if (!aligned(t.d_root_out, 4)) return fail(ACE_ERR_INVALID_ARG, "tree %u: d_root_out not 4-byte aligned", b);
        if (t.n_leaves) {
            if (!t.d_data || !t.d_off) return fail(ACE_ERR_INVALID_ARG, "tree %u: NULL array with n_leaves > 0", b);
            if (!aligned(t.d_off, 8)) return fail(ACE_ERR_INVALID_ARG, "tree %u: d_off not 8-byte aligned", b);
        }
        if (t.n_leaves > ACE_MAX_TX) return fail(ACE_ERR_RANGE, "tree %u: n_leaves too large", b);
        p.total += t.n_leaves;
        if (p.total > ACE_MAX_TX) return fail(ACE_ERR_RANGE, "total leaves exceed ACE_MAX_TX");
        uint32_t lv = 0;
        while (lv < 63 && (1ull << lv) < t.n_leaves) ++lv;
        p.levels = std::max(p.levels, lv);
    }
    size_t o = 0;
    p.off_table = o;  o = align_up(o + sizeof(MerkleDesc) * (size_t)n_trees, 256);
    p.off_nodes = o;  o = align_up(o + 32ull * p.total, 256);
    p.off_prefix = o; o = align_up(o + 8ull * p.levels * (n_trees + 1ull), 256);
    p.bytes = std::max<size_t>(o, 256);
    return ACE_OK;
}

}  // namespace

extern "C" {

ACE_API size_t ace_merkle_workspace_size(const ace_merkle_tree *trees, uint32_t n_trees)
{
    MerklePlan p{};
    if (merkle_plan(trees, n_trees, p) != ACE_OK) return 0;
    return p.bytes;
}

ACE_API int ace_merkle_roots(const ace_merkle_tree *trees, uint32_t n_trees, void *d_workspace,
                             size_t ws_bytes, void *stream)
{
    clear_error();
    MerklePlan p{};
    int rc = merkle_plan(trees, n_trees, p);
    if (rc) return rc;
    if (n_trees == 0) return ACE_OK;
    if (!d_workspace) return fail(ACE_ERR_INVALID_ARG, "d_workspace is NULL");
    if (!aligned(d_workspace, 256)) return fail(ACE_ERR_INVALID_ARG, "d_workspace not 256-byte aligned");
    if (ws_bytes < p.bytes) return fail(ACE_ERR_NO_MEMORY, "workspace %zu bytes, need %zu", ws_bytes, p.bytes);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t *ws = static_cast<uint8_t *>(d_workspace);
    MerkleDesc *table = reinterpret_cast<MerkleDesc *>(ws + p.off_table);
    uint32_t *nodes = reinterpret_cast<uint32_t *>(ws + p.off_nodes);
    unsigned long long *P = reinterpret_cast<unsigned long long *>(ws + p.off_prefix);

    MerkleChunk chunk;
    memset(&chunk, 0, sizeof chunk);
    uint64_t leaf0 = 0;
    for (uint32_t b = 0; b < n_trees; ++b) {
        MerkleDesc &d = chunk.d[chunk.count++];
        d.data = trees[b].d_data;
        d.off = trees[b].d_off;
        d.n = trees[b].n_leaves;
        d.root = trees[b].d_root_out;
        d.leaf0 = leaf0;
        leaf0 += d.n;
        if (chunk.count == kMerkleChunk || b + 1 == n_trees) {
            hipLaunchKernelGGL(k_merkle_put, dim3(1), dim3(kMerkleChunk), 0, s, table, chunk);
            if ((rc = launch_status("k_merkle_put launch"))) return rc;
            chunk.first = b + 1;
            chunk.count = 0;
        }
    }
    if (p.total) {
        hipLaunchKernelGGL(k_merkle_leaves, dim3((unsigned)((p.total + kWG - 1) / kWG)), dim3(kWG), 0, s,
                           table, n_trees, p.total, nodes);
        if ((rc = launch_status("k_merkle_leaves launch"))) return rc;
    }
    // levels below k0 one launch each over all trees; from k0, where no tree
    // has more than kTopNodes nodes, one launch for the rest
    uint32_t k0 = 0;
    for (uint32_t b = 0; b < n_trees; ++b)
        while (((trees[b].n_leaves + (1ull << k0) - 1) >> k0) > kTopNodes) ++k0;
    if (k0 > p.levels) k0 = p.levels;
    if (k0) {
        hipLaunchKernelGGL(k_merkle_plan, dim3(k0), dim3(kPlanThreads), 0, s, table, n_trees, P);
        if ((rc = launch_status("k_merkle_plan launch"))) return rc;
    }
    for (uint32_t k = 0; k < k0; ++k) {
        // this level's pairs over all trees, as the plan kernel counts them
        uint64_t pairs = 0;
        for (uint32_t b = 0; b < n_trees; ++b) {
            const uint64_t n = trees[b].n_leaves;
            pairs += ((n + (1ull << k) - 1) >> k) >> 1;
        }
        if (!pairs) continue;
        hipLaunchKernelGGL(k_merkle_level, dim3((unsigned)((pairs + kWG - 1) / kWG)), dim3(kWG), 0, s, table,
                           n_trees, k, P + (uint64_t)k * (n_trees + 1ull), nodes);
        if ((rc = launch_status("k_merkle_level launch"))) return rc;
    }
    if (k0 < p.levels) {
        hipLaunchKernelGGL(k_merkle_top, dim3(n_trees), dim3(kTopWG), 0, s, table, k0, nodes);
        if ((rc = launch_status("k_merkle_top launch"))) return rc;
    }
    hipLaunchKernelGGL(k_merkle_out, dim3((n_trees + kWG - 1) / kWG), dim3(kWG), 0, s, table, n_trees, nodes);
    return launch_status("k_merkle_out launch");
}

ACE_API size_t ace_verify_workspace_size(const ace_keyset *keys, const ace_block *blocks,
                                         uint32_t n_blocks, uint32_t flags)
{
    Plan p{};
    if (make_plan(keys, blocks, n_blocks, flags, p) != ACE_OK) return 0;
    return p.bytes;
}

}  // extern "C"

namespace {

// The block table and the launch sequence of a checked call, with `ws` as its
// workspace.  `noalloc`: no stage events, no second stream (both are created
// on first use).
int run_plan(const Plan &p, const ace_keyset *keys, const ace_block *blocks, uint32_t n_blocks,
             const HkdfParams &hp, uint8_t *ws, void *stream, bool noalloc)
{
    int rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ProfCall *prof = noalloc ? nullptr : prof_begin(s);
    DevBlock *table = reinterpret_cast<DevBlock *>(ws + p.off_descs);

    Batch bt;
    memset(&bt, 0, sizeof bt);
    bt.n_blocks = n_blocks;
    bt.total_tx = p.total_tx;
    bt.total_tiles = p.total_tiles;
    bt.total_waves = p.total_waves;
    DescChunk chunk;
    memset(&chunk, 0, sizeof chunk);
    uint64_t tx0 = 0, tile0 = 0, wave0 = 0;
    for (uint32_t b = 0; b < n_blocks; ++b) {
        DevBlock d = dev_block(blocks[b]);
        d.tx0 = tx0;
        d.tile0 = tile0;
        d.wave0 = wave0;
        tx0 += d.n;
        tile0 += (d.n + kTile - 1) / kTile;
        wave0 += (d.n + 63) / 64;
        if (n_blocks == 1) {
            bt.one = d;
            break;
        }
        chunk.d[chunk.count++] = d;
        if (chunk.count == kDescChunk || b + 1 == n_blocks) {
            hipLaunchKernelGGL(k_put_descs, dim3(1), dim3(64), 0, s, table, chunk);
            if ((rc = launch_status("k_put_descs launch"))) return rc;
            chunk.first = b + 1;
            chunk.count = 0;
        }
    }
    bt.table = n_blocks > 1 ? table : nullptr;
    return enqueue_stages(p, bt, keys, hp, ws, s, prof, false, !noalloc);
}

int verify_impl(const ace_keyset *keys, const ace_block *blocks, uint32_t n_blocks,
                void *d_workspace, size_t ws_bytes, uint32_t flags, void *stream, bool attest)
{
    clear_error();
    Plan p{};
    int rc = make_plan(keys, blocks, n_blocks, flags, p, attest);
    if (rc) return rc;
    if (n_blocks == 0) return ACE_OK;
    if (!d_workspace) return fail(ACE_ERR_INVALID_ARG, "d_workspace is NULL");
    if (!aligned(d_workspace, 256)) return fail(ACE_ERR_INVALID_ARG, "d_workspace not 256-byte aligned");
    if (ws_bytes < p.bytes)
        return fail(ACE_ERR_NO_MEMORY, "workspace %zu bytes, need %zu", ws_bytes, p.bytes);
    HkdfParams hp;
    memset(&hp, 0, sizeof hp);
    if (p.rev && (rc = fill_hkdf(hp, keys->h_salt, keys->salt_len, keys->h_info, keys->info_len)))
        return rc;
    return run_plan(p, keys, blocks, n_blocks, hp, static_cast<uint8_t *>(d_workspace), stream,
                    false);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Scratch memory of ace_verify_batch_noalloc: a static device array that every
// GPU the library runs on holds until the process ends.  Its name in host code
// is only a stand-in for the symbol; kernels get the device address that
// hipGetSymbolAddress returns for the current device.
// ------------------------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[ACE_SCRATCH_BYTES];

namespace {

// This device's address of `scratch`, looked up once per device (with that
// device current) on the first no-allocation call there.
int scratch_base(uint8_t **out)
{
    static std::mutex mu;
    static std::vector<uint8_t *> base;
    int dev = 0;
    int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)base.size() <= dev) base.resize(dev + 1, nullptr);
    if (!base[dev]) {
        void *ptr = nullptr;
        if ((rc = check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress")))
            return rc;
        if (!ptr || !aligned(ptr, 256))
            return fail(ACE_ERR_DEVICE, "scratch array at %p is not 256-byte aligned", ptr);
        base[dev] = static_cast<uint8_t *>(ptr);
    }
    *out = base[dev];
    return ACE_OK;
}

}  // namespace

extern "C" {

ACE_API int ace_verify_batch(const ace_keyset *keys, const ace_block *blocks, uint32_t n_blocks,
                             void *d_workspace, size_t ws_bytes, uint32_t flags, void *stream)
{
    return verify_impl(keys, blocks, n_blocks, d_workspace, ws_bytes, flags, stream, false);
}

ACE_API int ace_verify_attestations(const ace_keyset *keys, const ace_block *blocks,
                                    uint32_t n_blocks, void *d_workspace, size_t ws_bytes,
                                    uint32_t flags, void *stream)
{
    return verify_impl(keys, blocks, n_blocks, d_workspace, ws_bytes, flags, stream, true);
}

ACE_API int ace_verify_batch_noalloc(const ace_keyset *keys, const ace_block *blocks,
                                     uint32_t n_blocks, uint32_t flags, void *stream)
{
    clear_error();
    Plan p{};
    int rc = make_plan(keys, blocks, n_blocks, flags, p, false);
    if (rc) return rc;
    if (n_blocks == 0) return ACE_OK;
    if (p.bytes > (size_t)ACE_SCRATCH_BYTES)
        return fail(ACE_ERR_TOO_LARGE,
                    "the call needs %zu bytes of scratch, the library holds %zu per device "
                    "(ace_verify_batch takes a workspace of any size)",
                    p.bytes, (size_t)ACE_SCRATCH_BYTES);
    HkdfParams hp;
    memset(&hp, 0, sizeof hp);
    if (p.rev && (rc = fill_hkdf(hp, keys->h_salt, keys->salt_len, keys->h_info, keys->info_len)))
        return rc;
    uint8_t *ws = nullptr;
    if ((rc = scratch_base(&ws))) return rc;
    return run_plan(p, keys, blocks, n_blocks, hp, ws, stream, true);
}

ACE_API int ace_profile_enable(int on)
{
    clear_error();
    g_prof.on = on != 0;
    return ACE_OK;
}

ACE_API int ace_profile_read(ace_profile *out, int reset)
{
    clear_error();
    if (!out) return fail(ACE_ERR_INVALID_ARG, "out is NULL");
    memset(out, 0, sizeof *out);
    for (size_t i = 0; i < g_prof.used; ++i) {
        ProfCall &c = g_prof.calls[i];
        float ms[4];
        for (int k = 0; k < 4; ++k) {
            int rc = check_hip(hipEventSynchronize(c.ev[k + 1]), "hipEventSynchronize");
            if (rc) return rc;
            rc = check_hip(hipEventElapsedTime(&ms[k], c.ev[k], c.ev[k + 1]), "hipEventElapsedTime");
            if (rc) return rc;
        }
        out->derive_ms += ms[0];
        out->bin_ms += ms[1];
        out->verify_ms += ms[2];
        out->finalize_ms += ms[3];
        out->total_ms += ms[0] + ms[1] + ms[2] + ms[3];
        out->calls += 1;
    }
    if (reset) g_prof.used = 0;
    return ACE_OK;
}

ACE_API size_t ace_graph_workspace_size(const ace_keyset *keys, uint32_t max_blocks, uint64_t max_tx,
                                        uint32_t flags)
{
    Plan p{};
    if (check_keyset(keys, flags, p) != ACE_OK) return 0;
    if (max_blocks == 0 || max_blocks >= (1u << 24) || max_tx > ACE_MAX_TX) return 0;
    layout(keys, max_blocks, max_tx, 0, flags, true, p);
    return p.bytes;
}

ACE_API int ace_graph_create(const ace_keyset *keys, uint32_t max_blocks, uint64_t max_tx,
                             void *d_workspace, size_t ws_bytes, uint32_t flags, ace_graph **out)
{
    clear_error();
    if (!out) return fail(ACE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    Plan p{};
    int rc = check_keyset(keys, flags, p);
    if (rc) return rc;
    if (max_blocks == 0) return fail(ACE_ERR_INVALID_ARG, "max_blocks is 0");
    if (max_blocks >= (1u << 24)) return fail(ACE_ERR_RANGE, "max_blocks >= 2^24");
    if (max_tx > ACE_MAX_TX) return fail(ACE_ERR_RANGE, "max_tx exceeds ACE_MAX_TX");
    layout(keys, max_blocks, max_tx, 0, flags, true, p);
    p.total_tx = max_tx;
    p.total_tiles = 0;
    p.total_waves = 0;
    if (!d_workspace || !aligned(d_workspace, 256))
        return fail(ACE_ERR_INVALID_ARG, "d_workspace NULL or not 256-byte aligned");
    if (ws_bytes < p.bytes) return fail(ACE_ERR_NO_MEMORY, "workspace %zu bytes, need %zu", ws_bytes, p.bytes);
    HkdfParams hp;
    memset(&hp, 0, sizeof hp);
    if (p.rev && (rc = fill_hkdf(hp, keys->h_salt, keys->salt_len, keys->h_info, keys->info_len)))
        return rc;

    (void)cu_count();  // device queries happen before the capture starts
    ace_graph *g = new ace_graph;
    memset(g, 0, sizeof *g);
    g->plan = p;
    g->max_blocks = max_blocks;
    g->max_tx = max_tx;
    if ((rc = check_hip(hipGetDevice(&g->device), "hipGetDevice")) ||
        (rc = check_hip(hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking), "hipStreamCreate"))) {
        graph_free(g);
        return rc;
    }
    uint8_t *ws = static_cast<uint8_t *>(d_workspace);
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(ws + p.off_ctrl);
    BatchHdr *hdr = reinterpret_cast<BatchHdr *>(ws + p.off_hdr);
    DevBlock *table = reinterpret_cast<DevBlock *>(ws + p.off_descs);
    for (auto &sl : g->slot) {
        void *h = nullptr;
        const size_t hb = align_up((size_t)max_blocks * sizeof(DevBlock), 256) + 256;
        if ((rc = check_hip(hipHostMalloc(&h, hb, hipHostMallocDefault), "hipHostMalloc")) ||
            (rc = check_hip(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming), "hipEventCreate"))) {
            if (h && !sl.h_descs) (void)hipHostFree(h);
            graph_free(g);
            return rc;
        }
        memset(h, 0, hb);
        sl.h_descs = static_cast<DevBlock *>(h);
        sl.h_n = reinterpret_cast<uint32_t *>(static_cast<uint8_t *>(h) + hb - 256);
        void *dh = nullptr;  // the same pinned buffer as the device addresses it
        if ((rc = check_hip(hipHostGetDevicePointer(&dh, h, 0), "hipHostGetDevicePointer"))) {
            graph_free(g);
            return rc;
        }
        const DevBlock *d_descs = static_cast<const DevBlock *>(dh);
        const uint32_t *d_n = reinterpret_cast<const uint32_t *>(static_cast<uint8_t *>(dh) + hb - 256);

        Batch bt;
        memset(&bt, 0, sizeof bt);
        bt.table = table;
        bt.hdr = hdr;
        bt.n_blocks = max_blocks;
        if ((rc = check_hip(hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal),
                            "hipStreamBeginCapture"))) {
            graph_free(g);
            return rc;
        }
        hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanWG), 0, g->capture, d_descs, d_n,
                           max_blocks, table, hdr, p.mode == kBinned ? ctrl : (Ctrl *)nullptr);
        rc = launch_status("k_plan launch");
        if (!rc) rc = enqueue_stages(p, bt, keys, hp, ws, g->capture, nullptr, true);
        hipGraph_t graph = nullptr;
        const int rc_end = check_hip(hipStreamEndCapture(g->capture, &graph), "hipStreamEndCapture");
        sl.graph = graph;
        if (rc || (rc = rc_end) ||
            (rc = check_hip(hipGraphInstantiate(&sl.exec, sl.graph, nullptr, nullptr, 0),
                            "hipGraphInstantiate"))) {
            graph_free(g);
            return rc;
        }
    }
    *out = g;
    return ACE_OK;
}

ACE_API int ace_graph_launch(ace_graph *g, const ace_block *blocks, uint32_t n_blocks, void *stream)
{
    clear_error();
    if (!g) return fail(ACE_ERR_INVALID_ARG, "graph is NULL");
    if (n_blocks > g->max_blocks)
        return fail(ACE_ERR_RANGE, "n_blocks %u exceeds the graph's %u", n_blocks, g->max_blocks);
    uint64_t total, tiles, waves;
    int rc = check_blocks(blocks, n_blocks, total, tiles, waves);
    if (rc) return rc;
    if (total > g->max_tx)
        return fail(ACE_ERR_RANGE, "%llu transactions exceed the graph's %llu",
                    (unsigned long long)total, (unsigned long long)g->max_tx);
    auto &sl = g->slot[g->next];
    if (sl.used && (rc = check_hip(hipEventSynchronize(sl.done), "hipEventSynchronize"))) return rc;
    for (uint32_t b = 0; b < n_blocks; ++b) sl.h_descs[b] = dev_block(blocks[b]);
    *sl.h_n = n_blocks;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((rc = check_hip(hipGraphLaunch(sl.exec, s), "hipGraphLaunch"))) return rc;
    if ((rc = check_hip(hipEventRecord(sl.done, s), "hipEventRecord"))) return rc;
    sl.used = true;
    g->next ^= 1;
    return ACE_OK;
}

ACE_API int ace_graph_destroy(ace_graph *g)
{
    clear_error();
    if (!g) return ACE_OK;
    for (auto &sl : g->slot)
        if (sl.used) (void)hipEventSynchronize(sl.done);
    graph_free(g);
    return ACE_OK;
}

}  // extern "C"

// Serving engine (ace_verify_stream and friends), same translation unit.
#include "ace_stream.hip"
