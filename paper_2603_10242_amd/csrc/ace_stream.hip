// ace_stream.hip -- serving engine behind ace_verify_stream (continuous batching).
//
// Clients submit requests (one block of transactions each) from any thread.
// Submission copies the request into pinned staging memory and queues it.  A
// server thread admits queued requests into a batch as soon as device arena
// space and an in-flight slot are free, uploads them on the slot's stream,
// runs one multi-block ace_verify_batch over the whole batch, and copies the
// bitmasks and counts back; requests that arrive while batches are on the
// GPU go into the next batch, whose copies and kernels overlap the running
// ones on another stream.  Completed requests are retired as their batch's
// event fires, in any order, and their arena and staging space is reused.
//
// The device side is behind a small backend interface so that the queue,
// admission and retirement logic also runs on the CPU in tests (host
// backend: the "device" is host memory and verification is a callback).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>

namespace {

// First-fit allocator over [0, capacity) with coalescing frees.
class RangeAlloc {
  public:
    explicit RangeAlloc(size_t cap = 0) { reset(cap); }
    void reset(size_t cap)
    {
        free_.clear();
        cap_ = cap;
        used_ = peak_ = 0;
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t n, size_t &off)
    {
        n = align_up(n ? n : 1, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                used_ += n;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = align_up(n ? n : 1, 256);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
};

// Byte layout of one request's inputs (identical in staging and in the arena).
struct ReqLayout {
    size_t off_off, off_id, off_tag, off_msg, in_bytes, mask_bytes, out_bytes;
    static ReqLayout of(uint64_t n, size_t msg_bytes)
    {
        ReqLayout l;
        size_t o = 0;
        l.off_off = o;   o = align_up(o + 8 * (n + 1), 256);
        l.off_id = o;    o = align_up(o + 4 * n, 256);
        l.off_tag = o;   o = align_up(o + 32 * n, 256);
        l.off_msg = o;   o = align_up(o + msg_bytes + 4, 256);
        l.in_bytes = o;
        // outputs live in the batch's result area: bitmask words, then the count
        l.mask_bytes = align_up(4 * ((n + 31) / 32), 8);
        l.out_bytes = l.mask_bytes + 8;
        return l;
    }
};

struct Request {
    uint64_t ticket;
    uint64_t n;
    ReqLayout lay;
    size_t stage_off;     // inputs in staging
    size_t out_rel = 0;   // outputs within the batch's result area
    uint32_t *h_mask;
    uint64_t *h_count;
    double t_submit, t_admit = 0, t_done = 0;
    int status = ACE_ERR_AGAIN;  // ACE_OK when done, < 0 error
};

class Backend {
  public:
    virtual ~Backend() {}
    virtual uint8_t *arena() = 0;
    virtual int begin_slot(int slot) = 0;
    virtual int h2d(int slot, void *dst, const void *src, size_t n) = 0;
    // `flags` is chosen once per batch and passed to both calls, so the
    // workspace sized for a batch is the one its verify call needs
    virtual int verify(int slot, const ace_block *blocks, uint32_t n_blocks, void *ws,
                       size_t ws_bytes, uint32_t flags) = 0;
    virtual size_t ws_size(const ace_block *blocks, uint32_t n_blocks, uint32_t flags) = 0;
    // largest workspace a batch holding only one request of n transactions
    // can need (the binned layout contains the in-order one)
    size_t ws_bound(uint64_t n)
    {
        ace_block b;
        memset(&b, 0, sizeof b);
        const uintptr_t fake = 0x1000;  // non-NULL, aligned: only sizes are computed
        b.d_msg = reinterpret_cast<const uint8_t *>(fake);
        b.d_off = reinterpret_cast<const uint64_t *>(fake);
        b.d_id = reinterpret_cast<const uint32_t *>(fake);
        b.d_tag = reinterpret_cast<const uint8_t *>(fake);
        b.d_bitmask_out = reinterpret_cast<uint32_t *>(fake);
        b.d_count_out = reinterpret_cast<uint64_t *>(fake);
        b.n_tx = n;
        return ws_size(&b, 1, ACE_BUCKETED);
    }
    virtual int d2h(int slot, void *dst, const void *src, size_t n) = 0;
    virtual int end_slot(int slot) = 0;
    virtual int query(int slot) = 0;  // 1 done, 0 running, < 0 failed
    virtual int wait(int slot) = 0;   // until the slot's last completed batch is done
    // until everything queued on the slot so far has finished, including work
    // of a batch whose launch sequence failed part way (its copies may still
    // be writing into the arena)
    virtual int drain(int slot) = 0;
};

// ---- HIP backend -------------------------------------------------------------------------
class HipBackend : public Backend {
  public:
    HipBackend(const ace_keyset &keys, uint8_t *arena, uint32_t slots, int device)
        : keys_(keys), arena_(arena), device_(device), streams_(slots), done_(slots)
    {
    }
    int init()
    {
        int rc = check_hip(hipSetDevice(device_), "hipSetDevice");
        for (size_t i = 0; !rc && i < streams_.size(); ++i) {
            rc = check_hip(hipStreamCreateWithFlags(&streams_[i], hipStreamNonBlocking), "hipStreamCreate");
            if (!rc) rc = check_hip(hipEventCreateWithFlags(&done_[i], hipEventDisableTiming), "hipEventCreate");
        }
        return rc;
    }
    ~HipBackend() override
    {
        for (auto s : streams_)
            if (s) (void)hipStreamDestroy(s);
        for (auto e : done_)
            if (e) (void)hipEventDestroy(e);
    }
    uint8_t *arena() override { return arena_; }
    int begin_slot(int) override { return check_hip(hipSetDevice(device_), "hipSetDevice"); }
    int h2d(int slot, void *dst, const void *src, size_t n) override
    {
        return check_hip(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, streams_[slot]), "hipMemcpyAsync H2D");
    }
    size_t ws_size(const ace_block *blocks, uint32_t n_blocks, uint32_t flags) override
    {
        return ace_verify_workspace_size(&keys_, blocks, n_blocks, flags);
    }
    int verify(int slot, const ace_block *blocks, uint32_t n_blocks, void *ws, size_t ws_bytes,
               uint32_t flags) override
    {
        return ace_verify_batch(&keys_, blocks, n_blocks, ws, ws_bytes, flags, streams_[slot]);
    }
    int d2h(int slot, void *dst, const void *src, size_t n) override
    {
        return check_hip(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, streams_[slot]), "hipMemcpyAsync D2H");
    }
    int end_slot(int slot) override { return check_hip(hipEventRecord(done_[slot], streams_[slot]), "hipEventRecord"); }
    int query(int slot) override
    {
        const hipError_t e = hipEventQuery(done_[slot]);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        return check_hip(e, "hipEventQuery");
    }
    int wait(int slot) override { return check_hip(hipEventSynchronize(done_[slot]), "hipEventSynchronize"); }
    int drain(int slot) override { return check_hip(hipStreamSynchronize(streams_[slot]), "hipStreamSynchronize"); }

  private:
    ace_keyset keys_;
    uint8_t *arena_;
    int device_;
    std::vector<hipStream_t> streams_;
    std::vector<hipEvent_t> done_;
};

// ---- host backend (tests) ----------------------------------------------------------------
class HostBackend : public Backend {
  public:
    HostBackend(ace_host_verify_fn fn, void *user, size_t arena_bytes, uint32_t fail_after,
                bool fail_at_launch)
        : fn_(fn), user_(user), mem_(arena_bytes), fail_after_(fail_after),
          fail_at_launch_(fail_at_launch), slot_status_(64, 1)
    {
    }
    uint8_t *arena() override { return mem_.data(); }
    int begin_slot(int slot) override
    {
        slot_status_[slot] = 1;
        return ACE_OK;
    }
    int h2d(int, void *dst, const void *src, size_t n) override
    {
        memcpy(dst, src, n);
        return ACE_OK;
    }
    size_t ws_size(const ace_block *, uint32_t, uint32_t) override { return 256; }
    int verify(int slot, const ace_block *blocks, uint32_t n_blocks, void *, size_t, uint32_t) override
    {
        ++launches_;
        if (fail_after_ && launches_ == fail_after_ && fail_at_launch_)
            return fail(ACE_ERR_DEVICE, "injected launch failure on launch %llu",
                        (unsigned long long)launches_);
        if (fail_after_ && launches_ == fail_after_) {
            slot_status_[slot] = fail(ACE_ERR_DEVICE, "injected device failure on launch %llu",
                                      (unsigned long long)launches_);
            return ACE_OK;  // the failure shows when the batch completes
        }
        for (uint32_t b = 0; b < n_blocks; ++b) {
            const ace_block &k = blocks[b];
            const int rc = fn_(user_, k.d_msg, k.d_off, k.d_id, k.d_tag, k.n_tx, k.d_bitmask_out,
                               k.d_count_out);
            if (rc) slot_status_[slot] = fail(ACE_ERR_DEVICE, "host verify callback returned %d", rc);
        }
        return ACE_OK;
    }
    int d2h(int, void *dst, const void *src, size_t n) override
    {
        memcpy(dst, src, n);
        return ACE_OK;
    }
    int end_slot(int) override { return ACE_OK; }
    int query(int slot) override { return slot_status_[slot]; }
    int wait(int slot) override { return slot_status_[slot] < 0 ? slot_status_[slot] : ACE_OK; }
    int drain(int) override
    {
        ++drains_;
        return ACE_OK;
    }
    uint64_t drains() const { return drains_; }

  private:
    ace_host_verify_fn fn_;
    void *user_;
    std::vector<uint8_t> mem_;
    uint32_t fail_after_;
    bool fail_at_launch_;
    uint64_t drains_ = 0;
    uint64_t launches_ = 0;
    std::vector<int> slot_status_;
};

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// A client call inside the engine: counted under the lock so that
// ace_stream_destroy frees nothing while one is still running.
struct InCall {
    std::condition_variable &cv;
    uint32_t &n;
    // constructed and destroyed with the engine's lock held
    InCall(std::condition_variable &cv_, uint32_t &n_) : cv(cv_), n(n_) { ++n; }
    ~InCall()
    {
        if (--n == 0) cv.notify_all();
    }
};

constexpr uint32_t kMaxBatchRequests = 4096;
// A batch is capped so that its upload stays around a millisecond: requests
// queued behind a running batch then join the next one instead of one huge
// batch whose copy alone takes tens of milliseconds.
constexpr uint64_t kMaxBatchTx = 1ull << 20;
constexpr size_t kMaxBatchBytes = 32ull << 20;
constexpr uint64_t kMaxRequestTx = 16ull << 20;  // one request (it may form a batch alone)
// per-slot pinned result buffer: every request's bitmask (8-byte padded) and count
constexpr size_t kResultBytes = (16ull << 20) / 8 + 16ull * kMaxBatchRequests + 4096;

}  // namespace

struct ace_stream {
    std::unique_ptr<Backend> be;
    bool plain;
    uint32_t slots;
    double t0;
    // staging (pinned host memory) and arena (device memory) allocators
    uint8_t *staging = nullptr;
    bool staging_pinned = false;
    RangeAlloc stage_alloc, arena_alloc;
    size_t arena_reserved = 0;  // leading bytes of the arena used for derived midstates
    // queue and bookkeeping
    std::mutex mu;
    std::condition_variable cv_submit;   // server wakes on new work / stop
    std::condition_variable cv_done;     // clients wake on completions / freed staging
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    uint32_t in_calls = 0;  // client calls inside the engine (destroy waits for 0)
    struct Slot {
        bool busy = false;
        bool launching = false;
        std::vector<Request *> members;
        size_t arena_off = 0, arena_bytes = 0;  // inputs, outputs and workspace of the batch
        uint8_t *result = nullptr;              // pinned host copy of the batch's outputs
    };
    std::vector<Slot> slot;
    ace_stream_stats stats{};
    std::thread server;
};

namespace {

// Server side: retire finished batches (lock held).
void release_batch(ace_stream *s, ace_stream::Slot &sl)
{
    for (Request *r : sl.members) s->stage_alloc.release(r->stage_off, r->lay.in_bytes);
    if (sl.arena_bytes) s->arena_alloc.release(sl.arena_off, sl.arena_bytes);
    sl.members.clear();
    sl.arena_bytes = 0;
    sl.busy = false;
}

void retire(ace_stream *s, bool block)
{
    for (uint32_t i = 0; i < s->slots; ++i) {
        auto &sl = s->slot[i];
        if (!sl.busy || sl.launching) continue;
        int q;
        if (block) {
            s->mu.unlock();
            q = s->be->wait((int)i);
            s->mu.lock();
            q = q == ACE_OK ? 1 : q;
        } else {
            q = s->be->query((int)i);
        }
        if (q == 0) continue;
        const double t = now_s();
        const uint8_t *res = sl.result;
        for (Request *r : sl.members) {
            if (q > 0) {
                if (r->n) memcpy(r->h_mask, res + r->out_rel, 4 * ((r->n + 31) / 32));
                memcpy(r->h_count, res + r->out_rel + r->lay.mask_bytes, 8);
                r->status = ACE_OK;
                s->stats.completed++;
            } else {
                r->status = q;
                s->stats.failed++;
            }
            r->t_done = t;
        }
        release_batch(s, sl);
        s->cv_done.notify_all();
    }
}

// Server side: form and launch one batch on a free slot (lock held).  The
// batch takes one arena range -- every request's inputs back to back, then
// all outputs, then the workspace -- so requests whose staging copies are
// adjacent go up in one copy, and all results come back in one copy.
bool admit(ace_stream *s)
{
    if (s->pending.empty()) return false;
    int free_slot = -1;
    for (uint32_t i = 0; i < s->slots; ++i)
        if (!s->slot[i].busy) { free_slot = (int)i; break; }
    if (free_slot < 0) return false;
    // in plain mode one request at a time, and nothing else in flight
    if (s->plain)
        for (uint32_t i = 0; i < s->slots; ++i)
            if (s->slot[i].busy) return false;

    // candidates in arrival order, within the count and transaction caps
    const size_t limit = s->plain ? 1 : kMaxBatchRequests;
    size_t m = 0;
    uint64_t tx = 0, out = 0, in = 0;
    while (m < s->pending.size() && m < limit) {
        const Request *r = s->pending[m];
        if (m && (tx + r->n > kMaxBatchTx || out + r->lay.out_bytes > kResultBytes ||
                  in + r->lay.in_bytes > kMaxBatchBytes))
            break;
        tx += r->n;
        out += r->lay.out_bytes;
        in += r->lay.in_bytes;
        ++m;
    }
    // largest prefix whose arena range (inputs, outputs, workspace) and result
    // area fit now.  The launch form (in-order or binned) is fixed here from
    // one reading of the tuning and passed to both the workspace size and the
    // verify call, so a tuning change in between cannot make them disagree.
    const ace_tuning tn = tuning();
    std::vector<ace_block> blocks;
    size_t arena_off = 0, arena_bytes = 0, in_total = 0, out_total = 0;
    uint32_t vflags = ACE_ORDERED;
    while (m > 0) {
        in_total = out_total = 0;
        uint64_t m_tx = 0;
        blocks.assign(m, ace_block{});
        for (size_t k = 0; k < m; ++k) {
            const Request *r = s->pending[k];
            in_total += r->lay.in_bytes;
            out_total += r->lay.out_bytes;
            m_tx += r->n;
            ace_block &bk = blocks[k];
            const uintptr_t fake = 0x1000;  // sizes only: real addresses are set below
            bk.d_msg = reinterpret_cast<const uint8_t *>(fake);
            bk.d_off = reinterpret_cast<const uint64_t *>(fake);
            bk.d_id = reinterpret_cast<const uint32_t *>(fake);
            bk.d_tag = reinterpret_cast<const uint8_t *>(fake);
            bk.d_bitmask_out = reinterpret_cast<uint32_t *>(fake);
            bk.d_count_out = reinterpret_cast<uint64_t *>(fake);
            bk.n_tx = r->n;
        }
        vflags = m_tx >= tn.binned_min_tx ? (ACE_BUCKETED | (tn.auto_persistent ? ACE_PERSISTENT : 0u))
                                          : ACE_ORDERED;
        const size_t ws = align_up(s->be->ws_size(blocks.data(), (uint32_t)m, vflags), 256);
        arena_bytes = in_total + align_up(out_total, 256) + ws;
        if (ws && s->arena_alloc.alloc(arena_bytes, arena_off)) break;
        m = m > 1 ? m - std::max<size_t>(1, m / 4) : 0;
    }
    if (m == 0) return false;

    auto &sl = s->slot[free_slot];
    std::vector<Request *> batch(s->pending.begin(), s->pending.begin() + m);
    s->pending.erase(s->pending.begin(), s->pending.begin() + m);
    // Submitters finish their staging copies in any order, so the queue's
    // order is not the staging order: sorted by staging offset, requests
    // staged back to back go up in one copy (at saturation, 13.6 instead of
    // 27.6 copies per batch of about 33 requests).
    std::sort(batch.begin(), batch.end(),
              [](const Request *a, const Request *b) { return a->stage_off < b->stage_off; });
    uint8_t *arena = s->be->arena() + s->arena_reserved;
    uint8_t *base = arena + arena_off;
    uint8_t *out_base = base + in_total;
    size_t in_rel = 0, out_rel = 0;
    std::vector<size_t> in_pos(m);
    for (size_t k = 0; k < m; ++k) {
        Request *r = batch[k];
        in_pos[k] = in_rel;
        r->out_rel = out_rel;
        uint8_t *d = base + in_rel;
        ace_block &bk = blocks[k];
        bk.d_msg = d + r->lay.off_msg;
        bk.d_off = reinterpret_cast<const uint64_t *>(d + r->lay.off_off);
        bk.d_id = reinterpret_cast<const uint32_t *>(d + r->lay.off_id);
        bk.d_tag = d + r->lay.off_tag;
        bk.n_tx = r->n;
        bk.d_bitmask_out = reinterpret_cast<uint32_t *>(out_base + out_rel);
        bk.d_count_out = reinterpret_cast<uint64_t *>(out_base + out_rel + r->lay.mask_bytes);
        in_rel += r->lay.in_bytes;
        out_rel += r->lay.out_bytes;
    }
    uint8_t *ws_ptr = out_base + align_up(out_total, 256);
    const size_t ws_bytes = arena_bytes - in_total - align_up(out_total, 256);

    const double t = now_s();
    for (Request *r : batch) r->t_admit = t;
    sl.busy = true;
    sl.launching = true;  // retire() leaves the slot alone until everything is queued
    sl.members = batch;
    sl.arena_off = arena_off;
    sl.arena_bytes = arena_bytes;
    uint8_t *staging = s->staging;

    // device calls without the lock, so submitters are never held up by them
    s->mu.unlock();
    int rc = s->be->begin_slot(free_slot);
    for (size_t k = 0; !rc && k < m;) {
        // one copy per run of requests whose staging inputs are adjacent
        size_t j = k + 1, bytes = batch[k]->lay.in_bytes;
        while (j < m && batch[j]->stage_off == batch[j - 1]->stage_off + batch[j - 1]->lay.in_bytes) {
            bytes += batch[j]->lay.in_bytes;
            ++j;
        }
        rc = s->be->h2d(free_slot, base + in_pos[k], staging + batch[k]->stage_off, bytes);
        k = j;
    }
    if (!rc) rc = s->be->verify(free_slot, blocks.data(), (uint32_t)m, ws_ptr, ws_bytes, vflags);
    if (!rc) rc = s->be->d2h(free_slot, sl.result, out_base, out_total);
    if (!rc) rc = s->be->end_slot(free_slot);
    // A failure part way leaves this batch's copies (and maybe kernels) queued
    // on the slot's stream: wait for all of it before its arena and staging
    // ranges go back to the allocators, or another batch could be given memory
    // a copy is still writing into.
    if (rc) (void)s->be->drain(free_slot);
    s->mu.lock();
    sl.launching = false;
    if (rc) {
        // the batch never reached the device queue whole: fail its requests now
        const double te = now_s();
        for (Request *r : batch) {
            r->status = rc;
            r->t_done = te;
            s->stats.failed++;
        }
        release_batch(s, sl);
        s->cv_done.notify_all();
        return true;
    }
    s->stats.batches++;
    s->stats.max_batch_requests = std::max<uint64_t>(s->stats.max_batch_requests, m);
    return true;
}

void serve(ace_stream *s)
{
    std::unique_lock<std::mutex> lock(s->mu);
    for (;;) {
        retire(s, false);
        bool launched = false;
        while (admit(s)) launched = true;
        bool busy = false;
        for (auto &sl : s->slot) busy |= sl.busy;
        if (s->stop && s->pending.empty() && !busy) break;
        if (launched) continue;
        if (s->plain && busy) {
            retire(s, true);  // the plain form waits for each request
            continue;
        }
        if (busy) {
            // batches in flight: poll for completions, wake early on new work
            s->cv_submit.wait_for(lock, std::chrono::microseconds(20));
        } else {
            s->cv_submit.wait(lock, [s] { return s->stop || !s->pending.empty(); });
        }
    }
}

}  // namespace

extern "C" {

static int stream_start(ace_stream *s, size_t arena_bytes, size_t staging_bytes, uint32_t max_inflight,
                        uint32_t flags, bool pinned)
{
    s->plain = (flags & ACE_STREAM_PLAIN) != 0;
    s->slots = s->plain ? 1 : max_inflight;
    s->slot.resize(s->slots);
    s->t0 = now_s();
    s->arena_alloc.reset(arena_bytes - s->arena_reserved);
    if (pinned) {
        void *h = nullptr;
        int rc = check_hip(hipHostMalloc(&h, staging_bytes, hipHostMallocDefault), "hipHostMalloc staging");
        if (rc) return rc;
        s->staging = static_cast<uint8_t *>(h);
        s->staging_pinned = true;
    } else {
        s->staging = static_cast<uint8_t *>(malloc(staging_bytes));
        if (!s->staging) return fail(ACE_ERR_NO_MEMORY, "staging allocation failed");
    }
    s->stage_alloc.reset(staging_bytes);
    for (auto &sl : s->slot) {
        if (pinned) {
            void *h = nullptr;
            int rc = check_hip(hipHostMalloc(&h, kResultBytes, hipHostMallocDefault), "hipHostMalloc results");
            if (rc) return rc;
            sl.result = static_cast<uint8_t *>(h);
        } else {
            sl.result = static_cast<uint8_t *>(malloc(kResultBytes));
            if (!sl.result) return fail(ACE_ERR_NO_MEMORY, "result buffer allocation failed");
        }
    }
    s->server = std::thread(serve, s);
    return ACE_OK;
}

static void stream_free(ace_stream *s)
{
    if (!s) return;
    for (auto &sl : s->slot) {
        if (!sl.result) continue;
        if (s->staging_pinned) (void)hipHostFree(sl.result);
        else free(sl.result);
    }
    if (s->staging) {
        if (s->staging_pinned) (void)hipHostFree(s->staging);
        else free(s->staging);
    }
    delete s;
}

ACE_API int ace_stream_create(const ace_keyset *keys, void *d_arena, size_t arena_bytes,
                              size_t staging_bytes, uint32_t max_inflight, uint32_t flags,
                              ace_stream **out)
{
    clear_error();
    if (!out) return fail(ACE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    Plan p{};
    int rc = check_keyset(keys, 0, p);
    if (rc) return rc;
    if (flags & ~(uint32_t)ACE_STREAM_PLAIN) return fail(ACE_ERR_INVALID_ARG, "unknown flags");
    if (!d_arena || !aligned(d_arena, 256)) return fail(ACE_ERR_INVALID_ARG, "d_arena NULL or not 256-byte aligned");
    if (max_inflight < 1 || max_inflight > 64) return fail(ACE_ERR_INVALID_ARG, "max_inflight must be 1..64");
    if (staging_bytes < 4096) return fail(ACE_ERR_INVALID_ARG, "staging_bytes < 4096");
    ace_keyset ks = *keys;
    size_t reserved = 0;
    if (keys->kind == ACE_KEYS_REV) {
        // keep the registry's midstates resident: derive them once into the arena
        reserved = align_up(64ull * keys->n_id, 256);
        if (arena_bytes < reserved + 4096) return fail(ACE_ERR_NO_MEMORY, "arena too small for the midstate cache");
        uint32_t *mid = static_cast<uint32_t *>(d_arena);
        if (keys->n_id &&
            (rc = ace_derive_keys(keys->d_rev, keys->n_id, keys->h_salt, keys->salt_len, keys->h_info,
                                  keys->info_len, nullptr, mid, nullptr)))
            return rc;
        if ((rc = check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize"))) return rc;
        ks.kind = ACE_KEYS_MIDSTATE;
        ks.d_mid = mid;
        ks.d_rev = nullptr;
    }
    if (arena_bytes < reserved + 4096) return fail(ACE_ERR_NO_MEMORY, "arena too small");
    int dev = 0;
    if ((rc = check_hip(hipGetDevice(&dev), "hipGetDevice"))) return rc;
    ace_stream *s = new ace_stream;
    s->arena_reserved = reserved;
    auto be = std::make_unique<HipBackend>(ks, static_cast<uint8_t *>(d_arena),
                                           (flags & ACE_STREAM_PLAIN) ? 1 : max_inflight, dev);
    if ((rc = be->init())) {
        stream_free(s);
        return rc;
    }
    s->be = std::move(be);
    if ((rc = stream_start(s, arena_bytes, staging_bytes, max_inflight, flags, true))) {
        stream_free(s);
        return rc;
    }
    *out = s;
    return ACE_OK;
}

ACE_API int ace_stream_create_host(ace_host_verify_fn fn, void *user, size_t arena_bytes,
                                   size_t staging_bytes, uint32_t max_inflight, uint32_t flags,
                                   uint32_t fail_after, ace_stream **out)
{
    clear_error();
    if (!out || !fn) return fail(ACE_ERR_INVALID_ARG, "out or fn is NULL");
    *out = nullptr;
    if (flags & ~(uint32_t)(ACE_STREAM_PLAIN | ACE_STREAM_HOST_FAIL_LAUNCH))
        return fail(ACE_ERR_INVALID_ARG, "unknown flags");
    if (max_inflight < 1 || max_inflight > 64) return fail(ACE_ERR_INVALID_ARG, "max_inflight must be 1..64");
    if (arena_bytes < 4096 || staging_bytes < 4096) return fail(ACE_ERR_INVALID_ARG, "arena or staging < 4096 bytes");
    ace_stream *s = new ace_stream;
    s->be = std::make_unique<HostBackend>(fn, user, arena_bytes, fail_after,
                                          (flags & ACE_STREAM_HOST_FAIL_LAUNCH) != 0);
    int rc = stream_start(s, arena_bytes, staging_bytes, max_inflight,
                          flags & ~(uint32_t)ACE_STREAM_HOST_FAIL_LAUNCH, false);
    if (rc) {
        stream_free(s);
        return rc;
    }
    *out = s;
    return ACE_OK;
}

ACE_API int ace_verify_stream(ace_stream *s, const uint8_t *h_msg, const uint64_t *h_off,
                              const uint32_t *h_id, const uint8_t *h_tag, uint64_t n_tx,
                              uint32_t *h_bitmask_out, uint64_t *h_count_out, uint32_t flags,
                              uint64_t *ticket_out)
{
    clear_error();
    if (!s || !ticket_out || !h_count_out) return fail(ACE_ERR_INVALID_ARG, "NULL stream, ticket or count");
    if (flags & ~(uint32_t)ACE_NONBLOCK) return fail(ACE_ERR_INVALID_ARG, "unknown flags");
    if (n_tx && (!h_off || !h_id || !h_tag || !h_bitmask_out))
        return fail(ACE_ERR_INVALID_ARG, "NULL array with n_tx > 0");
    if (n_tx > (1ull << 31)) return fail(ACE_ERR_RANGE, "n_tx too large for one request");
    // span of the message bytes this request refers to
    uint64_t lo = 0, hi = 0;
    if (n_tx) {
        lo = hi = h_off[0];
        for (uint64_t i = 1; i <= n_tx; ++i) {
            lo = std::min(lo, h_off[i]);
            hi = std::max(hi, h_off[i]);
        }
        if (hi > lo && !h_msg) return fail(ACE_ERR_INVALID_ARG, "h_msg is NULL");
    }
    const size_t msg_bytes = (size_t)(hi - lo);
    const ReqLayout lay = ReqLayout::of(n_tx, msg_bytes);
    const size_t stage_need = lay.in_bytes;
    const size_t dev_need = lay.in_bytes + align_up(lay.out_bytes, 256) +
                            align_up(s->be->ws_bound(n_tx), 256);
    if (stage_need > s->stage_alloc.capacity() || dev_need > s->arena_alloc.capacity() ||
        n_tx > kMaxRequestTx)
        return fail(ACE_ERR_TOO_LARGE, "request needs %zu staging and %zu arena bytes; staging %zu, arena %zu",
                    stage_need, dev_need, s->stage_alloc.capacity(), s->arena_alloc.capacity());

    std::unique_lock<std::mutex> lock(s->mu);
    if (s->stop) return fail(ACE_ERR_INVALID_ARG, "stream is being destroyed");
    InCall guard(s->cv_done, s->in_calls);  // released with the lock held (declared after it)
    size_t stage_off;
    while (!s->stage_alloc.alloc(lay.in_bytes, stage_off)) {
        if (flags & ACE_NONBLOCK) return fail(ACE_ERR_AGAIN, "staging full");
        s->cv_done.wait(lock);
        if (s->stop) return fail(ACE_ERR_INVALID_ARG, "stream is being destroyed");
    }
    auto r = std::make_unique<Request>();
    r->ticket = s->next_ticket++;
    r->n = n_tx;
    r->lay = lay;
    r->stage_off = stage_off;
    r->h_mask = h_bitmask_out;
    r->h_count = h_count_out;
    r->t_submit = now_s();
    uint8_t *st = s->staging + stage_off;
    lock.unlock();
    // copy the request into its staging slot (offsets rebased to the copied span)
    uint64_t *off = reinterpret_cast<uint64_t *>(st + lay.off_off);
    if (n_tx) {
        for (uint64_t i = 0; i <= n_tx; ++i) off[i] = h_off[i] - lo;
        memcpy(st + lay.off_id, h_id, 4 * n_tx);
        memcpy(st + lay.off_tag, h_tag, 32 * n_tx);
        if (msg_bytes) memcpy(st + lay.off_msg, h_msg + lo, msg_bytes);
    } else {
        off[0] = 0;
    }
    lock.lock();
    if (s->stop) {
        // destroy began during the copy: the server may already have drained
        // the queue and left, so the request is not accepted
        s->stage_alloc.release(stage_off, lay.in_bytes);
        return fail(ACE_ERR_INVALID_ARG, "stream is being destroyed");
    }
    *ticket_out = r->ticket;
    s->pending.push_back(r.get());
    s->reqs.emplace(r->ticket, std::move(r));
    s->stats.submitted++;
    s->cv_submit.notify_one();
    return ACE_OK;
}

ACE_API int ace_stream_poll(ace_stream *s, uint64_t ticket, int wait)
{
    clear_error();
    if (!s) return fail(ACE_ERR_INVALID_ARG, "stream is NULL");
    std::unique_lock<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(ACE_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second.get();
    InCall guard(s->cv_done, s->in_calls);
    if (wait)
        s->cv_done.wait(lock, [r] { return r->status != ACE_ERR_AGAIN; });
    if (r->status == ACE_ERR_AGAIN) return ACE_ERR_AGAIN;
    if (r->status != ACE_OK) return fail(r->status, "request %llu failed", (unsigned long long)ticket);
    return ACE_OK;
}

ACE_API int ace_stream_ticket_times(ace_stream *s, uint64_t ticket, double *submit_s, double *admit_s,
                                    double *done_s)
{
    clear_error();
    if (!s) return fail(ACE_ERR_INVALID_ARG, "stream is NULL");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(ACE_ERR_INVALID_ARG, "unknown ticket");
    const Request *r = it->second.get();
    if (submit_s) *submit_s = r->t_submit;
    if (admit_s) *admit_s = r->t_admit;
    if (done_s) *done_s = r->t_done;
    return r->status == ACE_ERR_AGAIN ? ACE_ERR_AGAIN : ACE_OK;
}

ACE_API int ace_stream_release(ace_stream *s, uint64_t ticket)
{
    clear_error();
    if (!s) return fail(ACE_ERR_INVALID_ARG, "stream is NULL");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(ACE_ERR_INVALID_ARG, "unknown ticket");
    if (it->second->status == ACE_ERR_AGAIN) return fail(ACE_ERR_AGAIN, "request still pending");
    s->reqs.erase(it);
    return ACE_OK;
}

ACE_API int ace_stream_get_stats(ace_stream *s, ace_stream_stats *out)
{
    clear_error();
    if (!s || !out) return fail(ACE_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    *out = s->stats;
    out->arena_peak_bytes = s->arena_alloc.peak();
    out->arena_capacity_bytes = s->arena_alloc.capacity();
    out->pending = s->pending.size();
    return ACE_OK;
}

ACE_API int ace_stream_destroy(ace_stream *s)
{
    clear_error();
    if (!s) return ACE_OK;
    {
        std::unique_lock<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv_submit.notify_all();
        // submitters waiting for staging give up; pollers wait for their
        // requests, which the server still finishes
        s->cv_done.notify_all();
    }
    if (s->server.joinable()) s->server.join();
    {
        // no client call may still be inside the engine when it is freed
        std::unique_lock<std::mutex> lock(s->mu);
        s->cv_done.wait(lock, [s] { return s->in_calls == 0; });
    }
    stream_free(s);
    return ACE_OK;
}

}  // extern "C"
