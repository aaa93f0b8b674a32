// Race check of the serving engine (ace_stream_*), host side only: the
// engine runs with its host backend (a callback verifies each batch) while
// eight threads submit blocking and non-blocking requests, poll, read ticket
// times and statistics, and release tickets.  Built with ThreadSanitizer on
// the host code by tests/test_stream_tsan.py; exit status 0 when every count
// is right.
#include <stdio.h>
#include <stdint.h>
#include <string.h>
#include <thread>
#include <vector>
#include <atomic>
#include "ace.h"

static int verify_cb(void *user, const uint8_t *msg, const uint64_t *off, const uint32_t *id,
                     const uint8_t *tag, uint64_t n, uint32_t *mask, uint64_t *count)
{
    (void)user; (void)msg; (void)tag;
    uint64_t c = 0;
    memset(mask, 0, ((n + 31) / 32) * 4);
    for (uint64_t i = 0; i < n; ++i) {
        int v = (id[i] & 1) == 0 && off[i] <= off[i + 1];
        if (v) { mask[i / 32] |= 1u << (i % 32); ++c; }
    }
    *count = c;
    return 0;
}

int main()
{
    ace_stream *s = nullptr;
    int rc = ace_stream_create_host(verify_cb, nullptr, 64 << 20, 16 << 20, 4, 0, 0, &s);
    if (rc) { printf("create %d %s\n", rc, ace_last_error()); return 1; }
    std::atomic<int> bad{0};
    std::vector<std::thread> th;
    for (int t = 0; t < 8; ++t) {
        th.emplace_back([&, t]() {
            std::vector<uint8_t> msg(4096 * 64);
            std::vector<uint64_t> off(4097);
            std::vector<uint32_t> id(4096);
            std::vector<uint8_t> tag(4096 * 32);
            for (int i = 0; i <= 4096; ++i) off[i] = (uint64_t)i * 64;
            for (int r = 0; r < 300; ++r) {
                uint64_t n = 1 + (uint64_t)((r * 2654435761u + t * 97) % 4096);
                for (uint64_t i = 0; i < n; ++i) id[i] = (uint32_t)(i + r + t);
                std::vector<uint32_t> mask((n + 31) / 32);
                uint64_t count = 0, ticket = 0;
                uint32_t flags = (r % 3 == 0) ? ACE_NONBLOCK : 0;
                int rc = ace_verify_stream(s, msg.data(), off.data(), id.data(), tag.data(), n,
                                       mask.data(), &count, flags, &ticket);
                if (rc == ACE_ERR_AGAIN) { --r; std::this_thread::yield(); continue; }
                if (rc) { printf("submit %d %s\n", rc, ace_last_error()); bad++; return; }
                rc = ace_stream_poll(s, ticket, 1);
                if (rc) { printf("poll %d\n", rc); bad++; return; }
                uint64_t want = 0;
                for (uint64_t i = 0; i < n; ++i) want += ((id[i] & 1) == 0);
                if (count != want) { printf("count %lu != %lu\n", (unsigned long)count, (unsigned long)want); bad++; }
                double a, b, c;
                ace_stream_ticket_times(s, ticket, &a, &b, &c);
                ace_stream_release(s, ticket);
                ace_stream_stats st;
                ace_stream_get_stats(s, &st);
            }
        });
    }
    for (auto &x : th) x.join();
    ace_stream_stats st;
    ace_stream_get_stats(s, &st);
    printf("submitted %lu completed %lu batches %lu max_batch %lu bad %d\n", (unsigned long)st.submitted,
           (unsigned long)st.completed, (unsigned long)st.batches, (unsigned long)st.max_batch_requests, bad.load());
    ace_stream_destroy(s);
    return bad.load() != 0;
}
