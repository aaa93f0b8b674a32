/*
 * serving_client.c -- open-loop load generator of the serving benchmark.
 *
 * Request k arrives at arrivals[k] (CLOCK_MONOTONIC seconds) and is submitted
 * then, by one of n_threads submitter threads (request k goes to thread
 * k % n_threads), through the library's ace_verify_stream, whose address the
 * caller passes in (this file links to nothing but libc and pthreads).
 * Request k covers pool transactions starts[k] .. starts[k] + sizes[k]; its
 * bitmask goes to mask_out + mask_words[k], its count to count_out[k], its
 * ticket to tickets_out[k], and the time the submit call began to
 * submit_s_out[k].  Written natively so that the latency measured is the
 * engine's, not the pauses of an interpreter's threads.
 */
#define _GNU_SOURCE
#include <errno.h>
#include <pthread.h>
#include <stdint.h>
#include <string.h>
#include <time.h>

typedef int (*verify_stream_fn)(void *s, const uint8_t *h_msg, const uint64_t *h_off,
                                const uint32_t *h_id, const uint8_t *h_tag, uint64_t n_tx,
                                uint32_t *h_bitmask_out, uint64_t *h_count_out, uint32_t flags,
                                uint64_t *ticket_out);

typedef struct {
    verify_stream_fn fn;
    void *stream;
    const uint8_t *msg;
    const uint64_t *off;
    const uint32_t *ids;
    const uint8_t *tags;
    const uint64_t *starts, *sizes, *mask_words;
    const double *arrivals;
    uint64_t n_req;
    int n_threads, t;
    uint32_t *mask_out;
    uint64_t *count_out, *tickets_out;
    double *submit_s_out;
    int status;
} job_t;

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static void sleep_until(double t)
{
    struct timespec ts;
    ts.tv_sec = (time_t)t;
    ts.tv_nsec = (long)((t - (double)ts.tv_sec) * 1e9);
    if (ts.tv_nsec >= 1000000000L) { ts.tv_sec += 1; ts.tv_nsec -= 1000000000L; }
    while (clock_nanosleep(CLOCK_MONOTONIC, TIMER_ABSTIME, &ts, NULL) == EINTR) {
    }
}

static void *run(void *arg)
{
    job_t *j = (job_t *)arg;
    for (uint64_t k = (uint64_t)j->t; k < j->n_req; k += (uint64_t)j->n_threads) {
        if (now_s() < j->arrivals[k]) sleep_until(j->arrivals[k]);
        const uint64_t lo = j->starts[k];
        j->submit_s_out[k] = now_s();
        const int rc = j->fn(j->stream, j->msg, j->off + lo, j->ids + lo, j->tags + 32 * lo,
                             j->sizes[k], j->mask_out + j->mask_words[k], j->count_out + k, 0,
                             j->tickets_out + k);
        if (rc) {
            j->status = rc;
            return NULL;
        }
    }
    return NULL;
}

/* Returns 0, or the first nonzero status of a submit call. */
int client_drive(void *fn, void *stream, const uint8_t *msg, const uint64_t *off,
                 const uint32_t *ids, const uint8_t *tags, const uint64_t *starts,
                 const uint64_t *sizes, const uint64_t *mask_words, const double *arrivals,
                 uint64_t n_req, int n_threads, uint32_t *mask_out, uint64_t *count_out,
                 uint64_t *tickets_out, double *submit_s_out)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 64) n_threads = 64;
    job_t jobs[64];
    pthread_t th[64];
    int started[64];
    for (int t = 0; t < n_threads; ++t) {
        job_t *j = &jobs[t];
        memset(j, 0, sizeof *j);
        j->fn = (verify_stream_fn)fn;
        j->stream = stream;
        j->msg = msg; j->off = off; j->ids = ids; j->tags = tags;
        j->starts = starts; j->sizes = sizes; j->mask_words = mask_words; j->arrivals = arrivals;
        j->n_req = n_req; j->n_threads = n_threads; j->t = t;
        j->mask_out = mask_out; j->count_out = count_out; j->tickets_out = tickets_out;
        j->submit_s_out = submit_s_out;
        started[t] = pthread_create(&th[t], NULL, run, j) == 0;
    }
    int status = 0;
    for (int t = 0; t < n_threads; ++t) {
        if (started[t]) pthread_join(th[t], NULL);
        else run(&jobs[t]);
        if (jobs[t].status && !status) status = jobs[t].status;
    }
    return status;
}
