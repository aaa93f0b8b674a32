/*
 * ace.h -- C ABI of libace.so: batched verification of HMAC-SHA256
 * attestations under HKDF-SHA256 derived keys on one MI355X (gfx950).
 *
 * The operation is the attestation check of the ACE Runtime paper: Alg. 1,
 * Phase 1a (AttestCheck) recomputes, for every transaction, the credential
 * HMAC-SHA256(k, m) under the key of the transaction's identity and rejects
 * the transaction when it differs from the attached credential; the key is
 * k = HKDF-SHA256(REV, info, salt) (Def. 2.1, Def. 3.1 equation attestkey)
 * and the credential is equation credential of Def. 3.1.  The message m is
 * taken verbatim from the caller (the paper's m = obj_hash || domain is the
 * 40-byte case); an identity index outside the registry is rejected (the
 * identity existence check of Alg. 2).
 *
 * Around it: the paper's own attestation form with the validator's payload
 * binding (ace_verify_attestations), the keys of several HKDF streams
 * (ace_derive_keys_multi), the block header's Merkle roots
 * (ace_merkle_roots), segments of the hash-chain clock (ace_poh_verify), a
 * captured-graph form of the batch call and a continuous-batching serving
 * engine.
 *
 * Conventions shared by every entry point:
 *   - d_* arguments are HIP device pointers owned by the caller; h_* are host
 *     pointers read before the call returns.  The library never frees or
 *     retains caller memory and allocates no device memory: scratch space is
 *     the caller's workspace (ace_verify_batch_noalloc: a static array the
 *     library holds on each GPU).
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     asynchronously on it; outputs are valid once the stream has reached
 *     the end of the call's work.
 *   - A return value < 0 is an ace_status error.  Every argument error is
 *     detected before anything is enqueued; ace_last_error() then describes
 *     it (thread-local, valid until the next call on the same thread).
 *   - An invalid transaction is data, not an error: a wrong credential, a
 *     tampered message, a wrong key, an identity index >= n_id and an offset
 *     pair with off[i+1] < off[i] all give bit 0.
 *   - Bitmasks: bit i % 32 of 32-bit word i / 32 is transaction i (LSB
 *     first); unused bits of the last word are 0.
 *   - Midstates: for each identity, 16 native 32-bit words: words 0-7 are
 *     the SHA-256 state after the block K0 ^ ipad, words 8-15 after K0 ^ opad
 *     (RFC 2104 with B = 64; K0 = key || 32 zero bytes).
 */
#ifndef ACE_H
#define ACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ACE_API __attribute__((visibility("default")))

typedef enum {
    ACE_OK = 0,
    ACE_ERR_INVALID_ARG = -1, /* NULL where not allowed, bad length or flag */
    ACE_ERR_RANGE = -2,       /* a count exceeds what the layout can index   */
    ACE_ERR_NO_MEMORY = -3,   /* workspace or arena smaller than required    */
    ACE_ERR_DEVICE = -4,      /* a HIP call failed                           */
    ACE_ERR_AGAIN = -5,       /* non-blocking call: not done / no room yet   */
    ACE_ERR_TOO_LARGE = -6    /* a request can never fit the arena           */
} ace_status;

/* Limits. */
#define ACE_MAX_SALT_BYTES 1024u  /* HKDF salt; longer salts: ACE_ERR_INVALID_ARG */
#define ACE_MAX_INFO_BYTES 255u   /* HKDF info                                  */
#define ACE_MAX_TX 4294963200ull  /* 2^32 - 4096: total transactions per call   */

/* Flags of ace_verify_batch. */
#define ACE_ORDERED 0x1u    /* one transaction per lane in input order (no length bucketing) */
#define ACE_BUCKETED 0x2u   /* group transactions by block count before hashing */
#define ACE_PERSISTENT 0x4u /* fixed grid of workgroups pulling wave tiles from a counter */
#define ACE_PER_TX_KEYS 0x8u /* keyset of kind ACE_KEYS_REV: derive each transaction's key
                                inside the verify kernel instead of once per identity */
/* Neither ORDERED nor BUCKETED: the library picks (bucketed for large batches). */

/* Keyset kinds. */
#define ACE_KEYS_MIDSTATE 0 /* d_mid[n_id][16]: cached HMAC midstates (from ace_derive_keys) */
#define ACE_KEYS_REV 1      /* d_rev[n_id][32]: root entropy; keys derived in the call      */

/* Last error detail of the calling thread ("" when none). */
ACE_API const char *ace_last_error(void);
/* Library version string. */
ACE_API const char *ace_version(void);

/*
 * ace_derive_keys -- Def. 2.1 / equation attestkey, for n_id identities.
 *   k_j = HKDF-SHA256(salt, IKM = REV_j, info, L = 32)        (RFC 5869)
 * and, when d_mid_out is given, the HMAC midstates of k_j.
 *   d_rev      [n_id][32] bytes, root entropy of each identity.
 *   h_salt     salt_len bytes shared by all identities (the context; the
 *              paper's domain).  salt_len 0 means HashLen zero bytes.
 *              salt_len <= ACE_MAX_SALT_BYTES.
 *   h_info     info_len bytes, info_len <= ACE_MAX_INFO_BYTES.
 *   d_key_out  [n_id][32] bytes or NULL.
 *   d_mid_out  [n_id][16] uint32 or NULL (not both NULL).
 * n_id == 0 is a no-op.  Needs no workspace.
 */
ACE_API int ace_derive_keys(const uint8_t *d_rev, uint32_t n_id, const uint8_t *h_salt,
                            size_t salt_len, const uint8_t *h_info, size_t info_len,
                            uint8_t *d_key_out, uint32_t *d_mid_out, void *stream);

/*
 * ace_derive_keys_multi -- the keys of several HKDF streams for one registry:
 * the purpose streams of Def. 2.1 (one key per purpose string from the same
 * root entropy), the validator keys of the consensus and vote equations
 * (valkey, votekey), or the attestation keys of several slots (eq. attestkey,
 * one domain each).  For stream s and identity j
 *   k[s][j] = HKDF-SHA256(salt_s, IKM = REV_j, info_s, L = 32)
 * and, when d_mid_out is given, its HMAC midstates.
 *   h_streams  n_streams (salt, info) pairs in host memory, read before the
 *              call returns; salt_len <= ACE_MULTI_MAX_SALT_BYTES and
 *              info_len <= ACE_MULTI_MAX_INFO_BYTES (longer ones: one
 *              ace_derive_keys call per stream); salt_len 0 means HashLen zero
 *              bytes.
 *   d_key_out  [n_streams][n_id][32] bytes or NULL.
 *   d_mid_out  [n_streams][n_id][16] uint32 or NULL (not both NULL).
 * n_id == 0 or n_streams == 0 is a no-op.  Needs no workspace.
 */
#define ACE_MULTI_MAX_SALT_BYTES 64u
#define ACE_MULTI_MAX_INFO_BYTES 64u
typedef struct {
    const uint8_t *h_salt;
    size_t salt_len;
    const uint8_t *h_info;
    size_t info_len;
} ace_hkdf_stream;

ACE_API int ace_derive_keys_multi(const uint8_t *d_rev, uint32_t n_id,
                                  const ace_hkdf_stream *h_streams, uint32_t n_streams,
                                  uint8_t *d_key_out, uint32_t *d_mid_out, void *stream);

/* One block of transactions (Alg. 1 SelectTransactions output). */
typedef struct {
    const uint8_t *d_msg;    /* messages back to back; may be NULL only if n_tx == 0      */
    const uint64_t *d_off;   /* [n_tx + 1] byte offsets into d_msg; message i is
                                d_msg[off[i] .. off[i+1]).  Offsets must lie within the
                                message buffer (reading past it is undefined).           */
    const uint32_t *d_id;    /* [n_tx] identity index into the keyset                     */
    const uint8_t *d_tag;    /* [n_tx][32] credentials                                    */
    uint64_t n_tx;
    uint32_t *d_bitmask_out; /* [ceil(n_tx / 32)] words, fully written                    */
    uint64_t *d_count_out;   /* one uint64: number of valid transactions                  */
} ace_block;

/* The identity registry the transactions refer to. */
typedef struct {
    int kind;                /* ACE_KEYS_MIDSTATE or ACE_KEYS_REV                           */
    const uint32_t *d_mid;   /* kind MIDSTATE: [n_id][16]                                  */
    const uint8_t *d_rev;    /* kind REV: [n_id][32]                                        */
    uint32_t n_id;
    const uint8_t *h_salt;   /* kind REV: HKDF salt and info as in ace_derive_keys          */
    size_t salt_len;
    const uint8_t *h_info;
    size_t info_len;
} ace_keyset;

/* Workspace bytes ace_verify_batch (or ace_verify_attestations) needs for these
 * arguments (0 on bad arguments). */
ACE_API size_t ace_verify_workspace_size(const ace_keyset *keys, const ace_block *blocks,
                                         uint32_t n_blocks, uint32_t flags);

/*
 * ace_verify_batch -- Alg. 1 Phase 1a over n_blocks blocks in one pass.
 *   valid_i = (id_i < n_id) and (off_i <= off_{i+1}) and
 *             HMAC-SHA256(k_{id_i}, msg_i) == tag_i (full 32-byte compare,
 *             no early exit)
 * Writes every block's bitmask and count.  All blocks are scheduled
 * together, so many small blocks fill the GPU as one large one would.
 *   d_workspace  device memory of at least ace_verify_workspace_size() bytes,
 *                256-byte aligned; its content on entry is ignored.  It must
 *                not be used by another call until this call's work is done.
 *   flags        ACE_ORDERED / ACE_BUCKETED / ACE_PERSISTENT / ACE_PER_TX_KEYS.
 * Sum of n_tx over blocks must be <= ACE_MAX_TX (else ACE_ERR_RANGE).
 */
ACE_API int ace_verify_batch(const ace_keyset *keys, const ace_block *blocks, uint32_t n_blocks,
                             void *d_workspace, size_t ws_bytes, uint32_t flags, void *stream);

/*
 * ace_verify_attestations -- the paper's attestation form (Def. 3.1 with the
 * validator's payload binding of Alg. 2), over n_blocks blocks in one pass.
 * Each transaction carries a payload P and a 72-byte attestation record
 *   obj_hash (32 bytes) || domain (8 bytes, opaque) || credential (32 bytes)
 * and
 *   valid_i = (id_i < n_id) and (off_i <= off_{i+1}) and
 *             SHA-256(P_i) == obj_hash_i and
 *             HMAC-SHA256(k_{id_i}, obj_hash_i || domain_i) == credential_i
 * (both compares over all 32 bytes, no early exit).  The ace_block fields
 * are read as: d_msg / d_off the payloads, d_tag [n_tx][72] the attestation
 * records (4-byte aligned); the rest as in ace_verify_batch.  Keyset, flags,
 * workspace (ace_verify_workspace_size with the same arguments), errors and
 * stream semantics are those of ace_verify_batch.
 */
ACE_API int ace_verify_attestations(const ace_keyset *keys, const ace_block *blocks,
                                    uint32_t n_blocks, void *d_workspace, size_t ws_bytes,
                                    uint32_t flags, void *stream);

/*
 * ace_verify_batch_noalloc -- ace_verify_batch for callers that cannot
 * allocate device memory or pass a workspace: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  Same operation,
 * arguments (less the workspace), flags, results, errors and stream
 * semantics as ace_verify_batch; the call allocates nothing (no hipMalloc,
 * no stream or event) and uses instead a scratch array of
 * ACE_SCRATCH_BYTES that the library holds in each GPU's memory until the
 * process ends.
 *   - A call whose workspace (ace_verify_workspace_size with the same
 *     arguments) exceeds ACE_SCRATCH_BYTES returns ACE_ERR_TOO_LARGE before
 *     anything is enqueued.  A binned call needs about 28 bytes per
 *     transaction (64 MiB: about 2.3M transactions with cached midstates);
 *     keys derived in the call add 64 bytes per identity; an ordered call
 *     needs only the block table and those midstates.
 *   - Every call on one GPU uses that GPU's one array: calls that overlap on
 *     one GPU (on different streams, or from different threads, without
 *     ordering between them) race and give undefined results.  Calls ordered
 *     on one stream are safe; each clears what it needs.
 *   - With keys derived in a binned call, the derivation runs on `stream`
 *     before the binning passes (ace_verify_batch may run it beside them on
 *     a second stream).  Stage timing (ace_profile_enable) does not cover it.
 */
#define ACE_SCRATCH_BYTES (64u << 20)
ACE_API int ace_verify_batch_noalloc(const ace_keyset *keys, const ace_block *blocks,
                                     uint32_t n_blocks, uint32_t flags, void *stream);

/*
 * Tuning of the launch shapes (process-wide).  The autotuner measures the
 * candidates on the device and installs the fastest with ace_set_tuning.
 *   binned_min_tx      batches of at least this many transactions are binned
 *                      by block count when the caller leaves the mode open
 *   verify_wgs_per_cu  workgroups per CU of the persistent verify kernel and
 *                      of the graph's in-order verify ("tiles per CU")
 *   aux_wgs_per_cu     workgroups per CU of the binning and finalize passes
 *   auto_persistent    1: binned batches in the open mode use the persistent
 *                      verify kernel
 *   derive_wgs_per_cu  workgroups per CU of the key derivation while it runs
 *                      beside the binning passes (keys derived in a binned
 *                      call); 0: as with the GPU to itself (at most four
 *                      per CU, each lane striding over the identities)
 *   wide_min_len       binned calls: messages of at least this many bytes are
 *                      verified from their block's offsets instead of the
 *                      32-bit length of the bin-order record.  Default and
 *                      largest value 2^31 - 1 (the record's length limit);
 *                      lower values change no result and only move messages
 *                      onto that path (tests use them to reach it without
 *                      2 GiB messages).
 *   grab_cap           persistent verify kernel, per length bucket: a wave
 *                      that last worked on messages of b + 1 inner blocks
 *                      (b = 63: 64 or more) takes at most grab_cap[b] wave
 *                      tiles of 64 transactions per atomic grab of the work
 *                      counter; 0: no cap (8, fewer when the batch is too
 *                      small for every wave to make four grabs).
 * ace_set_tuning rejects workgroup counts outside 1..64 (derive_wgs_per_cu:
 * 0..64), wide_min_len outside 1..2^31 - 1 and grab caps above 8.
 */
#define ACE_LENGTH_BUCKETS 64
typedef struct {
    uint64_t binned_min_tx;
    uint32_t verify_wgs_per_cu;
    uint32_t aux_wgs_per_cu;
    uint32_t auto_persistent;
    uint32_t derive_wgs_per_cu;
    uint64_t wide_min_len;
    uint8_t grab_cap[ACE_LENGTH_BUCKETS];
} ace_tuning;

ACE_API int ace_get_tuning(ace_tuning *out);
ACE_API int ace_set_tuning(const ace_tuning *t);

/*
 * Captured batches (hipGraph).  ace_graph_create captures the whole pass for
 * up to max_blocks blocks and max_tx transactions in all, with the keyset
 * fixed, into two graph instances that read their block list from pinned host
 * memory through a device-side plan kernel; so one capture replays for any
 * mix of block count, block sizes and message lengths within the maxima.
 * Every grid is fixed: the binned verify kernel is launched for the largest
 * batch (surplus waves exit at once) or, with ACE_PERSISTENT, as the
 * persistent kernel; the in-order form (flag ACE_ORDERED) is a grid-stride
 * kernel.  The launch tuning in force at ace_graph_create is captured with
 * the graph; later ace_set_tuning calls do not change its replays.
 *   d_workspace  at least ace_graph_workspace_size() bytes, 256-byte aligned,
 *                owned by the graph until ace_graph_destroy.
 * ace_graph_launch enqueues one replay on `stream` for the given blocks (the
 * same validity rules as ace_verify_batch).  Replays must be ordered on one
 * stream (they share the workspace).  The call blocks only when the pinned
 * block list it is about to reuse still belongs to the replay before the
 * previous one.  The keyset's device arrays must outlive the graph.
 * ace_graph_destroy waits for outstanding replays and frees the graph.
 */
typedef struct ace_graph ace_graph;

ACE_API size_t ace_graph_workspace_size(const ace_keyset *keys, uint32_t max_blocks,
                                        uint64_t max_tx, uint32_t flags);
ACE_API int ace_graph_create(const ace_keyset *keys, uint32_t max_blocks, uint64_t max_tx,
                             void *d_workspace, size_t ws_bytes, uint32_t flags, ace_graph **out);
ACE_API int ace_graph_launch(ace_graph *g, const ace_block *blocks, uint32_t n_blocks,
                             void *stream);
ACE_API int ace_graph_destroy(ace_graph *g);

/*
 * Serving (continuous batching).  ace_stream_create starts a server thread
 * that owns the device arena `d_arena` (caller-allocated, 256-byte aligned)
 * and `staging_bytes` of pinned host memory (allocated here, once).
 * ace_verify_stream submits one request -- a block of transactions in host
 * memory -- and returns a ticket.  The request is copied into staging before
 * the call returns, so the caller may reuse its input buffers at once; the
 * outputs h_bitmask_out ([ceil(n_tx/32)] words) and h_count_out are written
 * when the ticket completes and must stay valid until then.  Queued requests
 * are admitted into a batch as soon as arena space and one of max_inflight
 * batch slots are free; each batch is one multi-block verify pass on its own
 * HIP stream, so a batch admitted while others run overlaps them on the
 * device.  A request's result does not depend on what it is batched with.
 *   keys   ACE_KEYS_MIDSTATE (the cache stays where it is), or ACE_KEYS_REV:
 *          the midstates are derived once into the front of the arena and
 *          stay resident.
 *   flags  ACE_STREAM_PLAIN: one request per launch, in arrival order, each
 *          finished before the next starts (the reference form).
 * ace_verify_stream errors: ACE_ERR_TOO_LARGE when the request can never fit
 * staging or arena (with its workspace); with ACE_NONBLOCK, ACE_ERR_AGAIN
 * when staging is full right now (without it the call waits for room).
 * ace_stream_poll returns ACE_OK when done, ACE_ERR_AGAIN while pending
 * (wait = 0), or the request's error.  ace_stream_ticket_times gives the
 * submit, admit and completion times in seconds of the monotonic clock
 * (CLOCK_MONOTONIC).
 * ace_stream_release forgets a completed ticket.  ace_stream_destroy finishes
 * every queued and running request, then frees the engine (not the arena).
 */
#define ACE_NONBLOCK 0x1u
#define ACE_STREAM_PLAIN 0x1u

typedef struct ace_stream ace_stream;
typedef struct {
    uint64_t submitted;
    uint64_t completed;
    uint64_t failed;
    uint64_t batches;
    uint64_t max_batch_requests;
    uint64_t pending;
    uint64_t arena_peak_bytes;
    uint64_t arena_capacity_bytes;
} ace_stream_stats;

ACE_API int ace_stream_create(const ace_keyset *keys, void *d_arena, size_t arena_bytes,
                              size_t staging_bytes, uint32_t max_inflight, uint32_t flags,
                              ace_stream **out);
ACE_API int ace_verify_stream(ace_stream *s, const uint8_t *h_msg, const uint64_t *h_off,
                              const uint32_t *h_id, const uint8_t *h_tag, uint64_t n_tx,
                              uint32_t *h_bitmask_out, uint64_t *h_count_out, uint32_t flags,
                              uint64_t *ticket_out);
ACE_API int ace_stream_poll(ace_stream *s, uint64_t ticket, int wait);
ACE_API int ace_stream_ticket_times(ace_stream *s, uint64_t ticket, double *submit_s,
                                    double *admit_s, double *done_s);
ACE_API int ace_stream_release(ace_stream *s, uint64_t ticket);
ACE_API int ace_stream_get_stats(ace_stream *s, ace_stream_stats *out);
ACE_API int ace_stream_destroy(ace_stream *s);

/*
 * Test hook: the same engine with a host backend -- the "arena" is host memory
 * allocated here, and each batch's blocks are verified by calling `fn` (for
 * example a CPU reference) -- so the queue, admission and retirement logic
 * runs without a GPU.  fail_after = k > 0 makes the k-th batch fail as a
 * device error would; only that batch's requests fail.  With the flag
 * ACE_STREAM_HOST_FAIL_LAUNCH the k-th batch's verify call itself returns the
 * error (after its input copies were queued), which takes the engine's
 * launch-failure path: the slot is drained before the batch's memory is
 * reused.
 */
#define ACE_STREAM_HOST_FAIL_LAUNCH 0x100u
typedef int (*ace_host_verify_fn)(void *user, const uint8_t *msg, const uint64_t *off,
                                  const uint32_t *id, const uint8_t *tag, uint64_t n_tx,
                                  uint32_t *bitmask_out, uint64_t *count_out);
ACE_API int ace_stream_create_host(ace_host_verify_fn fn, void *user, size_t arena_bytes,
                                   size_t staging_bytes, uint32_t max_inflight, uint32_t flags,
                                   uint32_t fail_after, ace_stream **out);

/*
 * Stage timing (tracing).  While enabled on the calling thread, every
 * ace_verify_batch call records HIP events on its own stream around its
 * stages: key derivation, length binning (count, scan, scatter), the verify
 * kernel and the finalize pass.  ace_profile_read() waits for the recorded
 * events and returns the summed milliseconds of all profiled calls since the
 * last reset (reset != 0 clears them).  Stages a call did not run add 0.
 * In the binned form with keys derived in the call, the derivation runs on
 * a second stream beside the binning passes; the derive stage then reads
 * about 0 and bin_ms covers both, up to the join before the verify kernel.
 */
typedef struct {
    double derive_ms;
    double bin_ms;
    double verify_ms;
    double finalize_ms;
    double total_ms;
    uint64_t calls;
} ace_profile;

ACE_API int ace_profile_enable(int on);
ACE_API int ace_profile_read(ace_profile *out, int reset);

/*
 * Merkle roots of the block header's transaction and attestation lists
 * (App. C, fields tx_merkle_root and attest_merkle_root; a validator
 * recomputes the attestation root before voting, Alg. 4).  The paper fixes
 * no leaf or odd-node rule; the one implemented: leaf node = SHA-256(leaf
 * bytes), parent = SHA-256(left || right), at a level with an odd count the
 * last node moves up unchanged (the left-complete shape of RFC 6962, without
 * its prefix bytes), and a tree without leaves has root SHA-256("").  A leaf
 * with off[i+1] < off[i] is hashed as the empty string.
 */
typedef struct {
    const uint8_t *d_data;   /* leaves back to back; may be NULL only if n_leaves == 0    */
    const uint64_t *d_off;   /* [n_leaves + 1] byte offsets into d_data (8-byte aligned) */
    uint64_t n_leaves;
    uint8_t *d_root_out;     /* 32 bytes, 4-byte aligned                                  */
} ace_merkle_tree;

/* Workspace bytes for these trees: 32 per leaf plus small tables (0 on bad arguments). */
ACE_API size_t ace_merkle_workspace_size(const ace_merkle_tree *trees, uint32_t n_trees);

/*
 * ace_merkle_roots -- the roots of n_trees trees in one pass: every leaf of
 * every tree hashed in parallel, then one launch per tree level over all
 * trees.  h-side `trees` is read before the call returns; d_workspace is at
 * least ace_merkle_workspace_size() bytes, 256-byte aligned.  Total leaves
 * <= ACE_MAX_TX, n_trees < 2^24.
 */
ACE_API int ace_merkle_roots(const ace_merkle_tree *trees, uint32_t n_trees, void *d_workspace,
                             size_t ws_bytes, void *stream);

/*
 * ace_poh_verify -- segments of the SHA-256 hash chain that the consensus
 * section uses as its clock (H_{i+1} = SHA-256(H_i), the 32 digest bytes
 * hashed as a 32-byte message).  Segment i is valid iff applying SHA-256
 * steps_i times to start[i] gives end[i] (full 32-byte compare), where
 * steps_i = d_steps[i], or `steps` for every segment when d_steps is NULL.
 *   d_start, d_end  [n_segments][32] bytes, 4-byte aligned.  For the
 *                   checkpoints C[0..n] of one chain pass d_start = C and
 *                   d_end = C + 32.
 *   d_bitmask_out   [ceil(n_segments / 32)] words, fully written.
 *   d_count_out     one uint64: number of valid segments (0 for n == 0).
 * Segments run in parallel, each one's hashes in sequence, so a launch
 * needs many segments (hundreds of thousands) to fill the device.
 */
ACE_API int ace_poh_verify(const uint8_t *d_start, const uint8_t *d_end, const uint32_t *d_steps,
                           uint32_t steps, uint64_t n_segments, uint32_t *d_bitmask_out,
                           uint64_t *d_count_out, void *stream);

/*
 * ace_valu_rate -- measurement aid, not a step of the method: the INT32 VALU
 * issue rate the verify kernels are priced against.  Launches wgs_per_cu
 * workgroups of 256 lanes per CU, each lane running `iters` x 192 dependent
 * alignbit / bitop3 / add3 instructions (eight independent chains), times the
 * launch with HIP events on `stream`, waits for it, and stores lane
 * instructions per second in *out_lane_instr_per_s.  d_sink: 4 bytes of
 * device memory the kernel never writes in practice (it keeps the compiler
 * from removing the work).  iters >= 1, wgs_per_cu in 1..64.
 */
ACE_API int ace_valu_rate(uint32_t iters, uint32_t wgs_per_cu, uint32_t *d_sink,
                          double *out_lane_instr_per_s, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ACE_H */
