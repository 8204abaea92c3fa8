/*
 * kbatch -- batch-mode SHA-3 on AMD MI355X (gfx950).
 *
 * C ABI of libkbatch.so.  Batch mode (Section 4 of "GPU Accelerated Keccak
 * (SHA3) Algorithm"): many independent messages, each hashed on its own with
 * SHA3-224/256/384/512 (Section 3.3, eqs. 13-16: Keccak[c = 2d] over
 * M || 01 with pad10*1, eq. 11, and Keccak-f[1600], Section 3.1), one digest
 * per message.  Tree mode (Section 4): merkle_root().
 *
 * Conventions shared by every entry point:
 *   - Pointers named d_* are device memory owned by the caller (for example
 *     a torch tensor's data_ptr()); the library never frees them.
 *   - Work is enqueued on `stream` (NULL = the default stream) and the call
 *     returns without waiting for it.  Inputs must stay valid and unchanged,
 *     and outputs untouched, until the stream reaches that point.
 *   - Messages are byte strings.  Message i is the d_lengths[i] bytes at
 *     d_data + d_offsets[i]; offsets may be unaligned and slices may
 *     overlap; length 0 is valid.  offsets[i] + lengths[i] must not exceed
 *     the d_data allocation: the library cannot check that on the host (the
 *     Python binding does).  d_offsets and d_lengths must be 8-byte aligned,
 *     d_digests 4-byte aligned, and digests must not alias any input.
 *   - n == 0 is a no-op returning KB_OK; NULL pointers are then allowed.
 *   - On error nothing is enqueued, the call returns a KB_E* code and
 *     keccak_last_error() (per host thread) describes it.
 *   - The library owns per-(device, stream) workspace that grows on demand;
 *     growing it waits for the device.  keccak_reserve() sizes it up front,
 *     keccak_release() frees it.  Calls on one stream are ordered; calls on
 *     different streams use different workspaces and may run concurrently.
 *     Host threads that share one stream must not call into the library on
 *     it at the same time (a call may grow the workspace another call on
 *     that stream is about to use).
 */
#ifndef KBATCH_H
#define KBATCH_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* SHA-3 variants (Section 3.3): digest d bits, capacity c = 2d, rate
 * r = 1600 - c.  Digest/rate in bytes: 28/144, 32/136, 48/104, 64/72. */
enum kb_variant { KB_SHA3_224 = 0, KB_SHA3_256 = 1, KB_SHA3_384 = 2, KB_SHA3_512 = 3 };

enum kb_status {
  KB_OK = 0,
  KB_EINVAL = -1, /* bad argument: variant, NULL pointer with n > 0, alignment, leaf_size 0 */
  KB_ENOMEM = -2, /* workspace could not be allocated */
  KB_EHIP = -3    /* a HIP runtime call or kernel launch failed */
};

/* Scheduling forms of a batch (all give identical digests). */
enum kb_mode {
  KB_MODE_PERSISTENT = 0, /* four launches, no host wait: arrival order, hashing every
                             64-message chunk of one-block messages at once; then a plan,
                             a scatter into buckets of equal block count, and a resident
                             grid hashing the buckets longest first (the longest messages
                             in the wide split form) */
  KB_MODE_PLAIN = 1,      /* one thread per message in arrival order, one launch (the
                             paper's "one thread per message", Section 4.1) */
  KB_MODE_PER_BUCKET = 2, /* bucket by block count, one plain launch per bucket (waits on
                             the host for the bucket sizes) */
  KB_MODE_SPLIT = 3,      /* latency form: five lanes of a wave share one state, eight
                             messages per wave in arrival order (the serial absorb chain
                             of Section 3.2 runs about twice as fast per message, at a
                             fraction of the batch throughput) */
  KB_MODE_WIDE = 4,       /* wide latency form: one 64-bit state word per lane, 32 lanes
                             per state, two messages per wave in arrival order (each
                             lane issues about twenty VALU instructions per round, with
                             two exchanges through LDS; for the fewest, longest chains) */
  KB_MODE_PAIR = 5        /* pair form: two lanes per state, each holding one 32-bit half
                             of every state word, 32 messages per wave in arrival order
                             (about 1.5 times one thread's chain speed at a third more
                             issue slots per permutation) */
};

/*
 * Tuning knobs of the persistent form; a zero field means "library default".
 * Messages are grouped by block count nb = floor(L / R) + 1 into
 * KB_NB_CLASSES classes, class c = floor(log2(nb)) capped at
 * KB_NB_CLASSES - 1 (1, 2-3, 4-7, ..., 128 or more blocks); the class
 * arrays give a choice per class, applied on the device to each bucket of
 * equal block counts.
 */
#define KB_NB_CLASSES 8
enum kb_staging {
  KB_STAGING_DEFAULT = 0,
  KB_STAGING_DIRECT = 1,   /* each block loaded when it is absorbed (fewer registers) */
  KB_STAGING_PREFETCH = 2  /* the next block's 16-byte chunks loaded into registers while
                              the current block is permuted (the default) */
};
typedef struct kb_tile {
  int32_t block_threads;    /* 0 or 256: the hashing kernels use 256-thread workgroups */
  int32_t waves_per_simd;   /* persistent grid: resident waves per SIMD (1..8) */
  int32_t steps_per_item;   /* wave-blocks of work per queue item (>= 1) */
  int32_t staging;          /* kb_staging: how a message's next block reaches the sponge */
  int32_t class_steps[KB_NB_CLASSES];    /* per class: steps per queue item (0 = steps_per_item) */
  int32_t class_threads[KB_NB_CLASSES];  /* per class: threads per state, 1 (one lane hashes a
                                            message) or KB_THREADS_WIDE (the split tail: 32
                                            lanes per state in the wide form, Section 3.2's
                                            absorb chain about three times as fast); 0 = the
                                            library's rule.  SHA-3 variants only; the split
                                            classes must be the longest ones (a class is split
                                            only if every longer class present is) */
} kb_tile;
#define KB_THREADS_WIDE 32

/*
 * keccak_batch -- SHA3-{224,256,384,512} of n messages (batch mode, Section
 * 4; the sponge of Section 3.2 over Keccak-f[1600] of Section 3.1).
 *   variant    kb_variant.
 *   d_data     message bytes.
 *   d_offsets  uint64[n] byte offsets into d_data.
 *   d_lengths  uint64[n] byte lengths.
 *   n          number of messages (< 2^32).
 *   d_digests  uint8[n * D] output, digest i at i * D (D = digest bytes).
 * Uses the persistent, length-bucketed form (KB_MODE_PERSISTENT).
 */
int keccak_batch(int variant, const uint8_t* d_data, const uint64_t* d_offsets,
                 const uint64_t* d_lengths, uint64_t n, uint8_t* d_digests, hipStream_t stream);

/*
 * keccak_batch_noalloc -- keccak_batch that allocates nothing, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The scheduling workspace
 * is one static array on each device (about 4.6 MiB, for up to
 * KB_NOALLOC_MAX_MSGS messages), present from the library's load until the
 * process ends; the first call on a device looks it up and clears it on
 * `stream`, and each call leaves it cleared for the next.  Every call on a
 * device shares that one array: calls that overlap on one device (on
 * different streams, or from host threads at once) race on it and give
 * wrong digests, so serialise them.  Same arguments, output and persistent
 * form as keccak_batch; KB_EINVAL for n > KB_NOALLOC_MAX_MSGS.
 */
#define KB_NOALLOC_MAX_MSGS (1u << 20)
int keccak_batch_noalloc(int variant, const uint8_t* d_data, const uint64_t* d_offsets,
                         const uint64_t* d_lengths, uint64_t n, uint8_t* d_digests,
                         hipStream_t stream);

/*
 * keccak_batch_mixed -- like keccak_batch with a variant per message.
 *   d_variants  uint8[n], each 0..3 (kb_variant).
 *   d_digests   uint8[n * 64]; slot i holds digest i followed by zeros.  A
 *               slot whose variant byte is out of range is all zeros.
 */
int keccak_batch_mixed(const uint8_t* d_variants, const uint8_t* d_data,
                       const uint64_t* d_offsets, const uint64_t* d_lengths, uint64_t n,
                       uint8_t* d_digests, hipStream_t stream);

/*
 * keccak_batch_xof -- SHAKE128 / SHAKE256 of n messages (Section 3.3, eqs.
 * 17-18: Keccak[c = 2 * security] over M || 1111 with pad10*1), each
 * squeezed to out_len bytes (Section 3.2: the output is read r bits at a
 * time with the permutation applied between reads).
 *   security   128 or 256.
 *   out_len    output bytes per message (> 0 when n > 0).
 *   d_out      uint8[n * out_len], output i at i * out_len (any alignment).
 * Persistent, length-bucketed form.  Other arguments as keccak_batch.
 */
int keccak_batch_xof(int security, const uint8_t* d_data, const uint64_t* d_offsets,
                     const uint64_t* d_lengths, uint64_t n, uint64_t out_len, uint8_t* d_out,
                     hipStream_t stream);

/*
 * keccak_batch_xof_ex -- keccak_batch_xof with an explicit scheduling mode
 * (KB_MODE_PERSISTENT, _PLAIN, _PER_BUCKET, _SPLIT or _WIDE; in the split
 * forms five or 32 lanes share each state and squeeze it, which shortens each
 * message's chain of permutations for a few long messages).  Same output;
 * KB_EINVAL for an unknown mode.
 */
int keccak_batch_xof_ex(int security, const uint8_t* d_data, const uint64_t* d_offsets,
                        const uint64_t* d_lengths, uint64_t n, uint64_t out_len, uint8_t* d_out,
                        int mode, hipStream_t stream);

/*
 * keccak_batch_ex -- either form above with an explicit scheduling mode and
 * tile (tile may be NULL).  variant = -1 selects the mixed form (d_variants
 * required, 64-byte output slots); otherwise d_variants is ignored.
 */
int keccak_batch_ex(int variant, const uint8_t* d_variants, const uint8_t* d_data,
                    const uint64_t* d_offsets, const uint64_t* d_lengths, uint64_t n,
                    uint8_t* d_digests, int mode, const kb_tile* tile, hipStream_t stream);

/*
 * merkle_root -- tree mode (Section 4: messages hashed in twos up to one
 * root).  The input is cut into n = max(1, ceil(total_len / leaf_size))
 * leaves of leaf_size bytes (the last may be short; total_len 0 gives one
 * empty leaf).  Leaf digest = H(leaf); a parent = H(left || right) over the
 * two D-byte child digests; an unpaired last node at a level is carried up
 * unchanged.  H is the SHA-3 `variant`.  The D-byte root is written to
 * d_root (device memory).  leaf_size 0 is KB_EINVAL.  Leaves take a faster
 * load path when leaf_size, total_len and d_data are all multiples of 8; the
 * root does not depend on it.
 */
int merkle_root(int variant, const uint8_t* d_data, uint64_t total_len, uint64_t leaf_size,
                uint8_t* d_root, hipStream_t stream);

/*
 * keccak_autotune -- choose the tile of the persistent form for this batch.
 * Searches, keeping the fastest so far at each stage: resident waves per
 * SIMD {occupancy maximum, 1, 2, 3} x staging {prefetch, direct}; then
 * steps_per_item {1, 2, 4, 8, 16, 32}; then threads per state by
 * block-count class (the wide split tail from each class present upward, or
 * one lane everywhere); then steps per queue item for each class present
 * {1, 4, 16}.  Every candidate's digests are first compared with the plain
 * form's bit for bit (a candidate that differs is discarded and counted in
 * *rejected); the verified ones are timed with HIP events (median of `reps`
 * runs).  The fastest goes to *best and its time to *best_ms.  Arguments as
 * keccak_batch_ex; variant -1 = mixed.  Synchronous; allocates two output
 * buffers of the batch's digest size for its duration.  Store the result
 * with keccak_tune_store to have batch calls pick it up.
 */
int keccak_autotune(int variant, const uint8_t* d_variants, const uint8_t* d_data,
                    const uint64_t* d_offsets, const uint64_t* d_lengths, uint64_t n, int reps,
                    kb_tile* best, double* best_ms, int* rejected, hipStream_t stream);

/*
 * The autotuner's cache (a JSON file; tune_cache.cpp documents the format).
 * Entries are keyed by (GPU architecture, ROCm version, variant, block-count
 * class, batch class = floor(log2(n))): the launch-wide knobs
 * (waves_per_simd, steps_per_item, staging) under block-count class "*", the
 * per-class knobs (class_steps, class_threads) under their class.  `arch`
 * and `rocm` name the key's device ("gfx950", "7.2"); pass both NULL for the
 * current HIP device (its architecture without target features, and the HIP
 * runtime's major.minor version).
 *
 * keccak_tune_store -- merge `tile`, as tuned for a batch of n messages of
 * `variant` (-1 = mixed), into the cache file at `path` (created if
 * missing), replacing entries with the same key; `ms` is recorded beside it
 * (< 0: none).  Entries are written for the launch-wide knobs and for each
 * class whose class_steps or class_threads is set.  KB_EINVAL for a NULL
 * path or tile, an unknown variant, n == 0, only one of arch/rocm given, a
 * malformed existing file or a write failure.
 *
 * keccak_tune_lookup -- the tile the cache at `path` (NULL: the file named
 * by the environment variable KBATCH_TUNE) holds for a batch of n messages
 * of `variant`: returns 1 and fills *out if any entry matches, 0 (and a zero
 * tile) if none does or no file is named, KB_EINVAL for a malformed file.
 *
 * With KBATCH_TUNE set, keccak_batch, keccak_batch_mixed and keccak_batch_ex
 * (persistent mode, tile NULL) look their batch up for the current device
 * and run the cached tile.  keccak_last_tile -- the tile the calling
 * thread's last such batch call ran (a zero tile: the library defaults);
 * returns 1 if it came from the cache, else 0.
 */
int keccak_tune_store(const char* path, const char* arch, const char* rocm, int variant,
                      uint64_t n, const kb_tile* tile, double ms);
int keccak_tune_lookup(const char* path, const char* arch, const char* rocm, int variant, uint64_t n,
                       kb_tile* out);
int keccak_last_tile(kb_tile* out);

/*
 * Keccak-p[b, n_r] (Section 3.1, eqs. 1-10; Table 1 gives the widths): apply
 * the permutation in place to n states of b bits each.
 *   b          25, 50, 100, 200, 400, 800 or 1600 (w = b/25 = 2^l)
 *   n_rounds   1..4096; round i_r runs from 12 + 2l - n_rounds to 12 + 2l - 1
 *              (FIPS 202's indexing, so b = 1600, n_rounds = 24 is
 *              Keccak-f[1600]); round constants by i_r mod 255
 *   d_states   device, n * ceil(b/8) bytes, state s at byte s * ceil(b/8);
 *              string bit k is bit (k mod 8) of byte k/8, so for b >= 200
 *              lane (x, y) is the w/8 little-endian bytes at (x + 5y) w/8.
 *              For b = 25, 50, 100 the unused high bits of each state's last
 *              byte are cleared.  Any alignment.
 * One thread per state; asynchronous on `stream`.  Returns KB_EINVAL for a
 * width not in Table 1, n_rounds out of range or a NULL d_states with n > 0.
 */
int keccak_p_batch(int b, int n_rounds, uint8_t* d_states, uint64_t n, hipStream_t stream);

/*
 * Graph capture of a whole batch (all scheduling kernels and the hashing
 * kernel) or a whole tree, for replay with one launch.  The arguments are
 * bound at capture time: replaying hashes whatever the bound buffers hold
 * then.  Each graph owns a private workspace (allocated at create, freed at
 * destroy), so direct calls and other graphs never disturb it; replays of
 * one graph must not overlap each other (replay it on one stream).  The
 * persistent, plain and split modes can be captured (not per-bucket, which
 * waits on the host).  `stream` is where the workspace is prepared and the
 * work recorded; a NULL stream records on a private stream, since the null
 * stream cannot be captured.  A graph replays on any stream.
 */
typedef struct kb_graph kb_graph;
int keccak_graph_create(int variant, const uint8_t* d_variants, const uint8_t* d_data,
                        const uint64_t* d_offsets, const uint64_t* d_lengths, uint64_t n,
                        uint8_t* d_digests, int mode, const kb_tile* tile, hipStream_t stream,
                        kb_graph** out);
/*
 * keccak_graph_create_counted -- capture the persistent form over a batch
 * whose message count is read from device memory each time the graph runs:
 * d_count (uint32, device) then holds n, taken as max_n if larger.  The
 * descriptor arrays and d_digests are sized for max_n messages.  For loops
 * with fixed-capacity buffers (a serving step fills the descriptors and the
 * count, then replays the graph).  max_n in [1, 2^32 - 1); other arguments
 * as keccak_graph_create (variant -1 = mixed).
 */
int keccak_graph_create_counted(int variant, const uint8_t* d_variants, const uint8_t* d_data,
                                const uint64_t* d_offsets, const uint64_t* d_lengths,
                                const uint32_t* d_count, uint64_t max_n, uint8_t* d_digests,
                                hipStream_t stream, kb_graph** out);
int keccak_graph_create_merkle(int variant, const uint8_t* d_data, uint64_t total_len,
                               uint64_t leaf_size, uint8_t* d_root, hipStream_t stream,
                               kb_graph** out);
int keccak_graph_launch(kb_graph* graph, hipStream_t stream);
int keccak_graph_destroy(kb_graph* graph);

/*
 * Serving: a continuous-batching request server over a device-resident byte
 * pool (batch mode of Section 4 applied to a stream of requests).  A request
 * is a variant and n slices (offset, length) of the pool, given as host
 * arrays (copied at submit).  A worker thread admits queued requests in
 * arrival order into steps while a step has room: at most max_step_msgs
 * message slots (the step's device buffers) and, if max_step_bytes is set,
 * at most that many message bytes (the step's work).  A request never
 * straddles steps; one larger than a step is rejected (KB_ENOMEM).  Up to
 * steps_in_flight steps run on the GPU at once, each with its own HIP
 * stream, pinned host buffers and device buffers (allocated at create), so
 * requests that arrive while steps run are admitted as soon as a step slot
 * frees up and their work overlaps the running steps.  Each step is one
 * replay of a HIP graph captured at create: the descriptor and count
 * uploads, both passes of the mixed-variant persistent form reading the
 * count from device memory, and the digest download (copy sizes set per
 * step).  Results are 64-byte digest slots, one per message, zero past the
 * digest.  Thread-safe: any thread may submit and poll.
 *
 * executor (optional): if set, the server never touches the GPU and instead
 * calls executor(user, variants, offsets, lengths, n, digests) on the worker
 * thread for every step (host arrays; the callback fills digests[n * 64] and
 * returns KB_OK).  d_pool is then not dereferenced.
 */
typedef int (*kb_step_executor)(void* user, const uint8_t* h_variants, const uint64_t* h_offsets,
                                const uint64_t* h_lengths, uint64_t n, uint8_t* h_digests);
enum { KB_SERVER_EAGER = 1 /* flags: steps as separate copies and launches, no graph */ };
typedef struct kb_server_config {
  const uint8_t* d_pool;   /* device byte pool the requests slice */
  uint64_t pool_bytes;     /* its size: every slice must lie inside */
  uint64_t max_step_msgs;  /* message slots per step */
  int32_t steps_in_flight; /* 1..8 */
  uint32_t flags;          /* KB_SERVER_EAGER or 0 */
  kb_step_executor executor;
  void* executor_user;
  uint64_t max_step_bytes; /* message bytes per step; 0 = no limit */
} kb_server_config;
typedef struct kb_server_stats {
  uint64_t steps, messages, bytes, completed, rejected, pending, max_step_msgs_seen;
  double step_busy_s; /* sum over steps of launch-to-completion time */
  double span_s;      /* first launch to last completion */
} kb_server_stats;
typedef struct kb_server kb_server;
int keccak_server_create(const kb_server_config* cfg, kb_server** out);
int keccak_server_submit(kb_server* server, int variant, const uint64_t* h_offsets,
                         const uint64_t* h_lengths, uint64_t n, uint64_t* request_id);
/* Ids of finished requests (up to max_ids), waiting up to wait_ms for one. */
int keccak_server_poll(kb_server* server, uint64_t* ids, uint64_t max_ids, uint64_t* count,
                       int wait_ms);
/* Copy a finished request's digests (n * 64 bytes) and latency (submit to
 * completion, ms) and forget the request. */
int keccak_server_result(kb_server* server, uint64_t id, uint8_t* h_out, uint64_t out_bytes,
                         double* latency_ms);
int keccak_server_stats(kb_server* server, kb_server_stats* out);
/* Finish every queued request, stop the worker and free the server. */
int keccak_server_destroy(kb_server* server);
/* Text of the last server error on the calling host thread. */
const char* keccak_server_last_error(void);

/* Bytes of device node buffer merkle_root uses for a tree of n_leaves leaves
 * of the SHA-3 `variant` (every level but the root, each level 16-byte
 * aligned, plus one digest); 0 for a variant out of range.  Host only. */
uint64_t keccak_tree_workspace_bytes(int variant, uint64_t n_leaves);

/* Digest and rate sizes in bytes of a variant; -1 if it is out of range. */
int keccak_digest_bytes(int variant);
int keccak_rate_bytes(int variant);

/* Pre-size the workspace of (current device, stream) for batches of up to
 * max_msgs messages and trees of up to max_leaves leaves. */
int keccak_reserve(uint64_t max_msgs, uint64_t max_leaves, hipStream_t stream);

/* Free every workspace this process holds (waits for the devices). */
int keccak_release(void);

/* Measurement hook.  While enabled (on != 0) every hashing-kernel launch
 * (both passes of the persistent form, the plain, split and tree kernels)
 * is bracketed by a pair of HIP events recorded on the stream it is launched
 * on.  Enabling clears the record.  Launches recorded into a graph are not
 * bracketed. */
int keccak_timing_enable(int on);

/* keccak_timing_enable restricted to the kernel kinds (enum kb_kernel) whose
 * bit, 1 << kind, is set in `kinds`; 0 disables timing, and enabling clears
 * the record.  Every bracket adds two event records to the launch stream,
 * each a few microseconds of stream time, so a caller that times one kind
 * of kernel inside a timed region brackets only that kind.  KB_EINVAL for a
 * bit above KB_KERNEL_PAIR. */
int keccak_timing_enable_kinds(uint32_t kinds);

/* Sum of the bracketed kernel durations in milliseconds and the number of
 * bracketed launches since timing was enabled; waits for those events. */
int keccak_timing_read(double* total_ms, uint64_t* launches);

/* Kinds of bracketed kernels. */
enum kb_kernel {
  KB_KERNEL_FIRST_PASS = 0,  /* persistent form: the arrival-order pass */
  KB_KERNEL_SECOND_PASS = 1, /* persistent form: the bucketed pass */
  KB_KERNEL_PLAIN = 2,       /* one thread per message (plain and per-bucket forms) */
  KB_KERNEL_SPLIT = 3,       /* lane-split form */
  KB_KERNEL_TREE = 4,        /* tree mode */
  KB_KERNEL_WIDE = 5,        /* wide lane-split form */
  KB_KERNEL_SCHEDULE = 6,    /* persistent form: the plan and the bucketing scatter */
  KB_KERNEL_PAIR = 7         /* pair form */
};

/* keccak_timing_read restricted to the kernels of one kind; KB_EINVAL for
 * an unknown kind. */
int keccak_timing_read_kernel(int kind, double* total_ms, uint64_t* launches);

/* Probe: sustained 32-bit VALU issue rate of the current device (tera
 * lane-operations per second; a grid of 8 waves per SIMD running `iters`
 * iterations of 16 independent v_bitop3 chains per lane) and the shader clock
 * seen by that kernel (MHz, from the shader and constant-rate counters).
 * Synchronous; allocates 20 bytes of device memory for its duration. */
int keccak_probe_valu(uint32_t iters, double* tops, double* sclk_mhz, hipStream_t stream);

/* Probe: throughput of the library's Keccak-f[1600] (Section 3.1) with the
 * states held in registers and no memory traffic: one state per thread,
 * `iters` permutations each, on a grid of `waves_per_simd` 256-thread
 * workgroups per compute unit (0 or more than fit at once: as many as fit).
 * *gperm_s = permutations per second / 1e9; *waves_used = waves per SIMD
 * launched.  This is the ceiling a hashing kernel reaches with its loads,
 * padding and stores fully hidden.  Synchronous; allocates 4 bytes of device
 * memory for its duration.  KB_EINVAL for null outputs, iters == 0 or a
 * negative wave count. */
int keccak_probe_perm(uint32_t iters, int waves_per_simd, double* gperm_s, int* waves_used,
                      hipStream_t stream);

/* Probe: one device-to-device copy of `bytes` (a multiple of 16, both
 * pointers 16-byte aligned); *gbps = 2 * bytes / time (read + write).
 * Synchronous.  Used to calibrate memory-traffic counters. */
int keccak_probe_copy(const uint8_t* d_src, uint8_t* d_dst, uint64_t bytes, double* gbps,
                      hipStream_t stream);

/* Text of the last error on the calling host thread ("" if none). */
const char* keccak_last_error(void);

/* Library version string: "kbatch <version> (gfx950) src <hash>", where <hash>
 * names the kernel sources the library was built from (the first 16 hex
 * digits of the SHA-256 over the kernel source directory). */
const char* keccak_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KBATCH_H */
