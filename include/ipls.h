/*
 * ipls.h: C ABI of the MI355X (gfx950) In-Place Parallel Learned Sort library.
 *
 * The library sorts numeric keys on one GPU with the IPLS distribution recursion: fit a linear
 * partition model with Fastest Minimum Conflict Degree (FMCD) on a sorted sample of a bucket,
 * classify every key of the bucket with one fp64 fused multiply-add, distribute the keys stably
 * into contiguous sub-buckets, recurse on sub-buckets above the base-case size and finish the
 * rest with an in-LDS base-case sort (paper: Proposed Algorithm chapter; the model and its
 * fit: Linear Models section; the sample -> sort -> train -> predict pipeline: Machine Learning
 * Models chapter).  Optionally a two-level piecewise-linear CDF model (Recursive Model Index
 * section) replaces FMCD on a bucket when its maximum sample load is lower; equality buckets
 * (IPS4o's, for heavily repeated values) and IPS4o's splitter tree (the comparison classifier,
 * Decision Trees section, as an A/B baseline) are available as options.  Beside the single-array
 * sort: a segmented (batched) sort with an autotuner, and a request server.
 *
 * Conventions for every entry point:
 *   - Array pointers are DEVICE pointers unless marked "host".  The caller owns them; the
 *     library never frees or keeps them after the call returns.
 *   - Work is enqueued on `stream` (NULL = the default stream).  The sort entry points read a
 *     few bytes back from the device once per recursion level to size the next level's
 *     launches (the device writes them into pinned host memory, where the calling thread polls
 *     for them), so they return only after the sort has completed on `stream`.  Each engine
 *     context also owns one stream of its own (non-blocking, default priority) on which the base
 *     case of a level runs beside the next level's partition (the last level's runs on
 *     `stream`); `stream` waits for it (events) before the call returns, so work the caller
 *     queues on `stream` afterwards sees the finished result.
 *   - Keys are ordered by IEEE 754 totalOrder (-0 before +0; NaNs are accepted and sort to the
 *     end their sign bit gives).  u64 keys are plain unsigned integers.
 *   - Results are deterministic and bit-identical for identical inputs and parameters; with a
 *     payload the sort is stable, so the output is unique.
 *   - Argument errors are reported synchronously and nothing is enqueued.  No C++ exception
 *     crosses this interface.  With IPLS_VERBOSE set in the environment, a HIP call that fails
 *     inside the library (the cause of IPLS_ERR_HIP) is reported on stderr with its error name.
 *   - With IPLS_DEBUG_CHECKS=1 in the environment (read on every call), the sort entry points
 *     that may allocate check the sort's invariants on the device: after every distribution pass
 *     each bucketed array's histogram sums to its key count, the pass moved the same multiset of
 *     keys (and payloads), and every key lies in the bucket its model gives it; at the end every
 *     segment is sorted and holds its input's multiset.  A failed check returns IPLS_ERR_DEVICE.
 *     The checks cost several extra passes over the data.  IPLS_DEBUG_CHECKS=2 also plants a
 *     mismatch in the final multiset comparison, to exercise that error path.
 *   - The plain entry points share one engine context per device: their calls are serialised
 *     (one runs at a time), and the buffers the library allocates for its own use are cached in
 *     that context and reused across calls.  The request server's lanes own contexts of their
 *     own and run concurrently on their own streams.
 */
#ifndef IPLS_H
#define IPLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { IPLS_F64 = 0, IPLS_F32 = 1, IPLS_U64 = 2 } ipls_dtype;

typedef enum {
    IPLS_OK = 0,
    IPLS_ERR_INVALID = 1,     /* bad argument: null pointer with n > 0, bad parameter, bad offsets */
    IPLS_ERR_DTYPE = 2,       /* unknown dtype */
    IPLS_ERR_OOM = 3,         /* device allocation failed */
    IPLS_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed */
    IPLS_ERR_DEVICE = 5,      /* a device-side check failed (capacity, recursion limit, offsets) */
    IPLS_ERR_UNSUPPORTED = 6  /* valid request outside what this build supports (e.g. K > 256) */
} ipls_status;

/* Model selection for each partitioned bucket. */
typedef enum {
    IPLS_MODEL_FMCD = 0, /* linear model fitted by FMCD (the paper's IPLS) */
    IPLS_MODEL_AUTO = 1, /* two-level model iff its max sample load is strictly lower than FMCD's */
    IPLS_MODEL_L2PL = 2, /* two-level model whenever it splits the sample (FMCD otherwise) */
    IPLS_MODEL_TREE = 3  /* splitter tree over the K-1 sample quantiles (IPS4o's comparison classifier,
                          * the Decision Trees section): the A/B baseline of the learned models */
} ipls_model_policy;

/* Tuning parameters.  ipls_default_params() fills the defaults. */
typedef struct {
    uint32_t num_buckets;    /* K, buckets per partition, 4..256 (default 256, Proposed Algorithm) */
    uint32_t base_case_max;  /* T, buckets of <= T keys go to the base case, 1..4096 (default 4096) */
    uint32_t sample_divisor; /* policy 0: sample size S = ceil(n / divisor), >= 2 (default 100: a 1% sample) */
    uint32_t sample_min;     /* ... raised to at least this (0 = 2K, or none under policy 1); <= base_case_max */
    uint64_t sample_max;     /* ... and capped at this (0 = no cap); S never exceeds n */
    uint64_t seed;           /* seed of the sample positions' jitter */
    uint32_t model;          /* ipls_model_policy */
    uint32_t leaves;         /* leaves M of the two-level model, 4..256 (default 256) */
    uint32_t train_iters;    /* gradient steps of the two-level model (default 4; each a Newton step) */
    uint32_t tile_keys;      /* keys per distribution tile: 4096 (0 = default) or 2048 */
    uint32_t sample_policy;  /* 0: the divisor rule above (Learned Sort's 1% sample, Background chapter);
                              * 1: IPLS's alpha*K - 1 with alpha = 0.2 log2(n), rounded to nearest,
                              *    at most ceil(n/2) (Proposed Algorithm chapter) */
    uint32_t equality;       /* 1: equality buckets (IPS4o's, applied to the linear model): a value whose
                              * run in the sorted sample is longer than S/K gets a bucket of its own (at
                              * most min(16, (K-4)/2) of them); the linear part is fitted on the sample
                              * without those runs with K - 2E buckets.  0 (default): the paper's IPLS */
    uint32_t inherit;        /* 1: sample inheritance (needs model 0 and equality 0).  A child bucket that is
                              * partitioned itself (more than T keys) reuses the parent's sorted sample
                              * restricted to it (the keys the parent's line sends there, still sorted)
                              * when that holds at least max(3, sample_min or 2K) keys and FMCD on it is
                              * usable; every other bucket draws a fresh sample.  The child's line is
                              * fitted before the parent's scatter, which also writes each key's class
                              * under it (one byte a key, in a library buffer of n bytes), so the child's
                              * counting pass reads one byte a key instead of the key.  Within the paper's
                              * sample -> sort -> train -> predict pipeline (Machine Learning Models
                              * chapter); the paper itself samples every bucket afresh.  0 (default) */
    uint32_t bucket_policy;  /* 1 (default): with the plain FMCD line (model 0, equality 0, inherit 0) a
                              * bucket of n keys is partitioned into the smallest power of two k >= 8n/T
                              * buckets, kept within [min(K, 64), K], and its sample's 2K minimum uses
                              * that k: IPS4o, whose bucket count IPLS keeps (Proposed Algorithm), gives
                              * subproblems near the base case fewer buckets.  0: K buckets everywhere.
                              * ipls_partition always uses K. */
} ipls_params;

/* FMCD linear model of a sample: bucket(x) = clamp(floor(fma(a, x, b)), 0, K-1). */
typedef struct {
    double a, b;         /* slope and offset */
    uint64_t D;          /* conflict degree the fit stopped at */
    uint32_t K;          /* buckets */
    uint32_t degenerate; /* 1 when the fit is unusable (S < 3, non-finite ends, a <= 0 or inf) */
} ipls_linear_model;

/* Statistics of the last sort (host struct, filled after the sort has completed). */
typedef struct {
    uint32_t levels;            /* distribution levels run (0 when every bucket went to the base case) */
    uint32_t sample_depth;      /* deepest nesting of sample sorts that needed a partition */
    uint64_t passes;            /* buckets partitioned, over all levels */
    uint64_t closed;            /* buckets closed by the homogeneity check */
    uint64_t fallback;          /* buckets split by the most-significant-digit fallback */
    uint64_t l2pl_used;         /* buckets partitioned with the two-level model */
    uint64_t base_buckets;      /* base-case sorts */
    uint64_t level1_max_load;   /* largest bucket after the first level */
    uint64_t keys_partitioned;  /* sum over levels of keys that went through a distribution pass */
    uint64_t inherited;         /* partitions whose line came from an inherited sample */
} ipls_stats;

/* Defaults: K 256, T 4096, divisor 100, sample_min 2K, no cap, FMCD, M 256, 4 steps, tile 4096, policy 0,
 * no equality buckets, no inheritance. */
void ipls_default_params(ipls_params* p);

/* Sort keys[0..n) (and payload[0..n) when non-null, stably) in place with default parameters.
 * keys: device array of n elements of `dtype`; payload: device uint32 array or NULL. */
ipls_status ipls_sort(void* keys, uint32_t* payload, size_t n, ipls_dtype dtype, void* stream);

/* ipls_sort with explicit parameters (NULL = defaults), an optional caller-owned device
 * workspace for the ping-pong copy of keys and payload (NULL = library cache; else at least
 * ipls_workspace_bytes() bytes, 256-byte aligned), and optional statistics (host pointer). */
ipls_status ipls_sort_ex(void* keys, uint32_t* payload, size_t n, ipls_dtype dtype, const ipls_params* p,
                         void* workspace, size_t workspace_bytes, ipls_stats* stats, void* stream);

/* Allocation-free variant of ipls_sort_ex, for callers that cannot allocate device memory (code
 * that must not call hipMalloc, serving loops that forbid allocation).  Same arguments, result and
 * statistics as ipls_sort_ex with no workspace; the ping-pong copy of keys and payload and every
 * per-level table are carved from a static device array of IPLS_NOALLOC_SCRATCH_BYTES that each
 * GPU the library runs on holds until the process ends.  The call allocates nothing: no device
 * or pinned memory, no stream or event; it runs entirely on `stream` and returns after the sort
 * has completed.  n above IPLS_NOALLOC_MAX_KEYS returns IPLS_ERR_UNSUPPORTED before any work;
 * IPLS_ERR_OOM means the parameters' tables did not fit the array.  Every call on one GPU uses
 * the same array and leaves its last contents there (each call clears what must start at zero).
 * Two calls on one GPU would race on it if they overlapped; the library prevents that: calls
 * from several host threads are serialised, and every call, also a failing one, returns only
 * after its stream has drained. */
#define IPLS_NOALLOC_MAX_KEYS (1ull << 22)
#define IPLS_NOALLOC_SCRATCH_BYTES (128ull << 20)
ipls_status ipls_sort_noalloc(void* keys, uint32_t* payload, size_t n, ipls_dtype dtype, const ipls_params* p,
                              ipls_stats* stats, void* stream);

/* Sort nseg independent segments [seg_offsets[s], seg_offsets[s+1]) of one array, each exactly as
 * ipls_sort would sort it alone (sample offsets are relative to the segment's start).
 * seg_offsets: device array of nseg+1 non-decreasing uint64; keys span seg_offsets[nseg] elements.
 * Decreasing offsets are reported as IPLS_ERR_DEVICE after the device has checked them. */
ipls_status ipls_sort_segmented(void* keys, uint32_t* payload, const uint64_t* seg_offsets, size_t nseg,
                                ipls_dtype dtype, const ipls_params* p, ipls_stats* stats, void* stream);

/* FMCD fit (Linear Models section) of a sample of S keys for K buckets, in fp64.  When
 * sample_is_sorted is 0 the library sorts a copy first (the caller's sample is not modified).
 * out: device pointer to one ipls_linear_model. */
ipls_status ipls_fit_model(const void* sample, size_t S, ipls_dtype dtype, int sample_is_sorted, uint32_t K,
                           ipls_linear_model* out, void* stream);

/* One distribution pass over the whole array (the first level of ipls_sort_ex): sample, fit,
 * classify, stable scatter.  keys (and payload) are left partitioned into contiguous buckets in
 * bucket order; counts (device, K uint64) receives the bucket sizes; model (device, nullable)
 * receives the linear model the pass used: the FMCD line (with equality buckets, its linear
 * part; with a two-level model, its root), or degenerate = 1 when the pass used none (the digit
 * fallback, a closed bucket, or the splitter tree).  A bucket whose fit is degenerate is split by
 * the digit fallback or, when all its keys are equal, left as it is (counts then all zero). */
ipls_status ipls_partition(void* keys, uint32_t* payload, size_t n, ipls_dtype dtype, const ipls_params* p,
                           uint64_t* counts, ipls_linear_model* model, void* stream);

/* Two-level piecewise-linear CDF model trained on a sorted fp64 sample x[0..S) for K buckets and
 * M leaves with `iters` gradient steps (Recursive Model Index section; training by MSE on K times
 * the eCDF, Machine Learning Models chapter).  Device outputs: root (2 doubles: the FMCD root's
 * a, b), leaf (4*M doubles: A, B, LO, HI per leaf), ab (2*M doubles: trained alpha, beta in each
 * leaf's centred coordinate, nullable).  Returns IPLS_ERR_DEVICE if the root fit is degenerate. */
ipls_status ipls_l2pl_train(const double* x, size_t S, uint32_t K, uint32_t M, uint32_t iters, double* root,
                            double* leaf, double* ab, void* stream);

/* Forward and backward pass of the two-level model's per-leaf MSE at given leaf parameters
 * ab (device, 2*M) on the sorted fp64 sample x[0..S): grad (device, 2*M) receives
 * (dL/dalpha, dL/dbeta) per leaf, loss (device, M, nullable) the per-leaf loss. */
ipls_status ipls_l2pl_grad(const double* x, size_t S, uint32_t K, uint32_t M, const double* ab, double* grad,
                           double* loss, void* stream);

/* Bytes of caller workspace ipls_sort_ex accepts for n keys: n * (key bytes + 4 if payload). */
size_t ipls_workspace_bytes(size_t n, ipls_dtype dtype, int has_payload, const ipls_params* p);

/* Status of the last sort call issued on `stream` (IPLS_OK if none). */
ipls_status ipls_stream_status(void* stream);

/* Static string naming a status code. */
const char* ipls_status_string(ipls_status st);

/* Kernel timing for measurement.  mask: bit k enables kernel id k, 0 (scatter), 1 (classify +
 * histogram), 2 (base case); 7 = all, 0 = off.  While enabled, the library records HIP events
 * around every launch of the enabled kernels on the stream it is launched on and accumulates
 * their elapsed times (each event record costs a few microseconds of host time, so time a run with
 * only the kernels it reports); ipls_profile_read returns, for a kernel id, the number of launches,
 * the summed milliseconds and the summed algorithmic bytes (keys and payload each kernel must read
 * and write).  Enabling resets the counters. */
void ipls_profile_enable(int mask);
void ipls_profile_read(int kernel, uint64_t* launches, double* ms, double* bytes);
/* The same figures for the launches of one recursion level (0 .. IPLS_PROFILE_LEVELS - 1; deeper
 * levels count in the last).  The counting and scatter launches of level L partition the buckets
 * that level L - 1 made (level 0: the input); a base-case launch counts in the level whose pass
 * made its buckets (level 0 for arrays or segments that needed no pass).  Levels out of range
 * leave the outputs unchanged. */
#define IPLS_PROFILE_LEVELS 16
void ipls_profile_read_level(int kernel, int level, uint64_t* launches, double* ms, double* bytes);

/* ---------------------------------------------------------------- batched form: autotuner
 * Picks num_buckets (K), base_case_max (T) and tile_keys for the segmented sort of a batch shaped
 * like the given one.  It times ipls_sort_segmented on a window of the batch's leading segments
 * (at least 2^25 keys, or all of them), copied to a private buffer so the caller's keys are not
 * modified, and walks the candidates one parameter at a time: tile_keys in {4096, 2048}, then T in
 * {4096, 2048, 1024}, then K in {256, 128, 64}, keeping each best.  The result is a sort of the
 * same keys (the output of a sort does not depend on these parameters); only its speed changes.
 * keys, seg_offsets: device (as ipls_sort_segmented); base: the other parameters (NULL =
 * defaults); out: host, receives the chosen parameters; report: host, nullable.  Synchronous. */
typedef struct {
    uint32_t trials;       /* configurations timed */
    uint32_t window_segments;
    uint64_t window_keys;
    double default_ms;     /* window sort time with the base parameters */
    double best_ms;        /* window sort time with the chosen parameters */
} ipls_tune_report;

ipls_status ipls_autotune_segmented(const void* keys, const uint64_t* seg_offsets, size_t nseg, ipls_dtype dtype,
                                    int has_payload, const ipls_params* base, ipls_params* out,
                                    ipls_tune_report* report, void* stream);

/* ---------------------------------------------------------------- served form: request server
 * Continuous batching of sort requests of mixed sizes and dtypes on one GPU.
 *   Memory: the caller gives the server one device arena (the HBM budget, 256-byte aligned,
 *   caller-owned, outlives the server).  ipls_server_reserve admits a request when its memory fits
 *   now and never blocks: a request of more than batch_max_keys keys gets its own slot (keys,
 *   payload) plus its sort workspace; a smaller one gets a slot at the end of the open batch
 *   buffer of its class (dtype, payload or not), so the slots of a batch are contiguous and the
 *   batch is sorted in place by one segmented sort.  IPLS_ERR_OOM means "not now": retry after a
 *   release.  Engine metadata (per-level tables, about 1.5 bytes per key of the largest request a
 *   lane has run) is allocated outside the arena.
 *   Flow: reserve -> caller writes the input into the slot (any stream) -> submit(stream) -> the
 *   server's sort waits for that stream's work with an event -> wait/poll -> caller reads the
 *   sorted slot -> release.
 *   Execution: `lanes` threads, each with its own stream and engine context, take submitted work
 *   in order: a large request, or the slots of a batch submitted so far (taking a batch closes it
 *   to new requests; its slots still only reserved are sorted once submitted, so a caller may wait
 *   on one request before submitting the others).  Lanes overlap on the device.  A request's result is bit-identical to ipls_sort_ex of its keys alone with the same
 *   parameters.  Timestamps are CLOCK_MONOTONIC seconds. */
typedef struct ipls_server ipls_server;

typedef struct {
    uint32_t lanes;              /* concurrent lanes, 1..16 (default 3) */
    uint32_t batch_max_requests; /* requests per batch (default 1024) */
    uint64_t batch_max_keys;     /* requests of at most this many keys are batched (default 2^18) */
    uint64_t batch_keys;         /* key capacity of one batch buffer, >= batch_max_keys (default 2^22) */
    ipls_params params;          /* sort parameters of every request */
} ipls_server_config;

typedef struct {
    uint64_t req_id;
    uint64_t n;
    ipls_status status;
    uint32_t batch_size;         /* requests sorted together with it (1 for a large request) */
    double t_reserve, t_submit, t_start, t_done;
} ipls_server_done;

typedef struct {
    uint64_t admitted, completed, rejected; /* rejected: reserve calls answered IPLS_ERR_OOM */
    uint64_t singles_run, batches_run, keys_sorted;
    uint64_t arena_bytes, bytes_in_use, peak_bytes_in_use;
    uint64_t queue_depth, max_queue_depth;
} ipls_server_stats;

void ipls_server_default_config(ipls_server_config* cfg);
ipls_status ipls_server_create(void* arena, size_t arena_bytes, const ipls_server_config* cfg, ipls_server** out);
/* keys, payload (host out-params) receive the slot's device pointers; payload may be NULL when
 * has_payload is 0. */
ipls_status ipls_server_reserve(ipls_server* srv, size_t n, ipls_dtype dtype, int has_payload, uint64_t* req_id,
                                void** keys, uint32_t** payload);
ipls_status ipls_server_submit(ipls_server* srv, uint64_t req_id, void* producer_stream);
/* Blocks until the request is done; returns its status; info (host, nullable) its timestamps. */
ipls_status ipls_server_wait(ipls_server* srv, uint64_t req_id, ipls_server_done* info);
/* Up to max completions not yet reported, in completion order. */
ipls_status ipls_server_poll(ipls_server* srv, ipls_server_done* out, size_t max, size_t* count);
/* Frees a done request's memory; its slot must not be used afterwards. */
ipls_status ipls_server_release(ipls_server* srv, uint64_t req_id);
ipls_status ipls_server_stats_get(ipls_server* srv, ipls_server_stats* out);
/* Finishes submitted work (requests reserved but never submitted are dropped), stops the lanes
 * and frees the server (not the arena). */
ipls_status ipls_server_destroy(ipls_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* IPLS_H */
