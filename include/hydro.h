/*
 * hydro.h -- C ABI of the MI355X (gfx950) engine for conjunctive ML-UDF queries.
 *
 * The engine evaluates  SELECT id FROM frames WHERE P_0(frame) AND ... AND P_{K-1}(frame)
 * where every P_k is a classifier (an MLP or a small CNN) followed by a class-subset
 * threshold test, and routes tuples through the predicates adaptively, batch by batch,
 * in the order that running cost and selectivity statistics favour.
 *
 * Paper: Hydro, "Adaptive Query Processing of ML Queries" (arXiv 2403.14902).
 *   - The conjunction and its answer: section 1 (motivating query) and section 4.1 (UC1 query).
 *   - Eddy routing, visited-predicate metadata, completion: section 3.2 ("Data Flow and
 *     Routing") and section 3.3 ("Metadata for Data Routing").
 *   - Eager dropping of failing tuples: section 3.3 ("Eager Materialization").
 *   - Routing batches: section 3.3 ("Batch Evaluation").
 *   - Policies: section 4.1 ("Cost-Driven Routing Policy": score = cost / (1 - selectivity),
 *     lowest first; "System Variants": no reordering, cost-, score- and selectivity-driven;
 *     selectivity from counts of filtered rows).
 *   - Warmup: section 4.1 ("Warmup Phase").
 *   - Content-based routing (the idea behind the learned router): section 2.2.
 *
 * Conventions
 *   - Every function returns an int status (hydro_status); nothing is thrown across the ABI.
 *     On error, output pointers are set to NULL / 0 and caller-owned outputs are left untouched;
 *     hydro_last_error() returns a thread-local message describing the last failure.
 *   - Pointers are borrowed for the duration of a call unless stated otherwise.
 *   - Device pointers are HIP device addresses on the current device; "host" pointers are
 *     ordinary process memory (pinned memory is copied asynchronously, pageable memory is
 *     staged through a pinned buffer).
 *   - Frames are NHWC with 3 channels, row-major, tightly packed.
 *   - Result ids are unique and sorted ascending (the query's answer is a set).
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYDRO_MAX_PREDICATES 8
#define HYDRO_MAX_LAYERS 4
#define HYDRO_N_CLASSES 10

typedef enum {
  HYDRO_OK = 0,
  HYDRO_EINVAL = -1,        /* bad argument (NULL pointer, size, shape mismatch, bad order)      */
  HYDRO_ENOMEM = -2,        /* device or pinned-host allocation failed                           */
  HYDRO_EDEVICE = -3,       /* a HIP call failed; the message carries HIP's error string         */
  HYDRO_EUNSUPPORTED = -4,  /* valid but not supported (K > 8, channels != 3, model shape, ...)  */
  HYDRO_ECAPACITY = -5,     /* more tuples than the session was created for                      */
  HYDRO_ESTATE = -6         /* call out of order (push after finish, finish without push, ...)   */
} hydro_status;

typedef enum { HYDRO_DTYPE_F32 = 0, HYDRO_DTYPE_BF16 = 1, HYDRO_DTYPE_U8 = 2 } hydro_dtype;
typedef enum { HYDRO_MEM_DEVICE = 0, HYDRO_MEM_HOST = 1 } hydro_mem;

/* A block of tuples.  Tuple i of the block has global id id_base + i.
 * data: n * h * w * 3 elements of dtype (F32: float; BF16: bfloat16 bit patterns; U8: uint8,
 * whose value is v / 255).  Ownership stays with the caller.  For where == HOST the caller keeps
 * the memory valid until hydro_session_finish returns. */
typedef struct {
  const void* data;
  int32_t dtype;
  int32_t where;
  int64_t n;
  int32_t h, w;
  int64_t id_base;
  const void* host_data;   /* optional, with where == DEVICE: the same frames in host memory, read by
                              HOST predicates (NULL: none); borrowed until hydro_session_finish     */
  const int32_t* crops;    /* optional, host memory [n][4]: tuple i's crop (y0, x0, h, w) of its frame,
                              the input of predicates with on_crop = 1 (NULL: none); copied         */
} hydro_frames;

typedef enum { HYDRO_ARCH_MLP = 0, HYDRO_ARCH_CNN = 1, HYDRO_ARCH_HOST = 2 } hydro_arch;

/* One predicate: a classifier with 10 logits z and a class subset S (class_mask bit c <=> c in S).
 * Its margin is d = max_{c in S} z_c - max_{c not in S} z_c and it holds iff d > theta (strict),
 * theta taken from the threshold table for the tuple's segment.  Every model first normalises
 * its input: x' = (x - 0.5) * 4, with x in [0,1] (u8: x = v / 255).
 *
 * MLP (arch = MLP): x' flattened in NHWC order (d_in = in_h * in_w * 3);
 *   h = ReLU(x' W1 + b1), z = h W2 + b2.  w1: [d_in][hidden], b1: [hidden], w2: [hidden][10],
 *   b2: [10], all fp32, row-major.
 * CNN (arch = CNN): n_layers conv3x3 layers, stride 2, zero padding 1 (in normalised space),
 *   each followed by ReLU; then the mean over all final positions; then z = g Wfc + bfc.
 *   conv_w[l]: [widths[l]][c_in][3][3] (c_in = 3 for l = 0, else widths[l-1]), conv_b[l]:
 *   [widths[l]]; fc_w: [widths[n_layers-1]][10], fc_b: [10]; all fp32, row-major.
 * HOST (arch = HOST): a cheap heuristic evaluated by the library's CPU threads concurrently with
 *   the GPU predicates (section 4.1: a colour classifier on the CPU beside a deep model on the
 *   GPU): d = the fraction of the frame's sampled pixels (rows and columns 0, s, 2s, ... with
 *   s = color_stride) whose three values x_c (in [0,1], as above) all lie in
 *   [color_lo[c], color_hi[c]]; it holds iff d > theta.  A session with a HOST predicate
 *   takes frames in host memory, or device frames with their host copy in host_data
 *   (EUNSUPPORTED otherwise); every round its queue is
 *   copied to the host, evaluated on up to HYDRO_HOST_THREADS (default: all) threads while the GPU
 *   evaluates the other queues, and the decisions are copied back and forwarded; its cost is the
 *   measured time per tuple of the thread pool, scaled to the GPU's scale of cost (device time
 *   per tuple summed over its compute units) by the ratio of compute units to threads, so that
 *   either resource's figure reads as that resource's wall time per tuple times the same
 *   constant (STATIC cost source: 6 operations per sampled pixel).  No weights,
 *   class_mask unused; not with route = LEARNED; pushes are not captured in graphs.
 * CNN with on_crop = 1: the same layers on the crop (y0, x0, h, w) of the tuple's frame, zero
 *   padding at the crop's border (the crop is the image), the mean over the crop's final positions,
 *   FC; any crop size from 1 x 1 to the frame (widths at most 256).  Evaluated in FP64 on the GPU
 *   (its decisions are final), one workgroup per tuple; work per tuple follows the crop's area, so
 *   policy.balance chooses how the tuples of a round are dealt to the workgroups.
 * Weights are copied (and re-packed per precision) when a session is created. */
typedef struct {
  int32_t arch;
  int32_t in_h, in_w;
  int32_t hidden;
  const float *w1, *b1, *w2, *b2;
  int32_t n_layers;
  int32_t widths[HYDRO_MAX_LAYERS];
  const float* conv_w[HYDRO_MAX_LAYERS];
  const float* conv_b[HYDRO_MAX_LAYERS];
  const float *fc_w, *fc_b;
  uint32_t class_mask;
  float color_lo[3], color_hi[3];   /* HOST: the channel box */
  int32_t color_stride;             /* HOST: pixels sampled every stride-th row and column
                                       (0 or 1: every pixel)                                     */
  int32_t on_crop;                  /* CNN: 1 = the input is the tuple's crop (hydro_frames.crops),
                                       a variable-size image (section 5.3: UDF composition such as
                                       a classifier on Crop(frame, bbox)); see below             */
} hydro_model;

typedef enum {
  HYDRO_ROUTE_FIXED = 0,    /* the written order in policy.order (no reordering)                 */
  HYDRO_ROUTE_SEL = 1,      /* lowest estimated selectivity first                                */
  HYDRO_ROUTE_SCORE = 2,    /* lowest cost / (1 - selectivity) first                             */
  HYDRO_ROUTE_COST = 3,     /* lowest estimated cost first                                       */
  HYDRO_ROUTE_LEARNED = 4   /* per-tuple keys from an online-trained router MLP, judged against
                               SCORE and falling back to it                                       */
} hydro_route;

/* First-pass arithmetic.  FP32: fp32 operands.  BF16: bf16 operands, fp32 accumulation; margins
 * within tau of the threshold are re-scored in FP32.  FP8: OCP e4m3 operands with per-output-channel
 * weight scales and per-layer activation scales, fp32 accumulation (4-layer 128x128 CNN predicates
 * conv 32-64-128-256 only; layer 1 runs bf16, exact for raw frame values); margins within tau are
 * re-scored in BF16, BF16 margins within tau16 in FP32 (BF16 with policy.rescore3 likewise: first-pass
 * margins within tau to a three-product tier, its margins within tau16 to FP32).  Every chain ends
 * with FP32 margins within
 * tau32 re-scored in FP64, which decides.  The answer never depends on the precision. */
typedef enum { HYDRO_PREC_FP32 = 0, HYDRO_PREC_BF16 = 1, HYDRO_PREC_FP8 = 2 } hydro_precision;
typedef enum { HYDRO_COST_MEASURED = 0, HYDRO_COST_STATIC = 1 } hydro_cost_source;

/* Execution policy.  Fill with hydro_policy_default() and override fields. */
typedef struct {
  int32_t route;                         /* hydro_route                                          */
  int32_t order[HYDRO_MAX_PREDICATES];   /* FIXED: a permutation of 0..K-1                       */
  int32_t routing_batch;                 /* tuples per routing batch (default 64)                */
  int32_t wave;                          /* tuples admitted per round (default 8192)             */
  int32_t warmup_batches;                /* routing batches per predicate in the warmup round
                                            (default 1; adaptive policies only)                  */
  float ewma_alpha;                      /* weight of the newest round in the running
                                            selectivity / cost estimates (default 0.5)           */
  int32_t cost_source;                   /* MEASURED: device time per evaluated tuple;
                                            STATIC: the model's FLOPs (deterministic routes)     */
  int32_t precision;                     /* first-pass arithmetic; see tau                       */
  float tau;                             /* BF16 first pass: |d - theta| < tau is re-scored in
                                            FP32.  <= 0 (default): automatic, see below          */
  float tau32;                           /* FP32 pass: |d - theta| < tau32 is re-scored in FP64.
                                            <= 0 (default): automatic.  Automatic bands are
                                            measured on the session's first push (up to 1,024 of
                                            its frames, as hydro_session_calibrate with safety 3)
                                            and never set below 0.015 / 1e-5                     */
  int32_t grouped;                       /* 1: one persistent launch per round and tier for all
                                            predicates (default 1)                               */
  int32_t use_graph;                     /* 1: replay the round sequence from a HIP graph        */
  int32_t log_routes;                    /* 1: record every tuple's visit sequence (debug)       */
  int32_t time_kernels;                  /* 1: bracket each round's phases with HIP events and
                                            report their summed durations in hydro_query_info    */
  int32_t autotune;                      /* 1: time each candidate GEMM tile shape on every MLP
                                            predicate at setup (first push) and keep the fastest;
                                            results cached in the JSON file named by
                                            HYDRO_TUNE_CACHE when that is set (default 0)        */
  float explore;                         /* LEARNED: fraction of routing batches kept on SCORE
                                            as the judge's control arm (default 0.05)            */
  uint64_t seed;                         /* LEARNED: router init / exploration seed              */
  void* stream;                          /* hipStream_t to run on; NULL: the session's own       */
  float tau16;                           /* FP8 first pass: |d - theta| < tau16 of the BF16
                                            re-score goes on to FP32 (rescore3: of the three-
                                            product re-score).  <= 0 (default): automatic        */
  int32_t reuse;                         /* UDF result reuse (section 4.3, "Reuse-aware Routing"):
                                            0 (default): none.  1: the session keeps a device
                                            cache per predicate of every decision it takes (tuple
                                            id -> pass/fail and the threshold it was decided
                                            against), kept across its queries; a tuple reaching
                                            a predicate whose cached decision still decides at the
                                            tuple's threshold takes it from the cache instead of
                                            being evaluated.  2: as 1, and routing is reuse-aware:
                                            within every batch of 64 routed tuples the ranking
                                            uses (1 - cache hit rate of the batch) x cost in place
                                            of the cost (SCORE and COST; SEL and FIXED only use
                                            the cache).  Not with LEARNED                          */
  int32_t cache_log2;                    /* reuse > 0: log2 of the cache slots per predicate
                                            (16 B each; 0: default 22, at most 28); a decision is
                                            not cached when its 16 probe slots are taken          */
  int32_t balance;                       /* on_crop predicates (section 5.3, "Data-Aware Load
                                            Balancing"): 0 (default) = each round's tuples dealt
                                            to the workgroups in queue order, round robin;
                                            1 = data-aware: ordered by estimated work (the crop's
                                            area, the input-size heuristic), largest first, each
                                            workgroup taking the next from a shared counter      */
  int32_t rescore3;                      /* BF16 first pass, every predicate a 4-layer 128x128
                                            CNN (32-64-128-256): 1 = first-pass margins within tau
                                            go to a re-score tier of three bf16 products per
                                            product (hi x hi + hi x mid + mid x hi of the operands
                                            split into bf16 terms, fp32 sums: about 2^-16
                                            relative), its margins within tau16 on to FP32.  tau16
                                            <= 0: automatic, floor 3e-4.  0 (default): none      */
} hydro_policy;

/* Per-predicate statistics of one query. */
typedef struct {
  uint64_t evaluated;          /* tuples this predicate was evaluated on                        */
  uint64_t passed;             /* of those, tuples that passed                                  */
  uint64_t rescored;           /* first-pass decisions deferred to the FP32 pass                */
  uint64_t escalated;          /* FP32 decisions deferred to the FP64 pass                      */
  double device_us;            /* summed device time of this predicate's first-pass tiles       */
  double cost_us_per_tuple;    /* final running cost estimate                                   */
  double selectivity;          /* passed / evaluated: conditional on the tuples it saw          */
  uint64_t rescored16;         /* FP8 first pass: BF16 decisions deferred to the FP32 pass;
                                  rescore3: three-product decisions deferred to the FP32 pass    */
  uint64_t cache_hits;         /* policy.reuse: decisions taken from the result cache (not
                                  counted in evaluated / passed)                                */
} hydro_pred_stats;

/* Whole-query counters. */
typedef struct {
  uint64_t n_tuples, n_result;
  uint32_t rounds, k;
  uint64_t learned_routed, stats_routed;   /* LEARNED: tuples routed by each arm                 */
  uint32_t learned_active;                 /* LEARNED: 1 if the judge kept the learned router    */
  uint32_t train_steps;                    /* LEARNED: optimiser steps taken                      */
  double elapsed_us;                       /* host time from first push to results on the host  */
  /* policy.time_kernels = 1: summed device durations (HIP events on the session's stream) */
  double route_ms;                         /* fold + router + learned-router work                */
  double first_pass_ms;                    /* first-pass inference launches (one per round)      */
  double f32_pass_ms;                      /* FP32 re-score launches                              */
  double f64_pass_ms;                      /* FP64 escalation launches                            */
  uint32_t timed_rounds;                   /* rounds bracketed                                    */
  uint32_t pad_;
  uint64_t learned_stale;                  /* LEARNED: learned-arm decisions whose keys had not
                                              been computed in the deciding round (routed by the
                                              statistics ranking instead; 0 in a correct run)    */
  double mid_pass_ms;                      /* policy.time_kernels, FP8 first pass: BF16 re-score */
  double arm_flops[2];                     /* LEARNED: UDF FLOPs spent on the routing batches of
                                              each arm (0: control arm, score routing; 1: learned
                                              arm) since the learned arm began routing            */
  double arm_tuples[2];                    /* ... and the tuples each arm finished (dropped or
                                              completed) over the same span                      */
} hydro_query_info;

/* One routing round of the last query (policy.log_routes = 1), for checking the router against
 * the policy definitions of section 4.1 ("Cost-Driven Routing Policy", "System Variants"): the
 * per-predicate counts of the previous round that were folded into the running estimates at the
 * start of this round, the estimates after the fold, and the ranking this round's router used. */
typedef struct {
  int32_t order[HYDRO_MAX_PREDICATES];              /* order[0] is the preferred predicate       */
  uint64_t folded_evaluated[HYDRO_MAX_PREDICATES];  /* previous round's first-pass evaluations   */
  uint64_t folded_passed[HYDRO_MAX_PREDICATES];     /* ... and passes                             */
  double selectivity[HYDRO_MAX_PREDICATES];         /* running estimates after the fold: EWMA of
                                                       (passed + 1) / (evaluated + 2)             */
  double cost[HYDRO_MAX_PREDICATES];                /* device ticks per evaluation, or the model's
                                                       FLOPs with cost_source = STATIC            */
  uint32_t seen_mask;                               /* bit k: predicate k had statistics when the
                                                       ranking was made (unseen ones go first)    */
  uint32_t pad_;
} hydro_round_record;

typedef struct hydro_session hydro_session;

/* Fill *p with defaults (SCORE, batch 64, wave 8192, BF16, grouped, no graph). */
void hydro_policy_default(hydro_policy* p);

/* One-shot query: create a session, push all frames, finish, destroy.
 * thresholds: fp32 [n_seg][K]; tuple id t uses row min(t / seg_len, n_seg - 1).
 * *out_ids: library-allocated int64[*out_n], sorted ascending; release with hydro_free.
 * out_stats: caller-allocated [K] (may be NULL). */
int hydro_query(const hydro_frames* frames, const hydro_model* models, int32_t k,
                const float* thresholds, int32_t n_seg, int64_t seg_len,
                const hydro_policy* policy, int64_t** out_ids, int64_t* out_n,
                hydro_pred_stats* out_stats);

/* Bytes of the device array that hydro_query_noalloc works in (one copy per GPU). */
#define HYDRO_NOALLOC_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory (serving loops and harnesses that forbid
 * hipMalloc, code that must not allocate between captured or timed regions): hydro_query without
 * any device allocation.  Every device buffer of the query (packed weights, queues, live lists,
 * statistics, result bitmap and ids, FP64-tier activations, learned-router state) is carved from
 * one library-owned device array of HYDRO_NOALLOC_BYTES bytes, one per GPU, held until the
 * process ends.  No stream, event or graph is created.  Differences from hydro_query:
 *   - frames must be in device memory (EUNSUPPORTED otherwise);
 *   - policy.use_graph, policy.autotune and policy.time_kernels must be 0 (EUNSUPPORTED);
 *   - the work runs on policy.stream, or on the null stream when that is NULL;
 *   - the ids are written to the caller's host array out_ids[out_cap], sorted ascending, and
 *     *out_n is their number; if the result has more than out_cap ids the call returns ECAPACITY
 *     with *out_n set to the number needed;
 *   - a query whose buffers do not fit the array returns ECAPACITY (the message names the size):
 *     e.g. two MLP 3072-256 predicates fit up to about 100k tuples, three 64x64 CNNs of the
 *     16-32-64 family up to about 1M; 4-layer 128x128 CNN predicates do not fit;
 *   - the FP64 tier evaluates at most 8 escalated tuples per predicate and round layer-parallel,
 *     the rest one per block on 16 blocks (same decisions, slower when many escalate).
 * Calls on one GPU share its array and keep nothing from the previous call (everything a call
 * reads is initialised by that call); calls that overlap on one GPU (several threads or streams)
 * race and must be serialised by the caller. */
int hydro_query_noalloc(const hydro_frames* frames, const hydro_model* models, int32_t k,
                        const float* thresholds, int32_t n_seg, int64_t seg_len,
                        const hydro_policy* policy, int64_t* out_ids, int64_t out_cap,
                        int64_t* out_n, hydro_pred_stats* out_stats);

/* Create a session: validates and uploads the K models (1 <= K <= 8), allocates device state
 * for pushes of at most max_push tuples of frame_h x frame_w x 3 frames.  The policy is copied.
 * Setup cost (weight upload and packing, buffer allocation) is paid here. */
int hydro_session_create(const hydro_model* models, int32_t k, const hydro_policy* policy,
                         int32_t frame_h, int32_t frame_w, int64_t max_push,
                         hydro_session** out);

/* Start a new query on an existing session: clears statistics, results and learned-router
 * state; keeps weights and buffers. */
int hydro_session_reset(hydro_session* s);

/* Evaluate one block of tuples: admit them in waves, route, evaluate and forward survivors
 * until every tuple of the block has completed or been dropped.  Enqueued on the policy's
 * stream; returns before the work finishes.  thresholds / n_seg / seg_len as in hydro_query
 * (copied).  Ids of different pushes must not overlap. */
int hydro_session_push(hydro_session* s, const hydro_frames* frames, const float* thresholds,
                       int32_t n_seg, int64_t seg_len);

/* Wait for all pushed work; return the sorted result ids (library-allocated, hydro_free) and
 * the statistics (out_stats: caller-allocated [K], may be NULL). */
int hydro_session_finish(hydro_session* s, int64_t** out_ids, int64_t* out_n,
                         hydro_pred_stats* out_stats);

/* Whole-query counters of the last finished query. */
int hydro_session_info(const hydro_session* s, hydro_query_info* out);

/* Debug: the visit sequence of the last finished query's tuples (policy.log_routes = 1).
 * out[i] describes tuple first_id + i: nibble j (bits 4j..4j+3) = 1 + the j-th predicate
 * evaluated, 0 after the last one.  n must not exceed the tuples of the last push. */
int hydro_session_routes(const hydro_session* s, int64_t first_id, int64_t n, uint32_t* out);

/* Debug: records first .. first + n - 1 of the last query's rounds (policy.log_routes = 1; at most
 * the first 16,384 rounds are recorded).  out: caller-allocated [n].  EINVAL outside the recorded
 * rounds, ESTATE without log_routes. */
int hydro_session_round_log(const hydro_session* s, int32_t first, int32_t n, hydro_round_record* out);

/* Evaluate predicate `pred`'s model on every given tuple at one arithmetic tier
 * (0 = the first-pass precision of the session, 1 = FP32, 2 = FP64, 3 = the BF16 re-score tier of
 * an FP8 session or the three-product tier of a rescore3 session; other sessions map 3 to their
 * first pass) and return its logits as
 * fp64 [n][10] in host memory.  Used for logit-error reports and kernel parity tests.  Runs between
 * queries only: ESTATE while a query is open (a push since the last reset or finish); it leaves
 * the session reset. */
int hydro_session_logits(hydro_session* s, int32_t pred, int32_t tier, const hydro_frames* frames,
                         double* out_logits);

/* Set every predicate's re-score bands from measurement: on the given device frames, each
 * predicate's first-pass, BF16 (FP8 sessions) and FP32 margins are compared with its FP64 margins;
 * tau_k, tau16_k and tau32_k become `safety` (>= 1) times the largest difference seen (floors 1e-4,
 * 1e-4 and 1e-6).  FP8 sessions first set each layer's activation scale so that the largest FP32
 * activation on these frames maps to 224 (half of e4m3's largest value).  Later pushes
 * use these bands instead of policy.tau / policy.tau32.  out_tau / out_tau32: caller-allocated
 * [K] (may be NULL).  Any number of frames (>= 1); more than the session's max_push are taken
 * in blocks of max_push.  This is the per-configuration band of the low-precision form: an
 * empirical bound, so the sample should be representative of the query's frames.  Runs between
 * queries only (ESTATE while a push is open); it leaves the session reset, and pushes captured in
 * HIP graphs under the old bands are discarded (they are re-captured with the new ones). */
int hydro_session_calibrate(hydro_session* s, const hydro_frames* frames, float safety, float* out_tau,
                            float* out_tau32);

/* The per-predicate bands the next push uses (policy values, automatic or calibrated): caller
 * arrays [K], each may be NULL.  tau: first pass; tau16: BF16 re-score of an FP8 first pass (the
 * three-product re-score of a rescore3 session);
 * tau32: FP32 pass. */
int hydro_session_bands(const hydro_session* s, float* tau, float* tau16, float* tau32);

/* Empty the session's result cache (policy.reuse > 0); the next queries start without cached
 * decisions.  ESTATE while a query is open or when the session keeps no cache. */
int hydro_session_cache_clear(hydro_session* s);

/* Debug: the learned router's current parameters (route = LEARNED), for evaluating its
 * predictions offline: W1 [192][64] | b1 [64] | W2 [64][8] | b2 [8] fp32 (12,872 values; output
 * j estimates the probability that predicate j rejects the tuple, as a logit; features: the frame
 * mean-pooled to 8x8x3 in (y, x, channel) order, normalised as the predicates normalise their
 * input, rounded to bf16).  out: caller array of n >= 12,872 floats.  ESTATE without a learned
 * router, EINVAL if n is too small. */
int hydro_session_router_params(const hydro_session* s, float* out, int32_t n);

/* Replace the written order that route = FIXED follows (section 4.1, "No Reordering": the
 * conjunction evaluated left to right) for the session's next queries.  order: a permutation of
 * 0..K-1.  EINVAL if it is not one; ESTATE while a query is open. */
int hydro_session_set_order(hydro_session* s, const int32_t* order);

/* Replace the routing policy (FIXED, SEL, SCORE or COST) of the session's next queries, so that
 * queries with different policies share one session and its result cache (section 4.3: earlier
 * exploratory queries fill the cache that a recurrent query reuses).  EINVAL for an unknown
 * route, EUNSUPPORTED for LEARNED or on a session created with it, ESTATE while a query is open. */
int hydro_session_set_route(hydro_session* s, int32_t route);

int hydro_session_destroy(hydro_session* s);

/* Debug: one launch of the learned router's online-training kernel (content-based routing,
 * section 2.2; the router MLP 192-64-8 predicts for each predicate the probability that it rejects
 * the tuple) on caller data in host memory, for checking its arithmetic.  n = 128 logged outcomes,
 * oldest first: feats [n][192] bf16 bit patterns, pred [n] (0 <= pred < k <= 8), rejected [n]
 * (1 = the predicate rejected the tuple).  The kernel takes two Adam steps (beta 0.9 / 0.999,
 * eps 1e-8, learning rate lr) of masked binary cross-entropy (only the output of the evaluated
 * predicate), first on samples 64..127, then on 0..63; steps_done is the number of steps already
 * taken (Adam's bias correction).  params: W1 [192][64] | b1 [64] | W2 [64][8] | b2 [8] fp32
 * (12,872 values), adam_m / adam_v the moments in the same layout; all three are updated in place.
 * Allocates and frees its own device memory; EINVAL on bad sizes, EDEVICE on a HIP failure. */
int hydro_router_train_debug(int32_t k, const uint16_t* feats, const int32_t* pred, const uint8_t* rejected,
                             int32_t n, float* params, float* adam_m, float* adam_v, int32_t steps_done, float lr);

/* Debug / measurement: the query path's routing, multi-split, forwarding and result
 * materialisation (sections 3.2 and 3.3: routing by the policy ranking, eager dropping of failing
 * tuples, the visited mask, completion) on n tuples whose predicate outcomes are given instead of
 * computed: tuple t passes predicate j iff bit t % 32 of word j * ceil(n / 32) + t / 32 of
 * pass_bits is set.  pass_bits: device memory, [k][ceil(n / 32)] uint32.  route: FIXED (order
 * 0..k-1), SEL, SCORE or COST, every predicate costing 1 (STATIC costs).  Tuples are admitted
 * `wave` at a time (64 <= wave <= 2^24) in pushes of at most 2^24.  out_ids: device memory of
 * n int64; receives the ids of the tuples that pass every predicate, ascending; *out_n their
 * number.  out_stats: caller-allocated [k] (may be NULL): evaluated and passed per predicate.
 * out_ms (may be NULL): [4] summed device milliseconds of fold + route, the decisions and
 * forwarding, result materialisation (bitmap clear, count, scan, write), and the whole run.
 * 1 <= k <= 8 (EUNSUPPORTED otherwise), 0 <= n <= 2^30 (EINVAL).  Allocates and frees its own
 * device buffers and stream; blocks until done. */
int hydro_compaction_debug(int32_t k, int64_t n, const uint32_t* pass_bits, int32_t route, int32_t wave,
                           int64_t* out_ids, int64_t* out_n, hydro_pred_stats* out_stats, double* out_ms);

/* Release memory returned by the library. */
void hydro_free(void* p);

/* Thread-local description of the last error on this thread ("" if none). */
const char* hydro_last_error(void);

/* Library version string. */
const char* hydro_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HYDRO_H */
