/*
 * pbh.h -- C ABI of the parallel bucket heap (parBucketHeap) and of
 * parDijkstra, for AMD Instinct MI355X (gfx950).
 *
 * The paper: Berney, Iacono, Karsin, Sitchinava, "A Parallel Priority Queue
 * with Fast Updates for GPU Architectures" (arXiv 1908.09378).
 *
 * Conventions shared by every entry point
 *   - Elements are (key: uint64, id: uint32) pairs: the paper's (priority,
 *     value) of Section 1.2.  Order is lexicographic on (key, id), so ties in
 *     priority are broken by id.  key == UINT64_MAX is reserved ("absent",
 *     "unreached") and is rejected as input.
 *   - Array arguments are DEVICE pointers (hipMalloc'd memory or a torch
 *     tensor's data_ptr() on the current GPU) unless the comment says "host".
 *     The caller owns every array; the library keeps no caller pointer after
 *     it returns.
 *   - Calls are synchronous: outputs are valid when the call returns.  Work
 *     is issued on the null stream (which orders it after earlier null-stream
 *     work, e.g. PyTorch's default stream) unless an _ex variant is given a
 *     stream.
 *   - Every call returns PBH_OK (0) or a negative error code and never aborts;
 *     pbh_last_error() gives a message for the calling thread's last failure.
 *     On PBH_EINVAL nothing was modified.
 *   - A handle must not be used by two threads at once.
 */
#ifndef PBH_H
#define PBH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PBH_OK = 0,
  PBH_EINVAL = -1,     /* bad argument: null pointer, id >= capacity, key == UINT64_MAX, bad CSR */
  PBH_ECAPACITY = -2,  /* the heap needed more levels than were allocated */
  PBH_ENOMEM = -3,     /* device allocation failed */
  PBH_EDEVICE = -4,    /* a HIP call failed */
  PBH_ETIMEOUT = -5,   /* a bounded device-side wait ran out */
  PBH_EINTERNAL = -6   /* a device-side consistency check failed (a bug) */
};

typedef struct pbh pbh_t; /* opaque; owned by the library */

/*
 * pbh_create: a parallel bucket heap over ids [0, id_capacity) with maximum
 * bulk size d (Section 2.2: bucket B_i holds d*2^(2i+1) elements and signal
 * buffer S_i holds d*2^(2i); q = ceil(log4(n/d)) + 1 levels).  Levels beyond
 * q are added on demand.  The handle owns its device arena: the levels, the
 * current key of every id (8 bytes x id_capacity) and scratch.
 * Errors: PBH_EINVAL if out is NULL, id_capacity == 0 or d == 0;
 * PBH_ENOMEM / PBH_EDEVICE.
 */
int pbh_create(pbh_t **out, uint32_t id_capacity, uint32_t d);

/*
 * pbh_create_ex: pbh_create with a choice of engine (same results, same
 * errors; opts may be NULL = automatic).
 *   engine 0 = automatic: the device-wide engine for d >= 16384, else the
 *              one-workgroup engine;
 *   engine 1 = one workgroup runs each operation and keeps the heap state on
 *              the device (suits small d: a few microseconds per operation);
 *   engine 2 = device-wide: every step of Resolve (merge with duplicate
 *              deletion, Select, the splits) is a grid-wide kernel and the
 *              host runs Resolve's control flow and the schedule, reading
 *              back a few sizes per step (suits large d: HBM-bound).
 *   schedule 0 = Theorem 1 (Resolve(i+1) after every fourth Resolve(i)),
 *   schedule 1 = on demand (Resolve(i+1) only when level i+1 needs it).
 * Errors: those of pbh_create, and PBH_EINVAL for engine > 2 or
 * schedule > 1.
 */
typedef struct pbh_opts {
  uint32_t engine;
  uint32_t schedule;
  uint32_t reserved[6]; /* must be zero */
} pbh_opts;
int pbh_create_ex(pbh_t **out, uint32_t id_capacity, uint32_t d, const pbh_opts *opts);

/*
 * pbh_bulk_update: BulkUpdate(U) of Section 1.2 -- update(e) for each of the
 * count pairs (keys[i], ids[i]) (device arrays): the element with that id gets
 * key min(current, keys[i]); an absent id is inserted.  Within a batch the
 * smallest key per id wins and order does not matter.  Batches larger than d
 * are applied in pieces of at most d (the paper's bound on |U|), with the same
 * result.  Errors: PBH_EINVAL (NULL handle, NULL arrays with count > 0, any
 * id >= id_capacity or key == UINT64_MAX; nothing is applied), PBH_ECAPACITY,
 * PBH_EDEVICE, PBH_ETIMEOUT (device-wide engine: a step's kernels ended
 * without publishing its results within a second), PBH_EINTERNAL.
 */
int pbh_bulk_update(pbh_t *h, const uint64_t *keys, const uint32_t *ids, uint64_t count);

/*
 * pbh_extract_min: batched ExtractMin (Section 1.2; Section 3.2 lets level 0
 * serve many extractions per Resolve(0)).  Removes the min(k, size) smallest
 * elements and writes them in ascending (key, id) order to keys_out[] and
 * ids_out[] (device arrays with room for k); *count_out (host) receives their
 * number.  Equal to k successive ExtractMins.  Errors: PBH_EINVAL (NULL handle
 * or count_out, NULL outputs with k > 0), PBH_EDEVICE, PBH_ETIMEOUT (as for
 * pbh_bulk_update), PBH_EINTERNAL.
 */
int pbh_extract_min(pbh_t *h, uint64_t k, uint64_t *keys_out, uint32_t *ids_out,
                    uint64_t *count_out);

/*
 * pbh_delete: Delete(e) of Section 1.2 for each of the count ids (device
 * array): the element with that id leaves the heap if the heap holds it;
 * absent ids and repeats are no-ops.  Section 2.1 sends a DEL priority down
 * the levels that removes matching elements when it meets them in a merge;
 * here the id's current key becomes "absent", which every merge and every
 * move into the top bucket treat the same way, and the top bucket is filtered
 * at once, followed by Resolve(0) and the schedule as after any operation.
 * Errors: PBH_EINVAL (NULL handle, NULL ids with count > 0, any id >=
 * id_capacity; nothing is applied), PBH_ECAPACITY, PBH_EDEVICE,
 * PBH_ETIMEOUT (as for pbh_bulk_update), PBH_EINTERNAL.
 */
int pbh_delete(pbh_t *h, const uint32_t *ids, uint64_t count);

/* pbh_size: number of elements in the heap (host *size_out). */
int pbh_size(pbh_t *h, uint64_t *size_out);

/*
 * pbh_traffic: heap elements (12 bytes each) read or written by the level
 * operations of Algorithm 1 (Merge, DeleteDuplicates, Select, the splits and
 * the copies into S_0) since the handle was created, counted as the engine
 * performs them (host *elements_out).  Used for the algorithmic-byte count
 * of a benchmark.
 */
int pbh_traffic(pbh_t *h, uint64_t *elements_out);

/*
 * pbh_merge_profile: for the device-wide engine, totals over the writing
 * passes of its merges (Merge + DeleteDuplicates, its largest kernel) run
 * while profiling was on: launches, algorithmic bytes (12 per input element
 * read + 12 per output element written) and summed HIP-event time in ms (host
 * outputs).  Zeros for the one-workgroup engine.
 */
int pbh_merge_profile(pbh_t *h, uint64_t *launches, uint64_t *bytes, double *ms);

/*
 * pbh_kernel_profile: for the device-wide engine, totals per kernel kind over
 * the launches made while profiling was on: launches, algorithmic bytes and
 * summed HIP-event time in ms (host outputs; zeros for the one-workgroup
 * engine).  kind < the number of kinds; pbh_kernel_name(kind) names it
 * (NULL past the last kind).  Algorithmic bytes per launch: merge writing
 * pass 12 per input + 12 per output element; merge counting pass 4 per input
 * (ids); Select pass and gather 12 per element (passes that return at once
 * are a kind of their own with 0 bytes); split counting 12 and writing 24 per
 * element; intake 20 per pair; mark compaction 1 per id (+ 20 per output in
 * the writing pass); extract sort 24 per element per pass; absent marking 12
 * per id.  Errors: PBH_EINVAL (NULL argument, kind out of range).
 */
int pbh_kernel_profile(pbh_t *h, uint32_t kind, uint64_t *launches, uint64_t *bytes, double *ms);
const char *pbh_kernel_name(uint32_t kind);

/*
 * pbh_set_profiling: on != 0 brackets every kernel launch of the device-wide
 * engine with HIP events (for pbh_kernel_profile and pbh_merge_profile); the
 * events add some microseconds to each launch, so profiling is off by
 * default.  No effect on results, nor on the one-workgroup engine.  Errors:
 * PBH_EINVAL (NULL handle).
 */
int pbh_set_profiling(pbh_t *h, int on);

/* pbh_destroy: frees the handle and its arena.  NULL is accepted. */
int pbh_destroy(pbh_t *h);

/*
 * Heap layout snapshot for invariant checks (Algorithm 1 pre/postconditions,
 * Theorem 1).  For each level i < *levels_out (host arrays of length
 * max_levels): sizes of B_i and S_i, the pivot p_i as (key, id) (UINT64_MAX
 * key = +infinity), and how many times Resolve(i) has run.  *ell_out receives
 * the deepest non-empty level (-1 when empty).
 */
int pbh_debug_levels(pbh_t *h, uint32_t max_levels, uint32_t *levels_out, int32_t *ell_out,
                     uint32_t *nB, uint32_t *nS, uint64_t *p_key, uint32_t *p_id,
                     uint64_t *resolves);

/*
 * sssp: single-source shortest paths by parDijkstra (Section 4.1): rounds of
 * ExtractMin of the closest vertex u, relaxation of all out-edges (u, v) in
 * parallel, and BulkUpdate of the ones that got shorter, on a parallel bucket
 * heap with d = maximum out-degree.  Graph in CSR form (device arrays):
 * offsets[n+1] (uint64; offsets[0] == 0, non-decreasing, offsets[n] == m),
 * targets[m] (uint32 < n), weights[m] (uint32, zero allowed).  Self-loops and
 * multi-edges are allowed.  dist_out[n] (device) receives the distances
 * (UINT64_MAX = unreachable).  Errors: PBH_EINVAL (NULL pointers, n == 0,
 * source >= n, malformed CSR), PBH_ENOMEM, PBH_EDEVICE, PBH_ECAPACITY,
 * PBH_ETIMEOUT, PBH_EINTERNAL.
 */
int sssp(const uint64_t *offsets, const uint32_t *targets, const uint32_t *weights, uint32_t n,
         uint64_t m, uint32_t source, uint64_t *dist_out);

/* Options for sssp_ex and sssp_batch.  Zero-initialised means "defaults". */
typedef struct {
  uint32_t d;             /* heap bulk size; 0 = maximum out-degree (the paper's choice) */
  uint32_t team;          /* threads of the workgroup that runs the rounds: 0 = auto, 64/256/1024 */
  uint32_t schedule;      /* 0 = Theorem 1 (Resolve(i) after every 4th Resolve(i-1)),
                             1 = on demand only (resolve a level when its buffers require it) */
  uint32_t lds_levels;    /* levels kept in LDS: 0 = as many as fit, k = exactly k,
                             0xFFFFFFFF = none (all levels in HBM) */
  uint64_t heap_capacity; /* elements the arena is sized for; 0 = auto (retried with the
                             safe bound m+1 on PBH_ECAPACITY) */
  /* How many minima each round extracts.  Rounds with k > 1 relax all out-edges
   * of the k vertices and re-insert any vertex whose distance later improves,
   * so distances stay exact for every rule. */
  uint32_t k_rule;        /* 0 = plain parDijkstra (k = 1, Section 4.1); 1 = k_fixed;
                             2 = learned: the MLP in k_model chooses k each round;
                             3 = k_seq[round % k_seq_len] */
  uint32_t k_fixed;
  uint32_t k_max;         /* cap on k (0 = 2d; never above 256); 1 makes every rule the plain one */
  uint32_t k_seq_len;
  const uint32_t *k_seq;  /* device array (rule 3) */
  const float *k_model;   /* device array of PBH_MLP_BLOB floats (rule 2): W1[8][64], b1[64],
                             W2[64][64], b2[64], w3[64], b3, mu[8], sd[8], scale
                             (weights input-major, already rounded to bfloat16); the
                             model maps 8 per-round features to y, k = 2^(scale*y) */
  /* Training traces: every trace_every-th round writes 8 features to
   * trace_features[8*i], the PBH_TRACE_K smallest (key, id) of B_0 in key order to
   * trace_keys[PBH_TRACE_K*i] / trace_ids[PBH_TRACE_K*i] (UINT64_MAX keys pad short lists) and the
   * query's index (0 for sssp_ex, the position in the queries array for
   * sssp_batch) to trace_query[i] (may be NULL), where i = atomicAdd(trace_count,
   * 1) while i < trace_cap.  All device arrays. */
  float *trace_features;
  uint64_t *trace_keys;
  uint32_t *trace_ids;
  uint32_t *trace_count;
  uint32_t *trace_query;
  uint32_t trace_every;
  uint32_t trace_cap;
  /* Trial limits (the autotuner's; distances are then incomplete): a round
   * does not start once the smallest key in the heap exceeds stop_key
   * (0 = no limit), nor after max_rounds rounds (0 = no limit). */
  uint64_t stop_key;
  uint32_t max_rounds;
  uint32_t d_scale;       /* with d == 0: d = maximum out-degree * max(1, d_scale) */
  float k_scale;          /* learned rule: k = 2^(k_scale * scale * y); 0 means 1 */
  uint32_t k_every;       /* learned rule: the model runs every k_every-th round and the
                             rounds between reuse its k (0 or 1 = every round) */
  /* Extraction record (may be NULL): settle_order[j] receives the id of the
   * j-th extracted vertex, for j < settle_cap (device array).  With the plain
   * rule this is parDijkstra's settle order; a round that extracts k > 1
   * writes its k ids in increasing id order.  sssp_ex and sssp_noalloc only
   * (sssp_batch ignores it). */
  uint32_t *settle_order;
  uint64_t settle_cap;
  /* Time accounting (sssp_ex only; 0 = off): the round loop reads the
   * device's constant-rate clock around every Resolve and between the steps
   * of each round, and sssp_stats.level_us / phase_us receive the totals.
   * Adds a little time to every round; no effect on results. */
  uint32_t profile;
  /* Large-heap form with deep-level workers (sssp_ex and sssp_noalloc;
   * Section 2.2.1, Theorem 1, Section 4.1's block per level).  0 = off: one
   * workgroup runs the rounds and resolves every level itself.  L > 0: every
   * level i >= max(L, 2, the LDS levels) gets a workgroup of its own that
   * runs Resolve(i) when the level above asks for it (after every fourth
   * Resolve of that level), while the rounds go on; levels two apart resolve
   * at the same time and adjacent ones never do.  The round loop and the
   * workers are one cooperative launch of 1 + (levels - first worker level)
   * workgroups; every wait between them is bounded (PBH_ETIMEOUT after 10 s
   * without progress).  This form also merges and selects on levels in HBM
   * through an LDS staging area (used whether or not a level gets a worker).
   * Same distances; rounds and relaxations as without it for the plain rule.
   * Needs schedule 0.  sssp_batch always uses the staging (no workers). */
  uint32_t deep_level;
} sssp_opts;

#define PBH_MLP_PARAMS (8 * 64 + 64 + 64 * 64 + 64 + 64 + 1)
#define PBH_TRACE_K 32 /* (key, id) pairs per trace record */
#define PBH_MLP_BLOB (PBH_MLP_PARAMS + 2 * 8 + 1)

/* Statistics of one sssp_ex run (host struct). */
typedef struct {
  uint64_t rounds;        /* rounds (one extraction each) */
  uint64_t relaxations;   /* edges scanned */
  uint64_t updates;       /* (key, id) pairs inserted into the heap */
  uint64_t heap_elems;    /* heap elements read + written by the level operations */
  uint64_t extracted;     /* elements extracted (= rounds for the plain rule) */
  uint64_t resolves[16];  /* Resolve(i) executions per level */
  uint32_t levels;        /* levels allocated */
  uint32_t d;             /* bulk size used */
  uint32_t team;          /* workgroup size used */
  uint32_t lds_levels;    /* levels resident in LDS */
  double kernel_ms;       /* device time of the round-loop kernel (HIP events) */
  uint64_t last_key;      /* smallest key left in the heap when the rounds stopped
                             (UINT64_MAX if the heap ran empty; largest over a batch) */
  /* With opts->profile (sssp_ex): microseconds inside Resolve(i) per level,
   * and per round step: [0] Resolve(0) + schedule + refills after each
   * operation (it includes the level times), [1] moving update pieces into
   * S_0, [2] features + MLP, [3] extraction from B_0, [4] relaxation,
   * [5] intake of the round's updates, [6] the rest, [7] waiting for a
   * deep-level worker (inside [0]).  With deep-level workers, level_us[i] of a
   * worker level is that worker's time inside Resolve(i), off the round
   * loop's path.  Zero otherwise. */
  double level_us[16];
  double phase_us[8];
} sssp_stats;

/*
 * sssp_ex: sssp with options, statistics (stats may be NULL) and a HIP stream
 * (hipStream_t passed as void*, NULL = null stream).  The call still returns
 * only when the result is in dist_out.
 */
int sssp_ex(const uint64_t *offsets, const uint32_t *targets, const uint32_t *weights, uint32_t n,
            uint64_t m, uint32_t source, uint64_t *dist_out, const sssp_opts *opts,
            sssp_stats *stats, void *stream);

/*
 * sssp_noalloc: sssp_ex for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and statistics as sssp_ex (except
 * stats->kernel_ms, which is 0: no events are created), but every buffer the
 * run needs beyond the caller's arrays -- the CSR check, the statistics block,
 * the heap levels that do not fit in LDS and the update lists of speculative
 * rounds -- is carved from one fixed 64 MiB array of device memory that the
 * library holds on each GPU it runs on until the process ends; nothing is
 * allocated or freed.  The array keeps the last call's contents (everything
 * a run reads is initialised by that run).  Calls are serialised inside the
 * library; calls that overlap on one GPU from outside it (e.g. through
 * another copy of the library) would race on the array.
 * Errors: those of sssp_ex, plus PBH_EINVAL (nothing run) when the query's
 * heap at its starting capacity needs more than the 64 MiB
 * (4096 + 12 x (HBM heap elements + list elements) bytes), and PBH_ECAPACITY
 * when the heap of a rule that pulls ahead outgrows it during the run.
 */
int sssp_noalloc(const uint64_t *offsets, const uint32_t *targets, const uint32_t *weights, uint32_t n,
                 uint64_t m, uint32_t source, uint64_t *dist_out, const sssp_opts *opts, sssp_stats *stats,
                 void *stream);

/* One query of sssp_batch: a CSR graph (device arrays, same rules as sssp),
 * a source and the distance output (device, n entries).  Queries may share
 * a graph. */
typedef struct {
  const uint64_t *offsets;
  const uint32_t *targets;
  const uint32_t *weights;
  uint64_t m;
  uint32_t n;
  uint32_t source;
  uint64_t *dist_out;
} sssp_query;

/*
 * sssp_batch: many independent parDijkstra queries in one persistent launch
 * (each query runs the rounds of Section 4.1 on its own parallel bucket heap;
 * every heap lives in one device arena; workgroups take queries from a queue,
 * largest first).  queries is a HOST array of nq descriptors.  opts as for
 * sssp_ex (d = 0 means each query uses its graph's maximum out-degree); stats
 * (may be NULL) receives totals over all queries and the launch's kernel
 * time.  Each dist_out is exactly what sssp would return for that query.
 * Errors: PBH_EINVAL (NULL or malformed query, nq == 0 is allowed and does
 * nothing), PBH_ENOMEM, PBH_EDEVICE, PBH_EINTERNAL.
 */
int sssp_batch(const sssp_query *queries, uint32_t nq, const sssp_opts *opts, sssp_stats *stats,
               void *stream);

/*
 * sssp_nearfar: single-source shortest paths by Near-Far, the GPU form of
 * Delta-stepping (Meyer and Sanders; Davidson et al. 2014) that the paper
 * compares parDijkstra against (Sections 1.1 and 4.2: Gunrock and ADDS are
 * Delta-stepping codes).  A baseline, not the paper's method: vertices whose
 * tentative distance is below a threshold T form the near frontier and are
 * scanned phase by phase; the others wait in a far pile until T has grown
 * past them by steps of delta (0 = Davidson et al.'s choice, mean weight x 64
 * / mean out-degree).  Exact for any delta.  One cooperative launch over
 * every compute unit; graph and dist_out as for sssp (device arrays).  stats
 * (host, may be NULL) receives edges scanned, phases, threshold steps, the
 * delta used, the workgroups and the kernel's HIP-event time.  The call
 * allocates and frees its own work space (about 40 bytes per vertex).
 * Errors: PBH_EINVAL (NULL arrays, n == 0, source >= n, malformed CSR),
 * PBH_ENOMEM, PBH_EDEVICE, PBH_ETIMEOUT (a grid barrier's bounded wait ran
 * out), PBH_EINTERNAL (a queue overflowed or the phase limit was reached);
 * sssp_nearfar_last_error() describes the last failure of the calling thread.
 */
typedef struct {
  uint64_t relaxations; /* edges scanned */
  uint32_t phases;      /* relax and threshold phases */
  uint32_t splits;      /* threshold steps */
  uint64_t delta;       /* delta used */
  uint32_t workgroups;
  uint32_t reserved;
  double kernel_ms;
} sssp_nearfar_stats;
int sssp_nearfar(const uint64_t *offsets, const uint32_t *targets, const uint32_t *weights, uint32_t n,
                 uint64_t m, uint32_t source, uint64_t *dist_out, uint64_t delta, sssp_nearfar_stats *stats,
                 void *stream);
const char *sssp_nearfar_last_error(void);

/*
 * sssp_autotune: picks opts->d and opts->k_max for this query by timing trial
 * runs on the query itself.  A plain trial of n/32 rounds finds a distance
 * frontier D (the smallest key left after them); then each candidate
 * (d = max out-degree * 1, 2, 4, ... up to 2048; team 64 or 256 threads for
 * d in [64, 2048] unless opts->team fixes it; k_max 1 (the plain rule), 64
 * or 256 when k_rule != 0) runs until every vertex closer than D is settled,
 * which is the
 * same work for every candidate; the three fastest run again to the frontier
 * of n/8 plain rounds, the two fastest there run to the end (the cost of a
 * large d grows with the heap, which the early frontiers do not show), and
 * the faster of those is written back into *opts (d, team, k_max; the other
 * fields, k_scale and deep_level included, are kept and used for the
 * trials).  With the learned rule and opts->k_every == 0, the winner also
 * runs once with the model every 4th and once with it every 16th round, and
 * opts->k_every becomes 1, 4 or 16, whichever was fastest.  A query that
 * finishes within a frontier
 * trial skips the later stages.
 * dist_out is used as scratch.  Errors: those of sssp_ex.
 */
int sssp_autotune(const uint64_t *offsets, const uint32_t *targets, const uint32_t *weights, uint32_t n,
                  uint64_t m, uint32_t source, uint64_t *dist_out, sssp_opts *opts, void *stream);

/*
 * sssp_batch_autotune: picks opts->d_scale (with opts->d = 0), opts->team and
 * opts->k_max for a batch: the largest query (the critical path of the
 * persistent launch) is tuned as by sssp_autotune; its (at most three) best
 * settings, and every multiple of the maximum out-degree up to d = 2048 with
 * the best setting's team and k_max (unless that is the plain rule), then
 * run the whole batch, each query's d being the multiple of its own maximum
 * out-degree; the fastest launch wins.  Every query's dist_out is used as
 * scratch.  Errors: those of sssp_ex and sssp_batch.
 */
int sssp_batch_autotune(const sssp_query *queries, uint32_t nq, sssp_opts *opts, void *stream);

/*
 * Training of the extraction-threshold model (not in the paper: an addition
 * that chooses k per round).  All arrays are device arrays; calls synchronous.
 *
 * mlp_trace_labels: labels[r] = log2 of the longest prefix of trace record r
 *   (its keys in order) whose keys equal dists[trace_query[r]][id], i.e. how
 *   many minima the round could have pulled with no wasted relaxation.
 *   dists is a device array of nq per-query distance arrays (final
 *   distances) and dist_n a device array of their lengths; a record whose
 *   query index is >= nq or whose ids are not below that query's length is
 *   rejected with PBH_EINVAL before any label is written.
 * mlp_feature_stats: writes the feature means and standard deviations of
 *   X[n][8] into blob (the mu and sd fields).
 * mlp_grad: gradient of the mean squared error of the model on (X[n][8],
 *   Y[n]) with respect to the PBH_MLP_PARAMS master weights of blob (forward
 *   with the weights rounded to bfloat16, FP32 accumulation; the rounding is
 *   taken as identity in the backward pass); loss[0] = the error.  n <= 65536.
 * mlp_train: `steps` Adam steps (lr, betas 0.9/0.999) over consecutive
 *   mini-batches of `batch` samples (the caller shuffles X), updating blob in
 *   place, then rounds the weights to bfloat16.  loss_trace (HOST, may be NULL)
 *   receives the loss of every step.
 * Errors: PBH_EINVAL (NULL or empty arguments), PBH_ENOMEM, PBH_EDEVICE.
 */
int mlp_trace_labels(const uint64_t *trace_keys, const uint32_t *trace_ids, const uint32_t *trace_query,
                     uint32_t count, const uint64_t *const *dists, const uint32_t *dist_n, uint32_t nq,
                     float *labels);
int mlp_feature_stats(const float *X, uint32_t n, float *blob);
int mlp_grad(const float *X, const float *Y, uint32_t n, const float *blob, float *grad, float *loss);
int mlp_train(const float *X, const float *Y, uint32_t n, float *blob, uint32_t batch, uint32_t steps, float lr,
              float *loss_trace);

/*
 * mlp_infer: the round loop's own inference of the model on n given feature
 * rows (device X[8n], blob as k_model, y[n] out): y[r] = scale * (network
 * output), i.e. k = 2^y before clamping.  team 64 or 256 selects the code
 * path the round loop uses with that team size (the wider one splits the
 * second layer over four threads per unit).  Errors: PBH_EINVAL (NULL
 * arrays, team not 64/256), PBH_EDEVICE.
 */
int mlp_infer(const float *X, uint32_t n, const float *blob, uint32_t team, float *y);

/* Message describing the calling thread's last failure ("" if none). */
const char *pbh_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PBH_H */
