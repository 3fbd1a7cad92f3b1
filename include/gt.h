/*
 * gt.h — stable CSR -> CSC graph transposition on one AMD MI355X (gfx950).
 *
 * Operation (Section II-A, Algorithm 1 of "On Optimizing Locality of Graph
 * Transposition on Modern Architectures"): given a directed graph in CSR form
 * (offsets[n+1], edges[m] holding destinations, optional 32-bit weight per
 * edge), produce its CSC form (offsets[n+1], edges[m] holding sources,
 * weights moved with their edges).  This library fixes the order inside each
 * CSC list, which the paper leaves open (Section II-B, optional sort): the
 * slots offsets[v] .. offsets[v+1]-1 hold the in-edges of v in increasing
 * CSR edge position, i.e. ascending source, and multi-edges from one source
 * in CSR order.  The result is therefore unique and deterministic.
 *
 * Types and layout (all arrays are device memory, owned by the caller):
 *   offsets  int64[n+1]   offsets[0] = 0, nondecreasing, offsets[n] = m
 *   indices  int32[m]     0 <= indices[e] < n;  n <= 2^31 - 1
 *   payload  uint32[m]    optional; 32-bit words copied bit-exactly (a float
 *                         payload is passed as its bit pattern)
 * Output arrays (caller-allocated, must not alias the input):
 *   offsets int64[n+1], indices int32[m], payload uint32[m] (NULL iff the
 *   input payload is NULL).
 *
 * Workspace: the library never allocates or frees device memory.  The caller
 * asks gt_workspace_size() for a byte count and passes a device buffer of at
 * least that size; its contents need no initialisation and are clobbered.
 *
 * Streams: gt_transpose / gt_transpose_batched enqueue kernels on `stream`
 * and return without synchronising, so they may be captured into a HIP graph.
 * gt_plan with the HEURISTIC or FIXED policy does no device work and no
 * synchronisation (it may be called while `stream` is being captured); the
 * MLP policy, GT_FLAG_FEATURES and GT_STRATEGY_PROBE sample or time the
 * graph on `stream` and synchronise it once.
 * A plan and a workspace must not be used by two streams at the same time.
 *
 * Errors: argument and size problems are reported synchronously by the
 * return code; nothing throws across this interface.  Conditions found on the
 * device (an invalid graph when validation is on, a count that does not add
 * up) are written to a status word in the workspace and read with
 * gt_plan_device_status() after the stream has been synchronised.
 */
#ifndef GT_H
#define GT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GT_OK = 0,
  GT_ERR_INVALID_ARGUMENT = 1,   /* NULL pointer, negative size, n > 2^31-1, payload mismatch */
  GT_ERR_INVALID_GRAPH = 2,      /* device-detected: bad offsets or an index outside [0, n) */
  GT_ERR_WORKSPACE_TOO_SMALL = 3,
  GT_ERR_UNSUPPORTED = 4,        /* a parameter outside the compiled kernel variants, or m > 2^32 */
  GT_ERR_HIP = 5,                /* a HIP runtime call failed */
  GT_ERR_COUNTER_OVERFLOW = 6,   /* device-detected: counts that do not add up to m (a wrapped counter) */
  GT_ERR_STALLED = 7             /* device-detected: a wait of the persistent batched kernel gave up */
} gt_status;

/* Largest edge count accepted (GT_ERR_UNSUPPORTED above it): with m <= 2^32
 * every 64-bit total and every 32-bit per-chunk prefix of one vertex's list
 * is exact.  The device still checks that every pass's digit counts add up
 * to m and every heavy bin's vertex counts to the bin's length; a mismatch
 * (only a wrapped counter can cause one) is reported as
 * GT_ERR_COUNTER_OVERFLOW by gt_plan_device_status(). */
#define GT_MAX_EDGES 4294967296LL

/* A CSR graph (input).  Device pointers; payload may be NULL. */
typedef struct {
  int64_t n, m;
  const int64_t *offsets;
  const int32_t *indices;
  const uint32_t *payload;
} gt_csr_t;

/* A CSC graph (output).  Device pointers; payload NULL iff the input's is. */
typedef struct {
  int64_t *offsets;
  int32_t *indices;
  uint32_t *payload;
} gt_csc_t;

/* Policies for choosing the kernel parameters of a plan. */
enum {
  GT_POLICY_HEURISTIC = 0,  /* from n and m alone (default): no device work while planning */
  GT_POLICY_FIXED = 1,      /* use fine_bits / digit_bits / variant as given */
  GT_POLICY_MLP = 2         /* learned choice from sampled features (falls back to HEURISTIC) */
};

/* Options; pass NULL for defaults.  Fields set to 0 take their default. */
typedef struct {
  int32_t policy;        /* GT_POLICY_* */
  int32_t fine_bits;     /* log2 of the vertex range sorted in LDS by the last kernel (4..9) */
  int32_t digit_bits;    /* maximum digit width of one stable partition pass (4..10) */
  int32_t variant;       /* tile variant of the partition kernels (0 = auto, 1..N) */
  int32_t validate;      /* 1: also check the offsets on the device (indices are always checked) */
  uint64_t seed;         /* seed of the degree-sampling pass */
  const char *model_path;/* weights of the learned policy (GT_POLICY_MLP) */
  int32_t flags;         /* GT_FLAG_* */
  int32_t strategy;      /* GT_STRATEGY_* (0 = the stable method) */
  int32_t hdv_max;       /* GT_STRATEGY_HLH: at most this many HDVs (0 = 8192, the maximum: Eq. 1 on 160 KB of LDS) */
} gt_options_t;

/* Strategies.  GT_STRATEGY_STABLE (the default) produces every CSC list in
 * increasing CSR edge position.  The other two are the paper's own methods
 * and leave the order inside each CSC list to the atomics, as the paper does
 * (the offsets and the multiset of every list are exact):
 *   GT_STRATEGY_HLH    PoTra (Section IV, Algorithm 2): HDVs found by a 1%
 *                      degree sample, counted and placed through per-chunk
 *                      LDS counters; LDVs through wave-aggregated global
 *                      atomics.
 *   GT_STRATEGY_ATOMIC Atomic GT (Algorithm 1): every destination through
 *                      wave-aggregated global atomics.
 *   GT_STRATEGY_PROBE  the probe of Section IV-C: gt_plan times the in-degree
 *                      count (Step 1) with and without the HDV table on a
 *                      sixteenth of the edges (the first sixteenth of every
 *                      edge chunk, on the grid of a full launch) and keeps
 *                      the faster of HLH and Atomic GT (gt_plan_strategy
 *                      reports it; an empty graph gets Atomic GT).  gt_plan
 *                      then needs a workspace of gt_workspace_size() bytes
 *                      (GT_ERR_WORKSPACE_TOO_SMALL otherwise) and
 *                      synchronises the stream. */
enum { GT_STRATEGY_STABLE = 0, GT_STRATEGY_HLH = 1, GT_STRATEGY_ATOMIC = 2, GT_STRATEGY_PROBE = 3 };

/* Flags.  GT_FLAG_WIDE_STATUS forces the 64-bit look-back words that graphs
 * with m >= 2^31 use, so that path can be tested on small graphs.
 * GT_FLAG_FEATURES makes gt_plan sample every graph and keep its feature
 * vector (gt_plan_features) whatever the policy; it then needs the sampling
 * scratch (gt_plan_scratch_size) and synchronises the stream. */
/* Step 3 (the scatter) of GT_STRATEGY_HLH / GT_STRATEGY_ATOMIC, Section V-F:
 * by default one workgroup per chunk of the edges, up to 2048 chunks, which
 * the GPU's dispatcher hands to free compute units (Step 1 uses the same
 * chunks).  GT_FLAG_STEP3_STATIC: as many chunks as workgroups of the
 * scatter kernel fit on the device at once, each scattered by its own
 * workgroup (the paper's static partition of Steps 1 and 3).
 * GT_FLAG_STEP3_STEAL: the same chunks, Step 3 in the two phases the paper
 * proposes: every workgroup first scatters the first 80% of its own chunk,
 * then claims the remaining parts of all chunks (four of 5% each) from one
 * atomic counter, in chunk order, until none is left.  Step 1 counts every
 * part's HDVs separately, so a part scattered by another workgroup still
 * places its HDV edges through LDS cursors.  GT_FLAG_STEP3_TIMES records
 * per-chunk wall-clock stamps of Step 3 (gt_plan_step3_times).  The output
 * does not depend on these flags beyond the order the atomics give. */
/* GT_FLAG_PERSISTENT: gt_transpose_batched runs the whole batch as one
 * persistent kernel launch (see there).  Its bodies take variant-1 tiles and
 * digits of at most 9 bits, so the plan's choice of every graph is adjusted
 * to that (gt_plan_set_config's too); gt_plan returns GT_ERR_UNSUPPORTED for
 * a graph that still does not fit (more than two partition passes, m >= 2^31,
 * GT_FLAG_WIDE_STATUS, an unordered strategy). */
/* GT_FLAG_DEVICE_PLAN (with GT_FLAG_PERSISTENT and GT_POLICY_MLP, at most
 * 4096 graphs): the learned choice of Section IV-C stays on the device.
 * gt_plan enqueues the sampling (Step 0), the network and the choice of every
 * graph on `stream` and returns without synchronising; the workspace it is
 * given must hold gt_plan_workspace_size() bytes (gt_workspace_size() is
 * enough) and is the one every gt_transpose_batched call of the plan must
 * use, since the choices live in it.  Each gt_transpose_batched call lays
 * the graphs out and builds the persistent kernel's tables in a planning
 * kernel on the device, so gt_plan and the transpositions capture into one
 * HIP graph.  Every graph's region is sized for any choice; a graph for
 * which one possible choice does not fit the persistent kernel is refused
 * (GT_ERR_UNSUPPORTED).  gt_plan_params reports the heuristic's parameters,
 * gt_plan_device_choice the learned ones; gt_transpose, gt_transpose_noalloc
 * and gt_plan_set_config refuse such plans (GT_ERR_UNSUPPORTED). */
enum { GT_FLAG_WIDE_STATUS = 1, GT_FLAG_FEATURES = 2, GT_FLAG_STEP3_STATIC = 4, GT_FLAG_STEP3_STEAL = 8,
       GT_FLAG_STEP3_TIMES = 16, GT_FLAG_PERSISTENT = 32, GT_FLAG_DEVICE_PLAN = 64 };

typedef struct gt_plan_st *gt_plan_t;

/* Bytes of workspace that suffice for gt_plan and for transposing `count`
 * graphs with any parameters any policy can pick (an upper bound). */
gt_status gt_workspace_size(const gt_csr_t *graphs, int32_t count, size_t *bytes_out);

/* Bytes of workspace gt_plan needs for `count` graphs: the degree-sampling
 * scratch and the learned policy's inputs (the MLP policy and
 * GT_FLAG_FEATURES; HEURISTIC and FIXED plans touch no workspace). */
gt_status gt_plan_scratch_size(const gt_csr_t *graphs, int32_t count, size_t *bytes_out);

/* Bytes of workspace gt_transpose / gt_transpose_batched need with the
 * parameters this plan holds (at most gt_workspace_size(); may change after
 * gt_plan_set_config). */
gt_status gt_plan_workspace_size(gt_plan_t plan, size_t *bytes_out);

/* Build a plan for `count` graphs (count == 1 for gt_transpose): the
 * preprocessing of Section IV-C (Step 0: a degree sample of 1% of |V| edge
 * positions, then the choice of parameters; Eq. 1 sizes the LDS-resident
 * work of the heuristic).
 *   graphs      host array of `count` descriptors (device pointers inside,
 *               read by the sampling kernels during this call only)
 *   opt         options, or NULL for the defaults
 *   workspace   device buffer of at least gt_plan_scratch_size() bytes for
 *               the MLP policy and GT_FLAG_FEATURES (may be NULL for
 *               HEURISTIC and FIXED); clobbered
 *   stream      HIP stream (hipStream_t) of the sampling kernels; the call
 *               synchronises it once when it samples (MLP, GT_FLAG_FEATURES,
 *               GT_STRATEGY_PROBE), and does not touch it otherwise
 *   plan_out    receives the plan (host memory only; gt_plan_destroy)
 * Errors: GT_ERR_INVALID_ARGUMENT (NULL pointer, count <= 0, n < 0, m < 0,
 * n > 2^31 - 1), GT_ERR_UNSUPPORTED (an option out of range, m > 2^32),
 * GT_ERR_WORKSPACE_TOO_SMALL, GT_ERR_HIP. */
gt_status gt_plan(const gt_csr_t *graphs, int32_t count, const gt_options_t *opt, void *workspace,
                  size_t workspace_bytes, void *stream, gt_plan_t *plan_out);

/* Transpose one graph (Section II-A; the result Algorithm 1 reaches when run
 * by one thread, lists in increasing CSR edge position for the stable
 * strategy).  The plan was built with count == 1 for a graph of the same n,
 * m and payload presence.
 *   g           CSR in device memory (offsets int64[n+1], indices int32[m],
 *               payload uint32[m] or NULL); not modified
 *   out         caller-allocated CSC: offsets int64[n+1], indices int32[m],
 *               payload uint32[m] (NULL iff g->payload is NULL); must not
 *               alias the input
 *   workspace   at least gt_plan_workspace_size() bytes; clobbered
 *   stream      HIP stream; the call only enqueues kernels (no host
 *               synchronisation, capturable into a HIP graph)
 * Errors: GT_ERR_INVALID_ARGUMENT (NULL pointers, sizes other than the
 * plan's), GT_ERR_WORKSPACE_TOO_SMALL, GT_ERR_HIP (a launch failed).  An
 * index outside [0, n) is always reported by gt_plan_device_status() after
 * the stream has completed (GT_ERR_INVALID_GRAPH); opt->validate adds the
 * check of the offsets.  The output of an invalid graph is undefined, but
 * every kernel stays inside its buffers: an edge whose destination does not
 * exist is never written outside the output arrays. */
gt_status gt_transpose(gt_plan_t plan, const gt_csr_t *g, gt_csc_t *out, void *workspace,
                       size_t workspace_bytes, void *stream);

/* Transpose `count` graphs (each as gt_transpose) for a plan built for the
 * same count and sizes.  graphs / outs: host arrays of `count` descriptors.
 * The call is one asynchronous, capturable launch sequence on `stream`.
 * Default: the kernels of different graphs run on the plan's internal
 * streams (forked from `stream` by one event and joined back by one event
 * per stream).  GT_FLAG_PERSISTENT plans: one copy of the graph descriptors
 * and the phase table from the plan's pinned staging buffer into the
 * workspace, one clear of the queue counters, then one launch of the
 * persistent kernel, whose resident workgroups take (graph, phase, item)
 * tickets from one device counter and run every phase of every graph in
 * dependency order (Section V-F's dynamic work distribution, over the whole
 * batch).  The call waits (on the host) for the previous call's copy out of
 * the staging buffer unless `stream` is being captured; a captured batch
 * copies the staging buffer's contents at replay, so a plan whose batch is
 * captured must not be run eagerly with other buffers between replays.
 * Errors as gt_transpose; a wait of the persistent kernel that gives up is
 * reported as GT_ERR_STALLED by gt_plan_device_status(). */
gt_status gt_transpose_batched(gt_plan_t plan, int32_t count, const gt_csr_t *graphs, gt_csc_t *outs,
                               void *workspace, size_t workspace_bytes, void *stream);

/* ---- For callers that cannot allocate device memory (code being captured
 * into a HIP graph, tight serving loops, harnesses that forbid hipMalloc):
 * gt_transpose with the library's own scratch instead of a workspace.
 * The scratch is one static device array of GT_NOALLOC_SCRATCH_BYTES per GPU,
 * held from the first call on that GPU until the process ends; the call
 * itself allocates nothing (no hipMalloc, no hipFree, no allocating library
 * routine) and does not synchronise.  Every call on one GPU shares that
 * GPU's scratch, so calls that overlap on one GPU (two streams, two host
 * threads) race: the caller serialises them.  The scratch keeps the last
 * call's contents; everything that must start at zero is cleared by the
 * call's own kernels.
 *   plan        built with count == 1 (any policy and strategy) for a graph
 *               of the same n, m and payload presence; its workspace need
 *               (gt_plan_workspace_size) must be at most
 *               GT_NOALLOC_SCRATCH_BYTES
 *   g, out      as gt_transpose
 *   status_out  NULL, or a device pointer to one uint32 that receives the
 *               device-detected status word when the stream reaches the end
 *               of the call: 0 = GT_OK, else bit 0 or 1 = GT_ERR_INVALID_GRAPH,
 *               bit 2 = GT_ERR_COUNTER_OVERFLOW (the conditions of
 *               gt_plan_device_status)
 *   stream      HIP stream of the current device (the scratch is that
 *               device's copy)
 * Errors: as gt_transpose; GT_ERR_WORKSPACE_TOO_SMALL when the plan needs
 * more than GT_NOALLOC_SCRATCH_BYTES; GT_ERR_INVALID_ARGUMENT when `stream`
 * belongs to another device than the current one. */
#define GT_NOALLOC_SCRATCH_BYTES (64u << 20)
gt_status gt_transpose_noalloc(gt_plan_t plan, const gt_csr_t *g, gt_csc_t *out, uint32_t *status_out,
                               void *stream);

/* After the stream has been synchronised: the device-detected status of the
 * last transposition run with this plan in `workspace`.  GT_OK;
 * GT_ERR_INVALID_GRAPH if an index lies outside [0, n) or (with validation)
 * the offsets are not nondecreasing from 0 to m; GT_ERR_COUNTER_OVERFLOW if
 * a count did not add up (see GT_MAX_EDGES); GT_ERR_STALLED if a dependency
 * wait of the persistent batched kernel gave up (after seconds; the output is
 * then undefined).  Reads 4 bytes of the workspace
 * with a blocking copy.  Errors: GT_ERR_INVALID_ARGUMENT (NULL plan or
 * workspace), GT_ERR_HIP. */
gt_status gt_plan_device_status(gt_plan_t plan, const void *workspace);

/* GT_FLAG_DEVICE_PLAN plans, after the stream of gt_plan has completed: the
 * parameters chosen on the device for graph `i` (fine bits, digit width as
 * given to the layout, tile variant, configuration index or -1 when the
 * graph's features were outside the network's training range and the
 * heuristic's choice stands).  Reads 16 bytes of `workspace` with a blocking
 * copy.  Errors: GT_ERR_INVALID_ARGUMENT (NULL plan or workspace, i out of
 * range), GT_ERR_UNSUPPORTED (not a device plan), GT_ERR_HIP. */
gt_status gt_plan_device_choice(gt_plan_t plan, const void *workspace, int32_t i, int32_t *fine_bits,
                                int32_t *digit_bits, int32_t *variant, int32_t *config);

/* The same status read without a plan (the status word is byte 0 of any
 * workspace the library has used). */
gt_status gt_device_status(const void *workspace);

/* Parameters a plan selected for graph `i` (for reporting and tests): fine
 * bits of the per-bin placement, widest digit, number of partition passes,
 * tile variant.  Any output pointer may be NULL. */
gt_status gt_plan_params(gt_plan_t plan, int32_t i, int32_t *fine_bits, int32_t *digit_bits,
                         int32_t *passes, int32_t *variant);

/* Whether the plan keeps the intermediate between the two partition passes
 * of graph `i` in packed form (Section II-B, Step 3 split into two stable
 * passes): 6 + payload bytes per edge (a 16-bit key holding the last pass's
 * digit and the low fine bits, the source word carrying the remaining fine
 * bits above the vertex-ID bits) instead of 8 + payload.  Chosen by the plan
 * for every two-pass graph whose fine bits, last digit bits and vertex-ID
 * bits add up to at most 48; the output does not depend on it.  `packed`
 * receives 1 or 0; errors: GT_ERR_INVALID_ARGUMENT for a NULL plan or
 * output, or `i` outside [0, count). */
gt_status gt_plan_packed(gt_plan_t plan, int32_t i, int32_t *packed);

/* The strategy a plan runs for graph `i` (GT_STRATEGY_*; a probed plan
 * reports the method the probe kept). */
gt_status gt_plan_strategy(gt_plan_t plan, int32_t i, int32_t *strategy);

/* After the stream has been synchronised: the Step 3 stamps of the last
 * transposition of graph `i` run with this plan in `workspace` (a plan of an
 * unordered strategy built with GT_FLAG_STEP3_TIMES).  Per chunk workgroup c,
 * out[3c], out[3c+1], out[3c+2] = wall-clock ticks at its start, when its own
 * chunk's head (or whole chunk) was done, and at its end; at most
 * `max_chunks` rows.  *nchunks_out = rows available; *clock_hz = ticks per
 * second.  Blocking copy.  Errors: GT_ERR_INVALID_ARGUMENT (NULL pointers,
 * `i` out of range, a plan without the flag), GT_ERR_HIP. */
gt_status gt_plan_step3_times(gt_plan_t plan, int32_t i, const void *workspace, uint64_t *out,
                              int32_t max_chunks, int32_t *nchunks_out, double *clock_hz);

/* Release the plan's host memory and internal streams/events.  Work already
 * enqueued with it is unaffected. */
gt_status gt_plan_destroy(gt_plan_t plan);

/* Per-kernel timing for measurement.  While enabled, gt_transpose records a
 * HIP event pair around every kernel launch on the launch stream (the
 * kernels themselves are unchanged).  gt_profile_read waits for the recorded
 * events, returns per kernel name the summed milliseconds and the number of
 * launches since profiling was enabled or last read (at most `max_kernels`
 * names of up to 31 characters), and clears the record. */
gt_status gt_profile(gt_plan_t plan, int32_t enable);
gt_status gt_profile_read(gt_plan_t plan, int32_t max_kernels, char (*names)[32], double *total_ms,
                          int32_t *launches, int32_t *count_out);

const char *gt_status_string(gt_status s);

/* ---- Degree sampling features (Section IV-C Step 0 sample of 1% of |V|
 * edge positions; Section V-G coverage) of graph i of a plan built with the
 * HEURISTIC or MLP policy: up to nmax floats; *nout = number available. */
gt_status gt_plan_features(gt_plan_t plan, int32_t i, float *out, int32_t nmax, int32_t *nout);

/* ---- Configuration grid of the learned and autotuned choices.  Every
 * configuration yields the same output; they differ in speed only. */
int32_t gt_num_configs(void);
gt_status gt_config(int32_t idx, int32_t *fine_bits, int32_t *digit_bits, int32_t *variant);

/* Autotuner: time every configuration on graph g (one warm-up, median of
 * `reps` runs, HIP events on `stream`); ms_out has gt_num_configs() entries.
 * Writes the transposition to `out`.  Synchronous. */
gt_status gt_autotune(const gt_csr_t *g, gt_csc_t *out, void *workspace, size_t workspace_bytes, void *stream,
                      int32_t reps, float *ms_out);

/* Use configuration `config` for graph i of a plan (e.g. the autotuner's
 * best).  The plan's workspace need (gt_plan_workspace_size) may change; it
 * never exceeds gt_workspace_size(). */
gt_status gt_plan_set_config(gt_plan_t plan, int32_t i, int32_t config);

/* ---- The learned parameter choice: MLP 16 -> 64 -> 64 -> 32 (ReLU, fp32),
 * parameters W1[16][64] b1[64] W2[64][64] b2[64] W3[64][32] b3[32] in one
 * device array.  Training primitives (device pointers, asynchronous):
 *   forward:  y[batch][32] from x[batch][16]
 *   gradient: y, loss = mean((y - target)^2), grad[nparams];
 *             work holds gt_mlp_work_floats(batch) floats
 *   adam:     one Adam step (step >= 1) on params with moments m1, m2 */
int32_t gt_mlp_num_params(void);
size_t gt_mlp_work_floats(int32_t batch);
gt_status gt_mlp_forward(const float *params, const float *x, int32_t batch, float *y, void *stream);
gt_status gt_mlp_gradient(const float *params, const float *x, const float *target, int32_t batch, float *y,
                          float *grad, float *loss, float *work, void *stream);
gt_status gt_mlp_adam(float *params, const float *grad, float *m1, float *m2, int32_t step, float lr, float beta1,
                      float beta2, float eps, void *stream);

/* ---- Random-access microbenchmark (Section III-B, Fig. 3; the per-access
 * times of Eq. 2 and Eq. 3, Section IV-B) -------------------------------------
 * blocks x 256 threads each make `per_thread` accesses of one kind at random
 * indices of a 32-bit array.  Thread t = block * 256 + lane draws access j at
 * index ((uint64)r * words) >> 32, r = fmix32(fmix32(seed ^ t) + (j + 1) *
 * 0x9E3779B9) (fmix32: the 32-bit MurmurHash3 finalizer), so the indices are
 * a pure function of (seed, t, j) and lie in [0, words).
 *   GT_ACCESS_READ    acc ^= a[idx]; sink[t] = acc at the end
 *   GT_ACCESS_WRITE   a[idx] = t (plain stores; the value that survives at an
 *                     index written by several threads is any one of theirs)
 *   GT_ACCESS_ATOMIC  atomicAdd(&a[idx], 1) (device-scope, no return value)
 *   GT_ACCESS_INDEX   acc ^= idx, no memory access (the generator's cost)
 * memory GT_MEMORY_GLOBAL: a = buf, a device array of `words` words
 *   (1 <= words <= 2^32); the size picks the level the accesses hit (L2,
 *   Infinity Cache or HBM).
 * memory GT_MEMORY_LDS: each workgroup b copies buf[b*words, (b+1)*words) into
 *   LDS, accesses it there and copies it back; buf holds blocks * words words,
 *   1 <= words <= 16384 (64 KB of LDS per workgroup).
 * sink: NULL, or a device array of blocks * 256 words written once per thread
 * (0 for WRITE and ATOMIC).  blocks in [1, 2^20], per_thread >= 0.  Enqueued
 * on `stream` without synchronising; the caller times it.  Errors:
 * GT_ERR_INVALID_ARGUMENT for a NULL buf, a zero size or an unknown kind or
 * memory, GT_ERR_UNSUPPORTED for words above the limits, GT_ERR_HIP when the
 * launch fails. */
enum { GT_ACCESS_READ = 0, GT_ACCESS_WRITE = 1, GT_ACCESS_ATOMIC = 2, GT_ACCESS_INDEX = 3 };
enum { GT_MEMORY_GLOBAL = 0, GT_MEMORY_LDS = 1 };
gt_status gt_random_access(uint32_t *buf, uint64_t words, int32_t kind, int32_t memory, uint32_t seed,
                           int64_t per_thread, int32_t blocks, uint32_t *sink, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GT_H */
