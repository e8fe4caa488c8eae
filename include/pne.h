/*
 * pne.h — C ABI of the MI355X (gfx950) partitioned-network-expansion library.
 *
 * What the library computes (Evenbly, Gray, Chan, "Partitioned Expansions for
 * Approximate Tensor Network Contractions"):
 *
 *   Input  : a tensor network — site tensors T_r joined by indices (Sec. II.A,
 *            Eq. (1)) — optionally with open indices (Sec. III.D).
 *   Method : every bond is a single-index partition P_b + Q_b = I (Eq. (2));
 *            P_b is the rank-1 projector made from the two fixed-point belief
 *            propagation messages on the bond (Eq. (8)), symmetrised by the
 *            gauge of Appendix B; the complete P/Q expansion (Eq. (4)) is
 *            truncated to configurations of at most K excited (Q) bonds that
 *            have no dangling excitation (Sec. III.A-B, "degree").
 *   Output : the approximate contraction value as (sign, ln|Z|), or, for a
 *            network with open legs, the open-index tensor with an FP64
 *            log-scale.
 *
 * Conventions for every call:
 *   - Integers describing the graph are int32; tensor values are FP64 at the
 *     boundary in every precision mode.
 *   - Site tensors are dense, C order over the site's leg slots 0..rank-1.
 *   - Ownership: the caller owns every descriptor array and every host or
 *     device buffer it passes.  The library copies host data, borrows device
 *     data (see pne_network_create), and never frees caller memory.
 *   - Errors: a negative pne_status is a failure (no result), a positive one
 *     is a warning with a result.  pne_last_error() gives a message.
 *   - Threading: a context is used by one thread at a time, except for the
 *     server calls, which are thread safe.
 *   - Streams: all device work is enqueued on the context's HIP stream.
 */
#ifndef PNE_H
#define PNE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PNE_OK = 0,
    PNE_WARN_BP_NOT_CONVERGED = 1, /* result computed from the last BP sweep */
    PNE_WARN_PRECISION = 2,        /* reduced term precision: the estimated error of the result
                                      (pne_result.term_err_est) exceeds pne_options.err_bound */
    PNE_ERR_INVALID_ARG = -1,      /* malformed network, options or pointer */
    PNE_ERR_UNSUPPORTED = -2,      /* outside the implemented envelope */
    PNE_ERR_OUT_OF_MEMORY = -3,    /* device allocation failed or budget exceeded */
    PNE_ERR_SINGULAR = -4,         /* a bond overlap a.c ~ 0 or a vacuum factor == 0 */
    PNE_ERR_DEVICE = -5,           /* HIP runtime error or no usable device */
    PNE_ERR_NOT_READY = -6,        /* pne_poll: request still running */
    PNE_ERR_CANCELLED = -7,        /* pne_poll: the request was cancelled (pne_cancel) */
    PNE_ERR_CHECK = -8             /* checked build (libpne_checked.so) only: a cluster
                                      kernel index left its table, frontier or slice
                                      buffer; the access was suppressed and the
                                      network's result is invalid (a library bug)   */
} pne_status;

/* pne_options.flags bits */
#define PNE_FLAG_PROFILE 1u /* time every kernel launch with HIP events on the context stream */
#define PNE_FLAG_NO_PERSISTENT 2u /* sweep every network launch by launch (no persistent BP kernel) */
#define PNE_FLAG_BP_JACOBI 4u /* persistent BP: Jacobi sweeps even on bipartite networks (see below) */
#define PNE_FLAG_SEPARATE_REGAUGE 8u /* gauge + slices in their own launch, not in the persistent BP block */
#define PNE_FLAG_GRAPH 16u /* capture a batch's launch sequence (and result copies) into a HIP graph on its
                              first launch and replay it; applies when every network's BP runs in the
                              persistent kernel, profiling is off and the stream is not the null stream */
#define PNE_FLAG_AUTOTUNE 32u /* pne_batch_create: pick PNE_FLAG_GRAPH / PNE_FLAG_SEPARATE_REGAUGE by
                                 measurement (pne_autotune), cached per batch signature in the context */

/* BP schedule.  Jacobi: every sweep updates every message from the previous
 * sweep's messages.  On a bipartite network (two site colours, every bond
 * joining different colours) the persistent kernel by default runs the
 * red-black schedule instead: step t updates only the messages leaving sites
 * of colour t mod 2, in place.  Its messages after step t equal Jacobi's on
 * one of the two independent message chains Jacobi carries on such a graph,
 * so it reaches the same fixed point in about as many steps while reading
 * half the site tensors per step.  It stops once two consecutive steps (both
 * colours) change no message by more than bp_tol; bp_iters then counts
 * steps.  The per-launch path always runs Jacobi sweeps. */

/* Precision of the excited slices and the cluster (term) contractions.  BP,
 * the bond gauge, vacuum log-norms and the cross-term sum are FP64 always. */
typedef enum {
    PNE_FP64 = 0, /* FP64 slices, FP64 arithmetic */
    PNE_FP32 = 1, /* FP32 slices, FP32 arithmetic with FP32 accumulation */
    PNE_BF16 = 2  /* BF16 slices, FP32 arithmetic with FP32 accumulation */
} pne_precision;

/* Which configurations are summed (Sec. II.A, Sec. III.A-B). */
typedef enum {
    PNE_MODE_LOOP = 0, /* degree <= K, no dangling site (a site with exactly one excited bond;
                          sites with open legs exempt): the retained terms of the method */
    PNE_MODE_FULL = 1, /* every configuration of degree <= K, dangling ones included.  With
                          K >= n_bonds this is the complete P/Q expansion of Eqs. (2)-(4), equal
                          to the exact contraction for any rank-1 projectors, converged or not: a
                          self-check for tiny networks.  Closed networks without user partitions,
                          at most 20 bonds (UNSUPPORTED otherwise). */
    PNE_MODE_CUMULANT = 2 /* the retained clusters of LOOP mode in exponentiated form: with the
                          clusters as polymers, incompatible when they share a site, ln(1 + S)
                          is replaced by its Mayer series to second order,
                            F = sum_c w_c - 1/2 sum_{(c,c') incompatible, |c|+|c'| <= K} w_c w_c'
                          (ordered pairs, c = c' included), and ln|Z| = ln|Z_BP| + F, sign that
                          of Z_BP.  F is additive over distant parts of a network (size
                          extensive).  Closed networks without user partitions, K < 3 x the
                          smallest cluster (UNSUPPORTED otherwise); pne_result.n_config_terms
                          then counts clusters. */
} pne_mode;

/* A tensor network (Sec. II.A).  Every leg slot of every site is either
 * joined by exactly one bond or listed exactly once as an open leg. */
typedef struct {
    int32_t n_sites;
    int32_t n_bonds;
    int32_t n_open;
    const int32_t *site_rank;     /* [n_sites] number of leg slots (>= 1)        */
    const int32_t *leg_dim;       /* [sum site_rank] dims of the slots, site-major */
    const int32_t *bond_site;     /* [2*n_bonds] (u, v) per bond, u != v           */
    const int32_t *bond_leg;      /* [2*n_bonds] (slot at u, slot at v)            */
    const int32_t *open_leg;      /* [2*n_open] (site, slot); may be NULL if 0     */
    const double *const *site_data; /* [n_sites] FP64 tensors, host or device      */
} pne_network_desc;

typedef struct {
    int32_t max_excited;  /* K: largest retained configuration degree (>= 0)   */
    int32_t precision;    /* pne_precision                                       */
    double bp_tol;        /* stop when the largest sign-insensitive inf-norm
                             message change of a sweep is <= bp_tol (1e-13)
                             (red-black schedule: of the last two steps), or
                             at the rounding floor (bp_stall_steps)            */
    int32_t bp_max_iter;  /* sweep cap (500)                                     */
    int32_t bp_check_every; /* sweeps between host convergence checks (0: auto) */
    uint32_t flags;       /* PNE_FLAG_* bits (0: defaults)                       */
    int32_t profile_kernels; /* with PNE_FLAG_PROFILE: bit k times kernel index k of
                                pne_batch_kernel_times only; 0 times every kernel  */
    int32_t mode;         /* pne_mode (PNE_MODE_LOOP)                            */
    int32_t bp_stall_steps; /* rounding-floor stop: BP also ends, as converged,
                             when its smallest residual so far is <= 100 *
                             bp_tol and no sweep has lowered it for this many
                             sweeps (0: 50; < 0: never).  The residual then sits
                             at the rounding floor of the messages, which a
                             badly conditioned bond gauge can raise above
                             bp_tol; bp_residual reports the value reached.    */
    double bp_damping;    /* 0 <= lambda < 1 (0): every stored message is the
                             normalised, sign-fixed mix (1-lambda) m_new +
                             lambda m_old of the normalised update and the same
                             directed message of the previous sweep; the
                             residual compares the stored message with m_old.
                             lambda > 0 runs Jacobi sweeps launch by launch.   */
    double err_bound;     /* reduced-precision bound (1e-5): a closed result whose
                             term_err_est / max(1, |ln|Z||) exceeds it, or an open
                             one whose term_err_est exceeds it, is returned with
                             PNE_WARN_PRECISION (FP64 mode never warns)          */
    /* Tile shape of the persistent BP kernel (execution only: results agree
     * to rounding; see pne_autotune, which picks them by measurement). */
    int32_t small_sites;     /* networks of at most this many sites run in
                                two-wave blocks, the others in eight-wave ones
                                (0: 64)                                         */
    int32_t tiles_in_flight; /* tiles per wavefront step for the register shapes
                                with all legs of dimension 2..4: 1 or 2 (0: by
                                shape: 2 where a tile holds at most 4 register
                                values per lane, else 1)                        */
    int32_t reg_budget;      /* 0: 128 VGPRs per lane, two blocks per CU, 79 KB
                                of LDS per block; 1: 256 VGPRs, one block per CU,
                                155 KB of LDS (larger networks stay in the
                                persistent kernel)                              */
    int32_t reserved1;
} pne_options;

/* One network's result.  Closed network: Z = sign * exp(log_abs).  Open
 * network: Out[i_0, i_1, ...] = open_values[...] * exp(log_abs), axes in the
 * order of the descriptor's open legs, C order. */
typedef struct {
    int32_t status;          /* pne_status of this network                     */
    int32_t sign;            /* +1, -1 (0 if Z == 0)                            */
    double log_abs;          /* ln|Z| (closed) or the log-scale (open)          */
    double log_abs_bp;       /* ln|Z_BP| (closed) or the vacuum log-scale       */
    int32_t bp_iters;        /* sweeps (red-black schedule: steps) performed    */
    int32_t n_open_values;   /* number of entries written to open_values        */
    double bp_residual;      /* last sweep's residual                            */
    int64_t n_cluster_terms; /* connected dangling-free clusters contracted      */
    int64_t n_config_terms;  /* retained configurations (collections), excl. 0  */
    double *open_values;     /* caller buffer for open networks, or NULL        */
    int64_t open_capacity;   /* entries available in open_values                */
    /* Size of the dropped dangling terms (Sec. III.A-B), 0 at a BP fixed
     * point: over every bond end at a site without open legs, the 2-norm of
     * the excited entries of the site's single-leg slice (the site tensor
     * with every other leg on its vacuum vector, over z'_v, in the excited
     * basis of Appendix B: an orthonormal basis of c^perp at the bond's
     * first site, Q^T of it at the second).  Read from the stored slices, so
     * in the term precision. */
    double dangling_max;
    /* First-order estimate of the error the term precision puts into the
     * result: with u the unit roundoff of the slices (2^-53, 2^-24, 2^-8),
     * v that of the term arithmetic (2^-53 in FP64 mode, else 2^-24), A_s the
     * sum of |w_c| over clusters of s bonds and A their total,
     *   E = (sum_s ((s + 1) u + s v) A_s) (1 + A)
     * (a term of s bonds multiplies at most s + 1 slices), reported as
     * E / |1 + S| for a closed network (an estimate of |delta ln|Z||) and
     * E / max|Out| for an open one (relative entry error).  It assumes no
     * cancellation inside a cluster's own index sum. */
    double term_err_est;
} pne_result;

typedef struct pne_ctx pne_ctx;
typedef struct pne_network pne_network;
typedef struct pne_batch pne_batch;
typedef struct pne_server pne_server;

/* Fill *opt with defaults: K=4, FP64, tol 1e-13, 500 sweeps, LOOP mode, no
 * damping, err_bound 1e-5. */
pne_status pne_options_default(pne_options *opt);

/* Create a context on HIP device `device`.  mem_budget_bytes bounds the
 * device memory the context may hold (0: no bound).  hip_stream is a
 * hipStream_t to enqueue on (NULL: the context creates its own stream).
 * Returns PNE_ERR_DEVICE if no device is usable. */
pne_status pne_ctx_create(int device, size_t mem_budget_bytes, void *hip_stream, pne_ctx **out);
/* Servers, batches and networks made on ctx must be destroyed first. */
pne_status pne_ctx_destroy(pne_ctx *ctx);
/* Message of the last failing call on ctx (never NULL; valid until the next call). */
const char *pne_last_error(const pne_ctx *ctx);

/* Validate desc and make a network object (Sec. II.A network definition).
 * data_on_device = 0: site_data are host pointers; the tensors are copied to
 * device memory owned by the network.  data_on_device = 1: site_data are
 * device pointers that the library borrows; the caller keeps them alive and
 * unchanged until pne_network_destroy.  Descriptor arrays are copied. */
pne_status pne_network_create(pne_ctx *ctx, const pne_network_desc *desc, int data_on_device,
                              pne_network **out);
pne_status pne_network_destroy(pne_network *net);

/* User partitions (Sec. II.A-C, Eqs. (4), (7), (9)-(11)).  Partition p transects
 * the bonds part_bond[part_begin[p] .. part_begin[p+1]) (part_begin has
 * n_partitions + 1 entries, part_begin[0] == 0); its projector is the product
 * of the rank-1 BP projectors of those bonds (Eq. (11)), so a multi-index
 * partition keeps its bonds together.  Bonds transected by no partition carry
 * the identity.  Partitions may share bonds.  n_partitions == 0 restores the
 * default (every bond expanded, degree cap only).
 *
 * Result of a network with partitions: the exact value minus the residue of
 * the linear or combinatorial form (both drop the same residue, the network
 * with Q_p on every partition), further restricted to configurations of at
 * most K excited bonds.  With K >= n_bonds (and K <= 32) it is exactly the
 * paper's partitioned expansion with the residue dropped; n_config_terms then
 * counts the retained loop configurations.  In the rank-1 BP gauge the
 * residue is the sum of the dangling-free configurations that excite at
 * least one bond of every partition (Eq. (10)), which is how the library
 * evaluates it: every retained configuration is listed at plan time, so the
 * envelope is small networks (at most 2^24 listed cluster entries).
 *
 * Closed networks only (open legs: PNE_ERR_UNSUPPORTED); 1 <= n_partitions
 * <= 32; every partition transects at least one bond, no bond twice.
 * Batches already created keep the partitions they were made with.  Arrays are
 * copied; the caller keeps ownership. */
pne_status pne_network_set_partitions(pne_network *net, int32_t n_partitions, const int32_t *part_begin,
                                      const int32_t *part_bond);

/* Recursive partitioning (Sec. IV.A).  The term of the first-level subset
 * x_mask (bit p: partition p inserts its P; a non-empty subset of the
 * partitions set above) is not contracted whole but expanded again, in the
 * combinatorial form, over its own sub-partitions (same layout as
 * pne_network_set_partitions); the sub-expansion drops its own residue.
 * Calling again for the same x_mask replaces its sub-partitions, n_sub == 0
 * removes them, and pne_network_set_partitions clears them all.  In the
 * library's evaluation a loop configuration then counts with an integer
 * coefficient: the signed number of first-level subsets that keep it (none
 * of their bonds excited, and, where refined, some sub-partition left
 * unexcited).  Same envelope as pne_network_set_partitions. */
pne_status pne_network_set_subpartitions(pne_network *net, uint32_t x_mask, int32_t n_sub,
                                         const int32_t *sub_begin, const int32_t *sub_bond);

/* Prepare a batch: enumerate (or fetch cached) retained clusters per network
 * geometry, build contraction plans and device tables, allocate the batch's
 * device working memory.  The networks must stay alive while the batch does. */
pne_status pne_batch_create(pne_ctx *ctx, pne_network *const *nets, int32_t n,
                            const pne_options *opt, pne_batch **out);
/* Enqueue the whole expansion for every network of the batch on the context
 * stream (BP sweeps, gauge, slices, cluster contractions, FP64 sum), followed
 * by the copy of its results to pinned host memory.  Up to two launches may
 * be outstanding (INVALID_ARG beyond that): the second is enqueued behind the
 * first and reuses the device buffers in stream order, so the host can
 * collect one launch's results while the next runs.  A batch with networks
 * swept launch by launch synchronises inside launch (convergence checks). */
pne_status pne_batch_launch(pne_batch *batch);
/* Wait for the oldest outstanding launch and fill results[0..n-1] (results
 * may be NULL).  The diagnostics below describe the launch last waited for
 * and are meaningful only when no other launch is outstanding. */
pne_status pne_batch_wait(pne_batch *batch, pne_result *results);
/* pne_batch_launch followed by pne_batch_wait. */
pne_status pne_batch_run(pne_batch *batch, pne_result *results);
pne_status pne_batch_destroy(pne_batch *batch);

/* One-shot forms: batch of one / batch of n, created, run and destroyed. */
pne_status pne_contract(pne_ctx *ctx, pne_network *net, const pne_options *opt, pne_result *res);
pne_status pne_contract_batch(pne_ctx *ctx, pne_network *const *nets, int32_t n,
                              const pne_options *opt, pne_result *results);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as pne_contract_batch, with every device table and buffer of the
 * batch placed in a fixed 64 MiB device array that the library holds on each
 * GPU it runs on until the process ends.  The call allocates no device or
 * pinned memory and creates no events (its host-side planning uses ordinary
 * host memory); results are copied to the caller's pne_result array and the
 * call returns after synchronising the context stream.  Networks are the
 * caller's inputs (made beforehand with pne_network_create).  Errors:
 * OUT_OF_MEMORY when the batch needs more than the array holds (16x16 D=4
 * networks need about 0.55 MB each with FP64 slices, 0.35 MB with FP32), INVALID_ARG for null arguments and for
 * PNE_FLAG_PROFILE / GRAPH / AUTOTUNE (they allocate), and every error of
 * pne_contract_batch.  Every call on a GPU shares that GPU's array, and the
 * array keeps the last call's contents: calls that overlap on one GPU (from
 * two threads, or on two contexts of one device) race and must not be made. */
pne_status pne_contract_batch_noalloc(pne_ctx *ctx, pne_network *const *nets, int32_t n,
                                      const pne_options *opt, pne_result *results);

/* --- introspection (parity tests and tooling) -------------------------- */

/* Host-only: list the retained clusters (connected bond sets of size <= K in
 * which every site has degree >= 2, sites with open legs >= 1) of a network
 * geometry.  With bonds == NULL only counts: *n_clusters and *n_entries.
 * Otherwise writes sizes[n_clusters] and bonds[n_entries] (each cluster's
 * bond ids ascending, clusters in the library's order). */
pne_status pne_enumerate_clusters(const pne_network_desc *desc, int32_t K, int64_t *n_clusters,
                                  int64_t *n_entries, int32_t *sizes, int32_t *bonds);

/* Host only (no device needed): the number of retained clusters and of
 * retained configurations (collections of vertex-disjoint clusters, the
 * empty one excluded) the library would evaluate for this geometry at degree
 * cap K in the given pne_mode, with the given partitions (n_partitions == 0:
 * none; same rules as pne_network_set_partitions; PNE_MODE_FULL takes none).
 * The counts equal pne_result's n_cluster_terms and n_config_terms. */
pne_status pne_count_configurations(const pne_network_desc *desc, int32_t K, int32_t mode, int32_t n_partitions,
                                    const int32_t *part_begin, const int32_t *part_bond, int64_t *n_clusters,
                                    int64_t *n_configs);

/* Autotune (Sec. II.D: the terms are evaluated in parallel; this picks how):
 * for the batch these networks and options would form, time the persistent
 * kernel's tile shapes (small_sites 64 or 256, tiles_in_flight by shape, 1 or
 * 2, reg_budget 0 or 1: twelve variants, eager launches), then graph replay of
 * the best when every network runs in the persistent kernel; `trials` runs
 * each after one warm-up run.  Variants that do not fit (LDS) are skipped.
 * *best receives the options with the fastest variant's tile options and
 * flags.  The choice is cached in the context per batch signature (multiset
 * of lattices, K, precision, mode, damping, BP flags): later calls and
 * batches created with PNE_FLAG_AUTOTUNE reuse it without running anything.
 * The variants agree to rounding (block size and the separate regauge order
 * sums differently; graph replay is bitwise the eager sequence).  The runs
 * use the context stream and block. */
pne_status pne_autotune(pne_ctx *ctx, pne_network *const *nets, int32_t n, const pne_options *opt, int32_t trials,
                        pne_options *best);
/* The context's tuning cache as a JSON file: {"pne_tune_cache": 1, "entries":
 * [{"signature": "<16 hex digits>", "flags", "small_sites",
 * "tiles_in_flight", "reg_budget", "ms", "default_ms"}, ...]} (ms: the chosen
 * and the default variant's run time when tuned).  Save writes every entry
 * (to path.tmp, then renamed); load adds or replaces entries and sets
 * *n_loaded (may be NULL).  INVALID_ARG for an unreadable or malformed file
 * (entries read before the error are kept).  Signatures hash lattice
 * geometries and options, not devices: a cache is meant for the machine that
 * wrote it. */
pne_status pne_tune_cache_save(pne_ctx *ctx, const char *path);
pne_status pne_tune_cache_load(pne_ctx *ctx, const char *path, int32_t *n_loaded);

/* Per-kernel device time accumulated over profiled runs (PNE_FLAG_PROFILE),
 * measured with HIP events recorded on the batch's stream around each launch.
 * Index k: 0 init, 1 BP sweep (per-launch), 2 BP close, 3 persistent BP
 * (both of its launches: large and small networks), 4 bond gauge (no
 * launches of its own: built inside the regauge kernels), 5 gauge + regauge
 * / slices, 6 cluster contraction, 7 combine.  A step with nothing to do for
 * a kernel launches nothing and counts nothing.  Writes n entries; reset != 0
 * clears the accumulators afterwards. */
pne_status pne_batch_kernel_times(pne_batch *batch, double *ms_total, int64_t *launches, int32_t n,
                                  int32_t reset);

/* After pne_batch_wait: phase durations of the persistent BP blocks of the
 * last run, from the device wall clock (microseconds): out[0] mean BP time per
 * block, out[1] mean in-block gauge + slice time, out[2] / out[3] their
 * maxima, out[4] span from the first block's start to the last BP end,
 * out[5] span to the last block's end.  Writes n entries (zeros when the
 * batch has no persistent networks). */
pne_status pne_batch_phase_times(pne_batch *batch, double *out, int32_t n);

/* Where each network of the batch runs (fixed at pne_batch_create): out[i]
 * has bit 0 set when its BP runs in a persistent block, bit 1 when that
 * block also builds its gauge and slices, bit 2 when it also contracts the
 * clusters and sums the terms (otherwise those steps have launches of their
 * own).  n must be the batch's network count. */
#define PNE_PATH_PERSISTENT 1
#define PNE_PATH_BLOCK_GAUGE 2
#define PNE_PATH_BLOCK_TERMS 4
pne_status pne_batch_paths(pne_batch *batch, int32_t *out, int32_t n);

/* After pne_batch_wait: copy network i's final BP messages to host.  For
 * every bond b, out holds the message arriving at the bond's first site
 * (dim d_b) followed by the message arriving at its second site; bonds in
 * order.  Capacity in doubles; returns INVALID_ARG if too small. */
pne_status pne_batch_messages(pne_batch *batch, int32_t i, double *out, int64_t capacity);
/* After pne_batch_wait: copy network i's cluster weights w_c (cluster order
 * of pne_enumerate_clusters; open clusters contribute their full tensors, so
 * *n_values may exceed the cluster count).  offsets[c] gives each cluster's
 * first value when offsets != NULL. */
pne_status pne_batch_cluster_weights(pne_batch *batch, int32_t i, double *out, int64_t capacity,
                                     int64_t *n_values, int64_t *offsets);

/* ------------------------------------------------------------------------
 * Request server (continuous batching of independent networks).
 *
 * Networks are independent work (terms of different networks never mix), so
 * a stream of requests is served by batching whatever has arrived: a worker
 * thread admits pending requests in arrival order while their estimated
 * device bytes fit mem_budget, runs requests with identical options as one
 * batch (the same kernels as pne_batch_*), and keeps up to pipeline_depth
 * batches in flight on their own streams so that preparing the next batch
 * overlaps the device work of the current one.  A request's tensors and
 * messages stay in device memory from admission to completion.  Its result
 * is the same as when it is contracted alone (same kernels, same per-network
 * reduction order).
 *
 * Ownership: pne_submit copies the descriptor arrays and the host tensors
 * (site_data must point to host memory); the caller may free them on return.
 * While a server exists, its worker thread is the only user of the context:
 * the caller must not use that context (or its networks and batches)
 * concurrently.  pne_submit, pne_poll and pne_server_get_stats may be called
 * from any thread.
 * ------------------------------------------------------------------------ */
typedef struct {
    size_t mem_budget;       /* device bytes admitted requests may hold (estimate); 0: no limit */
    int32_t max_batch;       /* networks per launch (default 1024) */
    int32_t pipeline_depth;  /* batches in flight, 1 or 2 (default 2) */
    int32_t completion_queue; /* 1: finished tickets are queued for pne_server_completed (default 0) */
    int32_t reserved[3];
} pne_server_options;

typedef struct {
    int64_t submitted, completed, failed, batches, pending;
    int64_t device_bytes_admitted;  /* estimate held by admitted requests now */
    double latency_p50_ms, latency_p99_ms, latency_mean_ms, latency_max_ms; /* submit -> result ready */
    double networks_per_s;          /* completed / (last completion - first submission) */
    double busy_s;                  /* wall time with at least one batch in flight */
    double prep_s;                  /* worker time creating networks / batches and launching */
    double wait_s;                  /* worker time blocked on batch completion */
    /* prep_s split: tensor staging and upload, network creation, batch
     * creation (tables, device arena), launch (which waits on the device
     * where a network's BP is swept launch by launch) */
    double upload_s, networks_s, batch_s, launch_s;
} pne_server_stats;

pne_status pne_server_options_default(pne_server_options *opt);
/* opt may be NULL (defaults).  Starts the worker thread on the calling
 * thread's current device. */
pne_status pne_server_create(pne_ctx *ctx, const pne_server_options *opt, pne_server **out);
/* Finishes every submitted request, then stops the worker. */
pne_status pne_server_destroy(pne_server *server);
/* Queue one network.  *ticket identifies it for pne_poll.  INVALID_ARG for
 * a malformed descriptor (further checks happen at admission and are
 * reported by pne_poll), OUT_OF_MEMORY if the request alone exceeds
 * mem_budget. */
pne_status pne_submit(pne_server *server, const pne_network_desc *desc, const pne_options *opt,
                      uint64_t *ticket);
/* PNE_ERR_NOT_READY while the request is pending or running.  Otherwise
 * fills *result (open values into result->open_values, capacity
 * result->open_capacity), returns the request's status and forgets the
 * ticket; with too small an open buffer it returns INVALID_ARG and keeps the
 * result for another poll. */
pne_status pne_poll(pne_server *server, uint64_t ticket, pne_result *result);
/* Cancels a request that is still queued (not yet admitted into a batch): it
 * leaves the queue and finishes at once with PNE_ERR_CANCELLED, which
 * pne_poll then returns (and pne_server_completed lists it; the statistics
 * count it as failed, outside the latencies).  PNE_ERR_NOT_READY when the
 * request is already admitted (it completes normally), INVALID_ARG for an
 * unknown or finished ticket. */
pne_status pne_cancel(pne_server *server, uint64_t ticket);
pne_status pne_server_get_stats(pne_server *server, pne_server_stats *out);
/* With completion_queue set: moves up to `capacity` tickets of finished
 * requests (success or failure), oldest first, into tickets[] and sets *n to
 * their count; a client then polls only those.  INVALID_ARG without the
 * option or with a NULL argument. */
pne_status pne_server_completed(pne_server *server, uint64_t *tickets, int32_t capacity, int32_t *n);

/* ------------------------------------------------------------------------
 * Strip expansion of an infinite, translation-invariant square lattice
 * (Sec. IV.C).  One tensor A repeats on every site; the result is the free
 * energy per site f = -lim ln Z_N / N.
 *
 * The lattice is expanded over width-L strip partitions: L vertical
 * partitions (every L-th column line at offsets 0..L-1, each transecting the
 * horizontal bonds that cross it) and, with two_d, L horizontal ones.  P on a
 * bond is the rank-1 projector of the uniform BP fixed point (Eq. (8), oblique
 * form, which includes 1 / (message overlap)).  Per unit cell (L x L sites,
 * or L sites of a row with vertical partitions only) the combinatorial form
 * (Eq. (7)) sums, over non-empty sets of partitions with sign + for an odd
 * count and - for an even one, the product of the pieces the partitions cut
 * the cell into:
 *   lam_k   leading eigenvalue of the width-k vertical transfer matrix (k
 *           sites in a row, the outer legs capped by the BP messages), over
 *           the horizontal bond overlap;
 *   gam_k   the same for width-k horizontal strips;
 *   Z_kp    the k-column, p-row patch with every outer leg capped, over
 *           n_v^k n_h^p;
 * strips of width g contribute lam_g per row (gam_g per column), patches
 * Z_(gv)(gh).  For L = 2 and vertical strips only this is
 * f = -ln(2 lam_2 - lam_1^2) / 2; with both directions it is the paper's
 * R_1 - R_2 + R_3 - R_4 form.
 *
 * Everything runs on the device: BP, power iteration of every transfer
 * matrix (k streaming passes per application over a chi^k vector), the
 * patches (the first L applications of the vertical iteration started from
 * the product of the top caps), and the cell sum.  Leading eigenvalues must
 * be real and dominant (positive tensors, for instance); a power iteration
 * that does not reach power_tol within power_max_iter steps gives the
 * warning status with its last estimate.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t L;              /* strip width, 1..16 (chi^(L+1) <= 2^28)                */
    int32_t two_d;          /* 1: vertical and horizontal strips; 0: vertical only  */
    double bp_tol;          /* BP stop: largest entry change (1e-14)                  */
    int32_t bp_max_iter;    /* BP sweep cap (10000)                                   */
    int32_t power_max_iter; /* power-iteration cap per strip (20000), >= L           */
    double power_tol;       /* stop when two successive relative changes of the
                               eigenvalue estimate are <= power_tol (1e-13)           */
    int32_t check_every;    /* iterations between host convergence checks (4)        */
    int32_t single_site_passes; /* 1: one site per pass over the vector; 0 (default):
                               two neighbouring sites per pass where chi <= 4        */
    int32_t reserved[2];
} pne_strip_options;

typedef struct {
    int32_t status;         /* pne_status; WARN_BP_NOT_CONVERGED also when a power
                               iteration hit its cap                                  */
    int32_t bp_iters;       /* BP sweeps                                              */
    double f;               /* free energy per site from the strip expansion         */
    double f_bp;            /* -ln(z / (n_h n_v)): the BP value per site              */
    double bp_residual;     /* last BP sweep's largest entry change                   */
    double cell_sum;        /* the per-cell sum, with every piece divided by the BP
                               value per site to the power of its site count          */
    int32_t power_iters;    /* power-iteration steps over all strips                  */
    int32_t n_unconverged;  /* strips whose power iteration hit the cap               */
    double *lam;            /* caller buffer [L] or NULL: lam_k / w_bp^k, k = 1..L   */
    double *gam;            /* caller buffer [L] or NULL (two_d): gam_k / w_bp^k     */
    double *patch;          /* caller buffer [L*L] or NULL (two_d): Z_kp / w_bp^(k p)
                               at [(k-1) L + (p-1)]                                   */
    int32_t *iters;         /* caller buffer [2*L] or NULL: power-iteration steps of
                               width k at [k-1] (vertical) and [L+k-1] (horizontal)  */
    int64_t reserved;
} pne_strip_result;

/* Defaults: L = 2, two_d = 1, tolerances and caps as listed above. */
pne_status pne_strip_options_default(pne_strip_options *opt);
/* A: host FP64 tensor, C order over (-x, +x, -y, +y), every leg of dimension
 * chi (2..6); copied.  res: filled; its lam/gam/patch buffers, when not
 * NULL, receive the per-width values.  Device memory: about
 * 16 (chi^L + chi^(L+1)) bytes, allocated and freed by the call; runs on the
 * context's stream and returns when done.  Errors: INVALID_ARG (null, L or
 * caps out of range, non-finite entry), UNSUPPORTED (chi, size),
 * OUT_OF_MEMORY, SINGULAR (BP value per site not positive, a zero bond
 * overlap, or a cell sum that is not positive). */
pne_status pne_strip_expand(pne_ctx *ctx, const double *A, int32_t chi, const pne_strip_options *opt,
                            pne_strip_result *res);

/* ------------------------------------------------------------------------
 * Rank-r projectors from weight passing (Sec. V, Appendix C), on batches of
 * small closed 2D lattices.
 *
 * Weight passing puts a diagonal weight S_b on every bond (initially 1) and
 * sweeps over the bonds: with A', B' the two site tensors with the weights of
 * their other bonds applied, A' = U_A S_A V_A^T (other legs x this leg),
 * B' = U_B S_B V_B^T (this leg x other legs), S_A V_A^T S_b U_B S_B =
 * U_C S_C V_C^T (Eqs. (C1), (C2)), the tensors take the gauge change of
 * Eq. (C3) and S_b becomes S_C^a (rescaled to a largest entry of 1, the
 * scale kept in log_scale).  a ramps linearly up to alpha over the first
 * ramp_sweeps sweeps; sweeps stop once no weight entry moves by more than tol.
 * In that gauge the weights decrease along each bond, and the rank-r
 * projector of a bond keeps its first r indices: P = diag(1_r, 0), Q = I - P.
 *
 * The expansion over the given partitions (bond lists) is the combinatorial
 * form (form 0, Eq. (7)) or the linear form (form 1, Eq. (4), single-index
 * partitions in the given order), the residue dropped; each term contracts
 * the gauged lattice exactly with S_b P, S_b Q or S_b on every bond.  With
 * r = chi every P is the identity and the result is the exact value.
 *
 * Envelope: every network in the call has the same geometry, a closed
 * Lx x Ly lattice with sites numbered x + Lx y, bonds between lattice
 * neighbours only, one bond dimension chi, Lx Ly <= 16, 1..16 partitions;
 * either chi <= 4 and chi^(Lx+1) <= 1024 (one wave per network), or
 * chi in {8, 16}, Lx >= 2, chi^(Lx-1) a multiple of 16 and
 * chi^(Lx+1) <= 65536 (a block per network for weight passing, the terms on
 * the FP64 matrix cores); anything else is UNSUPPORTED.  Networks are read in place (device
 * copies made by pne_network_create).  Device memory is allocated and freed
 * by the call; it returns when done.  Per network: status (SINGULAR when a
 * singular value vanished; WARN_BP_NOT_CONVERGED when weight passing hit
 * max_sweeps), sweeps, and (sign, ln|Z|).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t rank;        /* r, 1..chi (2)                                 */
    int32_t form;        /* 0: combinatorial (Eq. (7)); 1: linear (Eq. (4))  */
    double alpha;        /* weight exponent a (0.8)                        */
    int32_t ramp_sweeps; /* sweeps over which a ramps up to alpha (10)     */
    int32_t max_sweeps;  /* sweep cap (2000)                               */
    double tol;          /* largest weight change to stop (1e-12)          */
    int32_t profile;     /* != 0: time the phases (pne_rank_last_times) (0) */
    int32_t reserved[3];
} pne_rank_options;

typedef struct {
    int32_t status;      /* pne_status of the network                      */
    int32_t sweeps;      /* weight-passing sweeps                          */
    int32_t sign;        /* +1, -1 (0 if the sum is 0)                     */
    int32_t pad;
    double log_abs;      /* ln|Z| of the expansion                         */
    double log_scale;    /* the log-scale carried out of weight passing    */
} pne_rank_result;

pne_status pne_rank_options_default(pne_rank_options *opt);
/* nets[0..n-1]: the batch; Lx, Ly: the lattice shape; partitions as in
 * pne_network_set_partitions; results: n entries.  Returns the first
 * non-zero per-network status, or an argument error before any device work. */
pne_status pne_rank_expand(pne_ctx *ctx, pne_network *const *nets, int32_t n, int32_t Lx, int32_t Ly,
                           int32_t n_partitions, const int32_t *part_begin, const int32_t *part_bond,
                           const pne_rank_options *opt, pne_rank_result *results);

/* Device time of each phase of the last pne_rank_expand call on this context
 * that ran with opt->profile != 0, in milliseconds, from HIP events recorded
 * on the context stream between the launches: ms[0] gathering the site
 * tensors, ms[1] weight passing, ms[2] the dense site matrices (bond
 * dimension 8 and 16 only, else 0), ms[3] the expansion's terms, ms[4] their
 * signed sum.  Writes n <= 5 entries (INVALID_ARG otherwise); all zero when
 * the last call was not profiled or failed. */
pne_status pne_rank_last_times(pne_ctx *ctx, double *ms, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* PNE_H */
