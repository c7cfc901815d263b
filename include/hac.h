/*
 * hac.h -- C ABI of the MI355X heatmap-guided Max-Min Ant System decoder.
 *
 * The library decodes a travelling-salesman instance (symmetric TSP from
 * 2-D coordinates or a distance matrix, or the asymmetric TSP from a
 * matrix) together with a fixed edge-confidence heatmap into a tour, as
 * HeatACO does: g(H, D) -> feasible tour (Section II-B and Alg. 1 of the
 * paper).  Every step of the search runs in HIP kernels on one gfx950 GPU:
 * candidate lists (eq. 3), nearest-neighbour tour and pheromone bounds
 * (eq. 5-6), ant construction by eq. (4) with the nearest-unvisited
 * fallback (Alg. 2), the bounded pheromone update (eq. 7-8), the u_gb elite
 * schedule and the branching-factor restart (Section III-B), and
 * neighbour-list 2-opt (Section III-D).  The evidence factor and its scale
 * (eq. 9-14) are folded into FP32 heuristic weights on the host once per
 * instance, with the C library's exp/log, so that no transcendental
 * function is evaluated on the GPU.
 *
 * Determinism: a decode is a pure function of (instance, heatmap, params,
 * seed).  The plain, batched and served paths return identical tours and
 * lengths, bit for bit, whatever the launch configuration.
 *
 * Conventions for every call:
 *  - All pointers in hac_instance / hac_csr are host pointers unless the
 *    call's name ends in _dev.  Inputs are read-only, owned by the caller,
 *    and no longer referenced after the call returns.
 *  - Outputs are caller-allocated and are left untouched on any error.
 *  - No exception or abort crosses the ABI; every failure is a status code,
 *    with detail text from hac_last_error().
 *  - A hac_ctx is not re-entrant: use one per host thread.  A hac_server
 *    may be used from several threads.
 */
#ifndef HAC_H
#define HAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hac_status;
#define HAC_OK 0
#define HAC_EINVAL (-1)       /* malformed instance, heatmap or parameters   */
#define HAC_ENOMEM (-2)       /* device memory or budget cannot hold it      */
#define HAC_EDEVICE (-3)      /* a HIP call or a kernel's own check failed   */
#define HAC_EUNSUPPORTED (-4) /* valid for the method, not for this library  */
#define HAC_EBUSY (-5)        /* a served request is not finished yet        */
#define HAC_ECANCELLED (-6)   /* a served request was cancelled              */
#define HAC_ERANGE (-7)       /* weights would leave the FP32 normal range   */

#define HAC_COORDS_EUC2D 0 /* coords[n][2], d_ij = sqrt(dx^2 + dy^2) (FP64) */
#define HAC_MATRIX 1       /* dist[n][n] row-major, d_ij = dist[i*n + j]    */

/* Limits of this library (HAC_EUNSUPPORTED above them). */
#define HAC_MAX_K 64     /* construction candidates per node               */
#define HAC_MAX_KLS 32   /* local-search neighbours per node               */
#define HAC_MAX_N 1000000

/* The instance of Section II-A.  kind = HAC_COORDS_EUC2D implies a
 * symmetric instance; with HAC_MATRIX, symmetric = 1 requires
 * dist[i*n+j] == dist[j*n+i] exactly, symmetric = 0 is the ATSP. */
typedef struct hac_instance {
  int32_t n;
  int32_t kind;
  int32_t symmetric;
  const double* coords; /* [n][2] for HAC_COORDS_EUC2D, else NULL */
  const double* dist;   /* [n][n] for HAC_MATRIX, else NULL       */
} hac_instance;

/* The heatmap entries h_ij the decoder consumes (eq. 2): for a symmetric
 * instance the caller passes the already symmetrised (H + H^T)/2 or any
 * other symmetric or asymmetric confidence; for the ATSP the directed H.
 * CSR: row_ptr[n+1] monotone with row_ptr[0] = 0 and row_ptr[n] = nnz,
 * col[nnz] in [0, n) without duplicates inside a row, val[nnz] finite and
 * >= 0.  Absent entries are 0.  Diagonal entries are ignored. */
typedef struct hac_csr {
  int32_t n;
  int32_t nnz;
  const int32_t* row_ptr;
  const int32_t* col;
  const float* val;
} hac_csr;

/* Parameters (Section IV-C; hac_params_default fills them). */
typedef struct hac_params {
  int32_t ants;         /* m, ants per iteration                            */
  int32_t iterations;   /* I                                                */
  int32_t k;            /* candidate-list size (eq. 3), <= HAC_MAX_K        */
  int32_t k_ls;         /* local-search neighbour-list size, <= HAC_MAX_KLS */
  int32_t local_search; /* 0 none; 1 local search (ls_op: the 2-opt or   */
                        /* the 3-opt; the directed 2-opt on an ATSP) on    */
                        /* each iteration-best tour; 2 on every ant's tour */
                        /* (Alg. 1), the iteration best then taken among   */
                        /* the improved tours                              */
  double alpha;         /* pheromone exponent; only 1 is supported          */
  double beta;          /* heuristic exponent                               */
  double rho;           /* evaporation rate, in (0, 1)                      */
  double p_best;        /* for tau_min without local search (eq. 6)         */
  double c_cap;         /* evidence cap factor (eq. 14)                     */
  double theta_h;       /* heatmap threshold (eq. 3, 9)                     */
  double eps;           /* confidence floor (eq. 10-11)                     */
  double xi_bf;         /* branching-factor band fraction                   */
  double lambda_bf;     /* branching-factor restart threshold               */
  double clip;          /* clip of the log-weight kappa * log e             */
  int32_t degree_target;  /* d*: 0 = automatic (2 symmetric, 1 ATSP)       */
  int32_t bf_period;      /* iterations between branching-factor checks    */
  int32_t restart_stall;  /* restart only after more stalled iterations    */
  int32_t ugb_max;        /* first tier of the u_gb schedule               */
  int32_t baseline_scope; /* eq. (10) row: 0 candidate row, 1 heatmap row  */
  double kappa_fixed;     /* < 0: kappa from eq. (14); >= 0: kappa is this */
                          /* value (the fixed-scale ablation of Sec. IV-E  */
                          /* uses 1; 0 gives plain MMAS weights)           */
  int32_t ls_op;          /* local-search operator (Sec. III-D): 2 (or 0)  */
                          /* the 2-opt, 3 the 3-opt (the 2-opt moves, then */
                          /* segment exchanges); symmetric instances only, */
                          /* HAC_EUNSUPPORTED on an asymmetric matrix      */
} hac_params;

typedef struct hac_ctx hac_ctx;
typedef struct hac_server hac_server;

/* What the last decode call did (whole call, host wall clock). */
typedef struct hac_stats {
  double total_ms;       /* the whole call                                 */
  double prep_ms;        /* inputs up to the first iteration               */
  double search_ms;      /* the iterations                                 */
  double construct_ms;   /* summed construction-kernel time (HIP events);  */
                         /* only when timing is enabled, else 0            */
  int64_t construct_launches;
  int64_t ant_steps;       /* sum over instances of m (n-1) I               */
  int64_t fallback_steps;  /* steps that took the nearest-unvisited node    */
  int32_t restarts;        /* branching-factor restarts                     */
  int32_t instances;
  double kappa, q90, r_hat, l_nn; /* of the first instance of the call     */
  int32_t ants_per_block;         /* construction launch shape used         */
  int32_t lds_staged;             /* candidate table: 0 read from global    */
                                  /* memory; staged in LDS as 1 8-byte      */
                                  /* {id, weight} entries, 2 uint16 ids and */
                                  /* FP32 weights, 3 the same without the   */
                                  /* coordinates                            */
  int32_t ants_per_wave;          /* 1-4 ants per wave, 16 lanes each       */
  int32_t byte_marks;             /* 1: visited marks are bytes, 0: bits    */
  /* with timing enabled, as construct_ms / construct_launches: summed      */
  /* HIP-event times and launch counts of the 2-opt kernel (local search)   */
  /* and of the end-of-iteration kernel (control + pheromone update)        */
  double local_search_ms;
  int64_t local_search_launches;
  double update_ms;
  int64_t update_launches;
  int32_t geo_mode;  /* construction: how an exhausted row consults its     */
                     /* geometric list before a scan: 0 not at all, 1 int32 */
                     /* lists loaded every step, 2 uint16 lists a step ahead */
} hac_stats;

/* Fills the paper's settings (Section IV-C): m = 32, I = 5000, k = 20,
 * k_ls = 20, alpha = 1, beta = 2, q0 = 0, theta_h = 1e-4, eps = 1e-9,
 * c_cap = 0.5, branching check every 100 iterations with xi = 0.05 and
 * lambda = 1 + 1e-5, restart after > 250 stalled iterations, p_best = 0.05,
 * u_gb from 25.  rho is set to 0.2 (the paper uses 0.8 for the symmetric
 * TSP and 0.2 for the ATSP; set it per instance kind as needed). */
void hac_params_default(hac_params* p);

/* Static text for a status code. */
const char* hac_strerror(hac_status s);

/* Host-only check of an instance, heatmap and parameters, the same checks
 * every decode call makes first.  Touches no device.  HAC_OK, HAC_EINVAL or
 * HAC_EUNSUPPORTED. */
hac_status hac_validate(const hac_instance* inst, const hac_csr* heat, const hac_params* p);

/* Creates a context on HIP device `device`.  `stream` is a hipStream_t to
 * run on, or NULL for a stream the context creates and owns.
 * `hbm_budget_bytes` caps the device memory the context may hold (0 = no
 * cap).  The context owns all device memory it allocates. */
hac_status hac_create(hac_ctx** out, int32_t device, void* stream, uint64_t hbm_budget_bytes);
void hac_destroy(hac_ctx* ctx);
/* Detail text of the last failure on this context ("" if none). */
const char* hac_last_error(const hac_ctx* ctx);
/* 1 enables per-kernel HIP-event timing of the construction, 2-opt and
 * end-of-iteration kernels (hac_stats); the iterations then run as
 * separate launches instead of a replayed graph, which adds a few
 * microseconds per iteration.  0 disables it (default). */
hac_status hac_set_timing(hac_ctx* ctx, int32_t enable);

/* Decodes one instance (the plain path: one instance per launch
 * sequence).  tour_out[n] receives the best tour found, rotated to start
 * at node 0 and, for symmetric instances, oriented so that tour_out[1] <
 * tour_out[n-1]; length_out its length (eq. 1), summed in the order the
 * tour was built.  seed keys the per-ant random streams. */
hac_status hac_decode(hac_ctx* ctx, const hac_instance* inst, const hac_csr* heat,
                      const hac_params* p, uint64_t seed, int32_t* tour_out, double* length_out);

/* As hac_decode, with instance and heatmap arrays in device memory and the
 * results written to device memory (tour_out_dev int32[n],
 * length_out_dev double[1]).  The call is synchronous with respect to the
 * context's stream. */
hac_status hac_decode_dev(hac_ctx* ctx, const hac_instance* inst_dev, const hac_csr* heat_dev,
                          const hac_params* p, uint64_t seed, int32_t* tour_out_dev,
                          double* length_out_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * decode as hac_decode, with the same arguments, result and errors, but
 * every device buffer it uses (the instance's inputs, candidate lists,
 * pheromone and weights, ant tours, search state and launch tables) is
 * carved from one array of HAC_NOALLOC_BYTES that the library holds on each
 * GPU for the life of the process; the call allocates nothing and frees
 * nothing.  The launch shape is the tuner's cached choice for the
 * instance's shape class, else a fixed one (no timing launches), and the
 * iterations run as plain launches.  HAC_ENOMEM, with the byte count in
 * hac_last_error, if the instance needs more than the array holds (a
 * 10 000-node instance with 100 ants and 2-opt needs about 15 MB).
 * Calls on one GPU share its array, which keeps the last call's contents:
 * every buffer is written before it is read, and calls that would overlap
 * on one GPU (several threads or contexts) are serialised by a lock per
 * device, since they would otherwise race on the array.  The context's
 * stream and timing setting are used as by hac_decode (timing is ignored);
 * hac_debug_state and hac_debug_trace after such a call read the shared
 * array. */
#define HAC_NOALLOC_BYTES ((uint64_t)64 << 20)
hac_status hac_decode_noalloc(hac_ctx* ctx, const hac_instance* inst, const hac_csr* heat,
                              const hac_params* p, uint64_t seed, int32_t* tour_out,
                              double* length_out);

/* Decodes `count` independent instances of any sizes together (the
 * batched path): all instances' ants are constructed in shared launches,
 * with launch shapes chosen by the autotuner.  params[i], seeds[i] and
 * tours_out[i] (int32[n_i]) belong to instance i.  Every instance's result
 * is identical to hac_decode of that instance alone. */
hac_status hac_decode_batch(hac_ctx* ctx, int32_t count, const hac_instance* insts,
                            const hac_csr* heats, const hac_params* params, const uint64_t* seeds,
                            int32_t* const* tours_out, double* lengths_out);

/* As hac_decode_batch with every input array (coords/dist, row_ptr, col,
 * val) in device memory and the results written to device memory
 * (tours_out_dev[i] int32[n_i], lengths_out_dev double[count]).  The
 * instance and CSR structs themselves, params, seeds and the pointer
 * array tours_out_dev are host memory.  Validation and the evidence fold
 * read copies of the inputs on the host; the slots are filled
 * device-to-device.  Synchronous with respect to the context's stream. */
hac_status hac_decode_batch_dev(hac_ctx* ctx, int32_t count, const hac_instance* insts_dev,
                                const hac_csr* heats_dev, const hac_params* params,
                                const uint64_t* seeds, int32_t* const* tours_out_dev,
                                double* lengths_out_dev);

hac_status hac_last_stats(const hac_ctx* ctx, hac_stats* out);

/* Heatmap diagnostics against a known tour (Section V): how dense the
 * thresholded heatmap is, whether it holds the known tour's edges, and how
 * many of the candidate edges that eq. (11) marks with evidence (e > 1) lie
 * on that tour.  The candidate lists and the evidence are those a decode
 * with these parameters builds (the candidate kernel on the device, the
 * fold of eq. (9)-(11)); no iteration runs.
 *   edges_per_node  directed entries with h_ij > theta_h, i != j, over 2n
 *   coverage        share of the known tour's n edges present among them;
 *                   for a symmetric instance an edge counts if either
 *                   direction is present, for the ATSP the tour's direction
 *   miss_pct        100 (1 - coverage)
 *   p_evidence      share of candidate slots with e > 1 whose edge is on
 *                   the known tour (either tour neighbour for a symmetric
 *                   instance, the successor for the ATSP); 0 if none
 * Inputs are host pointers, read only; known_tour is int32[n], a
 * permutation of 0..n-1.  Errors: HAC_EINVAL (null argument, n < 2, a tour
 * that is not a permutation, or any decode input error), HAC_ERANGE as for
 * a decode; *out is untouched on error. */
typedef struct hac_diagnostics {
  double edges_per_node;
  double coverage;
  double miss_pct;
  double p_evidence;
  int64_t heatmap_edges;    /* directed entries above theta_h                 */
  int64_t evidence_slots;   /* candidate slots with e > 1                    */
  int64_t evidence_on_tour; /* those on the known tour                       */
} hac_diagnostics;

hac_status hac_heatmap_diagnostics(hac_ctx* ctx, const hac_instance* inst, const hac_csr* heat,
                                   const hac_params* params, const int32_t* known_tour,
                                   hac_diagnostics* out);

/* Test/inspection hook: after a decode, copies the final state of instance
 * `which` of the last call: candidate lists int32[n][k'], folded heuristic
 * float[n][k'], pheromone float[n][k'], choice weights float[n][k'], the
 * last iteration's ant tours int32[m][n] and lengths double[m], and the
 * (2-opted) NN tour int32[n] (k' = min(k, n-1)).  NULL skips an array. */
hac_status hac_debug_state(hac_ctx* ctx, int32_t which, int32_t* cand, float* heur, float* tau,
                           float* weight, int32_t* ant_tours, double* ant_len, int32_t* nn_tour);

/* Test/inspection hook: per-iteration trace of instance `which` of the
 * last call: iteration-best length, global-best length after the
 * iteration, and whether the restart-best tour deposited (each [I]). */
hac_status hac_debug_trace(hac_ctx* ctx, int32_t which, double* l_ib, double* l_gb,
                           int32_t* elite_rb);

/* ---- continuous-batching request loop ----------------------------------
 * A server owns a device memory budget and a number of instance slots.
 * Submitted requests are queued by size class of n (below 768, below 4096,
 * larger).  Each class has a loop thread and a stream of its own: it
 * admits the class's requests while a slot is free (slots go to requests
 * in arrival order across the classes) and the request's device footprint
 * fits in the free budget, and advances the class's admitted instances
 * together, iteration by iteration, so that requests arriving while others
 * run join the running batch, and the classes run concurrently on the
 * device.  Each
 * instance's pheromone, candidate lists and best tours stay on the device
 * from admission to completion.  Results equal hac_decode's. */

/* Device bytes one request holds while admitted: its inputs, candidate
 * lists, heuristic, pheromone and weights, ant tours and best tours. */
uint64_t hac_footprint(const hac_instance* inst, const hac_csr* heat, const hac_params* p);

/* The server runs its smallest size class on ctx's stream and two streams
 * of its own for the others; ctx must outlive it, and calls on ctx while
 * the server runs share that stream.  HIP's default of four hardware
 * queues per process then holds the three classes and the null stream. */
hac_status hac_server_create(hac_ctx* ctx, uint64_t budget_bytes, int32_t max_slots,
                             hac_server** out);
/* Queues a request.  Inputs are copied before return.  HAC_ENOMEM if the
 * request can never fit the budget. */
hac_status hac_server_submit(hac_server* srv, const hac_instance* inst, const hac_csr* heat,
                             const hac_params* p, uint64_t seed, uint64_t* ticket);
/* HAC_OK and the result if done (then the ticket is released), HAC_EBUSY
 * if not yet, HAC_ECANCELLED, or the request's own error status.
 * latency_s = completion time - submission time. */
hac_status hac_server_poll(hac_server* srv, uint64_t ticket, int32_t* tour_out,
                           double* length_out, double* latency_s);
/* Blocks until the request is done, then as hac_server_poll. */
hac_status hac_server_wait(hac_server* srv, uint64_t ticket, int32_t* tour_out,
                           double* length_out, double* latency_s);
/* Cancels a queued or running request. */
hac_status hac_server_cancel(hac_server* srv, uint64_t ticket);
/* Counters: requests admitted, completed, peak concurrent slots, peak bytes. */
hac_status hac_server_counters(hac_server* srv, int64_t* admitted, int64_t* completed,
                               int32_t* peak_slots, uint64_t* peak_bytes);
/* Per-lane figures of a server (lane 0, 1, 2: n below 768, below 4096,
 * larger), counted since hac_server_create.  Wall-clock times of the
 * lane's loop thread: prep_ms preparing admitted instances (uploads,
 * candidate lists, fold, NN tour), round_ms running rounds of iterations
 * up to their completion on the device, idle_ms waiting for work.
 * instance_iterations sums the admitted instances over every iteration
 * the lane ran. */
typedef struct hac_lane_stats {
  int32_t min_n, max_n;        /* the lane's size class, max_n exclusive (0: none) */
  int64_t admitted, completed; /* requests                                  */
  int64_t rounds, iterations, instance_iterations;
  int32_t peak_active;         /* most instances held at once               */
  double prep_ms, round_ms, idle_ms;
} hac_lane_stats;
#define HAC_SERVER_LANES 3
/* HAC_EINVAL for a lane outside 0 .. HAC_SERVER_LANES - 1. */
hac_status hac_server_lane_stats(hac_server* srv, int32_t lane, hac_lane_stats* out);
/* Stops the loop (cancelling what is left) and frees the server. */
void hac_server_destroy(hac_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* HAC_H */
