/*
 * Plain CPU oracle for the HeatACO decode loop (heatmap-guided Max-Min Ant
 * System).  TEST INFRASTRUCTURE: only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code with the HIP
 * library; both are fed by the seeded input generators.
 *
 * Everything here is single-threaded FP64 (FP32 where the method stores
 * FP32 state), compiled without contraction or fast-math.
 */
#ifndef HAC_ORACLE_H
#define HAC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_COORDS = 0, ORC_MATRIX = 1 };

typedef struct {
  /* instance: coords [n][2] (Euclidean, symmetric) or dist [n][n] row-major */
  int32_t n, kind, symmetric;
  const double* coords;
  const double* dist;
  /* heatmap h as consumed, CSR */
  const int32_t* row_ptr;
  const int32_t* col;
  const float* val;
  /* MMAS / HeatACO parameters (Section IV-C).  local_search: 0 none, 1 2-opt
     on the iteration best, 2 2-opt on every ant's tour (Alg. 1); for the
     ATSP the directed 2-opt */
  int32_t ants, iterations, k, k_ls, local_search;
  double alpha, beta, rho, p_best, c_cap, theta_h, eps, xi_bf, lambda_bf, clip;
  int32_t degree_target, bf_period, restart_stall, ugb_max, baseline_scope;
  uint64_t seed;
  /* kappa_fixed < 0: kappa from eq. (14); >= 0: kappa set to this value
     (Sec. IV-E ablation "fixed kappa = 1") */
  double kappa_fixed;
  /* local-search operator (Section III-D): 0 or 2 the 2-opt, 3 the 3-opt
     (symmetric instances only) */
  int32_t ls_op;
} orc_problem;

/* optional outputs; any pointer may be NULL */
typedef struct {
  int32_t k_eff;
  double q90, r_hat, kappa, l_nn, l_nn_raw;
  int64_t ant_steps, fallback_steps;
  int32_t restarts;
  double* l_ib;        /* [iterations] iteration-best length (after LS)  */
  double* l_gb;        /* [iterations] global-best length after the iteration */
  int32_t* elite_rb;   /* [iterations] 1 if the restart-best tour deposited  */
  int32_t* cand;       /* [n*k_eff] candidate lists                          */
  float* heur;         /* [n*k_eff] folded eta^beta * e^kappa                */
  float* tau;          /* [n*k_eff] pheromone after the last iteration       */
  float* weight;       /* [n*k_eff] choice weights after the last iteration  */
  int32_t* ant_tours;  /* [ants*n] tours of the last iteration (after the    */
                       /* local search when local_search = 2)               */
  double* ant_len;     /* [ants] their lengths                               */
  int32_t* nn_tour;    /* [n] the (optionally 2-opted) NN tour               */
  int32_t* ugb;        /* [iterations] u_gb in force when iteration t chose   */
                       /* its elite tour                                     */
  int32_t* restart;    /* [iterations] 1 if a branching-factor restart ended */
                       /* iteration t                                        */
} orc_trace;

/* Philox4x32-10 block */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* 32-bit uniform for (seed, iteration t, ant a, step s) */
uint32_t orc_draw(uint64_t seed, uint32_t t, uint32_t a, uint32_t s);

/* Candidate lists (eq. 3): writes n*k_eff ids, returns k_eff or <0 on error */
int32_t orc_candidates(const orc_problem* p, int32_t* cand);
/* Geometric nearest-neighbour lists of size kk (for local search) */
int32_t orc_nearest_lists(const orc_problem* p, int32_t kk, int32_t* out);

/* Evidence (eq. 9-11), scale (eq. 12-14) and fold.  Inputs: candidates.
 * Outputs (each may be NULL): conf c [n*k], base b [n], evid e [n*k],
 * heur S [n*k]; returns kappa, and q90 / r_hat through pointers. */
double orc_evidence(const orc_problem* p, const int32_t* cand, int32_t k_eff, double* conf,
                    double* base, double* evid, float* heur, double* q90, double* r_hat);

/* One roulette decision: chooses among the unvisited slots of a row.
 * Returns the chosen slot, or -1 if every slot is visited. */
int32_t orc_select(int32_t k, const int32_t* cand_row, const float* w_row,
                   const uint8_t* visited, uint32_t u);

/* Nearest-neighbour tour from node 0 (Alg. 1 preparation); returns length */
double orc_nn_tour(const orc_problem* p, int32_t* tour);
/* Tour length, summed in array order with the closing edge last (eq. 1) */
double orc_tour_length(const orc_problem* p, const int32_t* tour);
/* First-improvement neighbour-list 2-opt with a don't-look queue. */
void orc_two_opt(const orc_problem* p, const int32_t* nl, int32_t kk, double min_gain,
                 int32_t* tour);
/* First-improvement neighbour-list 3-opt (the 2-opt moves, then segment
 * exchanges) with the same queue, for symmetric instances. */
void orc_three_opt(const orc_problem* p, const int32_t* nl, int32_t kk, double min_gain,
                   int32_t* tour);

/* Incoming neighbour lists of size kk: for node i the nodes j with the
 * smallest d(j, i) (the directed 2-opt's predecessor side) */
int32_t orc_nearest_in_lists(const orc_problem* p, int32_t kk, int32_t* out);
/* Directed 2-opt for the ATSP (Section III-D): first improvement over the
 * outgoing (successor side) and incoming (predecessor side) lists with a
 * don't-look queue; each move reverses a path and prices it in its new
 * direction. */
void orc_two_opt_directed(const orc_problem* p, const int32_t* nl_out, const int32_t* nl_in, int32_t kk,
                          double min_gain, int32_t* tour);
/* One directed 2-opt move (test hook): its gain as the directed 2-opt
 * computes it, and the tour after it in out; NAN for a degenerate move. */
double orc_directed_move(const orc_problem* p, const int32_t* tour, int32_t a, int32_t c, int32_t dir,
                         int32_t* out);

/* Whole decode (Alg. 1).  tour_out [n] canonical, len_out.  0 on success. */
int32_t orc_decode(const orc_problem* p, int32_t* tour_out, double* len_out, orc_trace* tr);

/* Heatmap diagnostics against a known tour (Section V):
 *   out[0] Edges/n: directed heatmap entries h_ij > theta_h (i != j) over 2n
 *   out[1] coverage: share of the known tour's n edges among those entries
 *          (an undirected edge counts if either direction is present; ATSP
 *          edges are directed)
 *   out[2] Miss%: 100 (1 - coverage)
 *   out[3] P(e>1): share of the candidate slots with e > 1 (eq. 11) whose
 *          edge is on the known tour (0 when no slot has e > 1)
 *   counts[0] entries, counts[1] slots with e > 1, counts[2] those on the tour
 * Returns 0, or -1 on invalid input (tour not a permutation, n < 2). */
int32_t orc_diagnostics(const orc_problem* p, const int32_t* tour, double out[4], int64_t counts[3]);

#ifdef __cplusplus
}
#endif
#endif
