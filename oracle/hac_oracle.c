/*
 * Plain CPU oracle for the HeatACO decode loop (heatmap-guided Max-Min Ant
 * System for the TSP and the ATSP).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg are the only callers.  The product (the HIP library)
 * never links, loads or calls this file, and the two share no code.
 *
 * It is deliberately slow and literal: one thread, no blocking, no
 * vectorisation, FP64 unless the method keeps FP32 state.  Each function
 * names the passage of the paper it follows:
 *
 *   Section II-A, eq. (1)          tour length
 *   Section III-A, eq. (3)         candidate lists
 *   Section III-A, eq. (4), Alg. 2 ant construction, nearest-unvisited fallback
 *   Section III-B, eq. (5)-(8)     NN tour, pheromone bounds, bounded update,
 *                                  elite schedule, branching-factor restart
 *   Section III-C, eq. (9)-(14)    evidence factor and its scale kappa
 *   Section III-D                  neighbour-list 2-opt with don't-look bits
 *   Alg. 1                         the decode loop
 *
 * Where the paper leaves a detail open, the reading taken is stated at the
 * spot (candidate order, quantile rule, clip constant, start node, elite
 * choice, branching-factor normalisation, u_gb schedule, fixed-point
 * roulette, RNG, summation order, 2-opt move order).
 *
 * Parity status: every function is pinned by the CPU tests, the elite
 * choice and the shape of the u_gb schedule by the properties Section III-B
 * states.  Two readings no passage of the paper can pin: the u_gb tier
 * values with their stall thresholds, and the branching-factor
 * normalisation.  For those the oracle is "parity unpinned" against the
 * paper.
 */
#include "hac_oracle.h"

#include <float.h>
#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Ten rounds of two 32x32->64 multiplies, with    */
/* the key bumped by the Weyl constants between rounds.                      */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Each ant has its own stream (Section IV-C).  Reading: counter-based,
 * counter = (step s, ant a, iteration t, 0), key = the 64-bit seed; the
 * uniform is the first 32-bit output word. */
uint32_t orc_draw(uint64_t seed, uint32_t t, uint32_t a, uint32_t s) {
  uint32_t ctr[4] = {s, a, t, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return out[0];
}

/* floor(u * y / 2^32) for a 32-bit uniform u */
static uint64_t scale32(uint32_t u, uint64_t y) {
  return (uint64_t)(((unsigned __int128)u * (unsigned __int128)y) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Distances.  Coordinates: d_ij = sqrt(dx^2 + dy^2) in FP64; "nearest" is    */
/* decided on the squared distance, ties broken towards the lower index.     */
/* Matrix: d_ij as given, and the order key is d_ij itself.                   */
/* ------------------------------------------------------------------------ */
static double order_key(const orc_problem* p, int32_t i, int32_t j) {
  if (p->kind == ORC_COORDS) {
    double dx = p->coords[2 * i] - p->coords[2 * j];
    double dy = p->coords[2 * i + 1] - p->coords[2 * j + 1];
    return dx * dx + dy * dy;
  }
  return p->dist[(int64_t)i * p->n + j];
}

static double dist(const orc_problem* p, int32_t i, int32_t j) {
  if (p->kind == ORC_COORDS) return sqrt(order_key(p, i, j));
  return p->dist[(int64_t)i * p->n + j];
}

/* (key_a, a) < (key_b, b) */
static int closer(double ka, int32_t a, double kb, int32_t b) {
  return ka < kb || (ka == kb && a < b);
}

/* Eq. (1): sum of the n edges in array order, the closing edge last. */
double orc_tour_length(const orc_problem* p, const int32_t* tour) {
  int32_t n = p->n;
  if (n <= 1) return 0.0;
  double len = 0.0;
  for (int32_t s = 0; s + 1 < n; s++) len += dist(p, tour[s], tour[s + 1]);
  len += dist(p, tour[n - 1], tour[0]);
  return len;
}

/* Keep the `kk` smallest (key, j) seen so far in ascending order. */
typedef struct {
  int32_t kk, size;
  double* key;
  int32_t* id;
} topk_t;

static void topk_offer(topk_t* t, double key, int32_t j) {
  if (t->size == t->kk && !closer(key, j, t->key[t->size - 1], t->id[t->size - 1])) return;
  int32_t pos = t->size < t->kk ? t->size : t->kk - 1;
  while (pos > 0 && closer(key, j, t->key[pos - 1], t->id[pos - 1])) {
    t->key[pos] = t->key[pos - 1];
    t->id[pos] = t->id[pos - 1];
    pos--;
  }
  t->key[pos] = key;
  t->id[pos] = j;
  if (t->size < t->kk) t->size++;
}

/* ------------------------------------------------------------------------ */
/* Section III-A, eq. (3): candidate lists.                                  */
/* P_i = { j != i : h_ij > theta_h }.  With k' = min(k, n-1): if |P_i| >= k'  */
/* keep the k' members of P_i closest to i, else keep all of P_i and fill     */
/* with the nearest nodes outside P_i.                                        */
/* Reading: the list is stored in ascending (distance, index) order, which    */
/* fixes the slot order the roulette walks; the threshold compares the FP32   */
/* heatmap value widened to FP64; diagonal entries are ignored.               */
/* ------------------------------------------------------------------------ */
int32_t orc_candidates(const orc_problem* p, int32_t* cand) {
  int32_t n = p->n;
  int32_t k_eff = p->k < n - 1 ? p->k : n - 1;
  if (k_eff < 1) return 0;
  uint8_t* member = (uint8_t*)calloc((size_t)n, 1);
  topk_t sup = {k_eff, 0, (double*)malloc(sizeof(double) * k_eff), (int32_t*)malloc(4 * k_eff)};
  topk_t fill = {k_eff, 0, (double*)malloc(sizeof(double) * k_eff), (int32_t*)malloc(4 * k_eff)};
  double* mk = (double*)malloc(sizeof(double) * k_eff);
  int32_t* mj = (int32_t*)malloc(4 * k_eff);
  for (int32_t i = 0; i < n; i++) {
    sup.size = 0;
    fill.size = 0;
    int32_t np_i = 0;
    for (int32_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; e++) {
      int32_t j = p->col[e];
      if (j == i) continue;
      if ((double)p->val[e] > p->theta_h) {
        member[j] = 1;
        np_i++;
        topk_offer(&sup, order_key(p, i, j), j);
      }
    }
    if (np_i < k_eff) {
      for (int32_t j = 0; j < n; j++)
        if (j != i && !member[j]) topk_offer(&fill, order_key(p, i, j), j);
    }
    /* merge the two ascending lists: all of `sup` plus the first
       k_eff - |sup| of `fill` (the union is then sorted by (key, j)) */
    int32_t need = k_eff - sup.size, a = 0, b = 0, o = 0;
    for (int32_t q = 0; q < sup.size; q++) { mk[q] = sup.key[q]; mj[q] = sup.id[q]; }
    while (o < k_eff) {
      int take_sup;
      if (a >= sup.size) take_sup = 0;
      else if (b >= need) take_sup = 1;
      else take_sup = closer(mk[a], mj[a], fill.key[b], fill.id[b]);
      cand[(int64_t)i * k_eff + o] = take_sup ? mj[a++] : fill.id[b++];
      o++;
    }
    for (int32_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; e++) member[p->col[e]] = 0;
  }
  free(member); free(sup.key); free(sup.id); free(fill.key); free(fill.id); free(mk); free(mj);
  return k_eff;
}

/* Section III-D: geometric nearest-neighbour lists, independent of the
 * heatmap, ascending (distance, index). */
int32_t orc_nearest_lists(const orc_problem* p, int32_t kk, int32_t* out) {
  int32_t n = p->n;
  if (kk > n - 1) kk = n - 1;
  if (kk < 1) return 0;
  topk_t t = {kk, 0, (double*)malloc(sizeof(double) * kk), (int32_t*)malloc(4 * kk)};
  for (int32_t i = 0; i < n; i++) {
    t.size = 0;
    for (int32_t j = 0; j < n; j++)
      if (j != i) topk_offer(&t, order_key(p, i, j), j);
    for (int32_t q = 0; q < kk; q++) out[(int64_t)i * kk + q] = t.id[q];
  }
  free(t.key); free(t.id);
  return kk;
}

/* Incoming neighbour lists (matrix instances, for the directed 2-opt): for
 * node i the kk nodes j with the smallest d(j, i), ties to the lower index. */
int32_t orc_nearest_in_lists(const orc_problem* p, int32_t kk, int32_t* out) {
  int32_t n = p->n;
  if (kk > n - 1) kk = n - 1;
  if (kk < 1) return 0;
  topk_t t = {kk, 0, (double*)malloc(sizeof(double) * kk), (int32_t*)malloc(4 * kk)};
  for (int32_t i = 0; i < n; i++) {
    t.size = 0;
    for (int32_t j = 0; j < n; j++)
      if (j != i) topk_offer(&t, dist(p, j, i), j);
    for (int32_t q = 0; q < kk; q++) out[(int64_t)i * kk + q] = t.id[q];
  }
  free(t.key); free(t.id);
  return kk;
}

static int cmp_desc(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x < y) - (x > y);
}
static int cmp_asc(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

static int32_t degree_target(const orc_problem* p) {
  if (p->degree_target > 0) return p->degree_target;
  return (p->kind == ORC_COORDS || p->symmetric) ? 2 : 1;
}

static int is_sym(const orc_problem* p) { return p->kind == ORC_COORDS || p->symmetric; }

/* heatmap entry h_ij, or 0 when absent from row i */
static double heat(const orc_problem* p, int32_t i, int32_t j) {
  for (int32_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; e++)
    if (p->col[e] == j) return (double)p->val[e];
  return 0.0;
}

/* eta^beta: an integral beta is applied by repeated multiplication */
static double eta_pow(double eta, double beta) {
  if (beta == floor(beta) && beta >= 0.0 && beta <= 64.0) {
    double r = 1.0;
    for (int b = 0; b < (int)beta; b++) r = r * eta;
    return r;
  }
  return pow(eta, beta);
}

/* p_x = p_best^(1/n) (eq. 6) */
static double p_x(const orc_problem* p) { return pow(p->p_best, 1.0 / (double)p->n); }

/* Eq. (13) with eq. (5)/(6): R = tau_max / tau_min.  Both bounds scale with
 * 1/L, so the ratio does not depend on the tour length: 2n with local
 * search, ((k-1)/2) p_x / (1 - p_x) without. */
static double r_hat(const orc_problem* p, int32_t k_eff) {
  if (p->local_search) return 2.0 * (double)p->n;
  double px = p_x(p);
  return (((double)(k_eff - 1) / 2.0) * px) / (1.0 - px);
}

/* ------------------------------------------------------------------------ */
/* Section III-C: degree-aware evidence.                                     */
/*  eq. (9)  c_ij = h_ij if h_ij > theta_h else 0, for j in C_i              */
/*  eq. (10) b_i = max(c_i^(d*+1), eps), missing order statistics are 0      */
/*  eq. (11) e_ij = max(max(c_ij, eps) / b_i, 1)                             */
/*  eq. (12) q90 = 0.9-quantile of { log e_ij : e_ij > 1 }                   */
/*  eq. (14) kappa = c_cap alpha log R / q90 if q90 > 0 and R > 1, else 0    */
/* and the fold of e^kappa into the heuristic, S = eta^beta e^kappa, with    */
/* the log-weight kappa log e clipped at `clip`.                              */
/* Readings: "row i" of eq. (10) is the candidate row (c is defined for      */
/* j in C_i); baseline_scope = 1 takes the full heatmap row instead.  The    */
/* quantile is linear interpolation between order statistics.                */
/* ------------------------------------------------------------------------ */
double orc_evidence(const orc_problem* p, const int32_t* cand, int32_t k_eff, double* conf,
                    double* base, double* evid, float* heur, double* q90_out, double* r_out) {
  int32_t n = p->n, dstar = degree_target(p);
  int64_t nk = (int64_t)n * k_eff;
  double* c = (double*)malloc(sizeof(double) * (nk > 0 ? nk : 1));
  double* e = (double*)malloc(sizeof(double) * (nk > 0 ? nk : 1));
  double* b = (double*)malloc(sizeof(double) * n);
  int32_t rowcap = k_eff;
  for (int32_t i = 0; i < n; i++) {
    int32_t len = p->row_ptr[i + 1] - p->row_ptr[i];
    if (len > rowcap) rowcap = len;
  }
  double* sorted = (double*)malloc(sizeof(double) * (rowcap > 0 ? rowcap : 1));
  for (int32_t i = 0; i < n; i++) {
    for (int32_t u = 0; u < k_eff; u++) {
      double h = heat(p, i, cand[(int64_t)i * k_eff + u]);
      c[(int64_t)i * k_eff + u] = h > p->theta_h ? h : 0.0;
    }
    int32_t cnt = 0;
    if (p->baseline_scope == 0) {
      for (int32_t u = 0; u < k_eff; u++)
        if (c[(int64_t)i * k_eff + u] > 0.0) sorted[cnt++] = c[(int64_t)i * k_eff + u];
    } else {
      for (int32_t q = p->row_ptr[i]; q < p->row_ptr[i + 1]; q++) {
        double h = (double)p->val[q];
        if (p->col[q] != i && h > p->theta_h) sorted[cnt++] = h;
      }
    }
    qsort(sorted, (size_t)cnt, sizeof(double), cmp_desc);
    double order_stat = cnt >= dstar + 1 ? sorted[dstar] : 0.0;
    b[i] = order_stat > p->eps ? order_stat : p->eps;
    for (int32_t u = 0; u < k_eff; u++) {
      double ci = c[(int64_t)i * k_eff + u];
      double ratio = (ci > p->eps ? ci : p->eps) / b[i];
      e[(int64_t)i * k_eff + u] = ratio > 1.0 ? ratio : 1.0;
    }
  }
  /* eq. (12) */
  int64_t nl = 0;
  double* logs = (double*)malloc(sizeof(double) * (nk > 0 ? nk : 1));
  for (int64_t x = 0; x < nk; x++)
    if (e[x] > 1.0) logs[nl++] = log(e[x]);
  double q90 = 0.0;
  if (nl > 0) {
    qsort(logs, (size_t)nl, sizeof(double), cmp_asc);
    double h = 0.9 * (double)(nl - 1);
    int64_t lo = (int64_t)floor(h);
    double frac = h - (double)lo;
    q90 = lo + 1 < nl ? logs[lo] + frac * (logs[lo + 1] - logs[lo]) : logs[lo];
  }
  /* eq. (13)-(14) */
  double r = r_hat(p, k_eff);
  double kappa;
  if (p->kappa_fixed >= 0.0)
    kappa = p->kappa_fixed; /* the ablation replaces eq. (14) by a constant */
  else
    kappa = (q90 > 0.0 && r > 1.0) ? p->c_cap * p->alpha * log(r) / q90 : 0.0;
  /* fold */
  if (heur) {
    for (int32_t i = 0; i < n; i++)
      for (int32_t u = 0; u < k_eff; u++) {
        int64_t x = (int64_t)i * k_eff + u;
        double eta = 1.0 / dist(p, i, cand[x]);
        double lw = kappa * log(e[x]);
        if (lw > p->clip) lw = p->clip;
        heur[x] = (float)(eta_pow(eta, p->beta) * exp(lw));
      }
  }
  if (conf) memcpy(conf, c, sizeof(double) * nk);
  if (evid) memcpy(evid, e, sizeof(double) * nk);
  if (base) memcpy(base, b, sizeof(double) * n);
  if (q90_out) *q90_out = q90;
  if (r_out) *r_out = r;
  free(c); free(e); free(b); free(sorted); free(logs);
  return kappa;
}

/* ------------------------------------------------------------------------ */
/* Eq. (4) as a roulette over the unvisited slots of one candidate row.       */
/* Reading (a fixed-point discretisation of eq. 4 at the resolution of the   */
/* FP32 weights): with E the largest floor(log2 w) over the unvisited slots,  */
/* each slot gets the integer weight q = max(1, floor(w 2^(23-E))), so the    */
/* heaviest slot keeps its whole 24-bit significand; r = floor(u * sum(q) /   */
/* 2^32) for the 32-bit uniform u, and the choice is the first slot, in list  */
/* order, whose inclusive prefix sum of q exceeds r.  Each slot's probability */
/* is within (k+1) 2^-23 + 2^-32 of eq. (4).                                   */
/* ------------------------------------------------------------------------ */
int32_t orc_select(int32_t k, const int32_t* cand_row, const float* w_row, const uint8_t* visited,
                   uint32_t u) {
  int32_t emax = INT_MIN;
  for (int32_t s = 0; s < k; s++) {
    if (visited[cand_row[s]]) continue;
    int ex;
    frexpf(w_row[s], &ex); /* w = m 2^ex, m in [0.5, 1): floor(log2 w) = ex - 1 */
    if (ex - 1 > emax) emax = ex - 1;
  }
  if (emax == INT_MIN) return -1;
  uint64_t total = 0;
  uint64_t q[256];
  for (int32_t s = 0; s < k; s++) {
    if (visited[cand_row[s]]) continue;
    double scaled = floor(ldexp((double)w_row[s], 23 - emax));
    q[s] = scaled < 1.0 ? 1u : (uint64_t)scaled;
    total += q[s];
  }
  uint64_t r = scale32(u, total);
  uint64_t acc = 0;
  for (int32_t s = 0; s < k; s++) {
    if (visited[cand_row[s]]) continue;
    acc += q[s];
    if (acc > r) return s;
  }
  return -1; /* not reached */
}

/* nearest unvisited node to i by (key, index) */
static int32_t nearest_unvisited(const orc_problem* p, int32_t i, const uint8_t* visited) {
  int32_t best = -1;
  double bk = 0.0;
  for (int32_t j = 0; j < p->n; j++) {
    if (visited[j]) continue;
    double kj = order_key(p, i, j);
    if (best < 0 || closer(kj, j, bk, best)) { best = j; bk = kj; }
  }
  return best;
}

/* Alg. 1 preparation: nearest-neighbour tour.  Reading: it starts at node 0. */
double orc_nn_tour(const orc_problem* p, int32_t* tour) {
  int32_t n = p->n;
  uint8_t* vis = (uint8_t*)calloc((size_t)n, 1);
  tour[0] = 0;
  vis[0] = 1;
  for (int32_t s = 1; s < n; s++) {
    int32_t j = nearest_unvisited(p, tour[s - 1], vis);
    tour[s] = j;
    vis[j] = 1;
  }
  free(vis);
  return orc_tour_length(p, tour);
}

/* Alg. 2: one ant.  Random start (draw at step 0), then n-1 decisions by
 * eq. (4) over the unvisited candidates, or the nearest unvisited node when
 * none is left.  q0 = 0: every decision samples.  Returns the number of
 * fallback steps. */
static int64_t construct_ant(const orc_problem* p, int32_t k_eff, const int32_t* cand,
                             const float* w, uint32_t t, uint32_t a, uint8_t* vis,
                             int32_t* tour) {
  int32_t n = p->n;
  int64_t fallbacks = 0;
  memset(vis, 0, (size_t)n);
  int32_t start = (int32_t)scale32(orc_draw(p->seed, t, a, 0), (uint64_t)n);
  tour[0] = start;
  vis[start] = 1;
  for (int32_t s = 1; s < n; s++) {
    int32_t i = tour[s - 1];
    int32_t slot = orc_select(k_eff, cand + (int64_t)i * k_eff, w + (int64_t)i * k_eff, vis,
                              orc_draw(p->seed, t, a, (uint32_t)s));
    int32_t j;
    if (slot < 0) {
      j = nearest_unvisited(p, i, vis);
      fallbacks++;
    } else {
      j = cand[(int64_t)i * k_eff + slot];
    }
    tour[s] = j;
    vis[j] = 1;
  }
  return fallbacks;
}

/* ------------------------------------------------------------------------ */
/* Section III-D: first-improvement 2-opt on geometric neighbour lists with   */
/* don't-look bits, kept as a FIFO queue of nodes to examine.                */
/* Readings: the queue starts in tour order; for node a the succ direction   */
/* is tried before pred, each over a's list in order, stopping a direction   */
/* once d(a,c) >= d(a,b); the first move with gain > min_gain is applied,    */
/* its four end nodes re-queued (a, b, c, e, if absent), and a re-examined.  */
/* A move reverses the path b..c (succ) or c..b (pred) unless that path is   */
/* longer than n/2, in which case the complementary path is reversed.        */
/* ------------------------------------------------------------------------ */
static void reverse_path(int32_t n, int32_t* tour, int32_t* pos, int32_t x, int32_t y) {
  int32_t i = pos[x], j = pos[y];
  int32_t len = ((j - i + n) % n) + 1;
  if (2 * len > n) {
    int32_t ni = (j + 1) % n, nj = (i - 1 + n) % n;
    i = ni;
    j = nj;
    len = n - len;
  }
  for (int32_t s = 0; s < len / 2; s++) {
    int32_t ti = tour[i], tj = tour[j];
    tour[i] = tj;
    tour[j] = ti;
    pos[tj] = i;
    pos[ti] = j;
    i = (i + 1) % n;
    j = (j - 1 + n) % n;
  }
}

void orc_two_opt(const orc_problem* p, const int32_t* nl, int32_t kk, double min_gain,
                 int32_t* tour) {
  int32_t n = p->n;
  if (n < 5 || kk < 1) return;
  int32_t* pos = (int32_t*)malloc(4 * (size_t)n);
  int32_t* queue = (int32_t*)malloc(4 * (size_t)n);
  uint8_t* inq = (uint8_t*)malloc((size_t)n);
  for (int32_t s = 0; s < n; s++) { pos[tour[s]] = s; queue[s] = tour[s]; inq[s] = 1; }
  int32_t head = 0, count = n;
#define SUCC(x) tour[(pos[x] + 1) % n]
#define PRED(x) tour[(pos[x] - 1 + n) % n]
#define PUSH(x)                          \
  do {                                   \
    if (!inq[x]) {                       \
      queue[(head + count) % n] = (x);   \
      count++;                           \
      inq[x] = 1;                        \
    }                                    \
  } while (0)
  while (count > 0) {
    int32_t a = queue[head];
    head = (head + 1) % n;
    count--;
    inq[a] = 0;
    int improved = 1;
    while (improved) {
      improved = 0;
      for (int dir = 0; dir < 2 && !improved; dir++) {
        int32_t b = dir == 0 ? SUCC(a) : PRED(a);
        double dab = dist(p, a, b);
        for (int32_t q = 0; q < kk; q++) {
          int32_t c = nl[(int64_t)a * kk + q];
          double dac = dist(p, a, c);
          double g1 = dab - dac;
          if (g1 <= 0.0) break;
          int32_t e = dir == 0 ? SUCC(c) : PRED(c);
          if (e == a || c == b) continue;
          double gain = (dab + dist(p, c, e)) - (dac + dist(p, b, e));
          if (gain > min_gain) {
            if (dir == 0) reverse_path(n, tour, pos, b, c);
            else reverse_path(n, tour, pos, c, b);
            PUSH(a); PUSH(b); PUSH(c); PUSH(e);
            improved = 1;
            break;
          }
        }
      }
    }
  }
#undef SUCC
#undef PRED
#undef PUSH
  free(pos); free(queue); free(inq);
}

/* ------------------------------------------------------------------------ */
/* Section III-D: first-improvement 3-opt on the same geometric neighbour     */
/* lists, for symmetric instances.  Reading (the paper names the operator   */
/* but not its move set): the search is the 2-opt's (queue in tour order,    */
/* FIFO re-queueing of the end nodes if absent, re-examination of a, gain   */
/* threshold min_gain) over a larger neighbourhood.  For node a, the 2-opt  */
/* moves come first, exactly as in orc_two_opt; if none improves, the        */
/* segment exchange, the 3-opt reconnection that keeps every segment's       */
/* orientation:                                                             */
/*   t1 = a, t2 = the next node after t1 in the direction (succ, then pred); */
/*   t3 over t1's list in order, g1 = d(t1,t2) - d(t1,t3), stop at g1 <= 0;  */
/*   t4 = the node before t3 in the direction;                              */
/*   t5 over t4's list in order, g2 = (g1 + d(t4,t3)) - d(t4,t5), stop at    */
/*   g2 <= 0; t5 must come after t3 in the direction, or be t1 itself;      */
/*   t6 = the node before t5 in the direction;                              */
/*   gain = ((d12 + d43) + d65) - ((d13 + d45) + d62).                       */
/* Walking from t1 in the direction the tour reads t1 | t2..t4 | t3..t6 |    */
/* t5..; the move makes it t1 | t3..t6 | t2..t4 | t5.., replacing (t1,t2),   */
/* (t4,t3), (t6,t5) with (t1,t3), (t6,t2), (t4,t5).  In the array the two    */
/* segments trade places and keep their order (nothing is reversed).  The   */
/* first move with gain > min_gain is applied and its end nodes t1 .. t6    */
/* re-queued in that order if absent.  A run applies at most 64 n moves, as  */
/* the directed 2-opt: every move shortens the tour by more than the        */
/* threshold, so the bound only guards against a broken gain.               */
/* ------------------------------------------------------------------------ */
void orc_three_opt(const orc_problem* p, const int32_t* nl, int32_t kk, double min_gain,
                   int32_t* tour) {
  int32_t n = p->n;
  if (n < 5 || kk < 1) return;
  int32_t* pos = (int32_t*)malloc(4 * (size_t)n);
  int32_t* queue = (int32_t*)malloc(4 * (size_t)n);
  int32_t* tmp = (int32_t*)malloc(4 * (size_t)n);
  uint8_t* inq = (uint8_t*)malloc((size_t)n);
  for (int32_t s = 0; s < n; s++) { pos[tour[s]] = s; queue[s] = tour[s]; inq[s] = 1; }
  int32_t head = 0, count = n;
  int64_t moves = 0, max_moves = 64 * (int64_t)n;
#define SUCC(x) tour[(pos[x] + 1) % n]
#define PRED(x) tour[(pos[x] - 1 + n) % n]
#define PUSH(x)                          \
  do {                                   \
    if (!inq[x]) {                       \
      queue[(head + count) % n] = (x);   \
      count++;                           \
      inq[x] = 1;                        \
    }                                    \
  } while (0)
  while (count > 0 && moves < max_moves) {
    int32_t a = queue[head];
    head = (head + 1) % n;
    count--;
    inq[a] = 0;
    int improved = 1;
    while (improved && moves < max_moves) {
      improved = 0;
      /* the 2-opt moves of a, as in orc_two_opt */
      for (int dir = 0; dir < 2 && !improved; dir++) {
        int32_t b = dir == 0 ? SUCC(a) : PRED(a);
        double dab = dist(p, a, b);
        for (int32_t q = 0; q < kk; q++) {
          int32_t c = nl[(int64_t)a * kk + q];
          double dac = dist(p, a, c);
          if (dab - dac <= 0.0) break;
          int32_t e = dir == 0 ? SUCC(c) : PRED(c);
          if (e == a || c == b) continue;
          double gain = (dab + dist(p, c, e)) - (dac + dist(p, b, e));
          if (gain > min_gain) {
            if (dir == 0) reverse_path(n, tour, pos, b, c);
            else reverse_path(n, tour, pos, c, b);
            PUSH(a);
            PUSH(b);
            PUSH(c);
            PUSH(e);
            improved = 1;
            moves++;
            break;
          }
        }
      }
      if (improved) continue;
      /* the segment exchanges of a */
      for (int dir = 0; dir < 2 && !improved; dir++) {
        int32_t t1 = a, p1 = pos[a];
        /* steps from t1 in the direction */
#define OFF(x) (dir == 0 ? (pos[x] - p1 + n) % n : (p1 - pos[x] + n) % n)
        int32_t t2 = dir == 0 ? SUCC(t1) : PRED(t1);
        double d12 = dist(p, t1, t2);
        for (int32_t q = 0; q < kk && !improved; q++) {
          int32_t t3 = nl[(int64_t)t1 * kk + q];
          double d13 = dist(p, t1, t3);
          double g1 = d12 - d13;
          if (g1 <= 0.0) break;
          int32_t r3 = OFF(t3);
          if (r3 < 2) continue;
          int32_t t4 = dir == 0 ? PRED(t3) : SUCC(t3);
          double d43 = dist(p, t4, t3);
          for (int32_t q5 = 0; q5 < kk; q5++) {
            int32_t t5 = nl[(int64_t)t4 * kk + q5];
            double d45 = dist(p, t4, t5);
            double g2 = (g1 + d43) - d45;
            if (g2 <= 0.0) break;
            int32_t r5 = OFF(t5);
            if (!(r5 > r3 || r5 == 0)) continue;
            int32_t t6 = dir == 0 ? PRED(t5) : SUCC(t5);
            double gain = ((d12 + d43) + dist(p, t6, t5)) - ((d13 + d45) + dist(p, t6, t2));
            if (gain > min_gain) {
              /* walking from t1: the segment t2..t4 (r3 - 1 nodes), then
                 t3..t6 (up to the step before t5); afterwards t3..t6 comes
                 first, then t2..t4, both in their own order */
              int32_t len1 = r3 - 1, end = r5 == 0 ? n - 1 : r5 - 1, len2 = end - r3 + 1, w = 0;
              for (int32_t s = 0; s < len2; s++) tmp[w++] = tour[(dir == 0 ? p1 + r3 + s : p1 - r3 - s + 2 * n) % n];
              for (int32_t s = 0; s < len1; s++) tmp[w++] = tour[(dir == 0 ? p1 + 1 + s : p1 - 1 - s + 2 * n) % n];
              for (int32_t s = 0; s < w; s++) {
                int32_t at = (dir == 0 ? p1 + 1 + s : p1 - 1 - s + 2 * n) % n;
                tour[at] = tmp[s];
                pos[tmp[s]] = at;
              }
              PUSH(t1); PUSH(t2); PUSH(t3); PUSH(t4); PUSH(t5); PUSH(t6);
              improved = 1;
              moves++;
              break;
            }
          }
        }
#undef OFF
      }
    }
  }
#undef SUCC
#undef PRED
#undef PUSH
  free(pos); free(queue); free(tmp); free(inq);
}

/* ------------------------------------------------------------------------ */
/* Section III-D for the ATSP: directed 2-opt.  Reading of "a directed 2-opt */
/* based on the Jonker-Volgenant reduction": that reduction makes each city  */
/* a pair of nodes joined by an edge every tour keeps; a 2-opt move on the   */
/* reduced graph that keeps the pairs joined reverses a path and swaps each  */
/* pair's roles, which on the directed tour is the 2-opt move whose reversed */
/* path is priced in its new direction.  Moves:                              */
/*   successor side: b = succ(a), c from a's outgoing list, e = succ(c);     */
/*     (a->b), (c->e) become (a->c), (b->e), the path b..c reversed;         */
/*   predecessor side: b = pred(a), c from a's incoming list, e = pred(c);   */
/*     (b->a), (e->c) become (c->a), (e->b), the path c..b reversed.         */
/* gain = (removed edges + F) - (added edges + B), F and B the reversed      */
/* path's cost in its old and new direction, from prefix sums of the         */
/* directed edge lengths in tour order, summed in blocks of 64 positions:    */
/* in order within a block, and the block totals in order (reading: the      */
/* paper does not say how path costs are kept; two levels let a search       */
/* re-sum only the blocks a move changed).  Queue, side order, list stop rule,*/
/* threshold and re-queueing as in the symmetric 2-opt; the reversed part is */
/* always the path itself (its complement would give the opposite tour).    */
/* A run applies at most 64 n moves: every move shortens the tour by more    */
/* than the threshold, so this bound only guards against a broken gain.     */
/* ------------------------------------------------------------------------ */

/* pf[q] = the sum of e(t) = d(T[t], T[t+1]) over t < q, pb[q] the same
 * edges reversed, q = 0..n, the closing edge last (eq. (1)'s order).  With
 * block(q) = floor(q / 64): pf[q] = S[block(q)] + (the edges of q's block
 * before q, added in order from 0.0), S[0] = 0 and S[b + 1] = S[b] + (block
 * b's 64 edges added in order from 0.0). */
static void directed_prefix(const orc_problem* p, const int32_t* tour, double* pf, double* pb) {
  int32_t n = p->n;
  double sf = 0.0, sb = 0.0; /* S of the current block */
  for (int32_t b0 = 0; b0 <= n; b0 += 64) {
    double f = 0.0, r = 0.0; /* the block's edges so far */
    for (int32_t q = b0; q < b0 + 64 && q <= n; q++) {
      pf[q] = sf + f;
      pb[q] = sb + r;
      if (q < n) {
        int32_t x = tour[q], y = tour[(q + 1) % n];
        f += dist(p, x, y);
        r += dist(p, y, x);
      }
    }
    sf += f;
    sb += r;
  }
}

/* cost of the path from position i to position j (cyclic, forward) */
static double path_cost(const double* pre, int32_t n, int32_t i, int32_t j) {
  return i <= j ? pre[j] - pre[i] : (pre[n] - pre[i]) + pre[j];
}

/* reverse the tour positions i..j (cyclic) */
static void reverse_positions(int32_t n, int32_t* tour, int32_t* pos, int32_t i, int32_t j) {
  int32_t len = ((j - i + n) % n) + 1;
  for (int32_t s = 0; s < len / 2; s++) {
    int32_t ti = tour[i], tj = tour[j];
    tour[i] = tj;
    tour[j] = ti;
    pos[tj] = i;
    pos[ti] = j;
    i = (i + 1) % n;
    j = (j - 1 + n) % n;
  }
}

/* gain of the directed move at a with list node c (dir 0: successor side,
 * 1: predecessor side), or NAN when the move is degenerate; *pi, *pj get
 * the positions of the path to reverse */
static double directed_gain(const orc_problem* p, const int32_t* tour, const int32_t* pos,
                            const double* pf, const double* pb, int32_t a, int32_t c, int dir,
                            int32_t* pi, int32_t* pj) {
  int32_t n = p->n;
  if (dir == 0) {
    int32_t b = tour[(pos[a] + 1) % n], e = tour[(pos[c] + 1) % n];
    if (e == a || c == b || c == a) return NAN;
    int32_t i = pos[b], j = pos[c];
    double F = path_cost(pf, n, i, j), B = path_cost(pb, n, i, j);
    *pi = i;
    *pj = j;
    return ((dist(p, a, b) + dist(p, c, e)) + F) - ((dist(p, a, c) + dist(p, b, e)) + B);
  }
  int32_t b = tour[(pos[a] - 1 + n) % n], e = tour[(pos[c] - 1 + n) % n];
  if (e == a || c == b || c == a) return NAN;
  int32_t i = pos[c], j = pos[b];
  double F = path_cost(pf, n, i, j), B = path_cost(pb, n, i, j);
  *pi = i;
  *pj = j;
  return ((dist(p, b, a) + dist(p, e, c)) + F) - ((dist(p, c, a) + dist(p, e, b)) + B);
}

void orc_two_opt_directed(const orc_problem* p, const int32_t* nl_out, const int32_t* nl_in, int32_t kk,
                          double min_gain, int32_t* tour) {
  int32_t n = p->n;
  if (n < 5 || kk < 1) return;
  int32_t* pos = (int32_t*)malloc(4 * (size_t)n);
  int32_t* queue = (int32_t*)malloc(4 * (size_t)n);
  uint8_t* inq = (uint8_t*)malloc((size_t)n);
  double* pf = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  double* pb = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  for (int32_t s = 0; s < n; s++) { pos[tour[s]] = s; queue[s] = tour[s]; inq[s] = 1; }
  directed_prefix(p, tour, pf, pb);
  int32_t head = 0, count = n;
  int64_t moves = 0, max_moves = 64 * (int64_t)n;
#define DPUSH(x)                         \
  do {                                   \
    if (!inq[x]) {                       \
      queue[(head + count) % n] = (x);   \
      count++;                           \
      inq[x] = 1;                        \
    }                                    \
  } while (0)
  while (count > 0 && moves < max_moves) {
    int32_t a = queue[head];
    head = (head + 1) % n;
    count--;
    inq[a] = 0;
    int improved = 1;
    while (improved && moves < max_moves) {
      improved = 0;
      for (int dir = 0; dir < 2 && !improved; dir++) {
        int32_t b = dir == 0 ? tour[(pos[a] + 1) % n] : tour[(pos[a] - 1 + n) % n];
        double dab = dir == 0 ? dist(p, a, b) : dist(p, b, a);
        const int32_t* nl = dir == 0 ? nl_out : nl_in;
        for (int32_t q = 0; q < kk; q++) {
          int32_t c = nl[(int64_t)a * kk + q];
          double dac = dir == 0 ? dist(p, a, c) : dist(p, c, a);
          double g1 = dab - dac;
          if (g1 <= 0.0) break;
          int32_t i, j;
          double gain = directed_gain(p, tour, pos, pf, pb, a, c, dir, &i, &j);
          if (isnan(gain)) continue;
          if (gain > min_gain) {
            int32_t e = dir == 0 ? tour[(pos[c] + 1) % n] : tour[(pos[c] - 1 + n) % n];
            reverse_positions(n, tour, pos, i, j);
            directed_prefix(p, tour, pf, pb);
            moves++;
            DPUSH(a); DPUSH(b); DPUSH(c); DPUSH(e);
            improved = 1;
            break;
          }
        }
      }
    }
  }
#undef DPUSH
  free(pos); free(queue); free(inq); free(pf); free(pb);
}

/* One directed move (test hook): the gain the directed 2-opt computes for
 * the move at node a with list node c on `tour` (dir 0 successor side, 1
 * predecessor side), and the tour after the move in `out`; NAN (out
 * unchanged) for a degenerate move. */
double orc_directed_move(const orc_problem* p, const int32_t* tour, int32_t a, int32_t c, int32_t dir,
                         int32_t* out) {
  int32_t n = p->n;
  int32_t* pos = (int32_t*)malloc(4 * (size_t)n);
  double* pf = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  double* pb = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  for (int32_t s = 0; s < n; s++) { out[s] = tour[s]; pos[tour[s]] = s; }
  directed_prefix(p, tour, pf, pb);
  int32_t i = 0, j = 0;
  double gain = directed_gain(p, tour, pos, pf, pb, a, c, dir, &i, &j);
  if (!isnan(gain)) reverse_positions(n, out, pos, i, j);
  free(pos); free(pf); free(pb);
  return gain;
}

/* Eq. (5)/(6): bounds from a tour length */
static void tau_bounds(const orc_problem* p, int32_t k_eff, double len, double* tmax,
                       double* tmin) {
  *tmax = 1.0 / (p->rho * len);
  if (p->local_search) {
    *tmin = *tmax / (2.0 * (double)p->n);
  } else {
    double px = p_x(p);
    *tmin = *tmax * (1.0 - px) / (((double)(k_eff - 1) / 2.0) * px);
  }
}

/* u_gb tiers.  Reading: the paper only says u_gb tightens from 25 to 1 as the
 * search stalls; the tiers are keyed on iterations without restart-best
 * improvement.  (the tier values are parity unpinned; that the schedule
 * starts at u_gb_max, never grows without an improvement and ends at 1 is
 * pinned) */
static int32_t ugb_schedule(const orc_problem* p, int32_t stall) {
  if (stall < 25) return p->ugb_max;
  if (stall < 75) return 5;
  if (stall < 125) return 3;
  if (stall < 250) return 2;
  return 1;
}

static int valid_problem(const orc_problem* p) {
  if (p->n < 1 || p->ants < 1 || p->k < 1 || p->iterations < 0) return 0;
  if (!(p->rho > 0.0 && p->rho < 1.0) || !(p->p_best > 0.0 && p->p_best < 1.0)) return 0;
  if (p->alpha != 1.0) return 0;
  if (p->local_search < 0 || p->local_search > 2) return 0;
  /* the local-search operator: 0 or 2 the 2-opt, 3 the 3-opt (symmetric
     instances only; the paper's ATSP search is the directed 2-opt) */
  if (p->ls_op != 0 && p->ls_op != 2 && p->ls_op != 3) return 0;
  if (p->ls_op == 3 && !is_sym(p)) return 0;
  if (!isfinite(p->kappa_fixed)) return 0;
  if (p->row_ptr[0] != 0) return 0;
  for (int32_t i = 0; i < p->n; i++) {
    if (p->row_ptr[i + 1] < p->row_ptr[i]) return 0;
    for (int32_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; e++) {
      if (p->col[e] < 0 || p->col[e] >= p->n) return 0;
      if (!isfinite(p->val[e]) || p->val[e] < 0.0f) return 0;
      for (int32_t f = p->row_ptr[i]; f < e; f++)
        if (p->col[f] == p->col[e]) return 0;
    }
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Section V: heatmap diagnostics against a known tour.                       */
/* ------------------------------------------------------------------------ */
int32_t orc_diagnostics(const orc_problem* p, const int32_t* tour, double out[4], int64_t counts[3]) {
  int32_t n = p->n;
  if (!valid_problem(p) || n < 2) return -1;
  int sym = is_sym(p);
  /* the known tour's successor and predecessor of every node */
  int32_t* succ = (int32_t*)malloc(4 * (size_t)n);
  int32_t* pred = (int32_t*)malloc(4 * (size_t)n);
  uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
  for (int32_t s = 0; s < n; s++) {
    int32_t a = tour[s];
    if (a < 0 || a >= n || seen[a]) { free(succ); free(pred); free(seen); return -1; }
    seen[a] = 1;
  }
  for (int32_t s = 0; s < n; s++) {
    succ[tour[s]] = tour[(s + 1) % n];
    pred[tour[s]] = tour[(s + n - 1) % n];
  }
  /* E_theta: directed entries above the threshold; and which tour edges
     they cover (edge s is (tour[s], tour[s+1])) */
  int64_t entries = 0, covered = 0;
  uint8_t* has_out = (uint8_t*)calloc((size_t)n, 1); /* (a, succ a) present   */
  uint8_t* has_in = (uint8_t*)calloc((size_t)n, 1);  /* (succ a, a) present   */
  for (int32_t i = 0; i < n; i++)
    for (int32_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; e++) {
      int32_t j = p->col[e];
      if (j == i || !((double)p->val[e] > p->theta_h)) continue;
      entries++;
      if (j == succ[i]) has_out[i] = 1;
      if (j == pred[i]) has_in[j] = 1; /* the reversed direction of edge (j, i) */
    }
  for (int32_t a = 0; a < n; a++)
    if (has_out[a] || (sym && has_in[a])) covered++;
  /* P(e > 1) over the candidate slots */
  int32_t k_eff = p->k < n - 1 ? p->k : n - 1;
  int64_t nk = (int64_t)n * k_eff;
  int32_t* cand = (int32_t*)malloc(4 * nk);
  double* evid = (double*)malloc(sizeof(double) * nk);
  orc_candidates(p, cand);
  orc_evidence(p, cand, k_eff, NULL, NULL, evid, NULL, NULL, NULL);
  int64_t strong = 0, on_tour = 0;
  for (int32_t i = 0; i < n; i++)
    for (int32_t u = 0; u < k_eff; u++) {
      int64_t x = (int64_t)i * k_eff + u;
      if (!(evid[x] > 1.0)) continue;
      strong++;
      int32_t j = cand[x];
      if (j == succ[i] || (sym && j == pred[i])) on_tour++;
    }
  out[0] = (double)entries / (2.0 * (double)n);
  out[1] = (double)covered / (double)n;
  out[2] = 100.0 * (1.0 - out[1]);
  out[3] = strong > 0 ? (double)on_tour / (double)strong : 0.0;
  counts[0] = entries;
  counts[1] = strong;
  counts[2] = on_tour;
  free(succ); free(pred); free(seen); free(has_out); free(has_in); free(cand); free(evid);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1: the decode loop.                                                   */
/* ------------------------------------------------------------------------ */
int32_t orc_decode(const orc_problem* p, int32_t* tour_out, double* len_out, orc_trace* tr) {
  if (!valid_problem(p)) return -1;
  int32_t n = p->n;
  if (n == 1) {
    tour_out[0] = 0;
    *len_out = 0.0;
    return 0;
  }
  int sym = is_sym(p);
  int32_t k_eff = p->k < n - 1 ? p->k : n - 1;
  int64_t nk = (int64_t)n * k_eff;

  /* --- preparation, once per instance --- */
  int32_t* cand = (int32_t*)malloc(4 * nk);
  orc_candidates(p, cand);
  for (int64_t x = 0; x < nk; x++) {
    double d = dist(p, (int32_t)(x / k_eff), cand[x]);
    if (!(d > 0.0) || !isfinite(d)) { free(cand); return -1; }
  }
  float* heur = (float*)malloc(4 * nk);
  double q90, rh;
  double kappa = orc_evidence(p, cand, k_eff, NULL, NULL, NULL, heur, &q90, &rh);
  for (int64_t x = 0; x < nk; x++)
    if (!isfinite(heur[x]) || heur[x] < FLT_MIN) { free(cand); free(heur); return -2; }

  int32_t k_ls = p->k_ls < n - 1 ? p->k_ls : n - 1;
  int32_t* nl = NULL;
  int32_t* nl_in = NULL; /* the ATSP's incoming lists, for the directed 2-opt */
  if (p->local_search) {
    nl = (int32_t*)malloc(4 * (int64_t)n * (k_ls > 0 ? k_ls : 1));
    orc_nearest_lists(p, k_ls, nl);
    if (!sym) {
      nl_in = (int32_t*)malloc(4 * (int64_t)n * (k_ls > 0 ? k_ls : 1));
      orc_nearest_in_lists(p, k_ls, nl_in);
    }
  }
  /* Section III-D: 2-opt for symmetric instances, directed 2-opt for the ATSP */
#define LOCAL_SEARCH(t)                                                  \
  do {                                                                   \
    if (sym && p->ls_op == 3) orc_three_opt(p, nl, k_ls, min_gain, (t)); \
    else if (sym) orc_two_opt(p, nl, k_ls, min_gain, (t));               \
    else orc_two_opt_directed(p, nl, nl_in, k_ls, min_gain, (t));        \
  } while (0)

  int32_t* t_nn = (int32_t*)malloc(4 * (size_t)n);
  double l_nn_raw = orc_nn_tour(p, t_nn);
  double l_nn = l_nn_raw;
  /* reading: the 2-opt gain threshold is 1e-9 of the mean NN-tour edge */
  double min_gain = 1e-9 * l_nn_raw / (double)n;
  if (p->local_search) {
    LOCAL_SEARCH(t_nn);
    l_nn = orc_tour_length(p, t_nn);
  }

  double tmax, tmin;
  tau_bounds(p, k_eff, l_nn, &tmax, &tmin);
  float tmax_f = (float)tmax, tmin_f = (float)tmin;
  {
    /* the largest tau_max any later global best can give is bounded by a
       lower bound on every tour length: each node leaves once */
    double lb = 0.0;
    for (int32_t i = 0; i < n; i++) {
      double m = INFINITY;
      for (int32_t j = 0; j < n; j++)
        if (j != i && dist(p, i, j) < m) m = dist(p, i, j);
      lb += m;
    }
    float hmax = 0.0f, hmin = FLT_MAX;
    for (int64_t x = 0; x < nk; x++) {
      if (heur[x] > hmax) hmax = heur[x];
      if (heur[x] < hmin) hmin = heur[x];
    }
    if (!(lb > 0.0) || (double)(float)(1.0 / (p->rho * lb)) * (double)hmax >= (double)FLT_MAX / 2 ||
        (double)tmin_f * (double)hmin < (double)FLT_MIN * 2) {
      free(cand); free(heur); free(nl); free(nl_in); free(t_nn);
      return -2;
    }
  }

  float* tau = (float*)malloc(4 * nk);
  float* w = (float*)malloc(4 * nk);
  for (int64_t x = 0; x < nk; x++) { tau[x] = tmax_f; w[x] = tau[x] * heur[x]; }

  int32_t* t_gb = (int32_t*)malloc(4 * (size_t)n);
  int32_t* t_rb = (int32_t*)malloc(4 * (size_t)n);
  int32_t* t_ib = (int32_t*)malloc(4 * (size_t)n);
  int32_t* tours = (int32_t*)malloc(4 * (size_t)n * p->ants);
  double* lens = (double*)malloc(sizeof(double) * p->ants);
  int32_t* succ = (int32_t*)malloc(4 * (size_t)n);
  int32_t* pred = (int32_t*)malloc(4 * (size_t)n);
  uint8_t* vis = (uint8_t*)malloc((size_t)n);
  memcpy(t_gb, t_nn, 4 * (size_t)n);
  double l_gb = l_nn, l_rb = 0.0;
  int rb_valid = 0;
  int32_t stall = 0, ugb = p->ugb_max, restarts = 0;
  int32_t dstar = degree_target(p);
  int64_t fallbacks = 0;
  float keep = (float)(1.0 - p->rho);

  /* --- search --- */
  for (int32_t t = 1; t <= p->iterations; t++) {
    for (int32_t a = 0; a < p->ants; a++) {
      int32_t* ta = tours + (int64_t)a * n;
      fallbacks += construct_ant(p, k_eff, cand, w, (uint32_t)t, (uint32_t)a, vis, ta);
      /* Alg. 1 applies the local search to every constructed tour
         (local_search = 2); the iteration best is then taken among the
         improved tours */
      if (p->local_search == 2) LOCAL_SEARCH(ta);
      lens[a] = orc_tour_length(p, ta);
    }
    /* iteration best: the first ant with the smallest length */
    int32_t ib = 0;
    for (int32_t a = 1; a < p->ants; a++)
      if (lens[a] < lens[ib]) ib = a;
    memcpy(t_ib, tours + (int64_t)ib * n, 4 * (size_t)n);
    double l_ib = lens[ib];
    if (p->local_search == 1) {
      LOCAL_SEARCH(t_ib);
      l_ib = orc_tour_length(p, t_ib);
    }
    /* restart-best (strictly better replaces) */
    if (!rb_valid || l_ib < l_rb) {
      memcpy(t_rb, t_ib, 4 * (size_t)n);
      l_rb = l_ib;
      rb_valid = 1;
      stall = 0;
    } else {
      stall++;
    }
    /* global best, and the bounds follow it */
    if (l_ib < l_gb) {
      memcpy(t_gb, t_ib, 4 * (size_t)n);
      l_gb = l_ib;
      tau_bounds(p, k_eff, l_gb, &tmax, &tmin);
      tmax_f = (float)tmax;
      tmin_f = (float)tmin;
    }
    /* elite tour.  Reading: on every u_gb-th iteration the restart-best
       tour deposits (it equals the global best until the first restart). */
    int use_rb = (t % ugb) == 0;
    int restarted = 0;
    const int32_t* elite = use_rb ? t_rb : t_ib;
    double l_elite = use_rb ? l_rb : l_ib;
    for (int32_t s = 0; s < n; s++) {
      succ[elite[s]] = elite[(s + 1) % n];
      pred[elite[s]] = elite[(s - 1 + n) % n];
    }
    /* eq. (7)-(8) on the candidate edges; FP32 pheromone */
    float delta = (float)(1.0 / l_elite);
    for (int32_t i = 0; i < n; i++) {
      for (int32_t u = 0; u < k_eff; u++) {
        int64_t x = (int64_t)i * k_eff + u;
        int32_t j = cand[x];
        int on_tour = j == succ[i] || (sym && j == pred[i]);
        float v = keep * tau[x];
        v = v + (on_tour ? delta : 0.0f);
        v = fmaxf(tmin_f, v);
        v = fminf(tmax_f, v);
        tau[x] = v;
        w[x] = v * heur[x];
      }
    }
    /* branching-factor restart.  Reading: the lambda-branching factor is
       the count of candidate trails at or above lo + xi (hi - lo) per row,
       divided by n d*, so that a converged field reads 1.  (parity unpinned) */
    if (p->bf_period > 0 && t % p->bf_period == 0) {
      int64_t branches = 0;
      for (int32_t i = 0; i < n; i++) {
        double lo = tau[(int64_t)i * k_eff], hi = lo;
        for (int32_t u = 1; u < k_eff; u++) {
          double v = tau[(int64_t)i * k_eff + u];
          if (v < lo) lo = v;
          if (v > hi) hi = v;
        }
        double cut = lo + p->xi_bf * (hi - lo);
        for (int32_t u = 0; u < k_eff; u++)
          if ((double)tau[(int64_t)i * k_eff + u] >= cut) branches++;
      }
      double bf = (double)branches / ((double)n * (double)dstar);
      if (bf < p->lambda_bf && stall > p->restart_stall) {
        for (int64_t x = 0; x < nk; x++) { tau[x] = tmax_f; w[x] = tau[x] * heur[x]; }
        rb_valid = 0;
        stall = 0;
        restarts++;
        restarted = 1;
      }
    }
    if (tr) {
      if (tr->l_ib) tr->l_ib[t - 1] = l_ib;
      if (tr->l_gb) tr->l_gb[t - 1] = l_gb;
      if (tr->elite_rb) tr->elite_rb[t - 1] = use_rb;
      if (tr->ugb) tr->ugb[t - 1] = ugb;
      if (tr->restart) tr->restart[t - 1] = restarted;
    }
    ugb = ugb_schedule(p, stall);
  }

  /* canonical output: start at node 0; symmetric tours read with the
     smaller neighbour of node 0 second */
  int32_t r0 = 0;
  for (int32_t s = 0; s < n; s++)
    if (t_gb[s] == 0) r0 = s;
  for (int32_t s = 0; s < n; s++) tour_out[s] = t_gb[(r0 + s) % n];
  if (sym && n >= 3 && tour_out[1] > tour_out[n - 1]) {
    for (int32_t a = 1, b = n - 1; a < b; a++, b--) {
      int32_t tmp = tour_out[a];
      tour_out[a] = tour_out[b];
      tour_out[b] = tmp;
    }
  }
  *len_out = l_gb;

  if (tr) {
    tr->k_eff = k_eff;
    tr->q90 = q90;
    tr->r_hat = rh;
    tr->kappa = kappa;
    tr->l_nn = l_nn;
    tr->l_nn_raw = l_nn_raw;
    tr->ant_steps = (int64_t)p->ants * (n - 1) * p->iterations;
    tr->fallback_steps = fallbacks;
    tr->restarts = restarts;
    if (tr->cand) memcpy(tr->cand, cand, 4 * nk);
    if (tr->heur) memcpy(tr->heur, heur, 4 * nk);
    if (tr->tau) memcpy(tr->tau, tau, 4 * nk);
    if (tr->weight) memcpy(tr->weight, w, 4 * nk);
    if (tr->ant_tours) memcpy(tr->ant_tours, tours, 4 * (size_t)n * p->ants);
    if (tr->ant_len) memcpy(tr->ant_len, lens, sizeof(double) * p->ants);
    if (tr->nn_tour) memcpy(tr->nn_tour, t_nn, 4 * (size_t)n);
  }
#undef LOCAL_SEARCH
  free(cand); free(heur); free(nl); free(nl_in); free(t_nn); free(tau); free(w); free(t_gb); free(t_rb);
  free(t_ib); free(tours); free(lens); free(succ); free(pred); free(vis);
  return 0;
}
