// HIP kernels of the heatmap-guided MMAS decoder, written for gfx950
// (CDNA4, 64-lane wavefronts).
//
// Layout conventions (per instance, all row-major):
//   cand  int32[n][k]   candidate list of node i (eq. 3), ascending (distance, index)
//   heur  f32  [n][k]   S = eta^beta e^kappa (folded on the host)
//   tau   f32  [n][k]   pheromone on candidate edges only
//   w     f32  [n][k]   choice weights tau * S (rewritten by every update)
//   geo   int32[n][kg]  geometric nearest neighbours, kg = min(n-1, 64)
//
// Numerical contract: this file is compiled with -ffp-contract=off and
// without fast-math, so every FP32/FP64 expression rounds exactly as
// written.  The only FP64 library routine used is sqrt, which the gfx950
// lowering computes with a correctly rounded final residual step.
// Selection is integer arithmetic on the bits of the FP32 weights.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <cstdlib>
#include <mutex>
#include <type_traits>

#include "hac_internal.h"

// Device memory of the allocation-free entry point (hac_decode_noalloc):
// every buffer of such a decode is carved from this array, which each GPU
// the library runs on holds for the life of the process.  In host code its
// name is a host-side stand-in, not a device address: the address comes
// from hipGetSymbolAddress, taken once per device (noalloc_scratch_init).
static __device__ __align__(256) unsigned char scratch[hac::kNoAllocBytes];

namespace hac {

static constexpr int WAVE = 64;

// ------------------------------------------------------------------------
// wave primitives
// ------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

__device__ __forceinline__ int rd_lane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ double rd_lane_d(double v, int l) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// permutations that stay inside a 16-lane row: every lane has a source,
// so bound_ctrl only spares the compiler an "old" operand
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_all(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, true);
}

template <int CTRL>
__device__ __forceinline__ double dpp_all_f64(double v) {
  return __hiloint2double((int)dpp_all<CTRL>((uint32_t)__double2hiint(v)),
                          (int)dpp_all<CTRL>((uint32_t)__double2loint(v)));
}

__device__ __forceinline__ uint32_t swz_xor16(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x401f);  // lane ^ 16 inside 32 lanes
}

__device__ __forceinline__ double swz_xor16_f64(double v) {
  return __hiloint2double((int)swz_xor16((uint32_t)__double2hiint(v)),
                          (int)swz_xor16((uint32_t)__double2loint(v)));
}

// Butterfly inside each 16-lane row: lane ^ 1, lane ^ 2 (quad permutes),
// then the mirrored quad of the half row and the mirrored half of the row.
// Afterwards every lane holds the reduction over its row.
template <class Op>
__device__ __forceinline__ uint32_t row_reduce(uint32_t v, Op op) {
  v = op(v, dpp_all<0xB1>(v));   // quad_perm [1,0,3,2]
  v = op(v, dpp_all<0x4E>(v));   // quad_perm [2,3,0,1]
  v = op(v, dpp_all<0x141>(v));  // row_half_mirror
  v = op(v, dpp_all<0x140>(v));  // row_mirror
  return v;
}
struct OpMax {
  __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; }
};
struct OpMin {
  __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a < b ? a : b; }
};
struct OpOr {
  __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a | b; }
};
struct OpAdd {
  __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; }
};
struct OpMinI {
  __device__ uint32_t operator()(uint32_t a, uint32_t b) const {
    return (int32_t)a < (int32_t)b ? a : b;
  }
};

__device__ __forceinline__ double dmin(double a, double b) { return b < a ? b : a; }

__device__ __forceinline__ bool key_less(double ka, int ia, double kb, int ib) {
  return ka < kb || (ka == kb && ia < ib);
}

// Pointers known to address global memory, so that accesses compile to
// global_* instead of flat_* instructions (a flat access may alias LDS and
// forces waits on every later LDS access).
#define HAC_AS1 __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ HAC_AS1 T* as_global(T* p) {
  return (HAC_AS1 T*)p;
}

// The distance view the hot kernels use.
struct GDist {
  const HAC_AS1 double* xy = nullptr;
  const HAC_AS1 double* dist = nullptr;
  int n = 0;
  GDist() = default;
  __device__ explicit GDist(const InstDesc& D)
      : xy(D.xy ? as_global(D.xy) : nullptr), dist(D.dist ? as_global(D.dist) : nullptr), n(D.n) {}
  __device__ __forceinline__ double key(int i, int j) const {
    if (xy) {
      const double dx = xy[2 * i] - xy[2 * j];
      const double dy = xy[2 * i + 1] - xy[2 * j + 1];
      return dx * dx + dy * dy;
    }
    return dist[(int64_t)i * n + j];
  }
  __device__ __forceinline__ double len(int i, int j) const {
    if (xy) return sqrt(key(i, j));
    return dist[(int64_t)i * n + j];
  }
};

// lane mask of a > b for unsigned 64-bit values, straight from the compare
__device__ __forceinline__ uint64_t lanes_ugt(uint64_t a, uint64_t b) {
  return __builtin_amdgcn_uicmpl(a, b, 34 /* unsigned greater than */);
}

// Lexicographic (key, index) minimum over the wave, returned to all lanes.
// The smallest key comes from a DPP butterfly; a unique holder hands over
// its index directly, ties take the smallest index among the holders.
// Keys are never NaN.
__device__ __forceinline__ void wave_argmin(double& key, int& idx) {
  double m = key;
  m = dmin(m, dpp_all_f64<0xB1>(m));
  m = dmin(m, dpp_all_f64<0x4E>(m));
  m = dmin(m, dpp_all_f64<0x141>(m));
  m = dmin(m, dpp_all_f64<0x140>(m));
  m = dmin(m, swz_xor16_f64(m));
  const double M = dmin(rd_lane_d(m, 0), rd_lane_d(m, 32));
  const uint64_t eq = __builtin_amdgcn_ballot_w64(key == M);
  int j;
  if ((eq & (eq - 1)) == 0) {
    j = rd_lane(idx, (int)__builtin_ctzll(eq));
  } else {
    uint32_t v = row_reduce(key == M ? (uint32_t)idx : 0xffffffffu, OpMin());
    v = min(v, swz_xor16(v));
    j = (int)min((uint32_t)rd_lane((int)v, 0), (uint32_t)rd_lane((int)v, 32));
  }
  key = M;
  idx = j;
}

// ------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): two 32x32 multiplies
// per round, key bumped by the golden-ratio Weyl constants.  Returns the
// first output word, the step's 32-bit uniform.
// ------------------------------------------------------------------------
__device__ __forceinline__ uint32_t philox_x0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    uint32_t hi0 = __umulhi(m0, c0), lo0 = m0 * c0;
    uint32_t hi1 = __umulhi(m1, c2), lo1 = m1 * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c0;
}

// ------------------------------------------------------------------------
// distances
// ------------------------------------------------------------------------
__device__ __forceinline__ double order_key(const InstDesc& D, int i, int j) {
  if (D.xy) {
    double dx = D.xy[2 * i] - D.xy[2 * j];
    double dy = D.xy[2 * i + 1] - D.xy[2 * j + 1];
    return dx * dx + dy * dy;
  }
  return D.dist[(int64_t)i * D.n + j];
}

__device__ __forceinline__ double edge_len(const InstDesc& D, int i, int j) {
  if (D.xy) return sqrt(order_key(D, i, j));
  return D.dist[(int64_t)i * D.n + j];
}

// Sum of the n edges of a tour in array order, closing edge last (eq. 1).
// Lanes compute 64 edges at a time; the additions are sequential.
__device__ double tour_length_wave(const InstDesc& D, const int32_t* tour) {
  const int n = D.n, lane = lane_id();
  double len = 0.0;
  for (int b0 = 0; b0 < n; b0 += WAVE) {
    int s = b0 + lane;
    double d = 0.0;
    if (s >= 1 && s < n) d = edge_len(D, tour[s - 1], tour[s]);
    int last = min(WAVE, n - b0);
    for (int l = (b0 == 0 ? 1 : 0); l < last; ++l) len += rd_lane_d(d, l);
  }
  len += edge_len(D, tour[n - 1], tour[0]);
  return len;
}

// Nearest unvisited node to i by (key, index).  `vis` is the wave's LDS
// bitset (bits >= n set).  The geometric list holds the kg nearest nodes in
// that order, so its first unvisited entry, if any, is the answer;
// otherwise every node is scanned.
// ------------------------------------------------------------------------
// Candidate lists (eq. 3) and geometric neighbour lists.
// One wave per row.  The k nearest heatmap-supported nodes, or all of them
// plus the nearest unsupported ones; the final list is in ascending
// (key, index) order.  Top-K lists live in lanes 0..K-1, kept sorted.
// ------------------------------------------------------------------------
struct WaveTopK {
  double key;
  int id;
  int cnt;
  int K;
};

__device__ __forceinline__ void topk_init(WaveTopK& t, int K) {
  t.key = __builtin_huge_val();
  t.id = 0x7fffffff;
  t.cnt = 0;
  t.K = K;
}

__device__ void topk_offer(WaveTopK& t, double key, int id, bool valid) {
  const int lane = lane_id();
  double tk = __builtin_huge_val();
  int ti = 0x7fffffff;
  if (t.cnt == t.K) {
    tk = rd_lane_d(t.key, t.K - 1);
    ti = rd_lane(t.id, t.K - 1);
  }
  uint64_t m = __ballot(valid && key_less(key, id, tk, ti));
  while (m) {
    int l = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    double nk = rd_lane_d(key, l);
    int ni = rd_lane(id, l);
    if (t.cnt == t.K) {
      tk = rd_lane_d(t.key, t.K - 1);
      ti = rd_lane(t.id, t.K - 1);
      if (!key_less(nk, ni, tk, ti)) continue;
    }
    int rank = __popcll(__ballot(lane < t.cnt && key_less(t.key, t.id, nk, ni)));
    double pk = __shfl_up(t.key, 1);
    int pi = __shfl_up(t.id, 1);
    if (lane > rank) {
      t.key = pk;
      t.id = pi;
    } else if (lane == rank) {
      t.key = nk;
      t.id = ni;
    }
    if (t.cnt < t.K) t.cnt++;
  }
}

// One launch for a whole batch: blockIdx.y is the instance.
__global__ void __launch_bounds__(256) candidates_kernel(const InstDesc* insts) {
  const InstDesc& D = insts[blockIdx.y];
  const int n = D.n, k = D.k, kg = D.kg, lane = lane_id();
  const int i = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
  if (i >= n) return;
  // heatmap-supported members of row i, nearest k of them
  WaveTopK sup;
  topk_init(sup, k);
  const int e_beg = D.row_ptr[i], e_end = D.row_ptr[i + 1];
  for (int e0 = e_beg; e0 < e_end; e0 += WAVE) {
    int e = e0 + lane;
    bool mem = false;
    int j = 0;
    double key = 0.0;
    if (e < e_end) {
      j = D.col[e];
      mem = j != i && (double)D.val[e] > D.theta_h;
      if (mem) key = order_key(D, i, j);
    }
    topk_offer(sup, key, j, mem);
  }
  const int s = sup.cnt;  // = min(|P_i|, k)
  const int need = k - s;
  // one pass over all nodes: geometric list, and fill when needed
  WaveTopK geo, fill;
  topk_init(geo, kg);
  topk_init(fill, k);
  for (int j0 = 0; j0 < n; j0 += WAVE) {
    int j = j0 + lane;
    bool valid = j < n && j != i;
    double key = valid ? order_key(D, i, j) : 0.0;
    topk_offer(geo, key, j, valid);
    if (need > 0) {
      // |P_i| < k here, so every member of P_i is in `sup`
      bool member = false;
      for (int q = 0; q < s; ++q) member |= (j == rd_lane(sup.id, q));
      topk_offer(fill, key, j, valid && !member);
    }
  }
  // merge sup[0..s) and fill[0..need) by (key, index): each entry's
  // place is its index plus the number of smaller entries of the other list
  int rank_s = lane, rank_f = lane;
  for (int b = 0; b < need; ++b)
    if (key_less(rd_lane_d(fill.key, b), rd_lane(fill.id, b), sup.key, sup.id)) rank_s++;
  for (int a = 0; a < s; ++a)
    if (key_less(rd_lane_d(sup.key, a), rd_lane(sup.id, a), fill.key, fill.id)) rank_f++;
  int32_t* out = D.cand + (int64_t)i * k;
  if (lane < s) out[rank_s] = sup.id;
  if (lane < need) out[rank_f] = fill.id;
  if (lane < kg) D.geo[(int64_t)i * kg + lane] = geo.id;
  if (D.geo16) D.geo16[(int64_t)i * 64 + lane] = (uint16_t)(lane < kg ? geo.id : 0);
  // each node's nearest neighbour, for the host's lower bound on a tour;
  // the successor array holds it until the first update overwrites it
  if (lane == 0) D.succ[i] = geo.id;
}

// Visited tests over an ant's two representations: one bit per node, or
// one byte per node (no shift or mask on the hot path, used when it fits).
struct VisBits {
  const uint32_t* p;
  __device__ __forceinline__ bool operator()(int v) const { return (p[v >> 5] >> (v & 31)) & 1u; }
};
struct VisBytes {
  const uint8_t* p;
  __device__ __forceinline__ bool operator()(int v) const { return p[v] != 0; }
};

// ------------------------------------------------------------------------
// Exact nearest-unvisited search over a uniform grid (coordinate instances
// with n >= kGridMinN).  Rings of cells around i's cell are examined
// wave-wide, one cell per lane at a time; after rings 0..R every node not
// yet examined lies at least R * wmin away, so the search stops once the
// best (key, index) found has key < (R wmin)^2.  The key is the one every
// scan uses (squared FP64 distance), so the result is that of a full scan.
// ------------------------------------------------------------------------
struct GridView {
  const HAC_AS1 int32_t* start = nullptr;
  const HAC_AS1 int32_t* ids = nullptr;
  const HAC_AS1 double* xy = nullptr;
  GridPar par{};
  __device__ __forceinline__ int cellx(double x) const {
    const int c = (int)((x - par.x0) * par.ix);
    return c < 0 ? 0 : (c >= par.gx ? par.gx - 1 : c);
  }
  __device__ __forceinline__ int celly(double y) const {
    const int c = (int)((y - par.y0) * par.iy);
    return c < 0 ? 0 : (c >= par.gy ? par.gy - 1 : c);
  }
};

__device__ __forceinline__ int ring_cells(int r) { return r == 0 ? 1 : 8 * r; }

// cell offset of entry t of ring r (r >= 1): top row, bottom row, left and
// right columns
__device__ __forceinline__ void ring_cell(int r, int t, int& dx, int& dy) {
  if (r == 0) {
    dx = dy = 0;
  } else if (t < 2 * r + 1) {
    dx = t - r;
    dy = -r;
  } else if (t < 4 * r + 2) {
    dx = t - (2 * r + 1) - r;
    dy = r;
  } else if (t < 6 * r + 1) {
    dx = -r;
    dy = t - (4 * r + 2) - (r - 1);
  } else {
    dx = r;
    dy = t - (6 * r + 1) - (r - 1);
  }
}

template <class V>
__device__ int grid_nearest(const GridView& g, int n, double xi, double yi, V visited) {
  const int lane = lane_id();
  const int cxi = g.cellx(xi), cyi = g.celly(yi);
  const int rmax = max(max(cxi, g.par.gx - 1 - cxi), max(cyi, g.par.gy - 1 - cyi));
  double bk = __builtin_huge_val();
  int bj = 0x7fffffff;
  for (int r0 = 0;;) {
    // this pass: rings r0..r1, at most two cells per lane unless one ring is larger
    int r1 = r0, cells = ring_cells(r0);
    while (r1 < rmax && cells + ring_cells(r1 + 1) <= 2 * WAVE) {
      ++r1;
      cells += ring_cells(r1);
    }
    for (int t = lane; t < cells; t += WAVE) {
      int r = r0, tt = t;
      while (tt >= ring_cells(r)) {
        tt -= ring_cells(r);
        ++r;
      }
      int dx, dy;
      ring_cell(r, tt, dx, dy);
      const int cx = cxi + dx, cy = cyi + dy;
      if (cx < 0 || cy < 0 || cx >= g.par.gx || cy >= g.par.gy) continue;
      const int c = cy * g.par.gx + cx;
      const int s = g.start[c], e = g.start[c + 1];
      for (int p0 = s; p0 < e; p0 += 4) {
        int id[4];
        double px[4], py[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int p = min(p0 + u, e - 1);
          id[u] = g.ids[p];
          px[u] = g.xy[2 * p];
          py[u] = g.xy[2 * p + 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (p0 + u < e && !visited(id[u])) {
            const double ddx = xi - px[u], ddy = yi - py[u];
            const double kj = ddx * ddx + ddy * ddy;
            if (key_less(kj, id[u], bk, bj)) {
              bk = kj;
              bj = id[u];
            }
          }
        }
      }
    }
    wave_argmin(bk, bj);
    const double bound = (double)r1 * g.par.wmin;
    if (bk < bound * bound || r1 >= rmax) return bj < n ? bj : n - 1;
    r0 = r1 + 1;
  }
}

__device__ __forceinline__ GridView grid_view(const InstDesc& D) {
  GridView g;
  if (D.gside > 0) {
    g.start = as_global((const int32_t*)D.g_start);
    g.ids = as_global((const int32_t*)D.g_ids);
    g.xy = as_global((const double*)D.g_xy);
    g.par = *D.g_par;
  }
  return g;
}

// Nearest unvisited node to i by (key, index), for the preparation kernels.
template <int CH, class V>
__device__ int scan_unvisited_g(const GDist& G, int i, V visited);
template <class V>
__device__ __forceinline__ int geo_first_unvisited(const HAC_AS1 int32_t* geo, int kg, int i,
                                                   V visited);
__device__ int nearest_unvisited(const InstDesc& D, const GridView& g, int i, const uint32_t* vis) {
  const int jg = geo_first_unvisited(as_global(D.geo), D.kg, i, VisBits{vis});
  if (jg >= 0) return jg;
  if (D.gside > 0) return grid_nearest(g, D.n, D.xy[2 * i], D.xy[2 * i + 1], VisBits{vis});
  return scan_unvisited_g<8>(GDist(D), i, VisBits{vis});
}

// ------------------------------------------------------------------------
// Nearest-neighbour tour from node 0 (one wave per instance).  Writes the
// tour and, in the state, its length and the 2-opt gain threshold.
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(64) nn_tour_kernel(const InstDesc* insts) {
  const InstDesc& D = insts[blockIdx.x];
  extern __shared__ uint32_t vis[];
  const int n = D.n, lane = lane_id();
  const int words2 = ((n + 63) >> 6) << 1;
  for (int w = lane; w < words2; w += WAVE) {
    int lo = w * 32;
    uint32_t v = 0;
    for (int b = 0; b < 32; ++b)
      if (lo + b >= n) v |= 1u << b;
    vis[w] = v;
  }
  __syncthreads();
  int32_t* tour = D.nn_tour;
  int cur = 0;
  if (lane == 0) {
    tour[0] = 0;
    vis[0] |= 1u;
  }
  __syncthreads();
  const GridView g = grid_view(D);
  for (int s = 1; s < n; ++s) {
    int j = nearest_unvisited(D, g, cur, vis);
    if (lane == 0) {
      tour[s] = j;
      vis[j >> 5] |= 1u << (j & 31);
    }
    __syncthreads();
    cur = j;
  }
  __threadfence_block();
  double len = tour_length_wave(D, tour);
  if (lane == 0) {
    D.st->l_gb = len;
    D.st->l_ib = len;
    D.st->min_gain = 1e-9 * len / (double)n;
  }
}

// ------------------------------------------------------------------------
// First-improvement 2-opt over the geometric lists with a FIFO don't-look
// queue (Section III-D), one block of up to LS_WAVES waves per tour.
//
// Sequentially, node a leaves the queue head and its moves are scanned:
// successor direction, then predecessor, each in list order and stopping at
// the first neighbour c with d(a,c) >= d(a,b).  The first improving move is
// applied, its end nodes are queued if absent, and a is examined again.  A
// node without an improving move only leaves the queue.  The block
// therefore evaluates the next W queue entries at once (W = its waves), one wave per
// entry and all against the same tour (lanes 0..31 the successor moves,
// 32..63 the predecessor moves).  The entries before the first one with an
// improving move are consumed exactly as a sequential scan would consume
// them; that move is applied and its node re-examined, and the speculative
// results behind it are dropped.  The outcome is the sequential one.
// ------------------------------------------------------------------------
static constexpr int LS_WAVES = 16;

struct LsMove {
  int imp, a, b, c, e, dir;
};

// Mode 2 decides the 2-opt tests from an FP32 copy of the coordinates in
// LDS.  M is the largest coordinate magnitude.  With u = 2^-24, rounding
// the coordinates and computing a distance in FP32 (a square root within a
// few ulp) is off by at most 17 u M from the FP64 value, so
//   d(a,b) - d(a,c)         is within E1 = 2^-18 M (>= 34 u M + rounding),
//   (ab + ce) - (ac + be)   is within E2 = 2^-17 M (>= 68 u M + 17 u M).
// A lane whose FP32 result lies inside the bound recomputes its test in
// FP64 from global memory, so every decision is the FP64 one.

// candidate moves of node a against the current tour (one wave)
template <class IP>
__device__ __forceinline__ LsMove ls_eval(const GDist& G, const HAC_AS1 int32_t* geo, int kg, int kls,
                                          int n, IP tour, IP pos, int a, double min_gain) {
  const int lane = lane_id();
  const bool pred_dir = lane >= 32;
  const int q = lane & 31;
  const bool in_list = q < kls;
  const int c = geo[(int64_t)a * kg + min(q, kls - 1)];
  const int pa = pos[a];
  const int b = pred_dir ? tour[pa == 0 ? n - 1 : pa - 1] : tour[pa + 1 == n ? 0 : pa + 1];
  const double dab = G.len(a, b), dac = G.len(a, c);
  const bool g1pos = dab - dac > 0.0;
  // a direction stops at the first list entry that cannot gain
  const uint64_t stop = __builtin_amdgcn_ballot_w64(in_list && !g1pos);
  const uint64_t stop_s = stop & 0xffffffffull, stop_p = stop >> 32;
  const int lim_s = stop_s ? (int)__builtin_ctzll(stop_s) : 32;
  const int lim_p = stop_p ? (int)__builtin_ctzll(stop_p) : 32;
  const bool ok = in_list && q < (pred_dir ? lim_p : lim_s);
  const int pc = pos[c];
  const int e = pred_dir ? tour[pc == 0 ? n - 1 : pc - 1] : tour[pc + 1 == n ? 0 : pc + 1];
  const bool cand = ok && e != a && c != b;  // a move that may be taken
  const bool imp = cand && (dab + G.len(c, e)) - (dac + G.len(b, e)) > min_gain;
  const uint64_t mi = __builtin_amdgcn_ballot_w64(imp);
  LsMove m{0, a, 0, 0, 0, 0};
  if (mi) {
    const int l = (int)__builtin_ctzll(mi);
    m.imp = 1;
    m.b = rd_lane(b, l);
    m.c = rd_lane(c, l);
    m.e = rd_lane(e, l);
    m.dir = l >= 32;
  }
  return m;
}

// Reverse the tour path between positions i and j (or its complement when
// that is shorter); block-wide.  Every thread passes the same positions,
// read before any thread of the block can change pos.
template <class IP>
__device__ __forceinline__ void ls_reverse(int n, IP tour, IP pos, int i, int j) {
  int len = ((j - i + n) % n) + 1;
  if (2 * len > n) {
    const int ni = (j + 1) % n, nj = (i - 1 + n) % n;
    i = ni;
    j = nj;
    len = n - len;
  }
  const int half = len / 2;
  for (int s = threadIdx.x; s < half; s += blockDim.x) {
    int pi = i + s;
    if (pi >= n) pi -= n;
    int pj = j - s;
    if (pj < 0) pj += n;
    const int ti = tour[pi], tj = tour[pj];
    tour[pi] = tj;
    tour[pj] = ti;
    pos[tj] = pi;
    pos[ti] = pj;
  }
  __syncthreads();
}

template <class IP, class BP>
__device__ __forceinline__ void two_opt_block(const InstDesc& D, IP tour, IP pos, IP queue, BP inq, double min_gain) {
  __shared__ int sh_head, sh_count;
  __shared__ LsMove sh_mv[LS_WAVES];
  const int n = D.n, kls = D.kls, kg = D.kg, lane = lane_id(), wave = threadIdx.x / WAVE;
  const int nw = (int)(blockDim.x / WAVE);  // 1 .. LS_WAVES entries per batch
  if (n < 5 || kls < 1) return;
  const GDist G(D);
  const HAC_AS1 int32_t* geo = as_global(D.geo);
  for (int s = threadIdx.x; s < n; s += blockDim.x) {
    const int v = tour[s];
    pos[v] = s;
    queue[s] = v;
    inq[v] = 1;
  }
  if (threadIdx.x == 0) {
    sh_head = 0;
    sh_count = n;
  }
  __syncthreads();
  // A node whose move was just applied is examined again before the queue
  // moves on; that re-examination rides in wave 0 of the next batch, ahead
  // of the queue entries, so results are taken in the sequential order.
  int pend = -1;
  for (;;) {
    const int head = sh_head, count = sh_count;
    const int re = pend >= 0 ? 1 : 0;
    const int nq = min(nw - re, count);  // queue entries in this batch
    const int nb = nq + re;
    if (nb == 0) break;
    if (wave < nb) {
      int node = pend;
      if (wave >= re) {
        int slot = head + wave - re;
        if (slot >= n) slot -= n;
        node = queue[slot];
      }
      const LsMove m = ls_eval(G, geo, kg, kls, n, tour, pos, node, min_gain);
      if (lane == 0) sh_mv[wave] = m;
    }
    __syncthreads();
    // the first improving result in batch order: every lane reads one entry
    // at once, instead of a chain of dependent reads
    const uint64_t fm = __builtin_amdgcn_ballot_w64(lane < nb && sh_mv[min(lane, LS_WAVES - 1)].imp);
    const int f = fm ? (int)__builtin_ctzll(fm) : -1;
    // queue entries consumed as a sequential scan would: all of them if no
    // move improves, else those up to and including the improving one
    const int used = f < 0 ? nq : max(0, f + 1 - re);
    LsMove m{};
    int ri = 0, rj = 0;  // positions of the ends of the path to reverse
    if (f >= 0) {
      m = sh_mv[f];
      ri = pos[m.dir == 0 ? m.b : m.c];
      rj = pos[m.dir == 0 ? m.c : m.b];
    }
    if ((int)threadIdx.x < used) {
      int slot = head + threadIdx.x;
      if (slot >= n) slot -= n;
      inq[queue[slot]] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int h = head + used;
      if (h >= n) h -= n;
      sh_head = h;
      sh_count = count - used;
    }
    if (f < 0) {
      pend = -1;
      __syncthreads();
      continue;
    }
    // queue the move's end nodes, then apply it; its node is examined next.
    // The end nodes a, b, c, e (four distinct nodes) join the queue tail in
    // that order if absent: lanes 0..3 of wave 0 take one each, after lane 0
    // has moved the head (the queue and the tour are separate arrays, so
    // this may precede the reversal, whose closing barrier publishes both)
    if (threadIdx.x < 4) {
      const int z = threadIdx.x;
      const int x = z == 0 ? m.a : (z == 1 ? m.b : (z == 2 ? m.c : m.e));
      const bool absent = !inq[x];
      const uint32_t am = (uint32_t)__builtin_amdgcn_ballot_w64(absent) & 0xfu;
      if (absent) {
        int slot = sh_head + sh_count + __builtin_popcount(am & ((1u << z) - 1u));
        if (slot >= n) slot -= n;
        queue[slot] = x;
        inq[x] = 1;
      }
      __builtin_amdgcn_wave_barrier();
      if (z == 0) sh_count += __builtin_popcount(am);
    }
    ls_reverse(n, tour, pos, ri, rj);
    pend = m.a;
  }
}

// Mode 2 of the 2-opt keeps the FP32 coordinates in tour order (txy[p] is
// the node at position p), so one position read gives a node's tour
// neighbour and its coordinates together: after the neighbour-list load,
// the evaluation of a move is two dependent LDS reads deep (pos[c], then
// tour, txy at pc and pc +- 1) instead of five.  The evaluating wave also
// works out the path to reverse (the shorter side), so a round needs one
// barrier after the evaluations and one after the reversal; the queue
// bookkeeping stays in one wave (its LDS operations are ordered), which
// runs it while the other waves reverse the path.
struct LsMoveXY {
  int imp, a, b, c, e, i, j, half;
};

// What the evaluation of node a leaves for the 3-opt's exchange search (per
// lane: this half's direction, list entry q): a's position, its tour
// neighbour b and the list entry c with their positions and FP32
// coordinates and distances, and whether d(a,b) - d(a,c) > 0 in FP64.
struct LsNodeXY {
  int pa, b, c, pc;
  float2 xa, xb, xc;
  float lab, lac;
  bool g1pos;
};

// the hardware square root (within 1 ulp, inside the bound's allowance)
// instead of the correctly rounded library sequence
__device__ __forceinline__ float ls_len_xy(float2 p, float2 q) {
  const float dx = p.x - q.x, dy = p.y - q.y;
  return __builtin_amdgcn_sqrtf(dx * dx + dy * dy);
}

// position p + step (step = +-1) on a cycle of n, as selects rather than branches
__device__ __forceinline__ int cyc_step(int p, int step, int n) {
  const int r = p + step;
  return r < 0 ? r + n : (r >= n ? r - n : r);
}

__device__ __forceinline__ LsMoveXY ls_eval_xy(const GDist& G, const HAC_AS1 int32_t* geo, int kg, int kls,
                                              int n, const uint16_t* tour, const uint16_t* pos,
                                              const float2* txy, int a, double min_gain, double e1,
                                              double e2, LsNodeXY& nd) {
  const int lane = lane_id();
  const bool pred_dir = lane >= 32;
  const int q = lane & 31;
  const bool in_list = q < kls;
  const int c = geo[(int64_t)a * kg + min(q, kls - 1)];
  const int step = pred_dir ? -1 : 1;
  const int pa = pos[a];
  const int pb = cyc_step(pa, step, n);
  const int b = tour[pb];
  const float2 xa = txy[pa], xb = txy[pb];
  const int pc = pos[c];
  const int pe = cyc_step(pc, step, n);
  const int e = tour[pe];
  const float2 xc = txy[pc], xe = txy[pe];
  const float lab = ls_len_xy(xa, xb), lac = ls_len_xy(xa, xc);
  // d(a,b) - d(a,c) > 0, as computed in FP64: c == b gives exactly 0, and
  // only list entries whose FP32 difference lies inside the bound are
  // decided in FP64
  const double g1f = (double)(lab - lac);
  bool g1pos = c != b && g1f > e1;
  double dab = 0.0, dac = 0.0;
  bool have64 = false;
  if (in_list && c != b && !(g1f > e1) && !(g1f < -e1)) {
    dab = G.len(a, b);
    dac = G.len(a, c);
    have64 = true;
    g1pos = dab - dac > 0.0;
  }
  nd = LsNodeXY{pa, b, c, pc, xa, xb, xc, lab, lac, g1pos};
  // a direction stops at the first list entry that cannot gain
  const uint64_t stop = __builtin_amdgcn_ballot_w64(in_list && !g1pos);
  const uint64_t stop_s = stop & 0xffffffffull, stop_p = stop >> 32;
  const int lim_s = stop_s ? (int)__builtin_ctzll(stop_s) : 32;
  const int lim_p = stop_p ? (int)__builtin_ctzll(stop_p) : 32;
  const bool cand = in_list && q < (pred_dir ? lim_p : lim_s) && e != a && c != b;
  const double gf = (double)((lab + ls_len_xy(xc, xe)) - (lac + ls_len_xy(xb, xe)));
  bool imp = gf > min_gain + e2;
  if (cand && !(gf > min_gain + e2) && !(gf < min_gain - e2)) {
    if (!have64) {
      dab = G.len(a, b);
      dac = G.len(a, c);
    }
    imp = (dab + G.len(c, e)) - (dac + G.len(b, e)) > min_gain;
  }
  imp = imp && cand;
  const uint64_t mi = __builtin_amdgcn_ballot_w64(imp);
  LsMoveXY m{0, a, 0, 0, 0, 0, 0, 0};
  if (mi) {
    // the path b..c (successor side) or c..b (predecessor side), or its
    // complement when that is shorter
    int i = pred_dir ? pc : pb, j = pred_dir ? pb : pc;
    int len = (j >= i ? j - i : j - i + n) + 1;
    if (2 * len > n) {
      const int ni = j + 1 == n ? 0 : j + 1, nj = i == 0 ? n - 1 : i - 1;
      i = ni;
      j = nj;
      len = n - len;
    }
    const int l = (int)__builtin_ctzll(mi);
    m.imp = 1;
    m.b = rd_lane(b, l);
    m.c = rd_lane(c, l);
    m.e = rd_lane(e, l);
    m.i = rd_lane(i, l);
    m.j = rd_lane(j, l);
    m.half = rd_lane(len, l) / 2;
  }
  return m;
}

template <class BP>
__device__ __forceinline__ void two_opt_block_xy(const InstDesc& D, uint16_t* tour, uint16_t* pos, uint16_t* queue,
                                                 BP inq, float2* txy, double min_gain, double e1, double e2) {
  __shared__ int sh_head, sh_count;
  __shared__ LsMoveXY sh_mv[LS_WAVES];
  const int n = D.n, kls = D.kls, kg = D.kg, lane = lane_id(), wave = threadIdx.x / WAVE;
  const int nw = (int)(blockDim.x / WAVE);  // 1 .. LS_WAVES entries per batch
  if (n < 5 || kls < 1) return;
  const GDist G(D);
  const HAC_AS1 int32_t* geo = as_global(D.geo);
  for (int s = threadIdx.x; s < n; s += blockDim.x) {
    const int v = tour[s];
    pos[v] = (uint16_t)s;
    queue[s] = (uint16_t)v;
    inq[v] = 1;
  }
  if (threadIdx.x == 0) {
    sh_head = 0;
    sh_count = n;
  }
  __syncthreads();
  // the node of the last applied move is examined again, in wave 0 of the
  // next batch, ahead of the queue entries
  int pend = -1;
  for (;;) {
    const int head = sh_head, count = sh_count;
    const int re = pend >= 0 ? 1 : 0;
    const int nq = min(nw - re, count);  // queue entries in this batch
    const int nb = nq + re;
    if (nb == 0) break;
    if (wave < nb) {
      int node = pend;
      if (wave >= re) {
        int slot = head + wave - re;
        if (slot >= n) slot -= n;
        node = queue[slot];
      }
      LsNodeXY nd;
      const LsMoveXY m = ls_eval_xy(G, geo, kg, kls, n, tour, pos, txy, node, min_gain, e1, e2, nd);
      if (lane == 0) sh_mv[wave] = m;
    }
    __syncthreads();
    // the first improving result in batch order (one entry per lane)
    const uint64_t fm = __builtin_amdgcn_ballot_w64(lane < nb && sh_mv[min(lane, LS_WAVES - 1)].imp);
    const int f = fm ? (int)__builtin_ctzll(fm) : -1;
    // the queue bookkeeping runs in the last wave, beside the reversal in
    // the others (one wave does both when the block has one)
    const int bw = nw - 1;
    if (wave == bw) {
      // queue entries consumed as a sequential scan would: all of them if
      // no move improves, else those up to and including the improving one
      const int used = f < 0 ? nq : max(0, f + 1 - re);
      if (lane < used) {
        int slot = head + lane;
        if (slot >= n) slot -= n;
        inq[queue[slot]] = 0;
      }
      int h = head + used;
      if (h >= n) h -= n;
      int cnt = count - used;
      if (f >= 0) {
        // the end nodes a, b, c, e (four distinct nodes) join the queue
        // tail in that order if absent, one lane each
        const bool mine = lane < 4;
        int x = 0;
        if (mine) {
          const LsMoveXY& mv = sh_mv[f];
          x = lane == 0 ? mv.a : (lane == 1 ? mv.b : (lane == 2 ? mv.c : mv.e));
        }
        const bool absent = mine && !inq[x];
        const uint32_t am = (uint32_t)__builtin_amdgcn_ballot_w64(absent) & 0xfu;
        if (absent) {
          int slot = h + cnt + __builtin_popcount(am & ((1u << lane) - 1u));
          if (slot >= n) slot -= n;
          queue[slot] = (uint16_t)x;
          inq[x] = 1;
        }
        cnt += __builtin_popcount(am);
      }
      if (lane == 0) {
        sh_head = h;
        sh_count = cnt;
      }
    }
    if (f < 0) {
      pend = -1;
      __syncthreads();
      continue;
    }
    // reverse positions i .. j (cyclic) of the tour and its coordinates
    const int ri = sh_mv[f].i, rj = sh_mv[f].j, half = sh_mv[f].half;
    pend = sh_mv[f].a;
    const int rthreads = bw > 0 ? bw * WAVE : WAVE;
    for (int s2 = (bw > 0 && wave == bw) ? half : (int)threadIdx.x; s2 < half; s2 += rthreads) {
      int pi = ri + s2;
      if (pi >= n) pi -= n;
      int pj = rj - s2;
      if (pj < 0) pj += n;
      const int ti = tour[pi], tj = tour[pj];
      const float2 xi = txy[pi], xj = txy[pj];
      tour[pi] = (uint16_t)tj;
      tour[pj] = (uint16_t)ti;
      txy[pi] = xj;
      txy[pj] = xi;
      pos[tj] = (uint16_t)pi;
      pos[ti] = (uint16_t)pj;
    }
    __syncthreads();
  }
}

// Working arrays of the 2-opt, by mode:
//   2: tour, pos and queue as uint16, in-queue flags as uint8 and an FP32
//      copy of the coordinates in tour order, all in LDS (15 bytes per
//      node, n < 65536, coordinate instances);
//   1: tour, pos and queue as int32 and the flags in LDS (13 bytes per node);
//   0: global memory (the tour in place, the rest in the work area).
static __host__ __device__ inline size_t ls_lds_need(int n, int mode) {
  if (mode == 2) return ((size_t)6 * n + 15) / 16 * 16 + ((size_t)n + 15) / 16 * 16 + (size_t)8 * n;
  if (mode == 1) return (((size_t)13 * n + 15) / 16) * 16;
  return 0;
}

// Mode 2's arrays in LDS: the tour as uint16 and its FP32 coordinates in
// tour order, loaded from tour_g; returns the largest coordinate magnitude
// (for the FP32 error bounds).  The positions, queue and flags follow.
__device__ __forceinline__ double ls_stage_xy(const InstDesc& D, const int32_t* tour_g, uint16_t* tour,
                                              float2* txy) {
  __shared__ double sh_m[LS_WAVES];
  const int n = D.n;
  double mloc = 0.0;
  const HAC_AS1 double* xy = as_global(D.xy);
  for (int s = threadIdx.x; s < n; s += blockDim.x) {
    const int v = tour_g[s];
    tour[s] = (uint16_t)v;
    txy[s] = make_float2((float)xy[2 * v], (float)xy[2 * v + 1]);
    mloc = fmax(mloc, fmax(fabs(xy[2 * s]), fabs(xy[2 * s + 1])));
  }
  for (int off = 32; off >= 1; off >>= 1) mloc = fmax(mloc, __shfl_xor(mloc, off));
  if ((threadIdx.x & (WAVE - 1)) == 0) sh_m[threadIdx.x / WAVE] = mloc;
  __syncthreads();
  double M = 0.0;
  for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) M = fmax(M, sh_m[w]);
  return M;
}

template <int MODE>
__device__ __forceinline__ void two_opt_tour(const InstDesc& D, int32_t* tour_g, double min_gain,
                                             int32_t* work) {
  extern __shared__ int32_t ls_lds[];
  const int n = D.n;
  if constexpr (MODE == 2) {
    uint16_t* tour = reinterpret_cast<uint16_t*>(ls_lds);
    uint16_t* pos = tour + n;
    uint16_t* queue = pos + n;
    uint8_t* inq = reinterpret_cast<uint8_t*>(ls_lds) + ((size_t)6 * n + 15) / 16 * 16;
    float2* txy = reinterpret_cast<float2*>(reinterpret_cast<uint8_t*>(inq) + ((size_t)n + 15) / 16 * 16);
    const double M = ls_stage_xy(D, tour_g, tour, txy);
    two_opt_block_xy(D, tour, pos, queue, inq, txy, min_gain, M * 0x1p-18, M * 0x1p-17);
    __syncthreads();
    for (int s = threadIdx.x; s < n; s += blockDim.x) tour_g[s] = tour[s];
  } else if constexpr (MODE == 1) {
    int32_t* tour = ls_lds;
    int32_t* pos = tour + n;
    int32_t* queue = pos + n;
    uint8_t* inq = reinterpret_cast<uint8_t*>(queue + n);
    for (int s = threadIdx.x; s < n; s += blockDim.x) tour[s] = tour_g[s];
    __syncthreads();
    two_opt_block(D, tour, pos, queue, inq, min_gain);
    __syncthreads();
    for (int s = threadIdx.x; s < n; s += blockDim.x) tour_g[s] = tour[s];
  } else {
    HAC_AS1 int32_t* tour = as_global(tour_g);
    HAC_AS1 int32_t* pos = as_global(work);
    HAC_AS1 int32_t* queue = pos + n;
    HAC_AS1 uint8_t* inq = reinterpret_cast<HAC_AS1 uint8_t*>(queue + n);
    two_opt_block(D, tour, pos, queue, inq, min_gain);
  }
  __threadfence_block();
  __syncthreads();
}

// 2-opt of the NN tour (preparation, local search enabled).  One block per
// instance.
template <int MODE>
__global__ void __launch_bounds__(LS_WAVES * WAVE) two_opt_nn_kernel(const InstDesc* insts) {
  const InstDesc& D = insts[blockIdx.x];
  if (!D.local_search || !D.sym || D.ls_op == 3) return;  // the ATSP takes the directed 2-opt
  two_opt_tour<MODE>(D, D.nn_tour, D.st->min_gain, D.ls_work);
  if (threadIdx.x < WAVE) {
    const double len = tour_length_wave(D, D.nn_tour);
    if (threadIdx.x == 0) {
      D.st->l_gb = len;
      D.st->l_ib = len;
    }
  }
}

// ------------------------------------------------------------------------
// Bounds and pheromone initialisation (eq. 5-6): tau <- tau_max.
// ------------------------------------------------------------------------
__device__ __forceinline__ void bounds_from_length(const InstDesc& D, double len, double& tmax,
                                                   double& tmin) {
  tmax = 1.0 / (D.rho * len);
  if (D.local_search)
    tmin = tmax / (2.0 * (double)D.n);
  else
    tmin = tmax * (1.0 - D.p_x) / (((double)(D.k - 1) / 2.0) * D.p_x);
}

__global__ void __launch_bounds__(256) init_kernel(const InstDesc* insts) {
  const InstDesc& D = insts[blockIdx.x];
  State* st = D.st;
  __shared__ float s_tmax;
  if (threadIdx.x == 0) {
    double len = st->l_gb;
    double tmax, tmin;
    bounds_from_length(D, len, tmax, tmin);
    st->tmax = tmax;
    st->tmin = tmin;
    st->tmax_f = (float)tmax;
    st->tmin_f = (float)tmin;
    st->t = 1;
    st->stall = 0;
    st->ugb = D.ugb_max;
    st->rb_valid = 0;
    st->restarts = 0;
    st->ib = 0;
    st->fallbacks = 0;
    st->err = 0;
    s_tmax = (float)tmax;
  }
  __syncthreads();
  const float tm = s_tmax;
  const int64_t nk = (int64_t)D.n * D.k;
  for (int64_t x = threadIdx.x; x < nk; x += blockDim.x) {
    const float w = tm * D.heur[x];
    D.tau[x] = tm;
    D.w[x] = w;
    D.cw[x] = make_uint2((uint32_t)D.cand[x], __float_as_uint(w));
  }
  for (int s = threadIdx.x; s < D.n; s += blockDim.x) D.t_gb[s] = D.nn_tour[s];
}

// Full scans for the nearest unvisited node.  Each lane takes nodes
// j = b0 + 64c + lane; CH chunks are loaded before any is examined, so a
// batch costs one memory round trip.  Every lane keeps its own best
// (key, j) in increasing j, then the wave reduces.  Visited bits past n
// are set, so j < n need not be tested against the bitset.
template <int CH, class V>
__device__ int scan_unvisited_lds(const double2* xy, int n, int i, V visited) {
  const int lane = lane_id();
  const double2 pi = xy[i];
  double bk = __builtin_huge_val();
  int bj = 0x7fffffff;
  for (int b0 = 0; b0 < n; b0 += CH * WAVE) {
    bool open[CH];
    double2 p[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int j = b0 + c * WAVE + lane;
      const int jc = j < n ? j : n - 1;  // reads stay inside this ant's bitset
      open[c] = j < n && !visited(jc);
      p[c] = xy[jc];
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const double dx = pi.x - p[c].x, dy = pi.y - p[c].y;
      const double kj = dx * dx + dy * dy;
      if (open[c] && kj < bk) {
        bk = kj;
        bj = b0 + c * WAVE + lane;
      }
    }
  }
  wave_argmin(bk, bj);
  return bj < n ? bj : n - 1;
}

template <int CH, class V>
__device__ int scan_unvisited_g(const GDist& G, int i, V visited) {
  const int lane = lane_id(), n = G.n;
  double bk = __builtin_huge_val();
  int bj = 0x7fffffff;
  if (G.xy) {
    const HAC_AS1 double* xy = G.xy;
    const double xi = xy[2 * i], yi = xy[2 * i + 1];
    for (int b0 = 0; b0 < n; b0 += CH * WAVE) {
      bool open[CH];
      double px[CH], py[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int j = b0 + c * WAVE + lane;
        const int jc = j < n ? j : n - 1;
        open[c] = j < n && !visited(jc);
        px[c] = xy[2 * jc];
        py[c] = xy[2 * jc + 1];
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const double dx = xi - px[c], dy = yi - py[c];
        const double kj = dx * dx + dy * dy;
        if (open[c] && kj < bk) {
          bk = kj;
          bj = b0 + c * WAVE + lane;
        }
      }
    }
  } else {
    const HAC_AS1 double* row = G.dist + (int64_t)i * n;
    for (int b0 = 0; b0 < n; b0 += CH * WAVE) {
      bool open[CH];
      double v[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int j = b0 + c * WAVE + lane;
        const int jc = j < n ? j : n - 1;
        open[c] = j < n && !visited(jc);
        v[c] = row[jc];
      }
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (open[c] && v[c] < bk) {
          bk = v[c];
          bj = b0 + c * WAVE + lane;
        }
    }
  }
  wave_argmin(bk, bj);
  return bj < n ? bj : n - 1;
}

// Nearest unvisited node to i by (key, index) over an ant's list of nodes
// that were unvisited at its previous scan; the scan compacts the list in
// place to the nodes still unvisited.  The list starts as the implicit
// range 0..n-1 (cnt < 0) and stays in increasing order (compaction keeps
// order), so each lane meets its nodes in increasing index order and the
// result is that of a scan over all nodes.  Only the nodes visited since
// the previous scan are examined again.
template <int CH, class V>
__device__ int scan_list(const GDist& G, const double2* xy_lds, int i, V visited, uint16_t* list,
                         int& cnt) {
  const int lane = lane_id(), n = G.n;
  const bool all = cnt < 0;
  const int m = all ? n : cnt;  // at least 1: an unvisited node exists
  double xi = 0.0, yi = 0.0;
  const HAC_AS1 double* row = nullptr;
  if (xy_lds) {
    xi = xy_lds[i].x;
    yi = xy_lds[i].y;
  } else if (G.xy) {
    xi = G.xy[2 * i];
    yi = G.xy[2 * i + 1];
  } else {
    row = G.dist + (int64_t)i * n;
  }
  double bk = __builtin_huge_val();
  int bj = 0x7fffffff;
  int out = 0;
  for (int b0 = 0; b0 < m; b0 += CH * WAVE) {
    int id[CH];
    bool open[CH];
    double ka[CH], kb[CH];
    // every load is unconditional (indices clamped into the list), so the
    // whole batch is one round trip per dependent level
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int x = min(b0 + c * WAVE + lane, m - 1);
      id[c] = all ? x : (int)list[x];
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int v = id[c];
      open[c] = (b0 + c * WAVE + lane < m) & !visited(v);
      if (xy_lds) {
        ka[c] = xy_lds[v].x;
        kb[c] = xy_lds[v].y;
      } else if (G.xy) {
        ka[c] = G.xy[2 * v];
        kb[c] = G.xy[2 * v + 1];
      } else {
        ka[c] = row[v];
      }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      double kj;
      if (row) {
        kj = ka[c];
      } else {
        const double dx = xi - ka[c], dy = yi - kb[c];
        kj = dx * dx + dy * dy;
      }
      if (open[c] && kj < bk) {
        bk = kj;
        bj = id[c];
      }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {  // positions written never exceed positions read
      const uint64_t mk = __builtin_amdgcn_ballot_w64(open[c]);
      const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
      if (open[c]) list[out + below] = (uint16_t)id[c];
      out += (int)__builtin_popcountll(mk);
    }
  }
  cnt = out;
  wave_argmin(bk, bj);
  return bj < n ? bj : n - 1;
}

// one chunk when the list fits in a wave, batches of CH otherwise
template <int CH, class V>
__device__ __forceinline__ int scan_list_any(const GDist& G, const double2* xy_lds, int i, V visited,
                                             uint16_t* list, int& cnt) {
  if (cnt >= 0 && cnt <= WAVE) return scan_list<1>(G, xy_lds, i, visited, list, cnt);
  return scan_list<CH>(G, xy_lds, i, visited, list, cnt);
}

// The geometric list holds the kg nearest nodes in (key, index) order, so
// its first unvisited entry, if any, is the answer; otherwise a full scan.
template <class V>
__device__ __forceinline__ int geo_first_unvisited(const HAC_AS1 int32_t* geo, int kg, int i,
                                                   V visited) {
  const int lane = lane_id();
  int g = 0;
  bool open = false;
  if (lane < kg) {
    g = geo[(int64_t)i * kg + lane];
    open = !visited(g);
  }
  const uint64_t m = __builtin_amdgcn_ballot_w64(open);
  return m ? rd_lane(g, __ffsll((unsigned long long)m) - 1) : -1;
}

// ------------------------------------------------------------------------
// Ant construction (Alg. 2, eq. 4).
//
// Per step, for the ant at node i with candidate row C_i:
//   open slots  = candidates whose visited bit is clear (LDS bitset)
//   E           = largest biased exponent of the open weights
//   q           = max(1, floor(w 2^(23-E))): the 24-bit FP32 significand
//                 shifted right by E minus the slot's exponent (exact)
//   r           = floor(U * sum q / 2^32) for the step's 32-bit uniform U
//   choice      = the open slot whose exclusive prefix <= r < inclusive
//                 prefix, i.e. the first one whose inclusive prefix exceeds r
// and, when no slot is open, the nearest unvisited node.
//
// Rows.  A wave64 VALU instruction occupies a 16-lane SIMD for four
// cycles, so a wave spent on one 10- or 20-slot row would leave most of
// the chip idle.  An ant therefore owns one 16-lane row of the wave (four
// ants of one instance per wave) and each lane holds S consecutive slots
// of the candidate row (S = 1, 2 or 4 for k <= 16, 32, 64).  Every
// reduction is a DPP operation inside the row: a butterfly max of the
// exponents, one prefix scan of the per-lane sums, a broadcast of the
// row total, and a butterfly OR that hands the chosen id to all lanes
// (exactly one slot of a live row passes the prefix test, so no search for
// a first lane is needed).  The lane of the chosen slot marks the visited
// bit with the bitset word it has just read.
//
// Exhausted rows look up their geometric list (the kg <= 64 nearest nodes
// in (distance, index) order, so the first unvisited entry is the answer)
// inside their own row; rows whose list is exhausted as well run a
// wave-wide scan of all nodes, one row after another.
//
// Lane u of a row holds the 32-bit Philox output of step s0 + u; the row
// shifts them down one lane per step, so the current draw always sits in
// lane 0.  Chosen nodes are buffered in lane (s mod 16) and written, with
// their edge lengths added in step order, once per 16 steps.  STAGED
// copies the instance's {candidate, weight} table and coordinates into
// LDS at the start of the launch.
// ------------------------------------------------------------------------

// lane Q of each 16-lane row, to the whole row (row_newbcast)
template <int Q>
__device__ __forceinline__ uint32_t row_bcast(uint32_t v) {
  return dpp_all<0x150 + Q>(v);
}
template <int Q>
__device__ __forceinline__ double row_bcast_f64(double v) {
  return __hiloint2double((int)row_bcast<Q>((uint32_t)__double2hiint(v)),
                          (int)row_bcast<Q>((uint32_t)__double2loint(v)));
}

// DPP shifts inside a row; lanes without a source read 0 (bound_ctrl)
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_zero(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, true);
}

// inclusive prefix sum inside each 16-lane row
__device__ __forceinline__ uint32_t row_scan(uint32_t v) {
  v += dpp_zero<0x111>(v);  // row_shr:1
  v += dpp_zero<0x112>(v);  // row_shr:2
  v += dpp_zero<0x114>(v);  // row_shr:4
  v += dpp_zero<0x118>(v);  // row_shr:8
  return v;
}

// With a grid and an unvisited list both available, the list is scanned
// once at most this many nodes are left: the nearest unvisited node is then
// far away in cells, while the compacted list is short.
constexpr int kListScanMax = 1024;

// STAGED: 0 the candidate table is read from global memory; 1 it is copied
// to LDS as 8-byte {id, weight} entries; 2 as uint16 ids and FP32 weights
// (six bytes per slot, for tables that do not fit as 8-byte entries); 3 as
// in 2 but without the coordinates, which leaves room for unvisited lists.
template <int STAGED, int S, bool BYTES, int GEO, bool GRID>
struct AntRows {
  int n, k, kg, u, g;
  const HAC_AS1 char* cw_g;       // the candidate table in global memory
  uint32_t k8;                    // bytes per table row (STAGED 2: of the id table)
  uint32_t w_from_id;             // STAGED 2: weight address = 2 x id address + w_from_id
  uint32_t lane_off[S];           // byte offset of slot min(S u + s, k - 1) (staged: its LDS address;
                                  // STAGED 2: its id's)
  int t_base[S];                  // 150, or 150 + 1024 for a slot at or past k (never open)
  uint32_t vmask[S];              // all ones for a slot below k, else 0
  uint32_t ra[S];                 // where this lane's slots of the current row are
  const double2* xy_lds;
  GDist D;
  const HAC_AS1 int32_t* geo;
  const HAC_AS1 uint64_t* geo16;  // uint16 lists, 16 x 8 bytes (64 entries) per node
  // how an exhausted row consults its geometric list: 0 not at all, 1 int32
  // lists, 2 uint16 lists a step ahead (a template parameter, so that each
  // kernel's step holds only its own mode's code)
  static constexpr int geo_mode = GEO;
  uint64_t glr;                   // mode 2: entries 4u .. 4u + 3 of the current node's list
  uint32_t* vis_wave;  // visited marks of the wave's live rows, vis_words apart
  uint32_t* vis_g;     // this row's marks (row 0's for an idle row, which never writes)
  int vis_words;       // BYTES: one byte per node, else one bit

  __device__ __forceinline__ const uint8_t* vbytes(const uint32_t* w) const {
    return reinterpret_cast<const uint8_t*>(w);
  }
  __device__ __forceinline__ bool visited(const uint32_t* w, int v) const {
    if constexpr (BYTES) return vbytes(w)[v] != 0;
    return (w[v >> 5] >> (v & 31)) & 1u;
  }
  // the row's own marks: only a live row's lane calls this
  __device__ __forceinline__ void mark(int v) {
    if constexpr (BYTES)
      reinterpret_cast<uint8_t*>(vis_g)[v] = 1;
    else
      atomicOr(&vis_g[v >> 5], 1u << (v & 31));
  }
  GridView grid;        // coordinate grid (grid.start null: none)
  uint16_t* list_wave;  // unvisited lists of the wave's live rows, list_stride apart (or null)
  int list_stride;
  int lcnt;             // this row's list length (-1: all nodes)
  int left;             // unvisited nodes before this step's choice (same in every row of the wave)
  bool live;
  int cur;       // the row's current node (same in all its lanes)
  uint32_t fallbacks;
  uint32_t row_max;     // STAGED 0: byte offset of the last table row

  __device__ __forceinline__ uint64_t entry(uint32_t a) const {
    if constexpr (STAGED == 1) {
      return *reinterpret_cast<const __attribute__((address_space(3))) uint64_t*>((uintptr_t)a);
    } else if constexpr (STAGED >= 2) {
      // the id (uint16) at a and its weight (FP32) at 2a + w_from_id
      const uint32_t id = *reinterpret_cast<const __attribute__((address_space(3))) uint16_t*>((uintptr_t)a);
      const uint32_t wb = *reinterpret_cast<const __attribute__((address_space(3))) uint32_t*>(
          (uintptr_t)(2u * a + w_from_id));
      return (uint64_t)id | ((uint64_t)wb << 32);
    } else {
      return *reinterpret_cast<const HAC_AS1 uint64_t*>(cw_g + a);
    }
  }
  // the current node's row, from its byte offset in the table
  __device__ __forceinline__ void set_row(uint32_t rb) {
#pragma unroll
    for (int s = 0; s < S; ++s) ra[s] = rb + lane_off[s];
  }

  // one decision for every row of the wave; U is the row's uniform
  __device__ __forceinline__ int step(uint32_t U) {
    uint64_t e[S];
#pragma unroll
    for (int s = 0; s < S; ++s) e[s] = entry(ra[s]);
    // mode 1: the int32 geometric list of the current node, needed only if
    // the row is exhausted, loaded now so that its latency hides behind the
    // step (mode 2 loaded the uint16 list at the end of the previous step)
    int gl[4] = {0, 0, 0, 0};  // entries 4u .. 4u + 3 of the list
    if (geo_mode == 1) {
      const uint32_t go = __umul24((uint32_t)cur, (uint32_t)kg);
#pragma unroll
      for (int q = 0; q < 4; ++q) gl[q] = geo[go + (uint32_t)min(4 * u + q, kg - 1)];
    }
    int c[S];
    uint32_t wb[S], mk[S], vw[S], bit[S];
    // t = 150 - (biased exponent), plus 512 once the slot's node is visited
    // and 1024 for a slot past k.  The row minimum is the shift that brings
    // the largest open weight to 24 integer bits, and it is at least 256
    // exactly when no slot is open (open slots give at most 149).
    int tmin = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      c[s] = (int)(uint32_t)e[s];
      wb[s] = (uint32_t)(e[s] >> 32);
      if constexpr (BYTES) {
        mk[s] = vbytes(vis_g)[c[s]];
      } else {
        vw[s] = vis_g[c[s] >> 5];
        bit[s] = 1u << (c[s] & 31);
        mk[s] = (vw[s] >> (c[s] & 31)) & 1u;
      }
      const int t = (int)(mk[s] << 9) + (t_base[s] - (int)(wb[s] >> 23));
      tmin = min(tmin, t);
    }
    const int sh = (int)row_reduce((uint32_t)tmin, OpMinI());
    // q = floor(w 2^(23-E)) with E the largest floor(log2 w) of the open
    // slots: scaling by a power of two is exact and the conversion truncates;
    // open slots get at least 1, closed ones (weight masked to 0) exactly 0
    uint32_t q[S], a[S], acc = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t wm = wb[s] & (mk[s] - 1u) & vmask[s];
      const uint32_t op = (mk[s] ^ 1u) & vmask[s] & 1u;
      q[s] = max(__float2uint_rz(__builtin_ldexpf(__uint_as_float(wm), sh)), op);
      acc += q[s];
      a[s] = acc;
    }
    // inclusive prefix and row total, side by side
    const uint32_t P = row_scan(acc);
    const uint32_t tot = row_reduce(acc, OpAdd());
    uint32_t ex[S];  // exclusive prefix of each slot, ready before r
#pragma unroll
    for (int s = 0; s < S; ++s) {
      ex[s] = P - acc + a[s] - q[s];
      asm volatile("" : "+v"(ex[s]));  // kept as computed: one subtraction after r
    }
    const uint32_t r = __umulhi(U, tot);
    uint32_t pick = 0, pick_off = 0, wv = 0;
    int wi = 0;
    bool hit = false;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      // exclusive prefix <= r < inclusive prefix, i.e. r - exclusive < q
      const bool h = r - ex[s] < q[s];
      pick = h ? (uint32_t)c[s] : pick;
      pick_off = h ? __umul24((uint32_t)c[s], k8) : pick_off;
      if constexpr (!BYTES) {
        wi = h ? (c[s] >> 5) : wi;
        wv = h ? (vw[s] | bit[s]) : wv;
      }
      hit |= h;
    }
    // Exactly one slot of an open row passes the test.  Whatever happens,
    // the node and a global table row stay in range below, so a broken
    // pick gives an in-range wrong choice, never a wild address; it marks
    // a node the ant does not take, so its tour is no permutation, which
    // the tour checksums at the end of the launch report.
    const bool exhausted = sh >= 256;
    const uint64_t exh_mask = __builtin_amdgcn_ballot_w64(exhausted);
    int j = (int)row_reduce(pick, OpOr());
    // the next row's byte offset, alongside j.  At most one lane of a row
    // holds a nonzero offset, so after three levels one half of the row holds
    // it and the other zero, and the last level may add instead of or: for one
    // slot per lane it then adds the lane's own slot offset in the same step.
    uint32_t ro = pick_off;
    ro |= dpp_all<0xB1>(ro);
    ro |= dpp_all<0x4E>(ro);
    ro |= dpp_all<0x141>(ro);
    uint32_t rrow = ro + dpp_all<0x140>(ro);
    if constexpr (STAGED == 0) rrow = min(rrow, row_max);  // LDS reads out of range cannot fault
    if constexpr (S == 1) {
      ra[0] = rrow + lane_off[0];
    } else {
      set_row(rrow);
    }
    // the lane of the chosen slot marks it (only this row writes its marks;
    // a bitset word is rewritten with the value it has just read)
    if (hit && live) {
      if constexpr (BYTES)
        reinterpret_cast<uint8_t*>(vis_g)[pick] = 1;
      else
        vis_g[wi] = wv;
    }
    j = (int)min((uint32_t)j, (uint32_t)(n - 1));
    if (__builtin_expect(exh_mask != 0, 0)) {  // rare: keeps the fallback out of the step's straight line
      j = fallback(exhausted, j, gl);
      if (exhausted) set_row(__umul24((uint32_t)j, k8));
    }
    // mode 2: the next node's list, a whole step ahead of its use
    if (geo_mode == 2) glr = geo16[(uint32_t)j * 16u + (uint32_t)u];
    --left;
    return j;
  }

  __device__ __forceinline__ int fallback(bool exhausted, int j, int (&gl)[4]) {
    int jg = -1;
    if (geo_mode == 2) {
      gl[0] = (int)(glr & 0xffffu);
      gl[1] = (int)((glr >> 16) & 0xffffu);
      gl[2] = (int)((glr >> 32) & 0xffffu);
      gl[3] = (int)(glr >> 48);
    }
    if (exhausted && geo_mode != 0) {  // whole rows: the geometric list, four entries per lane
      bool o[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] = (4 * u + q < kg) & !visited(vis_g, gl[q]);  // ids are valid in every lane
      const uint64_t bm = __builtin_amdgcn_ballot_w64(o[0] | o[1] | o[2] | o[3]);
      const uint32_t field = (uint32_t)(bm >> (16 * g)) & 0xffffu;
      if (field) {
        const int f = (int)__builtin_ctz(field);
        const int first = o[0] ? gl[0] : (o[1] ? gl[1] : (o[2] ? gl[2] : gl[3]));
        jg = (int)row_reduce(u == f ? (uint32_t)first : 0u, OpOr());
      }
    }
    // live rows still without a node: wave-wide scans, one row at a time
    uint64_t miss = __builtin_amdgcn_ballot_w64(exhausted & (jg < 0) & (u == 0) & live);
    while (miss) {
      const int lead = (int)__builtin_ctzll(miss);
      miss &= miss - 1;
      const int gg = lead >> 4;
      const int ii = rd_lane(cur, lead);
      const uint32_t* vw_ = vis_wave + gg * vis_words;
      using VisT = typename std::conditional<BYTES, VisBytes, VisBits>::type;
      VisT vv;
      if constexpr (BYTES)
        vv = VisBytes{vbytes(vw_)};
      else
        vv = VisBits{vw_};
      int jj;
      if (GRID && grid.start && (!list_wave || left > kListScanMax)) {
        const double xi = xy_lds ? xy_lds[ii].x : D.xy[2 * ii];
        const double yi = xy_lds ? xy_lds[ii].y : D.xy[2 * ii + 1];
        jj = grid_nearest(grid, n, xi, yi, vv);
      } else if (list_wave) {
        int cnt = rd_lane(lcnt, lead);
        jj = (STAGED && xy_lds) ? scan_list_any<4>(D, xy_lds, ii, vv, list_wave + gg * list_stride, cnt)
                                : scan_list_any<8>(D, nullptr, ii, vv, list_wave + gg * list_stride, cnt);
        if (g == gg) lcnt = cnt;
      } else {
        jj = (STAGED && xy_lds) ? scan_unvisited_lds<4>(xy_lds, n, ii, vv)
                                : scan_unvisited_g<8>(D, ii, vv);
      }
      if (g == gg) jg = jj;
    }
    // idle rows take row 0's node, so that they stay in step with it (they
    // read its marks and draws) instead of wandering off and sending the
    // wave into this branch on steps where no live row is exhausted
    const int jg0 = rd_lane(jg, 0);
    if (!live) jg = jg0;
    if (exhausted) {
      j = jg < 0 ? 0 : jg;
      if (u == 0 && live) {
        mark(j);
        fallbacks++;
      }
    }
    return j;
  }
};

template <int Q>
__device__ __forceinline__ void sum_row_in_order(double& len, double d) {
  if constexpr (Q < 16) {
    len += row_bcast_f64<Q>(d);
    sum_row_in_order<Q + 1>(len, d);
  }
}

template <int STAGED, int S, bool BYTES, int GEO, bool GRID>
__global__ void __launch_bounds__(kMaxConstructWaves * WAVE) construct_kernel(const InstDesc* __restrict__ insts,
                                                         const BlockMap* __restrict__ map,
                                                         int ants_per_block, int rows_per_wave,
                                                         int lds_bytes, int step_cap) {
  const BlockMap bm = map[blockIdx.x];
  if (bm.inst < 0) return;
  const InstDesc I = insts[bm.inst];  // by value: the fields stay in registers
  const int t = I.st->t;
  if (t > I.iterations || I.st->err) return;
  extern __shared__ uint32_t lds[];
  const int n = I.n, k = I.k, lane = lane_id(), wave = threadIdx.x / WAVE;
  const int rpw = rows_per_wave;  // rows of a wave that carry ants (the others shadow row 0)
  const ConstructLds L = construct_lds_layout(n, k, ants_per_block, rpw, STAGED, true, BYTES);
  const bool use_list = n <= 65535 && L.total <= (size_t)lds_bytes;
  const int vis_words = (int)L.vis_words;
  const int rows = (int)L.rows;  // bitsets (and lists) of every row of the block
  const int list_off = rows * vis_words;
  const int staged_off = use_list ? list_off + rows * (int)L.list_words : list_off;
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const double2* xy_lds = nullptr;
  // words of the staged table before the coordinates, and of its id part
  const uint32_t ids_words = STAGED >= 2 ? (uint32_t)(staged_ids_bytes(n, k) / 4) : 0u;
  const uint32_t table_words = STAGED >= 2 ? ids_words + (uint32_t)((((size_t)n * k * 4 + 15) / 16) * 4)
                                           : (uint32_t)((((size_t)n * k * 8 + 15) / 16) * 4);
  if (STAGED) {
    const HAC_AS1 uint64_t* src = reinterpret_cast<const HAC_AS1 uint64_t*>(as_global(I.cw));
    if constexpr (STAGED >= 2) {
      // the {id, weight} table, split into uint16 ids and FP32 weights
      uint16_t* dst_id = reinterpret_cast<uint16_t*>(lds + staged_off);
      uint32_t* dst_w = lds + staged_off + ids_words;
      const int nk = n * k;
      for (int x = threadIdx.x; x < nk; x += blockDim.x) {
        const uint64_t e = src[x];
        dst_id[x] = (uint16_t)(uint32_t)e;
        dst_w[x] = (uint32_t)(e >> 32);
      }
    } else {
      u32x4* dst = reinterpret_cast<u32x4*>(lds + staged_off);
      const HAC_AS1 u32x4* src4 = reinterpret_cast<const HAC_AS1 u32x4*>(src);
      const int vec = (n * k * 8 + 15) / 16;
      for (int x = threadIdx.x; x < vec; x += blockDim.x) dst[x] = src4[x];
    }
    if (STAGED != 3 && I.xy) {
      u32x4* dxy = reinterpret_cast<u32x4*>(lds + staged_off + table_words);
      const HAC_AS1 u32x4* sxy = reinterpret_cast<const HAC_AS1 u32x4*>(as_global(I.xy));
      for (int x = threadIdx.x; x < n; x += blockDim.x) dxy[x] = sxy[x];
      xy_lds = reinterpret_cast<const double2*>(dxy);
    }
    __syncthreads();
  }
  const int first_ant = bm.ant0 + wave * rpw;
  if (wave * rpw >= ants_per_block || first_ant >= I.ants) return;  // whole wave idle

  AntRows<STAGED, S, BYTES, GEO, GRID> A{};
  A.n = n;
  A.k = k;
  A.kg = I.kg;
  A.u = lane & 15;
  A.g = lane >> 4;
  const int row = wave * rpw + A.g;
  A.live = A.g < rpw && row < ants_per_block && bm.ant0 + row < I.ants;
  // idle rows shadow the wave's first ant step for step, reading its bitset
  // and writing nothing, so only live rows need LDS
  const int ant = A.live ? bm.ant0 + row : first_ant;
  A.cw_g = reinterpret_cast<const HAC_AS1 char*>(as_global(I.cw));
  A.k8 = (STAGED >= 2 ? 2u : 8u) * (uint32_t)k;
  // LDS addresses of the staged ids and weights
  const uint32_t table_at =
      (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint32_t*)(lds + staged_off);
  const uint32_t weights_at = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint32_t*)(
      lds + staged_off + ids_words);
  A.w_from_id = weights_at - 2u * table_at;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int slot = S * A.u + s;
    A.lane_off[s] = (STAGED >= 2 ? 2u : 8u) * (uint32_t)min(slot, k - 1) + (STAGED ? table_at : 0u);
    A.t_base[s] = slot < k ? 150 : 150 + 1024;
    A.vmask[s] = slot < k ? 0xffffffffu : 0u;
    // opaque to the optimiser, so that the masking stays plain ALU work off
    // the step's dependency chain instead of selects on it
    asm volatile("" : "+v"(A.t_base[s]), "+v"(A.vmask[s]));
  }
  A.xy_lds = xy_lds;
  A.D = GDist(I);
  if (GRID) A.grid = grid_view(I);
  A.geo = as_global(I.geo);
  A.geo16 = reinterpret_cast<const HAC_AS1 uint64_t*>(as_global(I.geo16));
  A.vis_words = vis_words;
  A.vis_wave = lds + wave * rpw * vis_words;
  A.vis_g = A.vis_wave + (A.live ? A.g : 0) * vis_words;
  A.list_stride = 2 * (int)L.list_words;
  A.list_wave = use_list ? reinterpret_cast<uint16_t*>(lds + list_off) + wave * rpw * A.list_stride : nullptr;
  A.lcnt = -1;

  for (int w = lane; w < rpw * vis_words; w += WAVE) {
    uint32_t v = 0;  // bytes: all clear; bits: the bits past n are set
    if (!BYTES) {
      const int lo = (w % vis_words) * 32;
      if (lo >= n)
        v = 0xffffffffu;
      else if (lo + 32 > n)
        v = ~((1u << (n - lo)) - 1u);
    }
    A.vis_wave[w] = v;
  }
  __builtin_amdgcn_wave_barrier();

  const uint32_t k0 = I.seed_lo, k1 = I.seed_hi;
  HAC_AS1 int32_t* my_tour = as_global(I.tours) + (int64_t)ant * n;
  uint32_t rnd = philox_x0((uint32_t)A.u, (uint32_t)ant, (uint32_t)t, 0u, k0, k1);
  const int start = (int)__umulhi(row_bcast<0>(rnd), (uint32_t)n);
  rnd = dpp_zero<0x101>(rnd);  // row_shl:1, step 1's draw to lane 0
  A.cur = start;
  A.set_row(__umul24((uint32_t)start, A.k8));
  if (GEO == 2) A.glr = A.geo16[(uint32_t)start * 16u + (uint32_t)A.u];
  if (A.u == 0 && A.live) A.mark(start);
  A.fallbacks = 0;
  A.row_max = (uint32_t)(n - 1) * A.k8;
  A.left = n - 1;
  int tb = start;     // lane (s mod 16) holds T[s] of the current block of 16 steps
  int carry = start;  // T[s0 - 1]
  double len = 0.0;
  uint32_t csum = 0, csq = 0;  // sum and sum of squares (mod 2^32) of this lane's tour entries
  int q0 = 1;
  // a timing launch of the tuner stops after step_cap tour positions
  const int n_pos = min(n, step_cap);
  for (int s0 = 0; s0 < n_pos; s0 += 16) {
    if (s0 > 0) {
      rnd = philox_x0((uint32_t)(s0 + A.u), (uint32_t)ant, (uint32_t)t, 0u, k0, k1);
      q0 = 0;
    }
    const int cnt = min(16, n_pos - s0);
    for (int q = q0; q < cnt; ++q) {
      const int j = A.step(row_bcast<0>(rnd));
      rnd = dpp_zero<0x101>(rnd);
      tb = A.u == q ? j : tb;
      A.cur = j;
    }
    // write T[s0 .. s0+cnt-1] and add their incoming edges in step order
    if (A.live && A.u < cnt) my_tour[s0 + A.u] = tb;
    if (A.u < cnt) {
      csum += (uint32_t)tb;
      csq += __umul24((uint32_t)tb, (uint32_t)tb);  // node ids are below 2^24
    }
    int prev = (int)dpp_zero<0x111>((uint32_t)tb);  // T[s - 1] from the lane below
    if (A.u == 0) prev = carry;
    double dl = 0.0;
    if (A.u < cnt && s0 + A.u >= 1) {
      if (STAGED && xy_lds) {
        const double2 pa = xy_lds[prev], pb = xy_lds[tb];
        const double dx = pa.x - pb.x, dy = pa.y - pb.y;
        dl = sqrt(dx * dx + dy * dy);
      } else {
        dl = A.D.len(prev, tb);
      }
    }
    sum_row_in_order<0>(len, dl);  // adding 0.0 past the end leaves len unchanged
    carry = A.cur;
  }
  if (n_pos < n) return;  // a partial tour: no length, no checks
  if (STAGED && xy_lds) {
    const double2 pa = xy_lds[carry], pb = xy_lds[start];
    const double dx = pa.x - pb.x, dy = pa.y - pb.y;
    len += sqrt(dx * dx + dy * dy);
  } else {
    len += A.D.len(carry, start);
  }
  // the tour must be a permutation of 0..n-1: both checksums of the row
  // against their closed forms
  csum = row_reduce(csum, OpAdd());
  csq = row_reduce(csq, OpAdd());
  if (A.live && A.u == 0 && !tour_checksums_ok(n, csum, csq)) atomicOr(&I.st->err, 1u);
  if (A.live && A.u == 0) {
    I.lens[ant] = len;
    if (A.fallbacks) atomicAdd(&I.st->fallbacks, (unsigned long long)A.fallbacks);
  }
}

// ------------------------------------------------------------------------
// Local search on the iteration-best tour (one wave per instance).
// ------------------------------------------------------------------------
__device__ void iteration_best_wave(const InstDesc& D, int& ib, double& lib) {
  const int lane = lane_id();
  double bk = __builtin_huge_val();
  int bi = 0x7fffffff;
  for (int a = lane; a < D.ants; a += WAVE) {
    double v = D.lens[a];
    if (key_less(v, a, bk, bi)) {
      bk = v;
      bi = a;
    }
  }
  wave_argmin(bk, bi);
  ib = bi;
  lib = bk;
}

// Local search of one iteration.  local_search = 1: block (i, 0) improves
// a copy of instance i's iteration-best tour.  local_search = 2 (Alg. 1's
// placement): block (i, y) improves ant tours y, y + gridDim.y, ... in place
// and replaces their lengths, so the iteration best is then taken among the
// improved tours.
template <int MODE>
__global__ void __launch_bounds__(LS_WAVES * WAVE) local_search_kernel(const InstDesc* insts) {
  const InstDesc& D = insts[blockIdx.x];
  if (!D.local_search || !D.sym || D.ls_op == 3 || D.st->t > D.iterations || D.st->err) return;
  const int n = D.n;
  if (D.local_search == 2) {
    for (int a = blockIdx.y; a < D.ants; a += gridDim.y) {
      int32_t* tour = D.tours + (int64_t)a * n;
      two_opt_tour<MODE>(D, tour, D.st->min_gain, D.ls_work + (int64_t)a * 3 * n);
      if (threadIdx.x < WAVE) {
        const double len = tour_length_wave(D, tour);
        if (threadIdx.x == 0) D.lens[a] = len;
      }
      __syncthreads();
    }
    return;
  }
  if (blockIdx.y != 0) return;
  __shared__ int sh_ib;
  if (threadIdx.x < WAVE) {
    int ib;
    double lib;
    iteration_best_wave(D, ib, lib);
    if (threadIdx.x == 0) sh_ib = ib;
  }
  __syncthreads();
  const int ib = sh_ib;
  const int32_t* src = D.tours + (int64_t)ib * n;
  for (int s = threadIdx.x; s < n; s += blockDim.x) D.t_ib[s] = src[s];
  __threadfence_block();
  __syncthreads();
  two_opt_tour<MODE>(D, D.t_ib, D.st->min_gain, D.ls_work);
  if (threadIdx.x < WAVE) {
    const double len = tour_length_wave(D, D.t_ib);
    if (threadIdx.x == 0) {
      D.st->ib = ib;
      D.st->l_ib = len;
    }
  }
}

// ------------------------------------------------------------------------
// 3-opt for symmetric instances (Section III-D).  The search is the
// 2-opt's over a larger neighbourhood: for node a its 2-opt moves come
// first (ls_eval, in the 2-opt's order); if none improves, its segment
// exchanges.  With t2 the next node after t1 = a in the direction (the
// successor side, then the predecessor side), t3 runs over a's list while
// g1 = d(t1,t2) - d(t1,t3) > 0, t4 is the node before t3, t5 runs over
// t4's list while g2 = (g1 + d(t4,t3)) - d(t4,t5) > 0 and must come after
// t3 or be t1, and t6 is the node before t5; the move replaces (t1,t2),
// (t4,t3), (t6,t5) with (t1,t3), (t6,t2), (t4,t5), so the segments t2..t4
// and t3..t6 trade places, each keeping its order.  The first move whose
// gain ((d12 + d43) + d65) - ((d13 + d45) + d62) exceeds the threshold is
// applied, its end nodes t1 .. t6 are queued in that order if absent, and
// a is examined again; a search applies at most 64 n moves.
//
// A wave examines one node: for each t3 in list order, lanes 0..31 take
// t4's list entries on the successor side and lanes 32..63 on the
// predecessor side, so that the first improving entry of a side is one
// ballot away; the successor side's first move anywhere in t3's order
// comes before any predecessor-side move.
// ------------------------------------------------------------------------
struct Ls3Move {
  int imp, dir, t1, t2, t3, t4, t5, t6, r3, end;  // end: steps from t1 to t6
};

template <class IP>
__device__ Ls3Move ls3_eval(const GDist& G, const HAC_AS1 int32_t* geo, int kg, int kls, int n, IP tour,
                            IP pos, int a, double min_gain) {
  const int lane = lane_id();
  const int dir = lane >= 32 ? 1 : 0;
  const int q5 = lane & 31;
  const bool in5 = q5 < kls;
  const int p1 = pos[a];
  const int t2 = dir ? tour[p1 == 0 ? n - 1 : p1 - 1] : tour[p1 + 1 == n ? 0 : p1 + 1];
  const double d12 = G.len(a, t2);
  bool s_live = true, p_live = true, p_found = false;
  Ls3Move pm{0, 1, a, 0, 0, 0, 0, 0, 0, 0};
  for (int q = 0; q < kls && (s_live || p_live); ++q) {
    const int t3 = geo[(int64_t)a * kg + q];
    const double d13 = G.len(a, t3);
    const double g1 = d12 - d13;
    // a side stops at the first t3 that cannot gain
    const uint64_t gm = __builtin_amdgcn_ballot_w64(g1 > 0.0);
    s_live = s_live && (gm & 1ull);
    p_live = p_live && ((gm >> 32) & 1ull);
    const bool live = dir ? p_live : s_live;
    const int r3 = dir ? (p1 - pos[t3] + n) % n : (pos[t3] - p1 + n) % n;
    const bool use3 = live && r3 >= 2;
    int t4 = 0, t5 = 0, t6 = 0, r5 = 0;
    double d43 = 0.0, d45 = 0.0, g2 = 0.0;
    if (use3) {
      const int p3 = pos[t3];
      t4 = dir ? tour[p3 + 1 == n ? 0 : p3 + 1] : tour[p3 == 0 ? n - 1 : p3 - 1];
      d43 = G.len(t4, t3);
      t5 = geo[(int64_t)t4 * kg + min(q5, kls - 1)];
      d45 = G.len(t4, t5);
      g2 = (g1 + d43) - d45;
      r5 = dir ? (p1 - pos[t5] + n) % n : (pos[t5] - p1 + n) % n;
    }
    // t4's list stops at the first entry that cannot gain
    const uint64_t stop = __builtin_amdgcn_ballot_w64(use3 && in5 && !(g2 > 0.0));
    const uint64_t stop_s = stop & 0xffffffffull, stop_p = stop >> 32;
    const int lim = dir ? (stop_p ? (int)__builtin_ctzll(stop_p) : 32) : (stop_s ? (int)__builtin_ctzll(stop_s) : 32);
    const bool cand = use3 && in5 && q5 < lim && (r5 > r3 || r5 == 0);
    bool imp = false;
    double gain = 0.0;
    if (cand) {
      const int p5 = pos[t5];
      t6 = dir ? tour[p5 + 1 == n ? 0 : p5 + 1] : tour[p5 == 0 ? n - 1 : p5 - 1];
      gain = ((d12 + d43) + G.len(t6, t5)) - ((d13 + d45) + G.len(t6, t2));
      imp = gain > min_gain;
    }
    const uint64_t mi = __builtin_amdgcn_ballot_w64(imp);
    const uint64_t ms = mi & 0xffffffffull, mp = mi >> 32;
    if (ms) {
      const int l = (int)__builtin_ctzll(ms);
      Ls3Move m{1, 0, a, rd_lane(t2, l), t3, rd_lane(t4, l), rd_lane(t5, l), rd_lane(t6, l), rd_lane(r3, l), 0};
      m.end = (rd_lane(r5, l) == 0 ? n : rd_lane(r5, l)) - 1;
      return m;
    }
    if (mp && !p_found) {
      const int l = 32 + (int)__builtin_ctzll(mp);
      pm = Ls3Move{1, 1, a, rd_lane(t2, l), t3, rd_lane(t4, l), rd_lane(t5, l), rd_lane(t6, l), rd_lane(r3, l), 0};
      pm.end = (rd_lane(r5, l) == 0 ? n : rd_lane(r5, l)) - 1;
      p_found = true;
      p_live = false;
    }
  }
  if (p_found) return pm;
  return Ls3Move{0, 0, a, 0, 0, 0, 0, 0, 0, 0};
}

// Mode 2 of the 3-opt keeps the 2-opt's mode-2 arrays in LDS (uint16 tour,
// positions and queue, and the FP32 coordinates in tour order) and decides
// each test from FP32 distances when the result lies outside its error
// bound, else in FP64 from global memory, so every decision is the FP64
// one.  With every distance within 17 u M of its FP64 value (u = 2^-24, M
// the largest coordinate magnitude) and each FP32 addition rounding a value
// of at most 2 sqrt(2) M per distance it sums:
//   g1 = d12 - d13                        (2 distances)  within E1 = 2^-18 M,
//   g2 = (g1 + d43) - d45                 (4 distances)  within E2 = 2^-17 M,
//   ((d12 + d43) + d65) - ((d13 + d45) + d62)  (6)       within E3 = 2^-16 M.
// The 2-opt evaluation of a has just read a's list, one entry per lane of
// each half, with positions, coordinates, distances and g1 (nd); the
// exchange search adds each entry's steps from t1 and its t4 on that half's
// side, and t3's loop reads these from lane q of the half; t4's list is
// loaded two t3 ahead of its use.

__device__ __forceinline__ int side_lane(int v, int q, int dir) {
  const int s = __builtin_amdgcn_readlane(v, q);
  const int p = __builtin_amdgcn_readlane(v, q + 32);
  return dir ? p : s;
}

__device__ __forceinline__ float side_lane_f(float v, int q, int dir) {
  return __int_as_float(side_lane(__float_as_int(v), q, dir));
}

template <bool ABORT>
__device__ Ls3Move ls3_eval_xy(const GDist& G, const HAC_AS1 int32_t* geo, int kg, int kls, int n,
                               const uint16_t* tour, const uint16_t* pos, const float2* txy, int a,
                               const LsNodeXY& nd, double min_gain, double e2, double e3, int* first,
                               int wave) {
  const int lane = lane_id();
  const int dir = lane >= 32 ? 1 : 0;
  const int step = dir ? -1 : 1;
  const int q5 = lane & 31;
  const bool in5 = q5 < kls;
  const int p1 = nd.pa, t2 = nd.b;
  const float2 x2 = nd.xb;
  const float l12 = nd.lab;
  // list entry q5 of a (t3 = nd.c): its steps from t1 in this half's
  // direction, the node before it (t4) and the FP32 distances d13, d43
  const int t3l = nd.c, p3l = nd.pc;
  int r3l = dir ? p1 - p3l : p3l - p1;
  if (r3l < 0) r3l += n;
  const int p4l = cyc_step(p3l, -step, n);
  const int t4l = tour[p4l];
  const float2 x4l = txy[p4l];
  const float l13l = nd.lac, l43l = ls_len_xy(x4l, nd.xc);
  // ABORT: the lowest wave of the round with an improving move so far; once
  // it is ahead of this one, this wave's result will be dropped, so it stops
  const int fl0 = ABORT ? *(volatile int*)first : LS_WAVES;
  // a side stops at the first t3 that cannot gain (g1 as FP64 decides it)
  const uint64_t gstop = __builtin_amdgcn_ballot_w64(in5 && !nd.g1pos);
  const uint64_t gs = gstop & 0xffffffffull, gp = gstop >> 32;
  const int lim_s = min(gs ? (int)__builtin_ctzll(gs) : 32, kls);
  const int lim_p = min(gp ? (int)__builtin_ctzll(gp) : 32, kls);
  bool p_found = false;
  Ls3Move pm{0, 1, a, 0, 0, 0, 0, 0, 0, 0};
  if (ABORT && fl0 < wave) return pm;  // no move (imp 0)
  // t4's list entry q5 for the next two t3, loaded two steps ahead of use
  const int qmax = max(lim_s, lim_p);
  const int q5c = min(q5, kls - 1);
  int t5n = 0, t5nn = 0;
  if (qmax > 0) t5n = geo[(int64_t)side_lane(t4l, 0, dir) * kg + q5c];
  if (qmax > 1) t5nn = geo[(int64_t)side_lane(t4l, 1, dir) * kg + q5c];
  for (int q = 0; q < lim_s || (q < lim_p && !p_found); ++q) {
    const int t5 = t5n;
    t5n = t5nn;
    if (q + 2 < qmax) t5nn = geo[(int64_t)side_lane(t4l, q + 2, dir) * kg + q5c];
    const int fl = ABORT ? *(volatile int*)first : LS_WAVES;
    const bool live = dir ? (q < lim_p && !p_found) : q < lim_s;
    const int t3 = rd_lane(t3l, q);
    const int r3 = side_lane(r3l, q, dir);
    const bool use3 = live && r3 >= 2;
    int t4 = 0, t6 = 0, r5 = 0, p5 = 0;
    float l13 = 0.0f, l43 = 0.0f, l45 = 0.0f;
    float2 x5 = make_float2(0.0f, 0.0f);
    bool g2pos = false;
    if (use3) {
      t4 = side_lane(t4l, q, dir);
      const float2 x4 = make_float2(side_lane_f(x4l.x, q, dir), side_lane_f(x4l.y, q, dir));
      l13 = side_lane_f(l13l, q, dir);
      l43 = side_lane_f(l43l, q, dir);
      p5 = pos[t5];
      x5 = txy[p5];
      l45 = ls_len_xy(x4, x5);
      const float g2f = ((l12 - l13) + l43) - l45;
      g2pos = (double)g2f > e2;
      if (in5 && !g2pos && !((double)g2f < -e2)) {
        const double g1 = G.len(a, t2) - G.len(a, t3);
        g2pos = (g1 + G.len(t4, t3)) - G.len(t4, t5) > 0.0;
      }
      r5 = dir ? p1 - p5 : p5 - p1;
      if (r5 < 0) r5 += n;
    }
    // t4's list stops at the first entry that cannot gain
    const uint64_t stop = __builtin_amdgcn_ballot_w64(use3 && in5 && !g2pos);
    const uint64_t stop_s = stop & 0xffffffffull, stop_p = stop >> 32;
    const int lim = dir ? (stop_p ? (int)__builtin_ctzll(stop_p) : 32) : (stop_s ? (int)__builtin_ctzll(stop_s) : 32);
    const bool cand = use3 && in5 && q5 < lim && (r5 > r3 || r5 == 0);
    bool imp = false;
    if (cand) {
      const int p6 = cyc_step(p5, -step, n);
      t6 = tour[p6];
      const float2 x6 = txy[p6];
      const float gf = ((l12 + l43) + ls_len_xy(x6, x5)) - ((l13 + l45) + ls_len_xy(x6, x2));
      imp = (double)gf > min_gain + e3;
      if (!imp && !((double)gf < min_gain - e3)) {
        const double d12 = G.len(a, t2), d13 = G.len(a, t3), d43 = G.len(t4, t3), d45 = G.len(t4, t5);
        imp = ((d12 + d43) + G.len(t6, t5)) - ((d13 + d45) + G.len(t6, t2)) > min_gain;
      }
    }
    const uint64_t mi = __builtin_amdgcn_ballot_w64(imp);
    const uint64_t ms = mi & 0xffffffffull, mp = mi >> 32;
    if (ms) {
      const int l = (int)__builtin_ctzll(ms);
      Ls3Move m{1, 0, a, rd_lane(t2, l), t3, rd_lane(t4, l), rd_lane(t5, l), rd_lane(t6, l), rd_lane(r3, l), 0};
      m.end = (rd_lane(r5, l) == 0 ? n : rd_lane(r5, l)) - 1;
      return m;
    }
    if (mp && !p_found) {
      const int l = 32 + (int)__builtin_ctzll(mp);
      pm = Ls3Move{1, 1, a, rd_lane(t2, l), t3, rd_lane(t4, l), rd_lane(t5, l), rd_lane(t6, l), rd_lane(r3, l), 0};
      pm.end = (rd_lane(r5, l) == 0 ? n : rd_lane(r5, l)) - 1;
      p_found = true;
      if (ABORT && lane == 0) atomicMin(first, wave);  // this wave returns a move
    }
    if (ABORT && fl < wave) break;  // dropped either way
  }
  if (p_found) return pm;
  return Ls3Move{0, 0, a, 0, 0, 0, 0, 0, 0, 0};
}

// reverse the len tour positions from i on (cyclic), exactly these (no
// complement); block-wide, ends with a barrier
template <class IP>
__device__ __forceinline__ void ls_reverse_span(int n, IP tour, IP pos, int i, int len) {
  for (int s = threadIdx.x; s < len / 2; s += blockDim.x) {
    int pi = i + s;
    if (pi >= n) pi -= n;
    int pj = i + len - 1 - s;
    if (pj >= n) pj -= n;
    const int ti = tour[pi], tj = tour[pj];
    tour[pi] = tj;
    tour[pj] = ti;
    pos[tj] = pi;
    pos[ti] = pj;
  }
  __syncthreads();
}

// The move a wave found for its node: kind 0 none, 2 a 2-opt move, 3 a
// segment exchange.  In mode 2 a 2-opt move also carries the path to
// reverse (positions i .. j, the shorter side, and half its length).
struct Ls3Any {
  int kind, a, b, c, e, dir, t1, t2, t3, t4, t5, t6, r3, end, i, j, half;
};

// Swap tour positions i + s and j - s (cyclic) for s < half, with their
// FP32 coordinates; block-wide, ends with a barrier.
__device__ __forceinline__ void ls_reverse_xy(int n, uint16_t* tour, uint16_t* pos, float2* txy, int i, int j,
                                              int half) {
  for (int s = threadIdx.x; s < half; s += blockDim.x) {
    int pi = i + s;
    if (pi >= n) pi -= n;
    int pj = j - s;
    if (pj < 0) pj += n;
    const int ti = tour[pi], tj = tour[pj];
    const float2 xi = txy[pi], xj = txy[pj];
    tour[pi] = (uint16_t)tj;
    tour[pj] = (uint16_t)ti;
    txy[pi] = xj;
    txy[pj] = xi;
    pos[tj] = (uint16_t)pi;
    pos[ti] = (uint16_t)pj;
  }
  __syncthreads();
}

// One block of W waves per tour, organised like the 2-opt's: each round the
// waves evaluate the next queue entries against the same tour (wave 0 takes
// the node of the last applied move first, as the sequential search
// examines it again), the first improving result in queue order is
// applied, and the entries before it are consumed as the sequential search
// consumes them; the results behind it are dropped.  Thread 0 keeps the
// queue; the block reverses paths.  XY: mode 2 (FP32 coordinates in tour
// order beside the uint16 arrays, and the bounds e1 .. e3 of its filters).
// Returns rot: the final array is the sequential search's tour rotated,
// tour[x] = its [(x + rot) mod n] (see the segment exchange below).
template <bool XY, bool ABORT, class IP, class BP>
__device__ int three_opt_block(const InstDesc& D, IP tour, IP pos, IP queue, BP inq, double min_gain,
                               float2* txy = nullptr, double e1 = 0.0, double e2 = 0.0, double e3 = 0.0) {
  __shared__ int sh_head, sh_count;
  // ABORT (mode 2 only): the lowest wave of the round that has found an
  // improving move; a wave behind it stops its exchange search, whose result
  // the round drops.  It pays with many waves per block and costs registers.
  __shared__ int sh_first;
  __shared__ Ls3Any sh_mv[LS_WAVES];
  const int n = D.n, kls = D.kls, kg = D.kg, lane = lane_id(), wave = threadIdx.x / WAVE;
  const int nw = (int)(blockDim.x / WAVE);
  if (n < 5 || kls < 1) return 0;
  const GDist G(D);
  const HAC_AS1 int32_t* geo = as_global(D.geo);
  for (int s = threadIdx.x; s < n; s += blockDim.x) {
    const int v = tour[s];
    pos[v] = s;
    queue[s] = v;
    inq[v] = 1;
  }
  if (threadIdx.x == 0) {
    sh_head = 0;
    sh_count = n;
    if (ABORT) sh_first = LS_WAVES;
  }
  __syncthreads();
  const int64_t max_moves = 64 * (int64_t)n;
  int64_t moves = 0;
  int pend = -1;
  int rot = 0;  // the array holds the sequential search's tour rotated: tour[x] = its [(x + rot) mod n]
  while (moves < max_moves) {
    const int head = sh_head, count = sh_count;
    const int re = pend >= 0 ? 1 : 0;
    const int nq = min(nw - re, count);  // queue entries in this batch
    const int nb = nq + re;
    if (nb == 0) break;
    if (wave < nb) {
      int node = pend;
      if (wave >= re) {
        int slot = head + wave - re;
        if (slot >= n) slot -= n;
        node = queue[slot];
      }
      Ls3Any r{0, node, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      bool two = false;
      LsNodeXY nd;
      if constexpr (XY) {
        const LsMoveXY m = ls_eval_xy(G, geo, kg, kls, n, tour, pos, txy, node, min_gain, e1, e2, nd);
        if (m.imp) {
          if (ABORT && lane == 0) atomicMin(&sh_first, wave);
          two = true;
          r.kind = 2;
          r.b = m.b;
          r.c = m.c;
          r.e = m.e;
          r.i = m.i;
          r.j = m.j;
          r.half = m.half;
        }
      } else {
        const LsMove m = ls_eval(G, geo, kg, kls, n, tour, pos, node, min_gain);
        if (m.imp) {
          two = true;
          r.kind = 2;
          r.b = m.b;
          r.c = m.c;
          r.e = m.e;
          r.dir = m.dir;
        }
      }
      if (!two) {
        Ls3Move x;
        if constexpr (XY)
          x = ls3_eval_xy<ABORT>(G, geo, kg, kls, n, tour, pos, txy, node, nd, min_gain, e2, e3, &sh_first, wave);
        else
          x = ls3_eval(G, geo, kg, kls, n, tour, pos, node, min_gain);
        if (x.imp) {
          r.kind = 3;
          r.dir = x.dir;
          r.t1 = x.t1;
          r.t2 = x.t2;
          r.t3 = x.t3;
          r.t4 = x.t4;
          r.t5 = x.t5;
          r.t6 = x.t6;
          r.r3 = x.r3;
          r.end = x.end;
        }
      }
      if (lane == 0) sh_mv[wave] = r;
    }
    __syncthreads();
    // the first improving result in batch order (one entry per lane)
    const uint64_t fm = __builtin_amdgcn_ballot_w64(lane < nb && sh_mv[min(lane, LS_WAVES - 1)].kind != 0);
    const int f = fm ? (int)__builtin_ctzll(fm) : -1;
    if (ABORT && threadIdx.x == 0) sh_first = LS_WAVES;  // every wave is past its evaluation
    // queue entries consumed as a sequential scan would: all of them if no
    // move improves, else those up to and including the improving one
    const int used = f < 0 ? nq : max(0, f + 1 - re);
    Ls3Any mv{};
    int ri = 0, rj = 0;  // a 2-opt move's path, or an exchange's first position
    if (f >= 0) {
      mv = sh_mv[f];
      if (mv.kind == 2) {
        if constexpr (XY) {
          ri = mv.i;
          rj = mv.j;
        } else {
          ri = pos[mv.dir == 0 ? mv.b : mv.c];
          rj = pos[mv.dir == 0 ? mv.c : mv.b];
        }
      } else {
        const int p1 = pos[mv.a];
        ri = mv.dir == 0 ? p1 + 1 : p1 - mv.end;
        if (ri >= n) ri -= n;
        if (ri < 0) ri += n;
      }
    }
    if ((int)threadIdx.x < used) {
      int slot = head + threadIdx.x;
      if (slot >= n) slot -= n;
      inq[queue[slot]] = 0;
    }
    __syncthreads();
    if (f < 0) {
      if (threadIdx.x == 0) {
        int h = head + used;
        if (h >= n) h -= n;
        sh_head = h;
        sh_count = count - used;
      }
      pend = -1;
      __syncthreads();
      continue;
    }
    // thread 0 moves the head and queues the end nodes in order if absent
    // (an exchange's ends may repeat); the queue and the tour are separate
    // arrays, so this runs beside the reversals, whose barriers publish it
    if (threadIdx.x == 0) {
      int h = head + used;
      if (h >= n) h -= n;
      int cnt = count - used;
      auto push = [&](int x) {
        if (!inq[x]) {
          int slot = h + cnt;
          if (slot >= n) slot -= n;
          queue[slot] = x;
          inq[x] = 1;
          ++cnt;
        }
      };
      if (mv.kind == 2) {
        push(mv.a);
        push(mv.b);
        push(mv.c);
        push(mv.e);
      } else {
        push(mv.t1);
        push(mv.t2);
        push(mv.t3);
        push(mv.t4);
        push(mv.t5);
        push(mv.t6);
      }
      sh_head = h;
      sh_count = cnt;
    }
    if (mv.kind == 2) {
      if constexpr (XY)
        ls_reverse_xy(n, tour, pos, txy, ri, rj, mv.half);
      else
        ls_reverse(n, tour, pos, ri, rj);
    } else {
      // The segments t2..t4 (r3 - 1 nodes) and t3..t6 (end - r3 + 1) trade
      // places.  In array order from ri they are blocks P (pa nodes) and Q
      // (qb nodes); the rest of the tour, t1 among it, is block Z.  Swapping
      // any two of the three adjacent blocks gives the same cyclic tour in
      // the same direction, so the swap that moves the fewest nodes is made
      // (P with Q is the sequential search's); swapping Q with Z leaves the
      // array rotated by qb positions against it, Z with P by -pa, which rot
      // accumulates.  Later moves depend only on the cyclic tour, and the
      // rotation is undone when the tour is written back.
      const int qb = mv.dir == 0 ? mv.end - mv.r3 + 1 : mv.r3 - 1;  // the block that ends up first
      const int pa = mv.end - qb, zc = n - mv.end;
      // reverse the len positions from i (i < 2n, cyclic)
      auto span = [&](int i, int len) {
        if (i >= n) i -= n;
        if constexpr (XY) {
          int j = i + len - 1;
          if (j >= n) j -= n;
          ls_reverse_xy(n, tour, pos, txy, i, j, len / 2);
        } else {
          ls_reverse_span(n, tour, pos, i, len);
        }
      };
      // blocks [s, s + x) and [s + x, s + x + y) trade places
      auto swap_blocks = [&](int s0, int x, int y) {
        if (s0 >= n) s0 -= n;
        span(s0, x + y);
        span(s0, y);
        span(s0 + y, x);
      };
      if (mv.end <= n - pa && mv.end <= n - qb) {
        swap_blocks(ri, pa, qb);
      } else if (n - pa <= n - qb) {
        swap_blocks(ri + pa, qb, zc);
        rot += qb;
        if (rot >= n) rot -= n;
      } else {
        swap_blocks(ri + pa + qb, zc, pa);
        rot -= pa;
        if (rot < 0) rot += n;
      }
    }
    ++moves;
    pend = mv.a;
  }
  __syncthreads();
  return rot;
}

// working arrays: MODE 2 the 2-opt's mode-2 arrays (uint16 tour, positions
// and queue, byte flags, FP32 coordinates in tour order; 15 bytes per node),
// MODE 3 the same with waves that stop once their result will be dropped,
// MODE 1 int32 tour, positions and queue and byte flags in LDS (13 bytes per
// node), MODE 0 the tour in place and the rest in the tour's work area
template <int MODE>
__device__ __forceinline__ void three_opt_tour(const InstDesc& D, int32_t* tour_g, double min_gain,
                                               int32_t* work) {
  extern __shared__ int32_t ls_lds[];
  const int n = D.n;
  if constexpr (MODE >= 2) {
    uint16_t* tour = reinterpret_cast<uint16_t*>(ls_lds);
    uint16_t* pos = tour + n;
    uint16_t* queue = pos + n;
    uint8_t* inq = reinterpret_cast<uint8_t*>(ls_lds) + ((size_t)6 * n + 15) / 16 * 16;
    float2* txy = reinterpret_cast<float2*>(reinterpret_cast<uint8_t*>(inq) + ((size_t)n + 15) / 16 * 16);
    const double M = ls_stage_xy(D, tour_g, tour, txy);
    const int rot = three_opt_block<true, MODE == 3>(D, tour, pos, queue, inq, min_gain, txy, M * 0x1p-18, M * 0x1p-17,
                                          M * 0x1p-16);
    __syncthreads();
    for (int s = threadIdx.x; s < n; s += blockDim.x) tour_g[s] = tour[s - rot < 0 ? s - rot + n : s - rot];
  } else if constexpr (MODE == 1) {
    int32_t* tour = ls_lds;
    int32_t* pos = tour + n;
    int32_t* queue = pos + n;
    uint8_t* inq = reinterpret_cast<uint8_t*>(queue + n);
    for (int s = threadIdx.x; s < n; s += blockDim.x) tour[s] = tour_g[s];
    __syncthreads();
    const int rot = three_opt_block<false, false>(D, tour, pos, queue, inq, min_gain);
    for (int s = threadIdx.x; s < n; s += blockDim.x) tour_g[s] = tour[s - rot < 0 ? s - rot + n : s - rot];
  } else {
    HAC_AS1 int32_t* tour = as_global(tour_g);
    HAC_AS1 int32_t* pos = as_global(work);
    HAC_AS1 int32_t* queue = pos + n;
    HAC_AS1 uint8_t* inq = reinterpret_cast<HAC_AS1 uint8_t*>(queue + n);
    const int rot = three_opt_block<false, false>(D, tour, pos, queue, inq, min_gain);
    if (rot) {  // undo the rotation through the queue array, free by now
      for (int s = threadIdx.x; s < n; s += blockDim.x) queue[s] = tour[s];
      __threadfence_block();
      __syncthreads();
      for (int s = threadIdx.x; s < n; s += blockDim.x) tour[s] = queue[s - rot < 0 ? s - rot + n : s - rot];
    }
  }
  __threadfence_block();
  __syncthreads();
}

template <int MODE>
__global__ void __launch_bounds__(LS_WAVES * WAVE) three_opt_nn_kernel(const InstDesc* insts) {
  const InstDesc& D = insts[blockIdx.x];
  if (!D.local_search || !D.sym || D.ls_op != 3) return;
  three_opt_tour<MODE>(D, D.nn_tour, D.st->min_gain, D.ls_work);
  if (threadIdx.x < WAVE) {
    const double len = tour_length_wave(D, D.nn_tour);
    if (threadIdx.x == 0) {
      D.st->l_gb = len;
      D.st->l_ib = len;
    }
  }
}

// local_search = 1: block (i, 0) improves a copy of the iteration best;
// local_search = 2: block (i, y) improves ant tours y, y + gridDim.y, ...
// Modes 0-2 are held to 96 VGPRs (five waves per SIMD; mode 2 would take
// 106, four): with the 3-opt on every ant the tours outnumber the resident
// blocks, and at n = 1000 one wave more per SIMD makes the launch 5% faster
// (7.85 -> 7.45 ms for 4 096 tours) for a small spill.  Mode 3 (blocks of
// four or more waves) keeps four waves per SIMD and its registers.
template <int MODE>
__global__ void __launch_bounds__(LS_WAVES * WAVE) __attribute__((amdgpu_waves_per_eu(MODE == 3 ? 4 : 5)))
three_opt_kernel(const InstDesc* insts) {
  const InstDesc& D = insts[blockIdx.x];
  if (!D.local_search || !D.sym || D.ls_op != 3 || D.st->t > D.iterations || D.st->err) return;
  const int n = D.n;
  if (D.local_search == 2) {
    for (int a = blockIdx.y; a < D.ants; a += gridDim.y) {
      int32_t* tour = D.tours + (int64_t)a * n;
      three_opt_tour<MODE>(D, tour, D.st->min_gain, D.ls_work + (int64_t)a * 3 * n);
      if (threadIdx.x < WAVE) {
        const double len = tour_length_wave(D, tour);
        if (threadIdx.x == 0) D.lens[a] = len;
      }
      __syncthreads();
    }
    return;
  }
  if (blockIdx.y != 0) return;
  __shared__ int sh_ib;
  if (threadIdx.x < WAVE) {
    int ib;
    double lib;
    iteration_best_wave(D, ib, lib);
    if (threadIdx.x == 0) sh_ib = ib;
  }
  __syncthreads();
  const int ib = sh_ib;
  const int32_t* src = D.tours + (int64_t)ib * n;
  for (int s = threadIdx.x; s < n; s += blockDim.x) D.t_ib[s] = src[s];
  __threadfence_block();
  __syncthreads();
  three_opt_tour<MODE>(D, D.t_ib, D.st->min_gain, D.ls_work);
  if (threadIdx.x < WAVE) {
    const double len = tour_length_wave(D, D.t_ib);
    if (threadIdx.x == 0) {
      D.st->ib = ib;
      D.st->l_ib = len;
    }
  }
}

// ------------------------------------------------------------------------
// Directed 2-opt for the ATSP (Section III-D), one block per tour.
//
// A move reverses the tour path between its two inner nodes and prices it in
// its new direction: on the successor side of node a (b = succ a, c from a's
// outgoing list, e = succ c) the edges (a->b), (c->e) become (a->c), (b->e)
// and the path b..c is reversed; on the predecessor side (b = pred a, c from
// a's incoming list, e = pred c) (b->a), (e->c) become (c->a), (e->b) and
// the path c..b is reversed.  gain = (removed edges + F) - (added edges + B)
// with F and B the path's cost in its old and new direction, from prefix
// sums of the directed edge lengths in tour order (pf, pb), summed in blocks
// of 64 positions (dir_prefix) and brought up to date after each move from
// the first block whose edge changed, so that they equal a full
// recomputation.  The queue,
// the side order, the list stop rule, the threshold, the re-queueing of the
// end nodes and the re-examination of a are those of the symmetric 2-opt;
// the reversed part is always the path itself, and a search applies at most
// 64 n moves.  The 64 lanes of a wave evaluate a's moves at once: lanes
// 0..31 the successor side in list order, 32..63 the predecessor side; the
// first improving move in that order is the sequential one.
// ------------------------------------------------------------------------
struct DirWork {
  double* ef;   // [n] d(T[q], T[q+1]) (the closing edge at n - 1)
  double* eb;   // [n] d(T[q+1], T[q])
  double* pf;   // [n + 1] prefix sums of ef
  double* pb;   // [n + 1] prefix sums of eb
  double* tf;   // [n / 64 + 1] totals of ef over blocks of 64 positions
  double* tb;   // [n / 64 + 1] the same for eb
  double* sf;   // [n / 64 + 1] block offsets: sf[0] = 0, sf[b + 1] = sf[b] + tf[b]
  double* sb;   // [n / 64 + 1] the same for eb
  int32_t* tour;
  int32_t* pos;
  int32_t* queue;
  uint8_t* inq;
  uint16_t* lo;  // LDS copies of the outgoing and incoming lists ([n][kls] each), or null
  uint16_t* li;
};

__device__ __forceinline__ DirWork dir_work_at(char* base, int n) {
  DirWork w;
  w.ef = reinterpret_cast<double*>(base);
  w.eb = w.ef + n;
  w.pf = w.eb + n;
  w.pb = w.pf + (n + 1);
  const int nblk = n / 64 + 1;
  w.tf = w.pb + (n + 1);
  w.tb = w.tf + nblk;
  w.sf = w.tb + nblk;
  w.sb = w.sf + nblk;
  w.tour = reinterpret_cast<int32_t*>(w.sb + (nblk + 1));
  w.pos = w.tour + n;
  w.queue = w.pos + n;
  w.inq = reinterpret_cast<uint8_t*>(w.queue + n);
  return w;
}

__device__ __forceinline__ void wave_sync() {
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
}

// Prefix sums in blocks of 64 positions (the oracle's definition):
// pf[q] = sf[q / 64] + (the edges of q's block before q, added in order from
// 0.0), sf[0] = 0, sf[b + 1] = sf[b] + tf[b], tf[b] the block's 64 edges
// added in order from 0.0; pb alike.  After the edges lo .. hi changed, the
// wave reloads them, re-adds the totals of their blocks (a lane per block),
// then the block offsets from there (one lane), then every prefix from the
// first changed block on (a lane per block): a dependent chain of about
// 128 + n / 64 additions instead of n.  Within a block the loads run eight
// ahead of the additions.
__device__ __forceinline__ void dir_block_sums(const double* e, int q0, int q1, double& acc) {
  int q = q0;
  for (; q + 8 <= q1; q += 8) {
    double v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = e[q + t];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc += v[t];
  }
  for (; q < q1; ++q) acc += e[q];
}

__device__ void dir_prefix(const HAC_AS1 double* d, int n, const DirWork& w, int lo, int hi) {
  const int t = threadIdx.x, nt = blockDim.x;
  for (int q = lo + t; q <= hi; q += nt) {
    const int x = w.tour[q], y = w.tour[q + 1 == n ? 0 : q + 1];
    w.ef[q] = d[(int64_t)x * n + y];
    w.eb[q] = d[(int64_t)y * n + x];
  }
  __syncthreads();
  const int blo = lo / 64, bhi = hi / 64, blast = n / 64;
  for (int b = blo + t; b <= bhi; b += nt) {
    const int q0 = 64 * b, q1 = min(q0 + 64, n);
    double f = 0.0, r = 0.0;
    dir_block_sums(w.ef, q0, q1, f);
    dir_block_sums(w.eb, q0, q1, r);
    w.tf[b] = f;
    w.tb[b] = r;
  }
  __syncthreads();
  if (t == 0) {
    if (blo == 0) {
      w.sf[0] = 0.0;
      w.sb[0] = 0.0;
    }
    double f = w.sf[blo], r = w.sb[blo];
    for (int b = blo; b < blast; ++b) {
      f = f + w.tf[b];
      r = r + w.tb[b];
      w.sf[b + 1] = f;
      w.sb[b + 1] = r;
    }
  }
  __syncthreads();
  for (int b = blo + t; b <= blast; b += nt) {
    const int q0 = 64 * b, qe = min(q0 + 64, n + 1);
    const double s1 = w.sf[b], s2 = w.sb[b];
    double f = 0.0, r = 0.0;
    for (int q = q0; q < qe; ++q) {
      w.pf[q] = s1 + f;
      w.pb[q] = s2 + r;
      if (q < n) {
        f += w.ef[q];
        r += w.eb[q];
      }
    }
  }
  __syncthreads();
}

__device__ __forceinline__ double dir_path_cost(const double* pre, int n, int i, int j) {
  return i <= j ? pre[j] - pre[i] : (pre[n] - pre[i]) + pre[j];
}

struct DirMove {
  int imp, a, b, c, e, i, j;
};

// The search is block-wide, like the symmetric 2-opt: each round the waves
// evaluate the next queue entries against the same tour (wave 0 re-examines
// the node of the last applied move first), the first improving result in
// that order is applied, and the entries before it are consumed as the
// sequential scan would consume them; the results behind it are dropped.
// The last wave does the queue bookkeeping while the others reverse the
// path.  On an ant's tour most entries have no improving move, so a round
// consumes many of them.
__device__ void dir_two_opt(const InstDesc& D, int32_t* tour_g, double min_gain, const DirWork& w) {
  __shared__ int sh_head, sh_count;
  __shared__ DirMove sh_mv[LS_WAVES];
  const int n = D.n, kls = D.kls, lane = lane_id(), wave = threadIdx.x / WAVE;
  const int nw = (int)(blockDim.x / WAVE);
  if (n < 5 || kls < 1) return;
  const HAC_AS1 double* d = as_global(D.dist);
  const HAC_AS1 int32_t* in_l = as_global(D.nl_in);        // incoming lists: d(., a) order
  const HAC_AS1 int32_t* out_l = in_l + (int64_t)n * kls;   // outgoing lists: d(a, .) order
  if (w.lo) {
    for (int x = threadIdx.x; x < n * kls; x += blockDim.x) {
      w.lo[x] = (uint16_t)out_l[x];
      w.li[x] = (uint16_t)in_l[x];
    }
  }
  for (int s = threadIdx.x; s < n; s += blockDim.x) {
    const int v = tour_g[s];
    w.tour[s] = v;
    w.queue[s] = v;
  }
  __syncthreads();
  for (int s = threadIdx.x; s < n; s += blockDim.x) {
    w.pos[w.tour[s]] = s;
    w.inq[w.tour[s]] = 1;
  }
  if (threadIdx.x == 0) {
    sh_head = 0;
    sh_count = n;
  }
  __syncthreads();
  dir_prefix(d, n, w, 0, n - 1);
  const int64_t max_moves = 64 * (int64_t)n;
  int64_t moves = 0;
  int pend = -1;
  const bool pred_side = lane >= 32;
  const int q = lane & 31;
  const bool in_list = q < kls;
  const int step = pred_side ? -1 : 1;
  const int bw = nw - 1;  // the bookkeeping wave
  while (moves < max_moves) {
    const int head = sh_head, count = sh_count;
    const int re = pend >= 0 ? 1 : 0;
    const int nq = min(nw - re, count);  // queue entries in this batch
    const int nb = nq + re;
    if (nb == 0) break;
    if (wave < nb) {
      int a = pend;
      if (wave >= re) {
        int slot = head + wave - re;
        if (slot >= n) slot -= n;
        a = w.queue[slot];
      }
      // the tour edges a-b and c-e are entries of ef; only d(a,c) and
      // d(b,e) come from the matrix, both loaded once e is known
      const int pa = w.pos[a];
      const int pb = cyc_step(pa, step, n);
      const int b = w.tour[pb];
      const double dab = w.ef[pred_side ? pb : pa];  // d(a,b), or d(b,a) on the predecessor side
      const int at = a * kls + (in_list ? q : 0);
      const int c = w.lo ? (int)(pred_side ? w.li[at] : w.lo[at]) : (pred_side ? in_l[at] : out_l[at]);
      const int pc = w.pos[c];
      const int pe = cyc_step(pc, step, n);
      const int e = w.tour[pe];
      const double dce = w.ef[pred_side ? pe : pc];  // d(c,e), or d(e,c)
      const double dac = pred_side ? d[(int64_t)c * n + a] : d[(int64_t)a * n + c];
      const double dbe = pred_side ? d[(int64_t)e * n + b] : d[(int64_t)b * n + e];
      const bool g1pos = dab - dac > 0.0;
      // a side stops at its first list entry that cannot gain
      const uint64_t stop = __builtin_amdgcn_ballot_w64(in_list && !g1pos);
      const uint64_t stop_s = stop & 0xffffffffull, stop_p = stop >> 32;
      const int lim = pred_side ? (stop_p ? (int)__builtin_ctzll(stop_p) : 32)
                                : (stop_s ? (int)__builtin_ctzll(stop_s) : 32);
      const bool ok = in_list && q < lim;
      const bool degenerate = e == a || c == b || c == a;
      int i = 0, j = 0;
      bool imp = false;
      if (ok && !degenerate) {
        i = pred_side ? pc : pb;
        j = pred_side ? pb : pc;
        const double F = dir_path_cost(w.pf, n, i, j), B = dir_path_cost(w.pb, n, i, j);
        const double gain = ((dab + dce) + F) - ((dac + dbe) + B);
        imp = gain > min_gain;
      }
      const uint64_t mi = __builtin_amdgcn_ballot_w64(imp);
      DirMove m{0, a, 0, 0, 0, 0, 0};
      if (mi) {
        const int l = (int)__builtin_ctzll(mi);
        m.imp = 1;
        m.b = rd_lane(b, l);
        m.c = rd_lane(c, l);
        m.e = rd_lane(e, l);
        m.i = rd_lane(i, l);
        m.j = rd_lane(j, l);
      }
      if (lane == 0) sh_mv[wave] = m;
    }
    __syncthreads();
    // the first improving result in batch order (one entry per lane)
    const uint64_t fm = __builtin_amdgcn_ballot_w64(lane < nb && sh_mv[min(lane, LS_WAVES - 1)].imp);
    const int f = fm ? (int)__builtin_ctzll(fm) : -1;
    const DirMove mv = f >= 0 ? sh_mv[f] : DirMove{0, 0, 0, 0, 0, 0, 0};
    if (wave == bw) {
      // queue entries consumed as a sequential scan would: all of them if
      // no move improves, else those up to and including the improving one
      const int used = f < 0 ? nq : max(0, f + 1 - re);
      if (lane < used) {
        int slot = head + lane;
        if (slot >= n) slot -= n;
        w.inq[w.queue[slot]] = 0;
      }
      int h = head + used;
      if (h >= n) h -= n;
      int cnt = count - used;
      if (f >= 0) {
        // the end nodes a, b, c, e join the queue tail in that order if
        // absent, one lane each
        const bool mine = lane < 4;
        const int x = lane == 0 ? mv.a : (lane == 1 ? mv.b : (lane == 2 ? mv.c : mv.e));
        const bool absent = mine && !w.inq[x];
        const uint32_t am = (uint32_t)__builtin_amdgcn_ballot_w64(absent) & 0xfu;
        if (absent) {
          int slot = h + cnt + __builtin_popcount(am & ((1u << lane) - 1u));
          if (slot >= n) slot -= n;
          w.queue[slot] = x;
          w.inq[x] = 1;
        }
        cnt += __builtin_popcount(am);
      }
      if (lane == 0) {
        sh_head = h;
        sh_count = cnt;
      }
    }
    if (f < 0) {
      pend = -1;
      __syncthreads();
      continue;
    }
    // reverse the positions mv.i .. mv.j (cyclic), by the other waves
    const int len = (mv.j >= mv.i ? mv.j - mv.i : mv.j - mv.i + n) + 1;
    const int rthreads = bw > 0 ? bw * WAVE : WAVE;
    for (int s2 = (bw > 0 && wave == bw) ? len : (int)threadIdx.x; s2 < len / 2; s2 += rthreads) {
      int x = mv.i + s2;
      if (x >= n) x -= n;
      int y = mv.j - s2;
      if (y < 0) y += n;
      const int tx = w.tour[x], ty = w.tour[y];
      w.tour[x] = ty;
      w.tour[y] = tx;
      w.pos[ty] = x;
      w.pos[tx] = y;
    }
    __syncthreads();
    // the edges i - 1 .. j changed (all of them when the path wraps or
    // starts at position 0, where the closing edge changes too)
    if (mv.i >= 1 && mv.i <= mv.j)
      dir_prefix(d, n, w, mv.i - 1, mv.j);
    else
      dir_prefix(d, n, w, 0, n - 1);
    ++moves;
    pend = mv.a;
  }
  __syncthreads();
  for (int s = threadIdx.x; s < n; s += blockDim.x) tour_g[s] = w.tour[s];
  __syncthreads();
}

// the directed 2-opt's working arrays: in LDS when the launch gave room for
// them (lds_mode >= 1), else in the tour's part of the work area; with
// lds_mode 2 the neighbour lists are copied into LDS behind them as uint16
__device__ __forceinline__ DirWork dir_work_for(const InstDesc& D, int lds_mode, int tour_index) {
  extern __shared__ __align__(16) char dir_lds[];
  DirWork w = dir_work_at(lds_mode ? dir_lds
                                   : reinterpret_cast<char*>(D.ls_work) + (int64_t)tour_index * dir_work_stride(D.n),
                          D.n);
  w.lo = w.li = nullptr;
  if (lds_mode == 2) {
    w.lo = reinterpret_cast<uint16_t*>(dir_lds + ((dir_work_bytes(D.n) + 15) & ~(size_t)15));
    w.li = w.lo + (size_t)D.n * D.kls;
  }
  return w;
}

// incoming lists: for node i the kls nodes j with the smallest d(j, i),
// ties to the lower index (one wave per node; blockIdx.y is the instance)
__global__ void __launch_bounds__(256) in_lists_kernel(const InstDesc* insts) {
  const InstDesc& D = insts[blockIdx.y];
  if (!D.local_search || D.sym) return;
  const int n = D.n, kls = D.kls, lane = lane_id();
  const int i = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
  if (i >= n) return;
  const HAC_AS1 double* d = as_global(D.dist);
  WaveTopK t;
  topk_init(t, kls);
  for (int j0 = 0; j0 < n; j0 += WAVE) {
    const int j = j0 + lane;
    const bool valid = j < n && j != i;
    topk_offer(t, valid ? d[(int64_t)j * n + i] : 0.0, j, valid);
  }
  if (lane < kls) {
    D.nl_in[(int64_t)i * kls + lane] = t.id;
    // the first kls entries of the geometric list: the outgoing list
    D.nl_in[(int64_t)n * kls + (int64_t)i * kls + lane] = D.geo[(int64_t)i * D.kg + lane];
  }
}

__global__ void __launch_bounds__(LS_WAVES * WAVE) directed_two_opt_nn_kernel(const InstDesc* insts, int lds_mode) {
  const InstDesc& D = insts[blockIdx.x];
  if (!D.local_search || D.sym) return;
  dir_two_opt(D, D.nn_tour, D.st->min_gain, dir_work_for(D, lds_mode, 0));
  if (threadIdx.x < WAVE) {
    const double len = tour_length_wave(D, D.nn_tour);
    if (threadIdx.x == 0) {
      D.st->l_gb = len;
      D.st->l_ib = len;
    }
  }
}

// local_search = 1: block (i, 0) improves a copy of the iteration best;
// local_search = 2: block (i, y) improves ant tours y, y + gridDim.y, ...
__global__ void __launch_bounds__(LS_WAVES * WAVE) directed_local_search_kernel(const InstDesc* insts, int lds_mode) {
  const InstDesc& D = insts[blockIdx.x];
  if (!D.local_search || D.sym || D.st->t > D.iterations || D.st->err) return;
  const int n = D.n;
  if (D.local_search == 2) {
    for (int a = blockIdx.y; a < D.ants; a += gridDim.y) {
      int32_t* tour = D.tours + (int64_t)a * n;
      dir_two_opt(D, tour, D.st->min_gain, dir_work_for(D, lds_mode, a));
      if (threadIdx.x < WAVE) {
        const double len = tour_length_wave(D, tour);
        if (threadIdx.x == 0) D.lens[a] = len;
      }
      __syncthreads();
    }
    return;
  }
  if (blockIdx.y != 0) return;
  __shared__ int sh_ib;
  if (threadIdx.x < WAVE) {
    int ib;
    double lib;
    iteration_best_wave(D, ib, lib);
    if (threadIdx.x == 0) sh_ib = ib;
  }
  __syncthreads();
  const int ib = sh_ib;
  const int32_t* src = D.tours + (int64_t)ib * n;
  for (int s = threadIdx.x; s < n; s += blockDim.x) D.t_ib[s] = src[s];
  __threadfence_block();
  __syncthreads();
  dir_two_opt(D, D.t_ib, D.st->min_gain, dir_work_for(D, lds_mode, 0));
  if (threadIdx.x < WAVE) {
    const double len = tour_length_wave(D, D.t_ib);
    if (threadIdx.x == 0) {
      D.st->ib = ib;
      D.st->l_ib = len;
    }
  }
}

// ------------------------------------------------------------------------
// End of an iteration (Alg. 1): iteration/restart/global best, bounds,
// elite choice, fused evaporate + deposit + clamp + weights (eq. 7-8),
// branching-factor restart, u_gb schedule.  One block per instance.
// ------------------------------------------------------------------------
__device__ __forceinline__ int ugb_tier(int stall, int ugb_max) {
  if (stall < 25) return ugb_max;
  if (stall < 75) return 5;
  if (stall < 125) return 3;
  if (stall < 250) return 2;
  return 1;
}

__global__ void __launch_bounds__(1024) iter_end_kernel(const InstDesc* insts) {
  const InstDesc& D = insts[blockIdx.x];
  State* st = D.st;
  const int t = st->t;
  if (t > D.iterations || st->err) return;
  const int n = D.n, k = D.k, tid = threadIdx.x, nthr = blockDim.x;
  __shared__ double s_key[32];
  __shared__ int s_idx[32];
  __shared__ unsigned long long s_cnt[32];
  __shared__ int s_ib, s_rb_upd, s_gb_upd, s_use_rb, s_restart;
  __shared__ double s_lib, s_lel;
  __shared__ float s_tmax, s_tmin;

  // iteration best (first ant with the smallest length)
  const int32_t* t_ib;
  if (D.local_search == 1) {
    if (tid == 0) {
      s_ib = st->ib;
      s_lib = st->l_ib;
    }
    __syncthreads();
    t_ib = D.t_ib;
  } else {
    double bk = __builtin_huge_val();
    int bi = 0x7fffffff;
    for (int a = tid; a < D.ants; a += nthr) {
      double v = D.lens[a];
      if (key_less(v, a, bk, bi)) {
        bk = v;
        bi = a;
      }
    }
    wave_argmin(bk, bi);
    if (lane_id() == 0) {
      s_key[tid / WAVE] = bk;
      s_idx[tid / WAVE] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double k0 = s_key[0];
      int i0 = s_idx[0];
      for (int w = 1; w < nthr / WAVE; ++w)
        if (key_less(s_key[w], s_idx[w], k0, i0)) {
          k0 = s_key[w];
          i0 = s_idx[w];
        }
      s_ib = i0;
      s_lib = k0;
    }
    __syncthreads();
    t_ib = D.tours + (int64_t)s_ib * n;
  }

  // restart-best, global best, bounds, elite choice
  if (tid == 0) {
    const double lib = s_lib;
    int rb_upd = (!st->rb_valid || lib < st->l_rb);
    if (rb_upd) {
      st->l_rb = lib;
      st->rb_valid = 1;
      st->stall = 0;
    } else {
      st->stall += 1;
    }
    int gb_upd = lib < st->l_gb;
    if (gb_upd) {
      st->l_gb = lib;
      double tmax, tmin;
      bounds_from_length(D, lib, tmax, tmin);
      st->tmax = tmax;
      st->tmin = tmin;
      st->tmax_f = (float)tmax;
      st->tmin_f = (float)tmin;
    }
    int use_rb = (t % st->ugb) == 0;
    s_rb_upd = rb_upd;
    s_gb_upd = gb_upd;
    s_use_rb = use_rb;
    s_lel = use_rb ? st->l_rb : lib;
    s_tmax = st->tmax_f;
    s_tmin = st->tmin_f;
    st->ib = s_ib;
    st->l_ib = lib;
    if (D.tr_lib) D.tr_lib[t - 1] = lib;
    if (D.tr_lgb) D.tr_lgb[t - 1] = st->l_gb;
    if (D.tr_elite) D.tr_elite[t - 1] = use_rb;
  }
  __syncthreads();
  // the elite tour: the restart-best one (as just updated) or the iteration best
  const int32_t* elite = (s_use_rb && !s_rb_upd) ? D.t_rb : t_ib;
  for (int s = tid; s < n; s += nthr) {
    int v = elite[s];
    D.succ[v] = elite[s + 1 == n ? 0 : s + 1];
    D.pred[v] = elite[s == 0 ? n - 1 : s - 1];
  }
  if (s_rb_upd)
    for (int s = tid; s < n; s += nthr) D.t_rb[s] = t_ib[s];
  if (s_gb_upd)
    for (int s = tid; s < n; s += nthr) D.t_gb[s] = t_ib[s];
  __syncthreads();

  // eq. (7)-(8) on every candidate slot, then the choice weights
  const float keep = D.keep_f;
  const float delta = (float)(1.0 / s_lel);
  const float tmax_f = s_tmax, tmin_f = s_tmin;
  const int nk = n * k;
  const bool sym = D.sym != 0;
  // four slots per thread per pass, their inputs loaded before any store so
  // that the loads of the four are in flight together (each slot is
  // computed on its own, exactly as written above)
  constexpr int U = 4;
  for (int x0 = tid; x0 < nk; x0 += U * nthr) {
    int jv[U], sv[U], pv[U];
    float tv[U], hv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int x = x0 + u * nthr;
      if (x < nk) {
        const int i = x / k;
        jv[u] = D.cand[x];
        sv[u] = D.succ[i];
        pv[u] = D.pred[i];
        tv[u] = D.tau[x];
        hv[u] = D.heur[x];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int x = x0 + u * nthr;
      if (x < nk) {
        const bool on = jv[u] == sv[u] || (sym && jv[u] == pv[u]);
        float v = keep * tv[u];
        v = v + (on ? delta : 0.0f);
        v = fmaxf(tmin_f, v);
        v = fminf(tmax_f, v);
        const float w = v * hv[u];
        D.tau[x] = v;
        D.w[x] = w;
        D.cw[x].y = __float_as_uint(w);
      }
    }
  }

  // branching-factor restart
  if (D.bf_period > 0 && t % D.bf_period == 0) {
    __syncthreads();
    unsigned long long cnt = 0;
    for (int i = tid; i < n; i += nthr) {
      const float* row = D.tau + (int64_t)i * k;
      double lo = row[0], hi = lo;
      for (int u = 1; u < k; ++u) {
        double v = row[u];
        if (v < lo) lo = v;
        if (v > hi) hi = v;
      }
      double cut = lo + D.xi_bf * (hi - lo);
      for (int u = 0; u < k; ++u)
        if ((double)row[u] >= cut) cnt++;
    }
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
    if (lane_id() == 0) s_cnt[tid / WAVE] = cnt;
    __syncthreads();
    if (tid == 0) {
      unsigned long long total = 0;
      for (int w = 0; w < nthr / WAVE; ++w) total += s_cnt[w];
      double bf = (double)total / ((double)n * (double)D.dstar);
      int restart = bf < D.lambda_bf && st->stall > D.restart_stall;
      if (restart) {
        st->rb_valid = 0;
        st->stall = 0;
        st->restarts += 1;
      }
      s_restart = restart;
    }
    __syncthreads();
    if (s_restart) {
      for (int x = tid; x < nk; x += nthr) {
        const float w = tmax_f * D.heur[x];
        D.tau[x] = tmax_f;
        D.w[x] = w;
        D.cw[x].y = __float_as_uint(w);
      }
    }
  }
  if (tid == 0) {
    st->ugb = ugb_tier(st->stall, D.ugb_max);
    st->t = t + 1;
  }
}

// ------------------------------------------------------------------------
// Output: the global best rotated to start at node 0 and, for symmetric
// instances, read in the direction whose second node is the smaller.
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(64) finish_kernel(const InstDesc* insts, int32_t* const* outs,
                                                    double* out_lens) {
  const InstDesc& D = insts[blockIdx.x];
  const int n = D.n, lane = lane_id();
  if (D.st->err) {
    // a broken kernel contract: no tour is written, and the length is NaN,
    // which the host turns into HAC_EDEVICE
    if (lane == 0) out_lens[blockIdx.x] = __builtin_nan("");
    return;
  }
  const int32_t* tg = D.t_gb;
  int r0 = 0x7fffffff;
  for (int s = lane; s < n; s += WAVE)
    if (tg[s] == 0) r0 = s;
  for (int off = 32; off >= 1; off >>= 1) r0 = min(r0, __shfl_xor(r0, off));
  int32_t* out = outs[blockIdx.x];
  bool rev = false;
  if (D.sym && n >= 3) {
    int t1 = tg[(r0 + 1) % n], tl = tg[(r0 - 1 + n) % n];
    rev = t1 > tl;
  }
  for (int s = lane; s < n; s += WAVE) out[s] = rev ? tg[(r0 - s + n) % n] : tg[(r0 + s) % n];
  if (lane == 0) out_lens[blockIdx.x] = D.st->l_gb;
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
int32_t max_lds_bytes() { return 160 * 1024; }

bool construct_bytes_fit(int32_t n, int32_t k, int32_t ants_per_block, int32_t rows_per_wave,
                         int32_t staged) {
  // byte marks are used only together with the unvisited lists
  return n <= 65535 &&
         construct_lds_layout(n, k, ants_per_block, rows_per_wave, staged, true, true).total <=
             (size_t)max_lds_bytes();
}

size_t construct_lds_bytes(int32_t n, int32_t k, int32_t ants_per_block, int32_t rows_per_wave,
                           int32_t staged, int32_t bytes) {
  if (bytes) return construct_lds_layout(n, k, ants_per_block, rows_per_wave, staged, true, true).total;
  // bit marks: the unvisited lists are included whenever they fit
  const ConstructLds with = construct_lds_layout(n, k, ants_per_block, rows_per_wave, staged, true, false);
  if (n <= 65535 && with.total <= (size_t)max_lds_bytes()) return with.total;
  return construct_lds_layout(n, k, ants_per_block, rows_per_wave, staged, false, false).total;
}

hipError_t launch_candidates(const InstDesc* d_insts, int32_t count, int32_t max_n, hipStream_t s) {
  const int waves = 4;
  hipLaunchKernelGGL(candidates_kernel, dim3((max_n + waves - 1) / waves, count), dim3(waves * WAVE), 0, s,
                     d_insts);
  return hipGetLastError();
}

hipError_t launch_nn_tour(const InstDesc* d_insts, int32_t count, int32_t max_n, hipStream_t s) {
  size_t lds = (size_t)(((max_n + 63) >> 6) << 1) * 4;
  hipLaunchKernelGGL(nn_tour_kernel, dim3(count), dim3(WAVE), lds, s, d_insts);
  return hipGetLastError();
}

// largest static LDS of the 2-opt and 3-opt kernels (their __shared__
// variables), read from the compiled kernels once
static size_t ls_static_lds() {
  static size_t v = [] {
    size_t m = 0;
    const void* ks[] = {(const void*)two_opt_nn_kernel<2>, (const void*)two_opt_nn_kernel<1>,
                        (const void*)local_search_kernel<2>, (const void*)local_search_kernel<1>,
                        (const void*)three_opt_nn_kernel<3>, (const void*)three_opt_kernel<3>,
                        (const void*)three_opt_nn_kernel<2>, (const void*)three_opt_kernel<2>,
                        (const void*)three_opt_nn_kernel<1>, (const void*)three_opt_kernel<1>};
    for (const void* k : ks) {
      hipFuncAttributes a{};
      // on failure keep a generous reserve rather than overcommit LDS
      m = std::max(m, hipFuncGetAttributes(&a, k) == hipSuccess ? (size_t)a.sharedSizeBytes : (size_t)8192);
    }
    return m;
  }();
  return v;
}

// the 2-opt mode of a launch: 2 when every instance of the batch has
// coordinates and fits, else 1 when the int32 arrays fit, else 0
static int ls_mode(int32_t max_n, int32_t all_coords) {
  const size_t cap = (size_t)max_lds_bytes() - ls_static_lds();
  if (const char* f = std::getenv("HAC_LS_MODE")) {
    // pins a mode when it fits (used to show the modes give the same tours)
    const int m = std::atoi(f);
    if (m == 0 || (m == 1 && ls_lds_need(max_n, 1) <= cap) ||
        (m == 2 && all_coords && max_n < 65536 && ls_lds_need(max_n, 2) <= cap))
      return m;
  }
  if (all_coords && max_n < 65536 && ls_lds_need(max_n, 2) <= cap) return 2;
  if (ls_lds_need(max_n, 1) <= cap) return 1;
  return 0;
}

// Where the directed 2-opt of the largest ATSP instance keeps its arrays:
// mode 2 the work arrays and uint16 copies of both neighbour lists in LDS,
// 1 the work arrays in LDS, 0 the work area in global memory; and the LDS
// bytes that takes.  HAC_LS_MODE (0 or 1) pins mode 0 or 1.
static int dir_lds_mode(int32_t max_n_dir, int32_t max_kls_dir, size_t* bytes) {
  const size_t cap = (size_t)max_lds_bytes() - 1024;
  const size_t work = dir_work_bytes(max_n_dir);
  const size_t lists = ((work + 15) & ~(size_t)15) + (size_t)4 * max_n_dir * max_kls_dir;
  int mode = lists <= cap && max_n_dir <= 65535 ? 2 : (work <= cap ? 1 : 0);
  if (const char* f = std::getenv("HAC_LS_MODE")) {
    if (f[0] == '0') mode = 0;  // pins the work area to global memory (as for the symmetric 2-opt)
    if (f[0] == '1' && mode == 2) mode = 1;
  }
  *bytes = mode == 2 ? lists : (mode == 1 ? work : 0);
  return mode;
}

// Waves per directed 2-opt block, chosen as for the symmetric search: the
// full LS_WAVES while the tours number at most 256, else as few as 4 so that
// as many tours run at once as LDS allows on a CU.  HAC_LS_WAVES pins it.
// Results do not depend on it.
static int dir_block_waves(size_t lds, int64_t tours) {
  if (const char* env = std::getenv("HAC_LS_WAVES")) {
    const int w = std::atoi(env);
    if (w >= 1 && w <= LS_WAVES) return w;
  }
  if (tours <= 256) return LS_WAVES;
  const int by_lds = lds ? (int)std::max<size_t>(1, (size_t)max_lds_bytes() / lds) : 8;
  return std::max(4, std::min(LS_WAVES, 32 / std::min(by_lds, 8)));
}

static hipError_t launch_directed(const InstDesc* d_insts, int32_t count, int32_t max_n_dir, int32_t max_kls_dir,
                                  int32_t tpi, bool nn, hipStream_t s) {
  size_t lds = 0;
  const int mode = dir_lds_mode(max_n_dir, max_kls_dir, &lds);
  const int64_t tours = nn ? count : (int64_t)count * std::max(tpi, 1);
  const dim3 block(dir_block_waves(lds, tours) * WAVE);
  if (nn)
    hipLaunchKernelGGL(directed_two_opt_nn_kernel, dim3(count), block, lds, s, d_insts, mode);
  else
    hipLaunchKernelGGL(directed_local_search_kernel, dim3(count, std::max(tpi, 1)), block, lds, s, d_insts, mode);
  return hipGetLastError();
}

// Waves per 3-opt block: the fewest rounds of resident blocks first (every
// tour's block resident at once where some W allows it), then the most waves
// per tour (up to LS_WAVES, a power of two), with residency from the
// kernel's occupancy at its LDS size (registers and LDS per CU).  Where
// tours wait for a slot either way, more waves per tour pay; where one wave
// per tour keeps every tour resident and two would not, one wins (every
// ant's tour of 128 instances, 200 iterations, per launch: n = 500 1 wave
// 3.5 ms, 2 waves 3.7 ms, 4 waves 4.2 ms; n = 1000 10.3, 7.9, 9.2 ms).
// HAC_LS_WAVES pins the count.  kernel_wide: the kernel that blocks of four
// or more waves run (their residency is that kernel's).
static int three_opt_waves(const void* kernel, const void* kernel_wide, size_t lds, int64_t tours) {
  if (const char* env = std::getenv("HAC_LS_WAVES")) {
    const int w = std::atoi(env);
    if (w >= 1 && w <= LS_WAVES) return w;
  }
  // blocks per CU at W = 1, 2, .. 16, per (kernel, LDS size, device); a
  // fixed table, so that no launch allocates (a full table recomputes)
  struct Entry {
    const void* k;
    size_t lds;
    int dev;
    std::array<int, 5> per_cu;
  };
  thread_local std::array<Entry, 16> cache;
  thread_local int cached = 0;
  thread_local int cus = 0, cus_dev = -1;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (cus_dev != dev) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    cus_dev = dev;
  }
  std::array<int, 5> v{};
  bool found = false;
  for (int x = 0; x < cached && !found; ++x)
    if (cache[x].k == kernel && cache[x].lds == lds && cache[x].dev == dev) {
      v = cache[x].per_cu;
      found = true;
    }
  if (!found) {
    for (int x = 0, w = 1; w <= LS_WAVES; ++x, w *= 2) {
      int b = 0;
      v[x] = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, w >= 4 ? kernel_wide : kernel, w * WAVE, lds) ==
                     hipSuccess
                 ? b
                 : 0;
    }
    if (cached < (int)cache.size()) cache[cached++] = Entry{kernel, lds, dev, v};
  }
  const std::array<int, 5>* per_cu = &v;
  int best = 0;
  int64_t best_rounds = INT64_MAX;
  for (int x = 0, w = 1; w <= LS_WAVES; ++x, w *= 2) {
    const int64_t slots = (int64_t)(*per_cu)[x] * cus;
    if (slots < 1) continue;
    const int64_t rounds = (tours + slots - 1) / slots;
    if (rounds <= best_rounds) {
      best_rounds = rounds;
      best = w;
    }
  }
  if (best) return best;
  // no occupancy figure: the most waves with which 8 192 wave slots hold every tour
  int w = LS_WAVES;
  while (w > 1 && tours * w > 8192) w /= 2;
  return w;
}

// the 3-opt: one block per tour, the working arrays in LDS when they fit
// (mode 2 when every 3-opt instance has coordinates, as for the 2-opt; in
// blocks of four or more waves mode 2 runs as mode 3, whose waves stop once
// their result will be dropped)
static hipError_t launch_three_opt(const InstDesc* d_insts, int32_t count, int32_t max_n3, int32_t all_coords3,
                                   int32_t tpi, bool nn, hipStream_t s) {
  const int mode = ls_mode(max_n3, all_coords3);
  const size_t lds = ls_lds_need(max_n3, mode);
  const int t = nn ? 1 : std::max(tpi, 1);
  const void* nn_k[4] = {(const void*)three_opt_nn_kernel<0>, (const void*)three_opt_nn_kernel<1>,
                         (const void*)three_opt_nn_kernel<2>, (const void*)three_opt_nn_kernel<3>};
  const void* ls_k[4] = {(const void*)three_opt_kernel<0>, (const void*)three_opt_kernel<1>,
                         (const void*)three_opt_kernel<2>, (const void*)three_opt_kernel<3>};
  const void* const* ks = nn ? nn_k : ls_k;
  const int waves = three_opt_waves(ks[mode], ks[mode == 2 ? 3 : mode], lds, (int64_t)count * t);
  const int km = mode == 2 && waves >= 4 ? 3 : mode;
  const dim3 grid(count, t), block(waves * WAVE);
  if (nn) {
    if (km == 3)
      hipLaunchKernelGGL(three_opt_nn_kernel<3>, grid, block, lds, s, d_insts);
    else if (km == 2)
      hipLaunchKernelGGL(three_opt_nn_kernel<2>, grid, block, lds, s, d_insts);
    else if (km == 1)
      hipLaunchKernelGGL(three_opt_nn_kernel<1>, grid, block, lds, s, d_insts);
    else
      hipLaunchKernelGGL(three_opt_nn_kernel<0>, grid, block, 0, s, d_insts);
  } else {
    if (km == 3)
      hipLaunchKernelGGL(three_opt_kernel<3>, grid, block, lds, s, d_insts);
    else if (km == 2)
      hipLaunchKernelGGL(three_opt_kernel<2>, grid, block, lds, s, d_insts);
    else if (km == 1)
      hipLaunchKernelGGL(three_opt_kernel<1>, grid, block, lds, s, d_insts);
    else
      hipLaunchKernelGGL(three_opt_kernel<0>, grid, block, 0, s, d_insts);
  }
  return hipGetLastError();
}

hipError_t launch_two_opt_nn(const InstDesc* d_insts, int32_t count, int32_t max_n, int32_t all_coords,
                             int32_t max_n_dir, int32_t max_kls_dir, int32_t max_n3, int32_t all_coords3,
                             hipStream_t s) {
  if (max_n3 > 0) {
    const hipError_t e = launch_three_opt(d_insts, count, max_n3, all_coords3, 1, true, s);
    if (e != hipSuccess) return e;
  }
  if (max_n_dir > 0) {
    const int waves = 4;
    hipLaunchKernelGGL(in_lists_kernel, dim3((max_n_dir + waves - 1) / waves, count), dim3(waves * WAVE), 0, s,
                       d_insts);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_directed(d_insts, count, max_n_dir, max_kls_dir, 1, true, s);
    if (e != hipSuccess) return e;
  }
  if (max_n <= 0) return hipSuccess;  // no symmetric instance searches
  const int mode = ls_mode(max_n, all_coords);
  const dim3 grid(count), block(LS_WAVES * WAVE);
  if (mode == 2)
    hipLaunchKernelGGL(two_opt_nn_kernel<2>, grid, block, ls_lds_need(max_n, 2), s, d_insts);
  else if (mode == 1)
    hipLaunchKernelGGL(two_opt_nn_kernel<1>, grid, block, ls_lds_need(max_n, 1), s, d_insts);
  else
    hipLaunchKernelGGL(two_opt_nn_kernel<0>, grid, block, 0, s, d_insts);
  return hipGetLastError();
}

// One block per instance with a grid: bounding box, cell widths, counting
// sort of the nodes by cell (order inside a cell is irrelevant to the
// search), and the coordinates copied in cell order.
__global__ void __launch_bounds__(1024) grid_kernel(const InstDesc* insts) {
  const InstDesc& D = insts[blockIdx.x];
  if (D.gside <= 0) return;
  __shared__ double sh[4][32];
  __shared__ GridPar sp;
  __shared__ int s_tot[1024];
  const int n = D.n, G = D.gside, cells = G * G, tid = threadIdx.x, nt = blockDim.x;
  const HAC_AS1 double* xy = as_global(D.xy);
  double lx = __builtin_huge_val(), ly = lx, hx = -lx, hy = -lx;
  for (int j = tid; j < n; j += nt) {
    const double x = xy[2 * j], y = xy[2 * j + 1];
    lx = fmin(lx, x);
    ly = fmin(ly, y);
    hx = fmax(hx, x);
    hy = fmax(hy, y);
  }
  for (int off = 32; off >= 1; off >>= 1) {
    lx = fmin(lx, __shfl_xor(lx, off));
    ly = fmin(ly, __shfl_xor(ly, off));
    hx = fmax(hx, __shfl_xor(hx, off));
    hy = fmax(hy, __shfl_xor(hy, off));
  }
  if ((tid & (WAVE - 1)) == 0) {
    sh[0][tid / WAVE] = lx;
    sh[1][tid / WAVE] = ly;
    sh[2][tid / WAVE] = hx;
    sh[3][tid / WAVE] = hy;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < nt / WAVE; ++w) {
      lx = fmin(lx, sh[0][w]);
      ly = fmin(ly, sh[1][w]);
      hx = fmax(hx, sh[2][w]);
      hy = fmax(hy, sh[3][w]);
    }
    lx = fmin(lx, sh[0][0]);
    ly = fmin(ly, sh[1][0]);
    hx = fmax(hx, sh[2][0]);
    hy = fmax(hy, sh[3][0]);
    GridPar P;
    P.gx = P.gy = G;
    P.x0 = lx;
    P.y0 = ly;
    P.ix = hx > lx ? (double)G / (hx - lx) : 0.0;
    P.iy = hy > ly ? (double)G / (hy - ly) : 0.0;
    const double im = fmax(P.ix, P.iy);
    P.wmin = im > 0.0 ? (1.0 / im) * (1.0 - 1e-9) : 0.0;
    sp = P;
    *D.g_par = P;
  }
  for (int c = tid; c < cells; c += nt) D.g_cur[c] = 0;
  __syncthreads();
  GridView g;
  g.par = sp;
  for (int j = tid; j < n; j += nt) {
    const int c = g.celly(xy[2 * j + 1]) * G + g.cellx(xy[2 * j]);
    atomicAdd(&D.g_cur[c], 1);
  }
  __syncthreads();
  // exclusive prefix of the counts: each thread a contiguous chunk of cells
  const int chunk = (cells + nt - 1) / nt;
  const int c0 = min(cells, tid * chunk), c1 = min(cells, c0 + chunk);
  int local = 0;
  for (int c = c0; c < c1; ++c) local += D.g_cur[c];
  s_tot[tid] = local;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    const int v = tid >= off ? s_tot[tid - off] : 0;
    __syncthreads();
    s_tot[tid] += v;
    __syncthreads();
  }
  int run = s_tot[tid] - local;
  for (int c = c0; c < c1; ++c) {
    const int k = D.g_cur[c];
    D.g_start[c] = run;
    D.g_cur[c] = run;
    run += k;
  }
  if (tid == 0) D.g_start[cells] = n;
  __syncthreads();
  for (int j = tid; j < n; j += nt) {
    const double x = xy[2 * j], y = xy[2 * j + 1];
    const int c = g.celly(y) * G + g.cellx(x);
    const int p = atomicAdd(&D.g_cur[c], 1);
    D.g_ids[p] = j;
    D.g_xy[2 * p] = x;
    D.g_xy[2 * p + 1] = y;
  }
}

// Gathers many device-to-device copies into one launch: blockIdx.x is the
// item, blockIdx.y a 64 KiB chunk of it.
__global__ void __launch_bounds__(256) copy_items_kernel(const CopyItem* items) {
  const CopyItem it = items[blockIdx.x];
  const uint64_t words = it.bytes / 4;
  const uint64_t beg = (uint64_t)blockIdx.y * 16384u;
  if (beg >= words) return;
  const uint64_t end = beg + 16384u < words ? beg + 16384u : words;
  const HAC_AS1 uint32_t* src = as_global(static_cast<const uint32_t*>(it.src));
  HAC_AS1 uint32_t* dst = as_global(static_cast<uint32_t*>(it.dst));
  for (uint64_t w = beg + threadIdx.x; w < end; w += blockDim.x) dst[w] = src[w];
}

hipError_t launch_copy_items(const CopyItem* d_items, int32_t count, uint64_t max_bytes, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const uint64_t chunks = (max_bytes / 4 + 16383u) / 16384u;
  if (chunks == 0) return hipSuccess;
  if (chunks > 65535u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_items_kernel, dim3(count, (unsigned)chunks), dim3(256), 0, s, d_items);
  return hipGetLastError();
}

hipError_t launch_grid(const InstDesc* d_insts, int32_t count, hipStream_t s) {
  hipLaunchKernelGGL(grid_kernel, dim3(count), dim3(1024), 0, s, d_insts);
  return hipGetLastError();
}

hipError_t launch_init(const InstDesc* d_insts, int32_t count, hipStream_t s) {
  hipLaunchKernelGGL(init_kernel, dim3(count), dim3(256), 0, s, d_insts);
  return hipGetLastError();
}

int32_t construct_group_lanes(int32_t max_k) { (void)max_k; return 16; }

hipError_t launch_construct(const InstDesc* d_insts, const BlockMap* d_map, int32_t blocks,
                            int32_t ants_per_block, int32_t rows_per_wave, int32_t staged,
                            int32_t bytes, int32_t max_k, size_t lds_bytes, int32_t geo_mode,
                            int32_t grid, hipStream_t s, int32_t step_cap) {
  if (geo_mode < 0 || geo_mode > 2 || step_cap < 1) return hipErrorInvalidValue;
  if (rows_per_wave < 1 || rows_per_wave > 4) return hipErrorInvalidValue;
  const int waves = (ants_per_block + rows_per_wave - 1) / rows_per_wave;
  if (waves < 1 || waves > kMaxConstructWaves) return hipErrorInvalidValue;
  const dim3 grid_dim(blocks), block(waves * WAVE);
  const int S = max_k <= 16 ? 1 : (max_k <= 32 ? 2 : 4);
#define HAC_LAUNCH_GG(ST, SL, BY, GM, GR)                                                                  \
  hipLaunchKernelGGL((construct_kernel<ST, SL, BY, GM, GR>), grid_dim, block, lds_bytes, s, d_insts, d_map, \
                     ants_per_block, rows_per_wave, (int)lds_bytes, (int)step_cap)
#define HAC_LAUNCH_G(ST, SL, BY, GM)               \
  {                                                \
    if (grid) HAC_LAUNCH_GG(ST, SL, BY, GM, true); \
    else HAC_LAUNCH_GG(ST, SL, BY, GM, false);     \
  }
#define HAC_LAUNCH(ST, SL, BY)                                   \
  {                                                              \
    if (geo_mode == 0) HAC_LAUNCH_G(ST, SL, BY, 0)               \
    else if (geo_mode == 1) HAC_LAUNCH_G(ST, SL, BY, 1)          \
    else HAC_LAUNCH_G(ST, SL, BY, 2)                             \
  }
#define HAC_LAUNCH_S(ST, BY)             \
  {                                      \
    if (S == 1) HAC_LAUNCH(ST, 1, BY)    \
    else if (S == 2) HAC_LAUNCH(ST, 2, BY) \
    else HAC_LAUNCH(ST, 4, BY)           \
  }
  if (staged < 0 || staged > 3) return hipErrorInvalidValue;
  if (staged == 3) {
    if (bytes) HAC_LAUNCH_S(3, true) else HAC_LAUNCH_S(3, false)
  } else if (staged == 2) {
    if (bytes) HAC_LAUNCH_S(2, true) else HAC_LAUNCH_S(2, false)
  } else if (staged == 1) {
    if (bytes) HAC_LAUNCH_S(1, true) else HAC_LAUNCH_S(1, false)
  } else {
    if (bytes) HAC_LAUNCH_S(0, true) else HAC_LAUNCH_S(0, false)
  }
#undef HAC_LAUNCH_S
#undef HAC_LAUNCH
#undef HAC_LAUNCH_G
#undef HAC_LAUNCH_GG
  return hipGetLastError();
}

// Waves per 2-opt block.  Results do not depend on it (the speculative
// batch keeps the sequential outcome).  One tour per instance gets the full
// LS_WAVES; when every ant's tour is searched, blocks shrink to as few as 4
// waves so that as many tours run at once as LDS allows on a CU (32 waves
// per CU).  HAC_LS_WAVES pins the count.
static int ls_block_waves(int32_t max_n, int mode, int64_t tours) {
  if (const char* env = std::getenv("HAC_LS_WAVES")) {
    const int w = std::atoi(env);
    if (w >= 1 && w <= LS_WAVES) return w;
  }
  if (tours <= 256) return LS_WAVES;
  const size_t need = ls_lds_need(max_n, mode);
  const int by_lds = need ? (int)std::max<size_t>(1, (size_t)max_lds_bytes() / need) : 8;
  return std::max(4, std::min(LS_WAVES, 32 / std::min(by_lds, 8)));
}

hipError_t launch_local_search(const InstDesc* d_insts, int32_t count, int32_t max_n,
                               int32_t all_coords, int32_t tours_per_inst, int32_t max_n_dir,
                               int32_t max_kls_dir, int32_t max_n3, int32_t all_coords3, hipStream_t s) {
  if (max_n3 > 0) {
    const hipError_t e = launch_three_opt(d_insts, count, max_n3, all_coords3, tours_per_inst, false, s);
    if (e != hipSuccess) return e;
  }
  if (max_n_dir > 0) {
    const hipError_t e = launch_directed(d_insts, count, max_n_dir, max_kls_dir, tours_per_inst, false, s);
    if (e != hipSuccess) return e;
  }
  if (max_n <= 0) return hipSuccess;  // no symmetric instance searches
  const int mode = ls_mode(max_n, all_coords);
  const int tpi = std::max(tours_per_inst, 1);
  const int waves = tpi > 1 ? ls_block_waves(max_n, mode, (int64_t)count * tpi) : LS_WAVES;
  const dim3 grid(count, tpi), block(waves * WAVE);
  if (mode == 2)
    hipLaunchKernelGGL(local_search_kernel<2>, grid, block, ls_lds_need(max_n, 2), s, d_insts);
  else if (mode == 1)
    hipLaunchKernelGGL(local_search_kernel<1>, grid, block, ls_lds_need(max_n, 1), s, d_insts);
  else
    hipLaunchKernelGGL(local_search_kernel<0>, grid, block, 0, s, d_insts);
  return hipGetLastError();
}

hipError_t launch_iter_end(const InstDesc* d_insts, int32_t count, hipStream_t s) {
  hipLaunchKernelGGL(iter_end_kernel, dim3(count), dim3(1024), 0, s, d_insts);
  return hipGetLastError();
}

hipError_t launch_finish(const InstDesc* d_insts, int32_t count, int32_t* const* d_out_tours,
                         double* d_out_lens, hipStream_t s) {
  hipLaunchKernelGGL(finish_kernel, dim3(count), dim3(WAVE), 0, s, d_insts, d_out_tours,
                     d_out_lens);
  return hipGetLastError();
}

// ------------------------------------------------------------------------
// the allocation-free entry point's scratch array, per device
// ------------------------------------------------------------------------
static constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_init_mu;
static void* g_noalloc_ptr[kMaxDevices];
static std::mutex g_noalloc_call_mu[kMaxDevices];

hipError_t noalloc_scratch_init(int32_t device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_noalloc_init_mu);
  if (g_noalloc_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_noalloc_ptr[device] = ptr;
  return hipSuccess;
}

void* noalloc_scratch(int32_t device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_noalloc_init_mu);
  return g_noalloc_ptr[device];
}

std::mutex* noalloc_call_lock(int32_t device) {
  return (device >= 0 && device < kMaxDevices) ? &g_noalloc_call_mu[device] : nullptr;
}

}  // namespace hac
