// Internal declarations shared by the host runtime (hac_api.cpp,
// hac_fold.cpp, hac_server.cpp) and the HIP kernels (hac_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

namespace hac {

// Device-resident search state of one instance (Alg. 1 bookkeeping).
struct State {
  int32_t t;         // next iteration to run, 1-based
  int32_t stall;     // iterations without restart-best improvement
  int32_t ugb;       // current u_gb
  int32_t rb_valid;  // restart-best tour exists
  int32_t restarts;
  int32_t ib;        // ant index of the last iteration best
  double l_gb, l_rb, l_ib;
  double tmax, tmin;    // FP64 bounds (eq. 5-6)
  float tmax_f, tmin_f; // their FP32 casts, used by the update
  double min_gain;              // 2-opt gain threshold, 1e-9 L_nn / n
  unsigned long long fallbacks;  // nearest-unvisited steps so far
  // nonzero once a kernel found its own contract broken (the construction
  // step picked other than exactly one slot of an open row); the instance
  // then stops, and the host reports HAC_EDEVICE
  uint32_t err;
};

// Uniform grid over the coordinates of a coordinate instance with
// n >= kGridMinN, for exact nearest-unvisited searches by rings of cells.
// A node's cell is min(side - 1, floor((x - x0) * ix)) per axis; wmin is a
// lower bound on the cell widths 1/ix, 1/iy (shrunk by 1e-9 relative).
struct GridPar {
  int32_t gx, gy;
  double x0, y0, ix, iy, wmin;
};
static constexpr int32_t kGridMinN = 2048;
// cells per side: about two nodes per cell
__host__ __device__ inline int32_t grid_side(int32_t n) {
  int32_t g = 1;
  while ((int64_t)(g + 1) * (g + 1) * 2 <= (int64_t)n) ++g;
  return g;
}

// Everything a kernel needs to know about one instance.  Pointers are
// device pointers into the instance's slot.
struct InstDesc {
  int32_t n, k, kg, kls;      // k = candidates per node, kg = geometric list
  int32_t kind, sym, dstar;
  int32_t ants, iterations, local_search;
  int32_t ls_op;              // local-search operator: 2 the 2-opt, 3 the 3-opt (symmetric only)
  int32_t bf_period, restart_stall, ugb_max;
  uint32_t seed_lo, seed_hi;
  double rho, p_x, xi_bf, lambda_bf, min_gain;
  float keep_f;               // (float)(1 - rho)
  double theta_h;
  const double* xy;           // [n][2] or null
  const double* dist;         // [n][n] or null
  const int32_t* row_ptr;     // heatmap CSR
  const int32_t* col;
  const float* val;
  int32_t* cand;              // [n][k]
  uint2* cw;                  // [n][k] {candidate id, bits of tau * S}: one 8-byte load per slot
  const float* heur;          // [n][k]  S = eta^beta e^kappa
  float* tau;                 // [n][k]
  float* w;                   // [n][k]  tau * S
  int32_t* geo;               // [n][kg] geometric nearest neighbours
  uint16_t* geo16;            // [n][64] the same lists as uint16, rows padded to 64
                              // entries (n <= 65535, else null): one 8-byte load
                              // per lane reads four entries
  int32_t* tours;             // [ants][n]
  double* lens;               // [ants]
  int32_t* t_gb;              // [n]
  int32_t* t_rb;              // [n]
  int32_t* t_ib;              // [n] local-search copy of the iteration best
  int32_t* nn_tour;           // [n]
  int32_t* succ;              // [n]
  int32_t* pred;              // [n]
  int32_t* ls_work;           // [3n] pos, queue, in-queue for 2-opt ([ants][3n] when
                              // every ant's tour is searched; dir_work_stride(n) bytes
                              // per tour for the directed 2-opt's arrays)
  int32_t* nl_in;             // [2][n][kls] incoming, then outgoing lists (ATSP with local search), else null
  int32_t gside;              // grid cells per side (0: no grid)
  int32_t* g_start;           // [side^2 + 1] first slot of each cell
  int32_t* g_cur;             // [side^2] build cursors
  int32_t* g_ids;             // [n] node ids, grouped by cell
  double* g_xy;               // [n][2] their coordinates, same order
  GridPar* g_par;             // filled by the grid build
  State* st;
  double* tr_lib;             // [iterations] or null
  double* tr_lgb;             // [iterations] or null
  int32_t* tr_elite;          // [iterations] or null
};

// A tour of n nodes is a permutation of 0..n-1 only if the sum of its
// entries is n(n-1)/2 and the sum of their squares (n-1)n(2n-1)/6; here
// both modulo 2^32.  A construction step that took a wrong node (a duplicate
// in place of a missing node) changes both; the construction kernel checks
// them for every ant's tour.  The closed forms are evaluated exactly in 64
// bits (n <= 10^6) before the reduction.
__host__ __device__ inline bool tour_checksums_ok(int32_t n, uint32_t sum, uint32_t sum_sq) {
  const uint64_t N = (uint64_t)n;
  return sum == (uint32_t)(N * (N - 1) / 2) && sum_sq == (uint32_t)((N - 1) * N * (2 * N - 1) / 6);
}

// Bytes of the directed 2-opt's arrays for n nodes (edge lengths and prefix
// sums in both directions, block totals and block offsets of the prefix
// sums in both directions, tour, positions, queue, in-queue flags), and the
// 256-byte-aligned stride of one tour's part of the work area.
__host__ __device__ inline size_t dir_work_bytes(int32_t n) {
  return (size_t)8 * (4 * (size_t)n + 2) + (size_t)32 * ((size_t)n / 64 + 2) + (size_t)12 * n +
         (((size_t)n + 7) & ~(size_t)7);
}
__host__ __device__ inline size_t dir_work_stride(int32_t n) { return (dir_work_bytes(n) + 255) & ~(size_t)255; }

// One entry per construction block: instance and first ant (inst < 0: idle)
struct BlockMap {
  int32_t inst;
  int32_t ant0;
};

// One device-to-device copy of a gather: bytes is a multiple of 4 and both
// addresses are 4-byte aligned.
struct CopyItem {
  const void* src;
  void* dst;
  uint64_t bytes;
};

// ---- the allocation-free entry point (defined in hac_kernels.hip) ----
// bytes of the per-device scratch array every hac_decode_noalloc carves
static constexpr size_t kNoAllocBytes = (size_t)64 << 20;
// takes the array's device address on `device` (which must be current);
// once per device, later calls return at once
hipError_t noalloc_scratch_init(int32_t device);
// the address taken by noalloc_scratch_init, or null
void* noalloc_scratch(int32_t device);
// serialises allocation-free decodes on one device (they share its array)
std::mutex* noalloc_call_lock(int32_t device);

// ---- launchers (defined in hac_kernels.hip) ----
// all items of a list (device memory) in one launch; max_bytes bounds the
// largest item
hipError_t launch_copy_items(const CopyItem* d_items, int32_t count, uint64_t max_bytes, hipStream_t s);
// candidate and geometric lists of every instance (and each node's nearest
// neighbour, in the successor array)
hipError_t launch_candidates(const InstDesc* d_insts, int32_t count, int32_t max_n, hipStream_t s);
hipError_t launch_nn_tour(const InstDesc* d_insts, int32_t count, int32_t max_n, hipStream_t s);
// 2-opt launches: max_n is the largest symmetric instance with local search
// (0: none, and the symmetric kernel is not launched); all_coords = 1 when
// every such instance has coordinates (the FP32-filtered LDS mode needs
// them); max_n_dir: largest ATSP instance with local search (0: none); such
// instances take the directed 2-opt (and their neighbour lists are built
// first); max_kls_dir: their largest k_ls; max_n3: the largest symmetric
// instance with the 3-opt (0: none; such instances are left out of max_n);
// all_coords3 = 1 when every 3-opt instance has coordinates
hipError_t launch_two_opt_nn(const InstDesc* d_insts, int32_t count, int32_t max_n, int32_t all_coords,
                             int32_t max_n_dir, int32_t max_kls_dir, int32_t max_n3, int32_t all_coords3,
                             hipStream_t s);
hipError_t launch_init(const InstDesc* d_insts, int32_t count, hipStream_t s);
// builds the coordinate grid of every instance that has one
hipError_t launch_grid(const InstDesc* d_insts, int32_t count, hipStream_t s);
// Waves per construction block, at most (its launch bounds: 256 threads).
constexpr int kMaxConstructWaves = 4;

// geo_mode: how an exhausted row consults its geometric list before a
// scan: 0 not at all, 1 int32 lists loaded at the top of each step, 2
// uint16 lists loaded one step ahead (every instance has geo16).
// grid = 0 when no instance of the launch has a coordinate grid: the grid
// search is then compiled out of the kernel (results do not depend on it).
// step_cap < n (timing launches only): each ant stops after step_cap tour
// positions and writes neither its length nor its checks
hipError_t launch_construct(const InstDesc* d_insts, const BlockMap* d_map, int32_t blocks,
                            int32_t ants_per_block, int32_t rows_per_wave, int32_t staged,
                            int32_t bytes, int32_t max_k, size_t lds_bytes, int32_t geo_mode,
                            int32_t grid, hipStream_t s, int32_t step_cap = INT32_MAX);
// tours_per_inst: blocks per instance (the largest ant count among instances
// that search every ant's tour, else 1)
hipError_t launch_local_search(const InstDesc* d_insts, int32_t count, int32_t max_n,
                               int32_t all_coords, int32_t tours_per_inst, int32_t max_n_dir,
                               int32_t max_kls_dir, int32_t max_n3, int32_t all_coords3, hipStream_t s);
hipError_t launch_iter_end(const InstDesc* d_insts, int32_t count, hipStream_t s);
hipError_t launch_finish(const InstDesc* d_insts, int32_t count, int32_t* const* d_out_tours,
                         double* d_out_lens, hipStream_t s);

// lanes per ant in the construction kernel (one 16-lane row)
int32_t construct_group_lanes(int32_t max_k);
// LDS layout of one construction block, in 32-bit words: the visited
// bitsets of the rows that carry ants (rows_per_wave of each wave's four;
// the other rows follow row 0 of their wave and read its bitset),
// optionally each such row's list of unvisited nodes (uint16), and for
// staged launches the candidate table (8-byte {id, weight} entries, or ids
// as uint16 and weights as FP32, six bytes per slot) and the coordinates.
struct ConstructLds {
  size_t rows, vis_words, list_words, total;  // total in bytes
};
__host__ __device__ inline size_t staged_ids_bytes(int32_t n, int32_t k) {
  return (((size_t)n * k * 2 + 15) / 16) * 16;
}
// staged: 0 none, 1 8-byte {id, weight} entries, 2 uint16 ids + FP32 weights,
// 3 as 2 without the coordinates
__host__ __device__ inline ConstructLds construct_lds_layout(int32_t n, int32_t k, int32_t ants_per_block,
                                                             int32_t rows_per_wave, int32_t staged, bool lists,
                                                             bool bytes) {
  ConstructLds L;
  L.rows = (size_t)rows_per_wave * (size_t)((ants_per_block + rows_per_wave - 1) / rows_per_wave);
  // visited marks per row: one byte per node (16-byte aligned), or one bit
  L.vis_words = bytes ? (size_t)(((n + 15) >> 4) << 2) : (size_t)(((((n + 63) >> 6) << 1) + 3) & ~3);
  L.list_words = (size_t)(((n + 7) >> 3) << 2);  // n uint16 rounded up to 16 bytes
  size_t total = L.rows * L.vis_words * 4;
  if (lists) total += L.rows * L.list_words * 4;
  // staged table (8-byte entries, or uint16 ids then FP32 weights), then the coordinates
  if (staged == 1) total += (((size_t)n * k * 8 + 15) / 16) * 16 + (size_t)16 * n;
  if (staged == 2) total += staged_ids_bytes(n, k) + (((size_t)n * k * 4 + 15) / 16) * 16 + (size_t)16 * n;
  if (staged == 3) total += staged_ids_bytes(n, k) + (((size_t)n * k * 4 + 15) / 16) * 16;
  L.total = total;
  return L;
}
// whether byte marks (with unvisited lists) fit a construction block
bool construct_bytes_fit(int32_t n, int32_t k, int32_t ants_per_block, int32_t rows_per_wave,
                         int32_t staged);
// LDS the construction kernel needs for one block (with bit marks, the lists
// are included when they fit)
size_t construct_lds_bytes(int32_t n, int32_t k, int32_t ants_per_block, int32_t rows_per_wave,
                           int32_t staged, int32_t bytes);
int32_t max_lds_bytes();

}  // namespace hac
