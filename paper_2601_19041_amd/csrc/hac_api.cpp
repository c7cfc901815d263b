// C ABI and host runtime of the decoder: validation, device slots,
// preparation, launch shapes, iteration replay and results.  Every search
// step runs in the kernels of hac_kernels.hip; the host only marshals
// inputs, folds the evidence factor once per instance (hac_fold.cpp) and
// sequences launches.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hac_runtime.h"

namespace hac {

// ------------------------------------------------------------------------
// device arena
// ------------------------------------------------------------------------
DeviceArena::~DeviceArena() { release(); }

void DeviceArena::release() {
  if (base_) (void)hipFree(base_);
  base_ = nullptr;
  cap_ = used_ = 0;
}

hipError_t DeviceArena::reserve(size_t bytes) {
  used_ = 0;
  if (bytes <= cap_) return hipSuccess;
  release();
  hipError_t e = hipMalloc((void**)&base_, bytes);
  if (e != hipSuccess) {
    base_ = nullptr;
    return e;
  }
  cap_ = bytes;
  return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

void* DeviceArena::carve(size_t bytes) {
  void* p = base_ + used_;
  used_ += align256(bytes);
  return p;
}

// ------------------------------------------------------------------------
// validation (the same checks before any device work)
// ------------------------------------------------------------------------
int32_t degree_target_of(const hac_instance* inst, const hac_params* p) {
  if (p->degree_target > 0) return p->degree_target;
  return (inst->kind == HAC_COORDS_EUC2D || inst->symmetric) ? 2 : 1;
}

static bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

hac_status validate(const hac_instance* inst, const hac_csr* csr, const hac_params* p,
                    std::string* why) {
  auto fail = [&](hac_status s, const char* m) {
    if (why) *why = m;
    return s;
  };
  if (!inst || !csr || !p) return fail(HAC_EINVAL, "null argument");
  const int32_t n = inst->n;
  if (n < 1) return fail(HAC_EINVAL, "n < 1");
  if (n > HAC_MAX_N) return fail(HAC_EUNSUPPORTED, "n above HAC_MAX_N");
  if (csr->n != n) return fail(HAC_EINVAL, "heatmap size differs from n");
  if (inst->kind == HAC_COORDS_EUC2D) {
    if (!inst->coords) return fail(HAC_EINVAL, "coords missing");
    for (int64_t x = 0; x < 2 * (int64_t)n; ++x)
      if (!std::isfinite(inst->coords[x])) return fail(HAC_EINVAL, "non-finite coordinate");
  } else if (inst->kind == HAC_MATRIX) {
    if (!inst->dist) return fail(HAC_EINVAL, "distance matrix missing");
    for (int32_t i = 0; i < n; ++i)
      for (int32_t j = 0; j < n; ++j) {
        const double v = inst->dist[(int64_t)i * n + j];
        if (!std::isfinite(v) || (i != j && v < 0.0)) return fail(HAC_EINVAL, "bad distance entry");
        if (inst->symmetric && j < i && v != inst->dist[(int64_t)j * n + i])
          return fail(HAC_EINVAL, "symmetric matrix is not symmetric");
      }
  } else {
    return fail(HAC_EINVAL, "unknown instance kind");
  }
  if (!csr->row_ptr) return fail(HAC_EINVAL, "row_ptr missing");
  if (csr->row_ptr[0] != 0 || csr->row_ptr[n] != csr->nnz || csr->nnz < 0)
    return fail(HAC_EINVAL, "row_ptr does not span nnz");
  if (csr->nnz > 0 && (!csr->col || !csr->val)) return fail(HAC_EINVAL, "col/val missing");
  {
    std::vector<int32_t> seen(n, -1);
    for (int32_t i = 0; i < n; ++i) {
      if (csr->row_ptr[i + 1] < csr->row_ptr[i]) return fail(HAC_EINVAL, "row_ptr not monotone");
      for (int32_t e = csr->row_ptr[i]; e < csr->row_ptr[i + 1]; ++e) {
        const int32_t j = csr->col[e];
        if (j < 0 || j >= n) return fail(HAC_EINVAL, "column out of range");
        if (seen[j] == i) return fail(HAC_EINVAL, "duplicate column in a row");
        seen[j] = i;
        const float v = csr->val[e];
        if (!std::isfinite(v) || v < 0.0f) return fail(HAC_EINVAL, "heatmap value not finite/>=0");
      }
    }
  }
  if (p->ants < 1 || p->iterations < 0 || p->k < 1) return fail(HAC_EINVAL, "ants/k/iterations");
  if (!(p->rho > 0.0 && p->rho < 1.0)) return fail(HAC_EINVAL, "rho outside (0,1)");
  if (!(p->p_best > 0.0 && p->p_best < 1.0)) return fail(HAC_EINVAL, "p_best outside (0,1)");
  if (!finite_nonneg(p->beta) || !finite_nonneg(p->c_cap) || !finite_nonneg(p->theta_h) ||
      !(p->eps > 0.0 && std::isfinite(p->eps)) || !(p->xi_bf >= 0.0 && p->xi_bf <= 1.0) ||
      !std::isfinite(p->lambda_bf) || !finite_nonneg(p->clip) || !std::isfinite(p->kappa_fixed))
    return fail(HAC_EINVAL, "parameter out of range");
  if (p->degree_target < 0 || p->bf_period < 0 || p->restart_stall < 0 || p->ugb_max < 1 ||
      (p->baseline_scope != 0 && p->baseline_scope != 1) ||
      p->local_search < 0 || p->local_search > 2 || (p->local_search && p->k_ls < 1))
    return fail(HAC_EINVAL, "integer parameter out of range");
  if (p->alpha != 1.0) return fail(HAC_EUNSUPPORTED, "only alpha = 1 is supported");
  if (p->k > HAC_MAX_K) return fail(HAC_EUNSUPPORTED, "k above HAC_MAX_K");
  if (p->local_search && p->k_ls > HAC_MAX_KLS) return fail(HAC_EUNSUPPORTED, "k_ls above HAC_MAX_KLS");
  if (p->ls_op != 0 && p->ls_op != 2 && p->ls_op != 3) return fail(HAC_EINVAL, "ls_op is not 2 or 3");
  if (p->local_search && p->ls_op == 3 && inst->kind == HAC_MATRIX && !inst->symmetric)
    return fail(HAC_EUNSUPPORTED, "the 3-opt is for symmetric instances (the ATSP takes the directed 2-opt)");
  return HAC_OK;
}

// ------------------------------------------------------------------------
// slots
// ------------------------------------------------------------------------
Layout make_layout(const hac_instance* inst, const hac_csr* csr, const hac_params* p) {
  Layout L;
  L.n = inst->n;
  L.k = std::min(p->k, inst->n - 1);
  L.kg = std::min(inst->n - 1, 64);
  L.kls = p->local_search ? std::min(p->k_ls, inst->n - 1) : 0;
  L.ants = p->ants;
  L.iterations = p->iterations;
  L.coords = inst->kind == HAC_COORDS_EUC2D;
  L.ls = p->local_search != 0;
  L.directed = L.ls && inst->kind == HAC_MATRIX && !inst->symmetric;
  L.ls_tours = p->local_search == 2 ? p->ants : 1;
  L.three_opt = L.ls && !L.directed && p->ls_op == 3;
  L.nnz = csr->nnz;
  L.gside = (L.coords && L.n >= kGridMinN) ? grid_side(L.n) : 0;
  return L;
}

size_t Layout::bytes() const {
  const size_t nn = (size_t)n, nk = nn * (size_t)k;
  size_t b = 0;
  b += align256(coords ? 16 * nn : 8 * nn * nn);
  b += align256(4 * (nn + 1)) + align256(4 * (size_t)nnz) + align256(4 * (size_t)nnz);
  b += align256(4 * nk) + align256(8 * nk + 16) + 3 * align256(4 * nk + 16);
  b += align256(4 * nn * (size_t)kg);
  b += n <= 65535 ? align256(128 * nn) : 0;
  b += align256(4 * nn * (size_t)ants) + align256(8 * (size_t)ants);
  b += 6 * align256(4 * nn);
  b += ls ? align256((directed ? dir_work_stride(n) : 12 * nn) * (size_t)ls_tours) : 0;
  b += directed ? align256(8 * nn * (size_t)kls) : 0;
  if (gside > 0) {
    const size_t cells = (size_t)gside * gside;
    b += align256(4 * (cells + 1)) + align256(4 * cells) + align256(4 * nn) + align256(16 * nn) +
         align256(sizeof(GridPar));
  }
  b += align256(sizeof(State));
  b += 3 * align256(8 * (size_t)std::max(iterations, 1));
  return b;
}

void assign_slot(HostInst& h, const std::function<void*(size_t)>& carve) {
  const Layout& L = h.lay;
  const size_t nn = (size_t)L.n, nk = nn * (size_t)L.k;
  InstDesc& d = h.d;
  d.xy = L.coords ? (const double*)carve(16 * nn) : nullptr;
  d.dist = L.coords ? nullptr : (const double*)carve(8 * nn * nn);
  d.row_ptr = (const int32_t*)carve(4 * (nn + 1));
  d.col = (const int32_t*)carve(4 * (size_t)L.nnz);
  d.val = (const float*)carve(4 * (size_t)L.nnz);
  d.cand = (int32_t*)carve(4 * nk);
  d.cw = (uint2*)carve(8 * nk + 16);
  d.heur = (const float*)carve(4 * nk + 16);
  d.tau = (float*)carve(4 * nk + 16);
  d.w = (float*)carve(4 * nk + 16);
  d.geo = (int32_t*)carve(4 * nn * (size_t)L.kg);
  d.geo16 = L.n <= 65535 ? (uint16_t*)carve(128 * nn) : nullptr;
  d.tours = (int32_t*)carve(4 * nn * (size_t)L.ants);
  d.lens = (double*)carve(8 * (size_t)L.ants);
  d.t_gb = (int32_t*)carve(4 * nn);
  d.t_rb = (int32_t*)carve(4 * nn);
  d.t_ib = (int32_t*)carve(4 * nn);
  d.nn_tour = (int32_t*)carve(4 * nn);
  d.succ = (int32_t*)carve(4 * nn);
  d.pred = (int32_t*)carve(4 * nn);
  d.ls_work = L.ls ? (int32_t*)carve((L.directed ? dir_work_stride(L.n) : 12 * nn) * (size_t)L.ls_tours) : nullptr;
  d.nl_in = L.directed ? (int32_t*)carve(8 * nn * (size_t)L.kls) : nullptr;
  d.gside = L.gside;
  if (L.gside > 0) {
    const size_t cells = (size_t)L.gside * L.gside;
    d.g_start = (int32_t*)carve(4 * (cells + 1));
    d.g_cur = (int32_t*)carve(4 * cells);
    d.g_ids = (int32_t*)carve(4 * nn);
    d.g_xy = (double*)carve(16 * nn);
    d.g_par = (GridPar*)carve(sizeof(GridPar));
  } else {
    d.g_start = d.g_cur = d.g_ids = nullptr;
    d.g_xy = nullptr;
    d.g_par = nullptr;
  }
  d.st = (State*)carve(sizeof(State));
  const size_t it = 8 * (size_t)std::max(L.iterations, 1);
  d.tr_lib = (double*)carve(it);
  d.tr_lgb = (double*)carve(it);
  d.tr_elite = (int32_t*)carve(it);
}

void fill_desc_scalars(HostInst& h) {
  const Layout& L = h.lay;
  const hac_params& p = h.p;
  InstDesc& d = h.d;
  d.n = L.n;
  d.k = L.k;
  d.kg = L.kg;
  d.kls = L.kls;
  d.kind = h.inst.kind;
  d.sym = h.sym;
  d.dstar = h.dstar;
  d.ants = p.ants;
  d.iterations = p.iterations;
  d.local_search = p.local_search;
  d.ls_op = L.three_opt ? 3 : 2;
  d.bf_period = p.bf_period;
  d.restart_stall = p.restart_stall;
  d.ugb_max = p.ugb_max;
  d.seed_lo = (uint32_t)h.seed;
  d.seed_hi = (uint32_t)(h.seed >> 32);
  d.rho = p.rho;
  d.p_x = h.p_x;
  d.xi_bf = p.xi_bf;
  d.lambda_bf = p.lambda_bf;
  d.min_gain = 0.0;
  d.keep_f = (float)(1.0 - p.rho);
  d.theta_h = p.theta_h;
}

hipError_t upload_inputs(const HostInst& h, hipStream_t s) {
  const Layout& L = h.lay;
  const size_t nn = (size_t)L.n;
  const hac_instance& I = h.from_device ? h.dev_inst : h.inst;
  const hac_csr& C = h.from_device ? h.dev_csr : h.csr;
  const hipMemcpyKind kind = h.from_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  hipError_t e;
  if (L.coords)
    e = hipMemcpyAsync((void*)h.d.xy, I.coords, 16 * nn, kind, s);
  else
    e = hipMemcpyAsync((void*)h.d.dist, I.dist, 8 * nn * nn, kind, s);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync((void*)h.d.row_ptr, C.row_ptr, 4 * (nn + 1), kind, s);
  if (e != hipSuccess) return e;
  if (L.nnz > 0) {
    e = hipMemcpyAsync((void*)h.d.col, C.col, 4 * (size_t)L.nnz, kind, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync((void*)h.d.val, C.val, 4 * (size_t)L.nnz, kind, s);
  }
  return e;
}

// ------------------------------------------------------------------------
// preparation
// ------------------------------------------------------------------------
#define HAC_HIP(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) {                                                  \
      if (err) *err = std::string(#expr) + ": " + hipGetErrorString(e_);    \
      return HAC_EDEVICE;                                                    \
    }                                                                        \
  } while (0)

static void parallel_for(int count, const std::function<void(int)>& fn) {
  const int hw = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int workers = std::min(count, hw);
  if (workers <= 1) {
    for (int x = 0; x < count; ++x) fn(x);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  for (int w = 0; w < workers; ++w)
    pool.emplace_back([&] {
      for (int x = next++; x < count; x = next++) fn(x);
    });
  for (auto& t : pool) t.join();
}

// Moves many device arrays to or from one host blob through a staging
// arena: one gather (or scatter) launch and one copy instead of a copy per
// array.  `items` give the device side (src for a readback, dst for an
// upload) and the host offsets; the staging regions follow `base`.
static hipError_t stage_copies(DeviceArena& stage, std::vector<CopyItem>& items, const std::vector<size_t>& host_at,
                               char* host, size_t bytes, bool to_host, hipStream_t s) {
  const size_t list_bytes = sizeof(CopyItem) * items.size();
  hipError_t e = stage.reserve(align256(bytes) + align256(list_bytes));
  if (e != hipSuccess) return e;
  char* base = (char*)stage.carve(bytes);
  CopyItem* d_list = (CopyItem*)stage.carve(list_bytes);
  uint64_t maxb = 0;
  for (size_t q = 0; q < items.size(); ++q) {
    if (to_host)
      items[q].dst = base + host_at[q];
    else
      items[q].src = base + host_at[q];
    maxb = std::max<uint64_t>(maxb, items[q].bytes);
  }
  if (!to_host && (e = hipMemcpyAsync(base, host, bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(d_list, items.data(), list_bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
  e = launch_copy_items(d_list, (int32_t)items.size(), maxb, s);
  if (e == hipErrorInvalidValue) {  // an item too large for one launch
    e = hipSuccess;
    for (size_t q = 0; q < items.size() && e == hipSuccess; ++q)
      e = hipMemcpyAsync(items[q].dst, items[q].src, items[q].bytes, hipMemcpyDeviceToDevice, s);
  }
  if (e != hipSuccess) return e;
  if (to_host) e = hipMemcpyAsync(host, base, bytes, hipMemcpyDeviceToHost, s);
  return e;
}

hac_status prepare_instances(std::vector<HostInst>& hs, InstDesc* d_descs, hipStream_t s,
                             std::string* err, DeviceArena* stage) {
  const int count = (int)hs.size();
  int32_t max_n = 0;
  for (auto& h : hs) max_n = std::max(max_n, h.lay.n);
  // candidate and geometric lists (eq. 3)
  HAC_HIP(launch_candidates(d_descs, count, max_n, s));
  std::vector<std::vector<int32_t>> nn1(count);  // each node's nearest neighbour
  for (int x = 0; x < count; ++x) {
    HostInst& h = hs[x];
    h.cand_h.resize((size_t)h.lay.n * h.lay.k);
    nn1[x].resize((size_t)h.lay.n);
  }
  if (stage) {
    std::vector<CopyItem> items;
    std::vector<size_t> at;
    size_t bytes = 0;
    for (int x = 0; x < count; ++x) {
      const HostInst& h = hs[x];
      items.push_back(CopyItem{h.d.cand, nullptr, 4 * (uint64_t)h.cand_h.size()});
      at.push_back(bytes);
      bytes += align256(4 * h.cand_h.size());
      items.push_back(CopyItem{h.d.succ, nullptr, 4 * (uint64_t)h.lay.n});
      at.push_back(bytes);
      bytes += align256(4 * (size_t)h.lay.n);
    }
    std::vector<char> blob(bytes);
    HAC_HIP(stage_copies(*stage, items, at, blob.data(), bytes, true, s));
    HAC_HIP(hipStreamSynchronize(s));
    for (int x = 0; x < count; ++x) {
      std::memcpy(hs[x].cand_h.data(), blob.data() + at[2 * x], 4 * hs[x].cand_h.size());
      std::memcpy(nn1[x].data(), blob.data() + at[2 * x + 1], 4 * nn1[x].size());
    }
  } else {
    for (int x = 0; x < count; ++x) {
      HostInst& h = hs[x];
      HAC_HIP(hipMemcpyAsync(h.cand_h.data(), h.d.cand, 4 * h.cand_h.size(), hipMemcpyDeviceToHost, s));
      HAC_HIP(hipMemcpyAsync(nn1[x].data(), h.d.succ, 4 * (size_t)h.lay.n, hipMemcpyDeviceToHost, s));
    }
    HAC_HIP(hipStreamSynchronize(s));
  }
  // host fold (eq. 9-14)
  std::vector<std::vector<float>> heur(count);
  std::vector<int> frc(count, FOLD_OK);
  std::vector<double> lbs(count, 0.0);
  parallel_for(count, [&](int x) {
    HostInst& h = hs[x];
    const Layout& L = h.lay;
    FoldInput in{};
    in.n = L.n;
    in.k = L.k;
    in.dstar = h.dstar;
    in.local_search = h.p.local_search;
    in.baseline_scope = h.p.baseline_scope;
    in.coords = h.inst.kind == HAC_COORDS_EUC2D ? h.inst.coords : nullptr;
    in.dist = h.inst.kind == HAC_MATRIX ? h.inst.dist : nullptr;
    in.row_ptr = h.csr.row_ptr;
    in.col = h.csr.col;
    in.val = h.csr.val;
    in.theta_h = h.p.theta_h;
    in.eps = h.p.eps;
    in.c_cap = h.p.c_cap;
    in.kappa_fixed = h.p.kappa_fixed;
    in.alpha = h.p.alpha;
    in.beta = h.p.beta;
    in.clip = h.p.clip;
    in.p_best = h.p.p_best;
    in.rho = h.p.rho;
    const size_t nk = (size_t)L.n * L.k;
    if (h.want_evid) {
      h.evid_gt1.assign(nk, 0);
      in.evid_gt1 = h.evid_gt1.data();
    }
    heur[x].assign(nk + 4, 0.0f);
    frc[x] = fold_instance(in, h.cand_h.data(), heur[x].data(), &h.fold);
    // lower bound on any tour: every node leaves once, at least to its nearest
    double lb = 0.0;
    for (int32_t i = 0; i < L.n; ++i) {
      const int32_t j = nn1[x][(size_t)i];
      if (in.coords) {
        const double dx = in.coords[2 * i] - in.coords[2 * j];
        const double dy = in.coords[2 * i + 1] - in.coords[2 * j + 1];
        lb += std::sqrt(dx * dx + dy * dy);
      } else {
        lb += in.dist[(int64_t)i * L.n + j];
      }
    }
    lbs[x] = lb;
  });
  for (int x = 0; x < count; ++x) {
    if (frc[x] == FOLD_BAD_DISTANCE) {
      if (err) *err = "instance " + std::to_string(x) + ": a candidate edge has distance <= 0";
      return HAC_EINVAL;
    }
    if (frc[x] == FOLD_RANGE) {
      if (err) *err = "instance " + std::to_string(x) + ": heuristic weight outside FP32 range";
      return HAC_ERANGE;
    }
  }
  std::vector<char> heur_blob;  // kept until the stream is synchronised below
  if (stage) {
    std::vector<CopyItem> items;
    std::vector<size_t> at;
    size_t bytes = 0;
    for (int x = 0; x < count; ++x) {
      const size_t nk = (size_t)hs[x].lay.n * hs[x].lay.k;
      items.push_back(CopyItem{nullptr, (void*)hs[x].d.heur, 4 * (uint64_t)nk});
      at.push_back(bytes);
      bytes += align256(4 * nk);
    }
    heur_blob.resize(bytes);
    for (int x = 0; x < count; ++x) std::memcpy(heur_blob.data() + at[x], heur[x].data(), items[x].bytes);
    HAC_HIP(stage_copies(*stage, items, at, heur_blob.data(), bytes, false, s));
  } else {
    for (int x = 0; x < count; ++x) {
      HostInst& h = hs[x];
      const size_t nk = (size_t)h.lay.n * h.lay.k;
      HAC_HIP(hipMemcpyAsync((void*)h.d.heur, heur[x].data(), 4 * nk, hipMemcpyHostToDevice, s));
    }
  }
  // coordinate grids, NN tour (+ 2-opt), then the range check on the first bounds
  HAC_HIP(launch_grid(d_descs, count, s));
  HAC_HIP(launch_nn_tour(d_descs, count, max_n, s));
  bool any_ls = false;
  int32_t all_coords = 1, max_n_dir = 0, max_kls_dir = 0, max_n_sym = 0, max_n3 = 0, all_coords3 = 1;  // largest directed / symmetric
  for (auto& h : hs) {
    any_ls |= h.p.local_search != 0;
    if (h.lay.directed) max_n_dir = std::max(max_n_dir, h.lay.n), max_kls_dir = std::max(max_kls_dir, h.lay.kls);
    else if (h.lay.three_opt) max_n3 = std::max(max_n3, h.lay.n);
    else if (h.p.local_search) max_n_sym = std::max(max_n_sym, h.lay.n);
    if (h.p.local_search && !h.lay.directed && !h.lay.three_opt && !h.lay.coords) all_coords = 0;
    if (h.lay.three_opt && !h.lay.coords) all_coords3 = 0;
  }
  if (any_ls) HAC_HIP(launch_two_opt_nn(d_descs, count, max_n_sym, all_coords, max_n_dir, max_kls_dir, max_n3, all_coords3, s));
  std::vector<State> sts(count);
  if (stage) {
    // after the weights' scatter on the same stream: the staging arena is reused
    std::vector<CopyItem> items;
    std::vector<size_t> at;
    for (int x = 0; x < count; ++x) {
      items.push_back(CopyItem{hs[x].d.st, nullptr, sizeof(State)});
      at.push_back((size_t)x * align256(sizeof(State)));
    }
    std::vector<char> blob((size_t)count * align256(sizeof(State)));
    HAC_HIP(hipStreamSynchronize(s));
    HAC_HIP(stage_copies(*stage, items, at, blob.data(), blob.size(), true, s));
    HAC_HIP(hipStreamSynchronize(s));
    for (int x = 0; x < count; ++x) std::memcpy(&sts[x], blob.data() + at[x], sizeof(State));
  } else {
    for (int x = 0; x < count; ++x)
      HAC_HIP(hipMemcpyAsync(&sts[x], hs[x].d.st, sizeof(State), hipMemcpyDeviceToHost, s));
    HAC_HIP(hipStreamSynchronize(s));
  }
  for (int x = 0; x < count; ++x) {
    HostInst& h = hs[x];
    h.l_nn = sts[x].l_gb;
    FoldInput in{};
    in.n = h.lay.n;
    in.k = h.lay.k;
    in.local_search = h.p.local_search;
    in.rho = h.p.rho;
    if (fold_check_range(in, h.fold, lbs[x], h.l_nn, h.p_x) != FOLD_OK) {
      if (err) *err = "instance " + std::to_string(x) + ": choice weights would leave FP32 range";
      return HAC_ERANGE;
    }
  }
  HAC_HIP(launch_init(d_descs, count, s));
  return HAC_OK;
}

// ------------------------------------------------------------------------
// XCD-aware block map.  Workgroups are dealt to the 8 XCDs round-robin by
// block index, so block b = 8 r + x lands on XCD x; each instance's ant
// groups are kept on one XCD (its rows then live in that XCD's L2) unless
// it is large enough to fill several.
// ------------------------------------------------------------------------
static constexpr int kXcds = 8;

std::vector<BlockMap> build_block_map(const std::vector<HostInst>& hs, int32_t apb) {
  std::vector<std::vector<BlockMap>> bins(kXcds);
  std::vector<double> load(kXcds, 0.0);
  std::vector<int> order(hs.size());
  for (size_t x = 0; x < hs.size(); ++x) order[x] = (int)x;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    double la = (double)hs[a].lay.n * hs[a].p.ants, lb = (double)hs[b].lay.n * hs[b].p.ants;
    return la > lb || (la == lb && a < b);
  });
  for (int x : order) {
    const int groups = (hs[x].p.ants + apb - 1) / apb;
    const double per_group = (double)hs[x].lay.n * apb;
    if (groups >= 64) {
      for (int g = 0; g < groups; ++g) {
        int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        bins[b].push_back({x, g * apb});
        load[b] += per_group;
      }
    } else {
      int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      for (int g = 0; g < groups; ++g) bins[b].push_back({x, g * apb});
      load[b] += per_group * groups;
    }
  }
  size_t rounds = 0;
  for (auto& b : bins) rounds = std::max(rounds, b.size());
  std::vector<BlockMap> map(rounds * kXcds, BlockMap{-1, 0});
  for (int b = 0; b < kXcds; ++b)
    for (size_t r = 0; r < bins[b].size(); ++r) map[r * kXcds + b] = bins[b][r];
  return map;
}

// ------------------------------------------------------------------------
// launch-shape autotuner
// ------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<std::string, LaunchShape> g_tune_cache;
static bool g_tune_loaded = false;

static const char* tune_cache_path() { return std::getenv("HAC_TUNE_CACHE"); }

static void tune_cache_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[256];
  int a, st, rpw, geo;
  while (std::fscanf(f, "%255s %d %d %d %d", key, &a, &st, &rpw, &geo) == 5) {
    LaunchShape sh{a, st, 0, rpw, 0};
    sh.geo = geo;
    g_tune_cache[key] = sh;
  }
  std::fclose(f);
}

static void tune_cache_store() {
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  for (auto& kv : g_tune_cache)
    std::fprintf(f, "%s %d %d %d %d\n", kv.first.c_str(), kv.second.ants_per_block, kv.second.staged,
                 kv.second.rows_per_wave, kv.second.geo);
  std::fclose(f);
}

// byte marks when they fit every instance of the batch
static LaunchShape with_marks(const std::vector<HostInst>& hs, LaunchShape sh) {
  sh.bytes = 1;
  sh.grid = 0;
  for (auto& h : hs) {
    if (!construct_bytes_fit(h.lay.n, h.lay.k, sh.ants_per_block, sh.rows_per_wave, sh.staged)) sh.bytes = 0;
    if (h.lay.gside > 0) sh.grid = 1;
  }
  return sh;
}

static bool shape_fits(const std::vector<HostInst>& hs, LaunchShape sh) {
  for (auto& h : hs) {
    if (sh.rows_per_wave < 1 || sh.rows_per_wave > 4 ||
        construct_lds_bytes(h.lay.n, h.lay.k, sh.ants_per_block, sh.rows_per_wave, sh.staged, sh.bytes) >
            (size_t)max_lds_bytes())
      return false;
  }
  return true;
}

std::vector<int32_t> geo_modes(const std::vector<HostInst>& hs, int32_t staged) {
  bool all16 = true;
  for (auto& h : hs) all16 &= h.lay.n <= 65535;
  if (const char* f = std::getenv("HAC_GEO_MODE")) {
    const int m = std::atoi(f);
    if (m == 0 || m == 1 || (m == 2 && all16)) return {m};
  }
  // staged tables: uint16 lists a step ahead whenever every instance has them
  // (faster over whole decodes; the tuner's first-iteration timing cannot
  // tell the two list forms apart)
  if (staged) return {all16 ? 2 : 1};
  return {0, all16 ? 2 : 1};
}

int32_t batch_max_k(const std::vector<HostInst>& hs) {
  int32_t k = 1;
  for (auto& h : hs) k = std::max(k, h.lay.k);
  return k;
}

size_t shape_lds(const std::vector<HostInst>& hs, LaunchShape sh) {
  size_t b = 0;
  for (auto& h : hs)
    b = std::max(b, construct_lds_bytes(h.lay.n, h.lay.k, sh.ants_per_block, sh.rows_per_wave, sh.staged,
                                        sh.bytes));
  return b;
}

// construction blocks have at most kMaxConstructWaves waves (the kernel's
// launch bounds), so that it may hold more than 128 registers per lane
static bool waves_ok(const LaunchShape& sh) {
  return sh.rows_per_wave >= 1 && (sh.ants_per_block + sh.rows_per_wave - 1) / sh.rows_per_wave <= kMaxConstructWaves;
}

static std::string shape_key(const std::vector<HostInst>& hs, bool shared = false) {
  int32_t max_n = 0, k = 0;
  int64_t ants = 0;
  for (auto& h : hs) {
    max_n = std::max(max_n, h.lay.n);
    k = std::max(k, h.lay.k);
    ants += h.p.ants;
  }
  int nb = 0;
  while ((1 << nb) < max_n) nb++;
  int ab = 0;
  while ((1ll << ab) < ants) ab++;
  return "gfx950v2/n" + std::to_string(nb) + "/k" + std::to_string(k) + "/a" + std::to_string(ab) +
         (hs[0].lay.coords ? "/euc" : "/mat") + (shared ? "/lane" : "");
}

// A launch shape chosen without timing anything (the allocation-free path):
// the tuner's cached choice for the batch's shape class if there is one,
// else the first that fits of 16 ants per block with 8-byte LDS entries,
// the two packed LDS forms, and one ant per wave with the table in global
// memory.  Results do not depend on the shape.
LaunchShape default_shape(const std::vector<HostInst>& hs) {
  const int32_t kmax = batch_max_k(hs);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache_load();
    auto it = g_tune_cache.find(shape_key(hs));
    if (it != g_tune_cache.end()) {
      LaunchShape sh = with_marks(hs, {it->second.ants_per_block, it->second.staged, kmax,
                                       it->second.rows_per_wave, 0});
      sh.geo = geo_modes(hs, sh.staged)[0];
      if (waves_ok(sh) && shape_fits(hs, sh)) return sh;
    }
  }
  for (int st : {1, 2, 3}) {
    LaunchShape sh = with_marks(hs, {16, st, kmax, 4, 0});
    if (shape_fits(hs, sh)) {
      sh.geo = geo_modes(hs, st)[0];
      return sh;
    }
  }
  LaunchShape sh = with_marks(hs, {4, 0, kmax, 1, 0});
  sh.geo = geo_modes(hs, 0)[0];
  return sh;
}

LaunchShape tune_shape(const std::vector<HostInst>& hs, const InstDesc* d_descs, hipStream_t s,
                       DeviceArena& scratch, bool* ok, bool shared) {
  *ok = true;
  const int32_t kmax = batch_max_k(hs);
  if (const char* force = std::getenv("HAC_SHAPE")) {
    // "A,staged[,rows]" pins the launch shape (used to show shape
    // independence): A ants per block, rows (1..4, default 4) ants per wave
    LaunchShape sh{1, 0, kmax, 4, 0};
    const int got = std::sscanf(force, "%d,%d,%d", &sh.ants_per_block, &sh.staged, &sh.rows_per_wave);
    if (got >= 2 && sh.ants_per_block >= 1 && sh.staged >= 0 && sh.staged <= 3) {
      if (got < 3 || sh.rows_per_wave < 1 || sh.rows_per_wave > 4) sh.rows_per_wave = 4;
      sh = with_marks(hs, sh);
      if (const char* bits = std::getenv("HAC_BIT_MARKS")) {
        if (bits[0] == '1') sh.bytes = 0;  // pins bit marks (shows both give the same tours)
      }
      sh.geo = geo_modes(hs, sh.staged)[0];
      if (waves_ok(sh) && shape_fits(hs, sh)) return sh;
    }
  }
  const std::string key = shape_key(hs, shared);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache_load();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      LaunchShape sh = with_marks(hs, {it->second.ants_per_block, it->second.staged, kmax,
                                       it->second.rows_per_wave, 0});
      sh.geo = it->second.geo;
      const std::vector<int32_t> gm = geo_modes(hs, sh.staged);
      if (std::find(gm.begin(), gm.end(), sh.geo) == gm.end()) sh.geo = gm[0];
      if (waves_ok(sh) && shape_fits(hs, sh)) return sh;
    }
  }
  // Staging forms tried: the table in global memory, and 8-byte entries in
  // LDS, or where those do not fit in any shape, the two packed forms (the
  // packed read costs a little more than one 8-byte read, so 8-byte entries
  // win wherever they fit).
  bool fits8 = false;
  for (int rpw : {4, 2, 1})
    for (int waves : {1, 2, 4}) fits8 |= shape_fits(hs, with_marks(hs, {rpw * waves, 1, kmax, rpw, 0}));
  std::vector<int> forms = fits8 ? std::vector<int>{0, 1} : std::vector<int>{0, 2, 3};
  std::vector<LaunchShape> cands;
  for (int rpw : {4, 2, 1})
    for (int waves : {1, 2, 4})
      for (int st : forms) {
        LaunchShape sh = with_marks(hs, {rpw * waves, st, kmax, rpw, 0});
        if (!shape_fits(hs, sh)) continue;
        for (int32_t g : geo_modes(hs, st)) {
          sh.geo = g;
          cands.push_back(sh);
        }
      }
  LaunchShape best = with_marks(hs, {4, 0, kmax, 4, 0});
  best.geo = geo_modes(hs, 0)[0];
  float best_ms = 1e30f;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    *ok = false;
    return best;
  }
  // shortest of `reps` launches of shape sh, each ant stopping after `cap`
  // tour positions (construction only reads the state, so repeating it is
  // harmless); negative on a failed call
  auto time_shape = [&](const LaunchShape& sh, int32_t cap, int reps) -> float {
    std::vector<BlockMap> map = build_block_map(hs, sh.ants_per_block);
    scratch.reset();
    if (scratch.reserve(map.size() * sizeof(BlockMap)) != hipSuccess) return -1.0f;
    BlockMap* d_map = (BlockMap*)scratch.carve(map.size() * sizeof(BlockMap));
    if (hipMemcpyAsync(d_map, map.data(), map.size() * sizeof(BlockMap), hipMemcpyHostToDevice, s) !=
        hipSuccess)
      return -1.0f;
    float ms_min = 1e30f;
    for (int rep = 0; rep < reps; ++rep) {
      (void)hipEventRecord(e0, s);
      (void)launch_construct(d_descs, d_map, (int32_t)map.size(), sh.ants_per_block, sh.rows_per_wave,
                             sh.staged, sh.bytes, sh.kmax, shape_lds(hs, sh), sh.geo, sh.grid, s, cap);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) return -1.0f;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms_min = std::min(ms_min, ms);
    }
    return ms_min;
  };
  // Successive halving for large instances: every candidate is timed once
  // on the first eighth of the tours, and the four fastest shapes are then
  // timed on whole tours, each with every geometric-list mode it was tried
  // with (a prefix has few exhausted rows, so it cannot rank the modes; a
  // whole launch of a 10^4-node batch takes milliseconds, and a serving
  // lane tunes whenever its batch changes class).  Smaller instances are
  // timed whole, twice.
  int32_t max_n = 0;
  for (auto& h : hs) max_n = std::max(max_n, h.lay.n);
  const int32_t prefix = std::max<int32_t>(512, max_n / 8);
  const bool halve = prefix < max_n && cands.size() > 4;
  std::vector<std::pair<float, size_t>> first;
  for (size_t x = 0; x < cands.size() && *ok; ++x) {
    const float ms = time_shape(cands[x], halve ? prefix : INT32_MAX, halve ? 1 : 2);
    if (ms < 0.0f) *ok = false;
    first.emplace_back(ms, x);
  }
  if (*ok && halve) {
    std::sort(first.begin(), first.end());
    auto same_shape = [&](size_t x, size_t y) {
      const LaunchShape &a = cands[x], &b = cands[y];
      return a.ants_per_block == b.ants_per_block && a.staged == b.staged && a.rows_per_wave == b.rows_per_wave &&
             a.bytes == b.bytes;
    };
    std::vector<size_t> lead;  // the four fastest shapes
    for (auto& f : first) {
      bool seen = false;
      for (size_t y : lead) seen |= same_shape(f.second, y);
      if (!seen && lead.size() < 4) lead.push_back(f.second);
    }
    std::vector<std::pair<float, size_t>> second;
    for (size_t x = 0; x < cands.size() && *ok; ++x) {
      bool in = false;
      for (size_t y : lead) in |= same_shape(x, y);
      if (!in) continue;
      const float ms = time_shape(cands[x], INT32_MAX, 1);
      if (ms < 0.0f) *ok = false;
      second.emplace_back(ms, x);
    }
    first.swap(second);
  }
  for (auto& f : first) {
    if (*ok && f.first < best_ms) {
      best_ms = f.first;
      best = cands[f.second];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (*ok) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = best;
    tune_cache_store();
  }
  return best;
}

}  // namespace hac

using namespace hac;

// ------------------------------------------------------------------------
// context
// ------------------------------------------------------------------------
struct hac_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint64_t budget = 0;
  std::string err;
  hac_stats stats{};
  bool timing = false;
  DeviceArena arena, scratch;
  DeviceArena stage;  // gathered inputs and copy lists of the device-input path
  std::vector<HostInst> last;  // descriptors of the last call (debug hooks)
  std::vector<hipEvent_t> events;
};

hipStream_t hac_context_stream(const hac_ctx* ctx) { return ctx->stream; }

static hac_status set_err(hac_ctx* c, hac_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

extern "C" {

void hac_params_default(hac_params* p) {
  if (!p) return;
  p->ants = 32;
  p->iterations = 5000;
  p->k = 20;
  p->k_ls = 20;
  p->local_search = 0;
  p->ls_op = 2;
  p->alpha = 1.0;
  p->beta = 2.0;
  p->rho = 0.2;
  p->p_best = 0.05;
  p->c_cap = 0.5;
  p->kappa_fixed = -1.0;
  p->theta_h = 1e-4;
  p->eps = 1e-9;
  p->xi_bf = 0.05;
  p->lambda_bf = 1.0 + 1e-5;
  p->clip = 40.0;
  p->degree_target = 0;
  p->bf_period = 100;
  p->restart_stall = 250;
  p->ugb_max = 25;
  p->baseline_scope = 0;
}

const char* hac_strerror(hac_status s) {
  switch (s) {
    case HAC_OK: return "ok";
    case HAC_EINVAL: return "invalid argument";
    case HAC_ENOMEM: return "out of device memory or budget";
    case HAC_EDEVICE: return "HIP device error";
    case HAC_EUNSUPPORTED: return "unsupported by this library";
    case HAC_EBUSY: return "not finished";
    case HAC_ECANCELLED: return "cancelled";
    case HAC_ERANGE: return "weights outside the FP32 range";
    default: return "unknown status";
  }
}

hac_status hac_validate(const hac_instance* inst, const hac_csr* heat, const hac_params* p) {
  return validate(inst, heat, p, nullptr);
}

hac_status hac_create(hac_ctx** out, int32_t device, void* stream, uint64_t hbm_budget_bytes) {
  if (!out) return HAC_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return HAC_EDEVICE;
  if (device < 0 || device >= ndev) return HAC_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return HAC_EDEVICE;
  // the allocation-free entry point's array on this device (once per device)
  if (noalloc_scratch_init(device) != hipSuccess) return HAC_EDEVICE;
  hac_ctx* c = new hac_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes;
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return HAC_EDEVICE;
    }
    c->own_stream = true;
  }
  *out = c;
  return HAC_OK;
}

void hac_destroy(hac_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto e : c->events) (void)hipEventDestroy(e);
  c->arena.release();
  c->scratch.release();
  c->stage.release();
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* hac_last_error(const hac_ctx* c) { return c ? c->err.c_str() : ""; }

hac_status hac_set_timing(hac_ctx* c, int32_t enable) {
  if (!c) return HAC_EINVAL;
  c->timing = enable != 0;
  return HAC_OK;
}

hac_status hac_last_stats(const hac_ctx* c, hac_stats* out) {
  if (!c || !out) return HAC_EINVAL;
  *out = c->stats;
  return HAC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// the batch engine behind hac_decode / hac_decode_batch / hac_decode_dev
// ------------------------------------------------------------------------
namespace {

using Clock = std::chrono::steady_clock;
static double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

#define CTX_HIP(expr)                                                           \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess)                                                       \
      return set_err(c, HAC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// out_dev: per-instance device tour pointers (or null: results to host)
// Host copies of inputs that live in device memory: validation and the
// evidence fold read them on the host.
// Inputs that live in device memory are also needed on the host (the
// validation and the evidence fold read them).  Every array of every
// instance is gathered into one staging buffer by one copy kernel and
// brought back with one copy; hi / hc then point into `blob`.
hac_status mirror_inputs(hac_ctx* c, int32_t count, const hac_instance* insts, const hac_csr* csrs,
                         std::vector<char>& blob, std::vector<hac_instance>& hi, std::vector<hac_csr>& hc) {
  hi.assign(insts, insts + count);
  hc.assign(csrs, csrs + count);
  std::vector<CopyItem> items;
  std::vector<size_t> at;
  size_t total = 0;
  uint64_t maxb = 0;
  auto add = [&](const void* src, size_t bytes) {
    items.push_back(CopyItem{src, nullptr, (uint64_t)bytes});
    at.push_back(total);
    total += align256(bytes);
    maxb = std::max<uint64_t>(maxb, bytes);
    return at.back();
  };
  struct Off {
    size_t geo, rp, col, val;
  };
  std::vector<Off> off(count);
  for (int32_t x = 0; x < count; ++x) {
    const int32_t n = insts[x].n;
    if (n < 1 || n > HAC_MAX_N || csrs[x].n != n || csrs[x].nnz < 0 || !csrs[x].row_ptr)
      return set_err(c, HAC_EINVAL, "instance " + std::to_string(x) + ": bad sizes");
    if (insts[x].kind == HAC_COORDS_EUC2D) {
      if (!insts[x].coords) return set_err(c, HAC_EINVAL, "coords missing");
      off[x].geo = add(insts[x].coords, 16 * (size_t)n);
    } else {
      if (!insts[x].dist) return set_err(c, HAC_EINVAL, "distance matrix missing");
      off[x].geo = add(insts[x].dist, 8 * (size_t)n * n);
    }
    off[x].rp = add(csrs[x].row_ptr, 4 * (size_t)(n + 1));
    off[x].col = off[x].val = 0;
    if (csrs[x].nnz > 0) {
      if (!csrs[x].col || !csrs[x].val) return set_err(c, HAC_EINVAL, "col/val missing");
      off[x].col = add(csrs[x].col, 4 * (size_t)csrs[x].nnz);
      off[x].val = add(csrs[x].val, 4 * (size_t)csrs[x].nnz);
    }
  }
  const size_t data = total;
  const size_t list_at = total;
  total += align256(sizeof(CopyItem) * items.size());
  {
    hipError_t e = c->stage.reserve(total);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return set_err(c, HAC_ENOMEM, "device memory");
    CTX_HIP(e);
  }
  char* d = (char*)c->stage.carve(total);
  for (size_t q = 0; q < items.size(); ++q) items[q].dst = d + at[q];
  hipStream_t s = c->stream;
  CTX_HIP(hipMemcpyAsync(d + list_at, items.data(), sizeof(CopyItem) * items.size(), hipMemcpyHostToDevice, s));
  hipError_t ke = launch_copy_items((const CopyItem*)(d + list_at), (int32_t)items.size(), maxb, s);
  if (ke == hipErrorInvalidValue) {  // an item too large for one launch: copy them one by one
    ke = hipSuccess;
    for (size_t q = 0; q < items.size() && ke == hipSuccess; ++q)
      ke = hipMemcpyAsync(items[q].dst, items[q].src, items[q].bytes, hipMemcpyDeviceToDevice, s);
  }
  CTX_HIP(ke);
  blob.resize(std::max<size_t>(data, 16));
  CTX_HIP(hipMemcpyAsync(blob.data(), d, data, hipMemcpyDeviceToHost, s));
  CTX_HIP(hipStreamSynchronize(s));
  for (int32_t x = 0; x < count; ++x) {
    char* b = blob.data();
    if (insts[x].kind == HAC_COORDS_EUC2D)
      hi[x].coords = (const double*)(b + off[x].geo);
    else
      hi[x].dist = (const double*)(b + off[x].geo);
    hc[x].row_ptr = (const int32_t*)(b + off[x].rp);
    hc[x].col = (const int32_t*)(b + off[x].col);
    hc[x].val = (const float*)(b + off[x].val);
  }
  return HAC_OK;
}

// noalloc: every device buffer comes from the device's static scratch array
// (no hipMalloc, no graph, no events, no tuning launches); only for host
// inputs and outputs
hac_status run_batch(hac_ctx* c, int32_t count, const hac_instance* insts_in, const hac_csr* csrs_in,
                     const hac_params* params, const uint64_t* seeds, int32_t* const* tours_out,
                     double* lengths_out, bool outputs_on_device, bool inputs_on_device,
                     bool noalloc = false) {
  const auto t0 = Clock::now();
  c->err.clear();
  c->stats = hac_stats{};
  if (count < 1 || !insts_in || !csrs_in || !params || !seeds || !tours_out || !lengths_out)
    return set_err(c, HAC_EINVAL, "null or empty batch");
  std::vector<char> mir;
  std::vector<hac_instance> hi;
  std::vector<hac_csr> hc;
  if (inputs_on_device) {
    CTX_HIP(hipSetDevice(c->device));
    hac_status ms = mirror_inputs(c, count, insts_in, csrs_in, mir, hi, hc);
    if (ms != HAC_OK) return ms;
  }
  const hac_instance* insts = inputs_on_device ? hi.data() : insts_in;
  const hac_csr* csrs = inputs_on_device ? hc.data() : csrs_in;
  for (int32_t x = 0; x < count; ++x) {
    std::string why;
    hac_status s = validate(&insts[x], &csrs[x], &params[x], &why);
    if (s != HAC_OK) return set_err(c, s, "instance " + std::to_string(x) + ": " + why);
    if (!tours_out[x]) return set_err(c, HAC_EINVAL, "null tour output");
  }
  CTX_HIP(hipSetDevice(c->device));
  hipStream_t s = c->stream;

  // trivial instances (n = 1) need no search
  std::vector<HostInst> hs;
  std::vector<int32_t> which;
  for (int32_t x = 0; x < count; ++x) {
    if (insts[x].n == 1) continue;
    HostInst h{};
    h.inst = insts[x];
    h.csr = csrs[x];
    h.p = params[x];
    h.seed = seeds[x];
    h.lay = make_layout(&insts[x], &csrs[x], &params[x]);
    h.dstar = degree_target_of(&insts[x], &params[x]);
    h.sym = (insts[x].kind == HAC_COORDS_EUC2D || insts[x].symmetric) ? 1 : 0;
    h.p_x = fold_p_x(params[x].p_best, insts[x].n);
    h.from_device = inputs_on_device;
    if (inputs_on_device) {
      h.dev_inst = insts_in[x];
      h.dev_csr = csrs_in[x];
    }
    hs.push_back(h);
    which.push_back(x);
  }
  const int32_t m = (int32_t)hs.size();
  size_t total = align256(sizeof(InstDesc) * (size_t)std::max(m, 1)) +
                 align256(sizeof(int32_t*) * (size_t)std::max(m, 1)) + align256(8 * (size_t)std::max(m, 1));
  for (auto& h : hs) total += h.lay.bytes() + (outputs_on_device ? 0 : align256(4 * (size_t)h.lay.n));
  if (c->budget && total > c->budget) return set_err(c, HAC_ENOMEM, "batch exceeds the context budget");
  // device memory: the context's arena, or the static scratch array
  char* nb = nullptr;
  size_t nb_used = 0;
  if (noalloc) {
    // the block map follows the slots: at most one block per ant, and a
    // round of eight entries (one per XCD) per block at worst
    size_t ants = 0;
    for (auto& h : hs) ants += (size_t)h.p.ants;
    total += align256(sizeof(BlockMap) * 8 * ants);
    if (total > kNoAllocBytes)
      return set_err(c, HAC_ENOMEM, "the decode needs " + std::to_string(total) + " bytes of device memory; "
                                    "the allocation-free scratch holds " + std::to_string(kNoAllocBytes));
    nb = (char*)noalloc_scratch(c->device);
    if (!nb) return set_err(c, HAC_EDEVICE, "allocation-free scratch not set up on this device");
  } else if (m > 0) {
    hipError_t e = c->arena.reserve(total);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      return set_err(c, HAC_ENOMEM, "device memory");
    CTX_HIP(e);
  }
  auto carve = [&](size_t b) -> void* {
    if (!noalloc) return c->arena.carve(b);
    void* p = nb + nb_used;
    nb_used += align256(b);
    return p;
  };
  InstDesc* d_descs = m ? (InstDesc*)carve(sizeof(InstDesc) * m) : nullptr;
  int32_t** d_out_ptrs = m ? (int32_t**)carve(sizeof(int32_t*) * m) : nullptr;
  double* d_out_lens = m ? (double*)carve(8 * (size_t)m) : nullptr;
  std::vector<int32_t*> out_ptrs(m);
  std::vector<CopyItem> up;  // device-resident inputs, gathered in one launch
  for (int32_t y = 0; y < m; ++y) {
    HostInst& h = hs[y];
    assign_slot(h, carve);
    fill_desc_scalars(h);
    out_ptrs[y] = outputs_on_device ? tours_out[which[y]] : (int32_t*)carve(4 * (size_t)h.lay.n);
    if (h.from_device) {
      // the caller's device arrays, gathered into the slot below
      const Layout& L = h.lay;
      const size_t nn = (size_t)L.n;
      if (L.coords)
        up.push_back(CopyItem{h.dev_inst.coords, (void*)h.d.xy, 16 * nn});
      else
        up.push_back(CopyItem{h.dev_inst.dist, (void*)h.d.dist, 8 * nn * nn});
      up.push_back(CopyItem{h.dev_csr.row_ptr, (void*)h.d.row_ptr, 4 * (nn + 1)});
      if (L.nnz > 0) {
        up.push_back(CopyItem{h.dev_csr.col, (void*)h.d.col, 4 * (size_t)L.nnz});
        up.push_back(CopyItem{h.dev_csr.val, (void*)h.d.val, 4 * (size_t)L.nnz});
      }
    } else {
      CTX_HIP(upload_inputs(h, s));
    }
  }
  if (!up.empty()) {
    uint64_t maxb = 0;
    for (auto& it : up) maxb = std::max<uint64_t>(maxb, it.bytes);
    CTX_HIP(c->stage.reserve(align256(sizeof(CopyItem) * up.size())));
    CopyItem* d_up = (CopyItem*)c->stage.carve(sizeof(CopyItem) * up.size());
    CTX_HIP(hipMemcpyAsync(d_up, up.data(), sizeof(CopyItem) * up.size(), hipMemcpyHostToDevice, s));
    hipError_t ke = launch_copy_items(d_up, (int32_t)up.size(), maxb, s);
    if (ke == hipErrorInvalidValue) {
      ke = hipSuccess;
      for (size_t q = 0; q < up.size() && ke == hipSuccess; ++q)
        ke = hipMemcpyAsync(up[q].dst, up[q].src, up[q].bytes, hipMemcpyDeviceToDevice, s);
    }
    CTX_HIP(ke);
  }
  if (m > 0) {
    std::vector<InstDesc> descs(m);
    for (int32_t y = 0; y < m; ++y) descs[y] = hs[y].d;
    CTX_HIP(hipMemcpyAsync(d_descs, descs.data(), sizeof(InstDesc) * m, hipMemcpyHostToDevice, s));
    CTX_HIP(hipMemcpyAsync(d_out_ptrs, out_ptrs.data(), sizeof(int32_t*) * m, hipMemcpyHostToDevice, s));
    std::string err;
    hac_status ps = prepare_instances(hs, d_descs, s, &err, noalloc ? nullptr : &c->stage);
    if (ps != HAC_OK) return set_err(c, ps, err);
  }
  const double prep_ms = ms_since(t0);
  const auto t1 = Clock::now();

  double construct_ms = 0.0, ls_ms = 0.0, update_ms = 0.0;
  int64_t launches = 0, ls_launches = 0, update_launches = 0;
  LaunchShape used{0, 0, 0, 0, 0};
  if (m > 0) {
    bool any_ls = false;
    // max_n: the largest symmetric instance with 2-opt (0: none); max_n_dir: ATSP
    int32_t max_iter = 0, max_n = 0, all_coords = 1, ls_tours = 1, max_n_dir = 0, max_kls_dir = 0, max_n3 = 0, all_coords3 = 1;
    for (auto& h : hs) {
      any_ls |= h.p.local_search != 0;
      if (h.p.local_search == 2) ls_tours = std::max(ls_tours, h.p.ants);
      max_iter = std::max(max_iter, h.p.iterations);
      if (h.lay.directed) max_n_dir = std::max(max_n_dir, h.lay.n), max_kls_dir = std::max(max_kls_dir, h.lay.kls);
      else if (h.lay.three_opt) max_n3 = std::max(max_n3, h.lay.n);
      else if (h.p.local_search) max_n = std::max(max_n, h.lay.n);
      if (h.p.local_search && !h.lay.directed && !h.lay.three_opt && !h.lay.coords) all_coords = 0;
      if (h.lay.three_opt && !h.lay.coords) all_coords3 = 0;
    }
    LaunchShape shape{4, 0, 16, 4, 0};
    if (noalloc) {
      shape = default_shape(hs);
    } else if (max_iter > 0) {
      bool ok = true;
      shape = tune_shape(hs, d_descs, s, c->scratch, &ok);
      if (!ok) return set_err(c, HAC_EDEVICE, "autotuner launch failed");
      CTX_HIP(launch_init(d_descs, m, s));  // undo the tuner's fallback counts
    }
    if (const char* f = std::getenv("HAC_FORCE_DEVICE_ERROR")) {
      // test hook: flags instance f's error word as a failing kernel check
      // would, so that the error path can be exercised without one
      const int32_t x = std::atoi(f);
      if (x >= 0 && x < m) CTX_HIP(hipMemsetAsync(&hs[x].d.st->err, 0xff, sizeof(uint32_t), s));
    }
    used = shape;
    std::vector<BlockMap> map = build_block_map(hs, shape.ants_per_block);
    BlockMap* d_map;
    if (noalloc) {
      size_t ants = 0;
      for (auto& h : hs) ants += (size_t)h.p.ants;
      if (map.size() > 8 * ants) return set_err(c, HAC_EDEVICE, "block map larger than its reserve");
      d_map = (BlockMap*)carve(map.size() * sizeof(BlockMap));
    } else {
      c->scratch.reset();
      CTX_HIP(c->scratch.reserve(map.size() * sizeof(BlockMap)));
      d_map = (BlockMap*)c->scratch.carve(map.size() * sizeof(BlockMap));
    }
    CTX_HIP(hipMemcpyAsync(d_map, map.data(), map.size() * sizeof(BlockMap), hipMemcpyHostToDevice, s));
    const size_t lds = shape_lds(hs, shape);
    const int32_t blocks = (int32_t)map.size();
    auto one_iteration = [&]() -> hipError_t {
      hipError_t e = launch_construct(d_descs, d_map, blocks, shape.ants_per_block, shape.rows_per_wave, shape.staged,
                                      shape.bytes, shape.kmax, lds, shape.geo, shape.grid, s);
      if (e != hipSuccess) return e;
      if (any_ls) {
        e = launch_local_search(d_descs, m, max_n, all_coords, ls_tours, max_n_dir, max_kls_dir, max_n3, all_coords3, s);
        if (e != hipSuccess) return e;
      }
      return launch_iter_end(d_descs, m, s);
    };
    if (noalloc) {
      // plain launches: no graph, no events
      for (int32_t it = 0; it < max_iter; ++it) CTX_HIP(one_iteration());
      CTX_HIP(hipStreamSynchronize(s));
      launches = max_iter;
    } else if (c->timing) {
      // per-iteration launches with HIP events around each kernel: e[4 it]
      // .. e[4 it + 3] bracket construction, 2-opt and the update
      while ((int)c->events.size() < 4 * max_iter) {
        hipEvent_t e;
        CTX_HIP(hipEventCreate(&e));
        c->events.push_back(e);
      }
      for (int32_t it = 0; it < max_iter; ++it) {
        hipEvent_t* ev = &c->events[4 * it];
        CTX_HIP(hipEventRecord(ev[0], s));
        CTX_HIP(launch_construct(d_descs, d_map, blocks, shape.ants_per_block, shape.rows_per_wave, shape.staged,
                                      shape.bytes, shape.kmax, lds, shape.geo, shape.grid, s));
        CTX_HIP(hipEventRecord(ev[1], s));
        if (any_ls) CTX_HIP(launch_local_search(d_descs, m, max_n, all_coords, ls_tours, max_n_dir, max_kls_dir, max_n3, all_coords3, s));
        CTX_HIP(hipEventRecord(ev[2], s));
        CTX_HIP(launch_iter_end(d_descs, m, s));
        CTX_HIP(hipEventRecord(ev[3], s));
      }
      CTX_HIP(hipStreamSynchronize(s));
      for (int32_t it = 0; it < max_iter; ++it) {
        hipEvent_t* ev = &c->events[4 * it];
        float ms = 0;
        CTX_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        construct_ms += ms;
        if (any_ls) {
          CTX_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
          ls_ms += ms;
        }
        CTX_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
        update_ms += ms;
      }
      launches = max_iter;
      ls_launches = any_ls ? max_iter : 0;
      update_launches = max_iter;
    } else if (max_iter > 0) {
      // a graph of G iterations replayed; surplus iterations are no-ops
      const int32_t G = std::min<int32_t>(max_iter, 16);
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      CTX_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      hipError_t ce = hipSuccess;
      for (int32_t g = 0; g < G && ce == hipSuccess; ++g) ce = one_iteration();
      hipError_t ee = hipStreamEndCapture(s, &graph);
      if (ce != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return set_err(c, HAC_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce != hipSuccess ? ce : ee));
      }
      hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) return set_err(c, HAC_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
      const int32_t reps = (max_iter + G - 1) / G;
      hipError_t le = hipSuccess;
      for (int32_t r = 0; r < reps && le == hipSuccess; ++r) le = hipGraphLaunch(exec, s);
      hipError_t se = hipStreamSynchronize(s);
      (void)hipGraphExecDestroy(exec);
      if (le != hipSuccess || se != hipSuccess)
        return set_err(c, HAC_EDEVICE, std::string("graph replay: ") + hipGetErrorString(le != hipSuccess ? le : se));
      launches = (int64_t)reps * G;
    }
    CTX_HIP(launch_finish(d_descs, m, d_out_ptrs, d_out_lens, s));
  }
  // results
  std::vector<double> lens(m);
  std::vector<State> sts(m);
  if (m > 0) {
    CTX_HIP(hipMemcpyAsync(lens.data(), d_out_lens, 8 * (size_t)m, hipMemcpyDeviceToHost, s));
    // the final states, gathered into one readback
    std::vector<CopyItem> items;
    std::vector<size_t> at;
    for (int32_t y = 0; y < m; ++y) {
      items.push_back(CopyItem{hs[y].d.st, nullptr, sizeof(State)});
      at.push_back((size_t)y * align256(sizeof(State)));
    }
    std::vector<char> blob((size_t)m * align256(sizeof(State)));
    if (noalloc) {
      for (int32_t y = 0; y < m; ++y)
        CTX_HIP(hipMemcpyAsync(blob.data() + at[y], hs[y].d.st, sizeof(State), hipMemcpyDeviceToHost, s));
    } else {
      CTX_HIP(stage_copies(c->stage, items, at, blob.data(), blob.size(), true, s));
    }
    CTX_HIP(hipStreamSynchronize(s));
    for (int32_t y = 0; y < m; ++y) std::memcpy(&sts[y], blob.data() + at[y], sizeof(State));
    for (int32_t y = 0; y < m; ++y)
      if (sts[y].err || std::isnan(lens[y]))
        return set_err(c, HAC_EDEVICE, "instance " + std::to_string(which[y]) +
                                           ": an ant's tour failed its permutation check on the device "
                                           "(a construction step broke its pick contract)");
    if (!outputs_on_device)
      for (int32_t y = 0; y < m; ++y)
        CTX_HIP(hipMemcpyAsync(tours_out[which[y]], out_ptrs[y], 4 * (size_t)hs[y].lay.n,
                               hipMemcpyDeviceToHost, s));
    CTX_HIP(hipStreamSynchronize(s));
  }
  for (int32_t x = 0, y = 0; x < count; ++x) {
    if (insts[x].n == 1) {
      if (outputs_on_device) {
        const int32_t zero = 0;
        const double zl = 0.0;
        CTX_HIP(hipMemcpy(tours_out[x], &zero, 4, hipMemcpyHostToDevice));
        CTX_HIP(hipMemcpy(&lengths_out[x], &zl, 8, hipMemcpyHostToDevice));
      } else {
        tours_out[x][0] = 0;
        lengths_out[x] = 0.0;
      }
      continue;
    }
    if (outputs_on_device)
      CTX_HIP(hipMemcpy(&lengths_out[x], &lens[y], 8, hipMemcpyHostToDevice));
    else
      lengths_out[x] = lens[y];
    ++y;
  }
  hac_stats& st = c->stats;
  st.instances = count;
  st.prep_ms = prep_ms;
  st.search_ms = ms_since(t1);
  st.total_ms = ms_since(t0);
  st.construct_ms = construct_ms;
  st.construct_launches = launches;
  st.local_search_ms = ls_ms;
  st.local_search_launches = ls_launches;
  st.update_ms = update_ms;
  st.update_launches = update_launches;
  st.ants_per_block = used.ants_per_block;
  st.lds_staged = used.staged;
  st.ants_per_wave = used.rows_per_wave;
  st.byte_marks = used.bytes;
  st.geo_mode = used.geo;
  for (int32_t y = 0; y < m; ++y) {
    st.ant_steps += (int64_t)hs[y].p.ants * (hs[y].lay.n - 1) * hs[y].p.iterations;
    st.fallback_steps += (int64_t)sts[y].fallbacks;
    st.restarts += sts[y].restarts;
  }
  if (m > 0) {
    st.kappa = hs[0].fold.kappa;
    st.q90 = hs[0].fold.q90;
    st.r_hat = hs[0].fold.r_hat;
    st.l_nn = hs[0].l_nn;
  }
  c->last = hs;
  for (auto& h : c->last) h.cand_h.clear();
  return HAC_OK;
}

}  // namespace

extern "C" {

hac_status hac_decode(hac_ctx* c, const hac_instance* inst, const hac_csr* heat, const hac_params* p,
                      uint64_t seed, int32_t* tour_out, double* length_out) {
  if (!c) return HAC_EINVAL;
  int32_t* tours[1] = {tour_out};
  return run_batch(c, 1, inst, heat, p, &seed, tours, length_out, false, false);
}

hac_status hac_decode_noalloc(hac_ctx* c, const hac_instance* inst, const hac_csr* heat, const hac_params* p,
                              uint64_t seed, int32_t* tour_out, double* length_out) {
  if (!c) return HAC_EINVAL;
  std::mutex* lock = noalloc_call_lock(c->device);
  if (!lock) return HAC_EINVAL;
  std::lock_guard<std::mutex> g(*lock);
  int32_t* tours[1] = {tour_out};
  return run_batch(c, 1, inst, heat, p, &seed, tours, length_out, false, false, true);
}

hac_status hac_decode_batch(hac_ctx* c, int32_t count, const hac_instance* insts, const hac_csr* heats,
                            const hac_params* params, const uint64_t* seeds, int32_t* const* tours_out,
                            double* lengths_out) {
  if (!c) return HAC_EINVAL;
  return run_batch(c, count, insts, heats, params, seeds, tours_out, lengths_out, false, false);
}

hac_status hac_decode_batch_dev(hac_ctx* c, int32_t count, const hac_instance* insts_dev,
                                const hac_csr* heats_dev, const hac_params* params, const uint64_t* seeds,
                                int32_t* const* tours_out_dev, double* lengths_out_dev) {
  if (!c) return HAC_EINVAL;
  return run_batch(c, count, insts_dev, heats_dev, params, seeds, tours_out_dev, lengths_out_dev, true,
                   true);
}

hac_status hac_decode_dev(hac_ctx* c, const hac_instance* inst_dev, const hac_csr* heat_dev,
                          const hac_params* p, uint64_t seed, int32_t* tour_out_dev,
                          double* length_out_dev) {
  if (!c) return HAC_EINVAL;
  int32_t* tours[1] = {tour_out_dev};
  return run_batch(c, 1, inst_dev, heat_dev, p, &seed, tours, length_out_dev, true, true);
}

hac_status hac_debug_state(hac_ctx* c, int32_t which, int32_t* cand, float* heur, float* tau,
                           float* weight, int32_t* ant_tours, double* ant_len, int32_t* nn_tour) {
  if (!c || which < 0 || which >= (int32_t)c->last.size()) return HAC_EINVAL;
  const HostInst& h = c->last[which];
  const size_t nn = (size_t)h.lay.n, nk = nn * h.lay.k;
  hipStream_t s = c->stream;
  if (cand) CTX_HIP(hipMemcpyAsync(cand, h.d.cand, 4 * nk, hipMemcpyDeviceToHost, s));
  if (heur) CTX_HIP(hipMemcpyAsync(heur, h.d.heur, 4 * nk, hipMemcpyDeviceToHost, s));
  if (tau) CTX_HIP(hipMemcpyAsync(tau, h.d.tau, 4 * nk, hipMemcpyDeviceToHost, s));
  if (weight) CTX_HIP(hipMemcpyAsync(weight, h.d.w, 4 * nk, hipMemcpyDeviceToHost, s));
  if (ant_tours) CTX_HIP(hipMemcpyAsync(ant_tours, h.d.tours, 4 * nn * h.p.ants, hipMemcpyDeviceToHost, s));
  if (ant_len) CTX_HIP(hipMemcpyAsync(ant_len, h.d.lens, 8 * (size_t)h.p.ants, hipMemcpyDeviceToHost, s));
  if (nn_tour) CTX_HIP(hipMemcpyAsync(nn_tour, h.d.nn_tour, 4 * nn, hipMemcpyDeviceToHost, s));
  CTX_HIP(hipStreamSynchronize(s));
  return HAC_OK;
}

hac_status hac_heatmap_diagnostics(hac_ctx* c, const hac_instance* inst, const hac_csr* heat,
                                   const hac_params* p, const int32_t* known_tour, hac_diagnostics* out) {
  if (!c) return HAC_EINVAL;
  c->err.clear();
  if (!inst || !heat || !p || !known_tour || !out) return set_err(c, HAC_EINVAL, "null argument");
  std::string why;
  const hac_status vs = validate(inst, heat, p, &why);
  if (vs != HAC_OK) return set_err(c, vs, why);
  const int32_t n = inst->n;
  if (n < 2) return set_err(c, HAC_EINVAL, "diagnostics need n >= 2");
  std::vector<int32_t> succ(n), pred(n);
  std::vector<char> seen(n, 0);
  for (int32_t s = 0; s < n; ++s) {
    const int32_t a = known_tour[s];
    if (a < 0 || a >= n || seen[a]) return set_err(c, HAC_EINVAL, "known tour is not a permutation");
    seen[a] = 1;
  }
  for (int32_t s = 0; s < n; ++s) {
    succ[known_tour[s]] = known_tour[(s + 1) % n];
    pred[known_tour[s]] = known_tour[(s + n - 1) % n];
  }
  // the candidate lists and evidence of a decode with these parameters
  CTX_HIP(hipSetDevice(c->device));
  hipStream_t s = c->stream;
  hac_params q = *p;
  q.iterations = 0;
  HostInst h{};
  h.inst = *inst;
  h.csr = *heat;
  h.p = q;
  h.seed = 0;
  h.lay = make_layout(inst, heat, &q);
  h.dstar = degree_target_of(inst, &q);
  h.sym = (inst->kind == HAC_COORDS_EUC2D || inst->symmetric) ? 1 : 0;
  h.p_x = fold_p_x(q.p_best, n);
  h.want_evid = true;
  const size_t total = align256(sizeof(InstDesc)) + h.lay.bytes();
  if (c->budget && total > c->budget) return set_err(c, HAC_ENOMEM, "instance exceeds the context budget");
  {
    hipError_t e = c->arena.reserve(total);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return set_err(c, HAC_ENOMEM, "device memory");
    CTX_HIP(e);
  }
  InstDesc* d_descs = (InstDesc*)c->arena.carve(sizeof(InstDesc));
  assign_slot(h, [&](size_t b) { return c->arena.carve(b); });
  fill_desc_scalars(h);
  CTX_HIP(upload_inputs(h, s));
  CTX_HIP(hipMemcpyAsync(d_descs, &h.d, sizeof(InstDesc), hipMemcpyHostToDevice, s));
  std::vector<HostInst> hs{h};
  std::string err;
  const hac_status ps = prepare_instances(hs, d_descs, s, &err);
  if (ps != HAC_OK) return set_err(c, ps, err);
  CTX_HIP(hipStreamSynchronize(s));
  const HostInst& g = hs[0];
  // Edges/n and coverage, from the heatmap as given
  int64_t entries = 0, covered = 0;
  std::vector<char> has_out(n, 0), has_in(n, 0);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t e = heat->row_ptr[i]; e < heat->row_ptr[i + 1]; ++e) {
      const int32_t j = heat->col[e];
      if (j == i || !((double)heat->val[e] > q.theta_h)) continue;
      ++entries;
      if (j == succ[i]) has_out[i] = 1;
      if (j == pred[i]) has_in[j] = 1;  // the reverse of tour edge (j, i)
    }
  for (int32_t a = 0; a < n; ++a)
    if (has_out[a] || (g.sym && has_in[a])) ++covered;
  // P(e > 1) over the candidate slots
  int64_t strong = 0, on_tour = 0;
  const int32_t k = g.lay.k;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t u = 0; u < k; ++u) {
      const size_t x = (size_t)i * k + u;
      if (!g.evid_gt1[x]) continue;
      ++strong;
      const int32_t j = g.cand_h[x];
      if (j == succ[i] || (g.sym && j == pred[i])) ++on_tour;
    }
  out->edges_per_node = (double)entries / (2.0 * (double)n);
  out->coverage = (double)covered / (double)n;
  out->miss_pct = 100.0 * (1.0 - out->coverage);
  out->p_evidence = strong > 0 ? (double)on_tour / (double)strong : 0.0;
  out->heatmap_edges = entries;
  out->evidence_slots = strong;
  out->evidence_on_tour = on_tour;
  return HAC_OK;
}

hac_status hac_debug_trace(hac_ctx* c, int32_t which, double* l_ib, double* l_gb, int32_t* elite_rb) {
  if (!c || which < 0 || which >= (int32_t)c->last.size()) return HAC_EINVAL;
  const HostInst& h = c->last[which];
  const size_t it = (size_t)h.p.iterations;
  hipStream_t s = c->stream;
  if (it == 0) return HAC_OK;
  if (l_ib) CTX_HIP(hipMemcpyAsync(l_ib, h.d.tr_lib, 8 * it, hipMemcpyDeviceToHost, s));
  if (l_gb) CTX_HIP(hipMemcpyAsync(l_gb, h.d.tr_lgb, 8 * it, hipMemcpyDeviceToHost, s));
  if (elite_rb) CTX_HIP(hipMemcpyAsync(elite_rb, h.d.tr_elite, 4 * it, hipMemcpyDeviceToHost, s));
  CTX_HIP(hipStreamSynchronize(s));
  return HAC_OK;
}

}  // extern "C"
