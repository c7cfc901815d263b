// Continuous-batching request loop.
//
// The server owns a device memory pool of `budget` bytes and admits at most
// `max_slots` instances at a time.  Requests are split into three size
// classes by n (lanes: below 768, below 4096, and larger); each lane has
// its own loop thread and HIP stream, so the iterations of one class do not
// pace another's: their kernels run concurrently on the device.  Streams
// that share a hardware queue run one after the other, and HIP gives a
// process four queues by default, which the null stream and any other
// context also draw on; so the first lane runs on the context's own stream
// and only two streams are added.
// Slots go to requests in arrival order across the lanes: a lane admits a
// request only while the free slots exceed the requests of other lanes
// queued before it, so that a lane whose rounds are short does not take
// every slot a long-running lane frees.  Between rounds of iterations a lane
// admits queued requests of its class whose footprint fits a free block of
// the shared pool (first fit, in arrival order), prepares them on the device,
// and then advances every instance it holds together: each round launches
// the construction, local-search and end-of-iteration kernels once per
// iteration over the lane's admitted set.  An instance whose iterations are
// done is retired: its best tour is copied out, its pool block freed, its
// waiters woken.  Instances never leave the device between admission and
// retirement.  Every instance runs exactly the kernels and per-instance
// state of the plain path, so a served result equals hac_decode's bit for
// bit.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hac_runtime.h"

namespace hac {
namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over one device block, with coalescing on free.
class Pool {
 public:
  hipError_t init(size_t bytes) {
    cap_ = bytes;
    hipError_t e = hipMalloc((void**)&base_, bytes);
    if (e != hipSuccess) {
      base_ = nullptr;
      return e;
    }
    free_.clear();
    free_[0] = bytes;
    return hipSuccess;
  }
  ~Pool() {
    if (base_) (void)hipFree(base_);
  }
  // offset or -1
  int64_t alloc(size_t bytes) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return (int64_t)off;
      }
    }
    return -1;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  char* base() const { return base_; }
  size_t peak() const { return peak_; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

enum ReqState { QUEUED, RUNNING, DONE, CANCELLED, FAILED };

struct Request {
  uint64_t ticket = 0;
  int lane = 0;
  std::vector<double> coords, dist;
  std::vector<int32_t> row_ptr, col;
  std::vector<float> val;
  hac_instance inst{};
  hac_csr csr{};
  hac_params p{};
  uint64_t seed = 0;
  uint64_t bytes = 0;
  Clock::time_point t_submit, t_done;
  ReqState state = QUEUED;
  bool cancel = false;
  hac_status status = HAC_OK;
  std::vector<int32_t> tour;
  double length = 0.0;
};

struct Slot {
  std::shared_ptr<Request> req;
  HostInst h;
  int64_t off = -1;
  int32_t* d_tour = nullptr;  // output area in the slot
  int32_t done_iters = 0;
};

}  // namespace
}  // namespace hac

using namespace hac;

// One size class of requests with its own loop thread and stream.
struct Lane {
  int id = 0;
  hipStream_t stream = nullptr;
  DeviceArena meta, mapa, scratch;  // descriptor arrays, block map, tuner scratch
  std::vector<Slot> active;
  std::thread loop;
  hac_lane_stats st{};  // guarded by the server's mutex
};

// lane l takes the requests with kLaneBound[l - 1] <= n < kLaneBound[l]
static constexpr int kLanes = HAC_SERVER_LANES;
static constexpr int32_t kLaneBound[kLanes - 1] = {768, 4096};

static int lane_of(int32_t n) {
  int l = 0;
  while (l < kLanes - 1 && n >= kLaneBound[l]) ++l;
  return l;
}

struct hac_server {
  hac_ctx* ctx = nullptr;
  int device = 0;
  uint64_t budget = 0;
  int32_t max_slots = 0;
  Pool pool;
  Lane lanes[kLanes];
  std::mutex mu;
  std::condition_variable cv_done, cv_loop;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> reqs;
  int32_t active_total = 0;
  uint64_t gen = 0;  // bumped on every submission, release and cancel
  bool stop = false;
  uint64_t next_ticket = 1;
  int64_t admitted = 0, completed = 0;
  int32_t peak_slots = 0;
};

namespace {

uint64_t footprint_of(const hac_instance* inst, const hac_csr* csr, const hac_params* p) {
  Layout L = make_layout(inst, csr, p);
  return L.bytes() + align256(4 * (size_t)inst->n) + 256;
}

void finish_request(hac_server* S, const std::shared_ptr<Request>& r, ReqState st, hac_status code) {
  r->state = st;
  r->status = code;
  r->t_done = Clock::now();
  S->completed += (st == DONE);
}

// Marks every instance of a lane failed after a device error.
void fail_active(hac_server* S, Lane& LN, hac_status code) {
  std::lock_guard<std::mutex> g(S->mu);
  for (auto& s : LN.active) {
    finish_request(S, s.req, FAILED, code);
    S->pool.release((size_t)s.off, s.req->bytes);
  }
  S->active_total -= (int32_t)LN.active.size();
  LN.active.clear();
  S->gen++;
  S->cv_done.notify_all();
  S->cv_loop.notify_all();
}

// A failed HIP call fails the lane's requests with HAC_EDEVICE; the call
// that failed is not reported further.
bool hip_ok(hac_server* S, hipError_t e, const char* what) {
  (void)S;
  (void)what;
  return e == hipSuccess;
}

void serve_lane(hac_server* S, Lane* lane_ptr) {
  Lane& LN = *lane_ptr;
  (void)hipSetDevice(S->device);
  hipStream_t s = LN.stream;
  std::vector<BlockMap> map;
  bool dirty = true;
  LaunchShape shape{4, 0, 16, 4, 0};
  InstDesc* d_descs = nullptr;
  int32_t** d_outs = nullptr;
  double* d_lens = nullptr;
  BlockMap* d_map = nullptr;
  std::vector<double> lens;

  auto ms_since = [](Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  };
  for (;;) {
    // ---- admission ----
    std::vector<Slot> fresh;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      bool quit = false;
      for (;;) {
        if (S->stop && LN.active.empty()) {
          quit = true;
          break;
        }
        int32_t ahead = 0;  // other lanes' requests queued before this one
        for (auto it = S->queue.begin(); it != S->queue.end();) {
          auto& r = *it;
          if (r->lane != LN.id) {
            ahead += !r->cancel;
            ++it;
            continue;
          }
          if (r->cancel) {
            finish_request(S, r, CANCELLED, HAC_ECANCELLED);
            it = S->queue.erase(it);
            S->gen++;
            S->cv_done.notify_all();
            continue;
          }
          if (S->active_total + (int32_t)fresh.size() + ahead >= S->max_slots || S->stop) break;
          int64_t off = S->pool.alloc(r->bytes);
          if (off < 0) {
            ++it;
            continue;
          }
          Slot sl;
          sl.req = r;
          sl.off = off;
          r->state = RUNNING;
          fresh.push_back(std::move(sl));
          S->admitted++;
          it = S->queue.erase(it);
        }
        if (!fresh.empty() || !LN.active.empty()) break;
        // nothing to run: sleep until a submission, release or stop
        const uint64_t seen = S->gen;
        const Clock::time_point t_idle = Clock::now();
        S->cv_loop.wait(lk, [&] { return S->stop || S->gen != seen; });
        LN.st.idle_ms += ms_since(t_idle);
      }
      if (quit) break;
      S->active_total += (int32_t)fresh.size();
      LN.st.admitted += (int64_t)fresh.size();
    }
    const Clock::time_point t_prep = Clock::now();
    // ---- preparation of the newly admitted instances ----
    if (!fresh.empty()) {
      std::vector<HostInst> hs(fresh.size());
      for (size_t x = 0; x < fresh.size(); ++x) {
        Slot& sl = fresh[x];
        Request& r = *sl.req;
        HostInst& h = hs[x];
        h.inst = r.inst;
        h.csr = r.csr;
        h.p = r.p;
        h.seed = r.seed;
        h.lay = make_layout(&r.inst, &r.csr, &r.p);
        h.dstar = degree_target_of(&r.inst, &r.p);
        h.sym = (r.inst.kind == HAC_COORDS_EUC2D || r.inst.symmetric) ? 1 : 0;
        h.p_x = fold_p_x(r.p.p_best, r.inst.n);
        char* base = S->pool.base() + sl.off;
        size_t used = 0;
        auto carve = [&](size_t b) {
          void* ptr = base + used;
          used += align256(b);
          return ptr;
        };
        assign_slot(h, carve);
        sl.d_tour = (int32_t*)carve(4 * (size_t)r.inst.n);
        fill_desc_scalars(h);
      }
      bool ok = true;
      LN.scratch.reset();
      ok = hip_ok(S, LN.scratch.reserve(align256(sizeof(InstDesc) * hs.size())), "scratch");
      InstDesc* d_new = ok ? (InstDesc*)LN.scratch.carve(sizeof(InstDesc) * hs.size()) : nullptr;
      for (size_t x = 0; ok && x < hs.size(); ++x) ok = hip_ok(S, upload_inputs(hs[x], s), "upload");
      if (ok) {
        std::vector<InstDesc> dd(hs.size());
        for (size_t x = 0; x < hs.size(); ++x) dd[x] = hs[x].d;
        ok = hip_ok(S, hipMemcpyAsync(d_new, dd.data(), sizeof(InstDesc) * dd.size(),
                                      hipMemcpyHostToDevice, s), "descs");
      }
      hac_status ps = HAC_OK;
      if (ok) {
        std::string why;
        ps = prepare_instances(hs, d_new, s, &why);
      }
      std::lock_guard<std::mutex> g(S->mu);
      for (size_t x = 0; x < fresh.size(); ++x) {
        if (!ok || ps != HAC_OK) {
          finish_request(S, fresh[x].req, FAILED, ok ? ps : HAC_EDEVICE);
          S->pool.release((size_t)fresh[x].off, fresh[x].req->bytes);
          S->active_total -= 1;
          S->gen++;
          continue;
        }
        fresh[x].h = hs[x];
        fresh[x].h.cand_h.clear();
        LN.active.push_back(std::move(fresh[x]));
        dirty = true;
      }
      S->peak_slots = std::max(S->peak_slots, S->active_total);
      LN.st.peak_active = std::max(LN.st.peak_active, (int32_t)LN.active.size());
      LN.st.prep_ms += ms_since(t_prep);
      if (!ok || ps != HAC_OK) {
        S->cv_done.notify_all();
        S->cv_loop.notify_all();
      }
    }
    if (LN.active.empty()) continue;
    const Clock::time_point t_round = Clock::now();

    // ---- a round of iterations over the admitted set ----
    const int32_t m = (int32_t)LN.active.size();
    std::vector<HostInst> hs;
    hs.reserve(m);
    for (auto& sl : LN.active) hs.push_back(sl.h);
    if (dirty) {
      // descriptors first: the tuner times real construction launches
      bool ok = hip_ok(S, LN.meta.reserve(align256(sizeof(InstDesc) * m) + align256(sizeof(int32_t*) * m) +
                                          align256(8 * (size_t)m)), "meta");
      if (ok) {
        d_descs = (InstDesc*)LN.meta.carve(sizeof(InstDesc) * m);
        d_outs = (int32_t**)LN.meta.carve(sizeof(int32_t*) * m);
        d_lens = (double*)LN.meta.carve(8 * (size_t)m);
        std::vector<InstDesc> dd(m);
        std::vector<int32_t*> outs(m);
        for (int32_t x = 0; x < m; ++x) {
          dd[x] = LN.active[x].h.d;
          outs[x] = LN.active[x].d_tour;
        }
        ok = hip_ok(S, hipMemcpyAsync(d_descs, dd.data(), sizeof(InstDesc) * m, hipMemcpyHostToDevice, s), "descs") &&
             hip_ok(S, hipMemcpyAsync(d_outs, outs.data(), sizeof(int32_t*) * m, hipMemcpyHostToDevice, s), "outs");
      }
      if (ok) {
        // construction only reads the search state, so timing it here
        // leaves every instance's trajectory unchanged
        shape = tune_shape(hs, d_descs, s, LN.scratch, &ok, true);
      }
      if (ok) {
        map = build_block_map(hs, shape.ants_per_block);
        ok = hip_ok(S, LN.mapa.reserve(sizeof(BlockMap) * map.size()), "map");
        if (ok) {
          d_map = (BlockMap*)LN.mapa.carve(sizeof(BlockMap) * map.size());
          ok = hip_ok(S, hipMemcpyAsync(d_map, map.data(), sizeof(BlockMap) * map.size(), hipMemcpyHostToDevice, s), "map");
        }
      }
      if (!ok) {
        fail_active(S, LN, HAC_EDEVICE);
        continue;
      }
      dirty = false;
    }
    // max_n: the largest symmetric instance with 2-opt (0: none); max_n_dir: ATSP
    int32_t remaining = 1 << 30, max_n = 0, all_coords = 1, ls_tours = 1, max_n_dir = 0, max_kls_dir = 0, max_n3 = 0, all_coords3 = 1;
    bool any_ls = false;
    for (auto& sl : LN.active) {
      remaining = std::min(remaining, sl.h.p.iterations - sl.done_iters);
      any_ls |= sl.h.p.local_search != 0;
      if (sl.h.p.local_search == 2) ls_tours = std::max(ls_tours, sl.h.p.ants);
      if (sl.h.lay.directed) max_n_dir = std::max(max_n_dir, sl.h.lay.n), max_kls_dir = std::max(max_kls_dir, sl.h.lay.kls);
      else if (sl.h.lay.three_opt) max_n3 = std::max(max_n3, sl.h.lay.n);
      else if (sl.h.p.local_search) max_n = std::max(max_n, sl.h.lay.n);
      if (sl.h.p.local_search && !sl.h.lay.directed && !sl.h.lay.three_opt && !sl.h.lay.coords) all_coords = 0;
      if (sl.h.lay.three_opt && !sl.h.lay.coords) all_coords3 = 0;
    }
    bool queued = false;
    {
      std::lock_guard<std::mutex> g(S->mu);
      for (auto& r : S->queue) queued |= r->lane == LN.id;
    }
    // short rounds while requests wait, so they join soon
    const int32_t rounds = std::max(0, std::min(remaining, queued ? 2 : 8));
    const size_t lds = shape_lds(hs, shape);
    bool ok = true;
    for (int32_t r = 0; ok && r < rounds; ++r) {
      ok = hip_ok(S, launch_construct(d_descs, d_map, (int32_t)map.size(), shape.ants_per_block,
                                      shape.rows_per_wave, shape.staged, shape.bytes, shape.kmax, lds,
                                      shape.geo, shape.grid, s), "construct");
      if (ok && any_ls) ok = hip_ok(S, launch_local_search(d_descs, m, max_n, all_coords, ls_tours, max_n_dir, max_kls_dir, max_n3, all_coords3, s), "local search");
      if (ok) ok = hip_ok(S, launch_iter_end(d_descs, m, s), "iter end");
    }
    if (ok) ok = hip_ok(S, launch_finish(d_descs, m, d_outs, d_lens, s), "finish");
    lens.resize(m);
    if (ok) ok = hip_ok(S, hipMemcpyAsync(lens.data(), d_lens, 8 * (size_t)m, hipMemcpyDeviceToHost, s), "lens");
    std::vector<int32_t> finished;
    for (int32_t x = 0; x < m; ++x) {
      LN.active[x].done_iters += rounds;
      if (LN.active[x].done_iters >= LN.active[x].h.p.iterations) finished.push_back(x);
    }
    for (int32_t x : finished) {
      Slot& sl = LN.active[x];
      sl.req->tour.resize(sl.h.lay.n);
      if (ok)
        ok = hip_ok(S, hipMemcpyAsync(sl.req->tour.data(), sl.d_tour, 4 * (size_t)sl.h.lay.n,
                                      hipMemcpyDeviceToHost, s), "tour");
    }
    if (ok) ok = hip_ok(S, hipStreamSynchronize(s), "sync");
    if (!ok) {
      fail_active(S, LN, HAC_EDEVICE);
      continue;
    }
    // ---- retirement ----
    std::lock_guard<std::mutex> g(S->mu);
    LN.st.round_ms += ms_since(t_round);
    LN.st.rounds += 1;
    LN.st.iterations += rounds;
    LN.st.instance_iterations += (int64_t)rounds * m;
    std::vector<Slot> keep;
    for (int32_t x = 0; x < m; ++x) {
      Slot& sl = LN.active[x];
      const bool fin = std::find(finished.begin(), finished.end(), x) != finished.end();
      if (fin || sl.req->cancel || S->stop) {
        if (fin && !sl.req->cancel && std::isnan(lens[x])) {
          // the instance stopped on a broken kernel contract (no tour written)
          finish_request(S, sl.req, FAILED, HAC_EDEVICE);
        } else if (fin && !sl.req->cancel) {
          sl.req->length = lens[x];
          finish_request(S, sl.req, DONE, HAC_OK);
          LN.st.completed += 1;
        } else {
          finish_request(S, sl.req, CANCELLED, HAC_ECANCELLED);
        }
        S->pool.release((size_t)sl.off, sl.req->bytes);
        S->active_total -= 1;
        S->gen++;
        dirty = true;
      } else {
        keep.push_back(std::move(sl));
      }
    }
    LN.active.swap(keep);
    S->cv_done.notify_all();
    S->cv_loop.notify_all();  // freed memory or slots may admit another lane's request
  }
  // drain: cancel whatever of this class is still queued
  std::lock_guard<std::mutex> g(S->mu);
  for (auto it = S->queue.begin(); it != S->queue.end();) {
    if ((*it)->lane == LN.id) {
      finish_request(S, *it, CANCELLED, HAC_ECANCELLED);
      it = S->queue.erase(it);
    } else {
      ++it;
    }
  }
  S->cv_done.notify_all();
}

hac_status take_result(hac_server* S, std::unique_lock<std::mutex>& lk, uint64_t ticket,
                       int32_t* tour_out, double* len_out, double* latency_s, bool block) {
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return HAC_EINVAL;
  std::shared_ptr<Request> r = it->second;
  if (block)
    S->cv_done.wait(lk, [&] { return r->state == DONE || r->state == CANCELLED || r->state == FAILED; });
  if (r->state == QUEUED || r->state == RUNNING) return HAC_EBUSY;
  hac_status st = r->status;
  if (r->state == DONE) {
    if (tour_out) std::memcpy(tour_out, r->tour.data(), 4 * r->tour.size());
    if (len_out) *len_out = r->length;
  }
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  S->reqs.erase(it);
  return st;
}

}  // namespace

extern "C" {

uint64_t hac_footprint(const hac_instance* inst, const hac_csr* heat, const hac_params* p) {
  if (!inst || !heat || !p || inst->n < 1) return 0;
  return footprint_of(inst, heat, p);
}

hac_status hac_server_create(hac_ctx* ctx, uint64_t budget_bytes, int32_t max_slots, hac_server** out) {
  if (!ctx || !out || budget_bytes == 0 || max_slots < 1) return HAC_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HAC_EDEVICE;
  hac_server* S = new hac_server();
  S->ctx = ctx;
  S->device = dev;
  S->budget = budget_bytes;
  S->max_slots = max_slots;
  for (int l = 0; l < kLanes; ++l) {
    S->lanes[l].id = l;
    S->lanes[l].st.min_n = l == 0 ? 1 : kLaneBound[l - 1];
    S->lanes[l].st.max_n = l == kLanes - 1 ? 0 : kLaneBound[l];
    if (l == 0) {
      S->lanes[0].stream = hac_context_stream(ctx);
      continue;
    }
    if (hipStreamCreateWithFlags(&S->lanes[l].stream, hipStreamNonBlocking) != hipSuccess) {
      for (int q = 1; q < l; ++q) (void)hipStreamDestroy(S->lanes[q].stream);
      delete S;
      return HAC_EDEVICE;
    }
  }
  hipError_t e = S->pool.init(budget_bytes);
  if (e != hipSuccess) {
    for (int l = 1; l < kLanes; ++l) (void)hipStreamDestroy(S->lanes[l].stream);
    delete S;
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? HAC_ENOMEM : HAC_EDEVICE;
  }
  for (int l = 0; l < kLanes; ++l) S->lanes[l].loop = std::thread(serve_lane, S, &S->lanes[l]);
  *out = S;
  return HAC_OK;
}

hac_status hac_server_submit(hac_server* S, const hac_instance* inst, const hac_csr* heat,
                             const hac_params* p, uint64_t seed, uint64_t* ticket) {
  if (!S || !ticket) return HAC_EINVAL;
  hac_status v = validate(inst, heat, p, nullptr);
  if (v != HAC_OK) return v;
  auto r = std::make_shared<Request>();
  const int32_t n = inst->n;
  if (inst->kind == HAC_COORDS_EUC2D) {
    r->coords.assign(inst->coords, inst->coords + 2 * (size_t)n);
  } else {
    r->dist.assign(inst->dist, inst->dist + (size_t)n * n);
  }
  r->row_ptr.assign(heat->row_ptr, heat->row_ptr + n + 1);
  r->col.assign(heat->col, heat->col + heat->nnz);
  r->val.assign(heat->val, heat->val + heat->nnz);
  r->inst = *inst;
  r->inst.coords = r->coords.empty() ? nullptr : r->coords.data();
  r->inst.dist = r->dist.empty() ? nullptr : r->dist.data();
  r->csr = *heat;
  r->csr.row_ptr = r->row_ptr.data();
  r->csr.col = r->col.data();
  r->csr.val = r->val.data();
  r->p = *p;
  r->seed = seed;
  r->lane = lane_of(n);
  r->bytes = footprint_of(inst, heat, p);
  r->t_submit = Clock::now();
  if (r->bytes > S->budget) return HAC_ENOMEM;
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) return HAC_ECANCELLED;
  r->ticket = S->next_ticket++;
  if (n == 1) {
    r->tour.assign(1, 0);
    r->length = 0.0;
    r->state = DONE;
    r->t_done = Clock::now();
    S->completed++;
  } else {
    S->queue.push_back(r);
  }
  S->gen++;
  S->reqs[r->ticket] = r;
  *ticket = r->ticket;
  S->cv_loop.notify_all();
  return HAC_OK;
}

hac_status hac_server_poll(hac_server* S, uint64_t ticket, int32_t* tour_out, double* length_out,
                           double* latency_s) {
  if (!S) return HAC_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  return take_result(S, lk, ticket, tour_out, length_out, latency_s, false);
}

hac_status hac_server_wait(hac_server* S, uint64_t ticket, int32_t* tour_out, double* length_out,
                           double* latency_s) {
  if (!S) return HAC_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  return take_result(S, lk, ticket, tour_out, length_out, latency_s, true);
}

hac_status hac_server_cancel(hac_server* S, uint64_t ticket) {
  if (!S) return HAC_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return HAC_EINVAL;
  it->second->cancel = true;
  S->gen++;
  S->cv_loop.notify_all();
  return HAC_OK;
}

hac_status hac_server_counters(hac_server* S, int64_t* admitted, int64_t* completed, int32_t* peak_slots,
                               uint64_t* peak_bytes) {
  if (!S) return HAC_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  if (admitted) *admitted = S->admitted;
  if (completed) *completed = S->completed;
  if (peak_slots) *peak_slots = S->peak_slots;
  if (peak_bytes) *peak_bytes = S->pool.peak();
  return HAC_OK;
}

hac_status hac_server_lane_stats(hac_server* S, int32_t lane, hac_lane_stats* out) {
  if (!S || !out || lane < 0 || lane >= kLanes) return HAC_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  *out = S->lanes[lane].st;
  return HAC_OK;
}

void hac_server_destroy(hac_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->gen++;
    for (auto& ln : S->lanes)
      for (auto& sl : ln.active) sl.req->cancel = true;
    S->cv_loop.notify_all();
  }
  for (auto& ln : S->lanes)
    if (ln.loop.joinable()) ln.loop.join();
  for (auto& ln : S->lanes) {
    (void)hipStreamSynchronize(ln.stream);
    if (ln.id != 0) (void)hipStreamDestroy(ln.stream);  // lane 0 runs on the context's stream
  }
  delete S;
}

}  // extern "C"
