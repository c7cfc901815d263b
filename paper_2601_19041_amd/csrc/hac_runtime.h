// Host runtime shared by the C ABI (hac_api.cpp) and the request loop
// (hac_server.cpp).
#pragma once

#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/hac.h"
#include "hac_fold.h"
#include "hac_internal.h"

namespace hac {

// Grow-only device buffer with 256-byte aligned carving.
class DeviceArena {
 public:
  ~DeviceArena();
  hipError_t reserve(size_t bytes);
  void reset() { used_ = 0; }
  void* carve(size_t bytes);
  size_t capacity() const { return cap_; }
  void release();

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
};

// Sizes of the device arrays of one instance.
struct Layout {
  int32_t n, k, kg, kls, ants, iterations;
  bool coords, ls;
  bool directed;     // the ATSP with local search: directed 2-opt (incoming lists, larger work area)
  int32_t ls_tours;  // tours with their own 2-opt work area (ants when every ant is searched)
  bool three_opt = false;  // symmetric local search with the 3-opt
  int32_t gside;  // coordinate grid cells per side (0: none)
  int64_t nnz;
  size_t bytes() const;
};
Layout make_layout(const hac_instance* inst, const hac_csr* csr, const hac_params* p);

// Host view of one instance inside a batch.
struct HostInst {
  hac_instance inst;  // host pointers
  hac_csr csr;        // host pointers
  hac_params p;
  uint64_t seed;
  Layout lay;
  int32_t dstar, sym;
  double p_x;
  FoldOutput fold;
  double l_nn;
  InstDesc d;  // device pointers
  std::vector<int32_t> cand_h;  // host copy, used by the fold
  bool want_evid = false;         // keep the fold's e > 1 flags (diagnostics)
  std::vector<uint8_t> evid_gt1;
  // inputs that already live in device memory are copied device-to-device
  bool from_device = false;
  hac_instance dev_inst{};
  hac_csr dev_csr{};
};

// Chosen construction launch shape: ants per block, LDS staging of the
// candidate table, the widest candidate row of the batch (which sets the
// slots each of an ant's 16 lanes holds), and the ants per wave (one per
// 16-lane row; fewer than four keeps the other rows' fallback scans out of
// an ant's critical path).
struct LaunchShape {
  int32_t ants_per_block;
  int32_t staged;
  int32_t kmax;
  int32_t rows_per_wave;
  int32_t bytes;  // visited marks: one byte per node (when they fit every instance) or one bit
  int32_t geo = 1;  // geometric-list mode of the construction kernel (launch_construct)
  int32_t grid = 0; // some instance has a coordinate grid (else the grid search is compiled out)
};

// One decode batch: everything from uploaded inputs to results.
struct Engine {
  hipStream_t stream = nullptr;
  std::string* err = nullptr;
  bool timing = false;
  bool use_graph = true;
  // results of the last run
  double construct_ms = 0.0;
  int64_t construct_launches = 0;
  LaunchShape shape{4, 0, 16, 4, 0};
};

hac_status validate(const hac_instance* inst, const hac_csr* csr, const hac_params* p,
                    std::string* why);
int32_t degree_target_of(const hac_instance* inst, const hac_params* p);

// The geometric-list modes the tuner tries for a staging form: with the
// table in LDS, 1 (int32 lists loaded at each step); with the table in
// global memory, 0 (no list check) and 2 (uint16 lists loaded a step ahead,
// when every instance has them; else 1).  HAC_GEO_MODE (0, 1 or 2) pins
// the mode where it applies.
std::vector<int32_t> geo_modes(const std::vector<HostInst>& hs, int32_t staged);

// Builds the XCD-aware construction block map.
std::vector<BlockMap> build_block_map(const std::vector<HostInst>& hs, int32_t ants_per_block);

// Launch-shape autotuner: picks ants-per-block and LDS staging by timing
// the construction kernel; cached per shape class.  shared = true for the
// server's lanes, which run beside each other: their choices are timed and
// cached apart from those of decodes that have the GPU to themselves.
LaunchShape tune_shape(const std::vector<HostInst>& hs, const InstDesc* d_descs, hipStream_t s,
                       DeviceArena& scratch, bool* ok, bool shared = false);

// Prepares instances whose inputs are already uploaded into their slots:
// candidates, host fold, NN tour (+2-opt), range checks, initialisation.
// stage: when given, readbacks and uploads of the whole batch go through it
// as one gather launch and one copy each, instead of a copy per array
hac_status prepare_instances(std::vector<HostInst>& hs, InstDesc* d_descs, hipStream_t s,
                             std::string* err, DeviceArena* stage = nullptr);

// Fills the device pointers of h.d from a carver (256-byte aligned pieces).
void assign_slot(HostInst& h, const std::function<void*(size_t)>& carve);
// Fills the scalar fields of h.d from h's parameters.
void fill_desc_scalars(HostInst& h);
size_t align256(size_t bytes);
size_t shape_lds(const std::vector<HostInst>& hs, LaunchShape sh);
// largest candidate-list width of a batch (selects the reduction width)
int32_t batch_max_k(const std::vector<HostInst>& hs);

// Copies the host inputs of h into its slot (asynchronous on s).
hipError_t upload_inputs(const HostInst& h, hipStream_t s);

}  // namespace hac

// The stream a context runs on (the request loop's first lane uses it).
hipStream_t hac_context_stream(const hac_ctx* ctx);

namespace hac {

}  // namespace hac
