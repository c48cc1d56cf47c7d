// Host-side internals shared by the runtime (runtime.cpp) and the serving
// scheduler (server.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "letkf.h"
#include "desc.hpp"

namespace letkf {

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define LETKF_HIP(call)                                     \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return ::letkf::hip_fail(e_, #call); \
  } while (0)

// Byte offsets of every region of one instance workspace.
struct Layout {
  size_t desc, state, hdr, ens, Yp, d, Z, y, amean, pmean;
  size_t a1, a2, rowptr, col, val, dom, order, est, obs_row, obs_r, obs_sr, mptr, mrow, mw, mdom, pist_op;
  size_t pist_r, pist_c, pist_ptr, pist_row, pist_coef;
  size_t bigA, bigB, bigv, bigf;   // m > 128 only
  size_t dom_sweeps, Ascr, dbg, dbg_sweeps;
  size_t static_begin, static_end;  // [a1, end of tables) uploaded at create
  size_t total;
};

struct Problem {  // validated, host-side copy of the create arguments
  int n_act = 0, n_sub = 0, m = 0, prec = 0, n_dom = 0, nnz = 0;
  int obs_instant = 0;      // 0: H = [D 0], 1: H = [0 D]
  uint32_t flags = 0;
  double sigma_v = 0, inflation = 1;
  uint64_t seed = 0;
  std::vector<double> a1, a2, r_inv, d_val;
  std::vector<int32_t> d_rowptr, d_col;
  std::vector<int32_t> est_ptr, est_act, obs_ptr, obs_sub;
  std::vector<double> est_w, obs_taper;
  int p() const { return 2 * n_sub; }
  int sum_e() const { return est_ptr.back(); }
  int sum_s() const { return obs_ptr.back(); }
  int zrows() const { return 2 * sum_e(); }
  size_t piston_terms() const {  // sum over actuators of (covering domains)^2
    std::vector<int> k(n_act, 0);
    for (int a : est_act) ++k[a];
    size_t t = 0;
    for (int v : k) t += (size_t)v * v;
    return t;
  }
  size_t esize() const { return prec == LETKF_FP64 ? 8 : 4; }
  bool fp32_rot() const { return (flags & LETKF_FLAG_FP32_ROTATIONS) != 0; }
  int cls() const { return class_of(padded_members(m), prec, fp32_rot()); }
};

int validate(const letkf_dims* dims, const letkf_model* model, const letkf_domain_map* map,
             int precision, uint32_t flags, Problem& out);
Layout make_layout(const Problem& P);

// Writes the instance into `ws` (device) on `stream` and waits.  `X0` is
// host n x m FP64.  Fills `desc` (host copy of the device descriptor).
// For a handle owned by a server: LETKF_EAGAIN if it has frames queued or in
// flight, else waits for the server stream and returns it in *stream.
int server_idle_stream(letkf_handle* h, hipStream_t* stream);

int upload_instance(const Problem& P, const Layout& L, char* ws, const double* X0, hipStream_t stream,
                    InstDesc& desc);

// XCDs of the GPU (MI355X): consecutive workgroups of a launch go to them in turn.
constexpr int kXcds = 8;

// The order in which an instance's domains become work items (LETKF_ORDER_*).
std::vector<int32_t> domain_order(const Problem& P, int policy);
// The per-XCD order re-placed by cost (LETKF_ORDER_BALANCED), or decreasing
// cost when more than `resident` domains (the workgroups resident at once);
// cost[l] in Jacobi-sweep units.
std::vector<int32_t> balanced_order(const Problem& P, const std::vector<double>& cost, int num_cu, int resident);
// Writes the instance's domain order for `policy` (LETKF_ORDER_BALANCED: from
// the domains' sweep sums so far) to its workspace on `s` and waits; `used`
// (nullable) receives the order.
int upload_order(letkf_handle* h, int policy, hipStream_t s, std::vector<int32_t>* used = nullptr);
// Same for a given order (checked to be a permutation of the domains).
int upload_order_vec(letkf_handle* h, const std::vector<int32_t>& order, int policy, hipStream_t s);

// Autotuning of one class's analysis launch over the batch described by the
// device header `hdr` (instances `insts`, whose domain orders it sets).
// Fills `res` and returns the chosen grid in *grid_out.
int tune_class(int cls, const InstDesc* tab, BatchHdr* hdr, int slope_rows, int items,
               const std::vector<letkf_handle*>& insts, int num_cu, int reps, bool balanced, int max_grid,
               hipStream_t s, letkf_tuning* res, int* grid_out);

}  // namespace letkf

struct letkf_handle {
  letkf::Problem P;
  letkf::Layout L;
  letkf::InstDesc desc{};      // host mirror of the device descriptor
  char* ws = nullptr;          // device workspace (caller- or arena-owned)
  int device = 0;
  int mpad = 16;
  int cls = 0;
  double* h_y = nullptr;       // pinned staging
  double* h_out = nullptr;     // pinned staging of the output means
  hipEvent_t y_free = nullptr; // last H2D of h_y completed
  bool y_pending = false;
  // kernel timing (letkf_kernel_times): 4 events per recorded call
  bool timing = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;              // quads recorded since the last flush
  double ms_acc[3] = {0, 0, 0};
  uint64_t timed_calls = 0;
  // captured frame (LETKF_FLAG_GRAPH)
  hipStream_t graph_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // analysis launch: persistent grid and domain order (letkf_autotune)
  int ana_grid = 0;
  int num_cu = 0;            // CUs of the device (the analysis launch's issue-priority rule)
  int max_rows = 0;            // most state rows of a domain (2 e), for the m > 128 launch sequence
  int order = LETKF_ORDER_COST;
  // serving
  letkf_server* server = nullptr;
  int slot = -1;               // index in the server's instance table
  size_t arena_off = 0;
};
