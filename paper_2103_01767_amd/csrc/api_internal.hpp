// Host-side internals of the C ABI: the problem plan and the handle.
#pragma once
#include <string>
#include <vector>

#include "ptlm.h"
#include "internal.hpp"

namespace ptlm {

struct Offsets {
  size_t tw, pos, seg_start, seg_box, seg_off, otile_ptr, otile_seg, ptile_ptr, ptile_pos;
  size_t O_lin, P_lin, afield, w2, trace, strips, probe_part, partials, scratch, scal;
  size_t g, dx, prev, r, z, p, Ap, diag, ztrial, learned, lmstate;
  size_t afield2, w2_2, trace2, g2;  // spare linearisation (trial point of the LM)
};

// Everything derived on the host from the description and the positions.
struct Plan {
  ptlm_desc d{};
  int tpw = 1, grid = 1, nseg = 1;
  double grid_scale = 1.0;             // workgroups = scale x resident workgroups (autotuned)
  int max_grid = 1;                    // largest grid over the autotuner's candidates
  std::vector<int> seg_start;
  std::vector<int4> seg_box;           // (row0, col0, rows, cols)
  std::vector<long long> seg_off;
  long long strip_elems = 0;
  int oty = 0, otx = 0;
  std::vector<int> otile_ptr, otile_seg, ptile_ptr, ptile_pos;
  std::vector<float2> tw;
  std::vector<int> pos;
  size_t nvec = 0;                     // complex entries of one vector of R^(2n)
  Offsets off{};
  size_t ws_bytes = 0;
};

}  // namespace ptlm

struct ptlm_handle {
  ptlm::Plan plan;
  ptlm::Geometry g{};
  char* ws = nullptr;
  bool in_batch = false;    // a problem of a batch: its launch shape is fixed by the batch's tables
  ptlm_cnn_desc cnn{};      // registered preconditioner network (ptlm_lm_set_cnn)
  const float* cnn_params = nullptr;
  char* cnn_ws = nullptr;
  int cnn_every = 1;        // network refresh period in linearisations (0: once after registration)
  int cnn_count = 0;        // linearisations since registration
  bool cnn_ready = false;   // the network output r in cnn_ws is current
  // PCG look-ahead of ptlm_lm_step: pinned host slots the finalize kernels write the PCG
  // continuation flag to, and one event per slot
  int* cg_flags = nullptr;  // null for the handles of a batch: no look-ahead there
  int* ls_flags = nullptr;  // the same for the projected plug-in's line search (second half of
                            // the same pinned block; the events are shared)
  int cg_slots = 0;
  std::vector<hipEvent_t> cg_events;
  // Linearisation at the LM's trial point, computed into spare buffers and swapped in when the
  // step is accepted: the LM gradient in use and its spare, the spare phasors / weights /
  // traces, the linearisation generation (bumped by ptlm_linearize) when the swap was made and
  // the data pointer it used.
  float2* lm_g = nullptr;
  float2* lm_g_alt = nullptr;
  float2* afield_alt = nullptr;
  float* w2_alt = nullptr;
  double* trace_alt = nullptr;
  unsigned lin_gen = 0;
  unsigned kept_gen = ~0u;
  const float* kept_y = nullptr;
  int device = 0;                            // device current at creation
  hipEvent_t tune_ev[2] = {nullptr, nullptr}; // timing events of ptlm_autotune
  ~ptlm_handle();
};

namespace ptlm {
constexpr int kCgSlots = 129;  // PCG look-ahead slots of a single-problem handle (cg_max <= 128)
extern thread_local std::string g_last_error;
ptlm_status fail(ptlm_status st, const std::string& msg);
ptlm_status hip_fail(hipError_t e, const char* where);
ptlm_status make_plan(const ptlm_desc* d, const int32_t* h_pos, Plan& p, double grid_scale = 1.0);
// segment count scales the autotuner tries (the workspace holds the largest segment tables)
constexpr int kNumGridScales = 3;
constexpr int kNumTransforms = 3;  // ptlm_transform values
extern const double kGridScales[kNumGridScales];
// workgroups of the tile kernels at a grid scale; cut the positions into segments for them
int plan_grid(const Plan& p, double scale);
void segment(Plan& p, const int* h_pos, int grid);
ptlm_status linearize_impl(ptlm_handle* h, const float2* O, const float2* P, const float* y, double* d_f,
                           float2* gO, float2* gP, hipStream_t s);
ptlm_status ggnv_impl(ptlm_handle* h, const float2* vO, const float2* vP, double lam, const double* lam_dev,
                      const float* dO, const float* dP, float2* outO, float2* outP, const int* pred, hipStream_t s,
                      int stage = 3, double* pap = nullptr, const int* pap_block = nullptr);
ptlm_status diag_exact_impl(ptlm_handle* h, float* dO, float* dP, hipStream_t s, const int* pred = nullptr);
ptlm_status diag_stochastic_impl(ptlm_handle* h, int samples, unsigned long long seed, unsigned long long draw0,
                                 const int* draw_t, float* dO, float* dP, hipStream_t s, const int* pred = nullptr);
ptlm_status resegment(ptlm_handle* h, double scale, hipStream_t s);
ptlm_status autotune_impl(ptlm_handle* h, int reps, double* h_ms, double* h_scale, int32_t* h_xform,
                          hipStream_t s);
// run the handle's registered network on its features: from the linearisation's probe, or from P
// (a device probe of the handle's shape) when given
ptlm_status cnn_refresh(ptlm_handle* h, hipStream_t s, const float2* P = nullptr);
const float* cnn_output(const ptlm_handle* h);
ptlm_status init_handle(ptlm_handle* h, const ptlm_desc* desc, const int32_t* h_pos, void* d_ws, size_t ws_bytes,
                        hipStream_t s);
}  // namespace ptlm
