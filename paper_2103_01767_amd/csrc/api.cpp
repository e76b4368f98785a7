// C ABI of the library: handles, validation and the product calls (forward, loss,
// linearise, JVP, VJP, GGN-vector product, diagonals), the autotuner.  Planning and the
// workspace layout live in plan.cpp, the LM driver in lm.cpp.
#include "api_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

namespace ptlm {

thread_local std::string g_last_error;

ptlm_status fail(ptlm_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

ptlm_status hip_fail(hipError_t e, const char* where) {
  return fail(PTLM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Scratch of ptlm_loss_noalloc, the one entry point for callers that cannot allocate: the
// per-workgroup FP64 partial sums of the loss kernel (4 doubles a workgroup), in static device
// memory instead of the handle's workspace.  Each device holds its own copy until the process
// ends; host code reaches it only through the per-device address taken at handle creation.
constexpr int kNoAllocMaxBlocks = 8192;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocMaxBlocks * 4];
static double* g_scratch_ptr[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];
static std::once_flag g_scratch_once[kMaxDevices];

// Address of `scratch` on device `dev` (which must be current), taken once per device.
static hipError_t scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? (double*)p : nullptr;
  });
  return g_scratch_err[dev];
}

#define PTLM_CHECK_H(h)                                    \
  do {                                                     \
    if (!(h)) return fail(PTLM_EINVAL, "handle is null"); \
  } while (0)
#define PTLM_HIP(call, where)                         \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

ptlm_status diag_exact_impl(ptlm_handle* h, float* dO, float* dP, hipStream_t s, const int* pred) {
  TileArgs a{};
  a.O = h->g.O_lin;
  a.P = h->g.P_lin;
  a.predicate = pred;
  hipError_t e = launch_tile(h->g, OP_DIAG_EXACT, a, s);
  if (e != hipSuccess) return hip_fail(e, "diag exact");
  e = launch_reduce_pair(h->g, (float2*)dO, (float2*)dP, 0.0, nullptr, nullptr, nullptr, nullptr, nullptr, pred, s);
  if (e != hipSuccess) return hip_fail(e, "diag exact reduce");
  return PTLM_OK;
}

// Stochastic estimate of diag(G): the mean over `samples` draws of the squared real coordinates
// of J^T diag(sqrt(W)) r, r a sign field per draw.  Draw s of the call is draw0 + s, plus
// (*draw_t) * samples when draw_t is set (the LM's outer iteration).  The LM vector z serves
// as the per-draw scratch.
ptlm_status diag_stochastic_impl(ptlm_handle* h, int samples, unsigned long long seed, unsigned long long draw0,
                                 const int* draw_t, float* dO, float* dP, hipStream_t s, const int* pred) {
  Geometry& g = h->g;
  const size_t N = (size_t)g.ny * g.nx, M = (size_t)g.my * g.mx;
  float2* u = (float2*)(h->ws + h->plan.off.z);
  const float scale = 1.0f / (float)samples;
  for (int k = 0; k < samples; ++k) {
    TileArgs a{};
    a.O = g.O_lin;
    a.P = g.P_lin;
    a.predicate = pred;
    a.rseed = seed;
    a.rdraw = draw0 + (unsigned long long)k;
    a.rdraw_t = draw_t;
    a.rdraw_mul = samples;
    hipError_t e = launch_tile(g, OP_VJP_RAND, a, s);
    if (e != hipSuccess) return hip_fail(e, "stochastic diag");
    e = launch_obj_reduce(g, u, 0.0, nullptr, nullptr, nullptr, pred, s);
    if (e == hipSuccess) e = launch_sq_accum(u, (float2*)dO, N, scale, k == 0, pred, s);
    if (e == hipSuccess && dP) e = launch_probe_reduce(g, u + N, 0.0, nullptr, nullptr, nullptr, pred, s);
    if (e == hipSuccess && dP) e = launch_sq_accum(u + N, (float2*)dP, M, scale, k == 0, pred, s);
    if (e != hipSuccess) return hip_fail(e, "stochastic diag accumulate");
  }
  return PTLM_OK;
}

ptlm_status linearize_impl(ptlm_handle* h, const float2* O, const float2* P, const float* y, double* d_f,
                           float2* gO, float2* gP, hipStream_t s) {
  Geometry& g = h->g;
  h->lin_gen += 1;  // the LM may no longer adopt a linearisation it kept
  const size_t N = (size_t)g.ny * g.nx, M = (size_t)g.my * g.mx;
  if ((const void*)O != (const void*)g.O_lin)
    PTLM_HIP(hipMemcpyAsync(g.O_lin, O, N * sizeof(float2), hipMemcpyDeviceToDevice, s), "linearize copy O");
  if ((const void*)P != (const void*)g.P_lin)
    PTLM_HIP(hipMemcpyAsync(g.P_lin, P, M * sizeof(float2), hipMemcpyDeviceToDevice, s), "linearize copy P");
  TileArgs a{};
  a.O = g.O_lin;
  a.P = g.P_lin;
  a.y = y;
  PTLM_HIP(launch_tile(g, OP_LINEARIZE, a, s), "linearize");
  PTLM_HIP(launch_refine(g, a, s), "linearize refine");
  PTLM_HIP(launch_sum_partials(g.partials, g.grid, d_f, 2, s), "linearize sum");
  PTLM_HIP(launch_reduce_pair(g, gO, g.joint ? gP : nullptr, 0.0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                              s),
           "linearize gradient");
  return PTLM_OK;
}

ptlm_status ggnv_impl(ptlm_handle* h, const float2* vO, const float2* vP, double lam, const double* lam_dev,
                      const float* dO, const float* dP, float2* outO, float2* outP, const int* pred, hipStream_t s,
                      int stage, double* pap, const int* pap_block) {
  if (stage & 1) {
    TileArgs a{};
    a.O = h->g.O_lin;
    a.P = h->g.P_lin;
    a.vO = vO;
    a.vP = h->g.joint ? vP : nullptr;
    a.predicate = pred;
    PTLM_HIP(launch_tile(h->g, OP_GGNV, a, s), "ggn_vp");
  }
  if (stage & 2) {
    PTLM_HIP(launch_reduce_pair(h->g, outO, h->g.joint ? outP : nullptr, lam, lam_dev, dO, dP, vO, vP, pred, s, pap,
                                pap_block),
             "ggn_vp reduce");
  }
  return PTLM_OK;
}

ptlm_status init_handle(ptlm_handle* h, const ptlm_desc* desc, const int32_t* h_pos, void* d_ws, size_t ws_bytes,
                        hipStream_t s) {
  ptlm_status st = make_plan(desc, h_pos, h->plan);
  if (st != PTLM_OK) return st;
  Plan& p = h->plan;
  if (!d_ws || ws_bytes < p.ws_bytes) {
    char buf[128];
    snprintf(buf, sizeof buf, "workspace of %zu bytes, %zu needed", ws_bytes, p.ws_bytes);
    return fail(PTLM_EWORKSPACE, buf);
  }
  PTLM_HIP(hipGetDevice(&h->device), "ptlm_create device");
  PTLM_HIP(scratch_setup(h->device), "ptlm_create static scratch");
  PTLM_HIP(hipEventCreate(&h->tune_ev[0]), "ptlm_create autotune events");
  PTLM_HIP(hipEventCreate(&h->tune_ev[1]), "ptlm_create autotune events");
  h->ws = (char*)d_ws;
  Geometry& g = h->g;
  const ptlm_desc& d = p.d;
  g.ny = d.ny; g.nx = d.nx; g.my = d.my; g.mx = d.mx; g.K = d.K;
  g.metric = d.metric;
  g.ggn = d.ggn;
  g.joint = d.mode == PTLM_JOINT;
  g.background = d.background;
  g.nseg = p.nseg;
  g.grid = p.grid;
  auto at = [&](size_t o) { return (void*)(h->ws + o); };
  g.tw = (const float2*)at(p.off.tw);
  g.pos = (const int2*)at(p.off.pos);
  g.seg_start = (const int*)at(p.off.seg_start);
  g.seg_box = (const int4*)at(p.off.seg_box);
  g.seg_off = (const long long*)at(p.off.seg_off);
  g.otile_ptr = (const int*)at(p.off.otile_ptr);
  g.otile_seg = (const int*)at(p.off.otile_seg);
  g.ptile_ptr = (const int*)at(p.off.ptile_ptr);
  g.ptile_pos = (const int*)at(p.off.ptile_pos);
  g.otiles_y = p.oty;
  g.otiles_x = p.otx;
  g.O_lin = (float2*)at(p.off.O_lin);
  g.P_lin = (float2*)at(p.off.P_lin);
  g.afield = (float2*)at(p.off.afield);
  g.w2 = (d.metric == PTLM_POISSON || d.ggn == PTLM_GGN_INTENSITY) ? (float*)at(p.off.w2) : nullptr;
  g.trace = (double*)at(p.off.trace);
  g.strips = (float2*)at(p.off.strips);
  g.probe_part = (float2*)at(p.off.probe_part);
  g.partials = (double*)at(p.off.partials);
  g.scratch = d.my == 256 ? (float2*)at(p.off.scratch) : nullptr;
  g.xform = default_xform(d.my, d.mx);
  h->lm_g = (float2*)at(p.off.g);
  h->lm_g_alt = (float2*)at(p.off.g2);
  h->afield_alt = (float2*)at(p.off.afield2);
  h->w2_alt = g.w2 ? (float*)at(p.off.w2_2) : nullptr;
  h->trace_alt = (double*)at(p.off.trace2);
  h->lin_gen += 1;

  hipError_t e;
  auto up = [&](size_t off, const void* src, size_t bytes) {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(at(off), src, bytes, hipMemcpyHostToDevice, s);
  };
  if ((e = up(p.off.tw, p.tw.data(), p.tw.size() * sizeof(float2))) != hipSuccess ||
      (e = up(p.off.pos, p.pos.data(), p.pos.size() * sizeof(int))) != hipSuccess ||
      (e = up(p.off.seg_start, p.seg_start.data(), p.seg_start.size() * sizeof(int))) != hipSuccess ||
      (e = up(p.off.seg_box, p.seg_box.data(), p.seg_box.size() * sizeof(int4))) != hipSuccess ||
      (e = up(p.off.seg_off, p.seg_off.data(), p.seg_off.size() * sizeof(long long))) != hipSuccess ||
      (e = up(p.off.otile_ptr, p.otile_ptr.data(), p.otile_ptr.size() * sizeof(int))) != hipSuccess ||
      (e = up(p.off.otile_seg, p.otile_seg.data(), p.otile_seg.size() * sizeof(int))) != hipSuccess ||
      (e = up(p.off.ptile_ptr, p.ptile_ptr.data(), p.ptile_ptr.size() * sizeof(int))) != hipSuccess ||
      (e = up(p.off.ptile_pos, p.ptile_pos.data(), p.ptile_pos.size() * sizeof(int))) != hipSuccess ||
      (e = hipMemsetAsync(at(p.off.strips), 0, (size_t)p.strip_elems * sizeof(float2), s)) != hipSuccess ||
      (e = hipMemsetAsync(at(p.off.probe_part), 0, (size_t)p.nseg * d.my * d.mx * sizeof(float2), s)) !=
          hipSuccess) {
    return hip_fail(e, "ptlm_create upload");
  }
  return PTLM_OK;
}


// Re-segment the handle's positions for another grid scale and upload the segment tables
// (the stored phasor field and every other per-position array are unaffected).
ptlm_status resegment(ptlm_handle* h, double scale, hipStream_t s) {
  Plan& p = h->plan;
  segment(p, p.pos.data(), plan_grid(p, scale));
  p.grid_scale = scale;
  h->g.nseg = p.nseg;
  h->g.grid = p.grid;
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(h->ws + off, src, bytes, hipMemcpyHostToDevice, s);
  };
  PTLM_HIP(up(p.off.seg_start, p.seg_start.data(), p.seg_start.size() * sizeof(int)), "resegment");
  PTLM_HIP(up(p.off.seg_box, p.seg_box.data(), p.seg_box.size() * sizeof(int4)), "resegment");
  PTLM_HIP(up(p.off.seg_off, p.seg_off.data(), p.seg_off.size() * sizeof(long long)), "resegment");
  PTLM_HIP(up(p.off.otile_ptr, p.otile_ptr.data(), p.otile_ptr.size() * sizeof(int)), "resegment");
  PTLM_HIP(up(p.off.otile_seg, p.otile_seg.data(), p.otile_seg.size() * sizeof(int)), "resegment");
  // the host tables are rewritten by the next call: finish the copies first
  PTLM_HIP(hipStreamSynchronize(s), "resegment sync");
  return PTLM_OK;
}

ptlm_status autotune_impl(ptlm_handle* h, int reps, double* h_ms, double* h_scale, int32_t* h_xform,
                          hipStream_t s) {
  Plan& p = h->plan;
  const size_t N = (size_t)p.d.ny * p.d.nx;
  float2* out = (float2*)(h->ws + p.off.Ap);
  const float2* vO = h->g.O_lin;
  const float2* vP = h->g.joint ? h->g.P_lin : nullptr;
  hipEvent_t e0 = h->tune_ev[0], e1 = h->tune_ev[1];
  double best = 1e300;
  int bi = 1, bx = h->g.xform;
  ptlm_status st = PTLM_OK;
  const int nc = (int)(kNumGridScales);
  if (h_ms)
    for (int i = 0; i < kNumTransforms * nc; ++i) h_ms[i] = -1.0;
  for (int x = 0; x < kNumTransforms && st == PTLM_OK; ++x) {
    if ((x == PTLM_TRANSFORM_MFMA && !ggnv_mfma_supported(h->g.my, h->g.mx)) ||
        (x == PTLM_TRANSFORM_FFT_WIDE && !ggnv_wide_supported(h->g.my, h->g.mx)))
      continue;
    h->g.xform = x;
    for (int i = 0; i < nc && st == PTLM_OK; ++i) {
      st = resegment(h, kGridScales[i], s);
      if (st != PTLM_OK) break;
      st = ggnv_impl(h, vO, vP, 0.0, nullptr, nullptr, nullptr, out, h->g.joint ? out + N : nullptr, nullptr, s);
      if (st != PTLM_OK) break;
      hipEventRecord(e0, s);
      for (int r = 0; r < reps && st == PTLM_OK; ++r)
        st = ggnv_impl(h, vO, vP, 0.0, nullptr, nullptr, nullptr, out, h->g.joint ? out + N : nullptr, nullptr, s);
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      const double per = (double)ms / std::max(reps, 1);
      if (h_ms) h_ms[x * nc + i] = per;
      if (per < best) {
        best = per;
        bi = i;
        bx = x;
      }
    }
  }
  h->g.xform = bx;
  if (st != PTLM_OK) return st;
  if (h_scale) *h_scale = kGridScales[bi];
  if (h_xform) *h_xform = bx;
  return resegment(h, kGridScales[bi], s);
}
}  // namespace ptlm

using namespace ptlm;

extern "C" {

void ptlm_lm_default_params(ptlm_lm_params* p) {
  if (!p) return;
  p->mu0 = 1e-5;
  p->mu_min = 1e-8;
  p->kappa = 4.0;
  p->nu = 1.0;
  p->rho_min = 1e-4;
  p->beta = 0.1;
  p->diag_floor = 1e-6;
  p->cg_max = 10;
  p->retry_max = 10;
  p->scaling = 0;
  p->precond = 0;
  p->warm_start = 1;
  p->surrogate_T = 0;
  p->surrogate_s0 = 1.0;
  p->project = 0;
  p->ls_max = 30;
  p->o_max = 1.0;
  p->p_max = 1e8;
  p->sigma_ls = 1e-4;
  p->gamma = 1e-6;
  p->tau_s = 1e-8;
  p->p_s = 2.1;
  p->alternate = 0;
  p->stoch_samples = 8;
  p->stoch_seed = 0;
}

ptlm_status ptlm_workspace_bytes(const ptlm_desc* desc, const int32_t* h_pos, size_t* bytes) {
  if (!bytes) return fail(PTLM_EINVAL, "bytes is null");
  Plan p;
  ptlm_status st = make_plan(desc, h_pos, p);
  if (st != PTLM_OK) return st;
  *bytes = p.ws_bytes;
  return PTLM_OK;
}

}  // extern "C"

// Pinned host slots and events of the PCG and line-search look-ahead (ptlm_lm_step), made once
// with the handle so that no LM call allocates; solves with more than kCgSlots - 1 iterations
// (line searches with more than kCgSlots step sizes) enqueue all of them.
static ptlm_status cg_slots_create(ptlm_handle* h) {
  void* p = nullptr;
  PTLM_HIP(hipHostMalloc(&p, (size_t)(2 * kCgSlots) * sizeof(int), hipHostMallocCoherent), "pcg slots");
  h->cg_flags = (int*)p;
  h->ls_flags = h->cg_flags + kCgSlots;
  h->cg_slots = kCgSlots;
  for (int i = 0; i < kCgSlots; ++i) {
    hipEvent_t e;
    PTLM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "pcg events");
    h->cg_events.push_back(e);
  }
  return PTLM_OK;
}

extern "C" {

ptlm_status ptlm_create(const ptlm_desc* desc, const int32_t* h_pos, void* d_ws, size_t ws_bytes, void* stream,
                        ptlm_handle** out) {
  if (!out) return fail(PTLM_EINVAL, "out is null");
  *out = nullptr;
  ptlm_handle* h = new ptlm_handle();
  ptlm_status st = init_handle(h, desc, h_pos, d_ws, ws_bytes, (hipStream_t)stream);
  if (st == PTLM_OK) st = cg_slots_create(h);
  if (st != PTLM_OK) {
    delete h;
    return st;
  }
  *out = h;
  return PTLM_OK;
}

ptlm_status ptlm_destroy(ptlm_handle* h) {
  delete h;
  return PTLM_OK;
}

}  // extern "C"

ptlm_handle::~ptlm_handle() {
  for (hipEvent_t e : cg_events) (void)hipEventDestroy(e);
  for (hipEvent_t e : tune_ev)
    if (e) (void)hipEventDestroy(e);
  if (cg_flags) (void)hipHostFree(cg_flags);
}

extern "C" {

ptlm_status ptlm_forward(ptlm_handle* h, const float* d_O, const float* d_P, float* d_zeta, void* stream) {
  PTLM_CHECK_H(h);
  if (!d_O || !d_P || !d_zeta) return fail(PTLM_EINVAL, "null array");
  TileArgs a{};
  a.O = (const float2*)d_O;
  a.P = (const float2*)d_P;
  a.rout = d_zeta;
  PTLM_HIP(launch_tile(h->g, OP_FORWARD, a, (hipStream_t)stream), "forward");
  return PTLM_OK;
}

ptlm_status ptlm_loss(ptlm_handle* h, const float* d_O, const float* d_P, const float* d_y, double* d_f,
                      float* d_resid, void* stream) {
  PTLM_CHECK_H(h);
  if (!d_O || !d_P || !d_y || !d_f) return fail(PTLM_EINVAL, "null array");
  hipStream_t s = (hipStream_t)stream;
  TileArgs a{};
  a.O = (const float2*)d_O;
  a.P = (const float2*)d_P;
  a.y = d_y;
  a.rout = d_resid;
  PTLM_HIP(launch_tile(h->g, OP_LOSS, a, s), "loss");
  PTLM_HIP(launch_sum_partials(h->g.partials, h->g.grid, d_f, 1, s), "loss sum");
  return PTLM_OK;
}

ptlm_status ptlm_loss_noalloc(ptlm_handle* h, const float* d_O, const float* d_P, const float* d_y, double* d_f,
                              float* d_resid, void* stream) {
  PTLM_CHECK_H(h);
  if (!d_O || !d_P || !d_y || !d_f) return fail(PTLM_EINVAL, "null array");
  if (h->g.my == 256 && h->g.mx == 256)
    return fail(PTLM_EINVAL, "ptlm_loss_noalloc: 256 x 256 probes transform through the workspace; use ptlm_loss");
  if (h->g.grid > kNoAllocMaxBlocks) {
    char buf[160];
    snprintf(buf, sizeof buf, "ptlm_loss_noalloc: %d workgroups, the static scratch holds the partial sums of %d",
             h->g.grid, kNoAllocMaxBlocks);
    return fail(PTLM_EINVAL, buf);
  }
  int dev = -1;
  PTLM_HIP(hipGetDevice(&dev), "ptlm_loss_noalloc device");
  if (dev != h->device) return fail(PTLM_EINVAL, "ptlm_loss_noalloc: the handle's device is not current");
  double* part = g_scratch_ptr[h->device];
  if (!part) return fail(PTLM_EHIP, "ptlm_loss_noalloc: static scratch address unavailable");
  hipStream_t s = (hipStream_t)stream;
  Geometry g = h->g;
  g.partials = part;  // every workgroup of the loss kernel writes all four of its entries
  TileArgs a{};
  a.O = (const float2*)d_O;
  a.P = (const float2*)d_P;
  a.y = d_y;
  a.rout = d_resid;
  PTLM_HIP(launch_tile(g, OP_LOSS, a, s), "loss_noalloc");
  PTLM_HIP(launch_sum_partials(part, g.grid, d_f, 1, s), "loss_noalloc sum");
  return PTLM_OK;
}

ptlm_status ptlm_linearize(ptlm_handle* h, const float* d_O, const float* d_P, const float* d_y, double* d_f,
                           float* d_gO, float* d_gP, void* stream) {
  PTLM_CHECK_H(h);
  if (!d_O || !d_P || !d_y || !d_f || !d_gO) return fail(PTLM_EINVAL, "null array");
  if (h->g.joint && !d_gP) return fail(PTLM_EINVAL, "joint mode needs d_gP");
  return linearize_impl(h, (const float2*)d_O, (const float2*)d_P, d_y, d_f, (float2*)d_gO, (float2*)d_gP,
                        (hipStream_t)stream);
}

ptlm_status ptlm_jvp(ptlm_handle* h, const float* d_vO, const float* d_vP, float* d_out, void* stream) {
  PTLM_CHECK_H(h);
  if (!d_vO || !d_out) return fail(PTLM_EINVAL, "null array");
  if (h->g.joint && !d_vP) return fail(PTLM_EINVAL, "joint mode needs d_vP");
  TileArgs a{};
  a.O = h->g.O_lin;
  a.P = h->g.P_lin;
  a.vO = (const float2*)d_vO;
  a.vP = h->g.joint ? (const float2*)d_vP : nullptr;
  a.rout = d_out;
  PTLM_HIP(launch_tile(h->g, OP_JVP, a, (hipStream_t)stream), "jvp");
  return PTLM_OK;
}

ptlm_status ptlm_vjp(ptlm_handle* h, const float* d_w, float* d_outO, float* d_outP, void* stream) {
  PTLM_CHECK_H(h);
  if (!d_w || !d_outO) return fail(PTLM_EINVAL, "null array");
  if (h->g.joint && !d_outP) return fail(PTLM_EINVAL, "joint mode needs d_outP");
  hipStream_t s = (hipStream_t)stream;
  TileArgs a{};
  a.O = h->g.O_lin;
  a.P = h->g.P_lin;
  a.win = d_w;
  PTLM_HIP(launch_tile(h->g, OP_VJP, a, s), "vjp");
  PTLM_HIP(launch_reduce_pair(h->g, (float2*)d_outO, h->g.joint ? (float2*)d_outP : nullptr, 0.0, nullptr, nullptr,
                              nullptr, nullptr, nullptr, nullptr, s),
           "vjp reduce");
  return PTLM_OK;
}

ptlm_status ptlm_ggn_vp_stage(ptlm_handle* h, const float* d_vO, const float* d_vP, double lambda,
                              const float* d_dO, const float* d_dP, float* d_outO, float* d_outP, int32_t stage,
                              void* stream) {
  PTLM_CHECK_H(h);
  if (stage < 1 || stage > 3) return fail(PTLM_EINVAL, "stage must be 1, 2 or 3");
  if (!d_vO || ((stage & 2) && !d_outO)) return fail(PTLM_EINVAL, "null array");
  if (h->g.joint && (!d_vP || ((stage & 2) && !d_outP))) return fail(PTLM_EINVAL, "joint mode needs d_vP and d_outP");
  if (!std::isfinite(lambda) || lambda < 0.0) return fail(PTLM_EINVAL, "lambda must be finite and >= 0");
  return ggnv_impl(h, (const float2*)d_vO, (const float2*)d_vP, lambda, nullptr, d_dO, d_dP, (float2*)d_outO,
                   (float2*)d_outP, nullptr, (hipStream_t)stream, stage);
}

ptlm_status ptlm_ggn_vp(ptlm_handle* h, const float* d_vO, const float* d_vP, double lambda, const float* d_dO,
                        const float* d_dP, float* d_outO, float* d_outP, void* stream) {
  return ptlm_ggn_vp_stage(h, d_vO, d_vP, lambda, d_dO, d_dP, d_outO, d_outP, 3, stream);
}

ptlm_status ptlm_set_transform(ptlm_handle* h, int32_t transform) {
  PTLM_CHECK_H(h);
  if (h->in_batch) return fail(PTLM_EINVAL, "ptlm_set_transform: the handle belongs to a batch");
  if (transform != PTLM_TRANSFORM_FFT && transform != PTLM_TRANSFORM_MFMA && transform != PTLM_TRANSFORM_FFT_WIDE)
    return fail(PTLM_EINVAL, "ptlm_set_transform: unknown transform");
  if (transform == PTLM_TRANSFORM_MFMA && !ggnv_mfma_supported(h->g.my, h->g.mx))
    return fail(PTLM_EINVAL, "ptlm_set_transform: the matrix-product transform needs 16 x 16 or 32 x 32 probes");
  if (transform == PTLM_TRANSFORM_FFT_WIDE && !ggnv_wide_supported(h->g.my, h->g.mx))
    return fail(PTLM_EINVAL, "ptlm_set_transform: the wide grouping needs probe sides of 16-128 with at most 4096 pixels");
  h->g.xform = transform;
  return PTLM_OK;
}

ptlm_status ptlm_diag(ptlm_handle* h, float* d_dO, float* d_dP, int32_t exact, void* stream) {
  PTLM_CHECK_H(h);
  if (!d_dO) return fail(PTLM_EINVAL, "null array");
  if (h->g.joint && !d_dP) return fail(PTLM_EINVAL, "joint mode needs d_dP");
  if (exact) return diag_exact_impl(h, d_dO, h->g.joint ? d_dP : nullptr, (hipStream_t)stream);
  PTLM_HIP(launch_diag_paper(h->g, d_dO, h->g.joint ? d_dP : nullptr, (hipStream_t)stream), "diag");
  return PTLM_OK;
}

ptlm_status ptlm_diag_stochastic(ptlm_handle* h, int32_t samples, uint64_t seed, uint64_t draw0, float* d_dO,
                                 float* d_dP, void* stream) {
  PTLM_CHECK_H(h);
  if (!d_dO) return fail(PTLM_EINVAL, "null array");
  if (h->g.joint && !d_dP) return fail(PTLM_EINVAL, "joint mode needs d_dP");
  if (samples < 1) return fail(PTLM_EINVAL, "samples must be >= 1");
  return diag_stochastic_impl(h, samples, seed, draw0, nullptr, d_dO, h->g.joint ? d_dP : nullptr,
                              (hipStream_t)stream);
}

ptlm_status ptlm_autotune(ptlm_handle* h, int32_t reps, double* h_ms, double* h_scale, int32_t* h_transform,
                          void* stream) {
  PTLM_CHECK_H(h);
  if (reps < 1) return fail(PTLM_EINVAL, "reps must be >= 1");
  if (h->in_batch) return fail(PTLM_EINVAL, "ptlm_autotune: the handle belongs to a batch (its launch shape is fixed)");
  return autotune_impl(h, reps, h_ms, h_scale, h_transform, (hipStream_t)stream);
}

const char* ptlm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
