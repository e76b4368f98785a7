// Host driver of the truncated LM iteration (alg:lm_inexact).
//
// One outer iteration: linearise (f, g, weighted phasors, D), then attempts.
// Each attempt is a fixed launch sequence -- lambda/eta, PCG start, cg_max
// predicated PCG iterations, trial point, trial loss, gain ratio and damping
// update -- followed by one stream synchronisation to read the acceptance flag.
// All scalars of the method live in FP64 in the device state.
#include <cmath>
#include <cstring>

#include "api_internal.hpp"
#include "lm_internal.hpp"

namespace ptlm {

static LMArgs make_args(ptlm_handle* h, const ptlm_lm_params* prm, ptlm_lm_state* st, const float2* O,
                        const float2* P, const float* learned) {
  Plan& p = h->plan;
  auto at = [&](size_t o) { return (float2*)(h->ws + o); };
  LMArgs a{};
  a.g = at(p.off.g);
  a.dx = at(p.off.dx);
  a.prev = at(p.off.prev);
  a.r = at(p.off.r);
  a.z = at(p.off.z);
  a.p = at(p.off.p);
  a.Ap = at(p.off.Ap);
  a.ztrial = at(p.off.ztrial);
  a.diag = at(p.off.diag);
  a.learned = (const float2*)learned;
  a.O = O;
  a.P = P;
  a.n = p.nvec;
  a.nobj = (size_t)p.d.ny * p.d.nx;
  a.st = st;
  a.prm = *prm;
  a.partials = h->g.partials;
  a.scal = (double*)(h->ws + p.off.scal);
  a.use_warm = 0;
  return a;
}

#define LM_HIP(call, where)                           \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

static ptlm_status check_params(const ptlm_lm_params* p) {
  if (!p) return fail(PTLM_EINVAL, "params is null");
  if (!(p->mu0 > 0) || !(p->mu_min > 0) || !(p->kappa > 1) || !(p->nu >= 0) || !(p->rho_min > 0) ||
      !(p->beta > 0) || !(p->diag_floor >= 0) || p->cg_max < 0 || p->retry_max < 1 ||
      (p->scaling != 0 && p->scaling != 1) || p->precond < 0 || p->precond > 2)
    return fail(PTLM_EINVAL, "invalid LM parameters");
  return PTLM_OK;
}

// One GGN-vector product with the damping term lambda D read from the device state.
static ptlm_status ggnv_lm(ptlm_handle* h, const LMArgs& a, const float2* v, float2* out, const int* pred,
                           hipStream_t s) {
  const size_t N = a.nobj;
  const float* dO = a.prm.scaling ? (const float*)a.diag : nullptr;
  const float* dP = a.prm.scaling ? (const float*)(a.diag + N) : nullptr;
  return ggnv_impl(h, v, h->g.joint ? v + N : nullptr, 0.0, &a.st->lambda, dO, dP, out,
                   h->g.joint ? out + N : nullptr, pred, s);
}

static ptlm_status lm_step_impl(ptlm_handle* h, float2* O, float2* P, const float* y, const ptlm_lm_params* prm,
                                ptlm_lm_state* st, const float* learned, hipStream_t s) {
  Geometry& g = h->g;
  LMArgs a = make_args(h, prm, st, O, P, learned);
  const size_t N = a.nobj, M = (size_t)g.my * g.mx;
  // ---- linearisation of the outer iteration (reused by every retry)
  ptlm_status stt = linearize_impl(h, O, P, y, a.scal + SC_F, a.g, g.joint ? a.g + N : nullptr, s);
  if (stt != PTLM_OK) return stt;
  LM_HIP(launch_vec(V_GNORM, a, s), "lm gnorm");
  LM_HIP(launch_fin(F_LIN, a, LM_BLOCKS, s), "lm lin");
  if (prm->scaling == 1 || prm->precond == 1) {
    LM_HIP(launch_diag_paper(g, (float*)a.diag, g.joint ? (float*)(a.diag + N) : nullptr, s), "lm diag");
    LM_HIP(launch_vec(V_DIAGMAX, a, s), "lm diag max");
    LM_HIP(launch_fin(F_DIAGMAX, a, LM_BLOCKS, s), "lm diag max fin");
    LM_HIP(launch_vec(V_DIAGFLOOR, a, s), "lm diag floor");
  }
  if (prm->precond == 2 && h->cnn_params) {
    float2* lbuf = (float2*)(h->ws + h->plan.off.learned);
    stt = learned_from_cnn(h, (float*)lbuf, s);
    if (stt != PTLM_OK) return stt;
    a.learned = lbuf;
  }
  ptlm_lm_state hs;
  LM_HIP(hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, s), "lm read state");
  LM_HIP(hipStreamSynchronize(s), "lm sync");
  if (hs.nonfinite) {
    LM_HIP(launch_fin(F_STEP_END, a, 0, s), "lm step end");
    return fail(PTLM_ENUMERIC, "non-finite loss or gradient at the current iterate");
  }

  bool accepted = false;
  for (int retry = 0; retry < prm->retry_max && !accepted; ++retry) {
    a.use_warm = (prm->warm_start && retry == 0 && h->prev_valid) ? 1 : 0;
    LM_HIP(launch_fin(F_BEGIN, a, 0, s), "lm begin");
    if (a.use_warm) {
      stt = ggnv_lm(h, a, a.prev, a.Ap, nullptr, s);
      if (stt != PTLM_OK) return stt;
    }
    LM_HIP(launch_vec(V_CG_INIT, a, s), "cg init");
    LM_HIP(launch_fin(F_CG_INIT, a, LM_BLOCKS, s), "cg init fin");
    for (int i = 0; i < prm->cg_max; ++i) {
      stt = ggnv_lm(h, a, a.p, a.Ap, &st->cg_active, s);
      if (stt != PTLM_OK) return stt;
      LM_HIP(launch_vec(V_PAP, a, s), "cg pap");
      LM_HIP(launch_fin(F_PAP, a, LM_BLOCKS, s), "cg pap fin");
      LM_HIP(launch_vec(V_CG_UPDATE, a, s), "cg update");
      LM_HIP(launch_fin(F_CG_UPDATE, a, LM_BLOCKS, s), "cg update fin");
      LM_HIP(launch_vec(V_PUPDATE, a, s), "cg p");
    }
    // ---- trial point z + Delta, predicted and actual reductions, rho, mu
    LM_HIP(launch_vec(V_TRIAL, a, s), "lm trial");
    LM_HIP(launch_fin(F_PRED, a, LM_BLOCKS, s), "lm pred");
    TileArgs ta{};
    ta.O = a.ztrial;
    ta.P = g.joint ? a.ztrial + N : P;
    ta.y = y;
    LM_HIP(launch_tile(g, OP_LOSS, ta, s), "lm trial loss");
    LM_HIP(launch_fin(F_TRIAL_END, a, g.grid, s), "lm trial end");
    LM_HIP(hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, s), "lm read state");
    LM_HIP(hipStreamSynchronize(s), "lm sync");
    if (hs.accepted) {
      accepted = true;
      LM_HIP(hipMemcpyAsync(O, a.ztrial, N * sizeof(float2), hipMemcpyDeviceToDevice, s), "lm accept O");
      if (g.joint)
        LM_HIP(hipMemcpyAsync(P, a.ztrial + N, M * sizeof(float2), hipMemcpyDeviceToDevice, s), "lm accept P");
      LM_HIP(hipMemcpyAsync(a.prev, a.dx, a.n * sizeof(float2), hipMemcpyDeviceToDevice, s), "lm keep step");
      h->prev_valid = true;
    }
  }
  LM_HIP(launch_fin(F_STEP_END, a, 0, s), "lm step end");
  if (!accepted) return fail(PTLM_ENOTACCEPTED, "every retry of this outer iteration was rejected");
  return PTLM_OK;
}

}  // namespace ptlm

using namespace ptlm;

extern "C" {

ptlm_status ptlm_lm_init(ptlm_handle* h, const ptlm_lm_params* params, ptlm_lm_state* d_state, void* stream) {
  if (!h || !d_state) return fail(PTLM_EINVAL, "null handle or state");
  ptlm_status st = check_params(params);
  if (st != PTLM_OK) return st;
  LMArgs a = make_args(h, params, d_state, nullptr, nullptr, nullptr);
  h->prev_valid = false;
  LM_HIP(launch_fin(F_INIT, a, 0, (hipStream_t)stream), "lm init");
  return PTLM_OK;
}

ptlm_status ptlm_lm_step(ptlm_handle* h, float* d_O, float* d_P, const float* d_y, const ptlm_lm_params* params,
                         ptlm_lm_state* d_state, const float* d_precond, void* stream) {
  if (!h || !d_O || !d_P || !d_y || !d_state) return fail(PTLM_EINVAL, "null argument");
  ptlm_status st = check_params(params);
  if (st != PTLM_OK) return st;
  if (params->precond == 2 && !d_precond && !h->cnn_params)
    return fail(PTLM_EINVAL, "precond == 2 needs d_precond or a registered network");
  return lm_step_impl(h, (float2*)d_O, (float2*)d_P, d_y, params, d_state, d_precond, (hipStream_t)stream);
}

ptlm_status ptlm_lm_solve(ptlm_handle* h, float* d_O, float* d_P, const float* d_y, const ptlm_lm_params* params,
                          int32_t T, ptlm_lm_state* d_state, const float* d_precond, void* stream) {
  if (T < 0) return fail(PTLM_EINVAL, "T must be >= 0");
  ptlm_status last = PTLM_OK;
  for (int t = 0; t < T; ++t) {
    last = ptlm_lm_step(h, d_O, d_P, d_y, params, d_state, d_precond, stream);
    if (last != PTLM_OK && last != PTLM_ENOTACCEPTED) return last;
  }
  return last;
}

}  // extern "C"
