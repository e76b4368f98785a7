// Host driver of the truncated LM iteration (alg:lm_inexact) for one problem.
//
// An outer iteration is a sequence of attempts; each attempt is the launch sequence of
// lm_attempt.hpp (linearise when the previous attempt was accepted, unless the linearisation
// made at the accepted trial point is adopted; lambda/eta, PCG start, predicated PCG
// iterations enqueued one ahead of the device's stopping decision; trial point and its loss,
// gain ratio and damping update, accept copies), followed by one stream synchronisation to
// read the device state.  All scalars of the method live in FP64 in the device state.
#include <climits>
#include <cmath>
#include <cstring>
#include <utility>

#include "api_internal.hpp"
#include "lm_attempt.hpp"

namespace ptlm {

LMArgs make_lm_args(ptlm_handle* h, const ptlm_lm_params* prm, ptlm_lm_state* st, const float2* O,
                    const float2* P, const float* learned) {
  Plan& p = h->plan;
  auto at = [&](size_t o) { return (float2*)(h->ws + o); };
  LMArgs a{};
  a.g = h->lm_g;
  a.dx = at(p.off.dx);
  a.prev = at(p.off.prev);
  a.r = at(p.off.r);
  a.z = at(p.off.z);
  a.p = at(p.off.p);
  a.Ap = at(p.off.Ap);
  a.ztrial = at(p.off.ztrial);
  a.diag = at(p.off.diag);
  a.xdiag = at(p.off.learned);
  a.learned = prm && (prm->precond == 3 || prm->precond == 4) ? a.xdiag : (const float2*)learned;
  a.O = O;
  a.P = P;
  a.Olin = h->g.O_lin;
  a.Plin = h->g.P_lin;
  a.n = p.nvec;
  a.nobj = (size_t)p.d.ny * p.d.nx;
  a.nprobe = (size_t)p.d.my * p.d.mx;
  a.st = st;
  if (prm) a.prm = *prm;
  a.partials = h->g.partials;
  a.scal = (double*)(h->ws + p.off.scal);
  a.vec_blocks = lm_vec_blocks(a.n);
  a.pap_count = reduce_pair_blocks(h->g, h->g.joint);
  a.tile_grid = h->g.grid;
  a.t_max = INT_MAX;
  return a;
}

#define LM_HIP(call, where)                           \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

ptlm_status check_lm_params(const ptlm_lm_params* p) {
  if (!p) return fail(PTLM_EINVAL, "params is null");
  if (!(p->mu0 > 0) || !(p->mu_min > 0) || !(p->kappa > 1) || !(p->nu >= 0) || !(p->rho_min > 0) ||
      !(p->beta > 0) || !(p->diag_floor >= 0) || p->cg_max < 0 || p->retry_max < 1 ||
      (p->scaling != 0 && p->scaling != 1) || p->precond < 0 || p->precond > 4 ||
      (p->precond == 4 && p->stoch_samples < 1) || p->surrogate_T < 0 ||
      !(p->surrogate_s0 >= 0.0) || !std::isfinite(p->surrogate_s0) || (p->project != 0 && p->project != 1) ||
      (p->project && (p->ls_max < 0 || !(p->o_max > 0) || !(p->p_max > 0) || !(p->sigma_ls >= 0) ||
                      !(p->gamma >= 0) || !(p->tau_s >= 0) || !(p->p_s > 1))) ||
      (p->alternate != 0 && p->alternate != 1))
    return fail(PTLM_EINVAL, "invalid LM parameters");
  return PTLM_OK;
}

// Launches of one attempt for a single problem, with its arguments passed directly.
struct SingleOps {
  ptlm_handle* h;
  LMArgs a;
  float2* O;
  float2* P;
  const float* y;
  const float* user_learned;  // caller's learned diagonal (precond 2 without a network)
  bool lin_expected;          // host view: this attempt linearises (network refresh)
  hipStream_t s;
  bool spec = false;          // the trial point is evaluated as a linearisation (spare buffers)

  int* flag(int f) const { return reinterpret_cast<int*>(a.st) + f; }

  ptlm_status fin(int op, int kind, int fl) {
    const int count = kind == 1 ? a.vec_blocks : (kind == 2 ? a.tile_grid : 0);
    LM_HIP(launch_fin(op, a, count, fl, s), "lm finalize");
    return PTLM_OK;
  }
  ptlm_status vec(int op, int fl, int iter = 0) {
    LM_HIP(launch_vec(op, a, fl, s, iter), "lm vector");
    return PTLM_OK;
  }
  ptlm_status copy_lin() {
    Geometry& g = h->g;
    if (a.adopt_ok) {  // adopt the kept linearisation only if the iterate is the point it was made at
      LM_HIP(launch_vec(V_SAME, a, FL_LIN, s), "lm same point");
      LM_HIP(launch_fin(F_ADOPT, a, a.vec_blocks, FL_LIN, s), "lm adopt");
    }
    const CopyItem c[2] = {{O, g.O_lin, (size_t)g.ny * g.nx, flag(FL_LIN)},
                           {P, g.P_lin, (size_t)g.my * g.mx, flag(FL_LIN)}};
    LM_HIP(launch_copies(c, 2, s), "lm copy O, P");
    return PTLM_OK;
  }
  ptlm_status linearize() {
    Geometry& g = h->g;
    TileArgs ta{};
    ta.O = g.O_lin;
    ta.P = g.P_lin;
    ta.y = y;
    ta.predicate = flag(FL_TILE);
    ta.bg_add = &a.st->sigma;
    LM_HIP(launch_tile(g, OP_LINEARIZE, ta, s), "lm linearize");
    LM_HIP(launch_refine(g, ta, s), "lm linearize refine");
    LM_HIP(launch_sum_partials(g.partials, g.grid, a.scal + SC_F, 2, s, flag(FL_TILE)), "lm linearize sum");
    LM_HIP(launch_reduce_pair(g, a.g, g.joint ? a.g + a.nobj : nullptr, 0.0, nullptr, nullptr, nullptr, nullptr, nullptr,
                              flag(FL_TILE), s),
           "lm gradient");
    return PTLM_OK;
  }
  // geometry whose linearisation buffers are the spares (the trial's linearisation)
  Geometry spare_geometry() const {
    Geometry gs = h->g;
    gs.afield = h->afield_alt;
    gs.w2 = h->w2_alt;
    gs.trace = h->trace_alt;
    return gs;
  }
  ptlm_status diag_paper() {
    Geometry& g = h->g;
    LM_HIP(launch_diag_paper(g, (float*)a.diag, g.joint ? (float*)(a.diag + a.nobj) : nullptr, s, flag(FL_LIN)),
           "lm diag");
    return PTLM_OK;
  }
  ptlm_status learned() {
    if (h->cnn_params) {
      if (lin_expected) {
        // the network runs every cnn_every-th linearisation (0: only the first)
        const bool due = h->cnn_every > 0 ? (h->cnn_count % h->cnn_every == 0) : !h->cnn_ready;
        h->cnn_count += 1;
        if (due || !h->cnn_ready) PTLM_TRY(cnn_refresh(h, s));
      }
      // the learned diagonal is rebuilt from the kept output and the new floored App. B
      // diagonal at every linearisation
      a.cnn_r = cnn_output(h);
      LM_HIP(launch_vec(V_LEARNED, a, FL_LIN, s), "lm learned diagonal");
      a.learned = a.xdiag;
    } else {
      a.learned = (const float2*)user_learned;
    }
    return PTLM_OK;
  }
  ptlm_status exact_diag() {
    return diag_exact_impl(h, (float*)a.xdiag, h->g.joint ? (float*)(a.xdiag + a.nobj) : nullptr, s, flag(FL_LIN));
  }
  ptlm_status stoch_diag() {
    return diag_stochastic_impl(h, a.prm.stoch_samples, a.prm.stoch_seed, 0, &a.st->t, (float*)a.xdiag,
                                h->g.joint ? (float*)(a.xdiag + a.nobj) : nullptr, s, flag(FL_LIN));
  }
  ptlm_status ggnv(int which) {
    const float2* v = (which == GG_WARM && !a.prm.alternate) ? a.prev : a.p;
    const int* pred = which == GG_WARM ? flag(FL_WARM) : flag(FL_CG);
    const size_t N = a.nobj;
    const float* dO = a.prm.scaling ? (const float*)a.diag : nullptr;
    const float* dP = a.prm.scaling ? (const float*)(a.diag + N) : nullptr;
    // a PCG product leaves the parts of p.Ap for the step that follows it
    const bool pcg = which == GG_P;
    return ggnv_impl(h, v, h->g.joint ? v + N : nullptr, 0.0, &a.st->lambda, dO, dP, a.Ap,
                     h->g.joint ? a.Ap + N : nullptr, pred, s, 3, pcg ? a.partials : nullptr,
                     pcg && a.prm.alternate ? &a.st->block : nullptr);
  }
  ptlm_status trial_loss() {
    Geometry& g = h->g;
    TileArgs ta{};
    ta.O = a.ztrial;
    ta.P = g.joint ? a.ztrial + a.nobj : P;
    ta.y = y;
    ta.predicate = flag(FL_ALIVE);
    ta.bg_add = &a.st->sigma;
    // the loss partials of a linearisation are those of the loss, so F_TRIAL_END reads either
    if (spec) {
      const Geometry gs = spare_geometry();
      LM_HIP(launch_tile(gs, OP_LINEARIZE, ta, s), "lm trial linearize");
      LM_HIP(launch_refine(gs, ta, s), "lm trial refine");
    } else {
      LM_HIP(launch_tile(g, OP_LOSS, ta, s), "lm trial loss");
    }
    return PTLM_OK;
  }
  // after an accepted trial evaluated as a linearisation: its f and ||ell'||^2 for F_LIN of the
  // next outer iteration, and its gradient into the spare gradient buffer
  ptlm_status trial_finish() {
    if (!spec) return PTLM_OK;
    const Geometry gs = spare_geometry();
    LM_HIP(launch_sum_partials(gs.partials, gs.grid, a.scal + SC_F, 2, s, flag(FL_ACCEPTED)), "lm trial sums");
    LM_HIP(launch_reduce_pair(gs, h->lm_g_alt, gs.joint ? h->lm_g_alt + a.nobj : nullptr, 0.0, nullptr, nullptr, nullptr,
                              nullptr, nullptr, flag(FL_ACCEPTED), s),
           "lm trial gradient");
    return PTLM_OK;
  }
  // PCG look-ahead: iteration i is enqueued once the decision on iteration i - 1 is known
  // (the GPU is then still busy with iteration i - 1), so at most one iteration past the
  // end of the solve is launched, predicated off.  Without pinned slots every iteration is
  // enqueued.
  ptlm_status cg_mark(int j) {
    if (!a.cg_flags) return PTLM_OK;
    LM_HIP(hipEventRecord(h->cg_events[j], s), "lm pcg mark");
    return PTLM_OK;
  }
  ptlm_status cg_gate(int i, bool* go) {
    *go = true;
    if (!a.cg_flags || i < 1) return PTLM_OK;
    LM_HIP(hipEventSynchronize(h->cg_events[i - 1]), "lm pcg gate");
    *go = __atomic_load_n(a.cg_flags + (i - 1), __ATOMIC_ACQUIRE) != 0;
    return PTLM_OK;
  }
  ptlm_status trial_loss_if(int fl) {
    TileArgs ta{};
    ta.O = a.ztrial;
    ta.P = h->g.joint ? a.ztrial + a.nobj : P;
    ta.y = y;
    ta.predicate = flag(fl);
    ta.bg_add = &a.st->sigma;
    LM_HIP(launch_tile(h->g, OP_LOSS, ta, s), "lm plug-in loss");
    return PTLM_OK;
  }
  ptlm_status copy_plugin() {
    Geometry& g = h->g;
    const size_t M = (size_t)g.my * g.mx;
    const CopyItem c[4] = {{a.ztrial, O, a.nobj, flag(FL_LS_TAKE)},
                           {g.O_lin, O, a.nobj, flag(FL_LS_KEEP)},
                           {a.ztrial + a.nobj, P, M, flag(FL_LS_TAKE)},
                           {g.P_lin, P, M, flag(FL_LS_KEEP)}};
    LM_HIP(launch_copies(c, g.joint ? 4 : 2, s), "lm plug-in copies");
    return PTLM_OK;
  }
  // line-search look-ahead: step size i is enqueued once the test of size i - 2 is known (the
  // GPU is then still busy with size i - 1), so at most two sizes past the end are launched,
  // predicated off.  The PCG events are free again here (that solve is fully enqueued).
  ptlm_status ls_mark(int i) {
    if (!a.ls_flags) return PTLM_OK;
    LM_HIP(hipEventRecord(h->cg_events[i], s), "lm line-search mark");
    return PTLM_OK;
  }
  ptlm_status ls_gate(int i, bool* go) {
    *go = true;
    if (!a.ls_flags || i < 2) return PTLM_OK;
    LM_HIP(hipEventSynchronize(h->cg_events[i - 2]), "lm line-search gate");
    *go = __atomic_load_n(a.ls_flags + (i - 2), __ATOMIC_ACQUIRE) != 0;
    return PTLM_OK;
  }
  ptlm_status copy_accept() {
    // the accepted step's blocks (both, or the active one of the alternating update)
    Geometry& g = h->g;
    const size_t M = (size_t)g.my * g.mx;
    const CopyItem c[4] = {{a.ztrial, O, a.nobj, flag(FL_ACC_O)},
                           {a.dx, a.prev, a.nobj, flag(FL_ACC_O)},
                           {a.ztrial + a.nobj, P, M, flag(FL_ACC_P)},
                           {a.dx + a.nobj, a.prev + a.nobj, M, flag(FL_ACC_P)}};
    LM_HIP(launch_copies(c, g.joint ? 4 : 2, s), "lm accept copies");
    return PTLM_OK;
  }
};

static ptlm_status read_state(ptlm_lm_state* d, ptlm_lm_state* hs, hipStream_t s) {
  LM_HIP(hipMemcpyAsync(hs, d, sizeof *hs, hipMemcpyDeviceToHost, s), "lm read state");
  LM_HIP(hipStreamSynchronize(s), "lm sync");
  return PTLM_OK;
}

// One outer iteration: the attempts of alg:lm_inexact until one is accepted or retry_max are
// rejected -- once for the joint update, once per block (object, then probe) for the
// alternating update of alg:alt_LM_ptycho.
// known: the device state as last read back (ptlm_lm_solve between its steps), else read here;
// the state read after the last attempt is left in *last when it is given.
static ptlm_status lm_step_impl(ptlm_handle* h, float2* O, float2* P, const float* y, const ptlm_lm_params* prm,
                                ptlm_lm_state* st, const float* learned, hipStream_t s,
                                const ptlm_lm_state* known = nullptr, ptlm_lm_state* last = nullptr) {
  ptlm_lm_state hs;
  if (known) hs = *known;
  else PTLM_TRY(read_state(st, &hs, s));
  struct Keep {
    ptlm_lm_state* to;
    const ptlm_lm_state* from;
    ~Keep() { if (to) *to = *from; }
  } keep{last, &hs};
  if (hs.status == PTLM_ENUMERIC) return fail(PTLM_ENUMERIC, "non-finite loss or gradient at the current iterate");
  if (hs.t >= hs.t_max) return fail(PTLM_EINVAL, "the state has run its outer iterations (t_max)");
  const int t0 = hs.t;
  SingleOps o{h, make_lm_args(h, prm, st, O, P, learned), O, P, y, learned, false, s};
  // PCG look-ahead when the handle has slots for every iteration (else all are enqueued)
  const bool ahead = h->cg_flags && prm->cg_max + 1 <= h->cg_slots;
  o.a.cg_flags = ahead ? h->cg_flags : nullptr;
  const bool ls_ahead = h->ls_flags && prm->project && prm->ls_max <= h->cg_slots;
  o.a.ls_flags = ls_ahead ? h->ls_flags : nullptr;
  // trial points are evaluated as linearisations (kept for the next outer iteration when the
  // step is accepted) unless the projected plug-in may move the iterate off the trial point
  o.spec = !prm->project;
  o.a.Pcur = h->g.joint ? nullptr : P;
  bool rejected = false;
  const int subs = prm->alternate ? 2 : 1;
  for (int sub = 0; sub < subs; ++sub) {
    bool ended = false;
    for (int attempt = 0; attempt <= prm->retry_max && !ended; ++attempt) {
      o.lin_expected = hs.need_lin != 0;
      o.a.adopt_ok = (o.spec && h->kept_gen == h->lin_gen && h->kept_y == y) ? 1 : 0;
      // no kernel of an earlier attempt is in flight (its state was read back)
      if (ahead)
        for (int j = 0; j <= prm->cg_max; ++j) __atomic_store_n(h->cg_flags + j, 0, __ATOMIC_RELAXED);
      if (ls_ahead)
        for (int j = 0; j < prm->ls_max; ++j) __atomic_store_n(h->ls_flags + j, 0, __ATOMIC_RELAXED);
      PTLM_TRY(enqueue_attempt(o, *prm));
      PTLM_TRY(read_state(st, &hs, s));
      if (o.spec && hs.accepted) {
        // the trial's linearisation becomes the current one (its point is the new iterate)
        std::swap(h->g.afield, h->afield_alt);
        std::swap(h->g.w2, h->w2_alt);
        std::swap(h->g.trace, h->trace_alt);
        std::swap(h->lm_g, h->lm_g_alt);
        o.a.g = h->lm_g;
        h->kept_gen = h->lin_gen;
        h->kept_y = y;
      }
      if (hs.status == PTLM_ENUMERIC) return fail(PTLM_ENUMERIC, "non-finite loss or gradient at the current iterate");
      ended = hs.iter_done != 0;
    }
    if (!ended) return fail(PTLM_EHIP, "LM attempt sequence did not end the outer iteration");
    rejected = rejected || hs.status == PTLM_ENOTACCEPTED;
  }
  if (hs.t != t0 + 1) return fail(PTLM_EHIP, "LM attempt sequence did not end the outer iteration");
  if (rejected) return fail(PTLM_ENOTACCEPTED, "every retry of this outer iteration (or of one sub-step) was rejected");
  return PTLM_OK;
}

}  // namespace ptlm

using namespace ptlm;

extern "C" {

ptlm_status ptlm_lm_init(ptlm_handle* h, const ptlm_lm_params* params, ptlm_lm_state* d_state, void* stream) {
  if (!h || !d_state) return fail(PTLM_EINVAL, "null handle or state");
  ptlm_status st = check_lm_params(params);
  if (st != PTLM_OK) return st;
  if (params->alternate && !h->g.joint) return fail(PTLM_EINVAL, "the alternating update needs a PTLM_JOINT problem");
  h->lin_gen += 1;  // a new run linearises afresh
  LMArgs a = make_lm_args(h, params, d_state, nullptr, nullptr, nullptr);
  LM_HIP(launch_fin(F_INIT, a, 0, FL_NONE, (hipStream_t)stream), "lm init");
  return PTLM_OK;
}

static ptlm_status check_step_args(ptlm_handle* h, float* d_O, float* d_P, const float* d_y,
                                   const ptlm_lm_params* params, ptlm_lm_state* d_state, const float* d_precond) {
  if (!h || !d_O || !d_P || !d_y || !d_state) return fail(PTLM_EINVAL, "null argument");
  ptlm_status st = check_lm_params(params);
  if (st != PTLM_OK) return st;
  if (params->alternate && !h->g.joint) return fail(PTLM_EINVAL, "the alternating update needs a PTLM_JOINT problem");
  if (params->precond == 2 && !d_precond && !h->cnn_params)
    return fail(PTLM_EINVAL, "precond == 2 needs d_precond or a registered network");
  return PTLM_OK;
}

ptlm_status ptlm_lm_step(ptlm_handle* h, float* d_O, float* d_P, const float* d_y, const ptlm_lm_params* params,
                         ptlm_lm_state* d_state, const float* d_precond, void* stream) {
  PTLM_TRY(check_step_args(h, d_O, d_P, d_y, params, d_state, d_precond));
  return lm_step_impl(h, (float2*)d_O, (float2*)d_P, d_y, params, d_state, d_precond, (hipStream_t)stream);
}

ptlm_status ptlm_lm_solve(ptlm_handle* h, float* d_O, float* d_P, const float* d_y, const ptlm_lm_params* params,
                          int32_t T, ptlm_lm_state* d_state, const float* d_precond, void* stream) {
  if (T < 0) return fail(PTLM_EINVAL, "T must be >= 0");
  PTLM_TRY(check_step_args(h, d_O, d_P, d_y, params, d_state, d_precond));
  ptlm_status last = PTLM_OK;
  ptlm_lm_state hs;
  bool known = false;  // hs holds the device state read back at the end of the previous step
  for (int t = 0; t < T; ++t) {
    last = lm_step_impl(h, (float2*)d_O, (float2*)d_P, d_y, params, d_state, d_precond, (hipStream_t)stream,
                        known ? &hs : nullptr, &hs);
    if (last != PTLM_OK && last != PTLM_ENOTACCEPTED) return last;
    known = true;
  }
  return last;
}

}  // extern "C"
