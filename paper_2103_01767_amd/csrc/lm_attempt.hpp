// One LM attempt (alg:lm_inexact) as a fixed launch sequence, shared by the single-problem
// driver (direct launches with one problem's arguments) and the batched driver (one launch
// per step for every problem of a batch, from job tables in device memory).  Every launch is
// predicated on a flag of the device LM state, so the same sequence serves the first attempt
// of an outer iteration (which linearises) and its retries (which reuse the linearisation of
// z_t, since a rejected step leaves z_t unchanged), and the host never has to look at the
// state in between.
#pragma once
#include "lm_internal.hpp"

namespace ptlm {

// which direction / output a GGN-vector product of the attempt uses
enum GgnWhich : int { GG_WARM = 0, GG_P = 1 };

#define PTLM_TRY(x)                              \
  do {                                           \
    const ptlm_status st_ = (x);                 \
    if (st_ != PTLM_OK) return st_;              \
  } while (0)

// Ops provides: fin(op, count_kind, flag), vec(op, flag), copy_lin(), linearize(),
// diag_paper(), learned(), exact_diag(), stoch_diag(), ggnv(which), trial_loss(), trial_finish(),
// copy_accept(), trial_loss_if(flag) (loss at the trial buffer, predicated on a state flag),
// copy_plugin() (the iterate from the trial buffer or from z_t, by the plug-in's outcome),
// cg_mark(j) (after the launch that decides whether PCG iteration j runs) and
// cg_gate(i, &go) (before PCG iteration i is enqueued; go = false ends the enqueueing, every
// later iteration being predicated off anyway), and ls_mark(i) / ls_gate(i, &go), the same for
// the step sizes of the projected plug-in's line search.
// ggnv(GG_WARM) multiplies the last accepted step, or p when params.alternate is set.
template <class Ops>
ptlm_status enqueue_attempt(Ops& o, const ptlm_lm_params& prm) {
  PTLM_TRY(o.fin(F_ATTEMPT, 0, FL_NONE));
  // ---- linearisation at z_t (only after an accepted step or at the start)
  PTLM_TRY(o.copy_lin());
  PTLM_TRY(o.linearize());  // f, ||grad_zeta ell||^2, g, phasor field, traces
  if (prm.scaling == 1 || prm.precond == 1 || prm.precond == 2) {
    // App. B diagonal; ||g||^2 and the diagonal's block maxima in one pass; then its floor
    // (diag_floor x block maximum)
    PTLM_TRY(o.diag_paper());
    PTLM_TRY(o.vec(V_GNORM_DMAX, FL_LIN));
    PTLM_TRY(o.fin(F_LIN_DMAX, 1, FL_LIN));
    PTLM_TRY(o.vec(V_DIAGFLOOR, FL_LIN));
  } else {
    PTLM_TRY(o.vec(V_GNORM, FL_LIN));
    PTLM_TRY(o.fin(F_LIN, 1, FL_LIN));
  }
  if (prm.precond == 2) PTLM_TRY(o.learned());
  if (prm.precond == 3 || prm.precond == 4) {
    // exact Dg(G) or its stochastic estimate in place of the App. B one, floored alike
    if (prm.precond == 3) PTLM_TRY(o.exact_diag());
    else PTLM_TRY(o.stoch_diag());
    PTLM_TRY(o.vec(V_XMAX, FL_LIN));
    PTLM_TRY(o.fin(F_XMAX, 1, FL_LIN));
    PTLM_TRY(o.vec(V_XFLOOR, FL_LIN));
  }
  // ---- lambda, eta, PCG on (G + lambda D) Delta = -g
  PTLM_TRY(o.fin(F_BEGIN, 0, FL_ALIVE));
  // A Delta_0 for the warm start; the alternating update multiplies the last step of the
  // active block alone, staged in p (free until V_CG_INIT)
  if (prm.alternate) PTLM_TRY(o.vec(V_WARM_P, FL_WARM));
  PTLM_TRY(o.ggnv(GG_WARM));
  PTLM_TRY(o.vec(V_CG_INIT, FL_ALIVE));
  PTLM_TRY(o.fin(F_CG_INIT, 1, FL_ALIVE));
  PTLM_TRY(o.cg_mark(0));
  for (int i = 0; i < prm.cg_max; ++i) {
    bool go = true;
    PTLM_TRY(o.cg_gate(i, &go));
    if (!go) break;
    PTLM_TRY(o.ggnv(GG_P));                // A p, and the parts of p^T A p
    PTLM_TRY(o.vec(V_CG_STEP, FL_CG, i));  // alpha; Delta, r, z and the r.z, r.r partials
    PTLM_TRY(o.vec(V_P_STEP, FL_CG, i));   // beta, stopping test; p = z + beta p
    PTLM_TRY(o.cg_mark(i + 1));
  }
  // ---- trial point, predicted and actual reductions, gain ratio, damping, acceptance
  PTLM_TRY(o.vec(V_TRIAL, FL_ALIVE));
  PTLM_TRY(o.fin(F_PRED, 1, FL_ALIVE));
  PTLM_TRY(o.trial_loss());
  PTLM_TRY(o.fin(F_TRIAL_END, 2, FL_ALIVE));
  PTLM_TRY(o.trial_finish());  // gradient and sums of a trial evaluated as a linearisation
  PTLM_TRY(o.copy_accept());
  // ---- alg:projected_LM plug-in after an accepted step, decided on the device
  if (prm.project) {
    PTLM_TRY(o.vec(V_PROJ, FL_ACCEPTED));  // trial buffer <- Pi(z_t + Delta)
    PTLM_TRY(o.trial_loss_if(FL_ACCEPTED));
    PTLM_TRY(o.fin(F_PJ_CHECK, 2, FL_ACCEPTED));
    PTLM_TRY(o.vec(V_LS_DIR, FL_LS_DIR));  // s = Pi(z_t + Delta) - z_t, g.s, ||s||^2
    PTLM_TRY(o.fin(F_LS_DIR, 1, FL_LS_DIR));
    PTLM_TRY(o.vec(V_LS_NEG, FL_LS_NEG));  // s = -grad f
    PTLM_TRY(o.fin(F_LS_NEG, 1, FL_LS_NEG));
    for (int i = 0; i < prm.ls_max; ++i) {
      bool go = true;
      PTLM_TRY(o.ls_gate(i, &go));
      if (!go) break;
      PTLM_TRY(o.vec(V_LS_CAND, FL_LS_ON));  // trial buffer <- z_t + alpha s (projected)
      PTLM_TRY(o.trial_loss_if(FL_LS_ON));
      PTLM_TRY(o.fin(F_LS_TEST, 2, FL_LS_ON));
      PTLM_TRY(o.ls_mark(i));
    }
    PTLM_TRY(o.copy_plugin());
  }
  return PTLM_OK;
}

}  // namespace ptlm
