// Internal declarations of the LM / PCG kernels.
#pragma once
#include "ptlm.h"
#include "internal.hpp"

namespace ptlm {

constexpr int LM_BLOCKS = 1024;  // blocks of the vector kernels (partials per call)

// indices into the FP64 scalar scratch
enum { SC_F = 0, SC_L1SQ = 1, SC_DMAX_O = 2, SC_DMAX_P = 3, SC_FTRIAL = 4 };

enum VecOp : int { V_GNORM, V_DIAGMAX, V_DIAGFLOOR, V_CG_INIT, V_PAP, V_CG_UPDATE, V_PUPDATE, V_TRIAL };
enum FinOp : int { F_LIN, F_DIAGMAX, F_BEGIN, F_CG_INIT, F_PAP, F_CG_UPDATE, F_PRED, F_TRIAL_END, F_STEP_END, F_INIT };

struct LMArgs {
  float2 *g, *dx, *prev, *r, *z, *p, *Ap, *ztrial;
  float2* diag;            // (Re, Im) weights of Dg(G) per complex entry, floored
  const float2* learned;   // caller preconditioner diagonal (precond == 2)
  const float2 *O, *P;     // current iterate
  size_t n, nobj;          // complex entries of a vector / of its object part
  ptlm_lm_state* st;
  ptlm_lm_params prm;
  double* partials;        // >= LM_BLOCKS * 4
  double* scal;
  int use_warm;
};

hipError_t launch_vec(int op, const LMArgs& a, hipStream_t s);
hipError_t launch_fin(int op, const LMArgs& a, int count, hipStream_t s);

}  // namespace ptlm
