// Internal declarations of the LM / PCG kernels.
#pragma once
#include <cstddef>

#include "ptlm.h"
#include "internal.hpp"

namespace ptlm {

// blocks of the vector kernels of a problem with n complex entries per vector (a function of
// the problem alone, so a problem gets the same partial sums alone and in a batch)
inline int lm_vec_blocks(size_t n) {
  const size_t b = (n + 1023) / 1024;
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

// indices into the FP64 scalar scratch
enum { SC_F = 0, SC_L1SQ = 1, SC_DMAX_O = 2, SC_DMAX_P = 3, SC_XMAX_O = 5, SC_XMAX_P = 6,
       SC_LS1 = 13, SC_G2_O = 16, SC_G2_P = 17, SC_RZ = 18 /* and 19 */ };

enum VecOp : int { V_GNORM, V_DIAGFLOOR, V_CG_INIT, V_CG_STEP, V_P_STEP, V_TRIAL, V_XMAX, V_XFLOOR,
                   V_PROJ, V_LS_DIR, V_LS_NEG, V_LS_CAND, V_WARM_P, V_SAME, V_LEARNED, V_GNORM_DMAX };
enum FinOp : int { F_ATTEMPT, F_LIN, F_XMAX, F_BEGIN, F_CG_INIT, F_PRED, F_TRIAL_END, F_INIT, F_ADOPT,
                   F_PJ_CHECK, F_LS_DIR, F_LS_NEG, F_LS_TEST, F_LIN_DMAX };

// Device flags of the LM state that predicate a launch (int32 index into the state; -1: none).
enum LMFlag : int {
  FL_NONE = -1,
  FL_LIN = (int)(offsetof(ptlm_lm_state, lin_now) / 4),
  FL_ALIVE = (int)(offsetof(ptlm_lm_state, alive) / 4),
  FL_CG = (int)(offsetof(ptlm_lm_state, cg_active) / 4),
  FL_WARM = (int)(offsetof(ptlm_lm_state, use_warm) / 4),
  FL_ACCEPTED = (int)(offsetof(ptlm_lm_state, accepted) / 4),
  FL_ACC_O = (int)(offsetof(ptlm_lm_state, acc_o) / 4),
  FL_ACC_P = (int)(offsetof(ptlm_lm_state, acc_p) / 4),
  FL_TILE = (int)(offsetof(ptlm_lm_state, tile_now) / 4),
  FL_LS_DIR = (int)(offsetof(ptlm_lm_state, ls_dir) / 4),
  FL_LS_NEG = (int)(offsetof(ptlm_lm_state, ls_neg) / 4),
  FL_LS_ON = (int)(offsetof(ptlm_lm_state, ls_on) / 4),
  FL_LS_TAKE = (int)(offsetof(ptlm_lm_state, ls_take) / 4),
  FL_LS_KEEP = (int)(offsetof(ptlm_lm_state, ls_keep) / 4),
};

struct LMArgs {
  float2 *g, *dx, *prev, *r, *z, *p, *Ap, *ztrial;
  float2* diag;            // (Re, Im) weights of Dg(G) per complex entry, floored
  const float2* learned;   // learned (2), exact (3) or estimated (4) diagonal standing for Dg(G)
  float2* xdiag;           // exact / estimated diagonal buffer (precond 3, 4; floored in place)
  const float2 *O, *P;     // current iterate
  const float2 *Olin, *Plin;  // linearisation point z_t (projected plug-in)
  size_t n, nobj;          // complex entries of a vector / of its object part
  size_t nprobe;           // complex entries of the probe
  ptlm_lm_state* st;
  ptlm_lm_params prm;
  double* partials;        // >= max(vec_blocks, pap_count) * 4
  double* scal;
  int vec_blocks;          // blocks of the vector kernels (lm_vec_blocks(n))
  int pap_count;           // parts of p.Ap a PCG product leaves in column 0 of partials
  int tile_grid;           // workgroups of the tile kernels (partials of the trial loss)
  int t_max;               // outer iterations to run (ptlm_lm_init / batch binding)
  int* cg_flags;           // nullable, pinned host memory: slot j <- whether PCG iteration j runs
  int* ls_flags;           // nullable, pinned host memory: slot i <- whether the line search goes
                           // on after step size i
  const float2* Pcur;      // the caller's probe (V_SAME, object-only problems)
  const float* cnn_r;      // network output r (2 maps of the object grid) for V_LEARNED
  int adopt_ok;            // host: the linearisation buffers hold the one made at the last accepted
                           // trial point, unless O / P changed since (checked by V_SAME / F_ADOPT)
};

// One problem's part of a batched LM launch.
struct LMJob {
  LMArgs a;
  int block0;
};

// iter: the PCG iteration of V_CG_STEP / V_P_STEP (selects the r.z parity slot)
hipError_t launch_vec(int op, const LMArgs& a, int flag, hipStream_t s, int iter = 0);
hipError_t launch_fin(int op, const LMArgs& a, int count, int flag, hipStream_t s);
// batched: vector kernels over the blocks of every job; finalize kernels one block per job,
// reducing count_kind = 0 (none), 1 (the job's vector partials) or 2 (its tile partials)
hipError_t launch_vec_batch(int op, const LMJob* jobs, const int* job_of_block, int nblocks, int flag, hipStream_t s,
                            int iter = 0);
hipError_t launch_fin_batch(int op, const LMJob* jobs, int njobs, int count_kind, int flag, hipStream_t s);

}  // namespace ptlm
