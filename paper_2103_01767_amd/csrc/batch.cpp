// Batched LM over many independent problems of uneven sizes.
//
// Each problem keeps its own plan, workspace region and device LM state (its handle works
// for every single-problem call).  An LM attempt of the whole batch is the launch sequence of
// lm_attempt.hpp with every step issued once for all problems: tile kernels once per probe
// shape present, reductions, vector and finalize kernels once in total, each block finding its
// problem in a job table in device memory.  A problem's blocks, partial sums and their order
// are those of the problem alone, so a problem's iterates in a batch equal its iterates when
// solved alone.  After one eager attempt the sequence is captured into a HIP graph and
// replayed, one graph launch per attempt; problems that finished their outer iterations (or
// met a non-finite value) are predicated off on the device.
#include <algorithm>
#include <climits>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "api_internal.hpp"
#include "lm_attempt.hpp"

namespace ptlm {
LMArgs make_lm_args(ptlm_handle* h, const ptlm_lm_params* prm, ptlm_lm_state* st, const float2* O,
                    const float2* P, const float* learned);
ptlm_status check_lm_params(const ptlm_lm_params* p);
}  // namespace ptlm

using namespace ptlm;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// TK_PJ / TK_LS: loss at the trial buffer for the projected plug-in (predicated on the
// acceptance / on the running line search)
enum TileKind { TK_LIN = 0, TK_WARM = 1, TK_P = 2, TK_TRIAL = 3, TK_PJ = 4, TK_LS = 5, TK_N = 6 };
enum RedKind { RK_LIN = 0, RK_WARM = 1, RK_P = 2, RK_DIAG = 3, RK_N = 4 };

// device table region of a batch (offsets from the start of the region)
struct TableLayout {
  size_t jb_tile_off[16];   // per shape class: int job_of_block[nb_tile]
  size_t tile_jobs_off[16][TK_N];
  size_t jb_obj, jb_prb, jb_prb1, jb_dprb, jb_vec, jb_copy_lin, jb_copy_acc;
  size_t red_obj[RK_N], red_prb[RK_N], red_sum;
  size_t lm_jobs, copy_lin, copy_acc, copy_take, copy_keep;
  size_t bytes;
};

struct ShapeClass {
  int my, mx;
  std::vector<int> probs;
  std::vector<int> block0;  // per member, within the class launch
  int nblocks = 0;
};

}  // namespace

struct ptlm_batch {
  int n = 0;
  std::vector<ptlm_handle*> hs;
  std::vector<size_t> ws_off;
  char* ws = nullptr;
  size_t tables_off = 0;
  TableLayout L{};
  std::vector<ShapeClass> classes;
  int nb_obj = 0, nb_prb = 0, nb_prb1 = 0, nb_dprb = 0, nb_vec = 0, nb_copy_lin = 0, nb_copy_acc = 0;
  std::vector<int> obj_b0, prb_b0, prb1_b0, dprb_b0, vec_b0;
  // host copies of the tables (kept alive for the asynchronous uploads)
  std::vector<std::vector<int>> jb_tile;
  std::vector<int> jb_obj, jb_prb, jb_prb1, jb_dprb, jb_vec, jb_copy_lin, jb_copy_acc;
  std::vector<std::vector<TileJob>> tile_jobs;  // [class * TK_N + kind]
  std::vector<RedJob> red_obj[RK_N], red_prb[RK_N], red_sum;
  std::vector<LMJob> lm_jobs;
  std::vector<CopyJob> copy_lin, copy_acc, copy_take, copy_keep;  // take / keep: block table of copy_lin
  // binding
  bool bound = false;
  ptlm_lm_params prm{};
  int T = 0;
  ptlm_lm_state* d_states = nullptr;
  std::vector<ptlm_lm_state> h_states;
  std::vector<const float2*> bound_P;  // the bound probes (learned-preconditioner refresh)
  int use_graph = 0;
  bool eager_done = false;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  template <class T>
  T* dev(size_t off) const {
    return reinterpret_cast<T*>(ws + tables_off + off);
  }
};

namespace {

#define B_HIP(call, where)                            \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// Block tables: runs of blocks per job, each run rounded up to a multiple of `unit`.
int append_run(std::vector<int>& jb, int job, int count, int unit) {
  const int padded = (count + unit - 1) / unit * unit;
  const int b0 = (int)jb.size();
  jb.insert(jb.end(), padded, job);
  return b0;
}

struct BatchOps {
  ptlm_batch* b;
  hipStream_t s;

  ptlm_status fin(int op, int kind, int fl) {
    B_HIP(launch_fin_batch(op, b->dev<LMJob>(b->L.lm_jobs), b->n, kind, fl, s), "batch finalize");
    return PTLM_OK;
  }
  ptlm_status vec(int op, int fl, int iter = 0) {
    B_HIP(launch_vec_batch(op, b->dev<LMJob>(b->L.lm_jobs), b->dev<int>(b->L.jb_vec), b->nb_vec, fl, s, iter),
          "batch vector");
    return PTLM_OK;
  }
  ptlm_status tiles(int op, int kind) {
    for (size_t c = 0; c < b->classes.size(); ++c) {
      const ShapeClass& C = b->classes[c];
      B_HIP(launch_tile_batch(C.my, C.mx, op, b->dev<TileJob>(b->L.tile_jobs_off[c][kind]),
                              b->dev<int>(b->L.jb_tile_off[c]), C.nblocks, s),
            "batch tile");
    }
    return PTLM_OK;
  }
  ptlm_status reduce(int kind) {
    B_HIP(launch_reduce_pair_batch(b->dev<RedJob>(b->L.red_obj[kind]), b->dev<int>(b->L.jb_obj), b->nb_obj,
                                   b->dev<RedJob>(b->L.red_prb[kind]), b->dev<int>(b->L.jb_prb1), b->nb_prb1,
                                   b->dev<int>(b->L.jb_prb), b->nb_prb, s),
          "batch reduce");
    return PTLM_OK;
  }
  ptlm_status copy_lin() {
    B_HIP(launch_copy_batch(b->dev<CopyJob>(b->L.copy_lin), b->dev<int>(b->L.jb_copy_lin), b->nb_copy_lin, s),
          "batch copy");
    return PTLM_OK;
  }
  ptlm_status linearize() {
    PTLM_TRY(tiles(OP_LINEARIZE, TK_LIN));
    // each problem's own refinement launch (as it has alone), where its weights call for one
    for (size_t c = 0; c < b->classes.size(); ++c)
      for (const TileJob& j : b->tile_jobs[c * TK_N + TK_LIN]) B_HIP(launch_refine(j.g, j.a, s), "batch refine");
    B_HIP(launch_sum_partials_batch(b->dev<RedJob>(b->L.red_sum), b->n, 2, s), "batch linearize sum");
    return reduce(RK_LIN);
  }
  ptlm_status diag_paper() {
    B_HIP(launch_diag_paper_batch(b->dev<RedJob>(b->L.red_obj[RK_DIAG]), b->dev<int>(b->L.jb_obj), b->nb_obj,
                                  b->dev<RedJob>(b->L.red_prb[RK_DIAG]), b->dev<int>(b->L.jb_dprb), b->nb_dprb, s),
          "batch diag");
    return PTLM_OK;
  }
  ptlm_status learned() {
    // every problem's learned diagonal from its network output (computed at bind from the
    // bound probe: once per reconstruction) and its new floored App. B diagonal
    return vec(V_LEARNED, FL_LIN);
  }
  // exact diagonal / its stochastic estimate: each problem's own launches (the single-problem
  // kernels on its handle, predicated on its linearisation flag), so a batch equals its
  // problems alone
  ptlm_status exact_diag() {
    for (int i = 0; i < b->n; ++i) {
      ptlm_handle* h = b->hs[i];
      const LMArgs& a = b->lm_jobs[i].a;
      const int* lin = reinterpret_cast<const int*>(b->d_states + i) + FL_LIN;
      PTLM_TRY(diag_exact_impl(h, (float*)a.xdiag, h->g.joint ? (float*)(a.xdiag + a.nobj) : nullptr, s, lin));
    }
    return PTLM_OK;
  }
  ptlm_status stoch_diag() {
    for (int i = 0; i < b->n; ++i) {
      ptlm_handle* h = b->hs[i];
      const LMArgs& a = b->lm_jobs[i].a;
      const int* lin = reinterpret_cast<const int*>(b->d_states + i) + FL_LIN;
      PTLM_TRY(diag_stochastic_impl(h, a.prm.stoch_samples, a.prm.stoch_seed, 0, &b->d_states[i].t, (float*)a.xdiag,
                                    h->g.joint ? (float*)(a.xdiag + a.nobj) : nullptr, s, lin));
    }
    return PTLM_OK;
  }
  ptlm_status ggnv(int which) {
    PTLM_TRY(tiles(OP_GGNV, which == GG_WARM ? TK_WARM : TK_P));
    return reduce(which == GG_WARM ? RK_WARM : RK_P);
  }
  ptlm_status trial_loss() { return tiles(OP_LOSS, TK_TRIAL); }
  ptlm_status trial_loss_if(int fl) { return tiles(OP_LOSS, fl == FL_ACCEPTED ? TK_PJ : TK_LS); }
  ptlm_status copy_plugin() {
    B_HIP(launch_copy_batch(b->dev<CopyJob>(b->L.copy_take), b->dev<int>(b->L.jb_copy_lin), b->nb_copy_lin, s),
          "batch plug-in take");
    B_HIP(launch_copy_batch(b->dev<CopyJob>(b->L.copy_keep), b->dev<int>(b->L.jb_copy_lin), b->nb_copy_lin, s),
          "batch plug-in keep");
    return PTLM_OK;
  }
  ptlm_status trial_finish() { return PTLM_OK; }  // batched trials are losses only
  // the batch keeps one fixed launch sequence (graph capture): every PCG iteration is enqueued
  ptlm_status cg_mark(int) { return PTLM_OK; }
  ptlm_status cg_gate(int, bool* go) {
    *go = true;
    return PTLM_OK;
  }
  ptlm_status ls_mark(int) { return PTLM_OK; }
  ptlm_status ls_gate(int, bool* go) {
    *go = true;
    return PTLM_OK;
  }
  ptlm_status copy_accept() {
    B_HIP(launch_copy_batch(b->dev<CopyJob>(b->L.copy_acc), b->dev<int>(b->L.jb_copy_acc), b->nb_copy_acc, s),
          "batch accept");
    return PTLM_OK;
  }
};

// plan the batch: per-problem workspaces, shape classes, block tables, table layout
ptlm_status plan_batch(int n, const ptlm_desc* descs, const int32_t* const* h_pos, ptlm_batch& b,
                       std::vector<Plan>& plans, size_t* total) {
  if (n < 1) return fail(PTLM_EINVAL, "a batch needs at least one problem");
  if (!descs || !h_pos) return fail(PTLM_EINVAL, "null descs or positions");
  plans.resize(n);
  size_t off = 0;
  b.ws_off.resize(n);
  for (int i = 0; i < n; ++i) {
    const ptlm_status st = make_plan(&descs[i], h_pos[i], plans[i]);
    if (st != PTLM_OK) return fail(st, "problem " + std::to_string(i) + ": " + g_last_error);
    b.ws_off[i] = off;
    off = align_up(off + plans[i].ws_bytes);
  }
  b.tables_off = off;
  b.n = n;
  // shape classes (tile kernels are compiled per probe shape)
  std::map<std::pair<int, int>, int> cls;
  b.classes.clear();
  for (int i = 0; i < n; ++i) {
    const auto key = std::make_pair(descs[i].my, descs[i].mx);
    if (!cls.count(key)) {
      cls[key] = (int)b.classes.size();
      b.classes.push_back(ShapeClass{descs[i].my, descs[i].mx, {}, {}, 0});
    }
    b.classes[cls[key]].probs.push_back(i);
  }
  if (b.classes.size() > 16) return fail(PTLM_EINVAL, "at most 16 probe shapes per batch");
  // block tables
  b.jb_tile.assign(b.classes.size(), {});
  for (size_t c = 0; c < b.classes.size(); ++c) {
    ShapeClass& C = b.classes[c];
    C.block0.clear();
    for (size_t m = 0; m < C.probs.size(); ++m)
      C.block0.push_back(append_run(b.jb_tile[c], (int)m, plans[C.probs[m]].grid, 8));
    C.nblocks = (int)b.jb_tile[c].size();
  }
  b.jb_obj.clear(); b.jb_prb.clear(); b.jb_prb1.clear(); b.jb_dprb.clear(); b.jb_vec.clear(); b.jb_copy_lin.clear();
  b.jb_copy_acc.clear();
  b.obj_b0.assign(n, 0); b.prb_b0.assign(n, 0); b.prb1_b0.assign(n, 0); b.dprb_b0.assign(n, 0); b.vec_b0.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    const Plan& p = plans[i];
    const int M = p.d.my * p.d.mx;
    b.obj_b0[i] = append_run(b.jb_obj, i, p.otx * p.oty, 1);
    b.prb_b0[i] = append_run(b.jb_prb, i, p.d.mode == PTLM_JOINT ? (M + 63) / 64 : 0, 1);
    b.prb1_b0[i] = append_run(b.jb_prb1, i, p.d.mode == PTLM_JOINT ? (M + 63) / 64 * prb_chunk_count(M, p.nseg) : 0, 1);
    b.dprb_b0[i] = append_run(b.jb_dprb, i, p.d.mode == PTLM_JOINT ? (M + 63) / 64 : 0, 1);  // 64 pixels a block
    b.vec_b0[i] = append_run(b.jb_vec, i, lm_vec_blocks(p.nvec), 1);
  }
  // copy jobs: linearisation (O, P) and acceptance (O, P, previous step) per problem
  int job = 0;
  for (int i = 0; i < n; ++i) {
    const Plan& p = plans[i];
    append_run(b.jb_copy_lin, job++, copy_blocks((size_t)p.d.ny * p.d.nx), 1);
    append_run(b.jb_copy_lin, job++, copy_blocks((size_t)p.d.my * p.d.mx), 1);
  }
  job = 0;
  for (int i = 0; i < n; ++i) {
    const Plan& p = plans[i];
    // accepted object, object step, accepted probe, probe step
    append_run(b.jb_copy_acc, job++, copy_blocks((size_t)p.d.ny * p.d.nx), 1);
    append_run(b.jb_copy_acc, job++, copy_blocks((size_t)p.d.ny * p.d.nx), 1);
    append_run(b.jb_copy_acc, job++, copy_blocks((size_t)p.d.my * p.d.mx), 1);
    append_run(b.jb_copy_acc, job++, copy_blocks((size_t)p.d.my * p.d.mx), 1);
  }
  b.nb_obj = (int)b.jb_obj.size();
  b.nb_prb = (int)b.jb_prb.size();
  b.nb_prb1 = (int)b.jb_prb1.size();
  b.nb_dprb = (int)b.jb_dprb.size();
  b.nb_vec = (int)b.jb_vec.size();
  b.nb_copy_lin = (int)b.jb_copy_lin.size();
  b.nb_copy_acc = (int)b.jb_copy_acc.size();
  // table layout
  TableLayout& L = b.L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return at;
  };
  for (size_t c = 0; c < b.classes.size(); ++c) {
    L.jb_tile_off[c] = take(b.jb_tile[c].size() * sizeof(int));
    for (int k = 0; k < TK_N; ++k) L.tile_jobs_off[c][k] = take(b.classes[c].probs.size() * sizeof(TileJob));
  }
  L.jb_obj = take(b.jb_obj.size() * sizeof(int));
  L.jb_prb = take(b.jb_prb.size() * sizeof(int));
  L.jb_prb1 = take(b.jb_prb1.size() * sizeof(int));
  L.jb_dprb = take(b.jb_dprb.size() * sizeof(int));
  L.jb_vec = take(b.jb_vec.size() * sizeof(int));
  L.jb_copy_lin = take(b.jb_copy_lin.size() * sizeof(int));
  L.jb_copy_acc = take(b.jb_copy_acc.size() * sizeof(int));
  for (int k = 0; k < RK_N; ++k) {
    L.red_obj[k] = take(n * sizeof(RedJob));
    L.red_prb[k] = take(n * sizeof(RedJob));
  }
  L.red_sum = take(n * sizeof(RedJob));
  L.lm_jobs = take(n * sizeof(LMJob));
  L.copy_lin = take(2 * n * sizeof(CopyJob));
  L.copy_acc = take(4 * n * sizeof(CopyJob));
  L.copy_take = take(2 * n * sizeof(CopyJob));
  L.copy_keep = take(2 * n * sizeof(CopyJob));
  L.bytes = o;
  *total = b.tables_off + L.bytes;
  return PTLM_OK;
}

void release_graph(ptlm_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->eager_done = false;
}

}  // namespace

extern "C" {

ptlm_status ptlm_batch_workspace_bytes(int32_t n, const ptlm_desc* descs, const int32_t* const* h_pos,
                                       size_t* bytes) {
  if (!bytes) return fail(PTLM_EINVAL, "bytes is null");
  ptlm_batch b;
  std::vector<Plan> plans;
  return plan_batch(n, descs, h_pos, b, plans, bytes);
}

ptlm_status ptlm_batch_create(int32_t n, const ptlm_desc* descs, const int32_t* const* h_pos, void* d_ws,
                              size_t ws_bytes, void* stream, ptlm_batch** out) {
  if (!out) return fail(PTLM_EINVAL, "out is null");
  *out = nullptr;
  ptlm_batch* b = new ptlm_batch();
  std::vector<Plan> plans;
  size_t need = 0;
  ptlm_status st = plan_batch(n, descs, h_pos, *b, plans, &need);
  if (st != PTLM_OK) {
    delete b;
    return st;
  }
  if (!d_ws || ws_bytes < need) {
    delete b;
    return fail(PTLM_EWORKSPACE, "batch workspace of " + std::to_string(ws_bytes) + " bytes, " +
                                     std::to_string(need) + " needed");
  }
  b->ws = (char*)d_ws;
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < n; ++i) {
    ptlm_handle* h = new ptlm_handle();
    h->in_batch = true;
    st = init_handle(h, &descs[i], h_pos[i], b->ws + b->ws_off[i], plans[i].ws_bytes, s);
    if (st != PTLM_OK) {
      delete h;
      for (ptlm_handle* x : b->hs) delete x;
      delete b;
      return st;
    }
    b->hs.push_back(h);
  }
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(b->ws + b->tables_off + off, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  hipError_t e = hipSuccess;
  for (size_t c = 0; c < b->classes.size() && e == hipSuccess; ++c)
    e = up(b->L.jb_tile_off[c], b->jb_tile[c].data(), b->jb_tile[c].size() * sizeof(int));
  if (e == hipSuccess) e = up(b->L.jb_obj, b->jb_obj.data(), b->jb_obj.size() * sizeof(int));
  if (e == hipSuccess) e = up(b->L.jb_prb, b->jb_prb.data(), b->jb_prb.size() * sizeof(int));
  if (e == hipSuccess) e = up(b->L.jb_prb1, b->jb_prb1.data(), b->jb_prb1.size() * sizeof(int));
  if (e == hipSuccess) e = up(b->L.jb_dprb, b->jb_dprb.data(), b->jb_dprb.size() * sizeof(int));
  if (e == hipSuccess) e = up(b->L.jb_vec, b->jb_vec.data(), b->jb_vec.size() * sizeof(int));
  if (e == hipSuccess) e = up(b->L.jb_copy_lin, b->jb_copy_lin.data(), b->jb_copy_lin.size() * sizeof(int));
  if (e == hipSuccess) e = up(b->L.jb_copy_acc, b->jb_copy_acc.data(), b->jb_copy_acc.size() * sizeof(int));
  if (e != hipSuccess) {
    for (ptlm_handle* x : b->hs) delete x;
    delete b;
    return hip_fail(e, "batch tables");
  }
  *out = b;
  return PTLM_OK;
}

ptlm_handle* ptlm_batch_problem(ptlm_batch* b, int32_t i) {
  if (!b || i < 0 || i >= b->n) return nullptr;
  return b->hs[i];
}

ptlm_status ptlm_batch_bind(ptlm_batch* b, float* const* d_O, float* const* d_P, const float* const* d_y,
                            ptlm_lm_state* d_states, const ptlm_lm_params* params, int32_t T, int32_t use_graph,
                            void* stream) {
  if (!b || !d_O || !d_P || !d_y || !d_states) return fail(PTLM_EINVAL, "null argument");
  ptlm_status st = check_lm_params(params);
  if (st != PTLM_OK) return st;
  if (T < 0) return fail(PTLM_EINVAL, "T must be >= 0");
  for (int i = 0; i < b->n; ++i) {
    if (!d_O[i] || !d_P[i] || !d_y[i]) return fail(PTLM_EINVAL, "null array of problem " + std::to_string(i));
    if (params->precond == 2 && !b->hs[i]->cnn_params)
      return fail(PTLM_EINVAL, "precond == 2 in a batch needs a network on every problem (ptlm_lm_set_cnn)");
    if (params->alternate && !b->hs[i]->g.joint)
      return fail(PTLM_EINVAL, "the alternating update needs PTLM_JOINT problems (problem " + std::to_string(i) + ")");
  }
  hipStream_t s = (hipStream_t)stream;
  release_graph(b);
  b->prm = *params;
  b->T = T;
  b->d_states = d_states;
  b->use_graph = use_graph;
  const int n = b->n;
  b->bound_P.assign(n, nullptr);
  for (int i = 0; i < n; ++i) b->bound_P[i] = (const float2*)d_P[i];
  // tile jobs
  b->tile_jobs.assign(b->classes.size() * TK_N, {});
  for (size_t c = 0; c < b->classes.size(); ++c) {
    const ShapeClass& C = b->classes[c];
    for (int k = 0; k < TK_N; ++k) {
      auto& v = b->tile_jobs[c * TK_N + k];
      for (size_t m = 0; m < C.probs.size(); ++m) {
        const int i = C.probs[m];
        ptlm_handle* h = b->hs[i];
        const Geometry& g = h->g;
        const LMArgs a = make_lm_args(h, params, d_states + i, (const float2*)d_O[i], (const float2*)d_P[i], nullptr);
        int* flags = reinterpret_cast<int*>(d_states + i);
        TileJob j{};
        j.g = g;
        j.block0 = C.block0[m];
        j.nblk = g.grid;
        j.a.O = g.O_lin;
        j.a.P = g.P_lin;
        if (k == TK_LIN) {
          j.a.y = d_y[i];
          j.a.predicate = flags + FL_LIN;
          j.a.bg_add = &d_states[i].sigma;
        } else if (k == TK_WARM || k == TK_P) {
          const float2* v0 = (k == TK_WARM && !params->alternate) ? a.prev : a.p;
          j.a.vO = v0;
          j.a.vP = g.joint ? v0 + a.nobj : nullptr;
          j.a.predicate = flags + (k == TK_WARM ? FL_WARM : FL_CG);
        } else {  // TK_TRIAL, TK_PJ, TK_LS: loss at the trial buffer
          j.a.O = a.ztrial;
          j.a.P = g.joint ? a.ztrial + a.nobj : (const float2*)d_P[i];
          j.a.y = d_y[i];
          j.a.predicate = flags + (k == TK_TRIAL ? FL_ALIVE : (k == TK_PJ ? FL_ACCEPTED : FL_LS_ON));
          j.a.bg_add = &d_states[i].sigma;
        }
        v.push_back(j);
      }
    }
  }
  // reduction jobs
  for (int k = 0; k < RK_N; ++k) {
    b->red_obj[k].assign(n, RedJob{});
    b->red_prb[k].assign(n, RedJob{});
  }
  b->red_sum.assign(n, RedJob{});
  b->lm_jobs.assign(n, LMJob{});
  b->copy_lin.clear();
  b->copy_acc.clear();
  for (int i = 0; i < n; ++i) {
    ptlm_handle* h = b->hs[i];
    const Geometry& g = h->g;
    LMArgs a = make_lm_args(h, params, d_states + i, (const float2*)d_O[i], (const float2*)d_P[i], nullptr);
    a.t_max = T;
    if (params->precond == 2) {
      a.learned = a.xdiag;
      a.cnn_r = cnn_output(h);
    }
    int* flags = reinterpret_cast<int*>(d_states + i);
    const size_t N = a.nobj, M = (size_t)g.my * g.mx;
    for (int k = 0; k < RK_N; ++k) {
      RedJob r{};
      r.g = g;
      if (k == RK_LIN) {
        r.outO = a.g;
        r.outP = a.g + N;
        r.pred = flags + FL_LIN;
      } else if (k == RK_DIAG) {
        r.outO = a.diag;
        r.outP = a.diag + N;
        r.pred = flags + FL_LIN;
      } else {
        const float2* v0 = (k == RK_WARM && !params->alternate) ? a.prev : a.p;
        r.outO = a.Ap;
        r.outP = a.Ap + N;
        r.vO = v0;
        r.vP = v0 + N;
        if (params->scaling) {
          r.dO = (const float*)a.diag;
          r.dP = (const float*)(a.diag + N);
        }
        r.lam_dev = &d_states[i].lambda;
        r.pred = flags + (k == RK_WARM ? FL_WARM : FL_CG);
        if (k == RK_P) {  // a PCG product: the parts of p.Ap, laid out as the single-problem launch's
          r.pap = a.partials;
          r.pap_block = params->alternate ? &d_states[i].block : nullptr;
        }
      }
      RedJob ro = r, rp = r;
      ro.block0 = b->obj_b0[i];
      ro.nblk = g.otiles_x * g.otiles_y;
      rp.block0 = k == RK_DIAG ? b->dprb_b0[i] : b->prb_b0[i];
      rp.block1 = b->prb1_b0[i];
      rp.nblk = g.joint ? (int)((M + 63) / 64) : 0;  // 64 probe pixels per block (reduction and diagonal)
      ro.pap_base = rp.nblk;
      b->red_obj[k][i] = ro;
      b->red_prb[k][i] = rp;
    }
    RedJob rs{};
    rs.g = g;
    rs.sums = a.scal + SC_F;
    rs.pred = flags + FL_LIN;
    b->red_sum[i] = rs;
    LMJob lj{};
    lj.a = a;
    lj.block0 = b->vec_b0[i];
    b->lm_jobs[i] = lj;
    float2* O = (float2*)d_O[i];
    float2* P = (float2*)d_P[i];
    CopyJob c{};
    c.pred = flags + FL_LIN;
    c.src = O; c.dst = h->g.O_lin; c.n = N;
    b->copy_lin.push_back(c);
    c.src = P; c.dst = h->g.P_lin; c.n = M;
    b->copy_lin.push_back(c);
    // the accepted step's blocks (both, or the active one of the alternating update)
    c.pred = flags + FL_ACC_O;
    c.src = a.ztrial; c.dst = O; c.n = N;
    b->copy_acc.push_back(c);
    c.src = a.dx; c.dst = a.prev; c.n = N;
    b->copy_acc.push_back(c);
    c.pred = flags + FL_ACC_P;
    c.src = a.ztrial + N; c.dst = P; c.n = g.joint ? M : 0;
    b->copy_acc.push_back(c);
    c.src = a.dx + N; c.dst = a.prev + N; c.n = g.joint ? M : 0;
    b->copy_acc.push_back(c);
  }
  // block offsets of the copy jobs (runs in job order)
  {
    int b0 = 0, j = 0;
    for (CopyJob& c : b->copy_lin) {
      const int nb = copy_blocks(j % 2 == 0 ? (size_t)b->hs[j / 2]->g.ny * b->hs[j / 2]->g.nx
                                            : (size_t)b->hs[j / 2]->g.my * b->hs[j / 2]->g.mx);
      c.block0 = b0;
      c.nblk = nb;
      b0 += nb;
      ++j;
    }
    b0 = 0;
    j = 0;
    for (CopyJob& c : b->copy_acc) {
      ptlm_handle* h = b->hs[j / 4];
      const size_t len = j % 4 < 2 ? (size_t)h->g.ny * h->g.nx : (size_t)h->g.my * h->g.mx;
      const int nb = copy_blocks(len);
      c.block0 = b0;
      c.nblk = nb;
      b0 += nb;
      ++j;
    }
  }
  // plug-in copies, on the blocks of the linearisation copies (same lengths, same order)
  b->copy_take = b->copy_lin;
  b->copy_keep = b->copy_lin;
  for (int i = 0; i < n; ++i) {
    ptlm_handle* h = b->hs[i];
    const LMArgs& a = b->lm_jobs[i].a;
    int* flags = reinterpret_cast<int*>(d_states + i);
    CopyJob* t = &b->copy_take[2 * i];
    CopyJob* k = &b->copy_keep[2 * i];
    t[0].pred = t[1].pred = flags + FL_LS_TAKE;
    k[0].pred = k[1].pred = flags + FL_LS_KEEP;
    t[0].src = a.ztrial;
    t[1].src = a.ztrial + a.nobj;
    k[0].src = h->g.O_lin;
    k[1].src = h->g.P_lin;
    t[0].dst = k[0].dst = (float2*)d_O[i];
    t[1].dst = k[1].dst = (float2*)d_P[i];
    if (!h->g.joint) t[1].n = k[1].n = 0;
  }
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(b->ws + b->tables_off + off, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  hipError_t e = hipSuccess;
  for (size_t c = 0; c < b->classes.size() && e == hipSuccess; ++c)
    for (int k = 0; k < TK_N && e == hipSuccess; ++k) {
      const auto& v = b->tile_jobs[c * TK_N + k];
      e = up(b->L.tile_jobs_off[c][k], v.data(), v.size() * sizeof(TileJob));
    }
  for (int k = 0; k < RK_N && e == hipSuccess; ++k) {
    e = up(b->L.red_obj[k], b->red_obj[k].data(), n * sizeof(RedJob));
    if (e == hipSuccess) e = up(b->L.red_prb[k], b->red_prb[k].data(), n * sizeof(RedJob));
  }
  if (e == hipSuccess) e = up(b->L.red_sum, b->red_sum.data(), n * sizeof(RedJob));
  if (e == hipSuccess) e = up(b->L.lm_jobs, b->lm_jobs.data(), n * sizeof(LMJob));
  if (e == hipSuccess) e = up(b->L.copy_lin, b->copy_lin.data(), b->copy_lin.size() * sizeof(CopyJob));
  if (e == hipSuccess) e = up(b->L.copy_acc, b->copy_acc.data(), b->copy_acc.size() * sizeof(CopyJob));
  if (e == hipSuccess) e = up(b->L.copy_take, b->copy_take.data(), b->copy_take.size() * sizeof(CopyJob));
  if (e == hipSuccess) e = up(b->L.copy_keep, b->copy_keep.data(), b->copy_keep.size() * sizeof(CopyJob));
  if (e != hipSuccess) return hip_fail(e, "batch bind upload");
  // learned preconditioner: each network's output from the bound probe (once per reconstruction)
  if (params->precond == 2) {
    for (int i = 0; i < n; ++i) {
      ptlm_handle* h = b->hs[i];
      B_HIP(launch_copy((const float2*)d_P[i], h->g.P_lin, (size_t)h->g.my * h->g.mx, nullptr, s), "batch cnn probe");
      PTLM_TRY(cnn_refresh(h, s));
    }
  }
  // reset every state: mu = mu0, t = 0, t_max = T
  B_HIP(launch_fin_batch(F_INIT, b->dev<LMJob>(b->L.lm_jobs), n, 0, FL_NONE, s), "batch init");
  b->h_states.assign(n, ptlm_lm_state{});
  b->bound = true;
  return PTLM_OK;
}

ptlm_status ptlm_batch_cnn_refresh(ptlm_batch* b, void* stream) {
  if (!b || !b->bound) return fail(PTLM_EINVAL, "batch is not bound");
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < b->n; ++i)
    if (!b->hs[i]->cnn_params) return fail(PTLM_EINVAL, "problem " + std::to_string(i) + " has no network");
  // features from each problem's current probe; the linearisation state is not touched, and the
  // next linearisation of each problem builds its learned diagonal from the new output
  for (int i = 0; i < b->n; ++i) PTLM_TRY(cnn_refresh(b->hs[i], s, b->bound_P[i]));
  return PTLM_OK;
}

ptlm_status ptlm_batch_attempt(ptlm_batch* b, void* stream) {
  if (!b || !b->bound) return fail(PTLM_EINVAL, "batch is not bound");
  hipStream_t s = (hipStream_t)stream;
  if (!b->use_graph || !b->eager_done) {
    BatchOps o{b, s};
    PTLM_TRY(enqueue_attempt(o, b->prm));
    b->eager_done = true;
    return PTLM_OK;
  }
  if (!b->exec) {
    if (!b->cap) B_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "batch capture stream");
    B_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed), "batch begin capture");
    BatchOps o{b, b->cap};
    const ptlm_status st = enqueue_attempt(o, b->prm);
    hipGraph_t gph = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &gph);
    if (st != PTLM_OK) {
      if (gph) hipGraphDestroy(gph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "batch end capture");
    b->graph = gph;
    B_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "batch graph instantiate");
  }
  B_HIP(hipGraphLaunch(b->exec, s), "batch graph launch");
  return PTLM_OK;
}

// Run attempts until every problem has done its T outer iterations (or met a non-finite
// value), reading the states every `check_every` attempts; at most max_attempts attempts.
ptlm_status ptlm_batch_solve(ptlm_batch* b, int32_t max_attempts, int32_t check_every, int32_t* attempts_done,
                             void* stream) {
  if (!b || !b->bound) return fail(PTLM_EINVAL, "batch is not bound");
  if (max_attempts < 0 || check_every < 1) return fail(PTLM_EINVAL, "max_attempts >= 0, check_every >= 1");
  hipStream_t s = (hipStream_t)stream;
  int done = 0;
  bool finished = false;
  while (done < max_attempts && !finished) {
    PTLM_TRY(ptlm_batch_attempt(b, stream));
    ++done;
    if (done % check_every == 0 || done == max_attempts) {
      B_HIP(hipMemcpyAsync(b->h_states.data(), b->d_states, b->n * sizeof(ptlm_lm_state), hipMemcpyDeviceToHost, s),
            "batch read states");
      B_HIP(hipStreamSynchronize(s), "batch sync");
      finished = true;
      for (const ptlm_lm_state& x : b->h_states)
        if (x.t < b->T && x.status != PTLM_ENUMERIC) finished = false;
    }
  }
  if (attempts_done) *attempts_done = done;
  for (const ptlm_lm_state& x : b->h_states)
    if (x.status == PTLM_ENUMERIC) return fail(PTLM_ENUMERIC, "a problem of the batch met a non-finite value");
  if (!finished) return fail(PTLM_ENOTACCEPTED, "attempt budget spent before every problem finished");
  return PTLM_OK;
}

ptlm_status ptlm_batch_destroy(ptlm_batch* b) {
  if (!b) return PTLM_OK;
  release_graph(b);
  if (b->cap) hipStreamDestroy(b->cap);
  for (ptlm_handle* h : b->hs) delete h;
  delete b;
  return PTLM_OK;
}

}  // extern "C"
