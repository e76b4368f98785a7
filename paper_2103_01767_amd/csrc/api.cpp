// C ABI of the library: problem planning, workspace layout, validation and the
// product calls (forward, loss, linearise, JVP, VJP, GGN-vector product,
// diagonal).  The LM driver lives in lm.cpp.
#include "api_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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

#define PTLM_CHECK_H(h)                                    \
  do {                                                     \
    if (!(h)) return fail(PTLM_EINVAL, "handle is null"); \
  } while (0)
#define PTLM_HIP(call, where)                         \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

static size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Workgroups per CU the tile kernels can keep resident (LDS- and wave-limited).
static int wgs_per_cu(int my, int mx) {
  const size_t lds = tile_lds_bytes(my, mx);
  const int wg = tile_threads(my, mx);
  int by_lds = (int)((160 * 1024) / lds);
  int by_waves = 2048 / wg;
  return std::max(1, std::min(by_lds, by_waves));
}

// object 16x16 tiles -> items (segments or positions) whose box meets the tile (CSR)
template <class Boxes>
static void build_csr(const Plan& p, Boxes boxes, int count, std::vector<int>& ptr, std::vector<int>& idx) {
  const int ntiles = p.oty * p.otx;
  std::vector<int> cnt(ntiles + 1, 0);
  for (int i = 0; i < count; ++i) {
    int r0, c0, h, w;
    boxes(i, r0, c0, h, w);
    if (h <= 0 || w <= 0) continue;
    for (int ty = r0 / 16; ty <= (r0 + h - 1) / 16; ++ty)
      for (int tx = c0 / 16; tx <= (c0 + w - 1) / 16; ++tx) cnt[ty * p.otx + tx + 1]++;
  }
  for (int t = 0; t < ntiles; ++t) cnt[t + 1] += cnt[t];
  ptr = cnt;
  idx.assign(std::max(1, cnt[ntiles]), 0);
  std::vector<int> fill(cnt.begin(), cnt.end() - 1);
  for (int i = 0; i < count; ++i) {
    int r0, c0, h, w;
    boxes(i, r0, c0, h, w);
    if (h <= 0 || w <= 0) continue;
    for (int ty = r0 / 16; ty <= (r0 + h - 1) / 16; ++ty)
      for (int tx = c0 / 16; tx <= (c0 + w - 1) / 16; ++tx) idx[fill[ty * p.otx + tx]++] = i;
  }
}

// Workgroups of the tile kernels for a grid scale: scale x (resident workgroups of the chip),
// at most one per tiles-per-workgroup positions.
static int plan_grid(const Plan& p, double scale) {
  const int resident = 256 * wgs_per_cu(p.d.my, p.d.mx);
  const int gmax = std::max(1, (int)std::llround(resident * scale));
  return std::max(1, std::min((p.d.K + p.tpw - 1) / p.tpw, gmax));
}

// Contiguous segments of the position list, at most ceil(K / nseg) positions each, for
// `grid` workgroups.  Where the scan jumps (consecutive windows half a side or more apart, as
// at the end of a raster row) a segment is cut, if the cuts still leave at most nseg segments
// of that length: a segment across a jump has a bounding box (its strip) that is mostly
// outside its windows, which the tile kernel must clear and the gather must read.  Runs
// between jumps are split evenly, and the segments are spread over the nseg slots so that the
// empty ones do not bunch on one XCD.  Otherwise the list is cut evenly (lengths differing by
// at most one).  Then the strip boxes and offsets and the object-tile -> segment map.
static void segment(Plan& p, const int* h_pos, int grid) {
  const ptlm_desc* d = &p.d;
  const int K = d->K;
  p.grid = grid;
  p.nseg = p.grid * p.tpw;
  p.seg_start.resize(p.nseg + 1);
  const int L = (int)(((long long)K + p.nseg - 1) / p.nseg);
  std::vector<int> cuts{0};  // starts of the segments cut at jumps, then K
  int b = 0;
  for (int k = 1; k <= K && (int)cuts.size() <= p.nseg + 1; ++k) {
    const bool jump = k == K || std::abs(h_pos[2 * k] - h_pos[2 * k - 2]) * 2 >= d->my ||
                      std::abs(h_pos[2 * k + 1] - h_pos[2 * k - 1]) * 2 >= d->mx;
    if (!jump) continue;
    const int n = k - b, m = (n + L - 1) / L;
    for (int i = 1; i <= m; ++i) cuts.push_back(b + (int)(((long long)i * n) / m));
    b = k;
  }
  const int count = (int)cuts.size() - 1;
  if (b == K && count <= p.nseg) {
    // segment j goes to slot floor(j nseg / count): strictly increasing, so every other slot is empty
    int j = 0;
    for (int s = 0; s <= p.nseg; ++s) {
      while (j < count && (int)(((long long)j * p.nseg) / count) < s) ++j;
      p.seg_start[s] = cuts[j];
    }
  } else {
    for (int s = 0; s <= p.nseg; ++s) p.seg_start[s] = (int)(((long long)s * K) / p.nseg);
  }
  p.seg_box.assign(p.nseg, make_int4(0, 0, 0, 0));
  p.seg_off.assign(p.nseg, 0);
  long long off = 0;
  for (int s = 0; s < p.nseg; ++s) {
    const int b = p.seg_start[s], e = p.seg_start[s + 1];
    if (b == e) {
      p.seg_off[s] = off;
      continue;
    }
    int r0 = INT32_MAX, c0 = INT32_MAX, r1 = 0, c1 = 0;
    for (int k = b; k < e; ++k) {
      r0 = std::min(r0, h_pos[2 * k]);
      c0 = std::min(c0, h_pos[2 * k + 1]);
      r1 = std::max(r1, h_pos[2 * k] + d->my);
      c1 = std::max(c1, h_pos[2 * k + 1] + d->mx);
    }
    p.seg_box[s] = make_int4(r0, c0, r1 - r0, c1 - c0);
    p.seg_off[s] = off;
    off += (long long)(r1 - r0) * (c1 - c0);
  }
  p.strip_elems = off;
  build_csr(
      p,
      [&](int s, int& r0, int& c0, int& h, int& w) {
        r0 = p.seg_box[s].x; c0 = p.seg_box[s].y; h = p.seg_box[s].z; w = p.seg_box[s].w;
      },
      p.nseg, p.otile_ptr, p.otile_seg);
}

// grid scales the autotuner tries; the workspace holds the largest of their segment tables
static const double kGridScales[] = {0.5, 1.0, 2.0};

ptlm_status make_plan(const ptlm_desc* d, const int32_t* h_pos, Plan& p, double grid_scale) {
  if (!d) return fail(PTLM_EINVAL, "desc is null");
  if (!h_pos && d->K > 0) return fail(PTLM_EINVAL, "positions are null");
  if (d->K < 1) return fail(PTLM_EINVAL, "K must be >= 1");
  if (!tile_shape_supported(d->my, d->mx))
    return fail(PTLM_EINVAL, "probe sides must each be 16, 32, 64 or 128, or both 48, 96 or 256");
  if (d->ny < d->my || d->nx < d->mx) return fail(PTLM_EINVAL, "object smaller than probe");
  if (d->metric != PTLM_GAUSS && d->metric != PTLM_POISSON) return fail(PTLM_EINVAL, "unknown metric");
  if (d->ggn != PTLM_GGN_MAGNITUDE && d->ggn != PTLM_GGN_INTENSITY) return fail(PTLM_EINVAL, "unknown GGN kind");
  if (d->mode != PTLM_OBJECT && d->mode != PTLM_JOINT) return fail(PTLM_EINVAL, "unknown mode");
  if (!(d->background > 0.0f) || !std::isfinite(d->background))
    return fail(PTLM_EINVAL, "background must be finite and > 0");
  if ((long long)d->ny * d->nx > (1LL << 31)) return fail(PTLM_EINVAL, "object too large");
  for (int k = 0; k < d->K; ++k) {
    const int r = h_pos[2 * k], c = h_pos[2 * k + 1];
    if (r < 0 || c < 0 || r > d->ny - d->my || c > d->nx - d->mx) {
      char buf[160];
      snprintf(buf, sizeof buf, "position %d = (%d, %d) outside [0, %d] x [0, %d]", k, r, c, d->ny - d->my,
               d->nx - d->mx);
      return fail(PTLM_EINVAL, buf);
    }
  }
  p.d = *d;
  const int K = d->K, M = d->my * d->mx;
  const long long N = (long long)d->ny * d->nx;
  p.tpw = tile_per_wg(d->my, d->mx);
  p.oty = (d->ny + 15) / 16;
  p.otx = (d->nx + 15) / 16;
  // sizes of the segment-dependent regions over every autotuner candidate
  int max_grid = 1;
  size_t max_nseg = 1, max_otile = 1;
  long long max_strip = 0;
  for (double sc : kGridScales) {
    segment(p, h_pos, plan_grid(p, sc));
    max_grid = std::max(max_grid, p.grid);
    max_nseg = std::max(max_nseg, (size_t)p.nseg);
    max_otile = std::max(max_otile, p.otile_seg.size());
    max_strip = std::max(max_strip, p.strip_elems);
  }
  if (std::find(std::begin(kGridScales), std::end(kGridScales), grid_scale) == std::end(kGridScales))
    return fail(PTLM_EINVAL, "grid scale must be 0.5, 1 or 2");
  p.max_grid = max_grid;
  p.grid_scale = grid_scale;
  segment(p, h_pos, plan_grid(p, grid_scale));
  build_csr(
      p,
      [&](int k, int& r0, int& c0, int& h, int& w) {
        r0 = h_pos[2 * k]; c0 = h_pos[2 * k + 1]; h = d->my; w = d->mx;
      },
      K, p.ptile_ptr, p.ptile_pos);

  // twiddles W_L^(n k) = exp(-2 pi i n k / L), n < L/16, k < 16, L = 32, 64, 128, 256, 48, 96
  p.tw.assign(624, make_float2(0.f, 0.f));
  int base = 0;
  for (int L : {32, 64, 128, 256, 48, 96}) {
    for (int n = 0; n < L / 16; ++n)
      for (int k = 0; k < 16; ++k) {
        const double ang = -2.0 * M_PI * (double)(n * k) / (double)L;
        p.tw[base + n * 16 + k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      }
    base += (L / 16) * 16;
  }
  p.pos.assign(h_pos, h_pos + 2 * K);

  // workspace layout
  const bool joint = d->mode == PTLM_JOINT;
  const size_t n2 = (size_t)(N + (joint ? M : 0));  // complex entries of a vector of R^(2n)
  p.nvec = n2;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  p.off.tw = take(p.tw.size() * sizeof(float2));
  p.off.pos = take((size_t)K * sizeof(int2));
  p.off.seg_start = take((max_nseg + 1) * sizeof(int));
  p.off.seg_box = take(max_nseg * sizeof(int4));
  p.off.seg_off = take(max_nseg * sizeof(long long));
  p.off.otile_ptr = take(p.otile_ptr.size() * sizeof(int));
  p.off.otile_seg = take(max_otile * sizeof(int));
  p.off.ptile_ptr = take(p.ptile_ptr.size() * sizeof(int));
  p.off.ptile_pos = take(p.ptile_pos.size() * sizeof(int));
  p.off.O_lin = take((size_t)N * sizeof(float2));
  p.off.P_lin = take((size_t)M * sizeof(float2));
  p.off.afield = take((size_t)K * M * sizeof(float2));
  // sqrt of the GGN weight, kept where it is not 1 (the JVP / VJP divide it out of the phasors)
  const bool weighted = d->metric == PTLM_POISSON || d->ggn == PTLM_GGN_INTENSITY;
  p.off.w2 = weighted ? take((size_t)K * M * sizeof(float)) : 0;
  p.off.trace = take((size_t)K * sizeof(double));
  p.off.strips = take((size_t)max_strip * sizeof(float2));
  p.off.probe_part = take(max_nseg * M * sizeof(float2));
  p.off.partials = take((size_t)std::max(max_grid, 1024) * 4 * sizeof(double));
  p.off.scratch = d->my == 256 ? take((size_t)max_grid * M * sizeof(float2)) : 0;
  p.off.scal = take(64 * sizeof(double));  // [0..7], [12..17] LM scalars, [8..11] feature / learned-diagonal scratch
  // LM / PCG vectors (complex entries of R^(2n)) and real diagonals
  p.off.g = take(n2 * sizeof(float2));
  p.off.dx = take(n2 * sizeof(float2));
  p.off.prev = take(n2 * sizeof(float2));
  p.off.r = take(n2 * sizeof(float2));
  p.off.z = take(n2 * sizeof(float2));
  p.off.p = take(n2 * sizeof(float2));
  p.off.Ap = take(n2 * sizeof(float2));
  p.off.diag = take(n2 * sizeof(float2));
  p.off.ztrial = take(n2 * sizeof(float2));
  p.off.learned = take(n2 * sizeof(float2));
  p.off.lmstate = take(sizeof(ptlm_lm_state));
  p.off.afield2 = take((size_t)K * M * sizeof(float2));
  p.off.w2_2 = weighted ? take((size_t)K * M * sizeof(float)) : 0;
  p.off.trace2 = take((size_t)K * sizeof(double));
  p.off.g2 = take(n2 * sizeof(float2));
  p.ws_bytes = o;
  return PTLM_OK;
}

ptlm_status diag_exact_impl(ptlm_handle* h, float* dO, float* dP, hipStream_t s, const int* pred) {
  TileArgs a{};
  a.O = h->g.O_lin;
  a.P = h->g.P_lin;
  a.predicate = pred;
  hipError_t e = launch_tile(h->g, OP_DIAG_EXACT, a, s);
  if (e != hipSuccess) return hip_fail(e, "diag exact");
  e = launch_obj_reduce(h->g, (float2*)dO, 0.0, nullptr, nullptr, nullptr, pred, s);
  if (e != hipSuccess) return hip_fail(e, "diag exact O");
  if (dP) {
    e = launch_probe_reduce(h->g, (float2*)dP, 0.0, nullptr, nullptr, nullptr, pred, s);
    if (e != hipSuccess) return hip_fail(e, "diag exact P");
  }
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
  PTLM_HIP(launch_sum_partials(g.partials, g.grid, d_f, 2, s), "linearize sum");
  PTLM_HIP(launch_obj_reduce(g, gO, 0.0, nullptr, nullptr, nullptr, nullptr, s), "linearize gO");
  if (g.joint && gP) PTLM_HIP(launch_probe_reduce(g, gP, 0.0, nullptr, nullptr, nullptr, nullptr, s), "linearize gP");
  return PTLM_OK;
}

ptlm_status ggnv_impl(ptlm_handle* h, const float2* vO, const float2* vP, double lam, const double* lam_dev,
                      const float* dO, const float* dP, float2* outO, float2* outP, const int* pred, hipStream_t s,
                      int stage) {
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
    PTLM_HIP(launch_obj_reduce(h->g, outO, lam, lam_dev, dO, vO, pred, s), "ggn_vp O");
    if (h->g.joint) PTLM_HIP(launch_probe_reduce(h->g, outP, lam, lam_dev, dP, vP, pred, s), "ggn_vp P");
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

ptlm_status autotune_impl(ptlm_handle* h, int reps, double* h_ms, double* h_scale, hipStream_t s) {
  Plan& p = h->plan;
  const size_t N = (size_t)p.d.ny * p.d.nx;
  float2* out = (float2*)(h->ws + p.off.Ap);
  const float2* vO = h->g.O_lin;
  const float2* vP = h->g.joint ? h->g.P_lin : nullptr;
  hipEvent_t e0, e1;
  PTLM_HIP(hipEventCreate(&e0), "autotune event");
  PTLM_HIP(hipEventCreate(&e1), "autotune event");
  double best = 1e300;
  int bi = 1;
  ptlm_status st = PTLM_OK;
  const int nc = (int)(sizeof(kGridScales) / sizeof(kGridScales[0]));
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
    if (h_ms) h_ms[i] = per;
    if (per < best) {
      best = per;
      bi = i;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != PTLM_OK) return st;
  if (h_scale) *h_scale = kGridScales[bi];
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
  PTLM_HIP(launch_obj_reduce(h->g, (float2*)d_outO, 0.0, nullptr, nullptr, nullptr, nullptr, s), "vjp O");
  if (h->g.joint) PTLM_HIP(launch_probe_reduce(h->g, (float2*)d_outP, 0.0, nullptr, nullptr, nullptr, nullptr, s), "vjp P");
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

ptlm_status ptlm_autotune(ptlm_handle* h, int32_t reps, double* h_ms, double* h_scale, void* stream) {
  PTLM_CHECK_H(h);
  if (reps < 1) return fail(PTLM_EINVAL, "reps must be >= 1");
  return autotune_impl(h, reps, h_ms, h_scale, (hipStream_t)stream);
}

const char* ptlm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
