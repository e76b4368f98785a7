// Problem planning: validation of the description and positions, the position segments of
// the tile kernels and their strips, the object-tile lists of the gather kernels, the twiddle
// table and the workspace layout.  Host only.
#include "api_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>

namespace ptlm {

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
// at most one per tiles-per-workgroup positions, and with seg_len > 0 at most one per
// tiles-per-workgroup segments of seg_len positions.
int plan_grid(const Plan& p, double scale) {
  const int resident = 256 * wgs_per_cu(p.d.my, p.d.mx);
  int gmax = std::max(1, (int)std::llround(resident * scale));
  if (p.d.seg_len > 0) {
    const int nseg = (p.d.K + p.d.seg_len - 1) / p.d.seg_len;
    gmax = std::min(gmax, (nseg + p.tpw - 1) / p.tpw);
  }
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
void segment(Plan& p, const int* h_pos, int grid) {
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
const double kGridScales[kNumGridScales] = {0.5, 1.0, 2.0};

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
  if (d->seg_len < 0) return fail(PTLM_EINVAL, "seg_len must be >= 0");
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
  // FP64 partial sums: tile workgroups, vector-kernel blocks (at most 1024) and the p.Ap parts of
  // a PCG product's sums (one per block of the object and probe sums)
  const int pap_parts = (joint ? (M + 63) / 64 : 0) + p.oty * p.otx;
  p.off.partials = take((size_t)std::max({max_grid, 1024, pap_parts}) * 4 * sizeof(double));
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

}  // namespace ptlm
