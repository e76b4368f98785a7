// FP64 refinement of the GGN weighting at the pixels where the weight amplifies single-precision
// error (a project addition to the linearisation; Poisson metric or intensity-based GGN).
//
// The linearisation stores, per detector pixel, the phasor a = sqrt(W) psi_hat / zeta / sqrt(M)
// and sqrt(W) of the GGN weight W (ell'' = 2 + 2 y / h for the Poisson metric of
// eq:ell_magnitude, or its intensity-based form), computed from a single-precision far field.
// Where the model intensity h is far below the count y, W ~ 2 y / h is large and the FP32
// far field's absolute error (about 1e-9 of its peak) becomes a large relative error of h,
// hence of W: a handful of such pixels then dominate the rounding error of every GGN-vector
// product.  This kernel recomputes, for every pixel of a position whose stored weight exceeds
// W_REFINE, the far field F(P * S_k O) at that one frequency as a direct DFT in FP64 (exact
// FP32 products of the gathered exit wave, FP64 twiddles and sums), then h, W, the phasor and
// sqrt(W) from it, and corrects the position's trace of W by the change.  The loss, the
// residual and the gradient of the linearisation are left as computed.
//
// One workgroup per position: the flagged pixels are listed in pixel order (at most CAP of
// them; a position with more keeps the rest as computed), then refined NB at a time, each pass
// reading the position's window once; every sum runs in a fixed order.
#include "dft.hpp"
#include "internal.hpp"
#include "tile_pixel.hpp"

namespace ptlm {
namespace {

constexpr int NT = 256;
constexpr int NB = 8;       // pixels refined per pass over the window
constexpr int CAP = 512;    // pixels refined per position at most
constexpr double W_REFINE = 1e4;

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(NT) void refine_kernel(Geometry g, TileArgs a) {
  if (a.predicate && *a.predicate == 0) return;
  const int k = blockIdx.x;
  const int my = g.my, mx = g.mx, M = my * mx;
  const size_t base = (size_t)k * M;
  __shared__ double2 twy[256], twx[256];  // exp(-2 pi i j / my), exp(-2 pi i j / mx)
  __shared__ int list[CAP];
  __shared__ int wave_cnt[NT / 64];
  __shared__ int count;
  __shared__ double2 part[NT / 64][NB];
  __shared__ double dtrace;

  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const float wmin = (float)sqrt(W_REFINE);
  // ---- list the flagged pixels in pixel order
  if (t == 0) count = 0;
  __syncthreads();
  for (int m0 = 0; m0 < M; m0 += NT) {
    const int m = m0 + t;
    const bool fl = m < M && g.w2[base + m] > wmin;
    const unsigned long long bal = __ballot(fl);
    if (lane == 0) wave_cnt[wv] = __popcll(bal);
    __syncthreads();
    int off = count;
    for (int w = 0; w < wv; ++w) off += wave_cnt[w];
    const int rank = off + __popcll(bal & ((1ull << lane) - 1ull));
    if (fl && rank < CAP) list[rank] = m;
    __syncthreads();
    if (t == 0) {
      int c = count;
      for (int w = 0; w < NT / 64; ++w) c += wave_cnt[w];
      count = c < CAP ? c : CAP;
    }
    __syncthreads();
  }
  const int n = count;
  if (n == 0) return;

  for (int j = t; j < my; j += NT) {
    double s, c;
    sincospi(-2.0 * j / my, &s, &c);
    twy[j] = make_double2(c, s);
  }
  for (int j = t; j < mx; j += NT) {
    double s, c;
    sincospi(-2.0 * j / mx, &s, &c);
    twx[j] = make_double2(c, s);
  }
  if (t == 0) dtrace = 0.0;
  __syncthreads();

  const int2 pk = g.pos[k];
  const double bg = a.bg_add ? (double)g.background + *a.bg_add : (double)g.background;
  const bool poisson = g.metric != 0, intensity = g.ggn != 0;
  const double isq = 1.0 / sqrt((double)M);
  for (int b0 = 0; b0 < n; b0 += NB) {
    const int nb = n - b0 < NB ? n - b0 : NB;
    int ky[NB], kx[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int m = list[b0 + (i < nb ? i : 0)];
      ky[i] = m / mx;
      kx[i] = m % mx;
    }
    double2 acc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) acc[i] = make_double2(0.0, 0.0);
    // direct DFT at the nb frequencies: sum over the window pixels (y, x) of psi exp(...)
    for (int q = t; q < M; q += NT) {
      const int y = q / mx, x = q % mx;
      const float2 P = a.P[q];
      const float2 O = a.O[(size_t)(pk.x + y) * g.nx + pk.y + x];
      const double2 psi = zmul(make_double2(P.x, P.y), make_double2(O.x, O.y));
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const double2 w = zmul(twy[(ky[i] * y) % my], twx[(kx[i] * x) % mx]);
        const double2 v = zmul(psi, w);
        acc[i].x += v.x;
        acc[i].y += v.y;
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      for (int off = 32; off > 0; off >>= 1) {
        acc[i].x += __shfl_xor(acc[i].x, off, 64);
        acc[i].y += __shfl_xor(acc[i].y, off, 64);
      }
      if (lane == 0) part[wv][i] = acc[i];
    }
    __syncthreads();
    if (t < nb) {
      double2 ps = make_double2(0.0, 0.0);
      for (int w = 0; w < NT / 64; ++w) {
        ps.x += part[w][t].x;
        ps.y += part[w][t].y;
      }
      ps.x *= isq;
      ps.y *= isq;
      const size_t gi = base + list[b0 + t];
      const double yv = (double)a.y[gi];
      const double h = ps.x * ps.x + ps.y * ps.y + bg;
      const double zeta = sqrt(h);
      double W;
      if (!intensity) W = poisson ? 2.0 + 2.0 * yv / h : 1.0;
      else W = fmax(poisson ? 4.0 * yv / h : sqrt(yv) / zeta, 1e-30);
      const double w = sqrt(W);
      const float w_old = g.w2[gi];
      g.afield[gi] = make_float2((float)(w * ps.x / zeta * isq), (float)(w * ps.y / zeta * isq));
      g.w2[gi] = (float)w;
      part[0][t] = make_double2(W - (double)w_old * (double)w_old, 0.0);  // change of the trace
    }
    __syncthreads();
    if (t == 0) {
      double d = dtrace;
      for (int i = 0; i < nb; ++i) d += part[0][i].x;
      dtrace = d;
    }
    __syncthreads();
  }
  if (t == 0) g.trace[k] += dtrace;
}

}  // namespace

hipError_t launch_refine(const Geometry& g, const TileArgs& a, hipStream_t s) {
  if (!g.w2 || g.K <= 0) return hipSuccess;
  if (g.my > 256 || g.mx > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(refine_kernel, dim3(g.K), dim3(NT), 0, s, g, a);
  return hipGetLastError();
}

}  // namespace ptlm
