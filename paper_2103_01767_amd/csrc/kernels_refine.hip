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

// v / n and v mod n for 0 <= v < 2^24, 1 <= n <= 256, inv_n = 1.0f / n: the float quotient is
// within one of the true one (v and n exact, inv_n and the product each within half an ulp), so
// one correction step each way gives the exact result without an integer division
__device__ __forceinline__ int fdiv_small(int v, int n, float inv_n) {
  int q = (int)((float)v * inv_n);
  const int r = v - q * n;
  if (r < 0) --q;
  else if (r >= n) ++q;
  return q;
}
__device__ __forceinline__ int fmod_small(int v, int n, float inv_n) {
  int r = v - (int)((float)v * inv_n) * n;
  if (r < 0) r += n;
  else if (r >= n) r -= n;
  return r;
}

__global__ __launch_bounds__(NT) void refine_kernel(Geometry g, TileArgs a) {
  if (a.predicate && *a.predicate == 0) return;
  const int k = blockIdx.x;
  const int my = g.my, mx = g.mx, M = my * mx;
  const size_t base = (size_t)k * M;
  __shared__ double2 twy[256], twx[256];  // exp(-2 pi i j / my), exp(-2 pi i j / mx)
  __shared__ int list[CAP];
  __shared__ unsigned long long ballots[256][NT / 64];  // per round of NT pixels (M <= 65536)
  __shared__ int round_base[256];
  __shared__ int count;
  __shared__ double2 part[NT / 64][NB];
  __shared__ double dtrace;

  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const float wmin = (float)sqrt(W_REFINE);
  // ---- list the flagged pixels in pixel order.  Pixel m = t + NT j is read by thread t in round
  // j (coalesced) and each wavefront keeps its ballot of the round in LDS, so one barrier
  // separates the reads from the listing.  Pixel order is round-major: a flagged pixel's rank
  // is the flag count of every earlier round, plus the earlier wavefronts' count of its round,
  // plus the lower lanes' count in its own wavefront.
  const int rounds = (M + NT - 1) / NT;
  for (int j = 0; j < rounds; ++j) {
    const int m = t + NT * j;
    const bool fl = m < M && g.w2[base + m] > wmin;
    const unsigned long long bal = __ballot(fl);
    if (lane == 0) ballots[j][wv] = bal;
  }
  __syncthreads();
  if (t == 0) {
    int c = 0;
    for (int j = 0; j < rounds; ++j) {
      round_base[j] = c;
      for (int w = 0; w < NT / 64; ++w) c += __popcll(ballots[j][w]);
    }
    count = c < CAP ? c : CAP;
  }
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int j = 0; j < rounds; ++j) {
    const unsigned long long bal = ballots[j][wv];
    if (!((bal >> lane) & 1ull)) continue;
    int rank = round_base[j] + __popcll(bal & below);
    for (int w = 0; w < wv; ++w) rank += __popcll(ballots[j][w]);
    if (rank < CAP) list[rank] = t + NT * j;
  }
  __syncthreads();
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
  const float inv_my = 1.0f / (float)my, inv_mx = 1.0f / (float)mx;
  const bool xfix = NT % mx == 0;
  const int xcol = t % mx, ystep = NT / mx;
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
    // direct DFT at the nb frequencies: sum over the window pixels (y, x) of psi exp(...), each
    // thread over its pixels q = t, t + NT, ... in that order.  When NT is a multiple of the
    // window width a thread keeps one column x, so its x twiddles are read once per pass and
    // its row advances by NT / mx; otherwise the pixel's row, column and twiddle indices come
    // from the float-reciprocal quotient (all operands below 2^24, exact after the correction)
    if (xfix) {
      // the thread's column is fixed: sum psi exp(-2 pi i ky y / my) over its rows, then apply
      // the column's twiddle once; the row twiddle's index advances by ky * ystep mod my
      int y = t / mx;
      int iy[NB], dy[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        iy[i] = fmod_small(ky[i] * y, my, inv_my);
        dy[i] = fmod_small(ky[i] * ystep, my, inv_my);
      }
      for (int q = t; q < M; q += NT, y += ystep) {
        const float2 P = a.P[q];
        const float2 O = a.O[(size_t)(pk.x + y) * g.nx + pk.y + xcol];
        const double2 psi = zmul(make_double2(P.x, P.y), make_double2(O.x, O.y));
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const double2 v = zmul(psi, twy[iy[i]]);
          acc[i].x += v.x;
          acc[i].y += v.y;
          iy[i] += dy[i];
          if (iy[i] >= my) iy[i] -= my;
        }
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) acc[i] = zmul(acc[i], twx[fmod_small(kx[i] * xcol, mx, inv_mx)]);
    } else {
      for (int q = t; q < M; q += NT) {
        const int y = fdiv_small(q, mx, inv_mx), x = q - y * mx;
        const float2 P = a.P[q];
        const float2 O = a.O[(size_t)(pk.x + y) * g.nx + pk.y + x];
        const double2 psi = zmul(make_double2(P.x, P.y), make_double2(O.x, O.y));
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const double2 w = zmul(twy[fmod_small(ky[i] * y, my, inv_my)], twx[fmod_small(kx[i] * x, mx, inv_mx)]);
          const double2 v = zmul(psi, w);
          acc[i].x += v.x;
          acc[i].y += v.y;
        }
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
