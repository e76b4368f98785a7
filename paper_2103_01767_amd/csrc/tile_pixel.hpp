// Per-pixel work of the tile kernels in the frequency layout (between the forward and the
// inverse transform), for one detector pixel gi of position k:
//
//   FORWARD    zeta = sqrt(|psi_hat|^2 + b)                                  (eq:magnitude)
//   LOSS       ell, ell' summed in FP64; ell' (the residual) optionally stored (eq:ell_magnitude)
//   LINEARIZE  as LOSS, plus the stored phasor field a = sqrt(W) psi_hat / zeta / sqrt(M) for
//              the GGN weight W (ell'' or its intensity-based form), the trace of W and the
//              gradient field ell' psi_hat / zeta for F^H
//   JVP        Re(conj(e) F dpsi) (a divided by sqrt(W) where W is not 1)
//   GGNV       Re(conj(a) F dpsi) a   (loss-Hessian weighting of the GGN-vector product)
//   VJP        w a (divided by sqrt(W) where W is not 1)
//   VJP_RAND   r a for a generated sign field r (stochastic estimate of diag(G))
//
// v holds the unnormalised transform; isq = 1/sqrt(M) applies the unitary normalisation
// (eq:expected_count); bgv is the background (plus the surrogate term of App. E when set).
// Gaussian ell = (zeta - sqrt y)^2 / 2, Poisson ell = zeta^2 - y log zeta^2.
#pragma once
#include "dft.hpp"
#include "internal.hpp"

namespace ptlm {

// Streamed accesses (read or written once per call): the nontemporal hint keeps them from
// evicting the windows and strips that the tile kernels reuse from L2.
__device__ __forceinline__ float2 ld_once(const float2* p) {
  const double d = __builtin_nontemporal_load(reinterpret_cast<const double*>(p));
  return __builtin_bit_cast(float2, d);
}
__device__ __forceinline__ void st_once(float2* p, float2 v) {
  __builtin_nontemporal_store(__builtin_bit_cast(double, v), reinterpret_cast<double*>(p));
}

// Order this wave's LDS writes before its later LDS reads (exchanges whose readers are the
// writers' own wavefront need no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Give each
// XCD a contiguous run of segments -- consecutive scan positions, overlapping windows -- so
// the object windows it gathers stay in its L2.
__device__ __forceinline__ int xcd_block(int b, int n) {
  if (n % 8 != 0) return b;
  return (b % 8) * (n / 8) + b / 8;
}

// Output n >= 1 of the SplitMix64 generator seeded with `seed` (Steele, Lea and Flood 2014):
// Stafford's 64-bit finaliser of seed + n * golden gamma.  Counter-based, so every measurement
// draws its own sign independently.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long seed, unsigned long long n) {
  unsigned long long z = seed + n * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// MET (a constant, so pixel loops can carry no per-pixel branch on it): bit 0 the metric
// (0 Gaussian, 1 Poisson), bit 1 the GGN weight (0 magnitude-based ell''(zeta), 1 intensity-
// based 4 zeta^2 L''(zeta^2) = sqrt(y) / zeta (Gaussian) or 4 y / h (Poisson), floored at 1e-30
// so that the stored phasors keep the Jacobian recoverable where y = 0).  For the JVP / VJP
// MET != 0 means that g.w2 holds sqrt of the weight.  MET = -1 reads all of it from g per
// pixel (for loops where two specialised copies cost more registers than the branch).
template <int OP, int MET>
__device__ __forceinline__ void pixel_op(const Geometry& g, const TileArgs& a, size_t gi, float isq, float bgv,
                                         float2& v, double& s0, double& s1, double& tr) {
  // multiply-adds are fused only within one expression, so every MET variant of a kernel (and
  // the batched kernel, which reads MET per pixel) rounds identically
#pragma clang fp contract(on)
  if constexpr (OP == OP_FORWARD || OP == OP_LOSS || OP == OP_LINEARIZE) {
    const float2 ps = cscale(v, isq);
    const float h = fmaf(ps.x, ps.x, fmaf(ps.y, ps.y, bgv));
    const float iz = rsqrtf(h);
    const float zeta = h * iz;
    if constexpr (OP == OP_FORWARD) {
      a.rout[gi] = zeta;
    } else {
      const float yv = __builtin_nontemporal_load(a.y + gi);
      const bool poisson = MET >= 0 ? (MET & 1) != 0 : g.metric != 0;
      float l, l1;
      if (!poisson) {
        const float d = zeta - sqrtf(yv);
        l = 0.5f * d * d;
        l1 = d;
      } else {
        l = h - yv * logf(h);
        l1 = 2.0f * zeta - 2.0f * yv * iz;
      }
      s0 += (double)l;
      s1 += (double)l1 * (double)l1;
      if constexpr (OP == OP_LOSS) {
        if (a.rout) a.rout[gi] = l1;
      } else {
        const bool intensity = MET >= 0 ? (MET & 2) != 0 : g.ggn != 0;
        float l2;
        if (!intensity) l2 = poisson ? 2.0f + 2.0f * yv / h : 1.0f;
        else l2 = fmaxf(poisson ? 4.0f * yv / h : sqrtf(yv) * iz, 1e-30f);
        tr += (double)l2;
        const float w = sqrtf(l2);
        const float2 e = cscale(ps, iz);
        st_once(g.afield + gi, cscale(e, w * isq));
        if constexpr (MET > 0) __builtin_nontemporal_store(w, g.w2 + gi);
        if constexpr (MET < 0) {
          if (g.w2) __builtin_nontemporal_store(w, g.w2 + gi);
        }
        v = cscale(e, l1 * isq);
      }
    }
  } else if constexpr (OP == OP_JVP) {
    const float2 as = ld_once(g.afield + gi);
    float val = fmaf(as.x, v.x, as.y * v.y);
    if constexpr (MET > 0) val /= g.w2[gi];
    if constexpr (MET < 0) {
      if (g.w2) val /= g.w2[gi];
    }
    a.rout[gi] = val;
  } else if constexpr (OP == OP_GGNV) {
    const float2 as = ld_once(g.afield + gi);
    const float tt = fmaf(as.x, v.x, as.y * v.y);
    v = cscale(as, tt);
  } else if constexpr (OP == OP_VJP_RAND) {
    // r a with r = +-1 from the top bit of output draw * K * M + gi + 1: one draw of
    // J^T diag(sqrt(W)) r, whose squares estimate diag(G) without bias
    const unsigned long long draw = a.rdraw + (a.rdraw_t ? (unsigned long long)(*a.rdraw_t) * a.rdraw_mul : 0ull);
    const unsigned long long n = draw * ((unsigned long long)g.K * (unsigned long long)g.my * g.mx) + gi + 1ull;
    const float2 as = ld_once(g.afield + gi);
    v = (splitmix64(a.rseed, n) >> 63) ? make_float2(-as.x, -as.y) : as;
  } else if constexpr (OP == OP_VJP) {
    const float2 as = ld_once(g.afield + gi);
    float w = a.win[gi];
    if constexpr (MET > 0) w /= g.w2[gi];
    if constexpr (MET < 0) {
      if (g.w2) w /= g.w2[gi];
    }
    v = cscale(as, w);
  }
}

// MET code of an op for a problem (the template argument of single-problem launches)
inline int met_code(int op, const Geometry& g) {
  if (op == OP_LOSS) return g.metric;
  if (op == OP_LINEARIZE) return g.metric + 2 * g.ggn;
  if (op == OP_JVP || op == OP_VJP) return g.w2 ? 1 : 0;
  return 0;
}

}  // namespace ptlm
