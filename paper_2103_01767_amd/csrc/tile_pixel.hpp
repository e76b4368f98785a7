// Per-pixel work of the tile kernels in the frequency layout (between the forward and the
// inverse transform), for one detector pixel gi of position k:
//
//   FORWARD    zeta = sqrt(|psi_hat|^2 + b)                                  (eq:magnitude)
//   LOSS       ell, ell' summed in FP64; ell' (the residual) optionally stored (eq:ell_magnitude)
//   LINEARIZE  as LOSS, plus the stored phasor field a = sqrt(ell'') psi_hat / zeta / sqrt(M),
//              the trace of ell'' and the gradient field ell' psi_hat / zeta for F^H
//   JVP        Re(conj(e) F dpsi) (divided by sqrt(ell'') for the Poisson metric)
//   GGNV       Re(conj(a) F dpsi) a   (loss-Hessian weighting of the GGN-vector product)
//   VJP        w a (divided by sqrt(ell'') for the Poisson metric)
//
// v holds the unnormalised transform; isq = 1/sqrt(M) applies the unitary normalisation
// (eq:expected_count); bgv is the background (plus the surrogate term of App. E when set).
// The metric is a template parameter, so pixel loops carry no per-pixel branch on it.
// Gaussian ell = (zeta - sqrt y)^2 / 2, Poisson ell = zeta^2 - y log zeta^2.
#pragma once
#include <type_traits>

#include "dft.hpp"
#include "internal.hpp"

namespace ptlm {

__device__ __forceinline__ float2 ld_once(const float2* p) {
  const double d = __builtin_nontemporal_load(reinterpret_cast<const double*>(p));
  return __builtin_bit_cast(float2, d);
}

// Whether the per-pixel work of OP depends on the metric (the caller then dispatches the
// metric once, outside its pixel loop, so the loop has no per-pixel branches).
template <int OP>
constexpr bool metric_dependent() {
  return OP == OP_LOSS || OP == OP_LINEARIZE || OP == OP_JVP || OP == OP_VJP;
}

// MET: 0 Gaussian, 1 Poisson (g.w2 holds sqrt(ell'') for the Poisson metric only), -1 read
// from g per pixel (for loops where two specialised copies cost more registers than the branch)
template <int OP, int MET>
__device__ __forceinline__ void pixel_op(const Geometry& g, const TileArgs& a, size_t gi, float isq, float bgv,
                                         float2& v, double& s0, double& s1, double& tr) {
  if constexpr (OP == OP_FORWARD || OP == OP_LOSS || OP == OP_LINEARIZE) {
    const float2 ps = cscale(v, isq);
    const float h = fmaf(ps.x, ps.x, fmaf(ps.y, ps.y, bgv));
    const float iz = rsqrtf(h);
    const float zeta = h * iz;
    if constexpr (OP == OP_FORWARD) {
      a.rout[gi] = zeta;
    } else {
      const float yv = a.y[gi];
      float l, l1, l2;
      if (MET == 0 || (MET < 0 && g.metric == 0)) {
        const float d = zeta - sqrtf(yv);
        l = 0.5f * d * d;
        l1 = d;
        l2 = 1.0f;
      } else {
        l = h - yv * logf(h);
        l1 = 2.0f * zeta - 2.0f * yv * iz;
        l2 = 2.0f + 2.0f * yv / h;
      }
      s0 += (double)l;
      s1 += (double)l1 * (double)l1;
      if constexpr (OP == OP_LOSS) {
        if (a.rout) a.rout[gi] = l1;
      } else {
        tr += (double)l2;
        const float w = sqrtf(l2);
        const float2 e = cscale(ps, iz);
        g.afield[gi] = cscale(e, w * isq);
        if constexpr (MET == 1) g.w2[gi] = w;
        if constexpr (MET < 0) {
          if (g.w2) g.w2[gi] = w;
        }
        v = cscale(e, l1 * isq);
      }
    }
  } else if constexpr (OP == OP_JVP) {
    const float2 as = ld_once(g.afield + gi);
    float val = fmaf(as.x, v.x, as.y * v.y);
    if constexpr (MET == 1) val /= g.w2[gi];
    if constexpr (MET < 0) {
      if (g.w2) val /= g.w2[gi];
    }
    a.rout[gi] = val;
  } else if constexpr (OP == OP_GGNV) {
    const float2 as = ld_once(g.afield + gi);
    const float tt = fmaf(as.x, v.x, as.y * v.y);
    v = cscale(as, tt);
  } else if constexpr (OP == OP_VJP) {
    const float2 as = ld_once(g.afield + gi);
    float w = a.win[gi];
    if constexpr (MET == 1) w /= g.w2[gi];
    if constexpr (MET < 0) {
      if (g.w2) w /= g.w2[gi];
    }
    v = cscale(as, w);
  }
}

// Run body(std::integral_constant<int, MET>) with the problem's metric as a constant (once
// for metric-independent ops).
template <int OP, class F>
__device__ __forceinline__ void with_metric(const Geometry& g, F&& body) {
  if constexpr (metric_dependent<OP>()) {
    if (g.metric == 0) body(std::integral_constant<int, 0>{});
    else body(std::integral_constant<int, 1>{});
  } else {
    body(std::integral_constant<int, 0>{});
  }
}

}  // namespace ptlm
