// Truncated PCG (eq:lma_termination_magnitude) and the LM step control of
// alg:lm_inexact, on the GPU.  Vector kernels stream the R^(2n) vectors once
// and leave per-block FP64 partial sums; one-block finalize kernels reduce
// them in a fixed order and run the scalar logic in FP64 (CG alpha/beta,
// stopping test, damping lambda, forcing term eta, gain ratio rho, mu update,
// acceptance, the end of an outer iteration).  Every launch of an LM attempt
// can be predicated on a flag of the device state (linearising now, attempt
// running, PCG still running, warm start, step accepted) and returns at once
// when it is clear, so one fixed launch sequence serves every attempt of every
// problem without host synchronisation (and can be captured in a graph).
#include <cmath>

#include "lm_internal.hpp"

namespace ptlm {

__device__ __forceinline__ double rdot(float2 a, float2 b) {
  return (double)a.x * (double)b.x + (double)a.y * (double)b.y;
}

// z = M^{-1} r for the PCG preconditioner of this attempt (per real coordinate), from the entry's
// App. B diagonal d (read when the preconditioner or the damping uses it) and its learned,
// exact or estimated diagonal l (preconditioner codes 2 and up)
__device__ __forceinline__ bool minv_reads_diag(const LMArgs& a) {
  return a.prm.precond == 1 || (a.prm.precond >= 2 && a.prm.scaling);
}
__device__ __forceinline__ float2 minv_of(const LMArgs& a, float2 r, double lam, float2 d, float2 l) {
  if (a.prm.precond == 1) {
    if (a.prm.scaling) {
      const float s = (float)(1.0 + lam);
      return make_float2(r.x / (s * d.x), r.y / (s * d.y));
    }
    return make_float2(r.x / (d.x + (float)lam), r.y / (d.y + (float)lam));
  }
  if (a.prm.precond >= 2) {  // learned, exact or estimated Dg(G), plus lambda D
    const float2 D = a.prm.scaling ? d : make_float2(1.f, 1.f);
    return make_float2(r.x / fmaf((float)lam, D.x, l.x), r.y / fmaf((float)lam, D.y, l.y));
  }
  return r;
}
__device__ __forceinline__ float2 apply_minv(const LMArgs& a, size_t i, float2 r, double lam) {
  const float2 d = minv_reads_diag(a) ? a.diag[i] : make_float2(1.f, 1.f);
  const float2 l = a.prm.precond >= 2 ? a.learned[i] : make_float2(0.f, 0.f);
  return minv_of(a, r, lam, d, l);
}

// eq:projection for the sets of eq:constraints: clamp the magnitude of an object entry to
// o_max and of a probe entry to p_max (the phase is kept)
__device__ __forceinline__ float2 project_entry(const LMArgs& a, size_t i, float2 v) {
  const double m = i < a.nobj ? a.prm.o_max : a.prm.p_max;
  const double r = sqrt((double)v.x * v.x + (double)v.y * v.y);
  if (r <= m) return v;
  const double s = m / r;
  return make_float2((float)(v.x * s), (float)(v.y * s));
}

__device__ __forceinline__ float2 apply_D(const LMArgs& a, size_t i, float2 v) {
  if (a.prm.scaling) {
    const float2 d = a.diag[i];
    return make_float2(d.x * v.x, d.y * v.y);
  }
  return v;
}

// Entries [lo, hi) that the running step works on: every entry, or for the alternating
// update (alg:alt_LM_ptycho) the block of the current sub-step (object [0, nobj), probe
// [nobj, n)).
struct Range {
  size_t lo, hi;
};
__device__ __forceinline__ Range active_range(const LMArgs& a) {
  if (!a.prm.alternate) return Range{0, a.n};
  return a.st->block ? Range{a.nobj, a.n} : Range{0, a.nobj};
}

__device__ __forceinline__ bool flag_clear(const LMArgs& a, int flag) {
  return flag >= 0 && reinterpret_cast<const int*>(a.st)[flag] == 0;
}

// Sum of partials[i * 4 + col], i < count, over one 256-thread block in a fixed order: each
// thread sums a strided share, then a tree through LDS.  Every block that calls it, and the
// one-block finalize kernels, obtain the same value bit for bit.
__device__ __forceinline__ double block_sum_partials(const double* partials, int count, int col) {
  __shared__ double sh[256];
  double acc = 0.0;
  // (unrolled so that a thread's loads are in flight together; the sum keeps its order)
#pragma unroll 4
  for (int i = threadIdx.x; i < count; i += 256) acc += partials[i * 4 + col];
  __syncthreads();
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// PCG iteration `iter` keeps r.z in scal[SC_RZ + iter % 2] (no block of a kernel overwrites
// what another block of it still reads).
template <int OP>
__device__ __forceinline__ void vec_body(const LMArgs& a, int flag, int bid, int nblk, int iter) {
  if (flag_clear(a, flag)) return;
  const double lam = a.st->lambda;
  const bool warm = a.st->use_warm != 0;
  // V_CG_STEP: alpha = r.z / p^T A p from the parts the product's sums left (what a finalize
  //            kernel would do)
  // V_P_STEP:  beta = r'.z' / r.z from V_CG_STEP's partials, and the PCG stopping test
  float alpha = 0.f, beta = 0.f;
  if constexpr (OP == V_CG_STEP) {
    const double pap = block_sum_partials(a.partials, a.pap_count, 0);
    const bool curv = pap > 0.0 && isfinite(pap);
    const double al = curv ? a.scal[SC_RZ + (iter & 1)] / pap : 0.0;
    if (bid == 0 && threadIdx.x == 0) {
      ptlm_lm_state& st = *a.st;
      st.products += 1;
      st.pap = pap;
      if (curv) st.alpha = al;
      else st.cg_active = 0;  // non-positive curvature: keep the current iterate
    }
    if (!curv) return;
    alpha = (float)al;
  } else if constexpr (OP == V_P_STEP) {
    const double rz = block_sum_partials(a.partials, a.vec_blocks, 2);
    const double rr = block_sum_partials(a.partials, a.vec_blocks, 3);
    const double be = rz / a.scal[SC_RZ + (iter & 1)];
    if (bid == 0 && threadIdx.x == 0) {
      ptlm_lm_state& st = *a.st;
      const ptlm_lm_params& p = a.prm;
      a.scal[SC_RZ + ((iter + 1) & 1)] = rz;
      st.beta_cg = be;
      st.rz = rz;
      st.rr = rr;
      st.cg_iters += 1;
      st.cg_total += 1;
      st.cg_active = (st.cg_iters < p.cg_max && sqrt(rr) > st.eta * st.gnorm) ? 1 : 0;
      if (a.cg_flags)
        __hip_atomic_store(a.cg_flags + st.cg_iters, st.cg_active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    beta = (float)be;
  }
  double acc0 = 0.0, acc1 = 0.0;
  double acc2 = 0.0, acc3 = 0.0;  // V_GNORM_DMAX: the diagonal's block maxima
  // steps of the PCG recurrence and of the projected plug-in touch the active block only;
  // V_CG_INIT and V_WARM_P clear the rest of their vectors, V_TRIAL keeps it at the iterate
  constexpr bool BLOCK = OP == V_CG_STEP || OP == V_P_STEP || OP == V_PROJ || OP == V_LS_DIR ||
                         OP == V_LS_NEG;
  const Range act = active_range(a);
  const size_t lo = BLOCK ? act.lo : 0, hi = BLOCK ? act.hi : a.n;
  const size_t stride = (size_t)nblk * blockDim.x;
  constexpr bool PCG = OP == V_CG_STEP || OP == V_P_STEP;
  if constexpr (PCG) {
    // the PCG recurrence: a thread's entries i, i + stride, ... in groups of four, every load of a
    // group issued before its arithmetic (the same entries and the same order of the sums)
    constexpr int U = 4;
    const bool rd = minv_reads_diag(a), rl = a.prm.precond >= 2;
    for (size_t i0 = lo + (size_t)bid * blockDim.x + threadIdx.x; i0 < hi; i0 += U * stride) {
      float2 p[U], q[U], x[U], r[U], d[U], l[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t i = i0 + u * stride;
        if (i >= hi) continue;
        p[u] = a.p[i];
        if constexpr (OP == V_P_STEP) {
          q[u] = a.z[i];
        } else {
          q[u] = a.Ap[i];
        }
        if constexpr (OP == V_CG_STEP) {
          x[u] = a.dx[i];
          r[u] = a.r[i];
          d[u] = rd ? a.diag[i] : make_float2(1.f, 1.f);
          l[u] = rl ? a.learned[i] : make_float2(0.f, 0.f);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t i = i0 + u * stride;
        if (i >= hi) continue;
        if constexpr (OP == V_CG_STEP) {
          float2 xx = x[u], rr = r[u];
          xx.x = fmaf(alpha, p[u].x, xx.x);
          xx.y = fmaf(alpha, p[u].y, xx.y);
          rr.x = fmaf(-alpha, q[u].x, rr.x);
          rr.y = fmaf(-alpha, q[u].y, rr.y);
          const float2 z = minv_of(a, rr, lam, d[u], l[u]);
          a.dx[i] = xx;
          a.r[i] = rr;
          a.z[i] = z;
          acc0 += rdot(rr, z);
          acc1 += rdot(rr, rr);
        } else {
          a.p[i] = make_float2(fmaf(beta, p[u].x, q[u].x), fmaf(beta, p[u].y, q[u].y));
        }
      }
    }
  }
  for (size_t i = lo + (size_t)bid * blockDim.x + threadIdx.x; !PCG && i < hi; i += stride) {
    if constexpr (OP == V_GNORM) {  // ||g_O||^2, ||g_P||^2
      const float2 g = a.g[i];
      if (i < a.nobj) acc0 += rdot(g, g);
      else acc1 += rdot(g, g);
    } else if constexpr (OP == V_GNORM_DMAX) {  // the sums of V_GNORM and the App. B diagonal's maxima
      const float2 g = a.g[i];
      const float2 d = a.diag[i];
      const double m = fmax((double)d.x, (double)d.y);
      if (i < a.nobj) {
        acc0 += rdot(g, g);
        acc2 = fmax(acc2, m);
      } else {
        acc1 += rdot(g, g);
        acc3 = fmax(acc3, m);
      }
    } else if constexpr (OP == V_SAME) {  // entries of the iterate that differ from the last trial point
      const float2 z = i < a.nobj ? a.O[i] : a.P[i - a.nobj];
      const float2 t = a.ztrial[i];
      acc0 += (z.x != t.x || z.y != t.y) ? 1.0 : 0.0;
    } else if constexpr (OP == V_LEARNED) {
      // learned diagonal: on the object part s * exp(clamp(r, log floor, 2)) per real coordinate,
      // s the largest App. B object entry; the probe part is the floored App. B diagonal
      float2 d = a.diag[i];
      if (i < a.nobj) {
        const float sc = (float)a.scal[SC_DMAX_O], lo = (float)log(a.prm.diag_floor);
        d.x = sc * expf(fminf(fmaxf(a.cnn_r[i], lo), 2.f));
        d.y = sc * expf(fminf(fmaxf(a.cnn_r[a.nobj + i], lo), 2.f));
      }
      a.xdiag[i] = d;
    } else if constexpr (OP == V_WARM_P) {  // the warm-start vector restricted to the active block
      const bool in = i >= act.lo && i < act.hi;
      a.p[i] = in ? a.prev[i] : make_float2(0.f, 0.f);
    } else if constexpr (OP == V_DIAGFLOOR) {
      const float f = (float)(a.prm.diag_floor * (i < a.nobj ? a.scal[SC_DMAX_O] : a.scal[SC_DMAX_P]));
      const float2 d = a.diag[i];
      a.diag[i] = make_float2(fmaxf(d.x, f), fmaxf(d.y, f));
    } else if constexpr (OP == V_PROJ) {
      a.ztrial[i] = project_entry(a, i, a.ztrial[i]);
    } else if constexpr (OP == V_LS_DIR || OP == V_LS_NEG) {
      // search direction: the projected step s = Pi(z + Delta) - z, or -grad f
      const float2 g = a.g[i];
      float2 d;
      if constexpr (OP == V_LS_DIR) {
        const float2 zt = a.ztrial[i];
        const float2 z = i < a.nobj ? a.Olin[i] : a.Plin[i - a.nobj];
        d = make_float2(zt.x - z.x, zt.y - z.y);
      } else {
        d = make_float2(-g.x, -g.y);
      }
      a.r[i] = d;
      acc0 += rdot(g, d);
      acc1 += rdot(d, d);
    } else if constexpr (OP == V_LS_CAND) {
      const float2 z = i < a.nobj ? a.Olin[i] : a.Plin[i - a.nobj];
      float2 c = z;
      if (i >= act.lo && i < act.hi) {
        const float2 d = a.r[i];
        const float al = (float)a.st->ls_alpha;
        c = make_float2(fmaf(al, d.x, z.x), fmaf(al, d.y, z.y));
        if (a.st->ls_proj) c = project_entry(a, i, c);
      }
      a.ztrial[i] = c;
    } else if constexpr (OP == V_XMAX) {
      const float2 d = a.xdiag[i];
      const double m = fmax((double)d.x, (double)d.y);
      if (i < a.nobj) acc0 = fmax(acc0, m);
      else acc1 = fmax(acc1, m);
    } else if constexpr (OP == V_XFLOOR) {
      const float f = (float)(a.prm.diag_floor * (i < a.nobj ? a.scal[SC_XMAX_O] : a.scal[SC_XMAX_P]));
      const float2 d = a.xdiag[i];
      a.xdiag[i] = make_float2(fmaxf(d.x, f), fmaxf(d.y, f));
    } else if constexpr (OP == V_CG_INIT) {
      if (i < act.lo || i >= act.hi) {  // outside the active block: Delta = r = z = p = 0
        const float2 zero = make_float2(0.f, 0.f);
        a.dx[i] = zero;
        a.r[i] = zero;
        a.z[i] = zero;
        a.p[i] = zero;
        continue;
      }
      const float2 g = a.g[i];
      float2 r;
      if (warm) {
        const float2 ap = a.Ap[i];
        a.dx[i] = a.prev[i];
        r = make_float2(-g.x - ap.x, -g.y - ap.y);
      } else {
        a.dx[i] = make_float2(0.f, 0.f);
        r = make_float2(-g.x, -g.y);
      }
      const float2 z = apply_minv(a, i, r, lam);
      a.r[i] = r;
      a.z[i] = z;
      a.p[i] = z;
      acc0 += rdot(r, z);
      acc1 += rdot(r, r);
    } else if constexpr (OP == V_TRIAL) {
      const float2 x = a.dx[i];
      const float2 base = i < a.nobj ? a.O[i] : a.P[i - a.nobj];
      a.ztrial[i] = make_float2(base.x + x.x, base.y + x.y);
      const float2 dd = apply_D(a, i, x);
      const float2 g = a.g[i];
      acc0 += (double)x.x * (lam * (double)dd.x - (double)g.x) + (double)x.y * (lam * (double)dd.y - (double)g.y);
    }
  }
  if constexpr (OP == V_SAME) {
    // object-only problems: the probe the trial used is P_lin's copy of the caller's probe
    if (a.Pcur) {
      const size_t M = (size_t)a.nprobe;
      for (size_t i = (size_t)bid * blockDim.x + threadIdx.x; i < M; i += stride) {
        const float2 x = a.Pcur[i], y = a.Plin[i];
        acc0 += (x.x != y.x || x.y != y.y) ? 1.0 : 0.0;
      }
    }
  }
  constexpr bool MAXR = OP == V_XMAX;
  constexpr bool SUMS = OP == V_GNORM || MAXR || OP == V_CG_INIT || OP == V_CG_STEP ||
                        OP == V_TRIAL || OP == V_LS_DIR || OP == V_LS_NEG || OP == V_SAME;
  if constexpr (SUMS) {
    __shared__ double sh[256][2];
    sh[threadIdx.x][0] = acc0;
    sh[threadIdx.x][1] = acc1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        if constexpr (MAXR) {
          sh[threadIdx.x][0] = fmax(sh[threadIdx.x][0], sh[threadIdx.x + w][0]);
          sh[threadIdx.x][1] = fmax(sh[threadIdx.x][1], sh[threadIdx.x + w][1]);
        } else {
          sh[threadIdx.x][0] += sh[threadIdx.x + w][0];
          sh[threadIdx.x][1] += sh[threadIdx.x + w][1];
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      // V_CG_STEP leaves its sums in columns 2, 3: every block still reads the p.Ap parts in
      // column 0
      constexpr int c = OP == V_CG_STEP ? 2 : 0;
      a.partials[bid * 4 + c] = sh[0][0];
      a.partials[bid * 4 + c + 1] = sh[0][1];
    }
  }
  if constexpr (OP == V_GNORM_DMAX) {
    // columns 0, 1 summed as by V_GNORM, columns 2, 3 the maxima
    __shared__ double sh4[256][4];
    sh4[threadIdx.x][0] = acc0;
    sh4[threadIdx.x][1] = acc1;
    sh4[threadIdx.x][2] = acc2;
    sh4[threadIdx.x][3] = acc3;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        sh4[threadIdx.x][0] += sh4[threadIdx.x + w][0];
        sh4[threadIdx.x][1] += sh4[threadIdx.x + w][1];
        sh4[threadIdx.x][2] = fmax(sh4[threadIdx.x][2], sh4[threadIdx.x + w][2]);
        sh4[threadIdx.x][3] = fmax(sh4[threadIdx.x][3], sh4[threadIdx.x + w][3]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0)
      for (int c = 0; c < 4; ++c) a.partials[bid * 4 + c] = sh4[0][c];
  }
}

template <int OP>
__global__ __launch_bounds__(256) void vec_kernel(LMArgs a, int flag, int iter) {
  vec_body<OP>(a, flag, blockIdx.x, gridDim.x, iter);
}

template <int OP>
__global__ __launch_bounds__(256) void vec_batch_kernel(const LMJob* __restrict__ jobs,
                                                        const int* __restrict__ job_of_block, int flag, int iter) {
  const LMJob& J = jobs[job_of_block[blockIdx.x]];
  vec_body<OP>(J.a, flag, (int)blockIdx.x - J.block0, J.a.vec_blocks, iter);
}

__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

// sigma_t of the surrogate metric (App. E): s0 * 1e-6^(t / (T - 1)) for t < T, then 0
__device__ __forceinline__ double surrogate_sigma(const ptlm_lm_params& p, int t) {
  if (p.surrogate_T <= 0 || t >= p.surrogate_T) return 0.0;
  if (p.surrogate_T == 1) return p.surrogate_s0;
  return p.surrogate_s0 * pow(1e-6, (double)t / (double)(p.surrogate_T - 1));
}

// The projected plug-in's line search starts; with no step size to try (ls_max = 0) z_t is kept.
__device__ __forceinline__ void ls_start(ptlm_lm_state& st, const ptlm_lm_params& p) {
  if (p.ls_max > 0) {
    st.ls_on = 1;
  } else {
    st.ls_keep = 1;
    st.ls_alpha = 0.0;
    st.ls_branch = -1;
  }
}

// One block: reduce `count` partials (fixed order), then run the scalar step.
template <int OP>
__device__ __forceinline__ void fin_body(const LMArgs& a, int count, int flag) {
  if (flag_clear(a, flag)) return;
  // F_LIN_DMAX also takes the maxima V_GNORM_DMAX leaves in columns 2, 3
  constexpr bool BOTH = OP == F_LIN_DMAX;
  __shared__ double sh[256][BOTH ? 4 : 2];
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  constexpr bool MAXR = OP == F_XMAX;
  for (int i = threadIdx.x; i < count; i += 256) {
    if constexpr (MAXR) {
      acc0 = fmax(acc0, a.partials[i * 4]);
      acc1 = fmax(acc1, a.partials[i * 4 + 1]);
    } else {
      acc0 += a.partials[i * 4];
      acc1 += a.partials[i * 4 + 1];
    }
    if constexpr (BOTH) {
      acc2 = fmax(acc2, a.partials[i * 4 + 2]);
      acc3 = fmax(acc3, a.partials[i * 4 + 3]);
    }
  }
  sh[threadIdx.x][0] = acc0;
  sh[threadIdx.x][1] = acc1;
  if constexpr (BOTH) {
    sh[threadIdx.x][2] = acc2;
    sh[threadIdx.x][3] = acc3;
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      if constexpr (MAXR) {
        sh[threadIdx.x][0] = fmax(sh[threadIdx.x][0], sh[threadIdx.x + w][0]);
        sh[threadIdx.x][1] = fmax(sh[threadIdx.x][1], sh[threadIdx.x + w][1]);
      } else {
        sh[threadIdx.x][0] += sh[threadIdx.x + w][0];
        sh[threadIdx.x][1] += sh[threadIdx.x + w][1];
      }
      if constexpr (BOTH) {
        sh[threadIdx.x][2] = fmax(sh[threadIdx.x][2], sh[threadIdx.x + w][2]);
        sh[threadIdx.x][3] = fmax(sh[threadIdx.x][3], sh[threadIdx.x + w][3]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double s0 = sh[0][0], s1 = sh[0][1];
  ptlm_lm_state& st = *a.st;
  const ptlm_lm_params& p = a.prm;
  if constexpr (OP == F_ATTEMPT) {
    // an attempt runs while the outer-iteration budget lasts and no non-finite value was met;
    // it linearises first when the previous attempt was accepted (or at the start), or when
    // the surrogate term of the metric (App. E) changed with the outer iteration
    st.alive = (st.t < st.t_max && st.status != PTLM_ENUMERIC) ? 1 : 0;
    bool sigma_changed = false;
    if (st.alive) {
      const double sg = surrogate_sigma(p, st.t);
      if (sg != st.sigma) {
        st.sigma = sg;
        st.need_lin = 1;
        sigma_changed = true;
      }
    }
    st.lin_now = (st.alive && st.need_lin) ? 1 : 0;
    // a linearisation kept from the accepted trial point is adopted unless the surrogate term
    // changed (F_ADOPT also checks that the iterate is that point)
    st.tile_now = (st.lin_now && !(a.adopt_ok && !sigma_changed)) ? 1 : 0;
    if (st.alive && st.iter_done) {  // a new outer iteration (sub-step) starts: no rejections yet
      st.retries = 0;
      st.iter_done = 0;
      if (p.alternate) {  // alg:alt_LM_ptycho: the other block, with its own damping
        st.block ^= 1;
        const double m = st.mu;
        st.mu = st.mu_alt;
        st.mu_alt = m;
      }
    }
    st.cg_active = 0;
    st.accepted = 0;
    st.acc_o = 0;
    st.acc_p = 0;
    st.use_warm = 0;
    st.ls_dir = 0;
    st.ls_neg = 0;
    st.ls_on = 0;
    st.ls_take = 0;
    st.ls_keep = 0;
  } else if constexpr (OP == F_LIN || OP == F_LIN_DMAX) {
    // f and ||grad_zeta ell||^2 from the linearisation, ||g||^2 from V_GNORM (or V_GNORM_DMAX,
    // with the App. B diagonal's block maxima)
    if constexpr (BOTH) {
      a.scal[SC_DMAX_O] = sh[0][2];
      a.scal[SC_DMAX_P] = sh[0][3];
    }
    st.f = a.scal[SC_F];
    st.resid_norm = sqrt(a.scal[SC_L1SQ]);
    a.scal[SC_G2_O] = s0;
    a.scal[SC_G2_P] = s1;
    st.gnorm = sqrt(s0 + s1);
    st.nonfinite = (finite_d(st.f) && finite_d(st.gnorm)) ? 0 : 1;
    if (st.nonfinite) {
      st.status = PTLM_ENUMERIC;
      st.alive = 0;
    }
    st.need_lin = 0;
    st.retries = 0;
  } else if constexpr (OP == F_XMAX) {
    a.scal[SC_XMAX_O] = s0;
    a.scal[SC_XMAX_P] = s1;
  } else if constexpr (OP == F_ADOPT) {
    if (st.lin_now && s0 != 0.0) st.tile_now = 1;  // the iterate is not the kept point
  } else if constexpr (OP == F_PJ_CHECK) {
    // alg:projected_LM after an accepted step Delta from z_t: the projected point
    // Pi(z_t + Delta) (in the trial buffer, its loss reduced here) is taken when it cuts f
    // below gamma f(z_t); otherwise the projected step is tried as a search direction
    st.ls_iter = 0;
    st.ls_alpha = 1.0;
    if (s0 < p.gamma * st.f) {
      st.ls_take = 1;
      st.ls_branch = 0;
    } else {
      st.ls_dir = 1;
    }
  } else if constexpr (OP == F_LS_DIR) {
    // s = Pi(z_t + Delta) - z_t: line search along s when it is a sufficient descent
    // direction, g.s <= -tau_s ||s||^p_s; else along -grad f with projected candidates
    st.ls_dir = 0;
    if (s0 <= -p.tau_s * pow(sqrt(s1), p.p_s)) {
      st.ls_branch = 1;
      st.ls_proj = 0;
      a.scal[SC_LS1] = s1;
      ls_start(st, p);
    } else {
      st.ls_branch = 2;
      st.ls_proj = 1;
      st.ls_neg = 1;
    }
  } else if constexpr (OP == F_LS_NEG) {
    st.ls_neg = 0;
    a.scal[SC_LS1] = s1;  // ||grad f||^2
    ls_start(st, p);
  } else if constexpr (OP == F_LS_TEST) {
    // eq:armijo_criterion at the candidate in the trial buffer (its loss reduced here);
    // the step size halves until it passes or ls_max sizes were tried (then z_t is kept)
    const int tried = st.ls_iter;
    if (s0 <= st.f - p.sigma_ls * st.ls_alpha * a.scal[SC_LS1]) {
      st.ls_on = 0;
      st.ls_take = 1;
    } else {
      st.ls_alpha *= 0.5;
      st.ls_iter += 1;
      if (st.ls_iter >= p.ls_max) {
        st.ls_on = 0;
        st.ls_keep = 1;
        st.ls_alpha = 0.0;
        st.ls_branch = -1;
      }
    }
    if (a.ls_flags) __hip_atomic_store(a.ls_flags + tried, st.ls_on, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  } else if constexpr (OP == F_BEGIN) {
    // alg:lm_inexact: lambda = mu ||grad ell||^nu (D = I) or mu (D = Dg(G)); eta of
    // eq:lma_termination_eta read as min(beta, sqrt(||J^T grad ell||)).  The first attempt
    // of an outer iteration starts PCG from the last accepted step, a retry from zero.
    if (p.alternate) st.gnorm = sqrt(a.scal[st.block ? SC_G2_P : SC_G2_O]);  // ||g|| of the block
    st.lambda = p.scaling ? st.mu : st.mu * pow(st.resid_norm, p.nu);
    st.eta = fmin(p.beta, sqrt(st.gnorm));
    st.cg_iters = 0;
    st.cg_active = 0;
    st.accepted = 0;
    st.alpha = 0.0;
    st.beta_cg = 0.0;
    const int bit = (p.alternate && st.block) ? 2 : 1;
    st.use_warm = (p.warm_start && (st.prev_valid & bit) && st.retries == 0) ? 1 : 0;
  } else if constexpr (OP == F_CG_INIT) {
    if (st.use_warm) st.products += 1;
    st.rz = s0;
    st.rr = s1;
    st.cg_active = (p.cg_max > 0 && sqrt(s1) > st.eta * st.gnorm) ? 1 : 0;
    a.scal[SC_RZ] = s0;
    if (a.cg_flags) __hip_atomic_store(a.cg_flags, st.cg_active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  } else if constexpr (OP == F_PRED) {
    st.pred = 0.5 * s0;  // 1/2 Delta^T (lambda D Delta - g)
  } else if constexpr (OP == F_TRIAL_END) {
    st.attempts += 1;
    st.f_trial = s0;
    const double dfa = st.f - s0;
    const double dfp = st.pred;
    double rho = -INFINITY;
    if (dfp > 0.0 && finite_d(dfa) && finite_d(dfp)) {
      rho = dfa / dfp;
      if (!finite_d(rho)) rho = -INFINITY;
    }
    st.rho = rho;
    const double mu = st.mu;
    if (rho > 0.75) {
      st.mu = fmax(mu / p.kappa, p.mu_min);
      st.accepted = 1;
    } else if (rho > 0.25) {
      st.accepted = 1;
    } else if (rho > p.rho_min) {
      st.mu = p.kappa * mu;
      st.accepted = 1;
    } else {
      st.mu = p.kappa * mu;
      st.accepted = 0;
      st.retries += 1;
    }
    st.cg_active = 0;
    // the outer iteration ends with the sub-step of the probe in the alternating update
    const int last = !p.alternate || st.block == 1;
    if (st.accepted) {
      // the outer iteration (sub-step) ends with a step; the next attempt re-linearises at z + Delta
      const int bit = (p.alternate && st.block) ? 2 : 1;
      st.acc_o = (!p.alternate || st.block == 0) ? 1 : 0;
      st.acc_p = (!p.alternate || st.block == 1) ? 1 : 0;
      st.need_lin = 1;
      st.prev_valid |= bit;
      st.t += last;
      st.iter_done = 1;
      st.status = PTLM_OK;
    } else if (st.retries >= p.retry_max) {
      // every retry rejected: the outer iteration (sub-step) ends without moving (linearisation kept)
      st.t += last;
      st.iter_done = 1;
      st.status = PTLM_ENOTACCEPTED;
    }
  } else if constexpr (OP == F_INIT) {
    st = ptlm_lm_state{};
    st.mu = p.mu0;
    st.mu_alt = p.mu0;
    st.sigma = surrogate_sigma(p, 0);
    st.need_lin = 1;
    st.t_max = a.t_max;
    st.status = PTLM_OK;
  }
}

template <int OP>
__global__ __launch_bounds__(256) void fin_kernel(LMArgs a, int count, int flag) {
  fin_body<OP>(a, count, flag);
}

template <int OP>
__global__ __launch_bounds__(256) void fin_batch_kernel(const LMJob* __restrict__ jobs, int count_kind, int flag) {
  const LMJob& J = jobs[blockIdx.x];
  const int count = count_kind == 1 ? J.a.vec_blocks : (count_kind == 2 ? J.a.tile_grid : 0);
  fin_body<OP>(J.a, count, flag);
}

template <int OP>
static hipError_t vlaunch(const LMArgs& a, int flag, int iter, hipStream_t s) {
  hipLaunchKernelGGL(vec_kernel<OP>, dim3(a.vec_blocks), dim3(256), 0, s, a, flag, iter);
  return hipGetLastError();
}
template <int OP>
static hipError_t flaunch(const LMArgs& a, int count, int flag, hipStream_t s) {
  hipLaunchKernelGGL(fin_kernel<OP>, dim3(1), dim3(256), 0, s, a, count, flag);
  return hipGetLastError();
}
template <int OP>
static hipError_t vblaunch(const LMJob* jobs, const int* jb, int nb, int flag, int iter, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(vec_batch_kernel<OP>, dim3(nb), dim3(256), 0, s, jobs, jb, flag, iter);
  return hipGetLastError();
}
template <int OP>
static hipError_t fblaunch(const LMJob* jobs, int nj, int kind, int flag, hipStream_t s) {
  if (nj <= 0) return hipSuccess;
  hipLaunchKernelGGL(fin_batch_kernel<OP>, dim3(nj), dim3(256), 0, s, jobs, kind, flag);
  return hipGetLastError();
}

#define PTLM_VEC_CASES(X)                                                                                 \
  X(V_GNORM) X(V_DIAGFLOOR) X(V_CG_INIT) X(V_CG_STEP) X(V_P_STEP) X(V_TRIAL) X(V_XMAX) \
  X(V_XFLOOR) X(V_PROJ) X(V_LS_DIR) X(V_LS_NEG) X(V_LS_CAND) X(V_WARM_P) X(V_SAME) X(V_LEARNED) X(V_GNORM_DMAX)
#define PTLM_FIN_CASES(X)                                                                                 \
  X(F_ATTEMPT) X(F_LIN) X(F_XMAX) X(F_BEGIN) X(F_CG_INIT) X(F_PRED) X(F_TRIAL_END) \
  X(F_INIT) X(F_ADOPT) X(F_PJ_CHECK) X(F_LS_DIR) X(F_LS_NEG) X(F_LS_TEST) X(F_LIN_DMAX)

hipError_t launch_vec(int op, const LMArgs& a, int flag, hipStream_t s, int iter) {
  switch (op) {
#define C_(OP) case OP: return vlaunch<OP>(a, flag, iter, s);
    PTLM_VEC_CASES(C_)
#undef C_
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fin(int op, const LMArgs& a, int count, int flag, hipStream_t s) {
  switch (op) {
#define C_(OP) case OP: return flaunch<OP>(a, count, flag, s);
    PTLM_FIN_CASES(C_)
#undef C_
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_vec_batch(int op, const LMJob* jobs, const int* jb, int nb, int flag, hipStream_t s, int iter) {
  switch (op) {
#define C_(OP) case OP: return vblaunch<OP>(jobs, jb, nb, flag, iter, s);
    PTLM_VEC_CASES(C_)
#undef C_
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fin_batch(int op, const LMJob* jobs, int nj, int kind, int flag, hipStream_t s) {
  switch (op) {
#define C_(OP) case OP: return fblaunch<OP>(jobs, nj, kind, flag, s);
    PTLM_FIN_CASES(C_)
#undef C_
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ptlm
