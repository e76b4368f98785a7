// Gather-side reductions that finish the overlap-add, FP64 partial sums and the
// analytic GGN diagonal.  All sums run in a fixed order (no atomics), so every
// result is bit-reproducible run to run.
#include "dft.hpp"
#include "internal.hpp"

namespace ptlm {

// out_O[n] = sum over segments s whose strip covers n of strip_s[n]   (S_k^T overlap-add)
//          [+ lam * D .* v]; each strip entry read is reset to zero for the next call.
__global__ __launch_bounds__(256) void obj_reduce_kernel(Geometry g, float2* out, float lam_h, const double* lam_dev,
                                                         const float* d, const float2* v,
                                                         const int* pred) {
  if (pred && *pred == 0) return;
  const float lam = lam_dev ? (float)*lam_dev : lam_h;
  const int X = blockIdx.x * 16 + (threadIdx.x & 15);
  const int Y = blockIdx.y * 16 + (threadIdx.x >> 4);
  const bool in = X < g.nx && Y < g.ny;
  const int tile = blockIdx.y * g.otiles_x + blockIdx.x;
  float2 acc = make_float2(0.f, 0.f);
  const int b = g.otile_ptr[tile], e = g.otile_ptr[tile + 1];
  for (int i = b; i < e; ++i) {
    const int s = g.otile_seg[i];
    const int4 bx = g.seg_box[s];
    if (in && Y >= bx.x && Y < bx.x + bx.z && X >= bx.y && X < bx.y + bx.w) {
      float2* p = g.strips + g.seg_off[s] + (size_t)(Y - bx.x) * bx.w + (X - bx.y);
      acc = cadd(acc, *p);
      *p = make_float2(0.f, 0.f);
    }
  }
  if (!in) return;
  const size_t n = (size_t)Y * g.nx + X;
  if (lam != 0.f && v) {
    const float2 vv = v[n];
    if (d) {
      acc.x = fmaf(lam * d[2 * n], vv.x, acc.x);
      acc.y = fmaf(lam * d[2 * n + 1], vv.y, acc.y);
    } else {
      acc.x = fmaf(lam, vv.x, acc.x);
      acc.y = fmaf(lam, vv.y, acc.y);
    }
  }
  out[n] = acc;
}

// out_P[m] = sum_s probe_part[s][m] [+ lam * D .* v]
__global__ __launch_bounds__(256) void probe_reduce_kernel(Geometry g, float2* out, float lam_h, const double* lam_dev,
                                                           const float* d, const float2* v,
                                                           const int* pred) {
  if (pred && *pred == 0) return;
  const float lam = lam_dev ? (float)*lam_dev : lam_h;
  const int M = g.my * g.mx;
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= M) return;
  float2 acc = make_float2(0.f, 0.f);
  const float2* p = g.probe_part + m;
  for (int s = 0; s < g.nseg; ++s) acc = cadd(acc, p[(size_t)s * M]);
  if (lam != 0.f && v) {
    const float2 vv = v[m];
    if (d) {
      acc.x = fmaf(lam * d[2 * m], vv.x, acc.x);
      acc.y = fmaf(lam * d[2 * m + 1], vv.y, acc.y);
    } else {
      acc.x = fmaf(lam, vv.x, acc.x);
      acc.y = fmaf(lam, vv.y, acc.y);
    }
  }
  out[m] = acc;
}

// out[j] = sum_i partials[i*4 + j], j < nout, fixed-order tree
__global__ __launch_bounds__(256) void sum_partials_kernel(const double* partials, int count, double* out,
                                                           int nout) {
  __shared__ double sh[256][4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < count; i += 256)
    for (int j = 0; j < 4; ++j) acc[j] += partials[i * 4 + j];
  for (int j = 0; j < 4; ++j) sh[threadIdx.x][j] = acc[j];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int j = 0; j < 4; ++j) sh[threadIdx.x][j] += sh[threadIdx.x + w][j];
    __syncthreads();
  }
  if (threadIdx.x < nout) out[threadIdx.x] = sh[0][threadIdx.x];
}

// App. B diagonal, object part: d_n = (1/2M) sum_{k covering n} trace_k |P[n - r_k]|^2,
// the same weight for the Re and Im coordinates.
__global__ __launch_bounds__(256) void diag_paper_obj_kernel(Geometry g, float* dO) {
  const int X = blockIdx.x * 16 + (threadIdx.x & 15);
  const int Y = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (X >= g.nx || Y >= g.ny) return;
  const int tile = blockIdx.y * g.otiles_x + blockIdx.x;
  double acc = 0.0;
  for (int i = g.ptile_ptr[tile]; i < g.ptile_ptr[tile + 1]; ++i) {
    const int k = g.ptile_pos[i];
    const int2 r = g.pos[k];
    const int my = Y - r.x, mx = X - r.y;
    if (my >= 0 && my < g.my && mx >= 0 && mx < g.mx) {
      const float2 p = g.P_lin[my * g.mx + mx];
      acc += g.trace[k] * (double)(p.x * p.x + p.y * p.y);
    }
  }
  const float val = (float)(acc / (2.0 * g.my * g.mx));
  const size_t n = (size_t)Y * g.nx + X;
  dO[2 * n] = val;
  dO[2 * n + 1] = val;
}

// App. B diagonal, probe part: d_m = (1/2M) sum_k trace_k |O[r_k + m]|^2
__global__ __launch_bounds__(256) void diag_paper_probe_kernel(Geometry g, float* dP) {
  const int M = g.my * g.mx;
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= M) return;
  const int my = m / g.mx, mx = m % g.mx;
  double acc = 0.0;
  for (int k = 0; k < g.K; ++k) {
    const int2 r = g.pos[k];
    const float2 o = g.O_lin[(size_t)(r.x + my) * g.nx + r.y + mx];
    acc += g.trace[k] * (double)(o.x * o.x + o.y * o.y);
  }
  const float val = (float)(acc / (2.0 * M));
  dP[2 * m] = val;
  dP[2 * m + 1] = val;
}

hipError_t launch_obj_reduce(const Geometry& g, float2* outO, double lam, const double* lam_dev, const float* dO,
                             const float2* vO, const int* pred, hipStream_t s) {
  hipLaunchKernelGGL(obj_reduce_kernel, dim3(g.otiles_x, g.otiles_y), dim3(256), 0, s, g, outO, (float)lam, lam_dev,
                     dO, vO, pred);
  return hipGetLastError();
}

hipError_t launch_probe_reduce(const Geometry& g, float2* outP, double lam, const double* lam_dev, const float* dP,
                               const float2* vP, const int* pred, hipStream_t s) {
  const int M = g.my * g.mx;
  hipLaunchKernelGGL(probe_reduce_kernel, dim3((M + 255) / 256), dim3(256), 0, s, g, outP, (float)lam, lam_dev, dP,
                     vP, pred);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partials, int count, double* out, int nout, hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partials, count, out, nout);
  return hipGetLastError();
}

hipError_t launch_diag_paper(const Geometry& g, float* dO, float* dP, hipStream_t s) {
  hipLaunchKernelGGL(diag_paper_obj_kernel, dim3(g.otiles_x, g.otiles_y), dim3(256), 0, s, g, dO);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !dP) return e;
  const int M = g.my * g.mx;
  hipLaunchKernelGGL(diag_paper_probe_kernel, dim3((M + 255) / 256), dim3(256), 0, s, g, dP);
  return hipGetLastError();
}

}  // namespace ptlm
