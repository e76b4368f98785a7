// Small convolutional network that predicts the PCG preconditioner diagonal (a project
// addition to the method): direct 3x3 "same" convolutions with LDS-staged input tiles and
// weights, their data and weight gradients, a masked squared-error loss, Adam, the feature
// maps it reads on the object grid, and the assembly of the learned diagonal.
//
// Tensor layout: NCHW float32.  Parameter vector: for each layer W (Cout, Cin, 3, 3) then b.
#include <cmath>

#include "cnn_internal.hpp"
#include "dft.hpp"

namespace ptlm {

constexpr int CT = 16;  // output tile side (pixels) per block

// y[n,o,i,j] = b[o] + sum_{c,u,v} W[o,c,u,v] x[n,c,i+u-1,j+v-1]; optional ReLU on y and an
// optional multiplicative mask (mask > 0) on y.  Weights are read from wt laid out
// [c][u*3+v][o] (see transform kernels).  Grid: (ceil(w/16), ceil(h/16), n), 256 threads.
template <int COUT>
__global__ __launch_bounds__(256) void conv_kernel(const float* __restrict__ x, int cin, int h, int w,
                                                   const float* __restrict__ wt, const float* __restrict__ b,
                                                   float* __restrict__ y, int relu, const float* __restrict__ mask) {
  __shared__ float s_in[CNN_CMAX][CT + 2][CT + 3];
  __shared__ float4 s_w[CNN_CMAX * 9 * (COUT / 4 > 0 ? COUT / 4 : 1)];
  const int n = blockIdx.z;
  const int X0 = blockIdx.x * CT, Y0 = blockIdx.y * CT;
  const size_t plane = (size_t)h * w;
  const float* xn = x + (size_t)n * cin * plane;
  for (int i = threadIdx.x; i < cin * (CT + 2) * (CT + 2); i += 256) {
    const int c = i / ((CT + 2) * (CT + 2)), r = i % ((CT + 2) * (CT + 2));
    const int yy = Y0 + r / (CT + 2) - 1, xx = X0 + r % (CT + 2) - 1;
    s_in[c][r / (CT + 2)][r % (CT + 2)] =
        (yy >= 0 && yy < h && xx >= 0 && xx < w) ? xn[c * plane + (size_t)yy * w + xx] : 0.f;
  }
  constexpr int C4 = COUT / 4 > 0 ? COUT / 4 : 1;
  const float4* wt4 = reinterpret_cast<const float4*>(wt);
  for (int i = threadIdx.x; i < cin * 9 * C4; i += 256) s_w[i] = wt4[i];
  __syncthreads();
  const int ty = threadIdx.x / CT, tx = threadIdx.x % CT;
  float acc[COUT];
#pragma unroll
  for (int o = 0; o < COUT; ++o) acc[o] = b[o];
  for (int c = 0; c < cin; ++c) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float xv = s_in[c][ty + k / 3][tx + k % 3];
      const float4* wv = &s_w[(c * 9 + k) * C4];
#pragma unroll
      for (int q = 0; q < C4; ++q) {
        const float4 ww = wv[q];
        acc[4 * q + 0] = fmaf(ww.x, xv, acc[4 * q + 0]);
        if (4 * q + 1 < COUT) acc[4 * q + 1] = fmaf(ww.y, xv, acc[4 * q + 1]);
        if (4 * q + 2 < COUT) acc[4 * q + 2] = fmaf(ww.z, xv, acc[4 * q + 2]);
        if (4 * q + 3 < COUT) acc[4 * q + 3] = fmaf(ww.w, xv, acc[4 * q + 3]);
      }
    }
  }
  const int yy = Y0 + ty, xx = X0 + tx;
  if (yy >= h || xx >= w) return;
  const size_t at = (size_t)yy * w + xx;
  float* yn = y + (size_t)n * COUT * plane;
  const float* mn = mask ? mask + (size_t)n * COUT * plane : nullptr;
#pragma unroll
  for (int o = 0; o < COUT; ++o) {
    float val = relu ? fmaxf(acc[o], 0.f) : acc[o];
    if (mn && !(mn[o * plane + at] > 0.f)) val = 0.f;
    yn[o * plane + at] = val;
  }
}

// The same convolution for 32 output channels on the FP32 matrix cores: an implicit GEMM
// y[o, p] = b[o] + sum_q A[o, q] B[q, p] over the 16 x 16 output pixels p of a block, with
// q = (tap k, input channel c) in the order k * CIN_P + c (CIN_P = cin rounded up to 4, 8, 16
// or 32; padded channels are zero).  Each wavefront owns 64 pixels (rows 4 w .. 4 w + 3 of the
// tile) as two 32-pixel column blocks of v_mfma_f32_32x32x2_f32 (32 channels x 32 pixels,
// 2 values of q per instruction).  Lane l supplies A[l % 32][2 j + l / 32] (a weight, from LDS)
// and B[2 j + l / 32][l % 32] (an input pixel of channel 2 j + l / 32 at tap k, from the LDS
// tile with halo), and register r of its result holds channel 8 (r / 4) + 4 (l / 32) + r % 4 of
// pixel l % 32.  Exact FP32 products and sums, in another order than conv_kernel.
constexpr int CP = CT + 3;             // LDS row pitch of the input tile
constexpr int CPL = (CT + 2) * CP;     // LDS plane of one channel
typedef float v16f_c __attribute__((ext_vector_type(16)));

template <int CIN_P>
constexpr size_t conv32_lds_bytes() {
  return (size_t)(CIN_P * CPL + 9 * CIN_P * 32) * sizeof(float);
}

template <int CIN_P>
__global__ __launch_bounds__(256, 2) void conv32_mfma_kernel(const float* __restrict__ x, int cin, int h, int w,
                                                             const float* __restrict__ wt,
                                                             const float* __restrict__ b, float* __restrict__ y,
                                                             int relu, const float* __restrict__ mask) {
  extern __shared__ float smem_c[];
  float* s_in = smem_c;                  // [CIN_P][CT + 2][CP]
  float* s_w = smem_c + CIN_P * CPL;     // [9][CIN_P][32]: s_w[(k CIN_P + c) 32 + o] = W[o][c][k]
  const int n = blockIdx.z;
  const int X0 = blockIdx.x * CT, Y0 = blockIdx.y * CT;
  const size_t plane = (size_t)h * w;
  const float* xn = x + (size_t)n * cin * plane;
  for (int i = threadIdx.x; i < CIN_P * (CT + 2) * (CT + 2); i += 256) {
    const int c = i / ((CT + 2) * (CT + 2)), r = i % ((CT + 2) * (CT + 2));
    const int ry = r / (CT + 2), rx = r % (CT + 2);
    const int yy = Y0 + ry - 1, xx = X0 + rx - 1;
    s_in[c * CPL + ry * CP + rx] =
        (c < cin && yy >= 0 && yy < h && xx >= 0 && xx < w) ? xn[c * plane + (size_t)yy * w + xx] : 0.f;
  }
  for (int i = threadIdx.x; i < 9 * CIN_P * 32; i += 256) {
    const int o = i & 31, c = (i >> 5) % CIN_P, k = (i >> 5) / CIN_P;
    s_w[i] = c < cin ? wt[(c * 9 + k) * 32 + o] : 0.f;
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gq = lane >> 5, lo = lane & 31;
  const float* wa = s_w + gq * 32 + lo;
  const float* xb0 = s_in + gq * CPL + (4 * wv + (lo >> 4)) * CP + (lo & 15);  // rows 4 w, 4 w + 1
  const float* xb1 = xb0 + 2 * CP;                                            // rows 4 w + 2, 4 w + 3
  v16f_c acc0 = {}, acc1 = {};
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int koff = (k / 3) * CP + (k % 3);
#pragma unroll
    for (int j = 0; j < CIN_P / 2; ++j) {
      const float av = wa[(k * CIN_P + 2 * j) * 32];
      const float b0 = xb0[2 * j * CPL + koff];
      const float b1 = xb1[2 * j * CPL + koff];
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b1, acc1, 0, 0, 0);
    }
  }
  const int xx = X0 + (lo & 15);
  float* yn = y + (size_t)n * 32 * plane;
  const float* mn = mask ? mask + (size_t)n * 32 * plane : nullptr;
#pragma unroll
  for (int chk = 0; chk < 2; ++chk) {
    const int yy = Y0 + 4 * wv + 2 * chk + (lo >> 4);
    if (yy >= h || xx >= w) continue;
    const size_t at = (size_t)yy * w + xx;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int o = 8 * (r >> 2) + 4 * gq + (r & 3);
      float val = (chk == 0 ? acc0[r] : acc1[r]) + b[o];
      if (relu) val = fmaxf(val, 0.f);
      if (mn && !(mn[o * plane + at] > 0.f)) val = 0.f;
      yn[o * plane + at] = val;
    }
  }
}

template <int CIN_P>
static hipError_t launch_conv32(const float* x, int n, int cin, int h, int w, const float* wt, const float* b,
                                float* y, int relu, const float* mask, hipStream_t s) {
  static bool attr_set = false;
  constexpr size_t lds = conv32_lds_bytes<CIN_P>();
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void*)conv32_mfma_kernel<CIN_P>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  dim3 grid((w + CT - 1) / CT, (h + CT - 1) / CT, n);
  hipLaunchKernelGGL(conv32_mfma_kernel<CIN_P>, grid, dim3(256), lds, s, x, cin, h, w, wt, b, y, relu, mask);
  return hipGetLastError();
}

// forward weights W[o][c][k] -> wt[c][k][o4] (o padded to a multiple of 4 with zeros)
__global__ void wt_forward_kernel(const float* W, int cout, int cin, int cpad, float* wt) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= cin * 9 * cpad) return;
  const int o = i % cpad, k = (i / cpad) % 9, c = i / (cpad * 9);
  wt[i] = o < cout ? W[(o * cin + c) * 9 + k] : 0.f;
}
// data-gradient weights: flipped kernel, channels swapped: wt[o][k][c] = W[o][c][8-k]
// (the "input" of the transposed conv is indexed by o, its output by c)
__global__ void wt_backward_kernel(const float* W, int cout, int cin, int cpad, float* wt) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= cout * 9 * cpad) return;
  const int c = i % cpad, k = (i / cpad) % 9, o = i / (cpad * 9);
  wt[i] = c < cin ? W[(o * cin + c) * 9 + (8 - k)] : 0.f;
}

// Partial weight / bias gradients of one 16x16 tile of one image:
//   gW[o,c,u,v] = sum gz[n,o,i,j] a[n,c,i+u-1,j+v-1],   gb[o] = sum gz[n,o,i,j]
// written to part[block][cout*cin*9 + cout] (reduced over blocks in a fixed order).
__global__ __launch_bounds__(256) void conv_wgrad_kernel(const float* __restrict__ a, int cin, int h, int w,
                                                         const float* __restrict__ gz, int cout,
                                                         float* __restrict__ part) {
  __shared__ float s_a[CNN_CMAX][CT + 2][CT + 3];
  __shared__ float s_g[CNN_CMAX][CT][CT + 1];
  const int n = blockIdx.z;
  const int X0 = blockIdx.x * CT, Y0 = blockIdx.y * CT;
  const size_t plane = (size_t)h * w;
  for (int i = threadIdx.x; i < cin * (CT + 2) * (CT + 2); i += 256) {
    const int c = i / ((CT + 2) * (CT + 2)), r = i % ((CT + 2) * (CT + 2));
    const int yy = Y0 + r / (CT + 2) - 1, xx = X0 + r % (CT + 2) - 1;
    s_a[c][r / (CT + 2)][r % (CT + 2)] =
        (yy >= 0 && yy < h && xx >= 0 && xx < w) ? a[((size_t)n * cin + c) * plane + (size_t)yy * w + xx] : 0.f;
  }
  for (int i = threadIdx.x; i < cout * CT * CT; i += 256) {
    const int o = i / (CT * CT), r = i % (CT * CT);
    const int yy = Y0 + r / CT, xx = X0 + r % CT;
    s_g[o][r / CT][r % CT] = (yy < h && xx < w) ? gz[((size_t)n * cout + o) * plane + (size_t)yy * w + xx] : 0.f;
  }
  __syncthreads();
  const int nw = cout * cin * 9;
  const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  float* out = part + blk * (size_t)(nw + cout);
  for (int e = threadIdx.x; e < nw + cout; e += 256) {
    float acc = 0.f;
    if (e < nw) {
      const int o = e / (cin * 9), c = (e / 9) % cin, k = e % 9, u = k / 3, v = k % 3;
      for (int i = 0; i < CT; ++i)
#pragma unroll 4
        for (int j = 0; j < CT; ++j) acc = fmaf(s_g[o][i][j], s_a[c][i + u][j + v], acc);
    } else {
      const int o = e - nw;
      for (int i = 0; i < CT; ++i)
        for (int j = 0; j < CT; ++j) acc += s_g[o][i][j];
    }
    out[e] = acc;
  }
}

// g[e] = sum over blocks of part[b][e]  (fixed order, FP64 accumulation)
__global__ void reduce_blocks_kernel(const float* part, int nblk, int len, float* g) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= len) return;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += part[(size_t)b * len + e];
  g[e] = (float)acc;
}

// per-block partial sums of mask and mask*(r-t)^2 (FP64)
__global__ __launch_bounds__(256) void loss_partial_kernel(const float* r, const float* t, const float* mask,
                                                           size_t len, double* part) {
  __shared__ double sh[256][2];
  double a0 = 0.0, a1 = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (size_t)gridDim.x * 256) {
    const double m = mask[i] > 0.f ? 1.0 : 0.0;
    const double d = (double)r[i] - (double)t[i];
    a0 += m;
    a1 += m * d * d;
  }
  sh[threadIdx.x][0] = a0;
  sh[threadIdx.x][1] = a1;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sh[threadIdx.x][0] += sh[threadIdx.x + s][0];
      sh[threadIdx.x][1] += sh[threadIdx.x + s][1];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x * 2] = sh[0][0];
    part[blockIdx.x * 2 + 1] = sh[0][1];
  }
}

// scal[0] = count, scal[1] = loss = sum mask (r-t)^2 / (2 count)
__global__ __launch_bounds__(256) void loss_final_kernel(const double* part, int nb, double* scal) {
  __shared__ double sh[256][2];
  double a0 = 0.0, a1 = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a0 += part[2 * i];
    a1 += part[2 * i + 1];
  }
  sh[threadIdx.x][0] = a0;
  sh[threadIdx.x][1] = a1;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sh[threadIdx.x][0] += sh[threadIdx.x + s][0];
      sh[threadIdx.x][1] += sh[threadIdx.x + s][1];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double cnt = sh[0][0] > 1.0 ? sh[0][0] : 1.0;
    scal[0] = cnt;
    scal[1] = sh[0][1] / (2.0 * cnt);
  }
}

// gz = mask (r - t) / count
__global__ void loss_grad_kernel(const float* r, const float* t, const float* mask, size_t len,
                                 const double* scal, float* gz) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  gz[i] = mask[i] > 0.f ? (float)(((double)r[i] - (double)t[i]) / scal[0]) : 0.f;
}

__global__ void adam_kernel(size_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------------------
// features on the object grid (from the handle's linearisation probe and positions):
//   f0 = sum_k S_k^T |P|^2 / max,   f1 = (sum_k S_k^T |P|^4 / sum_k S_k^T |P|^2) / max|P|^2,
//   f2 = (sum_k S_k^T |P|^2 arg P / sum_k S_k^T |P|^2) / pi
__global__ __launch_bounds__(256) void feat_raw_kernel(Geometry g, float* feat) {
  __shared__ int2 s_pos[256];
  const int X = blockIdx.x * 16 + (threadIdx.x & 15);
  const int Y = blockIdx.y * 16 + (threadIdx.x >> 4);
  const bool in = X < g.nx && Y < g.ny;
  const int tile = blockIdx.y * g.otiles_x + blockIdx.x;
  const int b = g.ptile_ptr[tile], e = g.ptile_ptr[tile + 1];
  double s2 = 0.0, s4 = 0.0, sph = 0.0;
  for (int c0 = b; c0 < e; c0 += 256) {
    const int cnt = min(256, e - c0);
    __syncthreads();
    if (threadIdx.x < cnt) s_pos[threadIdx.x] = g.pos[g.ptile_pos[c0 + threadIdx.x]];
    __syncthreads();
    if (in) {
      for (int i = 0; i < cnt; ++i) {
        const int2 r = s_pos[i];
        const int my = Y - r.x, mx = X - r.y;
        if ((unsigned)my < (unsigned)g.my && (unsigned)mx < (unsigned)g.mx) {
          const float2 p = g.P_lin[my * g.mx + mx];
          const double q = (double)p.x * p.x + (double)p.y * p.y;
          s2 += q;
          s4 += q * q;
          sph += q * atan2((double)p.y, (double)p.x);
        }
      }
    }
  }
  if (!in) return;
  const size_t N = (size_t)g.ny * g.nx, n = (size_t)Y * g.nx + X;
  feat[n] = (float)s2;
  feat[N + n] = s2 > 0.0 ? (float)(s4 / s2) : 0.f;
  feat[2 * N + n] = s2 > 0.0 ? (float)(sph / s2 / M_PI) : 0.f;
}

// one block: max of feat[0..N) and of |P|^2 -> scal[0], scal[1]
__global__ __launch_bounds__(1024) void feat_max_kernel(Geometry g, const float* feat, double* scal) {
  __shared__ float sh[1024][2];
  const size_t N = (size_t)g.ny * g.nx;
  float a = 0.f, p = 0.f;
  for (size_t i = threadIdx.x; i < N; i += 1024) a = fmaxf(a, feat[i]);
  for (int i = threadIdx.x; i < g.my * g.mx; i += 1024) {
    const float2 q = g.P_lin[i];
    p = fmaxf(p, q.x * q.x + q.y * q.y);
  }
  sh[threadIdx.x][0] = a;
  sh[threadIdx.x][1] = p;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sh[threadIdx.x][0] = fmaxf(sh[threadIdx.x][0], sh[threadIdx.x + s][0]);
      sh[threadIdx.x][1] = fmaxf(sh[threadIdx.x][1], sh[threadIdx.x + s][1]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scal[0] = sh[0][0];
    scal[1] = sh[0][1];
  }
}

__global__ void feat_norm_kernel(size_t N, float* feat, const double* scal) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const float a = scal[0] > 0.0 ? (float)(1.0 / scal[0]) : 0.f;
  const float p = scal[1] > 0.0 ? (float)(1.0 / scal[1]) : 0.f;
  feat[i] *= a;
  feat[N + i] *= p;
}

// learned diagonal: object part s * exp(clamp(r, log floor, 2)), both coordinates from the two
// output channels, with s = scal[0] the largest entry of the paper's object diagonal (only the
// scale comes from App. B; the shape is the network's).  Probe part (joint): the paper's
// diagonal floored at floor * its block maximum scal[1].  d holds the paper diagonal on entry
// (2n floats, interleaved).
__global__ void learned_diag_kernel(size_t N, size_t n_all, float* d, const float* r, const double* scal,
                                    double floor_frac) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_all) return;
  float2 v = reinterpret_cast<float2*>(d)[i];
  if (i < N) {
    const float sc = (float)scal[0], lo = (float)log(floor_frac);
    v.x = sc * expf(fminf(fmaxf(r[i], lo), 2.f));
    v.y = sc * expf(fminf(fmaxf(r[N + i], lo), 2.f));
  } else {
    const float f = (float)(floor_frac * scal[1]);
    v.x = fmaxf(v.x, f);
    v.y = fmaxf(v.y, f);
  }
  reinterpret_cast<float2*>(d)[i] = v;
}

// one block: max over the object and probe blocks of an interleaved diagonal -> scal[0..1]
__global__ __launch_bounds__(1024) void diag_max_kernel(size_t N, size_t n_all, const float* d, double* scal) {
  __shared__ float sh[1024][2];
  float a = 0.f, p = 0.f;
  for (size_t i = threadIdx.x; i < n_all; i += 1024) {
    const float m = fmaxf(d[2 * i], d[2 * i + 1]);
    if (i < N) a = fmaxf(a, m);
    else p = fmaxf(p, m);
  }
  sh[threadIdx.x][0] = a;
  sh[threadIdx.x][1] = p;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sh[threadIdx.x][0] = fmaxf(sh[threadIdx.x][0], sh[threadIdx.x + s][0]);
      sh[threadIdx.x][1] = fmaxf(sh[threadIdx.x][1], sh[threadIdx.x + s][1]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scal[0] = sh[0][0];
    scal[1] = sh[0][1];
  }
}

// ---------------------------------------------------------------------------------------
static int padc(int c) { return (c + 3) / 4 * 4; }

hipError_t launch_conv(const float* x, int n, int cin, int h, int w, const float* wt, const float* b, float* y,
                       int cout, int relu, const float* mask, hipStream_t s) {
  // 32 output channels: the matrix-core form
  if (cout == 32 && cin <= 32) {
    if (cin <= 4) return launch_conv32<4>(x, n, cin, h, w, wt, b, y, relu, mask, s);
    if (cin <= 8) return launch_conv32<8>(x, n, cin, h, w, wt, b, y, relu, mask, s);
    if (cin <= 16) return launch_conv32<16>(x, n, cin, h, w, wt, b, y, relu, mask, s);
    return launch_conv32<32>(x, n, cin, h, w, wt, b, y, relu, mask, s);
  }
  dim3 grid((w + CT - 1) / CT, (h + CT - 1) / CT, n);
  switch (cout) {
    case 2: hipLaunchKernelGGL(conv_kernel<2>, grid, dim3(256), 0, s, x, cin, h, w, wt, b, y, relu, mask); break;
    case 3: hipLaunchKernelGGL(conv_kernel<3>, grid, dim3(256), 0, s, x, cin, h, w, wt, b, y, relu, mask); break;
    case 4: hipLaunchKernelGGL(conv_kernel<4>, grid, dim3(256), 0, s, x, cin, h, w, wt, b, y, relu, mask); break;
    case 8: hipLaunchKernelGGL(conv_kernel<8>, grid, dim3(256), 0, s, x, cin, h, w, wt, b, y, relu, mask); break;
    case 16: hipLaunchKernelGGL(conv_kernel<16>, grid, dim3(256), 0, s, x, cin, h, w, wt, b, y, relu, mask); break;
    case 32: hipLaunchKernelGGL(conv_kernel<32>, grid, dim3(256), 0, s, x, cin, h, w, wt, b, y, relu, mask); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_wt(const float* W, int cout, int cin, float* wt, bool backward, hipStream_t s) {
  if (!backward) {
    const int total = cin * 9 * padc(cout);
    hipLaunchKernelGGL(wt_forward_kernel, dim3((total + 255) / 256), dim3(256), 0, s, W, cout, cin, padc(cout), wt);
  } else {
    const int total = cout * 9 * padc(cin);
    hipLaunchKernelGGL(wt_backward_kernel, dim3((total + 255) / 256), dim3(256), 0, s, W, cout, cin, padc(cin), wt);
  }
  return hipGetLastError();
}

hipError_t launch_wgrad(const float* a, int n, int cin, int h, int w, const float* gz, int cout, float* part,
                        float* g, hipStream_t s) {
  dim3 grid((w + CT - 1) / CT, (h + CT - 1) / CT, n);
  hipLaunchKernelGGL(conv_wgrad_kernel, grid, dim3(256), 0, s, a, cin, h, w, gz, cout, part);
  const int len = cout * cin * 9 + cout;
  const int nblk = grid.x * grid.y * grid.z;
  hipLaunchKernelGGL(reduce_blocks_kernel, dim3((len + 255) / 256), dim3(256), 0, s, part, nblk, len, g);
  return hipGetLastError();
}

hipError_t launch_loss(const float* r, const float* t, const float* mask, size_t len, double* part, double* scal,
                       float* gz, hipStream_t s) {
  const int nb = 256;
  hipLaunchKernelGGL(loss_partial_kernel, dim3(nb), dim3(256), 0, s, r, t, mask, len, part);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, s, part, nb, scal);
  if (gz) hipLaunchKernelGGL(loss_grad_kernel, dim3((len + 255) / 256), dim3(256), 0, s, r, t, mask, len, scal, gz);
  return hipGetLastError();
}

hipError_t launch_adam(size_t n, float* p, const float* g, float* m, float* v, int step, float lr, float b1,
                       float b2, float eps, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, p, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_features(const Geometry& g, float* feat, double* scal, hipStream_t s) {
  hipLaunchKernelGGL(feat_raw_kernel, dim3(g.otiles_x, g.otiles_y), dim3(256), 0, s, g, feat);
  hipLaunchKernelGGL(feat_max_kernel, dim3(1), dim3(1024), 0, s, g, feat, scal);
  const size_t N = (size_t)g.ny * g.nx;
  hipLaunchKernelGGL(feat_norm_kernel, dim3((N + 255) / 256), dim3(256), 0, s, N, feat, scal);
  return hipGetLastError();
}

hipError_t launch_learned_diag(const Geometry& g, float* d, const float* r, double* scal, double floor_frac,
                               hipStream_t s) {
  const size_t N = (size_t)g.ny * g.nx;
  const size_t n_all = N + (g.joint ? (size_t)g.my * g.mx : 0);
  hipError_t e = launch_diag_paper(g, d, g.joint ? d + 2 * N : nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_max_kernel, dim3(1), dim3(1024), 0, s, N, n_all, d, scal);
  hipLaunchKernelGGL(learned_diag_kernel, dim3((n_all + 255) / 256), dim3(256), 0, s, N, n_all, d, r, scal,
                     floor_frac);
  return hipGetLastError();
}

}  // namespace ptlm
