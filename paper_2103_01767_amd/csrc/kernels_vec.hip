// Gather-side reductions that finish the overlap-add, FP64 partial sums and the
// analytic GGN diagonal.  All sums run in a fixed order (no atomics), so every
// result is bit-reproducible run to run.
#include "dft.hpp"
#include "internal.hpp"

namespace ptlm {

// out_O[n] = sum over segments s whose strip covers n of strip_s[n]   (S_k^T overlap-add)
//          [+ lam * D .* v].  Strips are only read: the tile kernels rewrite them each call.
// One block per 16x16 object tile: the tile's segment list (boxes, offsets) is staged in
// LDS, then every thread sums its pixel over the list with independent loads.
constexpr int OBJ_LIST = 256;
// p.Ap of a PCG iteration, folded into the sums that finish its product: each block of the
// object and probe sums adds the real inner product of v and out over its pixels (FP64; the
// pixels of the block the alternating update leaves inactive count zero) and stores it at
// pap[4 * pidx] for the next vector step to sum in a fixed order.
__device__ __forceinline__ double pdot(float2 a, float2 b) {
  return (double)a.x * (double)b.x + (double)a.y * (double)b.y;
}
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ __forceinline__ void obj_reduce_body(const Geometry& g, float2* out, float lam_h, const double* lam_dev,
                                                const float* d, const float2* v, const int* pred, int bx, int by,
                                                double* pap = nullptr, const int* pap_block = nullptr, int pidx = 0) {
  if (pred && *pred == 0) return;
  __shared__ int4 s_box[OBJ_LIST];
  __shared__ long long s_off[OBJ_LIST];
  const float lam = lam_dev ? (float)*lam_dev : lam_h;
  const int X = bx * 16 + (threadIdx.x & 15);
  const int Y = by * 16 + (threadIdx.x >> 4);
  const bool in = X < g.nx && Y < g.ny;
  const int tile = by * g.otiles_x + bx;
  const int b = g.otile_ptr[tile], e = g.otile_ptr[tile + 1];
  float2 acc = make_float2(0.f, 0.f);
  for (int c0 = b; c0 < e; c0 += OBJ_LIST) {
    const int cnt = min(OBJ_LIST, e - c0);
    __syncthreads();
    if (threadIdx.x < cnt) {
      const int s = g.otile_seg[c0 + threadIdx.x];
      s_box[threadIdx.x] = g.seg_box[s];
      s_off[threadIdx.x] = g.seg_off[s];
    }
    __syncthreads();
    // batches of 8 independent loads (misses read a valid dummy address and are dropped)
    for (int i0 = 0; i0 < cnt; i0 += 8) {
      float2 val[8];
      bool hit[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int i = min(i0 + j, cnt - 1);
        const int4 bx = s_box[i];
        const int ry = Y - bx.x, rx = X - bx.y;
        hit[j] = in && (i0 + j < cnt) && (unsigned)ry < (unsigned)bx.z && (unsigned)rx < (unsigned)bx.w;
        val[j] = g.strips[hit[j] ? s_off[i] + (size_t)ry * bx.w + rx : 0];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (hit[j]) {
          acc.x += val[j].x;
          acc.y += val[j].y;
        }
      }
    }
  }
  const bool dot = pap && v && (!pap_block || *pap_block == 0);
  double pd = 0.0;
  if (in) {
    const size_t n = (size_t)Y * g.nx + X;
    const float2 vv = v && (lam != 0.f || dot) ? v[n] : make_float2(0.f, 0.f);
    if (lam != 0.f && v) {
      if (d) {
        acc.x = fmaf(lam * d[2 * n], vv.x, acc.x);
        acc.y = fmaf(lam * d[2 * n + 1], vv.y, acc.y);
      } else {
        acc.x = fmaf(lam, vv.x, acc.x);
        acc.y = fmaf(lam, vv.y, acc.y);
      }
    }
    out[n] = acc;
    if (dot) pd = pdot(vv, acc);
  }
  if (pap) {
    // every thread of the block reaches this barrier (none has returned)
    __shared__ double wsum[4];
    pd = wave_sum(pd);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = pd;
    __syncthreads();
    if (threadIdx.x == 0) pap[(size_t)pidx * 4] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
  }
}

__global__ __launch_bounds__(256) void obj_reduce_kernel(Geometry g, float2* out, float lam_h, const double* lam_dev,
                                                         const float* d, const float2* v, const int* pred) {
  obj_reduce_body(g, out, lam_h, lam_dev, d, v, pred, blockIdx.x, blockIdx.y);
}

// Probe-sized sums of the per-segment probe partials, 64 pixels per block.  One pass,
// out_P[m] = sum_s probe_part[s][m] [+ lam * D .* v], unless the probe gives few blocks and there
// are many segments (prb_chunk_count); then two passes in place: pass one (one block per 64
// pixels and chunk) replaces row c * PRB_CHUNK of probe_part by the sum of its chunk's rows,
// pass two sums the chunk rows.  Every sum is split four ways over its rows and the four parts
// are added in a fixed order, so the result depends only on the probe size and the segment
// count.  The partials are scratch of one product (every per-position kernel rewrites them), so
// overwriting them loses nothing.
__device__ __forceinline__ float2 rows_sum4(const float2* p, int count, size_t stride, bool valid, int grp, int lane,
                                            float2 (*sh)[64]) {
  float2 acc = make_float2(0.f, 0.f);
  if (valid) {
#pragma unroll 8
    for (int i = grp; i < count; i += 4) {
      const float2 val = p[(size_t)i * stride];
      acc.x += val.x;
      acc.y += val.y;
    }
  }
  sh[grp][lane] = acc;
  __syncthreads();
  return cadd(cadd(sh[0][lane], sh[1][lane]), cadd(sh[2][lane], sh[3][lane]));
}

// pass one of a two-pass reduction: block (bx, chunk c)
__device__ __forceinline__ void probe_chunk_body(const Geometry& g, const int* pred, int bx, int c) {
  if (pred && *pred == 0) return;
  __shared__ float2 sh[4][64];
  const int M = g.my * g.mx;
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int m = bx * 64 + lane;
  const int s0 = c * PRB_CHUNK, cnt = min(PRB_CHUNK, g.nseg - s0);
  float2* row = g.probe_part + (size_t)s0 * M + m;
  // every read of the chunk's rows is done before the barrier inside, the one write after it
  const float2 acc = rows_sum4(row, cnt, M, m < M, grp, lane, sh);
  if (grp == 0 && m < M) *row = acc;
}

__device__ __forceinline__ void probe_reduce_body(const Geometry& g, float2* out, float lam_h, const double* lam_dev,
                                                  const float* d, const float2* v, const int* pred, int bx,
                                                  double* pap = nullptr, const int* pap_block = nullptr,
                                                  int pidx = 0) {
  if (pred && *pred == 0) return;
  __shared__ float2 sh[4][64];
  const float lam = lam_dev ? (float)*lam_dev : lam_h;
  const int M = g.my * g.mx;
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int m = bx * 64 + lane;
  const int nch = prb_chunk_count(M, g.nseg);
  const bool two = nch > 0;
  float2 acc = rows_sum4(g.probe_part + m, two ? nch : g.nseg,
                         two ? (size_t)PRB_CHUNK * M : (size_t)M, m < M, grp, lane, sh);
  if (grp != 0) return;  // the first wavefront holds the sums
  const bool dot = pap && v && (!pap_block || *pap_block != 0);
  double pd = 0.0;
  if (m < M) {
    const float2 vv = v && (lam != 0.f || dot) ? v[m] : make_float2(0.f, 0.f);
    if (lam != 0.f && v) {
      if (d) {
        acc.x = fmaf(lam * d[2 * m], vv.x, acc.x);
        acc.y = fmaf(lam * d[2 * m + 1], vv.y, acc.y);
      } else {
        acc.x = fmaf(lam, vv.x, acc.x);
        acc.y = fmaf(lam, vv.y, acc.y);
      }
    }
    out[m] = acc;
    if (dot) pd = pdot(vv, acc);
  }
  if (pap) {
    pd = wave_sum(pd);
    if (lane == 0) pap[(size_t)pidx * 4] = pd;
  }
}

// The object and probe sums of one product or gradient in one launch: blocks 0 .. nprb - 1 run
// the probe sum (started first: each adds every segment's partial), the rest the object
// tiles, with the bodies of the two separate kernels (same results).
// With pap, block b also leaves its part of p.Ap (p = v) at pap[4 b].
__global__ __launch_bounds__(256) void pair_reduce_kernel(Geometry g, float2* outO, float2* outP, float lam_h,
                                                          const double* lam_dev, const float* dO, const float* dP,
                                                          const float2* vO, const float2* vP, const int* pred,
                                                          int nprb, double* pap, const int* pap_block) {
  const int b = blockIdx.x;
  if (b < nprb) {
    probe_reduce_body(g, outP, lam_h, lam_dev, dP, vP, pred, b, pap, pap_block, b);
  } else {
    const int l = b - nprb;
    obj_reduce_body(g, outO, lam_h, lam_dev, dO, vO, pred, l % g.otiles_x, l / g.otiles_x, pap, pap_block, b);
  }
}

__global__ __launch_bounds__(256) void probe_chunk_kernel(Geometry g, const int* pred) {
  probe_chunk_body(g, pred, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void probe_reduce_kernel(Geometry g, float2* out, float lam_h, const double* lam_dev,
                                                           const float* d, const float2* v, const int* pred) {
  probe_reduce_body(g, out, lam_h, lam_dev, d, v, pred, blockIdx.x);
}

__global__ __launch_bounds__(256) void probe_chunk_batch_kernel(const RedJob* __restrict__ jobs,
                                                                const int* __restrict__ job_of_block) {
  const RedJob& J = jobs[job_of_block[blockIdx.x]];
  const int l = (int)blockIdx.x - J.block1;
  const int pb = (J.g.my * J.g.mx + 63) / 64;
  probe_chunk_body(J.g, J.pred, l % pb, l / pb);
}

// batched form of pair_reduce_kernel: blocks 0 .. nbp - 1 over the probe job table, the rest
// over the object job table
__global__ __launch_bounds__(256) void pair_reduce_batch_kernel(const RedJob* __restrict__ objjobs,
                                                                const int* __restrict__ objjb,
                                                                const RedJob* __restrict__ prbjobs,
                                                                const int* __restrict__ prbjb, int nbp) {
  const int b = blockIdx.x;
  if (b < nbp) {
    const RedJob& J = prbjobs[prbjb[b]];
    const int l = b - J.block0;
    probe_reduce_body(J.g, J.outP, 0.f, J.lam_dev, J.dP, J.vP, J.pred, l, J.pap, J.pap_block, l);
  } else {
    const RedJob& J = objjobs[objjb[b - nbp]];
    const int l = b - nbp - J.block0;
    obj_reduce_body(J.g, J.outO, 0.f, J.lam_dev, J.dO, J.vO, J.pred, l % J.g.otiles_x, l / J.g.otiles_x, J.pap,
                    J.pap_block, J.pap_base + l);
  }
}

// out[j] = sum_i partials[i*4 + j], j < nout, fixed-order tree
__device__ __forceinline__ void sum_partials_body(const double* partials, int count, double* out, int nout) {
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

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* partials, int count, double* out,
                                                           int nout, const int* pred) {
  if (pred && *pred == 0) return;
  sum_partials_body(partials, count, out, nout);
}

// one block per job: the tile kernel's partials of that problem
__global__ __launch_bounds__(256) void sum_partials_batch_kernel(const RedJob* __restrict__ jobs, int nout) {
  const RedJob& J = jobs[blockIdx.x];
  if (J.pred && *J.pred == 0) return;
  sum_partials_body(J.g.partials, J.g.grid, J.sums, nout);
}

// App. B diagonal, object part: d_n = (1/2M) sum_{k covering n} trace_k |P[n - r_k]|^2,
// the same weight for the Re and Im coordinates.  One 1024-thread block per 16x16 object
// tile: the tile's position list is staged in LDS, each pixel's sum is split four ways over
// the list and the four parts are added in a fixed order.
constexpr int DIAG_OBJ_THREADS = 1024;
__device__ __forceinline__ void diag_paper_obj_body(const Geometry& g, float* dO, int bx, int by) {
  __shared__ int2 s_pos[OBJ_LIST];
  __shared__ double s_tr[OBJ_LIST];
  __shared__ double s_part[4][256];
  const int px = threadIdx.x & 255, grp = threadIdx.x >> 8;
  const int X = bx * 16 + (px & 15);
  const int Y = by * 16 + (px >> 4);
  const bool in = X < g.nx && Y < g.ny;
  const int tile = by * g.otiles_x + bx;
  const int b = g.ptile_ptr[tile], e = g.ptile_ptr[tile + 1];
  double acc = 0.0;
  for (int c0 = b; c0 < e; c0 += OBJ_LIST) {
    const int cnt = min(OBJ_LIST, e - c0);
    __syncthreads();
    if (threadIdx.x < cnt) {
      const int k = g.ptile_pos[c0 + threadIdx.x];
      s_pos[threadIdx.x] = g.pos[k];
      s_tr[threadIdx.x] = g.trace[k];
    }
    __syncthreads();
    if (in) {
#pragma unroll 4
      for (int i = grp; i < cnt; i += 4) {
        const int2 r = s_pos[i];
        const int my = Y - r.x, mx = X - r.y;
        if ((unsigned)my < (unsigned)g.my && (unsigned)mx < (unsigned)g.mx) {
          const float2 p = g.P_lin[my * g.mx + mx];
          acc += s_tr[i] * (double)fmaf(p.x, p.x, p.y * p.y);
        }
      }
    }
  }
  s_part[grp][px] = acc;
  __syncthreads();
  if (!in || grp != 0) return;
  acc = (s_part[0][px] + s_part[1][px]) + (s_part[2][px] + s_part[3][px]);
  const float val = (float)(acc / (2.0 * g.my * g.mx));
  const size_t n = (size_t)Y * g.nx + X;
  dO[2 * n] = val;
  dO[2 * n + 1] = val;
}

__global__ __launch_bounds__(1024) void diag_paper_obj_batch_kernel(const RedJob* __restrict__ jobs,
                                                                   const int* __restrict__ job_of_block) {
  const RedJob& J = jobs[job_of_block[blockIdx.x]];
  if (J.pred && *J.pred == 0) return;
  const int l = (int)blockIdx.x - J.block0;
  diag_paper_obj_body(J.g, (float*)J.outO, l % J.g.otiles_x, l / J.g.otiles_x);
}

// App. B diagonal, probe part: d_m = (1/2M) sum_k trace_k |O[r_k + m]|^2; one 1024-thread
// block per 64 consecutive pixels (a wavefront reads one 512-byte run of an object row), the
// position sum split 16 ways (k mod 16, in increasing k) and combined in a fixed order.
// Positions and traces are staged in LDS in chunks, so the object read is the only global
// load of the loop.
constexpr int DIAG_PRB_THREADS = 1024;
constexpr int DIAG_PRB_PIX = 64;
constexpr int DIAG_PRB_CHUNK = 1024;  // a multiple of 16: a chunk keeps every group's k order
__device__ __forceinline__ void diag_paper_probe_body(const Geometry& g, float* dP, int bx) {
  __shared__ double sh[16][DIAG_PRB_PIX + 1];
  __shared__ int2 s_pos[DIAG_PRB_CHUNK];
  __shared__ double s_tr[DIAG_PRB_CHUNK];
  const int M = g.my * g.mx;
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int m = bx * DIAG_PRB_PIX + lane;
  const bool in = m < M;
  const float2* Om = g.O_lin + (in ? (size_t)(m / g.mx) * g.nx + m % g.mx : 0);
  double acc = 0.0;
  for (int c0 = 0; c0 < g.K; c0 += DIAG_PRB_CHUNK) {
    const int cnt = min(DIAG_PRB_CHUNK, g.K - c0);
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      s_pos[threadIdx.x] = g.pos[c0 + threadIdx.x];
      s_tr[threadIdx.x] = g.trace[c0 + threadIdx.x];
    }
    __syncthreads();
    if (in) {
#pragma unroll 8
      for (int i = grp; i < cnt; i += 16) {
        const int2 r = s_pos[i];
        const float2 o = Om[(size_t)r.x * g.nx + r.y];
        acc += s_tr[i] * (double)fmaf(o.x, o.x, o.y * o.y);
      }
    }
  }
  sh[grp][lane] = acc;
  __syncthreads();
  if (grp != 0 || !in) return;
  double sum = 0.0;
  for (int q = 0; q < 16; ++q) sum += sh[q][lane];
  const float val = (float)(sum / (2.0 * M));
  dP[2 * m] = val;
  dP[2 * m + 1] = val;
}

// both parts of the App. B diagonal in one launch: blocks 0 .. nprb - 1 the probe part (started
// first: each block walks every position), the rest the object tiles
__global__ __launch_bounds__(1024) void diag_paper_pair_kernel(Geometry g, float* dO, float* dP, const int* pred,
                                                               int nprb) {
  if (pred && *pred == 0) return;
  const int b = blockIdx.x;
  if (b < nprb) {
    diag_paper_probe_body(g, dP, b);
  } else {
    const int l = b - nprb;
    diag_paper_obj_body(g, dO, l % g.otiles_x, l / g.otiles_x);
  }
}

__global__ __launch_bounds__(256) void copy_kernel(const float2* __restrict__ src, float2* __restrict__ dst, size_t n,
                                                   const int* pred) {
  if (pred && *pred == 0) return;
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// up to MAX_COPIES independent copies in one launch; copy c owns blocks first[c] .. first[c+1]-1
struct CopySet {
  CopyItem item[MAX_COPIES];
  int first[MAX_COPIES + 1];
  int count;
};

__global__ __launch_bounds__(256) void copies_kernel(CopySet cs) {
  int c = 0;
  while (c + 1 < cs.count && (int)blockIdx.x >= cs.first[c + 1]) ++c;
  const CopyItem it = cs.item[c];
  if (it.pred && *it.pred == 0) return;
  const int nb = cs.first[c + 1] - cs.first[c];
  const size_t stride = (size_t)nb * 256;
  for (size_t i = (size_t)((int)blockIdx.x - cs.first[c]) * 256 + threadIdx.x; i < it.n; i += stride)
    it.dst[i] = it.src[i];
}

__global__ __launch_bounds__(1024) void diag_paper_probe_batch_kernel(const RedJob* __restrict__ jobs,
                                                                     const int* __restrict__ job_of_block) {
  const RedJob& J = jobs[job_of_block[blockIdx.x]];
  if (J.pred && *J.pred == 0) return;
  diag_paper_probe_body(J.g, (float*)J.outP, (int)blockIdx.x - J.block0);
}

// predicated batched copies: block b copies part of job job_of_block[b]
__global__ __launch_bounds__(256) void copy_batch_kernel(const CopyJob* __restrict__ jobs,
                                                         const int* __restrict__ job_of_block) {
  const CopyJob& J = jobs[job_of_block[blockIdx.x]];
  if (J.pred && *J.pred == 0) return;
  const size_t stride = (size_t)J.nblk * 256;
  for (size_t i = (size_t)((int)blockIdx.x - J.block0) * 256 + threadIdx.x; i < J.n; i += stride)
    J.dst[i] = J.src[i];
}

hipError_t launch_reduce_pair_batch(const RedJob* objjobs, const int* objjb, int nbo, const RedJob* prbjobs,
                                    const int* jb1, int nb1, const int* prbjb, int nbp, hipStream_t s) {
  if (nb1 > 0) {
    hipLaunchKernelGGL(probe_chunk_batch_kernel, dim3(nb1), dim3(256), 0, s, prbjobs, jb1);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nbo + nbp <= 0) return hipSuccess;
  hipLaunchKernelGGL(pair_reduce_batch_kernel, dim3(nbo + nbp), dim3(256), 0, s, objjobs, objjb, prbjobs, prbjb, nbp);
  return hipGetLastError();
}
hipError_t launch_sum_partials_batch(const RedJob* jobs, int njobs, int nout, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(sum_partials_batch_kernel, dim3(njobs), dim3(256), 0, s, jobs, nout);
  return hipGetLastError();
}
hipError_t launch_diag_paper_batch(const RedJob* objjobs, const int* objjb, int nbo, const RedJob* prbjobs,
                                   const int* prbjb, int nbp, hipStream_t s) {
  if (nbo > 0) hipLaunchKernelGGL(diag_paper_obj_batch_kernel, dim3(nbo), dim3(DIAG_OBJ_THREADS), 0, s, objjobs, objjb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nbp <= 0) return e;
  hipLaunchKernelGGL(diag_paper_probe_batch_kernel, dim3(nbp), dim3(DIAG_PRB_THREADS), 0, s, prbjobs, prbjb);
  return hipGetLastError();
}
hipError_t launch_copy_batch(const CopyJob* jobs, const int* jb, int nb, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_batch_kernel, dim3(nb), dim3(256), 0, s, jobs, jb);
  return hipGetLastError();
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
  if (prb_chunk_count(M, g.nseg) > 0) {
    hipLaunchKernelGGL(probe_chunk_kernel, dim3((M + 63) / 64, prb_chunk_count(M, g.nseg)), dim3(256), 0, s, g,
                       pred);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(probe_reduce_kernel, dim3((M + 63) / 64), dim3(256), 0, s, g, outP, (float)lam, lam_dev, dP,
                     vP, pred);
  return hipGetLastError();
}

hipError_t launch_reduce_pair(const Geometry& g, float2* outO, float2* outP, double lam, const double* lam_dev,
                              const float* dO, const float* dP, const float2* vO, const float2* vP, const int* pred,
                              hipStream_t s, double* pap, const int* pap_block) {
  const int M = g.my * g.mx;
  const int nprb = outP ? (M + 63) / 64 : 0;
  if (outP && prb_chunk_count(M, g.nseg) > 0) {
    hipLaunchKernelGGL(probe_chunk_kernel, dim3((M + 63) / 64, prb_chunk_count(M, g.nseg)), dim3(256), 0, s, g,
                       pred);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(pair_reduce_kernel, dim3(nprb + g.otiles_x * g.otiles_y), dim3(256), 0, s, g, outO, outP,
                     (float)lam, lam_dev, dO, dP, vO, vP, pred, nprb, pap, pap_block);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partials, int count, double* out, int nout, hipStream_t s,
                               const int* pred) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partials, count, out, nout, pred);
  return hipGetLastError();
}

hipError_t launch_diag_paper(const Geometry& g, float* dO, float* dP, hipStream_t s, const int* pred) {
  static_assert(DIAG_PRB_THREADS == DIAG_OBJ_THREADS, "one launch runs both diagonal parts");
  const int M = g.my * g.mx;
  const int nprb = dP ? (M + DIAG_PRB_PIX - 1) / DIAG_PRB_PIX : 0;
  hipLaunchKernelGGL(diag_paper_pair_kernel, dim3(nprb + g.otiles_x * g.otiles_y), dim3(DIAG_OBJ_THREADS), 0, s, g,
                     dO, dP, pred, nprb);
  return hipGetLastError();
}

int copy_blocks(size_t n) {
  const size_t b = (n + 2047) / 2048;
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

// d = (first ? 0 : d) + scale (Re u, Im u)^2 per complex entry: one draw's share of the
// stochastic diagonal estimate
__global__ __launch_bounds__(256) void sq_accum_kernel(const float2* __restrict__ u, float2* __restrict__ d, size_t n,
                                                       float scale, int first, const int* pred) {
  if (pred && *pred == 0) return;
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const float2 x = u[i];
    const float2 q = make_float2(scale * x.x * x.x, scale * x.y * x.y);
    if (first) {
      d[i] = q;
    } else {
      const float2 c = d[i];
      d[i] = make_float2(c.x + q.x, c.y + q.y);
    }
  }
}

hipError_t launch_sq_accum(const float2* u, float2* d, size_t n, float scale, int first, const int* pred,
                           hipStream_t s) {
  hipLaunchKernelGGL(sq_accum_kernel, dim3(copy_blocks(n)), dim3(256), 0, s, u, d, n, scale, first, pred);
  return hipGetLastError();
}

hipError_t launch_copy(const float2* src, float2* dst, size_t n, const int* pred, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(copy_blocks(n)), dim3(256), 0, s, src, dst, n, pred);
  return hipGetLastError();
}

hipError_t launch_copies(const CopyItem* items, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > MAX_COPIES) return hipErrorInvalidValue;
  CopySet cs{};
  cs.count = count;
  cs.first[0] = 0;
  for (int c = 0; c < count; ++c) {
    cs.item[c] = items[c];
    cs.first[c + 1] = cs.first[c] + copy_blocks(items[c].n);
  }
  hipLaunchKernelGGL(copies_kernel, dim3(cs.first[count]), dim3(256), 0, s, cs);
  return hipGetLastError();
}

}  // namespace ptlm
