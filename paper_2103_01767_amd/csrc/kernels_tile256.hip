// Per-position tile kernels for 256 x 256 probes (the large-scan regime).
//
// A 256 x 256 complex64 tile is 512 KiB, more than the 160 KiB of LDS, so the 2D
// transform of a position runs in three stages through a private scratch tile in
// global memory (one per workgroup, reused for every position of its segment; it
// stays in the L2 / last-level cache while the workgroup works on it):
//
//   stage 1  four blocks of 64 rows: gather (exit wave or its perturbation), length-256
//            x transform (radix 16 x 16, one LDS exchange inside each wavefront's own
//            four rows), store the rows (kx in natural order) to the scratch tile;
//   stage 2  four blocks of 64 columns: length-256 y transform (radix 16 x 16, one LDS
//            exchange across the workgroup), the per-pixel operation of the op in
//            registers with coalesced reads of the per-position fields, then the
//            inverse y transform and the columns back to the scratch tile;
//   stage 3  four blocks of 64 rows: inverse x transform and the overlap-add S_k^T
//            (Sec. 2) into the segment's private strip and probe slot.
//
// A thread's pixels in stages 1 and 3 are the same (row, rc + 16 j), so the scratch rows
// it writes in stage 1 of the next position are the ones it read in stage 3: no barrier
// is needed between positions.  The per-pixel operations, normalisation (unitary F,
// eq:expected_count), stored phasor field and overlap-add strips are those of the
// smaller tile kernels.
#include "dft.hpp"
#include "internal.hpp"
#include "tile_pixel.hpp"

namespace ptlm {

namespace {
constexpr int S = 256;          // tile side
constexpr int M256 = S * S;
constexpr int WG = 1024;        // threads: 64 rows x 16 (row stages), 64 columns x 16 (column stage)
constexpr int NWAVE = WG / 64;
constexpr int RB = 64;          // rows per row block
constexpr int CB = 64;          // columns per column block
constexpr int LDR = 272;        // LDS pitch of a row in a row block; element (n1, k1) at k1 * 17 + n1
constexpr int LDS_C = RB * LDR; // complex entries of the exchange area (column block needs S * CB)
static_assert(S * CB <= LDS_C, "column block must fit the exchange area");
constexpr int TW_OFF = 224;     // W_256^(n k), n, k < 16, in the geometry's twiddle table

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int xcd_map(int b, int n) {
  if (n % 8 != 0) return b;
  return (b % 8) * (n / 8) + b / 8;
}

__device__ __forceinline__ float2 ld_nt(const float2* p) {
  const double d = __builtin_nontemporal_load(reinterpret_cast<const double*>(p));
  return __builtin_bit_cast(float2, d);
}

// The transform tile is streamed through memory (512 KiB per workgroup never fits its L2
// share): streaming stores and loads leave L2 to the windows and strips that are reused.
__device__ __forceinline__ void st_nt(float2* p, float2 v) {
  __builtin_nontemporal_store(__builtin_bit_cast(double, v), reinterpret_cast<double*>(p));
}

// sum of x over the workgroup, returned to every thread (two barriers)
__device__ __forceinline__ double wg_sum(double x, double* red, int col) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  if ((threadIdx.x & 63) == 0) red[(threadIdx.x >> 6) * 2 + col] = x;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NWAVE; ++w) s += red[w * 2 + col];
  __syncthreads();
  return s;
}
}  // namespace

template <int OP>
__device__ __forceinline__ void tile256_body(const Geometry g, const TileArgs a, int bid, int nblk) {
  constexpr bool FWD_FFT = OP != OP_VJP && OP != OP_VJP_RAND;
  constexpr bool INV_FFT = OP == OP_LINEARIZE || OP == OP_VJP || OP == OP_GGNV || OP == OP_VJP_RAND;
  constexpr bool SCATTER = INV_FFT || OP == OP_DIAG_EXACT;
  constexpr bool SUMS = OP == OP_LOSS || OP == OP_LINEARIZE;
  if (a.predicate && *a.predicate == 0) return;

  extern __shared__ float2 smem[];
  double* red = reinterpret_cast<double*>(smem + LDS_C);  // [NWAVE][2]
  float2* tw = smem + LDS_C + 2 * NWAVE;                  // [16][16]
  for (int i = threadIdx.x; i < 256; i += WG) tw[i] = g.tw[TW_OFF + i];
  __syncthreads();

  const int t = threadIdx.x;
  const int rr = t >> 4, rc = t & 15;  // row stages: row in block, residue / frequency index
  const int cc = t & 63, cs = t >> 6;  // column stage: column in block, residue / frequency index
  const int seg = xcd_map(bid, nblk);
  const int kbeg = g.seg_start[seg], kend = g.seg_start[seg + 1];
  float2* scr = g.scratch + (size_t)bid * M256;
  float2* lrow = smem + rr * LDR;
  const float isq = 1.0f / 256.0f;
  const bool joint = g.joint != 0;
  const float bgv = a.bg_add ? (float)((double)g.background + *a.bg_add) : g.background;
  float2* pslot = g.probe_part + (size_t)seg * M256;
  double s0 = 0.0, s1 = 0.0;

  float2* strip = nullptr;
  int4 box = make_int4(0, 0, 0, 0);
  if constexpr (SCATTER) {
    strip = g.strips + g.seg_off[seg];
    box = g.seg_box[seg];
    if (kend > kbeg) {
      // strip pixels outside the first window are cleared here; the first position stores
      const int2 p0 = g.pos[kbeg];
      const int area = box.z * box.w;
      for (int i = t; i < area; i += WG) {
        const int Y = box.x + i / box.w, X = box.y + i % box.w;
        if ((unsigned)(Y - p0.x) >= (unsigned)S || (unsigned)(X - p0.y) >= (unsigned)S)
          strip[i] = make_float2(0.f, 0.f);
      }
    } else if (joint) {
      for (int i = t; i < M256; i += WG) pslot[i] = make_float2(0.f, 0.f);
    }
  }

  for (int k = kbeg; k < kend; ++k) {
    const int2 pk = g.pos[k];
    const int ry = pk.x, rx = pk.y;
    const size_t base = (size_t)k * M256;
    const bool first = k == kbeg;
    double asum = 0.0;  // OP_DIAG_EXACT: sum |a|^2 over this thread's pixels

    // ================= stage 1: x transforms of the rows -> scratch
    if constexpr (FWD_FFT) {
#pragma unroll 1
      for (int rb = 0; rb < 4; ++rb) {
        const int row = rb * RB + rr;
        float2 v[16];
        if constexpr (OP == OP_DIAG_EXACT) {
          const float2* arow = g.afield + base + row * S + rc;
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const float2 as = arow[16 * j];
            asum += (double)fmaf(as.x, as.x, as.y * as.y);
            v[j] = make_float2(fmaf(as.x, as.x, -as.y * as.y), -2.f * as.x * as.y);
          }
        } else {
          const float2* Orow = a.O + (size_t)(ry + row) * g.nx + rx + rc;
          const float2* Prow = a.P + row * S + rc;
          if constexpr (OP == OP_JVP || OP == OP_GGNV) {
            const float2* Vrow = a.vO + (size_t)(ry + row) * g.nx + rx + rc;
            if (a.vP) {
              const float2* VProw = a.vP + row * S + rc;
#pragma unroll
              for (int jj = 0; jj < 16; jj += 4) {
#pragma unroll
                for (int j = jj; j < jj + 4; ++j)
                  v[j] = cadd(cmul(Prow[16 * j], Vrow[16 * j]), cmul(VProw[16 * j], Orow[16 * j]));
                __builtin_amdgcn_sched_barrier(0);
              }
            } else {
#pragma unroll
              for (int j = 0; j < 16; ++j) v[j] = cmul(Prow[16 * j], Vrow[16 * j]);
            }
          } else {
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = cmul(Prow[16 * j], Orow[16 * j]);
          }
        }
        // x pass 1: DFT16 over n2 (x = rc + 16 n2), twiddle W_256^(rc k1)
        dft16<false>(v);
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[rc * 16 + k1]);
        wave_sync();
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) lrow[k1 * 17 + rc] = v[k1];
        wave_sync();
        // x pass 2: this thread now owns k1 = rc; DFT16 over n1 -> kx = rc + 16 k2
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) v[n1] = lrow[rc * 17 + n1];
        dft16<false>(v);
        float2* srow = scr + row * S + rc;
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) st_nt(srow + 16 * k2, v[k2]);
      }
      __syncthreads();
    }

    // ================= stage 2: columns (y transform, per-pixel op, inverse y transform)
    {
      double tr = 0.0;
#pragma unroll 1
      for (int cb = 0; cb < 4; ++cb) {
        const int kx = cb * CB + cc;
        float2 v[16];
        if constexpr (FWD_FFT) {
          // y pass 1: DFT16 over n2 (y = cs + 16 n2), twiddle W_256^(cs k1)
#pragma unroll
          for (int j = 0; j < 16; ++j) v[j] = ld_nt(scr + (cs + 16 * j) * S + kx);
          dft16<false>(v);
#pragma unroll
          for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[cs * 16 + k1]);
          __syncthreads();
#pragma unroll
          for (int k1 = 0; k1 < 16; ++k1) smem[(k1 * 16 + cs) * CB + cc] = v[k1];
          __syncthreads();
          // y pass 2: this thread owns k1 = cs; DFT16 over n1 -> ky = cs + 16 k2
#pragma unroll
          for (int n1 = 0; n1 < 16; ++n1) v[n1] = smem[(cs * 16 + n1) * CB + cc];
          dft16<false>(v);
        }
        // per-pixel work at (ky, kx) = (cs + 16 r, kx), in groups of four pixels
        if constexpr (OP == OP_DIAG_EXACT) {
#pragma unroll
          for (int r = 0; r < 16; ++r) scr[(cs + 16 * r) * S + kx] = v[r];  // B_k = DFT(conj(a)^2), frequency order
        } else {
          // the metric is read per pixel: specialised copies of this loop spill more
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            if (r % 4 == 0) __builtin_amdgcn_sched_barrier(0);
            const size_t gi = base + (size_t)(cs + 16 * r) * S + kx;
            pixel_op<OP, -1>(g, a, gi, isq, bgv, v[r], s0, s1, tr);
          }
        }
        if constexpr (INV_FFT) {
          // inverse y pass 2: DFT16 over k2 -> n1, conjugate twiddle W_256^(-n1 cs)
          dft16<true>(v);
#pragma unroll
          for (int n1 = 1; n1 < 16; ++n1) v[n1] = cmulc(v[n1], tw[n1 * 16 + cs]);
          __syncthreads();
#pragma unroll
          for (int n1 = 0; n1 < 16; ++n1) smem[(cs * 16 + n1) * CB + cc] = v[n1];
          __syncthreads();
          // inverse y pass 1: this thread owns n1 = cs; DFT16 over k1 -> y = cs + 16 n2
#pragma unroll
          for (int k1 = 0; k1 < 16; ++k1) v[k1] = smem[(k1 * 16 + cs) * CB + cc];
          dft16<true>(v);
#pragma unroll
          for (int j = 0; j < 16; ++j) st_nt(scr + (cs + 16 * j) * S + kx, v[j]);
        }
      }
      if constexpr (OP == OP_LINEARIZE) {
        tr = wg_sum(tr, red, 0);  // trace of the metric Hessian of this position (App. B)
        if (t == 0) g.trace[k] = tr;
      }
      // the column exchange area overlaps every wavefront's row area of stages 1 and 3
      __syncthreads();
    }

    // ================= stage 3: inverse x transforms of the rows + overlap-add
    if constexpr (INV_FFT) {
#pragma unroll 1
      for (int rb = 0; rb < 4; ++rb) {
        const int row = rb * RB + rr;
        float2 v[16];
        const float2* srow = scr + row * S + rc;
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) v[k2] = ld_nt(srow + 16 * k2);
        // inverse x pass 2 (this thread owns k1 = rc): DFT16 over k2 -> n1, W_256^(-n1 rc)
        dft16<true>(v);
#pragma unroll
        for (int n1 = 1; n1 < 16; ++n1) v[n1] = cmulc(v[n1], tw[n1 * 16 + rc]);
        wave_sync();
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) lrow[rc * 17 + n1] = v[n1];
        wave_sync();
        // inverse x pass 1 (this thread owns n1 = rc): DFT16 over k1 -> x = rc + 16 n2
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) v[k1] = lrow[k1 * 17 + rc];
        dft16<true>(v);
        const int Y = ry + row;
        float2* sp = strip + (size_t)(Y - box.x) * box.w + (rx + rc - box.y);
        const float2* Prow = a.P + row * S + rc;
        if (first) {
#pragma unroll
          for (int j = 0; j < 16; ++j) sp[16 * j] = cmulc(v[j], Prow[16 * j]);
        } else {
#pragma unroll
          for (int jj = 0; jj < 16; jj += 4) {
#pragma unroll
            for (int j = jj; j < jj + 4; ++j) sp[16 * j] = cadd(sp[16 * j], cmulc(v[j], Prow[16 * j]));
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        if (joint) {
          const float2* Orow = a.O + (size_t)Y * g.nx + rx + rc;
          float2* pp = pslot + row * S + rc;
          if (first) {
#pragma unroll
            for (int j = 0; j < 16; ++j) pp[16 * j] = cmulc(v[j], Orow[16 * j]);
          } else {
#pragma unroll
            for (int jj = 0; jj < 16; jj += 4) {
#pragma unroll
              for (int j = jj; j < jj + 4; ++j) pp[16 * j] = cadd(pp[16 * j], cmulc(v[j], Orow[16 * j]));
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
      }
    }

    // ================= exact diagonal: terms read at 2m' of B_k (see the smaller kernels)
    if constexpr (OP == OP_DIAG_EXACT) {
      const float A = (float)wg_sum(asum, red, 1);
#pragma unroll 1
      for (int rb = 0; rb < 4; ++rb) {
        const int row = rb * RB + rr;
        const int Y = ry + row;
        float2* sp = strip + (size_t)(Y - box.x) * box.w + (rx + rc - box.y);
        const float2* Prow = a.P + row * S + rc;
        const float2* Orow = a.O + (size_t)Y * g.nx + rx + rc;
        const float2* Brow = scr + ((2 * row) & (S - 1)) * S;
        float2* pp = pslot + row * S + rc;
#pragma unroll 4
        for (int j = 0; j < 16; ++j) {
          const int x = rc + 16 * j;
          const float2 B = Brow[(2 * x) & (S - 1)];
          const float2 q = Prow[16 * j];
          float bse = 0.5f * A * fmaf(q.x, q.x, q.y * q.y);
          float crs = 0.5f * (fmaf(q.x, q.x, -q.y * q.y) * B.x - 2.f * q.x * q.y * B.y);
          const float2 cur = first ? make_float2(0.f, 0.f) : sp[16 * j];
          sp[16 * j] = make_float2(cur.x + bse + crs, cur.y + bse - crs);
          if (joint) {
            const float2 o = Orow[16 * j];
            bse = 0.5f * A * fmaf(o.x, o.x, o.y * o.y);
            crs = 0.5f * (fmaf(o.x, o.x, -o.y * o.y) * B.x - 2.f * o.x * o.y * B.y);
            const float2 c0 = first ? make_float2(0.f, 0.f) : pp[16 * j];
            pp[16 * j] = make_float2(c0.x + bse + crs, c0.y + bse - crs);
          }
        }
      }
      // the next position's stage 2 overwrites B in the scratch tile
      __syncthreads();
    }
  }

  if constexpr (SUMS) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, 64);
      s1 += __shfl_xor(s1, off, 64);
    }
    __syncthreads();
    if ((t & 63) == 0) {
      red[(t >> 6) * 2] = s0;
      red[(t >> 6) * 2 + 1] = s1;
    }
    __syncthreads();
    if (t == 0) {
      double a0 = 0.0, a1 = 0.0;
      for (int w = 0; w < NWAVE; ++w) {
        a0 += red[w * 2];
        a1 += red[w * 2 + 1];
      }
      g.partials[bid * 4 + 0] = a0;
      g.partials[bid * 4 + 1] = a1;
      g.partials[bid * 4 + 2] = 0.0;
      g.partials[bid * 4 + 3] = 0.0;
    }
  }
}

template <int OP>
__global__ __launch_bounds__(WG) void tile256_kernel(Geometry g, TileArgs a) {
  tile256_body<OP>(g, a, blockIdx.x, gridDim.x);
}

template <int OP>
__global__ __launch_bounds__(WG) void tile256_batch_kernel(const TileJob* __restrict__ jobs,
                                                           const int* __restrict__ job_of_block) {
  const TileJob& J = jobs[job_of_block[blockIdx.x]];
  const int b = (int)blockIdx.x - J.block0;
  if (b >= J.g.grid) return;
  tile256_body<OP>(J.g, J.a, b, J.g.grid);
}

size_t tile256_lds_bytes() { return (size_t)LDS_C * sizeof(float2) + NWAVE * 2 * sizeof(double) + 256 * sizeof(float2); }
size_t tile256_scratch_elems() { return (size_t)M256; }

template <int OP>
static hipError_t launch256(const Geometry& g, const TileArgs& a, hipStream_t s) {
  const size_t lds = tile256_lds_bytes();
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)tile256_kernel<OP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((tile256_kernel<OP>), dim3(g.grid), dim3(WG), lds, s, g, a);
  return hipGetLastError();
}

template <int OP>
static hipError_t launch256_batch(const TileJob* jobs, const int* jb, int nb, hipStream_t s) {
  const size_t lds = tile256_lds_bytes();
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)tile256_batch_kernel<OP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((tile256_batch_kernel<OP>), dim3(nb), dim3(WG), lds, s, jobs, jb);
  return hipGetLastError();
}

hipError_t launch_tile256_batch(int op, const TileJob* jobs, const int* jb, int nb, hipStream_t s) {
  switch (op) {
    case OP_LOSS: return launch256_batch<OP_LOSS>(jobs, jb, nb, s);
    case OP_LINEARIZE: return launch256_batch<OP_LINEARIZE>(jobs, jb, nb, s);
    case OP_GGNV: return launch256_batch<OP_GGNV>(jobs, jb, nb, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tile256(const Geometry& g, int op, const TileArgs& a, hipStream_t s) {
  if (g.my != S || g.mx != S || !g.scratch) return hipErrorInvalidValue;
  switch (op) {
    case OP_FORWARD: return launch256<OP_FORWARD>(g, a, s);
    case OP_LOSS: return launch256<OP_LOSS>(g, a, s);
    case OP_LINEARIZE: return launch256<OP_LINEARIZE>(g, a, s);
    case OP_JVP: return launch256<OP_JVP>(g, a, s);
    case OP_VJP: return launch256<OP_VJP>(g, a, s);
    case OP_VJP_RAND: return launch256<OP_VJP_RAND>(g, a, s);
    case OP_GGNV: return launch256<OP_GGNV>(g, a, s);
    case OP_DIAG_EXACT: return launch256<OP_DIAG_EXACT>(g, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ptlm
