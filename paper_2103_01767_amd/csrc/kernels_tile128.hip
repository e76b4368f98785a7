// 128 x 128 tile kernels: gather -> 2D FFT -> per-pixel op -> inverse 2D FFT -> overlap-add.
//
// Same per-position work as the generic tile kernels (the transform F of eq:expected_count and
// its adjoint around the per-pixel operations of tile_pixel.hpp), arranged for the 128 x 128
// probe so that a position costs two workgroup barriers instead of six:
//
// * 1024 threads (16 wavefronts), 16 complex values per thread.  Wavefront w owns rows
//   8w..8w+7 of the tile in the x passes and columns 8w..8w+7 in the y passes.
// * Each 1D transform of length 128 is a product of a radix-16 and a radix-8 DFT in registers,
//   with the twiddle W_128 between them and an exchange among the 8 lanes of a row (or column)
//   in between.  Those lanes sit in one wavefront, so that exchange needs only the wavefront's
//   own LDS ordering, not a barrier.  Only the two transposes (x -> y after the forward x
//   passes, y -> x after the inverse y passes) take a workgroup barrier; after one, every
//   wavefront reads and writes its own columns (rows) alone until the next.
// * Along x the radix-8 DFT comes first (n = n1 + 16 n2, k = k2 + 8 k1): a lane holds the
//   pixel pairs (2 q, 2 q + 1) + 16 n2 of its row, so the gather and the overlap-add move two
//   adjacent complex values per 16-byte access (a wavefront access covers 8 whole 128-byte
//   lines).  Along y the radix-16 DFT comes first (n = n1 + 8 n2, k = k2 + 16 k1).
// * The exchange tile (152 KiB, layout at `at`) is free of bank conflicts for every exchange of
//   every pass under the LDS bank model measured on gfx950 (32 banks of 4 bytes; a 64-bit
//   access is served per half wavefront, at the cost of the most-hit bank).  The twiddle table
//   is padded to 17 entries a row for the same reason.
// * The probe part of the overlap-add is summed in registers across the segment, so only the
//   object strip is read-modify-written per position (except in the linearisation, which has no
//   registers to spare and read-modify-writes the segment's probe slot as well).
#include "dft.hpp"
#include "internal.hpp"
#include "tile_pixel.hpp"

namespace ptlm {
namespace t128 {

constexpr int L = 128, M = L * L;
constexpr int NTH = 1024;
constexpr int NW = NTH / 64;
constexpr int TW_OFF = 96;  // W_128^(n k), n < 8, k < 16, in the workspace twiddle table
// pixel pairs per lane per batch of gather loads and of overlap-add loads (batches of 2 to 8
// measured the same)
constexpr int NG = 2, NO = 2;

// two adjacent complex values (8-byte aligned: one 16-byte global access)
struct __attribute__((aligned(8))) c2 {
  float2 a, b;
};

// Exchange-tile index of element (r, c).  Rows are LP = 152 complex apart, a row holds its 128
// elements in 142 slots (two spare slots after every 16 columns), and rows are offset by one
// slot when bit 1 or bit 5 of r is set and by eight when bit 4 is.  Every exchange of the
// transform (element sets of the form lane part + loop part, in disjoint bits of r and c) then
// spreads each half wavefront's 32 accesses over the 16 bank pairs exactly twice, and the
// index is a per-lane base plus a compile-time offset, so the LDS accesses take immediate
// offsets.
constexpr int LP = 152, LDS_ELEMS = 127 * LP + 10 + 142;
__device__ __forceinline__ int at(int r, int c) {
  return r * LP + ((r >> 1) & 1) + 8 * ((r >> 4) & 1) + ((r >> 5) & 1) + c + 2 * (c >> 4);
}

constexpr size_t lds_bytes() {
  return (size_t)LDS_ELEMS * sizeof(float2) + 136 * sizeof(float2) + 4 * NW * sizeof(double);
}

template <int OP, int MET>
__device__ __forceinline__ void body(const Geometry g, const TileArgs a, int bid, int nblk) {
  constexpr bool FWD = OP != OP_VJP && OP != OP_VJP_RAND;
  constexpr bool INV = OP == OP_LINEARIZE || OP == OP_VJP || OP == OP_GGNV || OP == OP_VJP_RAND;
  constexpr bool SUMS = OP == OP_LOSS || OP == OP_LINEARIZE;
  if (a.predicate && *a.predicate == 0) return;

  extern __shared__ float2 smem[];
  float2* lds = smem;                                     // exchange tile
  float2* s_tw = smem + LDS_ELEMS;                        // W_128^(n k) at n * 17 + k
  double* red = reinterpret_cast<double*>(s_tw + 136);    // [NW][2] sums, then [2][NW] traces
  double* red_tr = red + 2 * NW;
  for (int i = threadIdx.x; i < 128; i += NTH) s_tw[(i >> 4) * 17 + (i & 15)] = g.tw[TW_OFF + i];
  __syncthreads();

  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane >> 3, lc = lane & 7;
  const int row = 8 * wv + lr;  // x phase: this lane's tile row
  const int col = 8 * wv + lc;  // y phase: this lane's tile column
  const int seg = xcd_block(bid, nblk);
  const int kbeg = g.seg_start[seg], kend = g.seg_start[seg + 1];
  const float isq = rsqrtf((float)M);
  const bool joint = g.joint != 0;
  const float bgv = a.bg_add ? (float)((double)g.background + *a.bg_add) : g.background;

  // probe partial of the overlap-add: accP[e * 8 + n2] <-> probe pixel (row, 2 lc + e + 16 n2).
  // The linearisation, which also keeps the loss sums and streams the counts and the phasor
  // field, has registers for only part of it or none: the groups n2 >= NREG are read-modify-
  // written in the segment's probe slot instead (the first position stores), in the same order
  // of the sums.  Half in registers measured fastest for the Gaussian metric (fewer spills
  // than all, less slot traffic than none); the other metric codes spill more and keep none.
  constexpr int NREG = OP != OP_LINEARIZE ? 8 : (MET == 0 ? 4 : 0);
  float2 accP[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) accP[j] = make_float2(0.f, 0.f);
  double s0 = 0.0, s1 = 0.0;

  // the segment's first position stores into the strip, later ones read-modify-write; strip
  // pixels outside the first window are cleared here
  float2* strip = nullptr;
  int4 box = make_int4(0, 0, 0, 0);
  if constexpr (INV) {
    strip = g.strips + g.seg_off[seg];
    box = g.seg_box[seg];
    if (kend > kbeg) {
      const int2 p0 = g.pos[kbeg];
      const int area = box.z * box.w;
      for (int i = threadIdx.x; i < area; i += NTH) {
        const int Y = box.x + i / box.w, X = box.y + i % box.w;
        if ((unsigned)(Y - p0.x) >= (unsigned)L || (unsigned)(X - p0.y) >= (unsigned)L)
          strip[i] = make_float2(0.f, 0.f);
      }
    }
  }

  // per-lane offsets of the pixel pairs (row, 2 lc + 16 n2) in an object window, the probe and
  // the strip; a position adds a uniform offset
  const size_t lane_o = (size_t)row * g.nx + 2 * lc;
  const int lane_p = row * L + 2 * lc;
  const size_t lane_s = (size_t)row * box.w + 2 * lc;

  for (int k = kbeg; k < kend; ++k) {
    const int2 p = g.pos[k];
    const int ry = p.x, rx = p.y;
    float2 v[16];

    if constexpr (FWD) {
      // ---------------- gather the exit wave (or its perturbation) at pixels (row, 2 lc + e + 16 n2)
      {
        const size_t orow = (size_t)ry * g.nx + rx + lane_o;
        const c2* Oq = reinterpret_cast<const c2*>(a.O + orow);
        const c2* Pq = reinterpret_cast<const c2*>(a.P + lane_p);
        if constexpr (OP == OP_JVP || OP == OP_GGNV) {
          const c2* Vq = reinterpret_cast<const c2*>(a.vO + orow);
          if (a.vP) {
            const c2* VPq = reinterpret_cast<const c2*>(a.vP + lane_p);
#pragma unroll
            for (int nn = 0; nn < 8; nn += NG) {
#pragma unroll
              for (int n2 = nn; n2 < nn + NG; ++n2) {
                const c2 pp = Pq[8 * n2], vv = Vq[8 * n2], vp = VPq[8 * n2], oo = Oq[8 * n2];
                v[n2] = cadd(cmul(pp.a, vv.a), cmul(vp.a, oo.a));
                v[8 + n2] = cadd(cmul(pp.b, vv.b), cmul(vp.b, oo.b));
              }
              __builtin_amdgcn_sched_barrier(0);
            }
          } else {
#pragma unroll
            for (int n2 = 0; n2 < 8; ++n2) {
              const c2 pp = Pq[8 * n2], vv = Vq[8 * n2];
              v[n2] = cmul(pp.a, vv.a);
              v[8 + n2] = cmul(pp.b, vv.b);
            }
          }
        } else {
#pragma unroll
          for (int n2 = 0; n2 < 8; ++n2) {
            const c2 pp = Pq[8 * n2], oo = Oq[8 * n2];
            v[n2] = cmul(pp.a, oo.a);
            v[8 + n2] = cmul(pp.b, oo.b);
          }
        }
      }
      // ---------------- x pass A: DFT8 over n2 for n1 = 2 lc + e, twiddle W^(n1 k2)
      dft8<false>(v);
      dft8<false>(v + 8);
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int k2 = 1; k2 < 8; ++k2) v[e * 8 + k2] = cmul(v[e * 8 + k2], s_tw[k2 * 17 + 2 * lc + e]);
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) lds[at(row, 16 * k2 + 2 * lc + e)] = v[e * 8 + k2];
      wave_lds_sync();
      // ---------------- x pass B: DFT16 over n1 for k2 = lc -> kx = lc + 8 k1
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) v[n1] = lds[at(row, 16 * lc + n1)];
      dft16<false>(v);
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) lds[at(row, lc + 8 * k1)] = v[k1];
      __syncthreads();
      // ---------------- y pass 1: DFT16 over j of column kx = col, rows lr + 8 j
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = lds[at(lr + 8 * j, col)];
      dft16<false>(v);
#pragma unroll
      for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], s_tw[lr * 17 + k1]);
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) lds[at(k1 * 8 + lr, col)] = v[k1];
      wave_lds_sync();
      // ---------------- y pass 2: DFT8 over n1 for k1 = 2 lr + g2 -> ky = k1 + 16 k2
#pragma unroll
      for (int g2 = 0; g2 < 2; ++g2)
#pragma unroll
        for (int n1 = 0; n1 < 8; ++n1) v[g2 * 8 + n1] = lds[at((2 * lr + g2) * 8 + n1, col)];
      dft8<false>(v);
      dft8<false>(v + 8);
    }

    // ---------------- per-pixel work: v[g2 * 8 + k2] <-> (ky = 2 lr + g2 + 16 k2, kx = col)
    {
      double tr = 0.0;
      const size_t base = (size_t)k * M;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ky = 2 * lr + (r >> 3) + 16 * (r & 7);
        pixel_op<OP, MET>(g, a, base + (size_t)ky * L + col, isq, bgv, v[r], s0, s1, tr);
      }
      if constexpr (OP == OP_LINEARIZE) {
        // per-position trace of the metric Hessian (App. B): each wavefront leaves its part in
        // the slot of this position's parity; thread 0 sums the slot after the y -> x transpose
        // barrier below, before it reaches the next position's first barrier, while the next
        // position's parts go to the other slot
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 64);
        if (lane == 0) red_tr[(k & 1) * NW + wv] = tr;
      }
    }

    if constexpr (INV) {
      // ---------------- inverse y pass 2: DFT8 over k2 -> n1, conjugate twiddle W^(n1 k1)
#pragma unroll
      for (int g2 = 0; g2 < 2; ++g2) {
        dft8<true>(v + g2 * 8);
#pragma unroll
        for (int n1 = 1; n1 < 8; ++n1) v[g2 * 8 + n1] = cmulc(v[g2 * 8 + n1], s_tw[n1 * 17 + 2 * lr + g2]);
      }
#pragma unroll
      for (int g2 = 0; g2 < 2; ++g2)
#pragma unroll
        for (int n1 = 0; n1 < 8; ++n1) lds[at((2 * lr + g2) * 8 + n1, col)] = v[g2 * 8 + n1];
      wave_lds_sync();
      // ---------------- inverse y pass 1: DFT16 over k1 -> rows lr + 8 j
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) v[k1] = lds[at(k1 * 8 + lr, col)];
      dft16<true>(v);
#pragma unroll
      for (int j = 0; j < 16; ++j) lds[at(lr + 8 * j, col)] = v[j];
      __syncthreads();
      if constexpr (OP == OP_LINEARIZE) {
        if (threadIdx.x == 0) {
          const double* slot = red_tr + (k & 1) * NW;
          double t = 0.0;
          for (int q = 0; q < NW; ++q) t += slot[q];
          g.trace[k] = t;
        }
      }
      // ---------------- inverse x pass B: DFT16 over k1 -> n1 for k2 = lc, conjugate twiddle
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) v[k1] = lds[at(row, lc + 8 * k1)];
      dft16<true>(v);
#pragma unroll
      for (int n1 = 1; n1 < 16; ++n1) v[n1] = cmulc(v[n1], s_tw[lc * 17 + n1]);
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) lds[at(row, 16 * lc + n1)] = v[n1];
      wave_lds_sync();
      // ---------------- inverse x pass A: DFT8 over k2 -> pixels (row, 2 lc + e + 16 n2); overlap-add
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) v[e * 8 + k2] = lds[at(row, 16 * k2 + 2 * lc + e)];
      dft8<true>(v);
      dft8<true>(v + 8);
      {
        c2* sq = reinterpret_cast<c2*>(strip + (size_t)(ry - box.x) * box.w + (rx - box.y) + lane_s);
        const c2* Pq = reinterpret_cast<const c2*>(a.P + lane_p);
        if (k == kbeg) {
#pragma unroll
          for (int n2 = 0; n2 < 8; ++n2) {
            const c2 pp = Pq[8 * n2];
            sq[8 * n2] = c2{cmulc(v[n2], pp.a), cmulc(v[8 + n2], pp.b)};
          }
        } else {
#pragma unroll
          for (int nn = 0; nn < 8; nn += NO) {
#pragma unroll
            for (int n2 = nn; n2 < nn + NO; ++n2) {
              const c2 pp = Pq[8 * n2], cur = sq[8 * n2];
              sq[8 * n2] = c2{cadd(cur.a, cmulc(v[n2], pp.a)), cadd(cur.b, cmulc(v[8 + n2], pp.b))};
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        if (joint) {
          const c2* Oq = reinterpret_cast<const c2*>(a.O + (size_t)ry * g.nx + rx + lane_o);
          c2* pq = reinterpret_cast<c2*>(g.probe_part + (size_t)seg * M + lane_p);
          const bool first = k == kbeg;
#pragma unroll
          for (int nn = 0; nn < 8; nn += NO) {
#pragma unroll
            for (int n2 = nn; n2 < nn + NO; ++n2) {
              const c2 oo = Oq[8 * n2];
              if (n2 < NREG) {
                accP[n2] = cadd(accP[n2], cmulc(v[n2], oo.a));
                accP[8 + n2] = cadd(accP[8 + n2], cmulc(v[8 + n2], oo.b));
              } else if (first) {
                pq[8 * n2] = c2{cmulc(v[n2], oo.a), cmulc(v[8 + n2], oo.b)};
              } else {
                const c2 cur = pq[8 * n2];
                pq[8 * n2] = c2{cadd(cur.a, cmulc(v[n2], oo.a)), cadd(cur.b, cmulc(v[8 + n2], oo.b))};
              }
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
    }
  }

  if constexpr (INV) {
    // (an empty segment leaves a zero slot in either form)
    if (joint) {
      c2* pp = reinterpret_cast<c2*>(g.probe_part + (size_t)seg * M + row * L + 2 * lc);
#pragma unroll
      for (int n2 = 0; n2 < 8; ++n2)
        if (n2 < NREG || kend == kbeg) pp[8 * n2] = c2{accP[n2], accP[8 + n2]};
    }
  }
  if constexpr (SUMS) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, 64);
      s1 += __shfl_xor(s1, off, 64);
    }
    __syncthreads();
    if (lane == 0) {
      red[wv * 2] = s0;
      red[wv * 2 + 1] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a0 = 0.0, a1 = 0.0;
      for (int q = 0; q < NW; ++q) {
        a0 += red[q * 2];
        a1 += red[q * 2 + 1];
      }
      g.partials[bid * 4 + 0] = a0;
      g.partials[bid * 4 + 1] = a1;
      g.partials[bid * 4 + 2] = 0.0;
      g.partials[bid * 4 + 3] = 0.0;
    }
  }
}

template <int OP, int MET>
__global__ __launch_bounds__(NTH) void kernel(Geometry g, TileArgs a) {
  body<OP, MET>(g, a, blockIdx.x, gridDim.x);
}

// batched: block b belongs to job job_of_block[b]; trailing blocks of a job's run exit
template <int OP>
__global__ __launch_bounds__(NTH) void batch_kernel(const TileJob* __restrict__ jobs,
                                                    const int* __restrict__ job_of_block) {
  const TileJob& J = jobs[job_of_block[blockIdx.x]];
  const int b = (int)blockIdx.x - J.block0;
  if (b >= J.g.grid) return;
  body<OP, -1>(J.g, J.a, b, J.g.grid);
}

template <int OP, int MET>
static hipError_t launch_met(const Geometry& g, const TileArgs& a, hipStream_t s) {
  static bool attr_set = false;  // per instantiation, host-side
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)kernel<OP, MET>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds_bytes());
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((kernel<OP, MET>), dim3(g.grid), dim3(NTH), lds_bytes(), s, g, a);
  return hipGetLastError();
}

template <int OP>
static hipError_t launch_one(const Geometry& g, const TileArgs& a, hipStream_t s) {
  switch (met_code(OP, g)) {
    case 0: return launch_met<OP, 0>(g, a, s);
    case 1:
      if constexpr (OP == OP_LOSS || OP == OP_LINEARIZE || OP == OP_JVP || OP == OP_VJP) return launch_met<OP, 1>(g, a, s);
      break;
    case 2:
      if constexpr (OP == OP_LINEARIZE) return launch_met<OP, 2>(g, a, s);
      break;
    case 3:
      if constexpr (OP == OP_LINEARIZE) return launch_met<OP, 3>(g, a, s);
      break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <int OP>
static hipError_t launch_one_batch(const TileJob* jobs, const int* job_of_block, int nblocks, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)batch_kernel<OP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds_bytes());
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((batch_kernel<OP>), dim3(nblocks), dim3(NTH), lds_bytes(), s, jobs, job_of_block);
  return hipGetLastError();
}

}  // namespace t128

bool tile128_handles(int op) { return op != OP_DIAG_EXACT; }

hipError_t launch_tile128(const Geometry& g, int op, const TileArgs& a, hipStream_t s) {
  using namespace t128;
  switch (op) {
    case OP_FORWARD: return launch_one<OP_FORWARD>(g, a, s);
    case OP_LOSS: return launch_one<OP_LOSS>(g, a, s);
    case OP_LINEARIZE: return launch_one<OP_LINEARIZE>(g, a, s);
    case OP_JVP: return launch_one<OP_JVP>(g, a, s);
    case OP_VJP: return launch_one<OP_VJP>(g, a, s);
    case OP_VJP_RAND: return launch_one<OP_VJP_RAND>(g, a, s);
    case OP_GGNV: return launch_one<OP_GGNV>(g, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tile128_batch(int op, const TileJob* jobs, const int* jb, int nb, hipStream_t s) {
  using namespace t128;
  switch (op) {
    case OP_LOSS: return launch_one_batch<OP_LOSS>(jobs, jb, nb, s);
    case OP_LINEARIZE: return launch_one_batch<OP_LINEARIZE>(jobs, jb, nb, s);
    case OP_GGNV: return launch_one_batch<OP_GGNV>(jobs, jb, nb, s);
    default: return hipErrorInvalidValue;
  }
}

size_t tile128_lds_bytes() { return t128::lds_bytes(); }
int tile128_threads() { return t128::NTH; }

}  // namespace ptlm
