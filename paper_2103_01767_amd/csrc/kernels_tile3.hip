// Per-position tile kernels for square probes of side L = 16 R with R = 3 or 6 (48 x 48 and
// 96 x 96), the non-power-of-two sides of the uneven batch.
//
// Same pipeline as the power-of-two kernels (gather -> 2D transform -> per-pixel op ->
// inverse transform -> atomic-free overlap-add into the segment's strip, probe part in
// registers, or in the segment's probe slot for the linearisation), with each length-L
// transform split as L = 16 x R (Cooley-Tukey,
// n = n1 + R n2, k = k1 + 16 k2):
//   pass 1  R threads per line, 16 values each: DFT16 over n2, twiddle W_L^(n1 k1);
//   pass 2  the 16 radix-R DFTs of a line (over n1, for each k1) dealt cyclically to the
//           line's R threads: thread c takes k1 = c, c + R, ... (at most ceil(16 / R) DFTs).
// A line's threads do not align with wavefronts (R does not divide 64), so every exchange
// uses a workgroup barrier.
#include "tile_pixel.hpp"

namespace ptlm {

template <int L>
struct Cfg3 {
  static constexpr int R = L / 16;
  static constexpr int M = L * L;
  static constexpr int NT = L * R;                          // threads per tile (16 values each)
  static constexpr int WG = 576;
  static constexpr int TPW = WG / NT;                       // 4 tiles of 48 x 48, 1 of 96 x 96
  // LDS row pitch (complex), chosen with the LDS bank model of gfx950 (32 banks of 4 bytes, a
  // 64-bit access served per half wavefront at the cost of its most-hit bank): L + 3 spreads
  // the x passes' row accesses best among the pitches up to L + 40 (largest bank load 1.6x the
  // least possible at 96, against 2.5x at L + 1); the y passes stay conflict-free
  static constexpr int LDX = L + 3;
  static constexpr int TILE = L * LDX;
  static constexpr int GMAX = (16 + R - 1) / R;             // radix-R DFTs per thread in pass 2
  static constexpr int VMAX = GMAX * R > 16 ? GMAX * R : 16;
  static constexpr int NWAVE = WG / 64;
  static constexpr int TW_OFF = L == 48 ? 480 : 528;        // W_L^(n k), n < R, k < 16
  static_assert(TPW * NT == WG, "tiles must fill the workgroup");
  static_assert(NT % 16 == 0, "the trace sums take 16 strided parts");
};

namespace {
__device__ __forceinline__ int xcd_map3(int b, int n) {
  if (n % 8 != 0) return b;
  return (b % 8) * (n / 8) + b / 8;
}
}  // namespace

template <int L, int OP>
__device__ __forceinline__ void tile3_body(const Geometry g, const TileArgs a, int bid, int nblk) {
  using C = Cfg3<L>;
  constexpr int R = C::R, NT = C::NT, LDX = C::LDX, GMAX = C::GMAX;
  constexpr bool FWD_FFT = OP != OP_VJP && OP != OP_VJP_RAND;
  constexpr bool INV_FFT = OP == OP_LINEARIZE || OP == OP_VJP || OP == OP_GGNV || OP == OP_VJP_RAND;
  constexpr bool SCATTER = INV_FFT || OP == OP_DIAG_EXACT;
  constexpr bool SUMS = OP == OP_LOSS || OP == OP_LINEARIZE;
  if (a.predicate && *a.predicate == 0) return;

  extern __shared__ float2 smem[];
  double* red = reinterpret_cast<double*>(smem + C::TPW * C::TILE);  // [NWAVE][2]
  double* tsum = red + 2 * C::NWAVE;                                 // [WG] per-thread values
  double* tpart = tsum + C::WG;                                      // [TPW][16] partial sums
  float2* tw = reinterpret_cast<float2*>(tpart + C::TPW * 16);       // [R][16]
  for (int i = threadIdx.x; i < R * 16; i += C::WG) tw[i] = g.tw[C::TW_OFF + i];
  __syncthreads();

  const int slot = threadIdx.x / NT;
  const int t = threadIdx.x % NT;
  float2* lds = smem + slot * C::TILE;
  const int blk = xcd_map3(bid, nblk);
  const int seg = blk * C::TPW + slot;
  const int kbeg = g.seg_start[seg], kend = g.seg_start[seg + 1];
  int maxlen = 0;
#pragma unroll
  for (int s = 0; s < C::TPW; ++s) {
    const int q = blk * C::TPW + s;
    maxlen = max(maxlen, g.seg_start[q + 1] - g.seg_start[q]);
  }
  const int xy = t / R, xc = t % R;  // x passes: line (row) and residue / pass-2 lane
  const int yc = t % L, ys = t / L;  // y passes: line (column) and residue / pass-2 lane
  const float isq = 1.0f / (float)L;
  const bool joint = g.joint != 0;
  const float bgv = a.bg_add ? (float)((double)g.background + *a.bg_add) : g.background;
  // probe partial of the overlap-add, in registers across the segment; the linearisation has
  // none to spare and read-modify-writes it in the segment's probe slot (same order of the sums)
  constexpr bool PREG = OP != OP_LINEARIZE;
  float2 accP[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) accP[j] = make_float2(0.f, 0.f);
  double s0 = 0.0, s1 = 0.0;

  float2* strip = nullptr;
  int4 box = make_int4(0, 0, 0, 0);
  if constexpr (SCATTER) {
    strip = g.strips + g.seg_off[seg];
    box = g.seg_box[seg];
    if (kend > kbeg) {
      const int2 p0 = g.pos[kbeg];
      const int area = box.z * box.w;
      for (int i = t; i < area; i += NT) {
        const int Y = box.x + i / box.w, X = box.y + i % box.w;
        if ((unsigned)(Y - p0.x) >= (unsigned)L || (unsigned)(X - p0.y) >= (unsigned)L)
          strip[i] = make_float2(0.f, 0.f);
      }
    }
  }

  for (int it = 0; it < maxlen; ++it) {
    const int k = kbeg + it;
    const bool act = k < kend;
    int ry = 0, rx = 0;
    if (act) {
      const int2 p = g.pos[k];
      ry = p.x;
      rx = p.y;
    }
    const size_t base = (size_t)k * C::M;
    float2 v[C::VMAX];
    double asum = 0.0;

    if constexpr (FWD_FFT) {
      // ---------------- gather, x pass 1 (DFT16 over n2, twiddle W_L^(n1 k1))
      if (act) {
        if constexpr (OP == OP_DIAG_EXACT) {
          const float2* arow = g.afield + base + xy * L + xc;
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const float2 as = arow[R * j];
            asum += (double)fmaf(as.x, as.x, as.y * as.y);
            v[j] = make_float2(fmaf(as.x, as.x, -as.y * as.y), -2.f * as.x * as.y);
          }
        } else {
          const float2* Orow = a.O + (size_t)(ry + xy) * g.nx + rx + xc;
          const float2* Prow = a.P + xy * L + xc;
          if constexpr (OP == OP_JVP || OP == OP_GGNV) {
            const float2* Vrow = a.vO + (size_t)(ry + xy) * g.nx + rx + xc;
            if (a.vP) {
              const float2* VProw = a.vP + xy * L + xc;
#pragma unroll
              for (int j = 0; j < 16; ++j)
                v[j] = cadd(cmul(Prow[R * j], Vrow[R * j]), cmul(VProw[R * j], Orow[R * j]));
            } else {
#pragma unroll
              for (int j = 0; j < 16; ++j) v[j] = cmul(Prow[R * j], Vrow[R * j]);
            }
          } else {
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = cmul(Prow[R * j], Orow[R * j]);
          }
        }
        dft16<false>(v);
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[xc * 16 + k1]);
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) lds[xy * LDX + k1 * R + xc] = v[k1];
      }
      __syncthreads();
      // ---------------- x pass 2 (DFT_R over n1 for k1 = xc + R gg) -> natural order
      if (act) {
#pragma unroll
        for (int gg = 0; gg < GMAX; ++gg) {
          const int k1 = xc + R * gg;
          if (k1 < 16) {
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) v[gg * R + n1] = lds[xy * LDX + k1 * R + n1];
          }
        }
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int gg = 0; gg < GMAX; ++gg) {
          const int k1 = xc + R * gg;
          if (k1 < 16) {
            dftR<R, false>(v + gg * R);
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) lds[xy * LDX + k1 + 16 * k2] = v[gg * R + k2];
          }
        }
      }
      __syncthreads();
      // ---------------- y pass 1
      if (act) {
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = lds[(ys + R * j) * LDX + yc];
        dft16<false>(v);
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[ys * 16 + k1]);
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) lds[(k1 * R + ys) * LDX + yc] = v[k1];
      }
      __syncthreads();
      // ---------------- y pass 2 -> v[gg R + k2] = X(ky = ys + R gg + 16 k2, kx = yc)
      if (act) {
#pragma unroll
        for (int gg = 0; gg < GMAX; ++gg) {
          const int k1 = ys + R * gg;
          if (k1 < 16) {
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) v[gg * R + n1] = lds[(k1 * R + n1) * LDX + yc];
            dftR<R, false>(v + gg * R);
          }
        }
      }
    }

    // ---------------- per-pixel work
    {
      double tr = 0.0;
      if (act) {
#pragma unroll
        for (int gg = 0; gg < GMAX; ++gg) {
          const int k1 = ys + R * gg;
          if (k1 < 16) {
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) {
              const size_t gi = base + (size_t)(k1 + 16 * k2) * L + yc;
              pixel_op<OP, -1>(g, a, gi, isq, bgv, v[gg * R + k2], s0, s1, tr);
            }
          }
        }
      }
      if constexpr (OP == OP_LINEARIZE) {
        // per-tile trace of ell'' (App. B): each thread leaves its part in LDS; the sum runs in
        // a fixed order after the next two barriers of the inverse transform (16 strided
        // partial sums per tile, then their sum), and the next position's parts are written
        // only after the position's last barrier
        tsum[threadIdx.x] = tr;
      } else if constexpr (OP == OP_DIAG_EXACT) {
        // per-tile sum of |a|^2 through LDS, fixed order, returned to every thread of the tile
        tsum[threadIdx.x] = asum;
        __syncthreads();
        if (t == 0) {
          double s = 0.0;
          for (int i = 0; i < NT; ++i) s += tsum[slot * NT + i];
          tsum[slot * NT] = s;
        }
        __syncthreads();
        asum = tsum[slot * NT];
        __syncthreads();
      }
    }

    if constexpr (OP == OP_DIAG_EXACT) {
      // B_k = DFT(conj(a)^2) to LDS in detector order; pixel m' reads B_k at 2m' mod L
      if (act) {
#pragma unroll
        for (int gg = 0; gg < GMAX; ++gg) {
          const int k1 = ys + R * gg;
          if (k1 < 16) {
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) lds[(k1 + 16 * k2) * LDX + yc] = v[gg * R + k2];
          }
        }
      }
      __syncthreads();
      if (act) {
        const float A = (float)asum;
        const int Y = ry + xy;
        float2* srow = strip + (size_t)(Y - box.x) * box.w + (rx + xc - box.y);
        const float2* Prow = a.P + xy * L + xc;
        const float2* Orow = a.O + (size_t)Y * g.nx + rx + xc;
        const int by = (2 * xy) % L;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int x = xc + R * j;
          const float2 B = lds[by * LDX + (2 * x) % L];
          const float2 q = Prow[R * j];
          float bse = 0.5f * A * fmaf(q.x, q.x, q.y * q.y);
          float crs = 0.5f * (fmaf(q.x, q.x, -q.y * q.y) * B.x - 2.f * q.x * q.y * B.y);
          const float2 cur = it == 0 ? make_float2(0.f, 0.f) : srow[R * j];
          srow[R * j] = make_float2(cur.x + bse + crs, cur.y + bse - crs);
          if (joint) {
            const float2 o = Orow[R * j];
            bse = 0.5f * A * fmaf(o.x, o.x, o.y * o.y);
            crs = 0.5f * (fmaf(o.x, o.x, -o.y * o.y) * B.x - 2.f * o.x * o.y * B.y);
            accP[j] = make_float2(accP[j].x + bse + crs, accP[j].y + bse - crs);
          }
        }
      }
      __syncthreads();
    }

    if constexpr (INV_FFT) {
      // ---------------- inverse y pass 2 (DFT_R over k2 -> n1, conjugate twiddle)
      if (act) {
#pragma unroll
        for (int gg = 0; gg < GMAX; ++gg) {
          const int k1 = ys + R * gg;
          if (k1 < 16) {
            dftR<R, true>(v + gg * R);
#pragma unroll
            for (int n1 = 1; n1 < R; ++n1) v[gg * R + n1] = cmulc(v[gg * R + n1], tw[n1 * 16 + k1]);
          }
        }
      }
      __syncthreads();
      if constexpr (OP == OP_LINEARIZE) {
        // trace, first level: partial sum j of tile ts over its parts j, j + 16, j + 32, ...
        if (threadIdx.x < C::TPW * 16) {
          const int ts = threadIdx.x / 16, j = threadIdx.x % 16;
          double s = 0.0;
          for (int i = 0; i < NT / 16; ++i) s += tsum[ts * NT + j + 16 * i];
          tpart[threadIdx.x] = s;
        }
      }
      if (act) {
#pragma unroll
        for (int gg = 0; gg < GMAX; ++gg) {
          const int k1 = ys + R * gg;
          if (k1 < 16) {
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) lds[(k1 * R + n1) * LDX + yc] = v[gg * R + n1];
          }
        }
      }
      __syncthreads();
      if constexpr (OP == OP_LINEARIZE) {
        // trace, second level: the tile's 16 partial sums in order
        if (act && t == 0) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < 16; ++j) s += tpart[slot * 16 + j];
          g.trace[k] = s;
        }
      }
      // ---------------- inverse y pass 1 (DFT16 over k1 -> n2): rows ys + R n2
      if (act) {
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) v[k1] = lds[(k1 * R + ys) * LDX + yc];
        dft16<true>(v);
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int j = 0; j < 16; ++j) lds[(ys + R * j) * LDX + yc] = v[j];
      }
      __syncthreads();
      // ---------------- inverse x pass 2
      if (act) {
#pragma unroll
        for (int gg = 0; gg < GMAX; ++gg) {
          const int k1 = xc + R * gg;
          if (k1 < 16) {
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) v[gg * R + k2] = lds[xy * LDX + k1 + 16 * k2];
          }
        }
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int gg = 0; gg < GMAX; ++gg) {
          const int k1 = xc + R * gg;
          if (k1 < 16) {
            dftR<R, true>(v + gg * R);
#pragma unroll
            for (int n1 = 1; n1 < R; ++n1) v[gg * R + n1] = cmulc(v[gg * R + n1], tw[n1 * 16 + k1]);
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) lds[xy * LDX + k1 * R + n1] = v[gg * R + n1];
          }
        }
      }
      __syncthreads();
      // ---------------- inverse x pass 1 -> pixel (xy, xc + R j), overlap-add
      if (act) {
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) v[k1] = lds[xy * LDX + k1 * R + xc];
        dft16<true>(v);
        const int Y = ry + xy;
        float2* srow = strip + (size_t)(Y - box.x) * box.w + (rx + xc - box.y);
        const float2* Prow = a.P + xy * L + xc;
        if (it == 0) {
#pragma unroll
          for (int j = 0; j < 16; ++j) srow[R * j] = cmulc(v[j], Prow[R * j]);
        } else {
#pragma unroll
          for (int j = 0; j < 16; ++j) srow[R * j] = cadd(srow[R * j], cmulc(v[j], Prow[R * j]));
        }
        if (joint) {
          const float2* Orow = a.O + (size_t)Y * g.nx + rx + xc;
          if constexpr (PREG) {
#pragma unroll
            for (int j = 0; j < 16; ++j) accP[j] = cadd(accP[j], cmulc(v[j], Orow[R * j]));
          } else {
            float2* pp = g.probe_part + (size_t)seg * C::M + xy * L + xc;
            if (it == 0) {
#pragma unroll
              for (int j = 0; j < 16; ++j) pp[R * j] = cmulc(v[j], Orow[R * j]);
            } else {
#pragma unroll
              for (int j = 0; j < 16; ++j) pp[R * j] = cadd(pp[R * j], cmulc(v[j], Orow[R * j]));
            }
          }
        }
      }
      // the next position's x pass 1 writes rows other threads may still read here
      __syncthreads();
    }
  }

  if constexpr (SCATTER) {
    // (an empty segment leaves a zero slot in either form)
    if (joint && (PREG || kend == kbeg)) {
      float2* pp = g.probe_part + (size_t)seg * C::M + xy * L + xc;
#pragma unroll
      for (int j = 0; j < 16; ++j) pp[R * j] = accP[j];
    }
  }
  if constexpr (SUMS) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, 64);
      s1 += __shfl_xor(s1, off, 64);
    }
    __syncthreads();
    const int wave = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
      red[wave * 2] = s0;
      red[wave * 2 + 1] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a0 = 0.0, a1 = 0.0;
      for (int w = 0; w < C::NWAVE; ++w) {
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

template <int L, int OP>
__global__ __launch_bounds__(576) void tile3_kernel(Geometry g, TileArgs a) {
  tile3_body<L, OP>(g, a, blockIdx.x, gridDim.x);
}

template <int L, int OP>
__global__ __launch_bounds__(576) void tile3_batch_kernel(const TileJob* __restrict__ jobs,
                                                          const int* __restrict__ job_of_block) {
  const TileJob& J = jobs[job_of_block[blockIdx.x]];
  const int b = (int)blockIdx.x - J.block0;
  if (b >= J.g.grid) return;
  tile3_body<L, OP>(J.g, J.a, b, J.g.grid);
}

template <int L>
size_t tile3_lds() {
  using C = Cfg3<L>;
  return (size_t)C::TPW * C::TILE * sizeof(float2) + (size_t)(2 * C::NWAVE + C::WG + C::TPW * 16) * sizeof(double) +
         (size_t)C::R * 16 * sizeof(float2);
}

size_t tile3_lds_bytes(int L) { return L == 48 ? tile3_lds<48>() : (L == 96 ? tile3_lds<96>() : 0); }
int tile3_per_wg(int L) { return L == 48 ? Cfg3<48>::TPW : (L == 96 ? Cfg3<96>::TPW : 0); }

template <int L, int OP>
static hipError_t launch3(const Geometry& g, const TileArgs& a, hipStream_t s) {
  const size_t lds = tile3_lds<L>();
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)tile3_kernel<L, OP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((tile3_kernel<L, OP>), dim3(g.grid), dim3(576), lds, s, g, a);
  return hipGetLastError();
}

template <int L>
static hipError_t launch3_op(const Geometry& g, int op, const TileArgs& a, hipStream_t s) {
  switch (op) {
    case OP_FORWARD: return launch3<L, OP_FORWARD>(g, a, s);
    case OP_LOSS: return launch3<L, OP_LOSS>(g, a, s);
    case OP_LINEARIZE: return launch3<L, OP_LINEARIZE>(g, a, s);
    case OP_JVP: return launch3<L, OP_JVP>(g, a, s);
    case OP_VJP: return launch3<L, OP_VJP>(g, a, s);
    case OP_VJP_RAND: return launch3<L, OP_VJP_RAND>(g, a, s);
    case OP_GGNV: return launch3<L, OP_GGNV>(g, a, s);
    case OP_DIAG_EXACT: return launch3<L, OP_DIAG_EXACT>(g, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int L, int OP>
static hipError_t launch3_batch(const TileJob* jobs, const int* jb, int nb, hipStream_t s) {
  const size_t lds = tile3_lds<L>();
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)tile3_batch_kernel<L, OP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((tile3_batch_kernel<L, OP>), dim3(nb), dim3(576), lds, s, jobs, jb);
  return hipGetLastError();
}

template <int L>
static hipError_t launch3_op_batch(int op, const TileJob* jobs, const int* jb, int nb, hipStream_t s) {
  switch (op) {
    case OP_LOSS: return launch3_batch<L, OP_LOSS>(jobs, jb, nb, s);
    case OP_LINEARIZE: return launch3_batch<L, OP_LINEARIZE>(jobs, jb, nb, s);
    case OP_GGNV: return launch3_batch<L, OP_GGNV>(jobs, jb, nb, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tile3_batch(int L, int op, const TileJob* jobs, const int* jb, int nb, hipStream_t s) {
  if (L == 48) return launch3_op_batch<48>(op, jobs, jb, nb, s);
  if (L == 96) return launch3_op_batch<96>(op, jobs, jb, nb, s);
  return hipErrorInvalidValue;
}

hipError_t launch_tile3(const Geometry& g, int op, const TileArgs& a, hipStream_t s) {
  if (g.my != g.mx) return hipErrorInvalidValue;
  if (g.my == 48) return launch3_op<48>(g, op, a, s);
  if (g.my == 96) return launch3_op<96>(g, op, a, s);
  return hipErrorInvalidValue;
}

}  // namespace ptlm
