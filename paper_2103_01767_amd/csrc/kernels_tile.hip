// Per-position tile kernels: gather -> 2D FFT -> per-pixel op -> inverse 2D FFT -> overlap-add.
//
// One workgroup owns a contiguous segment of scan positions (TPW concurrent
// tile slots for small probes, one slot for 64x64 and larger) and walks it
// position by position.  A position's My x Mx tile is transformed with a
// four-pass Stockham FFT per 2D transform: radix-16 then radix-(L/16) along x,
// the same along y.  Each thread holds 16 complex values in registers during
// a pass; passes exchange data through one padded LDS tile.  The last forward
// pass and the first inverse pass share the register layout, so the per-pixel
// work between the transforms (metric, weighting by the stored phasor field)
// happens in registers with coalesced global reads.
//
// Overlap-add (the adjoint S_k^T of the shift operator, Sec. 2) never uses
// atomics: each segment accumulates into its own private strip (the bounding
// box of its windows) with plain read-modify-write, and the probe part of the
// sum is kept in registers per thread across the segment.  Separate gather
// kernels sum strips and probe partials in a fixed order.
#include "dft.hpp"
#include "internal.hpp"
#include "tile_pixel.hpp"

namespace ptlm {

// W: workgroup width, 1 for tiles filling 256 threads, 2 for the wide grouping of the
// GGN-vector product (PTLM_TRANSFORM_FFT_WIDE: twice the tiles, the same segments)
template <int MY_, int MX_, int W_ = 1>
struct Cfg {
  static constexpr int MY = MY_, MX = MX_, M = MY * MX;
  static constexpr int NV = M / 16;                       // virtual threads per tile (16 values each)
  static constexpr int V = 1;                             // virtual threads per real thread
  static constexpr int NT = NV / V;                       // real threads per tile
  static constexpr int TPW = (NT >= 256 ? 1 : 256 / NT) * W_;  // tiles per workgroup
  static constexpr int WG = NT * TPW;
  static constexpr int RX = MX / 16, RY = MY / 16;        // second-pass radices
  static constexpr int GX = 16 / RX, GY = 16 / RY;        // second-pass groups per virtual thread
  // LDS layout (bank-conflict-free for every exchange of the four passes): after x pass 1
  // element (n1, k1) of a row sits at column k1 * XA + n1; rows are LDX complex apart.
  static constexpr int XA = MX == 16 ? 1 : (MX == 32 ? 2 : (MX == 64 ? 5 : 9));
  static constexpr int LDX = MX == 16 ? 17 : (MX == 32 ? 35 : (MX == 64 ? 83 : 144));
  static constexpr int TILE = MY * LDX;                   // LDS complex per tile
  static constexpr int NWAVE = WG / 64 > 0 ? WG / 64 : 1;
  // probe partial kept in registers across the segment, or read-modify-written in the
  // segment's global probe slot each position (largest tile: no register room)
  static constexpr bool PROBE_REGS = NT < 1024;
};

__device__ __forceinline__ const float2* tw_table(const float2* tw, int L) {
  return tw + (L == 32 ? 0 : (L == 64 ? 32 : 96));
}

// Sum of a double over the NT real threads of this thread's tile, returned to every
// thread of the tile.  Uses red[] (one slot per wave, column `col`) when the tile spans
// several waves; contains one workgroup barrier in that case.
template <class C>
__device__ __forceinline__ double tile_sum(double x, double* red, int col, int slot) {
  constexpr int L = C::NT < 64 ? C::NT : 64;
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  if constexpr (C::NT > 64) {
    if ((threadIdx.x & 63) == 0) red[(threadIdx.x / 64) * 2 + col] = x;
    __syncthreads();
    x = 0.0;
    for (int w = 0; w < C::NT / 64; ++w) x += red[(slot * (C::NT / 64) + w) * 2 + col];
  }
  return x;
}

// MET: the metric / GGN-weight code of the per-pixel op (tile_pixel.hpp); -1 reads it from g
// per pixel (batched launches mix problems)
template <int MY, int MX, int OP, int MET, int W = 1>
__device__ __forceinline__ void tile_body(const Geometry g, const TileArgs a, int bid, int nblk) {
  using C = Cfg<MY, MX, W>;
  constexpr int RX = C::RX, RY = C::RY, GX = C::GX, GY = C::GY, LDX = C::LDX, XA = C::XA, V = C::V, NT = C::NT;
  constexpr bool FWD_FFT = OP != OP_VJP && OP != OP_VJP_RAND;
  constexpr bool INV_FFT = OP == OP_LINEARIZE || OP == OP_VJP || OP == OP_GGNV || OP == OP_VJP_RAND;
  constexpr bool SCATTER = INV_FFT || OP == OP_DIAG_EXACT;
  constexpr bool SUMS = OP == OP_LOSS || OP == OP_LINEARIZE;
  if (a.predicate && *a.predicate == 0) return;

  extern __shared__ float2 smem[];
  double* red = reinterpret_cast<double*>(smem + C::TPW * C::TILE);  // [NWAVE][2]
  float2* s_tw = smem + C::TPW * C::TILE + 2 * C::NWAVE;             // twiddles W_L^(n k), L = 32, 64, 128
  for (int i = threadIdx.x; i < 224; i += C::WG) s_tw[i] = g.tw[i];
  __syncthreads();

  const int slot = threadIdx.x / NT;
  const int t = threadIdx.x % NT;
  float2* lds = smem + slot * C::TILE;
  const int blk = xcd_block(bid, nblk);
  const int seg = blk * C::TPW + slot;
  // a wide launch over an odd number of standard workgroups has slots past the last segment
  const bool real = seg < g.nseg;
  const int kbeg = real ? g.seg_start[seg] : 0, kend = real ? g.seg_start[seg + 1] : 0;
  int maxlen = 0;
#pragma unroll
  for (int s = 0; s < C::TPW; ++s) {
    const int q = blk * C::TPW + s;
    if (q < g.nseg) maxlen = max(maxlen, g.seg_start[q + 1] - g.seg_start[q]);
  }
  const float2* twx = tw_table(s_tw, MX);
  const float2* twy = tw_table(s_tw, MY);
  const float isq = rsqrtf((float)C::M);
  const bool joint = g.joint != 0;
  const float bgv = a.bg_add ? (float)((double)g.background + *a.bg_add) : g.background;

  constexpr int VA = C::PROBE_REGS ? V : 1;
  constexpr int JA = C::PROBE_REGS ? 16 : 1;
  float2 accP[VA][JA];
#pragma unroll
  for (int u = 0; u < VA; ++u)
#pragma unroll
    for (int j = 0; j < JA; ++j) accP[u][j] = make_float2(0.f, 0.f);
  float2* pslot = g.probe_part + (size_t)(real ? seg : 0) * C::M;  // this segment's probe partial
  double s0 = 0.0, s1 = 0.0;

  // The segment's first position stores its contribution into the strip (and the global
  // probe slot); later positions read-modify-write.  Strip pixels outside the first window
  // are cleared here, so no separate clearing pass is needed between calls.
  float2* strip = nullptr;
  int4 box = make_int4(0, 0, 0, 0);
  if constexpr (SCATTER) {
    if (real) {
      strip = g.strips + g.seg_off[seg];
      box = g.seg_box[seg];
    }
    if (kend > kbeg) {
      const int2 p0 = g.pos[kbeg];
      const int area = box.z * box.w;
      for (int i = t; i < area; i += NT) {
        const int Y = box.x + i / box.w, X = box.y + i % box.w;
        if ((unsigned)(Y - p0.x) >= (unsigned)MY || (unsigned)(X - p0.y) >= (unsigned)MX)
          strip[i] = make_float2(0.f, 0.f);
      }
    } else if (!C::PROBE_REGS && joint && real) {
      for (int i = t; i < C::M; i += NT) pslot[i] = make_float2(0.f, 0.f);
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
    float2 v[V][16];
    double asum = 0.0;  // OP_DIAG_EXACT: sum |a|^2 over this thread's pixels

    if constexpr (FWD_FFT) {
      // ---------------- gather the exit wave (or its perturbation), x-pass-1 layout
      if (act) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int tv = t + u * NT, xy = tv / RX, xn1 = tv % RX;
          if constexpr (OP == OP_DIAG_EXACT) {
            // conj(a)^2 of the stored phasor field, read as a My x Mx image
            const float2* arow = g.afield + (size_t)k * C::M + xy * MX + xn1;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
              const float2 as = arow[RX * j];
              asum += (double)fmaf(as.x, as.x, as.y * as.y);
              v[u][j] = make_float2(fmaf(as.x, as.x, -as.y * as.y), -2.f * as.x * as.y);
            }
          } else {
            const float2* Orow = a.O + (size_t)(ry + xy) * g.nx + rx + xn1;
            const float2* Prow = a.P + xy * MX + xn1;
            if constexpr (OP == OP_JVP || OP == OP_GGNV) {
              const float2* Vrow = a.vO + (size_t)(ry + xy) * g.nx + rx + xn1;
              if (a.vP) {
                const float2* VProw = a.vP + xy * MX + xn1;
#pragma unroll
                for (int jj = 0; jj < 16; jj += 4) {
#pragma unroll
                  for (int j = jj; j < jj + 4; ++j)
                    v[u][j] = cadd(cmul(Prow[RX * j], Vrow[RX * j]), cmul(VProw[RX * j], Orow[RX * j]));
                  __builtin_amdgcn_sched_barrier(0);
                }
              } else {
#pragma unroll
                for (int j = 0; j < 16; ++j) v[u][j] = cmul(Prow[RX * j], Vrow[RX * j]);
              }
            } else {
#pragma unroll
              for (int j = 0; j < 16; ++j) v[u][j] = cmul(Prow[RX * j], Orow[RX * j]);
            }
          }
          // x pass 1: DFT16 over j, twiddle W_MX^(n1 k1)
          dft16<false>(v[u]);
          if constexpr (RX > 1) {
#pragma unroll
            for (int k1 = 1; k1 < 16; ++k1) v[u][k1] = cmul(v[u][k1], twx[xn1 * 16 + k1]);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      // the x-pass exchanges touch only this wavefront's rows; after an inverse transform the
      // previous position's last reads of these rows (inverse x pass 1) came from this wave
      if constexpr (INV_FFT) wave_lds_sync();
      else __syncthreads();
      if (act) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int tv = t + u * NT, xy = tv / RX, xn1 = tv % RX;
#pragma unroll
          for (int k1 = 0; k1 < 16; ++k1) lds[xy * LDX + k1 * XA + xn1] = v[u][k1];
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if constexpr (RX > 1) wave_lds_sync();
      else __syncthreads();
      // ---------------- x pass 2
      if constexpr (RX > 1) {
        if (act) {
#pragma unroll
          for (int u = 0; u < V; ++u) {
            const int tv = t + u * NT;
#pragma unroll
            for (int gg = 0; gg < GX; ++gg) {
              const int q = tv * GX + gg, yy = q >> 4, k1 = q & 15;
#pragma unroll
              for (int n1 = 0; n1 < RX; ++n1) v[u][gg * RX + n1] = lds[yy * LDX + k1 * XA + n1];
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        wave_lds_sync();
        if (act) {
#pragma unroll
          for (int u = 0; u < V; ++u) {
            const int tv = t + u * NT;
#pragma unroll
            for (int gg = 0; gg < GX; ++gg) {
              const int q = tv * GX + gg, yy = q >> 4, k1 = q & 15;
              dftR<RX, false>(v[u] + gg * RX);
#pragma unroll
              for (int k2 = 0; k2 < RX; ++k2) lds[yy * LDX + k1 + 16 * k2] = v[u][gg * RX + k2];
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        __syncthreads();
      }
      // ---------------- y pass 1
      if (act) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int tv = t + u * NT, yc = tv % MX, ys = tv / MX;
#pragma unroll
          for (int j = 0; j < 16; ++j) v[u][j] = lds[(ys + RY * j) * LDX + yc];
          dft16<false>(v[u]);
          if constexpr (RY > 1) {
#pragma unroll
            for (int k1 = 1; k1 < 16; ++k1) v[u][k1] = cmul(v[u][k1], twy[ys * 16 + k1]);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if constexpr (RY > 1) {
        __syncthreads();
        if (act) {
#pragma unroll
          for (int u = 0; u < V; ++u) {
            const int tv = t + u * NT, yc = tv % MX, ys = tv / MX;
#pragma unroll
            for (int k1 = 0; k1 < 16; ++k1) lds[(k1 * RY + ys) * LDX + yc] = v[u][k1];
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        __syncthreads();
        // ---------------- y pass 2
        if (act) {
#pragma unroll
          for (int u = 0; u < V; ++u) {
            const int tv = t + u * NT, yc = tv % MX, ys = tv / MX;
#pragma unroll
            for (int gg = 0; gg < GY; ++gg) {
              const int k1 = ys * GY + gg;
#pragma unroll
              for (int n1 = 0; n1 < RY; ++n1) v[u][gg * RY + n1] = lds[(k1 * RY + n1) * LDX + yc];
              dftR<RY, false>(v[u] + gg * RY);
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
    }

    // ---------------- per-pixel work in the frequency layout: v[u][r] <-> (ky, kx)
    {
      double tr = 0.0;
      if (act) {
        const size_t base = (size_t)k * C::M;
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int tv = t + u * NT, yc = tv % MX, ys = tv / MX;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int ky = ys * GY + r / RY + 16 * (r % RY);
            const size_t gi = base + (size_t)ky * MX + yc;
            pixel_op<OP, MET>(g, a, gi, isq, bgv, v[u][r], s0, s1, tr);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if constexpr (OP == OP_LINEARIZE) {
        // per-position trace of the metric Hessian (App. B), reduced over the tile; a tile of
        // several wavefronts leaves their sums in LDS, added after the inverse transform's
        // next workgroup barrier
        if constexpr (C::NT > 64) {
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 64);
          if ((threadIdx.x & 63) == 0) red[(threadIdx.x / 64) * 2] = tr;
        } else {
          tr = tile_sum<C>(tr, red, 0, slot);
          if (act && t == 0) g.trace[k] = tr;
        }
      }
    }

    if constexpr (OP == OP_DIAG_EXACT) {
      // B_k = DFT(conj(a)^2) to LDS in detector order, then every pixel m' of the
      // window reads B_k at 2m' (mod the probe shape) and forms the exact diagonal
      // terms |Q|^2 A_k / 2 +- Re(Q^2 B_k[2m']) / 2, Q = P (object) or S_k O (probe).
      asum = tile_sum<C>(asum, red, 1, slot);
      __syncthreads();
      if (act) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int tv = t + u * NT, yc = tv % MX, ys = tv / MX;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int ky = ys * GY + r / RY + 16 * (r % RY);
            lds[ky * LDX + yc] = v[u][r];
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      __syncthreads();
      if (act) {
        const float A = (float)asum;
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int tv = t + u * NT, xy = tv / RX, xn1 = tv % RX;
          const int Y = ry + xy;
          float2* srow = strip + (size_t)(Y - box.x) * box.w + (rx + xn1 - box.y);
          const float2* Prow = a.P + xy * MX + xn1;
          const float2* Orow = a.O + (size_t)Y * g.nx + rx + xn1;
          const int by = (2 * xy) & (MY - 1);
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const int x = xn1 + RX * j;
            const float2 B = lds[by * LDX + ((2 * x) & (MX - 1))];
            const float2 q = Prow[RX * j];
            float base = 0.5f * A * fmaf(q.x, q.x, q.y * q.y);
            float cross = 0.5f * (fmaf(q.x, q.x, -q.y * q.y) * B.x - 2.f * q.x * q.y * B.y);
            const float2 cur = it == 0 ? make_float2(0.f, 0.f) : srow[RX * j];
            srow[RX * j] = make_float2(cur.x + base + cross, cur.y + base - cross);
            if (joint) {
              const float2 o = Orow[RX * j];
              base = 0.5f * A * fmaf(o.x, o.x, o.y * o.y);
              cross = 0.5f * (fmaf(o.x, o.x, -o.y * o.y) * B.x - 2.f * o.x * o.y * B.y);
              if constexpr (C::PROBE_REGS) {
                accP[u][j] = make_float2(accP[u][j].x + base + cross, accP[u][j].y + base - cross);
              } else {
                float2* pp = pslot + xy * MX + xn1 + RX * j;
                const float2 c0 = it == 0 ? make_float2(0.f, 0.f) : *pp;
                *pp = make_float2(c0.x + base + cross, c0.y + base - cross);
              }
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }

    if constexpr (INV_FFT) {
      // ---------------- inverse y pass 2 (DFT over k2 -> n1, conjugate twiddle)
      if constexpr (RY > 1) {
        if (act) {
#pragma unroll
          for (int u = 0; u < V; ++u) {
            const int tv = t + u * NT, ys = tv / MX;
#pragma unroll
            for (int gg = 0; gg < GY; ++gg) {
              const int k1 = ys * GY + gg;
              dftR<RY, true>(v[u] + gg * RY);
#pragma unroll
              for (int n1 = 1; n1 < RY; ++n1) v[u][gg * RY + n1] = cmulc(v[u][gg * RY + n1], twy[n1 * 16 + k1]);
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        __syncthreads();
        if (act) {
#pragma unroll
          for (int u = 0; u < V; ++u) {
            const int tv = t + u * NT, yc = tv % MX, ys = tv / MX;
#pragma unroll
            for (int gg = 0; gg < GY; ++gg) {
              const int k1 = ys * GY + gg;
#pragma unroll
              for (int n1 = 0; n1 < RY; ++n1) lds[(k1 * RY + n1) * LDX + yc] = v[u][gg * RY + n1];
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        __syncthreads();
        if (act) {
#pragma unroll
          for (int u = 0; u < V; ++u) {
            const int tv = t + u * NT, yc = tv % MX, ys = tv / MX;
#pragma unroll
            for (int k1 = 0; k1 < 16; ++k1) v[u][k1] = lds[(k1 * RY + ys) * LDX + yc];
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      // ---------------- inverse y pass 1 (DFT16 over k1 -> n2), natural rows
      if (act) {
#pragma unroll
        for (int u = 0; u < V; ++u) dft16<true>(v[u]);
      }
      __syncthreads();
      if constexpr (OP == OP_LINEARIZE && C::NT > 64) {
        // the trace's wavefront sums in order (the next position writes them after the
        // barrier below)
        if (act && t == 0) {
          double x = 0.0;
          for (int w = 0; w < C::NT / 64; ++w) x += red[(slot * (C::NT / 64) + w) * 2];
          g.trace[k] = x;
        }
      }
      if (act) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int tv = t + u * NT, yc = tv % MX, ys = tv / MX;
#pragma unroll
          for (int j = 0; j < 16; ++j) lds[(ys + RY * j) * LDX + yc] = v[u][j];
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      __syncthreads();
      // ---------------- inverse x pass 2
      if constexpr (RX > 1) {
        if (act) {
#pragma unroll
          for (int u = 0; u < V; ++u) {
            const int tv = t + u * NT;
#pragma unroll
            for (int gg = 0; gg < GX; ++gg) {
              const int q = tv * GX + gg, yy = q >> 4, k1 = q & 15;
#pragma unroll
              for (int k2 = 0; k2 < RX; ++k2) v[u][gg * RX + k2] = lds[yy * LDX + k1 + 16 * k2];
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        wave_lds_sync();
        if (act) {
#pragma unroll
          for (int u = 0; u < V; ++u) {
            const int tv = t + u * NT;
#pragma unroll
            for (int gg = 0; gg < GX; ++gg) {
              const int q = tv * GX + gg, yy = q >> 4, k1 = q & 15;
              dftR<RX, true>(v[u] + gg * RX);
#pragma unroll
              for (int n1 = 1; n1 < RX; ++n1)
                v[u][gg * RX + n1] = cmulc(v[u][gg * RX + n1], twx[n1 * 16 + k1]);
#pragma unroll
              for (int n1 = 0; n1 < RX; ++n1) lds[yy * LDX + k1 * XA + n1] = v[u][gg * RX + n1];
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        wave_lds_sync();
      }
      // ---------------- inverse x pass 1 -> pixel (xy, xn1 + RX j), then overlap-add
      if (act) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int tv = t + u * NT, xy = tv / RX, xn1 = tv % RX;
#pragma unroll
          for (int k1 = 0; k1 < 16; ++k1) v[u][k1] = lds[xy * LDX + k1 * XA + xn1];
          dft16<true>(v[u]);
          // object strip (plain RMW, segment-private) and probe registers
          const int Y = ry + xy;
          float2* srow = strip + (size_t)(Y - box.x) * box.w + (rx + xn1 - box.y);
          const float2* Prow = a.P + xy * MX + xn1;
          if (it == 0) {
#pragma unroll
            for (int j = 0; j < 16; ++j) srow[RX * j] = cmulc(v[u][j], Prow[RX * j]);
          } else {
#pragma unroll
            for (int jj = 0; jj < 16; jj += 4) {
#pragma unroll
              for (int j = jj; j < jj + 4; ++j) {
                const float2 cur = srow[RX * j];
                srow[RX * j] = cadd(cur, cmulc(v[u][j], Prow[RX * j]));
              }
              __builtin_amdgcn_sched_barrier(0);
            }
          }
          if (joint) {
            const float2* Orow = a.O + (size_t)Y * g.nx + rx + xn1;
            if constexpr (C::PROBE_REGS) {
#pragma unroll
              for (int jj = 0; jj < 16; jj += 4) {
#pragma unroll
                for (int j = jj; j < jj + 4; ++j) accP[u][j] = cadd(accP[u][j], cmulc(v[u][j], Orow[RX * j]));
                __builtin_amdgcn_sched_barrier(0);
              }
            } else {
              float2* prow = pslot + xy * MX + xn1;
              if (it == 0) {
#pragma unroll
                for (int j = 0; j < 16; ++j) prow[RX * j] = cmulc(v[u][j], Orow[RX * j]);
              } else {
#pragma unroll
                for (int jj = 0; jj < 16; jj += 4) {
#pragma unroll
                  for (int j = jj; j < jj + 4; ++j) prow[RX * j] = cadd(prow[RX * j], cmulc(v[u][j], Orow[RX * j]));
                  __builtin_amdgcn_sched_barrier(0);
                }
              }
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
  }

  if constexpr (SCATTER && C::PROBE_REGS) {
    if (joint && real) {
#pragma unroll
      for (int u = 0; u < V; ++u) {
        const int tv = t + u * NT, xy = tv / RX, xn1 = tv % RX;
        float2* pp = g.probe_part + (size_t)seg * C::M + xy * MX + xn1;
#pragma unroll
        for (int j = 0; j < 16; ++j) pp[RX * j] = accP[u][j];
        __builtin_amdgcn_sched_barrier(0);
      }
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

template <int MY, int MX, int OP, int MET, int W = 1>
__global__ __launch_bounds__((Cfg<MY, MX, W>::WG)) void tile_kernel(Geometry g, TileArgs a) {
  tile_body<MY, MX, OP, MET, W>(g, a, blockIdx.x, gridDim.x);
}

// batched: block b belongs to job job_of_block[b]; trailing blocks of a job's run exit
template <int MY, int MX, int OP>
__global__ __launch_bounds__((Cfg<MY, MX>::WG)) void tile_batch_kernel(const TileJob* __restrict__ jobs,
                                                                       const int* __restrict__ job_of_block) {
  const TileJob& J = jobs[job_of_block[blockIdx.x]];
  const int b = (int)blockIdx.x - J.block0;
  if (b >= J.g.grid) return;
  tile_body<MY, MX, OP, -1>(J.g, J.a, b, J.g.grid);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <int MY, int MX, int W = 1>
static size_t lds_bytes() {
  using C = Cfg<MY, MX, W>;
  return (size_t)C::TPW * C::TILE * sizeof(float2) + (size_t)C::NWAVE * 2 * sizeof(double) + 224 * sizeof(float2);
}

template <int MY, int MX, int OP, int MET>
static hipError_t launch_met(const Geometry& g, const TileArgs& a, hipStream_t s) {
  using C = Cfg<MY, MX>;
  const size_t lds = lds_bytes<MY, MX>();
  static bool attr_set = false;  // per instantiation, host-side
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)tile_kernel<MY, MX, OP, MET>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((tile_kernel<MY, MX, OP, MET>), dim3(g.grid), dim3(C::WG), lds, s, g, a);
  return hipGetLastError();
}

// one kernel per metric / GGN-weight code, so each variant gets its own register allocation
template <int MY, int MX, int OP>
static hipError_t launch_one(const Geometry& g, const TileArgs& a, hipStream_t s) {
  switch (met_code(OP, g)) {
    case 0: return launch_met<MY, MX, OP, 0>(g, a, s);
    case 1:
      if constexpr (OP == OP_LOSS || OP == OP_LINEARIZE || OP == OP_JVP || OP == OP_VJP)
        return launch_met<MY, MX, OP, 1>(g, a, s);
      break;
    case 2:
      if constexpr (OP == OP_LINEARIZE) return launch_met<MY, MX, OP, 2>(g, a, s);
      break;
    case 3:
      if constexpr (OP == OP_LINEARIZE) return launch_met<MY, MX, OP, 3>(g, a, s);
      break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <int MY, int MX, int OP>
static hipError_t launch_one_batch(const TileJob* jobs, const int* job_of_block, int nblocks, hipStream_t s) {
  using C = Cfg<MY, MX>;
  const size_t lds = lds_bytes<MY, MX>();
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)tile_batch_kernel<MY, MX, OP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((tile_batch_kernel<MY, MX, OP>), dim3(nblocks), dim3(C::WG), lds, s, jobs, job_of_block);
  return hipGetLastError();
}

// the batched LM attempt uses the linearisation, the GGN-vector product and the trial loss
template <int MY, int MX>
static hipError_t launch_op_batch(int op, const TileJob* jobs, const int* jb, int nb, hipStream_t s) {
  switch (op) {
    case OP_LOSS: return launch_one_batch<MY, MX, OP_LOSS>(jobs, jb, nb, s);
    case OP_LINEARIZE: return launch_one_batch<MY, MX, OP_LINEARIZE>(jobs, jb, nb, s);
    case OP_GGNV: return launch_one_batch<MY, MX, OP_GGNV>(jobs, jb, nb, s);
    default: return hipErrorInvalidValue;
  }
}

template <int MY, int MX>
static hipError_t launch_op(const Geometry& g, int op, const TileArgs& a, hipStream_t s) {
  switch (op) {
    case OP_FORWARD: return launch_one<MY, MX, OP_FORWARD>(g, a, s);
    case OP_LOSS: return launch_one<MY, MX, OP_LOSS>(g, a, s);
    case OP_LINEARIZE: return launch_one<MY, MX, OP_LINEARIZE>(g, a, s);
    case OP_JVP: return launch_one<MY, MX, OP_JVP>(g, a, s);
    case OP_VJP: return launch_one<MY, MX, OP_VJP>(g, a, s);
    case OP_VJP_RAND: return launch_one<MY, MX, OP_VJP_RAND>(g, a, s);
    case OP_GGNV: return launch_one<MY, MX, OP_GGNV>(g, a, s);
    case OP_DIAG_EXACT: return launch_one<MY, MX, OP_DIAG_EXACT>(g, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int MY>
static hipError_t launch_mx(const Geometry& g, int op, const TileArgs& a, hipStream_t s) {
  switch (g.mx) {
    case 16: return launch_op<MY, 16>(g, op, a, s);
    case 32: return launch_op<MY, 32>(g, op, a, s);
    case 64: return launch_op<MY, 64>(g, op, a, s);
    case 128: return launch_op<MY, 128>(g, op, a, s);
    default: return hipErrorInvalidValue;
  }
}

// GGN-vector product with the wide grouping: ceil(grid / 2) workgroups of twice the tiles
template <int MY, int MX>
static hipError_t launch_wide(const Geometry& g, const TileArgs& a, hipStream_t s) {
  using C = Cfg<MY, MX, 2>;
  const size_t lds = lds_bytes<MY, MX, 2>();
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)tile_kernel<MY, MX, OP_GGNV, 0, 2>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((tile_kernel<MY, MX, OP_GGNV, 0, 2>), dim3((g.grid + 1) / 2), dim3(C::WG), lds, s, g, a);
  return hipGetLastError();
}

// probe shapes of the generic kernel with at most 256 threads a tile (M <= 4096)
bool ggnv_wide_supported(int my, int mx) {
  const bool side = (my == 16 || my == 32 || my == 64 || my == 128) && (mx == 16 || mx == 32 || mx == 64 || mx == 128);
  return side && my * mx <= 4096;
}

#define PTLM_WIDE_SHAPES(X) \
  X(16, 16) X(16, 32) X(16, 64) X(16, 128) X(32, 16) X(32, 32) X(32, 64) X(32, 128) X(64, 16) X(64, 32) X(64, 64) \
  X(128, 16) X(128, 32)

static hipError_t launch_ggnv_wide(const Geometry& g, const TileArgs& a, hipStream_t s) {
#define PTLM_W(A, B) if (g.my == A && g.mx == B) return launch_wide<A, B>(g, a, s);
  PTLM_WIDE_SHAPES(PTLM_W)
#undef PTLM_W
  return hipErrorInvalidValue;
}

hipError_t launch_tile(const Geometry& g, int op, const TileArgs& a, hipStream_t s) {
  if (op == OP_GGNV && g.xform == 1 && ggnv_mfma_supported(g.my, g.mx)) return launch_ggnv_mfma(g, a, s);
  if (op == OP_GGNV && g.xform == 2 && ggnv_wide_supported(g.my, g.mx)) return launch_ggnv_wide(g, a, s);
  if (g.my == 256 && g.mx == 256) return launch_tile256(g, op, a, s);
  if (g.my == 128 && g.mx == 128 && tile128_handles(op)) return launch_tile128(g, op, a, s);
  if (g.my == g.mx && (g.my == 48 || g.my == 96)) return launch_tile3(g, op, a, s);
  switch (g.my) {
    case 16: return launch_mx<16>(g, op, a, s);
    case 32: return launch_mx<32>(g, op, a, s);
    case 64: return launch_mx<64>(g, op, a, s);
    case 128: return launch_mx<128>(g, op, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tile_batch(int my, int mx, int op, const TileJob* jobs, const int* jb, int nb, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  // a batch runs every problem with the transform its shape starts with
  // the matrix products where a shape starts with them; the wide grouping, which gives the
  // standard grouping's bits, is not used in batches (measured slower on the batch's short
  // segments of small problems)
  if (op == OP_GGNV && default_xform(my, mx) == 1) return launch_ggnv_mfma_batch(jobs, jb, nb, s);
  if (my == 256 && mx == 256) return launch_tile256_batch(op, jobs, jb, nb, s);
  if (my == 128 && mx == 128) return launch_tile128_batch(op, jobs, jb, nb, s);
  if (my == mx && (my == 48 || my == 96)) return launch_tile3_batch(my, op, jobs, jb, nb, s);
#define PTLM_B(A, B) if (my == A && mx == B) return launch_op_batch<A, B>(op, jobs, jb, nb, s);
  PTLM_B(16, 16) PTLM_B(16, 32) PTLM_B(16, 64) PTLM_B(16, 128)
  PTLM_B(32, 16) PTLM_B(32, 32) PTLM_B(32, 64) PTLM_B(32, 128)
  PTLM_B(64, 16) PTLM_B(64, 32) PTLM_B(64, 64) PTLM_B(64, 128)
  PTLM_B(128, 16) PTLM_B(128, 32) PTLM_B(128, 64)
#undef PTLM_B
  return hipErrorInvalidValue;
}

static bool side_ok(int m) { return m == 16 || m == 32 || m == 64 || m == 128; }
bool tile_shape_supported(int my, int mx) {
  return (side_ok(my) && side_ok(mx)) || (my == mx && (my == 48 || my == 96 || my == 256));
}

template <int MY, int MX>
static void cfg_of(int* wg, int* tpw, size_t* lds) {
  *wg = Cfg<MY, MX>::WG;
  *tpw = Cfg<MY, MX>::TPW;
  *lds = lds_bytes<MY, MX>();
}
static void cfg_dispatch(int my, int mx, int* wg, int* tpw, size_t* lds) {
  if (my == 128 && mx == 128) { *wg = tile128_threads(); *tpw = 1; *lds = tile128_lds_bytes(); return; }
#define PTLM_CFG(A, B) if (my == A && mx == B) { cfg_of<A, B>(wg, tpw, lds); return; }
  PTLM_CFG(16, 16) PTLM_CFG(16, 32) PTLM_CFG(16, 64) PTLM_CFG(16, 128)
  PTLM_CFG(32, 16) PTLM_CFG(32, 32) PTLM_CFG(32, 64) PTLM_CFG(32, 128)
  PTLM_CFG(64, 16) PTLM_CFG(64, 32) PTLM_CFG(64, 64) PTLM_CFG(64, 128)
  PTLM_CFG(128, 16) PTLM_CFG(128, 32) PTLM_CFG(128, 64)
#undef PTLM_CFG
  if (my == 256 && mx == 256) { *wg = 1024; *tpw = 1; *lds = tile256_lds_bytes(); return; }
  if (my == mx && (my == 48 || my == 96)) { *wg = 576; *tpw = tile3_per_wg(my); *lds = tile3_lds_bytes(my); return; }
  *wg = 0; *tpw = 0; *lds = 0;
}
int tile_threads(int my, int mx) { int w, t; size_t l; cfg_dispatch(my, mx, &w, &t, &l); return w; }
int tile_per_wg(int my, int mx) { int w, t; size_t l; cfg_dispatch(my, mx, &w, &t, &l); return t; }
size_t tile_lds_bytes(int my, int mx) { int w, t; size_t l; cfg_dispatch(my, mx, &w, &t, &l); return l; }

}  // namespace ptlm
