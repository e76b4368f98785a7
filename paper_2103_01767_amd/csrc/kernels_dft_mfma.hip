// DFT-as-MFMA form of the GGN-vector product for 16 x 16 and 32 x 32 probes: the alternative to
// the register / LDS FFT of the tile kernels, chosen per handle (the default for 16 x 16, where
// it is measured faster; ptlm_set_transform, ptlm_autotune).
//
// The unnormalised 2D DFT of an L x L tile X is Y = F X F with F[n][k] = exp(-2 pi i n k / L)
// (symmetric), the transform F of eq:expected_count up to the 1/L of the unitary form, which
// the stored phasor field carries.  Each wavefront runs its own segment of positions and does
// both products on the FP32 matrix cores: v_mfma_f32_16x16x4_f32 (L = 16: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; register r holds C[4 (l / 16) + r][l % 16]) or
// v_mfma_f32_32x32x2_f32 (L = 32: A[l % 32][l / 32], B[l / 32][l % 32]; register r holds
// C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]).  Write row(r, g) for the row of register r in lane
// group g (g = l / 16 or l / 32) and c for the column l % L.  Slice s of a product feeds the
// contraction index k = row(s, g) from lane group g, in both operands, so:
//   step 1  T^T = X^T F: lane (g, c) supplies X[row(s, g)][c] (its own pixels, gathered) and
//           F[row(s, g)][c]; the result holds T[c][row(r, g)] in register r;
//   step 2  Y = T F: lane (g, c) supplies T[c][row(s, g)] -- register s of step 1 -- and the
//           same F values; the result holds Y[row(r, g)][c] in register r.
// The output layout of step 2 is the input layout of step 1, so the per-pixel operation and the
// inverse transform (conj F) follow with no data exchange: no LDS, no barriers.  A complex
// product is four real products (the imaginary part of F negated where it enters a real part).
// The overlap-add is that of the tile kernels: the segment's private strip read-modify-written
// per position, the probe part summed in registers.
#include "dft.hpp"
#include "internal.hpp"
#include "tile_pixel.hpp"

namespace ptlm {
namespace mfmadft {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
constexpr int WAVES = 4;  // wavefronts (segments) per workgroup

template <int L>
struct Mf;
template <>
struct Mf<16> {
  static constexpr int NS = 4;  // slices of a product = registers of a result
  typedef v4f acc;
  __device__ static __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int r, int g) { return 4 * g + r; }
};
template <>
struct Mf<32> {
  static constexpr int NS = 16;
  typedef v16f acc;
  __device__ static __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int r, int g) { return 8 * (r / 4) + 4 * g + r % 4; }
};

// exp(-2 pi i m / L), from FP64
__device__ __forceinline__ float2 wL(int m, int L) {
  double s, c;
  sincospi(-2.0 * (double)(m % L) / (double)L, &s, &c);
  return make_float2((float)c, (float)s);
}

// one wavefront: every position of segment `seg`
template <int L>
__device__ __forceinline__ void ggnv_body(const Geometry& g, const TileArgs& a, int seg, int lane) {
  using X = Mf<L>;
  constexpr int NS = X::NS, M = L * L;
  typedef typename X::acc acc;
  const int lg = lane / L, lc = lane % L;  // lane group, matrix column
  const int kbeg = g.seg_start[seg], kend = g.seg_start[seg + 1];
  const bool joint = g.joint != 0;

  // F[row(s, lg)][lc] and its negated imaginary part
  float Fr[NS], Fi[NS], nFi[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const float2 w = wL(X::row(s, lg) * lc, L);
    Fr[s] = w.x;
    Fi[s] = w.y;
    nFi[s] = -w.y;
  }

  float2* strip = g.strips + g.seg_off[seg];
  const int4 box = g.seg_box[seg];
  if (kend > kbeg) {
    const int2 p0 = g.pos[kbeg];
    const int area = box.z * box.w;
    for (int i = lane; i < area; i += 64) {
      const int Y = box.x + i / box.w, Xc = box.y + i % box.w;
      if ((unsigned)(Y - p0.x) >= (unsigned)L || (unsigned)(Xc - p0.y) >= (unsigned)L)
        strip[i] = make_float2(0.f, 0.f);
    }
  }
  float2 accP[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) accP[r] = make_float2(0.f, 0.f);
  const float isq = rsqrtf((float)M);
  const float bgv = a.bg_add ? (float)((double)g.background + *a.bg_add) : g.background;
  double s0 = 0.0, s1 = 0.0, tr = 0.0;

  for (int k = kbeg; k < kend; ++k) {
    const int2 p = g.pos[k];
    const int ry = p.x, rx = p.y;
    // ---- gather d psi at pixels (row(s, lg), lc); keep P and the object window for the adjoint
    float Xr[NS], Xi[NS];
    float2 Pv[NS], Ov[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int row = X::row(s, lg);
      const size_t oi = (size_t)(ry + row) * g.nx + rx + lc;
      Pv[s] = a.P[row * L + lc];
      Ov[s] = a.O[oi];
      float2 x = cmul(Pv[s], a.vO[oi]);
      if (a.vP) x = cadd(x, cmul(a.vP[row * L + lc], Ov[s]));
      Xr[s] = x.x;
      Xi[s] = x.y;
    }
    // ---- forward transform: T^T = X^T F, then Y = T F
    acc Tr = {}, Ti = {}, Yr = {}, Yi = {};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      Tr = X::mma(Xr[s], Fr[s], Tr);
      Tr = X::mma(Xi[s], nFi[s], Tr);
      Ti = X::mma(Xr[s], Fi[s], Ti);
      Ti = X::mma(Xi[s], Fr[s], Ti);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      Yr = X::mma(Tr[s], Fr[s], Yr);
      Yr = X::mma(Ti[s], nFi[s], Yr);
      Yi = X::mma(Tr[s], Fi[s], Yi);
      Yi = X::mma(Ti[s], Fr[s], Yi);
    }
    // ---- loss-Hessian weighting at (ky, kx) = (row(r, lg), lc)
    float Qr[NS], Qi[NS];
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      float2 v = make_float2(Yr[r], Yi[r]);
      pixel_op<OP_GGNV, 0>(g, a, (size_t)k * M + X::row(r, lg) * L + lc, isq, bgv, v, s0, s1, tr);
      Qr[r] = v.x;
      Qi[r] = v.y;
    }
    // ---- inverse transform with conj F: W^T = Q^T conj F, then U = W conj F
    acc Wr = {}, Wi = {}, Ur = {}, Ui = {};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      Wr = X::mma(Qr[s], Fr[s], Wr);
      Wr = X::mma(Qi[s], Fi[s], Wr);
      Wi = X::mma(Qi[s], Fr[s], Wi);
      Wi = X::mma(Qr[s], nFi[s], Wi);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      Ur = X::mma(Wr[s], Fr[s], Ur);
      Ur = X::mma(Wi[s], Fi[s], Ur);
      Ui = X::mma(Wi[s], Fr[s], Ui);
      Ui = X::mma(Wr[s], nFi[s], Ui);
    }
    // ---- overlap-add: conj(P) u into the strip, conj(S_k O) u into the probe partial
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const float2 u = make_float2(Ur[r], Ui[r]);
      float2* sp = strip + (size_t)(ry + X::row(r, lg) - box.x) * box.w + (rx + lc - box.y);
      const float2 c = cmulc(u, Pv[r]);
      *sp = k == kbeg ? c : cadd(*sp, c);
      if (joint) accP[r] = cadd(accP[r], cmulc(u, Ov[r]));
    }
  }
  if (joint) {
    float2* pp = g.probe_part + (size_t)seg * M;
#pragma unroll
    for (int r = 0; r < NS; ++r) pp[X::row(r, lg) * L + lc] = accP[r];
  }
}

template <int L>
__global__ __launch_bounds__(64 * WAVES) void ggnv_kernel(Geometry g, TileArgs a) {
  if (a.predicate && *a.predicate == 0) return;
  const int seg = xcd_block(blockIdx.x, gridDim.x) * WAVES + (int)(threadIdx.x >> 6);
  if (seg >= g.nseg) return;
  ggnv_body<L>(g, a, seg, threadIdx.x & 63);
}

// batched 16 x 16 class: block b of a job runs the job's segments 16 b .. 16 b + 15 (those of
// the tile kernel's block b), one per wavefront
constexpr int BATCH_WAVES = 16;
__global__ __launch_bounds__(64 * BATCH_WAVES) void ggnv16_batch_kernel(const TileJob* __restrict__ jobs,
                                                                       const int* __restrict__ job_of_block) {
  const TileJob& J = jobs[job_of_block[blockIdx.x]];
  if (J.a.predicate && *J.a.predicate == 0) return;
  const int seg = ((int)blockIdx.x - J.block0) * BATCH_WAVES + (int)(threadIdx.x >> 6);
  if (seg >= J.g.nseg) return;
  ggnv_body<16>(J.g, J.a, seg, threadIdx.x & 63);
}

}  // namespace mfmadft

bool ggnv_mfma_supported(int my, int mx) { return my == mx && (my == 16 || my == 32); }
int default_xform(int my, int mx) {
  if (my == 16 && mx == 16) return 1;
  if (my == 32 && mx == 32) return 2;
  return 0;
}

hipError_t launch_ggnv_mfma_batch(const TileJob* jobs, const int* jb, int nb, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(mfmadft::ggnv16_batch_kernel, dim3(nb), dim3(64 * mfmadft::BATCH_WAVES), 0, s, jobs, jb);
  return hipGetLastError();
}

hipError_t launch_ggnv_mfma(const Geometry& g, const TileArgs& a, hipStream_t s) {
  const int nblk = (g.nseg + mfmadft::WAVES - 1) / mfmadft::WAVES;
  if (g.my == 16 && g.mx == 16)
    hipLaunchKernelGGL(mfmadft::ggnv_kernel<16>, dim3(nblk), dim3(64 * mfmadft::WAVES), 0, s, g, a);
  else if (g.my == 32 && g.mx == 32)
    hipLaunchKernelGGL(mfmadft::ggnv_kernel<32>, dim3(nblk), dim3(64 * mfmadft::WAVES), 0, s, g, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace ptlm
