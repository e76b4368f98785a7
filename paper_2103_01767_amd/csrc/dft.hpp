// Register-level DFT building blocks for gfx950 wavefronts.
//
// Small DFTs of length 2, 3, 4, 6, 8 and 16 on complex values held in registers,
// natural order in and out, unnormalised:
//   forward  X[k] = sum_n x[n] exp(-2 pi i n k / R)
//   inverse  X[k] = sum_n x[n] exp(+2 pi i n k / R)
// Lengths 8 and 16 use one Cooley-Tukey split (2 x 4 and 4 x 4) with the
// inner twiddles as exact constants cos(pi j / 8), sin(pi j / 8).  These are
// the butterflies of every pass of the tile FFT (the transform F of the
// far-field model, eq:expected_count).
#pragma once
#include <hip/hip_runtime.h>

namespace ptlm {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// twiddle exp(-+2 pi i j / 16) applied with a compile-time j
template <bool INV, int J>
__device__ __forceinline__ float2 tw16(float2 a) {
  constexpr float C1 = 0.92387953251128674f;  // cos(pi/8)
  constexpr float S1 = 0.38268343236508977f;  // sin(pi/8)
  constexpr float R2 = 0.70710678118654752f;  // cos(pi/4)
  constexpr int j = J & 15;
  // exp(-2 pi i j / 16) = cos(pi j/8) - i sin(pi j/8)
  constexpr float cr[16] = {1.f, C1, R2, S1, 0.f, -S1, -R2, -C1, -1.f, -C1, -R2, -S1, 0.f, S1, R2, C1};
  constexpr float si[16] = {0.f, S1, R2, C1, 1.f, C1, R2, S1, 0.f, -S1, -R2, -C1, -1.f, -C1, -R2, -S1};
  if constexpr (j == 0) return a;
  else if constexpr (j == 4) return rot90<INV>(a);
  else if constexpr (j == 8) return make_float2(-a.x, -a.y);
  else if constexpr (j == 12) return rot90<!INV>(a);
  else {
    const float2 w = make_float2(cr[j], INV ? si[j] : -si[j]);
    return cmul(a, w);
  }
}

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const float2 t2 = cadd(a1, a3), t3 = rot90<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// 8 = 2 x 4:  n = n1 + 2 n2, k = k1 + 4 k2
template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  o1 = tw16<INV, 2>(o1);
  o2 = tw16<INV, 4>(o2);
  o3 = tw16<INV, 6>(o3);
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// 16 = 4 x 4:  n = n1 + 4 n2, k = k1 + 4 k2
template <bool INV>
__device__ __forceinline__ void dft16(float2* v) {
  float2 y[16];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    float2 a0 = v[n1], a1 = v[n1 + 4], a2 = v[n1 + 8], a3 = v[n1 + 12];
    dft4<INV>(a0, a1, a2, a3);
    y[n1 * 4 + 0] = a0; y[n1 * 4 + 1] = a1; y[n1 * 4 + 2] = a2; y[n1 * 4 + 3] = a3;
  }
  // inner twiddles W16^(n1 k1)
  y[1 * 4 + 1] = tw16<INV, 1>(y[1 * 4 + 1]);
  y[1 * 4 + 2] = tw16<INV, 2>(y[1 * 4 + 2]);
  y[1 * 4 + 3] = tw16<INV, 3>(y[1 * 4 + 3]);
  y[2 * 4 + 1] = tw16<INV, 2>(y[2 * 4 + 1]);
  y[2 * 4 + 2] = tw16<INV, 4>(y[2 * 4 + 2]);
  y[2 * 4 + 3] = tw16<INV, 6>(y[2 * 4 + 3]);
  y[3 * 4 + 1] = tw16<INV, 3>(y[3 * 4 + 1]);
  y[3 * 4 + 2] = tw16<INV, 6>(y[3 * 4 + 2]);
  y[3 * 4 + 3] = tw16<INV, 9>(y[3 * 4 + 3]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a0 = y[k1], a1 = y[4 + k1], a2 = y[8 + k1], a3 = y[12 + k1];
    dft4<INV>(a0, a1, a2, a3);
    v[k1] = a0; v[k1 + 4] = a1; v[k1 + 8] = a2; v[k1 + 12] = a3;
  }
}

// 3-point DFT: X1,2 = a - (b + c)/2 -+ i (sqrt(3)/2) (b - c) (forward; signs swap for inverse)
template <bool INV>
__device__ __forceinline__ void dft3(float2& a, float2& b, float2& c) {
  constexpr float H = 0.86602540378443865f;  // sqrt(3) / 2
  const float2 s = cadd(b, c), d = csub(b, c);
  const float2 m = make_float2(fmaf(-0.5f, s.x, a.x), fmaf(-0.5f, s.y, a.y));
  const float2 r = rot90<INV>(make_float2(H * d.x, H * d.y));  // -+ i (sqrt(3)/2) d
  a = cadd(a, s);
  b = cadd(m, r);
  c = csub(m, r);
}

// 6 = 2 x 3 (decimation in time): even and odd 3-point DFTs, then W6^k and a butterfly
template <bool INV>
__device__ __forceinline__ void dft6(float2* v) {
  constexpr float H = 0.86602540378443865f;
  float2 e0 = v[0], e1 = v[2], e2 = v[4];
  float2 o0 = v[1], o1 = v[3], o2 = v[5];
  dft3<INV>(e0, e1, e2);
  dft3<INV>(o0, o1, o2);
  // W6^1 = 1/2 -+ i sqrt(3)/2, W6^2 = -1/2 -+ i sqrt(3)/2
  o1 = cmul(o1, make_float2(0.5f, INV ? H : -H));
  o2 = cmul(o2, make_float2(-0.5f, INV ? H : -H));
  v[0] = cadd(e0, o0); v[3] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[4] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[5] = csub(e2, o2);
}

// DFT of compile-time length R in {1, 2, 3, 4, 6, 8, 16} on v[0..R)
template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* v) {
  if constexpr (R == 2) dft2<INV>(v[0], v[1]);
  else if constexpr (R == 3) dft3<INV>(v[0], v[1], v[2]);
  else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 6) dft6<INV>(v);
  else if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 16) dft16<INV>(v);
}

}  // namespace ptlm
