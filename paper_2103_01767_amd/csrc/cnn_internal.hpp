// Internal declarations of the convolutional-preconditioner kernels.
#pragma once
#include "internal.hpp"

namespace ptlm {

constexpr int CNN_CMAX = 32;  // largest channel count of a layer

hipError_t launch_conv(const float* x, int n, int cin, int h, int w, const float* wt, const float* b, float* y,
                       int cout, int relu, const float* mask, hipStream_t s);
// re-lay weights W (cout, cin, 3, 3) for the forward conv (backward = false) or for the
// data-gradient conv (flipped kernel, swapped channels)
hipError_t launch_wt(const float* W, int cout, int cin, float* wt, bool backward, hipStream_t s);
// gW, gb of one layer into g (cout*cin*9 + cout floats); part: per-block scratch
hipError_t launch_wgrad(const float* a, int n, int cin, int h, int w, const float* gz, int cout, float* part,
                        float* g, hipStream_t s);
// scal[0] = count, scal[1] = loss; gz (nullable) = mask (r - t) / count
hipError_t launch_loss(const float* r, const float* t, const float* mask, size_t len, double* part, double* scal,
                       float* gz, hipStream_t s);
hipError_t launch_adam(size_t n, float* p, const float* g, float* m, float* v, int step, float lr, float b1,
                       float b2, float eps, hipStream_t s);
// 3 feature maps (ny*nx each) from the handle's linearisation probe; scal: 2 doubles
hipError_t launch_features(const Geometry& g, float* feat, double* scal, hipStream_t s);
// learned diagonal (2n floats) from the network output r (2 x ny x nx); scal: 2 doubles
hipError_t launch_learned_diag(const Geometry& g, float* d, const float* r, double* scal, double floor_frac,
                               hipStream_t s);

}  // namespace ptlm
