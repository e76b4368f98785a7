// C ABI of the convolutional preconditioner network: sizes, forward, loss + gradient,
// Adam, the object-grid features of a problem, the learned diagonal, and the hook that
// lets the LM step refresh its preconditioner from the network after every linearisation.
#include <algorithm>
#include <cstring>

#include "api_internal.hpp"
#include "cnn_internal.hpp"

namespace ptlm {

static size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

struct CnnLayout {
  size_t act[16];       // activations a_1..a_L (a_0 is the caller's input)
  size_t gz0, gz1;      // gradient ping-pong buffers
  size_t wt, wtb, zero; // re-laid weights (forward / data gradient), zero bias
  size_t part, lpart, scal;
  size_t feat, r;       // features (3 maps) and output (cout maps) for the LM hook
  size_t bytes;
};

static int chan(const ptlm_cnn_desc& d, int l) {  // channels of a_l
  if (l == 0) return d.cin;
  if (l == d.layers) return d.cout;
  return d.cmid;
}

static ptlm_status check_desc(const ptlm_cnn_desc* d) {
  if (!d) return fail(PTLM_EINVAL, "cnn desc is null");
  if (d->n < 1 || d->h < 1 || d->w < 1 || d->layers < 1 || d->layers > 15)
    return fail(PTLM_EINVAL, "cnn: n, h, w >= 1 and 1 <= layers <= 15");
  const int ok[] = {2, 3, 4, 8, 16, 32};
  auto good = [&](int c) { return std::find(std::begin(ok), std::end(ok), c) != std::end(ok); };
  if (d->cin < 1 || d->cin > CNN_CMAX || !good(d->cmid) || !good(d->cout) || !good(d->cin) )
    return fail(PTLM_EINVAL, "cnn: channel counts must be 2, 3, 4, 8, 16 or 32");
  return PTLM_OK;
}

static CnnLayout layout(const ptlm_cnn_desc& d) {
  CnnLayout L{};
  const size_t hw = (size_t)d.h * d.w;
  size_t o = 0;
  auto take = [&](size_t b) { const size_t at = o; o = align_up(o + b); return at; };
  for (int l = 1; l <= d.layers; ++l) L.act[l] = take((size_t)d.n * chan(d, l) * hw * sizeof(float));
  L.gz0 = take((size_t)d.n * CNN_CMAX * hw * sizeof(float));
  L.gz1 = take((size_t)d.n * CNN_CMAX * hw * sizeof(float));
  L.wt = take((size_t)CNN_CMAX * 9 * CNN_CMAX * sizeof(float));
  L.wtb = take((size_t)CNN_CMAX * 9 * CNN_CMAX * sizeof(float));
  L.zero = take(CNN_CMAX * sizeof(float));
  const size_t nblk = (size_t)d.n * ((d.h + 15) / 16) * ((d.w + 15) / 16);
  L.part = take(nblk * (CNN_CMAX * CNN_CMAX * 9 + CNN_CMAX) * sizeof(float));
  L.lpart = take(256 * 2 * sizeof(double));
  L.scal = take(4 * sizeof(double));
  L.feat = take((size_t)3 * hw * sizeof(float));
  L.r = take((size_t)d.cout * hw * sizeof(float));
  L.bytes = o;
  return L;
}

static size_t param_count(const ptlm_cnn_desc& d) {
  size_t n = 0;
  for (int l = 0; l < d.layers; ++l) n += (size_t)chan(d, l + 1) * chan(d, l) * 9 + chan(d, l + 1);
  return n;
}

#define CNN_HIP(call, where)                          \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// forward through all layers; the last layer writes `out` (or act[L] when out is null)
static ptlm_status cnn_forward_impl(const ptlm_cnn_desc& d, const float* params, const float* x, float* out,
                                    char* ws, hipStream_t s) {
  const CnnLayout L = layout(d);
  const float* a = x;
  size_t po = 0;
  for (int l = 0; l < d.layers; ++l) {
    const int ci = chan(d, l), co = chan(d, l + 1);
    const float* W = params + po;
    const float* b = W + (size_t)co * ci * 9;
    po += (size_t)co * ci * 9 + co;
    float* y = (l == d.layers - 1 && out) ? out : (float*)(ws + L.act[l + 1]);
    CNN_HIP(launch_wt(W, co, ci, (float*)(ws + L.wt), false, s), "cnn wt");
    CNN_HIP(launch_conv(a, d.n, ci, d.h, d.w, (const float*)(ws + L.wt), b, y, co, l < d.layers - 1, nullptr, s),
            "cnn conv");
    a = y;
  }
  return PTLM_OK;
}

}  // namespace ptlm

using namespace ptlm;

extern "C" {

ptlm_status ptlm_cnn_param_count(const ptlm_cnn_desc* d, size_t* count) {
  ptlm_status st = check_desc(d);
  if (st != PTLM_OK) return st;
  if (!count) return fail(PTLM_EINVAL, "count is null");
  *count = param_count(*d);
  return PTLM_OK;
}

ptlm_status ptlm_cnn_workspace_bytes(const ptlm_cnn_desc* d, size_t* bytes) {
  ptlm_status st = check_desc(d);
  if (st != PTLM_OK) return st;
  if (!bytes) return fail(PTLM_EINVAL, "bytes is null");
  *bytes = layout(*d).bytes;
  return PTLM_OK;
}

ptlm_status ptlm_cnn_forward(const ptlm_cnn_desc* d, const float* d_params, const float* d_x, float* d_out,
                             void* d_ws, size_t ws_bytes, void* stream) {
  ptlm_status st = check_desc(d);
  if (st != PTLM_OK) return st;
  if (!d_params || !d_x || !d_out) return fail(PTLM_EINVAL, "null array");
  if (!d_ws || ws_bytes < layout(*d).bytes) return fail(PTLM_EWORKSPACE, "cnn workspace too small");
  return cnn_forward_impl(*d, d_params, d_x, d_out, (char*)d_ws, (hipStream_t)stream);
}

ptlm_status ptlm_cnn_loss_grad(const ptlm_cnn_desc* d, const float* d_params, const float* d_x, const float* d_t,
                               const float* d_mask, double* d_loss, float* d_grad, void* d_ws, size_t ws_bytes,
                               void* stream) {
  ptlm_status st = check_desc(d);
  if (st != PTLM_OK) return st;
  if (!d_params || !d_x || !d_t || !d_mask || !d_loss || !d_grad) return fail(PTLM_EINVAL, "null array");
  const CnnLayout L = layout(*d);
  if (!d_ws || ws_bytes < L.bytes) return fail(PTLM_EWORKSPACE, "cnn workspace too small");
  char* ws = (char*)d_ws;
  hipStream_t s = (hipStream_t)stream;
  st = cnn_forward_impl(*d, d_params, d_x, nullptr, ws, s);
  if (st != PTLM_OK) return st;
  const size_t hw = (size_t)d->h * d->w;
  const float* r = (const float*)(ws + L.act[d->layers]);
  float* gz = (float*)(ws + L.gz0);
  float* gz_next = (float*)(ws + L.gz1);
  CNN_HIP(launch_loss(r, d_t, d_mask, (size_t)d->n * d->cout * hw, (double*)(ws + L.lpart),
                      (double*)(ws + L.scal), gz, s), "cnn loss");
  CNN_HIP(hipMemsetAsync(ws + L.zero, 0, CNN_CMAX * sizeof(float), s), "cnn zero");
  // parameter offsets per layer
  size_t offs[16];
  size_t po = 0;
  for (int l = 0; l < d->layers; ++l) {
    offs[l] = po;
    po += (size_t)chan(*d, l + 1) * chan(*d, l) * 9 + chan(*d, l + 1);
  }
  for (int l = d->layers - 1; l >= 0; --l) {
    const int ci = chan(*d, l), co = chan(*d, l + 1);
    const float* a_in = l == 0 ? d_x : (const float*)(ws + L.act[l]);
    CNN_HIP(launch_wgrad(a_in, d->n, ci, d->h, d->w, gz, co, (float*)(ws + L.part), d_grad + offs[l], s),
            "cnn wgrad");
    if (l > 0) {
      // d a_l = transposed conv of gz, times the ReLU derivative of a_l
      CNN_HIP(launch_wt(d_params + offs[l], co, ci, (float*)(ws + L.wtb), true, s), "cnn wtb");
      CNN_HIP(launch_conv(gz, d->n, co, d->h, d->w, (const float*)(ws + L.wtb), (const float*)(ws + L.zero),
                          gz_next, ci, 0, a_in, s), "cnn dgrad");
      std::swap(gz, gz_next);
    }
  }
  CNN_HIP(hipMemcpyAsync(d_loss, ws + L.scal + sizeof(double), sizeof(double), hipMemcpyDeviceToDevice, s),
          "cnn loss copy");
  return PTLM_OK;
}

ptlm_status ptlm_cnn_adam(size_t count, float* d_params, const float* d_grad, float* d_m, float* d_v, int32_t step,
                          float lr, float beta1, float beta2, float eps, void* stream) {
  if (!d_params || !d_grad || !d_m || !d_v) return fail(PTLM_EINVAL, "null array");
  if (step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(PTLM_EINVAL, "invalid Adam parameters");
  CNN_HIP(launch_adam(count, d_params, d_grad, d_m, d_v, step, lr, beta1, beta2, eps, (hipStream_t)stream), "adam");
  return PTLM_OK;
}

ptlm_status ptlm_cnn_features(ptlm_handle* h, float* d_feat, void* stream) {
  if (!h || !d_feat) return fail(PTLM_EINVAL, "null argument");
  CNN_HIP(launch_features(h->g, d_feat, (double*)(h->ws + h->plan.off.scal) + 8, (hipStream_t)stream), "features");
  return PTLM_OK;
}

ptlm_status ptlm_learned_precond(ptlm_handle* h, const float* d_r, float* d_precond, void* stream) {
  if (!h || !d_r || !d_precond) return fail(PTLM_EINVAL, "null argument");
  CNN_HIP(launch_learned_diag(h->g, d_precond, d_r, (double*)(h->ws + h->plan.off.scal) + 10, 1e-6,
                              (hipStream_t)stream), "learned precond");
  return PTLM_OK;
}

ptlm_status ptlm_lm_set_cnn(ptlm_handle* h, const ptlm_cnn_desc* d, const float* d_params, void* d_ws,
                            size_t ws_bytes) {
  if (!h) return fail(PTLM_EINVAL, "handle is null");
  if (!d) {  // unregister
    h->cnn_params = nullptr;
    return PTLM_OK;
  }
  ptlm_status st = check_desc(d);
  if (st != PTLM_OK) return st;
  if (d->n != 1 || d->h != h->g.ny || d->w != h->g.nx || d->cin != 3 || d->cout != 2)
    return fail(PTLM_EINVAL, "cnn for the LM: n = 1, h x w = object shape, 3 inputs, 2 outputs");
  if (!d_params) return fail(PTLM_EINVAL, "params are null");
  if (!d_ws || ws_bytes < layout(*d).bytes) return fail(PTLM_EWORKSPACE, "cnn workspace too small");
  h->cnn = *d;
  h->cnn_params = d_params;
  h->cnn_ws = (char*)d_ws;
  h->cnn_ready = false;
  h->cnn_count = 0;
  return PTLM_OK;
}

ptlm_status ptlm_lm_set_cnn_refresh(ptlm_handle* h, int32_t every) {
  if (!h) return fail(PTLM_EINVAL, "handle is null");
  if (every < 0) return fail(PTLM_EINVAL, "every must be >= 0");
  h->cnn_every = every;
  h->cnn_count = 0;
  return PTLM_OK;
}

}  // extern "C"

namespace ptlm {
// features (from the linearisation probe) -> network -> r, kept in the network workspace
ptlm_status cnn_refresh(ptlm_handle* h, hipStream_t s, const float2* P) {
  const CnnLayout L = layout(h->cnn);
  float* feat = (float*)(h->cnn_ws + L.feat);
  float* r = (float*)(h->cnn_ws + L.r);
  double* scal = (double*)(h->ws + h->plan.off.scal) + 8;
  Geometry gf = h->g;
  if (P) gf.P_lin = const_cast<float2*>(P);  // the features read the probe only
  CNN_HIP(launch_features(gf, feat, scal, s), "lm features");
  const ptlm_status st = cnn_forward_impl(h->cnn, h->cnn_params, feat, r, h->cnn_ws, s);
  if (st != PTLM_OK) return st;
  h->cnn_ready = true;
  return PTLM_OK;
}

// the kept network output r (2 maps of the object grid) of the handle's registered network
const float* cnn_output(const ptlm_handle* h) {
  const CnnLayout L = layout(h->cnn);
  return (const float*)(h->cnn_ws + L.r);
}
}  // namespace ptlm
