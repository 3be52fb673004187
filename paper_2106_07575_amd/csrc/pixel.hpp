// Per-pixel Poisson objective terms (Eqs. ML, gradient) and the device
// twiddle tables shared by the pattern kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "twiddles.h"

namespace ptyg {

constexpr float kLn2 = 0.69314718055994530942f;

// cos / sin (2 pi e / 256) for run-time indices
static __device__ const float kTwCosDev[kTwM] = PTYG_TW_COS;
static __device__ const float kTwSinDev[kTwM] = PTYG_TW_SIN;

// Per-pixel Poisson objective terms and residual factor (Eqs. ML, gradient).
//   phi   : deviance x - d - d log(max(x,eps)/d)  (x for d <= 0)
//   fterm : x - d log max(x, eps)                  (x for d <= 0)
//   fac   : 1 - d/x for x >= eps, 1 otherwise      (r = g * fac)
// The deviance is d * h with h = delta - log(1 + delta), delta = (x-d)/d:
// a series for |delta| < 0.1 (no cancellation near a fit), otherwise the
// log of the ratio x/d itself (1 + delta would round to 0 for x << d).
// A NaN intensity propagates into every term.
// Estimators: the Poisson maximum likelihood of Eq. ML, or least squares on
// the amplitudes (the paper's LS estimate; it gives no formula, the usual one
// is F = sum (|g| - sqrt d)^2 with the Wirtinger residual g - sqrt(d) g/|g|).
enum : int { kEstML = 0, kEstLS = 1 };

// Least-squares terms: phi = fterm = (sqrt x - sqrt d)^2, formed as
// ((x - d) / (sqrt x + sqrt d))^2 (x - d is exact near a fit); x for d <= 0;
// fac = 1 - sqrt(d / x) for x >= eps, 1 otherwise.  NaN intensities propagate.
__device__ __forceinline__ void pixel_terms_ls(float x, float d, float eps, float& phi, float& fac) {
  const bool dpos = !(d <= 0.0f);
  const bool big = x >= eps;
  const float sd = __builtin_sqrtf(dpos ? d : 0.0f);
  const float sx = __builtin_sqrtf(x);
  const float den = sx + sd;
  const float diff = (x - d) * __builtin_amdgcn_rcpf(den > 0.0f ? den : 1.0f);
  phi = dpos ? diff * diff : x;
  fac = (big && dpos) ? 1.0f - sd * __builtin_amdgcn_rsqf(big ? x : 1.0f) : 1.0f;
}

// Poisson terms, branch-free: both forms of the deviance are evaluated and
// selected (in the transform kernels the selects measured faster than
// skipping pixels without counts behind wave-uniform branches).
template <bool WANT_F, int EST = kEstML>
__device__ __forceinline__ void pixel_terms(float x, float d, float eps, float& phi, float& fterm,
                                            float& fac) {
  if constexpr (EST == kEstLS) {
    pixel_terms_ls(x, d, eps, phi, fac);
    if constexpr (WANT_F) fterm = phi;
    return;
  }
  const bool dpos = !(d <= 0.0f);  // NaN counts as positive so that it propagates
  const bool big = x >= eps;
  const float rd = __builtin_amdgcn_rcpf(dpos ? d : 1.0f);
  const float xg = big ? x : eps;
  const float delta = (xg - d) * rd;
  // series of delta - log1p(delta)
  float s = fmaf(-delta, 1.0f / 9.0f, 1.0f / 8.0f);
  s = fmaf(-delta, s, 1.0f / 7.0f);
  s = fmaf(-delta, s, 1.0f / 6.0f);
  s = fmaf(-delta, s, 1.0f / 5.0f);
  s = fmaf(-delta, s, 1.0f / 4.0f);
  s = fmaf(-delta, s, 1.0f / 3.0f);
  s = fmaf(-delta, s, 0.5f);
  const float hser = delta * delta * s;
  // x/d, scaled by 2^64 under the guard so that eps/d stays a normal number
  const float lr = __log2f(xg * rd * (big ? 1.0f : 0x1p64f)) - (big ? 0.0f : 64.0f);
  const float hlog = delta - lr * kLn2;
  const float h = fabsf(delta) < 0.1f ? hser : hlog;
  const float ph = d * h + (x - xg);
  phi = dpos ? ph : x;
  if constexpr (WANT_F) fterm = dpos ? x - d * __log2f(xg) * kLn2 : x;
  const float rx = __builtin_amdgcn_rcpf(big ? x : 1.0f);
  fac = (big && dpos) ? 1.0f - d * rx : 1.0f;
}

// The same terms with branches: on d > 0, and between the series and the
// logarithm, each skipped by a wave none of whose lanes needs it.  For the
// batched line search, whose elements all have counts and cluster near a
// fit or far from it trial by trial.
template <bool WANT_F, int EST = kEstML>
__device__ __forceinline__ void pixel_terms_br(float x, float d, float eps, float& phi, float& fterm,
                                               float& fac) {
  if constexpr (EST == kEstLS) {
    pixel_terms_ls(x, d, eps, phi, fac);
    if constexpr (WANT_F) fterm = phi;
    return;
  }
  phi = x;
  if constexpr (WANT_F) fterm = x;
  fac = 1.0f;
  if (!(d <= 0.0f)) {  // NaN counts as positive so that it propagates
    const bool big = x >= eps;
    const float rd = __builtin_amdgcn_rcpf(d);
    const float xg = big ? x : eps;
    const float delta = (xg - d) * rd;
    float h;
    if (fabsf(delta) < 0.1f) {
      float s = fmaf(-delta, 1.0f / 9.0f, 1.0f / 8.0f);
      s = fmaf(-delta, s, 1.0f / 7.0f);
      s = fmaf(-delta, s, 1.0f / 6.0f);
      s = fmaf(-delta, s, 1.0f / 5.0f);
      s = fmaf(-delta, s, 1.0f / 4.0f);
      s = fmaf(-delta, s, 1.0f / 3.0f);
      s = fmaf(-delta, s, 0.5f);
      h = delta * delta * s;
    } else {
      const float lr = __log2f(xg * rd * (big ? 1.0f : 0x1p64f)) - (big ? 0.0f : 64.0f);
      h = delta - lr * kLn2;
    }
    phi = d * h + (x - xg);
    if constexpr (WANT_F) fterm = x - d * __log2f(xg) * kLn2;
    fac = big ? 1.0f - d * __builtin_amdgcn_rcpf(x) : 1.0f;
  }
}

}  // namespace ptyg
