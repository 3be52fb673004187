// In-register FFT building blocks for gfx950 (wave64).
//
// The ptychography operator G = F Q (Eq. fwd_model) needs batched unitary
// 2-D DFTs of every exit wave, and G^H = Q^H F^H (text after Eq. gradient)
// needs their adjoints.  A 2-D transform is built from 1-D transforms held
// in registers: each lane owns whole lines (or half lines split across the
// two halves of the wave), so the butterflies need no shuffles, and one LDS
// transpose between the two axes (pattern.hpp) is the only exchange.
//
//  * dif<S, L>  : unnormalised length-L DFT with exponent sign S, radix-4
//                 decimation in frequency (one radix-2 stage first when
//                 log2 L is odd); natural order in, digit-reversed order out
//                 (freq_of_slot gives the frequency held by each slot).
//  * dit<S, L>  : the exact adjoint network (stages reversed, twiddles
//                 conjugated): digit-reversed order in, natural order out.
//                 dit<+1> after dif<-1> is L times the identity, so the
//                 inverse transform is the adjoint to rounding.
//  * xlane_*    : a radix-2 stage between lane l and lane l+32 using
//                 v_permlane32_swap, for lines of 128 split over two lanes.
//
// All indices and twiddles are compile-time constants after template
// expansion; the register arrays never see a run-time index.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "twiddles.h"

namespace ptyg {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by S*i (S = +1 or -1)
template <int S>
__device__ __forceinline__ float2 mul_si(float2 a) {
  if constexpr (S < 0) return make_float2(a.y, -a.x);
  else return make_float2(-a.y, a.x);
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// Multiply by W_L^E = exp(S * 2 pi i E / L), trivial angles special-cased.
template <int L, int E, int S>
__device__ __forceinline__ float2 tw(float2 a) {
  constexpr int e = ((E % L) + L) % L;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (2 * e == L) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (4 * e == L) {
    return mul_si<S>(a);
  } else if constexpr (4 * e == 3 * L) {
    return mul_si<-S>(a);
  } else {
    static_assert(kTwM % L == 0, "transform length exceeds the twiddle table");
    constexpr int idx = e * (kTwM / L);
    constexpr float c = kTwCos[idx];
    constexpr float s = S > 0 ? kTwSin[idx] : -kTwSin[idx];
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// Frequency held by slot `pos` after dif<S, L> (digit reversal, radix 4 with
// a radix-2 top stage when log2 L is odd).
constexpr int freq_of_slot(int L, int pos) {
  if (L == 1) return 0;
  if (ilog2(L) & 1) {
    const int h = L / 2;
    return 2 * freq_of_slot(h, pos % h) + pos / h;
  }
  const int q = L / 4;
  return 4 * freq_of_slot(q, pos % q) + pos / q;
}
constexpr int slot_of_freq(int L, int f) {
  for (int p = 0; p < L; ++p)
    if (freq_of_slot(L, p) == f) return p;
  return -1;
}

// ---------------------------------------------------------------- forward DIF
template <int S, int L, int OFF, int J>
__device__ __forceinline__ void dif_r2_bfly(float2* v) {
  constexpr int H = L / 2;
  const float2 a = v[OFF + J], b = v[OFF + J + H];
  v[OFF + J] = cadd(a, b);
  v[OFF + J + H] = tw<L, J, S>(csub(a, b));
}
template <int S, int L, int OFF, int J>
__device__ __forceinline__ void dif_r4_bfly(float2* v) {
  constexpr int Q = L / 4;
  const float2 x0 = v[OFF + J], x1 = v[OFF + J + Q], x2 = v[OFF + J + 2 * Q], x3 = v[OFF + J + 3 * Q];
  const float2 t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3);
  const float2 t3 = mul_si<S>(csub(x1, x3));
  v[OFF + J] = cadd(t0, t2);
  v[OFF + J + Q] = tw<L, J, S>(cadd(t1, t3));
  v[OFF + J + 2 * Q] = tw<L, 2 * J, S>(csub(t0, t2));
  v[OFF + J + 3 * Q] = tw<L, 3 * J, S>(csub(t1, t3));
}
template <int S, int L, int OFF, int... J>
__device__ __forceinline__ void dif_r2_stage(float2* v, std::integer_sequence<int, J...>) {
  (dif_r2_bfly<S, L, OFF, J>(v), ...);
}
template <int S, int L, int OFF, int... J>
__device__ __forceinline__ void dif_r4_stage(float2* v, std::integer_sequence<int, J...>) {
  (dif_r4_bfly<S, L, OFF, J>(v), ...);
}

template <int S, int L, int OFF = 0>
__device__ __forceinline__ void dif(float2* v) {
  if constexpr (L == 1) {
    return;
  } else if constexpr (ilog2(L) & 1) {
    dif_r2_stage<S, L, OFF>(v, std::make_integer_sequence<int, L / 2>{});
    dif<S, L / 2, OFF>(v);
    dif<S, L / 2, OFF + L / 2>(v);
  } else {
    constexpr int Q = L / 4;
    dif_r4_stage<S, L, OFF>(v, std::make_integer_sequence<int, Q>{});
    dif<S, Q, OFF>(v);
    dif<S, Q, OFF + Q>(v);
    dif<S, Q, OFF + 2 * Q>(v);
    dif<S, Q, OFF + 3 * Q>(v);
  }
}

// ------------------------------------------------------- adjoint network (DIT)
template <int S, int L, int OFF, int J>
__device__ __forceinline__ void dit_r2_bfly(float2* v) {
  constexpr int H = L / 2;
  const float2 a = v[OFF + J];
  const float2 b = tw<L, J, S>(v[OFF + J + H]);
  v[OFF + J] = cadd(a, b);
  v[OFF + J + H] = csub(a, b);
}
template <int S, int L, int OFF, int J>
__device__ __forceinline__ void dit_r4_bfly(float2* v) {
  constexpr int Q = L / 4;
  const float2 z0 = v[OFF + J];
  const float2 z1 = tw<L, J, S>(v[OFF + J + Q]);
  const float2 z2 = tw<L, 2 * J, S>(v[OFF + J + 2 * Q]);
  const float2 z3 = tw<L, 3 * J, S>(v[OFF + J + 3 * Q]);
  // x_q = sum_r (S i)^(q r) z_r
  const float2 t0 = cadd(z0, z2), t1 = csub(z0, z2), t2 = cadd(z1, z3);
  const float2 t3 = mul_si<S>(csub(z1, z3));
  v[OFF + J] = cadd(t0, t2);
  v[OFF + J + Q] = cadd(t1, t3);
  v[OFF + J + 2 * Q] = csub(t0, t2);
  v[OFF + J + 3 * Q] = csub(t1, t3);
}
template <int S, int L, int OFF, int... J>
__device__ __forceinline__ void dit_r2_stage(float2* v, std::integer_sequence<int, J...>) {
  (dit_r2_bfly<S, L, OFF, J>(v), ...);
}
template <int S, int L, int OFF, int... J>
__device__ __forceinline__ void dit_r4_stage(float2* v, std::integer_sequence<int, J...>) {
  (dit_r4_bfly<S, L, OFF, J>(v), ...);
}

template <int S, int L, int OFF = 0>
__device__ __forceinline__ void dit(float2* v) {
  if constexpr (L == 1) {
    return;
  } else if constexpr (ilog2(L) & 1) {
    dit<S, L / 2, OFF>(v);
    dit<S, L / 2, OFF + L / 2>(v);
    dit_r2_stage<S, L, OFF>(v, std::make_integer_sequence<int, L / 2>{});
  } else {
    constexpr int Q = L / 4;
    dit<S, Q, OFF>(v);
    dit<S, Q, OFF + Q>(v);
    dit<S, Q, OFF + 2 * Q>(v);
    dit<S, Q, OFF + 3 * Q>(v);
    dit_r4_stage<S, L, OFF>(v, std::make_integer_sequence<int, Q>{});
  }
}

// ------------------------------------------------ cross-lane radix-2 (l, l+32)
// Lines of 2E points split over lanes l (h = 0) and l + 32 (h = 1): lane h
// holds the E samples x[2m + h].  Forward: per-lane dif<S, E> gives E_h[k];
// then X[k'] = E_0[k'] + W^k' E_1[k'], X[k' + E] = E_0[k'] - W^k' E_1[k'],
// with lane h producing k' = k + (E/2) h for k < E/2.  Slot of E_h[k]
// (k < E/2) receives X[k + (E/2) h], slot of E_h[k + E/2] receives
// X[k + E + (E/2) h].
__device__ __forceinline__ void swap32(float2& a, float2& b) {
  auto rx = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.x), __float_as_uint(b.x), false, false);
  auto ry = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.y), __float_as_uint(b.y), false, false);
  a = make_float2(__uint_as_float(rx[0]), __uint_as_float(ry[0]));
  b = make_float2(__uint_as_float(rx[1]), __uint_as_float(ry[1]));
}

template <int S, int E, int K>
__device__ __forceinline__ void xlane_fwd_one(float2* v, bool h) {
  constexpr int sa = slot_of_freq(E, K), sb = slot_of_freq(E, K + E / 2);
  float2 a = v[sa], b = v[sb];
  swap32(a, b);  // lane h=0: (E0[k], E1[k]); lane h=1: (E0[k+E/2], E1[k+E/2])
  float2 c = tw<2 * E, K, S>(b);
  const float2 cr = mul_si<S>(c);  // W^(E/2) = S i for the upper lanes
  c = h ? cr : c;
  v[sa] = cadd(a, c);
  v[sb] = csub(a, c);
}
template <int S, int E, int... K>
__device__ __forceinline__ void xlane_fwd_all(float2* v, bool h, std::integer_sequence<int, K...>) {
  (xlane_fwd_one<S, E, K>(v, h), ...);
}
template <int S, int E>
__device__ __forceinline__ void xlane_fwd(float2* v, bool h) {
  xlane_fwd_all<S, E>(v, h, std::make_integer_sequence<int, E / 2>{});
}

// Adjoint of xlane_fwd<-S> (use S = +1 after a forward with S = -1).
template <int S, int E, int K>
__device__ __forceinline__ void xlane_adj_one(float2* v, bool h) {
  constexpr int sa = slot_of_freq(E, K), sb = slot_of_freq(E, K + E / 2);
  const float2 p = cadd(v[sa], v[sb]);
  float2 m = csub(v[sa], v[sb]);
  const float2 mr = mul_si<S>(m);
  m = h ? mr : m;
  float2 a = p;
  float2 b = tw<2 * E, K, S>(m);
  swap32(a, b);
  v[sa] = a;
  v[sb] = b;
}
template <int S, int E, int... K>
__device__ __forceinline__ void xlane_adj_all(float2* v, bool h, std::integer_sequence<int, K...>) {
  (xlane_adj_one<S, E, K>(v, h), ...);
}
template <int S, int E>
__device__ __forceinline__ void xlane_adj(float2* v, bool h) {
  xlane_adj_all<S, E>(v, h, std::make_integer_sequence<int, E / 2>{});
}

}  // namespace ptyg
