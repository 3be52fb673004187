// 256 x 256 patterns (the large one-GPU share: 8192^2 object, 256^2 probe).
//
// A 256^2 pattern (512 KiB) fits neither in LDS nor in one workgroup's
// registers, so its 2-D DFT is split by decimation in both axes into four
// 128^2 polyphase sub-transforms, Y_pq = DFT128(x[2u'+p][2v'+q]), p, q in
// {0, 1}, each run by the 128^2 register/LDS pipeline, followed by a
// pointwise 2x2 radix stage
//   X[a + 128 al][b + 128 be] = sum_pq (-1)^(al p + be q) W256^(a p + b q) Y_pq[a][b].
// The GRAD pass is three kernels sharing one per-pattern buffer U:
//   k_sub_fwd    gather (stride 2) * probe -> Y_pq (per sub-grid transposed)
//   k_combine    radix stage -> Poisson residual + objective (FP64) ->
//                adjoint radix stage (1/256 folded in) -> R_pq, in place
//   k_sub_inv    inverse sub-transforms -> u_pq, in place (polyphase layout)
// after which k_tile_sum / k_probe_partial form G^H with the polyphase
// index map.  A line-search trial is k_sub_fwd (psi + gamma eta) followed by
// the objective-only combine.  A GRAD pass runs its kernels chunk by chunk
// over the patterns (for_chunks below).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "pattern.hpp"
#include "pixel.hpp"

namespace ptyg {
namespace {

constexpr int NS = 128;                 // sub-transform size
constexpr int NB = 256;                 // pattern size
constexpr int SUB = NS * NS;            // elements per sub-grid
using G = Geo<NS>;

#define PTYG_SUB_KERNEL __launch_bounds__(G::WG) __attribute__((amdgpu_waves_per_eu(G::WAVES_PER_EU, G::WAVES_PER_EU)))

// W256^e, e in [0, 256)
__device__ __forceinline__ float2 w256(int e, int sign) {
  return make_float2(kTwCosDev[e & 255], sign * kTwSinDev[e & 255]);
}

// Gather the (p, q) sub-grid of (p + gamma dp) * (psi + gamma eta) patch k,
// or with LIN of the first-order direction term p * eta + dp * psi; with PS
// also the lane's FP64 patch sums ps[5] = (Re a b*, |b|^2, Re a c*,
// Re b c*, |c|^2) of a = p psi, b = p eta + dp psi, c = dp eta.
template <bool LINC_O, bool LINC_P, bool LIN = false, bool PS = false>
__device__ __forceinline__ void gather_sub(float2* v, const PatArgs& a, const Lane& L, int2 rc, int p, int q,
                                           double* ps = nullptr) {
  // slot m -> sub-row u' = 2m + h, sub-col v' = line -> patch (2u' + p, 2v' + q)
  const uint32_t lo = (L.h ? 2u * (uint32_t)a.W : 0u) + 2u * (uint32_t)L.line;
  const size_t corner = (size_t)(rc.x + p) * a.W + rc.y + q;
  if constexpr (LIN) {
    const uint32_t plo = (L.h ? 2u * NB : 0u) + 2u * (uint32_t)L.line;
    const float2* pb = a.probe + p * NB + q;
    const float2* dpb = a.dprobe + p * NB + q;
#pragma unroll
    for (int c = 0; c < G::E; c += 8) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = c; m < c + 8; ++m) {
        const size_t row = corner + (size_t)(4 * m) * a.W;
        const float2 o = (a.obj + row)[lo], e = (a.dobj + row)[lo];
        const float2 pr = (pb + 4 * m * NB)[plo], dp = (dpb + 4 * m * NB)[plo];
        const float2 bv = cadd(cmul(pr, e), cmul(dp, o));
        v[m] = bv;
        if constexpr (PS) {
          const float2 av = cmul(pr, o), cv = cmul(dp, e);
          ps[0] += (double)av.x * bv.x + (double)av.y * bv.y;
          ps[1] += (double)bv.x * bv.x + (double)bv.y * bv.y;
          ps[2] += (double)av.x * cv.x + (double)av.y * cv.y;
          ps[3] += (double)bv.x * cv.x + (double)bv.y * cv.y;
          ps[4] += (double)cv.x * cv.x + (double)cv.y * cv.y;
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    return;
  }
#pragma unroll
  for (int c = 0; c < G::E; c += 16) {
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = c; m < c + 16; ++m) {
      const size_t row = corner + (size_t)(4 * m) * a.W;
      float2 o = (a.obj + row)[lo];
      if constexpr (LINC_O) {
        const float2 e = (a.dobj + row)[lo];
        o = make_float2(fmaf(a.gamma, e.x, o.x), fmaf(a.gamma, e.y, o.y));
      }
      v[m] = o;
    }
  }
  const uint32_t plo = (L.h ? 2u * NB : 0u) + 2u * (uint32_t)L.line;
  const float2* pb = a.probe + p * NB + q;
  const float2* dpb = LINC_P ? a.dprobe + p * NB + q : nullptr;
#pragma unroll
  for (int c = 0; c < G::E; c += 8) {
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = c; m < c + 8; ++m) {
      float2 pr = (pb + 4 * m * NB)[plo];
      if constexpr (LINC_P) {
        const float2 dp = (dpb + 4 * m * NB)[plo];
        pr = make_float2(fmaf(a.gamma, dp.x, pr.x), fmaf(a.gamma, dp.y, pr.y));
      }
      v[m] = cmul(pr, v[m]);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

// U layout per pattern: [pq][b][a] for Y / R (transposed sub-grids, coalesced
// for the row layout), [pq][u'][v'] for u (natural sub-grids).
template <bool LINC_O, bool LINC_P, bool LIN = false, bool PS = false>
__global__ PTYG_SUB_KERNEL void k_sub_fwd(PatArgs a) {
  static_assert(!PS || LIN, "patch sums with the first-order term");
  __shared__ float2 lds[G::LDS_ELEMS];
  __shared__ double psred[PS ? 5 * (G::WG / 64) : 1];
  // workgroup b runs on XCD b % 8: the four sub-grids of a pattern (which
  // read the same cache lines of its patch, every other column each) go to
  // one XCD, consecutive patterns to consecutive XCDs
  const int g = blockIdx.x >> 5, r32 = blockIdx.x & 31;
  const int k = 8 * g + (r32 & 7), pq = r32 >> 3, p = pq >> 1, q = pq & 1;
  if (k >= a.K) return;  // the grid is 32 ceil(K / 8) blocks
  const int blk = 4 * k + pq;
  const Lane L = lane_info<NS>();
  const int2 rc = a.pos[k];
  float2 v[G::E];
  double ps[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  gather_sub<LINC_O, LINC_P, LIN, PS>(v, a, L, rc, p, q, ps);
  if constexpr (PS) {
    // block sums in a fixed order: lanes by shuffle, then the four waves
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) ps[i] += __shfl_xor(ps[i], off);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int i = 0; i < 5; ++i) psred[5 * (threadIdx.x >> 6) + i] = ps[i];
    __syncthreads();
    if (threadIdx.x < 8) {
      // row 0 (Re a b*, 0, |b|^2, 0), row 1 (Re a c*, Re b c*, |c|^2, 0)
      const int e = threadIdx.x & 3, r = threadIdx.x >> 2;
      const int si = r == 0 ? (e == 0 ? 0 : (e == 2 ? 1 : -1)) : (e == 3 ? -1 : 2 + e);
      double t = 0.0;
      if (si >= 0) {
#pragma unroll
        for (int w = 0; w < G::WG / 64; ++w) t += psred[5 * w + si];
      }
      a.ps_part[4 * ((r ? 4 * (size_t)a.ps_k : 0) + blk) + e] = t;
    }
  }
  fwd_line<NS>(v, L.h);
  transpose_c2r<NS>(v, lds, L);
  fwd_line<NS>(v, L.h);
  float2* y = a.ubuf + (size_t)k * NB * NB + (size_t)pq * SUB;
  const uint32_t lo = (L.h ? (uint32_t)(G::E / 2) * NS : 0u) + (uint32_t)L.line;
#pragma unroll
  for (int s = 0; s < G::E; ++s) (y + (size_t)kFreq<NS>.f[s] * NS)[lo] = v[s];
}

__global__ PTYG_SUB_KERNEL void k_sub_inv(PatArgs a) {
  __shared__ float2 lds[G::LDS_ELEMS];
  const int blk = blockIdx.x;
  const int k = blk >> 2, pq = blk & 3;
  if (k >= a.K) return;
  const Lane L = lane_info<NS>();
  float2 v[G::E];
  float2* y = a.ubuf + (size_t)k * NB * NB + (size_t)pq * SUB;
  const uint32_t lo = (L.h ? (uint32_t)(G::E / 2) * NS : 0u) + (uint32_t)L.line;
#pragma unroll
  for (int s = 0; s < G::E; ++s) v[s] = (y + (size_t)kFreq<NS>.f[s] * NS)[lo];
  inv_line<NS>(v, L.h);
  transpose_r2c<NS>(v, lds, L);
  inv_line<NS>(v, L.h);
  // every lane of the workgroup has read its R values (the transposes hold
  // barriers), so the sub-grid can be overwritten in place
  const uint32_t plo = (L.h ? (uint32_t)NS : 0u) + (uint32_t)L.line;
#pragma unroll
  for (int m = 0; m < G::E; ++m) (y + 2 * m * NS)[plo] = v[m];
}

// Compacted store of element e (a.cseg records, one per 32 elements of the
// per-pattern transposed far field): listed elements only, at the record's
// first index plus the listed elements before e in its segment.
__device__ __forceinline__ void store_listed(float2* out, uint2 r, size_t e, float2 v) {
  const uint32_t bit = (uint32_t)e & 31u;
  if ((r.x >> bit) & 1u) out[r.y + __popc(r.x & ((1u << bit) - 1u))] = v;
}

// Pointwise radix-2x2 stage.  Thread item i: a = i & 127, b = (i >> 7) & 127,
// k = i >> 14.  MODE 0: forward only (writes far, unitary).  MODE 1: GRAD
// (objective partials, residual adjoint written back as R).  MODE 2:
// objective only.  MODE 3: adjoint of a given far field (writes R).
// MODE 4 (test hook): MODE 1 with the far field taken from a.far (rows)
// instead of the forward radix stage; with a.gstore set the residual r is
// also written there (rows).
//
// The item loop is software-pipelined: an item's loads are issued before
// the previous item's stores (the wait for loaded data also waits for every
// older store), so a wave keeps one item's loads in flight while it stores.

// Element index of (A, B) in pattern k's far field / intensities.
template <DataLayout LAY>
__device__ __forceinline__ size_t far_index(int64_t k, int A, int B) {
  return (size_t)k * NB * NB + ((LAY == DataLayout::Transposed) ? (size_t)B * NB + A : (size_t)A * NB + B);
}

// Everything one item loads: the four sub-grid values (MODE 0-2) or given
// far-field values (MODE 3, 4), the intensities, the compacted-store records
// and the direction-sum operands, index j = al * 2 + be.
struct CombLoads {
  float2 y[4];
  float d[4];
  uint2 rec[4];
  float2 P[4], Q[4];
};

template <int MODE, DataLayout LAY>
__device__ __forceinline__ void comb_load(const PatArgs& a, int64_t i, CombLoads& L) {
  const int ai = (int)(i & 127), bi = (int)((i >> 7) & 127);
  const int64_t k = i >> 14;
  if constexpr (MODE == 3 || MODE == 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      L.y[j] = a.far[far_index<DataLayout::Rows>(k, ai + 128 * (j >> 1), bi + 128 * (j & 1))];
  } else {
    const float2* y = a.ubuf + (size_t)k * NB * NB + (size_t)bi * NS + ai;
#pragma unroll
    for (int j = 0; j < 4; ++j) L.y[j] = y[j * SUB];
  }
  if constexpr (MODE == 1 || MODE == 2 || MODE == 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j) L.d[j] = a.data[far_index<LAY>(k, ai + 128 * (j >> 1), bi + 128 * (j & 1))];
  }
  if constexpr (LAY == DataLayout::Transposed && (MODE == 0 || MODE == 1)) {
    if (MODE == 0 && a.zs_part) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const size_t e = far_index<LAY>(k, ai + 128 * (j >> 1), bi + 128 * (j & 1));
        L.P[j] = a.zs_p[e];
        if (a.zs_q) L.Q[j] = a.zs_q[e];
      }
    }
    if (a.cseg && (MODE == 0 || a.gstore)) {
#pragma unroll
      for (int j = 0; j < 4; ++j) L.rec[j] = a.cseg[far_index<LAY>(k, ai + 128 * (j >> 1), bi + 128 * (j & 1)) >> 5];
    }
  }
}

// One item's radix-stage work on its loaded operands (ly: sub-grid or given
// far-field values, ld: intensities, rec: compacted-store records, P / Q:
// direction-sum operands).  MODE 1, 3, 4 return the adjoint sub-grid values
// in ynew for the caller to store.
template <int MODE, DataLayout LAY, int EST, bool WF>
__device__ __forceinline__ void comb_item(const PatArgs& a, int ai, int bi, int64_t k, const float2* ly,
                                          const float* ld, const uint2* rec, const float2* P, const float2* Q,
                                          double& acc_phi, double& acc_f, double* z, float2* ynew) {
  const float inv = 1.0f / NB;
  float2 g[4];  // index al * 2 + be
  if constexpr (MODE == 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j) g[j] = ly[j];
  } else if constexpr (MODE != 3) {
    const float2 t00 = ly[0];
    const float2 t01 = cmul(w256(bi, -1), ly[1]);
    const float2 t10 = cmul(w256(ai, -1), ly[2]);
    const float2 t11 = cmul(w256(ai + bi, -1), ly[3]);
    const float2 s0 = cadd(t00, t10), s1 = csub(t00, t10);  // al = 0 / 1 over p
    const float2 e0 = cadd(t01, t11), e1 = csub(t01, t11);
    g[0] = cscale(cadd(s0, e0), inv);  // al 0 be 0
    g[1] = cscale(csub(s0, e0), inv);  // al 0 be 1
    g[2] = cscale(cadd(s1, e1), inv);  // al 1 be 0
    g[3] = cscale(csub(s1, e1), inv);  // al 1 be 1
  }
  if constexpr (MODE == 0) {
    // Rows: far [k][A][B]; Transposed: per pattern [B][A] (the order of
    // the transposed intensities, for the batched line search)
    if (LAY == DataLayout::Transposed && a.zs_part) {
      // sums Re(P conj y), Re(Q conj y), |y|^2
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float2 y = g[j];
        z[0] += (double)P[j].x * y.x + (double)P[j].y * y.y;
        if (a.zs_q) z[1] += (double)Q[j].x * y.x + (double)Q[j].y * y.y;
        z[2] += (double)y.x * y.x + (double)y.y * y.y;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const size_t e = far_index<LAY>(k, ai + 128 * (j >> 1), bi + 128 * (j & 1));
      if (LAY == DataLayout::Transposed && a.cseg) store_listed(a.far, rec[j], e, g[j]);
      else a.far[e] = g[j];
    }
    return;
  }
  float2 r[4];
  if constexpr (MODE == 3) {
#pragma unroll
    for (int j = 0; j < 4; ++j) r[j] = ly[j];
  } else {
    const bool cp = MODE == 1 && LAY == DataLayout::Transposed && a.gstore && a.cseg;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (MODE == 1 && LAY == DataLayout::Transposed) {
        if (a.gstore) {
          const size_t e = far_index<LAY>(k, ai + 128 * (j >> 1), bi + 128 * (j & 1));
          if (cp) store_listed(a.gstore, rec[j], e, g[j]);
          else a.gstore[e] = g[j];
        }
      }
      const float x = fmaf(g[j].x, g[j].x, g[j].y * g[j].y);
      // sum |G psi|^2 of the batched search: the FP32 x summed in FP64, the
      // form of the objective's zero-count terms and of the search pass
      if constexpr (MODE == 1 && LAY == DataLayout::Transposed)
        if (a.gstore) z[0] += (double)x;
      float phi, ft, fac;
      // F only where the caller reports it (the solver forms it from Phi)
      pixel_terms<WF, EST>(x, ld[j], a.eps, phi, ft, fac);
      acc_phi += (double)phi;
      if constexpr (WF) acc_f += (double)ft;
      r[j] = cscale(g[j], fac);
    }
    if constexpr (MODE == 4) {
      if (a.gstore) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          a.gstore[far_index<DataLayout::Rows>(k, ai + 128 * (j >> 1), bi + 128 * (j & 1))] = r[j];
      }
    }
  }
  if constexpr (MODE == 1 || MODE == 3 || MODE == 4) {
    // adjoint radix stage: R_pq = conj(W^(ap+bq)) sum (-1)^(al p + be q) r / 256
    const float2 s0 = cadd(r[0], r[2]), s1 = csub(r[0], r[2]);  // over al
    const float2 u0 = cadd(r[1], r[3]), u1 = csub(r[1], r[3]);
    const float2 r00 = cadd(s0, u0);        // p 0 q 0
    const float2 r01 = csub(s0, u0);        // p 0 q 1
    const float2 r10 = cadd(s1, u1);        // p 1 q 0
    const float2 r11 = csub(s1, u1);        // p 1 q 1
    ynew[0] = cscale(r00, inv);
    ynew[1] = cscale(cmul(w256(bi, +1), r01), inv);
    ynew[2] = cscale(cmul(w256(ai, +1), r10), inv);
    ynew[3] = cscale(cmul(w256(ai + bi, +1), r11), inv);
  }
}

template <int MODE, DataLayout LAY, int EST, bool WF>
__device__ __forceinline__ void comb_finish(const PatArgs& a, int64_t i, const CombLoads& L, double& acc_phi,
                                            double& acc_f, double* z) {
  const int ai = (int)(i & 127), bi = (int)((i >> 7) & 127);
  const int64_t k = i >> 14;
  float2 ynew[4];
  comb_item<MODE, LAY, EST, WF>(a, ai, bi, k, L.y, L.d, L.rec, L.P, L.Q, acc_phi, acc_f, z, ynew);
  if constexpr (MODE == 1 || MODE == 3 || MODE == 4) {
    float2* y = a.ubuf + (size_t)k * NB * NB + (size_t)bi * NS + ai;
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j * SUB] = ynew[j];
  }
}

// Transposed layout, MODE 0-2: two adjacent frequencies (a, a + 1) per
// thread, so the sub-grid values move as 16-byte and the intensities as
// 8-byte accesses.  Pair item i: a = 2 (i & 63), b = (i >> 6) & 127,
// k = i >> 13.
struct CombLoads2 {
  float4 y[4];
  float2 d[4];
  uint2 rec[4];  // (a, a + 1) share one 32-element record: a is even
  float4 P[4], Q[4];
};

template <int MODE>
__device__ __forceinline__ void comb_load2(const PatArgs& a, int64_t i, CombLoads2& L) {
  constexpr DataLayout T = DataLayout::Transposed;
  const int ai = 2 * (int)(i & 63), bi = (int)((i >> 6) & 127);
  const int64_t k = i >> 13;
  const float4* y = reinterpret_cast<const float4*>(a.ubuf + (size_t)k * NB * NB + (size_t)bi * NS + ai);
#pragma unroll
  for (int j = 0; j < 4; ++j) L.y[j] = y[j * (SUB / 2)];
  if constexpr (MODE == 1 || MODE == 2) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      L.d[j] = *reinterpret_cast<const float2*>(a.data + far_index<T>(k, ai + 128 * (j >> 1), bi + 128 * (j & 1)));
  }
  if constexpr (MODE == 0) {
    if (a.zs_part) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const size_t e = far_index<T>(k, ai + 128 * (j >> 1), bi + 128 * (j & 1));
        L.P[j] = *reinterpret_cast<const float4*>(a.zs_p + e);
        if (a.zs_q) L.Q[j] = *reinterpret_cast<const float4*>(a.zs_q + e);
      }
    }
  }
  if constexpr (MODE == 0 || MODE == 1) {
    if (a.cseg && (MODE == 0 || a.gstore)) {
#pragma unroll
      for (int j = 0; j < 4; ++j) L.rec[j] = a.cseg[far_index<T>(k, ai + 128 * (j >> 1), bi + 128 * (j & 1)) >> 5];
    }
  }
}

__device__ __forceinline__ float2 half_of(float4 v, int h) {
  return h ? make_float2(v.z, v.w) : make_float2(v.x, v.y);
}

template <int MODE, int EST, bool WF>
__device__ __forceinline__ void comb_finish2(const PatArgs& a, int64_t i, const CombLoads2& L, double& acc_phi,
                                             double& acc_f, double* z) {
  const int ai = 2 * (int)(i & 63), bi = (int)((i >> 6) & 127);
  const int64_t k = i >> 13;
  float2 yn[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float2 ly[4], P[4], Q[4];
    float ld[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      ly[j] = half_of(L.y[j], h);
      // operands a mode does not load are not read
      ld[j] = (MODE == 1 || MODE == 2) ? (h ? L.d[j].y : L.d[j].x) : 0.0f;
      P[j] = (MODE == 0 && a.zs_part) ? half_of(L.P[j], h) : make_float2(0.f, 0.f);
      Q[j] = (MODE == 0 && a.zs_part && a.zs_q) ? half_of(L.Q[j], h) : make_float2(0.f, 0.f);
    }
    comb_item<MODE, DataLayout::Transposed, EST, WF>(a, ai + h, bi, k, ly, ld, L.rec, P, Q, acc_phi, acc_f, z,
                                                     yn[h]);
  }
  if constexpr (MODE == 1) {
    float4* y = reinterpret_cast<float4*>(a.ubuf + (size_t)k * NB * NB + (size_t)bi * NS + ai);
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j * (SUB / 2)] = make_float4(yn[0][j].x, yn[0][j].y, yn[1][j].x, yn[1][j].y);
  }
}

template <int MODE, DataLayout LAY, int EST = 0, bool WF = false>
__global__ __launch_bounds__(256) void k_combine(PatArgs a, int64_t items) {
  static_assert(MODE != 4 || LAY == DataLayout::Rows, "given far field: row layout");
  constexpr bool RES = MODE == 1 || MODE == 4;
  __shared__ double red[16];
  double acc_phi = 0.0, acc_f = 0.0;
  double z[4] = {0.0, 0.0, 0.0, 0.0};  // with a.zs_part: MODE 0 direction sums, MODE 1 sum |G psi|^2
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if constexpr (LAY == DataLayout::Transposed && MODE <= 2) {
    const int64_t pairs = items >> 1;  // items = K * SUB is even
    CombLoads2 cur;
    if (i < pairs) comb_load2<MODE>(a, i, cur);
    for (; i < pairs; i += stride) {
      CombLoads2 nxt;
      if (i + stride < pairs) comb_load2<MODE>(a, i + stride, nxt);
      comb_finish2<MODE, EST, WF>(a, i, cur, acc_phi, acc_f, z);
      cur = nxt;
    }
  } else {
    CombLoads cur;
    if (i < items) comb_load<MODE, LAY>(a, i, cur);
    for (; i < items; i += stride) {
      CombLoads nxt;
      if (i + stride < items) comb_load<MODE, LAY>(a, i + stride, nxt);
      comb_finish<MODE, LAY, EST, WF>(a, i, cur, acc_phi, acc_f, z);
      cur = nxt;
    }
  }
  if constexpr ((MODE == 0 || MODE == 1) && LAY == DataLayout::Transposed) {
    if (a.zs_part && (MODE == 0 || a.gstore)) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) z[i] += __shfl_xor(z[i], off);
      if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[4 * (threadIdx.x >> 6) + i] = z[i];
      __syncthreads();
      const double t = (threadIdx.x < 4) ? red[threadIdx.x] + red[4 + threadIdx.x] + red[8 + threadIdx.x] +
                                                 red[12 + threadIdx.x]
                                           : 0.0;
      if (MODE == 0 && threadIdx.x < 4) a.zs_part[4 * blockIdx.x + threadIdx.x] = t;
      if (MODE == 1 && threadIdx.x == 0) a.zs_part[blockIdx.x] = t;
      __syncthreads();  // red is reused by the objective reduction below
    }
  }
  if constexpr (RES || MODE == 2) {
    asm volatile("" : "+v"(acc_phi), "+v"(acc_f));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      acc_phi += __shfl_xor(acc_phi, off);
      acc_f += __shfl_xor(acc_f, off);
    }
    if ((threadIdx.x & 63) == 0) {
      red[2 * (threadIdx.x >> 6)] = acc_phi;
      red[2 * (threadIdx.x >> 6) + 1] = acc_f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      a.partials[2 * blockIdx.x] = red[0] + red[2] + red[4] + red[6];
      a.partials[2 * blockIdx.x + 1] = red[1] + red[3] + red[5] + red[7];
    }
  }
}

// Staged chunks: a GRAD pass (three kernels, two of which read back what
// the previous one left in U) runs chunk by chunk over the patterns
// (sub-transforms, radix stage and inverse sub-transforms of kChunk256
// patterns, then the next chunk), so the 512 KiB per pattern staged in U is
// read back while the memory-side cache still holds it instead of after a
// whole 8 GiB pass.  A forward-only pass reads U back once; there the tail
// of every chunk's launches costs more than the cache saves, so it runs as
// one chunk.
constexpr int kChunk256 = 512;
constexpr int kChunkCombineBlocks = 2048;  // radix-stage workgroups per GRAD chunk
constexpr int kCombineBlocks = 8192;       // radix-stage workgroups of a one-chunk pass

int combine_blocks(int K, int cap) {
  const int64_t items = (int64_t)K * SUB;
  const int64_t nb = (items + 255) / 256;
  return (int)(nb < cap ? nb : cap);
}

int pass_blocks(int K, int chunk, int cap) {
  int t = 0;
  for (int k0 = 0; k0 < K; k0 += chunk) t += combine_blocks(K - k0 < chunk ? K - k0 : chunk, cap);
  return t;
}

// The arguments of one chunk [k0, k0 + kn): per-pattern arrays offset to
// pattern k0 (compacted stores keep their whole-array indices: their
// records are offset instead), per-workgroup rows after the `before` rows
// of the earlier chunks (zs_width doubles per row).
PatArgs chunk_of(const PatArgs& a, int k0, int kn, int before, int zs_width) {
  PatArgs c = a;
  const size_t off = (size_t)k0 * NB * NB;
  c.K = kn;
  c.ps_k = a.K;
  c.pos = a.pos + k0;
  c.ubuf = a.ubuf + off;
  if (a.data) c.data = a.data + off;
  if (a.far && !a.cseg) c.far = a.far + off;
  if (a.gstore && !a.cseg) c.gstore = a.gstore + off;
  if (a.cseg) c.cseg = a.cseg + off / 32;
  if (a.zs_p) c.zs_p = a.zs_p + off;
  if (a.zs_q) c.zs_q = a.zs_q + off;
  if (a.partials) c.partials = a.partials + 2 * (size_t)before;
  if (a.zs_part) c.zs_part = a.zs_part + (size_t)zs_width * before;
  if (a.ps_part) c.ps_part = a.ps_part + 16 * (size_t)k0;
  return c;
}

// Runs f(chunk arguments) over chunks of `chunk` patterns in ascending
// order; each chunk's radix stage takes combine_blocks(kn, cap) workgroups.
template <typename F>
hipError_t for_chunks(const PatArgs& a, int chunk, int cap, int zs_width, F&& f) {
  int before = 0;
  for (int k0 = 0; k0 < a.K; k0 += chunk) {
    const int kn = a.K - k0 < chunk ? a.K - k0 : chunk;
    if (hipError_t e = f(chunk_of(a, k0, kn, before, zs_width))) return e;
    before += combine_blocks(kn, cap);
  }
  return hipSuccess;
}

template <int MODE>
hipError_t combine(const PatArgs& a, DataLayout lay, int cap, hipStream_t s) {
  const int nb = combine_blocks(a.K, cap);
  const int64_t items = (int64_t)a.K * SUB;
  // the estimator only enters the modes with objective terms
  constexpr bool OBJ = MODE == 1 || MODE == 2 || MODE == 4;
  const int est = OBJ ? a.est : 0;
  return dispatch_est(est, [&](auto ec) {
    constexpr int E = OBJ ? decltype(ec)::value : 0;
    const bool wf = OBJ && a.want_f;
    auto go = [&](auto wc) {
      constexpr bool WF = OBJ && decltype(wc)::value;
      if constexpr (MODE == 4) {
        if (lay != DataLayout::Rows) return hipErrorInvalidValue;
      } else if (lay == DataLayout::Transposed) {
        hipLaunchKernelGGL((k_combine<MODE, DataLayout::Transposed, E, WF>), dim3(nb), dim3(256), 0, s, a, items);
        return hipGetLastError();
      }
      hipLaunchKernelGGL((k_combine<MODE, DataLayout::Rows, E, WF>), dim3(nb), dim3(256), 0, s, a, items);
      return hipGetLastError();
    };
    return wf ? go(std::integral_constant<bool, true>{}) : go(std::integral_constant<bool, false>{});
  });
}

// k_sub_fwd's grid: four workgroups per pattern, in groups of eight patterns
dim3 sub_fwd_grid(int K) { return dim3(32 * ((K + 7) / 8)); }

hipError_t sub_fwd(const PatArgs& a, hipStream_t s) {
  const dim3 g = sub_fwd_grid(a.K), b(G::WG);
  const bool lo = a.dobj != nullptr, lp = a.dprobe != nullptr;
  if (lo && lp) hipLaunchKernelGGL((k_sub_fwd<true, true>), g, b, 0, s, a);
  else if (lo) hipLaunchKernelGGL((k_sub_fwd<true, false>), g, b, 0, s, a);
  else if (lp) hipLaunchKernelGGL((k_sub_fwd<false, true>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_sub_fwd<false, false>), g, b, 0, s, a);
  return hipGetLastError();
}

hipError_t sub_inv(const PatArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_inv, dim3(4 * a.K), dim3(G::WG), 0, s, a);
  return hipGetLastError();
}

}  // namespace

// Every 256^2 launcher stages through a.ubuf (and the forward writes
// a.far): refuse null buffers on the host instead of launching.
bool staged_ok(const PatArgs& a) { return a.ubuf != nullptr && a.pos != nullptr; }

hipError_t launch_forward256(const PatArgs& a, hipStream_t s) {
  if (!staged_ok(a) || !a.far || !a.obj || !a.probe) return hipErrorInvalidValue;
  PatArgs b = a;
  b.dobj = nullptr;
  b.dprobe = nullptr;
  b.ps_k = a.K;
  if (hipError_t e = sub_fwd(b, s)) return e;
  return combine<0>(b, DataLayout::Rows, kCombineBlocks, s);
}

hipError_t launch_adjoint256(const PatArgs& a, hipStream_t s) {
  if (!staged_ok(a) || !a.far) return hipErrorInvalidValue;
  if (hipError_t e = combine<3>(a, DataLayout::Rows, kCombineBlocks, s)) return e;
  return sub_inv(a, s);
}

int grad256_blocks(int K) { return pass_blocks(K, kChunk256, kChunkCombineBlocks); }

hipError_t launch_grad256(const PatArgs& a, DataLayout lay, int* blocks_out, hipStream_t s) {
  if (!staged_ok(a) || !a.data || !a.partials || !a.obj || !a.probe) return hipErrorInvalidValue;
  PatArgs b = a;
  b.dobj = nullptr;
  b.dprobe = nullptr;
  if (blocks_out) *blocks_out = grad256_blocks(a.K);
  return for_chunks(b, kChunk256, kChunkCombineBlocks, 1, [&](const PatArgs& c) {
    if (hipError_t e = sub_fwd(c, s)) return e;
    if (hipError_t e = combine<1>(c, lay, kChunkCombineBlocks, s)) return e;
    return sub_inv(c, s);
  });
}

hipError_t launch_grad_far256(const PatArgs& a, int* blocks_out, hipStream_t s) {
  if (!staged_ok(a) || !a.far || !a.data || !a.partials) return hipErrorInvalidValue;
  if (blocks_out) *blocks_out = grad256_blocks(a.K);
  return for_chunks(a, kChunk256, kChunkCombineBlocks, 0, [&](const PatArgs& c) {
    if (hipError_t e = combine<4>(c, DataLayout::Rows, kChunkCombineBlocks, s)) return e;
    return sub_inv(c, s);
  });
}

int fwd_t256_blocks(int K) { return combine_blocks(K, kCombineBlocks); }

hipError_t launch_fwd_t256(const PatArgs& a, bool lin, hipStream_t s) {
  if (!staged_ok(a) || !a.far || !a.obj || !a.probe) return hipErrorInvalidValue;
  if (lin && (!a.dobj || !a.dprobe)) return hipErrorInvalidValue;
  PatArgs b = a;
  b.ps_k = a.K;
  const dim3 g = sub_fwd_grid(b.K), bl(G::WG);
  if (lin && b.ps_part) hipLaunchKernelGGL((k_sub_fwd<false, false, true, true>), g, bl, 0, s, b);
  else if (lin) hipLaunchKernelGGL((k_sub_fwd<false, false, true>), g, bl, 0, s, b);
  else hipLaunchKernelGGL((k_sub_fwd<false, false>), g, bl, 0, s, b);
  if (hipError_t e = hipGetLastError()) return e;
  return combine<0>(b, DataLayout::Transposed, kCombineBlocks, s);
}

hipError_t launch_minfunc256(const PatArgs& a, DataLayout lay, int* blocks_out, hipStream_t s) {
  if (!staged_ok(a) || !a.data || !a.partials || !a.obj || !a.probe) return hipErrorInvalidValue;
  if (blocks_out) *blocks_out = combine_blocks(a.K, kCombineBlocks);
  if (hipError_t e = sub_fwd(a, s)) return e;
  return combine<2>(a, lay, kCombineBlocks, s);
}

}  // namespace ptyg
