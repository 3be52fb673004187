// HIP kernels for gfx950: the ML-CG ptychography hot path.
//
//   forward  (Eq. fwd_model)    g_k = F (p * psi[s_k])
//   adjoint  (text after Eq. gradient) G^H = Q^H F^H with scatter-add
//   grad     (Eq. gradient, GRAD stage of Algorithm 1) fused:
//            gather -> *p -> F -> residual + objective terms -> F^H -> *conj p
//            -> scatter-add (+ probe gradient terms in joint mode)
//   minfunc  (MINFUNC of Algorithm 1, a line-search trial of Eq. linesearch)
//            gather (psi + gamma eta) -> *(p + gamma eta_p) -> F -> objective
//   vector kernels for the DIR and Update stages (Eqs. DaiYuan, update).
//
// F is the unitary 2-D DFT (1/N per transform), DC at [0][0].  Transform
// arithmetic is FP32; objective terms are accumulated per thread in FP64 and
// reduced deterministically (fixed workgroup -> pattern mapping, fixed
// reduction trees).  The object gradient is an ordered overlap sum of the
// per-pattern back-propagated waves (no atomics): results are bit-reproducible.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "pattern.hpp"
#include "pixel.hpp"

namespace ptyg {

namespace {

// Pattern kernels: the LDS transpose buffer allows Geo<N>::WAVES_PER_EU waves
// per SIMD; asking the register allocator for exactly that occupancy keeps
// the scheduler from hoisting every gather load at once.
#define PTYG_PATTERN_KERNEL(N) \
  __launch_bounds__(Geo<N>::WG) __attribute__((amdgpu_waves_per_eu(Geo<N>::WAVES_PER_EU, Geo<N>::WAVES_PER_EU)))

// Block-wide sum of two doubles; the result is valid in thread 0.
template <int WG>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
    red[2 * w] = a;
    red[2 * w + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0.0;
    b = 0.0;
#pragma unroll
    for (int i = 0; i < WG / 64; ++i) {
      a += red[2 * i];
      b += red[2 * i + 1];
    }
  }
}

// Block-wide sums of four doubles written to out[0..3] by thread 0.
template <int WG>
__device__ __forceinline__ void block_sum4_store(double (&v)[4], double* red, double* out) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0)
#pragma unroll
    for (int i = 0; i < 4; ++i) red[4 * w + i] = v[i];
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < WG / 64; ++i) t += red[4 * i + threadIdx.x];
    out[threadIdx.x] = t;
  }
}

// Addressing: every global access is written as a pointer that is uniform
// across the wave (computed from the pattern index and a compile-time slot
// offset) plus a 32-bit lane offset, so the loads use the scalar-base form
// and the 64 slots share one offset register.
template <int N>
__device__ __forceinline__ uint32_t lane_off(const Lane& L, uint32_t stride) {
  return (L.h ? stride : 0u) + (uint32_t)L.line;
}

// Intensity at (row arow = lane line, frequency column slot s).
template <int N, DataLayout LAY>
__device__ __forceinline__ float load_data(const float* data, int k, const Lane& L, int s) {
  constexpr int f = 0;
  (void)f;
  const float* dk = data + (size_t)k * N * N;
  if constexpr (LAY == DataLayout::Transposed) {
    // element (a, b) at b*N + a; b = kFreq[s] + (E/2) h, a = line
    return (dk + (size_t)kFreq<N>.f[s] * N)[lane_off<N>(L, (Geo<N>::E / 2) * N)];
  } else {
    return (dk + kFreq<N>.f[s])[(uint32_t)L.line * N + (L.h ? Geo<N>::E / 2 : 0)];
  }
}

// Gather p * psi patch (optionally (p + g eta_p) * (psi + g eta_psi)) into
// column-layout spatial slots.  The object loads go straight into the data
// registers (all in flight at once); the probe and direction loads follow in
// chunks fenced from the scheduler so that their results never occupy more
// than a few registers.
constexpr int kChunk = 8;
constexpr int kResChunk = 4;  // residual: many temporaries per pixel

template <int N, bool LINC_O, bool LINC_P>
__device__ __forceinline__ void gather_exit_wave(float2* v, const PatArgs& a, const Lane& L, int2 rc,
                                                 bool valid) {
  using G = Geo<N>;
  constexpr int T = G::TPC;
  const uint32_t lo = lane_off<N>(L, (uint32_t)a.W);
  const size_t corner = (size_t)rc.x * a.W + rc.y;
  if constexpr (!LINC_O) {
#pragma unroll
    for (int m = 0; m < G::E; ++m) v[m] = (a.obj + corner + (size_t)(m * T) * a.W)[lo];
  } else {
#pragma unroll
    for (int c = 0; c < G::E; c += 2 * kChunk) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = c; m < c + 2 * kChunk; ++m) {
        const size_t row = corner + (size_t)(m * T) * a.W;
        const float2 o = (a.obj + row)[lo], e = (a.dobj + row)[lo];
        v[m] = make_float2(fmaf(a.gamma, e.x, o.x), fmaf(a.gamma, e.y, o.y));
      }
    }
  }
  // probe (and probe direction) values one chunk ahead of their multiplies
  const uint32_t plo = lane_off<N>(L, N);
  constexpr int DP = LINC_P ? kChunk : 1;
  float2 pn[kChunk], dn[DP];
#pragma unroll
  for (int j = 0; j < kChunk; ++j) {
    pn[j] = (a.probe + j * T * N)[plo];
    if constexpr (LINC_P) dn[j] = (a.dprobe + j * T * N)[plo];
  }
#pragma unroll
  for (int c = 0; c < G::E; c += kChunk) {
    __builtin_amdgcn_sched_barrier(0);
    float2 pc[kChunk], dc[DP];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      pc[j] = pn[j];
      if constexpr (LINC_P) dc[j] = dn[j];
    }
    if (c + kChunk < G::E) {
#pragma unroll
      for (int j = 0; j < kChunk; ++j) {
        pn[j] = (a.probe + (c + kChunk + j) * T * N)[plo];
        if constexpr (LINC_P) dn[j] = (a.dprobe + (c + kChunk + j) * T * N)[plo];
      }
    }
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      float2 p = pc[j];
      if constexpr (LINC_P) p = make_float2(fmaf(a.gamma, dc[j].x, p.x), fmaf(a.gamma, dc[j].y, p.y));
      if (!valid) p = make_float2(0.f, 0.f);
      v[c + j] = cmul(p, v[c + j]);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

// Store the back-propagated wave u_k (column layout, spatial slots) of
// every pattern, or conj(p) u_k when only the object adjoint is wanted; the
// overlap sum follows in k_tile_sum (which then needs no probe), the probe
// adjoint in k_probe_partial (from the plain u_k).  A load issued after a
// store waits for it, so the probe comes in a few large chunks.
constexpr int kStoreChunk = 32;

template <int N>
__device__ __forceinline__ void store_u(const float2* v, const PatArgs& a, const Lane& L, int k, bool valid) {
  using G = Geo<N>;
  constexpr int T = G::TPC;
  constexpr int C = G::E < kStoreChunk ? G::E : kStoreChunk;
  if (!valid) return;
  const uint32_t plo = lane_off<N>(L, N);
  float2* uk = a.ubuf + (size_t)k * N * N;
  if (a.premul) {
#pragma unroll
    for (int c = 0; c < G::E; c += C) {
      __builtin_amdgcn_sched_barrier(0);
      float2 p[C];
#pragma unroll
      for (int m = c; m < c + C; ++m) p[m - c] = (a.probe + m * T * N)[plo];
#pragma unroll
      for (int m = c; m < c + C; ++m) (uk + m * T * N)[plo] = cmulc(p[m - c], v[m]);
    }
    __builtin_amdgcn_sched_barrier(0);
  } else {
#pragma unroll
    for (int m = 0; m < G::E; ++m) (uk + m * T * N)[plo] = v[m];
  }
}

// Pattern handled by this lane.  Lanes past the last pattern (only possible
// when several patterns share a workgroup) read pattern 0 so that every load
// stays in bounds, and their contributions are masked.  Returns false when
// the whole workgroup has no pattern (it then writes zero partials and exits
// before any barrier).
template <int N>
__device__ __forceinline__ bool pattern_of(const PatArgs& a, const Lane& L, int& k, bool& valid, int2& rc) {
  const int groups = (a.K + Geo<N>::PPW - 1) / Geo<N>::PPW;
  const int g = group_of_block(blockIdx.x, groups);
  if (g < 0) return false;
  k = g * Geo<N>::PPW + L.pslot;
  valid = k < a.K;
  if (!valid) k = 0;
  rc = a.pos[k];
  return true;
}

__device__ __forceinline__ void write_zero_partials(const PatArgs& a) {
  if (threadIdx.x == 0 && a.partials) {
    a.partials[2 * blockIdx.x] = 0.0;
    a.partials[2 * blockIdx.x + 1] = 0.0;
  }
}

// ----------------------------------------------------------------- kernels
template <int N>
__global__ PTYG_PATTERN_KERNEL(N) void k_forward(PatArgs a) {
  using G = Geo<N>;
  __shared__ float2 lds[G::LDS_ELEMS];
  const Lane L = lane_info<N>();
  int k;
  bool valid;
  int2 rc;
  if (!pattern_of<N>(a, L, k, valid, rc)) {
    write_zero_partials(a);
    return;
  }
  float2 v[G::E];
  gather_exit_wave<N, false, false>(v, a, L, rc, valid);
  fwd_line<N>(v, L.h);
  transpose_c2r<N>(v, lds, L);
  fwd_line<N>(v, L.h);
  if (!valid) return;
  const float invN = 1.0f / N;
#pragma unroll
  for (int s = 0; s < G::E; ++s) {
    const int b = fidx<N>(s, L.h);
    (a.far + (size_t)k * N * N + kFreq<N>.f[s])[(uint32_t)L.line * N + (L.h ? G::E / 2 : 0)] = cscale(v[s], invN);
  }
}

template <int N>
__global__ PTYG_PATTERN_KERNEL(N) void k_adjoint(PatArgs a) {
  using G = Geo<N>;
  __shared__ float2 lds[G::LDS_ELEMS];
  const Lane L = lane_info<N>();
  int k;
  bool valid;
  int2 rc;
  if (!pattern_of<N>(a, L, k, valid, rc)) {
    write_zero_partials(a);
    return;
  }
  float2 v[G::E];
  const float invN = 1.0f / N;
#pragma unroll
  for (int s = 0; s < G::E; ++s) {
    const int b = fidx<N>(s, L.h);
    v[s] = cscale((a.far + (size_t)k * N * N + kFreq<N>.f[s])[(uint32_t)L.line * N + (L.h ? G::E / 2 : 0)],
                  valid ? invN : 0.0f);
  }
  inv_line<N>(v, L.h);
  transpose_r2c<N>(v, lds, L);
  inv_line<N>(v, L.h);
  store_u<N>(v, a, L, k, valid);
}

// Exit-wave direction p * eta + dp * psi (first-order term of the joint
// trial (p + g dp)(psi + g eta)), column-layout spatial slots: the p * eta
// gather, then dp * psi added in chunks.
template <int N>
__device__ __forceinline__ void gather_lin(float2* v, const PatArgs& a, const Lane& L, int2 rc, bool valid) {
  using G = Geo<N>;
  constexpr int T = G::TPC;
  PatArgs b = a;
  b.obj = a.dobj;
  gather_exit_wave<N, false, false>(v, b, L, rc, valid);
  const uint32_t lo = lane_off<N>(L, (uint32_t)a.W);
  const uint32_t plo = lane_off<N>(L, N);
  const size_t corner = (size_t)rc.x * a.W + rc.y;
#pragma unroll
  for (int c = 0; c < G::E; c += kChunk) {
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = c; m < c + kChunk; ++m) {
      const float2 o = (a.obj + corner + (size_t)(m * T) * a.W)[lo];
      float2 dp = (a.dprobe + m * T * N)[plo];
      if (!valid) dp = make_float2(0.f, 0.f);
      v[m] = cadd(v[m], cmul(dp, o));
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

// Compacted far-field stores (n = 128): the pattern's segment records are
// staged in LDS at kernel start (ordered before their first use by the
// barrier of the first transpose); the lane's element of slot s, row
// f = kFreq[s] + (E/2) h and column `line`, lies in segment 4 f + line / 32.
constexpr int kSegPerPattern = 128 * 128 / 32;

__device__ __forceinline__ void stage_segments(uint2* srec, const PatArgs& a, int k) {
  const uint2* src = a.cseg + (size_t)k * kSegPerPattern;
  for (int i = threadIdx.x; i < kSegPerPattern; i += 256) srec[i] = src[i];
}

__device__ __forceinline__ void store_compact(float2* out, const uint2* srec, const Lane& L, int f, float2 v) {
  const uint2 r = srec[f * 4 + (L.line >> 5)];
  const uint32_t bit = (uint32_t)L.line & 31u;
  if ((r.x >> bit) & 1u) out[r.y + __popc(r.x & ((1u << bit) - 1u))] = v;
}

// Forward transform of a direction, stored per pattern transposed (the
// element order of the transposed intensities and of the stored G psi).
// ZS: also the sums over this workgroup's elements of Re(P conj y),
// Re(Q conj y) (Q nullable) and |y|^2 (P = a.zs_p, Q = a.zs_q stored far
// fields, y = the result).  They are formed before any store: loads wait on
// every earlier memory operation, stores included.
// CP (n = 128, no sums): only the listed elements, compacted (a.cseg).
template <int N, bool LIN, int ZS, bool CP = false>
__global__ PTYG_PATTERN_KERNEL(N) void k_fwd_t(PatArgs a) {
  using G = Geo<N>;
  static_assert(!CP || (N == 128 && ZS == 0), "compacted stores: n = 128 without sums");
  __shared__ float2 lds[G::LDS_ELEMS];
  __shared__ double red[4 * (G::WG / 64)];
  __shared__ uint2 srec[CP ? kSegPerPattern : 1];
  const Lane L = lane_info<N>();
  int k;
  bool valid;
  int2 rc;
  if (!pattern_of<N>(a, L, k, valid, rc)) {
    if (ZS > 0 && threadIdx.x < 4) a.zs_part[4 * blockIdx.x + threadIdx.x] = 0.0;
    return;
  }
  if constexpr (CP) stage_segments(srec, a, k);
  float2 v[G::E];
  if constexpr (LIN) gather_lin<N>(v, a, L, rc, valid);
  else gather_exit_wave<N, false, false>(v, a, L, rc, valid);
  fwd_line<N>(v, L.h);
  transpose_c2r<N>(v, lds, L);
  fwd_line<N>(v, L.h);
  const float invN = 1.0f / N;
  const size_t kb = (size_t)k * N * N;
  const uint32_t lo = lane_off<N>(L, (G::E / 2) * N);
#pragma unroll
  for (int s = 0; s < G::E; ++s) v[s] = cscale(v[s], invN);
  if constexpr (ZS > 0) {
    // lanes of a missing pattern hold y = 0 (zero probe): no masking needed
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    constexpr int CH = ZS == 1 ? 8 : 4;
#pragma unroll
    for (int c = 0; c < G::E; c += CH) {
      __builtin_amdgcn_sched_barrier(0);
      float2 P[CH], Q[CH];
#pragma unroll
      for (int s = c; s < c + CH; ++s) {
        const size_t off = kb + (size_t)kFreq<N>.f[s] * N;
        P[s - c] = (a.zs_p + off)[lo];
        if constexpr (ZS == 2) Q[s - c] = (a.zs_q + off)[lo];
      }
#pragma unroll
      for (int s = c; s < c + CH; ++s) {
        const float2 y = v[s];
        z[0] += (double)P[s - c].x * y.x + (double)P[s - c].y * y.y;
        if constexpr (ZS == 2) z[1] += (double)Q[s - c].x * y.x + (double)Q[s - c].y * y.y;
        z[2] += (double)y.x * y.x + (double)y.y * y.y;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    block_sum4_store<G::WG>(z, red, a.zs_part + 4 * blockIdx.x);
  }
  if constexpr (CP) {
#pragma unroll
    for (int s = 0; s < G::E; ++s) store_compact(a.far, srec, L, fidx<N>(s, L.h), v[s]);
  } else if (G::PPW == 1 || valid) {
#pragma unroll
    for (int s = 0; s < G::E; ++s) (a.far + kb + (size_t)kFreq<N>.f[s] * N)[lo] = v[s];
  }
}

// FARIN (test hook): the far field g = G psi is given in a.far (row layout)
// instead of being formed; everything after it -- residual and objective
// terms, inverse transform, stored waves -- is the same code as GRAD's.
// With a.gstore set it also writes the residual r (row layout).
template <int N, DataLayout LAY, bool SG, int EST, bool CP = false, bool FARIN = false, bool WF = true>
__global__ PTYG_PATTERN_KERNEL(N) void k_grad(PatArgs a) {
  using G = Geo<N>;
  static_assert(!CP || (N == 128 && SG), "compacted stores: n = 128 with the G psi store");
  static_assert(!FARIN || (!SG && LAY == DataLayout::Rows), "given far field: row layout, no G psi store");
  __shared__ float2 lds[G::LDS_ELEMS];
  __shared__ double red[2 * (G::WG / 64)];
  __shared__ uint2 srec[CP ? kSegPerPattern : 1];
  const Lane L = lane_info<N>();
  int k;
  bool valid;
  int2 rc;
  if (!pattern_of<N>(a, L, k, valid, rc)) {
    write_zero_partials(a);
    if (SG && threadIdx.x == 0) a.zs_part[blockIdx.x] = 0.0;
    return;
  }
  if constexpr (CP) stage_segments(srec, a, k);
  float2 v[G::E];
  if constexpr (FARIN) {
    // v = N g: the 1/N scaling below gives g back exactly (N a power of 2)
#pragma unroll
    for (int s = 0; s < G::E; ++s)
      v[s] = cscale((a.far + (size_t)k * N * N + kFreq<N>.f[s])[(uint32_t)L.line * N + (L.h ? G::E / 2 : 0)],
                    valid ? (float)N : 0.0f);
  } else {
    gather_exit_wave<N, false, false>(v, a, L, rc, valid);
    fwd_line<N>(v, L.h);
    transpose_c2r<N>(v, lds, L);
    fwd_line<N>(v, L.h);
  }
  const float invN = 1.0f / N;
  double acc_phi = 0.0, acc_f = 0.0, acc_aa = 0.0;
  // intensities PF chunks ahead: chunk c + PF's loads are issued before
  // chunk c's arithmetic, so their latency overlaps it.  With the G psi
  // stores, the first PF chunks go out before the stores, and a load issued
  // after them waits for every store (one in-order counter for loads and
  // stores): four chunks ahead, that wait comes four chunks of arithmetic
  // after the stores (the solver's GRAD 398 -> 387 us at 2048^2 / 4096
  // patterns, 246 VGPRs; six chunks spill)
  constexpr int PF = SG ? 4 : 1;
  float dn[PF][kResChunk];
#pragma unroll
  for (int q = 0; q < PF; ++q)
#pragma unroll
    for (int j = 0; j < kResChunk; ++j) dn[q][j] = load_data<N, LAY>(a.data, k, L, kOrd<N>.s[q * kResChunk + j]);
  if constexpr (SG) {
    // G psi for the batched line search, in the element order of the
    // transposed intensities (sum |G psi|^2 below).  All stores go out
    // together: stores between the residual loop's loads would each add a
    // wait, and doing them inside that loop spills.  (Lanes of a missing
    // pattern hold 0: zero probe.)
    const uint32_t lo = lane_off<N>(L, (G::E / 2) * N);
    float2* gk = a.gstore + (size_t)k * N * N;
#pragma unroll
    for (int s = 0; s < G::E; ++s) {
      if (s % 8 == 0) __builtin_amdgcn_sched_barrier(0);
      v[s] = cscale(v[s], invN);  // scaled in place: v now holds G psi
      if constexpr (CP) store_compact(a.gstore, srec, L, fidx<N>(s, L.h), v[s]);
      else if (G::PPW == 1 || valid) (gk + (size_t)kFreq<N>.f[s] * N)[lo] = v[s];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  // Eq. ML's F only where the caller reports it; the solver forms it from
  // Phi and the data constant
  constexpr bool WANT_F = WF;
#pragma unroll
  for (int c = 0; c < G::E; c += kResChunk) {
    __builtin_amdgcn_sched_barrier(0);
    const int q = (c / kResChunk) % PF;  // a constant once the loop is unrolled
    float dc[kResChunk];
#pragma unroll
    for (int j = 0; j < kResChunk; ++j) dc[j] = dn[q][j];
    if (c + PF * kResChunk < G::E) {
#pragma unroll
      for (int j = 0; j < kResChunk; ++j) dn[q][j] = load_data<N, LAY>(a.data, k, L, kOrd<N>.s[c + PF * kResChunk + j]);
    }
#pragma unroll
    for (int j = 0; j < kResChunk; ++j) {
      const int s = kOrd<N>.s[c + j];
      const float2 g = SG ? v[s] : cscale(v[s], invN);
      const float x = fmaf(g.x, g.x, g.y * g.y);
      // sum |G psi|^2 of the batched search in the form the objective and the
      // search pass use (the FP32 x, summed in FP64)
      if constexpr (SG) acc_aa += (double)x;
      float phi, ft, fac;
      pixel_terms<WANT_F, EST>(x, dc[j], a.eps, phi, ft, fac);
      acc_phi += (double)phi;
      if constexpr (WANT_F) acc_f += (double)ft;
      v[s] = cscale(g, fac * invN);
    }
  }
  if constexpr (FARIN) {
    // test hook: the residual r = g fac itself, row layout like a.far
    if (a.gstore && valid) {
#pragma unroll
      for (int s = 0; s < G::E; ++s)
        (a.gstore + (size_t)k * N * N + kFreq<N>.f[s])[(uint32_t)L.line * N + (L.h ? G::E / 2 : 0)] =
            cscale(v[s], (float)N);
    }
  }
  // The sums are only consumed by the final reduction; without this the
  // compiler sinks the objective terms past the inverse transform and keeps
  // every pixel's (x, d) alive across it.
  asm volatile("" : "+v"(acc_phi), "+v"(acc_f), "+v"(acc_aa));
  inv_line<N>(v, L.h);
  transpose_r2c<N>(v, lds, L);
  inv_line<N>(v, L.h);
  store_u<N>(v, a, L, k, valid);
  if (!valid) {
    acc_phi = 0.0;
    acc_f = 0.0;
  }
  block_sum2<G::WG>(acc_phi, acc_f, red);
  if (threadIdx.x == 0) {
    a.partials[2 * blockIdx.x] = acc_phi;
    a.partials[2 * blockIdx.x + 1] = acc_f;
  }
  if constexpr (SG) {
    double zero = 0.0;
    __syncthreads();
    block_sum2<G::WG>(acc_aa, zero, red);
    if (threadIdx.x == 0) a.zs_part[blockIdx.x] = acc_aa;
  }
}

template <int N, DataLayout LAY, bool LINC_O, bool LINC_P, int EST, bool WF = true>
__global__ PTYG_PATTERN_KERNEL(N) void k_minfunc(PatArgs a) {
  using G = Geo<N>;
  __shared__ float2 lds[G::LDS_ELEMS];
  __shared__ double red[2 * (G::WG / 64)];
  const Lane L = lane_info<N>();
  int k;
  bool valid;
  int2 rc;
  if (!pattern_of<N>(a, L, k, valid, rc)) {
    write_zero_partials(a);
    return;
  }
  float2 v[G::E];
  gather_exit_wave<N, LINC_O, LINC_P>(v, a, L, rc, valid);
  fwd_line<N>(v, L.h);
  transpose_c2r<N>(v, lds, L);
  fwd_line<N>(v, L.h);
  const float invN = 1.0f / N;
  double acc_phi = 0.0, acc_f = 0.0;
  // intensities one chunk ahead (as in GRAD)
  float dn[kResChunk];
#pragma unroll
  for (int j = 0; j < kResChunk; ++j) dn[j] = load_data<N, LAY>(a.data, k, L, kOrd<N>.s[j]);
  // the solver's line search needs only Phi
  constexpr bool WANT_F = WF;
#pragma unroll
  for (int c = 0; c < G::E; c += kResChunk) {
    __builtin_amdgcn_sched_barrier(0);
    float dc[kResChunk];
#pragma unroll
    for (int j = 0; j < kResChunk; ++j) dc[j] = dn[j];
    if (c + kResChunk < G::E) {
#pragma unroll
      for (int j = 0; j < kResChunk; ++j) dn[j] = load_data<N, LAY>(a.data, k, L, kOrd<N>.s[c + kResChunk + j]);
    }
#pragma unroll
    for (int j = 0; j < kResChunk; ++j) {
      const float2 g = cscale(v[kOrd<N>.s[c + j]], invN);
      const float x = fmaf(g.x, g.x, g.y * g.y);
      float phi, ft, fac;
      pixel_terms<WANT_F, EST>(x, dc[j], a.eps, phi, ft, fac);
      acc_phi += (double)phi;
      if constexpr (WANT_F) acc_f += (double)ft;
    }
  }
  if (!valid) {
    acc_phi = 0.0;
    acc_f = 0.0;
  }
  block_sum2<G::WG>(acc_phi, acc_f, red);
  if (threadIdx.x == 0) {
    a.partials[2 * blockIdx.x] = acc_phi;
    a.partials[2 * blockIdx.x + 1] = acc_f;
  }
}

// d [K][N][N] -> per-pattern transpose [K][N][N] (element (a,b) at b*N+a),
// tiled 32 x 32 through LDS.
__global__ __launch_bounds__(256) void k_transpose_data(const float* __restrict__ d, float* __restrict__ dt,
                                                         int N) {
  __shared__ float tile[32][33];
  const int tiles = N / 32;
  const int k = blockIdx.z;
  const int ta = blockIdx.y, tb = blockIdx.x;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const float* src = d + (size_t)k * N * N;
  float* dst = dt + (size_t)k * N * N;
  (void)tiles;
#pragma unroll
  for (int j = 0; j < 32; j += 8) tile[ty + j][tx] = src[(size_t)(ta * 32 + ty + j) * N + tb * 32 + tx];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 32; j += 8) dst[(size_t)(tb * 32 + ty + j) * N + ta * 32 + tx] = tile[tx][ty + j];
}

// Small-N transpose (N < 32): one thread per element.
__global__ void k_transpose_data_small(const float* __restrict__ d, float* __restrict__ dt, int K, int N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)K * N * N;
  if (i >= tot) return;
  const int64_t k = i / ((int64_t)N * N);
  const int r = (int)(i % ((int64_t)N * N));
  const int aa = r / N, bb = r % N;
  dt[k * N * N + (int64_t)bb * N + aa] = d[i];
}

template <int N>
__global__ PTYG_PATTERN_KERNEL(N) void k_debug_gather(PatArgs a, float2* patches) {
  using G = Geo<N>;
  const Lane L = lane_info<N>();
  int k;
  bool valid;
  int2 rc;
  if (!pattern_of<N>(a, L, k, valid, rc)) {
    write_zero_partials(a);
    return;
  }
  if (!valid) return;
#pragma unroll
  for (int m = 0; m < G::E; ++m) {
    const int u = sidx<N>(m, L.h);
    patches[(size_t)k * N * N + u * N + L.line] = a.obj[(size_t)(rc.x + u) * a.W + rc.y + L.line];
  }
}

template <int N>
__global__ PTYG_PATTERN_KERNEL(N) void k_debug_scatter(PatArgs a, const float2* patches) {
  using G = Geo<N>;
  const Lane L = lane_info<N>();
  int k;
  bool valid;
  int2 rc;
  if (!pattern_of<N>(a, L, k, valid, rc)) {
    write_zero_partials(a);
    return;
  }
  if (!valid) return;
#pragma unroll
  for (int m = 0; m < G::E; ++m) {
    const int u = sidx<N>(m, L.h);
    const float2 val = patches[(size_t)k * N * N + u * N + L.line];
    const size_t idx = (size_t)(rc.x + u) * a.W + rc.y + L.line;
    unsafeAtomicAdd(&a.gobj[idx].x, val.x);
    unsafeAtomicAdd(&a.gobj[idx].y, val.y);
  }
}

// Element-per-thread versions of the debug hooks (any probe size).
__global__ void k_debug_gather_any(PatArgs a, float2* patches) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)a.N * a.N;
  if (i >= (int64_t)a.K * nn) return;
  const int k = (int)(i / nn), r = (int)(i % nn), u = r / a.N, v = r % a.N;
  const int2 rc = a.pos[k];
  patches[i] = a.obj[(size_t)(rc.x + u) * a.W + rc.y + v];
}

__global__ void k_debug_scatter_any(PatArgs a, const float2* patches) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)a.N * a.N;
  if (i >= (int64_t)a.K * nn) return;
  const int k = (int)(i / nn), r = (int)(i % nn), u = r / a.N, v = r % a.N;
  const int2 rc = a.pos[k];
  const size_t idx = (size_t)(rc.x + u) * a.W + rc.y + v;
  unsafeAtomicAdd(&a.gobj[idx].x, patches[i].x);
  unsafeAtomicAdd(&a.gobj[idx].y, patches[i].y);
}

__global__ void k_check_positions(const int2* pos, int K, int H, int W, int N, int* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const int2 p = pos[i];
  if (p.x < 0 || p.y < 0 || p.x > H - N || p.y > W - N) atomicOr(flag, 1);
}

__global__ void k_debug_lane_swap(float* a, float* b) {
  const int t = threadIdx.x;
  float2 x = make_float2(a[t], 0.f), y = make_float2(b[t], 0.f);
  swap32(x, y);
  a[t] = x.x;
  b[t] = y.x;
}

// ------------------------------------------------- deterministic overlap sum
__device__ __forceinline__ bool overlaps(int2 p, int N, int y0, int x0) {
  return p.x < y0 + kTileH && p.x + N > y0 && p.y < x0 + kTileW && p.y + N > x0;
}

// Pattern-parallel tile lists: each pattern adds itself to the tiles its
// patch overlaps (integer atomics: exact counts), the lists are filled in
// arrival order, then each tile's list is sorted into ascending pattern
// order, so the overlap sums run in a fixed order.
__device__ __forceinline__ void patch_tiles(int2 p, int N, int H, int W, int& ty0, int& ty1, int& tx0, int& tx1) {
  ty0 = p.x / kTileH;
  ty1 = min(p.x + N - 1, H - 1) / kTileH;
  tx0 = p.y / kTileW;
  tx1 = min(p.y + N - 1, W - 1) / kTileW;
}

// One thread per (pattern, candidate tile) pair: the j-th tile of the
// tiles_per_patch(N) span starting at the patch's first tile, skipped when
// it lies past the patch.
__device__ __forceinline__ int pair_tile(const int2* pos, int64_t idx, int tpp, int span_x, int N, int H, int W) {
  const int k = (int)(idx / tpp), j = (int)(idx % tpp);
  int ty0, ty1, tx0, tx1;
  patch_tiles(pos[k], N, H, W, ty0, ty1, tx0, tx1);
  const int ty = ty0 + j / span_x, tx = tx0 + j % span_x;
  if (ty > ty1 || tx > tx1) return -1;
  return ty * tiles_x(W) + tx;
}

__global__ __launch_bounds__(256) void k_tile_count_k(const int2* __restrict__ pos, int64_t pairs, int tpp,
                                                       int span_x, int H, int W, int N, int* __restrict__ counts) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= pairs) return;
  const int t = pair_tile(pos, idx, tpp, span_x, N, H, W);
  if (t >= 0) atomicAdd(&counts[t], 1);
}

__global__ __launch_bounds__(256) void k_tile_fill_k(const int2* __restrict__ pos, int64_t pairs, int tpp,
                                                      int span_x, int H, int W, int N,
                                                      const int* __restrict__ offsets, int* __restrict__ cursor,
                                                      int* __restrict__ list) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= pairs) return;
  const int t = pair_tile(pos, idx, tpp, span_x, N, H, W);
  if (t >= 0) list[offsets[t] + atomicAdd(&cursor[t], 1)] = (int)(idx / tpp);
}

// One workgroup per tile: bitonic sort of its list (up to 64 patterns in
// one wave's lanes, up to kSortMax in LDS); a longer list is rebuilt in
// order by scanning every pattern, as the per-tile fill does.
constexpr int kSortMax = 2048;
__global__ __launch_bounds__(256) void k_tile_sort(const int2* __restrict__ pos, int K, int W, int N,
                                                    const int* __restrict__ offsets, int* __restrict__ list) {
  __shared__ int key[kSortMax];
  __shared__ int wsum[4];
  const int t = blockIdx.x;
  const int beg = offsets[t], len = offsets[t + 1] - beg;
  if (len <= 1) return;
  if (len <= 64) {
    // one wave, one key per lane: bitonic network over lane shuffles (the
    // keys are distinct pattern indices; padding sorts last)
    if (threadIdx.x >= 64) return;
    const int l = threadIdx.x;
    int key = l < len ? list[beg + l] : 0x7fffffff;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        const int other = __shfl_xor(key, j);
        key = (((l & k) == 0) == ((l & j) == 0)) ? min(key, other) : max(key, other);
      }
    }
    if (l < len) list[beg + l] = key;
    return;
  }
  if (len <= kSortMax) {
    int P = 1;
    while (P < len) P <<= 1;
    for (int i = threadIdx.x; i < P; i += 256) key[i] = i < len ? list[beg + i] : 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < P; i += 256) {
          const int l = i ^ j;
          if (l > i) {
            const int a = key[i], b = key[l];
            const bool up = (i & k) == 0;
            if ((a > b) == up) {
              key[i] = b;
              key[l] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = threadIdx.x; i < len; i += 256) list[beg + i] = key[i];
    return;
  }
  // long list: ascending scan over all patterns with a ballot prefix
  const int ntx = tiles_x(W);
  const int y0 = (t / ntx) * kTileH, x0 = (t % ntx) * kTileW;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  int base = beg;
  for (int k0 = 0; k0 < K; k0 += 256) {
    const int k = k0 + threadIdx.x;
    const bool f = k < K && overlaps(pos[k], N, y0, x0);
    const unsigned long long m = __ballot(f);
    const int before = __popcll(m & ((1ull << l) - 1ull));
    if (l == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int woff = 0;
    for (int i = 0; i < w; ++i) woff += wsum[i];
    const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (f) list[base + woff + before] = k;
    base += tot;
    __syncthreads();
  }
}

// Exclusive scan of counts[0..T) into offsets[0..T] (one workgroup); with
// clear, counts[] is zeroed behind the scan (the fill's cursor).
__global__ __launch_bounds__(1024) void k_scan(int* __restrict__ counts, int T, int* __restrict__ offsets,
                                               int clear) {
  __shared__ int part[1024];
  const int per = (T + 1023) / 1024;
  const int lo = threadIdx.x * per, hi = min(T, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += counts[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;  // exclusive prefix of this chunk
  for (int i = lo; i < hi; ++i) {
    offsets[i] = run;
    run += counts[i];
    if (clear) counts[i] = 0;  // each entry is read and cleared by this thread only
  }
  if (threadIdx.x == 1023) offsets[T] = part[1023];
}

// grad[y][x] = sum over the tile's patterns (ascending k) of conj(p) * u_k,
// or of the stored values themselves when they already carry conj(p).
// 256 threads on a 16 x 64 tile: lane l of wave w holds the column pair
// x = x0 + 2 (l mod 32), x + 1 in the rows y0 + 2 w + l / 32 + 8 i, so each
// row of the tile is one 512-byte run of 16-byte accesses.  The tile's pattern list
// and positions are staged in LDS (kTileStage at a time) so the loop issues
// its loads without waiting on scalar loads.
constexpr int kTileStage = 512;

// Offset of u_k[yy][xx] inside pattern k's block of U: natural row-major, or
// for 256^2 patterns the polyphase layout [2 (yy&1) + (xx&1)][yy/2][xx/2].
template <bool POLY>
__device__ __forceinline__ int u_off(int yy, int xx, int N) {
  if constexpr (POLY) return (((yy & 1) << 1) | (xx & 1)) * (N * N / 4) + (yy >> 1) * (N / 2) + (xx >> 1);
  else return yy * N + xx;
}

// The loads of kTileDepth patterns (half as many when the probe is loaded
// too) are issued before their adds, and no
// load sits behind a branch, so the adds still run in ascending pattern
// order.  Natural layout: one 16-byte buffer load per (pattern, row) reads
// the pair's two values (pattern columns xc, xc + 1 with xc clamped to
// [0, N - 2]; the lanes at the patch's left and right edge shift the pair);
// a row or pair outside the patch gets an offset past the buffer's range,
// which the hardware answers with zeros and no memory access.  Polyphase
// layout (always with the probe): the pair's columns lie in different
// planes, two 8-byte loads with the same out-of-range offset outside the
// patch; the probe's pair is one 16-byte load as in the natural layout.
constexpr int kTileDepth = 8;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufDword3 = 0x00020000;  // raw (untyped) buffer, 32-bit data format

__device__ __forceinline__ void pair_of(u32x4 w, int xx, int N, float2& v0, float2& v1) {
  const float4 f = __builtin_bit_cast(float4, w);
  const float2 lo = make_float2(f.x, f.y), hi = make_float2(f.z, f.w);
  const bool left = xx == -1, right = xx == N - 1;
  v0 = left ? make_float2(0.f, 0.f) : (right ? hi : lo);
  v1 = left ? lo : (right ? make_float2(0.f, 0.f) : hi);
}

// dot_parts (nullable): per tile (sum |out|^2, sum Re(conj(dot_b) out)) over
// the tile's pixels (the second 0 when dot_b is null), as written.
template <bool POLY, bool PROBE>
__global__ __launch_bounds__(256) void k_tile_sum(const float2* __restrict__ U, const float2* __restrict__ probe,
                                                   const int2* __restrict__ pos, const int* __restrict__ offsets,
                                                   const int* __restrict__ list, int H, int W, int N,
                                                   int64_t ustride, float2* __restrict__ out,
                                                   const float2* __restrict__ dot_b, double* __restrict__ dot_parts) {
  static_assert(kTileW == 64 && kTileH == 16, "32 column pairs per row, two rows per wave and step");
  static_assert(PROBE || !POLY, "polyphase waves are stored without conj(p)");
  __shared__ int sk[kTileStage];
  __shared__ int2 sp[kTileStage];
  __shared__ double red[2 * 4];
  const int ntx = tiles_x(W);
  const int t = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int x = (t % ntx) * kTileW + 2 * (lane & 31);
  const int yb = (t / ntx) * kTileH + 2 * (threadIdx.x >> 6) + (lane >> 5);
  constexpr int RS = 8;  // row step
  constexpr int R = kTileH / RS;
  constexpr int D = PROBE ? kTileDepth / 2 : kTileDepth;  // the probe's loads double the registers
  const int nrec = N * N * (int)sizeof(float2);
  float2 a0[R], a1[R];
#pragma unroll
  for (int i = 0; i < R; ++i) a0[i] = a1[i] = make_float2(0.f, 0.f);
  const __amdgpu_buffer_rsrc_t prs =
      __builtin_amdgcn_make_buffer_rsrc((void*)probe, (short)0, PROBE ? nrec : 0, kBufDword3);
  const int beg = offsets[t], end = offsets[t + 1];
  for (int s0 = beg; s0 < end; s0 += kTileStage) {
    const int n = min(kTileStage, end - s0);
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += 256) {
      const int k = list[s0 + j];
      sk[j] = k;
      sp[j] = pos[k];
    }
    __syncthreads();
    for (int j = 0; j < n; j += D) {
      if constexpr (!POLY) {
        u32x4 uv[D][R], pv[D][R];
        int xs[D];
#pragma unroll
        for (int q = 0; q < D; ++q) {
          const bool live = j + q < n;
          const int jj = live ? j + q : j;
          const int2 rc = sp[jj];
          const int k = __builtin_amdgcn_readfirstlane(sk[jj]);
          const int xx = x - rc.y;
          xs[q] = xx;
          const bool cv = live && xx >= -1 && xx < N;
          const int xc = min(max(xx, 0), N - 2);
          const __amdgpu_buffer_rsrc_t rs =
              __builtin_amdgcn_make_buffer_rsrc((void*)(U + (int64_t)k * ustride), (short)0, nrec, kBufDword3);
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const int yy = yb + RS * i - rc.x;
            const int off = (cv && (unsigned)yy < (unsigned)N) ? (yy * N + xc) * (int)sizeof(float2) : 0x7fffffff;
            uv[q][i] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
            if constexpr (PROBE) pv[q][i] = __builtin_amdgcn_raw_buffer_load_b128(prs, off, 0, 0);
          }
        }
        // keep every load of the group ahead of the first add
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < D; ++q) {
#pragma unroll
          for (int i = 0; i < R; ++i) {
            float2 v0, v1;
            pair_of(uv[q][i], xs[q], N, v0, v1);
            if constexpr (PROBE) {
              float2 p0, p1;
              pair_of(pv[q][i], xs[q], N, p0, p1);
              v0 = cmulc(p0, v0);
              v1 = cmulc(p1, v1);
            }
            a0[i] = cadd(a0[i], v0);
            a1[i] = cadd(a1[i], v1);
          }
        }
      } else {
        u32x2 u0[D][R], u1[D][R];
        u32x4 pv[D][R];
        int xs[D];
#pragma unroll
        for (int q = 0; q < D; ++q) {
          const bool live = j + q < n;
          const int jj = live ? j + q : j;
          const int2 rc = sp[jj];
          const int k = __builtin_amdgcn_readfirstlane(sk[jj]);
          const int xx = x - rc.y;
          xs[q] = xx;
          const bool c0 = live && (unsigned)xx < (unsigned)N, c1 = live && (unsigned)(xx + 1) < (unsigned)N;
          const bool cv = live && xx >= -1 && xx < N;
          const int xc = min(max(xx, 0), N - 2);
          const __amdgpu_buffer_rsrc_t rs =
              __builtin_amdgcn_make_buffer_rsrc((void*)(U + (int64_t)k * ustride), (short)0, nrec, kBufDword3);
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const int yy = yb + RS * i - rc.x;
            const bool r = (unsigned)yy < (unsigned)N;
            const int o0 = (c0 && r) ? u_off<true>(yy, xx, N) * (int)sizeof(float2) : 0x7fffffff;
            const int o1 = (c1 && r) ? u_off<true>(yy, xx + 1, N) * (int)sizeof(float2) : 0x7fffffff;
            u0[q][i] = __builtin_amdgcn_raw_buffer_load_b64(rs, o0, 0, 0);
            u1[q][i] = __builtin_amdgcn_raw_buffer_load_b64(rs, o1, 0, 0);
            // the probe is stored naturally: its pair is one 16-byte load
            const int op = (cv && r) ? (yy * N + xc) * (int)sizeof(float2) : 0x7fffffff;
            pv[q][i] = __builtin_amdgcn_raw_buffer_load_b128(prs, op, 0, 0);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < D; ++q) {
#pragma unroll
          for (int i = 0; i < R; ++i) {
            float2 p0, p1;
            pair_of(pv[q][i], xs[q], N, p0, p1);
            a0[i] = cadd(a0[i], cmulc(p0, __builtin_bit_cast(float2, u0[q][i])));
            a1[i] = cadd(a1[i], cmulc(p1, __builtin_bit_cast(float2, u1[q][i])));
          }
        }
      }
    }
  }
  // the dot products' other operand (loaded after the sum: held across the
  // loop it cost the kernel a third of its occupancy)
  float2 e0[R], e1[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int y = yb + RS * i;
    const bool row = dot_b && y < H;
    e0[i] = (row && x < W) ? dot_b[(size_t)y * W + x] : make_float2(0.f, 0.f);
    e1[i] = (row && x + 1 < W) ? dot_b[(size_t)y * W + x + 1] : make_float2(0.f, 0.f);
  }
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int y = yb + RS * i;
    if (y >= H) continue;
    if (x < W) {
      out[(size_t)y * W + x] = a0[i];
      if (dot_parts) {
        s1 += (double)a0[i].x * a0[i].x + (double)a0[i].y * a0[i].y;
        if (dot_b) s2 += (double)e0[i].x * a0[i].x + (double)e0[i].y * a0[i].y;
      }
    }
    if (x + 1 < W) {
      out[(size_t)y * W + x + 1] = a1[i];
      if (dot_parts) {
        s1 += (double)a1[i].x * a1[i].x + (double)a1[i].y * a1[i].y;
        if (dot_b) s2 += (double)e1[i].x * a1[i].x + (double)e1[i].y * a1[i].y;
      }
    }
  }
  if (dot_parts) {
    block_sum2<256>(s1, s2, red);
    if (threadIdx.x == 0) {
      dot_parts[2 * (size_t)t] = s1;
      dot_parts[2 * (size_t)t + 1] = s2;
    }
  }
}

// partial[c][u][v] = sum over the patterns of chunk c (ascending) of
// conj(obj[r_k + u][c_k + v]) u_k[u][v].
template <bool POLY>
__global__ __launch_bounds__(256) void k_probe_partial(const float2* __restrict__ U, const float2* __restrict__ obj,
                                                        const int2* __restrict__ pos, int K, int W, int N,
                                                        float2* __restrict__ partial) {
  const int px = blockIdx.x * 256 + threadIdx.x;
  const int nn = N * N;
  if (px >= nn) return;
  const int u = px / N, v = px % N;
  const int chunk = (K + kProbeChunks - 1) / kProbeChunks;
  const int k0 = blockIdx.y * chunk, k1 = min(K, k0 + chunk);
  float2 acc = make_float2(0.f, 0.f);
  for (int k = k0; k < k1; ++k) {
    const int2 rc = pos[k];
    const float2 o = obj[(size_t)(rc.x + u) * W + rc.y + v];
    acc = cadd(acc, cmulc(o, U[(size_t)k * nn + u_off<POLY>(u, v, N)]));
  }
  partial[(size_t)blockIdx.y * nn + px] = acc;
}

__global__ __launch_bounds__(256) void k_probe_reduce(const float2* __restrict__ partial, int nn,
                                                       float2* __restrict__ out) {
  const int px = blockIdx.x * 256 + threadIdx.x;
  if (px >= nn) return;
  float2 acc = make_float2(0.f, 0.f);
  for (int c = 0; c < kProbeChunks; ++c) acc = cadd(acc, partial[(size_t)c * nn + px]);
  out[px] = acc;
}

// ------------------------------------------------------------ vector kernels
constexpr int kVecWG = 256;
constexpr int kVecMaxBlocks = 2048;

__global__ __launch_bounds__(kVecWG) void k_zero(float2* x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kVecWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecWG)
    x[i] = make_float2(0.f, 0.f);
}
__global__ __launch_bounds__(kVecWG) void k_zero_f64(double* x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kVecWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecWG)
    x[i] = 0.0;
}

__global__ __launch_bounds__(kVecWG) void k_fill_i32(int* x, int64_t n, int value) {
  for (int64_t i = (int64_t)blockIdx.x * kVecWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecWG)
    x[i] = value;
}

// Per-block sums of d - d log d over the d > 0 elements (NaN propagates) of
// segment blockIdx.y (n elements each), accumulated in FP64: the constant
// between Eq. ML and its deviance form.  The logarithm is the FP32 one
// (relative error ~1e-7 per term, far below the 1e-5 the trace's F is
// reported to; an FP64 logarithm made this pass cost more than a GRAD).
__device__ __forceinline__ double data_const_term(float v) {
  const double dv = v;
  return !(v <= 0.0f) ? dv - dv * (double)(__log2f(v) * kLn2) : 0.0;
}
__global__ __launch_bounds__(kVecWG) void k_data_const(const float* __restrict__ d, int64_t n,
                                                        double* __restrict__ partials) {
  __shared__ double red[2 * (kVecWG / 64)];
  const float* ds = d + (int64_t)blockIdx.y * n;
  const int64_t stride = (int64_t)gridDim.x * kVecWG;
  double acc = 0.0, acc2 = 0.0;
  int64_t i = (int64_t)blockIdx.x * kVecWG + threadIdx.x;
  // four independent loads per step, two accumulators
  for (; i + 3 * stride < n; i += 4 * stride) {
    const float v0 = ds[i], v1 = ds[i + stride], v2 = ds[i + 2 * stride], v3 = ds[i + 3 * stride];
    acc += data_const_term(v0) + data_const_term(v1);
    acc2 += data_const_term(v2) + data_const_term(v3);
  }
  for (; i < n; i += stride) acc += data_const_term(ds[i]);
  acc += acc2;
  double unused = 0.0;
  block_sum2<kVecWG>(acc, unused, red);
  if (threadIdx.x == 0) partials[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

__global__ __launch_bounds__(kVecWG) void k_dot2(VecArgs v) {
  __shared__ double red[2 * (kVecWG / 64)];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kVecWG + threadIdx.x; i < v.n; i += (int64_t)gridDim.x * kVecWG) {
    const float2 g = v.a[i];
    s1 += (double)g.x * g.x + (double)g.y * g.y;
    if (v.b) {
      const float2 e = v.b[i];
      s2 += (double)e.x * g.x + (double)e.y * g.y;
    }
  }
  block_sum2<kVecWG>(s1, s2, red);
  if (threadIdx.x == 0) {
    v.partials[2 * blockIdx.x] = s1;
    v.partials[2 * blockIdx.x + 1] = s2;
  }
}

__global__ __launch_bounds__(kVecWG) void k_dir(VecArgs v) {
  __shared__ double red[2 * (kVecWG / 64)];
  __shared__ double red4[4 * (kVecWG / 64)];
  double s1 = 0.0, s2 = 0.0;
  double z[4] = {0.0, 0.0, 0.0, 0.0};
  const bool zs = v.zs_part != nullptr;
  double beta_d;
  bool rst;
  if (v.dy_n1) {
    const double num = *v.dy_n1, den = *v.dy_n2 - *v.dy_n3;
    const bool ok = !v.dy_restart && isfinite(den) && den > 0.0 && isfinite(num);
    beta_d = ok ? num / den : 0.0;
    rst = !ok;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      v.dy_out[0] = beta_d;
      v.dy_out[1] = rst ? 1.0 : 0.0;
    }
  } else {
    beta_d = v.alpha_dev ? *v.alpha_dev : v.alpha;
    rst = v.restart_dev && *v.restart_dev != 0.0;
  }
  const float beta = (float)beta_d;
  for (int64_t i = (int64_t)blockIdx.x * kVecWG + threadIdx.x; i < v.n; i += (int64_t)gridDim.x * kVecWG) {
    const float2 g = v.a[i];
    const float2 e = v.b[i];
    const float2 en = rst ? make_float2(-g.x, -g.y) : make_float2(fmaf(beta, e.x, -g.x), fmaf(beta, e.y, -g.y));
    v.b[i] = en;
    s1 += (double)en.x * g.x + (double)en.y * g.y;
    s2 += (double)en.x * en.x + (double)en.y * en.y;
    if (zs) {
      const float2 p = v.zs_psi[i];
      const double w = v.zs_w[i].x;
      z[0] += w * ((double)p.x * en.x + (double)p.y * en.y);
      z[2] += w * ((double)en.x * en.x + (double)en.y * en.y);
    }
  }
  block_sum2<kVecWG>(s1, s2, red);
  if (threadIdx.x == 0) {
    v.partials[2 * blockIdx.x] = s1;
    v.partials[2 * blockIdx.x + 1] = s2;
  }
  if (zs) block_sum4_store<kVecWG>(z, red4, v.zs_part + 4 * blockIdx.x);
}

__global__ void k_dy_beta(double* sc, int n1, int n2, int n3, int joint_off, int beta, int rst, int restart) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double num = sc[n1], a = sc[n2], b = sc[n3];
  if (joint_off > 0) {
    num += sc[n1 + joint_off];
    a += sc[n2 + joint_off];
    b += sc[n3 + joint_off];
  }
  const double den = a - b;
  const bool ok = !restart && isfinite(den) && den > 0.0 && isfinite(num);
  sc[beta] = ok ? num / den : 0.0;
  sc[rst] = ok ? 0.0 : 1.0;
}

// A zero step leaves `a` untouched (also when c holds NaN: the solver's
// device-side update after a search that accepted nothing).
__global__ __launch_bounds__(kVecWG) void k_axpy(VecArgs v) {
  const float al = (float)(v.alpha_dev ? *v.alpha_dev : v.alpha);
  if (al == 0.0f) return;
  for (int64_t i = (int64_t)blockIdx.x * kVecWG + threadIdx.x; i < v.n; i += (int64_t)gridDim.x * kVecWG) {
    const float2 x = v.a[i], c = v.c[i];
    v.a[i] = make_float2(fmaf(al, c.x, x.x), fmaf(al, c.y, x.y));
  }
}

__global__ __launch_bounds__(kVecWG) void k_sum_copies(const float2* src, int copies, int64_t n, float2* out) {
  for (int64_t i = (int64_t)blockIdx.x * kVecWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecWG) {
    float2 s = make_float2(0.f, 0.f);
    for (int c = 0; c < copies; ++c) {
      const float2 x = src[(int64_t)c * n + i];
      s.x += x.x;
      s.y += x.y;
    }
    out[i] = s;
  }
}

// Batched line search (linearity of G): trial j's far field is
// A + g_j B (+ g_j^2 C), evaluated with the same per-pixel deviance as a
// MINFUNC pass for every listed element (d > 0 or NaN), FP64 accumulation
// per trial, per-workgroup partials in a fixed order.
template <bool QUAD, int EST, bool CP>
__global__ __launch_bounds__(256) void k_ls_batch(LsArgs a) {
  __shared__ double red[4][kLsRow];
  double acc[kLsRow];
#pragma unroll
  for (int j = 0; j < kLsRow; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * 256) {
    const int64_t e = CP ? i : (int64_t)a.idx[i];
    const float2 av = a.A[e], bv = a.B[e];
    float2 cv = make_float2(0.f, 0.f);
    if constexpr (QUAD) cv = a.C[e];
    const float dv = a.d[e];
    // this element's share of the whole-array sums (the rest is d <= 0)
    acc[kLsBatch + 0] += (double)fmaf(av.x, av.x, av.y * av.y);  // as GRAD sums |G psi|^2
    acc[kLsBatch + 1] += (double)av.x * bv.x + (double)av.y * bv.y;
    acc[kLsBatch + 2] += (double)bv.x * bv.x + (double)bv.y * bv.y;
    if constexpr (QUAD) {
      acc[kLsBatch + 3] += (double)av.x * cv.x + (double)av.y * cv.y;
      acc[kLsBatch + 4] += (double)bv.x * cv.x + (double)bv.y * cv.y;
      acc[kLsBatch + 5] += (double)cv.x * cv.x + (double)cv.y * cv.y;
    }
#pragma unroll
    for (int j = 0; j < kLsBatch; ++j) {
      if (j < a.J) {
        const float gm = a.g[j];
        float xr = fmaf(gm, bv.x, av.x), xi = fmaf(gm, bv.y, av.y);
        if constexpr (QUAD) {
          const float g2 = gm * gm;
          xr = fmaf(g2, cv.x, xr);
          xi = fmaf(g2, cv.y, xi);
        }
        float phi, ft, fac;
        pixel_terms_br<false, EST>(fmaf(xr, xr, xi * xi), dv, a.eps, phi, ft, fac);
        acc[j] += (double)phi;
      }
    }
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < kLsRow; ++j) {
    double v = acc[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (l == 0) red[w][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < kLsRow)
    a.partials[(size_t)blockIdx.x * kLsRow + threadIdx.x] =
        red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// Compaction of the elements with !(d <= 0): per-block counts, then the
// indices in ascending order (wave ballots, waves in order, 256-element rounds).
__global__ __launch_bounds__(256) void k_nz_count(const float* __restrict__ d, int64_t n, int* counts) {
  __shared__ int red[4];
  const int64_t base = (int64_t)blockIdx.x * kNzChunk;
  int c = 0;
  for (int r = 0; r < kNzChunk / 256; ++r) {
    const int64_t e = base + r * 256 + threadIdx.x;
    c += (e < n && !(d[e] <= 0.0f)) ? 1 : 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_nz_fill(const float* __restrict__ d, int64_t n,
                                                 const int* __restrict__ offsets, int* __restrict__ idx,
                                                 uint2* __restrict__ seg, float* __restrict__ dc) {
  __shared__ int wcnt[4];
  const int64_t base = (int64_t)blockIdx.x * kNzChunk;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const uint64_t below = (l == 0) ? 0ull : (~0ull >> (64 - l));
  int run = offsets[blockIdx.x];
  for (int r = 0; r < kNzChunk / 256; ++r) {
    const int64_t e = base + r * 256 + threadIdx.x;
    const float de = e < n ? d[e] : 0.0f;
    const bool nz = e < n && !(de <= 0.0f);
    const uint64_t m = __ballot(nz);
    if (l == 0) wcnt[w] = __popcll(m);
    __syncthreads();
    int pre = 0;
    for (int i = 0; i < w; ++i) pre += wcnt[i];
    const int at = run + pre + __popcll(m & below);
    if (nz) {
      idx[at] = (int)e;
      if (dc) dc[at] = de;
    }
    // segment records: lanes 0 and 32 of the wave (32 elements each)
    if (seg && (l & 31) == 0 && e < n)
      seg[e >> 5] = make_uint2((uint32_t)(l ? (m >> 32) : (m & 0xffffffffull)), (uint32_t)at);
    run += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
}

// Joint-mode coefficients of the batched search in the pattern domain: with
// a' = p psi_k, b' = p eta_k + eta_p psi_k, c' = eta_p eta_k on every patch
// pixel, the unitary transform keeps the inner products, so the sums of
// Re(a b*), |b|^2, Re(a c*), Re(b c*), |c|^2 over the far fields equal the
// same sums over the patches.  Rows of 4 per block in two arrays:
// (Re a'b'*, 0, |b'|^2, 0) and (Re a'c'*, Re b'c'*, |c'|^2, 0); blocks walk
// 4096-pixel chunks in a fixed order.
constexpr int kPsChunk = 4096;
constexpr int kPsMaxBlocks = 8192;

__global__ __launch_bounds__(256) void k_patch_sums(const float2* __restrict__ obj, const float2* __restrict__ eta,
                                                     const float2* __restrict__ probe,
                                                     const float2* __restrict__ eta_p, const int2* __restrict__ pos,
                                                     int K, int W, int lgN, double* __restrict__ parts1,
                                                     double* __restrict__ parts2) {
  __shared__ double red1[4 * 4], red2[4 * 4];
  const int N = 1 << lgN;
  const int nn = N * N;
  const int cpp = (nn + kPsChunk - 1) / kPsChunk;
  const int64_t chunks = (int64_t)K * cpp;
  double z1[4] = {0.0, 0.0, 0.0, 0.0}, z2[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const int k = (int)(c / cpp);
    const int base = (int)(c % cpp) * kPsChunk;
    const int lim = min(kPsChunk, nn - base);
    const int2 rc = pos[k];
    for (int i = threadIdx.x; i < lim; i += 256) {
      const int px = base + i;
      const int u = px >> lgN, v = px & (N - 1);
      const size_t o = (size_t)(rc.x + u) * W + rc.y + v;
      const float2 x = obj[o], y = eta[o], p = probe[px], q = eta_p[px];
      const float2 a = cmul(p, x), b = cadd(cmul(p, y), cmul(q, x)), cc = cmul(q, y);
      z1[0] += (double)a.x * b.x + (double)a.y * b.y;
      z1[2] += (double)b.x * b.x + (double)b.y * b.y;
      z2[0] += (double)a.x * cc.x + (double)a.y * cc.y;
      z2[1] += (double)b.x * cc.x + (double)b.y * cc.y;
      z2[2] += (double)cc.x * cc.x + (double)cc.y * cc.y;
    }
  }
  block_sum4_store<256>(z1, red1, parts1 + 4 * blockIdx.x);
  block_sum4_store<256>(z2, red2, parts2 + 4 * blockIdx.x);
}

// One thread: the batched pass's decision (see launch_ls_accept).
__global__ void k_ls_accept(const double* sc, const double* zs, const double* row, double* out, LsAccept a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double phi = sc[0];
  const double* sh = row + kLsBatch;
  double zc[6] = {zs[0] - sh[0], zs[4] - sh[1], zs[6] - sh[2], 0.0, 0.0, 0.0};
  if (a.joint) {
    zc[3] = zs[8] - sh[3];
    zc[4] = zs[9] - sh[4];
    zc[5] = zs[10] - sh[5];
  }
  double gamma = 0.0, idx = 0.0, stop = 0.0;
  if (a.stop_check && a.target >= 0.0 && phi <= a.target) {
    stop = 1.0;
  } else {
    for (int i = 0; i < a.J; ++i) {
      const double g = (double)(float)a.gam[i];
      double zero = zc[0] + 2.0 * g * zc[1] + g * g * zc[2];
      if (a.joint) zero += 2.0 * g * g * zc[3] + 2.0 * g * g * g * zc[4] + g * g * g * g * zc[5];
      if (row[i] + zero <= phi + a.gam[i] * a.t) {
        gamma = a.gam[i];
        idx = (double)(i + 1);
        break;
      }
    }
  }
  out[0] = gamma;
  out[1] = idx;
  out[2] = stop;
}

// out[j] = sum over rows (in order) of partials[row][j]; one workgroup per j.
__global__ __launch_bounds__(256) void k_ls_finalize(const double* partials, int count, double* out) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const int per = (count + 255) / 256;
  const int lo = threadIdx.x * per, hi = min(count, lo + per);
  double acc = 0.0;
  for (int i = lo; i < hi; ++i) acc += partials[(size_t)i * kLsRow + j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

// ------------------------------------------------------ multi-view batch
// Per-view ordered sums of pattern-kernel partials: workgroup v walks every
// block, keeps those whose pattern group lies in view v (each thread a
// contiguous range of blocks, then a fixed tree).
__global__ __launch_bounds__(256) void k_finalize_views(const double* partials, int nblocks, int groups, int ppw,
                                                        int k_per_view, int width, double* out) {
  __shared__ double red[256 * 4];
  const int v = blockIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int per = (nblocks + 255) / 256;
  const int lo = threadIdx.x * per, hi = min(nblocks, lo + per);
  for (int b = lo; b < hi; ++b) {
    const int g = group_of_block(b, groups);
    if (g < 0 || (g * ppw) / k_per_view != v) continue;
    for (int j = 0; j < width; ++j) acc[j] += partials[(size_t)b * width + j];
  }
  for (int j = 0; j < 4; ++j) red[threadIdx.x * 4 + j] = acc[j];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int j = 0; j < 4; ++j) red[threadIdx.x * 4 + j] += red[(threadIdx.x + off) * 4 + j];
    __syncthreads();
  }
  if (threadIdx.x < width) out[(size_t)v * width + threadIdx.x] = red[threadIdx.x];
}

// grid (kSegBlocks, views): block (i, v) covers view v's elements with stride
__global__ __launch_bounds__(kVecWG) void k_dot2_views(const float2* a, const float2* b, int64_t n,
                                                       double* partials) {
  __shared__ double red[2 * (kVecWG / 64)];
  const int v = blockIdx.y;
  const float2* av = a + (size_t)v * n;
  const float2* bv = b ? b + (size_t)v * n : nullptr;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kVecWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecWG) {
    const float2 g = av[i];
    s1 += (double)g.x * g.x + (double)g.y * g.y;
    if (bv) {
      const float2 e = bv[i];
      s2 += (double)e.x * g.x + (double)e.y * g.y;
    }
  }
  block_sum2<kVecWG>(s1, s2, red);
  if (threadIdx.x == 0) {
    double* p = partials + ((size_t)v * gridDim.x + blockIdx.x) * 2;
    p[0] = s1;
    p[1] = s2;
  }
}

__global__ __launch_bounds__(kVecWG) void k_dir_views(const float2* a, float2* b, const double* beta, int64_t n,
                                                      double* partials) {
  __shared__ double red[2 * (kVecWG / 64)];
  const int v = blockIdx.y;
  const float2* av = a + (size_t)v * n;
  float2* bv = b + (size_t)v * n;
  const float bt = (float)beta[v];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kVecWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecWG) {
    const float2 g = av[i];
    const float2 e = bv[i];
    const float2 en = make_float2(fmaf(bt, e.x, -g.x), fmaf(bt, e.y, -g.y));
    bv[i] = en;
    s1 += (double)en.x * g.x + (double)en.y * g.y;
    s2 += (double)en.x * en.x + (double)en.y * en.y;
  }
  block_sum2<kVecWG>(s1, s2, red);
  if (threadIdx.x == 0) {
    double* p = partials + ((size_t)v * gridDim.x + blockIdx.x) * 2;
    p[0] = s1;
    p[1] = s2;
  }
}

__global__ __launch_bounds__(kVecWG) void k_axpy_views(float2* a, const float2* c, const double* alpha, int64_t n) {
  const int v = blockIdx.y;
  const float al = (float)alpha[v];
  if (al == 0.0f) return;  // a zero step leaves the view untouched
  float2* av = a + (size_t)v * n;
  const float2* cv = c + (size_t)v * n;
  for (int64_t i = (int64_t)blockIdx.x * kVecWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecWG) {
    const float2 x = av[i], y = cv[i];
    av[i] = make_float2(fmaf(al, y.x, x.x), fmaf(al, y.y, x.y));
  }
}

// one workgroup per view: ordered sum of its `rows` rows
__global__ __launch_bounds__(256) void k_finalize_seg(const double* partials, int rows, int width, double* out) {
  __shared__ double red[256 * 4];
  const int v = blockIdx.x;
  const double* base = partials + (size_t)v * rows * width;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int per = (rows + 255) / 256;
  const int lo = threadIdx.x * per, hi = min(rows, lo + per);
  for (int i = lo; i < hi; ++i)
    for (int j = 0; j < width; ++j) acc[j] += base[(size_t)i * width + j];
  for (int j = 0; j < 4; ++j) red[threadIdx.x * 4 + j] = acc[j];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int j = 0; j < 4; ++j) red[threadIdx.x * 4 + j] += red[(threadIdx.x + off) * 4 + j];
    __syncthreads();
  }
  if (threadIdx.x < width) out[(size_t)v * width + threadIdx.x] = red[threadIdx.x];
}

// Batched line-search pass, one row of kSegBlocks workgroups per view.
template <bool QUAD, int EST>
__global__ __launch_bounds__(256) void k_ls_batch_views(LsArgs a, const int* offsets, int chunks_per_view) {
  __shared__ double red[4][kLsRow];
  const int v = blockIdx.y;
  const int64_t beg = offsets[(size_t)v * chunks_per_view], end = offsets[(size_t)(v + 1) * chunks_per_view];
  double acc[kLsRow];
#pragma unroll
  for (int j = 0; j < kLsRow; ++j) acc[j] = 0.0;
  for (int64_t i = beg + (int64_t)blockIdx.x * 256 + threadIdx.x; i < end; i += (int64_t)gridDim.x * 256) {
    const int e = a.idx[i];
    const float2 av = a.A[e], bv = a.B[e];
    float2 cv = make_float2(0.f, 0.f);
    if constexpr (QUAD) cv = a.C[e];
    const float dv = a.d[e];
    acc[kLsBatch + 0] += (double)fmaf(av.x, av.x, av.y * av.y);  // as GRAD sums |G psi|^2
    acc[kLsBatch + 1] += (double)av.x * bv.x + (double)av.y * bv.y;
    acc[kLsBatch + 2] += (double)bv.x * bv.x + (double)bv.y * bv.y;
#pragma unroll
    for (int j = 0; j < kLsBatch; ++j) {
      if (j < a.J) {
        const float gm = a.g[j];
        float xr = fmaf(gm, bv.x, av.x), xi = fmaf(gm, bv.y, av.y);
        if constexpr (QUAD) {
          const float g2 = gm * gm;
          xr = fmaf(g2, cv.x, xr);
          xi = fmaf(g2, cv.y, xi);
        }
        float phi, ft, fac;
        pixel_terms_br<false, EST>(fmaf(xr, xr, xi * xi), dv, a.eps, phi, ft, fac);
        acc[j] += (double)phi;
      }
    }
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < kLsRow; ++j) {
    double x = acc[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if (l == 0) red[w][j] = x;
  }
  __syncthreads();
  if (threadIdx.x < kLsRow)
    a.partials[((size_t)v * gridDim.x + blockIdx.x) * kLsRow + threadIdx.x] =
        red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// grid (kLsRow, views): ordered sum of a view's kSegBlocks rows, one column
__global__ __launch_bounds__(256) void k_ls_finalize_views(const double* partials, double* out) {
  __shared__ double red[256];
  const int j = blockIdx.x, v = blockIdx.y;
  const double* base = partials + (size_t)v * kSegBlocks * kLsRow;
  double acc = 0.0;
  for (int i = threadIdx.x; i < kSegBlocks; i += 256) acc += base[(size_t)i * kLsRow + j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(size_t)v * kLsRow + j] = red[0];
}

// Stacked positions: view v's pattern j < k at its position shifted down by
// v * rows_per_view; the slots j in [k, kp) that pad each view to kp
// patterns at (pad_row, 0), on the zero rows below the last view.
__global__ void k_shift_views(const int2* pos, int k, int kp, int views, int rows_per_view, int pad_row,
                              int2* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kp * views) return;
  const int v = i / kp, j = i % kp;
  out[i] = j < k ? make_int2(pos[v * k + j].x + v * rows_per_view, pos[v * k + j].y) : make_int2(pad_row, 0);
}

// In-order reduction of `count` rows of `width` (<= 4) doubles, one workgroup.
// Ordered sum of per-block partial rows: each thread adds a contiguous run of
// rows in order (four rows loaded ahead of their adds), then a fixed tree.
template <int W>
__device__ __forceinline__ void finalize_rows(const FinJob& j, double* red) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int per = (j.count + 255) / 256;
  const int lo = threadIdx.x * per, hi = min(j.count, lo + per);
  int i = lo;
  for (; i + 4 <= hi; i += 4) {
    double r[4][W];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < W; ++c) r[q][c] = j.p[(size_t)(i + q) * W + c];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < W; ++c) acc[c] += r[q][c];
  }
  for (; i < hi; ++i)
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] += j.p[(size_t)i * W + c];
#pragma unroll
  for (int c = 0; c < 4; ++c) red[threadIdx.x * 4 + c] = acc[c];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off)
#pragma unroll
      for (int c = 0; c < 4; ++c) red[threadIdx.x * 4 + c] += red[(threadIdx.x + off) * 4 + c];
    __syncthreads();
  }
  if (threadIdx.x < W) j.out[threadIdx.x] = red[threadIdx.x];
}

// Workgroup b finalizes job b (up to four independent reductions per launch).
struct FinJobs {
  FinJob j[4];
};
__global__ __launch_bounds__(256) void k_finalize(FinJobs jobs) {
  __shared__ double red[256 * 4];
  const FinJob j = jobs.j[blockIdx.x];
  switch (j.width) {
    case 1: finalize_rows<1>(j, red); break;
    case 2: finalize_rows<2>(j, red); break;
    case 3: finalize_rows<3>(j, red); break;
    default: finalize_rows<4>(j, red); break;
  }
}

template <int N>
int pattern_blocks(int K) {
  return blocks_for_groups((K + Geo<N>::PPW - 1) / Geo<N>::PPW);
}

template <typename F>
hipError_t dispatch_n(int n, F&& f) {
  switch (n) {
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_forward(const PatArgs& a, hipStream_t s) {
  if (!a.far || !a.obj || !a.probe || !a.pos) return hipErrorInvalidValue;
  if (a.N == 256) return launch_forward256(a, s);
  return dispatch_n(a.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    hipLaunchKernelGGL(k_forward<N>, dim3(pattern_blocks<N>(a.K)), dim3(Geo<N>::WG), 0, s, a);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint(const PatArgs& a, hipStream_t s) {
  if (!a.ubuf || !a.far || !a.pos) return hipErrorInvalidValue;
  if (a.N == 256) return launch_adjoint256(a, s);
  return dispatch_n(a.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    hipLaunchKernelGGL(k_adjoint<N>, dim3(pattern_blocks<N>(a.K)), dim3(Geo<N>::WG), 0, s, a);
    return hipGetLastError();
  });
}

// Calls f with std::integral_constant<bool, b>.
template <typename F>
hipError_t dispatch_bool(bool b, F&& f) {
  return b ? f(std::integral_constant<bool, true>{}) : f(std::integral_constant<bool, false>{});
}

// n <= 128: the intensities are read in the row layout (a lane's four
// consecutive frequencies are one 16-byte load); n = 256 takes either.
hipError_t launch_grad(const PatArgs& a, DataLayout lay, int* blocks_out, hipStream_t s) {
  if (!a.ubuf || !a.data || !a.partials || !a.obj || !a.probe || !a.pos) return hipErrorInvalidValue;
  if (a.N == 256) return launch_grad256(a, lay, blocks_out, s);
  if (lay != DataLayout::Rows) return hipErrorInvalidValue;
  return dispatch_n(a.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    constexpr DataLayout R = DataLayout::Rows;
    const int nb = pattern_blocks<N>(a.K);
    if (blocks_out) *blocks_out = nb;
    const dim3 g(nb), b(Geo<N>::WG);
    return dispatch_est(a.est, [&](auto ec) {
      constexpr int E = decltype(ec)::value;
      return dispatch_bool(a.want_f != 0, [&](auto wc) {
        constexpr bool WF = decltype(wc)::value;
        if (a.gstore && a.cseg) {
          if constexpr (N == 128) hipLaunchKernelGGL((k_grad<N, R, true, E, true, false, WF>), g, b, 0, s, a);
          else return hipErrorInvalidValue;
        } else if (a.gstore) {
          hipLaunchKernelGGL((k_grad<N, R, true, E, false, false, WF>), g, b, 0, s, a);
        } else {
          hipLaunchKernelGGL((k_grad<N, R, false, E, false, false, WF>), g, b, 0, s, a);
        }
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_grad_far(const PatArgs& a, int* blocks_out, hipStream_t s) {
  if (!a.ubuf || !a.far || !a.data || !a.partials || !a.probe || !a.pos) return hipErrorInvalidValue;
  if (a.N == 256) return launch_grad_far256(a, blocks_out, s);
  return dispatch_n(a.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    const int nb = pattern_blocks<N>(a.K);
    if (blocks_out) *blocks_out = nb;
    return dispatch_est(a.est, [&](auto ec) {
      constexpr int E = decltype(ec)::value;
      hipLaunchKernelGGL((k_grad<N, DataLayout::Rows, false, E, false, true>), dim3(nb), dim3(Geo<N>::WG), 0, s, a);
      return hipGetLastError();
    });
  });
}

hipError_t launch_fwd_t(const PatArgs& a, bool lin, hipStream_t s) {
  if (!a.far || !a.obj || !a.probe || !a.pos) return hipErrorInvalidValue;
  if (lin && (!a.dobj || !a.dprobe)) return hipErrorInvalidValue;
  const bool zs = a.zs_part != nullptr;
  if (zs && !a.zs_p) return hipErrorInvalidValue;
  if (a.cseg && a.N == 128) {
    if (zs) return hipErrorInvalidValue;
    const dim3 g(pattern_blocks<128>(a.K)), b(Geo<128>::WG);
    if (lin) hipLaunchKernelGGL((k_fwd_t<128, true, 0, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_fwd_t<128, false, 0, true>), g, b, 0, s, a);
    return hipGetLastError();
  }
  if (a.cseg && a.N != 256) return hipErrorInvalidValue;
  if (a.N == 256) return launch_fwd_t256(a, lin, s);
  return dispatch_n(a.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    const dim3 g(pattern_blocks<N>(a.K)), b(Geo<N>::WG);
    const int z = zs ? (a.zs_q ? 2 : 1) : 0;
    if (lin) {
      if (z == 1) hipLaunchKernelGGL((k_fwd_t<N, true, 1>), g, b, 0, s, a);
      else if (z == 2) hipLaunchKernelGGL((k_fwd_t<N, true, 2>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_fwd_t<N, true, 0>), g, b, 0, s, a);
    } else {
      if (z == 1) hipLaunchKernelGGL((k_fwd_t<N, false, 1>), g, b, 0, s, a);
      else if (z == 2) hipLaunchKernelGGL((k_fwd_t<N, false, 2>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_fwd_t<N, false, 0>), g, b, 0, s, a);
    }
    return hipGetLastError();
  });
}

int fwd_t_blocks(int N, int K) {
  if (N == 256) return fwd_t256_blocks(K);
  int nb = 0;
  dispatch_n(N, [&](auto nc) {
    nb = pattern_blocks<decltype(nc)::value>(K);
    return hipSuccess;
  });
  return nb;
}

hipError_t launch_nz_count(const float* d, int64_t n, int* counts, int* offsets, hipStream_t s) {
  if (!d || !counts || !offsets || n < 1) return hipErrorInvalidValue;
  const int64_t blocks = (n + kNzChunk - 1) / kNzChunk;
  if (blocks > (1 << 30)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_nz_count, dim3((unsigned)blocks), dim3(256), 0, s, d, n, counts);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, (int)blocks, offsets, 0);
  return hipGetLastError();
}

hipError_t launch_nz_fill(const float* d, int64_t n, const int* offsets, int* idx, uint2* seg, float* dc,
                          hipStream_t s) {
  if (!d || !offsets || !idx || n < 1) return hipErrorInvalidValue;
  if (seg && n % 32) return hipErrorInvalidValue;
  const int64_t blocks = (n + kNzChunk - 1) / kNzChunk;
  if (blocks > (1 << 30)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_nz_fill, dim3((unsigned)blocks), dim3(256), 0, s, d, n, offsets, idx, seg, dc);
  return hipGetLastError();
}

// Number of elements with !(d <= 0), accumulated into *out (zeroed first).
__global__ __launch_bounds__(256) void k_count_listed(const float* __restrict__ d, int64_t n,
                                                       unsigned long long* out) {
  __shared__ unsigned long long red[4];
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    c += !(d[i] <= 0.0f) ? 1ull : 0ull;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, red[0] + red[1] + red[2] + red[3]);
}

__global__ void k_zero_u64(unsigned long long* x) { *x = 0ull; }

hipError_t launch_count_listed(const float* d, int64_t n, unsigned long long* out, hipStream_t s) {
  if (!d || !out || n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, out);
  const int64_t want = (n + 255) / 256;
  const int nb = (int)(want < 2048 ? want : 2048);
  hipLaunchKernelGGL(k_count_listed, dim3(nb), dim3(256), 0, s, d, n, out);
  return hipGetLastError();
}

hipError_t launch_nz_compact(const float* d, int64_t n, int* counts, int* offsets, int* idx, uint2* seg,
                             float* dc, hipStream_t s) {
  if (!d || !counts || !offsets || !idx || n < 1) return hipErrorInvalidValue;
  if (seg && n % 32) return hipErrorInvalidValue;
  const int64_t blocks = (n + kNzChunk - 1) / kNzChunk;
  if (blocks > (1 << 30)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_nz_count, dim3((unsigned)blocks), dim3(256), 0, s, d, n, counts);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, (int)blocks, offsets, 0);
  hipLaunchKernelGGL(k_nz_fill, dim3((unsigned)blocks), dim3(256), 0, s, d, n, offsets, idx, seg, dc);
  return hipGetLastError();
}

hipError_t launch_ls_batch(const LsArgs& a, int* blocks_out, hipStream_t s) {
  if (!a.A || !a.B || !a.d || (!a.idx && !a.compact) || !a.partials || a.n < 0 || a.J < 1 || a.J > kLsBatch)
    return hipErrorInvalidValue;
  const int64_t want = (a.n + 255) / 256;
  const int nb = (int)(want < 1 ? 1 : (want < kLsBlocks ? want : kLsBlocks));
  if (blocks_out) *blocks_out = nb;
  return dispatch_est(a.est, [&](auto ec) {
    constexpr int E = decltype(ec)::value;
    if (a.compact && a.C) hipLaunchKernelGGL((k_ls_batch<true, E, true>), dim3(nb), dim3(256), 0, s, a);
    else if (a.compact) hipLaunchKernelGGL((k_ls_batch<false, E, true>), dim3(nb), dim3(256), 0, s, a);
    else if (a.C) hipLaunchKernelGGL((k_ls_batch<true, E, false>), dim3(nb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_ls_batch<false, E, false>), dim3(nb), dim3(256), 0, s, a);
    return hipGetLastError();
  });
}

int patch_sums_blocks(int K, int N) {
  const int64_t chunks = (int64_t)K * ((N * N + kPsChunk - 1) / kPsChunk);
  return (int)(chunks < kPsMaxBlocks ? chunks : kPsMaxBlocks);
}

hipError_t launch_patch_sums(const float2* obj, const float2* eta, const float2* probe, const float2* eta_p,
                             const int2* pos, int K, int W, int N, double* parts1, double* parts2, hipStream_t s) {
  if (!obj || !eta || !probe || !eta_p || !pos || !parts1 || !parts2 || K < 1 || N < 1 || (N & (N - 1)))
    return hipErrorInvalidValue;
  int lg = 0;
  while ((1 << lg) < N) ++lg;
  hipLaunchKernelGGL(k_patch_sums, dim3(patch_sums_blocks(K, N)), dim3(256), 0, s, obj, eta, probe, eta_p, pos, K,
                     W, lg, parts1, parts2);
  return hipGetLastError();
}

hipError_t launch_ls_accept(double* sc, const double* zs, const double* row, double* out, const LsAccept& a,
                            hipStream_t s) {
  if (!sc || !zs || !row || !out || a.J < 1 || a.J > kLsBatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ls_accept, dim3(1), dim3(64), 0, s, sc, zs, row, out, a);
  return hipGetLastError();
}

hipError_t launch_ls_finalize(const double* partials, int count, double* out, hipStream_t s) {
  if (!partials || !out || count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ls_finalize, dim3(kLsRow), dim3(256), 0, s, partials, count, out);
  return hipGetLastError();
}

hipError_t launch_minfunc(const PatArgs& a, DataLayout lay, int* blocks_out, hipStream_t s) {
  if (!a.data || !a.partials || !a.obj || !a.probe || !a.pos) return hipErrorInvalidValue;
  if (a.N == 256) return launch_minfunc256(a, lay, blocks_out, s);
  if (lay != DataLayout::Rows) return hipErrorInvalidValue;
  return dispatch_n(a.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    const int nb = pattern_blocks<N>(a.K);
    if (blocks_out) *blocks_out = nb;
    const dim3 g(nb), b(Geo<N>::WG);
    const bool lo = a.dobj != nullptr, lp = a.dprobe != nullptr;
    return dispatch_est(a.est, [&](auto ec) {
      constexpr int E = decltype(ec)::value;
      return dispatch_bool(a.want_f != 0, [&](auto wc) {
        constexpr bool WF = decltype(wc)::value;
        constexpr DataLayout R = DataLayout::Rows;
        if (lo && lp) hipLaunchKernelGGL((k_minfunc<N, R, true, true, E, WF>), g, b, 0, s, a);
        else if (lo) hipLaunchKernelGGL((k_minfunc<N, R, true, false, E, WF>), g, b, 0, s, a);
        else if (lp) hipLaunchKernelGGL((k_minfunc<N, R, false, true, E, WF>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_minfunc<N, R, false, false, E, WF>), g, b, 0, s, a);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_transpose_data(const float* d, float* dt, int K, int N, hipStream_t s) {
  if (N >= 32) {
    hipLaunchKernelGGL(k_transpose_data, dim3(N / 32, N / 32, K), dim3(256), 0, s, d, dt, N);
  } else {
    const int64_t tot = (int64_t)K * N * N;
    hipLaunchKernelGGL(k_transpose_data_small, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, d, dt, K,
                       N);
  }
  return hipGetLastError();
}

hipError_t launch_debug_gather(const PatArgs& a, float2* patches, hipStream_t s) {
  if (a.N == 256) {
    const int64_t tot = (int64_t)a.K * a.N * a.N;
    hipLaunchKernelGGL(k_debug_gather_any, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a, patches);
    return hipGetLastError();
  }
  return dispatch_n(a.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    hipLaunchKernelGGL(k_debug_gather<N>, dim3(pattern_blocks<N>(a.K)), dim3(Geo<N>::WG), 0, s, a, patches);
    return hipGetLastError();
  });
}

hipError_t launch_debug_scatter(const PatArgs& a, const float2* patches, hipStream_t s) {
  if (a.N == 256) {
    const int64_t tot = (int64_t)a.K * a.N * a.N;
    hipLaunchKernelGGL(k_debug_scatter_any, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a, patches);
    return hipGetLastError();
  }
  return dispatch_n(a.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    hipLaunchKernelGGL(k_debug_scatter<N>, dim3(pattern_blocks<N>(a.K)), dim3(Geo<N>::WG), 0, s, a, patches);
    return hipGetLastError();
  });
}

hipError_t launch_check_positions(const int2* pos, int K, int H, int W, int N, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_positions, dim3((K + 255) / 256), dim3(256), 0, s, pos, K, H, W, N, flag);
  return hipGetLastError();
}

hipError_t launch_debug_lane_swap(float* a, float* b, hipStream_t s) {
  hipLaunchKernelGGL(k_debug_lane_swap, dim3(1), dim3(64), 0, s, a, b);
  return hipGetLastError();
}

hipError_t launch_tile_lists(const int2* pos, int K, int H, int W, int N, int* offsets, int* list, hipStream_t s) {
  const int T = tiles_x(W) * tiles_y(H);
  // the T counters (then cursors) sit after the list's capacity
  int* counts = list + (tile_list_ints(K, H, W, N) - (size_t)T);
  // candidate tiles per patch: a (N - 1) / kTileH + 2 by (N - 1) / kTileW + 2 span
  const int span_x = (N - 1) / kTileW + 2, tpp = tiles_per_patch(N);
  const int64_t pairs = (int64_t)K * tpp;
  const unsigned pb = (unsigned)((pairs + 255) / 256);
  if (hipError_t e = launch_fill_i32(counts, T, 0, s)) return e;
  hipLaunchKernelGGL(k_tile_count_k, dim3(pb), dim3(256), 0, s, pos, pairs, tpp, span_x, H, W, N, counts);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, T, offsets, 1);  // also zeroes the cursor
  hipLaunchKernelGGL(k_tile_fill_k, dim3(pb), dim3(256), 0, s, pos, pairs, tpp, span_x, H, W, N, offsets, counts,
                     list);
  hipLaunchKernelGGL(k_tile_sort, dim3(T), dim3(256), 0, s, pos, K, W, N, offsets, list);
  return hipGetLastError();
}

hipError_t launch_tile_sum(const float2* ubuf, const float2* probe, const int2* pos, const int* offsets,
                           const int* list, int K, int H, int W, int N, float2* out, hipStream_t s,
                           const float2* dot_b, double* dot_parts) {
  (void)K;
  const int T = tiles_x(W) * tiles_y(H);
  const int64_t us = (int64_t)N * N;
  if (N == 256) {
    if (!probe) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_tile_sum<true, true>), dim3(T), dim3(256), 0, s, ubuf, probe, pos, offsets, list, H, W, N,
                       us, out, dot_b, dot_parts);
  } else if (probe) {
    hipLaunchKernelGGL((k_tile_sum<false, true>), dim3(T), dim3(256), 0, s, ubuf, probe, pos, offsets, list, H, W,
                       N, us, out, dot_b, dot_parts);
  } else {
    hipLaunchKernelGGL((k_tile_sum<false, false>), dim3(T), dim3(256), 0, s, ubuf, probe, pos, offsets, list, H, W,
                       N, us, out, dot_b, dot_parts);
  }
  return hipGetLastError();
}

hipError_t launch_illum(const float2* probe, const int2* pos, const int* offsets, const int* list, int H, int W,
                        int N, float2* out, hipStream_t s) {
  if (!probe || !pos || !offsets || !list || !out) return hipErrorInvalidValue;
  const int T = tiles_x(W) * tiles_y(H);
  // every pattern's "u_k" is the probe itself (stride 0): sum conj(p) p
  hipLaunchKernelGGL((k_tile_sum<false, true>), dim3(T), dim3(256), 0, s, probe, probe, pos, offsets, list, H, W, N,
                     (int64_t)0, out, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_probe_grad(const float2* ubuf, const float2* obj, const int2* pos, int K, int W, int N,
                             float2* partial, float2* out, hipStream_t s) {
  const int nn = N * N;
  if (N == 256)
    hipLaunchKernelGGL(k_probe_partial<true>, dim3((nn + 255) / 256, kProbeChunks), dim3(256), 0, s, ubuf, obj, pos,
                       K, W, N, partial);
  else
    hipLaunchKernelGGL(k_probe_partial<false>, dim3((nn + 255) / 256, kProbeChunks), dim3(256), 0, s, ubuf, obj, pos,
                       K, W, N, partial);
  hipLaunchKernelGGL(k_probe_reduce, dim3((nn + 255) / 256), dim3(256), 0, s, partial, nn, out);
  return hipGetLastError();
}

int patterns_per_block(int N) {
  int ppw = 0;
  dispatch_n(N, [&](auto nc) {
    ppw = Geo<decltype(nc)::value>::PPW;
    return hipSuccess;
  });
  return ppw;
}

hipError_t launch_finalize_views(const double* partials, int N, int K, int k_per_view, int views, int width,
                                 double* out, hipStream_t s) {
  if (!partials || !out || N > 128 || views < 1 || k_per_view < 1 || width < 1 || width > 4)
    return hipErrorInvalidValue;
  int nb = 0, groups = 0, ppw = 0;
  hipError_t e = dispatch_n(N, [&](auto nc) {
    constexpr int NN = decltype(nc)::value;
    ppw = Geo<NN>::PPW;
    groups = (K + ppw - 1) / ppw;
    nb = pattern_blocks<NN>(K);
    return hipSuccess;
  });
  if (e != hipSuccess) return e;
  if (k_per_view % ppw) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finalize_views, dim3(views), dim3(256), 0, s, partials, nb, groups, ppw, k_per_view, width,
                     out);
  return hipGetLastError();
}

hipError_t launch_data_const(const float* d, int64_t n, int segs, double* partials, double* out, hipStream_t s) {
  if (!d || !partials || !out || n < 1 || segs < 1) return hipErrorInvalidValue;
  // one segment (a whole solve's data): enough blocks to fill the chip, at
  // most kVecMaxBlocks partials; several segments: kSegBlocks each
  int nb = kSegBlocks;
  if (segs == 1) {
    const int64_t want = n / ((int64_t)kVecWG * 32);
    nb = (int)(want < 1 ? 1 : (want > kVecMaxBlocks ? kVecMaxBlocks : want));
  }
  hipLaunchKernelGGL(k_data_const, dim3(nb, segs), dim3(kVecWG), 0, s, d, n, partials);
  if (hipError_t e = hipGetLastError()) return e;
  return launch_finalize_seg(partials, nb, 1, segs, out, s);
}

hipError_t launch_dot2_views(const float2* a, const float2* b, int64_t n, int views, double* partials,
                             hipStream_t s) {
  if (!a || !partials || n < 1 || views < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dot2_views, dim3(kSegBlocks, views), dim3(kVecWG), 0, s, a, b, n, partials);
  return hipGetLastError();
}

hipError_t launch_dir_views(const float2* a, float2* b, const double* beta, int64_t n, int views,
                            double* partials, hipStream_t s) {
  if (!a || !b || !beta || !partials || n < 1 || views < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dir_views, dim3(kSegBlocks, views), dim3(kVecWG), 0, s, a, b, beta, n, partials);
  return hipGetLastError();
}

hipError_t launch_axpy_views(float2* a, const float2* c, const double* alpha, int64_t n, int views,
                             hipStream_t s) {
  if (!a || !c || !alpha || n < 1 || views < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_axpy_views, dim3(kSegBlocks, views), dim3(kVecWG), 0, s, a, c, alpha, n);
  return hipGetLastError();
}

hipError_t launch_finalize_seg(const double* partials, int rows, int width, int views, double* out,
                               hipStream_t s) {
  if (!partials || !out || rows < 1 || width < 1 || width > 4 || views < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finalize_seg, dim3(views), dim3(256), 0, s, partials, rows, width, out);
  return hipGetLastError();
}

hipError_t launch_ls_batch_views(const LsArgs& a, const int* offsets, int chunks_per_view, int views,
                                 hipStream_t s) {
  if (!a.A || !a.B || !a.d || !a.idx || !a.partials || !offsets || a.J < 1 || a.J > kLsBatch || views < 1)
    return hipErrorInvalidValue;
  return dispatch_est(a.est, [&](auto ec) {
    constexpr int E = decltype(ec)::value;
    const dim3 g(kSegBlocks, views), b(256);
    if (a.C) hipLaunchKernelGGL((k_ls_batch_views<true, E>), g, b, 0, s, a, offsets, chunks_per_view);
    else hipLaunchKernelGGL((k_ls_batch_views<false, E>), g, b, 0, s, a, offsets, chunks_per_view);
    return hipGetLastError();
  });
}

hipError_t launch_ls_finalize_views(const double* partials, int views, double* out, hipStream_t s) {
  if (!partials || !out || views < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ls_finalize_views, dim3(kLsRow, views), dim3(256), 0, s, partials, out);
  return hipGetLastError();
}

hipError_t launch_shift_views(const int2* pos, int k, int kp, int views, int rows_per_view, int pad_row, int2* out,
                              hipStream_t s) {
  if (!pos || !out || k < 1 || kp < k || views < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_shift_views, dim3((kp * views + 255) / 256), dim3(256), 0, s, pos, k, kp, views, rows_per_view,
                     pad_row, out);
  return hipGetLastError();
}

int vec_blocks(int64_t n) {
  const int64_t nb = (n + kVecWG * 4 - 1) / (kVecWG * 4);
  return (int)(nb < 1 ? 1 : (nb > kVecMaxBlocks ? kVecMaxBlocks : nb));
}

hipError_t launch_zero(float2* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(vec_blocks(n)), dim3(kVecWG), 0, s, x, n);
  return hipGetLastError();
}
hipError_t launch_zero_f64(double* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f64, dim3(vec_blocks(n)), dim3(kVecWG), 0, s, x, n);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* x, int64_t n, int value, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(vec_blocks(n)), dim3(kVecWG), 0, s, x, n, value);
  return hipGetLastError();
}
hipError_t launch_dot2(const VecArgs& v, hipStream_t s) {
  hipLaunchKernelGGL(k_dot2, dim3(vec_blocks(v.n)), dim3(kVecWG), 0, s, v);
  return hipGetLastError();
}
hipError_t launch_dir(const VecArgs& v, hipStream_t s) {
  hipLaunchKernelGGL(k_dir, dim3(vec_blocks(v.n)), dim3(kVecWG), 0, s, v);
  return hipGetLastError();
}
hipError_t launch_axpy(const VecArgs& v, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(vec_blocks(v.n)), dim3(kVecWG), 0, s, v);
  return hipGetLastError();
}
hipError_t launch_sum_copies(const float2* src, int copies, int64_t n, float2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_copies, dim3(vec_blocks(n)), dim3(kVecWG), 0, s, src, copies, n, out);
  return hipGetLastError();
}
hipError_t launch_dy_beta(double* sc, int n1, int n2, int n3, int joint_off, int beta, int rst, int restart,
                          hipStream_t s) {
  if (!sc) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dy_beta, dim3(1), dim3(64), 0, s, sc, n1, n2, n3, joint_off, beta, rst, restart);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int count, int width, double* out, hipStream_t s) {
  const FinJob j{partials, count, width, out};
  return launch_finalize2(j, j, 1, s);
}

hipError_t launch_finalize2(const FinJob& a, const FinJob& b, int jobs, hipStream_t s) {
  if (jobs < 1 || jobs > 2) return hipErrorInvalidValue;
  const FinJob js[2] = {a, b};
  return launch_finalize_n(js, jobs, s);
}

hipError_t launch_finalize_n(const FinJob* jobs, int n, hipStream_t s) {
  if (!jobs || n < 1 || n > 4) return hipErrorInvalidValue;
  FinJobs all{};
  for (int i = 0; i < n; ++i) {
    const FinJob& j = jobs[i];
    if (!j.p || !j.out || j.count < 1 || j.width < 1 || j.width > 4) return hipErrorInvalidValue;
    all.j[i] = j;
  }
  hipLaunchKernelGGL(k_finalize, dim3(n), dim3(256), 0, s, all);
  return hipGetLastError();
}

}  // namespace ptyg
