// Per-pattern 2-D transform pipeline: thread layout, line transforms and the
// LDS transposes between the column axis and the row axis.
//
// Layouts (N x N pattern, "line" = column index in the column layout and row
// index in the row layout, both coalesced for row-major global arrays):
//   column layout  : lane owns column `line`; slot m holds row u = m*TPC + h.
//   row layout     : lane owns row `line`;    slot m holds col b = m*TPC + h.
//   after a forward line transform, slot s holds frequency fidx(s, h).
// N <= 64: one lane per line (TPC = 1), several patterns per workgroup.
// N = 128: two lanes per line (TPC = 2, lanes l and l+32, h = l >> 5),
//          64 values per lane, one pattern per 256-thread workgroup.
#pragma once
#include "fft.hpp"

namespace ptyg {

template <int N>
struct Geo {
  static_assert(N == 16 || N == 32 || N == 64 || N == 128, "unsupported probe size");
  static constexpr int TPC = (N == 128) ? 2 : 1;   // lanes per line
  static constexpr int E = N / TPC;                // values per lane
  static constexpr int TPP = N * TPC;              // threads per pattern
  static constexpr int WG = (N == 64) ? 128 : 256; // threads per workgroup
  static constexpr int PPW = WG / TPP;             // patterns per workgroup
  static constexpr int PITCH = N + 1;              // LDS row pitch (complex)
  // N = 128 transposes half the rows at a time (two phases).
  static constexpr int LDS_ELEMS = (TPC == 2) ? (N / 2) * PITCH : PPW * N * PITCH;
  // workgroups per CU allowed by 160 KiB of LDS, as waves per SIMD
  static constexpr int WG_PER_CU = (160 * 1024) / (LDS_ELEMS * 8 + 256);
  static constexpr int WAVES_PER_EU_RAW = WG_PER_CU * (WG / 64) / 4;
  static constexpr int WAVES_PER_EU = WAVES_PER_EU_RAW < 1 ? 1 : (WAVES_PER_EU_RAW > 8 ? 8 : WAVES_PER_EU_RAW);
};

struct Lane {
  int line;   // column (column layout) or row (row layout) within the pattern
  int pslot;  // pattern slot within the workgroup
  bool h;     // which half of a split line (TPC = 2)
};

template <int N>
__device__ __forceinline__ Lane lane_info() {
  const int t = threadIdx.x;
  if constexpr (Geo<N>::TPC == 2) {
    const int w = t >> 6, l = t & 63;
    return {32 * w + (l & 31), 0, (l >> 5) != 0};
  } else {
    return {t % N, t / N, false};
  }
}

// Frequency of each slot after a forward line transform, without the
// run-time half offset (added by fidx).
template <int N>
struct FreqTable {
  int f[Geo<N>::E];
  constexpr FreqTable() : f() {
    constexpr int E = Geo<N>::E;
    for (int s = 0; s < E; ++s) {
      const int k = freq_of_slot(E, s);
      f[s] = (Geo<N>::TPC == 1) ? k : (k < E / 2 ? k : k + E / 2);
    }
  }
};
template <int N>
inline constexpr FreqTable<N> kFreq{};

// Slots in ascending order of their base frequency: the residual loops take
// pixels in this order, four at a time, so a chunk's intensity loads in the
// row layout (one row per lane) fall in one cache line per lane.
template <int N>
struct SlotOrder {
  int s[Geo<N>::E];
  constexpr SlotOrder() : s() {
    for (int i = 0; i < Geo<N>::E; ++i) s[i] = slot_of_freq(Geo<N>::E, i);
  }
};
template <int N>
inline constexpr SlotOrder<N> kOrd{};

template <int N>
__device__ __forceinline__ int fidx(int s, bool h) {
  if constexpr (Geo<N>::TPC == 1) return kFreq<N>.f[s];
  else return kFreq<N>.f[s] + (h ? Geo<N>::E / 2 : 0);
}
template <int N>
__device__ __forceinline__ int sidx(int m, bool h) {
  return m * Geo<N>::TPC + (h ? 1 : 0);
}

// Forward / inverse unnormalised 1-D transform of the lane's line(s).
template <int N>
__device__ __forceinline__ void fwd_line(float2* v, bool h) {
  constexpr int E = Geo<N>::E;
  dif<-1, E>(v);
  if constexpr (Geo<N>::TPC == 2) xlane_fwd<-1, E>(v, h);
}
template <int N>
__device__ __forceinline__ void inv_line(float2* v, bool h) {
  constexpr int E = Geo<N>::E;
  if constexpr (Geo<N>::TPC == 2) xlane_adj<+1, E>(v, h);
  dit<+1, E>(v);
}

// Column-layout frequency slots -> row-layout spatial slots.
template <int N>
__device__ __forceinline__ void transpose_c2r(float2* v, float2* lds, const Lane& L) {
  using G = Geo<N>;
  constexpr int E = G::E, P = G::PITCH;
  if constexpr (G::TPC == 1) {
    float2* base = lds + L.pslot * N * P;
#pragma unroll
    for (int s = 0; s < E; ++s) base[fidx<N>(s, false) * P + L.line] = v[s];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = base[L.line * P + m];
    __syncthreads();
  } else {
    // phase 0: rows [0, N/2) = slots whose base frequency is < E/2
    float2 tmp[E / 2];
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int f = kFreq<N>.f[s];
      if (f < E / 2) lds[(f + (L.h ? E / 2 : 0)) * P + L.line] = v[s];
      else tmp[f - E] = v[s];
    }
    __syncthreads();
    if (L.line < N / 2) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = lds[L.line * P + sidx<N>(m, L.h)];
    }
    __syncthreads();
    // phase 1: rows [N/2, N)
#pragma unroll
    for (int j = 0; j < E / 2; ++j) lds[(j + (L.h ? E / 2 : 0)) * P + L.line] = tmp[j];
    __syncthreads();
    if (L.line >= N / 2) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = lds[(L.line - N / 2) * P + sidx<N>(m, L.h)];
    }
    __syncthreads();
  }
}

// Row-layout spatial slots -> column-layout frequency slots (mirror of c2r).
template <int N>
__device__ __forceinline__ void transpose_r2c(float2* v, float2* lds, const Lane& L) {
  using G = Geo<N>;
  constexpr int E = G::E, P = G::PITCH;
  if constexpr (G::TPC == 1) {
    float2* base = lds + L.pslot * N * P;
#pragma unroll
    for (int m = 0; m < E; ++m) base[L.line * P + m] = v[m];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < E; ++s) v[s] = base[fidx<N>(s, false) * P + L.line];
    __syncthreads();
  } else {
    float2 tmp[E / 2];
    if (L.line < N / 2) {
#pragma unroll
      for (int m = 0; m < E; ++m) lds[L.line * P + sidx<N>(m, L.h)] = v[m];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E / 2; ++j) tmp[j] = lds[(j + (L.h ? E / 2 : 0)) * P + L.line];
    __syncthreads();
    if (L.line >= N / 2) {
#pragma unroll
      for (int m = 0; m < E; ++m) lds[(L.line - N / 2) * P + sidx<N>(m, L.h)] = v[m];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int f = kFreq<N>.f[s];
      if (f < E / 2) v[s] = tmp[f];
      else v[s] = lds[(f - E + (L.h ? E / 2 : 0)) * P + L.line];
    }
    __syncthreads();
  }
}

// Workgroup -> pattern group, XCD-aware: workgroups are dispatched round-robin
// over the 8 XCDs, so workgroup b runs on XCD b % 8.  Each XCD is given a
// contiguous range of pattern groups; with a raster scan in row-major order
// neighbouring patches (which share object rows in L2) stay on one XCD.
__device__ __forceinline__ int group_of_block(int b, int groups) {
  const int x = b & 7, i = b >> 3;
  const int q = groups >> 3, r = groups & 7;
  const int cnt = q + (x < r ? 1 : 0);
  if (i >= cnt) return -1;
  return x * q + (x < r ? x : r) + i;
}
inline int blocks_for_groups(int groups) { return 8 * ((groups + 7) / 8); }

}  // namespace ptyg
