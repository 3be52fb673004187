// Learned CG warm start: HIP kernels of a small convolutional
// encoder-decoder (BF16 operands on MFMA, FP32 accumulation), its training
// (backward data / weight, Adam) and the stitching of predicted object
// patches into a CG starting guess.
//
// Tensors are NHWC with the channel count padded to a multiple of 8 (Cp);
// padded channels hold zeros.  A 3x3 convolution (zero padding 1) is an
// implicit GEMM:
//   forward      y[p][co]  = sum_{t, ci} w[co][t Cp_in + ci] x[p + o(t)][ci]
//   backward x   dx[p][ci] = sum_{t, co} wT[ci][t Cp_out + co] dz[p - o(t)][co]
//   backward w   dw[co][t Cp_in + ci] = sum_p dz[p][co] x[p + o(t)][ci]
// with o(t) = (t / 3 - 1, t % 3 - 1).  The GEMM core runs
// v_mfma_f32_16x16x32_bf16 from LDS-staged tiles: a 256-thread workgroup
// computes a BM x BN output tile (shape chosen by the problem), each wave a
// quarter of it, K in steps of 32; every operand fragment is 8
// consecutive-K bf16 values per lane.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <type_traits>

#include "../../include/ptyg_nn.h"
#include "fft.hpp"
#include "kernels.hpp"

namespace ptyg {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 z;
#pragma unroll
  for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
  return z;
}
__device__ __forceinline__ bf16x8 load8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

struct Geom {
  int B, H, W;  // images, rows, cols (output grid of the convolution)
  int P;        // B * H * W
};

__device__ __forceinline__ void pix(const Geom& g, int p, int& n, int& y, int& x) {
  n = p / (g.H * g.W);
  const int r = p - n * g.H * g.W;
  y = r / g.W;
  x = r - y * g.W;
}

// ---------------------------------------------------------------- loaders
struct FwdA {  // A[m = p][k = t Cpi + ci] = x[p + o(t)][ci]
  const __bf16* x;
  Geom g;
  int cpi;
  __device__ bf16x8 operator()(int m, int k) const {
    if (m >= g.P || k >= 9 * cpi) return zero8();
    const int t = k / cpi, ci = k - t * cpi;
    int n, y, xx;
    pix(g, m, n, y, xx);
    y += t / 3 - 1;
    xx += t % 3 - 1;
    if (y < 0 || y >= g.H || xx < 0 || xx >= g.W) return zero8();
    return load8(x + (((size_t)n * g.H + y) * g.W + xx) * cpi + ci);
  }
};
struct RowB {  // B[n][k] = w[n * ld + k], rows n < rows
  const __bf16* w;
  int rows, ld;
  __device__ bf16x8 operator()(int n, int k) const {
    if (n >= rows || k >= ld) return zero8();
    return load8(w + (size_t)n * ld + k);
  }
};
struct BwdA {  // A[m = p][k = t Cpo + co] = dz[p - o(t)][co]
  const __bf16* dz;
  Geom g;
  int cpo;
  __device__ bf16x8 operator()(int m, int k) const {
    if (m >= g.P || k >= 9 * cpo) return zero8();
    const int t = k / cpo, co = k - t * cpo;
    int n, y, xx;
    pix(g, m, n, y, xx);
    y -= t / 3 - 1;
    xx -= t % 3 - 1;
    if (y < 0 || y >= g.H || xx < 0 || xx >= g.W) return zero8();
    return load8(dz + (((size_t)n * g.H + y) * g.W + xx) * cpo + co);
  }
};
struct WgtA {  // A[m = co][k = p] = dzT[co][p]
  const __bf16* dzt;
  int rows, P;
  __device__ bf16x8 operator()(int m, int k) const {
    if (m >= rows || k >= P) return zero8();
    return load8(dzt + (size_t)m * P + k);
  }
};
struct WgtB {  // B[n = t Cpi + ci][k = p] = x[p + o(t)][ci]  (8 gathered pixels)
  const __bf16* x;
  Geom g;
  int cpi;
  __device__ bf16x8 operator()(int nn, int k) const {
    bf16x8 r = zero8();
    if (nn >= 9 * cpi || k >= g.P) return r;
    const int t = nn / cpi, ci = nn - t * cpi;
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    // the 8 pixels k..k+7 lie in one image row when W is a multiple of 8;
    // otherwise each is decomposed on its own
    int n, y, x0;
    pix(g, k, n, y, x0);
    y += dy;
    const bool row = (g.W & 7) == 0;
    if (row && (y < 0 || y >= g.H)) return r;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      int nj = n, yj = y, xj = x0 + j + dx;
      if (!row) {
        if (k + j >= g.P) continue;
        pix(g, k + j, nj, yj, xj);
        yj += dy;
        xj += dx;
        if (yj < 0 || yj >= g.H) continue;
      }
      if (xj >= 0 && xj < g.W) r[j] = x[(((size_t)nj * g.H + yj) * g.W + xj) * cpi + ci];
    }
    return r;
  }
};

// ----------------------------------------------------------------- stores
struct ConvStore {  // y[p][co] = act(acc + b[co]); padded channels get 0
  void* y;
  const float* bias;
  int P, cout, cpo, relu, f32;
  __device__ void operator()(int m, int n, float v) const {
    if (m >= P || n >= cpo) return;
    float r = 0.0f;
    if (n < cout) {
      r = v + bias[n];
      if (relu) r = fmaxf(r, 0.0f);
    }
    if (f32) static_cast<float*>(y)[(size_t)m * cpo + n] = r;
    else static_cast<__bf16*>(y)[(size_t)m * cpo + n] = (__bf16)r;
  }
};
struct DxStore {  // dx[p][ci]
  __bf16* dx;
  int P, cpi, cin;
  __device__ void operator()(int m, int n, float v) const {
    if (m >= P || n >= cpi) return;
    dx[(size_t)m * cpi + n] = (__bf16)(n < cin ? v : 0.0f);
  }
};
struct PartStore {  // partial[ks][m][n] (FP32, split-K)
  float* part;
  int M, N;
  __device__ void operator()(int m, int n, float v) const {
    if (m >= M || n >= N) return;
    part[((size_t)blockIdx.z * M + m) * N + n] = v;
  }
};

// ------------------------------------------------------------- GEMM core
// LDS-tiled MFMA GEMM: a 256-thread workgroup computes a BM x BN tile, each
// wave a (BM/2) x (BN/2) quarter as 16 x 16 MFMA blocks; K advances in steps
// of 32.  The A and B chunks of step k+1 (8 consecutive-K bf16 each, from
// the loaders) are fetched into registers while step k's fragments are read
// from LDS and multiplied.
template <int BM, int BN, class LA, class LB, class ST>
__global__ __launch_bounds__(256) void k_gemm(LA la, LB lb, ST st, int K, int kchunk) {
  constexpr int BK = 32, LDK = BK + 8;  // LDS row: 32 bf16 + 16 B of padding
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  constexpr int CA = (BM * 4 + 255) / 256, CB = (BN * 4 + 255) / 256;  // 16-byte chunks per thread
  __shared__ __attribute__((aligned(16))) __bf16 sa[BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 sb[BN * LDK];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int bm0 = blockIdx.x * BM, bn0 = blockIdx.y * BN;
  const int wm0 = (w >> 1) * WM, wn0 = (w & 1) * WN;
  const int r = l & 15, kq = (l >> 4) * 8;
  f4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  bf16x8 ra[CA], rb[CB];
  // chunk c: tile row c / 4, K offset (c % 4) * 8
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < CA; ++i) {
      const int c = tid + 256 * i;
      if (c < BM * 4) ra[i] = la(bm0 + (c >> 2), k0 + (c & 3) * 8);
    }
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      const int c = tid + 256 * i;
      if (c < BN * 4) rb[i] = lb(bn0 + (c >> 2), k0 + (c & 3) * 8);
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();  // the previous step's fragments have been read
#pragma unroll
    for (int i = 0; i < CA; ++i) {
      const int c = tid + 256 * i;
      if (c < BM * 4) *reinterpret_cast<bf16x8*>(&sa[(c >> 2) * LDK + (c & 3) * 8]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      const int c = tid + 256 * i;
      if (c < BN * 4) *reinterpret_cast<bf16x8*>(&sb[(c >> 2) * LDK + (c & 3) * 8]) = rb[i];
    }
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);
    bf16x8 fa[FM], fb[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) fa[i] = *reinterpret_cast<const bf16x8*>(&sa[(wm0 + 16 * i + r) * LDK + kq]);
#pragma unroll
    for (int j = 0; j < FN; ++j) fb[j] = *reinterpret_cast<const bf16x8*>(&sb[(wn0 + 16 * j + r) * LDK + kq]);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
  }
  // C fragment: lane l holds rows 4 (l >> 4) + e, column l & 15
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) st(bm0 + wm0 + 16 * i + 4 * (l >> 4) + e, bn0 + wn0 + 16 * j + r, acc[i][j][e]);
}

// Tile shape by problem shape: narrow outputs (N <= 32) take tall tiles.
template <class LA, class LB, class ST>
hipError_t gemm(const LA& la, const LB& lb, const ST& st, int M, int N, int K, int splits, hipStream_t s) {
  const int kpad = (K + 31) / 32 * 32;
  const int kchunk = ((kpad + splits - 1) / splits + 31) / 32 * 32;
  auto launch = [&](auto bm, auto bn) {
    constexpr int BM = decltype(bm)::value, BN = decltype(bn)::value;
    const dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, splits);
    hipLaunchKernelGGL((k_gemm<BM, BN, LA, LB, ST>), grid, dim3(256), 0, s, la, lb, st, kpad, kchunk);
  };
  if (M <= 64) launch(std::integral_constant<int, 64>{}, std::integral_constant<int, 128>{});
  else if (N <= 32) launch(std::integral_constant<int, 256>{}, std::integral_constant<int, 32>{});
  else if (N <= 64) launch(std::integral_constant<int, 128>{}, std::integral_constant<int, 64>{});
  else launch(std::integral_constant<int, 128>{}, std::integral_constant<int, 128>{});
  return hipGetLastError();
}

// ------------------------------------------------------- elementwise / misc
__global__ void k_reduce_parts(const float* part, int splits, int64_t n, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int k = 0; k < splits; ++k) s += part[(size_t)k * n + i];
  out[i] = s;
}

// db[co] = sum_p dzT[co][p] from the channel-major copy (contiguous rows):
// grid (kBiasChunks, cout), workgroup (c, co) sums its fixed pixel range
// (strided per thread, then a fixed tree) into part[co][c]; k_bias_reduce
// adds the chunks in order.
constexpr int kBiasChunks = 64;
__global__ __launch_bounds__(256) void k_bias_grad(const __bf16* dzt, int P, float* part) {
  __shared__ float red[256];
  const int c = blockIdx.x, co = blockIdx.y;
  const int per = (P + kBiasChunks - 1) / kBiasChunks;
  const int lo = c * per, hi = min(P, lo + per);
  const __bf16* row = dzt + (size_t)co * P;
  float s = 0.0f;
  for (int p = lo + threadIdx.x; p < hi; p += 256) s += (float)row[p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[co * kBiasChunks + c] = red[0];
}
__global__ void k_bias_reduce(const float* part, int cout, float* db) {
  const int co = blockIdx.x * blockDim.x + threadIdx.x;
  if (co >= cout) return;
  float s = 0.0f;
  for (int c = 0; c < kBiasChunks; ++c) s += part[co * kBiasChunks + c];
  db[co] = s;
}

// dzT[c][p] = dz[p][c]
__global__ __launch_bounds__(256) void k_transpose_pc(const __bf16* dz, int P, int cp, __bf16* dzt) {
  __shared__ __bf16 tile[32][33];
  const int p0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int j = ty; j < 32; j += 8) {
    const int p = p0 + j, c = c0 + tx;
    tile[j][tx] = (p < P && c < cp) ? dz[(size_t)p * cp + c] : (__bf16)0.0f;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int c = c0 + j, p = p0 + tx;
    if (c < cp && p < P) dzt[(size_t)c * P + p] = tile[tx][j];
  }
}

// Pack FP32 master weights w32[cout][9][cin] into w[cout][kpad] (k = t Cpi + ci)
// and wT[cpi][kpad2] (k = t Cpo + co); zero elsewhere.
__global__ void k_pack_weights(const float* w32, int cout, int cin, int cpi, int cpo, int kpad, int kpad2,
                               __bf16* w, __bf16* wt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n1 = (int64_t)cout * kpad, n2 = (int64_t)cpi * kpad2;
  if (i < n1) {
    const int co = (int)(i / kpad), k = (int)(i % kpad);
    const int t = k / cpi, ci = k - t * cpi;
    float v = 0.0f;
    if (t < 9 && ci < cin) v = w32[((size_t)co * 9 + t) * cin + ci];
    w[i] = (__bf16)v;
  } else if (i < n1 + n2) {
    const int64_t j = i - n1;
    const int ci = (int)(j / kpad2), k = (int)(j % kpad2);
    const int t = k / cpo, co = k - t * cpo;
    float v = 0.0f;
    if (t < 9 && co < cout && ci < cin) v = w32[((size_t)co * 9 + t) * cin + ci];
    wt[j] = (__bf16)v;
  }
}

// Unpack the weight gradient dwp[co][t Cpi + ci] into dw32[co][9][cin].
__global__ void k_unpack_wgrad(const float* dwp, int cout, int cin, int cpi, float* dw32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)cout * 9 * cin;
  if (i >= n) return;
  const int co = (int)(i / (9 * cin)), r = (int)(i % (9 * cin)), t = r / cin, ci = r % cin;
  dw32[i] = dwp[(size_t)co * 9 * cpi + t * cpi + ci];
}

// Elementwise layers on 8-channel (16-byte) groups: element i of the
// group index space is (pixel, channel group); all counts are multiples of 8.
__global__ void k_relu_bwd(const bf16x8* dy, const bf16x8* y, int64_t n8, bf16x8* dz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n8) return;
  const bf16x8 a = dy[i], b = y[i];
  bf16x8 r;
#pragma unroll
  for (int c = 0; c < 8; ++c) r[c] = ((float)b[c] > 0.0f) ? a[c] : (__bf16)0.0f;
  dz[i] = r;
}

// 2x2 average pooling (NHWC): out [B][H/2][W/2][cp]
__global__ void k_pool_fwd(const bf16x8* x, int B, int H, int W, int g8, bf16x8* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int Ho = H / 2, Wo = W / 2;
  if (i >= (int64_t)B * Ho * Wo * g8) return;
  const int c = (int)(i % g8);
  const int64_t q = i / g8;
  const int xo = (int)(q % Wo), yo = (int)((q / Wo) % Ho), n = (int)(q / ((int64_t)Wo * Ho));
  const size_t b = (((size_t)n * H + 2 * yo) * W + 2 * xo) * g8 + c;
  const size_t rs = (size_t)W * g8;
  const bf16x8 p0 = x[b], p1 = x[b + g8], p2 = x[b + rs], p3 = x[b + rs + g8];
  bf16x8 r;
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = (__bf16)(0.25f * ((float)p0[e] + (float)p1[e] + (float)p2[e] + (float)p3[e]));
  y[i] = r;
}
__global__ void k_pool_bwd(const bf16x8* dy, int B, int H, int W, int g8, bf16x8* dx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * H * W * g8) return;
  const int c = (int)(i % g8);
  const int64_t q = i / g8;
  const int x = (int)(q % W), y = (int)((q / W) % H), n = (int)(q / ((int64_t)W * H));
  const bf16x8 a = dy[(((size_t)n * (H / 2) + y / 2) * (W / 2) + x / 2) * g8 + c];
  bf16x8 r;
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = (__bf16)(0.25f * (float)a[e]);
  dx[i] = r;
}
// nearest 2x upsampling: out [B][2H][2W][cp]
__global__ void k_up_fwd(const bf16x8* x, int B, int H, int W, int g8, bf16x8* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int Ho = 2 * H, Wo = 2 * W;
  if (i >= (int64_t)B * Ho * Wo * g8) return;
  const int c = (int)(i % g8);
  const int64_t q = i / g8;
  const int xo = (int)(q % Wo), yo = (int)((q / Wo) % Ho), n = (int)(q / ((int64_t)Wo * Ho));
  y[i] = x[(((size_t)n * H + yo / 2) * W + xo / 2) * g8 + c];
}
__global__ void k_up_bwd(const bf16x8* dy, int B, int H, int W, int g8, bf16x8* dx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * H * W * g8) return;
  const int c = (int)(i % g8);
  const int64_t q = i / g8;
  const int x = (int)(q % W), y = (int)((q / W) % H), n = (int)(q / ((int64_t)W * H));
  const size_t Wo = 2 * (size_t)W;
  const size_t b = (((size_t)n * 2 * H + 2 * y) * Wo + 2 * x) * g8 + c;
  const bf16x8 p0 = dy[b], p1 = dy[b + g8], p2 = dy[b + Wo * g8], p3 = dy[b + Wo * g8 + g8];
  bf16x8 r;
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = (__bf16)((float)p0[e] + (float)p1[e] + (float)p2[e] + (float)p3[e]);
  dx[i] = r;
}

// Network input: x[b][u][v][0] = scale * log(1 + d[b][(u + n/2) % n][(v + n/2) % n])
// (the pattern with zero frequency moved to the centre), channels 1..7 = 0.
__global__ void k_input(const float* d, int B, int n, float scale, __bf16* x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npx = (int64_t)B * n * n;
  if (i >= npx * 8) return;
  const int c = (int)(i & 7);
  const int64_t p = i >> 3;
  const int b = (int)(p / (n * n)), r = (int)(p % (n * n)), u = r / n, v = r % n;
  const int h = n / 2;
  const float dv = d[(size_t)b * n * n + (size_t)((u + h) % n) * n + (v + h) % n];
  x[i] = (__bf16)(c == 0 ? scale * log1pf(fmaxf(dv, 0.0f)) : 0.0f);
}

// Squared error of the FP32 output (8 channels, the first 2 used) against
// the 2-channel target; writes the gradient (2/n)(out - t) into a bf16
// tensor with 8 channels, and per-block FP64 partial sums of the loss.
__global__ __launch_bounds__(256) void k_mse(const float* out, const float* tgt, int64_t npx, float inv_n,
                                              __bf16* dz, double* part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < npx; i += (int64_t)gridDim.x * 256) {
    const float e0 = out[8 * i] - tgt[2 * i], e1 = out[8 * i + 1] - tgt[2 * i + 1];
    s += (double)e0 * e0 + (double)e1 * e1;
    if (dz) {
      __bf16* g = dz + 8 * i;
      g[0] = (__bf16)(2.0f * inv_n * e0);
      g[1] = (__bf16)(2.0f * inv_n * e1);
#pragma unroll
      for (int c = 2; c < 8; ++c) g[c] = (__bf16)0.0f;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam step on FP32 parameters.
__global__ void k_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// ------------------------------------------------------------- stitching
// Predicted patch k covers the q x q window at (r_k + off, c_k + off).
// P_k = amp e^{i phase} from the network output (FP32, 8 channels).
__global__ void k_patches(const float* out, int64_t npx, float2* P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npx) return;
  const float a = out[8 * i], ph = out[8 * i + 1];
  float sn, cs;
  sincosf(ph, &sn, &cs);
  P[i] = make_float2(a * cs, a * sn);
}

// Neighbour lists of the overlap graph: j != k with overlapping windows,
// ascending j, at most maxnb per pattern.
__global__ void k_neighbours(const int2* pos, int K, int q, int maxnb, int* cnt, int* nb) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int2 a = pos[k];
  int c = 0;
  for (int j = 0; j < K && c < maxnb; ++j) {
    const int2 b = pos[j];
    if (j != k && abs(a.x - b.x) < q && abs(a.y - b.y) < q) nb[(size_t)k * maxnb + c++] = j;
  }
  cnt[k] = c;
}

// c[k][e] = sum over the overlap of conj(P_k) P_j (j = e-th neighbour), FP64
// accumulation in a fixed order.
__global__ __launch_bounds__(256) void k_overlaps(const float2* P, const int2* pos, const int* cnt, const int* nb,
                                                  int q, int maxnb, double2* c) {
  __shared__ double red[2][256];
  const int k = blockIdx.x;
  const int2 a = pos[k];
  const float2* pk = P + (size_t)k * q * q;
  for (int e = 0; e < cnt[k]; ++e) {
    const int j = nb[(size_t)k * maxnb + e];
    const int2 b = pos[j];
    const float2* pj = P + (size_t)j * q * q;
    const int dy = b.x - a.x, dx = b.y - a.y;  // window j = window k shifted by (dy, dx)
    double sr = 0.0, si = 0.0;
    for (int t = threadIdx.x; t < q * q; t += 256) {
      const int u = t / q, v = t - (t / q) * q;   // pixel of window k
      const int uj = u - dy, vj = v - dx;
      if (uj >= 0 && uj < q && vj >= 0 && vj < q) {
        const float2 x = pk[t], y = pj[uj * q + vj];
        sr += (double)x.x * y.x + (double)x.y * y.y;
        si += (double)x.x * y.y - (double)x.y * y.x;
      }
    }
    red[0][threadIdx.x] = sr;
    red[1][threadIdx.x] = si;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) {
        red[0][threadIdx.x] += red[0][threadIdx.x + off];
        red[1][threadIdx.x] += red[1][threadIdx.x + off];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) c[(size_t)k * maxnb + e] = make_double2(red[0][0], red[1][0]);
    __syncthreads();
  }
}

// One power-iteration step of phase synchronisation: z'_k = unit(z_k + sum_j c_kj z_j)
// (c_kj = <P_k, P_j> over the overlap, so z_k ~ e^{i theta_k} aligns P_k z_k with P_j z_j).
__global__ void k_sync_step(const double2* c, const int* cnt, const int* nb, int K, int maxnb, const double2* z,
                            double2* zn) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double sr = z[k].x, si = z[k].y;
  for (int e = 0; e < cnt[k]; ++e) {
    const double2 w = c[(size_t)k * maxnb + e], zj = z[nb[(size_t)k * maxnb + e]];
    sr += w.x * zj.x - w.y * zj.y;
    si += w.x * zj.y + w.y * zj.x;
  }
  const double m = sqrt(sr * sr + si * si);
  zn[k] = m > 0.0 ? make_double2(sr / m, si / m) : make_double2(1.0, 0.0);
}

// psi0[y][x] = sum over covering windows (ascending k, from the tile lists of
// the windows) of z_k P_k, divided by the count; 1 where nothing covers.
__global__ __launch_bounds__(256) void k_stitch(const float2* P, const double2* z, const int2* wpos,
                                                const int* offsets, const int* list, int H, int W, int q,
                                                float2* psi0) {
  // object tiles of the solver's tile lists: kTileH x kTileW, lane column x
  // in each 64-column part of the tile, rows yb + 4 i
  constexpr int R = kTileH / 4;
  const int ntx = tiles_x(W);
  const int t = blockIdx.x;
  const int yb = (t / ntx) * kTileH + (threadIdx.x >> 6);
  for (int part = 0; part < kTileW / 64; ++part) {
    const int x = (t % ntx) * kTileW + 64 * part + (threadIdx.x & 63);
    float2 acc[R];
    int n[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      acc[i] = make_float2(0.f, 0.f);
      n[i] = 0;
    }
    for (int e = offsets[t]; e < offsets[t + 1]; ++e) {
      const int k = list[e];
      const int2 rc = wpos[k];
      const int xx = x - rc.y;
      if ((unsigned)xx >= (unsigned)q) continue;
      const float2 zk = make_float2((float)z[k].x, (float)z[k].y);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int yy = yb + 4 * i - rc.x;
        if ((unsigned)yy < (unsigned)q) {
          acc[i] = cadd(acc[i], cmul(zk, P[(size_t)k * q * q + yy * q + xx]));
          n[i] += 1;
        }
      }
    }
    if (x >= W) continue;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int y = yb + 4 * i;
      if (y < H) psi0[(size_t)y * W + x] = n[i] ? cscale(acc[i], 1.0f / n[i]) : make_float2(1.f, 0.f);
    }
  }
}

// Adjoint of the stitch for fine-tuning: given g = dL/d conj(psi0) (object
// shape), d(amp, phase) of every window pixel, written as the bf16 gradient
// of the network output (8 channels).  count[y][x] = number of covering windows.
__global__ void k_stitch_adj(const float2* g, const float* out, const double2* z, const int2* wpos,
                             const int* count, int K, int W, int q, float scale, __bf16* dz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)K * q * q) return;
  const int k = (int)(i / (q * q)), r = (int)(i % (q * q)), u = r / q, v = r % q;
  const int2 rc = wpos[k];
  const size_t o = (size_t)(rc.x + u) * W + rc.y + v;
  const float2 gi = g[o];
  const float inv = 1.0f / (float)max(count[o], 1);
  // dL/dP = conj(z) g / count (Wirtinger); P = a e^{i ph}
  const float2 zc = make_float2((float)z[k].x, -(float)z[k].y);
  const float2 gp = cscale(cmul(zc, gi), inv);
  const float a = out[8 * i], ph = out[8 * i + 1];
  float sn, cs;
  sincosf(ph, &sn, &cs);
  // dL = 2 Re(conj(gp) dP), dP = e^{i ph} da + i a e^{i ph} dph
  const float re = gp.x * cs + gp.y * sn;  // Re(conj(gp) e^{i ph})
  const float im = gp.x * sn - gp.y * cs;  // Im(conj(gp) e^{i ph})
  // dL/da = 2 Re(conj(gp) e^{i ph}); dL/dph = 2 Re(conj(gp) i a e^{i ph}) = -2 a Im(...)
  __bf16* d = dz + 8 * i;
  d[0] = (__bf16)(scale * 2.0f * re);
  d[1] = (__bf16)(scale * -2.0f * a * im);
#pragma unroll
  for (int c = 2; c < 8; ++c) d[c] = (__bf16)0.0f;
}

// count[y][x] = number of windows covering the pixel
__global__ void k_cover_count(const int2* wpos, int K, int H, int W, int q, const int* offsets, const int* list,
                              int* count) {
  constexpr int R = kTileH / 4;
  const int ntx = tiles_x(W);
  const int t = blockIdx.x;
  const int yb = (t / ntx) * kTileH + (threadIdx.x >> 6);
  for (int part = 0; part < kTileW / 64; ++part) {
    const int x = (t % ntx) * kTileW + 64 * part + (threadIdx.x & 63);
    int n[R];
#pragma unroll
    for (int i = 0; i < R; ++i) n[i] = 0;
    for (int e = offsets[t]; e < offsets[t + 1]; ++e) {
      const int2 rc = wpos[list[e]];
      if ((unsigned)(x - rc.y) >= (unsigned)q) continue;
#pragma unroll
      for (int i = 0; i < R; ++i) n[i] += ((unsigned)(yb + 4 * i - rc.x) < (unsigned)q) ? 1 : 0;
    }
    if (x >= W) continue;
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (yb + 4 * i < H) count[(size_t)(yb + 4 * i) * W + x] = n[i];
  }
}

__global__ void k_fill_one(double2* z, int K) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) z[k] = make_double2(1.0, 0.0);
}
__global__ void k_copy2(const double2* a, double2* b, int K) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) b[k] = a[k];
}

__global__ void k_shift_pos(const int2* pos, int K, int off, int2* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) out[k] = make_int2(pos[k].x + off, pos[k].y + off);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace
}  // namespace ptyg

using namespace ptyg;

namespace {
thread_local char g_nn_err[256];
int nn_fail(const char* msg) {
  snprintf(g_nn_err, sizeof g_nn_err, "%s", msg);
  return -1;
}
#define NN_HIP(expr)                                                        \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) {                                                 \
      snprintf(g_nn_err, sizeof g_nn_err, "%s: %s", #expr, hipGetErrorString(e_)); \
      return -3;                                                            \
    }                                                                       \
  } while (0)
inline int cpad(int c) { return (c + 7) / 8 * 8; }
inline int kpad_of(int c) { return (9 * cpad(c) + 31) / 32 * 32; }
hipStream_t SS(void* s) { return reinterpret_cast<hipStream_t>(s); }
}  // namespace

extern "C" {

const char* ptyg_nn_last_error(void) { return g_nn_err; }

int32_t ptyg_nn_weight_sizes(int32_t cin, int32_t cout, int64_t* w_elems, int64_t* wt_elems) {
  if (cin < 1 || cout < 1 || !w_elems || !wt_elems) return nn_fail("bad arguments");
  *w_elems = (int64_t)cout * kpad_of(cin);
  *wt_elems = (int64_t)cpad(cin) * kpad_of(cout);
  return 0;
}

int32_t ptyg_nn_pack_weights(const float* w32, int32_t cin, int32_t cout, void* w, void* wt, void* stream) {
  if (!w32 || !w || !wt) return nn_fail("NULL argument");
  const int64_t n = (int64_t)cout * kpad_of(cin) + (int64_t)cpad(cin) * kpad_of(cout);
  hipLaunchKernelGGL(k_pack_weights, dim3(nblk(n)), dim3(256), 0, SS(stream), w32, cout, cin, cpad(cin), cpad(cout),
                     kpad_of(cin), kpad_of(cout), static_cast<__bf16*>(w), static_cast<__bf16*>(wt));
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_nn_conv3x3_fwd(const void* x, const void* w, const float* bias, void* y, int32_t B, int32_t H,
                            int32_t W, int32_t cin, int32_t cout, int32_t relu, int32_t out_f32, void* stream) {
  if (!x || !w || !bias || !y || B < 1 || H < 1 || W < 1 || cin < 1 || cout < 1) return nn_fail("bad arguments");
  const Geom g{B, H, W, B * H * W};
  FwdA la{static_cast<const __bf16*>(x), g, cpad(cin)};
  RowB lb{static_cast<const __bf16*>(w), cout, kpad_of(cin)};
  ConvStore st{y, bias, g.P, cout, cpad(cout), relu, out_f32};
  NN_HIP(gemm(la, lb, st, g.P, cpad(cout), kpad_of(cin), 1, SS(stream)));
  return 0;
}

int32_t ptyg_nn_conv3x3_bwd_data(const void* dz, const void* wt, void* dx, int32_t B, int32_t H, int32_t W,
                                 int32_t cin, int32_t cout, void* stream) {
  if (!dz || !wt || !dx || B < 1) return nn_fail("bad arguments");
  const Geom g{B, H, W, B * H * W};
  BwdA la{static_cast<const __bf16*>(dz), g, cpad(cout)};
  RowB lb{static_cast<const __bf16*>(wt), cpad(cin), kpad_of(cout)};
  DxStore st{static_cast<__bf16*>(dx), g.P, cpad(cin), cin};
  NN_HIP(gemm(la, lb, st, g.P, cpad(cin), kpad_of(cout), 1, SS(stream)));
  return 0;
}

int64_t ptyg_nn_wgrad_scratch(int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout) {
  const int64_t P = (int64_t)B * H * W;
  const int splits = (int)((P + 2047) / 2048);
  // dzT (bf16) + split-K partials + reduced packed gradient + bias chunk sums (fp32), in bytes
  return (int64_t)cpad(cout) * P * 2 + (int64_t)splits * cout * 9 * cpad(cin) * 4 +
         (int64_t)cout * 9 * cpad(cin) * 4 + (int64_t)kBiasChunks * cout * 4 + 1024;
}

int32_t ptyg_nn_conv3x3_bwd_weight(const void* x, const void* dz, float* dw32, float* db, int32_t B, int32_t H,
                                   int32_t W, int32_t cin, int32_t cout, void* scratch, int64_t scratch_bytes,
                                   void* stream) {
  if (!x || !dz || !dw32 || !db || !scratch) return nn_fail("bad arguments");
  if (scratch_bytes < ptyg_nn_wgrad_scratch(B, H, W, cin, cout)) return nn_fail("scratch too small");
  const Geom g{B, H, W, B * H * W};
  if (g.P % 8) return nn_fail("B*H*W must be a multiple of 8");
  const int cpi = cpad(cin), cpo = cpad(cout);
  const int splits = (g.P + 2047) / 2048;
  char* sp = static_cast<char*>(scratch);
  __bf16* dzt = reinterpret_cast<__bf16*>(sp);
  sp += (size_t)cpo * g.P * 2;
  sp = reinterpret_cast<char*>(((uintptr_t)sp + 255) & ~(uintptr_t)255);
  float* part = reinterpret_cast<float*>(sp);
  sp += (size_t)splits * cout * 9 * cpi * 4;
  float* dwp = reinterpret_cast<float*>(sp);
  hipStream_t s = SS(stream);
  hipLaunchKernelGGL(k_transpose_pc, dim3((g.P + 31) / 32, (cpo + 31) / 32), dim3(256), 0, s,
                     static_cast<const __bf16*>(dz), g.P, cpo, dzt);
  NN_HIP(hipGetLastError());
  WgtA la{dzt, cout, g.P};
  WgtB lb{static_cast<const __bf16*>(x), g, cpi};
  PartStore st{part, cout, 9 * cpi};
  NN_HIP(gemm(la, lb, st, cout, 9 * cpi, g.P, splits, s));
  const int64_t n = (int64_t)cout * 9 * cpi;
  hipLaunchKernelGGL(k_reduce_parts, dim3(nblk(n)), dim3(256), 0, s, part, splits, n, dwp);
  hipLaunchKernelGGL(k_unpack_wgrad, dim3(nblk((int64_t)cout * 9 * cin)), dim3(256), 0, s, dwp, cout, cin, cpi,
                     dw32);
  float* bpart = dwp + (size_t)cout * 9 * cpi;  // kBiasChunks * cout floats after the packed gradient
  hipLaunchKernelGGL(k_bias_grad, dim3(kBiasChunks, cout), dim3(256), 0, s, dzt, g.P, bpart);
  hipLaunchKernelGGL(k_bias_reduce, dim3((cout + 255) / 256), dim3(256), 0, s, bpart, cout, db);
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_nn_relu_bwd(const void* dy, const void* y, int64_t n, void* dz, void* stream) {
  if (!dy || !y || !dz) return nn_fail("NULL argument");
  if (n % 8) return nn_fail("element count must be a multiple of 8");
  hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(n / 8)), dim3(256), 0, SS(stream), static_cast<const bf16x8*>(dy),
                     static_cast<const bf16x8*>(y), n / 8, static_cast<bf16x8*>(dz));
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_nn_pool2(const void* x, void* y, int32_t B, int32_t H, int32_t W, int32_t c, int32_t backward,
                      void* stream) {
  if (!x || !y || (H & 1) || (W & 1)) return nn_fail("bad arguments");
  const int g8 = cpad(c) / 8;
  if (!backward)
    hipLaunchKernelGGL(k_pool_fwd, dim3(nblk((int64_t)B * (H / 2) * (W / 2) * g8)), dim3(256), 0, SS(stream),
                       static_cast<const bf16x8*>(x), B, H, W, g8, static_cast<bf16x8*>(y));
  else
    hipLaunchKernelGGL(k_pool_bwd, dim3(nblk((int64_t)B * H * W * g8)), dim3(256), 0, SS(stream),
                       static_cast<const bf16x8*>(x), B, H, W, g8, static_cast<bf16x8*>(y));
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_nn_up2(const void* x, void* y, int32_t B, int32_t H, int32_t W, int32_t c, int32_t backward,
                    void* stream) {
  if (!x || !y) return nn_fail("bad arguments");
  const int g8 = cpad(c) / 8;
  if (!backward)
    hipLaunchKernelGGL(k_up_fwd, dim3(nblk((int64_t)B * 4 * H * W * g8)), dim3(256), 0, SS(stream),
                       static_cast<const bf16x8*>(x), B, H, W, g8, static_cast<bf16x8*>(y));
  else
    hipLaunchKernelGGL(k_up_bwd, dim3(nblk((int64_t)B * H * W * g8)), dim3(256), 0, SS(stream),
                       static_cast<const bf16x8*>(x), B, H, W, g8, static_cast<bf16x8*>(y));
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_nn_input(const float* d, int32_t B, int32_t n, float scale, void* x, void* stream) {
  if (!d || !x || B < 1 || n < 2 || (n & 1)) return nn_fail("bad arguments");
  hipLaunchKernelGGL(k_input, dim3(nblk((int64_t)B * n * n * 8)), dim3(256), 0, SS(stream), d, B, n, scale,
                     static_cast<__bf16*>(x));
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_nn_mse(const float* out, const float* target, int64_t npx, void* dz, double* partials,
                    int32_t nparts, void* stream) {
  if (!out || !target || !partials || nparts < 1) return nn_fail("bad arguments");
  hipLaunchKernelGGL(k_mse, dim3(nparts), dim3(256), 0, SS(stream), out, target, npx, 1.0f / (float)(npx * 2),
                     static_cast<__bf16*>(dz), partials);
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_nn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                     float eps, int32_t step, void* stream) {
  if (!w || !g || !m || !v || step < 1) return nn_fail("bad arguments");
  const float c1 = 1.0f / (1.0f - powf(b1, (float)step)), c2 = 1.0f / (1.0f - powf(b2, (float)step));
  hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, SS(stream), w, g, m, v, n, lr, b1, b2, eps, c1, c2);
  NN_HIP(hipGetLastError());
  return 0;
}

int64_t ptyg_ws_tile_count(int32_t H, int32_t W) {
  if (H < 1 || W < 1) return 0;
  return (int64_t)tiles_x(W) * tiles_y(H);
}

int64_t ptyg_ws_tile_list_capacity(int32_t K, int32_t H, int32_t W, int32_t q) {
  if (K < 1 || H < 1 || W < 1 || q < 1) return 0;
  // the lists, then the build's per-tile counters
  return (int64_t)tile_list_ints(K, H, W, q);
}

int32_t ptyg_ws_tile_lists(const int32_t* wpos, int32_t K, int32_t H, int32_t W, int32_t q, int32_t* offsets,
                           int64_t offsets_len, int32_t* list, int64_t list_len, void* stream) {
  if (!wpos || !offsets || !list || K < 1 || q < 1 || H < 1 || W < 1) return nn_fail("bad arguments");
  if (offsets_len < ptyg_ws_tile_count(H, W) + 1) return nn_fail("offsets buffer too short");
  if (list_len < ptyg_ws_tile_list_capacity(K, H, W, q)) return nn_fail("list buffer too short");
  NN_HIP(launch_tile_lists(reinterpret_cast<const int2*>(wpos), K, H, W, q, offsets, list, SS(stream)));
  return 0;
}

int32_t ptyg_ws_patches(const float* out, int64_t npx, void* patches, void* stream) {
  if (!out || !patches) return nn_fail("NULL argument");
  hipLaunchKernelGGL(k_patches, dim3(nblk(npx)), dim3(256), 0, SS(stream), out, npx, static_cast<float2*>(patches));
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_ws_shift_positions(const int32_t* pos, int32_t K, int32_t off, int32_t* out, void* stream) {
  if (!pos || !out) return nn_fail("NULL argument");
  hipLaunchKernelGGL(k_shift_pos, dim3(nblk(K)), dim3(256), 0, SS(stream), reinterpret_cast<const int2*>(pos), K,
                     off, reinterpret_cast<int2*>(out));
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_ws_phase_sync(const void* patches, const int32_t* wpos, int32_t K, int32_t q, int32_t maxnb,
                           int32_t iters, int32_t* cnt, int32_t* nb, void* c, void* z, void* ztmp, void* stream) {
  if (!patches || !wpos || !cnt || !nb || !c || !z || !ztmp || K < 1 || q < 1 || maxnb < 1 || iters < 0)
    return nn_fail("bad arguments");
  hipStream_t s = SS(stream);
  const int2* p2 = reinterpret_cast<const int2*>(wpos);
  hipLaunchKernelGGL(k_neighbours, dim3(nblk(K)), dim3(256), 0, s, p2, K, q, maxnb, cnt, nb);
  hipLaunchKernelGGL(k_overlaps, dim3(K), dim3(256), 0, s, static_cast<const float2*>(patches), p2, cnt, nb, q,
                     maxnb, static_cast<double2*>(c));
  // z starts at 1 for every pattern; ping-pong between z and ztmp, ending in z
  hipLaunchKernelGGL(k_fill_one, dim3(nblk(K)), dim3(256), 0, s, static_cast<double2*>(z), K);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(k_sync_step, dim3(nblk(K)), dim3(256), 0, s, static_cast<const double2*>(c), cnt, nb, K,
                       maxnb, static_cast<const double2*>(z), static_cast<double2*>(ztmp));
    hipLaunchKernelGGL(k_copy2, dim3(nblk(K)), dim3(256), 0, s, static_cast<const double2*>(ztmp),
                       static_cast<double2*>(z), K);
  }
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_ws_stitch(const void* patches, const void* z, const int32_t* wpos, const int32_t* offsets,
                       const int32_t* list, int32_t H, int32_t W, int32_t q, void* psi0, void* stream) {
  if (!patches || !z || !wpos || !offsets || !list || !psi0) return nn_fail("NULL argument");
  const int T = tiles_x(W) * tiles_y(H);
  hipLaunchKernelGGL(k_stitch, dim3(T), dim3(256), 0, SS(stream), static_cast<const float2*>(patches),
                     static_cast<const double2*>(z), reinterpret_cast<const int2*>(wpos), offsets, list, H, W, q,
                     static_cast<float2*>(psi0));
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_ws_cover_count(const int32_t* wpos, int32_t K, int32_t H, int32_t W, int32_t q, const int32_t* offsets,
                            const int32_t* list, int32_t* count, void* stream) {
  if (!wpos || !offsets || !list || !count) return nn_fail("NULL argument");
  const int T = tiles_x(W) * tiles_y(H);
  hipLaunchKernelGGL(k_cover_count, dim3(T), dim3(256), 0, SS(stream), reinterpret_cast<const int2*>(wpos), K, H, W,
                     q, offsets, list, count);
  NN_HIP(hipGetLastError());
  return 0;
}

int32_t ptyg_ws_stitch_adjoint(const void* g, const float* out, const void* z, const int32_t* wpos,
                               const int32_t* count, int32_t K, int32_t W, int32_t q, float scale, void* dz,
                               void* stream) {
  if (!g || !out || !z || !wpos || !count || !dz) return nn_fail("NULL argument");
  hipLaunchKernelGGL(k_stitch_adj, dim3(nblk((int64_t)K * q * q)), dim3(256), 0, SS(stream),
                     static_cast<const float2*>(g), out, static_cast<const double2*>(z),
                     reinterpret_cast<const int2*>(wpos), count, K, W, q, scale, static_cast<__bf16*>(dz));
  NN_HIP(hipGetLastError());
  return 0;
}

}  // extern "C"
