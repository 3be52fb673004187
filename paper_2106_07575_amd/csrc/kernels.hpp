// Kernel argument blocks and launcher declarations shared by the kernel
// translation unit and the C-ABI host code.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace ptyg {

// Everything a pattern kernel may touch.  Unused pointers are null.
struct PatArgs {
  int H, W, K, N;
  const float2* obj;     // psi [H][W]
  const float2* dobj;    // eta_psi [H][W] (line-search trial: psi + gamma eta)
  const float2* probe;   // p [N][N]
  const float2* dprobe;  // eta_p [N][N] (joint line-search trial)
  float gamma;
  const int2* pos;       // [K] (row, col)
  const float* data;     // intensities, [K][N][N] or per-pattern transposed
  float2* far;           // far field [K][N][N] (forward out / adjoint in)
  float2* gobj;          // accumulator of the atomic debug scatter [H][W]
  float2* ubuf;          // per-pattern back-propagated waves u_k = F^H r_k, [K][N][N]
  int premul;            // GRAD / adjoint, n <= 128: store conj(p) u_k (object adjoint only)
  double* partials;      // per-workgroup (phi, f) pairs
  float eps;
  int est;               // estimator: kEstML (Eq. ML) or kEstLS (least squares on amplitudes)
  float2* gstore;        // GRAD: far field G psi, per-pattern transposed (batched line search); nullable
  // batched line search: GRAD with gstore writes per-workgroup sums of
  // |G psi|^2 to zs_part; the direction forward writes rows of 4:
  // sum Re(P conj y), sum Re(Q conj y) (0 if Q is null), sum |y|^2, 0
  // (y = its far field; P, Q stored far fields in the same element order)
  const float2* zs_p;
  const float2* zs_q;
  double* zs_part;
  // n = 128, batched search with the sums formed elsewhere: records of the
  // per-pattern transposed far field, one per 32-element segment {mask of
  // the listed elements (d > 0 or NaN), compacted index of the first}; when
  // set, gstore (GRAD) and far (direction forward) receive only the listed
  // elements, compacted in ascending element order
  const uint2* cseg;
  // GRAD / MINFUNC: also form Eq. ML's F per pixel (the API calls report it;
  // the solver forms it from Phi and a data constant)
  int want_f;
  // 256^2 joint direction forward (first-order term): when set, per-block
  // patch sums of a = p psi, b = p eta + eta_p psi, c = eta_p eta, two rows
  // of 4 per block: (Re a b*, 0, |b|^2, 0) at ps_part[4 blk], (Re a c*,
  // Re b c*, |c|^2, 0) at ps_part[4 (4 ps_k + blk)], blk = 4 k + sub-grid
  double* ps_part;
  int ps_k;  // patterns of the whole sequence of staged chunks (set by the 256^2 launchers)
};

// Batched line search over stored far fields: trial j evaluates the
// deviance at A + g_j B (+ g_j^2 C in joint mode) against the intensities d,
// all four arrays in the same per-pattern element order, over the elements
// listed in idx (those with d > 0 or NaN; the d <= 0 ones contribute
// |A + g B + g^2 C|^2, a polynomial in g formed from the zero-pixel sums).
constexpr int kLsBatch = 16;   // trials per pass
// Per-block row: kLsBatch trial sums, then the listed elements' shares of
// sum |A|^2, Re A B*, |B|^2, Re A C*, Re B C*, |C|^2, and padding.
constexpr int kLsRow = kLsBatch + 8;
constexpr int kLsBlocks = 4096;
struct LsArgs {
  const float2* A;
  const float2* B;
  const float2* C;  // joint mode only (else null)
  const float* d;
  const int* idx;   // compacted element indices (unused when compact)
  int compact;      // A, B and d hold the listed elements only, compacted
  int64_t n;        // number of listed elements
  int J;            // trials in this pass, 1..kLsBatch
  int est;          // estimator (as PatArgs::est)
  float eps;
  float g[kLsBatch];
  double* partials;  // [blocks][kLsRow]
};
// Elements per block of the compaction of the d > 0 elements.
constexpr int kNzChunk = 4096;

struct VecArgs {
  int64_t n;
  float2* a;
  float2* b;
  const float2* c;
  double alpha;
  double* partials;
  const double* alpha_dev;    // k_dir, k_axpy: coefficient read on the device (overrides alpha); k_dir also ...
  const double* restart_dev;  // ... and a restart flag (nonzero: b <- -a, the old b ignored)
  // k_dir, optional: rows (sum w Re(psi conj b), 0, sum w |b|^2, 0) per block
  // over the new direction b, w = zs_w[i].x (the illumination: these are
  // Re<G psi, G b> and ||G b||^2 when G^H G is diagonal)
  const float2* zs_psi;
  const float2* zs_w;
  double* zs_part;
  // k_dir, optional (overrides alpha / alpha_dev): the Dai-Yuan coefficient
  // beta = n1 / (n2 - n3) from device scalars, restart (beta 0) when
  // dy_restart is set or the denominator is not finite and positive;
  // workgroup 0 writes beta and the restart flag (0 / 1) to dy_out[0..1]
  const double* dy_n1;
  const double* dy_n2;
  const double* dy_n3;
  double* dy_out;
  int dy_restart;
};

enum class DataLayout { Rows = 0, Transposed = 1 };

// Calls f with std::integral_constant<int, est> for a supported estimator
// (0: Poisson ML, 1: least squares), else returns hipErrorInvalidValue.
template <typename F>
hipError_t dispatch_est(int est, F&& f) {
  switch (est) {
    case 0: return f(std::integral_constant<int, 0>{});
    case 1: return f(std::integral_constant<int, 1>{});
    default: return hipErrorInvalidValue;
  }
}

// Launchers; each returns hipSuccess or the launch error.  `blocks_out`
// receives the number of (phi, f) partial pairs written.
hipError_t launch_forward(const PatArgs& a, hipStream_t s);
// Both write u_k = F^H (far_k or residual_k) for every pattern into a.ubuf;
// the object and probe adjoints are then formed by launch_tile_sum and
// launch_probe_grad (no atomics, fixed summation order).
hipError_t launch_adjoint(const PatArgs& a, hipStream_t s);
hipError_t launch_grad(const PatArgs& a, DataLayout lay, int* blocks_out, hipStream_t s);
// Test hook: GRAD from a given far field a.far (row layout [K][N][N]) in
// place of G psi -- residual and objective partials, inverse transform and
// the stored waves in a.ubuf exactly as launch_grad writes them.
hipError_t launch_grad_far(const PatArgs& a, int* blocks_out, hipStream_t s);
hipError_t launch_grad_far256(const PatArgs& a, int* blocks_out, hipStream_t s);

// 256^2 patterns (kernels256.hip): four polyphase 128^2 sub-transforms and
// a pointwise radix stage; u_k is left in the polyphase layout.
hipError_t launch_forward256(const PatArgs& a, hipStream_t s);
hipError_t launch_adjoint256(const PatArgs& a, hipStream_t s);
hipError_t launch_grad256(const PatArgs& a, DataLayout lay, int* blocks_out, hipStream_t s);
hipError_t launch_minfunc256(const PatArgs& a, DataLayout lay, int* blocks_out, hipStream_t s);

// Object tiles of the deterministic scatter: kTileH x kTileW pixels.
constexpr int kTileH = 16, kTileW = 64;
__host__ __device__ inline int tiles_x(int W) { return (W + kTileW - 1) / kTileW; }
__host__ __device__ inline int tiles_y(int H) { return (H + kTileH - 1) / kTileH; }
// Upper bound of tiles one n x n patch overlaps.
inline int tiles_per_patch(int n) { return ((n - 1) / kTileH + 2) * ((n - 1) / kTileW + 2); }
// Per-tile lists of the patterns overlapping it, in ascending pattern order:
// offsets [T + 1], list [sum of counts] (at most K * tiles_per_patch(N)),
// followed by T ints of scratch: `list` must hold tile_list_ints() ints.
inline size_t tile_list_ints(int K, int H, int W, int N) {
  const size_t T = (size_t)tiles_x(W) * tiles_y(H);
  const size_t pairs = (size_t)K * tiles_per_patch(N);
  return (pairs > T ? pairs : T) + T;
}
hipError_t launch_tile_lists(const int2* pos, int K, int H, int W, int N, int* offsets, int* list, hipStream_t s);
// out[y][x] = sum over the tile's patterns k (ascending) of conj(p) * u_k at
// (y - r_k, x - c_k); every object pixel is written.  probe = NULL: ubuf
// already holds conj(p) * u_k (PatArgs::premul, n <= 128 only).
// dot_parts (nullable): per tile t, rows (sum |out|^2, sum Re(conj(dot_b) out))
// over the tile's pixels (dot_b nullable: second entry 0); tiles_x * tiles_y rows.
hipError_t launch_tile_sum(const float2* ubuf, const float2* probe, const int2* pos, const int* offsets,
                           const int* list, int K, int H, int W, int N, float2* out, hipStream_t s,
                           const float2* dot_b = nullptr, double* dot_parts = nullptr);
// out[y][x].x = sum over the tile's patterns k (ascending) of |p|^2 at
// (y - r_k, x - c_k): the illumination, the diagonal of G^H G.
hipError_t launch_illum(const float2* probe, const int2* pos, const int* offsets, const int* list, int H, int W,
                        int N, float2* out, hipStream_t s);
// out[u][v] = sum_k conj(obj[r_k + u][c_k + v]) u_k[u][v], in fixed order
// (chunks of patterns, then chunks summed in order); partial holds
// kProbeChunks * N * N values.
constexpr int kProbeChunks = 64;
hipError_t launch_probe_grad(const float2* ubuf, const float2* obj, const int2* pos, int K, int W, int N,
                             float2* partial, float2* out, hipStream_t s);
hipError_t launch_minfunc(const PatArgs& a, DataLayout lay, int* blocks_out, hipStream_t s);
// far (per-pattern transposed) = G applied to the direction: lin = false:
// F(probe * obj[pos]); lin = true: F(probe * dobj[pos] + dprobe * obj[pos])
// (the first-order term of (p + g dp)(psi + g eta)).
hipError_t launch_fwd_t(const PatArgs& a, bool lin, hipStream_t s);
hipError_t launch_fwd_t256(const PatArgs& a, bool lin, hipStream_t s);
// Rows of per-workgroup partials that a 256^2 direction forward / GRAD pass
// over K patterns writes (radix-stage workgroups; GRAD sums them over its
// staged chunks).
int fwd_t256_blocks(int K);
int grad256_blocks(int K);
// Objective partials of a.J trials; `blocks_out` rows of kLsRow doubles.
hipError_t launch_ls_batch(const LsArgs& a, int* blocks_out, hipStream_t s);
// Joint-mode search coefficients over the patches (a' = p psi_k,
// b' = p eta_k + eta_p psi_k, c' = eta_p eta_k): rows of 4 per block,
// parts1 (Re a'b'*, 0, |b'|^2, 0), parts2 (Re a'c'*, Re b'c'*, |c'|^2, 0);
// patch_sums_blocks rows each.  N a power of two.
int patch_sums_blocks(int K, int N);
hipError_t launch_patch_sums(const float2* obj, const float2* eta, const float2* probe, const float2* eta_p,
                             const int2* pos, int K, int W, int N, double* parts1, double* parts2, hipStream_t s);
// idx = ascending indices e < n with !(d[e] <= 0), count in offsets[blocks]
// (blocks = ceil(n / kNzChunk); offsets holds blocks + 1 ints, counts
// blocks ints of scratch).
// seg (nullable, n a multiple of 32): one {mask, first compacted index}
// record per 32 elements; dc (nullable): the listed d values, compacted.
hipError_t launch_nz_compact(const float* d, int64_t n, int* counts, int* offsets, int* idx, uint2* seg,
                             float* dc, hipStream_t s);
// The two halves of launch_nz_compact: the per-chunk counts and their scan
// (offsets[blocks] = total), then the fill.
hipError_t launch_nz_count(const float* d, int64_t n, int* counts, int* offsets, hipStream_t s);
hipError_t launch_nz_fill(const float* d, int64_t n, const int* offsets, int* idx, uint2* seg, float* dc,
                          hipStream_t s);
// *out = number of elements with !(d <= 0) (d > 0 or NaN); out is zeroed
// by a kernel first.
hipError_t launch_count_listed(const float* d, int64_t n, unsigned long long* out, hipStream_t s);
// Zero-pixel sums of the direction forward: rows of 4 doubles per block.
int fwd_t_blocks(int N, int K);

// ---- multi-view batch: V views of equal shape stacked into one launch.
// Patterns per workgroup of the n x n pattern kernels (n <= 128).
int patterns_per_block(int N);
// out[v][0..width) = ordered sums over the workgroups of a pattern kernel
// launch (blocks of `width` doubles) whose patterns belong to view v
// (k patterns per view, every workgroup inside one view).
hipError_t launch_finalize_views(const double* partials, int N, int K, int k_per_view, int views, int width,
                                 double* out, hipStream_t s);
// Segmented object-sized kernels: view v owns elements [v n, (v + 1) n);
// partial rows [v][kSegBlocks][2]; alpha (beta or gamma) per view from a
// device array.
constexpr int kSegBlocks = 256;
hipError_t launch_dot2_views(const float2* a, const float2* b, int64_t n, int views, double* partials,
                             hipStream_t s);
hipError_t launch_dir_views(const float2* a, float2* b, const double* beta, int64_t n, int views,
                            double* partials, hipStream_t s);
hipError_t launch_axpy_views(float2* a, const float2* c, const double* alpha, int64_t n, int views,
                             hipStream_t s);
// out[v] = sum over the d > 0 elements of segment v (n elements each) of
// d - d log d, in FP64 (F = Phi + this constant); partials holds
// segs * kSegBlocks doubles, or 2048 for a single segment.
hipError_t launch_data_const(const float* d, int64_t n, int segs, double* partials, double* out, hipStream_t s);
// out[v][0..width) = ordered sums of rows [v][0..rows) of `width` doubles.
hipError_t launch_finalize_seg(const double* partials, int rows, int width, int views, double* out,
                               hipStream_t s);
// Batched line-search pass per view: view v's listed elements are
// idx[offsets[v * chunks_per_view] .. offsets[(v + 1) * chunks_per_view]);
// partial rows [v][kSegBlocks][kLsRow].
hipError_t launch_ls_batch_views(const LsArgs& a, const int* offsets, int chunks_per_view, int views,
                                 hipStream_t s);
hipError_t launch_shift_views(const int2* pos, int k, int kp, int views, int rows_per_view, int pad_row, int2* out,
                              hipStream_t s);
// out[v][j] = ordered sum of rows [v][0..kSegBlocks) column j, j < kLsRow.
hipError_t launch_ls_finalize_views(const double* partials, int views, double* out, hipStream_t s);
// out[j] = in-order sum over `count` rows of partials[row][j], j < kLsRow.
hipError_t launch_ls_finalize(const double* partials, int count, double* out, hipStream_t s);
// Acceptance of a batched line-search pass on the device (Eq. linesearch):
// trial i (0-based) passes when row[i] + zero(g_i) <= phi + gam[i] t, with
// zero(g) the d <= 0 polynomial at the FP32 step g = (float) gam[i] whose
// coefficients are the whole-array sums minus the listed shares; the first
// passing trial is taken.  With stop_check, phi <= target (target >= 0)
// stops instead.  Writes out[0] = accepted step (0 if none or stop),
// out[1] = accepted trial (1-based, 0 if none), out[2] = 1 on stop.
struct LsAccept {
  double gam[kLsBatch];
  double t, target;
  int J, joint, stop_check;
};
hipError_t launch_ls_accept(double* sc, const double* zs, const double* row, double* out, const LsAccept& a,
                            hipStream_t s);
hipError_t launch_transpose_data(const float* d, float* dt, int K, int N, hipStream_t s);
hipError_t launch_debug_gather(const PatArgs& a, float2* patches, hipStream_t s);
hipError_t launch_debug_scatter(const PatArgs& a, const float2* patches, hipStream_t s);
hipError_t launch_check_positions(const int2* pos, int K, int H, int W, int N, int* flag, hipStream_t s);
hipError_t launch_debug_lane_swap(float* a, float* b, hipStream_t s);

// Vector kernels.  Partials: `vec_blocks(n)` pairs per call.
int vec_blocks(int64_t n);
hipError_t launch_zero(float2* x, int64_t n, hipStream_t s);
hipError_t launch_zero_f64(double* x, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int* x, int64_t n, int value, hipStream_t s);
// partials <- (||a||^2, Re<b, a>) ; b may be null
hipError_t launch_dot2(const VecArgs& v, hipStream_t s);
// b <- -a + alpha b ; partials <- (Re<b_new, a>, ||b_new||^2)
hipError_t launch_dir(const VecArgs& v, hipStream_t s);
// a <- a + alpha c
hipError_t launch_axpy(const VecArgs& v, hipStream_t s);
// Dai-Yuan coefficient on the device (Eq. DaiYuan): from sc[n1], sc[n2]
// (||g_m||^2, Re<eta_{m-1}, g_m>) and sc[n3] (Re<eta_{m-1}, g_{m-1}>), each
// plus its joint-mode probe term at +joint_off when joint_off > 0, writes
// sc[beta] and sc[rst] (1 if restarted: `restart`, or a denominator that is
// not positive and finite, or a non-finite numerator; beta is then 0).
hipError_t launch_dy_beta(double* sc, int n1, int n2, int n3, int joint_off, int beta, int rst, int restart,
                          hipStream_t s);
// out[j] (+)= sum over copies of probe-gradient copies (out[j] = sum_c src[c][j])
hipError_t launch_sum_copies(const float2* src, int copies, int64_t n, float2* out, hipStream_t s);
// out[0..width) = in-order sums of `count` rows of `width` doubles
hipError_t launch_finalize(const double* partials, int count, int width, double* out, hipStream_t s);
// One or two independent finalizations in one launch (jobs = 1 or 2).
struct FinJob {
  const double* p;  // [count][width] partial rows
  int count, width;  // width 1..4
  double* out;       // [width]
};
hipError_t launch_finalize2(const FinJob& a, const FinJob& b, int jobs, hipStream_t s);
// Up to four independent finalizations in one launch.
hipError_t launch_finalize_n(const FinJob* jobs, int n, hipStream_t s);

}  // namespace ptyg
