/* ptyg_nn: kernels of the learned CG warm start (BF16 MFMA, FP32 accumulate).
 *
 * A small convolutional encoder-decoder maps each log-intensity diffraction
 * pattern to the object patch at its scan position (amplitude, phase); the
 * predictions are stitched into the starting guess psi_0 of ML-CG
 * (Eq. update, Algorithm 1 of arXiv 2106.07575 start from an arbitrary
 * psi_0; the paper itself starts from a constant).  These entry points are
 * the network's layers and training step; the orchestration lives in the
 * Python package.
 *
 * Conventions: activations are NHWC bfloat16 device tensors [B][H][W][Cp]
 * with Cp = C rounded up to a multiple of 8 (padded channels are zero);
 * 3x3 convolutions use zero padding 1 and stride 1.  Weights are FP32
 * master copies w32[cout][3*3][cin] packed by ptyg_nn_pack_weights into the
 * bf16 GEMM layouts w[cout][kpad(cin)] and wt[cp(cin)][kpad(cout)],
 * kpad(c) = 9*Cp rounded up to 32.  All pointers are device pointers owned
 * by the caller, 16-byte aligned; calls are asynchronous on `stream` (a
 * hipStream_t).  Return 0, -1 for bad arguments, -3 for a HIP error
 * (ptyg_nn_last_error gives the text).  Results are deterministic (no
 * atomics; fixed reduction orders).
 */
#ifndef PTYG_NN_H
#define PTYG_NN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

const char* ptyg_nn_last_error(void);

/* Element counts of the packed bf16 weight layouts for a cin -> cout layer. */
int32_t ptyg_nn_weight_sizes(int32_t cin, int32_t cout, int64_t* w_elems, int64_t* wt_elems);
/* w32 [cout][9][cin] fp32 -> w (bf16, forward layout), wt (bf16, transposed for backward-data). */
int32_t ptyg_nn_pack_weights(const float* w32, int32_t cin, int32_t cout, void* w, void* wt, void* stream);

/* y = act(conv3x3(x, w) + bias): x [B][H][W][Cp(cin)] bf16, bias [cout] fp32,
 * y [B][H][W][Cp(cout)] bf16 (or fp32 if out_f32), act = ReLU if relu else identity. */
int32_t ptyg_nn_conv3x3_fwd(const void* x, const void* w, const float* bias, void* y, int32_t B, int32_t H,
                            int32_t W, int32_t cin, int32_t cout, int32_t relu, int32_t out_f32, void* stream);
/* dx = conv3x3^T(dz, w): dz [B][H][W][Cp(cout)] bf16, wt from pack_weights, dx [B][H][W][Cp(cin)] bf16. */
int32_t ptyg_nn_conv3x3_bwd_data(const void* dz, const void* wt, void* dx, int32_t B, int32_t H, int32_t W,
                                 int32_t cin, int32_t cout, void* stream);
/* Scratch bytes needed by ptyg_nn_conv3x3_bwd_weight. */
int64_t ptyg_nn_wgrad_scratch(int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout);
/* dw32 [cout][9][cin] = sum_p dz[p][co] x[p + offset][ci]; db [cout] = sum_p dz[p][co]
 * (FP32, split-K partial sums reduced in a fixed order).  B*H*W must be a multiple of 8. */
int32_t ptyg_nn_conv3x3_bwd_weight(const void* x, const void* dz, float* dw32, float* db, int32_t B, int32_t H,
                                   int32_t W, int32_t cin, int32_t cout, void* scratch, int64_t scratch_bytes,
                                   void* stream);
/* dz = dy * (y > 0), n elements (bf16, n a multiple of 8). */
int32_t ptyg_nn_relu_bwd(const void* dy, const void* y, int64_t n, void* dz, void* stream);
/* 2x2 average pooling of x [B][H][W][Cp(c)] (backward: x is dy [B][H/2][W/2], y is dx [B][H][W]). */
int32_t ptyg_nn_pool2(const void* x, void* y, int32_t B, int32_t H, int32_t W, int32_t c, int32_t backward,
                      void* stream);
/* Nearest 2x upsampling of x [B][H][W][Cp(c)] (backward: x is dy [B][2H][2W], y is dx [B][H][W]). */
int32_t ptyg_nn_up2(const void* x, void* y, int32_t B, int32_t H, int32_t W, int32_t c, int32_t backward,
                    void* stream);
/* Network input from B patterns d [B][n][n] (zero frequency at [0][0], n even):
 * x[b][u][v][0] = scale * log(1 + d[b][(u + n/2) % n][(v + n/2) % n]) (bf16 [B][n][n][8], channels
 * 1..7 = 0): the pattern re-centred so that the bright zero-order region is one connected image. */
int32_t ptyg_nn_input(const float* d, int32_t B, int32_t n, float scale, void* x, void* stream);
/* Loss sum |out - target|^2 over npx pixels of 2 channels: out fp32 [npx][8] (channels 0, 1),
 * target fp32 [npx][2]; dz (nullable) bf16 [npx][8] = 2 (out - target) / (2 npx);
 * partials (device double[nparts]) get per-block partial sums. */
int32_t ptyg_nn_mse(const float* out, const float* target, int64_t npx, void* dz, double* partials,
                    int32_t nparts, void* stream);
/* One Adam step (bias-corrected with `step` >= 1) on n FP32 parameters. */
int32_t ptyg_nn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                     float eps, int32_t step, void* stream);

/* ---- stitching of predicted patches into the CG start psi_0 ----
 * Window k is the q x q central part of patch k: its top-left corner wpos[k]
 * = pos[k] + (n - q)/2 (ptyg_ws_shift_positions).  A diffraction pattern is
 * blind to a constant phase of its patch, so the windows' phases are first
 * synchronised: z = leading eigenvector (power iteration, unit-modulus
 * entries) of the overlap matrix c_kj = sum_overlap conj(P_k) P_j. */
/* Per-tile lists (the solver's object tiles, ascending window order) of the
 * q x q windows at wpos: offsets int32[ptyg_ws_tile_count(H, W) + 1], list
 * int32[ptyg_ws_tile_list_capacity(K, H, W, q)] (the lists, followed by
 * one counter per tile that the build uses as scratch); offsets_len and
 * list_len give the caller's buffer lengths in elements, and buffers shorter
 * than those sizes are rejected (nothing is written).  The two size queries
 * are host functions (no GPU); they return 0 for a non-positive size. */
int64_t ptyg_ws_tile_count(int32_t H, int32_t W);
int64_t ptyg_ws_tile_list_capacity(int32_t K, int32_t H, int32_t W, int32_t q);
int32_t ptyg_ws_tile_lists(const int32_t* wpos, int32_t K, int32_t H, int32_t W, int32_t q, int32_t* offsets,
                           int64_t offsets_len, int32_t* list, int64_t list_len, void* stream);
/* patches [npx] complex64 = amp e^{i phase} from the network output fp32 [npx][8]. */
int32_t ptyg_ws_patches(const float* out, int64_t npx, void* patches, void* stream);
/* out[k] = pos[k] + (off, off). */
int32_t ptyg_ws_shift_positions(const int32_t* pos, int32_t K, int32_t off, int32_t* out, void* stream);
/* Phase synchronisation.  Scratch: cnt int32[K], nb int32[K*maxnb], c complex128[K*maxnb],
 * ztmp complex128[K]; result z complex128[K]. */
int32_t ptyg_ws_phase_sync(const void* patches, const int32_t* wpos, int32_t K, int32_t q, int32_t maxnb,
                           int32_t iters, int32_t* cnt, int32_t* nb, void* c, void* z, void* ztmp, void* stream);
/* psi0[y][x] = mean over covering windows (ascending k) of z_k P_k, 1 where none covers.
 * offsets/list: tile lists of the windows (ptyg_ws_tile_lists: the object gradient's tiles). */
int32_t ptyg_ws_stitch(const void* patches, const void* z, const int32_t* wpos, const int32_t* offsets,
                       const int32_t* list, int32_t H, int32_t W, int32_t q, void* psi0, void* stream);
/* count[y][x] = number of windows covering each object pixel. */
int32_t ptyg_ws_cover_count(const int32_t* wpos, int32_t K, int32_t H, int32_t W, int32_t q, const int32_t* offsets,
                            const int32_t* list, int32_t* count, void* stream);
/* Adjoint of the stitch: g = dL/d conj(psi0) (complex64, object shape) -> gradient of L
 * with respect to the network output (amp, phase), times `scale`, as bf16 [K*q*q][8]. */
int32_t ptyg_ws_stitch_adjoint(const void* g, const float* out, const void* z, const int32_t* wpos,
                               const int32_t* count, int32_t K, int32_t W, int32_t q, float scale, void* dz,
                               void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PTYG_NN_H */
