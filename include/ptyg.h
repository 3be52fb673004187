/* ptyg: maximum-likelihood conjugate-gradient ptychography on one MI355X.
 *
 * C ABI of libptyg.so.  The operations follow arXiv 2106.07575 ("Scalable and
 * accurate multi-GPU based image reconstruction of large-scale ptychography
 * data"), section "Background":
 *   forward model   Eq. fwd_model   |G psi|^2 = |F Q psi|^2 = d
 *   objective       Eq. ML          F(psi) = sum_j |G psi|_j^2 - 2 d_j log |G psi|_j
 *   gradient        Eq. gradient    grad F = G^H (G psi - d / conj(G psi)),
 *                                   G^H = Q^H F^H, Q^H multiplies by conj(p)
 *   CG update       Eq. update      psi_{m+1} = psi_m + gamma_m eta_m
 *   direction       Eq. DaiYuan     eta_m = -grad_m + ||grad_m||^2 /
 *                                   <eta_{m-1}, grad_m - grad_{m-1}> eta_{m-1}
 *   line search     Eq. linesearch  F(psi + gamma eta) <= F(psi) + gamma t
 *   workflow        Algorithm 1     GRAD -> DIR -> LS -> Update
 *
 * Conventions for every entry point:
 *   - Complex values are interleaved float32 (re, im), i.e. torch.complex64.
 *     Arrays are row-major and contiguous.
 *   - All array pointers are DEVICE pointers owned by the caller unless a
 *     parameter says "host".  The library never frees or retains them.
 *   - F is the unitary 2-D DFT (1/n per n x n transform); the zero frequency
 *     is at [0][0] (no shift).
 *   - Scan positions are int32 [k][2] = (row, col) of the patch's top-left
 *     corner; every patch must lie inside the object
 *     (0 <= row <= obj_h - n, 0 <= col <= obj_w - n).  The enqueue calls do
 *     not check this (ptyg_check_positions does; ptyg_cg_solve calls it).
 *   - Enqueue calls are asynchronous on `stream` (a hipStream_t; NULL is the
 *     default stream) and return after the launches.  Host-detectable
 *     argument errors return before anything is launched.
 *   - Scratch comes from a caller-provided device workspace of at least
 *     ptyg_workspace_size() bytes (256-byte aligned).  The calls allocate no
 *     device memory.  Concurrent calls must not share a workspace.
 *   - Supported probe sizes n: 16, 32, 64, 128, 256.  obj_h * obj_w * 8 bytes and
 *     n * n * k * 8 bytes must each stay below 2^31 elements' worth of
 *     indices (objects up to 32768 x 32768).
 *   - No C++ exception crosses the ABI; the last error text of the calling
 *     thread is available from ptyg_last_error().
 */
#ifndef PTYG_H
#define PTYG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  float re, im;
} ptyg_c64;

typedef int32_t ptyg_status;
enum {
  PTYG_OK = 0,
  PTYG_E_INVAL = -1,      /* null pointer, bad dims, unsupported n, misaligned workspace */
  PTYG_E_BOUNDS = -2,     /* a scan position puts its patch outside the object */
  PTYG_E_HIP = -3,        /* HIP launch or runtime error (see ptyg_last_error) */
  PTYG_E_NONFINITE = -4,  /* NaN or Inf in the objective at the current iterate */
  PTYG_E_WORKSPACE = -5   /* workspace smaller than ptyg_workspace_size() */
};

/* hipStream_t, passed as an opaque pointer so this header needs no HIP headers. */
typedef void* ptyg_stream_t;

/* Estimators.  PTYG_EST_ML: the Poisson maximum likelihood of Eq. ML (the
 * paper's worked formulation).  PTYG_EST_LS: least squares on the amplitudes,
 * which the paper names (section Background) without a formula; taken as
 * F = sum_j (|G psi|_j - sqrt(d_j))^2 with gradient
 * G^H (G psi - sqrt(d) G psi / |G psi|) in the same Wirtinger convention as
 * Eq. gradient (no factor 2); d <= 0 pixels contribute |G psi|^2.  Its Phi
 * and F are the same number. */
enum { PTYG_EST_ML = 0, PTYG_EST_LS = 1 };

typedef struct {
  int32_t obj_h, obj_w; /* object rows, columns */
  int32_t n;            /* probe side = detector side, in {16, 32, 64, 128, 256} */
  int32_t k;            /* number of scan positions = diffraction patterns, >= 1 */
} ptyg_dims;

/* Options of ptyg_cg_solve (Algorithm 1 and Eq. linesearch). */
typedef struct {
  int32_t iters;        /* iteration limit (Algorithm 1's iter_limit) */
  int32_t update_probe; /* 0: object only (the paper); 1: joint object+probe CG */
  double gamma0;        /* initial step of each line search (Algorithm 1: 1.0) */
  double tau;           /* step shrink factor (Algorithm 1: 0.5) */
  double t;             /* termination parameter of Eq. linesearch (0 in practice) */
  int32_t max_halvings; /* line-search trials before giving up (gamma = 0, restart); e.g. 40 */
  double eps;           /* guard on |G psi|^2 for log and division (e.g. 1e-32) */
  double target_phi;    /* stop before an iteration whose deviance is <= target; < 0 disables */
  int32_t line_search;  /* PTYG_LS_SEQUENTIAL: one MINFUNC pass (forward transform of
                           psi + gamma eta) per trial, as Algorithm 1 states it;
                           PTYG_LS_BATCHED: G is linear, so trial j's far field is
                           G psi + gamma_j G eta (+ gamma_j^2 G(eta_p eta) in joint
                           mode): the GRAD pass stores G psi, one forward pass forms
                           G eta, and up to 16 trials are evaluated per streaming pass
                           over the stored far fields (no transforms); the accepted
                           trial is the first that passes, as in the sequential order,
                           decided on the device.  The pixels with d <= 0 enter through
                           a polynomial in gamma whose coefficients are object sums
                           weighted by the illumination (object only) or patch sums
                           (joint); at n = 128 and 256 the far fields are stored for
                           the d > 0 pixels only.  Needs 2 (joint: 3) extra far fields
                           of workspace (ptyg_workspace_size counts them): k*n*n
                           complex64 each, or max_listed of them at n = 128 and 256. */
  int32_t estimator;    /* PTYG_EST_ML or PTYG_EST_LS */
  int64_t max_listed;   /* batched search at n = 128 and 256: capacity, in pixels, of the
                           compacted far-field regions, which hold only the pixels with
                           d > 0 (or NaN); < 0 reserves every pixel (k*n*n).  The
                           ptyg_listed_count of the data is the exact need; a solve whose
                           data list more pixels returns PTYG_E_WORKSPACE before it
                           writes them.  Ignored elsewhere. */
} ptyg_cg_opts;

enum { PTYG_LS_SEQUENTIAL = 0, PTYG_LS_BATCHED = 1 };

/* One row per completed iteration m of ptyg_cg_solve. */
typedef struct {
  double phi;       /* deviance form of Eq. ML at psi_m: sum d h((x-d)/d), h(u) = u - log(1+u) */
  double f_eq2;     /* Eq. ML at psi_m (2 d log|g| written as d log|g|^2), from the GRAD pass */
  double gamma;     /* accepted step gamma_m (0 if the line search failed) */
  double beta;      /* Dai-Yuan coefficient used for eta_m (0 on a restart) */
  double step_norm; /* ||psi_{m+1} - psi_m||_2 = gamma ||eta_m|| (the paper's convergence 2-norm) */
  int32_t halvings; /* index j of the accepted trial gamma0 tau^j (max_halvings if none passed):
                       the number of objective evaluations of the sequential search */
  int32_t restarted;/* 1 if eta_m = -grad_m (first iteration, bad denominator or failed search) */
} ptyg_cg_iter_stats;

/* Version of this ABI (increments on incompatible changes). */
int32_t ptyg_abi_version(void);
const char* ptyg_status_string(ptyg_status s);
/* Text of the last error raised on the calling thread ("" if none). */
const char* ptyg_last_error(void);

/* Bytes of workspace needed by every call below for these dims; `opts` may be
 * NULL (then the object-only solver with the sequential line search is
 * assumed).  Includes a transposed copy of the intensities (k*n*n floats)
 * for n = 256 and for the batched line search, and the stored far fields of
 * the batched line search when opts->line_search is PTYG_LS_BATCHED.  Returns 0 (error text set) for
 * invalid dims, and for the batched search when k*n*n >= 2^31 (it indexes the
 * intensities with 32-bit integers; ptyg_cg_solve rejects that case with
 * PTYG_E_INVAL). */
size_t ptyg_workspace_size(const ptyg_dims* dims, const ptyg_cg_opts* opts);

/* Number of pixels with d > 0 (or NaN) in data [k][n][n]: the listed pixels
 * whose far fields the batched line search stores (the others enter through
 * a polynomial in the step).  Synchronises `stream`; -1 on an error.  Uses a
 * counter inside the library (one per GPU): concurrent counts on one GPU
 * race. */
int64_t ptyg_listed_count(const ptyg_dims* dims, const float* data, ptyg_stream_t stream);

/* Checks that every scan position keeps its patch inside the object.
 * Synchronises `stream`.  Returns PTYG_OK or PTYG_E_BOUNDS. */
ptyg_status ptyg_check_positions(const ptyg_dims* dims, const int32_t* pos, void* ws, size_t ws_bytes,
                                 ptyg_stream_t stream);

/* Eq. fwd_model: far[k] = F(probe * obj[pos_k]) for every position.
 * obj [obj_h][obj_w], probe [n][n], pos [k][2], far [k][n][n] (written).
 * ws: workspace of ptyg_workspace_size() bytes, required for n = 256 (the
 * transform stages through it); may be NULL for n <= 128. */
ptyg_status ptyg_forward(const ptyg_dims* dims, const ptyg_c64* obj, const ptyg_c64* probe,
                         const int32_t* pos, ptyg_c64* far, void* ws, size_t ws_bytes, ptyg_stream_t stream);

/* G^H (text after Eq. gradient): obj_out = sum_k place_k(conj(probe) * F^H far[k]),
 * overwritten.  If probe_out != NULL (then obj must be given):
 * probe_out = sum_k conj(obj[pos_k]) * F^H far[k] (the adjoint of the map
 * probe -> G(obj, probe)).  Every output value is summed over k in a fixed
 * order (ascending k per object pixel), so results are bit-reproducible. */
ptyg_status ptyg_adjoint(const ptyg_dims* dims, const ptyg_c64* far, const ptyg_c64* probe,
                         const int32_t* pos, ptyg_c64* obj_out, const ptyg_c64* obj, ptyg_c64* probe_out,
                         void* ws, size_t ws_bytes, ptyg_stream_t stream);

/* GRAD stage (Eq. gradient, Wirtinger derivative dF/d conj(psi), no factor 2;
 * bit-reproducible like ptyg_adjoint):
 * grad_obj = G^H (g - d g / |g|^2) with g = G(obj) and the residual replaced
 * by g where |g|^2 < eps.  data: float32 intensities [k][n][n].
 * grad_probe (nullable): sum_k conj(obj[pos_k]) * F^H r_k.
 * objective (nullable, device double[2]): {deviance Phi, Eq. ML value F},
 * accumulated in FP64 with a fixed reduction order.  estimator: PTYG_EST_ML
 * (as above) or PTYG_EST_LS (residual g - sqrt(d) g / |g|, objective
 * sum (|g| - sqrt d)^2 in both slots). */
ptyg_status ptyg_grad(const ptyg_dims* dims, const ptyg_c64* obj, const ptyg_c64* probe,
                      const int32_t* pos, const float* data, float eps, int32_t estimator,
                      ptyg_c64* grad_obj, ptyg_c64* grad_probe, double* objective, void* ws,
                      size_t ws_bytes, ptyg_stream_t stream);

/* MINFUNC of Algorithm 1 (one line-search trial): objective (device
 * double[2], {Phi, F}) at obj + gamma*dir_obj and probe + gamma*dir_probe.
 * dir_obj / dir_probe may be NULL (no step in that block). */
ptyg_status ptyg_minfunc(const ptyg_dims* dims, const ptyg_c64* obj, const ptyg_c64* dir_obj,
                         const ptyg_c64* probe, const ptyg_c64* dir_probe, double gamma, const int32_t* pos,
                         const float* data, float eps, int32_t estimator, double* objective, void* ws,
                         size_t ws_bytes, ptyg_stream_t stream);

/* ptyg_minfunc without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, kernels and result as ptyg_minfunc
 * minus ws / ws_bytes.  Its per-workgroup partial sums live in a fixed
 * 1 MiB device array inside the library (65536 rows of two doubles, one row
 * per workgroup: k <= 65536 at n = 128, 131072 at n = 64, 524288 at n = 32,
 * 1048576 at n = 16); n = 256 and larger k return PTYG_E_INVAL.  Every call
 * on a GPU uses that GPU's one array: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.  The
 * array is written in full before it is read, so no clearing is needed.  It
 * allocates nothing. */
ptyg_status ptyg_minfunc_noalloc(const ptyg_dims* dims, const ptyg_c64* obj, const ptyg_c64* dir_obj,
                                 const ptyg_c64* probe, const ptyg_c64* dir_probe, double gamma, const int32_t* pos,
                                 const float* data, float eps, int32_t estimator, double* objective,
                                 ptyg_stream_t stream);

/* ML-CG reconstruction (Algorithm 1 on one GPU; Eqs. update, DaiYuan,
 * linesearch).  obj: in psi_0, out psi_iters.  probe: read, and updated when
 * opts->update_probe.  trace: HOST array of opts->iters rows (nullable).
 * iters_done: HOST (nullable).  Synchronous: it waits on `stream` once per
 * iteration and once per line-search trial (sequential search) or per pass of
 * up to 16 trials (batched search), a few bytes read back each time.
 * Returns PTYG_E_BOUNDS for a bad scan position, PTYG_E_NONFINITE if the
 * objective at an iterate is not finite (obj and probe then hold that
 * iterate: no update follows it), PTYG_E_WORKSPACE if the data list more pixels with
 * d > 0 than opts->max_listed reserved, and PTYG_E_INVAL for the batched
 * search on k*n*n >= 2^31 intensities. */
ptyg_status ptyg_cg_solve(const ptyg_dims* dims, ptyg_c64* obj, ptyg_c64* probe, const int32_t* pos,
                          const float* data, const ptyg_cg_opts* opts, void* ws, size_t ws_bytes,
                          ptyg_cg_iter_stats* trace, int32_t* iters_done, ptyg_stream_t stream);

/* Gradient descent (Eq. update2): obj_{m+1} = obj_m - gamma * grad F(obj_m)
 * with a constant step gamma >= 0 (the paper's slower baseline solver);
 * with update_probe the probe takes the same step along its gradient.
 * obj (and probe) are updated in place; phi_trace: HOST array of `iters`
 * doubles (nullable), the deviance Phi at obj_m from each GRAD pass.  Needs
 * the workspace of ptyg_cg_solve with the same update_probe and the
 * sequential line search.  The objectives are read back every 1024
 * iterations and at the end; a non-finite one returns PTYG_E_NONFINITE (the
 * iterates after it are then not meaningful). */
ptyg_status ptyg_gd_solve(const ptyg_dims* dims, ptyg_c64* obj, ptyg_c64* probe, const int32_t* pos,
                          const float* data, int32_t iters, double gamma, int32_t update_probe, float eps,
                          int32_t estimator, void* ws, size_t ws_bytes, double* phi_trace,
                          ptyg_stream_t stream);

/* Multi-view batch (3-D ptychography: many independent projections, which
 * the paper's introduction and outlook name as the larger use case; the
 * paper solves one projection at a time): `views` independent ML-CG solves
 * of equal shape run as one set of launches -- the views are stacked into
 * one object of views * obj_h rows, so the pattern kernels see views * k
 * patterns, and every reduction, direction, step and line-search decision
 * is per view.  Each view's iterates are those ptyg_cg_solve gives for it
 * alone, up to the order of floating-point sums.
 * dims: ONE view (obj_h, obj_w, n, k); n <= 128.  Each view's k patterns
 * are padded in the workspace to a multiple of the patterns per workgroup
 * (16 for n = 16, 8 for n = 32, 2 for n = 64) with k*n*n a multiple of 4096;
 * the padding patterns lie on n zero rows added below the stacked views,
 * with zero intensities, and contribute nothing.  With padding, the object
 * and the intensities are staged in the workspace and the iterates copied
 * back to obj before the call returns (also on an error return).
 * obj: [views][obj_h][obj_w] (in: psi_0, out: iterates); probe: [n][n],
 * shared and fixed (object-only); pos: [views][k][2], each inside its own
 * view's object; data: [views][k][n][n].  opts as for ptyg_cg_solve, with
 * update_probe = 0 and target_phi < 0.  trace: HOST [views][opts->iters]
 * rows (nullable); iters_done: HOST (nullable).  Workspace:
 * ptyg_views_workspace_size bytes (0 means invalid arguments). */
size_t ptyg_views_workspace_size(const ptyg_dims* dims, int32_t views, const ptyg_cg_opts* opts);
ptyg_status ptyg_cg_solve_views(const ptyg_dims* dims, int32_t views, ptyg_c64* obj, const ptyg_c64* probe,
                                const int32_t* pos, const float* data, const ptyg_cg_opts* opts, void* ws,
                                size_t ws_bytes, ptyg_cg_iter_stats* trace, int32_t* iters_done,
                                ptyg_stream_t stream);

/* Opt-in kernel timing for benchmarks: the fused GRAD kernel (kind 0), the
 * line-search kernel (kind 1: a MINFUNC pass, or a batched pass over stored
 * far fields), the forward transform of the search direction of the batched
 * line search (kind 2), the ordered overlap sum of the object gradient
 * (kind 3) and the whole GRAD stage -- transform kernel, overlap sum and
 * reductions, without the tile lists (kind 4) -- launched by the solver and
 * the GRAD call can be bracketed by HIP events on their stream.  `kinds_mask`: bit k times kind k (0 turns timing
 * off, -1 times every kind); each recorded event pair adds a few
 * microseconds between launches, so a timed run should time only the kinds
 * it reports.  ptyg_timing_read waits for the recorded events and returns,
 * per kind, the total elapsed milliseconds and the number of launches since
 * the last reset (arrays of `kinds` entries, kinds <= 5).  Timing is per
 * process and not thread-safe. */
void ptyg_timing_enable(int32_t kinds_mask);
void ptyg_timing_reset(void);
ptyg_status ptyg_timing_read(double* ms, int32_t* count, int32_t kinds);

/* Test hooks (no FFT): patches[k] = obj[pos_k] bit for bit; obj_out (zeroed
 * by the call) = sum_k place_k(patches[k]) with FP32 atomics. */
ptyg_status ptyg_debug_gather(const ptyg_dims* dims, const ptyg_c64* obj, const int32_t* pos,
                              ptyg_c64* patches, ptyg_stream_t stream);
ptyg_status ptyg_debug_scatter(const ptyg_dims* dims, const ptyg_c64* patches, const int32_t* pos,
                               ptyg_c64* obj_out, ptyg_stream_t stream);
/* Test hook: the GRAD stage (Eq. gradient) from a GIVEN far field g instead
 * of g = G(obj): the residual and objective terms, the inverse transform and
 * the ordered overlap sum run exactly as in ptyg_grad (the same kernels and
 * reductions).  far: [k][n][n] (the far field ptyg_forward would write);
 * grad_obj = Q^H F^H (g - d g / |g|^2) (residual g where |g|^2 < eps);
 * grad_probe (nullable, needs obj) and objective (nullable, device
 * double[2]) as for ptyg_grad; residual (nullable): [k][n][n], receives the
 * residual g - d g / |g|^2 itself.  Used to check the residual and adjoint
 * half of GRAD on an exactly known far field. */
ptyg_status ptyg_debug_grad_far(const ptyg_dims* dims, const ptyg_c64* far, const ptyg_c64* probe,
                                const int32_t* pos, const float* data, float eps, int32_t estimator,
                                ptyg_c64* grad_obj, const ptyg_c64* obj, ptyg_c64* grad_probe, double* objective,
                                ptyg_c64* residual, void* ws, size_t ws_bytes, ptyg_stream_t stream);
/* Test hook: the ordered overlap sum of the object gradient (the index part
 * of Q^H, text after Eq. gradient) as GRAD runs it -- tile lists built from
 * pos, then obj_out[y][x] = sum over the patterns k covering (y, x), in
 * ascending k, of conj(probe) * waves[k] at (y - r_k, x - c_k).
 * waves: [k][n*n] in the per-pattern layout GRAD stores: row-major
 * [u][v] for n <= 128; for n = 256 the polyphase layout, element (u, v) at
 * (2 (u & 1) + (v & 1)) n^2/4 + (u / 2) (n / 2) + v / 2.
 * probe: NULL for n <= 128 sums the waves themselves (GRAD's layout when no
 * probe gradient is wanted); required for n = 256.  obj_out is overwritten. */
ptyg_status ptyg_debug_tile_sum(const ptyg_dims* dims, const ptyg_c64* waves, const ptyg_c64* probe,
                                const int32_t* pos, ptyg_c64* obj_out, void* ws, size_t ws_bytes,
                                ptyg_stream_t stream);
/* Test hook: applies the lane exchange used by the split-line transforms to
 * two device float[64] arrays (lanes 32..63 of a <-> lanes 0..31 of b). */
ptyg_status ptyg_debug_lane_swap(float* a, float* b, ptyg_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PTYG_H */
