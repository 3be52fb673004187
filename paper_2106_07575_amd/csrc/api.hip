// C-ABI entry points of libptyg.so: argument validation, workspace layout,
// kernel sequencing and the ML-CG driver loop (Algorithm 1 on one GPU).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <numeric>
#include <vector>

#include "../../include/ptyg.h"
#include "kernels.hpp"

using namespace ptyg;

namespace {

thread_local std::string g_last_error;

ptyg_status fail(ptyg_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define PTYG_HIP(expr)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(PTYG_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr size_t kScalars = 64;
// Slots of the scalar region read back together once per line-search pass:
// solver scalars [0, 16), zero-pixel sums [16, 32), line-search row [32, 56).
constexpr int kZsSlot = 16, kLsSlot = 32;
// and the device's decision on the pass [56, 59): step, accepted trial, stop
constexpr int kAccSlot = kLsSlot + kLsRow;
static_assert(kAccSlot + 3 <= (int)kScalars, "scalar region too small");

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool n_supported(int n) { return n == 16 || n == 32 || n == 64 || n == 128 || n == 256; }

ptyg_status check_est(int32_t est) {
  if (est != PTYG_EST_ML && est != PTYG_EST_LS) return fail(PTYG_E_INVAL, "estimator=%d is not a PTYG_EST_* value", est);
  return PTYG_OK;
}

ptyg_status check_dims(const ptyg_dims* d) {
  if (!d) return fail(PTYG_E_INVAL, "dims is NULL");
  if (!n_supported(d->n)) return fail(PTYG_E_INVAL, "probe size n=%d not in {16,32,64,128,256}", d->n);
  if (d->k < 1) return fail(PTYG_E_INVAL, "k=%d must be >= 1", d->k);
  if (d->obj_h < d->n || d->obj_w < d->n)
    return fail(PTYG_E_INVAL, "object %dx%d smaller than the probe %d", d->obj_h, d->obj_w, d->n);
  if ((int64_t)d->obj_h * d->obj_w >= (int64_t(1) << 31))
    return fail(PTYG_E_INVAL, "object %dx%d too large", d->obj_h, d->obj_w);
  return PTYG_OK;
}

// Workspace regions (byte offsets, each 256-byte aligned).
constexpr int kGdTrace = 1024;  // objectives kept on the device between gradient-descent readbacks

struct Layout {
  size_t partials, scalars, gdtrace, flag, pparts, eta_obj, grad_obj, eta_probe, grad_probe, data_t, ubuf, toff, tlist,
      far_a, far_b, far_c, lsparts, lsphi, nz_counts, nz_offsets, nz_idx, zparts, zsums, illum, nz_seg, nz_dc, tparts,
      total;
  size_t nz_blocks, z_blocks;
  size_t n_partials;
  int64_t listed_cap;  // batched search: listed elements the compacted regions hold
};

// The regions of the batched line search come last, so the offsets of the
// others do not depend on it.
// `views`: the multi-view solver's stacked layout (no illumination or
// compacted far fields).
// `listed`: capacity for the elements with d > 0 (or NaN) that the batched
// search stores compacted (n = 128 and 256, single solve); < 0 means every
// element.
Layout layout(const ptyg_dims* d, bool joint, bool batched = false, bool views = false, int64_t listed = -1) {
  Layout L{};
  const size_t obj_n = (size_t)d->obj_h * d->obj_w;
  const size_t probe_n = (size_t)d->n * d->n;
  // partial (phi, f) pairs: pattern kernels use <= k + 8 blocks, a 256^2
  // GRAD pass grad256_blocks(k), vector kernels <= 2048
  L.n_partials = std::max<size_t>({(size_t)d->k + 16, 8192, d->n == 256 ? (size_t)grad256_blocks(d->k) : 0}) + 16;
  size_t o = 0;
  L.partials = o;
  o = align_up(o + L.n_partials * 2 * sizeof(double));
  L.scalars = o;
  o = align_up(o + kScalars * sizeof(double));
  L.gdtrace = o;  // slot i gets (Phi, F) of iteration i; the next iteration overwrites F
  o = align_up(o + (kGdTrace + 1) * sizeof(double));
  L.flag = o;
  o = align_up(o + sizeof(int));
  L.pparts = o;
  o = align_up(o + (size_t)kProbeChunks * probe_n * sizeof(float2));
  L.eta_obj = o;
  o = align_up(o + obj_n * sizeof(float2));
  L.grad_obj = o;
  o = align_up(o + obj_n * sizeof(float2));
  L.eta_probe = o;
  o = align_up(o + (joint ? probe_n : 1) * sizeof(float2));
  L.grad_probe = o;
  o = align_up(o + (joint ? probe_n : 1) * sizeof(float2));
  // per-pattern transposed intensities: read by the 256^2 radix stage and
  // the batched search's compaction only
  L.data_t = o;
  o = align_up(o + (batched || d->n == 256 ? (size_t)d->k * probe_n : 1) * sizeof(float));
  L.ubuf = o;
  o = align_up(o + (size_t)d->k * probe_n * sizeof(float2));
  const size_t T = (size_t)tiles_x(d->obj_w) * tiles_y(d->obj_h);
  L.toff = o;
  o = align_up(o + (T + 1) * sizeof(int));
  L.tlist = o;
  o = align_up(o + tile_list_ints(d->k, d->obj_h, d->obj_w, d->n) * sizeof(int));
  L.tparts = o;  // per-tile (|grad|^2, Re<eta, grad>) rows of the overlap sum
  o = align_up(o + 2 * T * sizeof(double));
  L.far_a = L.far_b = L.far_c = L.lsparts = L.lsphi = L.nz_counts = L.nz_offsets = L.nz_idx = L.zparts = L.zsums = 0;
  L.illum = L.nz_seg = L.nz_dc = 0;
  L.nz_blocks = L.z_blocks = 0;
  if (batched) {
    const size_t elems = (size_t)d->k * probe_n;
    // compacted stores: far fields, indices and intensities of the listed
    // elements only, so those regions scale with the listed count
    const bool compact = !views && (d->n == 128 || d->n == 256);
    const size_t cap = (compact && listed >= 0 && (size_t)listed < elems) ? (size_t)listed : elems;
    L.nz_blocks = (elems + kNzChunk - 1) / kNzChunk;
    L.z_blocks = (size_t)fwd_t_blocks(d->n, d->k);
    L.nz_counts = o;
    o = align_up(o + L.nz_blocks * sizeof(int));
    L.nz_offsets = o;
    o = align_up(o + (L.nz_blocks + 1) * sizeof(int));
    L.nz_idx = o;
    o = align_up(o + std::max<size_t>(cap, 1) * sizeof(int));
    // GRAD sums of |G psi|^2 (one per block), then the rows of the direction
    // sums (object only the DIR kernel's, joint the patch sums')
    L.zparts = o;
    // (256^2 joint: the direction forward's per-block patch sums, 2 rows of
    // its 4 k blocks)
    const size_t rows = std::max<size_t>({2 * L.z_blocks, (size_t)vec_blocks((int64_t)obj_n),
                                          2 * (size_t)patch_sums_blocks(d->k, d->n),
                                          d->n == 256 ? 8 * (size_t)d->k : 0});
    o = align_up(o + (L.n_partials + rows * 4) * sizeof(double));
    L.zsums = L.scalars + kZsSlot * sizeof(double);
    const size_t far_bytes = std::max<size_t>(cap, 1) * sizeof(float2);
    L.far_a = o;
    o = align_up(o + far_bytes);
    L.far_b = o;
    o = align_up(o + far_bytes);
    if (joint) {
      L.far_c = o;
      o = align_up(o + far_bytes);
    }
    L.lsparts = o;
    o = align_up(o + (size_t)kLsBlocks * kLsRow * sizeof(double));
    L.lsphi = L.scalars + kLsSlot * sizeof(double);
    if (!joint && !views) {
      // illumination sum_k |p(x - s_k)|^2: with the probe fixed, G^H G is
      // this diagonal, so Re<G psi, G eta> and ||G eta||^2 are object sums
      L.illum = o;
      o = align_up(o + obj_n * sizeof(float2));
    }
    if (!views && (d->n == 128 || d->n == 256)) {
      // far fields stored for the listed elements only (the d <= 0 part of
      // the search comes from sums formed elsewhere): segment records and
      // the listed intensities, compacted
      L.nz_seg = o;
      o = align_up(o + elems / 32 * sizeof(uint2));
      L.nz_dc = o;
      o = align_up(o + std::max<size_t>(cap, 1) * sizeof(float));
    }
  }
  L.total = o;
  L.listed_cap = batched ? (int64_t)((!views && (d->n == 128 || d->n == 256) && listed >= 0 &&
                                      listed < (int64_t)d->k * d->n * d->n)
                                         ? listed
                                         : (int64_t)d->k * d->n * d->n)
                         : 0;
  return L;
}

// The batched line search indexes the k n^2 intensities (and its listed
// elements) with 32-bit integers.
ptyg_status check_batched_size(const ptyg_dims* d) {
  if ((int64_t)d->k * d->n * d->n >= (int64_t(1) << 31))
    return fail(PTYG_E_INVAL, "k*n*n=%lld intensities: the batched line search takes fewer than 2^31 "
                "(use the sequential search)", (long long)d->k * d->n * d->n);
  return PTYG_OK;
}

ptyg_status check_ws(const ptyg_dims* d, void* ws, size_t ws_bytes, bool joint, Layout* out,
                     bool batched = false, int64_t listed = -1) {
  if (batched)
    if (ptyg_status st = check_batched_size(d)) return st;
  *out = layout(d, joint, batched, false, listed);
  if (!ws) return fail(PTYG_E_INVAL, "workspace is NULL");
  if (((uintptr_t)ws) % kAlign) return fail(PTYG_E_INVAL, "workspace not 256-byte aligned");
  if (ws_bytes < out->total)
    return fail(PTYG_E_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, out->total);
  return PTYG_OK;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

PatArgs base_args(const ptyg_dims* d) {
  PatArgs a{};
  a.H = d->obj_h;
  a.W = d->obj_w;
  a.K = d->k;
  a.N = d->n;
  a.eps = 1e-32f;
  return a;
}

hipStream_t S(ptyg_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

// ---- opt-in kernel timing (HIP events around the pattern kernels)
struct Timing {
  int mask = 0;  // bit k: time kind k
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  static constexpr int kKinds = 5;
  double ms[kKinds] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int count[kKinds] = {0, 0, 0, 0, 0};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    // device-scope events: a system-scope release at every record would
    // write back the caches between the timed kernels
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
  }
  // waits for every recorded pair and accumulates it
  void drain() {
    for (Rec& r : pending) {
      float t = 0.0f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.kind] += t;
        count[r.kind] += 1;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
};
Timing g_timing;

// Host side of the solver's scalar readbacks: pinned, so that a copy is
// asynchronous and one stream synchronisation covers it (a copy into pageable
// memory is staged and waits by itself).  One buffer per host thread,
// allocated on its first solve and freed when the thread ends (every solve
// has synchronised its stream before it returns, so no copy is pending).
struct PinnedScalars {
  double* p = nullptr;
  ~PinnedScalars() {
    if (p) (void)hipHostFree(p);
  }
};

double* readback_buffer() {
  thread_local PinnedScalars buf;
  if (!buf.p) {
    void* p = nullptr;
    if (hipHostMalloc(&p, kScalars * sizeof(double), hipHostMallocDefault) != hipSuccess) return nullptr;
    buf.p = static_cast<double*>(p);
  }
  return buf.p;
}

struct TimedLaunch {
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  TimedLaunch(int k, hipStream_t st) : kind(k), s(st) {
    if (!((g_timing.mask >> kind) & 1)) return;
    a = g_timing.get();
    b = g_timing.get();
    if (a && b) hipEventRecord(a, s);
  }
  ~TimedLaunch() {
    if (!a || !b) return;
    hipEventRecord(b, s);
    g_timing.pending.push_back({kind, a, b});
  }
};

// Counter of ptyg_listed_count (one per GPU; concurrent counts on one GPU race).
static __device__ unsigned long long listed_counter;

// Workspace-free objective pass (ptyg_minfunc_noalloc): its per-workgroup
// (Phi, F) partials live in this file-scope device array instead of a
// caller workspace.  Each GPU holds its own copy until the process ends; host
// code must use the per-device address from hipGetSymbolAddress, never the
// array's name (a host-side stand-in).
constexpr int kNoAllocMaxBlocks = 65536;
static __device__ __align__(256) double scratch[2 * kNoAllocMaxBlocks];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
ptyg_status scratch_address(double** out) {
  static std::mutex mu;
  static std::vector<double*> addr;
  int dev = 0;
  PTYG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    PTYG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PTYG_E_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
    addr[dev] = static_cast<double*>(p);
  }
  *out = addr[dev];
  return PTYG_OK;
}

}  // namespace

extern "C" {

int32_t ptyg_abi_version(void) { return 5; }

const char* ptyg_status_string(ptyg_status s) {
  switch (s) {
    case PTYG_OK: return "ok";
    case PTYG_E_INVAL: return "invalid argument";
    case PTYG_E_BOUNDS: return "scan position outside the object";
    case PTYG_E_HIP: return "HIP error";
    case PTYG_E_NONFINITE: return "non-finite objective";
    case PTYG_E_WORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

const char* ptyg_last_error(void) { return g_last_error.c_str(); }

size_t ptyg_workspace_size(const ptyg_dims* dims, const ptyg_cg_opts* opts) {
  if (check_dims(dims) != PTYG_OK) return 0;
  if (opts && opts->line_search != PTYG_LS_SEQUENTIAL && opts->line_search != PTYG_LS_BATCHED) {
    fail(PTYG_E_INVAL, "line_search=%d is not a PTYG_LS_* value", opts->line_search);
    return 0;
  }
  const bool batched = opts && opts->line_search == PTYG_LS_BATCHED;
  if (batched && check_batched_size(dims) != PTYG_OK) return 0;
  return layout(dims, opts && opts->update_probe, batched, false, opts ? opts->max_listed : -1).total;
}

int64_t ptyg_listed_count(const ptyg_dims* dims, const float* data, ptyg_stream_t stream) {
  if (check_dims(dims) != PTYG_OK) return -1;
  if (!data) {
    fail(PTYG_E_INVAL, "data is NULL");
    return -1;
  }
  unsigned long long* cnt = nullptr;
  if (hipGetSymbolAddress((void**)&cnt, HIP_SYMBOL(listed_counter)) != hipSuccess || !cnt) {
    fail(PTYG_E_HIP, "hipGetSymbolAddress(listed_counter): %s", hipGetErrorString(hipGetLastError()));
    return -1;
  }
  const hipStream_t s = S(stream);
  unsigned long long h = 0;
  if (launch_count_listed(data, (int64_t)dims->k * dims->n * dims->n, cnt, s) != hipSuccess ||
      hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    fail(PTYG_E_HIP, "counting the listed pixels: %s", hipGetErrorString(hipGetLastError()));
    return -1;
  }
  return (int64_t)h;
}

ptyg_status ptyg_check_positions(const ptyg_dims* dims, const int32_t* pos, void* ws, size_t ws_bytes,
                                 ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (!pos) return fail(PTYG_E_INVAL, "pos is NULL");
  Layout L;
  if (ptyg_status st = check_ws(dims, ws, ws_bytes, false, &L)) return st;
  int* flag = at<int>(ws, L.flag);
  PTYG_HIP(launch_fill_i32(flag, 1, 0, S(stream)));
  PTYG_HIP(launch_check_positions(reinterpret_cast<const int2*>(pos), dims->k, dims->obj_h, dims->obj_w,
                                  dims->n, flag, S(stream)));
  int h = 0;
  PTYG_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, S(stream)));
  PTYG_HIP(hipStreamSynchronize(S(stream)));
  if (h) return fail(PTYG_E_BOUNDS, "a scan position puts its patch outside the %dx%d object", dims->obj_h,
                     dims->obj_w);
  return PTYG_OK;
}

ptyg_status ptyg_forward(const ptyg_dims* dims, const ptyg_c64* obj, const ptyg_c64* probe,
                         const int32_t* pos, ptyg_c64* far, void* ws, size_t ws_bytes, ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (!obj || !probe || !pos || !far) return fail(PTYG_E_INVAL, "NULL array argument");
  PatArgs a = base_args(dims);
  a.obj = reinterpret_cast<const float2*>(obj);
  a.probe = reinterpret_cast<const float2*>(probe);
  a.pos = reinterpret_cast<const int2*>(pos);
  a.far = reinterpret_cast<float2*>(far);
  if (dims->n == 256) {
    Layout L;
    if (ptyg_status st = check_ws(dims, ws, ws_bytes, false, &L)) return st;
    a.ubuf = at<float2>(ws, L.ubuf);
  }
  PTYG_HIP(launch_forward(a, S(stream)));
  return PTYG_OK;
}

ptyg_status ptyg_adjoint(const ptyg_dims* dims, const ptyg_c64* far, const ptyg_c64* probe,
                         const int32_t* pos, ptyg_c64* obj_out, const ptyg_c64* obj, ptyg_c64* probe_out,
                         void* ws, size_t ws_bytes, ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (!far || !probe || !pos || !obj_out) return fail(PTYG_E_INVAL, "NULL array argument");
  if (probe_out && !obj) return fail(PTYG_E_INVAL, "probe_out requires obj");
  Layout L;
  if (ptyg_status st = check_ws(dims, ws, ws_bytes, false, &L)) return st;
  const hipStream_t s = S(stream);
  PatArgs a = base_args(dims);
  a.far = const_cast<float2*>(reinterpret_cast<const float2*>(far));
  a.probe = reinterpret_cast<const float2*>(probe);
  a.pos = reinterpret_cast<const int2*>(pos);
  a.obj = reinterpret_cast<const float2*>(obj);
  a.ubuf = at<float2>(ws, L.ubuf);
  // conj(p) folded into the stored waves unless the probe adjoint needs them plain
  a.premul = !probe_out && dims->n <= 128;
  PTYG_HIP(launch_tile_lists(a.pos, dims->k, dims->obj_h, dims->obj_w, dims->n, at<int>(ws, L.toff),
                             at<int>(ws, L.tlist), s));
  PTYG_HIP(launch_adjoint(a, s));
  PTYG_HIP(launch_tile_sum(a.ubuf, a.premul ? nullptr : a.probe, a.pos, at<int>(ws, L.toff), at<int>(ws, L.tlist),
                           dims->k, dims->obj_h, dims->obj_w, dims->n, reinterpret_cast<float2*>(obj_out), s));
  if (probe_out)
    PTYG_HIP(launch_probe_grad(a.ubuf, a.obj, a.pos, dims->k, dims->obj_w, dims->n, at<float2>(ws, L.pparts),
                               reinterpret_cast<float2*>(probe_out), s));
  return PTYG_OK;
}

namespace {
// One fused GRAD pass; writes {phi, f} to `objective` (device) when given.
// The tile lists of `pos` must already be in the workspace.
ptyg_status run_grad(const ptyg_dims* dims, const float2* obj, const float2* probe, const int2* pos,
                     const float* data, DataLayout lay, float eps, int est, float2* grad_obj, float2* grad_probe,
                     double* objective, void* ws, const Layout& L, hipStream_t s, float2* gstore = nullptr,
                     double* gsum = nullptr, const uint2* cseg = nullptr, const float2* dot_b = nullptr,
                     double* dot_out = nullptr, const float2* far_in = nullptr, float2* res_out = nullptr,
                     bool want_f = true) {
  PatArgs a = base_args(dims);
  a.est = est;
  a.want_f = want_f ? 1 : 0;
  if (dims->n == 256 && lay == DataLayout::Rows && !far_in) {
    // the 256^2 radix stage reads intensities coalesced only per pattern
    // transposed: transpose once into the workspace
    float* dt = at<float>(ws, L.data_t);
    PTYG_HIP(launch_transpose_data(data, dt, dims->k, dims->n, s));
    data = dt;
    lay = DataLayout::Transposed;
  }
  a.gstore = gstore;
  a.cseg = cseg;
  if (gstore) a.zs_part = at<double>(ws, L.zparts);
  a.obj = obj;
  a.probe = probe;
  a.pos = pos;
  a.data = data;
  a.eps = eps;
  a.ubuf = at<float2>(ws, L.ubuf);
  a.partials = at<double>(ws, L.partials);
  // conj(p) folded into the stored waves unless the probe gradient needs them plain
  a.premul = !grad_probe && dims->n <= 128;
  int nb = 0;
  // kind 4: the whole GRAD stage (transform kernel, overlap sum, reductions)
  TimedLaunch tl_unit(4, s);
  if (far_in) {
    // test hook: the far field is given (row layout)
    a.far = const_cast<float2*>(far_in);
    a.gstore = res_out;
    PTYG_HIP(launch_grad_far(a, &nb, s));
  } else {
    TimedLaunch tl(0, s);
    PTYG_HIP(launch_grad(a, lay, &nb, s));
  }
  double* tparts = dot_out ? at<double>(ws, L.tparts) : nullptr;
  {
    TimedLaunch tl(3, s);
    PTYG_HIP(launch_tile_sum(a.ubuf, a.premul ? nullptr : probe, pos, at<int>(ws, L.toff), at<int>(ws, L.tlist),
                             dims->k, dims->obj_h, dims->obj_w, dims->n, grad_obj, s, dot_b, tparts));
  }
  {
    // (phi, f), for the batched search sum |G psi|^2, and the overlap sum's
    // (||grad||^2, Re<dot_b, grad>): one launch
    FinJob jobs[3];
    int nj = 0;
    if (objective) jobs[nj++] = FinJob{a.partials, nb, 2, objective};
    if (gstore && gsum) jobs[nj++] = FinJob{a.zs_part, nb, 1, gsum};
    if (dot_out) jobs[nj++] = FinJob{tparts, tiles_x(dims->obj_w) * tiles_y(dims->obj_h), 2, dot_out};
    if (nj) PTYG_HIP(launch_finalize_n(jobs, nj, s));
  }
  if (grad_probe)
    PTYG_HIP(launch_probe_grad(a.ubuf, obj, pos, dims->k, dims->obj_w, dims->n, at<float2>(ws, L.pparts),
                               grad_probe, s));
  return PTYG_OK;
}

ptyg_status build_tiles(const ptyg_dims* dims, const int2* pos, void* ws, const Layout& L, hipStream_t s) {
  PTYG_HIP(launch_tile_lists(pos, dims->k, dims->obj_h, dims->obj_w, dims->n, at<int>(ws, L.toff),
                             at<int>(ws, L.tlist), s));
  return PTYG_OK;
}

ptyg_status run_minfunc(const ptyg_dims* dims, const float2* obj, const float2* dobj, const float2* probe,
                        const float2* dprobe, double gamma, const int2* pos, const float* data, DataLayout lay,
                        float eps, int est, double* objective, void* ws, const Layout& L, hipStream_t s,
                        bool want_f = true) {
  PatArgs a = base_args(dims);
  a.est = est;
  a.want_f = want_f ? 1 : 0;
  if (dims->n == 256 && lay == DataLayout::Rows) {
    float* dt = at<float>(ws, L.data_t);
    PTYG_HIP(launch_transpose_data(data, dt, dims->k, dims->n, s));
    data = dt;
    lay = DataLayout::Transposed;
  }
  a.obj = obj;
  a.dobj = dobj;
  a.probe = probe;
  a.dprobe = dprobe;
  a.gamma = (float)gamma;
  a.pos = pos;
  a.data = data;
  a.eps = eps;
  a.partials = at<double>(ws, L.partials);
  a.ubuf = at<float2>(ws, L.ubuf);  // staging of the 256^2 transforms
  int nb = 0;
  {
    TimedLaunch tl(1, s);
    PTYG_HIP(launch_minfunc(a, lay, &nb, s));
  }
  PTYG_HIP(launch_finalize(a.partials, nb, 2, objective, s));
  return PTYG_OK;
}
}  // namespace

ptyg_status ptyg_grad(const ptyg_dims* dims, const ptyg_c64* obj, const ptyg_c64* probe, const int32_t* pos,
                      const float* data, float eps, int32_t estimator, ptyg_c64* grad_obj, ptyg_c64* grad_probe,
                      double* objective, void* ws, size_t ws_bytes, ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (!obj || !probe || !pos || !data || !grad_obj) return fail(PTYG_E_INVAL, "NULL array argument");
  if (!(eps >= 0.0f)) return fail(PTYG_E_INVAL, "eps must be >= 0");
  if (ptyg_status st = check_est(estimator)) return st;
  Layout L;
  if (ptyg_status st = check_ws(dims, ws, ws_bytes, false, &L)) return st;
  if (ptyg_status st = build_tiles(dims, reinterpret_cast<const int2*>(pos), ws, L, S(stream))) return st;
  return run_grad(dims, reinterpret_cast<const float2*>(obj), reinterpret_cast<const float2*>(probe),
                  reinterpret_cast<const int2*>(pos), data, DataLayout::Rows, eps, estimator,
                  reinterpret_cast<float2*>(grad_obj), reinterpret_cast<float2*>(grad_probe), objective, ws, L,
                  S(stream), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, objective != nullptr);
}

ptyg_status ptyg_minfunc(const ptyg_dims* dims, const ptyg_c64* obj, const ptyg_c64* dir_obj,
                         const ptyg_c64* probe, const ptyg_c64* dir_probe, double gamma, const int32_t* pos,
                         const float* data, float eps, int32_t estimator, double* objective, void* ws,
                         size_t ws_bytes, ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (!obj || !probe || !pos || !data || !objective) return fail(PTYG_E_INVAL, "NULL array argument");
  if (!std::isfinite(gamma)) return fail(PTYG_E_INVAL, "gamma not finite");
  if (ptyg_status st = check_est(estimator)) return st;
  Layout L;
  if (ptyg_status st = check_ws(dims, ws, ws_bytes, false, &L)) return st;
  return run_minfunc(dims, reinterpret_cast<const float2*>(obj), reinterpret_cast<const float2*>(dir_obj),
                     reinterpret_cast<const float2*>(probe), reinterpret_cast<const float2*>(dir_probe), gamma,
                     reinterpret_cast<const int2*>(pos), data, DataLayout::Rows, eps, estimator, objective, ws, L,
                     S(stream));
}

ptyg_status ptyg_minfunc_noalloc(const ptyg_dims* dims, const ptyg_c64* obj, const ptyg_c64* dir_obj,
                                 const ptyg_c64* probe, const ptyg_c64* dir_probe, double gamma, const int32_t* pos,
                                 const float* data, float eps, int32_t estimator, double* objective,
                                 ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (!obj || !probe || !pos || !data || !objective) return fail(PTYG_E_INVAL, "NULL array argument");
  if (!std::isfinite(gamma)) return fail(PTYG_E_INVAL, "gamma not finite");
  if (!(eps >= 0.0f)) return fail(PTYG_E_INVAL, "eps must be >= 0");
  if (ptyg_status st = check_est(estimator)) return st;
  if (dims->n > 128)
    return fail(PTYG_E_INVAL, "ptyg_minfunc_noalloc supports n <= 128 (n = 256 stages every pattern through a workspace)");
  const int ppw = patterns_per_block(dims->n);
  const int64_t groups = ((int64_t)dims->k + ppw - 1) / ppw;
  const int64_t blocks = 8 * ((groups + 7) / 8);
  if (blocks > kNoAllocMaxBlocks)
    return fail(PTYG_E_INVAL, "k=%d needs %lld partial rows; ptyg_minfunc_noalloc holds at most %d (k <= %lld at n=%d)",
                dims->k, (long long)blocks, kNoAllocMaxBlocks, (long long)kNoAllocMaxBlocks * ppw, dims->n);
  double* sp = nullptr;
  if (ptyg_status st = scratch_address(&sp)) return st;
  PatArgs a = base_args(dims);
  a.est = estimator;
  a.obj = reinterpret_cast<const float2*>(obj);
  a.dobj = reinterpret_cast<const float2*>(dir_obj);
  a.probe = reinterpret_cast<const float2*>(probe);
  a.dprobe = reinterpret_cast<const float2*>(dir_probe);
  a.gamma = (float)gamma;
  a.pos = reinterpret_cast<const int2*>(pos);
  a.data = data;
  a.eps = eps;
  a.partials = sp;
  a.want_f = 1;
  int nb = 0;
  PTYG_HIP(launch_minfunc(a, DataLayout::Rows, &nb, S(stream)));
  PTYG_HIP(launch_finalize(sp, nb, 2, objective, S(stream)));
  return PTYG_OK;
}

ptyg_status ptyg_cg_solve(const ptyg_dims* dims, ptyg_c64* obj_c, ptyg_c64* probe_c, const int32_t* pos_i,
                          const float* data, const ptyg_cg_opts* opts, void* ws, size_t ws_bytes,
                          ptyg_cg_iter_stats* trace, int32_t* iters_done, ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (!obj_c || !probe_c || !pos_i || !data || !opts) return fail(PTYG_E_INVAL, "NULL argument");
  if (opts->iters < 0) return fail(PTYG_E_INVAL, "iters < 0");
  if (!(opts->tau > 0.0 && opts->tau < 1.0)) return fail(PTYG_E_INVAL, "tau must be in (0, 1)");
  if (!(opts->gamma0 > 0.0) || !std::isfinite(opts->gamma0)) return fail(PTYG_E_INVAL, "gamma0 must be > 0");
  if (opts->max_halvings < 1) return fail(PTYG_E_INVAL, "max_halvings must be >= 1");
  if (!(opts->eps >= 0.0)) return fail(PTYG_E_INVAL, "eps must be >= 0");
  if (opts->line_search != PTYG_LS_SEQUENTIAL && opts->line_search != PTYG_LS_BATCHED)
    return fail(PTYG_E_INVAL, "line_search=%d is not a PTYG_LS_* value", opts->line_search);
  if (ptyg_status st = check_est(opts->estimator)) return st;
  const int est = opts->estimator;
  const bool joint = opts->update_probe != 0;
  const bool batched = opts->line_search == PTYG_LS_BATCHED;
  Layout L;
  if (ptyg_status st = check_ws(dims, ws, ws_bytes, joint, &L, batched, opts->max_listed)) return st;
  if (iters_done) *iters_done = 0;
  if (ptyg_status st = ptyg_check_positions(dims, pos_i, ws, ws_bytes, stream)) return st;

  const hipStream_t s = S(stream);
  float2* obj = reinterpret_cast<float2*>(obj_c);
  float2* probe = reinterpret_cast<float2*>(probe_c);
  const int2* pos = reinterpret_cast<const int2*>(pos_i);
  const int64_t on = (int64_t)dims->obj_h * dims->obj_w;
  const int64_t pn = (int64_t)dims->n * dims->n;
  float2* eta_o = at<float2>(ws, L.eta_obj);
  float2* grad_o = at<float2>(ws, L.grad_obj);
  float2* eta_p = joint ? at<float2>(ws, L.eta_probe) : nullptr;
  float2* grad_p = joint ? at<float2>(ws, L.grad_probe) : nullptr;
  float* dt = at<float>(ws, L.data_t);
  double* partials = at<double>(ws, L.partials);
  double* sc = at<double>(ws, L.scalars);
  const float eps = (float)opts->eps;
  float2* far_a = batched ? at<float2>(ws, L.far_a) : nullptr;  // G psi_m (from the GRAD pass)
  float2* far_b = batched ? at<float2>(ws, L.far_b) : nullptr;  // first-order far field of the direction
  float2* far_c = batched && joint ? at<float2>(ws, L.far_c) : nullptr;  // G(eta_p, eta) (joint)
  double* lsparts = batched ? at<double>(ws, L.lsparts) : nullptr;
  double* lsphi = batched ? at<double>(ws, L.lsphi) : nullptr;
  int last_trials = kLsBatch;  // batched search: the previous accepted index sizes the first pass

  // The transform kernels of n <= 128 read the intensities as given (a
  // lane's four consecutive frequencies are one 16-byte load); the 256^2
  // radix stage and the compaction of the batched search read them per
  // pattern transposed, from a copy made once
  const bool big = dims->n == 256;
  if (batched || big) PTYG_HIP(launch_transpose_data(data, dt, dims->k, dims->n, s));
  const float* dgrad = big ? dt : data;
  const DataLayout lgrad = big ? DataLayout::Transposed : DataLayout::Rows;
  if (ptyg_status st = build_tiles(dims, pos, ws, L, s)) return st;
  float2* illum = batched && !joint ? at<float2>(ws, L.illum) : nullptr;
  // n = 128 and 256: G psi, G eta (and G(eta_p eta)) are stored for the listed elements only
  uint2* cseg = L.nz_seg ? at<uint2>(ws, L.nz_seg) : nullptr;
  float* dcomp = L.nz_dc ? at<float>(ws, L.nz_dc) : nullptr;
  if (illum)
    PTYG_HIP(launch_illum(probe, pos, at<int>(ws, L.toff), at<int>(ws, L.tlist), dims->obj_h, dims->obj_w, dims->n,
                          illum, s));
  // batched line search: the elements with d > 0 (or NaN) are evaluated per
  // trial; the d <= 0 ones through the zero-pixel sums
  int64_t nnz = 0;
  if (batched) {
    // count the listed elements first: the compacted regions hold at most
    // L.listed_cap of them
    int* offs = at<int>(ws, L.nz_offsets);
    const int64_t elems = (int64_t)dims->k * dims->n * dims->n;
    PTYG_HIP(launch_nz_count(dt, elems, at<int>(ws, L.nz_counts), offs, s));
    int h_nnz = 0;
    PTYG_HIP(hipMemcpyAsync(&h_nnz, offs + L.nz_blocks, sizeof(int), hipMemcpyDeviceToHost, s));
    PTYG_HIP(hipStreamSynchronize(s));
    nnz = h_nnz;
    if (nnz > L.listed_cap)
      return fail(PTYG_E_WORKSPACE, "the data list %lld pixels with d > 0 but the workspace was sized for %lld "
                  "(opts->max_listed)", (long long)nnz, (long long)L.listed_cap);
    PTYG_HIP(launch_nz_fill(dt, elems, offs, at<int>(ws, L.nz_idx), cseg, dcomp, s));
  }

  // scalar slots
  enum {
    PHI = 0, FEQ = 1, N1O = 2, N2O = 3, N1P = 4, N2P = 5, N3O = 6, EEO = 7, N3P = 8, EEP = 9,
    PHIT = 10,  // a trial's (Phi, F): two slots
    BETA = 12, RST = 13,
    DCONST = 15  // sum over d > 0 of d - d log d: Eq. ML's F = Phi + this
  };
  // the GRAD passes form the deviance only; Eq. ML's value for the trace is
  // Phi plus the data constant, summed once here and read back with the
  // first iteration's scalars
  PTYG_HIP(launch_data_const(data, (int64_t)dims->k * dims->n * dims->n, 1, partials, sc + DCONST, s));
  double* h = readback_buffer();
  if (!h) return fail(PTYG_E_HIP, "pinned readback buffer: %s", hipGetErrorString(hipGetLastError()));
  struct EventGuard {
    hipEvent_t e = nullptr;
    ~EventGuard() {
      if (e) (void)hipEventDestroy(e);
    }
  } rb;
  if (batched) PTYG_HIP(hipEventCreateWithFlags(&rb.e, hipEventDisableTiming));
  hipEvent_t rb_ev = rb.e;
  // every return, the error returns included, leaves no copy into h in flight
  struct StreamDrain {
    hipStream_t s;
    ~StreamDrain() { (void)hipStreamSynchronize(s); }
  } drain{s};
  bool restart = true;
  const int nvb_o = vec_blocks(on), nvb_p = vec_blocks(pn);
  // the direction update reads its coefficient from the device: start from a
  // finite (zero) direction
  PTYG_HIP(launch_zero(eta_o, on, s));
  if (joint) PTYG_HIP(launch_zero(eta_p, pn, s));

  for (int m = 0; m < opts->iters; ++m) {
    // GRAD stage
    // the overlap sum also forms ||g_m||^2 and Re<eta_{m-1}, g_m> (sc[N1O], sc[N2O])
    if (ptyg_status st = run_grad(dims, obj, probe, pos, dgrad, lgrad, eps, est, grad_o, grad_p, sc + PHI, ws, L, s,
                                  far_a, batched ? at<double>(ws, L.zsums) : nullptr, cseg, restart ? nullptr : eta_o,
                                  sc + N1O, nullptr, nullptr, false))
      return st;
    bool applied = false;  // the update was applied with the device's step
    if (joint) {
      VecArgs vp{};
      vp.n = pn;
      vp.a = grad_p;
      vp.b = restart ? nullptr : eta_p;
      vp.partials = partials;
      PTYG_HIP(launch_dot2(vp, s));
      PTYG_HIP(launch_finalize(partials, nvb_p, 2, sc + N1P, s));
    }

    // DIR stage (Eq. DaiYuan) on the device: beta = ||g_m||^2 /
    // Re<eta_{m-1}, g_m - g_{m-1}> (sc[N3O] still holds Re<eta_{m-1}, g_{m-1}>),
    // restart on a failed search or a bad denominator; no host round trip
    VecArgs v{};
    v.n = on;
    v.a = grad_o;
    v.b = eta_o;
    v.partials = partials;
    if (joint) {
      // both blocks' directions take the coefficient from the object and
      // probe scalars together
      PTYG_HIP(launch_dy_beta(sc, N1O, N2O, N3O, 2, BETA, RST, restart ? 1 : 0, s));
      v.alpha_dev = sc + BETA;
      v.restart_dev = sc + RST;
    } else {
      // the direction kernel forms the coefficient itself
      v.dy_n1 = sc + N1O;
      v.dy_n2 = sc + N2O;
      v.dy_n3 = sc + N3O;
      v.dy_out = sc + BETA;
      v.dy_restart = restart ? 1 : 0;
    }
    if (illum) {
      // Re<G psi, G eta> and ||G eta||^2 for the batched search, as
      // illumination-weighted object sums (rows of 4 like the direction
      // forward's sums)
      v.zs_psi = obj;
      v.zs_w = illum;
      v.zs_part = at<double>(ws, L.zparts) + L.n_partials;
    }
    PTYG_HIP(launch_dir(v, s));
    {
      const FinJob a{partials, nvb_o, 2, sc + N3O};
      const FinJob b{v.zs_part, nvb_o, 4, at<double>(ws, L.zsums) + 4};
      PTYG_HIP(launch_finalize2(a, b, illum ? 2 : 1, s));
    }
    if (joint) {
      VecArgs vp{};
      vp.n = pn;
      vp.a = grad_p;
      vp.b = eta_p;
      vp.alpha_dev = sc + BETA;
      vp.restart_dev = sc + RST;
      vp.partials = partials;
      PTYG_HIP(launch_dir(vp, s));
      PTYG_HIP(launch_finalize(partials, nvb_p, 2, sc + N3P, s));
    }
    // scalars of this iteration, read back with the first line-search result
    double phi_m = 0.0, f_m = 0.0, beta = 0.0;
    bool restarted = true, stop = false;
    auto take_scalars = [&]() -> ptyg_status {
      phi_m = h[PHI];
      f_m = phi_m + h[DCONST];
      beta = h[BETA];
      restarted = h[RST] != 0.0;
      if (!std::isfinite(phi_m)) return fail(PTYG_E_NONFINITE, "objective is %g at iteration %d", phi_m, m);
      if (opts->target_phi >= 0.0 && phi_m <= opts->target_phi) stop = true;
      return PTYG_OK;
    };

    // LS stage (Eq. linesearch, Algorithm 1 order: shrink, then evaluate)
    double gamma = opts->gamma0;
    bool accepted = false;
    int trials = 0;
    double eta2 = 0.0, n3 = 0.0;
    if (batched) {
      // far fields of the direction: Phi(psi + g eta [, p + g eta_p]) is the
      // deviance of A + g B (+ g^2 C), A = G psi stored by the GRAD pass
      PatArgs fa = base_args(dims);
      fa.pos = pos;
      fa.ubuf = at<float2>(ws, L.ubuf);  // staging of the 256^2 transforms
      fa.far = far_b;
      fa.cseg = cseg;
      double* zparts = at<double>(ws, L.zparts) + L.n_partials;
      double* zsums = at<double>(ws, L.zsums);
      {
        TimedLaunch tl_fwd(2, s);
        if (!joint) {
          fa.obj = eta_o;
          fa.probe = probe;
          PTYG_HIP(launch_fwd_t(fa, false, s));
        } else {
          fa.obj = obj;
          fa.dobj = eta_o;
          fa.probe = probe;
          fa.dprobe = eta_p;
          // 256^2: the first-order transform also forms the patch sums
          if (dims->n == 256) fa.ps_part = zparts;
          PTYG_HIP(launch_fwd_t(fa, true, s));
          PatArgs fc = fa;
          fc.ps_part = nullptr;
          fc.far = far_c;
          fc.obj = eta_o;
          fc.probe = eta_p;
          fc.dobj = nullptr;
          fc.dprobe = nullptr;
          PTYG_HIP(launch_fwd_t(fc, false, s));
        }
      }
      if (joint) {
        // the polynomial's coefficients over the patches (Parseval): rows
        // (Re a b*, 0, |b|^2, 0) and (Re a c*, Re b c*, |c|^2, 0); at 256^2
        // the first-order transform above wrote them per block
        int psb = 4 * dims->k;
        if (dims->n != 256) {
          psb = patch_sums_blocks(dims->k, dims->n);
          PTYG_HIP(launch_patch_sums(obj, eta_o, probe, eta_p, pos, dims->k, dims->obj_w, dims->n, zparts,
                                     zparts + 4 * (size_t)psb, s));
        }
        PTYG_HIP(launch_finalize2(FinJob{zparts, psb, 4, zsums + 4},
                                  FinJob{zparts + 4 * (size_t)psb, psb, 4, zsums + 8}, 2, s));
      }
      LsArgs la{};
      la.A = far_a;
      la.B = far_b;
      la.C = far_c;
      la.d = dt;
      la.idx = at<int>(ws, L.nz_idx);
      if (cseg) {
        la.compact = 1;
        la.d = dcomp;
      }
      la.n = nnz;
      la.eps = eps;
      la.est = est;
      // whole-array sums: [0] |a|^2 (GRAD), [4..7] direction pass, [8..11] joint pass
      la.partials = lsparts;
      int j0 = 1;
      bool first = true;
      double g_run = opts->gamma0;
      while (j0 <= opts->max_halvings && !accepted) {
        // the first pass covers up to two trials past the previous accepted index
        int J = std::min(kLsBatch, opts->max_halvings - j0 + 1);
        if (first) J = std::min(J, std::max(4, last_trials + 2));
        LsAccept acc{};
        for (int i = 0; i < J; ++i) {
          g_run *= opts->tau;  // the same sequence of doubles as the sequential search
          acc.gam[i] = g_run;
          la.g[i] = (float)g_run;
        }
        la.J = J;
        int nb = 0;
        {
          TimedLaunch tl(1, s);
          PTYG_HIP(launch_ls_batch(la, &nb, s));
        }
        PTYG_HIP(launch_ls_finalize(lsparts, nb, lsphi, s));
        // the decision is taken on the device (one source of truth for the
        // update below and for the step applied ahead of the host)
        acc.J = J;
        acc.t = opts->t;
        acc.target = opts->target_phi;
        acc.joint = joint ? 1 : 0;
        acc.stop_check = first ? 1 : 0;
        PTYG_HIP(launch_ls_accept(sc, sc + kZsSlot, lsphi, sc + kAccSlot, acc, s));
        if (first) {
          // one copy of the scalar region, then, ahead of the host, the update
          // with the device's step (0 when this pass accepted nothing or the
          // target is reached): the host waits for the copy only, so the
          // update runs during the round trip
          PTYG_HIP(hipMemcpyAsync(h, sc, (kAccSlot + 3) * sizeof(double), hipMemcpyDeviceToHost, s));
          PTYG_HIP(hipEventRecord(rb_ev, s));
          VecArgs u{};
          u.n = on;
          u.a = obj;
          u.c = eta_o;
          u.alpha_dev = sc + kAccSlot;
          PTYG_HIP(launch_axpy(u, s));
          if (joint) {
            VecArgs up{};
            up.n = pn;
            up.a = probe;
            up.c = eta_p;
            up.alpha_dev = sc + kAccSlot;
            PTYG_HIP(launch_axpy(up, s));
          }
          PTYG_HIP(hipEventSynchronize(rb_ev));
        } else {
          PTYG_HIP(hipMemcpyAsync(h + kLsSlot, lsphi, (kAccSlot + 3 - kLsSlot) * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
          PTYG_HIP(hipStreamSynchronize(s));
        }
        if (first) {
          if (ptyg_status st = take_scalars()) return st;
          if (stop) break;
          n3 = h[N3O] + (joint ? h[N3P] : 0.0);
          eta2 = h[EEO] + (joint ? h[EEP] : 0.0);
        }
        const int acc_trial = (int)h[kAccSlot + 1];
        if (acc_trial > 0) {
          accepted = true;
          trials = j0 + acc_trial - 1;
          gamma = h[kAccSlot];
          applied = first;  // the update already ran with the device's step
        } else {
          trials = j0 + J - 1;
        }
        j0 += J;
        first = false;
      }
      if (accepted) last_trials = trials;
    }
    for (int j = 1; !batched && j <= opts->max_halvings; ++j) {
      gamma *= opts->tau;
      trials = j;
      if (ptyg_status st = run_minfunc(dims, obj, eta_o, probe, eta_p, gamma, pos, dgrad, lgrad, eps, est,
                                       sc + PHIT, ws, L, s, false))
        return st;
      PTYG_HIP(hipMemcpyAsync(h, sc, (DCONST + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
      PTYG_HIP(hipStreamSynchronize(s));
      if (j == 1) {
        if (ptyg_status st = take_scalars()) return st;
        if (stop) break;
      }
      n3 = h[N3O] + (joint ? h[N3P] : 0.0);
      eta2 = h[EEO] + (joint ? h[EEP] : 0.0);
      const double phi_t = h[PHIT];
      if (phi_t <= phi_m + gamma * opts->t) {
        accepted = true;
        break;
      }
    }
    if (stop) break;  // target objective reached at psi_m: no update
    if (!accepted) gamma = 0.0;

    // Update stage (Eq. update); already applied when the first batched pass accepted
    if (gamma != 0.0 && !applied) {
      VecArgs u{};
      u.n = on;
      u.a = obj;
      u.c = eta_o;
      u.alpha = gamma;
      PTYG_HIP(launch_axpy(u, s));
      if (joint) {
        VecArgs up{};
        up.n = pn;
        up.a = probe;
        up.c = eta_p;
        up.alpha = gamma;
        PTYG_HIP(launch_axpy(up, s));
      }
    }
    if (trace) {
      ptyg_cg_iter_stats& t = trace[m];
      t.phi = phi_m;
      t.f_eq2 = f_m;
      t.gamma = gamma;
      t.beta = beta;
      t.step_norm = gamma * std::sqrt(eta2 > 0.0 ? eta2 : 0.0);
      t.halvings = trials;
      t.restarted = restarted ? 1 : 0;
    }
    restart = !accepted;
    if (iters_done) *iters_done = m + 1;
  }
  PTYG_HIP(hipStreamSynchronize(s));
  return PTYG_OK;
}

ptyg_status ptyg_gd_solve(const ptyg_dims* dims, ptyg_c64* obj_c, ptyg_c64* probe_c, const int32_t* pos_i,
                          const float* data, int32_t iters, double gamma, int32_t update_probe, float eps,
                          int32_t estimator, void* ws, size_t ws_bytes, double* phi_trace,
                          ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (ptyg_status st = check_est(estimator)) return st;
  if (!obj_c || !probe_c || !pos_i || !data) return fail(PTYG_E_INVAL, "NULL argument");
  if (iters < 0) return fail(PTYG_E_INVAL, "iters < 0");
  if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(PTYG_E_INVAL, "gamma must be finite and >= 0");
  if (!(eps >= 0.0f)) return fail(PTYG_E_INVAL, "eps must be >= 0");
  const bool joint = update_probe != 0;
  Layout L;
  if (ptyg_status st = check_ws(dims, ws, ws_bytes, joint, &L)) return st;
  if (ptyg_status st = ptyg_check_positions(dims, pos_i, ws, ws_bytes, stream)) return st;
  const hipStream_t s = S(stream);
  float2* obj = reinterpret_cast<float2*>(obj_c);
  float2* probe = reinterpret_cast<float2*>(probe_c);
  const int2* pos = reinterpret_cast<const int2*>(pos_i);
  float2* grad_o = at<float2>(ws, L.grad_obj);
  float2* grad_p = joint ? at<float2>(ws, L.grad_probe) : nullptr;
  float* dt = at<float>(ws, L.data_t);
  double* tr = at<double>(ws, L.gdtrace);
  // n <= 128 reads the intensities as given, 256^2 per pattern transposed
  const bool big = dims->n == 256;
  if (big) PTYG_HIP(launch_transpose_data(data, dt, dims->k, dims->n, s));
  const float* dgrad = big ? dt : data;
  const DataLayout lgrad = big ? DataLayout::Transposed : DataLayout::Rows;
  if (ptyg_status st = build_tiles(dims, pos, ws, L, s)) return st;
  std::vector<double> h(kGdTrace);
  for (int m0 = 0; m0 < iters; m0 += kGdTrace) {
    const int cnt = std::min(kGdTrace, iters - m0);
    for (int i = 0; i < cnt; ++i) {
      // GRAD stage; the objective of obj_m lands in the device trace
      if (ptyg_status st = run_grad(dims, obj, probe, pos, dgrad, lgrad, eps, estimator, grad_o, grad_p, tr + i, ws,
                                    L, s, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, false))
        return st;
      VecArgs u{};
      u.n = (int64_t)dims->obj_h * dims->obj_w;
      u.a = obj;
      u.c = grad_o;
      u.alpha = -gamma;
      PTYG_HIP(launch_axpy(u, s));
      if (joint) {
        VecArgs up{};
        up.n = (int64_t)dims->n * dims->n;
        up.a = probe;
        up.c = grad_p;
        up.alpha = -gamma;
        PTYG_HIP(launch_axpy(up, s));
      }
    }
    PTYG_HIP(hipMemcpyAsync(h.data(), tr, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
    PTYG_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < cnt; ++i) {
      if (phi_trace) phi_trace[m0 + i] = h[i];
      if (!std::isfinite(h[i])) return fail(PTYG_E_NONFINITE, "objective is %g at iteration %d", h[i], m0 + i);
    }
  }
  return PTYG_OK;
}

namespace {
// Multi-view batch: the views are stacked along the rows into one object of
// views * obj_h rows; their patterns follow each other.  Each view's patterns
// are padded to kp, a multiple of the patterns per workgroup and of the
// compaction chunk (kp = k when k already is one).  With padding, the stacked
// object gets n zero rows below the last view and the padding patterns sit
// there with zero intensities: their exit waves, objective terms and
// gradients are exactly 0, and no view's vector operations reach those rows,
// so they stay 0.  The object and the intensities are then copied into the
// workspace in the padded layout (the object back at the end).
struct ViewsLayout {
  ptyg_dims stacked;
  Layout L;  // of the stacked problem
  int kp;    // patterns per view after padding
  size_t pos2, vparts, vout, vbeta, valpha, objp, datap, total;
};

ptyg_status views_layout(const ptyg_dims* d, int32_t views, const ptyg_cg_opts* opts, ViewsLayout* out) {
  if (ptyg_status st = check_dims(d)) return st;
  if (views < 1) return fail(PTYG_E_INVAL, "views=%d must be >= 1", views);
  if (d->n > 128) return fail(PTYG_E_INVAL, "the multi-view batch supports n <= 128 (n=%d)", d->n);
  const int nn = d->n * d->n;
  const int unit = std::lcm(patterns_per_block(d->n), nn >= kNzChunk ? 1 : kNzChunk / nn);
  const int64_t kp = ((int64_t)d->k + unit - 1) / unit * unit;
  const bool pad = kp != d->k;
  const int64_t rows = (int64_t)d->obj_h * views + (pad ? d->n : 0);
  if (rows * d->obj_w >= (int64_t(1) << 31) || (int64_t)views * kp * nn >= (int64_t(1) << 31))
    return fail(PTYG_E_INVAL, "%d views of this size are too large", views);
  if (opts && opts->update_probe) return fail(PTYG_E_INVAL, "the multi-view batch is object-only");
  ViewsLayout V{};
  V.kp = (int)kp;
  V.stacked = *d;
  V.stacked.obj_h = (int)rows;
  V.stacked.k = (int)kp * views;
  V.L = layout(&V.stacked, false, opts && opts->line_search == PTYG_LS_BATCHED, true);
  size_t o = V.L.total;
  V.pos2 = o;
  o = align_up(o + (size_t)V.stacked.k * sizeof(int2));
  V.objp = V.datap = 0;
  if (pad) {
    V.objp = o;
    o = align_up(o + (size_t)rows * d->obj_w * sizeof(float2));
    V.datap = o;
    o = align_up(o + (size_t)V.stacked.k * nn * sizeof(float));
  }
  V.vparts = o;
  o = align_up(o + (size_t)views * kSegBlocks * kLsRow * sizeof(double));
  V.vout = o;
  o = align_up(o + (size_t)views * 32 * sizeof(double));
  V.vbeta = o;
  o = align_up(o + (size_t)views * sizeof(double));
  V.valpha = o;
  o = align_up(o + (size_t)views * sizeof(double));
  V.total = o;
  *out = V;
  return PTYG_OK;
}
}  // namespace

size_t ptyg_views_workspace_size(const ptyg_dims* dims, int32_t views, const ptyg_cg_opts* opts) {
  ViewsLayout V;
  if (views_layout(dims, views, opts, &V) != PTYG_OK) return 0;
  return V.total;
}

ptyg_status ptyg_cg_solve_views(const ptyg_dims* dims, int32_t views, ptyg_c64* obj_c, const ptyg_c64* probe_c,
                                const int32_t* pos_i, const float* data, const ptyg_cg_opts* opts, void* ws,
                                size_t ws_bytes, ptyg_cg_iter_stats* trace, int32_t* iters_done,
                                ptyg_stream_t stream) {
  if (!obj_c || !probe_c || !pos_i || !data || !opts) return fail(PTYG_E_INVAL, "NULL argument");
  ViewsLayout VL;
  if (ptyg_status st = views_layout(dims, views, opts, &VL)) return st;
  if (opts->iters < 0) return fail(PTYG_E_INVAL, "iters < 0");
  if (!(opts->tau > 0.0 && opts->tau < 1.0)) return fail(PTYG_E_INVAL, "tau must be in (0, 1)");
  if (!(opts->gamma0 > 0.0) || !std::isfinite(opts->gamma0)) return fail(PTYG_E_INVAL, "gamma0 must be > 0");
  if (opts->max_halvings < 1) return fail(PTYG_E_INVAL, "max_halvings must be >= 1");
  if (!(opts->eps >= 0.0)) return fail(PTYG_E_INVAL, "eps must be >= 0");
  if (opts->target_phi >= 0.0) return fail(PTYG_E_INVAL, "target_phi is not supported by the multi-view batch");
  if (opts->line_search != PTYG_LS_SEQUENTIAL && opts->line_search != PTYG_LS_BATCHED)
    return fail(PTYG_E_INVAL, "line_search=%d is not a PTYG_LS_* value", opts->line_search);
  if (ptyg_status st = check_est(opts->estimator)) return st;
  if (!ws || ((uintptr_t)ws) % kAlign) return fail(PTYG_E_INVAL, "workspace NULL or not 256-byte aligned");
  if (ws_bytes < VL.total) return fail(PTYG_E_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, VL.total);
  if (iters_done) *iters_done = 0;
  const int V = views;
  const bool batched = opts->line_search == PTYG_LS_BATCHED;
  const int est = opts->estimator;
  const float eps = (float)opts->eps;
  const ptyg_dims* D = &VL.stacked;
  const Layout& L = VL.L;
  const hipStream_t s = S(stream);
  // every position inside its own view's object
  {
    ptyg_dims d1 = *dims;
    d1.k = dims->k * V;
    if (ptyg_status st = ptyg_check_positions(&d1, pos_i, ws, ws_bytes, stream)) return st;
  }
  const int kp = VL.kp;  // patterns per view in the stacked problem
  const bool pad = VL.objp != 0;
  const int64_t on = (int64_t)dims->obj_h * dims->obj_w;  // per view
  const int64_t pe = (int64_t)kp * dims->n * dims->n;    // pattern elements per view
  // padded: the stacked object (views, then n zero rows) and the intensities
  // (each view's k patterns, then zeros up to kp) in the workspace
  float2* obj = pad ? at<float2>(ws, VL.objp) : reinterpret_cast<float2*>(obj_c);
  const float* dat = pad ? at<float>(ws, VL.datap) : data;
  // every return from here on leaves the iterates in obj_c with no copy in flight
  struct ViewsOut {
    hipStream_t s;
    ptyg_c64* dst;
    const float2* src;
    size_t bytes;
    ~ViewsOut() {
      if (src) (void)hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
      (void)hipStreamSynchronize(s);
    }
  } out{s, obj_c, nullptr, 0};
  if (pad) {
    const size_t pb = (size_t)dims->k * dims->n * dims->n * sizeof(float);
    PTYG_HIP(hipMemcpyAsync(obj, obj_c, (size_t)V * on * sizeof(float2), hipMemcpyDeviceToDevice, s));
    out.src = obj;
    out.bytes = (size_t)V * on * sizeof(float2);
    PTYG_HIP(launch_zero(obj + V * on, (int64_t)dims->n * dims->obj_w, s));
    PTYG_HIP(launch_fill_i32(reinterpret_cast<int*>(at<float>(ws, VL.datap)), (int64_t)V * pe, 0, s));
    PTYG_HIP(hipMemcpy2DAsync(at<float>(ws, VL.datap), (size_t)pe * sizeof(float), data, pb, pb, V,
                              hipMemcpyDeviceToDevice, s));
  }
  const float2* probe = reinterpret_cast<const float2*>(probe_c);
  int2* pos = at<int2>(ws, VL.pos2);
  PTYG_HIP(launch_shift_views(reinterpret_cast<const int2*>(pos_i), dims->k, kp, V, dims->obj_h, V * dims->obj_h,
                              pos, s));
  float2* eta_o = at<float2>(ws, L.eta_obj);
  float2* grad_o = at<float2>(ws, L.grad_obj);
  float* dt = at<float>(ws, L.data_t);
  double* partials = at<double>(ws, L.partials);
  double* vparts = at<double>(ws, VL.vparts);
  double* vout = at<double>(ws, VL.vout);  // [V][32]: per-view results
  double* dbeta = at<double>(ws, VL.vbeta);
  double* dalpha = at<double>(ws, VL.valpha);
  float2* far_a = batched ? at<float2>(ws, L.far_a) : nullptr;
  float2* far_b = batched ? at<float2>(ws, L.far_b) : nullptr;
  // the transform kernels read the intensities as given; the compaction of
  // the batched search reads a per-pattern transposed copy
  if (batched) PTYG_HIP(launch_transpose_data(dat, dt, D->k, D->n, s));
  PTYG_HIP(launch_zero(eta_o, (int64_t)D->obj_h * D->obj_w, s));
  if (ptyg_status st = build_tiles(D, pos, ws, L, s)) return st;
  const int cpv = (int)(pe / kNzChunk);  // compaction chunks per view
  if (batched)
    PTYG_HIP(launch_nz_compact(dt, pe * V, at<int>(ws, L.nz_counts), at<int>(ws, L.nz_offsets), at<int>(ws, L.nz_idx),
                               nullptr, nullptr, s));

  // per-view data constants: Eq. ML's F = Phi + sum over d > 0 of d - d log d
  std::vector<double> dconst(V, 0.0);
  PTYG_HIP(launch_data_const(dat, pe, V, at<double>(ws, VL.vparts), at<double>(ws, VL.vout), s));
  PTYG_HIP(hipMemcpyAsync(dconst.data(), at<double>(ws, VL.vout), V * sizeof(double), hipMemcpyDeviceToHost, s));
  PTYG_HIP(hipStreamSynchronize(s));
  // per-view state
  std::vector<double> h((size_t)V * 32), hbeta(V, 0.0), halpha(V, 0.0), phi_m(V), f_m(V), n3_prev(V, 0.0);
  std::vector<double> lsrow((size_t)V * kLsRow), zc((size_t)V * 3);
  std::vector<int> restart(V, 1), accepted(V), trials(V), last_trials(V, kLsBatch), restarted(V);
  std::vector<double> gamma_v(V), beta_v(V), n3(V), eta2(V);
  // vout slots: 0 phi, 1 f, 2 n1, 3 n2, 4 n3, 5 eta2, 6 |a|^2, 8..11 direction sums
  for (int m = 0; m < opts->iters; ++m) {
    // GRAD over every view in one launch; objectives and sums per view
    if (ptyg_status st = run_grad(D, obj, probe, pos, dat, DataLayout::Rows, eps, est, grad_o, nullptr,
                                  nullptr, ws, L, s, far_a, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                  false))
      return st;
    PTYG_HIP(launch_finalize_views(partials, D->n, D->k, kp, V, 2, vparts, s));
    PTYG_HIP(launch_dot2_views(grad_o, eta_o, on, V, vparts + 2 * V, s));
    PTYG_HIP(launch_finalize_seg(vparts + 2 * V, kSegBlocks, 2, V, vparts + (size_t)V * kSegBlocks * 2 + 2 * V,
                                 s));
    if (batched) PTYG_HIP(launch_finalize_views(at<double>(ws, L.zparts), D->n, D->k, kp, V, 1, dalpha, s));
    // gather [V][2] (phi, f), [V][2] (n1, n2), [V] |a|^2 to the host
    std::vector<double> pf(2 * V), nn(2 * V), aa(V, 0.0);
    PTYG_HIP(hipMemcpyAsync(pf.data(), vparts, 2 * V * sizeof(double), hipMemcpyDeviceToHost, s));
    PTYG_HIP(hipMemcpyAsync(nn.data(), vparts + (size_t)V * kSegBlocks * 2 + 2 * V, 2 * V * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    if (batched) PTYG_HIP(hipMemcpyAsync(aa.data(), dalpha, V * sizeof(double), hipMemcpyDeviceToHost, s));
    PTYG_HIP(hipStreamSynchronize(s));
    for (int v = 0; v < V; ++v) {
      phi_m[v] = pf[2 * v];
      f_m[v] = phi_m[v] + dconst[v];
      if (!std::isfinite(phi_m[v]))
        return fail(PTYG_E_NONFINITE, "objective is %g at iteration %d of view %d", phi_m[v], m, v);
      double beta = 0.0;
      restarted[v] = restart[v];
      if (!restart[v]) {
        const double den = nn[2 * v + 1] - n3_prev[v];
        if (std::isfinite(den) && den > 0.0 && std::isfinite(nn[2 * v])) beta = nn[2 * v] / den;
        else restarted[v] = 1;
      }
      beta_v[v] = restarted[v] ? 0.0 : beta;
      hbeta[v] = beta_v[v];
    }
    // DIR: eta_v = -grad_v + beta_v eta_v (beta 0 restarts; eta stays finite)
    PTYG_HIP(hipMemcpyAsync(dbeta, hbeta.data(), V * sizeof(double), hipMemcpyHostToDevice, s));
    PTYG_HIP(launch_dir_views(grad_o, eta_o, dbeta, on, V, vparts, s));
    PTYG_HIP(launch_finalize_seg(vparts, kSegBlocks, 2, V, vout, s));
    std::vector<double> de(2 * V);
    PTYG_HIP(hipMemcpyAsync(de.data(), vout, 2 * V * sizeof(double), hipMemcpyDeviceToHost, s));

    // LS: the same trial sequence for every view, per-view decisions
    for (int v = 0; v < V; ++v) {
      accepted[v] = 0;
      trials[v] = 0;
      gamma_v[v] = 0.0;
    }
    int pending = V;
    if (batched) {
      PatArgs fa = base_args(D);
      fa.pos = pos;
      fa.ubuf = at<float2>(ws, L.ubuf);
      fa.far = far_b;
      fa.obj = eta_o;
      fa.probe = probe;
      fa.zs_p = far_a;
      fa.zs_part = at<double>(ws, L.zparts) + L.n_partials;
      {
        TimedLaunch tl_fwd(2, s);
        PTYG_HIP(launch_fwd_t(fa, false, s));
      }
      PTYG_HIP(launch_finalize_views(fa.zs_part, D->n, D->k, kp, V, 4, vout + 2 * V, s));
      std::vector<double> zs4(4 * V);
      PTYG_HIP(hipMemcpyAsync(zs4.data(), vout + 2 * V, 4 * V * sizeof(double), hipMemcpyDeviceToHost, s));
      LsArgs la{};
      la.A = far_a;
      la.B = far_b;
      la.d = dt;
      la.idx = at<int>(ws, L.nz_idx);
      la.eps = eps;
      la.est = est;
      la.partials = vparts;
      int j0 = 1;
      bool first = true;
      double g_run = opts->gamma0;
      while (j0 <= opts->max_halvings && pending > 0) {
        int J = std::min(kLsBatch, opts->max_halvings - j0 + 1);
        if (first) {
          int want = 4;
          for (int v = 0; v < V; ++v) want = std::max(want, last_trials[v] + 2);
          J = std::min(J, want);
        }
        double gam[kLsBatch];
        for (int i = 0; i < J; ++i) {
          g_run *= opts->tau;
          gam[i] = g_run;
          la.g[i] = (float)g_run;
        }
        la.J = J;
        {
          TimedLaunch tl(1, s);
          PTYG_HIP(launch_ls_batch_views(la, at<int>(ws, L.nz_offsets), cpv, V, s));
        }
        PTYG_HIP(launch_ls_finalize_views(vparts, V, vout + 8 * V, s));
        PTYG_HIP(hipMemcpyAsync(lsrow.data(), vout + 8 * V, (size_t)V * kLsRow * sizeof(double),
                                hipMemcpyDeviceToHost, s));
        PTYG_HIP(hipStreamSynchronize(s));
        for (int v = 0; v < V; ++v) {
          const double* row = lsrow.data() + (size_t)v * kLsRow;
          if (first) {
            n3[v] = de[2 * v];
            eta2[v] = de[2 * v + 1];
            zc[3 * v + 0] = aa[v] - row[kLsBatch + 0];
            zc[3 * v + 1] = zs4[4 * v + 0] - row[kLsBatch + 1];
            zc[3 * v + 2] = zs4[4 * v + 2] - row[kLsBatch + 2];
          }
          if (accepted[v]) continue;
          for (int i = 0; i < J; ++i) {
            trials[v] = j0 + i;
            const double g = (double)la.g[i];
            const double zero = zc[3 * v] + 2.0 * g * zc[3 * v + 1] + g * g * zc[3 * v + 2];
            if (row[i] + zero <= phi_m[v] + gam[i] * opts->t) {
              accepted[v] = 1;
              gamma_v[v] = gam[i];
              --pending;
              break;
            }
          }
        }
        j0 += J;
        first = false;
      }
      for (int v = 0; v < V; ++v)
        if (accepted[v]) last_trials[v] = trials[v];
    } else {
      PTYG_HIP(hipStreamSynchronize(s));
      for (int v = 0; v < V; ++v) {
        n3[v] = de[2 * v];
        eta2[v] = de[2 * v + 1];
      }
      double gamma = opts->gamma0;
      for (int j = 1; j <= opts->max_halvings && pending > 0; ++j) {
        gamma *= opts->tau;
        PatArgs a = base_args(D);
        a.obj = obj;
        a.dobj = eta_o;
        a.probe = probe;
        a.gamma = (float)gamma;
        a.pos = pos;
        a.data = dat;
        a.eps = eps;
        a.est = est;
        a.partials = partials;
        a.ubuf = at<float2>(ws, L.ubuf);
        {
          TimedLaunch tl(1, s);
          PTYG_HIP(launch_minfunc(a, DataLayout::Rows, nullptr, s));
        }
        PTYG_HIP(launch_finalize_views(partials, D->n, D->k, kp, V, 2, vout + 8 * V, s));
        std::vector<double> pt(2 * V);
        PTYG_HIP(hipMemcpyAsync(pt.data(), vout + 8 * V, 2 * V * sizeof(double), hipMemcpyDeviceToHost, s));
        PTYG_HIP(hipStreamSynchronize(s));
        for (int v = 0; v < V; ++v) {
          if (accepted[v]) continue;
          trials[v] = j;
          if (pt[2 * v] <= phi_m[v] + gamma * opts->t) {
            accepted[v] = 1;
            gamma_v[v] = gamma;
            --pending;
          }
        }
      }
    }
    // Update: psi_v += gamma_v eta_v (0 for a failed search)
    for (int v = 0; v < V; ++v) halpha[v] = accepted[v] ? gamma_v[v] : 0.0;
    PTYG_HIP(hipMemcpyAsync(dalpha, halpha.data(), V * sizeof(double), hipMemcpyHostToDevice, s));
    PTYG_HIP(launch_axpy_views(obj, eta_o, dalpha, on, V, s));
    for (int v = 0; v < V; ++v) {
      if (trace) {
        ptyg_cg_iter_stats& t = trace[(size_t)v * opts->iters + m];
        t.phi = phi_m[v];
        t.f_eq2 = f_m[v];
        t.gamma = halpha[v];
        t.beta = beta_v[v];
        t.step_norm = halpha[v] * std::sqrt(eta2[v] > 0.0 ? eta2[v] : 0.0);
        t.halvings = accepted[v] ? trials[v] : opts->max_halvings;
        t.restarted = restarted[v];
      }
      n3_prev[v] = n3[v];
      restart[v] = !accepted[v];
    }
    // the host vectors copied to the device above must outlive the copies
    PTYG_HIP(hipStreamSynchronize(s));
    if (iters_done) *iters_done = m + 1;
  }
  if (pad) {
    PTYG_HIP(hipMemcpyAsync(obj_c, obj, out.bytes, hipMemcpyDeviceToDevice, s));
    out.src = nullptr;
  }
  PTYG_HIP(hipStreamSynchronize(s));
  return PTYG_OK;
}

void ptyg_timing_enable(int32_t kinds_mask) { g_timing.mask = kinds_mask & 0x1F; }

void ptyg_timing_reset(void) {
  g_timing.drain();
  for (int i = 0; i < Timing::kKinds; ++i) {
    g_timing.ms[i] = 0.0;
    g_timing.count[i] = 0;
  }
}

ptyg_status ptyg_timing_read(double* ms, int32_t* count, int32_t kinds) {
  if (!ms || !count || kinds < 0 || kinds > Timing::kKinds) return fail(PTYG_E_INVAL, "bad timing arguments");
  g_timing.drain();
  for (int i = 0; i < kinds; ++i) {
    ms[i] = g_timing.ms[i];
    count[i] = g_timing.count[i];
  }
  return PTYG_OK;
}

ptyg_status ptyg_debug_gather(const ptyg_dims* dims, const ptyg_c64* obj, const int32_t* pos,
                              ptyg_c64* patches, ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (!obj || !pos || !patches) return fail(PTYG_E_INVAL, "NULL array argument");
  PatArgs a = base_args(dims);
  a.obj = reinterpret_cast<const float2*>(obj);
  a.pos = reinterpret_cast<const int2*>(pos);
  PTYG_HIP(launch_debug_gather(a, reinterpret_cast<float2*>(patches), S(stream)));
  return PTYG_OK;
}

ptyg_status ptyg_debug_scatter(const ptyg_dims* dims, const ptyg_c64* patches, const int32_t* pos,
                               ptyg_c64* obj_out, ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (!patches || !pos || !obj_out) return fail(PTYG_E_INVAL, "NULL array argument");
  PatArgs a = base_args(dims);
  a.pos = reinterpret_cast<const int2*>(pos);
  a.gobj = reinterpret_cast<float2*>(obj_out);
  PTYG_HIP(launch_zero(a.gobj, (int64_t)dims->obj_h * dims->obj_w, S(stream)));
  PTYG_HIP(launch_debug_scatter(a, reinterpret_cast<const float2*>(patches), S(stream)));
  return PTYG_OK;
}

ptyg_status ptyg_debug_grad_far(const ptyg_dims* dims, const ptyg_c64* far, const ptyg_c64* probe,
                                const int32_t* pos, const float* data, float eps, int32_t estimator,
                                ptyg_c64* grad_obj, const ptyg_c64* obj, ptyg_c64* grad_probe, double* objective,
                                ptyg_c64* residual, void* ws, size_t ws_bytes, ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (!far || !probe || !pos || !data || !grad_obj) return fail(PTYG_E_INVAL, "NULL array argument");
  if (grad_probe && !obj) return fail(PTYG_E_INVAL, "grad_probe requires obj");
  if (!(eps >= 0.0f)) return fail(PTYG_E_INVAL, "eps must be >= 0");
  if (ptyg_status st = check_est(estimator)) return st;
  Layout L;
  if (ptyg_status st = check_ws(dims, ws, ws_bytes, false, &L)) return st;
  if (ptyg_status st = build_tiles(dims, reinterpret_cast<const int2*>(pos), ws, L, S(stream))) return st;
  return run_grad(dims, reinterpret_cast<const float2*>(obj), reinterpret_cast<const float2*>(probe),
                  reinterpret_cast<const int2*>(pos), data, DataLayout::Rows, eps, estimator,
                  reinterpret_cast<float2*>(grad_obj), reinterpret_cast<float2*>(grad_probe), objective, ws, L,
                  S(stream), nullptr, nullptr, nullptr, nullptr, nullptr, reinterpret_cast<const float2*>(far),
                  reinterpret_cast<float2*>(residual));
}

ptyg_status ptyg_debug_tile_sum(const ptyg_dims* dims, const ptyg_c64* waves, const ptyg_c64* probe,
                                const int32_t* pos, ptyg_c64* obj_out, void* ws, size_t ws_bytes,
                                ptyg_stream_t stream) {
  if (ptyg_status st = check_dims(dims)) return st;
  if (!waves || !pos || !obj_out) return fail(PTYG_E_INVAL, "NULL array argument");
  if (dims->n == 256 && !probe) return fail(PTYG_E_INVAL, "n = 256 needs the probe (the product path multiplies it in)");
  Layout L;
  if (ptyg_status st = check_ws(dims, ws, ws_bytes, false, &L)) return st;
  const int2* p = reinterpret_cast<const int2*>(pos);
  if (ptyg_status st = build_tiles(dims, p, ws, L, S(stream))) return st;
  PTYG_HIP(launch_tile_sum(reinterpret_cast<const float2*>(waves), reinterpret_cast<const float2*>(probe), p,
                           at<int>(ws, L.toff), at<int>(ws, L.tlist), dims->k, dims->obj_h, dims->obj_w, dims->n,
                           reinterpret_cast<float2*>(obj_out), S(stream)));
  return PTYG_OK;
}

ptyg_status ptyg_debug_lane_swap(float* a, float* b, ptyg_stream_t stream) {
  if (!a || !b) return fail(PTYG_E_INVAL, "NULL array argument");
  PTYG_HIP(launch_debug_lane_swap(a, b, S(stream)));
  return PTYG_OK;
}

}  // extern "C"
