// Host side of the C ABI declared in include/oica.h: context, workspace,
// argument checks (all before any device work) and launch orchestration.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "oica_internal.h"

using namespace oica;

// Fixed device array behind oica_kurtosis_noalloc (per-split partial sums of
// z^4), for callers that cannot allocate.  Every device the library runs on
// holds its own copy from module load until the process ends.  Host code
// never passes the array's name to a kernel: it uses the device address taken
// once per device below.
constexpr size_t NOALLOC_DOUBLES = (size_t)OICA_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on `device`, which must be current; taken on the
// first call for that device.
hipError_t scratch_address(int device, void **out) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
}  // namespace

constexpr int KURT_STREAMS = 4;  // a batched call's concurrent kurtosis passes

struct oica_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  int *small_dev = nullptr;    // 64 ints of device bookkeeping
  int *small_host = nullptr;   // 64 ints of pinned host memory
  std::vector<hipEvent_t> events;  // start/stop pairs for kernel timing
  std::map<std::string, std::vector<int>> tune;  // batched tile choices: {wk32, wk64, grid}
  void *scratch = nullptr;     // device address of the fixed noalloc array on `device`
  void *ws2 = nullptr;         // deflation driver's buffers (the calls it makes use ws)
  size_t ws2_bytes = 0;
  // streams (default priority) on which a batched call runs its datasets'
  // kurtosis passes side by side, with the events that order them against
  // `stream`; created by the first batched call
  hipStream_t aux[KURT_STREAMS] = {};
  hipEvent_t aux_ev[KURT_STREAMS + 1] = {};
  std::string err;
};

namespace {

int fail(oica_ctx *ctx, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(oica_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

#define HIP_TRY(ctx, expr)                                                            \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, OICA_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Calls on a context without a device stop where device work would begin.
int device_ready(oica_ctx *ctx) {
  return ctx->device < 0 ? fail(ctx, OICA_E_DEVICE, "context has no device (argument checks only)")
                         : OICA_OK;
}

int ensure_buf(oica_ctx *ctx, void **buf, size_t *have, size_t bytes) {
  if (int rc = device_ready(ctx)) return rc;
  if (bytes <= *have) return OICA_OK;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (*buf) {
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipFree(*buf));
    *buf = nullptr;
    *have = 0;
  }
  size_t want = bytes + bytes / 4 + (1u << 20);
  if (hipMalloc(buf, want) != hipSuccess) {
    (void)hipGetLastError();
    *buf = nullptr;
    return fail(ctx, OICA_E_NOMEM, "workspace allocation of %zu bytes failed", want);
  }
  *have = want;
  return OICA_OK;
}
int ensure_ws(oica_ctx *ctx, size_t bytes) { return ensure_buf(ctx, &ctx->ws, &ctx->ws_bytes, bytes); }

// The auxiliary streams and their events, created once per context.
int ensure_aux(oica_ctx *ctx) {
  for (int i = 0; i < KURT_STREAMS; ++i)
    if (!ctx->aux[i]) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->aux[i], hipStreamNonBlocking));
  for (int i = 0; i <= KURT_STREAMS; ++i)
    if (!ctx->aux_ev[i]) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->aux_ev[i], hipEventDisableTiming));
  return OICA_OK;
}

// Work enqueued on the auxiliary streams between aux_fork and aux_join runs
// after everything enqueued on the call's stream before the fork, and
// everything enqueued on the call's stream after the join waits for it.
int aux_fork(oica_ctx *ctx) {
  if (int rc = ensure_aux(ctx)) return rc;
  HIP_TRY(ctx, hipEventRecord(ctx->aux_ev[KURT_STREAMS], ctx->stream));
  for (int i = 0; i < KURT_STREAMS; ++i)
    HIP_TRY(ctx, hipStreamWaitEvent(ctx->aux[i], ctx->aux_ev[KURT_STREAMS], 0));
  return OICA_OK;
}
int aux_join(oica_ctx *ctx) {
  for (int i = 0; i < KURT_STREAMS; ++i) {
    HIP_TRY(ctx, hipEventRecord(ctx->aux_ev[i], ctx->aux[i]));
    HIP_TRY(ctx, hipStreamWaitEvent(ctx->stream, ctx->aux_ev[i], 0));
  }
  return OICA_OK;
}

struct Carve {
  char *p;
  template <typename T>
  T *take(size_t count) {
    T *r = (T *)p;
    p += (count * sizeof(T) + 255) & ~(size_t)255;
    return r;
  }
};

int check_dims(oica_ctx *ctx, int N, int64_t T) {
  if (N < 1) return fail(ctx, OICA_E_ARG, "N must be >= 1 (got %d)", N);
  if (N > OICA_MAX_N) return fail(ctx, OICA_E_UNSUPPORTED, "N=%d exceeds OICA_MAX_N=%d", N, OICA_MAX_N);
  if (T <= N) return fail(ctx, OICA_E_ARG, "T must exceed N (N=%d, T=%lld)", N, (long long)T);
  if (T > (int64_t)1 << 40) return fail(ctx, OICA_E_UNSUPPORTED, "T=%lld too large", (long long)T);
  return OICA_OK;
}

}  // namespace

extern "C" {

int oica_version(void) { return 10000; }

const char *oica_status_string(int status) {
  switch (status) {
    case OICA_OK: return "OICA_OK";
    case OICA_E_ARG: return "OICA_E_ARG";
    case OICA_E_SHAPE: return "OICA_E_SHAPE";
    case OICA_E_RANK: return "OICA_E_RANK";
    case OICA_E_NONFINITE: return "OICA_E_NONFINITE";
    case OICA_E_DEVICE: return "OICA_E_DEVICE";
    case OICA_E_NOMEM: return "OICA_E_NOMEM";
    case OICA_E_UNSUPPORTED: return "OICA_E_UNSUPPORTED";
    case OICA_E_NOCONV: return "OICA_E_NOCONV";
    default: return "OICA_E_UNKNOWN";
  }
}

const char *oica_last_error(const oica_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

int oica_create(oica_ctx **out, int device, void *hip_stream) {
  if (!out) return OICA_E_ARG;
  *out = nullptr;
  if (device == OICA_NO_DEVICE) {  // argument checks only: no HIP call at all
    oica_ctx *ctx = new oica_ctx();
    ctx->device = OICA_NO_DEVICE;
    *out = ctx;
    return OICA_OK;
  }
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return OICA_E_DEVICE;
  }
  if (device < 0 || device >= n) return OICA_E_ARG;
  oica_ctx *ctx = new oica_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess || scratch_address(device, &ctx->scratch) != hipSuccess ||
      hipMalloc(&ctx->small_dev, 64 * sizeof(int)) != hipSuccess ||
      hipHostMalloc(&ctx->small_host, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    if (ctx->small_dev) (void)hipFree(ctx->small_dev);
    delete ctx;
    return OICA_E_DEVICE;
  }
  *out = ctx;
  return OICA_OK;
}

void oica_destroy(oica_ctx *ctx) {
  if (!ctx) return;
  if (ctx->device < 0) {
    delete ctx;
    return;
  }
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->ws2) (void)hipFree(ctx->ws2);
  if (ctx->small_dev) (void)hipFree(ctx->small_dev);
  if (ctx->small_host) (void)hipHostFree(ctx->small_host);
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  for (hipStream_t a : ctx->aux)
    if (a) (void)hipStreamDestroy(a);
  for (hipEvent_t e : ctx->aux_ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

int oica_set_stream(oica_ctx *ctx, void *hip_stream) {
  if (!ctx) return OICA_E_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  return OICA_OK;
}

// ---------------------------------------------------------------------------
int oica_whiten(oica_ctx *ctx, int N, int64_t T, const void *X_raw, oica_dtype raw_t,
                int64_t ld_raw, void *Xw, oica_dtype out_t, float *Xw_f32, double *V,
                double *mean, double *eigval) {
  if (!ctx) return OICA_E_ARG;
  ctx->err.clear();
  int rc = check_dims(ctx, N, T);
  if (rc) return rc;
  if (!X_raw || !Xw) return fail(ctx, OICA_E_ARG, "X_raw and Xw must be non-null");
  if (raw_t != OICA_F64 && raw_t != OICA_F32)
    return fail(ctx, OICA_E_UNSUPPORTED, "raw_t must be OICA_F64 or OICA_F32");
  if (ld_raw < T)
    return fail(ctx, OICA_E_SHAPE, "ld_raw (%lld) must be >= T (%lld)", (long long)ld_raw,
                (long long)T);
  if (out_t != OICA_F32 && out_t != OICA_BF16)
    return fail(ctx, OICA_E_UNSUPPORTED, "out_t must be OICA_F32 or OICA_BF16");
  rc = ensure_ws(ctx, whiten_workspace_bytes(N, T));
  if (rc) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipMemsetAsync(ctx->small_dev, 0, 64 * sizeof(int), ctx->stream));
  HIP_TRY(ctx, launch_whiten(ctx->stream, N, T, X_raw, raw_t, ld_raw, Xw, out_t, Xw_f32, V, mean, eigval,
                             ctx->ws, ctx->ws_bytes, ctx->small_dev));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->small_host, ctx->small_dev, sizeof(int), hipMemcpyDeviceToHost,
                              ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  const int flags = ctx->small_host[0];
  if (flags & 1) return fail(ctx, OICA_E_NONFINITE, "X_raw contains NaN or Inf");
  if (flags & 4) return fail(ctx, OICA_E_NOCONV, "the Jacobi solve of the covariance did not converge");
  if (flags & 2) return fail(ctx, OICA_E_RANK, "covariance is rank deficient (eigenvalue ratio <= 1e-12)");
  return OICA_OK;
}

int oica_set_option(int option, int value) {
  switch (option) {
    case OICA_OPT_COOP_GIVE_UP:
      if (value != 0 && value != 1) return OICA_E_ARG;
      set_coop_give_up(value == 1);
      return OICA_OK;
    case OICA_OPT_JACOBI_MAX_SWEEPS:
      if (value < 0 || value > 30) return OICA_E_ARG;
      set_jacobi_max_sweeps(value == 0 ? 30 : value);
      return OICA_OK;
    case OICA_OPT_COOP_LAUNCH_API:
      if (value != 0 && value != 1) return OICA_E_ARG;
      set_coop_launch_api(value == 1);
      return OICA_OK;
    default:
      return OICA_E_ARG;
  }
}

int oica_get_option(int option, int *value) {
  if (!value) return OICA_E_ARG;
  switch (option) {
    case OICA_OPT_JACOBI_MAX_SWEEPS: *value = jacobi_max_sweeps(); return OICA_OK;
    case OICA_OPT_COOP_FALLBACKS: *value = coop_fallbacks(); return OICA_OK;
    case OICA_OPT_COOP_LAUNCH_API: *value = coop_launch_api(); return OICA_OK;
    default: return OICA_E_ARG;
  }
}

int oica_whiten_batched(oica_ctx *ctx, int D, oica_whiten_problem *problems, oica_dtype out_t) {
  if (!ctx) return OICA_E_ARG;
  ctx->err.clear();
  if (D < 1 || D > 1024) return fail(ctx, OICA_E_ARG, "D must be in [1, 1024]");
  if (!problems) return fail(ctx, OICA_E_ARG, "problems must be non-null");
  if (out_t != OICA_F32 && out_t != OICA_BF16)
    return fail(ctx, OICA_E_UNSUPPORTED, "out_t must be OICA_F32 or OICA_BF16");
  std::vector<oica::WhitenJob> jobs(D);
  for (int d = 0; d < D; ++d) {
    oica_whiten_problem &q = problems[d];
    q.status = OICA_OK;
    int rc = check_dims(ctx, q.N, q.T);
    if (rc) {
      const std::string why = ctx->err;
      return fail(ctx, rc, "problem %d: %s", d, why.c_str());
    }
    if (!q.X_raw || !q.Xw) return fail(ctx, OICA_E_ARG, "problem %d: X_raw and Xw must be non-null", d);
    if (q.raw_t != OICA_F64 && q.raw_t != OICA_F32)
      return fail(ctx, OICA_E_UNSUPPORTED, "problem %d: raw_t must be OICA_F64 or OICA_F32", d);
    if (q.ld_raw < q.T)
      return fail(ctx, OICA_E_SHAPE, "problem %d: ld_raw (%lld) must be >= T (%lld)", d,
                  (long long)q.ld_raw, (long long)q.T);
    jobs[d] = oica::WhitenJob{q.N,  q.T,     q.X_raw,  q.raw_t, q.ld_raw, q.Xw,
                              out_t, q.Xw_f32, q.V, q.mean,  q.eigval};
  }
  const size_t main_bytes = whiten_batched_workspace_bytes(D, jobs.data());
  int rc = ensure_ws(ctx, main_bytes + (size_t)D * sizeof(int) + 256);
  if (rc) return rc;
  int *flags = (int *)((char *)ctx->ws + ((main_bytes + 255) & ~(size_t)255));
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipMemsetAsync(flags, 0, (size_t)D * sizeof(int), ctx->stream));
  if (int rc2 = ensure_aux(ctx)) return rc2;
  HIP_TRY(ctx, launch_whiten_batched(ctx->stream, D, jobs.data(), ctx->ws, flags, ctx->aux[0],
                                     ctx->aux_ev[KURT_STREAMS], ctx->aux_ev[0]));
  std::vector<int> hf(D);
  HIP_TRY(ctx, hipMemcpyAsync(hf.data(), flags, (size_t)D * sizeof(int), hipMemcpyDeviceToHost,
                              ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  int first = OICA_OK;
  for (int d = 0; d < D; ++d) {
    const int st = (hf[d] & 1)   ? OICA_E_NONFINITE
                   : (hf[d] & 4) ? OICA_E_NOCONV
                   : (hf[d] & 2) ? OICA_E_RANK
                                 : OICA_OK;
    problems[d].status = st;
    if (st != OICA_OK && first == OICA_OK) {
      first = st;
      fail(ctx, st, "problem %d: %s", d,
           st == OICA_E_NONFINITE ? "X_raw contains NaN or Inf"
           : st == OICA_E_NOCONV  ? "the Jacobi solve of the covariance did not converge"
                                  : "covariance is rank deficient (eigenvalue ratio <= 1e-12)");
    }
  }
  return first;
}

// ---------------------------------------------------------------------------
namespace {

// The BF16 row form a run asks for (bf16_row_terms; 0 = the default, hi + lo).
int bf16_form(const oica_fp_params *p) {
  switch (p->bf16_row_terms) {
    case 1: return BF_ONE;
    case 3: return BF_SWITCH;
    case 4: return BF_LATE;
    default: return BF_HILO;
  }
}

int check_fp_params(oica_ctx *ctx, const oica_fp_params *p) {
  if (!p) return fail(ctx, OICA_E_ARG, "params must be non-null");
  if (p->max_iter < 1) return fail(ctx, OICA_E_ARG, "max_iter must be >= 1");
  if (!(p->tol > 0) || !isfinite(p->tol)) return fail(ctx, OICA_E_ARG, "tol must be > 0");
  if (p->precision != OICA_F32 && p->precision != OICA_BF16)
    return fail(ctx, OICA_E_UNSUPPORTED, "precision must be OICA_F32 or OICA_BF16");
  if (p->precision == OICA_BF16 && (!(p->tol_bf16 > 0) || !isfinite(p->tol_bf16)))
    return fail(ctx, OICA_E_ARG, "tol_bf16 must be > 0");
  if (p->refine_iters < 0) return fail(ctx, OICA_E_ARG, "refine_iters must be >= 0");
  if (p->traj_iters < 0 || p->traj_iters > 16) return fail(ctx, OICA_E_ARG, "traj_iters must be in [0, 16]");
  if (p->check_every < 0) return fail(ctx, OICA_E_ARG, "check_every must be >= 0");
  if (p->bf16_row_terms < 0 || p->bf16_row_terms > 4)
    return fail(ctx, OICA_E_ARG, "bf16_row_terms must be 0 to 4");
  if (p->bf16_switch_step < 0 || !isfinite(p->bf16_switch_step))
    return fail(ctx, OICA_E_ARG, "bf16_switch_step must be >= 0");
  return OICA_OK;
}

// Run passes on data X (F32) from the rows currently in B with active list
// act[0] (count already in ctl->kact[0]); returns the number of passes launched.
// Rows on the list a finish phase starts from (its counter's pass-0 count);
// synchronises.  Negative: an OICA_E_* code.
static int finish_rows(oica_ctx *ctx, const FpControl *ctl) {
  HIP_TRY(ctx, hipMemcpyAsync(ctx->small_host, ctl, sizeof(FpControl), hipMemcpyDeviceToHost,
                              ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return ((const FpControl *)ctx->small_host)->kact[0];
}

int run_passes(oica_ctx *ctx, const FusedPlan &plan, int N, int64_t T, const void *X, bool bf16,
               int K, float *B, int *act0, int *act1, float *gpart, float *s4part, double *red,
               FpControl *ctl,
               int max_iter, double tol, int check_every, int32_t *iters, uint8_t *status,
               float *traj, int traj_iters, bool profile, int *launched, double *kernel_ms,
               int exit_below = 0, int stall_polls = 0, const PrunerState *pruner = nullptr,
               int prune_pass = 0, int *keep = nullptr, int *prune_counts = nullptr,
               const double *proj = nullptr, int n_proj = 0, int bf_form = BF_HILO,
               double switch_step = 0.0, int *fine_list = nullptr) {
  // exit_below > 0: stop once at most exit_below rows are active;
  // stall_polls > 0: stop once the active count has not shrunk over that many polls
  // (switched BF16 form: the active count plus the one-term count, so a row
  // that moves to the hi + lo form counts as progress).
  if (!bf16) bf_form = BF_HILO;
  if ((bf_form == BF_SWITCH || bf_form == BF_LATE) && !fine_list) bf_form = BF_HILO;
  int kmax = K;  // upper bound on the active count (it never grows)
  int stalled = 0;
  long long work_prev = 2LL * K + 1;
  *launched = 0;
  *kernel_ms = 0.0;
  // few rows active: the thin items (FP32, up to THIN_PLAN_ROWS rows), or one
  // 32-row block per wave (BF16, at most one such row block; same splits)
  const int np = fused_np(N);
  const FusedPlan narrow = bf16 ? narrow_plan(plan, np) : thin_plan(plan);
  for (int pass = 0; pass < max_iter; ++pass) {
    int *cur = (pass & 1) ? act1 : act0;
    int *nxt = (pass & 1) ? act0 : act1;
    const bool few = bf16 ? (kmax <= bf16_waves(np) * 32 && plan.kwg > bf16_waves(np) * 32)
                          : kmax <= THIN_PLAN_ROWS;
    const FusedPlan &pp = few ? narrow : plan;
    if (profile) {
      while ((int)ctx->events.size() < 2 * (pass + 1)) {
        hipEvent_t e;
        HIP_TRY(ctx, hipEventCreate(&e));
        ctx->events.push_back(e);
      }
      HIP_TRY(ctx, hipEventRecord(ctx->events[2 * pass], ctx->stream));
    }
    // the z^4 sums only feed the trajectory; BF16 passes past it skip them
    float *s4p = (bf16 && pass >= traj_iters) ? nullptr : s4part;
    HIP_TRY(ctx, launch_fused_update(ctx->stream, pp, N, T, X, bf16, B, cur, &ctl->kact[0], 0,
                                     gpart, s4p, ctl, pass, bf_form));
    if (profile) HIP_TRY(ctx, hipEventRecord(ctx->events[2 * pass + 1], ctx->stream));
    *launched = pass + 1;
    HIP_TRY(ctx, launch_epilogue(ctx->stream, pp, N, T, kmax, B, cur, nxt, ctl, pass, gpart,
                                 s4p, red, tol, iters, status, traj, traj_iters, proj, n_proj,
                                 bf16 ? bf_form : 0, switch_step, fine_list));
    if (pruner && pass + 1 == prune_pass) {
      // the list of pass prune_pass is nxt, its count kact[prune_pass & 1]
      HIP_TRY(ctx, hipMemsetAsync(prune_counts, 0, sizeof(int), ctx->stream));
      HIP_TRY(ctx, launch_prune(ctx->stream, pruner, traj, 2 * traj_iters, nxt,
                                &ctl->kact[prune_pass & 1], kmax, status, keep, prune_counts,
                                prune_counts + 1));
      // the survivors are compacted in no particular order: every one of them
      // takes the hi + lo form from here on
      if (bf_form == BF_SWITCH)
        HIP_TRY(ctx, hipMemsetAsync(&ctl->kc[prune_pass & 1], 0, sizeof(int), ctx->stream));
      if (bf_form == BF_LATE)  // every survivor in the head: hi + lo from here on
        HIP_TRY(ctx, hipMemcpyAsync(&ctl->kc[prune_pass & 1], &ctl->kact[prune_pass & 1],
                                    sizeof(int), hipMemcpyDeviceToDevice, ctx->stream));
    }
    if ((pass + 1) % check_every == 0 || pass + 1 == max_iter) {
      HIP_TRY(ctx, hipMemcpyAsync(ctx->small_host, ctl, sizeof(FpControl), hipMemcpyDeviceToHost,
                                  ctx->stream));
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      const FpControl *h = (const FpControl *)ctx->small_host;
      const int left = h->kact[(pass + 1) & 1];
      if (left == 0) break;
      const long long work =
          left + ((bf_form == BF_SWITCH || bf_form == BF_LATE) ? (long long)h->kc[(pass + 1) & 1] : 0LL);
      stalled = (work >= work_prev) ? stalled + 1 : 0;
      work_prev = work;
      kmax = left;
      if (exit_below > 0 && left <= exit_below) break;
      if (stall_polls > 0 && stalled >= stall_polls) break;
    }
  }
  // every pass has been polled past, so all events have completed
  if (profile) {
    for (int i = 0; i < *launched; ++i) {
      float ms = 0.f;
      HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->events[2 * i], ctx->events[2 * i + 1]));
      *kernel_ms += ms;
    }
  }
  return OICA_OK;
}

}  // namespace

struct oica_pruner {
  int device = 0;
  PrunerState st;
};

// The fixed point of oica_fixed_point; proj (n_proj x N FP64 unit rows, device)
// adds Algorithm 1's projection of every start row and update onto the
// complement of those rows (n_proj = 0: none).
static int fixed_point_impl(oica_ctx *ctx, int N, int64_t T, const void *Xw, oica_dtype xw_t,
                            const float *Xw_f32, int K, const float *W0,
                            const oica_fp_params *params, float *W_out, double *kurt,
                            int32_t *iters, uint8_t *status, float *traj, oica_fp_stats *stats,
                            const double *proj, int n_proj);

int oica_fixed_point(oica_ctx *ctx, int N, int64_t T, const void *Xw, oica_dtype xw_t,
                     const float *Xw_f32, int K, const float *W0, const oica_fp_params *params,
                     float *W_out, double *kurt, int32_t *iters, uint8_t *status, float *traj,
                     oica_fp_stats *stats) {
  return fixed_point_impl(ctx, N, T, Xw, xw_t, Xw_f32, K, W0, params, W_out, kurt, iters, status,
                          traj, stats, nullptr, 0);
}

static int fixed_point_impl(oica_ctx *ctx, int N, int64_t T, const void *Xw, oica_dtype xw_t,
                            const float *Xw_f32, int K, const float *W0,
                            const oica_fp_params *params, float *W_out, double *kurt,
                            int32_t *iters, uint8_t *status, float *traj, oica_fp_stats *stats,
                            const double *proj, int n_proj) {
  if (!ctx) return OICA_E_ARG;
  ctx->err.clear();
  int rc = check_dims(ctx, N, T);
  if (rc) return rc;
  if (K < 1) return fail(ctx, OICA_E_ARG, "K must be >= 1 (got %d)", K);
  if (K > (1 << 24)) return fail(ctx, OICA_E_UNSUPPORTED, "K=%d too large", K);
  rc = check_fp_params(ctx, params);
  if (rc) return rc;
  if (!Xw || !Xw_f32 || !W0 || !W_out || !kurt || !iters || !status)
    return fail(ctx, OICA_E_ARG, "Xw, Xw_f32, W0, W_out, kurt, iters and status must be non-null");
  if (params->traj_iters > 0 && !traj) return fail(ctx, OICA_E_ARG, "traj must be non-null when traj_iters > 0");
  const bool bf16 = params->precision == OICA_BF16;
  if (bf16 && xw_t != OICA_BF16) return fail(ctx, OICA_E_ARG, "BF16 precision needs xw_t == OICA_BF16");
  if (!bf16 && xw_t != OICA_F32) return fail(ctx, OICA_E_ARG, "F32 precision needs xw_t == OICA_F32");
  const PrunerState *pruner = params->pruner ? &params->pruner->st : nullptr;
  const int prune_pass = params->prune_pass > 0 ? params->prune_pass : 8;
  const int guard_top = params->guard_top;  // 0: every accepted component
  const int guard_min = params->guard_min > 0 ? params->guard_min : 4;
  if (pruner) {
    if (params->pruner->device != ctx->device)
      return fail(ctx, OICA_E_ARG, "the pruner lives on another device");
    if (prune_pass < 8 || prune_pass > 16)
      return fail(ctx, OICA_E_ARG, "prune_pass must be in [8, 16] (the network reads passes 1-8)");
    if (params->traj_iters > 0 && params->traj_iters < prune_pass)
      return fail(ctx, OICA_E_ARG, "traj_iters must be 0 or >= prune_pass when pruning");
  }
  // the pruner reads the first prune_pass passes of the trajectory
  const int traj_n = pruner ? (params->traj_iters > 0 ? params->traj_iters : prune_pass)
                            : params->traj_iters;

  const auto t0 = std::chrono::steady_clock::now();
  // rows of X start on 16-byte boundaries for the vector loads of the passes:
  // when T does not give that, the passes read padded copies
  const long long ldx = aligned_ld(T, bf16 ? 2 : 4), ld32 = aligned_ld(T, 4);
  const bool pad_x = ldx != T;
  const bool pad_32 = ld32 != T && !(Xw_f32 == Xw && !bf16);
  FusedPlan plan = make_plan(N, T, K, bf16);
  plan.ld = ldx;
  auto plan_f32 = [&]() {
    FusedPlan q = make_plan(N, T, K, false);
    q.ld = ld32;
    return q;
  };
  // the partial and reduction buffers serve every plan of the run: the BF16
  // passes' and, for BF16 runs, the FP32 finish's and the kurtosis pass's
  size_t gfl = fp_workspace_floats(plan, N, K);
  size_t red_n = fp_reduce_doubles(plan, N, K);
  if (bf16) {
    const FusedPlan p32 = plan_f32();
    gfl = std::max(gfl, fp_workspace_floats(p32, N, K));
    red_n = std::max(red_n, fp_reduce_doubles(p32, N, K));
  }
  const int np = fused_np(N);
  const size_t rows_max = gfl / np;
  const int gcap = guard_top > 0 ? guard_top + 64 : K;  // room for the ties / every cluster
  size_t need = 0;
  need += gfl * sizeof(float) + 256;            // gpart
  need += rows_max * sizeof(float) + 256;       // s4part
  need += rows_max * sizeof(double) + 256;      // s4part64 (kurtosis)
  need += red_n * sizeof(double) + 256;         // split-group sums
  need += 6 * ((size_t)K * sizeof(int) + 256);  // act lists, kurtosis list, prune survivors,
                                                // rows entering the BF16 hi + lo form
  need += 4 * (sizeof(FpControl) + 256);
  need += unique_workspace_bytes(K, N) + 256;   // grouping of BF16 fixed points / guard
  if (pruner && !traj) need += (size_t)K * traj_n * 2 * sizeof(float) + 256;
  if (pruner) need += (size_t)gcap * (N * 8 + 8 + 8 + 4 + 4) + 5 * 256;
  if (pad_x) need += (size_t)N * ldx * (bf16 ? 2 : 4) + 256;
  if (pad_32) need += (size_t)N * ld32 * 4 + 256;
  rc = ensure_ws(ctx, need);
  if (rc) return rc;
  Carve cv{(char *)ctx->ws};
  float *gpart = cv.take<float>(gfl);
  float *s4part = cv.take<float>(rows_max);
  double *s4part64 = cv.take<double>(rows_max);
  double *red = cv.take<double>(red_n);
  int *act0 = cv.take<int>(K);
  int *act1 = cv.take<int>(K);
  int *act2 = cv.take<int>(K);
  int *kurt_list = cv.take<int>(K);
  int *keep = cv.take<int>(K);
  int *fine_list = cv.take<int>(K);
  FpControl *ctl = cv.take<FpControl>(1);
  FpControl *ctl2 = cv.take<FpControl>(1);
  (void)cv.take<FpControl>(1);  // third control block (kurtosis list), ctl2 + 256 bytes
  int *prune_counts = (int *)cv.take<FpControl>(1);  // [0] survivors, [1] pruned
  void *gwork = cv.take<char>(unique_workspace_bytes(K, N));
  float *traj_buf = traj;
  if (pruner && !traj) traj_buf = cv.take<float>((size_t)K * traj_n * 2);
  double *gU = nullptr, *gk = nullptr, *gu = nullptr;
  int32_t *grep = nullptr, *gsize = nullptr;
  if (pruner) {
    gU = cv.take<double>((size_t)gcap * N);
    gk = cv.take<double>(gcap);
    gu = cv.take<double>(gcap);
    grep = cv.take<int32_t>(gcap);
    gsize = cv.take<int32_t>(gcap);
  }
  const void *Xp = Xw;
  const float *X32p = Xw_f32;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (pad_x) {
    void *dst = cv.take<char>((size_t)N * ldx * (bf16 ? 2 : 4));
    HIP_TRY(ctx, launch_pad_rows(ctx->stream, Xw, bf16 ? 2 : 4, N, T, dst, ldx));
    Xp = dst;
    if (!bf16 && Xw_f32 == Xw) X32p = (const float *)dst;
  }
  if (pad_32) {
    float *dst = cv.take<float>((size_t)N * ld32);
    HIP_TRY(ctx, launch_pad_rows(ctx->stream, Xw_f32, 4, N, T, dst, ld32));
    X32p = dst;
  }
  HIP_TRY(ctx, hipMemsetAsync(ctl, 0, 4 * 256, ctx->stream));
  HIP_TRY(ctx, launch_init_rows(ctx->stream, K, N, W0, W_out, iters, status, act0, ctl, traj_buf,
                                traj_n, proj, n_proj));
  const int check_every = params->check_every > 0 ? params->check_every : 4;
  const bool profile = params->profile != 0;
  // The BF16 loop ends early once at most K/64 rows are left or the active
  // count stops shrinking (rows that sit at the BF16 rounding floor just above
  // tol_bf16 would otherwise use up max_iter passes); those rows finish on
  // FP32 data.
  const int bf16_exit = bf16 ? (K / 64 > 0 ? K / 64 : 1) : 0;
  const int bf16_stall = bf16 ? 2 : 0;
  long long main_ti = 0, refine_ti = 0;
  int main_passes = 0, launched_total = 0, pruned = 0, tripped = 0;
  double kernel_ms_total = 0.0;

  // attempt 0: every row (pruned at prune_pass when a pruner is set);
  // attempt 1: only when the guard trips, the pruned rows resumed
  for (int attempt = 0; attempt < 2; ++attempt) {
    int launched = 0;
    double kernel_ms = 0.0;
    const bool prune_now = pruner && attempt == 0;
    rc = run_passes(ctx, plan, N, T, Xp, bf16, K, W_out, act0, act1, gpart, s4part, red, ctl,
                    params->max_iter, bf16 ? params->tol_bf16 : params->tol, check_every, iters,
                    status, attempt == 0 ? traj_buf : nullptr, attempt == 0 ? traj_n : 0, profile,
                    &launched, &kernel_ms, bf16_exit, bf16_stall, prune_now ? pruner : nullptr,
                    prune_pass, keep, prune_counts, proj, n_proj, bf16_form(params),
                    params->bf16_switch_step > 0 ? params->bf16_switch_step : 3e-2, fine_list);
    if (rc) return rc;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->small_host, ctl, sizeof(FpControl), hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->small_host + 16, prune_counts, 2 * sizeof(int),
                                hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const FpControl main_ctl = *(const FpControl *)ctx->small_host;
    if (prune_now) pruned = ctx->small_host[17];
    main_ti += main_ctl.thread_iters;
    main_passes += main_ctl.passes;
    launched_total += launched;
    kernel_ms_total += kernel_ms;
    bool kurt_done = false;
    if (bf16) {
      const int left_rows = main_ctl.kact[launched & 1];
      const int *left_list = (launched & 1) ? act1 : act0;
      const int budget_left = params->max_iter - launched;
      const int fp32_passes = budget_left > params->refine_iters ? budget_left : params->refine_iters;
      const FusedPlan plan32 = plan_f32();
      int l2 = 0;
      double ms2 = 0.0;
      HIP_TRY(ctx, hipMemsetAsync(ctl2, 0, 2 * 256, ctx->stream));
      if (params->refine_groups) {
        // group rows that sit at numerically the same BF16 fixed point; one row
        // per group takes the FP32 passes and the kurtosis pass
        int *cluster = nullptr, *reps = nullptr;
        HIP_TRY(ctx, hipMemsetAsync(ctx->small_dev, 0, 4 * sizeof(int), ctx->stream));
        HIP_TRY(ctx, launch_groups(ctx->stream, N, K, W_out, status, 1e-6, gwork, ctx->small_dev,
                                   ctx->small_host, &cluster, &reps));
        FpControl *ctl3 = (FpControl *)((char *)ctl2 + 256);  // kurtosis list counter
        HIP_TRY(ctx, launch_group_lists(ctx->stream, K, cluster, reps, ctx->small_dev + 1, status,
                                        kurt, act2, ctl2, left_list, left_rows, kurt_list, ctl3));
        // the representatives' count bounds the FP32 passes' active rows, so
        // few of them take the thin items from the first pass on
        const int rows0 = finish_rows(ctx, ctl2);
        if (rows0 < 0) return rows0;
        if (fp32_passes > 0 && rows0 > 0) {
          rc = run_passes(ctx, plan32, N, T, X32p, false, rows0, W_out, act2, act0, gpart, s4part,
                          red, ctl2, fp32_passes, params->tol, check_every, iters, status, nullptr,
                          0, false, &l2, &ms2, 0, 0, nullptr, 0, nullptr, nullptr, proj, n_proj);
          if (rc) return rc;
        }
        HIP_TRY(ctx, launch_kurtosis(ctx->stream, plan32, N, T, X32p, K, W_out, s4part64, kurt,
                                     kurt_list, &ctl3->kact[0]));
        HIP_TRY(ctx, launch_propagate(ctx->stream, K, N, cluster, reps, W_out, status, kurt));
        kurt_done = true;
      } else {
        // FP32 passes for every row that converged on BF16 data or is still moving
        HIP_TRY(ctx, launch_refine_select(ctx->stream, K, status, act2, ctl2, left_list, left_rows));
        const int rows0 = finish_rows(ctx, ctl2);
        if (rows0 < 0) return rows0;
        if (fp32_passes > 0 && rows0 > 0) {
          rc = run_passes(ctx, plan32, N, T, X32p, false, rows0, W_out, act2, act0, gpart, s4part,
                          red, ctl2, fp32_passes, params->tol, check_every, iters, status, nullptr,
                          0, false, &l2, &ms2, 0, 0, nullptr, 0, nullptr, nullptr, proj, n_proj);
          if (rc) return rc;
        }
      }
      HIP_TRY(ctx, hipMemcpyAsync(ctx->small_host, ctl2, sizeof(FpControl), hipMemcpyDeviceToHost,
                                  ctx->stream));
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      refine_ti += ((const FpControl *)ctx->small_host)->thread_iters;
    }
    if (!kurt_done)
      HIP_TRY(ctx, launch_kurtosis(ctx->stream, plan_f32(), N, T, X32p, K, W_out,
                                   s4part64, kurt));
    if (!(prune_now && pruned > 0)) break;
    // guard: every checked component must keep guard_min rows in the pruned
    // run, else the pruned rows are resumed
    HIP_TRY(ctx, hipMemsetAsync(ctx->small_dev, 0, 64 * sizeof(int), ctx->stream));
    HIP_TRY(ctx, launch_unique(ctx->stream, N, T, K, W_out, kurt, status, 1e-3, 1, 0, gcap, gU, gk,
                               gu, grep, gsize, gwork, ctx->small_host, ctx->small_dev));
    const int n_acc = ctx->small_host[3];
    const int n_uni = ctx->small_host[1];
    const int n_need = guard_top > 0 ? n_acc : std::min(n_uni, n_acc + 1);
    const int n_got = n_need < gcap ? n_need : gcap;
    std::vector<int32_t> sizes(gcap);
    std::vector<double> ups(gcap);
    if (n_got > 0) {
      HIP_TRY(ctx, hipMemcpy(sizes.data(), gsize, (size_t)n_got * sizeof(int32_t),
                             hipMemcpyDeviceToHost));
      HIP_TRY(ctx, hipMemcpy(ups.data(), gu, (size_t)n_got * sizeof(double), hipMemcpyDeviceToHost));
    }
    // guard_top > 0: the top components, the first guard_top accepted ones and
    // every accepted one whose criterion is within a relative 1e-3 of the
    // guard_top-th (ties).  guard_top == 0: every accepted component and the
    // cluster where the eq. 3 walk stopped.
    bool ok = true;
    if (n_got > 0) {
      if (guard_top > 0) {
        const double cut = ups[(guard_top < n_got ? guard_top : n_got) - 1];
        for (int r = 0; r < n_got; ++r)
          if (r < guard_top || ups[r] >= cut - 1e-3 * fabs(cut)) ok &= sizes[r] >= guard_min;
      } else {
        for (int r = 0; r < n_got; ++r) ok &= sizes[r] >= guard_min;
      }
    }
    if (ok) break;
    tripped = 1;
    HIP_TRY(ctx, hipMemsetAsync(ctl, 0, 256, ctx->stream));
    HIP_TRY(ctx, launch_unprune(ctx->stream, K, status, act0, ctl));
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (stats) {
    stats->thread_iters = main_ti;
    stats->passes = main_passes;
    stats->refine_thread_iters = refine_ti;
    stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    stats->update_ms = profile ? kernel_ms_total : 0.0;
    stats->update_launches = profile ? launched_total : 0;
    stats->pruned = pruned;
    stats->guard_tripped = tripped;
  }
  return OICA_OK;
}

// ---------------------------------------------------------------------------
// Learned pruner
// ---------------------------------------------------------------------------
int oica_pruner_create(oica_ctx *ctx, const float *init_w, const float *feat_mean,
                       const float *feat_std, oica_pruner **out) {
  if (!ctx || !out) return OICA_E_ARG;
  *out = nullptr;
  ctx->err.clear();
  if (!init_w || !feat_mean || !feat_std) return fail(ctx, OICA_E_ARG, "null argument");
  for (int i = 0; i < 16; ++i)
    if (!(feat_std[i] > 0.f) || !isfinite(feat_std[i]) || !isfinite(feat_mean[i]))
      return fail(ctx, OICA_E_ARG, "feature statistics must be finite with std > 0");
  if (int rc = device_ready(ctx)) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  oica_pruner *p = new oica_pruner();
  p->device = ctx->device;
  hipError_t e = pruner_alloc(&p->st, init_w, feat_mean, feat_std);
  if (e != hipSuccess) {
    pruner_free(&p->st);
    delete p;
    return fail(ctx, OICA_E_DEVICE, "pruner allocation failed: %s", hipGetErrorString(e));
  }
  *out = p;
  return OICA_OK;
}

void oica_pruner_destroy(oica_pruner *p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  pruner_free(&p->st);
  delete p;
}

int oica_pruner_get_weights(oica_ctx *ctx, const oica_pruner *p, float *host_w) {
  if (!ctx || !p || !host_w) return OICA_E_ARG;
  if (int rc = device_ready(ctx)) return rc;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  HIP_TRY(ctx, hipMemcpy(host_w, p->st.w32, OICA_PRUNER_PARAMS * sizeof(float), hipMemcpyDeviceToHost));
  return OICA_OK;
}

int oica_pruner_set_threshold(oica_pruner *p, float theta) {
  if (!p || !(theta >= 0.f && theta <= 1.f)) return OICA_E_ARG;
  p->st.theta = theta;
  return OICA_OK;
}

int oica_pruner_predict(oica_ctx *ctx, const oica_pruner *p, const float *traj, int64_t R,
                        float *prob) {
  if (!ctx || !p) return OICA_E_ARG;
  ctx->err.clear();
  if (!traj || !prob || R < 1) return fail(ctx, OICA_E_ARG, "traj, prob must be non-null and R >= 1");
  if (int rc = device_ready(ctx)) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, launch_pruner_predict(ctx->stream, &p->st, traj, R, nullptr, nullptr, prob));
  return OICA_OK;
}

static int pruner_grad_impl(oica_ctx *ctx, const oica_pruner *p, const float *traj,
                            const uint8_t *labels, int64_t R, float w_pos, float *grad,
                            double *loss) {
  if (!traj || !labels || !grad || R < 1 || !(w_pos > 0.f))
    return fail(ctx, OICA_E_ARG, "traj, labels, grad non-null, R >= 1, w_pos > 0 required");
  int rc = ensure_ws(ctx, pruner_grad_workspace_bytes(R) + 512);
  if (rc) return rc;
  double *loss_dev = (double *)((char *)ctx->ws + ctx->ws_bytes - 256);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, launch_pruner_grad(ctx->stream, &p->st, traj, labels, R, RowPerm{}, 0, w_pos, ctx->ws,
                                  grad, loss_dev));
  if (loss) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->small_host, loss_dev, sizeof(double), hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    *loss = *(const double *)ctx->small_host / (double)R;
  }
  return OICA_OK;
}

int oica_pruner_grad(oica_ctx *ctx, const oica_pruner *p, const float *traj, const uint8_t *labels,
                     int64_t R, float w_pos, float *grad, double *loss) {
  if (!ctx || !p) return OICA_E_ARG;
  ctx->err.clear();
  return pruner_grad_impl(ctx, p, traj, labels, R, w_pos, grad, loss);
}

int oica_pruner_train_step(oica_ctx *ctx, oica_pruner *p, const float *traj, const uint8_t *labels,
                           int64_t R, float w_pos, float lr, double *loss) {
  if (!ctx || !p) return OICA_E_ARG;
  ctx->err.clear();
  if (!(lr > 0.f)) return fail(ctx, OICA_E_ARG, "lr must be > 0");
  if (!traj || !labels || R < 1 || !(w_pos > 0.f))
    return fail(ctx, OICA_E_ARG, "traj, labels non-null, R >= 1, w_pos > 0 required");
  // gradient goes to the first bytes of the small device buffer region of the
  // workspace tail; keep it separate from the partials
  int rc = ensure_ws(ctx, pruner_grad_workspace_bytes(R) + OICA_PRUNER_PARAMS * 4 + 1024);
  if (rc) return rc;
  float *grad = (float *)((char *)ctx->ws + ctx->ws_bytes - 512 - OICA_PRUNER_PARAMS * 4);
  rc = pruner_grad_impl(ctx, p, traj, labels, R, w_pos, grad, loss);
  if (rc) return rc;
  HIP_TRY(ctx, launch_pruner_adam(ctx->stream, &p->st, grad, lr));
  return OICA_OK;
}

int oica_pruner_train(oica_ctx *ctx, oica_pruner *p, const float *traj, const uint8_t *labels,
                      int64_t R, int epochs, int batch, float w_pos, float lr, uint64_t seed,
                      double *epoch_loss) {
  if (!ctx || !p) return OICA_E_ARG;
  ctx->err.clear();
  if (!traj || !labels || R < 1) return fail(ctx, OICA_E_ARG, "traj, labels non-null and R >= 1 required");
  if (epochs < 1 || epochs > 100000) return fail(ctx, OICA_E_ARG, "epochs must be in [1, 100000]");
  if (batch < 1) return fail(ctx, OICA_E_ARG, "batch must be >= 1");
  if (!(lr > 0.f)) return fail(ctx, OICA_E_ARG, "lr must be > 0");
  if (!(w_pos >= 0.f)) return fail(ctx, OICA_E_ARG, "w_pos must be >= 0 (0: from the labels)");
  const int64_t bs = std::min<int64_t>(batch, R);
  const int64_t nbat = (R + bs - 1) / bs;
  if ((double)nbat * epochs > 1e8) return fail(ctx, OICA_E_ARG, "too many training steps");
  // workspace: gradient partials of one step | gradient | per-step losses | counter
  const size_t part = (pruner_grad_workspace_bytes(bs) + 255) & ~(size_t)255;
  const size_t gbytes = ((size_t)OICA_PRUNER_PARAMS * 4 + 255) & ~(size_t)255;
  const size_t lbytes = (size_t)nbat * epochs * sizeof(double);
  int rc = ensure_ws(ctx, part + gbytes + lbytes + 1024);
  if (rc) return rc;
  char *w = (char *)ctx->ws;
  float *grad = (float *)(w + part);
  double *losses = (double *)(w + part + gbytes);
  unsigned long long *npos_dev =
      (unsigned long long *)(w + ((part + gbytes + lbytes + 255) & ~(size_t)255));
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (w_pos == 0.f) {
    HIP_TRY(ctx, hipMemsetAsync(npos_dev, 0, sizeof(unsigned long long), ctx->stream));
    HIP_TRY(ctx, launch_count_pos(ctx->stream, labels, R, npos_dev));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->small_host, npos_dev, sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const unsigned long long npos = *(const unsigned long long *)ctx->small_host;
    w_pos = (float)((double)(R - (int64_t)npos) / (double)std::max<unsigned long long>(npos, 1));
    if (!(w_pos > 0.f)) return fail(ctx, OICA_E_ARG, "every label is positive: w_pos would be 0");
  }
  for (int ep = 0; ep < epochs; ++ep) {
    const RowPerm perm = make_row_perm(R, seed, ep);
    for (int64_t b = 0; b < nbat; ++b) {
      const int64_t base = b * bs, rows = std::min<int64_t>(bs, R - base);
      HIP_TRY(ctx, launch_pruner_grad(ctx->stream, &p->st, traj, labels, rows, perm, base, w_pos,
                                      ctx->ws, grad, losses + (size_t)ep * nbat + b));
      HIP_TRY(ctx, launch_pruner_adam(ctx->stream, &p->st, grad, lr));
    }
  }
  if (epoch_loss) {
    std::vector<double> lh((size_t)nbat * epochs);
    HIP_TRY(ctx, hipMemcpyAsync(lh.data(), losses, lbytes, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int ep = 0; ep < epochs; ++ep) {
      double s = 0.0;
      for (int64_t b = 0; b < nbat; ++b)
        s += lh[(size_t)ep * nbat + b] / (double)std::min<int64_t>(bs, R - b * bs);
      epoch_loss[ep] = s / (double)nbat;
    }
  }
  return OICA_OK;
}

int oica_update(oica_ctx *ctx, int N, int64_t T, const void *Xw, oica_dtype xw_t, int K,
                const float *B, double *G, double *s4) {
  if (!ctx) return OICA_E_ARG;
  ctx->err.clear();
  int rc = check_dims(ctx, N, T);
  if (rc) return rc;
  if (K < 1) return fail(ctx, OICA_E_ARG, "K must be >= 1");
  if (!Xw || !B || !G || !s4) return fail(ctx, OICA_E_ARG, "Xw, B, G and s4 must be non-null");
  if (xw_t != OICA_F32 && xw_t != OICA_BF16)
    return fail(ctx, OICA_E_UNSUPPORTED, "xw_t must be OICA_F32 or OICA_BF16");
  const bool bf16 = xw_t == OICA_BF16;
  const FusedPlan plan = make_plan(N, T, K, bf16);
  const size_t gfl = fp_workspace_floats(plan, N, K);
  const size_t rows_max = gfl / fused_np(N);
  rc = ensure_ws(ctx, gfl * 4 + rows_max * 4 + 1024);
  if (rc) return rc;
  Carve cv{(char *)ctx->ws};
  float *gpart = cv.take<float>(gfl);
  float *s4part = cv.take<float>(rows_max);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, launch_fused_update(ctx->stream, plan, N, T, Xw, bf16, B, nullptr, nullptr, K, gpart,
                                   s4part, nullptr, 0));
  HIP_TRY(ctx, launch_update_out(ctx->stream, plan, N, T, K, B, gpart, s4part, G, s4));
  return OICA_OK;
}

int oica_kurtosis_noalloc(oica_ctx *ctx, int N, int64_t T, const float *Xw_f32, int K,
                          const float *W, double *kurt) {
  if (!ctx) return OICA_E_ARG;
  ctx->err.clear();
  int rc = check_dims(ctx, N, T);
  if (rc) return rc;
  if (K < 1) return fail(ctx, OICA_E_ARG, "K must be >= 1");
  if (!Xw_f32 || !W || !kurt) return fail(ctx, OICA_E_ARG, "Xw_f32, W and kurt must be non-null");
  const FusedPlan plan = make_plan(N, T, K, false);
  const size_t rows_max = fp_workspace_floats(plan, N, K) / fused_np(N);
  if (rows_max > NOALLOC_DOUBLES)
    return fail(ctx, OICA_E_UNSUPPORTED,
                "K=%d needs %zu partial sums; the fixed array holds %zu (%d bytes)", K, rows_max,
                NOALLOC_DOUBLES, (int)OICA_NOALLOC_SCRATCH_BYTES);
  if (int rc2 = device_ready(ctx)) return rc2;
  if (!ctx->scratch) return fail(ctx, OICA_E_DEVICE, "no device address for the fixed array");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  // every partial sum the second kernel reads is written by the first in this
  // call, so the array needs no clearing
  HIP_TRY(ctx, launch_kurtosis(ctx->stream, plan, N, T, Xw_f32, K, W, (double *)ctx->scratch,
                               kurt));
  return OICA_OK;
}

int oica_kurtosis(oica_ctx *ctx, int N, int64_t T, const float *Xw_f32, int K, const float *W,
                  double *kurt) {
  if (!ctx) return OICA_E_ARG;
  ctx->err.clear();
  int rc = check_dims(ctx, N, T);
  if (rc) return rc;
  if (K < 1) return fail(ctx, OICA_E_ARG, "K must be >= 1");
  if (!Xw_f32 || !W || !kurt) return fail(ctx, OICA_E_ARG, "Xw_f32, W and kurt must be non-null");
  const FusedPlan plan = make_plan(N, T, K, false);
  const size_t rows_max = fp_workspace_floats(plan, N, K) / fused_np(N);
  rc = ensure_ws(ctx, rows_max * 8 + 1024);
  if (rc) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, launch_kurtosis(ctx->stream, plan, N, T, Xw_f32, K, W, (double *)ctx->ws, kurt));
  return OICA_OK;
}

// ---------------------------------------------------------------------------
// Batched form
// ---------------------------------------------------------------------------
namespace {

int variant_of(int np, int wk, bool bf16) { return (bf16 ? 8 : 0) + (np / 32 - 1) * 2 + (wk - 1); }

std::string tune_key(int D, const oica_problem *pr, bool bf16) {
  // data type, and per padded-N bucket the problem count and log2 of sum K T
  double kt[5] = {0, 0, 0, 0, 0};
  int cnt[5] = {0, 0, 0, 0, 0};
  for (int d = 0; d < D; ++d) {
    const int b = fused_np(pr[d].N) / 32;
    kt[b] += (double)pr[d].K * (double)pr[d].T;
    cnt[b] += 1;
  }
  char buf[256];
  int o = snprintf(buf, sizeof buf, "gfx950|%s", bf16 ? "bf16" : "f32");
  for (int b = 1; b <= 4; ++b)
    if (cnt[b])
      o += snprintf(buf + o, sizeof buf - o, "|np%d:%d:%d", 32 * b, cnt[b],
                    (int)lround(log2(kt[b])));
  return std::string(buf);
}

void tune_cache_load(oica_ctx *ctx, const char *path) {
  if (!path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char line[512], key[300];
  int a, b, g;
  while (fgets(line, sizeof line, f))
    if (sscanf(line, "{\"key\": \"%299[^\"]\", \"wk32\": %d, \"wk64\": %d, \"grid\": %d}", key, &a,
               &b, &g) == 4)
      ctx->tune[key] = {a, b, g};
  fclose(f);
}

void tune_cache_store(const char *path, const std::string &key, const std::vector<int> &v) {
  if (!path) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "{\"key\": \"%s\", \"wk32\": %d, \"wk64\": %d, \"grid\": %d}\n", key.c_str(), v[0], v[1],
          v[2]);
  fclose(f);
}

void set_wk(BatchDesc &b, int wk, bool bf16) {
  b.wk = wk;
  b.kwg = WAVES_PER_WG * wk * 32;
  b.variant = variant_of(b.np, wk, bf16);
  b.n_sp = batch_splits(b.T);
}

// FP32 data, few active rows (thin_max_rows): the thin items, one 32-row
// block per item and one split per wave, with THIN_SPLITS times as many
// splits (rows are padded to 32 instead of 128, and the waves of a work-group
// all work on live rows)
void set_thin(BatchDesc &b) {
  b.wk = 1;
  b.kwg = 32;
  b.variant = THIN_VARIANT + b.np / 32 - 1;
  b.n_sp = THIN_SPLITS * batch_splits(b.T);
}

// Most active rows for the thin items: their partials (THIN_SPLITS times the
// splits, rows padded to 32) must fit the buffers sized for K + 256 rows.
int thin_max_rows(int K) { return K >= 256 ? 128 : 32; }

// Thin items of a problem with at most two row blocks left take four times the
// splits again (each wave walks a quarter of the samples, so a pass that only
// such problems still run finishes sooner; twice was 1 % slower on the
// many-dataset workload), when those splits' partials fit the buffers:
// 4 THIN_SPLITS x padded rows <= K + 256 per split of the problem's own
// partition, and their first-stage sums (groups x active rows) within
// red_doubles.  Returns whether the shape changed.
size_t red_doubles(int n_sp, int K, int np);
bool thin_wider(BatchDesc &b, int kd) {
  const int base = batch_splits(b.T);
  if (b.variant < THIN_VARIANT || b.n_sp != THIN_SPLITS * base || kd > 64 || kd <= 0) return false;
  const int wide = 4 * THIN_SPLITS * base;
  if ((size_t)wide * 32 * ((kd + 31) / 32) > (size_t)base * (b.K + 256)) return false;
  const size_t groups = (size_t)(wide + SPLIT_GROUP_HOST - 1) / SPLIT_GROUP_HOST;
  if (groups * (size_t)kd * (size_t)(b.np + 1) > red_doubles(base, b.K, b.np)) return false;
  b.n_sp = wide;
  return true;
}

// First-stage reduction sums of one problem: enough for the regular shapes
// (up to K rows) and for the thin ones.
size_t red_doubles(int n_sp, int K, int np) {
  const size_t wide = (size_t)((n_sp + SPLIT_GROUP_HOST - 1) / SPLIT_GROUP_HOST) * K;
  const size_t thin = (size_t)((THIN_SPLITS * n_sp + SPLIT_GROUP_HOST - 1) / SPLIT_GROUP_HOST) *
                      thin_max_rows(K);
  return std::max(wide, thin) * (size_t)(np + 1);
}
bool is_thin(const BatchDesc &b) { return b.variant >= THIN_VARIANT; }

void set_shapes(std::vector<BatchDesc> &hd, int wk32, int wk64, bool bf16) {
  for (auto &b : hd) set_wk(b, b.np == 32 ? wk32 : (b.np == 64 ? wk64 : 1), bf16);
}

}  // namespace

int oica_fixed_point_batched(oica_ctx *ctx, int D, const oica_problem *pr, oica_dtype xw_t,
                             const oica_fp_params *params, const oica_batch_params *bparams,
                             oica_batch_stats *stats) {
  if (!ctx) return OICA_E_ARG;
  ctx->err.clear();
  if (D < 1 || D > batch_max_datasets())
    return fail(ctx, OICA_E_ARG, "D must be in [1, %d] (got %d)", batch_max_datasets(), D);
  if (!pr) return fail(ctx, OICA_E_ARG, "problems must be non-null");
  int rc = check_fp_params(ctx, params);
  if (rc) return rc;
  if (params->traj_iters != 0) return fail(ctx, OICA_E_ARG, "traj_iters must be 0 in the batched form");
  const bool bf16 = params->precision == OICA_BF16;
  if (bf16 != (xw_t == OICA_BF16)) return fail(ctx, OICA_E_ARG, "xw_t must match params->precision");
  for (int d = 0; d < D; ++d) {
    const oica_problem &q = pr[d];
    rc = check_dims(ctx, q.N, q.T);
    if (rc) return fail(ctx, rc, "problem %d: %s", d, ctx->err.c_str());
    if (q.K < 1 || q.K > (1 << 24)) return fail(ctx, OICA_E_ARG, "problem %d: K=%d out of range", d, q.K);
    if (!q.Xw || !q.Xw_f32 || !q.W0 || !q.W_out || !q.kurt || !q.iters || !q.status)
      return fail(ctx, OICA_E_ARG, "problem %d: null pointer", d);
  }
  const auto t0 = std::chrono::steady_clock::now();
  const bool profile = params->profile != 0;
  const int check_every = params->check_every > 0 ? params->check_every : 4;

  // ---- layout --------------------------------------------------------------
  std::vector<BatchDesc> hd(D);
  size_t need = 0;
  auto add = [&](size_t bytes) { need += (bytes + 255) & ~(size_t)255; };
  long long ktot = 0;
  size_t kurt_rows = 0;
  for (int d = 0; d < D; ++d) {
    const oica_problem &q = pr[d];
    BatchDesc &b = hd[d];
    b.N = q.N; b.T = q.T; b.K = q.K;
    b.np = fused_np(q.N);
    // 16-byte row starts for the passes' vector loads (padded copies otherwise)
    b.ld = aligned_ld(q.T, bf16 ? 2 : 4);
    b.ld32 = aligned_ld(q.T, 4);
    if (b.ld != q.T) add((size_t)q.N * b.ld * (bf16 ? 2 : 4));
    if (b.ld32 != q.T && !(q.Xw_f32 == q.Xw && !bf16)) add((size_t)q.N * b.ld32 * 4);
    b.n_sp = batch_splits(q.T);
    b.n_sub = (int)((q.T + 31) / 32);
    const size_t rows_cap = (size_t)q.K + 256;
    add((size_t)b.n_sp * rows_cap * b.np * 4);                              // gpart
    add((size_t)b.n_sp * rows_cap * 4);                                     // s4part
    add(red_doubles(b.n_sp, q.K, b.np) * 8);                                // red
    add((size_t)q.K * 4 * 3);                                               // act lists
    ktot += q.K;
    const FusedPlan kp = make_plan(q.N, q.T, q.K, false);
    kurt_rows = std::max(kurt_rows, fp_workspace_floats(kp, q.N, q.K) / (size_t)fused_np(q.N));
  }
  add((size_t)D * sizeof(BatchDesc));
  add(sizeof(BatchCtl));
  add((size_t)(D + 1) * 4 * 2 + (size_t)(D + 1) * 8);
  add((size_t)D * 256 * 2);  // two control blocks per problem
  for (int i = 0; i < KURT_STREAMS; ++i) add(kurt_rows * 8);  // one partial buffer per stream
  const bool grouped = bf16 && params->refine_groups;
  if (grouped) {
    add((size_t)D * 256);                 // clustering control, 4 ints per problem
    add((size_t)D * sizeof(ClusterJob));
    for (int d = 0; d < D; ++d) {
      add(unique_workspace_bytes(pr[d].K, pr[d].N));  // grouping of the BF16 fixed points
      add((size_t)pr[d].K * 4);              // kurtosis list
    }
  }
  rc = ensure_ws(ctx, need + 4096);
  if (rc) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  Carve cv{(char *)ctx->ws};
  BatchDesc *ddesc = cv.take<BatchDesc>(D);
  BatchCtl *bctl = cv.take<BatchCtl>(1);
  int *item_start = cv.take<int>(D + 1);
  int *epi_start = cv.take<int>(D + 1);
  long long *red_start = cv.take<long long>(D + 1);
  char *ctl_base = cv.take<char>((size_t)D * 256 * 2);
  double *s4part64[KURT_STREAMS];
  for (int i = 0; i < KURT_STREAMS; ++i) s4part64[i] = cv.take<double>(kurt_rows);
  int *gctl = nullptr;
  ClusterJob *gjobs_dev = nullptr;
  std::vector<ClusterJob> gjobs;
  std::vector<ClusterWs> gws;
  std::vector<int *> kurt_list(D, nullptr);
  if (grouped) {
    gctl = cv.take<int>((size_t)D * 64);
    gjobs_dev = cv.take<ClusterJob>(D);
    gjobs.resize(D);
    gws.resize(D);
    for (int d = 0; d < D; ++d) {
      const int K = pr[d].K;
      gws[d] = carve_cluster_ws(cv.take<char>(unique_workspace_bytes(K, pr[d].N)), K, pr[d].N);
      gjobs[d] = ClusterJob{K, pr[d].N, pr[d].W_out, gws[d].Wt, gws[d].key, gws[d].cluster,
                            gws[d].reps, gctl + 64 * d};
      kurt_list[d] = cv.take<int>((size_t)K);
    }
  }
  std::vector<int *> act2(D);
  for (int d = 0; d < D; ++d) {
    const oica_problem &q = pr[d];
    BatchDesc &b = hd[d];
    const size_t rows_cap = (size_t)q.K + 256;
    b.gpart = cv.take<float>((size_t)b.n_sp * rows_cap * b.np);
    b.s4part = cv.take<float>((size_t)b.n_sp * rows_cap);
    b.red = cv.take<double>(red_doubles(b.n_sp, q.K, b.np));
    b.act0 = cv.take<int>(q.K);
    b.act1 = cv.take<int>(q.K);
    act2[d] = cv.take<int>(q.K);
    b.ctl = (FpControl *)(ctl_base + (size_t)d * 256);
    b.X = q.Xw;
    b.X32 = q.Xw_f32;
    if (b.ld != q.T) {
      void *dst = cv.take<char>((size_t)q.N * b.ld * (bf16 ? 2 : 4));
      HIP_TRY(ctx, launch_pad_rows(ctx->stream, q.Xw, bf16 ? 2 : 4, q.N, q.T, dst, b.ld));
      b.X = dst;
      if (!bf16 && q.Xw_f32 == q.Xw) b.X32 = (const float *)dst;
    }
    if (b.ld32 != q.T && !(q.Xw_f32 == q.Xw && !bf16)) {
      float *dst = cv.take<float>((size_t)q.N * b.ld32);
      HIP_TRY(ctx, launch_pad_rows(ctx->stream, q.Xw_f32, 4, q.N, q.T, dst, b.ld32));
      b.X32 = dst;
    }
    b.B = q.W_out;
    b.iters = q.iters;
    b.status = q.status;
    // the batched form has the one-term and the hi + lo row forms (the
    // switched form runs as hi + lo)
    b.bf_one = (bf16 && bf16_form(params) == BF_ONE) ? 1 : 0;
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipMemsetAsync(ctl_base, 0, (size_t)D * 256 * 2, ctx->stream));
  // the per-dataset launches of a few microseconds each (start rows here,
  // the grouping's preparation and lists below) side by side on the
  // auxiliary streams
  rc = aux_fork(ctx);
  if (rc) return rc;
  for (int d = 0; d < D; ++d)
    HIP_TRY(ctx, launch_init_rows(ctx->aux[d % KURT_STREAMS], pr[d].K, pr[d].N, pr[d].W0,
                                  pr[d].W_out, pr[d].iters, pr[d].status, hd[d].act0, hd[d].ctl,
                                  nullptr, 0));
  rc = aux_join(ctx);
  if (rc) return rc;

  // ---- tile shapes: forced, cached, tuned or default -------------------------
  int wk32 = 2, wk64 = 2, grid = 1024, tuned = 0;
  const oica_batch_params bp0 = {0, nullptr, 0, 0};
  const oica_batch_params &bp = bparams ? *bparams : bp0;
  const std::string key = tune_key(D, pr, bf16);
  if (bp.force_wk == 1 || bp.force_wk == 2) {
    wk32 = wk64 = bp.force_wk;
  } else if (bp.autotune) {
    tune_cache_load(ctx, bp.cache_path);
    auto it = ctx->tune.find(key);
    if (it != ctx->tune.end()) {
      wk32 = it->second[0];
      wk64 = it->second[1];
      grid = it->second[2];
      tuned = 2;
    } else {
      // time pass 0 (all rows active; it only writes partial buffers) for each
      // candidate shape, best of two runs
      bool has32 = false, has64 = false;
      for (auto &b : hd) {
        has32 |= b.np == 32;
        has64 |= b.np == 64;
      }
      std::vector<std::vector<int>> cands;
      for (int a : {1, 2})
        for (int c : {1, 2})
          for (int g : {512, 1024, 2048}) {
            if ((!has32 && a == 2) || (!has64 && c == 2)) continue;
            cands.push_back({a, c, g});
          }
      while ((int)ctx->events.size() < 2) {
        hipEvent_t e;
        HIP_TRY(ctx, hipEventCreate(&e));
        ctx->events.push_back(e);
      }
      float best = 1e30f;
      std::vector<int> pick = {2, 2, 1024};
      for (const auto &c : cands) {
        set_shapes(hd, c[0], c[1], bf16);
        HIP_TRY(ctx, hipMemcpyAsync(ddesc, hd.data(), (size_t)D * sizeof(BatchDesc),
                                    hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // hd is reused next
        float tbest = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
          HIP_TRY(ctx, launch_batch_plan(ctx->stream, ddesc, D, bctl, item_start, red_start, epi_start,
                                         0, true));
          HIP_TRY(ctx, hipEventRecord(ctx->events[0], ctx->stream));
          HIP_TRY(ctx, launch_fused_batched(ctx->stream, ddesc, D, bctl, item_start, 0, c[2], bf16));
          HIP_TRY(ctx, hipEventRecord(ctx->events[1], ctx->stream));
          HIP_TRY(ctx, hipEventSynchronize(ctx->events[1]));
          float ms = 0.f;
          HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->events[0], ctx->events[1]));
          tbest = std::min(tbest, ms);
        }
        if (tbest < best) {
          best = tbest;
          pick = c;
        }
      }
      wk32 = pick[0];
      wk64 = pick[1];
      grid = pick[2];
      tuned = 1;
      ctx->tune[key] = pick;
      tune_cache_store(bp.cache_path, key, pick);
    }
  }
  if (bp.force_grid > 0) grid = ((bp.force_grid + 7) / 8) * 8;
  set_shapes(hd, wk32, wk64, bf16);
  HIP_TRY(ctx, hipMemcpyAsync(ddesc, hd.data(), (size_t)D * sizeof(BatchDesc), hipMemcpyHostToDevice,
                              ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));

  // ---- passes -----------------------------------------------------------------
  std::vector<char> ctl_host((size_t)D * 256 * 2);
  // Early exit of the BF16 loop, per problem: a problem whose active count is
  // at most K/64, or has not shrunk over two polls, is parked (its count is set
  // to zero, its active list is left as it is) and its rows go on to the FP32
  // passes.  The decisions use the problem's own counts at the common poll
  // passes, so they do not depend on the other problems of the batch.
  std::vector<int> park_count(D, -1), park_parity(D, 0);
  auto run = [&](int max_passes, double tol, bool park, bool data_bf16, int *launched,
                 double *kernel_ms) -> int {
    long long kmax = ktot;
    std::vector<int> kprev(D), stalled(D, 0);
    for (int d = 0; d < D; ++d) kprev[d] = pr[d].K;
    *launched = 0;
    *kernel_ms = 0.0;
    for (int pass = 0; pass < max_passes; ++pass) {
      HIP_TRY(ctx, launch_batch_plan(ctx->stream, ddesc, D, bctl, item_start, red_start, epi_start,
                                     pass, false));
      if (profile) {
        while ((int)ctx->events.size() < 2 * (pass + 1)) {
          hipEvent_t e;
          HIP_TRY(ctx, hipEventCreate(&e));
          ctx->events.push_back(e);
        }
        HIP_TRY(ctx, hipEventRecord(ctx->events[2 * pass], ctx->stream));
      }
      HIP_TRY(ctx, launch_fused_batched(ctx->stream, ddesc, D, bctl, item_start, pass, grid,
                                        data_bf16));
      if (profile) HIP_TRY(ctx, hipEventRecord(ctx->events[2 * pass + 1], ctx->stream));
      HIP_TRY(ctx, launch_epilogue_batched(ctx->stream, ddesc, D, bctl, red_start, epi_start, pass,
                                           tol, (int)kmax));
      *launched = pass + 1;
      if ((pass + 1) % check_every == 0 || pass + 1 == max_passes) {
        HIP_TRY(ctx, hipMemcpyAsync(ctl_host.data(), hd[0].ctl, (size_t)D * 256, hipMemcpyDeviceToHost,
                                    ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        const int par = (pass + 1) & 1;
        long long left = 0;
        bool parked_now = false, reshaped = false;
        for (int d = 0; d < D; ++d) {
          int kd = ((const FpControl *)(ctl_host.data() + (size_t)d * 256))->kact[par];
          // at most one narrow row block left: one 32-row block per wave from
          // the next pass on (same sample splits, so the same arithmetic)
          if (hd[d].wk > 1 && kd <= WAVES_PER_WG * 32) {
            set_wk(hd[d], 1, data_bf16);
            reshaped = true;
          }
          if (!data_bf16 && !is_thin(hd[d]) && kd <= thin_max_rows(hd[d].K)) {
            set_thin(hd[d]);
            reshaped = true;
          }
          if (!data_bf16 && thin_wider(hd[d], kd)) reshaped = true;
          // BF16, few rows: THIN_SPLITS times the splits (shorter items, so the
          // long latency-bound items of a few problems no longer set the pass);
          // the partial buffers (K + 256 rows per split) must hold the
          // THIN_SPLITS x 128 padded rows
          if (data_bf16 && hd[d].wk == 1 && hd[d].n_sp == batch_splits(hd[d].T) &&
              kd <= thin_max_rows(hd[d].K) && THIN_SPLITS * hd[d].kwg <= hd[d].K + 256) {
            hd[d].n_sp = THIN_SPLITS * batch_splits(hd[d].T);
            reshaped = true;
          }
          if (park && park_count[d] < 0 && kd > 0) {
            stalled[d] = kd >= kprev[d] ? stalled[d] + 1 : 0;
            kprev[d] = kd;
            if (kd <= std::max(pr[d].K / 64, 1) || stalled[d] >= 2) {
              park_count[d] = kd;
              park_parity[d] = par;
              HIP_TRY(ctx, hipMemsetAsync(&hd[d].ctl->kact[par], 0, sizeof(int), ctx->stream));
              parked_now = true;
              kd = 0;
            }
          }
          left += kd;
        }
        if (reshaped)
          HIP_TRY(ctx, hipMemcpyAsync(ddesc, hd.data(), (size_t)D * sizeof(BatchDesc),
                                      hipMemcpyHostToDevice, ctx->stream));
        if (parked_now || reshaped) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (left == 0) break;
        kmax = left;
      }
    }
    if (profile)
      for (int i = 0; i < *launched; ++i) {
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->events[2 * i], ctx->events[2 * i + 1]));
        *kernel_ms += ms;
      }
    return OICA_OK;
  };
  int launched = 0;
  double kernel_ms = 0.0;
  rc = run(params->max_iter, bf16 ? params->tol_bf16 : params->tol, bf16, bf16, &launched,
           &kernel_ms);
  if (rc) return rc;
  HIP_TRY(ctx, hipMemcpyAsync(ctl_host.data(), hd[0].ctl, (size_t)D * 256, hipMemcpyDeviceToHost,
                              ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  long long main_ti = 0, refine_ti = 0;
  double main_flops = 0.0;
  int main_passes = 0;
  for (int d = 0; d < D; ++d) {
    const FpControl *c = (const FpControl *)(ctl_host.data() + (size_t)d * 256);
    main_ti += c->thread_iters;
    main_flops += 4.0 * pr[d].N * (double)pr[d].T * (double)c->thread_iters;
    main_passes = std::max(main_passes, c->passes);
  }
  if (bf16) {
    // FP32 passes: grouped, for one row per group of rows at numerically the
    // same BF16 fixed point (1 - |cos| <= 1e-6) plus the rows still moving;
    // otherwise for every row that converged on BF16 data or is still moving
    if (grouped) {
      HIP_TRY(ctx, hipMemsetAsync(gctl, 0, (size_t)D * 64 * sizeof(int), ctx->stream));
      rc = aux_fork(ctx);
      if (rc) return rc;
      for (int d = 0; d < D; ++d)
        HIP_TRY(ctx, launch_prep_groups(ctx->aux[d % KURT_STREAMS], pr[d].K, pr[d].N, pr[d].status,
                                        pr[d].W_out, gws[d]));
      rc = aux_join(ctx);
      if (rc) return rc;
      std::vector<ClusterJob> small;
      for (int d = 0; d < D; ++d)
        if (cluster_in_one_wg(pr[d].K, true)) small.push_back(gjobs[d]);
      if (!small.empty()) {
        HIP_TRY(ctx, hipMemcpyAsync(gjobs_dev, small.data(), small.size() * sizeof(ClusterJob),
                                    hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // `small` is a local table
        int k_small = 0;
        for (const ClusterJob &j : small) k_small = std::max(k_small, j.K);
        HIP_TRY(ctx, launch_cluster_wg(ctx->stream, (int)small.size(), gjobs_dev, small[0], 1e-6,
                                       k_small));
      }
      for (int d = 0; d < D; ++d)
        if (!cluster_in_one_wg(pr[d].K, true)) {
          int *reps = nullptr, *cl = nullptr;
          HIP_TRY(ctx, launch_groups(ctx->stream, pr[d].N, pr[d].K, pr[d].W_out, pr[d].status, 1e-6,
                                     (void *)gws[d].key, gjobs[d].ctl, ctx->small_host, &cl, &reps));
        }
    }
    rc = aux_fork(ctx);
    if (rc) return rc;
    for (int d = 0; d < D; ++d) {
      const FpControl *c = (const FpControl *)(ctl_host.data() + (size_t)d * 256);
      BatchDesc &b = hd[d];
      FpControl *c2 = (FpControl *)(ctl_base + (size_t)(D + d) * 256);
      const bool parked = park_count[d] >= 0;
      const int par = parked ? park_parity[d] : (launched & 1);
      const int *left_list = par ? b.act1 : b.act0;
      const int left = parked ? park_count[d] : c->kact[launched & 1];
      hipStream_t sd = ctx->aux[d % KURT_STREAMS];
      if (grouped)
        HIP_TRY(ctx, launch_group_lists(sd, b.K, gjobs[d].cluster, gjobs[d].reps,
                                        gjobs[d].ctl + 1, b.status, pr[d].kurt, act2[d], c2,
                                        left_list, left, kurt_list[d],
                                        (FpControl *)((char *)c2 + 128)));
      else
        HIP_TRY(ctx, launch_refine_select(sd, b.K, b.status, act2[d], c2, left_list, left));
      int *old0 = b.act0;
      b.act0 = act2[d];
      b.act1 = old0;
      b.ctl = c2;
      b.X = b.X32;
      b.ld = b.ld32;
      b.bf_one = 0;
    }
    rc = aux_join(ctx);
    if (rc) return rc;
    // the FP32 passes update few rows per problem: one 32-row block per wave,
    // and the thin items where few enough rows start
    set_shapes(hd, 1, 1, false);
    HIP_TRY(ctx, hipMemcpyAsync(ctl_host.data() + (size_t)D * 256, ctl_base + (size_t)D * 256,
                                (size_t)D * 256, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int d = 0; d < D; ++d) {
      const int k0 = ((const FpControl *)(ctl_host.data() + (size_t)(D + d) * 256))->kact[0];
      if (k0 <= thin_max_rows(hd[d].K)) {
        set_thin(hd[d]);
        thin_wider(hd[d], k0);
      }
    }
    HIP_TRY(ctx, hipMemcpyAsync(ddesc, hd.data(), (size_t)D * sizeof(BatchDesc),
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const int budget = params->max_iter - launched;
    const int passes32 = std::max(budget, params->refine_iters);
    int l2 = 0;
    double ms2 = 0.0;
    if (passes32 > 0) {
      rc = run(passes32, params->tol, false, false, &l2, &ms2);
      if (rc) return rc;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctl_host.data() + (size_t)D * 256, ctl_base + (size_t)D * 256,
                                (size_t)D * 256, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int d = 0; d < D; ++d)
      refine_ti += ((const FpControl *)(ctl_host.data() + (size_t)(D + d) * 256))->thread_iters;
  }
  // The datasets' kurtosis passes (each alone too small to fill the GPU) run
  // side by side on the auxiliary streams, dataset d on stream d mod
  // KURT_STREAMS with that stream's partial buffer; the streams start after
  // everything enqueued so far and the call's stream waits for all of them.
  rc = aux_fork(ctx);
  if (rc) return rc;
  for (int d = 0; d < D; ++d) {
    const oica_problem &q = pr[d];
    hipStream_t sd = ctx->aux[d % KURT_STREAMS];
    double *s4d = s4part64[d % KURT_STREAMS];
    FusedPlan kp = make_plan(q.N, q.T, q.K, false);
    kp.ld = hd[d].ld32;
    if (grouped) {
      // kurtosis of the group representatives and of the ungrouped rows, then
      // every group member takes its representative's row, status and kurtosis
      FpControl *c3 = (FpControl *)(ctl_base + (size_t)(D + d) * 256 + 128);
      HIP_TRY(ctx, launch_kurtosis(sd, kp, q.N, q.T, hd[d].X32, q.K, q.W_out, s4d, q.kurt,
                                   kurt_list[d], &c3->kact[0]));
      HIP_TRY(ctx, launch_propagate(sd, q.K, q.N, gjobs[d].cluster, gjobs[d].reps, q.W_out,
                                    q.status, q.kurt));
    } else {
      // final kurtosis of every row, FP32 data, FP64 sums
      HIP_TRY(ctx, launch_kurtosis(sd, kp, q.N, q.T, hd[d].X32, q.K, q.W_out, s4d, q.kurt));
    }
  }
  rc = aux_join(ctx);
  if (rc) return rc;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (stats) {
    stats->thread_iters = main_ti;
    stats->refine_thread_iters = refine_ti;
    stats->passes = main_passes;
    stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    stats->update_ms = profile ? kernel_ms : 0.0;
    stats->update_launches = profile ? launched : 0;
    stats->grid = grid;
    stats->wk32 = wk32;
    stats->wk64 = wk64;
    stats->tuned = tuned;
    stats->update_flops = main_flops;
  }
  return OICA_OK;
}

// ---------------------------------------------------------------------------
int oica_unique(oica_ctx *ctx, int N, int64_t T, int K, const float *W, const double *kurt,
                const uint8_t *status, const oica_unique_params *params, int cap, double *U,
                double *kurt_u, double *ups_u, int32_t *rep_thread, int32_t *cluster_size,
                int32_t *row_cluster, int *n_unique, int *n_accepted) {
  if (!ctx) return OICA_E_ARG;
  ctx->err.clear();
  int rc = check_dims(ctx, N, T);
  if (rc) return rc;
  if (K < 1) return fail(ctx, OICA_E_ARG, "K must be >= 1");
  if (!params) return fail(ctx, OICA_E_ARG, "params must be non-null");
  if (!(params->tau > 0.0 && params->tau < 1.0)) return fail(ctx, OICA_E_ARG, "tau must be in (0, 1)");
  if (params->n_top < 0) return fail(ctx, OICA_E_ARG, "n_top must be >= 0");
  if (cap < 0) return fail(ctx, OICA_E_ARG, "cap must be >= 0");
  if (!W || !kurt || !status || !n_unique || !n_accepted)
    return fail(ctx, OICA_E_ARG, "W, kurt, status, n_unique and n_accepted must be non-null");
  if (cap > 0 && (!U || !kurt_u || !ups_u || !rep_thread || !cluster_size))
    return fail(ctx, OICA_E_ARG, "output arrays must be non-null when cap > 0");
  rc = ensure_ws(ctx, unique_workspace_bytes(K, N));
  if (rc) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipMemsetAsync(ctx->small_dev, 0, 64 * sizeof(int), ctx->stream));
  HIP_TRY(ctx, launch_unique(ctx->stream, N, T, K, W, kurt, status, params->tau,
                             params->gaussianity_test, params->n_top, cap, U, kurt_u, ups_u,
                             rep_thread, cluster_size, ctx->ws, ctx->small_host, ctx->small_dev,
                             row_cluster));
  *n_unique = ctx->small_host[1];
  *n_accepted = ctx->small_host[3];
  if (cap < *n_unique)
    return fail(ctx, OICA_E_SHAPE, "cap=%d is smaller than the %d clusters found", cap, *n_unique);
  return OICA_OK;
}

int oica_deflation(oica_ctx *ctx, int N, int64_t T, const float *Xw, int L, const float *W0,
                   const oica_fp_params *params, double tau, int gaussianity_test, double *W_out,
                   int *n_found, oica_deflation_step *steps) {
  if (!ctx) return OICA_E_ARG;
  ctx->err.clear();
  int rc = check_dims(ctx, N, T);
  if (rc) return rc;
  if (L < 1 || L > (1 << 24)) return fail(ctx, OICA_E_ARG, "L must be in [1, 2^24] (got %d)", L);
  rc = check_fp_params(ctx, params);
  if (rc) return rc;
  if (params->pruner) return fail(ctx, OICA_E_ARG, "the deflation driver runs without the pruner");
  if (params->traj_iters != 0) return fail(ctx, OICA_E_ARG, "traj_iters must be 0");
  if (!(tau > 0.0 && tau < 1.0)) return fail(ctx, OICA_E_ARG, "tau must be in (0, 1)");
  if (!Xw || !W0 || !W_out || !n_found) return fail(ctx, OICA_E_ARG, "Xw, W0, W_out and n_found must be non-null");
  const bool bf16 = params->precision == OICA_BF16;
  *n_found = 0;
  // buffers of the driver itself (the calls below use the context workspace)
  const size_t nn = (size_t)N * N;
  size_t need = 0;
  need += (size_t)N * T * 4 + 256;                       // X~ FP32
  if (bf16) need += (size_t)N * T * 2 + 256;             // X~ BF16
  need += 5 * (nn * 8 + 256) + (size_t)N * 8 * 2 + 512;  // Ft, C, E (+eigenvalues), G, Wh, mean 0
  need += jacobi_log_entries(N) * (sizeof(double2) + sizeof(int)) + 512 + 256;
  need += (size_t)L * N * 4 + 256;                       // fixed-point rows
  need += (size_t)L * (8 + 4 + 1) + 3 * 256;             // kurt, iters, status
  need += (size_t)L * (N * 8 + 8 + 8 + 4 + 4) + 5 * 256; // unique outputs (cap L)
  rc = ensure_buf(ctx, &ctx->ws2, &ctx->ws2_bytes, need);
  if (rc) return rc;
  Carve cv{(char *)ctx->ws2};
  float *xt32 = cv.take<float>((size_t)N * T);
  uint16_t *xt16 = bf16 ? cv.take<uint16_t>((size_t)N * T) : nullptr;
  double *Ft = cv.take<double>(nn);
  double *C = cv.take<double>(nn);
  double *E = cv.take<double>(nn + N);
  double *G = cv.take<double>(nn);
  double *Wh = cv.take<double>(nn);
  double *zero = cv.take<double>(N);
  double2 *rot = cv.take<double2>(jacobi_log_entries(N));
  int *pq = cv.take<int>(jacobi_log_entries(N));
  int *sweeps = cv.take<int>(64);
  int *flag = cv.take<int>(64);
  float *B = cv.take<float>((size_t)L * N);
  double *kurt = cv.take<double>(L);
  int32_t *iters = cv.take<int32_t>(L);
  uint8_t *status = cv.take<uint8_t>(L);
  double *U = cv.take<double>((size_t)L * N);
  double *ku = cv.take<double>(L);
  double *uu = cv.take<double>(L);
  int32_t *rep = cv.take<int32_t>(L);
  int32_t *csz = cv.take<int32_t>(L);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipMemsetAsync(zero, 0, (size_t)N * 8, ctx->stream));
  size_t w0_off = 0;  // step i's start rows: L x (N - i + 1) after those of steps 1 .. i-1
  for (int i = 1; i <= N; ++i) {
    const int n_prev = i - 1, n = N - n_prev;
    // eqs. 6-8: F = I - W^T W without its bottom i-1 rows, G = (F~ F~^T)^(-1/2) F~,
    // X~ = G Xw (at i = 1: G = I)
    HIP_TRY(ctx, hipMemsetAsync(flag, 0, sizeof(int), ctx->stream));
    HIP_TRY(ctx, launch_defl_gram(ctx->stream, N, n_prev, W_out, Ft, C));
    HIP_TRY(ctx, launch_jacobi(ctx->stream, 1, nullptr,
                               JacJob{n, C, E, rot, pq, sweeps, flag, jacobi_max_sweeps()}, n));
    HIP_TRY(ctx, launch_defl_basis(ctx->stream, N, n_prev, Ft, E, 1e-12, G, Wh, flag));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->small_host + 8, flag, sizeof(int), hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->small_host[8] & 4)
      return fail(ctx, OICA_E_NOCONV, "step %d: the Jacobi solve of F~ F~^T did not converge", i);
    if (ctx->small_host[8])
      return fail(ctx, OICA_E_RANK, "step %d: F~ F~^T is singular (the first %d rows of "
                  "I - W^T W do not span the complement)", i, n);
    HIP_TRY(ctx, launch_apply_rows(ctx->stream, N, n, T, Xw, T, Wh, zero, xt32, xt16));
    oica_fp_stats st{};
    rc = oica_fixed_point(ctx, n, T, bf16 ? (const void *)xt16 : (const void *)xt32,
                          bf16 ? OICA_BF16 : OICA_F32, xt32, L, W0 + w0_off, params, B, kurt,
                          iters, status, nullptr, &st);
    if (rc) return rc;
    w0_off += (size_t)L * n;
    // p = argmax of the criterion over the converged rows (lowest row on
    // ties) with eq. 3's test at step i: the first cluster of oica_unique on
    // the n-dimensional rows, whose rank-1 threshold is 2(n+1)n/T
    const oica_unique_params up{tau, gaussianity_test ? 1 : 0, 1};
    int nu = 0, na = 0;
    rc = oica_unique(ctx, n, T, L, B, kurt, status, &up, L, U, ku, uu, rep, csz, nullptr, &nu, &na);
    if (rc) return rc;
    int32_t p = -1;
    double a = NAN, u = NAN;
    if (nu > 0) {
      HIP_TRY(ctx, hipMemcpy(&p, rep, sizeof(int32_t), hipMemcpyDeviceToHost));
      HIP_TRY(ctx, hipMemcpy(&a, ku, sizeof(double), hipMemcpyDeviceToHost));
      HIP_TRY(ctx, hipMemcpy(&u, uu, sizeof(double), hipMemcpyDeviceToHost));
    }
    if (steps) {
      oica_deflation_step &s = steps[i - 1];
      s.dim = n;
      s.rep = p;
      s.accepted = na > 0;
      s.passes = st.passes;
      s.thread_iters = st.thread_iters;
      s.refine_thread_iters = st.refine_thread_iters;
      s.alpha = a;
      s.upsilon = u;
      s.threshold = 2.0 * (double)(n + 1) * (double)n / (double)T;
    }
    if (na == 0) break;
    HIP_TRY(ctx, launch_defl_append(ctx->stream, N, n_prev, G, B, rep, W_out));
    *n_found = i;
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return OICA_OK;
}

int oica_ordering_original(oica_ctx *ctx, int N, int64_t T, const float *Xw, int L,
                           const float *W0, const oica_fp_params *params, double tau,
                           int gaussianity_test, double *W_out, int *n_found,
                           oica_deflation_step *steps) {
  if (!ctx) return OICA_E_ARG;
  ctx->err.clear();
  int rc = check_dims(ctx, N, T);
  if (rc) return rc;
  if (L < 1 || L > (1 << 24)) return fail(ctx, OICA_E_ARG, "L must be in [1, 2^24] (got %d)", L);
  rc = check_fp_params(ctx, params);
  if (rc) return rc;
  if (params->precision != OICA_F32)
    return fail(ctx, OICA_E_UNSUPPORTED, "the original algorithm runs in FP32 (precision OICA_F32)");
  if (params->pruner) return fail(ctx, OICA_E_ARG, "the original algorithm runs without the pruner");
  if (params->traj_iters != 0) return fail(ctx, OICA_E_ARG, "traj_iters must be 0");
  if (!(tau > 0.0 && tau < 1.0)) return fail(ctx, OICA_E_ARG, "tau must be in (0, 1)");
  if (!Xw || !W0 || !W_out || !n_found) return fail(ctx, OICA_E_ARG, "Xw, W0, W_out and n_found must be non-null");
  *n_found = 0;
  size_t need = (size_t)L * N * 4 + 256;                   // rows of the runs
  need += (size_t)L * (8 + 4 + 1) + 3 * 256;               // kurt, iters, status
  need += (size_t)L * (N * 8 + 8 + 8 + 4 + 4) + 5 * 256;   // selection outputs (cap L)
  rc = ensure_buf(ctx, &ctx->ws2, &ctx->ws2_bytes, need);
  if (rc) return rc;
  Carve cv{(char *)ctx->ws2};
  float *B = cv.take<float>((size_t)L * N);
  double *kurt = cv.take<double>(L);
  int32_t *iters = cv.take<int32_t>(L);
  uint8_t *status = cv.take<uint8_t>(L);
  double *U = cv.take<double>((size_t)L * N);
  double *ku = cv.take<double>(L);
  double *uu = cv.take<double>(L);
  int32_t *rep = cv.take<int32_t>(L);
  int32_t *csz = cv.take<int32_t>(L);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  for (int i = 1; i <= N; ++i) {
    const int n_prev = i - 1;
    // L runs of Algorithm 1's FastICA from step i's starts, every start row and
    // update projected with E = W^T W of the n_prev components found so far
    oica_fp_stats st{};
    rc = fixed_point_impl(ctx, N, T, Xw, OICA_F32, Xw, L, W0 + (size_t)(i - 1) * L * N, params, B,
                          kurt, iters, status, nullptr, &st, n_prev ? W_out : nullptr, n_prev);
    if (rc) return rc;
    // p = argmax of the criterion over every run (lowest row on ties)
    HIP_TRY(ctx, launch_mark_runs(ctx->stream, L, status));
    const oica_unique_params up{tau, 0, 1};
    int nu = 0, na = 0;
    rc = oica_unique(ctx, N, T, L, B, kurt, status, &up, L, U, ku, uu, rep, csz, nullptr, &nu, &na);
    if (rc) return rc;
    int32_t p = -1;
    double a = NAN, u = NAN;
    if (nu > 0) {
      HIP_TRY(ctx, hipMemcpy(&p, rep, sizeof(int32_t), hipMemcpyDeviceToHost));
      HIP_TRY(ctx, hipMemcpy(&a, ku, sizeof(double), hipMemcpyDeviceToHost));
      HIP_TRY(ctx, hipMemcpy(&u, uu, sizeof(double), hipMemcpyDeviceToHost));
    }
    // eq. 3 at step i (the selection above ran without the test: its
    // threshold would use the full dimension)
    const double thr = 2.0 * (double)(N - i + 2) * (double)(N - i + 1) / (double)T;
    const bool ok = nu > 0 && (!gaussianity_test || u >= thr);
    if (steps) {
      oica_deflation_step &s = steps[i - 1];
      s.dim = N;
      s.rep = p;
      s.accepted = ok;
      s.passes = st.passes;
      s.thread_iters = st.thread_iters;
      s.refine_thread_iters = st.refine_thread_iters;
      s.alpha = a;
      s.upsilon = u;
      s.threshold = thr;
    }
    if (!ok) break;
    HIP_TRY(ctx, launch_append_row(ctx->stream, N, n_prev, B, rep, W_out));
    *n_found = i;
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return OICA_OK;
}

int oica_unique_batched(oica_ctx *ctx, int D, oica_unique_problem *problems,
                        const oica_unique_params *params) {
  if (!ctx) return OICA_E_ARG;
  ctx->err.clear();
  if (D < 1 || D > 1024) return fail(ctx, OICA_E_ARG, "D must be in [1, 1024]");
  if (!problems) return fail(ctx, OICA_E_ARG, "problems must be non-null");
  if (!params) return fail(ctx, OICA_E_ARG, "params must be non-null");
  if (!(params->tau > 0.0 && params->tau < 1.0)) return fail(ctx, OICA_E_ARG, "tau must be in (0, 1)");
  if (params->n_top < 0) return fail(ctx, OICA_E_ARG, "n_top must be >= 0");
  std::vector<oica::UJob> jobs(D);
  for (int d = 0; d < D; ++d) {
    oica_unique_problem &q = problems[d];
    q.n_unique = q.n_accepted = 0;
    int rc = check_dims(ctx, q.N, q.T);
    if (rc) {
      const std::string why = ctx->err;
      return fail(ctx, rc, "problem %d: %s", d, why.c_str());
    }
    if (q.K < 1) return fail(ctx, OICA_E_ARG, "problem %d: K must be >= 1", d);
    if (q.cap < 0) return fail(ctx, OICA_E_ARG, "problem %d: cap must be >= 0", d);
    if (!q.W || !q.kurt || !q.status)
      return fail(ctx, OICA_E_ARG, "problem %d: W, kurt and status must be non-null", d);
    if (q.cap > 0 && (!q.U || !q.kurt_u || !q.ups_u || !q.rep_thread || !q.cluster_size))
      return fail(ctx, OICA_E_ARG, "problem %d: output arrays must be non-null when cap > 0", d);
    oica::UJob &j = jobs[d];
    j = oica::UJob{};
    j.K = q.K;
    j.N = q.N;
    j.T = q.T;
    j.W = q.W;
    j.kurt = q.kurt;
    j.status = q.status;
    j.tau = params->tau;
    j.gtest = params->gaussianity_test;
    j.n_top = params->n_top;
    j.cap = q.cap;
    j.U = q.U;
    j.kurt_u = q.kurt_u;
    j.ups_u = q.ups_u;
    j.rep_thread = q.rep_thread;
    j.csize = q.cluster_size;
    j.row_cluster = q.row_cluster;
  }
  int rc = ensure_ws(ctx, unique_batched_workspace_bytes(D, jobs.data()));
  if (rc) return rc;
  std::vector<int> counts((size_t)D * 4);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, launch_unique_batched(ctx->stream, D, jobs.data(), ctx->ws, counts.data()));
  int first = OICA_OK;
  for (int d = 0; d < D; ++d) {
    problems[d].n_unique = counts[4 * d + 1];
    problems[d].n_accepted = counts[4 * d + 3];
    if (problems[d].cap < problems[d].n_unique && first == OICA_OK)
      first = fail(ctx, OICA_E_SHAPE, "problem %d: cap=%d is smaller than the %d clusters found", d,
                   problems[d].cap, problems[d].n_unique);
  }
  return first;
}

}  // extern "C"
