// C ABI of the library: argument checks, reach selection, work memory,
// kernel sequencing per scheme.  All compute happens in the kernels.

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>
#include <utility>
#include <algorithm>
#include <vector>

#include "../../include/sla.h"
#include "common.h"

struct sla_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  float* work = nullptr;  // ping-pong field
  size_t work_cap = 0;    // floats
  bool work_borrowed = false;  // work is the caller's (sla_set_workspace): never allocate
  float* fpart = nullptr; // velocity-max partials (3 * kUmaxBlocks) + 3 results
  double* dpart = nullptr;// norm partials (5 * kNormBlocks) + 5 results
  int* flag = nullptr;    // set by a kernel that clamped an offset
  void* host = nullptr;   // pinned staging for small results (256 bytes)
  float* scratch = nullptr;  // this device's static work field (sla_advect_noalloc)
  std::string err;
  bool fused = true;    // SLA_OPT_FUSED
  int cec3d_kernel = 5;  // SLA_OPT_CEC3D_KERNEL
  int sweep_kernel = 3;  // SLA_OPT_SWEEP_KERNEL
  int ec_kernel = 3;     // SLA_OPT_EC_KERNEL
  int cec3d_shape = 0;   // SLA_OPT_CEC3D_SHAPE
  int ec_shape = 0;      // SLA_OPT_EC_SHAPE
  int backtrace = 0;     // SLA_OPT_BACKTRACE
  // fused-step choices measured by sla_tune (or loaded), per grid
  struct Tuned {
    int n[3];
    int variant[2], shape[2];  // [0] even steps, [1] odd
    double ms[2];
  };
  std::vector<Tuned> tuned;
  int learned_kernel = 1;  // SLA_OPT_LEARNED_KERNEL
  int multi = 4;           // SLA_OPT_SHARED_VELOCITY: largest group of fields
  // per-kernel timing
  bool timing = false;
  struct Mark { int kind; hipEvent_t a, b; };
  std::vector<Mark> marks;        // recorded, not yet read
  std::vector<hipEvent_t> spare;  // event pool
  int64_t launches[SLA_K_COUNT] = {};
  double ms[SLA_K_COUNT] = {};
};

struct sla_plan {
  int device = 0;
  int nprob = 0;
  int32_t steps = 0;
  int64_t step0 = 0;
  std::vector<float*> work;          // one work field per problem
  std::vector<float*> phis;          // caller's fields
  std::vector<size_t> cells;         // cells per problem
  float* uniform = nullptr;          // device: 3 floats per uniform problem
  sla::BatchProblem* dprobs = nullptr;
  int4* ditems = nullptr;
  int nitems = 0, ychunk = 0, blocks = 0;
  double step_ms = 0.0;
  // problems run by their own launches of the fused step (see plan_direct)
  std::vector<int> direct;
  // the direct problems in launch groups: problems with the same velocity,
  // grid and time step run together (up to four) through the
  // shared-velocity fused step
  std::vector<std::vector<int>> groups;
  std::vector<sla::Geo> geo;         // per problem
  std::vector<const float*> u;       // per problem (NULL: uniform velocity)
  int cec3d_kernel = 5;              // the creating context's fused-step choice
  hipStream_t cap = nullptr;         // private capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int* flag = nullptr;               // the creating context's overflow record
};

struct sla_model {
  int device = 0;
  float* master = nullptr;  // FP32 weights
  float* mo = nullptr;      // Adam first moment
  float* vo = nullptr;      // Adam second moment
  float* wr = nullptr;      // BF16-rounded weights as FP32
  void* wpack = nullptr;    // BF16 matrix-core operand layouts
  float* grad = nullptr;
  float* gpart = nullptr;   // per-block gradient partials
  float* lpart = nullptr;   // per-block squared errors
  double* loss = nullptr;   // device loss sum
  int64_t adam_t = 0;
  double range = 0.0;       // trained Courant range (0: untrained)
};

namespace {

int fail(sla_ctx* ctx, int code, const char* fmt, ...) {
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

int hip_fail(sla_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, SLA_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Makes the context's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int check_grid(sla_ctx* ctx, const sla_grid* g) {
  if (!g) return fail(ctx, SLA_EINVAL, "grid is NULL");
  if (g->ndim < 1 || g->ndim > 3) return fail(ctx, SLA_EINVAL, "ndim must be 1, 2 or 3 (got %d)", g->ndim);
  int64_t cells = 1;
  for (int d = 0; d < 3; ++d) {
    if (d < g->ndim) {
      if (g->n[d] < 8) return fail(ctx, SLA_EINVAL, "n[%d] = %d: need at least 8 cells", d, g->n[d]);
      if (!(g->dx[d] > 0.0) || !std::isfinite(g->dx[d]))
        return fail(ctx, SLA_EINVAL, "dx[%d] must be positive and finite", d);
    } else if (g->n[d] != 1) {
      return fail(ctx, SLA_EINVAL, "n[%d] must be 1 on an unused axis", d);
    }
    // each extent is below 2^31 and the running product stays below 2^31,
    // so the product cannot overflow before it is checked
    cells *= g->n[d];
    if (cells >= (int64_t(1) << 31)) return fail(ctx, SLA_EINVAL, "grid has 2^31 cells or more");
  }
  return SLA_OK;
}

sla::Geo make_geo(const sla_grid* g, double dt) {
  sla::Geo geo;
  geo.nx = g->n[0];
  geo.ny = g->n[1];
  geo.nz = g->n[2];
  geo.ncells = g->n[0] * g->n[1] * g->n[2];
  for (int d = 0; d < 3; ++d) geo.lam[d] = d < g->ndim ? float(dt / g->dx[d]) : 0.f;
  return geo;
}

// Per-axis max |c_d| measured on the device (synchronises).
int measure_courant(sla_ctx* ctx, const sla_grid* g, const sla::Geo& geo, const float* u,
                    float cmax[3]) {
  float* res = ctx->fpart + 3 * sla::kUmaxBlocks;
  hipError_t e = sla::launch_umax(g->ndim, geo.ncells, u, ctx->fpart, res, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "velocity max launch");
  float* h = static_cast<float*>(ctx->host);
  e = hipMemcpyAsync(h, res, 3 * sizeof(float), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "velocity max");
  for (int d = 0; d < 3; ++d) {
    if (d >= g->ndim) {
      cmax[d] = 0.f;
      continue;
    }
    if (!std::isfinite(h[d])) return fail(ctx, SLA_EINVAL, "velocity plane %d holds NaN or Inf", d);
    cmax[d] = h[d] * std::fabs(geo.lam[d]);  // FP32 product, as the kernels form c
  }
  return SLA_OK;
}

hipEvent_t take_event(sla_ctx* ctx) {
  if (!ctx->spare.empty()) {
    hipEvent_t e = ctx->spare.back();
    ctx->spare.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run one kernel launch; bracket it with events when timing is on.
template <typename F>
hipError_t run(sla_ctx* ctx, int kind, F&& launch) {
  if (!ctx->timing) return launch();
  hipEvent_t a = take_event(ctx), b = take_event(ctx);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, ctx->stream);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
  if (e != hipSuccess) {
    ctx->spare.push_back(a);
    ctx->spare.push_back(b);
    return e;
  }
  ctx->marks.push_back({kind, a, b});
  return hipSuccess;
}

// Fold recorded marks into the totals (the stream must be synchronised).
void fold_marks(sla_ctx* ctx) {
  for (auto& m : ctx->marks) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, m.a, m.b) == hipSuccess) {
      ctx->launches[m.kind] += 1;
      ctx->ms[m.kind] += t;
    }
    ctx->spare.push_back(m.a);
    ctx->spare.push_back(m.b);
  }
  ctx->marks.clear();
}

// True while the context's stream is being captured into a graph: a call
// must then neither synchronise nor allocate.
bool capturing(sla_ctx* ctx) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(ctx->stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// The tuned fused-step choice of a grid, if any.
const sla_ctx::Tuned* find_tuned(const sla_ctx* ctx, const sla::Geo& g) {
  for (const auto& t : ctx->tuned)
    if (t.n[0] == g.nx && t.n[1] == g.ny && t.n[2] == g.nz) return &t;
  return nullptr;
}
void put_tuned(sla_ctx* ctx, const sla_ctx::Tuned& e) {
  for (auto& t : ctx->tuned)
    if (t.n[0] == e.n[0] && t.n[1] == e.n[1] && t.n[2] == e.n[2]) {
      t = e;
      return;
    }
  ctx->tuned.push_back(e);
}

int ensure_work(sla_ctx* ctx, size_t floats) {
  if (ctx->work_cap >= floats) return SLA_OK;
  if (capturing(ctx))
    return fail(ctx, SLA_ECAPTURE, "work memory would be allocated while the stream is captured: "
                "run the call once before capturing, or set a workspace");
  if (ctx->work_borrowed)
    return fail(ctx, SLA_EINVAL, "the workspace holds %zu bytes, the call needs %zu",
                ctx->work_cap * sizeof(float), floats * sizeof(float));
  if (ctx->work) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "synchronise before growing work memory");
    (void)hipFree(ctx->work);
    ctx->work = nullptr;
    ctx->work_cap = 0;
  }
  if (hipMalloc(&ctx->work, floats * sizeof(float)) != hipSuccess) {
    ctx->work = nullptr;
    (void)hipGetLastError();
    return fail(ctx, SLA_ENOMEM, "cannot allocate %zu bytes of work memory", floats * sizeof(float));
  }
  ctx->work_cap = floats;
  return SLA_OK;
}

// Work memory of sla_advect_noalloc: one field of at most
// SLA_NOALLOC_MAX_CELLS cells per device, held from the library's load to the
// end of the process.  Host code must not use the array's name as an
// address: each device's copy is reached through the pointer that
// hipGetSymbolAddress returned on that device (scratch_on).
static __device__ __align__(256) float scratch[SLA_NOALLOC_MAX_CELLS];

constexpr int kScratchDevices = 64;
std::mutex scratch_mu;
float* scratch_dev[kScratchDevices] = {};

// The device address of `scratch` on `device` (which must be current),
// looked up once per device.
hipError_t scratch_on(int device, float** out) {
  *out = nullptr;
  if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_dev[device] = static_cast<float*>(p);
  }
  *out = scratch_dev[device];
  return hipSuccess;
}

}  // namespace

extern "C" {

const char* sla_strerror(int status) {
  switch (status) {
    case SLA_OK: return "success";
    case SLA_EINVAL: return "invalid argument";
    case SLA_ECOURANT: return "Courant number beyond the supported reach";
    case SLA_EHIP: return "HIP runtime error";
    case SLA_ENOMEM: return "out of device memory";
    case SLA_ENOMODEL: return "no usable model weights";
    case SLA_ECAPTURE: return "not allowed while the stream is captured into a graph";
  }
  return "unknown status";
}

const char* sla_last_error(const sla_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

int sla_create(sla_ctx** out, int device, void* stream) {
  if (!out) return SLA_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return SLA_EINVAL;
  }
  sla_ctx* ctx = new sla_ctx;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(stream);
  DeviceGuard guard(device);
  bool ok = guard.ok;
  ok = ok && hipMalloc(&ctx->fpart, (3 * sla::kUmaxBlocks + 3) * sizeof(float)) == hipSuccess;
  ok = ok && hipMalloc(&ctx->dpart, (5 * sla::kNormBlocks + 5) * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(&ctx->flag, sizeof(int)) == hipSuccess;
  ok = ok && hipHostMalloc(&ctx->host, 256, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipMemset(ctx->flag, 0, sizeof(int)) == hipSuccess;
  // the static work field of sla_advect_noalloc (that call fails without it)
  if (ok && scratch_on(device, &ctx->scratch) != hipSuccess) (void)hipGetLastError();
  if (!ok) {
    (void)hipGetLastError();
    sla_destroy(ctx);
    return SLA_ENOMEM;
  }
  *out = ctx;
  return SLA_OK;
}

void sla_destroy(sla_ctx* ctx) {
  if (!ctx) return;
  {
    DeviceGuard guard(ctx->device);
    if (ctx->stream || ctx->work) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->work && !ctx->work_borrowed) (void)hipFree(ctx->work);
    if (ctx->fpart) (void)hipFree(ctx->fpart);
    if (ctx->dpart) (void)hipFree(ctx->dpart);
    if (ctx->flag) (void)hipFree(ctx->flag);
    if (ctx->host) (void)hipHostFree(ctx->host);
    for (auto& m : ctx->marks) {
      (void)hipEventDestroy(m.a);
      (void)hipEventDestroy(m.b);
    }
    for (auto e : ctx->spare) (void)hipEventDestroy(e);
  }
  delete ctx;
}

int sla_set_stream(sla_ctx* ctx, void* stream) {
  if (!ctx) return SLA_EINVAL;
  ctx->stream = static_cast<hipStream_t>(stream);
  return SLA_OK;
}

int sla_courant_max(sla_ctx* ctx, const sla_grid* grid, const float* u, double dt, double* out) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (capturing(ctx)) return fail(ctx, SLA_ECAPTURE, "this call synchronises the stream");
  int rc = check_grid(ctx, grid);
  if (rc) return rc;
  if (!u || !out) return fail(ctx, SLA_EINVAL, "u and out must not be NULL");
  if (!std::isfinite(dt)) return fail(ctx, SLA_EINVAL, "dt must be finite");
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(ctx, SLA_EHIP, "cannot select device %d", ctx->device);
  const sla::Geo geo = make_geo(grid, dt);
  float cm[3];
  rc = measure_courant(ctx, grid, geo, u, cm);
  if (rc) return rc;
  *out = std::fmax(cm[0], std::fmax(cm[1], cm[2]));
  return SLA_OK;
}

}  // extern "C"

namespace {

// Arguments of sla_advect (and of each scalar or problem of the multi and
// batch calls) other than the Courant bound.
int check_advect(sla_ctx* ctx, const sla_grid* grid, const float* phi, const float* u, double dt,
                 int32_t scheme, int32_t steps, double courant_max) {
  int rc = check_grid(ctx, grid);
  if (rc) return rc;
  if (!phi || !u) return fail(ctx, SLA_EINVAL, "phi and u must not be NULL");
  if (!std::isfinite(dt)) return fail(ctx, SLA_EINVAL, "dt must be finite");
  if (scheme < SLA_CIR || scheme > SLA_CEC_LITERAL)
    return fail(ctx, SLA_EINVAL, "unknown scheme %d", scheme);
  if (steps < 0) return fail(ctx, SLA_EINVAL, "steps must be >= 0");
  if (std::isnan(courant_max)) return fail(ctx, SLA_EINVAL, "courant_max is NaN");
  return SLA_OK;
}

// Reach per axis: from the caller's bound on every axis, else measured.
int advect_reach(sla_ctx* ctx, const sla_grid* grid, const sla::Geo& geo, const float* u,
                 double courant_max, int reach[3]) {
  reach[0] = reach[1] = reach[2] = 1;
  if (courant_max > 0.0) {
    if (!(courant_max < SLA_MAX_REACH))
      return fail(ctx, SLA_ECOURANT, "courant_max %g: must be below %d", courant_max, SLA_MAX_REACH);
    const int r = int(std::floor(courant_max)) + 1;
    reach[0] = reach[1] = reach[2] = r;
    return SLA_OK;
  }
  if (capturing(ctx))
    return fail(ctx, SLA_ECAPTURE, "measuring the Courant bound synchronises the stream: "
                "pass courant_max > 0 while capturing");
  float cm[3];
  const int rc = measure_courant(ctx, grid, geo, u, cm);
  if (rc) return rc;
  for (int d = 0; d < grid->ndim; ++d) {
    if (!(cm[d] < float(SLA_MAX_REACH)))
      return fail(ctx, SLA_ECOURANT, "max Courant number %g on axis %d: must be below %d",
                  double(cm[d]), d, SLA_MAX_REACH);
    reach[d] = int(std::floor(cm[d])) + 1;
  }
  return SLA_OK;
}

// work: the ping-pong field to use, or NULL for the context's work memory
// (allocated on first use).
int advect_steps(sla_ctx* ctx, const sla_grid* grid, float* phi, const float* u, double dt,
                 int32_t scheme, int32_t steps, int64_t step0, const int reach[3],
                 float* work = nullptr);

}  // namespace

extern "C" {

int sla_advect(sla_ctx* ctx, const sla_grid* grid, float* phi, const float* u, double dt,
               int32_t scheme, int32_t steps, int64_t step0, double courant_max) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  int rc = check_advect(ctx, grid, phi, u, dt, scheme, steps, courant_max);
  if (rc) return rc;
  if (steps == 0) return SLA_OK;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(ctx, SLA_EHIP, "cannot select device %d", ctx->device);
  int reach[3];
  rc = advect_reach(ctx, grid, make_geo(grid, dt), u, courant_max, reach);
  if (rc) return rc;
  return advect_steps(ctx, grid, phi, u, dt, scheme, steps, step0, reach);
}

int sla_advect_noalloc(sla_ctx* ctx, const sla_grid* grid, float* phi, const float* u, double dt,
                       int32_t scheme, int32_t steps, int64_t step0, double courant_max) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  int rc = check_advect(ctx, grid, phi, u, dt, scheme, steps, courant_max);
  if (rc) return rc;
  const int64_t cells = int64_t(grid->n[0]) * grid->n[1] * grid->n[2];
  if (cells > SLA_NOALLOC_MAX_CELLS)
    return fail(ctx, SLA_EINVAL, "grid of %lld cells: sla_advect_noalloc takes at most %d",
                (long long)cells, SLA_NOALLOC_MAX_CELLS);
  if (!ctx->scratch) return fail(ctx, SLA_EHIP, "no static work memory on device %d", ctx->device);
  if (steps == 0) return SLA_OK;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(ctx, SLA_EHIP, "cannot select device %d", ctx->device);
  int reach[3];
  rc = advect_reach(ctx, grid, make_geo(grid, dt), u, courant_max, reach);
  if (rc) return rc;
  // per-launch timing would create events: this call's launches are not timed
  const bool timing = ctx->timing;
  ctx->timing = false;
  rc = advect_steps(ctx, grid, phi, u, dt, scheme, steps, step0, reach, ctx->scratch);
  ctx->timing = timing;
  return rc;
}

size_t sla_workspace_size(const sla_grid* grid, int32_t scheme, int32_t nscalars) {
  // the grid rules of sla_advect (check_grid records no message without a context)
  if (check_grid(nullptr, grid) != SLA_OK || scheme < SLA_CIR || scheme > SLA_CEC_LITERAL ||
      nscalars < 0)
    return 0;
  size_t cells = 1;
  for (int d = 0; d < 3; ++d) cells *= size_t(grid->n[d]);
  // one ping-pong field; third-order 3D runs of several fields take one per
  // field, up to four (the fields sharing a velocity run four at a time)
  size_t fields = 1;
  if (scheme == SLA_CEC && grid->ndim == 3) fields = size_t(std::min(std::max(nscalars, 1), 4));
  return fields * cells * sizeof(float);
}

int sla_set_workspace(sla_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (capturing(ctx)) return fail(ctx, SLA_ECAPTURE, "this call synchronises the stream");
  if (dev_ptr && bytes < sizeof(float)) return fail(ctx, SLA_EINVAL, "workspace of %zu bytes", bytes);
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(ctx, SLA_EHIP, "cannot select device %d", ctx->device);
  const hipError_t e = hipStreamSynchronize(ctx->stream);  // earlier calls may still use it
  if (e != hipSuccess) return hip_fail(ctx, e, "synchronise before changing the workspace");
  if (ctx->work && !ctx->work_borrowed) (void)hipFree(ctx->work);
  ctx->work = static_cast<float*>(dev_ptr);
  ctx->work_cap = dev_ptr ? bytes / sizeof(float) : 0;
  ctx->work_borrowed = dev_ptr != nullptr;
  return SLA_OK;
}

int sla_advect_multi(sla_ctx* ctx, const sla_grid* grid, int32_t nscalars, float* const* phis,
                     const float* u, double dt, int32_t scheme, int32_t steps, int64_t step0,
                     double courant_max) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (nscalars < 0 || (nscalars > 0 && !phis))
    return fail(ctx, SLA_EINVAL, "need nscalars >= 0 and the array of fields");
  for (int32_t k = 0; k < nscalars; ++k)
    if (!phis[k]) return fail(ctx, SLA_EINVAL, "field %d is NULL", k);
  int rc = check_advect(ctx, grid, nscalars > 0 ? phis[0] : u, u, dt, scheme, steps, courant_max);
  if (rc) return rc;
  if (steps == 0 || nscalars == 0) return SLA_OK;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(ctx, SLA_EHIP, "cannot select device %d", ctx->device);
  int reach[3];  // one Courant bound for all the fields
  const sla::Geo geo = make_geo(grid, dt);
  rc = advect_reach(ctx, grid, geo, u, courant_max, reach);
  if (rc) return rc;
  // third order in 3D at reach 1: the fields run up to four at a time
  // through the shared-velocity fused step, each with its own work field
  const bool shared = scheme == SLA_CEC && grid->ndim == 3 && ctx->fused && ctx->multi > 1 &&
                      ctx->backtrace == 0 &&
                      reach[0] == 1 && reach[1] == 1 && reach[2] == 1 && nscalars >= 2 &&
                      sla::offsets32_ok(geo);
  if (!shared) {
    for (int32_t k = 0; k < nscalars && rc == SLA_OK; ++k)
      rc = advect_steps(ctx, grid, phis[k], u, dt, scheme, steps, step0, reach);
    return rc;
  }
  const size_t n = size_t(geo.ncells);
  size_t kmax = size_t(std::min<int32_t>(nscalars, ctx->multi));
  if (ctx->work_borrowed) {
    kmax = std::min(kmax, ctx->work_cap / n);  // what the caller's workspace holds
    if (kmax == 0) return ensure_work(ctx, n);  // reports the size it needs
  } else {
    rc = ensure_work(ctx, kmax * n);
    if (rc) return rc;
  }
  hipError_t e = hipSuccess;
  for (int32_t f0 = 0; f0 < nscalars && e == hipSuccess;) {
    const int left = nscalars - f0;
    const int k = (left >= 4 && kmax >= 4) ? 4 : (left >= 2 && kmax >= 2) ? 2 : 1;
    float* cur[4];
    float* nxt[4];
    for (int f = 0; f < k; ++f) {
      cur[f] = phis[f0 + f];
      nxt[f] = ctx->work + size_t(f) * n;
    }
    for (int32_t s = 0; s < steps && e == hipSuccess; ++s) {
      const bool even = (step0 + s) % 2 == 0;
      e = run(ctx, SLA_K_CEC3D, [&] {
        return sla::launch_cec3d_multi(k, even, geo, cur, nxt, u, ctx->flag, ctx->stream);
      });
      for (int f = 0; f < k; ++f) std::swap(cur[f], nxt[f]);
    }
    for (int f = 0; f < k && e == hipSuccess; ++f)
      if (cur[f] != phis[f0 + f])
        e = run(ctx, SLA_K_COPY, [&] {
          return hipMemcpyAsync(phis[f0 + f], cur[f], n * sizeof(float), hipMemcpyDeviceToDevice,
                                ctx->stream);
        });
    f0 += k;
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "shared-velocity step launch");
  return SLA_OK;
}

}  // extern "C"

namespace {

__global__ __launch_bounds__(256) void k_fill_velocity(float* __restrict__ u, size_t n, int ndim,
                                                       float ux, float uy, float uz) {
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += size_t(gridDim.x) * 256) {
    u[i] = ux;
    if (ndim > 1) u[n + i] = uy;
    if (ndim > 2) u[2 * n + i] = uz;
  }
}

}  // namespace

extern "C" {

int sla_advect_batch(sla_ctx* ctx, int32_t nprob, const sla_problem* probs, int32_t scheme,
                     int32_t steps, int64_t step0, double courant_max) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (nprob < 0 || (nprob > 0 && !probs)) return fail(ctx, SLA_EINVAL, "need nprob >= 0 and probs");
  if (capturing(ctx)) return fail(ctx, SLA_ECAPTURE, "batches synchronise the stream");
  bool all3d = true;
  for (int32_t i = 0; i < nprob; ++i) {
    const sla_problem& p = probs[i];
    const float* any_u = p.u ? p.u : p.u_uniform;  // a uniform problem passes the pointer check
    int rc = check_advect(ctx, &p.grid, p.phi, any_u, p.dt, scheme, steps, courant_max);
    if (rc) return rc;
    if (!p.u)
      for (int d = 0; d < p.grid.ndim; ++d)
        if (!std::isfinite(p.u_uniform[d]))
          return fail(ctx, SLA_EINVAL, "problem %d: non-finite uniform velocity", i);
    all3d = all3d && p.grid.ndim == 3;
  }
  if (steps == 0 || nprob == 0) return SLA_OK;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(ctx, SLA_EHIP, "cannot select device %d", ctx->device);
  if (scheme == SLA_CEC && all3d && ctx->backtrace == 0) {
    // every Courant number below 1: one plan (a graph of all steps), run once
    sla_plan* plan = nullptr;
    int rc = sla_plan_create(ctx, &plan, nprob, probs, steps, step0, courant_max, 0);
    if (rc == SLA_OK) {
      rc = sla_plan_run(ctx, plan);
      const hipError_t e = hipStreamSynchronize(ctx->stream);  // before the plan's memory goes
      sla_plan_destroy(plan);
      if (rc == SLA_OK && e != hipSuccess) rc = hip_fail(ctx, e, "batched run");
      return rc;
    }
    if (rc != SLA_ECOURANT) return rc;
    ctx->err.clear();  // larger Courant numbers: problem by problem
  }
  // problem by problem; a uniform velocity is written into a temporary field
  float* tmp = nullptr;
  size_t tmp_cap = 0;
  int rc = SLA_OK;
  for (int32_t i = 0; i < nprob && rc == SLA_OK; ++i) {
    const sla_problem& p = probs[i];
    const float* u = p.u;
    if (!u) {
      const size_t n = size_t(p.grid.n[0]) * p.grid.n[1] * p.grid.n[2];
      const size_t need = size_t(p.grid.ndim) * n;
      if (need > tmp_cap) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess && tmp) e = hipFree(tmp);
        tmp = nullptr;
        tmp_cap = 0;
        if (e == hipSuccess) e = hipMalloc(&tmp, need * sizeof(float));
        if (e != hipSuccess) {
          tmp = nullptr;
          rc = hip_fail(ctx, e, "temporary velocity field");
          break;
        }
        tmp_cap = need;
      }
      hipLaunchKernelGGL(k_fill_velocity, dim3(1024), dim3(256), 0, ctx->stream, tmp, n, p.grid.ndim,
                         p.u_uniform[0], p.u_uniform[1], p.u_uniform[2]);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) {
        rc = hip_fail(ctx, e, "velocity fill");
        break;
      }
      u = tmp;
    }
    int reach[3];
    rc = advect_reach(ctx, &p.grid, make_geo(&p.grid, p.dt), u, courant_max, reach);
    if (rc == SLA_OK) rc = advect_steps(ctx, &p.grid, p.phi, u, p.dt, scheme, steps, step0, reach);
  }
  if (tmp) {
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(tmp);
    if (rc == SLA_OK && e != hipSuccess) rc = hip_fail(ctx, e, "batched run");
  }
  return rc;
}

int sla_model_load(sla_ctx* ctx, sla_model* model, const float* params, int64_t n) {
  return sla_model_set_params(ctx, model, params, n);
}

int sla_model_save(sla_ctx* ctx, const sla_model* model, float* params, int64_t n) {
  return sla_model_get_params(ctx, model, params, n);
}

}  // extern "C"

namespace {

// True if the x and y sweeps of a third-order step at reach rxy (the larger
// of the two axes') run in the kernel with two nodes per lane:
// SLA_OPT_SWEEP_KERNEL 3, an even nx and a reach of at most 3.
bool xy_pairs(const sla_ctx* ctx, const sla::Geo& g, int rxy) {
  return ctx->sweep_kernel == 3 && g.nx % 2 == 0 && rxy <= 3;
}

// The steps of sla_advect once the arguments are checked and the reach per
// axis is known (the device is selected).
int advect_steps(sla_ctx* ctx, const sla_grid* grid, float* phi, const float* u, double dt,
                 int32_t scheme, int32_t steps, int64_t step0, const int reach[3], float* work) {
  const sla::Geo geo = make_geo(grid, dt);
  const int ndim = grid->ndim;
  int rmax = 1;
  for (int d = 0; d < ndim; ++d) rmax = reach[d] > rmax ? reach[d] : rmax;

  const size_t n = size_t(geo.ncells);
  if (!work) {
    const int rc = ensure_work(ctx, n);
    if (rc) return rc;
    work = ctx->work;
  }

  // A 3D third-order step whose reach is 1 on every axis runs as one fused
  // kernel (20 B/cell); other cases run one sweep kernel per axis.  The
  // fused kernels address a field with 32-bit byte offsets: up to 2^30 cells.
  const bool fused3d = ctx->fused && ndim == 3 && rmax == 1 && sla::offsets32_ok(geo);
  float* cur = phi;
  float* nxt = work;
  hipError_t e = hipSuccess;
  for (int32_t k = 0; k < steps && e == hipSuccess; ++k) {
    const int64_t m = step0 + k;
    switch (scheme) {
      case SLA_CIR:
        e = run(ctx, SLA_K_CIR, [&] {
          return sla::launch_cir(ndim, geo, cur, u, nxt, ctx->flag, ctx->stream);
        });
        std::swap(cur, nxt);
        break;
      case SLA_FEC:
      case SLA_BEC: {
        const int kind = scheme == SLA_FEC ? SLA_K_FEC : SLA_K_BEC;
        // default (3): at reach 1 on a 3D grid all calls of the step in one
        // z-march (every stage in LDS); otherwise the gather chain, faster
        // than the LDS-tile kernel at every grid and Courant number measured
        // (256^3 and 512^3, CFL 0.9 to 2.5)
        if (ctx->ec_kernel == 3 && ndim == 3 && rmax == 1 && sla::offsets32_ok(geo)) {
          e = run(ctx, kind, [&] {
            return sla::launch_ec_march(scheme, geo, cur, u, nxt, ctx->flag, ctx->stream, ctx->ec_shape);
          });
          std::swap(cur, nxt);
          break;
        }
        if (ctx->ec_kernel == 0) {
          e = run(ctx, kind, [&] {
            return sla::launch_ec(ndim, scheme, rmax, geo, cur, u, nxt, ctx->flag, ctx->stream);
          });
          std::swap(cur, nxt);
          break;
        }
        // one gather kernel per call: Phi1 = L_U Phi into the work field, then
        // FEC's result (or BEC's psi) in place of Phi, then BEC's L_U psi
        e = run(ctx, kind, [&] {
          return sla::launch_cir(ndim, geo, cur, u, nxt, ctx->flag, ctx->stream);
        });
        if (e == hipSuccess)
          e = run(ctx, kind, [&] {
            return sla::launch_ec_gather(ndim, scheme == SLA_FEC ? 1 : 2, geo, nxt, cur, u, cur,
                                         ctx->flag, ctx->stream);
          });
        if (scheme == SLA_BEC && e == hipSuccess) {
          e = run(ctx, kind, [&] {
            return sla::launch_cir(ndim, geo, cur, u, nxt, ctx->flag, ctx->stream);
          });
          std::swap(cur, nxt);
        }
        break;
      }
      case SLA_CEC: {
        if (ctx->backtrace == 1) {  // midpoint backtrace: tile sweeps, the alternating order
          for (int j = 0; j < ndim && e == hipSuccess; ++j) {
            const int d = (m % 2 == 0) ? j : ndim - 1 - j;
            e = run(ctx, SLA_K_SWEEP_X + d, [&] {
              return sla::launch_cec_sweep_mid(d, reach[d], geo, cur, u + size_t(d) * n, nxt,
                                               ctx->flag, ctx->stream);
            });
            std::swap(cur, nxt);
          }
          break;
        }
        if (fused3d) {
          e = run(ctx, SLA_K_CEC3D, [&] {
            sla::Cec3dLaunch lc;
            lc.ychunk = ctx->cec3d_shape;
            int variant = ctx->cec3d_kernel;
            if (variant == 5) {
              const sla_ctx::Tuned* t = find_tuned(ctx, geo);
              if (t) {
                variant = t->variant[m % 2];
                lc.ychunk = t->shape[m % 2];
              }
            }
            return sla::launch_cec3d(variant, m % 2 == 0, geo, cur, u, nxt, ctx->flag,
                                     ctx->stream, lc);
          });
          std::swap(cur, nxt);
          break;
        }
        const int rxy = reach[0] > reach[1] ? reach[0] : reach[1];
        const bool pairs = xy_pairs(ctx, geo, rxy);
        if (ndim >= 2 && (pairs || (ctx->sweep_kernel >= 2 && rxy <= 2)) &&
            sla::offsets32_ok(geo)) {
          // x and y in one kernel: x,y then z on even steps, z then y,x on
          // odd.  With one node per lane up to reach 2: a 64-lane window
          // then yields 52 or more outputs; at reach 3 (46) the y sweep's
          // work on the halo lanes outweighs the saved traffic, and the
          // sweeps run one per axis.  Two nodes per lane: 108 at reach 3.
          const bool even = m % 2 == 0;
          for (int part = 0; part < 2 && e == hipSuccess; ++part) {
            const bool xy = (part == 0) == even;
            if (xy) {
              e = run(ctx, SLA_K_SWEEP_XY, [&] {
                return sla::launch_cec_sweep_xy(rxy, even, geo, cur, u, nxt, ctx->flag, ctx->stream,
                                                pairs);
              });
            } else {
              if (ndim < 3) continue;
              e = run(ctx, SLA_K_SWEEP_Z, [&] {
                return sla::launch_cec_sweep(2, reach[2], geo, cur, u + 2 * n, nxt, ctx->flag,
                                             ctx->stream, true);
              });
            }
            std::swap(cur, nxt);
          }
          break;
        }
        for (int j = 0; j < ndim && e == hipSuccess; ++j) {
          const int d = (m % 2 == 0) ? j : ndim - 1 - j;
          e = run(ctx, SLA_K_SWEEP_X + d, [&] {
            return sla::launch_cec_sweep(d, reach[d], geo, cur, u + size_t(d) * n, nxt,
                                         ctx->flag, ctx->stream, ctx->sweep_kernel != 0);
          });
          std::swap(cur, nxt);
        }
        break;
      }
      case SLA_FEC_SPLIT:
      case SLA_BEC_SPLIT:
      case SLA_CEC_LITERAL: {
        // one 1D FEC, BEC or literal-weight sweep per axis, x,y,z on even
        // steps, z,y,x on odd, by the kernels of the third order's sweeps
        // (x and y in one kernel where SLA_CEC runs them so)
        const int one = scheme == SLA_FEC_SPLIT ? sla::FEC
                        : scheme == SLA_BEC_SPLIT ? sla::BEC
                                                  : sla::CEC_LITERAL;
        const int rxy = reach[0] > reach[1] ? reach[0] : reach[1];
        const bool pairs = xy_pairs(ctx, geo, rxy);
        if (ndim >= 2 && (pairs || (ctx->sweep_kernel >= 2 && rxy <= 2)) &&
            sla::offsets32_ok(geo)) {
          const bool even = m % 2 == 0;
          for (int part = 0; part < 2 && e == hipSuccess; ++part) {
            const bool xy = (part == 0) == even;
            if (xy) {
              e = run(ctx, SLA_K_SWEEP_XY, [&] {
                return sla::launch_cec_sweep_xy(rxy, even, geo, cur, u, nxt, ctx->flag, ctx->stream,
                                                pairs, one);
              });
            } else {
              if (ndim < 3) continue;
              e = run(ctx, SLA_K_SWEEP_Z, [&] {
                return sla::launch_ec_sweep(one, 2, reach[2], geo, cur, u + 2 * n, nxt, ctx->flag,
                                            ctx->stream, true);
              });
            }
            std::swap(cur, nxt);
          }
          break;
        }
        for (int j = 0; j < ndim && e == hipSuccess; ++j) {
          const int d = (m % 2 == 0) ? j : ndim - 1 - j;
          e = run(ctx, SLA_K_SWEEP_X + d, [&] {
            return sla::launch_ec_sweep(one, d, reach[d], geo, cur, u + size_t(d) * n, nxt,
                                        ctx->flag, ctx->stream, ctx->sweep_kernel != 0);
          });
          std::swap(cur, nxt);
        }
        break;
      }
      case SLA_CEC_STRANG: {
        // half steps: lambda = fl32(dt/2/dx) = fl32(dt/dx)/2 exactly, so
        // every half-step Courant number is half the whole step's; their
        // reach is floor(max|c|/2) + 1 <= (reach - 1)/2 + 1
        const sla::Geo half = make_geo(grid, 0.5 * dt);
        int rh[3];
        for (int d = 0; d < 3; ++d) rh[d] = (reach[d] - 1) / 2 + 1;
        auto sweep = [&](int d, bool whole) {
          if (e != hipSuccess) return;
          e = run(ctx, SLA_K_SWEEP_X + d, [&] {
            return sla::launch_cec_sweep(d, whole ? reach[d] : rh[d], whole ? geo : half, cur,
                                         u + size_t(d) * n, nxt, ctx->flag, ctx->stream,
                                         ctx->sweep_kernel != 0);
          });
          std::swap(cur, nxt);
        };
        const int rxy = rh[0] > rh[1] ? rh[0] : rh[1];
        const bool pairs = xy_pairs(ctx, geo, rxy);
        if (ndim == 3 && (pairs || (ctx->sweep_kernel >= 2 && rxy <= 2)) && sla::offsets32_ok(geo)) {
          // x/2 then y/2 in one kernel, z, then y/2 then x/2 in one kernel
          for (int part = 0; part < 3 && e == hipSuccess; ++part) {
            if (part == 1) {
              sweep(2, true);
              continue;
            }
            e = run(ctx, SLA_K_SWEEP_XY, [&] {
              return sla::launch_cec_sweep_xy(rxy, part == 0, half, cur, u, nxt, ctx->flag,
                                              ctx->stream, pairs);
            });
            std::swap(cur, nxt);
          }
          break;
        }
        for (int d = 0; d < ndim - 1; ++d) sweep(d, false);
        sweep(ndim - 1, true);
        for (int d = ndim - 2; d >= 0; --d) sweep(d, false);
        break;
      }
    }
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "advection kernel launch");
  if (cur != phi) {
    e = run(ctx, SLA_K_COPY, [&] {
      return hipMemcpyAsync(phi, cur, n * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream);
    });
    if (e != hipSuccess) return hip_fail(ctx, e, "copy of the result");
  }
  return SLA_OK;
}

}  // namespace

extern "C" {

int sla_set_option(sla_ctx* ctx, int option, int64_t value) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  switch (option) {
    case SLA_OPT_FUSED:
      if (value != 0 && value != 1) return fail(ctx, SLA_EINVAL, "SLA_OPT_FUSED takes 0 or 1");
      ctx->fused = value != 0;
      return SLA_OK;
    case SLA_OPT_CEC3D_KERNEL:
      if (!sla::cec3d_variant_ok(int(value)))
        return fail(ctx, SLA_EINVAL, "SLA_OPT_CEC3D_KERNEL takes 1, 2 or 4 to 14");
      ctx->cec3d_kernel = int(value);
      return SLA_OK;
    case SLA_OPT_SWEEP_KERNEL:
      if (value < 0 || value > 3) return fail(ctx, SLA_EINVAL, "SLA_OPT_SWEEP_KERNEL takes 0 to 3");
      ctx->sweep_kernel = int(value);
      return SLA_OK;
    case SLA_OPT_EC_KERNEL:
      if (value < 0 || value > 3) return fail(ctx, SLA_EINVAL, "SLA_OPT_EC_KERNEL takes 0..3");
      ctx->ec_kernel = int(value);
      return SLA_OK;
    case SLA_OPT_SHARED_VELOCITY:
      if (value != 0 && value != 1 && value != 2 && value != 4)
        return fail(ctx, SLA_EINVAL, "SLA_OPT_SHARED_VELOCITY takes 0, 1, 2 or 4");
      ctx->multi = value <= 1 ? 1 : int(value);
      return SLA_OK;
    case SLA_OPT_EC_SHAPE:
      if (value < -4096 || value > 64) return fail(ctx, SLA_EINVAL, "SLA_OPT_EC_SHAPE takes -4096..64");
      ctx->ec_shape = int(value);
      return SLA_OK;
    case SLA_OPT_BACKTRACE:
      if (value != 0 && value != 1) return fail(ctx, SLA_EINVAL, "SLA_OPT_BACKTRACE takes 0 or 1");
      ctx->backtrace = int(value);
      return SLA_OK;
    case SLA_OPT_LEARNED_KERNEL:
      if (value != 0 && value != 1) return fail(ctx, SLA_EINVAL, "SLA_OPT_LEARNED_KERNEL takes 0 or 1");
      ctx->learned_kernel = int(value);
      return SLA_OK;
    case SLA_OPT_CEC3D_SHAPE:
      if (value < -4096 || value > 4096)
        return fail(ctx, SLA_EINVAL, "SLA_OPT_CEC3D_SHAPE takes -4096..4096");
      ctx->cec3d_shape = int(value);
      return SLA_OK;
  }
  return fail(ctx, SLA_EINVAL, "unknown option %d", option);
}

int sla_check(sla_ctx* ctx) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (capturing(ctx)) return fail(ctx, SLA_ECAPTURE, "this call synchronises the stream");
  DeviceGuard guard(ctx->device);
  int* h = static_cast<int*>(ctx->host);
  hipError_t e = hipMemcpyAsync(h, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "stream synchronise");
  if (*h) {
    e = hipMemsetAsync(ctx->flag, 0, sizeof(int), ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "clear the overflow record");
    return fail(ctx, SLA_ECOURANT, "a kernel met a Courant number beyond the reach it was built for");
  }
  return SLA_OK;
}

int sla_norms(sla_ctx* ctx, int64_t count, const float* a, const float* b, double* out) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (capturing(ctx)) return fail(ctx, SLA_ECAPTURE, "this call synchronises the stream");
  if (count < 0) return fail(ctx, SLA_EINVAL, "count must be >= 0");
  if (!out) return fail(ctx, SLA_EINVAL, "out must not be NULL");
  if (count == 0) {
    for (int k = 0; k < 5; ++k) out[k] = 0.0;
    return SLA_OK;
  }
  if (!a || !b) return fail(ctx, SLA_EINVAL, "a and b must not be NULL");
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(ctx, SLA_EHIP, "cannot select device %d", ctx->device);
  double* res = ctx->dpart + 5 * sla::kNormBlocks;
  hipError_t e = sla::launch_norms(count, a, b, ctx->dpart, res, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "norms launch");
  double* h = static_cast<double*>(ctx->host);
  e = hipMemcpyAsync(h, res, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "norms");
  for (int k = 0; k < 5; ++k) out[k] = h[k];
  return SLA_OK;
}

int sla_tune(sla_ctx* ctx, const sla_grid* grid, const float* phi, const float* u, double dt,
             const char* table_path) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (capturing(ctx)) return fail(ctx, SLA_ECAPTURE, "tuning synchronises the stream");
  int rc = check_grid(ctx, grid);
  if (rc) return rc;
  if (grid->ndim != 3) return fail(ctx, SLA_EINVAL, "the fused step is 3D");
  if (!phi || !u) return fail(ctx, SLA_EINVAL, "phi and u must not be NULL");
  if (!std::isfinite(dt)) return fail(ctx, SLA_EINVAL, "dt must be finite");
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(ctx, SLA_EHIP, "cannot select device %d", ctx->device);
  const sla::Geo geo = make_geo(grid, dt);
  if (!sla::offsets32_ok(geo))
    return fail(ctx, SLA_EINVAL, "the fused step takes fewer than 2^30 cells (or 2^30 with ny >= 2)");
  float cm[3];
  rc = measure_courant(ctx, grid, geo, u, cm);
  if (rc) return rc;
  if (!(cm[0] < 1.f && cm[1] < 1.f && cm[2] < 1.f))
    return fail(ctx, SLA_ECOURANT, "the fused step takes Courant numbers below 1 (max %g)",
                double(std::fmax(cm[0], std::fmax(cm[1], cm[2]))));
  const size_t n = size_t(geo.ncells);
  rc = ensure_work(ctx, n);
  if (rc) return rc;
  // candidates: (variant, launch shape)
  static const int cand[][2] = {{1, 0},    {2, 0},    {4, 0},   {6, 0},     {7, 0},     {7, 32},
                                {8, -64},  {8, -32},  {8, 0},   {9, -64},   {10, -32},  {11, -32},
                                {14, 0},   {14, -128}, {14, -64}, {14, -32}, {14, -16}};
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  sla_ctx::Tuned best = {{geo.nx, geo.ny, geo.nz}, {5, 5}, {0, 0}, {1e30, 1e30}};
  constexpr int kReps = 3;
  for (int par = 0; par < 2 && e == hipSuccess; ++par) {
    for (const auto& c : cand) {
      sla::Cec3dLaunch lc;
      lc.ychunk = c[1];
      auto launch = [&] {
        return sla::launch_cec3d(c[0], par == 0, geo, phi, u, ctx->work, ctx->flag, ctx->stream, lc);
      };
      e = launch();  // warm-up
      if (e == hipSuccess) e = hipEventRecord(a, ctx->stream);
      for (int r = 0; r < kReps && e == hipSuccess; ++r) e = launch();
      if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e != hipSuccess) break;
      const double avg = double(ms) / kReps;
      if (avg < best.ms[par]) {
        best.ms[par] = avg;
        best.variant[par] = c[0];
        best.shape[par] = c[1];
      }
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(ctx, e, "tuning launches");
  put_tuned(ctx, best);
  if (table_path) {
    // rewrite the table: other grids' lines kept, this grid's replaced
    std::vector<std::string> keep;
    if (FILE* f = std::fopen(table_path, "r")) {
      char line[256];
      while (std::fgets(line, sizeof line, f)) {
        int nx, ny, nz;
        if (line[0] == '#' || std::sscanf(line, "%d %d %d", &nx, &ny, &nz) != 3) continue;
        if (nx == geo.nx && ny == geo.ny && nz == geo.nz) continue;
        keep.push_back(line);
      }
      std::fclose(f);
    }
    FILE* f = std::fopen(table_path, "w");
    if (!f) return fail(ctx, SLA_EINVAL, "cannot write the tuning table %s", table_path);
    std::fprintf(f, "# nx ny nz even:variant shape ms odd:variant shape ms\n");
    for (const auto& l : keep) std::fputs(l.c_str(), f);
    std::fprintf(f, "%d %d %d %d %d %.4f %d %d %.4f\n", geo.nx, geo.ny, geo.nz, best.variant[0],
                 best.shape[0], best.ms[0], best.variant[1], best.shape[1], best.ms[1]);
    std::fclose(f);
  }
  return SLA_OK;
}

int sla_tune_load(sla_ctx* ctx, const char* table_path) {
  if (!ctx || !table_path) return SLA_EINVAL;
  ctx->err.clear();
  FILE* f = std::fopen(table_path, "r");
  if (!f) return fail(ctx, SLA_EINVAL, "cannot read the tuning table %s", table_path);
  char line[256];
  int rc = SLA_OK;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    sla_ctx::Tuned t;
    if (std::sscanf(line, "%d %d %d %d %d %lf %d %d %lf", &t.n[0], &t.n[1], &t.n[2], &t.variant[0],
                    &t.shape[0], &t.ms[0], &t.variant[1], &t.shape[1], &t.ms[1]) != 9 ||
        !sla::cec3d_variant_ok(t.variant[0]) || !sla::cec3d_variant_ok(t.variant[1]) ||
        t.variant[0] == 5 || t.variant[1] == 5 || t.shape[0] < -4096 || t.shape[0] > 4096 ||
        t.shape[1] < -4096 || t.shape[1] > 4096 || t.n[0] < 8 || t.n[1] < 8 || t.n[2] < 8) {
      rc = fail(ctx, SLA_EINVAL, "malformed tuning table line: %s", line);
      break;
    }
    put_tuned(ctx, t);
  }
  std::fclose(f);
  return rc;
}

int sla_tune_info(const sla_ctx* ctx, const sla_grid* grid, int32_t* variants, int32_t* shapes,
                  double* ms) {
  if (!ctx || !grid || grid->ndim != 3) return SLA_EINVAL;
  sla::Geo g;
  g.nx = grid->n[0];
  g.ny = grid->n[1];
  g.nz = grid->n[2];
  const sla_ctx::Tuned* t = find_tuned(ctx, g);
  if (!t) return SLA_EINVAL;
  for (int p = 0; p < 2; ++p) {
    if (variants) variants[p] = t->variant[p];
    if (shapes) shapes[p] = t->shape[p];
    if (ms) ms[p] = t->ms[p];
  }
  return SLA_OK;
}

int sla_timing(sla_ctx* ctx, int enable) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (enable) {
    DeviceGuard guard(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "stream synchronise");
    fold_marks(ctx);
    for (int k = 0; k < SLA_K_COUNT; ++k) {
      ctx->launches[k] = 0;
      ctx->ms[k] = 0.0;
    }
  }
  ctx->timing = enable != 0;
  return SLA_OK;
}

int sla_timing_read(sla_ctx* ctx, int64_t* launches, double* ms) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (!launches || !ms) return fail(ctx, SLA_EINVAL, "launches and ms must not be NULL");
  DeviceGuard guard(ctx->device);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "stream synchronise");
  fold_marks(ctx);
  for (int k = 0; k < SLA_K_COUNT; ++k) {
    launches[k] = ctx->launches[k];
    ms[k] = ctx->ms[k];
  }
  return SLA_OK;
}


// ------------------------------------------------------------------ models

void sla_model_destroy(sla_model* model) {
  if (!model) return;
  {
    DeviceGuard guard(model->device);
    for (void* p : {(void*)model->master, (void*)model->mo, (void*)model->vo, (void*)model->wr,
                    model->wpack, (void*)model->grad, (void*)model->gpart, (void*)model->lpart,
                    (void*)model->loss})
      if (p) (void)hipFree(p);
  }
  delete model;
}

int sla_model_create(sla_ctx* ctx, sla_model** out) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (!out) return fail(ctx, SLA_EINVAL, "out must not be NULL");
  *out = nullptr;
  DeviceGuard guard(ctx->device);
  sla_model* m = new sla_model;
  m->device = ctx->device;
  const size_t P = sla::kMlpParams * sizeof(float);
  bool ok = guard.ok;
  ok = ok && hipMalloc(&m->master, P) == hipSuccess;
  ok = ok && hipMalloc(&m->mo, P) == hipSuccess;
  ok = ok && hipMalloc(&m->vo, P) == hipSuccess;
  ok = ok && hipMalloc(&m->wr, P) == hipSuccess;
  ok = ok && hipMalloc(&m->wpack, sla::kMlpPackElems * 2) == hipSuccess;
  ok = ok && hipMalloc(&m->grad, P) == hipSuccess;
  ok = ok && hipMalloc(&m->gpart, size_t(sla::kMlpMaxBlocks) * sla::kMlpPartStride * sizeof(float)) ==
                  hipSuccess;
  ok = ok && hipMalloc(&m->lpart, sla::kMlpMaxBlocks * sizeof(float)) == hipSuccess;
  ok = ok && hipMalloc(&m->loss, sizeof(double)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    sla_model_destroy(m);
    return fail(ctx, SLA_ENOMEM, "cannot allocate model memory");
  }
  hipError_t e = hipMemsetAsync(m->master, 0, P, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->mo, 0, P, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->vo, 0, P, ctx->stream);
  if (e == hipSuccess) e = sla::launch_pack(m->master, m->wr, m->wpack, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    sla_model_destroy(m);
    return hip_fail(ctx, e, "model initialisation");
  }
  *out = m;
  return SLA_OK;
}

int sla_model_set_params(sla_ctx* ctx, sla_model* model, const float* params, int64_t n) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (!model || !params) return fail(ctx, SLA_EINVAL, "model and params must not be NULL");
  if (n != sla::kMlpParams) return fail(ctx, SLA_EINVAL, "need %d parameters", sla::kMlpParams);
  DeviceGuard guard(ctx->device);
  const size_t P = sla::kMlpParams * sizeof(float);
  hipError_t e = hipMemcpyAsync(model->master, params, P, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(model->mo, 0, P, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(model->vo, 0, P, ctx->stream);
  if (e == hipSuccess) e = sla::launch_pack(model->master, model->wr, model->wpack, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "set model parameters");
  model->adam_t = 0;
  return SLA_OK;
}

int sla_model_get_params(sla_ctx* ctx, const sla_model* model, float* params, int64_t n) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (!model || !params) return fail(ctx, SLA_EINVAL, "model and params must not be NULL");
  if (n != sla::kMlpParams) return fail(ctx, SLA_EINVAL, "need %d parameters", sla::kMlpParams);
  DeviceGuard guard(ctx->device);
  hipError_t e = hipMemcpyAsync(params, model->master, sla::kMlpParams * sizeof(float),
                                hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "get model parameters");
  return SLA_OK;
}

int sla_model_set_courant_range(sla_model* model, double range) {
  if (!model || !(range >= 0.0) || !std::isfinite(range)) return SLA_EINVAL;
  model->range = range;
  return SLA_OK;
}

int sla_make_pairs(sla_ctx* ctx, const sla_grid* grid, const float* phi1, const float* phi_next,
                   const float* u, double dt, const int32_t* cells, int64_t m, uint16_t* feats,
                   float* target, float* sigma) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  int rc = check_grid(ctx, grid);
  if (rc) return rc;
  if (grid->ndim != 3) return fail(ctx, SLA_EINVAL, "training pairs need a 3D grid");
  if (!phi1 || !phi_next || !u || !cells || !feats || !target || !sigma)
    return fail(ctx, SLA_EINVAL, "pointer arguments must not be NULL");
  if (m < 0 || m > (int64_t(1) << 30)) return fail(ctx, SLA_EINVAL, "bad row count");
  if (!std::isfinite(dt)) return fail(ctx, SLA_EINVAL, "dt must be finite");
  if (m == 0) return SLA_OK;
  DeviceGuard guard(ctx->device);
  const sla::Geo geo = make_geo(grid, dt);
  hipError_t e = sla::launch_make_pairs(geo, phi1, phi_next, u, cells, int(m), feats, target, sigma,
                                        ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "make pairs launch");
  return SLA_OK;
}

int sla_model_forward(sla_ctx* ctx, const sla_model* model, const uint16_t* feats, int64_t m,
                      float* y) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (!model || !feats || !y) return fail(ctx, SLA_EINVAL, "pointer arguments must not be NULL");
  if (m < 0 || m > (int64_t(1) << 30)) return fail(ctx, SLA_EINVAL, "bad row count");
  if (m == 0) return SLA_OK;
  DeviceGuard guard(ctx->device);
  hipError_t e = sla::launch_mlp(false, feats, nullptr, int(m), 0.f, model->wpack, model->wr, y,
                                 nullptr, nullptr, nullptr, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "network forward launch");
  return SLA_OK;
}

}  // extern "C"

namespace {
// The gradient of the mean squared error over the m rows into model->grad and
// the loss sum into model->loss; with lr >= 0 also the Adam step (the update
// in the reduction's kernel).
int model_gradient(sla_ctx* ctx, sla_model* model, const uint16_t* feats, const float* target,
                   int64_t m, double lr = -1.0) {
  if (!model || !feats || !target) return fail(ctx, SLA_EINVAL, "pointer arguments must not be NULL");
  if (m <= 0 || m > (int64_t(1) << 30)) return fail(ctx, SLA_EINVAL, "bad row count");
  int nblk = 0;
  hipError_t e = sla::launch_mlp(true, feats, target, int(m), float(2.0 / double(m)), model->wpack,
                                 model->wr, nullptr, model->gpart, model->lpart, &nblk, ctx->stream);
  if (e == hipSuccess && lr < 0.0)
    e = sla::launch_grad_reduce(model->gpart, model->lpart, nblk, model->grad, model->loss,
                                ctx->stream);
  if (e == hipSuccess && lr >= 0.0) {
    model->adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = float(1.0 - std::pow(b1, double(model->adam_t)));
    const float bc2 = float(1.0 - std::pow(b2, double(model->adam_t)));
    e = sla::launch_grad_adam(model->gpart, model->lpart, nblk, model->grad, model->loss,
                              model->master, model->mo, model->vo, float(lr), float(b1), float(b2),
                              1e-8f, bc1, bc2, model->wr, model->wpack, ctx->stream);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "network gradient launch");
  return SLA_OK;
}

int read_loss(sla_ctx* ctx, sla_model* model, int64_t m, double* loss) {
  double* h = static_cast<double*>(ctx->host);
  hipError_t e = hipMemcpyAsync(h, model->loss, sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "read loss");
  *loss = *h / double(m);
  return SLA_OK;
}
}  // namespace

extern "C" {

int sla_model_grads(sla_ctx* ctx, sla_model* model, const uint16_t* feats, const float* target,
                    int64_t m, float* grads, double* loss) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (!grads || !loss) return fail(ctx, SLA_EINVAL, "grads and loss must not be NULL");
  DeviceGuard guard(ctx->device);
  int rc = model_gradient(ctx, model, feats, target, m);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(grads, model->grad, sla::kMlpParams * sizeof(float),
                                hipMemcpyDeviceToHost, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "read gradient");
  return read_loss(ctx, model, m, loss);
}

int sla_model_train_step(sla_ctx* ctx, sla_model* model, const uint16_t* feats, const float* target,
                         int64_t m, double lr, double* loss) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (!(lr >= 0.0) || !std::isfinite(lr)) return fail(ctx, SLA_EINVAL, "bad learning rate");
  DeviceGuard guard(ctx->device);
  int rc = model_gradient(ctx, model, feats, target, m, lr);
  if (rc) return rc;
  if (loss) return read_loss(ctx, model, m, loss);
  return SLA_OK;
}

int sla_advect_learned(sla_ctx* ctx, const sla_model* model, const sla_grid* grid, float* phi,
                       const float* u, double dt, int32_t steps, int64_t step0,
                       double courant_max, int32_t* fell_back) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (fell_back) *fell_back = 0;
  int rc = check_grid(ctx, grid);
  if (rc) return rc;
  if (!model || !phi || !u) return fail(ctx, SLA_EINVAL, "model, phi and u must not be NULL");
  if (!std::isfinite(dt)) return fail(ctx, SLA_EINVAL, "dt must be finite");
  if (steps < 0) return fail(ctx, SLA_EINVAL, "steps must be >= 0");
  if (std::isnan(courant_max)) return fail(ctx, SLA_EINVAL, "courant_max is NaN");
  if (steps == 0) return SLA_OK;
  DeviceGuard guard(ctx->device);
  const sla::Geo geo = make_geo(grid, dt);
  double cm = courant_max;
  if (!(cm > 0.0)) {
    if (capturing(ctx))
      return fail(ctx, SLA_ECAPTURE, "measuring the Courant bound synchronises the stream: "
                  "pass courant_max > 0 while capturing");
    float c3[3];
    rc = measure_courant(ctx, grid, geo, u, c3);
    if (rc) return rc;
    cm = std::fmax(c3[0], std::fmax(c3[1], c3[2]));
  }
  int why = SLA_OK;
  if (grid->ndim != 3 || model->range <= 0.0) why = SLA_ENOMODEL;
  else if (cm > model->range) why = SLA_ECOURANT;
  if (why != SLA_OK) {
    if (!fell_back)
      return fail(ctx, why, why == SLA_ENOMODEL ? "model is untrained or the grid is not 3D"
                                                : "Courant bound %g beyond the model's range %g",
                  cm, model->range);
    *fell_back = 1;
    return sla_advect(ctx, grid, phi, u, dt, SLA_CEC, steps, step0, courant_max);
  }
  if (!(cm < SLA_MAX_REACH))
    return fail(ctx, SLA_ECOURANT, "Courant bound %g: must be below %d", cm, SLA_MAX_REACH);
  const size_t n = size_t(geo.ncells);
  rc = ensure_work(ctx, n);
  if (rc) return rc;
  hipError_t e = hipSuccess;
  for (int32_t k = 0; k < steps && e == hipSuccess; ++k) {
    e = run(ctx, SLA_K_CIR, [&] {
      return sla::launch_cir(3, geo, phi, u, ctx->work, ctx->flag, ctx->stream);
    });
    if (e == hipSuccess)
      e = run(ctx, SLA_K_LEARNED, [&] {
        return ctx->learned_kernel == 1
                   ? sla::launch_learned_march(geo, ctx->work, u, model->wpack, model->wr, phi,
                                               ctx->stream)
                   : sla::launch_learned_correct(geo, ctx->work, u, model->wpack, model->wr, phi,
                                                 ctx->stream);
      });
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "learned step launch");
  return SLA_OK;
}


// ------------------------------------------------------------------ plans

}  // extern "C"

namespace {

// Work items of every problem for a y extent ychunk.  Problems sharing a
// velocity (same pointer and grid) are interleaved so that the items of one
// tile for all of them have indices congruent modulo 8: with a persistent
// grid whose size is a multiple of 8, they land on the same accelerator
// partition (workgroups are dealt to the 8 partitions round-robin) in the
// same round, and share that partition's L2.
// Problems with their own velocity planes and at least 2^24 cells fill the
// GPU alone: they run one launch of the context's fused step per step (the
// same FP32 operations as the tiles of the persistent kernel), which is
// faster than their tiles in the work list.  The persistent kernel takes the
// rest, where many small problems share its launch.
constexpr size_t kPlanDirectCells = size_t(1) << 24;
bool plan_direct(const sla_problem& p) {
  return p.u && size_t(p.grid.n[0]) * p.grid.n[1] * p.grid.n[2] >= kPlanDirectCells;
}

std::vector<int4> build_items(const std::vector<sla_problem>& P, int ychunk,
                              const std::vector<bool>& skip) {
  std::vector<int4> items;
  std::vector<bool> done(skip);  // problems outside the work list count as done
  auto tiles_of = [&](const sla_problem& p, std::vector<int3>& t) {
    const int tx = (p.grid.n[0] + sla::kBatchTileX - 1) / sla::kBatchTileX;
    const int tz = (p.grid.n[2] + sla::kBatchTileZ - 1) / sla::kBatchTileZ;
    const int cy = (p.grid.n[1] + ychunk - 1) / ychunk;
    for (int c = 0; c < cy; ++c)
      for (int z = 0; z < tz; ++z)
        for (int x = 0; x < tx; ++x) t.push_back(make_int3(x, z, c));
  };
  for (size_t i = 0; i < P.size(); ++i) {
    if (done[i]) continue;
    std::vector<int> group{int(i)};
    done[i] = true;
    if (P[i].u)
      for (size_t j = i + 1; j < P.size(); ++j)
        if (!done[j] && P[j].u == P[i].u && P[j].grid.n[0] == P[i].grid.n[0] &&
            P[j].grid.n[1] == P[i].grid.n[1] && P[j].grid.n[2] == P[i].grid.n[2]) {
          group.push_back(int(j));
          done[j] = true;
        }
    std::vector<int3> tiles;
    tiles_of(P[i], tiles);
    const int S = int(group.size());
    if (S > 1)  // start a shared group on a partition boundary
      while (items.size() % 8) items.push_back(make_int4(-1, 0, 0, 0));
    for (size_t b = 0; b < tiles.size(); b += 8) {
      const int nb = int(std::min<size_t>(8, tiles.size() - b));
      for (int sidx = 0; sidx < S; ++sidx)
        for (int r = 0; r < 8; ++r) {
          if (r < nb)
            items.push_back(make_int4(group[sidx], tiles[b + r].x, tiles[b + r].y, tiles[b + r].z));
          else if (S > 1)
            items.push_back(make_int4(-1, 0, 0, 0));  // keep the partition alignment
        }
    }
  }
  // drop alignment holes at the very end; the kernel skips problem -1 items
  while (!items.empty() && items.back().x < 0) items.pop_back();
  return items;
}

int plan_upload(sla_ctx* ctx, sla_plan* pl, const std::vector<sla_problem>& P, int ychunk) {
  std::vector<sla::BatchProblem> bp(P.size());
  for (size_t i = 0; i < P.size(); ++i) bp[i].ychunk = std::min(ychunk, P[i].grid.n[1]);
  for (size_t i = 0; i < P.size(); ++i) {
    const sla_problem& p = P[i];
    const size_t n = pl->cells[i];
    bp[i].buf[0] = p.phi;
    bp[i].buf[1] = pl->work[i];
    if (p.u) {
      bp[i].u[0] = p.u;
      bp[i].u[1] = p.u + n;
      bp[i].u[2] = p.u + 2 * n;
      bp[i].umask = ~0u;
    } else {
      bp[i].u[0] = pl->uniform + 3 * i;
      bp[i].u[1] = pl->uniform + 3 * i + 1;
      bp[i].u[2] = pl->uniform + 3 * i + 2;
      bp[i].umask = 0u;
    }
    for (int d = 0; d < 3; ++d) {
      bp[i].n[d] = p.grid.n[d];
      bp[i].lam[d] = float(p.dt / p.grid.dx[d]);
    }
  }
  std::vector<bool> skip(P.size(), false);
  for (int i : pl->direct) skip[size_t(i)] = true;
  std::vector<int4> items = build_items(P, ychunk, skip);
  if (pl->ditems) (void)hipFree(pl->ditems);
  pl->ditems = nullptr;
  if (hipMalloc(&pl->ditems, std::max<size_t>(1, items.size()) * sizeof(int4)) != hipSuccess)
    return fail(ctx, SLA_ENOMEM, "plan work list");
  hipError_t e = hipMemcpy(pl->ditems, items.data(), items.size() * sizeof(int4),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(pl->dprobs, bp.data(), bp.size() * sizeof(sla::BatchProblem),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "plan upload");
  pl->nitems = int(items.size());
  pl->ychunk = ychunk;
  return SLA_OK;
}

// Launch the plan's steps on stream st (also used while capturing).
// Step k of a plan: the persistent kernel over the work list, then one
// fused-step launch per direct problem.  Even k reads the caller's fields
// and writes the work fields, odd k the reverse.
hipError_t plan_step(sla_plan* pl, hipStream_t st, int32_t k) {
  const bool even = (pl->step0 + k) % 2 == 0;
  hipError_t e = hipSuccess;
  if (pl->nitems > 0)
    e = sla::launch_cec3d_batch(even, pl->dprobs, pl->ditems, pl->nitems, k & 1, pl->blocks,
                                pl->flag, st);
  for (size_t j = 0; j < pl->groups.size() && e == hipSuccess; ++j) {
    const std::vector<int>& grp = pl->groups[j];
    const int h = grp[0];
    if (grp.size() == 1) {
      float* a = pl->phis[size_t(h)];
      float* b = pl->work[size_t(h)];
      e = sla::launch_cec3d(pl->cec3d_kernel, even, pl->geo[size_t(h)], (k & 1) ? b : a,
                            pl->u[size_t(h)], (k & 1) ? a : b, pl->flag, st);
      continue;
    }
    const float* in[4];
    float* out[4];
    for (size_t f = 0; f < grp.size(); ++f) {
      float* a = pl->phis[size_t(grp[f])];
      float* b = pl->work[size_t(grp[f])];
      in[f] = (k & 1) ? b : a;
      out[f] = (k & 1) ? a : b;
    }
    e = sla::launch_cec3d_multi(int(grp.size()), even, pl->geo[size_t(h)], in, out, pl->u[size_t(h)],
                                pl->flag, st);
  }
  return e;
}

hipError_t plan_launch(sla_plan* pl, hipStream_t st, int32_t steps) {
  hipError_t e = hipSuccess;
  for (int32_t k = 0; k < steps && e == hipSuccess; ++k) e = plan_step(pl, st, k);
  if (e == hipSuccess && (steps & 1))
    e = sla::launch_batch_copy_back(pl->dprobs, pl->nprob, st);
  return e;
}

}  // namespace

extern "C" {

void sla_plan_destroy(sla_plan* pl) {
  if (!pl) return;
  {
    DeviceGuard guard(pl->device);
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->cap) (void)hipStreamDestroy(pl->cap);
    for (float* w : pl->work)
      if (w) (void)hipFree(w);
    if (pl->uniform) (void)hipFree(pl->uniform);
    if (pl->dprobs) (void)hipFree(pl->dprobs);
    if (pl->ditems) (void)hipFree(pl->ditems);
  }
  delete pl;
}

int sla_plan_create(sla_ctx* ctx, sla_plan** out, int32_t nprob, const sla_problem* probs,
                    int32_t steps, int64_t step0, double courant_max, int32_t tune) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (!out || !probs || nprob <= 0) return fail(ctx, SLA_EINVAL, "need out, probs and nprob > 0");
  *out = nullptr;
  if (steps < 0) return fail(ctx, SLA_EINVAL, "steps must be >= 0");
  if (std::isnan(courant_max)) return fail(ctx, SLA_EINVAL, "courant_max is NaN");
  if (ctx->backtrace != 0)
    return fail(ctx, SLA_EINVAL, "plans run the arrival-node backtrace (SLA_OPT_BACKTRACE = 0)");
  if (capturing(ctx))
    return fail(ctx, SLA_ECAPTURE, "creating a plan allocates and synchronises the stream");
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return fail(ctx, SLA_EHIP, "cannot select device %d", ctx->device);
  std::vector<sla_problem> P(probs, probs + nprob);
  // validate; measure or check the Courant bound
  for (int i = 0; i < nprob; ++i) {
    int rc = check_grid(ctx, &P[i].grid);
    if (rc) return rc;
    if (P[i].grid.ndim != 3) return fail(ctx, SLA_EINVAL, "problem %d: plans take 3D grids", i);
    if (int64_t(P[i].grid.n[0]) * P[i].grid.n[1] * P[i].grid.n[2] > (int64_t(1) << 30))
      return fail(ctx, SLA_EINVAL, "problem %d: plans take grids of at most 2^30 cells", i);
    if (!P[i].phi) return fail(ctx, SLA_EINVAL, "problem %d: phi is NULL", i);
    if (!std::isfinite(P[i].dt)) return fail(ctx, SLA_EINVAL, "problem %d: dt must be finite", i);
    const sla::Geo geo = make_geo(&P[i].grid, P[i].dt);
    if (!sla::offsets32_ok(geo))
      return fail(ctx, SLA_EINVAL, "problem %d: a plan's grid of 2^30 cells needs ny >= 2", i);
    float cm = 0.f;
    if (!P[i].u) {
      for (int d = 0; d < 3; ++d) {
        if (!std::isfinite(P[i].u_uniform[d]))
          return fail(ctx, SLA_EINVAL, "problem %d: non-finite uniform velocity", i);
        cm = std::fmax(cm, std::fabs(P[i].u_uniform[d] * geo.lam[d]));
      }
    } else if (courant_max > 0.0) {
      cm = float(courant_max);
    } else {
      float c3[3];
      rc = measure_courant(ctx, &P[i].grid, geo, P[i].u, c3);
      if (rc) return rc;
      cm = std::fmax(c3[0], std::fmax(c3[1], c3[2]));
    }
    if (!(cm < 1.f))
      return fail(ctx, SLA_ECOURANT, "problem %d: Courant bound %g, plans need < 1", i, double(cm));
  }
  sla_plan* pl = new sla_plan;
  pl->device = ctx->device;
  pl->nprob = nprob;
  pl->steps = steps;
  pl->step0 = step0;
  pl->flag = ctx->flag;
  pl->cec3d_kernel = ctx->cec3d_kernel;
  for (int i = 0; i < nprob; ++i) {
    pl->geo.push_back(make_geo(&P[i].grid, P[i].dt));
    pl->u.push_back(P[i].u);
    if (plan_direct(P[i])) pl->direct.push_back(i);
  }
  for (size_t j = 0; j < pl->direct.size(); ++j) {
    const int i = pl->direct[j];
    bool placed = false;
    for (auto& grp : pl->groups) {
      const int h = grp[0];
      const sla::Geo &a = pl->geo[size_t(h)], &b = pl->geo[size_t(i)];
      const bool same = int(grp.size()) < ctx->multi && pl->u[size_t(h)] == pl->u[size_t(i)] &&
                        a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.lam[0] == b.lam[0] &&
                        a.lam[1] == b.lam[1] && a.lam[2] == b.lam[2];
      if (same) {
        grp.push_back(i);
        placed = true;
        break;
      }
    }
    if (!placed) pl->groups.push_back({i});
  }
  // groups of three run as two and one
  for (size_t q = 0; q < pl->groups.size(); ++q)
    if (pl->groups[q].size() == 3) {
      pl->groups.push_back({pl->groups[q][2]});
      pl->groups[q].pop_back();
    }
  bool ok = true;
  std::vector<float> uni(3 * size_t(nprob), 0.f);
  for (int i = 0; i < nprob; ++i) {
    const size_t n = size_t(P[i].grid.n[0]) * P[i].grid.n[1] * P[i].grid.n[2];
    pl->cells.push_back(n);
    pl->phis.push_back(P[i].phi);
    float* w = nullptr;
    ok = ok && hipMalloc(&w, n * sizeof(float)) == hipSuccess;
    pl->work.push_back(w);
    for (int d = 0; d < 3; ++d) uni[3 * i + d] = P[i].u_uniform[d];
  }
  ok = ok && hipMalloc(&pl->uniform, uni.size() * sizeof(float)) == hipSuccess;
  ok = ok && hipMalloc(&pl->dprobs, size_t(nprob) * sizeof(sla::BatchProblem)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    sla_plan_destroy(pl);
    return fail(ctx, SLA_ENOMEM, "cannot allocate plan memory");
  }
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpy(pl->uniform, uni.data(), uni.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    sla_plan_destroy(pl);
    return hip_fail(ctx, e, "plan set-up");
  }
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
  const int per_cu = sla::cec3d_batch_blocks_per_cu();
  const int full = std::max(8, (cus * per_cu) / 8 * 8);
  int best_y = 128, best_b = full;
  double best_ms = 0.0;
  if (tune && steps > 0) {
    // time one step (reads the fields, writes the work memory) per candidate
    hipEvent_t a = nullptr, b = nullptr;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    best_ms = 1e30;
    const int ychunks[] = {32, 64, 128, 256};
    const int blocks[] = {full, 2 * full};
    for (int yc : ychunks) {
      int rc = plan_upload(ctx, pl, P, yc);
      if (rc) {
        sla_plan_destroy(pl);
        return rc;
      }
      for (int bl : blocks) {
        pl->blocks = bl;
        float ms = 0.f, tot = 0.f;
        for (int r = 0; r < 3 && e == hipSuccess; ++r) {
          e = hipEventRecord(a, ctx->stream);
          if (e == hipSuccess) e = plan_step(pl, ctx->stream, 0);  // writes work fields only
          if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
          if (e == hipSuccess) e = hipEventSynchronize(b);
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
          if (r > 0) tot += ms;  // the first run warms up
        }
        if (e != hipSuccess) break;
        const double avg = tot / 2.0;
        if (avg < best_ms) {
          best_ms = avg;
          best_y = yc;
          best_b = bl;
        }
      }
      if (e != hipSuccess) break;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) {
      sla_plan_destroy(pl);
      return hip_fail(ctx, e, "plan tuning");
    }
  }
  int rc = plan_upload(ctx, pl, P, best_y);
  if (rc) {
    sla_plan_destroy(pl);
    return rc;
  }
  pl->blocks = best_b;
  pl->step_ms = best_ms;
  // capture all steps into one graph on a private stream
  e = hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = plan_launch(pl, pl->cap, steps);
    e = hipStreamEndCapture(pl->cap, &pl->graph);
    if (e == hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    sla_plan_destroy(pl);
    return hip_fail(ctx, e, "plan graph capture");
  }
  *out = pl;
  return SLA_OK;
}

int sla_plan_run(sla_ctx* ctx, sla_plan* plan) {
  if (!ctx) return SLA_EINVAL;
  ctx->err.clear();
  if (!plan) return fail(ctx, SLA_EINVAL, "plan is NULL");
  if (plan->device != ctx->device) return fail(ctx, SLA_EINVAL, "plan belongs to another device");
  if (plan->steps == 0) return SLA_OK;
  DeviceGuard guard(ctx->device);
  hipError_t e = run(ctx, SLA_K_CEC3D, [&] { return hipGraphLaunch(plan->exec, ctx->stream); });
  if (e != hipSuccess) return hip_fail(ctx, e, "plan launch");
  return SLA_OK;
}

int sla_plan_info(const sla_plan* plan, int32_t* ychunk, int32_t* blocks, int32_t* items,
                  double* step_ms) {
  if (!plan) return SLA_EINVAL;
  if (ychunk) *ychunk = plan->ychunk;
  if (blocks) *blocks = plan->blocks;
  if (items) *items = plan->nitems;
  if (step_ms) *step_ms = plan->step_ms;
  return SLA_OK;
}

}  // extern "C"
