// The extern "C" entry points of libpint: argument checks on the host, then
// dispatch to the small-d or dense-d kernels.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "../../include/pint.h"
#include "internal.h"

using namespace pint;

namespace {

int n_params_of(int32_t system, int32_t d) {
  switch (system) {
    case PINT_SYS_LINEAR: return d >= 1 ? d * d : -1;
    case PINT_SYS_LOGISTIC: return d == 1 ? 2 : -1;
    case PINT_SYS_VDP: return d == 2 ? 1 : -1;
    case PINT_SYS_CARTPOLE: return d == 4 ? 4 : -1;
    case PINT_SYS_LORENZ63: return d == 3 ? 3 : -1;
    case PINT_SYS_LORENZ96: return d >= 4 ? 1 : -1;
    case PINT_SYS_KURAMOTO: return d >= 1 ? d + 1 : -1;
    case PINT_SYS_ROBERTSON: return d == 3 ? 3 : -1;
  }
  return -1;
}

bool is_small(int32_t system, int32_t d) { return small_supported(system, d); }

int check_sys(const pint_system* sys, int64_t B) {
  if (!sys || B < 0) return PINT_ERR_INVALID_ARG;
  if (n_params_of(sys->system, sys->d) < 0) return PINT_ERR_INVALID_ARG;
  if (sys->n_params != n_params_of(sys->system, sys->d)) return PINT_ERR_INVALID_ARG;
  if (B > 0 && !sys->params) return PINT_ERR_INVALID_ARG;
  if (sys->method < PINT_RK4 || sys->method > PINT_TRAPEZOIDAL || sys->reserved != 0)
    return PINT_ERR_INVALID_ARG;
  if (!small_supported(sys->system, sys->d) && !dense_supported(sys->system, sys->d))
    return PINT_ERR_UNSUPPORTED;
  // the implicit rules are built for the small dimensions only
  if (sys->method != PINT_RK4 && !small_supported(sys->system, sys->d)) return PINT_ERR_UNSUPPORTED;
  return PINT_OK;
}

int check_opts(const pint_options* o) {
  if (!o) return PINT_ERR_INVALID_ARG;
  if (o->dtype != PINT_F64 && o->dtype != PINT_F32) return PINT_ERR_INVALID_ARG;
  if (o->guess != 0 && o->guess != 1) return PINT_ERR_INVALID_ARG;
  if (o->window < 0 || o->flags != 0 || o->tile < 0) return PINT_ERR_INVALID_ARG;
  if (o->block != 0 && o->block != 64 && o->block != 128 && o->block != 256) return PINT_ERR_INVALID_ARG;
  if (o->wg_per_cu < 0 || o->wg_per_cu > 16) return PINT_ERR_INVALID_ARG;
  if (!(o->tol > 0.0) || std::isnan(o->guard) || !(o->guard > 0.0)) return PINT_ERR_INVALID_ARG;
  return PINT_OK;
}

SolveArgs make_args(const pint_system* sys, int64_t B, const void* x0, double dt,
                    const int64_t* T_off, int64_t T_uniform, int64_t T_max,
                    const pint_options* o, void* traj, int64_t* iters, double* resid,
                    int32_t* status, void* ws, size_t ws_bytes, pint_stream_t stream) {
  SolveArgs a{};
  a.system = sys->system;
  a.d = sys->d;
  a.method = sys->method;
  a.dtype = o ? o->dtype : PINT_F64;
  a.B = B;
  a.x0 = x0;
  a.params = sys->params;
  a.pstride = sys->params_shared ? 0 : sys->n_params;
  a.T_off = T_off;
  a.T_uniform = T_uniform;
  a.T_max = T_max;
  a.traj = traj;
  a.dt = dt;
  if (o) {
    a.tol = o->tol;
    a.guard = o->guard;
    a.window = o->window;
    a.max_iter = o->max_iter > 0 ? o->max_iter : T_max + 1;
    a.guess = o->guess;
    a.tile = o->tile;
    a.block = o->block;
    a.wg_per_cu = o->wg_per_cu;
    a.order = o->order;
  }
  a.iters = iters;
  a.resid = resid;
  a.status = status;
  a.ws = ws;
  a.ws_bytes = ws_bytes;
  a.stream = reinterpret_cast<hipStream_t>(stream);
  return a;
}

uint64_t g_wait_limit = PINT_WAIT_LIMIT_DEFAULT;
uint32_t g_scan_delay = 0;
int g_dense_pipeline = 1;

}  // namespace

uint64_t pint::wait_limit() { return __atomic_load_n(&g_wait_limit, __ATOMIC_RELAXED); }
uint32_t pint::scan_delay() { return __atomic_load_n(&g_scan_delay, __ATOMIC_RELAXED); }
bool pint::dense_pipeline() { return __atomic_load_n(&g_dense_pipeline, __ATOMIC_RELAXED) != 0; }

extern "C" {

int pint_n_params(int32_t system, int32_t d) { return n_params_of(system, d); }

void pint_set_wait_limit(uint64_t polls) { __atomic_store_n(&g_wait_limit, polls, __ATOMIC_RELAXED); }

void pint_set_scan_delay(uint32_t sleeps) { __atomic_store_n(&g_scan_delay, sleeps, __ATOMIC_RELAXED); }

void pint_set_dense_pipeline(int on) { __atomic_store_n(&g_dense_pipeline, on ? 1 : 0, __ATOMIC_RELAXED); }

const char* pint_status_string(int32_t s) {
  switch (s) {
    case PINT_OK: return "ok";
    case PINT_ERR_INVALID_ARG: return "invalid argument";
    case PINT_ERR_DEVICE: return "device error";
    case PINT_ERR_WORKSPACE: return "workspace missing or too small";
    case PINT_NOT_CONVERGED: return "not converged within max_iter";
    case PINT_NONFINITE: return "non-finite residual or state";
    case PINT_ERR_UNSUPPORTED: return "unsupported system/dimension/dtype";
  }
  return "unknown status";
}

int pint_supported(int32_t system, int32_t d, int32_t dtype) {
  if (dtype != PINT_F64 && dtype != PINT_F32) return 0;
  if (n_params_of(system, d) < 0) return 0;
  return (small_supported(system, d) || dense_supported(system, d)) ? 1 : 0;
}

size_t pint_workspace_bytes(const pint_system* sys, int64_t B, int64_t T_total, int64_t T_max,
                            const pint_options* opts) {
  if (!sys || !opts || B < 0) return 0;
  pint_system s = *sys;
  SolveArgs a = make_args(&s, B, nullptr, 0.0, nullptr, T_max, T_max, opts, nullptr, nullptr,
                          nullptr, nullptr, nullptr, 0, nullptr);
  (void)T_total;
  if (is_small(sys->system, sys->d)) return small_ws_bytes(a);
  return dense_ws_bytes(a);
}

static pint_status solve_common(const pint_system* sys, int64_t B, const void* x0, double dt,
                                const int64_t* T_off, int64_t T_uniform, int64_t T_max,
                                const pint_options* opts, void* traj, int64_t* iters,
                                double* resid, int32_t* status, void* ws, size_t ws_bytes,
                                pint_stream_t stream) {
  if (int rc = check_sys(sys, B)) return (pint_status)rc;
  if (int rc = check_opts(opts)) return (pint_status)rc;
  if (!std::isfinite(dt) || T_max < 0 || T_uniform < 0) return PINT_ERR_INVALID_ARG;
  if (B == 0) return PINT_OK;
  if (!x0 || !iters || !resid || !status || (T_max > 0 && !traj)) return PINT_ERR_INVALID_ARG;
  SolveArgs a = make_args(sys, B, x0, dt, T_off, T_uniform, T_max, opts, traj, iters, resid,
                          status, ws, ws_bytes, stream);
  int rc;
  if (is_small(sys->system, sys->d)) {
    rc = small_solve(a);
  } else {
    if (T_off) return PINT_ERR_UNSUPPORTED;  // dense dimensions: uniform batches only
    if (opts->block != 0 || opts->wg_per_cu != 0 || opts->order) return PINT_ERR_UNSUPPORTED;
    rc = dense_solve(a);
  }
  return (pint_status)rc;
}

pint_status pint_solve_varlen(const pint_system* sys, int64_t B, const void* x0, double dt,
                              const int64_t* T_off, int64_t T_max, const pint_options* opts,
                              void* traj, int64_t* iters, double* resid, int32_t* status,
                              void* ws, size_t ws_bytes, pint_stream_t stream) {
  if (!T_off) return PINT_ERR_INVALID_ARG;
  return solve_common(sys, B, x0, dt, T_off, 0, T_max, opts, traj, iters, resid, status, ws,
                      ws_bytes, stream);
}

pint_status pint_solve(const pint_system* sys, int64_t B, const void* x0, double dt, int64_t T,
                       const pint_options* opts, void* traj, int64_t* iters, double* resid,
                       int32_t* status, void* ws, size_t ws_bytes, pint_stream_t stream) {
  return solve_common(sys, B, x0, dt, nullptr, T, T, opts, traj, iters, resid, status, ws,
                      ws_bytes, stream);
}

}  // extern "C"

struct pint_graph_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

pint_status pint_graph_capture_varlen(const pint_system* sys, int64_t B, const void* x0, double dt,
                                      const int64_t* T_off, int64_t T_max, const pint_options* opts,
                                      void* traj, int64_t* iters, double* resid, int32_t* status,
                                      void* ws, size_t ws_bytes, pint_graph* out) {
  if (!out) return PINT_ERR_INVALID_ARG;
  *out = nullptr;
  if (!T_off) return PINT_ERR_INVALID_ARG;
  if (int rc = check_sys(sys, B)) return (pint_status)rc;
  if (int rc = check_opts(opts)) return (pint_status)rc;
  if (!is_small(sys->system, sys->d)) return PINT_ERR_UNSUPPORTED;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return PINT_ERR_DEVICE;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return PINT_ERR_DEVICE;
  }
  const pint_status rc = solve_common(sys, B, x0, dt, T_off, 0, T_max, opts, traj, iters, resid,
                                      status, ws, ws_bytes, reinterpret_cast<pint_stream_t>(cs));
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &g);  // always end the capture
  (void)hipStreamDestroy(cs);
  if (rc != PINT_OK || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return rc != PINT_OK ? rc : PINT_ERR_DEVICE;
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess || !ex) {
    (void)hipGraphDestroy(g);
    return PINT_ERR_DEVICE;
  }
  pint_graph h = new (std::nothrow) pint_graph_s{g, ex};
  if (!h) {
    (void)hipGraphExecDestroy(ex);
    (void)hipGraphDestroy(g);
    return PINT_ERR_DEVICE;
  }
  *out = h;
  return PINT_OK;
}

pint_status pint_graph_launch(pint_graph graph, pint_stream_t stream) {
  if (!graph || !graph->exec) return PINT_ERR_INVALID_ARG;
  return hipGraphLaunch(graph->exec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? PINT_OK
                                                                                          : PINT_ERR_DEVICE;
}

pint_status pint_graph_destroy(pint_graph graph) {
  if (!graph) return PINT_ERR_INVALID_ARG;
  const bool ok = hipGraphExecDestroy(graph->exec) == hipSuccess && hipGraphDestroy(graph->graph) == hipSuccess;
  delete graph;
  return ok ? PINT_OK : PINT_ERR_DEVICE;
}

pint_status pint_seq_integrate(const pint_system* sys, int64_t B, const void* x0, double dt,
                               const int64_t* T_off, int64_t T_max, int32_t dtype, void* traj,
                               pint_stream_t stream) {
  if (int rc = check_sys(sys, B)) return (pint_status)rc;
  if ((dtype != PINT_F64 && dtype != PINT_F32) || T_max < 0 || !std::isfinite(dt))
    return PINT_ERR_INVALID_ARG;
  if (B == 0) return PINT_OK;
  if (!x0 || !T_off || (T_max > 0 && !traj)) return PINT_ERR_INVALID_ARG;
  pint_options o{};
  o.dtype = dtype;
  SolveArgs a = make_args(sys, B, x0, dt, T_off, 0, T_max, &o, traj, nullptr, nullptr, nullptr,
                          nullptr, 0, stream);
  int rc = is_small(sys->system, sys->d) ? small_seq(a) : dense_seq(a);
  return (pint_status)rc;
}

size_t pint_parareal_workspace_bytes(const pint_system* sys, int64_t B, int64_t M, int32_t dtype) {
  if (!sys || B < 0 || M < 0 || (dtype != PINT_F64 && dtype != PINT_F32)) return 0;
  return parareal_ws_bytes(sys->d, B, M, dtype);
}

pint_status pint_parareal(const pint_system* sys, int64_t B, const void* x0, double dt, int64_t M,
                          int64_t S, const pint_options* opts, void* traj, int64_t* iters,
                          double* resid, int32_t* status, double* hist, void* ws, size_t ws_bytes,
                          pint_stream_t stream) {
  if (int rc = check_sys(sys, B)) return (pint_status)rc;
  if (!is_small(sys->system, sys->d)) return PINT_ERR_UNSUPPORTED;
  if (!opts || (opts->dtype != PINT_F64 && opts->dtype != PINT_F32) || !(opts->tol > 0.0))
    return PINT_ERR_INVALID_ARG;
  if (opts->guess != 0 || opts->window != 0 || opts->tile != 0 || opts->flags != 0 ||
      opts->block != 0 || opts->wg_per_cu != 0 || opts->order)
    return PINT_ERR_INVALID_ARG;
  if (!std::isfinite(dt) || M < 0 || S < 0) return PINT_ERR_INVALID_ARG;
  if (M > 0 && S > INT64_MAX / M) return PINT_ERR_INVALID_ARG;
  if (B > 2147483647) return PINT_ERR_INVALID_ARG;  // one workgroup per instance
  if (B == 0) return PINT_OK;
  if (!x0 || !iters || !resid || !status || (M > 0 && S > 0 && !traj)) return PINT_ERR_INVALID_ARG;
  const int64_t max_iter = opts->max_iter > 0 ? opts->max_iter : M + 1;
  SolveArgs a = make_args(sys, B, x0, dt, nullptr, M * S, M * S, opts, traj, iters, resid, status,
                          ws, ws_bytes, stream);
  a.max_iter = max_iter;
  return (pint_status)parareal(a, M, S, hist);
}

pint_status pint_residual(const pint_system* sys, int64_t B, const void* x0, double dt, int64_t T,
                          int32_t dtype, const void* traj, void* h, double* hmax,
                          pint_stream_t stream) {
  if (int rc = check_sys(sys, B)) return (pint_status)rc;
  if ((dtype != PINT_F64 && dtype != PINT_F32) || T < 0 || !std::isfinite(dt))
    return PINT_ERR_INVALID_ARG;
  if (B == 0) return PINT_OK;
  if (!x0 || !hmax || (T > 0 && !traj)) return PINT_ERR_INVALID_ARG;
  pint_options o{};
  o.dtype = dtype;
  SolveArgs a = make_args(sys, B, x0, dt, nullptr, T, T, &o, const_cast<void*>(traj), nullptr,
                          nullptr, nullptr, nullptr, 0, stream);
  int rc = is_small(sys->system, sys->d) ? small_residual(a, h, hmax) : dense_residual(a, h, hmax);
  return (pint_status)rc;
}

pint_status pint_elements(const pint_system* sys, int64_t B, const void* x0, double dt, int64_t T,
                          int32_t dtype, const void* traj, void* A, void* b,
                          pint_stream_t stream) {
  if (int rc = check_sys(sys, B)) return (pint_status)rc;
  if ((dtype != PINT_F64 && dtype != PINT_F32) || T < 0 || !std::isfinite(dt))
    return PINT_ERR_INVALID_ARG;
  if (B == 0 || T == 0) return PINT_OK;
  if (!x0 || !traj || !A || !b) return PINT_ERR_INVALID_ARG;
  pint_options o{};
  o.dtype = dtype;
  SolveArgs a = make_args(sys, B, x0, dt, nullptr, T, T, &o, const_cast<void*>(traj), nullptr,
                          nullptr, nullptr, nullptr, 0, stream);
  int rc = is_small(sys->system, sys->d) ? small_elements(a, A, b) : dense_elements(a, A, b);
  return (pint_status)rc;
}

size_t pint_scan_workspace_bytes(int32_t d, int64_t B, int64_t N, int32_t tile, int32_t dtype) {
  return scan_ws_bytes(d, B, N, tile, dtype);
}

pint_status pint_affine_scan(int32_t d, int64_t B, int64_t N, int32_t dtype, const void* A,
                             const void* b, const void* z0, void* z, int32_t tile, void* ws,
                             size_t ws_bytes, pint_stream_t stream) {
  if (d < 1 || B < 0 || N < 0 || tile < 0 || (dtype != PINT_F64 && dtype != PINT_F32))
    return PINT_ERR_INVALID_ARG;
  if (B == 0 || N == 0) return PINT_OK;
  if (!A || !b || !z) return PINT_ERR_INVALID_ARG;
  return (pint_status)affine_scan(d, B, N, dtype, A, b, z0, z, tile, ws, ws_bytes,
                                  reinterpret_cast<hipStream_t>(stream));
}

pint_status pint_affine_scan_noalloc(int32_t d, int64_t B, int64_t N, int32_t dtype,
                                     const void* A, const void* b, const void* z0, void* z,
                                     int32_t tile, uint32_t* err, pint_stream_t stream) {
  if (d < 1 || B < 0 || N < 0 || tile < 0 || (dtype != PINT_F64 && dtype != PINT_F32))
    return PINT_ERR_INVALID_ARG;
  if (B == 0 || N == 0) return PINT_OK;
  if (!A || !b || !z) return PINT_ERR_INVALID_ARG;
  return (pint_status)affine_scan_noalloc(d, B, N, dtype, A, b, z0, z, tile, err,
                                          reinterpret_cast<hipStream_t>(stream));
}

size_t pint_scan_band_workspace_bytes(int32_t d, int32_t bw, int32_t boff, int64_t B, int64_t N,
                                      int32_t tile, int32_t dtype) {
  if (dtype != PINT_F64 && dtype != PINT_F32) return 0;
  return scan_band_ws_bytes(d, bw, boff, B, N, tile, dtype);
}

pint_status pint_affine_scan_band(int32_t d, int32_t bw, int32_t boff, int64_t B, int64_t N,
                                  int32_t dtype, const void* band, const void* b, const void* z0,
                                  void* z, int32_t tile, void* ws, size_t ws_bytes,
                                  pint_stream_t stream) {
  if (d < 1 || bw < 1 || boff < 0 || B < 0 || N < 0 || tile < 0 ||
      (dtype != PINT_F64 && dtype != PINT_F32))
    return PINT_ERR_INVALID_ARG;
  if (B == 0 || N == 0) return PINT_OK;
  if (!band || !b || !z) return PINT_ERR_INVALID_ARG;
  return (pint_status)affine_scan_band(d, bw, boff, B, N, dtype, band, b, z0, z, tile, ws,
                                       ws_bytes, reinterpret_cast<hipStream_t>(stream));
}

size_t pint_adjoint_workspace_bytes(const pint_system* sys, int64_t B, int64_t T, int64_t seg,
                                    int32_t dtype) {
  if (!sys || B < 0 || T < 0 || seg < 0) return 0;
  return adjoint_ws_bytes(sys->system, sys->d, B, T, seg, dtype);
}

pint_status pint_adjoint(const pint_system* sys, int64_t B, const void* x0, double dt, int64_t T,
                         int32_t dtype, const void* traj, const void* g, void* dL_dx0,
                         void* dL_dtheta, int64_t seg, void* ws, size_t ws_bytes,
                         pint_stream_t stream) {
  if (int rc = check_sys(sys, B)) return (pint_status)rc;
  if ((dtype != PINT_F64 && dtype != PINT_F32) || T < 0 || seg < 0 || !std::isfinite(dt))
    return PINT_ERR_INVALID_ARG;
  if (sys->system == PINT_SYS_CARTPOLE && dL_dtheta) return PINT_ERR_UNSUPPORTED;
  if (sys->method != PINT_RK4) return PINT_ERR_UNSUPPORTED;
  if (B == 0) return PINT_OK;
  if (!x0 || !dL_dx0 || (T > 0 && (!traj || !g))) return PINT_ERR_INVALID_ARG;
  pint_options o{};
  o.dtype = dtype;
  SolveArgs a = make_args(sys, B, x0, dt, nullptr, T, T, &o, const_cast<void*>(traj), nullptr,
                          nullptr, nullptr, ws, ws_bytes, stream);
  return (pint_status)adjoint(a, g, dL_dx0, dL_dtheta, seg);
}

}  // extern "C"
