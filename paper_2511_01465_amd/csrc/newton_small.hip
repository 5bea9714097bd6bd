// Small state dimension (d <= 4): one workgroup per instance runs the whole
// Newton loop of Sec. 3.2 on chip — residual, stop test, window search,
// element construction, affine scan and update — pulling instances from a
// device work queue, so a batch of any size and mix of horizons is one
// persistent launch.  Also the sequential RK4 comparator and the residual /
// element kernels used for checking.
#include "internal.h"
#include "systems_small.h"

namespace pint {

// Threads per workgroup = steps per chunk of the in-workgroup scan: 64, 128
// or 256 (a launch-shape choice; results do not depend on it).
constexpr int NT_SMALL = 256;

struct SmallKArgs {
  int64_t B;
  const void* x0;
  const void* params;
  int64_t pstride;
  const int64_t* T_off;
  int64_t T_uniform;
  void* traj;
  double dt, tol, guard;
  int64_t window, max_iter;
  int32_t guess;
  int64_t* iters;
  double* resid;
  int32_t* status;
  uint32_t* queue;
  const int64_t* order;  // [B] instance taken at each queue slot, or nullptr
};

template <typename T, int D>
__device__ __forceinline__ void load_state(const T* X, const T* x0, int64_t n, T* out) {
  if (n == 0) {
#pragma unroll
    for (int i = 0; i < D; i++) out[i] = x0[i];
  } else {
#pragma unroll
    for (int i = 0; i < D; i++) out[i] = X[(n - 1) * D + i];
  }
}

// ||h_n||_inf = ||x_n - Phi(x_{n-1})||_inf (eq. root-finding-problem),
// +inf if anything is non-finite.
template <typename T, class S>
__device__ __forceinline__ double step_resid(const T* P, T dt, const T* X, const T* x0, int64_t n) {
  constexpr int D = S::D;
  T xp[D], xc[D], phi[D];
  load_state<T, D>(X, x0, n - 1, xp);
  load_state<T, D>(X, x0, n, xc);
  rk4_phi<T, S>(P, dt, xp, phi);
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < D; i++) m = acc_norm(m, xc[i] - phi[i]);
  return m;
}

template <typename T, class S, int NT>
__global__ __launch_bounds__(NT) void k_newton_small(SmallKArgs a) {
  constexpr int D = S::D, NP = S::NP;
  __shared__ Aff<T, D> s_aff[NT / PINT_WAVE];
  __shared__ double s_red[NT / PINT_WAVE];
  __shared__ int64_t s_redi[NT / PINT_WAVE];
  __shared__ T s_z[D], s_xprev[D], s_xlast[D], s_zlast[D];
  __shared__ uint32_t s_slot;
  __shared__ double s_hp;
  const int tid = threadIdx.x;
  const T dt = (T)a.dt;

  for (;;) {
    if (tid == 0) s_slot = atomicAdd(a.queue, 1u);
    __syncthreads();
    const int64_t slot = s_slot;
    __syncthreads();
    if (slot >= a.B) break;
    const int64_t inst = a.order ? a.order[slot] : slot;
    if (inst < 0 || inst >= a.B) continue;  // not a permutation entry: skipped

    const int64_t t0 = a.T_off ? a.T_off[inst] : inst * a.T_uniform;
    const int64_t Tn = (a.T_off ? a.T_off[inst + 1] : t0 + a.T_uniform) - t0;
    T* X = static_cast<T*>(a.traj) + t0 * D;
    T P[NP], x0[D];
    {
      const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
#pragma unroll
      for (int i = 0; i < NP; i++) P[i] = Pg[i];
      const T* xg = static_cast<const T*>(a.x0) + inst * D;
#pragma unroll
      for (int i = 0; i < D; i++) x0[i] = xg[i];
    }
    if (a.guess == 0)
      for (int64_t n = tid; n < Tn; n += NT)
#pragma unroll
        for (int i = 0; i < D; i++) X[n * D + i] = x0[i];
    __syncthreads();

    const bool plain = (a.window <= 0);
    const int64_t W = a.window;
    int64_t k = 0, p = 1;
    int st = ST_OK;
    while (Tn > 0) {
      int64_t lo, hi;
      if (plain) {
        double r = 0.0;
        for (int64_t c0 = 1; c0 <= Tn; c0 += NT) {
          const int64_t n = c0 + tid;
          if (n <= Tn) r = fmax(r, step_resid<T, S>(P, dt, X, x0, n));
        }
        r = block_max<NT>(r, s_red);
        if (!(r < INFINITY)) { st = ST_NONFINITE; break; }
        if (r < a.tol) { st = ST_OK; break; }
        if (k >= a.max_iter) { st = ST_NOT_CONVERGED; break; }
        lo = 1;
        hi = Tn;
      } else {
        // first violation at or after p; steps before p are untouched
        int64_t fv = INT64_MAX;
        for (int64_t c0 = p; c0 <= Tn; c0 += NT) {
          const int64_t n = c0 + tid;
          int64_t v = INT64_MAX;
          double hn = 0.0;
          if (n <= Tn) {
            hn = step_resid<T, S>(P, dt, X, x0, n);
            if (!(hn < a.tol)) v = n;
          }
          fv = block_min_i64<NT>(v, s_redi);
          if (fv != INT64_MAX) {
            if (n == fv) s_hp = hn;
            break;
          }
        }
        __syncthreads();
        if (fv == INT64_MAX) { st = ST_OK; break; }
        p = fv;
        const double hp = s_hp;
        if (!(hp < INFINITY)) { st = ST_NONFINITE; break; }
        if (k >= a.max_iter) { st = ST_NOT_CONVERGED; break; }
        lo = p;
        hi = (W >= Tn - p + 1) ? Tn : p + W - 1;
      }

      // Newton step over [lo, hi] (eq. newton-step-recursion): the elements
      // (J(x_{n-1}), -h_n) are scanned chunk by chunk, dx_lo = -h_lo.
      if (tid < D) {
        s_z[tid] = T(0);
        s_xprev[tid] = (lo == 1) ? x0[tid] : X[(lo - 2) * D + tid];
      }
      __syncthreads();
      int64_t qcut = INT64_MAX;
      for (int64_t c0 = lo; c0 <= hi; c0 += NT) {
        const int64_t n = c0 + tid;
        const bool act = n <= hi;
        T xc[D];
        Aff<T, D> e;
        if (act) {
          T xp[D], phi[D];
          if (tid == 0) {
#pragma unroll
            for (int i = 0; i < D; i++) xp[i] = s_xprev[i];
          } else {
#pragma unroll
            for (int i = 0; i < D; i++) xp[i] = X[(n - 2) * D + i];
          }
#pragma unroll
          for (int i = 0; i < D; i++) xc[i] = X[(n - 1) * D + i];
          rk4_phi_jac<T, S>(P, dt, xp, phi, e.A);
#pragma unroll
          for (int i = 0; i < D; i++) e.b[i] = phi[i] - xc[i];
        } else {
          aff_identity(e);
#pragma unroll
          for (int i = 0; i < D; i++) xc[i] = T(0);
        }
        block_scan_aff<T, D, NT>(e, s_aff);
        T dx[D], xn[D];
        bool bad = false;
#pragma unroll
        for (int i = 0; i < D; i++) {
          T acc = e.b[i];
#pragma unroll
          for (int j = 0; j < D; j++) acc += e.A[i * D + j] * s_z[j];
          dx[i] = acc;
          xn[i] = xc[i] + acc;
          bad = bad || !finite_(xn[i]) || fabs((double)xn[i]) > a.guard;
        }
        int64_t q = INT64_MAX;
        if (!plain) q = block_min_i64<NT>((act && bad) ? n : INT64_MAX, s_redi);
        const int64_t last = (hi < c0 + NT - 1) ? hi : c0 + NT - 1;
        if (n == last) {
#pragma unroll
          for (int i = 0; i < D; i++) { s_xlast[i] = xc[i]; s_zlast[i] = dx[i]; }
        }
        if (act && n < q) {
#pragma unroll
          for (int i = 0; i < D; i++) X[(n - 1) * D + i] = xn[i];
        }
        __syncthreads();
        if (q != INT64_MAX) { qcut = q; break; }
        if (tid < D) { s_xprev[tid] = s_xlast[tid]; s_z[tid] = s_zlast[tid]; }
        __syncthreads();
      }
      if (qcut == lo) { st = ST_NONFINITE; break; }
      k++;
    }
    __syncthreads();
    double r = 0.0;
    for (int64_t n = 1 + tid; n <= Tn; n += NT) r = fmax(r, step_resid<T, S>(P, dt, X, x0, n));
    r = block_max<NT>(r, s_red);
    if (tid == 0) {
      a.iters[inst] = k;
      a.resid[inst] = r;
      a.status[inst] = st;
    }
    __syncthreads();
  }
}

// Sequential comparator: one thread per instance, x_n = Phi(x_{n-1}).
template <typename T, class S>
__global__ void k_seq_small(SmallKArgs a) {
  constexpr int D = S::D, NP = S::NP;
  const int64_t inst = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (inst >= a.B) return;
  const int64_t t0 = a.T_off ? a.T_off[inst] : inst * a.T_uniform;
  const int64_t Tn = (a.T_off ? a.T_off[inst + 1] : t0 + a.T_uniform) - t0;
  T* X = static_cast<T*>(a.traj) + t0 * D;
  T P[NP], x[D], y[D];
  const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
#pragma unroll
  for (int i = 0; i < NP; i++) P[i] = Pg[i];
  const T* xg = static_cast<const T*>(a.x0) + inst * D;
#pragma unroll
  for (int i = 0; i < D; i++) x[i] = xg[i];
  const T dt = (T)a.dt;
  for (int64_t n = 0; n < Tn; n++) {
    rk4_phi<T, S>(P, dt, x, y);
#pragma unroll
    for (int i = 0; i < D; i++) {
      x[i] = y[i];
      X[n * D + i] = y[i];
    }
  }
}

// h_n for every (instance, step) of a uniform batch, and per-instance max.
template <typename T, class S>
__global__ void k_residual_small(SmallKArgs a, T* h, double* hmax) {
  constexpr int D = S::D, NP = S::NP;
  const int64_t total = a.B * a.T_uniform;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t inst = g / a.T_uniform, n = g % a.T_uniform + 1;
    const T* X = static_cast<const T*>(a.traj) + inst * a.T_uniform * D;
    const T* x0 = static_cast<const T*>(a.x0) + inst * D;
    T P[NP], xp[D], phi[D];
    const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
#pragma unroll
    for (int i = 0; i < NP; i++) P[i] = Pg[i];
    load_state<T, D>(X, x0, n - 1, xp);
    rk4_phi<T, S>(P, (T)a.dt, xp, phi);
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < D; i++) {
      const T v = X[(n - 1) * D + i] - phi[i];
      if (h) h[g * D + i] = v;
      m = acc_norm(m, v);
    }
    atomic_max_nonneg(hmax + inst, m);
  }
}

// Elements (A_n, b_n) = (dPhi/dx(x_n), -h_{n+1}), n = 0..T-1.
template <typename T, class S>
__global__ void k_elements_small(SmallKArgs a, T* A, T* b) {
  constexpr int D = S::D, NP = S::NP;
  const int64_t total = a.B * a.T_uniform;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t inst = g / a.T_uniform, n = g % a.T_uniform;
    const T* X = static_cast<const T*>(a.traj) + inst * a.T_uniform * D;
    const T* x0 = static_cast<const T*>(a.x0) + inst * D;
    T P[NP], xn[D], phi[D], J[D * D];
    const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
#pragma unroll
    for (int i = 0; i < NP; i++) P[i] = Pg[i];
    load_state<T, D>(X, x0, n, xn);
    rk4_phi_jac<T, S>(P, (T)a.dt, xn, phi, J);
#pragma unroll
    for (int i = 0; i < D * D; i++) A[g * D * D + i] = J[i];
#pragma unroll
    for (int i = 0; i < D; i++) b[g * D + i] = phi[i] - X[n * D + i];
  }
}

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

int fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return ST_OK;
  const int blocks = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
}

// ------------------------------------------------------------- dispatch --

template <typename T, typename F>
static int dispatch_small_sys(int system, int d, F&& f) {
  switch (system) {
    case 0:
      switch (d) {
        case 1: return f(SysLinear<T, 1>{});
        case 2: return f(SysLinear<T, 2>{});
        case 3: return f(SysLinear<T, 3>{});
        case 4: return f(SysLinear<T, 4>{});
      }
      break;
    case 1: if (d == 1) return f(SysLogistic<T>{}); break;
    case 2: if (d == 2) return f(SysVdP<T>{}); break;
    case 3: if (d == 4) return f(SysCartPole<T>{}); break;
    case 4: if (d == 3) return f(SysLorenz63<T>{}); break;
  }
  return ST_UNSUPPORTED;
}

template <typename F>
static int dispatch_small(int dtype, int system, int d, F&& f) {
  if (dtype == 0) return dispatch_small_sys<double>(system, d, [&](auto s) { return f((double)0, s); });
  if (dtype == 1) return dispatch_small_sys<float>(system, d, [&](auto s) { return f((float)0, s); });
  return ST_UNSUPPORTED;
}

bool small_supported(int system, int d) {
  return dispatch_small(0, system, d, [](auto, auto) { return ST_OK; }) == ST_OK;
}

static SmallKArgs to_k(const SolveArgs& a) {
  SmallKArgs k{};
  k.B = a.B;
  k.x0 = a.x0;
  k.params = a.params;
  k.pstride = a.pstride;
  k.T_off = a.T_off;
  k.T_uniform = a.T_uniform;
  k.traj = a.traj;
  k.dt = a.dt;
  k.tol = a.tol;
  k.guard = a.guard;
  k.window = a.window;
  k.max_iter = a.max_iter;
  k.guess = a.guess;
  k.iters = a.iters;
  k.resid = a.resid;
  k.status = a.status;
  k.order = a.order;
  return k;
}

size_t small_ws_bytes(int64_t) { return 256; }

int small_solve(const SolveArgs& a) {
  if (a.ws_bytes < small_ws_bytes(a.B) || a.ws == nullptr) return ST_WORKSPACE;
  SmallKArgs k = to_k(a);
  k.queue = static_cast<uint32_t*>(a.ws);
  if (int rc = fill_u32(k.queue, 1, 0u, a.stream)) return rc;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t want = (int64_t)cus * (a.wg_per_cu > 0 ? a.wg_per_cu : 4);
  const int grid = (int)(a.B < want ? a.B : want);
  if (grid <= 0) return ST_OK;
  const int nt = a.block > 0 ? a.block : NT_SMALL;
  return dispatch_small(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    switch (nt) {
      case 64: hipLaunchKernelGGL((k_newton_small<T, S, 64>), dim3(grid), dim3(64), 0, a.stream, k); break;
      case 128: hipLaunchKernelGGL((k_newton_small<T, S, 128>), dim3(grid), dim3(128), 0, a.stream, k); break;
      case 256: hipLaunchKernelGGL((k_newton_small<T, S, 256>), dim3(grid), dim3(256), 0, a.stream, k); break;
      default: return (int)ST_INVALID;
    }
    return hipGetLastError() == hipSuccess ? (int)ST_OK : (int)ST_DEVICE;
  });
}

int small_seq(const SolveArgs& a) {
  SmallKArgs k = to_k(a);
  if (a.B <= 0) return ST_OK;
  const int grid = (int)((a.B + 63) / 64);
  return dispatch_small(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    hipLaunchKernelGGL((k_seq_small<T, S>), dim3(grid), dim3(64), 0, a.stream, k);
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

int small_residual(const SolveArgs& a, void* h, double* hmax) {
  SmallKArgs k = to_k(a);
  if (int rc = fill_u32(reinterpret_cast<uint32_t*>(hmax), (size_t)a.B * 2, 0u, a.stream)) return rc;
  const int64_t total = a.B * a.T_uniform;
  if (total <= 0) return ST_OK;
  const int grid = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  return dispatch_small(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    hipLaunchKernelGGL((k_residual_small<T, S>), dim3(grid), dim3(256), 0, a.stream, k,
                       static_cast<T*>(h), hmax);
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

int small_elements(const SolveArgs& a, void* A, void* b) {
  SmallKArgs k = to_k(a);
  const int64_t total = a.B * a.T_uniform;
  if (total <= 0) return ST_OK;
  const int grid = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  return dispatch_small(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    hipLaunchKernelGGL((k_elements_small<T, S>), dim3(grid), dim3(256), 0, a.stream, k,
                       static_cast<T*>(A), static_cast<T*>(b));
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

}  // namespace pint
