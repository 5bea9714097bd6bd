// Dense state dimension (Lorenz-96 d=40, Kuramoto d=128): one workgroup of
// 512 threads per instance runs the Newton loop of Sec. 3.2 on chip.  Waves
// evaluate RK4 steps (a lane per component), Jacobian columns are built by
// one thread (or a quad) per column from the stage points in LDS and stored
// transposed in the workspace, and the Newton step of the window is the
// affine recursion of eq. newton-step-recursion folded in order inside the
// workgroup (a window is one scan tile).  Instances come from a device work
// queue.  Also the wave-per-instance sequential comparator and the residual
// and element kernels.
#include "internal.h"
#include "systems_dense.h"

namespace pint {

struct DenseKArgs {
  int64_t B;
  const void* x0;
  const void* params;
  int64_t pstride;
  int64_t T_uniform;
  void* traj;
  double dt, tol, guard;
  int64_t window, max_iter;
  int32_t guess;
  int64_t* iters;
  double* resid;
  int32_t* status;
  uint32_t* queue;
  void* ws_elems;        // per workgroup slot: AT [Wt][D][D], b [Wt][D], dx [Wt][D]
  int64_t Wt;            // elements per slot (window length, or T in plain mode)
  int64_t slot_stride;   // scalars between consecutive workgroup slots
};

template <class S>
__host__ __device__ constexpr int64_t slot_scalars(int64_t Wt) {
  return Wt * (int64_t)S::D * S::D + 2 * Wt * (int64_t)S::D;
}

// Load this lane's components of state n (0 -> x0 from LDS).
template <typename T, class S>
__device__ __forceinline__ void wave_load(const T* X, const T* x0s, int64_t n, T (&x)[S::R], int lane) {
#pragma unroll
  for (int r = 0; r < S::R; r++) {
    const int i = lane + 64 * r;
    x[r] = (i < S::D) ? (n == 0 ? x0s[i] : X[(n - 1) * S::D + i]) : T(0);
  }
}

// ||x_n - Phi(x_{n-1})||_inf by one wave.
template <typename T, class S>
__device__ __forceinline__ double wave_resid(const T* P, T dt, const T* X, const T* x0s, int64_t n,
                                             int lane) {
  T xp[S::R], xc[S::R], phi[S::R];
  wave_load<T, S>(X, x0s, n - 1, xp, lane);
  wave_load<T, S>(X, x0s, n, xc, lane);
  wave_rk4<T, S>(P, dt, xp, phi, nullptr, lane);
  double m = 0.0;
#pragma unroll
  for (int r = 0; r < S::R; r++)
    if (lane + 64 * r < S::D) m = acc_norm(m, xc[r] - phi[r]);
  return wave_max(m);
}

template <typename T, class S>
__global__ __launch_bounds__(S::NT) void k_newton_dense(DenseKArgs a) {
  constexpr int D = S::D, NP = S::NP, NT = S::NT, NW = NT / PINT_WAVE;
  constexpr int SPP = S::SPP, JT = S::JT;
  // recursion: QC adjacent threads per row, D*QC <= NT
  constexpr int QC = (D * 4 <= NT && D % 4 == 0) ? 4 : ((D * 2 <= NT && D % 2 == 0) ? 2 : 1);
  constexpr int JC = D / QC;
  static_assert(D * QC <= NT, "row split");
  __shared__ typename S::Stage s_stage[SPP];
  __shared__ T s_P[NP], s_x0[D], s_z[2][D];
  __shared__ double s_red[NW];
  __shared__ int64_t s_redi[NW];
  __shared__ double s_wres[NW];
  __shared__ uint32_t s_slot;
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  const T dt = (T)a.dt;
  T* slot = static_cast<T*>(a.ws_elems) + (int64_t)blockIdx.x * a.slot_stride;
  T* AT = slot;
  T* bb = AT + a.Wt * D * D;
  T* dxb = bb + a.Wt * D;

  for (;;) {
    if (tid == 0) s_slot = atomicAdd(a.queue, 1u);
    __syncthreads();
    const int64_t inst = s_slot;
    __syncthreads();
    if (inst >= a.B) break;
    const int64_t Tn = a.T_uniform;
    T* X = static_cast<T*>(a.traj) + inst * Tn * D;
    {
      const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
      for (int i = tid; i < NP; i += NT) s_P[i] = Pg[i];
      const T* xg = static_cast<const T*>(a.x0) + inst * D;
      for (int i = tid; i < D; i += NT) s_x0[i] = xg[i];
    }
    __syncthreads();
    if (a.guess == 0)
      for (int64_t idx = tid; idx < Tn * D; idx += NT) X[idx] = s_x0[idx % D];
    __syncthreads();

    const bool plain = (a.window <= 0);
    const int64_t W = a.window;
    int64_t k = 0, p = 1;
    int st = ST_OK;
    while (Tn > 0) {
      int64_t lo, hi;
      if (plain) {
        double r = 0.0;
        for (int64_t n = 1 + wv; n <= Tn; n += NW) r = fmax(r, wave_resid<T, S>(s_P, dt, X, s_x0, n, lane));
        r = block_max<NT>(r, s_red);
        if (!(r < INFINITY)) { st = ST_NONFINITE; break; }
        if (r < a.tol) { st = ST_OK; break; }
        if (k >= a.max_iter) { st = ST_NOT_CONVERGED; break; }
        lo = 1;
        hi = Tn;
      } else {
        int64_t fv = INT64_MAX;
        double hp = 0.0;
        for (int64_t c0 = p; c0 <= Tn; c0 += NW) {
          const int64_t n = c0 + wv;
          int64_t v = INT64_MAX;
          double hn = 0.0;
          if (n <= Tn) {
            hn = wave_resid<T, S>(s_P, dt, X, s_x0, n, lane);
            if (!(hn < a.tol)) v = n;
          }
          if (lane == 0) s_wres[wv] = hn;
          fv = block_min_i64<NT>(v, s_redi);
          if (fv != INT64_MAX) {
            hp = s_wres[fv - c0];
            break;
          }
        }
        if (fv == INT64_MAX) { st = ST_OK; break; }
        p = fv;
        if (!(hp < INFINITY)) { st = ST_NONFINITE; break; }
        if (k >= a.max_iter) { st = ST_NOT_CONVERGED; break; }
        lo = p;
        hi = (W >= Tn - p + 1) ? Tn : p + W - 1;
      }
      const int64_t len = hi - lo + 1;

      // Elements of the window: e_m = (J(x_{lo+m-1}), Phi(x_{lo+m-1}) - x_{lo+m}).
      for (int64_t m0 = 0; m0 < len; m0 += SPP) {
        for (int sl = wv; sl < SPP; sl += NW) {
          const int64_t m = m0 + sl;
          if (m < len) {
            const int64_t n = lo + m;
            T xp[S::R], xc[S::R], phi[S::R];
            wave_load<T, S>(X, s_x0, n - 1, xp, lane);
            wave_load<T, S>(X, s_x0, n, xc, lane);
            wave_rk4<T, S>(s_P, dt, xp, phi, &s_stage[sl], lane);
#pragma unroll
            for (int r = 0; r < S::R; r++) {
              const int i = lane + 64 * r;
              if (i < D) bb[m * D + i] = phi[r] - xc[r];
            }
          }
        }
        __syncthreads();
        for (int t = tid; t < SPP * JT; t += NT) {
          const int sl = t / JT, sub = t % JT;
          const int64_t m = m0 + sl;
          if (m < len) S::jac_thread(&s_stage[sl], s_P, sub, dt, AT + m * D * D, 1, D);
        }
        __syncthreads();
      }

      // Newton step over the window: dx_{lo} = b_0, dx_{lo+m} = J dx + b_m.
      {
        const bool cth = tid < D * QC;
        const int ri = tid / QC, rq = tid % QC;
        if (tid < D) s_z[0][tid] = T(0);
        __syncthreads();
        // rows of the next element are prefetched into registers when they
        // fit (JC <= 16); otherwise read in the dot loop
        constexpr bool PF = JC <= 16;
        T an[PF ? JC : 1];
        if (PF && cth && len > 1)
#pragma unroll
          for (int jj = 0; jj < (PF ? JC : 1); jj++) an[jj] = AT[(int64_t)D * D + (int64_t)(rq * JC + jj) * D + ri];
        int cur = 0;
        for (int64_t m = 0; m < len; m++) {
          T part = T(0);
          if (cth && m > 0) {
            if constexpr (PF) {
#pragma unroll
              for (int jj = 0; jj < JC; jj++) part += an[jj] * s_z[cur][rq * JC + jj];
              if (m + 1 < len) {
                const T* An = AT + (m + 1) * D * D;
#pragma unroll
                for (int jj = 0; jj < JC; jj++) an[jj] = An[(int64_t)(rq * JC + jj) * D + ri];
              }
            } else {
              const T* Am = AT + m * D * D;
#pragma unroll 16
              for (int jj = 0; jj < JC; jj++) part += Am[(int64_t)(rq * JC + jj) * D + ri] * s_z[cur][rq * JC + jj];
            }
          }
#pragma unroll
          for (int off = 1; off < QC; off <<= 1) part += __shfl_xor(part, off, PINT_WAVE);
          if (cth && rq == 0) {
            const T z = part + bb[m * D + ri];
            s_z[cur ^ 1][ri] = z;
            dxb[m * D + ri] = z;
          }
          __syncthreads();
          cur ^= 1;
        }
      }

      // Accept below the first non-finite / out-of-guard updated state.
      int64_t q = INT64_MAX;
      if (!plain) {
        int64_t v = INT64_MAX;
        for (int64_t m = tid; m < len; m += NT) {
          bool bad = false;
          for (int i = 0; i < D; i++) {
            const T xn = X[(lo + m - 1) * D + i] + dxb[m * D + i];
            bad = bad || !finite_(xn) || fabs((double)xn) > a.guard;
          }
          if (bad) { v = lo + m; break; }
        }
        q = block_min_i64<NT>(v, s_redi);
      }
      for (int64_t idx = tid; idx < len * D; idx += NT) {
        const int64_t m = idx / D;
        if (lo + m < q) X[(lo - 1) * D + idx] += dxb[idx];
      }
      __syncthreads();
      if (q == lo) { st = ST_NONFINITE; break; }
      k++;
    }
    __syncthreads();
    double r = 0.0;
    for (int64_t n = 1 + wv; n <= Tn; n += NW) r = fmax(r, wave_resid<T, S>(s_P, dt, X, s_x0, n, lane));
    r = block_max<NT>(r, s_red);
    if (tid == 0) {
      a.iters[inst] = k;
      a.resid[inst] = r;
      a.status[inst] = st;
    }
    __syncthreads();
  }
}

// Sequential comparator: one wave per instance.
template <typename T, class S>
__global__ __launch_bounds__(64) void k_seq_dense(DenseKArgs a, const int64_t* T_off) {
  constexpr int D = S::D, NP = S::NP, R = S::R;
  __shared__ T s_P[NP];
  const int64_t inst = blockIdx.x;
  const int lane = threadIdx.x;
  const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
  for (int i = lane; i < NP; i += 64) s_P[i] = Pg[i];
  __syncthreads();
  const int64_t t0 = T_off ? T_off[inst] : inst * a.T_uniform;
  const int64_t Tn = (T_off ? T_off[inst + 1] : t0 + a.T_uniform) - t0;
  T* X = static_cast<T*>(a.traj) + t0 * D;
  const T* xg = static_cast<const T*>(a.x0) + inst * D;
  T x[R], y[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int i = lane + 64 * r;
    x[r] = i < D ? xg[i] : T(0);
  }
  const T dt = (T)a.dt;
  for (int64_t n = 0; n < Tn; n++) {
    wave_rk4<T, S>(s_P, dt, x, y, nullptr, lane);
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int i = lane + 64 * r;
      x[r] = y[r];
      if (i < D) X[n * D + i] = y[r];
    }
  }
}

// Residual of every step of a uniform batch: one wave per step.
template <typename T, class S>
__global__ __launch_bounds__(256) void k_residual_dense(DenseKArgs a, T* h, double* hmax) {
  constexpr int D = S::D, NP = S::NP, R = S::R;
  const int lane = threadIdx.x % 64;
  const int64_t g = blockIdx.x * 4 + threadIdx.x / 64;
  if (g >= a.B * a.T_uniform) return;
  const int64_t inst = g / a.T_uniform, n = g % a.T_uniform + 1;
  const T* P = static_cast<const T*>(a.params) + inst * a.pstride;
  const T* X = static_cast<const T*>(a.traj) + inst * a.T_uniform * D;
  const T* x0 = static_cast<const T*>(a.x0) + inst * D;
  T xp[R], phi[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int i = lane + 64 * r;
    xp[r] = i < D ? (n == 1 ? x0[i] : X[(n - 2) * D + i]) : T(0);
  }
  (void)NP;
  wave_rk4<T, S>(P, (T)a.dt, xp, phi, nullptr, lane);
  double m = 0.0;
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int i = lane + 64 * r;
    if (i < D) {
      const T v = X[(n - 1) * D + i] - phi[r];
      if (h) h[(inst * a.T_uniform + n - 1) * D + i] = v;
      m = acc_norm(m, v);
    }
  }
  m = wave_max(m);
  if (lane == 0) atomic_max_nonneg(hmax + inst, m);
}

// Elements A_n = dPhi/dx(x_n) (row-major), b_n = Phi(x_n) - x_{n+1}.
template <typename T, class S>
__global__ __launch_bounds__(S::NT) void k_elements_dense(DenseKArgs a, T* A, T* b) {
  constexpr int D = S::D, NP = S::NP, NT = S::NT, NW = NT / PINT_WAVE, SPP = S::SPP, JT = S::JT;
  __shared__ typename S::Stage s_stage[SPP];
  __shared__ T s_P[SPP][NP];
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int64_t total = a.B * a.T_uniform;
  const int64_t g0 = (int64_t)blockIdx.x * SPP;
  for (int sl = 0; sl < SPP; sl++) {
    const int64_t g = g0 + sl;
    if (g < total) {
      const T* P = static_cast<const T*>(a.params) + (g / a.T_uniform) * a.pstride;
      for (int i = tid; i < NP; i += NT) s_P[sl][i] = P[i];
    }
  }
  __syncthreads();
  for (int sl = wv; sl < SPP; sl += NW) {
    const int64_t g = g0 + sl;
    if (g >= total) continue;
    const int64_t inst = g / a.T_uniform, n = g % a.T_uniform;
    const T* X = static_cast<const T*>(a.traj) + inst * a.T_uniform * D;
    const T* x0 = static_cast<const T*>(a.x0) + inst * D;
    T xp[S::R], phi[S::R];
#pragma unroll
    for (int r = 0; r < S::R; r++) {
      const int i = lane + 64 * r;
      xp[r] = i < D ? (n == 0 ? x0[i] : X[(n - 1) * D + i]) : T(0);
    }
    wave_rk4<T, S>(s_P[sl], (T)a.dt, xp, phi, &s_stage[sl], lane);
#pragma unroll
    for (int r = 0; r < S::R; r++) {
      const int i = lane + 64 * r;
      if (i < D) b[g * D + i] = phi[r] - X[n * D + i];
    }
  }
  __syncthreads();
  for (int t = tid; t < SPP * JT; t += NT) {
    const int sl = t / JT, sub = t % JT;
    const int64_t g = g0 + sl;
    if (g < total) S::jac_thread(&s_stage[sl], s_P[sl], sub, (T)a.dt, A + g * D * D, D, 1);
  }
}

// ------------------------------------------------------------- dispatch --

template <typename T, typename F>
static int dispatch_dense_sys(int system, int d, F&& f) {
  if (system == 5 && d == 40) return f(DSysL96<T, 40>{});
  if (system == 6 && d == 128) return f(DSysKur<T, 128>{});
  if (system == 6 && d == 64) return f(DSysKur<T, 64>{});
  return ST_UNSUPPORTED;
}

template <typename F>
static int dispatch_dense(int dtype, int system, int d, F&& f) {
  if (dtype == 0) return dispatch_dense_sys<double>(system, d, [&](auto s) { return f((double)0, s); });
  if (dtype == 1) return dispatch_dense_sys<float>(system, d, [&](auto s) { return f((float)0, s); });
  return ST_UNSUPPORTED;
}

bool dense_supported(int system, int d) {
  return dispatch_dense(0, system, d, [](auto, auto) { return ST_OK; }) == ST_OK;
}

static DenseKArgs to_dk(const SolveArgs& a) {
  DenseKArgs k{};
  k.B = a.B;
  k.x0 = a.x0;
  k.params = a.params;
  k.pstride = a.pstride;
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
  return k;
}

static int num_cus() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus;
}

// Workgroups for the persistent dense solver: one per instance, at most one
// per compute unit.
static int dense_grid(int64_t B) {
  const int64_t cu = num_cus();
  return (int)(B < cu ? B : cu);
}

static int64_t dense_Wt(const SolveArgs& a) {
  const int64_t T = a.T_uniform;
  return (a.window <= 0 || a.window >= T) ? T : a.window;
}

size_t dense_ws_bytes(const SolveArgs& a) {
  size_t per = 0;
  dispatch_dense(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    per = (size_t)slot_scalars<S>(dense_Wt(a) > 0 ? dense_Wt(a) : 1) * sizeof(T);
    return ST_OK;
  });
  return 256 + align_up(per) * (size_t)(dense_grid(a.B > 0 ? a.B : 1));
}

int dense_solve(const SolveArgs& a) {
  if (!a.ws || a.ws_bytes < dense_ws_bytes(a)) return ST_WORKSPACE;
  DenseKArgs k = to_dk(a);
  k.queue = static_cast<uint32_t*>(a.ws);
  k.ws_elems = static_cast<char*>(a.ws) + 256;
  k.Wt = dense_Wt(a);
  if (int rc = fill_u32(k.queue, 1, 0u, a.stream)) return rc;
  const int grid = dense_grid(a.B);
  return dispatch_dense(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    k.slot_stride = (int64_t)(align_up((size_t)slot_scalars<S>(k.Wt > 0 ? k.Wt : 1) * sizeof(T)) /
                              sizeof(T));
    hipLaunchKernelGGL((k_newton_dense<T, S>), dim3(grid), dim3(S::NT), 0, a.stream, k);
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

int dense_seq(const SolveArgs& a) {
  DenseKArgs k = to_dk(a);
  if (a.B <= 0) return ST_OK;
  return dispatch_dense(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    hipLaunchKernelGGL((k_seq_dense<T, S>), dim3(a.B), dim3(64), 0, a.stream, k, a.T_off);
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

int dense_residual(const SolveArgs& a, void* h, double* hmax) {
  DenseKArgs k = to_dk(a);
  if (int rc = fill_u32(reinterpret_cast<uint32_t*>(hmax), (size_t)a.B * 2, 0u, a.stream)) return rc;
  const int64_t total = a.B * a.T_uniform;
  if (total <= 0) return ST_OK;
  return dispatch_dense(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    hipLaunchKernelGGL((k_residual_dense<T, S>), dim3((total + 3) / 4), dim3(256), 0, a.stream, k,
                       static_cast<T*>(h), hmax);
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

int dense_elements(const SolveArgs& a, void* A, void* b) {
  DenseKArgs k = to_dk(a);
  const int64_t total = a.B * a.T_uniform;
  if (total <= 0) return ST_OK;
  return dispatch_dense(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    const int64_t grid = (total + S::SPP - 1) / S::SPP;
    hipLaunchKernelGGL((k_elements_dense<T, S>), dim3(grid), dim3(S::NT), 0, a.stream, k,
                       static_cast<T*>(A), static_cast<T*>(b));
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

}  // namespace pint
