// Parareal (Sec. 2.2, eqs. parareal-init, fine-integrator,
// coarse-integrator), the method the paper compares against, for systems of
// small dimension (d <= 4) and every one-step rule of the small solver.
//
// One workgroup per instance.  The M windows are spread over the threads
// (thread t owns windows t, t + NT, ...): the fine sweep runs the S steps of
// each window in registers and writes the dense trajectory; the error
// R = max_m |x_{m+1} - F_m| is a block reduction; the coarse correction sweep
// is sequential over the windows, so one thread runs it while the others
// wait at the next barrier.  The iterate x_m, the fine end states F_m and the
// previous coarse values G(x_m) live in the caller's workspace, one block per
// instance; threads of the workgroup exchange them through global memory
// ordered by workgroup barriers (they share the CU's vector cache).
#include "newton_small.h"

namespace pint {

struct PararealKArgs {
  int64_t B, M, S, max_iter;
  const void* x0;
  const void* params;
  int64_t pstride;
  void* traj;      // [B][M*S][D]
  double dt, tol;
  int64_t* iters;  // [B] fine sweeps K
  double* resid;   // [B] last R
  int32_t* status; // [B]
  double* hist;    // [B][max_iter] or nullptr
  void* ws;        // [B][(3M+1)][D]: x_0..x_M, F_0..F_{M-1}, G_0..G_{M-1}
};

template <typename T, class Sys, int Meth, int NT>
__global__ __launch_bounds__(NT) void k_parareal_small(PararealKArgs a) {
  constexpr int D = Sys::D, NP = Sys::NP;
  using Rule = StepRule<T, Sys, Meth>;
  __shared__ double red[NT / PINT_WAVE];
  const int64_t inst = blockIdx.x;
  if (inst >= a.B) return;
  const int tid = threadIdx.x;
  const int64_t M = a.M, S = a.S;
  if (M <= 0 || S <= 0) {
    if (tid == 0) {
      a.iters[inst] = 0;
      a.resid[inst] = 0.0;
      a.status[inst] = ST_OK;
    }
    return;
  }
  T P[NP];
  const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
#pragma unroll
  for (int i = 0; i < NP; i++) P[i] = Pg[i];
  T* X = static_cast<T*>(a.ws) + inst * (3 * M + 1) * D;
  T* F = X + (M + 1) * D;
  T* G = F + M * D;
  T* traj = static_cast<T*>(a.traj) + inst * M * S * D;
  const T* x0 = static_cast<const T*>(a.x0) + inst * D;
  const T dt = (T)a.dt;
  const T H = (T)((double)S * a.dt);  // the coarse step spans one window

  // A step of an implicit rule whose Newton solve does not converge stops
  // the instance with NONFINITE: in the initial sweep with K = 0, in a fine
  // sweep before that sweep's R counts, in a correction sweep after it.
  __shared__ int s_bad;
  // eq. parareal-init: x_{m+1} = G(x_m), kept as G_m^(0) too
  if (tid == 0) {
    T x[D];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < D; i++) { x[i] = x0[i]; X[i] = x[i]; }
    for (int64_t m = 0; m < M && ok; m++) {
      T g[D];
      ok = Rule::advance_ok(P, H, x, g);
#pragma unroll
      for (int i = 0; i < D; i++) {
        G[m * D + i] = g[i];
        X[(m + 1) * D + i] = g[i];
        x[i] = g[i];
      }
    }
    s_bad = ok ? 0 : 1;
  }
  __syncthreads();

  int64_t k = 0;
  double R = 0.0;
  int st = s_bad ? ST_NONFINITE : ST_OK;
  while (st == ST_OK) {
    // eq. fine-integrator: every window from its own start, S fine steps
    double emax = 0.0;
    int bad = 0;
    for (int64_t m = tid; m < M; m += NT) {
      T y[D];
#pragma unroll
      for (int i = 0; i < D; i++) y[i] = X[m * D + i];
      T* out = traj + m * S * D;
      for (int64_t j = 0; j < S; j++) {
        T z[D];
        bad |= Rule::advance_ok(P, dt, y, z) ? 0 : 1;
#pragma unroll
        for (int i = 0; i < D; i++) {
          out[j * D + i] = z[i];
          y[i] = z[i];
        }
      }
#pragma unroll
      for (int i = 0; i < D; i++) {
        F[m * D + i] = y[i];
        emax = acc_norm(emax, X[(m + 1) * D + i] - y[i]);
      }
    }
    if (__syncthreads_or(bad)) { st = ST_NONFINITE; break; }
    const double Rk = block_max<NT>(emax, red);  // also orders the F stores before the coarse sweep
    R = Rk;
    if (a.hist && tid == 0) a.hist[inst * a.max_iter + k] = R;
    k++;
    if (!(R <= 1.79769313486231570e308)) { st = ST_NONFINITE; break; }
    if (R < a.tol) break;
    if (k >= a.max_iter) { st = ST_NOT_CONVERGED; break; }
    // eq. coarse-integrator: x_{m+1} <- G(x_m new) + F_m - G(x_m old), in order
    if (tid == 0) {
      T x[D], fn[D], gn[D];
#pragma unroll
      for (int i = 0; i < D; i++) { x[i] = x0[i]; fn[i] = F[i]; gn[i] = G[i]; }
      for (int64_t m = 0; m < M; m++) {
        T fc[D], gc[D];
#pragma unroll
        for (int i = 0; i < D; i++) { fc[i] = fn[i]; gc[i] = gn[i]; }
        if (m + 1 < M) {  // the next window's operands, loaded ahead of this step
#pragma unroll
          for (int i = 0; i < D; i++) { fn[i] = F[(m + 1) * D + i]; gn[i] = G[(m + 1) * D + i]; }
        }
        T g[D];
        if (!Rule::advance_ok(P, H, x, g)) { s_bad = 1; break; }
#pragma unroll
        for (int i = 0; i < D; i++) {
          const T xn = (g[i] + fc[i]) - gc[i];
          G[m * D + i] = g[i];
          X[(m + 1) * D + i] = xn;
          x[i] = xn;
        }
      }
    }
    __syncthreads();
    if (s_bad) st = ST_NONFINITE;
  }
  if (tid == 0) {
    a.iters[inst] = k;
    a.resid[inst] = R;
    a.status[inst] = st;
  }
}

template <int Meth>
static int parareal_launch(int dtype, int system, int d, int nt, const PararealKArgs& k,
                           hipStream_t s) {
  return dispatch_small(dtype, system, d, [&](auto t, auto sys) -> int {
    using T = decltype(t);
    using Sys = decltype(sys);
    if (nt == 1024)
      hipLaunchKernelGGL((k_parareal_small<T, Sys, Meth, 1024>), dim3((unsigned)k.B), dim3(1024), 0, s, k);
    else
      hipLaunchKernelGGL((k_parareal_small<T, Sys, Meth, 256>), dim3((unsigned)k.B), dim3(256), 0, s, k);
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

size_t parareal_ws_bytes(int d, int64_t B, int64_t M, int dtype) {
  if (B <= 0 || M <= 0 || d <= 0) return 0;
  return align_up((size_t)B * (size_t)(3 * M + 1) * (size_t)d * (dtype == 0 ? 8 : 4));
}

int parareal(const SolveArgs& a, int64_t M, int64_t S, double* hist) {
  if (a.B <= 0) return ST_OK;
  if (M > 0 && S > 0 && (a.ws == nullptr || a.ws_bytes < parareal_ws_bytes(a.d, a.B, M, a.dtype)))
    return ST_WORKSPACE;
  PararealKArgs k{};
  k.B = a.B;
  k.M = M;
  k.S = S;
  k.max_iter = a.max_iter;
  k.x0 = a.x0;
  k.params = a.params;
  k.pstride = a.pstride;
  k.traj = a.traj;
  k.dt = a.dt;
  k.tol = a.tol;
  k.iters = a.iters;
  k.resid = a.resid;
  k.status = a.status;
  k.hist = hist;
  k.ws = a.ws;
  // one thread per window when they fit in one workgroup of 1024
  const int nt = M > 256 ? 1024 : 256;
  switch (a.method) {
    case METHOD_RK4: return parareal_launch<METHOD_RK4>(a.dtype, a.system, a.d, nt, k, a.stream);
    case METHOD_BEULER: return parareal_launch<METHOD_BEULER>(a.dtype, a.system, a.d, nt, k, a.stream);
    case METHOD_TRAP: return parareal_launch<METHOD_TRAP>(a.dtype, a.system, a.d, nt, k, a.stream);
  }
  return ST_UNSUPPORTED;
}

}  // namespace pint
