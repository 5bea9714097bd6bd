// Reverse-time adjoint of the discrete solution map x_n = Phi(x_{n-1}; theta):
// H^T lambda = g for the block-bidiagonal H of eq. (jacobian), i.e.
//   lambda_T = g_T,  lambda_n = g_n + J(x_n)^T lambda_{n+1},
// evaluated with the affine scan over the reversed, transposed elements
//   e_0 = (., g_T),  e_i = (J(x_{T-i})^T, g_{T-i}) for 1 <= i < T,
//   e_T = (J(x_0)^T, 0),
// so that scan output i is lambda_{T-i} and output T is dL/dx0.  Elements are
// recomputed from the trajectory segment by segment when `seg` > 0 (memory
// seg*d*d per instance instead of T*d*d).  dL/dtheta = sum_n S(x_{n-1})^T
// lambda_n with S = dPhi/dtheta, reduced with atomics.
#include <type_traits>

#include "internal.h"
#include "systems_dense.h"
#include "systems_small.h"

namespace pint {

struct AdjArgs {
  int64_t B, T;
  const void* x0;
  const void* params;
  int64_t pstride;
  const void* traj;
  const void* g;
  double dt;
  int64_t i_lo, i_hi;  // element range [i_lo, i_hi) of this segment
  void* A;             // [B][i_hi-i_lo][D][D]  (row-major J^T), or its band
                       // [B][i_hi-i_lo][D][BW] for a banded system
  void* b;             // [B][i_hi-i_lo][D]
};

// state index of element i: x_{T-i} for 1 <= i < T, x_0 for i = T (n = 0)
__device__ __forceinline__ int64_t adj_state(int64_t T, int64_t i) { return i == T ? 0 : T - i; }

template <typename T, class S>
__global__ void k_adj_elems_small(AdjArgs a) {
  constexpr int D = S::D, NP = S::NP;
  const int64_t L = a.i_hi - a.i_lo, total = a.B * L;
  for (int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gi < total;
       gi += (int64_t)gridDim.x * blockDim.x) {
    const int64_t inst = gi / L, i = a.i_lo + gi % L;
    T* Ao = static_cast<T*>(a.A) + gi * D * D;
    T* bo = static_cast<T*>(a.b) + gi * D;
    const T* G = static_cast<const T*>(a.g) + inst * a.T * D;
    if (i == 0) {
#pragma unroll
      for (int r = 0; r < D * D; r++) Ao[r] = (r / D == r % D) ? T(1) : T(0);
#pragma unroll
      for (int r = 0; r < D; r++) bo[r] = G[(a.T - 1) * D + r];
      continue;
    }
    const int64_t n = adj_state(a.T, i);
    const T* X = static_cast<const T*>(a.traj) + inst * a.T * D;
    const T* x0 = static_cast<const T*>(a.x0) + inst * D;
    T P[NP], x[D], phi[D], J[D * D];
    const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
#pragma unroll
    for (int r = 0; r < NP; r++) P[r] = Pg[r];
#pragma unroll
    for (int r = 0; r < D; r++) x[r] = n == 0 ? x0[r] : X[(n - 1) * D + r];
    rk4_phi_jac<T, S>(P, (T)a.dt, x, phi, J);
#pragma unroll
    for (int r = 0; r < D; r++)
#pragma unroll
      for (int c = 0; c < D; c++) Ao[r * D + c] = J[c * D + r];
#pragma unroll
    for (int r = 0; r < D; r++) bo[r] = (i == a.T) ? T(0) : G[(n - 1) * D + r];
  }
}

template <typename T, class S>
__global__ __launch_bounds__(S::NT) void k_adj_elems_dense(AdjArgs a) {
  constexpr int D = S::D, NP = S::NP, NT = S::NT, NW = NT / PINT_WAVE, SPP = S::SPP, JT = S::JT;
  __shared__ typename S::Stage s_stage[SPP];
  __shared__ T s_P[SPP][NP];
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  const int64_t L = a.i_hi - a.i_lo, total = a.B * L;
  const int64_t g0 = (int64_t)blockIdx.x * SPP;
  for (int sl = 0; sl < SPP; sl++) {
    const int64_t gi = g0 + sl;
    if (gi < total) {
      const T* P = static_cast<const T*>(a.params) + (gi / L) * a.pstride;
      for (int r = tid; r < NP; r += NT) s_P[sl][r] = P[r];
    }
  }
  __syncthreads();
  for (int sl = wv; sl < SPP; sl += NW) {
    const int64_t gi = g0 + sl;
    if (gi >= total) continue;
    const int64_t inst = gi / L, i = a.i_lo + gi % L;
    const T* G = static_cast<const T*>(a.g) + inst * a.T * D;
    T* bo = static_cast<T*>(a.b) + gi * D;
    const int64_t n = adj_state(a.T, i);
    if (i == 0) {
      for (int r = lane; r < D; r += PINT_WAVE) bo[r] = G[(a.T - 1) * D + r];
      continue;
    }
    for (int r = lane; r < D; r += PINT_WAVE) bo[r] = (i == a.T) ? T(0) : G[(n - 1) * D + r];
    const T* X = static_cast<const T*>(a.traj) + inst * a.T * D;
    const T* x0 = static_cast<const T*>(a.x0) + inst * D;
    T xp[S::R], phi[S::R];
#pragma unroll
    for (int r = 0; r < S::R; r++) {
      const int c = lane + 64 * r;
      xp[r] = c < D ? (n == 0 ? x0[c] : X[(n - 1) * D + c]) : T(0);
    }
    wave_rk4<T, S>(s_P[sl], (T)a.dt, xp, phi, &s_stage[sl], lane);
  }
  __syncthreads();
  for (int t = tid; t < SPP * JT; t += NT) {
    const int sl = t / JT, sub = t % JT;
    const int64_t gi = g0 + sl;
    if (gi >= total) continue;
    const int64_t i = a.i_lo + gi % L;
    if constexpr (S::BANDED) {
      // the transposed band (row j of J^T from column j of J)
      T* Ao = static_cast<T*>(a.A) + gi * D * S::BW;
      if (i == 0) {  // identity: the diagonal is band column BOFFT
        if (sub == 0)
          for (int r = 0; r < D * S::BW; r++) Ao[r] = (r % S::BW == S::BOFFT) ? T(1) : T(0);
        continue;
      }
      S::jac_bandT_thread(&s_stage[sl], s_P[sl], sub, (T)a.dt, Ao);
    } else {
      T* Ao = static_cast<T*>(a.A) + gi * D * D;
      if (i == 0) {
        // identity (multiplies z_0 = 0)
        if (sub == 0)
          for (int r = 0; r < D * D; r++) Ao[r] = (r / D == r % D) ? T(1) : T(0);
        continue;
      }
      // J(i, j) -> Ao[j * D + i]: the row-major transpose
      S::jac_thread(&s_stage[sl], s_P[sl], sub, (T)a.dt, Ao, 1, D);
    }
  }
}

// Banded systems: the transposed band of each step, one thread per column
// of J (row of J^T) computing only the band (S::jac_band_column), BNT / D
// steps per workgroup; the stage points by one wave per step as above.
template <typename T, class S>
__global__ __launch_bounds__(256) void k_adj_elems_band(AdjArgs a) {
  constexpr int D = S::D, NP = S::NP, BW = S::BW, NT = 256, NW = NT / PINT_WAVE;
  constexpr int SPP = NT / D;  // steps per workgroup
  __shared__ typename S::Stage s_stage[SPP];
  __shared__ T s_P[SPP][NP];
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  const int64_t L = a.i_hi - a.i_lo, total = a.B * L;
  const int64_t g0 = (int64_t)blockIdx.x * SPP;
  for (int sl = 0; sl < SPP; sl++) {
    const int64_t gi = g0 + sl;
    if (gi < total) {
      const T* P = static_cast<const T*>(a.params) + (gi / L) * a.pstride;
      for (int r = tid; r < NP; r += NT) s_P[sl][r] = P[r];
    }
  }
  __syncthreads();
  for (int sl = wv; sl < SPP; sl += NW) {
    const int64_t gi = g0 + sl;
    if (gi >= total) continue;
    const int64_t inst = gi / L, i = a.i_lo + gi % L;
    const T* G = static_cast<const T*>(a.g) + inst * a.T * D;
    T* bo = static_cast<T*>(a.b) + gi * D;
    const int64_t n = adj_state(a.T, i);
    if (i == 0) {
      for (int r = lane; r < D; r += PINT_WAVE) bo[r] = G[(a.T - 1) * D + r];
      continue;
    }
    for (int r = lane; r < D; r += PINT_WAVE) bo[r] = (i == a.T) ? T(0) : G[(n - 1) * D + r];
    const T* X = static_cast<const T*>(a.traj) + inst * a.T * D;
    const T* x0 = static_cast<const T*>(a.x0) + inst * D;
    T xp[S::R], phi[S::R];
#pragma unroll
    for (int r = 0; r < S::R; r++) {
      const int c = lane + 64 * r;
      xp[r] = c < D ? (n == 0 ? x0[c] : X[(n - 1) * D + c]) : T(0);
    }
    wave_rk4<T, S>(s_P[sl], (T)a.dt, xp, phi, &s_stage[sl], lane);
  }
  __syncthreads();
  const int sl = tid / D, j = tid % D;
  const int64_t gi = g0 + sl;
  if (sl >= SPP || gi >= total) return;
  const int64_t i = a.i_lo + gi % L;
  T* row = static_cast<T*>(a.A) + gi * D * BW + (int64_t)j * BW;
  T col[BW];
  if (i == 0) {  // identity (multiplies z_0 = 0): the diagonal is band column BOFFT
#pragma unroll
    for (int r = 0; r < BW; r++) col[r] = (r == S::BOFFT) ? T(1) : T(0);
  } else {
    S::jac_band_column(&s_stage[sl], j, (T)a.dt, col);
  }
#pragma unroll
  for (int r = 0; r < BW; r++) row[r] = col[r];
}

// Copy this segment's scan outputs into lambda [B][T+1][D] and keep the
// last one as the next segment's starting vector.
template <typename T>
__global__ void k_adj_copy(int64_t B, int64_t T1, int64_t i_lo, int64_t L, int D, const T* zs,
                           T* lam, T* carry) {
  const int64_t total = B * L * D;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t inst = g / (L * D), rem = g % (L * D), m = rem / D, c = rem % D;
    const T v = zs[g];
    lam[(inst * T1 + i_lo + m) * D + c] = v;
    if (m == L - 1) carry[inst * D + c] = v;
  }
}

// dL/dtheta += S(x_{n-1})^T lambda_n, lambda_n = lam[T - n], n = 1..T.
template <typename T, class S>
__global__ void k_adj_theta_small(AdjArgs a, const T* lam, T* dth) {
  constexpr int D = S::D, NP = S::NP;
  const int64_t total = a.B * a.T;
  for (int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gi < total;
       gi += (int64_t)gridDim.x * blockDim.x) {
    const int64_t inst = gi / a.T, n = gi % a.T + 1;
    const T* X = static_cast<const T*>(a.traj) + inst * a.T * D;
    const T* x0 = static_cast<const T*>(a.x0) + inst * D;
    T P[NP], x[D], J[D * D], Sth[D * NP];
    const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
#pragma unroll
    for (int r = 0; r < NP; r++) P[r] = Pg[r];
#pragma unroll
    for (int r = 0; r < D; r++) x[r] = n == 1 ? x0[r] : X[(n - 2) * D + r];
    rk4_jac_ptheta<T, S>(P, (T)a.dt, x, J, Sth);
    const T* ln = lam + (inst * (a.T + 1) + (a.T - n)) * D;
#pragma unroll
    for (int j = 0; j < NP; j++) {
      T acc = T(0);
#pragma unroll
      for (int r = 0; r < D; r++) acc += Sth[r * NP + j] * ln[r];
      atomicAdd(dth + inst * NP + j, acc);
    }
  }
}

// Lorenz-96: theta = F, S = dPhi/dF by the chain rule through the stages
// (f_F = 1):  D1 = 1, D_s = Jf(x_s)(c D_{s-1}) + 1, S = dt/6 (D1+2D2+2D3+D4).
// One wave per run of TH_SPW consecutive steps of one instance (the stencil
// product by shuffles), the run's terms summed in registers and added to
// dL/dF with one atomic per wave.
constexpr int TH_SPW = 64;

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_adj_theta_l96(AdjArgs a, const T* lam, T* dth) {
  using S = DSysL96<T, DIM>;
  constexpr int D = DIM;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int64_t per_inst = (a.T + 4 * TH_SPW - 1) / (4 * TH_SPW);  // blocks per instance
  const int64_t inst = blockIdx.x / per_inst;
  const int64_t n0 = (blockIdx.x % per_inst) * 4 * TH_SPW + (int64_t)wv * TH_SPW + 1;
  if (inst >= a.B || n0 > a.T) return;
  const int64_t n1 = n0 + TH_SPW - 1 < a.T ? n0 + TH_SPW - 1 : a.T;
  const T* X = static_cast<const T*>(a.traj) + inst * a.T * D;
  const T* x0 = static_cast<const T*>(a.x0) + inst * D;
  const T* P = static_cast<const T*>(a.params) + inst * a.pstride;
  const int i = lane < D ? lane : 0;
  const T dt = (T)a.dt, h2 = T(0.5) * dt, c6 = dt / T(6);
  T part = T(0);
  for (int64_t n = n0; n <= n1; n++) {
    T x[1] = {lane < D ? (n == 1 ? x0[i] : X[(n - 2) * D + i]) : T(0)};
    T k[1], y[1] = {x[0]};
    T Dv = T(1), acc = T(1);
    S::f(P, x, k, lane);
    for (int s = 1; s < 4; s++) {
      const T cprev = (s == 3) ? dt : h2;  // x_{s+1} = x + c k_s
      y[0] = x[0] + cprev * k[0];
      // Jf(y) (cprev * Dv) + 1
      const T v = cprev * Dv;
      const T yp1 = __shfl(y[0], (i + 1) % D, 64), ym1 = __shfl(y[0], (i + D - 1) % D, 64);
      const T ym2 = __shfl(y[0], (i + D - 2) % D, 64);
      const T vp1 = __shfl(v, (i + 1) % D, 64), vm1 = __shfl(v, (i + D - 1) % D, 64);
      const T vm2 = __shfl(v, (i + D - 2) % D, 64);
      Dv = ym1 * (vp1 - vm2) + (yp1 - ym2) * vm1 - v + T(1);
      acc += ((s == 3) ? T(1) : T(2)) * Dv;
      S::f(P, y, k, lane);
    }
    const T* ln = lam + (inst * (a.T + 1) + (a.T - n)) * D;
    if (lane < D) part += c6 * acc * ln[i];
  }
  part = wave_sum(part);
  if (lane == 0) atomicAdd(dth + inst, part);
}

// ------------------------------------------- Lorenz-96, fused reverse pass --

// The whole reverse recursion of one Lorenz-96 instance in one workgroup,
// with the transposed elements built just before they are used and never
// stored: lambda_T = g_T, lambda_n = g_n + J(x_n)^T lambda_{n+1} for
// n = T-1 .. 1, dL/dx0 = J(x_0)^T lambda_1, and
// dL/dF = sum_{n=0}^{T-1} S(x_n) . lambda_{n+1} (S = dPhi/dF).
//
// Eight waves.  Six builder waves (1, 2, 3, 5, 6, 7) take the elements
// i = T - n round robin: each loads x_n and g_n, runs the RK4 stages, and
// puts into an LDS ring of AP_R slots the band of row j of J(x_n)^T for
// every j (column j of J over the 13 rows its tangent reaches) and
// S(x_n); then it publishes the slot.  Wave 0 runs the recursion, one lane
// per component: per element a 13-term row (the band against the
// neighbours of lambda, exchanged through LDS) and the dL/dF term; the
// next element's operands are loaded during the current one.  Wave 4 is
// idle so the recursion's SIMD (waves are spread over the SIMDs in turn)
// serves it alone.  Only the trajectory, g and the outputs touch HBM.  The
// waits are between waves of one workgroup; they are bounded all the same,
// and a wait that gives up stops the workgroup and leaves NaN in that
// instance's gradients.
constexpr int AP_NT = 512, AP_R = 24, AP_NB = 6;
__device__ __forceinline__ int ap_builder(int wv) {
  return wv >= 1 && wv <= 3 ? wv - 1 : (wv >= 5 ? wv - 2 : -1);
}

template <typename T, int D>
struct AdjPipeSmem {
  static constexpr int BW = DSysL96<T, D>::BW;
  T band[AP_R][BW][D];  // band[s][r][j] = J(j - 4 + r, j) = J^T(j, j - 4 + r)
  T g[AP_R][D];
  T sens[AP_R][D];      // S(x_n)
  StageL96<T, D> stage[AP_NB];
  T zx[D + BW - 1];     // zx[q] = lambda[(q - 4) mod D]
  int ready[AP_R];      // element index held by the slot (0: none yet)
  int consumed;         // last element the recursion has finished
  int abort_;
};

template <typename T, int D>
__global__ __launch_bounds__(AP_NT) void k_adj_pipe_l96(AdjArgs a, T* dx0, T* dth, uint64_t lim) {
  using S = DSysL96<T, D>;
  constexpr int BW = S::BW, LO = S::BOFFT, R = AP_R;
  static_assert(BW == 13 && LO == 4 && D <= PINT_WAVE, "Lorenz-96 band");
  extern __shared__ __align__(16) unsigned char dyn[];
  AdjPipeSmem<T, D>& sm = *reinterpret_cast<AdjPipeSmem<T, D>*>(dyn);
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  const int64_t inst = blockIdx.x;
  const int64_t Tn = a.T;
  const int j = lane < D ? lane : 0;  // lanes past D repeat lane 0
  const T dt = (T)a.dt;
  const T* G = static_cast<const T*>(a.g) + inst * Tn * D;
  const T* X = static_cast<const T*>(a.traj) + inst * Tn * D;
  const T* x0 = static_cast<const T*>(a.x0) + inst * D;
  if (tid < R) sm.ready[tid] = 0;
  if (tid == 0) {
    sm.consumed = 0;
    sm.abort_ = 0;
  }
  __syncthreads();
  auto spin = [&](uint64_t& it) -> bool {  // true: stop
    if (++it >= lim) {
      __hip_atomic_store(&sm.abort_, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return true;
    }
    __builtin_amdgcn_s_sleep(1);
    return __hip_atomic_load(&sm.abort_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
  };
  auto ld = [](const int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };
  auto st = [](int* p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };

  const int e = ap_builder(wv);
  if (e >= 0) {
    // ------------------------------------------------------- builders ---
    const T P[1] = {static_cast<const T*>(a.params)[inst * a.pstride]};
    const T h2 = T(0.5) * dt, c6 = dt / T(6);
    StageL96<T, D>* stg = &sm.stage[e];
    auto fetch = [&](int64_t i, T& xv, T& gv) {  // x_n and g_n of element i (n = T - i)
      const int64_t n = Tn - i;
      xv = n == 0 ? x0[j] : X[(n - 1) * D + j];
      gv = n == 0 ? T(0) : G[(n - 1) * D + j];
    };
    T xn = T(0), gn = T(0);
    if (1 + e <= Tn) fetch(1 + e, xn, gn);
    for (int64_t i = 1 + e; i <= Tn; i += AP_NB) {
      const T xc = xn, gc = gn;
      if (i + AP_NB <= Tn) fetch(i + AP_NB, xn, gn);  // the next element's loads fly meanwhile
      uint64_t it = 0;
      bool stop = false;
      while (ld(&sm.consumed) < i - R)  // the slot's previous element is used
        if ((stop = spin(it))) break;
      if (stop) break;
      const int slot = (int)(i % R);
      T xs[1] = {lane < D ? xc : T(0)}, phi[1];
      wave_rk4<T, S>(P, dt, xs, phi, stg, lane);
      T col[BW];
      S::jac_band_column(stg, j, dt, col);
      // S = dPhi/dF through the stages (f_F = 1): D_1 = 1,
      // D_s = Jf(y_s)(c D_{s-1}) + 1, S = dt/6 (D_1 + 2 D_2 + 2 D_3 + D_4)
      T Dv = T(1), acc = T(1);
#pragma unroll
      for (int s = 1; s < 4; s++) {
        const T c = (s == 3) ? dt : h2;
        const T v = c * Dv;
        const T* y = stg->x[s];
        const T yp1 = y[j + 1 == D ? 0 : j + 1], ym1 = y[j == 0 ? D - 1 : j - 1];
        const T ym2 = y[j >= 2 ? j - 2 : j + D - 2];
        const T vp1 = __shfl(v, (j + 1) % D, PINT_WAVE), vm1 = __shfl(v, (j + D - 1) % D, PINT_WAVE);
        const T vm2 = __shfl(v, (j + D - 2) % D, PINT_WAVE);
        Dv = ym1 * (vp1 - vm2) + (yp1 - ym2) * vm1 - v + T(1);
        acc += ((s == 3) ? T(1) : T(2)) * Dv;
      }
      if (lane < D) {
#pragma unroll
        for (int r = 0; r < BW; r++) sm.band[slot][r][lane] = col[r];
        sm.g[slot][lane] = gc;
        sm.sens[slot][lane] = c6 * acc;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0) st(&sm.ready[slot], (int)i);
    }
  } else if (wv == 0) {
    // ------------------------------------------------------ recursion ---
    __builtin_amdgcn_s_setprio(3);
    T z = Tn > 0 ? G[(Tn - 1) * D + j] : T(0);  // lambda_T = g_T
    T th = T(0);
    auto put_z = [&](T v) {  // zx[q] = lambda[(q - 4) mod D]
      if (lane < D) {
        sm.zx[lane + LO] = v;
        if (lane >= D - LO) sm.zx[lane + LO - D] = v;
        if (lane < BW - 1 - LO) sm.zx[lane + LO + D] = v;
      }
    };
    put_z(z);
    T zv[BW], bA[BW], bB[BW], gA = T(0), gB = T(0), sA = T(0), sB = T(0);
    bool stop = false;
    auto wait_el = [&](int64_t i) -> bool {  // true: element i is in its slot
      uint64_t it = 0;
      while (ld(&sm.ready[i % R]) != (int)i)
        if (spin(it)) return false;
      return true;
    };
    auto load_el = [&](int64_t i, T (&bv)[BW], T& gv, T& sv) {
      const int slot = (int)(i % R);
#pragma unroll
      for (int r = 0; r < BW; r++) bv[r] = sm.band[slot][r][j];
      gv = sm.g[slot][j];
      sv = sm.sens[slot][j];
    };
    if (Tn > 0) {
      stop = !wait_el(1);
      if (!stop) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
        for (int r = 0; r < BW; r++) zv[r] = sm.zx[j + r];
        load_el(1, bA, gA, sA);
      }
    }
    int nxt = Tn > 1 ? ld(&sm.ready[2 % R]) : 0;  // flag of the next element, read ahead
    // element i with operands (bc, gc, sc); the next one's go to (bn, gn, sn)
    auto step = [&](int64_t i, T (&bc)[BW], T& gc, T& sc, T (&bn)[BW], T& gn, T& sn)
        __attribute__((always_inline)) -> bool {
      const bool more = i < Tn;
      if (more) {
        if (nxt != (int)(i + 1)) {
          if (!wait_el(i + 1)) return false;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        load_el(i + 1, bn, gn, sn);
        nxt = i + 2 <= Tn ? ld(&sm.ready[(i + 2) % R]) : 0;
      }
      th += sc * z;  // S(x_n) . lambda_{n+1}
      z = band_row13<T>(gc, bc, zv);
      put_z(z);
      if (more) {
#pragma unroll
        for (int r = 0; r < BW; r++) zv[r] = sm.zx[j + r];
      }
      st(&sm.consumed, (int)i);
      return more;
    };
    if (!stop) {
      for (int64_t i = 1;;) {
        bool go = step(i, bA, gA, sA, bB, gB, sB);
        if (!go) break;
        i++;
        go = step(i, bB, gB, sB, bA, gA, sA);
        if (!go) break;
        i++;
      }
    }
    stop = ld(&sm.abort_) != 0;
    th = wave_sum(lane < D ? th : T(0));
    const T nan = T(__builtin_nan(""));
    if (lane < D) dx0[inst * D + lane] = stop ? nan : z;
    if (lane == 0 && dth) dth[inst] = stop ? nan : th;
  }
}

// ------------------------------------------------------------- host -------

template <typename F>
static int dispatch_adj(int dtype, int system, int d, F&& f) {
  auto go = [&](auto t) -> int {
    using T = decltype(t);
    switch (system) {
      case 0:
        switch (d) {
          case 1: return f(t, SysLinear<T, 1>{}, std::true_type{});
          case 2: return f(t, SysLinear<T, 2>{}, std::true_type{});
          case 3: return f(t, SysLinear<T, 3>{}, std::true_type{});
          case 4: return f(t, SysLinear<T, 4>{}, std::true_type{});
        }
        break;
      case 1: if (d == 1) return f(t, SysLogistic<T>{}, std::true_type{}); break;
      case 2: if (d == 2) return f(t, SysVdP<T>{}, std::true_type{}); break;
      case 3: if (d == 4) return f(t, SysCartPole<T>{}, std::true_type{}); break;
      case 4: if (d == 3) return f(t, SysLorenz63<T>{}, std::true_type{}); break;
      case 5: if (d == 40) return f(t, DSysL96<T, 40>{}, std::false_type{}); break;
      case 6:
        if (d == 128) return f(t, DSysKur<T, 128>{}, std::false_type{});
        if (d == 64) return f(t, DSysKur<T, 64>{}, std::false_type{});
        break;
    }
    return ST_UNSUPPORTED;
  };
  if (dtype == 0) return go((double)0);
  if (dtype == 1) return go((float)0);
  return ST_UNSUPPORTED;
}

struct AdjLayout {
  int64_t L;  // elements per segment
  size_t off_A, off_b, off_lam, off_zs, off_carry, off_scan, scan_bytes, total;
};

// Band width of the adjoint elements of a banded system (0: dense).
static int adj_band(int system, int d) {
  return (system == 5 && d == 40) ? DSysL96<double, 40>::BW : 0;
}

static AdjLayout adj_layout(int system, int d, int64_t B, int64_t T, int64_t seg, int dtype) {
  AdjLayout l{};
  const size_t s = dtype == 0 ? 8 : 4;
  const int64_t T1 = T + 1;
  const int bw = adj_band(system, d);
  l.L = (seg > 0 && seg < T1) ? seg : T1;
  size_t o = 0;
  l.off_A = o;     o += align_up((size_t)B * l.L * d * (bw ? bw : d) * s);
  l.off_b = o;     o += align_up((size_t)B * l.L * d * s);
  l.off_lam = o;   o += align_up((size_t)B * T1 * d * s);
  l.off_zs = o;    o += align_up((size_t)B * l.L * d * s);
  l.off_carry = o; o += align_up((size_t)B * d * s);
  l.off_scan = o;
  l.scan_bytes = bw ? scan_band_ws_bytes(d, bw, DSysL96<double, 40>::BOFFT, B, l.L, 0, dtype)
                   : scan_ws_bytes(d, B, l.L, 0, dtype);
  o += align_up(l.scan_bytes);
  l.total = o;
  return l;
}

// Lorenz-96 d = 40 takes the fused reverse pass (k_adj_pipe_l96) unless the
// pipelined kernels are switched off (pint_set_dense_pipeline).
static bool adj_fused(int system, int d) { return system == 5 && d == 40 && dense_pipeline(); }

template <typename T>
static int adj_pipe_launch(const AdjArgs& a, void* dL_dx0, void* dL_dth, hipStream_t st) {
  using SM = AdjPipeSmem<T, 40>;
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adj_pipe_l96<T, 40>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(SM)) != hipSuccess)
      return ST_DEVICE;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_adj_pipe_l96<T, 40>), dim3((unsigned)a.B), dim3(AP_NT), sizeof(SM), st, a,
                     static_cast<T*>(dL_dx0), static_cast<T*>(dL_dth), wait_limit());
  return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
}

size_t adjoint_ws_bytes(int system, int d, int64_t B, int64_t T, int64_t seg, int dtype) {
  if (!small_supported(system, d) && !dense_supported(system, d)) return 0;
  if (adj_fused(system, d)) return 256;  // no elements, no lambda: nothing beyond the call's outputs
  return adj_layout(system, d, B, T, seg, dtype).total;
}

int adjoint(const SolveArgs& sa, const void* g, void* dL_dx0, void* dL_dth, int64_t seg) {
  const int d = sa.d;
  const int64_t B = sa.B, T = sa.T_uniform, T1 = T + 1;
  if (sa.system == 6 && dL_dth) return ST_UNSUPPORTED;  // Kuramoto: dL/dx0 only
  if (adj_fused(sa.system, d)) {
    if (!sa.ws || sa.ws_bytes < 256) return ST_WORKSPACE;
    if (T == 0) {
      if (dL_dth)
        if (int rc = fill_u32(static_cast<uint32_t*>(dL_dth), (size_t)B * (sa.dtype == 0 ? 2 : 1), 0u, sa.stream))
          return rc;
      return fill_u32(static_cast<uint32_t*>(dL_dx0), (size_t)B * d * (sa.dtype == 0 ? 2 : 1), 0u, sa.stream);
    }
    AdjArgs a{};
    a.B = B;
    a.T = T;
    a.x0 = sa.x0;
    a.params = sa.params;
    a.pstride = sa.pstride;
    a.traj = sa.traj;
    a.g = g;
    a.dt = sa.dt;
    if (sa.dtype == 0) return adj_pipe_launch<double>(a, dL_dx0, dL_dth, sa.stream);
    if (sa.dtype == 1) return adj_pipe_launch<float>(a, dL_dx0, dL_dth, sa.stream);
    return ST_UNSUPPORTED;
  }
  const AdjLayout lay = adj_layout(sa.system, d, B, T, seg, sa.dtype);
  if (!sa.ws || sa.ws_bytes < lay.total) return ST_WORKSPACE;
  char* w = static_cast<char*>(sa.ws);
  hipStream_t st = sa.stream;
  const size_t s = sa.dtype == 0 ? 8 : 4;
  int np = 0;
  switch (sa.system) {
    case 0: np = d * d; break;   // linear: M
    case 1: np = 2; break;       // logistic: r, K
    case 2: np = 1; break;       // van der Pol: mu
    case 4: np = 3; break;       // Lorenz-63: sigma, rho, beta
    case 5: np = 1; break;       // Lorenz-96: F
    default: if (dL_dth) return ST_UNSUPPORTED;
  }
  if (dL_dth)
    if (int rc = fill_u32(static_cast<uint32_t*>(dL_dth), (size_t)B * np * s / 4, 0u, st)) return rc;
  if (T == 0)  // no loss terms: dL/dx0 = 0
    return fill_u32(static_cast<uint32_t*>(dL_dx0), (size_t)B * d * s / 4, 0u, st);
  return dispatch_adj(sa.dtype, sa.system, d, [&](auto t, auto sys, auto is_small) -> int {
    using T_ = decltype(t);
    using S = decltype(sys);
    constexpr int D = S::D;
    AdjArgs a{};
    a.B = B;
    a.T = T;
    a.x0 = sa.x0;
    a.params = sa.params;
    a.pstride = sa.pstride;
    a.traj = sa.traj;
    a.g = g;
    a.dt = sa.dt;
    a.A = w + lay.off_A;
    a.b = w + lay.off_b;
    T_* lam = reinterpret_cast<T_*>(w + lay.off_lam);
    T_* zs = reinterpret_cast<T_*>(w + lay.off_zs);
    T_* carry = reinterpret_cast<T_*>(w + lay.off_carry);
    const bool segmented = lay.L < T1;
    for (int64_t lo = 0; lo < T1; lo += lay.L) {
      const int64_t hi = lo + lay.L < T1 ? lo + lay.L : T1, L = hi - lo;
      a.i_lo = lo;
      a.i_hi = hi;
      const int64_t tot = B * L;
      if constexpr (decltype(is_small)::value) {
        const int grid = (int)((tot + 255) / 256 < 8192 ? (tot + 255) / 256 : 8192);
        hipLaunchKernelGGL((k_adj_elems_small<T_, S>), dim3(grid), dim3(256), 0, st, a);
      } else if constexpr (S::BANDED) {
        constexpr int spp = 256 / D;
        const int64_t grid = (tot + spp - 1) / spp;
        hipLaunchKernelGGL((k_adj_elems_band<T_, S>), dim3((unsigned)grid), dim3(256), 0, st, a);
      } else {
        const int64_t grid = (tot + S::SPP - 1) / S::SPP;
        hipLaunchKernelGGL((k_adj_elems_dense<T_, S>), dim3((unsigned)grid), dim3(S::NT), 0, st, a);
      }
      if (hipGetLastError() != hipSuccess) return ST_DEVICE;
      // the scan writes straight into lambda when there is one segment
      T_* zout = segmented ? zs : lam;
      // the scan needs B sequences of L elements: contiguous in A/b
      int rc = ST_OK;
      auto dense_scan = [&]() {
        return affine_scan(D, B, L, sa.dtype, a.A, a.b, lo == 0 ? nullptr : carry, zout, 0,
                           w + lay.off_scan, lay.scan_bytes, st);
      };
      if constexpr (decltype(is_small)::value) {
        rc = dense_scan();
      } else {
        if constexpr (S::BANDED)
          rc = affine_scan_band(D, S::BW, S::BOFFT, B, L, sa.dtype, a.A, a.b,
                                lo == 0 ? nullptr : carry, zout, 0, w + lay.off_scan,
                                lay.scan_bytes, st);
        else
          rc = dense_scan();
      }
      if (rc) return rc;
      if (segmented) {
        const int64_t n = B * L * D;
        const int grid = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
        hipLaunchKernelGGL((k_adj_copy<T_>), dim3(grid), dim3(256), 0, st, B, T1, lo, L, D,
                           (const T_*)zs, lam, carry);
        if (hipGetLastError() != hipSuccess) return ST_DEVICE;
      }
    }
    // dL/dx0 = lambda row T of every instance
    if (hipMemcpy2DAsync(dL_dx0, D * s, lam + T * D, T1 * D * s, D * s, B, hipMemcpyDeviceToDevice,
                         st) != hipSuccess)
      return ST_DEVICE;
    if (dL_dth) {
      if constexpr (decltype(is_small)::value) {
        const int64_t tot = B * T;
        const int grid = (int)((tot + 255) / 256 < 8192 ? (tot + 255) / 256 : 8192);
        if (tot > 0)
          hipLaunchKernelGGL((k_adj_theta_small<T_, S>), dim3(grid), dim3(256), 0, st, a,
                             (const T_*)lam, static_cast<T_*>(dL_dth));
      } else if constexpr (D == 40 && S::NP == 1) {
        const int64_t tot = B * T;
        const int64_t per_inst = (T + 4 * TH_SPW - 1) / (4 * TH_SPW);
        if (tot > 0)
          hipLaunchKernelGGL((k_adj_theta_l96<T_, 40>), dim3((unsigned)(B * per_inst)), dim3(256), 0,
                             st, a, (const T_*)lam, static_cast<T_*>(dL_dth));
      } else {
        return ST_UNSUPPORTED;
      }
      if (hipGetLastError() != hipSuccess) return ST_DEVICE;
    }
    return ST_OK;
  });
}

}  // namespace pint
