// Vector fields of small state dimension (d <= 4), evaluated per thread in
// registers, the classic RK4 step with its exact derivatives, and the step
// rules (explicit RK4, backward Euler, trapezoidal) the small solver runs.
#pragma once

#include "device_common.h"

namespace pint {

// Each system provides D (state dimension), NP (parameter count) and
//   f(P, x, out)  : out = f(x; P)
//   jf(P, x, J)   : J = df/dx (row-major D x D)
//   fth(P, x, G)  : G = df/dP (row-major D x NP)

template <typename T, int DIM>
struct SysLinear {  // f = M x, P = M row-major
  static constexpr int D = DIM, NP = DIM * DIM;
  __device__ static void f(const T* P, const T* x, T* out) {
#pragma unroll
    for (int i = 0; i < D; i++) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < D; j++) acc += P[i * D + j] * x[j];
      out[i] = acc;
    }
  }
  __device__ static void jf(const T* P, const T*, T* J) {
#pragma unroll
    for (int i = 0; i < D * D; i++) J[i] = P[i];
  }
  __device__ static void fth(const T*, const T* x, T* G) {
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
      for (int k = 0; k < NP; k++) G[i * NP + k] = (k / D == i) ? x[k % D] : T(0);
  }
};

template <typename T>
struct SysLogistic {  // dP/dt = r P (1 - P/K)   (Sec. 4.1)
  static constexpr int D = 1, NP = 2;
  __device__ static void f(const T* P, const T* x, T* out) { out[0] = P[0] * x[0] * (T(1) - x[0] / P[1]); }
  __device__ static void jf(const T* P, const T* x, T* J) { J[0] = P[0] * (T(1) - T(2) * x[0] / P[1]); }
  __device__ static void fth(const T* P, const T* x, T* G) {
    G[0] = x[0] * (T(1) - x[0] / P[1]);
    G[1] = P[0] * x[0] * x[0] / (P[1] * P[1]);
  }
};

template <typename T>
struct SysVdP {  // x'' = mu (1 - x^2) x' - x as (x, v)   (Sec. 4.1)
  static constexpr int D = 2, NP = 1;
  __device__ static void f(const T* P, const T* x, T* out) {
    out[0] = x[1];
    out[1] = P[0] * (T(1) - x[0] * x[0]) * x[1] - x[0];
  }
  __device__ static void jf(const T* P, const T* x, T* J) {
    J[0] = T(0);
    J[1] = T(1);
    J[2] = T(-2) * P[0] * x[0] * x[1] - T(1);
    J[3] = P[0] * (T(1) - x[0] * x[0]);
  }
  __device__ static void fth(const T*, const T* x, T* G) {
    G[0] = T(0);
    G[1] = (T(1) - x[0] * x[0]) * x[1];
  }
};

template <typename T>
struct SysCartPole {  // (p, th, p', th'), textbook form with th'^2   (Sec. 4.1)
  static constexpr int D = 4, NP = 4;
  __device__ static void f(const T* P, const T* x, T* out) {
    const T g = P[0], l = P[1], mc = P[2], mp = P[3];
    const T w = x[3];
    T s, c;
    sincos_(x[1], &s, &c);
    const T den = mc + mp * s * s;
    out[0] = x[2];
    out[1] = w;
    out[2] = mp * s * (l * w * w + g * c) / den;
    out[3] = (-mp * l * w * w * c * s - (mc + mp) * g * s) / (l * den);
  }
  __device__ static void jf(const T* P, const T* x, T* J) {
    const T g = P[0], l = P[1], mc = P[2], mp = P[3];
    const T w = x[3];
    T s, c;
    sincos_(x[1], &s, &c);
    const T den = mc + mp * s * s, dden = T(2) * mp * s * c;
    const T n1 = mp * s * (l * w * w + g * c);
    const T dn1 = mp * (c * (l * w * w + g * c) - g * s * s);
    const T n2 = -mp * l * w * w * c * s - (mc + mp) * g * s;
    const T dn2 = -mp * l * w * w * (c * c - s * s) - (mc + mp) * g * c;
#pragma unroll
    for (int i = 0; i < 16; i++) J[i] = T(0);
    J[0 * 4 + 2] = T(1);
    J[1 * 4 + 3] = T(1);
    J[2 * 4 + 1] = (dn1 * den - n1 * dden) / (den * den);
    J[2 * 4 + 3] = T(2) * mp * s * l * w / den;
    J[3 * 4 + 1] = (dn2 * den - n2 * dden) / (l * den * den);
    J[3 * 4 + 3] = T(-2) * mp * l * w * c * s / (l * den);
  }
  __device__ static void fth(const T*, const T*, T* G) {
    // not provided (the adjoint entry point rejects the cart-pole)
#pragma unroll
    for (int i = 0; i < 16; i++) G[i] = T(0);
  }
  __device__ static void sincos_(T a, T* s, T* c) {
    *s = sin(a);
    *c = cos(a);
  }
};

template <typename T>
struct SysLorenz63 {
  static constexpr int D = 3, NP = 3;
  __device__ static void f(const T* P, const T* x, T* out) {
    out[0] = P[0] * (x[1] - x[0]);
    out[1] = x[0] * (P[1] - x[2]) - x[1];
    out[2] = x[0] * x[1] - P[2] * x[2];
  }
  __device__ static void jf(const T* P, const T* x, T* J) {
    J[0] = -P[0];       J[1] = P[0]; J[2] = T(0);
    J[3] = P[1] - x[2]; J[4] = T(-1); J[5] = -x[0];
    J[6] = x[1];        J[7] = x[0]; J[8] = -P[2];
  }
  __device__ static void fth(const T*, const T* x, T* G) {
    G[0] = x[1] - x[0]; G[1] = T(0); G[2] = T(0);
    G[3] = T(0);        G[4] = x[0]; G[5] = T(0);
    G[6] = T(0);        G[7] = T(0); G[8] = -x[2];
  }
};

template <typename T>
struct SysRobertson {  // Robertson's reaction system (Sec. 4.2, eq. robertson), P = (k1, k2, k3)
  static constexpr int D = 3, NP = 3;
  __device__ static void f(const T* P, const T* x, T* out) {
    out[0] = -P[0] * x[0] + P[2] * x[1] * x[2];
    out[1] = P[0] * x[0] - P[1] * x[1] * x[1] - P[2] * x[1] * x[2];
    out[2] = P[1] * x[1] * x[1];
  }
  __device__ static void jf(const T* P, const T* x, T* J) {
    J[0] = -P[0]; J[1] = P[2] * x[2];                        J[2] = P[2] * x[1];
    J[3] = P[0];  J[4] = T(-2) * P[1] * x[1] - P[2] * x[2];  J[5] = -P[2] * x[1];
    J[6] = T(0);  J[7] = T(2) * P[1] * x[1];                 J[8] = T(0);
  }
  __device__ static void fth(const T*, const T* x, T* G) {
    G[0] = -x[0]; G[1] = T(0);           G[2] = x[1] * x[2];
    G[3] = x[0];  G[4] = -x[1] * x[1];   G[5] = -x[1] * x[2];
    G[6] = T(0);  G[7] = x[1] * x[1];    G[8] = T(0);
  }
};

// ---------------------------------------------------------------- RK4 -----

// Classic RK4 (eq. explicit-rk with c = (0, 1/2, 1/2, 1),
// b = (1/6, 1/3, 1/3, 1/6)):  phi = x + dt/6 (k1 + 2 k2 + 2 k3 + k4).
template <typename T, class S>
__device__ __forceinline__ void rk4_phi(const T* P, T dt, const T* x, T* phi) {
  constexpr int D = S::D;
  T k1[D], k2[D], k3[D], k4[D], y[D];
  const T h2 = T(0.5) * dt;
  S::f(P, x, k1);
#pragma unroll
  for (int i = 0; i < D; i++) y[i] = x[i] + h2 * k1[i];
  S::f(P, y, k2);
#pragma unroll
  for (int i = 0; i < D; i++) y[i] = x[i] + h2 * k2[i];
  S::f(P, y, k3);
#pragma unroll
  for (int i = 0; i < D; i++) y[i] = x[i] + dt * k3[i];
  S::f(P, y, k4);
  const T c6 = dt / T(6);
#pragma unroll
  for (int i = 0; i < D; i++) phi[i] = x[i] + c6 * (k1[i] + T(2) * k2[i] + T(2) * k3[i] + k4[i]);
}

// phi and J = dphi/dx by the chain rule through the stages:
//   K1 = Jf(x), K2 = Jf(x2)(I + dt/2 K1), K3 = Jf(x3)(I + dt/2 K2),
//   K4 = Jf(x4)(I + dt K3),  J = I + dt/6 (K1 + 2 K2 + 2 K3 + K4).
template <typename T, class S>
__device__ __forceinline__ void rk4_phi_jac(const T* P, T dt, const T* x, T* phi, T* J) {
  constexpr int D = S::D;
  T k[D], acc[D], y[D];
  T Jf[D * D], K[D * D], M[D * D], Jacc[D * D];
  const T h2 = T(0.5) * dt;
  const T c6 = dt / T(6);
  // stage 1
  S::f(P, x, k);
  S::jf(P, x, K);
#pragma unroll
  for (int i = 0; i < D; i++) { acc[i] = k[i]; y[i] = x[i] + h2 * k[i]; }
#pragma unroll
  for (int i = 0; i < D * D; i++) { Jacc[i] = K[i]; M[i] = h2 * K[i]; }
#pragma unroll
  for (int i = 0; i < D; i++) M[i * D + i] += T(1);
  // stages 2..4
#pragma unroll
  for (int s = 2; s <= 4; s++) {
    S::f(P, y, k);
    S::jf(P, y, Jf);
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
      for (int j = 0; j < D; j++) {
        T a = T(0);
#pragma unroll
        for (int q = 0; q < D; q++) a += Jf[i * D + q] * M[q * D + j];
        K[i * D + j] = a;
      }
    const T wgt = (s == 4) ? T(1) : T(2);
    const T step = (s == 3) ? dt : h2;  // coefficient for the next stage point
#pragma unroll
    for (int i = 0; i < D; i++) {
      acc[i] += wgt * k[i];
      y[i] = x[i] + step * k[i];
    }
#pragma unroll
    for (int i = 0; i < D * D; i++) {
      Jacc[i] += wgt * K[i];
      M[i] = step * K[i];
    }
#pragma unroll
    for (int i = 0; i < D; i++) M[i * D + i] += T(1);
  }
#pragma unroll
  for (int i = 0; i < D; i++) phi[i] = x[i] + c6 * acc[i];
#pragma unroll
  for (int i = 0; i < D * D; i++) J[i] = c6 * Jacc[i];
#pragma unroll
  for (int i = 0; i < D; i++) J[i * D + i] += T(1);
}

// S = dphi/dP (D x NP) by the chain rule:
//   D1 = f_P(x), D2 = Jf(x2)(dt/2 D1) + f_P(x2), D3 = Jf(x3)(dt/2 D2) + f_P(x3),
//   D4 = Jf(x4)(dt D3) + f_P(x4),  S = dt/6 (D1 + 2 D2 + 2 D3 + D4);
// also returns J = dphi/dx.
template <typename T, class S>
__device__ __forceinline__ void rk4_jac_ptheta(const T* P, T dt, const T* x, T* J, T* Sth) {
  constexpr int D = S::D, NP = S::NP;
  T phi[D];
  rk4_phi_jac<T, S>(P, dt, x, phi, J);
  T k[D], y[D], Jf[D * D], Dp[D * NP], G[D * NP], Sacc[D * NP];
  const T h2 = T(0.5) * dt, c6 = dt / T(6);
  S::f(P, x, k);
  S::fth(P, x, Dp);
#pragma unroll
  for (int i = 0; i < D * NP; i++) Sacc[i] = Dp[i];
#pragma unroll
  for (int i = 0; i < D; i++) y[i] = x[i] + h2 * k[i];
#pragma unroll
  for (int s = 2; s <= 4; s++) {
    const T prevc = (s == 4) ? dt : h2;  // coefficient multiplying D_{s-1}
    S::jf(P, y, Jf);
    S::fth(P, y, G);
    T Dn[D * NP];
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
      for (int j = 0; j < NP; j++) {
        T a = T(0);
#pragma unroll
        for (int q = 0; q < D; q++) a += Jf[i * D + q] * (prevc * Dp[q * NP + j]);
        Dn[i * NP + j] = a + G[i * NP + j];
      }
    S::f(P, y, k);
    const T wgt = (s == 4) ? T(1) : T(2);
    const T step = (s == 3) ? dt : h2;
#pragma unroll
    for (int i = 0; i < D * NP; i++) { Sacc[i] += wgt * Dn[i]; Dp[i] = Dn[i]; }
#pragma unroll
    for (int i = 0; i < D; i++) y[i] = x[i] + step * k[i];
  }
#pragma unroll
  for (int i = 0; i < D * NP; i++) Sth[i] = c6 * Sacc[i];
}

// ------------------------------------------------------ step rules -----

// Methods of the one-step map (the public pint_method numbering).
enum { METHOD_RK4 = 0, METHOD_BEULER = 1, METHOD_TRAP = 2 };

// Solve M X = R in registers for a D x D matrix M and NR right-hand sides
// (both row-major, overwritten; X is left in R).  Gaussian elimination with
// partial pivoting; every index is a compile-time constant, so a row
// exchange is a run of selects (a larger candidate is swapped into the pivot
// row as it is met, which leaves the column's largest entry there).  A zero
// pivot yields non-finite results, which the callers report.
template <typename T, int D, int NR>
__device__ __forceinline__ void solve_small(T* M, T* R) {
#pragma unroll
  for (int c = 0; c < D; c++) {
#pragma unroll
    for (int r = c + 1; r < D; r++) {
      const bool sw = fabs(M[r * D + c]) > fabs(M[c * D + c]);
#pragma unroll
      for (int k = c; k < D; k++) {
        const T u = M[c * D + k], v = M[r * D + k];
        M[c * D + k] = sw ? v : u;
        M[r * D + k] = sw ? u : v;
      }
#pragma unroll
      for (int k = 0; k < NR; k++) {
        const T u = R[c * NR + k], v = R[r * NR + k];
        R[c * NR + k] = sw ? v : u;
        R[r * NR + k] = sw ? u : v;
      }
    }
#pragma unroll
    for (int r = c + 1; r < D; r++) {
      const T l = M[r * D + c] / M[c * D + c];
#pragma unroll
      for (int k = c + 1; k < D; k++) M[r * D + k] -= l * M[c * D + k];
#pragma unroll
      for (int k = 0; k < NR; k++) R[r * NR + k] -= l * R[c * NR + k];
    }
  }
#pragma unroll
  for (int c = D - 1; c >= 0; c--)
#pragma unroll
    for (int k = 0; k < NR; k++) {
      T acc = R[c * NR + k];
#pragma unroll
      for (int q = c + 1; q < D; q++) acc -= M[c * D + q] * R[q * NR + k];
      R[c * NR + k] = acc / M[c * D + c];
    }
}

// A step rule supplies, for the step from x_{n-1} = xp to x_n = xc:
//   resid(P, dt, xp, xc, h)        the residual vector the solver tests;
//   element(P, dt, xp, xc, A, b)   the Newton-step element, dx_n = A dx_{n-1} + b;
//   advance(P, dt, xp, xn)         one step of the sequential integrator.
template <typename T, class S, int M>
struct StepRule;

// Explicit RK4 (eqs. root-finding-problem, newton-step-recursion):
// h_n = x_n - Phi(x_{n-1}), A = dPhi/dx(x_{n-1}), b = -h_n.
template <typename T, class S>
struct StepRule<T, S, METHOD_RK4> {
  static constexpr int D = S::D;
  __device__ static void resid(const T* P, T dt, const T* xp, const T* xc, T* h) {
    T phi[D];
    rk4_phi<T, S>(P, dt, xp, phi);
#pragma unroll
    for (int i = 0; i < D; i++) h[i] = xc[i] - phi[i];
  }
  __device__ static void element(const T* P, T dt, const T* xp, const T* xc, T* A, T* b) {
    T phi[D];
    rk4_phi_jac<T, S>(P, dt, xp, phi, A);
#pragma unroll
    for (int i = 0; i < D; i++) b[i] = phi[i] - xc[i];
  }
  __device__ static void advance(const T* P, T dt, const T* xp, T* xn) { rk4_phi<T, S>(P, dt, xp, xn); }
  __device__ static bool advance_ok(const T* P, T dt, const T* xp, T* xn) {
    rk4_phi<T, S>(P, dt, xp, xn);
    return true;
  }
};

// Implicit rules x_n = x_{n-1} + g(x_{n-1}, x_n) (Sec. 3.4, eq. implicit-ode):
// backward Euler g = dt f(x_n); trapezoidal g = dt/2 (f(x_{n-1}) + f(x_n)).
// With H = I - dg/dx_n (the diagonal block of eq. jacobian-implicit) and
// h_n = x_n - x_{n-1} - g, the Newton step of eq.
// newton-step-implicit-recursion is dx_n = H^{-1}(I + dg/dx_{n-1}) dx_{n-1}
// - H^{-1} h_n.  The residual tested is H^{-1} h_n: the quantity the paper
// reports for its implicit solver (its Dahlquist value from the zero guess is
// 1/(1 + dt), not |h_1| = 1).
template <typename T, class S, int M>
struct StepRule {
  static_assert(M == METHOD_BEULER || M == METHOD_TRAP, "unknown step rule");
  static constexpr int D = S::D;
  // h (unscaled), H = I - dg/dx_n, and with WANT_GP, Gp = dg/dx_{n-1}.
  template <bool WANT_GP>
  __device__ static void parts(const T* P, T dt, const T* xp, const T* xc, T* h, T* H, T* Gp) {
    T fc[D];
    S::f(P, xc, fc);
    S::jf(P, xc, H);
    if constexpr (M == METHOD_BEULER) {
#pragma unroll
      for (int i = 0; i < D; i++) h[i] = xc[i] - xp[i] - dt * fc[i];
#pragma unroll
      for (int q = 0; q < D * D; q++) H[q] = -dt * H[q];
      if constexpr (WANT_GP) {
#pragma unroll
        for (int q = 0; q < D * D; q++) Gp[q] = T(0);
      }
    } else {
      const T h2 = T(0.5) * dt;
      T fp[D];
      S::f(P, xp, fp);
#pragma unroll
      for (int i = 0; i < D; i++) h[i] = xc[i] - xp[i] - (h2 * fp[i] + h2 * fc[i]);
#pragma unroll
      for (int q = 0; q < D * D; q++) H[q] = -h2 * H[q];
      if constexpr (WANT_GP) {
        S::jf(P, xp, Gp);
#pragma unroll
        for (int q = 0; q < D * D; q++) Gp[q] = h2 * Gp[q];
      }
    }
#pragma unroll
    for (int i = 0; i < D; i++) H[i * D + i] += T(1);
  }
  __device__ static void resid(const T* P, T dt, const T* xp, const T* xc, T* h) {
    T H[D * D];
    parts<false>(P, dt, xp, xc, h, H, nullptr);
    solve_small<T, D, 1>(H, h);
  }
  __device__ static void element(const T* P, T dt, const T* xp, const T* xc, T* A, T* b) {
    constexpr int NR = D + 1;
    T h[D], H[D * D], Gp[D * D], R[D * NR];
    parts<true>(P, dt, xp, xc, h, H, Gp);
#pragma unroll
    for (int i = 0; i < D; i++) {
#pragma unroll
      for (int j = 0; j < D; j++) R[i * NR + j] = Gp[i * D + j] + (i == j ? T(1) : T(0));
      R[i * NR + D] = -h[i];
    }
    solve_small<T, D, NR>(H, R);
#pragma unroll
    for (int i = 0; i < D; i++) {
#pragma unroll
      for (int j = 0; j < D; j++) A[i * D + j] = R[i * NR + j];
      b[i] = R[i * NR + D];
    }
  }
  // Sequential step: Newton's method on x_n - xp - g(xp, x_n) = 0 from
  // x_n = xp, until the correction is within a few ulps of |x_n| (at most
  // 100 corrections).  advance_ok returns false when the 100 corrections
  // did not get there (a non-finite correction also ends the loop, as
  // converged: the non-finite state reports itself downstream).
  __device__ static bool advance_ok(const T* P, T dt, const T* xp, T* xn) {
    const T stop = sizeof(T) == 8 ? T(4 * 2.220446049250313e-16) : T(32 * 1.1920929e-7);
#pragma unroll
    for (int i = 0; i < D; i++) xn[i] = xp[i];
    for (int it = 0; it < 100; it++) {
      T h[D], H[D * D];
      parts<false>(P, dt, xp, xn, h, H, nullptr);
      solve_small<T, D, 1>(H, h);
      T dn = T(0), yn = T(0);
#pragma unroll
      for (int i = 0; i < D; i++) {
        xn[i] -= h[i];
        dn = fmax(dn, fabs(h[i]));
        yn = fmax(yn, fabs(xn[i]));
      }
      if (!(dn > stop * yn)) return true;
    }
    return false;
  }
  __device__ static void advance(const T* P, T dt, const T* xp, T* xn) {
    (void)advance_ok(P, dt, xp, xn);
  }
};

}  // namespace pint
