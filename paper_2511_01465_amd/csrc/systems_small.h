// Vector fields of small state dimension (d <= 4), evaluated per thread in
// registers, and the classic RK4 step with its exact derivatives.
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

}  // namespace pint
