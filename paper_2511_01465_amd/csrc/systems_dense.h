// Vector fields of dense state dimension, evaluated cooperatively by a wave
// (lane l holds components l, l+64, ...), and the columns of the RK4
// Jacobian computed from the stage points each system's way.
#pragma once

#include "device_common.h"

namespace pint {

// Stage points of one RK4 step kept in LDS for the Jacobian threads:
// x[s] is the point where stage s+1 evaluates f (x[0] = x_{n-1}).
template <typename T, int D>
struct StageL96 {
  T x[4][D];
};

template <typename T, int D>
struct StageKur {
  T c[4][D];  // cos of the stage points
  T s[4][D];  // sin of the stage points
  T C[4], S[4];
};

// One row of the banded recursion, b + sum_k band[k] * z[k] over the 13
// diagonals of the Lorenz-96 step Jacobian: the 13 products are independent,
// then summed as a balanced tree (a short dependency chain behind the
// operand loads).  Every solver that folds banded Lorenz-96 elements uses
// this one expression, so their results agree bit for bit.
// Products and sums are spelled out (fma, then rounded adds) so that no
// compiler contraction can make two call sites round differently.
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
template <typename T>
__device__ __forceinline__ T band_row13(T b, const T (&bv)[13], const T (&z)[13]) {
  T q[6];
#pragma unroll
  for (int k = 0; k < 6; k++) q[k] = fma(bv[2 * k], z[2 * k], mul_rn(bv[2 * k + 1], z[2 * k + 1]));
  const T s0 = add_rn(q[0], q[1]), s1 = add_rn(q[2], q[3]), s2 = add_rn(q[4], q[5]);
  const T t = fma(bv[12], z[12], b);
  return add_rn(add_rn(s0, s1), add_rn(s2, t));
}

// ------------------------------------------------------------ Lorenz-96 --

// f_i = (x_{i+1} - x_{i-2}) x_{i-1} - x_i + F, indices mod D (D <= 64).
template <typename T, int DIM>
struct DSysL96 {
  static constexpr int D = DIM, NP = 1, R = 1;
  static constexpr int NT = 256;           // threads per workgroup
  static constexpr int QB = 2;             // threads per Jacobian column
  static constexpr int RB = D / QB;        // rows per thread
  static constexpr int JT = D * QB;        // threads per step for the Jacobian
  static constexpr int SPP = NT >= JT ? NT / JT : 1;  // steps per Jacobian pass
  using Stage = StageL96<T, D>;
  static_assert(D >= 4 && D <= 64 && D % QB == 0 && RB >= 2, "Lorenz-96 dense path");
  // J = dPhi/dx is banded: f_i reads x_{i-2..i+1}, so the four chained stage
  // Jacobians of RK4 reach only j - i in [-8, 4] (cyclic); every other entry
  // is exactly zero.  Band storage: diagonal k = (j - i + BOFF) mod D,
  // k < BW, at band[k * D + i].
  static constexpr bool BANDED = true;
  static constexpr bool MATFREE = false;
  static constexpr int BW = 13, BOFF = 8;
  static_assert(D >= 2 * BW, "band must not wrap onto itself");

  template <bool FAST = false>  // (one form only)
  __device__ static void f(const T* P, const T (&x)[R], T (&out)[R], int lane) {
    const int i = lane < D ? lane : 0;
    const T xp1 = __shfl(x[0], (i + 1) % D, PINT_WAVE);
    const T xm1 = __shfl(x[0], (i + D - 1) % D, PINT_WAVE);
    const T xm2 = __shfl(x[0], (i + D - 2) % D, PINT_WAVE);
    out[0] = (xp1 - xm2) * xm1 - x[0] + P[0];
  }
  // Save stage point s (R values of this lane) into the step's LDS record.
  __device__ static void save_stage(Stage* st, int s, const T (&y)[R], int lane) {
    if (lane < D) st->x[s][lane] = y[0];
  }

  // Thread `sub` (< JT) of a step: rows [q*RB, q*RB+RB) of column j = sub/QB
  // of J = dPhi/dx; element (i, j) goes to out[i * rs + j * cs].  The QB
  // threads of a column are adjacent lanes.  With u the current column of
  // M_s and the cyclic stencil
  //   (Jf u)_i = x_{i-1}(u_{i+1} - u_{i-2}) + (x_{i+1} - x_{i-2}) u_{i-1} - u_i,
  // each thread needs u_{r0-2}, u_{r0-1} and u_{r0+RB} from its neighbours.
  __device__ static void jac_thread(const Stage* st, const T*, int sub, T dt, T* out, int rs, int cs) {
    T col[RB];
    jac_column(st, sub, dt, col);
    const int j = sub / QB, r0 = (sub % QB) * RB;
    T* o = out + j * cs;
#pragma unroll
    for (int k = 0; k < RB; k++) o[(r0 + k) * rs] = col[k];
  }

  // Rows [r0, r0+RB) of column j = sub/QB of J (r0 = (sub%QB)*RB).
  __device__ static void jac_column(const Stage* st, int sub, T dt, T (&col)[RB]) {
    const int j = sub / QB, q = sub % QB, r0 = q * RB;
    const int lane = threadIdx.x % PINT_WAVE, base = lane - q;
    const int nxt = base + (q + 1) % QB, prv = base + (q + QB - 1) % QB;
    const T h2 = T(0.5) * dt, c6 = dt / T(6);
    T u[RB], acc[RB];
#pragma unroll
    for (int i = 0; i < RB; i++) u[i] = (r0 + i == j) ? T(1) : T(0);
#pragma unroll
    for (int s = 0; s < 4; s++) {
      asm volatile("" ::: "memory");  // read this stage's LDS values here, not all up front
      const T* x = st->x[s];
      const T w = (s == 0 || s == 3) ? T(1) : T(2);
      const T c = (s == 2) ? dt : h2;
      // halo (old values): first row of the next part, last two of the previous
      const T up_next = __shfl(u[0], nxt, PINT_WAVE);
      T um1 = __shfl(u[RB - 1], prv, PINT_WAVE);
      T um2 = __shfl(u[RB - 2], prv, PINT_WAVE);
#pragma unroll
      for (int k = 0; k < RB; k++) {
        const int i = r0 + k;
        const int ip1 = i + 1 == D ? 0 : i + 1;
        const int im1 = i == 0 ? D - 1 : i - 1;
        const int im2 = i >= 2 ? i - 2 : i + D - 2;
        const T uk = u[k];
        const T up1 = (k + 1 < RB) ? u[k + 1] : up_next;
        const T K = x[im1] * (up1 - um2) + (x[ip1] - x[im2]) * um1 - uk;
        acc[k] = (s == 0) ? K : acc[k] + w * K;
        u[k] = ((i == j) ? T(1) : T(0)) + c * K;
        um2 = um1;
        um1 = uk;
      }
    }
#pragma unroll
    for (int k = 0; k < RB; k++) col[k] = ((r0 + k == j) ? T(1) : T(0)) + c6 * acc[k];
  }

  // As jac_thread, storing only the band (see BW): element (i, j) with
  // k = (j - i + BOFF) mod D < BW goes to band[k * D + i].
  __device__ static void jac_band_thread(const Stage* st, const T* P, int sub, T dt, T* band) {
    T col[RB];
    jac_column(st, sub, dt, col);
    const int j = sub / QB, r0 = (sub % QB) * RB;
#pragma unroll
    for (int k = 0; k < RB; k++) {
      const int i = r0 + k;
      int kb = j - i + BOFF;
      kb = kb < 0 ? kb + D : (kb >= D ? kb - D : kb);
      if (kb < BW) band[kb * D + i] = col[k];
    }
  }

  // Column j of J restricted to its band, by one thread: the tangent of
  // e_j through the four stages reaches rows j-1..j+2 after the first stage
  // product, and one row down / two rows up per further stage (the stencil
  // reads u_{i+1}, u_{i-2}, u_{i-1}, u_i), so it lives in rows
  // j-4 .. j+8 = j - BOFFT + r, r < BW, throughout; everything outside is
  // exactly zero.  col[r] = J(j - BOFFT + r, j), which is also row j of J^T
  // at band index r (offset BOFFT).
  __device__ static void jac_band_column(const Stage* st, int j, T dt, T (&col)[BW]) {
    static_assert(BW - 1 - BOFF == 4 && BOFF == 8, "stencil reach of the RK4 Jacobian");
    constexpr int LO = BW - 1 - BOFF;   // rows start at j - LO
    constexpr int YW = BW + 3;          // stage values read: rows j-LO-2 .. j-LO+BW
    int yi[YW];
#pragma unroll
    for (int w = 0; w < YW; w++) {
      int g = j - LO - 2 + w;
      g = g < 0 ? g + D : (g >= D ? g - D : g);
      yi[w] = g;
    }
    const T h2 = T(0.5) * dt, c6 = dt / T(6);
    T u[BW], acc[BW];
#pragma unroll
    for (int r = 0; r < BW; r++) {
      u[r] = (r == LO) ? T(1) : T(0);
      acc[r] = T(0);
    }
#pragma unroll
    for (int s = 0; s < 4; s++) {
      // before stage s the tangent is nonzero only in rows LO - s .. LO + 2s
      // (each stage's stencil reaches one row down and two up), so the
      // stage's product is nonzero only in rows LO - 1 - s .. LO + 2 + 2s;
      // the other rows keep their exact zeros
      const int r0 = LO - 1 - s > 0 ? LO - 1 - s : 0;
      const int r1 = LO + 2 + 2 * s < BW - 1 ? LO + 2 + 2 * s : BW - 1;
      const T* x = st->x[s];
      T y[YW];
#pragma unroll
      for (int w = 0; w < YW; w++)
        if (w >= r0 && w <= r1 + 3) y[w] = x[yi[w]];
      const T w_s = (s == 0 || s == 3) ? T(1) : T(2);
      const T c = (s == 2) ? dt : h2;
      T un[BW];
#pragma unroll
      for (int r = 0; r < BW; r++) {
        if (r < r0 || r > r1) {
          un[r] = u[r];
          continue;
        }
        // row i = j - LO + r: y_{i-1} = y[r+1], y_{i+1} = y[r+3], y_{i-2} = y[r]
        const T up1 = r + 1 < BW ? u[r + 1] : T(0);
        const T um1 = r >= 1 ? u[r - 1] : T(0);
        const T um2 = r >= 2 ? u[r - 2] : T(0);
        const T K = y[r + 1] * (up1 - um2) + (y[r + 3] - y[r]) * um1 - u[r];
        acc[r] = (s == 0) ? K : acc[r] + w_s * K;
        un[r] = ((r == LO) ? T(1) : T(0)) + c * K;
      }
#pragma unroll
      for (int r = 0; r < BW; r++) u[r] = un[r];
    }
#pragma unroll
    for (int r = 0; r < BW; r++) col[r] = ((r == LO) ? T(1) : T(0)) + c6 * acc[r];
  }

  // The transpose of the band, row-major: J^T(j, i) = J(i, j) is row j of
  // J^T, whose nonzero entries sit at columns (j + k' - BOFFT) mod D with
  // k' = BW - 1 - kb, BOFFT = BW - 1 - BOFF; stored at bandT[j * BW + k'].
  // The QB threads of column j of J fill row j of J^T (every k' once).
  static constexpr int BOFFT = BW - 1 - BOFF;
  __device__ static void jac_bandT_thread(const Stage* st, const T*, int sub, T dt, T* bandT) {
    T col[RB];
    jac_column(st, sub, dt, col);
    const int j = sub / QB, r0 = (sub % QB) * RB;
#pragma unroll
    for (int k = 0; k < RB; k++) {
      const int i = r0 + k;
      int kb = j - i + BOFF;
      kb = kb < 0 ? kb + D : (kb >= D ? kb - D : kb);
      if (kb < BW) bandT[j * BW + (BW - 1 - kb)] = col[k];
    }
  }
};

// ------------------------------------------------------------- Kuramoto --

// f_i = w_i + K sum_j sin(x_j - x_i) = w_i + K (cos x_i S - sin x_i C) with
// S = sum_j sin x_j, C = sum_j cos x_j (the same sum, expanded).
template <typename T, int DIM>
struct DSysKur {
  static constexpr int D = DIM, NP = DIM + 1, R = (DIM + 63) / 64;
  static constexpr int NT = 256;
  static constexpr int QB = 8;             // threads per Jacobian column
  static constexpr int RB = D / QB;        // rows per thread
  static constexpr int JT = D * QB;        // threads per step for the Jacobian
  static constexpr int SPP = NT >= JT ? NT / JT : 1;
  using Stage = StageKur<T, D>;
  static_assert(D % 64 == 0 && D % QB == 0, "Kuramoto dense path: d a multiple of 64");
  static constexpr bool BANDED = false;  // all-to-all coupling: J is dense
  static constexpr int BW = 0, BOFF = 0;
  // Inside the solvers J is applied without being formed: J_f(y) w =
  // K (c (c.w) + s (s.w)) - K (c C + s S) w costs two dot products over d
  // and O(d) work, so J v goes through the four RK4 stages (tangent) from
  // the stage data alone (cos, sin and their sums at the stage points:
  // STAGE_SCALARS values per step instead of d^2).
  static constexpr bool MATFREE = true;
  static constexpr int STAGE_SCALARS = 8 * D + 8;
  static_assert(sizeof(StageKur<T, D>) == STAGE_SCALARS * sizeof(T), "stage record layout");

  // FAST: the two wave sums as DPP row permutes (vector ALU) instead of a
  // shuffle butterfly (LDS unit); different rounding order.  Used where one
  // wave runs alone (the sequential integrator); the Newton solvers' many
  // element waves are bound by the vector ALU and keep the butterfly.
  template <bool FAST = false>
  __device__ static void sums(const T (&x)[R], T (&sn)[R], T (&cs)[R], T& S, T& C, int lane) {
    T ls = T(0), lc = T(0);
#pragma unroll
    for (int r = 0; r < R; r++) {
      if constexpr (sizeof(T) == 8)
        sincos(x[r], &sn[r], &cs[r]);  // one argument reduction for both
      else
        sincosf(x[r], &sn[r], &cs[r]);
      ls += sn[r];
      lc += cs[r];
    }
    if constexpr (FAST) {
      wave_sum2_dpp(ls, lc);
      S = ls;
      C = lc;
    } else {
      S = wave_sum(ls);
      C = wave_sum(lc);
    }
  }
  template <bool FAST = false>
  __device__ static void f(const T* P, const T (&x)[R], T (&out)[R], int lane) {
    T sn[R], cs[R], S, C;
    sums<FAST>(x, sn, cs, S, C, lane);
#pragma unroll
    for (int r = 0; r < R; r++) out[r] = P[1 + lane + 64 * r] + P[0] * (cs[r] * S - sn[r] * C);
  }
  __device__ static void save_stage(Stage* st, int s, const T (&y)[R], int lane) {
    T sn[R], cs[R], S, C;
    sums(y, sn, cs, S, C, lane);
#pragma unroll
    for (int r = 0; r < R; r++) {
      st->c[s][lane + 64 * r] = cs[r];
      st->s[s][lane + 64 * r] = sn[r];
    }
    if (lane == 0) {
      st->S[s] = S;
      st->C[s] = C;
    }
  }

  // Rows [q*RB, q*RB+RB) of column j = sub/QB of J = dPhi/dx.  With
  // c = cos x, s = sin x:  (Jf u)_i = K (c_i (c.u) + s_i (s.u))
  // - K (c_i C + s_i S) u_i, the dot products reduced over the QB adjacent
  // lanes of the column.
  __device__ static void jac_thread(const Stage* st, const T* P, int sub, T dt, T* out, int rs, int cs_) {
    const int j = sub / QB, q = sub % QB, r0 = q * RB;
    const T h2 = T(0.5) * dt, c6 = dt / T(6), Kc = P[0];
    T u[RB], acc[RB];
#pragma unroll
    for (int i = 0; i < RB; i++) u[i] = (r0 + i == j) ? T(1) : T(0);
#pragma unroll
    for (int s = 0; s < 4; s++) {
      asm volatile("" ::: "memory");  // read this stage's LDS values here, not all up front
      const T* cs = st->c[s] + r0;
      const T* sn = st->s[s] + r0;
      T a = T(0), b = T(0);
#pragma unroll
      for (int i = 0; i < RB; i++) {
        a += cs[i] * u[i];
        b += sn[i] * u[i];
      }
#pragma unroll
      for (int off = 1; off < QB; off <<= 1) {
        a += __shfl_xor(a, off, PINT_WAVE);
        b += __shfl_xor(b, off, PINT_WAVE);
      }
      const T C = st->C[s], S = st->S[s];
      const T w = (s == 0 || s == 3) ? T(1) : T(2);
      const T c = (s == 2) ? dt : h2;
#pragma unroll
      for (int i = 0; i < RB; i++) {
        const T ci = cs[i], si = sn[i];
        const T K = Kc * (ci * a + si * b) - Kc * (ci * C + si * S) * u[i];
        acc[i] = (s == 0) ? K : acc[i] + w * K;
        u[i] = ((r0 + i == j) ? T(1) : T(0)) + c * K;
      }
    }
    T* o = out + j * cs_;
#pragma unroll
    for (int i = 0; i < RB; i++) o[(r0 + i) * rs] = ((r0 + i == j) ? T(1) : T(0)) + c6 * acc[i];
  }
};

// --------------------------------------------------------- wave RK4 step --

// One RK4 step of a dense system by one wave.  x: this lane's components of
// x_{n-1}; returns phi.  If st != nullptr the four stage points are saved.
// FAST selects S::f's other form where it has one (see DSysKur::sums).
template <typename T, class S, bool FAST = false>
__device__ __forceinline__ void wave_rk4(const T* P, T dt, const T (&x)[S::R], T (&phi)[S::R],
                                         typename S::Stage* st, int lane) {
  constexpr int R = S::R;
  T k[R], acc[R], y[R];
  const T h2 = T(0.5) * dt, c6 = dt / T(6);
  if (st) S::save_stage(st, 0, x, lane);
  S::template f<FAST>(P, x, k, lane);
#pragma unroll
  for (int r = 0; r < R; r++) { acc[r] = k[r]; y[r] = x[r] + h2 * k[r]; }
  if (st) S::save_stage(st, 1, y, lane);
  S::template f<FAST>(P, y, k, lane);
#pragma unroll
  for (int r = 0; r < R; r++) { acc[r] += T(2) * k[r]; y[r] = x[r] + h2 * k[r]; }
  if (st) S::save_stage(st, 2, y, lane);
  S::template f<FAST>(P, y, k, lane);
#pragma unroll
  for (int r = 0; r < R; r++) { acc[r] += T(2) * k[r]; y[r] = x[r] + dt * k[r]; }
  if (st) S::save_stage(st, 3, y, lane);
  S::template f<FAST>(P, y, k, lane);
#pragma unroll
  for (int r = 0; r < R; r++) phi[r] = x[r] + c6 * (acc[r] + k[r]);
}

}  // namespace pint
