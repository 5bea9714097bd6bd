// Device-side building blocks shared by the libpint kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PINT_WAVE 64

namespace pint {

// ---------------------------------------------------------------- scalars --

template <typename T>
__device__ __forceinline__ bool finite_(T v) {
  return isfinite(v);
}

// Infinity norm accumulation: returns +inf as soon as a non-finite entry is
// seen (NaN must not vanish through fmax).
template <typename T>
__device__ __forceinline__ double acc_norm(double m, T v) {
  if (!finite_(v)) return INFINITY;
  double a = fabs((double)v);
  return a > m ? a : m;
}

// ---------------------------------------------------- wave / block reduce --

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, PINT_WAVE));
  return v;
}

__device__ __forceinline__ int64_t wave_min_i64(int64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    int64_t o = __shfl_xor(v, off, PINT_WAVE);
    v = o < v ? o : v;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, PINT_WAVE);
  return v;
}

// Butterfly exchanges inside each group of four lanes, as DPP quad
// permutations of a VALU move (no LDS round trip): dpp_xor1 returns the value
// of lane l^1, dpp_xor2 that of lane l^2.  Every lane of the quad must be
// active.
template <int CTRL>
__device__ __forceinline__ int dpp_quad(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, false);
}
constexpr int DPP_QUAD_XOR1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;  // quad_perm [2,3,0,1]

template <int CTRL>
__device__ __forceinline__ double dpp_quad(double v) {
  const int lo = dpp_quad<CTRL>(__double2loint(v)), hi = dpp_quad<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_quad(float v) {
  return __int_as_float(dpp_quad<CTRL>(__float_as_int(v)));
}
template <typename T>
__device__ __forceinline__ T dpp_xor1(T v) { return dpp_quad<DPP_QUAD_XOR1>(v); }
template <typename T>
__device__ __forceinline__ T dpp_xor2(T v) { return dpp_quad<DPP_QUAD_XOR2>(v); }

// Block-wide reductions for blockDim.x = NT (a multiple of 64).  `red` is a
// shared scratch of at least NT/64 doubles; the result is returned to every
// thread.  Contains two __syncthreads.
template <int NT>
__device__ __forceinline__ double block_max(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x / PINT_WAVE, l = threadIdx.x % PINT_WAVE;
  if (l == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int i = 1; i < NT / PINT_WAVE; i++) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t* red) {
  v = wave_min_i64(v);
  const int w = threadIdx.x / PINT_WAVE, l = threadIdx.x % PINT_WAVE;
  if (l == 0) red[w] = v;
  __syncthreads();
  int64_t r = red[0];
#pragma unroll
  for (int i = 1; i < NT / PINT_WAVE; i++) r = red[i] < r ? red[i] : r;
  __syncthreads();
  return r;
}

// Workgroup barrier that orders LDS only: it waits for this wave's LDS
// operations but leaves its outstanding global loads in flight, so register
// prefetches survive it (__syncthreads waits for every memory operation).
// Only for loops whose cross-wave communication is through LDS.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ------------------------------------------------------- affine elements --

// An affine map z -> A z + b on R^D (A row-major).
template <typename T, int D>
struct Aff {
  T A[D * D];
  T b[D];
};

template <typename T, int D>
__device__ __forceinline__ void aff_identity(Aff<T, D>& e) {
#pragma unroll
  for (int i = 0; i < D; i++) {
#pragma unroll
    for (int j = 0; j < D; j++) e.A[i * D + j] = (i == j) ? T(1) : T(0);
    e.b[i] = T(0);
  }
}

// l <- l o e : first e, then l.  (A_l A_e, A_l b_e + b_l)
template <typename T, int D>
__device__ __forceinline__ void aff_after(Aff<T, D>& l, const Aff<T, D>& e) {
  Aff<T, D> r;
#pragma unroll
  for (int i = 0; i < D; i++) {
#pragma unroll
    for (int j = 0; j < D; j++) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < D; k++) acc += l.A[i * D + k] * e.A[k * D + j];
      r.A[i * D + j] = acc;
    }
    T acc = l.b[i];
#pragma unroll
    for (int k = 0; k < D; k++) acc += l.A[i * D + k] * e.b[k];
    r.b[i] = acc;
  }
  l = r;
}

template <typename T, int D>
__device__ __forceinline__ void aff_shfl_up(Aff<T, D>& out, const Aff<T, D>& in, int delta) {
#pragma unroll
  for (int i = 0; i < D * D; i++) out.A[i] = __shfl_up(in.A[i], delta, PINT_WAVE);
#pragma unroll
  for (int i = 0; i < D; i++) out.b[i] = __shfl_up(in.b[i], delta, PINT_WAVE);
}

// Inclusive scan of one element per thread across a block of NT threads
// (NT/64 waves): on return e is the composition of the elements of threads
// 0..threadIdx.x, earliest applied first.  `lds` holds NT/64 elements.
// Kogge-Stone inside each wave via shuffles, then wave aggregates through
// LDS.  Contains two __syncthreads.
template <typename T, int D, int NT>
__device__ __forceinline__ void block_scan_aff(Aff<T, D>& e, Aff<T, D>* lds) {
  const int lane = threadIdx.x % PINT_WAVE, w = threadIdx.x / PINT_WAVE;
#pragma unroll
  for (int off = 1; off < PINT_WAVE; off <<= 1) {
    Aff<T, D> prev;
    aff_shfl_up(prev, e, off);
    if (lane >= off) aff_after(e, prev);
  }
  if (lane == PINT_WAVE - 1) lds[w] = e;
  __syncthreads();
  if (w > 0) {
    Aff<T, D> c = lds[0];
    for (int i = 1; i < w; i++) {
      Aff<T, D> t = lds[i];
      aff_after(t, c);
      c = t;
    }
    aff_after(e, c);
  }
  __syncthreads();
}

// ---------------------------------------------------------------- atomics --

__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  // For v >= 0 (including +inf) the IEEE bit patterns order like uint64.
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            (unsigned long long)__double_as_longlong(v));
}

}  // namespace pint
