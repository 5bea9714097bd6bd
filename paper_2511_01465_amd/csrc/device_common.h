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

// Sum over the 64 lanes of two values at once, every lane getting the same
// bits: DPP butterflies inside each row of 16 lanes (quad swaps, then the
// half-row and row mirrors), then the four row sums read from lanes 0, 16,
// 32, 48 and added in a fixed order.  No LDS round trip.
constexpr int DPP_ROW_MIRROR = 0x140;       // lane i <- lane 15 - i within its row
constexpr int DPP_ROW_HALF_MIRROR = 0x141;  // lane i <- lane 7 - i within its half row
__device__ __forceinline__ double read_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <typename T>
__device__ __forceinline__ void wave_sum2_dpp(T& a, T& b);

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

// DPP row operations of a VALU move (gfx9): the value of another lane of
// the same wave without an LDS round trip.  Lanes whose source is out of
// range, or whose row is masked off, get `old`.
constexpr int DPP_ROW_SHR = 0x110;    // + n: lane i <- lane i - n within its row of 16
constexpr int DPP_ROW_BCAST15 = 0x142;  // rows 1, 3 (mask 0xa) <- lane 15 of the row below
constexpr int DPP_ROW_BCAST31 = 0x143;  // rows 2, 3 (mask 0xc) <- lane 31
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_row(double old, double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_row(float old, float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// One level of the wave scan: e <- e o (the map CTRL brings from an earlier
// lane), on the lanes that have one.
template <typename T, int D, int CTRL, int ROW_MASK>
__device__ __forceinline__ void wave_scan_level(Aff<T, D>& e, bool has) {
  Aff<T, D> o;
#pragma unroll
  for (int i = 0; i < D * D; i++) o.A[i] = dpp_row<CTRL, ROW_MASK>(T(0), e.A[i]);
#pragma unroll
  for (int i = 0; i < D; i++) o.b[i] = dpp_row<CTRL, ROW_MASK>(T(0), e.b[i]);
  if (has) aff_after(e, o);
}

// Inclusive scan of one element per lane across the wave: e becomes the
// composition of lanes 0..lane, earliest applied first.  Kogge-Stone within
// rows of 16 lanes (shifts 1, 2, 4, 8), then the rows joined by broadcasts
// of lane 15 (to rows 1, 3) and lane 31 (to rows 2, 3); all DPP moves.
template <typename T, int D>
__device__ __forceinline__ void wave_scan_aff(Aff<T, D>& e) {
  const int lane = threadIdx.x % PINT_WAVE, r = lane & 15;
  wave_scan_level<T, D, DPP_ROW_SHR + 1, 0xf>(e, r >= 1);
  wave_scan_level<T, D, DPP_ROW_SHR + 2, 0xf>(e, r >= 2);
  wave_scan_level<T, D, DPP_ROW_SHR + 4, 0xf>(e, r >= 4);
  wave_scan_level<T, D, DPP_ROW_SHR + 8, 0xf>(e, r >= 8);
  wave_scan_level<T, D, DPP_ROW_BCAST15, 0xa>(e, (lane & 16) != 0);
  wave_scan_level<T, D, DPP_ROW_BCAST31, 0xc>(e, lane >= 32);
}

// Inclusive scan of one element per thread across a block of NT threads
// (NT/64 waves): on return e is the composition of the elements of threads
// 0..threadIdx.x, earliest applied first.  `lds` holds NT/64 elements.
// The wave scan in DPP moves, then wave aggregates through LDS.  Contains
// two workgroup barriers: full ones, or (LDS_ONLY) ones that order LDS only
// and leave this thread's global loads in flight.
template <typename T, int D, int NT, bool LDS_ONLY = false>
__device__ __forceinline__ void block_scan_aff(Aff<T, D>& e, Aff<T, D>* lds) {
  const int lane = threadIdx.x % PINT_WAVE, w = threadIdx.x / PINT_WAVE;
  wave_scan_aff<T, D>(e);
  if (lane == PINT_WAVE - 1) lds[w] = e;
  if constexpr (LDS_ONLY) lds_barrier(); else __syncthreads();
  if (w > 0) {
    Aff<T, D> c = lds[0];
    for (int i = 1; i < w; i++) {
      Aff<T, D> t = lds[i];
      aff_after(t, c);
      c = t;
    }
    aff_after(e, c);
  }
  if constexpr (LDS_ONLY) lds_barrier(); else __syncthreads();
}

template <typename T>
__device__ __forceinline__ void wave_sum2_dpp(T& a, T& b) {
  a += dpp_xor1(a);
  b += dpp_xor1(b);
  a += dpp_xor2(a);
  b += dpp_xor2(b);
  a += dpp_row<DPP_ROW_HALF_MIRROR, 0xf>(T(0), a);
  b += dpp_row<DPP_ROW_HALF_MIRROR, 0xf>(T(0), b);
  a += dpp_row<DPP_ROW_MIRROR, 0xf>(T(0), a);
  b += dpp_row<DPP_ROW_MIRROR, 0xf>(T(0), b);
  a = (read_lane(a, 0) + read_lane(a, 16)) + (read_lane(a, 32) + read_lane(a, 48));
  b = (read_lane(b, 0) + read_lane(b, 16)) + (read_lane(b, 32) + read_lane(b, 48));
}

// ---------------------------------------------------------------- atomics --

__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  // For v >= 0 (including +inf) the IEEE bit patterns order like uint64.
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            (unsigned long long)__double_as_longlong(v));
}

// Bounded wait of one thread on a cross-workgroup condition.  Polls `ready`
// (device-coherent loads inside it) and the instance's error word `err`,
// which any workgroup raises when one of its own waits gives up.  Returns
// false once `ready` holds; true when the error word is set, or when
// `limit` polls have gone by, in which case it raises the error word itself
// (limit 0: at once, without polling).  A caller that gets true must not use
// anything the awaited workgroups publish, and leaves its loop.
template <class F>
__device__ __forceinline__ bool bounded_wait(uint32_t* err, uint64_t limit, F&& ready) {
  for (uint64_t it = 0;; it++) {
    if (it >= limit) {
      atomicOr(err, 1u);
      return true;
    }
    if (ready()) return false;
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
    __builtin_amdgcn_s_sleep(1);
  }
}

}  // namespace pint
