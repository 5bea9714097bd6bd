// Small state dimension (d <= 4): one workgroup per instance runs the whole
// Newton loop of Sec. 3.2 (Sec. 3.4 for the implicit rules) on chip —
// residual, stop test, window search, element construction, affine scan and
// update — pulling instances from a device work queue, so a batch of any
// size and mix of horizons is one persistent launch.  Also the sequential
// comparator and the residual / element kernels used for checking.  Every
// kernel is templated on the step rule M (StepRule in systems_small.h); the
// launchers are instantiated per rule in newton_small.hip (RK4) and
// implicit_small.hip (backward Euler, trapezoidal).
#pragma once

#include "internal.h"
#include "systems_small.h"

namespace pint {

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
  uint64_t wait_limit;   // cooperative solver: polls before a wait gives up
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

// Infinity norm of the residual the rule tests at step n (eq.
// root-finding-problem for RK4), +inf if anything is non-finite.
template <typename T, class S, int M>
__device__ __forceinline__ double step_resid(const T* P, T dt, const T* X, const T* x0, int64_t n) {
  constexpr int D = S::D;
  T xp[D], xc[D], h[D];
  load_state<T, D>(X, x0, n - 1, xp);
  load_state<T, D>(X, x0, n, xc);
  StepRule<T, S, M>::resid(P, dt, xp, xc, h);
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < D; i++) m = acc_norm(m, h[i]);
  return m;
}

template <typename T, class S, int M, int NT>
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
          if (n <= Tn) r = fmax(r, step_resid<T, S, M>(P, dt, X, x0, n));
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
            hn = step_resid<T, S, M>(P, dt, X, x0, n);
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

      // Newton step over [lo, hi] (eq. newton-step-recursion, or
      // newton-step-implicit-recursion): the elements of the rule are
      // scanned chunk by chunk from dx_{lo-1} = 0.
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
          T xp[D];
          if (tid == 0) {
#pragma unroll
            for (int i = 0; i < D; i++) xp[i] = s_xprev[i];
          } else {
#pragma unroll
            for (int i = 0; i < D; i++) xp[i] = X[(n - 2) * D + i];
          }
#pragma unroll
          for (int i = 0; i < D; i++) xc[i] = X[(n - 1) * D + i];
          StepRule<T, S, M>::element(P, dt, xp, xc, e.A, e.b);
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
    for (int64_t n = 1 + tid; n <= Tn; n += NT) r = fmax(r, step_resid<T, S, M>(P, dt, X, x0, n));
    r = block_max<NT>(r, s_red);
    if (tid == 0) {
      a.iters[inst] = k;
      a.resid[inst] = r;
      a.status[inst] = st;
    }
    __syncthreads();
  }
}

// ------------------------------------------------ cooperative variant --

// Cross-workgroup data of the cooperative solver moves with device-scope
// atomic stores and loads, which are coherent across the chip's L2 slices
// by themselves: a writer waits for its stores to complete (vmcnt) before
// it raises a counter or flag, a reader loads only after it has seen it.
// No device-wide cache writeback or invalidate is needed, because no
// workgroup reads trajectory states that another workgroup wrote.
template <typename T>
__device__ __forceinline__ void co_store(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T co_load(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-instance control block (64 bytes) and the counters of its barrier
// groups (16 workgroups each, one 64-byte line per counter).
struct SmallCtl {
  uint32_t gen, top, err, pad[13];
};
static_assert(sizeof(SmallCtl) == 64, "control block size");
constexpr int COOP_GROUP = 16;
constexpr int LINE_U32 = 16;

// Two-level barrier among the G workgroups of one instance: a workgroup
// arrives on its group's counter; the last of a group arrives on the top
// counter; the last of those resets the counters and raises the generation
// that everyone waits for.  The wait is bounded (bounded_wait); returns, in
// every thread, true if the instance's error word was seen (a wait of this
// or another workgroup gave up), and the caller leaves its loop.
__device__ __forceinline__ bool coop_sync(SmallCtl* c, uint32_t* grp, int G, int g, uint32_t& gen,
                                          uint64_t limit) {
  __shared__ int s_fail;
  __syncthreads();
  if (threadIdx.x == 0) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's posts are complete
    const uint32_t target = gen + 1;
    const int gi = g / COOP_GROUP;
    const int gsize = (G - gi * COOP_GROUP) < COOP_GROUP ? (G - gi * COOP_GROUP) : COOP_GROUP;
    const int ngrp = (G + COOP_GROUP - 1) / COOP_GROUP;
    bool released = false;
    const uint32_t prev = atomicAdd(&grp[gi * LINE_U32], 1u);
    if (prev == (uint32_t)(gsize - 1)) {
      co_store(&grp[gi * LINE_U32], 0u);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      const uint32_t p2 = atomicAdd(&c->top, 1u);
      if (p2 == (uint32_t)(ngrp - 1)) {
        co_store(&c->top, 0u);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        co_store(&c->gen, target);
        released = true;
      }
    }
    bool fail = false;
    if (!released) fail = bounded_wait(&c->err, limit, [&] { return co_load(&c->gen) == target; });
    gen = target;
    s_fail = fail;
  }
  __syncthreads();
  return s_fail != 0;
}

// Workspace of the cooperative solver, per instance (offsets in bytes from
// the instance's base; see small_coop_stride on the host).
struct CoopLayout {
  int G, ngrp;
  size_t grp_off, agg_off, r_off, bnd_off, flag_off, stride;
};

__host__ __device__ inline CoopLayout coop_layout(int G, int D, int elem_bytes) {
  CoopLayout l{};
  const size_t E = (size_t)D * D + D;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  l.G = G;
  l.ngrp = (G + COOP_GROUP - 1) / COOP_GROUP;
  l.grp_off = up(sizeof(SmallCtl));
  l.agg_off = l.grp_off + up((size_t)l.ngrp * LINE_U32 * 4);
  l.r_off = l.agg_off + up(2 * (size_t)G * E * elem_bytes);
  l.bnd_off = l.r_off + up(2 * (size_t)G * 8);
  l.flag_off = l.bnd_off + up(2 * (size_t)G * D * elem_bytes);
  l.stride = l.flag_off + up((size_t)G * LINE_U32 * 4);
  return l;
}

// The paper's plain Newton method (Sec. 3.2 / 3.4) for a few long
// instances, each spread over G co-resident workgroups (cooperative
// launch); workgroup g owns the contiguous steps [1 + gL, min(T, (g+1)L)],
// L = ceil(T / G).  Per iteration k:
//   A. with x_{lo-1} (x0, or the state workgroup g-1 published at the end
//      of iteration k-1), each workgroup evaluates the elements of its
//      steps in registers (the Jacobians are never stored), their residual
//      maximum and the composition of its elements, and posts both;
//   B. after one barrier every workgroup reads all posts: the global
//      residual gives the stop decision (the same everywhere), the
//      compositions of the workgroups before it, scanned in LDS, give dx at
//      the start of its range;
//   C. it re-evaluates its elements, scans them chunk by chunk from that dx,
//      writes x += dx in place and publishes its new last state for
//      workgroup g+1.
// Posts are double-buffered by the parity of k.  Results, iteration counts
// and status follow k_newton_small's plain mode.
template <typename T, class S, int M, int NT>
__global__ __launch_bounds__(NT) void k_newton_small_coop(SmallKArgs a, int G, char* ws) {
  constexpr int D = S::D, NP = S::NP, E = D * D + D;
  // Ranges of at most KC chunks keep phase A's scanned elements and old
  // states in registers, so phase C only applies them to the carry-in (x is
  // read once and written once per iteration); longer ranges re-evaluate.
  constexpr int KC = D <= 2 ? 2 : (D == 3 ? 1 : 0);
  constexpr int KR = KC > 0 ? KC : 1;
  __shared__ Aff<T, D> s_aff[NT / PINT_WAVE];
  __shared__ double s_red[NT / PINT_WAVE];
  __shared__ T s_z[D], s_xprev[D], s_xlast[D], s_zlast[D], s_xb[D];
  __shared__ Aff<T, D> s_run;
  __shared__ Aff<T, D> s_cagg[KR];
  __shared__ int s_fail;
  const int tid = threadIdx.x;
  const int64_t inst = blockIdx.x / G;
  const int g = (int)(blockIdx.x % G);
  const CoopLayout lay = coop_layout(G, D, (int)sizeof(T));
  char* base = ws + inst * lay.stride;
  SmallCtl* c = reinterpret_cast<SmallCtl*>(base);
  uint32_t* grp = reinterpret_cast<uint32_t*>(base + lay.grp_off);
  T* post_agg = reinterpret_cast<T*>(base + lay.agg_off);      // [2][G][E]
  double* post_r = reinterpret_cast<double*>(base + lay.r_off);  // [2][G]
  T* bnd = reinterpret_cast<T*>(base + lay.bnd_off);            // [2][G][D]
  uint32_t* bflag = reinterpret_cast<uint32_t*>(base + lay.flag_off);  // [G] (one line each)
  const T dt = (T)a.dt;
  const int64_t Tn = a.T_uniform;
  T* X = static_cast<T*>(a.traj) + inst * Tn * D;
  const T* xg = static_cast<const T*>(a.x0) + inst * D;
  T P[NP], x0[D];
  {
    const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
#pragma unroll
    for (int i = 0; i < NP; i++) P[i] = Pg[i];
#pragma unroll
    for (int i = 0; i < D; i++) x0[i] = xg[i];
  }
  const int64_t L = (Tn + G - 1) / G;
  const int64_t lo = 1 + (int64_t)g * L;
  const int64_t hi = (int64_t)(g + 1) * L < Tn ? (int64_t)(g + 1) * L : Tn;  // empty when lo > hi
  const int nch = lo <= hi ? (int)((hi - lo) / NT + 1) : 0;
  const bool fast = nch <= KC;
  Aff<T, D> eS[KR];
  T xS[KR][D];
  if (a.guess == 0)
    for (int64_t n = lo + tid; n <= hi; n += NT)
#pragma unroll
      for (int i = 0; i < D; i++) X[(n - 1) * D + i] = x0[i];
  // x_{lo-1} of the first iteration: x0, or the caller's initial iterate
  // (read before any workgroup can have updated it: workgroup g-1 writes
  // only after the first barrier, which waits for this workgroup)
  if (tid < D) {
    const int64_t jb = (lo >= 2 && lo <= hi) ? lo - 2 : 0;  // clamped into the trajectory
    const T xv = X[jb * D + tid];
    s_xb[tid] = (lo == 1 || lo > hi || a.guess == 0) ? xg[tid] : xv;
  }
  uint32_t gen = 0;
  int64_t k = 0;
  int st = ST_OK;
  double rg = 0.0;
  for (;;) {
    const int par = (int)(k & 1);
    // ---- A: residual maximum and composition of this workgroup's elements
    if (k > 0 && g > 0 && lo <= hi) {
      if (tid == 0)  // the state workgroup g-1 published at the end of iteration k-1
        s_fail = bounded_wait(&c->err, a.wait_limit,
                              [&] { return co_load(&bflag[(g - 1) * LINE_U32]) >= (uint32_t)k; });
      __syncthreads();
      if (s_fail) { st = ST_DEVICE; break; }
      if (tid < D) s_xb[tid] = co_load(&bnd[((1 - par) * G + (g - 1)) * D + tid]);
    }
    if (tid == 0) aff_identity(s_run);
    __syncthreads();
    double r = 0.0;
    // one chunk of phase A: element of step n (identity past the range),
    // residual, in-chunk inclusive scan, composition into the range's map
    auto chunk_a = [&](int64_t c0, Aff<T, D>& e, T (&xc)[D]) {
      const int64_t n = c0 + tid;
      if (n <= hi) {
        T xp[D];
        const T* xq = X + (n >= 2 ? n - 2 : 0) * D;  // x_{n-1} when n > lo
#pragma unroll
        for (int i = 0; i < D; i++) {
          xp[i] = (n == lo) ? s_xb[i] : xq[i];
          xc[i] = X[(n - 1) * D + i];
        }
        StepRule<T, S, M>::element(P, dt, xp, xc, e.A, e.b);
#pragma unroll
        for (int i = 0; i < D; i++) r = acc_norm(r, e.b[i]);  // |b_n| is the tested residual
      } else {
        aff_identity(e);
#pragma unroll
        for (int i = 0; i < D; i++) xc[i] = T(0);
      }
      block_scan_aff<T, D, NT>(e, s_aff);
      if (tid == NT - 1) {
        Aff<T, D> run = s_run;
        Aff<T, D> ch = e;
        aff_after(ch, run);  // this chunk after everything before it
        s_run = ch;
      }
      __syncthreads();
    };
    if (fast) {
#pragma unroll
      for (int ci = 0; ci < KC; ci++)
        if (ci < nch) {
          chunk_a(lo + (int64_t)ci * NT, eS[ci], xS[ci]);
          if (tid == NT - 1) s_cagg[ci] = eS[ci];
        }
    } else {
      for (int64_t c0 = lo; c0 <= hi; c0 += NT) {
        Aff<T, D> e;
        T xc[D];
        chunk_a(c0, e, xc);
      }
    }
    r = block_max<NT>(r, s_red);
    if (tid < D * D) co_store(&post_agg[(par * G + g) * E + tid], s_run.A[tid]);
    if (tid < D) co_store(&post_agg[(par * G + g) * E + D * D + tid], s_run.b[tid]);
    if (tid == 0) co_store(&post_r[par * G + g], r);
    if (coop_sync(c, grp, G, g, gen, a.wait_limit)) { st = ST_DEVICE; break; }

    // ---- B: global residual and stop test; dx at the start of this range
    double rr = 0.0;
    for (int j = tid; j < G; j += NT) rr = fmax(rr, co_load(&post_r[par * G + j]));
    rg = block_max<NT>(rr, s_red);
    if (!(rg < INFINITY)) { st = ST_NONFINITE; break; }
    if (rg < a.tol) { st = ST_OK; break; }
    if (k >= a.max_iter) { st = ST_NOT_CONVERGED; break; }
    {
      // compositions 0..g-1 in order: thread t folds a contiguous run of
      // them, then a block scan; the whole map applied to dx = 0 is its b-part
      const int q = (g + NT - 1) / NT;
      Aff<T, D> e;
      aff_identity(e);
      for (int j = tid * q; j < (tid + 1) * q && j < g; j++) {
        Aff<T, D> f;
        const T* pj = post_agg + (par * G + j) * E;
#pragma unroll
        for (int i = 0; i < D * D; i++) f.A[i] = co_load(&pj[i]);
#pragma unroll
        for (int i = 0; i < D; i++) f.b[i] = co_load(&pj[D * D + i]);
        aff_after(f, e);
        e = f;
      }
      block_scan_aff<T, D, NT>(e, s_aff);
      if (tid == NT - 1) {
#pragma unroll
        for (int i = 0; i < D; i++) s_z[i] = e.b[i];
      }
      if (tid < D) s_xprev[tid] = s_xb[tid];
      __syncthreads();
    }

    // ---- C: the update over this workgroup's range
    if (fast) {
      // dx_n = (in-chunk prefix of step n) applied to dx at the chunk's
      // start; that dx goes from chunk to chunk through the chunk maps
      T z[D];
#pragma unroll
      for (int i = 0; i < D; i++) z[i] = s_z[i];
#pragma unroll
      for (int ci = 0; ci < KC; ci++)
        if (ci < nch) {
          const int64_t n = lo + (int64_t)ci * NT + tid;
          if (n <= hi) {
            T xn[D];
#pragma unroll
            for (int i = 0; i < D; i++) {
              T acc = eS[ci].b[i];
#pragma unroll
              for (int j = 0; j < D; j++) acc += eS[ci].A[i * D + j] * z[j];
              xn[i] = xS[ci][i] + acc;
              X[(n - 1) * D + i] = xn[i];
            }
            if (n == hi && g + 1 < G) {  // publish the new last state for workgroup g+1
#pragma unroll
              for (int i = 0; i < D; i++) co_store(&bnd[(par * G + g) * D + i], xn[i]);
              asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
              co_store(&bflag[g * LINE_U32], (uint32_t)(k + 1));
            }
          }
          const Aff<T, D> cg = s_cagg[ci];
          T zn[D];
#pragma unroll
          for (int i = 0; i < D; i++) {
            T acc = cg.b[i];
#pragma unroll
            for (int j = 0; j < D; j++) acc += cg.A[i * D + j] * z[j];
            zn[i] = acc;
          }
#pragma unroll
          for (int i = 0; i < D; i++) z[i] = zn[i];
        }
      __syncthreads();
    }
    for (int64_t c0 = lo; c0 <= hi && !fast; c0 += NT) {
      const int64_t n = c0 + tid;
      const bool act = n <= hi;
      T xc[D];
      Aff<T, D> e;
      if (act) {
        T xp[D];
        const T* xq = X + (n >= 2 ? n - 2 : 0) * D;  // x_{n-1} when tid > 0
#pragma unroll
        for (int i = 0; i < D; i++) {
          xp[i] = (tid == 0) ? s_xprev[i] : xq[i];
          xc[i] = X[(n - 1) * D + i];
        }
        StepRule<T, S, M>::element(P, dt, xp, xc, e.A, e.b);
      } else {
        aff_identity(e);
#pragma unroll
        for (int i = 0; i < D; i++) xc[i] = T(0);
      }
      block_scan_aff<T, D, NT>(e, s_aff);
      T dx[D];
#pragma unroll
      for (int i = 0; i < D; i++) {
        T acc = e.b[i];
#pragma unroll
        for (int j = 0; j < D; j++) acc += e.A[i * D + j] * s_z[j];
        dx[i] = acc;
      }
      const int64_t last = (hi < c0 + NT - 1) ? hi : c0 + NT - 1;
      if (n == last) {
#pragma unroll
        for (int i = 0; i < D; i++) { s_xlast[i] = xc[i]; s_zlast[i] = dx[i]; }
      }
      if (act) {
#pragma unroll
        for (int i = 0; i < D; i++) X[(n - 1) * D + i] = xc[i] + dx[i];
      }
      if (n == hi && g + 1 < G) {  // publish the new last state for workgroup g+1
#pragma unroll
        for (int i = 0; i < D; i++) co_store(&bnd[(par * G + g) * D + i], xc[i] + dx[i]);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        co_store(&bflag[g * LINE_U32], (uint32_t)(k + 1));
      }
      __syncthreads();
      if (tid < D) { s_xprev[tid] = s_xlast[tid]; s_z[tid] = s_zlast[tid]; }
      __syncthreads();
    }
    k++;
  }
  if (g == 0 && tid == 0) {
    a.iters[inst] = k;
    a.resid[inst] = rg;
    // a bounded wait that gave up (error word) makes the result unreliable
    a.status[inst] = co_load(&c->err) ? ST_DEVICE : st;
  }
}

// Sequential comparator: one thread per instance, x_n from x_{n-1} by the
// rule's own step (RK4, or a converged per-step Newton solve).
template <typename T, class S, int M>
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
    StepRule<T, S, M>::advance(P, dt, x, y);
#pragma unroll
    for (int i = 0; i < D; i++) {
      x[i] = y[i];
      X[n * D + i] = y[i];
    }
  }
}

// The rule's residual for every (instance, step) of a uniform batch, and
// the per-instance max.
template <typename T, class S, int M>
__global__ void k_residual_small(SmallKArgs a, T* h, double* hmax) {
  constexpr int D = S::D, NP = S::NP;
  const int64_t total = a.B * a.T_uniform;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t inst = g / a.T_uniform, n = g % a.T_uniform + 1;
    const T* X = static_cast<const T*>(a.traj) + inst * a.T_uniform * D;
    const T* x0 = static_cast<const T*>(a.x0) + inst * D;
    T P[NP], xp[D], xc[D], hv[D];
    const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
#pragma unroll
    for (int i = 0; i < NP; i++) P[i] = Pg[i];
    load_state<T, D>(X, x0, n - 1, xp);
    load_state<T, D>(X, x0, n, xc);
    StepRule<T, S, M>::resid(P, (T)a.dt, xp, xc, hv);
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < D; i++) {
      if (h) h[g * D + i] = hv[i];
      m = acc_norm(m, hv[i]);
    }
    atomic_max_nonneg(hmax + inst, m);
  }
}

// Elements (A_n, b_n) of the step from x_n to x_{n+1}, n = 0..T-1.
template <typename T, class S, int M>
__global__ void k_elements_small(SmallKArgs a, T* A, T* b) {
  constexpr int D = S::D, NP = S::NP;
  const int64_t total = a.B * a.T_uniform;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t inst = g / a.T_uniform, n = g % a.T_uniform;
    const T* X = static_cast<const T*>(a.traj) + inst * a.T_uniform * D;
    const T* x0 = static_cast<const T*>(a.x0) + inst * D;
    T P[NP], xn[D], xnext[D], J[D * D], bv[D];
    const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
#pragma unroll
    for (int i = 0; i < NP; i++) P[i] = Pg[i];
    load_state<T, D>(X, x0, n, xn);
    load_state<T, D>(X, x0, n + 1, xnext);
    StepRule<T, S, M>::element(P, (T)a.dt, xn, xnext, J, bv);
#pragma unroll
    for (int i = 0; i < D * D; i++) A[g * D * D + i] = J[i];
#pragma unroll
    for (int i = 0; i < D; i++) b[g * D + i] = bv[i];
  }
}

// ------------------------------------------------------------- dispatch --

template <typename T, typename F>
int dispatch_small_sys(int system, int d, F&& f) {
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
    case 7: if (d == 3) return f(SysRobertson<T>{}); break;
  }
  return ST_UNSUPPORTED;
}

template <typename F>
int dispatch_small(int dtype, int system, int d, F&& f) {
  if (dtype == 0) return dispatch_small_sys<double>(system, d, [&](auto s) { return f((double)0, s); });
  if (dtype == 1) return dispatch_small_sys<float>(system, d, [&](auto s) { return f((float)0, s); });
  return ST_UNSUPPORTED;
}

// One launch of the small-d kernels for rule M; which kernel by `op`.
enum SmallOp { OP_SOLVE = 0, OP_SEQ = 1, OP_RESIDUAL = 2, OP_ELEMENTS = 3, OP_COOP = 4,
               OP_COOP_OCCUPANCY = 5 };

constexpr int NT_COOP = 256;  // threads per workgroup of the cooperative solver

struct SmallLaunch {
  int op, dtype, system, d;
  int grid, block;
  hipStream_t stream;
  void* out0;      // residual: h; elements: A
  void* out1;      // elements: b
  double* hmax;    // residual
  char* coop_ws;   // coop: per-instance control blocks and posts (coop_layout)
  int G;           // coop: workgroups per instance
  int* occupancy;  // coop occupancy query: resident workgroups per CU
};

template <int M>
int small_launch(const SmallKArgs& k, const SmallLaunch& l) {
  return dispatch_small(l.dtype, l.system, l.d, [&](auto t, auto s) -> int {
    using T = decltype(t);
    using S = decltype(s);
    switch (l.op) {
      case OP_SOLVE:
        switch (l.block) {
          case 64: hipLaunchKernelGGL((k_newton_small<T, S, M, 64>), dim3(l.grid), dim3(64), 0, l.stream, k); break;
          case 128: hipLaunchKernelGGL((k_newton_small<T, S, M, 128>), dim3(l.grid), dim3(128), 0, l.stream, k); break;
          case 256: hipLaunchKernelGGL((k_newton_small<T, S, M, 256>), dim3(l.grid), dim3(256), 0, l.stream, k); break;
          default: return ST_INVALID;
        }
        break;
      case OP_SEQ:
        hipLaunchKernelGGL((k_seq_small<T, S, M>), dim3(l.grid), dim3(l.block), 0, l.stream, k);
        break;
      case OP_RESIDUAL:
        hipLaunchKernelGGL((k_residual_small<T, S, M>), dim3(l.grid), dim3(l.block), 0, l.stream, k,
                           static_cast<T*>(l.out0), l.hmax);
        break;
      case OP_ELEMENTS:
        hipLaunchKernelGGL((k_elements_small<T, S, M>), dim3(l.grid), dim3(l.block), 0, l.stream, k,
                           static_cast<T*>(l.out0), static_cast<T*>(l.out1));
        break;
      case OP_COOP_OCCUPANCY:
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                   l.occupancy, k_newton_small_coop<T, S, M, NT_COOP>, NT_COOP, 0) == hipSuccess
                   ? ST_OK : ST_DEVICE;
      case OP_COOP: {
        SmallKArgs kk = k;
        int G = l.G;
        char* cw = l.coop_ws;
        void* args[] = {&kk, &G, &cw};
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_newton_small_coop<T, S, M, NT_COOP>),
                                          dim3(l.grid), dim3(NT_COOP), args, 0, l.stream) == hipSuccess
                   ? ST_OK : ST_DEVICE;
      }
      default: return ST_INVALID;
    }
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

// Launchers of the implicit rules (implicit_small.hip).
int small_launch_implicit(int method, const SmallKArgs& k, const SmallLaunch& l);

}  // namespace pint
