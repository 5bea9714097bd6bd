// Windowed Newton (Sec. 3.2 with the windowed safeguard) for Lorenz-96 as a
// pipeline of updates.
//
// Update u searches its window start p_u = the first step whose residual of
// iterate u-1 violates tol (from p_{u-1} on), folds the recursion of eq.
// newton-step-recursion over [p_u, e_u], e_u = min(T, p_u + W - 1), and
// accepts the states below the first one that is non-finite or beyond the
// guard.  Update u needs iterate u-1 only step by step, in increasing order:
// residual n needs states n-1 and n, fold step n the element at n-1 and the
// state at n.  So update u can run while update u-1 is still folding, a few
// steps behind it.  The updates are the same as those of the one-at-a-time
// solver (same p_u, same window, same cut); only their overlap in time
// differs.
//
// G workgroups ("agents", one per compute unit, cooperative launch) take the
// updates round robin: agent g runs updates g+1, g+1+G, ...  Inside an agent
// (8 waves), for its update u:
//   wave 1 (loader)   streams the states of iterate u-1 from the trajectory
//                     into an LDS ring as they become final (as the agent of
//                     update u-1 publishes them), x_m for m = p_{u-1}-1, ...;
//   4 waves           build the element of each staged state: Phi(x_m) and
//                     the 13-diagonal band of dPhi/dx(x_m), into the ring;
//   wave 0 (fold)     evaluates the residuals from the ring to find p_u,
//                     then folds dx_n = J_{n-1} dx_{n-1} - h_n over the
//                     window, each updated state into an LDS output ring;
//   wave 2 (writer)   checks each updated state against the guard, writes
//                     it into the trajectory and publishes how far iterate
//                     u is final; the first state that fails is the cut.
// Only states cross between agents: written with device-scope atomic stores
// (the trajectory is updated in place), announced by a per-agent progress
// word stored after the writes complete.  A state of iterate u-1 is final
// when the agent of update u-1 has passed it, or lies beyond that update's
// window (then it is the initial iterate).  All cross-agent waits are
// bounded; the first agent that meets the end of the iteration (converged,
// non-finite, or the update limit) records it, agents of later updates
// stop, earlier ones finish.
#include "internal.h"
#include "systems_dense.h"

namespace pint {

// Per agent (64 bytes): progress and window start of its current update,
// each tagged with the update index in the upper 32 bits.
struct alignas(64) PipeRec {
  unsigned long long prog;   // (u << 32) | last step at which iterate u is final (T: all)
  unsigned long long start;  // (u << 32) | p_u
  unsigned long long pad[6];
};
// Per instance (64 bytes).
struct alignas(64) PipeCtl {
  unsigned long long done;   // 0 while running; else DONE_BIT | status << 40 | updates applied
  unsigned long long rmax;   // final residual (bits of a non-negative double)
  uint32_t err;              // a bounded wait gave up
  uint32_t bar_count, bar_gen, pad0;
  unsigned long long pad[4];
};
static_assert(sizeof(PipeRec) == 64 && sizeof(PipeCtl) == 64, "control block sizes");

constexpr unsigned long long DONE_BIT = 1ull << 63;
// 8 waves.  Waves are spread over the compute unit's four SIMDs in turn
// (wave w on SIMD w % 4), so wave 4 stays idle: the fold (wave 0) then has
// its SIMD to itself and is never held up behind the element waves'
// multiply-adds.  Wave 1 loads, wave 2 writes, waves 3, 5, 6 and 7 build
// elements (one of them alone on its SIMD, the others beside the light
// loader and writer).  Two waves per SIMD leave each up to 256 registers.
constexpr int PIPE_NT = 512;
constexpr int PIPE_NE = 5;
__device__ __forceinline__ int pipe_elem_index(int wv) {
  // waves 3..7 -> 0..4; -1 for the others
  return wv >= 3 ? wv - 3 : -1;
}
constexpr int PIPE_R = 24;      // ring slots (steps)

struct PipeKArgs {
  int64_t B, T;
  const void* x0;
  const void* params;
  int64_t pstride;
  void* traj;
  double dt, tol, guard;
  int64_t window, max_iter;
  int32_t guess;
  int64_t* iters;
  double* resid;
  int32_t* status;
  PipeCtl* ctl;    // [B]
  PipeRec* rec;    // [B][G]
  uint64_t wait_limit;
};

template <typename T, class S>
struct PipeSmem {
  static constexpr int D = S::D, BW = S::BW, R = PIPE_R;
  T sx[R][D];              // staged states x_m of iterate u-1
  T sphi[R][D];            // Phi(x_m)
  T sband[R][BW * D];      // band of dPhi/dx(x_m): entry (i, (i + k - BOFF) mod D) at [k * D + i]
  T xo[R][D];              // updated states x_n of iterate u (fold -> writer)
  typename S::Stage stage[PIPE_NE];
  T zx[2 * D];             // the fold's previous dx, zx[q] = dx[(q - BOFF) mod D]
  T P[S::NP], x0[D];
  double red[PIPE_NT / PINT_WAVE];
  int staged[R], ready[R];
  int f_pos;       // last step the fold (or its search) has completed; in the
                   // fold, also the last step whose updated state is in xo
  int written;     // last step the writer has taken from xo
  int pprev;       // p_{u-1}; 0 until known
  int p_u, e_u;    // this update's window; 0 until known
  int fold_end;    // -1 until the writer has published the update; then its last accepted step
  int abort_;      // this agent stops (the iteration ended, or a wait gave up)
};

__device__ __forceinline__ int lds_ld(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void wg_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup"); }
__device__ __forceinline__ void wg_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup"); }

template <typename T>
__device__ __forceinline__ void pst(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T pld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long gld(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gst(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int done_iters(unsigned long long d) { return (int)(d & 0xffffffffffull); }
__device__ __forceinline__ int done_status(unsigned long long d) { return (int)((d >> 40) & 0xff); }

// Record the end of the iteration (the first caller wins): `k` updates
// applied, status `st`.
__device__ __forceinline__ void pipe_finish(PipeCtl* c, int st, int64_t k) {
  const unsigned long long v = DONE_BIT | ((unsigned long long)st << 40) | (unsigned long long)k;
  atomicCAS(&c->done, 0ull, v);
}

// Whether this agent must stop before update u: the iteration ended with
// fewer than u updates, or a wait gave up.
__device__ __forceinline__ bool pipe_stop(PipeCtl* c, int64_t u) {
  const unsigned long long d = gld(&c->done);
  if (d != 0 && (int64_t)done_iters(d) < u) return true;
  return __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Barrier of the G agents of one instance (thread 0 of each), bounded.
__device__ __forceinline__ void pipe_barrier(PipeCtl* c, int G, uint32_t& gen, uint64_t limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t target = gen + 1;
    if (atomicAdd(&c->bar_count, 1u) == (uint32_t)(G - 1)) {
      __hip_atomic_store(&c->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      __hip_atomic_store(&c->bar_gen, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      for (uint64_t it = 0;
           __hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != target; it++) {
        if (it >= limit) {  // give up: the results are flagged unreliable
          atomicOr(&c->err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __threadfence();
    gen = target;
  }
  __syncthreads();
}

template <typename T, class S>
__global__ __launch_bounds__(PIPE_NT) void k_newton_pipe(PipeKArgs a, int G) {
  constexpr int D = S::D, BW = S::BW, BOFF = S::BOFF, R = PIPE_R;
  static_assert(D <= PINT_WAVE && S::R == 1, "one lane per component");
  static_assert(BW == 13, "the row sum is written for 13 diagonals");
  extern __shared__ __align__(16) unsigned char dyn[];
  PipeSmem<T, S>& sm = *reinterpret_cast<PipeSmem<T, S>*>(dyn);
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  const int64_t inst = blockIdx.x / G;
  const int g = blockIdx.x % G;
  const int64_t Tn = a.T, W = a.window;
  const T dt = (T)a.dt;
  PipeCtl* c = a.ctl + inst;
  PipeRec* rec = a.rec + inst * G;
  T* X = static_cast<T*>(a.traj) + inst * Tn * D;
  const uint64_t lim = a.wait_limit;
  uint32_t gen = 0;

  for (int i = tid; i < S::NP; i += PIPE_NT)
    sm.P[i] = static_cast<const T*>(a.params)[inst * a.pstride + i];
  for (int i = tid; i < D; i += PIPE_NT) sm.x0[i] = static_cast<const T*>(a.x0)[inst * D + i];
  __syncthreads();
  if (a.guess == 0)
    for (int64_t idx = (int64_t)g * PIPE_NT + tid; idx < Tn * D; idx += (int64_t)G * PIPE_NT)
      X[idx] = sm.x0[idx % D];
  if (g == 0 && tid == 0 && Tn == 0) pipe_finish(c, ST_OK, 0);
  pipe_barrier(c, G, gen, lim);  // the initial iterate is in memory

  // bounded spin: true when the wait gave up or the agent must stop
  auto spin = [&](uint64_t& it) -> bool {
    if (++it >= lim) {
      atomicOr(&c->err, 1u);
      lds_st(&sm.abort_, 1);
      return true;
    }
    __builtin_amdgcn_s_sleep(1);
    return lds_ld(&sm.abort_) != 0;
  };

  for (int64_t u = g + 1;; u += G) {
    if (tid == 0) {
      for (int r = 0; r < R; r++) {
        sm.staged[r] = -1;
        sm.ready[r] = -1;
      }
      sm.f_pos = -1;
      sm.written = -1;
      sm.pprev = 0;
      sm.p_u = 0;
      sm.e_u = 0;
      sm.fold_end = -1;
      sm.abort_ = pipe_stop(c, u) ? 1 : 0;
    }
    __syncthreads();
    if (sm.abort_) break;
    const int64_t aprev = (u - 2) % G;  // agent of update u-1 (u >= 2)

    if (wv == 1) {
      // ------------------------------------------------------- loader ---
      __builtin_amdgcn_s_setprio(2);
      uint64_t it = 0;
      int64_t pprev = 1, eprev = 0;  // update 0: none; iterate 0 is final everywhere
      if (u >= 2) {
        for (;;) {  // the previous update's window start
          const unsigned long long s = gld(&rec[aprev].start);
          if ((int64_t)(s >> 32) == u - 1) {
            pprev = (int64_t)(s & 0xffffffffull);
            break;
          }
          if (pipe_stop(c, u)) {
            lds_st(&sm.abort_, 1);
            break;
          }
          if (spin(it)) break;
        }
        eprev = (W >= Tn - pprev + 1) ? Tn : pprev + W - 1;
      }
      if (lane == 0) {
        // the search starts at p_{u-1}: the ring holds steps from p_{u-1} - 1
        lds_st(&sm.f_pos, (int)(pprev - 1));
        wg_release();
        lds_st(&sm.pprev, (int)pprev);
      }
      int64_t final_upto = u >= 2 ? pprev - 1 : Tn;
      int64_t m = pprev - 1;
      // how far iterate u-1 is final, from a progress word of update u-1
      auto take_prog = [&](unsigned long long pr) {
        const int64_t tag = (int64_t)(pr >> 32);
        if (tag > u - 1) final_upto = Tn;
        else if (tag == u - 1 && (int64_t)(pr & 0xffffffffull) > final_upto) final_upto = (int64_t)(pr & 0xffffffffull);
      };
      uint32_t polls = 0;
      while (!lds_ld(&sm.abort_) && lds_ld(&sm.fold_end) < 0 && m <= Tn) {
        const int e_u = lds_ld(&sm.e_u);
        int64_t lim_m = (int64_t)lds_ld(&sm.f_pos) + R - 1;  // ring space
        if (e_u > 0 && lim_m > e_u) lim_m = e_u;
        if (lim_m > Tn) lim_m = Tn;
        if (m > lim_m) {
          if (spin(it)) break;
          continue;
        }
        if (m > final_upto && m <= eprev) {
          take_prog(gld(&rec[aprev].prog));
          if (m > final_upto) {
            // whether the iteration ended before update u-1 (then no more
            // progress comes) is checked now and then, off the poll's path
            if ((++polls & 31) == 0 && pipe_stop(c, u)) {
              lds_st(&sm.abort_, 1);
              break;
            }
            if (spin(it)) break;
            continue;
          }
        }
        // a batch of consecutive final states (at or below final_upto, or
        // beyond the previous window), loads all in flight
        int64_t hi = lim_m;
        if (hi > m + 7) hi = m + 7;
        if (m <= eprev && final_upto < eprev && hi > final_upto) hi = final_upto;
        T v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const int64_t mm = m + j;
          v[j] = T(0);
          if (mm <= hi && lane < D) v[j] = mm == 0 ? sm.x0[lane] : pld(X + (mm - 1) * D + lane);
        }
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const int64_t mm = m + j;
          if (mm <= hi && lane < D) sm.sx[mm % R][lane] = v[j];
        }
        wg_release();
        if (lane == 0)
          for (int64_t mm = m; mm <= hi; mm++) lds_st(&sm.staged[mm % R], (int)mm);
        m = hi + 1;
        it = 0;
      }
      __builtin_amdgcn_s_setprio(0);
    } else if (wv == 2) {
      // ------------------------------------------------------- writer ---
      // Publishes the window start, then takes the updated states from xo
      // in order: each is checked against the guard (finite, within
      // `guard`) before it is stored, so the first state that fails is the
      // cut and nothing from it on is published.  The writer then records
      // the last accepted step (fold_end), which ends the update's roles.
      __builtin_amdgcn_s_setprio(2);
      uint64_t it = 0;
      int p = 0;
      while (!lds_ld(&sm.abort_) && (p = lds_ld(&sm.p_u)) == 0)
        if (spin(it)) break;
      if (p > 0 && !lds_ld(&sm.abort_)) {
        wg_acquire();
        const int e = lds_ld(&sm.e_u);
        const int i = lane < D ? lane : 0;
        if (lane == 0) {
          gst(&rec[g].start, ((unsigned long long)u << 32) | (unsigned)p);
          wait_stores();
          gst(&rec[g].prog, ((unsigned long long)u << 32) | (unsigned)(p - 1));
        }
        int w = p - 1, fe = -1;
        it = 0;
        for (;;) {
          const int avail = lds_ld(&sm.f_pos);  // steps up to avail are in xo
          if (avail > w) {
            wg_acquire();
            // up to 8 states at a time: all their LDS reads in flight, then
            // each checked and stored in order
            const int hi = avail - w > 8 ? w + 8 : avail;
            T v[8];
#pragma unroll
            for (int j = 0; j < 8; j++)
              if (w + 1 + j <= hi) v[j] = sm.xo[(w + 1 + j) % R][i];
            int n = w + 1;
#pragma unroll
            for (int j = 0; j < 8; j++) {
              if (n > hi) break;
              if (__ballot(lane < D && (!finite_(v[j]) || fabs((double)v[j]) > a.guard))) break;
              if (lane < D) pst(X + (int64_t)(n - 1) * D + lane, v[j]);
              n++;
            }
            const int last = n - 1;
            // the xo slots are read (the stores hold the values)
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            if (lane == 0) lds_st(&sm.written, last);
            wait_stores();
            if (lane == 0 && last > w) gst(&rec[g].prog, ((unsigned long long)u << 32) | (unsigned)last);
            w = last;
            it = 0;
            if (n <= hi) {  // state n fails the guard: the cut
              fe = n - 1;
              break;
            }
            if (w >= e) {
              fe = e;
              break;
            }
            continue;
          }
          if (lds_ld(&sm.abort_)) break;
          if (spin(it)) break;
        }
        if (fe >= 0 && !lds_ld(&sm.abort_)) {
          if (fe == p - 1) {  // the first updated state is unusable
            if (lane == 0) {
              pipe_finish(c, ST_NONFINITE, u - 1);
              lds_st(&sm.abort_, 1);
            }
          } else {
            if (lane == 0) {
              wg_release();
              lds_st(&sm.fold_end, fe);
            }
            if (fe < e && u >= 2) {
              // cut at fe + 1: iterate u equals iterate u-1 on (fe, e]; wait
              // until that is final before declaring iterate u final
              it = 0;
              for (;;) {
                const unsigned long long pr = gld(&rec[aprev].prog);
                const int64_t tag = (int64_t)(pr >> 32);
                if (tag > u - 1 || (tag == u - 1 && (int64_t)(pr & 0xffffffffull) >= e)) break;
                // beyond the previous window the states are the initial iterate
                const unsigned long long s0 = gld(&rec[aprev].start);
                const int64_t pp = (int64_t)(s0 & 0xffffffffull);
                if ((int64_t)(s0 >> 32) == u - 1 && ((W >= Tn - pp + 1) ? Tn : pp + W - 1) < fe + 1) break;
                if (pipe_stop(c, u)) {
                  lds_st(&sm.abort_, 1);
                  break;
                }
                if (spin(it)) break;
              }
            }
            if (lane == 0 && !lds_ld(&sm.abort_))
              gst(&rec[g].prog, ((unsigned long long)u << 32) | (unsigned long long)Tn);
          }
        }
      }
      __builtin_amdgcn_s_setprio(0);
    } else if (wv == 0) {
      // --------------------------------------------------------- fold ---
      __builtin_amdgcn_s_setprio(3);
      uint64_t it = 0;
      int pprev = 0;
      while ((pprev = lds_ld(&sm.pprev)) == 0)
        if (spin(it)) break;
      const int i = lane < D ? lane : 0;  // lanes past D repeat lane 0
      const int tn = (int)Tn;
      bool stop = lds_ld(&sm.abort_) != 0 || pprev == 0;
      // Ring slots of steps n-1 and n, advanced with n (no divisions).
      int n = pprev;
      int sp = (n - 1) % R, sc = n % R;
      auto advance = [&]() {
        n++;
        sp = sc;
        sc = sc + 1 == R ? 0 : sc + 1;
      };
      // Wait for element n-1 and state n (and, in the fold, for the writer
      // to have taken the output slot's previous occupant n - R when that
      // was a step of this update): the three flags are read together.  In
      // the fold the wait also ends when the writer has cut the update.
      auto await = [&](int xo_from) -> bool {
        uint64_t w = 0;
        for (;;) {
          const int fr = lds_ld(&sm.ready[sp]), fs = lds_ld(&sm.staged[sc]), fw = lds_ld(&sm.written);
          if ((fr == n - 1) & (fs == n) & (xo_from == 0 || n - R < xo_from || fw >= n - R)) break;
          if (xo_from != 0 && lds_ld(&sm.fold_end) >= 0) return false;
          if (spin(w)) return false;
        }
        wg_acquire();
        return true;
      };
      T h = T(0);
      bool violated = false, nonfinite = false;
      while (!stop) {  // the first violation of iterate u-1 at or after p_{u-1}
        if (n > tn) {
          if (lane == 0) pipe_finish(c, ST_OK, u - 1);
          stop = true;
          break;
        }
        if (!await(0)) {
          stop = true;
          break;
        }
        h = sm.sx[sc][i] - sm.sphi[sp][i];
        // ||h_n||_inf >= tol (or not finite) in any component
        const bool fin = finite_(h);
        violated = __ballot(lane < D && !(fabs((double)h) < a.tol)) != 0;
        nonfinite = __ballot(lane < D && !fin) != 0;
        if (violated) break;
        if (lane == 0) lds_st(&sm.f_pos, n);
        advance();
      }
      if (!stop) {
        if (nonfinite) {
          if (lane == 0) pipe_finish(c, ST_NONFINITE, u - 1);
          stop = true;
        } else if (u - 1 >= a.max_iter) {
          if (lane == 0) pipe_finish(c, ST_NOT_CONVERGED, u - 1);
          stop = true;
        }
      }
      if (stop) {
        if (lane == 0) lds_st(&sm.abort_, 1);
      } else {
        const int p = n;
        const int e = (W >= Tn - p + 1) ? tn : (int)(p + W - 1);
        if (lane == 0) {
          lds_st(&sm.e_u, e);
          wg_release();
          lds_st(&sm.p_u, p);
        }
        // dx_p = -h_p, then dx_n = J(x_{n-1}) dx_{n-1} - h_n.  Only
        // register dependences wait: one wave's LDS operations are
        // performed in issue order, so dx_n's neighbours are read right
        // after they are written, and a step's updated state and its f_pos
        // store need no fence between them (the writer reads f_pos, then
        // the slot).  A step issues the next step's operand loads (band row,
        // Phi(x_n), x_{n+1}, checked ready by flags read a step earlier)
        // before its own row sum, and the reads of dx_n's neighbours right
        // after the writes.  The guard is the writer's.
        auto cbar = [] { asm volatile("" ::: "memory"); };
        // every lane writes dx twice: at zx[i + BOFF], and at its wrap-around
        // copy (rows D-BOFF.. and 0..BW-BOFF-2) or else a spare slot
        const int zw2 = (i >= D - BOFF) ? i + BOFF - D : (i + BOFF + D < D + BW - 1 ? i + BOFF + D : 2 * D - 1);
        static_assert(D + BW - 1 < 2 * D - 1, "spare zx slot");
        auto put = [&](T dxn, T xn) {
          sm.zx[i + BOFF] = dxn;
          sm.zx[zw2] = dxn;
          sm.xo[sc][i] = xn;
        };
        T bvA[BW], bvB[BW], zv[BW], phA = T(0), phB = T(0), xA = sm.sx[sc][i], xB = T(0);
        int fr = 0, fs = 0, fw = 0;  // flags of the step after the current one
        put(-h, xA - h);
        cbar();
        lds_st(&sm.f_pos, n);
        if (n < e) {
          advance();
          if (!await(p)) {
            stop = true;
          } else {
            cbar();
#pragma unroll
            for (int k = 0; k < BW; k++) zv[k] = sm.zx[i + k];
            const T* band = sm.sband[sp];
#pragma unroll
            for (int k = 0; k < BW; k++) bvA[k] = band[k * D + i];
            phA = sm.sphi[sp][i];
            xA = sm.sx[sc][i];
            cbar();
            const int sn = sc + 1 == R ? 0 : sc + 1;
            fr = lds_ld(&sm.ready[sc]);
            fs = lds_ld(&sm.staged[sn]);
            fw = lds_ld(&sm.written);
          }
          // step n with operands (bA, pA, xA); step n+1's go to (bB, pB, xB)
          auto step = [&](T (&bA)[BW], T& pA, T& xA_, T (&bB)[BW], T& pB, T& xB_)
              __attribute__((always_inline)) -> int {
            const int sn = sc + 1 == R ? 0 : sc + 1;
            const bool more = n < e;
            if (more) {
              if (!((fr == n) & (fs == n + 1) & (n + 1 - R < p || fw >= n + 1 - R))) {
                // not ready when read: wait on fresh flags
                advance();
                const bool ok = await(p);
                n--;
                sc = sp;
                sp = sp == 0 ? R - 1 : sp - 1;
                if (!ok) return 2;
              }
              cbar();
              const T* band = sm.sband[sc];
#pragma unroll
              for (int k = 0; k < BW; k++) bB[k] = band[k * D + i];
              pB = sm.sphi[sc][i];
              xB_ = sm.sx[sn][i];
              cbar();
              const int sn2 = sn + 1 == R ? 0 : sn + 1;
              fr = lds_ld(&sm.ready[sn]);
              fs = lds_ld(&sm.staged[sn2]);
              fw = lds_ld(&sm.written);
            }
            const T dxn = band_row13<T>(pA - xA_, bA, zv);
            put(dxn, xA_ + dxn);
            if (more) {
#pragma unroll
              for (int k = 0; k < BW; k++) zv[k] = sm.zx[i + k];
            }
            cbar();
            lds_st(&sm.f_pos, n);
            if (!more) return 1;
            advance();
            return 0;
          };
          while (!stop) {
            int r = step(bvA, phA, xA, bvB, phB, xB);
            if (r) break;
            r = step(bvB, phB, xB, bvA, phA, xA);
            if (r) break;
          }
        }
      }
      __builtin_amdgcn_s_setprio(0);
    } else if (pipe_elem_index(wv) >= 0) {
      // ----------------------------------------------------- elements ---
      const int e = pipe_elem_index(wv);
      uint64_t it = 0;
      int pprev = 0;
      while ((pprev = lds_ld(&sm.pprev)) == 0)
        if (spin(it)) break;
      typename S::Stage* st = &sm.stage[e];
      for (int64_t m = pprev - 1 + e; pprev > 0 && m < Tn; m += PIPE_NE) {
        bool go = false;
        it = 0;
        for (;;) {
          if (lds_ld(&sm.abort_) || lds_ld(&sm.fold_end) >= 0) break;
          const int eu = lds_ld(&sm.e_u);
          if (eu > 0 && m > eu - 1) break;
          if (lds_ld(&sm.staged[m % R]) == (int)m) {
            go = true;
            break;
          }
          if (spin(it)) break;
        }
        if (!go) break;
        wg_acquire();
        // the lane index, opaque to the optimiser here: the per-lane
        // indices below are recomputed for each element instead of being
        // hoisted out of the update loop, where they would hold registers
        // through every role's code
        int ln = lane;
        asm volatile("" : "+v"(ln));
        T x[1], phi[1];
        x[0] = ln < D ? sm.sx[m % R][ln] : T(0);
        wave_rk4<T, S>(sm.P, dt, x, phi, st, ln);
        if (ln < D) {
          sm.sphi[m % R][ln] = phi[0];
          T col[BW];
          S::jac_band_column(st, ln, dt, col);
          T* band = sm.sband[m % R];
#pragma unroll
          for (int r = 0; r < BW; r++) {
            int row = ln - S::BOFFT + r;
            row = row < 0 ? row + D : (row >= D ? row - D : row);
            band[(BW - 1 - r) * D + row] = col[r];
          }
        }
        wg_release();
        if (lane == 0) lds_st(&sm.ready[m % R], (int)m);
      }
    }
    __syncthreads();  // every role of update u has finished
    if (sm.abort_) break;
  }

  // the iteration has ended: every agent stops; final residual over all steps
  pipe_barrier(c, G, gen, lim);
  double r = 0.0;
  for (int64_t nn = 1 + (int64_t)g * (PIPE_NT / PINT_WAVE) + wv; nn <= Tn; nn += (int64_t)G * (PIPE_NT / PINT_WAVE)) {
    T xp[1], xc[1], phi[1];
    xp[0] = lane < D ? (nn == 1 ? sm.x0[lane] : pld(X + (nn - 2) * D + lane)) : T(0);
    xc[0] = lane < D ? pld(X + (nn - 1) * D + lane) : T(0);
    wave_rk4<T, S>(sm.P, dt, xp, phi, nullptr, lane);
    r = fmax(r, lane < D ? acc_norm(0.0, xc[0] - phi[0]) : 0.0);
  }
  r = wave_max(r);
  if (lane == 0) atomic_max_nonneg(reinterpret_cast<double*>(&c->rmax), r);
  pipe_barrier(c, G, gen, lim);
  if (g == 0 && tid == 0) {
    const unsigned long long d = gld(&c->done);
    const bool err = __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    a.iters[inst] = d ? done_iters(d) : 0;
    a.resid[inst] = __longlong_as_double((long long)gld(&c->rmax));
    a.status[inst] = (err || d == 0) ? ST_DEVICE : done_status(d);
  }
}

// ---------------------------------------------------- matrix-free systems --
//
// The same pipeline for a system whose step Jacobian is applied through the
// RK4 tangent from the step's stage record instead of being stored (Kuramoto:
// J_f is a diagonal plus two rank-one terms).  The element of a staged state
// is Phi and the stage record (the cosines, sines and their sums at the four
// stage points); the fold applies J_{n-1} to dx_{n-1} through the four stages
// with the arithmetic of the one-at-a-time solver's fold, so the updates are
// the same bit for bit.  D = 64 RC components, RC per lane; the ring holds
// fewer steps than the banded one (a record is 8 D + 8 values).
constexpr int PIPE_MF_R = 10;  // ring slots (steps)
// 12 waves (768 threads): wave 0 folds, 1 loads, 2 writes, 3..11 build
// elements.  Building elements (four sincos per component and step) bounds
// the pipeline's throughput: 5 element waves (512 threads) measured 10.6 ms,
// 9 (768) 8.6 ms and 13 (1024) 9.2 ms for 8 x 4096 at W = 256 (before the
// sincos change); keeping the fold's SIMD free of element waves was slower.
constexpr int PIPE_MF_NT = 768;
constexpr int PIPE_MF_NW = PIPE_MF_NT / PINT_WAVE;
constexpr int PIPE_MF_NE = PIPE_MF_NW - 3;
__host__ __device__ constexpr int mf_elem_index(int wv) { return wv >= 3 ? wv - 3 : -1; }

template <typename T, class S>
struct PipeSmemMF {
  static constexpr int D = S::D, R = PIPE_MF_R;
  T sx[R][D];                       // staged states x_m of iterate u-1
  T sphi[R][D];                     // Phi(x_m)
  typename S::Stage srec[R];        // stage record of the step from x_m
  T xo[R][D];                       // updated states of iterate u (fold -> writer)
  T P[S::NP], x0[D];
  int staged[R], ready[R];
  int f_pos, written, pprev, p_u, e_u, fold_end, abort_;  // as in PipeSmem
};

template <typename T, class S>
__global__ __launch_bounds__(PIPE_MF_NT) void k_newton_pipe_mf(PipeKArgs a, int G) {
  constexpr int D = S::D, RC = S::R, R = PIPE_MF_R;
  static_assert(S::MATFREE && D == PINT_WAVE * RC, "whole lanes, RC components each");
  extern __shared__ __align__(16) unsigned char dyn[];
  PipeSmemMF<T, S>& sm = *reinterpret_cast<PipeSmemMF<T, S>*>(dyn);
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  const int64_t inst = blockIdx.x / G;
  const int g = blockIdx.x % G;
  const int64_t Tn = a.T, W = a.window;
  const T dt = (T)a.dt;
  PipeCtl* c = a.ctl + inst;
  PipeRec* rec = a.rec + inst * G;
  T* X = static_cast<T*>(a.traj) + inst * Tn * D;
  const uint64_t lim = a.wait_limit;
  uint32_t gen = 0;

  for (int i = tid; i < S::NP; i += PIPE_MF_NT)
    sm.P[i] = static_cast<const T*>(a.params)[inst * a.pstride + i];
  for (int i = tid; i < D; i += PIPE_MF_NT) sm.x0[i] = static_cast<const T*>(a.x0)[inst * D + i];
  __syncthreads();
  if (a.guess == 0)
    for (int64_t idx = (int64_t)g * PIPE_MF_NT + tid; idx < Tn * D; idx += (int64_t)G * PIPE_MF_NT)
      X[idx] = sm.x0[idx % D];
  if (g == 0 && tid == 0 && Tn == 0) pipe_finish(c, ST_OK, 0);
  pipe_barrier(c, G, gen, lim);  // the initial iterate is in memory

  auto spin = [&](uint64_t& it) -> bool {
    if (++it >= lim) {
      atomicOr(&c->err, 1u);
      lds_st(&sm.abort_, 1);
      return true;
    }
    __builtin_amdgcn_s_sleep(1);
    return lds_ld(&sm.abort_) != 0;
  };

  for (int64_t u = g + 1;; u += G) {
    if (tid == 0) {
      for (int r = 0; r < R; r++) {
        sm.staged[r] = -1;
        sm.ready[r] = -1;
      }
      sm.f_pos = -1;
      sm.written = -1;
      sm.pprev = 0;
      sm.p_u = 0;
      sm.e_u = 0;
      sm.fold_end = -1;
      sm.abort_ = pipe_stop(c, u) ? 1 : 0;
    }
    __syncthreads();
    if (sm.abort_) break;
    const int64_t aprev = (u - 2) % G;  // agent of update u-1 (u >= 2)

    if (wv == 1) {
      // ------------------------------------------------------- loader ---
      __builtin_amdgcn_s_setprio(2);
      uint64_t it = 0;
      int64_t pprev = 1, eprev = 0;  // update 0: none; iterate 0 is final everywhere
      if (u >= 2) {
        for (;;) {
          const unsigned long long s = gld(&rec[aprev].start);
          if ((int64_t)(s >> 32) == u - 1) {
            pprev = (int64_t)(s & 0xffffffffull);
            break;
          }
          if (pipe_stop(c, u)) {
            lds_st(&sm.abort_, 1);
            break;
          }
          if (spin(it)) break;
        }
        eprev = (W >= Tn - pprev + 1) ? Tn : pprev + W - 1;
      }
      if (lane == 0) {
        lds_st(&sm.f_pos, (int)(pprev - 1));
        wg_release();
        lds_st(&sm.pprev, (int)pprev);
      }
      int64_t final_upto = u >= 2 ? pprev - 1 : Tn;
      int64_t m = pprev - 1;
      auto take_prog = [&](unsigned long long pr) {
        const int64_t tag = (int64_t)(pr >> 32);
        if (tag > u - 1) final_upto = Tn;
        else if (tag == u - 1 && (int64_t)(pr & 0xffffffffull) > final_upto) final_upto = (int64_t)(pr & 0xffffffffull);
      };
      uint32_t polls = 0;
      while (!lds_ld(&sm.abort_) && lds_ld(&sm.fold_end) < 0 && m <= Tn) {
        const int e_u = lds_ld(&sm.e_u);
        int64_t lim_m = (int64_t)lds_ld(&sm.f_pos) + R - 1;  // ring space
        if (e_u > 0 && lim_m > e_u) lim_m = e_u;
        if (lim_m > Tn) lim_m = Tn;
        if (m > lim_m) {
          if (spin(it)) break;
          continue;
        }
        if (m > final_upto && m <= eprev) {
          take_prog(gld(&rec[aprev].prog));
          if (m > final_upto) {
            if ((++polls & 31) == 0 && pipe_stop(c, u)) {
              lds_st(&sm.abort_, 1);
              break;
            }
            if (spin(it)) break;
            continue;
          }
        }
        int64_t hi = lim_m;
        if (hi > m + 3) hi = m + 3;
        if (m <= eprev && final_upto < eprev && hi > final_upto) hi = final_upto;
        T v[4][RC];
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int64_t mm = m + j;
#pragma unroll
          for (int r = 0; r < RC; r++) {
            v[j][r] = T(0);
            if (mm <= hi) v[j][r] = mm == 0 ? sm.x0[lane + PINT_WAVE * r] : pld(X + (mm - 1) * D + lane + PINT_WAVE * r);
          }
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int64_t mm = m + j;
#pragma unroll
          for (int r = 0; r < RC; r++)
            if (mm <= hi) sm.sx[mm % R][lane + PINT_WAVE * r] = v[j][r];
        }
        wg_release();
        if (lane == 0)
          for (int64_t mm = m; mm <= hi; mm++) lds_st(&sm.staged[mm % R], (int)mm);
        m = hi + 1;
        it = 0;
      }
      __builtin_amdgcn_s_setprio(0);
    } else if (wv == 2) {
      // ------------------------------------------------------- writer ---
      // As in the banded pipeline: the window start, then the updated states
      // in order, each checked against the guard; the first that fails is
      // the cut.
      __builtin_amdgcn_s_setprio(2);
      uint64_t it = 0;
      int p = 0;
      while (!lds_ld(&sm.abort_) && (p = lds_ld(&sm.p_u)) == 0)
        if (spin(it)) break;
      if (p > 0 && !lds_ld(&sm.abort_)) {
        wg_acquire();
        const int e = lds_ld(&sm.e_u);
        if (lane == 0) {
          gst(&rec[g].start, ((unsigned long long)u << 32) | (unsigned)p);
          wait_stores();
          gst(&rec[g].prog, ((unsigned long long)u << 32) | (unsigned)(p - 1));
        }
        int w = p - 1, fe = -1;
        it = 0;
        for (;;) {
          const int avail = lds_ld(&sm.f_pos);
          if (avail > w) {
            wg_acquire();
            const int hi = avail - w > 4 ? w + 4 : avail;
            T v[4][RC];
#pragma unroll
            for (int j = 0; j < 4; j++)
#pragma unroll
              for (int r = 0; r < RC; r++)
                if (w + 1 + j <= hi) v[j][r] = sm.xo[(w + 1 + j) % R][lane + PINT_WAVE * r];
            int n = w + 1;
#pragma unroll
            for (int j = 0; j < 4; j++) {
              if (n > hi) break;
              bool badj = false;
#pragma unroll
              for (int r = 0; r < RC; r++) badj = badj || !finite_(v[j][r]) || fabs((double)v[j][r]) > a.guard;
              if (__ballot(badj)) break;
#pragma unroll
              for (int r = 0; r < RC; r++) pst(X + (int64_t)(n - 1) * D + lane + PINT_WAVE * r, v[j][r]);
              n++;
            }
            const int last = n - 1;
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            if (lane == 0) lds_st(&sm.written, last);
            wait_stores();
            if (lane == 0 && last > w) gst(&rec[g].prog, ((unsigned long long)u << 32) | (unsigned)last);
            w = last;
            it = 0;
            if (n <= hi) {
              fe = n - 1;
              break;
            }
            if (w >= e) {
              fe = e;
              break;
            }
            continue;
          }
          if (lds_ld(&sm.abort_)) break;
          if (spin(it)) break;
        }
        if (fe >= 0 && !lds_ld(&sm.abort_)) {
          if (fe == p - 1) {
            if (lane == 0) {
              pipe_finish(c, ST_NONFINITE, u - 1);
              lds_st(&sm.abort_, 1);
            }
          } else {
            if (lane == 0) {
              wg_release();
              lds_st(&sm.fold_end, fe);
            }
            if (fe < e && u >= 2) {
              it = 0;
              for (;;) {
                const unsigned long long pr = gld(&rec[aprev].prog);
                const int64_t tag = (int64_t)(pr >> 32);
                if (tag > u - 1 || (tag == u - 1 && (int64_t)(pr & 0xffffffffull) >= e)) break;
                const unsigned long long s0 = gld(&rec[aprev].start);
                const int64_t pp = (int64_t)(s0 & 0xffffffffull);
                if ((int64_t)(s0 >> 32) == u - 1 && ((W >= Tn - pp + 1) ? Tn : pp + W - 1) < fe + 1) break;
                if (pipe_stop(c, u)) {
                  lds_st(&sm.abort_, 1);
                  break;
                }
                if (spin(it)) break;
              }
            }
            if (lane == 0 && !lds_ld(&sm.abort_))
              gst(&rec[g].prog, ((unsigned long long)u << 32) | (unsigned long long)Tn);
          }
        }
      }
      __builtin_amdgcn_s_setprio(0);
    } else if (wv == 0) {
      // --------------------------------------------------------- fold ---
      __builtin_amdgcn_s_setprio(3);
      uint64_t it = 0;
      int pprev = 0;
      while ((pprev = lds_ld(&sm.pprev)) == 0)
        if (spin(it)) break;
      const int tn = (int)Tn;
      bool stop = lds_ld(&sm.abort_) != 0 || pprev == 0;
      int n = pprev;
      int sp = (n - 1) % R, sc = n % R;
      auto advance = [&]() {
        n++;
        sp = sc;
        sc = sc + 1 == R ? 0 : sc + 1;
      };
      // element n-1 and state n (and in the fold the output slot's previous
      // occupant taken by the writer), as in the banded pipeline
      auto await = [&](int xo_from) -> bool {
        uint64_t w = 0;
        for (;;) {
          const int fr = lds_ld(&sm.ready[sp]), fs = lds_ld(&sm.staged[sc]), fw = lds_ld(&sm.written);
          if ((fr == n - 1) & (fs == n) & (xo_from == 0 || n - R < xo_from || fw >= n - R)) break;
          if (xo_from != 0 && lds_ld(&sm.fold_end) >= 0) return false;
          if (spin(w)) return false;
        }
        wg_acquire();
        return true;
      };
      T h[RC];
      bool violated = false, nonfinite = false;
      while (!stop) {  // the first violation of iterate u-1 at or after p_{u-1}
        if (n > tn) {
          if (lane == 0) pipe_finish(c, ST_OK, u - 1);
          stop = true;
          break;
        }
        if (!await(0)) {
          stop = true;
          break;
        }
        bool viol = false, nf = false;
#pragma unroll
        for (int r = 0; r < RC; r++) {
          h[r] = sm.sx[sc][lane + PINT_WAVE * r] - sm.sphi[sp][lane + PINT_WAVE * r];
          viol = viol || !(fabs((double)h[r]) < a.tol);
          nf = nf || !finite_(h[r]);
        }
        violated = __ballot(viol) != 0;
        nonfinite = __ballot(nf) != 0;
        if (violated) break;
        if (lane == 0) lds_st(&sm.f_pos, n);
        advance();
      }
      if (!stop) {
        if (nonfinite) {
          if (lane == 0) pipe_finish(c, ST_NONFINITE, u - 1);
          stop = true;
        } else if (u - 1 >= a.max_iter) {
          if (lane == 0) pipe_finish(c, ST_NOT_CONVERGED, u - 1);
          stop = true;
        }
      }
      if (stop) {
        if (lane == 0) lds_st(&sm.abort_, 1);
      } else {
        const int p = n;
        const int e = (W >= Tn - p + 1) ? tn : (int)(p + W - 1);
        if (lane == 0) {
          lds_st(&sm.e_u, e);
          wg_release();
          lds_st(&sm.p_u, p);
        }
        const T h2 = T(0.5) * dt, c6 = dt / T(6), Kc = sm.P[0];
        T v[RC];  // dx_n, this lane's components
        // dx_p = -h_p
#pragma unroll
        for (int r = 0; r < RC; r++) {
          v[r] = -h[r];
          sm.xo[sc][lane + PINT_WAVE * r] = sm.sx[sc][lane + PINT_WAVE * r] + v[r];
        }
        asm volatile("" ::: "memory");
        lds_st(&sm.f_pos, n);
        while (n < e) {
          advance();
          {
            const int fr = lds_ld(&sm.ready[sp]), fs = lds_ld(&sm.staged[sc]), fw = lds_ld(&sm.written);
            if (!((fr == n - 1) & (fs == n) & (n - R < p || fw >= n - R))) {
              if (!await(p)) break;
            } else {
              wg_acquire();
            }
          }
          // dx_n = J(x_{n-1}) dx_{n-1} + (Phi(x_{n-1}) - x_n), J through the
          // RK4 tangent from step n-1's stage record
          const typename S::Stage* st = &sm.srec[sp];
          T z[RC], uu[RC], acc[RC];
#pragma unroll
          for (int r = 0; r < RC; r++) {
            z[r] = sm.sphi[sp][lane + PINT_WAVE * r] - sm.sx[sc][lane + PINT_WAVE * r];
            uu[r] = v[r];
          }
#pragma unroll
          for (int s = 0; s < 4; s++) {
            T cs[RC], sn[RC];
            T pa = T(0), pb = T(0);
#pragma unroll
            for (int r = 0; r < RC; r++) {
              cs[r] = st->c[s][lane + PINT_WAVE * r];
              sn[r] = st->s[s][lane + PINT_WAVE * r];
              pa += cs[r] * uu[r];
              pb += sn[r] * uu[r];
            }
            const T C = st->C[s], Sg = st->S[s];
            wave_sum2_dpp(pa, pb);
            const T w = (s == 0 || s == 3) ? T(1) : T(2);
            const T cc = (s == 2) ? dt : h2;
#pragma unroll
            for (int r = 0; r < RC; r++) {
              const T K = Kc * (cs[r] * pa + sn[r] * pb) - Kc * (cs[r] * C + sn[r] * Sg) * uu[r];
              acc[r] = (s == 0) ? K : acc[r] + w * K;
              uu[r] = v[r] + cc * K;
            }
          }
#pragma unroll
          for (int r = 0; r < RC; r++) {
            z[r] = (v[r] + c6 * acc[r]) + z[r];
            v[r] = z[r];
            sm.xo[sc][lane + PINT_WAVE * r] = sm.sx[sc][lane + PINT_WAVE * r] + z[r];
          }
          asm volatile("" ::: "memory");
          lds_st(&sm.f_pos, n);
        }
      }
      __builtin_amdgcn_s_setprio(0);
    } else if (mf_elem_index(wv) >= 0) {
      // ----------------------------------------------------- elements ---
      const int e = mf_elem_index(wv);
      uint64_t it = 0;
      int pprev = 0;
      while ((pprev = lds_ld(&sm.pprev)) == 0)
        if (spin(it)) break;
      for (int64_t m = pprev - 1 + e; pprev > 0 && m < Tn; m += PIPE_MF_NE) {
        bool go = false;
        it = 0;
        for (;;) {
          if (lds_ld(&sm.abort_) || lds_ld(&sm.fold_end) >= 0) break;
          const int eu = lds_ld(&sm.e_u);
          if (eu > 0 && m > eu - 1) break;
          if (lds_ld(&sm.staged[m % R]) == (int)m) {
            go = true;
            break;
          }
          if (spin(it)) break;
        }
        if (!go) break;
        wg_acquire();
        int ln = lane;
        asm volatile("" : "+v"(ln));
        T x[RC], phi[RC];
#pragma unroll
        for (int r = 0; r < RC; r++) x[r] = sm.sx[m % R][ln + PINT_WAVE * r];
        wave_rk4<T, S>(sm.P, dt, x, phi, &sm.srec[m % R], ln);
#pragma unroll
        for (int r = 0; r < RC; r++) sm.sphi[m % R][ln + PINT_WAVE * r] = phi[r];
        wg_release();
        if (lane == 0) lds_st(&sm.ready[m % R], (int)m);
      }
    }
    __syncthreads();  // every role of update u has finished
    if (sm.abort_) break;
  }

  // the iteration has ended: every agent stops; final residual over all steps
  pipe_barrier(c, G, gen, lim);
  double r = 0.0;
  for (int64_t nn = 1 + (int64_t)g * (PIPE_MF_NT / PINT_WAVE) + wv; nn <= Tn; nn += (int64_t)G * (PIPE_MF_NT / PINT_WAVE)) {
    T xp[RC], xc[RC], phi[RC];
#pragma unroll
    for (int q = 0; q < RC; q++) {
      const int i = lane + PINT_WAVE * q;
      xp[q] = nn == 1 ? sm.x0[i] : pld(X + (nn - 2) * D + i);
      xc[q] = pld(X + (nn - 1) * D + i);
    }
    wave_rk4<T, S>(sm.P, dt, xp, phi, nullptr, lane);
#pragma unroll
    for (int q = 0; q < RC; q++) r = acc_norm(r, xc[q] - phi[q]);
  }
  r = wave_max(r);
  if (lane == 0) atomic_max_nonneg(reinterpret_cast<double*>(&c->rmax), r);
  pipe_barrier(c, G, gen, lim);
  if (g == 0 && tid == 0) {
    const unsigned long long d = gld(&c->done);
    const bool err = __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    a.iters[inst] = d ? done_iters(d) : 0;
    a.resid[inst] = __longlong_as_double((long long)gld(&c->rmax));
    a.status[inst] = (err || d == 0) ? ST_DEVICE : done_status(d);
  }
}

// ------------------------------------------------------------ host side --

template <typename T, typename F>
static int dispatch_pipe_sys(int system, int d, F&& f) {
  if (system == 5 && d == 40) return f(DSysL96<T, 40>{});
  if (system == 6 && d == 128) return f(DSysKur<T, 128>{});
  if (system == 6 && d == 64) return f(DSysKur<T, 64>{});
  return ST_UNSUPPORTED;
}

static int pipe_cus() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus;
}

// Agents per instance: 16 (about twice the updates in flight at once for
// windows of 32-64 steps), fewer when the batch would not fit one agent per
// compute unit, down to one (then an instance's updates run one after the
// other on its agent, still with every element kept in the agent's LDS
// ring); 0 when the pipeline does not apply.
static int pipe_agents(const SolveArgs& a) {
  if (a.window <= 0 || a.B <= 0 || a.T_uniform <= 0 || a.T_off) return 0;
  if (a.T_uniform > 0x7fffffffLL) return 0;
  const int cus = pipe_cus();
  int64_t G = 16;
  while (G >= 2 && a.B * G > cus) G /= 2;
  return G >= 1 && a.B * G <= cus ? (int)G : 0;
}

template <typename T, class S>
static size_t pipe_lds() {
  if constexpr (S::MATFREE)
    return sizeof(PipeSmemMF<T, S>);
  else
    return sizeof(PipeSmem<T, S>);
}

// Threads per agent of a system's kernel.
template <class S>
static constexpr int pipe_nt() {
  if constexpr (S::MATFREE)
    return PIPE_MF_NT;
  else
    return PIPE_NT;
}

// The kernel of a system: banded (Lorenz-96) or matrix-free (Kuramoto).
template <typename T, class S>
static const void* pipe_kernel() {
  if constexpr (S::MATFREE)
    return reinterpret_cast<const void*>(&k_newton_pipe_mf<T, S>);
  else
    return reinterpret_cast<const void*>(&k_newton_pipe<T, S>);
}

size_t pipe_ws_bytes(const SolveArgs& a) {
  const int G = pipe_agents(a);
  if (G == 0) return 0;
  if (dispatch_pipe_sys<double>(a.system, a.d, [](auto) { return ST_OK; }) != ST_OK) return 0;
  return align_up((size_t)a.B * sizeof(PipeCtl)) + align_up((size_t)a.B * G * sizeof(PipeRec));
}

// Runs the pipelined solve when it applies (Lorenz-96 or Kuramoto, windowed,
// a batch small enough for one agent per compute unit); *used says whether
// it ran.
int pipe_solve(const SolveArgs& a, bool* used) {
  *used = false;
  const int G = pipe_agents(a);
  if (G == 0) return ST_OK;
  if (dispatch_pipe_sys<double>(a.system, a.d, [](auto) { return ST_OK; }) != ST_OK) return ST_OK;
  auto run = [&](auto t, auto s) -> int {
    using T = decltype(t);
    using S = decltype(s);
    const size_t need = pipe_ws_bytes(a);
    if (!a.ws || a.ws_bytes < need) return ST_WORKSPACE;
    const size_t lds = pipe_lds<T, S>();
    static bool attr_set = false;
    if (!attr_set) {
      if (hipFuncSetAttribute(pipe_kernel<T, S>(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
          hipSuccess)
        return ST_DEVICE;
      attr_set = true;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pipe_kernel<T, S>(), pipe_nt<S>(), lds) !=
            hipSuccess ||
        per_cu < 1)
      return ST_OK;  // not resident: the caller uses another solver
    char* w = static_cast<char*>(a.ws);
    if (int rc = fill_u32(reinterpret_cast<uint32_t*>(w), need / 4, 0u, a.stream)) return rc;
    PipeKArgs k{};
    k.B = a.B;
    k.T = a.T_uniform;
    k.x0 = a.x0;
    k.params = a.params;
    k.pstride = a.pstride;
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
    k.ctl = reinterpret_cast<PipeCtl*>(w);
    k.rec = reinterpret_cast<PipeRec*>(w + align_up((size_t)a.B * sizeof(PipeCtl)));
    k.wait_limit = wait_limit();
    int Gv = G;
    void* args[] = {&k, &Gv};
    const hipError_t e = hipLaunchCooperativeKernel(pipe_kernel<T, S>(),
                                                    dim3((unsigned)(a.B * G)), dim3(pipe_nt<S>()), args, lds,
                                                    a.stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return ST_OK;  // the caller falls back
    }
    *used = true;
    return ST_OK;
  };
  if (a.dtype == 0) return dispatch_pipe_sys<double>(a.system, a.d, [&](auto s) { return run((double)0, s); });
  if (a.dtype == 1) return dispatch_pipe_sys<float>(a.system, a.d, [&](auto s) { return run((float)0, s); });
  return ST_OK;
}

}  // namespace pint
