// Single-pass prefix scan of affine elements (eq. prefix-sum over the
// operator of eq. assoc-operator): z_{n+1} = A_n z_n + b_n for B independent
// sequences, with decoupled lookback across tiles.
//
// Every tile takes its id from an atomic counter at start (so a tile only
// ever waits on tiles that are already running), reduces its elements to an
// aggregate map, publishes it, then walks back over its predecessors'
// descriptors until it finds one whose inclusive prefix is known.  Because
// the prefix starts from a known z_0, an inclusive prefix is just the vector
// z at the tile's end, and stepping back over an aggregate-only predecessor
// costs a matrix-vector product, not a matrix product.
//
// Descriptor protocol.  The payload (aggregate map, inclusive vector) is
// written and read with device-scope atomic accesses, which are coherent
// across the chip's L2 slices on their own; the writer waits for its payload
// stores to complete (vmcnt) before it stores the flag, and a reader issues
// its payload loads only after it has seen the flag.  A generic device-scope
// fence would write back and invalidate the whole L2 of the writer's and the
// reader's die on every publish and every wait, which serialises the tiles.
// Waits are bounded so every wave exits even if a predecessor never
// publishes.
//
//   d <= 3: tiles staged through LDS, each thread folds a run of elements,
//     wave shuffles + LDS scan the thread aggregates;
//   d = 4..8: one wave per tile, each lane folds a run of 64 elements read
//     from global memory, scan and lookback through LDS;
//   dense d (16..128): each tile folds its elements with MFMA matrix
//     products (FP64 16x16x4 or FP32 16x16x4), the running product in LDS.
#include <mutex>
#include <type_traits>

#include "../../include/pint.h"
#include "internal.h"
#include "device_common.h"

namespace pint {

struct ScanArgs {
  int64_t B, N, tiles_per_seq;
  int32_t L;               // elements per tile
  const void* A;
  const void* b;
  const void* z0;
  void* z;
  uint32_t* counter;
  uint32_t* err;
  uint32_t* flags;         // [B * tiles_per_seq]
  void* agg;               // [B * tiles_per_seq][D*D + D]
  void* incl;              // [B * tiles_per_seq][D]
  uint32_t delay;          // test hook: sleeps before some publishes (0 = off)
};

constexpr uint32_t FLAG_AGG = 1, FLAG_INCL = 2;
constexpr uint64_t SPIN_LIMIT = 1ull << 24;

template <typename T>
__device__ __forceinline__ void st_payload(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T ld_payload(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by the thread that stored the payload (or after a workgroup barrier,
// which itself waits for every wave's stores): the payload stores complete
// before the flag store is issued.
// With the test hook `delay` set, tile ts sleeps `delay` times before it
// publishes its aggregate when ts % 3 == 1, and before it publishes its
// inclusive prefix when ts % 3 == 2: successors then find predecessors not
// yet published, or published as aggregate only, and must wait for them or
// look further back.
__device__ __forceinline__ void publish_flag(uint32_t* flags, int64_t ts, uint32_t v,
                                             uint32_t delay) {
  if (delay != 0 && ts % 3 == (int64_t)v)
    for (uint32_t i = 0; i < delay; i++) __builtin_amdgcn_s_sleep(16);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __hip_atomic_store(flags + ts, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-parallel lookback search (all 64 lanes of one wave call it): lanes
// read the flags of predecessors end, end-1, ..., end-63 at once.  Returns,
// in every lane, the number k of aggregate-only predecessors directly before
// the first inclusive one within the window (k = 64: none inclusive yet, all
// 64 aggregates), after waiting until no predecessor in front of the first
// inclusive one is still unpublished.  `f_out` receives this lane's flag.
// Payload reads after the return must use ld_payload.
__device__ __forceinline__ int lookback_window(const uint32_t* flags, int64_t end, uint32_t* err,
                                               uint32_t& f_out) {
  const int lane = threadIdx.x % PINT_WAVE;
  const int64_t idx = end - lane;
  for (uint64_t it = 0;; it++) {
    const uint32_t f = idx >= 0 ? __hip_atomic_load(flags + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                : FLAG_INCL;
    const uint64_t incl = __ballot(f == FLAG_INCL);
    const uint64_t zero = __ballot(f == 0);
    const int first = incl ? __ffsll((long long)incl) - 1 : PINT_WAVE;
    const uint64_t before = first >= PINT_WAVE ? ~0ull : ((1ull << first) - 1);
    if (!(zero & before)) {
      f_out = f;
      return first;
    }
    if (it > SPIN_LIMIT) {
      if (lane == 0) atomicOr(err, 1u);
      f_out = FLAG_INCL;
      return first;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// ----------------------------------------------------------- small d ------

// Widest load/store unit (in scalars, 16 or 8 bytes, else 1) that divides a
// per-thread run of `run` scalars.
template <typename T>
constexpr int vec_width(int run) {
  return (run * (int)sizeof(T)) % 16 == 0 ? 16 / (int)sizeof(T)
         : (run * (int)sizeof(T)) % 8 == 0 ? 8 / (int)sizeof(T) : 1;
}

// Tile shape of the small-d scan: NT threads, S consecutive elements per
// thread in each chunk, a chunk staged in LDS within a 48 KiB budget.  A
// tile is C chunks: each thread keeps its runs of the first K in registers
// from the first pass to the second (HC registers a chunk, K*HC within the
// HOLD budget) and the last stays in LDS, so every element is read from
// memory once.  PD chunk loads are in flight ahead of the chunk composed;
// WPE waves per SIMD (two or three workgroups per compute unit) bound the
// registers.  HOLD, PD and WPE per d and precision are the fastest measured
// on 2^24 orthogonal elements (FP64 d = 1/2/3: 0.118 / 0.304 / 0.766 ms,
// FP32: 0.074 / 0.172 / 0.428 ms, against 0.127 / 0.356 / 0.80 and
// 0.079 / 0.196 / 0.469 ms when every chunk but the last was read again in
// the second pass); two chunks in flight were no faster.  RA / RB: scalars of A / b per thread run.  FP32 runs are
// sized as FP64 ones for d = 1 and 3 and by their own size for d = 2.
template <int D, typename T>
struct SmallShape {
  static constexpr bool F64 = sizeof(T) == 8;
  static constexpr int NT = 256;
  static constexpr int E = D * D + D;
  static constexpr int SB = D == 2 ? (int)sizeof(T) : 8;  // bytes counted per scalar
  static constexpr int S0 = 49152 / (E * SB * NT);
  static constexpr int S = S0 < 1 ? 1 : (S0 > 16 ? 16 : S0);
  static constexpr int CH = NT * S;   // elements per chunk (one LDS staging)
  static constexpr int HC = S * E * (int)sizeof(T) / 4;  // registers per kept chunk
  static constexpr int HOLD = F64 ? (D == 1 ? 144 : 48) : (D == 1 ? 48 : D == 2 ? 144 : 72);
  static constexpr int PD0 = 1;
  static constexpr int WPE = F64 ? (D == 2 ? 3 : 2) : (D == 2 ? 2 : 3);
  static constexpr int K0 = HOLD / HC;
  static constexpr int K = K0 < 1 ? 1 : (K0 > 11 ? 11 : K0);  // chunks kept in registers
  static constexpr int C = K + 1;     // chunks per tile (one lookback per tile)
  static constexpr int PD = PD0 < C ? PD0 : C;
  // each thread's prefix within a kept chunk is kept from pass 1 too, so
  // pass 2 does not refold it (FP64 d = 2: 0.322 -> 0.304 ms); not for FP32
  // d = 3, whose three kept chunks leave no registers for it
  static constexpr bool KA = D <= 2 || F64;
  static constexpr int TILE = CH * C;
  static constexpr int RA = S * D * D, RB = S * D;
  static constexpr int VA = vec_width<T>(RA), VB = vec_width<T>(RB);
};

// f(integral_constant<int, i>) for i = I .. N-1 in turn: a loop whose index
// is a compile-time constant, so it can select a register array.
template <int I, int N, typename F>
__device__ __forceinline__ void unroll_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    unroll_for<I + 1, N>(f);
  }
}

// Global -> LDS copy of n <= NT*RUN scalars into the blocked layout in which
// thread t's run of RUN scalars starts at t*(RUN+1) (one pad scalar per run,
// so the runs read back at an odd stride hit distinct LDS banks).  Global
// reads are striped over the block, so each wave instruction reads one
// contiguous span, and all are issued before the first LDS write; vectors of
// V scalars when the tile is full and g is aligned.
template <typename T, int RUN, int V, int NT>
__device__ __forceinline__ void stage_in(const T* __restrict__ g, T* lds, int n, int tid) {
  if constexpr (V > 1) {
    if (n == NT * RUN && (reinterpret_cast<uintptr_t>(g) % (V * sizeof(T))) == 0) {
      typedef T vec_t __attribute__((ext_vector_type(V)));
      constexpr int NV = RUN / V;
      vec_t r[NV];
#pragma unroll
      for (int j = 0; j < NV; j++) r[j] = reinterpret_cast<const vec_t*>(g)[j * NT + tid];
#pragma unroll
      for (int j = 0; j < NV; j++) {
        const int q = (j * NT + tid) * V;
        const int p = q + q / RUN;
#pragma unroll
        for (int c = 0; c < V; c++) lds[p + c] = r[j][c];
      }
      return;
    }
  }
  T r[RUN];
#pragma unroll
  for (int j = 0; j < RUN; j++) {
    const int q = j * NT + tid;
    r[j] = q < n ? g[q] : T(0);
  }
#pragma unroll
  for (int j = 0; j < RUN; j++) {
    const int q = j * NT + tid;
    if (q < n) lds[q + q / RUN] = r[j];
  }
}

// LDS (blocked, padded as in stage_in) -> global, striped over the block.
template <typename T, int RUN, int V, int NT>
__device__ __forceinline__ void stage_out(T* __restrict__ g, const T* lds, int n, int tid) {
  if constexpr (V > 1) {
    if (n == NT * RUN && (reinterpret_cast<uintptr_t>(g) % (V * sizeof(T))) == 0) {
      typedef T vec_t __attribute__((ext_vector_type(V)));
      constexpr int NV = RUN / V;
#pragma unroll
      for (int j = 0; j < NV; j++) {
        const int q = (j * NT + tid) * V;
        const int p = q + q / RUN;
        vec_t v;
#pragma unroll
        for (int c = 0; c < V; c++) v[c] = lds[p + c];
        reinterpret_cast<vec_t*>(g)[j * NT + tid] = v;
      }
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < RUN; j++) {
    const int q = j * NT + tid;
    if (q < n) g[q] = lds[q + q / RUN];
  }
}

// A run of RUN scalars per thread in registers, in the striped order of
// stage_in (vector j of thread t covers scalars (j*NT + t)*V ..): fetched
// from global memory ahead of its use, then stashed into the padded LDS
// layout, so a chunk's loads fly while the previous chunk is composed.
template <typename T, int RUN, int V>
struct RunRegs {
  typedef T vec_t __attribute__((ext_vector_type(V)));
  vec_t r[RUN / V];
};

template <typename T, int RUN, int V, int NT>
__device__ __forceinline__ void fetch_run(const T* __restrict__ g, int n, int tid, RunRegs<T, RUN, V>& R) {
  using vec_t = typename RunRegs<T, RUN, V>::vec_t;
  constexpr int NV = RUN / V;
  if (n == NT * RUN && (reinterpret_cast<uintptr_t>(g) % (V * sizeof(T))) == 0) {
#pragma unroll
    for (int j = 0; j < NV; j++) R.r[j] = reinterpret_cast<const vec_t*>(g)[j * NT + tid];
  } else {
#pragma unroll
    for (int j = 0; j < NV; j++)
#pragma unroll
      for (int c = 0; c < V; c++) {
        const int q = (j * NT + tid) * V + c;
        R.r[j][c] = q < n ? g[q] : T(0);
      }
  }
}

template <typename T, int RUN, int V, int NT>
__device__ __forceinline__ void stash_run(T* lds, int n, int tid, const RunRegs<T, RUN, V>& R) {
  constexpr int NV = RUN / V;
#pragma unroll
  for (int j = 0; j < NV; j++)
#pragma unroll
    for (int c = 0; c < V; c++) {
      const int q = (j * NT + tid) * V + c;
      if (q < n) lds[q + q / RUN] = R.r[j][c];
    }
}

// A tile is C chunks of NT*S elements, each staged once through LDS.  Pass 1
// folds the chunks in turn into the tile's aggregate, keeping each chunk's
// aggregate and, in registers, each thread's runs of the first K chunks (the
// last chunk stays in LDS).  One lookback per tile gives the z at the tile
// start, hence at every chunk start; pass 2 walks the chunks backwards (the
// last one first, while LDS still holds it), takes each thread's prefix
// within the chunk (kept from pass 1, or for FP32 d = 3 refolded from the
// run in registers) and writes the outputs.  A chunk's loads go to
// registers PD chunks ahead, and the barriers between order LDS only, so
// the loads stay in flight while the previous chunk is composed.
template <typename T, int D>
__global__ __launch_bounds__((SmallShape<D, T>::NT)) __attribute__((amdgpu_waves_per_eu(SmallShape<D, T>::WPE)))
void k_scan_small(ScanArgs a) {
  using SH = SmallShape<D, T>;
  constexpr int NT = SH::NT, S = SH::S, CH = SH::CH, TILE = SH::TILE, NW = NT / PINT_WAVE, E = SH::E;
  constexpr int C = SH::C, K = SH::K;
  constexpr int RA = SH::RA, RB = SH::RB, PA = RA + 1, PB = RB + 1;
  __shared__ T sA[NT * PA];
  __shared__ T sb[NT * PB];
  __shared__ Aff<T, D> s_aff[NW];
  __shared__ Aff<T, D> s_tagg;
  __shared__ Aff<T, D> s_cagg[C];  // each chunk's aggregate (pass 1)
  __shared__ T s_zc[C][D];         // z at each chunk start (after the lookback)
  __shared__ T s_wz[NW][D];
  __shared__ uint32_t s_tile;
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  if (tid == 0) {
    s_tile = atomicAdd(a.counter, 1u);
    aff_identity(s_tagg);
  }
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t seq = tile / a.tiles_per_seq, ts = tile % a.tiles_per_seq;
  const int64_t e0 = ts * TILE;
  const int n_el = (int)((a.N - e0) < TILE ? (a.N - e0) : TILE);
  const int nch = (n_el + CH - 1) / CH;
  const T* Ag = static_cast<const T*>(a.A) + (seq * a.N + e0) * D * D;
  const T* bg = static_cast<const T*>(a.b) + (seq * a.N + e0) * D;
  const T* myA = sA + tid * PA;
  const T* myb = sb + tid * PB;

  constexpr int PD = SH::PD;  // chunks in flight ahead of the one composed
  RunRegs<T, RA, SH::VA> rA[PD];
  RunRegs<T, RB, SH::VB> rB[PD];
  T hA[K][RA], hb[K][RB];  // this thread's runs of chunks 0..K-1
  Aff<T, D> hagg[SH::KA ? K : 1];  // and (KA) its prefix within each of them
  auto chunk_len = [&](int c) { return (n_el - c * CH) < CH ? (n_el - c * CH) : CH; };
  auto fetch = [&](int c, auto& ra, auto& rb) __attribute__((always_inline)) {
    const int c0 = c * CH, n = chunk_len(c);
    fetch_run<T, RA, SH::VA, NT>(Ag + (int64_t)c0 * D * D, n * D * D, tid, ra);
    fetch_run<T, RB, SH::VB, NT>(bg + (int64_t)c0 * D, n * D, tid, rb);
  };
  // this thread's run (registers or LDS) folded, then the block scan: agg =
  // composition of the runs of threads 0..tid of the chunk
  auto run_scan = [&](const T* ra, const T* rb, int cn, Aff<T, D>& agg) __attribute__((always_inline)) {
    aff_identity(agg);
#pragma unroll
    for (int s = 0; s < S; s++) {
      if (tid * S + s < cn) {
        Aff<T, D> e;
#pragma unroll
        for (int i = 0; i < D * D; i++) e.A[i] = ra[s * D * D + i];
#pragma unroll
        for (int i = 0; i < D; i++) e.b[i] = rb[s * D + i];
        aff_after(e, agg);
        agg = e;
      }
    }
    block_scan_aff<T, D, NT, true>(agg, s_aff);
  };

  // pass 1: the tile's aggregate
  Aff<T, D> agg;
  int cn = 0;
  unroll_for<0, PD>([&](auto ci) __attribute__((always_inline)) {
    constexpr int c = decltype(ci)::value;
    if (c < nch) fetch(c, rA[c], rB[c]);
  });
  unroll_for<0, C>([&](auto ci) __attribute__((always_inline)) {
    constexpr int c = decltype(ci)::value;
    if (c < nch) {
      cn = chunk_len(c);
      stash_run<T, RA, SH::VA, NT>(sA, cn * D * D, tid, rA[c % PD]);
      stash_run<T, RB, SH::VB, NT>(sb, cn * D, tid, rB[c % PD]);
      lds_barrier();
      if (c + PD < nch) fetch(c + PD, rA[c % PD], rB[c % PD]);
      if constexpr (c < K) {
#pragma unroll
        for (int i = 0; i < RA; i++) hA[c][i] = myA[i];
#pragma unroll
        for (int i = 0; i < RB; i++) hb[c][i] = myb[i];
        run_scan(hA[c], hb[c], cn, agg);
        if constexpr (SH::KA) hagg[c] = agg;
      } else {
        run_scan(myA, myb, cn, agg);
      }
      if (tid == NT - 1) {
        s_cagg[c] = agg;
        Aff<T, D> t = agg;
        aff_after(t, s_tagg);  // this chunk after the earlier ones
        s_tagg = t;
      }
      if (c + 1 < nch) lds_barrier();  // the chunk's LDS may be rewritten
    }
  });
  lds_barrier();  // s_tagg, s_cagg written
  // lookback by wave 0: z at the start of this tile
  if (wv == 0) {
    const int64_t base = seq * a.tiles_per_seq;
    uint32_t* flags = a.flags + base;
    T* aggp = static_cast<T*>(a.agg) + base * E;
    T* inclp = static_cast<T*>(a.incl) + base * D;
    T z[D];
    if (ts == 0) {
#pragma unroll
      for (int i = 0; i < D; i++) z[i] = a.z0 ? static_cast<const T*>(a.z0)[seq * D + i] : T(0);
    } else {
      if (lane == 0) {
#pragma unroll
        for (int i = 0; i < D * D; i++) st_payload(aggp + ts * E + i, s_tagg.A[i]);
#pragma unroll
        for (int i = 0; i < D; i++) st_payload(aggp + ts * E + D * D + i, s_tagg.b[i]);
        publish_flag(flags, ts, FLAG_AGG, a.delay);
      }
      // acc = composition of the aggregates passed so far (newest applied last)
      Aff<T, D> acc;
      aff_identity(acc);
      int64_t end = ts - 1;
      for (;;) {
        uint32_t f;
        const int k = lookback_window(flags, end, a.err, f);
        // this lane's aggregate if it lies before the first inclusive lane
        Aff<T, D> v;
        const int64_t idx = end - lane;
        if (lane < k) {
#pragma unroll
          for (int i = 0; i < D * D; i++) v.A[i] = ld_payload(aggp + idx * E + i);
#pragma unroll
          for (int i = 0; i < D; i++) v.b[i] = ld_payload(aggp + idx * E + D * D + i);
        } else {
          aff_identity(v);
        }
        // ordered reduction: lane 0 (newest) o lane 1 o ... o lane 63 (oldest)
#pragma unroll
        for (int off = 1; off < PINT_WAVE; off <<= 1) {
          Aff<T, D> o;
#pragma unroll
          for (int i = 0; i < D * D; i++) o.A[i] = __shfl_down(v.A[i], off, PINT_WAVE);
#pragma unroll
          for (int i = 0; i < D; i++) o.b[i] = __shfl_down(v.b[i], off, PINT_WAVE);
          if ((lane & (2 * off - 1)) == 0) aff_after(v, o);
        }
#pragma unroll
        for (int i = 0; i < D * D; i++) v.A[i] = __shfl(v.A[i], 0, PINT_WAVE);
#pragma unroll
        for (int i = 0; i < D; i++) v.b[i] = __shfl(v.b[i], 0, PINT_WAVE);
        aff_after(acc, v);
        if (k < PINT_WAVE) {
          const int64_t j = end - k;  // the inclusive predecessor
          T zi[D];
#pragma unroll
          for (int i = 0; i < D; i++) zi[i] = j >= 0 ? ld_payload(inclp + j * D + i) : T(0);
#pragma unroll
          for (int i = 0; i < D; i++) {
            T t = acc.b[i];
#pragma unroll
            for (int q = 0; q < D; q++) t += acc.A[i * D + q] * zi[q];
            z[i] = t;
          }
          break;
        }
        end -= PINT_WAVE;
      }
    }
    if (lane == 0) {
      // z at each chunk start
#pragma unroll
      for (int i = 0; i < D; i++) s_zc[0][i] = z[i];
      T zc[D];
#pragma unroll
      for (int i = 0; i < D; i++) zc[i] = z[i];
      for (int c = 1; c < nch; c++) {
        T t[D];
#pragma unroll
        for (int i = 0; i < D; i++) {
          T acc = s_cagg[c - 1].b[i];
#pragma unroll
          for (int q = 0; q < D; q++) acc += s_cagg[c - 1].A[i * D + q] * zc[q];
          t[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < D; i++) {
          zc[i] = t[i];
          s_zc[c][i] = t[i];
        }
      }
      // this tile's inclusive prefix: its aggregate applied to z_in
#pragma unroll
      for (int i = 0; i < D; i++) {
        T t = s_tagg.b[i];
#pragma unroll
        for (int q = 0; q < D; q++) t += s_tagg.A[i * D + q] * z[q];
        st_payload(inclp + ts * D + i, t);
      }
      publish_flag(flags, ts, FLAG_INCL, a.delay);
    }
  }
  lds_barrier();  // s_zc written

  // pass 2: outputs chunk by chunk, last chunk first (agg and cn are still
  // pass 1's for it); the chunks before it are refolded from registers
  T* zg = static_cast<T*>(a.z) + (seq * a.N + e0) * D;
  unroll_for<0, C>([&](auto ci) __attribute__((always_inline)) {
    constexpr int c = C - 1 - decltype(ci)::value;
    if (c < nch) {
      if constexpr (c < K) {
        if (c < nch - 1) {
          cn = chunk_len(c);
          if constexpr (SH::KA)
            agg = hagg[c];
          else
            run_scan(hA[c], hb[c], cn, agg);
        }
      }
      // z at the end of each thread's run, then at its start (previous thread)
      T zin[D], zend[D], z[D];
#pragma unroll
      for (int i = 0; i < D; i++) zin[i] = s_zc[c][i];
#pragma unroll
      for (int i = 0; i < D; i++) {
        T acc = agg.b[i];
#pragma unroll
        for (int k = 0; k < D; k++) acc += agg.A[i * D + k] * zin[k];
        zend[i] = acc;
      }
      if (lane == PINT_WAVE - 1)
#pragma unroll
        for (int i = 0; i < D; i++) s_wz[wv][i] = zend[i];
      lds_barrier();
#pragma unroll
      for (int i = 0; i < D; i++) {
        const T up = __shfl_up(zend[i], 1, PINT_WAVE);
        z[i] = lane > 0 ? up : (wv > 0 ? s_wz[wv - 1][i] : zin[i]);
      }
      T out[S][D];
      auto outputs = [&](const T* ra, const T* rb) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < S; s++) {
          if (tid * S + s < cn) {
            T t[D];
#pragma unroll
            for (int i = 0; i < D; i++) {
              T acc = rb[s * D + i];
#pragma unroll
              for (int k = 0; k < D; k++) acc += ra[s * D * D + i * D + k] * z[k];
              t[i] = acc;
            }
#pragma unroll
            for (int i = 0; i < D; i++) {
              z[i] = t[i];
              out[s][i] = t[i];
            }
          }
        }
      };
      if constexpr (c < K)
        outputs(hA[c], hb[c]);
      else
        outputs(myA, myb);
      lds_barrier();  // every thread has read s_wz and its b run
#pragma unroll
      for (int s = 0; s < S; s++) {
        if (tid * S + s < cn)
#pragma unroll
          for (int i = 0; i < D; i++) sb[tid * PB + s * D + i] = out[s][i];
      }
      lds_barrier();
      stage_out<T, RB, SH::VB, NT>(zg + (int64_t)c * CH * D, sb, cn * D, tid);
      lds_barrier();  // the staging area is reloaded by the next chunk
    }
  });
}

// ------------------------------------------------------- d = 4 .. 8 ------

// One wave per workgroup, a run of S consecutive elements per lane.  An 8x8 affine map and a
// composition partner do not both fit a lane's registers alongside a
// shuffled copy, so the in-wave scan and the lookback reduction pass maps
// through LDS and stream the partner's rows while composing.  Every hand-off
// through LDS between lanes is separated by a workgroup barrier: within one
// thread the reads of a partner's map and the writes of its own never alias,
// so nothing else would keep the compiler from reordering them.
// Elements are read straight from global memory and read again for the
// outputs; LDS holds only the scan and a 16-map lookback buffer.  Each lane
// takes its elements UF (fold) or UO (outputs) at a time, all loads of a
// group issued before its first use, so a lane waits for memory once per
// group rather than once per element.  The group sizes follow the registers
// an element takes; in FP64 the fold keeps UF = 1, since the registers of a
// second staged element cost more occupancy than the overlap gains (measured
// at d = 4: 1.57 ms with UF = 1, 2.10 ms with UF = 2, for 2^24 elements).
template <int D, typename T>
struct WideShape {
  static constexpr int NT = 64, E = D * D + D, EP = E + 1, LW = 16;  // LW: lookback maps per pass
  static constexpr int S = 64, TILE = NT * S;  // S consecutive elements per lane
  static constexpr int EB = E * (int)sizeof(T);
  static constexpr int UF = sizeof(T) == 8 ? 1 : (EB <= 96 ? 4 : (EB <= 192 ? 2 : 1));
  static constexpr int UO = EB <= 80 ? 8 : (EB <= 160 ? 4 : (EB <= 352 ? 2 : 1));
  static constexpr size_t OFF_Y = (size_t)NT * EP;
  static constexpr size_t OFF_ACC = OFF_Y + (size_t)LW * EP;
  static constexpr size_t OFF_T = OFF_ACC + EP;
  static constexpr size_t OFF_Z = OFF_T + EP;
  static constexpr size_t LDS = (OFF_Z + 2 * D) * sizeof(T);
};

// l <- l o P (P applied first); P in LDS as A row-major then b.
template <typename T, int D>
__device__ __forceinline__ void aff_after_lds(Aff<T, D>& l, const T* P) {
  Aff<T, D> r;
#pragma unroll
  for (int i = 0; i < D; i++) {
#pragma unroll
    for (int j = 0; j < D; j++) r.A[i * D + j] = T(0);
    r.b[i] = l.b[i];
  }
#pragma unroll
  for (int k = 0; k < D; k++) {
    T prow[D + 1];
#pragma unroll
    for (int j = 0; j < D; j++) prow[j] = P[k * D + j];
    prow[D] = P[D * D + k];
#pragma unroll
    for (int i = 0; i < D; i++) {
      const T lik = l.A[i * D + k];
#pragma unroll
      for (int j = 0; j < D; j++) r.A[i * D + j] += lik * prow[j];
      r.b[i] += lik * prow[D];
    }
  }
  l = r;
}

// l <- E o l (E applied last), E read row by row from global memory.
template <typename T, int D>
__device__ __forceinline__ void aff_before_g(Aff<T, D>& l, const T* EA, const T* Eb) {
  Aff<T, D> r;
#pragma unroll
  for (int i = 0; i < D; i++) {
    T er[D];
#pragma unroll
    for (int k = 0; k < D; k++) er[k] = EA[i * D + k];
    T bi = Eb[i];
#pragma unroll
    for (int j = 0; j < D; j++) {
      T t = T(0);
#pragma unroll
      for (int k = 0; k < D; k++) t += er[k] * l.A[k * D + j];
      r.A[i * D + j] = t;
    }
#pragma unroll
    for (int k = 0; k < D; k++) bi += er[k] * l.b[k];
    r.b[i] = bi;
  }
  l = r;
}

// One element (A row-major, b) from global memory into registers.
template <typename T, int D>
__device__ __forceinline__ void wide_load_el(T* ea, T* eb, const T* EA, const T* Eb) {
#pragma unroll
  for (int i = 0; i < D * D; i++) ea[i] = EA[i];
#pragma unroll
  for (int i = 0; i < D; i++) eb[i] = Eb[i];
}

// z <- A z + b for one element, the new z also stored to out.
template <typename T, int D>
__device__ __forceinline__ void wide_apply(T* z, const T* EA, const T* Eb, T* out) {
  T t[D];
#pragma unroll
  for (int i = 0; i < D; i++) {
    T acc = Eb[i];
#pragma unroll
    for (int q = 0; q < D; q++) acc += EA[i * D + q] * z[q];
    t[i] = acc;
  }
#pragma unroll
  for (int i = 0; i < D; i++) {
    z[i] = t[i];
    out[i] = t[i];
  }
}

template <typename T, int D>
__device__ __forceinline__ void aff_store_lds(T* p, const Aff<T, D>& e) {
#pragma unroll
  for (int i = 0; i < D * D; i++) p[i] = e.A[i];
#pragma unroll
  for (int i = 0; i < D; i++) p[D * D + i] = e.b[i];
}

template <typename T, int D>
__device__ __forceinline__ void aff_load_lds(Aff<T, D>& e, const T* p) {
#pragma unroll
  for (int i = 0; i < D * D; i++) e.A[i] = p[i];
#pragma unroll
  for (int i = 0; i < D; i++) e.b[i] = p[D * D + i];
}

template <typename T, int D>
__device__ __forceinline__ void aff_identity_lds(T* p) {
#pragma unroll
  for (int i = 0; i < D * D; i++) p[i] = (i / D == i % D) ? T(1) : T(0);
#pragma unroll
  for (int i = 0; i < D; i++) p[D * D + i] = T(0);
}

template <typename T, int D>
__global__ __launch_bounds__(64) void k_scan_wide(ScanArgs a) {
  using SH = WideShape<D, T>;
  constexpr int NT = SH::NT, S = SH::S, TILE = SH::TILE, E = SH::E, EP = SH::EP, LW = SH::LW;
  extern __shared__ __align__(16) unsigned char wide_lds[];
  T* L = reinterpret_cast<T*>(wide_lds);
  T* sX = L;                // [NT][EP]: inclusive prefixes of the tile
  T* sY = L + SH::OFF_Y;    // [LW][EP]: lookback maps
  T* sAcc = L + SH::OFF_ACC;
  T* sT = L + SH::OFF_T;    // the tile's aggregate
  T* sZ = L + SH::OFF_Z;    // z_in (D), then the inclusive vector found (D)
  __shared__ uint32_t s_tile;
  const int lane = threadIdx.x;
  if (lane == 0) s_tile = atomicAdd(a.counter, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t seq = tile / a.tiles_per_seq, ts = tile % a.tiles_per_seq;
  const int64_t e0 = ts * TILE;
  const int n_el = (int)((a.N - e0) < TILE ? (a.N - e0) : TILE);
  const int my_n = n_el - lane * S < 0 ? 0 : (n_el - lane * S < S ? n_el - lane * S : S);  // elements of this lane
  const int64_t el = seq * a.N + e0 + (int64_t)lane * S;
  const T* Ae = static_cast<const T*>(a.A) + el * D * D;
  const T* be = static_cast<const T*>(a.b) + el * D;

  Aff<T, D> agg;
  aff_identity(agg);
  {
    constexpr int U = SH::UF;
    int s = 0;
    for (; s + U <= my_n; s += U) {
      T ea[U][D * D], eb[U][D];
#pragma unroll
      for (int u = 0; u < U; u++)
        wide_load_el<T, D>(ea[u], eb[u], Ae + (int64_t)(s + u) * D * D, be + (int64_t)(s + u) * D);
#pragma unroll
      for (int u = 0; u < U; u++) aff_before_g<T, D>(agg, ea[u], eb[u]);
    }
    for (; s < my_n; s++) aff_before_g<T, D>(agg, Ae + (int64_t)s * D * D, be + (int64_t)s * D);
  }
  // inclusive scan over the lanes (Hillis-Steele, partners read from LDS;
  // every lane's reads of a level precede its writes)
  aff_store_lds<T, D>(sX + lane * EP, agg);
  __syncthreads();
#pragma unroll
  for (int o = 1; o < NT; o <<= 1) {
    if (lane >= o) aff_after_lds<T, D>(agg, sX + (lane - o) * EP);
    __syncthreads();  // every lane has read the previous level
    aff_store_lds<T, D>(sX + lane * EP, agg);
    __syncthreads();
  }
  if (lane == NT - 1) aff_store_lds<T, D>(sT, agg);
  __syncthreads();

  const int64_t base = seq * a.tiles_per_seq;
  uint32_t* flags = a.flags + base;
  T* aggp = static_cast<T*>(a.agg) + base * E;
  T* inclp = static_cast<T*>(a.incl) + base * D;
  if (ts == 0) {
    if (lane < D) sZ[lane] = a.z0 ? static_cast<const T*>(a.z0)[seq * D + lane] : T(0);
  } else {
    for (int i = lane; i < E; i += NT) st_payload(aggp + ts * E + i, sT[i]);
    if (lane == 0) {
      publish_flag(flags, ts, FLAG_AGG, a.delay);
      aff_identity_lds<T, D>(sAcc);
    }
    __syncthreads();
    int64_t end = ts - 1;
    for (;;) {
      uint32_t f;
      const int k = lookback_window(flags, end, a.err, f);
      // aggregates end, end-1, ..., end-k+1, LW at a time (newest first):
      // acc <- acc o (m_0 o m_1 o ... o m_{n-1})
      for (int c0 = 0; c0 < k; c0 += LW) {
        const int n = (k - c0) < LW ? (k - c0) : LW;
        if (lane < LW) {
          T* my = sY + lane * EP;
          if (lane < n) {
            const T* src = aggp + (end - c0 - lane) * E;
            for (int i = 0; i < E; i++) my[i] = ld_payload(src + i);
          } else {
            aff_identity_lds<T, D>(my);
          }
        }
        __syncthreads();
#pragma unroll
        for (int off = 1; off < LW; off <<= 1) {
          // lane reads lane+off (not written at this level) and writes itself
          if (lane < LW && (lane & (2 * off - 1)) == 0) {
            Aff<T, D> v;
            aff_load_lds<T, D>(v, sY + lane * EP);
            aff_after_lds<T, D>(v, sY + (lane + off) * EP);
            aff_store_lds<T, D>(sY + lane * EP, v);
          }
          __syncthreads();
        }
        if (lane == 0) {
          Aff<T, D> v;
          aff_load_lds<T, D>(v, sAcc);
          aff_after_lds<T, D>(v, sY);
          aff_store_lds<T, D>(sAcc, v);
        }
        __syncthreads();  // sY is rewritten by the next pass; sAcc read below
      }
      if (k < PINT_WAVE) {
        const int64_t j = end - k;  // the inclusive predecessor
        if (lane < D) sZ[D + lane] = j >= 0 ? ld_payload(inclp + j * D + lane) : T(0);
        __syncthreads();
        if (lane < D) {
          T t = sAcc[D * D + lane];
#pragma unroll
          for (int q = 0; q < D; q++) t += sAcc[lane * D + q] * sZ[D + q];
          sZ[lane] = t;
        }
        break;
      }
      end -= PINT_WAVE;
    }
  }
  __syncthreads();  // z_in in sZ
  // this tile's inclusive vector
  if (lane < D) {
    T t = sT[D * D + lane];
#pragma unroll
    for (int q = 0; q < D; q++) t += sT[lane * D + q] * sZ[q];
    st_payload(inclp + ts * D + lane, t);
  }
  if (lane == 0) publish_flag(flags, ts, FLAG_INCL, a.delay);

  // outputs of this lane's run, from z at its start (the previous lane's
  // inclusive prefix applied to z_in)
  if (my_n > 0) {
    T z[D];
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < D; i++) z[i] = sZ[i];
    } else {
      const T* P = sX + (lane - 1) * EP;
#pragma unroll
      for (int i = 0; i < D; i++) {
        T t = P[D * D + i];
#pragma unroll
        for (int q = 0; q < D; q++) t += P[i * D + q] * sZ[q];
        z[i] = t;
      }
    }
    T* zg = static_cast<T*>(a.z) + el * D;
    constexpr int U = SH::UO;
    int s = 0;
    for (; s + U <= my_n; s += U) {
      T ea[U][D * D], eb[U][D];
#pragma unroll
      for (int u = 0; u < U; u++)
        wide_load_el<T, D>(ea[u], eb[u], Ae + (int64_t)(s + u) * D * D, be + (int64_t)(s + u) * D);
#pragma unroll
      for (int u = 0; u < U; u++) wide_apply<T, D>(z, ea[u], eb[u], zg + (int64_t)(s + u) * D);
    }
    for (; s < my_n; s++)
      wide_apply<T, D>(z, Ae + (int64_t)s * D * D, be + (int64_t)s * D, zg + (int64_t)s * D);
  }
}

// ----------------------------------------------------------- dense d ------

typedef double pint_d4 __attribute__((ext_vector_type(4)));
typedef float pint_f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {  // v_mfma_f64_16x16x4f64: acc (lane l, reg r) = (l/16 + 4r, l%16)
  using acc_t = pint_d4;
  __device__ static acc_t mma(double x, double y, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int r) { return lane / 16 + 4 * r; }
};
template <>
struct Mfma<float> {  // v_mfma_f32_16x16x4f32: acc (lane l, reg r) = (4(l/16) + r, l%16)
  using acc_t = pint_f4;
  __device__ static acc_t mma(float x, float y, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int r) { return 4 * (lane / 16) + r; }
};

// STAT ("stationary product", FP64): the running product stays in the MFMA
// accumulators, each wave owning ceil(NTL/4) column tiles (zero padded to DP)
// -- the FP64 16x16x4 accumulator layout (lane l, reg r) = (l/16 + 4r, l%16)
// is exactly the B-operand layout of the next product's k-steps -- and only
// the element being folded passes through LDS (rows padded to DP + 4).
// Otherwise the product lives in LDS and the element is read from HBM.
template <typename T, int D>
struct DenseScanShape {
  static constexpr int DP = (D + 15) / 16 * 16;    // padded to MFMA tiles
  static constexpr int NTL = DP / 16;               // 16x16 tiles per dimension
  static constexpr int NT = 256, NW = 4;
  static constexpr bool STAT = sizeof(T) == 8 && D % 2 == 0;
  static constexpr int CT = (NTL + NW - 1) / NW;    // STAT: column tiles per wave
  static constexpr int PS = STAT ? DP + 4 : ((DP % 32 == 0) ? DP + 16 : DP);  // LDS row stride
  static constexpr int RT = (NTL + NW - 1) / NW;   // row tiles per wave
};

template <typename T, int D>
constexpr size_t dense_scan_lds() {
  using SH = DenseScanShape<T, D>;
  return (size_t)SH::DP * SH::PS * sizeof(T) + 5 * (size_t)SH::DP * sizeof(T);
}

// z <- M z + c for a D x D row-major M in global memory, by the whole block;
// z, c and the result in LDS (tmp holds the new vector).
template <typename T, int D, int NT>
__device__ __forceinline__ void block_matvec_g(const T* M, const T* c, T* z, T* tmp, bool payload) {
  constexpr int QC = (D * 2 <= NT) ? ((D * 4 <= NT) ? 4 : 2) : 1;
  static_assert(D % QC == 0, "split");
  const int tid = threadIdx.x, i = tid / QC, q = tid % QC;
  T part = T(0);
  if (i < D) {
    const T* row = M + (int64_t)i * D + q * (D / QC);
    for (int k = 0; k < D / QC; k++)
      part += (payload ? ld_payload(row + k) : row[k]) * z[q * (D / QC) + k];
  }
#pragma unroll
  for (int off = 1; off < QC; off <<= 1) part += __shfl_xor(part, off, PINT_WAVE);
  if (i < D && q == 0) tmp[i] = part + (payload ? ld_payload(c + i) : c[i]);
  __syncthreads();
  if (tid < D) z[tid] = tmp[tid];
  __syncthreads();
}

// The tile's exclusive prefix z_in, into sz, for a tile whose aggregate
// (P, q) is in LDS (P with row stride PS, q in sq): publish the aggregate,
// look back to the nearest predecessor whose inclusive prefix is known,
// apply the aggregates in between, then publish this tile's inclusive prefix
// P z_in + q.  Whole block (NT threads); st is a D-vector of LDS scratch.
template <typename T, int D, int NT>
__device__ void tile_prefix(const ScanArgs& a, int64_t seq, int64_t ts, const T* sP, int PS,
                            const T* sq, T* sz, T* st) {
  constexpr int E = D * D + D;
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  const int64_t base = seq * a.tiles_per_seq;
  uint32_t* flags = a.flags + base;
  T* aggp = static_cast<T*>(a.agg) + base * E;
  T* inclp = static_cast<T*>(a.incl) + base * D;
  __shared__ int64_t s_j;
  if (ts == 0) {
    for (int i = tid; i < D; i += NT) sz[i] = a.z0 ? static_cast<const T*>(a.z0)[seq * D + i] : T(0);
    __syncthreads();
  } else {
    for (int idx = tid; idx < D * D; idx += NT) st_payload(aggp + ts * E + idx, sP[(idx / D) * PS + idx % D]);
    for (int i = tid; i < D; i += NT) st_payload(aggp + ts * E + D * D + i, sq[i]);
    __syncthreads();
    if (tid == 0) publish_flag(flags, ts, FLAG_AGG, a.delay);
    if (wv == 0) {
      // nearest predecessor whose inclusive prefix is known
      int64_t end = ts - 1;
      for (;;) {
        uint32_t f;
        const int k = lookback_window(flags, end, a.err, f);
        if (k < PINT_WAVE) {
          end -= k;
          break;
        }
        end -= PINT_WAVE;
      }
      if (lane == 0) s_j = end;
    }
    __syncthreads();
    const int64_t j = s_j;
    for (int i = tid; i < D; i += NT) sz[i] = ld_payload(inclp + j * D + i);
    __syncthreads();
    // the aggregates in between, oldest first, as matrix-vector products
    for (int64_t mm = j + 1; mm < ts; mm++)
      block_matvec_g<T, D, NT>(aggp + mm * E, aggp + mm * E + D * D, sz, st, true);
  }
  // publish this tile's inclusive prefix: P z_in + q
  {
    constexpr int QC = (D * 2 <= NT) ? ((D * 4 <= NT) ? 4 : 2) : 1;
    const int i = tid / QC, q = tid % QC;
    T part = T(0);
    if (i < D)
      for (int k = 0; k < D / QC; k++) part += sP[i * PS + q * (D / QC) + k] * sz[q * (D / QC) + k];
#pragma unroll
    for (int off = 1; off < QC; off <<= 1) part += __shfl_xor(part, off, PINT_WAVE);
    if (i < D && q == 0) st_payload(inclp + ts * D + i, part + sq[i]);
    __syncthreads();
    if (tid == 0) publish_flag(flags, ts, FLAG_INCL, a.delay);
  }
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_scan_dense(ScanArgs a) {
  using SH = DenseScanShape<T, D>;
  using MF = Mfma<T>;
  constexpr int DP = SH::DP, NTL = SH::NTL, PS = SH::PS, NT = SH::NT, RT = SH::RT;
  constexpr int E = D * D + D;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sP = reinterpret_cast<T*>(smem_raw);          // running product, DP x PS
  T* sq = sP + DP * PS;                             // running b-part
  T* sz = sq + DP;                                  // z vector
  T* st = sz + DP;                                  // scratch vector
  T* sq2 = st + DP;                                 // STAT: second b-part buffer
  T* sbm = sq2 + DP;                                // STAT: b_m of the element being folded
  __shared__ uint32_t s_tile;
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  if (tid == 0) s_tile = atomicAdd(a.counter, 1u);
  __syncthreads();
  // sequences interleaved in tile order: early tiles of every sequence first
  const int64_t tile = s_tile;
  const int64_t seq = tile % a.B, ts = tile / a.B;
  const int64_t e0 = ts * (int64_t)a.L;
  const int n_el = (int)((a.N - e0) < a.L ? (a.N - e0) : a.L);
  const T* Aseq = static_cast<const T*>(a.A) + (seq * a.N + e0) * D * D;
  const T* bseq = static_cast<const T*>(a.b) + (seq * a.N + e0) * D;

  // One tile per sequence: it starts from z0 and has no successor, so its
  // aggregate is never used; straight to the outputs.
  if (a.tiles_per_seq == 1) {
    for (int i = tid; i < D; i += NT) sz[i] = a.z0 ? static_cast<const T*>(a.z0)[seq * D + i] : T(0);
    __syncthreads();
  } else {
  if constexpr (SH::STAT) {
    // ---- stationary product: P in accumulators, A_m staged through LDS ----
    // AUG (D < DP): the element is staged as the augmented matrix
    // [[A_m, b_m], [0, 1]] in the padded rows and columns, and the product
    // holds [[P, q], [0, 1]], so the MFMA products carry the b-part too.
    static_assert(D % 2 == 0, "stationary shape: element pairs");
    constexpr bool AUG = D < DP;
    constexpr int CT = SH::CT, NPAIR = D * D / 2, NPF = (NPAIR + NT - 1) / NT;  // double2 loads per thread
    typedef double v2_t __attribute__((ext_vector_type(2)));
    // this wave's column tiles col0 .. col0+CT-1 (those < NTL); wave-uniform,
    // so the tests below are scalar branches around whole MFMA sequences
    // (a wave with only some of its CT tiles in range exists only when CT
    // does not divide NTL; otherwise a wave has all of them or none)
    constexpr bool PARTIAL = NTL % CT != 0;
    const int col0 = __builtin_amdgcn_readfirstlane(wv * CT);
    const bool mf_any = col0 < NTL, mf_full = col0 + CT <= NTL;
    auto col_ok = [&](int ct) { return !PARTIAL || mf_full || col0 + ct < NTL; };
    // the staging area starts zero except the augmented corner
    for (int i = tid; i < DP * PS; i += NT) sP[i] = (AUG && i == D * PS + D) ? T(1) : T(0);
    pint_d4 P[NTL][CT];
#pragma unroll
    for (int it = 0; it < NTL; it++)
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int row = 16 * it + lane / 16 + 4 * r, col = 16 * (col0 + ct) + lane % 16;
          T v = (row < D && col < D) ? Aseq[row * D + col] : T(0);
          if (AUG && col == D) v = row < D ? bseq[row] : (row == D ? T(1) : T(0));
          P[it][ct][r] = v;
        }
    if (!AUG)
      for (int i = tid; i < DP; i += NT) sq[i] = i < D ? bseq[i] : T(0);
    // the next PF elements in a register ring (slot u holds element m0 + u),
    // b_m included: a load issued after the ring's would make its use wait
    // for the whole ring.  The barriers in the loop order LDS only, so the
    // ring's loads stay in flight across them.
    constexpr int PF = NPF >= 16 ? 1 : (NPF >= 8 ? 2 : 4);
    constexpr int QC = (D * 4 <= NT) ? 4 : 2;  // !AUG b-part: threads per row
    v2_t pf[PF][NPF];
    T pb[PF];
    const int bi = tid < D ? tid : 0;
    // (unconditional loads, the last pair re-read past the end: a load
    // under a divergent branch makes the compiler's wait counts conservative
    // and the ring drains at every element)
    auto prefetch = [&](int m, v2_t (&slot)[NPF], T& bv) {
      const v2_t* src = reinterpret_cast<const v2_t*>(Aseq + (int64_t)m * D * D);
#pragma unroll
      for (int j = 0; j < NPF; j++) slot[j] = src[min(j * NT + tid, NPAIR - 1)];
      bv = bseq[(int64_t)m * D + bi];
    };
#pragma unroll
    for (int u = 0; u < PF; u++) prefetch(min(1 + u, n_el - 1), pf[u], pb[u]);
    // every load complete at the loop entry: one still pending there (in
    // whatever order the compiler issued the ring's first fill) would set
    // the wait counts inside the loop to zero, draining the ring each time
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();  // the staging area and b-part are visible
    // one element: stage slot, refill it with element m + PF, fold
    auto fold_one = [&](const int m, v2_t (&slot)[NPF], T& bslot) __attribute__((always_inline)) {
      lds_barrier();  // A_{m-1} (and the old b-part) no longer read
#pragma unroll
      for (int j = 0; j < NPF; j++) {
        if (j * NT + tid < NPAIR) {
          const int q = 2 * (j * NT + tid), i = q / D, k = q % D;
          sP[i * PS + k] = slot[j][0];
          sP[i * PS + k + 1] = slot[j][1];
        }
      }
      // b_m staged too (read back from LDS, not kept in a register across the
      // slot's refill: that makes the compiler wait for the refill)
      if (tid < D) {
        if (AUG) sP[tid * PS + D] = bslot;
        else sbm[tid] = bslot;
      }
      lds_barrier();  // A_m staged
      // refilled unconditionally (the last element again near the end): a
      // skipped refill on some path would shrink the wait counts everywhere
      prefetch(min(m + PF, n_el - 1), slot, bslot);  // lands while later elements run
      if (mf_any) {
        pint_d4 Pn[NTL][CT];
#pragma unroll
        for (int it = 0; it < NTL; it++)
#pragma unroll
          for (int ct = 0; ct < CT; ct++) Pn[it][ct] = pint_d4{};
#pragma unroll
        for (int kt = 0; kt < NTL; kt++) {
#pragma unroll
          for (int qk = 0; qk < 4; qk++) {
#pragma unroll
            for (int it = 0; it < NTL; it++) {
              const double av = sP[(16 * it + lane % 16) * PS + 16 * kt + 4 * qk + lane / 16];
#pragma unroll
              for (int ct = 0; ct < CT; ct++)
                if (col_ok(ct))
                  Pn[it][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, P[kt][ct][qk], Pn[it][ct], 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int it = 0; it < NTL; it++)
#pragma unroll
          for (int ct = 0; ct < CT; ct++) P[it][ct] = Pn[it][ct];
      }
      if constexpr (!AUG) {  // b-part A_m q + b_m, four chains per thread
        const T* qo = (m & 1) ? sq : sq2;  // after element m-1
        T* qn = (m & 1) ? sq2 : sq;        // after element m
        constexpr int SEG = D / QC;
        static_assert(SEG % 4 == 0, "b-part chains");
        const int i = tid / QC, h = tid % QC;
        if (i < D) {
          const T* row = sP + i * PS + h * SEG;
          const T* qv = qo + h * SEG;
          T c0 = h == 0 ? sbm[i] : T(0), c1 = T(0), c2 = T(0), c3 = T(0);
#pragma unroll
          for (int k = 0; k < SEG; k += 4) {
            c0 += row[k] * qv[k];
            c1 += row[k + 1] * qv[k + 1];
            c2 += row[k + 2] * qv[k + 2];
            c3 += row[k + 3] * qv[k + 3];
          }
          T part = (c0 + c1) + (c2 + c3);
          part += dpp_xor1(part);
          if (QC == 4) part += dpp_xor2(part);
          if (h == 0) qn[i] = part;
        }
      }
    };
    // whole groups of PF elements, then the rest: no exit from inside a
    // group, so on every path through the loop each slot is refilled once
    // per group and the wait counts keep the other slots' loads in flight
    int m0 = 1;
    for (; m0 + PF <= n_el; m0 += PF)
#pragma unroll
      for (int u = 0; u < PF; u++) fold_one(m0 + u, pf[u], pb[u]);
#pragma unroll
    for (int u = 0; u + 1 < PF; u++)
      if (m0 + u < n_el) fold_one(m0 + u, pf[u], pb[u]);
    // the tile's product into LDS (row stride PS) for the rest of the kernel
    __syncthreads();
    if (mf_any)
#pragma unroll
      for (int it = 0; it < NTL; it++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
          if (col_ok(ct))
#pragma unroll
            for (int r = 0; r < 4; r++)
              sP[(16 * it + lane / 16 + 4 * r) * PS + 16 * (col0 + ct) + lane % 16] = P[it][ct][r];
    if (!AUG && (n_el & 1) == 0)  // the final b-part is in sq2
      for (int i = tid; i < DP; i += NT) sq[i] = sq2[i];
    __syncthreads();
    if (AUG) {  // the b-part is column D of the product
      for (int i = tid; i < DP; i += NT) sq[i] = i < D ? sP[i * PS + D] : T(0);
      __syncthreads();
    }
  } else {
    // P <- A_0 (zero padded), q <- b_0
    for (int idx = tid; idx < DP * DP; idx += NT) {
      const int i = idx / DP, j = idx % DP;
      sP[i * PS + j] = (i < D && j < D) ? Aseq[i * D + j] : T(0);
    }
    for (int i = tid; i < DP; i += NT) sq[i] = i < D ? bseq[i] : T(0);
    __syncthreads();

  // fold the remaining elements: (P, q) <- (A_m P, A_m q + b_m)
  for (int m = 1; m < n_el; m++) {
    const T* Am = Aseq + (int64_t)m * D * D;
    typename MF::acc_t acc[RT][NTL];
#pragma unroll
    for (int r = 0; r < RT; r++)
#pragma unroll
      for (int c = 0; c < NTL; c++) acc[r][c] = typename MF::acc_t{};
#pragma unroll 2
    for (int kk = 0; kk < DP / 4; kk++) {
      const int k = kk * 4 + lane / 16;
      T av[RT];
#pragma unroll
      for (int r = 0; r < RT; r++) {
        const int rt = wv + r * SH::NW;
        const int i = rt * 16 + lane % 16;
        av[r] = (rt < NTL && i < D && k < D) ? Am[i * D + k] : T(0);
      }
#pragma unroll
      for (int c = 0; c < NTL; c++) {
        const T bv = sP[k * PS + c * 16 + lane % 16];
#pragma unroll
        for (int r = 0; r < RT; r++)
          if (wv + r * SH::NW < NTL) acc[r][c] = MF::mma(av[r], bv, acc[r][c]);
      }
    }
    // q_new = A_m q + b_m (uses the old q, before P and q are overwritten)
    {
      constexpr int QC = (D * 2 <= NT) ? ((D * 4 <= NT) ? 4 : 2) : 1;
      const int i = tid / QC, q = tid % QC;
      T part = T(0);
      if (i < D)
        for (int k = 0; k < D / QC; k++) part += Am[(int64_t)i * D + q * (D / QC) + k] * sq[q * (D / QC) + k];
#pragma unroll
      for (int off = 1; off < QC; off <<= 1) part += __shfl_xor(part, off, PINT_WAVE);
      if (i < D && q == 0) st[i] = part + bseq[(int64_t)m * D + i];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RT; r++) {
      const int rt = wv + r * SH::NW;
      if (rt < NTL)
#pragma unroll
        for (int c = 0; c < NTL; c++)
#pragma unroll
          for (int v = 0; v < 4; v++) sP[(rt * 16 + MF::row(lane, v)) * PS + c * 16 + lane % 16] = acc[r][c][v];
    }
    if (tid < D) sq[tid] = st[tid];
    __syncthreads();
  }
  }  // generic fold

  tile_prefix<T, D, NT>(a, seq, ts, sP, PS, sq, sz, st);
  }  // tiles_per_seq > 1

  // outputs: z_{e0+m+1} = A_m z + b_m in order.  QC threads per row; each
  // thread's row segment of A_{m+1} and b_{m+1} are loaded during element m
  // (the barriers order LDS only, so those loads stay in flight).
  T* zg = static_cast<T*>(a.z) + (seq * a.N + e0) * D;
  {
    constexpr int QC = (D * 2 <= NT) ? ((D * 4 <= NT) ? 4 : 2) : 1, SEG = D / QC;
    static_assert(D % QC == 0, "row split");
    const int i = tid / QC, h = tid % QC;
    const bool act = i < D;
    const int ii = act ? i : 0;
    // ring of the next PO elements' row segments (slot u: element m0 + u)
    constexpr int PO = SEG > 16 ? 2 : 4;
    T ring[PO][SEG], rb[PO];
    auto fetch = [&](int m, T (&seg)[SEG], T& bv) {
      const T* Am = Aseq + (int64_t)m * D * D + (int64_t)ii * D + h * SEG;
#pragma unroll
      for (int k = 0; k < SEG; k++) seg[k] = Am[k];
      bv = bseq[(int64_t)m * D + ii];
    };
#pragma unroll
    for (int u = 0; u < PO; u++) fetch(min(u, n_el - 1), ring[u], rb[u]);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): as in the fold
    // z alternates between sz (even m reads it) and st (odd m reads it): a
    // buffer is rewritten only after the barrier that ends its readers
    auto out_one = [&](const int m, T (&seg)[SEG], T& bv) __attribute__((always_inline)) {
      const T* zc = (m & 1) ? st : sz;
      T* zn = (m & 1) ? sz : st;
      // b_m enters at the head of the chain (lane h == 0), so the slot's old
      // value is dead before its refill is issued
      T c0 = h == 0 ? bv : T(0), c1 = T(0);
#pragma unroll
      for (int k = 0; k + 1 < SEG; k += 2) {
        c0 += seg[k] * zc[h * SEG + k];
        c1 += seg[k + 1] * zc[h * SEG + k + 1];
      }
      if (SEG & 1) c0 += seg[SEG - 1] * zc[h * SEG + SEG - 1];
      T part = c0 + c1;
      if (QC >= 2) part += dpp_xor1(part);
      if (QC >= 4) part += dpp_xor2(part);
      const T zv = part;
      fetch(min(m + PO, n_el - 1), seg, bv);  // unconditional: see the fold
      if (act && h == 0) {
        zn[i] = zv;
        zg[(int64_t)m * D + i] = zv;
      }
      lds_barrier();
    };
    int m0 = 0;  // whole groups, then the rest (as in the fold)
    for (; m0 + PO <= n_el; m0 += PO)
#pragma unroll
      for (int u = 0; u < PO; u++) out_one(m0 + u, ring[u], rb[u]);
#pragma unroll
    for (int u = 0; u + 1 < PO; u++)
      if (m0 + u < n_el) out_one(m0 + u, ring[u], rb[u]);
  }
}

// ------------------------------------------------------- banded scan ------
//
// Elements whose A is cyclically banded with BW diagonals,
//   A(i, (i + k - BOFF) mod D) = band[i * BW + k]  for k < BW,
// every other entry zero: the Jacobian of an RK4 step of a short-stencil
// system, or its transpose in the adjoint.  An element is D*BW band values
// (row-major) plus b.  The tile's running product fills in after a few
// elements, so P stays dense; only the element is banded, and
//   (A_m P)(i, c) = sum_k band_m[i][k] P((i + k - BOFF) mod D, c)
// costs BW multiply-adds per entry on the vector units (instead of D, padded,
// on matrix tiles).  The b-part rides along as column D of [P | q]: b_m
// enters that column only.  Each wave owns RW rows of the product, its lanes
// the D + 1 columns; a lane reads its column of the old product once per
// element (WIN rows).  The element is staged diagonal-major, so for each
// diagonal k the RW band values of the wave's rows are one contiguous LDS
// broadcast feeding RW independent accumulators.
//
// Output pass (k_scan_band_out): one wave per tile walks the tile's
// elements, lane i holding row i of the band in registers (a ring of the
// next PO elements' rows) and reading z from an extended copy
// zx[j] = z[(j - BOFF) mod D], j < D + BW - 1, so its BW operands are
// zx[i .. i+BW-1].
template <typename T, int D, int BW, int BOFF>
struct BandScanShape {
  static constexpr int NT = 256, NW = NT / PINT_WAVE;
  static constexpr int RW = (D + NW - 1) / NW;  // product rows per wave
  static constexpr int NC = D + 1;              // columns: P and q
  static constexpr int PSB = D + 1;             // LDS row stride of [P | q]
  static constexpr int EL = (BW + 1) * D;        // staged element: band[k][i] (k-major), then b
  static constexpr int NB = D * BW;             // band values per element
  static constexpr int NPR = NB / 2;            // ... as pairs
  static constexpr int NLD = (NPR + NT - 1) / NT;  // pair loads per thread per element
  static constexpr int ZX = D + BW - 1;         // extended z
  static constexpr int WIN = RW + BW - 1;       // rows of the old product one wave reads
  static constexpr int PF = 4, PO = 4;          // ring depths (fold, output)
  static_assert(NB % 2 == 0, "band values in pairs");
  static_assert(NC <= PINT_WAVE, "a column per lane");
  static_assert(D >= 2 * BW && BOFF < BW, "band must not wrap onto itself");
};

template <typename T, int D, int BW, int BOFF>
__global__ __launch_bounds__(256) void k_scan_band(ScanArgs a) {
  using SH = BandScanShape<T, D, BW, BOFF>;
  constexpr int NT = SH::NT, RW = SH::RW, NC = SH::NC, PSB = SH::PSB, EL = SH::EL;
  constexpr int NB = SH::NB, NPR = SH::NPR, NLD = SH::NLD, WIN = SH::WIN, PF = SH::PF;
  __shared__ T sPb[2][D * PSB];  // [P | q], ping-pong
  __shared__ T sEl[2][EL];       // staged elements, ping-pong
  __shared__ T sq[D], sz[D], st[D];
  __shared__ uint32_t s_tile;
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  if (tid == 0) s_tile = atomicAdd(a.counter, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t seq = tile % a.B, ts = tile / a.B;
  const int64_t e0 = ts * (int64_t)a.L;
  const int n_el = (int)((a.N - e0) < a.L ? (a.N - e0) : a.L);
  const T* Bseq = static_cast<const T*>(a.A) + (seq * a.N + e0) * NB;
  const T* bseq = static_cast<const T*>(a.b) + (seq * a.N + e0) * D;

  typedef T v2_t __attribute__((ext_vector_type(2)));
  const int bi = tid < D ? tid : 0;
  // unconditional loads (the last pair / element again past the end), as
  // in the dense scan: the ring's loads stay in flight across the loop
  auto fetch = [&](int m, v2_t (&slot)[NLD], T& bv) {
    const v2_t* src = reinterpret_cast<const v2_t*>(Bseq + (int64_t)m * NB);
#pragma unroll
    for (int j = 0; j < NLD; j++) slot[j] = src[min(j * NT + tid, NPR - 1)];
    bv = bseq[(int64_t)m * D + bi];
  };
  auto stage = [&](const v2_t (&slot)[NLD], T bv, T* el) {
#pragma unroll
    for (int j = 0; j < NLD; j++) {
      const int pr = j * NT + tid;
      if (pr < NPR) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const int f = 2 * pr + h, i = f / BW, k = f % BW;
          el[k * D + i] = slot[j][h];
        }
      }
    }
    if (tid < D) el[BW * D + tid] = bv;
  };

  // ---- prologue: elements 0 and 1 staged, P <- A_0 (dense), q <- b_0 ----
  v2_t ring[PF][NLD];
  T rb[PF];
  {
    v2_t s0[NLD], s1[NLD];
    T b0, b1;
    fetch(0, s0, b0);
    fetch(min(1, n_el - 1), s1, b1);
#pragma unroll
    for (int u = 0; u < PF; u++) fetch(min(2 + u, n_el - 1), ring[u], rb[u]);
    stage(s0, b0, sEl[0]);
    stage(s1, b1, sEl[1]);
  }
  __syncthreads();
  for (int idx = tid; idx < D * PSB; idx += NT) {
    const int r = idx / PSB, c = idx % PSB;
    T v = T(0);
    if (c == D) {
      v = sEl[0][BW * D + r];
    } else {
      int k = c - r + BOFF;
      k = k < 0 ? k + D : (k >= D ? k - D : k);
      if (k < BW) v = sEl[0][k * D + r];
    }
    sPb[0][idx] = v;
  }
  // every load complete at the loop entry (see the dense scan's fold)
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  __syncthreads();

  // ---- fold: step m computes P_m = A_m P_{m-1} (element m staged in step
  // m-1) and stages element m+1; one barrier per step ----
  const int r0 = wv * RW;
  auto fold_one = [&](const int m, v2_t (&slot)[NLD], T& bslot) __attribute__((always_inline)) {
    stage(slot, bslot, sEl[(m + 1) & 1]);  // last read in step m-1
    fetch(min(m + 1 + PF, n_el - 1), slot, bslot);
    const T* el = sEl[m & 1];
    const T* Po = sPb[(m - 1) & 1];
    T* Pn = sPb[m & 1];
    if (lane < NC && r0 < D) {
      T pc[WIN];
#pragma unroll
      for (int w = 0; w < WIN; w++) {
        int row = r0 - BOFF + w;
        row = row < 0 ? row + D : (row >= D ? row - D : row);
        pc[w] = Po[row * PSB + lane];
      }
      static_assert(D % SH::NW == 0, "whole row blocks per wave");
      T acc[RW];
#pragma unroll
      for (int rr = 0; rr < RW; rr++) acc[rr] = lane == D ? el[BW * D + r0 + rr] : T(0);
#pragma unroll
      for (int k = 0; k < BW; k++)
#pragma unroll
        for (int rr = 0; rr < RW; rr++) acc[rr] += el[k * D + r0 + rr] * pc[rr + k];
#pragma unroll
      for (int rr = 0; rr < RW; rr++) Pn[(r0 + rr) * PSB + lane] = acc[rr];
    }
    lds_barrier();
  };
  int m0 = 1;  // whole groups of PF steps, then the rest
  for (; m0 + PF <= n_el; m0 += PF)
#pragma unroll
    for (int u = 0; u < PF; u++) fold_one(m0 + u, ring[u], rb[u]);
#pragma unroll
  for (int u = 0; u + 1 < PF; u++)
    if (m0 + u < n_el) fold_one(m0 + u, ring[u], rb[u]);
  const T* Pf = sPb[(n_el - 1) & 1];
  for (int i = tid; i < D; i += NT) sq[i] = Pf[i * PSB + D];
  __syncthreads();

  tile_prefix<T, D, NT>(a, seq, ts, Pf, PSB, sq, sz, st);

}

// Output pass of the banded scan, a launch of its own after k_scan_band (so
// the fold keeps few registers and four workgroups per compute unit): one
// wave per tile walks its elements, z_{e0+m+1} = A_m z + b_m, from the
// tile's starting vector (the previous tile's published inclusive prefix,
// or z0).  Lane i holds row i of the band for the next PO elements in
// registers and reads z from the extended copy zx (see above).
template <typename T, int D, int BW, int BOFF>
__global__ __launch_bounds__(64) void k_scan_band_out(ScanArgs a) {
  using SH = BandScanShape<T, D, BW, BOFF>;
  constexpr int NB = SH::NB, ZX = SH::ZX, PO = SH::PO;
  __shared__ T zx[2][ZX];
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t seq = tile % a.B, ts = tile / a.B;
  const int64_t e0 = ts * (int64_t)a.L;
  const int n_el = (int)((a.N - e0) < a.L ? (a.N - e0) : a.L);
  const T* Bseq = static_cast<const T*>(a.A) + (seq * a.N + e0) * NB;
  const T* bseq = static_cast<const T*>(a.b) + (seq * a.N + e0) * D;
  T* zg = static_cast<T*>(a.z) + (seq * a.N + e0) * D;
  const bool act = lane < D;
  const int i = act ? lane : 0;
  auto put = [&](T* zb, T v) {
    zb[i + BOFF] = v;
    if (i + BOFF >= D) zb[i + BOFF - D] = v;
    if (i + BOFF + D < ZX) zb[i + BOFF + D] = v;
  };
  T zin;
  if (ts == 0)
    zin = a.z0 ? static_cast<const T*>(a.z0)[seq * D + i] : T(0);
  else
    zin = static_cast<const T*>(a.incl)[(seq * a.tiles_per_seq + ts - 1) * D + i];
  if (act) put(zx[0], zin);
  T row[PO][BW], rbo[PO];
  auto fetch_row = [&](int m, T (&rw)[BW], T& bv) {
    const T* src = Bseq + (int64_t)m * NB + i * BW;
#pragma unroll
    for (int k = 0; k < BW; k++) rw[k] = src[k];
    bv = bseq[(int64_t)m * D + i];
  };
#pragma unroll
  for (int u = 0; u < PO; u++) fetch_row(min(u, n_el - 1), row[u], rbo[u]);
  // every load complete at the loop entry (see the dense scan's fold)
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  __builtin_amdgcn_wave_barrier();
  auto out_one = [&](const int m, T (&rw)[BW], T& bv) __attribute__((always_inline)) {
    const T* zc = zx[m & 1];
    T* zn = zx[(m + 1) & 1];
    T acc0 = bv, acc1 = T(0);
#pragma unroll
    for (int k = 0; k + 1 < BW; k += 2) {
      acc0 += rw[k] * zc[i + k];
      acc1 += rw[k + 1] * zc[i + k + 1];
    }
    if (BW & 1) acc0 += rw[BW - 1] * zc[i + BW - 1];
    const T zv = acc0 + acc1;
    fetch_row(min(m + PO, n_el - 1), rw, bv);
    if (act) {
      put(zn, zv);
      zg[(int64_t)m * D + i] = zv;
    }
    // the wave's LDS operations complete in order: the next element's reads
    // see these writes; keep the compiler from moving them across
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
  };
  int m0 = 0;  // whole groups of PO, then the rest (as in the dense scan)
  for (; m0 + PO <= n_el; m0 += PO)
#pragma unroll
    for (int u = 0; u < PO; u++) out_one(m0 + u, row[u], rbo[u]);
#pragma unroll
  for (int u = 0; u + 1 < PO; u++)
    if (m0 + u < n_el) out_one(m0 + u, row[u], rbo[u]);
}

// ------------------------------------------------------------- host -------

static int scan_tile_elems(int d, int dtype, int tile) {
  if (d <= 8) {
    switch (d) {
#define PINT_SMALL_TILE(DD)                                                               \
  case DD:                                                                                \
    return dtype == 0 ? (DD >= 4 ? WideShape<DD, double>::TILE : SmallShape<DD, double>::TILE) \
                      : (DD >= 4 ? WideShape<DD, float>::TILE : SmallShape<DD, float>::TILE);
      PINT_SMALL_TILE(1) PINT_SMALL_TILE(2) PINT_SMALL_TILE(3) PINT_SMALL_TILE(4)
      PINT_SMALL_TILE(5) PINT_SMALL_TILE(6) PINT_SMALL_TILE(7) PINT_SMALL_TILE(8)
#undef PINT_SMALL_TILE
    }
    return 0;
  }
  if (tile > 0) return tile;
  return 0;  // dense default: chosen from N, B and the CU count (dense_tile_len)
}

// Dense default tile length: enough tiles for one per compute unit, so the
// chain of inclusive prefixes between tiles stays short; one tile per
// sequence (no fold, see k_scan_dense) once the sequences alone fill half of
// the compute units.
static int dense_tile_len(int64_t B, int64_t N) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t per_seq_tiles = 2 * B >= cus ? 1 : (cus + B - 1) / B;
  int64_t L = (N + per_seq_tiles - 1) / per_seq_tiles;
  if (L < 1) L = 1;
  if (L > (1 << 20)) L = 1 << 20;
  return (int)L;
}

static bool scan_dense_d(int d) { return d == 16 || d == 32 || d == 40 || d == 64 || d == 128; }

size_t scan_ws_bytes(int d, int64_t B, int64_t N, int tile, int dtype) {
  if (d < 1 || B < 0 || N < 0) return 0;
  if (d > 8 && !scan_dense_d(d)) return 0;
  int L = scan_tile_elems(d, dtype, tile);
  if (L <= 0 && d > 8) L = dense_tile_len(B, N);
  if (L <= 0) return 0;
  const int64_t tps = (N + L - 1) / L;
  const int64_t nt = B * tps;
  const size_t s = dtype == 0 ? 8 : 4;
  return 256 + align_up((size_t)nt * 4) + align_up((size_t)nt * (d * d + d) * s) +
         align_up((size_t)nt * d * s);
}

template <typename T, int D>
static int launch_small(const ScanArgs& sa, int64_t grid, hipStream_t s) {
  if constexpr (D >= 4) {
    constexpr size_t lds = WideShape<D, T>::LDS;
    static bool attr_set = false;
    if (!attr_set) {
      if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_scan_wide<T, D>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return ST_DEVICE;
      attr_set = true;
    }
    hipLaunchKernelGGL((k_scan_wide<T, D>), dim3((unsigned)grid), dim3(64), lds, s, sa);
  } else {
    hipLaunchKernelGGL((k_scan_small<T, D>), dim3((unsigned)grid), dim3(SmallShape<D, T>::NT), 0, s, sa);
  }
  return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
}

template <typename T, int D>
static int launch_dense(const ScanArgs& sa, int64_t grid, hipStream_t s) {
  const size_t lds = dense_scan_lds<T, D>();
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_scan_dense<T, D>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return ST_DEVICE;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_scan_dense<T, D>), dim3((unsigned)grid), dim3(256), lds, s, sa);
  return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
}

int affine_scan(int d, int64_t B, int64_t N, int dtype, const void* A, const void* b,
                const void* z0, void* z, int tile, void* ws, size_t ws_bytes, hipStream_t s) {
  if (d > 8 && !scan_dense_d(d)) return ST_UNSUPPORTED;
  if (dtype != 0 && dtype != 1) return ST_INVALID;
  const size_t need = scan_ws_bytes(d, B, N, tile, dtype);
  if (!ws || ws_bytes < need) return ST_WORKSPACE;
  int L = scan_tile_elems(d, dtype, tile);
  if (L <= 0 && d > 8) L = dense_tile_len(B, N);
  if (L <= 0) return ST_INVALID;
  const int64_t tps = (N + L - 1) / L;
  const int64_t nt = B * tps;
  if (nt > 0x7fffffffLL) return ST_INVALID;
  const size_t sz = dtype == 0 ? 8 : 4;
  char* w = static_cast<char*>(ws);
  ScanArgs sa{};
  sa.B = B;
  sa.N = N;
  sa.tiles_per_seq = tps;
  sa.L = L;
  sa.A = A;
  sa.b = b;
  sa.z0 = z0;
  sa.z = z;
  sa.counter = reinterpret_cast<uint32_t*>(w);
  sa.err = reinterpret_cast<uint32_t*>(w) + 1;
  sa.flags = reinterpret_cast<uint32_t*>(w + 256);
  sa.agg = w + 256 + align_up((size_t)nt * 4);
  sa.incl = w + 256 + align_up((size_t)nt * 4) + align_up((size_t)nt * (d * d + d) * sz);
  sa.delay = scan_delay();
  // reset the tile counter, error word and flags (a kernel, not a memset)
  if (int rc = fill_u32(reinterpret_cast<uint32_t*>(w), 64 + (size_t)nt, 0u, s)) return rc;
#define PINT_CASE_SMALL(DD) \
  case DD: return dtype == 0 ? launch_small<double, DD>(sa, nt, s) : launch_small<float, DD>(sa, nt, s);
#define PINT_CASE_DENSE(DD) \
  case DD: return dtype == 0 ? launch_dense<double, DD>(sa, nt, s) : launch_dense<float, DD>(sa, nt, s);
  switch (d) {
    PINT_CASE_SMALL(1) PINT_CASE_SMALL(2) PINT_CASE_SMALL(3) PINT_CASE_SMALL(4)
    PINT_CASE_SMALL(5) PINT_CASE_SMALL(6) PINT_CASE_SMALL(7) PINT_CASE_SMALL(8)
    PINT_CASE_DENSE(16) PINT_CASE_DENSE(32) PINT_CASE_DENSE(40) PINT_CASE_DENSE(64)
    PINT_CASE_DENSE(128)
  }
#undef PINT_CASE_SMALL
#undef PINT_CASE_DENSE
  return ST_UNSUPPORTED;
}


// ------------------------------------------------------------ banded ------

// Band shapes compiled: d = 40 with 13 diagonals, offset 8 (the RK4 Jacobian
// of Lorenz-96) or 4 (its transpose).
static bool scan_band_shape(int d, int bw, int boff) {
  return d == 40 && bw == 13 && (boff == 4 || boff == 8);
}

// Band default tile length.  With at least half as many sequences as compute
// units the sequences alone fill the device: one tile per sequence, whose
// starting vector is known, so no fold at all (the output pass is the plain
// recursion, BW multiply-adds per entry instead of the fold's D*BW).
// Otherwise about four tiles per compute unit.
static int band_tile_len(int64_t B, int64_t N) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (2 * B >= cus) return (int)(N < 1 ? 1 : (N > (1 << 30) ? (1 << 30) : N));
  const int64_t per_seq_tiles = (4 * (int64_t)cus + B - 1) / B;
  int64_t L = (N + per_seq_tiles - 1) / per_seq_tiles;
  if (L < 16) L = 16;
  if (L > (1 << 20)) L = 1 << 20;
  return (int)L;
}

size_t scan_band_ws_bytes(int d, int bw, int boff, int64_t B, int64_t N, int tile, int dtype) {
  if (!scan_band_shape(d, bw, boff) || B < 0 || N < 0 || tile < 0) return 0;
  const int L = tile > 0 ? tile : band_tile_len(B, N);
  const int64_t nt = B * ((N + L - 1) / L);
  const size_t s = dtype == 0 ? 8 : 4;
  return 256 + align_up((size_t)nt * 4) + align_up((size_t)nt * (d * d + d) * s) +
         align_up((size_t)nt * d * s);
}

template <typename T, int BOFF>
static int launch_band(const ScanArgs& sa, int64_t grid, hipStream_t s) {
  // one tile per sequence: every tile starts from z0, no aggregates needed
  if (sa.tiles_per_seq > 1) {
    hipLaunchKernelGGL((k_scan_band<T, 40, 13, BOFF>), dim3((unsigned)grid), dim3(256), 0, s, sa);
    if (hipGetLastError() != hipSuccess) return ST_DEVICE;
  }
  hipLaunchKernelGGL((k_scan_band_out<T, 40, 13, BOFF>), dim3((unsigned)grid), dim3(64), 0, s, sa);
  return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
}

int affine_scan_band(int d, int bw, int boff, int64_t B, int64_t N, int dtype, const void* band,
                     const void* b, const void* z0, void* z, int tile, void* ws, size_t ws_bytes,
                     hipStream_t s) {
  if (!scan_band_shape(d, bw, boff)) return ST_UNSUPPORTED;
  if ((dtype != 0 && dtype != 1) || tile < 0) return ST_INVALID;
  const size_t sz = dtype == 0 ? 8 : 4;
  // the band is read in pairs of values
  if (reinterpret_cast<uintptr_t>(band) % (2 * sz) != 0) return ST_INVALID;
  const size_t need = scan_band_ws_bytes(d, bw, boff, B, N, tile, dtype);
  if (!ws || ws_bytes < need) return ST_WORKSPACE;
  const int L = tile > 0 ? tile : band_tile_len(B, N);
  const int64_t tps = (N + L - 1) / L;
  const int64_t nt = B * tps;
  if (nt > 0x7fffffffLL) return ST_INVALID;
  char* w = static_cast<char*>(ws);
  ScanArgs sa{};
  sa.B = B;
  sa.N = N;
  sa.tiles_per_seq = tps;
  sa.L = L;
  sa.A = band;
  sa.b = b;
  sa.z0 = z0;
  sa.z = z;
  sa.counter = reinterpret_cast<uint32_t*>(w);
  sa.err = reinterpret_cast<uint32_t*>(w) + 1;
  sa.flags = reinterpret_cast<uint32_t*>(w + 256);
  sa.agg = w + 256 + align_up((size_t)nt * 4);
  sa.incl = w + 256 + align_up((size_t)nt * 4) + align_up((size_t)nt * (d * d + d) * sz);
  sa.delay = scan_delay();
  if (int rc = fill_u32(reinterpret_cast<uint32_t*>(w), 64 + (size_t)nt, 0u, s)) return rc;
  if (boff == 4) return dtype == 0 ? launch_band<double, 4>(sa, nt, s) : launch_band<float, 4>(sa, nt, s);
  return dtype == 0 ? launch_band<double, 8>(sa, nt, s) : launch_band<float, 8>(sa, nt, s);
}

// ------------------------------------------- fixed-scratch scan variant --

// The scratch of pint_affine_scan_noalloc: a file-scope device array in place
// of a caller workspace, one copy per device, reserved when the library's code
// object is loaded on that device and held until the process ends.  In host
// code `scratch` names a host-side stand-in, not device memory: its device
// address is looked up once per device with hipGetSymbolAddress (that device
// current) and only that address is ever passed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = PINT_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

static int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return ST_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ST_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ST_OK;
}

__global__ void k_copy_word(const uint32_t* src, uint32_t* dst) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    *dst = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

int affine_scan_noalloc(int d, int64_t B, int64_t N, int dtype, const void* A, const void* b,
                        const void* z0, void* z, int tile, uint32_t* err_out, hipStream_t s) {
  if (d > 8 && !scan_dense_d(d)) return ST_UNSUPPORTED;
  if (dtype != 0 && dtype != 1) return ST_INVALID;
  const size_t need = scan_ws_bytes(d, B, N, tile, dtype);
  if (need == 0) return ST_INVALID;
  if (need > NOALLOC_SCRATCH_BYTES) return ST_WORKSPACE;
  void* p = nullptr;
  if (int rc = scratch_address(&p)) return rc;
  // affine_scan clears the tile counter, the error word and the flags it
  // uses with a fill kernel first, so what an earlier call left is harmless
  if (int rc = affine_scan(d, B, N, dtype, A, b, z0, z, tile, p, NOALLOC_SCRATCH_BYTES, s))
    return rc;
  if (err_out) {  // the error word sits at byte offset 4 of the scratch
    hipLaunchKernelGGL(k_copy_word, dim3(1), dim3(64), 0, s,
                       static_cast<const uint32_t*>(p) + 1, err_out);
    if (hipGetLastError() != hipSuccess) return ST_DEVICE;
  }
  return ST_OK;
}

}  // namespace pint
