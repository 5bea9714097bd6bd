// Dense state dimension (Lorenz-96 d=40, Kuramoto d=128): one workgroup of
// 512 threads per instance runs the Newton loop of Sec. 3.2 on chip.  Waves
// evaluate RK4 steps (a lane per component), Jacobian columns are built by
// one thread (or a quad) per column from the stage points in LDS and stored
// transposed in the workspace, and the Newton step of the window is the
// affine recursion of eq. newton-step-recursion folded in order inside the
// workgroup (a window is one scan tile).  Instances come from a device work
// queue.  Also the wave-per-instance sequential comparator and the residual
// and element kernels.
#include "internal.h"
#include "systems_dense.h"

namespace pint {

struct DenseKArgs {
  int64_t B;
  const void* x0;
  const void* params;
  int64_t pstride;
  int64_t T_uniform;
  void* traj;
  double dt, tol, guard;
  int64_t window, max_iter;
  int32_t guess;
  int64_t* iters;
  double* resid;
  int32_t* status;
  uint32_t* queue;
  void* ws_elems;        // per workgroup slot: AT [Wt][D][D], b [Wt][D], dx [Wt][D], hn [Wt]
  int64_t Wt;            // elements per slot (window + slack, or T in plain mode)
  int64_t slot_stride;   // scalars between consecutive workgroup slots
  uint64_t wait_limit;   // polls before a cross-workgroup wait gives up
};

// Slot: AT [Wt][D][D] (or the band), b [Wt][D], dx [Wt][D], then the
// per-step residual norms hn [Wt] (double, 8-byte aligned).
template <class S>
__host__ __device__ constexpr int64_t slot_hn_offset(int64_t Wt) {
  return (Wt * (int64_t)S::D * S::D + 2 * Wt * (int64_t)S::D + 1) / 2 * 2;
}
template <class S>
__host__ __device__ constexpr int64_t slot_scalars(int64_t Wt) {
  return slot_hn_offset<S>(Wt) + 2 * Wt;  // hn in doubles (2 scalars of float each)
}

// Speculative slack of the cooperative solver: each update builds the
// elements of W + slack steps from the previous window start, so the next
// first violation (which moves ahead some steps per update) is read off
// their residuals instead of being searched for separately.
__host__ __device__ constexpr int64_t spec_slack(int64_t W) { return W / 2 > 32 ? W / 2 : 32; }

// Load this lane's components of state n (0 -> x0 from LDS).
template <typename T, class S>
__device__ __forceinline__ void wave_load(const T* X, const T* x0s, int64_t n, T (&x)[S::R], int lane) {
#pragma unroll
  for (int r = 0; r < S::R; r++) {
    const int i = lane + 64 * r;
    x[r] = (i < S::D) ? (n == 0 ? x0s[i] : X[(n - 1) * S::D + i]) : T(0);
  }
}

// ||x_n - Phi(x_{n-1})||_inf by one wave.
template <typename T, class S>
__device__ __forceinline__ double wave_resid(const T* P, T dt, const T* X, const T* x0s, int64_t n,
                                             int lane) {
  T xp[S::R], xc[S::R], phi[S::R];
  wave_load<T, S>(X, x0s, n - 1, xp, lane);
  wave_load<T, S>(X, x0s, n, xc, lane);
  wave_rk4<T, S>(P, dt, xp, phi, nullptr, lane);
  double m = 0.0;
#pragma unroll
  for (int r = 0; r < S::R; r++)
    if (lane + 64 * r < S::D) m = acc_norm(m, xc[r] - phi[r]);
  return wave_max(m);
}

// ------------------------------------------------- workgroup phases ------

template <class S>
struct DenseShape {
  static constexpr int D = S::D, NT = S::NT, NW = NT / PINT_WAVE;
  // recursion: QC adjacent threads per row, D*QC <= NT
  static constexpr int QC = (D * 4 <= NT && D % 4 == 0) ? 4 : ((D * 2 <= NT && D % 2 == 0) ? 2 : 1);
  static constexpr int JC = D / QC;
  static_assert(D * QC <= NT, "row split");
};

// Element pass shape: steps per pass and Jacobian threads per step.  A
// banded system builds one band column per thread (S::jac_band_column), so
// NT / D steps fit in a pass; otherwise S::SPP steps of S::JT threads.
template <class S, bool B = S::BANDED>
struct ElemShape {
  static constexpr int JT = S::JT, SPP = S::SPP;
};
template <class S>
struct ElemShape<S, true> {
  static constexpr int JT = S::D, SPP = S::NT / S::D;
};

// Shared-memory state of a dense solver workgroup.
template <typename T, class S>
struct DenseSmem {
  typename S::Stage stage[ElemShape<S>::SPP];
  T P[S::NP], x0[S::D], z[2][S::D];
  double red[S::NT / PINT_WAVE];
  int64_t redi[S::NT / PINT_WAVE];
  double wres[S::NT / PINT_WAVE];
};

// First step n >= p with ||h_n|| >= tol (or not finite): rounds of NW steps,
// a wave per step.  Returns INT64_MAX if none; *hp receives ||h_fv||.
template <typename T, class S>
__device__ __forceinline__ int64_t dn_search(DenseSmem<T, S>& sm, T dt, const T* X, int64_t Tn, int64_t p, double tol,
                             double* hp) {
  constexpr int NT = S::NT, NW = NT / PINT_WAVE;
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  int64_t fv = INT64_MAX;
  *hp = 0.0;
  for (int64_t c0 = p; c0 <= Tn; c0 += NW) {
    const int64_t n = c0 + wv;
    int64_t v = INT64_MAX;
    double hn = 0.0;
    if (n <= Tn) {
      hn = wave_resid<T, S>(sm.P, dt, X, sm.x0, n, lane);
      if (!(hn < tol)) v = n;
    }
    if (lane == 0) sm.wres[wv] = hn;
    fv = block_min_i64<NT>(v, sm.redi);
    if (fv != INT64_MAX) {
      *hp = sm.wres[fv - c0];
      break;
    }
  }
  return fv;
}

// max_n ||h_n|| over steps n = first, first + stride, ... <= Tn (a wave per step).
template <typename T, class S>
__device__ __forceinline__ double dn_resid_max(DenseSmem<T, S>& sm, T dt, const T* X, int64_t Tn, int64_t first,
                               int64_t stride) {
  constexpr int NT = S::NT, NW = NT / PINT_WAVE;
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  double r = 0.0;
  for (int64_t n = first + wv * stride; n <= Tn; n += NW * stride)
    r = fmax(r, wave_resid<T, S>(sm.P, dt, X, sm.x0, n, lane));
  return block_max<NT>(r, sm.red);
}

// Elements of window steps m = m_first, m_first + m_stride, ... < len (in
// groups of SPP): AT[m] = J(x_{lo+m-1}) transposed, bb[m] = Phi - x_{lo+m}.
template <typename T, class S>
__device__ __forceinline__ void dn_elements(DenseSmem<T, S>& sm, T dt, const T* X, int64_t lo, int64_t len,
                            int64_t m_first, int64_t m_stride, T* AT, T* bb, double* hn = nullptr) {
  constexpr int D = S::D, NT = S::NT, NW = NT / PINT_WAVE;
  constexpr int SPP = ElemShape<S>::SPP, JT = ElemShape<S>::JT;
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  if constexpr (S::MATFREE) {
    // a wave per step: the RK4 step stores its stage record straight into
    // the element slot (the fold applies J from it), and b
    for (int64_t m = m_first + (int64_t)wv * m_stride; m < len; m += (int64_t)NW * m_stride) {
      const int64_t n = lo + m;
      T xp[S::R], xc[S::R], phi[S::R];
      wave_load<T, S>(X, sm.x0, n - 1, xp, lane);
      wave_load<T, S>(X, sm.x0, n, xc, lane);
      wave_rk4<T, S>(sm.P, dt, xp, phi, reinterpret_cast<typename S::Stage*>(AT + m * S::STAGE_SCALARS), lane);
      double hm = 0.0;
#pragma unroll
      for (int r = 0; r < S::R; r++) {
        const int i = lane + 64 * r;
        if (i < D) {
          bb[m * D + i] = phi[r] - xc[r];
          hm = acc_norm(hm, xc[r] - phi[r]);
        }
      }
      if (hn) {
        hm = wave_max(hm);
        if (lane == 0) hn[m] = hm;
      }
    }
    __syncthreads();
    return;
  }
  for (int64_t g0 = m_first; g0 < len; g0 += m_stride * SPP) {
    for (int sl = wv; sl < SPP; sl += NW) {
      const int64_t m = g0 + sl * m_stride;
      if (m < len) {
        const int64_t n = lo + m;
        T xp[S::R], xc[S::R], phi[S::R];
        wave_load<T, S>(X, sm.x0, n - 1, xp, lane);
        wave_load<T, S>(X, sm.x0, n, xc, lane);
        wave_rk4<T, S>(sm.P, dt, xp, phi, &sm.stage[sl], lane);
        double hm = 0.0;
#pragma unroll
        for (int r = 0; r < S::R; r++) {
          const int i = lane + 64 * r;
          if (i < D) {
            bb[m * D + i] = phi[r] - xc[r];
            hm = acc_norm(hm, xc[r] - phi[r]);
          }
        }
        if (hn) {  // ||h_n||_inf of the current iterate, as dn_search evaluates it
          hm = wave_max(hm);
          if (lane == 0) hn[m] = hm;
        }
      }
    }
    __syncthreads();
    for (int t = tid; t < SPP * JT; t += NT) {
      const int sl = t / JT, sub = t % JT;
      const int64_t m = g0 + sl * m_stride;
      if (m < len) {
        if constexpr (S::BANDED) {
          // column j = sub of J: rows j - BOFFT + r, stored diagonal-major
          // at band[(BW - 1 - r) * D + row] (diagonal k = j - row + BOFF)
          T col[S::BW];
          S::jac_band_column(&sm.stage[sl], sub, dt, col);
          T* band = AT + m * S::BW * D;
#pragma unroll
          for (int r = 0; r < S::BW; r++) {
            int row = sub - S::BOFFT + r;
            row = row < 0 ? row + D : (row >= D ? row - D : row);
            band[(S::BW - 1 - r) * D + row] = col[r];
          }
        } else {
          S::jac_thread(&sm.stage[sl], sm.P, sub, dt, AT + m * D * D, 1, D);
        }
      }
    }
    __syncthreads();
  }
}

// The window's Newton step, folded in order (eq. newton-step-recursion):
// dx_0 = b_0, dx_m = J dx_{m-1} + b_m.  Writes the updated states
// x_{lo+m} + dx_m to xnb and returns (block-uniform) the first window index
// whose updated state is non-finite or beyond the guard (len if none; the
// guard is not checked in plain mode).  The element rows, b and the old
// states a thread needs are prefetched PD elements ahead into registers (a
// ring with compile-time slots): they were written by other compute units.
template <typename T, class S>
__device__ __forceinline__ int64_t dn_fold(DenseSmem<T, S>& sm, const T* AT, const T* bb, const T* Xw,
                                           T* xnb, int64_t len, bool plain, double guard) {
  constexpr int D = S::D, NT = S::NT, QC = DenseShape<S>::QC, JC = DenseShape<S>::JC;
  constexpr bool RING = JC <= 16;
  constexpr int PD = RING ? (JC <= 10 ? 6 : 4) : 1;  // prefetch depth (elements)
  const int tid = threadIdx.x;
  const bool cth = tid < D * QC;
  const int ri = tid / QC, rq = tid % QC;
  int64_t bad_m = INT64_MAX;
  T ring[PD][RING ? JC : 1], rb[PD], rx[PD];
  if (cth)
#pragma unroll
    for (int u = 0; u < PD; u++) {
      const int64_t m = u;
      if (m < len) {
        if constexpr (RING) {
          if (m > 0)
#pragma unroll
            for (int jj = 0; jj < JC; jj++) ring[u][jj] = AT[m * D * D + (int64_t)(rq * JC + jj) * D + ri];
        }
        rb[u] = bb[m * D + ri];
        rx[u] = Xw[m * D + ri];
      }
    }
  int cur = 0;
  for (int64_t m0 = 0; m0 < len; m0 += PD) {
#pragma unroll
    for (int u = 0; u < PD; u++) {
      const int64_t m = m0 + u;
      if (m < len) {
        T part = T(0);
        if (cth && m > 0) {
          if constexpr (RING) {
#pragma unroll
            for (int jj = 0; jj < JC; jj++) part += ring[u][jj] * sm.z[cur][rq * JC + jj];
          } else {
            // every load of the step's slice in flight at once (one memory
            // latency per step), then the multiply-adds
            const T* Am = AT + m * D * D;
            T av[JC];
#pragma unroll
            for (int jj = 0; jj < JC; jj++) av[jj] = Am[(int64_t)(rq * JC + jj) * D + ri];
#pragma unroll
            for (int jj = 0; jj < JC; jj++) part += av[jj] * sm.z[cur][rq * JC + jj];
          }
        }
        T bm = T(0), xm = T(0);
        if (cth) {
          bm = rb[u];
          xm = rx[u];
          const int64_t mn = m + PD;
          if (mn < len) {
            if constexpr (RING)
#pragma unroll
              for (int jj = 0; jj < JC; jj++) ring[u][jj] = AT[mn * D * D + (int64_t)(rq * JC + jj) * D + ri];
            rb[u] = bb[mn * D + ri];
            rx[u] = Xw[mn * D + ri];
          }
        }
#pragma unroll
        for (int off = 1; off < QC; off <<= 1) part += __shfl_xor(part, off, PINT_WAVE);
        if (cth && rq == 0) {
          const T z = part + bm;
          const T xn = xm + z;
          sm.z[cur ^ 1][ri] = z;
          xnb[m * D + ri] = xn;
          if (!plain && bad_m == INT64_MAX && (!finite_(xn) || fabs((double)xn) > guard)) bad_m = m;
        }
        lds_barrier();
        cur ^= 1;
      }
    }
  }
  __syncthreads();
  const int64_t q = block_min_i64<NT>(bad_m, sm.redi);
  return q == INT64_MAX ? len : q;
}

// Banded systems: the window's Newton step from band-stored Jacobians.
// The folding workgroup stages the window through LDS in chunks of CH steps,
// double-buffered: while wave 0 runs the recursion over chunk c (lane i owns
// row i: BW multiply-adds, the previous step's dx exchanged by wave
// shuffles, no workgroup barrier per step), waves 1.. copy chunk c+1 from
// the workspace (written by other compute units) with all loads in flight.
template <class S>
struct BandShape {
  static constexpr int CH = 12;                     // steps per chunk
  static constexpr int NB = S::BW * S::D;            // band scalars per step
  static constexpr int PER = NB + 2 * S::D;          // per step: band, b, old x
};

// Matrix-free systems: per step the stage record, b and the old state.
template <class S>
struct MfShape {
  static constexpr int CH = 6;                       // steps per chunk
  static constexpr int SP = S::STAGE_SCALARS;        // stage record scalars
  static constexpr int PER = SP + 2 * S::D;
};

// Dynamic LDS of the folding workgroup: two chunks of staged steps.
template <typename T, class S>
constexpr size_t fold_lds_bytes() {
  if constexpr (S::BANDED)
    return 2 * (size_t)BandShape<S>::CH * BandShape<S>::PER * sizeof(T);
  else if constexpr (S::MATFREE)
    return 2 * (size_t)MfShape<S>::CH * MfShape<S>::PER * sizeof(T);
  else
    return 0;
}

// Scalars per stored window element: the band, the stage record, or J.
template <class S>
constexpr int64_t elem_scalars() {
  if constexpr (S::BANDED)
    return (int64_t)S::BW * S::D;
  else if constexpr (S::MATFREE)
    return S::STAGE_SCALARS;
  else
    return (int64_t)S::D * S::D;
}

// Copy n consecutive scalars from global src to LDS dst with threads
// t, t+nt, ...: 16-byte vectors when both ends are aligned, MAXV loads per
// thread issued before their LDS stores.
template <typename T, int MAXV>
__device__ __forceinline__ void lds_copy(T* dst, const T* __restrict__ src, int n, int t, int nt) {
  constexpr int V = 16 / sizeof(T);
  typedef T v_t __attribute__((ext_vector_type(V)));
  const bool vec = (reinterpret_cast<uintptr_t>(src) % 16 == 0) && (reinterpret_cast<uintptr_t>(dst) % 16 == 0);
  if (vec) {
    const int nv = n / V;
    for (int v0 = 0; v0 < nv; v0 += MAXV * nt) {
      v_t r[MAXV];
#pragma unroll
      for (int u = 0; u < MAXV; u++) {
        const int v = v0 + u * nt + t;
        if (v < nv) r[u] = reinterpret_cast<const v_t*>(src)[v];
      }
#pragma unroll
      for (int u = 0; u < MAXV; u++) {
        const int v = v0 + u * nt + t;
        if (v < nv) reinterpret_cast<v_t*>(dst)[v] = r[u];
      }
    }
    for (int q = nv * V + t; q < n; q += nt) dst[q] = src[q];
  } else {
    for (int q0 = 0; q0 < n; q0 += MAXV * nt) {
      T r[MAXV];
#pragma unroll
      for (int u = 0; u < MAXV; u++) {
        const int q = q0 + u * nt + t;
        if (q < n) r[u] = src[q];
      }
#pragma unroll
      for (int u = 0; u < MAXV; u++) {
        const int q = q0 + u * nt + t;
        if (q < n) dst[q] = r[u];
      }
    }
  }
}

// Three lds_copy's at once: every global load of the three arrays is issued
// before the first LDS store, so staging costs one memory latency, not
// three.  16-byte vectors when every pointer is aligned and every length is
// a whole number of vectors; otherwise the three copies one after another.
template <typename T, int MV1, int MV2>
__device__ __forceinline__ void lds_copy3(T* d1, const T* __restrict__ s1, int n1, T* d2,
                                          const T* __restrict__ s2, int n2, T* d3,
                                          const T* __restrict__ s3, int n3, int t, int nt) {
  constexpr int V = 16 / sizeof(T);
  typedef T v_t __attribute__((ext_vector_type(V)));
  auto al = [](const void* q) { return reinterpret_cast<uintptr_t>(q) % 16 == 0; };
  if (!(al(d1) && al(s1) && al(d2) && al(s2) && al(d3) && al(s3) && n1 % V == 0 && n2 % V == 0 &&
        n3 % V == 0)) {
    lds_copy<T, MV1>(d1, s1, n1, t, nt);
    lds_copy<T, MV2>(d2, s2, n2, t, nt);
    lds_copy<T, MV2>(d3, s3, n3, t, nt);
    return;
  }
  const int nv1 = n1 / V, nv2 = n2 / V, nv3 = n3 / V;
  for (int v1 = 0, v2 = 0; v1 < nv1 || v2 < nv2 || v2 < nv3; v1 += MV1 * nt, v2 += MV2 * nt) {
    v_t r1[MV1], r2[MV2], r3[MV2];
#pragma unroll
    for (int u = 0; u < MV1; u++) {
      const int v = v1 + u * nt + t;
      if (v < nv1) r1[u] = reinterpret_cast<const v_t*>(s1)[v];
    }
#pragma unroll
    for (int u = 0; u < MV2; u++) {
      const int v = v2 + u * nt + t;
      if (v < nv2) r2[u] = reinterpret_cast<const v_t*>(s2)[v];
      if (v < nv3) r3[u] = reinterpret_cast<const v_t*>(s3)[v];
    }
#pragma unroll
    for (int u = 0; u < MV1; u++) {
      const int v = v1 + u * nt + t;
      if (v < nv1) reinterpret_cast<v_t*>(d1)[v] = r1[u];
    }
#pragma unroll
    for (int u = 0; u < MV2; u++) {
      const int v = v2 + u * nt + t;
      if (v < nv2) reinterpret_cast<v_t*>(d2)[v] = r2[u];
      if (v < nv3) reinterpret_cast<v_t*>(d3)[v] = r3[u];
    }
  }
}

template <typename T, class S>
__device__ __forceinline__ int64_t dn_fold_band(DenseSmem<T, S>& sm, T* lbuf, const T* Bd, const T* bb,
                                                const T* Xw, T* xnb, int64_t len, bool plain, double guard) {
  constexpr int D = S::D, NT = S::NT, BW = S::BW, BOFF = S::BOFF;
  using BS = BandShape<S>;
  constexpr int CH = BS::CH, NB = BS::NB, PER = BS::PER;
  static_assert(D <= PINT_WAVE && NT > PINT_WAVE, "one wave owns the rows");
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  const int nl = NT - PINT_WAVE, lt = tid - PINT_WAVE;  // loader threads (waves 1..)
  // chunk in half h: [CH][NB] band, then [CH][D] b, then [CH][D] old x
  constexpr int V = 16 / sizeof(T), NL = NT - PINT_WAVE;
  constexpr int MVB = (CH * NB / V + NL - 1) / NL, MVX = (CH * D / V + NL - 1) / NL;
  auto load = [&](int64_t c0, int n, int h) {
    T* dst = lbuf + (size_t)h * CH * PER;
    lds_copy3<T, MVB, MVX>(dst, Bd + c0 * NB, n * NB, dst + CH * NB, bb + c0 * D, n * D,
                           dst + CH * NB + CH * D, Xw + c0 * D, n * D, lt, nl);
  };
  const int64_t nch = (len + CH - 1) / CH;
  if (wv > 0 && len > 0) load(0, (int)(len < CH ? len : CH), 0);
  lds_barrier();  // the chunks travel through LDS only
  // wave 0: lane i < D owns row i.  The previous step's dx goes through LDS
  // as zx[p] = dx[(p - BOFF) mod D], p < D + BW - 1, so row i reads the
  // consecutive zx[i .. i+BW-1] (one wave writes and reads: in order).
  static_assert(D + BW - 1 <= 2 * D, "zx fits in sm.z");
  int64_t bad = INT64_MAX;
  // Lorenz-96's shape (d = 40, 13 diagonals from offset -8): dx stays in
  // registers.  Lane l < 52 holds dx of row (l - 8) mod d; lanes 8..47 own
  // rows 0..39, lanes 0..7 and 48..51 are copies.  Row i's neighbours
  // dx_{i-8} .. dx_{i+4} are then lanes l-8 .. l+4 of the owner lane l, one
  // chain of whole-wave DPP shifts to each side; after a step the copies are
  // refreshed from their owners by one lane permutation.
  constexpr bool REG_FOLD = (D == 40 && BW == 13 && BOFF == 8);
  if constexpr (REG_FOLD) {
    constexpr int DPP_WAVE_SHR1 = 0x138;  // lane l <- lane l - 1
    constexpr int DPP_WAVE_SHL1 = 0x130;  // lane l <- lane l + 1
    const bool owner = lane >= 8 && lane < 8 + D;
    const int row = lane < 52 ? (lane + D - 8) % D : 0;
    const int src = lane < 8 ? lane + D : (lane >= 8 + D && lane < 52 ? lane - D : lane);
    T zr = T(0);
    for (int64_t c = 0; c < nch; c++) {
      const int64_t c0 = c * CH;
      const int n = (int)((len - c0) < CH ? (len - c0) : CH);
      if (wv > 0) {
        if (c + 1 < nch) {
          const int64_t c1 = c0 + CH;
          load(c1, (int)((len - c1) < CH ? (len - c1) : CH), (int)((c + 1) & 1));
        }
      } else if (bad == INT64_MAX) {
        const T* L = lbuf + (size_t)(c & 1) * CH * PER;
        for (int m = 0; m < n; m++) {
          const T* band = L + m * NB;
          T bv[BW];
#pragma unroll
          for (int k = 0; k < BW; k++) bv[k] = band[k * D + row];
          T z = L[CH * NB + m * D + row];
          if (c0 + m > 0) {
            T nb[BW];
            nb[BOFF] = zr;
            T t = zr;
#pragma unroll
            for (int q = 1; q <= BOFF; q++) {
              t = dpp_row<DPP_WAVE_SHR1, 0xf>(T(0), t);
              nb[BOFF - q] = t;
            }
            t = zr;
#pragma unroll
            for (int q = 1; q < BW - BOFF; q++) {
              t = dpp_row<DPP_WAVE_SHL1, 0xf>(T(0), t);
              nb[BOFF + q] = t;
            }
            z = band_row13<T>(z, bv, nb);
          }
          // copies take their owner's new value
          if constexpr (sizeof(T) == 8) {
            const int lo = __builtin_amdgcn_ds_bpermute(src * 4, __double2loint((double)z));
            const int hi = __builtin_amdgcn_ds_bpermute(src * 4, __double2hiint((double)z));
            zr = (T)__hiloint2double(hi, lo);
          } else {
            zr = __int_as_float(__builtin_amdgcn_ds_bpermute(src * 4, __float_as_int((float)z)));
          }
          const T xn = L[CH * NB + CH * D + m * D + row] + z;
          if (owner && !plain && (!finite_(xn) || fabs((double)xn) > guard)) bad = c0 + m;
          // the first cut step ends the fold; it and later steps stay unwritten
          if (!plain && __ballot(bad != INT64_MAX)) break;
          if (owner) xnb[(c0 + m) * D + row] = xn;
        }
        bad = wave_min_i64(owner ? bad : INT64_MAX);
      }
      lds_barrier();  // chunk c+1 staged, chunk c folded
    }
  } else {
    T* zx = &sm.z[0][0];
    const int i = lane < D ? lane : 0;
    for (int64_t c = 0; c < nch; c++) {
      const int64_t c0 = c * CH;
      const int n = (int)((len - c0) < CH ? (len - c0) : CH);
      if (wv > 0) {
        if (c + 1 < nch) {
          const int64_t c1 = c0 + CH;
          load(c1, (int)((len - c1) < CH ? (len - c1) : CH), (int)((c + 1) & 1));
        }
      } else if (bad == INT64_MAX) {
        const T* L = lbuf + (size_t)(c & 1) * CH * PER;
        for (int m = 0; m < n; m++) {
          const T* band = L + m * NB;
          T z = L[CH * NB + m * D + i];
          if (c0 + m > 0) {
            // issue all LDS reads of the step, then the multiply-adds
            T bv[BW], zv[BW];
  #pragma unroll
            for (int k = 0; k < BW; k++) {
              bv[k] = band[k * D + i];
              zv[k] = zx[i + k];
            }
            __builtin_amdgcn_sched_barrier(0);
            z = band_row13<T>(z, bv, zv);
          }
          if (lane < D) {
            zx[i + BOFF] = z;
            if (i >= D - BOFF) zx[i + BOFF - D] = z;
            if (i + BOFF + D < D + BW - 1) zx[i + BOFF + D] = z;
          }
          // other lanes read these next step; within one thread those addresses
          // need not alias, so keep the compiler from moving reads above them
          // (the hardware completes one wave's LDS operations in order)
          asm volatile("" ::: "memory");
          const T xn = L[CH * NB + CH * D + m * D + i] + z;
          if (lane < D && !plain && (!finite_(xn) || fabs((double)xn) > guard)) bad = c0 + m;
          // the first cut step ends the fold; it and later steps stay unwritten
          if (!plain && __ballot(bad != INT64_MAX)) break;
          if (lane < D) xnb[(c0 + m) * D + i] = xn;
        }
        bad = wave_min_i64(lane < D ? bad : INT64_MAX);
      }
      lds_barrier();  // chunk c+1 staged, chunk c folded
    }
  }
  if (tid == 0) sm.redi[0] = bad;
  __syncthreads();  // also: wave 0's updated states are visible to dn_commit
  const int64_t q = sm.redi[0];
  __syncthreads();
  return q == INT64_MAX ? len : q;
}

// Matrix-free systems (Kuramoto): the window's Newton step with J applied
// through the RK4 tangent from each step's stage record,
//   u_1 = v, K_s = J_f(y_s) u_s, u_{s+1} = v + c_s K_s,
//   J v = v + dt/6 (K_1 + 2 K_2 + 2 K_3 + K_4),
// J_f(y) u = K (c (c.u) + s (s.u)) - K (c C + s S) u — the same chain the
// dense Jacobian columns follow, applied to dx_{m-1} instead of to the unit
// vectors.  Wave 0 folds, two components per lane, the two dot products of
// a stage as one DPP wave sum; waves 1.. stage the next chunk of records
// through LDS meanwhile, as in the banded fold.
template <typename T, class S>
__device__ __forceinline__ int64_t dn_fold_mf(DenseSmem<T, S>& sm, T* lbuf, const T* St, const T* bb,
                                              const T* Xw, T* xnb, int64_t len, bool plain, double guard,
                                              T dt) {
  constexpr int D = S::D, NT = S::NT;
  using MS = MfShape<S>;
  constexpr int CH = MS::CH, SP = MS::SP, PER = MS::PER;
  constexpr int R = D / PINT_WAVE;  // components per lane of wave 0
  static_assert(D % PINT_WAVE == 0 && NT > PINT_WAVE, "whole lanes of wave 0");
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  const int nl = NT - PINT_WAVE, lt = tid - PINT_WAVE;
  constexpr int V = 16 / sizeof(T), NL = NT - PINT_WAVE;
  constexpr int MVS = (CH * SP / V + NL - 1) / NL, MVX = (CH * D / V + NL - 1) / NL;
  auto load = [&](int64_t c0, int n, int h) {
    T* dst = lbuf + (size_t)h * CH * PER;
    lds_copy3<T, MVS, MVX>(dst, St + c0 * SP, n * SP, dst + CH * SP, bb + c0 * D, n * D,
                           dst + CH * SP + CH * D, Xw + c0 * D, n * D, lt, nl);
  };
  const int64_t nch = (len + CH - 1) / CH;
  if (wv > 0 && len > 0) load(0, (int)(len < CH ? len : CH), 0);
  lds_barrier();
  int64_t bad = INT64_MAX;
  const T h2 = T(0.5) * dt, c6 = dt / T(6), Kc = sm.P[0];
  T v[R];  // dx_{m-1}, components lane + 64 r
#pragma unroll
  for (int r = 0; r < R; r++) v[r] = T(0);
  for (int64_t c = 0; c < nch; c++) {
    const int64_t c0 = c * CH;
    const int n = (int)((len - c0) < CH ? (len - c0) : CH);
    if (wv > 0) {
      if (c + 1 < nch) {
        const int64_t c1 = c0 + CH;
        load(c1, (int)((len - c1) < CH ? (len - c1) : CH), (int)((c + 1) & 1));
      }
    } else if (bad == INT64_MAX) {
      const T* L = lbuf + (size_t)(c & 1) * CH * PER;
      for (int m = 0; m < n; m++) {
        const T* rec = L + m * SP;  // c[4][D], s[4][D], C[4], S[4]
        T z[R];
#pragma unroll
        for (int r = 0; r < R; r++) z[r] = L[CH * SP + m * D + lane + PINT_WAVE * r];
        if (c0 + m > 0) {
          T u[R], acc[R];
#pragma unroll
          for (int r = 0; r < R; r++) u[r] = v[r];
#pragma unroll
          for (int s = 0; s < 4; s++) {
            T cs[R], sn[R];
            T pa = T(0), pb = T(0);
#pragma unroll
            for (int r = 0; r < R; r++) {
              cs[r] = rec[s * D + lane + PINT_WAVE * r];
              sn[r] = rec[4 * D + s * D + lane + PINT_WAVE * r];
              pa += cs[r] * u[r];
              pb += sn[r] * u[r];
            }
            const T C = rec[8 * D + s], Sg = rec[8 * D + 4 + s];
            wave_sum2_dpp(pa, pb);
            const T w = (s == 0 || s == 3) ? T(1) : T(2);
            const T cc = (s == 2) ? dt : h2;
#pragma unroll
            for (int r = 0; r < R; r++) {
              const T K = Kc * (cs[r] * pa + sn[r] * pb) - Kc * (cs[r] * C + sn[r] * Sg) * u[r];
              acc[r] = (s == 0) ? K : acc[r] + w * K;
              u[r] = v[r] + cc * K;
            }
          }
#pragma unroll
          for (int r = 0; r < R; r++) z[r] = (v[r] + c6 * acc[r]) + z[r];
        }
        bool badm = false;
        T xn[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
          v[r] = z[r];
          xn[r] = L[CH * SP + CH * D + m * D + lane + PINT_WAVE * r] + z[r];
          badm = badm || !finite_(xn[r]) || fabs((double)xn[r]) > guard;
        }
        if (!plain && badm) bad = c0 + m;
        // the first cut step ends the fold; it and later steps stay unwritten
        if (!plain && __ballot(bad != INT64_MAX)) break;
#pragma unroll
        for (int r = 0; r < R; r++) xnb[(c0 + m) * D + lane + PINT_WAVE * r] = xn[r];
      }
      bad = wave_min_i64(bad);
    }
    lds_barrier();  // chunk c+1 staged, chunk c folded
  }
  if (tid == 0) sm.redi[0] = bad;
  __syncthreads();  // also: wave 0's updated states are visible to the commit
  const int64_t q = sm.redi[0];
  __syncthreads();
  return q == INT64_MAX ? len : q;
}

// Write the accepted part [0, q) of the updated window states.
template <typename T, class S>
__device__ __forceinline__ void dn_commit(T* Xw, const T* xnb, int64_t q) {
  for (int64_t idx = threadIdx.x; idx < q * S::D; idx += S::NT) Xw[idx] = xnb[idx];
  __syncthreads();
}

template <typename T, class S>
__device__ __forceinline__ void dn_load_inst(DenseSmem<T, S>& sm, const DenseKArgs& a, int64_t inst) {
  const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
  for (int i = threadIdx.x; i < S::NP; i += S::NT) sm.P[i] = Pg[i];
  const T* xg = static_cast<const T*>(a.x0) + inst * S::D;
  for (int i = threadIdx.x; i < S::D; i += S::NT) sm.x0[i] = xg[i];
  __syncthreads();
}

// One workgroup per instance (device work queue), whole Newton loop.
template <typename T, class S>
__global__ __launch_bounds__(S::NT) void k_newton_dense(DenseKArgs a) {
  constexpr int D = S::D, NT = S::NT;
  __shared__ DenseSmem<T, S> sm;
  __shared__ uint32_t s_slot;
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  T* band_buf = reinterpret_cast<T*>(dyn_lds);  // fold_lds_bytes<T, S>() bytes
  const int tid = threadIdx.x;
  const T dt = (T)a.dt;
  T* slot = static_cast<T*>(a.ws_elems) + (int64_t)blockIdx.x * a.slot_stride;
  T* AT = slot;
  T* bb = AT + a.Wt * D * D;
  T* dxb = bb + a.Wt * D;

  for (;;) {
    if (tid == 0) s_slot = atomicAdd(a.queue, 1u);
    __syncthreads();
    const int64_t inst = s_slot;
    __syncthreads();
    if (inst >= a.B) break;
    const int64_t Tn = a.T_uniform;
    T* X = static_cast<T*>(a.traj) + inst * Tn * D;
    dn_load_inst<T, S>(sm, a, inst);
    if (a.guess == 0)
      for (int64_t idx = tid; idx < Tn * D; idx += NT) X[idx] = sm.x0[idx % D];
    __syncthreads();

    const bool plain = (a.window <= 0);
    const int64_t W = a.window;
    int64_t k = 0, p = 1;
    int st = ST_OK;
    while (Tn > 0) {
      int64_t lo, hi;
      if (plain) {
        const double r = dn_resid_max<T, S>(sm, dt, X, Tn, 1, 1);
        if (!(r < INFINITY)) { st = ST_NONFINITE; break; }
        if (r < a.tol) { st = ST_OK; break; }
        if (k >= a.max_iter) { st = ST_NOT_CONVERGED; break; }
        lo = 1;
        hi = Tn;
      } else {
        double hp;
        const int64_t fv = dn_search<T, S>(sm, dt, X, Tn, p, a.tol, &hp);
        if (fv == INT64_MAX) { st = ST_OK; break; }
        p = fv;
        if (!(hp < INFINITY)) { st = ST_NONFINITE; break; }
        if (k >= a.max_iter) { st = ST_NOT_CONVERGED; break; }
        lo = p;
        hi = (W >= Tn - p + 1) ? Tn : p + W - 1;
      }
      const int64_t len = hi - lo + 1;
      dn_elements<T, S>(sm, dt, X, lo, len, 0, 1, AT, bb);
      int64_t q;
      if constexpr (S::BANDED)
        // the accepted states go straight into the trajectory
        q = dn_fold_band<T, S>(sm, band_buf, AT, bb, X + (lo - 1) * D, X + (lo - 1) * D, len, plain, a.guard);
      else if constexpr (S::MATFREE)
        q = dn_fold_mf<T, S>(sm, band_buf, AT, bb, X + (lo - 1) * D, dxb, len, plain, a.guard, dt);
      else
        q = dn_fold<T, S>(sm, AT, bb, X + (lo - 1) * D, dxb, len, plain, a.guard);
      if constexpr (!S::BANDED) dn_commit<T, S>(X + (lo - 1) * D, dxb, q);
      if (q == 0) { st = ST_NONFINITE; break; }
      k++;
    }
    __syncthreads();
    const double r = dn_resid_max<T, S>(sm, dt, X, Tn, 1, 1);
    if (tid == 0) {
      a.iters[inst] = k;
      a.resid[inst] = r;
      a.status[inst] = st;
    }
    __syncthreads();
  }
}

// ---------------------------------------------- cooperative variant -----

// Per-instance control block of the cooperative solver (64 bytes).
struct CoopCtl {
  uint32_t bar_count, bar_gen;
  int64_t lo, hi;     // window decided by workgroup 0
  int32_t done, st;
  int64_t k;
  unsigned long long rmax;  // final residual (bits of a non-negative double)
  uint32_t err, go;         // go: the last round whose update workgroup 0 released
  uint32_t arrive, pad0;    // arrive: element passes completed, all workgroups
};
static_assert(sizeof(CoopCtl) == 64, "control block size");

// Barrier among the G workgroups of one instance.  Release fence before
// arriving, acquire fence after leaving.  The wait is bounded
// (bounded_wait); returns, in every thread, true if the instance's error
// word was seen (a wait of this or another workgroup gave up): the caller
// then leaves its round loop.
__device__ __forceinline__ bool coop_barrier(CoopCtl* c, int G, uint32_t& gen, uint64_t limit) {
  __shared__ int s_fail;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t target = gen + 1;
    const uint32_t prev = atomicAdd(&c->bar_count, 1u);
    bool fail = false;
    if (prev == (uint32_t)(G - 1)) {
      __hip_atomic_store(&c->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      __hip_atomic_store(&c->bar_gen, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      fail = bounded_wait(&c->err, limit, [&] {
        return __hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == target;
      });
    }
    __threadfence();
    gen = target;
    s_fail = fail;
  }
  __syncthreads();
  return s_fail != 0;
}

// One-way signals of a round (thread 0 of a workgroup).  Every workgroup
// releases its elements by incrementing `arrive`; only workgroup 0 waits for
// all of them.  Workgroup 0 releases the committed update by storing the
// round in `go`; only the others wait for it.  The wait returns true when
// the error word was seen (see bounded_wait).
__device__ __forceinline__ void coop_arrive(CoopCtl* c) {
  __threadfence();
  atomicAdd(&c->arrive, 1u);
}
__device__ __forceinline__ bool coop_wait_at_least(CoopCtl* c, const uint32_t* word, uint32_t target,
                                                   uint64_t limit) {
  const bool fail = bounded_wait(&c->err, limit, [&] {
    return __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
  });
  __threadfence();
  return fail;
}
__device__ __forceinline__ void coop_release_go(CoopCtl* c, uint32_t round) {
  __threadfence();
  __hip_atomic_store(&c->go, round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// G workgroups per instance (windowed mode): all of them build the
// window's elements (speculatively, W + SPEC_SLACK steps from the previous
// window start, with their residual norms); workgroup 0 picks the window,
// folds the recursion and applies the guarded update.  Two barriers per
// update.  Needs all workgroups resident at once (cooperative launch).
template <typename T, class S>
__global__ __launch_bounds__(S::NT) void k_newton_dense_coop(DenseKArgs a, int G, CoopCtl* ctl) {
  constexpr int D = S::D, NT = S::NT;
  __shared__ DenseSmem<T, S> sm;
  __shared__ int64_t s_win[2];
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  T* band_buf = reinterpret_cast<T*>(dyn_lds);  // fold_lds_bytes<T, S>() bytes
  __shared__ int32_t s_done;
  const int tid = threadIdx.x;
  const int64_t inst = blockIdx.x / G;
  const int g = blockIdx.x % G;
  const T dt = (T)a.dt;
  CoopCtl* c = ctl + inst;
  T* slot = static_cast<T*>(a.ws_elems) + inst * a.slot_stride;
  T* AT = slot;
  T* bb = AT + a.Wt * D * D;
  T* dxb = bb + a.Wt * D;
  const int64_t Tn = a.T_uniform;
  T* X = static_cast<T*>(a.traj) + inst * Tn * D;
  const int64_t W = a.window;
  uint32_t gen = 0;

  dn_load_inst<T, S>(sm, a, inst);
  if (a.guess == 0)
    for (int64_t idx = (int64_t)g * NT + tid; idx < Tn * D; idx += (int64_t)G * NT) X[idx] = sm.x0[idx % D];

  // workgroup 0 owns the iteration state.  One round: (1) all workgroups
  // build elements of the current iterate from step `base`; (2) workgroup 0
  // takes the window [p, min(T, p+W-1)] with p the first violation at or
  // after base, folds it and commits the cut update.
  //   Banded (cheap) Jacobians: the round builds W + slack steps from base =
  // the previous window start, with their residual norms, and p is read off
  // them (searching further only if there is none); if the window reaches
  // past the built steps nothing is updated and the next round builds from
  // p.  Dense Jacobians: workgroup 0 searches p after each update and the
  // round builds exactly the window.  Both are the iteration that searches
  // from the previous window start after each update.
  constexpr bool SPEC = S::BANDED;
  const int64_t Wcap = a.Wt;
  double* hn = reinterpret_cast<double*>(slot + slot_hn_offset<S>(Wcap));
  int64_t k = 0;
  int st = ST_OK;
  // search from p0 (dense Jacobians): publish the window, or finish
  auto decide = [&](int64_t p0) {
    double hp = 0.0;
    const int64_t p = Tn > 0 ? dn_search<T, S>(sm, dt, X, Tn, p0, a.tol, &hp) : INT64_MAX;
    int done = 0;
    int64_t hi = 0;
    if (p == INT64_MAX) {
      st = ST_OK;
      done = 1;
    } else if (!(hp < INFINITY)) {
      st = ST_NONFINITE;
      done = 1;
    } else if (k >= a.max_iter) {
      st = ST_NOT_CONVERGED;
      done = 1;
    } else {
      hi = (W >= Tn - p + 1) ? Tn : p + W - 1;
    }
    if (tid == 0) {
      c->lo = done ? 0 : p;
      c->hi = hi;
      c->done = done;
    }
  };
  const uint64_t lim = a.wait_limit;
  __shared__ int s_fail;
  // a wait that gave up (error word) ends the solve in every workgroup
  bool fail = coop_barrier(c, G, gen, lim);  // initial iterate written everywhere
  if (!fail && g == 0) {
    if constexpr (SPEC) {
      if (tid == 0) {
        c->lo = 1;
        c->done = Tn > 0 ? 0 : 1;
      }
    } else {
      decide(1);
    }
  }
  if (!fail) fail = coop_barrier(c, G, gen, lim);
  for (uint32_t rnd = 1; !fail; rnd++) {
    if (tid == 0) {
      s_win[0] = c->lo;
      s_win[1] = c->hi;
      s_done = c->done;
      // the error word, loaded with the window: a workgroup that gave up
      // may have left the window unset
      s_fail = __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
      const int64_t lo = s_win[0], hi = SPEC ? lo : s_win[1];
      if (!s_done && !s_fail && !(lo >= 1 && lo <= Tn && hi >= lo && hi <= Tn)) {
        atomicOr(&c->err, 1u);  // never for a consistent control block
        s_fail = 1;
      }
    }
    __syncthreads();
    if (s_done || s_fail) break;
    const int64_t base = s_win[0];
    const int64_t slen = SPEC ? ((Tn - base + 1) < Wcap ? (Tn - base + 1) : Wcap) : s_win[1] - base + 1;
    dn_elements<T, S>(sm, dt, X, base, slen, g, G, AT, bb, SPEC ? hn : nullptr);
    __syncthreads();  // this workgroup's element stores are issued
    if (tid == 0) coop_arrive(c);
    if (g == 0) {
      if (tid == 0) s_fail = coop_wait_at_least(c, &c->arrive, (uint32_t)G * rnd, lim);
      __syncthreads();
      if (s_fail) {
        // some elements may be missing: no update; release the others, who
        // find the solve done
        if (tid == 0) {
          c->done = 1;
          coop_release_go(c, rnd);
        }
        break;
      }
      int64_t p = base, next = 0;
      int done = 0;
      bool fold = true;
      if constexpr (SPEC) {
        // first violation among the built steps
        int64_t fv = INT64_MAX;
        for (int64_t m0 = 0; m0 < slen && fv == INT64_MAX; m0 += NT) {
          const int64_t m = m0 + tid;
          const int64_t v = (m < slen && !(hn[m] < a.tol)) ? m : INT64_MAX;
          fv = block_min_i64<NT>(v, sm.redi);
        }
        double hp = 0.0;
        bool have = true;  // the window's elements are in the slot at offset p - base
        p = INT64_MAX;
        if (fv != INT64_MAX) {
          p = base + fv;
          hp = hn[fv];
        } else if (base + slen - 1 < Tn) {
          p = dn_search<T, S>(sm, dt, X, Tn, base + slen, a.tol, &hp);
          have = false;
        }
        if (p == INT64_MAX) {
          st = ST_OK;
          done = 1;
        } else if (!(hp < INFINITY)) {
          st = ST_NONFINITE;
          done = 1;
        } else if (k >= a.max_iter) {
          st = ST_NOT_CONVERGED;
          done = 1;
        } else {
          const int64_t len = ((W >= Tn - p + 1) ? Tn : p + W - 1) - p + 1;
          fold = have && (p - base) + len <= slen;  // else rebuild from p
          next = p;
        }
        if (done) fold = false;
      }
      if (fold) {
        const int64_t len = ((W >= Tn - p + 1) ? Tn : p + W - 1) - p + 1;
        const int64_t off = p - base;
        constexpr int64_t ES = elem_scalars<S>();  // scalars per element
        int64_t q;
        if constexpr (S::BANDED)
          // the accepted states go straight into the trajectory
          q = dn_fold_band<T, S>(sm, band_buf, AT + off * ES, bb + off * D, X + (p - 1) * D, X + (p - 1) * D,
                                 len, false, a.guard);
        else if constexpr (S::MATFREE)
          q = dn_fold_mf<T, S>(sm, band_buf, AT + off * ES, bb + off * D, X + (p - 1) * D, dxb, len, false,
                               a.guard, dt);
        else
          q = dn_fold<T, S>(sm, AT + off * ES, bb + off * D, X + (p - 1) * D, dxb, len, false, a.guard);
        if constexpr (!S::BANDED) dn_commit<T, S>(X + (p - 1) * D, dxb, q);
        if (q == 0) {
          st = ST_NONFINITE;
          done = 1;
        } else {
          k++;
        }
      }
      if constexpr (SPEC) {
        if (tid == 0) {
          c->lo = next;
          c->done = done;
        }
      } else {
        if (done) {
          if (tid == 0) c->done = 1;
        } else {
          decide(p);
        }
      }
      __syncthreads();  // the committed update and the next window are written
      if (tid == 0) coop_release_go(c, rnd);
    } else {
      if (tid == 0) s_fail = coop_wait_at_least(c, &c->go, rnd, lim);
      __syncthreads();
      if (s_fail) break;
    }
  }
  // final residual: steps split over the G workgroups
  const double r = dn_resid_max<T, S>(sm, dt, X, Tn, 1 + g, G);
  if (tid == 0) atomic_max_nonneg(reinterpret_cast<double*>(&c->rmax), r);
  (void)coop_barrier(c, G, gen, lim);
  if (g == 0 && tid == 0) {
    a.iters[inst] = k;
    a.resid[inst] = __longlong_as_double((long long)__hip_atomic_load(&c->rmax, __ATOMIC_RELAXED,
                                                                      __HIP_MEMORY_SCOPE_AGENT));
    // a wait that gave up (error word) makes the result unreliable
    a.status[inst] = __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                         ? ST_DEVICE : st;
  }
}

// Sequential comparator: one wave per instance.
template <typename T, class S>
__global__ __launch_bounds__(64) void k_seq_dense(DenseKArgs a, const int64_t* T_off) {
  constexpr int D = S::D, NP = S::NP, R = S::R;
  __shared__ T s_P[NP];
  const int64_t inst = blockIdx.x;
  const int lane = threadIdx.x;
  const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
  for (int i = lane; i < NP; i += 64) s_P[i] = Pg[i];
  __syncthreads();
  const int64_t t0 = T_off ? T_off[inst] : inst * a.T_uniform;
  const int64_t Tn = (T_off ? T_off[inst + 1] : t0 + a.T_uniform) - t0;
  T* X = static_cast<T*>(a.traj) + t0 * D;
  const T* xg = static_cast<const T*>(a.x0) + inst * D;
  T x[R], y[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int i = lane + 64 * r;
    x[r] = i < D ? xg[i] : T(0);
  }
  const T dt = (T)a.dt;
  if constexpr (S::BANDED && D == 40) {
    // Lorenz-96: lane l holds component (l - 16) mod 40; lanes 16..55 own the
    // components, lanes 0..15 and 56..63 hold copies.  f reads offsets
    // -2..+1, so each stage's values are valid two lanes less on the left
    // and one less on the right: two RK4 steps (eight stages) use up the
    // copies exactly and leave the owners' states right, and one lane
    // permutation per two steps refreshes the copies.  Neighbours come by
    // whole-wave DPP shifts instead of a shuffle per neighbour; the
    // arithmetic is that of DSysL96::f and wave_rk4 (the same states bit for
    // bit).
    constexpr int DPP_WAVE_SHR1 = 0x138;  // lane l <- lane l - 1
    constexpr int DPP_WAVE_SHL1 = 0x130;  // lane l <- lane l + 1
    constexpr int HL = 16;                // copies on the left
    const bool owner = lane >= HL && lane < HL + D;
    const int comp = (lane + D - HL) % D;
    const int src = lane < HL ? lane + D : (lane >= HL + D ? lane - D : lane);
    const T F = s_P[0], h2 = T(0.5) * dt, c6 = dt / T(6);
    T xr = xg[comp];
    auto f = [&](T yv) -> T {
      const T xp1 = dpp_row<DPP_WAVE_SHL1, 0xf>(T(0), yv);
      const T xm1 = dpp_row<DPP_WAVE_SHR1, 0xf>(T(0), yv);
      const T xm2 = dpp_row<DPP_WAVE_SHR1, 0xf>(T(0), xm1);
      return (xp1 - xm2) * xm1 - yv + F;
    };
    auto rk4 = [&](T xv) -> T {
      T k = f(xv);
      T acc = k, yv = xv + h2 * k;
      k = f(yv);
      acc += T(2) * k;
      yv = xv + h2 * k;
      k = f(yv);
      acc += T(2) * k;
      yv = xv + dt * k;
      k = f(yv);
      return xv + c6 * (acc + k);
    };
    for (int64_t n = 0; n < Tn; n += 2) {
      const T x1 = rk4(xr);
      if (owner) X[n * D + comp] = x1;
      if (n + 1 >= Tn) break;
      const T x2 = rk4(x1);
      if (owner) X[(n + 1) * D + comp] = x2;
      // the copies take their owners' values
      if constexpr (sizeof(T) == 8) {
        const int lo = __builtin_amdgcn_ds_bpermute(src * 4, __double2loint((double)x2));
        const int hi = __builtin_amdgcn_ds_bpermute(src * 4, __double2hiint((double)x2));
        xr = (T)__hiloint2double(hi, lo);
      } else {
        xr = __int_as_float(__builtin_amdgcn_ds_bpermute(src * 4, __float_as_int((float)x2)));
      }
    }
    return;
  }
  for (int64_t n = 0; n < Tn; n++) {
    wave_rk4<T, S, true>(s_P, dt, x, y, nullptr, lane);
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int i = lane + 64 * r;
      x[r] = y[r];
      if (i < D) X[n * D + i] = y[r];
    }
  }
}

// Sequential comparator for Kuramoto with d = 64 R (R > 1): the R waves of
// one workgroup share an instance, one component per lane, so each wave
// evaluates one sincos per stage point instead of R in a row; the stage
// sums of sin and cos meet through LDS (wave sums by DPP row permutes, then
// the R partial sums in wave order).  One barrier per stage (two buffers).
template <typename T, class S>
__global__ __launch_bounds__(64 * S::R) void k_seq_kur_split(DenseKArgs a, const int64_t* T_off) {
  constexpr int D = S::D, NP = S::NP, NW = S::R;
  static_assert(S::MATFREE && D == 64 * NW && NW > 1, "one component per lane");
  __shared__ T s_P[NP];
  __shared__ T s_red[2][NW][2];
  const int64_t inst = blockIdx.x;
  const int tid = threadIdx.x, lane = tid % PINT_WAVE, wv = tid / PINT_WAVE;
  const T* Pg = static_cast<const T*>(a.params) + inst * a.pstride;
  for (int i = tid; i < NP; i += 64 * NW) s_P[i] = Pg[i];
  __syncthreads();
  const int64_t t0 = T_off ? T_off[inst] : inst * a.T_uniform;
  const int64_t Tn = (T_off ? T_off[inst + 1] : t0 + a.T_uniform) - t0;
  T* X = static_cast<T*>(a.traj) + t0 * D;
  const T* xg = static_cast<const T*>(a.x0) + inst * D;
  const T dt = (T)a.dt, h2 = T(0.5) * dt, c6 = dt / T(6);
  const T Kc = s_P[0], om = s_P[1 + tid];
  int buf = 0;
  auto f = [&](T y) -> T {
    T sn, cs;
    if constexpr (sizeof(T) == 8)
      sincos(y, &sn, &cs);
    else
      sincosf(y, &sn, &cs);
    T ls = sn, lc = cs;
    wave_sum2_dpp(ls, lc);
    if (lane == 0) {
      s_red[buf][wv][0] = ls;
      s_red[buf][wv][1] = lc;
    }
    __syncthreads();
    T Ssum = s_red[buf][0][0], Csum = s_red[buf][0][1];
#pragma unroll
    for (int w = 1; w < NW; w++) {
      Ssum += s_red[buf][w][0];
      Csum += s_red[buf][w][1];
    }
    buf ^= 1;
    return om + Kc * (cs * Ssum - sn * Csum);
  };
  T x = xg[tid];
  for (int64_t n = 0; n < Tn; n++) {
    T k = f(x);
    T acc = k, y = x + h2 * k;
    k = f(y);
    acc += T(2) * k;
    y = x + h2 * k;
    k = f(y);
    acc += T(2) * k;
    y = x + dt * k;
    k = f(y);
    x = x + c6 * (acc + k);
    X[n * D + tid] = x;
  }
}

// Residual of every step of a uniform batch: one wave per step.
template <typename T, class S>
__global__ __launch_bounds__(256) void k_residual_dense(DenseKArgs a, T* h, double* hmax) {
  constexpr int D = S::D, NP = S::NP, R = S::R;
  const int lane = threadIdx.x % 64;
  const int64_t g = blockIdx.x * 4 + threadIdx.x / 64;
  if (g >= a.B * a.T_uniform) return;
  const int64_t inst = g / a.T_uniform, n = g % a.T_uniform + 1;
  const T* P = static_cast<const T*>(a.params) + inst * a.pstride;
  const T* X = static_cast<const T*>(a.traj) + inst * a.T_uniform * D;
  const T* x0 = static_cast<const T*>(a.x0) + inst * D;
  T xp[R], phi[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int i = lane + 64 * r;
    xp[r] = i < D ? (n == 1 ? x0[i] : X[(n - 2) * D + i]) : T(0);
  }
  (void)NP;
  wave_rk4<T, S>(P, (T)a.dt, xp, phi, nullptr, lane);
  double m = 0.0;
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int i = lane + 64 * r;
    if (i < D) {
      const T v = X[(n - 1) * D + i] - phi[r];
      if (h) h[(inst * a.T_uniform + n - 1) * D + i] = v;
      m = acc_norm(m, v);
    }
  }
  m = wave_max(m);
  if (lane == 0) atomic_max_nonneg(hmax + inst, m);
}

// Elements A_n = dPhi/dx(x_n) (row-major), b_n = Phi(x_n) - x_{n+1}.
template <typename T, class S>
__global__ __launch_bounds__(S::NT) void k_elements_dense(DenseKArgs a, T* A, T* b) {
  constexpr int D = S::D, NP = S::NP, NT = S::NT, NW = NT / PINT_WAVE, SPP = S::SPP, JT = S::JT;
  __shared__ typename S::Stage s_stage[SPP];
  __shared__ T s_P[SPP][NP];
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int64_t total = a.B * a.T_uniform;
  const int64_t g0 = (int64_t)blockIdx.x * SPP;
  for (int sl = 0; sl < SPP; sl++) {
    const int64_t g = g0 + sl;
    if (g < total) {
      const T* P = static_cast<const T*>(a.params) + (g / a.T_uniform) * a.pstride;
      for (int i = tid; i < NP; i += NT) s_P[sl][i] = P[i];
    }
  }
  __syncthreads();
  for (int sl = wv; sl < SPP; sl += NW) {
    const int64_t g = g0 + sl;
    if (g >= total) continue;
    const int64_t inst = g / a.T_uniform, n = g % a.T_uniform;
    const T* X = static_cast<const T*>(a.traj) + inst * a.T_uniform * D;
    const T* x0 = static_cast<const T*>(a.x0) + inst * D;
    T xp[S::R], phi[S::R];
#pragma unroll
    for (int r = 0; r < S::R; r++) {
      const int i = lane + 64 * r;
      xp[r] = i < D ? (n == 0 ? x0[i] : X[(n - 1) * D + i]) : T(0);
    }
    wave_rk4<T, S>(s_P[sl], (T)a.dt, xp, phi, &s_stage[sl], lane);
#pragma unroll
    for (int r = 0; r < S::R; r++) {
      const int i = lane + 64 * r;
      if (i < D) b[g * D + i] = phi[r] - X[n * D + i];
    }
  }
  __syncthreads();
  for (int t = tid; t < SPP * JT; t += NT) {
    const int sl = t / JT, sub = t % JT;
    const int64_t g = g0 + sl;
    if (g < total) S::jac_thread(&s_stage[sl], s_P[sl], sub, (T)a.dt, A + g * D * D, D, 1);
  }
}

// ------------------------------------------------------------- dispatch --

template <typename T, typename F>
static int dispatch_dense_sys(int system, int d, F&& f) {
  if (system == 5 && d == 40) return f(DSysL96<T, 40>{});
  if (system == 6 && d == 128) return f(DSysKur<T, 128>{});
  if (system == 6 && d == 64) return f(DSysKur<T, 64>{});
  return ST_UNSUPPORTED;
}

template <typename F>
static int dispatch_dense(int dtype, int system, int d, F&& f) {
  if (dtype == 0) return dispatch_dense_sys<double>(system, d, [&](auto s) { return f((double)0, s); });
  if (dtype == 1) return dispatch_dense_sys<float>(system, d, [&](auto s) { return f((float)0, s); });
  return ST_UNSUPPORTED;
}

bool dense_supported(int system, int d) {
  return dispatch_dense(0, system, d, [](auto, auto) { return ST_OK; }) == ST_OK;
}

static DenseKArgs to_dk(const SolveArgs& a) {
  DenseKArgs k{};
  k.B = a.B;
  k.x0 = a.x0;
  k.params = a.params;
  k.pstride = a.pstride;
  k.T_uniform = a.T_uniform;
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
  k.wait_limit = wait_limit();
  return k;
}

static int num_cus() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus;
}

// Workgroups for the one-workgroup-per-instance solver: at most one per CU.
static int dense_grid(int64_t B) {
  const int64_t cu = num_cus();
  return (int)(B < cu ? B : cu);
}

// Elements per workgroup slot: T in plain mode, else the window (plus the
// speculative slack of the cooperative solver for banded Jacobians), at most T.
template <class S>
static int64_t dense_Wt(const SolveArgs& a) {
  const int64_t T = a.T_uniform;
  if (a.window <= 0 || a.window >= T) return T;
  const int64_t w = a.window + (S::BANDED ? spec_slack(a.window) : 0);
  return w < T ? w : T;
}

// Workgroups per instance for the cooperative solver (windowed mode only):
// enough for one Jacobian pass per workgroup over the window, all of them
// resident at once; 1 means "use the one-workgroup solver".
template <typename T, class S>
static int coop_groups(const SolveArgs& a) {
  if (a.window <= 0 || a.B <= 0 || a.T_uniform <= 0) return 1;
  const int64_t W = dense_Wt<S>(a);
  int64_t G = (W + S::SPP - 1) / S::SPP;
  if (G > 64) G = 64;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_newton_dense_coop<T, S>, S::NT,
                                                   fold_lds_bytes<T, S>()) != hipSuccess)
    return 1;
  const int64_t cap = (int64_t)per_cu * num_cus();
  while (G > 1 && a.B * G > cap) G--;
  return G >= 2 ? (int)G : 1;
}

struct DenseWs {
  size_t ctl_off, slots_off, per_slot, total;
  int64_t nslots;
};

template <typename T, class S>
static DenseWs dense_ws_layout(const SolveArgs& a) {
  DenseWs l{};
  const int64_t Wt = dense_Wt<S>(a) > 0 ? dense_Wt<S>(a) : 1;
  const int64_t B = a.B > 0 ? a.B : 1;
  l.per_slot = align_up((size_t)slot_scalars<S>(Wt) * sizeof(T));
  l.nslots = B > dense_grid(B) ? B : dense_grid(B);
  l.ctl_off = 256;
  l.slots_off = l.ctl_off + align_up((size_t)B * sizeof(CoopCtl));
  l.total = l.slots_off + l.per_slot * (size_t)l.nslots;
  return l;
}

size_t dense_ws_bytes(const SolveArgs& a) {
  size_t total = 0;
  dispatch_dense(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    total = dense_ws_layout<T, S>(a).total;
    return ST_OK;
  });
  const size_t pipe = pipe_ws_bytes(a);
  return total > pipe ? total : pipe;
}

int dense_solve(const SolveArgs& a) {
  if (!a.ws || a.ws_bytes < dense_ws_bytes(a)) return ST_WORKSPACE;
  if (dense_pipeline()) {  // Lorenz-96, windowed: the pipelined solver when it fits
    bool used = false;
    if (int rc = pipe_solve(a, &used)) return rc;
    if (used) return ST_OK;
  }
  return dispatch_dense(a.dtype, a.system, a.d, [&](auto t, auto s) -> int {
    using T = decltype(t);
    using S = decltype(s);
    const DenseWs l = dense_ws_layout<T, S>(a);
    char* w = static_cast<char*>(a.ws);
    DenseKArgs k = to_dk(a);
    k.queue = reinterpret_cast<uint32_t*>(w);
    k.ws_elems = w + l.slots_off;
    k.Wt = dense_Wt<S>(a);
    k.slot_stride = (int64_t)(l.per_slot / sizeof(T));
    CoopCtl* ctl = reinterpret_cast<CoopCtl*>(w + l.ctl_off);
    // queue counter and control blocks start at zero (a kernel, not a memset)
    if (int rc = fill_u32(reinterpret_cast<uint32_t*>(w), l.slots_off / 4, 0u, a.stream)) return rc;
    const size_t lds = fold_lds_bytes<T, S>();
    static bool attr_set = false;  // per (T, S) instantiation
    if (!attr_set && lds > 0) {
      if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_newton_dense_coop<T, S>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
          hipFuncSetAttribute(reinterpret_cast<const void*>(&k_newton_dense<T, S>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return ST_DEVICE;
      attr_set = true;
    }
    const int G = coop_groups<T, S>(a);
    if (G >= 2) {
      int Gv = G;
      void* args[] = {&k, &Gv, &ctl};
      const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_newton_dense_coop<T, S>),
                                                      dim3((unsigned)(a.B * G)), dim3(S::NT), args, lds, a.stream);
      if (e == hipSuccess) return ST_OK;
      (void)hipGetLastError();  // fall back to one workgroup per instance
    }
    hipLaunchKernelGGL((k_newton_dense<T, S>), dim3(dense_grid(a.B)), dim3(S::NT), lds, a.stream, k);
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

int dense_seq(const SolveArgs& a) {
  DenseKArgs k = to_dk(a);
  if (a.B <= 0) return ST_OK;
  return dispatch_dense(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    if constexpr (S::MATFREE && S::R > 1)
      hipLaunchKernelGGL((k_seq_kur_split<T, S>), dim3(a.B), dim3(64 * S::R), 0, a.stream, k, a.T_off);
    else
      hipLaunchKernelGGL((k_seq_dense<T, S>), dim3(a.B), dim3(64), 0, a.stream, k, a.T_off);
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

int dense_residual(const SolveArgs& a, void* h, double* hmax) {
  DenseKArgs k = to_dk(a);
  if (int rc = fill_u32(reinterpret_cast<uint32_t*>(hmax), (size_t)a.B * 2, 0u, a.stream)) return rc;
  const int64_t total = a.B * a.T_uniform;
  if (total <= 0) return ST_OK;
  return dispatch_dense(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    hipLaunchKernelGGL((k_residual_dense<T, S>), dim3((total + 3) / 4), dim3(256), 0, a.stream, k,
                       static_cast<T*>(h), hmax);
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

int dense_elements(const SolveArgs& a, void* A, void* b) {
  DenseKArgs k = to_dk(a);
  const int64_t total = a.B * a.T_uniform;
  if (total <= 0) return ST_OK;
  return dispatch_dense(a.dtype, a.system, a.d, [&](auto t, auto s) {
    using T = decltype(t);
    using S = decltype(s);
    const int64_t grid = (total + S::SPP - 1) / S::SPP;
    hipLaunchKernelGGL((k_elements_dense<T, S>), dim3(grid), dim3(S::NT), 0, a.stream, k,
                       static_cast<T*>(A), static_cast<T*>(b));
    return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
  });
}

}  // namespace pint
