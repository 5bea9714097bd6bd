// Host-side interface between the C entry points and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pint {

// Everything a batched solve needs (device pointers unless noted).
struct SolveArgs {
  int32_t system, d, dtype;
  int32_t method;         // one-step rule: 0 RK4, 1 backward Euler, 2 trapezoidal
  int64_t B;
  const void* x0;
  const void* params;
  int64_t pstride;        // scalars between instances' parameter vectors (0 = shared)
  const int64_t* T_off;   // [B+1] or nullptr (uniform)
  int64_t T_uniform;      // used when T_off == nullptr
  int64_t T_max;          // host value
  void* traj;
  double dt, tol, guard;
  int64_t window, max_iter;
  int32_t guess;
  int32_t tile;
  int32_t block;          // batched small-d solver: threads per workgroup (0 = 256)
  int32_t wg_per_cu;      // batched small-d solver: persistent workgroups per CU (0 = 4)
  const int64_t* order;   // [B] order in which instances are taken, or nullptr
  int64_t* iters;
  double* resid;
  int32_t* status;
  void* ws;
  size_t ws_bytes;
  hipStream_t stream;
};

// Status codes shared with the public header.
enum { ST_OK = 0, ST_INVALID = 1, ST_DEVICE = 2, ST_WORKSPACE = 3, ST_NOT_CONVERGED = 4,
       ST_NONFINITE = 5, ST_UNSUPPORTED = 6 };

bool small_supported(int system, int d);
bool dense_supported(int system, int d);

size_t small_ws_bytes(const SolveArgs& a);
int small_solve(const SolveArgs& a);
int small_seq(const SolveArgs& a);
int small_residual(const SolveArgs& a, void* h, double* hmax);
int small_elements(const SolveArgs& a, void* A, void* b);

size_t dense_ws_bytes(const SolveArgs& a);
// The pipelined windowed solver for Lorenz-96 (newton_pipe.hip): workspace
// bytes (0 when it does not apply) and the launch (*used: whether it ran).
size_t pipe_ws_bytes(const SolveArgs& a);
int pipe_solve(const SolveArgs& a, bool* used);
// Process-wide switch between the pipelined solver and the one-update-at-a-
// time cooperative solver (pint_set_dense_pipeline); on by default.
bool dense_pipeline();
int dense_solve(const SolveArgs& a);
int dense_seq(const SolveArgs& a);
int dense_residual(const SolveArgs& a, void* h, double* hmax);
int dense_elements(const SolveArgs& a, void* A, void* b);

size_t scan_ws_bytes(int d, int64_t B, int64_t N, int tile, int dtype);
int affine_scan(int d, int64_t B, int64_t N, int dtype, const void* A, const void* b,
                const void* z0, void* z, int tile, void* ws, size_t ws_bytes, hipStream_t s);

// pint_affine_scan with the library's fixed device scratch (scan.hip).
int affine_scan_noalloc(int d, int64_t B, int64_t N, int dtype, const void* A, const void* b,
                        const void* z0, void* z, int tile, uint32_t* err_out, hipStream_t s);

size_t scan_band_ws_bytes(int d, int bw, int boff, int64_t B, int64_t N, int tile, int dtype);
int affine_scan_band(int d, int bw, int boff, int64_t B, int64_t N, int dtype, const void* band,
                     const void* b, const void* z0, void* z, int tile, void* ws, size_t ws_bytes,
                     hipStream_t s);

size_t adjoint_ws_bytes(int system, int d, int64_t B, int64_t T, int64_t seg, int dtype);
int adjoint(const SolveArgs& a, const void* g, void* dL_dx0, void* dL_dth, int64_t seg);

// Parareal (parareal.hip): M windows of S fine steps; hist [B][max_iter] or nullptr.
size_t parareal_ws_bytes(int d, int64_t B, int64_t M, int dtype);
int parareal(const SolveArgs& a, int64_t M, int64_t S, double* hist);

// Polls before a cross-workgroup wait of the cooperative solvers gives up
// (process-wide; set through pint_set_wait_limit).
uint64_t wait_limit();

// Test hook of the decoupled-lookback scans (process-wide; set through
// pint_set_scan_delay): sleeps injected before some tiles publish.
uint32_t scan_delay();

// Zero `n` 32-bit words with a kernel (no memset nodes in captured graphs).
int fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

}  // namespace pint
