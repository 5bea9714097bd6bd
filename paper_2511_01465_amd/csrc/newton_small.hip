// Host side of the small-d solver (d <= 4): launch shapes and the RK4
// instantiation of the kernels in newton_small.h; the implicit rules are
// instantiated in implicit_small.hip.  Also the fill kernel the library uses
// instead of memset nodes.
#include "newton_small.h"

namespace pint {

// Threads per workgroup = steps per chunk of the in-workgroup scan: 64, 128
// or 256 (a launch-shape choice; results do not depend on it).
constexpr int NT_SMALL = 256;

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

int fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return ST_OK;
  const int blocks = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError() == hipSuccess ? ST_OK : ST_DEVICE;
}

bool small_supported(int system, int d) {
  return dispatch_small(0, system, d, [](auto, auto) { return ST_OK; }) == ST_OK;
}

static SmallKArgs to_k(const SolveArgs& a) {
  SmallKArgs k{};
  k.B = a.B;
  k.x0 = a.x0;
  k.params = a.params;
  k.pstride = a.pstride;
  k.T_off = a.T_off;
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
  k.order = a.order;
  k.wait_limit = wait_limit();
  return k;
}

static int run(const SolveArgs& a, const SmallKArgs& k, SmallLaunch l) {
  l.dtype = a.dtype;
  l.system = a.system;
  l.d = a.d;
  l.stream = a.stream;
  if (a.method == METHOD_RK4) return small_launch<METHOD_RK4>(k, l);
  return small_launch_implicit(a.method, k, l);
}

static int num_cus_small() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus;
}

// Workgroups per instance of the cooperative solver, or 0 when the batched
// one-workgroup-per-instance solver is used instead: plain mode, `tile`
// steps per workgroup (rounded up to whole chunks of NT_COOP; 0 means one
// chunk), at least four workgroups, all B * G of them resident at once.
static int coop_groups_small(const SolveArgs& a) {
  if (a.window > 0 || a.B <= 0) return 0;
  const int64_t T = a.T_off ? a.T_max : a.T_uniform;
  const int64_t per = a.tile > 0 ? ((int64_t)a.tile + NT_COOP - 1) / NT_COOP * NT_COOP : NT_COOP;
  int64_t G = (T + per - 1) / per;
  int per_cu = 0;
  SmallLaunch l{};
  l.op = OP_COOP_OCCUPANCY;
  l.occupancy = &per_cu;
  if (run(a, SmallKArgs{}, l) != ST_OK || per_cu <= 0) return 0;
  const int64_t cap = (int64_t)per_cu * num_cus_small();
  if (a.B * G > cap) G = cap / a.B;
  if (G < 4) return 0;
  G = (T + (T + G - 1) / G - 1) / ((T + G - 1) / G);  // no empty range at the end
  return G >= 4 ? (int)G : 0;
}

static size_t coop_bytes(const SolveArgs& a, int G) {
  if (G <= 0) return 0;
  return coop_layout(G, a.d, a.dtype == 0 ? 8 : 4).stride * (size_t)a.B;
}

size_t small_ws_bytes(const SolveArgs& a) { return 256 + coop_bytes(a, coop_groups_small(a)); }

int small_solve(const SolveArgs& a) {
  const int G = a.T_off ? 0 : coop_groups_small(a);
  const size_t need = 256 + coop_bytes(a, G);
  if (a.ws_bytes < need || a.ws == nullptr) return ST_WORKSPACE;
  SmallKArgs k = to_k(a);
  char* w = static_cast<char*>(a.ws);
  if (G > 0) {
    // control blocks, counters and flags start at zero (a kernel, not a memset)
    if (int rc = fill_u32(reinterpret_cast<uint32_t*>(w + 256), coop_bytes(a, G) / 4, 0u, a.stream))
      return rc;
    SmallLaunch l{};
    l.op = OP_COOP;
    l.grid = (int)(a.B * G);
    l.G = G;
    l.coop_ws = w + 256;
    if (run(a, k, l) == ST_OK) return ST_OK;
    (void)hipGetLastError();  // not launchable cooperatively: the batched solver below
  }
  k.queue = reinterpret_cast<uint32_t*>(w);
  if (int rc = fill_u32(k.queue, 1, 0u, a.stream)) return rc;
  const int cus = num_cus_small();
  const int64_t want = (int64_t)cus * (a.wg_per_cu > 0 ? a.wg_per_cu : 4);
  const int grid = (int)(a.B < want ? a.B : want);
  if (grid <= 0) return ST_OK;
  SmallLaunch l{};
  l.op = OP_SOLVE;
  l.grid = grid;
  l.block = a.block > 0 ? a.block : NT_SMALL;
  return run(a, k, l);
}

int small_seq(const SolveArgs& a) {
  SmallKArgs k = to_k(a);
  if (a.B <= 0) return ST_OK;
  SmallLaunch l{};
  l.op = OP_SEQ;
  l.grid = (int)((a.B + 63) / 64);
  l.block = 64;
  return run(a, k, l);
}

int small_residual(const SolveArgs& a, void* h, double* hmax) {
  SmallKArgs k = to_k(a);
  if (int rc = fill_u32(reinterpret_cast<uint32_t*>(hmax), (size_t)a.B * 2, 0u, a.stream)) return rc;
  const int64_t total = a.B * a.T_uniform;
  if (total <= 0) return ST_OK;
  SmallLaunch l{};
  l.op = OP_RESIDUAL;
  l.grid = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  l.block = 256;
  l.out0 = h;
  l.hmax = hmax;
  return run(a, k, l);
}

int small_elements(const SolveArgs& a, void* A, void* b) {
  SmallKArgs k = to_k(a);
  const int64_t total = a.B * a.T_uniform;
  if (total <= 0) return ST_OK;
  SmallLaunch l{};
  l.op = OP_ELEMENTS;
  l.grid = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  l.block = 256;
  l.out0 = A;
  l.out1 = b;
  return run(a, k, l);
}

}  // namespace pint
