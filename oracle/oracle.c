/*
 * Plain, slow CPU oracle for the parallel-in-time Newton ODE solver
 * (Iacob, Razavi, Sarkka, "A parallel-in-time Newton's method-based ODE
 * solver", arXiv 2511.01465).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU leg of the
 * benchmark do.  It shares no code, header or constant generator with the HIP
 * library.
 *
 * Everything is double precision, written loop by loop in the order the paper
 * states it, and built without floating-point contraction.
 *
 * Contents
 *   - vector fields f, their Jacobians J_f and parameter derivatives f_theta
 *     (logistic, van der Pol, cart-pole from Sec. 4.1; Lorenz-63,
 *     Lorenz-96, Kuramoto and the linear field x' = M x in their textbook
 *     forms);
 *   - the classic four-stage explicit Runge-Kutta step Phi of eq.
 *     (explicit-rk) and its exact derivatives dPhi/dx and dPhi/dtheta by the
 *     chain rule through the stages;
 *   - O1: sequential integration x_{n+1} = Phi(x_n)               (eq. explicit-ode);
 *   - the residual h(xi) of eq. (root-finding-problem);
 *   - O2: Newton's method on h with the Newton step computed by the
 *     sequential forward substitution of eq. (newton-step-recursion), in the
 *     paper's plain form (every step updated every iteration) and in a
 *     windowed form (see orc_newton);
 *   - the affine recursion z_{n+1} = F_n z_n + c_n of eq. (linear-model) and
 *     the composition operator of eq. (assoc-operator);
 *   - O3: the sequential discrete adjoint of x_n = Phi(x_{n-1}; theta)
 *     (block back substitution with H^T) and the tangent recursion used to
 *     check it.
 *
 * Parity status: every function here is pinned by tests under tests/ (the
 * paper's printed residual histories and iteration counts, closed forms,
 * invariants and finite differences), except where a function's comment says
 * "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* System identifiers (the same numbering as the public C interface). */
enum {
  ORC_LINEAR = 0,
  ORC_LOGISTIC = 1,
  ORC_VDP = 2,
  ORC_CARTPOLE = 3,
  ORC_LORENZ63 = 4,
  ORC_LORENZ96 = 5,
  ORC_KURAMOTO = 6,
  ORC_ROBERTSON = 7
};

/* One-step rules: the explicit RK4 step, and the implicit rules of
 * eq. (implicit-ode) with g_n = dt f(x_{n+1}) (backward Euler,
 * eq. implicit-euler) or g_n = dt/2 (f(x_n) + f(x_{n+1})) (trapezoidal). */
enum { ORC_RK4 = 0, ORC_BEULER = 1, ORC_TRAP = 2 };

/* Status codes returned by orc_newton (same numbering as the C interface). */
enum { ORC_OK = 0, ORC_NOT_CONVERGED = 4, ORC_NONFINITE = 5 };

/* Number of parameters of each system for state dimension d; -1 if the
 * dimension is not allowed for that system. */
int orc_n_params(int sys, int d) {
  switch (sys) {
    case ORC_LINEAR: return d >= 1 ? d * d : -1;
    case ORC_LOGISTIC: return d == 1 ? 2 : -1;         /* r, K            */
    case ORC_VDP: return d == 2 ? 1 : -1;              /* mu              */
    case ORC_CARTPOLE: return d == 4 ? 4 : -1;         /* g, l, m_c, m_p  */
    case ORC_LORENZ63: return d == 3 ? 3 : -1;         /* sigma, rho, beta*/
    case ORC_LORENZ96: return d >= 4 ? 1 : -1;         /* F               */
    case ORC_KURAMOTO: return d >= 1 ? d + 1 : -1;     /* K, omega_1..d   */
    case ORC_ROBERTSON: return d == 3 ? 3 : -1;        /* k1, k2, k3      */
  }
  return -1;
}

/* ---------------------------------------------------------------------- */
/* Vector fields f(x; theta)                                               */
/* ---------------------------------------------------------------------- */

/* Cart-pole (Sec. 4.1, eq. cartpole).  State (p, theta, p', theta').  The
 * printed equations use l*theta' (not squared) for the cart and an undefined
 * omega for the pole; both are read as the textbook theta'^2 with
 * omega = theta'. */
static void cartpole_f(const double* P, const double* x, double* out) {
  double g = P[0], l = P[1], mc = P[2], mp = P[3];
  double th = x[1], w = x[3];
  double s = sin(th), c = cos(th);
  double D = mc + mp * s * s;
  out[0] = x[2];
  out[1] = w;
  out[2] = mp * s * (l * w * w + g * c) / D;
  out[3] = (-mp * l * w * w * c * s - (mc + mp) * g * s) / (l * D);
}

void orc_f(int sys, int d, const double* P, const double* x, double* out) {
  int i, j;
  switch (sys) {
    case ORC_LINEAR: /* f = M x */
      for (i = 0; i < d; i++) {
        double acc = 0.0;
        for (j = 0; j < d; j++) acc += P[i * d + j] * x[j];
        out[i] = acc;
      }
      break;
    case ORC_LOGISTIC: /* dP/dt = r P (1 - P/K), eq. (logistic) */
      out[0] = P[0] * x[0] * (1.0 - x[0] / P[1]);
      break;
    case ORC_VDP: /* eq. (vdp) as a first-order system in (x, x') */
      out[0] = x[1];
      out[1] = P[0] * (1.0 - x[0] * x[0]) * x[1] - x[0];
      break;
    case ORC_CARTPOLE:
      cartpole_f(P, x, out);
      break;
    case ORC_LORENZ63:
      out[0] = P[0] * (x[1] - x[0]);
      out[1] = x[0] * (P[1] - x[2]) - x[1];
      out[2] = x[0] * x[1] - P[2] * x[2];
      break;
    case ORC_LORENZ96: /* f_i = (x_{i+1} - x_{i-2}) x_{i-1} - x_i + F, cyclic */
      for (i = 0; i < d; i++) {
        double xp1 = x[(i + 1) % d];
        double xm1 = x[(i + d - 1) % d];
        double xm2 = x[(i + d - 2) % d];
        out[i] = (xp1 - xm2) * xm1 - x[i] + P[0];
      }
      break;
    case ORC_KURAMOTO: /* f_i = omega_i + K sum_j sin(theta_j - theta_i) */
      for (i = 0; i < d; i++) {
        double acc = 0.0;
        for (j = 0; j < d; j++) acc += sin(x[j] - x[i]);
        out[i] = P[1 + i] + P[0] * acc;
      }
      break;
    case ORC_ROBERTSON: /* eq. (robertson), P = (k1, k2, k3) */
      out[0] = -P[0] * x[0] + P[2] * x[1] * x[2];
      out[1] = P[0] * x[0] - P[1] * x[1] * x[1] - P[2] * x[1] * x[2];
      out[2] = P[1] * x[1] * x[1];
      break;
  }
}

/* Jacobian J_f = df/dx, dense, row-major d x d. */
void orc_jf(int sys, int d, const double* P, const double* x, double* J) {
  int i, j;
  memset(J, 0, sizeof(double) * (size_t)d * (size_t)d);
  switch (sys) {
    case ORC_LINEAR:
      for (i = 0; i < d * d; i++) J[i] = P[i];
      break;
    case ORC_LOGISTIC:
      J[0] = P[0] * (1.0 - 2.0 * x[0] / P[1]);
      break;
    case ORC_VDP:
      J[0] = 0.0;
      J[1] = 1.0;
      J[2] = -2.0 * P[0] * x[0] * x[1] - 1.0;
      J[3] = P[0] * (1.0 - x[0] * x[0]);
      break;
    case ORC_CARTPOLE: {
      double g = P[0], l = P[1], mc = P[2], mp = P[3];
      double th = x[1], w = x[3];
      double s = sin(th), c = cos(th);
      double D = mc + mp * s * s;
      double dD = 2.0 * mp * s * c;
      double N1 = mp * s * (l * w * w + g * c);
      double dN1 = mp * (c * (l * w * w + g * c) - g * s * s);
      double N2 = -mp * l * w * w * c * s - (mc + mp) * g * s;
      double dN2 = -mp * l * w * w * (c * c - s * s) - (mc + mp) * g * c;
      J[0 * 4 + 2] = 1.0;
      J[1 * 4 + 3] = 1.0;
      J[2 * 4 + 1] = (dN1 * D - N1 * dD) / (D * D);
      J[2 * 4 + 3] = 2.0 * mp * s * l * w / D;
      J[3 * 4 + 1] = (dN2 * D - N2 * dD) / (l * D * D);
      J[3 * 4 + 3] = -2.0 * mp * l * w * c * s / (l * D);
      break;
    }
    case ORC_LORENZ63:
      J[0] = -P[0]; J[1] = P[0]; J[2] = 0.0;
      J[3] = P[1] - x[2]; J[4] = -1.0; J[5] = -x[0];
      J[6] = x[1]; J[7] = x[0]; J[8] = -P[2];
      break;
    case ORC_LORENZ96:
      for (i = 0; i < d; i++) {
        int ip1 = (i + 1) % d, im1 = (i + d - 1) % d, im2 = (i + d - 2) % d;
        J[i * d + ip1] += x[im1];
        J[i * d + im2] += -x[im1];
        J[i * d + im1] += x[ip1] - x[im2];
        J[i * d + i] += -1.0;
      }
      break;
    case ORC_KURAMOTO:
      for (i = 0; i < d; i++) {
        double diag = 0.0;
        for (j = 0; j < d; j++) {
          if (j == i) continue;
          double cij = P[0] * cos(x[j] - x[i]);
          J[i * d + j] = cij;
          diag -= cij;
        }
        J[i * d + i] = diag;
      }
      break;
    case ORC_ROBERTSON:
      J[0] = -P[0]; J[1] = P[2] * x[2]; J[2] = P[2] * x[1];
      J[3] = P[0]; J[4] = -2.0 * P[1] * x[1] - P[2] * x[2]; J[5] = -P[2] * x[1];
      J[6] = 0.0; J[7] = 2.0 * P[1] * x[1]; J[8] = 0.0;
      break;
  }
}

/* Parameter derivative df/dtheta, row-major d x n_params.  Returns 0, or -1
 * for the cart-pole (no parameter derivative is provided for it). */
int orc_ftheta(int sys, int d, const double* P, const double* x, double* G) {
  int i, np = orc_n_params(sys, d);
  if (np < 0) return -1;
  memset(G, 0, sizeof(double) * (size_t)d * (size_t)np);
  switch (sys) {
    case ORC_LINEAR: /* d(Mx)_i / dM_{ij} = x_j */
      for (i = 0; i < d; i++)
        for (int j = 0; j < d; j++) G[i * np + i * d + j] = x[j];
      return 0;
    case ORC_LOGISTIC:
      G[0] = x[0] * (1.0 - x[0] / P[1]);
      G[1] = P[0] * x[0] * x[0] / (P[1] * P[1]);
      return 0;
    case ORC_VDP:
      G[0] = 0.0;
      G[1] = (1.0 - x[0] * x[0]) * x[1];
      return 0;
    case ORC_LORENZ63:
      G[0 * 3 + 0] = x[1] - x[0];
      G[1 * 3 + 1] = x[0];
      G[2 * 3 + 2] = -x[2];
      return 0;
    case ORC_LORENZ96:
      for (i = 0; i < d; i++) G[i] = 1.0;
      return 0;
    case ORC_KURAMOTO:
      for (i = 0; i < d; i++) {
        double acc = 0.0;
        for (int j = 0; j < d; j++) acc += sin(x[j] - x[i]);
        G[i * np + 0] = acc;
        G[i * np + 1 + i] = 1.0;
      }
      return 0;
    case ORC_ROBERTSON:
      G[0 * 3 + 0] = -x[0]; G[0 * 3 + 2] = x[1] * x[2];
      G[1 * 3 + 0] = x[0]; G[1 * 3 + 1] = -x[1] * x[1]; G[1 * 3 + 2] = -x[1] * x[2];
      G[2 * 3 + 1] = x[1] * x[1];
      return 0;
  }
  return -1;
}

/* ---------------------------------------------------------------------- */
/* Classic RK4 step, eq. (explicit-rk) with c = (0, 1/2, 1/2, 1),          */
/* a21 = a32 = 1/2, a43 = 1, b = (1/6, 1/3, 1/3, 1/6)                     */
/* ---------------------------------------------------------------------- */

/* Small dense helpers: C = A B for d x d (row-major), y = A x.  Every
 * entry C_ij is summed from 0 over k = 0, 1, ..., d-1 in that order (the
 * k loop sits outside the j loop only so that B is read row by row). */
static void matmul(int d, const double* A, const double* B, double* C) {
  for (int i = 0; i < d; i++) {
    double* c = C + (size_t)i * d;
    for (int j = 0; j < d; j++) c[j] = 0.0;
    for (int k = 0; k < d; k++) {
      const double a = A[i * d + k];
      const double* b = B + (size_t)k * d;
      for (int j = 0; j < d; j++) c[j] += a * b[j];
    }
  }
}

static void matvec(int d, const double* A, const double* x, double* y) {
  for (int i = 0; i < d; i++) {
    double acc = 0.0;
    for (int k = 0; k < d; k++) acc += A[i * d + k] * x[k];
    y[i] = acc;
  }
}

/* Phi(x) = x + dt/6 (k1 + 2 k2 + 2 k3 + k4). */
void orc_rk4_step(int sys, int d, const double* P, double dt, const double* x,
                  double* xn) {
  double* w = (double*)malloc(sizeof(double) * 5 * (size_t)d);
  double *k1 = w, *k2 = w + d, *k3 = w + 2 * d, *k4 = w + 3 * d, *y = w + 4 * d;
  int i;
  orc_f(sys, d, P, x, k1);
  for (i = 0; i < d; i++) y[i] = x[i] + 0.5 * dt * k1[i];
  orc_f(sys, d, P, y, k2);
  for (i = 0; i < d; i++) y[i] = x[i] + 0.5 * dt * k2[i];
  orc_f(sys, d, P, y, k3);
  for (i = 0; i < d; i++) y[i] = x[i] + dt * k3[i];
  orc_f(sys, d, P, y, k4);
  for (i = 0; i < d; i++)
    xn[i] = x[i] + dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  free(w);
}

/* The four stage points x, x2, x3, x4 of one RK4 step (each length d). */
static void rk4_stage_points(int sys, int d, const double* P, double dt,
                             const double* x, double* x2, double* x3,
                             double* x4) {
  double* k = (double*)malloc(sizeof(double) * (size_t)d);
  int i;
  orc_f(sys, d, P, x, k);
  for (i = 0; i < d; i++) x2[i] = x[i] + 0.5 * dt * k[i];
  orc_f(sys, d, P, x2, k);
  for (i = 0; i < d; i++) x3[i] = x[i] + 0.5 * dt * k[i];
  orc_f(sys, d, P, x3, k);
  for (i = 0; i < d; i++) x4[i] = x[i] + dt * k[i];
  free(k);
}

/* dPhi/dx by the chain rule through the stages:
 *   K1 = Jf(x), K2 = Jf(x2)(I + dt/2 K1), K3 = Jf(x3)(I + dt/2 K2),
 *   K4 = Jf(x4)(I + dt K3),  J = I + dt/6 (K1 + 2K2 + 2K3 + K4). */
void orc_rk4_jac(int sys, int d, const double* P, double dt, const double* x,
                 double* J) {
  size_t dd = (size_t)d * (size_t)d;
  double* w = (double*)malloc(sizeof(double) * (3 * (size_t)d + 7 * dd));
  double *x2 = w, *x3 = w + d, *x4 = w + 2 * d;
  double *Jf = w + 3 * d, *M = Jf + dd, *K1 = M + dd, *K2 = K1 + dd,
         *K3 = K2 + dd, *K4 = K3 + dd;
  size_t i;
  int r;
  rk4_stage_points(sys, d, P, dt, x, x2, x3, x4);
  orc_jf(sys, d, P, x, K1);
  /* K2 */
  for (i = 0; i < dd; i++) M[i] = 0.5 * dt * K1[i];
  for (r = 0; r < d; r++) M[r * d + r] += 1.0;
  orc_jf(sys, d, P, x2, Jf);
  matmul(d, Jf, M, K2);
  /* K3 */
  for (i = 0; i < dd; i++) M[i] = 0.5 * dt * K2[i];
  for (r = 0; r < d; r++) M[r * d + r] += 1.0;
  orc_jf(sys, d, P, x3, Jf);
  matmul(d, Jf, M, K3);
  /* K4 */
  for (i = 0; i < dd; i++) M[i] = dt * K3[i];
  for (r = 0; r < d; r++) M[r * d + r] += 1.0;
  orc_jf(sys, d, P, x4, Jf);
  matmul(d, Jf, M, K4);
  for (i = 0; i < dd; i++)
    J[i] = dt / 6.0 * (K1[i] + 2.0 * K2[i] + 2.0 * K3[i] + K4[i]);
  for (r = 0; r < d; r++) J[r * d + r] += 1.0;
  free(w);
}

/* dPhi/dtheta (d x np) by the chain rule through the stages:
 *   D1 = f_th(x), D2 = Jf(x2)(dt/2 D1) + f_th(x2),
 *   D3 = Jf(x3)(dt/2 D2) + f_th(x3), D4 = Jf(x4)(dt D3) + f_th(x4),
 *   S = dt/6 (D1 + 2 D2 + 2 D3 + D4).  Returns -1 if f_th is unavailable. */
int orc_rk4_ptheta(int sys, int d, const double* P, double dt, const double* x,
                   double* S) {
  int np = orc_n_params(sys, d);
  if (np < 0) return -1;
  size_t dd = (size_t)d * (size_t)d, dp = (size_t)d * (size_t)np;
  double* w = (double*)malloc(sizeof(double) * (3 * (size_t)d + dd + 6 * dp));
  double *x2 = w, *x3 = w + d, *x4 = w + 2 * d, *Jf = w + 3 * d;
  double *D1 = Jf + dd, *D2 = D1 + dp, *D3 = D2 + dp, *D4 = D3 + dp,
         *G = D4 + dp, *Y = G + dp;
  size_t i;
  int rc = 0;
  rk4_stage_points(sys, d, P, dt, x, x2, x3, x4);
  if (orc_ftheta(sys, d, P, x, D1) != 0) { rc = -1; goto done; }
  /* D2 */
  orc_jf(sys, d, P, x2, Jf);
  for (i = 0; i < dp; i++) Y[i] = 0.5 * dt * D1[i];
  for (int a = 0; a < d; a++)
    for (int b = 0; b < np; b++) {
      double acc = 0.0;
      for (int k = 0; k < d; k++) acc += Jf[a * d + k] * Y[k * np + b];
      D2[a * np + b] = acc;
    }
  orc_ftheta(sys, d, P, x2, G);
  for (i = 0; i < dp; i++) D2[i] += G[i];
  /* D3 */
  orc_jf(sys, d, P, x3, Jf);
  for (i = 0; i < dp; i++) Y[i] = 0.5 * dt * D2[i];
  for (int a = 0; a < d; a++)
    for (int b = 0; b < np; b++) {
      double acc = 0.0;
      for (int k = 0; k < d; k++) acc += Jf[a * d + k] * Y[k * np + b];
      D3[a * np + b] = acc;
    }
  orc_ftheta(sys, d, P, x3, G);
  for (i = 0; i < dp; i++) D3[i] += G[i];
  /* D4 */
  orc_jf(sys, d, P, x4, Jf);
  for (i = 0; i < dp; i++) Y[i] = dt * D3[i];
  for (int a = 0; a < d; a++)
    for (int b = 0; b < np; b++) {
      double acc = 0.0;
      for (int k = 0; k < d; k++) acc += Jf[a * d + k] * Y[k * np + b];
      D4[a * np + b] = acc;
    }
  orc_ftheta(sys, d, P, x4, G);
  for (i = 0; i < dp; i++) D4[i] += G[i];
  for (i = 0; i < dp; i++)
    S[i] = dt / 6.0 * (D1[i] + 2.0 * D2[i] + 2.0 * D3[i] + D4[i]);
done:
  free(w);
  return rc;
}

/* ---------------------------------------------------------------------- */
/* O1: sequential integration                                             */
/* ---------------------------------------------------------------------- */

/* traj[n-1] = x_n for n = 1..T with x_n = Phi(x_{n-1}), x_0 = x0. */
void orc_integrate(int sys, int d, const double* P, double dt, int64_t T,
                   const double* x0, double* traj) {
  const double* prev = x0;
  for (int64_t n = 1; n <= T; n++) {
    double* cur = traj + (size_t)(n - 1) * (size_t)d;
    orc_rk4_step(sys, d, P, dt, prev, cur);
    prev = cur;
  }
}

/* ---------------------------------------------------------------------- */
/* Residual h(xi) of eq. (root-finding-problem)                            */
/* ---------------------------------------------------------------------- */

/* h_n = x_n - x_{n-1} - g_{n-1}(x_{n-1}) = x_n - Phi(x_{n-1}),
 * with xi = (x_1..x_T) and x_0 = x0 fixed.  Writes h[n-1], n = 1..T. */
void orc_residual(int sys, int d, const double* P, double dt, int64_t T,
                  const double* x0, const double* traj, double* h) {
  double* phi = (double*)malloc(sizeof(double) * (size_t)d);
  for (int64_t n = 1; n <= T; n++) {
    const double* prev = n == 1 ? x0 : traj + (size_t)(n - 2) * (size_t)d;
    const double* cur = traj + (size_t)(n - 1) * (size_t)d;
    orc_rk4_step(sys, d, P, dt, prev, phi);
    for (int i = 0; i < d; i++) h[(size_t)(n - 1) * (size_t)d + i] = cur[i] - phi[i];
  }
  free(phi);
}

/* Infinity norm of a vector; +inf if any entry is NaN or infinite. */
static double norm_inf(const double* v, size_t n) {
  double m = 0.0;
  for (size_t i = 0; i < n; i++) {
    if (!isfinite(v[i])) return INFINITY;
    double a = fabs(v[i]);
    if (a > m) m = a;
  }
  return m;
}

/* ---------------------------------------------------------------------- */
/* Affine recursion, eq. (linear-model), and the operator of               */
/* eq. (assoc-operator)                                                    */
/* ---------------------------------------------------------------------- */

/* z_{n+1} = F_n z_n + c_n for n = 0..N-1 from z_0 = z0 (z0 may be NULL for
 * zero).  Writes z[n] = z_{n+1}.  F is [N][d][d], c is [N][d]. */
void orc_affine_seq(int d, int64_t N, const double* F, const double* c,
                    const double* z0, double* z) {
  double* prev = (double*)calloc((size_t)d, sizeof(double));
  if (z0) memcpy(prev, z0, sizeof(double) * (size_t)d);
  for (int64_t n = 0; n < N; n++) {
    const double* Fn = F + (size_t)n * (size_t)d * (size_t)d;
    double* out = z + (size_t)n * (size_t)d;
    matvec(d, Fn, prev, out);
    for (int i = 0; i < d; i++) out[i] += c[(size_t)n * (size_t)d + i];
    memcpy(prev, out, sizeof(double) * (size_t)d);
  }
  free(prev);
}

/* (F_ji, c_ji) (x) (F_nj, c_nj) = (F_ji F_nj, F_ji c_nj + c_ji): the later
 * map (j->i) is the left operand and the earlier map (n->j) the right one. */
void orc_combine(int d, const double* Fl, const double* cl, const double* Fe,
                 const double* ce, double* F, double* c) {
  double* t = (double*)malloc(sizeof(double) * (size_t)d * ((size_t)d + 1));
  matmul(d, Fl, Fe, t);
  matvec(d, Fl, ce, t + (size_t)d * (size_t)d);
  for (int i = 0; i < d * d; i++) F[i] = t[i];
  for (int i = 0; i < d; i++) c[i] = t[d * d + i] + cl[i];
  free(t);
}

/* ---------------------------------------------------------------------- */
/* O2: Newton's method on h(xi) = 0, eqs. (newton-step), (newton-iterates) */
/* ---------------------------------------------------------------------- */

/*
 * traj holds the initial guess xi^(0) on entry and the last iterate on exit.
 *
 * Plain form (window <= 0), the paper's method: at iteration k
 * evaluate h(xi^(k)) over all T steps and r_k = ||h||_inf; stop if r_k < tol;
 * otherwise compute the Newton step by the forward substitution
 *   dx_1 = -h_1,  dx_n = (I + dg_{n-1}/dx_{n-1}) dx_{n-1} - h_n,
 * where I + dg/dx = dPhi/dx at x_{n-1}, and set xi <- xi + dxi.
 *
 * Windowed form (window >= 1, also when window >= T), a safeguard the paper
 * does not state:
 * the steps before the first violation p = min{n : ||h_n||_inf >= tol} are
 * left untouched (their residuals no longer change), the forward
 * substitution runs only over [p, min(T, p + W - 1)] starting from
 * dx_p = -h_p, and the update is accepted only below the first step whose
 * updated state is non-finite or exceeds `guard` in absolute value.
 * Convergence is declared when no step violates the tolerance.
 *
 * hist (length >= max_iter + 1, may be NULL) receives r_k for each
 * evaluation: the global residual in plain form, the residual maximum over
 * the window [p, min(T, p+W-1)] in windowed form.  *iters receives the number
 * of updates applied; *final_resid the global ||h||_inf of the returned
 * iterate.  Returns ORC_OK, ORC_NOT_CONVERGED or ORC_NONFINITE.
 */
int orc_newton(int sys, int d, const double* P, double dt, int64_t T,
               const double* x0, double* traj, double tol, int64_t max_iter,
               int64_t window, double guard, double* hist, int64_t* iters,
               double* final_resid) {
  size_t sd = (size_t)d;
  int status = ORC_OK;
  int64_t k = 0;
  if (T <= 0) {
    if (iters) *iters = 0;
    if (final_resid) *final_resid = 0.0;
    return ORC_OK;
  }
  double* h = (double*)malloc(sizeof(double) * (size_t)T * sd);
  double* dx = (double*)malloc(sizeof(double) * (size_t)T * sd);
  double* J = (double*)malloc(sizeof(double) * sd * sd);
  double* phi = (double*)malloc(sizeof(double) * sd);
  int plain = (window <= 0);

  if (plain) {
    for (k = 0;; k++) {
      orc_residual(sys, d, P, dt, T, x0, traj, h);
      double r = norm_inf(h, (size_t)T * sd);
      if (hist) hist[k] = r;
      if (!isfinite(r)) { status = ORC_NONFINITE; break; }
      if (r < tol) { status = ORC_OK; break; }
      if (k >= max_iter) { status = ORC_NOT_CONVERGED; break; }
      /* forward substitution, eq. (newton-step-recursion) */
      for (int i = 0; i < d; i++) dx[i] = -h[i];
      for (int64_t n = 2; n <= T; n++) {
        const double* xprev = traj + (size_t)(n - 2) * sd;
        orc_rk4_jac(sys, d, P, dt, xprev, J);
        matvec(d, J, dx + (size_t)(n - 2) * sd, dx + (size_t)(n - 1) * sd);
        for (int i = 0; i < d; i++)
          dx[(size_t)(n - 1) * sd + i] -= h[(size_t)(n - 1) * sd + i];
      }
      for (size_t i = 0; i < (size_t)T * sd; i++) traj[i] += dx[i];
    }
  } else {
    int64_t p = 1; /* every step before p has ||h_n|| < tol */
    for (k = 0;; k++) {
      /* first violation at or after p (h_n for n < p cannot have changed) */
      double hp_norm = 0.0;
      for (; p <= T; p++) {
        const double* prev = p == 1 ? x0 : traj + (size_t)(p - 2) * sd;
        orc_rk4_step(sys, d, P, dt, prev, phi);
        for (int i = 0; i < d; i++)
          h[(size_t)(p - 1) * sd + i] = traj[(size_t)(p - 1) * sd + i] - phi[i];
        hp_norm = norm_inf(h + (size_t)(p - 1) * sd, sd);
        if (!(hp_norm < tol)) break;
      }
      if (p > T) { status = ORC_OK; break; }
      if (!isfinite(hp_norm)) { status = ORC_NONFINITE; break; }
      if (k >= max_iter) { status = ORC_NOT_CONVERGED; break; }
      int64_t end = (window >= T - p + 1) ? T : p + window - 1;
      /* residuals over the rest of the window */
      double rwin = hp_norm;
      for (int64_t n = p + 1; n <= end; n++) {
        orc_rk4_step(sys, d, P, dt, traj + (size_t)(n - 2) * sd, phi);
        for (int i = 0; i < d; i++)
          h[(size_t)(n - 1) * sd + i] = traj[(size_t)(n - 1) * sd + i] - phi[i];
        double a = norm_inf(h + (size_t)(n - 1) * sd, sd);
        if (a > rwin) rwin = a;
      }
      if (hist) hist[k] = rwin;
      /* forward substitution restricted to the window */
      for (int i = 0; i < d; i++) dx[(size_t)(p - 1) * sd + i] = -h[(size_t)(p - 1) * sd + i];
      for (int64_t n = p + 1; n <= end; n++) {
        orc_rk4_jac(sys, d, P, dt, traj + (size_t)(n - 2) * sd, J);
        matvec(d, J, dx + (size_t)(n - 2) * sd, dx + (size_t)(n - 1) * sd);
        for (int i = 0; i < d; i++)
          dx[(size_t)(n - 1) * sd + i] -= h[(size_t)(n - 1) * sd + i];
      }
      /* accept below the first non-finite or out-of-guard updated state */
      int64_t q = end + 1;
      for (int64_t n = p; n <= end; n++) {
        int bad = 0;
        for (int i = 0; i < d; i++) {
          double v = traj[(size_t)(n - 1) * sd + i] + dx[(size_t)(n - 1) * sd + i];
          if (!isfinite(v) || fabs(v) > guard) bad = 1;
        }
        if (bad) { q = n; break; }
      }
      if (q == p) { status = ORC_NONFINITE; break; }
      for (int64_t n = p; n < q; n++)
        for (int i = 0; i < d; i++)
          traj[(size_t)(n - 1) * sd + i] += dx[(size_t)(n - 1) * sd + i];
    }
  }
  if (iters) *iters = k;
  if (final_resid) {
    orc_residual(sys, d, P, dt, T, x0, traj, h);
    *final_resid = norm_inf(h, (size_t)T * sd);
  }
  free(h);
  free(dx);
  free(J);
  free(phi);
  return status;
}

/* ---------------------------------------------------------------------- */
/* Implicit one-step rules (Sec. 3.4)                                      */
/* ---------------------------------------------------------------------- */

/* g = g_{n-1}(x_{n-1}, x_n) of eq. (implicit-ode) and its partial
 * derivatives Gp = dg/dx_{n-1}, Gc = dg/dx_n (d x d, row-major):
 *   backward Euler: g = dt f(x_n),                Gp = 0,            Gc = dt Jf(x_n);
 *   trapezoidal:    g = dt/2 (f(x_{n-1}) + f(x_n)), Gp = dt/2 Jf(x_{n-1}), Gc = dt/2 Jf(x_n). */
static void implicit_g(int method, int sys, int d, const double* P, double dt,
                       const double* xp, const double* xc, double* g, double* Gp,
                       double* Gc) {
  size_t dd = (size_t)d * (size_t)d;
  double* w = (double*)malloc(sizeof(double) * (size_t)d);
  int i;
  if (method == ORC_BEULER) {
    orc_f(sys, d, P, xc, g);
    for (i = 0; i < d; i++) g[i] *= dt;
    if (Gp) memset(Gp, 0, sizeof(double) * dd);
    if (Gc) {
      orc_jf(sys, d, P, xc, Gc);
      for (size_t q = 0; q < dd; q++) Gc[q] *= dt;
    }
  } else { /* ORC_TRAP */
    orc_f(sys, d, P, xp, g);
    orc_f(sys, d, P, xc, w);
    for (i = 0; i < d; i++) g[i] = 0.5 * dt * g[i] + 0.5 * dt * w[i];
    if (Gp) {
      orc_jf(sys, d, P, xp, Gp);
      for (size_t q = 0; q < dd; q++) Gp[q] *= 0.5 * dt;
    }
    if (Gc) {
      orc_jf(sys, d, P, xc, Gc);
      for (size_t q = 0; q < dd; q++) Gc[q] *= 0.5 * dt;
    }
  }
  free(w);
}

/* Solve M X = B for d x d M and B with nrhs columns (row-major, B
 * overwritten by X), Gaussian elimination with partial pivoting on a copy
 * of M.  Returns -1 when a pivot is exactly zero. */
static int solve_lin(int d, const double* M, double* B, int nrhs) {
  double* A = (double*)malloc(sizeof(double) * (size_t)d * (size_t)d);
  memcpy(A, M, sizeof(double) * (size_t)d * (size_t)d);
  int rc = 0;
  for (int c = 0; c < d; c++) {
    int piv = c;
    for (int r = c + 1; r < d; r++)
      if (fabs(A[r * d + c]) > fabs(A[piv * d + c])) piv = r;
    if (A[piv * d + c] == 0.0) { rc = -1; break; }
    if (piv != c) {
      for (int k = 0; k < d; k++) {
        double t = A[c * d + k]; A[c * d + k] = A[piv * d + k]; A[piv * d + k] = t;
      }
      for (int k = 0; k < nrhs; k++) {
        double t = B[c * nrhs + k]; B[c * nrhs + k] = B[piv * nrhs + k]; B[piv * nrhs + k] = t;
      }
    }
    for (int r = c + 1; r < d; r++) {
      double l = A[r * d + c] / A[c * d + c];
      for (int k = c; k < d; k++) A[r * d + k] -= l * A[c * d + k];
      for (int k = 0; k < nrhs; k++) B[r * nrhs + k] -= l * B[c * nrhs + k];
    }
  }
  if (rc == 0)
    for (int c = d - 1; c >= 0; c--)
      for (int k = 0; k < nrhs; k++) {
        double acc = B[c * nrhs + k];
        for (int q = c + 1; q < d; q++) acc -= A[c * d + q] * B[q * nrhs + k];
        B[c * nrhs + k] = acc / A[c * d + c];
      }
  free(A);
  return rc;
}

/* h_n = x_n - x_{n-1} - g_{n-1}(x_{n-1}, x_n), n = 1..T, of eq.
 * (root-finding-problem-implicit); h[n-1] receives h_n.  With `scaled`, the
 * quantity the paper plots for its implicit solver instead:
 * (I - dg_{n-1}/dx_n)^{-1} h_n (a reading: its printed first values are
 * these, not ||h||; e.g. 1/(1 + dt) for the Dahlquist problem from the
 * zero guess, where h_1 = -x_0). */
void orc_residual_implicit(int method, int sys, int d, const double* P, double dt,
                           int64_t T, const double* x0, const double* traj, int scaled,
                           double* h) {
  size_t sd = (size_t)d;
  double* g = (double*)malloc(sizeof(double) * sd);
  double* Gc = (double*)malloc(sizeof(double) * sd * sd);
  for (int64_t n = 1; n <= T; n++) {
    const double* xp = n == 1 ? x0 : traj + (size_t)(n - 2) * sd;
    const double* xc = traj + (size_t)(n - 1) * sd;
    double* hn = h + (size_t)(n - 1) * sd;
    implicit_g(method, sys, d, P, dt, xp, xc, g, NULL, Gc);
    for (int i = 0; i < d; i++) hn[i] = xc[i] - xp[i] - g[i];
    if (scaled) {
      for (size_t q = 0; q < sd * sd; q++) Gc[q] = -Gc[q];
      for (int i = 0; i < d; i++) Gc[i * d + i] += 1.0;
      if (solve_lin(d, Gc, hn, 1) != 0)
        for (int i = 0; i < d; i++) hn[i] = NAN;
    }
  }
  free(g);
  free(Gc);
}

/* O1 for an implicit rule: x_n solves x_n - x_{n-1} - g(x_{n-1}, x_n) = 0,
 * step by step, by Newton's method from x_{n-1} until the correction is
 * below 4 eps |x_n| (at most 100 corrections per step).  traj[n-1] = x_n.
 * Returns 0, or -1 if a step did not converge. */
int orc_integrate_implicit(int method, int sys, int d, const double* P, double dt,
                           int64_t T, const double* x0, double* traj) {
  size_t sd = (size_t)d;
  double* g = (double*)malloc(sizeof(double) * sd);
  double* M = (double*)malloc(sizeof(double) * sd * sd);
  double* r = (double*)malloc(sizeof(double) * sd);
  int rc = 0;
  const double* prev = x0;
  for (int64_t n = 1; n <= T && rc == 0; n++) {
    double* y = traj + (size_t)(n - 1) * sd;
    for (int i = 0; i < d; i++) y[i] = prev[i];
    int ok = 0;
    for (int it = 0; it < 100; it++) {
      implicit_g(method, sys, d, P, dt, prev, y, g, NULL, M);
      for (size_t q = 0; q < sd * sd; q++) M[q] = -M[q];
      for (int i = 0; i < d; i++) M[i * d + i] += 1.0;
      for (int i = 0; i < d; i++) r[i] = y[i] - prev[i] - g[i];
      if (solve_lin(d, M, r, 1) != 0) break;
      double dn = 0.0, yn = 0.0;
      for (int i = 0; i < d; i++) {
        y[i] -= r[i];
        if (fabs(r[i]) > dn) dn = fabs(r[i]);
        if (fabs(y[i]) > yn) yn = fabs(y[i]);
      }
      if (dn <= 4.0 * 2.220446049250313e-16 * yn) { ok = 1; break; }
    }
    if (!ok) rc = -1;
    prev = y;
  }
  free(g);
  free(M);
  free(r);
  return rc;
}

/*
 * O2 for an implicit rule: Newton's method on eq. (root-finding-problem-
 * implicit) with the step of eq. (newton-step-implicit-recursion),
 *   dx_1 = -(I - dg_0/dx_1)^{-1} h_1,
 *   dx_n = -(I - dg_{n-1}/dx_n)^{-1} [(-I - dg_{n-1}/dx_{n-1}) dx_{n-1} + h_n],
 * evaluated in order.  The residual recorded in hist, tested against tol
 * and returned in *final_resid is the scaled one of orc_residual_implicit
 * (max over steps and components).  Plain (window <= 0) and windowed forms
 * as in orc_newton, with p the first step whose scaled residual is >= tol.
 * A singular (I - dg/dx_n) stops with ORC_NONFINITE.
 */
int orc_newton_implicit(int method, int sys, int d, const double* P, double dt,
                        int64_t T, const double* x0, double* traj, double tol,
                        int64_t max_iter, int64_t window, double guard, double* hist,
                        int64_t* iters, double* final_resid) {
  size_t sd = (size_t)d, dd = sd * sd;
  int status = ORC_OK;
  int64_t k = 0;
  if (T <= 0) {
    if (iters) *iters = 0;
    if (final_resid) *final_resid = 0.0;
    return ORC_OK;
  }
  double* h = (double*)malloc(sizeof(double) * (size_t)T * sd);
  double* dx = (double*)malloc(sizeof(double) * (size_t)T * sd);
  double* g = (double*)malloc(sizeof(double) * sd);
  double* Gp = (double*)malloc(sizeof(double) * dd);
  double* Gc = (double*)malloc(sizeof(double) * dd);
  double* v = (double*)malloc(sizeof(double) * sd);
  double* hs = (double*)malloc(sizeof(double) * sd);
  int plain = (window <= 0);
  int64_t p = 1;

  /* dx over [lo, hi] from dx_{lo-1} = 0; returns -1 on a singular step */
  #define STEP_RANGE(lo, hi)                                                     \
    for (int64_t n = (lo); n <= (hi); n++) {                                     \
      const double* xp = n == 1 ? x0 : traj + (size_t)(n - 2) * sd;             \
      const double* xc = traj + (size_t)(n - 1) * sd;                            \
      double* dn = dx + (size_t)(n - 1) * sd;                                    \
      implicit_g(method, sys, d, P, dt, xp, xc, g, Gp, Gc);                      \
      for (int i = 0; i < d; i++) {                                              \
        double acc = xc[i] - xp[i] - g[i]; /* h_n */                             \
        if (n > (lo)) {                                                          \
          const double* dp = dx + (size_t)(n - 2) * sd;                          \
          double t = -dp[i];                                                     \
          for (int q = 0; q < d; q++) t -= Gp[i * d + q] * dp[q];                \
          acc += t;                                                              \
        }                                                                        \
        v[i] = -acc;                                                             \
      }                                                                          \
      for (size_t q = 0; q < dd; q++) Gc[q] = -Gc[q];                            \
      for (int i = 0; i < d; i++) Gc[i * d + i] += 1.0;                          \
      if (solve_lin(d, Gc, v, 1) != 0) { singular = 1; break; }                  \
      for (int i = 0; i < d; i++) dn[i] = v[i];                                  \
    }

  for (k = 0;; k++) {
    int singular = 0;
    int64_t lo, hi;
    double r = 0.0;
    if (plain) {
      orc_residual_implicit(method, sys, d, P, dt, T, x0, traj, 1, h);
      r = norm_inf(h, (size_t)T * sd);
      if (hist) hist[k] = r;
      if (!isfinite(r)) { status = ORC_NONFINITE; break; }
      if (r < tol) { status = ORC_OK; break; }
      if (k >= max_iter) { status = ORC_NOT_CONVERGED; break; }
      lo = 1;
      hi = T;
    } else {
      /* first violation at or after p */
      double hp = 0.0;
      for (; p <= T; p++) {
        const double* xp = p == 1 ? x0 : traj + (size_t)(p - 2) * sd;
        const double* xc = traj + (size_t)(p - 1) * sd;
        implicit_g(method, sys, d, P, dt, xp, xc, g, NULL, Gc);
        for (int i = 0; i < d; i++) hs[i] = xc[i] - xp[i] - g[i];
        for (size_t q = 0; q < dd; q++) Gc[q] = -Gc[q];
        for (int i = 0; i < d; i++) Gc[i * d + i] += 1.0;
        if (solve_lin(d, Gc, hs, 1) != 0) { hp = INFINITY; break; }
        hp = norm_inf(hs, sd);
        if (!(hp < tol)) break;
      }
      if (p > T) { status = ORC_OK; break; }
      if (!isfinite(hp)) { status = ORC_NONFINITE; break; }
      if (k >= max_iter) { status = ORC_NOT_CONVERGED; break; }
      if (hist) hist[k] = hp;
      lo = p;
      hi = (window >= T - p + 1) ? T : p + window - 1;
    }
    STEP_RANGE(lo, hi)
    if (singular) { status = ORC_NONFINITE; break; }
    /* accept below the first non-finite or out-of-guard updated state */
    int64_t q = hi + 1;
    if (!plain)
      for (int64_t n = lo; n <= hi; n++) {
        int bad = 0;
        for (int i = 0; i < d; i++) {
          double val = traj[(size_t)(n - 1) * sd + i] + dx[(size_t)(n - 1) * sd + i];
          if (!isfinite(val) || fabs(val) > guard) bad = 1;
        }
        if (bad) { q = n; break; }
      }
    if (q == lo) { status = ORC_NONFINITE; break; }
    for (int64_t n = lo; n < q; n++)
      for (int i = 0; i < d; i++) traj[(size_t)(n - 1) * sd + i] += dx[(size_t)(n - 1) * sd + i];
  }
  #undef STEP_RANGE
  if (iters) *iters = k;
  if (final_resid) {
    orc_residual_implicit(method, sys, d, P, dt, T, x0, traj, 1, h);
    *final_resid = norm_inf(h, (size_t)T * sd);
  }
  free(h);
  free(dx);
  free(g);
  free(Gp);
  free(Gc);
  free(v);
  free(hs);
  return status;
}

/* ---------------------------------------------------------------------- */
/* O3: sequential discrete adjoint and the tangent recursion               */
/* ---------------------------------------------------------------------- */

/*
 * For x_n = Phi(x_{n-1}; theta), n = 1..T, and a loss L(x_1..x_T) with
 * g_n = dL/dx_n (g is [T][d]):
 *   lambda_T = g_T,  lambda_n = g_n + J(x_n)^T lambda_{n+1}  (n = T-1..1),
 *   dL/dx0 = J(x_0)^T lambda_1,  dL/dtheta = sum_{n=1..T} S(x_{n-1})^T lambda_n,
 * with J = dPhi/dx and S = dPhi/dtheta.  This is the back substitution
 * H^T lambda = g with the block-bidiagonal H of eq. (jacobian).
 * dL_dtheta may be NULL.  Returns -1 if S is unavailable for the system.
 */
int orc_adjoint(int sys, int d, const double* P, double dt, int64_t T,
                const double* x0, const double* traj, const double* g,
                double* dL_dx0, double* dL_dtheta) {
  int np = orc_n_params(sys, d);
  size_t sd = (size_t)d;
  double* lam = (double*)malloc(sizeof(double) * sd);
  double* nl = (double*)malloc(sizeof(double) * sd);
  double* J = (double*)malloc(sizeof(double) * sd * sd);
  double* S = (double*)malloc(sizeof(double) * sd * (size_t)(np > 0 ? np : 1));
  int rc = 0;
  if (dL_dtheta)
    for (int j = 0; j < np; j++) dL_dtheta[j] = 0.0;
  if (T <= 0) {
    for (int i = 0; i < d; i++) dL_dx0[i] = 0.0;
    goto done;
  }
  for (int i = 0; i < d; i++) lam[i] = g[(size_t)(T - 1) * sd + i];
  for (int64_t n = T; n >= 1; n--) {
    /* lam holds lambda_n here */
    const double* xprev = n == 1 ? x0 : traj + (size_t)(n - 2) * sd;
    if (dL_dtheta) {
      if (orc_rk4_ptheta(sys, d, P, dt, xprev, S) != 0) { rc = -1; goto done; }
      for (int j = 0; j < np; j++) {
        double acc = 0.0;
        for (int i = 0; i < d; i++) acc += S[i * np + j] * lam[i];
        dL_dtheta[j] += acc;
      }
    }
    orc_rk4_jac(sys, d, P, dt, xprev, J);
    /* J(x_{n-1})^T lambda_n */
    for (int i = 0; i < d; i++) {
      double acc = 0.0;
      for (int k = 0; k < d; k++) acc += J[k * d + i] * lam[k];
      nl[i] = acc;
    }
    if (n == 1) {
      for (int i = 0; i < d; i++) dL_dx0[i] = nl[i];
    } else {
      for (int i = 0; i < d; i++) lam[i] = nl[i] + g[(size_t)(n - 2) * sd + i];
    }
  }
done:
  free(lam);
  free(nl);
  free(J);
  free(S);
  return rc;
}

/* Tangent of the trajectory: v_0 = dx0, v_n = J(x_{n-1}) v_{n-1} +
 * S(x_{n-1}) dtheta (dtheta may be NULL).  Writes v[n-1], n = 1..T.
 * Returns -1 if S is needed but unavailable. */
int orc_tangent(int sys, int d, const double* P, double dt, int64_t T,
                const double* x0, const double* traj, const double* dx0,
                const double* dtheta, double* v) {
  int np = orc_n_params(sys, d);
  size_t sd = (size_t)d;
  double* J = (double*)malloc(sizeof(double) * sd * sd);
  double* S = (double*)malloc(sizeof(double) * sd * (size_t)(np > 0 ? np : 1));
  double* prevv = (double*)malloc(sizeof(double) * sd);
  int rc = 0;
  memcpy(prevv, dx0, sizeof(double) * sd);
  for (int64_t n = 1; n <= T; n++) {
    const double* xprev = n == 1 ? x0 : traj + (size_t)(n - 2) * sd;
    double* out = v + (size_t)(n - 1) * sd;
    orc_rk4_jac(sys, d, P, dt, xprev, J);
    matvec(d, J, prevv, out);
    if (dtheta) {
      if (orc_rk4_ptheta(sys, d, P, dt, xprev, S) != 0) { rc = -1; break; }
      for (int i = 0; i < d; i++) {
        double acc = 0.0;
        for (int j = 0; j < np; j++) acc += S[i * np + j] * dtheta[j];
        out[i] += acc;
      }
    }
    memcpy(prevv, out, sizeof(double) * sd);
  }
  free(J);
  free(S);
  free(prevv);
  return rc;
}

/* ---------------------------------------------------------------------- */
/* Parareal, the comparison method of Sec. 2.2                             */
/* ---------------------------------------------------------------------- */

/* One step of the rule `method` from x to out with step size h: the RK4 map
 * Phi for ORC_RK4, else the implicit step solved by orc_integrate_implicit.
 * Returns 0, or -1 if an implicit step did not converge. */
static int one_step(int method, int sys, int d, const double* P, double h,
                    const double* x, double* out) {
  if (method == ORC_RK4) {
    orc_rk4_step(sys, d, P, h, x, out);
    return 0;
  }
  return orc_integrate_implicit(method, sys, d, P, h, 1, x, out);
}

/*
 * Parareal (Sec. 2.2, eqs. parareal-init, fine-integrator,
 * coarse-integrator) over M windows of S fine steps each:
 *   coarse G(x) = one step of the rule with step size S*dt,
 *   fine   F(x) = S steps of the rule with step size dt.
 * Initial coarse sweep x_{m+1} = G(x_m), x_0 = x0; then per iteration
 *   F_m = F(x_m) for every window (independent of each other),
 *   R = max_m ||x_{m+1} - F_m||_inf (the paper's error measure R^(k)),
 *   stop if R < tol (strict), else the sequential correction
 *   x_{m+1} <- G(x_m new) + F_m - G(x_m old).
 * The paper takes M = floor(sqrt(N)) and S = floor(N / M) (a reading: with
 * them this function reproduces the paper's printed R histories).
 *
 * traj ([M*S][d]) receives the dense trajectory of the last fine sweep:
 * traj[m*S + j] is the state after j+1 fine steps of window m.  hist
 * (length >= max_iter, may be NULL) receives R of each fine sweep.  *iters
 * receives K, the number of fine sweeps (= residual evaluations, the count
 * the paper plots); *final_resid the last R.  Returns ORC_OK,
 * ORC_NOT_CONVERGED (max_iter sweeps without R < tol) or ORC_NONFINITE (a
 * non-finite R or an implicit step that did not converge).
 */
int orc_parareal(int method, int sys, int d, const double* P, double dt, int64_t M,
                 int64_t S, const double* x0, double tol, int64_t max_iter,
                 double* traj, double* hist, int64_t* iters, double* final_resid) {
  size_t sd = (size_t)d;
  int status = ORC_OK;
  int64_t k = 0;
  double R = 0.0;
  if (M <= 0 || S <= 0) {
    if (iters) *iters = 0;
    if (final_resid) *final_resid = 0.0;
    return ORC_OK;
  }
  double H = (double)S * dt;
  double* x = (double*)malloc(sizeof(double) * (size_t)(M + 1) * sd);    /* x_0..x_M   */
  double* xn = (double*)malloc(sizeof(double) * (size_t)(M + 1) * sd);   /* next iterate */
  double* F = (double*)malloc(sizeof(double) * (size_t)M * sd);          /* F_m        */
  double* Gold = (double*)malloc(sizeof(double) * (size_t)M * sd);       /* G(x_m) old */
  double* Gnew = (double*)malloc(sizeof(double) * sd);

  /* eq. parareal-init */
  memcpy(x, x0, sizeof(double) * sd);
  for (int64_t m = 0; m < M && status == ORC_OK; m++) {
    if (one_step(method, sys, d, P, H, x + (size_t)m * sd, Gold + (size_t)m * sd) != 0)
      status = ORC_NONFINITE;
    memcpy(x + (size_t)(m + 1) * sd, Gold + (size_t)m * sd, sizeof(double) * sd);
  }
  while (status == ORC_OK) {
    /* eq. fine-integrator: every window from its own start */
    for (int64_t m = 0; m < M && status == ORC_OK; m++) {
      const double* prev = x + (size_t)m * sd;
      for (int64_t j = 0; j < S; j++) {
        double* cur = traj + (size_t)(m * S + j) * sd;
        if (one_step(method, sys, d, P, dt, prev, cur) != 0) { status = ORC_NONFINITE; break; }
        prev = cur;
      }
      memcpy(F + (size_t)m * sd, prev, sizeof(double) * sd);
    }
    if (status != ORC_OK) break;
    /* R = max over windows of |x_{m+1} - F_m| */
    R = 0.0;
    for (int64_t m = 0; m < M; m++)
      for (size_t i = 0; i < sd; i++) {
        double e = x[(size_t)(m + 1) * sd + i] - F[(size_t)m * sd + i];
        if (!isfinite(e)) R = INFINITY;
        else if (fabs(e) > R) R = fabs(e);
      }
    if (hist) hist[k] = R;
    k++;
    if (!isfinite(R)) { status = ORC_NONFINITE; break; }
    if (R < tol) break;
    if (k >= max_iter) { status = ORC_NOT_CONVERGED; break; }
    /* eq. coarse-integrator: sequential correction sweep */
    memcpy(xn, x0, sizeof(double) * sd);
    for (int64_t m = 0; m < M; m++) {
      if (one_step(method, sys, d, P, H, xn + (size_t)m * sd, Gnew) != 0) {
        status = ORC_NONFINITE;
        break;
      }
      for (size_t i = 0; i < sd; i++)
        xn[(size_t)(m + 1) * sd + i] = (Gnew[i] + F[(size_t)m * sd + i]) - Gold[(size_t)m * sd + i];
      memcpy(Gold + (size_t)m * sd, Gnew, sizeof(double) * sd);
    }
    double* t = x; x = xn; xn = t;
  }
  if (iters) *iters = k;
  if (final_resid) *final_resid = R;
  free(x);
  free(xn);
  free(F);
  free(Gold);
  free(Gnew);
  return status;
}
