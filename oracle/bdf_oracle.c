/*
 * bdf_oracle.c -- plain FP64 CPU reference for per-cell variable-order BDF
 * integration of mass-action kinetics.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library) shares no code with it and never calls it.
 *
 * What it computes (arXiv 2405.01713, Balos et al.):
 *   For every cell independently, y' = R(y) + F with y(t0) = y0 over one outer
 *   step [t0, t_out] (the spatially decoupled ODE of Sec. 3.1, Eq. (7)), where
 *   R is mass-action kinetics and F a constant forcing.  Integration is
 *   CVODE-style variable-order (1..5), variable-step BDF (Sec. 2, Eq. (1)):
 *   local error tested in the WRMS norm of Sec. 2, Eq. (3); modified Newton
 *   with the stopping test of Sec. 2, Eq. (4) (c_eps = 0.1, c_r = 0.3);
 *   Newton matrix I - gamma*J with an analytic Jacobian (Table 1, approaches
 *   2A/2B) factored by dense LU with partial pivoting (Sec. 4.1.4).
 *   Step and order are controlled per cell (the paper's batches run in lock
 *   step; per-cell control removes the "stiffest cell dictates the step"
 *   limitation of Sec. 2).  Options: a Jacobian by difference quotients
 *   (approaches 3A/3B), or an inexact Newton iteration whose linear systems
 *   are solved by matrix-free GMRES on the scaled system of Sec. 2,
 *   Eqs. (5) and (6) (approaches 1A/1B).
 *
 * The paper gives no BDF coefficients, heuristics or constants beyond
 * Eqs. (3) and (4).  Where it is silent the following readings are used, each
 * stated where it is implemented: Nordsieck variable-coefficient BDF with
 * Lambda(x) = prod_i (1 + x/xi_i); error constant 1/(l_1 xi_{q+1});
 * interpolation-preserving order changes; the initial-step estimate; the
 * failure-recovery and setup heuristics.
 *
 * Non-isothermal cells (a mechanism with heat capacities): temperature is
 * the state's last component and the rate constants are re-evaluated from it
 * at every right-hand side (the Arrhenius terms of Sec. 3.1 with T varying,
 * as in the zero-dimensional constant-internal-energy reactor of Sec. 4.1.3).  The reactor is adiabatic at constant volume with synthetic
 * species energies u_i(T) = u0_i + cv_i T, so the total energy
 * sum_i y_i u_i(T) is constant: dT/dt = F_T - sum_i u_i(T) dy_i/dt / sum_i
 * cv_i y_i.
 *
 * Everything is scalar, straightforward and unblocked so that it can be
 * checked against the mathematics by eye.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXS 64
#define ORC_QMAX 5
#define ORC_SLOTS 3
#define ORC_UROUND 2.220446049250313e-16
#define ORC_GMRES_MAXL 10
#define ORC_MAXB 16                    /* cells per lock-step batch */
#define ORC_MAXN (ORC_MAXS * ORC_MAXB) /* state length of a lock-step batch */

/* Per-cell status codes. */
#define ORC_SUCCESS 0
#define ORC_TOO_MUCH_WORK (-1)
#define ORC_ERR_FAILURE (-3)
#define ORC_CONV_FAILURE (-4)
#define ORC_SETUP_FAILURE (-6)
#define ORC_NONFINITE (-9)
#define ORC_RECORD_FULL (-10)

typedef struct {
  int32_t n_species, n_reactions;
  const int32_t *reac; /* [R][3] reactant species, -1 = empty */
  const int32_t *prod; /* [R][3] product species, -1 = empty */
  const double *lnA;   /* [R] ln of the forward pre-exponential factor */
  const double *EaR;   /* [R] activation temperature Ea/R (K); NULL = 0 */
  const double *lnK;   /* [R] ln equilibrium constant; NULL = irreversible */
  const double *cv;    /* [S] heat capacity per unit amount; NULL = isothermal */
  const double *u0;    /* [S] energy at T = 0 per unit amount (with cv) */
} orc_mech;

typedef struct {
  double rtol;
  const double *atol; /* [atol_len] */
  int32_t atol_len;   /* 1 or >= S */
  int32_t max_order;  /* 1..5 */
  int32_t max_steps;  /* per integrate call */
  int32_t jac_dq;     /* 1: Jacobian by difference quotients (approaches 3A/3B), 0: analytic */
  int32_t gmres_maxl; /* 1..ORC_GMRES_MAXL: inexact Newton with GMRES of this Krylov dimension
                         (approaches 1A/1B); 0: modified Newton with a direct solve */
  int32_t max_netf;   /* error-test failures in one step that fail the cell (0 = 7) */
  int32_t max_ncf;    /* Newton convergence failures in one step that fail the cell (0 = 10) */
} orc_opts;

typedef struct {
  int32_t status, nst, nfe, nni, nsetups, netf, ncfn, q_last;
  int32_t nli, ncfl; /* GMRES iterations, linear solves that did not converge */
  double h_last, t_reached;
} orc_stats;

/* Per-cell record of accepted steps, for the frozen replay / adjoint. */
typedef struct {
  int32_t cap, n;    /* capacity (steps) and number recorded */
  double h_pad;      /* value the step-size history was padded with */
  double *y;         /* [cap][S] accepted solutions y_n */
  double *h;         /* [cap] accepted step sizes h_n */
  int32_t *q;        /* [cap] order used for step n */
  int32_t *rebuild;  /* [cap] 1 if z was rebuilt at order 1 before step n */
} orc_record;

/* ------------------------------------------------------------------------ */
/* Kinetics: rates, right-hand side, analytic Jacobian                       */
/* ------------------------------------------------------------------------ */

/* Arrhenius rate constants k_f = exp(lnA - Ea/(R T)) * scale and, for
 * reversible reactions, k_r = k_f / K = k_f * exp(-lnK). */
void orc_rates(const orc_mech *m, double T, const double *kscale, double *kf, double *kr) {
  for (int r = 0; r < m->n_reactions; ++r) {
    double lk = m->lnA[r];
    if (m->EaR) lk -= m->EaR[r] / T;
    kf[r] = exp(lk);
    if (kscale) kf[r] *= kscale[r];
    kr[r] = m->lnK ? kf[r] * exp(-m->lnK[r]) : 0.0;
  }
}

/* Net rate of every reaction: q_r = k_f prod(y_reac) - k_r prod(y_prod). */
static void orc_reaction_rates(const orc_mech *m, const double *kf, const double *kr,
                               const double *y, double *qr) {
  for (int r = 0; r < m->n_reactions; ++r) {
    double fwd = kf[r], rev = kr[r];
    for (int s = 0; s < ORC_SLOTS; ++s) {
      int a = m->reac[r * ORC_SLOTS + s];
      int b = m->prod[r * ORC_SLOTS + s];
      if (a >= 0) fwd *= y[a];
      if (b >= 0) rev *= y[b];
    }
    qr[r] = fwd - rev;
  }
}

/* f = F + sum_r nu_r q_r (mass-action chemistry source term R plus forcing). */
void orc_rhs(const orc_mech *m, const double *kf, const double *kr, const double *F,
             const double *y, double *f) {
  double qr[4096];
  double *q = m->n_reactions <= 4096 ? qr : (double *)malloc(sizeof(double) * m->n_reactions);
  int S = m->n_species;
  for (int i = 0; i < S; ++i) f[i] = F ? F[i] : 0.0;
  orc_reaction_rates(m, kf, kr, y, q);
  for (int r = 0; r < m->n_reactions; ++r) {
    for (int s = 0; s < ORC_SLOTS; ++s) {
      int a = m->reac[r * ORC_SLOTS + s];
      int b = m->prod[r * ORC_SLOTS + s];
      if (a >= 0) f[a] -= q[r];
      if (b >= 0) f[b] += q[r];
    }
  }
  if (q != qr) free(q);
}

/* Analytic Jacobian J[i][j] = d f_i / d y_j (row-major S x S).
 * d(prod_l y_{a_l}) / d y_j = sum over slots l with a_l = j of the product of
 * the other slots. */
void orc_jac(const orc_mech *m, const double *kf, const double *kr, const double *y, double *J) {
  int S = m->n_species;
  memset(J, 0, sizeof(double) * S * S);
  for (int r = 0; r < m->n_reactions; ++r) {
    const int32_t *side[2] = {m->reac + r * ORC_SLOTS, m->prod + r * ORC_SLOTS};
    double kside[2] = {kf[r], -kr[r]}; /* q_r = kf*P_reac - kr*P_prod */
    for (int sd = 0; sd < 2; ++sd) {
      if (kside[sd] == 0.0) continue;
      for (int l = 0; l < ORC_SLOTS; ++l) {
        int j = side[sd][l];
        if (j < 0) continue;
        double d = kside[sd];
        for (int o = 0; o < ORC_SLOTS; ++o)
          if (o != l && side[sd][o] >= 0) d *= y[side[sd][o]];
        /* d = d q_r / d y_j contribution of slot l; distribute with nu */
        for (int s = 0; s < ORC_SLOTS; ++s) {
          int a = m->reac[r * ORC_SLOTS + s];
          int b = m->prod[r * ORC_SLOTS + s];
          if (a >= 0) J[a * S + j] -= d;
          if (b >= 0) J[b * S + j] += d;
        }
      }
    }
  }
}

/* Non-isothermal right-hand side: x = (y_0 .. y_{S-1}, T), f the same
 * length.  Rates at T = x[S]; species rates as in orc_rhs (forcing F[0..S-1]);
 * dT/dt = F[S] - N / D with N = sum_i u_i(T) f_i, D = sum_i cv_i y_i and
 * u_i(T) = u0_i + cv_i T (constant-volume adiabatic energy balance). */
void orc_rhs_thermal(const orc_mech *m, const double *kscale, const double *F, const double *x,
                     double *f) {
  int S = m->n_species;
  double kf[4096], kr[4096];
  double T = x[S];
  orc_rates(m, T, kscale, kf, kr);
  orc_rhs(m, kf, kr, F, x, f);
  double N = 0.0, D = 0.0;
  for (int i = 0; i < S; ++i) {
    N += (m->u0[i] + m->cv[i] * T) * f[i];
    D += m->cv[i] * x[i];
  }
  f[S] = (F ? F[S] : 0.0) - N / D;
}

/* Analytic Jacobian of orc_rhs_thermal, (S+1) x (S+1) row-major.
 *   species block: orc_jac at the rates of T;
 *   T column: d f_i / dT = sum_r nu_ir q_r EaR_r / T^2 (both rate constants
 *     carry the factor exp(-EaR_r / T));
 *   T row: d f_T / dy_j = -(sum_i u_i J_ij) / D + N cv_j / D^2,
 *          d f_T / dT = -(sum_i cv_i f_i + sum_i u_i J_iT) / D. */
void orc_jac_thermal(const orc_mech *m, const double *kscale, const double *F, const double *x,
                     double *J) {
  int S = m->n_species, n = S + 1;
  double kf[4096], kr[4096], Js[ORC_MAXS * ORC_MAXS], f[ORC_MAXS];
  double qr[4096];
  double T = x[S];
  orc_rates(m, T, kscale, kf, kr);
  orc_jac(m, kf, kr, x, Js);
  orc_rhs(m, kf, kr, F, x, f);
  memset(J, 0, sizeof(double) * n * n);
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) J[i * n + j] = Js[i * S + j];
  orc_reaction_rates(m, kf, kr, x, qr);
  for (int r = 0; r < m->n_reactions; ++r) {
    double dq = qr[r] * (m->EaR ? m->EaR[r] : 0.0) / (T * T);
    for (int s = 0; s < ORC_SLOTS; ++s) {
      int a = m->reac[r * ORC_SLOTS + s];
      int b = m->prod[r * ORC_SLOTS + s];
      if (a >= 0) J[a * n + S] -= dq;
      if (b >= 0) J[b * n + S] += dq;
    }
  }
  double N = 0.0, D = 0.0, cf = 0.0;
  for (int i = 0; i < S; ++i) {
    N += (m->u0[i] + m->cv[i] * T) * f[i];
    D += m->cv[i] * x[i];
    cf += m->cv[i] * f[i];
  }
  for (int j = 0; j <= S; ++j) {
    double uj = 0.0;
    for (int i = 0; i < S; ++i) uj += (m->u0[i] + m->cv[i] * T) * J[i * n + j];
    if (j < S)
      J[S * n + j] = -uj / D + N * m->cv[j] / (D * D);
    else
      J[S * n + S] = -(cf + uj) / D;
  }
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting (the dense direct solver of Sec. 4.1.4).   */
/* Ties in |pivot| go to the lowest original row index.                      */
/* ------------------------------------------------------------------------ */

/* Factor A (n x n, row-major) in place: P A = L U, unit lower L stored below
 * the diagonal.  perm[i] = original index of the row now at position i.
 * Returns 0, or k+1 if the pivot of column k is exactly zero. */
int32_t orc_lu_factor(int n, double *A, int32_t *perm) {
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = fabs(A[k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = fabs(A[i * n + k]);
      if (v > best || (v == best && perm[i] < perm[p])) {
        best = v;
        p = i;
      }
    }
    if (best == 0.0) return k + 1;
    if (p != k) {
      for (int j = 0; j < n; ++j) {
        double t = A[k * n + j];
        A[k * n + j] = A[p * n + j];
        A[p * n + j] = t;
      }
      int32_t t = perm[k];
      perm[k] = perm[p];
      perm[p] = t;
    }
    for (int i = k + 1; i < n; ++i) {
      double l = A[i * n + k] / A[k * n + k];
      A[i * n + k] = l;
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
    }
  }
  return 0;
}

/* Solve A x = b with the factors of orc_lu_factor; b is overwritten by x. */
void orc_lu_solve(int n, const double *LU, const int32_t *perm, double *b) {
  double y[ORC_MAXS];
  for (int i = 0; i < n; ++i) {
    double s = b[perm[i]];
    for (int j = 0; j < i; ++j) s -= LU[i * n + j] * y[j];
    y[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int j = i + 1; j < n; ++j) s -= LU[i * n + j] * b[j];
    b[i] = s / LU[i * n + i];
  }
}

/* Solve A^T x = b with the factors of A (P A = L U  =>  A^T = U^T L^T P). */
static void orc_lu_solve_transposed(int n, const double *LU, const int32_t *perm, double *b) {
  double w[ORC_MAXS];
  for (int i = 0; i < n; ++i) { /* U^T w = b */
    double s = b[i];
    for (int j = 0; j < i; ++j) s -= LU[j * n + i] * w[j];
    w[i] = s / LU[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) { /* L^T v = w */
    double s = w[i];
    for (int j = i + 1; j < n; ++j) s -= LU[j * n + i] * w[j];
    w[i] = s;
  }
  for (int i = 0; i < n; ++i) b[perm[i]] = w[i]; /* x = P^T v */
}

/* ------------------------------------------------------------------------ */
/* Norms and BDF coefficients                                               */
/* ------------------------------------------------------------------------ */

/* Weighted root-mean-square norm, Sec. 2, Eq. (3): sqrt(1/N sum (w_i v_i)^2). */
double orc_wrms(int n, const double *v, const double *w) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += (v[i] * w[i]) * (v[i] * w[i]);
  return sqrt(s / n);
}

/* Error weights of Sec. 2, Eq. (3): w_i = 1/(rtol |y_i| + atol_i), for n
 * entries that are consecutive cell states of S entries each (atol per entry
 * of a cell's state). */
static void orc_ewt(int n, int S, const double *y, const orc_opts *o, double *w) {
  for (int i = 0; i < n; ++i) {
    double a = o->atol_len == 1 ? o->atol[0] : o->atol[i % S];
    w[i] = 1.0 / (o->rtol * fabs(y[i]) + a);
  }
}

/* Coefficients of the variable-coefficient BDF of order q in Nordsieck form.
 * xi[i] = (t_n - t_{n-i}) / h_n for i = 1..q+1 (xi[0] unused).
 * l[j] = coefficient of x^j in Lambda(x) = prod_{i=1}^{q} (1 + x/xi_i), so the
 * corrected polynomial z + l e keeps interpolating the q past values.
 * The local error estimate is Cerr * e with Cerr = 1/(l_1 xi_{q+1}); for
 * constant steps this is 1/((q+1) H_q) (H_q the harmonic number). */
void orc_bdf_coeffs(int q, const double *xi, double *l, double *Cerr) {
  for (int j = 0; j <= ORC_QMAX + 1; ++j) l[j] = 0.0;
  l[0] = 1.0;
  for (int i = 1; i <= q; ++i)
    for (int j = i; j >= 1; --j) l[j] += l[j - 1] / xi[i];
  *Cerr = 1.0 / (l[1] * xi[q + 1]);
}

/* xi_i for a step of size h given accepted-step history hist[0] = h_{n-1},
 * hist[1] = h_{n-2}, ...: xi_1 = 1, xi_i = (h + hist[0] + ... + hist[i-2])/h. */
static void orc_xi(double h, const double *hist, int q, double *xi) {
  double sum = h;
  xi[1] = 1.0;
  for (int i = 2; i <= q + 1; ++i) {
    sum += hist[i - 2];
    xi[i] = sum / h;
  }
}

/* ------------------------------------------------------------------------ */
/* Nordsieck array operations.  z[j] = h^j y^(j) / j!, j = 0..q.              */
/* ------------------------------------------------------------------------ */

/* Predictor: z <- z * Pascal (Taylor shift by one step). */
static void orc_predict(int S, int q, double z[][ORC_MAXN]) {
  for (int k = 1; k <= q; ++k)
    for (int j = q; j >= k; --j)
      for (int i = 0; i < S; ++i) z[j - 1][i] += z[j][i];
}

/* Exact inverse of orc_predict (restore after a rejected attempt). */
static void orc_unpredict(int S, int q, double z[][ORC_MAXN]) {
  for (int k = 1; k <= q; ++k)
    for (int j = q; j >= k; --j)
      for (int i = 0; i < S; ++i) z[j - 1][i] -= z[j][i];
}

/* Change of step size h -> eta h: z_j <- eta^j z_j. */
static void orc_rescale(int S, int q, double eta, double z[][ORC_MAXN]) {
  double f = 1.0;
  for (int j = 1; j <= q; ++j) {
    f *= eta;
    for (int i = 0; i < S; ++i) z[j][i] *= f;
  }
}

/* Order q -> q+1 after an accepted step (reading of Sec. 2, "the method order
 * may be changed"): add (e/xi_{q+1}) x Lambda(x), the degree-(q+1) term that
 * makes z also interpolate the value the predictor interpolated at
 * t_{n-q-1}; l and xi are those of the step just accepted. */
static void orc_order_up(int S, int q, const double *l, const double *xi, const double *e,
                         double z[][ORC_MAXN]) {
  double c = 1.0 / xi[q + 1];
  for (int i = 0; i < S; ++i) z[q + 1][i] = 0.0;
  for (int j = 1; j <= q + 1; ++j)
    for (int i = 0; i < S; ++i) z[j][i] += c * l[j - 1] * e[i];
}

/* Order q -> q-1: subtract z_q x prod_{i=1}^{q-1} (x + xi_i), which removes
 * the x^q term and keeps interpolation at t_n, ..., t_{n-q+1}. */
static void orc_order_down(int S, int q, const double *xi, double z[][ORC_MAXN]) {
  double c[ORC_QMAX + 2];
  for (int j = 0; j <= q; ++j) c[j] = 0.0;
  c[1] = 1.0; /* polynomial x */
  for (int i = 1; i <= q - 1; ++i) /* multiply by (x + xi_i) */
    for (int j = i + 1; j >= 1; --j) c[j] = c[j - 1] + xi[i] * c[j];
  for (int j = 1; j < q; ++j)
    for (int i = 0; i < S; ++i) z[j][i] -= c[j] * z[q][i];
  for (int i = 0; i < S; ++i) z[q][i] = 0.0;
}

static double orc_harmonic(int k) {
  double s = 0.0;
  for (int i = 1; i <= k; ++i) s += 1.0 / i;
  return s;
}

static double orc_factorial(int k) {
  double s = 1.0;
  for (int i = 2; i <= k; ++i) s *= i;
  return s;
}

/* Local-error estimates of the neighbouring orders, used to choose the order
 * (Sec. 2: CVODE may change the method order after an accepted step; the
 * estimates are a reading, the paper gives none).  With constant steps the
 * local truncation error of the order-k BDF is h^{k+1} y^{(k+1)} / ((k+1) H_k),
 * H_k the harmonic number (the error constants 1/2, 2/9, 3/22, 12/125,
 * 10/137).
 *   order q-1: h^q y^{(q)} = q! z_q, so the estimate is (q-1)!/H_{q-1} ||z_q||;
 *   order q+1: each correction e is ~ h^{q+1} y^{(q+1)} times a constant, so
 *              the change e_n - (h_n/h_{n-1})^{q+1} e_{n-1} between successive
 *              steps is ~ h^{q+2} y^{(q+2)}; the estimate is its norm over
 *              (q+2) H_{q+1}.
 * Norms are the WRMS norm of Eq. (3) with weights ewt over n entries. */
double orc_lte_lower(int n, int q, const double *zq, const double *ewt) {
  return orc_factorial(q - 1) / orc_harmonic(q - 1) * orc_wrms(n, zq, ewt);
}

double orc_lte_higher(int n, int q, const double *e, const double *eprev, double h, double hprev,
                      const double *ewt) {
  double r = pow(h / hprev, q + 1), d[ORC_MAXN];
  for (int i = 0; i < n; ++i) d[i] = e[i] - r * eprev[i];
  return orc_wrms(n, d, ewt) / ((q + 2) * orc_harmonic(q + 1));
}

static int orc_all_finite(int n, const double *v) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Per-cell adaptive integration                                            */
/* ------------------------------------------------------------------------ */

/* The system one integration advances: one cell, or nb cells of the same
 * mechanism in lock step (their states concatenated, cell b at entries
 * [b S, (b+1) S); rates of cell b at kf + b R, kr + b R; forcing at F + b S;
 * non-isothermal rate scales at kscale + b R). */
typedef struct {
  const orc_mech *m;
  const double *kf, *kr, *F;
  int S;                 /* state length of a cell: species, plus 1 for a non-isothermal cell */
  const double *kscale;  /* non-isothermal: per-reaction scale for the rates at T */
  int nb;                /* cells (1 unless integrated in lock step) */
} orc_sys;

static int sys_thermal(const orc_sys *s) { return s->m->cv != NULL; }

static void sys_f(const orc_sys *s, const double *y, double *f) {
  const int S = s->S, R = s->m->n_reactions;
  for (int b = 0; b < s->nb; ++b) {
    const double *F = s->F ? s->F + b * S : NULL;
    if (sys_thermal(s))
      orc_rhs_thermal(s->m, s->kscale ? s->kscale + b * R : NULL, F, y + b * S, f + b * S);
    else
      orc_rhs(s->m, s->kf + b * R, s->kr + b * R, F, y + b * S, f + b * S);
  }
}

/* Jacobian blocks: J + b S S is the S x S Jacobian of cell b (the system's
 * Jacobian is block diagonal). */
static void sys_jac(const orc_sys *s, const double *y, double *J) {
  const int S = s->S, R = s->m->n_reactions;
  for (int b = 0; b < s->nb; ++b) {
    const double *F = s->F ? s->F + b * S : NULL;
    if (sys_thermal(s))
      orc_jac_thermal(s->m, s->kscale ? s->kscale + b * R : NULL, F, y + b * S, J + b * S * S);
    else
      orc_jac(s->m, s->kf + b * R, s->kr + b * R, y + b * S, J + b * S * S);
  }
}

/* Initial step size (reading; the paper is silent).  Bounds
 * h_lb = 100 u max(|t0|, |t_out|), h_ub = min(0.1 |t_out - t0|,
 * 1 / max_i(|f0_i| / (0.1 |y0_i| + atol_i))); then up to four refinements
 * of h = sqrt(2 / ||y''||) with y'' ~ (f(y0 + h f0) - f0)/h, stopping when the
 * new value is within a factor 2 of the previous; h0 = 0.5 h clamped to
 * [h_lb, h_ub] (h_ub if y'' vanishes). */
static double orc_initial_step(const orc_sys *s, const orc_opts *o, double t0, double tout,
                               const double *y0, const double *f0, const double *ewt, int *nfe) {
  int S = s->S, n = s->S * s->nb;
  double tdist = fabs(tout - t0);
  double hlb = 100.0 * ORC_UROUND * fmax(fabs(t0), fabs(tout));
  double hub = 0.1 * tdist;
  double hub_inv = 0.0;
  for (int i = 0; i < n; ++i) {
    double a = o->atol_len == 1 ? o->atol[0] : o->atol[i % S];
    double v = fabs(f0[i]) / (0.1 * fabs(y0[i]) + a);
    if (v > hub_inv) hub_inv = v;
  }
  if (hub * hub_inv > 1.0) hub = 1.0 / hub_inv;
  if (hub < hlb) return hub;
  double hg = sqrt(hlb * hub), hnew = hg;
  double ytmp[ORC_MAXN], ftmp[ORC_MAXN], ydd[ORC_MAXN];
  for (int it = 0; it < 4; ++it) {
    for (int i = 0; i < n; ++i) ytmp[i] = y0[i] + hg * f0[i];
    sys_f(s, ytmp, ftmp);
    (*nfe)++;
    for (int i = 0; i < n; ++i) ydd[i] = (ftmp[i] - f0[i]) / hg;
    double yddnrm = orc_wrms(n, ydd, ewt);
    if (!(yddnrm > 0.0)) return hub;
    hnew = sqrt(2.0 / yddnrm);
    double ratio = hnew / hg;
    hg = hnew;
    if (ratio >= 0.5 && ratio <= 2.0) break;
  }
  double h0 = 0.5 * hnew;
  if (h0 < hlb) h0 = hlb;
  if (h0 > hub) h0 = hub;
  return h0;
}

/* Jacobian by forward difference quotients, one right-hand side per column
 * (Table 1, approaches 3A/3B; the increments follow the dense
 * difference-quotient scheme documented for CVODE): with f0 = f(y),
 * ||f0|| its WRMS norm under the weights w and u the unit round-off,
 *   min_inc = 1000 |h| u n ||f0||  (1 if ||f0|| = 0),
 *   inc_j   = max(sqrt(u) |y_j|, min_inc / w_j),
 *   J[i][j] = (f_i(y + inc_j e_j) - f0_i) / inc_j.
 * Adds n + 1 right-hand sides to *nfe. */
static void orc_jac_dq(const orc_sys *s, const double *y, const double *ewt, double h, double *J,
                       int32_t *nfe) {
  const int n = s->S;
  double f0[ORC_MAXS], f1[ORC_MAXS], yp[ORC_MAXS];
  sys_f(s, y, f0);
  (*nfe)++;
  double fnorm = orc_wrms(n, f0, ewt);
  double min_inc = fnorm != 0.0 ? 1000.0 * fabs(h) * ORC_UROUND * n * fnorm : 1.0;
  double srur = sqrt(ORC_UROUND);
  for (int j = 0; j < n; ++j) {
    double inc = fmax(srur * fabs(y[j]), min_inc / ewt[j]);
    for (int i = 0; i < n; ++i) yp[i] = y[i];
    yp[j] = y[j] + inc;
    sys_f(s, yp, f1);
    (*nfe)++;
    for (int i = 0; i < n; ++i) J[i * n + j] = (f1[i] - f0[i]) / inc;
  }
}

/* Test hook: the difference-quotient Jacobian of one cell at y (rates from T
 * and kscale for an isothermal mechanism; from y's temperature otherwise). */
void orc_jacobian_dq(const orc_mech *m, double T, const double *kscale, const double *F,
                     const double *y, const double *ewt, double h, double *J) {
  double kf[4096], kr[4096];
  const int thermal = m->cv != NULL;
  if (!thermal) orc_rates(m, T, kscale, kf, kr);
  orc_sys s = {m, kf, kr, F, m->n_species + thermal, kscale, 1};
  int32_t nfe = 0;
  orc_jac_dq(&s, y, ewt, h, J, &nfe);
}

/* Linear solve of the inexact Newton iteration (Table 1, approaches 1A/1B):
 * GMRES on the scaled system of Sec. 2, Eq. (5), with S1 = S2 =
 * diag(w) and no preconditioner (P1 = P2 = I), for A = I - gamma J(y), b.
 * A is applied without forming J: the product J v is the difference quotient
 * (f(y + sigma v) - f(y)) / sigma with sigma = 1 / ||v||_wrms and fy = f(y).
 * The initial guess is 0; the Arnoldi basis is orthogonalised by modified
 * Gram-Schmidt; Givens rotations turn the Hessenberg matrix into triangular
 * form and give the residual norm of the scaled system as the magnitude of
 * the last rotated right-hand-side entry, without forming the residual
 * (Sec. 2, after Eq. (6); Saad, Iterative Methods for Sparse
 * Linear Systems, Sec. 6.5).  Iteration stops at maxl basis vectors or when
 * that residual norm is at most delta (Eq. (6); delta is passed in
 * the 2-norm of the scaled system).  Returns 0 when converged, 1 when the
 * residual was reduced but not to delta, 2 otherwise; x receives the
 * solution of the unscaled system.  *nli counts iterations (one product J v,
 * hence one right-hand side each), *rho_out the final residual norm. */
static int orc_gmres(const orc_sys *s, const double *y, const double *fy, const double *ewt,
                     double gamma, int maxl, double delta, const double *b, double *x,
                     int32_t *nli, double *rho_out) {
  const int n = s->S;
  double V[ORC_GMRES_MAXL + 1][ORC_MAXS];
  double H[ORC_GMRES_MAXL + 1][ORC_GMRES_MAXL];
  double cs[ORC_GMRES_MAXL], sn[ORC_GMRES_MAXL], g[ORC_GMRES_MAXL + 1], c[ORC_GMRES_MAXL];
  double v[ORC_MAXS], yp[ORC_MAXS], fp[ORC_MAXS], w[ORC_MAXS];
  if (maxl > ORC_GMRES_MAXL) maxl = ORC_GMRES_MAXL;

  for (int i = 0; i < n; ++i) x[i] = 0.0;
  /* residual of the initial guess 0 in the scaled system: b~ = S1 b */
  double beta = 0.0;
  for (int i = 0; i < n; ++i) {
    V[0][i] = ewt[i] * b[i];
    beta += V[0][i] * V[0][i];
  }
  beta = sqrt(beta);
  *rho_out = beta;
  if (beta <= delta) return 0;
  for (int i = 0; i < n; ++i) V[0][i] /= beta;
  g[0] = beta;

  int k = 0; /* columns of the triangular system */
  double rho = beta;
  for (int l = 0; l < maxl; ++l) {
    /* w = A~ V_l = S1 (v - gamma J v), v = S2^{-1} V_l */
    for (int i = 0; i < n; ++i) v[i] = V[l][i] / ewt[i];
    double sigma = 1.0 / orc_wrms(n, v, ewt);
    for (int i = 0; i < n; ++i) yp[i] = y[i] + sigma * v[i];
    sys_f(s, yp, fp);
    (*nli)++;
    for (int i = 0; i < n; ++i) w[i] = ewt[i] * (v[i] - gamma * ((fp[i] - fy[i]) / sigma));
    /* modified Gram-Schmidt against V_0..V_l */
    for (int j = 0; j <= l; ++j) {
      double d = 0.0;
      for (int i = 0; i < n; ++i) d += w[i] * V[j][i];
      H[j][l] = d;
      for (int i = 0; i < n; ++i) w[i] -= d * V[j][i];
    }
    double hn = 0.0;
    for (int i = 0; i < n; ++i) hn += w[i] * w[i];
    hn = sqrt(hn);
    H[l + 1][l] = hn;
    /* earlier rotations, then the one that zeroes H[l+1][l] */
    for (int j = 0; j < l; ++j) {
      double a0 = H[j][l], a1 = H[j + 1][l];
      H[j][l] = cs[j] * a0 + sn[j] * a1;
      H[j + 1][l] = -sn[j] * a0 + cs[j] * a1;
    }
    double r = hypot(H[l][l], H[l + 1][l]);
    if (!(r > 0.0)) break; /* singular Hessenberg column: stop with k columns */
    cs[l] = H[l][l] / r;
    sn[l] = H[l + 1][l] / r;
    H[l][l] = r;
    H[l + 1][l] = 0.0;
    g[l + 1] = -sn[l] * g[l];
    g[l] = cs[l] * g[l];
    rho = fabs(g[l + 1]);
    k = l + 1;
    if (rho <= delta) break;
    if (l + 1 < maxl) {
      if (!(hn > 0.0)) break;
      for (int i = 0; i < n; ++i) V[l + 1][i] = w[i] / hn;
    }
  }
  *rho_out = rho;
  /* back substitution for the coefficients, x = S2^{-1} sum_j c_j V_j */
  for (int i = k - 1; i >= 0; --i) {
    double t = g[i];
    for (int j = i + 1; j < k; ++j) t -= H[i][j] * c[j];
    c[i] = t / H[i][i];
  }
  for (int i = 0; i < n; ++i) {
    double t = 0.0;
    for (int j = 0; j < k; ++j) t += c[j] * V[j][i];
    x[i] = t / ewt[i];
  }
  if (rho <= delta) return 0;
  return rho < beta ? 1 : 2;
}

/* Test hook: one GMRES solve of (I - gamma J(y)) x = b for one cell (rates
 * as in orc_jacobian_dq); returns orc_gmres's code, *nli and *rho. */
int32_t orc_gmres_solve(const orc_mech *m, double T, const double *kscale, const double *F,
                        const double *y, const double *ewt, double gamma, int32_t maxl,
                        double delta, const double *b, double *x, int32_t *nli, double *rho) {
  double kf[4096], kr[4096], fy[ORC_MAXS];
  const int thermal = m->cv != NULL;
  if (!thermal) orc_rates(m, T, kscale, kf, kr);
  orc_sys s = {m, kf, kr, F, m->n_species + thermal, kscale, 1};
  sys_f(&s, y, fy);
  *nli = 0;
  return orc_gmres(&s, y, fy, ewt, gamma, maxl, delta, b, x, nli, rho);
}

/* eta = 1 / ((bias * err)^(1/p) + 1e-6): step ratio that would bring an
 * error estimate err of an order-(p-1) method to 1/bias. */
static double orc_eta(double bias, double err, int p) {
  return 1.0 / (pow(bias * err, 1.0 / p) + 1.0e-6);
}

/* Integrate one cell from t0 to tout.  y (length S) is the initial state on
 * entry and the final state (or the last accepted state on failure) on exit.
 *
 * Step loop (Sec. 2): weights from y^{n-1} (Eq. (3)); predict; Newton on
 * G(e) = e - gamma f(z_0 + e) + z_1/l_1 with M = I - gamma J (modified
 * Newton, Sec. 3.1), stopped by Eq. (4) with c_eps = 0.1, c_r = 0.3 and
 * eps = 1/Cerr; accept when Cerr ||e|| <= 1, otherwise cut h (and possibly
 * the order) and retry; after acceptance choose the next h and q.
 *
 * Readings where the paper is silent: at most 3 Newton iterations,
 * divergence when ||delta_m|| > 2 ||delta_{m-1}||; the convergence rate R
 * persists across steps and is reset to 1 at every setup; the Newton matrix
 * is rebuilt (fresh J) on the first step, 20 steps after the last setup,
 * when |gamma/gamma_setup - 1| > 0.3 and after a convergence failure with a
 * stale matrix; when gamma differs from the factored one, delta is scaled by
 * 2/(1 + gamma/gamma_setup).  Convergence failure with a fresh matrix cuts
 * h by 4; 10 in one step (o->max_ncf) fail the cell (-4).  Error-test
 * failure: 7 in one step (o->max_netf) fail the cell (-3), which keeps its
 * last accepted state and time; from the third, restart at order 1 from y with
 * eta = 0.1; otherwise eta = max(0.1, eta_q) and eta <= 0.2 from the second.
 * After every accepted step the next step size is chosen (Sec. 2) from
 * eta_q (bias 6); the order is reconsidered only when qwait reaches 0
 * (qwait = q+1 after an order change, 2 at the start, after a restart and
 * after each order decision), adding candidates eta_{q-1} (bias 6) and
 * eta_{q+1} (bias 10, from the difference of successive corrections); the
 * largest wins, ties going to q then q-1.  Ratios below 1.5 change
 * nothing; growth is capped by eta_max (1e4 on the first step, 10
 * afterwards); right after a failure h and q are held for that step.
 * The last step is clipped to land on tout exactly.
 *
 * With o->gmres_maxl > 0 (Table 1, approaches 1A/1B) each Newton system is
 * solved by orc_gmres at the current iterate (inexact Newton): no Jacobian
 * or Newton matrix is formed, so there are no setups and no gamma-ratio
 * scaling.  A linear solve that does not reach its tolerance ends the Newton
 * iteration as a convergence failure (a reduced residual is accepted on the
 * first Newton iteration), which always cuts h by 4.  Right-hand sides of the
 * products J v count in nfe.
 */
static int32_t orc_integrate_core(const orc_sys *s, const orc_opts *o, double t0, double tout,
                                  double *y, orc_stats *st, orc_record *rec, double *zout) {
  const int S = s->S, n = s->S * s->nb; /* entries per cell, entries of the system */
  const int qmax = o->max_order < 1 ? 1 : (o->max_order > ORC_QMAX ? ORC_QMAX : o->max_order);
  const int krylov = o->gmres_maxl > 0;
  const int max_netf = o->max_netf > 0 ? o->max_netf : 7;
  const int max_ncf = o->max_ncf > 0 ? o->max_ncf : 10;
  double z[ORC_QMAX + 2][ORC_MAXN];
  double ewt[ORC_MAXN], e[ORC_MAXN], eprev[ORC_MAXN], ycur[ORC_MAXN], f[ORC_MAXN], G[ORC_MAXN];
  double delta[ORC_MAXN];
  int32_t perm[ORC_MAXN];
  double hist[ORC_QMAX + 1];
  double xi[ORC_QMAX + 2], l[ORC_QMAX + 2], Cerr = 0.5;

  memset(st, 0, sizeof(*st));
  st->t_reached = t0;
  if (rec) rec->n = 0;
  if (!orc_all_finite(n, y)) {
    st->status = ORC_NONFINITE;
    return st->status;
  }
  for (int j = 0; j <= ORC_QMAX + 1; ++j)
    for (int i = 0; i < ORC_MAXN; ++i) z[j][i] = 0.0;

  double t = t0;
  int q = 1;
  for (int i = 0; i < n; ++i) z[0][i] = y[i];
  sys_f(s, y, f);
  st->nfe = 1;
  if (!orc_all_finite(n, f)) {
    st->status = ORC_NONFINITE;
    return st->status;
  }
  orc_ewt(n, S, y, o, ewt);
  double h = orc_initial_step(s, o, t0, tout, y, f, ewt, &st->nfe);
  for (int i = 0; i < n; ++i) z[1][i] = h * f[i];
  for (int k = 0; k <= ORC_QMAX; ++k) hist[k] = h;
  if (rec) rec->h_pad = h;

  /* Jacobian and Newton-matrix blocks, one S x S block per cell */
  double *J = malloc(sizeof(double) * (size_t)s->nb * S * S);
  double *M = malloc(sizeof(double) * (size_t)s->nb * S * S);
  int qwait = 2;
  double Rrate = 1.0, eta_max = 1.0e4, gamma_bar = 0.0;
  int need_setup = 1, nst_setup = 0, have_eprev = 0, rebuilt = 0;
  double hprev = h;
  int status = ORC_SUCCESS;

  while (t < tout) {
    if (st->nst >= o->max_steps) {
      status = ORC_TOO_MUCH_WORK;
      break;
    }
    if (rec && rec->n >= rec->cap) {
      /* the record is full and time is left: stop at the last recorded step,
       * so that the returned state is the end point of the recorded map */
      status = ORC_RECORD_FULL;
      break;
    }
    orc_ewt(n, S, z[0], o, ewt); /* from y^{n-1}, held through retries */
    int nef_step = 0, ncf_step = 0, nsf_step = 0;
    double dsm = 0.0, tn = t, gamma = h;
    int accepted = 0;
    while (!accepted) {
      /* land exactly on tout */
      int landing = 0;
      if (t + h >= tout * (1.0 - 4.0 * ORC_UROUND)) {
        double hnew = tout - t;
        orc_rescale(n, q, hnew / h, z);
        h = hnew;
        landing = 1;
      }
      if (h <= 4.0 * ORC_UROUND * fabs(t)) {
        status = ORC_ERR_FAILURE; /* step too small to advance t */
        break;
      }
      tn = landing ? tout : t + h;
      orc_predict(n, q, z);
      orc_xi(h, hist, q, xi);
      orc_bdf_coeffs(q, xi, l, &Cerr);
      gamma = h / l[1];

      int fresh = 0;
      if (!krylov &&
          (need_setup || st->nst >= nst_setup + 20 || fabs(gamma / gamma_bar - 1.0) > 0.3)) {
        if (o->jac_dq)
          orc_jac_dq(s, z[0], ewt, h, J, &st->nfe);
        else
          sys_jac(s, z[0], J);
        /* block b of M = I - gamma J is cell b's S x S Newton matrix */
        for (int b = 0; b < s->nb; ++b)
          for (int i = 0; i < S; ++i)
            for (int j = 0; j < S; ++j)
              M[(b * S + i) * S + j] = (i == j ? 1.0 : 0.0) - gamma * J[(b * S + i) * S + j];
        st->nsetups++;
        nst_setup = st->nst;
        gamma_bar = gamma;
        Rrate = 1.0;
        need_setup = 0;
        fresh = 1;
        int singular = 0;
        for (int b = 0; b < s->nb; ++b)
          if (orc_lu_factor(S, M + b * S * S, perm + b * S) != 0) singular = 1;
        if (singular) {
          /* singular Newton matrix: recoverable once per step by cutting h */
          orc_unpredict(n, q, z);
          need_setup = 1;
          if (++nsf_step >= 2) {
            status = ORC_SETUP_FAILURE;
            break;
          }
          orc_rescale(n, q, 0.25, z);
          h *= 0.25;
          eta_max = 1.0;
          continue;
        }
      }

      /* Newton iteration, stopping test of Eq. (4) */
      int conv = 0;
      double dprev = 0.0;
      for (int i = 0; i < n; ++i) e[i] = 0.0;
      for (int mit = 0; mit < 3; ++mit) {
        for (int i = 0; i < n; ++i) ycur[i] = z[0][i] + e[i];
        sys_f(s, ycur, f);
        st->nfe++;
        st->nni++;
        for (int i = 0; i < n; ++i) G[i] = e[i] - gamma * f[i] + z[1][i] / l[1];
        for (int i = 0; i < n; ++i) delta[i] = -G[i];
        if (krylov) {
          /* inexact Newton: J at the current iterate, Eq. (6) with
           * c_l = 0.05 on the Newton tolerance c_eps eps = 0.1 / Cerr, in
           * WRMS units (the scaled 2-norm is sqrt(S) times the WRMS norm) */
          double rhs_b[ORC_MAXN], rho;
          for (int i = 0; i < n; ++i) rhs_b[i] = delta[i];
          int32_t nli = 0;
          int lret = orc_gmres(s, ycur, f, ewt, gamma, o->gmres_maxl, 0.05 * (0.1 / Cerr) * sqrt(n),
                               rhs_b, delta, &nli, &rho);
          st->nli += nli;
          st->nfe += nli;
          /* a reduced but unconverged residual is accepted on the first
           * iteration only */
          if (lret != 0) st->ncfl++;
          if (lret == 2 || (lret == 1 && mit > 0)) break;
        } else {
          for (int b = 0; b < s->nb; ++b)
            orc_lu_solve(S, M + b * S * S, perm + b * S, delta + b * S);
        }
        if (!krylov && gamma != gamma_bar) {
          double c = 2.0 / (1.0 + gamma / gamma_bar);
          for (int i = 0; i < n; ++i) delta[i] *= c;
        }
        for (int i = 0; i < n; ++i) e[i] += delta[i];
        double d = orc_wrms(n, delta, ewt);
        if (!isfinite(d)) break;
        if (mit >= 1) {
          double ratio = d / dprev;
          Rrate = 0.3 * Rrate > ratio ? 0.3 * Rrate : ratio;
        }
        if ((Rrate < 1.0 ? Rrate : 1.0) * d <= 0.1 / Cerr) {
          conv = 1;
          break;
        }
        if (mit >= 1 && d > 2.0 * dprev) break;
        dprev = d;
      }

      if (!conv) {
        st->ncfn++;
        orc_unpredict(n, q, z);
        if (++ncf_step >= max_ncf) {
          status = ORC_CONV_FAILURE;
          break;
        }
        if (fresh || krylov) {
          orc_rescale(n, q, 0.25, z);
          h *= 0.25;
          eta_max = 1.0;
        }
        need_setup = 1;
        continue;
      }

      /* local error test, ||LTE|| <= 1 (Sec. 2) */
      dsm = Cerr * orc_wrms(n, e, ewt);
      if (!(dsm <= 1.0)) {
        st->netf++;
        orc_unpredict(n, q, z);
        if (++nef_step >= max_netf) {
          status = ORC_ERR_FAILURE;
          break;
        }
        eta_max = 1.0;
        if (nef_step >= 3) {
          /* restart at order 1 from the last accepted y */
          double hnew = 0.1 * h;
          q = 1;
          sys_f(s, z[0], f);
          st->nfe++;
          for (int j = 1; j <= ORC_QMAX + 1; ++j)
            for (int i = 0; i < n; ++i) z[j][i] = 0.0;
          for (int i = 0; i < n; ++i) z[1][i] = hnew * f[i];
          h = hnew;
          qwait = 2;
          have_eprev = 0;
          rebuilt = 1;
        } else {
          double eta = orc_eta(6.0, dsm, q + 1);
          if (eta < 0.1) eta = 0.1;
          if (nef_step >= 2 && eta > 0.2) eta = 0.2;
          orc_rescale(n, q, eta, z);
          h *= eta;
        }
        continue;
      }
      accepted = 1;
    }
    if (status != ORC_SUCCESS) break;

    /* accept: correct the Nordsieck array */
    t = tn;
    for (int j = 0; j <= q; ++j)
      for (int i = 0; i < n; ++i) z[j][i] += l[j] * e[i];
    st->nst++;
    for (int k = ORC_QMAX; k >= 1; --k) hist[k] = hist[k - 1];
    hist[0] = h;
    if (rec) {
      for (int i = 0; i < n; ++i) rec->y[(size_t)rec->n * S + i] = z[0][i];
      rec->h[rec->n] = h;
      rec->q[rec->n] = q;
      rec->rebuild[rec->n] = rebuilt;
      rec->n++;
    }
    rebuilt = 0;
    double hstep = h;
    qwait--;
    if (qwait == 1 && q < qmax) {
      for (int i = 0; i < n; ++i) eprev[i] = e[i];
      hprev = hstep;
      have_eprev = 1;
    }

    /* next step size (every accepted step) and order (when qwait reaches 0) */
    if (t < tout) {
      if (eta_max == 1.0) {
        if (qwait < 2) qwait = 2; /* right after a failure: hold h and q */
      } else {
        double eta = orc_eta(6.0, dsm, q + 1);
        int qnew = q;
        if (qwait == 0) {
          qwait = 2;
          if (q > 1) {
            double eta_qm1 = orc_eta(6.0, orc_lte_lower(n, q, z[q], ewt), q);
            if (eta_qm1 > eta) {
              eta = eta_qm1;
              qnew = q - 1;
            }
          }
          if (q < qmax && have_eprev) {
            double lte = orc_lte_higher(n, q, e, eprev, hstep, hprev, ewt);
            double eta_qp1 = orc_eta(10.0, lte, q + 2);
            if (eta_qp1 > eta) {
              eta = eta_qp1;
              qnew = q + 1;
            }
          }
        }
        if (eta >= 1.5) {
          if (eta > eta_max) eta = eta_max;
          if (qnew == q + 1) orc_order_up(n, q, l, xi, e, z);
          if (qnew == q - 1) orc_order_down(n, q, xi, z);
          if (qnew != q) {
            q = qnew;
            qwait = q + 1;
            have_eprev = 0;
          }
          orc_rescale(n, q, eta, z);
          h *= eta;
        }
      }
    }
    eta_max = 10.0;
  }

  free(J);
  free(M);
  for (int i = 0; i < n; ++i) y[i] = z[0][i];
  if (zout)
    for (int j = 0; j <= ORC_QMAX; ++j)
      for (int i = 0; i < n; ++i) zout[j * S + i] = j <= q ? z[j][i] : 0.0;
  st->status = status;
  st->q_last = q;
  st->h_last = h;
  st->t_reached = t;
  return status;
}

/* One cell: rates from T (and optional per-reaction scale), then integrate. */
int32_t orc_integrate_cell(const orc_mech *m, const orc_opts *o, double T, const double *kscale,
                           const double *F, double t0, double tout, double *y, orc_stats *st,
                           orc_record *rec, double *zout) {
  double kf[4096], kr[4096];
  if (m->n_reactions > 4096 || m->n_species > ORC_MAXS) {
    memset(st, 0, sizeof(*st));
    st->status = ORC_NONFINITE;
    return st->status;
  }
  const int thermal = m->cv != NULL;
  if (thermal) {
    if (m->n_species + 1 > ORC_MAXS) {
      memset(st, 0, sizeof(*st));
      st->status = ORC_NONFINITE;
      return st->status;
    }
    T = y[m->n_species];  /* temperature is the last state component */
  } else {
    orc_rates(m, T, kscale, kf, kr);
  }
  orc_sys s = {m, kf, kr, F, m->n_species + thermal, kscale, 1};
  if (!isfinite(T)) {
    memset(st, 0, sizeof(*st));
    st->t_reached = t0;
    st->status = ORC_NONFINITE;
    return st->status;
  }
  return orc_integrate_core(&s, o, t0, tout, y, st, rec, zout);
}

/* Initial step size of one cell, as orc_integrate_cell would choose it
 * (test hook for orc_initial_step): rates from T and kscale, f0 = f(y0),
 * weights of Eq. (3) at y0.  *nfe receives the right-hand sides used
 * (1 for f0 plus the refinements).  Returns 0 for input the integrator
 * would reject as non-finite. */
double orc_initial_step_cell(const orc_mech *m, const orc_opts *o, double T, const double *kscale,
                             const double *F, double t0, double tout, const double *y0,
                             int32_t *nfe) {
  double kf[4096], kr[4096], f0[ORC_MAXS], ewt[ORC_MAXS];
  const int thermal = m->cv != NULL;
  const int n = m->n_species + thermal;
  *nfe = 0;
  if (m->n_reactions > 4096 || n > ORC_MAXS) return 0.0;
  if (thermal)
    T = y0[m->n_species];
  else
    orc_rates(m, T, kscale, kf, kr);
  if (!isfinite(T) || !orc_all_finite(n, y0)) return 0.0;
  orc_sys s = {m, kf, kr, F, n, kscale, 1};
  sys_f(&s, y0, f0);
  *nfe = 1;
  if (!orc_all_finite(n, f0)) return 0.0;
  orc_ewt(n, n, y0, o, ewt);
  int32_t extra = 0;
  double h0 = orc_initial_step(&s, o, t0, tout, y0, f0, ewt, &extra);
  *nfe += extra;
  return h0;
}

/* Batch of N cells (each one independent), OpenMP over cells.  y is [N][ldy]
 * (cell-major), the cell's mechanism is mechs[cell_mech[c]] (cell_mech NULL
 * = mechanism 0); T [N] (NULL: T = 1, use with zero activation energies),
 * kscale [N][ldk] or NULL, F [N][ldy] or NULL. */
void orc_integrate_batch(int64_t N, const orc_mech *mechs, const int32_t *cell_mech,
                         const orc_opts *o, const double *T, const double *kscale, int32_t ldk,
                         const double *F, int32_t ldy, double t0, double tout, double *y,
                         orc_stats *stats, int32_t nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t c = 0; c < N; ++c) {
    const orc_mech *m = &mechs[cell_mech ? cell_mech[c] : 0];
    orc_integrate_cell(m, o, T ? T[c] : 1.0, kscale ? kscale + c * ldk : NULL,
                       F ? F + c * ldy : NULL, t0, tout, y + c * ldy, &stats[c], NULL, NULL);
  }
}

/* Cells integrated in lock step (the paper's batches, Sec. 2: all cells of
 * a batch share one integrator, so the step size is the one the stiffest
 * cell allows): the nb cells cells[0..nb-1] of mechanism m form one system
 * of nb S entries -- one step size and order, one WRMS norm over all nb S
 * entries (N = nb S in Eq. (3)), one Newton iteration whose matrix is block
 * diagonal with one S x S block per cell (each block is factored on its own:
 * partial pivoting on the whole matrix picks the same pivots, the entries
 * outside a block being zero).  The batch succeeds or fails as a whole and
 * every cell of it receives the batch's statistics.  Direct solver with the
 * analytic Jacobian only.  T, kscale, F and y are the arrays of
 * orc_integrate_batch.  Returns the batch status.  Arguments outside these
 * limits (or a mechanism too large for the oracle, as in
 * orc_integrate_cell) give every cell of the batch status ORC_NONFINITE
 * with y unchanged. */
int32_t orc_integrate_lockstep(const orc_mech *m, const orc_opts *o, int32_t nb,
                               const int64_t *cells, const double *T, const double *kscale,
                               int32_t ldk, const double *F, int32_t ldy, double t0, double tout,
                               double *y, orc_stats *stats) {
  const int thermal = m->cv != NULL;
  const int S = m->n_species + thermal, R = m->n_reactions;
  if (nb < 1 || nb > ORC_MAXB || S > ORC_MAXS || R > 4096 || o->jac_dq || o->gmres_maxl > 0) {
    for (int b = 0; b < nb; ++b) {
      memset(&stats[cells[b]], 0, sizeof(orc_stats));
      stats[cells[b]].t_reached = t0;
      stats[cells[b]].status = ORC_NONFINITE;
    }
    return ORC_NONFINITE;
  }
  double *yb = malloc(sizeof(double) * (size_t)nb * S);
  double *kf = malloc(sizeof(double) * (size_t)nb * R);
  double *kr = malloc(sizeof(double) * (size_t)nb * R);
  double *Fb = F ? malloc(sizeof(double) * (size_t)nb * S) : NULL;
  double *ks = (thermal && kscale) ? malloc(sizeof(double) * (size_t)nb * R) : NULL;
  int finite = 1;
  for (int b = 0; b < nb; ++b) {
    const int64_t c = cells[b];
    for (int i = 0; i < S; ++i) yb[b * S + i] = y[c * ldy + i];
    if (Fb)
      for (int i = 0; i < S; ++i) Fb[b * S + i] = F[c * ldy + i];
    if (thermal) {
      if (ks)
        for (int r = 0; r < R; ++r) ks[b * R + r] = kscale[c * ldk + r];
    } else {
      const double Tc = T ? T[c] : 1.0;
      if (!isfinite(Tc)) finite = 0;
      orc_rates(m, Tc, kscale ? kscale + c * ldk : NULL, kf + b * R, kr + b * R);
    }
  }
  orc_sys s = {m, kf, kr, Fb, S, ks, nb};
  orc_stats st;
  if (finite) {
    orc_integrate_core(&s, o, t0, tout, yb, &st, NULL, NULL);
  } else {
    memset(&st, 0, sizeof(st));
    st.t_reached = t0;
    st.status = ORC_NONFINITE;
  }
  for (int b = 0; b < nb; ++b) {
    const int64_t c = cells[b];
    for (int i = 0; i < S; ++i) y[c * ldy + i] = yb[b * S + i];
    stats[c] = st;
  }
  free(yb);
  free(kf);
  free(kr);
  free(Fb);
  free(ks);
  return st.status;
}

/* All cells in lock-step batches of `batch` cells: the cells of each
 * mechanism, in increasing index order, are cut into consecutive batches
 * (the last one may be shorter); OpenMP over the batches of a mechanism.
 * Arguments as orc_integrate_batch, plus the number of mechanisms. */
void orc_integrate_lockstep_batch(int64_t N, int32_t batch, int32_t n_mech,
                                  const orc_mech *mechs, const int32_t *cell_mech,
                                  const orc_opts *o, const double *T, const double *kscale,
                                  int32_t ldk, const double *F, int32_t ldy, double t0,
                                  double tout, double *y, orc_stats *stats, int32_t nthreads) {
  int64_t *list = malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  for (int32_t mm = 0; mm < n_mech; ++mm) {
    int64_t cnt = 0;
    for (int64_t c = 0; c < N; ++c)
      if ((cell_mech ? cell_mech[c] : 0) == mm) list[cnt++] = c;
    const int64_t nbatches = (cnt + batch - 1) / batch;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t k = 0; k < nbatches; ++k) {
      const int64_t first = k * batch;
      const int32_t nb = (int32_t)(cnt - first < batch ? cnt - first : batch);
      orc_integrate_lockstep(&mechs[mm], o, nb, list + first, T, kscale, ldk, F, ldy, t0, tout,
                             y, stats);
    }
  }
  free(list);
}

int32_t orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* OpenMP threads of later batch integrations (n > 0; otherwise unchanged). */
void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Fixed order / fixed step mode (order-of-accuracy checks)                  */
/* ------------------------------------------------------------------------ */

/* Take nsteps steps of size h at order q from the Nordsieck array z
 * ([q+1][S] row-major, in units of h), Newton iterated to convergence with a
 * fresh Jacobian each iteration.  Constant steps: xi_i = i.  Returns 0 or -4. */
int32_t orc_fixed_steps(const orc_mech *m, const double *kf, const double *kr, const double *F,
                        int q, double h, int nsteps, double *zio) {
  int S = m->n_species;
  orc_sys s = {m, kf, kr, F, S, NULL, 1};
  double z[ORC_QMAX + 2][ORC_MAXN];
  double xi[ORC_QMAX + 2], l[ORC_QMAX + 2], Cerr, e[ORC_MAXS], yv[ORC_MAXS], f[ORC_MAXS];
  double J[ORC_MAXS * ORC_MAXS];
  int32_t perm[ORC_MAXS];
  for (int j = 0; j <= q; ++j)
    for (int i = 0; i < S; ++i) z[j][i] = zio[j * S + i];
  for (int i = 1; i <= q + 1; ++i) xi[i] = i;
  orc_bdf_coeffs(q, xi, l, &Cerr);
  double gamma = h / l[1];
  for (int n = 0; n < nsteps; ++n) {
    orc_predict(S, q, z);
    for (int i = 0; i < S; ++i) e[i] = 0.0;
    int ok = 0;
    for (int it = 0; it < 50; ++it) {
      for (int i = 0; i < S; ++i) yv[i] = z[0][i] + e[i];
      sys_f(&s, yv, f);
      orc_jac(m, kf, kr, yv, J);
      for (int i = 0; i < S; ++i)
        for (int j = 0; j < S; ++j) J[i * S + j] = (i == j ? 1.0 : 0.0) - gamma * J[i * S + j];
      if (orc_lu_factor(S, J, perm)) return ORC_SETUP_FAILURE;
      double d[ORC_MAXS], dn = 0.0, yn = 0.0;
      for (int i = 0; i < S; ++i) d[i] = -(e[i] - gamma * f[i] + z[1][i] / l[1]);
      orc_lu_solve(S, J, perm, d);
      for (int i = 0; i < S; ++i) {
        e[i] += d[i];
        dn = fmax(dn, fabs(d[i]));
        yn = fmax(yn, fabs(z[0][i] + e[i]));
      }
      if (dn <= 1e-15 * (yn > 1e-300 ? yn : 1.0)) {
        ok = 1;
        break;
      }
    }
    if (!ok) return ORC_CONV_FAILURE;
    for (int j = 0; j <= q; ++j)
      for (int i = 0; i < S; ++i) z[j][i] += l[j] * e[i];
  }
  for (int j = 0; j <= q; ++j)
    for (int i = 0; i < S; ++i) zio[j * S + i] = z[j][i];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Frozen discrete map: replay, tangent-linear and adjoint                   */
/* ------------------------------------------------------------------------ */
/*
 * The adaptive run is a sequence of accepted steps n = 1..Nst with sizes
 * h_n and orders q_n.  Between accepted steps the Nordsieck array only
 * undergoes linear maps (order change, rescale, exact restore after a
 * rejected attempt) or, after repeated error-test failures, a rebuild
 * z = [y, h f(y)] at order 1.  Freezing (h_n, q_n, rebuild_n) and solving
 * each corrector exactly gives a smooth map (y0, lnA) -> y(t_out); these
 * functions evaluate it (replay), its derivative (tangent) and the
 * transpose of its derivative (adjoint).  The gradients are those of the
 * discrete map, not of the ODE solution.
 */

/* step n (1-based) ingredients from the record */
static void rec_xi(const orc_record *rec, int n, double *xi, double *l, double *Cerr) {
  double hist[ORC_QMAX + 1];
  for (int k = 0; k <= ORC_QMAX; ++k) {
    int idx = n - 2 - k; /* hist[k] = h_{n-1-k} */
    hist[k] = idx >= 0 ? rec->h[idx] : rec->h_pad;
  }
  orc_xi(rec->h[n - 1], hist, rec->q[n - 1], xi);
  orc_bdf_coeffs(rec->q[n - 1], xi, l, Cerr);
}

/* Newton to convergence for y - gamma f(y) = a, starting at y (in/out).
 * Full Newton with a fresh Jacobian each iteration. */
static int orc_solve_exact(const orc_sys *s, double gamma, const double *a, double *y) {
  int S = s->S;
  double f[ORC_MAXS], J[ORC_MAXS * ORC_MAXS], d[ORC_MAXS];
  int32_t perm[ORC_MAXS];
  for (int it = 0; it < 60; ++it) {
    sys_f(s, y, f);
    orc_jac(s->m, s->kf, s->kr, y, J);
    for (int i = 0; i < S; ++i)
      for (int j = 0; j < S; ++j) J[i * S + j] = (i == j ? 1.0 : 0.0) - gamma * J[i * S + j];
    if (orc_lu_factor(S, J, perm)) return -1;
    for (int i = 0; i < S; ++i) d[i] = a[i] - (y[i] - gamma * f[i]);
    orc_lu_solve(S, J, perm, d);
    double dn = 0.0, yn = 0.0;
    for (int i = 0; i < S; ++i) {
      y[i] += d[i];
      dn = fmax(dn, fabs(d[i]));
      yn = fmax(yn, fabs(y[i]));
    }
    if (dn <= 4.0 * ORC_UROUND * (yn > 0 ? yn : 1.0)) return 0;
  }
  return 0; /* converged to round-off level (stagnation) */
}

/* Steps of the variable-coefficient BDF at a fixed order q with prescribed
 * sizes h[0..nsteps-1] (test hook for the local-error estimate and the order
 * estimates).  z ([q+1][S], row-major) is the Nordsieck array at the start,
 * in units of h[0]; hist0[k] is the size of the (k+1)-th step before the
 * first one (k = 0..ORC_QMAX), which sets the xi of the first steps.  Each
 * step: rescale the array to the step's size, predict, coefficients from the
 * step history, corrector solved to round-off (fresh Jacobian every
 * iteration), correct.  Per step n it writes the accepted y_n (yout
 * [nsteps][S]), the correction e_n = y_n - predicted value (eout
 * [nsteps][S]) and the error constant Cerr_n (cerr [nsteps]); on exit z is
 * the array after the last step, in units of its size.  Returns 0, -6 for a
 * singular Newton matrix, -9 for arguments outside the oracle's limits. */
int32_t orc_steps(const orc_mech *m, const double *kf, const double *kr, const double *F, int q,
                  int nsteps, const double *h, const double *hist0, double *zio, double *yout,
                  double *eout, double *cerr) {
  const int S = m->n_species;
  if (q < 1 || q > ORC_QMAX || S > ORC_MAXS || m->cv != NULL) return ORC_NONFINITE;
  orc_sys s = {m, kf, kr, F, S, NULL, 1};
  double z[ORC_QMAX + 2][ORC_MAXN];
  double hist[ORC_QMAX + 1], xi[ORC_QMAX + 2], l[ORC_QMAX + 2], Cerr, a[ORC_MAXS], y[ORC_MAXS];
  memset(z, 0, sizeof(z));
  for (int j = 0; j <= q; ++j)
    for (int i = 0; i < S; ++i) z[j][i] = zio[j * S + i];
  for (int k = 0; k <= ORC_QMAX; ++k) hist[k] = hist0[k];
  for (int n = 0; n < nsteps; ++n) {
    if (n > 0) orc_rescale(S, q, h[n] / h[n - 1], z);
    orc_predict(S, q, z);
    orc_xi(h[n], hist, q, xi);
    orc_bdf_coeffs(q, xi, l, &Cerr);
    double gamma = h[n] / l[1];
    for (int i = 0; i < S; ++i) {
      a[i] = z[0][i] - z[1][i] / l[1];
      y[i] = z[0][i];
    }
    if (orc_solve_exact(&s, gamma, a, y)) return ORC_SETUP_FAILURE;
    for (int i = 0; i < S; ++i) {
      double e = y[i] - z[0][i];
      eout[(size_t)n * S + i] = e;
      for (int j = 0; j <= q; ++j) z[j][i] += l[j] * e;
      yout[(size_t)n * S + i] = z[0][i];
    }
    cerr[n] = Cerr;
    for (int k = ORC_QMAX; k >= 1; --k) hist[k] = hist[k - 1];
    hist[0] = h[n];
  }
  for (int j = 0; j <= q; ++j)
    for (int i = 0; i < S; ++i) zio[j * S + i] = z[j][i];
  return 0;
}

/* Replay the frozen step sequence of rec from y0; writes the final state to
 * yout and, if yrec != NULL, the replayed y_n to yrec [n][S]. */
int32_t orc_replay_cell(const orc_mech *m, const double *kf, const double *kr, const double *F,
                        const double *y0, const orc_record *rec, double *yout, double *yrec) {
  int S = m->n_species;
  orc_sys s = {m, kf, kr, F, S, NULL, 1};
  double z[ORC_QMAX + 2][ORC_MAXN], f[ORC_MAXS], a[ORC_MAXS], y[ORC_MAXS], e[ORC_MAXS];
  double xi[ORC_QMAX + 2], l[ORC_QMAX + 2], Cerr;
  double xip[ORC_QMAX + 2], lp[ORC_QMAX + 2];
  memset(z, 0, sizeof(z));
  if (rec->n == 0) {
    for (int i = 0; i < S; ++i) yout[i] = y0[i];
    return 0;
  }
  for (int i = 0; i < S; ++i) z[0][i] = y0[i];
  sys_f(&s, y0, f);
  for (int i = 0; i < S; ++i) z[1][i] = rec->h[0] * f[i];
  int q = 1;
  for (int n = 1; n <= rec->n; ++n) {
    double hn = rec->h[n - 1];
    int qn = rec->q[n - 1];
    if (n > 1) {
      double hp = rec->h[n - 2];
      if (rec->rebuild[n - 1]) {
        sys_f(&s, z[0], f);
        for (int j = 1; j <= ORC_QMAX + 1; ++j)
          for (int i = 0; i < S; ++i) z[j][i] = 0.0;
        for (int i = 0; i < S; ++i) z[1][i] = hn * f[i];
      } else {
        if (qn == q + 1) orc_order_up(S, q, lp, xip, e, z);
        if (qn == q - 1) orc_order_down(S, q, xip, z);
        orc_rescale(S, qn, hn / hp, z);
      }
    }
    q = qn;
    orc_predict(S, q, z);
    rec_xi(rec, n, xi, l, &Cerr);
    double gamma = hn / l[1];
    for (int i = 0; i < S; ++i) {
      a[i] = z[0][i] - z[1][i] / l[1];
      y[i] = rec->y[(size_t)(n - 1) * S + i]; /* start from the recorded value */
    }
    if (orc_solve_exact(&s, gamma, a, y)) return ORC_SETUP_FAILURE;
    for (int i = 0; i < S; ++i) e[i] = y[i] - z[0][i];
    for (int j = 0; j <= q; ++j)
      for (int i = 0; i < S; ++i) z[j][i] += l[j] * e[i];
    if (yrec)
      for (int i = 0; i < S; ++i) yrec[(size_t)(n - 1) * S + i] = z[0][i];
    memcpy(xip, xi, sizeof(xi));
    memcpy(lp, l, sizeof(l));
  }
  for (int i = 0; i < S; ++i) yout[i] = z[0][i];
  return 0;
}

/* d f / d lnA_r applied to a direction: sum_r nu_r q_r(y) dp_r. */
static void orc_fp_dir(const orc_sys *s, const double *y, const double *dp, double *out) {
  const orc_mech *m = s->m;
  double q[4096];
  orc_reaction_rates(m, s->kf, s->kr, y, q);
  for (int i = 0; i < s->S; ++i) out[i] = 0.0;
  for (int r = 0; r < m->n_reactions; ++r) {
    double v = q[r] * dp[r];
    for (int k = 0; k < ORC_SLOTS; ++k) {
      int a = m->reac[r * ORC_SLOTS + k], b = m->prod[r * ORC_SLOTS + k];
      if (a >= 0) out[a] -= v;
      if (b >= 0) out[b] += v;
    }
  }
}

/* Transpose of orc_fp_dir: pbar_r += scale * q_r(y) * (nu_r . mu). */
static void orc_fp_adj(const orc_sys *s, const double *y, const double *mu, double scale,
                       double *pbar) {
  const orc_mech *m = s->m;
  double q[4096];
  orc_reaction_rates(m, s->kf, s->kr, y, q);
  for (int r = 0; r < m->n_reactions; ++r) {
    double dot = 0.0;
    for (int k = 0; k < ORC_SLOTS; ++k) {
      int a = m->reac[r * ORC_SLOTS + k], b = m->prod[r * ORC_SLOTS + k];
      if (a >= 0) dot -= mu[a];
      if (b >= 0) dot += mu[b];
    }
    pbar[r] += scale * q[r] * dot;
  }
}

static void matvec(int S, const double *A, const double *x, double *out) {
  for (int i = 0; i < S; ++i) {
    double s = 0.0;
    for (int j = 0; j < S; ++j) s += A[i * S + j] * x[j];
    out[i] = s;
  }
}

static void matvec_t(int S, const double *A, const double *x, double *out) {
  for (int j = 0; j < S; ++j) out[j] = 0.0;
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) out[j] += A[i * S + j] * x[i];
}

/* Tangent-linear (forward sensitivity) of the frozen map along the states
 * in yrec ([n][S], typically the replayed ones): direction (dy0, dp) ->
 * dy(t_out). */
int32_t orc_tangent_cell(const orc_mech *m, const double *kf, const double *kr, const double *F,
                         const double *y0, const orc_record *rec, const double *yrec,
                         const double *dy0, const double *dp, double *dyout) {
  int S = m->n_species;
  orc_sys s = {m, kf, kr, F, S, NULL, 1};
  double dz[ORC_QMAX + 2][ORC_MAXN], J[ORC_MAXS * ORC_MAXS], t1[ORC_MAXS], t2[ORC_MAXS];
  double da[ORC_MAXS], de[ORC_MAXS];
  double xi[ORC_QMAX + 2], l[ORC_QMAX + 2], Cerr, xip[ORC_QMAX + 2], lp[ORC_QMAX + 2];
  int32_t perm[ORC_MAXS];
  memset(dz, 0, sizeof(dz));
  if (rec->n == 0) {
    for (int i = 0; i < S; ++i) dyout[i] = dy0[i];
    return 0;
  }
  /* z = [y0, h_1 f(y0)] */
  orc_jac(m, kf, kr, y0, J);
  matvec(S, J, dy0, t1);
  orc_fp_dir(&s, y0, dp, t2);
  for (int i = 0; i < S; ++i) {
    dz[0][i] = dy0[i];
    dz[1][i] = rec->h[0] * (t1[i] + t2[i]);
  }
  int q = 1;
  for (int n = 1; n <= rec->n; ++n) {
    double hn = rec->h[n - 1];
    int qn = rec->q[n - 1];
    if (n > 1) {
      const double *yp = yrec + (size_t)(n - 2) * S;
      if (rec->rebuild[n - 1]) {
        orc_jac(m, kf, kr, yp, J);
        matvec(S, J, dz[0], t1);
        orc_fp_dir(&s, yp, dp, t2);
        for (int j = 1; j <= ORC_QMAX + 1; ++j)
          for (int i = 0; i < S; ++i) dz[j][i] = 0.0;
        for (int i = 0; i < S; ++i) dz[1][i] = hn * (t1[i] + t2[i]);
      } else {
        if (qn == q + 1) orc_order_up(S, q, lp, xip, de, dz);
        if (qn == q - 1) orc_order_down(S, q, xip, dz);
        orc_rescale(S, qn, hn / rec->h[n - 2], dz);
      }
    }
    q = qn;
    orc_predict(S, q, dz);
    rec_xi(rec, n, xi, l, &Cerr);
    double gamma = hn / l[1];
    const double *yn = yrec + (size_t)(n - 1) * S;
    orc_jac(m, kf, kr, yn, J);
    for (int i = 0; i < S; ++i)
      for (int j = 0; j < S; ++j) J[i * S + j] = (i == j ? 1.0 : 0.0) - gamma * J[i * S + j];
    if (orc_lu_factor(S, J, perm)) return ORC_SETUP_FAILURE;
    orc_fp_dir(&s, yn, dp, t2);
    for (int i = 0; i < S; ++i) da[i] = dz[0][i] - dz[1][i] / l[1] + gamma * t2[i];
    orc_lu_solve(S, J, perm, da); /* da <- dy_n */
    for (int i = 0; i < S; ++i) de[i] = da[i] - dz[0][i];
    for (int j = 0; j <= q; ++j)
      for (int i = 0; i < S; ++i) dz[j][i] += l[j] * de[i];
    memcpy(xip, xi, sizeof(xi));
    memcpy(lp, l, sizeof(l));
  }
  for (int i = 0; i < S; ++i) dyout[i] = dz[0][i];
  return 0;
}

/* Adjoint of the frozen map along yrec: given ybar = dL/dy(t_out), returns
 * y0bar = dL/dy0 and adds dL/dlnA_r into pbar [R]. */
int32_t orc_adjoint_cell(const orc_mech *m, const double *kf, const double *kr, const double *F,
                         const double *y0, const orc_record *rec, const double *yrec,
                         const double *ybar, double *y0bar, double *pbar) {
  int S = m->n_species;
  orc_sys s = {m, kf, kr, F, S, NULL, 1};
  double zb[ORC_QMAX + 2][ORC_MAXN], J[ORC_MAXS * ORC_MAXS], mu[ORC_MAXS], t1[ORC_MAXS];
  double ebar_extra[ORC_MAXS], eb[ORC_MAXS];
  double xi[ORC_QMAX + 2], l[ORC_QMAX + 2], Cerr;
  int32_t perm[ORC_MAXS];
  memset(zb, 0, sizeof(zb));
  int N = rec->n;
  if (N == 0) {
    for (int i = 0; i < S; ++i) y0bar[i] = ybar[i];
    return 0;
  }
  for (int i = 0; i < S; ++i) {
    zb[0][i] = ybar[i];
    ebar_extra[i] = 0.0;
  }
  for (int n = N; n >= 1; --n) {
    int q = rec->q[n - 1];
    double hn = rec->h[n - 1];
    rec_xi(rec, n, xi, l, &Cerr);
    double gamma = hn / l[1];
    const double *yn = yrec + (size_t)(n - 1) * S;
    /* z_n = zp + l e,  e = y_n - zp_0 */
    for (int i = 0; i < S; ++i) {
      double acc = ebar_extra[i];
      for (int j = 0; j <= q; ++j) acc += l[j] * zb[j][i];
      eb[i] = acc;
      zb[0][i] -= acc; /* from e = y - zp_0 */
    }
    /* y_n = Y(a), (I - gamma J) dy = da + gamma f_p dp */
    orc_jac(m, kf, kr, yn, J);
    for (int i = 0; i < S; ++i)
      for (int j = 0; j < S; ++j) J[i * S + j] = (i == j ? 1.0 : 0.0) - gamma * J[i * S + j];
    if (orc_lu_factor(S, J, perm)) return ORC_SETUP_FAILURE;
    for (int i = 0; i < S; ++i) mu[i] = eb[i];
    orc_lu_solve_transposed(S, J, perm, mu);
    orc_fp_adj(&s, yn, mu, gamma, pbar);
    /* a = zp_0 - zp_1 / l_1 */
    for (int i = 0; i < S; ++i) {
      zb[0][i] += mu[i];
      zb[1][i] -= mu[i] / l[1];
    }
    /* predictor transpose: zp = A z  =>  zbar <- A^T zpbar (reverse order) */
    for (int k = q; k >= 1; --k)
      for (int j = k; j <= q; ++j)
        for (int i = 0; i < S; ++i) zb[j][i] += zb[j - 1][i];
    /* transition from step n-1 into step n */
    for (int i = 0; i < S; ++i) ebar_extra[i] = 0.0;
    if (n == 1) {
      /* z = [y0, h_1 f(y0)] */
      orc_jac(m, kf, kr, y0, J);
      matvec_t(S, J, zb[1], t1);
      for (int i = 0; i < S; ++i) y0bar[i] = zb[0][i] + hn * t1[i];
      orc_fp_adj(&s, y0, zb[1], hn, pbar);
      break;
    }
    int qp = rec->q[n - 2];
    const double *yp = yrec + (size_t)(n - 2) * S;
    if (rec->rebuild[n - 1]) {
      orc_jac(m, kf, kr, yp, J);
      matvec_t(S, J, zb[1], t1);
      orc_fp_adj(&s, yp, zb[1], hn, pbar);
      for (int i = 0; i < S; ++i) zb[0][i] += hn * t1[i];
      for (int j = 1; j <= ORC_QMAX + 1; ++j)
        for (int i = 0; i < S; ++i) zb[j][i] = 0.0;
    } else {
      /* rescale by eta = h_n / h_{n-1} (diagonal) */
      double eta = hn / rec->h[n - 2], fct = 1.0;
      for (int j = 1; j <= q; ++j) {
        fct *= eta;
        for (int i = 0; i < S; ++i) zb[j][i] *= fct;
      }
      if (q == qp + 1) {
        /* z_j += (l'_{j-1}/xi'_{qp+1}) e_{n-1}, j = 1..qp+1 (primes: step n-1) */
        double xip[ORC_QMAX + 2], lp[ORC_QMAX + 2], Cp;
        rec_xi(rec, n - 1, xip, lp, &Cp);
        double c = 1.0 / xip[qp + 1];
        for (int j = 1; j <= qp + 1; ++j)
          for (int i = 0; i < S; ++i) ebar_extra[i] += c * lp[j - 1] * zb[j][i];
        for (int i = 0; i < S; ++i) zb[qp + 1][i] = 0.0;
      } else if (q == qp - 1) {
        /* z_j -= c_j z_qp, j = 1..qp-1; z_qp dropped */
        double xip[ORC_QMAX + 2], lp[ORC_QMAX + 2], Cp, c[ORC_QMAX + 2];
        rec_xi(rec, n - 1, xip, lp, &Cp);
        for (int j = 0; j <= qp; ++j) c[j] = 0.0;
        c[1] = 1.0;
        for (int i = 1; i <= qp - 1; ++i)
          for (int j = i + 1; j >= 1; --j) c[j] = c[j - 1] + xip[i] * c[j];
        for (int i = 0; i < S; ++i) {
          double acc = 0.0;
          for (int j = 1; j < qp; ++j) acc -= c[j] * zb[j][i];
          zb[qp][i] = acc;
        }
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Outer-step perturbation (counter-based SplitMix64)                        */
/* ------------------------------------------------------------------------ */

/* SplitMix64 output for generator state x (Steele, Lea & Flood, OOPSLA 2014):
 * advance the state by the golden gamma, then apply the variant-13 mixer. */
uint64_t orc_splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

/* Uniform in [-1, 1) for (seed, outer step, cell, species):
 * key = splitmix64(seed); u53 = splitmix64(key ^ counter) >> 11 with
 * counter = step * 2^40 + cell * 2^8 + species. */
double orc_perturb_uniform(uint64_t seed, int64_t step, int64_t cell, int32_t species) {
  uint64_t key = orc_splitmix64(seed);
  uint64_t ctr = ((uint64_t)step << 40) + ((uint64_t)cell << 8) + (uint64_t)species;
  uint64_t v = orc_splitmix64(key ^ ctr);
  double u = (double)(v >> 11) * (1.0 / 9007199254740992.0);
  return 2.0 * u - 1.0;
}

/* y_i <- max(0, y_i (1 + amp u_i)), then rescale the cell so that
 * sum_i w_i y_i keeps its value from before the perturbation.  Row c of y is
 * the cell with index cell_index[c] (NULL: c) in the perturbation's key. */
void orc_perturb_cells(int64_t N, const int64_t *cell_index, const int32_t *n_species_of_cell,
                       int32_t ldy, double *y, const double *const *weights_of_cell,
                       uint64_t seed, int64_t step, double amp) {
  for (int64_t c = 0; c < N; ++c) {
    int S = n_species_of_cell[c];
    const double *w = weights_of_cell[c];
    const int64_t cell = cell_index ? cell_index[c] : c;
    double *yc = y + c * ldy;
    double before = 0.0, after = 0.0;
    for (int i = 0; i < S; ++i) before += w[i] * yc[i];
    for (int i = 0; i < S; ++i) {
      double v = yc[i] * (1.0 + amp * orc_perturb_uniform(seed, step, cell, i));
      yc[i] = v > 0.0 ? v : 0.0;
      after += w[i] * yc[i];
    }
    if (after > 0.0) {
      double s = before / after;
      for (int i = 0; i < S; ++i) yc[i] *= s;
    }
  }
}

/* The rows of y are the cells 0..N-1. */
void orc_perturb_batch(int64_t N, const int32_t *n_species_of_cell, int32_t ldy, double *y,
                       const double *const *weights_of_cell, uint64_t seed, int64_t step,
                       double amp) {
  orc_perturb_cells(N, NULL, n_species_of_cell, ldy, y, weights_of_cell, seed, step, amp);
}
