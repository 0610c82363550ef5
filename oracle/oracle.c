/*
 * CPU oracle for the coupled displacement / phase-field operator.
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path. Plain FP64 C
 * (the 3x3 eigensolver runs in long double), no sum factorisation, no shared
 * code with the HIP library.
 *
 * Each step cites the passage of the paper it follows. Where the paper is
 * silent the reading used is stated next to the code:
 *  - the matrix Prandtl branch carries linear hardening, optionally the Voce term of
 *    eq:plasticity-strain-hardening-law, and an overstress factor
 *    (1 + visc * dgamma / dt) on the yield stress; visc = 0 gives Box 2 exactly;
 *    linear hardening takes the closed-form root of the consistency equation, Voce
 *    hardening Box 2's Newton iteration (kept inside the admissible bracket);
 *  - degradation enters the Prandtl update through g*mu and g*q_tr
 *    (eq:degraded-trial-stress) with hardening kept in Box 2's equation;
 *  - tension branch of the Amor split at tr(eps^e) >= 0; history switch active
 *    only for psi^+ > H_n; plastic only for f > 0;
 *  - the eigenvector derivative of App. B is used in its divided-difference form
 *    (ln b_i - ln b_j)/(b_i - b_j), which equals the printed distinct-eigenvalue
 *    expression and stays finite when eigenvalues coincide;
 *  - the inelastic state is stored as D = Cin^-1 - I so that b_tr - I is formed
 *    without cancellation before log1p (Appendix A's log1p remark);
 *  - extra branches in parallel (Section 2.3): each has its own spring (mu_k,
 *    kappa_k), its own state and principal frame; every branch is degraded by the
 *    Amor split of its own trial volumetric strain, the total psi^+ is the sum of
 *    the branches' and drives the history, and the per-phase parameters (Gc,
 *    sigma0, visc) are those of the phase's first block. A Maxwell branch uses the
 *    degraded modulus g mu in its closed-form update
 *    (eq:principal-directions-format-1); an extra Hooke branch has Cin^-1 = I.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* 1-D rules: Legendre polynomials by the three-term recurrence, roots by    */
/* bisection (slow and obviously convergent), all in long double.            */
/* ------------------------------------------------------------------------ */

/* P_n(x) and P_n'(x) (P_k' = k P_{k-1} + x P_{k-1}'). */
static void legendre(int n, long double x, long double* pn, long double* dpn) {
  long double p0 = 1.0L, d0 = 0.0L;
  if (n == 0) { *pn = p0; *dpn = d0; return; }
  long double p1 = x, d1 = 1.0L;
  for (int k = 2; k <= n; k++) {
    long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
    long double d2 = k * p1 + x * d1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  (void)d0;
  *pn = p1; *dpn = d1;
}

typedef long double (*scalar_fn)(int, long double);

static long double fn_p(int n, long double x) { long double p, d; legendre(n, x, &p, &d); return p; }
static long double fn_dp(int n, long double x) { long double p, d; legendre(n, x, &p, &d); return d; }

/* All roots of f(n, .) in (-1, 1), found by scanning and bisecting. */
static int roots_in_interval(scalar_fn f, int n, long double* out, int max_roots) {
  const int M = 20000;
  int cnt = 0;
  long double xa = -1.0L + 1e-12L, fa = f(n, xa);
  for (int i = 1; i <= M && cnt < max_roots; i++) {
    long double xb = -1.0L + 1e-12L + (2.0L - 2e-12L) * i / M;
    long double fb = f(n, xb);
    if ((fa < 0) != (fb < 0)) {
      long double lo = xa, hi = xb, flo = fa;
      for (int it = 0; it < 200; it++) {
        long double mid = 0.5L * (lo + hi);
        long double fm = f(n, mid);
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
        if (hi - lo < 1e-30L) break;
      }
      out[cnt++] = 0.5L * (lo + hi);
    }
    xa = xb; fa = fb;
  }
  return cnt;
}

void or_gauss(int n, double* x, double* w) {
  long double r[16];
  int k = roots_in_interval(fn_p, n, r, 16);
  for (int i = 0; i < k && i < n; i++) {
    long double p, d;
    legendre(n, r[i], &p, &d);
    x[i] = (double)r[i];
    w[i] = (double)(2.0L / ((1.0L - r[i] * r[i]) * d * d));
  }
}

void or_gll(int n, double* x) {
  /* n points: -1, roots of P_{n-1}', +1 */
  long double r[16];
  x[0] = -1.0;
  x[n - 1] = 1.0;
  if (n > 2) {
    int k = roots_in_interval(fn_dp, n - 1, r, 16);
    for (int i = 0; i < k && i < n - 2; i++) x[i + 1] = (double)r[i];
  }
}

/* Lagrange basis on nodes xn[0..n-1] and its derivative, at t. */
static void lagrange(int n, const double* xn, double t, double* val, double* der) {
  for (int i = 0; i < n; i++) {
    double v = 1.0;
    for (int j = 0; j < n; j++)
      if (j != i) v *= (t - xn[j]) / (xn[i] - xn[j]);
    double d = 0.0;
    for (int k = 0; k < n; k++) {
      if (k == i) continue;
      double term = 1.0 / (xn[i] - xn[k]);
      for (int j = 0; j < n; j++)
        if (j != i && j != k) term *= (t - xn[j]) / (xn[i] - xn[j]);
      d += term;
    }
    val[i] = v;
    der[i] = d;
  }
}

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra (row-major 3x3).                               */
/* ------------------------------------------------------------------------ */

static void mm3(const double A[3][3], const double B[3][3], double C[3][3]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0.0;
      for (int k = 0; k < 3; k++) s += A[i][k] * B[k][j];
      C[i][j] = s;
    }
}

static void tr3(const double A[3][3], double T[3][3]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) T[i][j] = A[j][i];
}

static double inv3(const double A[3][3], double Ai[3][3]) {
  double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
  Ai[0][0] = c00 / det;
  Ai[1][0] = c01 / det;
  Ai[2][0] = c02 / det;
  Ai[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
  Ai[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
  Ai[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
  Ai[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
  Ai[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
  Ai[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
  return det;
}

static void voigt_to_mat(const double v[6], double M[3][3]) {
  M[0][0] = v[0]; M[1][1] = v[1]; M[2][2] = v[2];
  M[1][2] = M[2][1] = v[3];
  M[0][2] = M[2][0] = v[4];
  M[0][1] = M[1][0] = v[5];
}

/* Cyclic Jacobi in long double, run to convergence. Eigenvalues ascending,
 * eigenvectors as the columns of V. Any backward-stable symmetric solver
 * serves (the paper only asks for the spectral decomposition). */
static void eig_sym3_ld(const long double A[3][3], long double lam[3], long double V[3][3]) {
  long double a[3][3], v[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      a[i][j] = 0.5L * (A[i][j] + A[j][i]);
      v[i][j] = (i == j) ? 1.0L : 0.0L;
    }
  for (int sweep = 0; sweep < 60; sweep++) {
    long double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    long double nrm = off;
    for (int i = 0; i < 3; i++) nrm += a[i][i] * a[i][i];
    if (off == 0.0L || off <= 1e-40L * nrm) break;
    for (int p = 0; p < 2; p++)
      for (int q = p + 1; q < 3; q++) {
        if (a[p][q] == 0.0L) continue;
        long double th = (a[q][q] - a[p][p]) / (2.0L * a[p][q]);
        long double t = (th >= 0.0L ? 1.0L : -1.0L) / (fabsl(th) + sqrtl(th * th + 1.0L));
        long double c = 1.0L / sqrtl(t * t + 1.0L), s = t * c;
        long double R[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        R[p][p] = c; R[q][q] = c; R[p][q] = s; R[q][p] = -s;
        long double tmp[3][3], an[3][3], vn[3][3];
        /* a <- R^T a R, v <- v R */
        for (int i = 0; i < 3; i++)
          for (int j = 0; j < 3; j++) {
            long double sum = 0.0L;
            for (int k = 0; k < 3; k++) sum += a[i][k] * R[k][j];
            tmp[i][j] = sum;
          }
        for (int i = 0; i < 3; i++)
          for (int j = 0; j < 3; j++) {
            long double sum = 0.0L;
            for (int k = 0; k < 3; k++) sum += R[k][i] * tmp[k][j];
            an[i][j] = sum;
          }
        for (int i = 0; i < 3; i++)
          for (int j = 0; j < 3; j++) {
            long double sum = 0.0L;
            for (int k = 0; k < 3; k++) sum += v[i][k] * R[k][j];
            vn[i][j] = sum;
          }
        memcpy(a, an, sizeof a);
        memcpy(v, vn, sizeof v);
        a[p][q] = a[q][p] = 0.0L;
      }
  }
  int idx[3] = {0, 1, 2};
  for (int i = 0; i < 3; i++)
    for (int j = i + 1; j < 3; j++)
      if (a[idx[j]][idx[j]] < a[idx[i]][idx[i]]) { int t = idx[i]; idx[i] = idx[j]; idx[j] = t; }
  for (int i = 0; i < 3; i++) {
    lam[i] = a[idx[i]][idx[i]];
    for (int r = 0; r < 3; r++) V[r][i] = v[r][idx[i]];
  }
}

static void eig_sym3(const double A[3][3], double lam[3], double V[3][3]) {
  long double Al[3][3], l[3], Vl[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) Al[i][j] = A[i][j];
  eig_sym3_ld(Al, l, Vl);
  for (int i = 0; i < 3; i++) {
    lam[i] = (double)l[i];
    for (int r = 0; r < 3; r++) V[r][i] = (double)Vl[r][i];
  }
}

/* (ln b_i - ln b_j) / (b_i - b_j) with b = 1 + beta, finite as b_i -> b_j. */
static double log_divdiff(double bi_m1, double bj_m1) {
  long double bi = 1.0L + bi_m1, bj = 1.0L + bj_m1;
  long double x = ((long double)bi_m1 - (long double)bj_m1) / bj;   /* b_i/b_j - 1 */
  long double r;
  if (fabsl(x) < 1e-3L) {
    /* log1p(x)/x = 1 - x/2 + x^2/3 - ... */
    r = 1.0L - x / 2.0L + x * x / 3.0L - x * x * x / 4.0L + x * x * x * x / 5.0L
        - x * x * x * x * x / 6.0L + x * x * x * x * x * x / 7.0L;
  } else {
    r = log1pl(x) / x;
  }
  (void)bi;
  return (double)(r / bj);
}

double or_log_divdiff(double bi_m1, double bj_m1) { return log_divdiff(bi_m1, bj_m1); }

/* ------------------------------------------------------------------------ */
/* Pointwise constitutive state: R1-R11.                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  double mu, kappa, Gc, sigma0, H, a; int plastic;
  double sinf, bv;  /* Voce saturation stress and rate; bv = 0: linear hardening */
  int maxwell;      /* Maxwell branch (Section 2.3.2) */
  double am;        /* mu dt / eta_d of a Maxwell branch */
} mat_t;

static mat_t make_mat(const or_phase* ph, const or_frac* fr) {
  mat_t m;
  m.mu = ph->E / (2.0 * (1.0 + ph->nu));
  m.kappa = ph->E / (3.0 * (1.0 - 2.0 * ph->nu));
  m.Gc = ph->Gc;
  m.sigma0 = ph->sigma0;
  m.H = ph->H;
  m.a = ph->visc / fr->dt;
  m.plastic = ph->plastic;
  m.sinf = ph->sigma_inf;
  m.bv = ph->voce_beta;
  m.maxwell = 0;
  m.am = 0.0;
  return m;
}

/* Material of an extra branch (Section 2.3): its own spring; a Prandtl branch as the
 * first block's; a Maxwell branch with am = mu dt / eta_d. Gc is the phase's. */
static mat_t make_branch_mat(const or_branch* b, const or_frac* fr, double Gc) {
  mat_t m;
  memset(&m, 0, sizeof m);
  m.mu = b->E / (2.0 * (1.0 + b->nu));
  m.kappa = b->E / (3.0 * (1.0 - 2.0 * b->nu));
  m.Gc = Gc;
  if (b->kind == OR_BR_PRANDTL) {
    m.plastic = 1;
    m.sigma0 = b->sigma0;
    m.H = b->H;
    m.a = b->visc / fr->dt;
    m.sinf = b->sigma_inf;
    m.bv = b->voce_beta;
  } else if (b->kind == OR_BR_MAXWELL) {
    m.maxwell = 1;
    m.am = m.mu * fr->dt / b->eta_d;
  }
  return m;
}

/* Yield stress and hardening modulus (eq:plasticity-strain-hardening-law):
 * sigma_y = sigma0 + H ep + (sinf - sigma0)(1 - exp(-bv ep)). */
static double yield_stress(const mat_t* m, double ep) {
  return m->sigma0 + m->H * ep + (m->bv > 0.0 ? (m->sinf - m->sigma0) * (1.0 - exp(-m->bv * ep)) : 0.0);
}
static double yield_slope(const mat_t* m, double ep) {
  return m->H + (m->bv > 0.0 ? (m->sinf - m->sigma0) * m->bv * exp(-m->bv * ep) : 0.0);
}

typedef struct {
  double F[3][3], Fi[3][3], detF;
  double b[3][3];          /* b_tr = I + A */
  double beta[3], N[3][3]; /* eigenpairs of A (columns of N) */
  double eps[3], theta, e[3];
  double g, gp;
  double q, sn, dgamma, c, Heff, den, ep;
  int plastic;
  double tau[3];           /* undegraded block principal stresses */
  double taud[3];          /* degraded principal stresses */
  double psi;              /* psi^+ */
  double Hn, H; int Hactive;
  double c0, alpha_p, alpha_pp;
  double L;
  double tau_degr[3][3];
  int nonphysical;
} qp_state;

/* Steps R1-R8 and R11 of one branch: st = D[6] (Voigt), ebar_p. */
static void qp_branch(const mat_t* m, const or_frac* fr, const double G[9], double phi,
                      const double st[7], qp_state* s) {
  memset(s, 0, sizeof *s);
  double Gm[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) Gm[i][j] = G[i * 3 + j];
  /* R1: F = I + grad_X u (Section 2.1) */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) s->F[i][j] = (i == j ? 1.0 : 0.0) + Gm[i][j];
  s->detF = inv3(s->F, s->Fi);
  /* R2: b_tr = F Cin^-1 F^T (eq:inelasticity-be-update); with Cin^-1 = I + D,
   * A = b_tr - I = G + G^T + G G^T + F D F^T. */
  double D[3][3], GGt[3][3], Gt[3][3], FD[3][3], Ft[3][3], FDFt[3][3], A[3][3];
  voigt_to_mat(st, D);
  tr3(Gm, Gt);
  mm3(Gm, Gt, GGt);
  mm3(s->F, D, FD);
  tr3(s->F, Ft);
  mm3(FD, Ft, FDFt);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      A[i][j] = Gm[i][j] + Gm[j][i] + GGt[i][j] + FDFt[i][j];
      s->b[i][j] = (i == j ? 1.0 : 0.0) + A[i][j];
    }
  /* R3: spectral decomposition (eq:inelasticity-spectral-decomposition) */
  eig_sym3(A, s->beta, s->N);
  s->nonphysical = (s->detF <= 0.0);
  for (int i = 0; i < 3; i++)
    if (1.0 + s->beta[i] <= 0.0) s->nonphysical = 1;
  /* R4: principal log strains with log1p (eq:inelasticity-log-strain-principal) */
  s->theta = 0.0;
  for (int i = 0; i < 3; i++) {
    s->eps[i] = 0.5 * log1p(s->beta[i]);
    s->theta += s->eps[i];
  }
  for (int i = 0; i < 3; i++) s->e[i] = s->eps[i] - s->theta / 3.0;
  /* R5: degradation g = (1-phi)^2 + eta (eq:degr-funct) */
  s->g = (1.0 - phi) * (1.0 - phi) + fr->eta;
  s->gp = -2.0 * (1.0 - phi);
  /* R6: Box 2 with the degraded trial stress (eq:degraded-yield-condition) */
  double ee = s->e[0] * s->e[0] + s->e[1] * s->e[1] + s->e[2] * s->e[2];
  s->q = 2.0 * m->mu * sqrt(1.5 * ee);       /* q = sqrt(3/2)|tau_d^tr|, tau_d^tr = 2 mu e */
  s->sn = yield_stress(m, st[6]);            /* sigma_y(ebar_p,n) */
  s->c = 1.0;
  s->dgamma = 0.0;
  s->plastic = 0;
  if (m->plastic) {
    double f = s->g * s->q - s->sn;
    if (f > 0.0) {
      if (m->bv > 0.0) {
        /* Box 2 Newton on g q - 3 g mu dg - sigma_y(ebar_n + dg)(1 + a dg) = 0 from
         * dg = 0; the equation is positive at 0 and negative at q / (3 mu) (c = 0),
         * and a step leaving that bracket is replaced by bisection */
        double lo = 0.0, hi = s->q / (3.0 * m->mu), dg = 0.0;
        for (int it = 0; it < 200; it++) {
          double sy = yield_stress(m, st[6] + dg), hy = yield_slope(m, st[6] + dg);
          double ft = s->g * s->q - 3.0 * s->g * m->mu * dg - sy * (1.0 + m->a * dg);
          if (ft > 0.0) lo = dg; else hi = dg;
          double nd = dg + ft / (3.0 * s->g * m->mu + hy * (1.0 + m->a * dg) + m->a * sy);
          if (!(nd > lo && nd < hi)) nd = 0.5 * (lo + hi);
          double step = fabs(nd - dg);
          dg = nd;
          if (step <= 1e-15 * dg || hi - lo <= 1e-15 * hi) break;
        }
        s->dgamma = dg;
      } else {
        /* g q - 3 g mu dg - (sn + H dg)(1 + a dg) = 0, smaller positive root */
        double B = 3.0 * s->g * m->mu + m->H + m->a * s->sn;
        s->dgamma = 2.0 * f / (B + sqrt(B * B + 4.0 * m->a * m->H * f));
      }
      s->c = 1.0 - 3.0 * m->mu * s->dgamma / s->q;   /* eq:plasticity-deviatoric-strain-update */
      /* d/d dg of sigma_y(ebar_n + dg)(1 + a dg) */
      s->Heff = yield_slope(m, st[6] + s->dgamma) * (1.0 + m->a * s->dgamma) +
                m->a * yield_stress(m, st[6] + s->dgamma);
      s->den = 3.0 * s->g * m->mu + s->Heff;
      s->ep = st[6] + s->dgamma;
      s->plastic = 1;
    }
  } else if (m->maxwell) {
    /* Maxwell branch, closed form with the degraded modulus g mu
     * (eq:viscoelasticity-deviatoric-strain-update-hencky, eq:principal-directions-format-1) */
    s->c = 1.0 / (1.0 + m->am * s->g);
  }
  /* R7: block principal stress (eq:principal-stress-update-eigenvalues) */
  for (int i = 0; i < 3; i++) s->tau[i] = 2.0 * m->mu * s->c * s->e[i] + m->kappa * s->theta;
  /* R8: Amor split (eq:linear-degraded-stress), principal psi^+ (App. A) */
  double cee = s->c * s->c * ee;
  if (s->theta >= 0.0) {
    for (int i = 0; i < 3; i++) s->taud[i] = s->g * s->tau[i];
    s->psi = m->mu * cee + 0.5 * m->kappa * s->theta * s->theta;
  } else {
    for (int i = 0; i < 3; i++)
      s->taud[i] = s->g * (s->tau[i] - m->kappa * s->theta) + m->kappa * s->theta;
    s->psi = m->mu * cee;
  }
  /* R11: tau_degr = sum_i taud_i n_i (x) n_i (eq:principal-stress-update-eigenvalues-2) */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double sum = 0.0;
      for (int k = 0; k < 3; k++) sum += s->taud[k] * s->N[i][k] * s->N[j][k];
      s->tau_degr[i][j] = sum;
    }
}

/* Steps R9-R10: history and local phase-field residual from the point's total psi^+. */
static void qp_fracture(const mat_t* m, const or_frac* fr, double phi, double phi_n, double Hn,
                        double psi, qp_state* s) {
  /* R9: history (Miehe), strict switch */
  s->Hn = Hn;
  s->Hactive = (psi > s->Hn);
  s->H = s->Hactive ? psi : s->Hn;
  /* R10: L (eq:L-viscous), AT1/AT2 (eq:AT1-AT2) */
  if (fr->at == 2) { s->c0 = 2.0; s->alpha_p = 2.0 * phi; s->alpha_pp = 2.0; }
  else { s->c0 = 8.0 / 3.0; s->alpha_p = 1.0; s->alpha_pp = 0.0; }
  s->L = s->gp * s->H + m->Gc / (s->c0 * fr->l0) * s->alpha_p + fr->zeta * (phi - phi_n) / fr->dt;
}

/* Single block: R1-R11 with st = D[6], ebar_p, H_n. */
static void qp_eval(const mat_t* m, const or_frac* fr, const double G[9], double phi,
                    double phi_n, const double st[8], qp_state* s) {
  qp_branch(m, fr, G, phi, st, s);
  qp_fracture(m, fr, phi, phi_n, st[7], s->psi, s);
}

static void first_piola(const double tau[3][3], const double Fi[3][3], double P[9]) {
  /* P = tau F^-T (eq:mechanical-gradient-transformation) */
  for (int i = 0; i < 3; i++)
    for (int J = 0; J < 3; J++) {
      double sum = 0.0;
      for (int k = 0; k < 3; k++) sum += tau[i][k] * Fi[J][k];
      P[i * 3 + J] = sum;
    }
}

void or_qf_residual(const or_phase* ph, const or_frac* fr, const double G[9], double phi,
                    const double gphi[3], double phi_n, const double st[8], or_qp_out* out) {
  mat_t m = make_mat(ph, fr);
  qp_state s;
  qp_eval(&m, fr, G, phi, phi_n, st, &s);
  first_piola(s.tau_degr, s.Fi, out->P);
  /* R12: f0 = s_phi L, f1 = s_phi (2 Gc l0 / c0) grad_X phi
   * (eq:physical-residual-integrands with eq:phase-gradient-transformation) */
  out->f0 = fr->s_phi * s.L;
  double kf = fr->s_phi * 2.0 * m.Gc * fr->l0 / s.c0;
  for (int J = 0; J < 3; J++) out->f1[J] = kf * gphi[J];
  out->tau[0] = s.tau_degr[0][0]; out->tau[1] = s.tau_degr[1][1]; out->tau[2] = s.tau_degr[2][2];
  out->tau[3] = s.tau_degr[1][2]; out->tau[4] = s.tau_degr[0][2]; out->tau[5] = s.tau_degr[0][1];
  for (int i = 0; i < 3; i++) { out->beta[i] = s.beta[i]; out->eps[i] = s.eps[i]; }
  out->theta = s.theta;
  out->q = s.q;
  out->dgamma = s.dgamma;
  out->c = s.c;
  out->psi_plus = s.psi;
  out->H = s.H;
  out->L = s.L;
  out->g = s.g;
  out->plastic_active = s.plastic;
  out->nonphysical = s.nonphysical;
}

/* ------------------------------------------------------------------------ */
/* Pointwise directional derivative: J1-J12 (Appendices B and C).            */
/* ------------------------------------------------------------------------ */

/* Steps J1-J10 of one branch: dP of its degraded stress and d psi^+ (before the history
 * switch). */
static void qp_tangent_branch(const mat_t* m, const qp_state* s, const double dG[9], double dphi,
                              double dP[9], double* dpsi) {
  double dGm[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) dGm[i][j] = dG[i * 3 + j];
  /* J1: dl = dF F^-1 (spatial velocity-gradient form, eq:hyperelastic-damage-linearization-current) */
  double dl[3][3];
  mm3(dGm, s->Fi, dl);
  /* J2: db_tr = dF Cin^-1 F^T + F Cin^-1 dF^T = dl b + b dl^T (App. B) */
  double dlb[3][3], dA[3][3];
  mm3(dl, s->b, dlb);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) dA[i][j] = dlb[i][j] + dlb[j][i];
  /* J3: rotate into the eigenframe, db~ = N^T db N */
  double Nt[3][3], tmp[3][3], dbt[3][3];
  tr3(s->N, Nt);
  mm3(Nt, dA, tmp);
  mm3(tmp, s->N, dbt);
  /* J4: principal strain derivatives d eps_i = d b_i / (2 b_i) (App. B) */
  double deps[3], dth = 0.0, de[3];
  for (int i = 0; i < 3; i++) {
    deps[i] = dbt[i][i] / (2.0 * (1.0 + s->beta[i]));
    dth += deps[i];
  }
  for (int i = 0; i < 3; i++) de[i] = deps[i] - dth / 3.0;
  /* J5: linearised deviatoric update (Box A1, generalised to degradation,
   * hardening and overstress): d(c e)_i */
  double dce[3];
  if (s->plastic) {
    double dq = 6.0 * m->mu * m->mu * (s->e[0] * de[0] + s->e[1] * de[1] + s->e[2] * de[2]) / s->q;
    double ddg = (s->g * dq + s->gp * (s->q - 3.0 * m->mu * s->dgamma) * dphi) / s->den;
    double k = -(3.0 * m->mu / s->q) * (ddg - s->dgamma * dq / s->q);
    for (int i = 0; i < 3; i++) dce[i] = s->c * de[i] + k * s->e[i];
  } else if (m->maxwell) {
    /* c = 1 / (1 + am g): dc = -am g' c^2 dphi (eq:maxwell-dtau-dphi) */
    double k = -m->am * s->gp * s->c * s->c * dphi;
    for (int i = 0; i < 3; i++) dce[i] = s->c * de[i] + k * s->e[i];
  } else {
    for (int i = 0; i < 3; i++) dce[i] = de[i];
  }
  /* J6/J7: principal degraded stress derivative (eq:linear-degraded-stress-linearization) */
  double dtaud[3];
  for (int i = 0; i < 3; i++) {
    double dtau = 2.0 * m->mu * dce[i] + m->kappa * dth;
    if (s->theta >= 0.0)
      dtaud[i] = s->g * dtau + s->gp * dphi * s->tau[i];
    else
      dtaud[i] = s->g * (dtau - m->kappa * dth) + m->kappa * dth
                 + s->gp * dphi * (s->tau[i] - m->kappa * s->theta);
  }
  /* J8/J9: assemble in the eigenframe: diagonal plus the eigenvector-rotation
   * terms (eq:hencky-stress-linearization) in divided-difference form */
  double X[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      if (i == j) X[i][j] = dtaud[i];
      else X[i][j] = dbt[i][j] * s->g * m->mu * s->c * log_divdiff(s->beta[i], s->beta[j]);
    }
  double dtau_degr[3][3];
  mm3(s->N, X, tmp);
  mm3(tmp, Nt, dtau_degr);
  /* dP = (dtau - tau dl^T) F^-T */
  double dlt[3][3], tdl[3][3], M[3][3];
  tr3(dl, dlt);
  mm3(s->tau_degr, dlt, tdl);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) M[i][j] = dtau_degr[i][j] - tdl[i][j];
  first_piola(M, s->Fi, dP);
  /* J10: psi^+ derivative (eq:energy-displacement-linearization, eq:maxwell-energy-dphi) */
  double ce_dce = 0.0;
  for (int i = 0; i < 3; i++) ce_dce += s->c * s->e[i] * dce[i];
  *dpsi = 2.0 * m->mu * ce_dce;
  if (s->theta >= 0.0) *dpsi += m->kappa * s->theta * dth;
}

/* Steps J11-J12 from the history derivative dH (eq:history-field-linearization: zero
 * when the switch is off); s carries the point's H, c0 and alpha''. */
static void qp_tangent_fracture(const mat_t* m, const or_frac* fr, const qp_state* s, double dH,
                                double dphi, const double dgphi[3], double* df0, double df1[3]) {
  /* J11: dL (eq:linearized-local-damage-residual), g'' = 2 */
  double dL = (2.0 * s->H + m->Gc / (s->c0 * fr->l0) * s->alpha_pp + fr->zeta / fr->dt) * dphi
              + s->gp * dH;
  /* J12 */
  *df0 = fr->s_phi * dL;
  double kf = fr->s_phi * 2.0 * m->Gc * fr->l0 / s->c0;
  for (int J = 0; J < 3; J++) df1[J] = kf * dgphi[J];
}

static void qp_tangent(const mat_t* m, const or_frac* fr, const qp_state* s, const double dG[9],
                       double dphi, const double dgphi[3], double dP[9], double* df0, double df1[3]) {
  double dpsi;
  qp_tangent_branch(m, s, dG, dphi, dP, &dpsi);
  qp_tangent_fracture(m, fr, s, s->Hactive ? dpsi : 0.0, dphi, dgphi, df0, df1);
}

void or_qf_jacobian(const or_phase* ph, const or_frac* fr, const double G[9], double phi,
                    const double gphi[3], double phi_n, const double st[8], const double dG[9],
                    double dphi, const double dgphi[3], double dP[9], double* df0, double df1[3]) {
  mat_t m = make_mat(ph, fr);
  qp_state s;
  (void)gphi;
  qp_eval(&m, fr, G, phi, phi_n, st, &s);
  qp_tangent(&m, fr, &s, dG, dphi, dgphi, dP, df0, df1);
}

/* Partial derivatives of the pointwise outputs with respect to the phase's
 * (Gc, sigma0, visc) at fixed kinematics. */
static void qp_param_partials(const mat_t* m, const or_frac* fr, const qp_state* s,
                              const double gphi[3], double dP[27], double df0[3], double df1[9]) {
  memset(dP, 0, 27 * sizeof(double));
  memset(df0, 0, 3 * sizeof(double));
  memset(df1, 0, 9 * sizeof(double));
  /* Gc enters only the phase-field rows: L through Gc alpha'/(c0 l0), f1 through 2 Gc l0/c0 */
  df0[0] = fr->s_phi * s->alpha_p / (s->c0 * fr->l0);
  for (int J = 0; J < 3; J++) df1[0 * 3 + J] = fr->s_phi * 2.0 * fr->l0 / s->c0 * gphi[J];
  if (!s->plastic) return;
  /* sigma0 and visc enter through dgamma (implicit function of Box 2's equation) */
  double ddg[3];
  /* d sigma_y / d sigma0 = exp(-bv ep) (1 for linear hardening) */
  const double dsy = m->bv > 0.0 ? exp(-m->bv * s->ep) : 1.0;
  ddg[1] = -(1.0 + m->a * s->dgamma) * dsy / s->den;                            /* d/d sigma0 */
  ddg[2] = -yield_stress(m, s->ep) * (s->dgamma / fr->dt) / s->den;              /* d/d visc  */
  for (int k = 1; k < 3; k++) {
    double dce[3], dtaud[3];
    for (int i = 0; i < 3; i++) dce[i] = -(3.0 * m->mu / s->q) * ddg[k] * s->e[i];
    for (int i = 0; i < 3; i++) dtaud[i] = s->g * 2.0 * m->mu * dce[i];
    double dt3[3][3];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        double sum = 0.0;
        for (int l = 0; l < 3; l++) sum += dtaud[l] * s->N[i][l] * s->N[j][l];
        dt3[i][j] = sum;
      }
    first_piola(dt3, s->Fi, dP + 9 * k);
    if (s->Hactive) {
      double dH = 0.0;
      for (int i = 0; i < 3; i++) dH += 2.0 * m->mu * s->c * s->e[i] * dce[i];
      df0[k] = fr->s_phi * s->gp * dH;
    }
  }
}

void or_qf_param_partials(const or_phase* ph, const or_frac* fr, const double G[9], double phi,
                          const double gphi[3], double phi_n, const double st[8], double dP[27],
                          double df0[3], double df1[9]) {
  mat_t m = make_mat(ph, fr);
  qp_state s;
  qp_eval(&m, fr, G, phi, phi_n, st, &s);
  qp_param_partials(&m, fr, &s, gphi, dP, df0, df1);
}

/* ------------------------------------------------------------------------ */
/* Branches in parallel (Section 2.3): tau = sum_k tau_k, psi = sum_k psi_k.  */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nb;                        /* branches evaluated: the block, then the extra ones */
  mat_t m[1 + OR_MAX_EXTRA];
  qp_state s[1 + OR_MAX_EXTRA];  /* s[0] also holds the point's H, switch and L */
  double tau_degr[3][3];         /* total degraded Kirchhoff stress */
  double psi;                    /* total psi^+ */
  int nonphysical;
} mb_point;

/* xs: the extra branches' states, 7 values each (D[6] Voigt, ebar_p); an extra Hooke
 * branch has Cin^-1 = I and reads none. */
static void mb_eval(const or_phase* ph, const or_branch* xb, int n_extra, const or_frac* fr,
                    const double G[9], double phi, double phi_n, const double st[8], const double* xs,
                    mb_point* p) {
  static const double zero7[7] = {0, 0, 0, 0, 0, 0, 0};
  p->m[0] = make_mat(ph, fr);
  qp_branch(&p->m[0], fr, G, phi, st, &p->s[0]);
  p->nb = 1;
  for (int j = 0; j < n_extra; j++) {
    if (xb[j].kind == OR_BR_NONE) continue;
    p->m[p->nb] = make_branch_mat(&xb[j], fr, ph->Gc);
    qp_branch(&p->m[p->nb], fr, G, phi, xb[j].kind == OR_BR_HOOKE ? zero7 : xs + 7 * j, &p->s[p->nb]);
    p->nb++;
  }
  p->psi = 0.0;
  p->nonphysical = 0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) p->tau_degr[i][j] = 0.0;
  for (int k = 0; k < p->nb; k++) {
    p->psi += p->s[k].psi;
    p->nonphysical |= p->s[k].nonphysical;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) p->tau_degr[i][j] += p->s[k].tau_degr[i][j];
  }
  qp_fracture(&p->m[0], fr, phi, phi_n, st[7], p->psi, &p->s[0]);
}

/* Directional derivative of the point: the branches' dP and d psi^+ summed, the
 * history switch of the total psi^+. */
static void mb_tangent(const mb_point* p, const or_frac* fr, const double dG[9], double dphi,
                       const double dgphi[3], double dP[9], double* df0, double df1[3]) {
  double dpsi = 0.0;
  for (int r = 0; r < 9; r++) dP[r] = 0.0;
  for (int k = 0; k < p->nb; k++) {
    double dPk[9], dpk;
    qp_tangent_branch(&p->m[k], &p->s[k], dG, dphi, dPk, &dpk);
    for (int r = 0; r < 9; r++) dP[r] += dPk[r];
    dpsi += dpk;
  }
  qp_tangent_fracture(&p->m[0], fr, &p->s[0], p->s[0].Hactive ? dpsi : 0.0, dphi, dgphi, df0, df1);
}

void or_qf_residual_mb(const or_phase* ph, const or_branch* xb, int n_extra, const or_frac* fr,
                       const double G[9], double phi, const double gphi[3], double phi_n,
                       const double st[8], const double* xs, or_qp_out* out) {
  mb_point p;
  mb_eval(ph, xb, n_extra, fr, G, phi, phi_n, st, xs, &p);
  const qp_state* s = &p.s[0];
  first_piola(p.tau_degr, s->Fi, out->P);
  out->f0 = fr->s_phi * s->L;
  double kf = fr->s_phi * 2.0 * p.m[0].Gc * fr->l0 / s->c0;
  for (int J = 0; J < 3; J++) out->f1[J] = kf * gphi[J];
  out->tau[0] = p.tau_degr[0][0]; out->tau[1] = p.tau_degr[1][1]; out->tau[2] = p.tau_degr[2][2];
  out->tau[3] = p.tau_degr[1][2]; out->tau[4] = p.tau_degr[0][2]; out->tau[5] = p.tau_degr[0][1];
  for (int i = 0; i < 3; i++) { out->beta[i] = s->beta[i]; out->eps[i] = s->eps[i]; }
  out->theta = s->theta;
  out->q = s->q;
  out->dgamma = s->dgamma;
  out->c = s->c;
  out->psi_plus = p.psi;
  out->H = s->H;
  out->L = s->L;
  out->g = s->g;
  out->plastic_active = s->plastic;
  out->nonphysical = p.nonphysical;
}

void or_qf_jacobian_mb(const or_phase* ph, const or_branch* xb, int n_extra, const or_frac* fr,
                       const double G[9], double phi, const double gphi[3], double phi_n,
                       const double st[8], const double* xs, const double dG[9], double dphi,
                       const double dgphi[3], double dP[9], double* df0, double df1[3]) {
  mb_point p;
  (void)gphi;
  mb_eval(ph, xb, n_extra, fr, G, phi, phi_n, st, xs, &p);
  mb_tangent(&p, fr, dG, dphi, dgphi, dP, df0, df1);
}

/* ------------------------------------------------------------------------ */
/* State commit after a converged step (Section 2, exponential-map update).  */
/* ------------------------------------------------------------------------ */

/* New per-point state from the converged (u, phi): the elastic log strain is the
 * trial one with its deviator scaled by the return factor c and the volumetric part
 * kept (eq:inelasticity-deviatoric-strain-update-2), b^e = exp(2 eps^e) in the
 * principal frame of b_tr, Cin^-1_{n+1} = F^-1 b^e F^-T
 * (eq:inelasticity-deviatoric-strain-update-3), stored as D = Cin^-1 - I; the
 * accumulated plastic strain grows by dgamma (eq:plasticity-accumulated-plastic-update)
 * and the history field becomes max(H_n, psi^+). The decisions and c, dgamma, psi^+
 * come from the same pointwise evaluation as the residual; the frame, the
 * exponential and the products are taken in long double. */
/* D_new = F^-1 b^e F^-T - I for one branch with state D (Voigt) and return factor c. */
static void commit_exp_map(const double G[9], const double* st, double c, double D_new[6]) {
  long double F[3][3], A[3][3], D[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) F[i][j] = (i == j ? 1.0L : 0.0L) + (long double)G[i * 3 + j];
  D[0][0] = st[0]; D[1][1] = st[1]; D[2][2] = st[2];
  D[1][2] = D[2][1] = st[3];
  D[0][2] = D[2][0] = st[4];
  D[0][1] = D[1][0] = st[5];
  /* b_tr - I = F (I + D) F^T - I */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      long double sum = 0.0L;
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) sum += F[i][k] * ((k == l ? 1.0L : 0.0L) + D[k][l]) * F[j][l];
      A[i][j] = sum - (i == j ? 1.0L : 0.0L);
    }
  long double beta[3], N[3][3], eps[3], th = 0.0L;
  eig_sym3_ld(A, beta, N);
  for (int i = 0; i < 3; i++) {
    eps[i] = 0.5L * log1pl(beta[i]);
    th += eps[i];
  }
  long double be[3][3] = {{0}}, bev[3];
  for (int i = 0; i < 3; i++) bev[i] = expl(2.0L * ((long double)c * (eps[i] - th / 3.0L) + th / 3.0L));
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) be[i][j] += bev[k] * N[i][k] * N[j][k];
  /* F^-1 by cofactors */
  long double det = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                    F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                    F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  long double Fi[3][3];
  Fi[0][0] = (F[1][1] * F[2][2] - F[1][2] * F[2][1]) / det;
  Fi[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) / det;
  Fi[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) / det;
  Fi[1][0] = (F[1][2] * F[2][0] - F[1][0] * F[2][2]) / det;
  Fi[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) / det;
  Fi[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) / det;
  Fi[2][0] = (F[1][0] * F[2][1] - F[1][1] * F[2][0]) / det;
  Fi[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) / det;
  Fi[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) / det;
  long double C[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      long double sum = 0.0L;
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) sum += Fi[i][k] * be[k][l] * Fi[j][l];
      C[i][j] = sum - (i == j ? 1.0L : 0.0L);
    }
  D_new[0] = (double)C[0][0]; D_new[1] = (double)C[1][1]; D_new[2] = (double)C[2][2];
  D_new[3] = (double)C[1][2]; D_new[4] = (double)C[0][2]; D_new[5] = (double)C[0][1];
}

void or_qf_commit(const or_phase* ph, const or_frac* fr, const double G[9], double phi,
                  const double st[8], double st_new[8]) {
  mat_t m = make_mat(ph, fr);
  qp_state s;
  qp_eval(&m, fr, G, phi, phi, st, &s);
  commit_exp_map(G, st, s.c, st_new);
  st_new[6] = st[6] + s.dgamma;
  st_new[7] = s.H;
}

/* With extra branches (Box 1 step 4 for every branch): the block as or_qf_commit with the
 * history field of the point's total psi^+; each Maxwell or Prandtl branch's D by the same
 * exponential map with its own factor c, and its ebar_p + dgamma; the rows of Hooke
 * branches and empty slots are copied. */
void or_qf_commit_mb(const or_phase* ph, const or_branch* xb, int n_extra, const or_frac* fr,
                     const double G[9], double phi, const double st[8], const double* xs, double st_new[8],
                     double* xs_new) {
  mb_point p;
  mb_eval(ph, xb, n_extra, fr, G, phi, phi, st, xs, &p);
  commit_exp_map(G, st, p.s[0].c, st_new);
  st_new[6] = st[6] + p.s[0].dgamma;
  st_new[7] = p.s[0].H;
  for (int j = 0, k = 1; j < n_extra; j++) {
    const int kind = xb[j].kind;
    for (int r = 0; r < 7; r++) xs_new[7 * j + r] = xs[7 * j + r];
    if (kind == OR_BR_NONE) continue;
    const qp_state* sj = &p.s[k++];
    if (kind == OR_BR_HOOKE) continue;
    commit_exp_map(G, xs + 7 * j, sj->c, xs_new + 7 * j);
    xs_new[7 * j + 6] = xs[7 * j + 6] + sj->dgamma;
  }
}

/* ------------------------------------------------------------------------ */
/* Element operators with dense element matrices (Section 4).                */
/* ------------------------------------------------------------------------ */

typedef struct {
  int P, Q, nP, nQ;          /* 1-D counts, nodes/qps per element */
  double* N;                 /* [nQ][nP] basis values */
  double* dN;                /* [nQ][nP][3] physical gradients */
  double* wdet;              /* [nQ] quadrature weight times det J */
  double* dNr;               /* [nQ][nP][3] reference gradients (d/dxi) */
  double* wq3;               /* [nQ] quadrature weights on the reference cube */
  int nx1, ny1;
} elem_tab;

static int make_tab(const or_mesh* m, elem_tab* t) {
  int P = m->p + 1, Q = m->q;
  if (m->p < 1 || m->p > 8 || Q < 1 || Q > 12) return -1;
  double xn[16], xq[16], wq[16], B1[16][16], D1[16][16];
  or_gll(P, xn);
  or_gauss(Q, xq, wq);
  for (int q = 0; q < Q; q++) lagrange(P, xn, xq[q], B1[q], D1[q]);
  /* affine box factors (a table-restricted mesh is always mapped: these are then unused) */
  double hx = m->conn ? 2.0 : m->lx / m->nx, hy = m->conn ? 2.0 : m->ly / m->ny, hz = m->conn ? 2.0 : m->lz / m->nz;
  t->P = P; t->Q = Q; t->nP = P * P * P; t->nQ = Q * Q * Q;
  t->N = (double*)malloc(sizeof(double) * t->nQ * t->nP);
  t->dN = (double*)malloc(sizeof(double) * t->nQ * t->nP * 3);
  t->wdet = (double*)malloc(sizeof(double) * t->nQ);
  t->dNr = (double*)malloc(sizeof(double) * t->nQ * t->nP * 3);
  t->wq3 = (double*)malloc(sizeof(double) * t->nQ);
  if (!t->N || !t->dN || !t->wdet || !t->dNr || !t->wq3) return -1;
  for (int qz = 0; qz < Q; qz++)
    for (int qy = 0; qy < Q; qy++)
      for (int qx = 0; qx < Q; qx++) {
        int qq = qx + Q * (qy + Q * qz);
        t->wdet[qq] = wq[qx] * wq[qy] * wq[qz] * (hx * hy * hz / 8.0);
        t->wq3[qq] = wq[qx] * wq[qy] * wq[qz];
        for (int az = 0; az < P; az++)
          for (int ay = 0; ay < P; ay++)
            for (int ax = 0; ax < P; ax++) {
              int a = ax + P * (ay + P * az);
              t->N[qq * t->nP + a] = B1[qx][ax] * B1[qy][ay] * B1[qz][az];
              t->dN[(qq * t->nP + a) * 3 + 0] = (2.0 / hx) * D1[qx][ax] * B1[qy][ay] * B1[qz][az];
              t->dN[(qq * t->nP + a) * 3 + 1] = (2.0 / hy) * B1[qx][ax] * D1[qy][ay] * B1[qz][az];
              t->dN[(qq * t->nP + a) * 3 + 2] = (2.0 / hz) * B1[qx][ax] * B1[qy][ay] * D1[qz][az];
              t->dNr[(qq * t->nP + a) * 3 + 0] = D1[qx][ax] * B1[qy][ay] * B1[qz][az];
              t->dNr[(qq * t->nP + a) * 3 + 1] = B1[qx][ax] * D1[qy][ay] * B1[qz][az];
              t->dNr[(qq * t->nP + a) * 3 + 2] = B1[qx][ax] * B1[qy][ay] * D1[qz][az];
            }
      }
  t->nx1 = m->p * m->nx + 1;
  t->ny1 = m->p * m->ny + 1;
  return 0;
}

static void free_tab(elem_tab* t) { free(t->N); free(t->dN); free(t->wdet); free(t->dNr); free(t->wq3); }

/* Mapped element (Section 4's isoparametric geometry): with node positions X [3][n_nodes]
 * the map x(xi) = sum_a X_a N_a(xi) has J_iK = sum_a X_a,i dN_a/dxi_K at each point; the
 * physical gradients are dN/dx_J = sum_K dN/dxi_K (J^-1)_KJ and the weight w det J.
 * Returns 1 if some det J <= 0. */
static int64_t mesh_nodes(const or_mesh* m, const elem_tab* t);
static int elem_geometry(const or_mesh* m, const elem_tab* t, const int64_t* idx, double* dNe, double* wde) {
  int64_t n_nodes = mesh_nodes(m, t);
  int bad = 0;
  for (int qq = 0; qq < t->nQ; qq++) {
    double J[3][3] = {{0}}, Ji[3][3];
    for (int a = 0; a < t->nP; a++) {
      const double* dr = t->dNr + ((size_t)qq * t->nP + a) * 3;
      for (int i = 0; i < 3; i++)
        for (int K = 0; K < 3; K++) J[i][K] += m->X[i * n_nodes + idx[a]] * dr[K];
    }
    double det = inv3(J, Ji);
    if (!(det > 0.0)) bad = 1;
    wde[qq] = t->wq3[qq] * det;
    for (int a = 0; a < t->nP; a++) {
      const double* dr = t->dNr + ((size_t)qq * t->nP + a) * 3;
      double* dp = dNe + ((size_t)qq * t->nP + a) * 3;
      for (int Jc = 0; Jc < 3; Jc++) dp[Jc] = dr[0] * Ji[0][Jc] + dr[1] * Ji[1][Jc] + dr[2] * Ji[2][Jc];
    }
  }
  return bad;
}

/* Number of nodes and elements: the table's when the restriction is a table, else the lattice's. */
static int64_t mesh_nodes(const or_mesh* m, const elem_tab* t) {
  return m->conn ? m->n_nodes : (int64_t)t->nx1 * t->ny1 * (m->p * m->nz + 1);
}
static int64_t mesh_elems(const or_mesh* m) {
  return m->conn ? m->n_elem : (int64_t)m->nx * m->ny * m->nz;
}

/* Global nodes of element e (the restriction E_e): the table's row, or lattice arithmetic. */
static void elem_nodes(const or_mesh* m, const elem_tab* t, int64_t e, int64_t* idx) {
  if (m->conn) {
    for (int a = 0; a < t->nP; a++) idx[a] = m->conn[e * t->nP + a];
    return;
  }
  int64_t ex = e % m->nx, ey = (e / m->nx) % m->ny, ez = e / ((int64_t)m->nx * m->ny);
  int P = t->P;
  for (int az = 0; az < P; az++)
    for (int ay = 0; ay < P; ay++)
      for (int ax = 0; ax < P; ax++) {
        int64_t gx = ex * m->p + ax, gy = ey * m->p + ay, gz = ez * m->p + az;
        idx[ax + P * (ay + P * az)] = gx + (int64_t)t->nx1 * (gy + (int64_t)t->ny1 * gz);
      }
}

/* Interpolate element nodal data (4 fields) to one qp: G, phi, grad phi. */
static void interp_qp(const elem_tab* t, int qq, const double* ze /*[4][nP]*/, double G[9],
                      double* phi, double gphi[3]) {
  const double* N = t->N + qq * t->nP;
  const double* dN = t->dN + (size_t)qq * t->nP * 3;
  for (int k = 0; k < 9; k++) G[k] = 0.0;
  *phi = 0.0;
  gphi[0] = gphi[1] = gphi[2] = 0.0;
  for (int a = 0; a < t->nP; a++) {
    for (int i = 0; i < 3; i++)
      for (int J = 0; J < 3; J++) G[i * 3 + J] += ze[i * t->nP + a] * dN[a * 3 + J];
    *phi += ze[3 * t->nP + a] * N[a];
    for (int J = 0; J < 3; J++) gphi[J] += ze[3 * t->nP + a] * dN[a * 3 + J];
  }
}

/* re[4][nP] += wdet * B^T (P, f0, f1) at one qp */
static void test_qp(const elem_tab* t, int qq, double wdet, const double P[9], double f0,
                    const double f1[3], double* re) {
  const double* N = t->N + qq * t->nP;
  const double* dN = t->dN + (size_t)qq * t->nP * 3;
  for (int a = 0; a < t->nP; a++) {
    for (int i = 0; i < 3; i++) {
      double s = 0.0;
      for (int J = 0; J < 3; J++) s += P[i * 3 + J] * dN[a * 3 + J];
      re[i * t->nP + a] += wdet * s;
    }
    double s = N[a] * f0;
    for (int J = 0; J < 3; J++) s += f1[J] * dN[a * 3 + J];
    re[3 * t->nP + a] += wdet * s;
  }
}

enum { K_RES = 0, K_JAC = 1, K_ADJ = 2 };

typedef struct {
  const or_mesh* m; const or_phase* ph; int nph;
  const or_branch* xbr; int n_extra;  /* [nph][n_extra] extra branches */
  const or_frac* fr;
  const uint8_t* phase; const double* state; const double* xstate; const double* phi_n;
  const double* z; const double* w; /* dz or v */
} apply_args;

/* Element-local result of one element: out[4][nP]; gp[nph*3] for the adjoint. */
static int elem_apply(const apply_args* A, const elem_tab* t, int kind, int64_t e, double* out,
                      double* gp, int64_t* idx, double* ze, double* we) {
  const or_mesh* m = A->m;
  int nP = t->nP, nQ = t->nQ;
  int64_t n_nodes = mesh_nodes(m, t);
  int64_t n_q = mesh_elems(m) * nQ;
  int bad = 0;
  elem_nodes(m, t, e, idx);
  for (int f = 0; f < 4; f++)
    for (int a = 0; a < nP; a++) {
      ze[f * nP + a] = A->z[f * n_nodes + idx[a]];
      we[f * nP + a] = A->w ? A->w[f * n_nodes + idx[a]] : 0.0;
    }
  /* mapped geometry: the element's own gradients and weights in a copy of the table */
  elem_tab te;
  double* geo = NULL;
  if (m->X) {
    geo = (double*)malloc(sizeof(double) * ((size_t)nQ * nP * 3 + nQ));
    if (!geo) return -1;
    te = *t;
    te.dN = geo;
    te.wdet = geo + (size_t)nQ * nP * 3;
    bad |= elem_geometry(m, t, idx, te.dN, te.wdet);
    t = &te;
  }
  for (int k = 0; k < 4 * nP; k++) out[k] = 0.0;
  for (int qq = 0; qq < nQ; qq++) {
    int64_t gq = e * nQ + qq;
    int pid = A->phase[gq];
    if (pid >= A->nph) { free(geo); return -1; }
    double G[9], phi, gphi[3], st[8], xs[7 * OR_MAX_EXTRA];
    interp_qp(t, qq, ze, G, &phi, gphi);
    double phin = 0.0;
    for (int a = 0; a < nP; a++) phin += A->phi_n[idx[a]] * t->N[qq * nP + a];
    for (int k = 0; k < 8; k++) st[k] = A->state[k * n_q + gq];
    for (int k = 0; k < 7 * A->n_extra; k++) xs[k] = A->xstate[k * n_q + gq];
    mb_point pt;
    mb_eval(&A->ph[pid], A->xbr + (size_t)pid * A->n_extra, A->n_extra, A->fr, G, phi, phin, st, xs, &pt);
    const qp_state* s = &pt.s[0];
    bad |= pt.nonphysical;
    double wdet = t->wdet[qq];
    double c0 = s->c0, kf = A->fr->s_phi * 2.0 * pt.m[0].Gc * A->fr->l0 / c0;
    if (kind == K_RES) {
      double P[9], f1[3];
      first_piola(pt.tau_degr, s->Fi, P);
      for (int J = 0; J < 3; J++) f1[J] = kf * gphi[J];
      test_qp(t, qq, wdet, P, A->fr->s_phi * s->L, f1, out);
    } else if (kind == K_JAC) {
      double dG[9], dphi, dgphi[3], dP[9], df0, df1[3];
      interp_qp(t, qq, we, dG, &dphi, dgphi);
      mb_tangent(&pt, A->fr, dG, dphi, dgphi, dP, &df0, df1);
      test_qp(t, qq, wdet, dP, df0, df1, out);
    } else {
      /* cotangent at the qp, in the output pairing of test_qp: (grad v_u, v_phi, grad v_phi) */
      double cv[13], vphi;
      interp_qp(t, qq, we, cv, &vphi, cv + 10);
      cv[9] = vphi;
      /* explicit pointwise tangent matrix T (13 x 13), column k = T e_k */
      double T[13][13];
      for (int k = 0; k < 13; k++) {
        double in[13] = {0};
        in[k] = 1.0;
        double dP[9], df0, df1[3];
        mb_tangent(&pt, A->fr, in, in[9], in + 10, dP, &df0, df1);
        for (int r = 0; r < 9; r++) T[r][k] = dP[r];
        T[9][k] = df0;
        for (int r = 0; r < 3; r++) T[10 + r][k] = df1[r];
      }
      double g[13];
      for (int k = 0; k < 13; k++) {
        double sum = 0.0;
        for (int r = 0; r < 13; r++) sum += T[r][k] * cv[r];
        g[k] = sum;
      }
      test_qp(t, qq, wdet, g, g[9], g + 10, out);
      /* parameter partials, paired with the same cotangent */
      double dPp[27], df0p[3], df1p[9];
      qp_param_partials(&pt.m[0], A->fr, s, gphi, dPp, df0p, df1p);
      for (int k = 0; k < 3; k++) {
        double sum = df0p[k] * cv[9];
        for (int r = 0; r < 9; r++) sum += dPp[9 * k + r] * cv[r];
        for (int r = 0; r < 3; r++) sum += df1p[3 * k + r] * cv[10 + r];
        gp[pid * 3 + k] += wdet * sum;
      }
    }
  }
  free(geo);
  return bad;
}

static int run_apply(const apply_args* A, int kind, double* outv, double* gparams,
                     const int32_t* elems, int64_t n_elems) {
  const or_mesh* m = A->m;
  if (!m || !A->ph || A->nph < 1 || !A->fr || !A->phase || !A->state || !A->z || !outv) return -1;
  if (A->n_extra < 0 || A->n_extra > OR_MAX_EXTRA || (A->n_extra > 0 && (!A->xbr || !A->xstate))) return -1;
  if (m->conn && (!m->X || m->n_elem < 0 || m->n_nodes < 1)) return -1;
  elem_tab t;
  if (make_tab(m, &t)) return -1;
  int64_t ne_all = mesh_elems(m);
  int64_t n = elems ? n_elems : ne_all;
  int64_t n_nodes = mesh_nodes(m, &t);
  if (m->conn) {
    for (int64_t k = 0; k < ne_all * t.nP; k++)
      if (m->conn[k] < 0 || m->conn[k] >= n_nodes) { free_tab(&t); return -1; }
  }
  int nP = t.nP;
  double* eres = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 4 * nP);
  /* per-element parameter partials, summed serially afterwards (deterministic) */
  double* gpart = (double*)calloc((size_t)(n > 0 ? n : 1) * A->nph * 3, sizeof(double));
  int bad = 0, err = 0;
  if (!eres || !gpart) { free(eres); free(gpart); free_tab(&t); return -1; }
#pragma omp parallel reduction(| : bad, err)
  {
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * nP);
    double* ze = (double*)malloc(sizeof(double) * 4 * nP);
    double* we = (double*)malloc(sizeof(double) * 4 * nP);
#pragma omp for schedule(dynamic, 4)
    for (int64_t k = 0; k < n; k++) {
      int64_t e = elems ? elems[k] : k;
      if (e < 0 || e >= ne_all) { err = 1; continue; }
      int r = elem_apply(A, &t, kind, e, eres + (size_t)k * 4 * nP, gpart + (size_t)k * A->nph * 3,
                         idx, ze, we);
      if (r < 0) err = 1; else bad |= r;
    }
    free(idx); free(ze); free(we);
  }
  /* serial scatter-add in element-list order */
  memset(outv, 0, sizeof(double) * 4 * n_nodes);
  if (!err) {
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * nP);
    for (int64_t k = 0; k < n; k++) {
      int64_t e = elems ? elems[k] : k;
      elem_nodes(m, &t, e, idx);
      for (int f = 0; f < 4; f++)
        for (int a = 0; a < nP; a++) outv[f * n_nodes + idx[a]] += eres[(size_t)k * 4 * nP + f * nP + a];
    }
    free(idx);
    if (gparams) {
      for (int k = 0; k < A->nph * 3; k++) {
        double s = 0.0;
        for (int64_t j = 0; j < n; j++) s += gpart[(size_t)j * A->nph * 3 + k];
        gparams[k] = s;
      }
    }
  }
  free(eres); free(gpart); free_tab(&t);
  if (err) return -1;
  return bad ? 1 : 0;
}

int or_residual(const or_mesh* m, const or_phase* ph, int nph, const or_branch* xbr, int n_extra,
                const or_frac* fr, const uint8_t* phase, const double* state, const double* xstate,
                const double* phi_n, const double* z, double* r, const int32_t* elems, int64_t n_elems) {
  apply_args A = {m, ph, nph, xbr, n_extra, fr, phase, state, xstate, phi_n, z, NULL};
  return run_apply(&A, K_RES, r, NULL, elems, n_elems);
}

int or_jacobian(const or_mesh* m, const or_phase* ph, int nph, const or_branch* xbr, int n_extra,
                const or_frac* fr, const uint8_t* phase, const double* state, const double* xstate,
                const double* phi_n, const double* z, const double* dz, double* y,
                const int32_t* elems, int64_t n_elems) {
  if (!dz) return -1;
  apply_args A = {m, ph, nph, xbr, n_extra, fr, phase, state, xstate, phi_n, z, dz};
  return run_apply(&A, K_JAC, y, NULL, elems, n_elems);
}

int or_adjoint(const or_mesh* m, const or_phase* ph, int nph, const or_branch* xbr, int n_extra,
               const or_frac* fr, const uint8_t* phase, const double* state, const double* xstate,
               const double* phi_n, const double* z, const double* v, double* gz, double* gparams,
               const int32_t* elems, int64_t n_elems) {
  if (!v) return -1;
  apply_args A = {m, ph, nph, xbr, n_extra, fr, phase, state, xstate, phi_n, z, v};
  return run_apply(&A, K_ADJ, gz, gparams, elems, n_elems);
}

int or_element_jacobian(const or_mesh* m, const or_phase* ph, int nph, const or_branch* xbr, int n_extra,
                        const or_frac* fr, const uint8_t* phase, const double* state, const double* xstate,
                        const double* phi_n, const double* z, int64_t e, double* Ke) {
  if (n_extra < 0 || n_extra > OR_MAX_EXTRA || (n_extra > 0 && (!xbr || !xstate))) return -1;
  if (m->conn && !m->X) return -1;
  elem_tab t;
  if (make_tab(m, &t)) return -1;
  int nP = t.nP, nd = 4 * nP;
  int64_t n_nodes = mesh_nodes(m, &t);
  /* column j = element apply of the unit element vector e_j; a unit vector
   * placed in a private global-size buffer keeps the same gather path */
  double* unit = (double*)calloc((size_t)4 * n_nodes, sizeof(double));
  double* col = (double*)malloc(sizeof(double) * nd);
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * nP);
  double* ze = (double*)malloc(sizeof(double) * nd);
  double* we = (double*)malloc(sizeof(double) * nd);
  apply_args A = {m, ph, nph, xbr, n_extra, fr, phase, state, xstate, phi_n, z, unit};
  int bad = 0;
  elem_nodes(m, &t, e, idx);
  for (int j = 0; j < nd; j++) {
    int f = j / nP, a = j % nP;
    unit[f * n_nodes + idx[a]] = 1.0;
    int r = elem_apply(&A, &t, K_JAC, e, col, NULL, idx, ze, we);
    unit[f * n_nodes + idx[a]] = 0.0;
    if (r < 0) { bad = -1; break; }
    bad |= r;
    for (int i = 0; i < nd; i++) Ke[(size_t)i * nd + j] = col[i];
  }
  free(unit); free(col); free(idx); free(ze); free(we); free_tab(&t);
  return bad;
}

/* Commit over all points of the mesh: state_new[8][n_q] from z (see or_qf_commit); with
 * extra branches also xstate_new[7*n_extra][n_q] (see or_qf_commit_mb). */
int or_commit_state_mb(const or_mesh* m, const or_phase* ph, int nph, const or_branch* xbr, int n_extra,
                       const or_frac* fr, const uint8_t* phase, const double* state, const double* xstate,
                       const double* z, double* state_new, double* xstate_new) {
  if (n_extra < 0 || n_extra > OR_MAX_EXTRA || (n_extra > 0 && (!xbr || !xstate || !xstate_new))) return -1;
  if (m->conn && !m->X) return -1;
  elem_tab t;
  if (make_tab(m, &t)) return -1;
  int nP = t.nP, nQ = t.nQ;
  int64_t n_nodes = mesh_nodes(m, &t);
  int64_t n_el = mesh_elems(m);
  int64_t n_q = n_el * nQ;
  int err = 0;
#pragma omp parallel
  {
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * nP);
    double* ze = (double*)malloc(sizeof(double) * 4 * nP);
    double* geo = (double*)malloc(sizeof(double) * ((size_t)nQ * nP * 3 + nQ));
#pragma omp for schedule(static)
    for (int64_t e = 0; e < n_el; e++) {
      elem_nodes(m, &t, e, idx);
      for (int f = 0; f < 4; f++)
        for (int a = 0; a < nP; a++) ze[f * nP + a] = z[f * n_nodes + idx[a]];
      elem_tab te = t;
      if (m->X) {
        te.dN = geo;
        te.wdet = geo + (size_t)nQ * nP * 3;
        elem_geometry(m, &t, idx, te.dN, te.wdet);
      }
      for (int qq = 0; qq < nQ; qq++) {
        int64_t gq = e * nQ + qq;
        int pid = phase[gq];
        if (pid >= nph) { err = 1; continue; }
        double G[9], phi, gphi[3], st[8], sn[8], xs[7 * OR_MAX_EXTRA], xn[7 * OR_MAX_EXTRA];
        interp_qp(&te, qq, ze, G, &phi, gphi);
        for (int k = 0; k < 8; k++) st[k] = state[k * n_q + gq];
        if (n_extra == 0) {
          or_qf_commit(&ph[pid], fr, G, phi, st, sn);
        } else {
          for (int k = 0; k < 7 * n_extra; k++) xs[k] = xstate[k * n_q + gq];
          or_qf_commit_mb(&ph[pid], xbr + (size_t)pid * n_extra, n_extra, fr, G, phi, st, xs, sn, xn);
          for (int k = 0; k < 7 * n_extra; k++) xstate_new[k * n_q + gq] = xn[k];
        }
        for (int k = 0; k < 8; k++) state_new[k * n_q + gq] = sn[k];
      }
    }
    free(idx); free(ze); free(geo);
  }
  free_tab(&t);
  return err ? -1 : 0;
}

int or_commit_state(const or_mesh* m, const or_phase* ph, int nph, const or_frac* fr, const uint8_t* phase,
                    const double* state, const double* z, double* state_new) {
  return or_commit_state_mb(m, ph, nph, NULL, 0, fr, phase, state, NULL, z, state_new, NULL);
}
