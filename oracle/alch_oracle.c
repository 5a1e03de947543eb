/*
 * CPU oracle for the alchemical short-range nonbonded potential.
 *
 * TEST INFRASTRUCTURE ONLY.  This file defines, in plain FP64 C, what the GPU
 * library must compute.  It shares no code, header, table or constant
 * generator with the GPU library; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.
 *
 * What is computed (one periodic orthorhombic box at a time):
 *   every unordered atom pair i<j that is not excluded and lies within the
 *   cutoff under the minimum-image convention is evaluated once.
 *   - Pairs inside the solvent or inside the solute are lambda independent
 *     (the U_solv and U_solu terms of the paper's potential decomposition,
 *     Linear Basis Function section, eq. 4).
 *   - Solute-solvent pairs are the alchemically coupled ones (the coupling
 *     route of the same section): only these depend on lambda.
 *
 * Pair potential (units: Angstrom, kcal/mol, e):
 *   LJ(r)    = 4 eps [(sig/r)^12 - (sig/r)^6], Lorentz-Berthelot combination
 *              sig = (sig_i + sig_j)/2, eps = sqrt(eps_i eps_j).
 *   S(r)     = 1 - S22((r - r_s)/(r_c - r_s)) on (r_s, r_c), 1 below r_s;
 *              S22 is the paper's smoothstep (eq. 9), applied to every
 *              Lennard-Jones-like term (a switch starting before the
 *              cutoff, Simulation Details section).
 *   D(r)     = damped shifted-force Coulomb kernel
 *              erfc(a r)/r - erfc(a r_c)/r_c
 *              + [erfc(a r_c)/r_c^2 + 2a/sqrt(pi) exp(-a^2 r_c^2)/r_c] (r - r_c),
 *              which vanishes with its first derivative at r_c; with the
 *              Ewald flag (OR_ELEC_EWALD) D(r) = erfc(a r)/r instead, the
 *              real-space part of an Ewald sum (long-range electrostatics
 *              by PME, Simulation Details section; oracle/pme.py adds the
 *              reciprocal, self and exclusion parts).
 *   plain    u = LJ(r) S(r) + k_e q_i q_j D(r)
 *   Beutler  u = lv 4 eps (x^2 - x) S(r) + le k_e q_i q_j D(r),
 *              x = 1/(alpha_sc (1 - lv) + (r/sig)^6),
 *              lv = min(1, 2 lambda), le = max(0, 2 lambda - 1)
 *              (the conventional soft-core form the paper contrasts with
 *              its LBF form).
 *   LBF      u = hA(lambda) [LJ S + k_e q q D] + hB(lambda) eps u_cap(r/sig) S
 *              with u_cap from eq. 6 and hA, hB from eqs. 7-10.
 *
 * dU/dlambda (eq. 2 integrates its conditional mean): Beutler uses the left
 * derivative at the kink lambda = 1/2 (dlv/dlambda = 2 for lambda <= 1/2,
 * dle/dlambda = 2 for lambda > 1/2); LBF is hA' U_A + hB' U_B.
 *
 * The canonical pair test: positions are wrapped x' = x - L floor(x/L); the
 * displacement d = x'_j - x'_i is shifted by -L if d > L/2 and by +L if
 * d < -L/2; r^2 = (dx*dx + dy*dy) + dz*dz evaluated without fused
 * multiply-add.  A pair is evaluated when r^2 < r_c^2 and belongs to the
 * neighbour-list pair set when r^2 < (r_c + skin)^2.
 *
 * Sums are FP64 with Neumaier compensation in a fixed order; erfc and exp
 * come from libm.  Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_KE 332.06371          /* Coulomb constant, kcal A / (mol e^2) */
#define OR_NTERMS 10
/* term slots */
enum {
  T_SOLV_SOLV = 0, T_SOLU_SOLU = 1, T_SS_VDW = 2, T_SS_ELEC = 3, T_UA = 4, T_UB = 5,
  T_DUDL_VDW = 6, T_DUDL_ELEC = 7, T_TOTAL = 8, T_DUDL = 9
};
enum { SCHED_BEUTLER = 0, SCHED_LBF = 1 };

typedef struct {
  double cutoff, switch_width, dsf_alpha, sc_alpha;
  int schedule;
  int ewald;  /* 1: Ewald real space erfc(a r)/r in place of D(r) */
} or_params;

/* The schedule argument of the entry points carries the electrostatics in
 * bit 2: clear = damped shifted force D(r); OR_ELEC_EWALD = the real-space
 * part of an Ewald sum, erfc(a r)/r truncated at r_c without shift (the
 * reciprocal part, self and exclusion terms are computed elsewhere). */
#define OR_ELEC_EWALD 4
static or_params make_params(double cutoff, double switch_width, double alpha, double sc_alpha, int code) {
  or_params p = {cutoff, switch_width, alpha, sc_alpha, code & 3, (code & OR_ELEC_EWALD) ? 1 : 0};
  return p;
}

/* ---------------------------------------------------------------- helpers */

typedef struct { double s, c; } ksum;  /* Neumaier compensated sum */
static void ks_add(ksum *k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x; else k->c += (x - t) + k->s;
  k->s = t;
}
static double ks_val(const ksum *k) { return k->s + k->c; }

/* paper eq. 9: S22(x) = 6x^5 - 15x^4 + 10x^3 and its derivative */
static double s22(double x) { return 6 * pow(x, 5) - 15 * pow(x, 4) + 10 * pow(x, 3); }
static double s22_d(double x) { return 30 * pow(x, 4) - 60 * pow(x, 3) + 30 * pow(x, 2); }
/* paper eq. 10: S32(x) = 10x^6 - 24x^5 + 15x^4 for 0 < x <= 1, 0 for x <= 0 */
static double s32(double x) {
  if (x <= 0) return 0.0;
  if (x > 1) x = 1;  /* the smoothstep saturates at 1 */
  return 10 * pow(x, 6) - 24 * pow(x, 5) + 15 * pow(x, 4);
}
static double s32_d(double x) {
  if (x <= 0 || x >= 1) return 0.0;
  return 60 * pow(x, 5) - 120 * pow(x, 4) + 60 * pow(x, 3);
}

/* paper eqs. 7-8: hA = S32((l - 0.35)/0.65), hB = S22(l) - hA */
void oracle_lbf_switches(double l, double out[4]) {
  double xa = (l - 0.35) / 0.65;
  double hA = s32(xa), dhA = s32_d(xa) / 0.65;
  double hB = s22(l) - hA, dhB = s22_d(l) - dhA;
  out[0] = hA; out[1] = hB; out[2] = dhA; out[3] = dhB;
}

/* paper eq. 6: u_cap(x) and du_cap/dx */
void oracle_ucap(double x, double out[2]) {
  if (x < 1.0) {
    out[0] = -868.0 * pow(x, 6) + 2188.8 * pow(x, 5) - 1440.0 * pow(x, 4) + 119.2;
    out[1] = -6 * 868.0 * pow(x, 5) + 5 * 2188.8 * pow(x, 4) - 4 * 1440.0 * pow(x, 3);
  } else {
    out[0] = 4.0 * pow(x, -12) - 4.0 * pow(x, -6);
    out[1] = -48.0 * pow(x, -13) + 24.0 * pow(x, -7);
  }
}

/* switch S(r) and dS/dr; width 0 means hard truncation */
void oracle_switch(double r, double rc, double width, double out[2]) {
  if (width <= 0.0 || r <= rc - width) { out[0] = 1.0; out[1] = 0.0; return; }
  double t = (r - (rc - width)) / width;
  out[0] = 1.0 - s22(t);
  out[1] = -s22_d(t) / width;
}

/* damped shifted-force kernel D(r) and dD/dr */
void oracle_dsf(double r, double rc, double a, double out[2]) {
  const double two_over_sqrt_pi = 2.0 / sqrt(M_PI);
  double erfc_c = erfc(a * rc);
  double slope = erfc_c / (rc * rc) + a * two_over_sqrt_pi * exp(-a * a * rc * rc) / rc;
  out[0] = erfc(a * r) / r - erfc_c / rc + slope * (r - rc);
  out[1] = -erfc(a * r) / (r * r) - a * two_over_sqrt_pi * exp(-a * a * r * r) / r + slope;
}

/* Ewald real-space kernel erfc(a r)/r and its r derivative */
void oracle_ewald_real(double r, double a, double out[2]) {
  const double two_over_sqrt_pi = 2.0 / sqrt(M_PI);
  out[0] = erfc(a * r) / r;
  out[1] = -erfc(a * r) / (r * r) - a * two_over_sqrt_pi * exp(-a * a * r * r) / r;
}

/* Lennard-Jones 4 eps [(s/r)^12 - (s/r)^6] and its r, sigma, eps derivatives */
static void lj(double r, double sig, double eps, double *u, double *du_dr, double *du_ds, double *du_de) {
  double sr6 = pow(sig / r, 6), sr12 = sr6 * sr6;
  *u = 4 * eps * (sr12 - sr6);
  *du_dr = 4 * eps * (-12 * sr12 + 6 * sr6) / r;
  *du_ds = 4 * eps * (12 * sr12 - 6 * sr6) / sig;
  *du_de = 4 * (sr12 - sr6);
}

/* ------------------------------------------------------------- pair kernel */

/* Per-pair result: energy contributions by slot, dU/dr, dU/dlambda parts,
 * and derivatives with respect to the combined parameters sig, eps, qq. */
typedef struct {
  double u_plain;            /* plain pair energy (non-alchemical pairs) */
  double ss_vdw, ss_elec;    /* lambda-scaled solute-solvent energies */
  double ua, ub;             /* LBF bases (zero for Beutler) */
  double dl_vdw, dl_elec;    /* dU/dlambda parts */
  double du_dr;              /* total dU/dr */
  double du_dsig, du_deps, du_dqq;
} pair_out;

typedef struct {
  double lv, le, dlv, dle;   /* Beutler stage factors */
  double hA, hB, dhA, dhB;   /* LBF switches */
} lam_state;

static void lam_state_init(double lambda, int schedule, lam_state *s) {
  memset(s, 0, sizeof(*s));
  if (schedule == SCHED_BEUTLER) {
    s->lv = fmin(1.0, 2.0 * lambda);
    s->le = fmax(0.0, 2.0 * lambda - 1.0);
    s->dlv = (lambda <= 0.5) ? 2.0 : 0.0;
    s->dle = (lambda > 0.5) ? 2.0 : 0.0;
  } else {
    double h[4];
    oracle_lbf_switches(lambda, h);
    s->hA = h[0]; s->hB = h[1]; s->dhA = h[2]; s->dhB = h[3];
  }
}

static void eval_pair(double r, double sig, double eps, double qq, int alchemical, const or_params *p,
                      const lam_state *ls, pair_out *o) {
  memset(o, 0, sizeof(*o));
  double sw[2], dsf[2];
  oracle_switch(r, p->cutoff, p->switch_width, sw);
  if (p->ewald) oracle_ewald_real(r, p->dsf_alpha, dsf);
  else oracle_dsf(r, p->cutoff, p->dsf_alpha, dsf);
  double ulj, dlj_dr, dlj_ds, dlj_de;
  lj(r, sig, eps, &ulj, &dlj_dr, &dlj_ds, &dlj_de);
  /* switched LJ and Coulomb pieces shared by plain pairs and LBF's U_A */
  double vdw = ulj * sw[0];
  double dvdw_dr = dlj_dr * sw[0] + ulj * sw[1];
  double elec = OR_KE * qq * dsf[0];
  double delec_dr = OR_KE * qq * dsf[1];
  if (!alchemical) {
    o->u_plain = vdw + elec;
    o->du_dr = dvdw_dr + delec_dr;
    o->du_dsig = dlj_ds * sw[0];
    o->du_deps = dlj_de * sw[0];
    o->du_dqq = OR_KE * dsf[0];
    return;
  }
  if (p->schedule == SCHED_BEUTLER) {
    double a = p->sc_alpha, lv = ls->lv;
    double y = pow(r / sig, 6);               /* (r/sig)^6 */
    double x = 1.0 / (a * (1.0 - lv) + y);
    double core = 4 * eps * (x * x - x);      /* soft-core LJ without lv and S */
    double dcore_dx = 4 * eps * (2 * x - 1);
    double dx_dy = -x * x;
    double dy_dr = 6 * y / r, dy_ds = -6 * y / sig;
    double dx_dlv = a * x * x;
    o->ss_vdw = lv * core * sw[0];
    o->ss_elec = ls->le * elec;
    o->du_dr = lv * (dcore_dx * dx_dy * dy_dr * sw[0] + core * sw[1]) + ls->le * delec_dr;
    /* d/dlv [lv core(x(lv))] = core + lv dcore/dx dx/dlv */
    o->dl_vdw = ls->dlv * (core + lv * dcore_dx * dx_dlv) * sw[0];
    o->dl_elec = ls->dle * elec;
    o->du_dsig = lv * dcore_dx * dx_dy * dy_ds * sw[0];
    o->du_deps = lv * 4 * (x * x - x) * sw[0];
    o->du_dqq = ls->le * OR_KE * dsf[0];
  } else {
    double uc[2];
    oracle_ucap(r / sig, uc);
    double ub = eps * uc[0] * sw[0];
    double dub_dr = eps * (uc[1] / sig * sw[0] + uc[0] * sw[1]);
    double ua = vdw + elec;
    o->ua = ua;
    o->ub = ub;
    o->ss_vdw = ls->hA * vdw + ls->hB * ub;
    o->ss_elec = ls->hA * elec;
    o->du_dr = ls->hA * (dvdw_dr + delec_dr) + ls->hB * dub_dr;
    o->dl_vdw = ls->dhA * vdw + ls->dhB * ub;
    o->dl_elec = ls->dhA * elec;
    o->du_dsig = ls->hA * dlj_ds * sw[0] + ls->hB * eps * uc[1] * (-r / (sig * sig)) * sw[0];
    o->du_deps = ls->hA * dlj_de * sw[0] + ls->hB * uc[0] * sw[0];
    o->du_dqq = ls->hA * OR_KE * dsf[0];
  }
}

/* ---------------------------------------------------------- minimum image */

static void wrap3(const double *x, const double *box, double *out) {
  for (int d = 0; d < 3; ++d) out[d] = x[d] - box[d] * floor(x[d] / box[d]);
}

/* canonical displacement j - i and r^2 (no FMA: compiled with -ffp-contract=off) */
static double min_image(const double *wi, const double *wj, const double *box, double *d) {
  for (int k = 0; k < 3; ++k) {
    double v = wj[k] - wi[k];
    if (v > 0.5 * box[k]) v -= box[k];
    else if (v < -0.5 * box[k]) v += box[k];
    d[k] = v;
  }
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* exclusion lookup: excl sorted by (i, j) with i < j; CSR start per atom */
typedef struct { const int32_t *excl; int64_t *start; int n; } excl_index;

static int excl_build(int n, int n_excl, const int32_t *excl, excl_index *ix) {
  ix->excl = excl; ix->n = n;
  ix->start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!ix->start) return -1;
  for (int e = 0; e < n_excl; ++e) {
    int i = excl[2 * e], j = excl[2 * e + 1];
    if (i < 0 || j <= i || j >= n) { free(ix->start); return -2; }
    if (e > 0) {
      int pi = excl[2 * e - 2], pj = excl[2 * e - 1];
      if (i < pi || (i == pi && j <= pj)) { free(ix->start); return -3; }
    }
    ix->start[i + 1]++;
  }
  for (int i = 0; i < n; ++i) ix->start[i + 1] += ix->start[i];
  return 0;
}
static int is_excluded(const excl_index *ix, int i, int j) {
  for (int64_t e = ix->start[i]; e < ix->start[i + 1]; ++e)
    if (ix->excl[2 * e + 1] == j) return 1;
  return 0;
}

/* ------------------------------------------------------------- public API */

/*
 * Evaluate one box.  Inputs: n atoms, positions [n][3], per-atom type and
 * solute flag, exclusions [n_excl][2] (i<j, sorted), box edges [3], per-type
 * sigma/epsilon/charge [n_types].  Outputs (each may be NULL):
 *   terms[10]      slots as in the enum above;
 *   forces[n][3]   -dU/dx;
 *   pgrad[3][n_types]  dU/dsigma_t, dU/dsqrt(eps_t), dU/dq_t (per type);
 *   n_pairs        pairs with r < r_c that were evaluated.
 * Returns 0 on success, <0 on invalid input.
 */
int oracle_eval(int n, const double *pos, const int32_t *type, const uint8_t *is_solute, int n_excl,
                const int32_t *excl, const double *box, int n_types, const double *sigma, const double *epsilon,
                const double *charge, double cutoff, double switch_width, double dsf_alpha, double sc_alpha,
                int schedule, double lambda, double *terms, double *forces, double *pgrad, int64_t *n_pairs,
                double *abs_terms, int n_threads) {
  if (n < 0 || cutoff <= 0 || ((schedule & 3) != SCHED_BEUTLER && (schedule & 3) != SCHED_LBF) ||
      (schedule & ~(3 | OR_ELEC_EWALD)) != 0)
    return -1;
  for (int d = 0; d < 3; ++d)
    if (!(box[d] >= 2.0 * cutoff)) return -4;
  for (int i = 0; i < n; ++i)
    if (type[i] < 0 || type[i] >= n_types) return -5;
  excl_index ix;
  if (excl_build(n, n_excl, excl, &ix) != 0) return -6;
  const or_params p = make_params(cutoff, switch_width, dsf_alpha, sc_alpha, schedule);
  lam_state ls;
  lam_state_init(lambda, p.schedule, &ls);

  double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) wrap3(pos + 3 * i, box, w + 3 * i);
  const double rc2 = cutoff * cutoff;
#ifdef _OPENMP
  int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
  int nt = 1;
  (void)n_threads;
#endif
  /* per-thread accumulators, combined in thread order afterwards */
  enum { ACC_PLAIN_SOLV, ACC_PLAIN_SOLU, ACC_SS_VDW, ACC_SS_ELEC, ACC_UA, ACC_UB, ACC_DL_VDW, ACC_DL_ELEC, NACC };
  /* sums of |pair contribution| per slot: the scale against which summed
   * quantities with cancellation are compared */
  double *absth = (double *)calloc((size_t)nt * NACC, sizeof(double));
  ksum *acc = (ksum *)calloc((size_t)nt * NACC, sizeof(ksum));
  double *fth = forces ? (double *)calloc((size_t)nt * 3 * (size_t)n, sizeof(double)) : NULL;
  double *gth = pgrad ? (double *)calloc((size_t)nt * 3 * (size_t)n_types, sizeof(double)) : NULL;
  int64_t *cnt = (int64_t *)calloc((size_t)nt, sizeof(int64_t));

#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
  {
#ifdef _OPENMP
    int tid = omp_get_thread_num();
#else
    int tid = 0;
#endif
    ksum *a = acc + (size_t)tid * NACC;
    double *f = fth ? fth + (size_t)tid * 3 * n : NULL;
    double *g = gth ? gth + (size_t)tid * 3 * n_types : NULL;
#ifdef _OPENMP
#pragma omp for schedule(static, 16)
#endif
    for (int i = 0; i < n; ++i) {
      for (int j = i + 1; j < n; ++j) {
        double d[3];
        double r2 = min_image(w + 3 * i, w + 3 * j, box, d);
        if (!(r2 < rc2)) continue;
        if (is_excluded(&ix, i, j)) continue;
        int ti = type[i], tj = type[j];
        double sig = 0.5 * (sigma[ti] + sigma[tj]);
        double eps = sqrt(epsilon[ti] * epsilon[tj]);
        double qq = charge[ti] * charge[tj];
        int alch = (is_solute[i] != 0) != (is_solute[j] != 0);
        double r = sqrt(r2);
        pair_out o;
        eval_pair(r, sig, eps, qq, alch, &p, &ls, &o);
        cnt[tid]++;
        double *ab = absth + (size_t)tid * NACC;
        if (!alch) {
          if (is_solute[i]) ks_add(&a[ACC_PLAIN_SOLU], o.u_plain);
          else ks_add(&a[ACC_PLAIN_SOLV], o.u_plain);
          ab[is_solute[i] ? ACC_PLAIN_SOLU : ACC_PLAIN_SOLV] += fabs(o.u_plain);
        } else {
          ab[ACC_SS_VDW] += fabs(o.ss_vdw);
          ab[ACC_SS_ELEC] += fabs(o.ss_elec);
          ab[ACC_UA] += fabs(o.ua);
          ab[ACC_UB] += fabs(o.ub);
          ab[ACC_DL_VDW] += fabs(o.dl_vdw);
          ab[ACC_DL_ELEC] += fabs(o.dl_elec);
          ks_add(&a[ACC_SS_VDW], o.ss_vdw);
          ks_add(&a[ACC_SS_ELEC], o.ss_elec);
          ks_add(&a[ACC_UA], o.ua);
          ks_add(&a[ACC_UB], o.ub);
          ks_add(&a[ACC_DL_VDW], o.dl_vdw);
          ks_add(&a[ACC_DL_ELEC], o.dl_elec);
        }
        if (f) {
          /* force on j is -dU/dr * d/r, force on i the opposite */
          for (int k = 0; k < 3; ++k) {
            double fk = -o.du_dr * d[k] / r;
            f[3 * j + k] += fk;
            f[3 * i + k] -= fk;
          }
        }
        if (g) {
          /* sig = (s_i + s_j)/2; eps = e_i e_j with e = sqrt(epsilon); qq = q_i q_j */
          double ei = sqrt(epsilon[ti]), ej = sqrt(epsilon[tj]);
          g[0 * n_types + ti] += 0.5 * o.du_dsig;
          g[0 * n_types + tj] += 0.5 * o.du_dsig;
          g[1 * n_types + ti] += o.du_deps * ej;
          g[1 * n_types + tj] += o.du_deps * ei;
          g[2 * n_types + ti] += o.du_dqq * charge[tj];
          g[2 * n_types + tj] += o.du_dqq * charge[ti];
        }
      }
    }
  }
  ksum tot[NACC];
  memset(tot, 0, sizeof(tot));
  int64_t npairs = 0;
  for (int t = 0; t < nt; ++t) {
    for (int k = 0; k < NACC; ++k) ks_add(&tot[k], ks_val(&acc[(size_t)t * NACC + k]));
    npairs += cnt[t];
  }
  if (terms) {
    double e_solv = ks_val(&tot[ACC_PLAIN_SOLV]), e_solu = ks_val(&tot[ACC_PLAIN_SOLU]);
    double e_vdw = ks_val(&tot[ACC_SS_VDW]), e_elec = ks_val(&tot[ACC_SS_ELEC]);
    double dl_v = ks_val(&tot[ACC_DL_VDW]), dl_e = ks_val(&tot[ACC_DL_ELEC]);
    terms[T_SOLV_SOLV] = e_solv;
    terms[T_SOLU_SOLU] = e_solu;
    terms[T_SS_VDW] = e_vdw;
    terms[T_SS_ELEC] = e_elec;
    terms[T_UA] = ks_val(&tot[ACC_UA]);
    terms[T_UB] = ks_val(&tot[ACC_UB]);
    terms[T_DUDL_VDW] = dl_v;
    terms[T_DUDL_ELEC] = dl_e;
    ksum e = {0, 0};
    ks_add(&e, e_solv); ks_add(&e, e_solu); ks_add(&e, e_vdw); ks_add(&e, e_elec);
    terms[T_TOTAL] = ks_val(&e);
    terms[T_DUDL] = dl_v + dl_e;
  }
  if (forces) {
    memset(forces, 0, sizeof(double) * 3 * (size_t)n);
    for (int t = 0; t < nt; ++t)
      for (size_t k = 0; k < 3 * (size_t)n; ++k) forces[k] += fth[(size_t)t * 3 * n + k];
  }
  if (pgrad) {
    memset(pgrad, 0, sizeof(double) * 3 * (size_t)n_types);
    for (int t = 0; t < nt; ++t)
      for (int k = 0; k < 3 * n_types; ++k) pgrad[k] += gth[(size_t)t * 3 * n_types + k];
  }
  if (n_pairs) *n_pairs = npairs;
  if (abs_terms) {
    double ab[NACC];
    memset(ab, 0, sizeof(ab));
    for (int t = 0; t < nt; ++t)
      for (int k = 0; k < NACC; ++k) ab[k] += absth[(size_t)t * NACC + k];
    for (int k = 0; k < NACC; ++k) abs_terms[k] = ab[k];  /* slots 0-7 match the term slots */
    abs_terms[T_TOTAL] = ab[ACC_PLAIN_SOLV] + ab[ACC_PLAIN_SOLU] + ab[ACC_SS_VDW] + ab[ACC_SS_ELEC];
    abs_terms[T_DUDL] = ab[ACC_DL_VDW] + ab[ACC_DL_ELEC];
  }
  free(absth);
  free(w); free(acc); free(fth); free(gth); free(cnt); free(ix.start);
  return 0;
}

/*
 * Neighbour-list pair set: all i<j, not excluded, with canonical r^2 <
 * r_list^2.  Written as int32 pairs in (i, j) lexicographic order.  With
 * pairs == NULL only the count is returned.  Returns 0, or -2 if cap is
 * too small (n_out still holds the full count).
 */
int oracle_pairs(int n, const double *pos, int n_excl, const int32_t *excl, const double *box, double r_list,
                 int32_t *pairs, int64_t cap, int64_t *n_out) {
  excl_index ix;
  if (excl_build(n, n_excl, excl, &ix) != 0) return -6;
  double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) wrap3(pos + 3 * i, box, w + 3 * i);
  const double rl2 = r_list * r_list;
  int64_t m = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double d[3];
      double r2 = min_image(w + 3 * i, w + 3 * j, box, d);
      if (!(r2 < rl2) || is_excluded(&ix, i, j)) continue;
      if (pairs && m < cap) { pairs[2 * m] = i; pairs[2 * m + 1] = j; }
      ++m;
    }
  *n_out = m;
  free(w); free(ix.start);
  return (pairs && m > cap) ? -2 : 0;
}

/*
 * Energy of one atom with all its neighbours (used for O(N) finite
 * differences of the total energy in one coordinate of atom a).  Returns the
 * sum over j != a of the pair energies that involve a.
 */
double oracle_atom_energy(int a, int n, const double *pos, const int32_t *type, const uint8_t *is_solute,
                          int n_excl, const int32_t *excl, const double *box, int n_types, const double *sigma,
                          const double *epsilon, const double *charge, double cutoff, double switch_width,
                          double dsf_alpha, double sc_alpha, int schedule, double lambda) {
  (void)n_types;
  const or_params p = make_params(cutoff, switch_width, dsf_alpha, sc_alpha, schedule);
  lam_state ls;
  lam_state_init(lambda, p.schedule, &ls);
  double wa[3];
  wrap3(pos + 3 * a, box, wa);
  ksum e = {0, 0};
  for (int j = 0; j < n; ++j) {
    if (j == a) continue;
    int lo = a < j ? a : j, hi = a < j ? j : a;
    int ex = 0;
    for (int k = 0; k < n_excl; ++k)
      if (excl[2 * k] == lo && excl[2 * k + 1] == hi) { ex = 1; break; }
    if (ex) continue;
    double wj[3], d[3];
    wrap3(pos + 3 * j, box, wj);
    double r2 = (lo == a) ? min_image(wa, wj, box, d) : min_image(wj, wa, box, d);
    if (!(r2 < cutoff * cutoff)) continue;
    int ti = type[a], tj = type[j];
    pair_out o;
    int alch = (is_solute[a] != 0) != (is_solute[j] != 0);
    eval_pair(sqrt(r2), 0.5 * (sigma[ti] + sigma[tj]), sqrt(epsilon[ti] * epsilon[tj]), charge[ti] * charge[tj],
              alch, &p, &ls, &o);
    ks_add(&e, alch ? o.ss_vdw + o.ss_elec : o.u_plain);
  }
  return ks_val(&e);
}

/*
 * Per-atom sums for a selection of atoms (the plain definition restricted to
 * the pairs that involve each selected atom a): the force on a, -dU/dx_a,
 * the sum of the pair energies of a, the sum of the lambda derivatives of
 * its solute-solvent pairs and the number of its pairs within the cutoff.
 * Summed over all solute atoms the derivatives give dU/dlambda of the box,
 * since every solute-solvent pair has exactly one solute atom.  Outputs
 * [n_sel][3], [n_sel], [n_sel], [n_sel]; O(n) per selected atom.
 */
int oracle_atoms_terms(int n_sel, const int32_t *sel, int n, const double *pos, const int32_t *type,
                       const uint8_t *is_solute, int n_excl, const int32_t *excl, const double *box, int n_types,
                       const double *sigma, const double *epsilon, const double *charge, double cutoff,
                       double switch_width, double dsf_alpha, double sc_alpha, int schedule, double lambda,
                       double *force, double *energy, double *dudl, int64_t *n_pairs, int n_threads) {
  if (n < 0 || cutoff <= 0 || ((schedule & 3) != SCHED_BEUTLER && (schedule & 3) != SCHED_LBF) ||
      (schedule & ~(3 | OR_ELEC_EWALD)) != 0)
    return -1;
  for (int d = 0; d < 3; ++d)
    if (!(box[d] >= 2.0 * cutoff)) return -4;
  for (int i = 0; i < n; ++i)
    if (type[i] < 0 || type[i] >= n_types) return -5;
  for (int s = 0; s < n_sel; ++s)
    if (sel[s] < 0 || sel[s] >= n) return -7;
  excl_index ix;
  if (excl_build(n, n_excl, excl, &ix) != 0) return -6;
  const or_params p = make_params(cutoff, switch_width, dsf_alpha, sc_alpha, schedule);
  lam_state ls;
  lam_state_init(lambda, p.schedule, &ls);
  double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) wrap3(pos + 3 * i, box, w + 3 * i);
  const double rc2 = cutoff * cutoff;
#ifdef _OPENMP
  int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
#else
  (void)n_threads;
#endif
  for (int s = 0; s < n_sel; ++s) {
    const int a = sel[s];
    ksum e = {0, 0}, dl = {0, 0}, f[3] = {{0, 0}, {0, 0}, {0, 0}};
    int64_t cnt = 0;
    for (int j = 0; j < n; ++j) {
      if (j == a) continue;
      const int lo = a < j ? a : j, hi = a < j ? j : a;
      double d[3];
      /* canonical displacement of the pair (hi - lo), as in the full sum */
      double r2 = min_image(w + 3 * lo, w + 3 * hi, box, d);
      if (!(r2 < rc2)) continue;
      if (is_excluded(&ix, lo, hi)) continue;
      const int ti = type[lo], tj = type[hi];
      const int alch = (is_solute[lo] != 0) != (is_solute[hi] != 0);
      const double r = sqrt(r2);
      pair_out o;
      eval_pair(r, 0.5 * (sigma[ti] + sigma[tj]), sqrt(epsilon[ti] * epsilon[tj]), charge[ti] * charge[tj], alch,
                &p, &ls, &o);
      ++cnt;
      ks_add(&e, alch ? o.ss_vdw + o.ss_elec : o.u_plain);
      if (alch) ks_add(&dl, o.dl_vdw + o.dl_elec);
      /* force on hi is -dU/dr d/r, on lo the opposite */
      const double sgn = (a == hi) ? 1.0 : -1.0;
      for (int k = 0; k < 3; ++k) ks_add(&f[k], sgn * (-o.du_dr * d[k] / r));
    }
    for (int k = 0; k < 3; ++k) force[3 * s + k] = ks_val(&f[k]);
    energy[s] = ks_val(&e);
    dudl[s] = ks_val(&dl);
    n_pairs[s] = cnt;
  }
  free(w);
  free(ix.start);
  return 0;
}

/* Single-pair probe for closed-form tests: writes
 * out = {u, -du/dr, du/dlambda, du/dsig, du/deps, du/dqq}. */
void oracle_pair_probe(double r, double sig, double eps, double qq, int alchemical, double cutoff,
                       double switch_width, double dsf_alpha, double sc_alpha, int schedule, double lambda,
                       double *out) {
  const or_params p = make_params(cutoff, switch_width, dsf_alpha, sc_alpha, schedule);
  lam_state ls;
  lam_state_init(lambda, p.schedule, &ls);
  pair_out o;
  eval_pair(r, sig, eps, qq, alchemical, &p, &ls, &o);
  out[0] = alchemical ? o.ss_vdw + o.ss_elec : o.u_plain;
  out[1] = -o.du_dr;
  out[2] = o.dl_vdw + o.dl_elec;
  out[3] = o.du_dsig;
  out[4] = o.du_deps;
  out[5] = o.du_dqq;
}
