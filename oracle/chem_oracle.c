/* Plain serial FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see chem_oracle.h).
 *
 * Written for readability against the model equations, not for speed:
 * natural index order in every sum, no blocking, no fusion. Each function
 * names the part of the method it follows. Build with -ffp-contract=off so
 * that no multiply-add is fused behind the reader's back.
 */
#define _GNU_SOURCE
#include "chem_oracle.h"

#include <errno.h>
#include <limits.h>
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define R_GAS 8.314462618   /* J mol^-1 K^-1 */
#define P_ATM 101325.0      /* Pa */
#define MAXSIDE 4
#define LN10 2.302585092994045684

static __thread char g_err[512];
const char* orc_last_error(void) { return g_err; }

typedef struct {
  int type;        /* 0 elementary, 1 third body, 2 Troe falloff */
  int rev;
  int nr, np;
  int rs[MAXSIDE], ro[MAXSIDE];   /* reactant species, orders */
  int ps[MAXSIDE], po[MAXSIDE];   /* product species, orders */
  double A, b, Ea;
  int neff;
  int* eff_sp;
  double* eff_a;
  double A0, b0, Ea0, ta, T3, T1, T2;
  int has_T2;
} orc_rxn;

struct orc_mech {
  int ns, nr, ne;
  int* elem;       /* [ns][ne] atoms of each element per molecule */
  double* W;       /* [ns] kg/mol */
  double* trange;  /* [ns][3] Tlow Tmid Thigh */
  double* lo;      /* [ns][7] */
  double* hi;      /* [ns][7] */
  orc_rxn* rx;
};

/* ------------------------------------------------------------------------ */
/* parser                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct { char** tok; int n, pos; } toks;

static int tk_next(toks* t, const char** s) {
  if (t->pos >= t->n) return -1;
  *s = t->tok[t->pos++];
  return 0;
}
static int tk_int(toks* t, int* v) {
  const char* s; char* e;
  if (tk_next(t, &s)) return -1;
  errno = 0;
  long x = strtol(s, &e, 10);
  if (*e || errno == ERANGE || x < INT_MIN || x > INT_MAX) return -1;
  *v = (int)x;
  return 0;
}
static int tk_dbl(toks* t, double* v) {
  const char* s; char* e;
  if (tk_next(t, &s)) return -1;
  *v = strtod(s, &e);
  if (*e || !isfinite(*v)) return -1;
  return 0;
}
static int tk_expect(toks* t, const char* w) {
  const char* s;
  if (tk_next(t, &s)) return -1;
  return strcmp(s, w) ? -1 : 0;
}

void orc_mech_free(orc_mech* m) {
  if (!m) return;
  if (m->rx) {
    for (int r = 0; r < m->nr; ++r) { free(m->rx[r].eff_sp); free(m->rx[r].eff_a); }
  }
  free(m->rx); free(m->elem); free(m->W); free(m->trange); free(m->lo); free(m->hi);
  free(m);
}

#define PFAIL(msg) do { snprintf(g_err, sizeof g_err, "oracle parse: %s (token %d)", msg, t.pos); goto fail; } while (0)

int orc_mech_load(const char* path, orc_mech** out) {
  FILE* f = fopen(path, "rb");
  if (!f) { snprintf(g_err, sizeof g_err, "cannot open %s", path); return -2; }
  fseek(f, 0, SEEK_END);
  long sz = ftell(f);
  fseek(f, 0, SEEK_SET);
  char* buf = (char*)malloc(sz + 1);
  if (fread(buf, 1, sz, f) != (size_t)sz) { fclose(f); free(buf); return -2; }
  buf[sz] = 0;
  fclose(f);
  /* strip comments */
  for (char* p = buf; *p; ++p) {
    if (*p == '#') while (*p && *p != '\n') *p++ = ' ';
    if (!*p) break;
  }
  toks t = {0, 0, 0};
  int cap = 1024;
  t.tok = (char**)malloc(sizeof(char*) * cap);
  for (char* s = strtok(buf, " \t\r\n"); s; s = strtok(NULL, " \t\r\n")) {
    if (t.n == cap) { cap *= 2; t.tok = (char**)realloc(t.tok, sizeof(char*) * cap); }
    t.tok[t.n++] = s;
  }
  orc_mech* m = (orc_mech*)calloc(1, sizeof(orc_mech));
  int ne, ver;
  if (tk_expect(&t, "chemmech") || tk_int(&t, &ver) || ver != 1) PFAIL("header");
  /* the size limits keep every array size below int range */
  if (tk_expect(&t, "elements") || tk_int(&t, &ne) || ne < 1 || ne > 1024) PFAIL("elements");
  for (int e = 0; e < ne; ++e) {
    const char* s; double w;
    if (tk_next(&t, &s) || tk_dbl(&t, &w)) PFAIL("element line");
  }
  if (tk_expect(&t, "species") || tk_int(&t, &m->ns) || m->ns < 1 || m->ns > (1 << 16)) PFAIL("species");
  m->ne = ne;
  m->elem = (int*)calloc((size_t)m->ns * ne, sizeof(int));
  m->W = (double*)calloc((size_t)m->ns, sizeof(double));
  m->trange = (double*)calloc((size_t)3 * m->ns, sizeof(double));
  m->lo = (double*)calloc((size_t)7 * m->ns, sizeof(double));
  m->hi = (double*)calloc((size_t)7 * m->ns, sizeof(double));
  for (int i = 0; i < m->ns; ++i) {
    const char* s; int c;
    if (tk_next(&t, &s) || tk_dbl(&t, &m->W[i])) PFAIL("species line");
    for (int k = 0; k < 3; ++k) if (tk_dbl(&t, &m->trange[3 * i + k])) PFAIL("T range");
    for (int e = 0; e < ne; ++e) {
      if (tk_int(&t, &c) || c < 0) PFAIL("element count");
      m->elem[i * ne + e] = c;
    }
    for (int k = 0; k < 7; ++k) if (tk_dbl(&t, &m->lo[7 * i + k])) PFAIL("nasa lo");
    for (int k = 0; k < 7; ++k) if (tk_dbl(&t, &m->hi[7 * i + k])) PFAIL("nasa hi");
    if (!(m->W[i] > 0)) PFAIL("W <= 0");
  }
  if (tk_expect(&t, "reactions") || tk_int(&t, &m->nr) || m->nr < 0 || m->nr > (1 << 24)) PFAIL("reactions");
  m->rx = (orc_rxn*)calloc(m->nr > 0 ? m->nr : 1, sizeof(orc_rxn));
  for (int r = 0; r < m->nr; ++r) {
    orc_rxn* x = &m->rx[r];
    if (tk_expect(&t, "reaction") || tk_int(&t, &x->type) || tk_int(&t, &x->rev)) PFAIL("reaction");
    if (x->type < 0 || x->type > 2) PFAIL("reaction type");
    if (tk_int(&t, &x->nr) || x->nr < 1 || x->nr > MAXSIDE) PFAIL("n reactants");
    for (int k = 0; k < x->nr; ++k)
      if (tk_int(&t, &x->rs[k]) || tk_int(&t, &x->ro[k]) || x->rs[k] < 0 || x->rs[k] >= m->ns || x->ro[k] < 1)
        PFAIL("reactant");
    if (tk_int(&t, &x->np) || x->np < 1 || x->np > MAXSIDE) PFAIL("n products");
    for (int k = 0; k < x->np; ++k)
      if (tk_int(&t, &x->ps[k]) || tk_int(&t, &x->po[k]) || x->ps[k] < 0 || x->ps[k] >= m->ns || x->po[k] < 1)
        PFAIL("product");
    if (tk_dbl(&t, &x->A) || tk_dbl(&t, &x->b) || tk_dbl(&t, &x->Ea)) PFAIL("arrhenius");
    if (!(x->A > 0)) PFAIL("A <= 0");
    if (x->type >= 1) {
      if (tk_expect(&t, "eff") || tk_int(&t, &x->neff) || x->neff < 0 || x->neff > m->ns) PFAIL("eff");
      x->eff_sp = (int*)calloc(x->neff + 1, sizeof(int));
      x->eff_a = (double*)calloc(x->neff + 1, sizeof(double));
      for (int k = 0; k < x->neff; ++k)
        if (tk_int(&t, &x->eff_sp[k]) || tk_dbl(&t, &x->eff_a[k]) || x->eff_sp[k] < 0 || x->eff_sp[k] >= m->ns)
          PFAIL("eff entry");
    }
    if (x->type == 2) {
      double h2;
      if (tk_expect(&t, "troe") || tk_dbl(&t, &x->A0) || tk_dbl(&t, &x->b0) || tk_dbl(&t, &x->Ea0) ||
          tk_dbl(&t, &x->ta) || tk_dbl(&t, &x->T3) || tk_dbl(&t, &x->T1) || tk_dbl(&t, &x->T2) ||
          tk_dbl(&t, &h2))
        PFAIL("troe");
      x->has_T2 = h2 != 0.0;
      if (!(x->A0 > 0) || !(x->T3 > 0) || !(x->T1 > 0)) PFAIL("troe values");
    }
  }
  if (tk_expect(&t, "end")) PFAIL("end");
  free(t.tok); free(buf);
  *out = m;
  return 0;
fail:
  free(t.tok); free(buf);
  orc_mech_free(m);
  return -2;
}

int orc_mech_dims(const orc_mech* m, int* ns, int* nr) {
  if (!m) return -1;
  if (ns) *ns = m->ns;
  if (nr) *nr = m->nr;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* thermodynamics: NASA 7-coefficient polynomials                            */
/* ------------------------------------------------------------------------ */

void orc_thermo(const orc_mech* m, double T, double* cp_R, double* h_RT, double* s_R,
                double* dcp) {
  for (int i = 0; i < m->ns; ++i) {
    const double* a = (T < m->trange[3 * i + 1]) ? &m->lo[7 * i] : &m->hi[7 * i];
    double T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    if (cp_R) cp_R[i] = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
    if (h_RT) h_RT[i] = a[0] + a[1] * T / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 + a[4] * T4 / 5.0 + a[5] / T;
    if (s_R) s_R[i] = a[0] * log(T) + a[1] * T + a[2] * T2 / 2.0 + a[3] * T3 / 3.0 + a[4] * T4 / 4.0 + a[6];
    if (dcp) dcp[i] = a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T2 + 4.0 * a[4] * T3;
  }
}

/* ------------------------------------------------------------------------ */
/* kinetics                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
  double kf, kr;        /* forward / reverse rate constants (k_inf for falloff) */
  double Pf, Pr;        /* mass-action products of reactant / product concentrations */
  double q0;            /* kf Pf - kr Pr */
  double theta;         /* 1, [M], or Pr/(1+Pr) F */
  double q;             /* theta * q0 */
  /* for derivatives */
  double dlnkf, dlnkr;  /* d ln k / dT */
  double dtheta_dM;     /* d theta / d[M]  (1 for third body, Phi'(Pr) k0/kinf for falloff) */
  double dtheta_dT;     /* d theta / dT at fixed concentrations */
} rx_eval;

static double mass_action(const int* sp, const int* ord, int k, const double* C) {
  double P = 1.0;
  for (int j = 0; j < k; ++j)
    for (int o = 0; o < ord[j]; ++o) P = P * C[sp[j]];
  return P;
}

/* d(prod_k C_k^o_k)/dC_s without dividing by C_s: product rule over every
 * entry of the side that names species s (a species may be listed twice). */
static double mass_action_deriv(const int* sp, const int* ord, int k, const double* C, int s) {
  double D = 0.0;
  for (int j = 0; j < k; ++j) {
    if (sp[j] != s) continue;
    double term = (double)ord[j];
    for (int o = 0; o < ord[j] - 1; ++o) term = term * C[sp[j]];
    for (int l = 0; l < k; ++l) {
      if (l == j) continue;
      for (int o = 0; o < ord[l]; ++o) term = term * C[sp[l]];
    }
    D = D + term;
  }
  return D;
}

static double third_body_conc(const orc_rxn* x, const double* C, int ns) {
  /* [M] = sum_i alpha_i C_i with alpha_i = 1 unless listed */
  double M = 0.0;
  for (int i = 0; i < ns; ++i) {
    double a = 1.0;
    for (int k = 0; k < x->neff; ++k) if (x->eff_sp[k] == i) a = x->eff_a[k];
    M = M + a * C[i];
  }
  return M;
}

static double efficiency(const orc_rxn* x, int i) {
  for (int k = 0; k < x->neff; ++k) if (x->eff_sp[k] == i) return x->eff_a[k];
  return 1.0;
}

/* Evaluate one reaction at temperature T and concentrations C; g_RT and
 * h_RT are the species' g/(RT) and h/(RT) at T. */
static void eval_reaction(const orc_mech* m, const orc_rxn* x, double T, const double* C,
                          const double* g_RT, const double* h_RT, rx_eval* e) {
  double RT = R_GAS * T;
  e->kf = x->A * pow(T, x->b) * exp(-x->Ea / RT);
  e->dlnkf = (x->b + x->Ea / RT) / T;
  if (x->rev) {
    /* Kc = exp(-sum nu g/RT) (p_atm/RT)^(sum nu) */
    double sum_g = 0.0, sum_h = 0.0;
    int dnu = 0;
    for (int k = 0; k < x->nr; ++k) { sum_g -= x->ro[k] * g_RT[x->rs[k]]; sum_h -= x->ro[k] * h_RT[x->rs[k]]; dnu -= x->ro[k]; }
    for (int k = 0; k < x->np; ++k) { sum_g += x->po[k] * g_RT[x->ps[k]]; sum_h += x->po[k] * h_RT[x->ps[k]]; dnu += x->po[k]; }
    double Kc = exp(-sum_g) * pow(P_ATM / RT, (double)dnu);
    e->kr = e->kf / Kc;
    double dlnKc = sum_h / T - (double)dnu / T;
    e->dlnkr = e->dlnkf - dlnKc;
  } else {
    e->kr = 0.0;
    e->dlnkr = 0.0;
  }
  e->Pf = mass_action(x->rs, x->ro, x->nr, C);
  e->Pr = mass_action(x->ps, x->po, x->np, C);
  e->q0 = e->kf * e->Pf - e->kr * e->Pr;
  e->theta = 1.0;
  e->dtheta_dM = 0.0;
  e->dtheta_dT = 0.0;
  if (x->type == 1) {
    e->theta = third_body_conc(x, C, m->ns);
    e->dtheta_dM = 1.0;
  } else if (x->type == 2) {
    double M = third_body_conc(x, C, m->ns);
    double k0 = x->A0 * pow(T, x->b0) * exp(-x->Ea0 / RT);
    double dlnk0 = (x->b0 + x->Ea0 / RT) / T;
    double Pr = k0 * M / e->kf;
    if (Pr < 1e-300) Pr = 1e-300;
    /* Troe broadening */
    double e3 = exp(-T / x->T3), e1 = exp(-T / x->T1);
    double Fcent = (1.0 - x->ta) * e3 + x->ta * e1;
    double dFcent = -(1.0 - x->ta) / x->T3 * e3 - x->ta / x->T1 * e1;
    if (x->has_T2) {
      double e2 = exp(-x->T2 / T);
      Fcent = Fcent + e2;
      dFcent = dFcent + x->T2 / (T * T) * e2;
    }
    if (Fcent < 1e-300) Fcent = 1e-300;
    double L = log10(Fcent);
    double c = -0.4 - 0.67 * L;
    double N = 0.75 - 1.27 * L;
    double d = 0.14;
    double X = log10(Pr) + c;
    double den = N - d * X;
    double f1 = X / den;
    double log10F = L / (1.0 + f1 * f1);
    double F = pow(10.0, log10F);
    double lind = Pr / (1.0 + Pr);
    e->theta = lind * F;
    /* d log10F / d Pr at fixed T */
    double df1_dX = N / (den * den);
    double dlogF_dX = -L * 2.0 * f1 / ((1.0 + f1 * f1) * (1.0 + f1 * f1)) * df1_dX;
    double dlogF_dPr = dlogF_dX / (Pr * LN10);
    double dPhi_dPr = F / ((1.0 + Pr) * (1.0 + Pr)) + lind * F * LN10 * dlogF_dPr;
    e->dtheta_dM = dPhi_dPr * k0 / e->kf;
    /* d theta / dT at fixed C: through Pr (k0/kinf) and through Fcent */
    double dPr_dT = Pr * (dlnk0 - e->dlnkf);
    double dL_dT = dFcent / (Fcent * LN10);
    double dX_dL = -0.67;
    double dN_dL = -1.27;
    double df1_dL = (dX_dL * den - X * (dN_dL - d * dX_dL)) / (den * den);
    double dlogF_dL = 1.0 / (1.0 + f1 * f1) - L * 2.0 * f1 * df1_dL / ((1.0 + f1 * f1) * (1.0 + f1 * f1));
    double dF_dT_fixedPr = F * LN10 * dlogF_dL * dL_dT;
    e->dtheta_dT = dPhi_dPr * dPr_dT + lind * dF_dT_fixedPr;
  }
  e->q = e->theta * e->q0;
}

/* Concentrations from (T, p, Y): 1/Wbar = sum Y/W, rho = p Wbar/(RT), C = rho Y / W. */
static void state_from_y(const orc_mech* m, double p, double T, const double* Y, double* C,
                         double* rho, double* Wbar) {
  double inv = 0.0;
  for (int j = 0; j < m->ns; ++j) inv = inv + Y[j] / m->W[j];
  *Wbar = 1.0 / inv;
  *rho = p * (*Wbar) / (R_GAS * T);
  for (int j = 0; j < m->ns; ++j) C[j] = (*rho) * Y[j] / m->W[j];
}

void orc_rates(const orc_mech* m, double T, double p, const double* Y, double* kf, double* kr,
               double* q) {
  int ns = m->ns;
  double* C = (double*)malloc(sizeof(double) * ns * 5);
  double *cp = C + ns, *h = C + 2 * ns, *s = C + 3 * ns, *g = C + 4 * ns;
  double rho, Wbar;
  state_from_y(m, p, T, Y, C, &rho, &Wbar);
  orc_thermo(m, T, cp, h, s, NULL);
  for (int i = 0; i < ns; ++i) g[i] = h[i] - s[i];
  for (int r = 0; r < m->nr; ++r) {
    rx_eval e;
    eval_reaction(m, &m->rx[r], T, C, g, h, &e);
    if (kf) kf[r] = e.kf;
    if (kr) kr[r] = e.kr;
    if (q) q[r] = e.q;
  }
  free(C);
}

static int stoich(const orc_rxn* x, int i) {
  int v = 0;
  for (int k = 0; k < x->nr; ++k) if (x->rs[k] == i) v -= x->ro[k];
  for (int k = 0; k < x->np; ++k) if (x->ps[k] == i) v += x->po[k];
  return v;
}

void orc_omega(const orc_mech* m, double T, double p, const double* Y, double* omega) {
  double* q = (double*)malloc(sizeof(double) * (m->nr + 1));
  orc_rates(m, T, p, Y, NULL, NULL, q);
  for (int i = 0; i < m->ns; ++i) omega[i] = 0.0;
  for (int r = 0; r < m->nr; ++r) {
    const orc_rxn* x = &m->rx[r];
    for (int i = 0; i < m->ns; ++i) {
      int v = stoich(x, i);
      if (v) omega[i] = omega[i] + v * q[r];
    }
  }
  free(q);
}

/* f = dy/dt for y = (T, Y): dY_i/dt = W_i omega_i / rho,
 * dT/dt = -(sum_i h_i omega_i) / (rho cp). */
void orc_rhs(const orc_mech* m, double p, const double* y, double* f) {
  int ns = m->ns;
  double T = y[0];
  const double* Y = y + 1;
  double* omega = (double*)malloc(sizeof(double) * ns * 3);
  double *cp = omega + ns, *h = omega + 2 * ns;
  orc_omega(m, T, p, Y, omega);
  orc_thermo(m, T, cp, h, NULL, NULL);
  double rho, Wbar;
  double* C = (double*)malloc(sizeof(double) * ns);
  state_from_y(m, p, T, Y, C, &rho, &Wbar);
  double cpmix = 0.0, Q = 0.0;
  for (int i = 0; i < ns; ++i) cpmix = cpmix + Y[i] * cp[i] * R_GAS / m->W[i];
  for (int i = 0; i < ns; ++i) Q = Q + h[i] * R_GAS * T * omega[i];
  f[0] = -Q / (rho * cpmix);
  for (int i = 0; i < ns; ++i) f[1 + i] = m->W[i] * omega[i] / rho;
  free(C);
  free(omega);
}

/* Analytical Jacobian of f with respect to y = (T, Y_1..Y_Ns).
 * D_ij = d omega_i / d C_j and wT_i = d omega_i / dT, both at fixed C, are
 * built reaction by reaction; the chain rule through C(T, p, Y) and rho
 * then gives the species rows and the temperature row. */
void orc_jac(const orc_mech* m, double p, const double* y, double* J) {
  int ns = m->ns, n = ns + 1;
  double T = y[0];
  const double* Y = y + 1;
  double* D = (double*)calloc((size_t)ns * ns, sizeof(double));
  double* buf = (double*)calloc((size_t)ns * 10, sizeof(double));
  double *C = buf, *cp = buf + ns, *h = buf + 2 * ns, *s = buf + 3 * ns, *g = buf + 4 * ns;
  double *dcp = buf + 5 * ns, *omega = buf + 6 * ns, *wT = buf + 7 * ns, *sv = buf + 8 * ns;
  double *dwdY_row = buf + 9 * ns;
  double rho, Wbar;
  state_from_y(m, p, T, Y, C, &rho, &Wbar);
  orc_thermo(m, T, cp, h, s, dcp);
  for (int i = 0; i < ns; ++i) g[i] = h[i] - s[i];

  double* dq = (double*)calloc(ns, sizeof(double));
  for (int r = 0; r < m->nr; ++r) {
    const orc_rxn* x = &m->rx[r];
    rx_eval e;
    eval_reaction(m, x, T, C, g, h, &e);
    /* dq/dT at fixed C */
    double dq_dT = e.theta * (e.kf * e.dlnkf * e.Pf - e.kr * e.dlnkr * e.Pr) + e.q0 * e.dtheta_dT;
    /* dq/dC_j = theta (kf dPf/dC_j - kr dPr/dC_j) + q0 dtheta/d[M] alpha_j */
    for (int j = 0; j < ns; ++j) {
      double dPf = mass_action_deriv(x->rs, x->ro, x->nr, C, j);
      double dPr = mass_action_deriv(x->ps, x->po, x->np, C, j);
      double v = e.theta * (e.kf * dPf - e.kr * dPr);
      if (x->type >= 1) v = v + e.q0 * e.dtheta_dM * efficiency(x, j);
      dq[j] = v;
    }
    for (int i = 0; i < ns; ++i) {
      int v = stoich(x, i);
      if (!v) continue;
      omega[i] = omega[i] + v * e.q;
      wT[i] = wT[i] + v * dq_dT;
      for (int j = 0; j < ns; ++j) D[(size_t)i * ns + j] = D[(size_t)i * ns + j] + v * dq[j];
    }
  }
  free(dq);
  /* s_i = sum_k D_ik C_k */
  for (int i = 0; i < ns; ++i) {
    double a = 0.0;
    for (int k = 0; k < ns; ++k) a = a + D[(size_t)i * ns + k] * C[k];
    sv[i] = a;
  }
  double cpmix = 0.0, dcpmix = 0.0;
  for (int i = 0; i < ns; ++i) {
    cpmix = cpmix + Y[i] * cp[i] * R_GAS / m->W[i];
    dcpmix = dcpmix + Y[i] * dcp[i] * R_GAS / m->W[i];
  }
  double Q = 0.0;
  for (int i = 0; i < ns; ++i) Q = Q + h[i] * R_GAS * T * omega[i];
  double fT = -Q / (rho * cpmix);
  double rcp = rho * cpmix;

  /* species rows */
  double* dQdY = (double*)calloc(ns, sizeof(double));
  double dQdT = 0.0;
  for (int i = 0; i < ns; ++i) {
    double fi = m->W[i] * omega[i] / rho;
    double hi = h[i] * R_GAS * T;                       /* J/mol */
    for (int j = 0; j < ns; ++j) {
      double dw = (rho / m->W[j]) * D[(size_t)i * ns + j] - (Wbar / m->W[j]) * sv[i];
      dwdY_row[j] = dw;
      J[(size_t)(1 + i) * n + (1 + j)] = (m->W[i] / rho) * dw + fi * Wbar / m->W[j];
      dQdY[j] = dQdY[j] + hi * dw;
    }
    double dwdT = wT[i] - sv[i] / T;                    /* at fixed p, Y */
    J[(size_t)(1 + i) * n + 0] = (m->W[i] / rho) * dwdT + fi / T;
    dQdT = dQdT + cp[i] * R_GAS * omega[i] + hi * dwdT;
  }
  /* temperature row */
  for (int j = 0; j < ns; ++j) {
    double drcp = rho * cp[j] * R_GAS / m->W[j] - rcp * Wbar / m->W[j];
    J[1 + j] = -(dQdY[j] + fT * drcp) / rcp;
  }
  {
    double drcp = -rcp / T + rho * dcpmix;
    J[0] = -(dQdT + fT * drcp) / rcp;
  }
  free(dQdY);
  free(buf);
  free(D);
}

/* Forward differences, one more f per column: the way ODE codes form J
 * when no analytical Jacobian is given (paper: Introduction, the costly
 * finite-difference Jacobian; Fig. 2). The increment rule s_j =
 * sqrt(u max(1e-5, |y_j|)) is the one of Hairer and Wanner's Rosenbrock
 * codes; the divisor is the step actually taken, (y_j + s_j) - y_j. */
#define FD_UROUND 1.1102230246251565e-16
void orc_jac_fd(const orc_mech* m, double p, const double* y, const double* f0, double* J) {
  int n = m->ns + 1;
  double* yp = (double*)malloc(sizeof(double) * 2 * n);
  double* fp = yp + n;
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) yp[i] = y[i];
    double s = sqrt(FD_UROUND * fmax(1e-5, fabs(y[j])));
    yp[j] = y[j] + s;
    double d = yp[j] - y[j];
    orc_rhs(m, p, yp, fp);
    for (int i = 0; i < n; ++i) J[(size_t)i * n + j] = (fp[i] - f0[i]) / d;
  }
  free(yp);
}

/* ------------------------------------------------------------------------ */
/* dense LU with partial pivoting (getrf / getrs semantics)                  */
/* ------------------------------------------------------------------------ */

int orc_lu(int n, double* A, int* piv) {
  int info = 0;
  for (int k = 0; k < n; ++k) {
    /* first index of the largest |a_ik|, i >= k */
    int p = k;
    double best = fabs(A[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = fabs(A[(size_t)i * n + k]);
      if (v > best) { best = v; p = i; }
    }
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        double tmp = A[(size_t)k * n + j];
        A[(size_t)k * n + j] = A[(size_t)p * n + j];
        A[(size_t)p * n + j] = tmp;
      }
    double akk = A[(size_t)k * n + k];
    if (akk == 0.0) { if (!info) info = k + 1; continue; }
    for (int i = k + 1; i < n; ++i) {
      double l = A[(size_t)i * n + k] / akk;
      A[(size_t)i * n + k] = l;
      for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] = A[(size_t)i * n + j] - l * A[(size_t)k * n + j];
    }
  }
  return info;
}

void orc_lu_solve(int n, const double* LU, const int* piv, double* b) {
  for (int k = 0; k < n; ++k) {
    int p = piv[k];
    if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
  }
  for (int i = 0; i < n; ++i) {
    double a = b[i];
    for (int j = 0; j < i; ++j) a = a - LU[(size_t)i * n + j] * b[j];
    b[i] = a;
  }
  for (int i = n - 1; i >= 0; --i) {
    double a = b[i];
    for (int j = i + 1; j < n; ++j) a = a - LU[(size_t)i * n + j] * b[j];
    b[i] = a / LU[(size_t)i * n + i];
  }
}

/* ------------------------------------------------------------------------ */
/* The integrated state. Full: y = (T, Y_1..Y_Ns), n = Ns + 1. Bath gas      */
/* dropped (pyJac's convention): the last species is not integrated, its     */
/* mass fraction is 1 - sum of the others, y = (T, Y_1..Y_Ns-1), n = Ns.     */
/* Its f is the full f without the last row; its Jacobian follows by the     */
/* chain rule through Y_Ns = 1 - sum_j Y_j: column j of a species gets the   */
/* full Jacobian's column j minus the last column.                           */
/* ------------------------------------------------------------------------ */

typedef struct {
  const orc_mech* m;
  int red;               /* 1: bath gas (last species) dropped */
  double *yfull, *ffull, *Jfull;
  long nfev, njac;       /* evaluations of f and of J (analytical or by differences) */
} model_t;

static void model_init(model_t* mo, const orc_mech* m, int red) {
  int nf = m->ns + 1;
  mo->m = m;
  mo->red = red;
  mo->nfev = 0;
  mo->njac = 0;
  mo->yfull = (double*)calloc((size_t)nf * (nf + 2), sizeof(double));
  mo->ffull = mo->yfull + nf;
  mo->Jfull = mo->ffull + nf;
}
static void model_free(model_t* mo) { free(mo->yfull); }
static int model_n(const model_t* mo) { return mo->m->ns + (mo->red ? 0 : 1); }

/* Full state from the integrated one: Y_Ns = 1 - sum of the others, summed in
 * ascending order. */
static void model_full(const model_t* mo, const double* y, double* yf) {
  int ns = mo->m->ns;
  double sum = 0.0;
  for (int i = 0; i < ns; ++i) yf[i] = y[i];
  for (int i = 1; i < ns; ++i) sum = sum + y[i];
  yf[ns] = 1.0 - sum;
}

static void model_rhs(model_t* mo, double p, const double* y, double* f) {
  mo->nfev++;
  if (!mo->red) { orc_rhs(mo->m, p, y, f); return; }
  int ns = mo->m->ns;
  model_full(mo, y, mo->yfull);
  orc_rhs(mo->m, p, mo->yfull, mo->ffull);
  for (int i = 0; i < ns; ++i) f[i] = mo->ffull[i];
}

static void model_jac(model_t* mo, double p, const double* y, double* J) {
  mo->njac++;
  if (!mo->red) { orc_jac(mo->m, p, y, J); return; }
  int ns = mo->m->ns, nf = ns + 1;
  model_full(mo, y, mo->yfull);
  orc_jac(mo->m, p, mo->yfull, mo->Jfull);
  for (int i = 0; i < ns; ++i) {
    J[(size_t)i * ns] = mo->Jfull[(size_t)i * nf];
    for (int j = 1; j < ns; ++j) J[(size_t)i * ns + j] = mo->Jfull[(size_t)i * nf + j] - mo->Jfull[(size_t)i * nf + ns];
  }
}

/* forward differences of the integrated f (same increment rule as orc_jac_fd) */
static void model_jac_fd(model_t* mo, double p, const double* y, const double* f0, double* J) {
  int n = model_n(mo);
  mo->njac++;
  double* yp = (double*)malloc(sizeof(double) * 2 * n);
  double* fp = yp + n;
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) yp[i] = y[i];
    double s = sqrt(FD_UROUND * fmax(1e-5, fabs(y[j])));
    yp[j] = y[j] + s;
    double d = yp[j] - y[j];
    model_rhs(mo, p, yp, fp);
    for (int i = 0; i < n; ++i) J[(size_t)i * n + j] = (fp[i] - f0[i]) / d;
  }
  free(yp);
}

int orc_state_rhs(const orc_mech* m, int state, double p, const double* y, double* f) {
  if (!m || (state != ORC_STATE_FULL && state != ORC_STATE_NO_BATH) || (state == ORC_STATE_NO_BATH && m->ns < 2))
    return -1;
  model_t mo;
  model_init(&mo, m, state == ORC_STATE_NO_BATH);
  model_rhs(&mo, p, y, f);
  model_free(&mo);
  return 0;
}

int orc_state_jac(const orc_mech* m, int state, double p, const double* y, double* J) {
  if (!m || (state != ORC_STATE_FULL && state != ORC_STATE_NO_BATH) || (state == ORC_STATE_NO_BATH && m->ns < 2))
    return -1;
  model_t mo;
  model_init(&mo, m, state == ORC_STATE_NO_BATH);
  model_jac(&mo, p, y, J);
  model_free(&mo);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Rosenbrock methods in the transformed form: unknowns u_i, matrix          */
/* M = I/(gamma h) - J, stage i solves                                       */
/*   M u_i = f(y + sum_j a_ij u_j) + sum_j (c_ij / h) u_j,                   */
/* y_new = y + sum_j m_j u_j, error estimate sum_j e_j u_j.                  */
/* ------------------------------------------------------------------------ */

typedef struct {
  int stages;
  double gamma;
  double a[4][4], c[4][4]; /* strictly lower, row = stage */
  double m[4], e[4];
  int est_order;           /* order of the embedded solution: the error
                              estimate is O(h^(est_order+1)) */
} tableau_t;

/* Rodas3 (Sandu et al. 1997): order 3, embedded order 2, L-stable, stiffly
 * accurate. Stage 2 has a zero a-row and reuses f(y). */
static const tableau_t RODAS3 = {
    4, 0.5,
    {{0, 0, 0, 0}, {0, 0, 0, 0}, {2, 0, 0, 0}, {2, 0, 1, 0}},
    {{0, 0, 0, 0}, {4, 0, 0, 0}, {1, -1, 0, 0}, {1, -1, -8.0 / 3.0, 0}},
    {2, 0, 1, 1},
    {0, 0, 0, 1},
    2};

/* ROS4 of Shampine (1982), the first coefficient set of Hairer and Wanner's
 * Rosenbrock code family: order 4, embedded order 3, gamma = 1/2. Stage 4
 * has the a-row of stage 3 and so the same argument of f. */
static const tableau_t ROS4 = {
    4, 0.5,
    {{0, 0, 0, 0}, {2, 0, 0, 0}, {48.0 / 25.0, 6.0 / 25.0, 0, 0}, {48.0 / 25.0, 6.0 / 25.0, 0, 0}},
    {{0, 0, 0, 0}, {-8, 0, 0, 0}, {372.0 / 25.0, 12.0 / 5.0, 0, 0}, {-112.0 / 125.0, -54.0 / 125.0, -2.0 / 5.0, 0}},
    {19.0 / 9.0, 1.0 / 2.0, 25.0 / 108.0, 125.0 / 108.0},
    {17.0 / 54.0, 7.0 / 36.0, 0, 125.0 / 108.0},
    3};

static const tableau_t* tableau_of(int scheme) {
  if (scheme == ORC_RODAS3) return &RODAS3;
  if (scheme == ORC_ROS4) return &ROS4;
  return NULL;
}

int orc_tableau(int scheme, double* gamma, double* a, double* c, double* mw, double* e) {
  const tableau_t* tb = tableau_of(scheme);
  if (!tb) return -1;
  *gamma = tb->gamma;
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) { a[4 * i + j] = tb->a[i][j]; c[4 * i + j] = tb->c[i][j]; }
    mw[i] = tb->m[i];
    e[i] = tb->e[i];
  }
  return tb->stages;
}

void orc_rodas3_tableau(double* gamma, double* a, double* c, double* mw, double* e) {
  orc_tableau(ORC_RODAS3, gamma, a, c, mw, e);
}

typedef struct {
  int n;
  double *f0, *J, *M, *u, *ys, *fs, *rhs;
  int* piv;
} work_t;

static void work_alloc(work_t* w, int n) {
  w->n = n;
  w->f0 = (double*)calloc(n, sizeof(double));
  w->J = (double*)calloc((size_t)n * n, sizeof(double));
  w->M = (double*)calloc((size_t)n * n, sizeof(double));
  w->u = (double*)calloc((size_t)4 * n, sizeof(double));
  w->ys = (double*)calloc(n, sizeof(double));
  w->fs = (double*)calloc(n, sizeof(double));
  w->rhs = (double*)calloc(n, sizeof(double));
  w->piv = (int*)calloc(n, sizeof(int));
}
static void work_free(work_t* w) {
  free(w->f0); free(w->J); free(w->M); free(w->u); free(w->ys); free(w->fs); free(w->rhs); free(w->piv);
}

/* Where stage s takes its f from: 0 = f(y) (its a-row is zero), 1 = the f of
 * stage s-1 (its a-row equals stage s-1's, so the argument is the same), 2 =
 * a new evaluation at y + sum_j a_sj u_j. */
static int stage_f_source(const tableau_t* tb, int s) {
  int zero = 1, same = s > 0;
  for (int j = 0; j < 4; ++j) {
    if (j < s && tb->a[s][j] != 0.0) zero = 0;
    if (s > 0 && tb->a[s][j] != tb->a[s - 1][j]) same = 0;
  }
  if (zero) return 0;
  if (same && stage_f_source(tb, s - 1) == 2) return 1;
  return 2;
}

/* One attempted step of size h from y, with f0 = f(y) and J = J(y) given.
 * Returns the LU status. */
static int ros_attempt(model_t* mo, const tableau_t* tb, double p, const double* y, double h, work_t* w,
                       double* y_new, double* err_vec) {
  int n = w->n;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      w->M[(size_t)i * n + j] = (i == j ? 1.0 / (tb->gamma * h) : 0.0) - w->J[(size_t)i * n + j];
  int info = orc_lu(n, w->M, w->piv);
  if (info) return info;
  for (int s = 0; s < tb->stages; ++s) {
    int src = stage_f_source(tb, s);
    if (src == 2) {
      for (int i = 0; i < n; ++i) {
        double v = y[i];
        for (int j = 0; j < s; ++j) v = v + tb->a[s][j] * w->u[j * n + i];
        w->ys[i] = v;
      }
      model_rhs(mo, p, w->ys, w->fs);
    } else if (src == 0) {
      for (int i = 0; i < n; ++i) w->fs[i] = w->f0[i];
    } /* src == 1: fs still holds stage s-1's f */
    for (int i = 0; i < n; ++i) {
      double v = w->fs[i];
      for (int j = 0; j < s; ++j) v = v + (tb->c[s][j] / h) * w->u[j * n + i];
      w->rhs[i] = v;
    }
    orc_lu_solve(n, w->M, w->piv, w->rhs);
    for (int i = 0; i < n; ++i) w->u[s * n + i] = w->rhs[i];
  }
  for (int i = 0; i < n; ++i) {
    double v = y[i], e = 0.0;
    for (int j = 0; j < tb->stages; ++j) {
      v = v + tb->m[j] * w->u[j * n + i];
      e = e + tb->e[j] * w->u[j * n + i];
    }
    y_new[i] = v;
    err_vec[i] = e;
  }
  return 0;
}

int orc_step(const orc_mech* m, int scheme, double p, const double* y, double h, double* y_new,
             double* err_vec) {
  const tableau_t* tb = tableau_of(scheme);
  if (!tb) return -1;
  work_t w;
  model_t mo;
  model_init(&mo, m, 0);
  work_alloc(&w, m->ns + 1);
  orc_rhs(m, p, y, w.f0);
  orc_jac(m, p, y, w.J);
  int info = ros_attempt(&mo, tb, p, y, h, &w, y_new, err_vec);
  work_free(&w);
  model_free(&mo);
  return info;
}

int orc_rodas3_step(const orc_mech* m, double p, const double* y, double h, double* y_new,
                    double* err_vec) {
  return orc_step(m, ORC_RODAS3, p, y, h, y_new, err_vec);
}

/* Step-size controller constants (fixed; the GPU library uses the same). */
#define FAC_MIN 0.2
#define FAC_MAX 6.0
#define FAC_SAFE 0.9
#define FAC_REJ 0.1
#define H_MIN 1e-20
#define T_MIN 200.0
#define T_MAX 6000.0

/* Adaptive integration of one cell over [0, dt]; y (length n) in/out. */
static int integrate_cell(model_t* mo, double p, double dt, const orc_opts* o, double* y,
                          double* h_io, int* nacc_out, int* nrej_out, work_t* w, double* y_new,
                          double* err_vec) {
  int n = model_n(mo);
  mo->nfev = 0;
  mo->njac = 0;
  const tableau_t* tb = tableau_of(o->scheme);
  int nacc = 0, nrej = 0, attempts = 0, status = ORC_OK;
  for (int i = 0; i < n; ++i) if (!isfinite(y[i])) status = ORC_NONFINITE;
  if (!isfinite(p) || !(p > 0.0)) status = ORC_NONFINITE;
  double h = (h_io && *h_io > 0.0) ? *h_io : dt;
  double h_next = h;
  double t = 0.0;
  int need_start = 1, consec_rej = 0;
  while (status == ORC_OK && t < dt) {
    if (attempts >= o->max_steps) { status = ORC_MAX_STEPS; break; }
    if (need_start) {
      model_rhs(mo, p, y, w->f0);
      if (o->jacobian == ORC_JAC_FD) model_jac_fd(mo, p, y, w->f0, w->J);
      else model_jac(mo, p, y, w->J);
      need_start = 0;
    }
    double rem = dt - t;
    double hc = h;
    int clipped = 0;
    if (hc >= rem) { hc = rem; clipped = 1; }
    if (hc < H_MIN) { status = ORC_H_UNDERFLOW; break; }
    int info = ros_attempt(mo, tb, p, y, hc, w, y_new, err_vec);
    attempts++;
    if (info) { status = ORC_SINGULAR; break; }
    /* RMS error over all components */
    double acc = 0.0;
    int finite = 1;
    for (int i = 0; i < n; ++i) {
      double sc = o->atol + o->rtol * fmax(fabs(y[i]), fabs(y_new[i]));
      double r = err_vec[i] / sc;
      acc = acc + r * r;
      if (!isfinite(y_new[i])) finite = 0;
    }
    double err = sqrt(acc / n);
    double hnew;
    if (!finite || !isfinite(err)) {
      /* a non-finite trial step is rejected and the step cut by FAC_REJ */
      err = INFINITY;
      hnew = hc * FAC_REJ;
    } else {
      /* err is O(h^(q+1)) for an embedded solution of order q, so the step
       * factor goes as err^(-1/(q+1)): a cube root for Rodas3 (q = 2), a
       * fourth root for ROS4 (q = 3), taken as two correctly rounded square
       * roots */
      const double ef = fmax(err, 1e-10);
      double fac = FAC_SAFE / (tb->est_order == 3 ? sqrt(sqrt(ef)) : cbrt(ef));
      fac = fmin(FAC_MAX, fmax(FAC_MIN, fac));
      hnew = hc * fac;
    }
    if (err <= 1.0) {
      if (consec_rej > 0) hnew = fmin(hnew, hc);
      if (!(y_new[0] >= T_MIN && y_new[0] <= T_MAX)) { status = ORC_T_RANGE; break; }
      for (int i = 0; i < n; ++i) y[i] = y_new[i];
      nacc++;
      t = clipped ? dt : t + hc;
      h_next = clipped ? fmax(hnew, h) : hnew;
      h = hnew;
      consec_rej = 0;
      need_start = 1;
    } else {
      nrej++;
      consec_rej++;
      if (consec_rej >= 2) hnew = hc * FAC_REJ;
      h = hnew;
    }
  }
  if (status != ORC_OK) h_next = h;
  if (h_io) *h_io = h_next;
  *nacc_out = nacc;
  *nrej_out = nrej;
  return status;
}

typedef struct {
  const orc_mech* m;
  long n_cells;
  double dt;
  const orc_opts* o;
  const double* in;
  double* out;
  double* h_io;
  int *nacc, *nrej;
  int *njac, *nfev;
  signed char* status;
  atomic_long next;
} job_t;

static void* worker(void* arg) {
  job_t* jb = (job_t*)arg;
  int ns = jb->m->ns, w2 = ns + 2;
  model_t mo;
  model_init(&mo, jb->m, jb->o->state == ORC_STATE_NO_BATH);
  int n = model_n(&mo);
  work_t w;
  work_alloc(&w, n);
  double* y = (double*)malloc(sizeof(double) * (ns + 1) * 3);
  double *y_new = y + ns + 1, *err = y + 2 * (ns + 1);
  for (;;) {
    long c = atomic_fetch_add(&jb->next, 1);
    if (c >= jb->n_cells) break;
    const double* pin = jb->in + (size_t)c * w2;
    double p = pin[1];
    y[0] = pin[0];
    for (int i = 0; i < ns; ++i) y[1 + i] = pin[2 + i];
    double h = jb->h_io ? jb->h_io[c] : 0.0;
    int na = 0, nr = 0;
    /* without the bath gas, the input's last mass fraction is not read: it
     * is 1 - the sum of the others, before and after the step */
    int st = integrate_cell(&mo, p, jb->dt, jb->o, y, &h, &na, &nr, &w, y_new, err);
    if (mo.red) {
      double sum = 0.0;
      for (int i = 1; i < ns; ++i) sum = sum + y[i];
      y[ns] = 1.0 - sum;
    }
    double* pout = jb->out + (size_t)c * w2;
    pout[0] = y[0];
    pout[1] = p;
    for (int i = 0; i < ns; ++i) pout[2 + i] = y[1 + i];
    if (jb->h_io) jb->h_io[c] = h;
    if (jb->nacc) jb->nacc[c] = na;
    if (jb->nrej) jb->nrej[c] = nr;
    if (jb->njac) jb->njac[c] = (int)mo.njac;
    if (jb->nfev) jb->nfev[c] = (int)mo.nfev;
    if (jb->status) jb->status[c] = (signed char)st;
  }
  free(y);
  work_free(&w);
  model_free(&mo);
  return NULL;
}

int orc_integrate(const orc_mech* m, long n_cells, double dt, const orc_opts* o,
                  const double* phi_in, double* phi_out, double* h_io, int* n_acc, int* n_rej,
                  signed char* status, int n_threads) {
  return orc_integrate_counts(m, n_cells, dt, o, phi_in, phi_out, h_io, n_acc, n_rej, NULL, NULL, status, n_threads);
}

int orc_integrate_counts(const orc_mech* m, long n_cells, double dt, const orc_opts* o,
                         const double* phi_in, double* phi_out, double* h_io, int* n_acc, int* n_rej,
                         int* n_jac, int* n_fev, signed char* status, int n_threads) {
  if (!m || !o || n_cells < 0 || !(dt > 0.0) || (n_cells > 0 && (!phi_in || !phi_out)) || !tableau_of(o->scheme) ||
      (o->jacobian != ORC_JAC_ANALYTICAL && o->jacobian != ORC_JAC_FD) ||
      (o->state != ORC_STATE_FULL && o->state != ORC_STATE_NO_BATH) || (o->state == ORC_STATE_NO_BATH && m->ns < 2)) {
    snprintf(g_err, sizeof g_err, "orc_integrate: bad argument");
    return -1;
  }
  if (n_cells == 0) return 0;
  job_t jb;
  jb.m = m; jb.n_cells = n_cells; jb.dt = dt; jb.o = o; jb.in = phi_in; jb.out = phi_out;
  jb.h_io = h_io; jb.nacc = n_acc; jb.nrej = n_rej; jb.status = status;
  jb.njac = n_jac; jb.nfev = n_fev;
  atomic_init(&jb.next, 0);
  if (n_threads < 1) n_threads = 1;
  if (n_threads == 1) { worker(&jb); return 0; }
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * n_threads);
  for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, worker, &jb);
  for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
  free(th);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* mixture fraction (Methodology: zonal reference mapping)                   */
/* ------------------------------------------------------------------------ */

int orc_mech_elements(const orc_mech* m, int* ne, int* counts) {
  if (!m) return -1;
  if (ne) *ne = m->ne;
  if (counts) memcpy(counts, m->elem, sizeof(int) * (size_t)m->ns * m->ne);
  return 0;
}

/* Bilger's coupling function of one composition: moles of element e per kg of
 * mixture are sum_i a_{e,i} Y_i / W_i, so
 *   beta(Y) = sum_e coupling[e] sum_i a_{e,i} Y_i / W_i = sum_i Y_i b_i,
 *   b_i = (sum_e coupling[e] a_{e,i}) / W_i.
 * Sums run in natural index order, each term added by one fused multiply-add. */
static double bilger_coef(const orc_mech* m, const double* coupling, int i) {
  double s = 0.0;
  for (int e = 0; e < m->ne; ++e) s = fma(coupling[e], (double)m->elem[i * m->ne + e], s);
  return s / m->W[i];
}

static double bilger_beta(const orc_mech* m, const double* coupling, const double* Y) {
  double beta = 0.0;
  for (int i = 0; i < m->ns; ++i) beta = fma(Y[i], bilger_coef(m, coupling, i), beta);
  return beta;
}

/* Z = (beta - beta_ox) / (beta_fuel - beta_ox): 0 in the oxidiser stream, 1 in
 * the fuel stream, linear in Y in between (a conserved scalar when every
 * reaction conserves the elements). Returns -1 if the two streams have the
 * same beta. */
int orc_mixture_fraction(const orc_mech* m, const double* coupling, const double* y_fuel,
                         const double* y_ox, long n, const double* phi, double* z) {
  if (!m || !coupling || !y_fuel || !y_ox || n < 0 || (n > 0 && (!phi || !z))) {
    snprintf(g_err, sizeof g_err, "orc_mixture_fraction: bad argument");
    return -1;
  }
  const double bf = bilger_beta(m, coupling, y_fuel);
  const double bo = bilger_beta(m, coupling, y_ox);
  if (!(bf != bo) || !isfinite(bf) || !isfinite(bo)) {
    snprintf(g_err, sizeof g_err, "orc_mixture_fraction: fuel and oxidiser streams have the same beta");
    return -1;
  }
  const int stride = m->ns + 2;
  for (long c = 0; c < n; ++c)
    z[c] = (bilger_beta(m, coupling, phi + c * stride + 2) - bo) / (bf - bo);
  return 0;
}
