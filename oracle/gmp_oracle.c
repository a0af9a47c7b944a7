/*
 * Plain FP64 CPU oracle for Gaussian Multipole (GMP) features.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the HIP library.
 *
 * What it computes (the method of GMP-Featurizer, arXiv 2303.12980, section
 * "Examples": features are the Cartesian product of MCSH angular orders and
 * Gaussian radial widths, order-major; the cutoff is inferred from the
 * overlap threshold; derivatives are taken with respect to atom positions):
 *
 *   probe        G_s(u) = (2 pi s^2)^(-3/2) exp(-|u|^2 / (2 s^2)),  alpha = 1/(2 s^2)
 *   angular      P_abc(u) = (-1)^l |u|^(2l+1) d^a_x d^b_y d^c_z (1/|u|),  a+b+c = l
 *   density      rho_i(r) = sum_{(j,n)} sum_k B_{e_j,k} exp(-beta_{e_j,k} |r - R_j - n.cell|^2)
 *   component    mu_{i,l,s,abc} = int rho_i(r) P_abc(r - R_i) G_s(r - R_i) d^3r
 *              = sum_{(j,n)} c_{l,s,e_j}(|d|^2) P_abc(d),   d = R_j + n.cell - R_i
 *   radial       c_{l,s,e}(q) = sum_k B (alpha/lam)^(3/2) (beta/lam)^l exp(-gam q),
 *                lam = alpha + beta, gam = alpha beta / lam
 *   feature      F_{i,l,s} = sqrt( sum_{a+b+c=l} l!/(a!b!c!) mu_{i,l,s,abc}^2 )
 *   cutoff       rc(s)^2 = max over elements, primitives of ln(|A0|/tau)/gam,
 *                A0 = B (alpha/lam)^(3/2); 0 when |A0| <= tau
 *
 * Order -1 is the local density at the centre (section "Examples": it takes
 * no width and gives one feature, placed where -1 stands in the orders):
 *   rho_i = sum_{(j,n)} sum_k B_{e_j,k} exp(-beta_{e_j,k} |d|^2),  F_{i,-1} = |rho_i|
 * the limit s -> 0 of the order-0 component (the probe Gaussian tends to a
 * delta function: alpha/lam -> 1, gam -> beta).  Its cutoff is the same
 * limit of the rule above, rc_{-1}^2 = max ln(|B|/tau)/beta, held in one
 * extra cutoff slot after the sigmas ("slots" below are the sigmas plus,
 * when order -1 is requested, the density).
 *
 * Disordered structures (section "Overview": fractional site occupancy):
 * atom j carries an occupancy w_j (1 when none is given) that scales its
 * density, w_j sum_k B exp(-beta r^2), so every term of pair (j, n) is
 * multiplied by w_j; a site shared by several species is one atom entry per
 * species at the same position.  Cutoffs and neighbour sets do not depend on
 * the occupancies, and a centre's own occupancy enters only through its self
 * term.
 *
 * The closed form follows from the Gaussian product theorem and the mean
 * value property of harmonic polynomials; the test suite pins it against
 * brute-force quadrature of the integral.
 *
 * Neighbour set and its floating-point operation order (no FMA contraction:
 * build with -ffp-contract=off):
 *   reciprocal rows b1 = (a2 x a3)/V, b2 = (a3 x a1)/V, b3 = (a1 x a2)/V, V = a1.(a2 x a3)
 *   f_k  = (x b_k.x + y b_k.y) + z b_k.z ;  m_k = floor(f_k) on periodic axes, else 0
 *   Rw   = R - ((m1 a1 + m2 a2) + m3 a3)
 *   s(n) = (n1 a1 + n2 a2) + n3 a3
 *   d    = (Rw_j - Rw_i) + s(n) ;  q = (d.x^2 + d.y^2) + d.z^2
 *   (j, n) is a neighbour of i when q <= max_s rc(s)^2, n ranging over Z^3 on
 *   periodic axes (the centre itself and its own images included).
 *   shell(q) = number of slots with rc^2 < q; a slot uses the pairs with
 *   q <= its rc^2, i.e. shell(q) <= #{slots with a smaller rc^2}.
 *   Canonical order: ascending (shell, species of j, j, n1, n2, n3), so the
 *   pairs every sigma uses form a prefix of the list.
 *
 * Gradient of L = sum G_{i,l,s} F_{i,l,s} with the pair set held fixed:
 *   W = G w_abc mu / F (0 when F = 0);  v_{ijn} = sum W grad_d[c(q) P(d)]
 *   dL/dR_j += v, dL/dR_i -= v, dL/da_m += (n_m - m_j,m + m_i,m) v.
 * The derivative of c(q) P(d) is taken with forward-mode dual numbers.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVALID 1
#define OR_E_CELL 3
#define OR_E_CAPACITY 4

/* ------------------------------------------------------------------ */
/* dual numbers: value and gradient with respect to d = (x, y, z)      */
/* ------------------------------------------------------------------ */
typedef struct { double v, g[3]; } dual;

static dual dconst(double c) { dual r = {c, {0.0, 0.0, 0.0}}; return r; }
static dual dvar(double v, int k) { dual r = dconst(v); r.g[k] = 1.0; return r; }
static dual dadd(dual a, dual b) {
  dual r; r.v = a.v + b.v;
  for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] + b.g[k];
  return r;
}
static dual dsub(dual a, dual b) {
  dual r; r.v = a.v - b.v;
  for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] - b.g[k];
  return r;
}
static dual dmul(dual a, dual b) {
  dual r; r.v = a.v * b.v;
  for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] * b.v + a.v * b.g[k];
  return r;
}
static dual dscale(double c, dual a) {
  dual r; r.v = c * a.v;
  for (int k = 0; k < 3; ++k) r.g[k] = c * a.g[k];
  return r;
}
static dual dexp(dual a) {
  dual r; r.v = exp(a.v);
  for (int k = 0; k < 3; ++k) r.g[k] = r.v * a.g[k];
  return r;
}

/* ------------------------------------------------------------------ */
/* Solid Maxwell-Cartesian harmonics P_abc, written out per exponent    */
/* pattern.  u, s, t are the coordinates sorted by descending exponent. */
/* ------------------------------------------------------------------ */
static dual solid_harmonic(int a, int b, int c, dual x, dual y, dual z) {
  int e[3] = {a, b, c};
  dual v[3] = {x, y, z};
  /* stable sort of the three (exponent, variable) pairs, descending */
  for (int i = 1; i < 3; ++i)
    for (int k = i; k > 0 && e[k] > e[k - 1]; --k) {
      int te = e[k]; e[k] = e[k - 1]; e[k - 1] = te;
      dual tv = v[k]; v[k] = v[k - 1]; v[k - 1] = tv;
    }
  dual u = v[0], s = v[1], t = v[2];
  dual r2 = dadd(dadd(dmul(x, x), dmul(y, y)), dmul(z, z));
  dual u2 = dmul(u, u);
  int p = e[0] * 100 + e[1] * 10 + e[2];
  switch (p) {
    case 0:   return dconst(1.0);
    case 100: return u;
    case 200: return dsub(dscale(3.0, u2), r2);                     /* 3u^2 - r^2 */
    case 110: return dscale(3.0, dmul(u, s));                       /* 3us */
    case 300: return dsub(dscale(15.0, dmul(u2, u)),                /* 15u^3 - 9u r^2 */
                          dscale(9.0, dmul(u, r2)));
    case 210: return dsub(dscale(15.0, dmul(u2, s)),                /* 15u^2 s - 3 s r^2 */
                          dscale(3.0, dmul(s, r2)));
    case 111: return dscale(15.0, dmul(dmul(u, s), t));             /* 15ust */
    case 400: {                                                     /* 105u^4 - 90u^2 r^2 + 9r^4 */
      dual a4 = dscale(105.0, dmul(u2, u2));
      dual b4 = dscale(90.0, dmul(u2, r2));
      dual c4 = dscale(9.0, dmul(r2, r2));
      return dadd(dsub(a4, b4), c4);
    }
    case 310:                                                       /* 105u^3 s - 45 u s r^2 */
      return dsub(dscale(105.0, dmul(dmul(u2, u), s)), dscale(45.0, dmul(dmul(u, s), r2)));
    case 220: {                                                     /* 105u^2s^2 - 15u^2r^2 - 15s^2r^2 + 3r^4 */
      dual s2 = dmul(s, s);
      dual a4 = dscale(105.0, dmul(u2, s2));
      dual b4 = dscale(15.0, dmul(u2, r2));
      dual c4 = dscale(15.0, dmul(s2, r2));
      dual d4 = dscale(3.0, dmul(r2, r2));
      return dadd(dsub(dsub(a4, b4), c4), d4);
    }
    case 211:                                                       /* 105u^2 s t - 15 s t r^2 */
      return dsub(dscale(105.0, dmul(u2, dmul(s, t))), dscale(15.0, dmul(dmul(s, t), r2)));
    default:  return dconst(NAN);
  }
}

static int ncomp(int l) { return (l + 1) * (l + 2) / 2; }

/* components of order l in the order (a desc, then b desc) */
static void comp_abc(int l, int idx, int *a, int *b, int *c) {
  int k = 0;
  *a = *b = *c = 0;
  for (int aa = l; aa >= 0; --aa)
    for (int bb = l - aa; bb >= 0; --bb) {
      if (k == idx) { *a = aa; *b = bb; *c = l - aa - bb; return; }
      ++k;
    }
}

static double factorial(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

static double comp_weight(int a, int b, int c) {
  return factorial(a + b + c) / (factorial(a) * factorial(b) * factorial(c));
}

/* ------------------------------------------------------------------ */
/* probes and cutoffs                                                  */
/* ------------------------------------------------------------------ */
typedef struct {
  int n_orders; const int32_t *orders;
  int n_sigmas; const double *sigmas;
  int n_elements; const int32_t *prim_offsets;
  const double *B, *beta;
  double tau;
  int screen;  /* per-primitive screening (see primitive_used) */
} probes_t;

int oracle_cutoffs(int n_sigmas, const double *sigmas, int n_elements,
                   const int32_t *prim_offsets, const double *B, const double *beta,
                   double tau, double *rc2) {
  if (!(tau > 0.0)) return OR_E_INVALID;
  for (int s = 0; s < n_sigmas; ++s) {
    double sg = sigmas[s];
    if (!(sg > 0.0)) return OR_E_INVALID;
    double alpha = 1.0 / (2.0 * sg * sg);
    double best = 0.0;
    for (int e = 0; e < n_elements; ++e)
      for (int k = prim_offsets[e]; k < prim_offsets[e + 1]; ++k) {
        if (!(beta[k] > 0.0)) return OR_E_INVALID;
        double lam = alpha + beta[k];
        double gam = alpha * beta[k] / lam;
        double A0 = fabs(B[k]) * pow(alpha / lam, 1.5);
        if (A0 <= tau) continue;
        double r2 = log(A0 / tau) / gam;
        if (r2 > best) best = r2;
      }
    rc2[s] = best;
  }
  return OR_OK;
}

/* rc_{-1}^2 = max over primitives with |B| > tau of ln(|B|/tau)/beta */
int oracle_density_cutoff(int n_elements, const int32_t *prim_offsets, const double *B,
                          const double *beta, double tau, double *rc2) {
  if (!(tau > 0.0)) return OR_E_INVALID;
  double best = 0.0;
  for (int e = 0; e < n_elements; ++e)
    for (int k = prim_offsets[e]; k < prim_offsets[e + 1]; ++k) {
      if (!(beta[k] > 0.0)) return OR_E_INVALID;
      if (fabs(B[k]) <= tau) continue;
      double r2 = log(fabs(B[k]) / tau) / beta[k];
      if (r2 > best) best = r2;
    }
  *rc2 = best;
  return OR_OK;
}

static int has_density(const probes_t *P) {
  for (int o = 0; o < P->n_orders; ++o) if (P->orders[o] == -1) return 1;
  return 0;
}
static int n_slots(const probes_t *P) { return P->n_sigmas + has_density(P); }

/* cutoffs of every slot: the sigmas in order, then the density if requested */
static int slot_cutoffs(const probes_t *P, double *rc2) {
  int st = oracle_cutoffs(P->n_sigmas, P->sigmas, P->n_elements, P->prim_offsets, P->B, P->beta,
                          P->tau, rc2);
  if (!st && has_density(P))
    st = oracle_density_cutoff(P->n_elements, P->prim_offsets, P->B, P->beta, P->tau,
                               rc2 + P->n_sigmas);
  return st;
}

/*
 * Per-primitive screening (a speed variant of the cutoff rule, off by
 * default): primitive k of element e contributes to a slot only where its own
 * l = 0 overlap reaches the threshold, |A0| exp(-gamma q) >= tau, i.e. for
 * q <= r_k^2 = ln(|A0|/tau)/gamma (never when |A0| <= tau); for the density
 * slot A0 = B and gamma = beta.  The decision compares q and r_k^2 rounded to
 * FP32, the precision the GPU kernels take it in.  Every skipped term is
 * below tau (beta/lambda)^l <= tau in its radial factor.
 */
static int primitive_used(const probes_t *P, double A0abs, double gam, double qsel) {
  if (!P->screen) return 1;
  double thr = A0abs > P->tau ? log(A0abs / P->tau) / gam : -1.0;
  return (float)qsel <= (float)thr;
}

/* density of element e's primitives at squared distance q, as a dual number;
 * qsel decides the screened primitives */
static dual density(const probes_t *P, int e, dual q, double qsel) {
  dual acc = dconst(0.0);
  for (int k = P->prim_offsets[e]; k < P->prim_offsets[e + 1]; ++k) {
    if (!primitive_used(P, fabs(P->B[k]), P->beta[k], qsel)) continue;
    acc = dadd(acc, dscale(P->B[k], dexp(dscale(-P->beta[k], q))));
  }
  return acc;
}

/* radial factor c_{l,s,e}(q) as a dual number in d; qsel decides the
 * screened primitives */
static dual radial(const probes_t *P, int l, int s, int e, dual q, double qsel) {
  double sg = P->sigmas[s];
  double alpha = 1.0 / (2.0 * sg * sg);
  dual acc = dconst(0.0);
  for (int k = P->prim_offsets[e]; k < P->prim_offsets[e + 1]; ++k) {
    double lam = alpha + P->beta[k];
    double gam = alpha * P->beta[k] / lam;
    if (!primitive_used(P, fabs(P->B[k]) * pow(alpha / lam, 1.5), gam, qsel)) continue;
    double A = P->B[k] * pow(alpha / lam, 1.5) * pow(P->beta[k] / lam, (double)l);
    acc = dadd(acc, dscale(A, dexp(dscale(-gam, q))));
  }
  return acc;
}

/* ------------------------------------------------------------------ */
/* lattice                                                             */
/* ------------------------------------------------------------------ */
static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

/* reciprocal rows; returns 0 on success, OR_E_CELL for a singular cell */
static int reciprocal(const double *cell, double *b /* 9 */) {
  const double *a1 = cell, *a2 = cell + 3, *a3 = cell + 6;
  double c23[3], c31[3], c12[3];
  cross3(a2, a3, c23); cross3(a3, a1, c31); cross3(a1, a2, c12);
  double V = dot3(a1, c23);
  if (!(fabs(V) > 0.0) || !isfinite(V)) return OR_E_CELL;
  for (int k = 0; k < 3; ++k) { b[k] = c23[k] / V; b[3 + k] = c31[k] / V; b[6 + k] = c12[k] / V; }
  return OR_OK;
}

/* Wrap every atom into the home cell along periodic axes. */
int oracle_wrap(int n_atoms, const double *pos, const double *cell, int pbc,
                double *rw, int32_t *m) {
  double b[9];
  if (pbc) { int st = reciprocal(cell, b); if (st) return st; }
  for (int i = 0; i < n_atoms; ++i) {
    const double *R = pos + 3 * i;
    int mi[3] = {0, 0, 0};
    if (pbc)
      for (int k = 0; k < 3; ++k)
        if (pbc & (1 << k)) {
          double f = dot3(R, b + 3 * k);
          if (!isfinite(f)) return OR_E_INVALID;
          mi[k] = (int)floor(f);
        }
    for (int c = 0; c < 3; ++c) {
      double t = (double)mi[0] * cell[c] + (double)mi[1] * cell[3 + c];
      t = t + (double)mi[2] * cell[6 + c];
      rw[3 * i + c] = R[c] - (pbc ? t : 0.0);
    }
    m[3 * i + 0] = mi[0]; m[3 * i + 1] = mi[1]; m[3 * i + 2] = mi[2];
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* neighbours of one centre, by brute force over atoms and images      */
/* ------------------------------------------------------------------ */
typedef struct { int32_t e, shell, j, n[3]; double q, d[3], w; } pair_t;  /* w: occupancy of j */

static int pair_cmp(const void *pa, const void *pb) {
  const pair_t *x = (const pair_t *)pa, *y = (const pair_t *)pb;
  if (x->shell != y->shell) return x->shell < y->shell ? -1 : 1;
  if (x->e != y->e) return x->e < y->e ? -1 : 1;
  if (x->j != y->j) return x->j < y->j ? -1 : 1;
  for (int k = 0; k < 3; ++k)
    if (x->n[k] != y->n[k]) return x->n[k] < y->n[k] ? -1 : 1;
  return 0;
}

typedef struct {
  int n_atoms; const double *rw; const int32_t *species; const double *cell; int pbc;
  int nimg[3];
  const double *occ;  /* [n_atoms] occupancies or NULL (all 1) */
} sys_t;

static int image_reach(const double *cell, int pbc, double rcmax, int nimg[3]) {
  nimg[0] = nimg[1] = nimg[2] = 0;
  if (!pbc) return OR_OK;
  double b[9];
  int st = reciprocal(cell, b);
  if (st) return st;
  for (int k = 0; k < 3; ++k)
    if (pbc & (1 << k)) {
      double inv_h = sqrt(dot3(b + 3 * k, b + 3 * k));
      double r = floor(rcmax * inv_h) + 2.0;
      if (!(r < 1.0e6)) return OR_E_INVALID;
      nimg[k] = (int)r;
    }
  return OR_OK;
}

/* sorted neighbour list of a centre at wrapped position Ri (an atom's or a
 * reference point's) into a malloc'd array */
static int64_t collect_at(const sys_t *S, const double *Ri, int n_sigmas, const double *rc2, pair_t **out) {
  double rcmax2 = 0.0;
  for (int s = 0; s < n_sigmas; ++s) if (rc2[s] > rcmax2) rcmax2 = rc2[s];
  int64_t cap = 256, n = 0;
  pair_t *buf = (pair_t *)malloc(sizeof(pair_t) * cap);
  const double *a1 = S->cell, *a2 = S->cell + 3, *a3 = S->cell + 6;
  for (int n1 = -S->nimg[0]; n1 <= S->nimg[0]; ++n1)
    for (int n2 = -S->nimg[1]; n2 <= S->nimg[1]; ++n2)
      for (int n3 = -S->nimg[2]; n3 <= S->nimg[2]; ++n3) {
        double sh[3];
        for (int c = 0; c < 3; ++c) {
          if (S->pbc) {
            double t = (double)n1 * a1[c] + (double)n2 * a2[c];
            sh[c] = t + (double)n3 * a3[c];
          } else {
            sh[c] = 0.0;
          }
        }
        for (int j = 0; j < S->n_atoms; ++j) {
          const double *Rj = S->rw + 3 * j;
          double d[3];
          for (int c = 0; c < 3; ++c) d[c] = (Rj[c] - Ri[c]) + sh[c];
          double q = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
          if (!(q <= rcmax2)) continue;
          if (n == cap) { cap *= 2; buf = (pair_t *)realloc(buf, sizeof(pair_t) * cap); }
          pair_t *p = buf + n++;
          p->e = S->species[j]; p->j = j; p->w = S->occ ? S->occ[j] : 1.0;
          p->n[0] = n1; p->n[1] = n2; p->n[2] = n3;
          p->q = q; p->d[0] = d[0]; p->d[1] = d[1]; p->d[2] = d[2];
          int sh_ = 0;
          for (int s = 0; s < n_sigmas; ++s) if (rc2[s] < q) ++sh_;
          p->shell = sh_;
        }
      }
  qsort(buf, (size_t)n, sizeof(pair_t), pair_cmp);
  *out = buf;
  return n;
}

static int64_t collect(const sys_t *S, int i, int n_sigmas, const double *rc2, pair_t **out) {
  return collect_at(S, S->rw + 3 * i, n_sigmas, rc2, out);
}

static int make_sys(sys_t *S, int n_atoms, const double *pos, const int32_t *species,
                    const double *cell, int pbc, double rcmax2, double **rw_out, int32_t **m_out) {
  double *rw = (double *)malloc(sizeof(double) * 3 * (n_atoms > 0 ? n_atoms : 1));
  int32_t *m = (int32_t *)malloc(sizeof(int32_t) * 3 * (n_atoms > 0 ? n_atoms : 1));
  int st = oracle_wrap(n_atoms, pos, cell, pbc, rw, m);
  if (!st) st = image_reach(cell, pbc, sqrt(rcmax2), S->nimg);
  if (st) { free(rw); free(m); return st; }
  S->n_atoms = n_atoms; S->rw = rw; S->species = species; S->cell = cell; S->pbc = pbc; S->occ = NULL;
  *rw_out = rw; *m_out = m;
  return OR_OK;
}

/*
 * Canonical neighbour list of one centre.  Writes up to `cap` entries and
 * returns the full count (a count larger than `cap` means truncated).
 * out_n is [cap*3], shifts relative to the wrapped positions.
 */
int64_t oracle_neighbors(int n_atoms, const double *pos, const int32_t *species,
                         const double *cell, int pbc, int n_sigmas, const double *rc2,
                         int centre, int64_t cap, int32_t *out_j, int32_t *out_n,
                         double *out_q, int32_t *out_shell, int32_t *status) {
  double rcmax2 = 0.0;
  for (int s = 0; s < n_sigmas; ++s) if (rc2[s] > rcmax2) rcmax2 = rc2[s];
  sys_t S; double *rw; int32_t *m;
  *status = make_sys(&S, n_atoms, pos, species, cell, pbc, rcmax2, &rw, &m);
  if (*status) return 0;
  pair_t *P;
  int64_t n = collect(&S, centre, n_sigmas, rc2, &P);
  for (int64_t k = 0; k < n && k < cap; ++k) {
    out_j[k] = P[k].j;
    out_n[3 * k] = P[k].n[0]; out_n[3 * k + 1] = P[k].n[1]; out_n[3 * k + 2] = P[k].n[2];
    out_q[k] = P[k].q; out_shell[k] = P[k].shell;
  }
  free(P); free(rw); free(m);
  return n;
}

/*
 * Canonical lists of many centres at once (the same lists as
 * oracle_neighbors, computed in parallel over centres): centre list[t]'s
 * entries go to [offs[t], offs[t+1]) of the outputs.  Pass 1 (out_j NULL)
 * fills offs [n_list+1] only; pass 2 writes j, n [3 each], q and shell for
 * at most cap entries.  Returns the total count.
 */
int64_t oracle_neighbors_many(int n_atoms, const double *pos, const int32_t *species,
                              const double *cell, int pbc, int n_sigmas, const double *rc2,
                              int n_list, const int32_t *list, int64_t *offs, int64_t cap,
                              int32_t *out_j, int32_t *out_n, double *out_q, int32_t *out_shell,
                              int32_t *status) {
  double rcmax2 = 0.0;
  for (int s = 0; s < n_sigmas; ++s) if (rc2[s] > rcmax2) rcmax2 = rc2[s];
  sys_t S; double *rw; int32_t *m;
  *status = make_sys(&S, n_atoms, pos, species, cell, pbc, rcmax2, &rw, &m);
  if (*status) return 0;
  for (int t = 0; t < n_list; ++t)
    if (list[t] < 0 || list[t] >= n_atoms) { *status = OR_E_INVALID; free(rw); free(m); return 0; }
  int64_t *cnt = (int64_t *)calloc((size_t)(n_list > 0 ? n_list : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < n_list; ++t) {
    pair_t *P;
    int64_t n = collect(&S, list[t], n_sigmas, rc2, &P);
    cnt[t] = n;
    if (out_j && offs[t] + n <= cap) {
      for (int64_t k = 0; k < n; ++k) {
        const int64_t o = offs[t] + k;
        out_j[o] = P[k].j;
        out_n[3 * o] = P[k].n[0]; out_n[3 * o + 1] = P[k].n[1]; out_n[3 * o + 2] = P[k].n[2];
        out_q[o] = P[k].q; out_shell[o] = P[k].shell;
      }
    }
    free(P);
  }
  int64_t total = 0;
  if (!out_j) {
    offs[0] = 0;
    for (int t = 0; t < n_list; ++t) offs[t + 1] = offs[t] + cnt[t];
  }
  for (int t = 0; t < n_list; ++t) total += cnt[t];
  free(cnt); free(rw); free(m);
  return total;
}

/* ------------------------------------------------------------------ */
/* features                                                            */
/* ------------------------------------------------------------------ */
/* components and features of one order: order -1 has one of each */
static int order_comps(const probes_t *P, int l) { return l < 0 ? 1 : P->n_sigmas * ncomp(l); }
static int order_feats(const probes_t *P, int l) { return l < 0 ? 1 : P->n_sigmas; }

static int total_comps(const probes_t *P) {
  int t = 0;
  for (int o = 0; o < P->n_orders; ++o) t += order_comps(P, P->orders[o]);
  return t;
}

static int total_feats(const probes_t *P) {
  int t = 0;
  for (int o = 0; o < P->n_orders; ++o) t += order_feats(P, P->orders[o]);
  return t;
}

static int check_probes(const probes_t *P) {
  if (P->n_orders < 1 || P->n_sigmas < 1 || P->n_elements < 1) return OR_E_INVALID;
  for (int o = 0; o < P->n_orders; ++o)
    if (P->orders[o] < -1 || P->orders[o] > 4) return OR_E_INVALID;
  return OR_OK;
}

/* add one pair's terms to mu, laid out [order][sigma][comp] (order -1: one
 * entry); `use` is the squared distance that decides which slots see the
 * pair, (x, y, z) and q the displacement and squared distance evaluated */
static void pair_terms_mode(const probes_t *P, const pair_t *pp, double use, const double *rc2, double *mu,
                            int absval);
static void pair_terms(const probes_t *P, const pair_t *pp, double use, const double *rc2, double *mu) {
  pair_terms_mode(P, pp, use, rc2, mu, 0);
}

/* absval = 1 adds |term| instead of term (the conditioning reference
 * F_abs: the feature of the absolute values of the pair terms) */
static void pair_terms_mode(const probes_t *P, const pair_t *pp, double use, const double *rc2, double *mu,
                            int absval) {
  dual x = dconst(pp->d[0]), y = dconst(pp->d[1]), z = dconst(pp->d[2]);
  dual q = dconst(pp->q);
  int off = 0;
  for (int o = 0; o < P->n_orders; ++o) {
    int l = P->orders[o];
    if (l < 0) {
      if (use <= rc2[P->n_sigmas]) {
        const double t = pp->w * density(P, pp->e, q, use).v;
        mu[off] += absval ? fabs(t) : t;
      }
      off += 1;
      continue;
    }
    for (int s = 0; s < P->n_sigmas; ++s) {
      if (!(use <= rc2[s])) continue;
      double c = radial(P, l, s, pp->e, q, use).v;
      for (int k = 0; k < ncomp(l); ++k) {
        int a, b, cc; comp_abc(l, k, &a, &b, &cc);
        const double t = pp->w * (c * solid_harmonic(a, b, cc, x, y, z).v);
        mu[(size_t)(off + s * ncomp(l) + k)] += absval ? fabs(t) : t;
      }
    }
    off += order_comps(P, l);
  }
}

/* features from mu: weighted root-sum-square per (order, sigma); |rho| for order -1 */
static void norms(const probes_t *P, const double *mu, double *F) {
  int off = 0, f = 0;
  for (int o = 0; o < P->n_orders; ++o) {
    int l = P->orders[o];
    if (l < 0) {
      F[f++] = fabs(mu[off]);
      off += 1;
      continue;
    }
    for (int s = 0; s < P->n_sigmas; ++s) {
      double acc = 0.0;
      for (int k = 0; k < ncomp(l); ++k) {
        int a, b, cc; comp_abc(l, k, &a, &b, &cc);
        double v = mu[off + s * ncomp(l) + k];
        acc += comp_weight(a, b, cc) * v * v;
      }
      F[f++] = sqrt(acc);
    }
    off += order_comps(P, l);
  }
}

/* mu and F for centre i from its pair list */
static void centre_features(const probes_t *P, const pair_t *pairs, int64_t np,
                            const double *rc2, double *mu, double *F) {
  memset(mu, 0, sizeof(double) * (size_t)total_comps(P));
  for (int64_t p = 0; p < np; ++p) pair_terms(P, pairs + p, pairs[p].q, rc2, mu);
  norms(P, mu, F);
}

/*
 * Features of the listed centres of one structure (all centres when
 * n_centres < 0).  F is [n_centres][nf], nf = sum over orders of n_sigmas
 * (1 for order -1); mu (optional) is [n_centres][nc], nc = sum over orders
 * of n_sigmas*ncomp(l) (1 for order -1), in (order, sigma, component) order.
 * occ: [n_atoms] occupancies, or NULL for all 1.
 */
int oracle_features(int n_atoms, const double *pos, const int32_t *species,
                    const double *cell, int pbc,
                    int n_orders, const int32_t *orders, int n_sigmas, const double *sigmas,
                    int n_elements, const int32_t *prim_offsets, const double *B,
                    const double *beta, double tau, int screen,
                    int n_centres, const int32_t *centres, double *F, double *mu,
                    const double *occ) {
  probes_t P = {n_orders, orders, n_sigmas, sigmas, n_elements, prim_offsets, B, beta, tau, screen};
  int st = check_probes(&P);
  if (st) return st;
  for (int i = 0; i < n_atoms; ++i)
    if (species[i] < 0 || species[i] >= n_elements) return OR_E_INVALID;
  const int ns = n_slots(&P);
  double *rc2 = (double *)malloc(sizeof(double) * ns);
  st = slot_cutoffs(&P, rc2);
  double rcmax2 = 0.0;
  for (int s = 0; s < ns; ++s) if (rc2[s] > rcmax2) rcmax2 = rc2[s];
  sys_t S; double *rw = NULL; int32_t *m = NULL;
  if (!st) st = make_sys(&S, n_atoms, pos, species, cell, pbc, rcmax2, &rw, &m);
  if (st) { free(rc2); return st; }
  S.occ = occ;
  int nc = total_comps(&P);
  int ncent = n_centres < 0 ? n_atoms : n_centres;
  int nf = total_feats(&P);
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < ncent; ++t) {
    int i = n_centres < 0 ? t : centres[t];
    pair_t *pairs;
    int64_t np = collect(&S, i, ns, rc2, &pairs);
    double *mu_i = (double *)malloc(sizeof(double) * (size_t)nc);
    centre_features(&P, pairs, np, rc2, mu_i, F + (size_t)t * nf);
    if (mu) memcpy(mu + (size_t)t * nc, mu_i, sizeof(double) * (size_t)nc);
    free(mu_i); free(pairs);
  }
  free(rc2); free(rw); free(m);
  return OR_OK;
}

/*
 * Conditioning reference of the listed centres: F_abs, the features computed
 * from the absolute values of every pair term (same layout as
 * oracle_features).  F_abs / F bounds how far a feature is the remainder of
 * cancelling terms: a result whose every pair term carries a relative error
 * e is within e F_abs of the exact feature.
 */
int oracle_features_abs(int n_atoms, const double *pos, const int32_t *species,
                        const double *cell, int pbc,
                        int n_orders, const int32_t *orders, int n_sigmas, const double *sigmas,
                        int n_elements, const int32_t *prim_offsets, const double *B,
                        const double *beta, double tau, int screen,
                        int n_centres, const int32_t *centres, double *F, const double *occ) {
  probes_t P = {n_orders, orders, n_sigmas, sigmas, n_elements, prim_offsets, B, beta, tau, screen};
  int st = check_probes(&P);
  if (st) return st;
  for (int i = 0; i < n_atoms; ++i)
    if (species[i] < 0 || species[i] >= n_elements) return OR_E_INVALID;
  const int ns = n_slots(&P);
  double *rc2 = (double *)malloc(sizeof(double) * ns);
  st = slot_cutoffs(&P, rc2);
  double rcmax2 = 0.0;
  for (int s = 0; s < ns; ++s) if (rc2[s] > rcmax2) rcmax2 = rc2[s];
  sys_t S; double *rw = NULL; int32_t *m = NULL;
  if (!st) st = make_sys(&S, n_atoms, pos, species, cell, pbc, rcmax2, &rw, &m);
  if (st) { free(rc2); return st; }
  S.occ = occ;
  const int nc = total_comps(&P), nf = total_feats(&P);
  const int ncent = n_centres < 0 ? n_atoms : n_centres;
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < ncent; ++t) {
    int i = n_centres < 0 ? t : centres[t];
    pair_t *pairs;
    int64_t np = collect(&S, i, ns, rc2, &pairs);
    double *mu = (double *)calloc((size_t)nc, sizeof(double));
    for (int64_t p = 0; p < np; ++p) pair_terms_mode(&P, pairs + p, pairs[p].q, rc2, mu, 1);
    norms(&P, mu, F + (size_t)t * nf);
    free(mu); free(pairs);
  }
  free(rc2); free(rw); free(m);
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* gradient of L = sum G F                                             */
/* ------------------------------------------------------------------ */
/* v = sum W grad_d[term] over the pair's terms (same layout as mu) */
static void pair_v(const probes_t *P, const pair_t *pp, const double *rc2, const double *W,
                   double v[3]) {
  dual x = dvar(pp->d[0], 0), y = dvar(pp->d[1], 1), z = dvar(pp->d[2], 2);
  dual q = dadd(dadd(dmul(x, x), dmul(y, y)), dmul(z, z));
  v[0] = v[1] = v[2] = 0.0;
  int off = 0;
  for (int o = 0; o < P->n_orders; ++o) {
    int l = P->orders[o];
    if (l < 0) {
      if (pp->q <= rc2[P->n_sigmas] && W[off] != 0.0) {
        dual t = density(P, pp->e, q, pp->q);
        v[0] += W[off] * t.g[0]; v[1] += W[off] * t.g[1]; v[2] += W[off] * t.g[2];
      }
      off += 1;
      continue;
    }
    for (int s = 0; s < P->n_sigmas; ++s) {
      if (!(pp->q <= rc2[s])) continue;
      dual c = radial(P, l, s, pp->e, q, pp->q);
      for (int k = 0; k < ncomp(l); ++k) {
        int a, b, cc; comp_abc(l, k, &a, &b, &cc);
        double w = W[off + s * ncomp(l) + k];
        if (w == 0.0) continue;
        dual t = dmul(c, solid_harmonic(a, b, cc, x, y, z));
        v[0] += w * t.g[0]; v[1] += w * t.g[1]; v[2] += w * t.g[2];
      }
    }
    off += order_comps(P, l);
  }
  for (int k = 0; k < 3; ++k) v[k] *= pp->w;
}

/* W = dL/dmu = G dF/dmu: G w mu / F per component (0 when F = 0); for
 * order -1, F = |rho| and W = G rho / |rho| */
static void make_W(const probes_t *P, const double *mu, const double *F, const double *G, double *W) {
  int off = 0, f = 0;
  for (int o = 0; o < P->n_orders; ++o) {
    int l = P->orders[o];
    if (l < 0) {
      W[off] = F[f] > 0.0 ? G[f] * mu[off] / F[f] : 0.0;
      ++f;
      off += 1;
      continue;
    }
    for (int s = 0; s < P->n_sigmas; ++s, ++f) {
      for (int k = 0; k < ncomp(l); ++k) {
        int a, b, cc; comp_abc(l, k, &a, &b, &cc);
        int idx = off + s * ncomp(l) + k;
        W[idx] = F[f] > 0.0 ? G[f] * comp_weight(a, b, cc) * mu[idx] / F[f] : 0.0;
      }
    }
    off += order_comps(P, l);
  }
}

/*
 * Analytic gradient of L = sum_{i,f} G[i][f] F[i][f] for one structure.
 * grad_pos [n_atoms*3], grad_cell [9] (row m = d/d a_m).
 * Also returns F [n_atoms*nf] when F_out is not NULL.  occ as in oracle_features.
 */
int oracle_grad(int n_atoms, const double *pos, const int32_t *species,
                const double *cell, int pbc,
                int n_orders, const int32_t *orders, int n_sigmas, const double *sigmas,
                int n_elements, const int32_t *prim_offsets, const double *B,
                const double *beta, double tau, int screen,
                const double *G, double *grad_pos, double *grad_cell, double *F_out,
                const double *occ) {
  probes_t P = {n_orders, orders, n_sigmas, sigmas, n_elements, prim_offsets, B, beta, tau, screen};
  int st = check_probes(&P);
  if (st) return st;
  for (int i = 0; i < n_atoms; ++i)
    if (species[i] < 0 || species[i] >= n_elements) return OR_E_INVALID;
  const int ns = n_slots(&P);
  double *rc2 = (double *)malloc(sizeof(double) * ns);
  st = slot_cutoffs(&P, rc2);
  double rcmax2 = 0.0;
  for (int s = 0; s < ns; ++s) if (rc2[s] > rcmax2) rcmax2 = rc2[s];
  sys_t S; double *rw = NULL; int32_t *m = NULL;
  if (!st) st = make_sys(&S, n_atoms, pos, species, cell, pbc, rcmax2, &rw, &m);
  if (st) { free(rc2); return st; }
  S.occ = occ;
  int nc = total_comps(&P);
  int nf = total_feats(&P);
  memset(grad_pos, 0, sizeof(double) * 3 * n_atoms);
  memset(grad_cell, 0, sizeof(double) * 9);
  double *mu = (double *)malloc(sizeof(double) * (size_t)nc);
  double *W = (double *)malloc(sizeof(double) * (size_t)nc);
  double *Fi = (double *)malloc(sizeof(double) * nf);
  for (int i = 0; i < n_atoms; ++i) {
    pair_t *pairs;
    int64_t np = collect(&S, i, ns, rc2, &pairs);
    centre_features(&P, pairs, np, rc2, mu, Fi);
    if (F_out) memcpy(F_out + (size_t)i * nf, Fi, sizeof(double) * nf);
    make_W(&P, mu, Fi, G + (size_t)i * nf, W);
    for (int64_t p = 0; p < np; ++p) {
      double v[3];
      pair_v(&P, pairs + p, rc2, W, v);
      int j = pairs[p].j;
      for (int k = 0; k < 3; ++k) { grad_pos[3 * j + k] += v[k]; grad_pos[3 * i + k] -= v[k]; }
      for (int a = 0; a < 3; ++a) {
        double nt = (double)(pairs[p].n[a] - m[3 * j + a] + m[3 * i + a]);
        for (int k = 0; k < 3; ++k) grad_cell[3 * a + k] += nt * v[k];
      }
    }
    free(pairs);
  }
  free(mu); free(W); free(Fi); free(rc2); free(rw); free(m);
  return OR_OK;
}

/*
 * Gradient of L restricted to listed centres: L = sum over the n_list centres
 * list[t] of sum_f G[t][f] F[list[t]][f] (the upstream gradient is zero on
 * every other centre), with the same definitions as oracle_grad.  Centres
 * are independent, so their pair vectors are computed in parallel into
 * per-centre buffers; the scatter into grad_pos / grad_cell then runs in list
 * order, one centre after another, as oracle_grad's loop does.  grad_pos
 * [n_atoms*3], grad_cell [9]; occ as in oracle_features.
 */
int oracle_grad_centres(int n_atoms, const double *pos, const int32_t *species,
                        const double *cell, int pbc,
                        int n_orders, const int32_t *orders, int n_sigmas, const double *sigmas,
                        int n_elements, const int32_t *prim_offsets, const double *B,
                        const double *beta, double tau, int screen,
                        int n_list, const int32_t *list, const double *G,
                        double *grad_pos, double *grad_cell, const double *occ) {
  probes_t P = {n_orders, orders, n_sigmas, sigmas, n_elements, prim_offsets, B, beta, tau, screen};
  int st = check_probes(&P);
  if (st) return st;
  for (int i = 0; i < n_atoms; ++i)
    if (species[i] < 0 || species[i] >= n_elements) return OR_E_INVALID;
  for (int t = 0; t < n_list; ++t)
    if (list[t] < 0 || list[t] >= n_atoms) return OR_E_INVALID;
  const int ns = n_slots(&P);
  double *rc2 = (double *)malloc(sizeof(double) * ns);
  st = slot_cutoffs(&P, rc2);
  double rcmax2 = 0.0;
  for (int s = 0; s < ns; ++s) if (rc2[s] > rcmax2) rcmax2 = rc2[s];
  sys_t S; double *rw = NULL; int32_t *m = NULL;
  if (!st) st = make_sys(&S, n_atoms, pos, species, cell, pbc, rcmax2, &rw, &m);
  if (st) { free(rc2); return st; }
  S.occ = occ;
  const int nc = total_comps(&P), nf = total_feats(&P);
  pair_t **pairs = (pair_t **)calloc((size_t)(n_list > 0 ? n_list : 1), sizeof(pair_t *));
  int64_t *np = (int64_t *)calloc((size_t)(n_list > 0 ? n_list : 1), sizeof(int64_t));
  double **vv = (double **)calloc((size_t)(n_list > 0 ? n_list : 1), sizeof(double *));
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < n_list; ++t) {
    double *mu = (double *)malloc(sizeof(double) * (size_t)nc);
    double *W = (double *)malloc(sizeof(double) * (size_t)nc);
    double *Fi = (double *)malloc(sizeof(double) * nf);
    np[t] = collect(&S, list[t], ns, rc2, &pairs[t]);
    centre_features(&P, pairs[t], np[t], rc2, mu, Fi);
    make_W(&P, mu, Fi, G + (size_t)t * nf, W);
    vv[t] = (double *)malloc(sizeof(double) * 3 * (size_t)(np[t] > 0 ? np[t] : 1));
    for (int64_t p = 0; p < np[t]; ++p) pair_v(&P, pairs[t] + p, rc2, W, vv[t] + 3 * p);
    free(mu); free(W); free(Fi);
  }
  memset(grad_pos, 0, sizeof(double) * 3 * (size_t)n_atoms);
  memset(grad_cell, 0, sizeof(double) * 9);
  for (int t = 0; t < n_list; ++t) {
    const int i = list[t];
    for (int64_t p = 0; p < np[t]; ++p) {
      const double *v = vv[t] + 3 * p;
      const int j = pairs[t][p].j;
      for (int k = 0; k < 3; ++k) { grad_pos[3 * j + k] += v[k]; grad_pos[3 * i + k] -= v[k]; }
      for (int a = 0; a < 3; ++a) {
        double nt = (double)(pairs[t][p].n[a] - m[3 * j + a] + m[3 * i + a]);
        for (int k = 0; k < 3; ++k) grad_cell[3 * a + k] += nt * v[k];
      }
    }
    free(vv[t]); free(pairs[t]);
  }
  free(vv); free(pairs); free(np); free(rc2); free(rw); free(m);
  return OR_OK;
}

/*
 * L = sum G F evaluated over a FROZEN pair set, for finite differences that
 * do not see cutoff crossings.  Pairs of centre i are
 * pj[po[i]..po[i+1]), with raw-position image shifts pn (3 ints each,
 * d = R_j - R_i + pn.cell) and base squared distances pq deciding which
 * slots use each pair (q_base <= rc2 of the slot).  occ as in oracle_features.
 */
static int loss_frozen_impl(const probes_t *Pp, const double *pos, const int32_t *species,
                            const double *cell, int n_centres, const double *cpos,
                            const int64_t *po, const int32_t *pj, const int32_t *pn, const double *pq,
                            const double *G, double *L_out, const double *occ) {
  probes_t P = *Pp;
  int st = check_probes(&P);
  if (st) return st;
  const int ns = n_slots(&P);
  double *rc2 = (double *)malloc(sizeof(double) * ns);
  st = slot_cutoffs(&P, rc2);
  if (st) { free(rc2); return st; }
  int nc = total_comps(&P);
  int nf = total_feats(&P);
  double L = 0.0;
  double *mu = (double *)malloc(sizeof(double) * (size_t)nc);
  double *Fi = (double *)malloc(sizeof(double) * nf);
  for (int i = 0; i < n_centres; ++i) {
    memset(mu, 0, sizeof(double) * (size_t)nc);
    for (int64_t g = po[i]; g < po[i + 1]; ++g) {
      int j = pj[g];
      pair_t pp;
      pp.j = j; pp.e = species[j]; pp.w = occ ? occ[j] : 1.0;
      for (int c = 0; c < 3; ++c) {
        double sh = (double)pn[3 * g] * cell[c] + (double)pn[3 * g + 1] * cell[3 + c] +
                    (double)pn[3 * g + 2] * cell[6 + c];
        pp.d[c] = (pos[3 * j + c] - cpos[3 * i + c]) + sh;
      }
      pp.q = (pp.d[0] * pp.d[0] + pp.d[1] * pp.d[1]) + pp.d[2] * pp.d[2];
      /* membership from the base configuration, value from the current one */
      pair_terms(&P, &pp, pq[g], rc2, mu);
    }
    norms(&P, mu, Fi);
    for (int f = 0; f < nf; ++f) L += G[(size_t)i * nf + f] * Fi[f];
  }
  free(mu); free(Fi); free(rc2);
  *L_out = L;
  return OR_OK;
}

int oracle_loss_frozen(int n_atoms, const double *pos, const int32_t *species,
                       const double *cell,
                       int n_orders, const int32_t *orders, int n_sigmas, const double *sigmas,
                       int n_elements, const int32_t *prim_offsets, const double *B,
                       const double *beta, double tau, int screen,
                       const int64_t *po, const int32_t *pj, const int32_t *pn, const double *pq,
                       const double *G, double *L_out, const double *occ) {
  probes_t P = {n_orders, orders, n_sigmas, sigmas, n_elements, prim_offsets, B, beta, tau, screen};
  return loss_frozen_impl(&P, pos, species, cell, n_atoms, pos, po, pj, pn, pq, G, L_out, occ);
}

/*
 * Full feature Jacobian (the paper's feature derivatives with respect to
 * the atom positions, "Examples"), per pair: for centre i and pair p = (j, n)
 * of its canonical list, J[p][f][k] = dF_{i,f} / d d_p,k, the derivative with
 * respect to the pair's displacement d_p = R_j + n.cell - R_i.  Then
 *   dF_{i,f}/dR_j = sum over pairs p of i with neighbour j of J[p][f]
 *                   minus, for j = i, the sum over all pairs of i,
 * and dF_{i,f}/da_m = sum_p (n_m - m_j,m + m_i,m) J[p][f].  Pairs of centre
 * i start at the running sum of the list lengths of the centres before it;
 * writes at most cap pairs and returns the total pair count.
 */
int64_t oracle_jacobian(int n_atoms, const double *pos, const int32_t *species,
                        const double *cell, int pbc,
                        int n_orders, const int32_t *orders, int n_sigmas, const double *sigmas,
                        int n_elements, const int32_t *prim_offsets, const double *B,
                        const double *beta, double tau, int screen, int64_t cap, double *jac,
                        const double *occ, int32_t *status) {
  probes_t P = {n_orders, orders, n_sigmas, sigmas, n_elements, prim_offsets, B, beta, tau, screen};
  *status = check_probes(&P);
  if (*status) return 0;
  for (int i = 0; i < n_atoms; ++i)
    if (species[i] < 0 || species[i] >= n_elements) { *status = OR_E_INVALID; return 0; }
  const int ns = n_slots(&P);
  double *rc2 = (double *)malloc(sizeof(double) * ns);
  int st = slot_cutoffs(&P, rc2);
  double rcmax2 = 0.0;
  for (int s = 0; s < ns; ++s) if (rc2[s] > rcmax2) rcmax2 = rc2[s];
  sys_t S; double *rw = NULL; int32_t *m = NULL;
  if (!st) st = make_sys(&S, n_atoms, pos, species, cell, pbc, rcmax2, &rw, &m);
  if (st) { free(rc2); *status = st; return 0; }
  S.occ = occ;
  const int nc = total_comps(&P), nf = total_feats(&P);
  double *mu = (double *)malloc(sizeof(double) * (size_t)nc);
  double *W = (double *)malloc(sizeof(double) * (size_t)nc);
  double *Fi = (double *)malloc(sizeof(double) * nf);
  double *G = (double *)malloc(sizeof(double) * nf);
  int64_t base = 0;
  for (int i = 0; i < n_atoms; ++i) {
    pair_t *pairs;
    int64_t np = collect(&S, i, ns, rc2, &pairs);
    centre_features(&P, pairs, np, rc2, mu, Fi);
    for (int f = 0; f < nf; ++f) {
      /* dF_f / dmu = W with the upstream gradient the unit vector of f */
      for (int t = 0; t < nf; ++t) G[t] = t == f ? 1.0 : 0.0;
      make_W(&P, mu, Fi, G, W);
      for (int64_t p = 0; p < np; ++p) {
        if (base + p >= cap) break;
        double v[3];
        pair_v(&P, pairs + p, rc2, W, v);
        for (int k = 0; k < 3; ++k) jac[((size_t)(base + p) * nf + f) * 3 + k] = v[k];
      }
    }
    base += np;
    free(pairs);
  }
  free(mu); free(W); free(Fi); free(G); free(rc2); free(rw); free(m);
  return base;
}

/* ------------------------------------------------------------------ */
/* reference points                                                    */
/* ------------------------------------------------------------------ */
/*
 * Features at reference points instead of atoms (section "Overview": any set
 * of positions inside the system).  A point r is a centre that is not an
 * atom: its wrapped position Pw_r and wrap indices m_r follow the atoms'
 * rule, its pairs are every atom image (j, n) with q <= max rc^2,
 * d = (Rw_j - Pw_r) + s(n), in the canonical order, and its features follow
 * the same formulas (a point has no self term of its own).  In the gradient
 * the point is a variable of its own:
 *   dL/dR_j += v,  dL/dP_r -= v,  dL/da_m += (n_m - m_j,m + m_r,m) v.
 */
typedef struct {
  sys_t S; double *rw; int32_t *m;   /* atoms */
  double *prw; int32_t *pm;          /* points, wrapped */
  double *rc2; int ns;
} point_sys_t;

static void point_sys_free(point_sys_t *Q) {
  free(Q->rw); free(Q->m); free(Q->prw); free(Q->pm); free(Q->rc2);
}

static int point_sys(point_sys_t *Q, const probes_t *P, int n_atoms, const double *pos,
                     const int32_t *species, const double *cell, int pbc, int n_points,
                     const double *points) {
  memset(Q, 0, sizeof(*Q));
  int st = check_probes(P);
  if (st) return st;
  for (int i = 0; i < n_atoms; ++i)
    if (species[i] < 0 || species[i] >= P->n_elements) return OR_E_INVALID;
  Q->ns = n_slots(P);
  Q->rc2 = (double *)malloc(sizeof(double) * Q->ns);
  st = slot_cutoffs(P, Q->rc2);
  double rcmax2 = 0.0;
  for (int s = 0; s < Q->ns; ++s) if (Q->rc2[s] > rcmax2) rcmax2 = Q->rc2[s];
  if (!st) st = make_sys(&Q->S, n_atoms, pos, species, cell, pbc, rcmax2, &Q->rw, &Q->m);
  if (st) { free(Q->rc2); Q->rc2 = NULL; return st; }
  Q->prw = (double *)malloc(sizeof(double) * 3 * (n_points > 0 ? n_points : 1));
  Q->pm = (int32_t *)malloc(sizeof(int32_t) * 3 * (n_points > 0 ? n_points : 1));
  st = oracle_wrap(n_points, points, cell, pbc, Q->prw, Q->pm);
  if (st) point_sys_free(Q);
  return st;
}

/* canonical list of one reference point (n_slots, rc2 as in oracle_neighbors) */
int64_t oracle_point_neighbors(int n_atoms, const double *pos, const int32_t *species,
                               const double *cell, int pbc, int n_slots_, const double *rc2,
                               const double *point, int64_t cap, int32_t *out_j, int32_t *out_n,
                               double *out_q, int32_t *out_shell, int32_t *status) {
  double rcmax2 = 0.0;
  for (int s = 0; s < n_slots_; ++s) if (rc2[s] > rcmax2) rcmax2 = rc2[s];
  sys_t S; double *rw; int32_t *m;
  *status = make_sys(&S, n_atoms, pos, species, cell, pbc, rcmax2, &rw, &m);
  if (*status) return 0;
  double prw[3]; int32_t pm[3];
  *status = oracle_wrap(1, point, cell, pbc, prw, pm);
  if (*status) { free(rw); free(m); return 0; }
  pair_t *Pl;
  int64_t n = collect_at(&S, prw, n_slots_, rc2, &Pl);
  for (int64_t k = 0; k < n && k < cap; ++k) {
    out_j[k] = Pl[k].j;
    out_n[3 * k] = Pl[k].n[0]; out_n[3 * k + 1] = Pl[k].n[1]; out_n[3 * k + 2] = Pl[k].n[2];
    out_q[k] = Pl[k].q; out_shell[k] = Pl[k].shell;
  }
  free(Pl); free(rw); free(m);
  return n;
}

/* F [n_points][nf] and optionally mu [n_points][nc] at the reference points */
int oracle_point_features(int n_atoms, const double *pos, const int32_t *species,
                          const double *cell, int pbc,
                          int n_orders, const int32_t *orders, int n_sigmas, const double *sigmas,
                          int n_elements, const int32_t *prim_offsets, const double *B,
                          const double *beta, double tau, int screen,
                          int n_points, const double *points, double *F, double *mu, const double *occ) {
  probes_t P = {n_orders, orders, n_sigmas, sigmas, n_elements, prim_offsets, B, beta, tau, screen};
  point_sys_t Q;
  int st = point_sys(&Q, &P, n_atoms, pos, species, cell, pbc, n_points, points);
  if (st) return st;
  Q.S.occ = occ;
  const int nc = total_comps(&P), nf = total_feats(&P);
#pragma omp parallel for schedule(dynamic, 1)
  for (int r = 0; r < n_points; ++r) {
    pair_t *pairs;
    int64_t np = collect_at(&Q.S, Q.prw + 3 * r, Q.ns, Q.rc2, &pairs);
    double *mu_r = (double *)malloc(sizeof(double) * (size_t)nc);
    centre_features(&P, pairs, np, Q.rc2, mu_r, F + (size_t)r * nf);
    if (mu) memcpy(mu + (size_t)r * nc, mu_r, sizeof(double) * (size_t)nc);
    free(mu_r); free(pairs);
  }
  point_sys_free(&Q);
  return OR_OK;
}

/* gradient of L = sum G F over the points' features: grad_pos [n_atoms*3],
 * grad_points [n_points*3], grad_cell [9]; F_out [n_points*nf] optional */
int oracle_point_grad(int n_atoms, const double *pos, const int32_t *species,
                      const double *cell, int pbc,
                      int n_orders, const int32_t *orders, int n_sigmas, const double *sigmas,
                      int n_elements, const int32_t *prim_offsets, const double *B,
                      const double *beta, double tau, int screen,
                      int n_points, const double *points, const double *G, double *grad_pos,
                      double *grad_points, double *grad_cell, double *F_out, const double *occ) {
  probes_t P = {n_orders, orders, n_sigmas, sigmas, n_elements, prim_offsets, B, beta, tau, screen};
  point_sys_t Q;
  int st = point_sys(&Q, &P, n_atoms, pos, species, cell, pbc, n_points, points);
  if (st) return st;
  Q.S.occ = occ;
  const int nc = total_comps(&P), nf = total_feats(&P);
  memset(grad_pos, 0, sizeof(double) * 3 * n_atoms);
  memset(grad_points, 0, sizeof(double) * 3 * n_points);
  memset(grad_cell, 0, sizeof(double) * 9);
  double *mu = (double *)malloc(sizeof(double) * (size_t)nc);
  double *W = (double *)malloc(sizeof(double) * (size_t)nc);
  double *Fr = (double *)malloc(sizeof(double) * nf);
  for (int r = 0; r < n_points; ++r) {
    pair_t *pairs;
    int64_t np = collect_at(&Q.S, Q.prw + 3 * r, Q.ns, Q.rc2, &pairs);
    centre_features(&P, pairs, np, Q.rc2, mu, Fr);
    if (F_out) memcpy(F_out + (size_t)r * nf, Fr, sizeof(double) * nf);
    make_W(&P, mu, Fr, G + (size_t)r * nf, W);
    for (int64_t p = 0; p < np; ++p) {
      double v[3];
      pair_v(&P, pairs + p, Q.rc2, W, v);
      int j = pairs[p].j;
      for (int k = 0; k < 3; ++k) { grad_pos[3 * j + k] += v[k]; grad_points[3 * r + k] -= v[k]; }
      for (int a = 0; a < 3; ++a) {
        double nt = (double)(pairs[p].n[a] - Q.m[3 * j + a] + Q.pm[3 * r + a]);
        for (int k = 0; k < 3; ++k) grad_cell[3 * a + k] += nt * v[k];
      }
    }
    free(pairs);
  }
  free(mu); free(W); free(Fr);
  point_sys_free(&Q);
  return OR_OK;
}

/* L over a frozen pair set of reference points (pairs as in
 * oracle_loss_frozen, d = R_j - P_r + pn.cell) */
int oracle_point_loss_frozen(int n_atoms, const double *pos, const int32_t *species,
                             const double *cell,
                             int n_orders, const int32_t *orders, int n_sigmas, const double *sigmas,
                             int n_elements, const int32_t *prim_offsets, const double *B,
                             const double *beta, double tau, int screen, int n_points, const double *points,
                             const int64_t *po, const int32_t *pj, const int32_t *pn, const double *pq,
                             const double *G, double *L_out, const double *occ) {
  (void)n_atoms;
  probes_t P = {n_orders, orders, n_sigmas, sigmas, n_elements, prim_offsets, B, beta, tau, screen};
  return loss_frozen_impl(&P, pos, species, cell, n_points, points, po, pj, pn, pq, G, L_out, occ);
}

/* rc^2 of every slot (the sigmas, then the density when order -1 is requested) */
int oracle_slot_cutoffs(int n_orders, const int32_t *orders, int n_sigmas, const double *sigmas,
                        int n_elements, const int32_t *prim_offsets, const double *B,
                        const double *beta, double tau, int screen, double *rc2) {
  probes_t P = {n_orders, orders, n_sigmas, sigmas, n_elements, prim_offsets, B, beta, tau, screen};
  int st = check_probes(&P);
  if (st) return st;
  return slot_cutoffs(&P, rc2);
}

/* P_abc and its gradient at npts points (pts [npts*3]); out_g [npts*3] */
void oracle_solid_harmonic(int a, int b, int c, int npts, const double *pts,
                           double *out_v, double *out_g) {
  for (int p = 0; p < npts; ++p) {
    dual x = dvar(pts[3 * p], 0), y = dvar(pts[3 * p + 1], 1), z = dvar(pts[3 * p + 2], 2);
    dual r = solid_harmonic(a, b, c, x, y, z);
    out_v[p] = r.v;
    if (out_g) { out_g[3 * p] = r.g[0]; out_g[3 * p + 1] = r.g[1]; out_g[3 * p + 2] = r.g[2]; }
  }
}

/* c_{l,s,e}(q) at npts values of q (plain value) */
void oracle_radial(int l, double sigma, int n_prims, const double *B, const double *beta,
                   int npts, const double *q, double *out) {
  double alpha = 1.0 / (2.0 * sigma * sigma);
  for (int p = 0; p < npts; ++p) {
    double acc = 0.0;
    for (int k = 0; k < n_prims; ++k) {
      double lam = alpha + beta[k];
      double gam = alpha * beta[k] / lam;
      acc += B[k] * pow(alpha / lam, 1.5) * pow(beta[k] / lam, (double)l) * exp(-gam * q[p]);
    }
    out[p] = acc;
  }
}

/* Threads of the parallel loops over centres (timing of the CPU baseline on
 * one core and on all cores); returns the previous setting. */
int oracle_set_threads(int n) {
  int prev = omp_get_max_threads();
  if (n > 0) omp_set_num_threads(n);
  return prev;
}
