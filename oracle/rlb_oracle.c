/*
 * rlb_oracle.c -- plain FP64 CPU reference ("oracle") of the per-cell,
 * per-timestep update of the ultra-relativistic lattice Boltzmann (RLB)
 * model of Mohseni, Mendoza, Succi and Herrmann (arXiv:1302.1125).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this code.  It shares nothing with
 * the HIP library: its own lattice ordering, its own tables (evaluated from
 * the paper's formulas at run time), its own equilibrium form (the
 * chi/xi form of the expansion rather than a coefficient table), its own
 * recovery route and explicit ghost layers instead of index mapping.
 *
 * The method is an explicit iteration, so the oracle takes its steps in the
 * paper's order and notation, one full-array pass per step part, with no
 * fusion or blocking.  Equation numbers are those of the paper's displayed
 * equations in order of appearance.
 *
 * Readings taken where the paper is silent or garbled (each also pinned by a
 * test in tests/test_oracle_*.py):
 *   - equilibrium: the printed second-order expansion, Eq. (29), does not
 *     satisfy the moment condition Eq. (36); the oracle uses the unique
 *     degree-2 lattice polynomial with the printed structure that does
 *     ("reading M"; see orc_feq_L);
 *   - minmod streaming, Eqs. (47)-(53): the right state uses the differences
 *     of f^{a-} and the divergence is taken between the interfaces x+1/2 and
 *     x-1/2 (conservative upwind MUSCL reading);
 *   - history at the first step: f^eq(t - dt) := f^eq(t);
 *   - open boundaries: zero-gradient copy into two ghost layers;
 *   - Euler mode: equilibrium of the post-streaming moments;
 *   - admissibility guard (optional, off by default): continuous projection
 *     of the energy-momentum moments into the cone |T^{0a}| <= m_max T^{00}.
 *   - basic model (Sec. II): energy-momentum distribution f only (the paper
 *     introduces the density distribution h and its weights with the
 *     extended set); ghost edges needed by the diagonal links are filled axis
 *     by axis (x, then y over the x ghosts, then z), so a later axis's FIXED
 *     face wins at an edge.
 * The shear viscosity the scheme realises is pinned by a Chapman-Enskog
 * expansion (tests/test_oracle_viscosity.py): eta/(eps+p) = (4/27) times the
 * relaxation time (basic: (1/omega - 1/2) dt; extended: dt/omega), which
 * differs from Eq. (41) by the factor 4/sqrt(27) on tau; the eta/s mode
 * uses Eq. (41) as printed.
 */
#include "rlb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  double nu;
  int basic;     /* 0: extended set, 1: basic set      */
  double r;      /* c_t / c_0 = sqrt(27)/nu, Eq. (46) */
  double ca;     /* c_a = sqrt(13)/nu (extended, Eq. (46)) or sqrt(19)/nu (basic) */
  double c0;     /* c_0 = (3/8)(9 - 2 sqrt 3), Eq. (46) */
  int e[ORC_Q][3];
  double xi[ORC_Q][4];
  double w[ORC_Q];
  double wp[ORC_Q];
} lattice_t;

/* Extended D3Q19 set, Eq. (42): rest, c_a(+-1,0,0)_FS, 2 c_a(+-1,+-1,0)_FS;
   4-velocities xi_i = (c_t/c_0, c_a e_i) (Sec. II, after Eq. (30));
   weights Eqs. (43)-(45); density weights Eqs. (59)-(60).
   Basic set (Sec. II, the D3Q19 configuration and its quadrature):
   rest, c_a(+-1,0,0)_FS, c_a(+-1,+-1,0)_FS with c_a = sqrt(19)/nu and the
   same c_t/c_0 and c_0; weights w_0 = 1 + 4 c_t^2 nu^2/(361 c_0^2)
   - c_t^2/(c_a^2 c_0^2), w_1..6 = c_t^2 (361 - 8 c_a^2 nu^2)/(2166 c_0^2 c_a^2),
   w_7..18 = c_t^2 nu^2/(1083 c_0^2); no density weights (f only).
   Density weights (extended set).  Eq. (58) needs sum_i w'_i = 1 and
   sum_i w'_i c^a c^b = delta^{ab}/3 (so that N^mu = n U^mu); with one weight
   per shell that leaves one free parameter.  dens_w = ORC_DENSW_PAPER takes
   the paper's choice, Eqs. (59)-(60) (w'_0 = 1/10; the diagonal weight is
   negative for c_a^2 > 10/9, e.g. at nu = 27^(1/4)).  dens_w =
   ORC_DENSW_ISOTROPIC (not in the paper) fixes the free parameter by
   isotropy of the fourth moment instead, sum w' (c^x)^4 = 3 sum w' (c^x)^2
   (c^y)^2: w'_7..18 = 1/(288 c_a^2), w'_1..6 = 1/(9 c_a^2), w'_0 = 1 -
   17/(24 c_a^2), all non-negative for c_a^2 >= 17/24 (nu <= 4.28). */
static void make_lattice(double nu, int basic, int dens_w, lattice_t* L) {
  memset(L, 0, sizeof(*L));
  L->nu = nu;
  L->basic = basic;
  L->r = sqrt(27.0) / nu;
  L->ca = (basic ? sqrt(19.0) : sqrt(13.0)) / nu;
  L->c0 = 3.0 / 8.0 * (9.0 - 2.0 * sqrt(3.0));
  const int d = basic ? 1 : 2; /* length factor of the diagonal links */
  int k = 1; /* e_0 = 0 */
  for (int a = 0; a < 3; ++a)
    for (int s = 1; s >= -1; s -= 2) {
      L->e[k][a] = s;
      ++k;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = a + 1; b < 3; ++b)
      for (int sa = 1; sa >= -1; sa -= 2)
        for (int sb = 1; sb >= -1; sb -= 2) {
          L->e[k][a] = d * sa;
          L->e[k][b] = d * sb;
          ++k;
        }
  const double r2 = L->r * L->r, ca2 = L->ca * L->ca, nu2 = nu * nu;
  double w0, w1, w2, wp0, wp1, wp2;
  if (basic) {
    w0 = 1.0 + 4.0 * r2 * nu2 / 361.0 - r2 / ca2;
    w1 = r2 / (2166.0 * ca2) * (361.0 - 8.0 * ca2 * nu2);
    w2 = r2 * nu2 / 1083.0;
    wp0 = wp1 = wp2 = NAN; /* no density distribution in the basic model */
  } else {
    w0 = 1.0 + 7.0 * r2 * nu2 / 676.0 - r2 / ca2;
    w1 = r2 / (1014.0 * ca2) * (169.0 - 2.0 * ca2 * nu2);
    w2 = r2 * nu2 / 8112.0;
    if (dens_w == ORC_DENSW_ISOTROPIC) {
      wp0 = 1.0 - 17.0 / (24.0 * ca2);
      wp1 = 1.0 / (9.0 * ca2);
      wp2 = 1.0 / (288.0 * ca2);
    } else {
      wp0 = 1.0 / 10.0;
      wp1 = 6.0 / 35.0 - 1.0 / (42.0 * ca2);
      wp2 = 1.0 / (84.0 * ca2) - 3.0 / 280.0;
    }
  }
  for (int i = 0; i < ORC_Q; ++i) {
    const int zeros = (L->e[i][0] == 0) + (L->e[i][1] == 0) + (L->e[i][2] == 0);
    L->xi[i][0] = L->r;
    for (int a = 0; a < 3; ++a) L->xi[i][1 + a] = L->ca * L->e[i][a];
    /* rest (3 zero components), axis links (2), diagonal links (1) */
    L->w[i] = (zeros == 3) ? w0 : (zeros == 2) ? w1 : w2;
    L->wp[i] = (zeros == 3) ? wp0 : (zeros == 2) ? wp1 : wp2;
  }
}

void orc_lattice(double nu, int basic, int dens_w, int* e, double* xi, double* w, double* wp) {
  lattice_t L;
  make_lattice(nu, basic, dens_w, &L);
  for (int i = 0; i < ORC_Q; ++i) {
    for (int a = 0; a < 3; ++a) e[3 * i + a] = L.e[i][a];
    for (int a = 0; a < 4; ++a) xi[4 * i + a] = L.xi[i][a];
    w[i] = L.w[i];
    wp[i] = L.wp[i];
  }
}

/* Discrete Maxwell-Juttner equilibrium (reading M).
 *
 * The expansion keeps the structure of Eq. (29): a first-order term
 * proportional to (xi . chi), off-diagonal second-order terms
 * xi^a xi^b chi^a chi^b with coefficient 1, diagonal terms
 * (xi^a)^2 (chi^a)^2 and an isotropic |chi|^2 term.  With constant xi^0
 * (Sec. II, after Eq. (30)) the temporal components are xi^0 = c_t/c_0 and
 * chi^0 -> chi^0 / c_0, chi^0 = nu gamma.  The first-order coefficient keeps
 * the part of the printed coefficient of Eq. (29) proportional to chi^0,
 * i.e. (chi^0/c_0) xi^0 / 2 - (chi^0/c_0)/nu = gamma (sqrt27/2 - 1)/c_0.
 * The diagonal (+4/15) and isotropic (-16/(15 nu^2)) coefficients and the
 * amplitude A = nu^2 eps / 27 are the unique values for which the discrete
 * second moments satisfy Eq. (36) with eps = 3p (Eq. (38)) exactly;
 * the constant 3/2 - xi^0 nu / 4 of the printed first-order coefficient and
 * its printed diagonal/isotropic coefficients violate Eq. (36) and are not
 * used.  chi^a = U^a / c_s = nu gamma u^a (Sec. II, Eqs. (4)-(8), c = 1). */
static void feq_L(const lattice_t* L, double eps, double ux, double uy,
                  double uz, double* feq) {
  const double nu = L->nu;
  const double u2 = ux * ux + uy * uy + uz * uz;
  const double gam = 1.0 / sqrt(1.0 - u2);
  const double chi[3] = {nu * gam * ux, nu * gam * uy, nu * gam * uz};
  const double chi2 = chi[0] * chi[0] + chi[1] * chi[1] + chi[2] * chi[2];
  const double A = nu * nu * eps / 27.0;
  const double first = gam * (sqrt(27.0) / 2.0 - 1.0) / L->c0;
  for (int i = 0; i < ORC_Q; ++i) {
    const double* x = &L->xi[i][1];
    const double xc = x[0] * chi[0] + x[1] * chi[1] + x[2] * chi[2];
    const double off = x[0] * x[1] * chi[0] * chi[1] +
                       x[0] * x[2] * chi[0] * chi[2] +
                       x[1] * x[2] * chi[1] * chi[2];
    const double dia = x[0] * x[0] * chi[0] * chi[0] +
                       x[1] * x[1] * chi[1] * chi[1] +
                       x[2] * x[2] * chi[2] * chi[2];
    feq[i] = A * L->w[i] *
             (1.0 - 16.0 / (15.0 * nu * nu) * chi2 + first * xc + off +
              4.0 / 15.0 * dia);
  }
}

/* Density equilibrium, Eq. (58): h_i = w'_i n gamma (c_0/c_t + 3 (c.u)
   + 9/2 (c.u)^2 - 3/2 |u|^2), with c the spatial lattice vector c_a e_i. */
static void heq_L(const lattice_t* L, double n, double ux, double uy,
                  double uz, double* heq) {
  const double u2 = ux * ux + uy * uy + uz * uz;
  const double gam = 1.0 / sqrt(1.0 - u2);
  for (int i = 0; i < ORC_Q; ++i) {
    const double cu = L->xi[i][1] * ux + L->xi[i][2] * uy + L->xi[i][3] * uz;
    heq[i] = L->wp[i] * n * gam *
             (1.0 / L->r + 3.0 * cu + 4.5 * cu * cu - 1.5 * u2);
  }
}

void orc_feq(double nu, int basic, double eps, double ux, double uy, double uz,
             double* feq) {
  lattice_t L;
  make_lattice(nu, basic, ORC_DENSW_PAPER, &L);
  feq_L(&L, eps, ux, uy, uz, feq);
}

void orc_heq(double nu, int basic, int dens_w, double n, double ux, double uy, double uz,
             double* heq) {
  lattice_t L;
  make_lattice(nu, basic, dens_w, &L);
  heq_L(&L, n, ux, uy, uz, heq);
}

/* T^{0 mu} = sum_i xi^0 xi^mu f_i and N^0 = sum_i xi^0 h_i (Eq. (36) and the
   number current of Sec. II), summed in the oracle's population order. */
static void moments_L(const lattice_t* L, const double* f, long fs,
                      const double* h, long hs, double* T0, double* N0) {
  double t[4] = {0, 0, 0, 0}, n0 = 0;
  for (int i = 0; i < ORC_Q; ++i) {
    const double fi = f[i * fs];
    for (int m = 0; m < 4; ++m) t[m] += L->xi[i][0] * L->xi[i][m] * fi;
    if (h) n0 += L->xi[i][0] * h[i * hs];
  }
  for (int m = 0; m < 4; ++m) T0[m] = t[m];
  *N0 = n0;
}

void orc_moments(double nu, int basic, const double* f, const double* h, double* T0,
                 double* N0) {
  lattice_t L;
  make_lattice(nu, basic, ORC_DENSW_PAPER, &L); /* the moments do not use w' */
  moments_L(&L, f, 1, h, 1, T0, N0);
}

/* Fields from T^{00}, T^{0a} (and N^0) with the ultra-relativistic equation of
 * state eps = 3p, Eq. (38) (Sec. II: four equations for eps, U^a).
 * With T^{00} = (eps+p) gamma^2 - p and T^{0a} = (eps+p) gamma^2 u^a the ratio
 * m = |T^{0a}|/T^{00} = 4|u|/(3+|u|^2); |u| is the root in [0,1) of
 * m u^2 - 4u + 3m = 0, then eps = 3 T^{00}/(4 gamma^2 - 1), n = N^0/gamma.
 * Without h, n is the lattice-unit equilibrium density n = T^3 with
 * eps = 3 T^4 (fugacity 1).  Returns -1 (fields NaN) when T^{00} <= 0,
 * |T^{0a}| >= T^{00}, N^0 <= 0 (with h) or anything is non-finite. */
int orc_recover(double T00, double T0x, double T0y, double T0z, double N0,
                int with_h, double* fields) {
  const double Mabs = sqrt(T0x * T0x + T0y * T0y + T0z * T0z);
  const int ok = isfinite(T00) && isfinite(Mabs) && T00 > 0.0 &&
                 Mabs < T00 && (!with_h || (isfinite(N0) && N0 > 0.0));
  if (!ok) {
    for (int k = 0; k < 5; ++k) fields[k] = NAN;
    return -1;
  }
  const double m = Mabs / T00;
  const double u = 3.0 * m / (2.0 + sqrt(4.0 - 3.0 * m * m));
  const double g2 = 1.0 / ((1.0 - u) * (1.0 + u));
  const double eps = 3.0 * T00 / (4.0 * g2 - 1.0);
  const double s = (Mabs > 0.0) ? u / Mabs : 0.0;
  fields[0] = eps;
  fields[1] = s * T0x;
  fields[2] = s * T0y;
  fields[3] = s * T0z;
  fields[4] = with_h ? N0 / sqrt(g2) : pow(eps / 3.0, 0.75);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Whole-domain stepper                                                      */
/* ------------------------------------------------------------------------ */

struct orc_state {
  orc_config cfg;
  lattice_t L;
  int n[3], pad[3], N[3];
  long ncell, npad;
  double *f, *h, *fn, *hn, *fs, *hs; /* [i][padded cell]          */
  double *fields, *hist;              /* [k][cell], k = eps,ux,uy,uz,n */
  double* obst_fields;                /* [k][cell]                  */
  uint8_t* obst;                      /* [cell] or NULL             */
  double face_f[6][ORC_Q], face_h[6][ORC_Q];
  double m1, mmax;                    /* guard ramp                 */
  int64_t step, guard_events;
};

/* Padded index of (x,y,z); axes of size 1 map every coordinate to 0, so the
   neighbour of the single cell is itself (a periodic axis of length 1). */
static inline long pidx(const orc_state* S, int x, int y, int z) {
  const int c[3] = {x, y, z};
  long id = 0;
  for (int a = 2; a >= 0; --a) {
    const int q = (S->n[a] == 1) ? 0 : c[a] + S->pad[a];
    id = id * S->N[a] + q;
  }
  return id;
}

static inline long cidx(const orc_state* S, int x, int y, int z) {
  return x + (long)S->n[0] * (y + (long)S->n[1] * z);
}

static double* alloc_nan(long count) {
  double* p = (double*)malloc(sizeof(double) * (size_t)count);
  if (p)
    for (long k = 0; k < count; ++k) p[k] = NAN;
  return p;
}

static void guard_ramp(double umax, double* m1, double* mmax) {
  /* T^{0a}/T^{00} at speed u is 4u/(3+u^2); the blend ramps over speeds
     [1 - 2(1-umax), umax]. */
  const double u1 = 1.0 - 2.0 * (1.0 - umax);
  *mmax = 4.0 * umax / (3.0 + umax * umax);
  *m1 = 4.0 * u1 / (3.0 + u1 * u1);
}

orc_state* orc_create(const orc_config* cfg) {
  if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return NULL;
  if (cfg->guard_umax > 0 && !(cfg->guard_umax < 1 && cfg->guard_efloor > 0))
    return NULL;
  const int n[3] = {cfg->nx, cfg->ny, cfg->nz};
  for (int a = 0; a < 3; ++a) {
    const int lo = cfg->bc[2 * a], hi = cfg->bc[2 * a + 1];
    if ((lo == ORC_BC_PERIODIC) != (hi == ORC_BC_PERIODIC)) return NULL;
    if (n[a] == 1 && (lo == ORC_BC_FIXED || hi == ORC_BC_FIXED)) return NULL;
    if (n[a] == 1 && lo != ORC_BC_PERIODIC) return NULL;
  }
  if (cfg->basic && (cfg->euler || cfg->alpha != 0.0 || cfg->guard_umax > 0 || cfg->with_h))
    return NULL;
  if (cfg->dens_w != ORC_DENSW_PAPER && cfg->dens_w != ORC_DENSW_ISOTROPIC) return NULL;
  if (cfg->flux != ORC_FLUX_MINMOD && cfg->flux != ORC_FLUX_RUSANOV) return NULL;
  if (cfg->flux == ORC_FLUX_RUSANOV && cfg->basic) return NULL;
  if (cfg->dens_w == ORC_DENSW_ISOTROPIC &&
      (cfg->basic || 13.0 / (cfg->nu * cfg->nu) < 17.0 / 24.0))
    return NULL; /* extended set only; w'_0 >= 0 needs c_a^2 >= 17/24 */
  orc_state* S = (orc_state*)calloc(1, sizeof(orc_state));
  S->cfg = *cfg;
  make_lattice(cfg->nu, cfg->basic, cfg->dens_w, &S->L);
  S->ncell = 1;
  S->npad = 1;
  for (int a = 0; a < 3; ++a) {
    S->n[a] = n[a];
    S->pad[a] = (n[a] > 1) ? 2 : 0;
    S->N[a] = n[a] + 2 * S->pad[a];
    S->ncell *= n[a];
    S->npad *= S->N[a];
  }
  const long P = ORC_Q * S->npad;
  S->f = alloc_nan(P);
  S->fn = alloc_nan(P);
  S->fs = (cfg->euler || cfg->basic) ? alloc_nan(P) : NULL;
  if (cfg->with_h) {
    S->h = alloc_nan(P);
    S->hn = alloc_nan(P);
    S->hs = (cfg->euler || cfg->basic) ? alloc_nan(P) : NULL;
  }
  S->fields = alloc_nan(5 * S->ncell);
  S->hist = alloc_nan(5 * S->ncell);
  for (int s = 0; s < 6; ++s) {
    const double* q = cfg->face[s];
    feq_L(&S->L, q[0], q[1], q[2], q[3], S->face_f[s]);
    heq_L(&S->L, q[4], q[1], q[2], q[3], S->face_h[s]);
  }
  if (cfg->guard_umax > 0) guard_ramp(cfg->guard_umax, &S->m1, &S->mmax);
  return S;
}

void orc_destroy(orc_state* S) {
  if (!S) return;
  free(S->f); free(S->fn); free(S->fs);
  free(S->h); free(S->hn); free(S->hs);
  free(S->fields); free(S->hist); free(S->obst_fields); free(S->obst);
  free(S);
}

int orc_init(orc_state* S, const double* eps, const double* ux,
             const double* uy, const double* uz, const double* n,
             const uint8_t* obstacle) {
  const long NC = S->ncell;
  for (long c = 0; c < NC; ++c) {
    const double u2 = ux[c] * ux[c] + uy[c] * uy[c] + uz[c] * uz[c];
    if (!(isfinite(eps[c]) && isfinite(u2) && eps[c] > 0 && u2 < 1.0)) return -4;
    if (S->cfg.with_h && !(n && isfinite(n[c]) && n[c] > 0)) return -4;
  }
  for (int z = 0; z < S->n[2]; ++z)
    for (int y = 0; y < S->n[1]; ++y)
      for (int x = 0; x < S->n[0]; ++x) {
        const long c = cidx(S, x, y, z), p = pidx(S, x, y, z);
        double fe[ORC_Q], he[ORC_Q];
        feq_L(&S->L, eps[c], ux[c], uy[c], uz[c], fe);
        for (int i = 0; i < ORC_Q; ++i) S->f[i * S->npad + p] = fe[i];
        if (S->cfg.with_h) {
          heq_L(&S->L, n[c], ux[c], uy[c], uz[c], he);
          for (int i = 0; i < ORC_Q; ++i) S->h[i * S->npad + p] = he[i];
        }
        /* history := initial fields, so f^eq(t - dt) = f^eq(t) at step 1 */
        S->hist[0 * NC + c] = eps[c];
        S->hist[1 * NC + c] = ux[c];
        S->hist[2 * NC + c] = uy[c];
        S->hist[3 * NC + c] = uz[c];
        S->hist[4 * NC + c] = S->cfg.with_h ? n[c] : pow(eps[c] / 3.0, 0.75);
      }
  free(S->obst);
  free(S->obst_fields);
  S->obst = NULL;
  S->obst_fields = NULL;
  if (obstacle) {
    S->obst = (uint8_t*)malloc((size_t)NC);
    memcpy(S->obst, obstacle, (size_t)NC);
    S->obst_fields = (double*)malloc(sizeof(double) * 5 * (size_t)NC);
    memcpy(S->obst_fields, S->hist, sizeof(double) * 5 * (size_t)NC);
  }
  S->step = 0;
  S->guard_events = 0;
  return 0;
}

/* Ghost layers (two, faces only: the stencil is star-shaped) per boundary
   condition: periodic copy, fixed state (the face's equilibrium, as for the
   paper's inlet in Sec. III) or zero-gradient outflow ("open" boundaries). */
static void fill_ghosts(orc_state* S, double* arr, const double face[6][ORC_Q]) {
  for (int a = 0; a < 3; ++a) {
    if (S->n[a] == 1) continue;
    const int b = (a + 1) % 3, d = (a + 2) % 3;
    for (int g = 1; g <= 2; ++g)
      for (int side = 0; side < 2; ++side) {
        const int bc = S->cfg.bc[2 * a + side];
        const int ghost = side ? S->n[a] - 1 + g : -g;
        int src;
        if (bc == ORC_BC_PERIODIC) src = side ? g - 1 : S->n[a] - g;
        else src = side ? S->n[a] - 1 : 0;
        for (int jb = 0; jb < S->n[b]; ++jb)
          for (int jd = 0; jd < S->n[d]; ++jd) {
            int cg[3], cs[3];
            cg[a] = ghost; cg[b] = jb; cg[d] = jd;
            cs[a] = src; cs[b] = jb; cs[d] = jd;
            const long pg = pidx(S, cg[0], cg[1], cg[2]);
            const long ps = pidx(S, cs[0], cs[1], cs[2]);
            for (int i = 0; i < ORC_Q; ++i)
              arr[i * S->npad + pg] = (bc == ORC_BC_FIXED)
                                          ? face[2 * a + side][i]
                                          : arr[i * S->npad + ps];
          }
      }
  }
}

/* minmod(X,Y) = 1/2 min(|X|,|Y|) [Sign(X) + Sign(Y)], Eq. (53), Sign(0) = 0 */
static inline double sgn(double v) { return (v > 0) - (v < 0); }
static inline double minmod(double X, double Y) {
  return 0.5 * fmin(fabs(X), fabs(Y)) * (sgn(X) + sgn(Y));
}

/* Interface flux h_i^a(X) between cells X and X + e_a, Eqs. (48)-(52):
   h = f^{aL}(X) + f^{aR}(X), f^{a+-} = 1/2 (p +- |p|) f,
   f^{aL}(X) = f^{a+}(X) + 1/2 minmod(df^{a+}(X), df^{a+}(X - e_a)),
   f^{aR}(X) = f^{a-}(X + e_a) - 1/2 minmod(df^{a-}(X), df^{a-}(X + e_a)),
   df(X) = f(X + e_a) - f(X).  (The printed f^{aR} uses df^{a+}; the upwind
   reading with df^{a-} is the one that reduces to the standard limited
   scheme for p < 0.)  fm1..fp2 are f_i at X-1 .. X+2 along a. */
static inline double iface_flux(double p, double fm1, double f0, double fp1,
                                double fp2) {
  const double pp = 0.5 * (p + fabs(p)), pm = 0.5 * (p - fabs(p));
  const double Lp_m1 = pp * fm1, Lp_0 = pp * f0, Lp_1 = pp * fp1;
  const double Rm_0 = pm * f0, Rm_1 = pm * fp1, Rm_2 = pm * fp2;
  const double fL = Lp_0 + 0.5 * minmod(Lp_1 - Lp_0, Lp_0 - Lp_m1);
  const double fR = Rm_1 - 0.5 * minmod(Rm_1 - Rm_0, Rm_2 - Rm_1);
  return fL + fR;
}

static inline double at_off(const orc_state* S, const double* arr_i, int x,
                            int y, int z, int a, int k) {
  int c[3] = {x, y, z};
  c[a] += k;
  return arr_i[pidx(S, c[0], c[1], c[2])];
}

/* Rusanov (local Lax-Friedrichs) interface flux, first order -- beyond the
   paper: h = 1/2 p (f(X) + f(X + e_a)) - 1/2 s (f(X + e_a) - f(X)) with one
   dissipation speed s for every population, moving or not.  With s = xi^0 =
   c_t/c_0 (the speed of light in the units of p) the moments of the update
   are the Rusanov scheme of the macroscopic equations; the divergence of h
   is returned directly. */
static inline double rusanov_div(double p, double s, double fm1, double f0,
                                 double fp1) {
  return 0.5 * p * (fp1 - fm1) - 0.5 * s * ((fp1 - f0) - (f0 - fm1));
}

/* Bulk-term coefficient lambda_i / (c_0 nu dt / c_t) of population i: alpha
   for the moving populations, 0 for the rest population (Eq. (55)).  With the
   Rusanov flux (beyond the paper) the rest population takes the bulk term too:
   its weight is negative, and without it the term would move energy at a
   cell by -kappa times the Laplacian of the rest population's energy, which
   breaks the convexity that keeps that flux's moment update admissible; with
   it the term is kappa times the Laplacian of every moment. */
static inline double bulk_lambda(const orc_state* S, int i) {
  if (i == 0 && S->cfg.flux != ORC_FLUX_RUSANOV) return 0.0;
  return S->cfg.alpha;
}

/* Sum over axes of [h_i^a(x) - h_i^a(x - e_a)] / dx: the divergence of the
   limited flux of p_i^a f_i between the interfaces x +- 1/2 (Eq. (47),
   conservative reading), with p_i^a = xi_i^a; or of the Rusanov flux above
   (ORC_FLUX_RUSANOV, every population along every axis). */
static double div_flux(const orc_state* S, const double* arr_i, int i, int x,
                       int y, int z) {
  double d = 0.0;
  if (S->cfg.flux == ORC_FLUX_RUSANOV) {
    const double s = S->L.xi[i][0];
    for (int a = 0; a < 3; ++a)
      d += rusanov_div(S->L.xi[i][1 + a], s, at_off(S, arr_i, x, y, z, a, -1),
                       arr_i[pidx(S, x, y, z)], at_off(S, arr_i, x, y, z, a, +1));
    return d;
  }
  for (int a = 0; a < 3; ++a) {
    const double p = S->L.xi[i][1 + a];
    if (p == 0.0) continue;
    double v[5];
    for (int k = -2; k <= 2; ++k) v[k + 2] = at_off(S, arr_i, x, y, z, a, k);
    const double right = iface_flux(p, v[1], v[2], v[3], v[4]);
    const double left = iface_flux(p, v[0], v[1], v[2], v[3]);
    d += right - left;
  }
  return d;
}

/* Central second difference sum_a [f(x+e_a) - 2 f(x) + f(x-e_a)] / dx^2
   (the operator of the bulk term, Eq. (54)). */
static double laplacian(const orc_state* S, const double* arr_i, int x, int y,
                        int z) {
  double s = 0.0;
  const double c = arr_i[pidx(S, x, y, z)];
  for (int a = 0; a < 3; ++a)
    s += at_off(S, arr_i, x, y, z, a, +1) - 2.0 * c +
         at_off(S, arr_i, x, y, z, a, -1);
  return s;
}

/* Relaxation time.  UNIFORM: given.  ETA_OVER_S: from Eq. (41),
   tau = 1/2 + nu^2 (eta/s) s / (eps + p), with the entropy density of
   Sec. III, s = 4n - n ln(lambda), lambda = n / n_eq, n_eq = T^3 in lattice
   units (d_G / pi^2 := 1) and T = p / n (p = n T). */
static double tau_of(const orc_state* S, const double* fl) {
  if (S->cfg.tau_mode == ORC_TAU_UNIFORM) return S->cfg.tau;
  const double eps = fl[0], n = fl[4];
  const double p = eps / 3.0;
  const double T = p / n;
  const double lam = n / (T * T * T);
  const double s = 4.0 * n - n * log(lam);
  const double nu = S->L.nu;
  return 0.5 + nu * nu * S->cfg.eta_over_s * s / (eps + p);
}

static void fields_at(const double* arr, long NC, long c, double* out) {
  for (int k = 0; k < 5; ++k) out[k] = arr[k * NC + c];
}

/* Continuous admissibility guard (off unless guard_umax > 0).  Not part of
 * the paper, which is silent on states with T^{00} <= 0, |T^{0a}| >= T^{00}
 * or N^0 <= 0.  Given the moments (T^{00}, T^{0a}, N^0) of a cell's new
 * populations it returns
 *   theta_f: 1 if |T^{0a}| <= m_1 T^{00}, 0 if |T^{0a}| >= m_max T^{00} or
 *            T^{00} <= 0, linear in |T^{0a}|/T^{00} between;
 *   theta_h: min(theta_f, ramp of n_g = N^0/gamma_c from 0 at n_g <= floor to
 *            1 at n_g >= 2 floor);
 *   fc:      fields of the projected moments T^{00}_c = max(T^{00}, floor),
 *            |T^{0a}_c| = min(|T^{0a}|, m_max T^{00}_c), n_c = max(n_g, floor).
 * The populations are then blended f := f^eq(fc) + theta_f (f - f^eq(fc)),
 * h := h^eq(fc) + theta_h (h - h^eq(fc)).  Every step is continuous in the
 * moments.  Returns 1 if theta_f < 1 or theta_h < 1, 0 otherwise (and 0 for
 * non-finite moments, which the next recovery reports). */
static int guard_project(const orc_state* S, const double* T0, double N0,
                         double* theta_f, double* theta_h, double* fc) {
  const int with_h = S->cfg.with_h;
  const double fl = S->cfg.guard_efloor;
  const double E = T0[0];
  const double M = sqrt(T0[1] * T0[1] + T0[2] * T0[2] + T0[3] * T0[3]);
  *theta_f = 1.0;
  *theta_h = 1.0;
  if (!(isfinite(E) && isfinite(M) && (!with_h || isfinite(N0)))) return 0;
  double th;
  if (!(E > 0.0)) th = 0.0;
  else {
    const double m = M / E;
    th = (m <= S->m1) ? 1.0 : (m >= S->mmax) ? 0.0
                                             : (S->mmax - m) / (S->mmax - S->m1);
  }
  const double Ec = fmax(E, fl);
  const double Mc = fmin(M, S->mmax * Ec);
  const double sc = (M > 0.0) ? Mc / M : 0.0;
  orc_recover(Ec, sc * T0[1], sc * T0[2], sc * T0[3], 0.0, 0, fc);
  double thh = th;
  if (with_h) {
    const double u2 = fc[1] * fc[1] + fc[2] * fc[2] + fc[3] * fc[3];
    const double ng = N0 * sqrt(1.0 - u2); /* N^0 / gamma_c */
    const double tn = (ng >= 2.0 * fl) ? 1.0 : (ng <= fl) ? 0.0 : (ng - fl) / fl;
    thh = fmin(th, tn);
    fc[4] = fmax(ng, fl);
  }
  *theta_f = th;
  *theta_h = thh;
  return (th < 1.0 || thh < 1.0) ? 1 : 0;
}

/* Ghost layers of the basic model, whose diagonal links also read the edge
   ghosts: the axes are filled in turn (x, then y over the filled x range,
   then z over the filled x and y ranges), each by its own boundary
   condition as in fill_ghosts, so at an edge a later axis's FIXED face wins
   and otherwise the earlier axis's value is carried along. */
static void fill_ghosts_edges(orc_state* S, double* arr, const double face[6][ORC_Q]) {
  for (int a = 0; a < 3; ++a) {
    if (S->n[a] == 1) continue;
    int lo[3], hi[3];
    for (int b = 0; b < 3; ++b) {
      lo[b] = (b < a) ? -S->pad[b] : 0;
      hi[b] = (b < a) ? S->n[b] + S->pad[b] : S->n[b];
    }
    for (int g = 1; g <= 2; ++g)
      for (int side = 0; side < 2; ++side) {
        const int bc = S->cfg.bc[2 * a + side];
        const int ghost = side ? S->n[a] - 1 + g : -g;
        const int src = (bc == ORC_BC_PERIODIC) ? (side ? g - 1 : S->n[a] - g)
                                                : (side ? S->n[a] - 1 : 0);
        const int b = (a + 1) % 3, d = (a + 2) % 3;
        for (int jb = lo[b]; jb < hi[b]; ++jb)
          for (int jd = lo[d]; jd < hi[d]; ++jd) {
            int cg[3], cs[3];
            cg[a] = ghost; cg[b] = jb; cg[d] = jd;
            cs[a] = src; cs[b] = jb; cs[d] = jd;
            const long pg = pidx(S, cg[0], cg[1], cg[2]);
            const long ps = pidx(S, cs[0], cs[1], cs[2]);
            for (int i = 0; i < ORC_Q; ++i)
              arr[i * S->npad + pg] = (bc == ORC_BC_FIXED)
                                          ? face[2 * a + side][i]
                                          : arr[i * S->npad + ps];
          }
      }
  }
}

/* One step of the basic model (Sec. II):
 *   f_i(x + c_a (c_0/c_t) dt e_i, t + dt) - f_i(x, t)
 *       = -(c_0 nu dt / (tau c_t)) (f_i - f_i^eq),
 * with dt = c_t dx / (c_a c_0), so each population moves exactly one link
 * e_i per step; no bulk term, no limiter, no density distribution.  The
 * collision is applied at every cell, the post-collision values are copied
 * into the ghost layers, and every population is then pulled from x - e_i. */
static int64_t step_basic(orc_state* S, int64_t nsteps) {
  const lattice_t* L = &S->L;
  const long NC = S->ncell, NP = S->npad;
  const double dt = L->r / L->ca;           /* c_t dx / (c_a c_0), dx = 1 */
  const double omega_tau = L->nu * dt / L->r; /* c_0 nu dt / c_t */
  for (int64_t it = 0; it < nsteps; ++it) {
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long c = 0; c < NC; ++c) {
      const int x = (int)(c % S->n[0]);
      const int y = (int)((c / S->n[0]) % S->n[1]);
      const int z = (int)(c / ((long)S->n[0] * S->n[1]));
      const long p = pidx(S, x, y, z);
      double fl[5], fe[ORC_Q];
      if (S->obst && S->obst[c]) {
        /* held at the equilibrium of its prescribed state */
        fields_at(S->obst_fields, NC, c, fl);
        feq_L(L, fl[0], fl[1], fl[2], fl[3], fe);
        for (int i = 0; i < ORC_Q; ++i) S->fs[i * NP + p] = fe[i];
        continue;
      }
      double T0[4], N0;
      moments_L(L, S->f + p, NP, NULL, NP, T0, &N0);
      if (orc_recover(T0[0], T0[1], T0[2], T0[3], N0, 0, fl) != 0) {
        bad = 1;
        continue;
      }
      const double omega = omega_tau / tau_of(S, fl);
      feq_L(L, fl[0], fl[1], fl[2], fl[3], fe);
      for (int i = 0; i < ORC_Q; ++i) {
        const double fi = S->f[i * NP + p];
        S->fs[i * NP + p] = fi - omega * (fi - fe[i]);
      }
    }
    if (bad) return 1 + S->step;
    fill_ghosts_edges(S, S->fs, (const double(*)[ORC_Q])S->face_f);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < NC; ++c) {
      const int x = (int)(c % S->n[0]);
      const int y = (int)((c / S->n[0]) % S->n[1]);
      const int z = (int)(c / ((long)S->n[0] * S->n[1]));
      const long p = pidx(S, x, y, z);
      for (int i = 0; i < ORC_Q; ++i) {
        const long q = pidx(S, x - L->e[i][0], y - L->e[i][1], z - L->e[i][2]);
        S->fn[i * NP + p] = S->fs[i * NP + q];
      }
      if (S->obst && S->obst[c])
        for (int i = 0; i < ORC_Q; ++i) S->fn[i * NP + p] = S->fs[i * NP + p];
    }
    double* t = S->f; S->f = S->fn; S->fn = t;
    S->step += 1;
  }
  return 0;
}

int64_t orc_step(orc_state* S, int64_t nsteps) {
  if (S->cfg.basic) return step_basic(S, nsteps);
  const lattice_t* L = &S->L;
  const long NC = S->ncell, NP = S->npad;
  const int with_h = S->cfg.with_h;
  const double dt = S->cfg.dt, nu = L->nu;
  const double c0_ct = 1.0 / L->r;
  const int guard = S->cfg.guard_umax > 0;
  for (int64_t it = 0; it < nsteps; ++it) {
    fill_ghosts(S, S->f, (const double(*)[ORC_Q])S->face_f);
    if (with_h) fill_ghosts(S, S->h, (const double(*)[ORC_Q])S->face_h);

    /* 1-2: moments and fields at time t */
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long c = 0; c < NC; ++c) {
      const int x = (int)(c % S->n[0]);
      const int y = (int)((c / S->n[0]) % S->n[1]);
      const int z = (int)(c / ((long)S->n[0] * S->n[1]));
      const long p = pidx(S, x, y, z);
      double T0[4], N0, fl[5];
      moments_L(L, S->f + p, NP, with_h ? S->h + p : NULL, NP, T0, &N0);
      const int rc = orc_recover(T0[0], T0[1], T0[2], T0[3], N0, with_h, fl);
      for (int k = 0; k < 5; ++k) S->fields[k * NC + c] = fl[k];
      if (rc != 0 && !(S->obst && S->obst[c])) bad = 1;
    }
    if (bad) return 1 + S->step;

    int64_t events = 0;
    if (S->cfg.euler) {
      /* streaming and bulk term without collision, then f := f^eq of the
         post-streaming moments (Sec. III, inviscid case) */
#pragma omp parallel for schedule(static)
      for (long c = 0; c < NC; ++c) {
        const int x = (int)(c % S->n[0]);
        const int y = (int)((c / S->n[0]) % S->n[1]);
        const int z = (int)(c / ((long)S->n[0] * S->n[1]));
        const long p = pidx(S, x, y, z);
        for (int i = 0; i < ORC_Q; ++i) {
          const double* fi = S->f + i * NP;
          const double lam = bulk_lambda(S, i);
          const double B = c0_ct * nu * dt * lam * laplacian(S, fi, x, y, z);
          S->fs[i * NP + p] = fi[p] - c0_ct * dt * div_flux(S, fi, i, x, y, z) + B;
          if (with_h) {
            const double* hi = S->h + i * NP;
            S->hs[i * NP + p] = hi[p] - c0_ct * dt * div_flux(S, hi, i, x, y, z);
          }
        }
      }
#pragma omp parallel for schedule(static) reduction(| : bad) reduction(+ : events)
      for (long c = 0; c < NC; ++c) {
        const int x = (int)(c % S->n[0]);
        const int y = (int)((c / S->n[0]) % S->n[1]);
        const int z = (int)(c / ((long)S->n[0] * S->n[1]));
        const long p = pidx(S, x, y, z);
        if (S->obst && S->obst[c]) continue;
        double T0[4], N0, fl[5], fe[ORC_Q], he[ORC_Q];
        moments_L(L, S->fs + p, NP, with_h ? S->hs + p : NULL, NP, T0, &N0);
        double thf, thh;
        if (guard && guard_project(S, T0, N0, &thf, &thh, fl)) events += 1;
        else if (orc_recover(T0[0], T0[1], T0[2], T0[3], N0, with_h, fl) != 0) bad = 1;
        feq_L(L, fl[0], fl[1], fl[2], fl[3], fe);
        for (int i = 0; i < ORC_Q; ++i) S->fn[i * NP + p] = fe[i];
        if (with_h) {
          heq_L(L, fl[4], fl[1], fl[2], fl[3], he);
          for (int i = 0; i < ORC_Q; ++i) S->hn[i * NP + p] = he[i];
        }
      }
      if (bad) return 1 + S->step;
    } else {
      /* implicit BGK/Marle update with bulk term, Eq. (57) */
#pragma omp parallel for schedule(static) reduction(+ : events)
      for (long c = 0; c < NC; ++c) {
        const int x = (int)(c % S->n[0]);
        const int y = (int)((c / S->n[0]) % S->n[1]);
        const int z = (int)(c / ((long)S->n[0] * S->n[1]));
        const long p = pidx(S, x, y, z);
        if (S->obst && S->obst[c]) continue;
        double fl[5], hl[5];
        fields_at(S->fields, NC, c, fl);
        fields_at(S->hist, NC, c, hl);
        const double tau = tau_of(S, fl);
        const double omega = c0_ct * nu * dt / tau;
        double fe[ORC_Q], fe_prev[ORC_Q], he[ORC_Q], he_prev[ORC_Q];
        feq_L(L, fl[0], fl[1], fl[2], fl[3], fe);
        feq_L(L, hl[0], hl[1], hl[2], hl[3], fe_prev);
        if (with_h) {
          heq_L(L, fl[4], fl[1], fl[2], fl[3], he);
          heq_L(L, hl[4], hl[1], hl[2], hl[3], he_prev);
        }
        double fnew[ORC_Q], hnew[ORC_Q];
        for (int i = 0; i < ORC_Q; ++i) {
          const double* fi = S->f + i * NP;
          const double lam = bulk_lambda(S, i);
          const double B = c0_ct * nu * dt * lam * laplacian(S, fi, x, y, z);
          const double D = c0_ct * dt * div_flux(S, fi, i, x, y, z);
          fnew[i] = (fi[p] - D + omega * (2.0 * fe[i] - fe_prev[i]) + B) /
                    (1.0 + omega);
          if (with_h) {
            const double* hi = S->h + i * NP;
            const double Dh = c0_ct * dt * div_flux(S, hi, i, x, y, z);
            hnew[i] = (hi[p] - Dh + omega * (2.0 * he[i] - he_prev[i])) /
                      (1.0 + omega);
          }
        }
        if (guard) {
          double T0[4], N0, thf, thh, fc[5];
          moments_L(L, fnew, 1, with_h ? hnew : NULL, 1, T0, &N0);
          if (guard_project(S, T0, N0, &thf, &thh, fc)) {
            double ge[ORC_Q], gh[ORC_Q];
            feq_L(L, fc[0], fc[1], fc[2], fc[3], ge);
            for (int i = 0; i < ORC_Q; ++i) fnew[i] = ge[i] + thf * (fnew[i] - ge[i]);
            if (with_h) {
              heq_L(L, fc[4], fc[1], fc[2], fc[3], gh);
              for (int i = 0; i < ORC_Q; ++i) hnew[i] = gh[i] + thh * (hnew[i] - gh[i]);
            }
            events += 1;
          }
        }
        for (int i = 0; i < ORC_Q; ++i) {
          S->fn[i * NP + p] = fnew[i];
          if (with_h) S->hn[i * NP + p] = hnew[i];
        }
        for (int k = 0; k < 5; ++k) S->hist[k * NC + c] = fl[k];
      }
    }
    /* obstacle cells are held at the equilibrium of their prescribed state
       (Sec. III, astrophysical application) */
    if (S->obst) {
      for (long c = 0; c < NC; ++c) {
        if (!S->obst[c]) continue;
        const int x = (int)(c % S->n[0]);
        const int y = (int)((c / S->n[0]) % S->n[1]);
        const int z = (int)(c / ((long)S->n[0] * S->n[1]));
        const long p = pidx(S, x, y, z);
        double of[5], fe[ORC_Q], he[ORC_Q];
        fields_at(S->obst_fields, NC, c, of);
        feq_L(L, of[0], of[1], of[2], of[3], fe);
        for (int i = 0; i < ORC_Q; ++i) S->fn[i * NP + p] = fe[i];
        if (with_h) {
          heq_L(L, of[4], of[1], of[2], of[3], he);
          for (int i = 0; i < ORC_Q; ++i) S->hn[i * NP + p] = he[i];
        }
      }
    }
    double* t = S->f; S->f = S->fn; S->fn = t;
    if (with_h) { t = S->h; S->h = S->hn; S->hn = t; }
    S->guard_events += events;
    S->step += 1;
  }
  return 0;
}

void orc_fields(const orc_state* S, double* eps, double* ux, double* uy,
                double* uz, double* n) {
  const long NC = S->ncell, NP = S->npad;
  for (int z = 0; z < S->n[2]; ++z)
    for (int y = 0; y < S->n[1]; ++y)
      for (int x = 0; x < S->n[0]; ++x) {
        const long c = cidx(S, x, y, z), p = pidx(S, x, y, z);
        double T0[4], N0, fl[5];
        moments_L(&S->L, S->f + p, NP, S->cfg.with_h ? S->h + p : NULL, NP,
                  T0, &N0);
        orc_recover(T0[0], T0[1], T0[2], T0[3], N0, S->cfg.with_h, fl);
        eps[c] = fl[0]; ux[c] = fl[1]; uy[c] = fl[2]; uz[c] = fl[3];
        if (n) n[c] = fl[4];
      }
  (void)NC;
}

void orc_get_pops(const orc_state* S, double* f, double* h) {
  const long NC = S->ncell, NP = S->npad;
  for (int z = 0; z < S->n[2]; ++z)
    for (int y = 0; y < S->n[1]; ++y)
      for (int x = 0; x < S->n[0]; ++x) {
        const long c = cidx(S, x, y, z), p = pidx(S, x, y, z);
        for (int i = 0; i < ORC_Q; ++i) {
          f[i * NC + c] = S->f[i * NP + p];
          if (h && S->cfg.with_h) h[i * NC + c] = S->h[i * NP + p];
        }
      }
}

void orc_set_pops(orc_state* S, const double* f, const double* h,
                  const double* hist) {
  const long NC = S->ncell, NP = S->npad;
  for (int z = 0; z < S->n[2]; ++z)
    for (int y = 0; y < S->n[1]; ++y)
      for (int x = 0; x < S->n[0]; ++x) {
        const long c = cidx(S, x, y, z), p = pidx(S, x, y, z);
        for (int i = 0; i < ORC_Q; ++i) {
          S->f[i * NP + p] = f[i * NC + c];
          if (h && S->cfg.with_h) S->h[i * NP + p] = h[i * NC + c];
        }
      }
  if (hist) memcpy(S->hist, hist, sizeof(double) * 5 * (size_t)NC);
}

void orc_get_hist(const orc_state* S, double* hist) {
  memcpy(hist, S->hist, sizeof(double) * 5 * (size_t)S->ncell);
}

int64_t orc_guard_events(const orc_state* S) { return S->guard_events; }

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads later parallel regions use (timing of the oracle at one thread and
   at all cores); no effect on results. */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
