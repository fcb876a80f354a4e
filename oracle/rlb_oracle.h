/*
 * rlb_oracle.h -- plain FP64 CPU reference ("oracle") of the per-cell,
 * per-timestep update of the ultra-relativistic lattice Boltzmann model of
 * Mohseni, Mendoza, Succi and Herrmann, "Lattice Boltzmann model for
 * ultra-relativistic flows" (arXiv:1302.1125).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant with the HIP implementation.
 *
 * Equation numbers follow the order of the displayed equations of the paper
 * (Eq. (36) is the energy-momentum moment condition, Eq. (57) the full
 * extended update, Eq. (58) the density equilibrium).
 *
 * Parity status of each function is stated in its comment in rlb_oracle.c.
 */
#ifndef RLB_ORACLE_H
#define RLB_ORACLE_H

#include <stdint.h>

#define ORC_Q 19

enum { ORC_BC_PERIODIC = 0, ORC_BC_FIXED = 1, ORC_BC_OUTFLOW = 2 };
enum { ORC_TAU_UNIFORM = 0, ORC_TAU_ETA_OVER_S = 1 };

typedef struct {
  int nx, ny, nz;
  double nu;          /* nu = c / c_s, Sec. II                                  */
  double dt;          /* delta t / delta x (delta x = 1)                        */
  int euler;          /* 1: collision replaced by f := f^eq (Sec. III)           */
  int tau_mode;       /* ORC_TAU_UNIFORM | ORC_TAU_ETA_OVER_S                   */
  double tau;         /* relaxation time when tau_mode == UNIFORM               */
  double eta_over_s;  /* eta/s when tau_mode == ETA_OVER_S                      */
  double alpha;       /* bulk-viscosity constant alpha, Eq. (55)                */
  int with_h;         /* carry the density distribution h_i, Eq. (58)           */
  int bc[6];          /* -x,+x,-y,+y,-z,+z                                      */
  double face[6][5];  /* (eps,ux,uy,uz,n) of FIXED faces                        */
  double guard_umax;  /* admissibility guard; 0 = off                           */
  double guard_efloor;/* energy floor used by the guard                        */
  int basic;          /* 1: the basic model of Sec. II (standard D3Q19, exact
                         streaming with dt = c_t dx/(c_a c_0), explicit Marle
                         collision, no bulk term, no limiter, f only); euler,
                         alpha, with_h and the guard must be off; dt unused   */
  int dens_w;         /* density weights w'_i of Eq. (58): ORC_DENSW_PAPER
                         (Eqs. (59)-(60)) or ORC_DENSW_ISOTROPIC (beyond the
                         paper, see make_lattice); extended set only          */
  int flux;           /* streaming flux: ORC_FLUX_MINMOD (Eqs. (47)-(53)) or
                         ORC_FLUX_RUSANOV (beyond the paper, see div_flux);
                         extended set only                                    */
} orc_config;

enum { ORC_DENSW_PAPER = 0, ORC_DENSW_ISOTROPIC = 1 };
enum { ORC_FLUX_MINMOD = 0, ORC_FLUX_RUSANOV = 1 };

typedef struct orc_state orc_state;

/* Lattice (basic = 0: the extended set of Sec. II.A, Eq. (42); basic = 1: the
   basic D3Q19 set of Sec. II): velocity e_i (integer, 3 per pop), 4-vector
   xi_i = (c_t/c_0, c_a e_i), weights w_i and density weights w'_i. */
void orc_lattice(double nu, int basic, int dens_w, int* e /*19x3*/, double* xi /*19x4*/,
                 double* w /*19*/, double* wp /*19*/);

/* Discrete equilibria (reading M of Eq. (29) fixed by Eq. (36)) and Eq. (58). */
void orc_feq(double nu, int basic, double eps, double ux, double uy, double uz, double* feq);
void orc_heq(double nu, int basic, int dens_w, double n, double ux, double uy, double uz,
             double* heq);

/* Moments T^{00}, T^{0a} of f and N^0 of h; fields (eps,ux,uy,uz,n) from them.
   Returns 0 if admissible, -1 if not (fields then hold NaN). */
void orc_moments(double nu, int basic, const double* f, const double* h /*nullable*/,
                 double* T0 /*4: T^00,T^0x,T^0y,T^0z*/, double* N0);
int orc_recover(double T00, double T0x, double T0y, double T0z, double N0,
                int with_h, double* fields /*5*/);

/* Whole-domain time stepper. */
orc_state* orc_create(const orc_config* cfg);
void orc_destroy(orc_state* S);
int orc_init(orc_state* S, const double* eps, const double* ux,
             const double* uy, const double* uz, const double* n /*nullable*/,
             const uint8_t* obstacle /*nullable*/);
/* Advance nsteps; returns 0, or (1 + index of the first step whose recovery
   met an inadmissible or non-finite state). */
int64_t orc_step(orc_state* S, int64_t nsteps);
void orc_fields(const orc_state* S, double* eps, double* ux, double* uy,
                double* uz, double* n /*nullable*/);
/* Populations in the oracle's own order (orc_lattice), layout [i][cell]. */
void orc_get_pops(const orc_state* S, double* f, double* h /*nullable*/);
void orc_set_pops(orc_state* S, const double* f, const double* h /*nullable*/,
                  const double* hist /*5 x cells, nullable*/);
void orc_get_hist(const orc_state* S, double* hist /*5 x cells*/);
int64_t orc_guard_events(const orc_state* S);
int orc_num_threads(void);
void orc_set_num_threads(int n);

#endif
