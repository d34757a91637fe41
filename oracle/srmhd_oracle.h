/*
 * srmhd_oracle.h -- plain FP64 CPU oracle for 3D ideal special-relativistic
 * MHD in flat space (Cartesian, periodic box), one SSP-RK3 step at a time.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path; it is
 * loaded by the test suite, by the package's smoke check and by the CPU
 * baseline leg of the benchmark, never by the product path.  It shares no
 * code with the HIP library.
 *
 * Paper: Del Zanna, Landi, Serafini, Bugli, Papini, "A GPU-Accelerated Modern
 * Fortran Version of the ECHO Code for Relativistic Magnetohydrodynamics",
 * Fluids 2024 (arXiv 2401.03008).  Equations: Sec. 2 (ideal SRMHD system and
 * definitions of D, S, U, W_ij, p_tot, ideal-gas h), Sec. 3 (semi-discrete
 * point-value scheme, staggered B, the five steps of a Runge-Kutta substep,
 * the global max of the characteristic speeds).  The paper names MP5, upwind
 * (HLL/LLF) fluxes, UCT and a Newton inversion but prints none of their
 * formulas; the readings used here are listed in the source.
 *
 * Layout: every grid array is nx*ny*nz doubles, x fastest:
 *   a[(k*ny + j)*nx + i].
 * Primitive vectors: {rho, vx, vy, vz, p, Bx, By, Bz}.
 * Conserved vectors: {D, Sx, Sy, Sz, U, Bx, By, Bz}.
 * Face field bf[0][i,j,k] is B_x at x_{i+1/2}; bf[1] is B_y at y_{j+1/2};
 * bf[2] is B_z at z_{k+1/2}.  Edge field E[0][i,j,k] is E_x at
 * (x_i, y_{j+1/2}, z_{k+1/2}); E[1] is E_y at (x_{i+1/2}, y_j, z_{k+1/2});
 * E[2] is E_z at (x_{i+1/2}, y_{j+1/2}, z_k).
 */
#ifndef SRMHD_ORACLE_H
#define SRMHD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int nx, ny, nz;
  double lx, ly, lz;
  double gam;      /* adiabatic index */
  double cfl;      /* Courant number for the sum-over-directions rule */
  double dt_fixed; /* > 0: use this dt instead of the CFL rule */
  int riemann;     /* 0 = HLL, 1 = LLF */
  int maxit;       /* Newton iteration cap */
  double tol;      /* Newton relative step tolerance on W */
  double pfloor;   /* pressure floor as a fraction of rho (0 = none) */
  int recon;       /* 0 = MP5, 1 = linear with the MC limiter */
  int time_order;  /* 3 = SSP-RK3, 2 = SSP-RK2 */
  int ho;          /* 1 = high-order INT and DER (sixth-order central forms) */
} orc_cfg;

typedef struct {
  long newton_iters;     /* sum of Newton iterations over all inversions */
  long newton_hist[32];  /* histogram of iteration counts (last bin = >=31) */
  long c2p_fail;         /* inversions that did not converge */
  long recon_fallbacks;  /* face states replaced by first-order values */
  long floors;           /* pressure floors applied */
} orc_stats;

/* ---- point physics ---- */
void orc_prim2cons(double gam, const double *pr, double *u);
void orc_flux(double gam, const double *pr, int d, double *f);
void orc_speeds(double gam, const double *pr, int d, double *lm, double *lp);
int orc_con2prim(double gam, const double *u, double *W, int maxit, double tol,
                 double pfloor, double *pr, int *iters, int *floored);
double orc_mp5(const double *s);
double orc_mp5_point(const double *s);
double orc_mc(const double *s);
double orc_int_ho(const double *b);
double orc_der_ho(const double *f);
void orc_riemann(int kind, double gam, const double *prL, const double *prR,
                 int d, double *fhat, double *ap, double *am);
double orc_uct_formula(const double *Eab, double axp, double axm, double ayp,
                       double aym, double byL, double byR, double bxL,
                       double bxR);

/* ---- grid operations ---- */
int orc_init(const orc_cfg *c, double *const *prim5, double *const *bf,
             double **cons, double *W);
int orc_c2p(const orc_cfg *c, double *const *cons, double *const *bf,
            double *W, double **prim, int *iters, orc_stats *st);
int orc_rhs(const orc_cfg *c, double *const *prim, double *const *bf,
            double **rhs, double *amax, double **fhat, double **apm,
            double **face_v, double **edge_e, orc_stats *st);
int orc_rhs_cells(const orc_cfg *c, double *const *prim, double *const *bf, int ncells,
                  const long *cells, double *out);
int orc_step(const orc_cfg *c, double **cons, double **bf, double *W,
             int nsteps, double *t, double *dt_last, orc_stats *st);
double orc_divb_max(const orc_cfg *c, double *const *bf);
int orc_num_threads(void);
void orc_set_num_threads(int n);
void orc_sums(const orc_cfg *c, double *const *cons, double *const *bf,
              double *sums);

#ifdef __cplusplus
}
#endif
#endif
