/*
 * dbm_oracle.h -- plain FP64 CPU oracle of the multi-component D2V16 discrete
 * Boltzmann model (Lin, Luo, Fei, Succi, "A multi-component discrete Boltzmann
 * model for nonequilibrium reactive flows", arXiv:2006.15932).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.  Only
 * the test suite, the package smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no source, header, table or helper with the GPU library.
 *
 * Layout of every field array: row-major, x fastest.
 *   f      : [S][16][ny][nx]
 *   scalar : [ny][nx]
 *   species: [S][ny][nx]
 */
#ifndef DBM_ORACLE_H
#define DBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define OR_NV 16        /* discrete velocities per species (D2V16) */
#define OR_MAXS 16      /* species limit of the oracle */

enum { OR_BC_PERIODIC = 0, OR_BC_OUTFLOW = 1, OR_BC_WALL = 2 };
enum { OR_EULER = 0, OR_RK3 = 1 };
enum { OR_LIM_MINMOD = 0, OR_LIM_NONE = 1 };
enum { OR_FORCE_T_EXACT = 0, OR_FORCE_T_SAME = 1 };

typedef struct {
  double m;        /* molar mass m^sigma                                   */
  double I;        /* extra degrees of freedom I^sigma                      */
  double tau;      /* relaxation time tau^sigma                             */
  double a;        /* stoichiometric coefficient a^sigma (<0 reactant)      */
  double v[4];     /* v_a, v_b, v_c, v_d                                    */
  double eta[4];   /* eta_a, eta_b, eta_c, eta_d                            */
} or_species;

/* One step of a multi-step mechanism: rate k n^fuel n^oxid exp(-Ea_over_R/T)
 * (Eq.2 per step), heat Q per unit extent, stoichiometric coefficients a[s]. */
#define OR_MAXR 4
typedef struct {
  int fuel, oxid;
  double k, Ea_over_R, Q;
  double a[OR_MAXS];
} or_reaction_step;

typedef struct {
  int nx, ny;
  double dx, dy, dt;
  int bc_x, bc_y;
  int S;
  const or_species *sp;
  int reaction_on;           /* 0: no chemistry                                 */
  int fuel, oxid;            /* species indices of the two reactants            */
  double k_ov, Ea_over_R, Q; /* rate constant, activation temperature, heat     */
  double ax, ay;             /* external acceleration                           */
  int scheme;                /* OR_EULER | OR_RK3                               */
  int limiter;               /* OR_LIM_MINMOD (NND) | OR_LIM_NONE               */
  int force_T_mode;          /* OR_FORCE_T_EXACT | OR_FORCE_T_SAME              */
  int nchem;                 /* > 0: these steps replace the one-step reaction */
  const or_reaction_step *chem;
} or_config;

typedef struct or_model or_model;

/* Validate the configuration and build every per-species table.
 * Returns 0, or -1 bad argument, -2 singular moment matrix, -5 unsupported. */
int or_create(const or_config *cfg, or_model **out);
void or_destroy(or_model *md);

/* Number of OpenMP threads used by the field loops (1 = serial). */
void or_set_threads(int n);
int or_get_threads(void);

/* Per-species tables: velocities (16 each), moment matrix M and its inverse
 * (16x16 row-major, M[r*16+i]). */
int or_tables(const or_model *md, int s, double *vx, double *vy, double *eta,
              double *M, double *Minv);

/* Equilibrium moments fhat (16) of the closed forms after Eq.(14). */
void or_fhat(double n, double ux, double uy, double theta, double I, double *h);

/* Discrete equilibrium f^eq = M^{-1} fhat of species s, Eq.(16). */
int or_feq(const or_model *md, int s, double n, double ux, double uy, double T,
           double *feq);

/* Collision + reaction + force source of one cell: fc[S*16] -> src[S*16]. */
int or_cell_source(const or_model *md, const double *fc, double *src);

/* f := f^eq(n^sigma, u, T) in every cell. */
int or_init_equilibrium(const or_model *md, const double *n_sp, const double *ux,
                        const double *uy, const double *T, double *f);

/* Right-hand side of Eq.(3): L = -v.grad f + Omega + R + G. */
int or_rhs(const or_model *md, const double *f, double *L);

/* Advance f in place by nsteps time steps. */
int or_run(const or_model *md, double *f, int nsteps);

/* Macroscopic fields: rho^sigma [S][ny][nx], mixture ux, uy, T. */
int or_moments(const or_model *md, const double *f, double *rho_sp, double *ux,
               double *uy, double *T);

/* Nonequilibrium measures of Eqs.(17)-(20) (12 per species per cell, may be
 * NULL) and domain totals [S+3] = mass^sigma, Px, Py, E. */
int or_noneq(const or_model *md, const double *f, double *delta, double *totals);

/* Translational energies and energy fluxes defined after Eqs.(21)-(23), per
 * species and cell (8 per species, may be NULL): 1/2 m sum f v_x^2,
 * 1/2 m sum f v_y^2, the same over f^eq(n^s, u, T), 1/2 m sum f q v_x,
 * 1/2 m sum f q v_y, the same over f^eq (q = v^2 + eta^2); totals [S][8] are
 * their domain integrals (may be NULL). */
int or_energy(const or_model *md, const double *f, double *fields, double *totals);

#ifdef __cplusplus
}
#endif
#endif
