/*
 * dbm.h -- C ABI of libdbm: the per-time-step update of the multi-component
 * D2V16 discrete Boltzmann model (Lin, Luo, Fei and Succi, "A multi-component
 * discrete Boltzmann model for nonequilibrium reactive flows",
 * arXiv:2006.15932) on AMD Instinct MI355X (gfx950).
 *
 * One step advances every species' 16 discrete distributions f_i^s on a 2-D
 * grid (Eq.3): NND upwind convection, per-cell moments, f^eq = M^{-1} fhat
 * (Eq.16) with M inverted once on the host in FP64, BGK collision (Eq.4) plus
 * reaction (Eq.5) and force (Eq.6) sources, and the Runge-Kutta stage combine
 * (forward Euler, the paper's scheme, or third-order TVD Runge-Kutta).
 *
 * Conventions shared by every entry point
 *  - Return value: DBM_OK (0) or a negative DBM_ERR_* code; nothing throws or
 *    aborts across the ABI.  dbm_last_error() gives a thread-local message.
 *  - Host arrays are owned by the caller, always FP64, row-major with x
 *    fastest: species fields [S][ny][nx], scalar fields [ny][nx], the
 *    distribution [S][16][ny][nx].  Conversion to the storage precision
 *    happens inside the library.
 *  - Device memory: the caller allocates one workspace of
 *    dbm_workspace_bytes() bytes (for example a torch uint8 tensor on the
 *    GPU) and keeps it alive until dbm_destroy().  The library allocates no
 *    device memory of its own; the handle owns only host tables, HIP events
 *    and the captured HIP graphs.
 *  - Streams: all device work is ordered on the hip_stream given to
 *    dbm_create (NULL = the legacy default stream).  dbm_step is
 *    asynchronous; every entry point that returns data to the host
 *    synchronises the stream first.  Kernel failures surface at the next
 *    synchronising call as DBM_ERR_HIP.
 *  - Velocity ordering of the 16 planes of one species (Eq.15): group a
 *    (i=0..3) = v_a*{(1,0),(0,1),(-1,0),(0,-1)}, group b (4..7) =
 *    v_b*{(1,1),(-1,1),(-1,-1),(1,-1)}, group c (8..11) like a with v_c,
 *    group d (12..15) like b with v_d; eta_g is shared within group g.
 */
#ifndef DBM_H
#define DBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DBM_OK = 0,
  DBM_ERR_ARG = -1,          /* invalid argument or configuration            */
  DBM_ERR_SINGULAR_M = -2,   /* moment matrix rank < 16 or cond_1 > 1e12     */
  DBM_ERR_HIP = -3,          /* HIP runtime failure (message kept)           */
  DBM_ERR_NONFINITE = -4,    /* NaN/Inf or negative density found by check   */
  DBM_ERR_UNSUPPORTED = -5,  /* valid but not supported (see each call)      */
  DBM_ERR_WORKSPACE = -6     /* workspace missing, misaligned or too small   */
};

/* Storage and bulk arithmetic of f: FP64; FP32-bulk (FP32 storage and bulk
 * arithmetic, FP64 moments/T and conserved rows); FP32X (each value stored as
 * FP32 plus the bfloat16 rounding of its remainder, about 32 significant bits
 * in 6 bytes, with FP64 arithmetic). */
enum { DBM_FP64 = 0, DBM_FP32_BULK = 1, DBM_FP32X = 2 };
enum { DBM_EULER = 0, DBM_TVD_RK3 = 1 };         /* time scheme               */
enum { DBM_LIM_MINMOD = 0, DBM_LIM_NONE = 1 };   /* NND limiter or unlimited  */
enum { DBM_BC_PERIODIC = 0, DBM_BC_OUTFLOW = 1, DBM_BC_WALL = 2 };
enum { DBM_FORCE_T_EXACT = 0, DBM_FORCE_T_SAME = 1 };

/* One species (Eq.7 and Eq.15): molar mass m, extra degrees of freedom I,
 * relaxation time tau (Eq.4), stoichiometric coefficient a (Eq.1, negative
 * for reactants), speeds v[g] and internal-energy parameters eta[g] of the
 * four velocity groups g = a, b, c, d. */
typedef struct {
  double m, I, tau, a_stoich;
  double v[4];
  double eta[4];
} dbm_species;

/* One-step overall reaction of Eqs.(1)-(2): rate omega = k_ov n^F n^O
 * exp(-Ea_over_R / T); extent xi = omega*tau within the relaxation time;
 * Q = heat released per unit extent.  k_ov == 0 disables the source. */
typedef struct {
  int fuel, oxidiser;
  double k_ov, Ea_over_R, Q;
} dbm_reaction;

/* One step of a multi-step mechanism (the text after Eqs.(1)-(2) allows
 * detailed or reduced multi-step kinetics): the rate law of Eq.(2) with its
 * own reactant pair and constants, heat Q per unit extent, and its own
 * stoichiometric coefficients a[s] (< 0 reactant, > 0 product) for species
 * 0 .. nspecies-1 (entries beyond nspecies are ignored).  fuel and oxidiser
 * may be the same species (rate k n^2 exp(-Ea/RT)).  With several steps,
 * n^s* = n^s + sum_r a_r^s xi_r, xi_r = omega_r tau, and one common factor
 * scales every xi_r when a reactant would otherwise be overdrawn. */
#define DBM_MAX_REACTION_STEPS 4
typedef struct {
  int fuel, oxidiser;
  double k_ov, Ea_over_R, Q;
  double a[16];
} dbm_reaction_step;

/* One simulation instance. */
typedef struct {
  int nx, ny;                    /* grid size, >= 1                           */
  double dx, dy, dt;             /* spacings and time step, > 0               */
  int bc_x, bc_y;                /* DBM_BC_*; walls are specular              */
  int nspecies;                  /* 1 .. 16                                   */
  const dbm_species *species;    /* nspecies entries                          */
  const dbm_reaction *reaction;  /* NULL = no chemistry                       */
  double accel[2];               /* external acceleration a (Eq.6)            */
  int precision;                 /* DBM_FP64 | DBM_FP32_BULK | DBM_FP32X      */
  int time_scheme;               /* DBM_EULER | DBM_TVD_RK3                   */
  int limiter;                   /* DBM_LIM_MINMOD | DBM_LIM_NONE             */
  int force_T_mode;              /* temperature T_dagger of Eq.(6)            */
  int nchem;                     /* 0 .. DBM_MAX_REACTION_STEPS; > 0: the     */
  const dbm_reaction_step *chem; /* mechanism replaces `reaction` and the    */
                                 /* species' a_stoich                         */
} dbm_config;

typedef struct dbm_s *dbm_handle;

/* Bytes of device workspace needed by ninst instances (0 on invalid input).
 * Pure host computation; no GPU needed. */
size_t dbm_workspace_bytes(const dbm_config *cfgs, int ninst);

/* Validate the configurations, build per-species tables (velocity set of
 * Eq.15, moment matrix rows listed after Eq.14 with row 9 = (v^2+eta^2) v_y,
 * its FP64 inverse and the symmetry blocks derived from it), upload them into
 * dev_workspace and return a handle.  ninst > 1 makes a batched handle: every
 * instance must share nspecies, precision, time_scheme and limiter; each
 * dbm_step advances all of them with one launch per stage.
 * Errors: DBM_ERR_ARG (bad sizes, indices, non-positive m, tau, dt, dx, dy,
 * negative I), DBM_ERR_SINGULAR_M, DBM_ERR_UNSUPPORTED (reaction with unequal
 * tau across species, or mixed template parameters in a batch),
 * DBM_ERR_WORKSPACE (NULL, unaligned to 256 bytes, or ws_bytes too small),
 * DBM_ERR_HIP.
 * Path: the one-pass stage kernels serve nspecies <= 4 with periodic or
 * outflow x boundaries and under 4 GiB per species and buffer (16 planes in
 * the storage type, FP32 part for FP32X); any other configuration runs the
 * plain kernels (DBM_OPT_PATH reads 1), with the same results to rounding. */
int dbm_create(const dbm_config *cfgs, int ninst, void *hip_stream, void *dev_workspace,
               size_t ws_bytes, dbm_handle *out);

/* Release host resources (graphs, events).  The workspace stays the caller's. */
int dbm_destroy(dbm_handle h);

/* f := f^eq(n^s, u, T) in every cell of instance inst (Eq.16).
 * n_sp [S][ny][nx] molar concentrations, ux, uy, T [ny][nx]. */
int dbm_set_fields(dbm_handle h, int inst, const double *n_sp, const double *ux,
                   const double *uy, const double *T);

/* Write / read the distribution [S][16][ny][nx] (FP64 host arrays), rounded
 * to / widened from the storage precision.  With OM storage (FP32-bulk, see
 * DBM_OPT_STORAGE) dbm_set_f also sets the storage reference from f (the least
 * density of each species and the least temperature) and stores f in that
 * representation; a get/set round trip then agrees to FP32 rounding of the
 * stored values, not always bit for bit: bit-exact checkpoints use
 * dbm_save_state / dbm_load_state. */
int dbm_set_f(dbm_handle h, int inst, const double *f);
int dbm_get_f(dbm_handle h, int inst, double *f);

/* Checkpoint and restart, bit for bit: the state of instance inst (its
 * distribution exactly as stored, the reference of OM storage and the step
 * counter of stochastic rounding) as an opaque host blob of
 * dbm_state_bytes() bytes (0 on a bad handle or index).  dbm_load_state
 * accepts only a blob saved by a handle of the same precision, storage
 * representation (DBM_OPT_STORAGE), species count and grid size
 * (DBM_ERR_ARG otherwise); the caller owns both host buffers.  Synchronise. */
size_t dbm_state_bytes(dbm_handle h, int inst);
int dbm_save_state(dbm_handle h, int inst, void *dst, size_t bytes);
int dbm_load_state(dbm_handle h, int inst, const void *src, size_t bytes);

/* Advance every instance by nsteps time steps of the discrete Boltzmann
 * equation, Eq.(3): the right-hand side is the NND upwind convection -v.grad f
 * plus the collision, reaction and force terms of Eqs.(4)-(6), and the time
 * discretisation is forward Euler (the scheme of the paper's simulation
 * section, with NND in space) or third-order TVD Runge-Kutta, per
 * dbm_config.time_scheme.  Asynchronous on the stream unless the non-finite
 * check is enabled (then DBM_ERR_NONFINITE may be returned after a
 * synchronisation).  nsteps < 0: DBM_ERR_ARG; nsteps == 0 does nothing. */
int dbm_step(dbm_handle h, int nsteps);

/* Macroscopic fields of instance inst, from the moments of f that the
 * collision conserves (the statement under Eq.(6), with the kinetic moments of
 * Eqs.(8)-(10)): rho^s = m^s n^s with n^s = sum_i f_i^s [S][ny][nx]; the
 * mixture velocity u = sum_s m^s sum_i f_i^s v_i / rho and temperature
 * T = (sum_s m^s sum_i f_i^s (v_i^2 + eta_i^2) - rho u^2) / sum_s (D + I^s) n^s
 * [ny][nx] (any pointer may be NULL).  Synchronises. */
int dbm_moments(dbm_handle h, int inst, double *rho_sp, double *ux, double *uy, double *T);

/* Nonequilibrium measures of Eqs.(17)-(20), taken against f^eq(n^s, u, T):
 * delta [S][12][ny][nx] in the order Delta_2 xx, xy, yy; Delta_3,1 x, y;
 * Delta_3 xxx, xxy, xyy, yyy; Delta_4,2 xx, xy, yy (may be NULL), and FP64
 * domain totals [S+3] = mass^s, momentum x, y, energy (times dx dy), reduced
 * in a fixed order (may be NULL).  Synchronises. */
int dbm_noneq_moments(dbm_handle h, int inst, double *delta, double *totals);

/* For callers that cannot allocate device memory or touch a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the FP64 domain totals of dbm_noneq_moments ([S+3] = mass^s,
 * momentum x, y, energy, times dx dy; same kernels, same fixed reduction
 * order, same values) with the per-workgroup partial sums kept in a fixed
 * 80 KiB array of the library's own device memory, one per GPU, held until
 * the process ends, instead of the handle's workspace.  Allocates nothing.
 * All calls on one GPU share that array (each call rewrites what it reads):
 * calls that overlap in time on one GPU, from other host threads or
 * streams, race.  DBM_ERR_ARG if the partial sums would exceed the array
 * (they cannot for nspecies <= 16) or totals is NULL.  Synchronises. */
int dbm_noneq_totals_noalloc(dbm_handle h, int inst, double *totals);

/* Translational energies and energy fluxes defined with the nonequilibrium
 * measures (the paragraph after Eqs.(21)-(23)), per species, with
 * M2aa(g) = m sum_i g_i v_ia^2 and M31a(g) = m sum_i g_i (v_i^2 + eta_i^2) v_ia
 * and f^eq = f^eq(n^s, u, T): fields [S][8][ny][nx] in the order
 *   1/2 M2xx(f), 1/2 M2yy(f)        translational energy in x, y
 *   1/2 M2xx(f^eq), 1/2 M2yy(f^eq)  its equilibrium part
 *   1/2 M31x(f), 1/2 M31y(f)        total energy flux in x, y
 *   1/2 M31x(f^eq), 1/2 M31y(f^eq)  organised energy flux
 * (the nonorganised energy and flux are the differences, i.e. 1/2 Delta_2aa
 * and 1/2 Delta_3,1a), and FP64 domain totals [S][8] (times dx dy, reduced in
 * a fixed order).  Either pointer may be NULL.  Synchronises. */
int dbm_energy_moments(dbm_handle h, int inst, double *fields, double *totals);

/* Options (dbm_set_option / dbm_get_option). */
enum {
  DBM_OPT_PATH = 1,         /* 0 fused one-pass kernels (default), 1 plain    */
  DBM_OPT_GRAPH = 2,        /* 1 replay captured HIP graphs (default), 0 eager */
  DBM_OPT_TILE_ROWS = 3,    /* rows marched per wavefront; 0 = autotune        */
  DBM_OPT_CHECK_EVERY = 4,  /* non-finite check every K steps; 0 = off         */
  DBM_OPT_BATCH_MODE = 5,   /* 0 one launch per stage for all instances,
                               1 one launch per instance (comparison mode)     */
  DBM_OPT_GRAPH_CHUNK = 6,  /* steps captured per graph (default 256)         */
  DBM_OPT_PERSISTENT = 7,   /* read only: resident workgroups of a launch      */
  DBM_OPT_SPLIT = 8,        /* form of the one-pass kernel: 0 default (= 1),
                               1 one wavefront per species, 2 two wavefronts
                               per species, each holding 8 of the 16 planes;
                               get: 1 or 2 in use */
  DBM_OPT_PIPELINE = 9,     /* FP32 full form: row k+1's collision formed
                               while row k's stencils are; 0 tuned with the
                               tile rows (default; off when the rows are set),
                               1 off, 2 on; get: 1 or 2 in use */
  DBM_OPT_ROUNDING = 10,    /* FP32-bulk stores of f: 0 round to nearest
                               (default), 1 stochastic rounding (unbiased:
                               up or down with probabilities in proportion to
                               the distances, 8 random bits per value hashed
                               from the cell, species and state, so runs are
                               deterministic); DBM_ERR_UNSUPPORTED for other
                               precisions and with the split form */
  DBM_OPT_STORAGE = 12,     /* FP32-bulk representation of f in the buffers:
                               0 (default) OM storage wherever the one-pass
                               path runs its full form without the row
                               pipeline: per cell and species the A-block
                               moments (n, E and two more) of f - fref and
                               the orbit components B, X, Y of f, fref an
                               equilibrium at rest with the row means of
                               n^s and T per grid row (the grid means for
                               every row unless some row mean differs from
                               them by more than 1e-3 of them), fixed when
                               the fields or f are set; 1 the 16
                               values f_i themselves; 2 OM storage where
                               0 would use it, each A-block value also
                               keeping the rounding remainder of its FP32
                               value as a bfloat16 (8 more bytes per cell
                               and species, summed in FP64 at each store:
                               mass and energy to about 33 bits; round to
                               nearest only, DBM_ERR_UNSUPPORTED with
                               stochastic rounding).
                               0 and 1 keep 16 FP32 values per cell and
                               species; OM storage rounds mass and energy
                               relative to their deviation from fref and
                               momentum relative to itself.  Setting it (or
                               an option that excludes OM storage) converts
                               the state in place; get: 0 OM storage in
                               use, 1 f, 2 OM storage with A-block
                               residuals */
  DBM_OPT_DRAIN = 13,       /* one-pass kernel on OM storage, Euler stages
                               (RK3 stages keep one form of their own):
                               every other row waits for the loads of its
                               refill (the row three ahead) at once, which
                               halves the loads in flight; 0 tuned with the
                               tile rows (default; on when the rows are
                               set), 1 off (the refills stay in flight), 2
                               on; get: 1 or 2 in use.  Results are the same
                               bits either way */
  DBM_OPT_CHAIN_WAVE = 11   /* one-pass path, nspecies <= 3: one more wavefront
                               per workgroup forms each row's mixture chain
                               (u, T, reaction) while the species' wavefronts
                               form their stencils; 0 tuned with the tile rows
                               (default), 1 off, 2 on; excludes the split
                               form and the row pipeline
                               (DBM_ERR_UNSUPPORTED); get: 1 or 2 in use */
};
int dbm_set_option(dbm_handle h, int option, int value);
int dbm_get_option(dbm_handle h, int option, int *value);

/* Time the dominant kernel (one stage of the fused or plain path) with HIP
 * events recorded on the handle's stream around each of reps eager launches
 * that write only a spare buffer; returns the mean duration in milliseconds.
 * The simulation state is not changed.  Synchronises. */
int dbm_time_stage_kernel(dbm_handle h, int reps, double *ms_per_launch);

/* Measurement reference, not part of the method: copies `bytes` (a multiple
 * of 16, both pointers device memory aligned to 16 bytes, not overlapping)
 * from src to dst with a grid-stride streaming copy of 16-byte words (each
 * thread keeping `words` = 1, 2, 4 or 8 of them in flight per iteration,
 * non-temporal stores) on `grid` workgroups of 256 threads, `reps` times
 * after one warm-up copy, on hip_stream (NULL = default stream), and returns
 * the mean duration of one copy in milliseconds from HIP events.  The
 * achievable HBM rate is then 2 bytes / time.  Synchronises; DBM_ERR_ARG on
 * bad arguments. */
int dbm_copy_rate(const void *src, void *dst, size_t bytes, int grid, int words, int reps,
                  void *hip_stream, double *ms_per_copy);

/* Thread-local description of the last error. */
const char *dbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
