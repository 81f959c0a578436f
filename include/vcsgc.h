/*
 * vcsgc.h -- C ABI of the MI355X (gfx950) implementation of parallel
 * variance-constrained semi-grandcanonical (VC-SGC) transmutation Monte Carlo
 * with an embedded-atom (EAM) potential, interleaved with velocity-Verlet MD
 * (Sadigh, Erhart, Stukowski, Caro, Martinez, Zepeda-Ruiz, "A scalable parallel
 * Monte Carlo algorithm for atomistic simulations of precipitation in alloys").
 *
 * Conventions
 *  - Every call except vcsgc_last_error returns a vcsgc_status (0 = OK, < 0 =
 *    error).  No exception crosses the ABI.  On an argument error nothing is
 *    modified.  A device error is sticky: later calls on the context return
 *    VCSGC_E_STATE; vcsgc_last_error gives the message.
 *  - Pointers in vcsgc_system are DEVICE pointers owned by the caller.  They
 *    are borrowed for the lifetime of the context and must not be written by
 *    the caller while a call is in flight.  Library scratch (cells, neighbour
 *    lists, density cache, stage records, counters) is owned by the context
 *    and released by vcsgc_destroy.
 *  - All work is ordered on the stream given at creation and is asynchronous,
 *    except calls that return host values (statistics, energies, counts),
 *    which synchronize that stream.
 *  - Species: 0 = A, 1 = B ("spin 1" of Sec. II; c = n_B / N).  Positions are
 *    Cartesian in an orthorhombic periodic box and must lie in [0, L).
 *  - Units: Angstrom, eV, fs, atomic mass units, K.
 */
#ifndef VCSGC_H
#define VCSGC_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vcsgc_ctx vcsgc_ctx; /* opaque, library-owned */
typedef struct vcsgc_mlp vcsgc_mlp; /* opaque surrogate network, library-owned */

/* vcsgc_system.flags */
#define VCSGC_FLAG_DESCRIPTOR 1u /* keep the r < 4.41 A descriptor list (surrogate, sample log) */
/* A finer colouring than the eight octants of Sec. III.A: cells of edge
 * >= r_dep / 2, a multiple of three per dimension, coloured by their indices
 * modulo 3 (27 colours); same-colour cells are two cell edges, >= r_dep,
 * apart, so their trials stay independent.  A stage draws its colour as
 * floor(w0 27 / 2^64) from its Philox word (eight colours: w0 >> 61), and a
 * sweep has 27 ceil(N / N_cells) stages, each with about 2.4 times the
 * trials of an eight-colour stage. */
#define VCSGC_FLAG_COLOURS27 2u

typedef enum {
  VCSGC_OK = 0,
  VCSGC_E_INVALID_ARG = -1,
  VCSGC_E_BOX_TOO_SMALL = -2,
  VCSGC_E_OUT_OF_MEMORY = -3,
  VCSGC_E_DEVICE = -4,
  VCSGC_E_STATE = -5,
  VCSGC_E_NO_SURROGATE = -6,
  VCSGC_E_BARRIER_TIMEOUT = -7, /* a bounded wait of the persistent sweep timed out (sticky) */
  VCSGC_E_OVERFLOW = -8
} vcsgc_status;

/* Analytic Finnis-Sinclair EAM (zero for r >= rc):
 *   pair      phi_XY(r) = eps_XY (rc - r)^2 (c0 + c1 r)
 *   density   f_X(r)    = t_X (rc - r)^2
 *   embedding F_X(rho)  = -A_X sqrt(rho)
 * mass_a / mass_b are the species masses for MD (u). */
typedef struct {
  double rc, c0, c1, eps_aa, eps_ab, eps_bb, t_a, t_b, a_a, a_b, mass_a, mass_b;
} vcsgc_eam_fs;

/* A tabulated two-species EAM (a general embedded-atom potential, the
 * class of short-range potentials named in the Introduction and Sec. III;
 * published EAM potentials are commonly distributed as such tables):
 * f_A, f_B and phi_AA, phi_AB, phi_BB at the radial knots r_k = k dr
 * (k = 0 .. nr-1), F_A and F_B at the density knots rho_k = k drho
 * (k = 0 .. nrho-1).  Each function is interpolated by the cubic Hermite
 * interpolant whose knot slopes are central differences (one-sided at the
 * two ends): on interval k, with t = x/h - k,
 *   p(t) = ((a3 t + a2) t + a1) t + a0,  a0 = y_k,  a1 = m_k,
 *   a2 = (3 d - 2 m_k) - m_{k+1},  a3 = (m_k + m_{k+1}) - 2 d,
 *   d = y_{k+1} - y_k,  m_k = (y_{k+1} - y_{k-1}) / 2,
 * with k = floor(x/h) limited to [0, n-2] (outside the knots the end
 * interval's cubic continues) and x/h formed as x times the rounded 1/h;
 * derivatives are p'(t) / h.  f and phi are zero for r >= rc.  The arrays
 * are host memory, read during vcsgc_create. */
typedef struct {
  int32_t nr, nrho;   /* knots, >= 2 each */
  double dr, drho;    /* knot spacings, > 0 */
  double rc;          /* cutoff, > 0, at most (nr - 1) dr */
  const double *f[2];    /* f_A, f_B: nr values each */
  const double *phi[3];  /* phi_AA, phi_AB, phi_BB: nr values each */
  const double *F[2];    /* F_A, F_B: nrho values each */
} vcsgc_eam_table;

typedef struct {
  int64_t n_atoms;  /* N >= 2 */
  double box[3];    /* orthorhombic periodic box edges, Angstrom */
  double *x, *y, *z;    /* positions in [0, L), device, N each */
  double *vx, *vy, *vz; /* velocities (A/fs), device; NULL => MC-only context */
  double *fx, *fy, *fz; /* forces (eV/A), device; NULL allowed for MC-only */
  uint8_t *species;     /* device, N entries in {0, 1} */
  vcsgc_eam_fs pot;
  double skin;   /* MD neighbour-list skin (A), >= 0; typical 0.3 */
  double r_dep;  /* independence distance for the cell colouring; 0 => 2 rc */
  uint32_t flags;        /* VCSGC_FLAG_* */
  /* NULL: the analytic potential pot; else the tabulated potential (then
   * pot supplies only mass_a and mass_b, and rc is table->rc) */
  const vcsgc_eam_table *table;
  /* > 0: grown domains (Sec. III.A, Fig. 6) instead of the colouring:
   * cells of edge e >= max(grow_edge, 2 r_dep) per axis (at least one),
   * each holding eight overlapping cubic domains of edge e - r_dep, one per
   * corner (bit d of corner k: [0, e - r_dep) or [r_dep', e) along axis d,
   * r_dep' = e - (e - r_dep), from the cell's corner).  A stage draws the
   * corner k = floor(w0 8 / 2^64) of Philox(key, (w, s, 0, 0)) and every cell
   * makes one trial in its domain k (none if it is empty): with W the
   * domain's summed weights 8 / m (m the number of the cell's domains
   * holding the atom, ascending atom order), the site is the first whose
   * running sum exceeds floor(w0 W / 2^64), w0 from Philox(key, (w, s, cell,
   * 1)).  Same-corner domains of different cells are r_dep apart.  A sweep
   * has ceil(N / N_cells) stages.  Single-system contexts with the
   * eight-colour scheme; sweeps run on the pipeline strategies (the default
   * becomes three stages per batch); the cell grid is that of creation.
   * 0: the colouring. */
  double grow_edge;
} vcsgc_system;

/* Per-call statistics (host struct). */
typedef struct {
  int64_t trials;         /* local trials made (sites drawn in non-empty active cells) */
  int64_t local_accepts;  /* trials passing the local factor */
  int64_t stages;         /* stages run */
  int64_t stage_accepts;  /* stages whose composite move passed the global factor */
  int64_t flips;          /* transmutations committed */
  int64_t near_ties;      /* decisions with |ln u + x| < 1e-9 */
  int64_t n_final;        /* n_B after the call */
  double sum_n, sum_n2;   /* sum over sweeps of n_B and n_B^2 after each sweep */
  int64_t stage1_pass;    /* trials passing the surrogate stage (= trials without one) */
} vcsgc_stats;

typedef struct {
  uint64_t sweeps_done; /* cumulative sweep counter w (Philox counter word 0) */
  int64_t n_b;          /* current number of B atoms (get only; set recounts it) */
  uint64_t seed;        /* Philox key word 0 of the last sweep call (0 before any) */
  double *rho_dev;      /* caller DEVICE buffer of N doubles or NULL: get copies the
                           density cache into it, set restores the cache from it */
} vcsgc_state;

typedef struct {
  int32_t n_cells[3];   /* link cells per dimension (even, edge >= r_dep) */
  int64_t stages_per_sweep; /* S = 8 ceil(N / N_cells) */
  int32_t kmax;         /* neighbour-list row capacity */
  int32_t mc_kmax_used; /* largest row of the r < rc list */
  int64_t mc_pairs;     /* entries of the r < rc list (0 before it is built) */
  int64_t md_pairs;     /* entries of the r < rc + skin list (0 before it is built) */
  int64_t md_rebuilds;  /* MD neighbour-list rebuilds so far */
} vcsgc_info;

/* Create a context for one system.  Validates the arguments and the input
 * arrays (positions inside the box, species in {0, 1}), bins the sites into
 * link cells of edge >= r_dep (an even number per dimension), builds the
 * r < rc neighbour list and the density cache rho_i = sum_j f_{s_j}(r_ij).
 * Sec. III.A: the independent-domain decomposition with R_c = 2 rc for a
 * many-body potential.  Errors: VCSGC_E_INVALID_ARG, VCSGC_E_BOX_TOO_SMALL
 * (fewer than two cells of edge r_dep in some dimension),
 * VCSGC_E_OUT_OF_MEMORY, VCSGC_E_OVERFLOW (a site with more than kmax
 * neighbours), VCSGC_E_DEVICE.  *out is set only on success. */
vcsgc_status vcsgc_create(const vcsgc_system *sys, hipStream_t stream, vcsgc_ctx **out);

/* Release a context and its scratch (synchronizes its stream). NULL is a no-op. */
vcsgc_status vcsgc_destroy(vcsgc_ctx *ctx);

/* Run n_sweeps sweeps of the parallel VC-SGC Monte Carlo of Sec. III.B.2 on
 * the species array.  Ensemble (Eq. pi_vcsgc, kappa per site):
 *   pi(sigma) ~ exp[-beta (U + phi n + (kappa/N) n^2)],  phi = dmu0 - 2 kappa cbar.
 * A sweep has S = 8 ceil(N/N_cells) stages (one MC cycle = N trials, Sec.
 * IV.B).  In each stage a colour is drawn (one of the eight independent
 * domain sets, Sec. III.A) and every non-empty cell of that colour makes one
 * trial at a uniformly drawn site, accepted locally with
 *   min{1, exp[-beta (dU_i + dmu0 dn_i)]}            (Eq. trans_vcsgc_par1);
 * the composite move is then accepted with
 *   min{1, exp[-beta (kappa/N) dn_tot (dn_tot + 2 (n - N cbar))]}
 * (Eq. trans_vcsgc_par2, the sign under which the two factors multiply to the
 * ensemble's weight ratio) and committed, updating the density cache.
 * Random numbers are Philox4x64-10 keyed (seed, 0) with counters
 * (w, s, 0, 0) for the stage and (w, s, cell, 1) for a trial, w the
 * cumulative sweep counter, so sweep(a) followed by sweep(b) equals
 * sweep(a + b).  kappa = 0 is plain SGC.  With velocities present a
 * transmuted atom's velocity is scaled by sqrt(m_old / m_new).
 * dmu0 in eV, kappa in eV per site (>= 0), cbar in [0, 1], T_K > 0,
 * n_sweeps >= 0.  out (host, may be NULL) receives the statistics of this call. */
vcsgc_status vcsgc_sweep(vcsgc_ctx *ctx, double dmu0, double kappa, double cbar, double T_K,
                         int64_t n_sweeps, uint64_t seed, vcsgc_stats *out);

/* Local chains (single-system contexts): every active cell makes k trials
 * per stage (1 <= k <= 64; default 1, the scheme of Sec. III.B), each on the
 * state left by the previous ones, with site and uniform from Philox counters
 * (w, s, cell, 1 + q), q = 0..k-1.  A locally accepted trial is applied at
 * once; the global factor of Eq. trans_vcsgc_par2 on the net change of n
 * keeps or undoes the stage as a whole (the local chain is reversible with
 * respect to the semi-grand-canonical weight at dmu0, so the product with the
 * global factor samples the same VC-SGC ensemble).  A sweep then has
 * 8 ceil(ceil(N / N_cells) / k) stages.  Such sweeps use per-stage launches;
 * delayed acceptance and the sample log need k = 1.  Applies to later calls. */
vcsgc_status vcsgc_set_local_steps(vcsgc_ctx *ctx, int32_t k);

/* Batch of independent replicas (for example a scan over T, kappa and cbar
 * as in phase-diagram work): one context, one persistent launch per call.
 * sys describes the concatenated arrays (n_atoms = sum of rep_atoms; replica
 * r occupies the next rep_atoms[r] entries); sys->box is ignored and
 * rep_box[3 r .. 3 r + 2] gives replica r's box.  Each replica gets its own
 * cells, stage count and Philox key (seed, r).  MC only: md_verlet_step,
 * eam_energy_forces and vcsgc_atom_energies reject batch contexts.
 * rep_atoms and rep_box are host arrays of n_rep and 3 n_rep entries. */
vcsgc_status vcsgc_create_batch(const vcsgc_system *sys, int32_t n_rep, const int64_t *rep_atoms,
                                const double *rep_box, hipStream_t stream, vcsgc_ctx **out);

/* n_sweeps sweeps of every replica of a batch (as vcsgc_sweep, per replica),
 * with per-replica parameters in host arrays of n_rep entries.  out (host,
 * n_rep entries, may be NULL) receives per-replica statistics.  All replicas
 * run in one persistent launch (wrapped in a HIP graph by default); each
 * replica's workgroups synchronize among themselves only. */
vcsgc_status vcsgc_sweep_batch(vcsgc_ctx *ctx, const double *dmu0, const double *kappa,
                               const double *cbar, const double *T_K, int64_t n_sweeps,
                               uint64_t seed, vcsgc_stats *out);

/* Execution tuning of the sweep (results do not depend on it):
 *   strategy 0: persistent launch captured in a HIP graph (default),
 *            1: persistent cooperative launch without a graph,
 *            2: the stage pipeline, one kernel per stage: the global test of
 *               the stage before it and the trials of its own (single
 *               system only);
 *            3: the batched stage pipeline: each kernel makes the trials of
 *               up to trials_per_group consecutive stages of a sweep on the
 *               state as it is, and the global tests of the batch tried by
 *               the kernel before it, in order, up to the first accepted
 *               stage, after which the trials are made again (single system
 *               only; trials_per_group in [1, 16], capped at half the stages
 *               of a sweep; with trial or stage logs on, or fewer than two
 *               stages per sweep, it runs as strategy 2);
 *   trials_per_group: strategies 0 and 1: active cells handled by each
 *            16-lane trial group per stage in the persistent kernel (sets
 *            the number of workgroups per replica; raised automatically if
 *            the grid would not fit); strategy 3: stages per batch.
 * Synchronizes the stream. */
vcsgc_status vcsgc_set_tuning(vcsgc_ctx *ctx, int32_t strategy, int32_t trials_per_group);
/* Current tuning and the persistent grid size (any output may be NULL). */
vcsgc_status vcsgc_get_tuning(vcsgc_ctx *ctx, int32_t *strategy, int32_t *trials_per_group,
                              int32_t *workgroups);

/* Bound on the waits of the persistent sweep (strategies 0 and 1): a
 * workgroup that polls a per-replica barrier `polls` times without seeing
 * every workgroup of its replica arrive abandons the call; vcsgc_sweep and
 * vcsgc_sweep_batch then return VCSGC_E_BARRIER_TIMEOUT and the context is
 * left in the error state (part of a stage may have been committed).
 * polls >= 1; the default, 2^24 polls with a short sleep each, is seconds.
 * For failure-handling tests and diagnostics. */
vcsgc_status vcsgc_set_wait_limit(vcsgc_ctx *ctx, uint32_t polls);

/* Fresh EAM evaluation at the current positions and species: rho, per-atom
 * energies E_i = F_{s_i}(rho_i) + 1/2 sum_j phi(r_ij) and, if want_forces,
 * forces F_i = sum_j [phi'(r) + F'_i f'_{s_j}(r) + F'_j f'_{s_i}(r)] (x_j - x_i)/r
 * written to sys.fx/fy/fz (which must then be non-NULL).  energy_eV (host,
 * may be NULL) receives U = sum_i E_i from a fixed-shape reduction tree. */
vcsgc_status eam_energy_forces(vcsgc_ctx *ctx, double *energy_eV, int want_forces);

/* n_steps velocity-Verlet steps of dt_fs with EAM forces (NVE; the MD half of
 * the hybrid MD/MC scheme of Sec. IV.A).  Forces are evaluated at the incoming
 * positions first; per step: v += dt/2 a, x += dt v (wrapped), forces,
 * v += dt/2 a, with a = F * 9.648533212e-3 / m.  The r < rc + skin list is
 * rebuilt whenever an atom has moved more than skin/2 since the last build.
 * Requires velocities and forces in the system.  The sweep's cell lists,
 * r < rc list and density cache are rebuilt from the new positions before the
 * next sweep. */
vcsgc_status md_verlet_step(vcsgc_ctx *ctx, double dt_fs, int64_t n_steps);

/* Nose-Hoover barostat for later md_verlet_step calls (the paper's Fe-Cu runs
 * hold temperature and pressure with the Nose-Hoover thermostat and
 * barostat, Sec. IV.B); it needs the thermostat on (vcsgc_set_thermostat).
 * Isotropic form of Martyna, Tobias and Klein (J. Chem. Phys. 101, 4177
 * (1994)) with the thermostat acting on particles and barostat:
 *   dx/dt = v + ve x,  dv/dt = F/m - (1 + 3/g) ve v - xi v,  dL/dt = ve L,
 *   dpe/dt = 3V (P - p_ext) + (3/g) 2K - xi pe,  ve = pe / W,
 *   dxi/dt = (2K + pe^2/W - (g + 1) kB T) / Q,  deta/dt = xi,
 * g = 3N - 3, Q = (g + 1) kB T tau_T^2, W = (g + 1) kB T tau_p_fs^2,
 * P = (2K + Vir) / (3V), Vir = -1/2 sum_i sum_j s_ij r_ij over r < rc
 * (s_ij = phi'(r) + F'_i f'_{s_j}(r) + F'_j f'_{s_i}(r)).  Conserved:
 * K + U + pe^2/(2W) + p_ext V + Q xi^2/2 + (g + 1) kB T eta.  A step of dt
 * (h = dt/2) is T(h) B(h) V(h) X(dt) [forces] V(h) B(h) T(h):
 *   T(h): xi += (h/2) G; s = (1 - xi h/2)/(1 + xi h/2); v *= s; pe *= s;
 *         K *= s^2; eta += xi h; xi += (h/2) G  (G from the current K, pe);
 *   B(h): pe += h (3V (P - p_ext) + (3/g) 2K);
 *   V(h): c = exp(-(1 + 3/g) ve h/2); v *= c; v += h a; v *= c;
 *   X(dt): q = exp(ve h); x = (x q + dt v) q, wrapped; every edge L *= q q;
 * K is summed afresh after each closing kick and at the start of a call,
 * and carried through the scalings otherwise; K and the virial are summed
 * in the fixed shape of eam_energy_forces.  p_ext in eV/A^3
 * (1 eV/A^3 = 160.2176634 GPa), pe in eV fs; tau_p_fs = 0 switches the
 * barostat off.  The search bins follow the box (at most the grid of
 * creation); a box that shrinks below two bins per axis ends
 * md_verlet_step with VCSGC_E_BOX_TOO_SMALL, and a sweep on a box whose
 * cells have shrunk below r_dep fails the same way.  Single-system MD
 * contexts.  Errors: VCSGC_E_INVALID_ARG. */
vcsgc_status vcsgc_set_barostat(vcsgc_ctx *ctx, double p_ext, double tau_p_fs, double pe);

/* The barostat momentum (eV fs), the box edges (A, host box[3]) and the
 * virial of the last force evaluation of an NPT call (eV); any pointer may
 * be NULL. */
vcsgc_status vcsgc_get_barostat(vcsgc_ctx *ctx, double *pe, double *box, double *virial);

/* Conjugate-gradient relaxation of the positions at fixed species and box
 * (Sec. IV.B relaxes the nanocrystal's grain boundaries by conjugate-gradient
 * minimization before its MD and MC/MD runs).  Nonlinear conjugate gradients
 * with the Polak-Ribiere coefficient clipped at zero and a backtracking
 * line search under the sufficient-decrease condition (Nocedal and Wright,
 * Numerical Optimization, Secs. 3.1, 3.5 and 5.2):
 *   E, F at x;  d = F;  gg = F.F;  then per iteration:
 *     stop if sqrt(gg) <= ftol (FORCE), iterations == max_iter (ITER) or
 *       evaluations >= max_eval (EVAL), in that order;
 *     sl = F.d, and if sl <= 0: d = F, sl = F.d (restart);
 *     a = dmax / max_i |d_i|, after the first iteration at most
 *       2 dE_prev / sl (dE_prev the last iteration's decrease);
 *     up to VCSGC_CG_TRIALS trials x' = wrap(x + a d), E' and F' at x',
 *       accepted when E' <= E - VCSGC_CG_C1 a sl and E' < E, else a /= 2;
 *       none accepted: stop (LINESEARCH) with x, E and F unchanged;
 *     b = max(0, (F'.F' - F'.F) / gg);  d = F' + b d;
 *     dE = E - E';  x, E, F, gg = x', E', F', F'.F';
 *     stop if dE <= etol |E| (ENERGY).
 * E is summed over the atoms' energies, and each dot product over the
 * per-atom terms (a_x b_x + a_y b_y) + a_z b_z, in the fixed shape of
 * eam_energy_forces.  sys.x/y/z are relaxed in place and sys.fx/fy/fz
 * (required) hold the forces at the final positions; velocities and species
 * are untouched.  The MD list is rebuilt as in md_verlet_step; the sweep's
 * lists are rebuilt before the next sweep.  res (host, may be NULL)
 * receives the counts, the final energy and |F|.  Single-system contexts.
 * Errors: VCSGC_E_INVALID_ARG (no force arrays, max_iter or max_eval < 0,
 * non-finite etol, ftol < 0, dmax outside (0, half the shortest box
 * edge)). */
#define VCSGC_CG_TRIALS 41
#define VCSGC_CG_C1 1e-4
enum { VCSGC_CG_FORCE = 1, VCSGC_CG_ENERGY = 2, VCSGC_CG_ITER = 3, VCSGC_CG_EVAL = 4,
       VCSGC_CG_LINESEARCH = 5 };
typedef struct {
  int64_t max_iter;  /* line searches */
  int64_t max_eval;  /* energy evaluations (checked before each line search) */
  double etol;       /* relative energy decrease that ends the run */
  double ftol;       /* |F| (2-norm of the 3N-vector, eV/A) that ends the run */
  double dmax;       /* largest single-atom move of a line search's first trial (A) */
} vcsgc_cg_params;
typedef struct {
  int64_t iterations, evaluations;
  double energy;  /* eV, at the final positions */
  double fnorm;   /* eV/A */
  int32_t reason; /* VCSGC_CG_* */
} vcsgc_cg_result;
vcsgc_status vcsgc_minimize(vcsgc_ctx *ctx, const vcsgc_cg_params *params,
                            vcsgc_cg_result *res);

/* Nose-Hoover thermostat for later md_verlet_step calls (the paper's Fe-Cu
 * runs thermostat their MD, Sec. IV.B).  T_K > 0 switches it on: equations
 * of motion dx/dt = v, dv/dt = F/m - xi v, dxi/dt = (2K - g kB T)/Q,
 * deta/dt = xi, with K the kinetic energy, g = 3N - 3 and
 * Q = g kB T tau_fs^2 (eV fs^2); T_K = 0 switches it off (NVE).  xi (1/fs)
 * and eta set the thermostat state.  A step is the symmetric splitting
 *   thermostat(dt/2); v += dt/2 a; x += dt v; forces; v += dt/2 a;
 *   thermostat(dt/2),
 * where a thermostat half step is xi += (dt/4) G; v *= s; K *= s^2;
 * eta += xi dt/2; xi += (dt/4) G, G = (2K - g kB T)/Q, with
 * s = (1 - xi dt/4)/(1 + xi dt/4) (the (1,1) Pade form of exp(-xi dt/2),
 * which keeps the splitting time reversible) and K summed afresh after each
 * closing kick in a fixed order (chunks of 256 atoms).  The conserved
 * quantity is K + U + Q xi^2 / 2 + g kB T eta.  Needs a single-system
 * context with velocities.  Errors: VCSGC_E_INVALID_ARG. */
vcsgc_status vcsgc_set_thermostat(vcsgc_ctx *ctx, double T_K, double tau_fs, double xi,
                                  double eta);
/* Current thermostat state (either output may be NULL; synchronizes). */
vcsgc_status vcsgc_get_thermostat(vcsgc_ctx *ctx, double *xi, double *eta);

/* Message of the last error on this context (or of the last failed create when
 * ctx is NULL).  The string is owned by the library. */
const char *vcsgc_last_error(const vcsgc_ctx *ctx);

/* Parity logging.  While enabled, every trial appends 8 doubles
 * (w, s, cell, site, dn, local_accept, dU, ln u + x) to tlog and every stage
 * appends (w, s, colour, dn_tot, n_records, global_accept or -1, x_g,
 * ln u_g + x_g) to slog, in completion order, until the capacities (in
 * records) are reached.  Buffers are caller-owned device memory.  Passing
 * NULL buffers disables logging and resets the counters. */
vcsgc_status vcsgc_set_log(vcsgc_ctx *ctx, double *tlog_dev, int64_t tcap, double *slog_dev,
                           int64_t scap);
/* Number of records written so far (may exceed the capacity). */
vcsgc_status vcsgc_log_counts(vcsgc_ctx *ctx, int64_t *n_trials, int64_t *n_stages);

/* Chain state for checkpoint/resume: the cumulative sweep counter, n_B, the
 * seed of the last sweep call and, through rho_dev, the density cache
 * rho_i = sum_j f_{s_j}(r_ij) that the trials of Eq. trans_vcsgc_par1 read.
 * The cache is updated in place by every committed flip, so after many
 * commits it differs in the last bits from a fresh sum; restoring it (with
 * the caller's species and positions) continues the chain bit for bit.
 * set_state: sets the counter and the recorded seed, recounts n_B from the
 * species, rebuilds the cell and neighbour lists from the positions and, if
 * rho_dev is not NULL, replaces the fresh density cache by rho_dev (else the
 * fresh sum is kept).  Synchronizes the stream.  Errors: VCSGC_E_INVALID_ARG
 * for a NULL state. */
vcsgc_status vcsgc_get_state(vcsgc_ctx *ctx, vcsgc_state *out);
vcsgc_status vcsgc_set_state(vcsgc_ctx *ctx, const vcsgc_state *in);

/* Copy the density cache (N doubles) into a caller device buffer. */
vcsgc_status vcsgc_copy_rho(vcsgc_ctx *ctx, double *rho_dev);
/* Per-atom energies at the current state (fresh density) into a device buffer. */
vcsgc_status vcsgc_atom_energies(vcsgc_ctx *ctx, double *e_dev);
/* Geometry of the context. */
vcsgc_status vcsgc_get_info(vcsgc_ctx *ctx, vcsgc_info *out);

/* Kernel classes for per-kernel timing. */
#define VCSGC_KT_TRIAL 0      /* sweep: trial + local factor */
#define VCSGC_KT_COMMIT 1     /* sweep: global factor + commit */
#define VCSGC_KT_DENSITY 2    /* EAM density + embedding derivative */
#define VCSGC_KT_FORCES 3     /* EAM forces */
#define VCSGC_KT_KICKDRIFT 4  /* velocity Verlet first half + drift */
#define VCSGC_KT_KICK 5       /* velocity Verlet second half */
#define VCSGC_KT_BUILD 6      /* cell binning + neighbour list */
#define VCSGC_KT_ENERGY 7     /* per-atom energies */
#define VCSGC_KT_PERSIST 8    /* persistent sweep (one launch per call) */
#define VCSGC_KT_STAGE 9      /* sweep: fused stage kernel (global factor of one stage,
                                 then, unless it accepts, the trials of the next) */
#define VCSGC_KT_CLASSES 10

typedef struct {
  double total_ms[VCSGC_KT_CLASSES]; /* summed event-to-event durations */
  int64_t count[VCSGC_KT_CLASSES];   /* timed launches */
  int64_t launches[VCSGC_KT_CLASSES]; /* all launches of the class (timed or not) */
} vcsgc_ktimes;

/* Time every launch of the kernel classes in mask (bit k = class k) with a
 * pair of HIP events recorded on the context's stream around the launch;
 * resets the accumulated times.  mask = 0 disables timing. */
vcsgc_status vcsgc_kernel_timing(vcsgc_ctx *ctx, uint32_t mask);
/* As vcsgc_kernel_timing, but only one launch in `every` (>= 1) of each
 * class is timed (launch index mod every == 0 since this call), so that the
 * event pairs themselves add little host and stream work next to kernels
 * launched hundreds of times per call; count then holds the timed launches.
 * (The pipelines time the span of whole graph replays either way.) */
vcsgc_status vcsgc_kernel_timing_sampled(vcsgc_ctx *ctx, uint32_t mask, int32_t every);
/* Accumulated times since the last vcsgc_kernel_timing call (synchronizes). */
vcsgc_status vcsgc_get_kernel_timing(vcsgc_ctx *ctx, vcsgc_ktimes *out);

/* ---- surrogate delayed acceptance -------------------------------------
 * A small network (10 -> 64 -> 64 -> 1, SiLU; BF16 weights and activations
 * on the MFMA units, FP32 accumulation) predicts the transmutation energy
 * change from a local descriptor of the site:
 *   [s_i, nB1, nB2, nB3, n1, n2, n3, rho1, rho2, rho3]
 * (species of the site; B and total neighbour counts and mean neighbour
 * density in the shells r < 2.68, [2.68, 3.46), [3.46, 4.41) A).  It is used
 * only as the first stage of a delayed-acceptance test (Christen and Fox):
 * the exact FP64 energy change decides every accepted move, so the sampled
 * ensemble is that of vcsgc_sweep.  Contexts need VCSGC_FLAG_DESCRIPTOR. */

typedef struct {
  int64_t epochs;   /* passes over the samples */
  int64_t batch;    /* minibatch size (samples drawn with replacement) */
  double lr, beta1, beta2, eps; /* Adam */
  uint64_t seed;    /* minibatch draws */
} vcsgc_train_cfg;

typedef struct {
  double loss_first, loss_last; /* mean squared error of the normalized output */
  int64_t steps;
} vcsgc_train_report;

/* New network with random FP32 weights (seed) on the calling device. */
vcsgc_status vcsgc_mlp_create(uint64_t seed, hipStream_t stream, vcsgc_mlp **out);
vcsgc_status vcsgc_mlp_destroy(vcsgc_mlp *m);
/* Host copies of the 4929 parameters (w1[64][10], b1[64], w2[64][64], b2[64],
 * w3[64], b3) and of the normalization (mu[10], sd[10], out_mu, out_sd). */
vcsgc_status vcsgc_mlp_set_params(vcsgc_mlp *m, const float *params, const float *mu,
                                  const float *sd, float out_mu, float out_sd);
vcsgc_status vcsgc_mlp_get_params(vcsgc_mlp *m, float *params, float *mu, float *sd,
                                  float *out_mu, float *out_sd);
/* Input and output normalization from n samples (device arrays
 * desc[n][10] FP64, dE[n] eV): per-column mean and standard deviation. */
vcsgc_status vcsgc_mlp_fit_normalization(vcsgc_mlp *m, const double *desc_dev,
                                         const double *dE_dev, int64_t n);
/* Train on n device samples (Adam on FP32 master weights, mean squared error
 * of the normalized output); report may be NULL. */
vcsgc_status vcsgc_mlp_train(vcsgc_mlp *m, const double *desc_dev, const double *dE_dev,
                             int64_t n, const vcsgc_train_cfg *cfg, vcsgc_train_report *report);
/* dE_dev[k] = network(desc_dev[k]) in eV for n samples. */
vcsgc_status vcsgc_mlp_forward(vcsgc_mlp *m, const double *desc_dev, int64_t n, double *dE_dev);
/* Gradient of the loss over all n samples (host, 4929 floats) and the loss. */
vcsgc_status vcsgc_mlp_grad(vcsgc_mlp *m, const double *desc_dev, const double *dE_dev, int64_t n,
                            float *grad_host, double *loss);

/* Allocation-free form of vcsgc_mlp_grad, for callers that cannot allocate
 * device memory (code under HIP graph capture, training loops that forbid
 * allocation): the same forward and backward kernels on n <= 4096 samples,
 * with the batch's workspace in a fixed device array of the library
 * (about 7.6 MB per device, held until the process ends) instead of the
 * network's own buffers, which vcsgc_mlp_grad grows with hipMalloc.
 * desc_dev[n][10] (FP64) and dE_dev[n] (eV) are inputs; grad_dev receives the
 * 4929 gradient values (parameter order of vcsgc_mlp_set_params) and
 * loss_dev the mean squared error of the normalized output, both DEVICE
 * memory owned by the caller.  The network is only read.  Asynchronous on
 * the network's stream: no synchronization, no host copy, no allocation.
 * Calls that overlap on one device share the workspace and race; run them
 * in one stream.  Errors: VCSGC_E_INVALID_ARG (NULL pointers, n outside
 * [1, 4096]), VCSGC_E_DEVICE (launch failure). */
#define VCSGC_NOALLOC_MAX_SAMPLES 4096
vcsgc_status vcsgc_mlp_grad_noalloc(const vcsgc_mlp *m, const double *desc_dev,
                                    const double *dE_dev, int64_t n, float *grad_dev,
                                    double *loss_dev);

/* Record (descriptor, exact dU) of every stride-th trial of later sweeps into
 * caller device buffers desc_dev[cap][10], dE_dev[cap] (training samples);
 * NULL buffers stop recording.  Needs VCSGC_FLAG_DESCRIPTOR. */
vcsgc_status vcsgc_set_sample_log(vcsgc_ctx *ctx, double *desc_dev, double *dE_dev, int64_t cap,
                                  int64_t stride);
vcsgc_status vcsgc_sample_count(vcsgc_ctx *ctx, int64_t *n_logged);

/* Surrogate stage for later sweeps: mode 0 plain, 1 the network m, 2 perfect
 * surrogate (dE = exact dU; equals the plain chain), 3 zero surrogate.  Mode 1
 * needs VCSGC_FLAG_DESCRIPTOR and r_dep >= 4.41 + rc (the descriptor reads
 * densities that depend on species up to that distance).  The network must
 * outlive its use.  Delayed acceptance runs with per-stage launches. */
vcsgc_status vcsgc_set_surrogate(vcsgc_ctx *ctx, const vcsgc_mlp *m, int32_t mode);
/* While enabled, every delayed-acceptance trial appends (w, s, cell, dE_f,
 * dE_r or NaN) to a caller device buffer of cap rows. */
vcsgc_status vcsgc_set_surrogate_log(vcsgc_ctx *ctx, double *log_dev, int64_t cap);
/* Descriptors (out_dev[n][10]) of the given sites at the current state, or of
 * the states with each site flipped (flip != 0).  Diagnostics. */
vcsgc_status vcsgc_descriptors(vcsgc_ctx *ctx, const int32_t *sites_dev, int64_t n, int32_t flip,
                               double *out_dev);

/* Diagnostics: out[i] = sqrt(in[i]) in FP64 on the device, n >= 0. */
vcsgc_status vcsgc_selftest_sqrt(const double *in_dev, double *out_dev, int64_t n,
                                 hipStream_t stream);
/* Diagnostics: the square root and quotient of the MD density and force
 * passes, sqrt_dev[i] = sqrt(a[i]) and div_dev[i] = a[i] / b[i] (Newton-
 * Raphson refinements of reciprocal(-square-root) estimates with a final
 * fused-multiply-add correction; meant for 2^-767 <= a[i] <= DBL_MAX and, for
 * the quotient, normal operands whose quotient is far from the ends of the
 * exponent range, where both are correctly rounded), n >= 0. */
vcsgc_status vcsgc_selftest_md_math(const double *a_dev, const double *b_dev, double *sqrt_dev,
                                    double *div_dev, int64_t n, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* VCSGC_H */
