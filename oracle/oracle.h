/*
 * Plain serial FP64 reference ("oracle") of the parallel VC-SGC transmutation
 * Monte Carlo and EAM molecular dynamics of Sadigh et al., "A scalable parallel
 * Monte Carlo algorithm for atomistic simulations of precipitation in alloys".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this code; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (see oracle/build_oracle.py).
 */
#ifndef VCSGC_ORACLE_H
#define VCSGC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Analytic Finnis-Sinclair EAM: phi_XY = eps_XY (rc-r)^2 (c0 + c1 r),
 * f_X = t_X (rc-r)^2, F_X(rho) = -A_X sqrt(rho); zero for r >= rc.
 * With tab != 0 the potential is tabulated instead (a general embedded-atom
 * potential, the class named in the Introduction and Sec. III):
 * f_A, f_B and phi_AA, phi_AB, phi_BB at the radial knots r_k = k dr
 * (k = 0 .. nr-1), F_A and F_B at the density knots rho_k = k drho
 * (k = 0 .. nrho-1), each interpolated by the piecewise cubic of
 * or_spline_coeffs (cf, cphi, cF: 4 coefficients per interval); f and phi are
 * zero for r >= rc, and F is evaluated outside its knots by the end
 * intervals' cubics.  Only rc of the analytic fields is used then. */
typedef struct {
  double rc, c0, c1, eps_aa, eps_ab, eps_bb, t_a, t_b, a_a, a_b;
  int32_t tab, nr, nrho, pad_;
  double inv_dr, inv_drho;
  const double *cf[2], *cphi[3], *cF[2];
} or_pot;

/* Piecewise cubic through y[0 .. n-1] (n >= 2) at unit-spaced knots: the
 * cubic Hermite interpolant whose knot slopes are central differences
 * m_k = (y_{k+1} - y_{k-1}) / 2, one-sided at the two ends.  Interval k
 * (0 <= k < n-1) gets c[4k .. 4k+3] = (a0, a1, a2, a3) with
 * p(t) = ((a3 t + a2) t + a1) t + a0 for t in [0, 1]:
 *   a0 = y_k, a1 = m_k, a2 = (3 d - 2 m_k) - m_{k+1}, a3 = (m_k + m_{k+1}) - 2 d,
 *   d = y_{k+1} - y_k. */
void or_spline_coeffs(int32_t n, const double *y, double *c);
/* The interpolant at x (knots at x = k h, inv_h = 1/h) and, if der != NULL,
 * its derivative in x: p = x inv_h, k = floor(p) limited to [0, n-2],
 * t = p - k (outside the knots the end interval's cubic continues). */
double or_spline_eval(const double *c, int32_t n, double x, double inv_h, double *der);

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void or_philox4x64_10(const uint64_t key[2], const uint64_t ctr[4], uint64_t out[4]);

/* All pairs (j, image) with r < cutoff, rows in ascending (j, image) order.
 * mode 0: automatic; 1: brute force, minimum image; 2: brute force image sum.
 * Requires every box edge > cutoff (image sum) or >= 2*cutoff (minimum image).
 * Returns the number of entries; if it exceeds cap nothing past cap is written.
 * Returns -1 on an invalid box. */
int64_t or_neighbors(int64_t n, const double *x, const double *y, const double *z,
                     const double box[3], double cutoff, int mode, int64_t cap,
                     int64_t *start, int32_t *nj, double *nr,
                     double *ndx, double *ndy, double *ndz);

void or_density(int64_t n, const int64_t *start, const int32_t *nj, const double *nr,
                const uint8_t *species, const or_pot *p, double *rho);
void or_energy_atoms(int64_t n, const int64_t *start, const int32_t *nj, const double *nr,
                     const uint8_t *species, const or_pot *p, const double *rho, double *e);
double or_energy_total(int64_t n, const double *e);
void or_forces(int64_t n, const int64_t *start, const int32_t *nj, const double *nr,
               const double *ndx, const double *ndy, const double *ndz,
               const uint8_t *species, const or_pot *p, const double *rho,
               double *fx, double *fy, double *fz);
double or_delta_u(int64_t i, const int64_t *start, const int32_t *nj, const double *nr,
                  const uint8_t *species, const double *rho, const or_pot *p);

/* Link cells for the sweep: 2*floor(L/(2 r_dep)) cells per dimension. */
int or_cell_grid(const double box[3], double r_dep, int32_t nc[3]);
/* With colour period P (2 or 3): P*floor(L/(P r_dep/(P-1))) cells per
 * dimension, of edge >= r_dep/(P-1); colours are the indices modulo P. */
int or_cell_grid_p(const double box[3], double r_dep, int period, int32_t nc[3]);

typedef struct {
  double dmu0;      /* eV: Delta mu_0 = phi + 2 kappa c0 (local factor) */
  double kappa;     /* eV per site (ensemble weight exp[-beta kappa n^2 / N]) */
  double cbar;      /* c0 of the global factor */
  double temp;      /* K */
  uint64_t seed, replica;
  int64_t w0, n_sweeps;
  double r_dep;     /* independence distance: cell edge >= r_dep */
  int32_t one_cell; /* serial mode: one cell holding every site, N stages per sweep */
  double mass_a, mass_b; /* for velocity rescaling on transmutation */
  int32_t local_steps;   /* trials per active cell per stage (0 or 1: one) */
  int32_t colour_period; /* 0 or 2: eight colours; 3: 27 colours on cells of edge >= r_dep/2 */
  double grow_edge;      /* > 0: grown domains in cells of edge >= max(grow_edge, 2 r_dep) */
} or_sweep_args;

typedef struct {
  int64_t trials, local_accepts, stages, stage_accepts, flips, near_ties, n_final;
  double sum_n, sum_n2;
} or_stats;

/* One pass of n_sweeps sweeps.  species, rho and n (count of species 1)
 * are updated in place.  vx/vy/vz may be NULL.
 * With local_steps = k > 1 every active cell runs a local Metropolis chain
 * of k trials per stage (each on the state left by the previous one, sites
 * and uniforms from Philox(key, (w, s, cell, 1 + q)), q = 0..k-1); the
 * composite move of the stage is the product of these chains and is kept or
 * undone as a whole by the global factor on its net dn_tot.  A sweep then has
 * 8 ceil(ceil(N / N_cells) / k) stages (ceil(N / k) in one-cell mode).  In the
 * trial log and the overrides the cell field holds cell * k + q.
 * With grow_edge > 0 the domains are grown (Sec. III.A, Fig. 6): cells of
 * edge e >= max(grow_edge, 2 r_dep) per axis, and in each cell eight
 * overlapping cubic domains of edge e - r_dep, one per corner; a stage
 * draws one of the eight and every cell makes a trial in it, the site drawn
 * with weight 8 / m (m the number of the cell's domains holding the atom);
 * a sweep has ceil(ceil(N / N_cells) / k) stages (see or_grown_lists).
 * tlog: trial log, 8 doubles per trial (w, s, cell, site, dn, acc, dU, margin),
 * slog: stage log, 8 doubles per stage (w, s, colour, dn_tot, nrec, acc, xg, margin),
 * over: near-tie decisions to adopt, 4 doubles each (w, s, cell or -1, decision).
 * Returns 0, or a negative code on invalid input. */
int or_sweep(int64_t n, const double *x, const double *y, const double *z, const double box[3],
             const int64_t *start, const int32_t *nj, const double *nr,
             uint8_t *species, double *rho, int64_t *n_b, const or_pot *p,
             const or_sweep_args *a, double *vx, double *vy, double *vz,
             double *tlog, int64_t tcap, int64_t *tn,
             double *slog, int64_t scap, int64_t *sn,
             const double *over, int64_t n_over, or_stats *st);

/* All-core CPU baseline of or_sweep for the plain scheme (local_steps 1, no
 * one-cell mode, no trial log or overrides): the trials of each stage run on
 * n_threads OpenMP threads; counters, records, the global test and the
 * commits are those of or_sweep, so the chain is bitwise the same. */
int or_sweep_omp(int64_t n, const double *x, const double *y, const double *z,
                 const double box[3], const int64_t *start, const int32_t *nj,
                 const double *nr, uint8_t *species, double *rho, int64_t *n_b,
                 const or_pot *p, const or_sweep_args *a, double *vx, double *vy, double *vz,
                 double *slog, int64_t scap, int64_t *sn, int n_threads, or_stats *st);

/* ---- surrogate delayed acceptance ------------------------------------ */

/* Local descriptor of site i (10 values): [s_i, nB1, nB2, nB3, n1, n2, n3,
 * rho1, rho2, rho3], shells r < 2.68, [2.68, 3.46), [3.46, 4.41) A; nBk / nk
 * count B / all neighbours in shell k, rhok is the mean density of the
 * shell's neighbours (0 for an empty shell).  The list (CSR) must hold every
 * pair with r < 4.41.  With flip != 0 the descriptor is that of the state
 * with s_i flipped: rho_j of every neighbour with r < rc is shifted by
 * f_{s'}(r) - f_s(r) (summed over images). */
void or_descriptor(int64_t i, const int64_t *start, const int32_t *nj, const double *nr,
                   const uint8_t *species, const double *rho, const or_pot *p, int flip,
                   double out[10]);

/* Round a float to bfloat16 (round to nearest, ties to even), returned as a
 * float holding the rounded value. */
float or_bf16(float v);

/* MLP 10 -> 64 -> 64 -> 1 with SiLU, parameters in FP32:
 * w1[64*10], b1[64], w2[64*64], b2[64], w3[64], b3[1]; input normalization
 * z_k = (float)((d_k - mu_k) / sd_k); output dE = y * out_sd + out_mu.
 * With bf16 != 0 the operands of the products (z, weights, hidden
 * activations) are rounded to bfloat16 as the device does; sums are FP64. */
typedef struct {
  const float *w1, *b1, *w2, *b2, *w3, *b3, *mu, *sd;
  float out_mu, out_sd;
} or_mlp;

/* Forward for n samples of raw descriptors d[n*10] (FP64); y[n] (normalized
 * output) and dE[n] (eV) may be NULL. */
void or_mlp_forward(const or_mlp *m, int64_t n, const double *d, int bf16, double *y, double *dE);

/* Mean squared error of the normalized output against (t - out_mu)/out_sd
 * over n samples and its gradient (FP64) in the parameter order
 * w1, b1, w2, b2, w3, b3 (4929 values). Returns the loss. */
double or_mlp_grad(const or_mlp *m, int64_t n, const double *d, const double *t, int bf16,
                   double *grad);

/* Surrogate modes of the delayed-acceptance sweep. */
#define OR_DA_OFF 0     /* plain sweep */
#define OR_DA_TABLE 1   /* surrogate values taken from a table (w, s, cell, fwd, rev) */
#define OR_DA_PERFECT 2 /* forward = exact dU, reverse = -dU */
#define OR_DA_ZERO 3    /* forward = reverse = 0 */
#define OR_DA_MLP 4     /* the MLP above on the descriptors (bf16 emulation) */

typedef struct {
  int mode;
  const double *table; /* OR_DA_TABLE: n_table rows (w, s, cell, fwd, rev) sorted by (w, s, cell) */
  int64_t n_table;
  const or_mlp *mlp;   /* OR_DA_MLP */
  const int64_t *dstart; /* descriptor list (r < 4.41), OR_DA_MLP */
  const int32_t *dnj;
  const double *dnr;
  int64_t stage1_pass; /* out: trials passing the surrogate stage */
  /* OR_DA_TABLE with the descriptor list given: every trial appends
   * (w, s, cell, descriptor of the current state [10], descriptor of the
   * state with the site flipped [10]) to dlog (23 doubles per row, at most
   * dcap rows); dn counts the rows (it may exceed dcap). */
  double *dlog;
  int64_t dcap, dn;
} or_da;

/* The same sweep with the delayed-acceptance local test (Christen & Fox):
 * stage 1 accepts with min{1, exp(-beta (dE_f + dmu0 dn))} using u1 = unit(w1);
 * a survivor is accepted with
 *   min{1, exp(-beta (dU + dmu0 dn)) min{1, exp(-beta s_r)} / min{1, exp(-beta s_f)}},
 * s_f = dE_f + dmu0 dn, s_r = dE_r - dmu0 dn, dE_r the surrogate value for
 * the reverse move, using u2 = unit(w2); the global factor is unchanged.
 * The trial log's dU column holds the exact dU for survivors and NaN for
 * stage-1 rejections; its margin column the margin of the deciding test. */
int or_sweep_da(int64_t n, const double *x, const double *y, const double *z, const double box[3],
                const int64_t *start, const int32_t *nj, const double *nr,
                uint8_t *species, double *rho, int64_t *n_b, const or_pot *p,
                const or_sweep_args *a, or_da *da,
                double *tlog, int64_t tcap, int64_t *tn,
                double *slog, int64_t scap, int64_t *sn, or_stats *st);

/* Velocity Verlet, n_steps steps of dt (fs).  Forces are evaluated at the
 * incoming positions first; on return fx/fy/fz and rho hold the values at the
 * final positions. */
int or_md(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
          const uint8_t *species, const double box[3], const or_pot *p,
          double mass_a, double mass_b, double dt, int64_t n_steps,
          double *fx, double *fy, double *fz, double *rho);

/* or_md with the atoms of every loop split over n_threads OpenMP threads
 * (all-core CPU baseline; bitwise or_md). */
int or_md_omp(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
              const uint8_t *species, const double box[3], const or_pot *p,
              double mass_a, double mass_b, double dt, int64_t n_steps,
              double *fx, double *fy, double *fz, double *rho, int n_threads);

/* Fixed-shape sum (chunks of 256 summed by halving strides, chunk c added to
 * accumulator c mod 256 in ascending c, accumulators combined by halving
 * strides): the order in which totals that steer a trajectory are taken. */
double or_tree_sum(int64_t n, const double *v);

/* Nose-Hoover NVT velocity Verlet, n_steps steps of dt (fs) at temp (K) with
 * coupling time tau (fs): Q = g kB T tau^2, g = 3N - 3.  xi_io / eta_io carry
 * the thermostat friction (1/fs) and its time integral in and out.  tau =
 * infinity gives or_md's NVE steps bit for bit. */
int or_md_nvt(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
              const uint8_t *species, const double box[3], const or_pot *p, double mass_a,
              double mass_b, double dt, int64_t n_steps, double temp, double tau, double *xi_io,
              double *eta_io, double *fx, double *fy, double *fz, double *rho);

/* Isotropic NPT velocity Verlet (Nose-Hoover thermostat and MTK barostat;
 * the equations and the splitting are listed above or_md_npt in oracle.c):
 * n_steps of dt (fs) at temp (K), thermostat time tau_t (fs), pressure p_ext
 * (eV/A^3) and barostat time tau_p (fs).  box (in/out) scales with the
 * positions; state = (xi, eta, pe) in and out; vir_out receives the virial
 * of the last force evaluation (eV). */
int or_md_npt(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
              const uint8_t *species, double box[3], const or_pot *p, double mass_a,
              double mass_b, double dt, int64_t n_steps, double temp, double tau_t,
              double p_ext, double tau_p, double *state, double *fx, double *fy, double *fz,
              double *rho, double *vir_out);

/* Conjugate-gradient relaxation (PR+ nonlinear CG with a backtracking
 * Armijo line search; the steps are listed above or_cg in oracle.c).  x, y,
 * z are relaxed in place; fx, fy, fz and rho are those at the final
 * positions.  steepest != 0 forces b = 0 (steepest descent, for tests).
 * log (may be NULL) receives per iteration (E, E', a, sl, b, restart).
 * Stop reasons: */
enum { OR_CG_FORCE = 1, OR_CG_ENERGY = 2, OR_CG_ITER = 3, OR_CG_EVAL = 4, OR_CG_LINESEARCH = 5 };
int or_cg(int64_t n, double *x, double *y, double *z, const uint8_t *species,
          const double box[3], const or_pot *p, int64_t max_iter, int64_t max_eval, double etol,
          double ftol, double dmax, int steepest, double *fx, double *fy, double *fz,
          double *rho, int64_t *iters_out, int64_t *evals_out, double *e_out, double *fnorm_out,
          int *reason_out, double *log, int64_t log_cap);

#ifdef __cplusplus
}
#endif
#endif
