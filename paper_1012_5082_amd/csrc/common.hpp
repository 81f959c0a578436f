// Shared declarations of the HIP library: context, device helpers (Philox,
// Finnis-Sinclair EAM), launch helpers.  gfx950 only.
//
// Floating-point policy: every FP64 expression is evaluated exactly in the
// order written (the library is compiled with -ffp-contract=off), sums over
// neighbours run in ascending neighbour index, and no floating-point atomics
// are used, so results are reproducible bit for bit run to run.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "vcsgc.h"

namespace vc {

constexpr double KB = 8.617333262e-5;   // eV/K
constexpr double ACC = 9.648533212e-3;  // (eV/A)/u -> A/fs^2
constexpr double TIE = 1e-9;            // near-tie margin on |ln u + x|
constexpr int KMAX = 32;                // neighbour-list row capacity
constexpr int BLOCK = 256;
constexpr double DESC_CUT = 4.41;  // outer edge of the third descriptor shell (A)
constexpr int NPART = 5;           // trial-kernel partials: trials, accepts, sum dn, ties, stage-1 passes

// Potential in device-friendly form; eps is indexed by s_i + s_j.
struct PotD {
  double rc, c0, c1;
  double eps[3];
  double t[2];
  double A[2];
  double cm[2];    // ACC / mass
  double mass[2];  // u
  // tabulated potential (tab != 0; then only rc, cm and mass above are
  // used): piecewise-cubic coefficients, 4 per interval, of f_A, f_B,
  // phi_AA, phi_AB, phi_BB over the nr - 1 radial intervals, then F_A, F_B
  // over the nrho - 1 density intervals
  int tab, nr, nrho;
  double inv_dr, inv_drho;
  const double *tc;
};

// Progress of the fused stage pipeline of one call: stage s of sweep w and
// what its next kernel does with it.  Kept twice, indexed by the parity of
// the launch: a kernel reads one copy and its block 0 writes the other.
enum : int { SM_TRIAL = 0, SM_DECIDE = 1, SM_DONE = 2 };
struct StageMachine {
  unsigned long long w;  // sweep of the stage
  long long s;           // stage within the sweep
  long long nb;          // n_B before the global test of stage (w, s)
  int phase;             // SM_TRIAL: its trials are next; SM_DECIDE: its global test is next
  int pad;
};
// Progress of the batched pipeline: each kernel makes the trials of a batch
// of up to SPEC_MAX consecutive stages of one sweep (on the state as it is,
// that is, assuming that every stage of the batch before them is rejected)
// and the global tests of the batch the kernel before it tried.  A batch is
// none when its length is 0; the call is done when both are none.
constexpr int SPEC_MAX = 16;  // stages per batch, at most
constexpr int SPEC_NDEC = 32; // blocks that make the global tests (and share a commit)
struct SpecMachine {
  unsigned long long dw, tw;  // sweep of the batch to test / to try
  long long ds, ts;           // its first stage
  long long nb;               // n_B before the batch to test
  int dn, tn;                 // batch lengths
};
struct StageProgress {
  StageMachine sm[2];
  SpecMachine spec[2];
  unsigned long long w_end;    // first sweep past the end of the call
  unsigned long long used;     // pipeline kernels that did work in the call
};

// Device-resident counters and chain scalars of one context.
struct DevState {
  unsigned long long trials, local_acc, stages, stage_acc, flips, near_ties;
  long long n_b[2];             // n_B, ping-pong by stage parity within a call
  long long n_b_cur;            // n_B after the last committed stage
  long long dn[2];              // per-stage sum of dn over local accepts
  unsigned long long nrec[2];   // per-stage count of local accepts
  double sum_n, sum_n2;
  unsigned long long tlog_n, slog_n;
  int overflow;   // a neighbour row exceeded KMAX
  int bin_overflow;  // a search bin exceeded its capacity
  int bad_input;  // position outside the box / species not in {0,1}
  int rebuild[2];  // MD: an atom moved more than skin/2 (by the parity of the step)
  int kmax_used;  // longest row of the current r < rc list
  int kmax_md;    // longest row of the current r < rc + skin list
  unsigned long long pairs_mc, pairs_md;  // entries of the last r < rc / r < rc + skin lists
  unsigned long long stage1_pass;         // trials passing the surrogate stage
  unsigned long long smp_n, dalog_n;      // sample-log and surrogate-log records written
  unsigned long long md_rebuilds;         // MD list rebuilds taken on the device
  unsigned long long wcur;                // sweep counter of a graph-replayed sweep
  StageProgress pipe;                     // fused stage pipeline of the current call
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round
// multiplies words 0 and 2 by the two round constants (full 128-bit
// products), swaps and xors the high halves with words 1/3 and the key; the
// key advances by the two Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct U4 {
  uint64_t v[4];
};

__device__ __forceinline__ U4 philox(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1,
                                     uint64_t c2, uint64_t c3) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t a = hi1 ^ c1 ^ k0, b = hi0 ^ c3 ^ k1;
    c0 = a;
    c1 = lo1;
    c2 = b;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  U4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// uniform double in (0,1): ((w >> 11) + 1/2) 2^-53
__device__ __forceinline__ double unit_open(uint64_t w) {
  return ((double)(w >> 11) + 0.5) * 0x1p-53;
}

// uniform index in [0, m): floor(w m / 2^64)
// colour of a stage: floor(w ncol / 2^64) (w >> 61 for eight colours)
__device__ __forceinline__ int stage_colour(uint64_t w, int ncol) {
  return (int)__umul64hi(w, (uint64_t)ncol);
}

__device__ __forceinline__ uint32_t draw_index(uint64_t w, uint32_t m) {
  return (uint32_t)__umul64hi(w, (uint64_t)m);
}

// ---------------------------------------------------------------------------
// Finnis-Sinclair EAM pieces.  With d = rc - r, dd = d*d, g = c0 + c1 r:
//   phi_XY = (eps_XY dd) g,  f_X = t_X dd,  F_X(rho) = -A_X sqrt(max(rho,0)).
// ---------------------------------------------------------------------------
// (rc - r)^2 and c0 + c1 r of a pair at distance r < rc (the r < rc list
// keeps r; every user forms these the same way)
__device__ __forceinline__ double pair_dd(const PotD &p, double r) {
  const double d = p.rc - r;
  return d * d;
}
__device__ __forceinline__ double pair_g(const PotD &p, double r) { return p.c0 + p.c1 * r; }

// Square root of the MD passes, for 2^-767 <= x <= DBL_MAX: an estimate of
// 1/sqrt(x) refined by one coupled Newton-Raphson step for g ~ sqrt(x) and
// h ~ 1/(2 sqrt(x)) (Goldschmidt's iteration), then two corrections
// g += (x - g^2) h whose residuals are exact in a fused multiply-add
// (Markstein, IA-64 and Elementary Functions, 2000).  Over that range the
// result is the correctly rounded square root (vcsgc_selftest_md_math checks
// it against the host's); outside it (0, denormals, inf) it is not meant to
// be used: there the library's sqrt rescales the argument first.
__device__ __forceinline__ double sqrt_md(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = __builtin_fma(-h, g, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  double d = __builtin_fma(-g, g, x);
  g = __builtin_fma(d, h, g);
  d = __builtin_fma(-g, g, x);
  return __builtin_fma(d, h, g);
}

// Quotient a / b of the force pass, for normal b and a whose quotient stays
// far from the ends of the exponent range (the force pass divides an
// O(1) eV/A scalar by r in [1e-3, 10] A): a reciprocal estimate refined by
// two Newton-Raphson steps, the quotient q = a y, and one correction
// q + (a - b q) y with the residual exact in a fused multiply-add
// (Markstein's theorem for the last step).  Over that range it is the
// correctly rounded quotient (vcsgc_selftest_md_math checks it against the
// host's division); a zero a may come back with either sign.
__device__ __forceinline__ double div_md(double a, double b) {
  double y = __builtin_amdgcn_rcp(b);
  double t = __builtin_fma(-b, y, 1.0);
  y = __builtin_fma(y, t, y);
  t = __builtin_fma(-b, y, 1.0);
  y = __builtin_fma(y, t, y);
  const double q = a * y;
  const double e = __builtin_fma(-b, q, a);
  return __builtin_fma(e, y, q);
}

// The interpolant of a tabulated EAM function (a general embedded-atom
// potential, Introduction and Sec. III): knots at x = k h (k < n),
// coefficients (a0, a1, a2, a3) per interval of the
// cubic Hermite interpolant with central-difference knot slopes (one-sided
// at the ends), p = x / h by the rounded 1/h, k = floor(p) limited to
// [0, n - 2], t = p - k (outside the knots the end interval continues):
// value ((a3 t + a2) t + a1) t + a0, derivative ((3 a3 t + 2 a2) t + a1) / h.
__device__ __forceinline__ double spline_at(const double *c, int n, double x, double inv_h,
                                            double *der) {
  const double p = x * inv_h;
  const double top = (double)(n - 1);
  const double pc = p > 0.0 ? (p < top ? p : top) : 0.0;  // (a NaN p gives 0)
  int k = (int)pc;
  k = k > n - 2 ? n - 2 : k;
  const double t = p - (double)k;
  const double4 a = *(const double4 *)(c + 4 * (int64_t)k);
  if (der) *der = (((3.0 * a.w) * t + 2.0 * a.z) * t + a.y) * inv_h;
  return ((a.w * t + a.z) * t + a.y) * t + a.x;
}
// radial table k: 0, 1 = f_A, f_B; 2, 3, 4 = phi_AA, phi_AB, phi_BB
__device__ __forceinline__ const double *tab_radial(const PotD &p, int k) {
  return p.tc + 4 * (int64_t)k * (p.nr - 1);
}
__device__ __forceinline__ const double *tab_embed(const PotD &p, int s) {
  return p.tc + 4 * (5 * (int64_t)(p.nr - 1) + (int64_t)s * (p.nrho - 1));
}

// The potential's form for the helpers below: F = 0 analytic, 1 tabulated
// (fixed at compile time), -1 (the default) read from p.tab.
template <int F>
__device__ __forceinline__ bool pot_tab(const PotD &p) {
  return F < 0 ? p.tab != 0 : F == 1;
}

// f_X(r), f'_X(r), phi_XY(r), phi'_XY(r) for r < rc: the Finnis-Sinclair
// forms t_X d^2, (-2 t_X) d, (eps_XY d^2)(c0 + c1 r) and
// eps_XY ((-2 d)(c0 + c1 r) + c1 d^2) with d = rc - r, or the tables
template <int F = -1>
__device__ __forceinline__ double pot_f(const PotD &p, int s, double r) {
  if (pot_tab<F>(p)) return spline_at(tab_radial(p, s), p.nr, r, p.inv_dr, nullptr);
  return p.t[s] * pair_dd(p, r);
}
template <int F = -1>
__device__ __forceinline__ double pot_df(const PotD &p, int s, double r) {
  if (pot_tab<F>(p)) {
    double g;
    spline_at(tab_radial(p, s), p.nr, r, p.inv_dr, &g);
    return g;
  }
  return -2.0 * p.t[s] * (p.rc - r);
}
template <int F = -1>
__device__ __forceinline__ double pot_phi(const PotD &p, int a, int b, double r) {
  if (pot_tab<F>(p)) return spline_at(tab_radial(p, 2 + a + b), p.nr, r, p.inv_dr, nullptr);
  return p.eps[a + b] * pair_dd(p, r) * pair_g(p, r);
}
template <int F = -1>
__device__ __forceinline__ double pot_dphi(const PotD &p, int a, int b, double r) {
  if (pot_tab<F>(p)) {
    double g;
    spline_at(tab_radial(p, 2 + a + b), p.nr, r, p.inv_dr, &g);
    return g;
  }
  const double d = p.rc - r;
  return p.eps[a + b] * (-2.0 * d * (p.c0 + p.c1 * r) + p.c1 * (d * d));
}

// F_X(rho) = -A_X sqrt(max(rho, 0)) and F'_X(rho) (0 at rho <= 0), or the tables
template <int F = -1>
__device__ __forceinline__ double embed(const PotD &p, int s, double rho) {
  if (pot_tab<F>(p)) return spline_at(tab_embed(p, s), p.nrho, rho, p.inv_drho, nullptr);
  return -p.A[s] * sqrt(rho > 0.0 ? rho : 0.0);
}

template <int F = -1>
__device__ __forceinline__ double dembed(const PotD &p, int s, double rho) {
  if (pot_tab<F>(p)) {
    double g;
    spline_at(tab_embed(p, s), p.nrho, rho, p.inv_drho, &g);
    return g;
  }
  return rho > 0.0 ? -p.A[s] / (2.0 * sqrt(rho)) : 0.0;
}

// What flipping a site from species s to 1 - s changes, in the order every
// sweep path evaluates it (Eq. of the transmutation energy), for a
// neighbour entry at distance r < rc:
//   the neighbour's density shifts by f_{1-s}(r) - f_s(r);
//   the pair energy with a neighbour of species sj by
//     phi_{1-s,sj}(r) - phi_{s,sj}(r);
//   that neighbour's embedding energy by F_sj(rho_j + shift) - F_sj(rho_j);
//   the site's own embedding energy by F_{1-s}(rho_i) - F_s(rho_i).
// dU is the own term plus the in-order sums of the pair and embedding terms.
// (Finnis-Sinclair: with dd = (rc - r)^2, g = c0 + c1 r the shift is
// t_{1-s} dd - t_s dd and the pair change (eps_{1-s,sj} dd) g - (eps_{s,sj} dd) g.)
// the Finnis-Sinclair forms from dd and g formed beforehand
__device__ __forceinline__ double flip_rho_shift_fs(const PotD &p, int s, double dd) {
  return p.t[1 - s] * dd - p.t[s] * dd;
}
__device__ __forceinline__ double flip_pair_term_fs(const PotD &p, int s, int sj, double dd,
                                                    double g) {
  return p.eps[1 - s + sj] * dd * g - p.eps[s + sj] * dd * g;
}
template <int F = -1>
__device__ __forceinline__ double flip_rho_shift(const PotD &p, int s, double r) {
  if (pot_tab<F>(p)) return pot_f<F>(p, 1 - s, r) - pot_f<F>(p, s, r);
  return flip_rho_shift_fs(p, s, pair_dd(p, r));
}
template <int F = -1>
__device__ __forceinline__ double flip_pair_term(const PotD &p, int s, int sj, double r) {
  if (pot_tab<F>(p)) return pot_phi<F>(p, 1 - s, sj, r) - pot_phi<F>(p, s, sj, r);
  return flip_pair_term_fs(p, s, sj, pair_dd(p, r), pair_g(p, r));
}
template <int F = -1>
__device__ __forceinline__ double flip_embed_term(const PotD &p, int sj, double rj, double shift) {
  return embed<F>(p, sj, rj + shift) - embed<F>(p, sj, rj);
}
template <int F = -1>
__device__ __forceinline__ double flip_own_term(const PotD &p, int s, double ri) {
  return embed<F>(p, 1 - s, ri) - embed<F>(p, s, ri);
}

// The in-order sums of the (pair, embedding) terms of entries 0 .. m-1 held
// in LDS slots (written by the lanes of one wave, whose LDS accesses are
// performed in order): eight slots are read per round, so the reads do not
// wait on the additions.
__device__ __forceinline__ void sum_flip_terms(const double2 *grp, int m, double &pair,
                                               double &emb) {
  pair = 0.0;
  emb = 0.0;
  for (int k0 = 0; k0 < KMAX; k0 += 8) {
    if (k0 >= m) break;
    double2 q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] = grp[k0 + u];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < m) {
        pair += q[u].x;
        emb += q[u].y;
      }
  }
}

__device__ __forceinline__ double min_image(double d, double L) {
  const double h = 0.5 * L;
  if (d > h) return d - L;
  if (d < -h) return d + L;
  return d;
}

__device__ __forceinline__ double wrap_box(double u, double L) {
  if (u < 0.0) u += L;
  if (u >= L) u -= L;
  return u;
}

// cell coordinate along one axis: (int)(u / (L / nc)), clamped
__device__ __forceinline__ int cell_coord(double u, double L, int nc) {
  int c = (int)(u / (L / (double)nc));
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// Workgroups are dispatched to the eight XCDs round robin (workgroup b runs on
// XCD b mod 8), and each XCD has its own L2.  For gather kernels whose
// neighbouring atoms have neighbouring indices, this maps the launch so that
// each XCD gets one contiguous eighth of the logical blocks: the data shared
// by adjacent blocks then stays in one L2.  A bijection on [0, gridDim.x).
__device__ __forceinline__ int64_t xcd_block() {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

constexpr int SCAN_CHUNK = 1024;  // values per block of the cell-count scan

// Sums of N integer values over the block (exact, so the order is free):
// butterfly inside each wave, then the per-wave totals through LDS.  sh
// needs N * (BLOCK / 64) entries; contains two barriers (one with TAIL =
// false, when sh is not written again before the kernel ends), so every
// thread of the block must call it.
template <int N, bool TAIL = true>
__device__ __forceinline__ void block_sums(long long (&v)[N], long long *sh) {
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) sh[wv * N + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    long long t = 0;
    for (int q = 0; q < BLOCK / 64; ++q) t += sh[q * N + k];
    v[k] = t;
  }
  if (TAIL) __syncthreads();
}

inline int grid_for(int64_t n, int block = BLOCK) {
  int64_t g = (n + block - 1) / block;
  return (int)(g < 1 ? 1 : g);
}

}  // namespace vc

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
// Geometry of one replica of a batch (a single system is a batch of one).
// Atoms of replica r occupy [aoff, aoff + n) of the concatenated arrays.
struct RepHost {
  int64_t n = 0, aoff = 0;
  double box[3] = {0, 0, 0};
  int nc[3] = {0, 0, 0};     // link cells per dimension (a multiple of the colour period)
  int64_t ncells = 0;
  int64_t coff = 0;          // offset of the replica's cells in per-cell arrays
  int64_t cso = 0;           // offset of its (ncells + 1)-entry cell_start block
  int64_t S = 0;             // stages per sweep
  int64_t ncpc = 0, roff = 0;  // active cells per stage, offset in the record array
  int nb[3] = {0, 0, 0};     // search bins per dimension
  int64_t nbins = 0, boff = 0;
  int g0 = 0, G = 1;         // workgroups of the persistent sweep
};

struct vcsgc_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  int64_t n = 0;
  double box[3] = {0, 0, 0};
  double *x = nullptr, *y = nullptr, *z = nullptr;
  double *vx = nullptr, *vy = nullptr, *vz = nullptr;
  double *fx = nullptr, *fy = nullptr, *fz = nullptr;
  uint8_t *sp = nullptr;
  vc::PotD pot{};
  double skin = 0.3, r_dep = 7.2;
  std::vector<RepHost> reps;  // batch geometry (reps[0] mirrors the fields below)

  // link cells (edge >= r_dep, even count per dimension)
  int nc[3] = {0, 0, 0};
  int64_t ncells = 0, S = 0;
  int32_t *cell_count = nullptr, *cell_start = nullptr, *cell_atoms = nullptr,
          *cell_fill = nullptr;
  int32_t *scan_tmp = nullptr;  // chunk sums of the cell-count scan
  double *snap = nullptr;       // x, y, z, vx, vy, vz at the start of an MD call (6 n)
  // Nose-Hoover thermostat of md_verlet_step (off while nvt_T == 0): device
  // state nvt = (xi, eta, K, s1, s2, xi and eta at the call's start), per-chunk
  // kinetic-energy sums nvt_part [ceil(n / 256)]
  double nvt_T = 0.0, nvt_tau = 0.0;
  double *nvt = nullptr, *nvt_part = nullptr;
  double *tab_coef = nullptr;  // tabulated potential's coefficients (PotD::tc)
  // conjugate-gradient relaxation: direction d, start positions x0 and
  // forces f0 of the line search (3 n each), chunk values, totals
  double *cg = nullptr;
  // grown domains (single system): cells of edge >= max(grow_edge, 2 r_dep),
  // per (cell c, corner k) at q = 8 c + k the domain's atoms g_list and
  // inclusive weight sums g_cum from g_start[q] to g_start[q + 1]; g_cnt the
  // counts of the build
  bool grown = false;
  double grow_edge = 0.0;
  int32_t *g_start = nullptr, *g_list = nullptr, *g_cum = nullptr, *g_cnt = nullptr;
  // Nose-Hoover barostat of md_verlet_step (off while npt_tau == 0): external
  // pressure (eV/A^3), coupling time, momentum pe (eV fs) and the last
  // virial (eV), host-side; npt_part: chunk values [2 ceil(n / 256) + 8];
  // box_build: the box at the last MD-list build; nb_max and bin_edge: the
  // search-bin grid of creation and its minimum edge
  double npt_p = 0.0, npt_tau = 0.0, npt_pe = 0.0, npt_vir = 0.0;
  double *npt_part = nullptr;
  double box_build[3] = {0, 0, 0};
  int nb_max[3] = {0, 0, 0};
  double bin_edge = 0.0;

  // search bins for neighbour lists: edge >= rc + skin, fixed capacity per bin
  int nb[3] = {0, 0, 0};
  int64_t nbins = 0;
  int bmax = 16;
  int32_t *bin_count = nullptr, *bin_atoms = nullptr;
  double4 *bin_pos = nullptr;  // (x, y, z, index) per bin slot (single-system contexts)
  int32_t *sites = nullptr;  // trial sites of one sweep, S x (cells / 8) (single-system)
  double *site_lnu = nullptr;  // ln u of those trials
  double *stage_lnug = nullptr;  // ln u_g of the sweep's stages
  int local_steps = 1;          // trials per active cell per stage (local chain length)
  int32_t *u_site = nullptr, *u_j = nullptr;  // undo log of a stage of local chains
  double *u_rho = nullptr, *u_v = nullptr;
  void *stage_graph = nullptr;  // per-stage sweep replayed as a HIP graph (sweep.hip)
  int64_t nbins_total = 0;     // bins of all replicas

  // r < rc list, row-major rows [i * KMAX + k]: neighbour and r
  int32_t *mc_j = nullptr;
  double *mc_r = nullptr;  // r of each r < rc entry
  uint8_t *mc_cnt = nullptr;
  // r < 4.41 A descriptor list (row-major: neighbour, distance), when enabled
  bool desc = false;
  int32_t *d_j = nullptr;
  double *d_r = nullptr;
  uint8_t *d_cnt = nullptr;
  // surrogate delayed acceptance and sample logging
  const struct vcsgc_mlp *mlp = nullptr;
  int da_mode = 0;  // 0 off, 1 network, 2 perfect, 3 zero
  double *smp_desc = nullptr, *smp_de = nullptr;
  int64_t smp_cap = 0, smp_stride = 1;
  double *dalog = nullptr;
  int64_t dacap = 0;
  // r < rc + skin list for MD, ascending neighbour index, column-major
  // [k * n + i] (md_rows: the search's unsorted row-major rows
  // [i * KMAX + k], sorted into md_j by the finishing pass); and positions
  // at its build
  int32_t *md_j = nullptr, *md_rows = nullptr;
  uint8_t *md_cnt = nullptr;
  double *xr = nullptr, *yr = nullptr, *zr = nullptr;

  double4 *ps4 = nullptr;  // MD: (x, y, z, species) packed for neighbour gathers
  double4 *pf4 = nullptr;  // MD: (x, y, z, F') written by the density pass
  double *rho = nullptr;                        // density cache of the sweep
  double *rho_f = nullptr;  // fresh density (energy, MD)
  double *eatom = nullptr, *red = nullptr;
  int32_t *rec = nullptr;  // per active cell: locally accepted site or -1
  // fused stage pipeline (single system, one trial per cell and stage): site
  // tables of two sweeps [w & 1][s][t], ln u of their local tests and of the
  // stages' global tests, and records and trial-block sums of two stages
  int32_t *m_sites = nullptr;
  double *m_lnu = nullptr, *m_lnug = nullptr;
  double *m_lnu2 = nullptr;  // ln u of the delayed-acceptance second stage
  int32_t *m_rec = nullptr;
  long long *m_part = nullptr;
  int32_t *s_rec = nullptr;    // batched pipeline: [2][SPEC_MAX][ncpc] records
  long long *s_part = nullptr; // [2][SPEC_MAX][trial blocks][3] block counts
  // pinned copy of the device state, read by the pipeline's progress checks;
  // h_state_final: the last check saw the call's end (statistics included)
  vc::DevState *h_state = nullptr;
  bool h_state_final = false;
  double m_acc_rate = 0.05;             // accepted stages per stage, last call
  double m_spec_rate = 0.0;             // batched pipeline: kernels per stage, last call
  void *pipe_graph = nullptr;           // graphs of pipeline kernels
  long long *part = nullptr;  // per trial block: trials, local accepts, sum dn, near ties
  int64_t npart = 0;
  vc::DevState *ds = nullptr;

  bool mc_valid = false, md_valid = false;
  // rho_f holds the densities at the current positions and species (set by
  // the MD and energy paths, cleared by anything that changes species)
  bool rho_f_fresh = false;
  uint64_t w = 0;  // sweep counter
  // colour period per axis: 2 (eight colours, cells of edge >= r_dep) or 3
  // (27 colours, cells of edge >= r_dep / 2); ncol = per^3
  int per = 2, ncol = 8;
  uint64_t last_seed = 0;  // seed of the last sweep call (checkpoint state)
  int kmax_used = 0;
  bool mc_stats_stale = false;  // the r < rc list's row statistics not yet taken
  int64_t md_rebuilds = 0;

  double *tlog = nullptr, *slog = nullptr;
  int64_t tcap = 0, scap = 0;

  // optional per-kernel timing with HIP events on the context's stream
  uint32_t tmask = 0;
  int32_t t_every = 1;                          // time one launch in t_every
  int64_t kt_seen[VCSGC_KT_CLASSES] = {};       // launches per class since enabling
  struct Pending {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pending> ev_pending;
  double kt_ms[VCSGC_KT_CLASSES] = {};
  int64_t kt_n[VCSGC_KT_CLASSES] = {};

  // persistent batched sweep
  void *d_reps = nullptr;     // per-replica parameters (device)
  void *h_reps = nullptr;     // pinned staging buffer for them
  void *d_rs = nullptr;       // per-replica chain state and counters
  int32_t *d_wg_rep = nullptr;  // workgroup -> replica
  int grid_total = 0;
  int trials_per_group = 1;   // tiling: active cells per trial group and stage
  int strategy = 0;           // 0: persistent (graph), 1: persistent (direct), 2: per-stage
  unsigned int spin_limit = 1u << 24;
  hipEvent_t stage_ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool graph_coop = false;
  double *graph_args_tlog = nullptr, *graph_args_slog = nullptr;
  alignas(16) unsigned char graph_args_storage[512];  // kernel arguments of the graph node

  std::string err;
  bool sticky = false;
};

// internal host entry points implemented across the .hip files
namespace vc {
// Kernel timing: tstart records a start event when the class is enabled and
// returns a handle (or -1); tstop records the matching end event.
int tstart(vcsgc_ctx *c, int cls);
void tstop(vcsgc_ctx *c, int h);

// Stages per sweep of a single-system context: 8 ceil(ceil(N / N_cells) / k)
// for local chains of k trials (8 ceil(N / N_cells) for k = 1).
// active cells of a stage: the cells of one colour, or every cell with
// grown domains (one trial in the stage's domain of each)
inline int64_t active_cells(const vcsgc_ctx *c) {
  return c->grown ? c->ncells : c->ncells / c->ncol;
}

inline int64_t stages_per_sweep(const vcsgc_ctx *c) {
  const int64_t m = (c->n + c->ncells - 1) / c->ncells;
  const int64_t per_cell = (m + c->local_steps - 1) / c->local_steps;
  return c->grown ? per_cell : (int64_t)c->ncol * per_cell;
}

hipError_t launch_bin_cells(vcsgc_ctx *c, const RepHost &r);
hipError_t launch_bin_search(vcsgc_ctx *c, const RepHost &r);
hipError_t launch_build_mc_list(vcsgc_ctx *c, const RepHost &r);
hipError_t launch_build_md_list(vcsgc_ctx *c);
hipError_t launch_md_rebuild_cond(vcsgc_ctx *c, int par);
bool md_rebuild_on_device(const vcsgc_ctx *c);
hipError_t launch_mc_row_stats(vcsgc_ctx *c);
hipError_t launch_build_desc_list(vcsgc_ctx *c, const RepHost &r);
hipError_t launch_descriptors(vcsgc_ctx *c, const int32_t *sites, int64_t n, int flip,
                              double *out);
hipError_t launch_density_mc(vcsgc_ctx *c);
hipError_t launch_mc_from_md(vcsgc_ctx *c);
void free_stage_graph(vcsgc_ctx *c);
void free_pipe_graph(vcsgc_ctx *c);
hipError_t launch_energy(vcsgc_ctx *c);  // fresh rho (MD list) + per-atom energies
hipError_t launch_forces(vcsgc_ctx *c);  // fresh rho, F', forces (MD list)
hipError_t launch_validate(vcsgc_ctx *c, const RepHost &r);
hipError_t launch_reduce_sum(vcsgc_ctx *c, const double *v, int64_t n, double *out_dev);
hipError_t launch_sweeps(vcsgc_ctx *c, double dmu0, double kappa, double cbar, double T,
                         int64_t n_sweeps, uint64_t seed);
hipError_t launch_pack(vcsgc_ctx *c);
hipError_t launch_kick_drift(vcsgc_ctx *c, double dt, bool kick_first, int par);
// density and force passes whose forces go straight into the next step's
// kick and drift (the forces are not stored)
hipError_t launch_forces_kick_drift(vcsgc_ctx *c, double dt, bool kick_first, int par);
hipError_t launch_kick(vcsgc_ctx *c, double dt);
// Nose-Hoover NVT (md.hip)
hipError_t launch_nvt_ke(vcsgc_ctx *c, double dt, bool closing_kick);
hipError_t launch_nvt_thermo(vcsgc_ctx *c, double dt, int mode);  // bit 0: end half, 1: start half
hipError_t launch_nvt_kick_drift(vcsgc_ctx *c, double dt, int par);
hipError_t launch_nvt_scale(vcsgc_ctx *c);
// conjugate-gradient relaxation: trial positions x = wrap(x0 + a d); the
// totals (mode 0: F . u and max |u_i|^2; mode 1: F . F and F . u) into
// out[0..1] through part [2 ceil(n / BLOCK)]; d = F or d = F + b d
hipError_t launch_cg_move(vcsgc_ctx *c, const double *x0, const double *d, double a);
hipError_t launch_cg_totals(vcsgc_ctx *c, int mode, const double *u, double *part, double *out);
hipError_t launch_cg_dir(vcsgc_ctx *c, double *d, double b, bool copy);
// NPT: forces with the per-atom virial terms w; the step's scalings, kick
// and drift (launch_npt_kick_drift); the closing kick (if kick) with the
// totals of m v^2 and w into out[0..1] through part [2 ceil(n / BLOCK)];
// v *= s
hipError_t launch_forces_virial(vcsgc_ctx *c, double *w);
hipError_t launch_npt_kick_drift(vcsgc_ctx *c, double f1, double f2, double cv, double h,
                                 double dt, double q, const double lam[3], double thr);
hipError_t launch_npt_sums(vcsgc_ctx *c, bool kick, double cv, double h, const double *w,
                           double *part, double *out);
hipError_t launch_scale_v(vcsgc_ctx *c, double s);
hipError_t launch_sqrt(const double *in, double *out, int64_t n, hipStream_t s);
hipError_t launch_md_math(const double *a, const double *b, double *sq, double *q, int64_t n,
                          hipStream_t s);
// persistent sweep (persist.hip)
int persist_block();
int persist_groups();
size_t repd_size();
size_t repstate_size();
hipError_t persist_max_blocks(int *per_cu, bool tab);
hipError_t persist_stage_params(vcsgc_ctx *c, const double *dmu0, const double *kappa,
                                const double *cbar, const double *T, int64_t n_sweeps,
                                uint64_t seed);
hipError_t launch_persistent(vcsgc_ctx *c, bool use_graph);
hipError_t persist_read_stats(vcsgc_ctx *c, vcsgc_stats *out, int *err);
hipError_t persist_count(vcsgc_ctx *c);
hipError_t persist_sync_nb_to_stage(vcsgc_ctx *c);
hipError_t persist_sync_nb_from_stage(vcsgc_ctx *c);
}  // namespace vc
