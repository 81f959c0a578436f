// Parallel VC-SGC sweep (Sec. III.B.2), one stage at a time:
//   k_trial  : every cell of the stage's colour draws a site, computes the
//              transmutation energy dU from the density cache and applies
//              the local factor min{1, exp[-beta (dU + dmu0 dn)]}
//              (Eq. trans_vcsgc_par1); the block sums of dn over local
//              accepts go to a per-stage accumulator;
//   k_commit : every thread evaluates the same global factor
//              min{1, exp[-beta (kappa/N) dn_tot (dn_tot + 2 (n - N cbar))]}
//              (Eq. trans_vcsgc_par2) and, if it passes, commits the flips of
//              its cell: species, density cache rho_j += delta_j of every
//              neighbour, and the velocity rescaling.
// Cells of one colour are at least one cell edge (>= 2 rc) apart, so their
// energy changes are independent and every rho_j has at most one writer per
// stage.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "mlp_device.hpp"

namespace vc {

struct SweepArgs {
  int64_t n;
  int n0, n1, n2;
  int64_t ncpc;  // cells per colour
  int per, ncol;  // colour period per axis, colours
  int64_t S;
  double beta, dmu0, kN, ncbar;
  uint64_t seed, replica;
  PotD p;
  const int32_t *cstart, *catoms;
  const int32_t *nj;
  const double *nr;  // r of each r < rc entry
  const uint8_t *cnt;
  uint8_t *sp;
  double *rho;
  double *vx, *vy, *vz;
  int32_t *rec;
  long long *part;  // [nblocks][4] partial sums of the trial kernel
  int nblk;
  DevState *ds;
  double *tlog;
  int64_t tcap;
  double *slog;
  int64_t scap;
  // descriptor list and surrogate
  const int32_t *dj;
  const double *dr;
  const uint8_t *dcnt;
  MlpDev md;
  int da_mode;
  double *dalog;
  int64_t dacap;
  // training-sample log: every stride-th trial's (descriptor, dU)
  double *smp_desc, *smp_de;
  int64_t smp_cap, smp_stride;
  // sites of every stage of the current sweep, [s][t] (-1: empty cell), and
  // ln u of their local tests
  int32_t *sites;
  double *site_lnu;
  double *site_lnu2;  // DA second-stage ln u per site-table entry (fused pipeline only)
  double *stage_lnug;  // ln u_g of every stage's global test
  // graph replay: the sweep counter is read from here instead of the
  // kernel argument (advanced by k_next_sweep at the end of each sweep)
  const unsigned long long *wdev;
  // local chains of K > 1 trials per active cell per stage: per (cell, step)
  // the site flipped (-1: none), the old velocity, and per neighbour entry
  // the index and old density, to undo a rejected stage
  int K;
  int32_t *u_site, *u_j;
  double *u_rho, *u_v;
  // batched pipeline: stages per batch (at most SPEC_MAX and S / 2)
  int D;
  // grown domains: every cell active, the stage's colour is the corner of
  // the domain drawn in; per (cell, corner) the domain's atoms and weight sums
  int grown;
  const int32_t *gstart, *glist, *gcum;
};

__device__ __forceinline__ uint64_t sweep_of(const SweepArgs &a, uint64_t w) {
  return a.wdev ? (uint64_t)*a.wdev : w;
}

// Lanes per trial: lane k of a group handles neighbour entries k and k + TL.
constexpr int TL = 16;
// lanes per trial in the batched pipeline's plain trials (four entries each):
// twice the trials in flight per wave, which that throughput-bound kernel
// needs (measured: 16 lanes 7% slower per sweep, 4 lanes within 1%)
constexpr int TL_BATCH = 8;
static_assert(KMAX <= 2 * TL, "a trial group covers at most 2*TL neighbours");

// What one lane of a group of L lanes reads for the trial at site i: the
// site's species, density and row length, and its neighbour entries
// k = lane + h L with their species and densities.  Entries k < 16 always lie
// inside the KMAX-entry row, so their row reads are issued together with
// those of the site (unused entries beyond the row length are never
// dereferenced); rows longer than 16 entries are rare.
template <int L>
struct TrialInT {
  static constexpr int H = KMAX / L;
  int s, m;
  double ri;
  int32_t j[H];
  // Finnis-Sinclair: dd = (rc - r)^2 and g = c0 + c1 r, formed while the
  // gathers are in flight; tabulated potential: dd holds r
  double dd[H], g[H], rj[H];
  int sj[H];
};
typedef TrialInT<TL> TrialIn;

// F: the potential's form (0 analytic, 1 tabulated, -1 read from a.p.tab)
template <int L, int F>
__device__ __forceinline__ void load_trial(const SweepArgs &a, int64_t i, int lane,
                                           TrialInT<L> &v) {
  constexpr int H = KMAX / L;
  v.s = a.sp[i];
  v.ri = a.rho[i];
  v.m = a.cnt[i];
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int k = lane + h * L;
    v.j[h] = 0;
    v.dd[h] = v.g[h] = 0.0;
    v.sj[h] = 0;
    v.rj[h] = 0.0;
    if ((h + 1) * L <= 16 || k < v.m) {
      const int64_t e = i * KMAX + k;
      v.j[h] = a.nj[e];
      const double r = a.nr[e];
      if (pot_tab<F>(a.p)) {
        v.dd[h] = r;
      } else {
        v.dd[h] = pair_dd(a.p, r);
        v.g[h] = pair_g(a.p, r);
      }
    }
  }
#pragma unroll
  for (int h = 0; h < H; ++h)
    if (lane + h * L < v.m) {
      v.sj[h] = a.sp[v.j[h]];
      v.rj[h] = a.rho[v.j[h]];
    }
}

// Per trial group, the (pair, embedding) terms of its KMAX entries in LDS.
typedef double2 GroupTerms[KMAX];

// dU of s_i -> 1 - s_i, evaluated by the L lanes of one group:
//   (F_{s'}(rho_i) - F_s(rho_i)) + sum_j [phi_{s's_j}(r) - phi_{s s_j}(r)]
//   + sum_j [F_{s_j}(rho_j + (f_{s'}(r) - f_s(r))) - F_{s_j}(rho_j)]
// Each lane computes the terms of its entries and stores them in the group's
// LDS slots; every lane then forms both sums in ascending entry order from
// there (the rounding of the sequential sums; the slot reads do not wait on
// the additions, so there is one LDS round trip per eight entries rather than
// one per entry).  A group is L lanes of one wave, whose LDS accesses are
// performed in order.  Every lane of the group returns the same value.
template <int L, int F>
__device__ __forceinline__ double delta_u_of(const SweepArgs &a, const TrialInT<L> &v, int lane,
                                             double2 *grp) {
  constexpr int H = KMAX / L;
  const int s = v.s;
  const int m = v.m;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int k = lane + h * L;
    double tp = 0.0, te = 0.0;
    if (k < m) {
      const int sj = v.sj[h];
      const double rj = v.rj[h];
      if (pot_tab<F>(a.p)) {
        const double r = v.dd[h];
        tp = flip_pair_term<1>(a.p, s, sj, r);
        te = flip_embed_term<1>(a.p, sj, rj, flip_rho_shift<1>(a.p, s, r));
      } else {
        const double dd = v.dd[h], g = v.g[h];
        tp = flip_pair_term_fs(a.p, s, sj, dd, g);
        te = flip_embed_term<0>(a.p, sj, rj, flip_rho_shift_fs(a.p, s, dd));
      }
    }
    grp[k] = make_double2(tp, te);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // two independent in-order chains
  double pair, emb;
  sum_flip_terms(grp, m, pair, emb);
  const double own = flip_own_term<F>(a.p, s, v.ri);
  return own + pair + emb;
}

template <int F = -1>
__device__ __forceinline__ double delta_u_group(const SweepArgs &a, int64_t i, int lane,
                                                double2 *grp) {
  TrialIn v;
  load_trial<TL, F>(a, i, lane, v);
  return delta_u_of<TL, F>(a, v, lane, grp);
}

// Descriptor of site i (or of the state with s_i flipped), by the TL lanes
// of a group: [s_i, nB1, nB2, nB3, n1, n2, n3, rho1, rho2, rho3] over the
// shells r < 2.68, [2.68, 3.46), [3.46, 4.41) A; the shell sums run in
// ascending neighbour order.  In the flipped state every neighbour within rc
// has rho_j + (f_{s'}(r) - f_s(r)).  All lanes return the same values.
__device__ __forceinline__ void descriptor_group(const SweepArgs &a, int64_t i, int lane,
                                                 bool flip, double out[10]) {
  const int s = a.sp[i], s1 = 1 - s;
  const int m = a.dcnt[i];
  int shl[2] = {-1, -1}, bj[2] = {0, 0};
  double rj[2] = {0.0, 0.0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = lane + h * TL;
    if (k < m) {
      const int64_t e = i * KMAX + k;
      const int32_t j = a.dj[e];
      const double r = a.dr[e];
      shl[h] = r < 2.68 ? 0 : (r < 3.46 ? 1 : (r < DESC_CUT ? 2 : -1));
      bj[h] = a.sp[j];
      double rho = a.rho[j];
      if (flip && r < a.p.rc) rho = rho + flip_rho_shift(a.p, s, r);
      rj[h] = rho;
    }
  }
  double cnt[3] = {0.0, 0.0, 0.0}, cb[3] = {0.0, 0.0, 0.0}, rs[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < m; ++k) {
    const int h = k / TL;
    const int sk = __shfl(h ? shl[1] : shl[0], k % TL, TL);
    const int bk = __shfl(h ? bj[1] : bj[0], k % TL, TL);
    const double rk = __shfl(h ? rj[1] : rj[0], k % TL, TL);
    if (sk >= 0) {
      cnt[sk] += 1.0;
      cb[sk] += (double)bk;
      rs[sk] += rk;
    }
  }
  out[0] = (double)(flip ? s1 : s);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    out[1 + k] = cb[k];
    out[4 + k] = cnt[k];
    out[7 + k] = cnt[k] > 0.0 ? rs[k] / cnt[k] : 0.0;
  }
}

// Forward and flipped descriptors of site i and dU of its transmutation from
// one gather of the r < 4.41 A list, by the TL lanes of a group.  The shell
// sums are those of descriptor_group; dU is formed from the entries with
// r < rc exactly as delta_u_group forms it from the r < rc list (the same
// entries in the same order, the same (rc - r)^2 and c0 + c1 r from the same
// r), so both give the same value.  Each lane reads both of its row entries
// with the site (inside the KMAX-entry row), computes their terms and stores
// them in the group's LDS slots; every lane then forms all sums in ascending
// entry order from there, eight entries per LDS round trip.  All lanes
// return the same values.
struct DescTerm {
  double rj, rjf, tp, te;
  int code;  // shell + 1 (0: outside), B flag << 2, r < rc flag << 3
};
typedef DescTerm DescSlots[KMAX];

__device__ __forceinline__ void desc_du_group(const SweepArgs &a, int64_t i, int lane,
                                              double fwd[10], double flp[10], double &du,
                                              DescTerm *slot) {
  const int s = a.sp[i], s1 = 1 - s;
  const double ri = a.rho[i];
  const int m = a.dcnt[i];
  int32_t jr[2];
  double rr[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t e = i * KMAX + lane + h * TL;
    jr[h] = a.dj[e];
    rr[h] = a.dr[e];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = lane + h * TL;
    DescTerm q;
    q.rj = q.rjf = q.tp = q.te = 0.0;
    q.code = 0;
    if (k < m) {
      const int32_t j = jr[h];
      const double r = rr[h];
      const int shl = r < 2.68 ? 0 : (r < 3.46 ? 1 : (r < DESC_CUT ? 2 : -1));
      const int sj = a.sp[j];
      const double rho = a.rho[j];
      q.rj = rho;
      q.rjf = rho;
      int in = 0;
      if (r < a.p.rc) {
        const double delta = flip_rho_shift(a.p, s, r);
        q.rjf = rho + delta;
        q.tp = flip_pair_term(a.p, s, sj, r);
        q.te = flip_embed_term(a.p, sj, rho, delta);
        in = 1;
      }
      q.code = (shl + 1) | (sj << 2) | (in << 3);
    }
    slot[k] = q;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double cnt[3] = {0.0, 0.0, 0.0}, cb[3] = {0.0, 0.0, 0.0};
  double rs[3] = {0.0, 0.0, 0.0}, rsf[3] = {0.0, 0.0, 0.0};
  double pair = 0.0, emb = 0.0;
  for (int k0 = 0; k0 < KMAX; k0 += 8) {
    if (k0 >= m) break;
    DescTerm q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] = slot[k0 + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (k0 + u >= m) break;
      const int ck = q[u].code;
      const int sk = (ck & 3) - 1;
#pragma unroll
      for (int sh = 0; sh < 3; ++sh)
        if (sk == sh) {
          cnt[sh] += 1.0;
          cb[sh] += (double)((ck >> 2) & 1);
          rs[sh] += q[u].rj;
          rsf[sh] += q[u].rjf;
        }
      if (ck & 8) {
        pair += q[u].tp;
        emb += q[u].te;
      }
    }
  }
  fwd[0] = (double)s;
  flp[0] = (double)s1;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    fwd[1 + k] = flp[1 + k] = cb[k];
    fwd[4 + k] = flp[4 + k] = cnt[k];
    fwd[7 + k] = cnt[k] > 0.0 ? rs[k] / cnt[k] : 0.0;
    flp[7 + k] = cnt[k] > 0.0 ? rsf[k] / cnt[k] : 0.0;
  }
  const double own = flip_own_term(a.p, s, ri);
  du = own + pair + emb;
}

// Grown domains: the site of draw w0 in domain (cell, corner) q, the first
// atom whose inclusive weight sum exceeds floor(w0 W / 2^64), W the
// domain's total weight (the domain holds at least one atom).
__device__ __forceinline__ int32_t grown_pick(const SweepArgs &a, int64_t q, uint64_t w0) {
  int32_t lo = a.gstart[q], hi = a.gstart[q + 1] - 1;
  const uint32_t r = draw_index(w0, (uint32_t)a.gcum[hi]);
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if ((uint32_t)a.gcum[mid] > r)
      hi = mid;
    else
      lo = mid + 1;
  }
  return a.glist[lo];
}

// Cell of active-cell index t (< ncpc < 2^31) in a stage of the given colour:
// cell (per ia + colour % per, per ib + (colour / per) % per, per ic + colour / per^2).
__device__ __forceinline__ int64_t colour_cell(const SweepArgs &a, int colour, int64_t t) {
  if (a.grown) return t;  // every cell is active
  const uint32_t P = (uint32_t)a.per;
  const uint32_t hx = (uint32_t)a.n0 / P, hy = (uint32_t)a.n1 / P;
  const uint32_t u = (uint32_t)t, q = u / hx, ia = u - q * hx, ic = q / hy, ib = q - ic * hy;
  const uint32_t k = (uint32_t)colour, k1 = k / P;
  const int64_t cx = (int64_t)(P * ia + (k - k1 * P)), cy = (int64_t)(P * ib + (k1 % P)),
                cz = (int64_t)(P * ic + k1 / P);
  return cx + (int64_t)a.n0 * (cy + (int64_t)a.n1 * cz);
}

__global__ void __launch_bounds__(BLOCK) k_init(DevState *ds) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ds->n_b[0] = ds->n_b_cur;
    ds->dn[0] = 0;
    ds->nrec[0] = 0;
    ds->trials = ds->local_acc = ds->stages = ds->stage_acc = ds->flips = ds->near_ties = 0;
    ds->stage1_pass = 0;
    ds->sum_n = 0.0;
    ds->sum_n2 = 0.0;
  }
}

__global__ void k_set_sweep(DevState *ds, unsigned long long w) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ds->wcur = w;
}

__global__ void k_next_sweep(DevState *ds) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ds->wcur += 1ull;
}

// The trials of a whole sweep: for stage s and active cell t, the site drawn
// from the cell's atoms, or -1 for an empty cell, and ln u of the trial's
// local test (the same draws, in the same precision, as a per-trial
// evaluation).  The cell lists do not change during a sweep.
__global__ void __launch_bounds__(BLOCK) k_sites(SweepArgs a, uint64_t w_arg) {
  const uint64_t w = sweep_of(a, w_arg);
  const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (q >= a.S * a.ncpc) return;
  const int64_t s = q / a.ncpc, t = q - s * a.ncpc;
  const U4 g = philox(a.seed, a.replica, w, (uint64_t)s, 0, 0);
  if (t == 0) a.stage_lnug[s] = log(unit_open(g.v[1]));
  const int colour = stage_colour(g.v[0], a.ncol);
  const int64_t cell = colour_cell(a, colour, t);
  const int64_t gq = 8 * cell + colour;
  const int32_t st = a.grown ? a.gstart[gq] : a.cstart[cell];
  const uint32_t m = (uint32_t)((a.grown ? a.gstart[gq + 1] : a.cstart[cell + 1]) - st);
  // trial k of the cell's chain: Philox(key, (w, s, cell, 1 + k))
  for (int k = 0; k < a.K; ++k) {
    int32_t site = -1;
    double lnu = 0.0;
    if (m > 0) {
      const U4 r = philox(a.seed, a.replica, w, (uint64_t)s, (uint64_t)cell, 1 + (uint64_t)k);
      site = a.grown ? grown_pick(a, gq, r.v[0]) : a.catoms[st + draw_index(r.v[0], m)];
      lnu = log(unit_open(r.v[1]));
    }
    a.sites[q * a.K + k] = site;
    a.site_lnu[q * a.K + k] = lnu;
  }
}

// one group of TL lanes per active cell; F: the potential's form (0
// analytic, 1 tabulated)
template <int F>
__global__ void __launch_bounds__(BLOCK) k_trial(SweepArgs a, uint64_t w_arg, int64_t s, int par) {
  const uint64_t w = sweep_of(a, w_arg);
  __shared__ long long sh[BLOCK];
  __shared__ GroupTerms terms[BLOCK / TL];
  const int lane = threadIdx.x % TL;
  const int64_t t = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / TL;
  long long valid = 0, acc = 0, dn_acc = 0, tie = 0;
  if (t < a.ncpc) {
    const int32_t si = a.sites[s * a.ncpc + t];
    const double lnu = a.site_lnu[s * a.ncpc + t];
    int32_t site = -1;
    if (si >= 0) {
      const int64_t i = si;
      const double du = delta_u_group<F>(a, i, lane, terms[threadIdx.x / TL]);
      if (a.smp_cap > 0 && ((int64_t)(w * (uint64_t)a.S + (uint64_t)s) * a.ncpc + t) % a.smp_stride == 0) {
        double d[10];
        descriptor_group(a, i, lane, false, d);
        if (lane == 0) {
          const unsigned long long idx = atomicAdd(&a.ds->smp_n, 1ull);
          if ((int64_t)idx < a.smp_cap) {
            for (int k = 0; k < 10; ++k) a.smp_desc[10 * idx + k] = d[k];
            a.smp_de[idx] = du;
          }
        }
      }
      if (lane == 0) {
        const int dn = 1 - 2 * (int)a.sp[i];
        const double xl = a.beta * (du + a.dmu0 * (double)dn);
        const double margin = lnu + xl;
        const bool ok = lnu < -xl;
        valid = 1;
        tie = fabs(margin) < TIE;
        if (ok) {
          acc = 1;
          dn_acc = dn;
          site = (int32_t)i;
        }
        if (a.tlog) {
          const unsigned long long idx = atomicAdd(&a.ds->tlog_n, 1ull);
          if ((int64_t)idx < a.tcap) {
            const U4 g = philox(a.seed, a.replica, w, (uint64_t)s, 0, 0);
            double *L = a.tlog + 8 * idx;
            L[0] = (double)w;
            L[1] = (double)s;
            L[2] = (double)colour_cell(a, stage_colour(g.v[0], a.ncol), t);
            L[3] = (double)i;
            L[4] = (double)dn;
            L[5] = ok ? 1.0 : 0.0;
            L[6] = du;
            L[7] = margin;
          }
        }
      }
    }
    if (lane == 0) a.rec[t] = site;
  }
  // per-block partial sums (no atomics): the commit kernel reduces them
  long long v4[4] = {valid, acc, dn_acc, tie};
  block_sums<4>(v4, sh);
  if (threadIdx.x == 0) {
    long long *P = a.part + NPART * blockIdx.x;
    P[0] = v4[0];
    P[1] = v4[1];
    P[2] = v4[2];
    P[3] = v4[3];
    P[4] = v4[0];  // no surrogate stage: every trial goes to the exact test
  }
}

// Local chains (K > 1): the TL lanes of a group run the K trials of their
// cell in order, each on the state left by the previous ones.  An accepted
// trial is applied at once (densities of the neighbours, species, velocity),
// with the overwritten values kept in the undo log; the block synchronizes
// between trials so that every lane sees the group's updates.  Chains of
// different active cells touch disjoint atoms (same-colour cells are a cell
// edge >= 2 rc apart), so they run side by side.
template <int F>
__global__ void __launch_bounds__(BLOCK) k_trial_chain(SweepArgs a, uint64_t w_arg, int64_t s,
                                                       int par) {
  const uint64_t w = sweep_of(a, w_arg);
  __shared__ long long sh[BLOCK];
  __shared__ GroupTerms terms[BLOCK / TL];
  const int lane = threadIdx.x % TL;
  const int64_t t = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / TL;
  const bool live = t < a.ncpc;
  long long valid = 0, acc = 0, dn_acc = 0, tie = 0;
  for (int k = 0; k < a.K; ++k) {
    const int64_t q = (s * a.ncpc + t) * a.K + k;  // the sweep's table
    const int64_t uq = t * a.K + k;                // this stage's undo log
    const int32_t si = live ? a.sites[q] : -1;
    int32_t flipped = -1;
    if (si >= 0) {
      const int64_t i = si;
      const double lnu = a.site_lnu[q];
      const double du = delta_u_group<F>(a, i, lane, terms[threadIdx.x / TL]);
      const int s0 = a.sp[i];
      const int dn = 1 - 2 * s0;
      const double xl = a.beta * (du + a.dmu0 * (double)dn);
      const double margin = lnu + xl;
      const bool ok = lnu < -xl;  // the same on every lane of the group
      if (lane == 0) {
        valid += 1;
        tie += fabs(margin) < TIE ? 1 : 0;
        if (ok) {
          acc += 1;
          dn_acc += dn;
        }
        if (a.tlog) {
          const unsigned long long idx = atomicAdd(&a.ds->tlog_n, 1ull);
          if ((int64_t)idx < a.tcap) {
            const U4 g = philox(a.seed, a.replica, w, (uint64_t)s, 0, 0);
            double *L = a.tlog + 8 * idx;
            L[0] = (double)w;
            L[1] = (double)s;
            L[2] = (double)(colour_cell(a, stage_colour(g.v[0], a.ncol), t) * a.K + k);
            L[3] = (double)i;
            L[4] = (double)dn;
            L[5] = ok ? 1.0 : 0.0;
            L[6] = du;
            L[7] = margin;
          }
        }
      }
      if (ok) {
        const int s1 = 1 - s0;
        const int m = a.cnt[i];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int e = lane + h * TL;
          if (e < m) {
            const int64_t ee = i * KMAX + e;
            const int32_t j = a.nj[ee];
            const double r = a.nr[ee];
            const double old = a.rho[j];
            a.u_j[uq * KMAX + e] = j;
            a.u_rho[uq * KMAX + e] = old;
            a.rho[j] = old + flip_rho_shift<F>(a.p, s0, r);
          }
        }
        if (lane == 0) {
          a.sp[i] = (uint8_t)s1;
          if (a.vx) {
            const double f = sqrt(a.p.mass[s0] / a.p.mass[s1]);
            a.u_v[3 * uq + 0] = a.vx[i];
            a.u_v[3 * uq + 1] = a.vy[i];
            a.u_v[3 * uq + 2] = a.vz[i];
            a.vx[i] = a.vx[i] * f;
            a.vy[i] = a.vy[i] * f;
            a.vz[i] = a.vz[i] * f;
          }
        }
        flipped = si;
      }
    }
    if (live && lane == 0) a.u_site[uq] = flipped;
    __syncthreads();  // the group's updates are seen by its next trial
  }
  long long v4[4] = {valid, acc, dn_acc, tie};
  block_sums<4>(v4, sh);
  if (threadIdx.x == 0) {
    long long *P = a.part + NPART * blockIdx.x;
    P[0] = v4[0];
    P[1] = v4[1];
    P[2] = v4[2];
    P[3] = v4[3];
    P[4] = v4[0];
  }
}

// Delayed acceptance (Christen and Fox), one group of TL lanes per active
// cell and 16 cells per block:
//   stage 1: surrogate dE_f of the move, accepted with min{1, exp(-beta s_f)},
//            s_f = dE_f + dmu0 dn, using u1 = unit(w1) (the plain test's u);
//   stage 2 (survivors): exact dU and the surrogate dE_r of the reverse move
//            (descriptor of the proposed state), accepted with
//            min{1, exp(-beta (dU + dmu0 dn)) min{1, exp(-beta s_r)} / min{1, exp(-beta s_f)}},
//            s_r = dE_r - dmu0 dn, using u2 = unit(w2).
// The network runs on the block's 16 descriptors at once (BF16 MFMA).
// Surrogate modes: 1 network, 2 perfect (dE_f = dU, dE_r = -dU), 3 zero.
__global__ void __launch_bounds__(BLOCK) k_trial_da(SweepArgs a, uint64_t w_arg, int64_t s,
                                                    int par) {
  const uint64_t w = sweep_of(a, w_arg);
  __shared__ long long sh[BLOCK];
  __shared__ GroupTerms terms[BLOCK / TL];
  __shared__ __bf16 zs[16 * MLP_KP];
  __shared__ __bf16 h1[16 * MLP_H], h2[16 * MLP_H];
  __shared__ float yv[16];
  __shared__ DescSlots dslots[BLOCK / TL];
  const int lane = threadIdx.x % TL, grp = threadIdx.x / TL;
  const int64_t t = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / TL;
  // site and ln u1 from the sweep's table (the plain test's draws)
  const int64_t i = t < a.ncpc ? a.sites[s * a.ncpc + t] : -1;
  const double lnu1 = t < a.ncpc ? a.site_lnu[s * a.ncpc + t] : 0.0;
  const bool has = i >= 0;
  const int dn = has ? 1 - 2 * (int)a.sp[i] : 0;
  // one gather gives the forward and flipped descriptors and the exact dU
  // (contexts without the descriptor list: dU from the r < rc list)
  double du = 0.0, ef = 0.0, er = 0.0;
  double dfw[10] = {}, dfl[10] = {};
  if (has) {
    if (a.dj)
      desc_du_group(a, i, lane, dfw, dfl, du, dslots[threadIdx.x / TL]);
    else
      du = delta_u_group(a, i, lane, terms[threadIdx.x / TL]);
  }
  // ---- surrogate value of the forward move
  if (a.da_mode == 1) {
    for (int k = lane; k < MLP_KP; k += TL) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < MLP_IN; ++q) v = q == k ? dfw[q] : v;  // static indices
      zs[grp * MLP_KP + k] = (has && k < MLP_IN) ? mlp_input(a.md, k, v) : to_bf16(0.0f);
    }
    __syncthreads();
    mlp_block16(a.md, zs, h1, h2, yv);
    ef = (double)(yv[grp] * a.md.out_sd + a.md.out_mu);
  } else if (a.da_mode == 2) {
    ef = du;
  }
  // ---- stage 1 (every lane of the group evaluates the same test)
  const double sf = ef + a.dmu0 * (double)dn;
  const double x1 = a.beta * sf;
  const bool pass1 = has && lnu1 < -x1;
  // ---- surrogate value of the reverse move for the survivors
  if (a.da_mode == 1) {
    const int any = __syncthreads_or(pass1 ? 1 : 0);
    if (any) {
      for (int k = lane; k < MLP_KP; k += TL) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < MLP_IN; ++q) v = q == k ? dfl[q] : v;
        zs[grp * MLP_KP + k] = (pass1 && k < MLP_IN) ? mlp_input(a.md, k, v) : to_bf16(0.0f);
      }
      __syncthreads();
      mlp_block16(a.md, zs, h1, h2, yv);
      er = (double)(yv[grp] * a.md.out_sd + a.md.out_mu);
    }
  } else if (a.da_mode == 2) {
    er = -du;
  }
  int64_t cell = -1;
  U4 r = {};
  if (has && (pass1 || a.tlog || a.dalog)) {
    const U4 g = philox(a.seed, a.replica, w, (uint64_t)s, 0, 0);
    cell = colour_cell(a, stage_colour(g.v[0], a.ncol), t);
    r = philox(a.seed, a.replica, w, (uint64_t)s, (uint64_t)cell, 1);
  }
  long long valid = 0, acc = 0, dn_acc = 0, tie = 0, p1 = 0;
  if (lane == 0 && t < a.ncpc) {
    int32_t site = -1;
    if (has) {
      bool ok = false;
      double margin = lnu1 + x1;
      if (pass1) {
        const double sr = er - a.dmu0 * (double)dn;
        const double xl = a.beta * (du + a.dmu0 * (double)dn);
        const double xr = -(a.beta * sr);
        const double l2 = (-xl + (xr < 0.0 ? xr : 0.0)) - (-x1 < 0.0 ? -x1 : 0.0);
        const double lnu2 = log(unit_open(r.v[2]));
        ok = lnu2 < l2;
        margin = lnu2 - l2;
      }
      valid = 1;
      p1 = pass1 ? 1 : 0;
      tie = fabs(margin) < TIE;
      if (ok) {
        acc = 1;
        dn_acc = dn;
        site = (int32_t)i;
      }
      if (a.tlog) {
        const unsigned long long idx = atomicAdd(&a.ds->tlog_n, 1ull);
        if ((int64_t)idx < a.tcap) {
          double *L = a.tlog + 8 * idx;
          L[0] = (double)w;
          L[1] = (double)s;
          L[2] = (double)cell;
          L[3] = (double)i;
          L[4] = (double)dn;
          L[5] = ok ? 1.0 : 0.0;
          L[6] = pass1 ? du : __builtin_nan("");
          L[7] = margin;
        }
      }
      if (a.dalog) {
        const unsigned long long idx = atomicAdd(&a.ds->dalog_n, 1ull);
        if ((int64_t)idx < a.dacap) {
          double *L = a.dalog + 5 * idx;
          L[0] = (double)w;
          L[1] = (double)s;
          L[2] = (double)cell;
          L[3] = ef;
          L[4] = pass1 ? er : __builtin_nan("");
        }
      }
    }
    a.rec[t] = site;
  }
  long long v5[5] = {valid, acc, dn_acc, tie, p1};
  block_sums<5>(v5, sh);
  if (threadIdx.x == 0) {
    long long *P = a.part + NPART * blockIdx.x;
#pragma unroll
    for (int k = 0; k < 5; ++k) P[k] = v5[k];
  }
}

// The global test of a stage (Eq. trans_vcsgc_par2): every block reduces the
// trial kernel's partial sums itself, in a fixed order.  Returns 1 (accept),
// 0 (reject) or -1 (nothing to decide).  Must be called by the whole block.
struct StageDecision {
  unsigned long long nrec;
  long long dn_tot, nb;
  double xg, mg;
  int gacc;
};

__device__ __forceinline__ StageDecision stage_decision(const SweepArgs &a, uint64_t w, int64_t s,
                                                        int par, long long *sh) {
  const double lnug = a.stage_lnug[s];  // issued before the reduction
  long long pa = 0, pd = 0;
  for (int b = threadIdx.x; b < a.nblk; b += BLOCK) {
    pa += a.part[NPART * b + 1];
    pd += a.part[NPART * b + 2];
  }
  long long v2[2] = {pa, pd};
  block_sums<2>(v2, sh);
  StageDecision d;
  d.nrec = (unsigned long long)v2[0];
  d.dn_tot = v2[1];
  d.nb = a.ds->n_b[par];
  d.gacc = -1;
  d.xg = 0.0;
  d.mg = 0.0;
  if (d.nrec > 0) {
    const double tt = (double)d.nb - a.ncbar;
    const double dnd = (double)d.dn_tot;
    d.xg = a.beta * a.kN * dnd * (dnd + 2.0 * tt);
    d.mg = lnug + d.xg;
    d.gacc = lnug < -d.xg ? 1 : 0;
  }
  return d;
}

// Statistics and the stage log after the decision (block 0; the whole block
// calls it).
__device__ __forceinline__ void stage_stats(const SweepArgs &a, uint64_t w, int64_t s, int par,
                                            int last, const StageDecision &dc, long long *sh) {
  const int gacc = dc.gacc;
  const unsigned long long nrec = dc.nrec;
  const long long dn_tot = dc.dn_tot, nb = dc.nb;
  const double xg = dc.xg, mg = dc.mg;
  long long pv = 0, pt = 0, p1 = 0;
  if (blockIdx.x == 0) {
    for (int b = threadIdx.x; b < a.nblk; b += BLOCK) {
      pv += a.part[NPART * b + 0];
      pt += a.part[NPART * b + 3];
      p1 += a.part[NPART * b + 4];
    }
    long long v3[3] = {pv, pt, p1};
    block_sums<3>(v3, sh);
    pv = v3[0];
    pt = v3[1];
    p1 = v3[2];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const long long nb_new = nb + (gacc == 1 ? dn_tot : 0);
    DevState *ds = a.ds;
    ds->n_b[par ^ 1] = nb_new;
    ds->n_b_cur = nb_new;
    ds->trials += (unsigned long long)pv;
    ds->stage1_pass += (unsigned long long)p1;
    ds->local_acc += nrec;
    ds->near_ties += (unsigned long long)pt;
    ds->stages += 1;
    if (gacc == 1) {
      ds->stage_acc += 1;
      ds->flips += nrec;
    }
    if (nrec > 0 && fabs(mg) < TIE) ds->near_ties += 1;
    if (last) {
      ds->sum_n += (double)nb_new;
      ds->sum_n2 += (double)nb_new * (double)nb_new;
    }
    if (a.slog) {
      const unsigned long long idx = ds->slog_n++;
      if ((int64_t)idx < a.scap) {
        double *L = a.slog + 8 * idx;
        L[0] = (double)w;
        L[1] = (double)s;
        L[2] = (double)stage_colour(philox(a.seed, a.replica, w, (uint64_t)s, 0, 0).v[0], a.ncol);
        L[3] = (double)dn_tot;
        L[4] = (double)nrec;
        L[5] = (double)gacc;
        L[6] = xg;
        L[7] = mg;
      }
    }
  }
}


// one group of TL lanes per active cell: lane k updates rho of entries k, k + TL
template <int F>
__global__ void __launch_bounds__(BLOCK) k_commit(SweepArgs a, uint64_t w_arg, int64_t s, int par,
                                                  int last) {
  const uint64_t w = sweep_of(a, w_arg);
  __shared__ long long sh[BLOCK];
  const int lane = threadIdx.x % TL;
  const int64_t t = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / TL;
  // the group's record and its row are read before the decision, so that
  // these loads overlap the reduction below
  int32_t i = -1;
  int s0 = 0, m = 0;
  int32_t jr[2] = {0, 0};
  double rr[2] = {0.0, 0.0};
  if (t < a.ncpc) {
    i = a.rec[t];
    if (i >= 0) {
      s0 = a.sp[i];
      m = a.cnt[i];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = lane + h * TL;
        if (k < m) {
          const int64_t e = (int64_t)i * KMAX + k;
          jr[h] = a.nj[e];
          rr[h] = a.nr[e];
        }
      }
    }
  }
  const StageDecision dc = stage_decision(a, w, s, par, sh);
  const int gacc = dc.gacc;
  if (gacc == 1 && i >= 0) {
    const int s1 = 1 - s0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = lane + h * TL;
      if (k < m) {
        const double delta = flip_rho_shift<F>(a.p, s0, rr[h]);
        a.rho[jr[h]] = a.rho[jr[h]] + delta;
      }
    }
    if (lane == 0) {
      a.sp[i] = (uint8_t)s1;
      if (a.vx) {
        const double f = sqrt(a.p.mass[s0] / a.p.mass[s1]);
        a.vx[i] = a.vx[i] * f;
        a.vy[i] = a.vy[i] * f;
        a.vz[i] = a.vz[i] * f;
      }
    }
  }
  stage_stats(a, w, s, par, last, dc, sh);
}

// Global test of a stage of local chains: a rejected stage is undone, each
// group restoring its cell's accepted trials in reverse order.
__global__ void __launch_bounds__(BLOCK) k_commit_chain(SweepArgs a, uint64_t w_arg, int64_t s,
                                                        int par, int last) {
  const uint64_t w = sweep_of(a, w_arg);
  __shared__ long long sh[BLOCK];
  const int lane = threadIdx.x % TL;
  const int64_t t = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / TL;
  const StageDecision dc = stage_decision(a, w, s, par, sh);
  if (dc.gacc == 0) {  // uniform over the grid
    for (int k = a.K - 1; k >= 0; --k) {
      const int64_t uq = t * a.K + k;
      const int32_t i = t < a.ncpc ? a.u_site[uq] : -1;
      if (i >= 0) {
        const int m = a.cnt[i];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int e = lane + h * TL;
          if (e < m) a.rho[a.u_j[uq * KMAX + e]] = a.u_rho[uq * KMAX + e];
        }
        if (lane == 0) {
          a.sp[i] = (uint8_t)(1 - a.sp[i]);
          if (a.vx) {
            a.vx[i] = a.u_v[3 * uq + 0];
            a.vy[i] = a.u_v[3 * uq + 1];
            a.vz[i] = a.u_v[3 * uq + 2];
          }
        }
      }
      __syncthreads();  // later trials are undone before earlier ones
    }
  }
  stage_stats(a, w, s, par, last, dc, sh);
}

// ---------------------------------------------------------------------------
// Fused stage pipeline (one trial per active cell and stage).  A stage whose
// global test fails leaves the state untouched, so the trials of the next
// stage can be evaluated by the same kernel that evaluates the global test;
// only an accepted stage, whose flips must be visible to every block first,
// costs a kernel of its own for the next stage's trials.  Each kernel reads
// the pipeline state left by block 0 of the kernel before it:
//   SM_TRIAL  (w, s): trials of (w, s)                         -> SM_DECIDE (w, s)
//   SM_DECIDE (w, s): global test of (w, s); accepted: commit  -> SM_TRIAL next
//                                  otherwise: trials of next   -> SM_DECIDE next
// and the stage after the last one of the call leads to SM_DONE (kernels
// launched beyond that do nothing).  The draws are those of the per-stage
// path, so both give the same chain.  The site table of sweep w + 1, stage s
// is drawn by extra blocks of the kernel that tests (w, s): every stage's
// sites are drawn once, after the entries they replace (sweep w - 1) were
// last read and before the trials that read them.
// ---------------------------------------------------------------------------

// Site of active cell t in stage s of sweep w and ln u of its local test
// (the draws of k_sites for one trial per cell); t == 0 also writes ln u_g.
// g: the stage's own counter draw, philox(seed, replica, w, s, 0, 0).
__device__ __forceinline__ void draw_site_g(const SweepArgs &a, uint64_t w, int64_t s, int64_t t,
                                            const U4 &g, int32_t *sites, double *lnus,
                                            double *lnug, double *lnus2) {
  if (t == 0) *lnug = log(unit_open(g.v[1]));
  const int colour = stage_colour(g.v[0], a.ncol);
  const int64_t cell = colour_cell(a, colour, t);
  const int64_t gq = 8 * cell + colour;
  const int32_t st = a.grown ? a.gstart[gq] : a.cstart[cell];
  const uint32_t m = (uint32_t)((a.grown ? a.gstart[gq + 1] : a.cstart[cell + 1]) - st);
  int32_t site = -1;
  double lnu = 0.0;
  if (m > 0) {
    const U4 r = philox(a.seed, a.replica, w, (uint64_t)s, (uint64_t)cell, 1);
    site = a.grown ? grown_pick(a, gq, r.v[0]) : a.catoms[st + draw_index(r.v[0], m)];
    lnu = log(unit_open(r.v[1]));
    if (lnus2) lnus2[t] = log(unit_open(r.v[2]));
  }
  sites[t] = site;
  lnus[t] = lnu;
}

__device__ __forceinline__ void draw_site(const SweepArgs &a, uint64_t w, int64_t s, int64_t t,
                                          int32_t *sites, double *lnus, double *lnug,
                                          double *lnus2) {
  draw_site_g(a, w, s, t, philox(a.seed, a.replica, w, (uint64_t)s, 0, 0), sites, lnus, lnug,
              lnus2);
}

// The whole site table of sweep w (into its half of the two-sweep ring).
// (When a stage has at least BLOCK active cells, a block spans at most two
// stages, whose counter draws two threads make for the whole block.)
__global__ void __launch_bounds__(BLOCK) k_sites_ring(SweepArgs a, uint64_t w) {
  __shared__ U4 gs[2];
  const int64_t q0 = (int64_t)blockIdx.x * BLOCK, q = q0 + threadIdx.x;
  const int64_t s0 = q0 / a.ncpc;
  const bool shared = a.ncpc >= BLOCK;
  if (shared) {
    if (threadIdx.x < 2 && s0 + threadIdx.x < a.S)
      gs[threadIdx.x] = philox(a.seed, a.replica, w, (uint64_t)(s0 + threadIdx.x), 0, 0);
    __syncthreads();
  }
  if (q >= a.S * a.ncpc) return;
  const int64_t s = q / a.ncpc, t = q - s * a.ncpc;
  const int64_t row = (int64_t)(w & 1) * a.S + s;
  const U4 g = shared ? gs[s - s0] : philox(a.seed, a.replica, w, (uint64_t)s, 0, 0);
  draw_site_g(a, w, s, t, g, a.sites + row * a.ncpc, a.site_lnu + row * a.ncpc,
              a.stage_lnug + row, a.site_lnu2 ? a.site_lnu2 + row * a.ncpc : nullptr);
}

__global__ void k_pipe_init(DevState *ds, unsigned long long w0, unsigned long long w_end) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    StageMachine m;
    m.w = w0;
    m.s = 0;
    m.nb = ds->n_b_cur;
    m.phase = w0 < w_end ? SM_TRIAL : SM_DONE;
    m.pad = 0;
    ds->pipe.sm[0] = m;
    ds->pipe.sm[1] = m;
    ds->pipe.w_end = w_end;
    ds->pipe.used = 0;
  }
}

// Local tests of stage (w, s) from the loaded trial data: the record of the
// group's cell, the trial log, and the block's two count words into P.
template <int F, int W>
__device__ __forceinline__ void pipe_trials_finish(const SweepArgs &a, uint64_t w, int64_t s,
                                                   int64_t t, int lane, int32_t i, double lnu,
                                                   const TrialInT<W> &v, int32_t *rec,
                                                   long long *P, long long *sh,
                                                   double2 *grp) {
  long long valid = 0, dn_acc = 0, tie = 0;
  if (t < a.ncpc) {
    int32_t site = -1;
    if (i >= 0) {
      const double du = delta_u_of<W, F>(a, v, lane, grp);
      if (lane == 0) {
        const int dn = 1 - 2 * v.s;
        const double xl = a.beta * (du + a.dmu0 * (double)dn);
        const double margin = lnu + xl;
        const bool ok = lnu < -xl;
        valid = 1;
        tie = fabs(margin) < TIE;
        if (ok) {
          dn_acc = dn;
          site = i;
        }
        if (a.tlog) {
          const unsigned long long idx = atomicAdd(&a.ds->tlog_n, 1ull);
          if ((int64_t)idx < a.tcap) {
            const U4 g = philox(a.seed, a.replica, w, (uint64_t)s, 0, 0);
            double *L = a.tlog + 8 * idx;
            L[0] = (double)w;
            L[1] = (double)s;
            L[2] = (double)colour_cell(a, stage_colour(g.v[0], a.ncol), t);
            L[3] = (double)i;
            L[4] = (double)dn;
            L[5] = ok ? 1.0 : 0.0;
            L[6] = du;
            L[7] = margin;
          }
        }
      }
    }
    if (lane == 0) rec[t] = site;
  }
  // counts packed two to a word (each 32-bit field's sum over the grid stays
  // below 2^31): (trials | accepts with dn = +1), (accepts with dn = -1 | ties);
  // sh is this call's own scratch (no trailing barrier)
  long long v2[2] = {valid | ((dn_acc > 0 ? 1ll : 0ll) << 32),
                     (dn_acc < 0 ? 1ll : 0ll) | (tie << 32)};
  block_sums<2, false>(v2, sh);
  if (threadIdx.x == 0) {
    P[0] = v2[0];
    P[1] = v2[1];
  }
}

// Site and trial data of group t in stage (w, s) (site -1: empty cell or
// past the last active cell).
template <int F, int L>
__device__ __forceinline__ void pipe_trials_load(const SweepArgs &a, uint64_t w, int64_t s,
                                                 int64_t t, int lane, int32_t &i, double &lnu,
                                                 TrialInT<L> &v) {
  i = -1;
  lnu = 0.0;
  v.m = 0;
  v.s = 0;
  v.ri = 0.0;
  if (t < a.ncpc) {
    const int64_t q = ((int64_t)(w & 1) * a.S + s) * a.ncpc + t;
    i = a.sites[q];
    lnu = a.site_lnu[q];
    if (i >= 0) load_trial<L, F>(a, i, lane, v);
  }
}

// Commit of an accepted trial at site i by the TL lanes of its group: rho_j
// += delta_j of every neighbour entry, then the species and the velocity.
template <int F>
__device__ __forceinline__ void pipe_commit(const SweepArgs &a, int32_t i, int lane) {
  const int s0 = a.sp[i], s1 = 1 - s0;
  const int m = a.cnt[i];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = lane + h * TL;
    if (k < m) {
      const int64_t e = (int64_t)i * KMAX + k;
      const int32_t j = a.nj[e];
      const double delta = flip_rho_shift<F>(a.p, s0, a.nr[e]);
      a.rho[j] = a.rho[j] + delta;
    }
  }
  if (lane == 0) {
    a.sp[i] = (uint8_t)s1;
    if (a.vx) {
      const double f = sqrt(a.p.mass[s0] / a.p.mass[s1]);
      a.vx[i] = a.vx[i] * f;
      a.vy[i] = a.vy[i] * f;
      a.vz[i] = a.vz[i] * f;
    }
  }
}

// Delayed-acceptance trials of stage (w, s) in the pipeline (the two-stage
// test of k_trial_da for the block's 16 cells, sites and ln u from the
// two-sweep ring): the record of each cell, the trial and surrogate logs,
// and the block's three count words into P ((trials | accepts with dn = +1
// << 32), (accepts with dn = -1 | ties << 32), stage-1 passes).  Every
// thread of the block calls it.
struct DaShared {
  DescSlots dslots[BLOCK / TL];
  __bf16 zs[32 * MLP_KP];  // rows 0..15 the current, 16..31 the flipped descriptors
  __bf16 h1[32 * MLP_H], h2[32 * MLP_H];
  float yv[32];
  float w3[MLP_H];  // output-layer weights
};
static_assert(BLOCK / TL == 16, "one network row per lane group");

template <int F>
__device__ __forceinline__ void pipe_trials_da(const SweepArgs &a, uint64_t w, int64_t s,
                                               int64_t t, int lane, int32_t *rec,
                                               long long *P, long long *sh, double2 *grpt,
                                               DaShared &ds_) {
  const int grp = threadIdx.x / TL;
  // the network's weights first: their reads overlap the descriptor reads
  MlpFrag mf;
  if (a.da_mode == 1) {
    mf = mlp_frag(a.md);
    if (threadIdx.x < MLP_H) ds_.w3[threadIdx.x] = a.md.w3[threadIdx.x];
  }
  const int64_t q = ((int64_t)(w & 1) * a.S + s) * a.ncpc + t;
  const int64_t i = t < a.ncpc ? a.sites[q] : -1;
  const double lnu1 = t < a.ncpc ? a.site_lnu[q] : 0.0;
  const double lnu2 = t < a.ncpc ? a.site_lnu2[q] : 0.0;  // drawn with the site
  const bool has = i >= 0;
  const int dn = has ? 1 - 2 * (int)a.sp[i] : 0;
  double du = 0.0, ef = 0.0, er = 0.0;
  double dfw[10] = {}, dfl[10] = {};
  if (has) {
    if (a.dj)
      desc_du_group(a, i, lane, dfw, dfl, du, ds_.dslots[grp]);
    else
      du = delta_u_group<F>(a, i, lane, grpt);
  }
  // both network values in one pass; the flipped one is used only when the
  // first stage passes
  if (a.da_mode == 1) {
    for (int k = lane; k < MLP_KP; k += TL) {
      double v = 0.0, vl = 0.0;
#pragma unroll
      for (int qq = 0; qq < MLP_IN; ++qq) {  // static indices
        v = qq == k ? dfw[qq] : v;
        vl = qq == k ? dfl[qq] : vl;
      }
      const bool in = has && k < MLP_IN;
      ds_.zs[grp * MLP_KP + k] = in ? mlp_input(a.md, k, v) : to_bf16(0.0f);
      ds_.zs[(16 + grp) * MLP_KP + k] = in ? mlp_input(a.md, k, vl) : to_bf16(0.0f);
    }
    __syncthreads();
    mlp_block32f(a.md, mf, ds_.w3, ds_.zs, ds_.h1, ds_.h2, ds_.yv);
    ef = (double)(ds_.yv[grp] * a.md.out_sd + a.md.out_mu);
    er = (double)(ds_.yv[16 + grp] * a.md.out_sd + a.md.out_mu);
  } else if (a.da_mode == 2) {
    ef = du;
    er = -du;
  }
  const double sf = ef + a.dmu0 * (double)dn;
  const double x1 = a.beta * sf;
  const bool pass1 = has && lnu1 < -x1;
  int64_t cell = -1;  // for the logs only
  if (has && (a.tlog || a.dalog)) {
    const U4 g = philox(a.seed, a.replica, w, (uint64_t)s, 0, 0);
    cell = colour_cell(a, stage_colour(g.v[0], a.ncol), t);
  }
  long long valid = 0, dn_acc = 0, tie = 0, p1 = 0;
  if (lane == 0 && t < a.ncpc) {
    int32_t site = -1;
    if (has) {
      bool ok = false;
      double margin = lnu1 + x1;
      if (pass1) {
        const double sr = er - a.dmu0 * (double)dn;
        const double xl = a.beta * (du + a.dmu0 * (double)dn);
        const double xr = -(a.beta * sr);
        const double l2 = (-xl + (xr < 0.0 ? xr : 0.0)) - (-x1 < 0.0 ? -x1 : 0.0);
        ok = lnu2 < l2;
        margin = lnu2 - l2;
      }
      valid = 1;
      p1 = pass1 ? 1 : 0;
      tie = fabs(margin) < TIE;
      if (ok) {
        dn_acc = dn;
        site = (int32_t)i;
      }
      if (a.tlog) {
        const unsigned long long idx = atomicAdd(&a.ds->tlog_n, 1ull);
        if ((int64_t)idx < a.tcap) {
          double *L = a.tlog + 8 * idx;
          L[0] = (double)w;
          L[1] = (double)s;
          L[2] = (double)cell;
          L[3] = (double)i;
          L[4] = (double)dn;
          L[5] = ok ? 1.0 : 0.0;
          L[6] = pass1 ? du : __builtin_nan("");
          L[7] = margin;
        }
      }
      if (a.dalog) {
        const unsigned long long idx = atomicAdd(&a.ds->dalog_n, 1ull);
        if ((int64_t)idx < a.dacap) {
          double *L = a.dalog + 5 * idx;
          L[0] = (double)w;
          L[1] = (double)s;
          L[2] = (double)cell;
          L[3] = ef;
          L[4] = pass1 ? er : __builtin_nan("");
        }
      }
    }
    rec[t] = site;
  }
  long long v3[3] = {valid | ((dn_acc > 0 ? 1ll : 0ll) << 32),
                     (dn_acc < 0 ? 1ll : 0ll) | (tie << 32), p1};
  block_sums<3, false>(v3, sh);
  if (threadIdx.x == 0) {
    P[0] = v3[0];
    P[1] = v3[1];
    P[2] = v3[2];
  }
}

// One kernel of the pipeline; par is the launch parity (state read from
// pipe.sm[par], written to pipe.sm[par ^ 1]).  Blocks [0, nblk) hold one
// group of TL lanes per active cell; the blocks after them draw sites.
// DA: the trials are delayed-acceptance trials (three count words per
// trial block instead of two).  F: the potential's form (0 analytic, 1
// tabulated).
template <bool DA, int F>
__global__ void __launch_bounds__(BLOCK) k_stage(SweepArgs a, int par) {
  constexpr int NPW = DA ? 3 : 2;  // count words per trial block
  __shared__ long long sh[BLOCK];  // the trials' block counts
  __shared__ long long shd[BLOCK / 64 * 3];  // the global test's counts
  __shared__ GroupTerms terms[BLOCK / TL];
  __shared__ typename std::conditional<DA, DaShared, char>::type dash;
  DevState *ds = a.ds;
  const StageMachine m = ds->pipe.sm[par];
  const uint64_t w_end = ds->pipe.w_end;
  if (m.phase == SM_DONE) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ds->pipe.sm[par ^ 1] = m;
    return;
  }
  const int64_t S = a.S, ncpc = a.ncpc;
  if ((int64_t)blockIdx.x >= a.nblk) {
    const int64_t t = ((int64_t)blockIdx.x - a.nblk) * BLOCK + threadIdx.x;
    if (m.phase == SM_DECIDE && m.w + 1 < w_end && t < ncpc) {
      const uint64_t w1 = m.w + 1;
      const int64_t row = (int64_t)(w1 & 1) * S + m.s;
      draw_site(a, w1, m.s, t, a.sites + row * ncpc, a.site_lnu + row * ncpc,
                a.stage_lnug + row, a.site_lnu2 ? a.site_lnu2 + row * ncpc : nullptr);
    }
    return;
  }
  const int lane = threadIdx.x % TL;
  const int64_t t = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / TL;
  // the parity of the stage counter picks the record and partial-sum buffers
  const uint64_t gs = m.w * (uint64_t)S + (uint64_t)m.s;
  const int64_t rstride = ncpc, pstride = NPW * (int64_t)a.nblk;
  if (m.phase == SM_TRIAL) {
    if constexpr (DA) {
      pipe_trials_da<F>(a, m.w, m.s, t, lane, a.rec + (gs & 1) * rstride,
                        a.part + (gs & 1) * pstride + NPW * blockIdx.x, sh,
                        terms[threadIdx.x / TL], dash);
    } else {
      int32_t i;
      double lnu;
      TrialIn v;
      pipe_trials_load<F>(a, m.w, m.s, t, lane, i, lnu, v);
      pipe_trials_finish<F>(a, m.w, m.s, t, lane, i, lnu, v, a.rec + (gs & 1) * rstride,
                            a.part + (gs & 1) * pstride + NPW * blockIdx.x, sh,
                            terms[threadIdx.x / TL]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      StageMachine n = m;
      n.phase = SM_DECIDE;
      ds->pipe.sm[par ^ 1] = n;
      ds->pipe.used += 1;
    }
    return;
  }
  // SM_DECIDE: the next stage's trial data are read before the global test
  // (they are used only if the test fails and the state stays as it is)
  uint64_t w2 = m.w;
  int64_t s2 = m.s + 1;
  if (s2 == S) {
    w2 += 1;
    s2 = 0;
  }
  const bool more = w2 < w_end;
  // the trial blocks' counts of (w, s) and ln u_g first: their reads then
  // overlap the trial reads below
  const double lnug = a.stage_lnug[(int64_t)(m.w & 1) * S + m.s];
  const long long *P = a.part + (gs & 1) * pstride;
  long long c3[3] = {0, 0, 0};
  for (int b = threadIdx.x; b < a.nblk; b += BLOCK) {
#pragma unroll
    for (int k = 0; k < NPW; ++k) c3[k] += P[NPW * b + k];
  }
  int32_t i2 = -1;
  double lnu2 = 0.0;
  TrialIn v;
  v.m = 0;
  v.s = 0;
  v.ri = 0.0;
  if (!DA && more) pipe_trials_load<F>(a, w2, s2, t, lane, i2, lnu2, v);
  // global test of (w, s) (Eq. trans_vcsgc_par2) from the trial blocks' counts
  block_sums<3, false>(c3, shd);
  const long long n_valid = c3[0] & 0xffffffffll, n_plus = c3[0] >> 32;
  const long long n_minus = c3[1] & 0xffffffffll, n_tie = c3[1] >> 32;
  long long v5[5] = {n_valid, n_plus + n_minus, n_plus - n_minus, n_tie,
                     DA ? c3[2] : n_valid};
  const unsigned long long nrec = (unsigned long long)v5[1];
  const long long dn_tot = v5[2];
  int gacc = -1;
  double xg = 0.0, mg = 0.0;
  if (nrec > 0) {
    const double tt = (double)m.nb - a.ncbar;
    const double dnd = (double)dn_tot;
    xg = a.beta * a.kN * dnd * (dnd + 2.0 * tt);
    mg = lnug + xg;
    gacc = lnug < -xg ? 1 : 0;
  }
  const long long nb_new = m.nb + (gacc == 1 ? dn_tot : 0);
  if (gacc == 1) {
    if (t < ncpc) {
      const int32_t i = a.rec[(gs & 1) * rstride + t];
      if (i >= 0) pipe_commit<F>(a, i, lane);
    }
  } else if (more) {
    if constexpr (DA)
      pipe_trials_da<F>(a, w2, s2, t, lane, a.rec + ((gs + 1) & 1) * rstride,
                        a.part + ((gs + 1) & 1) * pstride + NPW * blockIdx.x, sh,
                        terms[threadIdx.x / TL], dash);
    else
      pipe_trials_finish<F>(a, w2, s2, t, lane, i2, lnu2, v, a.rec + ((gs + 1) & 1) * rstride,
                            a.part + ((gs + 1) & 1) * pstride + NPW * blockIdx.x, sh,
                            terms[threadIdx.x / TL]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ds->n_b_cur = nb_new;
    ds->trials += (unsigned long long)v5[0];
    ds->stage1_pass += (unsigned long long)v5[4];
    ds->local_acc += nrec;
    ds->near_ties += (unsigned long long)v5[3];
    ds->stages += 1;
    if (gacc == 1) {
      ds->stage_acc += 1;
      ds->flips += nrec;
    }
    if (nrec > 0 && fabs(mg) < TIE) ds->near_ties += 1;
    if (m.s == S - 1) {
      ds->sum_n += (double)nb_new;
      ds->sum_n2 += (double)nb_new * (double)nb_new;
    }
    if (a.slog) {
      const unsigned long long idx = ds->slog_n++;
      if ((int64_t)idx < a.scap) {
        double *L = a.slog + 8 * idx;
        L[0] = (double)m.w;
        L[1] = (double)m.s;
        L[2] = (double)stage_colour(philox(a.seed, a.replica, m.w, (uint64_t)m.s, 0, 0).v[0], a.ncol);
        L[3] = (double)dn_tot;
        L[4] = (double)nrec;
        L[5] = (double)gacc;
        L[6] = xg;
        L[7] = mg;
      }
    }
    StageMachine n;
    n.w = w2;
    n.s = s2;
    n.nb = nb_new;
    n.phase = !more ? SM_DONE : (gacc == 1 ? SM_TRIAL : SM_DECIDE);
    n.pad = 0;
    ds->pipe.sm[par ^ 1] = n;
    ds->pipe.used += 1;
  }
}

__global__ void __launch_bounds__(BLOCK)
    k_descriptors(SweepArgs a, const int32_t *__restrict__ sites, int64_t n, int flip,
                  double *out) {
  const int lane = threadIdx.x % TL;
  const int64_t t = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / TL;
  if (t >= n) return;  // whole group leaves together
  const int32_t i = sites[t];
  if (i < 0 || (int64_t)i >= a.n) {  // invalid site: NaN row
    if (lane == 0)
      for (int k = 0; k < 10; ++k) out[10 * t + k] = __builtin_nan("");
    return;
  }
  double d[10];
  descriptor_group(a, i, lane, flip != 0, d);
  if (lane == 0)
    for (int k = 0; k < 10; ++k) out[10 * t + k] = d[k];
}

hipError_t launch_descriptors(vcsgc_ctx *c, const int32_t *sites, int64_t n, int flip,
                              double *out) {
  SweepArgs a = {};
  a.n = c->n;
  a.p = c->pot;
  a.sp = c->sp;
  a.rho = c->rho;
  a.dj = c->d_j;
  a.dr = c->d_r;
  a.dcnt = c->d_cnt;
  if (n <= 0) return hipSuccess;
  k_descriptors<<<grid_for(n * TL), BLOCK, 0, c->stream>>>(a, sites, n, flip, out);
  return hipGetLastError();
}

// Arguments of the kernel nodes of the per-stage sweep graph (kept with the
// context while the graph lives).
struct StageNodeArgs {
  SweepArgs a;
  uint64_t w;
  int64_t s;
  int par, last;
};

struct StageGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<StageNodeArgs> args;
  double key[4] = {0, 0, 0, 0};
  uint64_t seed = 0;
  int K = 1;
  int da_mode = 0;
  MlpDev md{};  // the network's device view baked into delayed-acceptance nodes
};

void free_stage_graph(vcsgc_ctx *c) {
  StageGraph *g = (StageGraph *)c->stage_graph;
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  c->stage_graph = nullptr;
}

// One sweep as a graph: the site table, then trial and commit of every stage,
// then the sweep counter advance.  Physical parameters and the seed are baked
// in (the graph is rebuilt when they change); the sweep counter is read from
// device memory.
static hipError_t build_stage_graph(vcsgc_ctx *c, const SweepArgs &a0, double dmu0, double kappa,
                                    double cbar, double T, uint64_t seed, void *f_trial,
                                    void *f_commit) {
  free_stage_graph(c);
  StageGraph *g = new StageGraph();
  c->stage_graph = g;
  g->key[0] = dmu0;
  g->key[1] = kappa;
  g->key[2] = cbar;
  g->key[3] = T;
  g->seed = seed;
  g->K = a0.K;
  g->da_mode = a0.da_mode;
  g->md = a0.md;
  hipError_t e = hipGraphCreate(&g->graph, 0);
  if (e != hipSuccess) return e;
  const int64_t S = a0.S;
  g->args.resize((size_t)(2 * S + 1));
  SweepArgs a = a0;
  a.wdev = &c->ds->wcur;
  const unsigned gb = (unsigned)grid_for(a.ncpc * TL);
  hipGraphNode_t prev = nullptr;
  auto add = [&](void *fn, unsigned grid, void **params) -> hipError_t {
    hipKernelNodeParams kp = {};
    kp.func = fn;
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(BLOCK);
    kp.kernelParams = params;
    hipGraphNode_t node;
    hipError_t e2 = hipGraphAddKernelNode(&node, g->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    if (e2 == hipSuccess) prev = node;
    return e2;
  };
  StageNodeArgs &sa = g->args[0];
  sa.a = a;
  sa.w = 0;
  void *sp_[] = {&sa.a, &sa.w};
  e = add((void *)k_sites, (unsigned)grid_for(a.S * a.ncpc), sp_);
  if (e != hipSuccess) return e;
  for (int64_t s = 0; s < S; ++s) {
    StageNodeArgs &t = g->args[(size_t)(1 + 2 * s)];
    t.a = a;
    t.w = 0;
    t.s = s;
    t.par = (int)(s & 1);
    t.last = 0;
    void *tp[] = {&t.a, &t.w, &t.s, &t.par};
    e = add(f_trial, gb, tp);
    if (e != hipSuccess) return e;
    StageNodeArgs &u = g->args[(size_t)(2 + 2 * s)];
    u = t;
    u.last = s == S - 1 ? 1 : 0;
    void *up[] = {&u.a, &u.w, &u.s, &u.par, &u.last};
    e = add(f_commit, gb, up);
    if (e != hipSuccess) return e;
  }
  DevState *ds = c->ds;
  void *np[] = {&ds};
  {
    hipKernelNodeParams kp = {};
    kp.func = (void *)k_next_sweep;
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(64);
    kp.kernelParams = np;
    hipGraphNode_t node;
    e = hipGraphAddKernelNode(&node, g->graph, &prev, 1, &kp);
    if (e != hipSuccess) return e;
  }
  return hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
}

// ---------------------------------------------------------------------------
// Batched pipeline.  A stage whose global test fails leaves the state as it
// was, so the trials of the stages after it are those made on the state
// before it.  Each kernel therefore makes the trials of a batch of up to D
// consecutive stages of one sweep at once, and the next kernel tests the
// batch's stages in order: every stage up to the first accepted one is
// decided, that stage is committed, and the trials after it (and the batch
// tried meanwhile, on the state before the commit) are made again.  The
// chain is the one-stage-at-a-time chain, stage for stage.
//
// Site tables: the rows of sweep w + 1 are drawn for the stages of each tested
// batch of sweep w.  With D <= S / 2, a batch tried in the kernel that tests
// the last batch of sweep w lies in [0, D) of sweep w + 1, whose rows were
// drawn when the first stages of sweep w were tested, and the rows being drawn
// lie in [S - D, S).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void spec_after(uint64_t w, int64_t s, int64_t n, int64_t S,
                                           unsigned long long &w2, long long &s2) {
  s2 = s + n;
  w2 = w;
  if (s2 >= S) {
    w2 += 1;
    s2 -= S;
  }
}

__device__ __forceinline__ int spec_len(uint64_t w, int64_t s, int64_t S, uint64_t w_end, int D) {
  return w < w_end ? (int)(S - s < D ? S - s : D) : 0;
}

__global__ void k_spec_init(DevState *ds, unsigned long long w0, unsigned long long w_end,
                            long long S, int D) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    SpecMachine m;
    m.dw = m.tw = w0;
    m.ds = m.ts = 0;
    m.nb = ds->n_b_cur;
    m.dn = 0;
    m.tn = spec_len(w0, 0, S, w_end, D);
    ds->pipe.spec[0] = m;
    ds->pipe.spec[1] = m;
    ds->pipe.w_end = w_end;
    ds->pipe.used = 0;
  }
}

// One kernel of the batched pipeline; par is the launch parity (state read
// from pipe.spec[par], written to pipe.spec[par ^ 1]; the batch tried here
// goes to slot par of the record and count buffers, the tested batch is in
// slot par ^ 1).  Blocks [0, SPEC_NDEC) test the batch (each on its own,
// block 0 writes the results) and share the commit; the next D nblk blocks
// hold one group of TL lanes per active cell and stage of the tried batch;
// the blocks after them draw the site tables of the next sweep.
template <bool DA, int F>
__global__ void __launch_bounds__(BLOCK) k_stage_spec(SweepArgs a, int par) {
  constexpr int NPW = DA ? 3 : 2;  // count words per trial block
  constexpr int LT = DA ? TL : TL_BATCH;  // lanes per trial
  __shared__ long long sh[BLOCK];
  // delayed acceptance: the descriptor slots of a group also hold its dU terms
  // when there is no descriptor list (the two are never used together)
  static_assert(sizeof(DescSlots) >= sizeof(GroupTerms), "terms fit the descriptor slots");
  __shared__ typename std::conditional<DA, char, GroupTerms[BLOCK / LT]>::type terms;
  __shared__ typename std::conditional<DA, DaShared, char>::type dash;
  __shared__ long long tot[SPEC_MAX][NPW];
  __shared__ double lg[SPEC_MAX];
  __shared__ int kacc;
  DevState *ds = a.ds;
  const SpecMachine m = ds->pipe.spec[par];
  if (m.dn == 0 && m.tn == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ds->pipe.spec[par ^ 1] = m;
    return;
  }
  const int64_t S = a.S, ncpc = a.ncpc, nblk = a.nblk;
  const int64_t kstride = nblk * NPW;  // count words per stage
  const int64_t b = blockIdx.x;
  if (b >= SPEC_NDEC) {
    const int64_t bt = b - SPEC_NDEC;
    if (bt < (int64_t)a.D * nblk) {
      const int k = (int)(bt / nblk);
      if (k >= m.tn) return;
      const int lane = threadIdx.x % LT, grp = threadIdx.x / LT;
      const int64_t lb = bt - (int64_t)k * nblk;
      const int64_t t = lb * (BLOCK / LT) + grp;
      const int64_t s = m.ts + k;
      int32_t *rec = a.rec + ((int64_t)par * SPEC_MAX + k) * ncpc;
      long long *P = a.part + ((int64_t)par * SPEC_MAX + k) * kstride + lb * NPW;
      if constexpr (DA) {
        pipe_trials_da<F>(a, m.tw, s, t, lane, rec, P, sh, (double2 *)dash.dslots[grp], dash);
      } else {
        int32_t i;
        double lnu;
        TrialInT<LT> v;
        pipe_trials_load<F>(a, m.tw, s, t, lane, i, lnu, v);
        pipe_trials_finish<F>(a, m.tw, s, t, lane, i, lnu, v, rec, P, sh, terms[grp]);
      }
      return;
    }
    const int64_t q = (bt - (int64_t)a.D * nblk) * BLOCK + threadIdx.x;
    const int64_t k = q / ncpc, t = q - k * ncpc;
    if (k < m.dn && m.dw + 1 < ds->pipe.w_end) {
      const uint64_t w1 = m.dw + 1;
      const int64_t row = (int64_t)(w1 & 1) * S + m.ds + k;
      draw_site(a, w1, m.ds + k, t, a.sites + row * ncpc, a.site_lnu + row * ncpc,
                a.stage_lnug + row, a.site_lnu2 ? a.site_lnu2 + row * ncpc : nullptr);
    }
    return;
  }
  const uint64_t w_end = ds->pipe.w_end;
  if (m.dn == 0) {
    // nothing to test: the batch tried now starts from the committed state
    if (b == 0 && threadIdx.x == 0) {
      SpecMachine n;
      n.nb = m.nb;
      n.dw = m.tw;
      n.ds = m.ts;
      n.dn = m.tn;
      spec_after(m.tw, m.ts, m.tn, S, n.tw, n.ts);
      n.tn = spec_len(n.tw, n.ts, S, w_end, a.D);
      ds->pipe.spec[par ^ 1] = n;
      ds->pipe.used += 1;
    }
    return;
  }
  // the tested batch's counts per stage (exact integer sums) and ln u_g
  {
    const long long *P0 = a.part + (int64_t)(par ^ 1) * SPEC_MAX * kstride;
    const int wv = threadIdx.x >> 6, wl = threadIdx.x & 63;
    for (int k = wv; k < m.dn; k += BLOCK / 64) {
      long long c[NPW];
#pragma unroll
      for (int q = 0; q < NPW; ++q) c[q] = 0;
      for (int64_t lb = wl; lb < nblk; lb += 64)
#pragma unroll
        for (int q = 0; q < NPW; ++q) c[q] += P0[k * kstride + lb * NPW + q];
#pragma unroll
      for (int q = 0; q < NPW; ++q)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) c[q] += __shfl_xor(c[q], off);
      if (wl == 0)
#pragma unroll
        for (int q = 0; q < NPW; ++q) tot[k][q] = c[q];
    }
    if (threadIdx.x < m.dn)
      lg[threadIdx.x] = log(unit_open(
          philox(a.seed, a.replica, m.dw, (uint64_t)(m.ds + threadIdx.x), 0, 0).v[1]));
  }
  __syncthreads();
  // global tests (Eq. trans_vcsgc_par2) in stage order, up to the first accepted one
  if (threadIdx.x == 0) {
    long long nb = m.nb;
    int ka = -1, nk = 0;
    unsigned long long trials = 0, pass1 = 0, lacc = 0, ties = 0, flips = 0;
    bool sweep_end = false;
    for (int k = 0; k < m.dn; ++k) {
      const long long c0 = tot[k][0], c1 = tot[k][1];
      const long long n_valid = c0 & 0xffffffffll, n_plus = c0 >> 32;
      const long long n_minus = c1 & 0xffffffffll, n_tie = c1 >> 32;
      const long long nrec = n_plus + n_minus, dn_tot = n_plus - n_minus;
      int gacc = -1;
      double mg = 0.0;
      if (nrec > 0) {
        const double tt = (double)nb - a.ncbar;
        const double dnd = (double)dn_tot;
        const double xg = a.beta * a.kN * dnd * (dnd + 2.0 * tt);
        mg = lg[k] + xg;
        gacc = lg[k] < -xg ? 1 : 0;
      }
      if (gacc == 1) nb += dn_tot;
      trials += (unsigned long long)n_valid;
      pass1 += (unsigned long long)(DA ? tot[k][NPW - 1] : n_valid);
      lacc += (unsigned long long)nrec;
      ties += (unsigned long long)n_tie;
      if (nrec > 0 && fabs(mg) < TIE) ties += 1;
      nk = k + 1;
      if (m.ds + k == S - 1) sweep_end = true;
      if (gacc == 1) {
        ka = k;
        flips = (unsigned long long)nrec;
        break;
      }
    }
    kacc = ka;
    if (b == 0) {
      ds->n_b_cur = nb;
      ds->trials += trials;
      ds->stage1_pass += pass1;
      ds->local_acc += lacc;
      ds->near_ties += ties;
      ds->stages += (unsigned long long)nk;
      if (ka >= 0) {
        ds->stage_acc += 1;
        ds->flips += flips;
      }
      if (sweep_end) {
        ds->sum_n += (double)nb;
        ds->sum_n2 += (double)nb * (double)nb;
      }
      SpecMachine n;
      n.nb = nb;
      if (ka >= 0) {
        // the batch tried now saw the state before the commit: it is dropped
        n.dw = m.dw;
        n.ds = m.ds;
        n.dn = 0;
        spec_after(m.dw, m.ds, ka + 1, S, n.tw, n.ts);
      } else {
        n.dw = m.tw;
        n.ds = m.ts;
        n.dn = m.tn;
        spec_after(m.tw, m.ts, m.tn, S, n.tw, n.ts);
      }
      n.tn = spec_len(n.tw, n.ts, S, w_end, a.D);
      ds->pipe.spec[par ^ 1] = n;
      ds->pipe.used += 1;
    }
  }
  __syncthreads();
  const int ka = kacc;
  if (ka < 0) return;
  // commit of the accepted stage: 16 records per group of TL lanes, the
  // groups' flips one after the other (sites of one stage have disjoint
  // neighbourhoods)
  const int lane = threadIdx.x % TL, grp = threadIdx.x / TL;
  const int32_t *R = a.rec + ((int64_t)(par ^ 1) * SPEC_MAX + ka) * ncpc;
  for (int64_t t0 = (b * (BLOCK / TL) + grp) * TL; t0 < ncpc; t0 += (int64_t)SPEC_NDEC * BLOCK) {
    const int64_t tt = t0 + lane;
    const int32_t r = tt < ncpc ? R[tt] : -1;
    const unsigned long long bal = __ballot(r >= 0);
    unsigned gm = (unsigned)(bal >> ((threadIdx.x & 63) & ~(TL - 1))) & 0xFFFFu;
    while (gm) {
      const int src = __ffs(gm) - 1;
      gm &= gm - 1;
      pipe_commit<F>(a, __shfl(r, src, TL), lane);
    }
  }
}

// Graphs of pipeline kernels: `big` holds S launches (one sweep's worth when
// no stage is accepted), `small` PIPE_SMALL; both have even length, so every
// replay starts at launch parity 0.  The kernel arguments (parameters, seed)
// are baked in; the graphs are rebuilt when they change.
constexpr int PIPE_SMALL = 4;

// With per-kernel timing on, `big` also starts and ends with an event-record
// node: the span of its last replay, read when the call ends, over its
// kernel count is the mean time per pipeline kernel (gaps between kernels
// included).  Events between the kernels would stretch the pipeline.
struct PipeGraph {
  hipGraphExec_t big = nullptr, small = nullptr;
  int64_t nbig = 0;
  SweepArgs a0[2];  // arguments of the even / odd nodes
  int par[2] = {0, 1};
  double key[4] = {0, 0, 0, 0};
  uint64_t seed = 0;
  bool timed = false;
  int da_mode = 0;
  int spec_d = 0;  // batched pipeline: stages per batch (0: one stage per kernel)
  bool big_ran = false;  // `big` launched in the current call (its events recorded)
  MlpDev md{};  // the network's device view baked into delayed-acceptance nodes
  std::vector<hipEvent_t> ev;
};

static void *pipe_kernel(const SweepArgs &a) {
  if (a.p.tab) {
    if (a.D > 0) return a.da_mode ? (void *)k_stage_spec<true, 1> : (void *)k_stage_spec<false, 1>;
    return a.da_mode ? (void *)k_stage<true, 1> : (void *)k_stage<false, 1>;
  }
  if (a.D > 0) return a.da_mode ? (void *)k_stage_spec<true, 0> : (void *)k_stage_spec<false, 0>;
  return a.da_mode ? (void *)k_stage<true, 0> : (void *)k_stage<false, 0>;
}

void free_pipe_graph(vcsgc_ctx *c) {
  PipeGraph *g = (PipeGraph *)c->pipe_graph;
  if (!g) return;
  if (g->big) (void)hipGraphExecDestroy(g->big);
  if (g->small) (void)hipGraphExecDestroy(g->small);
  for (hipEvent_t e : g->ev) (void)hipEventDestroy(e);
  delete g;
  c->pipe_graph = nullptr;
}

static hipError_t pipe_graph_of(PipeGraph *g, int64_t len, unsigned grid, bool timed,
                                hipGraphExec_t *out) {
  hipGraph_t graph;
  hipError_t e = hipGraphCreate(&graph, 0);
  if (e != hipSuccess) return e;
  hipGraphNode_t prev = nullptr;
  void *params[2][2] = {{&g->a0[0], &g->par[0]}, {&g->a0[1], &g->par[1]}};
  auto add_event = [&]() -> hipError_t {
    hipEvent_t ev;
    hipError_t e2 = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence);
    if (e2 != hipSuccess) return e2;
    g->ev.push_back(ev);
    hipGraphNode_t node;
    e2 = hipGraphAddEventRecordNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, ev);
    if (e2 == hipSuccess) prev = node;
    return e2;
  };
  if (timed) e = add_event();
  for (int64_t q = 0; q < len && e == hipSuccess; ++q) {
    hipKernelNodeParams kp = {};
    kp.func = pipe_kernel(g->a0[0]);
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(BLOCK);
    kp.kernelParams = params[q & 1];
    hipGraphNode_t node;
    e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    prev = node;
  }
  if (e == hipSuccess && timed) e = add_event();
  if (e == hipSuccess) e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  return e;
}

// Launch k (even) pipeline kernels starting at parity 0.
static hipError_t pipe_launch(vcsgc_ctx *c, const SweepArgs &a, unsigned grid, int64_t k,
                              PipeGraph *g) {
  if (g) {
    while (k >= g->nbig) {
      hipError_t e = hipGraphLaunch(g->big, c->stream);
      if (e != hipSuccess) return e;
      g->big_ran = true;
      k -= g->nbig;
    }
    while (k > 0) {
      hipError_t e = hipGraphLaunch(g->small, c->stream);
      if (e != hipSuccess) return e;
      k -= PIPE_SMALL;
    }
    return hipSuccess;
  }
  void *f = pipe_kernel(a);
  for (int64_t q = 0; q < k; ++q) {
    const int h = tstart(c, VCSGC_KT_STAGE);
    int par = (int)(q & 1);
    SweepArgs aq = a;
    void *args[] = {&aq, &par};
    hipError_t e = hipLaunchKernel(f, dim3(grid), dim3(BLOCK), args, 0, c->stream);
    tstop(c, h);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// Sweeps w .. w + n_sweeps - 1 through the fused pipeline (a.D = 0: one
// stage per kernel; the kernels a call needs are one per stage, plus one,
// plus one per accepted stage) or the batched pipeline (a.D stages per
// kernel; about one kernel per D stages plus one per accepted stage).  The
// host launches its estimate, reads the pipeline's progress and launches
// more until the last stage has been decided.
static hipError_t launch_pipeline(vcsgc_ctx *c, SweepArgs a, double dmu0, double kappa,
                                  double cbar, double T, int64_t n_sweeps, bool use_graph,
                                  bool timed) {
  const bool spec = a.D > 0;
  a.sites = c->m_sites;
  a.site_lnu = c->m_lnu;
  a.site_lnu2 = a.da_mode ? c->m_lnu2 : nullptr;
  a.stage_lnug = c->m_lnug;
  a.rec = spec ? c->s_rec : c->m_rec;
  a.part = spec ? c->s_part : c->m_part;
  a.nblk = grid_for(a.ncpc * (spec && !a.da_mode ? TL_BATCH : TL));
  a.wdev = nullptr;
  const unsigned grid =
      spec ? (unsigned)(SPEC_NDEC + (int64_t)a.D * a.nblk + grid_for((int64_t)a.D * a.ncpc))
           : (unsigned)(a.nblk + grid_for(a.ncpc));
  PipeGraph *g = nullptr;
  if (use_graph) {
    g = (PipeGraph *)c->pipe_graph;
    if (!g || g->key[0] != dmu0 || g->key[1] != kappa || g->key[2] != cbar || g->key[3] != T ||
        g->seed != a.seed || g->timed != timed || g->da_mode != a.da_mode ||
        g->spec_d != a.D || memcmp(&g->md, &a.md, sizeof(MlpDev)) != 0) {
      free_pipe_graph(c);
      g = new PipeGraph();
      c->pipe_graph = g;
      g->key[0] = dmu0;
      g->key[1] = kappa;
      g->key[2] = cbar;
      g->key[3] = T;
      g->seed = a.seed;
      g->da_mode = a.da_mode;
      g->spec_d = a.D;
      g->md = a.md;
      g->a0[0] = g->a0[1] = a;
      // one sweep's kernels when no stage is accepted (the batched pipeline
      // needs one more to test its last batch)
      const int64_t per_sweep = spec ? (a.S + a.D - 1) / a.D + 1 : a.S;
      g->nbig = per_sweep + (per_sweep & 1);
      g->timed = timed;
      hipError_t e = pipe_graph_of(g, g->nbig, grid, timed, &g->big);
      if (e == hipSuccess) e = pipe_graph_of(g, PIPE_SMALL, grid, false, &g->small);
      if (e != hipSuccess) {
        free_pipe_graph(c);
        return e;
      }
    }
  }
  if (g) g->big_ran = false;
  const uint64_t w0 = c->w, w_end = c->w + (uint64_t)n_sweeps;
  k_sites_ring<<<grid_for(a.S * a.ncpc), BLOCK, 0, c->stream>>>(a, w0);
  if (spec)
    k_spec_init<<<1, 64, 0, c->stream>>>(a.ds, (unsigned long long)w0,
                                         (unsigned long long)w_end, (long long)a.S, a.D);
  else
    k_pipe_init<<<1, 64, 0, c->stream>>>(a.ds, (unsigned long long)w0,
                                         (unsigned long long)w_end);
  const int64_t G = n_sweeps * a.S;
  const int64_t step = use_graph ? PIPE_SMALL : 2;
  auto round_up = [&](int64_t k) { return (k + step - 1) / step * step; };
  const double spec_rate = c->m_spec_rate > 0.0 ? c->m_spec_rate : 1.0 / a.D + 0.1;
  auto estimate = [&](int64_t left) {
    if (spec) return round_up((int64_t)std::ceil((double)left * spec_rate) + 1);
    return round_up(left + 1 + (int64_t)std::ceil((double)left * c->m_acc_rate) + 2);
  };
  int64_t k = estimate(G);
  hipError_t e = pipe_launch(c, a, grid, k, g);
  if (e != hipSuccess) return e;
  // every kernel before the end decides a stage or tries a batch that the
  // next one tests, so 2 G + 1 kernels always suffice; more would mean a
  // broken pipeline state
  int64_t launched = k;
  for (;;) {
    // the persistent path's n_B and the whole device state: when the call
    // has ended, this one read also serves its statistics
    e = persist_sync_nb_from_stage(c);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->h_state, a.ds, sizeof(DevState), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    int64_t left;
    if (spec) {
      const SpecMachine m = c->h_state->pipe.spec[0];
      if (m.dn == 0 && m.tn == 0) break;
      left = m.dn > 0 ? (int64_t)(w_end - m.dw) * a.S - m.ds
                      : (int64_t)(w_end - m.tw) * a.S - m.ts;
    } else {
      const StageMachine m = c->h_state->pipe.sm[0];
      if (m.phase == SM_DONE) break;
      // stages still to decide, the pending trials, and the accepts expected among them
      left = (int64_t)(w_end - m.w) * a.S - m.s;
    }
    k = estimate(left);
    if (left <= 0 || launched > 2 * G + 2 * step + 1) return hipErrorUnknown;
    launched += k;
    e = pipe_launch(c, a, grid, k, g);
    if (e != hipSuccess) return e;
  }
  if (G > 0) {
    if (spec) {
      c->m_spec_rate = (double)c->h_state->pipe.used / (double)G;
    } else {
      const double extra = (double)c->h_state->pipe.used - 1.0 - (double)G;
      c->m_acc_rate = extra > 0.0 ? extra / (double)G : 0.0;
    }
  }
  if (g && g->timed) {
    // span of the last replay of `big` (the stream is synchronized)
    float ms = 0.f;
    if (g->big_ran && g->ev.size() == 2 &&
        hipEventElapsedTime(&ms, g->ev[0], g->ev[1]) == hipSuccess) {
      c->kt_ms[VCSGC_KT_STAGE] += ms;
      c->kt_n[VCSGC_KT_STAGE] += g->nbig;
    }
    c->kt_seen[VCSGC_KT_STAGE] += launched;
  }
  c->h_state_final = true;
  return hipSuccess;
}

hipError_t launch_sweeps(vcsgc_ctx *c, double dmu0, double kappa, double cbar, double T,
                         int64_t n_sweeps, uint64_t seed) {
  SweepArgs a = {};
  a.n = c->n;
  a.n0 = c->nc[0];
  a.n1 = c->nc[1];
  a.n2 = c->nc[2];
  a.per = c->per;
  a.ncol = c->ncol;
  a.ncpc = active_cells(c);
  a.K = c->local_steps;
  a.S = stages_per_sweep(c);
  a.grown = c->grown ? 1 : 0;
  a.gstart = c->g_start;
  a.glist = c->g_list;
  a.gcum = c->g_cum;
  a.beta = 1.0 / (KB * T);
  a.dmu0 = dmu0;
  a.kN = kappa / (double)c->n;
  a.ncbar = (double)c->n * cbar;
  a.seed = seed;
  a.replica = 0;
  a.p = c->pot;
  a.cstart = c->cell_start;
  a.catoms = c->cell_atoms;
  a.nj = c->mc_j;
  a.nr = c->mc_r;
  a.cnt = c->mc_cnt;
  a.sp = c->sp;
  a.rho = c->rho;
  a.vx = c->vx;
  a.vy = c->vy;
  a.vz = c->vz;
  a.rec = c->rec;
  a.part = c->part;
  a.ds = c->ds;
  a.tlog = c->tlog;
  a.tcap = c->tcap;
  a.slog = c->slog;
  a.scap = c->scap;
  a.dj = c->d_j;
  a.dr = c->d_r;
  a.dcnt = c->d_cnt;
  a.da_mode = c->da_mode;
  if (c->mlp) a.md = mlp_dev(c->mlp);
  a.dalog = c->dalog;
  a.dacap = c->dacap;
  a.smp_desc = c->smp_desc;
  a.smp_de = c->smp_de;
  a.smp_cap = c->smp_cap;
  a.smp_stride = c->smp_stride < 1 ? 1 : c->smp_stride;
  a.sites = c->sites;
  a.site_lnu = c->site_lnu;
  a.stage_lnug = c->stage_lnug;
  a.wdev = nullptr;
  a.u_site = c->u_site;
  a.u_j = c->u_j;
  a.u_rho = c->u_rho;
  a.u_v = c->u_v;
  const bool tab = a.p.tab != 0;
  void *f_trial = a.da_mode ? (void *)k_trial_da
                  : a.K > 1 ? (tab ? (void *)k_trial_chain<1> : (void *)k_trial_chain<0>)
                            : (tab ? (void *)k_trial<1> : (void *)k_trial<0>);
  void *f_commit = a.K > 1 ? (void *)k_commit_chain : (tab ? (void *)k_commit<1> : (void *)k_commit<0>);
  const int gb = grid_for(a.ncpc * TL);
  a.nblk = gb;
  k_init<<<1, BLOCK, 0, c->stream>>>(c->ds);
  // one trial per cell and stage: the fused pipeline (graphs of its kernels
  // unless logs or per-kernel timing are on)
  if (a.K == 1 && a.smp_cap == 0) {
    if (n_sweeps == 0) return hipGetLastError();
    const bool timed = (c->tmask & (1u << VCSGC_KT_STAGE)) != 0;
    const bool logs = a.tlog || a.slog || a.dalog;
    // batches of stages (strategy 3) when nothing is logged per trial or
    // stage: a dropped batch's trials would otherwise be logged
    if (c->strategy == 3 && !logs && a.S >= 2)
      a.D = (int)std::min<int64_t>({(int64_t)c->trials_per_group, (int64_t)SPEC_MAX, a.S / 2});
    return launch_pipeline(c, a, dmu0, kappa, cbar, T, n_sweeps, !logs, timed);
  }
  // sweeps with no logs and no per-kernel timing replay a graph of one sweep
  // (no host work per stage); everything else launches stage by stage
  const bool per_kernel_timing = (c->tmask & ((1u << VCSGC_KT_TRIAL) | (1u << VCSGC_KT_COMMIT))) != 0;
  if (!a.tlog && !a.slog && !a.dalog && a.smp_cap == 0 && !per_kernel_timing && n_sweeps > 0) {
    StageGraph *g = (StageGraph *)c->stage_graph;
    if (!g || !g->exec || g->key[0] != dmu0 || g->key[1] != kappa || g->key[2] != cbar ||
        g->key[3] != T || g->seed != seed || g->K != a.K || g->da_mode != a.da_mode ||
        memcmp(&g->md, &a.md, sizeof(MlpDev)) != 0) {
      hipError_t e = build_stage_graph(c, a, dmu0, kappa, cbar, T, seed, f_trial, f_commit);
      if (e != hipSuccess) {
        free_stage_graph(c);
        return e;
      }
      g = (StageGraph *)c->stage_graph;
    }
    k_set_sweep<<<1, 64, 0, c->stream>>>(c->ds, (unsigned long long)c->w);
    int h = tstart(c, VCSGC_KT_PERSIST);
    for (int64_t sw = 0; sw < n_sweeps; ++sw) {
      hipError_t e = hipGraphLaunch(g->exec, c->stream);
      if (e != hipSuccess) return e;
    }
    tstop(c, h);
    return hipGetLastError();
  }
  int64_t q = 0;
  for (int64_t sw = 0; sw < n_sweeps; ++sw) {
    const uint64_t w = c->w + (uint64_t)sw;
    k_sites<<<grid_for(a.S * a.ncpc), BLOCK, 0, c->stream>>>(a, w);
    for (int64_t s = 0; s < a.S; ++s, ++q) {
      const int par = (int)(q & 1);
      int last = s == a.S - 1;
      void *ta[] = {&a, (void *)&w, &s, (void *)&par};
      void *ca[] = {&a, (void *)&w, &s, (void *)&par, &last};
      int h = tstart(c, VCSGC_KT_TRIAL);
      hipError_t e = hipLaunchKernel(f_trial, dim3(gb), dim3(BLOCK), ta, 0, c->stream);
      tstop(c, h);
      if (e != hipSuccess) return e;
      h = tstart(c, VCSGC_KT_COMMIT);
      e = hipLaunchKernel(f_commit, dim3(gb), dim3(BLOCK), ca, 0, c->stream);
      tstop(c, h);
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace vc
