// Persistent parallel VC-SGC sweep for a batch of independent replicas
// (a single system is a batch of one), one cooperative launch for all
// sweeps of a call.
//
// Replica r owns workgroups [g0, g0 + G) of the grid.  Per stage (w, s):
//   1. every workgroup draws the stage colour (Philox (w, s, 0, 0)) and makes
//      the trials of its share of the replica's active cells (TL lanes per
//      trial, the same arithmetic as the per-stage kernels): local factor of
//      Eq. trans_vcsgc_par1, record of the locally accepted site;
//   2. its partial sums (trials, accepts, sum of dn, near ties) are published
//      and the replica's workgroups meet at a barrier;
//   3. every workgroup sums the partials in workgroup order and evaluates the
//      same global factor of Eq. trans_vcsgc_par2 (identical decision);
//   4. it commits its own accepted records (species, density cache, velocity
//      rescaling); workgroup 0 of the replica advances n_B and the counters;
//   5. second barrier, so the next stage reads the committed state.
// A replica with one workgroup synchronizes with __syncthreads only.
// Barrier waits are bounded: a wait that exceeds the spin limit sets the
// replica's error flag and the workgroup leaves the kernel, so the launch
// always drains.
#include "common.hpp"

namespace vc {

constexpr int PTL = 16;                 // lanes per trial
constexpr int PGROUPS = BLOCK / PTL;    // trials per workgroup pass
static_assert(KMAX <= 2 * PTL, "a trial group covers at most 2*PTL neighbours");

struct RepD {
  int64_t n, aoff;
  int n0, n1, n2;
  int per, ncol;  // colour period per axis, colours
  int64_t cso, ncpc, roff, S;
  double beta, dmu0, kN, ncbar;
  uint64_t seed, key1;
  int g0, G;
  int64_t n_sweeps, w0;
};

struct RepState {
  long long n_b[2];
  unsigned long long trials, local_acc, stages, stage_acc, flips, near_ties;
  double sum_n, sum_n2;
  // 64-bit arrival counter: it grows by G per barrier (two barriers per
  // stage) and is zeroed only once per call, so a 32-bit counter would wrap
  // within one long call (2 S G per sweep)
  unsigned long long bar;
  int err;
  long long n_final;
};

struct PersistArgs {
  const RepD *reps;
  RepState *rs;
  const int32_t *wg_rep;
  const int32_t *cstart, *catoms, *nj;
  const double *nr;  // r of each r < rc entry
  const uint8_t *cnt;
  uint8_t *sp;
  double *rho;
  double *vx, *vy, *vz;
  int32_t *rec;
  long long *part;  // [grid][NPART]
  PotD p;
  double *tlog;
  int64_t tcap;
  double *slog;
  int64_t scap;
  unsigned long long *log_n;  // [2]: trial and stage records written
  unsigned int spin_limit;
};

// Barrier of the G workgroups of one replica on a monotonically increasing
// counter; returns false if the wait timed out.
__device__ __forceinline__ bool rep_barrier(RepState *st, int G, unsigned long long target,
                                            unsigned int spin_limit, int *flag) {
  if (G == 1) {
    __syncthreads();
    return true;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *flag = 0;
    // one release on arrival (writes back this CU's dirty L2 lines once) ...
    __hip_atomic_fetch_add(&st->bar, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    // ... polling with relaxed device-coherent loads (an acquiring load would
    // invalidate the caches on every poll) ...
    unsigned int it = 0;
    while (__hip_atomic_load(&st->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++it > spin_limit) {
        __hip_atomic_fetch_or(&st->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *flag = 1;
        break;
      }
    }
    // ... and one acquire once the count is reached
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return *flag == 0;
}

__device__ __forceinline__ int64_t p_colour_cell(const RepD &r, int colour, int64_t t) {
  const int P = r.per;
  const int hx = r.n0 / P, hy = r.n1 / P;
  const int64_t ia = t % hx, ib = (t / hx) % hy, ic = t / ((int64_t)hx * hy);
  const int64_t cx = P * ia + colour % P, cy = P * ib + (colour / P) % P,
                cz = P * ic + colour / (P * P);
  return cx + (int64_t)r.n0 * (cy + (int64_t)r.n1 * cz);
}

// transmutation energy change by the PTL lanes of a group (in-order sums of
// the terms the lanes leave in the group's LDS slots; a group is 16 lanes of
// one wave, whose LDS accesses are performed in order)
template <int F>
__device__ __forceinline__ double p_delta_u(const PersistArgs &a, int64_t i, int lane,
                                            double2 *grp) {
  const int s = a.sp[i];
  const double ri = a.rho[i];
  const int m = a.cnt[i];
  double tp[2] = {0.0, 0.0}, te[2] = {0.0, 0.0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = lane + h * PTL;
    if (k < m) {
      const int64_t e = i * KMAX + k;
      const int32_t j = a.nj[e];
      const int sj = a.sp[j];
      const double r = a.nr[e];
      const double rj = a.rho[j];
      tp[h] = flip_pair_term<F>(a.p, s, sj, r);
      te[h] = flip_embed_term<F>(a.p, sj, rj, flip_rho_shift<F>(a.p, s, r));
    }
  }
  grp[lane] = make_double2(tp[0], te[0]);
  grp[lane + PTL] = make_double2(tp[1], te[1]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double pair, emb;
  sum_flip_terms(grp, m, pair, emb);
  const double own = flip_own_term<F>(a.p, s, ri);
  return own + pair + emb;
}

// TAB: the potential's form (analytic or tabulated) fixed at compile time,
// so each variant keeps only its own arithmetic and registers.
template <bool TAB>
__global__ void __launch_bounds__(BLOCK) k_sweep_persistent(PersistArgs a) {
  constexpr int F = TAB ? 1 : 0;
  __shared__ long long sh[BLOCK];
  __shared__ double2 pterms[PGROUPS][KMAX];
  __shared__ int bflag;
  const int g = blockIdx.x;
  const int rix = a.wg_rep[g];
  const RepD r = a.reps[rix];
  RepState *st = a.rs + rix;
  const int q = g - r.g0;  // rank inside the replica
  const int lane = threadIdx.x % PTL, grp = threadIdx.x / PTL;
  // contiguous share of the active cells; consecutive shares on one XCD
  // (workgroup ids advance round-robin over the 8 XCDs)
  int qc = q;
  if ((r.G & 7) == 0 && (r.g0 & 7) == 0) qc = (q & 7) * (r.G >> 3) + (q >> 3);
  const int64_t chunk = (r.ncpc + r.G - 1) / r.G;
  const int64_t t_lo = (int64_t)qc * chunk;
  const int64_t t_hi = t_lo + chunk < r.ncpc ? t_lo + chunk : r.ncpc;
  const int32_t *cstart = a.cstart + r.cso;
  const int32_t *catoms = a.catoms + r.aoff;
  int32_t *rec = a.rec + r.roff;
  unsigned long long nbar = 0;
  int64_t stage_no = 0;

  for (int64_t sw = 0; sw < r.n_sweeps; ++sw) {
    const uint64_t w = (uint64_t)(r.w0 + sw);
    for (int64_t s = 0; s < r.S; ++s, ++stage_no) {
      const int par = (int)(stage_no & 1);
      const U4 gs = philox(r.seed, r.key1, w, (uint64_t)s, 0, 0);
      const int colour = stage_colour(gs.v[0], r.ncol);
      long long valid = 0, acc = 0, dn_acc = 0, tie = 0;
      // ---- trials
      for (int64_t t = t_lo + grp; t < t_hi; t += PGROUPS) {
        const int64_t cell = p_colour_cell(r, colour, t);
        const int32_t c0 = cstart[cell];
        const uint32_t m = (uint32_t)(cstart[cell + 1] - c0);
        int32_t site = -1;
        if (m > 0) {
          const U4 rr = philox(r.seed, r.key1, w, (uint64_t)s, (uint64_t)cell, 1);
          const int64_t i = catoms[c0 + draw_index(rr.v[0], m)];
          const double du = p_delta_u<F>(a, i, lane, pterms[grp]);
          if (lane == 0) {
            const double u = unit_open(rr.v[1]);
            const int dn = 1 - 2 * (int)a.sp[i];
            const double xl = r.beta * (du + r.dmu0 * (double)dn);
            const double lnu = log(u);
            const double margin = lnu + xl;
            const bool ok = lnu < -xl;
            valid += 1;
            tie += fabs(margin) < TIE ? 1 : 0;
            if (ok) {
              acc += 1;
              dn_acc += dn;
              site = (int32_t)i;
            }
            if (a.tlog) {
              const unsigned long long idx = atomicAdd(&a.log_n[0], 1ull);
              if ((int64_t)idx < a.tcap) {
                double *L = a.tlog + 8 * idx;
                L[0] = (double)w;
                L[1] = (double)s;
                L[2] = (double)cell;
                L[3] = (double)(i - r.aoff);
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
      long long v4[4] = {valid, acc, dn_acc, tie};
      block_sums<4>(v4, sh);
      if (threadIdx.x == 0) {
        long long *P = a.part + NPART * (int64_t)g;
        P[0] = v4[0];
        P[1] = v4[1];
        P[2] = v4[2];
        P[3] = v4[3];
      }
      nbar += 1;
      if (!rep_barrier(st, r.G, nbar * (unsigned long long)r.G, a.spin_limit, &bflag)) return;
      // ---- global factor, identical in every workgroup of the replica
      long long pa = 0, pd = 0, pv = 0, pt = 0;
      for (int k = threadIdx.x; k < r.G; k += BLOCK) {
        const long long *P = a.part + NPART * (int64_t)(r.g0 + k);
        pv += P[0];
        pa += P[1];
        pd += P[2];
        pt += P[3];
      }
      long long r4[4] = {pa, pd, pv, pt};
      block_sums<4>(r4, sh);
      const long long nrec = r4[0], dn_tot = r4[1];
      const long long nb = st->n_b[par];
      int gacc = -1;
      double xg = 0.0, mg = 0.0;
      if (nrec > 0) {
        const double tt = (double)nb - r.ncbar;
        const double dnd = (double)dn_tot;
        xg = r.beta * r.kN * dnd * (dnd + 2.0 * tt);
        const double lnug = log(unit_open(gs.v[1]));
        mg = lnug + xg;
        gacc = lnug < -xg ? 1 : 0;
      }
      // ---- commit own records
      if (gacc == 1) {
        for (int64_t t = t_lo + grp; t < t_hi; t += PGROUPS) {
          const int32_t i = rec[t];
          if (i < 0) continue;
          const int s0 = a.sp[i], s1 = 1 - s0;
          const int m = a.cnt[i];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int k = lane + h * PTL;
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
      }
      const long long sv = r4[2], stt = r4[3];
      if (q == 0 && threadIdx.x == 0) {
        const long long nb_new = nb + (gacc == 1 ? dn_tot : 0);
        st->n_b[par ^ 1] = nb_new;
        st->trials += (unsigned long long)sv;
        st->local_acc += (unsigned long long)nrec;
        st->near_ties += (unsigned long long)stt;
        st->stages += 1;
        if (gacc == 1) {
          st->stage_acc += 1;
          st->flips += (unsigned long long)nrec;
        }
        if (nrec > 0 && fabs(mg) < TIE) st->near_ties += 1;
        if (s == r.S - 1) {
          st->sum_n += (double)nb_new;
          st->sum_n2 += (double)nb_new * (double)nb_new;
        }
        st->n_final = nb_new;
        if (a.slog) {
          const unsigned long long idx = atomicAdd(&a.log_n[1], 1ull);
          if ((int64_t)idx < a.scap) {
            double *L = a.slog + 8 * idx;
            L[0] = (double)w;
            L[1] = (double)s;
            L[2] = (double)colour;
            L[3] = (double)dn_tot;
            L[4] = (double)nrec;
            L[5] = (double)gacc;
            L[6] = xg;
            L[7] = mg;
          }
        }
      }
      nbar += 1;
      if (!rep_barrier(st, r.G, nbar * (unsigned long long)r.G, a.spin_limit, &bflag)) return;
    }
  }
}

// zero the barrier counters, the timeout flag and the per-call counters;
// n_b[0] <- current n_B
__global__ void k_persist_reset(RepState *rs, int R) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= R) return;
  RepState &s = rs[k];
  s.n_b[0] = s.n_final;
  s.n_b[1] = s.n_final;
  s.trials = s.local_acc = s.stages = s.stage_acc = s.flips = s.near_ties = 0;
  s.sum_n = 0.0;
  s.sum_n2 = 0.0;
  s.bar = 0;
  s.err = 0;
}

}  // namespace vc

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace vc {

int persist_block() { return BLOCK; }
int persist_groups() { return PGROUPS; }
size_t repd_size() { return sizeof(RepD); }
size_t repstate_size() { return sizeof(RepState); }

static const void *persist_kernel(bool tab) {
  return tab ? (const void *)k_sweep_persistent<true> : (const void *)k_sweep_persistent<false>;
}

hipError_t persist_max_blocks(int *per_cu, bool tab) {
  return tab ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_sweep_persistent<true>,
                                                             BLOCK, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_sweep_persistent<false>,
                                                             BLOCK, 0);
}

static PersistArgs make_args(vcsgc_ctx *c) {
  PersistArgs a;
  a.reps = (const RepD *)c->d_reps;
  a.rs = (RepState *)c->d_rs;
  a.wg_rep = c->d_wg_rep;
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
  a.p = c->pot;
  a.tlog = c->tlog;
  a.tcap = c->tcap;
  a.slog = c->slog;
  a.scap = c->scap;
  a.log_n = &c->ds->tlog_n;
  a.spin_limit = c->spin_limit;
  return a;
}

// Fill the per-call replica parameters (pinned staging buffer) and copy them
// to the device; the previous call's copy must have completed before the
// staging buffer is rewritten.
hipError_t persist_stage_params(vcsgc_ctx *c, const double *dmu0, const double *kappa,
                                const double *cbar, const double *T, int64_t n_sweeps,
                                uint64_t seed) {
  hipError_t e = hipEventSynchronize(c->stage_ev);
  if (e != hipSuccess) return e;
  RepD *h = (RepD *)c->h_reps;
  for (size_t k = 0; k < c->reps.size(); ++k) {
    const RepHost &r = c->reps[k];
    RepD &d = h[k];
    d.n = r.n;
    d.aoff = r.aoff;
    d.n0 = r.nc[0];
    d.per = c->per;
    d.ncol = c->ncol;
    d.n1 = r.nc[1];
    d.n2 = r.nc[2];
    d.cso = r.cso;
    d.ncpc = r.ncpc;
    d.roff = r.roff;
    d.S = r.S;
    d.beta = 1.0 / (KB * T[k]);
    d.dmu0 = dmu0[k];
    d.kN = kappa[k] / (double)r.n;
    d.ncbar = (double)r.n * cbar[k];
    d.seed = seed;
    d.key1 = (uint64_t)k;
    d.g0 = r.g0;
    d.G = r.G;
    d.n_sweeps = n_sweeps;
    d.w0 = (int64_t)c->w;
  }
  e = hipMemcpyAsync(c->d_reps, h, sizeof(RepD) * c->reps.size(), hipMemcpyHostToDevice,
                     c->stream);
  if (e != hipSuccess) return e;
  return hipEventRecord(c->stage_ev, c->stream);
}

static hipError_t build_graph(vcsgc_ctx *c) {
  if (c->graph_exec) {
    (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
  }
  if (c->graph) {
    (void)hipGraphDestroy(c->graph);
    c->graph = nullptr;
  }
  hipError_t e = hipGraphCreate(&c->graph, 0);
  if (e != hipSuccess) return e;
  const int R = (int)c->reps.size();
  RepState *rs = (RepState *)c->d_rs;
  int Rv = R;
  void *rargs[] = {&rs, &Rv};
  hipKernelNodeParams rp = {};
  rp.func = (void *)k_persist_reset;
  rp.gridDim = dim3((unsigned)grid_for(R));
  rp.blockDim = dim3(BLOCK);
  rp.kernelParams = rargs;
  hipGraphNode_t n_reset, n_sweep;
  e = hipGraphAddKernelNode(&n_reset, c->graph, nullptr, 0, &rp);
  if (e != hipSuccess) return e;
  static_assert(sizeof(PersistArgs) <= sizeof(c->graph_args_storage), "argument storage");
  PersistArgs *ga = reinterpret_cast<PersistArgs *>(c->graph_args_storage);
  *ga = make_args(c);
  void *sargs[] = {ga};
  hipKernelNodeParams sp = {};
  sp.func = const_cast<void *>(persist_kernel(c->pot.tab != 0));
  sp.gridDim = dim3((unsigned)c->grid_total);
  sp.blockDim = dim3(BLOCK);
  sp.kernelParams = sargs;
  e = hipGraphAddKernelNode(&n_sweep, c->graph, &n_reset, 1, &sp);
  if (e != hipSuccess) return e;
  hipLaunchAttributeValue v = {};
  v.cooperative = 1;
  c->graph_coop = hipGraphKernelNodeSetAttribute(n_sweep, hipLaunchAttributeCooperative, &v) ==
                  hipSuccess;
  (void)hipGetLastError();
  e = hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return e;
  c->graph_args_tlog = c->tlog;
  c->graph_args_slog = c->slog;
  return hipSuccess;
}

hipError_t launch_persistent(vcsgc_ctx *c, bool use_graph) {
  const int R = (int)c->reps.size();
  if (use_graph) {
    if (!c->graph_exec || c->graph_args_tlog != c->tlog || c->graph_args_slog != c->slog) {
      hipError_t e = build_graph(c);
      if (e != hipSuccess) return e;
    }
    return hipGraphLaunch(c->graph_exec, c->stream);
  }
  k_persist_reset<<<grid_for(R), BLOCK, 0, c->stream>>>((RepState *)c->d_rs, R);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  PersistArgs a = make_args(c);
  void *args[] = {&a};
  return hipLaunchCooperativeKernel(persist_kernel(c->pot.tab != 0), dim3((unsigned)c->grid_total),
                                    dim3(BLOCK), args, 0, c->stream);
}

// per-replica statistics after the call (synchronizes)
hipError_t persist_read_stats(vcsgc_ctx *c, vcsgc_stats *out, int *err) {
  const int R = (int)c->reps.size();
  std::vector<RepState> h(R);
  hipError_t e = hipMemcpyAsync(h.data(), c->d_rs, sizeof(RepState) * R, hipMemcpyDeviceToHost,
                                c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  *err = 0;
  for (int k = 0; k < R; ++k) {
    if (h[k].err) *err = 1;
    if (!out) continue;
    out[k].trials = (int64_t)h[k].trials;
    out[k].local_accepts = (int64_t)h[k].local_acc;
    out[k].stages = (int64_t)h[k].stages;
    out[k].stage_accepts = (int64_t)h[k].stage_acc;
    out[k].flips = (int64_t)h[k].flips;
    out[k].near_ties = (int64_t)h[k].near_ties;
    out[k].n_final = h[k].n_final;
    out[k].sum_n = h[k].sum_n;
    out[k].sum_n2 = h[k].sum_n2;
    out[k].stage1_pass = (int64_t)h[k].trials;
  }
  return hipSuccess;
}

// n_final of replica k (used to seed the per-stage path's counter)
__global__ void k_set_nfinal(RepState *rs, int k, const long long *src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) rs[k].n_final = *src;
}
__global__ void k_get_nfinal(const RepState *rs, int k, long long *dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = rs[k].n_final;
}

hipError_t persist_sync_nb_to_stage(vcsgc_ctx *c) {
  k_get_nfinal<<<1, 64, 0, c->stream>>>((const RepState *)c->d_rs, 0, &c->ds->n_b_cur);
  return hipGetLastError();
}
hipError_t persist_sync_nb_from_stage(vcsgc_ctx *c) {
  k_set_nfinal<<<1, 64, 0, c->stream>>>((RepState *)c->d_rs, 0, &c->ds->n_b_cur);
  return hipGetLastError();
}

// per-replica n_B from the species (into n_final)
__global__ void k_count_rep(int64_t n, const uint8_t *__restrict__ sp, RepState *st) {
  __shared__ long long sh[BLOCK];
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  sh[threadIdx.x] = i < n ? (long long)sp[i] : 0;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && sh[0])
    atomicAdd((unsigned long long *)&st->n_final, (unsigned long long)sh[0]);
}

hipError_t persist_count(vcsgc_ctx *c) {
  hipError_t e = hipMemsetAsync(c->d_rs, 0, sizeof(RepState) * c->reps.size(), c->stream);
  if (e != hipSuccess) return e;
  for (size_t k = 0; k < c->reps.size(); ++k) {
    const RepHost &r = c->reps[k];
    k_count_rep<<<grid_for(r.n), BLOCK, 0, c->stream>>>(r.n, c->sp + r.aoff,
                                                        (RepState *)c->d_rs + k);
  }
  return hipGetLastError();
}

}  // namespace vc
