// C ABI: context lifecycle, argument validation, scratch management and the
// host side of the sweep / EAM / MD calls.  See include/vcsgc.h.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "common.hpp"

namespace {

std::string g_create_error;

template <typename T>
hipError_t dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void **)p, sizeof(T) * count);
}

void free_all(vcsgc_ctx *c) {
  void *ptrs[] = {c->bin_count,  c->bin_atoms,  c->cell_count, c->cell_start, c->cell_atoms,
                  c->cell_fill,  c->mc_j,       c->mc_dd,
                  c->mc_g,       c->mc_cnt,     c->md_j,       c->md_cnt,    c->xr,   c->yr,
                  c->zr,         c->rho,        c->rho_f,      c->fp,        c->eatom, c->red,
                  c->rec,        c->ds,         c->ps4,        c->pf4,       c->part};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
}

vcsgc_status fail(vcsgc_ctx *c, vcsgc_status st, const std::string &msg) {
  if (c) {
    c->err = msg;
    if (st == VCSGC_E_DEVICE) c->sticky = true;
  } else {
    g_create_error = msg;
  }
  return st;
}

vcsgc_status dev_fail(vcsgc_ctx *c, hipError_t e, const char *where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, VCSGC_E_DEVICE, m);
}

#define VC_CHECK(ctx, expr, where)                      \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return dev_fail(ctx, _e, where); \
  } while (0)

bool is_fin(double v) { return std::isfinite(v); }

__global__ void k_count_b(int64_t n, const uint8_t *__restrict__ sp, vc::DevState *ds) {
  __shared__ long long sh[vc::BLOCK];
  const int64_t i = (int64_t)blockIdx.x * vc::BLOCK + threadIdx.x;
  sh[threadIdx.x] = i < n ? (long long)sp[i] : 0;
  __syncthreads();
  for (int h = vc::BLOCK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && sh[0]) atomicAdd((unsigned long long *)&ds->n_b_cur,
                                           (unsigned long long)sh[0]);
}

vc::DevState read_state(vcsgc_ctx *c, hipError_t *e) {
  vc::DevState h;
  std::memset(&h, 0, sizeof(h));
  *e = hipMemcpyAsync(&h, c->ds, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (*e == hipSuccess) *e = hipStreamSynchronize(c->stream);
  return h;
}

// Grow the search bins after an overflow (capacity doubles).
vcsgc_status grow_bins(vcsgc_ctx *c) {
  if (c->bmax >= 1024) return fail(c, VCSGC_E_OVERFLOW, "more than 1024 atoms in a search bin");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  (void)hipFree(c->bin_atoms);
  c->bin_atoms = nullptr;
  c->bmax *= 2;
  VC_CHECK(c, dalloc(&c->bin_atoms, (size_t)c->nbins * c->bmax), "allocation");
  int zero = 0;
  VC_CHECK(c, hipMemcpyAsync(&c->ds->bin_overflow, &zero, sizeof(int), hipMemcpyHostToDevice,
                             c->stream),
           "reset");
  return VCSGC_OK;
}

// Rebuild cells + the r < rc list + the density cache; checks row overflow.
vcsgc_status refresh_mc(vcsgc_ctx *c) {
  for (;;) {
    VC_CHECK(c, vc::launch_bin_cells(c), "binning");
    VC_CHECK(c, vc::launch_bin_search(c), "binning");
    VC_CHECK(c, vc::launch_build_mc_list(c), "neighbour list");
    VC_CHECK(c, vc::launch_density_mc(c), "density");
    hipError_t e;
    vc::DevState h = read_state(c, &e);
    if (e != hipSuccess) return dev_fail(c, e, "neighbour list");
    if (h.bin_overflow) {
      vcsgc_status st = grow_bins(c);
      if (st) return st;
      continue;
    }
    if (h.overflow)
      return fail(c, VCSGC_E_OVERFLOW, "a site has more than 32 neighbours within rc");
    c->kmax_used = h.kmax_used;
    c->mc_valid = true;
    return VCSGC_OK;
  }
}

vcsgc_status refresh_md(vcsgc_ctx *c) {
  for (;;) {
    VC_CHECK(c, vc::launch_bin_search(c), "binning");
    VC_CHECK(c, vc::launch_build_md_list(c), "neighbour list (MD)");
    hipError_t e;
    vc::DevState h = read_state(c, &e);
    if (e != hipSuccess) return dev_fail(c, e, "neighbour list (MD)");
    if (h.bin_overflow) {
      vcsgc_status st = grow_bins(c);
      if (st) return st;
      continue;
    }
    if (h.overflow)
      return fail(c, VCSGC_E_OVERFLOW, "a site has more than 32 neighbours within rc + skin");
    c->md_valid = true;
    c->md_rebuilds += 1;
    return VCSGC_OK;
  }
}

vcsgc_status check_ctx(vcsgc_ctx *c) {
  if (!c) return VCSGC_E_INVALID_ARG;
  if (c->sticky) return VCSGC_E_STATE;
  (void)hipSetDevice(c->device);
  return VCSGC_OK;
}

}  // namespace

namespace vc {

int tstart(vcsgc_ctx *c, int cls) {
  if (!(c->tmask & (1u << cls))) return -1;
  hipEvent_t ev[2];
  for (int k = 0; k < 2; ++k) {
    if (!c->ev_pool.empty()) {
      ev[k] = c->ev_pool.back();
      c->ev_pool.pop_back();
    } else if (hipEventCreate(&ev[k]) != hipSuccess) {
      if (k == 1) c->ev_pool.push_back(ev[0]);
      return -1;
    }
  }
  if (hipEventRecord(ev[0], c->stream) != hipSuccess) {
    c->ev_pool.push_back(ev[0]);
    c->ev_pool.push_back(ev[1]);
    return -1;
  }
  c->ev_pending.push_back({cls, ev[0], ev[1]});
  return (int)c->ev_pending.size() - 1;
}

void tstop(vcsgc_ctx *c, int h) {
  if (h < 0) return;
  (void)hipEventRecord(c->ev_pending[h].b, c->stream);
}

}  // namespace vc

namespace {

// fold pending event pairs into the per-class totals (synchronizes)
hipError_t drain_timers(vcsgc_ctx *c) {
  if (c->ev_pending.empty()) return hipSuccess;
  hipError_t e = hipStreamSynchronize(c->stream);
  for (auto &p : c->ev_pending) {
    float ms = 0.f;
    if (e == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->kt_ms[p.cls] += ms;
      c->kt_n[p.cls] += 1;
    }
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->ev_pending.clear();
  return e;
}

}  // namespace

extern "C" {

vcsgc_status vcsgc_kernel_timing(vcsgc_ctx *c, uint32_t mask) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  VC_CHECK(c, drain_timers(c), "timing");
  c->tmask = mask & ((1u << VCSGC_KT_CLASSES) - 1);
  for (int k = 0; k < VCSGC_KT_CLASSES; ++k) {
    c->kt_ms[k] = 0.0;
    c->kt_n[k] = 0;
  }
  return VCSGC_OK;
}

vcsgc_status vcsgc_get_kernel_timing(vcsgc_ctx *c, vcsgc_ktimes *out) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!out) return fail(c, VCSGC_E_INVALID_ARG, "null output");
  VC_CHECK(c, drain_timers(c), "timing");
  for (int k = 0; k < VCSGC_KT_CLASSES; ++k) {
    out->total_ms[k] = c->kt_ms[k];
    out->count[k] = c->kt_n[k];
  }
  return VCSGC_OK;
}

vcsgc_status vcsgc_create(const vcsgc_system *sys, hipStream_t stream, vcsgc_ctx **out) {
  if (!sys || !out) return fail(nullptr, VCSGC_E_INVALID_ARG, "null argument");
  const vcsgc_eam_fs &P = sys->pot;
  if (sys->n_atoms < 2 || sys->n_atoms > (int64_t)0x7fffffff)
    return fail(nullptr, VCSGC_E_INVALID_ARG, "n_atoms must be in [2, 2^31)");
  if (!sys->x || !sys->y || !sys->z || !sys->species)
    return fail(nullptr, VCSGC_E_INVALID_ARG, "positions and species are required");
  for (int d = 0; d < 3; ++d)
    if (!(sys->box[d] > 0.0) || !is_fin(sys->box[d]))
      return fail(nullptr, VCSGC_E_INVALID_ARG, "box edges must be positive and finite");
  const double pv[] = {P.rc, P.c0, P.c1, P.eps_aa, P.eps_ab, P.eps_bb, P.t_a, P.t_b, P.a_a, P.a_b};
  for (double v : pv)
    if (!is_fin(v)) return fail(nullptr, VCSGC_E_INVALID_ARG, "non-finite potential parameter");
  if (!(P.rc > 0.0)) return fail(nullptr, VCSGC_E_INVALID_ARG, "rc must be positive");
  if (!(sys->skin >= 0.0) || !is_fin(sys->skin) || sys->skin > P.rc)
    return fail(nullptr, VCSGC_E_INVALID_ARG, "skin must be in [0, rc]");
  const bool has_v = sys->vx || sys->vy || sys->vz;
  if (has_v && !(sys->vx && sys->vy && sys->vz))
    return fail(nullptr, VCSGC_E_INVALID_ARG, "velocities must be all set or all NULL");
  const bool has_f = sys->fx || sys->fy || sys->fz;
  if (has_f && !(sys->fx && sys->fy && sys->fz))
    return fail(nullptr, VCSGC_E_INVALID_ARG, "forces must be all set or all NULL");
  if (has_v && (!(P.mass_a > 0.0) || !(P.mass_b > 0.0) || !is_fin(P.mass_a) || !is_fin(P.mass_b)))
    return fail(nullptr, VCSGC_E_INVALID_ARG, "masses must be positive with velocities");
  double r_dep = sys->r_dep == 0.0 ? 2.0 * P.rc : sys->r_dep;
  if (!(r_dep >= 2.0 * P.rc) || !is_fin(r_dep))
    return fail(nullptr, VCSGC_E_INVALID_ARG, "r_dep must be >= 2 rc");

  int nc[3];
  for (int d = 0; d < 3; ++d) {
    nc[d] = 2 * (int)std::floor(sys->box[d] / (2.0 * r_dep));
    if (nc[d] < 2)
      return fail(nullptr, VCSGC_E_BOX_TOO_SMALL,
                  "box must hold two cells of edge r_dep in every dimension");
  }

  vcsgc_ctx *c = new vcsgc_ctx();
  (void)hipGetDevice(&c->device);
  c->stream = stream;
  c->n = sys->n_atoms;
  for (int d = 0; d < 3; ++d) {
    c->box[d] = sys->box[d];
    c->nc[d] = nc[d];
  }
  c->x = sys->x;
  c->y = sys->y;
  c->z = sys->z;
  c->vx = sys->vx;
  c->vy = sys->vy;
  c->vz = sys->vz;
  c->fx = sys->fx;
  c->fy = sys->fy;
  c->fz = sys->fz;
  c->sp = sys->species;
  c->skin = sys->skin;
  c->r_dep = r_dep;
  vc::PotD &p = c->pot;
  p.rc = P.rc;
  p.c0 = P.c0;
  p.c1 = P.c1;
  p.eps[0] = P.eps_aa;
  p.eps[1] = P.eps_ab;
  p.eps[2] = P.eps_bb;
  p.t[0] = P.t_a;
  p.t[1] = P.t_b;
  p.A[0] = P.a_a;
  p.A[1] = P.a_b;
  p.mass[0] = P.mass_a;
  p.mass[1] = P.mass_b;
  p.cm[0] = P.mass_a > 0.0 ? vc::ACC / P.mass_a : 0.0;
  p.cm[1] = P.mass_b > 0.0 ? vc::ACC / P.mass_b : 0.0;
  c->ncells = (int64_t)nc[0] * nc[1] * nc[2];
  c->S = 8 * ((c->n + c->ncells - 1) / c->ncells);
  for (int d = 0; d < 3; ++d) c->nb[d] = (int)std::floor(sys->box[d] / (P.rc + sys->skin));
  c->nbins = (int64_t)c->nb[0] * c->nb[1] * c->nb[2];
  c->bmax = 16;

  const int64_t n = c->n, K = vc::KMAX;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  A(dalloc(&c->bin_count, c->nbins));
  A(dalloc(&c->bin_atoms, c->nbins * c->bmax));
  A(dalloc(&c->cell_count, c->ncells));
  A(dalloc(&c->cell_start, c->ncells + 1));
  A(dalloc(&c->cell_fill, c->ncells));
  A(dalloc(&c->cell_atoms, n));
  A(dalloc(&c->mc_j, K * n));
  A(dalloc(&c->mc_dd, K * n));
  A(dalloc(&c->mc_g, K * n));
  A(dalloc(&c->mc_cnt, n));
  A(dalloc(&c->md_j, K * n));
  A(dalloc(&c->md_cnt, n));
  A(dalloc(&c->xr, n));
  A(dalloc(&c->yr, n));
  A(dalloc(&c->zr, n));
  A(dalloc(&c->ps4, n));
  A(dalloc(&c->pf4, n));
  A(dalloc(&c->rho, n));
  A(dalloc(&c->rho_f, n));
  A(dalloc(&c->fp, n));
  A(dalloc(&c->eatom, n));
  A(dalloc(&c->red, (n + vc::BLOCK - 1) / vc::BLOCK + 8));
  A(dalloc(&c->rec, c->ncells / 8));
  c->npart = (c->ncells / 8 * 16 + vc::BLOCK - 1) / vc::BLOCK;
  A(dalloc(&c->part, 4 * c->npart));
  A(dalloc(&c->ds, 1));
  if (e != hipSuccess) {
    free_all(c);
    delete c;
    (void)hipGetLastError();
    return fail(nullptr, e == hipErrorOutOfMemory ? VCSGC_E_OUT_OF_MEMORY : VCSGC_E_DEVICE,
                std::string("allocation: ") + hipGetErrorString(e));
  }
  auto bail = [&](vcsgc_status st) {
    g_create_error = c->err;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
    return st;
  };
  if ((e = hipMemsetAsync(c->ds, 0, sizeof(vc::DevState), c->stream)) != hipSuccess)
    return bail(dev_fail(c, e, "init"));
  if ((e = vc::launch_validate(c)) != hipSuccess) return bail(dev_fail(c, e, "validate"));
  {
    hipError_t e2;
    vc::DevState h = read_state(c, &e2);
    if (e2 != hipSuccess) return bail(dev_fail(c, e2, "validate"));
    if (h.bad_input)
      return bail(fail(c, VCSGC_E_INVALID_ARG,
                       "positions must lie in [0, L) and species in {0, 1}"));
  }
  k_count_b<<<vc::grid_for(n), vc::BLOCK, 0, c->stream>>>(n, c->sp, c->ds);
  if ((e = hipGetLastError()) != hipSuccess) return bail(dev_fail(c, e, "count"));
  vcsgc_status st = refresh_mc(c);
  if (st != VCSGC_OK) return bail(st);
  *out = c;
  return VCSGC_OK;
}

vcsgc_status vcsgc_destroy(vcsgc_ctx *c) {
  if (!c) return VCSGC_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto &p : c->ev_pending) {
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  for (hipEvent_t ev : c->ev_pool) (void)hipEventDestroy(ev);
  free_all(c);
  delete c;
  return VCSGC_OK;
}

const char *vcsgc_last_error(const vcsgc_ctx *c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

vcsgc_status vcsgc_sweep(vcsgc_ctx *c, double dmu0, double kappa, double cbar, double T_K,
                         int64_t n_sweeps, uint64_t seed, vcsgc_stats *out) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!is_fin(dmu0) || !is_fin(kappa) || !(kappa >= 0.0) || !is_fin(cbar) || cbar < 0.0 ||
      cbar > 1.0 || !is_fin(T_K) || !(T_K > 0.0) || n_sweeps < 0)
    return fail(c, VCSGC_E_INVALID_ARG,
                "need finite dmu0, kappa >= 0, cbar in [0,1], T > 0, n_sweeps >= 0");
  if (!c->mc_valid) {
    st = refresh_mc(c);
    if (st) return st;
  }
  VC_CHECK(c, vc::launch_sweeps(c, dmu0, kappa, cbar, T_K, n_sweeps, seed), "sweep");
  c->w += (uint64_t)n_sweeps;
  if (out) {
    hipError_t e;
    vc::DevState h = read_state(c, &e);
    if (e != hipSuccess) return dev_fail(c, e, "sweep");
    out->trials = (int64_t)h.trials;
    out->local_accepts = (int64_t)h.local_acc;
    out->stages = (int64_t)h.stages;
    out->stage_accepts = (int64_t)h.stage_acc;
    out->flips = (int64_t)h.flips;
    out->near_ties = (int64_t)h.near_ties;
    out->n_final = h.n_b_cur;
    out->sum_n = h.sum_n;
    out->sum_n2 = h.sum_n2;
  }
  return VCSGC_OK;
}

vcsgc_status eam_energy_forces(vcsgc_ctx *c, double *energy_eV, int want_forces) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (want_forces && !c->fx)
    return fail(c, VCSGC_E_INVALID_ARG, "forces requested but the system has no force arrays");
  if (!c->md_valid) {
    st = refresh_md(c);
    if (st) return st;
  }
  VC_CHECK(c, vc::launch_pack(c), "pack");
  VC_CHECK(c, vc::launch_energy(c), "energy");
  if (want_forces) VC_CHECK(c, vc::launch_forces(c), "forces");
  if (energy_eV) {
    VC_CHECK(c, vc::launch_reduce_sum(c, c->eatom, c->n, c->red + (c->n + vc::BLOCK - 1) / vc::BLOCK + 1),
             "reduce");
    double h = 0.0;
    VC_CHECK(c, hipMemcpyAsync(&h, c->red + (c->n + vc::BLOCK - 1) / vc::BLOCK + 1, sizeof(double),
                               hipMemcpyDeviceToHost, c->stream),
             "copy");
    VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
    *energy_eV = h;
  }
  return VCSGC_OK;
}

vcsgc_status md_verlet_step(vcsgc_ctx *c, double dt_fs, int64_t n_steps) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!c->vx || !c->fx)
    return fail(c, VCSGC_E_INVALID_ARG, "MD needs velocity and force arrays");
  if (!is_fin(dt_fs) || !(dt_fs > 0.0) || n_steps < 0)
    return fail(c, VCSGC_E_INVALID_ARG, "need dt > 0 and n_steps >= 0");
  if (!c->md_valid) {
    st = refresh_md(c);
    if (st) return st;
  }
  VC_CHECK(c, vc::launch_pack(c), "pack");
  VC_CHECK(c, vc::launch_forces(c), "forces");
  for (int64_t k = 0; k < n_steps; ++k) {
    // the closing half-kick of step k-1 is fused into the opening one of step k
    VC_CHECK(c, vc::launch_kick_drift(c, dt_fs, k > 0), "kick-drift");
    int flag = 0;
    VC_CHECK(c, hipMemcpyAsync(&flag, &c->ds->rebuild, sizeof(int), hipMemcpyDeviceToHost,
                               c->stream),
             "copy");
    VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
    c->mc_valid = false;
    if (flag) {
      VC_CHECK(c, hipMemsetAsync(&c->ds->rebuild, 0, sizeof(int), c->stream), "reset");
      st = refresh_md(c);
      if (st) return st;
    }
    VC_CHECK(c, vc::launch_forces(c), "forces");
  }
  if (n_steps > 0) VC_CHECK(c, vc::launch_kick(c, dt_fs), "kick");
  return VCSGC_OK;
}

vcsgc_status vcsgc_set_log(vcsgc_ctx *c, double *tlog, int64_t tcap, double *slog, int64_t scap) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if ((tlog && tcap < 0) || (slog && scap < 0))
    return fail(c, VCSGC_E_INVALID_ARG, "negative log capacity");
  c->tlog = tlog;
  c->tcap = tlog ? tcap : 0;
  c->slog = slog;
  c->scap = slog ? scap : 0;
  const unsigned long long zero[2] = {0, 0};
  VC_CHECK(c, hipMemcpyAsync(&c->ds->tlog_n, zero, 2 * sizeof(unsigned long long),
                             hipMemcpyHostToDevice, c->stream),
           "log reset");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  return VCSGC_OK;
}

vcsgc_status vcsgc_log_counts(vcsgc_ctx *c, int64_t *n_trials, int64_t *n_stages) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  hipError_t e;
  vc::DevState h = read_state(c, &e);
  if (e != hipSuccess) return dev_fail(c, e, "log counts");
  if (n_trials) *n_trials = (int64_t)h.tlog_n;
  if (n_stages) *n_stages = (int64_t)h.slog_n;
  return VCSGC_OK;
}

vcsgc_status vcsgc_get_state(vcsgc_ctx *c, vcsgc_state *out) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!out) return fail(c, VCSGC_E_INVALID_ARG, "null output");
  hipError_t e;
  vc::DevState h = read_state(c, &e);
  if (e != hipSuccess) return dev_fail(c, e, "state");
  out->sweeps_done = c->w;
  out->n_b = h.n_b_cur;
  return VCSGC_OK;
}

vcsgc_status vcsgc_set_state(vcsgc_ctx *c, const vcsgc_state *in) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!in) return fail(c, VCSGC_E_INVALID_ARG, "null input");
  c->w = in->sweeps_done;
  long long zero = 0;
  VC_CHECK(c, hipMemcpyAsync(&c->ds->n_b_cur, &zero, sizeof(zero), hipMemcpyHostToDevice,
                             c->stream),
           "state");
  k_count_b<<<vc::grid_for(c->n), vc::BLOCK, 0, c->stream>>>(c->n, c->sp, c->ds);
  VC_CHECK(c, hipGetLastError(), "state");
  c->mc_valid = false;  // species may have been restored: fresh density cache
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  return VCSGC_OK;
}

vcsgc_status vcsgc_copy_rho(vcsgc_ctx *c, double *rho_dev) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!rho_dev) return fail(c, VCSGC_E_INVALID_ARG, "null output");
  if (!c->mc_valid) {
    st = refresh_mc(c);
    if (st) return st;
  }
  VC_CHECK(c, hipMemcpyAsync(rho_dev, c->rho, sizeof(double) * c->n, hipMemcpyDeviceToDevice,
                             c->stream),
           "copy");
  return VCSGC_OK;
}

vcsgc_status vcsgc_atom_energies(vcsgc_ctx *c, double *e_dev) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!e_dev) return fail(c, VCSGC_E_INVALID_ARG, "null output");
  if (!c->md_valid) {
    st = refresh_md(c);
    if (st) return st;
  }
  VC_CHECK(c, vc::launch_pack(c), "pack");
  VC_CHECK(c, vc::launch_energy(c), "energy");
  VC_CHECK(c, hipMemcpyAsync(e_dev, c->eatom, sizeof(double) * c->n, hipMemcpyDeviceToDevice,
                             c->stream),
           "copy");
  return VCSGC_OK;
}

vcsgc_status vcsgc_get_info(vcsgc_ctx *c, vcsgc_info *out) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!out) return fail(c, VCSGC_E_INVALID_ARG, "null output");
  for (int d = 0; d < 3; ++d) out->n_cells[d] = c->nc[d];
  out->stages_per_sweep = c->S;
  out->kmax = vc::KMAX;
  out->mc_kmax_used = c->kmax_used;
  hipError_t e;
  vc::DevState h = read_state(c, &e);
  if (e != hipSuccess) return dev_fail(c, e, "info");
  out->mc_pairs = c->mc_valid ? (int64_t)h.pairs_mc : 0;
  out->md_pairs = c->md_valid ? (int64_t)h.pairs_md : 0;
  out->md_rebuilds = c->md_rebuilds;
  return VCSGC_OK;
}

vcsgc_status vcsgc_selftest_sqrt(const double *in_dev, double *out_dev, int64_t n,
                                 hipStream_t stream) {
  if (n < 0 || (n > 0 && (!in_dev || !out_dev))) return VCSGC_E_INVALID_ARG;
  hipError_t e = vc::launch_sqrt(in_dev, out_dev, n, stream);
  return e == hipSuccess ? VCSGC_OK : VCSGC_E_DEVICE;
}

}  // extern "C"
