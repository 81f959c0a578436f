// C ABI: context lifecycle, argument validation, scratch management and the
// host side of the sweep / EAM / MD calls.  See include/vcsgc.h.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

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
                  c->cell_fill,  c->mc_j,       c->mc_r,
                  c->mc_cnt,     c->md_j,       c->md_cnt,    c->xr,   c->yr,
                  c->zr,         c->rho,        c->rho_f,      c->eatom, c->red,
                  c->rec,        c->ds,         c->ps4,        c->pf4,       c->part,
                  c->d_reps,     c->d_rs,       c->d_wg_rep,   c->d_j,        c->d_r,
                  c->d_cnt,      c->scan_tmp,   c->snap,       c->bin_pos,
                  c->md_rows,    c->sites,      c->site_lnu,
                  c->u_site,     c->u_j,        c->u_rho,      c->u_v,
                  c->stage_lnug, c->m_sites,   c->m_lnu,      c->m_lnu2,     c->m_lnug,   c->m_rec,
                  c->m_part,     c->s_rec,      c->s_part,     c->nvt,        c->nvt_part,
                  c->tab_coef,   c->cg,         c->npt_part,   c->g_start,    c->g_list,
                  c->g_cum,      c->g_cnt};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (c->h_reps) (void)hipHostFree(c->h_reps);
  if (c->h_state) (void)hipHostFree(c->h_state);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->stage_ev) (void)hipEventDestroy(c->stage_ev);
  vc::free_stage_graph(c);
  vc::free_pipe_graph(c);
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

vc::DevState read_state(vcsgc_ctx *c, hipError_t *e) {
  vc::DevState h;
  std::memset(&h, 0, sizeof(h));
  // through the pinned copy when there is one (a pageable copy is staged)
  vc::DevState *dst = c->h_state ? c->h_state : &h;
  *e = hipMemcpyAsync(dst, c->ds, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (*e == hipSuccess) *e = hipStreamSynchronize(c->stream);
  if (*e == hipSuccess && dst != &h) h = *dst;
  return h;
}

// Grow the search bins after an overflow (capacity doubles).
vcsgc_status grow_bins(vcsgc_ctx *c) {
  if (c->bmax >= 1024) return fail(c, VCSGC_E_OVERFLOW, "more than 1024 atoms in a search bin");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  (void)hipFree(c->bin_atoms);
  (void)hipFree(c->bin_pos);
  c->bin_atoms = nullptr;
  c->bin_pos = nullptr;
  c->bmax *= 2;
  VC_CHECK(c, dalloc(&c->bin_atoms, (size_t)c->nbins_total * c->bmax), "allocation");
  if (c->reps.size() == 1)
    VC_CHECK(c, dalloc(&c->bin_pos, (size_t)c->nbins_total * c->bmax), "allocation");
  int zero = 0;
  VC_CHECK(c, hipMemcpyAsync(&c->ds->bin_overflow, &zero, sizeof(int), hipMemcpyHostToDevice,
                             c->stream),
           "reset");
  return VCSGC_OK;
}

// Rebuild cells + the r < rc list + the density cache; checks row overflow.
vcsgc_status refresh_mc(vcsgc_ctx *c) {
  for (;;) {
    for (const RepHost &r : c->reps) {
      VC_CHECK(c, vc::launch_bin_cells(c, r), "binning");
      VC_CHECK(c, vc::launch_bin_search(c, r), "binning");
      VC_CHECK(c, vc::launch_build_mc_list(c, r), "neighbour list");
      if (c->desc) VC_CHECK(c, vc::launch_build_desc_list(c, r), "descriptor list");
    }
    VC_CHECK(c, vc::launch_mc_row_stats(c), "neighbour list");
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
    c->mc_stats_stale = false;
    c->mc_valid = true;
    return VCSGC_OK;
  }
}

// After MD the r < rc + skin list is valid for the current positions and
// rho_f holds the current densities: the cells are re-binned, the r < rc rows
// are filtered out of the MD rows and the density cache is a copy of rho_f
// (both bitwise what a fresh build gives).  No row can overflow here.
vcsgc_status refresh_mc_from_md(vcsgc_ctx *c) {
  VC_CHECK(c, vc::launch_bin_cells(c, c->reps[0]), "binning");
  VC_CHECK(c, vc::launch_mc_from_md(c), "neighbour list");
  c->mc_stats_stale = true;  // taken when asked for (vcsgc_get_info)
  VC_CHECK(c, hipMemcpyAsync(c->rho, c->rho_f, sizeof(double) * c->n, hipMemcpyDeviceToDevice,
                             c->stream),
           "density");
  c->mc_valid = true;
  return VCSGC_OK;
}

vcsgc_status ensure_mc(vcsgc_ctx *c) {
  if (c->mc_valid) return VCSGC_OK;
  if (c->rho_f_fresh && c->md_valid && !c->desc && c->reps.size() == 1)
    return refresh_mc_from_md(c);
  return refresh_mc(c);
}

vcsgc_status refresh_md(vcsgc_ctx *c) {
  for (;;) {
    VC_CHECK(c, vc::launch_bin_search(c, c->reps[0]), "binning");
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
    for (int d = 0; d < 3; ++d) c->box_build[d] = c->box[d];
    return VCSGC_OK;
  }
}

// Workgroups of the persistent sweep: replica r gets about
// ncpc / (groups per workgroup * trials_per_group) of them (at least one);
// replicas with 8 or more get a multiple of 8 starting at a multiple of 8 so
// that their shares can be laid out XCD by XCD.  The grid must fit the
// co-resident capacity; trials_per_group doubles until it does.
vcsgc_status assign_workgroups(vcsgc_ctx *c) {
  int dev_cu = 0, per_cu = 0;
  VC_CHECK(c, hipDeviceGetAttribute(&dev_cu, hipDeviceAttributeMultiprocessorCount, c->device),
           "device query");
  VC_CHECK(c, vc::persist_max_blocks(&per_cu, c->pot.tab != 0), "occupancy query");
  const int cap = dev_cu * (per_cu > 0 ? per_cu : 1);
  const int R = (int)c->reps.size();
  if (R > cap) return fail(c, VCSGC_E_INVALID_ARG, "more replicas than co-resident workgroups");
  int tpg = c->trials_per_group < 1 ? 1 : c->trials_per_group;
  for (;;) {
    std::vector<int> want(R);
    int64_t total = 0;
    for (int k = 0; k < R; ++k) {
      const int64_t per = (int64_t)vc::persist_groups() * tpg;
      int64_t g = (c->reps[k].ncpc + per - 1) / per;
      if (g < 1) g = 1;
      if (g >= 8) g = (g + 7) / 8 * 8;
      want[k] = (int)g;
      total += g;
    }
    if (total <= cap || tpg >= (1 << 20)) {
      if (total > cap) return fail(c, VCSGC_E_INVALID_ARG, "persistent grid does not fit");
      // large replicas first (aligned), then the single-digit ones
      std::vector<int> order(R);
      for (int k = 0; k < R; ++k) order[k] = k;
      std::stable_sort(order.begin(), order.end(),
                       [&](int a, int b) { return (want[a] >= 8) > (want[b] >= 8); });
      std::vector<int32_t> map((size_t)total);
      int g0 = 0;
      for (int k : order) {
        c->reps[k].g0 = g0;
        c->reps[k].G = want[k];
        for (int q = 0; q < want[k]; ++q) map[g0 + q] = k;
        g0 += want[k];
      }
      if (c->d_wg_rep) (void)hipFree(c->d_wg_rep);
      c->d_wg_rep = nullptr;
      VC_CHECK(c, dalloc(&c->d_wg_rep, (size_t)total), "allocation");
      VC_CHECK(c, hipMemcpy(c->d_wg_rep, map.data(), sizeof(int32_t) * total,
                            hipMemcpyHostToDevice),
               "copy");
      c->grid_total = (int)total;
      c->trials_per_group = tpg;
      if (c->graph_exec) {
        (void)hipGraphExecDestroy(c->graph_exec);
        c->graph_exec = nullptr;
      }
      return VCSGC_OK;
    }
    tpg *= 2;
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
  if (c->kt_seen[cls]++ % c->t_every != 0) return -1;
  // timing-only events: no system-scope fence when recorded (the stream is
  // synchronized before the times are read)
  hipEvent_t ev[2];
  for (int k = 0; k < 2; ++k) {
    if (!c->ev_pool.empty()) {
      ev[k] = c->ev_pool.back();
      c->ev_pool.pop_back();
    } else if (hipEventCreateWithFlags(&ev[k], hipEventDisableSystemFence) != hipSuccess) {
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

vcsgc_status vcsgc_kernel_timing_sampled(vcsgc_ctx *c, uint32_t mask, int32_t every) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (every < 1) return fail(c, VCSGC_E_INVALID_ARG, "every must be >= 1");
  VC_CHECK(c, drain_timers(c), "timing");
  c->tmask = mask & ((1u << VCSGC_KT_CLASSES) - 1);
  c->t_every = every;
  for (int k = 0; k < VCSGC_KT_CLASSES; ++k) {
    c->kt_ms[k] = 0.0;
    c->kt_n[k] = 0;
    c->kt_seen[k] = 0;
  }
  return VCSGC_OK;
}

vcsgc_status vcsgc_kernel_timing(vcsgc_ctx *c, uint32_t mask) {
  return vcsgc_kernel_timing_sampled(c, mask, 1);
}

vcsgc_status vcsgc_get_kernel_timing(vcsgc_ctx *c, vcsgc_ktimes *out) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!out) return fail(c, VCSGC_E_INVALID_ARG, "null output");
  VC_CHECK(c, drain_timers(c), "timing");
  for (int k = 0; k < VCSGC_KT_CLASSES; ++k) {
    out->total_ms[k] = c->kt_ms[k];
    out->count[k] = c->kt_n[k];
    out->launches[k] = c->kt_seen[k];
  }
  return VCSGC_OK;
}

}  // extern "C"

namespace {

// Coefficients (a0, a1, a2, a3) per interval of the cubic Hermite
// interpolant through y[0 .. n-1] at unit-spaced knots, knot slopes by
// central differences and one-sided at the two ends (the interpolation
// vcsgc_eam_table defines).
void hermite_coeffs(int32_t n, const double *y, double *c) {
  for (int32_t k = 0; k + 1 < n; ++k) {
    const double m0 = k == 0 ? y[1] - y[0] : 0.5 * (y[k + 1] - y[k - 1]);
    const double m1 = k + 2 == n ? y[n - 1] - y[n - 2] : 0.5 * (y[k + 2] - y[k]);
    const double d = y[k + 1] - y[k];
    double *a = c + 4 * (int64_t)k;
    a[0] = y[k];
    a[1] = m0;
    a[2] = (3.0 * d - 2.0 * m0) - m1;
    a[3] = (m0 + m1) - 2.0 * d;
  }
}

// Shared by vcsgc_create (one replica) and vcsgc_create_batch.
vcsgc_status create_impl(const vcsgc_system *sys, int R, const int64_t *rep_atoms,
                         const double *rep_box, hipStream_t stream, vcsgc_ctx **out) {
  if (!sys || !out) return fail(nullptr, VCSGC_E_INVALID_ARG, "null argument");
  const vcsgc_eam_fs &P = sys->pot;
  if (sys->n_atoms < 2 || sys->n_atoms > (int64_t)0x7fffffff)
    return fail(nullptr, VCSGC_E_INVALID_ARG, "n_atoms must be in [2, 2^31)");
  if (!sys->x || !sys->y || !sys->z || !sys->species)
    return fail(nullptr, VCSGC_E_INVALID_ARG, "positions and species are required");
  const vcsgc_eam_table *T = sys->table;
  if (T) {
    if (T->nr < 2 || T->nrho < 2 || !(T->dr > 0.0) || !(T->drho > 0.0) || !is_fin(T->dr) ||
        !is_fin(T->drho) || !(T->rc > 0.0) || !is_fin(T->rc) ||
        T->rc > (double)(T->nr - 1) * T->dr)
      return fail(nullptr, VCSGC_E_INVALID_ARG,
                  "table needs nr, nrho >= 2, dr, drho > 0 and 0 < rc <= (nr - 1) dr");
    const double *arrs[] = {T->f[0], T->f[1], T->phi[0], T->phi[1], T->phi[2], T->F[0], T->F[1]};
    for (int k = 0; k < 7; ++k) {
      if (!arrs[k]) return fail(nullptr, VCSGC_E_INVALID_ARG, "missing table");
      const int32_t nk = k < 5 ? T->nr : T->nrho;
      for (int32_t q = 0; q < nk; ++q)
        if (!is_fin(arrs[k][q])) return fail(nullptr, VCSGC_E_INVALID_ARG, "non-finite table value");
    }
  } else {
    const double pv[] = {P.rc, P.c0, P.c1, P.eps_aa, P.eps_ab, P.eps_bb,
                         P.t_a, P.t_b, P.a_a, P.a_b};
    for (double v : pv)
      if (!is_fin(v)) return fail(nullptr, VCSGC_E_INVALID_ARG, "non-finite potential parameter");
  }
  const double rc = T ? T->rc : P.rc;
  if (!(rc > 0.0)) return fail(nullptr, VCSGC_E_INVALID_ARG, "rc must be positive");
  if (!(sys->skin >= 0.0) || !is_fin(sys->skin) || sys->skin > rc)
    return fail(nullptr, VCSGC_E_INVALID_ARG, "skin must be in [0, rc]");
  const bool has_v = sys->vx || sys->vy || sys->vz;
  if (has_v && !(sys->vx && sys->vy && sys->vz))
    return fail(nullptr, VCSGC_E_INVALID_ARG, "velocities must be all set or all NULL");
  const bool has_f = sys->fx || sys->fy || sys->fz;
  if (has_f && !(sys->fx && sys->fy && sys->fz))
    return fail(nullptr, VCSGC_E_INVALID_ARG, "forces must be all set or all NULL");
  if (has_v && (!(P.mass_a > 0.0) || !(P.mass_b > 0.0) || !is_fin(P.mass_a) || !is_fin(P.mass_b)))
    return fail(nullptr, VCSGC_E_INVALID_ARG, "masses must be positive with velocities");
  const double r_dep = sys->r_dep == 0.0 ? 2.0 * rc : sys->r_dep;
  if (!(r_dep >= 2.0 * rc) || !is_fin(r_dep))
    return fail(nullptr, VCSGC_E_INVALID_ARG, "r_dep must be >= 2 rc");
  const int per = (sys->flags & VCSGC_FLAG_COLOURS27) ? 3 : 2, ncol = per * per * per;
  const double ge = sys->grow_edge;
  if (!is_fin(ge) || ge < 0.0) return fail(nullptr, VCSGC_E_INVALID_ARG, "grow_edge must be >= 0");
  const bool grown = ge > 0.0;
  if (grown && (R != 1 || per != 2))
    return fail(nullptr, VCSGC_E_INVALID_ARG,
                "grown domains need a single system and the eight-colour scheme");

  std::vector<RepHost> reps((size_t)R);
  int64_t aoff = 0, coff = 0, boff = 0, roff = 0;
  for (int k = 0; k < R; ++k) {
    RepHost &r = reps[k];
    r.n = rep_atoms[k];
    if (r.n < 2) return fail(nullptr, VCSGC_E_INVALID_ARG, "every replica needs >= 2 atoms");
    r.aoff = aoff;
    for (int d = 0; d < 3; ++d) {
      r.box[d] = rep_box[3 * k + d];
      if (!(r.box[d] > 0.0) || !is_fin(r.box[d]))
        return fail(nullptr, VCSGC_E_INVALID_ARG, "box edges must be positive and finite");
      if (grown) {
        r.nc[d] = (int)std::floor(r.box[d] / std::max(ge, 2.0 * r_dep));
        if (r.nc[d] < 1)
          return fail(nullptr, VCSGC_E_BOX_TOO_SMALL,
                      "box must hold one cell of edge max(grow_edge, 2 r_dep) in every dimension");
      } else {
        r.nc[d] = per * (int)std::floor(r.box[d] / ((double)per * (r_dep / (double)(per - 1))));
        if (r.nc[d] < per)
          return fail(nullptr, VCSGC_E_BOX_TOO_SMALL,
                      per == 2 ? "box must hold two cells of edge r_dep in every dimension"
                               : "box must hold three cells of edge r_dep / 2 in every dimension");
      }
      const double bin_edge = (sys->flags & VCSGC_FLAG_DESCRIPTOR)
                                  ? std::max(rc + sys->skin, vc::DESC_CUT)
                                  : rc + sys->skin;
      r.nb[d] = (int)std::floor(r.box[d] / bin_edge);
      if (r.nb[d] < 2)
        return fail(nullptr, VCSGC_E_BOX_TOO_SMALL, "box too small for the neighbour search");
    }
    r.ncells = (int64_t)r.nc[0] * r.nc[1] * r.nc[2];
    r.coff = coff;
    r.cso = coff + k;
    r.S = (grown ? 1 : (int64_t)ncol) * ((r.n + r.ncells - 1) / r.ncells);
    r.ncpc = grown ? r.ncells : r.ncells / ncol;
    r.roff = roff;
    r.nbins = (int64_t)r.nb[0] * r.nb[1] * r.nb[2];
    r.boff = boff;
    aoff += r.n;
    coff += r.ncells;
    boff += r.nbins;
    roff += r.ncpc;
  }
  if (aoff != sys->n_atoms)
    return fail(nullptr, VCSGC_E_INVALID_ARG, "replica sizes must add up to n_atoms");

  vcsgc_ctx *c = new vcsgc_ctx();
  (void)hipGetDevice(&c->device);
  c->stream = stream;
  c->n = sys->n_atoms;
  c->reps = reps;
  const RepHost &r0 = reps[0];
  for (int d = 0; d < 3; ++d) {
    c->box[d] = r0.box[d];
    c->nc[d] = r0.nc[d];
    c->nb[d] = r0.nb[d];
  }
  c->ncells = r0.ncells;
  c->per = per;
  c->ncol = ncol;
  c->S = r0.S;
  c->nbins = r0.nbins;
  c->nbins_total = boff;
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
  p.rc = rc;
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
  c->bmax = 16;
  c->strategy = 0;
  c->grown = grown;
  c->grow_edge = ge;
  c->desc = (sys->flags & VCSGC_FLAG_DESCRIPTOR) != 0;
  c->bin_edge = c->desc ? std::max(rc + sys->skin, vc::DESC_CUT) : rc + sys->skin;
  for (int d = 0; d < 3; ++d) {
    c->nb_max[d] = r0.nb[d];
    c->box_build[d] = r0.box[d];
  }
  if (T) {
    // the interpolants' coefficients: f_A, f_B, phi_AA, phi_AB, phi_BB, then F_A, F_B
    const int64_t nir = T->nr - 1, nid = T->nrho - 1;
    std::vector<double> co((size_t)(4 * (5 * nir + 2 * nid)));
    const double *arrs[] = {T->f[0], T->f[1], T->phi[0], T->phi[1], T->phi[2], T->F[0], T->F[1]};
    size_t o = 0;
    for (int k = 0; k < 7; ++k) {
      const int32_t nk = k < 5 ? T->nr : T->nrho;
      hermite_coeffs(nk, arrs[k], co.data() + o);
      o += (size_t)4 * (nk - 1);
    }
    hipError_t e1 = dalloc(&c->tab_coef, co.size());
    if (e1 == hipSuccess)
      e1 = hipMemcpy(c->tab_coef, co.data(), sizeof(double) * co.size(), hipMemcpyHostToDevice);
    if (e1 != hipSuccess) {
      free_all(c);
      delete c;
      return fail(nullptr, VCSGC_E_OUT_OF_MEMORY, "table upload");
    }
    p.tab = 1;
    p.nr = T->nr;
    p.nrho = T->nrho;
    p.inv_dr = 1.0 / T->dr;
    p.inv_drho = 1.0 / T->drho;
    p.tc = c->tab_coef;
  }

  const int64_t n = c->n, K = vc::KMAX;
  const bool single = R == 1;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t rr) {
    if (e == hipSuccess) e = rr;
  };
  A(dalloc(&c->bin_count, boff));
  A(dalloc(&c->bin_atoms, boff * c->bmax));
  if (single) {
    A(dalloc(&c->bin_pos, boff * c->bmax));
    A(dalloc(&c->sites, reps[0].S * reps[0].ncpc));
    A(dalloc(&c->site_lnu, reps[0].S * reps[0].ncpc));
    A(dalloc(&c->stage_lnug, reps[0].S));
    // fused stage pipeline: two sweeps of site tables, two stages of records
    // and trial-block sums
    const int64_t S1 = reps[0].S, nc1 = reps[0].ncpc;
    A(dalloc(&c->m_sites, 2 * S1 * nc1));
    A(dalloc(&c->m_lnu, 2 * S1 * nc1));
    A(dalloc(&c->m_lnu2, 2 * S1 * nc1));
    A(dalloc(&c->m_lnug, 2 * S1));
    A(dalloc(&c->m_rec, 2 * nc1));
    A(dalloc(&c->m_part, 2 * vc::NPART * (int64_t)vc::grid_for(nc1 * 16)));
    A(dalloc(&c->s_rec, 2 * vc::SPEC_MAX * nc1));
    A(dalloc(&c->s_part, 2 * vc::SPEC_MAX * 3 * (int64_t)vc::grid_for(nc1 * 16)));
    A(hipHostMalloc((void **)&c->h_state, sizeof(vc::DevState), hipHostMallocDefault));
  }
  A(dalloc(&c->cell_count, coff));
  A(dalloc(&c->cell_start, coff + R));
  A(dalloc(&c->cell_fill, coff));
  A(dalloc(&c->cell_atoms, n));
  {
    int64_t mx = 1;
    for (const RepHost &r : c->reps)
      mx = std::max<int64_t>(mx, (std::max({r.ncells, r.nbins, grown ? 8 * r.ncells : 0}) +
                                  vc::SCAN_CHUNK - 1) / vc::SCAN_CHUNK);
    A(dalloc(&c->scan_tmp, mx));
  }
  if (grown) {
    A(dalloc(&c->g_start, 8 * c->ncells + 1));
    A(dalloc(&c->g_cnt, 8 * c->ncells));
    A(dalloc(&c->g_list, 8 * n));
    A(dalloc(&c->g_cum, 8 * n));
  }
  A(dalloc(&c->mc_j, K * n));
  A(dalloc(&c->mc_r, K * n));
  A(dalloc(&c->mc_cnt, n));
  if (single) {
    A(dalloc(&c->md_j, K * n));
    A(dalloc(&c->md_rows, K * n));
    A(dalloc(&c->md_cnt, n));
    A(dalloc(&c->xr, n));
    A(dalloc(&c->yr, n));
    A(dalloc(&c->zr, n));
    A(dalloc(&c->ps4, n));
    A(dalloc(&c->pf4, n));
    A(dalloc(&c->rho_f, n));
    A(dalloc(&c->eatom, n));
    A(dalloc(&c->nvt, 8));
    A(dalloc(&c->nvt_part, (n + vc::BLOCK - 1) / vc::BLOCK));
  }
  if (c->desc) {
    A(dalloc(&c->d_j, K * n));
    A(dalloc(&c->d_r, K * n));
    A(dalloc(&c->d_cnt, n));
  }
  A(dalloc(&c->rho, n));
  A(dalloc(&c->red, (n + vc::BLOCK - 1) / vc::BLOCK + 8));
  A(dalloc(&c->rec, roff));
  A(dalloc(&c->ds, 1));
  A(dalloc((unsigned char **)&c->d_reps, vc::repd_size() * R));
  A(dalloc((unsigned char **)&c->d_rs, vc::repstate_size() * R));
  if (e == hipSuccess) e = hipHostMalloc(&c->h_reps, vc::repd_size() * R, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming);
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
  vcsgc_status st = assign_workgroups(c);
  if (st) return bail(st);
  // trial-kernel partial sums: the larger of the two strategies' needs
  const int64_t npart_stage = (r0.ncpc * 16 + vc::BLOCK - 1) / vc::BLOCK + 1;
  c->npart = std::max<int64_t>(npart_stage, c->grid_total);
  if ((e = dalloc(&c->part, vc::NPART * c->npart)) != hipSuccess)
    return bail(dev_fail(c, e, "allocation"));
  if ((e = hipMemsetAsync(c->ds, 0, sizeof(vc::DevState), c->stream)) != hipSuccess)
    return bail(dev_fail(c, e, "init"));
  // MD rows hold valid indices beyond their lengths too (empty until built)
  if (c->md_j &&
      ((e = hipMemsetAsync(c->md_j, 0, sizeof(int32_t) * vc::KMAX * n, c->stream)) != hipSuccess ||
       (e = hipMemsetAsync(c->md_rows, 0, sizeof(int32_t) * vc::KMAX * n, c->stream)) != hipSuccess ||
       (e = hipMemsetAsync(c->md_cnt, 0, sizeof(uint8_t) * n, c->stream)) != hipSuccess))
    return bail(dev_fail(c, e, "init"));
  for (const RepHost &r : c->reps) {
    if ((e = vc::launch_validate(c, r)) != hipSuccess) return bail(dev_fail(c, e, "validate"));
  }
  {
    hipError_t e2;
    vc::DevState h = read_state(c, &e2);
    if (e2 != hipSuccess) return bail(dev_fail(c, e2, "validate"));
    if (h.bad_input)
      return bail(fail(c, VCSGC_E_INVALID_ARG,
                       "positions must lie in [0, L) and species in {0, 1}"));
  }
  if ((e = vc::persist_count(c)) != hipSuccess) return bail(dev_fail(c, e, "count"));
  if (grown) {  // the batched pipeline, three stages per batch
    c->strategy = 3;
    c->trials_per_group = 3;
  }
  st = refresh_mc(c);
  if (st != VCSGC_OK) return bail(st);
  *out = c;
  return VCSGC_OK;
}

}  // namespace

extern "C" {

vcsgc_status vcsgc_create(const vcsgc_system *sys, hipStream_t stream, vcsgc_ctx **out) {
  if (!sys || !out) return fail(nullptr, VCSGC_E_INVALID_ARG, "null argument");
  const int64_t n = sys->n_atoms;
  return create_impl(sys, 1, &n, sys->box, stream, out);
}

vcsgc_status vcsgc_create_batch(const vcsgc_system *sys, int32_t n_rep, const int64_t *rep_atoms,
                                const double *rep_box, hipStream_t stream, vcsgc_ctx **out) {
  if (!sys || !out || n_rep < 1 || !rep_atoms || !rep_box)
    return fail(nullptr, VCSGC_E_INVALID_ARG, "null argument or n_rep < 1");
  return create_impl(sys, n_rep, rep_atoms, rep_box, stream, out);
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

}  // extern "C"

namespace {

bool valid_params(double dmu0, double kappa, double cbar, double T) {
  return is_fin(dmu0) && is_fin(kappa) && kappa >= 0.0 && is_fin(cbar) && cbar >= 0.0 &&
         cbar <= 1.0 && is_fin(T) && T > 0.0;
}

// Sweeps of every replica with per-replica parameters; stats may be NULL.
vcsgc_status sweep_impl(vcsgc_ctx *c, const double *dmu0, const double *kappa, const double *cbar,
                        const double *T, int64_t n_sweeps, uint64_t seed, vcsgc_stats *out) {
  const int R = (int)c->reps.size();
  if (n_sweeps < 0) return fail(c, VCSGC_E_INVALID_ARG, "n_sweeps must be >= 0");
  for (int k = 0; k < R; ++k)
    if (!valid_params(dmu0[k], kappa[k], cbar[k], T[k]))
      return fail(c, VCSGC_E_INVALID_ARG,
                  "need finite dmu0, kappa >= 0, cbar in [0,1], T > 0 for every replica");
  if (R == 1)  // the box may have changed under the barostat
    for (int d = 0; d < 3; ++d)
      if (c->box[d] / (double)c->nc[d] <
          (c->grown ? 2.0 * c->r_dep : c->r_dep / (double)(c->per - 1)))
        return fail(c, VCSGC_E_BOX_TOO_SMALL,
                    "the box has shrunk below the sweep's cell grid (edge < r_dep)");
  {
    vcsgc_status st = ensure_mc(c);
    if (st) return st;
  }
  c->last_seed = seed;
  if (n_sweeps > 0) c->rho_f_fresh = false;
  if (c->local_steps > 1 && (c->da_mode || c->smp_cap > 0))
    return fail(c, VCSGC_E_INVALID_ARG,
                "delayed acceptance and the sample log need one trial per cell per stage");
  // delayed acceptance, the training-sample log and local chains run with
  // per-stage launches
  if ((c->strategy >= 2 || c->da_mode || c->smp_cap > 0 || c->local_steps > 1) && R == 1) {
    // one trial kernel and one commit kernel per stage
    VC_CHECK(c, vc::persist_sync_nb_to_stage(c), "sweep");
    c->h_state_final = false;
    VC_CHECK(c, vc::launch_sweeps(c, dmu0[0], kappa[0], cbar[0], T[0], n_sweeps, seed), "sweep");
    // the pipelines end with the device state read and n_B synchronized
    const bool have = c->h_state_final;
    c->h_state_final = false;
    if (!have) VC_CHECK(c, vc::persist_sync_nb_from_stage(c), "sweep");
    c->w += (uint64_t)n_sweeps;
    if (out) {
      hipError_t e = hipSuccess;
      vc::DevState h = have ? *c->h_state : read_state(c, &e);
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
      out->stage1_pass = (int64_t)h.stage1_pass;
    }
    return VCSGC_OK;
  }
  VC_CHECK(c, vc::persist_stage_params(c, dmu0, kappa, cbar, T, n_sweeps, seed), "sweep");
  if (n_sweeps > 0) {
    int h = vc::tstart(c, VCSGC_KT_PERSIST);
    VC_CHECK(c, vc::launch_persistent(c, c->strategy == 0), "persistent sweep");
    vc::tstop(c, h);
  }
  c->w += (uint64_t)n_sweeps;
  // the timeout flags are read after every call, with or without statistics:
  // a workgroup that left a timed-out wait may have committed part of a stage
  int err = 0;
  VC_CHECK(c, vc::persist_read_stats(c, out, &err), "sweep");
  if (err) {
    c->sticky = true;
    return fail(c, VCSGC_E_BARRIER_TIMEOUT, "persistent sweep: a barrier wait exceeded its limit");
  }
  return VCSGC_OK;
}

}  // namespace

extern "C" {

vcsgc_status vcsgc_sweep(vcsgc_ctx *c, double dmu0, double kappa, double cbar, double T_K,
                         int64_t n_sweeps, uint64_t seed, vcsgc_stats *out) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (c->reps.size() != 1) return fail(c, VCSGC_E_INVALID_ARG, "batch context: use vcsgc_sweep_batch");
  return sweep_impl(c, &dmu0, &kappa, &cbar, &T_K, n_sweeps, seed, out);
}

vcsgc_status vcsgc_sweep_batch(vcsgc_ctx *c, const double *dmu0, const double *kappa,
                               const double *cbar, const double *T, int64_t n_sweeps,
                               uint64_t seed, vcsgc_stats *out) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!dmu0 || !kappa || !cbar || !T) return fail(c, VCSGC_E_INVALID_ARG, "null parameter array");
  return sweep_impl(c, dmu0, kappa, cbar, T, n_sweeps, seed, out);
}

vcsgc_status vcsgc_set_wait_limit(vcsgc_ctx *c, uint32_t polls) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (polls < 1) return fail(c, VCSGC_E_INVALID_ARG, "polls must be >= 1");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  c->spin_limit = polls;
  if (c->graph_exec) {  // its kernel node holds the old limit
    (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
  }
  return VCSGC_OK;
}

vcsgc_status vcsgc_set_tuning(vcsgc_ctx *c, int32_t strategy, int32_t trials_per_group) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (strategy < 0 || strategy > 3 || trials_per_group < 1 || trials_per_group > 64)
    return fail(c, VCSGC_E_INVALID_ARG, "strategy in {0,1,2,3}, trials_per_group in [1,64]");
  if (strategy == 3 && trials_per_group > vc::SPEC_MAX)
    return fail(c, VCSGC_E_INVALID_ARG, "stages per batch in [1,16]");
  if (strategy >= 2 && c->reps.size() != 1)
    return fail(c, VCSGC_E_INVALID_ARG, "per-stage launches need a single-system context");
  if (strategy < 2 && c->grown)
    return fail(c, VCSGC_E_INVALID_ARG, "grown domains run on the pipeline strategies (2, 3)");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  c->strategy = strategy;
  if (trials_per_group != c->trials_per_group) {
    c->trials_per_group = trials_per_group;
    st = assign_workgroups(c);
    if (st) return st;
    if (c->grid_total > c->npart) {
      vc::free_stage_graph(c);  // its nodes hold the old buffer
      (void)hipFree(c->part);
      c->part = nullptr;
      c->npart = c->grid_total;
      VC_CHECK(c, dalloc(&c->part, vc::NPART * c->npart), "allocation");
    }
  }
  return VCSGC_OK;
}

vcsgc_status vcsgc_set_local_steps(vcsgc_ctx *c, int32_t k) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (c->reps.size() != 1) return fail(c, VCSGC_E_INVALID_ARG, "local chains need a single system");
  if (k < 1 || k > 64) return fail(c, VCSGC_E_INVALID_ARG, "local chain length in [1, 64]");
  if (k == c->local_steps) return VCSGC_OK;
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  vc::free_stage_graph(c);  // its nodes hold the old buffers
  void *old[] = {c->sites, c->site_lnu, c->stage_lnug, c->u_site, c->u_j, c->u_rho, c->u_v};
  for (void *p : old)
    if (p) (void)hipFree(p);
  c->sites = c->u_site = c->u_j = nullptr;
  c->site_lnu = c->stage_lnug = c->u_rho = c->u_v = nullptr;
  c->local_steps = k;
  const int64_t ncpc = vc::active_cells(c), K = k;
  const int64_t tab = vc::stages_per_sweep(c) * ncpc * K;
  VC_CHECK(c, dalloc(&c->sites, tab), "allocation");
  VC_CHECK(c, dalloc(&c->site_lnu, tab), "allocation");
  VC_CHECK(c, dalloc(&c->stage_lnug, vc::stages_per_sweep(c)), "allocation");
  if (K > 1) {
    VC_CHECK(c, dalloc(&c->u_site, ncpc * K), "allocation");
    VC_CHECK(c, dalloc(&c->u_j, ncpc * K * vc::KMAX), "allocation");
    VC_CHECK(c, dalloc(&c->u_rho, ncpc * K * vc::KMAX), "allocation");
    VC_CHECK(c, dalloc(&c->u_v, ncpc * K * 3), "allocation");
  }
  return VCSGC_OK;
}

vcsgc_status vcsgc_get_tuning(vcsgc_ctx *c, int32_t *strategy, int32_t *trials_per_group,
                              int32_t *workgroups) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (strategy) *strategy = c->strategy;
  if (trials_per_group) *trials_per_group = c->trials_per_group;
  if (workgroups) *workgroups = c->grid_total;
  return VCSGC_OK;
}

vcsgc_status eam_energy_forces(vcsgc_ctx *c, double *energy_eV, int want_forces) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (c->reps.size() != 1) return fail(c, VCSGC_E_INVALID_ARG, "not available on a batch context");
  if (want_forces && !c->fx)
    return fail(c, VCSGC_E_INVALID_ARG, "forces requested but the system has no force arrays");
  if (!c->md_valid) {
    st = refresh_md(c);
    if (st) return st;
  }
  VC_CHECK(c, vc::launch_pack(c), "pack");
  VC_CHECK(c, vc::launch_energy(c), "energy");
  if (want_forces) VC_CHECK(c, vc::launch_forces(c), "forces");
  c->rho_f_fresh = true;
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

}  // extern "C"

namespace {

// Steps with the rebuild decision taken on the host after every drift
// (handles bin growth); used when the device path cannot be.
vcsgc_status md_steps_host(vcsgc_ctx *c, double dt_fs, int64_t n_steps) {
  VC_CHECK(c, vc::launch_pack(c), "pack");
  VC_CHECK(c, vc::launch_forces(c), "forces");
  for (int64_t k = 0; k < n_steps; ++k) {
    // the closing half-kick of step k-1 is fused into the opening one of step k
    VC_CHECK(c, vc::launch_kick_drift(c, dt_fs, k > 0, 0), "kick-drift");
    int flag = 0;
    VC_CHECK(c, hipMemcpyAsync(&flag, &c->ds->rebuild[0], sizeof(int), hipMemcpyDeviceToHost,
                               c->stream),
             "copy");
    VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
    if (flag) {
      VC_CHECK(c, hipMemsetAsync(&c->ds->rebuild[0], 0, sizeof(int), c->stream), "reset");
      vcsgc_status st = refresh_md(c);
      if (st) return st;
    }
    VC_CHECK(c, vc::launch_forces(c), "forces");
  }
  if (n_steps > 0) VC_CHECK(c, vc::launch_kick(c, dt_fs), "kick");
  return VCSGC_OK;
}

// Steps with the rebuild decided on the device (no host round trip per step).
// State at entry is kept; if a bin or a row overflowed on the way, it is
// restored and the steps are redone on the host-decided path.
vcsgc_status md_steps_device(vcsgc_ctx *c, double dt_fs, int64_t n_steps) {
  const size_t nb = sizeof(double) * (size_t)c->n;
  if (!c->snap) VC_CHECK(c, dalloc(&c->snap, 6 * (size_t)c->n), "allocation");
  double *state[6] = {c->x, c->y, c->z, c->vx, c->vy, c->vz};
  for (int k = 0; k < 6; ++k)
    VC_CHECK(c, hipMemcpyAsync(c->snap + k * c->n, state[k], nb, hipMemcpyDeviceToDevice,
                               c->stream),
             "snapshot");
  VC_CHECK(c, hipMemsetAsync(&c->ds->md_rebuilds, 0, sizeof(unsigned long long), c->stream),
           "reset");
  VC_CHECK(c, hipMemsetAsync(c->ds->rebuild, 0, 2 * sizeof(int), c->stream), "reset");
  VC_CHECK(c, vc::launch_pack(c), "pack");
  // step k uses the rebuild flag of parity k & 1 (its drift clears the
  // other); its kick and drift run inside the force pass before it, and
  // the last force pass stores the forces for the closing half kick
  VC_CHECK(c, vc::launch_forces_kick_drift(c, dt_fs, false, 0), "forces");
  for (int64_t k = 0; k < n_steps; ++k) {
    VC_CHECK(c, vc::launch_md_rebuild_cond(c, (int)(k & 1)), "neighbour list (MD)");
    if (k + 1 < n_steps)
      VC_CHECK(c, vc::launch_forces_kick_drift(c, dt_fs, true, (int)((k + 1) & 1)), "forces");
    else
      VC_CHECK(c, vc::launch_forces(c), "forces");
  }
  VC_CHECK(c, vc::launch_kick(c, dt_fs), "kick");
  hipError_t e;
  vc::DevState h = read_state(c, &e);
  if (e != hipSuccess) return dev_fail(c, e, "MD");
  c->md_rebuilds += (int64_t)h.md_rebuilds;
  if (!h.bin_overflow && !h.overflow) return VCSGC_OK;
  for (int k = 0; k < 6; ++k)
    VC_CHECK(c, hipMemcpyAsync(state[k], c->snap + k * c->n, nb, hipMemcpyDeviceToDevice,
                               c->stream),
             "restore");
  const int zero[2] = {0, 0};
  VC_CHECK(c, hipMemcpyAsync(&c->ds->overflow, zero, 2 * sizeof(int), hipMemcpyHostToDevice,
                             c->stream),
           "reset");
  VC_CHECK(c, hipMemsetAsync(c->ds->rebuild, 0, 2 * sizeof(int), c->stream), "reset");
  if (h.bin_overflow) {
    vcsgc_status st = grow_bins(c);
    if (st) return st;
  }
  vcsgc_status st = refresh_md(c);
  if (st) return st;
  return md_steps_host(c, dt_fs, n_steps);
}

// Nose-Hoover NVT steps: per step the thermostat's half steps at the step
// boundary, the scaled kick and drift, the rebuild decision (on the device
// when the search bins allow it, else read by the host), forces, and the
// closing kick with the kinetic-energy chunk sums.  On a bin or row overflow
// of a device-decided rebuild the call's entry state (positions,
// velocities, xi, eta) is restored and the steps are redone with host
// decisions.
vcsgc_status md_nvt_steps(vcsgc_ctx *c, double dt_fs, int64_t n_steps, bool dev) {
  const size_t nb = sizeof(double) * (size_t)c->n;
  double *state[6] = {c->x, c->y, c->z, c->vx, c->vy, c->vz};
  if (dev) {
    if (!c->snap) VC_CHECK(c, dalloc(&c->snap, 6 * (size_t)c->n), "allocation");
    for (int k = 0; k < 6; ++k)
      VC_CHECK(c, hipMemcpyAsync(c->snap + k * c->n, state[k], nb, hipMemcpyDeviceToDevice,
                                 c->stream),
               "snapshot");
    VC_CHECK(c, hipMemcpyAsync(c->nvt + 5, c->nvt, 2 * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream),
             "snapshot");
    VC_CHECK(c, hipMemsetAsync(&c->ds->md_rebuilds, 0, sizeof(unsigned long long), c->stream),
             "reset");
  }
  VC_CHECK(c, hipMemsetAsync(c->ds->rebuild, 0, 2 * sizeof(int), c->stream), "reset");
  VC_CHECK(c, vc::launch_pack(c), "pack");
  VC_CHECK(c, vc::launch_forces(c), "forces");
  VC_CHECK(c, vc::launch_nvt_ke(c, dt_fs, false), "thermostat");
  VC_CHECK(c, vc::launch_nvt_thermo(c, dt_fs, 2), "thermostat");
  for (int64_t k = 0; k < n_steps; ++k) {
    const int par = dev ? (int)(k & 1) : 0;
    VC_CHECK(c, vc::launch_nvt_kick_drift(c, dt_fs, par), "kick-drift");
    if (dev) {
      VC_CHECK(c, vc::launch_md_rebuild_cond(c, par), "neighbour list (MD)");
    } else {
      int flag = 0;
      VC_CHECK(c, hipMemcpyAsync(&flag, &c->ds->rebuild[0], sizeof(int), hipMemcpyDeviceToHost,
                                 c->stream),
               "copy");
      VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
      if (flag) {
        VC_CHECK(c, hipMemsetAsync(&c->ds->rebuild[0], 0, sizeof(int), c->stream), "reset");
        vcsgc_status st = refresh_md(c);
        if (st) return st;
      }
    }
    VC_CHECK(c, vc::launch_forces(c), "forces");
    VC_CHECK(c, vc::launch_nvt_ke(c, dt_fs, true), "thermostat");
    VC_CHECK(c, vc::launch_nvt_thermo(c, dt_fs, k + 1 < n_steps ? 3 : 1), "thermostat");
  }
  if (n_steps > 0) VC_CHECK(c, vc::launch_nvt_scale(c), "thermostat");
  if (!dev) return VCSGC_OK;
  hipError_t e;
  vc::DevState h = read_state(c, &e);
  if (e != hipSuccess) return dev_fail(c, e, "MD");
  c->md_rebuilds += (int64_t)h.md_rebuilds;
  if (!h.bin_overflow && !h.overflow) return VCSGC_OK;
  for (int k = 0; k < 6; ++k)
    VC_CHECK(c, hipMemcpyAsync(state[k], c->snap + k * c->n, nb, hipMemcpyDeviceToDevice,
                               c->stream),
             "restore");
  VC_CHECK(c, hipMemcpyAsync(c->nvt, c->nvt + 5, 2 * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream),
           "restore");
  const int zero[2] = {0, 0};
  VC_CHECK(c, hipMemcpyAsync(&c->ds->overflow, zero, 2 * sizeof(int), hipMemcpyHostToDevice,
                             c->stream),
           "reset");
  if (h.bin_overflow) {
    vcsgc_status st = grow_bins(c);
    if (st) return st;
  }
  vcsgc_status st = refresh_md(c);
  if (st) return st;
  return md_nvt_steps(c, dt_fs, n_steps, false);
}

// Energy (fixed-shape total into *e) and forces at the current positions:
// the MD list is rebuilt first when the last move raised ds->rebuild[0].
vcsgc_status cg_eval(vcsgc_ctx *c, bool check_list, double *e) {
  if (check_list) {
    int flag = 0;
    VC_CHECK(c, hipMemcpyAsync(&flag, &c->ds->rebuild[0], sizeof(int), hipMemcpyDeviceToHost,
                               c->stream),
             "copy");
    VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
    if (flag) {
      VC_CHECK(c, hipMemsetAsync(&c->ds->rebuild[0], 0, sizeof(int), c->stream), "reset");
      vcsgc_status st = refresh_md(c);
      if (st) return st;
    }
  }
  VC_CHECK(c, vc::launch_energy(c), "energy");
  VC_CHECK(c, vc::launch_forces(c), "forces");
  double *out = c->red + (c->n + vc::BLOCK - 1) / vc::BLOCK + 1;
  VC_CHECK(c, vc::launch_reduce_sum(c, c->eatom, c->n, out), "reduce");
  VC_CHECK(c, hipMemcpyAsync(e, out, sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  return VCSGC_OK;
}

// the two totals of mode 0 or 1 (launch_cg_totals) on the host
vcsgc_status cg_totals(vcsgc_ctx *c, int mode, const double *u, double out[2]) {
  const int64_t nch = (c->n + vc::BLOCK - 1) / vc::BLOCK;
  double *part = c->cg + 9 * c->n, *dev_out = part + 2 * nch;
  VC_CHECK(c, vc::launch_cg_totals(c, mode, u, part, dev_out), "relaxation");
  VC_CHECK(c, hipMemcpyAsync(out, dev_out, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream),
           "copy");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  return VCSGC_OK;
}

// three device vectors of n doubles into one of 3 n
vcsgc_status cg_gather3(vcsgc_ctx *c, double *dst, double *a, double *b, double *d) {
  const size_t nb = sizeof(double) * (size_t)c->n;
  double *src[3] = {a, b, d};
  for (int k = 0; k < 3; ++k)
    VC_CHECK(c, hipMemcpyAsync(dst + k * c->n, src[k], nb, hipMemcpyDeviceToDevice, c->stream),
             "copy");
  return VCSGC_OK;
}

// New box edges L (single-system context): the search bins are re-gridded
// to floor(L / bin_edge) per axis, at most the grid of creation (whose
// arrays hold it).  False if an axis would hold fewer than two bins.
bool set_box(vcsgc_ctx *c, const double L[3]) {
  int nb[3];
  for (int d = 0; d < 3; ++d) {
    nb[d] = std::min(c->nb_max[d], (int)std::floor(L[d] / c->bin_edge));
    if (nb[d] < 2) return false;
  }
  RepHost &r = c->reps[0];
  for (int d = 0; d < 3; ++d) {
    c->box[d] = r.box[d] = L[d];
    c->nb[d] = r.nb[d] = nb[d];
  }
  c->nbins = r.nbins = (int64_t)nb[0] * nb[1] * nb[2];
  return true;
}

// the thermostat's half step with the barostat momentum (as in the NPT
// splitting documented at vcsgc_set_barostat); returns the velocity factor
double npt_thermo(double h, double g1kT, double Q, double W, double &K, double &pe, double &xi,
                  double &eta) {
  const double q = 0.5 * h;
  xi = xi + q * ((2.0 * K + pe * pe / W - g1kT) / Q);
  const double a = xi * q;
  const double s = (1.0 - a) / (1.0 + a);
  K = K * s * s;
  pe = pe * s;
  eta = eta + xi * h;
  xi = xi + q * ((2.0 * K + pe * pe / W - g1kT) / Q);
  return s;
}

// Forces with the virial terms at the current positions, the closing kick
// (if kick), and the totals: *K (eV) and *vir (eV).
vcsgc_status npt_forces_sums(vcsgc_ctx *c, bool kick, double cv, double h, double *K,
                             double *vir) {
  const int64_t nch = (c->n + vc::BLOCK - 1) / vc::BLOCK;
  double *out = c->npt_part + 2 * nch;
  VC_CHECK(c, vc::launch_forces_virial(c, c->eatom), "forces");
  VC_CHECK(c, vc::launch_npt_sums(c, kick, cv, h, c->eatom, c->npt_part, out), "barostat");
  double t[2];
  VC_CHECK(c, hipMemcpyAsync(t, out, sizeof(t), hipMemcpyDeviceToHost, c->stream), "copy");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  *K = 0.5 * t[0] / vc::ACC;
  *vir = -0.5 * t[1];
  return VCSGC_OK;
}

// Nose-Hoover NPT steps, driven from the host (the box changes every step;
// its edges are kernel arguments).  The MD list is rebuilt on the host's
// decision; c->eatom holds the per-atom virial terms.
vcsgc_status md_npt_steps(vcsgc_ctx *c, double dt, int64_t n_steps) {
  const int64_t n = c->n;
  if (!c->npt_part)
    VC_CHECK(c, dalloc(&c->npt_part, 2 * (size_t)((n + vc::BLOCK - 1) / vc::BLOCK) + 8),
             "allocation");
  double th[2];
  VC_CHECK(c, hipMemcpyAsync(th, c->nvt, sizeof(th), hipMemcpyDeviceToHost, c->stream), "copy");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  double xi = th[0], eta = th[1], pe = c->npt_pe;
  const double h = 0.5 * dt;
  const double g = 3.0 * (double)n - 3.0;
  const double g1kT = (g + 1.0) * (vc::KB * c->nvt_T);
  const double Q = g1kT * c->nvt_tau * c->nvt_tau;
  const double W = g1kT * c->npt_tau * c->npt_tau;
  const double rc = c->pot.rc, reach = c->pot.rc + c->skin;
  VC_CHECK(c, hipMemsetAsync(&c->ds->rebuild[0], 0, sizeof(int), c->stream), "reset");
  VC_CHECK(c, vc::launch_pack(c), "pack");
  double K = 0.0, vir = 0.0;
  vcsgc_status st = npt_forces_sums(c, false, 1.0, h, &K, &vir);
  if (st) return st;
  double s_pend = 1.0;
  // writes the thermostat and barostat state back (the velocities take the
  // pending end-of-step factor)
  auto finish = [&](double xi_, double eta_, double pe_) -> vcsgc_status {
    VC_CHECK(c, vc::launch_scale_v(c, s_pend), "barostat");
    th[0] = xi_;
    th[1] = eta_;
    VC_CHECK(c, hipMemcpyAsync(c->nvt, th, sizeof(th), hipMemcpyHostToDevice, c->stream), "copy");
    VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
    c->npt_pe = pe_;
    c->npt_vir = vir;
    return VCSGC_OK;
  };
  for (int64_t k = 0; k < n_steps; ++k) {
    const double xi0 = xi, eta0 = eta, pe0 = pe;
    const double s = npt_thermo(h, g1kT, Q, W, K, pe, xi, eta);
    double V = c->box[0] * c->box[1] * c->box[2];
    double P = (2.0 * K + vir) / (3.0 * V);
    pe = pe + h * (3.0 * V * (P - c->npt_p) + (3.0 / g) * (2.0 * K));
    const double ve = pe / W;
    const double cv = std::exp(-(1.0 + 3.0 / g) * ve * (0.5 * h));
    const double q = std::exp(ve * h);
    const double L[3] = {c->box[0] * q * q, c->box[1] * q * q, c->box[2] * q * q};
    if (!set_box(c, L)) {  // the state of the last complete step is kept
      if ((st = finish(xi0, eta0, pe0))) return st;
      return fail(c, VCSGC_E_BOX_TOO_SMALL, "the box has shrunk below two search bins");
    }
    double lam[3], lmin = 1e300;
    for (int d = 0; d < 3; ++d) {
      lam[d] = L[d] / c->box_build[d];
      lmin = std::min(lmin, lam[d]);
    }
    const double thr = 0.5 * (lmin * reach - rc);
    VC_CHECK(c, vc::launch_npt_kick_drift(c, s_pend, s, cv, h, dt, q, lam, thr), "kick-drift");
    int flag = 0;
    VC_CHECK(c, hipMemcpyAsync(&flag, &c->ds->rebuild[0], sizeof(int), hipMemcpyDeviceToHost,
                               c->stream),
             "copy");
    VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
    if (flag) {
      VC_CHECK(c, hipMemsetAsync(&c->ds->rebuild[0], 0, sizeof(int), c->stream), "reset");
      if ((st = refresh_md(c))) return st;
    }
    if ((st = npt_forces_sums(c, true, cv, h, &K, &vir))) return st;
    V = c->box[0] * c->box[1] * c->box[2];
    P = (2.0 * K + vir) / (3.0 * V);
    pe = pe + h * (3.0 * V * (P - c->npt_p) + (3.0 / g) * (2.0 * K));
    s_pend = npt_thermo(h, g1kT, Q, W, K, pe, xi, eta);
  }
  return finish(xi, eta, pe);
}

}  // namespace

extern "C" {

vcsgc_status vcsgc_set_thermostat(vcsgc_ctx *c, double T_K, double tau_fs, double xi,
                                  double eta) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (c->reps.size() != 1 || !c->nvt)
    return fail(c, VCSGC_E_INVALID_ARG, "the thermostat needs a single-system MD context");
  if (!is_fin(T_K) || T_K < 0.0 || !(tau_fs > 0.0) || !is_fin(xi) || !is_fin(eta))
    return fail(c, VCSGC_E_INVALID_ARG, "need T >= 0, tau > 0 and finite xi, eta");
  const double h[2] = {xi, eta};
  VC_CHECK(c, hipMemcpyAsync(c->nvt, h, sizeof(h), hipMemcpyHostToDevice, c->stream), "copy");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  c->nvt_T = T_K;
  c->nvt_tau = tau_fs;
  return VCSGC_OK;
}

vcsgc_status vcsgc_set_barostat(vcsgc_ctx *c, double p_ext, double tau_p_fs, double pe) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (c->reps.size() != 1 || !c->nvt)
    return fail(c, VCSGC_E_INVALID_ARG, "the barostat needs a single-system MD context");
  if (!is_fin(p_ext) || !is_fin(tau_p_fs) || tau_p_fs < 0.0 || !is_fin(pe))
    return fail(c, VCSGC_E_INVALID_ARG, "need finite p_ext and pe and tau_p >= 0");
  c->npt_p = p_ext;
  c->npt_tau = tau_p_fs;
  c->npt_pe = pe;
  return VCSGC_OK;
}

vcsgc_status vcsgc_get_barostat(vcsgc_ctx *c, double *pe, double *box, double *virial) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (pe) *pe = c->npt_pe;
  if (box)
    for (int d = 0; d < 3; ++d) box[d] = c->box[d];
  if (virial) *virial = c->npt_vir;
  return VCSGC_OK;
}

vcsgc_status vcsgc_get_thermostat(vcsgc_ctx *c, double *xi, double *eta) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!c->nvt) return fail(c, VCSGC_E_INVALID_ARG, "not an MD context");
  double h[2];
  VC_CHECK(c, hipMemcpyAsync(h, c->nvt, sizeof(h), hipMemcpyDeviceToHost, c->stream), "copy");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  if (xi) *xi = h[0];
  if (eta) *eta = h[1];
  return VCSGC_OK;
}

vcsgc_status vcsgc_minimize(vcsgc_ctx *c, const vcsgc_cg_params *prm, vcsgc_cg_result *res) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (c->reps.size() != 1) return fail(c, VCSGC_E_INVALID_ARG, "not available on a batch context");
  if (!prm || !c->fx)
    return fail(c, VCSGC_E_INVALID_ARG, "relaxation needs parameters and force arrays");
  const double lmin = std::min({c->box[0], c->box[1], c->box[2]});
  if (prm->max_iter < 0 || prm->max_eval < 0 || !is_fin(prm->etol) || !is_fin(prm->ftol) ||
      prm->ftol < 0.0 || !is_fin(prm->dmax) || !(prm->dmax > 0.0) || !(prm->dmax < 0.5 * lmin))
    return fail(c, VCSGC_E_INVALID_ARG,
                "need max_iter, max_eval >= 0, finite etol, ftol >= 0, 0 < dmax < L/2");
  const int64_t n = c->n;
  if (!c->cg) VC_CHECK(c, dalloc(&c->cg, 9 * (size_t)n + 2 * (size_t)((n + vc::BLOCK - 1) / vc::BLOCK) + 8),
                       "allocation");
  double *d = c->cg, *x0 = c->cg + 3 * n, *f0 = c->cg + 6 * n;
  c->rho_f_fresh = false;
  if (!c->md_valid) {
    st = refresh_md(c);
    if (st) return st;
  }
  VC_CHECK(c, hipMemsetAsync(&c->ds->rebuild[0], 0, sizeof(int), c->stream), "reset");
  VC_CHECK(c, vc::launch_pack(c), "pack");
  double E = 0.0;
  st = cg_eval(c, false, &E);
  if (st) return st;
  VC_CHECK(c, vc::launch_cg_dir(c, d, 0.0, true), "relaxation");
  double t[2];
  st = cg_totals(c, 1, d, t);
  if (st) return st;
  double gg = t[0], dE_prev = 0.0;
  int64_t it = 0, ev = 0;
  int32_t reason = 0;
  bool moved = false;
  for (;;) {
    if (std::sqrt(gg) <= prm->ftol) {
      reason = VCSGC_CG_FORCE;
      break;
    }
    if (it >= prm->max_iter) {
      reason = VCSGC_CG_ITER;
      break;
    }
    if (ev >= prm->max_eval) {
      reason = VCSGC_CG_EVAL;
      break;
    }
    if ((st = cg_totals(c, 0, d, t))) return st;
    double sl = t[0], dm2 = t[1];
    if (!(sl > 0.0)) {  // not a descent direction: restart along the force
      VC_CHECK(c, vc::launch_cg_dir(c, d, 0.0, true), "relaxation");
      if ((st = cg_totals(c, 0, d, t))) return st;
      sl = t[0];
      dm2 = t[1];
    }
    double a = prm->dmax / std::sqrt(dm2);
    if (it > 0) {
      const double a1 = 2.0 * dE_prev / sl;
      if (a1 < a) a = a1;
    }
    if ((st = cg_gather3(c, x0, c->x, c->y, c->z))) return st;
    if ((st = cg_gather3(c, f0, c->fx, c->fy, c->fz))) return st;
    double Et = 0.0;
    bool accepted = false;
    for (int k = 0; k < VCSGC_CG_TRIALS; ++k) {
      VC_CHECK(c, vc::launch_cg_move(c, x0, d, a), "relaxation");
      moved = true;
      if ((st = cg_eval(c, true, &Et))) return st;
      ev += 1;
      if (Et <= E - VCSGC_CG_C1 * a * sl && Et < E) {
        accepted = true;
        break;
      }
      a = a * 0.5;
    }
    if (!accepted) {  // back to the line search's start (forces recomputed there)
      VC_CHECK(c, vc::launch_cg_move(c, x0, d, 0.0), "relaxation");
      double e_back = 0.0;
      if ((st = cg_eval(c, true, &e_back))) return st;
      reason = VCSGC_CG_LINESEARCH;
      break;
    }
    if ((st = cg_totals(c, 1, f0, t))) return st;
    const double g_new = t[0], g_mix = t[1];
    double b = (g_new - g_mix) / gg;
    if (!(b > 0.0)) b = 0.0;
    VC_CHECK(c, vc::launch_cg_dir(c, d, b, false), "relaxation");
    const double dE = E - Et;
    dE_prev = dE;
    E = Et;
    gg = g_new;
    it += 1;
    if (dE <= prm->etol * std::fabs(E)) {
      reason = VCSGC_CG_ENERGY;
      break;
    }
  }
  if (moved) c->mc_valid = false;
  c->rho_f_fresh = true;  // the last evaluation ran at the final positions
  if (res) {
    res->iterations = it;
    res->evaluations = ev;
    res->energy = E;
    res->fnorm = std::sqrt(gg);
    res->reason = reason;
  }
  return VCSGC_OK;
}

vcsgc_status md_verlet_step(vcsgc_ctx *c, double dt_fs, int64_t n_steps) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (c->reps.size() != 1) return fail(c, VCSGC_E_INVALID_ARG, "not available on a batch context");
  if (!c->vx || !c->fx)
    return fail(c, VCSGC_E_INVALID_ARG, "MD needs velocity and force arrays");
  if (!is_fin(dt_fs) || !(dt_fs > 0.0) || n_steps < 0)
    return fail(c, VCSGC_E_INVALID_ARG, "need dt > 0 and n_steps >= 0");
  c->rho_f_fresh = false;
  if (!c->md_valid) {
    st = refresh_md(c);
    if (st) return st;
  }
  if (c->npt_tau > 0.0 && !(c->nvt_T > 0.0))
    return fail(c, VCSGC_E_INVALID_ARG, "the barostat needs the thermostat (vcsgc_set_thermostat)");
  if (n_steps > 0) c->mc_valid = false;
  if (c->npt_tau > 0.0)
    st = md_npt_steps(c, dt_fs, n_steps);
  else if (c->nvt_T > 0.0)
    st = md_nvt_steps(c, dt_fs, n_steps, vc::md_rebuild_on_device(c));
  else
    st = (n_steps > 0 && vc::md_rebuild_on_device(c)) ? md_steps_device(c, dt_fs, n_steps)
                                                      : md_steps_host(c, dt_fs, n_steps);
  if (st) return st;
  c->rho_f_fresh = true;  // the last force pass ran at the final positions
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
  vcsgc_stats s;
  int err = 0;
  VC_CHECK(c, vc::persist_read_stats(c, &s, &err), "state");  // n_final of replica 0
  out->sweeps_done = c->w;
  out->n_b = s.n_final;
  out->seed = c->last_seed;
  if (out->rho_dev) {
    st = ensure_mc(c);
    if (st) return st;
    VC_CHECK(c, hipMemcpyAsync(out->rho_dev, c->rho, sizeof(double) * c->n,
                               hipMemcpyDeviceToDevice, c->stream),
             "state");
    VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  }
  return VCSGC_OK;
}

vcsgc_status vcsgc_set_state(vcsgc_ctx *c, const vcsgc_state *in) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!in) return fail(c, VCSGC_E_INVALID_ARG, "null input");
  c->w = in->sweeps_done;
  c->last_seed = in->seed;
  VC_CHECK(c, vc::persist_count(c), "state");  // n_B recounted from the species
  c->mc_valid = false;  // species may have been restored: fresh density cache
  c->rho_f_fresh = false;
  if (in->rho_dev) {
    // lists for the current positions (with a fresh cache), then the saved cache
    st = refresh_mc(c);
    if (st) return st;
    VC_CHECK(c, hipMemcpyAsync(c->rho, in->rho_dev, sizeof(double) * c->n,
                               hipMemcpyDeviceToDevice, c->stream),
             "state");
  }
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  return VCSGC_OK;
}

vcsgc_status vcsgc_copy_rho(vcsgc_ctx *c, double *rho_dev) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!rho_dev) return fail(c, VCSGC_E_INVALID_ARG, "null output");
  st = ensure_mc(c);
  if (st) return st;
  VC_CHECK(c, hipMemcpyAsync(rho_dev, c->rho, sizeof(double) * c->n, hipMemcpyDeviceToDevice,
                             c->stream),
           "copy");
  return VCSGC_OK;
}

vcsgc_status vcsgc_atom_energies(vcsgc_ctx *c, double *e_dev) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (c->reps.size() != 1) return fail(c, VCSGC_E_INVALID_ARG, "not available on a batch context");
  if (!e_dev) return fail(c, VCSGC_E_INVALID_ARG, "null output");
  if (!c->md_valid) {
    st = refresh_md(c);
    if (st) return st;
  }
  VC_CHECK(c, vc::launch_pack(c), "pack");
  VC_CHECK(c, vc::launch_energy(c), "energy");
  c->rho_f_fresh = true;
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
  out->stages_per_sweep = c->reps.size() == 1 ? vc::stages_per_sweep(c) : c->S;
  out->kmax = vc::KMAX;
  if (c->mc_valid && c->mc_stats_stale) {
    VC_CHECK(c, vc::launch_mc_row_stats(c), "neighbour list");
    c->mc_stats_stale = false;
  }
  hipError_t e;
  vc::DevState h = read_state(c, &e);
  if (e != hipSuccess) return dev_fail(c, e, "info");
  out->mc_kmax_used = c->mc_valid ? h.kmax_used : 0;
  out->mc_pairs = c->mc_valid ? (int64_t)h.pairs_mc : 0;
  out->md_pairs = c->md_valid ? (int64_t)h.pairs_md : 0;
  out->md_rebuilds = c->md_rebuilds;
  return VCSGC_OK;
}

vcsgc_status vcsgc_set_sample_log(vcsgc_ctx *c, double *desc_dev, double *dE_dev, int64_t cap,
                                  int64_t stride) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (desc_dev && (!c->desc || !dE_dev || cap < 0 || stride < 1))
    return fail(c, VCSGC_E_INVALID_ARG,
                "sample log needs VCSGC_FLAG_DESCRIPTOR, both buffers, cap >= 0, stride >= 1");
  if (desc_dev && c->reps.size() != 1)
    return fail(c, VCSGC_E_INVALID_ARG, "sample log needs a single-system context");
  c->smp_desc = desc_dev;
  c->smp_de = desc_dev ? dE_dev : nullptr;
  c->smp_cap = desc_dev ? cap : 0;
  c->smp_stride = stride < 1 ? 1 : stride;
  const unsigned long long zero = 0;
  VC_CHECK(c, hipMemcpyAsync(&c->ds->smp_n, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream),
           "reset");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  return VCSGC_OK;
}

vcsgc_status vcsgc_sample_count(vcsgc_ctx *c, int64_t *n_logged) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!n_logged) return fail(c, VCSGC_E_INVALID_ARG, "null output");
  hipError_t e;
  vc::DevState h = read_state(c, &e);
  if (e != hipSuccess) return dev_fail(c, e, "sample count");
  *n_logged = (int64_t)h.smp_n;
  return VCSGC_OK;
}

vcsgc_status vcsgc_set_surrogate(vcsgc_ctx *c, const vcsgc_mlp *m, int32_t mode) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (mode < 0 || mode > 3) return fail(c, VCSGC_E_INVALID_ARG, "mode must be in [0, 3]");
  if (mode != 0 && c->reps.size() != 1)
    return fail(c, VCSGC_E_INVALID_ARG, "delayed acceptance needs a single-system context");
  if (mode == 1) {
    if (!m) return fail(c, VCSGC_E_NO_SURROGATE, "mode 1 needs a network");
    if (!c->desc) return fail(c, VCSGC_E_INVALID_ARG, "mode 1 needs VCSGC_FLAG_DESCRIPTOR");
    if (c->r_dep < vc::DESC_CUT + c->pot.rc)
      return fail(c, VCSGC_E_INVALID_ARG, "mode 1 needs r_dep >= 4.41 + rc");
  }
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  c->mlp = mode == 1 ? m : nullptr;
  c->da_mode = mode;
  return VCSGC_OK;
}

vcsgc_status vcsgc_set_surrogate_log(vcsgc_ctx *c, double *log_dev, int64_t cap) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (log_dev && cap < 0) return fail(c, VCSGC_E_INVALID_ARG, "negative capacity");
  c->dalog = log_dev;
  c->dacap = log_dev ? cap : 0;
  const unsigned long long zero = 0;
  VC_CHECK(c, hipMemcpyAsync(&c->ds->dalog_n, &zero, sizeof(zero), hipMemcpyHostToDevice,
                             c->stream),
           "reset");
  VC_CHECK(c, hipStreamSynchronize(c->stream), "sync");
  return VCSGC_OK;
}

vcsgc_status vcsgc_descriptors(vcsgc_ctx *c, const int32_t *sites_dev, int64_t n, int32_t flip,
                               double *out_dev) {
  vcsgc_status st = check_ctx(c);
  if (st) return st;
  if (!c->desc) return fail(c, VCSGC_E_INVALID_ARG, "needs VCSGC_FLAG_DESCRIPTOR");
  if (n < 0 || (n > 0 && (!sites_dev || !out_dev))) return fail(c, VCSGC_E_INVALID_ARG, "bad arguments");
  st = ensure_mc(c);
  if (st) return st;
  VC_CHECK(c, vc::launch_descriptors(c, sites_dev, n, flip, out_dev), "descriptors");
  return VCSGC_OK;
}

vcsgc_status vcsgc_selftest_sqrt(const double *in_dev, double *out_dev, int64_t n,
                                 hipStream_t stream) {
  if (n < 0 || (n > 0 && (!in_dev || !out_dev))) return VCSGC_E_INVALID_ARG;
  hipError_t e = vc::launch_sqrt(in_dev, out_dev, n, stream);
  return e == hipSuccess ? VCSGC_OK : VCSGC_E_DEVICE;
}

vcsgc_status vcsgc_selftest_md_math(const double *a_dev, const double *b_dev, double *sqrt_dev,
                                    double *div_dev, int64_t n, hipStream_t stream) {
  if (n < 0 || (n > 0 && (!a_dev || !b_dev || !sqrt_dev || !div_dev)))
    return VCSGC_E_INVALID_ARG;
  hipError_t e = vc::launch_md_math(a_dev, b_dev, sqrt_dev, div_dev, n, stream);
  return e == hipSuccess ? VCSGC_OK : VCSGC_E_DEVICE;
}

}  // extern "C"
