// EAM density, embedding derivative, per-atom energy and forces from the
// r < rc + skin list (gather only: every atom sums its own row, no atomics),
// and the velocity-Verlet kick/drift updates.
#include "common.hpp"

namespace vc {

struct Box {
  double L0, L1, L2;
};

constexpr int IB = 16;  // neighbour indices loaded per round
constexpr int UNR = 4;  // neighbour gathers in flight per lane

// Minimum image without branches: both shifted values are formed and one is
// selected (the same number min_image returns), so the pair bodies below
// are straight-line code the compiler can interleave.
__device__ __forceinline__ double min_image_sel(double d, double L) {
  const double h = 0.5 * L;
  const double lo = d + L, hi = d - L;
  return d > h ? hi : (d < -h ? lo : d);
}

// (x, y, z, species) of every atom, packed for the density pass
__global__ void k_pack(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                       const double *__restrict__ z, const uint8_t *__restrict__ sp,
                       double4 *ps4) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ps4[i] = make_double4(x[i], y[i], z[i], (double)sp[i]);
}

hipError_t launch_pack(vcsgc_ctx *c) {
  k_pack<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->x, c->y, c->z, c->sp, c->ps4);
  return hipGetLastError();
}

// rho_i = sum_{j: r < rc} f_{s_j}(r) over the row of i, in entry order
// (f_X = t_X (rc - r)^2, or the tables when TAB): the indices of up to IB
// entries in one round, then the gathers UNR at a time
template <bool TAB>
__device__ __forceinline__ double density_row(int64_t n, int64_t i, int m, const double4 &qi,
                                              const double4 *__restrict__ ps4,
                                              const int32_t *__restrict__ nj, const Box &b,
                                              const PotD &p) {
  const double t0 = p.t[0], t1 = p.t[1];
  double s = 0.0;
  for (int k0 = 0; k0 < m; k0 += IB) {
    int32_t jb[IB];
#pragma unroll
    for (int u = 0; u < IB; ++u) jb[u] = k0 + u < m ? nj[(int64_t)(k0 + u) * n + i] : (int32_t)i;
#pragma unroll
    for (int g = 0; g < IB; g += UNR) {
      if (k0 + g >= m) break;
      double4 q[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) q[u] = ps4[jb[g + u]];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const double dx = min_image_sel(q[u].x - qi.x, b.L0);
        const double dy = min_image_sel(q[u].y - qi.y, b.L1);
        const double dz = min_image_sel(q[u].z - qi.z, b.L2);
        const double r = sqrt_md((dx * dx + dy * dy) + dz * dz);
        const bool in = k0 + g + u < m && r < p.rc;
        double term;
        if (TAB) {
          term = spline_at(tab_radial(p, q[u].w != 0.0 ? 1 : 0), p.nr, in ? r : 0.0, p.inv_dr,
                           nullptr);
        } else {
          const double d = p.rc - r;
          term = (q[u].w != 0.0 ? t1 : t0) * (d * d);
        }
        // a skipped pair adds +0.0: s is never -0.0, so s + 0.0 == s (the
        // padding entries, the atom itself at r^2 = 0, have r = NaN from
        // sqrt_md, which the select drops)
        s += in ? term : 0.0;
      }
    }
  }
  return s;
}

// rho_i, and (x_i, y_i, z_i, F'_i) with F'_i = F'_{s_i}(rho_i) for the force
// pass
template <bool TAB>
__global__ void __launch_bounds__(BLOCK)
    k_density_md(int64_t n, const double4 *__restrict__ ps4, const int32_t *__restrict__ nj,
                 const uint8_t *__restrict__ cnt, const uint8_t *__restrict__ sp, Box b, PotD p,
                 double *rho, double4 *pf4) {
  const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 qi = ps4[i];
  const int m = cnt[i];
  const double s = density_row<TAB>(n, i, m, qi, ps4, nj, b, p);
  rho[i] = s;
  const double f = dembed(p, sp[i], s);
  pf4[i] = make_double4(qi.x, qi.y, qi.z, f);
}

// [v += (dt/2)(F cm) (closing the previous step) ;] v += (dt/2)(F cm);
// x = wrap(x + dt v); raise ds->rebuild[par] when an atom has moved more than
// skin/2 from its position at the last build.  Also readies the next
// device-decided rebuild: the flag of the other parity (read by the previous
// step's rebuild kernels, which have finished) is cleared, and so are the
// search-bin counts (bcount may be NULL).
struct KickDrift {
  double *x, *y, *z, *vx, *vy, *vz;
  const double *xr, *yr, *zr;  // positions at the last MD-list build
  double4 *ps4;
  double dt, half_skin2;
  int kick_first, par;
  int32_t *bcount;
  int64_t nbins;
  DevState *ds;
  const double *nvt;  // Nose-Hoover: v = (v s1) s2 before the kick (nvt[3], nvt[4]); NULL: none
};

// The step's clearing work, by thread i of a grid of `threads`.
__device__ __forceinline__ void kick_drift_clear(const KickDrift &k, int64_t i, int64_t threads) {
  if (k.bcount)
    for (int64_t q = i; q < k.nbins; q += threads) k.bcount[q] = 0;
  if (i == 0) k.ds->rebuild[k.par ^ 1] = 0;
}

// Kick and drift of atom i (species s) from its force; every active lane of
// the wave takes part in the rebuild vote.
__device__ __forceinline__ void kick_drift_atom(const KickDrift &k, int64_t i, int s, double x0,
                                                double y0, double z0, double fxi, double fyi,
                                                double fzi, const Box &b, const PotD &p) {
  const double cm = p.cm[s];
  const double hdt = 0.5 * k.dt;
  const double ax = fxi * cm, ay = fyi * cm, az = fzi * cm;
  double ux = k.vx[i], uy = k.vy[i], uz = k.vz[i];
  if (k.nvt) {
    const double s1 = k.nvt[3], s2 = k.nvt[4];
    ux = ux * s1;
    uy = uy * s1;
    uz = uz * s1;
    ux = ux * s2;
    uy = uy * s2;
    uz = uz * s2;
  }
  if (k.kick_first) {
    ux = ux + hdt * ax;
    uy = uy + hdt * ay;
    uz = uz + hdt * az;
  }
  ux = ux + hdt * ax;
  uy = uy + hdt * ay;
  uz = uz + hdt * az;
  k.vx[i] = ux;
  k.vy[i] = uy;
  k.vz[i] = uz;
  const double nx = wrap_box(x0 + k.dt * ux, b.L0);
  const double ny = wrap_box(y0 + k.dt * uy, b.L1);
  const double nz = wrap_box(z0 + k.dt * uz, b.L2);
  k.x[i] = nx;
  k.y[i] = ny;
  k.z[i] = nz;
  k.ps4[i] = make_double4(nx, ny, nz, (double)s);
  const double ex = min_image(nx - k.xr[i], b.L0);
  const double ey = min_image(ny - k.yr[i], b.L1);
  const double ez = min_image(nz - k.zr[i], b.L2);
  const unsigned long long moved = __ballot((ex * ex + ey * ey) + ez * ez > k.half_skin2);
  if (moved && __lane_id() == __ffsll((long long)moved) - 1) atomicOr(&k.ds->rebuild[k.par], 1);
}

// F_i = sum_j [phi'(r) + F'_i f'_{s_j}(r) + F'_j f'_{s_i}(r)] (x_j - x_i) / r with
// phi'(r) = eps ((-2 d)(c0 + c1 r) + c1 d^2) and f'_X(r) = (-2 t_X) d, d = rc - r,
// summed in entry order (Finnis-Sinclair forms, or the tables when TAB).
// VIR: also *wv += s r for each pair, s = phi'(r) + F'_i f'_{s_j}(r) + F'_j f'_{s_i}(r)
// (the atom's share of the virial sum), in the same order.
template <bool TAB, bool VIR = false>
__device__ __forceinline__ void force_row(int64_t n, int64_t i, int m, int si, const double4 &qi,
                                          const double4 *__restrict__ pf4,
                                          const int32_t *__restrict__ nj,
                                          const uint8_t *__restrict__ sp, const Box &b,
                                          const PotD &p, double &ax, double &ay, double &az,
                                          double *wv = nullptr) {
  const double fpi = qi.w;
  const double e0 = p.eps[si], e1 = p.eps[si + 1], t0 = p.t[0], t1 = p.t[1], ti = p.t[si];
  for (int k0 = 0; k0 < m; k0 += IB) {
    int32_t jb[IB];
#pragma unroll
    for (int u = 0; u < IB; ++u) jb[u] = k0 + u < m ? nj[(int64_t)(k0 + u) * n + i] : (int32_t)i;
#pragma unroll
    for (int g = 0; g < IB; g += UNR) {
      if (k0 + g >= m) break;
      double4 q[UNR];
      int sj[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        q[u] = pf4[jb[g + u]];
        sj[u] = sp[jb[g + u]];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const double dx = min_image(q[u].x - qi.x, b.L0);
        const double dy = min_image(q[u].y - qi.y, b.L1);
        const double dz = min_image(q[u].z - qi.z, b.L2);
        const double r = sqrt_md((dx * dx + dy * dy) + dz * dz);
        // branch kept here: the select form evaluates the FP64 division for
        // every list entry and measured slower than this one
        if (k0 + g + u < m && r < p.rc) {
          double dphi, dfj, dfi;
          if (TAB) {
            spline_at(tab_radial(p, 2 + si + sj[u]), p.nr, r, p.inv_dr, &dphi);
            spline_at(tab_radial(p, sj[u]), p.nr, r, p.inv_dr, &dfj);
            spline_at(tab_radial(p, si), p.nr, r, p.inv_dr, &dfi);
          } else {
            const double d = p.rc - r;
            const double eps = sj[u] ? e1 : e0, tj = sj[u] ? t1 : t0;
            dphi = eps * (-2.0 * d * (p.c0 + p.c1 * r) + p.c1 * (d * d));
            dfj = -2.0 * tj * d;
            dfi = -2.0 * ti * d;
          }
          const double s = dphi + fpi * dfj + q[u].w * dfi;
          if (VIR) *wv = *wv + s * r;
          const double coef = div_md(s, r);
          ax += coef * dx;
          ay += coef * dy;
          az += coef * dz;
        }
      }
    }
  }
}

// KD: the forces are not stored but go straight into the next step's kick
// and drift (the positions it writes are not read by this pass, which
// gathers pf4).  TAB: tabulated potential.
template <bool KD, bool TAB>
__global__ void __launch_bounds__(BLOCK)
    k_forces(int64_t n, const double4 *__restrict__ pf4, const int32_t *__restrict__ nj,
             const uint8_t *__restrict__ cnt, const uint8_t *__restrict__ sp, Box b, PotD p,
             double *fx, double *fy, double *fz, KickDrift kd) {
  const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
  if (KD) kick_drift_clear(kd, i, (int64_t)gridDim.x * blockDim.x);
  if (i >= n) return;
  const double4 qi = pf4[i];
  const int si = sp[i];
  const int m = cnt[i];
  double ax = 0.0, ay = 0.0, az = 0.0;
  force_row<TAB>(n, i, m, si, qi, pf4, nj, sp, b, p, ax, ay, az);
  if (KD) {
    // the packed positions equal x, y, z bit for bit
    kick_drift_atom(kd, i, si, qi.x, qi.y, qi.z, ax, ay, az, b, p);
  } else {
    fx[i] = ax;
    fy[i] = ay;
    fz[i] = az;
  }
}

// forces and w_i = sum_j s_ij r_ij (the virial is -1/2 sum_i w_i)
template <bool TAB>
__global__ void __launch_bounds__(BLOCK)
    k_forces_vir(int64_t n, const double4 *__restrict__ pf4, const int32_t *__restrict__ nj,
                 const uint8_t *__restrict__ cnt, const uint8_t *__restrict__ sp, Box b, PotD p,
                 double *fx, double *fy, double *fz, double *w) {
  const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 qi = pf4[i];
  const int si = sp[i];
  const int m = cnt[i];
  double ax = 0.0, ay = 0.0, az = 0.0, wv = 0.0;
  force_row<TAB, true>(n, i, m, si, qi, pf4, nj, sp, b, p, ax, ay, az, &wv);
  fx[i] = ax;
  fy[i] = ay;
  fz[i] = az;
  w[i] = wv;
}

// E_i = F_{s_i}(rho_i) + 0.5 sum_j phi_{s_i s_j}(r)
__global__ void k_energy(int64_t n, const double4 *__restrict__ ps4, const int32_t *__restrict__ nj,
                         const uint8_t *__restrict__ cnt, const double *__restrict__ rho, Box b,
                         PotD p, double *e) {
  const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 qi = ps4[i];
  const int si = (int)qi.w;
  double ps = 0.0;
  const int m = cnt[i];
  for (int k = 0; k < m; ++k) {
    const int32_t j = nj[(int64_t)k * n + i];
    const double4 qj = ps4[j];
    const double dx = min_image(qj.x - qi.x, b.L0);
    const double dy = min_image(qj.y - qi.y, b.L1);
    const double dz = min_image(qj.z - qi.z, b.L2);
    const double r = sqrt((dx * dx + dy * dy) + dz * dz);
    if (!(r < p.rc)) continue;
    ps += pot_phi(p, si, (int)qj.w, r);
  }
  e[i] = embed(p, si, rho[i]) + 0.5 * ps;
}

// the density pass and the force pass for the context's potential form
static void density_md_launch(vcsgc_ctx *c, const Box &b) {
  if (c->pot.tab)
    k_density_md<true><<<grid_for(c->n), BLOCK, 0, c->stream>>>(
        c->n, c->ps4, c->md_j, c->md_cnt, c->sp, b, c->pot, c->rho_f, c->pf4);
  else
    k_density_md<false><<<grid_for(c->n), BLOCK, 0, c->stream>>>(
        c->n, c->ps4, c->md_j, c->md_cnt, c->sp, b, c->pot, c->rho_f, c->pf4);
}

template <bool KD>
static void forces_launch(vcsgc_ctx *c, const Box &b, const KickDrift &kd) {
  if (c->pot.tab)
    k_forces<KD, true><<<grid_for(c->n), BLOCK, 0, c->stream>>>(
        c->n, c->pf4, c->md_j, c->md_cnt, c->sp, b, c->pot, c->fx, c->fy, c->fz, kd);
  else
    k_forces<KD, false><<<grid_for(c->n), BLOCK, 0, c->stream>>>(
        c->n, c->pf4, c->md_j, c->md_cnt, c->sp, b, c->pot, c->fx, c->fy, c->fz, kd);
}

hipError_t launch_forces(vcsgc_ctx *c) {
  Box b{c->box[0], c->box[1], c->box[2]};
  int h = tstart(c, VCSGC_KT_DENSITY);
  density_md_launch(c, b);
  tstop(c, h);
  h = tstart(c, VCSGC_KT_FORCES);
  forces_launch<false>(c, b, KickDrift{});
  tstop(c, h);
  return hipGetLastError();
}

static KickDrift kick_drift_args(vcsgc_ctx *c, double dt, bool kick_first, int par) {
  const double hs = 0.5 * c->skin;
  KickDrift k{};
  k.x = c->x;
  k.y = c->y;
  k.z = c->z;
  k.vx = c->vx;
  k.vy = c->vy;
  k.vz = c->vz;
  k.xr = c->xr;
  k.yr = c->yr;
  k.zr = c->zr;
  k.ps4 = c->ps4;
  k.dt = dt;
  k.half_skin2 = hs * hs;
  k.kick_first = kick_first ? 1 : 0;
  k.par = par;
  k.bcount = c->bin_count;
  k.nbins = c->reps[0].nbins;
  k.ds = c->ds;
  return k;
}

hipError_t launch_forces_kick_drift(vcsgc_ctx *c, double dt, bool kick_first, int par) {
  Box b{c->box[0], c->box[1], c->box[2]};
  int h = tstart(c, VCSGC_KT_DENSITY);
  density_md_launch(c, b);
  tstop(c, h);
  h = tstart(c, VCSGC_KT_FORCES);
  forces_launch<true>(c, b, kick_drift_args(c, dt, kick_first, par));
  tstop(c, h);
  return hipGetLastError();
}

hipError_t launch_energy(vcsgc_ctx *c) {
  Box b{c->box[0], c->box[1], c->box[2]};
  int h = tstart(c, VCSGC_KT_ENERGY);
  density_md_launch(c, b);
  k_energy<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->ps4, c->md_j, c->md_cnt, c->rho_f,
                                                    b, c->pot, c->eatom);
  tstop(c, h);
  return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK)
    k_kick_drift(int64_t n, const double *__restrict__ fx, const double *__restrict__ fy,
                 const double *__restrict__ fz, const uint8_t *__restrict__ sp, Box b, PotD p,
                 KickDrift k) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  kick_drift_clear(k, i, (int64_t)gridDim.x * blockDim.x);
  if (i >= n) return;
  kick_drift_atom(k, i, sp[i], k.x[i], k.y[i], k.z[i], fx[i], fy[i], fz[i], b, p);
}

__global__ void k_kick(int64_t n, double *vx, double *vy, double *vz, const double *__restrict__ fx,
                       const double *__restrict__ fy, const double *__restrict__ fz,
                       const uint8_t *__restrict__ sp, PotD p, double dt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double cm = p.cm[sp[i]];
  const double hdt = 0.5 * dt;
  vx[i] = vx[i] + hdt * (fx[i] * cm);
  vy[i] = vy[i] + hdt * (fy[i] * cm);
  vz[i] = vz[i] + hdt * (fz[i] * cm);
}

hipError_t launch_kick_drift(vcsgc_ctx *c, double dt, bool kick_first, int par) {
  Box b{c->box[0], c->box[1], c->box[2]};
  int h = tstart(c, VCSGC_KT_KICKDRIFT);
  k_kick_drift<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->fx, c->fy, c->fz, c->sp, b,
                                                        c->pot,
                                                        kick_drift_args(c, dt, kick_first, par));
  tstop(c, h);
  return hipGetLastError();
}

hipError_t launch_kick(vcsgc_ctx *c, double dt) {
  int h = tstart(c, VCSGC_KT_KICK);
  k_kick<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->vx, c->vy, c->vz, c->fx, c->fy, c->fz,
                                                  c->sp, c->pot, dt);
  tstop(c, h);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Nose-Hoover NVT.  Per step: the thermostat's half steps at the step
// boundary (one block), the scaled kick and drift, forces, the closing kick
// fused with the kinetic-energy chunk sums.  The kinetic energy that steers
// the thermostat is summed in a fixed shape: chunks of 256 atoms by halving
// strides (one block per chunk), chunk c into accumulator c mod 256, and the
// accumulators by halving strides again.
// ---------------------------------------------------------------------------
// chunk sums of m ((vx^2 + vy^2) + vz^2), after the closing half kick if KICK
template <bool KICK>
__global__ void __launch_bounds__(BLOCK)
    k_nvt_ke(int64_t n, double *vx, double *vy, double *vz, const double *__restrict__ fx,
             const double *__restrict__ fy, const double *__restrict__ fz,
             const uint8_t *__restrict__ sp, PotD p, double dt, double *part) {
  __shared__ double a[BLOCK];
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  double t = 0.0;
  if (i < n) {
    const int s = sp[i];
    double ux = vx[i], uy = vy[i], uz = vz[i];
    if (KICK) {
      const double cm = p.cm[s];
      const double hdt = 0.5 * dt;
      ux = ux + hdt * (fx[i] * cm);
      uy = uy + hdt * (fy[i] * cm);
      uz = uz + hdt * (fz[i] * cm);
      vx[i] = ux;
      vy[i] = uy;
      vz[i] = uz;
    }
    t = p.mass[s] * ((ux * ux + uy * uy) + uz * uz);
  }
  a[threadIdx.x] = t;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) a[threadIdx.x] = a[threadIdx.x] + a[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = a[0];
}

struct NvtPar {
  double dt, g, kT, Q;
};

// one half step (dt/2) of xi, eta and the carried kinetic energy K; returns
// the velocity factor s = (1 - xi dt/4) / (1 + xi dt/4)
__device__ __forceinline__ double nh_half(const NvtPar &q, double &K, double &xi, double &eta) {
  const double q4 = 0.25 * q.dt;
  xi = xi + q4 * ((2.0 * K - q.g * q.kT) / q.Q);
  const double a = xi * q4;
  const double s = (1.0 - a) / (1.0 + a);
  K = K * s * s;
  eta = eta + xi * (0.5 * q.dt);
  xi = xi + q4 * ((2.0 * K - q.g * q.kT) / q.Q);
  return s;
}

// K from the chunk sums; the end-of-step half (mode bit 0) and the next
// step's opening half (bit 1); nvt = (xi, eta, K, s1, s2)
__global__ void __launch_bounds__(BLOCK)
    k_nvt_thermo(int64_t nch, const double *__restrict__ part, double *nvt, NvtPar q, int mode) {
  __shared__ double a[BLOCK];
  double acc = 0.0;
  for (int64_t c = threadIdx.x; c < nch; c += BLOCK) acc = acc + part[c];
  a[threadIdx.x] = acc;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) a[threadIdx.x] = a[threadIdx.x] + a[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double K = 0.5 * a[0] / ACC;
    double xi = nvt[0], eta = nvt[1];
    double s1 = 1.0, s2 = 1.0;
    if (mode & 1) s1 = nh_half(q, K, xi, eta);
    if (mode & 2) s2 = nh_half(q, K, xi, eta);
    nvt[0] = xi;
    nvt[1] = eta;
    nvt[2] = K;
    nvt[3] = s1;
    nvt[4] = s2;
  }
}

// v = v s1 (the last end-of-step half of a call)
__global__ void k_nvt_scale(int64_t n, double *vx, double *vy, double *vz,
                            const double *__restrict__ nvt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s1 = nvt[3];
  vx[i] = vx[i] * s1;
  vy[i] = vy[i] * s1;
  vz[i] = vz[i] * s1;
}

hipError_t launch_nvt_ke(vcsgc_ctx *c, double dt, bool closing_kick) {
  const unsigned nch = (unsigned)((c->n + BLOCK - 1) / BLOCK);
  int h = tstart(c, VCSGC_KT_KICK);
  if (closing_kick)
    k_nvt_ke<true><<<nch, BLOCK, 0, c->stream>>>(c->n, c->vx, c->vy, c->vz, c->fx, c->fy, c->fz,
                                                 c->sp, c->pot, dt, c->nvt_part);
  else
    k_nvt_ke<false><<<nch, BLOCK, 0, c->stream>>>(c->n, c->vx, c->vy, c->vz, c->fx, c->fy,
                                                  c->fz, c->sp, c->pot, dt, c->nvt_part);
  tstop(c, h);
  return hipGetLastError();
}

hipError_t launch_nvt_thermo(vcsgc_ctx *c, double dt, int mode) {
  NvtPar q;
  q.dt = dt;
  q.g = 3.0 * (double)c->n - 3.0;
  q.kT = KB * c->nvt_T;
  q.Q = q.g * q.kT * c->nvt_tau * c->nvt_tau;
  k_nvt_thermo<<<1, BLOCK, 0, c->stream>>>((c->n + BLOCK - 1) / BLOCK, c->nvt_part, c->nvt, q,
                                          mode);
  return hipGetLastError();
}

hipError_t launch_nvt_kick_drift(vcsgc_ctx *c, double dt, int par) {
  Box b{c->box[0], c->box[1], c->box[2]};
  KickDrift k = kick_drift_args(c, dt, false, par);
  k.nvt = c->nvt;
  int h = tstart(c, VCSGC_KT_KICKDRIFT);
  k_kick_drift<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->fx, c->fy, c->fz, c->sp, b,
                                                        c->pot, k);
  tstop(c, h);
  return hipGetLastError();
}

hipError_t launch_nvt_scale(vcsgc_ctx *c) {
  k_nvt_scale<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->vx, c->vy, c->vz, c->nvt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Conjugate-gradient relaxation: the per-atom work of the minimizer driven
// from the host (trial positions, the fixed-shape totals that steer it, the
// direction update).  Vectors of 3n doubles hold the x, y and z components
// one after the other.  Totals are taken in the fixed shape of the energy
// reduction: chunks of BLOCK atoms by halving strides, chunk c into
// accumulator c mod BLOCK, the accumulators by halving strides.
// ---------------------------------------------------------------------------
// x = wrap(x0 + a d) per component, ps4 packed alongside; raises
// ds->rebuild[0] when an atom is more than skin/2 from its position at the
// last MD-list build
__global__ void __launch_bounds__(BLOCK)
    k_cg_move(int64_t n, const double *__restrict__ x0, const double *__restrict__ d, double a,
              double *x, double *y, double *z, const uint8_t *__restrict__ sp, double4 *ps4,
              const double *__restrict__ xr, const double *__restrict__ yr,
              const double *__restrict__ zr, Box b, double half_skin2, DevState *ds) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  bool far = false;
  if (i < n) {
    const double nx = wrap_box(x0[i] + a * d[i], b.L0);
    const double ny = wrap_box(x0[n + i] + a * d[n + i], b.L1);
    const double nz = wrap_box(x0[2 * n + i] + a * d[2 * n + i], b.L2);
    x[i] = nx;
    y[i] = ny;
    z[i] = nz;
    ps4[i] = make_double4(nx, ny, nz, (double)sp[i]);
    const double ex = min_image(nx - xr[i], b.L0);
    const double ey = min_image(ny - yr[i], b.L1);
    const double ez = min_image(nz - zr[i], b.L2);
    far = (ex * ex + ey * ey) + ez * ez > half_skin2;
  }
  const unsigned long long moved = __ballot(far);
  if (moved && __lane_id() == __ffsll((long long)moved) - 1) atomicOr(&ds->rebuild[0], 1);
}

// Chunk values of two totals, per-atom dot terms (a_x b_x + a_y b_y) + a_z b_z:
// MODE 0: F . u and max_i |u_i|^2;  MODE 1: F . F and F . u.
// part[c] and part[nch + c] for chunk c.
template <int MODE>
__global__ void __launch_bounds__(BLOCK)
    k_cg_part(int64_t n, const double *__restrict__ fx, const double *__restrict__ fy,
              const double *__restrict__ fz, const double *__restrict__ u, double *part) {
  __shared__ double s0[BLOCK], s1[BLOCK];
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * BLOCK + t;
  double a = 0.0, q = 0.0;
  if (i < n) {
    const double gx = fx[i], gy = fy[i], gz = fz[i];
    const double ux = u[i], uy = u[n + i], uz = u[2 * n + i];
    if (MODE == 0) {
      a = (gx * ux + gy * uy) + gz * uz;
      q = (ux * ux + uy * uy) + uz * uz;
    } else {
      a = (gx * gx + gy * gy) + gz * gz;
      q = (gx * ux + gy * uy) + gz * uz;
    }
  }
  s0[t] = a;
  s1[t] = q;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if (t < h) {
      s0[t] = s0[t] + s0[t + h];
      s1[t] = MODE == 0 ? fmax(s1[t], s1[t + h]) : s1[t] + s1[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    const int64_t nch = gridDim.x;
    part[blockIdx.x] = s0[0];
    part[nch + blockIdx.x] = s1[0];
  }
}

// the two totals from the chunk values (one block): out[0], out[1]
template <int MODE>
__global__ void __launch_bounds__(BLOCK)
    k_cg_total(int64_t nch, const double *__restrict__ part, double *out) {
  __shared__ double s0[BLOCK], s1[BLOCK];
  const int t = threadIdx.x;
  double a = 0.0, q = 0.0;
  for (int64_t c = t; c < nch; c += BLOCK) {
    a = a + part[c];
    q = MODE == 0 ? fmax(q, part[nch + c]) : q + part[nch + c];
  }
  s0[t] = a;
  s1[t] = q;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if (t < h) {
      s0[t] = s0[t] + s0[t + h];
      s1[t] = MODE == 0 ? fmax(s1[t], s1[t + h]) : s1[t] + s1[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
  }
}

// d = F (copy) or d = F + b d
__global__ void __launch_bounds__(BLOCK)
    k_cg_dir(int64_t n, const double *__restrict__ fx, const double *__restrict__ fy,
             const double *__restrict__ fz, double *d, double b, int copy) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  if (copy) {
    d[i] = fx[i];
    d[n + i] = fy[i];
    d[2 * n + i] = fz[i];
  } else {
    d[i] = fx[i] + b * d[i];
    d[n + i] = fy[i] + b * d[n + i];
    d[2 * n + i] = fz[i] + b * d[2 * n + i];
  }
}

hipError_t launch_cg_move(vcsgc_ctx *c, const double *x0, const double *d, double a) {
  Box b{c->box[0], c->box[1], c->box[2]};
  const double hs = 0.5 * c->skin;
  k_cg_move<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, x0, d, a, c->x, c->y, c->z, c->sp,
                                                     c->ps4, c->xr, c->yr, c->zr, b, hs * hs,
                                                     c->ds);
  return hipGetLastError();
}

hipError_t launch_cg_totals(vcsgc_ctx *c, int mode, const double *u, double *part, double *out) {
  const int nch = grid_for(c->n);
  if (mode == 0) {
    k_cg_part<0><<<nch, BLOCK, 0, c->stream>>>(c->n, c->fx, c->fy, c->fz, u, part);
    k_cg_total<0><<<1, BLOCK, 0, c->stream>>>(nch, part, out);
  } else {
    k_cg_part<1><<<nch, BLOCK, 0, c->stream>>>(c->n, c->fx, c->fy, c->fz, u, part);
    k_cg_total<1><<<1, BLOCK, 0, c->stream>>>(nch, part, out);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Isotropic NPT (Nose-Hoover thermostat and barostat), the per-atom parts of
// a step driven from the host: the scalings, kicks and drift of the
// splitting T(h) B(h) V(h) X(dt) [forces] V(h) B(h) T(h) (h = dt/2) take
// their factors from the host, which integrates the thermostat and barostat
// variables from the fixed-shape totals of the kinetic energy and virial.
// ---------------------------------------------------------------------------
// v = ((v f1) f2) c; v += h a; v = v c; x = wrap((x q + dt v) q) in the new
// box; ps4 packed; raises ds->rebuild[0] when some atom is farther than thr
// from its list-build position scaled to the new box (lam = L / L_build per
// axis), or always when thr <= 0
__global__ void __launch_bounds__(BLOCK)
    k_npt_kick_drift(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                     double *vz, const double *__restrict__ fx, const double *__restrict__ fy,
                     const double *__restrict__ fz, const uint8_t *__restrict__ sp, PotD p,
                     double f1, double f2, double c, double h, double dt, double q, Box b,
                     double lx, double ly, double lz, double thr,
                     const double *__restrict__ xr, const double *__restrict__ yr,
                     const double *__restrict__ zr, double4 *ps4, DevState *ds) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  bool far = false;
  if (i < n) {
    const int s = sp[i];
    const double cm = p.cm[s];
    double ux = vx[i], uy = vy[i], uz = vz[i];
    ux = ux * f1;
    uy = uy * f1;
    uz = uz * f1;
    ux = ux * f2;
    uy = uy * f2;
    uz = uz * f2;
    ux = ux * c;
    uy = uy * c;
    uz = uz * c;
    ux = ux + h * (fx[i] * cm);
    uy = uy + h * (fy[i] * cm);
    uz = uz + h * (fz[i] * cm);
    ux = ux * c;
    uy = uy * c;
    uz = uz * c;
    vx[i] = ux;
    vy[i] = uy;
    vz[i] = uz;
    const double nx = wrap_box((x[i] * q + dt * ux) * q, b.L0);
    const double ny = wrap_box((y[i] * q + dt * uy) * q, b.L1);
    const double nz = wrap_box((z[i] * q + dt * uz) * q, b.L2);
    x[i] = nx;
    y[i] = ny;
    z[i] = nz;
    ps4[i] = make_double4(nx, ny, nz, (double)s);
    const double ex = min_image(nx - lx * xr[i], b.L0);
    const double ey = min_image(ny - ly * yr[i], b.L1);
    const double ez = min_image(nz - lz * zr[i], b.L2);
    far = !(thr > 0.0) || (ex * ex + ey * ey) + ez * ez > thr * thr;
  }
  const unsigned long long moved = __ballot(far);
  if (moved && __lane_id() == __ffsll((long long)moved) - 1) atomicOr(&ds->rebuild[0], 1);
}

// [v = v c; v += h a; v = v c;] chunk values of m ((vx^2 + vy^2) + vz^2)
// into part[c] and of w into part[nch + c]
template <bool KICK>
__global__ void __launch_bounds__(BLOCK)
    k_npt_kick_sums(int64_t n, double *vx, double *vy, double *vz,
                    const double *__restrict__ fx, const double *__restrict__ fy,
                    const double *__restrict__ fz, const uint8_t *__restrict__ sp, PotD p,
                    double c, double h, const double *__restrict__ w, double *part) {
  __shared__ double s0[BLOCK], s1[BLOCK];
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * BLOCK + t;
  double a = 0.0, q = 0.0;
  if (i < n) {
    const int s = sp[i];
    double ux = vx[i], uy = vy[i], uz = vz[i];
    if (KICK) {
      const double cm = p.cm[s];
      ux = ux * c;
      uy = uy * c;
      uz = uz * c;
      ux = ux + h * (fx[i] * cm);
      uy = uy + h * (fy[i] * cm);
      uz = uz + h * (fz[i] * cm);
      ux = ux * c;
      uy = uy * c;
      uz = uz * c;
      vx[i] = ux;
      vy[i] = uy;
      vz[i] = uz;
    }
    a = p.mass[s] * ((ux * ux + uy * uy) + uz * uz);
    q = w[i];
  }
  s0[t] = a;
  s1[t] = q;
  __syncthreads();
  for (int hh = BLOCK / 2; hh > 0; hh >>= 1) {
    if (t < hh) {
      s0[t] = s0[t] + s0[t + hh];
      s1[t] = s1[t] + s1[t + hh];
    }
    __syncthreads();
  }
  if (t == 0) {
    const int64_t nch = gridDim.x;
    part[blockIdx.x] = s0[0];
    part[nch + blockIdx.x] = s1[0];
  }
}

// v *= s
__global__ void k_scale_v(int64_t n, double *vx, double *vy, double *vz, double s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  vx[i] = vx[i] * s;
  vy[i] = vy[i] * s;
  vz[i] = vz[i] * s;
}

hipError_t launch_forces_virial(vcsgc_ctx *c, double *w) {
  Box b{c->box[0], c->box[1], c->box[2]};
  int h = tstart(c, VCSGC_KT_DENSITY);
  density_md_launch(c, b);
  tstop(c, h);
  h = tstart(c, VCSGC_KT_FORCES);
  if (c->pot.tab)
    k_forces_vir<true><<<grid_for(c->n), BLOCK, 0, c->stream>>>(
        c->n, c->pf4, c->md_j, c->md_cnt, c->sp, b, c->pot, c->fx, c->fy, c->fz, w);
  else
    k_forces_vir<false><<<grid_for(c->n), BLOCK, 0, c->stream>>>(
        c->n, c->pf4, c->md_j, c->md_cnt, c->sp, b, c->pot, c->fx, c->fy, c->fz, w);
  tstop(c, h);
  return hipGetLastError();
}

hipError_t launch_npt_kick_drift(vcsgc_ctx *c, double f1, double f2, double cv, double h,
                                 double dt, double q, const double lam[3], double thr) {
  Box b{c->box[0], c->box[1], c->box[2]};
  int t = tstart(c, VCSGC_KT_KICKDRIFT);
  k_npt_kick_drift<<<grid_for(c->n), BLOCK, 0, c->stream>>>(
      c->n, c->x, c->y, c->z, c->vx, c->vy, c->vz, c->fx, c->fy, c->fz, c->sp, c->pot, f1, f2,
      cv, h, dt, q, b, lam[0], lam[1], lam[2], thr, c->xr, c->yr, c->zr, c->ps4, c->ds);
  tstop(c, t);
  return hipGetLastError();
}

hipError_t launch_npt_sums(vcsgc_ctx *c, bool kick, double cv, double h, const double *w,
                           double *part, double *out) {
  const int nch = grid_for(c->n);
  int t = tstart(c, VCSGC_KT_KICK);
  if (kick)
    k_npt_kick_sums<true><<<nch, BLOCK, 0, c->stream>>>(c->n, c->vx, c->vy, c->vz, c->fx, c->fy,
                                                        c->fz, c->sp, c->pot, cv, h, w, part);
  else
    k_npt_kick_sums<false><<<nch, BLOCK, 0, c->stream>>>(c->n, c->vx, c->vy, c->vz, c->fx,
                                                         c->fy, c->fz, c->sp, c->pot, cv, h, w,
                                                         part);
  k_cg_total<1><<<1, BLOCK, 0, c->stream>>>(nch, part, out);
  tstop(c, t);
  return hipGetLastError();
}

hipError_t launch_scale_v(vcsgc_ctx *c, double s) {
  k_scale_v<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->vx, c->vy, c->vz, s);
  return hipGetLastError();
}

hipError_t launch_cg_dir(vcsgc_ctx *c, double *d, double b, bool copy) {
  k_cg_dir<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->fx, c->fy, c->fz, d, b,
                                                    copy ? 1 : 0);
  return hipGetLastError();
}

}  // namespace vc
