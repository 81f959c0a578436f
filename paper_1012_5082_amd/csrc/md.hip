// EAM density, embedding derivative, per-atom energy and forces from the
// r < rc + skin list (gather only: every atom sums its own row, no atomics),
// and the velocity-Verlet kick/drift updates.
#include "common.hpp"

namespace vc {

struct Box {
  double L0, L1, L2;
};

// rho_i = sum_{j: r < rc} t_{s_j} (rc - r)^2 and F'_i = -A_{s_i} / (2 sqrt(rho_i))
__global__ void k_density_md(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                             const double *__restrict__ z, const int32_t *__restrict__ nj,
                             const uint8_t *__restrict__ cnt, const uint8_t *__restrict__ sp,
                             Box b, PotD p, double *rho, double *fp) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i], zi = z[i];
  double s = 0.0;
  const int m = cnt[i];
  for (int k = 0; k < m; ++k) {
    const int32_t j = nj[(int64_t)k * n + i];
    const double dx = min_image(x[j] - xi, b.L0);
    const double dy = min_image(y[j] - yi, b.L1);
    const double dz = min_image(z[j] - zi, b.L2);
    const double r = sqrt((dx * dx + dy * dy) + dz * dz);
    if (!(r < p.rc)) continue;
    const double d = p.rc - r;
    s += p.t[sp[j]] * (d * d);
  }
  rho[i] = s;
  fp[i] = dembed(p, sp[i], s);
}

// F_i = sum_j [phi'(r) + F'_i f'_{s_j}(r) + F'_j f'_{s_i}(r)] (x_j - x_i) / r with
// phi'(r) = eps ((-2 d)(c0 + c1 r) + c1 d^2) and f'_X(r) = (-2 t_X) d, d = rc - r
__global__ void k_forces(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                         const double *__restrict__ z, const int32_t *__restrict__ nj,
                         const uint8_t *__restrict__ cnt, const uint8_t *__restrict__ sp,
                         const double *__restrict__ fp, Box b, PotD p, double *fx, double *fy,
                         double *fz) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i], zi = z[i];
  const int si = sp[i];
  const double fpi = fp[i];
  double ax = 0.0, ay = 0.0, az = 0.0;
  const int m = cnt[i];
  for (int k = 0; k < m; ++k) {
    const int32_t j = nj[(int64_t)k * n + i];
    const double dx = min_image(x[j] - xi, b.L0);
    const double dy = min_image(y[j] - yi, b.L1);
    const double dz = min_image(z[j] - zi, b.L2);
    const double r = sqrt((dx * dx + dy * dy) + dz * dz);
    if (!(r < p.rc)) continue;
    const int sj = sp[j];
    const double d = p.rc - r;
    const double dphi = p.eps[si + sj] * (-2.0 * d * (p.c0 + p.c1 * r) + p.c1 * (d * d));
    const double dfj = -2.0 * p.t[sj] * d;
    const double dfi = -2.0 * p.t[si] * d;
    const double s = dphi + fpi * dfj + fp[j] * dfi;
    const double coef = s / r;
    ax += coef * dx;
    ay += coef * dy;
    az += coef * dz;
  }
  fx[i] = ax;
  fy[i] = ay;
  fz[i] = az;
}

// E_i = F_{s_i}(rho_i) + 0.5 sum_j (eps d^2)(c0 + c1 r)
__global__ void k_energy(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                         const double *__restrict__ z, const int32_t *__restrict__ nj,
                         const uint8_t *__restrict__ cnt, const uint8_t *__restrict__ sp,
                         const double *__restrict__ rho, Box b, PotD p, double *e) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i], zi = z[i];
  const int si = sp[i];
  double ps = 0.0;
  const int m = cnt[i];
  for (int k = 0; k < m; ++k) {
    const int32_t j = nj[(int64_t)k * n + i];
    const double dx = min_image(x[j] - xi, b.L0);
    const double dy = min_image(y[j] - yi, b.L1);
    const double dz = min_image(z[j] - zi, b.L2);
    const double r = sqrt((dx * dx + dy * dy) + dz * dz);
    if (!(r < p.rc)) continue;
    const double d = p.rc - r;
    ps += p.eps[si + sp[j]] * (d * d) * (p.c0 + p.c1 * r);
  }
  e[i] = embed(p, si, rho[i]) + 0.5 * ps;
}

hipError_t launch_forces(vcsgc_ctx *c) {
  Box b{c->box[0], c->box[1], c->box[2]};
  k_density_md<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->x, c->y, c->z, c->md_j,
                                                        c->md_cnt, c->sp, b, c->pot, c->rho_f,
                                                        c->fp);
  k_forces<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->x, c->y, c->z, c->md_j, c->md_cnt,
                                                    c->sp, c->fp, b, c->pot, c->fx, c->fy, c->fz);
  return hipGetLastError();
}

hipError_t launch_energy(vcsgc_ctx *c) {
  Box b{c->box[0], c->box[1], c->box[2]};
  k_density_md<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->x, c->y, c->z, c->md_j,
                                                        c->md_cnt, c->sp, b, c->pot, c->rho_f,
                                                        c->fp);
  k_energy<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->x, c->y, c->z, c->md_j, c->md_cnt,
                                                    c->sp, c->rho_f, b, c->pot, c->eatom);
  return hipGetLastError();
}

// v += (dt/2)(F cm); x = wrap(x + dt v); flag a list rebuild when an atom has
// moved more than skin/2 from its position at the last build
__global__ void k_kick_drift(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                             double *vz, const double *__restrict__ fx,
                             const double *__restrict__ fy, const double *__restrict__ fz,
                             const uint8_t *__restrict__ sp, const double *__restrict__ xr,
                             const double *__restrict__ yr, const double *__restrict__ zr, Box b,
                             PotD p, double dt, double half_skin2, DevState *ds) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double cm = p.cm[sp[i]];
  const double hdt = 0.5 * dt;
  const double ux = vx[i] + hdt * (fx[i] * cm);
  const double uy = vy[i] + hdt * (fy[i] * cm);
  const double uz = vz[i] + hdt * (fz[i] * cm);
  vx[i] = ux;
  vy[i] = uy;
  vz[i] = uz;
  const double nx = wrap_box(x[i] + dt * ux, b.L0);
  const double ny = wrap_box(y[i] + dt * uy, b.L1);
  const double nz = wrap_box(z[i] + dt * uz, b.L2);
  x[i] = nx;
  y[i] = ny;
  z[i] = nz;
  const double ex = min_image(nx - xr[i], b.L0);
  const double ey = min_image(ny - yr[i], b.L1);
  const double ez = min_image(nz - zr[i], b.L2);
  if ((ex * ex + ey * ey) + ez * ez > half_skin2) atomicOr(&ds->rebuild, 1);
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

hipError_t launch_kick_drift(vcsgc_ctx *c, double dt) {
  Box b{c->box[0], c->box[1], c->box[2]};
  const double hs = 0.5 * c->skin;
  k_kick_drift<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->x, c->y, c->z, c->vx, c->vy,
                                                        c->vz, c->fx, c->fy, c->fz, c->sp, c->xr,
                                                        c->yr, c->zr, b, c->pot, dt, hs * hs,
                                                        c->ds);
  return hipGetLastError();
}

hipError_t launch_kick(vcsgc_ctx *c, double dt) {
  k_kick<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->vx, c->vy, c->vz, c->fx, c->fy, c->fz,
                                                  c->sp, c->pot, dt);
  return hipGetLastError();
}

}  // namespace vc
