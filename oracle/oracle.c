/*
 * Plain serial FP64 reference ("oracle") of the parallel VC-SGC transmutation
 * Monte Carlo and EAM molecular dynamics of Sadigh et al. (arXiv:1012.5082).
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares no
 * code with the HIP library.  Compiled with -O2 -ffp-contract=off so that every
 * expression below is evaluated exactly as written (no fused multiply-add).
 *
 * Every floating-point expression is written in the order stated in its
 * comment; the reading of the paper that each step follows is cited there.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_KB 8.617333262e-5      /* Boltzmann constant, eV/K */
#define OR_ACC 9.648533212e-3     /* (eV/Angstrom)/u -> Angstrom/fs^2 */
#define OR_TIE 1e-9               /* near-tie margin |ln u + x| */

/* ------------------------------------------------------------------------ */
/* Philox4x64-10: ten rounds of two 64x64->128 multiplies and a Feistel-like  */
/* mix; the key is bumped by the Weyl constants between rounds.              */
/* ------------------------------------------------------------------------ */
static const uint64_t PH_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PH_M1 = 0xCA5A826395121157ULL;
static const uint64_t PH_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t PH_W1 = 0xBB67AE8584CAA73BULL;

void or_philox4x64_10(const uint64_t key[2], const uint64_t ctr[4], uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += PH_W0;
      k1 += PH_W1;
    }
    unsigned __int128 p0 = (unsigned __int128)PH_M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)PH_M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* floor(w * m / 2^64): a uniform index in [0, m) from a 64-bit word. */
static uint64_t or_index(uint64_t w, uint64_t m) {
  return (uint64_t)(((unsigned __int128)w * m) >> 64);
}

/* (w >> 11 + 1/2) 2^-53: a uniform double strictly inside (0, 1). */
static double or_unit(uint64_t w) {
  return ((double)(w >> 11) + 0.5) * 0x1p-53;
}

/* ------------------------------------------------------------------------ */
/* Neighbour lists                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t j, code;
  double r, dx, dy, dz;
} nent;

static int cmp_nent(const void *a, const void *b) {
  const nent *u = (const nent *)a, *v = (const nent *)b;
  if (u->j != v->j) return u->j < v->j ? -1 : 1;
  if (u->code != v->code) return u->code < v->code ? -1 : 1;
  return 0;
}

/* Minimum-image separation along one periodic axis. */
static double or_mimage(double d, double L) {
  double h = 0.5 * L;
  if (d > h) return d - L;
  if (d < -h) return d + L;
  return d;
}

typedef struct {
  nent *e;
  int64_t n, cap;
} nbuf;

static void nbuf_push(nbuf *b, nent v) {
  if (b->n == b->cap) {
    b->cap = b->cap ? 2 * b->cap : 64;
    b->e = (nent *)realloc(b->e, (size_t)b->cap * sizeof(nent));
  }
  b->e[b->n++] = v;
}

/* Separation r = sqrt((dx^2 + dy^2) + dz^2); a pair is a neighbour iff r < cutoff.
 * (The squared test only skips pairs that are certainly farther away.) */
static int or_try_pair(nbuf *row, int32_t j, int32_t code, double dx, double dy, double dz,
                       double cutoff) {
  double r2 = (dx * dx + dy * dy) + dz * dz;
  if (r2 > 1.000001 * cutoff * cutoff) return 0;
  double r = sqrt(r2);
  if (r < cutoff) {
    nent v = {j, code, r, dx, dy, dz};
    nbuf_push(row, v);
    return 1;
  }
  return 0;
}

/* Candidate search of a neighbour list: mode 1 minimum image over all
 * pairs, 2 explicit image sums, 3 the 27 bins of edge >= cutoff around the
 * atom's bin. */
typedef struct {
  int mode, nb[3];
  int32_t *bin_start, *bin_atoms, *bin_of;
} nbr_grid;

/* Row i of the neighbour list (all j with r < cutoff), ascending (j, image). */
static void or_nbr_row(int64_t i, int64_t n, const double *x, const double *y, const double *z,
                       const double box[3], double cutoff, const nbr_grid *G, nbuf *rowp) {
  const int mode = G->mode;
  const int *nb = G->nb;
  const int32_t *bin_start = G->bin_start, *bin_atoms = G->bin_atoms, *bin_of = G->bin_of;
  nbuf row = *rowp;
  row.n = 0;
  if (mode == 1) {
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      or_try_pair(&row, (int32_t)j, 13, or_mimage(x[j] - x[i], box[0]),
                  or_mimage(y[j] - y[i], box[1]), or_mimage(z[j] - z[i], box[2]), cutoff);
    }
  } else if (mode == 2) {
    for (int64_t j = 0; j < n; ++j) {
      for (int sz = -1; sz <= 1; ++sz)
        for (int sy = -1; sy <= 1; ++sy)
          for (int sx = -1; sx <= 1; ++sx) {
            if (j == i && sx == 0 && sy == 0 && sz == 0) continue;
            int code = (sx + 1) + 3 * ((sy + 1) + 3 * (sz + 1));
            or_try_pair(&row, (int32_t)j, code, (x[j] - x[i]) + sx * box[0],
                        (y[j] - y[i]) + sy * box[1], (z[j] - z[i]) + sz * box[2], cutoff);
          }
    }
  } else {
    int b = bin_of[i];
    int bx = b % nb[0], by = (b / nb[0]) % nb[1], bz = b / (nb[0] * nb[1]);
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          int cx = (bx + ox + nb[0]) % nb[0];
          int cy = (by + oy + nb[1]) % nb[1];
          int cz = (bz + oz + nb[2]) % nb[2];
          int c = cx + nb[0] * (cy + nb[1] * cz);
          for (int32_t k = bin_start[c]; k < bin_start[c + 1]; ++k) {
            int32_t j = bin_atoms[k];
            if (j == i) continue;
            or_try_pair(&row, j, 13, or_mimage(x[j] - x[i], box[0]),
                        or_mimage(y[j] - y[i], box[1]), or_mimage(z[j] - z[i], box[2]),
                        cutoff);
          }
        }
  }
  /* ascending (j, image) by insertion sort */
  for (int64_t a = 1; a < row.n; ++a) {
    nent v = row.e[a];
    int64_t b = a - 1;
    while (b >= 0 && cmp_nent(&row.e[b], &v) > 0) {
      row.e[b + 1] = row.e[b];
      --b;
    }
    row.e[b + 1] = v;
  }
  *rowp = row;
}

/* Mode choice (mode 0: bins when the box holds three cutoffs per axis,
 * else minimum image, else image sums) and, for mode 3, the bins. */
static int or_nbr_setup(int64_t n, const double *x, const double *y, const double *z,
                        const double box[3], double cutoff, int mode, nbr_grid *G) {
  double Lmin = box[0];
  if (box[1] < Lmin) Lmin = box[1];
  if (box[2] < Lmin) Lmin = box[2];
  if (!(Lmin > cutoff)) return -1;
  if (mode == 0) mode = (Lmin >= 3.0 * cutoff) ? 3 : (Lmin >= 2.0 * cutoff ? 1 : 2);
  if (mode == 1 && !(Lmin >= 2.0 * cutoff)) return -1;
  if (mode == 3 && !(Lmin >= 3.0 * cutoff)) return -1;

  /* mode 3: candidates from the 27 surrounding bins of edge >= cutoff */
  int nb[3] = {1, 1, 1};
  int32_t *bin_start = NULL, *bin_atoms = NULL, *bin_of = NULL;
  if (mode == 3) {
    for (int d = 0; d < 3; ++d) nb[d] = (int)(box[d] / cutoff);
    int64_t nbins = (int64_t)nb[0] * nb[1] * nb[2];
    bin_start = (int32_t *)calloc((size_t)nbins + 1, sizeof(int32_t));
    bin_atoms = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    bin_of = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
      const double *u[3] = {x, y, z};
      int b[3];
      for (int d = 0; d < 3; ++d) {
        b[d] = (int)(u[d][i] / (box[d] / nb[d]));
        if (b[d] < 0) b[d] = 0;
        if (b[d] >= nb[d]) b[d] = nb[d] - 1;
      }
      bin_of[i] = b[0] + nb[0] * (b[1] + nb[1] * b[2]);
      bin_start[bin_of[i] + 1]++;
    }
    for (int64_t c = 0; c < nbins; ++c) bin_start[c + 1] += bin_start[c];
    int32_t *fill = (int32_t *)malloc((size_t)nbins * sizeof(int32_t));
    memcpy(fill, bin_start, (size_t)nbins * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) bin_atoms[fill[bin_of[i]]++] = (int32_t)i;
    free(fill);
  }

  G->mode = mode;
  for (int d = 0; d < 3; ++d) G->nb[d] = nb[d];
  G->bin_start = bin_start;
  G->bin_atoms = bin_atoms;
  G->bin_of = bin_of;
  return 0;
}

static void or_nbr_free(nbr_grid *G) {
  free(G->bin_start);
  free(G->bin_atoms);
  free(G->bin_of);
}

int64_t or_neighbors(int64_t n, const double *x, const double *y, const double *z,
                     const double box[3], double cutoff, int mode, int64_t cap,
                     int64_t *start, int32_t *nj, double *nr,
                     double *ndx, double *ndy, double *ndz) {
  nbr_grid G;
  if (or_nbr_setup(n, x, y, z, box, cutoff, mode, &G)) return -1;

  nbuf row = {0, 0, 0};
  int64_t total = 0;
  for (int64_t i = 0; i < n; ++i) {
    or_nbr_row(i, n, x, y, z, box, cutoff, &G, &row);
    if (start) start[i] = total;
    for (int64_t k = 0; k < row.n; ++k, ++total) {
      if (total < cap) {
        nj[total] = row.e[k].j;
        nr[total] = row.e[k].r;
        if (ndx) ndx[total] = row.e[k].dx;
        if (ndy) ndy[total] = row.e[k].dy;
        if (ndz) ndz[total] = row.e[k].dz;
      }
    }
  }
  if (start) start[n] = total;
  free(row.e);
  or_nbr_free(&G);
  return total;
}

/* ------------------------------------------------------------------------ */
/* Potential (Finnis-Sinclair form or tables; species 0 = A, 1 = B)         */
/* ------------------------------------------------------------------------ */
void or_spline_coeffs(int32_t n, const double *y, double *c) {
  for (int32_t k = 0; k + 1 < n; ++k) {
    double mk = k == 0 ? y[1] - y[0] : 0.5 * (y[k + 1] - y[k - 1]);
    double mk1 = k + 2 == n ? y[n - 1] - y[n - 2] : 0.5 * (y[k + 2] - y[k]);
    double d = y[k + 1] - y[k];
    c[4 * k + 0] = y[k];
    c[4 * k + 1] = mk;
    c[4 * k + 2] = (3.0 * d - 2.0 * mk) - mk1;
    c[4 * k + 3] = (mk + mk1) - 2.0 * d;
  }
}

double or_spline_eval(const double *c, int32_t n, double x, double inv_h, double *der) {
  double p = x * inv_h;
  double top = (double)(n - 1);
  double pc = p < 0.0 ? 0.0 : (p > top ? top : p);
  int32_t k = (int32_t)pc;
  if (k > n - 2) k = n - 2;
  double t = p - (double)k;
  const double *a = c + 4 * k;
  if (der) *der = (((3.0 * a[3]) * t + 2.0 * a[2]) * t + a[1]) * inv_h;
  return ((a[3] * t + a[2]) * t + a[1]) * t + a[0];
}

static double or_eps(const or_pot *p, int a, int b) {
  int s = a + b;
  return s == 0 ? p->eps_aa : (s == 1 ? p->eps_ab : p->eps_bb);
}

/* phi_XY(r) = (eps_XY (rc - r)^2) (c0 + c1 r), or the table's */
static double or_phi(const or_pot *p, int a, int b, double r) {
  if (p->tab) return or_spline_eval(p->cphi[a + b], p->nr, r, p->inv_dr, NULL);
  double d = p->rc - r;
  return or_eps(p, a, b) * (d * d) * (p->c0 + p->c1 * r);
}

/* phi'_XY(r) = eps_XY ((-2 (rc - r)) (c0 + c1 r) + c1 (rc - r)^2), or the table's */
static double or_dphi(const or_pot *p, int a, int b, double r) {
  if (p->tab) {
    double g;
    or_spline_eval(p->cphi[a + b], p->nr, r, p->inv_dr, &g);
    return g;
  }
  double d = p->rc - r;
  return or_eps(p, a, b) * (-2.0 * d * (p->c0 + p->c1 * r) + p->c1 * (d * d));
}

/* f_X(r) = t_X (rc - r)^2, or the table's */
static double or_f(const or_pot *p, int a, double r) {
  if (p->tab) return or_spline_eval(p->cf[a], p->nr, r, p->inv_dr, NULL);
  double d = p->rc - r;
  return (a ? p->t_b : p->t_a) * (d * d);
}

/* f'_X(r) = (-2 t_X) (rc - r), or the table's */
static double or_df(const or_pot *p, int a, double r) {
  if (p->tab) {
    double g;
    or_spline_eval(p->cf[a], p->nr, r, p->inv_dr, &g);
    return g;
  }
  double d = p->rc - r;
  return -2.0 * (a ? p->t_b : p->t_a) * d;
}

/* F_X(rho) = -A_X sqrt(max(rho, 0)), or the table's */
static double or_embed(const or_pot *p, int a, double rho) {
  if (p->tab) return or_spline_eval(p->cF[a], p->nrho, rho, p->inv_drho, NULL);
  double A = a ? p->a_b : p->a_a;
  return -A * sqrt(rho > 0.0 ? rho : 0.0);
}

/* F'_X(rho) = -A_X / (2 sqrt(rho)), and 0 at rho = 0; or the table's */
static double or_dembed(const or_pot *p, int a, double rho) {
  if (p->tab) {
    double g;
    or_spline_eval(p->cF[a], p->nrho, rho, p->inv_drho, &g);
    return g;
  }
  double A = a ? p->a_b : p->a_a;
  return rho > 0.0 ? -A / (2.0 * sqrt(rho)) : 0.0;
}

/* rho_i = sum_j f_{s_j}(r_ij), in neighbour order. */
static double or_density_row(int64_t i, const int64_t *start, const int32_t *nj,
                             const double *nr, const uint8_t *species, const or_pot *p) {
  double s = 0.0;
  for (int64_t e = start[i]; e < start[i + 1]; ++e)
    if (nr[e] < p->rc) s += or_f(p, species[nj[e]], nr[e]);
  return s;
}

void or_density(int64_t n, const int64_t *start, const int32_t *nj, const double *nr,
                const uint8_t *species, const or_pot *p, double *rho) {
  for (int64_t i = 0; i < n; ++i) rho[i] = or_density_row(i, start, nj, nr, species, p);
}

/* E_i = F_{s_i}(rho_i) + (1/2) sum_j phi_{s_i s_j}(r_ij); U = sum_i E_i. */
void or_energy_atoms(int64_t n, const int64_t *start, const int32_t *nj, const double *nr,
                     const uint8_t *species, const or_pot *p, const double *rho, double *e) {
  for (int64_t i = 0; i < n; ++i) {
    double ps = 0.0;
    for (int64_t k = start[i]; k < start[i + 1]; ++k)
      if (nr[k] < p->rc) ps += or_phi(p, species[i], species[nj[k]], nr[k]);
    e[i] = or_embed(p, species[i], rho[i]) + 0.5 * ps;
  }
}

double or_energy_total(int64_t n, const double *e) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += e[i];
  return s;
}

static void or_force_row(int64_t i, const int64_t *start, const int32_t *nj, const double *nr,
                         const double *ndx, const double *ndy, const double *ndz,
                         const uint8_t *species, const or_pot *p, const double *fp,
                         double *fx, double *fy, double *fz) {
  double ax = 0.0, ay = 0.0, az = 0.0;
  int si = species[i];
  for (int64_t e = start[i]; e < start[i + 1]; ++e) {
    double r = nr[e];
    if (!(r < p->rc)) continue;
    int32_t j = nj[e];
    int sj = species[j];
    double s = or_dphi(p, si, sj, r) + fp[i] * or_df(p, sj, r) + fp[j] * or_df(p, si, r);
    double coef = s / r;
    ax += coef * ndx[e];
    ay += coef * ndy[e];
    az += coef * ndz[e];
  }
  fx[i] = ax;
  fy[i] = ay;
  fz[i] = az;
}

/* F_i = -dU/dx_i = sum_j [phi'(r) + F'_i f'_{s_j}(r) + F'_j f'_{s_i}(r)] (x_j - x_i) / r */
void or_forces(int64_t n, const int64_t *start, const int32_t *nj, const double *nr,
               const double *ndx, const double *ndy, const double *ndz,
               const uint8_t *species, const or_pot *p, const double *rho,
               double *fx, double *fy, double *fz) {
  double *fp = (double *)malloc((size_t)n * sizeof(double));
  for (int64_t i = 0; i < n; ++i) fp[i] = or_dembed(p, species[i], rho[i]);
  for (int64_t i = 0; i < n; ++i)
    or_force_row(i, start, nj, nr, ndx, ndy, ndz, species, p, fp, fx, fy, fz);
  free(fp);
}

/*
 * Energy change of the transmutation s_i -> 1 - s_i (Sec. II.A, the
 * definition of Delta U), written locally for an EAM potential:
 *   dU = [F_{s'}(rho_i) - F_s(rho_i)]                              own embedding
 *      + sum_j [phi_{s' s_j}(r_ij) - phi_{s s_j}(r_ij)]            pair terms
 *      + sum_j [F_{s_j}(rho_j + delta_j) - F_{s_j}(rho_j)]         neighbours' embedding
 * with delta_j = sum over the images of i near j of [f_{s'}(r) - f_s(r)]
 * (one image per neighbour unless the box is smaller than twice the cutoff).
 * Evaluated as (own + pair) + emb, each sum in neighbour order.
 */
double or_delta_u(int64_t i, const int64_t *start, const int32_t *nj, const double *nr,
                  const uint8_t *species, const double *rho, const or_pot *p) {
  int s = species[i], s1 = 1 - s;
  double own = or_embed(p, s1, rho[i]) - or_embed(p, s, rho[i]);
  double pair = 0.0, emb = 0.0;
  for (int64_t e = start[i]; e < start[i + 1]; ++e) {
    if (!(nr[e] < p->rc)) continue;
    int sj = species[nj[e]];
    pair += or_phi(p, s1, sj, nr[e]) - or_phi(p, s, sj, nr[e]);
  }
  for (int64_t e = start[i]; e < start[i + 1]; ++e) {
    if (e > start[i] && nj[e] == nj[e - 1]) continue;  /* images already aggregated */
    int32_t j = nj[e];
    double delta = 0.0;
    int any = 0;
    for (int64_t e2 = e; e2 < start[i + 1] && nj[e2] == j; ++e2) {
      if (!(nr[e2] < p->rc)) continue;
      delta += or_f(p, s1, nr[e2]) - or_f(p, s, nr[e2]);
      any = 1;
    }
    if (!any) continue;
    int sj = species[j];
    emb += or_embed(p, sj, rho[j] + delta) - or_embed(p, sj, rho[j]);
  }
  return own + pair + emb;
}

/* Commit of a transmutation at i: rho_j += delta_j for every neighbour, then flip. */
static void or_commit(int64_t i, const int64_t *start, const int32_t *nj, const double *nr,
                      uint8_t *species, double *rho, const or_pot *p) {
  int s = species[i], s1 = 1 - s;
  for (int64_t e = start[i]; e < start[i + 1]; ++e) {
    if (e > start[i] && nj[e] == nj[e - 1]) continue;
    int32_t j = nj[e];
    double delta = 0.0;
    int any = 0;
    for (int64_t e2 = e; e2 < start[i + 1] && nj[e2] == j; ++e2) {
      if (!(nr[e2] < p->rc)) continue;
      delta += or_f(p, s1, nr[e2]) - or_f(p, s, nr[e2]);
      any = 1;
    }
    if (any) rho[j] = rho[j] + delta;
  }
  species[i] = (uint8_t)s1;
}

/* ------------------------------------------------------------------------ */
/* Cells (Sec. III.A): with colour period P per axis, the box is cut into a  */
/* multiple of P cells of edge >= r_dep / (P - 1) per dimension; cells whose */
/* indices agree modulo P form one of P^3 colours, and same-colour cells are */
/* P - 1 cell edges (>= r_dep) apart, so trial sites chosen in them do not    */
/* interact.  P = 2 is the octant scheme of Fig. 5 (eight colours); P = 3 a  */
/* finer colouring (27 colours on cells of edge >= r_dep / 2).               */
/* ------------------------------------------------------------------------ */
int or_cell_grid_p(const double box[3], double r_dep, int period, int32_t nc[3]) {
  if (period < 2 || period > 3) return -1;
  const double edge = r_dep / (double)(period - 1);
  for (int d = 0; d < 3; ++d) {
    nc[d] = period * (int32_t)floor(box[d] / ((double)period * edge));
    if (nc[d] < period) return -1;
  }
  return 0;
}

int or_cell_grid(const double box[3], double r_dep, int32_t nc[3]) {
  return or_cell_grid_p(box, r_dep, 2, nc);
}

/* Colour of cell (cx, cy, cz): its indices modulo P, (cx % P) + P ((cy % P) + P (cz % P)). */
static int or_cell_colour(int64_t c, const int32_t nc[3], int period) {
  int cx = (int)(c % nc[0]), cy = (int)((c / nc[0]) % nc[1]), cz = (int)(c / ((int64_t)nc[0] * nc[1]));
  return (cx % period) + period * ((cy % period) + period * (cz % period));
}

/* Colour of a stage: floor(w0 C / 2^64) for C = P^3 colours (w0 >> 61 for eight). */
static int or_stage_colour(uint64_t w0, int ncol) {
  return (int)or_index(w0, (uint64_t)ncol);
}

static int or_over(const double *over, int64_t n_over, int64_t w, int64_t s, int64_t cell,
                   int *dec) {
  for (int64_t k = 0; k < n_over; ++k) {
    const double *o = over + 4 * k;
    if ((int64_t)o[0] == w && (int64_t)o[1] == s && (int64_t)o[2] == cell) {
      *dec = o[3] != 0.0;
      return 1;
    }
  }
  return 0;
}

/*
 * Parallel VC-SGC Monte Carlo sweeps (Sec. III.B.2).
 *
 * Ensemble: pi(sigma) ~ exp[-beta (U + phi n + (kappa/N) n^2)], kappa per site,
 * phi = dmu0 - 2 kappa cbar (Eq. pi_vcsgc with kappa_paper = kappa/N).
 *
 * A sweep has S = 8 ceil(N / N_cells) stages (one MC cycle = N trials, Sec. IV.B).
 * In each stage s of sweep w:
 *   1. colour k = top 3 bits of Philox(key, (w, s, 0, 0)).w0  (shared random
 *      choice of the independent domain set, Sec. III.A);
 *   2. every cell c of colour k with m_c > 0 sites, in ascending c, draws
 *      Philox(key, (w, s, c, 1)): site = its floor(w0 m_c / 2^64)-th atom in
 *      ascending index, u = unit(w1); the local test of Eq. trans_vcsgc_par1
 *      accepts iff ln u < -beta (dU_i + dmu0 dn_i), dn_i = 1 - 2 s_i;
 *   3. with dn_tot the sum over locally accepted moves, the composite move is
 *      accepted iff ln u_g < -beta (kappa/N) dn_tot (dn_tot + 2 (n - N cbar)),
 *      u_g = unit(Philox(key, (w, s, 0, 0)).w1) (Eq. trans_vcsgc_par2 with the
 *      sign of the (c - c0) term that makes the product of the two factors
 *      equal the full VC-SGC weight ratio);
 *   4. if accepted every locally accepted flip is committed (rho cache updated).
 * key = (seed, replica).
 */
static int or_da_local(const or_da *da, int64_t w, int64_t s, int64_t c, int64_t i,
                       const int64_t *start, const int32_t *nj, const double *nr,
                       const uint8_t *species, const double *rho, const or_pot *p,
                       double beta, double dmu0, const uint64_t t[4], double *du_out,
                       double *margin_out, int *pass1, int *status);

/* Undo log of the tentative flips of one stage (local chains of k > 1
 * steps): the values a flip overwrites, restored in reverse order when the
 * global factor rejects the stage. */
typedef struct {
  int64_t idx;
  int kind; /* 0: rho[idx], 1: species[idx], 2: velocity of idx */
  double v[3];
} or_undo;

typedef struct {
  or_undo *e;
  int64_t n, cap;
} or_undo_log;

static void undo_push(or_undo_log *u, int64_t idx, int kind, double a, double b, double c) {
  if (u->n == u->cap) {
    u->cap = u->cap ? 2 * u->cap : 1024;
    u->e = (or_undo *)realloc(u->e, (size_t)u->cap * sizeof(or_undo));
  }
  or_undo *x = &u->e[u->n++];
  x->idx = idx;
  x->kind = kind;
  x->v[0] = a;
  x->v[1] = b;
  x->v[2] = c;
}

/* Flip at i applied in place with its undo records (the same arithmetic as
 * or_commit). */
static void or_apply_logged(int64_t i, const int64_t *start, const int32_t *nj, const double *nr,
                            uint8_t *species, double *rho, const or_pot *p, double *vx,
                            double *vy, double *vz, double mass_a, double mass_b,
                            or_undo_log *u) {
  for (int64_t e = start[i]; e < start[i + 1]; ++e) {
    if (e > start[i] && nj[e] == nj[e - 1]) continue;
    if (!(nr[e] < p->rc)) {
      int any = 0;
      for (int64_t e2 = e; e2 < start[i + 1] && nj[e2] == nj[e]; ++e2) any |= nr[e2] < p->rc;
      if (!any) continue;
    }
    undo_push(u, nj[e], 0, rho[nj[e]], 0.0, 0.0);
  }
  int s0 = species[i];
  undo_push(u, i, 1, (double)s0, 0.0, 0.0);
  or_commit(i, start, nj, nr, species, rho, p);
  if (vx) {
    undo_push(u, i, 2, vx[i], vy[i], vz[i]);
    double m0 = s0 ? mass_b : mass_a, m1 = s0 ? mass_a : mass_b;
    double f = sqrt(m0 / m1);
    vx[i] = vx[i] * f;
    vy[i] = vy[i] * f;
    vz[i] = vz[i] * f;
  }
}

static void undo_all(or_undo_log *u, uint8_t *species, double *rho, double *vx, double *vy,
                     double *vz) {
  for (int64_t k = u->n - 1; k >= 0; --k) {
    const or_undo *x = &u->e[k];
    if (x->kind == 0) rho[x->idx] = x->v[0];
    else if (x->kind == 1) species[x->idx] = (uint8_t)x->v[0];
    else {
      vx[x->idx] = x->v[0];
      vy[x->idx] = x->v[1];
      vz[x->idx] = x->v[2];
    }
  }
  u->n = 0;
}

/* The local test of Eq. trans_vcsgc_par1 for site i of trial block t:
 * accept iff ln u < -beta (dU_i + dmu0 dn_i), u = unit(t[1]).  Returns the
 * decision; dU, dn and the margin ln u + beta (dU + dmu0 dn) go out. */
static int or_local_test(int64_t i, const uint64_t t[4], const int64_t *start,
                         const int32_t *nj, const double *nr, const uint8_t *species,
                         const double *rho, const or_pot *p, double beta, double dmu0,
                         double *du_out, int *dn_out, double *margin_out) {
  int dn = 1 - 2 * (int)species[i];
  double u = or_unit(t[1]);
  double du = or_delta_u(i, start, nj, nr, species, rho, p);
  double xl = beta * (du + dmu0 * (double)dn);
  double lnu = log(u);
  *du_out = du;
  *dn_out = dn;
  *margin_out = lnu + xl;
  return lnu < -xl;
}

/* ------------------------------------------------------------------------ */
/* Grown domains (Sec. III.A, Fig. 6): cells of edge e per axis (at least     */
/* 2 r_dep), each holding eight cubic domains of edge e - r_dep, one per     */
/* corner: domain k spans [0, e - r_dep) along axis d when bit d of k is 0   */
/* and [e - (e - r_dep), e) when it is 1, in coordinates u = x - b e from    */
/* the cell's corner (b the cell index along the axis).  Domains of one k in */
/* different cells are r_dep apart, so trials in them do not interact; the   */
/* domains of a cell overlap, and an atom in m of them gets weight 8 / m, so */
/* that the centre is not sampled more often than the rim.  Lists per (cell, */
/* k): the atoms of the domain in ascending index with the inclusive prefix  */
/* sums of their weights.                                                     */
/* ------------------------------------------------------------------------ */
static int or_grown_grid(const double box[3], double r_dep, double grow_edge, int32_t nc[3]) {
  double emin = grow_edge > 2.0 * r_dep ? grow_edge : 2.0 * r_dep;
  for (int d = 0; d < 3; ++d) {
    nc[d] = (int32_t)floor(box[d] / emin);
    if (nc[d] < 1) return -1;
  }
  return 0;
}

/* domain bits of atom i (bit 2d: in the low interval of axis d, bit 2d+1: in
 * the high one) and its weight 8 / m */
static int or_grown_bits(int64_t i, const double *x, const double *y, const double *z,
                         const double box[3], const int32_t nc[3], double r_dep, int *w) {
  const double *pos[3] = {x, y, z};
  int bits = 0, m = 1;
  for (int d = 0; d < 3; ++d) {
    double e = box[d] / (double)nc[d];
    double ld = e - r_dep;
    int b = (int)(pos[d][i] / (box[d] / (double)nc[d]));
    if (b < 0) b = 0;
    if (b >= nc[d]) b = nc[d] - 1;
    double u = pos[d][i] - (double)b * e;
    int lo = u < ld, hi = u >= e - ld;
    bits |= (lo << (2 * d)) | (hi << (2 * d + 1));
    m *= lo + hi;
  }
  *w = 8 / m;
  return bits;
}

static int or_in_domain(int bits, int k) {
  for (int d = 0; d < 3; ++d)
    if (!((bits >> (2 * d + ((k >> d) & 1))) & 1)) return 0;
  return 1;
}

/* per (cell c, domain k) at q = 8 c + k: dstart[q] .. dstart[q + 1] into
 * dlist (atom) and dcum (inclusive prefix sums of the weights) */
static void or_grown_lists(int64_t ncells, const int32_t *cstart, const int32_t *catoms,
                           const double *x, const double *y, const double *z, const double box[3],
                           const int32_t nc[3], double r_dep, int32_t *dstart, int32_t *dlist,
                           int32_t *dcum) {
  int32_t o = 0;
  for (int64_t c = 0; c < ncells; ++c) {
    for (int k = 0; k < 8; ++k) {
      dstart[8 * c + k] = o;
      int32_t cum = 0;
      for (int32_t q = cstart[c]; q < cstart[c + 1]; ++q) {
        int32_t i = catoms[q];
        int w;
        int bits = or_grown_bits(i, x, y, z, box, nc, r_dep, &w);
        if (!or_in_domain(bits, k)) continue;
        cum += w;
        dlist[o] = i;
        dcum[o] = cum;
        o++;
      }
    }
  }
  dstart[8 * ncells] = o;
}

/* Site of a trial in domain k of cell c: with W the domain's total weight,
 * r = floor(w0 W / 2^64) and the first atom whose prefix sum exceeds r;
 * -1 for an empty domain. */
static int64_t or_grown_site(const uint64_t t[4], const int32_t *dstart, const int32_t *dlist,
                             const int32_t *dcum, int64_t c, int k) {
  int32_t a = dstart[8 * c + k], b = dstart[8 * c + k + 1];
  if (a == b) return -1;
  uint64_t r = or_index(t[0], (uint64_t)dcum[b - 1]);
  for (int32_t q = a; q < b; ++q)
    if ((uint64_t)dcum[q] > r) return dlist[q];
  return -1;
}

/* Site of a trial: the floor(w0 m / 2^64)-th of the cell's m atoms. */
static int64_t or_site(const uint64_t t[4], const int32_t *cstart, const int32_t *catoms,
                       int64_t c) {
  int64_t m = cstart[c + 1] - cstart[c];
  return catoms[cstart[c] + (int64_t)or_index(t[0], (uint64_t)m)];
}

static int sweep_core(int64_t n, const double *x, const double *y, const double *z,
                      const double box[3], const int64_t *start, const int32_t *nj,
                      const double *nr, uint8_t *species, double *rho, int64_t *n_b,
                      const or_pot *p, const or_sweep_args *a, double *vx, double *vy,
                      double *vz, double *tlog, int64_t tcap, int64_t *tn, double *slog,
                      int64_t scap, int64_t *sn, const double *over, int64_t n_over,
                      or_stats *st, or_da *da) {
  const int64_t K = a->local_steps > 1 ? a->local_steps : 1;
  if (K > 1 && da && da->mode != OR_DA_OFF) return -3; /* delayed acceptance: one step only */
  if (n < 1 || !(a->temp > 0.0) || !(a->kappa >= 0.0)) return -1;
  const int grown = a->grow_edge > 0.0 && !a->one_cell;
  const int P = grown ? 2 : (a->colour_period > 0 ? a->colour_period : 2);
  const int NCOL = P * P * P;
  int32_t nc[3] = {1, 1, 1};
  int64_t ncells = 1;
  if (grown) {
    if (!(a->r_dep > 0.0) || or_grown_grid(box, a->r_dep, a->grow_edge, nc)) return -2;
    ncells = (int64_t)nc[0] * nc[1] * nc[2];
  } else if (!a->one_cell) {
    if (or_cell_grid_p(box, a->r_dep, P, nc)) return -2;
    ncells = (int64_t)nc[0] * nc[1] * nc[2];
  }
  /* counting sort of sites into cells; ascending index inside each cell */
  int32_t *cstart = (int32_t *)calloc((size_t)ncells + 1, sizeof(int32_t));
  int32_t *catoms = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *cof = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *ccol = (int32_t *)malloc((size_t)ncells * sizeof(int32_t));
  for (int64_t i = 0; i < n; ++i) {
    if (a->one_cell) {
      cof[i] = 0;
    } else {
      const double *u[3] = {x, y, z};
      int b[3];
      for (int d = 0; d < 3; ++d) {
        b[d] = (int)(u[d][i] / (box[d] / nc[d]));
        if (b[d] < 0) b[d] = 0;
        if (b[d] >= nc[d]) b[d] = nc[d] - 1;
      }
      cof[i] = b[0] + nc[0] * (b[1] + nc[1] * b[2]);
    }
    cstart[cof[i] + 1]++;
  }
  for (int64_t c = 0; c < ncells; ++c) cstart[c + 1] += cstart[c];
  {
    int32_t *fill = (int32_t *)malloc((size_t)ncells * sizeof(int32_t));
    memcpy(fill, cstart, (size_t)ncells * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) catoms[fill[cof[i]]++] = (int32_t)i;
    free(fill);
  }
  for (int64_t c = 0; c < ncells; ++c) ccol[c] = or_cell_colour(c, nc, P);
  int32_t *dstart = NULL, *dlist = NULL, *dcum = NULL;
  if (grown) {
    dstart = (int32_t *)malloc((size_t)(8 * ncells + 1) * sizeof(int32_t));
    dlist = (int32_t *)malloc((size_t)(8 * n) * sizeof(int32_t));
    dcum = (int32_t *)malloc((size_t)(8 * n) * sizeof(int32_t));
    or_grown_lists(ncells, cstart, catoms, x, y, z, box, nc, a->r_dep, dstart, dlist, dcum);
  }
  int64_t S = a->one_cell ? (n + K - 1) / K
              : grown     ? (((n + ncells - 1) / ncells) + K - 1) / K
                          : NCOL * ((((n + ncells - 1) / ncells) + K - 1) / K);

  double beta = 1.0 / (OR_KB * a->temp);
  double kN = a->kappa / (double)n;
  uint64_t key[2] = {a->seed, a->replica};
  int32_t *rec = (int32_t *)malloc((size_t)ncells * sizeof(int32_t));
  or_undo_log ulog = {NULL, 0, 0};
  memset(st, 0, sizeof(*st));
  int64_t ntl = 0, nsl = 0;

  for (int64_t w = a->w0; w < a->w0 + a->n_sweeps; ++w) {
    for (int64_t s = 0; s < S; ++s) {
      uint64_t ctr[4] = {(uint64_t)w, (uint64_t)s, 0, 0}, g[4];
      or_philox4x64_10(key, ctr, g);
      int colour = or_stage_colour(g[0], NCOL);
      int64_t nrec = 0, dn_tot = 0;
      if (K > 1) {
        /* local chains: every step on the state left by the previous one;
         * accepted flips are applied at once and logged for undoing */
        for (int64_t c = 0; c < ncells; ++c) {
          if (!a->one_cell && !grown && ccol[c] != colour) continue;
          int64_t m = grown ? dstart[8 * c + colour + 1] - dstart[8 * c + colour]
                            : cstart[c + 1] - cstart[c];
          if (m == 0) continue;
          for (int64_t q = 0; q < K; ++q) {
            uint64_t tc[4] = {(uint64_t)w, (uint64_t)s, (uint64_t)c, (uint64_t)(1 + q)}, t[4];
            or_philox4x64_10(key, tc, t);
            int64_t i = grown ? or_grown_site(t, dstart, dlist, dcum, c, colour)
                              : or_site(t, cstart, catoms, c);
            int dn;
            double du, margin;
            int acc = or_local_test(i, t, start, nj, nr, species, rho, p, beta, a->dmu0, &du, &dn,
                                    &margin);
            if (fabs(margin) < OR_TIE) {
              st->near_ties++;
              int dec;
              if (over && or_over(over, n_over, w, s, c * K + q, &dec)) acc = dec;
            }
            st->trials++;
            if (acc) {
              st->local_accepts++;
              nrec++;
              dn_tot += dn;
              or_apply_logged(i, start, nj, nr, species, rho, p, vx, vy, vz, a->mass_a,
                              a->mass_b, &ulog);
            }
            if (tlog && ntl < tcap) {
              double *L = tlog + 8 * ntl;
              L[0] = (double)w; L[1] = (double)s; L[2] = (double)(c * K + q); L[3] = (double)i;
              L[4] = (double)dn; L[5] = (double)acc; L[6] = du; L[7] = margin;
            }
            ntl++;
          }
        }
      }
      for (int64_t c = 0; c < ncells && K == 1; ++c) {
        if (!a->one_cell && !grown && ccol[c] != colour) continue;
        int64_t m = grown ? dstart[8 * c + colour + 1] - dstart[8 * c + colour]
                          : cstart[c + 1] - cstart[c];
        if (m == 0) continue;
        uint64_t tc[4] = {(uint64_t)w, (uint64_t)s, (uint64_t)c, 1}, t[4];
        or_philox4x64_10(key, tc, t);
        int64_t i = grown ? or_grown_site(t, dstart, dlist, dcum, c, colour)
                          : or_site(t, cstart, catoms, c);
        int dn = 1 - 2 * (int)species[i];
        double du, margin;
        int acc;
        if (da && da->mode != OR_DA_OFF) {
          int pass1 = 0, status = 0;
          acc = or_da_local(da, w, s, c, i, start, nj, nr, species, rho, p, beta, a->dmu0, t,
                            &du, &margin, &pass1, &status);
          if (status) {
            free(rec); free(cstart); free(catoms); free(cof); free(ccol);
            free(dstart); free(dlist); free(dcum);
            return status;
          }
          if (pass1) da->stage1_pass++;
          if (fabs(margin) < OR_TIE) st->near_ties++;
        } else {
          acc = or_local_test(i, t, start, nj, nr, species, rho, p, beta, a->dmu0, &du, &dn,
                              &margin);
          if (fabs(margin) < OR_TIE) {
            st->near_ties++;
            int dec;
            if (over && or_over(over, n_over, w, s, c, &dec)) acc = dec;
          }
        }
        st->trials++;
        if (acc) {
          st->local_accepts++;
          rec[nrec++] = (int32_t)i;
          dn_tot += dn;
        }
        if (tlog && ntl < tcap) {
          double *L = tlog + 8 * ntl;
          L[0] = (double)w; L[1] = (double)s; L[2] = (double)c; L[3] = (double)i;
          L[4] = (double)dn; L[5] = (double)acc; L[6] = du; L[7] = margin;
        }
        ntl++;
      }
      st->stages++;
      int gacc = -1;
      double xg = 0.0, mg = 0.0;
      if (nrec > 0) {
        double tt = (double)*n_b - (double)n * a->cbar;
        double dnd = (double)dn_tot;
        xg = beta * kN * dnd * (dnd + 2.0 * tt);
        double lnug = log(or_unit(g[1]));
        mg = lnug + xg;
        gacc = lnug < -xg;
        if (fabs(mg) < OR_TIE) {
          st->near_ties++;
          int dec;
          if (over && or_over(over, n_over, w, s, -1, &dec)) gacc = dec;
        }
        if (K > 1) {
          if (gacc) ulog.n = 0; /* the tentative flips stay */
          else undo_all(&ulog, species, rho, vx, vy, vz);
          if (gacc) {
            *n_b += dn_tot;
            st->flips += nrec;
            st->stage_accepts++;
          }
        } else if (gacc) {
          for (int64_t k = 0; k < nrec; ++k) {
            int64_t i = rec[k];
            int s0 = species[i];
            or_commit(i, start, nj, nr, species, rho, p);
            if (vx) {
              double m0 = s0 ? a->mass_b : a->mass_a, m1 = s0 ? a->mass_a : a->mass_b;
              double f = sqrt(m0 / m1);
              vx[i] = vx[i] * f;
              vy[i] = vy[i] * f;
              vz[i] = vz[i] * f;
            }
          }
          *n_b += dn_tot;
          st->flips += nrec;
          st->stage_accepts++;
        }
      }
      if (slog && nsl < scap) {
        double *L = slog + 8 * nsl;
        L[0] = (double)w; L[1] = (double)s; L[2] = (double)colour; L[3] = (double)dn_tot;
        L[4] = (double)nrec; L[5] = (double)gacc; L[6] = xg; L[7] = mg;
      }
      nsl++;
    }
    st->sum_n += (double)*n_b;
    st->sum_n2 += (double)*n_b * (double)*n_b;
  }
  st->n_final = *n_b;
  if (tn) *tn = ntl;
  if (sn) *sn = nsl;
  free(ulog.e);
  free(rec);
  free(cstart);
  free(catoms);
  free(cof);
  free(ccol);
  free(dstart);
  free(dlist);
  free(dcum);
  return 0;
}

int or_sweep(int64_t n, const double *x, const double *y, const double *z, const double box[3],
             const int64_t *start, const int32_t *nj, const double *nr,
             uint8_t *species, double *rho, int64_t *n_b, const or_pot *p,
             const or_sweep_args *a, double *vx, double *vy, double *vz,
             double *tlog, int64_t tcap, int64_t *tn,
             double *slog, int64_t scap, int64_t *sn,
             const double *over, int64_t n_over, or_stats *st) {
  return sweep_core(n, x, y, z, box, start, nj, nr, species, rho, n_b, p, a, vx, vy, vz, tlog,
                    tcap, tn, slog, scap, sn, over, n_over, st, NULL);
}

int or_sweep_da(int64_t n, const double *x, const double *y, const double *z, const double box[3],
                const int64_t *start, const int32_t *nj, const double *nr,
                uint8_t *species, double *rho, int64_t *n_b, const or_pot *p,
                const or_sweep_args *a, or_da *da,
                double *tlog, int64_t tcap, int64_t *tn,
                double *slog, int64_t scap, int64_t *sn, or_stats *st) {
  if (!da) return -1;
  da->stage1_pass = 0;
  return sweep_core(n, x, y, z, box, start, nj, nr, species, rho, n_b, p, a, NULL, NULL, NULL,
                    tlog, tcap, tn, slog, scap, sn, NULL, 0, st, da);
}

/* ------------------------------------------------------------------------ */
/* Surrogate: descriptor, bfloat16 rounding, MLP, delayed acceptance         */
/* ------------------------------------------------------------------------ */
static int or_shell(double r) {
  if (r < 2.68) return 0;
  if (r < 3.46) return 1;
  if (r < 4.41) return 2;
  return -1;
}

void or_descriptor(int64_t i, const int64_t *start, const int32_t *nj, const double *nr,
                   const uint8_t *species, const double *rho, const or_pot *p, int flip,
                   double out[10]) {
  int s = species[i], s1 = 1 - s;
  double cnt[3] = {0.0, 0.0, 0.0}, cb[3] = {0.0, 0.0, 0.0}, rs[3] = {0.0, 0.0, 0.0};
  for (int64_t e = start[i]; e < start[i + 1]; ++e) {
    int k = or_shell(nr[e]);
    if (k < 0) continue;
    int32_t j = nj[e];
    double rj = rho[j];
    if (flip) {
      /* the density of j in the flipped state: the commit's aggregated shift */
      int64_t e0 = e;
      while (e0 > start[i] && nj[e0 - 1] == j) --e0;
      double delta = 0.0;
      int any = 0;
      for (int64_t e2 = e0; e2 < start[i + 1] && nj[e2] == j; ++e2) {
        if (!(nr[e2] < p->rc)) continue;
        delta += or_f(p, s1, nr[e2]) - or_f(p, s, nr[e2]);
        any = 1;
      }
      if (any) rj = rj + delta;
    }
    cnt[k] += 1.0;
    cb[k] += (double)species[j];
    rs[k] += rj;
  }
  out[0] = (double)(flip ? s1 : s);
  for (int k = 0; k < 3; ++k) {
    out[1 + k] = cb[k];
    out[4 + k] = cnt[k];
    out[7 + k] = cnt[k] > 0.0 ? rs[k] / cnt[k] : 0.0;
  }
}

float or_bf16(float v) {
  uint32_t b;
  memcpy(&b, &v, sizeof(b));
  b = b + 0x7FFFu + ((b >> 16) & 1u);
  b &= 0xFFFF0000u;
  float r;
  memcpy(&r, &b, sizeof(r));
  return r;
}

static double or_sig(double a) { return 1.0 / (1.0 + exp(-a)); }

/* one sample: activations kept for the gradient */
typedef struct {
  double z[10], a1[64], h1[64], a2[64], h2[64], y;
} or_act;

static double or_w(float w, int bf16) { return bf16 ? (double)or_bf16(w) : (double)w; }

static void or_mlp_one(const or_mlp *m, const double *d, int bf16, or_act *A) {
  for (int k = 0; k < 10; ++k) {
    float zk = (float)((d[k] - (double)m->mu[k]) / (double)m->sd[k]);
    A->z[k] = bf16 ? (double)or_bf16(zk) : (double)zk;
  }
  for (int j = 0; j < 64; ++j) {
    double acc = (double)m->b1[j];
    for (int k = 0; k < 10; ++k) acc += or_w(m->w1[j * 10 + k], bf16) * A->z[k];
    A->a1[j] = acc;
    double h = acc * or_sig(acc);
    A->h1[j] = bf16 ? (double)or_bf16((float)h) : h;
  }
  for (int j = 0; j < 64; ++j) {
    double acc = (double)m->b2[j];
    for (int k = 0; k < 64; ++k) acc += or_w(m->w2[j * 64 + k], bf16) * A->h1[k];
    A->a2[j] = acc;
    double h = acc * or_sig(acc);
    A->h2[j] = bf16 ? (double)or_bf16((float)h) : h;
  }
  double y = (double)m->b3[0];
  for (int k = 0; k < 64; ++k) y += or_w(m->w3[k], bf16) * A->h2[k];
  A->y = y;
}

void or_mlp_forward(const or_mlp *m, int64_t n, const double *d, int bf16, double *y, double *dE) {
  or_act A;
  for (int64_t b = 0; b < n; ++b) {
    or_mlp_one(m, d + 10 * b, bf16, &A);
    if (y) y[b] = A.y;
    if (dE) dE[b] = A.y * (double)m->out_sd + (double)m->out_mu;
  }
}

/* d SiLU / da = s (1 + a (1 - s)), s = sigmoid(a) */
static double or_dsilu(double a) {
  double sg = or_sig(a);
  return sg * (1.0 + a * (1.0 - sg));
}

static double or_bfd(double v, int bf16) { return bf16 ? (double)or_bf16((float)v) : v; }

double or_mlp_grad(const or_mlp *m, int64_t n, const double *d, const double *t, int bf16,
                   double *grad) {
  double *gw1 = grad, *gb1 = grad + 640, *gw2 = grad + 704, *gb2 = grad + 4800,
         *gw3 = grad + 4864, *gb3 = grad + 4928;
  memset(grad, 0, 4929 * sizeof(double));
  double loss = 0.0;
  or_act A;
  for (int64_t b = 0; b < n; ++b) {
    or_mlp_one(m, d + 10 * b, bf16, &A);
    double tn = (t[b] - (double)m->out_mu) / (double)m->out_sd;
    double r = A.y - tn;
    loss += r * r;
    double dy = 2.0 * r / (double)n;
    gb3[0] += dy;
    double da2[64], da1[64];
    for (int k = 0; k < 64; ++k) {
      gw3[k] += dy * A.h2[k];
      double dh2 = dy * or_w(m->w3[k], bf16);
      da2[k] = dh2 * or_dsilu(A.a2[k]);
    }
    for (int j = 0; j < 64; ++j) {
      gb2[j] += da2[j];
      double dq = or_bfd(da2[j], bf16);
      for (int k = 0; k < 64; ++k) gw2[j * 64 + k] += dq * A.h1[k];
    }
    for (int k = 0; k < 64; ++k) {
      double acc = 0.0;
      for (int j = 0; j < 64; ++j) acc += or_bfd(da2[j], bf16) * or_w(m->w2[j * 64 + k], bf16);
      da1[k] = acc * or_dsilu(A.a1[k]);
    }
    for (int j = 0; j < 64; ++j) {
      gb1[j] += da1[j];
      double dq = or_bfd(da1[j], bf16);
      for (int k = 0; k < 10; ++k) gw1[j * 10 + k] += dq * A.z[k];
    }
  }
  return loss / (double)n;
}

static int or_table_find(const or_da *da, int64_t w, int64_t s, int64_t c, double *f, double *r) {
  int64_t lo = 0, hi = da->n_table - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    const double *row = da->table + 5 * mid;
    int64_t rw = (int64_t)row[0], rs = (int64_t)row[1], rc = (int64_t)row[2];
    int cmp = rw != w ? (rw < w ? -1 : 1) : (rs != s ? (rs < s ? -1 : 1) : (rc != c ? (rc < c ? -1 : 1) : 0));
    if (cmp == 0) {
      *f = row[3];
      *r = row[4];
      return 1;
    }
    if (cmp < 0) lo = mid + 1; else hi = mid - 1;
  }
  return 0;
}

/* Delayed-acceptance local test (stage 1 with the surrogate, stage 2 exact). */
static int or_da_local(const or_da *da, int64_t w, int64_t s, int64_t c, int64_t i,
                       const int64_t *start, const int32_t *nj, const double *nr,
                       const uint8_t *species, const double *rho, const or_pot *p,
                       double beta, double dmu0, const uint64_t t[4], double *du_out,
                       double *margin_out, int *pass1, int *status) {
  int dn = 1 - 2 * (int)species[i];
  double ef = 0.0, er = 0.0, du = NAN;
  int have_du = 0;
  *status = 0;
  if (da->mode == OR_DA_TABLE) {
    if (!or_table_find(da, w, s, c, &ef, &er)) {
      *status = -3;
      return 0;
    }
    if (da->dlog && da->dstart) {
      /* the descriptors the surrogate values were computed from, at this
       * trial's state, for checking those values against or_mlp_forward */
      or_da *dm = (or_da *)da;
      if (dm->dn < dm->dcap) {
        double *L = dm->dlog + 23 * dm->dn;
        L[0] = (double)w; L[1] = (double)s; L[2] = (double)c;
        or_descriptor(i, da->dstart, da->dnj, da->dnr, species, rho, p, 0, L + 3);
        or_descriptor(i, da->dstart, da->dnj, da->dnr, species, rho, p, 1, L + 13);
      }
      dm->dn++;
    }
  } else if (da->mode == OR_DA_PERFECT) {
    du = or_delta_u(i, start, nj, nr, species, rho, p);
    have_du = 1;
    ef = du;
    er = -du;
  } else if (da->mode == OR_DA_MLP) {
    double dx[10], dy[10];
    or_descriptor(i, da->dstart, da->dnj, da->dnr, species, rho, p, 0, dx);
    or_descriptor(i, da->dstart, da->dnj, da->dnr, species, rho, p, 1, dy);
    or_mlp_forward(da->mlp, 1, dx, 1, NULL, &ef);
    or_mlp_forward(da->mlp, 1, dy, 1, NULL, &er);
  }
  /* stage 1: min{1, exp(-beta s_f)}, s_f = dE_f + dmu0 dn */
  double sf = ef + dmu0 * (double)dn;
  double x1 = beta * sf;
  double lnu1 = log(or_unit(t[1]));
  *pass1 = lnu1 < -x1;
  if (!*pass1) {
    *du_out = NAN;
    *margin_out = lnu1 + x1;
    return 0;
  }
  /* stage 2: exp(-beta (dU + dmu0 dn)) min{1, exp(-beta s_r)} / min{1, exp(-beta s_f)} */
  if (!have_du) du = or_delta_u(i, start, nj, nr, species, rho, p);
  double sr = er - dmu0 * (double)dn;
  double xl = beta * (du + dmu0 * (double)dn);
  double xr = -(beta * sr);
  double l2 = (-xl + (xr < 0.0 ? xr : 0.0)) - (-x1 < 0.0 ? -x1 : 0.0);
  double lnu2 = log(or_unit(t[2]));
  *du_out = du;
  *margin_out = lnu2 - l2;
  return lnu2 < l2;
}

/* ------------------------------------------------------------------------ */
/* Velocity Verlet MD with EAM forces (Sec. IV.A hybrid scheme, NVE)         */
/* ------------------------------------------------------------------------ */
static double or_wrap(double u, double L) {
  if (u < 0.0) u += L;
  if (u >= L) u -= L;
  return u;
}

static int or_eval_forces(int64_t n, const double *x, const double *y, const double *z,
                          const uint8_t *species, const double box[3], const or_pot *p,
                          double *fx, double *fy, double *fz, double *rho) {
  int64_t cap = 32 * n + 64;
  for (;;) {
    int64_t *start = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *nj = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    double *nr = (double *)malloc((size_t)cap * sizeof(double));
    double *dx = (double *)malloc((size_t)cap * sizeof(double));
    double *dy = (double *)malloc((size_t)cap * sizeof(double));
    double *dz = (double *)malloc((size_t)cap * sizeof(double));
    int64_t tot = or_neighbors(n, x, y, z, box, p->rc, 0, cap, start, nj, nr, dx, dy, dz);
    if (tot < 0) {
      free(start); free(nj); free(nr); free(dx); free(dy); free(dz);
      return -1;
    }
    if (tot <= cap) {
      or_density(n, start, nj, nr, species, p, rho);
      or_forces(n, start, nj, nr, dx, dy, dz, species, p, rho, fx, fy, fz);
      free(start); free(nj); free(nr); free(dx); free(dy); free(dz);
      return 0;
    }
    free(start); free(nj); free(nr); free(dx); free(dy); free(dz);
    cap = tot;
  }
}

/*
 * Per step, per atom, with a = F (ACC / m):
 *   v = v + (dt/2) a;  x = wrap(x + dt v);  forces at the new positions;  v = v + (dt/2) a.
 */
int or_md(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
          const uint8_t *species, const double box[3], const or_pot *p,
          double mass_a, double mass_b, double dt, int64_t n_steps,
          double *fx, double *fy, double *fz, double *rho) {
  double cm[2] = {OR_ACC / mass_a, OR_ACC / mass_b};
  double hdt = 0.5 * dt;
  if (or_eval_forces(n, x, y, z, species, box, p, fx, fy, fz, rho)) return -1;
  for (int64_t step = 0; step < n_steps; ++step) {
    for (int64_t i = 0; i < n; ++i) {
      double c = cm[species[i]];
      vx[i] = vx[i] + hdt * (fx[i] * c);
      vy[i] = vy[i] + hdt * (fy[i] * c);
      vz[i] = vz[i] + hdt * (fz[i] * c);
      x[i] = or_wrap(x[i] + dt * vx[i], box[0]);
      y[i] = or_wrap(y[i] + dt * vy[i], box[1]);
      z[i] = or_wrap(z[i] + dt * vz[i], box[2]);
    }
    if (or_eval_forces(n, x, y, z, species, box, p, fx, fy, fz, rho)) return -1;
    for (int64_t i = 0; i < n; ++i) {
      double c = cm[species[i]];
      vx[i] = vx[i] + hdt * (fx[i] * c);
      vy[i] = vy[i] + hdt * (fy[i] * c);
      vz[i] = vz[i] + hdt * (fz[i] * c);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* All-core CPU baseline of the plain sweep (one trial per active cell per   */
/* stage, no surrogate).  Same chain as or_sweep: the trials of a stage's    */
/* active cells read only state that no other trial of the stage writes     */
/* (same-colour cells are at least r_dep >= 2 rc apart, Sec. III.A), so they */
/* are evaluated by several threads; the integer sum dn_tot, the counters    */
/* and the record list are then taken serially in ascending cell order, the  */
/* global test is the serial one, and the commits touch disjoint             */
/* neighbourhoods.  Every value is therefore bitwise that of or_sweep.       */
/* ------------------------------------------------------------------------ */
#include <omp.h>

int or_sweep_omp(int64_t n, const double *x, const double *y, const double *z,
                 const double box[3], const int64_t *start, const int32_t *nj,
                 const double *nr, uint8_t *species, double *rho, int64_t *n_b,
                 const or_pot *p, const or_sweep_args *a, double *vx, double *vy, double *vz,
                 double *slog, int64_t scap, int64_t *sn, int n_threads, or_stats *st) {
  if (a->local_steps > 1 || a->one_cell || a->grow_edge > 0.0) return -3;
  if (n < 1 || !(a->temp > 0.0) || !(a->kappa >= 0.0)) return -1;
  const int P = a->colour_period > 0 ? a->colour_period : 2;
  const int NCOL = P * P * P;
  int32_t nc[3];
  if (or_cell_grid_p(box, a->r_dep, P, nc)) return -2;
  int64_t ncells = (int64_t)nc[0] * nc[1] * nc[2];
  int32_t *cstart = (int32_t *)calloc((size_t)ncells + 1, sizeof(int32_t));
  int32_t *catoms = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *cof = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  for (int64_t i = 0; i < n; ++i) {
    const double *u[3] = {x, y, z};
    int b[3];
    for (int d = 0; d < 3; ++d) {
      b[d] = (int)(u[d][i] / (box[d] / nc[d]));
      if (b[d] < 0) b[d] = 0;
      if (b[d] >= nc[d]) b[d] = nc[d] - 1;
    }
    cof[i] = b[0] + nc[0] * (b[1] + nc[1] * b[2]);
    cstart[cof[i] + 1]++;
  }
  for (int64_t c = 0; c < ncells; ++c) cstart[c + 1] += cstart[c];
  {
    int32_t *fill = (int32_t *)malloc((size_t)ncells * sizeof(int32_t));
    memcpy(fill, cstart, (size_t)ncells * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) catoms[fill[cof[i]]++] = (int32_t)i;
    free(fill);
  }
  /* the cells of each colour in ascending id */
  int64_t *col_cells = (int64_t *)malloc((size_t)ncells * sizeof(int64_t));
  int64_t col_start[28] = {0};
  for (int64_t c = 0; c < ncells; ++c) col_start[1 + or_cell_colour(c, nc, P)]++;
  for (int k = 0; k < NCOL; ++k) col_start[k + 1] += col_start[k];
  {
    int64_t fill[27];
    memcpy(fill, col_start, sizeof(fill));
    for (int64_t c = 0; c < ncells; ++c) col_cells[fill[or_cell_colour(c, nc, P)]++] = c;
  }
  int64_t S = NCOL * ((n + ncells - 1) / ncells);
  double beta = 1.0 / (OR_KB * a->temp);
  double kN = a->kappa / (double)n;
  uint64_t key[2] = {a->seed, a->replica};
  int64_t maxc = 0;
  for (int k = 0; k < NCOL; ++k)
    if (col_start[k + 1] - col_start[k] > maxc) maxc = col_start[k + 1] - col_start[k];
  int64_t *t_site = (int64_t *)malloc((size_t)(maxc > 0 ? maxc : 1) * sizeof(int64_t));
  int8_t *t_state = (int8_t *)malloc((size_t)(maxc > 0 ? maxc : 1)); /* -1 empty, 0 reject, 1 accept */
  int8_t *t_tie = (int8_t *)malloc((size_t)(maxc > 0 ? maxc : 1));
  int32_t *rec = (int32_t *)malloc((size_t)(maxc > 0 ? maxc : 1) * sizeof(int32_t));
  memset(st, 0, sizeof(*st));
  int64_t nsl = 0;
  if (n_threads < 1) n_threads = 1;

  for (int64_t w = a->w0; w < a->w0 + a->n_sweeps; ++w) {
    for (int64_t s = 0; s < S; ++s) {
      uint64_t ctr[4] = {(uint64_t)w, (uint64_t)s, 0, 0}, g[4];
      or_philox4x64_10(key, ctr, g);
      int colour = or_stage_colour(g[0], NCOL);
      const int64_t *cells = col_cells + col_start[colour];
      int64_t m_act = col_start[colour + 1] - col_start[colour];
#pragma omp parallel for schedule(static) num_threads(n_threads)
      for (int64_t q = 0; q < m_act; ++q) {
        int64_t c = cells[q];
        if (cstart[c + 1] == cstart[c]) {
          t_state[q] = -1;
          continue;
        }
        uint64_t tc[4] = {(uint64_t)w, (uint64_t)s, (uint64_t)c, 1}, t[4];
        or_philox4x64_10(key, tc, t);
        int64_t i = or_site(t, cstart, catoms, c);
        int dn;
        double du, margin;
        int acc = or_local_test(i, t, start, nj, nr, species, rho, p, beta, a->dmu0, &du, &dn,
                                &margin);
        t_site[q] = i;
        t_state[q] = (int8_t)acc;
        t_tie[q] = (int8_t)(fabs(margin) < OR_TIE);
      }
      int64_t nrec = 0, dn_tot = 0;
      for (int64_t q = 0; q < m_act; ++q) {
        if (t_state[q] < 0) continue;
        st->trials++;
        st->near_ties += t_tie[q];
        if (t_state[q]) {
          st->local_accepts++;
          rec[nrec++] = (int32_t)t_site[q];
          dn_tot += 1 - 2 * (int)species[t_site[q]];
        }
      }
      st->stages++;
      int gacc = -1;
      double xg = 0.0, mg = 0.0;
      if (nrec > 0) {
        double tt = (double)*n_b - (double)n * a->cbar;
        double dnd = (double)dn_tot;
        xg = beta * kN * dnd * (dnd + 2.0 * tt);
        double lnug = log(or_unit(g[1]));
        mg = lnug + xg;
        gacc = lnug < -xg;
        if (fabs(mg) < OR_TIE) st->near_ties++;
        if (gacc) {
#pragma omp parallel for schedule(static) num_threads(n_threads)
          for (int64_t k = 0; k < nrec; ++k) {
            int64_t i = rec[k];
            int s0 = species[i];
            or_commit(i, start, nj, nr, species, rho, p);
            if (vx) {
              double m0 = s0 ? a->mass_b : a->mass_a, m1 = s0 ? a->mass_a : a->mass_b;
              double f = sqrt(m0 / m1);
              vx[i] = vx[i] * f;
              vy[i] = vy[i] * f;
              vz[i] = vz[i] * f;
            }
          }
          *n_b += dn_tot;
          st->flips += nrec;
          st->stage_accepts++;
        }
      }
      if (slog && nsl < scap) {
        double *L = slog + 8 * nsl;
        L[0] = (double)w; L[1] = (double)s; L[2] = (double)colour; L[3] = (double)dn_tot;
        L[4] = (double)nrec; L[5] = (double)gacc; L[6] = xg; L[7] = mg;
      }
      nsl++;
    }
    st->sum_n += (double)*n_b;
    st->sum_n2 += (double)*n_b * (double)*n_b;
  }
  st->n_final = *n_b;
  if (sn) *sn = nsl;
  free(t_site); free(t_state); free(t_tie); free(rec);
  free(col_cells); free(cstart); free(catoms); free(cof);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Nose-Hoover thermostat (NVT) for the MD part of the hybrid scheme         */
/* ------------------------------------------------------------------------ */
/* Fixed-shape sum of v[0..n): the values are cut into chunks of 256
 * consecutive entries (zeros past n); a chunk's sum is taken by halving
 * strides (a[t] += a[t + h] for h = 128, 64, ..., 1); chunk sum c is added,
 * in ascending c, to accumulator c mod 256 (each starting at 0); the 256
 * accumulators are combined by halving strides again. */
double or_tree_sum(int64_t n, const double *v) {
  int64_t nch = (n + 255) / 256;
  double acc[256];
  for (int t = 0; t < 256; ++t) acc[t] = 0.0;
  for (int64_t c = 0; c < nch; ++c) {
    double a[256];
    for (int t = 0; t < 256; ++t) {
      int64_t i = 256 * c + t;
      a[t] = i < n ? v[i] : 0.0;
    }
    for (int h = 128; h > 0; h >>= 1)
      for (int t = 0; t < h; ++t) a[t] = a[t] + a[t + h];
    acc[c % 256] = acc[c % 256] + a[0];
  }
  for (int h = 128; h > 0; h >>= 1)
    for (int t = 0; t < h; ++t) acc[t] = acc[t] + acc[t + h];
  return acc[0];
}

/* Kinetic energy (eV): K = 1/2 sum_i m_i |v_i|^2 / ACC, with the per-atom
 * terms m_i ((vx^2 + vy^2) + vz^2) summed by or_tree_sum. */
static double or_kinetic(int64_t n, const double *vx, const double *vy, const double *vz,
                         const uint8_t *species, double mass_a, double mass_b, double *work) {
  for (int64_t i = 0; i < n; ++i) {
    double m = species[i] ? mass_b : mass_a;
    work[i] = m * ((vx[i] * vx[i] + vy[i] * vy[i]) + vz[i] * vz[i]);
  }
  return 0.5 * or_tree_sum(n, work) / OR_ACC;
}

/* Half step (dt/2) of the thermostat variables for kinetic energy *K, with
 * G = (2K - g kB T) / Q:
 *   xi += (dt/4) G;  s = (1 - xi dt/4) / (1 + xi dt/4);  K <- K s s;
 *   eta += xi dt/2;  xi += (dt/4) G(K);
 * s is the (1,1) Pade form of exp(-xi dt/2), the factor the friction
 * -xi v applies to the velocities over dt/2; s(-xi) = 1/s(xi), so the
 * splitting stays time reversible.  Returns s. */
static double or_nh_half(double dt, double g, double kT, double Q, double *K, double *xi,
                         double *eta) {
  double q4 = 0.25 * dt;
  *xi = *xi + q4 * ((2.0 * *K - g * kT) / Q);
  double a = *xi * q4;
  double s = (1.0 - a) / (1.0 + a);
  *K = *K * s * s;
  *eta = *eta + *xi * (0.5 * dt);
  *xi = *xi + q4 * ((2.0 * *K - g * kT) / Q);
  return s;
}

/*
 * Nose-Hoover NVT (one thermostat; equations of motion dx/dt = v,
 * dv/dt = F/m - xi v, dxi/dt = (2K - g kB T)/Q, deta/dt = xi, with
 * g = 3N - 3 and Q = g kB T tau^2), integrated by the symmetric splitting
 *   thermostat(dt/2); v += (dt/2) a; x = wrap(x + dt v); forces;
 *   v += (dt/2) a; thermostat(dt/2),
 * with K computed fresh (or_kinetic) at the start of each thermostat half
 * step that follows a kick or starts the call, and carried by K <- K s s
 * otherwise.  The velocity factors of consecutive half steps are applied one
 * after the other, v = (v s1) s2.  xi (1/fs) and eta (fs^-1 * fs) carry over
 * between calls through xi_io and eta_io.  Conserved:
 *   H = K + U + Q xi^2 / 2 + g kB T eta.
 */
int or_md_nvt(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
              const uint8_t *species, const double box[3], const or_pot *p, double mass_a,
              double mass_b, double dt, int64_t n_steps, double temp, double tau, double *xi_io,
              double *eta_io, double *fx, double *fy, double *fz, double *rho) {
  double cm[2] = {OR_ACC / mass_a, OR_ACC / mass_b};
  double hdt = 0.5 * dt;
  double g = 3.0 * (double)n - 3.0;
  double kT = OR_KB * temp;
  double Q = g * kT * tau * tau;
  double xi = *xi_io, eta = *eta_io;
  double *work = (double *)malloc((size_t)n * sizeof(double));
  if (!work) return -1;
  if (or_eval_forces(n, x, y, z, species, box, p, fx, fy, fz, rho)) {
    free(work);
    return -1;
  }
  double K = or_kinetic(n, vx, vy, vz, species, mass_a, mass_b, work);
  double s_pend = 1.0; /* factor of the end-of-step half step, not yet applied */
  int have_pend = 0;
  for (int64_t step = 0; step < n_steps; ++step) {
    double s = or_nh_half(dt, g, kT, Q, &K, &xi, &eta);
    for (int64_t i = 0; i < n; ++i) {
      double c = cm[species[i]];
      if (have_pend) {
        vx[i] = vx[i] * s_pend;
        vy[i] = vy[i] * s_pend;
        vz[i] = vz[i] * s_pend;
      }
      vx[i] = vx[i] * s;
      vy[i] = vy[i] * s;
      vz[i] = vz[i] * s;
      vx[i] = vx[i] + hdt * (fx[i] * c);
      vy[i] = vy[i] + hdt * (fy[i] * c);
      vz[i] = vz[i] + hdt * (fz[i] * c);
      x[i] = or_wrap(x[i] + dt * vx[i], box[0]);
      y[i] = or_wrap(y[i] + dt * vy[i], box[1]);
      z[i] = or_wrap(z[i] + dt * vz[i], box[2]);
    }
    if (or_eval_forces(n, x, y, z, species, box, p, fx, fy, fz, rho)) {
      free(work);
      return -1;
    }
    for (int64_t i = 0; i < n; ++i) {
      double c = cm[species[i]];
      vx[i] = vx[i] + hdt * (fx[i] * c);
      vy[i] = vy[i] + hdt * (fy[i] * c);
      vz[i] = vz[i] + hdt * (fz[i] * c);
    }
    K = or_kinetic(n, vx, vy, vz, species, mass_a, mass_b, work);
    s_pend = or_nh_half(dt, g, kT, Q, &K, &xi, &eta);
    have_pend = 1;
  }
  if (have_pend) {
    for (int64_t i = 0; i < n; ++i) {
      vx[i] = vx[i] * s_pend;
      vy[i] = vy[i] * s_pend;
      vz[i] = vz[i] * s_pend;
    }
  }
  *xi_io = xi;
  *eta_io = eta;
  free(work);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Isotropic NPT: the Nose-Hoover thermostat and barostat of the paper's     */
/* Fe-Cu runs (Sec. IV.B), in the form of Martyna, Tobias and Klein,        */
/* J. Chem. Phys. 101, 4177 (1994), with one thermostat acting on the        */
/* particles and on the barostat:                                             */
/*   dx/dt = v + ve x,  dv/dt = F/m - (1 + 3/g) ve v - xi v,  dL/dt = ve L    */
/*   dpe/dt = 3V (P - P_ext) + (3/g) 2K - xi pe,   ve = pe / W                */
/*   dxi/dt = (2K + pe^2/W - (g + 1) kB T) / Q,    deta/dt = xi               */
/* with g = 3N - 3, Q = (g + 1) kB T tau_T^2, W = (g + 1) kB T tau_P^2, the   */
/* pressure P = (2K + Vir) / (3V) and the virial Vir = -1/2 sum_i w_i,        */
/* w_i = sum_j s_ij r_ij (s_ij the pair factor of F_i, r < rc).  Conserved:   */
/*   H = K + U + pe^2/(2W) + P_ext V + Q xi^2/2 + (g + 1) kB T eta.           */
/* A step of dt (h = dt/2) is the symmetric splitting                         */
/*   T(h) B(h) V(h) X(dt) [forces] V(h) B(h) T(h):                            */
/*   T(h): xi += (h/2) G; s = (1 - xi h/2)/(1 + xi h/2); v *= s; pe *= s;     */
/*         K *= s^2; eta += xi h; xi += (h/2) G (G from the updated K, pe)    */
/*   B(h): pe += h (3V (P - P_ext) + (3/g) 2K)                                */
/*   V(h): c = exp(-(1 + 3/g) ve h/2); v *= c; v += h a; v *= c               */
/*   X(dt): q = exp(ve h); x *= q; x += dt v; x *= q; L *= q twice; wrap      */
/* K is summed afresh (or_kinetic) at the start and after the second V(h),   */
/* and carried through the thermostat's scalings otherwise; Vir is that of    */
/* the last force evaluation.  Totals are or_tree_sum over the atoms.         */
/* ------------------------------------------------------------------------ */
static void or_virial(int64_t n, const int64_t *start, const int32_t *nj, const double *nr,
                      const uint8_t *species, const or_pot *p, const double *rho, double *w) {
  for (int64_t i = 0; i < n; ++i) {
    double fpi = or_dembed(p, species[i], rho[i]);
    int si = species[i];
    double acc = 0.0;
    for (int64_t e = start[i]; e < start[i + 1]; ++e) {
      double r = nr[e];
      if (!(r < p->rc)) continue;
      int32_t j = nj[e];
      int sj = species[j];
      double fpj = or_dembed(p, sj, rho[j]);
      double s = or_dphi(p, si, sj, r) + fpi * or_df(p, sj, r) + fpj * or_df(p, si, r);
      acc += s * r;
    }
    w[i] = acc;
  }
}

/* forces, densities and the virial Vir = -1/2 sum_i w_i at x */
static int or_eval_forces_virial(int64_t n, const double *x, const double *y, const double *z,
                                 const uint8_t *species, const double box[3], const or_pot *p,
                                 double *fx, double *fy, double *fz, double *rho, double *w,
                                 double *vir) {
  int64_t cap = 32 * n + 64;
  for (;;) {
    int64_t *start = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *nj = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    double *nr = (double *)malloc((size_t)cap * sizeof(double));
    double *dx = (double *)malloc((size_t)cap * sizeof(double));
    double *dy = (double *)malloc((size_t)cap * sizeof(double));
    double *dz = (double *)malloc((size_t)cap * sizeof(double));
    int64_t tot = or_neighbors(n, x, y, z, box, p->rc, 0, cap, start, nj, nr, dx, dy, dz);
    int ok = tot >= 0 && tot <= cap;
    if (ok) {
      or_density(n, start, nj, nr, species, p, rho);
      or_forces(n, start, nj, nr, dx, dy, dz, species, p, rho, fx, fy, fz);
      or_virial(n, start, nj, nr, species, p, rho, w);
      *vir = -0.5 * or_tree_sum(n, w);
    }
    free(start); free(nj); free(nr); free(dx); free(dy); free(dz);
    if (tot < 0) return -1;
    if (ok) return 0;
    cap = tot;
  }
}

/* the thermostat's half step T(h) with the barostat momentum; returns s */
static double or_npt_thermo(double h, double g1kT, double Q, double W, double *K, double *pe,
                            double *xi, double *eta) {
  double q = 0.5 * h;
  *xi = *xi + q * ((2.0 * *K + *pe * *pe / W - g1kT) / Q);
  double a = *xi * q;
  double s = (1.0 - a) / (1.0 + a);
  *K = *K * s * s;
  *pe = *pe * s;
  *eta = *eta + *xi * h;
  *xi = *xi + q * ((2.0 * *K + *pe * *pe / W - g1kT) / Q);
  return s;
}

int or_md_npt(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
              const uint8_t *species, double box[3], const or_pot *p, double mass_a,
              double mass_b, double dt, int64_t n_steps, double temp, double tau_t,
              double p_ext, double tau_p, double *state, double *fx, double *fy, double *fz,
              double *rho, double *vir_out) {
  double cm[2] = {OR_ACC / mass_a, OR_ACC / mass_b};
  double h = 0.5 * dt;
  double g = 3.0 * (double)n - 3.0;
  double g1kT = (g + 1.0) * (OR_KB * temp);
  double Q = g1kT * tau_t * tau_t;
  double W = g1kT * tau_p * tau_p;
  double xi = state[0], eta = state[1], pe = state[2];
  double *work = (double *)malloc((size_t)n * sizeof(double));
  if (!work) return -1;
  double vir = 0.0;
  if (or_eval_forces_virial(n, x, y, z, species, box, p, fx, fy, fz, rho, work, &vir)) {
    free(work);
    return -1;
  }
  double K = or_kinetic(n, vx, vy, vz, species, mass_a, mass_b, work);
  for (int64_t step = 0; step < n_steps; ++step) {
    /* T(h) */
    double s = or_npt_thermo(h, g1kT, Q, W, &K, &pe, &xi, &eta);
    for (int64_t i = 0; i < n; ++i) {
      vx[i] = vx[i] * s;
      vy[i] = vy[i] * s;
      vz[i] = vz[i] * s;
    }
    /* B(h) */
    double V = box[0] * box[1] * box[2];
    double P = (2.0 * K + vir) / (3.0 * V);
    pe = pe + h * (3.0 * V * (P - p_ext) + (3.0 / g) * (2.0 * K));
    /* V(h) X(dt) */
    double ve = pe / W;
    double c = exp(-(1.0 + 3.0 / g) * ve * (0.5 * h));
    double q = exp(ve * h);
    double L[3] = {box[0] * q * q, box[1] * q * q, box[2] * q * q};
    for (int64_t i = 0; i < n; ++i) {
      double k = cm[species[i]];
      vx[i] = vx[i] * c;
      vy[i] = vy[i] * c;
      vz[i] = vz[i] * c;
      vx[i] = vx[i] + h * (fx[i] * k);
      vy[i] = vy[i] + h * (fy[i] * k);
      vz[i] = vz[i] + h * (fz[i] * k);
      vx[i] = vx[i] * c;
      vy[i] = vy[i] * c;
      vz[i] = vz[i] * c;
      x[i] = or_wrap((x[i] * q + dt * vx[i]) * q, L[0]);
      y[i] = or_wrap((y[i] * q + dt * vy[i]) * q, L[1]);
      z[i] = or_wrap((z[i] * q + dt * vz[i]) * q, L[2]);
    }
    box[0] = L[0];
    box[1] = L[1];
    box[2] = L[2];
    if (or_eval_forces_virial(n, x, y, z, species, box, p, fx, fy, fz, rho, work, &vir)) {
      free(work);
      return -1;
    }
    /* V(h) */
    for (int64_t i = 0; i < n; ++i) {
      double k = cm[species[i]];
      vx[i] = vx[i] * c;
      vy[i] = vy[i] * c;
      vz[i] = vz[i] * c;
      vx[i] = vx[i] + h * (fx[i] * k);
      vy[i] = vy[i] + h * (fy[i] * k);
      vz[i] = vz[i] + h * (fz[i] * k);
      vx[i] = vx[i] * c;
      vy[i] = vy[i] * c;
      vz[i] = vz[i] * c;
    }
    K = or_kinetic(n, vx, vy, vz, species, mass_a, mass_b, work);
    /* B(h) */
    V = box[0] * box[1] * box[2];
    P = (2.0 * K + vir) / (3.0 * V);
    pe = pe + h * (3.0 * V * (P - p_ext) + (3.0 / g) * (2.0 * K));
    /* T(h) */
    s = or_npt_thermo(h, g1kT, Q, W, &K, &pe, &xi, &eta);
    for (int64_t i = 0; i < n; ++i) {
      vx[i] = vx[i] * s;
      vy[i] = vy[i] * s;
      vz[i] = vz[i] * s;
    }
  }
  state[0] = xi;
  state[1] = eta;
  state[2] = pe;
  *vir_out = vir;
  free(work);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Conjugate-gradient relaxation of the positions at fixed species and box   */
/* (Sec. IV.B relaxes the nanocrystal's grain boundaries by conjugate-       */
/* gradient minimization before its MD and MC/MD runs; the variant is not    */
/* given there).  Nonlinear conjugate gradients with the Polak-Ribiere        */
/* coefficient clipped at zero (PR+) and a backtracking line search under    */
/* the sufficient-decrease (Armijo) condition, as in Nocedal and Wright,     */
/* Numerical Optimization (2nd ed.), Sec. 3.1 (backtracking) and Sec. 5.2    */
/* (PR+).  The steps, in order:                                               */
/*   E, F at x;  d = F;  gg = F.F                                             */
/*   loop:                                                                     */
/*     sqrt(gg) <= ftol: FORCE;  it >= max_iter: ITER;  ev >= max_eval: EVAL  */
/*     sl = F.d;  sl <= 0: d = F, sl = F.d (restart along the force)          */
/*     dm = sqrt(max_i |d_i|^2);  a = dmax / dm, after the first iteration    */
/*       the smaller of that and 2 dE_prev / sl (the minimizer of the        */
/*       quadratic through the last decrease, Nocedal and Wright, Sec. 3.5)  */
/*     up to CG_TRIALS trials: x' = wrap(x + a d) per component, E' and F'   */
/*       at x' (ev += 1); E' <= E - c1 a sl and E' < E: accepted (the      */
/*       second test matters only once c1 a sl is below the rounding of E); */
/*       else a = a / 2                                                       */
/*     none accepted: LINESEARCH (x, E, F unchanged)                           */
/*     b = (F'.F' - F'.F) / gg, clipped at 0;  d = F' + b d                    */
/*     dE = E - E';  x, E, F, gg = x', E', F', F'.F';  it += 1                 */
/*     dE <= etol |E|: ENERGY                                                   */
/* E = or_tree_sum of the atoms' energies; each dot product is or_tree_sum   */
/* of the per-atom terms (ax bx + ay by) + az bz.                             */
/* ------------------------------------------------------------------------ */
#define CG_TRIALS 41
#define CG_C1 1e-4

/* energy (returned through *e_tot), forces and densities at x */
static int or_eval_energy_forces(int64_t n, const double *x, const double *y, const double *z,
                                 const uint8_t *species, const double box[3], const or_pot *p,
                                 double *fx, double *fy, double *fz, double *rho, double *e,
                                 double *e_tot) {
  int64_t cap = 32 * n + 64;
  for (;;) {
    int64_t *start = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *nj = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    double *nr = (double *)malloc((size_t)cap * sizeof(double));
    double *dx = (double *)malloc((size_t)cap * sizeof(double));
    double *dy = (double *)malloc((size_t)cap * sizeof(double));
    double *dz = (double *)malloc((size_t)cap * sizeof(double));
    int64_t tot = or_neighbors(n, x, y, z, box, p->rc, 0, cap, start, nj, nr, dx, dy, dz);
    int ok = tot >= 0 && tot <= cap;
    if (ok) {
      or_density(n, start, nj, nr, species, p, rho);
      or_energy_atoms(n, start, nj, nr, species, p, rho, e);
      or_forces(n, start, nj, nr, dx, dy, dz, species, p, rho, fx, fy, fz);
      *e_tot = or_tree_sum(n, e);
    }
    free(start); free(nj); free(nr); free(dx); free(dy); free(dz);
    if (tot < 0) return -1;
    if (ok) return 0;
    cap = tot;
  }
}

/* or_tree_sum of (ax bx + ay by) + az bz over the atoms */
static double or_dot3(int64_t n, const double *ax, const double *ay, const double *az,
                      const double *bx, const double *by, const double *bz, double *work) {
  for (int64_t i = 0; i < n; ++i) work[i] = (ax[i] * bx[i] + ay[i] * by[i]) + az[i] * bz[i];
  return or_tree_sum(n, work);
}

int or_cg(int64_t n, double *x, double *y, double *z, const uint8_t *species,
          const double box[3], const or_pot *p, int64_t max_iter, int64_t max_eval, double etol,
          double ftol, double dmax, int steepest, double *fx, double *fy, double *fz,
          double *rho, int64_t *iters_out, int64_t *evals_out, double *e_out, double *fnorm_out,
          int *reason_out, double *log, int64_t log_cap) {
  size_t nb = (size_t)n * sizeof(double);
  double *buf = (double *)malloc(12 * nb);
  if (!buf) return -1;
  double *dx = buf, *dy = buf + n, *dz = buf + 2 * n;
  double *xt = buf + 3 * n, *yt = buf + 4 * n, *zt = buf + 5 * n;
  double *gx = buf + 6 * n, *gy = buf + 7 * n, *gz = buf + 8 * n;
  double *e = buf + 9 * n, *work = buf + 10 * n, *rt = buf + 11 * n;
  double E = 0.0;
  int rc = -1;
  if (or_eval_energy_forces(n, x, y, z, species, box, p, fx, fy, fz, rho, e, &E)) goto out;
  for (int64_t i = 0; i < n; ++i) {
    dx[i] = fx[i];
    dy[i] = fy[i];
    dz[i] = fz[i];
  }
  double gg = or_dot3(n, fx, fy, fz, fx, fy, fz, work);
  int64_t it = 0, ev = 0;
  int reason;
  double dE_prev = 0.0;
  for (;;) {
    if (sqrt(gg) <= ftol) {
      reason = OR_CG_FORCE;
      break;
    }
    if (it >= max_iter) {
      reason = OR_CG_ITER;
      break;
    }
    if (ev >= max_eval) {
      reason = OR_CG_EVAL;
      break;
    }
    double sl = or_dot3(n, fx, fy, fz, dx, dy, dz, work);
    int restart = 0;
    if (!(sl > 0.0)) {
      for (int64_t i = 0; i < n; ++i) {
        dx[i] = fx[i];
        dy[i] = fy[i];
        dz[i] = fz[i];
      }
      sl = or_dot3(n, fx, fy, fz, dx, dy, dz, work);
      restart = 1;
    }
    double dm2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double q = (dx[i] * dx[i] + dy[i] * dy[i]) + dz[i] * dz[i];
      if (q > dm2) dm2 = q;
    }
    double a = dmax / sqrt(dm2);
    if (it > 0) {
      double a1 = 2.0 * dE_prev / sl;
      if (a1 < a) a = a1;
    }
    double Et = 0.0;
    int accepted = 0;
    for (int t = 0; t < CG_TRIALS; ++t) {
      for (int64_t i = 0; i < n; ++i) {
        xt[i] = or_wrap(x[i] + a * dx[i], box[0]);
        yt[i] = or_wrap(y[i] + a * dy[i], box[1]);
        zt[i] = or_wrap(z[i] + a * dz[i], box[2]);
      }
      if (or_eval_energy_forces(n, xt, yt, zt, species, box, p, gx, gy, gz, rt, e, &Et)) goto out;
      ev += 1;
      if (Et <= E - CG_C1 * a * sl && Et < E) {
        accepted = 1;
        break;
      }
      a = a * 0.5;
    }
    if (!accepted) {
      reason = OR_CG_LINESEARCH;
      break;
    }
    double g_new = or_dot3(n, gx, gy, gz, gx, gy, gz, work);
    double g_mix = or_dot3(n, gx, gy, gz, fx, fy, fz, work);
    double b = (g_new - g_mix) / gg;
    if (!(b > 0.0) || steepest) b = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      dx[i] = gx[i] + b * dx[i];
      dy[i] = gy[i] + b * dy[i];
      dz[i] = gz[i] + b * dz[i];
    }
    double dE = E - Et;
    dE_prev = dE;
    if (log && it < log_cap) {
      double *L = log + 6 * it;
      L[0] = E;
      L[1] = Et;
      L[2] = a;
      L[3] = sl;
      L[4] = b;
      L[5] = (double)restart;
    }
    memcpy(x, xt, nb);
    memcpy(y, yt, nb);
    memcpy(z, zt, nb);
    memcpy(fx, gx, nb);
    memcpy(fy, gy, nb);
    memcpy(fz, gz, nb);
    memcpy(rho, rt, nb);
    E = Et;
    gg = g_new;
    it += 1;
    if (dE <= etol * fabs(E)) {
      reason = OR_CG_ENERGY;
      break;
    }
  }
  *iters_out = it;
  *evals_out = ev;
  *e_out = E;
  *fnorm_out = sqrt(gg);
  *reason_out = reason;
  rc = 0;
out:
  free(buf);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* All-core CPU baseline of or_md: the same per-atom arithmetic (neighbour   */
/* rows, densities, forces, kicks) with the atoms split over n_threads       */
/* OpenMP threads.  Rows are built twice (count, then fill at the row's      */
/* offset), so the list is the serial one and every value is bitwise         */
/* or_md's.                                                                  */
/* ------------------------------------------------------------------------ */
static int or_eval_forces_omp(int64_t n, const double *x, const double *y, const double *z,
                              const uint8_t *species, const double box[3], const or_pot *p,
                              double *fx, double *fy, double *fz, double *rho, int n_threads) {
  nbr_grid G;
  if (or_nbr_setup(n, x, y, z, box, p->rc, 0, &G)) return -1;
  int64_t *start = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
#pragma omp parallel num_threads(n_threads)
  {
    nbuf row = {0, 0, 0};
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      or_nbr_row(i, n, x, y, z, box, p->rc, &G, &row);
      start[i + 1] = row.n;
    }
    free(row.e);
  }
  start[0] = 0;
  for (int64_t i = 0; i < n; ++i) start[i + 1] += start[i];
  int64_t tot = start[n];
  int32_t *nj = (int32_t *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(int32_t));
  double *nr = (double *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(double));
  double *dx = (double *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(double));
  double *dy = (double *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(double));
  double *dz = (double *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(double));
  double *fp = (double *)malloc((size_t)n * sizeof(double));
#pragma omp parallel num_threads(n_threads)
  {
    nbuf row = {0, 0, 0};
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      or_nbr_row(i, n, x, y, z, box, p->rc, &G, &row);
      for (int64_t k = 0; k < row.n; ++k) {
        int64_t e = start[i] + k;
        nj[e] = row.e[k].j;
        nr[e] = row.e[k].r;
        dx[e] = row.e[k].dx;
        dy[e] = row.e[k].dy;
        dz[e] = row.e[k].dz;
      }
    }
    free(row.e);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) rho[i] = or_density_row(i, start, nj, nr, species, p);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) fp[i] = or_dembed(p, species[i], rho[i]);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i)
      or_force_row(i, start, nj, nr, dx, dy, dz, species, p, fp, fx, fy, fz);
  }
  or_nbr_free(&G);
  free(start); free(nj); free(nr); free(dx); free(dy); free(dz); free(fp);
  return 0;
}

int or_md_omp(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
              const uint8_t *species, const double box[3], const or_pot *p,
              double mass_a, double mass_b, double dt, int64_t n_steps,
              double *fx, double *fy, double *fz, double *rho, int n_threads) {
  double cm[2] = {OR_ACC / mass_a, OR_ACC / mass_b};
  double hdt = 0.5 * dt;
  if (n_threads < 1) n_threads = 1;
  if (or_eval_forces_omp(n, x, y, z, species, box, p, fx, fy, fz, rho, n_threads)) return -1;
  for (int64_t step = 0; step < n_steps; ++step) {
#pragma omp parallel for schedule(static) num_threads(n_threads)
    for (int64_t i = 0; i < n; ++i) {
      double c = cm[species[i]];
      vx[i] = vx[i] + hdt * (fx[i] * c);
      vy[i] = vy[i] + hdt * (fy[i] * c);
      vz[i] = vz[i] + hdt * (fz[i] * c);
      x[i] = or_wrap(x[i] + dt * vx[i], box[0]);
      y[i] = or_wrap(y[i] + dt * vy[i], box[1]);
      z[i] = or_wrap(z[i] + dt * vz[i], box[2]);
    }
    if (or_eval_forces_omp(n, x, y, z, species, box, p, fx, fy, fz, rho, n_threads)) return -1;
#pragma omp parallel for schedule(static) num_threads(n_threads)
    for (int64_t i = 0; i < n; ++i) {
      double c = cm[species[i]];
      vx[i] = vx[i] + hdt * (fx[i] * c);
      vy[i] = vy[i] + hdt * (fy[i] * c);
      vz[i] = vz[i] + hdt * (fz[i] * c);
    }
  }
  return 0;
}
