// Link cells and neighbour lists (Sec. III.A: cells of edge >= the
// independence distance, an even number per dimension so that cells whose
// index parities agree are a full cell edge apart), the density cache of the
// sweep, input validation and a fixed-shape FP64 reduction.
#include "common.hpp"

namespace vc {

// ----------------------------------------------------------------------------
// validation: positions inside [0, L), species in {0, 1}
// ----------------------------------------------------------------------------
__global__ void k_validate(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                           const double *__restrict__ z, const uint8_t *__restrict__ sp, double L0,
                           double L1, double L2, DevState *ds) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = x[i], b = y[i], c = z[i];
  const bool ok = (a >= 0.0 && a < L0) && (b >= 0.0 && b < L1) && (c >= 0.0 && c < L2) &&
                  sp[i] <= 1;
  if (!ok) atomicOr(&ds->bad_input, 1);
}

hipError_t launch_validate(vcsgc_ctx *c, const RepHost &r) {
  k_validate<<<grid_for(r.n), BLOCK, 0, c->stream>>>(r.n, c->x + r.aoff, c->y + r.aoff,
                                                     c->z + r.aoff, c->sp + r.aoff, r.box[0],
                                                     r.box[1], r.box[2], c->ds);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// binning: count, exclusive scan, scatter, then sort each cell ascending
// ----------------------------------------------------------------------------
struct Grid {
  double L0, L1, L2;
  int n0, n1, n2;
};

__device__ __forceinline__ int cell_of(const Grid &g, double a, double b, double c) {
  const int cx = cell_coord(a, g.L0, g.n0);
  const int cy = cell_coord(b, g.L1, g.n1);
  const int cz = cell_coord(c, g.L2, g.n2);
  return cx + g.n0 * (cy + g.n1 * cz);
}

// atomicAdd(&counter[key], 1) for every active lane, with one atomic per
// distinct key in the wave (neighbouring atoms mostly share a cell); returns
// the lane's old value plus its rank among the lanes with the same key
__device__ __forceinline__ int32_t wave_add_one(int32_t *counter, int key) {
  const int lane = __lane_id();
  unsigned long long todo = __ballot(1);
  int32_t slot = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lkey = __shfl(key, leader);
    const unsigned long long same = __ballot(key == lkey) & todo;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(&counter[lkey], (int32_t)__popcll(same));
    base = __shfl(base, leader);
    if (same & (1ull << lane)) slot = base + (int32_t)__popcll(same & ((1ull << lane) - 1ull));
    todo &= ~same;
  }
  return slot;
}

__global__ void k_cell_count(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                             const double *__restrict__ z, Grid g, int32_t *count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  (void)wave_add_one(count, cell_of(g, x[i], y[i], z[i]));
}

// exclusive scan of count[0..m) into start[0..m] (and a copy in fill):
// chunks of SCAN_CHUNK values, first the chunk sums, then every chunk adds
// the sums of the chunks before it to its own scan
// Values are clamped to cap; fill may be NULL; cond (may be NULL): run only
// when *cond != 0.
__global__ void __launch_bounds__(256) k_scan_sums(int64_t m, const int32_t *__restrict__ count,
                                                   int32_t *bsum, int cap, const int *cond) {
  if (cond && *cond == 0) return;
  __shared__ int32_t s[256];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
  int32_t v = 0;
  for (int k = threadIdx.x; k < SCAN_CHUNK; k += 256)
    if (base + k < m) v += min(count[base + k], cap);
  s[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(256) k_scan_apply(int64_t m, const int32_t *__restrict__ count,
                                                    const int32_t *__restrict__ bsum,
                                                    int32_t *start, int32_t *fill, int cap,
                                                    const int *cond) {
  if (cond && *cond == 0) return;
  __shared__ int32_t s[256];
  const int t = threadIdx.x;
  // offset of this chunk
  int32_t o = 0;
  for (int k = t; k < (int)blockIdx.x; k += 256) o += bsum[k];
  s[t] = o;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) s[t] += s[t + h];
    __syncthreads();
  }
  const int32_t off = s[0];
  __syncthreads();
  // thread t owns values 4t .. 4t+3 of the chunk
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + 4 * t;
  int32_t v[4], own = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[q] = base + q < m ? min(count[base + q], cap) : 0;
    own += v[q];
  }
  s[t] = own;
  __syncthreads();
  for (int h = 1; h < 256; h <<= 1) {
    const int32_t add = t >= h ? s[t - h] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  int32_t run = off + s[t] - own;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (base + q < m) {
      start[base + q] = run;
      if (fill) fill[base + q] = run;
    }
    run += v[q];
  }
  if (blockIdx.x == gridDim.x - 1 && t == 255) start[m] = off + s[255];
}

__global__ void k_cell_fill(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                            const double *__restrict__ z, Grid g, int32_t *fill, int32_t *atoms,
                            int64_t aoff) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cell_of(g, x[i], y[i], z[i]);
  atoms[wave_add_one(fill, c)] = (int32_t)(aoff + i);
}

// canonical order inside a cell: ascending site index.  One wave per cell:
// a rank sort in LDS (every index is distinct); cells larger than the LDS
// buffer fall back to an insertion sort by one lane.
constexpr int SORT_CAP = 2048;

__global__ void __launch_bounds__(64) k_cell_sort(int64_t m, const int32_t *__restrict__ start,
                                                  int32_t *atoms) {
  __shared__ int32_t v[SORT_CAP];
  const int64_t c = blockIdx.x;
  const int32_t lo = start[c], hi = start[c + 1];
  const int cnt = hi - lo;
  if (cnt <= 1) return;
  if (cnt > SORT_CAP) {
    if (threadIdx.x == 0) {
      for (int32_t a = lo + 1; a < hi; ++a) {
        const int32_t x = atoms[a];
        int32_t b = a - 1;
        while (b >= lo && atoms[b] > x) {
          atoms[b + 1] = atoms[b];
          --b;
        }
        atoms[b + 1] = x;
      }
    }
    return;
  }
  for (int e = threadIdx.x; e < cnt; e += 64) v[e] = atoms[lo + e];
  __syncthreads();
  for (int e = threadIdx.x; e < cnt; e += 64) {
    const int32_t x = v[e];
    int rank = 0;
    for (int f = 0; f < cnt; ++f) rank += v[f] < x ? 1 : 0;
    atoms[lo + rank] = x;
  }
}

// cells of one replica; cell_atoms holds global atom indices, cell_start the
// positions inside the replica's segment of cell_atoms
hipError_t launch_bin_cells(vcsgc_ctx *c, const RepHost &r) {
  Grid g{r.box[0], r.box[1], r.box[2], r.nc[0], r.nc[1], r.nc[2]};
  int32_t *count = c->cell_count + r.coff, *fill = c->cell_fill + r.coff;
  int32_t *start = c->cell_start + r.cso, *atoms = c->cell_atoms + r.aoff;
  hipError_t e = hipMemsetAsync(count, 0, sizeof(int32_t) * r.ncells, c->stream);
  if (e != hipSuccess) return e;
  const double *x = c->x + r.aoff, *y = c->y + r.aoff, *z = c->z + r.aoff;
  k_cell_count<<<grid_for(r.n), BLOCK, 0, c->stream>>>(r.n, x, y, z, g, count);
  const int nchunk = (int)((r.ncells + SCAN_CHUNK - 1) / SCAN_CHUNK);
  k_scan_sums<<<nchunk, 256, 0, c->stream>>>(r.ncells, count, c->scan_tmp, INT32_MAX, nullptr);
  k_scan_apply<<<nchunk, 256, 0, c->stream>>>(r.ncells, count, c->scan_tmp, start, fill,
                                              INT32_MAX, nullptr);
  k_cell_fill<<<grid_for(r.n), BLOCK, 0, c->stream>>>(r.n, x, y, z, g, fill, atoms, r.aoff);
  k_cell_sort<<<(unsigned)r.ncells, 64, 0, c->stream>>>(r.ncells, start, atoms);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// search bins: edge >= rc + skin, at most bmax atoms each (overflow flagged)
// ----------------------------------------------------------------------------
// cond (may be NULL): run only when *cond != 0 (device-decided MD rebuild)
// pos (may be NULL) receives (x, y, z, i) of the atom in its slot
__global__ void k_bin_search(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                             const double *__restrict__ z, Grid g, int bmax, int32_t *count,
                             int32_t *atoms, double4 *pos, DevState *ds, const int *cond) {
  if (cond && *cond == 0) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = x[i], b2 = y[i], c2 = z[i];
  const int b = cell_of(g, a, b2, c2);
  const int slot = atomicAdd(&count[b], 1);
  if (slot < bmax) {
    atoms[(int64_t)b * bmax + slot] = (int32_t)i;
    if (pos) pos[(int64_t)b * bmax + slot] = make_double4(a, b2, c2, (double)i);
  } else {
    atomicOr(&ds->bin_overflow, 1);
  }
}

// search bins of one replica (local atom indices)
hipError_t launch_bin_search(vcsgc_ctx *c, const RepHost &r) {
  Grid g{r.box[0], r.box[1], r.box[2], r.nb[0], r.nb[1], r.nb[2]};
  int32_t *count = c->bin_count + r.boff, *atoms = c->bin_atoms + r.boff * c->bmax;
  hipError_t e = hipMemsetAsync(count, 0, sizeof(int32_t) * r.nbins, c->stream);
  if (e != hipSuccess) return e;
  k_bin_search<<<grid_for(r.n), BLOCK, 0, c->stream>>>(r.n, c->x + r.aoff, c->y + r.aoff,
                                                       c->z + r.aoff, g, c->bmax, count, atoms,
                                                       c->reps.size() == 1 ? c->bin_pos : nullptr,
                                                       c->ds, nullptr);
  return hipGetLastError();
}

// clears the bin counts and the MD row statistics when a rebuild is pending
__global__ void k_bins_clear_cond(int64_t nbins, int32_t *count, DevState *ds) {
  if (ds->rebuild == 0) return;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) {
    ds->pairs_md = 0ull;
    ds->kmax_md = 0;
  }
  if (b < nbins) count[b] = 0;
}

// closes a pending rebuild: the list now matches the positions
__global__ void k_rebuild_done(DevState *ds) {
  if (threadIdx.x == 0 && ds->rebuild != 0) {
    ds->rebuild = 0;
    ds->md_rebuilds += 1ull;
  }
}

// ----------------------------------------------------------------------------
// neighbour lists from the search bins.  Every pair with r < cutoff, r from
// the minimum-image separation as sqrt((dx^2 + dy^2) + dz^2), rows sorted by
// neighbour index.  Column-major rows: entry k of atom i at [k * n + i].
// MC rows additionally store dd = (rc - r)^2 and g = c0 + c1 r.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double pair_r(const double *__restrict__ x,
                                         const double *__restrict__ y,
                                         const double *__restrict__ z, const Grid &g, double xi,
                                         double yi, double zi, int32_t j) {
  const double dx = min_image(x[j] - xi, g.L0);
  const double dy = min_image(y[j] - yi, g.L1);
  const double dz = min_image(z[j] - zi, g.L2);
  return sqrt((dx * dx + dy * dy) + dz * dz);
}

// One group of BG lanes per atom; lane L walks the L-th of the 27 (or fewer,
// with two bins along an axis) surrounding search bins.  Hits are appended to
// an LDS row through an LDS counter (arbitrary order), then every hit is
// stored at its rank among the row's neighbour indices, so rows come out
// sorted and independent of the append order.  Rows are row-major
// ([i * KMAX + k]) for the group-per-trial sweep kernels.
constexpr int BG = 32;

// MODE 1: MC rows ((rc - r)^2 and c0 + c1 r), 2: descriptor rows (r)
template <int MODE>
__global__ void __launch_bounds__(BLOCK)
    k_build(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
            const double *__restrict__ z, Grid g, const int32_t *__restrict__ bcount,
            const int32_t *__restrict__ batoms, int bmax, double cutoff, PotD p, int32_t *nj,
            double *ndd, double *ng, uint8_t *cnt, DevState *ds, int64_t aoff) {
  __shared__ int32_t rowbuf[BLOCK / BG][KMAX];
  __shared__ int rowcount[BLOCK / BG];
  const int lane = threadIdx.x % BG, grp = threadIdx.x / BG;
  const int64_t i = (xcd_block() * BLOCK + threadIdx.x) / BG;
  const bool live = i < n;
  if (lane == 0) rowcount[grp] = 0;
  __syncthreads();
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (live) {
    xi = x[i];
    yi = y[i];
    zi = z[i];
    const int n0 = g.n0 >= 3 ? 3 : 2, n1 = g.n1 >= 3 ? 3 : 2, n2 = g.n2 >= 3 ? 3 : 2;
    if (lane < n0 * n1 * n2) {
      const int ox = (g.n0 >= 3 ? -1 : 0) + lane % n0;
      const int oy = (g.n1 >= 3 ? -1 : 0) + (lane / n0) % n1;
      const int oz = (g.n2 >= 3 ? -1 : 0) + lane / (n0 * n1);
      const int xx = (cell_coord(xi, g.L0, g.n0) + ox + g.n0) % g.n0;
      const int yy = (cell_coord(yi, g.L1, g.n1) + oy + g.n1) % g.n1;
      const int zz = (cell_coord(zi, g.L2, g.n2) + oz + g.n2) % g.n2;
      const int64_t bb = xx + (int64_t)g.n0 * (yy + (int64_t)g.n1 * zz);
      int m = bcount[bb];
      m = m < bmax ? m : bmax;
      for (int k = 0; k < m; ++k) {
        const int32_t j = batoms[bb * bmax + k];
        if (j != i && pair_r(x, y, z, g, xi, yi, zi, j) < cutoff) {
          const int pos = atomicAdd(&rowcount[grp], 1);
          if (pos < KMAX) rowbuf[grp][pos] = j;
        }
      }
    }
  }
  __syncthreads();
  if (live) {
    int count = rowcount[grp];
    if (count > KMAX) {
      if (lane == 0) atomicOr(&ds->overflow, 1);
      count = KMAX;
    }
    const int64_t ig = aoff + i;  // global row
    if (lane == 0) cnt[ig] = (uint8_t)count;
    for (int a = lane; a < count; a += BG) {
      const int32_t j = rowbuf[grp][a];
      int rank = 0;
      for (int b = 0; b < count; ++b) rank += rowbuf[grp][b] < j ? 1 : 0;
      const int64_t e = ig * KMAX + rank;
      nj[e] = (int32_t)(aoff + j);
      const double r = pair_r(x, y, z, g, xi, yi, zi, j);
      if (MODE == 1) {
        const double d = p.rc - r;
        ndd[e] = d * d;
        ng[e] = p.c0 + p.c1 * r;
      } else {
        ndd[e] = r;
      }
    }
  }
}

// sum and maximum of the row lengths: one atomic pair per block
__global__ void __launch_bounds__(BLOCK) k_row_stats(int64_t n, const uint8_t *__restrict__ cnt,
                                                     unsigned long long *sum, int *mx,
                                                     const int *cond) {
  if (cond && *cond == 0) return;
  __shared__ unsigned int ss[BLOCK];
  __shared__ int sm[BLOCK];
  unsigned int a = 0;
  int b = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * BLOCK) {
    const int v = cnt[i];
    a += v;
    b = v > b ? v : b;
  }
  ss[threadIdx.x] = a;
  sm[threadIdx.x] = b;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      ss[threadIdx.x] += ss[threadIdx.x + h];
      sm[threadIdx.x] = sm[threadIdx.x] > sm[threadIdx.x + h] ? sm[threadIdx.x] : sm[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(sum, (unsigned long long)ss[0]);
    atomicMax(mx, sm[0]);
  }
}

// r < rc list of one replica (rows and neighbour indices global)
hipError_t launch_build_mc_list(vcsgc_ctx *c, const RepHost &r) {
  Grid g{r.box[0], r.box[1], r.box[2], r.nb[0], r.nb[1], r.nb[2]};
  int h = tstart(c, VCSGC_KT_BUILD);
  k_build<1><<<grid_for(r.n * BG), BLOCK, 0, c->stream>>>(
      r.n, c->x + r.aoff, c->y + r.aoff, c->z + r.aoff, g, c->bin_count + r.boff,
      c->bin_atoms + r.boff * c->bmax, c->bmax, c->pot.rc, c->pot, c->mc_j, c->mc_dd, c->mc_g,
      c->mc_cnt, c->ds, r.aoff);
  tstop(c, h);
  return hipGetLastError();
}

// r < 4.41 A descriptor list of one replica (row-major, with distances)
hipError_t launch_build_desc_list(vcsgc_ctx *c, const RepHost &r) {
  Grid g{r.box[0], r.box[1], r.box[2], r.nb[0], r.nb[1], r.nb[2]};
  k_build<2><<<grid_for(r.n * BG), BLOCK, 0, c->stream>>>(
      r.n, c->x + r.aoff, c->y + r.aoff, c->z + r.aoff, g, c->bin_count + r.boff,
      c->bin_atoms + r.boff * c->bmax, c->bmax, DESC_CUT, c->pot, c->d_j, c->d_r, nullptr,
      c->d_cnt, c->ds, r.aoff);
  return hipGetLastError();
}

hipError_t launch_mc_row_stats(vcsgc_ctx *c) {
  hipError_t e = hipMemsetAsync(&c->ds->pairs_mc, 0, sizeof(unsigned long long), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(&c->ds->kmax_used, 0, sizeof(int), c->stream);
  if (e != hipSuccess) return e;
  k_row_stats<<<512, BLOCK, 0, c->stream>>>(c->n, c->mc_cnt, &c->ds->pairs_mc, &c->ds->kmax_used,
                                            nullptr);
  return hipGetLastError();
}

// r < rc + skin list, one lane per atom (used when some axis has fewer than
// four search bins): the lane walks the surrounding search bins through the
// packed (x, y, z, index) slots, appends hits to its
// column-major row, then reloads the row into registers, sorts it by a fixed
// bitonic network (ascending neighbour index) and writes it back.  The test
// is r^2 < cut2: the list only has to hold every pair that can come within
// rc before the next rebuild (its users test r < rc themselves).
// cond (may be NULL): run only when *cond != 0.
__global__ void __launch_bounds__(BLOCK)
    k_build_md(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
               const double *__restrict__ z, Grid g, const int32_t *__restrict__ bcount,
               const double4 *__restrict__ bpos, int bmax, double cut2, int32_t *nj, uint8_t *cnt,
               double *xr, double *yr, double *zr, DevState *ds, const int *cond) {
  if (cond && *cond == 0) return;
  const int64_t i = xcd_block() * BLOCK + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i], zi = z[i];
  const int bx = cell_coord(xi, g.L0, g.n0), by = cell_coord(yi, g.L1, g.n1),
            bz = cell_coord(zi, g.L2, g.n2);
  const int n0 = g.n0 >= 3 ? 3 : 2, n1 = g.n1 >= 3 ? 3 : 2, n2 = g.n2 >= 3 ? 3 : 2;
  const int s0 = g.n0 >= 3 ? -1 : 0, s1 = g.n1 >= 3 ? -1 : 0, s2 = g.n2 >= 3 ? -1 : 0;
  int c = 0;
  for (int oz = 0; oz < n2; ++oz) {
    const int zz = (bz + s2 + oz + g.n2) % g.n2;
    for (int oy = 0; oy < n1; ++oy) {
      const int yy = (by + s1 + oy + g.n1) % g.n1;
      for (int ox = 0; ox < n0; ++ox) {
        const int xx = (bx + s0 + ox + g.n0) % g.n0;
        const int64_t nb = xx + (int64_t)g.n0 * (yy + (int64_t)g.n1 * zz);
        const int m = min(bcount[nb], bmax);
        const double4 *slot = bpos + nb * bmax;
        for (int t = 0; t < m; t += 4) {
          double4 q[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) q[u] = t + u < m ? slot[t + u] : make_double4(0, 0, 0, -1.0);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int32_t j = (int32_t)q[u].w;
            if (t + u < m && j != (int32_t)i) {
              const double dx = min_image(q[u].x - xi, g.L0);
              const double dy = min_image(q[u].y - yi, g.L1);
              const double dz = min_image(q[u].z - zi, g.L2);
              if ((dx * dx + dy * dy) + dz * dz < cut2) {
                if (c < KMAX) nj[(int64_t)c * n + i] = j;
                ++c;
              }
            }
          }
        }
      }
    }
  }
  if (c > KMAX) {
    atomicOr(&ds->overflow, 1);
    c = KMAX;
  }
  int32_t v[KMAX];
#pragma unroll
  for (int u = 0; u < KMAX; ++u) v[u] = u < c ? nj[(int64_t)u * n + i] : INT32_MAX;
#pragma unroll
  for (int k = 2; k <= KMAX; k <<= 1) {
#pragma unroll
    for (int h = k >> 1; h > 0; h >>= 1) {
#pragma unroll
      for (int a = 0; a < KMAX; ++a) {
        const int b = a ^ h;
        if (b > a) {
          const int32_t lo = min(v[a], v[b]), hi = max(v[a], v[b]);
          const bool up = (a & k) == 0;
          v[a] = up ? lo : hi;
          v[b] = up ? hi : lo;
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < KMAX; ++u)
    if (u < c) nj[(int64_t)u * n + i] = v[u];
  cnt[i] = (uint8_t)c;
  xr[i] = xi;
  yr[i] = yi;
  zr[i] = zi;
}

// r < rc + skin list by super-bins of 2 x 2 x 2 search bins (every axis needs
// at least four bins).  A block stages the 4 x 4 x 4 bins around its
// super-bin in LDS once (positions relative to the super-bin origin, in
// float, periodic images resolved), then four lanes per own atom test the
// atom's 27 neighbouring bins from LDS and append hits to an LDS row.  The
// float test uses cut2f = (cut + 1e-3)^2, a superset of r < cut (coordinates
// are below 20 A, so the float error is below 1e-5 A); users of the list test
// r < rc in FP64 themselves.  Rows go out unsorted, row-major, to tmp; the
// finishing kernel sorts them and writes the column-major list.
// Dynamic LDS: 64 * bmax float4.
constexpr int SB_OWN = 64;  // own atoms per pass (four lanes each)

__global__ void __launch_bounds__(BLOCK)
    k_build_md_sb(Grid g, int nsx, int nsy, const int32_t *__restrict__ bcount,
                  const double4 *__restrict__ bpos, int bmax, float cut2f, int32_t *tmp,
                  int32_t *tcnt, const int *cond) {
  if (cond && *cond == 0) return;
  extern __shared__ float4 cand[];
  __shared__ int cnt[64], off[65], gbin[64];
  __shared__ double shx[64], shy[64], shz[64];
  __shared__ int rowlen[SB_OWN];
  __shared__ int32_t hit[SB_OWN * KMAX];
  __shared__ int own_bins[8], n_own_bins;
  const int tid = threadIdx.x;
  const int64_t sb = xcd_block();
  const int sx = (int)(sb % nsx), sy = (int)((sb / nsx) % nsy), sz = (int)(sb / ((int64_t)nsx * nsy));
  const double bw0 = g.L0 / g.n0, bw1 = g.L1 / g.n1, bw2 = g.L2 / g.n2;
  // origin of the super-bin
  const double o0 = (2 * sx) * bw0, o1 = (2 * sy) * bw1, o2 = (2 * sz) * bw2;
  if (tid < 64) {
    const int ux = tid & 3, uy = (tid >> 2) & 3, uz = tid >> 4;
    int gx = 2 * sx - 1 + ux, gy = 2 * sy - 1 + uy, gz = 2 * sz - 1 + uz;
    double hx = 0.0, hy = 0.0, hz = 0.0;  // image shift
    if (gx < 0) { gx += g.n0; hx = -g.L0; } else if (gx >= g.n0) { gx -= g.n0; hx = g.L0; }
    if (gy < 0) { gy += g.n1; hy = -g.L1; } else if (gy >= g.n1) { gy -= g.n1; hy = g.L1; }
    if (gz < 0) { gz += g.n2; hz = -g.L2; } else if (gz >= g.n2) { gz -= g.n2; hz = g.L2; }
    const int b = gx + g.n0 * (gy + g.n1 * gz);
    gbin[tid] = b;
    shx[tid] = hx;
    shy[tid] = hy;
    shz[tid] = hz;
    cnt[tid] = min(bcount[b], bmax);
  }
  if (tid == 0) {
    // own bins: local coordinates 1..2 that exist on the grid
    int k = 0;
    for (int uz = 1; uz <= 2; ++uz)
      for (int uy = 1; uy <= 2; ++uy)
        for (int ux = 1; ux <= 2; ++ux)
          if (2 * sx + ux - 1 < g.n0 && 2 * sy + uy - 1 < g.n1 && 2 * sz + uz - 1 < g.n2)
            own_bins[k++] = ux + 4 * (uy + 4 * uz);
    n_own_bins = k;
  }
  __syncthreads();
  if (tid == 0) {
    off[0] = 0;
    for (int u = 0; u < 64; ++u) off[u + 1] = off[u] + cnt[u];
  }
  __syncthreads();
  // stage every slot of the 64 bins: (x, y, z) relative to the origin, index in w
  for (int q = tid; q < 64 * bmax; q += BLOCK) {
    const int u = q / bmax, t = q - u * bmax;
    if (t < cnt[u]) {
      const double4 p = bpos[(int64_t)gbin[u] * bmax + t];
      cand[off[u] + t] = make_float4((float)(p.x + shx[u] - o0), (float)(p.y + shy[u] - o1),
                                     (float)(p.z + shz[u] - o2), __int_as_float((int32_t)p.w));
    }
  }
  int n_own = 0;
  for (int k = 0; k < n_own_bins; ++k) n_own += cnt[own_bins[k]];
  __syncthreads();
  for (int base = 0; base < n_own; base += SB_OWN) {
    const int a = tid >> 2, l = tid & 3;
    // own atom base + a: its bin and staged index
    int ob = -1, si = -1;
    {
      int q = base + a;
      for (int k = 0; k < n_own_bins && q >= 0; ++k) {
        const int u = own_bins[k];
        if (q < cnt[u]) {
          ob = u;
          si = off[u] + q;
          q = -1;
        } else {
          q -= cnt[u];
        }
      }
    }
    if (l == 0) rowlen[a] = 0;
    __syncthreads();
    if (si >= 0) {
      const float4 me = cand[si];
      const int lx = ob & 3, ly = (ob >> 2) & 3, lz = ob >> 4;
      int phase = l;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
          const int u0 = (lx - 1) + 4 * ((ly + dy) + 4 * (lz + dz));
          const int a0 = off[u0], len = off[u0 + 3] - a0;
          int t = phase;
          for (; t < len; t += 4) {
            const int ci = a0 + t;
            if (ci == si) continue;
            const float4 c = cand[ci];
            const float dx = c.x - me.x, dyy = c.y - me.y, dzz = c.z - me.z;
            if (dx * dx + dyy * dyy + dzz * dzz < cut2f) {
              const int pos = atomicAdd(&rowlen[a], 1);
              if (pos < KMAX) hit[a * KMAX + pos] = __float_as_int(c.w);
            }
          }
          phase = t - len;
        }
    }
    __syncthreads();
    if (si >= 0) {
      const int32_t i = __float_as_int(cand[si].w);
      const int len = rowlen[a];
      const int c = len < KMAX ? len : KMAX;
      for (int k = l; k < c; k += 4) tmp[(int64_t)i * KMAX + k] = hit[a * KMAX + k];
      if (l == 0) tcnt[i] = len;
    }
    __syncthreads();
  }
}

// Sorts the rows of tmp (row-major, unsorted, tcnt entries) by a fixed
// bitonic network, writes them column-major, and keeps the positions of this
// build.  One lane per atom.
__global__ void __launch_bounds__(BLOCK)
    k_md_rows_finish(int64_t n, const int32_t *__restrict__ tmp, const int32_t *__restrict__ tcnt,
                     const double *__restrict__ x, const double *__restrict__ y,
                     const double *__restrict__ z, int32_t *nj, uint8_t *cnt, double *xr,
                     double *yr, double *zr, DevState *ds, const int *cond) {
  if (cond && *cond == 0) return;
  const int64_t i = xcd_block() * BLOCK + threadIdx.x;
  if (i >= n) return;
  int c = tcnt[i];
  if (c > KMAX) {
    atomicOr(&ds->overflow, 1);
    c = KMAX;
  }
  int32_t v[KMAX];
#pragma unroll
  for (int u = 0; u < KMAX; ++u) v[u] = u < c ? tmp[i * KMAX + u] : INT32_MAX;
#pragma unroll
  for (int k = 2; k <= KMAX; k <<= 1) {
#pragma unroll
    for (int h = k >> 1; h > 0; h >>= 1) {
#pragma unroll
      for (int a = 0; a < KMAX; ++a) {
        const int b = a ^ h;
        if (b > a) {
          const int32_t lo = min(v[a], v[b]), hi = max(v[a], v[b]);
          const bool up = (a & k) == 0;
          v[a] = up ? lo : hi;
          v[b] = up ? hi : lo;
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < KMAX; ++u)
    if (u < c) nj[(int64_t)u * n + i] = v[u];
  cnt[i] = (uint8_t)c;
  xr[i] = x[i];
  yr[i] = y[i];
  zr[i] = z[i];
}

// the list build from filled search bins (super-bins when every axis has at
// least four bins and the staged bins fit in LDS, else one lane per atom)
hipError_t launch_md_build_chain(vcsgc_ctx *c, const Grid &g, const int *cond) {
  const RepHost &r = c->reps[0];
  const double cut = c->pot.rc + c->skin;
  if (g.n0 >= 4 && g.n1 >= 4 && g.n2 >= 4 && c->bmax <= 32) {
    const int nsx = (g.n0 + 1) / 2, nsy = (g.n1 + 1) / 2, nsz = (g.n2 + 1) / 2;
    const float cf = (float)(cut + 1e-3);
    const size_t lds = sizeof(float4) * 64 * (size_t)c->bmax;
    k_build_md_sb<<<(unsigned)((int64_t)nsx * nsy * nsz), BLOCK, lds, c->stream>>>(
        g, nsx, nsy, c->bin_count, c->bin_pos, c->bmax, cf * cf, c->md_tmp, c->md_tcnt, cond);
    k_md_rows_finish<<<grid_for(r.n), BLOCK, 0, c->stream>>>(r.n, c->md_tmp, c->md_tcnt, c->x,
                                                              c->y, c->z, c->md_j, c->md_cnt,
                                                              c->xr, c->yr, c->zr, c->ds, cond);
  } else {
    k_build_md<<<grid_for(r.n), BLOCK, 0, c->stream>>>(r.n, c->x, c->y, c->z, g, c->bin_count,
                                                       c->bin_pos, c->bmax, cut * cut, c->md_j,
                                                       c->md_cnt, c->xr, c->yr, c->zr, c->ds,
                                                       cond);
  }
  return hipGetLastError();
}

// r < rc + skin list (single-system contexts)
hipError_t launch_build_md_list(vcsgc_ctx *c) {
  const RepHost &r = c->reps[0];
  Grid g{r.box[0], r.box[1], r.box[2], r.nb[0], r.nb[1], r.nb[2]};
  hipError_t e = hipMemsetAsync(&c->ds->pairs_md, 0, sizeof(unsigned long long), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(&c->ds->kmax_md, 0, sizeof(int), c->stream);
  if (e != hipSuccess) return e;
  int h = tstart(c, VCSGC_KT_BUILD);
  e = launch_md_build_chain(c, g, nullptr);
  tstop(c, h);
  if (e != hipSuccess) return e;
  k_row_stats<<<512, BLOCK, 0, c->stream>>>(c->n, c->md_cnt, &c->ds->pairs_md, &c->ds->kmax_md,
                                            nullptr);
  return hipGetLastError();
}

// MD list rebuild decided on the device: every kernel of the chain returns
// at once unless the last drift raised ds->rebuild.
// Overflows are flagged as in the host-decided path; the caller checks them
// once at the end of its steps.
hipError_t launch_md_rebuild_cond(vcsgc_ctx *c) {
  const RepHost &r = c->reps[0];
  Grid g{r.box[0], r.box[1], r.box[2], r.nb[0], r.nb[1], r.nb[2]};
  const int *cond = &c->ds->rebuild;
  int h = tstart(c, VCSGC_KT_BUILD);
  k_bins_clear_cond<<<grid_for(r.nbins), BLOCK, 0, c->stream>>>(r.nbins, c->bin_count, c->ds);
  k_bin_search<<<grid_for(r.n), BLOCK, 0, c->stream>>>(r.n, c->x, c->y, c->z, g, c->bmax,
                                                       c->bin_count, c->bin_atoms, c->bin_pos,
                                                       c->ds, cond);
  hipError_t e = launch_md_build_chain(c, g, cond);
  if (e != hipSuccess) return e;
  k_row_stats<<<512, BLOCK, 0, c->stream>>>(c->n, c->md_cnt, &c->ds->pairs_md, &c->ds->kmax_md,
                                            cond);
  k_rebuild_done<<<1, 64, 0, c->stream>>>(c->ds);
  tstop(c, h);
  return hipGetLastError();
}

bool md_rebuild_on_device(const vcsgc_ctx *c) { return c->bin_pos != nullptr; }

// ----------------------------------------------------------------------------
// density cache: rho_i = sum_j t_{s_j} (rc - r_ij)^2, ascending j (row-major MC rows)
// ----------------------------------------------------------------------------
__global__ void k_density_mc(int64_t n, const int32_t *__restrict__ nj,
                             const double *__restrict__ ndd, const uint8_t *__restrict__ cnt,
                             const uint8_t *__restrict__ sp, PotD p, double *rho) {
  const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  const int m = cnt[i];
  for (int k = 0; k < m; ++k) {
    const int32_t j = nj[i * KMAX + k];
    s += p.t[sp[j]] * ndd[i * KMAX + k];
  }
  rho[i] = s;
}

// The r < rc rows taken from a valid r < rc + skin list (MD rows, column-major,
// ascending j): same entries, same order and the same dd, g values as a build
// from the search bins, since r is evaluated by the same expression (the
// packed positions are current whenever the MD list and its densities are).  A group
// of MFM_G lanes per atom: lane l tests entries l, l + MFM_G, ...; the hits of
// a pass are placed by a ballot prefix count, so the row keeps the MD order
// and the stores of a group are contiguous.
constexpr int MFM_G = 16;

__global__ void __launch_bounds__(BLOCK)
    k_mc_from_md(int64_t n, const double4 *__restrict__ ps4, Grid g, const int32_t *__restrict__ mdj,
                 const uint8_t *__restrict__ mdcnt, PotD p, int32_t *nj, double *ndd, double *ng,
                 uint8_t *cnt) {
  const int64_t gid = xcd_block() * BLOCK + threadIdx.x;
  const int64_t i = gid / MFM_G;
  const int l = (int)(gid % MFM_G);
  if (i >= n) return;  // whole groups leave together
  const int wl = threadIdx.x & 63, gb = wl & ~(MFM_G - 1);
  const double4 qi = ps4[i];
  const int m = mdcnt[i];
  int base = 0;
  for (int k0 = 0; k0 < m; k0 += MFM_G) {
    const int k = k0 + l;
    bool hit = false;
    int32_t j = 0;
    double r = 0.0;
    if (k < m) {
      j = mdj[(int64_t)k * n + i];
      const double4 qj = ps4[j];
      const double dx = min_image(qj.x - qi.x, g.L0);
      const double dy = min_image(qj.y - qi.y, g.L1);
      const double dz = min_image(qj.z - qi.z, g.L2);
      r = sqrt((dx * dx + dy * dy) + dz * dz);
      hit = r < p.rc;
    }
    const unsigned long long gm = (__ballot(hit) >> gb) & ((1ull << MFM_G) - 1ull);
    if (hit) {
      const int64_t e = i * KMAX + base + __popcll(gm & ((1ull << l) - 1ull));
      nj[e] = j;
      const double d = p.rc - r;
      ndd[e] = d * d;
      ng[e] = p.c0 + p.c1 * r;
    }
    base += __popcll(gm);
  }
  if (l == 0) cnt[i] = (uint8_t)base;
}

hipError_t launch_mc_from_md(vcsgc_ctx *c) {
  const RepHost &r = c->reps[0];
  Grid g{r.box[0], r.box[1], r.box[2], r.nb[0], r.nb[1], r.nb[2]};
  int h = tstart(c, VCSGC_KT_BUILD);
  k_mc_from_md<<<grid_for(c->n * MFM_G), BLOCK, 0, c->stream>>>(
      c->n, c->ps4, g, c->md_j, c->md_cnt, c->pot, c->mc_j, c->mc_dd, c->mc_g,
      c->mc_cnt);
  tstop(c, h);
  return hipGetLastError();
}

hipError_t launch_density_mc(vcsgc_ctx *c) {
  k_density_mc<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->mc_j, c->mc_dd, c->mc_cnt, c->sp,
                                                        c->pot, c->rho);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// fixed-shape reduction: 256-wide blocks summed by a fixed binary tree, then
// the block sums by the same scheme in one block (deterministic for given n)
// ----------------------------------------------------------------------------
__global__ void k_reduce_blocks(int64_t n, const double *__restrict__ v, double *out) {
  __shared__ double s[BLOCK];
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * BLOCK + t;
  s[t] = i < n ? v[i] : 0.0;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if (t < h) s[t] = s[t] + s[t + h];
    __syncthreads();
  }
  if (t == 0) out[blockIdx.x] = s[0];
}

__global__ void k_reduce_final(int64_t m, const double *__restrict__ part, double *out) {
  __shared__ double s[BLOCK];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int64_t k = t; k < m; k += BLOCK) acc = acc + part[k];
  s[t] = acc;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if (t < h) s[t] = s[t] + s[t + h];
    __syncthreads();
  }
  if (t == 0) *out = s[0];
}

hipError_t launch_reduce_sum(vcsgc_ctx *c, const double *v, int64_t n, double *out_dev) {
  const int nb = grid_for(n);
  k_reduce_blocks<<<nb, BLOCK, 0, c->stream>>>(n, v, c->red);
  k_reduce_final<<<1, BLOCK, 0, c->stream>>>(nb, c->red, out_dev);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// diagnostics
// ----------------------------------------------------------------------------
__global__ void k_sqrt(int64_t n, const double *__restrict__ in, double *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = sqrt(in[i]);
}

hipError_t launch_sqrt(const double *in, double *out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_sqrt<<<grid_for(n), BLOCK, 0, s>>>(n, in, out);
  return hipGetLastError();
}

}  // namespace vc
