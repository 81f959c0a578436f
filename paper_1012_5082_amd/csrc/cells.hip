// Link cells and neighbour lists (Sec. III.A: cells of edge >= the
// independence distance, an even number per dimension so that cells whose
// index parities agree are a full cell edge apart), the density cache of the
// sweep, input validation and a fixed-shape FP64 reduction.
#include <algorithm>

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
// the lane's old value plus its rank among the lanes with the same key.  The
// lanes are first grouped by key (ballots only); then the first lane of every
// group adds the group's size, all groups at once, so the wave waits for one
// round of atomics rather than one per distinct key.
__device__ __forceinline__ int32_t wave_add_one(int32_t *counter, int key) {
  const int lane = __lane_id();
  unsigned long long todo = __ballot(1);
  int leader_of = lane, rank = 0, size = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lkey = __shfl(key, leader);
    const unsigned long long same = __ballot(key == lkey) & todo;
    if (same & (1ull << lane)) {
      leader_of = leader;
      rank = (int)__popcll(same & ((1ull << lane) - 1ull));
    }
    if (lane == leader) size = (int)__popcll(same);
    todo &= ~same;
  }
  int32_t base = 0;
  if (lane == leader_of) base = atomicAdd(&counter[key], (int32_t)size);
  base = __shfl(base, leader_of);
  return base + (int32_t)rank;
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
// ----------------------------------------------------------------------------
// grown domains: in cells of edge e, eight cubic domains of edge e - r_dep,
// one per corner (bit d of the corner k: the low interval [0, e - r_dep) or
// the high one [e - (e - r_dep), e) along axis d, in coordinates from the
// cell's corner).  Per (cell c, corner k) at q = 8 c + k: the atoms of the
// domain in ascending index and the inclusive sums of their weights 8 / m,
// m the number of the cell's domains holding the atom.
// ----------------------------------------------------------------------------
struct GrownGeo {
  double L0, L1, L2, r_dep;
  int n0, n1, n2;
};

// domain bits (2d: low interval of axis d, 2d + 1: high one) and weight
__device__ __forceinline__ int grown_bits(double px, double py, double pz, const GrownGeo &g,
                                          int &w) {
  const double pos[3] = {px, py, pz}, L[3] = {g.L0, g.L1, g.L2};
  const int nc[3] = {g.n0, g.n1, g.n2};
  int bits = 0, m = 1;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double e = L[d] / (double)nc[d];
    const double ld = e - g.r_dep;
    const int b = cell_coord(pos[d], L[d], nc[d]);
    const double u = pos[d] - (double)b * e;
    const int lo = u < ld, hi = u >= e - ld;
    bits |= (lo << (2 * d)) | (hi << (2 * d + 1));
    m *= lo + hi;
  }
  w = 8 / m;
  return bits;
}

// One wave per cell, 64 of its atoms (ascending index) at a time: every lane
// takes one atom's domain bits and weight, and per corner a ballot ranks the
// members and a wave scan sums their weights.  FILL false writes the
// domains' counts to cnt[8 c + k]; FILL true writes the lists from start[q].
constexpr int GROWN_WAVES = BLOCK / 64;

template <bool FILL>
__global__ void __launch_bounds__(BLOCK)
    k_grown_lists(int64_t ncells, const int32_t *__restrict__ cstart,
                  const int32_t *__restrict__ catoms, const double *__restrict__ x,
                  const double *__restrict__ y, const double *__restrict__ z, GrownGeo g,
                  int32_t *cnt, const int32_t *__restrict__ start, int32_t *list, int32_t *cum) {
  const int64_t c = (int64_t)blockIdx.x * GROWN_WAVES + threadIdx.x / 64;
  if (c >= ncells) return;  // whole waves leave together
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  int32_t off[8], run[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    off[k] = FILL ? start[8 * c + k] : 0;
    run[k] = 0;
  }
  const int32_t lo = cstart[c], hi = cstart[c + 1];
  for (int32_t j0 = lo; j0 < hi; j0 += 64) {
    const int32_t j = j0 + lane;
    int bits = 0, w = 0, i = 0;
    if (j < hi) {
      i = catoms[j];
      bits = grown_bits(x[i], y[i], z[i], g, w);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool in = ((bits >> (k & 1)) & 1) && ((bits >> (2 + ((k >> 1) & 1))) & 1) &&
                      ((bits >> (4 + ((k >> 2) & 1))) & 1);
      const unsigned long long mask = __ballot(in);
      if (FILL) {
        // inclusive sum of the members' weights over the lanes up to this one
        int v = in ? w : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const int u = __shfl_up(v, d, 64);
          if (lane >= d) v += u;
        }
        if (in) {
          const int32_t o = off[k] + (int32_t)__popcll(mask & below);
          list[o] = i;
          cum[o] = run[k] + v;
        }
        run[k] += __shfl(v, 63, 64);
      }
      off[k] += (int32_t)__popcll(mask);
    }
  }
  if (!FILL && lane < 8) {
    int32_t v = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) v = lane == k ? off[k] : v;
    cnt[8 * c + lane] = v;
  }
}

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
  if (c->grown) {  // single-system contexts only
    GrownGeo gg{r.box[0], r.box[1], r.box[2], c->r_dep, r.nc[0], r.nc[1], r.nc[2]};
    const int64_t nq = 8 * r.ncells;
    const unsigned gb = (unsigned)((r.ncells + GROWN_WAVES - 1) / GROWN_WAVES);
    k_grown_lists<false><<<gb, BLOCK, 0, c->stream>>>(r.ncells, start, atoms, x, y, z, gg,
                                                      c->g_cnt, nullptr, nullptr, nullptr);
    const int nch = (int)((nq + SCAN_CHUNK - 1) / SCAN_CHUNK);
    k_scan_sums<<<nch, 256, 0, c->stream>>>(nq, c->g_cnt, c->scan_tmp, INT32_MAX, nullptr);
    k_scan_apply<<<nch, 256, 0, c->stream>>>(nq, c->g_cnt, c->scan_tmp, c->g_start, nullptr,
                                             INT32_MAX, nullptr);
    k_grown_lists<true><<<gb, BLOCK, 0, c->stream>>>(r.ncells, start, atoms, x, y, z, gg,
                                                     nullptr, c->g_start, c->g_list, c->g_cum);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// search bins: edge >= rc + skin, at most bmax atoms each (overflow flagged)
// ----------------------------------------------------------------------------
// Grid-stride over the atoms (one atomic per distinct bin in a wave).
// cond (may be NULL): run only when *cond != 0 (device-decided MD rebuild);
// such a run also zeroes the MD row statistics that the list build then
// accumulates.  pos (may be NULL) receives (x, y, z, i) of the atom in its slot.
__global__ void k_bin_search(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                             const double *__restrict__ z, Grid g, int bmax, int32_t *count,
                             int32_t *atoms, double4 *pos, DevState *ds, const int *cond) {
  if (cond && *cond == 0) return;
  if (cond && blockIdx.x == 0 && threadIdx.x == 0) {
    ds->pairs_md = 0ull;
    ds->kmax_md = 0;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double a = x[i], b2 = y[i], c2 = z[i];
    const int b = cell_of(g, a, b2, c2);
    const int slot = wave_add_one(count, b);
    if (slot < bmax) {
      atoms[(int64_t)b * bmax + slot] = (int32_t)i;
      if (pos) pos[(int64_t)b * bmax + slot] = make_double4(a, b2, c2, (double)i);
    } else {
      atomicOr(&ds->bin_overflow, 1);
    }
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

// ----------------------------------------------------------------------------
// neighbour lists from the search bins.  Every pair with r < cutoff, r from
// the minimum-image separation as sqrt((dx^2 + dy^2) + dz^2), rows sorted by
// neighbour index.  Row-major rows: entry k of atom i at [i * KMAX + k],
// with the neighbour's index and r (its users form (rc - r)^2 and c0 + c1 r
// from r).
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

// MODE 1: MC rows, 2: descriptor rows (both keep r)
template <int MODE>
__global__ void __launch_bounds__(BLOCK)
    k_build(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
            const double *__restrict__ z, Grid g, const int32_t *__restrict__ bcount,
            const int32_t *__restrict__ batoms, int bmax, double cutoff, PotD p, int32_t *nj,
            double *nr, uint8_t *cnt, DevState *ds, int64_t aoff) {
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
      nr[e] = pair_r(x, y, z, g, xi, yi, zi, j);
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
      c->bin_atoms + r.boff * c->bmax, c->bmax, c->pot.rc, c->pot, c->mc_j, c->mc_r,
      c->mc_cnt, c->ds, r.aoff);
  tstop(c, h);
  return hipGetLastError();
}

// r < 4.41 A descriptor list of one replica (row-major, with distances)
hipError_t launch_build_desc_list(vcsgc_ctx *c, const RepHost &r) {
  Grid g{r.box[0], r.box[1], r.box[2], r.nb[0], r.nb[1], r.nb[2]};
  k_build<2><<<grid_for(r.n * BG), BLOCK, 0, c->stream>>>(
      r.n, c->x + r.aoff, c->y + r.aoff, c->z + r.aoff, g, c->bin_count + r.boff,
      c->bin_atoms + r.boff * c->bmax, c->bmax, DESC_CUT, c->pot, c->d_j, c->d_r,
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

// Row statistics of a list (entries, longest row, overflow) of the block:
// reduced in the block, then one atomic each into sum, mx and (when set)
// ovf_flag.  Every thread of the block calls it, after its last use of LDS.
__device__ __forceinline__ void block_row_stats(long long pairs, int kmx, bool ovf,
                                                unsigned long long *sum, int *mx, int *ovf_flag) {
  __shared__ long long sp[BLOCK / 64];
  __shared__ int sk[BLOCK / 64], so[BLOCK / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    pairs += __shfl_xor(pairs, off);
    const int o = __shfl_xor(kmx, off);
    kmx = o > kmx ? o : kmx;
  }
  const int any_ovf = __ballot(ovf) != 0ull ? 1 : 0;
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sp[wv] = pairs;
    sk[wv] = kmx;
    so[wv] = any_ovf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tp = 0;
    int tk = 0, to = 0;
    for (int q = 0; q < BLOCK / 64; ++q) {
      tp += sp[q];
      tk = sk[q] > tk ? sk[q] : tk;
      to |= so[q];
    }
    if (tp) atomicAdd(sum, (unsigned long long)tp);
    if (tk) atomicMax(mx, tk);
    if (to && ovf_flag) atomicOr(ovf_flag, 1);
  }
}

__device__ __forceinline__ void md_row_stats(long long pairs, int kmx, bool ovf, DevState *ds) {
  block_row_stats(pairs, kmx, ovf, &ds->pairs_md, &ds->kmax_md, &ds->overflow);
}

// v[0 .. KMAX) sorted ascending in place by a fixed bitonic network (static
// register indices throughout).
__device__ __forceinline__ void sort_row(int32_t (&v)[KMAX]) {
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
}

// r < rc + skin list, one lane per atom (used when some axis has fewer than
// four search bins): the lane walks the surrounding search bins through the
// packed (x, y, z, index) slots and appends hits to its row; INT32_MAX fills
// the rest of the row.  The test is r^2 < cut2: the list only has to hold
// every pair that can come within rc before the next rebuild (its users test
// r < rc themselves).  Row-major rows [i * KMAX + k], unsorted (k_md_finish
// then sorts them into the column-major list and writes the row lengths and
// the positions of this build).
// cond (may be NULL): run only when *cond != 0 (and count the rebuild).
__global__ void __launch_bounds__(BLOCK)
    k_build_md(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
               const double *__restrict__ z, Grid g, const int32_t *__restrict__ bcount,
               const double4 *__restrict__ bpos, int bmax, double cut2, int32_t *nj, DevState *ds,
               const int *cond) {
  if (cond && *cond == 0) return;
  if (cond && blockIdx.x == 0 && threadIdx.x == 0) ds->md_rebuilds += 1ull;
  const int64_t i = xcd_block() * BLOCK + threadIdx.x;
  int c = 0;
  if (i < n) {
    const double xi = x[i], yi = y[i], zi = z[i];
    const int bx = cell_coord(xi, g.L0, g.n0), by = cell_coord(yi, g.L1, g.n1),
              bz = cell_coord(zi, g.L2, g.n2);
    const int n0 = g.n0 >= 3 ? 3 : 2, n1 = g.n1 >= 3 ? 3 : 2, n2 = g.n2 >= 3 ? 3 : 2;
    const int s0 = g.n0 >= 3 ? -1 : 0, s1 = g.n1 >= 3 ? -1 : 0, s2 = g.n2 >= 3 ? -1 : 0;
    int32_t *row = nj + i * KMAX;
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
            for (int u = 0; u < 4; ++u)
              q[u] = t + u < m ? slot[t + u] : make_double4(0, 0, 0, -1.0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int32_t j = (int32_t)q[u].w;
              if (t + u < m && j != (int32_t)i) {
                const double dx = min_image(q[u].x - xi, g.L0);
                const double dy = min_image(q[u].y - yi, g.L1);
                const double dz = min_image(q[u].z - zi, g.L2);
                if ((dx * dx + dy * dy) + dz * dz < cut2) {
                  if (c < KMAX) row[c] = j;
                  ++c;
                }
              }
            }
          }
        }
      }
    }
    for (int u = c; u < KMAX; ++u) row[u] = INT32_MAX;
  }
  md_row_stats(c < KMAX ? c : KMAX, c < KMAX ? c : KMAX, c > KMAX, ds);
}

// Block barrier for LDS traffic only: the fences are restricted to LDS, so
// the barrier waits for this wave's LDS accesses but not for its global
// loads and stores.
__device__ __forceinline__ void block_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Exclusive scans over the block of two per-thread values (one value per
// thread; BLOCK / 64 waves); returns the block totals.  Contains barriers:
// every thread of the block calls it.
__device__ __forceinline__ int2 block_scan2(int &a, int &b, int2 *wtot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int va = a, vb = b;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int ta = __shfl_up(va, d), tb = __shfl_up(vb, d);
    if (lane >= d) {
      va += ta;
      vb += tb;
    }
  }
  if (lane == 63) wtot[wv] = make_int2(va, vb);
  block_sync_lds();
  int ba = 0, bb = 0, sa = 0, sb = 0;
#pragma unroll
  for (int q = 0; q < BLOCK / 64; ++q) {
    const int2 t = wtot[q];
    if (q < wv) {
      ba += t.x;
      bb += t.y;
    }
    sa += t.x;
    sb += t.y;
  }
  a = ba + va - a;
  b = bb + vb - b;
  block_sync_lds();  // wtot may be written again after this
  return make_int2(sa, sb);
}

// r < rc + skin list by regions of 4 x 4 x RZ search bins (every axis needs at
// least four bins).  For each of its regions a block stages the 6 x 6 x
// (RZ + 2) bins around it in LDS: positions relative to the region origin in
// float, periodic images resolved, each bin's atoms contiguous (at most CAP
// staged atoms: a denser region raises the bin-overflow flag, which has the
// bins grown to the next capacity, whose kernel stages every slot).  One lane
// per own atom then walks the atom's 27 neighbouring bins (nine runs of three
// staged bins consecutive in x) and notes the staged index of each hit in its
// own LDS column; at the end it stores the whole row of its hits' atom
// indices (row-major, unsorted, INT32_MAX after the last hit) in 16-byte
// pieces, so that every line of a row is written at once.  The float test uses
// cut2f = (cut + 1e-3)^2, a superset of r < cut (the float rounding of the
// relative coordinates stays below 1e-4 A); users of the list test r < rc in
// FP64 themselves.  Grid-stride: the blocks on XCD x (blockIdx mod 8 == x;
// the grid is a multiple of 8) take the x-th eighth of the regions, so
// neighbouring regions share that XCD's L2.  BMAX is the bin capacity.
// cond (may be NULL): run only when *cond != 0 (and count the rebuild).
constexpr int RG_X = 4, RG_Y = 4;  // own bins of a region along x and y
constexpr int RG_GRID = 2048;      // blocks of a region launch (at most)

template <int BMAX, int RZ, int CAP>
__global__ void __launch_bounds__(BLOCK)
    k_md_search(Grid g, int nrx, int nry, int64_t nreg, const int32_t *__restrict__ bcount,
                const double4 *__restrict__ bpos, float cut2f, int32_t *rows, DevState *ds,
                const int *cond) {
  constexpr int SX = RG_X + 2, SY = RG_Y + 2, SZ = RZ + 2, NST = SX * SY * SZ;
  constexpr int OWN_CAP = RG_X * RG_Y * RZ * BMAX;
  static_assert(NST <= BLOCK && NST <= 256, "one thread per staged bin, bin ids in a byte");
  static_assert(CAP <= NST * BMAX && CAP + 3 <= 65536, "staged indices in 16 bits");
  if (cond && *cond == 0) return;
  if (cond && blockIdx.x == 0 && threadIdx.x == 0) ds->md_rebuilds += 1ull;
  __shared__ float4 cand[CAP + 3];  // + 3: the search reads up to 3 past a run
  __shared__ int off[NST + 1];
  __shared__ int gbin[NST];
  __shared__ char4 shc[NST];                // periodic image of staged bin u: -1, 0, +1 per axis
  __shared__ int own_si[OWN_CAP];           // staged index of own atom q
  __shared__ unsigned char own_b[OWN_CAP];  // staged bin of own atom q
  __shared__ int own_off[NST];
  // column t: staged indices of lane t's hits, its own atom among them; the
  // slot after the last hit takes every later candidate, so with KMAX
  // neighbours (KMAX + 1 hits) that slot is row KMAX + 1, past the last hit
  __shared__ unsigned short hit[KMAX + 2][BLOCK];
  __shared__ int2 wtot[BLOCK / 64];
  const int tid = threadIdx.x;
  const int xcd = (int)(blockIdx.x & 7u);
  const int64_t per_xcd = gridDim.x >> 3;
  const int64_t lo = nreg * xcd / 8, hi = nreg * (xcd + 1) / 8;
  const double bw0 = g.L0 / g.n0, bw1 = g.L1 / g.n1, bw2 = g.L2 / g.n2;
  long long pairs = 0;
  int kmx = 0;
  bool ovf = false;
  for (int64_t rg = lo + (int64_t)(blockIdx.x >> 3); rg < hi; rg += per_xcd) {
    const int rx = (int)(rg % nrx), ry = (int)((rg / nrx) % nry),
              rz = (int)(rg / ((int64_t)nrx * nry));
    const double o0 = (RG_X * rx) * bw0, o1 = (RG_Y * ry) * bw1, o2 = (RZ * rz) * bw2;
    // staged bin tid: global bin, image shift, occupancy, own or not
    int cn = 0, ocn = 0;
    if (tid < NST) {
      const int ux = tid % SX, uy = (tid / SX) % SY, uz = tid / (SX * SY);
      int gx = RG_X * rx - 1 + ux, gy = RG_Y * ry - 1 + uy, gz = RZ * rz - 1 + uz;
      const bool own = ux >= 1 && ux <= RG_X && uy >= 1 && uy <= RG_Y && uz >= 1 && uz <= RZ &&
                       gx < g.n0 && gy < g.n1 && gz < g.n2;
      signed char hx = 0, hy = 0, hz = 0;
      if (gx < 0) { gx += g.n0; hx = -1; } else if (gx >= g.n0) { gx -= g.n0; hx = 1; }
      if (gy < 0) { gy += g.n1; hy = -1; } else if (gy >= g.n1) { gy -= g.n1; hy = 1; }
      if (gz < 0) { gz += g.n2; hz = -1; } else if (gz >= g.n2) { gz -= g.n2; hz = 1; }
      const int b = gx + g.n0 * (gy + g.n1 * gz);
      cn = min(bcount[b], BMAX);
      ocn = own ? cn : 0;
      gbin[tid] = b;
      shc[tid] = make_char4(hx, hy, hz, 0);
    }
    block_sync_lds();  // the previous region's readers of off / cand are done
    int os = cn, oo = ocn;
    const int2 tot = block_scan2(os, oo, wtot);
    if (tot.x > CAP) {  // uniform over the block
      if (tid == 0) atomicOr(&ds->bin_overflow, 1);
      continue;
    }
    if (tid < NST) {
      off[tid] = os;
      own_off[tid] = oo;
    }
    if (tid == 0) off[NST] = tot.x;
    block_sync_lds();
    // stage: staged atom c of bin u (off[u] <= c < off[u + 1]); two in flight
    // (four raised the kernel past 128 registers, to three waves per SIMD)
#pragma unroll 1
    for (int c0 = 0; c0 < tot.x; c0 += 2 * BLOCK) {
      double4 p[2];
      int uu[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int c = c0 + k * BLOCK + tid;
        uu[k] = -1;
        if (c < tot.x) {
          int lo_u = 0, hi_u = NST;  // off[lo_u] <= c < off[hi_u]
          while (hi_u - lo_u > 1) {
            const int mid = (lo_u + hi_u) >> 1;
            if (off[mid] <= c) lo_u = mid; else hi_u = mid;
          }
          uu[k] = lo_u;
          p[k] = bpos[(int64_t)gbin[lo_u] * BMAX + (c - off[lo_u])];
        }
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int u = uu[k];
        if (u >= 0) {
          const int c = c0 + k * BLOCK + tid;
          const char4 h = shc[u];
          // the image shift is exactly -L, 0 or +L
          cand[c] = make_float4((float)(p[k].x + h.x * g.L0 - o0),
                                (float)(p[k].y + h.y * g.L1 - o1),
                                (float)(p[k].z + h.z * g.L2 - o2), __int_as_float((int32_t)p[k].w));
          const int ub = u % SX, vb = (u / SX) % SY, wb = u / (SX * SY);
          if (ub >= 1 && ub <= RG_X && vb >= 1 && vb <= RG_Y && wb >= 1 && wb <= RZ &&
              own_off[u] < (u + 1 < NST ? own_off[u + 1] : tot.y)) {
            const int q = own_off[u] + (c - off[u]);
            own_si[q] = c;
            own_b[q] = (unsigned char)u;
          }
        }
      }
    }
    block_sync_lds();
    // search: one lane per own atom
    for (int q = tid; q < tot.y; q += BLOCK) {
      const int si = own_si[q], u = own_b[q];
      const float4 me = cand[si];
      const int32_t i = __float_as_int(me.w);
      const int lx = u % SX, ly = (u / SX) % SY, lz = u / (SX * SY);
      // every candidate's index goes to slot c, which advances on a hit (no
      // branch per candidate); the atom itself (d2 = 0) is one of the hits
      int c = 0;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
          const int u0 = (lx - 1) + SX * ((ly + dy) + SY * (lz + dz));
          const int a1 = off[u0 + 3];
          // four candidates in flight (at most three read past the run)
#pragma unroll 1
          for (int k0 = off[u0]; k0 < a1; k0 += 4) {
            float4 cc[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) cc[v] = cand[k0 + v];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const float dx = cc[v].x - me.x, dyy = cc[v].y - me.y, dzz = cc[v].z - me.z;
              const float d2 = __builtin_fmaf(dzz, dzz, __builtin_fmaf(dyy, dyy, dx * dx));
              hit[min(c, KMAX + 1)][tid] = (unsigned short)(k0 + v);
              c += (k0 + v < a1 && d2 < cut2f) ? 1 : 0;
            }
          }
        }
      // c - 1 neighbours; the atom's own slot is skipped by taking the last
      // stored slot in its place (the own slot is the last one, or the last
      // one lies beyond the entries read)
      const int nb = c - 1, cc = nb < KMAX ? nb : KMAX;
      const int last = hit[min(c - 1, KMAX + 1)][tid];
#pragma unroll
      for (int u = 0; u < KMAX; u += 4) {
        int32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          int sk = hit[u + k][tid];
          sk = sk == si ? last : sk;
          w[k] = u + k < cc ? __float_as_int(cand[min(sk, CAP - 1)].w) : INT32_MAX;
        }
        *(int4 *)(rows + (int64_t)i * KMAX + u) = make_int4(w[0], w[1], w[2], w[3]);
      }
      pairs += cc;
      kmx = nb > kmx ? nb : kmx;
      ovf = ovf || nb > KMAX;
    }
  }
  md_row_stats(pairs, kmx < KMAX ? kmx : KMAX, ovf, ds);
}

// The rows written by the search (row-major [i * KMAX + k], unsorted,
// INT32_MAX after the last entry) sorted into the column-major list
// [k * n + i] of the lane-per-atom MD passes, with the row lengths and the
// positions of this build (the search ran at the current positions).  One
// lane per atom: the row's 16-byte pieces into registers, a fixed sorting
// network, then the entries before the padding stored column-major
// (consecutive atoms, consecutive addresses).  Grid-stride; cond (may be
// NULL): run only when *cond != 0.
constexpr int FIN_GRID = 4096;

__global__ void __launch_bounds__(BLOCK)
    k_md_finish(int64_t n, const int32_t *__restrict__ rows, const double *__restrict__ x,
                const double *__restrict__ y, const double *__restrict__ z, int32_t *nj,
                uint8_t *cnt, double *xr, double *yr, double *zr, const int *cond) {
  if (cond && *cond == 0) return;
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = xcd_block() * BLOCK + threadIdx.x; i < n; i += stride) {
    int32_t v[KMAX];
#pragma unroll
    for (int u = 0; u < KMAX; u += 4) {
      const int4 q = *(const int4 *)(rows + i * KMAX + u);
      v[u] = q.x;
      v[u + 1] = q.y;
      v[u + 2] = q.z;
      v[u + 3] = q.w;
    }
    sort_row(v);
    int m = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (v[k] != INT32_MAX) nj[(int64_t)k * n + i] = v[k];
      m += v[k] != INT32_MAX ? 1 : 0;
    }
    cnt[i] = (uint8_t)m;
    xr[i] = x[i];
    yr[i] = y[i];
    zr[i] = z[i];
  }
}

// the list build from filled search bins (regions when every axis has at
// least four bins and a bin holds at most 32 atoms, else one lane per atom),
// then the column-major rows, their lengths and the positions of the build
hipError_t launch_md_build_chain(vcsgc_ctx *c, const Grid &g, const int *cond) {
  const RepHost &r = c->reps[0];
  const double cut = c->pot.rc + c->skin;
  if (g.n0 >= 4 && g.n1 >= 4 && g.n2 >= 4 && (c->bmax == 16 || c->bmax == 32)) {
    const float cf = (float)(cut + 1e-3);
    const int nrx = (g.n0 + RG_X - 1) / RG_X, nry = (g.n1 + RG_Y - 1) / RG_Y;
    const int rz = c->bmax == 16 ? 2 : 1;
    const int nrz = (g.n2 + rz - 1) / rz;
    const int64_t nreg = (int64_t)nrx * nry * nrz;
    const unsigned G = (unsigned)std::min<int64_t>((nreg + 7) / 8 * 8, RG_GRID);
    // 16-slot bins: up to eight staged atoms per bin on average (a denser
    // region has the bins grown); 32-slot bins: every slot
    if (c->bmax == 16)
      k_md_search<16, 2, 6 * 6 * 4 * 8><<<G, BLOCK, 0, c->stream>>>(
          g, nrx, nry, nreg, c->bin_count, c->bin_pos, cf * cf, c->md_rows, c->ds, cond);
    else
      k_md_search<32, 1, 6 * 6 * 3 * 32><<<G, BLOCK, 0, c->stream>>>(
          g, nrx, nry, nreg, c->bin_count, c->bin_pos, cf * cf, c->md_rows, c->ds, cond);
  } else {
    k_build_md<<<grid_for(r.n), BLOCK, 0, c->stream>>>(r.n, c->x, c->y, c->z, g, c->bin_count,
                                                       c->bin_pos, c->bmax, cut * cut,
                                                       c->md_rows, c->ds, cond);
  }
  const unsigned GF = (unsigned)std::min<int64_t>((r.n + BLOCK - 1) / BLOCK, FIN_GRID);
  k_md_finish<<<GF, BLOCK, 0, c->stream>>>(r.n, c->md_rows, c->x, c->y, c->z, c->md_j, c->md_cnt,
                                           c->xr, c->yr, c->zr, cond);
  return hipGetLastError();
}

// r < rc + skin list (single-system contexts), from bins already filled
hipError_t launch_build_md_list(vcsgc_ctx *c) {
  const RepHost &r = c->reps[0];
  Grid g{r.box[0], r.box[1], r.box[2], r.nb[0], r.nb[1], r.nb[2]};
  hipError_t e = hipMemsetAsync(&c->ds->pairs_md, 0, sizeof(unsigned long long), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(&c->ds->kmax_md, 0, sizeof(int), c->stream);
  if (e != hipSuccess) return e;
  int h = tstart(c, VCSGC_KT_BUILD);
  e = launch_md_build_chain(c, g, nullptr);
  tstop(c, h);
  return e;
}

// MD list rebuild decided on the device, for step parity par: every kernel
// returns at once unless the last drift raised ds->rebuild[par].  The bin
// counts were cleared by that drift.  Overflows are flagged as in the
// host-decided path; the caller checks them once at the end of its steps.
constexpr int BIN_GRID = 2048;  // blocks of a device-decided binning (at most)

hipError_t launch_md_rebuild_cond(vcsgc_ctx *c, int par) {
  const RepHost &r = c->reps[0];
  Grid g{r.box[0], r.box[1], r.box[2], r.nb[0], r.nb[1], r.nb[2]};
  const int *cond = &c->ds->rebuild[par];
  int h = tstart(c, VCSGC_KT_BUILD);
  k_bin_search<<<std::min(grid_for(r.n), BIN_GRID), BLOCK, 0, c->stream>>>(
      r.n, c->x, c->y, c->z, g, c->bmax, c->bin_count, c->bin_atoms, c->bin_pos, c->ds, cond);
  hipError_t e = launch_md_build_chain(c, g, cond);
  tstop(c, h);
  return e;
}

bool md_rebuild_on_device(const vcsgc_ctx *c) { return c->bin_pos != nullptr; }

// ----------------------------------------------------------------------------
// density cache: rho_i = sum_j f_{s_j}(r_ij), ascending j (row-major MC rows)
// ----------------------------------------------------------------------------
__global__ void k_density_mc(int64_t n, const int32_t *__restrict__ nj,
                             const double *__restrict__ nr, const uint8_t *__restrict__ cnt,
                             const uint8_t *__restrict__ sp, PotD p, double *rho) {
  const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  const int m = cnt[i];
  for (int k = 0; k < m; ++k) {
    const int32_t j = nj[i * KMAX + k];
    s += pot_f(p, sp[j], nr[i * KMAX + k]);
  }
  rho[i] = s;
}

// The r < rc rows taken from a valid r < rc + skin list (the column-major MD
// list, ascending j): same entries, same order and the same r values as a
// build from the search bins, since r is evaluated by the same expression
// (the packed positions are current whenever the MD list and its densities
// are).  A group of MFM_G lanes per atom: lane l tests entries l, l + MFM_G,
// ...; the hits of a pass are placed by a ballot prefix count, so the row
// keeps the MD order and the stores of a group are contiguous.  An index
// load of a wave covers MFM_G entries of 64 / MFM_G consecutive atoms.
constexpr int MFM_G = 8;  // measured per sweep: 16 lanes 1% and 4 lanes 12% slower

__global__ void __launch_bounds__(BLOCK)
    k_mc_from_md(int64_t n, const double4 *__restrict__ ps4, Grid g, const int32_t *__restrict__ mdj,
                 const uint8_t *__restrict__ mdcnt, PotD p, int32_t *nj, double *nr,
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
      nr[e] = r;
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
      c->n, c->ps4, g, c->md_j, c->md_cnt, c->pot, c->mc_j, c->mc_r, c->mc_cnt);
  tstop(c, h);
  return hipGetLastError();
}

hipError_t launch_density_mc(vcsgc_ctx *c) {
  k_density_mc<<<grid_for(c->n), BLOCK, 0, c->stream>>>(c->n, c->mc_j, c->mc_r, c->mc_cnt, c->sp,
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

__global__ void k_md_math(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                          double *sq, double *q) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    sq[i] = sqrt_md(a[i]);
    q[i] = div_md(a[i], b[i]);
  }
}

hipError_t launch_md_math(const double *a, const double *b, double *sq, double *q, int64_t n,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_md_math<<<grid_for(n), BLOCK, 0, s>>>(n, a, b, sq, q);
  return hipGetLastError();
}

}  // namespace vc
