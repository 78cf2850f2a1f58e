// Cell binning, stable counting sort, atom reordering and the full Verlet
// list build (the cell machinery of the paper's section "Cell list approach",
// used here only to find neighbours; the list itself is what the kernels of
// its "Neighbor list approach" read).
#include "md_internal.hpp"

namespace md {
namespace {

constexpr int kBuildChunk = 1024;   // candidates staged in LDS per pass (32 KB)

__global__ __launch_bounds__(kBlock) void k_fill_int(int* __restrict__ p, int64_t count,
                                                      int value) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) p[i] = value;
}

// Wrap one coordinate into [0, L): x - L floor(x / L), an exact L mapped to 0.
__device__ inline double wrap_coord(double x, double L) {
  double r = x - L * floor(x / L);
  if (r < 0.0) r += L;
  if (r >= L) r = 0.0;
  return r;
}

__device__ inline int cell_coord(double r, int nc, double L) {
  int c = (int)((r * (double)nc) / L);
  return c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
}

// Exclusive scan of one int per thread over a 256-thread block; *total gets
// the block sum.  sh holds 4 ints.
__device__ inline int block_excl_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  int x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  if (lane == kWave - 1) sh[wave] = x;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    before += w < wave ? sh[w] : 0;
    tot += sh[w];
  }
  __syncthreads();
  *total = tot;
  return x - v + before;
}

// Wrap x in place, bin, and count atoms per cell.  Runs of equal cells inside
// a wavefront (the common case once atoms are cell-sorted) take one atomic per
// run; each atom's arrival slot in its cell is written to slot[].  The last
// workgroup to finish turns the counts into cell_start (exclusive scan) and
// clears the counters and the ticket for the next use.
__global__ __launch_bounds__(kBlock) void k_bin_count(double* __restrict__ x, int n, BoxK box,
                                                       int nc0, int nc1, int nc2,
                                                       int* __restrict__ atom_cell,
                                                       int* __restrict__ count,
                                                       int* __restrict__ slot,
                                                       int* __restrict__ cell_start,
                                                       int* __restrict__ ticket,
                                                       const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int sh[kBlock / kWave];
  __shared__ int is_last;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const bool live = i < n;
  int c = -1;
  if (live) {
    const double rx = wrap_coord(x[i], box.L[0]);
    const double ry = wrap_coord(x[n + i], box.L[1]);
    const double rz = wrap_coord(x[2 * n + i], box.L[2]);
    x[i] = rx;
    x[n + i] = ry;
    x[2 * n + i] = rz;
    c = cell_coord(rx, nc0, box.L[0]) +
        nc0 * (cell_coord(ry, nc1, box.L[1]) + nc1 * cell_coord(rz, nc2, box.L[2]));
    atom_cell[i] = c;
  }
  // runs of equal cell ids among consecutive lanes
  const int prev = __shfl_up(c, 1, kWave);
  const bool head = live && (lane == 0 || prev != c);
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  const int hl = 63 - __clzll(heads & upto);                       // my run's head lane
  const unsigned long long after = heads & ~upto;                  // heads above me
  const int next = after ? __ffsll((long long)after) - 1 : kWave;  // next run's head
  int base = 0;
  if (head) {
    const int live_end = min(next, n - (i - lane));              // lanes of this run that are live
    base = atomicAdd(&count[c], live_end - lane);
  }
  base = __shfl(base, hl < 0 ? 0 : hl, kWave);
  if (live) slot[i] = base + (lane - hl);

  // last workgroup: scan
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(ticket, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  const int ncell = nc0 * nc1 * nc2;
  volatile int* vcount = count;
  int carry = 0;
  for (int t0 = 0; t0 < ncell; t0 += kBlock) {
    const int cc = t0 + (int)threadIdx.x;
    const int v = cc < ncell ? vcount[cc] : 0;
    int tot;
    const int ex = block_excl_scan(v, sh, &tot);
    if (cc < ncell) {
      cell_start[cc] = carry + ex;
      count[cc] = 0;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    cell_start[ncell] = carry;
    *ticket = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter(const int* __restrict__ atom_cell,
                                                     const int* __restrict__ slot,
                                                     const int* __restrict__ cell_start, int n,
                                                     int* __restrict__ tmp_perm,
                                                     const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  tmp_perm[cell_start[atom_cell[i]] + slot[i]] = i;
}

// One wavefront per cell.  The atomic arrival order is replaced by the rank of
// each atom index among the cell's members, which is the stable counting-sort
// order.  Cells hold tens to a few hundred atoms, so the O(cnt^2 / 64) rank
// count per cell is cheap and needs no scratch.
__global__ __launch_bounds__(kBlock) void k_cell_sort(
    const int* __restrict__ tmp_perm, const int* __restrict__ cell_start, int ncell,
    int* __restrict__ perm, const double* __restrict__ x, const double* __restrict__ v,
    const int* __restrict__ id, const double* __restrict__ f, int n, double* __restrict__ sx,
    double* __restrict__ sv, int* __restrict__ sid, double* __restrict__ sf,
    const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int cell = (blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (cell >= ncell) return;
  const int b = cell_start[cell];
  const int cnt = cell_start[cell + 1] - b;
  for (int q = lane; q < cnt; q += kWave) {
    const int key = tmp_perm[b + q];
    int rank = 0;
    for (int r = 0; r < cnt; ++r) rank += tmp_perm[b + r] < key ? 1 : 0;
    const int p = b + rank;
    perm[p] = key;
    if (sx) {
      sx[p] = x[key];
      sx[n + p] = x[n + key];
      sx[2 * n + p] = x[2 * n + key];
    }
    if (sv) {
      sv[p] = v[key];
      sv[n + p] = v[n + key];
      sv[2 * n + p] = v[2 * n + key];
    }
    if (sid) sid[p] = id[key];
    if (sf) {
      sf[p] = f[key];
      sf[n + p] = f[n + key];
      sf[2 * n + p] = f[2 * n + key];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_copy_back(double* __restrict__ x,
                                                       double* __restrict__ v,
                                                       int* __restrict__ id,
                                                       double* __restrict__ f,
                                                       double* __restrict__ xr,
                                                       const double* __restrict__ sx,
                                                       const double* __restrict__ sv,
                                                       const int* __restrict__ sid,
                                                       const double* __restrict__ sf, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int d = 0; d < 3; ++d) {
    x[d * n + i] = sx[d * n + i];
    if (v) v[d * n + i] = sv[d * n + i];
    if (f) f[d * n + i] = sf[d * n + i];
    if (xr) xr[d * n + i] = sx[d * n + i];
  }
  if (id) id[i] = sid[i];
}

__global__ __launch_bounds__(kBlock) void k_gather3(const int* __restrict__ perm, int n,
                                                     const double* __restrict__ src,
                                                     double* __restrict__ dst) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const int q = perm[p];
  dst[p] = src[q];
  dst[n + p] = src[n + q];
  dst[2 * n + p] = src[2 * n + q];
}

__global__ __launch_bounds__(kBlock) void k_gather_int(const int* __restrict__ perm, int n,
                                                        const int* __restrict__ src,
                                                        int* __restrict__ dst) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p < n) dst[p] = src[perm[p]];
}

// Distinct neighbour cells along one dimension: c-1, c, c+1 (mod nc) in that
// order, duplicates dropped (nc < 3).
__device__ inline int stencil1(int c, int nc, int* out) {
  int k = 0;
  for (int o = -1; o <= 1; ++o) {
    int v = c + o;
    v = v < 0 ? v + nc : (v >= nc ? v - nc : v);
    bool dup = false;
    for (int q = 0; q < k; ++q) dup |= out[q] == v;
    if (!dup) out[k++] = v;
  }
  return k;
}

// Minimum image d - L rint(d / L); the image index is taken from d * (1/L),
// which selects the same image as d / L except within rounding of |d| = L/2,
// a separation never inside the list radius because L > 2 rl.
__device__ inline double min_image(double d, double L, double inv) {
  return d - L * rint(d * inv);
}

__device__ inline int wave_max(int v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
  return v;
}

// One workgroup per cell.  The candidates -- atoms of the (up to) 27
// surrounding cells, in cell order and slot order inside a cell -- are staged
// in LDS in chunks; each wavefront takes home atoms in turn and tests 64
// candidates at a time, appending accepted ones in candidate order through a
// ballot prefix count.  r^2 = (dx dx + dy dy) + dz dz < rl^2 exactly as the
// FP64 definition.  Status words get one atomic per workgroup.
__global__ __launch_bounds__(kBlock) void k_build(BuildArgs a) {
  if (a.gate && *a.gate == 0) return;
  __shared__ double cxs[kBuildChunk], cys[kBuildChunk], czs[kBuildChunk];
  __shared__ int cjs[kBuildChunk];
  __shared__ int st_start[27], st_cnt[27], st_n;
  __shared__ int red[kBlock / kWave];
  const int cell = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int n = a.n;
  const double* __restrict__ x = a.x;
  const bool sorted = a.sorted != 0;
  if (cell == 0 && tid == 0) atomicAdd(&a.status[MD_ST_BUILDS], 1);
  if (tid == 0) {
    const int cx = cell % a.nc[0], cy = (cell / a.nc[0]) % a.nc[1];
    const int cz = cell / (a.nc[0] * a.nc[1]);
    int ox[3], oy[3], oz[3];
    const int kx = stencil1(cx, a.nc[0], ox), ky = stencil1(cy, a.nc[1], oy),
              kz = stencil1(cz, a.nc[2], oz);
    int q = 0;
    for (int p = 0; p < kz; ++p)
      for (int r = 0; r < ky; ++r)
        for (int s = 0; s < kx; ++s) {
          const int c2 = ox[s] + a.nc[0] * (oy[r] + a.nc[1] * oz[p]);
          st_start[q] = a.cell_start[c2];
          st_cnt[q] = a.cell_start[c2 + 1] - st_start[q];
          ++q;
        }
    st_n = q;
  }
  __syncthreads();
  int total = 0;
  for (int q = 0; q < st_n; ++q) total += st_cnt[q];
  const int hb = a.cell_start[cell], he = a.cell_start[cell + 1];
  const unsigned long long below = (1ull << lane) - 1;
  for (int c0 = 0; c0 < total; c0 += kBuildChunk) {
    const int clen = min(kBuildChunk, total - c0);
    for (int q = tid; q < clen; q += kBlock) {
      int idx = c0 + q, sc = 0;
      while (idx >= st_cnt[sc]) idx -= st_cnt[sc++];
      const int sl = st_start[sc] + idx;
      const int j = sorted ? sl : a.perm[sl];
      cjs[q] = j;
      cxs[q] = x[j];
      cys[q] = x[n + j];
      czs[q] = x[2 * n + j];
    }
    __syncthreads();
    for (int h = hb + wave; h < he; h += kBlock / kWave) {
      const int i = sorted ? h : a.perm[h];
      const double xi = x[i], yi = x[n + i], zi = x[2 * n + i];
      int cnt = c0 == 0 ? 0 : a.numneigh[i];
      for (int t = 0; t < clen; t += kWave) {
        const int q = t + lane;
        bool take = false;
        int j = 0;
        if (q < clen) {
          j = cjs[q];
          const double dx = min_image(xi - cxs[q], a.box.L[0], a.box.inv[0]);
          const double dy = min_image(yi - cys[q], a.box.L[1], a.box.inv[1]);
          const double dz = min_image(zi - czs[q], a.box.L[2], a.box.inv[2]);
          const double r2 = dx * dx + dy * dy + dz * dz;
          take = (j != i) && (r2 < a.rl2);
        }
        const unsigned long long m = __ballot(take);
        if (take) {
          const int pos = cnt + __popcll(m & below);
          if (pos < a.cap) a.neigh[nl_index(i, pos, a.cap, a.layout)] = j;
        }
        cnt += __popcll(m);
      }
      if (lane == 0) a.numneigh[i] = cnt;
    }
    __syncthreads();
  }
  // per-atom bookkeeping of the home atoms (after every wave has written numneigh)
  int mx = 0;
  for (int h = hb + tid; h < he; h += kBlock) {
    const int i = sorted ? h : a.perm[h];
    mx = max(mx, a.numneigh[i]);
    const double xi = x[i], yi = x[n + i], zi = x[2 * n + i];
    if (a.x_ref) {
      a.x_ref[i] = xi;
      a.x_ref[n + i] = yi;
      a.x_ref[2 * n + i] = zi;
    }
    if (a.x_out) {
      a.x_out[i] = xi;
      a.x_out[n + i] = yi;
      a.x_out[2 * n + i] = zi;
      a.v_out[i] = a.v_in[i];
      a.v_out[n + i] = a.v_in[n + i];
      a.v_out[2 * n + i] = a.v_in[2 * n + i];
      a.id_out[i] = a.id_in[i];
    }
  }
  mx = wave_max(mx);
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  if (tid == 0) {
    int m = red[0];
    for (int w = 1; w < kBlock / kWave; ++w) m = max(m, red[w]);
    if (m > 0) atomicMax(&a.status[MD_ST_MAXNEIGH], m);
    if (m > a.cap) atomicOr(&a.status[MD_ST_ERRORS], 1);
  }
}

inline unsigned blocks_for(int64_t n, int per = kBlock) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_fill_int(int* p, int64_t count, int value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_fill_int<<<blocks_for(count), kBlock, 0, s>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_bin_count(double* x, int n, BoxK box, const int nc[3], int* atom_cell,
                            int* count, int* slot, int* cell_start, int* ticket,
                            const int* gate, hipStream_t s) {
  k_bin_count<<<blocks_for(n), kBlock, 0, s>>>(x, n, box, nc[0], nc[1], nc[2], atom_cell, count,
                                                slot, cell_start, ticket, gate);
  return hipGetLastError();
}

hipError_t launch_scatter(const int* atom_cell, const int* slot, const int* cell_start, int n,
                          int* tmp_perm, const int* gate, hipStream_t s) {
  k_scatter<<<blocks_for(n), kBlock, 0, s>>>(atom_cell, slot, cell_start, n, tmp_perm, gate);
  return hipGetLastError();
}

hipError_t launch_cell_sort(const int* tmp_perm, const int* cell_start, int ncell, int* perm,
                            const double* x, const double* v, const int* id, const double* f,
                            int n, double* sx, double* sv, int* sid, double* sf,
                            const int* gate, hipStream_t s) {
  k_cell_sort<<<blocks_for((int64_t)ncell * kWave), kBlock, 0, s>>>(
      tmp_perm, cell_start, ncell, perm, x, v, id, f, n, sx, sv, sid, sf, gate);
  return hipGetLastError();
}

hipError_t launch_copy_back(double* x, double* v, int* id, double* f, double* xr,
                            const double* sx, const double* sv, const int* sid,
                            const double* sf, int n, hipStream_t s) {
  k_copy_back<<<blocks_for(n), kBlock, 0, s>>>(x, v, id, f, xr, sx, sv, sid, sf, n);
  return hipGetLastError();
}

hipError_t launch_gather3(const int* perm, int n, const double* src, double* dst,
                          hipStream_t s) {
  k_gather3<<<blocks_for(n), kBlock, 0, s>>>(perm, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_gather_int(const int* perm, int n, const int* src, int* dst, hipStream_t s) {
  k_gather_int<<<blocks_for(n), kBlock, 0, s>>>(perm, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_build(const BuildArgs& a, hipStream_t s) {
  const unsigned ncell = (unsigned)(a.nc[0] * a.nc[1] * a.nc[2]);
  k_build<<<ncell, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace md
