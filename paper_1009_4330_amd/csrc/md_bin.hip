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

// Wrap x in place, bin, and count atoms per cell and per super-cell (64
// consecutive cells).  Runs of equal cells inside a wavefront (the common case
// once atoms are cell-sorted) take one atomic per run; with slot != null each
// atom's arrival slot in its cell is written too.  No fence: the counts are
// read by later kernels.
__global__ __launch_bounds__(kBlock) void k_bin_count(double* __restrict__ x, int n, BoxK box,
                                                       int nc0, int nc1, int nc2,
                                                       int* __restrict__ atom_cell,
                                                       int* __restrict__ count,
                                                       int* __restrict__ scount,
                                                       int* __restrict__ slot,
                                                       const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
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
    const int len = min(next, n - (i - lane)) - lane;            // live lanes of this run
    base = atomicAdd(&count[c], len);
    atomicAdd(&scount[c >> kSuperShift], len);
  }
  base = __shfl(base, hl < 0 ? 0 : hl, kWave);
  if (live && slot) slot[i] = base + (lane - hl);
}

// One workgroup: exclusive scan of the per-cell counts into cell_start[0..ncell]
// (each thread a contiguous chunk, loads unrolled).
__global__ __launch_bounds__(kBlock) void k_scan_cells(const int* __restrict__ count, int ncell,
                                                        int* __restrict__ cell_start) {
  __shared__ int sh[kBlock / kWave];
  const int per = (ncell + kBlock - 1) / kBlock;
  const int c0 = min(ncell, (int)threadIdx.x * per), c1 = min(ncell, c0 + per);
  int sum = 0;
#pragma unroll 8
  for (int cc = c0; cc < c1; ++cc) sum += count[cc];
  int tot;
  int run = block_excl_scan(sum, sh, &tot);
#pragma unroll 8
  for (int cc = c0; cc < c1; ++cc) {
    cell_start[cc] = run;
    run += count[cc];
  }
  if (threadIdx.x == 0) cell_start[ncell] = tot;
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

// Wrapped coordinates of the (up to 27) distinct cells around `cell`, one per
// lane 0..26 in z, y, x offset order; *kept is false for lanes >= 27 and for
// offsets that wrap onto an earlier offset's cell (fewer than 3 cells in a
// dimension).
__device__ inline int stencil_lane(int cell, int lane, const int* nc, bool* kept) {
  *kept = false;
  if (lane >= 27) return 0;
  const int o[3] = {lane % 3 - 1, (lane / 3) % 3 - 1, lane / 9 - 1};
  const int home[3] = {cell % nc[0], (cell / nc[0]) % nc[1], cell / (nc[0] * nc[1])};
  int w[3];
  bool k = true;
  for (int d = 0; d < 3; ++d) {
    int v = home[d] + o[d];
    v = v < 0 ? v + nc[d] : (v >= nc[d] ? v - nc[d] : v);
    w[d] = v;
    for (int e = -1; e < o[d]; ++e) {
      int u = home[d] + e;
      u = u < 0 ? u + nc[d] : (u >= nc[d] ? u - nc[d] : u);
      k = k && u != v;
    }
  }
  *kept = k;
  return w[0] + nc[0] * (w[1] + nc[1] * w[2]);
}

// Rebuild-time sort of atoms that are already in the previous build's cell
// order and have moved less than a cell edge since: one wavefront per new
// cell collects its members from the old ranges of the surrounding cells,
// visited in increasing cell index (so in increasing atom index), which is the
// stable counting-sort order without any atomic arrival slots.  The state is
// gathered into the sorted staging buffers.  If fewer members are found than
// were counted (an atom moved further than a cell edge), status bit 2 is set.
// The cell's first slot is the count of all earlier cells, summed from the
// per-super-cell counts before its super-cell plus the counts of the earlier
// cells of its own super-cell; it is written to new_start.
__global__ __launch_bounds__(kBlock) void k_gather_sort(
    const int* __restrict__ old_start, int* __restrict__ new_start,
    const int* __restrict__ count, const int* __restrict__ scount,
    const int* __restrict__ atom_cell, int nc0, int nc1, int nc2, int* __restrict__ perm,
    const double* __restrict__ x, const double* __restrict__ v, const int* __restrict__ id,
    int n, double* __restrict__ sx, double* __restrict__ sv, int* __restrict__ sid,
    int* __restrict__ status, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int cell = (xcd_block() * kBlock + threadIdx.x) / kWave;
  const int ncell = nc0 * nc1 * nc2;
  if (cell >= ncell) return;
  const int nc[3] = {nc0, nc1, nc2};
  bool kept;
  const int c2 = stencil_lane(cell, lane, nc, &kept);
  const int key = kept ? c2 : 0x7fffffff;
  int b = 0, e = 0;
  if (kept) {
    b = old_start[c2];
    e = old_start[c2 + 1];
  }
  int rank = 0;
  for (int q = 0; q < 27; ++q) rank += __shfl(key, q, kWave) < key ? 1 : 0;
  const int nkept = __popcll(__ballot(kept));
  int part = 0;
  const int sc = cell >> kSuperShift;
  for (int q = lane; q < sc; q += kWave) part += scount[q];
  if ((sc << kSuperShift) + lane < cell) part += count[(sc << kSuperShift) + lane];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, kWave);
  const int base = part;
  const int want = count[cell];
  if (lane == 0) {
    new_start[cell] = base;
    if (cell == ncell - 1) new_start[ncell] = base + want;
  }
  const unsigned long long below = (1ull << lane) - 1;
  int found = 0;
  // Take one member candidate (lane-th atom of a range, first 64 atoms of
  // ranges r..r+3 at once so their cell loads overlap), then any tail.
  auto take = [&](int i, bool mine) {
    const unsigned long long m = __ballot(mine);
    if (mine) {
      const int pos = found + __popcll(m & below);
      if (pos < want) {
        const int p = base + pos;
        perm[p] = i;
        sx[p] = x[i];
        sx[n + p] = x[n + i];
        sx[2 * n + p] = x[2 * n + i];
        sv[p] = v[i];
        sv[n + p] = v[n + i];
        sv[2 * n + p] = v[2 * n + i];
        sid[p] = id[i];
      }
    }
    found += __popcll(m);
  };
  constexpr int U = 4;
  for (int r0 = 0; r0 < nkept; r0 += U) {
    int rb[U], re[U], ci[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + u;
      const unsigned long long sel = __ballot(kept && rank == r);
      const int src = sel ? __ffsll((long long)sel) - 1 : 0;
      rb[u] = sel ? __shfl(b, src, kWave) : 0;
      re[u] = sel ? __shfl(e, src, kWave) : 0;
      const int i = rb[u] + lane;
      ci[u] = i < re[u] ? atom_cell[i] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      take(rb[u] + lane, ci[u] == cell);
      for (int t = rb[u] + kWave; t < re[u]; t += kWave) {
        const int i = t + lane;
        take(i, i < re[u] && atom_cell[i] == cell);
      }
    }
  }
  if (lane == 0 && found != want) atomicOr(&status[MD_ST_ERRORS], 4);
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

// Home atoms of one staged chunk: each wavefront takes home atoms in turn and
// tests 64 staged candidates at a time; accepted candidates are appended in
// candidate order through a ballot prefix count.  WRAP applies the minimum
// image (home cells touching a box face).
template <bool WRAP>
__device__ inline void build_home(const BuildArgs& a, const double* cxs, const double* cys,
                                  const double* czs, const int* cjs, int c0, int clen, int hb,
                                  int he, int lane, int wave, unsigned long long below) {
  const int n = a.n;
  const double* __restrict__ x = a.x;
  const bool sorted = a.sorted != 0;
  // layout K = 2^lk lanes per atom: index arithmetic by shifts and masks
  const int lk = __ffs(a.layout) - 1;
  const int gs = 6 - lk;
  const size_t rows = nl_rows(a.cap, a.layout);
  for (int h = hb + wave; h < he; h += kBlock / kWave) {
    const int i = sorted ? h : a.perm[h];
    const double xi = x[i], yi = x[n + i], zi = x[2 * n + i];
    int* __restrict__ row0 =
        a.neigh + (size_t)(i >> gs) * rows * kWave + ((i & ((1 << gs) - 1)) << lk);
    int cnt = c0 == 0 ? 0 : a.numneigh[i];
    for (int t = 0; t < clen; t += kWave) {
      const int q = t + lane;
      bool take = false;
      int j = 0;
      if (q < clen) {
        j = cjs[q];
        double dx = xi - cxs[q], dy = yi - cys[q], dz = zi - czs[q];
        if (WRAP) {
          dx = min_image(dx, a.box.L[0], a.box.inv[0]);
          dy = min_image(dy, a.box.L[1], a.box.inv[1]);
          dz = min_image(dz, a.box.L[2], a.box.inv[2]);
        }
        const double r2 = dx * dx + dy * dy + dz * dz;
        take = (j != i) && (r2 < a.rl2);
      }
      const unsigned long long m = __ballot(take);
      if (take) {
        const int pos = cnt + __popcll(m & below);
        if (pos < a.cap) row0[(size_t)(pos >> lk) * kWave + (pos & ((1 << lk) - 1))] = j;
      }
      cnt += __popcll(m);
    }
    if (lane == 0) a.numneigh[i] = cnt;
  }
}

// One workgroup per cell.  The candidates -- atoms of the (up to) 27
// surrounding cells, in cell order and slot order inside a cell -- are staged
// in LDS in chunks; each wavefront takes home atoms in turn and tests 64
// candidates at a time, appending accepted ones in candidate order through a
// ballot prefix count.  r^2 = (dx dx + dy dy) + dz dz < rl^2 exactly as the
// FP64 definition.  Status words get one atomic per workgroup.
__global__ __launch_bounds__(kBlock) void k_build(BuildArgs a) {
  if (a.gate && *a.gate == 0) return;
  const int cell = xcd_block();
  __shared__ double cxs[kBuildChunk], cys[kBuildChunk], czs[kBuildChunk];
  __shared__ int cjs[kBuildChunk];
  __shared__ int st_start[27], st_cnt[27], st_off[28], st_n;
  __shared__ int red[kBlock / kWave];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int n = a.n;
  const double* __restrict__ x = a.x;
  const bool sorted = a.sorted != 0;
  if (cell == 0 && tid == 0) atomicAdd(&a.status[MD_ST_BUILDS], 1);
  if (wave == 0) {
    // Stencil entry (oz, oy, ox) = lane, all 27 looked up at once; the kept
    // entries keep the z, y, x offset order of the FP64 definition.
    bool kept;
    const int c2 = stencil_lane(cell, lane, a.nc, &kept);
    const unsigned long long km = __ballot(kept);
    if (kept) {
      const int pos = __popcll(km & ((1ull << lane) - 1));
      const int b = a.cell_start[c2];
      st_start[pos] = b;
      st_cnt[pos] = a.cell_start[c2 + 1] - b;
    }
    if (lane == 0) st_n = __popcll(km);
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int q = 0; q < st_n; ++q) {
      st_off[q] = acc;
      acc += st_cnt[q];
    }
    st_off[st_n] = acc;
  }
  __syncthreads();
  const int total = st_off[st_n];
  const int hb = a.cell_start[cell], he = a.cell_start[cell + 1];
  // A home cell at least one cell away from every box face (with >= 3 cells
  // per dimension) has an unwrapped stencil: candidate and home positions are
  // wrapped into [0, L) and at most two cell edges apart, so an accepted pair
  // has rint(d / L) = 0 and d = x_i - x_j is the FP64 minimum image bit for bit,
  // while any other image is at least L / 3 >= r_l away.
  bool wrap = false;
  {
    const int home[3] = {cell % a.nc[0], (cell / a.nc[0]) % a.nc[1],
                         cell / (a.nc[0] * a.nc[1])};
    for (int d = 0; d < 3; ++d)
      wrap = wrap || a.nc[d] < 3 || home[d] == 0 || home[d] == a.nc[d] - 1;
  }
  if (tid == 0) {
    if (a.cell_start_out) {
      a.cell_start_out[cell] = hb;
      if (cell == (int)gridDim.x - 1) a.cell_start_out[cell + 1] = he;
    }
    // the binning counters have been consumed: clear them for the next rebuild
    if (a.count_clear) a.count_clear[cell] = 0;
    if (a.scount_clear && (cell & ((1 << kSuperShift) - 1)) == 0)
      a.scount_clear[cell >> kSuperShift] = 0;
  }
  const unsigned long long below = (1ull << lane) - 1;
  for (int c0 = 0; c0 < total; c0 += kBuildChunk) {
    const int clen = min(kBuildChunk, total - c0);
    for (int q = tid; q < clen; q += kBlock) {
      const int idx = c0 + q;
      int sc = 0;
      while (idx >= st_off[sc + 1]) ++sc;
      const int sl = st_start[sc] + (idx - st_off[sc]);
      const int j = sorted ? sl : a.perm[sl];
      cjs[q] = j;
      cxs[q] = x[j];
      cys[q] = x[n + j];
      czs[q] = x[2 * n + j];
    }
    __syncthreads();
    if (wrap)
      build_home<true>(a, cxs, cys, czs, cjs, c0, clen, hb, he, lane, wave, below);
    else
      build_home<false>(a, cxs, cys, czs, cjs, c0, clen, hb, he, lane, wave, below);
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
    // one device-scope atomic per workgroup at most: skipped when the word
    // already holds at least m (a stale read only costs an extra atomic)
    if (m > 0 && m > __hip_atomic_load(&a.status[MD_ST_MAXNEIGH], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&a.status[MD_ST_MAXNEIGH], m);
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
                            int* count, int* scount, int* slot, const int* gate, hipStream_t s) {
  k_bin_count<<<blocks_for(n), kBlock, 0, s>>>(x, n, box, nc[0], nc[1], nc[2], atom_cell, count,
                                                scount, slot, gate);
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

hipError_t launch_gather_sort(const int* old_start, int* new_start, const int* count,
                              const int* scount, const int* atom_cell, const int nc[3],
                              int* perm, const double* x, const double* v, const int* id, int n,
                              double* sx, double* sv, int* sid, int* status, const int* gate,
                              hipStream_t s) {
  const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
  k_gather_sort<<<blocks_for(ncell * kWave), kBlock, 0, s>>>(
      old_start, new_start, count, scount, atom_cell, nc[0], nc[1], nc[2], perm, x, v, id, n, sx,
      sv, sid, status, gate);
  return hipGetLastError();
}

hipError_t launch_scan_cells(const int* count, int ncell, int* cell_start, hipStream_t s) {
  k_scan_cells<<<1, kBlock, 0, s>>>(count, ncell, cell_start);
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
