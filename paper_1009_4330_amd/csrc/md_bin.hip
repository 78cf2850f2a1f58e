// Cell binning, stable counting sort, atom reordering and the full Verlet
// list build (the cell machinery of the paper's section "Cell list approach",
// used here only to find neighbours; the list itself is what the kernels of
// its "Neighbor list approach" read).
#include <algorithm>
#include <climits>
#include <cmath>

#include "md_internal.hpp"

namespace md {
namespace {


__global__ __launch_bounds__(kBlock) void k_fill_int(int* __restrict__ p, int64_t count,
                                                      int value) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) p[i] = value;
}

__global__ __launch_bounds__(kBlock) void k_fill_double(double* __restrict__ p, int64_t count,
                                                         double value) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) p[i] = value;
}

// Half list from a full one, in place: thread i walks its row in order and
// keeps the partners j > i at the front (a kept entry never lands past the
// entry being read, so the walk reads only entries not yet overwritten).
__global__ __launch_bounds__(kBlock) void k_halve(int* __restrict__ neigh,
                                                   int* __restrict__ numneigh, int n, int cap,
                                                   int layout) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int cnt = min(numneigh[i], cap);
  int kept = 0;
  for (int m = 0; m < cnt; ++m) {
    const int j = neigh[nl_index(i, m, cap, layout)];
    if (j > i) neigh[nl_index(i, kept++, cap, layout)] = j;
  }
  numneigh[i] = kept;
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

// Wrap x in place, bin, and count atoms per cell; each atom's arrival slot in
// its cell is recorded for the scatter.  Runs of equal cells inside a
// wavefront (the common case once atoms are cell-sorted) take one atomic per
// run.
__global__ __launch_bounds__(kBlock) void k_bin_count(double* __restrict__ x, int n, BoxK box,
                                                       int nc0, int nc1, int nc2,
                                                       int* __restrict__ atom_cell,
                                                       int* __restrict__ count,
                                                       int* __restrict__ slot) {
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
  }
  base = __shfl(base, hl < 0 ? 0 : hl, kWave);
  if (live) slot[i] = base + (lane - hl);
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
    const int* __restrict__ id, const double* __restrict__ f, const int* __restrict__ type,
    int n, double* __restrict__ sx, double* __restrict__ sv, int* __restrict__ sid,
    double* __restrict__ sf, int* __restrict__ stype, const int* __restrict__ gate) {
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
    if (stype) stype[p] = type[key];
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


// The same cells along x as runs of consecutive cells: [*a, *b) for run k of
// the returned count (1, or 2 when the stencil wraps around the box).
__device__ inline int x_runs(int c, int nc) { return nc >= 3 && (c == 0 || c == nc - 1) ? 2 : 1; }
__device__ inline void x_run(int c, int nc, int k, int* a, int* b) {
  if (nc < 3) {
    *a = 0;
    *b = nc;
  } else if (c == 0) {
    *a = k == 0 ? 0 : nc - 1;
    *b = k == 0 ? 2 : nc;
  } else if (c == nc - 1) {
    *a = k == 0 ? 0 : nc - 2;
    *b = k == 0 ? 1 : nc;
  } else {
    *a = c - 1;
    *b = c + 2;
  }
}

// The previous build's atoms around a cell as contiguous segments: each (z, y)
// row of the 3x3x3 stencil is one or two runs of consecutive cells, whose
// atoms are contiguous in the previous cell order.  Lane s < n holds segment
// s's range [b, b + len); segments come in increasing cell index, so visiting
// s = 0, 1, ... visits the atoms in increasing index (the previous order).
constexpr int kMaxSegs = 18;
struct Segs {
  int b, len;
  int n;       // segments (wave-uniform, at most 18)
  bool fits;   // every segment holds at most 128 atoms (wave-uniform)
};

__device__ inline Segs old_segments(int cell, int lane, const int* nc,
                                    const int* __restrict__ old_start) {
  const int cx = cell % nc[0], cy = (cell / nc[0]) % nc[1], cz = cell / (nc[0] * nc[1]);
  const int nxs = x_runs(cx, nc[0]), ny = min(nc[1], 3), nz = min(nc[2], 3);
  Segs S;
  S.n = nxs * ny * nz;
  S.b = 0;
  S.len = 0;
  if (lane < S.n) {
    const int xr = lane % nxs, yr = (lane / nxs) % ny, zr = lane / (nxs * ny);
    int xa, xb;
    x_run(cx, nc[0], xr, &xa, &xb);
    const int row = (nbr_sorted(cz, nc[2], zr) * nc[1] + nbr_sorted(cy, nc[1], yr)) * nc[0];
    S.b = old_start[row + xa];
    S.len = old_start[row + xb] - S.b;
  }
  S.fits = __ballot(S.len > 2 * kWave) == 0;
  return S;
}

// Short segments (S.fits): the new cell of atoms b + lane and b + 64 + lane of
// every segment, all loads in flight together; -1 past a segment's end.
__device__ inline void seg_cells(const Segs& S, int lane, const int* __restrict__ atom_cell,
                                 int (*cid)[2], int* sb) {
#pragma unroll
  for (int q = 0; q < kMaxSegs; ++q) {
    int b = 0, len = 0;
    if (q < S.n) {
      b = __builtin_amdgcn_readlane(S.b, q);
      len = __builtin_amdgcn_readlane(S.len, q);
    }
    sb[q] = b;
    cid[q][0] = lane < len ? atom_cell[b + lane] : -1;
    cid[q][1] = lane + kWave < len ? atom_cell[b + kWave + lane] : -1;
  }
}

// The rebuild sort's super-cells (consecutive cells in the cell order, one
// wavefront each) and its workgroup.
constexpr int kSortCells = 16;
constexpr int kSortBlock = kWave * kSortCells;

// Gather member i into sorted slot p: its position from the packed records
// (wrapped into the box), velocity and id from the state.
__device__ inline void put_member(int i, int p, int n, const BoxK& box,
                                  const double* __restrict__ xq, const double* __restrict__ v,
                                  const int* __restrict__ id, const int* __restrict__ type,
                                  int* __restrict__ perm, double* __restrict__ sx,
                                  double* __restrict__ sv, int* __restrict__ sid,
                                  int* __restrict__ stype) {
  const double2 q = *reinterpret_cast<const double2*>(xq + 4 * (size_t)i);
  const double x2 = xq[4 * (size_t)i + 2];
  const double v0 = v[i], v1 = v[n + i], v2 = v[2 * n + i];
  const int idi = id[i];
  perm[p] = i;
  sx[p] = wrap_coord(q.x, box.L[0]);
  sx[n + p] = wrap_coord(q.y, box.L[1]);
  sx[2 * n + p] = wrap_coord(x2, box.L[2]);
  sv[p] = v0;
  sv[n + p] = v1;
  sv[2 * n + p] = v2;
  sid[p] = idi;
  if (stype) stype[p] = type[i];
}

// Members of new cell `cell` among the previous build's atoms around it, in
// increasing atom index (the previous order, so the stable counting-sort
// order, with no atomic arrival slots), gathered into sorted slots
// base .. base + want - 1.  With short segments (S.fits) the candidates' new
// cells are the registers cid / sb that seg_cells filled; otherwise they are
// read again.  Fewer or more members than want sets status bit 2.
__device__ inline void gather_members(const Segs& S, const int (*cid)[2], const int* sb,
                                      const int* __restrict__ atom_cell, int cell, int base,
                                      int want, const BoxK& box, int* __restrict__ perm,
                                      const double* __restrict__ xq, const double* __restrict__ v,
                                      const int* __restrict__ id, const int* __restrict__ type,
                                      int n, double* __restrict__ sx, double* __restrict__ sv,
                                      int* __restrict__ sid, int* __restrict__ stype,
                                      int* __restrict__ status, int lane, int* row) {
  const unsigned long long below = (1ull << lane) - 1;
  int found = 0;
  if (S.fits && want <= kWave) {
    // member indices in order into this wave's LDS row, then one gather
#pragma unroll
    for (int q = 0; q < kMaxSegs; ++q) {
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const bool mine = cid[q][hh] == cell;
        const unsigned long long m = __ballot(mine);
        const int pos = found + __popcll(m & below);
        if (mine && pos < kWave) row[pos] = sb[q] + hh * kWave + lane;
        found += __popcll(m);
      }
    }
    __builtin_amdgcn_wave_barrier();   // a wavefront's LDS accesses complete in order
    if (lane < want && lane < found)
      put_member(row[lane], base + lane, n, box, xq, v, id, type, perm, sx, sv, sid, stype);
  } else {
    for (int q = 0; q < S.n; ++q) {
      const int b = __builtin_amdgcn_readlane(S.b, q);
      const int len = __builtin_amdgcn_readlane(S.len, q);
      for (int t = 0; t < len; t += kWave) {
        const int i = b + t + lane;
        const bool mine = t + lane < len && atom_cell[i] == cell;
        const unsigned long long m = __ballot(mine);
        const int pos = found + __popcll(m & below);
        if (mine && pos < want)
          put_member(i, base + pos, n, box, xq, v, id, type, perm, sx, sv, sid, stype);
        found += __popcll(m);
      }
    }
  }
  if (lane == 0 && found != want) atomicOr(&status[MD_ST_ERRORS], 4);
}

// Look-back words of the rebuild sort, one per super-cell: the flag in the
// top two bits (0: nothing yet, 1: the super-cell's total, 2: its inclusive
// prefix) and the value in the low 32.  After them: the ticket counter and
// the count of workgroups that have finished their walk.
constexpr unsigned long long kLbTotal = 1ull << 62, kLbPrefix = 2ull << 62;
constexpr int kLbSpinLimit = 1 << 18;   // sleeps before a wait gives up (about 0.1 s)

// Rebuild-time sort of atoms that are already in the previous build's cell
// order and have moved less than a cell edge since, in one launch: one
// workgroup of kSortCells wavefronts per super-cell of as many consecutive
// cells, the super-cells taken in order from a ticket counter.  Each wavefront counts its new cell's
// members among the previous ranges of the 27 cells around it (keeping the
// candidates' new cells in registers); the first wavefront publishes the
// super-cell's total and adds the totals before it by a decoupled look-back:
// walking down the earlier super-cells 64 at a time (one per lane), the
// nearest published inclusive prefix ends the walk, published totals are
// added and the walk goes on.  A workgroup waits only on
// super-cells whose tickets were taken before its own, by workgroups already
// running, so every wait ends; each wait is bounded all the same, and giving
// up sets status bit 2.  Then every wavefront writes its cell's start and
// gathers the state into the sorted staging buffers (positions wrapped into
// the box).  The last workgroup to finish its walk clears the words and both
// counters for the next rebuild (they start zeroed: launch_sort_clear).
// Status bit 2 is also set if the counts do not add up to n (an atom moved
// further than a cell edge).
// Built for eight waves per SIMD (two workgroups per CU; the compiler's
// choice, 106 SGPRs, left room for one): the working pass takes 33.9 instead
// of 36.5 us on the 256k melt, its SGPR spills going to VGPR lanes.
__global__ __launch_bounds__(kSortBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_sort_cells(
    const int* __restrict__ old_start, int* __restrict__ new_start,
    const int* __restrict__ atom_cell, int nc0, int nc1, int nc2, BoxK box0,
    const double* __restrict__ boxd, int* __restrict__ perm, const double* __restrict__ xq,
    const double* __restrict__ v, const int* __restrict__ id, const int* __restrict__ type, int n,
    double* __restrict__ sx, double* __restrict__ sv, int* __restrict__ sid,
    int* __restrict__ stype, int* __restrict__ status, unsigned long long* __restrict__ lb,
    const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int part[kSortCells];
  __shared__ int rows[kSortCells * kWave];
  __shared__ int sh_sc, sh_pre, sh_last;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int ncell = nc0 * nc1 * nc2;
  const int nsuper = (ncell + kSortCells - 1) / kSortCells;
  unsigned* const ticket = reinterpret_cast<unsigned*>(lb + nsuper);
  unsigned* const done = reinterpret_cast<unsigned*>(lb + nsuper + 1);
  if (threadIdx.x == 0) sh_sc = (int)atomicAdd(ticket, 1u);
  __syncthreads();
  const int sc = sh_sc;
  const int nc[3] = {nc0, nc1, nc2};
  const int cell = __builtin_amdgcn_readfirstlane(sc * kSortCells + wave);
  const bool live = cell < ncell;
  Segs S{};
  int cid[kMaxSegs][2], sb[kMaxSegs];
  int cnt = 0;
  if (live) {
    S = old_segments(cell, lane, nc, old_start);
    if (S.fits) {
      seg_cells(S, lane, atom_cell, cid, sb);
#pragma unroll
      for (int q = 0; q < kMaxSegs; ++q)
        cnt += __popcll(__ballot(cid[q][0] == cell)) + __popcll(__ballot(cid[q][1] == cell));
    } else {
      for (int q = 0; q < S.n; ++q) {
        const int b = __builtin_amdgcn_readlane(S.b, q);
        const int len = __builtin_amdgcn_readlane(S.len, q);
        for (int t = 0; t < len; t += kWave)
          cnt += __popcll(__ballot(t + lane < len && atom_cell[b + t + lane] == cell));
      }
    }
  }
  if (lane == 0) part[wave] = cnt;
  __syncthreads();
  if (wave == 0) {
    int tot = 0;
#pragma unroll
    for (int w = 0; w < kSortCells; ++w) tot += part[w];
    if (lane == 0)
      __hip_atomic_store(lb + sc, kLbTotal | (unsigned)tot, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    // the walk, 64 super-cells per step: lane l reads super-cell top - l (the
    // box's start, below super-cell 0, reads as a prefix of 0) until every
    // lane has a word; the nearest prefix ends the walk, else all 64 totals
    // are added and the walk moves 64 further down
    int pre = 0;
    bool ok = true;
    for (int top = sc - 1; top >= 0 && ok; top -= kWave) {
      const int j = top - lane;
      unsigned long long w = j >= 0 ? 0 : kLbPrefix;
      for (int spin = 0;; ++spin) {
        if (j >= 0 && (w >> 62) == 0)
          w = __hip_atomic_load(lb + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__ballot((w >> 62) == 0) == 0) break;
        if (spin == kLbSpinLimit) {
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      const unsigned long long pm = __ballot((w >> 62) == 2);
      // lanes up to and including the nearest prefix (all 64 if none)
      const int upto = pm ? __builtin_ctzll(pm) : kWave - 1;
      int val = lane <= upto ? (int)(unsigned)w : 0;
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) val += __shfl_xor(val, off, kWave);
      pre += val;
      if (pm) break;
    }
    if (lane == 0) {
      if (!ok) atomicOr(&status[MD_ST_ERRORS], 4);
      __hip_atomic_store(lb + sc, kLbPrefix | (unsigned)(pre + tot), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      sh_pre = pre;
      sh_last = atomicAdd(done, 1u) == (unsigned)(nsuper - 1);
    }
  }
  __syncthreads();
  if (sh_last) {
    // every walk has ended: nothing reads the words any more
    for (int k = threadIdx.x; k < nsuper + 2; k += kSortBlock) lb[k] = 0;
  }
  if (!live) return;
  int base = sh_pre;
  for (int w = 0; w < wave; ++w) base += part[w];
  if (lane == 0) {
    new_start[cell] = base;
    if (cell == ncell - 1) {
      new_start[ncell] = base + cnt;
      if (base + cnt != n) atomicOr(&status[MD_ST_ERRORS], 4);
    }
  }
  const BoxK box = boxd ? box_load(boxd) : box0;
  gather_members(S, cid, sb, atom_cell, cell, base, cnt, box, perm, xq, v, id, type, n, sx, sv,
                 sid, stype, status, lane, rows + wave * kWave);
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

// Append candidate j at position pos of the list whose first row starts at
// row0 (K = 2^lk lanes per atom: entry pos sits in row pos / K, column pos % K).
__device__ inline void put_entry(int* __restrict__ row0, int pos, int lk, int j) {
  row0[((pos >> lk) << 6) + (pos & ((1 << lk) - 1))] = j;
}

// put_entry as a relaxed atomic store: the same global store, but an
// operation the compiler does not merge with the LDS stores it sits beside
// (a merged store would go through a flat pointer).
__device__ inline void put_entry_apart(int* __restrict__ row0, int pos, int lk, int j) {
  __hip_atomic_store(row0 + ((pos >> lk) << 6) + (pos & ((1 << lk) - 1)), j, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// LDS of the list-build kernels.
constexpr int kListBuf = 128;   // buffered list entries per home atom and pass
constexpr int kListRow = 2 * kListBuf + kWave;   // per wavefront: two buffers and a sink row
struct BuildLds {
  double* cxs;   // staged candidates: positions and indices
  double* cys;
  double* czs;
  int* cjs;
  int* hcnt;     // [kBlock] list lengths of the current cell's first 256 home atoms
  int* lbuf;     // [waves][kListRow] accepted entries of a wavefront's two home atoms
};

// Where one pass finds its candidates: LDS slots [base[s], base[s] + pad[s]) of
// each of n segments, every segment padded to a multiple of 64 with entries
// that are never accepted (NaN position, index -1).
struct CandSegs {
  int base[3];
  int pad[3];
  int n;
};

// Home atoms of one pass, two at a time per wavefront: every candidate of the
// pass (64 at a time) is tested against both, and accepted ones are appended
// in candidate order through a ballot prefix count -- into the wavefront's
// LDS buffer (anything past kListBuf straight to the list), copied into the
// list layout when the atom's pass is done.  WRAP applies the minimum image
// (home cells touching a box face).  HOME_LDS: the home atoms are staged at
// LDS slots hl, hl + 1, ...; otherwise their positions are read from x (one
// address space per instantiation, so no access goes through a flat
// pointer, which would make LDS waits wait for global memory too).  FIRST:
// the lists start empty, else they continue from hcnt / numneigh.  Each home
// atom's count goes to numneigh and, for the first 256, to hcnt.
template <bool WRAP, bool HOME_LDS, bool FIRST>
__device__ inline void build_home(const BuildArgs& a, const BuildLds& L, const CandSegs& cs,
                                  int hl, int hb, int he, int lane, int wave) {
  const int n = a.n;
  const double* __restrict__ x = a.x;
  const bool sorted = a.sorted != 0;
  const double nan = __builtin_nan("");
  // layout K = 2^lk lanes per atom: index arithmetic by shifts and masks
  const int lk = __ffs(a.layout) - 1;
  const int gs = 6 - lk;
  const size_t rows = nl_rows(a.cap, a.layout);
  const double rl2 = a.rl2;
  // this wavefront's LDS row: buffer of atom 0, buffer of atom 1, then one
  // sink slot per lane where rejected candidates land
  int* __restrict__ lrow = L.lbuf + wave * kListRow;
  const int sink = 2 * kListBuf + lane;
  for (int h = __builtin_amdgcn_readfirstlane(hb + 2 * wave); h < he;
       h += 2 * (kBlock / kWave)) {
    const bool two = h + 1 < he;
    const int i0 = sorted ? h : a.perm[h];
    const int i1 = two ? (sorted ? h + 1 : a.perm[h + 1]) : -1;
    const int k1 = two ? i1 : i0;   // a valid index for the address arithmetic
    double x0, y0, z0, x1, y1, z1;
    if (HOME_LDS) {
      const int q0 = hl + (h - hb);
      x0 = L.cxs[q0];
      y0 = L.cys[q0];
      z0 = L.czs[q0];
      x1 = L.cxs[q0 + 1];
      y1 = L.cys[q0 + 1];
      z1 = L.czs[q0 + 1];
    } else {
      x0 = x[i0];
      y0 = x[n + i0];
      z0 = x[2 * n + i0];
      x1 = x[k1];
      y1 = x[n + k1];
      z1 = x[2 * n + k1];
    }
    if (!two) x1 = y1 = z1 = nan;
    int* __restrict__ r0 =
        a.neigh + (size_t)(i0 >> gs) * rows * kWave + ((i0 & ((1 << gs) - 1)) << lk);
    int* __restrict__ r1 =
        a.neigh + (size_t)(k1 >> gs) * rows * kWave + ((k1 & ((1 << gs) - 1)) << lk);
    int base0 = 0, base1 = 0;
    if (!FIRST) {
      // LDS copy for the first kBlock home atoms, else the global count (an
      // atomic load, so that the two loads never share one flat access)
      base0 = h - hb < kBlock ? L.hcnt[h - hb]
                              : __hip_atomic_load(&a.numneigh[i0], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
      if (two)
        base1 = h + 1 - hb < kBlock ? L.hcnt[h + 1 - hb]
                                    : __hip_atomic_load(&a.numneigh[k1], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
    }
    // entries of this pass, relative to base0 / base1
    int cnt0 = 0, cnt1 = 0;
    for (int sg = 0; sg < cs.n; ++sg) {
      const int sbase = cs.base[sg], spad = cs.pad[sg];
      for (int t = 0; t < spad; t += kWave) {
        const int q = sbase + t + lane;
        const int j = L.cjs[q];
        const double cx = L.cxs[q], cy = L.cys[q], cz = L.czs[q];
        double ax = x0 - cx, ay = y0 - cy, az = z0 - cz;
        double bx = x1 - cx, by = y1 - cy, bz = z1 - cz;
        if (WRAP) {
          ax = min_image(ax, a.box.L[0], a.box.inv[0]);
          ay = min_image(ay, a.box.L[1], a.box.inv[1]);
          az = min_image(az, a.box.L[2], a.box.inv[2]);
          bx = min_image(bx, a.box.L[0], a.box.inv[0]);
          by = min_image(by, a.box.L[1], a.box.inv[1]);
          bz = min_image(bz, a.box.L[2], a.box.inv[2]);
        }
        const double ra = ax * ax + ay * ay + az * az;
        const double rb = bx * bx + by * by + bz * bz;
        const bool ta = (ra < rl2) & (j != i0);
        const bool tb = (rb < rl2) & (j != i1);
        // each ballot taken straight from one compare (no mask materialised in VGPRs)
        const unsigned long long ma =
            __builtin_amdgcn_ballot_w64(ra < rl2) & __builtin_amdgcn_ballot_w64(j != i0);
        const unsigned long long mb =
            __builtin_amdgcn_ballot_w64(rb < rl2) & __builtin_amdgcn_ballot_w64(j != i1);
        const int pa = cnt0 + __builtin_amdgcn_mbcnt_hi(
                                  (unsigned)(ma >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)ma, 0u));
        const int pb = cnt1 + __builtin_amdgcn_mbcnt_hi(
                                  (unsigned)(mb >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mb, 0u));
        const int na = __popcll(ma), nb = __popcll(mb);
        // every lane writes its LDS slot, rejected (or past-the-buffer) ones
        // into their sink, so no lane mask changes on the common path
        lrow[ta && pa < kListBuf ? pa : sink] = j;
        lrow[tb && pb < kListBuf ? kListBuf + pb : sink] = j;
        if (cnt0 + na > kListBuf || cnt1 + nb > kListBuf) {   // wave-uniform, long lists only
          if (ta && pa >= kListBuf && base0 + pa < a.cap) put_entry(r0, base0 + pa, lk, j);
          if (tb && pb >= kListBuf && base1 + pb < a.cap) put_entry(r1, base1 + pb, lk, j);
        }
        cnt0 += na;
        cnt1 += nb;
      }
    }
    // copy the buffered entries into the list layout (this wave's own LDS
    // rows; a wavefront's LDS accesses complete in order)
    __builtin_amdgcn_wave_barrier();
    const int lim0 = min(min(cnt0, kListBuf), a.cap - base0);
    const int lim1 = min(min(cnt1, kListBuf), a.cap - base1);
    for (int m = lane; m < lim0; m += kWave) put_entry(r0, base0 + m, lk, lrow[m]);
    for (int m = lane; m < lim1; m += kWave) put_entry(r1, base1 + m, lk, lrow[kListBuf + m]);
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      a.numneigh[i0] = base0 + cnt0;
      if (h - hb < kBlock) L.hcnt[h - hb] = base0 + cnt0;
      if (two) {
        a.numneigh[i1] = base1 + cnt1;
        if (h + 1 - hb < kBlock) L.hcnt[h + 1 - hb] = base1 + cnt1;
      }
    }
  }
}

// A home cell at least one cell away from every box face (with >= 3 cells per
// dimension) has an unwrapped stencil: candidate and home positions are
// wrapped into [0, L) and at most two cell edges apart, so an accepted pair
// has rint(d / L) = 0 and d = x_i - x_j is the FP64 minimum image bit for bit,
// while any other image is at least L / 3 >= r_l away.
__device__ inline bool cell_wraps(int cx, int cy, int cz, const int* nc) {
  const int c[3] = {cx, cy, cz};
  bool w = false;
  for (int d = 0; d < 3; ++d) w = w || nc[d] < 3 || c[d] == 0 || c[d] == nc[d] - 1;
  return w;
}

// build_home for the per-cell path's runtime cases.
template <bool WRAP>
__device__ inline void build_home_any(const BuildArgs& a, const BuildLds& L, const CandSegs& cs,
                                      bool first, int hl, int hb, int he, int lane, int wave) {
  if (first) {
    if (hl >= 0)
      build_home<WRAP, true, true>(a, L, cs, hl, hb, he, lane, wave);
    else
      build_home<WRAP, false, true>(a, L, cs, hl, hb, he, lane, wave);
  } else {
    if (hl >= 0)
      build_home<WRAP, true, false>(a, L, cs, hl, hb, he, lane, wave);
    else
      build_home<WRAP, false, false>(a, L, cs, hl, hb, he, lane, wave);
  }
}

// Copies of the home atoms' state after their lists are done: lengths for the
// running maximum, x_ref / packed / sorted-back positions (HOME_LDS: from LDS
// slot hl + t, else from x), and v, id back from staging (thread t's first
// atom from the prefetched pv / pid).  Lengths of the first 256 home atoms
// come from hcnt, of any further ones from numneigh.  Returns this thread's
// largest list length.
template <bool HOME_LDS>
__device__ inline void finish_one(const BuildArgs& a, const BuildLds& L, int hl, int t, int i,
                                  bool mine, double pv0, double pv1, double pv2, int pid) {
  const int n = a.n;
  double xi, yi, zi;
  if (HOME_LDS) {
    xi = L.cxs[hl + t];
    yi = L.cys[hl + t];
    zi = L.czs[hl + t];
  } else {
    xi = a.x[i];
    yi = a.x[n + i];
    zi = a.x[2 * n + i];
  }
  if (a.x_ref) {
    a.x_ref[i] = xi;
    a.x_ref[n + i] = yi;
    a.x_ref[2 * n + i] = zi;
  }
  const int ti = a.type_in ? a.type_in[i] : 0;
  if (a.xq_out) store_packed(a.xq_out, i, xi, yi, zi, ti);
  if (a.type_out) a.type_out[i] = ti;
  if (a.x_out) {
    a.x_out[i] = xi;
    a.x_out[n + i] = yi;
    a.x_out[2 * n + i] = zi;
    if (mine) {
      a.v_out[i] = pv0;
      a.v_out[n + i] = pv1;
      a.v_out[2 * n + i] = pv2;
      a.id_out[i] = pid;
    } else {
      a.v_out[i] = a.v_in[i];
      a.v_out[n + i] = a.v_in[n + i];
      a.v_out[2 * n + i] = a.v_in[2 * n + i];
      a.id_out[i] = a.id_in[i];
    }
  }
}

template <bool HOME_LDS>
__device__ inline int finish_home(const BuildArgs& a, const BuildLds& L, int hl, int hb, int he,
                                  int tid, bool pre, int pi, double pv0, double pv1, double pv2,
                                  int pid) {
  const bool sorted = a.sorted != 0;
  int mx = 0;
  if (hb + tid < he) {
    const int i = pre ? pi : (sorted ? hb + tid : a.perm[hb + tid]);
    mx = L.hcnt[tid];
    finish_one<HOME_LDS>(a, L, hl, tid, i, pre, pv0, pv1, pv2, pid);
  }
  for (int h = hb + tid + kBlock; h < he; h += kBlock) {
    const int i = sorted ? h : a.perm[h];
    mx = max(mx, a.numneigh[i]);
    finish_one<HOME_LDS>(a, L, hl, h - hb, i, false, 0.0, 0.0, 0.0, 0);
  }
  return mx;
}

// Prefetch of the state finish_home copies back (thread t: home atom hb + t).
struct HomePrefetch {
  bool pre = false;
  int pi = 0, pid = 0;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  __device__ inline void load(const BuildArgs& a, int hb, int he, int tid) {
    pre = a.x_out && hb + tid < he;
    if (pre) {
      pi = a.sorted ? hb + tid : a.perm[hb + tid];
      v0 = a.v_in[pi];
      v1 = a.v_in[a.n + pi];
      v2 = a.v_in[2 * a.n + pi];
      pid = a.id_in[pi];
    }
  }
};

constexpr int kBuildChunk = 768;   // candidates per pass of the per-cell path, a multiple of 64
static_assert(kBuildChunk % 64 == 0, "a padded chunk stays inside the arrays");
constexpr int kStageHalf = 4;   // stencil entries per wave staged together (two halves cover 27)
static_assert(2 * kStageHalf * (kBlock / kWave) >= 27, "staging covers the stencil");

// Per-cell path: wave w stages stencil entries w + 4 (k0 + k), k < kStageHalf,
// the first 64 in-chunk atoms of each with all loads in flight together.
__device__ inline void stage_entries(const BuildArgs& a, const BuildLds& L, int k0, int c0,
                                     int clen, int nst, const int* st_start, const int* st_off,
                                     int lane, int wave) {
  const int n = a.n;
  const double* __restrict__ x = a.x;
  const bool sorted = a.sorted != 0;
  double sx[kStageHalf], sy[kStageHalf], sz[kStageHalf];
  int sj[kStageHalf], sq[kStageHalf];
#pragma unroll
  for (int k = 0; k < kStageHalf; ++k) {
    const int e = wave + (k0 + k) * (kBlock / kWave);
    sq[k] = -1;
    sj[k] = 0;
    if (e < nst) {
      const int lo = max(st_off[e], c0), hi = min(st_off[e + 1], c0 + clen);
      const int q = lo + lane;
      if (q < hi) {
        const int sl = st_start[e] + (q - st_off[e]);
        sq[k] = q - c0;
        sj[k] = sorted ? sl : a.perm[sl];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kStageHalf; ++k) {
    if (sq[k] >= 0) {
      sx[k] = x[sj[k]];
      sy[k] = x[n + sj[k]];
      sz[k] = x[2 * n + sj[k]];
    }
  }
#pragma unroll
  for (int k = 0; k < kStageHalf; ++k) {
    if (sq[k] >= 0) {
      L.cjs[sq[k]] = sj[k];
      L.cxs[sq[k]] = sx[k];
      L.cys[sq[k]] = sy[k];
      L.czs[sq[k]] = sz[k];
    }
  }
}

__device__ inline void pad_slots(const BuildLds& L, int from, int to, int tid) {
  for (int q = from + tid; q < to; q += kBlock) {
    L.cjs[q] = -1;
    L.cxs[q] = __builtin_nan("");
    L.cys[q] = __builtin_nan("");
    L.czs[q] = __builtin_nan("");
  }
}

// Home atoms [hb, he) of one cell against its staged stencil (general path):
// the candidates in chunks of kBuildChunk, then the copies of the home atoms'
// state.  home_off is the candidate offset of atom hb within the stencil.
__device__ inline int build_piece(const BuildArgs& a, const BuildLds& L, int hb, int he,
                                  int home_off, int total, int nst, bool wrap,
                                  const int* st_start, const int* st_off, int lane, int wave,
                                  int tid) {
  HomePrefetch P;
  P.load(a, hb, he, tid);
  // home atoms staged in the chunk that holds them all, else read from x
  int hl_last = -1;
  for (int c0 = 0; c0 < total; c0 += kBuildChunk) {
    const int clen = min(kBuildChunk, total - c0);
    const int cpad = (clen + kWave - 1) & ~(kWave - 1);
    stage_entries(a, L, 0, c0, clen, nst, st_start, st_off, lane, wave);
    stage_entries(a, L, kStageHalf, c0, clen, nst, st_start, st_off, lane, wave);
    for (int e = wave; e < nst; e += kBlock / kWave) {
      const int lo = max(st_off[e], c0), hi = min(st_off[e + 1], c0 + clen);
      for (int q = lo + kWave + lane; q < hi; q += kWave) {
        const int sl = st_start[e] + (q - st_off[e]);
        const int j = a.sorted ? sl : a.perm[sl];
        L.cjs[q - c0] = j;
        L.cxs[q - c0] = a.x[j];
        L.cys[q - c0] = a.x[a.n + j];
        L.czs[q - c0] = a.x[2 * a.n + j];
      }
    }
    pad_slots(L, clen, cpad, tid);
    __syncthreads();
    const int hl = home_off >= c0 && home_off + (he - hb) <= c0 + clen ? home_off - c0 : -1;
    CandSegs cs;
    cs.n = 1;
    cs.base[0] = 0;
    cs.pad[0] = cpad;
    if (wrap)
      build_home_any<true>(a, L, cs, c0 == 0, hl, hb, he, lane, wave);
    else
      build_home_any<false>(a, L, cs, c0 == 0, hl, hb, he, lane, wave);
    __syncthreads();
    hl_last = hl;
  }
  const int mx =
      hl_last >= 0 ? finish_home<true>(a, L, hl_last, hb, he, tid, P.pre, P.pi, P.v0, P.v1, P.v2,
                                       P.pid)
                   : finish_home<false>(a, L, hl_last, hb, he, tid, P.pre, P.pi, P.v0, P.v1,
                                        P.v2, P.pid);
  __syncthreads();   // LDS (candidates, hcnt) free for the next piece
  return mx;
}

// Home atoms per piece when a cell's home atoms are split over several
// workgroups (dense cells: long cutoffs, few cells).
constexpr int kHomePiece = 64;

// The lists of one cell's home atoms, general path: the (up to) 27 stencil
// entries, in stencil order and slot order inside a cell, staged in chunks of
// kBuildChunk.  With parts > 1 the home atoms come in pieces of kHomePiece and
// this workgroup takes pieces part, part + parts, ...; each piece stages the
// whole stencil again.  Every thread of the workgroup calls it.  Returns this
// thread's largest list length; part 0 copies cell_start into cell_start_out.
__device__ inline int build_cell(const BuildArgs& a, const BuildLds& L, int cell, int part,
                                 int parts, int* st_start, int* st_off, int* st_meta) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int hb = a.cell_start[cell], he = a.cell_start[cell + 1];
  if (wave == 0) {
    // Stencil entry (oz, oy, ox) = lane, all 27 looked up at once; the kept
    // entries keep the z, y, x offset order, their offsets by a wave scan.
    bool kept;
    const int c2 = stencil_lane(cell, lane, a.nc, &kept);
    const unsigned long long km = __ballot(kept);
    int b = 0, cnt = 0;
    if (kept) {
      b = a.cell_start[c2];
      cnt = a.cell_start[c2 + 1] - b;
    }
    int inc = cnt;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int y = __shfl_up(inc, off, kWave);
      if (lane >= off) inc += y;
    }
    if (kept) {
      const int pos = __popcll(km & ((1ull << lane) - 1));
      st_start[pos] = b;
      st_off[pos] = inc - cnt;
      if (c2 == cell) st_meta[1] = pos;
    }
    if (lane == kWave - 1) {
      st_meta[0] = __popcll(km);
      st_off[__popcll(km)] = inc;
    }
  }
  __syncthreads();
  const int nst = st_meta[0];
  const int total = st_off[nst];
  const int home_off = st_off[st_meta[1]];
  const int cx = cell % a.nc[0], cy = (cell / a.nc[0]) % a.nc[1], cz = cell / (a.nc[0] * a.nc[1]);
  const bool wrap = cell_wraps(cx, cy, cz, a.nc);
  if (tid == 0 && part == 0 && a.cell_start_out) {
    a.cell_start_out[cell] = hb;
    if (cell == a.nc[0] * a.nc[1] * a.nc[2] - 1) a.cell_start_out[cell + 1] = he;
  }
  const int piece = parts > 1 ? kHomePiece : max(he - hb, 1);
  int mx = 0;
  for (int h0 = hb + part * piece; h0 < he; h0 += parts * piece) {   // uniform
    mx = max(mx, build_piece(a, L, h0, min(he, h0 + piece), home_off + (h0 - hb), total, nst,
                             wrap, st_start, st_off, lane, wave, tid));
  }
  __syncthreads();   // stencil tables free for the next cell (also when no piece ran)
  return mx;
}

// A build's view of its arguments: the box from device memory when the run
// keeps it there (NPT), whose edges the first thread records as the box of
// this build.
__device__ inline BuildArgs build_view(const BuildArgs& a0) {
  BuildArgs a = a0;
  if (a0.boxd) {
    a.box = box_load(a0.boxd);
    if (a0.lref && blockIdx.x == 0 && threadIdx.x == 0)
      for (int d = 0; d < 3; ++d) a0.lref[d] = a.box.L[d];
  }
  return a;
}

// Running maximum and overflow flag: one device-scope atomic per workgroup at
// most, skipped when the word already holds at least m (a stale read only
// costs an extra atomic).
__device__ inline void report_max(const BuildArgs& a, int mx, int* red) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  mx = wave_max(mx);
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = red[0];
    for (int w = 1; w < kBlock / kWave; ++w) m = max(m, red[w]);
    if (m > 0 && m > __hip_atomic_load(&a.status[MD_ST_MAXNEIGH], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&a.status[MD_ST_MAXNEIGH], m);
    if (m > a.cap) atomicOr(&a.status[MD_ST_ERRORS], 1);
  }
}

// General path: `parts` workgroups per cell, consecutive in the (XCD-aware)
// numbering so a cell's pieces share one L2.
__global__ __launch_bounds__(kBlock) void k_build(BuildArgs a0, int parts) {
  if (a0.gate && *a0.gate == 0) return;
  const BuildArgs a = build_view(a0);
  __shared__ double cxs[kBuildChunk], cys[kBuildChunk], czs[kBuildChunk];
  __shared__ int cjs[kBuildChunk];
  __shared__ int hcnt[kBlock];
  __shared__ int lbuf[(kBlock / kWave) * kListRow];
  __shared__ int st_start[27], st_off[28], st_meta[2];
  __shared__ int red[kBlock / kWave];
  const BuildLds L{cxs, cys, czs, cjs, hcnt, lbuf};
  const int blk = xcd_block();
  const int cell = blk / parts, part = blk % parts;
  if (blk == 0 && threadIdx.x == 0) atomicAdd(&a.status[MD_ST_BUILDS], 1);
  const int mx = build_cell(a, L, cell, part, parts, st_start, st_off, st_meta);
  report_max(a, mx, red);
}

// Row path.  A workgroup takes a run of up to kRowCells consecutive cells of
// one x row.  Slab u is the (up to 9) cells (wy, wz) around the row at x index
// cx0 - 1 + u, in increasing cell order; all kRowCells + 2 slabs of the run
// sit back to back in LDS, so the 27-cell stencil of home cell k is the one
// contiguous candidate range slabs k .. k + 2.  Candidate order: slab x - 1,
// x, x + 1, cells in increasing order inside a slab, slot order inside a cell.
constexpr int kRowCells = 2;
constexpr int kMaxSlabs = kRowCells + 2;
constexpr int kRowCells9 = kMaxSlabs * 9;   // (slab, cell) entries of a run
constexpr int kRowCap = 960;                // candidates of a run held in LDS
// The last iteration of a pair's loop prefetches one row of 64 slots past its
// range: the arrays extend two rows past kRowCap.
constexpr int kRowSlots = kRowCap + 2 * kWave;
static_assert(kRowSlots >= kBuildChunk, "the per-cell fallback fits the row arrays");

// Minimum image along the dimensions set in WM (home cells touching a box face
// there, or fewer than 3 cells); along the others the candidates are the
// unwrapped neighbours and the plain difference is the minimum image of every
// accepted pair, bit for bit (see cell_wraps).
template <int WM>
__device__ inline void pair_image(double& dx, double& dy, double& dz, const BoxK& box) {
  if (WM & 1) dx = min_image(dx, box.L[0], box.inv[0]);
  if (WM & 2) dy = min_image(dy, box.L[1], box.inv[1]);
  if (WM & 4) dz = min_image(dz, box.L[2], box.inv[2]);
}

// Home atoms tested together per candidate batch in the row path: each batch
// of 64 candidates read from LDS serves kGroup independent distance chains.
constexpr int kGroup = 4;
constexpr int kGroupRow = kGroup * kListBuf;   // per wavefront: one buffer per home atom
constexpr int kLbufRow = kGroupRow > kListRow ? kGroupRow : kListRow;

// Lists of the nh (<= kGroup) consecutive home atoms i0, i0 + 1, ... staged
// at LDS slots s0, s0 + 1, ..., against the candidates in LDS slots [c0, c1).
// 64 candidates per iteration, tested against every atom of the group; the
// next 64 are read from LDS while these are tested.  Past c1 (last
// iteration) and at the home atoms' own slots a scalar lane mask drops the
// candidate.  Accepted ones go, in candidate order, through a ballot prefix
// count into the atom's LDS buffer (anything past kListBuf straight into the
// list) and are copied into the list layout when the group is done.  hidx:
// index of i0 among the workgroup's home atoms (for hcnt).
template <int WM>
__device__ inline void build_group(const BuildArgs& a, const BuildLds& L, int c0, int c1, int s0,
                                   int i0, int nh, int hidx, int lane, int wave) {
  const int lk = __ffs(a.layout) - 1;
  const int gs = 6 - lk;
  const size_t rows = nl_rows(a.cap, a.layout);
  const double rl2 = a.rl2;
  const BoxK box = a.box;
  int* __restrict__ lrow = L.lbuf + wave * kLbufRow;
  double hx[kGroup], hy[kGroup], hz[kGroup];
  int* r[kGroup];
  int cnt[kGroup];
#pragma unroll
  for (int g = 0; g < kGroup; ++g) {
    // an atom past nh keeps NaN coordinates: it accepts nothing
    hx[g] = g < nh ? L.cxs[s0 + g] : __builtin_nan("");
    hy[g] = g < nh ? L.cys[s0 + g] : __builtin_nan("");
    hz[g] = g < nh ? L.czs[s0 + g] : __builtin_nan("");
    const int ig = g < nh ? i0 + g : i0;
    r[g] = a.neigh + (size_t)(ig >> gs) * rows * kWave + ((ig & ((1 << gs) - 1)) << lk);
    cnt[g] = 0;
  }
  const int total = c1 - c0;
  const int ks = s0 - c0;   // candidate index of i0 itself (the others follow it)
  // Test the 64 candidates (j, cx, cy, cz) of iteration t against the group.
  auto test = [&](int t, int j, double cx, double cy, double cz) {
    unsigned long long m[kGroup];
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
      double dx = hx[g] - cx, dy = hy[g] - cy, dz = hz[g] - cz;
      pair_image<WM>(dx, dy, dz, box);
      const double r2 = dx * dx + dy * dy + dz * dz;
      m[g] = __builtin_amdgcn_ballot_w64(r2 < rl2);
    }
    // scalar masks, only in the (one or two) iterations that need them: lanes
    // past the range, and each home atom's own slot
    const int rem = total - t;
    const int d = ks - t;
    if (rem < kWave || (unsigned)(d + kGroup - 1) < (unsigned)(kWave + kGroup - 1)) {
      const unsigned long long vm = rem >= kWave ? ~0ull : (1ull << rem) - 1ull;
#pragma unroll
      for (int g = 0; g < kGroup; ++g) {
        const unsigned long long self =
            (unsigned)(d + g) < (unsigned)kWave ? 1ull << (d + g) : 0ull;
        m[g] &= vm & ~self;
      }
    }
    int n[kGroup], rk[kGroup];
    bool fits = true;
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
      n[g] = __popcll(m[g]);
      // rank among this iteration's accepted candidates
      rk[g] = __builtin_amdgcn_mbcnt_hi((unsigned)(m[g] >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)m[g], 0u));
      fits = fits && cnt[g] + n[g] <= kListBuf;
    }
    // accepted lanes append to the atom's LDS buffer at cnt + rank; past
    // kListBuf (wave-uniform, long lists only) entries go to the list itself
    if (fits) {
#pragma unroll
      for (int g = 0; g < kGroup; ++g)
        if (__builtin_amdgcn_inverse_ballot_w64(m[g])) lrow[g * kListBuf + cnt[g] + rk[g]] = j;
    } else {
#pragma unroll
      for (int g = 0; g < kGroup; ++g) {
        const bool t = __builtin_amdgcn_inverse_ballot_w64(m[g]);
        const int p = cnt[g] + rk[g];
        if (t && p < kListBuf) lrow[g * kListBuf + p] = j;
        if (t && p >= kListBuf && p < a.cap) put_entry_apart(r[g], p, lk, j);
      }
    }
#pragma unroll
    for (int g = 0; g < kGroup; ++g) cnt[g] += n[g];
  };
  // two register sets alternate: the next 64 candidates are read while the
  // current ones are tested
  int q = c0 + lane;
  int ja = L.cjs[q];
  double xa = L.cxs[q], ya = L.cys[q], za = L.czs[q];
  for (int t = 0; t < total; t += 2 * kWave) {
    const int jb = L.cjs[q + kWave];
    const double xb = L.cxs[q + kWave], yb = L.cys[q + kWave], zb = L.czs[q + kWave];
    __builtin_amdgcn_sched_barrier(0);
    test(t, ja, xa, ya, za);
    if (t + kWave >= total) break;
    q += 2 * kWave;
    ja = L.cjs[q];
    xa = L.cxs[q];
    ya = L.cys[q];
    za = L.czs[q];
    __builtin_amdgcn_sched_barrier(0);
    test(t + kWave, jb, xb, yb, zb);
  }
  // copy the buffered entries into the list layout (this wave's own LDS
  // rows; a wavefront's LDS accesses complete in order)
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int g = 0; g < kGroup; ++g) {
    const int lim = g < nh ? min(min(cnt[g], kListBuf), a.cap) : 0;
    for (int mm = lane; mm < lim; mm += kWave) put_entry(r[g], mm, lk, lrow[g * kListBuf + mm]);
  }
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) {
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
      if (g < nh) {
        a.numneigh[i0 + g] = cnt[g];
        if (hidx + g < kBlock) L.hcnt[hidx + g] = cnt[g];
      }
    }
  }
}

template <int WM>
__device__ inline void build_cell_groups(const BuildArgs& a, const BuildLds& L, int c0, int c1,
                                         int slot, int hb, int nhome, int hidx, int first,
                                         int lane, int wave) {
  for (int p = first; kGroup * p < nhome; p += kBlock / kWave)
    build_group<WM>(a, L, c0, c1, slot + kGroup * p, hb + kGroup * p,
                    min(kGroup, nhome - kGroup * p), hidx + kGroup * p, lane, wave);
}


// Row segment wg (a run of up to kRowCells consecutive cells of an x row) of
// the row path; every thread of the workgroup calls it.  The run's slabs are
// staged once; the home atoms of all its cells, two per work item, are dealt
// to the wavefronts in turn with no barrier between cells.  Runs whose slabs
// hold more than kRowCap atoms take the per-cell path.  Returns this
// thread's largest list length.
__device__ inline int build_row_segment(const BuildArgs& a, const BuildLds& L, int wg,
                                        int* g_off, int* g_start, int* st_start, int* st_off,
                                        int* st_meta, int* big) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int nc0 = a.nc[0], nc1 = a.nc[1], nc2 = a.nc[2];
  const int spr = (nc0 + kRowCells - 1) / kRowCells;   // row segments per row
  const int row = wg / spr, seg = wg % spr;
  const int cy = row % nc1, cz = row / nc1;
  const int cx0 = seg * kRowCells;
  const int nh = min(kRowCells, nc0 - cx0);
  const int nslab = nh + 2;
  const int ny = min(nc1, 3), nz = min(nc2, 3), ncs = ny * nz;
  const int ne = nslab * ncs;   // (slab, cell) entries, entry u * ncs + e
  if (wg == 0 && tid == 0) atomicAdd(&a.status[MD_ST_BUILDS], 1);
  if (wave == 0) {
    const int u = lane / ncs, e = lane % ncs;
    int b = 0, cnt = 0;
    if (lane < ne) {
      int sx = cx0 - 1 + u;
      sx = sx < 0 ? sx + nc0 : (sx >= nc0 ? sx - nc0 : sx);
      const int c = (nbr_sorted(cz, nc2, e / ny) * nc1 + nbr_sorted(cy, nc1, e % ny)) * nc0 + sx;
      b = a.cell_start[c];
      cnt = a.cell_start[c + 1] - b;
    }
    int inc = cnt;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int y = __shfl_up(inc, off, kWave);
      if (lane >= off) inc += y;
    }
    if (lane < ne) {
      g_start[lane] = b;
      g_off[lane] = inc - cnt;
      if (lane == ne - 1) {
        g_off[ne] = inc;
        *big = inc > kRowCap;
      }
    }
  }
  __syncthreads();
  int mx = 0;
  if (*big) {
    for (int k = 0; k < nh; ++k)
      mx = max(mx, build_cell(a, L, (cz * nc1 + cy) * nc0 + cx0 + k, 0, 1, st_start, st_off,
                              st_meta));
    __syncthreads();
    return mx;
  }
  const int eh = self_rank(cz, nc2) * ny + self_rank(cy, nc1);   // home cell within a slab
  const int hb0 = __builtin_amdgcn_readfirstlane(g_start[ncs + eh]);   // first home atom of the run
  const int hend = g_start[nh * ncs + eh] + (g_off[nh * ncs + eh + 1] - g_off[nh * ncs + eh]);
  HomePrefetch P;
  P.load(a, hb0, hend, tid);
  {
    // stage the slabs: slot q holds the atom at sorted index g_start[c] + q -
    // g_off[c], c the last entry with g_off[c] <= q (a binary search; empty
    // cells share their offset with the next entry and are skipped by it)
    const int total = g_off[ne];
    constexpr int kRounds = 3;
    for (int q0 = 0; q0 < total; q0 += kRounds * kBlock) {
      int jr[kRounds];
      double xr[kRounds], yr[kRounds], zr[kRounds];
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        const int q = q0 + r * kBlock + tid;
        jr[r] = -1;
        if (q < total) {
          int lo = 0, hi = ne;
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (g_off[mid] <= q) lo = mid; else hi = mid;
          }
          jr[r] = g_start[lo] + (q - g_off[lo]);
        }
      }
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        if (jr[r] >= 0) {
          xr[r] = a.x[jr[r]];
          yr[r] = a.x[a.n + jr[r]];
          zr[r] = a.x[2 * a.n + jr[r]];
        }
      }
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        const int q = q0 + r * kBlock + tid;
        if (jr[r] >= 0) {
          L.cjs[q] = jr[r];
          L.cxs[q] = xr[r];
          L.cys[q] = yr[r];
          L.czs[q] = zr[r];
        }
      }
    }
  }
  __syncthreads();
  // work items: group p (kGroup home atoms) of home cell k is item
  // g = (groups before cell k) + p, taken by wavefront g % 4
  int g0 = 0;
  const bool ywrap = nc1 < 3 || cy == 0 || cy == nc1 - 1;
  const bool zwrap = nc2 < 3 || cz == 0 || cz == nc2 - 1;
  for (int k = 0; k < nh; ++k) {
    // LDS values the whole workgroup shares: kept in scalar registers
    const int eo = (k + 1) * ncs + eh;
    const int slot = __builtin_amdgcn_readfirstlane(g_off[eo]);
    const int hb = __builtin_amdgcn_readfirstlane(g_start[eo]);
    const int nhome = __builtin_amdgcn_readfirstlane(g_off[eo + 1]) - slot;
    const int c0 = __builtin_amdgcn_readfirstlane(g_off[k * ncs]);
    const int c1 = __builtin_amdgcn_readfirstlane(g_off[(k + 3) * ncs]);
    const int first = (wave - g0) & (kBlock / kWave - 1);
    const int cx = cx0 + k;
    const int wm = (cx == 0 || cx == nc0 - 1 ? 1 : 0) | (ywrap ? 2 : 0) | (zwrap ? 4 : 0);
    const int hidx = hb - hb0;
    switch (wm) {
      case 0: build_cell_groups<0>(a, L, c0, c1, slot, hb, nhome, hidx, first, lane, wave); break;
      case 1: build_cell_groups<1>(a, L, c0, c1, slot, hb, nhome, hidx, first, lane, wave); break;
      case 2: build_cell_groups<2>(a, L, c0, c1, slot, hb, nhome, hidx, first, lane, wave); break;
      case 3: build_cell_groups<3>(a, L, c0, c1, slot, hb, nhome, hidx, first, lane, wave); break;
      case 4: build_cell_groups<4>(a, L, c0, c1, slot, hb, nhome, hidx, first, lane, wave); break;
      case 5: build_cell_groups<5>(a, L, c0, c1, slot, hb, nhome, hidx, first, lane, wave); break;
      case 6: build_cell_groups<6>(a, L, c0, c1, slot, hb, nhome, hidx, first, lane, wave); break;
      default: build_cell_groups<7>(a, L, c0, c1, slot, hb, nhome, hidx, first, lane, wave); break;
    }
    g0 += (nhome + kGroup - 1) / kGroup;
    if (tid == 0 && a.cell_start_out) {
      const int cell = (cz * nc1 + cy) * nc0 + cx;
      a.cell_start_out[cell] = hb;
      if (cell == nc0 * nc1 * nc2 - 1) a.cell_start_out[cell + 1] = hb + nhome;
    }
  }
  __syncthreads();
  // copies of the home atoms' state (home atom h - hb0 of the run: its cell k
  // found by the run's cell boundaries, its LDS slot from the cell's)
  for (int h = hb0 + tid; h < hend; h += kBlock) {
    int k = 0;
    while (k + 1 < nh && h >= g_start[(k + 2) * ncs + eh]) ++k;
    const int eo = (k + 1) * ncs + eh;
    const int slot = g_off[eo] + (h - g_start[eo]);
    const int t = h - hb0;
    mx = max(mx, t < kBlock ? L.hcnt[t]
                            : __hip_atomic_load(&a.numneigh[h], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT));
    const bool mine = P.pre && t == tid;
    finish_one<true>(a, L, slot, 0, h, mine, P.v0, P.v1, P.v2, P.pid);
  }
  __syncthreads();   // LDS tables and slabs are reused by the next segment
  return mx;
}

// Sorted atoms, at least 3 cells along x: the row segments
// (build_row_segment), one per workgroup as launched; a smaller grid would
// loop over several.
__global__ __launch_bounds__(kBlock, 4) void k_build_rows(BuildArgs a0) {
  if (a0.gate && *a0.gate == 0) return;
  const BuildArgs a = build_view(a0);
  __shared__ double cxs[kRowSlots], cys[kRowSlots], czs[kRowSlots];
  __shared__ int cjs[kRowSlots];
  __shared__ int hcnt[kBlock];
  __shared__ int lbuf[(kBlock / kWave) * kLbufRow];
  __shared__ int g_off[kRowCells9 + 1], g_start[kRowCells9];
  __shared__ int st_start[27], st_off[28], st_meta[2];
  __shared__ int red[kBlock / kWave];
  __shared__ int big;
  const BuildLds L{cxs, cys, czs, cjs, hcnt, lbuf};
  const int nc0 = a.nc[0], nc1 = a.nc[1], nc2 = a.nc[2];
  const int spr = (nc0 + kRowCells - 1) / kRowCells;   // row segments per row
  const BlockRange br = xcd_range(spr * nc1 * nc2);
  int mx = 0;
  for (int wg = br.first; wg < br.end; wg += br.step)
    mx = max(mx, build_row_segment(a, L, wg, g_off, g_start, st_start, st_off, st_meta, &big));
  report_max(a, mx, red);
}

// Tile list from a full list in layout K: one workgroup per run (a resident
// grid looping over them).  Wave 0 lays out the run's window segments and
// sorts them by first atom; each wavefront then takes run-relative groups of
// G = 64 / K home atoms and, row by row of the tile layout, maps every listed
// partner j to its window index: the last segment (by first atom) starting at
// or below j, plus j's offset in it.  A partner outside the window cannot
// occur for a list built on the same cell starts; if it did (or a window had
// more atoms than 16 bits index), status bit 2 marks the state unusable.
__global__ __launch_bounds__(kBlock) void k_tile_convert(const int* __restrict__ neigh,
                                                         const int* __restrict__ numneigh, int n,
                                                         int cap, int k,
                                                         const int* __restrict__ cs, TileGeom g,
                                                         unsigned short* __restrict__ tile,
                                                         int* status, const int* gate) {
  if (gate && *gate == 0) return;
  __shared__ int s_lo[kTileSegs], s_len[kTileSegs], s_base[kTileSegs];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int lk = __ffs(k) - 1;
  const int G = kWave >> lk;
  const int rows = (int)nl_rows(cap, k);
  const int nruns = tile_nruns(g);
  const BlockRange br = xcd_range(nruns);
  for (int r = br.first; r < br.end; r += br.step) {
    const TileRun t = tile_run(g, r, cs);
    if (wave == 0) {
      int lo = 0, len = 0;
      if (lane < kTileSegs) tile_segment(g, t, lane, cs, &lo, &len);
      int inc = len;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += y;
      }
      // rank by first atom (empty segments last), ties by window order
      const int key = len > 0 ? lo : INT_MAX;
      int rank = 0;
      for (int u = 0; u < kTileSegs; ++u) {
        const int ku = __shfl(key, u, kWave);
        rank += (ku < key || (ku == key && u < lane)) ? 1 : 0;
      }
      if (lane < kTileSegs) {
        s_lo[rank] = key;
        s_len[rank] = len;
        s_base[rank] = inc - len;
      }
      if (lane == kTileSegs - 1 && inc > 65536) atomicOr(&status[MD_ST_ERRORS], 4);
    }
    __syncthreads();
    const int nh = t.he - t.hb;
    const int ngroups = (nh + G - 1) / G;
    for (int gi = wave; gi < ngroups; gi += kBlock / kWave) {
      const int q = gi * G + (lane >> lk);
      const int m0 = lane & (k - 1);
      const int i = t.hb + q;
      const bool live = q < nh;
      const int nn = live ? min(numneigh[i], cap) : 0;
      const int cnt = nn > m0 ? ((nn - m0 + k - 1) >> lk) : 0;
      int tmax = cnt;
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) tmax = max(tmax, __shfl_xor(tmax, off, kWave));
      // 16-bit elements of this lane's words: word tt / 2, half tt % 2
      unsigned short* row0 =
          tile + (((size_t)(t.hb / G + r + gi) * ((rows + 1) / 2)) * kWave + lane) * 2;
      // consecutive entries mostly fall in the segment of the previous one
      // (lists follow the stencil's cell order): try that first, search else
      int c_lo = 0, c_len = 0, c_base = 0;
      constexpr int kConv = 4;   // entries per lane whose loads go out together
      for (int t0 = 0; t0 < tmax; t0 += kConv) {
        int jv[kConv];
#pragma unroll
        for (int u = 0; u < kConv; ++u)
          jv[u] = t0 + u < cnt ? neigh[nl_index(i, (t0 + u) * k + m0, cap, k)] : -1;
#pragma unroll
        for (int u = 0; u < kConv; ++u) {
          const int tt = t0 + u;
          if (tt >= cnt) continue;
          const int j = jv[u];
          if ((unsigned)(j - c_lo) >= (unsigned)c_len) {
            int lo = 0, hi = kTileSegs;   // last segment whose first atom is <= j
            while (hi - lo > 1) {
              const int mid = (lo + hi) >> 1;
              if (s_lo[mid] <= j) lo = mid; else hi = mid;
            }
            c_lo = s_lo[lo];
            c_len = s_len[lo];
            c_base = s_base[lo];
          }
          const int off = j - c_lo;
          const bool in = off >= 0 && off < c_len;
          if (!in) atomicOr(&status[MD_ST_ERRORS], 4);
          row0[(size_t)(tt >> 1) * (2 * kWave) + (tt & 1)] =
              (unsigned short)(in ? c_base + off : 0);
        }
      }
    }
    __syncthreads();   // segment tables are reused by the next run
  }
}

inline unsigned blocks_for(int64_t n, int per = kBlock) { return (unsigned)((n + per - 1) / per); }

}  // namespace

bool tile_geom(int64_t n, const int nc[3], TileGeom* g) {
  if (nc[0] < 4 || nc[1] < 3 || nc[2] < 3 || n < 1) return false;
  const double per_cell = (double)n / ((double)nc[0] * nc[1] * nc[2]);
  const int rmax = std::min(kTileMaxR, (nc[0] - 2) & ~1);
  const int cap_atoms = kTileLdsBytes / (3 * (int)sizeof(double));
  for (int R = rmax; R >= 2; R -= 2) {
    const double mean = 9.0 * (R + 2) * per_cell;
    // room for density fluctuations: the mean plus eight standard deviations
    const int need = (int)std::ceil(mean + 8.0 * std::sqrt(mean) + 64.0);
    const int wcap = (need + 63) & ~63;
    if (wcap <= cap_atoms) {
      g->nc[0] = nc[0];
      g->nc[1] = nc[1];
      g->nc[2] = nc[2];
      g->R = R;
      g->runs_x = (nc[0] + R - 1) / R;
      g->wcap = wcap;
      return true;
    }
  }
  return false;
}

size_t tile_list_entries(int64_t n, int cap, const TileGeom& g) {
  size_t most = 0;
  for (int k = 1; k <= kTileMaxK; k *= 2)
    most = std::max(most, tile_groups((int)n, k, tile_nruns(g)) * tile_words(cap, k) * kWave * 2);
  return most;
}

hipError_t launch_tile_convert(const int* neigh, const int* numneigh, int n, int cap, int k,
                               const int* cell_start, const TileGeom& g, unsigned short* tile,
                               int* status, const int* gate, hipStream_t s) {
  k_tile_convert<<<resident_grid(8, tile_nruns(g)), kBlock, 0, s>>>(
      neigh, numneigh, n, cap, k, cell_start, g, tile, status, gate);
  return hipGetLastError();
}

unsigned resident_grid(int per_cu, int64_t need) {
  // compute-unit count per device, looked up once
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cus[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        v <= 0)
      v = 256;
    cus[dev] = v;
  }
  const int64_t g = ((int64_t)cus[dev] * per_cu + kXcds - 1) / kXcds * kXcds;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, need));
}

hipError_t launch_fill_double(double* p, int64_t count, double value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_fill_double<<<blocks_for(count), kBlock, 0, s>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_halve(int* neigh, int* numneigh, int n, int cap, int layout, hipStream_t s) {
  k_halve<<<blocks_for(n), kBlock, 0, s>>>(neigh, numneigh, n, cap, layout);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int64_t count, int value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_fill_int<<<blocks_for(count), kBlock, 0, s>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_bin_count(double* x, int n, BoxK box, const int nc[3], int* atom_cell,
                            int* count, int* slot, hipStream_t s) {
  k_bin_count<<<blocks_for(n), kBlock, 0, s>>>(x, n, box, nc[0], nc[1], nc[2], atom_cell, count,
                                                slot);
  return hipGetLastError();
}

hipError_t launch_scatter(const int* atom_cell, const int* slot, const int* cell_start, int n,
                          int* tmp_perm, const int* gate, hipStream_t s) {
  k_scatter<<<blocks_for(n), kBlock, 0, s>>>(atom_cell, slot, cell_start, n, tmp_perm, gate);
  return hipGetLastError();
}

hipError_t launch_cell_sort(const int* tmp_perm, const int* cell_start, int ncell, int* perm,
                            const double* x, const double* v, const int* id, const double* f,
                            const int* type, int n, double* sx, double* sv, int* sid,
                            double* sf, int* stype, const int* gate, hipStream_t s) {
  k_cell_sort<<<blocks_for((int64_t)ncell * kWave), kBlock, 0, s>>>(
      tmp_perm, cell_start, ncell, perm, x, v, id, f, type, n, sx, sv, sid, sf,
      type ? stype : nullptr, gate);
  return hipGetLastError();
}

size_t sort_words(int64_t ncell) {
  return (size_t)((ncell + kSortCells - 1) / kSortCells) + 2;
}

hipError_t launch_sort_clear(unsigned long long* lb, int64_t ncell, hipStream_t s) {
  return launch_fill_int(reinterpret_cast<int*>(lb), 2 * (int64_t)sort_words(ncell), 0, s);
}

hipError_t launch_sort_cells(const int* old_start, int* new_start, const int* atom_cell,
                             const int nc[3], BoxK box, const double* boxd, int* perm,
                             const double* xq, const double* v, const int* id, const int* type,
                             int n, double* sx, double* sv, int* sid, int* stype, int* status,
                             unsigned long long* lb, const int* gate, hipStream_t s) {
  const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
  k_sort_cells<<<(unsigned)((ncell + kSortCells - 1) / kSortCells), kSortBlock, 0, s>>>(
      old_start, new_start, atom_cell, nc[0], nc[1], nc[2], box, boxd, perm, xq, v, id, type, n,
      sx, sv, sid, type ? stype : nullptr, status, lb, gate);
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

// The row path needs a run's slabs (kMaxSlabs x 9 cells) in LDS.  It is
// taken when their mean count plus three standard deviations of an ideal
// gas's count (a liquid or solid varies less) fits kRowCap, so that runs
// falling back to one cell at a time stay rare; denser cells (long cutoffs)
// would fall back everywhere, and the general path with home pieces is taken.
hipError_t launch_build(const BuildArgs& a, hipStream_t s) {
  const int64_t ncell = (int64_t)a.nc[0] * a.nc[1] * a.nc[2];
  const double per_cell = (double)a.n / (double)ncell;
  const double run = kMaxSlabs * 9 * per_cell;
  if (a.sorted && a.nc[0] >= 3 && run + 3.0 * std::sqrt(run) <= kRowCap) {
    const int64_t segs = (int64_t)((a.nc[0] + kRowCells - 1) / kRowCells) * a.nc[1] * a.nc[2];
    // one workgroup per row segment: the hardware deals the segments, whose
    // work varies with their atom counts, to the CUs as they free up (a
    // resident grid taking a fixed share each was 5 % slower, its tail the
    // workgroups with one segment more)
    k_build_rows<<<(unsigned)segs, kBlock, 0, s>>>(a);
  } else {
    // pieces of kHomePiece home atoms at the mean occupancy; denser cells
    // loop over further pieces
    const int parts = (int)std::min<int64_t>(
        64, std::max<int64_t>(1, (int64_t)std::ceil(per_cell / kHomePiece)));
    k_build<<<(unsigned)(ncell * parts), kBlock, 0, s>>>(a, parts);
  }
  return hipGetLastError();
}

}  // namespace md
