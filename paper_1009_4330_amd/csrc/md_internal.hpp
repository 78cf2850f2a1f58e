// Internal declarations of the MI355X MD library: kernel parameter blocks,
// workspace layout and the host-side launchers each .hip file provides.
// All device code is compiled with -ffp-contract=off: every FMA in the force
// math is written out with fma()/fmaf(), and the distance / cutoff / wrap /
// integration arithmetic is evaluated exactly as written.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "md.h"

namespace md {

constexpr int kBlock = 256;          // threads per workgroup (4 wavefronts)
constexpr int kWave = 64;            // CDNA wavefront width
#define kWaveConst 64
constexpr int kReduceBlocks = 512;   // first-stage blocks of the deterministic sums
constexpr int kReduceCols = 8;       // values reduced per thermo / energy pass

// Neighbour-list layout with K lanes per atom (K a power of two in [1, 64]):
// groups of G = 64 / K consecutive atoms share rows of 64 ints, and entry m of
// atom i lives at ((i / G) * ceil(cap / K) + m / K) * 64 + (i % G) * K + m % K.
// Lane (i % G) * K + s of a wavefront reads entries m = s, s + K, ... of atom
// i, so each row of 64 entries is one contiguous 256-byte read.  K = 1 is the
// thread-per-atom list, K = 64 one row-major list per atom.
__host__ __device__ inline size_t nl_rows(int cap, int k) { return (size_t)((cap + k - 1) / k); }
__host__ __device__ inline size_t nl_index(int i, int m, int cap, int k) {
  const int g = kWaveConst / k;
  return ((size_t)(i / g) * nl_rows(cap, k) + (size_t)(m / k)) * kWaveConst + (i % g) * k + m % k;
}
inline bool lanes_ok(int k) { return k >= 1 && k <= 64 && (k & (k - 1)) == 0; }

// MI355X spreads the workgroups of a dispatch round-robin over its 8 XCDs, each
// with its own L2.  Renumbering so that XCD x runs one contiguous range of
// logical blocks keeps each XCD's gathers (neighbour positions of cell-sorted
// atoms) inside its own L2 instead of every XCD touching the whole box.
constexpr int kXcds = 8;
__device__ inline int xcd_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  const int q = nb / kXcds, r = nb % kXcds;
  const int xcd = b % kXcds, local = b / kXcds;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}
// Logical blocks [0, nb) worked through by a grid of any size (a resident
// grid looping over its share): the blocks of XCD x (physical blocks
// x, x + 8, ...) take the contiguous chunk x of the logical range in strides
// of their own count, so neighbouring logical blocks still share an L2.
struct BlockRange {
  int first, end, step;
};
__device__ inline BlockRange xcd_range(int nb) {
  const int p = blockIdx.x, g = gridDim.x;
  const int xcd = p % kXcds, local = p / kXcds;
  const int phys = g / kXcds + (xcd < g % kXcds ? 1 : 0);   // physical blocks on this XCD
  const int q = nb / kXcds, r = nb % kXcds;
  const int lo = xcd * q + (xcd < r ? xcd : r);
  return BlockRange{lo + local, lo + q + (xcd < r ? 1 : 0), phys};
}


// Periodic box as kernels see it: edges and their reciprocals (the reciprocal
// only picks the image index; the image shift itself is d - L * k).
struct BoxK {
  double L[3];
  double inv[3];
};

// The box of a run whose box lives in device memory (NPT): edges at Ld[0..2],
// reciprocals formed here exactly as the host forms them.
__device__ inline BoxK box_load(const double* Ld) {
  BoxK b;
  for (int d = 0; d < 3; ++d) {
    b.L[d] = Ld[d];
    b.inv[d] = 1.0 / Ld[d];
  }
  return b;
}

// Wrap one coordinate into [0, L): x - L floor(x / L), an exact L mapped to 0.
__device__ inline double wrap_coord(double x, double L) {
  double r = x - L * floor(x / L);
  if (r < 0.0) r += L;
  if (r >= L) r = 0.0;
  return r;
}

// Cell coordinate floor(r nc / L) of a wrapped coordinate, clamped to [0, nc).
__device__ inline int cell_coord(double r, int nc, double L) {
  int c = (int)((r * (double)nc) / L);
  return c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
}

// Cell of the wrapped image of (x, y, z), x fastest.
__device__ inline int cell_of(double x, double y, double z, const BoxK& box, const int* nc) {
  return cell_coord(wrap_coord(x, box.L[0]), nc[0], box.L[0]) +
         nc[0] * (cell_coord(wrap_coord(y, box.L[1]), nc[1], box.L[1]) +
                  nc[1] * cell_coord(wrap_coord(z, box.L[2]), nc[2], box.L[2]));
}

// Where the integrator records each atom's cell after the drift (the cell of
// its wrapped image), for the gated rebuild; atom_cell == null skips it.
// Packed position record of atom i: (x, y, z, 0) at xq[4 i], 32-byte aligned.
// Packed record of atom i: x, y, z and the atom's species (as a double; 0
// for single-species potentials).
__device__ inline void store_packed(double* xq, int i, double x, double y, double z,
                                    int type = 0) {
  double2* q = reinterpret_cast<double2*>(xq + 4 * (size_t)i);
  q[0] = make_double2(x, y);
  q[1] = make_double2(z, (double)type);
}

// The integrator also refreshes the packed positions the force kernels read.
struct BinOut {
  BoxK box;
  const double* boxd;   // nullable: the box in device memory (overrides box)
  int nc[3];
  int* atom_cell;
  double* xq;    // nullable: packed [n][4] copy of x
  int* flag;     // the rebuild-request word this drift sets
  const int* type;   // nullable: species per atom (stored in the packed records)
};

// Flags of a drift: a rebuild request (to bin.flag) when |x - x_ref|^2 >
// (skin/2)^2 and a non-finite value; one atomic per wavefront for each (every lane of the
// wavefront calls it; `live` lanes own an atom).  With bin.atom_cell, the cell
// of the atom's wrapped image is recorded (the gated rebuild sorts by it);
// with bin.xq, the packed position.
__device__ inline void drift_flags(const double* xn, const double* dd, double trig2, int i,
                                   bool finite, bool live, int* status, const BinOut& bin) {
  const double d2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
  const unsigned long long far = __ballot(live && d2 > trig2);
  const unsigned long long bad = __ballot(live && !finite);
  const bool leader = (threadIdx.x & (kWave - 1)) == 0;
  if (leader && far) atomicOr(bin.flag, 1);
  if (leader && bad) atomicOr(&status[MD_ST_ERRORS], 2);
  if (live && bin.atom_cell)
    bin.atom_cell[i] = cell_of(xn[0], xn[1], xn[2], bin.boxd ? box_load(bin.boxd) : bin.box,
                               bin.nc);
  if (live && bin.xq) store_packed(bin.xq, i, xn[0], xn[1], xn[2], bin.type ? bin.type[i] : 0);
}

// Velocity-Verlet work a force kernel does for each atom once its force is
// summed (md_step), so that no separate integration pass reads the state:
//   MD_INT_NONE:  store f (and energy / virial) only;
//   MD_INT_STEP:  closing kick of this step (v += dtfm f; |v|^2 to keatom when
//                 set), the next step's kick and drift (x from the packed
//                 positions the kernel read, the result to bin.xq, a buffer
//                 the kernel does not read) and its displacement check;
//   MD_INT_LAST:  closing kick only, then f and x stored in the state.
enum { MD_INT_NONE = 0, MD_INT_STEP = 1, MD_INT_LAST = 2 };
struct IntArgs {
  int mode;
  double* v;
  const double* xr;      // x_ref of the current list
  double* x;             // state positions (MD_INT_LAST)
  double* keatom;        // nullable: |v|^2 of the full-step velocity
  int* status;
  double dtfm, dt, trig2;
  BinOut bin;            // drift outputs (MD_INT_STEP)
  const double* kick;    // nullable (NPT): the closing kick is v a + (dtfm f) b, (a, b) = kick[0..1]
};

// Lennard-Jones constants in both precisions.
struct LJK {
  double rc2, sig2, eps4, eps24, eps48, ecut;
  float sig2f, eps4f, eps24f, eps48f, ecutf;
  double inv_sig;   // 1/sigma, for dg/dsigma in the adjoint
};

// Sutton-Chen constants.
struct SCK {
  double rc2, a2, eps, neps, mepsc_half, epsc;
  double meps_half, c;          // (m/2) eps (the embedding pair factor per unit c), c
  float a2f, nepsf, mepsc_halff, meps_halff, cf;
  int n, m;
};

// Buckingham + cut Coulomb: per species pair ab = a * 4 + b the row
// A, A / rho, 1 / rho, C, 6 C, qqr2e q_a q_b (A / rho and 1 / rho are 0 where
// A is), in FP64 and FP32 (whose 1 / rho is scaled by log2(e) for a base-2
// exponential).
struct BuckK {
  double rc2;
  double row[16][6];
  float rowf[16][6];
};

// Where per-atom energy / virial / kinetic terms go for the thermo sums.
struct EVOut {
  double* eatom;   // [n] or null
  double* vatom;   // [6][n] or null
  // [n] or null: half atom i's virial trace (w_xx + w_yy) + w_zz, the value
  // the barostat sums.  Alone (eatom and vatom null) it asks the LJ kernel for
  // that trace only, with fused integration; the other kernels then evaluate
  // everything and store just the trace.
  double* vtrace;
};

// Workspace carve-up (offsets in bytes from the workspace base).
struct WsLayout {
  size_t count;      // int [ncell]       per-cell counters (kept zero between uses)
  size_t slot;       // int [n]           arrival slot of each atom in its cell
  size_t tmp_perm;   // int [n]           unsorted cell members
  size_t tmp_x;      // double [3][n]     sorted staging of x
  size_t tmp_v;      // double [3][n]     sorted staging of v
  size_t tmp_f;      // double [3][n]     sorted staging of f / x_ref
  size_t tmp_id;     // int [n]           sorted staging of ids
  size_t tmp_type;   // int [n]           sorted staging of species
  size_t eatom;      // double [n]
  size_t vatom;      // double [6][n]
  size_t keatom;     // double [n]
  size_t vtrace;     // double [n]        virial trace (NPT)
  size_t sc_e;       // double [n]        Sutton-Chen rho^-1/2
  size_t partials;   // double [kReduceBlocks][kReduceCols]
  size_t scalars;    // double [16]       reduced values
  size_t sortlb;     // u64 [sort_words] look-back words of the rebuild sort
  size_t new_start;  // int [ncell + 1]   cell starts of a rebuild in progress
  size_t xq;         // double [n][4]     packed positions (x, y, z, 0) for the force gathers
  size_t xq2;        // double [n][4]     second packed buffer (md_step alternates the two)
  size_t total;
};

WsLayout ws_layout(int64_t n, int64_t ncell);

// ------------------------------------------------------------ launchers --
// Every launcher enqueues on `s` and returns hipGetLastError().

// Binning.  `gate` (nullable) makes the kernels return at once when *gate == 0.
// launch_bin_count wraps x in place, bins and adds to the per-cell counters
// (zero on entry) and records each atom's arrival slot in its cell.
// launch_scan_cells turns the counts into cell_start.
hipError_t launch_fill_int(int* p, int64_t count, int value, hipStream_t s);
// Workgroups that fit on the current device at once with `per_cu` of them per
// compute unit (a multiple of 8), capped at `need`.
unsigned resident_grid(int per_cu, int64_t need);

hipError_t launch_bin_count(double* x, int n, BoxK box, const int nc[3], int* atom_cell,
                            int* count, int* slot, hipStream_t s);
hipError_t launch_scan_cells(const int* count, int ncell, int* cell_start, hipStream_t s);
hipError_t launch_scatter(const int* atom_cell, const int* slot, const int* cell_start, int n,
                          int* tmp_perm, const int* gate, hipStream_t s);
// Stable order inside each cell; optionally gathers x, v, id, species (and
// f) into the sorted staging buffers (null destinations are skipped).
hipError_t launch_cell_sort(const int* tmp_perm, const int* cell_start, int ncell, int* perm,
                            const double* x, const double* v, const int* id, const double* f,
                            const int* type, int n, double* sx, double* sv, int* sid,
                            double* sf, int* stype, const int* gate, hipStream_t s);
// Rebuild-time sort for atoms already in the previous build's cell order that
// moved less than a cell edge, with atom_cell holding their new cells, in one
// launch: each new cell's members counted among the old ranges of its 27
// neighbours, the new cell starts (a decoupled look-back over super-cells of
// consecutive cells, in the words lb of sort_words(ncell) 64-bit entries, zeroed by
// launch_sort_clear before the first use and left zeroed by every sort), and
// the state (x wrapped) gathered into staging in the stable order.  Status
// bit 2 is set if the counts do not add up to n (some atom moved further).
size_t sort_words(int64_t ncell);
hipError_t launch_sort_clear(unsigned long long* lb, int64_t ncell, hipStream_t s);
hipError_t launch_sort_cells(const int* old_start, int* new_start, const int* atom_cell,
                             const int nc[3], BoxK box, const double* boxd, int* perm,
                             const double* xq, const double* v, const int* id, const int* type,
                             int n, double* sx, double* sv, int* sid, int* stype, int* status,
                             unsigned long long* lb, const int* gate, hipStream_t s);
hipError_t launch_copy_back(double* x, double* v, int* id, double* f, double* xr,
                            const double* sx, const double* sv, const int* sid,
                            const double* sf, int n, hipStream_t s);

hipError_t launch_gather3(const int* perm, int n, const double* src, double* dst,
                          hipStream_t s);
hipError_t launch_gather_int(const int* perm, int n, const int* src, int* dst, hipStream_t s);

// Neighbour list.  sorted == 0: x is in input order and the members of cell c
// are perm[cell_start[c] .. cell_start[c+1]); sorted != 0: x is in cell order
// (slot k holds atom perm[k]) and the members are the slots themselves.  With
// x_out (md_step), x is the sorted staging buffer and the same kernel copies
// the state (x, v, id) back from staging.
struct BuildArgs {
  const double* x;       // positions the list is built from
  int n;
  int sorted;
  BoxK box;
  int nc[3];
  const int* cell_start;
  int* cell_start_out;   // nullable: receives a copy of cell_start
  const int* atom_cell;  // cell of each atom, input order
  const int* perm;
  double rl2;
  int cap, layout;
  int* neigh;
  int* numneigh;
  double* x_ref;
  int* status;
  double* xq_out;        // nullable: packed [n][4] copy of the home atoms' positions
  // md_step extras
  double* x_out;
  double* v_out;
  const double* v_in;
  int* id_out;
  const int* id_in;
  int* type_out;         // nullable: species copied back like id
  const int* type_in;    // nullable: species of the home atoms (for xq_out and type_out)
  const int* gate;
  const double* boxd;    // nullable: the box in device memory (overrides box)
  double* lref;          // nullable: receives the box edges of this build (NPT)
};
hipError_t launch_build(const BuildArgs& a, hipStream_t s);

// k-th smallest of the distinct cells {c - 1, c, c + 1} of a periodic
// dimension with nc cells (min(nc, 3) of them).
__device__ inline int nbr_sorted(int c, int nc, int k) {
  if (nc < 3) return k;
  if (c == 0) return k == 2 ? nc - 1 : k;
  if (c == nc - 1) return k == 0 ? 0 : nc - 3 + k;
  return c - 1 + k;
}

// Rank of c among the distinct cells {c - 1, c, c + 1} in increasing order
// (see nbr_sorted).
__device__ inline int self_rank(int c, int nc) {
  if (nc < 3) return c;
  return c == 0 ? 0 : (c == nc - 1 ? 2 : 1);
}

// ------------------------------------------------ LDS-tiled force kernels --
// Atoms in cell order are grouped into runs of up to R consecutive cells of
// one x row of cells.  The workgroup that owns a run stages its window -- the
// 3 x 3 rows of cells around the run's row (in the sorted order of their
// distinct row indices), each from cell x0 - 1 to x0 + Rr, where every list
// partner of the run's atoms lies -- into LDS, and gathers neighbours there.
// The window of a row is one contiguous range of atoms, or two where it wraps
// around the box in x.  A tile list holds, per entry, the partner's index in
// its run's window (16 bits), in the K-lane row layout with groups of
// G = 64 / K atoms counted from each run's first atom, two consecutive
// entries of a lane in one 32-bit word (entry t = m / K of the lane in half
// t % 2 of word t / 2, so one coalesced load brings each lane two entries):
// with T = ceil(ceil(cap / K) / 2) words per lane, entry m of atom i (run r,
// first atom hb) is 16-bit element
//   (((hb / G + r + (i - hb) / G) * T + m / K / 2) * 64 + ((i - hb) % G) * K + m % K) * 2
//     + (m / K) % 2.
constexpr int kTileMaxR = 16;                    // home cells per run, at most
constexpr int kTileSegs = 18;                    // window segments: 9 rows x (1 or 2)
constexpr int kTileMaxK = 8;                     // lanes per atom of the tiled kernels
constexpr int kTileBlock = 512;                  // threads per workgroup of the tiled kernels
constexpr int kTileLdsBytes = 48 * 1024;         // LDS budget of a window's positions
struct TileGeom {
  int nc[3];
  int R;        // home cells per run: even, 2 <= R <= nc[0] - 2
  int runs_x;   // runs per x row: ceil(nc[0] / R)
  int wcap;     // window atoms that fit in LDS (larger windows read positions from memory)
};
__host__ __device__ inline int tile_nruns(const TileGeom& g) {
  return g.runs_x * g.nc[1] * g.nc[2];
}
__host__ __device__ inline size_t tile_groups(int n, int k, int nruns) {
  return (size_t)((n + kWaveConst / k - 1) / (kWaveConst / k)) + (size_t)nruns;
}
// 32-bit words per lane of a tile list row group.
__host__ __device__ inline size_t tile_words(int cap, int k) { return (nl_rows(cap, k) + 1) / 2; }
// 16-bit element of entry m of atom i (run r with first atom hb) in a tile list.
__host__ __device__ inline size_t tile_index(int i, int m, int hb, int r, int cap, int k) {
  const int g = kWaveConst / k;
  const int t = m / k;
  return (((size_t)(hb / g + r + (i - hb) / g) * tile_words(cap, k) + (size_t)(t / 2)) *
              kWaveConst +
          (size_t)(((i - hb) % g) * k + m % k)) * 2 + (size_t)(t % 2);
}
// Tile geometry for n atoms in a grid nc (false: the tiled kernels do not
// apply -- fewer than 4 cells along x or 3 along y / z, or no run's mean
// window fits the LDS budget).
bool tile_geom(int64_t n, const int nc[3], TileGeom* g);
// 16-bit entries a tile list needs for every K the tiled kernels take.
size_t tile_list_entries(int64_t n, int cap, const TileGeom& g);
// Tile list from a full list in layout K (atoms in cell order, cell_start of
// the same build): each partner index becomes its index in the window of the
// atom's run.  Gated like the build.
hipError_t launch_tile_convert(const int* neigh, const int* numneigh, int n, int cap, int k,
                               const int* cell_start, const TileGeom& g, unsigned short* tile,
                               int* status, const int* gate, hipStream_t s);

// Run r of a tile geometry: its row (y, z), first cell x0, cells Rr, and the
// range [hb, he) of its atoms (cell order).
struct TileRun {
  int x0, Rr, y, z, hb, he;
};
__device__ inline TileRun tile_run(const TileGeom& g, int r, const int* __restrict__ cs) {
  TileRun t;
  const int rx = r % g.runs_x, row = r / g.runs_x;
  t.y = row % g.nc[1];
  t.z = row / g.nc[1];
  t.x0 = rx * g.R;
  t.Rr = min(g.R, g.nc[0] - t.x0);
  const int base = (t.z * g.nc[1] + t.y) * g.nc[0];
  t.hb = cs[base + t.x0];
  t.he = cs[base + t.x0 + t.Rr];
  return t;
}
// Segment l (0 <= l < kTileSegs) of run t's window: row e = l / 2 of the 3 x 3
// rows, piece l % 2; [*lo, *lo + *len) in cell order.  A row's cells x0 - 1
// .. x0 + Rr are one range, or two when they wrap in x: (cell nc0 - 1 | cells
// 0 .. Rr) for the first run of a row, (cells x0 - 1 .. nc0 - 1 | cell 0) for
// one ending at the last cell.  Segments in increasing l are the window order.
__device__ inline void tile_segment(const TileGeom& g, const TileRun& t, int l,
                                    const int* __restrict__ cs, int* lo, int* len) {
  const int e = l >> 1, piece = l & 1;
  const int nc0 = g.nc[0];
  const int zr = nbr_sorted(t.z, g.nc[2], e / 3), yr = nbr_sorted(t.y, g.nc[1], e % 3);
  const int base = (zr * g.nc[1] + yr) * nc0;
  int a = 0, b = 0;   // cell range [a, b) of the row
  if (t.x0 == 0) {
    a = piece == 0 ? nc0 - 1 : 0;
    b = piece == 0 ? nc0 : t.Rr + 1;
  } else if (t.x0 + t.Rr == nc0) {
    a = piece == 0 ? t.x0 - 1 : 0;
    b = piece == 0 ? nc0 : 1;
  } else if (piece == 0) {
    a = t.x0 - 1;
    b = t.x0 + t.Rr + 1;
  }
  *lo = cs[base + a];
  *len = cs[base + b] - *lo;
}
// The window segment holding the run's own atoms (the run's row, the piece
// that starts at x0 - 1, or at x0 = 0 for the first run of a row).
__device__ inline int tile_home_segment(const TileGeom& g, const TileRun& t) {
  const int e = self_rank(t.z, g.nc[2]) * 3 + self_rank(t.y, g.nc[1]);
  return 2 * e + (t.x0 == 0 ? 1 : 0);
}

// Forces.  kernel: MD_KERNEL_TPA / MD_KERNEL_WPA.  clear (nullable) is zeroed
// by the first thread, after every rebuild kernel of the step has finished.
// Positions come packed: atom i at xq[4 i .. 4 i + 2], xq[4 i + 3] = 0, so one
// neighbour is one aligned 32-byte record (two loads, one cache line).
struct ForceArgs {
  const double* xq;
  int n;
  BoxK box;
  double margin;         // interior margin r_l + skin = 2 r_l - r_c (+inf: always wrap)
  const int* neigh;
  const int* numneigh;
  int cap;
  double* f;
  EVOut ev;
  int* clear;
  hipEvent_t t0, t1;     // non-null: timed launch
  IntArgs in;            // mode MD_INT_NONE unless md_step fuses integration
  // tiled kernels (kernel K | MD_LAYOUT_TILE): the tile list, the cell starts
  // of its build and the geometry
  const unsigned short* tile;
  const int* cell_start;
  TileGeom tg;
  const double* boxd;    // nullable: the box in device memory (overrides box)
};
hipError_t launch_pack_positions(const double* x, int n, double* xq, const int* type,
                                 hipStream_t s);
hipError_t launch_buck(const ForceArgs& a, const BuckK& p, int prec, int lanes, hipStream_t s);
// LJ from a half list: f must be zero on entry (forces are added atomically).
hipError_t launch_lj_half(const ForceArgs& a, const LJK& p, int prec, int lanes, hipStream_t s);
// Keep only the partners j > i of each row, in order (in place).
hipError_t launch_halve(int* neigh, int* numneigh, int n, int cap, int layout, hipStream_t s);
hipError_t launch_fill_double(double* p, int64_t count, double value, hipStream_t s);
hipError_t launch_lj(const ForceArgs& a, const LJK& p, int prec, int kernel, hipStream_t s);
hipError_t launch_sc(const ForceArgs& a, const SCK& p, int prec, int kernel, double* sc_e,
                     hipStream_t s);
// LJ force adjoint: gx = (dF/dx)^T u and, with bp set, per-workgroup sums of
// u_i . F_i and of the sigma term in rows of two doubles (*rows of them, in
// atom order), for launch_sum_parts.
hipError_t launch_lj_vjp(const ForceArgs& a, const LJK& p, int prec, int lanes,
                         const double* u, double* gx, double* bp, int* rows, hipStream_t s);

// Integration.
// scale (device scalar, nullable): v is multiplied by it before the kick.
hipError_t launch_kick_drift_check(double* x, double* v, const double* f, const double* xr,
                                   int n, double dtfm, double dt, double trig2, int* status,
                                   const BinOut& bin, const double* scale, hipStream_t s);
// v *= *scale.
hipError_t launch_scale_v(double* v, int n, const double* scale, hipStream_t s);

// Nose-Hoover chain update (one thread).  ke2 = mke * (*vsum) (sum m v^2 in
// energy units) or, with vsum null, the value carried in the state.  end:
// the half step closing a step (vsum_out, if set, receives vsum times the
// square of its factor, for the thermo row); then the chain energy is stored;
// start: the half step opening the next step.  The product of the factors
// is stored in the state's scale word.
struct NhcArgs {
  double* state;
  int M;
  double Q0, Qj, kT, nf, dt, mke;
  const double* vsum;
  double* vsum_out;
  int end, start;
};
hipError_t launch_nhc(const NhcArgs& a, hipStream_t s);
constexpr int kNhcEnergy = 16, kNhcScale = 17, kNhcKe2 = 18;   // state words after the chain
hipError_t launch_ke(const double* v, int n, double* keatom, hipStream_t s);

// Parameter gradients of the force adjoints, finished from their two sums
// (out[0], out[1]) on the sum's last stage.  LJ: dL/deps = out[0] / eps,
// dL/dsigma = out[1].  Sutton-Chen, with L = LA + c LB, LA ~ a^n and
// c LB ~ a^(m/2): dL/deps = (LA + c LB) / eps, dL/da = (n LA + m/2 c LB) / a,
// dL/dc = LB.
enum { kParamsNone = 0, kParamsLJ = 1, kParamsSC = 2 };
struct ParamArgs {
  int kind = kParamsNone;
  double eps = 1.0, a = 1.0, c = 0.0, nexp = 0.0, mexp = 0.0;
  double* gparam = nullptr;
};

// Deterministic sums: cols arrays of n doubles (col c at base[c]; a null
// column sums to 0) -> out[cols]; then, with params.kind set, the adjoint's
// parameter gradients from out.
struct SumArgs {
  const double* col[kReduceCols];
  int cols;
  int n;
  double* partials;
  double* out;
  ParamArgs params;
  // 0: the partials are stage 1's (kReduceBlocks rows of kReduceCols);
  // otherwise nparts rows of cols each, written by the caller's kernel
  int nparts;
};
struct NhcArgs;
// With nhc, the thermostat chain update (launch_nhc) runs at the end of the
// sum's last stage, on the sums it wrote.
hipError_t launch_sum(const SumArgs& a, hipStream_t s, const NhcArgs* nhc = nullptr);
// The last stage alone, over a.nparts rows of partials another kernel wrote.
hipError_t launch_sum_parts(const SumArgs& a, hipStream_t s);
// Thermo row from out = {pe, W0..W5, sv} sums.
struct ThermoArgs {
  const double* sums;  // pe, w0..w5, sum v^2
  const double* extra; // nullable: an energy added to pe + ke in a ninth column
  double* row;
  double step, mass, mvv2e, boltz, dof, volume;
  const int* status;
  const double* vol;   // nullable (NPT): the volume in device memory, also a tenth column
};
hipError_t launch_thermo_row(const ThermoArgs& a, hipStream_t s);
// Sutton-Chen adjoint: density pass into e, then the pass for lam (dL/drho),
// la and lb (per-atom parameter sums) and the packed (u_i, lam_i) records uq
// ([n][4] scratch), then the position pass into gx.
hipError_t launch_sc_vjp(const ForceArgs& a, const SCK& p, int prec, int lanes, const double* u,
                         double* e, double* lam, double* la, double* lb, double* uq, double* gx,
                         hipStream_t s);

// ------------------------------------------------------------------ NPT --
// Barostat state (md_step_npt), doubles of md_npt.state: both chains, the
// barostat momentum, the box, the box of the last build, and the factors the
// update kernel leaves for the step's kick / drift kernels.
enum {
  kNptEta = 0,          // particle chain positions [MD_NHC_MAX]
  kNptVeta = 8,         // particle chain velocities
  kNptXi = 16,          // barostat chain positions
  kNptVxi = 24,         // barostat chain velocities
  kNptPeps = 32,        // barostat momentum
  kNptL = 33,           // box edges [3]
  kNptLref = 36,        // box edges at the last build [3]
  kNptScale = 39,       // velocity scale (particle thermostat) before the next kick
  kNptKa = 40,          // kick factors a, b: v <- v a + (dtfm f) b
  kNptKb = 41,
  kNptDc = 42,          // drift factors c, e: x <- x c + e v
  kNptDe = 43,
  kNptSb = 44,          // box scale since the last build
  kNptThr2 = 45,        // rebuild bound squared (negative: rebuild)
  kNptKe2 = 46,         // scaled kinetic term carried to the next half step
  kNptEnergy = 47,      // extended energy beyond pe + ke (thermo)
  kNptVol = 48,         // volume
  kNptWords = 49
};
struct NptArgs {
  double* state;
  int M;
  double Q0, Qj, Qb, W, kT, nf, alpha, dt, mke, ptarget, skin, rl;
  int nc[3];            // cell grid of the run: the box must keep L_d >= nc_d rl
  int* status;
  const double* vsum;   // sum v^2 (from the sums), or null: the carried kinetic term
  const double* trw;    // the virial trace summed over the atoms (enters G_eps)
  double* vsum_out;     // nullable: sum v^2 after the closing half step (thermo)
  int end, start;
};
// Barostat / thermostat update (the first wavefront) at the end of the sum's last
// stage: with end, the closing half of a step (G_eps half step, particle
// chain, barostat chain; the extended energy stored); with start, the
// opening half of the next (barostat chain, particle chain, G_eps half step,
// the new box and the factors of its kick and drift).
hipError_t launch_sum_npt(const SumArgs& a, const NptArgs& npt, hipStream_t s);
// v <- v scale; v <- v a + (dtfm f) b; x <- x c + e v; rebuild request when
// |x - sb x_ref|^2 > thr2 (or thr2 < 0); cell of each atom in the new box.
hipError_t launch_kick_drift_npt(double* x, double* v, const double* f, const double* xr, int n,
                                 double dtfm, int* status, const BinOut& bin,
                                 const double* state, hipStream_t s);

}  // namespace md
