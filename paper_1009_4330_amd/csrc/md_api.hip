// C ABI of the MD hot path: argument validation, workspace carve-up, and the
// orchestration of the kernels in md_bin.hip, md_forces.hip and
// md_integrate.hip.  Nothing here allocates device memory.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "md_internal.hpp"

using namespace md;

namespace {

#define MD_CK(call)                                   \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return MD_ERR_HIP;          \
  } while (0)

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

md_status check_box(const md_box* box, double rl) {
  if (!box || !finite_pos(rl)) return MD_ERR_INVALID_ARG;
  for (int d = 0; d < 3; ++d) {
    if (!finite_pos(box->L[d])) return MD_ERR_INVALID_ARG;
    if (!(box->L[d] > 2.0 * rl)) return MD_ERR_BOX_TOO_SMALL;
  }
  return MD_OK;
}

bool cell_dims(const md_box* box, double rl, int nc[3], int64_t* ncell) {
  int64_t prod = 1;
  for (int d = 0; d < 3; ++d) {
    const double q = std::floor(box->L[d] / rl);
    if (!(q >= 1.0) || q > 1e6) return false;
    nc[d] = (int)q;
    prod *= nc[d];
  }
  if (prod > INT_MAX / 2) return false;
  *ncell = prod;
  return true;
}

// Margin of the interior fast path: an atom at least r_l + skin = 2 r_l - r_c
// from every face has all its list partners in its own periodic image.
double interior_margin(const md_potential* p, double rl) {
  return rl > p->rc ? 2.0 * rl - p->rc : HUGE_VAL;
}

BoxK make_box(const md_box* b) {
  BoxK k;
  for (int d = 0; d < 3; ++d) {
    k.L[d] = b->L[d];
    k.inv[d] = 1.0 / b->L[d];
  }
  return k;
}

bool n_ok(int64_t n) { return n >= 1 && n <= (int64_t)MD_MAX_ATOMS; }

// Lanes per atom of a list layout (the tiled flag off) and whether a layout
// value is valid: K a power of two in [1, 64], or MD_LAYOUT_TILE | K with
// K <= kTileMaxK.
int lanes_of(int layout) { return layout & ~MD_LAYOUT_TILE; }
bool is_tile(int layout) { return (layout & MD_LAYOUT_TILE) != 0; }
bool layout_ok(int layout) {
  const int k = lanes_of(layout);
  return lanes_ok(k) && (!is_tile(layout) || k <= kTileMaxK);
}

// Whether the list's tile buffer covers the tiled layouts of n atoms in the
// grid nc (and the grid takes them); fills the geometry.
bool tile_fits(const md_nlist* nl, int64_t n, const int nc[3], TileGeom* tg) {
  return nl->tile && !nl->half && tile_geom(n, nc, tg) &&
         nl->tile_entries >= tile_list_entries(n, nl->capacity, *tg);
}

md_status check_pot(const md_potential* p) {
  if (!p || !finite_pos(p->rc)) return MD_ERR_INVALID_ARG;
  if (p->kind == MD_POT_LJ) {
    if (!finite_pos(p->lj_eps) || !finite_pos(p->lj_sigma)) return MD_ERR_INVALID_ARG;
    return MD_OK;
  }
  if (p->kind == MD_POT_SC) {
    if (!finite_pos(p->sc_eps) || !finite_pos(p->sc_a) || !std::isfinite(p->sc_c) ||
        p->sc_n < 1 || p->sc_m < 1 || p->sc_n > 64 || p->sc_m > 64)
      return MD_ERR_INVALID_ARG;
    return MD_OK;
  }
  if (p->kind == MD_POT_BUCK) {
    if (!p->type || !finite_pos(p->qqr2e)) return MD_ERR_INVALID_ARG;
    for (int q = 0; q < 4; ++q)
      if (!std::isfinite(p->q[q])) return MD_ERR_INVALID_ARG;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const int ab = 4 * a + b, ba = 4 * b + a;
        const double A = p->buck_A[ab], rho = p->buck_rho[ab], C = p->buck_C[ab];
        if (!(A >= 0.0) || !std::isfinite(A) || !(C >= 0.0) || !std::isfinite(C))
          return MD_ERR_INVALID_ARG;
        if (A > 0.0 && !finite_pos(rho)) return MD_ERR_INVALID_ARG;
        if (A != p->buck_A[ba] || C != p->buck_C[ba] ||
            (A > 0.0 && rho != p->buck_rho[ba]))
          return MD_ERR_INVALID_ARG;
      }
    return MD_OK;
  }
  return MD_ERR_INVALID_ARG;
}

// Species of the atoms a call works on (Buckingham only; the other kinds
// ignore species and read none).
const int* species(const md_potential* p) { return p->kind == MD_POT_BUCK ? p->type : nullptr; }

BuckK make_buck(const md_potential* p) {
  BuckK k;
  k.rc2 = p->rc * p->rc;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const int ab = 4 * a + b;
      const double A = p->buck_A[ab];
      const double irho = A > 0.0 ? 1.0 / p->buck_rho[ab] : 0.0;
      const double row[6] = {A, A * irho, irho, p->buck_C[ab], 6.0 * p->buck_C[ab],
                             p->qqr2e * p->q[a] * p->q[b]};
      // the FP32 row's 1 / rho carries log2(e): e^(-r / rho) = 2^(-r log2(e) / rho)
      // for the hardware base-2 exponential
      for (int c = 0; c < 6; ++c) {
        k.row[ab][c] = row[c];
        k.rowf[ab][c] = (float)(c == 2 ? row[c] * 1.4426950408889634 : row[c]);
      }
    }
  return k;
}

LJK make_lj(const md_potential* p) {
  LJK k;
  const double eps = p->lj_eps, sig = p->lj_sigma;
  k.rc2 = p->rc * p->rc;
  k.sig2 = sig * sig;
  k.eps4 = 4.0 * eps;
  k.eps24 = 24.0 * eps;
  k.eps48 = 48.0 * eps;
  k.ecut = 0.0;
  if (p->lj_shift) {
    const double r = k.sig2 / k.rc2;
    const double sr6 = r * r * r;
    k.ecut = k.eps4 * (sr6 * sr6 - sr6);
  }
  k.sig2f = (float)k.sig2;
  k.eps4f = (float)k.eps4;
  k.eps24f = (float)k.eps24;
  k.eps48f = (float)k.eps48;
  k.ecutf = (float)k.ecut;
  k.inv_sig = 1.0 / sig;
  return k;
}

SCK make_sc(const md_potential* p) {
  SCK k;
  k.rc2 = p->rc * p->rc;
  k.a2 = p->sc_a * p->sc_a;
  k.eps = p->sc_eps;
  k.neps = p->sc_n * p->sc_eps;
  k.mepsc_half = 0.5 * p->sc_m * p->sc_eps * p->sc_c;
  k.epsc = p->sc_eps * p->sc_c;
  k.meps_half = 0.5 * p->sc_m * p->sc_eps;
  k.c = p->sc_c;
  k.meps_halff = (float)k.meps_half;
  k.cf = (float)k.c;
  k.a2f = (float)k.a2;
  k.nepsf = (float)k.neps;
  k.mepsc_halff = (float)k.mepsc_half;
  k.n = p->sc_n;
  k.m = p->sc_m;
  return k;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

md_status check_ws(void* ws, size_t ws_bytes, const WsLayout& L) {
  if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MD_ERR_WORKSPACE;
  return MD_OK;
}

// ------------------------------------------------------------ timing --

struct Timing {
  std::mutex mu;
  int every = 0;
  int64_t counter = 0;
  std::vector<hipEvent_t> pool;          // pairs: [2k] start, [2k+1] stop
  size_t used = 0;                       // pairs recorded since the last read
  int64_t launches = 0;
  double total_ms = 0.0;
};
Timing g_timing;
constexpr size_t kTimingPairs = 4096;

// Events for the next force launch, or nulls when this launch is not sampled.
void timing_events(hipEvent_t* t0, hipEvent_t* t1) {
  *t0 = *t1 = nullptr;
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (g_timing.every <= 0) return;
  if (g_timing.counter++ % g_timing.every != 0) return;
  if (g_timing.used >= kTimingPairs || g_timing.pool.size() < 2 * kTimingPairs) return;
  *t0 = g_timing.pool[2 * g_timing.used];
  *t1 = g_timing.pool[2 * g_timing.used + 1];
  ++g_timing.used;
}

// ------------------------------------------------------ AUTO selection --

// Key: device, potential kind, precision, log2 buckets of the largest
// neighbour count and of the atom count (the winner moves with both: a small
// system needs more lanes per atom to fill the chip).
using AutoKey = std::tuple<int, int, int, int, int, int>;
std::mutex g_auto_mu;
std::map<AutoKey, md_kernel> g_auto_cache;

int count_bucket(int maxcount) {
  int b = 0;
  while ((1 << b) < maxcount && b < 30) ++b;
  return b;
}

// `tiled`: whether the tiled kernels were among the candidates.
AutoKey auto_key(const md_potential* p, md_precision prec, int maxcount, int n, bool tiled) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return std::make_tuple(dev, p->kind, (int)prec, count_bucket(maxcount), count_bucket(n),
                         tiled ? 1 : 0);
}

md_status force_dispatch(const md_potential* p, const ForceArgs& fa, md_precision prec,
                         int kernel, double* sc_e, hipStream_t s) {
  hipError_t e;
  if (p->kind == MD_POT_LJ)
    e = launch_lj(fa, make_lj(p), prec, kernel, s);
  else if (p->kind == MD_POT_BUCK)
    e = launch_buck(fa, make_buck(p), prec, kernel, s);
  else
    e = launch_sc(fa, make_sc(p), prec, kernel, sc_e, s);
  return e == hipSuccess ? MD_OK : MD_ERR_HIP;
}

// Build a list in `layout` from positions x (sorted or input order).  A tiled
// layout (sorted atoms only) also writes the tile list.
md_status build_list(const double* x, int n, int sorted, const md_box* box, const int nc[3],
                     const md_cells* cells, double rl, md_nlist* nl, int layout,
                     hipStream_t s) {
  TileGeom tg{};
  if (is_tile(layout) && (!sorted || !tile_fits(nl, n, nc, &tg))) return MD_ERR_UNSUPPORTED;
  BuildArgs a{};
  a.x = x;
  a.n = n;
  a.sorted = sorted;
  a.box = make_box(box);
  for (int d = 0; d < 3; ++d) a.nc[d] = nc[d];
  a.cell_start = cells->cell_start;
  a.atom_cell = cells->atom_cell;
  a.perm = cells->perm;
  a.rl2 = rl * rl;
  a.cap = nl->capacity;
  a.layout = lanes_of(layout);
  a.neigh = nl->neigh;
  a.numneigh = nl->numneigh;
  a.x_ref = nl->x_ref;
  a.status = nl->status;
  MD_CK(launch_build(a, s));
  if (nl->half) MD_CK(launch_halve(nl->neigh, nl->numneigh, n, nl->capacity, layout, s));
  if (is_tile(layout))
    MD_CK(launch_tile_convert(nl->neigh, nl->numneigh, n, nl->capacity, lanes_of(layout),
                              cells->cell_start, tg, nl->tile, nl->status, nullptr, s));
  nl->layout = layout;
  nl->rl = rl;
  return MD_OK;
}

// Steps per list build assumed when the mini-benchmark weighs a tiled
// kernel's conversion against its force time (the LJ melt rebuilds about
// every five steps).
constexpr int kTileBuildEvery = 5;

// Time `reps` force launches for every lanes-per-atom count K = 1, 2, ..., 64
// (each with its own list layout) and keep the fastest.  Leaves the list in
// the winner's layout.  The trial builds are not counted as builds of the run.
md_status autoselect_impl(const md_potential* p, const double* x, int n, int sorted,
                          const md_box* box, const md_cells* cells, double rl, md_nlist* nl,
                          md_precision prec, int reps, md_kernel* choice, void* ws,
                          const WsLayout& L, hipStream_t s, bool tiled_ok = true) {
  int nc[3] = {cells->nc[0], cells->nc[1], cells->nc[2]};
  int before[MD_STATUS_WORDS];
  MD_CK(hipMemcpyAsync(before, nl->status, sizeof(before), hipMemcpyDeviceToHost, s));
  MD_CK(hipStreamSynchronize(s));
  hipEvent_t e0, e1;
  MD_CK(hipEventCreate(&e0));
  MD_CK(hipEventCreate(&e1));
  float best = 1e30f;
  int win = MD_KERNEL_TPA;
  int maxcount = 0;
  double* xq = at<double>(ws, L.xq);
  MD_CK(launch_pack_positions(x, n, xq, species(p), s));
  // candidates: K = 1 .. 64, then the tiled K = 1 .. 8 where they apply
  std::vector<int> trials;
  for (int k = 1; k <= kWave; k *= 2) trials.push_back(k);
  TileGeom tg{};
  if (sorted && tiled_ok && p->kind == MD_POT_LJ && tile_fits(nl, n, nc, &tg))
    for (int k = 1; k <= kTileMaxK; k *= 2) trials.push_back(MD_LAYOUT_TILE | k);
  // builds the list in layout k and times reps force evaluations on it
  auto time_k = [&](int k, float* out) -> md_status {
    md_status st = build_list(x, n, sorted, box, nc, cells, rl, nl, k, s);
    if (st != MD_OK) return st;
    ForceArgs fa{};
    fa.xq = xq;
    fa.n = n;
    fa.box = make_box(box);
    fa.margin = interior_margin(p, rl);
    fa.neigh = nl->neigh;
    fa.numneigh = nl->numneigh;
    fa.cap = nl->capacity;
    fa.tile = nl->tile;
    fa.cell_start = cells->cell_start;
    fa.tg = tg;
    fa.f = at<double>(ws, L.tmp_f);   // scratch forces: the caller's f is untouched
    st = force_dispatch(p, fa, prec, k, at<double>(ws, L.sc_e), s);
    if (st != MD_OK) return st;
    MD_CK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) {
      st = force_dispatch(p, fa, prec, k, at<double>(ws, L.sc_e), s);
      if (st != MD_OK) return st;
      // a tiled list is also converted at every build: charge one
      // conversion per kTileBuildEvery force evaluations
      if (is_tile(k) && r % kTileBuildEvery == 0)
        MD_CK(launch_tile_convert(nl->neigh, nl->numneigh, n, nl->capacity, lanes_of(k),
                                  cells->cell_start, tg, nl->tile, nl->status, nullptr, s));
    }
    MD_CK(hipEventRecord(e1, s));
    MD_CK(hipEventSynchronize(e1));
    MD_CK(hipEventElapsedTime(out, e0, e1));
    return MD_OK;
  };
  std::vector<float> ms(trials.size(), 0.f);
  for (size_t t = 0; t < trials.size(); ++t) {
    const md_status st = time_k(trials[t], &ms[t]);
    if (st != MD_OK) return st;
  }
  // the two fastest are timed once more and each keeps its better time, so
  // that a close call does not turn on one noisy measurement (the early
  // candidates can run before the clocks have settled)
  size_t a = 0, b = trials.size() > 1 ? 1 : 0;
  if (ms[b] < ms[a]) std::swap(a, b);
  for (size_t t = 2; t < trials.size(); ++t) {
    if (ms[t] < ms[a]) {
      b = a;
      a = t;
    } else if (ms[t] < ms[b]) {
      b = t;
    }
  }
  int last = trials.back();
  if (b != a) {
    for (size_t t : {b, a}) {
      float again = 0.f;
      const md_status st = time_k(trials[t], &again);
      if (st != MD_OK) return st;
      ms[t] = std::min(ms[t], again);
    }
    last = trials[a];
  }
  for (size_t t = 0; t < trials.size(); ++t) {
    if (ms[t] < best) {
      best = ms[t];
      win = trials[t];
    }
  }
  int words[MD_STATUS_WORDS];
  MD_CK(hipMemcpyAsync(words, nl->status, sizeof(words), hipMemcpyDeviceToHost, s));
  MD_CK(hipStreamSynchronize(s));
  maxcount = words[MD_ST_MAXNEIGH];
  MD_CK(hipEventDestroy(e0));
  MD_CK(hipEventDestroy(e1));
  if (win != last) {
    md_status st = build_list(x, n, sorted, box, nc, cells, rl, nl, win, s);
    if (st != MD_OK) return st;
  }
  MD_CK(hipMemcpyAsync(nl->status + MD_ST_BUILDS, before + MD_ST_BUILDS, sizeof(int),
                       hipMemcpyHostToDevice, s));
  MD_CK(hipStreamSynchronize(s));
  {
    std::lock_guard<std::mutex> lk(g_auto_mu);
    g_auto_cache[auto_key(p, prec, maxcount, n, trials.back() != kWave)] = (md_kernel)win;
  }
  *choice = (md_kernel)win;
  return MD_OK;
}

// Cached AUTO winner for this device, potential, precision and size buckets.
bool cached_choice(const md_potential* p, md_precision prec, int maxcount, int n, bool tiled,
                   int* lanes) {
  std::lock_guard<std::mutex> lk(g_auto_mu);
  auto it = g_auto_cache.find(auto_key(p, prec, maxcount, n, tiled));
  if (it == g_auto_cache.end()) return false;
  *lanes = (int)it->second;
  return true;
}

// The lanes-per-atom count a kernel request resolves to for a list layout,
// or 0 when the request does not match the layout.
int resolve_lanes(md_kernel k, int layout) {
  if (!layout_ok(layout)) return 0;
  const int lanes = lanes_of(layout);
  if (k == MD_KERNEL_AUTO) return lanes;
  return ((int)k == layout || (int)k == lanes) ? lanes : 0;
}

md_status status_from_words(const int* w) {
  if (w[MD_ST_ERRORS] & 4) return MD_ERR_UNSTABLE;
  if (w[MD_ST_ERRORS] & 8) return MD_ERR_BOX_TOO_SMALL;
  if (w[MD_ST_ERRORS] & 2) return MD_ERR_NONFINITE;
  if (w[MD_ST_ERRORS] & 1) return MD_ERR_NLIST_OVERFLOW;
  return MD_OK;
}

}  // namespace

namespace md {

WsLayout ws_layout(int64_t n, int64_t ncell) {
  WsLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += align256(bytes);
    return r;
  };
  const size_t nn = (size_t)n;
  L.count = take(sizeof(int) * (size_t)(ncell > 0 ? ncell : 1));
  L.slot = take(sizeof(int) * nn);
  L.tmp_perm = take(sizeof(int) * nn);
  L.tmp_x = take(sizeof(double) * 3 * nn);
  L.tmp_v = take(sizeof(double) * 3 * nn);
  L.tmp_f = take(sizeof(double) * 3 * nn);
  L.tmp_id = take(sizeof(int) * nn);
  L.tmp_type = take(sizeof(int) * nn);
  L.eatom = take(sizeof(double) * nn);
  L.vatom = take(sizeof(double) * 6 * nn);
  L.keatom = take(sizeof(double) * nn);
  L.vtrace = take(sizeof(double) * nn);
  L.sc_e = take(sizeof(double) * nn);
  L.partials = take(sizeof(double) * kReduceBlocks * kReduceCols);
  L.scalars = take(sizeof(double) * 16);
  L.sortlb = take(sizeof(unsigned long long) * sort_words(ncell > 0 ? ncell : 1));
  L.new_start = take(sizeof(int) * (size_t)((ncell > 0 ? ncell : 1) + 1));
  L.xq = take(sizeof(double) * 4 * nn);
  L.xq2 = take(sizeof(double) * 4 * nn);
  L.total = o;
  return L;
}

}  // namespace md

extern "C" {

size_t md_workspace_bytes(int64_t n, const md_box* box, double rl) {
  if (!n_ok(n) || check_box(box, rl) != MD_OK) return 0;
  int nc[3];
  int64_t ncell;
  if (!cell_dims(box, rl, nc, &ncell)) return 0;
  return ws_layout(n, ncell).total;
}

size_t md_nlist_ints(int64_t n, int capacity) {
  if (!n_ok(n) || capacity < 1) return 0;
  size_t most = 0;
  for (int k = 1; k <= kWave; k *= 2) {
    const size_t groups = (size_t)((n + kWave / k - 1) / (kWave / k));
    const size_t ints = groups * nl_rows(capacity, k) * kWave;
    most = ints > most ? ints : most;
  }
  return most;
}

size_t md_nlist_tile_entries(int64_t n, int capacity, const md_box* box, double rl) {
  if (!n_ok(n) || capacity < 1 || check_box(box, rl) != MD_OK) return 0;
  int nc[3];
  int64_t ncell;
  TileGeom tg{};
  if (!cell_dims(box, rl, nc, &ncell) || !tile_geom(n, nc, &tg)) return 0;
  return tile_list_entries(n, capacity, tg);
}

int md_thermo_rows(int nsteps, int thermo_every, int setup) {
  if (nsteps < 0 || thermo_every < 1) return 0;
  return nsteps / thermo_every + (setup ? 1 : 0);
}

const char* md_status_string(md_status s) {
  switch (s) {
    case MD_OK: return "ok";
    case MD_ERR_INVALID_ARG: return "invalid argument";
    case MD_ERR_BOX_TOO_SMALL: return "box edge not larger than twice the list radius";
    case MD_ERR_NLIST_OVERFLOW: return "neighbour list capacity exceeded";
    case MD_ERR_NONFINITE: return "non-finite position or force";
    case MD_ERR_UNSUPPORTED: return "unsupported request";
    case MD_ERR_HIP: return "HIP runtime error";
    case MD_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case MD_ERR_UNSTABLE: return "an atom moved more than a cell edge between list builds";
    case MD_ERR_SCRATCH: return "the call needs more scratch than the fixed no-allocation array holds";
  }
  return "unknown status";
}

md_status md_bin_cells(double* x, int64_t n, const md_box* box, double rl, md_cells* cells,
                       void* ws, size_t ws_bytes, void* stream) {
  if (!x || !cells || !cells->cell_start || !cells->atom_cell || !cells->perm || !n_ok(n))
    return MD_ERR_INVALID_ARG;
  md_status st = check_box(box, rl);
  if (st != MD_OK) return st;
  int nc[3];
  int64_t ncell;
  if (!cell_dims(box, rl, nc, &ncell) || ncell > cells->ncell_cap) return MD_ERR_INVALID_ARG;
  const WsLayout L = ws_layout(n, ncell);
  if ((st = check_ws(ws, ws_bytes, L)) != MD_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ni = (int)n;
  int* count = at<int>(ws, L.count);
  MD_CK(launch_fill_int(count, ncell, 0, s));
  MD_CK(launch_bin_count(x, ni, make_box(box), nc, cells->atom_cell, count, at<int>(ws, L.slot),
                         s));
  MD_CK(launch_scan_cells(count, (int)ncell, cells->cell_start, s));
  MD_CK(launch_scatter(cells->atom_cell, at<int>(ws, L.slot), cells->cell_start, ni,
                       at<int>(ws, L.tmp_perm), nullptr, s));
  MD_CK(launch_cell_sort(at<int>(ws, L.tmp_perm), cells->cell_start, (int)ncell, cells->perm,
                         nullptr, nullptr, nullptr, nullptr, nullptr, ni, nullptr, nullptr,
                         nullptr, nullptr, nullptr, nullptr, s));
  for (int d = 0; d < 3; ++d) cells->nc[d] = nc[d];
  return MD_OK;
}

md_status md_sort_atoms(md_state* st, const md_cells* cells, double* x_ref, void* ws,
                        size_t ws_bytes, void* stream) {
  if (!st || !cells || !cells->perm || !st->x || !st->v || !st->id || !n_ok(st->n))
    return MD_ERR_INVALID_ARG;
  const WsLayout L = ws_layout(st->n, 1);
  md_status s0 = check_ws(ws, ws_bytes, L);
  if (s0 != MD_OK) return s0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = (int)st->n;
  double* tx = at<double>(ws, L.tmp_x);
  double* tv = at<double>(ws, L.tmp_v);
  double* tf = at<double>(ws, L.tmp_f);
  int* tid = at<int>(ws, L.tmp_id);
  MD_CK(launch_gather3(cells->perm, n, st->x, tx, s));
  MD_CK(launch_gather3(cells->perm, n, st->v, tv, s));
  MD_CK(launch_gather_int(cells->perm, n, st->id, tid, s));
  if (st->f) MD_CK(launch_gather3(cells->perm, n, st->f, tf, s));
  MD_CK(launch_copy_back(st->x, st->v, st->id, st->f, nullptr, tx, tv, tid, tf, n, s));
  if (x_ref) {
    MD_CK(launch_gather3(cells->perm, n, x_ref, tx, s));
    MD_CK(launch_copy_back(x_ref, nullptr, nullptr, nullptr, nullptr, tx, nullptr, nullptr,
                           nullptr, n, s));
  }
  return MD_OK;
}

md_status md_build_neighbors(const double* x, int64_t n, const md_box* box,
                             const md_cells* cells, double rc, double skin, md_nlist* nl,
                             void* stream) {
  if (!x || !cells || !nl || !nl->neigh || !nl->numneigh || !nl->status || !n_ok(n) ||
      nl->capacity < 1 || !(skin >= 0.0) || !std::isfinite(skin) || !layout_ok(nl->layout) ||
      !cells->cell_start || !cells->atom_cell || !cells->perm)
    return MD_ERR_INVALID_ARG;
  const double rl = rc + skin;
  md_status st = check_box(box, rl);
  if (st != MD_OK) return st;
  int nc[3];
  int64_t ncell;
  if (!cell_dims(box, rl, nc, &ncell)) return MD_ERR_INVALID_ARG;
  for (int d = 0; d < 3; ++d)
    if (cells->nc[d] != nc[d]) return MD_ERR_INVALID_ARG;  // cells were binned at another rl
  return build_list(x, (int)n, 0, box, nc, cells, rl, nl, nl->layout,
                    static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

// Scratch of one md_compute_forces call: packed positions [n][4], the
// Sutton-Chen density column [n], per-atom energy [n] and virial [6][n], and
// the partial sums of the energy / virial reduction.
struct ForceScratch {
  double* xq;
  double* sc_e;
  double* eatom;
  double* vatom;
  double* partials;
};

md_status check_forces_args(const md_potential* p, const double* x, int64_t n,
                            const md_box* box, const md_nlist* nl, md_precision prec,
                            md_kernel k, int flags, double* f, double* ev, int* kernel) {
  md_status st = check_pot(p);
  if (st != MD_OK) return st;
  if (!x || !nl || !nl->neigh || !nl->numneigh || !f || !n_ok(n) || nl->capacity < 1 ||
      (prec != MD_FP64 && prec != MD_MIXED) || (flags & ~(MD_EFLAG | MD_VFLAG)) ||
      (flags && !ev))
    return MD_ERR_INVALID_ARG;
  *kernel = resolve_lanes(k, nl->layout);
  if (!*kernel) return MD_ERR_INVALID_ARG;
  if (nl->half && p->kind != MD_POT_LJ) return MD_ERR_UNSUPPORTED;
  return check_box(box, nl->rl > p->rc ? nl->rl : p->rc);
}

// md_compute_forces after validation, with its scratch given.
md_status compute_forces_impl(const md_potential* p, const double* x, int n, const md_box* box,
                              const md_nlist* nl, md_precision prec, int kernel, int flags,
                              double* f, double* ev, const ForceScratch& sc, hipStream_t s) {
  MD_CK(launch_pack_positions(x, n, sc.xq, species(p), s));
  ForceArgs fa{};
  fa.xq = sc.xq;
  fa.n = n;
  fa.box = make_box(box);
  fa.margin = interior_margin(p, nl->rl);
  fa.neigh = nl->neigh;
  fa.numneigh = nl->numneigh;
  fa.cap = nl->capacity;
  fa.f = f;
  if (flags) {
    fa.ev.eatom = sc.eatom;
    fa.ev.vatom = sc.vatom;
  }
  timing_events(&fa.t0, &fa.t1);
  if (nl->half) {
    // each pair once; both atoms' shares are added atomically into f
    MD_CK(launch_fill_double(f, 3 * (int64_t)n, 0.0, s));
    MD_CK(launch_lj_half(fa, make_lj(p), prec, kernel, s));
  } else {
    const md_status st = force_dispatch(p, fa, prec, kernel, sc.sc_e, s);
    if (st != MD_OK) return st;
  }
  if (flags) {
    SumArgs sa{};
    sa.cols = 7;
    sa.col[0] = fa.ev.eatom;
    for (int q = 0; q < 6; ++q) sa.col[1 + q] = fa.ev.vatom + (size_t)q * n;
    sa.n = n;
    sa.partials = sc.partials;
    sa.out = ev;
    MD_CK(launch_sum(sa, s));
  }
  return MD_OK;
}

// ------------------------------------------- fixed scratch (no allocation) --

// The scratch of md_compute_forces_noalloc: one array per device, held from
// the library's load until the process ends.  Host code never uses this name
// as an address (on the host it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[MD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there), or null if the lookup fails.
void* scratch_on_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

// Carve-up of the fixed scratch for n atoms (offsets from its base); total
// is the bytes needed.
struct NoAllocLayout {
  size_t xq, sc_e, eatom, vatom, partials, total;
};
NoAllocLayout noalloc_layout(int64_t n, bool sc, bool ev) {
  NoAllocLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += align256(bytes);
    return r;
  };
  const size_t nn = (size_t)n;
  L.xq = take(sizeof(double) * 4 * nn);
  L.sc_e = sc ? take(sizeof(double) * nn) : 0;
  if (ev) {
    L.eatom = take(sizeof(double) * nn);
    L.vatom = take(sizeof(double) * 6 * nn);
    L.partials = take(sizeof(double) * kReduceBlocks * kReduceCols);
  }
  L.total = o;
  return L;
}

}  // namespace

extern "C" {

md_status md_compute_forces(const md_potential* p, const double* x, int64_t n,
                            const md_box* box, const md_nlist* nl, md_precision prec,
                            md_kernel k, int flags, double* f, double* ev, void* ws,
                            size_t ws_bytes, void* stream) {
  int kernel = 0;
  md_status st = check_forces_args(p, x, n, box, nl, prec, k, flags, f, ev, &kernel);
  if (st != MD_OK) return st;
  const WsLayout L = ws_layout(n, 1);
  if ((st = check_ws(ws, ws_bytes, L)) != MD_OK) return st;
  ForceScratch sc;
  sc.xq = at<double>(ws, L.xq);
  sc.sc_e = at<double>(ws, L.sc_e);
  sc.eatom = at<double>(ws, L.eatom);
  sc.vatom = at<double>(ws, L.vatom);
  sc.partials = at<double>(ws, L.partials);
  return compute_forces_impl(p, x, (int)n, box, nl, prec, kernel, flags, f, ev, sc,
                             static_cast<hipStream_t>(stream));
}

size_t md_compute_forces_noalloc_bytes(int64_t n, int kind, int flags) {
  if (!n_ok(n)) return 0;
  return noalloc_layout(n, kind == MD_POT_SC, flags != 0).total;
}

md_status md_compute_forces_noalloc(const md_potential* p, const double* x, int64_t n,
                                    const md_box* box, const md_nlist* nl, md_precision prec,
                                    md_kernel k, int flags, double* f, double* ev,
                                    void* stream) {
  int kernel = 0;
  md_status st = check_forces_args(p, x, n, box, nl, prec, k, flags, f, ev, &kernel);
  if (st != MD_OK) return st;
  const NoAllocLayout L = noalloc_layout(n, p->kind == MD_POT_SC, flags != 0);
  if (L.total > (size_t)MD_NOALLOC_SCRATCH_BYTES) return MD_ERR_SCRATCH;
  void* base = scratch_on_current_device();
  if (!base) return MD_ERR_HIP;
  // nothing in the scratch has to start at zero: every word a kernel reads
  // was written earlier in the same call
  ForceScratch sc;
  sc.xq = at<double>(base, L.xq);
  sc.sc_e = p->kind == MD_POT_SC ? at<double>(base, L.sc_e) : nullptr;
  sc.eatom = flags ? at<double>(base, L.eatom) : nullptr;
  sc.vatom = flags ? at<double>(base, L.vatom) : nullptr;
  sc.partials = flags ? at<double>(base, L.partials) : nullptr;
  return compute_forces_impl(p, x, (int)n, box, nl, prec, kernel, flags, f, ev, sc,
                             static_cast<hipStream_t>(stream));
}

md_status md_force_vjp(const md_potential* p, const double* x, int64_t n, const md_box* box,
                       const md_nlist* nl, md_precision prec, const double* u, double* gx,
                       double* gparam, void* ws, size_t ws_bytes, void* stream) {
  md_status st = check_pot(p);
  if (st != MD_OK) return st;
  if ((p->kind != MD_POT_LJ && p->kind != MD_POT_SC) || (nl && nl->half))
    return MD_ERR_UNSUPPORTED;
  if (!x || !nl || !nl->neigh || !nl->numneigh || !u || !gx || !n_ok(n) || nl->capacity < 1 ||
      (prec != MD_FP64 && prec != MD_MIXED) || !layout_ok(nl->layout))
    return MD_ERR_INVALID_ARG;
  if ((st = check_box(box, nl->rl > p->rc ? nl->rl : p->rc)) != MD_OK) return st;
  const WsLayout L = ws_layout(n, 1);
  if ((st = check_ws(ws, ws_bytes, L)) != MD_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* xq = at<double>(ws, L.xq);
  MD_CK(launch_pack_positions(x, (int)n, xq, species(p), s));
  ForceArgs fa{};
  fa.xq = xq;
  fa.n = (int)n;
  fa.box = make_box(box);
  fa.margin = interior_margin(p, nl->rl);
  fa.neigh = nl->neigh;
  fa.numneigh = nl->numneigh;
  fa.cap = nl->capacity;
  timing_events(&fa.t0, &fa.t1);
  if (p->kind == MD_POT_SC) {
    // e, lam, la, lb in the workspace's per-atom columns
    double* e = at<double>(ws, L.sc_e);
    double* lam = at<double>(ws, L.vatom);
    double* la = at<double>(ws, L.eatom);
    double* lb = at<double>(ws, L.keatom);
    const SCK k = make_sc(p);
    MD_CK(launch_sc_vjp(fa, k, prec, lanes_of(nl->layout), u, e, lam, la, lb, at<double>(ws, L.xq2), gx,
                        s));
    if (gparam) {
      SumArgs sa{};
      sa.cols = 2;
      sa.col[0] = la;
      sa.col[1] = lb;
      sa.n = (int)n;
      sa.partials = at<double>(ws, L.partials);
      sa.out = at<double>(ws, L.scalars);
      sa.params.kind = kParamsSC;
      sa.params.eps = k.eps;
      sa.params.a = p->sc_a;
      sa.params.c = k.c;
      sa.params.nexp = (double)k.n;
      sa.params.mexp = (double)k.m;
      sa.params.gparam = gparam;
      MD_CK(launch_sum(sa, s));
    }
    return MD_OK;
  }
  // the kernel's workgroups leave their sums of u_i . F_i and of the sigma
  // term in rows of two in the per-atom energy column (at most n / 2 doubles)
  double* bp = gparam ? at<double>(ws, L.eatom) : nullptr;
  int rows = 0;
  MD_CK(launch_lj_vjp(fa, make_lj(p), prec, lanes_of(nl->layout), u, gx, bp, &rows, s));
  if (gparam) {
    SumArgs sa{};
    sa.cols = 2;
    sa.nparts = rows;
    sa.partials = bp;
    sa.out = at<double>(ws, L.scalars);
    // dL/deps = (sum_i u_i . F_i) / eps; the second sum is dL/dsigma already
    sa.params.kind = kParamsLJ;
    sa.params.eps = p->lj_eps;
    sa.params.gparam = gparam;
    MD_CK(launch_sum_parts(sa, s));
  }
  return MD_OK;
}

md_status md_nlist_status(const md_nlist* nl, int* words, void* stream) {
  if (!nl || !nl->status || !words) return MD_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  MD_CK(hipMemcpyAsync(words, nl->status, sizeof(int) * MD_STATUS_WORDS, hipMemcpyDeviceToHost,
                       s));
  MD_CK(hipStreamSynchronize(s));
  return MD_OK;
}

md_status md_autoselect(const md_potential* p, const double* x, int64_t n, const md_box* box,
                        const md_cells* cells, double skin, md_nlist* nl, md_precision prec,
                        int reps, md_kernel* choice, void* ws, size_t ws_bytes, void* stream) {
  md_status st = check_pot(p);
  if (st != MD_OK) return st;
  if (!x || !cells || !nl || !nl->neigh || !nl->numneigh || !nl->status || !choice ||
      !n_ok(n) || nl->capacity < 1 || reps < 1 || (prec != MD_FP64 && prec != MD_MIXED) ||
      !(skin >= 0.0))
    return MD_ERR_INVALID_ARG;
  if (nl->half) return MD_ERR_UNSUPPORTED;
  const double rl = p->rc + skin;
  if ((st = check_box(box, rl)) != MD_OK) return st;
  int nc[3];
  int64_t ncell;
  if (!cell_dims(box, rl, nc, &ncell)) return MD_ERR_INVALID_ARG;
  for (int d = 0; d < 3; ++d)
    if (cells->nc[d] != nc[d]) return MD_ERR_INVALID_ARG;
  const WsLayout L = ws_layout(n, ncell);
  if ((st = check_ws(ws, ws_bytes, L)) != MD_OK) return st;
  return autoselect_impl(p, x, (int)n, 0, box, cells, rl, nl, prec, reps, choice, ws, L,
                         static_cast<hipStream_t>(stream));
}

// md_step and md_step_nvt: NVE when nhc is null, else the Nose-Hoover chain
// splitting around the same velocity-Verlet step.
// The cell grid of an NPT run: edges of at least rl also after the box has
// shrunk by kNptGridMargin.
constexpr double kNptGridMargin = 0.05;

static md_status step_impl(md_state* stt, const md_potential* p, md_box* box,
                           md_cells* cells, md_nlist* nl, md_precision prec, md_kernel k,
                           double skin, double dt, const md_nhc* nhc, const md_npt* npt,
                           int nsteps, int thermo_every, int setup, double* thermo, void* ws,
                           size_t ws_bytes, void* stream) {
  md_status st = check_pot(p);
  if (st != MD_OK) return st;
  if (!stt || !stt->x || !stt->v || !stt->f || !stt->id || stt->n < 2 || !n_ok(stt->n) ||
      !cells || !cells->cell_start || !cells->atom_cell || !cells->perm || !nl || !nl->neigh ||
      !nl->numneigh || !nl->x_ref || !nl->status || nl->capacity < 1 || nsteps < 0 ||
      thermo_every < 1 || !(skin > 0.0) || !std::isfinite(skin) || !finite_pos(dt) ||
      !finite_pos(stt->mass) || !finite_pos(stt->ftm2v) || !finite_pos(stt->mvv2e) ||
      !finite_pos(stt->boltz) || (prec != MD_FP64 && prec != MD_MIXED) ||
      (k != MD_KERNEL_AUTO && !layout_ok((int)k)))
    return MD_ERR_INVALID_ARG;
  if (nl->half) return MD_ERR_UNSUPPORTED;
  const double rl = p->rc + skin;
  if ((st = check_box(box, rl)) != MD_OK) return st;
  int nc[3];
  int64_t ncell;
  if (npt) {
    // NPT: the grid is chosen at setup with room for the box to shrink, and
    // kept while every edge stays at least nc rl
    if (!npt->state || !(npt->p_damp > 0.0) || !std::isfinite(npt->p_target) ||
        !(npt->t_target > 0.0) || !(npt->t_damp > 0.0) || npt->chain < 1 ||
        npt->chain > MD_NHC_MAX)
      return MD_ERR_INVALID_ARG;
    if (setup) {
      md_box shrunk = *box;
      for (int d = 0; d < 3; ++d) shrunk.L[d] = box->L[d] * (1.0 - kNptGridMargin);
      if (!cell_dims(&shrunk, rl, nc, &ncell)) return MD_ERR_BOX_TOO_SMALL;
    } else {
      ncell = 1;
      for (int d = 0; d < 3; ++d) {
        nc[d] = cells->nc[d];
        ncell *= nc[d];
        if (nc[d] < 1 || box->L[d] < nc[d] * rl) return MD_ERR_BOX_TOO_SMALL;
      }
    }
    if (ncell > cells->ncell_cap) return MD_ERR_INVALID_ARG;
  } else if (!cell_dims(box, rl, nc, &ncell) || ncell > cells->ncell_cap) {
    return MD_ERR_INVALID_ARG;
  }
  // tiled kernels: LJ, a tile buffer, and a grid they apply to
  TileGeom tg{};
  const bool tile_ok = !npt && p->kind == MD_POT_LJ && tile_fits(nl, stt->n, nc, &tg);
  if (k != MD_KERNEL_AUTO && is_tile((int)k) && !tile_ok) return MD_ERR_UNSUPPORTED;
  if (!setup) {
    for (int d = 0; d < 3; ++d)
      if (cells->nc[d] != nc[d]) return MD_ERR_INVALID_ARG;
    // a run continues in the layout of its setup (tiled or not)
    if (!layout_ok(nl->layout) || (k != MD_KERNEL_AUTO && (int)k != nl->layout))
      return MD_ERR_INVALID_ARG;
    if (is_tile(nl->layout) && !tile_ok) return MD_ERR_UNSUPPORTED;
  }
  const WsLayout L = ws_layout(stt->n, ncell);
  if ((st = check_ws(ws, ws_bytes, L)) != MD_OK) return st;

  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = (int)stt->n;
  const BoxK bk = make_box(box);
  // NPT keeps the box in device memory (the barostat state); every kernel
  // after the setup binning reads it there
  double* const nstate = npt ? npt->state : nullptr;
  const double* const boxd = npt ? nstate + kNptL : nullptr;
  if (npt && setup) {
    double init[6] = {box->L[0], box->L[1], box->L[2], box->L[0], box->L[1], box->L[2]};
    MD_CK(hipMemcpyAsync(nstate + kNptL, init, sizeof(init), hipMemcpyHostToDevice, s));
    MD_CK(hipStreamSynchronize(s));   // init is a host stack buffer
  }
  const double dtfm = (0.5 * dt * stt->ftm2v) / stt->mass;
  const double trig = 0.5 * skin;
  const double trig2 = trig * trig;
  int* status = nl->status;
  // Rebuild requests alternate between two words: the drift of step t sets
  // gates[t & 1], the rebuild before step t's forces is gated by it, and the
  // force kernel of step t clears it while its own drift sets the other word,
  // so no kernel clears a word that it also sets.
  int* const gates[2] = {status + MD_ST_REBUILD2, status + MD_ST_REBUILD};
  int* gate = gates[1];
  int* count = at<int>(ws, L.count);
  int* slot = at<int>(ws, L.slot);
  int* tmp_perm = at<int>(ws, L.tmp_perm);
  double* sx = at<double>(ws, L.tmp_x);
  double* sv = at<double>(ws, L.tmp_v);
  int* sid = at<int>(ws, L.tmp_id);
  // species travel with the atoms through every rebuild (Buckingham only)
  int* const type = const_cast<int*>(species(p));
  int* stype = at<int>(ws, L.tmp_type);
  double* eatom = at<double>(ws, L.eatom);
  double* vatom = at<double>(ws, L.vatom);
  double* keatom = at<double>(ws, L.keatom);
  double* sums = at<double>(ws, L.scalars);
  // NPT: every force pass leaves each atom's virial trace, which the barostat sums
  double* const vtrace = npt ? at<double>(ws, L.vtrace) : nullptr;

  // the rebuild sort's look-back words, zeroed for this call's first sort
  unsigned long long* const sortlb = at<unsigned long long>(ws, L.sortlb);
  MD_CK(launch_sort_clear(sortlb, ncell, s));
  int* new_start = at<int>(ws, L.new_start);
  // packed positions: the setup build and the force kernels read xq[0]
  // first; each fused step reads one buffer and drifts into the other
  double* const xqs[2] = {at<double>(ws, L.xq), at<double>(ws, L.xq2)};

  // Rebuild chain.  At setup (no gate; atoms in arbitrary order): wrap + bin +
  // count, scan, scatter, stable in-cell order with the state gathered into
  // staging, list build that copies the state back.  During a run (gated;
  // atoms in the previous build's cell order, their new cells recorded by the
  // drift kernel): one sort kernel (per-cell counts from the previous ranges,
  // new cell starts, the state gathered into staging), list build, which also
  // copies the new starts into cells->cell_start.  Gated kernels return at
  // once unless the rebuild flag is set.
  auto rebuild = [&](const int* g, int layout, double* xq) -> md_status {
    int* starts = g ? new_start : cells->cell_start;
    if (g) {
      MD_CK(launch_sort_cells(cells->cell_start, new_start, cells->atom_cell, nc, bk, boxd,
                              cells->perm, xq, stt->v, stt->id, type, n, sx, sv, sid, stype,
                              status, sortlb, g, s));
    } else {
      MD_CK(launch_fill_int(count, ncell, 0, s));
      MD_CK(launch_bin_count(stt->x, n, bk, nc, cells->atom_cell, count, slot, s));
      MD_CK(launch_scan_cells(count, (int)ncell, starts, s));
      MD_CK(launch_scatter(cells->atom_cell, slot, starts, n, tmp_perm, g, s));
      MD_CK(launch_cell_sort(tmp_perm, starts, (int)ncell, cells->perm, stt->x, stt->v, stt->id,
                             nullptr, type, n, sx, sv, sid, nullptr, stype, g, s));
    }
    BuildArgs a{};
    a.x = sx;
    a.n = n;
    a.sorted = 1;
    a.box = bk;
    for (int d = 0; d < 3; ++d) a.nc[d] = nc[d];
    a.cell_start = starts;
    a.cell_start_out = g ? cells->cell_start : nullptr;
    a.atom_cell = cells->atom_cell;
    a.perm = cells->perm;
    a.rl2 = rl * rl;
    a.cap = nl->capacity;
    a.layout = lanes_of(layout);
    a.neigh = nl->neigh;
    a.numneigh = nl->numneigh;
    a.x_ref = nl->x_ref;
    a.status = status;
    a.xq_out = xq;
    a.x_out = stt->x;
    a.v_out = stt->v;
    a.v_in = sv;
    a.id_out = stt->id;
    a.id_in = sid;
    a.type_out = type;
    a.type_in = type ? stype : nullptr;
    a.gate = g;
    a.boxd = boxd;
    a.lref = npt ? nstate + kNptLref : nullptr;
    MD_CK(launch_build(a, s));
    // the tile list from the new list, on the new cell starts
    if (is_tile(layout))
      MD_CK(launch_tile_convert(nl->neigh, nl->numneigh, n, nl->capacity, lanes_of(layout),
                                cells->cell_start, tg, nl->tile, status, g, s));
    return MD_OK;
  };

  // Forces at the positions in xq; with `in`, the kernel also integrates.
  auto forces = [&](bool ev, int kernel, const double* xq, const IntArgs* in) -> md_status {
    ForceArgs fa{};
    fa.xq = xq;
    if (in) fa.in = *in;
    fa.n = n;
    fa.box = bk;
    // a changing box voids the interior argument: the minimum image always
    fa.margin = npt ? HUGE_VAL : interior_margin(p, rl);
    fa.boxd = boxd;
    fa.neigh = nl->neigh;
    fa.numneigh = nl->numneigh;
    fa.cap = nl->capacity;
    fa.tile = nl->tile;
    fa.cell_start = cells->cell_start;
    fa.tg = tg;
    fa.f = stt->f;
    if (ev) {
      fa.ev.eatom = eatom;
      fa.ev.vatom = vatom;
    }
    fa.ev.vtrace = vtrace;
    fa.clear = gate;
    timing_events(&fa.t0, &fa.t1);
    return force_dispatch(p, fa, prec, kernel, at<double>(ws, L.sc_e), s);
  };

  const double dof = 3.0 * (double)n - 3.0;
  const double volume = box->L[0] * box->L[1] * box->L[2];
  int row = 0;
  const int row_cols = npt ? 10 : (nhc ? 9 : 8);
  auto sums_out = [&](const NhcArgs* h) -> md_status {
    SumArgs sa{};
    sa.cols = 8;
    sa.col[0] = eatom;
    for (int q = 0; q < 6; ++q) sa.col[1 + q] = vatom + (size_t)q * n;
    sa.col[7] = keatom;
    sa.n = n;
    sa.partials = at<double>(ws, L.partials);
    sa.out = sums;
    MD_CK(launch_sum(sa, s, h));
    return MD_OK;
  };
  auto row_out = [&](double stepno) -> md_status {
    ThermoArgs ta{};
    ta.sums = sums;
    ta.extra = nhc ? nhc->state + kNhcEnergy : nullptr;
    ta.row = thermo + (size_t)row_cols * (size_t)row++;
    ta.step = stepno;
    ta.mass = stt->mass;
    ta.mvv2e = stt->mvv2e;
    ta.boltz = stt->boltz;
    ta.dof = dof;
    ta.volume = volume;
    ta.status = status;
    if (npt) {
      ta.extra = nstate + kNptEnergy;
      ta.vol = nstate + kNptVol;
    }
    MD_CK(launch_thermo_row(ta, s));
    return MD_OK;
  };
  auto thermo_out = [&](double stepno) -> md_status {
    md_status r = sums_out(nullptr);
    return r != MD_OK ? r : row_out(stepno);
  };
  // Nose-Hoover chain constants and the kinetic-energy-only sum (into
  // sums[8]) that steps without a thermo row use.
  NhcArgs na{};
  SumArgs ka{};
  double* const nhc_scale = nhc ? nhc->state + kNhcScale : nullptr;
  if (nhc) {
    const double kT = stt->boltz * nhc->t_target;
    na.state = nhc->state;
    na.M = nhc->chain;
    na.kT = kT;
    na.nf = dof;
    na.Q0 = dof * kT * nhc->t_damp * nhc->t_damp;
    na.Qj = kT * nhc->t_damp * nhc->t_damp;
    na.dt = dt;
    na.mke = stt->mass * stt->mvv2e;
    ka.cols = 1;
    ka.col[0] = keatom;
    ka.n = n;
    ka.partials = at<double>(ws, L.partials);
    ka.out = sums + 8;
  }

  int kernel = nl->layout;   // lanes per atom == list layout
  if (setup) {
    kernel = k == MD_KERNEL_AUTO ? MD_KERNEL_TPA : (int)k;
    if ((st = rebuild(nullptr, kernel, xqs[0])) != MD_OK) return st;
    for (int d = 0; d < 3; ++d) cells->nc[d] = nc[d];
    nl->layout = kernel;
    nl->rl = rl;
    if (k == MD_KERNEL_AUTO) {
      int words[MD_STATUS_WORDS];
      MD_CK(hipMemcpyAsync(words, status, sizeof(words), hipMemcpyDeviceToHost, s));
      MD_CK(hipStreamSynchronize(s));
      int lanes = 0;
      if (cached_choice(p, prec, words[MD_ST_MAXNEIGH], n, tile_ok, &lanes)) {
        if (lanes != kernel) {
          st = build_list(stt->x, n, 1, box, nc, cells, rl, nl, lanes, s);
          if (st != MD_OK) return st;
          MD_CK(hipMemcpyAsync(status + MD_ST_BUILDS, words + MD_ST_BUILDS, sizeof(int),
                               hipMemcpyHostToDevice, s));
          MD_CK(hipStreamSynchronize(s));
        }
        kernel = lanes;
      } else {
        md_kernel choice = MD_KERNEL_TPA;
        st = autoselect_impl(p, stt->x, n, 1, box, cells, rl, nl, prec, 5, &choice, ws, L, s,
                             tile_ok);
        if (st != MD_OK) return st;
        kernel = (int)choice;
      }
    }
    const bool ev = thermo != nullptr && !npt;   // NPT evaluates its setup forces below
    if (!npt && (st = forces(ev, kernel, xqs[0], nullptr)) != MD_OK) return st;
    if (ev) {
      MD_CK(launch_ke(stt->v, n, keatom, s));
      // with a thermostat, also the chain energy of the state as given
      if ((st = sums_out(nhc ? &na : nullptr)) != MD_OK) return st;
      if ((st = row_out(0.0)) != MD_OK) return st;
    }
  }
  const int layout = kernel;
  auto is_thermo = [&](int step) { return thermo && step >= 1 && step % thermo_every == 0; };
  // Step 1 opens with a kick and drift from the state (its forces current),
  // into xq[1].  Then for s = 1 .. nsteps: gated rebuild of the positions in
  // xq[s & 1], and one force kernel that also integrates -- closing kick of
  // step s, then (s < nsteps) step s + 1's kick, drift into xq[(s + 1) & 1]
  // and check, or (s = nsteps) the state's x and f.  The thermo row of step s
  // is summed right after its force kernel.
  if (npt) {
    // Per call: forces with energy and virial at the current positions (the
    // virial enters the barostat force), the kinetic sum, and the update
    // that opens step 1.  Per step: the scaled kick + drift + check (factors
    // from the update), gated rebuild in the current box, forces with the
    // closing kick (factors a, b) storing x, f, v and |v|^2 (and, on thermo
    // steps, energy and virial; otherwise the virial trace alone), the sums,
    // whose last kernel runs the update closing this step and opening the
    // next, and the thermo row.
    const double kT = stt->boltz * npt->t_target;
    NptArgs pa{};
    pa.state = nstate;
    pa.M = npt->chain;
    pa.nf = dof;
    pa.kT = kT;
    pa.Q0 = dof * kT * npt->t_damp * npt->t_damp;
    pa.Qj = kT * npt->t_damp * npt->t_damp;
    pa.Qb = kT * npt->p_damp * npt->p_damp;
    pa.W = (dof + 3.0) * kT * npt->p_damp * npt->p_damp;
    pa.alpha = 1.0 + 3.0 / dof;
    pa.dt = dt;
    pa.mke = stt->mass * stt->mvv2e;
    pa.ptarget = npt->p_target;
    pa.skin = skin;
    pa.rl = rl;
    for (int d = 0; d < 3; ++d) pa.nc[d] = nc[d];
    pa.status = status;
    // Sums of a force pass with energy and virial (setup, thermo steps): pe,
    // the virial's diagonal (the row's pressure), the trace, |v|^2 into
    // sums[0..7] (5 and 6 unused).  Other steps: the trace and |v|^2 only,
    // into sums[9], sums[10].  The barostat takes the trace column's sum in
    // both, so a thermo row leaves the trajectory unchanged.
    SumArgs sa{};
    sa.cols = 8;
    sa.col[0] = eatom;
    for (int q = 0; q < 3; ++q) sa.col[1 + q] = vatom + (size_t)q * n;
    sa.col[4] = vtrace;
    sa.col[7] = keatom;
    sa.n = n;
    sa.partials = at<double>(ws, L.partials);
    sa.out = sums;
    SumArgs sb = sa;
    sb.cols = 2;
    sb.col[0] = vtrace;
    sb.col[1] = keatom;
    for (int q = 2; q < kReduceCols; ++q) sb.col[q] = nullptr;
    sb.out = sums + 9;
    MD_CK(launch_pack_positions(stt->x, n, xqs[0], type, s));
    if ((st = forces(true, kernel, xqs[0], nullptr)) != MD_OK) return st;
    MD_CK(launch_ke(stt->v, n, keatom, s));
    {
      NptArgs a = pa;
      a.vsum = sums + 7;
      a.trw = sums + 4;
      a.start = nsteps > 0;
      MD_CK(launch_sum_npt(sa, a, s));
    }
    if (setup && thermo && (st = row_out(0.0)) != MD_OK) return st;
    BinOut bin{};
    bin.box = bk;
    bin.boxd = boxd;
    for (int d = 0; d < 3; ++d) bin.nc[d] = nc[d];
    bin.atom_cell = cells->atom_cell;
    bin.xq = xqs[1];
    bin.flag = gates[1];
    bin.type = type;
    if (nsteps > 0) {
      MD_CK(launch_fill_int(gates[0], 1, 0, s));
      MD_CK(launch_fill_int(gates[1], 1, 0, s));
      MD_CK(launch_kick_drift_npt(stt->x, stt->v, stt->f, nl->x_ref, n, dtfm, status, bin,
                                  nstate, s));
    }
    for (int step = 1; step <= nsteps; ++step) {
      double* cur = xqs[step & 1];
      gate = gates[step & 1];
      if ((st = rebuild(gate, layout, cur)) != MD_OK) return st;
      const bool th = is_thermo(step);
      IntArgs in{};
      in.mode = MD_INT_LAST;
      in.v = stt->v;
      in.xr = nl->x_ref;
      in.x = stt->x;
      in.keatom = keatom;
      in.status = status;
      in.dtfm = dtfm;
      in.dt = dt;
      in.trig2 = trig2;
      in.bin = bin;
      in.kick = nstate + kNptKa;
      if ((st = forces(th, kernel, cur, &in)) != MD_OK) return st;
      NptArgs a = pa;
      a.vsum = th ? sums + 7 : sums + 10;
      a.trw = th ? sums + 4 : sums + 9;
      a.vsum_out = th ? sums + 7 : nullptr;
      a.end = 1;
      a.start = step < nsteps;
      MD_CK(launch_sum_npt(th ? sa : sb, a, s));
      if (th && (st = row_out((double)step)) != MD_OK) return st;
      if (step < nsteps) {
        bin.xq = xqs[(step + 1) & 1];
        bin.flag = gates[(step + 1) & 1];
        MD_CK(launch_kick_drift_npt(stt->x, stt->v, stt->f, nl->x_ref, n, dtfm, status, bin,
                                    nstate, s));
      } else {
        MD_CK(launch_scale_v(stt->v, n, nstate + kNptScale, s));
      }
    }
    MD_CK(hipMemcpyAsync(box->L, nstate + kNptL, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  } else if (nsteps > 0 && nhc) {
    // Per step: thermostat half step and kick + drift + check (one kernel
    // reading the scale the chain update left), gated rebuild, forces with
    // the closing kick only (x, f, v and |v|^2 stored), the kinetic-energy
    // sum, the closing half step fused with the next step's opening half
    // step, and the thermo row.  The first opening half step takes its
    // kinetic energy from a sum over the current velocities.
    BinOut bin{};
    bin.box = bk;
    for (int d = 0; d < 3; ++d) bin.nc[d] = nc[d];
    bin.atom_cell = cells->atom_cell;
    bin.xq = xqs[1];
    bin.flag = gates[1];
    bin.type = type;
    MD_CK(launch_fill_int(gates[0], 1, 0, s));
    MD_CK(launch_fill_int(gates[1], 1, 0, s));
    MD_CK(launch_ke(stt->v, n, keatom, s));
    {
      NhcArgs a = na;
      a.vsum = sums + 8;
      a.start = 1;
      MD_CK(launch_sum(ka, s, &a));
    }
    MD_CK(launch_kick_drift_check(stt->x, stt->v, stt->f, nl->x_ref, n, dtfm, dt, trig2, status,
                                  bin, nhc_scale, s));
    for (int step = 1; step <= nsteps; ++step) {
      double* cur = xqs[step & 1];
      gate = gates[step & 1];
      if ((st = rebuild(gate, layout, cur)) != MD_OK) return st;
      const bool th = is_thermo(step);
      IntArgs in{};
      in.mode = MD_INT_LAST;
      in.v = stt->v;
      in.xr = nl->x_ref;
      in.x = stt->x;
      in.keatom = keatom;
      in.status = status;
      in.dtfm = dtfm;
      in.dt = dt;
      in.trig2 = trig2;
      in.bin = bin;
      if ((st = forces(th, kernel, cur, &in)) != MD_OK) return st;
      // kinetic-energy sum (all thermo columns on thermo steps), then the
      // chain update in the sum's last kernel
      NhcArgs a = na;
      a.vsum = th ? sums + 7 : sums + 8;
      a.vsum_out = th ? sums + 7 : nullptr;
      a.end = 1;
      a.start = step < nsteps;
      if (th) {
        if ((st = sums_out(&a)) != MD_OK) return st;
      } else {
        MD_CK(launch_sum(ka, s, &a));
      }
      if (th && (st = row_out((double)step)) != MD_OK) return st;
      if (step < nsteps) {
        bin.xq = xqs[(step + 1) & 1];
        bin.flag = gates[(step + 1) & 1];
        MD_CK(launch_kick_drift_check(stt->x, stt->v, stt->f, nl->x_ref, n, dtfm, dt, trig2,
                                      status, bin, nhc_scale, s));
      } else {
        MD_CK(launch_scale_v(stt->v, n, nhc_scale, s));
      }
    }
  } else if (nsteps > 0) {
    BinOut bin{};
    bin.box = bk;
    for (int d = 0; d < 3; ++d) bin.nc[d] = nc[d];
    bin.atom_cell = cells->atom_cell;
    bin.xq = xqs[1];
    bin.flag = gates[1];
    bin.type = type;
    MD_CK(launch_fill_int(gates[0], 1, 0, s));
    MD_CK(launch_fill_int(gates[1], 1, 0, s));
    MD_CK(launch_kick_drift_check(stt->x, stt->v, stt->f, nl->x_ref, n, dtfm, dt, trig2, status,
                                  bin, nullptr, s));
    for (int step = 1; step <= nsteps; ++step) {
      double* cur = xqs[step & 1];
      gate = gates[step & 1];
      if ((st = rebuild(gate, layout, cur)) != MD_OK) return st;
      const bool th = is_thermo(step);
      IntArgs in{};
      in.mode = step < nsteps ? MD_INT_STEP : MD_INT_LAST;
      in.v = stt->v;
      in.xr = nl->x_ref;
      in.x = stt->x;
      in.keatom = th ? keatom : nullptr;
      in.status = status;
      in.dtfm = dtfm;
      in.dt = dt;
      in.trig2 = trig2;
      in.bin = bin;
      in.bin.xq = xqs[(step + 1) & 1];
      in.bin.flag = gates[(step + 1) & 1];
      if ((st = forces(th, kernel, cur, &in)) != MD_OK) return st;
      if (th && (st = thermo_out((double)step)) != MD_OK) return st;
    }
  }
  int words[MD_STATUS_WORDS];
  MD_CK(hipMemcpyAsync(words, status, sizeof(words), hipMemcpyDeviceToHost, s));
  MD_CK(hipStreamSynchronize(s));
  return status_from_words(words);
}

md_status md_step(md_state* stt, const md_potential* p, const md_box* box, md_cells* cells,
                  md_nlist* nl, md_precision prec, md_kernel k, double skin, double dt,
                  int nsteps, int thermo_every, int setup, double* thermo, void* ws,
                  size_t ws_bytes, void* stream) {
  // the box is written only by NPT runs
  return step_impl(stt, p, const_cast<md_box*>(box), cells, nl, prec, k, skin, dt, nullptr,
                   nullptr, nsteps, thermo_every, setup, thermo, ws, ws_bytes, stream);
}

md_status md_step_nvt(md_state* stt, const md_potential* p, const md_box* box, md_cells* cells,
                      md_nlist* nl, md_precision prec, md_kernel k, double skin, double dt,
                      const md_nhc* nhc, int nsteps, int thermo_every, int setup,
                      double* thermo, void* ws, size_t ws_bytes, void* stream) {
  if (!nhc || !nhc->state || nhc->chain < 1 || nhc->chain > MD_NHC_MAX ||
      !finite_pos(nhc->t_target) || !finite_pos(nhc->t_damp))
    return MD_ERR_INVALID_ARG;
  return step_impl(stt, p, const_cast<md_box*>(box), cells, nl, prec, k, skin, dt, nhc, nullptr,
                   nsteps, thermo_every, setup, thermo, ws, ws_bytes, stream);
}

md_status md_step_npt(md_state* stt, const md_potential* p, md_box* box, md_cells* cells,
                      md_nlist* nl, md_precision prec, md_kernel k, double skin, double dt,
                      const md_npt* npt, int nsteps, int thermo_every, int setup,
                      double* thermo, void* ws, size_t ws_bytes, void* stream) {
  if (!npt) return MD_ERR_INVALID_ARG;
  return step_impl(stt, p, box, cells, nl, prec, k, skin, dt, nullptr, npt, nsteps, thermo_every,
                   setup, thermo, ws, ws_bytes, stream);
}

md_status md_timing_enable(int every) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (every > 0 && g_timing.pool.empty()) {
    g_timing.pool.resize(2 * kTimingPairs);
    for (auto& e : g_timing.pool)
      if (hipEventCreate(&e) != hipSuccess) {
        g_timing.pool.clear();
        return MD_ERR_HIP;
      }
  }
  g_timing.every = every;
  g_timing.counter = 0;
  g_timing.used = 0;
  g_timing.launches = 0;
  g_timing.total_ms = 0.0;
  return MD_OK;
}

md_status md_timing_read(int64_t* launches, double* total_ms) {
  if (!launches || !total_ms) return MD_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (g_timing.used) MD_CK(hipDeviceSynchronize());
  for (size_t q = 0; q < g_timing.used; ++q) {
    float ms = 0.f;
    MD_CK(hipEventElapsedTime(&ms, g_timing.pool[2 * q], g_timing.pool[2 * q + 1]));
    g_timing.total_ms += ms;
    ++g_timing.launches;
  }
  g_timing.used = 0;
  *launches = g_timing.launches;
  *total_ms = g_timing.total_ms;
  g_timing.launches = 0;
  g_timing.total_ms = 0.0;
  return MD_OK;
}

}  // extern "C"
