// Pair-force kernels over a full Verlet list (the paper's section "Neighbor
// list approach").  The paper's two designs are the ends of one family here:
// K lanes of a 64-wide wavefront share one atom i and split its neighbour
// list; K = 1 is thread-per-atom (the TpA listing), K = 64 is one wavefront per
// atom (the block-per-atom listing, its block reduction becoming a register
// butterfly with no LDS and no barrier).  Intermediate K trade per-lane loop
// length (latency hiding, lane utilisation) against reduction cost; the
// setup-time mini-benchmark picks K.  Potentials: 12-6 Lennard-Jones and
// two-pass Sutton-Chen; plus the LJ force adjoint.
//
// Precision.  FP64: everything in double.  MIXED: d and r^2 = (dx dx + dy dy)
// + dz dz and the cutoff test stay FP64 (so the interacting pair set equals the
// FP64 one bit for bit), the scalar pair function is evaluated in FP32, and
// the force vector, energy and virial are accumulated in FP64.
#include <hip/hip_ext.h>

#include "md_internal.hpp"

namespace md {
namespace {

constexpr int kUnroll = 4;   // neighbour entries whose loads are issued together

struct FK {
  const double* __restrict__ xq;   // packed positions, atom i at xq[4 i]
  int n;
  BoxK box;
  const double* boxd;     // nullable: the box in device memory (replaces box at kernel entry)
  double margin;          // interior test: every coordinate in [margin, L - margin)
  const int* __restrict__ neigh;
  const int* __restrict__ numneigh;
  int cap;
  double* __restrict__ f;
  double* __restrict__ eatom;
  double* __restrict__ vatom;
  double* __restrict__ vtrace;
  int* clear;
  IntArgs in;
};

// Raw buffer view of the packed positions: 32-bit byte offsets (record j at
// 32 j) and hardware range checking (reads past num_records return 0).
constexpr int kBufWord3 = 0x00020000;   // gfx9-family raw buffer, 32-bit data format
typedef double f64x2 __attribute__((ext_vector_type(2)));
__device__ inline __amdgpu_buffer_rsrc_t buffer_of(const double* p, int n_records) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0,
                                           (int)((unsigned)n_records * 32u), kBufWord3);
}
// 16 bytes of the packed records: (x, y) at +0, (z, pad) at +16.
__device__ inline f64x2 load16(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  return __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, 0));
}

// 12 bytes of the packed records: bytes [0, 12) are x and the low word of y,
// bytes [12, 24) the high word of y and z.
using u32x3 = unsigned __attribute__((ext_vector_type(3)));
__device__ inline u32x3 load12(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  return __builtin_bit_cast(u32x3, __builtin_amdgcn_raw_buffer_load_b96(r, (int)byte_off, 0, 0));
}

// Value of the partner lane (lane ^ 1): a quad permute [1, 0, 3, 2].
__device__ inline int swap_pair(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
}
__device__ inline unsigned swap_pair(unsigned v) { return (unsigned)swap_pair((int)v); }
__device__ inline double swap_pair(double v) {
  const int2 w = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(swap_pair(w.x), swap_pair(w.y)));
}
// Home atom position (plain loads).
__device__ inline void home_pos(const FK& a, int i, double& x, double& y, double& z) {
  const double2 q = *reinterpret_cast<const double2*>(a.xq + 4 * (size_t)i);
  x = q.x;
  y = q.y;
  z = a.xq[4 * (size_t)i + 2];
}

// An atom is "interior" when every coordinate lies in [margin, L - margin),
// margin = r_l + skin.  Its list partners then sit within r_l + skin of it in
// the same periodic image (positions are wrapped at each build and move at most
// skin/2 before the next), so d = x_i - x_j already is the minimum image:
// rint(d / L) = 0 and d - L * 0 == d bit for bit.
__device__ inline bool interior(double xi, double yi, double zi, const FK& a) {
  const double m = a.margin;
  return xi >= m && xi < a.box.L[0] - m && yi >= m && yi < a.box.L[1] - m && zi >= m &&
         zi < a.box.L[2] - m;
}

__device__ inline double min_image(double d, double L, double inv) {
  return d - L * rint(d * inv);
}

// 1/s to full FP64 precision: hardware reciprocal estimate + two Newton steps.
__device__ inline double rcp64(double s) {
  double r = __builtin_amdgcn_rcp(s);
  double e = fma(-s, r, 1.0);
  r = fma(r, e, r);
  e = fma(-s, r, 1.0);
  return fma(r, e, r);
}

// Sum over the K aligned lanes that share an atom (butterfly; every lane of
// the group ends with the total).
template <int K>
__device__ inline double group_sum(double v) {
#pragma unroll
  for (int off = K / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Where this lane works: atom i, its sub-lane s, how many list entries
// (s, s+K, ...) it owns, and the wavefront's view of its row group: entry t of
// this lane is the int at byte t * 256 + 4 * lane of the group, read through a
// buffer resource with scalar row offsets (rows past the group read 0).
template <int K>
struct Lane {
  int i;          // atom (may be >= n for padding lanes)
  int s;          // sub-lane 0..K-1
  bool live;      // i < n
  int count;      // entries owned by this lane
  int tmax;       // largest count in the wavefront (uniform)
  __amdgpu_buffer_rsrc_t nb;   // the wavefront's row group of the list
  unsigned voff;               // 4 * lane
  __device__ inline Lane(const FK& a) {
    const int g = xcd_block() * kBlock + threadIdx.x;   // contiguous atoms per XCD
    const int lane = g & (kWave - 1);
    i = (g / kWave) * (kWave / K) + lane / K;
    s = lane % K;
    live = i < a.n;
    const int nn = live ? min(a.numneigh[i], a.cap) : 0;
    count = nn > s ? (nn - s + K - 1) / K : 0;
    int m = count;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, kWave));
    tmax = __builtin_amdgcn_readfirstlane(m);
    const int rows = (int)nl_rows(a.cap, K);
    const int* base = a.neigh + (size_t)__builtin_amdgcn_readfirstlane(g / kWave) * rows * kWave;
    nb = __builtin_amdgcn_make_buffer_rsrc(const_cast<int*>(base), (short)0, rows * kWave * 4,
                                           kBufWord3);
    voff = 4u * (unsigned)lane;
  }
  // index of this lane's entry t (0 past the group's rows)
  __device__ inline int entry(int t) const {
    return (int)__builtin_amdgcn_raw_buffer_load_b32(nb, (int)voff, t * kWave * 4, 0);
  }
};

// Separations of kUnroll entries starting at entry t: the position gathers
// of the batch go out first (one 32-byte record per entry through the buffer
// view), then the next batch's index loads, then the arithmetic, so each
// batch waits for one memory latency instead of two.  ok[] marks the lane's
// own entries; the others use atom 0 and are masked.  WRAP applies
// the minimum image; interior wavefronts skip it (see interior()).
struct Batch {
  int j[kUnroll];
  int t[kUnroll];   // species of j (TYPED batches only)
  double w3[kUnroll];   // fourth word of j's record (FOURTH batches only)
  bool ok[kUnroll];
  double dx[kUnroll], dy[kUnroll], dz[kUnroll], s[kUnroll];
};

struct XView {
  __amdgpu_buffer_rsrc_t r;   // the packed [n][4] positions
};

// PAIRED: lanes 2m and 2m + 1 fetch their two records together.  In each
// 12-byte load both lanes of the pair read one record (one cache-line lookup
// instead of two, and the 24 bytes the record holds), the even lane's record
// first, then the odd lane's; each lane then holds the first half of its own
// record and the second half of its partner's, and a three-word lane swap
// completes every lane's record.  Otherwise each lane reads (x, y) and z of
// its own record with a 16- and an 8-byte load.
template <int K, bool WRAP, bool PAIRED, bool TYPED = false, bool FOURTH = false>
__device__ inline void load_batch(const FK& a, const XView& xv, const Lane<K>& ln, int t,
                                  int* jn, double xi, double yi, double zi, Batch& b) {
  double xj[kUnroll], yj[kUnroll], zj[kUnroll];
  const bool odd = (threadIdx.x & 1) != 0;
  const unsigned half = odd ? 12u : 0u;
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    // entries past the lane's count are never used as indices: atom 0 stands in
    b.ok[u] = t + u < ln.count;
    b.j[u] = b.ok[u] ? jn[u] : 0;
    if (PAIRED) {
      const int pj = swap_pair(b.j[u]);
      const unsigned je = (unsigned)(odd ? pj : b.j[u]);   // the even lane's entry
      const unsigned jo = (unsigned)(odd ? b.j[u] : pj);   // the odd lane's entry
      // first halves (x, low word of y) to the owner, second halves (high
      // word of y, z) to the partner, which hands them back with one swap
      const u32x3 p = load12(xv.r, je * 32u + half);          // even: first half of je
      const u32x3 q = load12(xv.r, jo * 32u + (12u - half));  // even: second half of jo
      const u32x3 own = odd ? q : p;
      const u32x3 give = odd ? p : q;
      const unsigned r0 = swap_pair(give.x), r1 = swap_pair(give.y), r2 = swap_pair(give.z);
      xj[u] = __builtin_bit_cast(double, make_uint2(own.x, own.y));
      yj[u] = __builtin_bit_cast(double, make_uint2(own.z, r0));
      zj[u] = __builtin_bit_cast(double, make_uint2(r1, r2));
    } else if (TYPED || FOURTH) {
      // (x, y) and (z, fourth word) of the record
      const unsigned off = (unsigned)b.j[u] * 32u;
      const f64x2 xy = load16(xv.r, off);
      const f64x2 zt = load16(xv.r, off + 16u);
      xj[u] = xy.x;
      yj[u] = xy.y;
      zj[u] = zt.x;
      if (TYPED) b.t[u] = (int)zt.y & 3;   // species 0..3 (the mask keeps table reads in bounds)
      if (FOURTH) b.w3[u] = zt.y;
    } else {
      const unsigned off = (unsigned)b.j[u] * 32u;
      const f64x2 xy = load16(xv.r, off);
      xj[u] = xy.x;
      yj[u] = xy.y;
      zj[u] = __builtin_bit_cast(double,
                                 __builtin_amdgcn_raw_buffer_load_b64(xv.r, (int)off, 16, 0));
    }
  }
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) jn[u] = ln.entry(t + kUnroll + u);
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    b.dx[u] = xi - xj[u];
    b.dy[u] = yi - yj[u];
    b.dz[u] = zi - zj[u];
    if (WRAP) {
      b.dx[u] = min_image(b.dx[u], a.box.L[0], a.box.inv[0]);
      b.dy[u] = min_image(b.dy[u], a.box.L[1], a.box.inv[1]);
      b.dz[u] = min_image(b.dz[u], a.box.L[2], a.box.inv[2]);
    }
    // (dx dx + dy dy) + dz dz, evaluated as written
    b.s[u] = b.dx[u] * b.dx[u] + b.dy[u] * b.dy[u] + b.dz[u] * b.dz[u];
  }
}

__device__ inline XView xview(const FK& a) { return XView{buffer_of(a.xq, a.n)}; }

// A packed [n][4] record of per-atom cotangent data (u_j and one more word),
// gathered like the position records: two 16-byte loads.
__device__ inline void load_rec(__amdgpu_buffer_rsrc_t r, int j, double& w0, double& w1,
                                double& w2, double& w3) {
  const unsigned off = (unsigned)j * 32u;
  const f64x2 a = load16(r, off);
  const f64x2 b = load16(r, off + 16u);
  w0 = a.x;
  w1 = a.y;
  w2 = b.x;
  w3 = b.y;
}

// Runs body(batch) over the wavefront's list entries (a uniform loop to the
// largest count).  The choice between the plain and the minimum-image
// separation is uniform over the wavefront.
template <int K, bool PAIRED, bool TYPED = false, bool FOURTH = false, typename F>
__device__ inline void for_each_batch(const FK& a, const Lane<K>& ln, double xi, double yi,
                                      double zi, F&& body) {
  const XView xv = xview(a);
  int jn[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) jn[u] = ln.entry(u);
  if (__all(interior(xi, yi, zi, a))) {
    for (int t = 0; t < ln.tmax; t += kUnroll) {
      Batch b;
      load_batch<K, false, PAIRED, TYPED, FOURTH>(a, xv, ln, t, jn, xi, yi, zi, b);
      body(b);
    }
  } else {
    for (int t = 0; t < ln.tmax; t += kUnroll) {
      Batch b;
      load_batch<K, true, PAIRED, TYPED, FOURTH>(a, xv, ln, t, jn, xi, yi, zi, b);
      body(b);
    }
  }
}

struct Acc {
  double fx = 0, fy = 0, fz = 0, e = 0, w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0;
  __device__ inline void add_force(double g, double dx, double dy, double dz) {
    fx = fma(g, dx, fx);
    fy = fma(g, dy, fy);
    fz = fma(g, dz, fz);
  }
  // the diagonal of add_virial alone, with the same arithmetic
  __device__ inline void add_trace(double g, double dx, double dy, double dz) {
    const double gx = g * dx, gy = g * dy;
    w0 = fma(gx, dx, w0);
    w1 = fma(gy, dy, w1);
    w2 = fma(g * dz, dz, w2);
  }
  __device__ inline void add_virial(double g, double dx, double dy, double dz) {
    const double gx = g * dx, gy = g * dy;
    w0 = fma(gx, dx, w0);
    w1 = fma(gy, dy, w1);
    w2 = fma(g * dz, dz, w2);
    w3 = fma(gx, dy, w3);
    w4 = fma(gx, dz, w4);
    w5 = fma(gy, dz, w5);
  }
  template <int K>
  __device__ inline void reduce(bool ev, bool tr = false) {
    fx = group_sum<K>(fx);
    fy = group_sum<K>(fy);
    fz = group_sum<K>(fz);
    if (tr && !ev) {
      w0 = group_sum<K>(w0);
      w1 = group_sum<K>(w1);
      w2 = group_sum<K>(w2);
    }
    if (ev) {
      e = group_sum<K>(e);
      w0 = group_sum<K>(w0);
      w1 = group_sum<K>(w1);
      w2 = group_sum<K>(w2);
      w3 = group_sum<K>(w3);
      w4 = group_sum<K>(w4);
      w5 = group_sum<K>(w5);
    }
  }
  // Pair energy and virial are split half to each atom of the pair.  With
  // tr (a trace-only kernel) or ev, a.vtrace (if set) gets the virial trace.
  __device__ inline void store(const FK& a, int i, bool ev, double e_extra) const {
    const int n = a.n;
    a.f[i] = fx;
    a.f[n + i] = fy;
    a.f[2 * n + i] = fz;
    store_ev(a, i, ev, e_extra);
  }
  __device__ inline void store_ev(const FK& a, int i, bool ev, double e_extra,
                                  bool tr = false) const {
    const int n = a.n;
    if ((ev || tr) && a.vtrace) a.vtrace[i] = (0.5 * w0 + 0.5 * w1) + 0.5 * w2;
    if (ev) {
      if (a.eatom) a.eatom[i] = 0.5 * e + e_extra;
      if (a.vatom) {
        a.vatom[i] = 0.5 * w0;
        a.vatom[n + i] = 0.5 * w1;
        a.vatom[2 * n + i] = 0.5 * w2;
        a.vatom[3 * n + i] = 0.5 * w3;
        a.vatom[4 * n + i] = 0.5 * w4;
        a.vatom[5 * n + i] = 0.5 * w5;
      }
    }
  }
};

// End of a force kernel for atom i (own: this lane holds atom i's sums and
// writes for it; every lane of the wavefront calls this).  Without fused
// integration (FUSED false, the kernels md_compute_forces and the setup run)
// the force is stored; otherwise the velocity-Verlet steps of IntArgs
// (mode MD_INT_STEP or MD_INT_LAST) follow, with exactly the arithmetic of the separate integration
// kernels: vh = v + dtfm f (closing kick), then v' = vh + dtfm f,
// x' = x + dt v' and the half-skin check, or, on the last step, v = vh and
// the state's x and f stored.
template <bool FUSED>
__device__ inline void finish_atom_with(const FK& a, const Acc& acc, int i, bool own, double xi,
                                        double yi, double zi, bool ev, double e_extra,
                                        const double* vi, const double* xri,
                                        bool tr = false) {
  const IntArgs& in = a.in;
  if (!FUSED) {
    if (own) acc.store(a, i, ev, e_extra);
    return;
  }
  const int n = a.n;
  bool finite = true;
  double xn[3] = {0.0, 0.0, 0.0}, dd[3] = {0.0, 0.0, 0.0};
  if (own) {
    acc.store_ev(a, i, ev, e_extra, tr);
    const double fq[3] = {acc.fx, acc.fy, acc.fz};
    const double xo[3] = {xi, yi, zi};
    double vh[3];
    if (in.kick) {
      const double ka = in.kick[0], kb = in.kick[1];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        finite = finite && isfinite(fq[d]);
        vh[d] = vi[d] * ka + (in.dtfm * fq[d]) * kb;
      }
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        finite = finite && isfinite(fq[d]);
        vh[d] = vi[d] + in.dtfm * fq[d];
      }
    }
    if (in.keatom) in.keatom[i] = vh[0] * vh[0] + vh[1] * vh[1] + vh[2] * vh[2];
    if (in.mode == MD_INT_LAST) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        in.v[d * n + i] = vh[d];
        in.x[d * n + i] = xo[d];
        a.f[d * n + i] = fq[d];
      }
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double vn = vh[d] + in.dtfm * fq[d];
        xn[d] = xo[d] + in.dt * vn;
        in.v[d * n + i] = vn;
        dd[d] = xn[d] - xri[d];
        finite = finite && isfinite(xn[d]);
      }
    }
  }
  if (in.mode == MD_INT_STEP) {
    drift_flags(xn, dd, in.trig2, i, finite, own, in.status, in.bin);
  } else {
    const unsigned long long bad = __ballot(own && !finite);
    if ((threadIdx.x & (kWave - 1)) == 0 && bad) atomicOr(&in.status[MD_ST_ERRORS], 2);
  }
}

// The state an atom's integration reads (velocity and list reference
// position), loaded ahead by kernels that want the loads in flight early.
__device__ inline void load_int_state(const FK& a, int i, bool own, double* vi, double* xri) {
  const int n = a.n;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    vi[d] = own ? a.in.v[d * n + i] : 0.0;
    xri[d] = own && a.in.mode == MD_INT_STEP ? a.in.xr[d * n + i] : 0.0;
  }
}

template <bool FUSED>
__device__ inline void finish_atom(const FK& a, const Acc& acc, int i, bool own, double xi,
                                   double yi, double zi, bool ev, double e_extra,
                                   bool tr = false) {
  double vi[3] = {0.0, 0.0, 0.0}, xri[3] = {0.0, 0.0, 0.0};
  if (FUSED) load_int_state(a, i, own, vi, xri);
  finish_atom_with<FUSED>(a, acc, i, own, xi, yi, zi, ev, e_extra, vi, xri, tr);
}

// The kernel's view of its arguments with the box taken from device memory
// when the run keeps it there (NPT).
__device__ inline FK with_box(const FK& a0) {
  FK a = a0;
  if (a0.boxd) a.box = box_load(a0.boxd);
  return a;
}

// ------------------------------------------------------------------ LJ --

// g(s) with F_ij = g d, and phi(s) (unshifted).
template <int PREC>
__device__ inline void lj_pair(double s, const LJK& p, double& g, double& phi) {
  if (PREC == MD_FP64) {
    const double r2i = rcp64(s);
    const double sr2 = p.sig2 * r2i;
    const double sr6 = sr2 * sr2 * sr2;
    g = r2i * sr6 * fma(p.eps48, sr6, -p.eps24);
    phi = sr6 * fma(p.eps4, sr6, -p.eps4);
  } else {
    const float r2i = __builtin_amdgcn_rcpf((float)s);
    const float sr2 = p.sig2f * r2i;
    const float sr6 = sr2 * sr2 * sr2;
    g = (double)(r2i * sr6 * fmaf(p.eps48f, sr6, -p.eps24f));
    phi = (double)(sr6 * fmaf(p.eps4f, sr6, -p.eps4f));
  }
}

// FP32-mixed instances without energy / virial and with K >= 4 lanes per
// atom are held to six waves per SIMD (at most 80 VGPRs, reached without
// spills): on the 256k melt the fused kernel runs 2 % faster at K = 4, 5 % at
// K = 8, 1 % at K = 16, but 6 % slower at K = 1 and 3.5 % at K = 2, which
// keep the compiler's choice.  The trace-only ones are capped for K = 4 and 8
// (beyond, they would spill).  FP64 and energy / virial instances keep the
// compiler's choice too: six waves made the FP64 kernel 9 % slower and the
// energy / virial one spill.
constexpr int lj_waves_per_eu(int prec, bool ev, bool tr, int k) {
  return prec == MD_MIXED && !ev && k >= 4 && (!tr || k <= 8) ? 6 : 1;
}

// TR (with EV false): the virial's diagonal only, for its trace (a.vtrace),
// as the barostat's steps without a thermo row need it.
template <int PREC, bool EV, int K, bool FUSED, bool TR = false>
__global__ __launch_bounds__(kBlock, lj_waves_per_eu(PREC, EV, TR, K)) void k_lj(FK a0, LJK p) {
  const FK a = with_box(a0);
  if (a.clear && blockIdx.x == 0 && threadIdx.x == 0) *a.clear = 0;
  const Lane<K> ln(a);
  const int n = a.n;
  const int io = ln.live ? ln.i : n - 1;
  double xi, yi, zi;
  home_pos(a, io, xi, yi, zi);
  Acc acc;
  for_each_batch<K, PREC == MD_MIXED>(a, ln, xi, yi, zi, [&](const Batch& b) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      // every lane evaluates the pair function; pairs outside the cutoff or
      // past the lane's list contribute an exact zero (a select, no branch)
      const bool use = b.ok[u] && b.s[u] < p.rc2;
      double g, phi;
      lj_pair<PREC>(use ? b.s[u] : 1.0, p, g, phi);
      g = use ? g : 0.0;
      acc.add_force(g, b.dx[u], b.dy[u], b.dz[u]);
      if (EV) {
        acc.e += use ? phi - p.ecut : 0.0;
        acc.add_virial(g, b.dx[u], b.dy[u], b.dz[u]);
      } else if (TR) {
        acc.add_trace(g, b.dx[u], b.dy[u], b.dz[u]);
      }
    }
  });
  if (K > 1) acc.reduce<K>(EV, TR);
  finish_atom<FUSED>(a, acc, ln.i, ln.live && ln.s == 0, xi, yi, zi, EV, 0.0, TR);
}

// ---------------------------------------------------- LJ, LDS-tiled --

// Window positions a tiled workgroup holds in LDS (x, y and z arrays of
// kTileCap atoms each; the fixed stride lets one address serve all three).
constexpr int kTileCap = kTileLdsBytes / (3 * (int)sizeof(double));

struct TileArgs {
  const unsigned short* __restrict__ tile;
  const int* __restrict__ cs;
  TileGeom g;
};

// Tiled LJ (lists in layout MD_LAYOUT_TILE | K): one workgroup per run.  The
// run's window -- every atom any of its atoms can list -- is staged into LDS
// with coalesced loads of the packed records, one segment of consecutive
// atoms after another; each wavefront then takes groups of G = 64 / K of the
// run's atoms, K lanes each as in k_lj, and gathers its partners' positions
// from LDS through the 16-bit window indices of the tile list.  Everything a
// wavefront's first group reads from memory (list lengths, the words of up to
// 16 entries per lane, and with fused integration the velocity and reference
// position) is requested together with the staging loads, so one memory
// latency covers them all; longer lists load further words 16 entries at a
// time.  The arithmetic per pair (FP64 separation, minimum image off the
// interior, the cutoff test, the pair function, accumulation, the fused
// integration) is k_lj's.  A window with more atoms than the LDS holds (a
// rare density fluctuation) reads the same records from memory instead.
constexpr int kTileWords = 8;    // 32-bit tile words (two entries each) a lane holds at once

template <int PREC, bool EV, int K, bool FUSED>
__global__ __launch_bounds__(kTileBlock, 2) void k_lj_tile(FK a0, LJK p, TileArgs ta) {
  const FK a = with_box(a0);
  __shared__ double wpos[3 * kTileCap];
  __shared__ int s_lo[kTileSegs], s_base[kTileSegs + 1];
  if (a.clear && blockIdx.x == 0 && threadIdx.x == 0) *a.clear = 0;
  const TileGeom& g = ta.g;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int r = xcd_block();
  const TileRun t = tile_run(g, r, ta.cs);
  if (wave == 0) {
    int lo = 0, len = 0;
    if (lane < kTileSegs) tile_segment(g, t, lane, ta.cs, &lo, &len);
    int inc = len;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int y = __shfl_up(inc, off, kWave);
      if (lane >= off) inc += y;
    }
    if (lane < kTileSegs) {
      s_lo[lane] = lo;
      s_base[lane] = inc - len;
    }
    if (lane == kTileSegs - 1) s_base[kTileSegs] = inc;
  }
  constexpr int G = kWave / K;
  const int nh = t.he - t.hb;
  const int ngroups = (nh + G - 1) / G;
  const int T = (int)tile_words(a.cap, K);
  const unsigned* __restrict__ tw = reinterpret_cast<const unsigned*>(ta.tile);
  // per-group lane data: atom, list length and the first words of its entries
  int q = 0, i = 0, count = 0;
  bool live = false;
  unsigned wd[kTileWords];
  double vi[3] = {0.0, 0.0, 0.0}, xri[3] = {0.0, 0.0, 0.0};
  const int sl = lane % K;
  auto words = [&](int gi, int c) {
    const size_t base = ((size_t)(t.hb / G + r + gi) * T + kTileWords * c) * kWave + lane;
#pragma unroll
    for (int u = 0; u < kTileWords; ++u)
      wd[u] = kTileWords * c + u < T ? tw[base + (size_t)u * kWave] : 0u;
  };
  auto open_group = [&](int gi) {
    q = gi * G + lane / K;
    live = q < nh;
    i = t.hb + (live ? q : nh - 1);
    words(gi, 0);
    const int nn = live ? min(a.numneigh[i], a.cap) : 0;
    count = nn > sl ? (nn - sl + K - 1) / K : 0;
    if (FUSED) load_int_state(a, i, live && sl == 0, vi, xri);
  };
  if (wave < ngroups) open_group(wave);
  __syncthreads();
  const int W = s_base[kTileSegs];
  const bool fits = W <= kTileCap;
  // window index -> atom: the last segment whose window base is <= w
  auto atom_of = [&](int w) {
    int lo = 0, hi = kTileSegs;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_base[mid] <= w) lo = mid; else hi = mid;
    }
    return s_lo[lo] + (w - s_base[lo]);
  };
  const __amdgpu_buffer_rsrc_t xr = buffer_of(a.xq, a.n);
  if (fits) {
    constexpr int kStage = 4;   // window atoms per thread whose loads go out together
    for (int q0 = 0; q0 < W; q0 += kStage * kTileBlock) {
      f64x2 xy[kStage];
      double zz[kStage];
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int qq = q0 + u * kTileBlock + (int)threadIdx.x;
        const unsigned off = qq < W ? (unsigned)atom_of(qq) * 32u : 0u;
        xy[u] = load16(xr, off);
        zz[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(xr, (int)off, 16, 0));
      }
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int qq = q0 + u * kTileBlock + (int)threadIdx.x;
        if (qq < W) {
          wpos[qq] = xy[u].x;
          wpos[kTileCap + qq] = xy[u].y;
          wpos[2 * kTileCap + qq] = zz[u];
        }
      }
    }
  }
  __syncthreads();
  const int hs = tile_home_segment(g, t);
  const int wh0 = s_base[hs] + (t.hb - s_lo[hs]);   // window index of the run's first atom
  // the pair loop, compiled once for positions in LDS and once for the
  // fallback that reads them from memory (kept apart so that LDS reads never
  // wait on the fallback's loads)
  auto groups = [&](auto fits_c) {
    constexpr bool FITS = decltype(fits_c)::value;
    auto pos = [&](int w, double& x, double& y, double& z) {
      if constexpr (FITS) {
        x = wpos[w];
        y = wpos[kTileCap + w];
        z = wpos[2 * kTileCap + w];
      } else {
        const unsigned off = (unsigned)atom_of(w) * 32u;
        const f64x2 v2 = load16(xr, off);
        x = v2.x;
        y = v2.y;
        z = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(xr, (int)off, 16, 0));
      }
    };
  for (int gi = wave; gi < ngroups; gi += kTileBlock / kWave) {
    if (gi != wave) open_group(gi);
    int tm = count;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) tm = max(tm, __shfl_xor(tm, off, kWave));
    const int tmax = __builtin_amdgcn_readfirstlane(tm);
    double xi, yi, zi;
    pos(wh0 + (live ? q : nh - 1), xi, yi, zi);
    const bool wrap = !__all(interior(xi, yi, zi, a));
    Acc acc;
    for (int c = 0; 2 * kTileWords * c < tmax; ++c) {
      if (c > 0) words(gi, c);
#pragma unroll
      for (int b = 0; b < 2 * kTileWords; b += kUnroll) {
        const int tt = 2 * kTileWords * c + b;
        if (tt >= tmax) break;
        double dx[kUnroll], dy[kUnroll], dz[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int e = b + u;
          ok[u] = tt + u < count;
          const int w = ok[u] ? (int)((wd[e >> 1] >> (16 * (e & 1))) & 0xFFFFu) : 0;
          double xj, yj, zj;
          pos(w, xj, yj, zj);
          dx[u] = xi - xj;
          dy[u] = yi - yj;
          dz[u] = zi - zj;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          if (wrap) {
            dx[u] = min_image(dx[u], a.box.L[0], a.box.inv[0]);
            dy[u] = min_image(dy[u], a.box.L[1], a.box.inv[1]);
            dz[u] = min_image(dz[u], a.box.L[2], a.box.inv[2]);
          }
          const double sv = dx[u] * dx[u] + dy[u] * dy[u] + dz[u] * dz[u];
          const bool use = ok[u] && sv < p.rc2;
          double gg, phi;
          lj_pair<PREC>(use ? sv : 1.0, p, gg, phi);
          gg = use ? gg : 0.0;
          acc.add_force(gg, dx[u], dy[u], dz[u]);
          if (EV) {
            acc.e += use ? phi - p.ecut : 0.0;
            acc.add_virial(gg, dx[u], dy[u], dz[u]);
          }
        }
      }
    }
    if (K > 1) acc.reduce<K>(EV);
    finish_atom_with<FUSED>(a, acc, i, live && sl == 0, xi, yi, zi, EV, 0.0, vi, xri);
  }
  };
  if (fits)
    groups(std::true_type());
  else
    groups(std::false_type());
}

// LJ from a half list (each pair once, Newton's third law): atom i's own sum
// as in k_lj, and -F_ij added to atom j with an FP64 atomic add per
// component; atom i's total is added atomically too (other rows add into it
// concurrently), so f must be zero on entry.  The whole pair energy and
// virial go to atom i.
template <int PREC, bool EV, int K>
__global__ __launch_bounds__(kBlock) void k_lj_half(FK a, LJK p) {
  const Lane<K> ln(a);
  const int n = a.n;
  const int io = ln.live ? ln.i : n - 1;
  double xi, yi, zi;
  home_pos(a, io, xi, yi, zi);
  Acc acc;
  double* __restrict__ f = a.f;
  for_each_batch<K, PREC == MD_MIXED>(a, ln, xi, yi, zi, [&](const Batch& b) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const bool use = b.ok[u] && b.s[u] < p.rc2;
      double g, phi;
      lj_pair<PREC>(use ? b.s[u] : 1.0, p, g, phi);
      g = use ? g : 0.0;
      acc.add_force(g, b.dx[u], b.dy[u], b.dz[u]);
      if (use) {
        const int j = b.j[u];
        unsafeAtomicAdd(f + j, -(g * b.dx[u]));
        unsafeAtomicAdd(f + n + j, -(g * b.dy[u]));
        unsafeAtomicAdd(f + 2 * n + j, -(g * b.dz[u]));
      }
      if (EV) {
        acc.e += use ? phi - p.ecut : 0.0;
        acc.add_virial(g, b.dx[u], b.dy[u], b.dz[u]);
      }
    }
  });
  if (K > 1) acc.reduce<K>(EV);
  if (!ln.live || ln.s != 0) return;
  const int i = ln.i;
  unsafeAtomicAdd(f + i, acc.fx);
  unsafeAtomicAdd(f + n + i, acc.fy);
  unsafeAtomicAdd(f + 2 * n + i, acc.fz);
  if (EV) {
    // store_ev halves its sums (full-list convention); the half list's are whole
    Acc whole = acc;
    whole.e *= 2.0;
    whole.w0 *= 2.0;
    whole.w1 *= 2.0;
    whole.w2 *= 2.0;
    whole.w3 *= 2.0;
    whole.w4 *= 2.0;
    whole.w5 *= 2.0;
    whole.store_ev(a, i, true, 0.0);
  }
}

// ------------------------------------------- Buckingham + cut Coulomb --

// g = -(dphi/dr) / r and phi at r^2 = s for one species pair, from its row
// (A, A / rho, 1 / rho, C, 6 C, qq): phi = A e - C / r^6 + qq / r with
// e = exp(-r / rho), -(dphi/dr) = (A / rho) e - 6 C / r^7 + qq / r^2.
template <int PREC>
__device__ inline void buck_pair(double s, const double* row, const float* rowf, double& g,
                                 double& phi) {
  if (PREC == MD_FP64) {
    const double r = sqrt(s);
    const double ri = rcp64(r);
    const double r2i = ri * ri;
    const double r6i = r2i * r2i * r2i;
    const double ex = exp(-r * row[2]);
    phi = row[0] * ex - row[3] * r6i + row[5] * ri;
    g = ri * (row[1] * ex - row[4] * r6i * ri + row[5] * r2i);
  } else {
    const float sf = (float)s;
    const float r = __builtin_sqrtf(sf);
    const float ri = __builtin_amdgcn_rcpf(r);
    const float r2i = ri * ri;
    const float r6i = r2i * r2i * r2i;
    const float ex = __builtin_amdgcn_exp2f(-r * rowf[2]);   // rowf[2] = log2(e) / rho
    phi = (double)(rowf[0] * ex - rowf[3] * r6i + rowf[5] * ri);
    g = (double)(ri * (rowf[1] * ex - rowf[4] * r6i * ri + rowf[5] * r2i));
  }
}

template <int PREC, bool EV, int K, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_buck(FK a0, BuckK p) {
  const FK a = with_box(a0);
  // the species-pair rows, staged once per workgroup
  __shared__ double rows[16 * 6];
  __shared__ float rowsf[16 * 6];
  if (threadIdx.x < 16 * 6) {
    rows[threadIdx.x] = p.row[threadIdx.x / 6][threadIdx.x % 6];
    rowsf[threadIdx.x] = p.rowf[threadIdx.x / 6][threadIdx.x % 6];
  }
  __syncthreads();
  if (a.clear && blockIdx.x == 0 && threadIdx.x == 0) *a.clear = 0;
  const Lane<K> ln(a);
  const int n = a.n;
  const int io = ln.live ? ln.i : n - 1;
  double xi, yi, zi;
  home_pos(a, io, xi, yi, zi);
  const int ti = (int)a.xq[4 * (size_t)io + 3] & 3;
  Acc acc;
  for_each_batch<K, false, true>(a, ln, xi, yi, zi, [&](const Batch& b) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      // pairs outside the cutoff or past the lane's list contribute an exact zero
      const bool use = b.ok[u] && b.s[u] < p.rc2;
      const int ab = 6 * (4 * ti + b.t[u]);
      double g, phi;
      buck_pair<PREC>(use ? b.s[u] : 1.0, rows + ab, rowsf + ab, g, phi);
      g = use ? g : 0.0;
      acc.add_force(g, b.dx[u], b.dy[u], b.dz[u]);
      if (EV) {
        acc.e += use ? phi : 0.0;
        acc.add_virial(g, b.dx[u], b.dy[u], b.dz[u]);
      }
    }
  });
  if (K > 1) acc.reduce<K>(EV);
  finish_atom<FUSED>(a, acc, ln.i, ln.live && ln.s == 0, xi, yi, zi, EV, 0.0);
}

// --------------------------------------------------------- Sutton-Chen --

// t^(k/2) for integer k >= 0.
template <typename T>
__device__ inline T half_power(T t, int k) {
  T r = (T)1;
  for (int q = 0; q < k / 2; ++q) r *= t;
  if (k & 1) r *= sqrt(t);
  return r;
}

// Pass 1: rho_i = sum_j (a^2/s)^(m/2); stores e_i = rho_i^(-1/2) (0 if rho_i = 0)
// in e_out and in the fourth word of atom i's packed record (xq_w: the same
// buffer as a.xq, of which this pass reads only the first three words), where
// pass 2 finds it with the neighbour's position; with EV, also the embedding
// energy -eps c sqrt(rho_i).
template <int PREC, bool EV, int K>
__global__ __launch_bounds__(kBlock) void k_sc_density(FK a0, SCK p, double* __restrict__ e_out,
                                                        double* xq_w) {
  const FK a = with_box(a0);
  const Lane<K> ln(a);
  const int n = a.n;
  const int io = ln.live ? ln.i : n - 1;
  double xi, yi, zi;
  home_pos(a, io, xi, yi, zi);
  double rho = 0.0;
  for_each_batch<K, PREC == MD_MIXED>(a, ln, xi, yi, zi, [&](const Batch& b) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (b.ok[u] && b.s[u] < p.rc2) {
        if (PREC == MD_FP64)
          rho += half_power(p.a2 * rcp64(b.s[u]), p.m);
        else
          rho += (double)half_power(p.a2f * __builtin_amdgcn_rcpf((float)b.s[u]), p.m);
      }
    }
  });
  if (K > 1) rho = group_sum<K>(rho);
  if (!ln.live || ln.s != 0) return;
  const double ei = rho > 0.0 ? 1.0 / sqrt(rho) : 0.0;
  e_out[ln.i] = ei;
  xq_w[4 * (size_t)ln.i + 3] = ei;
  if (EV && a.eatom) a.eatom[ln.i] = -p.epsc * sqrt(rho);
}

// Pass 2: F_ij = [n eps t^(n/2) - (m eps c / 2)(e_i + e_j) t^(m/2)] d / s, t = a^2/s.
template <int PREC, bool EV, int K, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_sc_force(FK a0, SCK p,
                                                      const double* __restrict__ e_in) {
  const FK a = with_box(a0);
  if (a.clear && blockIdx.x == 0 && threadIdx.x == 0) *a.clear = 0;
  const Lane<K> ln(a);
  const int n = a.n;
  const int io = ln.live ? ln.i : n - 1;
  double xi, yi, zi;
  home_pos(a, io, xi, yi, zi);
  const double ei = e_in[io];
  Acc acc;
  // e_j comes with j's position: the fourth word of its record (pass 1)
  for_each_batch<K, false, false, true>(a, ln, xi, yi, zi, [&](const Batch& b) {
    const double* ej = b.w3;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (b.ok[u] && b.s[u] < p.rc2) {
        double h, pn;
        if (PREC == MD_FP64) {
          const double r2i = rcp64(b.s[u]);
          const double tt = p.a2 * r2i;
          pn = half_power(tt, p.n);
          const double pm = half_power(tt, p.m);
          h = (p.neps * pn - p.mepsc_half * (ei + ej[u]) * pm) * r2i;
        } else {
          const float r2i = __builtin_amdgcn_rcpf((float)b.s[u]);
          const float tt = p.a2f * r2i;
          const float pnf = half_power(tt, p.n);
          const float pmf = half_power(tt, p.m);
          const float eij = (float)(ei + ej[u]);
          h = (double)((p.nepsf * pnf - p.mepsc_halff * eij * pmf) * r2i);
          pn = (double)pnf;
        }
        acc.add_force(h, b.dx[u], b.dy[u], b.dz[u]);
        if (EV) {
          acc.e += pn;
          acc.add_virial(h, b.dx[u], b.dy[u], b.dz[u]);
        }
      }
    }
  });
  if (K > 1) acc.reduce<K>(EV);
  // energy: eps/2 sum_j t^(n/2) is the pair repulsion share, plus the embedding
  // term pass 1 stored
  const bool own = ln.live && ln.s == 0;
  const double emb = (EV && a.eatom && own) ? a.eatom[ln.i] : 0.0;
  acc.e *= p.eps;
  finish_atom<FUSED>(a, acc, ln.i, own, xi, yi, zi, EV, emb);
}

// ------------------------------------------------------------- LJ VJP --

// Sums of a and b over the workgroup in a fixed order (lane shuffles down
// each wavefront, then the wavefronts in order), written by thread 0 to
// out[0], out[1].  Every thread of the workgroup calls it.
__device__ inline void block_sum2(double a, double b, double* out) {
  __shared__ double sh[2][kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    a += __shfl_down(a, off, kWave);
    b += __shfl_down(b, off, kWave);
  }
  if (lane == 0) {
    sh[0][wave] = a;
    sh[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = sh[0][0], sb = sh[1][0];
#pragma unroll
    for (int w = 1; w < kBlock / kWave; ++w) {
      sa += sh[0][w];
      sb += sh[1][w];
    }
    out[0] = sa;
    out[1] = sb;
  }
}

// gx_i = sum_j [g (u_i - u_j) + 2 g' ((u_i - u_j) . d) d];
// pe_i = u_i . F_i (for dL/deps = sum pe / eps); ps_i = sum_j (dg/dsigma)(u_i . d).
template <int PREC, int K>
__global__ __launch_bounds__(kBlock) void k_lj_vjp(FK a, LJK p, const double* __restrict__ u,
                                                    double* __restrict__ gx,
                                                    double* __restrict__ bp) {
  const Lane<K> ln(a);
  const int n = a.n;
  const int io = ln.live ? ln.i : n - 1;
  double xi, yi, zi;
  home_pos(a, io, xi, yi, zi);
  const double uxi = u[io], uyi = u[n + io], uzi = u[2 * n + io];
  double gxa = 0, gya = 0, gza = 0, fx = 0, fy = 0, fz = 0, dsig = 0;
  for_each_batch<K, PREC == MD_MIXED>(a, ln, xi, yi, zi, [&](const Batch& b) {
    double ux[kUnroll], uy[kUnroll], uz[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      ux[q] = u[b.j[q]];
      uy[q] = u[n + b.j[q]];
      uz[q] = u[2 * n + b.j[q]];
    }
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      if (!(b.ok[q] && b.s[q] < p.rc2)) continue;
      double g, gp, dg;
      if (PREC == MD_FP64) {
        const double r2i = rcp64(b.s[q]);
        const double sr2 = p.sig2 * r2i;
        const double sr6 = sr2 * sr2 * sr2;
        const double sr12 = sr6 * sr6;
        g = r2i * (2.0 * p.eps24 * sr12 - p.eps24 * sr6);
        gp = r2i * r2i * (-14.0 * p.eps24 * sr12 + 4.0 * p.eps24 * sr6);
        dg = p.inv_sig * r2i * (24.0 * p.eps24 * sr12 - 6.0 * p.eps24 * sr6);
      } else {
        const float r2i = __builtin_amdgcn_rcpf((float)b.s[q]);
        const float sr2 = p.sig2f * r2i;
        const float sr6 = sr2 * sr2 * sr2;
        const float sr12 = sr6 * sr6;
        g = (double)(r2i * (2.0f * p.eps24f * sr12 - p.eps24f * sr6));
        gp = (double)(r2i * r2i * (-14.0f * p.eps24f * sr12 + 4.0f * p.eps24f * sr6));
        dg = p.inv_sig * (double)(r2i * (24.0f * p.eps24f * sr12 - 6.0f * p.eps24f * sr6));
      }
      const double dux = uxi - ux[q], duy = uyi - uy[q], duz = uzi - uz[q];
      const double c2 = 2.0 * gp * (dux * b.dx[q] + duy * b.dy[q] + duz * b.dz[q]);
      gxa += g * dux + c2 * b.dx[q];
      gya += g * duy + c2 * b.dy[q];
      gza += g * duz + c2 * b.dz[q];
      fx = fma(g, b.dx[q], fx);
      fy = fma(g, b.dy[q], fy);
      fz = fma(g, b.dz[q], fz);
      dsig += dg * (uxi * b.dx[q] + uyi * b.dy[q] + uzi * b.dz[q]);
    }
  });
  if (K > 1) {
    gxa = group_sum<K>(gxa);
    gya = group_sum<K>(gya);
    gza = group_sum<K>(gza);
    fx = group_sum<K>(fx);
    fy = group_sum<K>(fy);
    fz = group_sum<K>(fz);
    dsig = group_sum<K>(dsig);
  }
  const bool own = ln.live && ln.s == 0;
  if (own) {
    const int i = ln.i;
    gx[i] = gxa;
    gx[n + i] = gya;
    gx[2 * n + i] = gza;
  }
  // the workgroup's sums of u_i . F_i and of the sigma term, into its row
  // of bp (rows in atom order)
  if (bp)
    block_sum2(own ? uxi * fx + uyi * fy + uzi * fz : 0.0, own ? dsig : 0.0,
               bp + 2 * (size_t)xcd_block());
}

// ------------------------------------------------------- Sutton-Chen VJP --

// Pair factors of the Sutton-Chen forces at r^2 = s, t = a^2 / s:
// A = n eps t^(n/2) / s and Bc = -(m/2) eps t^(m/2) / s (B = c Bc), so that
// F_i = sum_j [A + B (e_i + e_j)] d_ij; psi = t^(m/2).
template <int PREC>
__device__ inline void sc_pair_factors(const SCK& p, double s, double& r2i, double& A,
                                       double& Bc, double& psi) {
  if (PREC == MD_FP64) {
    r2i = rcp64(s);
    const double tt = p.a2 * r2i;
    psi = half_power(tt, p.m);
    A = p.neps * half_power(tt, p.n) * r2i;
    Bc = -p.meps_half * psi * r2i;
  } else {
    const float rf = __builtin_amdgcn_rcpf((float)s);
    const float tt = p.a2f * rf;
    const float pm = half_power(tt, p.m);
    r2i = (double)rf;
    psi = (double)pm;
    A = (double)(p.nepsf * half_power(tt, p.n) * rf);
    Bc = (double)(-p.meps_halff * pm * rf);
  }
}

// Pass 2 of the adjoint: with w_ij = (u_i - u_j) . d_ij, g_i / c = sum_j Bc w,
// la_i = 1/2 sum_j A w; stores lam_i = -1/2 e_i^3 c (g_i / c) (= dL/drho_i),
// la_i and lb_i = e_i (g_i / c).
template <int PREC, int K>
__global__ __launch_bounds__(kBlock) void k_sc_vjp_rho(FK a, SCK p, const double* __restrict__ u,
                                                        const double* __restrict__ e,
                                                        double* __restrict__ lam,
                                                        double* __restrict__ la,
                                                        double* __restrict__ lb,
                                                        double* __restrict__ uq) {
  const Lane<K> ln(a);
  const int n = a.n;
  const int io = ln.live ? ln.i : n - 1;
  double xi, yi, zi;
  home_pos(a, io, xi, yi, zi);
  const double uxi = u[io], uyi = u[n + io], uzi = u[2 * n + io];
  double gc = 0.0, lai = 0.0;
  for_each_batch<K, PREC == MD_MIXED>(a, ln, xi, yi, zi, [&](const Batch& b) {
    double ux[kUnroll], uy[kUnroll], uz[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      ux[q] = u[b.j[q]];
      uy[q] = u[n + b.j[q]];
      uz[q] = u[2 * n + b.j[q]];
    }
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      if (!(b.ok[q] && b.s[q] < p.rc2)) continue;
      double r2i, A, Bc, psi;
      sc_pair_factors<PREC>(p, b.s[q], r2i, A, Bc, psi);
      const double w = (uxi - ux[q]) * b.dx[q] + (uyi - uy[q]) * b.dy[q] +
                       (uzi - uz[q]) * b.dz[q];
      gc = fma(Bc, w, gc);
      lai = fma(0.5 * A, w, lai);
    }
  });
  if (K > 1) {
    gc = group_sum<K>(gc);
    lai = group_sum<K>(lai);
  }
  if (!ln.live || ln.s != 0) return;
  const int i = ln.i;
  const double ei = e[i];
  const double li = -0.5 * ei * ei * ei * (p.c * gc);
  lam[i] = li;
  la[i] = lai;
  lb[i] = ei * gc;
  // (u_i, lam_i) packed for the position pass's neighbour gathers
  double2* rec = reinterpret_cast<double2*>(uq + 4 * (size_t)i);
  rec[0] = make_double2(uxi, uyi);
  rec[1] = make_double2(uzi, li);
}

// Pass 3: dL/dx_i = sum_j [h (u_i - u_j) + 2 h' w d + 2 (lam_i + lam_j) psi' d],
// h = A + B (e_i + e_j), h' = -(n/2 + 1) A / s - (m/2 + 1) B (e_i + e_j) / s,
// psi' = -(m/2) psi / s.
template <int PREC, int K>
__global__ __launch_bounds__(kBlock) void k_sc_vjp_x(FK a, SCK p, const double* __restrict__ u,
                                                      const double* __restrict__ e,
                                                      const double* __restrict__ lam,
                                                      const double* __restrict__ uq,
                                                      double* __restrict__ gx) {
  const Lane<K> ln(a);
  const int n = a.n;
  const int io = ln.live ? ln.i : n - 1;
  double xi, yi, zi;
  home_pos(a, io, xi, yi, zi);
  const double uxi = u[io], uyi = u[n + io], uzi = u[2 * n + io];
  const double ei = e[io], li = lam[io];
  const double hn = 0.5 * p.n + 1.0, hm = 0.5 * p.m + 1.0, mh = 0.5 * p.m;
  double gxa = 0.0, gya = 0.0, gza = 0.0;
  const __amdgpu_buffer_rsrc_t ur = buffer_of(uq, n);
  // e_j comes with j's position (the density pass stored it in the record),
  // u_j and lam_j with the record the previous pass packed
  for_each_batch<K, false, false, true>(a, ln, xi, yi, zi, [&](const Batch& b) {
    double ux[kUnroll], uy[kUnroll], uz[kUnroll], lj[kUnroll];
    const double* ej = b.w3;
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) load_rec(ur, b.j[q], ux[q], uy[q], uz[q], lj[q]);
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      if (!(b.ok[q] && b.s[q] < p.rc2)) continue;
      double r2i, A, Bc, psi;
      sc_pair_factors<PREC>(p, b.s[q], r2i, A, Bc, psi);
      const double Be = p.c * Bc * (ei + ej[q]);
      const double h = A + Be;
      const double hp = -(hn * A + hm * Be) * r2i;
      const double lp = -2.0 * mh * (li + lj[q]) * psi * r2i;   // 2 (lam_i + lam_j) psi'
      const double dux = uxi - ux[q], duy = uyi - uy[q], duz = uzi - uz[q];
      const double c2 = 2.0 * hp * (dux * b.dx[q] + duy * b.dy[q] + duz * b.dz[q]) + lp;
      gxa += h * dux + c2 * b.dx[q];
      gya += h * duy + c2 * b.dy[q];
      gza += h * duz + c2 * b.dz[q];
    }
  });
  if (K > 1) {
    gxa = group_sum<K>(gxa);
    gya = group_sum<K>(gya);
    gza = group_sum<K>(gza);
  }
  if (!ln.live || ln.s != 0) return;
  const int i = ln.i;
  gx[i] = gxa;
  gx[n + i] = gya;
  gx[2 * n + i] = gza;
}

// ------------------------------------------------------------ launching --

FK make_fk(const ForceArgs& a) {
  FK k;
  k.xq = a.xq;
  k.n = a.n;
  k.box = a.box;
  k.boxd = a.boxd;
  k.margin = a.margin;
  k.neigh = a.neigh;
  k.numneigh = a.numneigh;
  k.cap = a.cap;
  k.f = a.f;
  k.eatom = a.ev.eatom;
  k.vatom = a.ev.vatom;
  k.vtrace = a.ev.vtrace;
  k.clear = a.clear;
  k.in = a.in;
  return k;
}

template <typename... KArgs, typename... Args>
hipError_t launch_timed(void (*kern)(KArgs...), unsigned grid, hipStream_t s, hipEvent_t t0,
                        hipEvent_t t1, Args... args) {
  if (t0 && t1)
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, t0, t1, 0, args...);
  else
    kern<<<grid, kBlock, 0, s>>>(args...);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_pack_positions(const double* __restrict__ x, int n,
                                                            double* __restrict__ xq,
                                                            const int* __restrict__ type) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) store_packed(xq, i, x[i], x[n + i], x[2 * n + i], type ? type[i] : 0);
}

// Workgroups covering n atoms with K lanes each.
unsigned grid_for(int n, int k) {
  const int64_t lanes = (int64_t)((n + (kWave / k) - 1) / (kWave / k)) * kWave;
  return (unsigned)((lanes + kBlock - 1) / kBlock);
}

// Calls f(std::integral_constant<int, K>) for the runtime lane count.
template <typename F>
hipError_t with_lanes(int k, F&& f) {
  switch (k) {
    case 1: return f(std::integral_constant<int, 1>());
    case 2: return f(std::integral_constant<int, 2>());
    case 4: return f(std::integral_constant<int, 4>());
    case 8: return f(std::integral_constant<int, 8>());
    case 16: return f(std::integral_constant<int, 16>());
    case 32: return f(std::integral_constant<int, 32>());
    case 64: return f(std::integral_constant<int, 64>());
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_pack_positions(const double* x, int n, double* xq, const int* type,
                                 hipStream_t s);


hipError_t launch_pack_positions(const double* x, int n, double* xq, const int* type,
                                 hipStream_t s) {
  k_pack_positions<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(x, n, xq, type);
  return hipGetLastError();
}

// Tiled LJ: one workgroup of kTileBlock threads per run.
static hipError_t launch_lj_tile(const ForceArgs& a, const LJK& p, int prec, int lanes,
                                 hipStream_t s) {
  const FK k = make_fk(a);
  const bool ev = a.ev.eatom || a.ev.vatom || a.ev.vtrace;
  const TileArgs ta{a.tile, a.cell_start, a.tg};
  const unsigned grid = (unsigned)tile_nruns(a.tg);
  const bool fused = a.in.mode != MD_INT_NONE;
  auto go = [&](auto kern) -> hipError_t {
    if (a.t0 && a.t1)
      hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kTileBlock), 0, s, a.t0, a.t1, 0, k, p, ta);
    else
      kern<<<grid, kTileBlock, 0, s>>>(k, p, ta);
    return hipGetLastError();
  };
  auto pick = [&](auto kc) -> hipError_t {
    constexpr int K = decltype(kc)::value;
    if (prec == MD_FP64) {
      if (fused) return ev ? go(k_lj_tile<MD_FP64, true, K, true>) : go(k_lj_tile<MD_FP64, false, K, true>);
      return ev ? go(k_lj_tile<MD_FP64, true, K, false>) : go(k_lj_tile<MD_FP64, false, K, false>);
    }
    if (fused) return ev ? go(k_lj_tile<MD_MIXED, true, K, true>) : go(k_lj_tile<MD_MIXED, false, K, true>);
    return ev ? go(k_lj_tile<MD_MIXED, true, K, false>) : go(k_lj_tile<MD_MIXED, false, K, false>);
  };
  switch (lanes) {
    case 1: return pick(std::integral_constant<int, 1>());
    case 2: return pick(std::integral_constant<int, 2>());
    case 4: return pick(std::integral_constant<int, 4>());
    case 8: return pick(std::integral_constant<int, 8>());
  }
  return hipErrorInvalidValue;
}

hipError_t launch_lj(const ForceArgs& a, const LJK& p, int prec, int lanes, hipStream_t s) {
  if (lanes & MD_LAYOUT_TILE) return launch_lj_tile(a, p, prec, lanes & ~MD_LAYOUT_TILE, s);
  const FK k = make_fk(a);
  const bool ev = a.ev.eatom || a.ev.vatom;
  const bool fused = a.in.mode != MD_INT_NONE;
  const bool tr = !ev && a.ev.vtrace;   // the trace alone: fused kernels only
  if (tr && !fused) return hipErrorInvalidValue;
  return with_lanes(lanes, [&](auto kc) -> hipError_t {
    constexpr int K = decltype(kc)::value;
    const unsigned g = grid_for(a.n, K);
    if (tr)
      return prec == MD_FP64
                 ? launch_timed(k_lj<MD_FP64, false, K, true, true>, g, s, a.t0, a.t1, k, p)
                 : launch_timed(k_lj<MD_MIXED, false, K, true, true>, g, s, a.t0, a.t1, k, p);
    if (prec == MD_FP64) {
      if (fused)
        return ev ? launch_timed(k_lj<MD_FP64, true, K, true>, g, s, a.t0, a.t1, k, p)
                  : launch_timed(k_lj<MD_FP64, false, K, true>, g, s, a.t0, a.t1, k, p);
      return ev ? launch_timed(k_lj<MD_FP64, true, K, false>, g, s, a.t0, a.t1, k, p)
                : launch_timed(k_lj<MD_FP64, false, K, false>, g, s, a.t0, a.t1, k, p);
    }
    if (fused)
      return ev ? launch_timed(k_lj<MD_MIXED, true, K, true>, g, s, a.t0, a.t1, k, p)
                : launch_timed(k_lj<MD_MIXED, false, K, true>, g, s, a.t0, a.t1, k, p);
    return ev ? launch_timed(k_lj<MD_MIXED, true, K, false>, g, s, a.t0, a.t1, k, p)
              : launch_timed(k_lj<MD_MIXED, false, K, false>, g, s, a.t0, a.t1, k, p);
  });
}

hipError_t launch_lj_half(const ForceArgs& a, const LJK& p, int prec, int lanes, hipStream_t s) {
  const FK k = make_fk(a);
  const bool ev = a.ev.eatom || a.ev.vatom || a.ev.vtrace;
  return with_lanes(lanes, [&](auto kc) -> hipError_t {
    constexpr int K = decltype(kc)::value;
    const unsigned g = grid_for(a.n, K);
    if (prec == MD_FP64)
      return ev ? launch_timed(k_lj_half<MD_FP64, true, K>, g, s, a.t0, a.t1, k, p)
                : launch_timed(k_lj_half<MD_FP64, false, K>, g, s, a.t0, a.t1, k, p);
    return ev ? launch_timed(k_lj_half<MD_MIXED, true, K>, g, s, a.t0, a.t1, k, p)
              : launch_timed(k_lj_half<MD_MIXED, false, K>, g, s, a.t0, a.t1, k, p);
  });
}

hipError_t launch_buck(const ForceArgs& a, const BuckK& p, int prec, int lanes, hipStream_t s) {
  const FK k = make_fk(a);
  const bool ev = a.ev.eatom || a.ev.vatom || a.ev.vtrace;
  return with_lanes(lanes, [&](auto kc) -> hipError_t {
    constexpr int K = decltype(kc)::value;
    const unsigned g = grid_for(a.n, K);
    const bool fused = a.in.mode != MD_INT_NONE;
    if (prec == MD_FP64) {
      if (fused)
        return ev ? launch_timed(k_buck<MD_FP64, true, K, true>, g, s, a.t0, a.t1, k, p)
                  : launch_timed(k_buck<MD_FP64, false, K, true>, g, s, a.t0, a.t1, k, p);
      return ev ? launch_timed(k_buck<MD_FP64, true, K, false>, g, s, a.t0, a.t1, k, p)
                : launch_timed(k_buck<MD_FP64, false, K, false>, g, s, a.t0, a.t1, k, p);
    }
    if (fused)
      return ev ? launch_timed(k_buck<MD_MIXED, true, K, true>, g, s, a.t0, a.t1, k, p)
                : launch_timed(k_buck<MD_MIXED, false, K, true>, g, s, a.t0, a.t1, k, p);
    return ev ? launch_timed(k_buck<MD_MIXED, true, K, false>, g, s, a.t0, a.t1, k, p)
              : launch_timed(k_buck<MD_MIXED, false, K, false>, g, s, a.t0, a.t1, k, p);
  });
}

hipError_t launch_sc(const ForceArgs& a, const SCK& p, int prec, int lanes, double* sc_e,
                     hipStream_t s) {
  const FK k = make_fk(a);
  const bool ev = a.ev.eatom || a.ev.vatom || a.ev.vtrace;
  return with_lanes(lanes, [&](auto kc) -> hipError_t {
    constexpr int K = decltype(kc)::value;
    const unsigned g = grid_for(a.n, K);
    const double* e = sc_e;
    // pass 1 (density) is not timed; the timed launch is the force pass
    const bool fused = a.in.mode != MD_INT_NONE;
    auto force = [&](auto prec_c, auto ev_c) -> hipError_t {
      constexpr int P = decltype(prec_c)::value;
      constexpr bool E = decltype(ev_c)::value;
      k_sc_density<P, E, K><<<g, kBlock, 0, s>>>(k, p, sc_e, const_cast<double*>(a.xq));
      return fused ? launch_timed(k_sc_force<P, E, K, true>, g, s, a.t0, a.t1, k, p, e)
                   : launch_timed(k_sc_force<P, E, K, false>, g, s, a.t0, a.t1, k, p, e);
    };
    using F64 = std::integral_constant<int, MD_FP64>;
    using MIX = std::integral_constant<int, MD_MIXED>;
    using YES = std::integral_constant<bool, true>;
    using NO = std::integral_constant<bool, false>;
    if (prec == MD_FP64) return ev ? force(F64(), YES()) : force(F64(), NO());
    return ev ? force(MIX(), YES()) : force(MIX(), NO());
  });
}

hipError_t launch_lj_vjp(const ForceArgs& a, const LJK& p, int prec, int lanes,
                         const double* u, double* gx, double* bp, int* rows, hipStream_t s) {
  const FK k = make_fk(a);
  return with_lanes(lanes, [&](auto kc) -> hipError_t {
    constexpr int K = decltype(kc)::value;
    const unsigned g = grid_for(a.n, K);
    if (rows) *rows = (int)g;
    if (prec == MD_FP64)
      return launch_timed(k_lj_vjp<MD_FP64, K>, g, s, a.t0, a.t1, k, p, u, gx, bp);
    return launch_timed(k_lj_vjp<MD_MIXED, K>, g, s, a.t0, a.t1, k, p, u, gx, bp);
  });
}

hipError_t launch_sc_vjp(const ForceArgs& a, const SCK& p, int prec, int lanes, const double* u,
                         double* e, double* lam, double* la, double* lb, double* uq, double* gx,
                         hipStream_t s) {
  const FK k = make_fk(a);
  return with_lanes(lanes, [&](auto kc) -> hipError_t {
    constexpr int K = decltype(kc)::value;
    const unsigned g = grid_for(a.n, K);
    auto run = [&](auto prec_c) -> hipError_t {
      constexpr int P = decltype(prec_c)::value;
      k_sc_density<P, false, K><<<g, kBlock, 0, s>>>(k, p, e, const_cast<double*>(a.xq));
      k_sc_vjp_rho<P, K><<<g, kBlock, 0, s>>>(k, p, u, e, lam, la, lb, uq);
      return launch_timed(k_sc_vjp_x<P, K>, g, s, a.t0, a.t1, k, p, u,
                          static_cast<const double*>(e), static_cast<const double*>(lam),
                          static_cast<const double*>(uq), gx);
    };
    if (prec == MD_FP64) return run(std::integral_constant<int, MD_FP64>());
    return run(std::integral_constant<int, MD_MIXED>());
  });
}

}  // namespace md
