// Velocity-Verlet NVE kernels, the half-skin displacement check, and the
// deterministic two-stage sums behind energy, virial and thermo output.
#include "md_internal.hpp"

namespace md {
namespace {

// v += dtfm f; x += dt v; request a rebuild when |x - x_ref|^2 > (skin/2)^2.
// With a thermostat the velocities are first multiplied by *scale.  All
// products and sums are evaluated as written (no contraction), so the
// trajectory arithmetic is plain IEEE double.
__global__ __launch_bounds__(kBlock) void k_kick_drift_check(
    double* __restrict__ x, double* __restrict__ v, const double* __restrict__ f,
    const double* __restrict__ xr, int n, double dtfm, double dt, double trig2,
    int* __restrict__ status, BinOut bin, const double* __restrict__ scale) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool live = i < n;
  bool finite = true;
  double xn[3] = {0.0, 0.0, 0.0}, dd[3] = {0.0, 0.0, 0.0};
  if (live) {
    const double sc = scale ? *scale : 1.0;
    for (int d = 0; d < 3; ++d) {
      const int q = d * n + i;
      const double vs = scale ? v[q] * sc : v[q];
      const double vn = vs + dtfm * f[q];
      xn[d] = x[q] + dt * vn;
      v[q] = vn;
      x[q] = xn[d];
      dd[d] = xn[d] - xr[q];
      finite = finite && isfinite(xn[d]);
    }
  }
  drift_flags(xn, dd, trig2, i, finite, live, status, bin);
}

__global__ __launch_bounds__(kBlock) void k_scale_v(double* __restrict__ v, int n,
                                                     const double* __restrict__ scale) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= 3 * n) return;
  v[i] = v[i] * *scale;
}

// Nose-Hoover chain half step over a time dt/2 (Martyna-Tuckerman-Klein
// splitting): chain velocities updated from the last thermostat down to the
// first, particle velocities scaled by exp(-dt/2 w_1), chain positions
// advanced, chain velocities updated back up.  Thermostat forces:
// G_1 = (ke2 - nf kT) / Q_1, G_j = (Q_{j-1} w_{j-1}^2 - kT) / Q_j.  Each
// velocity update: w_j <- w_j c^2 + (dt/4) G_j c with c = exp(-(dt/8) w_{j+1})
// (no factor for the last thermostat).  The chain lives in registers (loops
// over the fixed maximum length, guarded by M).  Returns the scale factor and
// leaves ke2 scaled.
__device__ double nhc_half_step(const NhcArgs& a, double (&eta)[MD_NHC_MAX],
                                double (&w)[MD_NHC_MAX], double& ke2) {
  const int M = a.M;
  const double h4 = 0.25 * a.dt, h8 = 0.125 * a.dt;
  auto update = [&](int j) {
    const double G = j == 0 ? (ke2 - a.nf * a.kT) / a.Q0
                            : ((j == 1 ? a.Q0 : a.Qj) * w[j - 1] * w[j - 1] - a.kT) / a.Qj;
    if (j == M - 1) {
      w[j] = w[j] + h4 * G;
    } else {
      const double c = exp(-h8 * w[j + 1 < MD_NHC_MAX ? j + 1 : j]);
      w[j] = w[j] * c * c + h4 * G * c;
    }
  };
#pragma unroll
  for (int j = MD_NHC_MAX - 1; j >= 0; --j)
    if (j < M) update(j);
  const double sc = exp(-0.5 * a.dt * w[0]);
  ke2 = ke2 * sc * sc;
#pragma unroll
  for (int j = 0; j < MD_NHC_MAX; ++j)
    if (j < M) eta[j] = eta[j] + 0.5 * a.dt * w[j];
#pragma unroll
  for (int j = 0; j < MD_NHC_MAX; ++j)
    if (j < M) update(j);
  return sc;
}

// The chain update of one step (see NhcArgs), by one thread.
__device__ void nhc_update(const NhcArgs& a) {
  double eta[MD_NHC_MAX], w[MD_NHC_MAX];
#pragma unroll
  for (int j = 0; j < MD_NHC_MAX; ++j) {
    eta[j] = a.state[j];
    w[j] = a.state[MD_NHC_MAX + j];
  }
  double ke2 = a.vsum ? a.mke * *a.vsum : a.state[kNhcKe2];
  double sc = 1.0;
  if (a.end) {
    const double f = nhc_half_step(a, eta, w, ke2);
    if (a.vsum_out) *a.vsum_out = *a.vsum * f * f;
    sc = f;
  }
  double e = a.nf * a.kT * eta[0];
#pragma unroll
  for (int j = 0; j < MD_NHC_MAX; ++j)
    if (j < a.M) e += 0.5 * (j == 0 ? a.Q0 : a.Qj) * w[j] * w[j];
#pragma unroll
  for (int j = 1; j < MD_NHC_MAX; ++j)
    if (j < a.M) e += a.kT * eta[j];
  if (a.start) sc = sc * nhc_half_step(a, eta, w, ke2);
#pragma unroll
  for (int j = 0; j < MD_NHC_MAX; ++j) {
    a.state[j] = eta[j];
    a.state[MD_NHC_MAX + j] = w[j];
  }
  a.state[kNhcEnergy] = e;
  a.state[kNhcScale] = sc;
  a.state[kNhcKe2] = ke2;
}

__global__ void k_nhc(NhcArgs a) {
  if (threadIdx.x == 0 && blockIdx.x == 0) nhc_update(a);
}

__global__ __launch_bounds__(kBlock) void k_ke(const double* __restrict__ v, int n,
                                                double* __restrict__ keatom) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double a = v[i], b = v[n + i], c = v[2 * n + i];
  keatom[i] = a * a + b * b + c * c;
}

// Block tree sums of the first `cols` of the kReduceCols values each thread
// holds, all columns at once: the levels across wavefronts in LDS (sh holds
// NT x kReduceCols doubles), the levels within the first wavefront by lane
// shuffles.  Pairing and order are those of the plain halving tree
// (s[t] += s[t + off] for off = NT/2 .. 1), so the sums are deterministic;
// thread 0 ends with them in v.
template <int NT>
__device__ inline void block_sums(double (&v)[kReduceCols], int cols, double* sh) {
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < kReduceCols; ++c)
    if (c < cols) sh[c * NT + t] = v[c];
#pragma unroll
  for (int off = NT / 2; off >= kWave; off >>= 1) {
    __syncthreads();
    if (t < off) {
#pragma unroll
      for (int c = 0; c < kReduceCols; ++c)
        if (c < cols) sh[c * NT + t] += sh[c * NT + t + off];
    }
  }
  __syncthreads();
  if (t < kWave) {
#pragma unroll
    for (int c = 0; c < kReduceCols; ++c) {
      if (c < cols) {
        double s = sh[c * NT + t];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_down(s, off, kWave);
        v[c] = s;
      }
    }
  }
}

// Stage 1: block b sums its contiguous chunk of each column (the columns
// read side by side).
__global__ __launch_bounds__(kBlock) void k_sum_stage1(SumArgs a) {
  __shared__ double sh[kReduceCols * kBlock];
  const int per = (a.n + kReduceBlocks - 1) / kReduceBlocks;
  const int b0 = blockIdx.x * per;
  const int b1 = min(a.n, b0 + per);
  double s[kReduceCols];
#pragma unroll
  for (int c = 0; c < kReduceCols; ++c) s[c] = 0.0;
  for (int i = b0 + threadIdx.x; i < b1; i += kBlock) {
#pragma unroll
    for (int c = 0; c < kReduceCols; ++c)
      if (c < a.cols && a.col[c]) s[c] += a.col[c][i];
  }
  block_sums<kBlock>(s, a.cols, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < kReduceCols; ++c)
      if (c < a.cols) a.partials[blockIdx.x * kReduceCols + c] = s[c];
  }
}

// Stage 2's sums: the partials of each column, into a.out.  Stage 1's
// kReduceBlocks rows give each thread one row; other partials (a.nparts
// rows) are first added row by row, thread t taking rows t, t + kReduceBlocks, ...
__device__ inline void sum_partials(const SumArgs& a, double* sh) {
  double s[kReduceCols];
  if (a.nparts == 0) {
#pragma unroll
    for (int c = 0; c < kReduceCols; ++c)
      s[c] = c < a.cols ? a.partials[threadIdx.x * kReduceCols + c] : 0.0;
  } else {
#pragma unroll
    for (int c = 0; c < kReduceCols; ++c) s[c] = 0.0;
    for (int r = threadIdx.x; r < a.nparts; r += kReduceBlocks) {
#pragma unroll
      for (int c = 0; c < kReduceCols; ++c)
        if (c < a.cols) s[c] += a.partials[(size_t)r * a.cols + c];
    }
  }
  block_sums<kReduceBlocks>(s, a.cols, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < kReduceCols; ++c)
      if (c < a.cols) a.out[c] = s[c];
  }
}

// The adjoints' parameter gradients from the two sums (ParamArgs).
__device__ inline void finish_params(const ParamArgs& p, const double* out) {
  if (p.kind == kParamsLJ) {
    p.gparam[0] = out[0] / p.eps;
    p.gparam[1] = out[1];
  } else if (p.kind == kParamsSC) {
    p.gparam[0] = (out[0] + p.c * out[1]) / p.eps;
    p.gparam[1] = (p.nexp * out[0] + 0.5 * p.mexp * p.c * out[1]) / p.a;
    p.gparam[2] = out[1];
  }
}

// Stage 2: one block sums the kReduceBlocks partials of each column; thread
// 0 then runs, on the sums it wrote, the thermostat chain update (NHC) and
// the adjoints' parameter gradients (a.params).
template <bool NHC>
__global__ __launch_bounds__(kReduceBlocks) void k_sum_stage2(SumArgs a, NhcArgs h) {
  __shared__ double sh[kReduceCols * kReduceBlocks];
  sum_partials(a, sh);
  if (NHC && threadIdx.x == 0) nhc_update(h);
  if (threadIdx.x == 0 && a.params.kind != kParamsNone) finish_params(a.params, a.out);
}

__global__ void k_thermo_row(ThermoArgs a) {
  if (threadIdx.x != 0) return;
  const double* s = a.sums;
  const double pe = s[0];
  const double ke = 0.5 * a.mvv2e * a.mass * s[7];
  const double volume = a.vol ? *a.vol : a.volume;
  a.row[0] = a.step;
  a.row[1] = pe;
  a.row[2] = ke;
  a.row[3] = pe + ke;
  a.row[4] = 2.0 * ke / (a.dof * a.boltz);
  a.row[5] = (2.0 * ke + (s[1] + s[2] + s[3])) / (3.0 * volume);
  a.row[6] = (double)a.status[MD_ST_BUILDS];
  a.row[7] = (double)a.status[MD_ST_MAXNEIGH];
  if (a.extra) a.row[8] = a.row[3] + *a.extra;
  if (a.vol) a.row[9] = volume;
}

// ------------------------------------------------------------------ NPT --

// sinh(x) / x; near 0 its Taylor series (to x^8, exact to rounding there).
__device__ inline double sinh_over_x(double x) {
  if (fabs(x) < 1e-3) {
    const double q = x * x;
    return 1.0 + q / 6.0 * (1.0 + q / 20.0 * (1.0 + q / 42.0 * (1.0 + q / 72.0)));
  }
  return sinh(x) / x;
}

// The barostat / thermostat update of md_step_npt (one thread).  Isotropic
// barostat of Martyna, Tobias and Klein: momentum p_eps of mass W, force
// G_eps = alpha ke2 + tr W - 3 V P_ext (alpha = 1 + 3 / Nf), a Nose-Hoover
// chain on the particles (nhc_half_step as for NVT) and one on the barostat
// (the same step with G_1 = (p_eps^2 / W - kT) / Q'_1, scaling p_eps).
// Closing half (end): p_eps half step, particle chain, barostat chain; then
// the extended energy (both chain energies, p_eps^2 / 2W, P_ext V).  Opening
// half (start): barostat chain, particle chain, p_eps half step, then with
// v_e = p_eps / W the step's factors: kick a = exp(-alpha v_e dt/2),
// b = exp(-alpha v_e dt/4) sinh(x)/x at x = alpha v_e dt/4; drift c = exp(v_e dt),
// e = dt exp(v_e dt/2) sinh(y)/y at y = v_e dt/2; the box grows by c, and the
// rebuild bound is skin/2 - (1 - s) rl/2 with s the box scale since the last
// build (negative: rebuild now).  A box edge below nc rl (the run's cell grid
// no longer covers rl) sets status bit 3.
//
// Run by the 64 lanes of one wavefront: the two chains are independent
// within each half, so even lanes step the particle chain and odd lanes the
// barostat chain in the same instructions, and the results are exchanged by
// lane shuffles (the arithmetic of each chain is unchanged).  Lane 0 writes
// the state, lane 1 the barostat chain.
__device__ void npt_update(const NptArgs& a) {
  double* st = a.state;
  const int lane = threadIdx.x & (kWave - 1);
  const bool baro = lane & 1;
  double ch[MD_NHC_MAX], cw[MD_NHC_MAX];   // this lane's chain
#pragma unroll
  for (int j = 0; j < MD_NHC_MAX; ++j) {
    ch[j] = st[(baro ? kNptXi : kNptEta) + j];
    cw[j] = st[(baro ? kNptVxi : kNptVeta) + j];
  }
  double peps = st[kNptPeps];
  double L[3] = {st[kNptL], st[kNptL + 1], st[kNptL + 2]};
  const double lref = st[kNptLref];
  double vol = L[0] * L[1] * L[2];
  const double trw = *a.trw;
  const double vs = a.vsum ? *a.vsum : 0.0;
  double ke2 = a.vsum ? a.mke * vs : st[kNptKe2];
  NhcArgs c{};
  c.M = a.M;
  c.Q0 = baro ? a.Qb : a.Q0;
  c.Qj = baro ? a.Qb : a.Qj;
  c.kT = a.kT;
  c.nf = baro ? 1.0 : a.nf;
  c.dt = a.dt;
  // one half step of both chains: the particle chain on ke2, the barostat
  // chain on p_eps^2 / W; returns (particle factor, barostat factor)
  auto chains = [&](double& fp, double& fb) {
    double q = baro ? peps * peps / a.W : ke2;
    const double f = nhc_half_step(c, ch, cw, q);
    fp = __shfl(f, 0, kWave);
    fb = __shfl(f, 1, kWave);
    ke2 = __shfl(q, 0, kWave);
  };
  double sc = 1.0, vs_out = 0.0;
  if (a.end) {
    peps = peps + 0.5 * a.dt * (a.alpha * ke2 + trw - 3.0 * vol * a.ptarget);
    double fp, fb;
    chains(fp, fb);
    vs_out = vs * fp * fp;
    sc = fp;
    peps = peps * fb;
  }
  double eta[MD_NHC_MAX], w[MD_NHC_MAX], xi[MD_NHC_MAX], wx[MD_NHC_MAX];
#pragma unroll
  for (int j = 0; j < MD_NHC_MAX; ++j) {
    eta[j] = __shfl(ch[j], 0, kWave);
    w[j] = __shfl(cw[j], 0, kWave);
    xi[j] = __shfl(ch[j], 1, kWave);
    wx[j] = __shfl(cw[j], 1, kWave);
  }
  double e = a.nf * a.kT * eta[0] + a.kT * xi[0] + 0.5 * a.Qb * wx[0] * wx[0];
#pragma unroll
  for (int j = 0; j < MD_NHC_MAX; ++j)
    if (j < a.M) e += 0.5 * (j == 0 ? a.Q0 : a.Qj) * w[j] * w[j];
#pragma unroll
  for (int j = 1; j < MD_NHC_MAX; ++j)
    if (j < a.M) e += a.kT * eta[j] + a.kT * xi[j] + 0.5 * a.Qb * wx[j] * wx[j];
  e += 0.5 * peps * peps / a.W + a.ptarget * vol;
  const double vol_state = vol;   // the volume of this state (thermo), before the next box
  double ka = 0.0, kb = 0.0, dc = 0.0, de = 0.0, sb = 0.0, thr2 = 0.0;
  bool small = false;
  if (a.start) {
    double fp, fb;
    chains(fp, fb);
    peps = peps * fb;
    sc = sc * fp;
    peps = peps + 0.5 * a.dt * (a.alpha * ke2 + trw - 3.0 * vol * a.ptarget);
    const double ve = peps / a.W;
    const double xa = a.alpha * ve * 0.25 * a.dt;
    ka = exp(-a.alpha * ve * 0.5 * a.dt);
    kb = exp(-xa) * sinh_over_x(xa);
    dc = exp(ve * a.dt);
    de = a.dt * exp(ve * 0.5 * a.dt) * sinh_over_x(ve * 0.5 * a.dt);
    for (int d = 0; d < 3; ++d) {
      L[d] = L[d] * dc;
      small = small || L[d] < (double)a.nc[d] * a.rl;
    }
    sb = L[0] / lref;
    const double thr = 0.5 * a.skin - 0.5 * (1.0 - sb) * a.rl;
    thr2 = thr < 0.0 ? -1.0 : thr * thr;
  }
  if (lane == 1) {
#pragma unroll
    for (int j = 0; j < MD_NHC_MAX; ++j) {
      st[kNptXi + j] = ch[j];
      st[kNptVxi + j] = cw[j];
    }
  }
  if (lane != 0) return;
#pragma unroll
  for (int j = 0; j < MD_NHC_MAX; ++j) {
    st[kNptEta + j] = ch[j];
    st[kNptVeta + j] = cw[j];
  }
  if (a.end && a.vsum_out) *a.vsum_out = vs_out;
  st[kNptVol] = vol_state;
  if (a.start) {
    st[kNptKa] = ka;
    st[kNptKb] = kb;
    st[kNptDc] = dc;
    st[kNptDe] = de;
    for (int d = 0; d < 3; ++d) st[kNptL + d] = L[d];
    if (small) atomicOr(&a.status[MD_ST_ERRORS], 8);
    st[kNptSb] = sb;
    st[kNptThr2] = thr2;
  }
  st[kNptPeps] = peps;
  st[kNptScale] = sc;
  st[kNptKe2] = ke2;
  st[kNptEnergy] = e;
}

// The update runs on the first wavefront once thread 0's sums are written
// (the barrier makes them visible to the other lanes).
__global__ __launch_bounds__(kReduceBlocks) void k_sum_stage2_npt(SumArgs a, NptArgs h) {
  __shared__ double sh[kReduceCols * kReduceBlocks];
  sum_partials(a, sh);
  __syncthreads();
  if (threadIdx.x < kWave) npt_update(h);
}

// v <- v scale; v <- v a + (dtfm f) b; x <- x c + e v (factors from the
// update kernel); rebuild request when |x - s x_ref|^2 exceeds the bound.
__global__ __launch_bounds__(kBlock) void k_kick_drift_npt(
    double* __restrict__ x, double* __restrict__ v, const double* __restrict__ f,
    const double* __restrict__ xr, int n, double dtfm, int* __restrict__ status, BinOut bin,
    const double* __restrict__ st) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool live = i < n;
  const double sc = st[kNptScale], ka = st[kNptKa], kb = st[kNptKb], dc = st[kNptDc],
               de = st[kNptDe], sb = st[kNptSb], thr2 = st[kNptThr2];
  bool finite = true;
  double xn[3] = {0.0, 0.0, 0.0}, dd[3] = {0.0, 0.0, 0.0};
  if (live) {
    for (int d = 0; d < 3; ++d) {
      const int q = d * n + i;
      const double vs = v[q] * sc;
      const double vn = vs * ka + (dtfm * f[q]) * kb;
      xn[d] = x[q] * dc + de * vn;
      v[q] = vn;
      x[q] = xn[d];
      dd[d] = xn[d] - sb * xr[q];
      finite = finite && isfinite(xn[d]);
    }
  }
  drift_flags(xn, dd, thr2, i, finite, live, status, bin);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_kick_drift_check(double* x, double* v, const double* f, const double* xr,
                                   int n, double dtfm, double dt, double trig2, int* status,
                                   const BinOut& bin, const double* scale, hipStream_t s) {
  k_kick_drift_check<<<blocks_for(n), kBlock, 0, s>>>(x, v, f, xr, n, dtfm, dt, trig2, status,
                                                       bin, scale);
  return hipGetLastError();
}

hipError_t launch_scale_v(double* v, int n, const double* scale, hipStream_t s) {
  k_scale_v<<<blocks_for(3 * (int64_t)n), kBlock, 0, s>>>(v, n, scale);
  return hipGetLastError();
}

hipError_t launch_nhc(const NhcArgs& a, hipStream_t s) {
  k_nhc<<<1, 64, 0, s>>>(a);
  return hipGetLastError();
}



hipError_t launch_ke(const double* v, int n, double* keatom, hipStream_t s) {
  k_ke<<<blocks_for(n), kBlock, 0, s>>>(v, n, keatom);
  return hipGetLastError();
}

hipError_t launch_sum(const SumArgs& a, hipStream_t s, const NhcArgs* nhc) {
  k_sum_stage1<<<kReduceBlocks, kBlock, 0, s>>>(a);
  hipError_t st = hipGetLastError();
  if (st != hipSuccess) return st;
  if (nhc)
    k_sum_stage2<true><<<1, kReduceBlocks, 0, s>>>(a, *nhc);
  else
    k_sum_stage2<false><<<1, kReduceBlocks, 0, s>>>(a, NhcArgs{});
  return hipGetLastError();
}

hipError_t launch_sum_parts(const SumArgs& a, hipStream_t s) {
  k_sum_stage2<false><<<1, kReduceBlocks, 0, s>>>(a, NhcArgs{});
  return hipGetLastError();
}

hipError_t launch_sum_npt(const SumArgs& a, const NptArgs& npt, hipStream_t s) {
  k_sum_stage1<<<kReduceBlocks, kBlock, 0, s>>>(a);
  hipError_t st = hipGetLastError();
  if (st != hipSuccess) return st;
  k_sum_stage2_npt<<<1, kReduceBlocks, 0, s>>>(a, npt);
  return hipGetLastError();
}

hipError_t launch_kick_drift_npt(double* x, double* v, const double* f, const double* xr, int n,
                                 double dtfm, int* status, const BinOut& bin,
                                 const double* state, hipStream_t s) {
  k_kick_drift_npt<<<blocks_for(n), kBlock, 0, s>>>(x, v, f, xr, n, dtfm, status, bin, state);
  return hipGetLastError();
}

hipError_t launch_thermo_row(const ThermoArgs& a, hipStream_t s) {
  k_thermo_row<<<1, 64, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace md
