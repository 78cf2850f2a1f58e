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

// Block tree sum in LDS (fixed shape, so the result is deterministic).
__device__ inline double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (t < off) sh[t] += sh[t + off];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Stage 1: block b sums its contiguous chunk of each column.
__global__ __launch_bounds__(kBlock) void k_sum_stage1(SumArgs a) {
  __shared__ double sh[kBlock];
  const int per = (a.n + kReduceBlocks - 1) / kReduceBlocks;
  const int b0 = blockIdx.x * per;
  const int b1 = min(a.n, b0 + per);
  for (int c = 0; c < a.cols; ++c) {
    double s = 0.0;
    const double* col = a.col[c];
    for (int i = b0 + threadIdx.x; i < b1; i += kBlock) s += col[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) a.partials[blockIdx.x * kReduceCols + c] = s;
  }
}

// Stage 2: one block sums the kReduceBlocks partials of each column; with
// NHC, thread 0 then runs the thermostat chain update on the sums it wrote.
template <bool NHC>
__global__ __launch_bounds__(kReduceBlocks) void k_sum_stage2(SumArgs a, NhcArgs h) {
  __shared__ double sh[kReduceBlocks];
  for (int c = 0; c < a.cols; ++c) {
    const double s = block_sum(a.partials[threadIdx.x * kReduceCols + c], sh);
    if (threadIdx.x == 0) a.out[c] = s;
  }
  if (NHC && threadIdx.x == 0) nhc_update(h);
}

__global__ void k_thermo_row(ThermoArgs a) {
  if (threadIdx.x != 0) return;
  const double* s = a.sums;
  const double pe = s[0];
  const double ke = 0.5 * a.mvv2e * a.mass * s[7];
  a.row[0] = a.step;
  a.row[1] = pe;
  a.row[2] = ke;
  a.row[3] = pe + ke;
  a.row[4] = 2.0 * ke / (a.dof * a.boltz);
  a.row[5] = (2.0 * ke + (s[1] + s[2] + s[3])) / (3.0 * a.volume);
  a.row[6] = (double)a.status[MD_ST_BUILDS];
  a.row[7] = (double)a.status[MD_ST_MAXNEIGH];
  if (a.extra) a.row[8] = a.row[3] + *a.extra;
}

__global__ void k_vjp_params(const double* sums, double eps, double* gparam) {
  if (threadIdx.x != 0) return;
  gparam[0] = sums[0] / eps;
  gparam[1] = sums[1];
}

// Sutton-Chen: L = LA + c LB with LA ~ a^n and c LB ~ a^(m/2) (A ~ a^n,
// B ~ a^m, e ~ a^(-m/2)); sums = (LA, LB).
__global__ void k_sc_vjp_params(const double* sums, double eps, double a, double c, double n,
                                double m, double* gparam) {
  if (threadIdx.x != 0) return;
  gparam[0] = (sums[0] + c * sums[1]) / eps;
  gparam[1] = (n * sums[0] + 0.5 * m * c * sums[1]) / a;
  gparam[2] = sums[1];
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

hipError_t launch_thermo_row(const ThermoArgs& a, hipStream_t s) {
  k_thermo_row<<<1, 64, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_sc_vjp_params(const double* sums, const SCK& p, double a, double* gparam,
                                hipStream_t s) {
  k_sc_vjp_params<<<1, 64, 0, s>>>(sums, p.eps, a, p.c, (double)p.n, (double)p.m, gparam);
  return hipGetLastError();
}

hipError_t launch_vjp_params(const double* sums, double eps, double* gparam, hipStream_t s) {
  k_vjp_params<<<1, 64, 0, s>>>(sums, eps, gparam);
  return hipGetLastError();
}

}  // namespace md
