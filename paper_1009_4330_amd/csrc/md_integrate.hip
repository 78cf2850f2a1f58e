// Velocity-Verlet NVE kernels, the half-skin displacement check, and the
// deterministic two-stage sums behind energy, virial and thermo output.
#include "md_internal.hpp"

namespace md {
namespace {

// v += dtfm f; x += dt v; request a rebuild when |x - x_ref|^2 > (skin/2)^2.
// All products and sums are evaluated as written (no contraction), so the
// trajectory arithmetic is plain IEEE double.
__global__ __launch_bounds__(kBlock) void k_kick_drift_check(
    double* __restrict__ x, double* __restrict__ v, const double* __restrict__ f,
    const double* __restrict__ xr, int n, double dtfm, double dt, double trig2,
    int* __restrict__ status, BinOut bin) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool live = i < n;
  bool finite = true;
  double xn[3] = {0.0, 0.0, 0.0}, dd[3] = {0.0, 0.0, 0.0};
  if (live) {
    for (int d = 0; d < 3; ++d) {
      const int q = d * n + i;
      const double vn = v[q] + dtfm * f[q];
      xn[d] = x[q] + dt * vn;
      v[q] = vn;
      x[q] = xn[d];
      dd[d] = xn[d] - xr[q];
      finite = finite && isfinite(xn[d]);
    }
  }
  drift_flags(xn, dd, trig2, i, finite, live, status, bin);
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

// Stage 2: one block sums the kReduceBlocks partials of each column.
__global__ __launch_bounds__(kReduceBlocks) void k_sum_stage2(SumArgs a) {
  __shared__ double sh[kReduceBlocks];
  for (int c = 0; c < a.cols; ++c) {
    const double s = block_sum(a.partials[threadIdx.x * kReduceCols + c], sh);
    if (threadIdx.x == 0) a.out[c] = s;
  }
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
                                   const BinOut& bin, hipStream_t s) {
  k_kick_drift_check<<<blocks_for(n), kBlock, 0, s>>>(x, v, f, xr, n, dtfm, dt, trig2, status,
                                                       bin);
  return hipGetLastError();
}



hipError_t launch_ke(const double* v, int n, double* keatom, hipStream_t s) {
  k_ke<<<blocks_for(n), kBlock, 0, s>>>(v, n, keatom);
  return hipGetLastError();
}

hipError_t launch_sum(const SumArgs& a, hipStream_t s) {
  k_sum_stage1<<<kReduceBlocks, kBlock, 0, s>>>(a);
  hipError_t st = hipGetLastError();
  if (st != hipSuccess) return st;
  k_sum_stage2<<<1, kReduceBlocks, 0, s>>>(a);
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
