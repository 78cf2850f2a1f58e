/*
 * md_oracle.c -- plain FP64 CPU reference for the short-range MD hot path.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The HIP library never
 * calls it, and the two share no source: no headers, kernels, helpers or
 * tables.  Inputs come from the seeded generators, never from the HIP path.
 *
 * Everything is IEEE FP64, built with -O2 -ffp-contract=off -fno-fast-math so
 * that every expression is evaluated exactly as written (no FMA contraction).
 * OpenMP parallelises only loops over atoms whose iterations write disjoint
 * outputs; every sum over atoms is then taken sequentially in index order.
 *
 * What is computed (the method of the paper, section "Neighbor list approach",
 * with the textbook physics it leaves implicit):
 *   - wrap into the periodic box and bin atoms into cells of edge >= r_l
 *     (cell list of section "Cell list approach");
 *   - a full Verlet list: every ordered pair (i, j), i != j, whose minimum-
 *     image separation satisfies r^2 < r_l^2, r_l = r_c + skin (the per-atom
 *     neighbor loop of the TpA/BpA listings reads such a list);
 *   - 12-6 Lennard-Jones (lj/cut of Appendix A), analytic Sutton-Chen
 *     (standing in for the EAM system of Appendix A) and Buckingham + cut
 *     Coulomb (the silicate system of Appendix A) forces, energy, virial;
 *   - velocity-Verlet NVE integration ("NVE integrator", section "Design
 *     objectives") with a rebuild of the list whenever an atom moved more than
 *     skin/2 since the last build;
 *   - NVT integration (the NVT integrator named in "Design objectives") by a
 *     Nose-Hoover chain thermostat in the standard time-reversible splitting
 *     of Martyna, Tuckerman and Klein: a thermostat half step, the
 *     velocity-Verlet step, a thermostat half step;
 *   - isotropic NPT integration (the NPT integrator named in "Design
 *     objectives"): the barostat of Martyna, Tobias and Klein with
 *     Nose-Hoover chains on the particles and on the barostat, in the
 *     splitting of Tuckerman et al.  One term of it is parity unpinned: the
 *     3 / N_f part of the barostat's kinetic factor alpha = 1 + 3 / N_f keeps
 *     the extended energy conserved with or without it and moves the volume
 *     distribution only at order 1 / N, so no test isolates it;
 *   - the vector-Jacobian products of the LJ forces (with respect to
 *     positions and (eps, sigma)) and of the Sutton-Chen forces (positions and
 *     (eps, a, c)).
 * Status codes: 0 ok, 1 invalid argument, 2 box too small, 3 list overflow
 * (numneigh still holds the true counts; *max_count the largest).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_EBOX 2
#define ORC_EOVERFLOW 3

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* ---------------------------------------------------------------- cells -- */

/* Cells per dimension: the largest count whose edge L/nc is still >= r_l. */
int orc_cell_dims(const double* L, double rl, int* nc) {
  for (int d = 0; d < 3; ++d) {
    if (!(L[d] > 2.0 * rl)) return ORC_EBOX;
    nc[d] = (int)floor(L[d] / rl);
  }
  return ORC_OK;
}

/* Map one coordinate into [0, L). */
static double wrap1(double x, double L) {
  double r = x - L * floor(x / L);
  if (r < 0.0) r += L;
  if (r >= L) r = 0.0;
  return r;
}

/* Cell index of a wrapped coordinate, clamped to [0, nc-1]. */
static int cell1(double r, int nc, double L) {
  int c = (int)((r * (double)nc) / L);
  if (c < 0) c = 0;
  if (c > nc - 1) c = nc - 1;
  return c;
}

/* Wrap x (SoA [3][n]) in place, bin into cells (x fastest), and produce the
   stable counting-sort permutation: perm lists atom indices cell by cell, in
   increasing atom index inside each cell; cell_start has ncell+1 entries. */
int orc_bin(int64_t n, double* x, const double* L, double rl, int* nc,
            int* atom_cell, int* cell_start, int* perm) {
  if (n <= 0 || !x || !L || !nc || !atom_cell || !cell_start || !perm) return ORC_EINVAL;
  int st = orc_cell_dims(L, rl, nc);
  if (st) return st;
  const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
  for (int d = 0; d < 3; ++d)
    for (int64_t i = 0; i < n; ++i) x[d * n + i] = wrap1(x[d * n + i], L[d]);
  for (int64_t i = 0; i < n; ++i) {
    int cx = cell1(x[i], nc[0], L[0]);
    int cy = cell1(x[n + i], nc[1], L[1]);
    int cz = cell1(x[2 * n + i], nc[2], L[2]);
    atom_cell[i] = cx + nc[0] * (cy + nc[1] * cz);
  }
  for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = 0;
  for (int64_t i = 0; i < n; ++i) cell_start[atom_cell[i] + 1] += 1;
  for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
  int* cursor = (int*)malloc(sizeof(int) * (size_t)ncell);
  if (!cursor) return ORC_EINVAL;
  for (int64_t c = 0; c < ncell; ++c) cursor[c] = cell_start[c];
  for (int64_t i = 0; i < n; ++i) perm[cursor[atom_cell[i]]++] = (int)i;
  free(cursor);
  return ORC_OK;
}

/* Minimum-image component: d - L * rint(d / L). */
static double min_image(double d, double L) { return d - L * rint(d / L); }

/* Squared distance as ((dx*dx + dy*dy) + dz*dz), minimum image. */
static double dist2(const double* x, int64_t n, const double* L, int64_t i, int64_t j,
                    double* d) {
  d[0] = min_image(x[i] - x[j], L[0]);
  d[1] = min_image(x[n + i] - x[n + j], L[1]);
  d[2] = min_image(x[2 * n + i] - x[2 * n + j], L[2]);
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* Distinct neighbour cell coordinates along one dimension (c-1, c, c+1 mod nc,
   duplicates dropped in that order). Returns how many. */
static int stencil1(int c, int nc, int* out) {
  int k = 0;
  for (int o = -1; o <= 1; ++o) {
    int v = ((c + o) % nc + nc) % nc;
    int dup = 0;
    for (int q = 0; q < k; ++q) dup |= (out[q] == v);
    if (!dup) out[k++] = v;
  }
  return k;
}

/* Full Verlet list from a binned configuration.  For every atom i, the atoms of
   the (up to) 27 surrounding cells are tested in cell order and, inside each
   cell, in perm order; j is kept when r^2 < rl*rl.  The list is row-major,
   neigh[i*cap + k].  Counts beyond cap are still counted, not stored. */
int orc_build_nlist(int64_t n, const double* x, const double* L, const int* nc,
                    const int* atom_cell, const int* cell_start, const int* perm,
                    double rl, int cap, int* numneigh, int* neigh, int* max_count) {
  if (n <= 0 || cap < 1 || !x || !numneigh || !neigh) return ORC_EINVAL;
  const double rl2 = rl * rl;
  int maxc = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(max : maxc)
  for (int64_t i = 0; i < n; ++i) {
    int c = atom_cell[i];
    int cx = c % nc[0], cy = (c / nc[0]) % nc[1], cz = c / (nc[0] * nc[1]);
    int sx[3], sy[3], sz[3];
    int kx = stencil1(cx, nc[0], sx), ky = stencil1(cy, nc[1], sy), kz = stencil1(cz, nc[2], sz);
    int cnt = 0;
    for (int a = 0; a < kz; ++a)
      for (int b = 0; b < ky; ++b)
        for (int e = 0; e < kx; ++e) {
          int cc = sx[e] + nc[0] * (sy[b] + nc[1] * sz[a]);
          for (int p = cell_start[cc]; p < cell_start[cc + 1]; ++p) {
            int64_t j = perm[p];
            if (j == i) continue;
            double d[3];
            if (dist2(x, n, L, i, j, d) < rl2) {
              if (cnt < cap) neigh[i * (int64_t)cap + cnt] = (int)j;
              ++cnt;
            }
          }
        }
    numneigh[i] = cnt;
    if (cnt > maxc) maxc = cnt;
  }
  if (max_count) *max_count = maxc;
  return maxc > cap ? ORC_EOVERFLOW : ORC_OK;
}

/* ------------------------------------------------------- Lennard-Jones -- */

/* 12-6 LJ over a full list.  For every listed pair with s = r^2 < rc*rc:
     sr6 = (sigma^2/s)^3,  phi = 4 eps (sr6^2 - sr6),
     g = 24 eps sr6 (2 sr6 - 1) / s  (so that F_ij = g d, d = x_i - x_j).
   f_i = sum_j g d; the pair energy and virial d (x) d g are split half to each
   atom of the pair (each unordered pair appears twice in a full list).  With
   shift != 0 phi(rc) is subtracted per interacting pair.  Outputs: f [3][n];
   eatom [n] and vatom [6][n] (xx yy zz xy xz yz) may be NULL; energy [1] and
   virial [6] totals are sums over atoms in index order (may be NULL). */
int orc_lj_forces(int64_t n, const double* x, const double* L, const int* numneigh,
                  const int* neigh, int cap, double rc, double eps, double sigma,
                  int shift, double* f, double* eatom, double* vatom, double* energy,
                  double* virial) {
  if (n <= 0 || !x || !numneigh || !neigh || !f) return ORC_EINVAL;
  const double rc2 = rc * rc, sig2 = sigma * sigma;
  double ecut = 0.0;
  if (shift) {
    double sr6c = (sig2 / rc2) * (sig2 / rc2) * (sig2 / rc2);
    ecut = 4.0 * eps * (sr6c * sr6c - sr6c);
  }
  double* ea = (double*)calloc((size_t)n, sizeof(double));
  double* va = (double*)calloc((size_t)n * 6, sizeof(double));
  if (!ea || !va) { free(ea); free(va); return ORC_EINVAL; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double fi[3] = {0.0, 0.0, 0.0}, ei = 0.0, wi[6] = {0, 0, 0, 0, 0, 0};
    int cnt = numneigh[i] < cap ? numneigh[i] : cap;
    for (int k = 0; k < cnt; ++k) {
      int64_t j = neigh[i * (int64_t)cap + k];
      double d[3];
      double s = dist2(x, n, L, i, j, d);
      if (!(s < rc2)) continue;
      double sr2 = sig2 / s;
      double sr6 = sr2 * sr2 * sr2;
      double g = 24.0 * eps * sr6 * (2.0 * sr6 - 1.0) / s;
      double phi = 4.0 * eps * (sr6 * sr6 - sr6) - ecut;
      for (int q = 0; q < 3; ++q) fi[q] += g * d[q];
      ei += 0.5 * phi;
      wi[0] += 0.5 * d[0] * d[0] * g;
      wi[1] += 0.5 * d[1] * d[1] * g;
      wi[2] += 0.5 * d[2] * d[2] * g;
      wi[3] += 0.5 * d[0] * d[1] * g;
      wi[4] += 0.5 * d[0] * d[2] * g;
      wi[5] += 0.5 * d[1] * d[2] * g;
    }
    for (int q = 0; q < 3; ++q) f[q * n + i] = fi[q];
    ea[i] = ei;
    for (int q = 0; q < 6; ++q) va[q * n + i] = wi[q];
  }
  double et = 0.0, vt[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = 0; i < n; ++i) {
    et += ea[i];
    for (int q = 0; q < 6; ++q) vt[q] += va[q * n + i];
  }
  if (eatom) memcpy(eatom, ea, sizeof(double) * (size_t)n);
  if (vatom) memcpy(vatom, va, sizeof(double) * (size_t)n * 6);
  if (energy) *energy = et;
  if (virial) for (int q = 0; q < 6; ++q) virial[q] = vt[q];
  free(ea);
  free(va);
  return ORC_OK;
}

/* ------------------------------------------ Buckingham + cut Coulomb -- */

/* Buckingham with a plain cut Coulomb term (buck/coul/cut, the potential of
   Appendix A's silicate system), one cutoff rc for both terms:
     phi_ab(r) = A_ab exp(-r / rho_ab) - C_ab / r^6 + qqr2e q_a q_b / r,  r < rc,
   a = type[i], b = type[j] (species 0..3; tables indexed a * 4 + b).  With
     dphi/dr = -(A_ab / rho_ab) exp(-r / rho_ab) + 6 C_ab / r^7 - qqr2e q_a q_b / r^2
   the force on i from j is F_ij = -(dphi/dr) d / r, d = x_i - x_j (minimum
   image).  No energy shift at rc.  Outputs as for LJ. */
int orc_buck_forces(int64_t n, const double* x, const double* L, const int* numneigh,
                    const int* neigh, int cap, double rc, const int* type, const double* A,
                    const double* rho, const double* C, const double* q, double qqr2e,
                    double* f, double* eatom, double* vatom, double* energy, double* virial) {
  if (n <= 0 || !x || !numneigh || !neigh || !f || !type || !A || !rho || !C || !q)
    return ORC_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    if (type[i] < 0 || type[i] > 3) return ORC_EINVAL;
  const double rc2 = rc * rc;
  double* ea = (double*)calloc((size_t)n, sizeof(double));
  double* va = (double*)calloc((size_t)n * 6, sizeof(double));
  if (!ea || !va) { free(ea); free(va); return ORC_EINVAL; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double fb[3] = {0.0, 0.0, 0.0}, eb = 0.0, wb[6] = {0, 0, 0, 0, 0, 0};
    int cnt = numneigh[i] < cap ? numneigh[i] : cap;
    for (int k = 0; k < cnt; ++k) {
      int64_t j = neigh[i * (int64_t)cap + k];
      double d[3];
      double s = dist2(x, n, L, i, j, d);
      if (!(s < rc2)) continue;
      int ab = type[i] * 4 + type[j];
      double r = sqrt(s);
      double ex = A[ab] * exp(-r / rho[ab]);
      double r6 = s * s * s;
      double qq = qqr2e * q[type[i]] * q[type[j]];
      double phi = ex - C[ab] / r6 + qq / r;
      double dphidr = -ex / rho[ab] + 6.0 * C[ab] / (r6 * r) - qq / s;
      double g = -dphidr / r;
      for (int c = 0; c < 3; ++c) fb[c] += g * d[c];
      eb += 0.5 * phi;
      wb[0] += 0.5 * d[0] * d[0] * g;
      wb[1] += 0.5 * d[1] * d[1] * g;
      wb[2] += 0.5 * d[2] * d[2] * g;
      wb[3] += 0.5 * d[0] * d[1] * g;
      wb[4] += 0.5 * d[0] * d[2] * g;
      wb[5] += 0.5 * d[1] * d[2] * g;
    }
    for (int c = 0; c < 3; ++c) f[c * n + i] = fb[c];
    ea[i] = eb;
    for (int c = 0; c < 6; ++c) va[c * n + i] = wb[c];
  }
  double et = 0.0, vt[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = 0; i < n; ++i) {
    et += ea[i];
    for (int c = 0; c < 6; ++c) vt[c] += va[c * n + i];
  }
  if (eatom) memcpy(eatom, ea, sizeof(double) * (size_t)n);
  if (vatom) memcpy(vatom, va, sizeof(double) * (size_t)n * 6);
  if (energy) *energy = et;
  if (virial) for (int c = 0; c < 6; ++c) virial[c] = vt[c];
  free(ea);
  free(va);
  return ORC_OK;
}

/* --------------------------------------------------------- Sutton-Chen -- */

/* Sutton-Chen (Phil. Mag. Lett. 61, 139 (1990)), truncated at rc:
     E = eps * sum_i [ 1/2 sum_j (a/r_ij)^n - c sqrt(rho_i) ],
     rho_i = sum_j (a/r_ij)^m.
   Pass 1 gives rho_i; with e_i = rho_i^(-1/2) (0 for rho_i = 0), pass 2 gives
     F_ij = [ n eps (a/r)^n - (m eps c / 2)(e_i + e_j)(a/r)^m ] d / r^2,
   which is -dE/dx_i split by pair.  Powers are taken as pow(a^2/s, k/2).
   rho [n] receives rho_i; eatom/vatom/energy/virial as for LJ. */
int orc_sc_forces(int64_t n, const double* x, const double* L, const int* numneigh,
                  const int* neigh, int cap, double rc, double eps, double a, double c,
                  int nexp, int mexp, double* f, double* rho, double* eatom, double* vatom,
                  double* energy, double* virial) {
  if (n <= 0 || !x || !numneigh || !neigh || !f) return ORC_EINVAL;
  const double rc2 = rc * rc, a2 = a * a;
  double* r = (double*)calloc((size_t)n, sizeof(double));
  double* em = (double*)calloc((size_t)n, sizeof(double));
  double* ea = (double*)calloc((size_t)n, sizeof(double));
  double* va = (double*)calloc((size_t)n * 6, sizeof(double));
  if (!r || !em || !ea || !va) { free(r); free(em); free(ea); free(va); return ORC_EINVAL; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double ri = 0.0;
    int cnt = numneigh[i] < cap ? numneigh[i] : cap;
    for (int k = 0; k < cnt; ++k) {
      int64_t j = neigh[i * (int64_t)cap + k];
      double d[3];
      double s = dist2(x, n, L, i, j, d);
      if (s < rc2) ri += pow(a2 / s, 0.5 * mexp);
    }
    r[i] = ri;
    em[i] = ri > 0.0 ? 1.0 / sqrt(ri) : 0.0;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double fi[3] = {0.0, 0.0, 0.0}, rep = 0.0, wi[6] = {0, 0, 0, 0, 0, 0};
    int cnt = numneigh[i] < cap ? numneigh[i] : cap;
    for (int k = 0; k < cnt; ++k) {
      int64_t j = neigh[i * (int64_t)cap + k];
      double d[3];
      double s = dist2(x, n, L, i, j, d);
      if (!(s < rc2)) continue;
      double pn = pow(a2 / s, 0.5 * nexp);
      double pm = pow(a2 / s, 0.5 * mexp);
      double h = (nexp * eps * pn - 0.5 * mexp * eps * c * (em[i] + em[j]) * pm) / s;
      for (int q = 0; q < 3; ++q) fi[q] += h * d[q];
      rep += pn;
      wi[0] += 0.5 * d[0] * d[0] * h;
      wi[1] += 0.5 * d[1] * d[1] * h;
      wi[2] += 0.5 * d[2] * d[2] * h;
      wi[3] += 0.5 * d[0] * d[1] * h;
      wi[4] += 0.5 * d[0] * d[2] * h;
      wi[5] += 0.5 * d[1] * d[2] * h;
    }
    for (int q = 0; q < 3; ++q) f[q * n + i] = fi[q];
    ea[i] = eps * (0.5 * rep - c * sqrt(r[i]));
    for (int q = 0; q < 6; ++q) va[q * n + i] = wi[q];
  }
  double et = 0.0, vt[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = 0; i < n; ++i) {
    et += ea[i];
    for (int q = 0; q < 6; ++q) vt[q] += va[q * n + i];
  }
  if (rho) memcpy(rho, r, sizeof(double) * (size_t)n);
  if (eatom) memcpy(eatom, ea, sizeof(double) * (size_t)n);
  if (vatom) memcpy(vatom, va, sizeof(double) * (size_t)n * 6);
  if (energy) *energy = et;
  if (virial) for (int q = 0; q < 6; ++q) virial[q] = vt[q];
  free(r);
  free(em);
  free(ea);
  free(va);
  return ORC_OK;
}

/* ------------------------------------------------------------- LJ VJP -- */

/* Vector-Jacobian product of the LJ forces.  With F_i = sum_j g(s) d and the
   symmetric pair block M = g I + 2 g'(s) d d^T, the cotangent u (on F, [3][n])
   maps to
     gx_i = sum_j [ g (u_i - u_j) + 2 g' ((u_i - u_j) . d) d ]   (= -H u),
   g'(s) = 24 eps (-14 sigma^12 s^-8 + 4 sigma^6 s^-5),
   dL/deps = sum_i u_i . F_i / eps,
   dL/dsigma = sum_i sum_j (dg/dsigma)(s) (u_i . d),
   dg/dsigma = 24 eps (24 sigma^11 s^-7 - 6 sigma^5 s^-4).
   The pair set is the listed pairs with s < rc*rc (rc does not scale with
   sigma).  gparam [2] may be NULL. */
int orc_lj_vjp(int64_t n, const double* x, const double* L, const int* numneigh,
               const int* neigh, int cap, double rc, double eps, double sigma,
               const double* u, double* gx, double* gparam) {
  if (n <= 0 || !x || !numneigh || !neigh || !u || !gx) return ORC_EINVAL;
  const double rc2 = rc * rc;
  const double s6 = pow(sigma, 6.0), s12 = pow(sigma, 12.0);
  const double s5 = pow(sigma, 5.0), s11 = pow(sigma, 11.0);
  double* pe = (double*)calloc((size_t)n, sizeof(double));
  double* ps = (double*)calloc((size_t)n, sizeof(double));
  if (!pe || !ps) { free(pe); free(ps); return ORC_EINVAL; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double gi[3] = {0.0, 0.0, 0.0}, fi[3] = {0.0, 0.0, 0.0}, dsig = 0.0;
    double ui[3] = {u[i], u[n + i], u[2 * n + i]};
    int cnt = numneigh[i] < cap ? numneigh[i] : cap;
    for (int k = 0; k < cnt; ++k) {
      int64_t j = neigh[i * (int64_t)cap + k];
      double d[3];
      double s = dist2(x, n, L, i, j, d);
      if (!(s < rc2)) continue;
      double g = 24.0 * eps * (2.0 * s12 * pow(s, -7.0) - s6 * pow(s, -4.0));
      double gp = 24.0 * eps * (-14.0 * s12 * pow(s, -8.0) + 4.0 * s6 * pow(s, -5.0));
      double dg = 24.0 * eps * (24.0 * s11 * pow(s, -7.0) - 6.0 * s5 * pow(s, -4.0));
      double du[3] = {ui[0] - u[j], ui[1] - u[n + j], ui[2] - u[2 * n + j]};
      double dud = du[0] * d[0] + du[1] * d[1] + du[2] * d[2];
      for (int q = 0; q < 3; ++q) {
        gi[q] += g * du[q] + 2.0 * gp * dud * d[q];
        fi[q] += g * d[q];
      }
      dsig += dg * (ui[0] * d[0] + ui[1] * d[1] + ui[2] * d[2]);
    }
    for (int q = 0; q < 3; ++q) gx[q * n + i] = gi[q];
    pe[i] = ui[0] * fi[0] + ui[1] * fi[1] + ui[2] * fi[2];
    ps[i] = dsig;
  }
  if (gparam) {
    double te = 0.0, ts = 0.0;
    for (int64_t i = 0; i < n; ++i) { te += pe[i]; ts += ps[i]; }
    gparam[0] = te / eps;
    gparam[1] = ts;
  }
  free(pe);
  free(ps);
  return ORC_OK;
}

/* Vector-Jacobian product of the Sutton-Chen forces.  With s = r^2,
   phi(s) = (a^2/s)^(n/2), psi(s) = (a^2/s)^(m/2), rho_i = sum_j psi(s_ij) and
   e_i = rho_i^(-1/2) (0 for an atom without partners), the force is
   F_i = sum_j h_ij d_ij with
     h_ij = A(s_ij) + B(s_ij) (e_i + e_j),
     A(s) = n eps phi / s,   B(s) = -(m/2) eps c psi / s.
   For L = sum_i u_i . F_i = 1/2 sum_ij h_ij w_ij, w_ij = (u_i - u_j) . d_ij,
   differentiating at fixed e and then through e_i(rho_i(x)) gives
     g_i   = sum_j B(s_ij) w_ij                      (dL/de_i)
     lam_i = -1/2 e_i^3 g_i                          (dL/drho_i)
     dL/dx_i = sum_j [ h_ij (u_i - u_j) + 2 h'_ij w_ij d_ij
                       + 2 (lam_i + lam_j) psi'(s_ij) d_ij ]
   with h' = A'(s) + B'(s) (e_i + e_j), A' = -(n/2 + 1) A / s,
   B' = -(m/2 + 1) B / s, psi' = -(m/2) psi / s.  The parameters enter through
   LA = 1/2 sum_ij A_ij w_ij and LB = sum_i e_i g_i (L = LA + LB):
   dL/deps = L / eps, dL/dc = LB / c, dL/da = (n LA + (m/2) LB) / a
   (A ~ a^n, B ~ a^m, e ~ a^(-m/2)).  B and g are carried per unit c, so that
   dL/dc = sum_i e_i g_i / c stays defined at c = 0.  Three passes over the
   list. */
int orc_sc_vjp(int64_t n, const double* x, const double* L, const int* numneigh,
               const int* neigh, int cap, double rc, double eps, double a, double c,
               int nexp, int mexp, const double* u, double* gx, double* gparam) {
  if (n <= 0 || !x || !numneigh || !neigh || !u || !gx) return ORC_EINVAL;
  const double rc2 = rc * rc, a2 = a * a;
  double* e = (double*)calloc((size_t)n, sizeof(double));
  double* lam = (double*)calloc((size_t)n, sizeof(double));
  double* la = (double*)calloc((size_t)n, sizeof(double));
  double* lb = (double*)calloc((size_t)n, sizeof(double));
  if (!e || !lam || !la || !lb) { free(e); free(lam); free(la); free(lb); return ORC_EINVAL; }
  /* pass 1: densities */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double rho_i = 0.0;
    int cnt = numneigh[i] < cap ? numneigh[i] : cap;
    for (int k = 0; k < cnt; ++k) {
      int64_t j = neigh[i * (int64_t)cap + k];
      double d[3];
      double s = dist2(x, n, L, i, j, d);
      if (s < rc2) rho_i += pow(a2 / s, 0.5 * mexp);
    }
    e[i] = rho_i > 0.0 ? 1.0 / sqrt(rho_i) : 0.0;
  }
  /* pass 2: g_i, lam_i and the per-atom parts of LA, LB */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double gci = 0.0, lai = 0.0;   /* gci = g_i / c */
    int cnt = numneigh[i] < cap ? numneigh[i] : cap;
    for (int k = 0; k < cnt; ++k) {
      int64_t j = neigh[i * (int64_t)cap + k];
      double d[3];
      double s = dist2(x, n, L, i, j, d);
      if (!(s < rc2)) continue;
      double A = nexp * eps * pow(a2 / s, 0.5 * nexp) / s;
      double Bc = -0.5 * mexp * eps * pow(a2 / s, 0.5 * mexp) / s;   /* B / c */
      double w = (u[i] - u[j]) * d[0] + (u[n + i] - u[n + j]) * d[1] +
                 (u[2 * n + i] - u[2 * n + j]) * d[2];
      gci += Bc * w;
      lai += 0.5 * A * w;
    }
    lam[i] = -0.5 * e[i] * e[i] * e[i] * (c * gci);
    la[i] = lai;
    lb[i] = e[i] * gci;               /* per unit c */
  }
  /* pass 3: dL/dx */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double gi[3] = {0.0, 0.0, 0.0};
    int cnt = numneigh[i] < cap ? numneigh[i] : cap;
    for (int k = 0; k < cnt; ++k) {
      int64_t j = neigh[i * (int64_t)cap + k];
      double d[3];
      double s = dist2(x, n, L, i, j, d);
      if (!(s < rc2)) continue;
      double phi = pow(a2 / s, 0.5 * nexp), psi = pow(a2 / s, 0.5 * mexp);
      double A = nexp * eps * phi / s;
      double B = -0.5 * mexp * eps * c * psi / s;
      double h = A + B * (e[i] + e[j]);
      double hp = -(0.5 * nexp + 1.0) * A / s - (0.5 * mexp + 1.0) * B / s * (e[i] + e[j]);
      double psip = -0.5 * mexp * psi / s;
      double du[3] = {u[i] - u[j], u[n + i] - u[n + j], u[2 * n + i] - u[2 * n + j]};
      double w = du[0] * d[0] + du[1] * d[1] + du[2] * d[2];
      for (int q = 0; q < 3; ++q)
        gi[q] += h * du[q] + 2.0 * hp * w * d[q] + 2.0 * (lam[i] + lam[j]) * psip * d[q];
    }
    for (int q = 0; q < 3; ++q) gx[q * n + i] = gi[q];
  }
  if (gparam) {
    double ta = 0.0, tb = 0.0;
    for (int64_t i = 0; i < n; ++i) { ta += la[i]; tb += lb[i]; }
    gparam[0] = (ta + c * tb) / eps;
    gparam[1] = (nexp * ta + 0.5 * mexp * c * tb) / a;
    gparam[2] = tb;
  }
  free(e);
  free(lam);
  free(la);
  free(lb);
  return ORC_OK;
}

/* ------------------------------------------------------ NVE integration -- */

typedef struct {
  int kind;                      /* 0 = Lennard-Jones, 1 = Sutton-Chen, 2 = Buckingham + Coulomb */
  double rc, skin;
  double lj_eps, lj_sigma;
  int lj_shift;
  double sc_eps, sc_a, sc_c;
  int sc_n, sc_m;
  double mass, dt, ftm2v, mvv2e, boltz;
  double buck_A[16], buck_rho[16], buck_C[16], q[4], qqr2e;
  const int* type;               /* kind 2: species per atom, input order */
} orc_params;

typedef struct {                 /* per-run working storage */
  int nc[3];
  int *atom_cell, *cell_start, *perm, *numneigh, *neigh;
  double* xref;
  int cap, maxcount;
} orc_work;

static int rebuild(const orc_params* p, int64_t n, double* x, const double* L, orc_work* w) {
  double rl = p->rc + p->skin;
  int st = orc_cell_dims(L, rl, w->nc);
  if (st) return st;
  int64_t ncell = (int64_t)w->nc[0] * w->nc[1] * w->nc[2];
  free(w->cell_start);
  w->cell_start = (int*)malloc(sizeof(int) * (size_t)(ncell + 1));
  st = orc_bin(n, x, L, rl, w->nc, w->atom_cell, w->cell_start, w->perm);
  if (st) return st;
  st = orc_build_nlist(n, x, L, w->nc, w->atom_cell, w->cell_start, w->perm, rl, w->cap,
                       w->numneigh, w->neigh, &w->maxcount);
  memcpy(w->xref, x, sizeof(double) * 3 * (size_t)n);
  return st;
}

static int forces(const orc_params* p, int64_t n, const double* x, const double* L,
                  orc_work* w, double* f, double* pe, double* vir) {
  if (p->kind == 0)
    return orc_lj_forces(n, x, L, w->numneigh, w->neigh, w->cap, p->rc, p->lj_eps,
                         p->lj_sigma, p->lj_shift, f, NULL, NULL, pe, vir);
  if (p->kind == 2)
    return orc_buck_forces(n, x, L, w->numneigh, w->neigh, w->cap, p->rc, p->type, p->buck_A,
                           p->buck_rho, p->buck_C, p->q, p->qqr2e, f, NULL, NULL, pe, vir);
  return orc_sc_forces(n, x, L, w->numneigh, w->neigh, w->cap, p->rc, p->sc_eps, p->sc_a,
                       p->sc_c, p->sc_n, p->sc_m, f, NULL, NULL, NULL, pe, vir);
}

/* Thermo row: step, pe, ke, etot, temp, press, rebuilds, max neighbour count.
   KE = 1/2 m mvv2e sum v^2; T = 2 KE / ((3N-3) kB); P = (2 KE + tr W) / (3V). */
static void thermo_row(const orc_params* p, int64_t n, const double* v, const double* L,
                       double step, double pe, const double* vir, double rebuilds,
                       double maxcount, double* row) {
  double sv = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double a = v[i], b = v[n + i], c = v[2 * n + i];
    sv += (a * a + b * b) + c * c;
  }
  double ke = 0.5 * p->mvv2e * p->mass * sv;
  double dof = 3.0 * (double)n - 3.0;
  double vol = L[0] * L[1] * L[2];
  row[0] = step;
  row[1] = pe;
  row[2] = ke;
  row[3] = pe + ke;
  row[4] = 2.0 * ke / (dof * p->boltz);
  row[5] = (2.0 * ke + (vir[0] + vir[1] + vir[2])) / (3.0 * vol);
  row[6] = rebuilds;
  row[7] = maxcount;
}

/* Velocity-Verlet NVE run (LAMMPS fix nve order):
     setup: wrap + bin + build (x_ref = x), forces, thermo row for step 0;
     each step: v += dtfm f; x += dt v;
                if max_i |x_i - x_ref_i|^2 > (skin/2)^2: wrap + bin + build;
                forces; v += dtfm f;
                thermo row when step % thermo_every == 0,
   with dtfm = (0.5 dt ftm2v) / mass.  x, v (SoA [3][n]) are updated in place
   and stay in input order.  thermo gets 1 + nsteps/thermo_every rows of 8;
   rebuilt[s] (s = 0..nsteps, may be NULL) is 1 where the list was built. */
int orc_md_run(const orc_params* p, int64_t n, double* x, double* v, const double* L,
               int nsteps, int thermo_every, int cap, double* thermo, int* rebuilt,
               double* f_out) {
  if (n <= 1 || !p || !x || !v || !L || nsteps < 0 || thermo_every < 1 || cap < 1)
    return ORC_EINVAL;
  orc_work w;
  memset(&w, 0, sizeof(w));
  w.cap = cap;
  w.atom_cell = (int*)malloc(sizeof(int) * (size_t)n);
  w.perm = (int*)malloc(sizeof(int) * (size_t)n);
  w.numneigh = (int*)malloc(sizeof(int) * (size_t)n);
  w.neigh = (int*)malloc(sizeof(int) * (size_t)n * (size_t)cap);
  w.xref = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  int st = ORC_OK;
  if (!w.atom_cell || !w.perm || !w.numneigh || !w.neigh || !w.xref || !f) {
    st = ORC_EINVAL;
    goto done;
  }
  const double dtfm = (0.5 * p->dt * p->ftm2v) / p->mass;
  const double trig = 0.5 * p->skin;
  const double trig2 = trig * trig;
  double pe = 0.0, vir[6];
  int nreb = 0, row = 0, maxc = 0;
  st = rebuild(p, n, x, L, &w);
  if (st) goto done;
  ++nreb;
  maxc = w.maxcount;
  if (rebuilt) rebuilt[0] = 1;
  st = forces(p, n, x, L, &w, f, &pe, vir);
  if (st) goto done;
  if (thermo) thermo_row(p, n, v, L, 0.0, pe, vir, nreb, maxc, thermo + 8 * row++);
  for (int s = 1; s <= nsteps; ++s) {
    for (int d = 0; d < 3; ++d)
      for (int64_t i = 0; i < n; ++i) {
        v[d * n + i] = v[d * n + i] + dtfm * f[d * n + i];
        x[d * n + i] = x[d * n + i] + p->dt * v[d * n + i];
      }
    double dmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double a = x[i] - w.xref[i], b = x[n + i] - w.xref[n + i], c = x[2 * n + i] - w.xref[2 * n + i];
      double d2 = (a * a + b * b) + c * c;
      if (d2 > dmax) dmax = d2;
    }
    int reb = dmax > trig2;
    if (rebuilt) rebuilt[s] = reb;
    if (reb) {
      st = rebuild(p, n, x, L, &w);
      if (st) goto done;
      ++nreb;
      if (w.maxcount > maxc) maxc = w.maxcount;
    }
    st = forces(p, n, x, L, &w, f, &pe, vir);
    if (st) goto done;
    for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] + dtfm * f[i];
    if (thermo && s % thermo_every == 0)
      thermo_row(p, n, v, L, (double)s, pe, vir, nreb, maxc, thermo + 8 * row++);
  }
  if (f_out) memcpy(f_out, f, sizeof(double) * 3 * (size_t)n);
done:
  free(w.atom_cell);
  free(w.perm);
  free(w.numneigh);
  free(w.neigh);
  free(w.xref);
  free(w.cell_start);
  free(f);
  return st;
}

/* ------------------------------------------------- Nose-Hoover chain NVT -- */

/* One thermostat half step (a time dt/2) of a Nose-Hoover chain of length M
   acting on kinetic energy ke2 = sum m v^2 (energy units), in the Trotter
   splitting of Martyna, Tuckerman and Klein: the chain velocities are updated
   from the end of the chain down to the first thermostat, the particle
   velocities are scaled by exp(-dt/2 veta_1), the chain positions advance,
   and the chain velocities are updated back up.  The forces on the
   thermostats are G_1 = (ke2 - Nf kT) / Q_1 and
   G_j = (Q_{j-1} veta_{j-1}^2 - kT) / Q_j; each velocity update is
   veta_j <- veta_j exp(-dt/8 veta_{j+1})^2 + dt/4 G_j exp(-dt/8 veta_{j+1}).
   Returns the velocity scale factor; *ke2 is updated to the scaled value. */
static double nhc_half(int M, const double* Q, double* eta, double* veta, double kT,
                       double nf, double dt, double* ke2) {
  const double dt2 = 0.5 * dt, dt4 = 0.25 * dt, dt8 = 0.125 * dt;
  double G;
  G = M > 1 ? (Q[M - 2] * veta[M - 2] * veta[M - 2] - kT) / Q[M - 1] : (*ke2 - nf * kT) / Q[0];
  veta[M - 1] = veta[M - 1] + dt4 * G;
  for (int j = M - 2; j >= 0; --j) {
    double aa = exp(-dt8 * veta[j + 1]);
    G = j == 0 ? (*ke2 - nf * kT) / Q[0] : (Q[j - 1] * veta[j - 1] * veta[j - 1] - kT) / Q[j];
    veta[j] = veta[j] * aa * aa + dt4 * G * aa;
  }
  double scale = exp(-dt2 * veta[0]);
  *ke2 = *ke2 * scale * scale;
  for (int j = 0; j < M; ++j) eta[j] = eta[j] + dt2 * veta[j];
  for (int j = 0; j < M - 1; ++j) {
    double aa = exp(-dt8 * veta[j + 1]);
    G = j == 0 ? (*ke2 - nf * kT) / Q[0] : (Q[j - 1] * veta[j - 1] * veta[j - 1] - kT) / Q[j];
    veta[j] = veta[j] * aa * aa + dt4 * G * aa;
  }
  G = M > 1 ? (Q[M - 2] * veta[M - 2] * veta[M - 2] - kT) / Q[M - 1] : (*ke2 - nf * kT) / Q[0];
  veta[M - 1] = veta[M - 1] + dt4 * G;
  return scale;
}

/* Energy of the chain: sum_j Q_j veta_j^2 / 2 + Nf kT eta_1 + kT sum_{j>1} eta_j;
   with it, pe + ke + this is conserved by the exact NVT flow. */
static double nhc_energy(int M, const double* Q, const double* eta, const double* veta,
                         double kT, double nf) {
  double e = 0.0;
  for (int j = 0; j < M; ++j) e += 0.5 * Q[j] * veta[j] * veta[j];
  e += nf * kT * eta[0];
  for (int j = 1; j < M; ++j) e += kT * eta[j];
  return e;
}

/* NVT run: per step a thermostat half step, the velocity-Verlet step (with the
   half-skin rebuild rule of orc_md_run), a thermostat half step.  Thermostat
   masses Q_1 = Nf kT t_damp^2, Q_j = kT t_damp^2 (j > 1), Nf = 3n - 3,
   kT = boltz t_target.  chain [in/out] holds eta[0..M) then veta[0..M).
   Thermo rows have nine columns: the eight of orc_md_run and
   pe + ke + the chain energy.  The kinetic energy entering the first half
   step of a step is the scaled value the previous half step left (the
   scaling multiplies it by scale^2), not a recount. */
int orc_md_run_nvt(const orc_params* p, int64_t n, double* x, double* v, const double* L,
                   int nsteps, int thermo_every, int cap, double t_target, double t_damp,
                   int M, double* chain, double* thermo, int* rebuilt, double* f_out) {
  if (n <= 1 || !p || !x || !v || !L || nsteps < 0 || thermo_every < 1 || cap < 1 || M < 1 ||
      M > 8 || !chain || !(t_target > 0.0) || !(t_damp > 0.0))
    return ORC_EINVAL;
  orc_work w;
  memset(&w, 0, sizeof(w));
  w.cap = cap;
  w.atom_cell = (int*)malloc(sizeof(int) * (size_t)n);
  w.perm = (int*)malloc(sizeof(int) * (size_t)n);
  w.numneigh = (int*)malloc(sizeof(int) * (size_t)n);
  w.neigh = (int*)malloc(sizeof(int) * (size_t)n * (size_t)cap);
  w.xref = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  int st = ORC_OK;
  if (!w.atom_cell || !w.perm || !w.numneigh || !w.neigh || !w.xref || !f) {
    st = ORC_EINVAL;
    goto done;
  }
  const double kick = (0.5 * p->dt * p->ftm2v) / p->mass;   /* dt/2 F/m factor */
  const double trig = 0.5 * p->skin;
  const double trig2 = trig * trig;
  const double kT = p->boltz * t_target;
  const double nf = 3.0 * (double)n - 3.0;
  double Q[8];
  Q[0] = nf * kT * t_damp * t_damp;
  for (int j = 1; j < M; ++j) Q[j] = kT * t_damp * t_damp;
  double* eta = chain;
  double* veta = chain + M;
  double pe = 0.0, vir[6];
  int nreb = 0, row = 0, maxc = 0;
  st = rebuild(p, n, x, L, &w);
  if (st) goto done;
  ++nreb;
  maxc = w.maxcount;
  if (rebuilt) rebuilt[0] = 1;
  st = forces(p, n, x, L, &w, f, &pe, vir);
  if (st) goto done;
  double ke2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double a = v[i], b = v[n + i], c = v[2 * n + i];
    ke2 += (a * a + b * b) + c * c;
  }
  ke2 = p->mass * p->mvv2e * ke2;
  if (thermo) {
    thermo_row(p, n, v, L, 0.0, pe, vir, nreb, maxc, thermo + 9 * row);
    thermo[9 * row + 8] = thermo[9 * row + 3] + nhc_energy(M, Q, eta, veta, kT, nf);
    ++row;
  }
  for (int s = 1; s <= nsteps; ++s) {
    double scale = nhc_half(M, Q, eta, veta, kT, nf, p->dt, &ke2);
    for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] * scale;
    for (int d = 0; d < 3; ++d)
      for (int64_t i = 0; i < n; ++i) {
        v[d * n + i] = v[d * n + i] + kick * f[d * n + i];
        x[d * n + i] = x[d * n + i] + p->dt * v[d * n + i];
      }
    double dmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double a = x[i] - w.xref[i], b = x[n + i] - w.xref[n + i], c = x[2 * n + i] - w.xref[2 * n + i];
      double d2 = (a * a + b * b) + c * c;
      if (d2 > dmax) dmax = d2;
    }
    const int rebuild_now = dmax > trig2;
    if (rebuilt) rebuilt[s] = rebuild_now;
    if (rebuild_now) {
      st = rebuild(p, n, x, L, &w);
      if (st) goto done;
      ++nreb;
      if (w.maxcount > maxc) maxc = w.maxcount;
    }
    st = forces(p, n, x, L, &w, f, &pe, vir);
    if (st) goto done;
    for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] + kick * f[i];
    ke2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double a = v[i], b = v[n + i], c = v[2 * n + i];
      ke2 += (a * a + b * b) + c * c;
    }
    ke2 = p->mass * p->mvv2e * ke2;
    scale = nhc_half(M, Q, eta, veta, kT, nf, p->dt, &ke2);
    for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] * scale;
    if (thermo && s % thermo_every == 0) {
      thermo_row(p, n, v, L, (double)s, pe, vir, nreb, maxc, thermo + 9 * row);
      thermo[9 * row + 8] = thermo[9 * row + 3] + nhc_energy(M, Q, eta, veta, kT, nf);
      ++row;
    }
  }
  if (f_out) memcpy(f_out, f, sizeof(double) * 3 * (size_t)n);
done:
  free(w.atom_cell);
  free(w.perm);
  free(w.numneigh);
  free(w.neigh);
  free(w.xref);
  free(w.cell_start);
  free(f);
  return st;
}

/* ------------------------------------------- isotropic NPT (MTK + chains) -- */

/* sinh(x) / x, by its Taylor series where x is small (the series to x^8 is
   exact to rounding for |x| < 1e-3). */
static double sinhc(double x) {
  if (fabs(x) < 1e-3) {
    const double x2 = x * x;
    return 1.0 + x2 / 6.0 * (1.0 + x2 / 20.0 * (1.0 + x2 / 42.0 * (1.0 + x2 / 72.0)));
  }
  return sinh(x) / x;
}

/* Force on the barostat momentum: G_eps = alpha ke2 + tr W - 3 V P_ext, i.e.
   3V (P_int - P_ext) plus the kinetic term's share (3 / Nf) ke2 that the
   equations of motion of Martyna, Tobias and Klein add. */
static double npt_geps(double alpha, double ke2, const double* vir, double vol,
                       double p_target) {
  return alpha * ke2 + (vir[0] + vir[1] + vir[2]) - 3.0 * vol * p_target;
}

/* NPT run: isotropic barostat in the equations of Martyna, Tobias and Klein
   (box edges L_d = L0_d exp(eps), eps with momentum p_eps and mass W) with a
   Nose-Hoover chain on the particles and another on the barostat, integrated
   in the time-reversible splitting of Tuckerman et al.  Per step:
     barostat chain half step (acts on p_eps; G_1 = (p_eps^2 / W - kT) / Q'_1),
     particle chain half step (scales v, as orc_md_run_nvt),
     p_eps += dt/2 G_eps,  G_eps = alpha ke2 + tr W - 3 V P_ext,  alpha = 1 + 3 / Nf,
     v <- v a + dtfm f b, a = exp(-alpha v_e dt/2), b = exp(-alpha v_e dt/4) sinhc(alpha v_e dt/4),
     x <- x c + e v,      c = exp(v_e dt),         e = dt exp(v_e dt/2) sinhc(v_e dt/2),
     L <- L c,   (v_e = p_eps / W)
     rebuild if max_i |x_i - s x_ref_i|^2 > (skin/2 - (1 - s) rl/2)^2, s = L / L_ref (or if
       that bound is negative), wrapping and re-gridding in the current box,
     forces and virial at the new positions and box,
     v <- v a + dtfm f b,  ke2 = sum m v^2 (recount),
     p_eps += dt/2 G_eps,
     particle chain half step, barostat chain half step.
   The rebuild bound keeps every pair that may come within rc in the list: a
   pair outside r_l at the build is at least s r_l - 2 max |x - s x_ref| apart.
   Masses: W = (Nf + 3) kT p_damp^2, Q'_j = kT p_damp^2, particle chain as in
   orc_md_run_nvt.  Conserved: pe + ke + particle chain energy + p_eps^2 / (2W)
   + P_ext V + barostat chain energy (sum_j Q'_j w_j^2 / 2 + kT sum_j xi_j).
   L [in/out] is the box; chain [in/out] holds eta[M], veta[M] (particles),
   xi[M], w[M] (barostat), p_eps.  Thermo rows have ten columns: the eight of
   orc_md_run (P with the current volume), the conserved energy, the volume.
   With p_damp huge (W beyond any G_eps) v_e rounds to a factor of exactly 1
   everywhere and the run is orc_md_run_nvt's, operation for operation. */
int orc_md_run_npt(const orc_params* p, int64_t n, double* x, double* v, double* L,
                   int nsteps, int thermo_every, int cap, double t_target, double t_damp,
                   int M, double p_target, double p_damp, double* chain, double* thermo,
                   int* rebuilt, double* f_out) {
  if (n <= 1 || !p || !x || !v || !L || nsteps < 0 || thermo_every < 1 || cap < 1 || M < 1 ||
      M > 8 || !chain || !(t_target > 0.0) || !(t_damp > 0.0) || !(p_damp > 0.0) ||
      !isfinite(p_target))
    return ORC_EINVAL;
  orc_work w;
  memset(&w, 0, sizeof(w));
  w.cap = cap;
  w.atom_cell = (int*)malloc(sizeof(int) * (size_t)n);
  w.perm = (int*)malloc(sizeof(int) * (size_t)n);
  w.numneigh = (int*)malloc(sizeof(int) * (size_t)n);
  w.neigh = (int*)malloc(sizeof(int) * (size_t)n * (size_t)cap);
  w.xref = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  int st = ORC_OK;
  if (!w.atom_cell || !w.perm || !w.numneigh || !w.neigh || !w.xref || !f) {
    st = ORC_EINVAL;
    goto done;
  }
  {
    const double kick = (0.5 * p->dt * p->ftm2v) / p->mass;
    const double rl = p->rc + p->skin;
    const double kT = p->boltz * t_target;
    const double nf = 3.0 * (double)n - 3.0;
    const double alpha = 1.0 + 3.0 / nf;
    double Q[8], Qb[8];
    Q[0] = nf * kT * t_damp * t_damp;
    for (int j = 1; j < M; ++j) Q[j] = kT * t_damp * t_damp;
    for (int j = 0; j < M; ++j) Qb[j] = kT * p_damp * p_damp;
    const double W = (nf + 3.0) * kT * p_damp * p_damp;
    double* eta = chain;
    double* veta = chain + M;
    double* xi = chain + 2 * M;
    double* vxi = chain + 3 * M;
    double* peps = chain + 4 * M;
    double Lref[3] = {L[0], L[1], L[2]};
    double pe = 0.0, vir[6];
    int nreb = 0, row = 0, maxc = 0;
    st = rebuild(p, n, x, L, &w);
    if (st) goto done;
    ++nreb;
    maxc = w.maxcount;
    if (rebuilt) rebuilt[0] = 1;
    st = forces(p, n, x, L, &w, f, &pe, vir);
    if (st) goto done;
    double ke2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double a = v[i], b = v[n + i], c = v[2 * n + i];
      ke2 += (a * a + b * b) + c * c;
    }
    ke2 = p->mass * p->mvv2e * ke2;
    /* conserved energy of the extended system (beyond pe + ke) */
#define NPT_EXTRA()                                                                    \
  (nhc_energy(M, Q, eta, veta, kT, nf) + nhc_energy(M, Qb, xi, vxi, kT, 1.0) +        \
   0.5 * *peps * *peps / W + p_target * (L[0] * L[1] * L[2]))
    if (thermo) {
      thermo_row(p, n, v, L, 0.0, pe, vir, nreb, maxc, thermo + 10 * row);
      thermo[10 * row + 8] = thermo[10 * row + 3] + NPT_EXTRA();
      thermo[10 * row + 9] = L[0] * L[1] * L[2];
      ++row;
    }
    for (int s = 1; s <= nsteps; ++s) {
      /* barostat chain and particle chain half steps */
      double kb2 = *peps * *peps / W;
      *peps = *peps * nhc_half(M, Qb, xi, vxi, kT, 1.0, p->dt, &kb2);
      double scale = nhc_half(M, Q, eta, veta, kT, nf, p->dt, &ke2);
      for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] * scale;
      double vol = L[0] * L[1] * L[2];
      *peps = *peps + 0.5 * p->dt * npt_geps(alpha, ke2, vir, vol, p_target);
      const double ve = *peps / W;
      const double ka = exp(-alpha * ve * 0.5 * p->dt);
      const double kb = exp(-alpha * ve * 0.25 * p->dt) * sinhc(alpha * ve * 0.25 * p->dt);
      const double dc = exp(ve * p->dt);
      const double de = p->dt * exp(ve * 0.5 * p->dt) * sinhc(ve * 0.5 * p->dt);
      for (int d = 0; d < 3; ++d)
        for (int64_t i = 0; i < n; ++i) {
          v[d * n + i] = v[d * n + i] * ka + kick * f[d * n + i] * kb;
          x[d * n + i] = x[d * n + i] * dc + de * v[d * n + i];
        }
      for (int d = 0; d < 3; ++d) L[d] = L[d] * dc;
      const double sb = L[0] / Lref[0];
      const double thr = 0.5 * p->skin - 0.5 * (1.0 - sb) * rl;
      double dmax = 0.0;
      for (int64_t i = 0; i < n; ++i) {
        double a = x[i] - sb * w.xref[i], b = x[n + i] - sb * w.xref[n + i],
               c = x[2 * n + i] - sb * w.xref[2 * n + i];
        double d2 = (a * a + b * b) + c * c;
        if (d2 > dmax) dmax = d2;
      }
      const int rebuild_now = thr < 0.0 || dmax > thr * thr;
      if (rebuilt) rebuilt[s] = rebuild_now;
      if (rebuild_now) {
        st = rebuild(p, n, x, L, &w);
        if (st) goto done;
        for (int d = 0; d < 3; ++d) Lref[d] = L[d];
        ++nreb;
        if (w.maxcount > maxc) maxc = w.maxcount;
      }
      st = forces(p, n, x, L, &w, f, &pe, vir);
      if (st) goto done;
      for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] * ka + kick * f[i] * kb;
      ke2 = 0.0;
      for (int64_t i = 0; i < n; ++i) {
        double a = v[i], b = v[n + i], c = v[2 * n + i];
        ke2 += (a * a + b * b) + c * c;
      }
      ke2 = p->mass * p->mvv2e * ke2;
      vol = L[0] * L[1] * L[2];
      *peps = *peps + 0.5 * p->dt * npt_geps(alpha, ke2, vir, vol, p_target);
      scale = nhc_half(M, Q, eta, veta, kT, nf, p->dt, &ke2);
      for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] * scale;
      kb2 = *peps * *peps / W;
      *peps = *peps * nhc_half(M, Qb, xi, vxi, kT, 1.0, p->dt, &kb2);
      if (thermo && s % thermo_every == 0) {
        thermo_row(p, n, v, L, (double)s, pe, vir, nreb, maxc, thermo + 10 * row);
        thermo[10 * row + 8] = thermo[10 * row + 3] + NPT_EXTRA();
        thermo[10 * row + 9] = L[0] * L[1] * L[2];
        ++row;
      }
    }
#undef NPT_EXTRA
  }
  if (f_out) memcpy(f_out, f, sizeof(double) * 3 * (size_t)n);
done:
  free(w.atom_cell);
  free(w.perm);
  free(w.numneigh);
  free(w.neigh);
  free(w.xref);
  free(w.cell_start);
  free(f);
  return st;
}
