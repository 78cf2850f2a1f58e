/*
 * md.h -- C ABI of the MI355X short-range molecular-dynamics hot path.
 *
 * The operation is the per-atom pair-force evaluation over a full Verlet
 * neighbour list described in the paper's section "Neighbor list approach"
 * (the TpA and BpA listings: load atom i, loop over numneigh[i] entries of
 * neighbors[i][.], accumulate the pair force, store f[i]), together with what
 * feeds it on the GPU: cell binning of the periodic box (section "Cell list
 * approach"), the list build with a skin and a half-skin rebuild trigger, and
 * NVE velocity-Verlet integration ("NVE integrator", section "Design
 * objectives, features and usage"); precision modes follow the same section
 * (double, and mixed: pair forces in single precision, integration in double).
 * Kernel choice follows the TpA / BpA discussion and the built-in
 * mini-benchmark of section "Neighbor list approach".  Beyond that path the
 * library has the Buckingham + cut Coulomb potential of the silicate system
 * (Appendix A), the force adjoints (LJ and Sutton-Chen) for force matching,
 * NVT integration with a Nose-Hoover chain, isotropic NPT integration, half
 * lists with Newton's third law for forces, and LDS-staged neighbour tiles.
 *
 * Conventions
 *  - Every pointer is a DEVICE pointer unless marked [host].  The caller owns
 *    every buffer; no call allocates or frees device memory, and no call
 *    synchronises except md_step, md_step_nvt and md_step_npt (once, at their end),
 *    md_nlist_status and md_autoselect.  Work is enqueued on `stream` (a hipStream_t; NULL is the
 *    default stream).
 *  - Per-atom vectors are SoA FP64 [3][n]: n x values, then n y, then n z.
 *  - n (atoms) is at most MD_MAX_ATOMS; larger n returns MD_ERR_INVALID_ARG.
 *  - The box is orthorhombic, periodic, with origin 0 and edges L[0..2].
 *  - Errors are returned; nothing is thrown across the ABI.  Host-detectable
 *    errors return before anything is enqueued.  Device-detected errors
 *    (neighbour overflow, non-finite values) are recorded in nl->status and
 *    reported by md_step / md_nlist_status.
 *  - `ws` is a caller-owned device workspace of at least
 *    md_workspace_bytes(...) bytes, 256-byte aligned.  Calls on one workspace
 *    must not overlap in time (use one stream, or one workspace per stream).
 */
#ifndef MD_MI355X_H
#define MD_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest atom count: the force kernels address positions with 32-bit byte
   offsets into 32-byte records. */
#define MD_MAX_ATOMS 134217727

typedef enum {
  MD_OK = 0,
  MD_ERR_INVALID_ARG = 1,    /* null pointer, n <= 0, bad enum, capacity < 1, ... */
  MD_ERR_BOX_TOO_SMALL = 2,  /* some L_d <= 2 (rc + skin): minimum image not unique */
  MD_ERR_NLIST_OVERFLOW = 3, /* an atom has more neighbours than nl->capacity */
  MD_ERR_NONFINITE = 4,      /* a position or force became NaN / Inf */
  MD_ERR_UNSUPPORTED = 5,    /* valid request the library does not implement */
  MD_ERR_HIP = 6,            /* a HIP runtime call failed */
  MD_ERR_WORKSPACE = 7,      /* ws is NULL or smaller than md_workspace_bytes */
  MD_ERR_UNSTABLE = 8,       /* md_step: an atom moved more than a cell edge between builds */
  MD_ERR_SCRATCH = 9,        /* md_compute_forces_noalloc: the call needs more than its fixed scratch */
  MD_STATUS_INT_MIN_ = -2147483647 - 1,   /* range markers: see md_precision */
  MD_STATUS_INT_MAX_ = 2147483647
} md_status;

/* The enums taken as arguments span the whole int range (the two _INT_
   markers), so every value a caller passes, valid or not, is a value of the
   type that the argument checks can see and reject with MD_ERR_INVALID_ARG
   (in C++ an enum holds only the values its enumerators' bit width covers). */
typedef enum {
  MD_FP64 = 0,
  MD_MIXED = 1,
  MD_PRECISION_INT_MIN_ = -2147483647 - 1,
  MD_PRECISION_INT_MAX_ = 2147483647
} md_precision;

/* Force kernels.  The paper's thread-per-atom (TpA) and block-per-atom (BpA)
   designs are the two ends of one family: K lanes of a 64-wide wavefront share
   an atom and split its neighbour list, K a power of two in [1, 64].
   MD_KERNEL_TPA is K = 1 (one lane per atom), MD_KERNEL_WPA is K = 64 (one
   wavefront per atom, reduced with cross-lane operations); any power of two in
   between may be passed as an md_kernel value.  MD_KERNEL_AUTO picks K with a
   mini-benchmark (md_autoselect). */
typedef enum {
  MD_KERNEL_AUTO = 0,
  MD_KERNEL_TPA = 1,
  MD_KERNEL_WPA = 64,
  MD_KERNEL_INT_MIN_ = -2147483647 - 1,   /* range markers: see md_precision */
  MD_KERNEL_INT_MAX_ = 2147483647
} md_kernel;
enum { MD_EFLAG = 1, MD_VFLAG = 2 };
enum { MD_POT_LJ = 0, MD_POT_SC = 1, MD_POT_BUCK = 2 };

/* Neighbour-list layout K (lanes per atom, as above): groups of G = 64 / K
   consecutive atoms share rows of 64 ints, and entry m of atom i lives at
     neigh[((i / G) * ceil(capacity / K) + m / K) * 64 + (i % G) * K + m % K],
   so each row a wavefront reads is one contiguous 256-byte block.  K = 1:
   entry m of atom i at ((i / 64) * capacity + m) * 64 + i % 64; K = 64: the
   entries of atom i are consecutive.  A force kernel reads only a list of its
   own K.  md_nlist_ints() gives the buffer size that fits every K. */
enum { MD_LAYOUT_TPA = 1, MD_LAYOUT_WPA = 64 };

/* LDS-tiled layouts (md_step / md_step_nvt only).  Layout MD_LAYOUT_TILE | K,
   K in {1, 2, 4, 8}, is the layout-K list above in neigh plus, in nl->tile, a
   copy whose entries are 16-bit indices into a window of atoms that the force
   kernel stages in LDS (the paper's shared-memory staging of neighbour
   positions, section "Cell list approach", applied to the neighbour-list
   kernels): atoms in cell order are grouped into runs of up to R consecutive
   cells along x, and a run's window is the 3 x 3 rows of cells around it, from
   one cell before the run to one after.  The same value as an md_kernel asks
   md_step for that kernel; MD_KERNEL_AUTO also tries them.  Every other call
   reads the neigh part of such a list with the K-lane kernel.  Needs at least
   4 cells along x and 3 along y and z, and a tile buffer of
   md_nlist_tile_entries() entries (nl->tile_entries); not used in NPT runs,
   whose cell grid differs from the box's. */
enum { MD_LAYOUT_TILE = 256 };

/* nl->status words (device int[MD_STATUS_WORDS]). */
enum {
  MD_ST_ERRORS = 0,    /* bit 0: list overflow, bit 1: non-finite value */
  MD_ST_MAXNEIGH = 1,  /* largest neighbour count of the last build (the required capacity) */
  MD_ST_BUILDS = 2,    /* number of list builds so far (md_step increments it) */
  MD_ST_REBUILD = 3,   /* internal: rebuild requested by the displacement check */
  MD_ST_REBUILD2 = 4,  /* internal: the same for alternate steps of md_step */
  MD_STATUS_WORDS = 8
};

typedef struct { double L[3]; } md_box; /* [host] */

/* [host] Potential.  LJ: phi(r) = 4 eps ((sigma/r)^12 - (sigma/r)^6) for r < rc
   (lj/cut, the paper's Appendix A "LJ"); lj_shift != 0 subtracts phi(rc) from
   the reported energy (forces unchanged).  SC (Sutton-Chen, standing in for the
   paper's EAM benchmark): E = eps sum_i [1/2 sum_j (a/r_ij)^n - c sqrt(rho_i)],
   rho_i = sum_j (a/r_ij)^m, both sums truncated at rc.  BUCK (Buckingham + cut
   Coulomb, the paper's Appendix A "Silicate (cutoff)" system):
     phi_ab(r) = A_ab exp(-r / rho_ab) - C_ab / r^6 + qqr2e q_a q_b / r,  r < rc,
   a, b the species of the two atoms (0..3), tables indexed a * 4 + b and
   symmetric; no shift at rc.  `type` [device, int per atom] gives the
   species in the order of the positions a call works on: md_compute_forces
   and md_autoselect read it in the order of their x; md_step reads it in the
   state's order and permutes it along with the atoms (like st->id).  Pairs
   with A_ab = 0 ignore rho_ab. */
typedef struct {
  int kind;          /* MD_POT_LJ, MD_POT_SC or MD_POT_BUCK */
  double rc;         /* force cutoff */
  double lj_eps, lj_sigma;
  int lj_shift;
  double sc_eps, sc_a, sc_c;
  int sc_n, sc_m;
  double buck_A[16], buck_rho[16], buck_C[16];
  double q[4];       /* charge per species */
  double qqr2e;      /* Coulomb constant in the run's units */
  int* type;         /* BUCK: species per atom (see above); unused otherwise */
} md_potential;

/* Cell grid: nc_d = floor(L_d / rl) cells per dimension (edge >= rl), linear
   cell index cx + nc0 * (cy + nc1 * cz). */
typedef struct {
  int nc[3];           /* [out] set by md_bin_cells */
  int64_t ncell_cap;   /* capacity: cell_start holds ncell_cap + 1 ints */
  int* cell_start;     /* [ncell+1] first sorted slot of each cell */
  int* atom_cell;      /* [n] cell of each atom (input order) */
  int* perm;           /* [n] stable sort: atom indices cell by cell, increasing inside a cell */
} md_cells;

/* Full Verlet list: every ordered pair i != j with r_ij^2 < rl^2 appears in
   row i, rl = rc + skin.  With half = 1 (Newton's third law, after the
   paper's section "Cell list approach": each pair computed once), row i holds
   only the partners j > i, in the order the full row would list them;
   capacity must still hold the full row while it is built, and
   status[MD_ST_MAXNEIGH] reports the full count.  Half lists serve
   md_build_neighbors and md_compute_forces (LJ); md_step, md_step_nvt,
   md_autoselect and md_force_vjp return MD_ERR_UNSUPPORTED for them. */
typedef struct {
  int capacity;        /* entries per atom the neigh buffer holds */
  int layout;          /* lanes per atom K (MD_LAYOUT_TPA = 1 ... MD_LAYOUT_WPA = 64) */
  double rl;           /* [out] list radius of the last build */
  int* neigh;          /* see layouts above */
  int* numneigh;       /* [n] */
  double* x_ref;       /* [3][n] positions at the last build (rebuild trigger reference) */
  int* status;         /* [MD_STATUS_WORDS], zero it once before first use */
  int half;            /* 0: full list; 1: half list (see above) */
  unsigned short* tile;  /* nullable: 16-bit entries for the tiled layouts
                            (MD_LAYOUT_TILE | K); written by md_step's builds */
  size_t tile_entries;   /* entries tile holds; the tiled layouts are used only when this
                            covers md_nlist_tile_entries() of the run's box and grid */
} md_nlist;

/* Dynamic state advanced by md_step.  Units: ftm2v converts force/mass * time
   to velocity, mvv2e converts m v^2 to energy, boltz is k_B (all 1 in LJ
   units). */
typedef struct {
  int64_t n;
  double* x;           /* [3][n] */
  double* v;           /* [3][n] */
  double* f;           /* [3][n] */
  int* id;             /* [n] caller's atom ids, permuted along with the atoms */
  double mass;
  double ftm2v, mvv2e, boltz;
} md_state;

/* Workspace bytes needed by any call for n atoms in this box with list radius
   rl (covers the largest of all calls).  Returns 0 on invalid input. */
size_t md_workspace_bytes(int64_t n, const md_box* box, double rl);

/* Ints the neigh buffer must hold for n atoms and this capacity, in any
   layout K (md_step and md_autoselect may switch layouts).  0 on bad input. */
size_t md_nlist_ints(int64_t n, int capacity);

/* 16-bit entries nl->tile must hold for the tiled layouts of n atoms with
   this capacity in this box at list radius rl (every K they take).  0 when
   the tiled kernels do not apply to this system (too few cells, or windows
   too large for LDS) or on bad input. */
size_t md_nlist_tile_entries(int64_t n, int capacity, const md_box* box, double rl);

/* Number of thermo rows md_step writes. */
int md_thermo_rows(int nsteps, int thermo_every, int setup);

/* Paper: section "Cell list approach" (the box cut into cells at least a
   cutoff wide, each atom binned to one; here the cells serve the list build).
   Cell binning (wrap + bin + stable counting sort).  Wraps x in place into
   [0, L) (x - L floor(x / L), an L result mapped to 0), bins each atom to
   clamp((int)(x_d nc_d / L_d), 0, nc_d - 1), and writes atom_cell,
   cell_start and perm.  Cells per dimension follow from box and rl; the call
   fails with MD_ERR_INVALID_ARG if their product exceeds cells->ncell_cap. */
md_status md_bin_cells(double* x, int64_t n, const md_box* box, double rl,
                       md_cells* cells, void* ws, size_t ws_bytes, void* stream);

/* Reorder atoms into cell order (slot k takes atom cells->perm[k]): x, v, id
   and, when not NULL, f and x_ref are gathered through perm.  Makes neighbour
   gathers spatially local (the paper assumes spatially ordered atoms for its
   cached neighbour reads).  Per-atom data outside md_state (Buckingham
   species) is the caller's to gather through cells->perm. */
md_status md_sort_atoms(md_state* st, const md_cells* cells, double* x_ref, void* ws,
                        size_t ws_bytes, void* stream);

/* Paper: section "Neighbor list approach" (the numneigh[i] / neighbors[i][jj]
   arrays its TpA and BpA listings read, built from the cells of "Cell list
   approach" with a skin added to the cutoff).
   Full neighbour list at rl = rc + skin from binned positions (x as wrapped by
   md_bin_cells, in any atom order: cell members are taken through perm).
   Distances use the minimum image d - L rint(d / L) and
   r^2 = (dx dx + dy dy) + dz dz without fused multiply-add, so the pair set is
   exactly that of the FP64 definition.  Sets nl->rl, copies x to nl->x_ref,
   records the largest count in status[MD_ST_MAXNEIGH] and sets the overflow
   bit if it exceeds nl->capacity (entries past capacity are dropped). */
md_status md_build_neighbors(const double* x, int64_t n, const md_box* box,
                             const md_cells* cells, double rc, double skin, md_nlist* nl,
                             void* stream);

/* Paper: section "Neighbor list approach" (the TpA and BpA listings: per atom,
   sum the pair force over its listed neighbours inside the cutoff, store f[i]);
   lj/cut and the EAM and silicate systems of Appendix A; precision modes of
   "Design objectives, features and usage".
   Forces (and, on flags, energy / virial) from a list.  f [3][n] is
   overwritten.  ev, when flags != 0, receives 7 doubles: energy, then virial
   xx yy zz xy xz yz, W = 1/2 sum_i sum_j d_ij (x) F_ij.  Only pairs with
   r^2 < rc^2 (FP64, as above) contribute, in either precision.  MD_MIXED
   forms d and r^2 in FP64, evaluates the scalar pair function in FP32, and
   accumulates forces, energy and virial in FP64.  k = AUTO uses the kernel
   matching nl->layout; TPA / WPA must match the layout (else
   MD_ERR_INVALID_ARG).  From a half list (LJ only) each pair is evaluated
   once and its force added to both atoms with FP64 atomic adds, so the
   summation order (and the last bits) can change from call to call; the
   whole pair energy and virial go to the atom with the smaller index. */
md_status md_compute_forces(const md_potential* p, const double* x, int64_t n,
                            const md_box* box, const md_nlist* nl, md_precision prec,
                            md_kernel k, int flags, double* f, double* ev, void* ws,
                            size_t ws_bytes, void* stream);

/* Paper: "Design objectives, features and usage" (the NVE integrator, with
   integration in double precision in the mixed mode) around the force
   evaluation of "Neighbor list approach"; the whole step stays on the GPU
   (the GPU-resident workflow of the same section).
   nsteps of velocity-Verlet NVE (dtfm = (0.5 dt ftm2v) / mass):
     v += dtfm f; x += dt v;
     rebuild (wrap, bin, sort, list) if max_i |x_i - x_ref_i|^2 > (skin/2)^2;
     f = forces(x); v += dtfm f.
   With setup != 0 the state is first wrapped, binned, sorted and listed and
   forces are computed (a thermo row for that state is written first).  With
   setup == 0, st, cells and nl must be as a previous md_step on the same
   system left them (atoms in cell order, list and forces current); rebuilds
   then re-sort by gathering each cell's atoms from the previous cell ranges,
   and MD_ERR_UNSTABLE reports an atom that moved more than a cell edge (the
   state is then unusable; this status takes precedence over every other).
   thermo (device, md_thermo_rows(...) x 8 doubles, or NULL for none): for
   each step s with s % thermo_every == 0: s, pe, ke, pe + ke,
   T = 2 ke / ((3n - 3) kB), P = (2 ke + tr W) / (3 V), builds so far,
   largest neighbour count.
   Atoms are kept in cell order; st->id tracks them.  k = AUTO runs the
   TpA / WPA mini-benchmark at setup (see md_autoselect).  Synchronises the
   stream once at the end and returns the device status (overflow /
   non-finite); after an overflow the state is not valid: grow the list and
   restart from a saved state. */
md_status md_step(md_state* st, const md_potential* p, const md_box* box, md_cells* cells,
                  md_nlist* nl, md_precision prec, md_kernel k, double skin, double dt,
                  int nsteps, int thermo_every, int setup, double* thermo, void* ws,
                  size_t ws_bytes, void* stream);

/* Nose-Hoover chain thermostat for md_step_nvt (the NVT integrator among the
   integrators listed in the paper's "Design objectives"), in the
   time-reversible splitting of Martyna, Tuckerman and Klein.  Masses
   Q_1 = Nf kB T t_damp^2, Q_j = kB T t_damp^2 (j > 1), Nf = 3n - 3.
   state [device, MD_NHC_STATE doubles, caller-owned, zero for a fresh
   thermostat]: eta[0..MD_NHC_MAX), eta_dot[0..MD_NHC_MAX), then the chain
   energy sum_j Q_j eta_dot_j^2 / 2 + Nf kB T eta_1 + kB T sum_{j>1} eta_j at the
   last step, then two words of working storage.  md_step_nvt updates it in
   place; pass it unchanged to the next call to continue the run. */
enum { MD_NHC_MAX = 8, MD_NHC_STATE = 2 * MD_NHC_MAX + 4 };
typedef struct {
  double t_target;   /* target temperature, the run's units */
  double t_damp;     /* thermostat period, time units */
  int chain;         /* chain length, 1..MD_NHC_MAX */
  double* state;     /* [device] MD_NHC_STATE doubles (see above) */
} md_nhc;

/* md_step under the Nose-Hoover chain thermostat nhc: each step is a
   thermostat half step (velocities scaled by exp(-dt/2 eta_dot_1)), the
   velocity-Verlet step of md_step (same kick, drift, rebuild rule and
   forces), and a thermostat half step.  The kinetic energy entering a step's
   first half step is the one the previous half step left (scaled by the
   square of its factor); at the start of a call it is summed from v.  thermo
   rows have nine doubles: the eight of md_step (pe, ke and T after the
   step's thermostat half step) and pe + ke + chain energy, which the exact
   NVT flow conserves.  Every other argument, status and rule as md_step. */
md_status md_step_nvt(md_state* st, const md_potential* p, const md_box* box, md_cells* cells,
                      md_nlist* nl, md_precision prec, md_kernel k, double skin, double dt,
                      const md_nhc* nhc, int nsteps, int thermo_every, int setup,
                      double* thermo, void* ws, size_t ws_bytes, void* stream);

/* Fixed device scratch of md_compute_forces_noalloc, per GPU (64 MiB). */
#define MD_NOALLOC_SCRATCH_BYTES 67108864

/* Scratch bytes md_compute_forces_noalloc needs for n atoms of potential kind
   `kind` (MD_POT_*) with these flags: 32 per atom for the packed positions,
   8 more for Sutton-Chen, 56 more and 32 KiB with flags != 0, each part
   rounded up to 256 bytes.  0 for n out of range.  Host only. */
size_t md_compute_forces_noalloc_bytes(int64_t n, int kind, int flags);

/* md_compute_forces for callers that cannot allocate device memory or pass a
   workspace (code under HIP graph capture, serving loops, harnesses that
   forbid allocation).  Same arguments, results, kernels and rules as
   md_compute_forces, without ws: its scratch (packed positions, Sutton-Chen
   densities, per-atom energy / virial and partial sums) lives in one fixed
   array of MD_NOALLOC_SCRATCH_BYTES per GPU, held by the library from its
   load until the process ends.  The caller still owns x, f, ev and the list.
   Calls that need more than MD_NOALLOC_SCRATCH_BYTES
   (md_compute_forces_noalloc_bytes) return MD_ERR_SCRATCH before anything
   is enqueued; the limit is about 2 million atoms for forces alone, 700,000
   with energy / virial.  The call allocates nothing: no hipMalloc, no
   workspace, no library call that allocates.  Every call on one GPU uses
   that GPU's one array, and nothing in it is kept from call to call: calls
   that overlap in time on one GPU (several streams or host threads) race on
   it and must be serialised by the caller.  The first call on a device looks
   the array's address up there (not an allocation). */
md_status md_compute_forces_noalloc(const md_potential* p, const double* x, int64_t n,
                                    const md_box* box, const md_nlist* nl, md_precision prec,
                                    md_kernel k, int flags, double* f, double* ev,
                                    void* stream);

/* Isotropic barostat for md_step_npt (the NPT integrator among the
   integrators listed in the paper's "Design objectives"): the equations of
   Martyna, Tobias and Klein, box edges L_d scaled together, with a
   Nose-Hoover chain on the particles (as md_nhc) and one on the barostat, in
   the time-reversible splitting of Tuckerman et al.  Barostat mass
   W = (Nf + 3) kB T p_damp^2, barostat chain masses kB T p_damp^2, Nf = 3n - 3.
   state [device, MD_NPT_STATE doubles, caller-owned, zero for a fresh
   barostat and thermostat]: particle chain eta[8], eta_dot[8], barostat chain
   xi[8], xi_dot[8], the barostat momentum, the box edges, then working
   storage; md_step_npt updates it in place (pass it unchanged to continue a
   run). */
enum { MD_NPT_STATE = 64 };
typedef struct {
  double t_target;   /* target temperature, the run's units */
  double t_damp;     /* thermostat period */
  int chain;         /* chain length of both thermostats, 1..MD_NHC_MAX */
  double p_target;   /* target pressure, energy / volume units */
  double p_damp;     /* barostat period */
  double* state;     /* [device] MD_NPT_STATE doubles (see above) */
} md_npt;

/* md_step under the barostat npt: each step is a barostat-chain and
   particle-chain half step, a half step of the barostat momentum
   (G = (1 + 3/Nf) sum m v^2 + tr W - 3 V P_target), the kick
   v <- v exp(-(1 + 3/Nf) v_e dt/2) + (dt/2) F/m exp(-(1 + 3/Nf) v_e dt/4) sinhc,
   the drift x <- x exp(v_e dt) + dt v exp(v_e dt/2) sinhc with the box scaled
   by exp(v_e dt) (v_e = p_eps / W, sinhc(y) = sinh(y)/y at the half
   arguments), the rebuild check, forces, the closing kick, the closing half
   steps in reverse order.  Lists stay valid under the box scale s since the
   last build: a rebuild happens when max |x - s x_ref| exceeds
   skin/2 - (1 - s) rl/2.  The box lives in npt->state during the call; box
   [host] gives it at setup and receives the final box.  The cell grid is
   fixed at setup from the box shrunk by 5 %; if an edge later falls below
   nc rl the run returns MD_ERR_BOX_TOO_SMALL (the state is then unusable: run
   setup again from a saved state).  thermo rows have ten doubles: the eight
   of md_step (P with the current volume), pe + ke plus the extended energy
   (both chains, p_eps^2 / 2W, P_target V), which the exact flow conserves,
   and the volume.  Every other argument, status and rule as md_step. */
md_status md_step_npt(md_state* st, const md_potential* p, md_box* box, md_cells* cells,
                      md_nlist* nl, md_precision prec, md_kernel k, double skin, double dt,
                      const md_npt* npt, int nsteps, int thermo_every, int setup,
                      double* thermo, void* ws, size_t ws_bytes, void* stream);

/* Not a passage of the paper: an extension of this library beyond the
   paper's method (differentiating the paper's force evaluation for force
   matching), with the same pair set and list.
   Vector-Jacobian product of the forces for L = sum_i u_i . F_i:
   gx = (dF/dx)^T u = -H u, with u, gx [device, 3][n]; gparam [device, may be
   NULL] receives the parameter gradients of L.  LJ: dL/deps, dL/dsigma
   (2 doubles).  SC: dL/deps, dL/da, dL/dc (3 doubles); its Hessian includes
   the many-body embedding term, through a density pass, a pass for
   dL/drho_i and the position pass.  Pair set: listed pairs with r^2 < rc^2
   (rc is not scaled by sigma or a).  Buckingham returns MD_ERR_UNSUPPORTED.
   Uses the workspace's per-atom columns (not preserved). */
md_status md_force_vjp(const md_potential* p, const double* x, int64_t n, const md_box* box,
                       const md_nlist* nl, md_precision prec, const double* u, double* gx,
                       double* gparam, void* ws, size_t ws_bytes, void* stream);

/* Mini-benchmark (the paper's setup-time TpA/BpA selection, over every K):
   for K = 1, 2, 4, ..., 64 build the list in layout K from x and time `reps`
   force launches; *choice [host] gets the fastest K.  The list is left in
   that layout.  Synchronises.  The winner is cached per (device, potential
   type, precision, power-of-two bucket of the largest neighbour count,
   power-of-two bucket of n) and md_step's AUTO reuses it. */
md_status md_autoselect(const md_potential* p, const double* x, int64_t n, const md_box* box,
                        const md_cells* cells, double skin, md_nlist* nl, md_precision prec,
                        int reps, md_kernel* choice, void* ws, size_t ws_bytes, void* stream);

/* Copy the status words to the host (synchronises the stream). */
md_status md_nlist_status(const md_nlist* nl, int* words /*[host] MD_STATUS_WORDS*/,
                          void* stream);

/* Kernel timing.  While enabled, every `every`-th force-kernel launch made by
   md_step / md_compute_forces is bracketed by start/stop timestamps recorded
   inside its dispatch (hipExtLaunchKernel events).  md_timing_read returns the
   number of timed launches and their summed duration in ms, and resets the
   sums.  Reading synchronises the device. */
md_status md_timing_enable(int every);
md_status md_timing_read(int64_t* launches /*[host]*/, double* total_ms /*[host]*/);

const char* md_status_string(md_status s);

#ifdef __cplusplus
}
#endif
#endif /* MD_MI355X_H */
