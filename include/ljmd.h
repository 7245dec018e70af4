/*
 * ljmd.h -- C ABI of the MI355X (gfx950) short-range Lennard-Jones MD hot path.
 *
 * The paper (Introduction; Cabana "Particle Sorting", "Neighbor List
 * Creation", "Parallel Loops" and "CabanaMD" subsections) splits a short-range
 * MD timestep into: sort particles by spatial bin, build Verlet neighbor lists
 * from a distance criterion on a binning grid, evaluate the per-particle force
 * kernel over the neighbor list, and propagate positions; the library side
 * owns sorting, lists and neighbor indexing, the application side owns the
 * force model and integration, and the library is callable from C through
 * memory-wrapping interfaces over caller-owned data.  This header is that
 * boundary:
 *
 *   ljmd_bin              counting sort of atoms into cells (cell-major, id-minor)
 *   ljmd_build_neighbors  Verlet lists over the 27-cell stencil (full or half)
 *   ljmd_compute_forces   12-6 LJ forces, per-atom energy, energy + virial
 *   ljmd_integrate        velocity-Verlet half kick + drift + wrap / half kick
 *   ljmd_md_step          forces and both half kicks + drift of one step, fused
 *   ljmd_md_step_chained, ljmd_md_step_sums
 *                         the same step with its energy sums formed during the
 *                         next step's launch (one launch per step)
 *   ljmd_md_step_noalloc  the fused step for callers that cannot allocate
 *   ljmd_max_displacement largest displacement since a list was built (the
 *                         dangerous-build check of a fixed rebuild cadence)
 *   ljmd_build_neighbors_csr, ljmd_list_to_csr, ljmd_compute_forces_csr
 *                         compressed list form and team-per-atom traversal
 *   ljmd_compute_forces_aosoa, ljmd_aosoa_convert
 *                         forces with positions in AoSoA layouts
 *   ljmd_force_backward   vector-Jacobian product of the forces (adjoint)
 *   ljmd_sph_density, ljmd_sph_accel, ljmd_sph_accel_step
 *                         SPH density summation and pressure acceleration over
 *                         the same lists (second short-range pair kernel)
 *   ljmd_ewald_real, ljmd_spme_recip
 *                         long-range electrostatics: Ewald real space over the
 *                         lists, smooth particle-mesh Ewald in reciprocal space
 *
 * plus a few helpers (grid, workspace sizes, errors) and the elementwise
 * steps of the discrete trajectory adjoint.
 *
 * Conventions, common to every call:
 *  - Units: LJ reduced units, k_B = 1.  Orthorhombic periodic box [0, L).
 *  - Positions, velocities, forces: FP64, [n][3] row-major (x, y, z per atom).
 *  - Every array argument is a DEVICE pointer owned by the caller, except
 *    where marked (host).  The library allocates and frees nothing and keeps
 *    no state between calls, except the static scratch array of
 *    ljmd_md_step_noalloc.  Outputs never alias inputs unless stated.
 *  - `stream` is a hipStream_t passed as void* (NULL: the null stream).  All
 *    device work is enqueued asynchronously on it; no call synchronizes.
 *  - Return value: LJMD_OK or an error code; no exception crosses the ABI.
 *    ljmd_last_error() gives a thread-local message for the last failure.
 *  - Minimum image: for positions within L/2 of [0, L), d = x_i - x_j folded
 *    to its representative nearest zero per component.  Requires
 *    rlist <= (1/2 - 1e-9) * min(L) (else LJMD_EBOX).
 *  - r^2 = (dx*dx + dy*dy) + dz*dz in FP64 without contraction; the neighbor
 *    test is r^2 < rlist*rlist and the force cutoff r^2 < rc*rc (strict).
 *  - Atom counts are limited to n < 2^31 - 64.
 */
#ifndef LJMD_H
#define LJMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define LJMD_OK 0
#define LJMD_EINVAL 1     /* null pointer, bad size, bad enum, non-positive rc/dt/mass */
#define LJMD_EBOX 2       /* non-positive box edge or rlist too large for minimum image */
#define LJMD_EWORKSPACE 3 /* workspace or cell buffer smaller than required */
#define LJMD_EHIP 4       /* HIP launch/runtime error; see ljmd_last_error() */

/* ---- enums ---- */
#define LJMD_FP64 0   /* all pair arithmetic in FP64 */
#define LJMD_MIXED 1  /* FP64 displacement, r^2 and cutoff test; FP32 pair math
                         (the pair energy: FP64 from the FP32 reciprocal after one
                         FP64 Newton step); FP64 accumulation of forces, energies,
                         virial, gradients */
#define LJMD_FULL 0   /* every ordered pair (i, j): each atom owns all its neighbors */
#define LJMD_HALF 1   /* each unordered pair once, owned by the lower sorted index */
#define LJMD_KICK_DRIFT 0 /* v += dt/2 F/m; x += dt v; wrap x into [0, L) */
#define LJMD_KICK 1       /* v += dt/2 F/m */
#define LJMD_KINETIC 2    /* no update: only the kinetic energy 1/2 m sum v^2 into ke */
#define LJMD_KICK_KICK_DRIFT 3 /* end of one step and start of the next, one pass:
                                  v += dt/2 F/m (ke taken here); v += dt/2 F/m;
                                  x += dt v; wrap -- bitwise equal to KICK then KICK_DRIFT */

/* workspace queries (ljmd_workspace_bytes) */
#define LJMD_OP_BIN 0
#define LJMD_OP_FORCES 1
#define LJMD_OP_BACKWARD 2
#define LJMD_OP_INTEGRATE 3
#define LJMD_OP_LOSS 4
#define LJMD_OP_CSR 5        /* ljmd_list_to_csr */
#define LJMD_OP_FORCES_CSR 6 /* ljmd_compute_forces_csr (any team) */
#define LJMD_OP_SPH 7        /* ljmd_sph_density (with u_total), ljmd_sph_accel(_step) */
#define LJMD_OP_EWALD_REAL 8 /* ljmd_ewald_real */
#define LJMD_OP_SPME 9       /* ljmd_spme_recip; ncells = K[0]*K[1]*K[2] grid points */
#define LJMD_OP_MD_CHAIN 10  /* ljmd_md_step_chained, ljmd_md_step_sums (two halves) */
#define LJMD_OP_DISPLACEMENT 11 /* ljmd_max_displacement */
#define LJMD_OP_BUILD_CSR 12    /* ljmd_build_neighbors_csr */
#define LJMD_SPME_MAX_GRID 256 /* largest grid edge of ljmd_spme_recip */

#define LJMD_MAX_TYPES 8
#define LJMD_TILE 64     /* atoms per neighbor-list tile: one wavefront */
#define LJMD_MAX_TEAM 16 /* largest team (lanes per atom) of ljmd_compute_forces_csr */
/* Tiled FULL-list forces (ljmd_compute_forces, ljmd_compute_forces_aosoa, the
 * fused steps) take four lanes per atom up to this many atoms (one 128-atom
 * block per compute unit), two beyond: the team size fixes the summation order. */
#define LJMD_SMALL_GRID_ATOMS 32768

typedef struct {
  double L[3]; /* box edges; periodic in all three dimensions, origin at 0 */
} ljmd_box;

/* Cell grid for binning at list cutoff rlist (host only, no device work):
 * nc[k] = floor(L[k]/rlist), reduced by one while L[k]/nc[k] is not above
 * rlist by a relative 1e-10, and at least 1.  The number of cells is
 * nc[0]*nc[1]*nc[2]; cell (cx, cy, cz) has linear index (cz*nc[1] + cy)*nc[0] + cx.
 * Errors: LJMD_EINVAL (null), LJMD_EBOX (L <= 0 or rlist too large). */
int ljmd_grid(const ljmd_box *box, double rlist, int32_t nc[3]);

/* Bytes of device workspace `op` needs for n atoms (ncells: cells of the
 * grid, used by LJMD_OP_BIN; ntypes: used by LJMD_OP_BACKWARD). 0 on bad op. */
size_t ljmd_workspace_bytes(int op, int64_t n, int64_t ncells, int32_t ntypes);

/* Human-readable text for a return code; thread-local detail of the last error. */
const char *ljmd_error_string(int code);
const char *ljmd_last_error(void);

/*
 * ljmd_bin -- re-sort particles by spatial bin (paper: Cabana "Particle
 * Sorting", geometric binning; Introduction: particles are re-sorted to begin
 * the next timestep).
 *
 * Cell of atom i: c_k = min(floor(x_ik / h_k), nc_k - 1), h_k = L_k / nc_k, with
 * nc from ljmd_grid(box, rlist).  Output order: cell-major, and inside a cell
 * ascending id.  The result is a deterministic permutation (it does not
 * depend on the order of atomic operations inside the sort).
 *   x_in [n][3]          positions in [0, L) (values outside are clamped to
 *                        the border cells, which the neighbor search
 *                        then cannot guarantee to find)
 *   v_in [n][3]          velocities, or NULL (then v_out is ignored)
 *   type_in [n]          int32 types, or NULL (then type_out is ignored)
 *   id_in [n]            int64 unique ids, or NULL (ids := input positions)
 *   x_out, v_out, type_out, id_out   permuted copies ([n][3], [n][3], [n], [n])
 *   cell_start [ncells+1] int32: sorted positions [cell_start[c], cell_start[c+1])
 *                        hold cell c; cell_start[ncells] = n
 *   cell_cap             length of cell_start; must be >= ncells+1 (else EWORKSPACE)
 *   ws, ws_bytes         device workspace, >= ljmd_workspace_bytes(LJMD_OP_BIN, n, ncells, 0)
 */
int ljmd_bin(const ljmd_box *box, double rlist, int64_t n, const double *x_in,
             const double *v_in, const int32_t *type_in, const int64_t *id_in, double *x_out,
             double *v_out, int32_t *type_out, int64_t *id_out, int32_t *cell_start,
             int64_t cell_cap, void *ws, size_t ws_bytes, void *stream);

/*
 * ljmd_build_neighbors -- Verlet lists by binning (paper: Cabana "Neighbor
 * List Creation": distance-criterion lists built on a search grid, dense
 * storage).  Requires atoms already sorted by ljmd_bin with the SAME box and
 * rlist (cell_start from that call).
 *
 * kind LJMD_FULL: N(i) = { j != i : r^2_ij < rlist^2 }.
 * kind LJMD_HALF: the pairs of the full relation with j > i (sorted indices).
 * r^2_ij is the FP64 (dx*dx + dy*dy) + dz*dz of the minimum-image
 * displacement.  The kernel settles most pairs with an integer test on 16-bit
 * lattice coordinates about each cell's centre, whose error bound keeps it to
 * pairs clearly inside or outside rlist; every other pair takes the FP64 test,
 * so each decision is that test's.
 * Storage is tiled ELL, one tile per 64 consecutive sorted atoms:
 *   neighbor k of atom i is nbr[((i / 64) * maxn + k) * 64 + (i % 64)], k < nnbr[i]
 * so nbr holds ceil(n/64)*64*maxn int32 (sorted indices).  Order inside a row
 * is unspecified.
 *   x          sorted positions [n][3]
 *   cell_start from ljmd_bin
 *   maxn       row capacity (>= 1)
 *   nbr, nnbr  outputs as above; nnbr[i] = min(|N(i)|, maxn)
 *   max_count  device int32 scalar, overwritten with max_i |N(i)|.  If it
 *              exceeds maxn after the stream has run, rows were truncated:
 *              the caller enlarges maxn and calls again (capacity overflow
 *              is reported on the device, not as a return code).
 */
int ljmd_build_neighbors(const ljmd_box *box, double rlist, int kind, int64_t n,
                         const double *x, const int32_t *cell_start, int32_t maxn,
                         int32_t *nbr, int32_t *nnbr, int32_t *max_count, void *stream);

/*
 * ljmd_build_neighbors_csr -- the same lists as ljmd_build_neighbors, built
 * straight into compressed (CSR) storage (paper: Cabana "Neighbor List
 * Creation" -- compressed lists, row offsets plus one flat index array, built
 * from the binning grid): a counting pass over the stencil, an exclusive scan
 * of the row lengths, then a filling pass.  Row order as ljmd_build_neighbors'
 * for the same kind.
 *   offsets  int64 [n+1] output: row i is nbr[offsets[i] .. offsets[i+1]);
 *            offsets[n] = total entries
 *   nbr      int32 [cap] output; entries at positions >= cap are not written,
 *            so a too-small cap is seen as offsets[n] > cap once the call
 *            completes (the caller builds again with cap >= offsets[n])
 *   ws       >= ljmd_workspace_bytes(LJMD_OP_BUILD_CSR, n, 0, 0)
 * Other arguments and errors as in ljmd_build_neighbors.
 */
int ljmd_build_neighbors_csr(const ljmd_box *box, double rlist, int kind, int64_t n,
                             const double *x, const int32_t *cell_start, int64_t *offsets,
                             int32_t *nbr, int64_t cap, void *ws, size_t ws_bytes, void *stream);

/*
 * ljmd_compute_forces -- 12-6 Lennard-Jones forces over the neighbor list
 * (paper: CabanaMD's Lennard-Jones short-range force kernel, written as a
 * neighbor parallel loop; Introduction: per-particle forces from the
 * neighborhood description).
 *
 * For each listed pair with r^2 < rc^2 and parameters (eps, sigma) of the
 * type pair:  u = 4 eps [(sigma/r)^12 - (sigma/r)^6],  s = -u'(r)/r,
 *   F_i = sum_j s d_ij,  e_i = 1/2 sum_j u_ij,
 *   ev = { E = sum_i e_i, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz },  W = 1/2 sum_i sum_j d_ij (s d_ij)^T
 * (truncated, unshifted; one absolute rc for every type pair).
 *   precision  LJMD_FP64 or LJMD_MIXED
 *   kind       list kind built by ljmd_build_neighbors.  FULL: a team of
 *              lanes per atom (four up to LJMD_SMALL_GRID_ATOMS atoms, else
 *              two), no atomics, bitwise deterministic.  HALF: Newton's third
 *              law with FP64 atomic updates (summation order not fixed).
 *   ntypes     1..LJMD_MAX_TYPES; eps_packed/sigma_packed: device FP64
 *              [ntypes(ntypes+1)/2], upper triangle row-major:
 *              entry (a, b), a <= b, at a*ntypes - a(a-1)/2 + (b - a)
 *   type       int32 [n] sorted types, or NULL when ntypes == 1
 *   F          [n][3] overwritten
 *   e_atom     [n] overwritten, or NULL
 *   ev         [7] overwritten, or NULL
 *   ws         >= ljmd_workspace_bytes(LJMD_OP_FORCES, n, 0, ntypes)
 */
int ljmd_compute_forces(const ljmd_box *box, int precision, int kind, double rc,
                        int32_t ntypes, const double *eps_packed, const double *sigma_packed,
                        int64_t n, const double *x, const int32_t *type, const int32_t *nbr,
                        const int32_t *nnbr, int32_t maxn, double *F, double *e_atom,
                        double *ev, void *ws, size_t ws_bytes, void *stream);

/*
 * ljmd_integrate -- velocity Verlet (paper: CabanaMD keeps the position
 * integration in the application; Introduction: forces propagate particles
 * to new positions).  In place on x and v.
 *   stage LJMD_KICK_DRIFT: v += dt/2 F/m; x += dt v; wrap each component:
 *         if x >= L: x -= L, else if x < 0: x += L; then if x >= L: x -= L
 *   stage LJMD_KICK:       v += dt/2 F/m
 *   stage LJMD_KINETIC:    nothing is updated (x, F may be NULL, dt is ignored);
 *                          ke is required
 *   stage LJMD_KICK_KICK_DRIFT: LJMD_KICK followed by LJMD_KICK_DRIFT with the
 *                          same F, in one pass; ke (if given) is the kinetic
 *                          energy between the two kicks (the integer time step)
 *   ke    device FP64 scalar receiving 1/2 m sum v^2 after the update, or NULL
 *   ws    >= ljmd_workspace_bytes(LJMD_OP_INTEGRATE, n, 0, 0) when ke != NULL
 */
int ljmd_integrate(int stage, double dt, double mass, const ljmd_box *box, int64_t n,
                   double *x, double *v, const double *F, double *ke, void *ws,
                   size_t ws_bytes, void *stream);

/*
 * ljmd_compute_forces_aosoa -- ljmd_compute_forces on a FULL list with positions
 * and forces in an AoSoA(vlen) layout (paper: Cabana "Particle abstractions:
 * data structures" -- arrays of structs of arrays with a vector length; the
 * CabanaMD LJ kernel is the vehicle for its layout studies).  Layout: chunks of
 * vlen consecutive atoms, each holding its x's, then its y's, then its z's;
 * the last chunk holds the m = n mod vlen remaining atoms (when nonzero) the
 * same way, so the array is exactly 3n doubles.  Component k of atom i, in
 * chunk c = i / vlen of width w = min(vlen, n - c*vlen), is at
 * c*3*vlen + k*w + (i - c*vlen).
 *   vlen     1 (the [n][3] arrays of every other call), 8, 64, or 0 for plain
 *            SoA (component k of atom i at k*n + i); n <= 2^24 unless vlen = 1
 *   x        [3n] positions in that layout; F [3n] output forces in it
 * Same list traversal and summation order as ljmd_compute_forces: forces,
 * energies and virial are bitwise the same in every layout.  Other arguments,
 * workspace (LJMD_OP_FORCES) and errors as in ljmd_compute_forces.
 */
int ljmd_compute_forces_aosoa(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                              const double *eps_packed, const double *sigma_packed, int64_t n,
                              int32_t vlen, const double *x, const int32_t *type,
                              const int32_t *nbr, const int32_t *nnbr, int32_t maxn, double *F,
                              double *e_atom, double *ev, void *ws, size_t ws_bytes,
                              void *stream);

/* Rearranges [n][3] rows into AoSoA(vlen) (to_aosoa = 1) or back (0); src and
 * dst must not alias.  vlen as in ljmd_compute_forces_aosoa. */
int ljmd_aosoa_convert(int64_t n, int32_t vlen, int to_aosoa, const double *src, double *dst,
                       void *stream);

/*
 * ljmd_force_backward -- adjoint of ljmd_compute_forces (FULL list only).
 * For a cotangent g = dL/dF [n][3], with the list and the pair set r < rc held
 * fixed (the truncation is not differentiated), K_ij = s I + 2 s' d d^T and
 * s' = ds/d(r^2):
 *   gx_i     = sum_j K_ij (g_i - g_j)
 *   geps[p]  = sum over ordered pairs (i, j) of type pair p of g_i . d_ij ds/deps
 *   gsigma[p]= the same with ds/dsigma
 *   accumulate  0: gx, geps, gsigma are overwritten; 1: added to
 *   ws          >= ljmd_workspace_bytes(LJMD_OP_BACKWARD, n, 0, ntypes)
 * Other arguments as in ljmd_compute_forces.  Bitwise deterministic.
 */
int ljmd_force_backward(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                        const double *eps_packed, const double *sigma_packed, int64_t n,
                        const double *x, const int32_t *type, const int32_t *nbr,
                        const int32_t *nnbr, int32_t maxn, const double *g, double *gx,
                        double *geps, double *gsigma, int accumulate, void *ws,
                        size_t ws_bytes, void *stream);

/*
 * ljmd_md_step -- one fused velocity-Verlet step on a FULL list: the forces of
 * ljmd_compute_forces at x, then for every atom the closing half kick
 * v += dt/2 F/m (the kinetic energy is taken here), and, when open_next is
 * nonzero, the next step's opening half kick v += dt/2 F/m, drift
 * x_next = x + dt v and wrap (paper: the MD timestep computes each particle's
 * forces and propagates it -- Introduction; CabanaMD keeps force kernel and
 * integration together in the application).  Positions, velocities and
 * forces are bitwise the same as ljmd_compute_forces followed by
 * ljmd_integrate(LJMD_KICK) and ljmd_integrate(LJMD_KICK_DRIFT); the kinetic
 * energy is summed per atom first, so it can differ from LJMD_KICK's in the
 * last bits.
 *   x        positions at this step (read by every lane: must not alias x_next)
 *   v        [n][3] in/out: half-step velocities in, updated velocities out
 *   x_next   [n][3] output positions of the next step (ignored, may be NULL,
 *            when open_next == 0)
 *   F        [n][3] output forces, or NULL
 *   e_atom   [n] output per-atom energy, or NULL
 *   ev       [8] output: E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz, kinetic energy
 *   ws       >= ljmd_workspace_bytes(LJMD_OP_FORCES, n, 0, ntypes)
 * Other arguments as in ljmd_compute_forces and ljmd_integrate.
 */
int ljmd_md_step(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                 const double *eps_packed, const double *sigma_packed, int64_t n,
                 const double *x, const int32_t *type, const int32_t *nbr, const int32_t *nnbr,
                 int32_t maxn, double dt, double mass, double *v, double *x_next, int open_next,
                 double *F, double *e_atom, double *ev, void *ws, size_t ws_bytes, void *stream);

/*
 * ljmd_md_step_noalloc -- ljmd_md_step without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  It runs the same
 * kernels with the same results, bitwise; its per-block energy/virial/kinetic
 * rows go to a static device array of LJMD_NOALLOC_SCRATCH_BYTES that every GPU
 * the library runs on holds until the process ends.  The first call on a
 * device looks up that device's copy (hipGetSymbolAddress, the device current
 * at the call; `stream` must belong to it); no call allocates or frees memory.
 * Limits and sharing:
 *   n        at most LJMD_NOALLOC_MAX_ATOMS (else LJMD_EWORKSPACE, nothing runs)
 *   calls that overlap on one GPU (different streams or threads, or another
 *   call enqueued before this one's launch has run) share the array and race:
 *   serialize them on one stream.  Each call writes every row it reads, so the
 *   previous call's contents never enter a result.
 * Other arguments and errors as in ljmd_md_step.
 */
#define LJMD_NOALLOC_SCRATCH_BYTES (2u << 20)
#define LJMD_NOALLOC_MAX_ATOMS 4194304 /* (2 MiB / 64 B per 128-atom block) * 128 */
int ljmd_md_step_noalloc(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                         const double *eps_packed, const double *sigma_packed, int64_t n,
                         const double *x, const int32_t *type, const int32_t *nbr,
                         const int32_t *nnbr, int32_t maxn, double dt, double mass, double *v,
                         double *x_next, int open_next, double *F, double *e_atom, double *ev,
                         void *stream);

/*
 * ljmd_md_step_chained -- ljmd_md_step without its own column-sum launch: the
 * step's energy/virial/kinetic partial rows (one per block) stay in half `half`
 * of ws, and the launch's first workgroup also sums the rows the previous
 * chained call left in the other half into ev_prev.  A run of steps alternates
 * half = 0, 1, 0, ... and so costs one launch per step; the sums of the last
 * step come from ljmd_md_step_sums.  Positions, velocities, forces and per-atom
 * energies are bitwise those of ljmd_md_step, and so are the sums from
 * ljmd_md_step_sums; ev_prev holds the same totals added in another order
 * (equal to rounding).  Same paper passage as ljmd_md_step.
 *   half     0 or 1: the half of ws that receives this step's partial rows
 *   ev_prev  [8] output: E, W (6), kinetic energy of the previous step, summed
 *            from the other half, or NULL when there is no previous step (the
 *            other half is then not read).  The previous call must have had the
 *            same n and the other half, and must precede this one on the stream.
 *   ws       >= ljmd_workspace_bytes(LJMD_OP_MD_CHAIN, n, 0, ntypes), kept
 *            between the calls of a run
 * Other arguments as in ljmd_md_step.
 */
int ljmd_md_step_chained(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                         const double *eps_packed, const double *sigma_packed, int64_t n,
                         const double *x, const int32_t *type, const int32_t *nbr,
                         const int32_t *nnbr, int32_t maxn, double dt, double mass, double *v,
                         double *x_next, int open_next, double *F, double *e_atom, int half,
                         double *ev_prev, void *ws, size_t ws_bytes, void *stream);

/*
 * ljmd_md_step_sums -- ev [8] (E, W (6), kinetic energy) of the ljmd_md_step_chained
 * call that wrote half `half` of ws, with n atoms; bitwise the ev of ljmd_md_step
 * on the same step.  ws as in that call.
 */
int ljmd_md_step_sums(int64_t n, int half, const void *ws, size_t ws_bytes, double *ev,
                      void *stream);

/*
 * ljmd_list_to_csr -- compressed (CSR) copy of a tiled neighbor list (paper:
 * Cabana stores neighbor lists either compressed -- row offsets plus one flat
 * index array -- or dense, with a fixed row capacity; "Neighbor List
 * Creation").  Rows keep their order.
 *   nbr, nnbr, maxn  a list from ljmd_build_neighbors (rows of min(nnbr, maxn))
 *   offsets  int64 [n+1] output: row i is csr[offsets[i] .. offsets[i+1])
 *   csr      int32 [cap] output; entries at positions >= cap are not written,
 *            so a too-small cap is seen as offsets[n] > cap once the call completes
 *   ws       >= ljmd_workspace_bytes(LJMD_OP_CSR, n, 0, 0)
 */
int ljmd_list_to_csr(int64_t n, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                     int64_t *offsets, int32_t *csr, int64_t cap, void *ws, size_t ws_bytes,
                     void *stream);

/*
 * ljmd_compute_forces_csr -- the FULL-list forces of ljmd_compute_forces over a
 * CSR list (ljmd_list_to_csr of a FULL list), with `team` lanes per atom
 * (paper: Cabana's hierarchical neighbor traversal -- one thread per particle
 * or a team of threads per particle; "Parallel Loops").  Lane t of a team takes
 * row entries t, t + team, ...; the team's sums are combined in a fixed
 * butterfly order, so results are bitwise deterministic.  ljmd_compute_forces
 * walks a FULL tiled list with teams of four up to LJMD_SMALL_GRID_ATOMS atoms
 * and of two beyond; with the same team the forces and per-atom energies here
 * are bitwise those (E and W agree to rounding).
 *   team     1, 2, 4, 8 or 16
 *   offsets, csr  as produced by ljmd_list_to_csr (entries must be in [0, n))
 *   ws       >= ljmd_workspace_bytes(LJMD_OP_FORCES_CSR, n, 0, ntypes) when
 *            ev or e_atom is given
 * Other arguments as in ljmd_compute_forces.
 */
int ljmd_compute_forces_csr(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                            const double *eps_packed, const double *sigma_packed, int64_t n,
                            const double *x, const int32_t *type, const int64_t *offsets,
                            const int32_t *csr, int32_t team, double *F, double *e_atom,
                            double *ev, void *ws, size_t ws_bytes, void *stream);

/*
 * ljmd_sph_density, ljmd_sph_accel -- smoothed-particle hydrodynamics over the
 * same binned full lists (paper: SPH is, beside MD, a user of the short-range
 * particle-particle sub-motif and of Verlet neighbor lists -- Introduction;
 * Cabana "Neighbor List Creation").  The paper prints no SPH equations; the
 * textbook forms are used, all in FP64:
 *   cubic-spline kernel (Monaghan & Lattanzio 1985), support 2h, q = r/h:
 *     W(r) = w(q)/(pi h^3), w = 1 - 3/2 q^2 + 3/4 q^3 (q < 1), 1/4 (2-q)^3 (1 <= q < 2), 0 beyond
 *   rho_i = m W(0) + sum_{j in row i, r_ij^2 < (2h)^2} m W(r_ij)
 *   p = c0^2 (rho - rho0)
 *   a_i = - sum_j m (p_i/rho_i^2 + p_j/rho_j^2) W'(r_ij)/r_ij d_ij   (Monaghan 1992,
 *         no artificial viscosity; d_ij = minimum-image x_i - x_j)
 *   U = sum_i m c0^2 (ln(rho_i/rho0) + rho0/rho_i - 1), so that m a_i = -dU/dx_i.
 * The list (nbr, nnbr, maxn) is a FULL list from ljmd_build_neighbors with
 * rlist >= 2h over the same sorted positions x; pairs farther than 2h are
 * skipped, pairs missing from the list are not seen.  Summation order is fixed:
 * results are bitwise reproducible.
 *   h, mass, rho0 > 0; c0 >= 0; 2h <= (1/2 - 1e-9) min(L) (else LJMD_EBOX)
 *   rho      [n] overwritten (density pass); read by the acceleration pass
 *            (values from the density pass are >= m/(pi h^3) > 0)
 *   u_total  device FP64 scalar receiving U, or NULL
 *   acc      [n][3] overwritten with a_i
 *   ws       >= ljmd_workspace_bytes(LJMD_OP_SPH, n, 0, 0) bytes: the density pass
 *            needs it only when u_total is given; the acceleration pass always
 *            (n > 0) and requires it 32-byte aligned (LJMD_EINVAL otherwise)
 */
int ljmd_sph_density(const ljmd_box *box, double h, double mass, double c0, double rho0, int64_t n,
                     const double *x, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                     double *rho, double *u_total, void *ws, size_t ws_bytes, void *stream);
int ljmd_sph_accel(const ljmd_box *box, double h, double mass, double c0, double rho0, int64_t n,
                   const double *x, const double *rho, const int32_t *nbr, const int32_t *nnbr,
                   int32_t maxn, double *acc, void *ws, size_t ws_bytes, void *stream);

/*
 * ljmd_sph_accel_step -- ljmd_sph_accel followed, in the same pass, by the
 * closing half kick of this step and the next step's opening half kick, drift
 * and wrap (velocity Verlet with the acceleration as F/m): per component
 * v += dt/2 a twice, x += dt v, wrapped into [0, L).  x, v and acc are bitwise
 * those of ljmd_sph_accel then ljmd_integrate(LJMD_KICK_KICK_DRIFT, dt,
 * mass 1, F = acc) (the paper's MD timestep: forces, then propagation --
 * Introduction).
 *   x     [n][3] in/out: positions of this step in, of the next step out
 *   v     [n][3] in/out: half-step velocities
 *   dt    nonzero, finite
 *   acc   [n][3] output of a_i, or NULL
 * Other arguments as in ljmd_sph_accel.
 */
int ljmd_sph_accel_step(const ljmd_box *box, double h, double mass, double c0, double rho0,
                        int64_t n, double *x, double *v, const double *rho, const int32_t *nbr,
                        const int32_t *nnbr, int32_t maxn, double dt, double *acc, void *ws,
                        size_t ws_bytes, void *stream);

/*
 * ljmd_ewald_real, ljmd_spme_recip -- electrostatics of point charges by smooth
 * particle-mesh Ewald (paper: CabanaMD's long-range forces -- real-space
 * energies and forces through the neighbor parallel loops; reciprocal space by
 * spline spreading of charge to a uniform grid, 3-D FFTs and a gradient kernel
 * that gathers forces back; Cabana "Long Range Solvers", "Particle-Grid
 * Interpolation").  The method is SPME as defined by Essmann et al. (1995),
 * Gaussian units (k_e = 1), neutral system, conducting boundary, FP64:
 *   E_dir  = 1/2 sum_i sum_{j in row i, r < rc} q_i q_j erfc(alpha r)/r
 *   E_rec  = 1/2 sum_{m != 0} B(m) C(m) |F(Q)(m)|^2 with the order-n cardinal
 *            B-spline charge grid Q on K[0] x K[1] x K[2] points (x fastest),
 *            B(m) = prod_a |b_a(m_a)|^2, C(m) = exp(-pi^2 |m'|^2/alpha^2)/(pi V |m'|^2)
 *   E_self = -alpha/sqrt(pi) sum_i q_i^2
 * and the forces are minus the gradients of E_dir and E_rec.
 *
 * ljmd_ewald_real: the list is a FULL list (ljmd_build_neighbors, rlist >= rc)
 *   over the same sorted x; q [n] charges in the same order.  F [n][3] receives
 *   the direct-space forces (accumulate 0: overwritten, 1: added); e_total (device
 *   FP64 scalar, or NULL) receives E_dir.  ws >= ljmd_workspace_bytes(
 *   LJMD_OP_EWALD_REAL, n, 0, 0), 32-byte aligned.  Fixed summation order.
 * ljmd_spme_recip: order 4, 6 or 8; K (host int32[3]) powers of two in
 *   [8, LJMD_SPME_MAX_GRID]; x [n][3] in [0, L) (any order), q [n].  F receives
 *   the reciprocal-space forces (accumulate as above); e_total (or NULL)
 *   receives E_rec + E_self.  ws >= ljmd_workspace_bytes(LJMD_OP_SPME, n,
 *   K[0]*K[1]*K[2], 0), 32-byte aligned; it holds the real charge grid and its
 *   half-complex transform.  The charge
 *   spreading uses FP64 atomic additions: results agree run to run to rounding,
 *   not bit for bit.
 *   alpha > 0; rc as for the other pair kernels (LJMD_EBOX if too large).
 */
int ljmd_ewald_real(const ljmd_box *box, double alpha, double rc, int64_t n, const double *x,
                    const double *q, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                    double *F, double *e_total, int accumulate, void *ws, size_t ws_bytes,
                    void *stream);
int ljmd_spme_recip(const ljmd_box *box, double alpha, int32_t order, const int32_t K[3],
                    int64_t n, const double *x, const double *q, double *F, double *e_total,
                    int accumulate, void *ws, size_t ws_bytes, void *stream);

/* ---- elementwise steps of the discrete velocity-Verlet adjoint ----
 *
 * Reverse of one step (x_n, v_n) -> (x_{n+1}, v_{n+1}) once the VJP at
 * x_{n+1} has been folded into xbar:  vbar += dt * xbar, then the VJP at x_n
 * with cotangent w * dt * vbar.  The kicks add dt/(2m) F, so w = 1/m where the
 * two half kicks meeting at an interior x_n are merged and 1/(2m) at the
 * first step.
 * ljmd_adjoint_kick: vbar += dt * xbar; g = w * dt * vbar.  [n][3] each. */
int ljmd_adjoint_kick(int64_t n, double dt, double w, const double *xbar, double *vbar,
                      double *g, void *stream);

/*
 * ljmd_max_displacement -- the largest squared minimum-image displacement
 * max_i |x_i - x_ref_i|^2 since the positions x_ref at which a list was built
 * (same atom order), the test of a dangerous build: a Verlet list of cutoff
 * rc + skin holds every pair inside rc only while no atom has moved more than
 * skin/2 since it was built (paper, Introduction: lists are reused between
 * rebuilds; Cabana "Neighbor List Creation").  With a fixed rebuild cadence a
 * caller checks it at each rebuild to learn whether the window that ends there
 * may have missed pairs.
 *   x, x_ref  [n][3] positions now and at the build; must not alias
 *   max_d2    device scalar output (0 for n = 0)
 *   ws        >= ljmd_workspace_bytes(LJMD_OP_DISPLACEMENT, n, 0, 1)
 * Errors: LJMD_EINVAL (null, aliasing), LJMD_EBOX, LJMD_EWORKSPACE, LJMD_EHIP.
 */
int ljmd_max_displacement(const ljmd_box *box, int64_t n, const double *x, const double *x_ref,
                          double *max_d2, void *ws, size_t ws_bytes, void *stream);

/* Trajectory loss on final positions: d = minimum image of (x - xref) (equal
 * to the unwrapped difference while the two trajectories stay within L/2),
 * xbar = d, loss = 1/2 sum |d|^2 (device scalar; deterministic reduction).
 * ws >= ljmd_workspace_bytes(LJMD_OP_LOSS, n, 0, 0). */
int ljmd_traj_loss(const ljmd_box *box, int64_t n, const double *x, const double *xref,
                   double *xbar, double *loss, void *ws, size_t ws_bytes, void *stream);

/* Row scatter through ids: dst[id[k]] = src[k] for rows of `width` doubles
 * (maps sorted-order results back to the caller's atom order).  Rows whose
 * id lies outside [0, n) are skipped. */
int ljmd_scatter_rows(int64_t n, int32_t width, const int64_t *id, const double *src,
                      double *dst, void *stream);

/* Row gather through ids: dst[k] = src[id[k]] (brings caller-order data into
 * sorted order).  Rows whose id lies outside [0, n) are left untouched. */
int ljmd_gather_rows(int64_t n, int32_t width, const int64_t *id, const double *src,
                     double *dst, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LJMD_H */
