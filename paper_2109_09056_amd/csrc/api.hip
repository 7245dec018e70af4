// extern "C" entry points of libljmd: argument validation, dispatch to the
// gfx950 kernels, error reporting.  Declared and documented in ljmd.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <mutex>

#include "common.h"

namespace ljmd {

// kernels' host launchers (one per source file)
size_t bin_workspace(int64_t n, int64_t ncells);
int launch_bin(const GridK &g, int64_t n, const double *x_in, const double *v_in,
               const int32_t *type_in, const int64_t *id_in, double *x_out, double *v_out,
               int32_t *type_out, int64_t *id_out, int32_t *cell_start, void *ws, hipStream_t st);
size_t build_csr_workspace(int64_t n);
int launch_build_csr(const GridK &g, const BoxK &b, double rlist, int kind, int64_t n,
                     const double *x, const int32_t *cell_start, int64_t *offsets, int32_t *csr,
                     int64_t cap, void *ws, hipStream_t st);
int launch_build(const GridK &g, const BoxK &b, double rlist, int kind, int64_t n, const double *x,
                 const int32_t *cell_start, int32_t maxn, int32_t *nbr, int32_t *nnbr,
                 int32_t *max_count, hipStream_t st);
size_t force_workspace(int64_t n);
int64_t force_workspace_atoms();
int launch_forces(const BoxK &b, int precision, int kind, double rc, int32_t ntypes,
                  const double *eps, const double *sig, int64_t n, const double *x,
                  const int32_t *type, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                  double *F, double *e_atom, double *ev, void *ws, hipStream_t st);
int launch_md_step(const BoxK &b, int precision, double rc, int32_t ntypes, const double *eps,
                   const double *sig, int64_t n, const double *x, const int32_t *type,
                   const int32_t *nbr, const int32_t *nnbr, int32_t maxn, double dt, double mass,
                   double *v, double *x_next, int open_next, double *F, double *e_atom, double *ev,
                   double *partial, const double *prev_partial, double *prev_ev, hipStream_t st);
int launch_md_step_sums(int64_t n, const double *partial, double *ev, hipStream_t st);
int launch_forces_aosoa(const BoxK &b, int precision, double rc, int32_t ntypes, const double *eps,
                        const double *sig, int64_t n, int vlen, const double *x,
                        const int32_t *type, const int32_t *nbr, const int32_t *nnbr,
                        int32_t maxn, double *F, double *e_atom, double *ev, void *ws,
                        hipStream_t st);
int launch_aosoa_convert(int64_t n, int vlen, int to_aosoa, const double *src, double *dst,
                         hipStream_t st);
size_t bwd_workspace(int64_t n, int32_t ntypes);
int launch_backward(const BoxK &b, int precision, double rc, int32_t ntypes, const double *eps,
                    const double *sig, int64_t n, const double *x, const int32_t *type,
                    const int32_t *nbr, const int32_t *nnbr, int32_t maxn, const double *g,
                    double *gx, double *geps, double *gsig, int accumulate, void *ws,
                    hipStream_t st);
size_t csr_workspace(int64_t n);
int launch_list_to_csr(int64_t n, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                       int64_t *offsets, int32_t *csr, int64_t cap, void *ws, hipStream_t st);
size_t csr_force_workspace(int64_t n);
int launch_forces_csr(const BoxK &b, int precision, double rc, int32_t ntypes, const double *eps,
                      const double *sig, int64_t n, const double *x, const int32_t *type,
                      const int64_t *offsets, const int32_t *csr, int team, double *F,
                      double *e_atom, double *ev, void *ws, hipStream_t st);
size_t sph_workspace(int64_t n);
int launch_sph_density(const BoxK &b, double h, double mass, double c0, double rho0, int64_t n,
                       const double *x, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                       double *rho, double *u_total, void *ws, hipStream_t st);
int launch_sph_accel(const BoxK &b, double h, double mass, double c0, double rho0, int64_t n,
                     const double *x, const double *rho, const int32_t *nbr,
                     const int32_t *nnbr, int32_t maxn, double *acc, double dt, double *v,
                     double *x_out, void *ws, hipStream_t st);
size_t ewald_real_workspace(int64_t n);
size_t spme_workspace(int64_t n, int64_t npts);
int launch_ewald_real(const BoxK &b, double alpha, double rc, int64_t n, const double *x,
                      const double *q, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                      double *F, double *e_total, int accumulate, void *ws, hipStream_t st);
int launch_spme_recip(const BoxK &b, double alpha, int32_t order, const int32_t K[3], int64_t n,
                      const double *x, const double *q, double *F, double *e_total,
                      int accumulate, void *ws, hipStream_t st);
size_t stream_workspace(int64_t n);
int launch_integrate(int stage, double dt, double mass, const BoxK &b, int64_t n, double *x,
                     double *v, const double *F, double *ke, void *ws, hipStream_t st);
int launch_adjoint_kick(int64_t n, double dt, double w, const double *xbar, double *vbar,
                        double *g, hipStream_t st);
int launch_max_displacement(const BoxK &b, int64_t n, const double *x, const double *xref,
                            double *max_d2, void *ws, hipStream_t st);
int launch_loss(const BoxK &b, int64_t n, const double *x, const double *xref, double *xbar,
                double *loss, void *ws, hipStream_t st);
int launch_scatter_rows(int64_t n, int32_t width, const int64_t *id, const double *src,
                        double *dst, hipStream_t st);
int launch_gather_rows(int64_t n, int32_t width, const int64_t *id, const double *src,
                       double *dst, hipStream_t st);

namespace {
thread_local char g_msg[512] = "";
constexpr int64_t kMaxAtoms = (int64_t)2147483647 - 64;
}  // namespace

int set_error(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
  va_end(ap);
  return code;
}

int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(LJMD_EHIP, "%s: %s", what, hipGetErrorString(e));
  return LJMD_OK;
}

BoxK make_box(const ljmd_box *b) {
  BoxK k;
  for (int d = 0; d < 3; ++d) {
    k.L[d] = b->L[d];
    k.invL[d] = 1.0 / b->L[d];
  }
  return k;
}

static int check_box(const ljmd_box *b) {
  if (!b) return set_error(LJMD_EINVAL, "box is NULL");
  for (int d = 0; d < 3; ++d)
    if (!(b->L[d] > 0.0) || !isfinite(b->L[d]))
      return set_error(LJMD_EBOX, "box edge L[%d] = %g must be finite and > 0", d, b->L[d]);
  return LJMD_OK;
}

static int check_cutoff(const ljmd_box *b, double r, const char *name) {
  if (!(r > 0.0) || !isfinite(r)) return set_error(LJMD_EINVAL, "%s = %g must be > 0", name, r);
  double lmin = fmin(b->L[0], fmin(b->L[1], b->L[2]));
  if (r > (0.5 - 1e-9) * lmin)
    return set_error(LJMD_EBOX, "%s = %g too large for minimum image in a box of edge %g", name,
                     r, lmin);
  return LJMD_OK;
}

int make_grid(const ljmd_box *b, double rlist, GridK *g) {
  int64_t total = 1;
  for (int d = 0; d < 3; ++d) {
    int64_t c = (int64_t)floor(b->L[d] / rlist);
    while (c > 1 && b->L[d] / (double)c < rlist * (1.0 + 1e-10)) --c;
    if (c < 1) c = 1;
    if (c > (int64_t)1 << 20) return set_error(LJMD_EBOX, "grid too fine (%lld cells)", (long long)c);
    g->nc[d] = (int32_t)c;
    g->h[d] = b->L[d] / (double)c;
    total *= c;
  }
  if (total > ((int64_t)1 << 30)) return set_error(LJMD_EBOX, "grid has %lld cells", (long long)total);
  g->ncells = (int32_t)total;
  return LJMD_OK;
}

static int check_n(int64_t n) {
  if (n < 0 || n > kMaxAtoms) return set_error(LJMD_EINVAL, "n = %lld out of range", (long long)n);
  return LJMD_OK;
}

static int check_ws(void *ws, size_t have, size_t need) {
  if (need > 0 && (!ws || have < need))
    return set_error(LJMD_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                     ws ? have : (size_t)0);
  return LJMD_OK;
}

static int check_params(int32_t ntypes, const double *eps, const double *sig, const int32_t *type,
                        int64_t n) {
  if (ntypes < 1 || ntypes > LJMD_MAX_TYPES)
    return set_error(LJMD_EINVAL, "ntypes = %d outside [1, %d]", ntypes, LJMD_MAX_TYPES);
  if (!eps || !sig) return set_error(LJMD_EINVAL, "eps/sigma is NULL");
  if (ntypes > 1 && n > 0 && !type) return set_error(LJMD_EINVAL, "type is NULL with ntypes > 1");
  return LJMD_OK;
}

}  // namespace ljmd

using namespace ljmd;

#define LJMD_TRY(expr)             \
  do {                             \
    int rc_ = (expr);              \
    if (rc_ != LJMD_OK) return rc_; \
  } while (0)

// Arguments common to ljmd_md_step and ljmd_md_step_chained.
static int check_md_step(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                         const double *eps_packed, const double *sigma_packed, int64_t n,
                         const double *x, const int32_t *type, const int32_t *nbr,
                         const int32_t *nnbr, int32_t maxn, double dt, double mass,
                         const double *v, const double *x_next, int open_next) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_cutoff(box, rc, "rc"));
  LJMD_TRY(check_n(n));
  if (precision != LJMD_FP64 && precision != LJMD_MIXED)
    return set_error(LJMD_EINVAL, "bad precision %d", precision);
  LJMD_TRY(check_params(ntypes, eps_packed, sigma_packed, type, n));
  if (maxn < 1) return set_error(LJMD_EINVAL, "maxn = %d must be >= 1", maxn);
  if (!isfinite(dt) || dt == 0.0) return set_error(LJMD_EINVAL, "dt = %g", dt);
  if (!(mass > 0.0) || !isfinite(mass)) return set_error(LJMD_EINVAL, "mass = %g", mass);
  if (open_next != 0 && open_next != 1)
    return set_error(LJMD_EINVAL, "open_next = %d must be 0 or 1", open_next);
  if (n > 0 && (!x || !nbr || !nnbr || !v || (open_next && !x_next)))
    return set_error(LJMD_EINVAL, "x/nbr/nnbr/v/x_next is NULL");
  if (n > 0 && open_next && x_next == x)
    return set_error(LJMD_EINVAL, "x_next must not alias x");
  return LJMD_OK;
}

// Scratch of the allocation-free step (ljmd_md_step_noalloc): the per-block energy /
// virial / kinetic rows of one fused step launch.  Every GPU the library runs on holds
// its own copy until the process ends.  In host code the array's name is a host-side
// stand-in, not a device address: kernels get the per-device address that
// hipGetSymbolAddress returns.
constexpr size_t kScratchBytes = LJMD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch, looked up once per device.
static int scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(LJMD_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(LJMD_EHIP, "device %d beyond the %d the scratch table holds", dev,
                     kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(LJMD_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                       hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LJMD_OK;
}

extern "C" {

const char *ljmd_error_string(int code) {
  switch (code) {
    case LJMD_OK: return "ok";
    case LJMD_EINVAL: return "invalid argument";
    case LJMD_EBOX: return "invalid box or cutoff";
    case LJMD_EWORKSPACE: return "workspace or buffer too small";
    case LJMD_EHIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

const char *ljmd_last_error(void) { return g_msg; }

int ljmd_grid(const ljmd_box *box, double rlist, int32_t nc[3]) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_cutoff(box, rlist, "rlist"));
  if (!nc) return set_error(LJMD_EINVAL, "nc is NULL");
  GridK g;
  LJMD_TRY(make_grid(box, rlist, &g));
  for (int d = 0; d < 3; ++d) nc[d] = g.nc[d];
  return LJMD_OK;
}

size_t ljmd_workspace_bytes(int op, int64_t n, int64_t ncells, int32_t ntypes) {
  if (n < 0) n = 0;
  switch (op) {
    case LJMD_OP_BIN: return bin_workspace(n, ncells > 0 ? ncells : 1);
    case LJMD_OP_FORCES: return force_workspace(n);
    case LJMD_OP_MD_CHAIN: return 2 * force_workspace(n);
    case LJMD_OP_BACKWARD:
      return bwd_workspace(n, ntypes < 1 ? 1 : (ntypes > LJMD_MAX_TYPES ? LJMD_MAX_TYPES : ntypes));
    case LJMD_OP_INTEGRATE:
    case LJMD_OP_LOSS:
    case LJMD_OP_DISPLACEMENT: return stream_workspace(n);
    case LJMD_OP_BUILD_CSR: return build_csr_workspace(n);
    case LJMD_OP_CSR: return csr_workspace(n);
    case LJMD_OP_FORCES_CSR: return csr_force_workspace(n);
    case LJMD_OP_SPH: return sph_workspace(n);
    case LJMD_OP_EWALD_REAL: return ewald_real_workspace(n);
    case LJMD_OP_SPME: return spme_workspace(n, ncells > 0 ? ncells : 1);
    default: return 0;
  }
}

int ljmd_bin(const ljmd_box *box, double rlist, int64_t n, const double *x_in,
             const double *v_in, const int32_t *type_in, const int64_t *id_in, double *x_out,
             double *v_out, int32_t *type_out, int64_t *id_out, int32_t *cell_start,
             int64_t cell_cap, void *ws, size_t ws_bytes, void *stream) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_cutoff(box, rlist, "rlist"));
  LJMD_TRY(check_n(n));
  GridK g;
  LJMD_TRY(make_grid(box, rlist, &g));
  if (!cell_start) return set_error(LJMD_EINVAL, "cell_start is NULL");
  if (cell_cap < (int64_t)g.ncells + 1)
    return set_error(LJMD_EWORKSPACE, "cell_start holds %lld entries, %d needed",
                     (long long)cell_cap, g.ncells + 1);
  if (n > 0) {
    if (!x_in || !x_out || !id_out) return set_error(LJMD_EINVAL, "x_in/x_out/id_out is NULL");
    if (v_in && !v_out) return set_error(LJMD_EINVAL, "v_out is NULL while v_in is given");
    if (type_in && !type_out) return set_error(LJMD_EINVAL, "type_out is NULL while type_in is given");
  }
  LJMD_TRY(check_ws(ws, ws_bytes, bin_workspace(n, g.ncells)));
  return launch_bin(g, n, x_in, v_in, type_in, id_in, x_out, v_out, type_out, id_out, cell_start,
                    ws, (hipStream_t)stream);
}

int ljmd_build_neighbors(const ljmd_box *box, double rlist, int kind, int64_t n,
                         const double *x, const int32_t *cell_start, int32_t maxn,
                         int32_t *nbr, int32_t *nnbr, int32_t *max_count, void *stream) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_cutoff(box, rlist, "rlist"));
  LJMD_TRY(check_n(n));
  if (kind != LJMD_FULL && kind != LJMD_HALF) return set_error(LJMD_EINVAL, "bad kind %d", kind);
  if (maxn < 1) return set_error(LJMD_EINVAL, "maxn = %d must be >= 1", maxn);
  if (!max_count || !cell_start) return set_error(LJMD_EINVAL, "max_count/cell_start is NULL");
  if (n > 0 && (!x || !nbr || !nnbr)) return set_error(LJMD_EINVAL, "x/nbr/nnbr is NULL");
  if ((n + LJMD_TILE - 1) / LJMD_TILE * LJMD_TILE * (int64_t)maxn > ((int64_t)1 << 40))
    return set_error(LJMD_EINVAL, "list of n = %lld rows x maxn = %d is too large", (long long)n, maxn);
  GridK g;
  LJMD_TRY(make_grid(box, rlist, &g));
  return launch_build(g, make_box(box), rlist, kind, n, x, cell_start, maxn, nbr, nnbr, max_count,
                      (hipStream_t)stream);
}

int ljmd_build_neighbors_csr(const ljmd_box *box, double rlist, int kind, int64_t n,
                             const double *x, const int32_t *cell_start, int64_t *offsets,
                             int32_t *nbr, int64_t cap, void *ws, size_t ws_bytes, void *stream) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_cutoff(box, rlist, "rlist"));
  LJMD_TRY(check_n(n));
  if (kind != LJMD_FULL && kind != LJMD_HALF) return set_error(LJMD_EINVAL, "bad kind %d", kind);
  if (!cell_start || !offsets) return set_error(LJMD_EINVAL, "cell_start/offsets is NULL");
  if (cap < 0) return set_error(LJMD_EINVAL, "cap = %lld must be >= 0", (long long)cap);
  if (n > 0 && (!x || (cap > 0 && !nbr))) return set_error(LJMD_EINVAL, "x/nbr is NULL");
  LJMD_TRY(check_ws(ws, ws_bytes, build_csr_workspace(n)));
  GridK g;
  LJMD_TRY(make_grid(box, rlist, &g));
  return launch_build_csr(g, make_box(box), rlist, kind, n, x, cell_start, offsets, nbr, cap, ws,
                          (hipStream_t)stream);
}

int ljmd_compute_forces(const ljmd_box *box, int precision, int kind, double rc,
                        int32_t ntypes, const double *eps_packed, const double *sigma_packed,
                        int64_t n, const double *x, const int32_t *type, const int32_t *nbr,
                        const int32_t *nnbr, int32_t maxn, double *F, double *e_atom,
                        double *ev, void *ws, size_t ws_bytes, void *stream) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_cutoff(box, rc, "rc"));
  LJMD_TRY(check_n(n));
  if (precision != LJMD_FP64 && precision != LJMD_MIXED)
    return set_error(LJMD_EINVAL, "bad precision %d", precision);
  if (kind != LJMD_FULL && kind != LJMD_HALF) return set_error(LJMD_EINVAL, "bad kind %d", kind);
  LJMD_TRY(check_params(ntypes, eps_packed, sigma_packed, type, n));
  if (maxn < 1) return set_error(LJMD_EINVAL, "maxn = %d must be >= 1", maxn);
  if (n > 0 && (!x || !nbr || !nnbr || !F)) return set_error(LJMD_EINVAL, "x/nbr/nnbr/F is NULL");
  const bool want_ev = ev != nullptr || e_atom != nullptr;
  LJMD_TRY(check_ws(ws, ws_bytes, want_ev ? force_workspace(n) : 0));
  return launch_forces(make_box(box), precision, kind, rc, ntypes, eps_packed, sigma_packed, n, x,
                       type, nbr, nnbr, maxn, F, e_atom, ev, ws, (hipStream_t)stream);
}

static int check_vlen(int32_t vlen) {
  if (vlen != 0 && vlen != 1 && vlen != 8 && vlen != 64)
    return set_error(LJMD_EINVAL, "vlen = %d must be 0 (SoA), 1, 8 or 64", vlen);
  return LJMD_OK;
}

int ljmd_compute_forces_aosoa(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                              const double *eps_packed, const double *sigma_packed, int64_t n,
                              int32_t vlen, const double *x, const int32_t *type,
                              const int32_t *nbr, const int32_t *nnbr, int32_t maxn, double *F,
                              double *e_atom, double *ev, void *ws, size_t ws_bytes,
                              void *stream) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_cutoff(box, rc, "rc"));
  LJMD_TRY(check_n(n));
  LJMD_TRY(check_vlen(vlen));
  if (precision != LJMD_FP64 && precision != LJMD_MIXED)
    return set_error(LJMD_EINVAL, "bad precision %d", precision);
  LJMD_TRY(check_params(ntypes, eps_packed, sigma_packed, type, n));
  if (maxn < 1) return set_error(LJMD_EINVAL, "maxn = %d must be >= 1", maxn);
  if (n > 0 && (!x || !nbr || !nnbr || !F)) return set_error(LJMD_EINVAL, "x/nbr/nnbr/F is NULL");
  if (n > kNarrowAtoms && vlen != 1)
    return set_error(LJMD_EINVAL, "AoSoA layouts take at most %lld atoms", (long long)kNarrowAtoms);
  const bool want_ev = ev != nullptr || e_atom != nullptr;
  LJMD_TRY(check_ws(ws, ws_bytes, want_ev ? force_workspace(n) : 0));
  return launch_forces_aosoa(make_box(box), precision, rc, ntypes, eps_packed, sigma_packed, n,
                             vlen, x, type, nbr, nnbr, maxn, F, e_atom, ev, ws,
                             (hipStream_t)stream);
}

int ljmd_aosoa_convert(int64_t n, int32_t vlen, int to_aosoa, const double *src, double *dst,
                       void *stream) {
  LJMD_TRY(check_n(n));
  LJMD_TRY(check_vlen(vlen));
  if (to_aosoa != 0 && to_aosoa != 1)
    return set_error(LJMD_EINVAL, "to_aosoa = %d must be 0 or 1", to_aosoa);
  if (n > 0 && (!src || !dst)) return set_error(LJMD_EINVAL, "src/dst is NULL");
  if (n > 0 && src == dst) return set_error(LJMD_EINVAL, "dst must not alias src");
  return launch_aosoa_convert(n, vlen, to_aosoa, src, dst, (hipStream_t)stream);
}

static int check_sph(const ljmd_box *box, double h, double mass, double c0, double rho0, int64_t n,
                     const double *x, const int32_t *nbr, const int32_t *nnbr, int32_t maxn) {
  LJMD_TRY(check_box(box));
  if (!(h > 0.0) || !isfinite(h)) return set_error(LJMD_EINVAL, "h = %g must be > 0", h);
  LJMD_TRY(check_cutoff(box, 2.0 * h, "2h"));
  LJMD_TRY(check_n(n));
  if (!(mass > 0.0) || !isfinite(mass)) return set_error(LJMD_EINVAL, "mass = %g must be > 0", mass);
  if (!(c0 >= 0.0) || !isfinite(c0)) return set_error(LJMD_EINVAL, "c0 = %g must be >= 0", c0);
  if (!(rho0 > 0.0) || !isfinite(rho0)) return set_error(LJMD_EINVAL, "rho0 = %g must be > 0", rho0);
  if (maxn < 1) return set_error(LJMD_EINVAL, "maxn = %d must be >= 1", maxn);
  if (n > 0 && (!x || !nbr || !nnbr)) return set_error(LJMD_EINVAL, "x/nbr/nnbr is NULL");
  return LJMD_OK;
}

int ljmd_sph_density(const ljmd_box *box, double h, double mass, double c0, double rho0, int64_t n,
                     const double *x, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                     double *rho, double *u_total, void *ws, size_t ws_bytes, void *stream) {
  LJMD_TRY(check_sph(box, h, mass, c0, rho0, n, x, nbr, nnbr, maxn));
  if (n > 0 && !rho) return set_error(LJMD_EINVAL, "rho is NULL");
  LJMD_TRY(check_ws(ws, ws_bytes, u_total ? sph_workspace(n) : 0));
  return launch_sph_density(make_box(box), h, mass, c0, rho0, n, x, nbr, nnbr, maxn, rho, u_total,
                            ws, (hipStream_t)stream);
}

int ljmd_sph_accel(const ljmd_box *box, double h, double mass, double c0, double rho0, int64_t n,
                   const double *x, const double *rho, const int32_t *nbr, const int32_t *nnbr,
                   int32_t maxn, double *acc, void *ws, size_t ws_bytes, void *stream) {
  LJMD_TRY(check_sph(box, h, mass, c0, rho0, n, x, nbr, nnbr, maxn));
  if (n > 0 && (!rho || !acc)) return set_error(LJMD_EINVAL, "rho/acc is NULL");
  LJMD_TRY(check_ws(ws, ws_bytes, n > 0 ? sph_workspace(n) : 0));
  if (n > 0 && ((uintptr_t)ws & 31u) != 0)
    return set_error(LJMD_EINVAL, "ws must be aligned to 32 bytes");
  return launch_sph_accel(make_box(box), h, mass, c0, rho0, n, x, rho, nbr, nnbr, maxn, acc, 0.0,
                          nullptr, nullptr, ws, (hipStream_t)stream);
}

int ljmd_sph_accel_step(const ljmd_box *box, double h, double mass, double c0, double rho0,
                        int64_t n, double *x, double *v, const double *rho, const int32_t *nbr,
                        const int32_t *nnbr, int32_t maxn, double dt, double *acc, void *ws,
                        size_t ws_bytes, void *stream) {
  LJMD_TRY(check_sph(box, h, mass, c0, rho0, n, x, nbr, nnbr, maxn));
  if (n > 0 && (!rho || !v)) return set_error(LJMD_EINVAL, "rho/v is NULL");
  if (!isfinite(dt) || dt == 0.0) return set_error(LJMD_EINVAL, "dt = %g", dt);
  LJMD_TRY(check_ws(ws, ws_bytes, n > 0 ? sph_workspace(n) : 0));
  if (n > 0 && ((uintptr_t)ws & 31u) != 0)
    return set_error(LJMD_EINVAL, "ws must be aligned to 32 bytes");
  return launch_sph_accel(make_box(box), h, mass, c0, rho0, n, x, rho, nbr, nnbr, maxn, acc, dt,
                          n > 0 ? v : nullptr, x, ws, (hipStream_t)stream);
}

int ljmd_ewald_real(const ljmd_box *box, double alpha, double rc, int64_t n, const double *x,
                    const double *q, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                    double *F, double *e_total, int accumulate, void *ws, size_t ws_bytes,
                    void *stream) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_cutoff(box, rc, "rc"));
  LJMD_TRY(check_n(n));
  if (!(alpha > 0.0) || !isfinite(alpha)) return set_error(LJMD_EINVAL, "alpha = %g must be > 0", alpha);
  if (maxn < 1) return set_error(LJMD_EINVAL, "maxn = %d must be >= 1", maxn);
  if (accumulate != 0 && accumulate != 1)
    return set_error(LJMD_EINVAL, "accumulate = %d must be 0 or 1", accumulate);
  if (n > 0 && (!x || !q || !nbr || !nnbr || !F))
    return set_error(LJMD_EINVAL, "x/q/nbr/nnbr/F is NULL");
  LJMD_TRY(check_ws(ws, ws_bytes, ewald_real_workspace(n)));
  if (((uintptr_t)ws & 31u) != 0) return set_error(LJMD_EINVAL, "ws must be aligned to 32 bytes");
  return launch_ewald_real(make_box(box), alpha, rc, n, x, q, nbr, nnbr, maxn, F, e_total,
                           accumulate, ws, (hipStream_t)stream);
}

int ljmd_spme_recip(const ljmd_box *box, double alpha, int32_t order, const int32_t K[3],
                    int64_t n, const double *x, const double *q, double *F, double *e_total,
                    int accumulate, void *ws, size_t ws_bytes, void *stream) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_n(n));
  if (!(alpha > 0.0) || !isfinite(alpha)) return set_error(LJMD_EINVAL, "alpha = %g must be > 0", alpha);
  if (order != 4 && order != 6 && order != 8)
    return set_error(LJMD_EINVAL, "order = %d must be 4, 6 or 8", order);
  if (!K) return set_error(LJMD_EINVAL, "K is NULL");
  for (int d = 0; d < 3; ++d)
    if (K[d] < 8 || K[d] > LJMD_SPME_MAX_GRID || (K[d] & (K[d] - 1)) != 0)
      return set_error(LJMD_EINVAL, "K[%d] = %d must be a power of two in [8, %d]", d, K[d],
                       LJMD_SPME_MAX_GRID);
  if (accumulate != 0 && accumulate != 1)
    return set_error(LJMD_EINVAL, "accumulate = %d must be 0 or 1", accumulate);
  if (n > 0 && (!x || !q || !F)) return set_error(LJMD_EINVAL, "x/q/F is NULL");
  const int64_t npts = (int64_t)K[0] * K[1] * K[2];
  LJMD_TRY(check_ws(ws, ws_bytes, spme_workspace(n, npts)));
  if (((uintptr_t)ws & 31u) != 0) return set_error(LJMD_EINVAL, "ws must be aligned to 32 bytes");
  return launch_spme_recip(make_box(box), alpha, order, K, n, x, q, F, e_total, accumulate, ws,
                           (hipStream_t)stream);
}

int ljmd_list_to_csr(int64_t n, const int32_t *nbr, const int32_t *nnbr, int32_t maxn,
                     int64_t *offsets, int32_t *csr, int64_t cap, void *ws, size_t ws_bytes,
                     void *stream) {
  LJMD_TRY(check_n(n));
  if (maxn < 1) return set_error(LJMD_EINVAL, "maxn = %d must be >= 1", maxn);
  if (cap < 0) return set_error(LJMD_EINVAL, "cap = %lld must be >= 0", (long long)cap);
  if (!offsets) return set_error(LJMD_EINVAL, "offsets is NULL");
  if (n > 0 && (!nbr || !nnbr)) return set_error(LJMD_EINVAL, "nbr/nnbr is NULL");
  if (cap > 0 && !csr) return set_error(LJMD_EINVAL, "csr is NULL with cap > 0");
  LJMD_TRY(check_ws(ws, ws_bytes, csr_workspace(n)));
  return launch_list_to_csr(n, nbr, nnbr, maxn, offsets, csr, cap, ws, (hipStream_t)stream);
}

int ljmd_compute_forces_csr(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                            const double *eps_packed, const double *sigma_packed, int64_t n,
                            const double *x, const int32_t *type, const int64_t *offsets,
                            const int32_t *csr, int32_t team, double *F, double *e_atom,
                            double *ev, void *ws, size_t ws_bytes, void *stream) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_cutoff(box, rc, "rc"));
  LJMD_TRY(check_n(n));
  if (precision != LJMD_FP64 && precision != LJMD_MIXED)
    return set_error(LJMD_EINVAL, "bad precision %d", precision);
  if (team != 1 && team != 2 && team != 4 && team != 8 && team != 16)
    return set_error(LJMD_EINVAL, "team = %d must be 1, 2, 4, 8 or 16", team);
  LJMD_TRY(check_params(ntypes, eps_packed, sigma_packed, type, n));
  if (n > 0 && (!x || !offsets || !csr || !F))
    return set_error(LJMD_EINVAL, "x/offsets/csr/F is NULL");
  const bool want_ev = ev != nullptr || e_atom != nullptr;
  LJMD_TRY(check_ws(ws, ws_bytes, want_ev ? csr_force_workspace(n) : 0));
  return launch_forces_csr(make_box(box), precision, rc, ntypes, eps_packed, sigma_packed, n, x,
                           type, offsets, csr, team, F, e_atom, ev, ws, (hipStream_t)stream);
}

int ljmd_integrate(int stage, double dt, double mass, const ljmd_box *box, int64_t n,
                   double *x, double *v, const double *F, double *ke, void *ws,
                   size_t ws_bytes, void *stream) {
  LJMD_TRY(check_n(n));
  if (stage != LJMD_KICK_DRIFT && stage != LJMD_KICK && stage != LJMD_KINETIC &&
      stage != LJMD_KICK_KICK_DRIFT)
    return set_error(LJMD_EINVAL, "bad stage %d", stage);
  if (stage == LJMD_KINETIC) {
    if (!ke) return set_error(LJMD_EINVAL, "ke is NULL for the kinetic-energy stage");
    if (n > 0 && !v) return set_error(LJMD_EINVAL, "v is NULL");
  } else if (!isfinite(dt) || dt == 0.0) {
    return set_error(LJMD_EINVAL, "dt = %g", dt);
  }
  if (!(mass > 0.0) || !isfinite(mass)) return set_error(LJMD_EINVAL, "mass = %g", mass);
  const bool drift = stage == LJMD_KICK_DRIFT || stage == LJMD_KICK_KICK_DRIFT;
  if (drift) LJMD_TRY(check_box(box));
  if (n > 0 && stage != LJMD_KINETIC && (!v || !F || (drift && !x)))
    return set_error(LJMD_EINVAL, "x/v/F is NULL");
  if (ke) LJMD_TRY(check_ws(ws, ws_bytes, stream_workspace(n)));
  BoxK b = drift ? make_box(box) : BoxK{};
  return launch_integrate(stage, dt, mass, b, n, x, v, F, ke, ws, (hipStream_t)stream);
}

int ljmd_md_step(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                 const double *eps_packed, const double *sigma_packed, int64_t n,
                 const double *x, const int32_t *type, const int32_t *nbr, const int32_t *nnbr,
                 int32_t maxn, double dt, double mass, double *v, double *x_next, int open_next,
                 double *F, double *e_atom, double *ev, void *ws, size_t ws_bytes, void *stream) {
  LJMD_TRY(check_md_step(box, precision, rc, ntypes, eps_packed, sigma_packed, n, x, type, nbr,
                         nnbr, maxn, dt, mass, v, x_next, open_next));
  if (!ev) return set_error(LJMD_EINVAL, "ev is NULL");
  LJMD_TRY(check_ws(ws, ws_bytes, force_workspace(n)));
  return launch_md_step(make_box(box), precision, rc, ntypes, eps_packed, sigma_packed, n, x, type,
                        nbr, nnbr, maxn, dt, mass, v, x_next, open_next, F, e_atom, ev,
                        (double *)ws, nullptr, nullptr, (hipStream_t)stream);
}

int ljmd_md_step_noalloc(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                         const double *eps_packed, const double *sigma_packed, int64_t n,
                         const double *x, const int32_t *type, const int32_t *nbr,
                         const int32_t *nnbr, int32_t maxn, double dt, double mass, double *v,
                         double *x_next, int open_next, double *F, double *e_atom, double *ev,
                         void *stream) {
  LJMD_TRY(check_md_step(box, precision, rc, ntypes, eps_packed, sigma_packed, n, x, type, nbr,
                         nnbr, maxn, dt, mass, v, x_next, open_next));
  if (!ev) return set_error(LJMD_EINVAL, "ev is NULL");
  if (force_workspace(n) > kScratchBytes)
    return set_error(LJMD_EWORKSPACE,
                     "n = %lld needs %zu bytes of step scratch; the static scratch holds %zu "
                     "(at most %lld atoms): use ljmd_md_step with a workspace",
                     (long long)n, force_workspace(n), kScratchBytes,
                     (long long)(kScratchBytes / force_workspace(1)) * force_workspace_atoms());
  void *rows = nullptr;
  LJMD_TRY(scratch_address(&rows));
  return launch_md_step(make_box(box), precision, rc, ntypes, eps_packed, sigma_packed, n, x, type,
                        nbr, nnbr, maxn, dt, mass, v, x_next, open_next, F, e_atom, ev,
                        (double *)rows, nullptr, nullptr, (hipStream_t)stream);
}

int ljmd_md_step_chained(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                         const double *eps_packed, const double *sigma_packed, int64_t n,
                         const double *x, const int32_t *type, const int32_t *nbr,
                         const int32_t *nnbr, int32_t maxn, double dt, double mass, double *v,
                         double *x_next, int open_next, double *F, double *e_atom, int half,
                         double *ev_prev, void *ws, size_t ws_bytes, void *stream) {
  LJMD_TRY(check_md_step(box, precision, rc, ntypes, eps_packed, sigma_packed, n, x, type, nbr,
                         nnbr, maxn, dt, mass, v, x_next, open_next));
  if (half != 0 && half != 1) return set_error(LJMD_EINVAL, "half = %d must be 0 or 1", half);
  LJMD_TRY(check_ws(ws, ws_bytes, 2 * force_workspace(n)));
  double *rows = (double *)ws;
  const size_t h = force_workspace(n) / sizeof(double);
  return launch_md_step(make_box(box), precision, rc, ntypes, eps_packed, sigma_packed, n, x, type,
                        nbr, nnbr, maxn, dt, mass, v, x_next, open_next, F, e_atom, nullptr,
                        rows + half * h, rows + (1 - half) * h, ev_prev, (hipStream_t)stream);
}

int ljmd_md_step_sums(int64_t n, int half, const void *ws, size_t ws_bytes, double *ev,
                      void *stream) {
  LJMD_TRY(check_n(n));
  if (half != 0 && half != 1) return set_error(LJMD_EINVAL, "half = %d must be 0 or 1", half);
  if (!ev) return set_error(LJMD_EINVAL, "ev is NULL");
  LJMD_TRY(check_ws(const_cast<void *>(ws), ws_bytes, 2 * force_workspace(n)));
  const size_t h = force_workspace(n) / sizeof(double);
  return launch_md_step_sums(n, (const double *)ws + half * h, ev, (hipStream_t)stream);
}

int ljmd_force_backward(const ljmd_box *box, int precision, double rc, int32_t ntypes,
                        const double *eps_packed, const double *sigma_packed, int64_t n,
                        const double *x, const int32_t *type, const int32_t *nbr,
                        const int32_t *nnbr, int32_t maxn, const double *g, double *gx,
                        double *geps, double *gsigma, int accumulate, void *ws,
                        size_t ws_bytes, void *stream) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_cutoff(box, rc, "rc"));
  LJMD_TRY(check_n(n));
  if (precision != LJMD_FP64 && precision != LJMD_MIXED)
    return set_error(LJMD_EINVAL, "bad precision %d", precision);
  LJMD_TRY(check_params(ntypes, eps_packed, sigma_packed, type, n));
  if (maxn < 1) return set_error(LJMD_EINVAL, "maxn = %d must be >= 1", maxn);
  if (!geps || !gsigma) return set_error(LJMD_EINVAL, "geps/gsigma is NULL");
  if (n > 0 && (!x || !nbr || !nnbr || !g || !gx))
    return set_error(LJMD_EINVAL, "x/nbr/nnbr/g/gx is NULL");
  if (accumulate != 0 && accumulate != 1)
    return set_error(LJMD_EINVAL, "accumulate = %d must be 0 or 1", accumulate);
  LJMD_TRY(check_ws(ws, ws_bytes, bwd_workspace(n, ntypes)));
  return launch_backward(make_box(box), precision, rc, ntypes, eps_packed, sigma_packed, n, x,
                         type, nbr, nnbr, maxn, g, gx, geps, gsigma, accumulate, ws,
                         (hipStream_t)stream);
}

int ljmd_adjoint_kick(int64_t n, double dt, double w, const double *xbar, double *vbar,
                      double *g, void *stream) {
  LJMD_TRY(check_n(n));
  if (!isfinite(dt) || !isfinite(w)) return set_error(LJMD_EINVAL, "dt/w not finite");
  if (n > 0 && (!xbar || !vbar || !g)) return set_error(LJMD_EINVAL, "xbar/vbar/g is NULL");
  return launch_adjoint_kick(n, dt, w, xbar, vbar, g, (hipStream_t)stream);
}

int ljmd_max_displacement(const ljmd_box *box, int64_t n, const double *x, const double *x_ref,
                          double *max_d2, void *ws, size_t ws_bytes, void *stream) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_n(n));
  if (!max_d2) return set_error(LJMD_EINVAL, "max_d2 is NULL");
  if (n > 0 && (!x || !x_ref)) return set_error(LJMD_EINVAL, "x/x_ref is NULL");
  if (n > 0 && x == x_ref) return set_error(LJMD_EINVAL, "x_ref must not alias x");
  LJMD_TRY(check_ws(ws, ws_bytes, stream_workspace(n)));
  return launch_max_displacement(make_box(box), n, x, x_ref, max_d2, ws, (hipStream_t)stream);
}

int ljmd_traj_loss(const ljmd_box *box, int64_t n, const double *x, const double *xref,
                   double *xbar, double *loss, void *ws, size_t ws_bytes, void *stream) {
  LJMD_TRY(check_box(box));
  LJMD_TRY(check_n(n));
  if (!loss) return set_error(LJMD_EINVAL, "loss is NULL");
  if (n > 0 && (!x || !xref || !xbar)) return set_error(LJMD_EINVAL, "x/xref/xbar is NULL");
  LJMD_TRY(check_ws(ws, ws_bytes, stream_workspace(n)));
  return launch_loss(make_box(box), n, x, xref, xbar, loss, ws, (hipStream_t)stream);
}

int ljmd_scatter_rows(int64_t n, int32_t width, const int64_t *id, const double *src,
                      double *dst, void *stream) {
  LJMD_TRY(check_n(n));
  if (width < 1 || width > 1024) return set_error(LJMD_EINVAL, "width = %d", width);
  if (n > 0 && (!id || !src || !dst)) return set_error(LJMD_EINVAL, "id/src/dst is NULL");
  return launch_scatter_rows(n, width, id, src, dst, (hipStream_t)stream);
}

int ljmd_gather_rows(int64_t n, int32_t width, const int64_t *id, const double *src,
                     double *dst, void *stream) {
  LJMD_TRY(check_n(n));
  if (width < 1 || width > 1024) return set_error(LJMD_EINVAL, "width = %d", width);
  if (n > 0 && (!id || !src || !dst)) return set_error(LJMD_EINVAL, "id/src/dst is NULL");
  return launch_gather_rows(n, width, id, src, dst, (hipStream_t)stream);
}

}  // extern "C"
