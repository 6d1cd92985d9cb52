// dcf_api.hip -- host runtime behind the C ABI declared in include/dcf.h:
// argument validation, workspace carving, and the enqueue sequences of the
// forward step, the adjoint step and the checkpointed trajectory gradient.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dcf.h"
#include "dcf_adjoint.hpp"
#include "dcf_kernels.hpp"

using namespace dcf;

namespace {
thread_local std::string g_last_error;

dcf_status fail(dcf_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define DCF_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(DCF_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base((char *)b) {}
  template <class T> T *take(size_t count) {
    T *p = base ? (T *)(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

// Device addresses of `scratch` (below), one per device, resolved by
// dcf_create with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};
}  // namespace

// Workspace of dcf_rk3_step_noalloc: a fixed array in every device's copy of
// the code object, held from the first use of the library on a device until
// the process ends.  Host code never passes `scratch` itself to a kernel (on
// the host the name is only a stand-in): it uses the per-device address that
// hipGetSymbolAddress returned.
static __device__ __align__(256) unsigned char scratch[DCF_NOALLOC_SCRATCH_BYTES];

struct dcf_ctx {
  int device = 0;
  dcf_grid grid;
  dcf_gas gas;
  Dev g;
  double *metric_mem = nullptr;
  int cost_face = -1;
  double cost_pref = 0.0;
  int nK = 0;
  // workspace
  void *ws = nullptr;
  size_t ws_bytes = 0;
  int ws_mode = -1;
  int ws_nsteps = 0, ws_seg = 0;
  double *U1 = nullptr, *U2 = nullptr, *part = nullptr, *force = nullptr;
  double *dtpart = nullptr;  // per-block signal rates of the last stage (fused CFL step)
  BoxOut qalt;               // second primitive box (fused stages alternate the two)
  AdjBuffers adj;
  double *ckpt = nullptr;  // gradient checkpoints
  double *seg = nullptr;   // per-segment recomputed states
  double *sst = nullptr;   // per-segment stage states U1, U2 of every step
  double *boxc = nullptr;  // mode 3: primitive boxes of every stage of a segment
  int box_arrays = 0;      // box arrays per cached stage
  double *lam_a = nullptr, *lam_b = nullptr, *gbuf = nullptr, *zero_dt = nullptr;
  Probe probe;  // dcf_probe_begin / dcf_probe_end
  // incremental gradient state (dcf_gradient_begin / advance / finish)
  struct {
    bool active = false;
    int phase = 0;   // 0 forward sweep, 1 segment recompute, 2 reverse steps, 3 done
    int n = 0;       // forward: steps taken; recompute: step within segment; reverse: step index
    int sgi = 0;     // current segment (reverse)
    int nsteps = 0, seg_len = 0;
    const double *dt = nullptr;
    double *J = nullptr, *dJdK = nullptr;
    double *lam = nullptr, *lam_prev = nullptr;
  } gr;
};

// Validates a grid and a gas and lays out the device-side description of a
// solve on them (sizes, strides, gas constants, boundaries all periodic; no
// device memory, no metric arrays yet).
static dcf_status describe(const dcf_grid *grid, const dcf_gas *gas, Dev &g) {
  if (grid->ndim < 1 || grid->ndim > 3) return fail(DCF_EINVAL, "ndim must be 1, 2 or 3");
  for (int d = 0; d < 3; ++d) {
    if (d < grid->ndim) {
      if (grid->n[d] < 3) return fail(DCF_EINVAL, "axis %d needs at least 3 cells", d);
      if (!(grid->hi[d] > grid->lo[d])) return fail(DCF_EINVAL, "axis %d: hi <= lo", d);
      if (grid->stretch[d] < 0 || grid->stretch[d] > 2)
        return fail(DCF_EINVAL, "axis %d: unknown stretching", d);
      if (grid->stretch[d] != 0 && !(grid->beta[d] > 0.0))
        return fail(DCF_EINVAL, "axis %d: stretching needs beta > 0", d);
    } else if (grid->n[d] != 1) {
      return fail(DCF_EINVAL, "unused axis %d must have n = 1", d);
    }
  }
  if (!(gas->gamma > 1.0) || !(gas->R > 0.0))
    return fail(DCF_EINVAL, "gas needs gamma > 1 and R > 0");
  if (gas->visc_law < 0 || gas->visc_law > 2) return fail(DCF_EINVAL, "unknown viscosity law");
  if (gas->visc_law != 0 && (!(gas->Pr > 0.0) || !(gas->T_ref > 0.0) || gas->mu_ref < 0.0))
    return fail(DCF_EINVAL, "viscous gas needs Pr > 0, T_ref > 0, mu_ref >= 0");
  long ncell = (long)grid->n[0] * grid->n[1] * grid->n[2];
  long nboxc = 1;
  for (int d = 0; d < 3; ++d) nboxc *= grid->n[d] + (d < grid->ndim ? 2 * NH : 0);
  // kernels index cells with 32-bit thread indices
  if (ncell > (1L << 31) - 1 || nboxc > (1L << 32) - 1)
    return fail(DCF_EINVAL, "grid too large");

  memset(&g, 0, sizeof g);
  g.ndim = grid->ndim;
  g.nv = grid->ndim + 2;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = grid->n[d];
    g.h[d] = d < grid->ndim ? NH : 0;
    g.N[d] = g.n[d] + 2 * g.h[d];
  }
  g.ncell = ncell;
  g.nbox = (long)g.N[0] * g.N[1] * g.N[2];
  g.ho[0] = 16;
  g.ho[1] = g.h[1];
  g.ho[2] = g.h[2];
  const long pitch = ((long)g.ho[0] + g.n[0] + g.h[0] + 15) / 16 * 16;
  g.sb[0] = 1;
  g.sb[1] = pitch;
  g.sb[2] = pitch * g.N[1];
  g.nboxp = pitch * g.N[1] * g.N[2];
  for (int D = 0; D < 3; ++D) {
    for (int e = 0; e < 3; ++e) g.fn[D][e] = g.n[e] + (e == D ? 1 : 0);
    g.fcount[D] = (long)g.fn[D][0] * g.fn[D][1] * g.fn[D][2];
  }
  g.gamma = gas->gamma;
  g.R = gas->R;
  g.Pr = gas->Pr;
  g.cp = gas->gamma * gas->R / (gas->gamma - 1.0);
  g.gm1i = 1.0 / (gas->gamma - 1.0);
  g.cpPr = g.cp / gas->Pr;
  g.iR = 1.0 / gas->R;
  g.mu_ref = gas->mu_ref;
  g.T_ref = gas->T_ref;
  g.iTref = 1.0 / gas->T_ref;
  g.vparam = gas->visc_param;
  g.visc = gas->visc_law;
  for (int f = 0; f < 6; ++f) {
    g.bck[f] = BC_PERIODIC;
    g.doff[f] = -1;
  }
  g.pface = -1;
  g.source = SRC_NONE;

  return DCF_OK;
}

extern "C" {

const char *dcf_last_error(void) { return g_last_error.c_str(); }

dcf_status dcf_create(const dcf_grid *grid, const dcf_gas *gas, dcf_ctx **out) {
  if (!grid || !gas || !out) return fail(DCF_EINVAL, "dcf_create: null argument");
  *out = nullptr;
  Dev g0;
  dcf_status st0 = describe(grid, gas, g0);
  if (st0) return st0;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= kMaxDevices)
    return fail(DCF_EDEVICE, "no usable current device");
  {
    // the static scratch of dcf_rk3_step_noalloc: its address on this device,
    // taken once per device with the device current
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
      void *ptr = nullptr;
      const hipError_t es = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (es != hipSuccess || !ptr)
        return fail(DCF_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(es));
      g_scratch_addr[device] = ptr;
    }
  }
  dcf_ctx *c = new (std::nothrow) dcf_ctx();
  if (!c) return fail(DCF_ENOMEM, "host allocation failed");
  c->device = device;
  c->grid = *grid;
  c->gas = *gas;
  Dev &g = c->g;
  g = g0;
  size_t total = 0;
  for (int d = 0; d < 3; ++d) total += 5 * (size_t)(g.n[d] + 1);
  // (one more double: the x line length, computed once on the device)
  hipError_t e = hipMalloc((void **)&c->metric_mem, (total + 1) * sizeof(double));
  if (e != hipSuccess) {
    delete c;
    return fail(DCF_EDEVICE, "hipMalloc(metrics): %s", hipGetErrorString(e));
  }
  double *p = c->metric_mem;
  for (int d = 0; d < 3; ++d) {
    size_t m = g.n[d] + 1;
    g.dx[d] = p;
    g.idx[d] = p + m;
    g.mc[d] = p + 2 * m;
    g.mf[d] = p + 3 * m;
    g.xm[d] = p + 4 * m;
    double lo = grid->lo[d], hi = grid->hi[d];
    int kind = d < grid->ndim ? grid->stretch[d] : 0;
    if (d >= grid->ndim) {  // unused axis: unit width
      lo = 0.0;
      hi = 1.0;
    }
    e = launch_metrics(kind, lo, hi, grid->beta[d], g.n[d], (double *)g.dx[d], (double *)g.idx[d],
                       (double *)g.mc[d], (double *)g.mf[d], (double *)g.xm[d], 0);
    if (e == hipSuccess) e = hipStreamSynchronize(0);
    if (e != hipSuccess) {
      (void)hipFree(c->metric_mem);
      delete c;
      return fail(DCF_EDEVICE, "metrics kernel: %s", hipGetErrorString(e));
    }
    p += 5 * m;
  }
  // the body force's volume term reads the x line length; summed once here in
  // the order the reductions used to sum it per line
  e = launch_line_length(g.dx[0], g.n[0], c->metric_mem + total, 0);
  if (e == hipSuccess) e = hipMemcpy(&g.Lx, c->metric_mem + total, sizeof(double),
                                     hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    (void)hipFree(c->metric_mem);
    delete c;
    return fail(DCF_EDEVICE, "line length: %s", hipGetErrorString(e));
  }
  *out = c;
  return DCF_OK;
}

dcf_status dcf_destroy(dcf_ctx *c) {
  if (!c) return DCF_OK;
  (void)hipDeviceSynchronize();
  if (c->metric_mem) (void)hipFree(c->metric_mem);
  if (c->probe.ev) {
    for (int i = 0; i < 2 * c->probe.cap; ++i) (void)hipEventDestroy(c->probe.ev[i]);
    delete[] c->probe.ev;
  }
  delete c;
  return DCF_OK;
}

dcf_status dcf_state_info(const dcf_ctx *c, int *nv, long *ncell, size_t *bytes) {
  if (!c) return fail(DCF_EINVAL, "null context");
  if (nv) *nv = c->g.nv;
  if (ncell) *ncell = c->g.ncell;
  if (bytes) *bytes = sizeof(double) * (size_t)c->g.nv * c->g.ncell;
  return DCF_OK;
}

int dcf_num_params(const dcf_ctx *c) { return c ? c->nK : 0; }

}  // extern "C"

// Lays the workspace out (or only measures it when base == nullptr).
static size_t carve(dcf_ctx *c, void *base, int mode, int nsteps, int seg_len) {
  Carver cv(base);
  Dev &g = c->g;
  const long nbox = g.nboxp, ncell = g.ncell, nv = g.nv;
  for (int q = 0; q < NQ; ++q) g.Q[q] = cv.take<double>(nbox);
  for (int D = 0; D < 3; ++D) g.F[D] = D < g.ndim ? cv.take<double>(5 * g.fcount[D]) : nullptr;
  c->U1 = cv.take<double>(nv * ncell);
  c->U2 = cv.take<double>(nv * ncell);
  c->part = cv.take<double>(8 * RED_BLOCKS);
  c->force = cv.take<double>(4);
  c->dtpart = cv.take<double>(std::max(update_blocks(g), flux_update_blocks(g)));
  g.flags = cv.take<unsigned>(64);
  for (int q = 0; q < NQ; ++q) c->qalt.Q[q] = g.ndim >= 2 ? cv.take<double>(nbox) : nullptr;
  if (mode >= 1) carve_adjoint(cv, g, c->adj);
  if (mode >= 2) {
    int nseg = (nsteps + seg_len - 1) / seg_len;
    c->ckpt = cv.take<double>((size_t)nseg * nv * ncell);
    c->seg = cv.take<double>((size_t)(seg_len + 1) * nv * ncell);
    c->sst = cv.take<double>((size_t)2 * seg_len * nv * ncell);
    c->lam_a = cv.take<double>(nv * ncell);
    c->lam_b = cv.take<double>(nv * ncell);
    c->gbuf = cv.take<double>(nv * ncell);
  }
  c->boxc = nullptr;
  c->box_arrays = 0;
  if (mode >= 3) {
    c->box_arrays = NQ;
    c->boxc = cv.take<double>((size_t)3 * seg_len * NQ * nbox);
  }
  return cv.off;
}

extern "C" {

dcf_status dcf_workspace_size(const dcf_ctx *c, int mode, int nsteps, int seg_len,
                              size_t *bytes) {
  if (!c || !bytes) return fail(DCF_EINVAL, "null argument");
  if (mode < 0 || mode > 3) return fail(DCF_EINVAL, "mode must be 0, 1, 2 or 3");
  if (mode >= 2 && (nsteps < 1 || seg_len < 1))
    return fail(DCF_EINVAL, "gradient workspace needs nsteps >= 1 and seg_len >= 1");
  dcf_ctx tmp = *c;
  *bytes = carve(&tmp, nullptr, mode, nsteps, seg_len);
  return DCF_OK;
}

dcf_status dcf_workspace_size_for(const dcf_grid *grid, const dcf_gas *gas, int mode,
                                  int nsteps, int seg_len, size_t *bytes) {
  if (!grid || !gas || !bytes) return fail(DCF_EINVAL, "null argument");
  if (mode < 0 || mode > 3) return fail(DCF_EINVAL, "mode must be 0, 1, 2 or 3");
  if (mode >= 2 && (nsteps < 1 || seg_len < 1))
    return fail(DCF_EINVAL, "gradient workspace needs nsteps >= 1 and seg_len >= 1");
  dcf_ctx tmp = dcf_ctx();  // host-side description only
  dcf_status s = describe(grid, gas, tmp.g);
  if (s) return s;
  *bytes = carve(&tmp, nullptr, mode, nsteps, seg_len);
  return DCF_OK;
}

dcf_status dcf_set_workspace(dcf_ctx *c, int mode, int nsteps, int seg_len, void *dev,
                             size_t bytes) {
  if (!c || !dev) return fail(DCF_EINVAL, "null argument");
  if (((uintptr_t)dev) & 255) return fail(DCF_EINVAL, "workspace must be 256-byte aligned");
  if (mode < 0 || mode > 3) return fail(DCF_EINVAL, "mode must be 0, 1, 2 or 3");
  if (mode >= 2 && (nsteps < 1 || seg_len < 1))
    return fail(DCF_EINVAL, "gradient workspace needs nsteps >= 1 and seg_len >= 1");
  dcf_ctx tmp = *c;
  size_t need = carve(&tmp, nullptr, mode, nsteps, seg_len);
  if (need > bytes) return fail(DCF_ENOMEM, "workspace needs %zu bytes, got %zu", need, bytes);
  carve(c, dev, mode, nsteps, seg_len);
  DCF_HIP(hipMemset(c->g.flags, 0, 64 * sizeof(unsigned)));
  // the adjoint boxes start at zero; the reverse kernels keep every cell no
  // stage writes at zero from then on
  if (mode >= 1) DCF_HIP(hipMemset(c->adj.zero_begin, 0, c->adj.zero_count * sizeof(double)));
  DCF_HIP(hipStreamSynchronize(nullptr));  // done before work on any stream can use them
  c->ws = dev;
  c->ws_bytes = bytes;
  c->ws_mode = mode;
  c->ws_nsteps = mode >= 2 ? nsteps : 0;
  c->ws_seg = mode >= 2 ? seg_len : 0;
  return DCF_OK;
}

dcf_status dcf_set_bc(dcf_ctx *c, int face, const dcf_bc *bc) {
  if (!c || !bc) return fail(DCF_EINVAL, "null argument");
  if (face < 0 || face > 5) return fail(DCF_EINVAL, "face must be 0..5");
  int d = face / 2;
  if (d >= c->g.ndim) return fail(DCF_EINVAL, "face %d is on an unused axis", face);
  if (bc->kind < 0 || bc->kind > 5) return fail(DCF_EINVAL, "unknown boundary kind");
  Dev &g = c->g;
  if (is_wall(bc->kind)) {
    if (!(bc->T_wall >= 0.0) || bc->T_wall > 1e300)
      return fail(DCF_EINVAL, "wall needs T_wall > 0 (isothermal) or 0 (adiabatic)");
  }

  if (bc->kind == BC_DIRICHLET && !bc->dirichlet)
    return fail(DCF_EINVAL, "Dirichlet face needs a profile");
  if (bc->kind == BC_POROUS) {
    if (g.pface >= 0 && g.pface != face) return fail(DCF_EUNSUPPORTED, "only one porous face");
    int t1 = tan1(d);
    int nt1 = g.n[t1];
    if (bc->porous_begin < 0 || bc->porous_end > nt1 || bc->porous_begin >= bc->porous_end)
      return fail(DCF_EINVAL, "porous strip [%d,%d) outside [0,%d)", bc->porous_begin,
                  bc->porous_end, nt1);
    if (!(bc->p_inf > 0.0)) return fail(DCF_EINVAL, "porous wall needs p_inf > 0");
    g.pface = face;
    g.pb = bc->porous_begin;
    g.pe = bc->porous_end;
    g.pinf = bc->p_inf;
  } else if (g.pface == face) {
    g.pface = -1;
  }
  g.bck[face] = bc->kind;
  g.Tw[face] = is_wall(bc->kind) ? bc->T_wall : 0.0;
  g.dir[face] = bc->dirichlet;
  // boundary-parameter layout: porous K_i first, then (A, kappa) of each
  // disturbance face in face order
  int nk = g.pface >= 0 ? (g.pe - g.pb) * g.n[tan2(g.pface / 2)] : 0;
  for (int f = 0; f < 6; ++f) {
    g.doff[f] = -1;
    if (f / 2 < g.ndim && g.bck[f] == BC_DISTURB) {
      g.doff[f] = nk;
      nk += 2;
    }
  }
  if (nk != c->nK) g.K = nullptr;  // layout changed: parameters must be set again
  c->nK = nk;
  return DCF_OK;
}

dcf_status dcf_set_params(dcf_ctx *c, const double *K, int nK) {
  if (!c) return fail(DCF_EINVAL, "null context");
  if (nK != c->nK) return fail(DCF_EINVAL, "expected %d porous coefficients, got %d", c->nK, nK);
  if (nK > 0 && !K) return fail(DCF_EINVAL, "null K");
  c->g.K = K;
  return DCF_OK;
}

dcf_status dcf_set_scheme(dcf_ctx *c, int scheme) {
  if (!c) return fail(DCF_EINVAL, "null context");
  if (scheme != DCF_SCHEME_WENO5 && scheme != DCF_SCHEME_TENO6A)
    return fail(DCF_EINVAL, "unknown scheme %d", scheme);
  c->g.scheme = scheme == DCF_SCHEME_TENO6A ? SCHEME_TENO6A : SCHEME_WENO5;
  return DCF_OK;
}

dcf_status dcf_set_source(dcf_ctx *c, int kind) {
  if (!c) return fail(DCF_EINVAL, "null context");
  if (kind != SRC_NONE && kind != SRC_MASSFLUX) return fail(DCF_EINVAL, "unknown source");
  c->g.source = kind;
  return DCF_OK;
}

dcf_status dcf_set_cost(dcf_ctx *c, int face, double pref) {
  if (!c) return fail(DCF_EINVAL, "null context");
  if (face < -1 || face > 5 || (face >= 0 && face / 2 >= c->g.ndim))
    return fail(DCF_EINVAL, "bad cost face %d", face);
  c->cost_face = face;
  c->cost_pref = pref;
  return DCF_OK;
}

}  // extern "C"

// Checks that the context is complete before anything is enqueued
// (need_mode -1: no workspace needed).
static dcf_status ready(dcf_ctx *c, int need_mode) {
  if (!c) return fail(DCF_EINVAL, "null context");
  if (c->ws_mode < need_mode)
    return fail(DCF_ENOMEM, "workspace for mode %d not set (have mode %d)", need_mode, c->ws_mode);
  int dev = -1;
  (void)hipGetDevice(&dev);
  if (dev != c->device) return fail(DCF_EINVAL, "context belongs to device %d, current is %d",
                                    c->device, dev);
  const Dev &g = c->g;
  for (int d = 0; d < g.ndim; ++d) {
    bool p0 = g.bck[2 * d] == BC_PERIODIC, p1 = g.bck[2 * d + 1] == BC_PERIODIC;
    if (p0 != p1) return fail(DCF_EINVAL, "axis %d: periodic faces must come in pairs", d);
  }
  if (c->nK > 0 && !g.K)
    return fail(DCF_EINVAL, "boundary parameters not set (dcf_set_params)");
  return DCF_OK;
}

// One right-hand-side evaluation into the face-flux buffers (and the force).
static dcf_status eval_fluxes(dcf_ctx *c, const double *U, hipStream_t st) {
  Dev &g = c->g;
  DCF_HIP(launch_prim_halo(g, U, st));
  DCF_HIP(launch_fluxes(g, st));
  if (g.source == SRC_MASSFLUX) DCF_HIP(launch_force(g, c->part, c->force, st));
  return DCF_OK;
}

// One RK3 step in place; the stage states go to U1, U2 (default: scratch).
// The last direction's fluxes are fused into the stage update where there is
// no source term, or the constant-mass-flux source with a periodic last
// direction: the body force needs every boundary flux, and a periodic
// direction's boundary terms vanish, so the force is reduced from the other
// directions' fluxes before the fused kernel applies it.
static bool fused_stages(const dcf_ctx *c) {
  const Dev &g = c->g;
  if (g.ndim < 2) return false;
  if (g.source == SRC_NONE) return true;
  // the body force needs every boundary flux: only the last direction's can
  // be left to the fused kernel, and only where they cancel (periodic)
  const int f = 2 * (g.ndim - 1);
  return g.source == SRC_MASSFLUX && g.bck[f] == BC_PERIODIC && g.bck[f + 1] == BC_PERIODIC;
}

// A CFL step reduction left pending by the previous step (nparts partial
// maxima in dtpart): the next fused step runs it with its first ghost fill.
struct PendingDt {
  int nparts;
  double cfl, dt_max;
  double *dt;  // the step (also what the stages read)
};

// Fused steps chain their primitive boxes: stage k of a step works on box
// (base + k) & 1 (0: g.Q, 1: qalt).  With box_ready the interior of the
// first stage's box already holds the primitives of U (written by the
// previous step's last update), so only its ghosts are filled; with
// write_next the last update writes the primitives of the new state into
// box (base + 1) & 1, the first box of a following step with the other base.
// With pend (box_ready only) the first ghost fill also reduces the previous
// step's partial maxima into dt, before any stage reads it.  With nstages = 2
// only the stage states U1 and U2 are made (U is not written): the step's
// inner states exactly as the full step makes them.
static dcf_status rk3_stages(dcf_ctx *c, double *U, const double *dt, hipStream_t st,
                             double *U1 = nullptr, double *U2 = nullptr,
                             double *dtpart = nullptr, int base = 0, bool box_ready = false,
                             bool write_next = false, const PendingDt *pend = nullptr,
                             int nstages = 3) {
  Dev &g = c->g;
  if (!U1) U1 = c->U1;
  if (!U2) U2 = c->U2;
  if (fused_stages(c)) {
    const double *in[3] = {U, U1, U2};
    double *out[3] = {U1, U2, U};
    const double a[3] = {0.0, 0.75, 1.0 / 3.0}, b[3] = {1.0, 0.25, 2.0 / 3.0};
    // the stages' primitive boxes alternate between g.Q and qalt: each
    // stage's update also writes the interior of the next stage's box, which
    // then only needs its ghosts
    Dev gs[2] = {g, g};
    BoxOut bo[2];
    for (int q = 0; q < NQ; ++q) {
      gs[1].Q[q] = c->qalt.Q[q];
      bo[0].Q[q] = g.Q[q];
      bo[1].Q[q] = c->qalt.Q[q];
    }
    Probe &pr = c->probe;
    for (int k = 0; k < nstages; ++k) {
      const Dev &gk = gs[(base + k) & 1];
      if (k == 0 && !box_ready) {
        DCF_HIP(launch_prim_halo(gk, in[k], st));
      } else if (k == 0 && pend) {
        pr.before(8, st);
        DCF_HIP(launch_prim_ghost_dt(gk, c->dtpart, pend->nparts, pend->cfl, pend->dt_max,
                                     pend->dt, st));
        pr.after(8, st);
      } else {
        pr.before(8, st);
        DCF_HIP(launch_prim_ghost(gk, st));
        pr.after(8, st);
      }
      const bool next = k < 2 || write_next;
      DCF_HIP(launch_fluxes_update(gk, U, in[k], out[k], dt, a[k], b[k], k == 2 ? dtpart : nullptr,
                                   st, next ? bo[(base + k + 1) & 1] : BoxOut{}, c->part,
                                   g.source == SRC_MASSFLUX ? c->force : nullptr, &pr));
    }
    return DCF_OK;
  }
  dcf_status s;
  if ((s = eval_fluxes(c, U, st))) return s;
  DCF_HIP(launch_update(g, U, U, U1, nullptr, dt, 0.0, 1.0, c->force, st));
  if ((s = eval_fluxes(c, U1, st))) return s;
  DCF_HIP(launch_update(g, U, U1, U2, nullptr, dt, 0.75, 0.25, c->force, st));
  if (nstages < 3) return DCF_OK;
  if ((s = eval_fluxes(c, U2, st))) return s;
  DCF_HIP(launch_update(g, U, U2, U, nullptr, dt, 1.0 / 3.0, 2.0 / 3.0, c->force, st, dtpart));
  return DCF_OK;
}

extern "C" {

dcf_status dcf_init_state(dcf_ctx *c, const double *P, double *U, void *stream) {
  dcf_status s = ready(c, -1);
  if (s) return s;
  if (!P || !U) return fail(DCF_EINVAL, "null array");
  DCF_HIP(launch_init_state(c->g, P, U, (hipStream_t)stream));
  return DCF_OK;
}

dcf_status dcf_rhs(dcf_ctx *c, const double *U, double *R, void *stream) {
  dcf_status s = ready(c, 0);
  if (s) return s;
  if (!U || !R) return fail(DCF_EINVAL, "null array");
  hipStream_t st = (hipStream_t)stream;
  if ((s = eval_fluxes(c, U, st))) return s;
  DCF_HIP(launch_update(c->g, U, U, nullptr, R, nullptr, 0.0, 0.0, c->force, st));
  return DCF_OK;
}

dcf_status dcf_compute_dt(dcf_ctx *c, const double *U, double cfl, double dt_max, double *dt,
                          void *stream) {
  dcf_status s = ready(c, 0);
  if (s) return s;
  if (!U || !dt) return fail(DCF_EINVAL, "null array");
  if (!(cfl > 0.0)) return fail(DCF_EINVAL, "cfl must be > 0");
  if (!(dt_max > 0.0)) dt_max = 1.0e300;
  DCF_HIP(launch_dt(c->g, U, cfl, dt_max, c->part, dt, (hipStream_t)stream));
  return DCF_OK;
}

dcf_status dcf_rk3_step(dcf_ctx *c, double *U, const double *dt, void *stream) {
  dcf_status s = ready(c, 0);
  if (s) return s;
  if (!U || !dt) return fail(DCF_EINVAL, "null array");
  return rk3_stages(c, U, dt, (hipStream_t)stream);
}

dcf_status dcf_rk3_step_keep(dcf_ctx *c, double *U, const double *dt, double *stages,
                             void *stream) {
  dcf_status s = ready(c, 0);
  if (s) return s;
  if (!U || !dt || !stages) return fail(DCF_EINVAL, "null array");
  const long M = (long)c->g.nv * c->g.ncell;
  if (stages + 2 * M > U && U + M > stages)
    return fail(DCF_EINVAL, "the stage states may not overlap U");
  return rk3_stages(c, U, dt, (hipStream_t)stream, stages, stages + M);
}

dcf_status dcf_rk3_step_noalloc(dcf_ctx *c, double *U, const double *dt, unsigned *flags,
                                void *stream) {
  dcf_status s = ready(c, -1);
  if (s) return s;
  if (!U || !dt) return fail(DCF_EINVAL, "null array");
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch_addr[c->device];
  }
  if (!base) return fail(DCF_EDEVICE, "static scratch not resolved on device %d", c->device);
  // the forward workspace laid out over the scratch, in a copy of the
  // context: the caller's own workspace (if any) is left alone
  dcf_ctx tmp = *c;
  tmp.probe = Probe{};
  tmp.gr.active = false;
  const size_t need = carve(&tmp, nullptr, 0, 0, 0);
  if (need > DCF_NOALLOC_SCRATCH_BYTES)
    return fail(DCF_EBUDGET, "the step needs %zu bytes of scratch, the static scratch holds %zu",
                need, (size_t)DCF_NOALLOC_SCRATCH_BYTES);
  carve(&tmp, base, 0, 0, 0);
  // every scratch buffer is written before it is read within the step; the
  // flag word only collects bits (into the caller's word when given)
  if (flags) tmp.g.flags = flags;
  return rk3_stages(&tmp, U, dt, (hipStream_t)stream);
}

dcf_status dcf_batch_table_bytes(int n, size_t *bytes) {
  if (n < 1 || !bytes) return fail(DCF_EINVAL, "need n >= 1 and a result pointer");
  *bytes = (size_t)n * sizeof(BatchEntry);
  return DCF_OK;
}

// Validates a batch and writes its table entries into h (host memory of at
// least n entries).
static dcf_status batch_fill(dcf_ctx *const *ctxs, double *const *U, double *const *dt, int n,
                             BatchEntry *h) {
  for (int i = 0; i < n; ++i) {
    dcf_ctx *c = ctxs[i];
    dcf_status s = ready(c, 0);
    if (s) return s;
    if (!U[i] || !dt[i]) return fail(DCF_EINVAL, "null state or step of solve %d", i);
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(DCF_EINVAL, "context of solve %d repeats solve %d", i, j);
    const Dev &g = c->g;
    if (g.ndim != ctxs[0]->g.ndim || (g.visc != VISC_NONE) != (ctxs[0]->g.visc != VISC_NONE))
      return fail(DCF_EUNSUPPORTED, "solve %d: a batch needs one dimension and viscous flag", i);
    if (g.source != SRC_NONE)
      return fail(DCF_EUNSUPPORTED, "solve %d: source terms are not batched", i);
    if (g.scheme != SCHEME_WENO5)
      return fail(DCF_EUNSUPPORTED, "solve %d: batched steps are of the WENO5-JS scheme", i);
    BatchEntry e;
    e.g = g;
    e.gb = g;
    if (g.ndim >= 2)
      for (int q = 0; q < NQ; ++q) e.gb.Q[q] = c->qalt.Q[q];
    e.U = U[i];
    e.U1 = c->U1;
    e.U2 = c->U2;
    e.dt = dt[i];
    e.part = c->part;
    batch_entry_sizes(e);
    memcpy(&h[i], &e, sizeof e);
  }
  return DCF_OK;
}

dcf_status dcf_batch_rk3_step(dcf_ctx *const *ctxs, double *const *U, double *const *dt, int n,
                              double cfl, void *table, size_t table_bytes, void *stream) {
  if (n < 1 || !ctxs || !U || !dt || !table) return fail(DCF_EINVAL, "null argument or n < 1");
  if (table_bytes < (size_t)n * sizeof(BatchEntry))
    return fail(DCF_EINVAL, "table needs %zu bytes, got %zu", (size_t)n * sizeof(BatchEntry),
                table_bytes);
  if (((uintptr_t)table) & 15) return fail(DCF_EINVAL, "table must be 16-byte aligned");
  static thread_local std::vector<BatchEntry> h;
  h.resize(n);
  dcf_status s = batch_fill(ctxs, U, dt, n, h.data());
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  DCF_HIP(hipMemcpyAsync(table, h.data(), (size_t)n * sizeof(BatchEntry), hipMemcpyHostToDevice,
                         st));
  DCF_HIP(launch_batch_step((const BatchEntry *)table, h.data(), n, cfl, st));
  return DCF_OK;
}

dcf_status dcf_batch_table_fill(dcf_ctx *const *ctxs, double *const *U, double *const *dt, int n,
                                void *table_host, size_t table_bytes) {
  if (n < 1 || !ctxs || !U || !dt || !table_host)
    return fail(DCF_EINVAL, "null argument or n < 1");
  if (table_bytes < (size_t)n * sizeof(BatchEntry))
    return fail(DCF_EINVAL, "table needs %zu bytes, got %zu", (size_t)n * sizeof(BatchEntry),
                table_bytes);
  if (((uintptr_t)table_host) & 15) return fail(DCF_EINVAL, "table must be 16-byte aligned");
  return batch_fill(ctxs, U, dt, n, (BatchEntry *)table_host);
}

dcf_status dcf_batch_rk3_step_table(const void *table_dev, const void *table_host, int n,
                                    double cfl, void *stream) {
  if (n < 1 || !table_dev || !table_host) return fail(DCF_EINVAL, "null argument or n < 1");
  if ((((uintptr_t)table_dev) | ((uintptr_t)table_host)) & 15)
    return fail(DCF_EINVAL, "tables must be 16-byte aligned");
  const BatchEntry *h = (const BatchEntry *)table_host;
  for (int i = 0; i < n; ++i)
    if (h[i].g.ndim != h[0].g.ndim || (h[i].g.visc != VISC_NONE) != (h[0].g.visc != VISC_NONE) ||
        h[i].g.ndim < 1 || h[i].g.ndim > 3)
      return fail(DCF_EINVAL, "table entry %d is not a filled entry of this batch", i);
  DCF_HIP(launch_batch_step((const BatchEntry *)table_dev, h, n, cfl, (hipStream_t)stream));
  return DCF_OK;
}

dcf_status dcf_rk3_step_cfl(dcf_ctx *c, double *U, const double *dt, double cfl, double dt_max,
                            double *dt_next, void *stream) {
  dcf_status s = ready(c, 0);
  if (s) return s;
  if (!U || !dt || !dt_next) return fail(DCF_EINVAL, "null array");
  if (!(cfl > 0.0)) return fail(DCF_EINVAL, "cfl must be > 0");
  if (!(dt_max > 0.0)) dt_max = 1.0e300;
  hipStream_t st = (hipStream_t)stream;
  if ((s = rk3_stages(c, U, dt, st, nullptr, nullptr, c->dtpart))) return s;
  const unsigned nparts = fused_stages(c) ? flux_update_blocks(c->g) : update_blocks(c->g);
  DCF_HIP(launch_dt_final(c->dtpart, (int)nparts, cfl, dt_max, dt_next, st));
  return DCF_OK;
}

dcf_status dcf_rk3_steps_cfl(dcf_ctx *c, double *U, double *dt, int nsteps, double cfl,
                             double dt_max, void *stream) {
  dcf_status s = ready(c, 0);
  if (s) return s;
  if (!U || !dt) return fail(DCF_EINVAL, "null array");
  if (nsteps < 1) return fail(DCF_EINVAL, "nsteps must be >= 1");
  if (!(cfl > 0.0)) return fail(DCF_EINVAL, "cfl must be > 0");
  if (!(dt_max > 0.0)) dt_max = 1.0e300;
  hipStream_t st = (hipStream_t)stream;
  const bool fused = fused_stages(c);
  const unsigned nparts = fused ? flux_update_blocks(c->g) : update_blocks(c->g);
  const PendingDt pend{(int)nparts, cfl, dt_max, dt};
  for (int n = 0; n < nsteps; ++n) {
    // U is not touched between the steps of this call: each step after the
    // first starts from the primitive box the previous one left, and its
    // first ghost fill finishes the previous step's CFL reduction
    const bool chained = fused && n + 1 < nsteps;
    if ((s = rk3_stages(c, U, dt, st, nullptr, nullptr, c->dtpart, n & 1, fused && n > 0, chained,
                        fused && n > 0 ? &pend : nullptr)))
      return s;
    if (!chained) DCF_HIP(launch_dt_final(c->dtpart, (int)nparts, cfl, dt_max, dt, st));
  }
  return DCF_OK;
}

dcf_status dcf_diagnostics(dcf_ctx *c, const double *U, double *out, void *stream) {
  dcf_status s = ready(c, 0);
  if (s) return s;
  if (!U || !out) return fail(DCF_EINVAL, "null array");
  hipStream_t st = (hipStream_t)stream;
  DCF_HIP(launch_prim_halo(c->g, U, st));
  DCF_HIP(launch_diag(c->g, U, c->part, out, st));
  return DCF_OK;
}

dcf_status dcf_cost_term(dcf_ctx *c, const double *U, double w, double *J, double *grad,
                         void *stream) {
  dcf_status s = ready(c, 0);
  if (s) return s;
  if (!U || !J) return fail(DCF_EINVAL, "null array");
  if (c->cost_face < 0) return fail(DCF_EINVAL, "no cost face set (dcf_set_cost)");
  DCF_HIP(launch_cost(c->g, c->cost_face, c->cost_pref, U, w, J, grad, (hipStream_t)stream));
  return DCF_OK;
}

dcf_status dcf_flags(dcf_ctx *c, unsigned *flags_host, void *stream) {
  if (!c || !flags_host) return fail(DCF_EINVAL, "null argument");
  if (c->ws_mode < 0) return fail(DCF_ENOMEM, "workspace not set");
  hipStream_t st = (hipStream_t)stream;
  unsigned f = 0;
  DCF_HIP(hipMemcpyAsync(&f, c->g.flags, sizeof f, hipMemcpyDeviceToHost, st));
  DCF_HIP(hipStreamSynchronize(st));
  *flags_host = f;
  if (f) {
    unsigned z = 0;
    DCF_HIP(hipMemcpyAsync(c->g.flags, &z, sizeof z, hipMemcpyHostToDevice, st));
    DCF_HIP(hipStreamSynchronize(st));
  }
  return DCF_OK;
}

dcf_status dcf_vjp_step(dcf_ctx *c, const double *Un, const double *stages, const double *dt,
                        const double *lam1, double *lam0, double *dJdK, void *stream) {
  dcf_status s = ready(c, 1);
  if (s) return s;
  if (!Un || !dt || !lam1 || !lam0) return fail(DCF_EINVAL, "null array");
  if (lam0 == lam1) return fail(DCF_EINVAL, "lam_n may not alias lam_np1");
  if (c->g.scheme != SCHEME_WENO5)
    return fail(DCF_EUNSUPPORTED, "the adjoint is of the WENO5-JS scheme only");
  const long M = (long)c->g.nv * c->g.ncell;
  hipStream_t st = (hipStream_t)stream;
  // without the caller's stage states: the two stage states of Un as the
  // forward step makes them (its first two stages; Un is only read)
  if (!stages) {
    dcf_status s2 = rk3_stages(c, const_cast<double *>(Un), dt, st, c->U1, c->U2, nullptr, 0,
                               false, false, nullptr, 2);
    if (s2) return s2;
  }
  const double *S1 = stages ? stages : c->U1;
  const double *S2 = stages ? stages + M : c->U2;
  return vjp_step(c->g, c->adj, Un, S1, S2, dt, lam1, lam0, dJdK, st)
             ? fail(DCF_EDEVICE, "vjp launch failed")
             : DCF_OK;
}

dcf_status dcf_gradient_begin(dcf_ctx *c, const double *U0, int nsteps, const double *dt,
                              int seg_len, double *J, double *dJdK, void *stream) {
  dcf_status s = ready(c, 2);
  if (s) return s;
  if (nsteps < 1 || nsteps > c->ws_nsteps || c->ws_seg != seg_len)
    return fail(DCF_EINVAL, "workspace was sized for up to nsteps=%d with seg_len=%d, not %d/%d",
                c->ws_nsteps, c->ws_seg, nsteps, seg_len);
  if (!U0 || !dt || !J) return fail(DCF_EINVAL, "null array");
  if (c->cost_face < 0) return fail(DCF_EINVAL, "no cost face set (dcf_set_cost)");
  if (c->g.scheme != SCHEME_WENO5)
    return fail(DCF_EUNSUPPORTED, "the adjoint is of the WENO5-JS scheme only");
  hipStream_t st = (hipStream_t)stream;
  const long M = (long)c->g.nv * c->g.ncell;
  auto &gr = c->gr;
  gr = {};
  gr.active = true;
  gr.nsteps = nsteps;
  gr.seg_len = seg_len;
  gr.dt = dt;
  gr.J = J;
  gr.dJdK = c->nK > 0 ? dJdK : nullptr;
  gr.lam = c->lam_a;
  gr.lam_prev = c->lam_b;
  DCF_HIP(launch_fill(J, 0.0, 1, st));
  if (gr.dJdK) DCF_HIP(launch_fill(gr.dJdK, 0.0, c->nK, st));
  DCF_HIP(launch_copy(c->seg, U0, M, st));  // running state of the forward sweep
  return DCF_OK;
}

// One unit of gradient work: a forward step (with checkpoint and cost), a
// recomputed step of the current segment, or a reverse step.
// A copy of the context whose primitive box is the cached
// ones of stage s of step n of the current segment (workspace mode 3).
static Dev stage_box(const dcf_ctx *c, int n, int s) {
  Dev d = c->g;
  double *p = c->boxc + (size_t)(3 * n + s) * c->box_arrays * d.nboxp;
  for (int q = 0; q < NQ; ++q, p += d.nboxp) d.Q[q] = p;
  return d;
}

// Step k of the current segment, keeping what the reverse sweep needs:
// seg[k+1] from seg[k], the two inner stage states and (mode 3) every
// stage's primitive box.
static dcf_status segment_step(dcf_ctx *c, int k, hipStream_t st) {
  auto &gr = c->gr;
  Dev &g = c->g;
  const long M = (long)g.nv * g.ncell;
  double *Ua = c->seg + (long)k * M, *Ub = Ua + M;
  DCF_HIP(launch_copy(Ub, Ua, M, st));
  double *S1 = c->sst + (long)(2 * k) * M, *S2 = S1 + M;
  if (c->boxc && g.source == SRC_NONE) {  // the same three stages, keeping each stage's boxes
    const double *in[3] = {Ub, S1, S2};
    double *out[3] = {S1, S2, Ub};
    const double a[3] = {0.0, 0.75, 1.0 / 3.0}, b[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int s = 0; s < 3; ++s) {
      const Dev gs = stage_box(c, k, s);
      if (fused_stages(c)) {
        // as rk3_stages: each update writes the interior of the next
        // stage's cached box
        BoxOut next;
        if (s < 2) {
          const Dev gn = stage_box(c, k, s + 1);
          for (int q = 0; q < NQ; ++q) next.Q[q] = gn.Q[q];
        }
        if (s == 0) DCF_HIP(launch_prim_halo(gs, in[s], st));
        else DCF_HIP(launch_prim_ghost(gs, st));
        DCF_HIP(launch_fluxes_update(gs, Ub, in[s], out[s], gr.dt, a[s], b[s], nullptr, st,
                                     next));
      } else {
        DCF_HIP(launch_prim_halo(gs, in[s], st));
        DCF_HIP(launch_fluxes(gs, st));
        DCF_HIP(launch_update(gs, Ub, in[s], out[s], nullptr, gr.dt, a[s], b[s], nullptr, st));
      }
    }
    return DCF_OK;
  }
  return rk3_stages(c, Ub, gr.dt, st, S1, S2);
}

static dcf_status gradient_unit(dcf_ctx *c, hipStream_t st) {
  auto &gr = c->gr;
  Dev &g = c->g;
  const long M = (long)g.nv * g.ncell;
  const double w = 1.0 / gr.nsteps;
  const int nseg = (gr.nsteps + gr.seg_len - 1) / gr.seg_len;
  const int last0 = (nseg - 1) * gr.seg_len;  // first step of the last segment
  dcf_status s;
  if (gr.phase == 0) {  // forward sweep
    if (gr.n % gr.seg_len == 0)
      DCF_HIP(launch_copy(c->ckpt + (long)(gr.n / gr.seg_len) * M, c->seg, M, st));
    const double *Unew = c->seg;
    if (gr.n >= last0) {
      // the last segment is the first one reversed: its steps keep their
      // states now, so it needs no recompute (seg[0] holds U^last0)
      const int k = gr.n - last0;
      if ((s = segment_step(c, k, st))) return s;
      Unew = c->seg + (long)(k + 1) * M;
    } else if ((s = rk3_stages(c, c->seg, gr.dt, st))) {
      return s;
    }
    DCF_HIP(launch_cost(g, c->cost_face, c->cost_pref, Unew, w, gr.J, nullptr, st));
    if (++gr.n == gr.nsteps) {
      gr.phase = 2;
      gr.sgi = nseg - 1;
      DCF_HIP(launch_fill(gr.lam, 0.0, M, st));
    }
    return DCF_OK;
  }
  const int n0 = gr.sgi * gr.seg_len;
  const int n1 = n0 + gr.seg_len < gr.nsteps ? n0 + gr.seg_len : gr.nsteps;
  if (gr.phase == 1) {  // recompute U^{n0+1} .. U^{n1} of the segment, keeping stage data
    if ((s = segment_step(c, gr.n, st))) return s;
    if (++gr.n == n1 - n0) {
      gr.phase = 2;
      gr.n = n1;
    }
    return DCF_OK;
  }
  if (gr.phase == 2) {  // reverse step n -> n-1
    const int n = gr.n;
    const double *Ucur = c->seg + (long)(n - n0) * M;
    DCF_HIP(launch_cost(g, c->cost_face, c->cost_pref, Ucur, w, c->force + 2, gr.lam, st));
    const double *Uprev = c->seg + (long)(n - 1 - n0) * M;
    double *S1 = c->sst + (long)(2 * (n - 1 - n0)) * M, *S2 = S1 + M;
    Dev boxes[3];
    const bool cached = c->boxc && g.source == SRC_NONE;
    if (cached)
      for (int k = 0; k < 3; ++k) boxes[k] = stage_box(c, n - 1 - n0, k);
    if (vjp_step(g, c->adj, Uprev, S1, S2, gr.dt, gr.lam, gr.lam_prev, gr.dJdK, st,
                 cached ? boxes : nullptr))
      return fail(DCF_EDEVICE, "vjp launch failed");
    double *t = gr.lam;
    gr.lam = gr.lam_prev;
    gr.lam_prev = t;
    gr.n = n - 1;
    if (gr.n == n0) {
      if (gr.sgi == 0) {
        gr.phase = 3;
      } else {
        gr.sgi -= 1;
        gr.phase = 1;
        gr.n = 0;
        DCF_HIP(launch_copy(c->seg, c->ckpt + (long)gr.sgi * M, M, st));
      }
    }
    return DCF_OK;
  }
  return DCF_OK;
}

dcf_status dcf_gradient_advance(dcf_ctx *c, int max_units, int *done, void *stream) {
  if (!c || !done) return fail(DCF_EINVAL, "null argument");
  if (!c->gr.active) return fail(DCF_EINVAL, "no gradient in progress (dcf_gradient_begin)");
  hipStream_t st = (hipStream_t)stream;
  dcf_status s;
  for (int u = 0; u < max_units && c->gr.phase != 3; ++u)
    if ((s = gradient_unit(c, st))) return s;
  *done = c->gr.phase == 3 ? 1 : 0;
  return DCF_OK;
}

dcf_status dcf_gradient_finish(dcf_ctx *c, double *dJdU0, void *stream) {
  if (!c) return fail(DCF_EINVAL, "null context");
  if (!c->gr.active || c->gr.phase != 3) return fail(DCF_EINVAL, "gradient not complete");
  if (dJdU0)
    DCF_HIP(launch_copy(dJdU0, c->gr.lam, (long)c->g.nv * c->g.ncell, (hipStream_t)stream));
  c->gr.active = false;
  return DCF_OK;
}

dcf_status dcf_gradient(dcf_ctx *c, const double *U0, int nsteps, const double *dt, int seg_len,
                        double *J, double *dJdK, double *dJdU0, void *stream) {
  dcf_status s = dcf_gradient_begin(c, U0, nsteps, dt, seg_len, J, dJdK, stream);
  if (s) return s;
  int done = 0;
  if ((s = dcf_gradient_advance(c, 1 << 30, &done, stream))) return s;
  return dcf_gradient_finish(c, dJdU0, stream);
}

dcf_status dcf_time_kernel(dcf_ctx *c, const double *U, int which, int reps, double *avg_ms,
                           void *stream) {
  dcf_status s = ready(c, 0);
  if (s) return s;
  if (!U || !avg_ms || reps < 1) return fail(DCF_EINVAL, "bad argument");
  if (which < 0 || which > 9 || (which >= 1 && which <= 3 && which > c->g.ndim))
    return fail(DCF_EINVAL, "unknown kernel %d", which);
  if (which == 5 || which == 9)
    return fail(DCF_EINVAL, "kernel %d does not exist: the flux kernels compute the velocity "
                            "derivatives while staging", which);
  if (which == 6 && !fused_stages(c))
    return fail(DCF_EINVAL, "no fused flux + update kernel for this case (1D or source term)");
  if (which == 7 && c->g.ndim != 3)
    return fail(DCF_EINVAL, "the combined x + y flux launch is for 3D grids");
  hipStream_t st = (hipStream_t)stream;
  Dev &g = c->g;
  if ((s = eval_fluxes(c, U, st))) return s;
  DCF_HIP(launch_fill(c->U2, 1.0e-3, 1, st));  // a tiny dt for the update kernel
  hipEvent_t e0, e1;
  DCF_HIP(hipEventCreate(&e0));
  DCF_HIP(hipEventCreate(&e1));
  DCF_HIP(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) {
    hipError_t e = hipSuccess;
    if (which == 0) e = launch_prim_halo(g, U, st);
    else if (which <= 3) e = launch_flux_dir(g, which - 1, st);
    else if (which == 6)
      e = launch_flux_update_last(g, U, U, c->U1, c->U2, 0.0, 1.0, nullptr, st, BoxOut{},
                                  g.source == SRC_MASSFLUX ? c->force : nullptr);
    else if (which == 7) e = launch_flux_xy(g, st);
    else if (which == 8) e = launch_prim_ghost(g, st);
    else e = launch_update(g, U, U, c->U1, nullptr, c->U2, 0.0, 1.0, c->force, st);
    if (e != hipSuccess) return fail(DCF_EDEVICE, "launch: %s", hipGetErrorString(e));
  }
  DCF_HIP(hipEventRecord(e1, st));
  DCF_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  DCF_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = ms / reps;
  return DCF_OK;
}

dcf_status dcf_probe_begin(dcf_ctx *c, int which, int max_launches) {
  dcf_status s = ready(c, 0);
  if (s) return s;
  if (!(which == 1 || (which >= 6 && which <= 8)))
    return fail(DCF_EINVAL, "kernel %d cannot be probed", which);
  if (max_launches < 1 || max_launches > (1 << 20)) return fail(DCF_EINVAL, "bad max_launches");
  if (c->probe.ev) return fail(DCF_EINVAL, "a probe is already armed");
  hipEvent_t *ev = new hipEvent_t[2 * (size_t)max_launches];
  for (int i = 0; i < 2 * max_launches; ++i) {
    const hipError_t e = hipEventCreate(&ev[i]);
    if (e != hipSuccess) {
      for (int k = 0; k < i; ++k) (void)hipEventDestroy(ev[k]);
      delete[] ev;
      return fail(DCF_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
  }
  c->probe.which = which;
  c->probe.ev = ev;
  c->probe.cap = max_launches;
  c->probe.n = 0;
  return DCF_OK;
}

dcf_status dcf_probe_end(dcf_ctx *c, int *launches, double *avg_ms) {
  if (!c) return fail(DCF_EINVAL, "null context");
  if (!launches || !avg_ms) return fail(DCF_EINVAL, "null argument");
  Probe &p = c->probe;
  if (!p.ev) return fail(DCF_EINVAL, "no probe armed");
  double sum = 0.0;
  hipError_t err = hipSuccess;
  if (p.n > 0) err = hipEventSynchronize(p.ev[2 * p.n - 1]);
  for (int i = 0; i < p.n && err == hipSuccess; ++i) {
    float ms = 0.f;
    err = hipEventElapsedTime(&ms, p.ev[2 * i], p.ev[2 * i + 1]);
    sum += ms;
  }
  *launches = p.n;
  *avg_ms = p.n > 0 ? sum / p.n : 0.0;
  for (int i = 0; i < 2 * p.cap; ++i) (void)hipEventDestroy(p.ev[i]);
  delete[] p.ev;
  p = Probe{};
  if (err != hipSuccess) return fail(DCF_EDEVICE, "probe events: %s", hipGetErrorString(err));
  return DCF_OK;
}

}  // extern "C"
