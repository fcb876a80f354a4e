// rlb_api.cpp -- C ABI (include/rlb.h) of the MI355X implementation of the
// ultra-relativistic lattice Boltzmann update (arXiv:1302.1125): validation,
// device memory ownership, step scheduling and error reporting.  All
// arithmetic of the update runs in the kernels of rlb_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/rlb.h"
#include "rlb_internal.h"

namespace {

thread_local std::string g_last_error;

rlb_status fail(rlb_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

rlb_status hip_fail(hipError_t e, const char* where) {
  return fail(RLB_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

constexpr unsigned long long kNoBadStep = ~0ull;

}  // namespace

struct rlb_ctx {
  rlb_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int act_mask = 1;
  bool fp64 = true;
  size_t elem = 8;
  long long ncell = 0;   // dense cells nx * ny * nz
  int px = 0, py = 0;    // row pitch, rows per plane (rlb::row_pitch, rlb::plane_rows)
  long long nstore = 0;  // storage cells px * py * nz
  void* f[2] = {nullptr, nullptr};
  void* h[2] = {nullptr, nullptr};
  int cur = 0;
  double* hist = nullptr;
  double* hist_alt = nullptr;  // 1D extended grids: the second copy for blocked launches
  float* hist32 = nullptr;  // compact previous-step fields (see compact_history)
  uint8_t* obst = nullptr;
  double* face_states = nullptr;   // [6][5]
  unsigned long long* counters = nullptr;  // [0] bad step, [1] guard events, [2] moments flag
  unsigned long long* host_counters = nullptr;  // pinned copy
  double* sums_partial = nullptr;
  double* sums_out = nullptr;
  int sums_blocks = 0;
  double* scratch = nullptr;  // this device's fixed read-back array (rlb::scratch_address)
  int tb_steps = 8;      // 1D: steps per temporally blocked launch (1: one step per launch)
  bool initialised = false;
  bool poisoned = false;
  long long steps = 0;
  long long first_bad = -1;
  rlb::StepParams base{};
};

namespace {

bool valid_bc(int b) { return b == RLB_BC_PERIODIC || b == RLB_BC_FIXED || b == RLB_BC_OUTFLOW; }

rlb_status validate(const rlb_config* c) {
  if (!c) return fail(RLB_E_INVALID_ARG, "config is NULL");
  if (c->struct_size != sizeof(rlb_config)) return fail(RLB_E_INVALID_ARG, "struct_size mismatch");
  if (c->nx < 2 || c->ny < 1 || c->nz < 1) return fail(RLB_E_INVALID_ARG, "grid: nx >= 2, ny, nz >= 1");
  if (c->ny == 1 && c->nz != 1) return fail(RLB_E_INVALID_ARG, "ny == 1 requires nz == 1");
  const long long nc = static_cast<long long>(rlb::row_pitch(c->nx, c->ny)) * rlb::plane_rows(c->ny) * c->nz;
  if (nc > rlb::kMaxCells)
    return fail(RLB_E_INVALID_ARG,
                "grid too large (at most 2^28 - 128 cells, nx padded to 64 and ny to 4 in 2D/3D)");
  if (c->precision != RLB_FP64 && c->precision != RLB_MIXED) return fail(RLB_E_INVALID_ARG, "precision");
  if (c->collision != RLB_COLL_IMPLICIT && c->collision != RLB_COLL_EULER)
    return fail(RLB_E_INVALID_ARG, "collision");
  if (c->tau_mode != RLB_TAU_UNIFORM && c->tau_mode != RLB_TAU_ETA_OVER_S)
    return fail(RLB_E_INVALID_ARG, "tau_mode");
  if (!(c->nu > 0 && std::isfinite(c->nu))) return fail(RLB_E_INVALID_ARG, "nu must be > 0");
  if (c->lattice != RLB_LATTICE_EXTENDED && c->lattice != RLB_LATTICE_BASIC)
    return fail(RLB_E_INVALID_ARG, "lattice");
  if (c->lattice == RLB_LATTICE_BASIC) {
    if (c->collision != RLB_COLL_IMPLICIT || c->with_density || c->alpha != 0.0 || c->guard_umax != 0.0)
      return fail(RLB_E_INVALID_ARG,
                  "basic lattice: regular collision only, no density, alpha = 0, guard off");
  } else if (!(c->dt_over_dx > 0 && c->dt_over_dx <= 0.5)) {
    return fail(RLB_E_INVALID_ARG, "dt_over_dx in (0, 0.5]");
  }
  if (c->density_weights != RLB_DENSW_PAPER && c->density_weights != RLB_DENSW_ISOTROPIC)
    return fail(RLB_E_INVALID_ARG, "density_weights");
  if (c->density_weights == RLB_DENSW_ISOTROPIC &&
      (c->lattice != RLB_LATTICE_EXTENDED || 13.0 / (c->nu * c->nu) < 17.0 / 24.0))
    return fail(RLB_E_INVALID_ARG, "isotropic density weights: extended lattice, nu <= 4.28");
  if (c->flux != RLB_FLUX_MINMOD && c->flux != RLB_FLUX_RUSANOV) return fail(RLB_E_INVALID_ARG, "flux");
  if (c->flux == RLB_FLUX_RUSANOV && c->lattice != RLB_LATTICE_EXTENDED)
    return fail(RLB_E_INVALID_ARG, "Rusanov flux: extended lattice only");
  if (c->tau_mode == RLB_TAU_UNIFORM && !(c->tau > 0 && std::isfinite(c->tau)))
    return fail(RLB_E_INVALID_ARG, "tau must be > 0");
  if (!(c->eta_over_s >= 0 && std::isfinite(c->eta_over_s))) return fail(RLB_E_INVALID_ARG, "eta_over_s >= 0");
  if (!(c->alpha >= 0 && std::isfinite(c->alpha))) return fail(RLB_E_INVALID_ARG, "alpha >= 0");
  if (c->guard_umax != 0.0 && !(c->guard_umax > 0 && c->guard_umax < 1 && c->guard_efloor > 0))
    return fail(RLB_E_INVALID_ARG, "guard_umax in (0,1) with guard_efloor > 0");
  const int n[3] = {c->nx, c->ny, c->nz};
  for (int a = 0; a < 3; ++a) {
    const int lo = c->bc[2 * a], hi = c->bc[2 * a + 1];
    if (!valid_bc(lo) || !valid_bc(hi)) return fail(RLB_E_INVALID_ARG, "bc value");
    if ((lo == RLB_BC_PERIODIC) != (hi == RLB_BC_PERIODIC))
      return fail(RLB_E_INVALID_ARG, "periodic faces come in pairs");
    if (n[a] == 1 && lo != RLB_BC_PERIODIC) return fail(RLB_E_INVALID_ARG, "axes of size 1 must be periodic");
    for (int side = 0; side < 2; ++side) {
      if (c->bc[2 * a + side] != RLB_BC_FIXED) continue;
      const double* q = c->face_states[2 * a + side];
      const double u2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
      bool ok = std::isfinite(q[0]) && q[0] > 0 && std::isfinite(u2) && u2 < 1.0;
      if (c->with_density) ok = ok && std::isfinite(q[4]) && q[4] > 0;
      if (!ok) return fail(RLB_E_INVALID_ARG, "inadmissible face state");
    }
  }
  return RLB_OK;
}

// The implicit mixed-precision step of 2D and 3D grids of the extended model
// keeps the previous-step fields in FP32 as (eps, gamma u, n) (StepParams::hist32).
bool compact_history(const rlb_config* c) {
  return c->precision != RLB_FP64 && (c->ny > 1 || c->nz > 1) && c->collision == RLB_COLL_IMPLICIT &&
         c->lattice == RLB_LATTICE_EXTENDED;
}

// 1D grids of the extended model step in temporally blocked launches, which
// move the previous-step fields between two copies (StepParams::hist_out).
bool blocked_1d(const rlb_config* c) {
  return c->ny == 1 && c->nz == 1 && c->lattice == RLB_LATTICE_EXTENDED;
}

uint64_t footprint(const rlb_config* c) {
  const uint64_t nc = static_cast<uint64_t>(c->nx) * c->ny * c->nz;
  const uint64_t ns = static_cast<uint64_t>(rlb::row_pitch(c->nx, c->ny)) * rlb::plane_rows(c->ny) * c->nz;
  const uint64_t ps = static_cast<uint64_t>(rlb::population_stride(static_cast<long long>(ns)));
  const uint64_t elem = c->precision == RLB_FP64 ? 8 : 4;
  uint64_t b = 2 * rlb::Q * ps * elem;            // f, ping-pong
  if (c->with_density) b += 2 * rlb::Q * ps * elem;
  b += 5 * ns * 8;                                // previous-step fields
  if (blocked_1d(c)) b += 5 * ns * 8;             // their second copy
  if (compact_history(c)) b += 5 * ns * 4;        // and their FP32 form
  b += (nc + 255) / 256 * 5 * 8;                  // reduction partials
  b += 6 * 5 * 8 + 4 * 8 + 8 * 8;                 // face states, counters, sums
  return b;
}

void free_all(rlb_ctx* x) {
  for (int k = 0; k < 2; ++k) {
    if (x->f[k]) (void)hipFree(x->f[k]);
    if (x->h[k]) (void)hipFree(x->h[k]);
  }
  if (x->hist) (void)hipFree(x->hist);
  if (x->hist_alt) (void)hipFree(x->hist_alt);
  if (x->hist32) (void)hipFree(x->hist32);
  if (x->obst) (void)hipFree(x->obst);
  if (x->face_states) (void)hipFree(x->face_states);
  if (x->counters) (void)hipFree(x->counters);
  if (x->host_counters) (void)hipHostFree(x->host_counters);
  if (x->sums_partial) (void)hipFree(x->sums_partial);
  if (x->sums_out) (void)hipFree(x->sums_out);
  if (x->own_stream && x->stream) (void)hipStreamDestroy(x->stream);
}

template <typename P>
rlb_status dalloc(P** p, size_t bytes, const char* what) {
  void* q = nullptr;
  const hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(RLB_E_OUT_OF_MEMORY, std::string("hipMalloc ") + what + ": " + hipGetErrorString(e));
  }
  *p = static_cast<P*>(q);
  return RLB_OK;
}

void fill_constants(const rlb_config& c, rlb::StepParams& p);

int largest_divisor_at_most(int n, int cap) {
  for (int d = cap < n ? cap : n; d > 1; --d)
    if (n % d == 0) return d;
  return 1;
}

void fill_params(rlb_ctx* x) {
  const rlb_config& c = x->cfg;
  rlb::StepParams& p = x->base;
  p = rlb::StepParams{};
  p.ncell = x->nstore;
  p.pstride = rlb::population_stride(x->nstore);
  p.nx = c.nx;
  p.ny = c.ny;
  p.nz = c.nz;
  p.px = x->px;
  p.py = x->py;
  if (c.ny == 1) {
    p.tile_x = rlb::kBlock;
    p.tile_y = 1;
  } else {
    p.tile_x = 64;
    p.tile_y = rlb::kBlock / 64;
  }
  p.ntx = (c.nx + p.tile_x - 1) / p.tile_x;
  p.nty = (c.ny + p.tile_y - 1) / p.tile_y;
  p.ntiles = static_cast<long long>(p.ntx) * p.nty * c.nz;
  // Pencil shape: the largest divisors of ntx / nty not above the targets
  // (3D: 8 x 3 tiles = 512 x 12 cells marched in z; 2D: strips 16 tiles
  // wide), chosen by measurement on MI355X.
  int want_w = c.nz > 1 ? 8 : 16, want_h = c.nz > 1 ? 3 : 1 << 30;
  if (const char* e = std::getenv("RLB_PENCIL")) {  // tuning override "pw,ph"
    int a = 0, b = 0;
    if (std::sscanf(e, "%d,%d", &a, &b) == 2 && a > 0 && b > 0) {
      want_w = a;
      want_h = b;
    }
  }
  p.pw = largest_divisor_at_most(p.ntx, want_w);
  p.ph = largest_divisor_at_most(p.nty, want_h);
  if (c.nz >= rlb::kXcds) {
    // 3D: each XCD owns a z-slab and marches pencils through it
    p.order = 1;
    p.zslab = (c.nz + rlb::kXcds - 1) / rlb::kXcds;
    p.tiles_per_xcd = static_cast<long long>(p.zslab) * p.ntx * p.nty;
  } else {
    p.order = 0;
    p.zslab = 1;
    p.tiles_per_xcd = (p.ntiles + rlb::kXcds - 1) / rlb::kXcds;
  }
  // z-marching runs (3D mixed-precision implicit step) of 16 planes
  // (measured on MI355X at 384^3: 8-16 planes per run equally fast, 48
  // planes 3% slower)
  p.zm_len = 0;
  if (c.nz >= 8 && c.precision == RLB_MIXED && c.collision == RLB_COLL_IMPLICIT &&
      c.lattice == RLB_LATTICE_EXTENDED && p.pstride <= rlb::kZmMaxStride) {
    int len = 16;
    if (const char* e = std::getenv("RLB_ZMARCH")) len = std::atoi(e);  // tuning override, 0 = off
    if (len > 0) {
      p.zm_len = len < c.nz ? len : c.nz;
      const long long runs = (c.nz + p.zm_len - 1) / p.zm_len;
      p.zm_total = runs * p.ntx * p.nty;
      p.zm_per_xcd = (p.zm_total + rlb::kXcds - 1) / rlb::kXcds;
    }
  }
  for (int k = 0; k < 6; ++k) p.bc[k] = c.bc[k];
  fill_constants(c, p);
  p.hist = x->hist;
  p.hist32 = x->hist32;
  p.obst = nullptr;
  p.cell0 = 0;
  p.range = x->ncell;
  p.bad_step = x->counters;
  p.guard_count = x->counters + 1;
}

}  // namespace

// Lattice and run constants of a configuration (shared with the server).
void rlb_fill_constants(const rlb_config& c, rlb::StepParams& p) { fill_constants(c, p); }
rlb_status rlb_validate_config(const rlb_config* c) { return validate(c); }
rlb_status rlb_set_error(rlb_status s, const std::string& msg) { return fail(s, msg); }

namespace {

void fill_constants(const rlb_config& c, rlb::StepParams& p) {
  const double nu = c.nu;
  const bool basic = c.lattice == RLB_LATTICE_BASIC;
  // (c_a nu)^2: 13 for the extended set (Eq. (46)), 19 for the basic set
  const double ca2nu2 = basic ? 19.0 : 13.0;
  // basic model: exact streaming fixes dt = c_t dx / (c_a c_0) = sqrt(27/19)
  const double dt = basic ? std::sqrt(27.0 / 19.0) : c.dt_over_dx;
  p.lattice = basic ? 1 : 0;
  p.a_scale = nu * nu / 27.0;
  p.r = std::sqrt(27.0) / nu;
  p.ca = std::sqrt(ca2nu2) / nu;
  p.ca2 = ca2nu2 / (nu * nu);
  p.rca = p.r * p.ca;
  p.inv_r = nu / std::sqrt(27.0);
  if (c.density_weights == RLB_DENSW_ISOTROPIC) {
    // sum w' = 1, sum w' c^a c^b = delta/3 and an isotropic fourth moment
    p.wp0 = 1.0 - 17.0 / (24.0 * p.ca2);
    p.wp1 = 1.0 / (9.0 * p.ca2);
    p.wp2 = 1.0 / (288.0 * p.ca2);
  } else {  // Eqs. (59)-(60)
    p.wp0 = 0.1;
    p.wp1 = 6.0 / 35.0 - 1.0 / (42.0 * p.ca2);
    p.wp2 = 1.0 / (84.0 * p.ca2) - 3.0 / 280.0;
  }
  p.k1 = 4.0 * std::sqrt(ca2nu2 / 27.0);
  p.omega_c = nu * nu * dt / std::sqrt(27.0);
  p.kappa = p.omega_c * c.alpha;
  p.dtv = dt * std::sqrt(ca2nu2 / 27.0);
  p.tau = c.tau;
  p.nu2_etas = nu * nu * c.eta_over_s;
  p.tau_mode = c.tau_mode;
  p.flux = c.flux == RLB_FLUX_RUSANOV ? rlb::kFluxRusanov : rlb::kFluxMinmod;
  p.guard = c.guard_umax > 0 ? 1 : 0;
  if (p.guard) {
    const double um = c.guard_umax, u1 = 1.0 - 2.0 * (1.0 - um);
    p.mmax = 4.0 * um / (3.0 + um * um);
    p.m1 = 4.0 * u1 / (3.0 + u1 * u1);
    p.efloor = c.guard_efloor;
    p.gmax = 1.0 / std::sqrt((1.0 - um) * (1.0 + um));
  }
}

rlb_status check_ctx(rlb_ctx* x) {
  if (!x) return fail(RLB_E_INVALID_ARG, "ctx is NULL");
  if (!x->initialised) return fail(RLB_E_STATE, "rlb_init_fields has not been called");
  if (x->poisoned) return fail(RLB_E_STATE, "context poisoned by an inadmissible step; call rlb_init_fields");
  return RLB_OK;
}

rlb_status set_device(rlb_ctx* x) {
  const hipError_t e = hipSetDevice(x->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return RLB_OK;
}

rlb_status read_counters(rlb_ctx* x) {
  hipError_t e = hipMemcpyAsync(x->host_counters, x->counters, 3 * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, x->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(counters)");
  e = hipStreamSynchronize(x->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return RLB_OK;
}

// Fields of the current populations through the device staging buffer
// `stage` ([5][ncell] FP64), copied into the caller's host arrays; returns
// after the copies are done.  Allocates nothing.
hipError_t read_fields(rlb_ctx* x, double* stage, double* const dst[5]) {
  rlb::StepParams p = x->base;
  p.f_in = x->f[x->cur];
  p.h_in = x->h[x->cur];
  hipError_t e = rlb::launch_moments(p, x->fp64, x->cfg.with_density != 0, stage, x->counters + 2,
                                     x->stream);
  const size_t nb = sizeof(double) * x->ncell;
  for (int k = 0; k < 5 && e == hipSuccess; ++k)
    if (dst[k]) e = hipMemcpyAsync(dst[k], stage + k * x->ncell, nb, hipMemcpyDeviceToHost, x->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
  return e;
}
}  // namespace

extern "C" {

rlb_status rlb_config_default(rlb_config* c) {
  if (!c) return fail(RLB_E_INVALID_ARG, "config is NULL");
  std::memset(c, 0, sizeof(*c));
  c->struct_size = sizeof(rlb_config);
  c->nx = 64;
  c->ny = 1;
  c->nz = 1;
  c->precision = RLB_FP64;
  c->collision = RLB_COLL_IMPLICIT;
  c->tau_mode = RLB_TAU_UNIFORM;
  c->with_density = 0;
  c->nu = std::pow(27.0, 0.25);
  c->dt_over_dx = 0.25;
  c->tau = 1.0;
  c->eta_over_s = 0.0;
  c->alpha = 0.0;
  for (int k = 0; k < 6; ++k) {
    c->bc[k] = RLB_BC_PERIODIC;
    c->face_states[k][0] = 3.0;
    c->face_states[k][4] = 1.0;
  }
  c->guard_umax = 0.0;
  c->guard_efloor = 1e-10;
  return RLB_OK;
}

uint64_t rlb_footprint_bytes(const rlb_config* cfg) {
  if (validate(cfg) != RLB_OK) return 0;
  return footprint(cfg);
}

rlb_status rlb_create(const rlb_config* cfg, void* hip_stream, rlb_ctx** out) {
  if (!out) return fail(RLB_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  rlb_status st = validate(cfg);
  if (st != RLB_OK) return st;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(RLB_E_DEVICE, "no HIP device available (this library has no CPU path)");
  }
  rlb_ctx* x = new (std::nothrow) rlb_ctx();
  if (!x) return fail(RLB_E_OUT_OF_MEMORY, "host allocation");
  x->cfg = *cfg;
  e = hipGetDevice(&x->device);
  if (e != hipSuccess) {
    delete x;
    return hip_fail(e, "hipGetDevice");
  }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, x->device);
  if (e != hipSuccess) {
    delete x;
    return hip_fail(e, "hipGetDeviceProperties");
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    delete x;
    return fail(RLB_E_DEVICE, std::string("built for gfx950, device is ") + prop.gcnArchName);
  }
  // the fixed read-back array of rlb_moments_noalloc on this device (looked
  // up once per device, with the device current)
  e = rlb::scratch_address(x->device, &x->scratch);
  if (e != hipSuccess) {
    delete x;
    return hip_fail(e, "hipGetSymbolAddress(scratch)");
  }
  x->fp64 = cfg->precision == RLB_FP64;
  x->elem = x->fp64 ? 8 : 4;
  x->ncell = static_cast<long long>(cfg->nx) * cfg->ny * cfg->nz;
  x->px = rlb::row_pitch(cfg->nx, cfg->ny);
  x->py = rlb::plane_rows(cfg->ny);
  x->nstore = static_cast<long long>(x->px) * x->py * cfg->nz;
  x->act_mask = cfg->nz > 1 ? 7 : (cfg->ny > 1 ? 3 : 1);
  if (const char* e = std::getenv("RLB_TB_STEPS")) {  // tuning override, 1 = off
    const int v = std::atoi(e);
    x->tb_steps = v < 1 ? 1 : (v > rlb::kTbMaxSteps ? rlb::kTbMaxSteps : v);
  } else if (x->act_mask == 1) {
    // a 1D grid that gives every workgroup a CU of its own even at 16 steps
    // per launch leaves CUs idle anyway: the wider recomputed overlap then
    // costs no wall time and the launches halve (on MI355X 6.9% more
    // cell-updates per second at 1000 cells, 5.6% at 8192)
    const int kb = rlb::kTbMaxSteps;
    const long long tiles = (cfg->nx + rlb::tb_cells_per_tile(kb) - 1) / rlb::tb_cells_per_tile(kb);
    if (tiles <= prop.multiProcessorCount) x->tb_steps = kb;
  }
  if (hip_stream) {
    x->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    e = hipStreamCreateWithFlags(&x->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete x;
      return hip_fail(e, "hipStreamCreate");
    }
    x->own_stream = true;
  }
  const size_t pop_bytes = static_cast<size_t>(rlb::Q) * rlb::population_stride(x->nstore) * x->elem;
  x->sums_blocks = static_cast<int>((x->ncell + rlb::kBlock - 1) / rlb::kBlock);
  st = RLB_OK;
  for (int k = 0; k < 2 && st == RLB_OK; ++k) {
    st = dalloc(&x->f[k], pop_bytes, "f");
    if (st == RLB_OK && cfg->with_density) st = dalloc(&x->h[k], pop_bytes, "h");
  }
  if (st == RLB_OK) st = dalloc(&x->hist, 5 * sizeof(double) * x->nstore, "fields");
  if (st == RLB_OK && blocked_1d(cfg)) st = dalloc(&x->hist_alt, 5 * sizeof(double) * x->nstore, "fields");
  if (st == RLB_OK && compact_history(cfg))
    st = dalloc(&x->hist32, 5 * sizeof(float) * x->nstore, "fields (FP32)");
  if (st == RLB_OK) st = dalloc(&x->face_states, 6 * 5 * sizeof(double), "face_states");
  if (st == RLB_OK) st = dalloc(&x->counters, 4 * sizeof(unsigned long long), "counters");
  if (st == RLB_OK) st = dalloc(&x->sums_partial, static_cast<size_t>(x->sums_blocks) * 5 * sizeof(double), "sums");
  if (st == RLB_OK) st = dalloc(&x->sums_out, 8 * sizeof(double), "sums_out");
  if (st == RLB_OK) {
    e = hipHostMalloc(reinterpret_cast<void**>(&x->host_counters), 4 * sizeof(unsigned long long));
    if (e != hipSuccess) st = hip_fail(e, "hipHostMalloc");
  }
  if (st != RLB_OK) {
    free_all(x);
    delete x;
    return st;
  }
  fill_params(x);
  e = hipMemcpyAsync(x->face_states, cfg->face_states, 6 * 5 * sizeof(double), hipMemcpyHostToDevice,
                     x->stream);
  if (e == hipSuccess)
    e = rlb::launch_face_slots(x->base, x->fp64, x->face_states, x->f[0], x->f[1], x->h[0], x->h[1],
                               x->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
  if (e != hipSuccess) {
    st = hip_fail(e, "face equilibria");
    free_all(x);
    delete x;
    return st;
  }
  *out = x;
  return RLB_OK;
}

void rlb_destroy(rlb_ctx* x) {
  if (!x) return;
  (void)hipSetDevice(x->device);
  if (x->stream) (void)hipStreamSynchronize(x->stream);
  free_all(x);
  delete x;
}

rlb_status rlb_init_fields(rlb_ctx* x, const double* eps, const double* ux, const double* uy,
                           const double* uz, const double* n, const uint8_t* obstacle) {
  if (!x) return fail(RLB_E_INVALID_ARG, "ctx is NULL");
  if (!eps || !ux || !uy || !uz) return fail(RLB_E_INVALID_ARG, "eps, ux, uy, uz are required");
  const bool wh = x->cfg.with_density != 0;
  if (wh && !n) return fail(RLB_E_INVALID_ARG, "n is required with density");
  for (long long c = 0; c < x->ncell; ++c) {
    const double u2 = ux[c] * ux[c] + uy[c] * uy[c] + uz[c] * uz[c];
    bool ok = std::isfinite(eps[c]) && eps[c] > 0 && std::isfinite(u2) && u2 < 1.0;
    if (wh) ok = ok && std::isfinite(n[c]) && n[c] > 0;
    if (!ok) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "inadmissible initial state at cell %lld", c);
      return fail(RLB_E_INADMISSIBLE, buf);
    }
  }
  rlb_status st = set_device(x);
  if (st != RLB_OK) return st;
  // dense host planes [z][y][x] into device planes of py rows of pitch px
  const size_t nx = static_cast<size_t>(x->cfg.nx), ny = static_cast<size_t>(x->cfg.ny);
  const size_t nz = static_cast<size_t>(x->cfg.nz);
  const size_t px = static_cast<size_t>(x->px), py = static_cast<size_t>(x->py);
  auto upload = [&](void* dst, const void* src, size_t elem) {
    if (px == nx && py == ny)
      return hipMemcpyAsync(dst, src, elem * nx * ny * nz, hipMemcpyHostToDevice, x->stream);
    hipError_t r = hipSuccess;
    for (size_t z = 0; z < nz && r == hipSuccess; ++z)
      r = hipMemcpy2DAsync(static_cast<char*>(dst) + z * py * px * elem, px * elem,
                           static_cast<const char*>(src) + z * ny * nx * elem, nx * elem, nx * elem, ny,
                           hipMemcpyHostToDevice, x->stream);
    return r;
  };
  const double* src[5] = {eps, ux, uy, uz, wh ? n : nullptr};
  hipError_t e = hipSuccess;
  for (int k = 0; k < 5 && e == hipSuccess; ++k)
    if (src[k]) e = upload(x->hist + k * x->nstore, src[k], sizeof(double));
  if (e != hipSuccess) return hip_fail(e, "upload(fields)");
  if (obstacle) {
    if (!x->obst) {
      st = dalloc(&x->obst, static_cast<size_t>(x->nstore), "obstacle");
      if (st != RLB_OK) return st;
    }
    e = hipMemsetAsync(x->obst, 0, static_cast<size_t>(x->nstore), x->stream);
    if (e == hipSuccess) e = upload(x->obst, obstacle, 1);
    if (e != hipSuccess) return hip_fail(e, "upload(obstacle)");
  }
  x->cur = 0;
  rlb::StepParams p = x->base;
  p.f_out = x->f[0];
  p.h_out = x->h[0];
  p.hist = x->hist;
  e = rlb::launch_init(p, x->fp64, wh, x->stream);
  if (e != hipSuccess) return hip_fail(e, "init kernel");
  const unsigned long long init_counters[4] = {kNoBadStep, 0ull, kNoBadStep, 0ull};
  e = hipMemcpyAsync(x->counters, init_counters, sizeof init_counters, hipMemcpyHostToDevice, x->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
  if (e != hipSuccess) return hip_fail(e, "init");
  x->base.obst = obstacle ? x->obst : nullptr;
  x->initialised = true;
  x->poisoned = false;
  x->steps = 0;
  x->first_bad = -1;
  g_last_error.clear();
  return RLB_OK;
}

rlb_status rlb_step_async(rlb_ctx* x, int64_t nsteps) {
  rlb_status st = check_ctx(x);
  if (st != RLB_OK) return st;
  if (nsteps < 0) return fail(RLB_E_INVALID_ARG, "nsteps < 0");
  st = set_device(x);
  if (st != RLB_OK) return st;
  const bool wh = x->cfg.with_density != 0;
  const bool eu = x->cfg.collision == RLB_COLL_EULER;
  const bool rusanov = x->cfg.flux == RLB_FLUX_RUSANOV;  // built in the blocked step only
  if (x->act_mask == 1 && x->cfg.lattice == RLB_LATTICE_EXTENDED && (x->tb_steps > 1 || rusanov)) {
    // 1D: temporally blocked launches of up to tb_steps steps each; the
    // previous-step fields alternate between the two copies like f and h
    for (int64_t k = 0; k < nsteps;) {
      const int kb = static_cast<int>(std::min<int64_t>(x->tb_steps, nsteps - k));
      const int cells = rlb::tb_cells_per_tile(kb);
      const unsigned grid = static_cast<unsigned>((x->cfg.nx + cells - 1) / cells);
      rlb::StepParams p = x->base;
      p.f_in = x->f[x->cur];
      p.f_out = x->f[1 - x->cur];
      p.h_in = x->h[x->cur];
      p.h_out = x->h[1 - x->cur];
      p.hist = x->hist;
      p.hist_out = x->hist_alt;
      p.step_index = x->steps;
      const hipError_t e = rlb::launch_step_tb(p, x->fp64, wh, eu, kb, false, grid, x->stream);
      if (e != hipSuccess) return hip_fail(e, "step kernel");
      std::swap(x->hist, x->hist_alt);
      x->base.hist = x->hist;
      x->cur = 1 - x->cur;
      x->steps += kb;
      k += kb;
    }
    return RLB_OK;
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    rlb::StepParams p = x->base;
    p.f_in = x->f[x->cur];
    p.f_out = x->f[1 - x->cur];
    p.h_in = x->h[x->cur];
    p.h_out = x->h[1 - x->cur];
    p.step_index = x->steps;
    const hipError_t e = rlb::launch_step(p, x->fp64, x->act_mask, wh, eu, x->stream);
    if (e != hipSuccess) return hip_fail(e, "step kernel");
    x->cur = 1 - x->cur;
    x->steps += 1;
  }
  return RLB_OK;
}

rlb_status rlb_sync(rlb_ctx* x) {
  if (!x) return fail(RLB_E_INVALID_ARG, "ctx is NULL");
  if (!x->initialised) return fail(RLB_E_STATE, "rlb_init_fields has not been called");
  rlb_status st = set_device(x);
  if (st != RLB_OK) return st;
  st = read_counters(x);
  if (st != RLB_OK) return st;
  if (x->host_counters[0] != kNoBadStep) {
    x->first_bad = static_cast<long long>(x->host_counters[0]);
    x->poisoned = true;
    char buf[160];
    std::snprintf(buf, sizeof buf, "inadmissible state met in step %lld", x->first_bad);
    return fail(RLB_E_INADMISSIBLE, buf);
  }
  return RLB_OK;
}

rlb_status rlb_step(rlb_ctx* x, int64_t nsteps) {
  rlb_status st = rlb_step_async(x, nsteps);
  if (st != RLB_OK) return st;
  return rlb_sync(x);
}


rlb_status rlb_moments(rlb_ctx* x, double* eps, double* ux, double* uy, double* uz, double* n) {
  if (!x) return fail(RLB_E_INVALID_ARG, "ctx is NULL");
  if (!x->initialised) return fail(RLB_E_STATE, "rlb_init_fields has not been called");
  rlb_status st = set_device(x);
  if (st != RLB_OK) return st;
  double* out = nullptr;
  st = dalloc(&out, 5 * sizeof(double) * x->ncell, "moments");
  if (st != RLB_OK) return st;
  double* const dst[5] = {eps, ux, uy, uz, n};
  const hipError_t e = read_fields(x, out, dst);
  (void)hipFree(out);
  if (e != hipSuccess) return hip_fail(e, "moments");
  return RLB_OK;
}

rlb_status rlb_moments_noalloc(rlb_ctx* x, double* eps, double* ux, double* uy, double* uz,
                               double* n) {
  if (!x) return fail(RLB_E_INVALID_ARG, "ctx is NULL");
  if (!x->initialised) return fail(RLB_E_STATE, "rlb_init_fields has not been called");
  if (x->ncell > rlb::kScratchCells) {
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "rlb_moments_noalloc: grid of %lld cells exceeds the fixed read-back array "
                  "(at most %lld cells); use rlb_moments",
                  x->ncell, rlb::kScratchCells);
    return fail(RLB_E_INVALID_ARG, buf);
  }
  if (!x->scratch) return fail(RLB_E_DEVICE, "fixed read-back array not resolved");
  rlb_status st = set_device(x);
  if (st != RLB_OK) return st;
  double* const dst[5] = {eps, ux, uy, uz, n};
  const hipError_t e = read_fields(x, x->scratch, dst);
  if (e != hipSuccess) return hip_fail(e, "moments (no allocation)");
  return RLB_OK;
}

int32_t rlb_steps_per_launch(const rlb_ctx* x) {
  if (!x) return 0;
  return (x->act_mask == 1 && x->cfg.lattice == RLB_LATTICE_EXTENDED) ? x->tb_steps : 1;
}

rlb_status rlb_stats_get(rlb_ctx* x, rlb_stats* out) {
  if (!x || !out) return fail(RLB_E_INVALID_ARG, "NULL argument");
  if (!x->initialised) return fail(RLB_E_STATE, "rlb_init_fields has not been called");
  rlb_status st = set_device(x);
  if (st != RLB_OK) return st;
  rlb::StepParams p = x->base;
  p.f_in = x->f[x->cur];
  p.h_in = x->h[x->cur];
  hipError_t e = rlb::launch_sums(p, x->fp64, x->cfg.with_density != 0, x->sums_partial, x->sums_blocks,
                                  x->sums_out, x->stream);
  double sums[5] = {0, 0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(sums, x->sums_out, sizeof sums, hipMemcpyDeviceToHost, x->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
  if (e != hipSuccess) return hip_fail(e, "stats");
  st = read_counters(x);
  if (st != RLB_OK) return st;
  if (x->host_counters[0] != kNoBadStep && x->first_bad < 0) {
    x->first_bad = static_cast<long long>(x->host_counters[0]);
    x->poisoned = true;
  }
  out->steps = x->steps;
  out->guard_events = static_cast<int64_t>(x->host_counters[1]);
  out->first_bad_step = x->first_bad;
  out->sum_T00 = sums[0];
  out->sum_T0x = sums[1];
  out->sum_T0y = sums[2];
  out->sum_T0z = sums[3];
  out->sum_N0 = sums[4];
  return RLB_OK;
}

const char* rlb_status_str(rlb_status s) {
  switch (s) {
    case RLB_OK: return "ok";
    case RLB_E_INVALID_ARG: return "invalid argument";
    case RLB_E_OUT_OF_MEMORY: return "out of device memory";
    case RLB_E_DEVICE: return "HIP device error";
    case RLB_E_INADMISSIBLE: return "inadmissible state";
    case RLB_E_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* rlb_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
