// rlb_server.cpp -- continuous batching of many independent 1D solves of the
// ultra-relativistic lattice Boltzmann update (arXiv:1302.1125) on one GPU.
//
// One device arena holds every resident request as a segment (ghost, n cells,
// ghost) of the population arrays; one fused launch per step advances all of
// them (k_step in segment mode), chained in hipGraph chunks.  A worker thread
// admits queued requests whenever an arena range and a slot are free, runs
// chunks while anything is resident, and retires finished requests (fields
// read back, memory freed).  All arithmetic of the update is in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/rlb.h"
#include "rlb_internal.h"

// shared with rlb_api.cpp
void rlb_fill_constants(const rlb_config& c, rlb::StepParams& p);
rlb_status rlb_validate_config(const rlb_config* c);
rlb_status rlb_set_error(rlb_status s, const std::string& msg);

namespace {

using Clock = std::chrono::steady_clock;

constexpr long long kAlign = 64;           // arena allocation unit (cells)
constexpr unsigned kGridBucket = 512;      // graph grid sizes are multiples of this
constexpr unsigned long long kNoBad = ~0ull;

enum ReqState { kPending = 0, kActive = 1, kDone = 2, kFailed = 3 };

struct Req {
  uint64_t id = 0;
  int n = 0;
  long long steps = 0;
  double eta_over_s = 0, tau = 1, alpha = 0;
  int bc_lo = RLB_BC_FIXED, bc_hi = RLB_BC_FIXED;
  double face[2][5] = {};
  std::vector<double> io;  // [5][n]: initial fields, then the result
  Clock::time_point arrival, done_at;
  int state = kPending;
  long long base = -1, cells = 0, start = 0;
  int slot = -1;
  long long first_bad = -1;
  unsigned long long guard = 0;
};

long long round_up(long long v, long long a) { return (v + a - 1) / a * a; }

}  // namespace

struct rlb_server {
  rlb_config cfg{};
  bool fp64 = false, with_h = false, euler = false;
  size_t elem = 4;
  long long cap = 0, pstride = 0;
  int max_slots = 0, chunk = 64;
  int tb = 1;          // steps per temporally blocked launch (1: one step per launch)
  int tile_cells = rlb::kBlock;  // cells per workgroup tile
  int device = 0;
  hipStream_t stream = nullptr;
  void* f[2] = {nullptr, nullptr};
  void* h[2] = {nullptr, nullptr};
  // previous-step fields, two copies: blocked launches read one and write the
  // other (a chunk has an even number of launches and ends on copy 0);
  // one-step launches update copy 0 in place
  double* hist[2] = {nullptr, nullptr};
  rlb::SegDesc* d_segs = nullptr;
  rlb::SegDesc* h_segs = nullptr;  // pinned
  int2* d_tiles = nullptr;
  int2* h_tiles = nullptr;         // pinned
  long long max_tiles = 0;
  long long* d_gstep = nullptr;
  long long* h_gstep = nullptr;    // pinned
  unsigned long long* d_bad = nullptr;
  unsigned long long* d_guard = nullptr;
  unsigned long long* h_bad = nullptr;       // pinned [max_slots] copy of d_bad
  unsigned long long* h_guard = nullptr;     // pinned [max_slots] copy of d_guard
  unsigned long long* h_reset = nullptr;     // pinned {kNoBad, 0}
  double* d_face = nullptr;                  // [max_slots][2][5]
  double* h_face = nullptr;                  // pinned [max_slots][2][5]
  double* d_out = nullptr;                   // moments staging
  double* h_out = nullptr;                   // pinned
  long long out_cells = 0;
  rlb::StepParams base{};
  std::map<unsigned, hipGraphExec_t> graphs;
  hipEvent_t ev = nullptr;

  // host-side scheduling state (worker thread + callers)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::unordered_map<uint64_t, Req> reqs;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> active;
  std::vector<int> free_slots;
  std::map<long long, long long> free_ranges;  // start -> length (cells)
  uint64_t next_id = 1;
  long long gstep = 0;
  bool tables_dirty = true;
  unsigned grid = 0;
  std::atomic<bool> stop{false};
  std::thread worker;
  std::string worker_error;

  // statistics
  uint64_t n_sub = 0, n_adm = 0, n_done = 0, n_fail = 0, n_rej = 0, n_chunks = 0;
  long long resident_cells = 0, peak_cells = 0, peak_reqs = 0;
  double cell_updates = 0, busy = 0;
  bool any_sub = false;
  Clock::time_point first_sub, last_done;
  std::vector<double> latencies;
};

namespace {

uint64_t bytes_per_cell(const rlb_config& c) {
  const uint64_t e = c.precision == RLB_FP64 ? 8 : 4;
  return 2 * rlb::Q * e * (c.with_density ? 2 : 1) + 2 * 5 * 8;
}

long long footprint_cells(int n) { return round_up(static_cast<long long>(n) + 2, kAlign); }

template <typename P>
hipError_t dmalloc(P** p, size_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  *p = static_cast<P*>(q);
  return e;
}

template <typename P>
hipError_t hmalloc(P** p, size_t bytes) {
  void* q = nullptr;
  hipError_t e = hipHostMalloc(&q, bytes);
  *p = static_cast<P*>(q);
  return e;
}

void free_server(rlb_server* s) {
  for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.second);
  s->graphs.clear();
  for (int k = 0; k < 2; ++k) {
    if (s->f[k]) (void)hipFree(s->f[k]);
    if (s->h[k]) (void)hipFree(s->h[k]);
  }
  void* dev[] = {s->hist[0], s->hist[1], s->d_segs, s->d_tiles, s->d_gstep,
                 s->d_bad,     s->d_guard,   s->d_face, s->d_out};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  void* host[] = {s->h_segs, s->h_tiles, s->h_gstep, s->h_guard, s->h_bad, s->h_reset, s->h_face,
                  s->h_out};
  for (void* p : host)
    if (p) (void)hipHostFree(p);
  if (s->ev) (void)hipEventDestroy(s->ev);
  if (s->stream) (void)hipStreamDestroy(s->stream);
}

// First-fit arena allocation; returns -1 if no range fits.
long long arena_alloc(rlb_server* s, long long cells) {
  for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it) {
    if (it->second < cells) continue;
    const long long at = it->first, len = it->second;
    s->free_ranges.erase(it);
    if (len > cells) s->free_ranges[at + cells] = len - cells;
    return at;
  }
  return -1;
}

void arena_free(rlb_server* s, long long at, long long cells) {
  auto it = s->free_ranges.emplace(at, cells).first;
  auto nx = std::next(it);
  if (nx != s->free_ranges.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    s->free_ranges.erase(nx);
  }
  if (it != s->free_ranges.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      s->free_ranges.erase(it);
    }
  }
}

// Graph of `chunk` segment-step launches over `grid` workgroups.
hipError_t graph_for(rlb_server* s, unsigned grid, hipGraphExec_t* out) {
  auto it = s->graphs.find(grid);
  if (it != s->graphs.end()) {
    *out = it->second;
    return hipSuccess;
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  // chunk / tb launches (an even number, so the chunk ends on copy 0)
  for (int j = 0; j < s->chunk / s->tb && e == hipSuccess; ++j) {
    rlb::StepParams p = s->base;
    p.f_in = s->f[j % 2];
    p.f_out = s->f[(j + 1) % 2];
    p.h_in = s->h[j % 2];
    p.h_out = s->h[(j + 1) % 2];
    if (s->tb > 1) {
      p.hist = s->hist[j % 2];
      p.hist_out = s->hist[(j + 1) % 2];
    }
    p.step_in_chunk = j * s->tb;
    e = s->tb > 1 ? rlb::launch_step_tb(p, s->fp64, s->with_h, s->euler, s->tb, true, grid, s->stream)
                  : rlb::launch_seg_step(p, s->fp64, s->with_h, s->euler, grid, s->stream);
  }
  hipError_t e2 = hipStreamEndCapture(s->stream, &g);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return e;
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return e;
  s->graphs[grid] = x;
  *out = x;
  return hipSuccess;
}

// Admit pending requests that fit (FIFO with backfill).  Called by the
// worker with the lock held; device work is enqueued on the server stream.
hipError_t admit(rlb_server* s) {
  for (auto it = s->pending.begin(); it != s->pending.end();) {
    Req& r = s->reqs[*it];
    if (s->free_slots.empty()) break;
    const long long cells = footprint_cells(r.n);
    const long long at = arena_alloc(s, cells);
    if (at < 0) {
      ++it;
      continue;
    }
    const int slot = s->free_slots.back();
    s->free_slots.pop_back();
    r.base = at;
    r.cells = cells;
    r.slot = slot;
    r.start = s->gstep;
    r.state = kActive;
    // fields into the previous-step array, then f := f^eq, h := h^eq in copy 0
    hipError_t e = hipSuccess;
    for (int k = 0; k < 5 && e == hipSuccess; ++k) {
      if (k == 4 && !s->with_h) continue;
      e = hipMemcpyAsync(s->hist[0] + k * s->cap + at + 1, r.io.data() + k * r.n, sizeof(double) * r.n,
                         hipMemcpyHostToDevice, s->stream);
    }
    if (e != hipSuccess) return e;
    rlb::StepParams p = s->base;
    p.f_out = s->f[0];
    p.h_out = s->h[0];
    p.cell0 = at + 1;
    p.range = r.n;
    e = rlb::launch_init(p, s->fp64, s->with_h, s->stream);
    if (e != hipSuccess) return e;
    double* hf = s->h_face + slot * 10;
    std::memcpy(hf, r.face, sizeof(r.face));
    e = hipMemcpyAsync(s->d_face + slot * 10, hf, 10 * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
      e = rlb::launch_seg_ghosts(s->base, s->fp64, at, at + 1 + r.n, s->d_face + slot * 10, s->f[0],
                                 s->f[1], s->h[0], s->h[1], s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->d_bad + slot, s->h_reset, sizeof(unsigned long long), hipMemcpyHostToDevice,
                         s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->d_guard + slot, s->h_reset + 1, sizeof(unsigned long long),
                         hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return e;
    rlb::SegDesc& d = s->h_segs[slot];
    d.base = at;
    d.start = r.start;
    d.steps = r.steps;
    d.n = r.n;
    d.bc_lo = r.bc_lo;
    d.bc_hi = r.bc_hi;
    d.id = slot;
    d.nu2_etas = s->cfg.nu * s->cfg.nu * r.eta_over_s;
    d.kappa = s->base.omega_c * r.alpha;
    d.tau = r.tau;
    d.bad = s->d_bad;
    d.guard = s->d_guard;
    s->active.push_back(r.id);
    s->resident_cells += cells;
    s->peak_cells = std::max(s->peak_cells, s->resident_cells);
    s->peak_reqs = std::max<long long>(s->peak_reqs, static_cast<long long>(s->active.size()));
    s->n_adm += 1;
    s->tables_dirty = true;
    it = s->pending.erase(it);
  }
  return hipSuccess;
}

hipError_t upload_tables(rlb_server* s) {
  long long nt = 0;
  for (uint64_t id : s->active) {
    const Req& r = s->reqs[id];
    const int tiles = (r.n + s->tile_cells - 1) / s->tile_cells;
    for (int t = 0; t < tiles; ++t) s->h_tiles[nt++] = make_int2(r.slot, t);
  }
  s->grid = static_cast<unsigned>(round_up(std::max<long long>(nt, 1), kGridBucket));
  if (s->grid > s->max_tiles) s->grid = static_cast<unsigned>(s->max_tiles);
  for (long long t = nt; t < s->grid; ++t) s->h_tiles[t] = make_int2(-1, 0);
  hipError_t e = hipMemcpyAsync(s->d_tiles, s->h_tiles, sizeof(int2) * s->grid, hipMemcpyHostToDevice,
                                s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_segs, s->h_segs, sizeof(rlb::SegDesc) * s->max_slots, hipMemcpyHostToDevice,
                       s->stream);
  s->tables_dirty = false;
  return e;
}

// Retire requests whose steps are done after the chunk that ended at
// s->gstep, and requests that met an inadmissible state (they end at the
// first chunk boundary after it).  s->h_bad holds the per-slot flags copied
// after the chunk.  The moments of all retiring requests are computed and
// copied back under one synchronisation.
hipError_t retire(rlb_server* s) {
  std::vector<uint64_t> done;
  long long total = 0;
  for (uint64_t id : s->active) {
    const Req& r = s->reqs[id];
    if (s->gstep - r.start >= r.steps || s->h_bad[r.slot] != kNoBad) {
      done.push_back(id);
      total += r.n;
    }
  }
  if (done.empty()) return hipSuccess;
  hipError_t e = hipSuccess;
  if (s->out_cells < total) {
    if (s->d_out) (void)hipFree(s->d_out);
    if (s->h_out) (void)hipHostFree(s->h_out);
    s->d_out = nullptr;
    s->h_out = nullptr;
    s->out_cells = std::max<long long>(total, 1 << 16);
    e = dmalloc(&s->d_out, 5 * sizeof(double) * s->out_cells);
    if (e == hipSuccess) e = hmalloc(&s->h_out, 5 * sizeof(double) * s->out_cells);
    if (e != hipSuccess) return e;
  }
  long long off = 0;
  for (uint64_t id : done) {
    const Req& r = s->reqs[id];
    rlb::StepParams p = s->base;
    p.f_in = s->f[0];  // chunks are even, so the current copy is 0
    p.h_in = s->h[0];
    p.cell0 = r.base + 1;
    p.range = r.n;
    e = rlb::launch_moments(p, s->fp64, s->with_h, s->d_out + 5 * off, s->d_bad + s->max_slots,
                            s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->h_guard + r.slot, s->d_guard + r.slot, sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return e;
    off += r.n;
  }
  e = hipMemcpyAsync(s->h_out, s->d_out, 5 * sizeof(double) * total, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return e;
  off = 0;
  for (uint64_t id : done) {
    Req& r = s->reqs[id];
    std::memcpy(r.io.data(), s->h_out + 5 * off, 5 * sizeof(double) * r.n);
    off += r.n;
    const unsigned long long bad = s->h_bad[r.slot];
    r.first_bad = bad == kNoBad ? -1 : static_cast<long long>(bad);
    r.guard = s->h_guard[r.slot];
    r.done_at = Clock::now();
    r.state = r.first_bad >= 0 ? kFailed : kDone;
    s->n_done += 1;
    if (r.first_bad >= 0) s->n_fail += 1;
    const long long ran = std::min<long long>(r.steps, s->gstep - r.start);
    s->cell_updates += static_cast<double>(r.n) * static_cast<double>(ran);
    s->latencies.push_back(std::chrono::duration<double>(r.done_at - r.arrival).count());
    s->last_done = r.done_at;
    arena_free(s, r.base, r.cells);
    s->resident_cells -= r.cells;
    s->free_slots.push_back(r.slot);
    s->active.erase(std::find(s->active.begin(), s->active.end(), id));
    s->tables_dirty = true;
  }
  s->cv_done.notify_all();
  return hipSuccess;
}

void worker_loop(rlb_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv_work.wait(lk, [&] { return s->stop.load() || !s->pending.empty() || !s->active.empty(); });
    if (s->stop.load()) break;
    hipError_t e = admit(s);
    if (e == hipSuccess && s->active.empty()) {
      // an empty arena fits any accepted request, so this cannot persist;
      // fail the head rather than spin
      if (!s->pending.empty()) {
        s->reqs[s->pending.front()].state = kFailed;
        s->pending.pop_front();
        s->cv_done.notify_all();
      }
      continue;
    }
    if (e == hipSuccess && s->tables_dirty) e = upload_tables(s);
    hipGraphExec_t g = nullptr;
    if (e == hipSuccess) e = graph_for(s, s->grid, &g);
    if (e == hipSuccess) {
      *s->h_gstep = s->gstep;
      e = hipMemcpyAsync(s->d_gstep, s->h_gstep, sizeof(long long), hipMemcpyHostToDevice, s->stream);
    }
    const auto t0 = Clock::now();
    if (e == hipSuccess) e = hipGraphLaunch(g, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->h_bad, s->d_bad, sizeof(unsigned long long) * s->max_slots,
                         hipMemcpyDeviceToHost, s->stream);
    // let callers submit while the chunk runs
    lk.unlock();
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    lk.lock();
    s->busy += std::chrono::duration<double>(Clock::now() - t0).count();
    s->n_chunks += 1;
    s->gstep += s->chunk;
    if (e == hipSuccess) e = retire(s);
    if (e != hipSuccess) {
      s->worker_error = std::string("server loop: ") + hipGetErrorString(e);
      for (uint64_t id : s->active) s->reqs[id].state = kFailed;
      for (uint64_t id : s->pending) s->reqs[id].state = kFailed;
      s->active.clear();
      s->pending.clear();
      s->cv_done.notify_all();
      break;
    }
  }
  // requests still queued when the loop stops fail
  for (uint64_t id : s->pending) s->reqs[id].state = kFailed;
  for (uint64_t id : s->active) s->reqs[id].state = kFailed;
  s->cv_done.notify_all();
}

rlb_status check_request(const rlb_server* s, const rlb_request* r) {
  if (!r || r->struct_size != sizeof(rlb_request)) return rlb_set_error(RLB_E_INVALID_ARG, "request struct_size");
  if (r->n < 4 || r->steps < 0) return rlb_set_error(RLB_E_INVALID_ARG, "request: n >= 4, steps >= 0");
  if (!r->eps || !r->ux || !r->uy || !r->uz || (s->with_h && !r->dens))
    return rlb_set_error(RLB_E_INVALID_ARG, "request fields missing");
  auto bc_ok = [](int b) { return b == RLB_BC_PERIODIC || b == RLB_BC_FIXED || b == RLB_BC_OUTFLOW; };
  if (!bc_ok(r->bc_lo) || !bc_ok(r->bc_hi) || ((r->bc_lo == RLB_BC_PERIODIC) != (r->bc_hi == RLB_BC_PERIODIC)))
    return rlb_set_error(RLB_E_INVALID_ARG, "request boundary conditions");
  if (!(r->alpha >= 0 && std::isfinite(r->alpha)) || !(r->eta_over_s >= 0 && std::isfinite(r->eta_over_s)))
    return rlb_set_error(RLB_E_INVALID_ARG, "request alpha / eta_over_s");
  if (s->cfg.tau_mode == RLB_TAU_UNIFORM && !(r->tau > 0 && std::isfinite(r->tau)))
    return rlb_set_error(RLB_E_INVALID_ARG, "request tau");
  const double* faces[2] = {r->face_lo, r->face_hi};
  const int bcs[2] = {r->bc_lo, r->bc_hi};
  for (int k = 0; k < 2; ++k) {
    if (bcs[k] != RLB_BC_FIXED) continue;
    const double* q = faces[k];
    const double u2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    bool ok = std::isfinite(q[0]) && q[0] > 0 && std::isfinite(u2) && u2 < 1.0;
    if (s->with_h) ok = ok && std::isfinite(q[4]) && q[4] > 0;
    if (!ok) return rlb_set_error(RLB_E_INVALID_ARG, "inadmissible end state");
  }
  for (int c = 0; c < r->n; ++c) {
    const double u2 = r->ux[c] * r->ux[c] + r->uy[c] * r->uy[c] + r->uz[c] * r->uz[c];
    bool ok = std::isfinite(r->eps[c]) && r->eps[c] > 0 && std::isfinite(u2) && u2 < 1.0;
    if (s->with_h) ok = ok && std::isfinite(r->dens[c]) && r->dens[c] > 0;
    if (!ok) return rlb_set_error(RLB_E_INADMISSIBLE, "inadmissible initial state");
  }
  if (footprint_cells(r->n) > s->cap)
    return rlb_set_error(RLB_E_OUT_OF_MEMORY, "request larger than the server arena");
  return RLB_OK;
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (v.size() - 1);
  const size_t lo = static_cast<size_t>(std::floor(pos)), hi = static_cast<size_t>(std::ceil(pos));
  return v[lo] + (v[hi] - v[lo]) * (pos - lo);
}

}  // namespace

extern "C" {

uint64_t rlb_request_footprint_bytes(const rlb_config* common, int32_t n) {
  if (!common || n < 1) return 0;
  return static_cast<uint64_t>(footprint_cells(n)) * bytes_per_cell(*common);
}

rlb_status rlb_server_create(const rlb_config* common, uint64_t budget_bytes, int32_t chunk_steps,
                             rlb_server** out) {
  if (!out) return rlb_set_error(RLB_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!common) return rlb_set_error(RLB_E_INVALID_ARG, "config is NULL");
  rlb_config c = *common;
  c.nx = 8;
  c.ny = c.nz = 1;
  for (int k = 0; k < 6; ++k) c.bc[k] = RLB_BC_PERIODIC;
  if (c.tau_mode == RLB_TAU_UNIFORM && !(c.tau > 0)) c.tau = 1.0;
  rlb_status st = rlb_validate_config(&c);
  if (st != RLB_OK) return st;
  if (c.lattice != RLB_LATTICE_EXTENDED)
    return rlb_set_error(RLB_E_INVALID_ARG, "the server runs the extended lattice only");
  if (c.flux != RLB_FLUX_MINMOD) return rlb_set_error(RLB_E_INVALID_ARG, "the server runs the minmod flux only");
  if (chunk_steps < 2 || chunk_steps % 2 != 0 || chunk_steps > 4096)
    return rlb_set_error(RLB_E_INVALID_ARG, "chunk_steps must be even, 2..4096");
  const uint64_t bpc = bytes_per_cell(c);
  long long cap = static_cast<long long>(budget_bytes / bpc) / kAlign * kAlign;
  cap = std::min(cap, rlb::kMaxCells / kAlign * kAlign);
  if (cap < kAlign * 2) return rlb_set_error(RLB_E_INVALID_ARG, "budget too small");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return rlb_set_error(RLB_E_DEVICE, "no HIP device available (this library has no CPU path)");
  }
  rlb_server* s = new (std::nothrow) rlb_server();
  if (!s) return rlb_set_error(RLB_E_OUT_OF_MEMORY, "host allocation");
  (void)hipGetDevice(&s->device);
  s->cfg = c;
  s->fp64 = c.precision == RLB_FP64;
  s->with_h = c.with_density != 0;
  s->euler = c.collision == RLB_COLL_EULER;
  s->elem = s->fp64 ? 8 : 4;
  s->cap = cap;
  s->pstride = rlb::population_stride(cap);
  s->chunk = chunk_steps;
  {
    // temporal blocking: the largest tb <= the requested steps per launch
    // (default 8; RLB_TB_STEPS tuning override, 1 = off) with an even number
    // of launches per chunk
    int want = 8;
    if (const char* v = std::getenv("RLB_TB_STEPS")) want = std::atoi(v);
    want = std::max(1, std::min(want, rlb::kTbMaxSteps));
    s->tb = 1;
    for (int d = want; d > 1; --d)
      if (chunk_steps % (2 * d) == 0) {
        s->tb = d;
        break;
      }
    s->tile_cells = s->tb > 1 ? rlb::tb_cells_per_tile(s->tb) : rlb::kBlock;
  }
  s->max_slots = static_cast<int>(std::min<long long>(65536, cap / kAlign));
  s->max_tiles = round_up(cap / s->tile_cells + s->max_slots + 1, kGridBucket);
  hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  const size_t pop = static_cast<size_t>(rlb::Q) * s->pstride * s->elem;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = dmalloc(&s->f[k], pop);
    if (e == hipSuccess && s->with_h) e = dmalloc(&s->h[k], pop);
  }
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = dmalloc(&s->hist[k], 5 * sizeof(double) * cap);
  if (e == hipSuccess) e = dmalloc(&s->d_segs, sizeof(rlb::SegDesc) * s->max_slots);
  if (e == hipSuccess) e = hmalloc(&s->h_segs, sizeof(rlb::SegDesc) * s->max_slots);
  if (e == hipSuccess) e = dmalloc(&s->d_tiles, sizeof(int2) * s->max_tiles);
  if (e == hipSuccess) e = hmalloc(&s->h_tiles, sizeof(int2) * s->max_tiles);
  if (e == hipSuccess) e = dmalloc(&s->d_gstep, sizeof(long long));
  if (e == hipSuccess) e = hmalloc(&s->h_gstep, sizeof(long long));
  if (e == hipSuccess) e = dmalloc(&s->d_bad, sizeof(unsigned long long) * (s->max_slots + 1));
  if (e == hipSuccess) e = dmalloc(&s->d_guard, sizeof(unsigned long long) * s->max_slots);
  if (e == hipSuccess) e = hmalloc(&s->h_guard, sizeof(unsigned long long) * s->max_slots);
  if (e == hipSuccess) e = hmalloc(&s->h_bad, sizeof(unsigned long long) * s->max_slots);
  if (e == hipSuccess) e = hmalloc(&s->h_reset, sizeof(unsigned long long) * 2);
  if (e == hipSuccess) e = dmalloc(&s->d_face, sizeof(double) * 10 * s->max_slots);
  if (e == hipSuccess) e = hmalloc(&s->h_face, sizeof(double) * 10 * s->max_slots);
  if (e == hipSuccess) e = hipEventCreate(&s->ev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    free_server(s);
    delete s;
    return rlb_set_error(RLB_E_OUT_OF_MEMORY, std::string("server allocation: ") + hipGetErrorString(e));
  }
  s->h_reset[0] = kNoBad;
  s->h_reset[1] = 0;
  std::memset(s->h_segs, 0, sizeof(rlb::SegDesc) * s->max_slots);
  rlb_fill_constants(c, s->base);
  s->base.ncell = cap;
  s->base.pstride = s->pstride;
  s->base.nx = static_cast<int>(std::min<long long>(cap, 1 << 30));
  s->base.ny = s->base.nz = 1;
  s->base.px = s->base.nx;
  s->base.py = 1;
  s->base.hist = s->hist[0];
  s->base.obst = nullptr;
  s->base.segs = s->d_segs;
  s->base.tiles = s->d_tiles;
  s->base.gstep = s->d_gstep;
  s->base.bad_step = s->d_bad + s->max_slots;
  s->base.guard_count = s->d_guard;
  for (int k = s->max_slots - 1; k >= 0; --k) s->free_slots.push_back(k);
  s->free_ranges[0] = cap;
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return RLB_OK;
}

rlb_status rlb_server_submit(rlb_server* s, const rlb_request* r, uint64_t* id) {
  if (!s || !id) return rlb_set_error(RLB_E_INVALID_ARG, "NULL argument");
  const auto now = Clock::now();
  rlb_status st = check_request(s, r);
  std::lock_guard<std::mutex> lk(s->mu);
  if (st != RLB_OK) {
    if (st == RLB_E_OUT_OF_MEMORY) s->n_rej += 1;
    return st;
  }
  if (!s->worker_error.empty()) return rlb_set_error(RLB_E_DEVICE, s->worker_error);
  Req q;
  q.id = s->next_id++;
  q.n = r->n;
  q.steps = r->steps;
  q.eta_over_s = r->eta_over_s;
  q.tau = r->tau;
  q.alpha = r->alpha;
  q.bc_lo = r->bc_lo;
  q.bc_hi = r->bc_hi;
  std::memcpy(q.face[0], r->face_lo, sizeof(q.face[0]));
  std::memcpy(q.face[1], r->face_hi, sizeof(q.face[1]));
  q.io.resize(5 * static_cast<size_t>(r->n));
  const double* src[5] = {r->eps, r->ux, r->uy, r->uz, r->dens};
  for (int k = 0; k < 5; ++k)
    if (src[k]) std::memcpy(q.io.data() + k * r->n, src[k], sizeof(double) * r->n);
  q.arrival = now;
  if (!s->any_sub) {
    s->any_sub = true;
    s->first_sub = now;
  }
  *id = q.id;
  s->pending.push_back(q.id);
  s->reqs.emplace(q.id, std::move(q));
  s->n_sub += 1;
  s->cv_work.notify_one();
  return RLB_OK;
}

rlb_status rlb_server_poll(rlb_server* s, uint64_t id, int32_t* done) {
  if (!s || !done) return rlb_set_error(RLB_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return rlb_set_error(RLB_E_INVALID_ARG, "unknown request id");
  *done = it->second.state >= kDone ? 1 : 0;
  return RLB_OK;
}

rlb_status rlb_server_result(rlb_server* s, uint64_t id, double* eps, double* ux, double* uy, double* uz,
                             double* n, double* latency_s, int64_t* first_bad, int64_t* guard_events) {
  if (!s) return rlb_set_error(RLB_E_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->reqs.find(id) == s->reqs.end()) return rlb_set_error(RLB_E_INVALID_ARG, "unknown request id");
  // iterators of the map may be invalidated by submissions while waiting
  s->cv_done.wait(lk, [&] { return s->reqs.find(id)->second.state >= kDone; });
  auto it = s->reqs.find(id);
  Req& r = it->second;
  if (r.done_at.time_since_epoch().count() == 0) {
    const std::string msg = s->worker_error.empty() ? "server stopped before the request ran" : s->worker_error;
    s->reqs.erase(it);
    return rlb_set_error(RLB_E_DEVICE, msg);
  }
  double* dst[5] = {eps, ux, uy, uz, n};
  for (int k = 0; k < 5; ++k)
    if (dst[k]) std::memcpy(dst[k], r.io.data() + k * r.n, sizeof(double) * r.n);
  if (latency_s) *latency_s = std::chrono::duration<double>(r.done_at - r.arrival).count();
  if (first_bad) *first_bad = r.first_bad;
  if (guard_events) *guard_events = static_cast<int64_t>(r.guard);
  const bool bad = r.first_bad >= 0;
  s->reqs.erase(it);
  if (bad) return rlb_set_error(RLB_E_INADMISSIBLE, "a step of the request was inadmissible");
  return RLB_OK;
}

rlb_status rlb_server_drain(rlb_server* s) {
  if (!s) return rlb_set_error(RLB_E_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return (s->pending.empty() && s->active.empty()) || !s->worker_error.empty(); });
  if (!s->worker_error.empty()) return rlb_set_error(RLB_E_DEVICE, s->worker_error);
  return RLB_OK;
}

rlb_status rlb_server_stats_get(rlb_server* s, rlb_server_stats* o) {
  if (!s || !o) return rlb_set_error(RLB_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(o, 0, sizeof(*o));
  o->submitted = s->n_sub;
  o->admitted = s->n_adm;
  o->completed = s->n_done;
  o->failed = s->n_fail;
  o->rejected = s->n_rej;
  o->capacity_cells = static_cast<uint64_t>(s->cap);
  o->resident_cells_peak = static_cast<uint64_t>(s->peak_cells);
  o->resident_requests_peak = static_cast<uint64_t>(s->peak_reqs);
  o->chunks = s->n_chunks;
  o->global_steps = static_cast<uint64_t>(s->gstep);
  o->cell_updates = s->cell_updates;
  o->busy_seconds = s->busy;
  if (s->any_sub && s->n_done > 0)
    o->wall_seconds = std::chrono::duration<double>(s->last_done - s->first_sub).count();
  o->latency_p50 = percentile(s->latencies, 0.50);
  o->latency_p99 = percentile(s->latencies, 0.99);
  o->latency_max = s->latencies.empty() ? 0.0 : *std::max_element(s->latencies.begin(), s->latencies.end());
  return RLB_OK;
}

void rlb_server_destroy(rlb_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop.store(true);
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipStreamSynchronize(s->stream);
  free_server(s);
  delete s;
}

}  // extern "C"
