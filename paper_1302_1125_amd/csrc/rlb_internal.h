// rlb_internal.h -- types shared by the C-ABI host code and the HIP kernels
// of the ultra-relativistic lattice Boltzmann update (arXiv:1302.1125).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rlb {

constexpr int Q = 19;            // extended D3Q19 set, Sec. II.A, Eq. (42)
constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts)
constexpr int kXcds = 8;         // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kFaceSlots = 6;    // per population: equilibria of the 6 faces
constexpr int kBcPeriodic = 0, kBcFixed = 1, kBcOutflow = 2;

// Population arrays hold pstride elements per population: storage cells
// [0, ncell) in the order x + px (y + py z), then one slot per face
// [ncell, ncell + 6) holding the equilibrium of that face's fixed state
// (written once at creation in both ping-pong copies).  A neighbour index
// that crosses a FIXED face points at the face slot, so boundary conditions
// are pure index mapping inside the step kernel.
//
// Padded storage of 2D/3D grids: each x-row holds px = nx rounded up to a
// multiple of 64 cells and each z-plane py = ny rounded up to a multiple of
// kBlock / 64 rows, i.e. exactly the cells covered by the 64 x 4 tiles of the
// step kernel.  Every lane of a ragged tile then owns a storage cell: lanes
// past the x or y end store their (discarded) results at their own pad cell,
// in the same coalesced row writes as their neighbours, instead of all lanes
// of the grid sharing one scratch slot (a single L2 line that serialised
// those stores: 4x at nx = 200).  Rows also start on 256-byte boundaries.
// Pad cells are written by those lanes only and never read.  1D grids and the
// serving arena keep px = nx, py = 1.  ncell here is the storage count
// px py nz; host fields stay dense [z][y][x].
constexpr int kRowAlign = 64;
inline int row_pitch(int nx, int ny) {
  return ny > 1 ? (nx + kRowAlign - 1) / kRowAlign * kRowAlign : nx;
}
inline int plane_rows(int ny) {
  constexpr int r = kBlock / 64;
  return ny > 1 ? (ny + r - 1) / r * r : ny;
}
// Elements per population array: the ncell storage cells and the kFaceSlots
// face slots, padded to a multiple of 64.
inline long long population_stride(long long ncell) {
  return (ncell + kFaceSlots + 63) / 64 * 64;
}

// Largest grid (storage cells px py nz) or serving arena in cells.  Kernels address every array by
// 32-bit byte offsets from a per-array base; with FP64 arrays (populations in
// FP64 mode, previous-step fields always) 8 * population_stride must stay
// below 2^31.  The serving arena obeys the same limit.
constexpr long long kMaxCells = (1ll << 28) - 128;

// Streaming flux of the extended model: the paper's minmod-limited upwind
// flux, or the first-order Rusanov flux (beyond the paper; k_step_tb in 1D,
// the staged k_step in 2D and 3D).
constexpr int kFluxMinmod = 0;
constexpr int kFluxRusanov = 1;

// Everything a step kernel needs, passed by value (kernarg segment).
struct StepParams {
  const void* f_in;
  void* f_out;
  const void* h_in;
  void* h_out;
  double* hist;            // [5][ncell]: eps, ux, uy, uz, n of the previous step
  // Temporally blocked 1D launches (k_step_tb) read hist and write the fields
  // they leave to hist_out, a second array of the same shape: a workgroup
  // reads the fields of halo cells that neighbouring workgroups own and
  // rewrite in the same launch, so the two must not alias.
  double* hist_out;
  // [5][ncell] FP32: eps, gamma ux, gamma uy, gamma uz, n of the previous step.
  // Used instead of hist by the implicit mixed-precision step of 2D and 3D grids
  // (nullptr otherwise); hist then keeps the initial (obstacle) fields.
  float* hist32;
  const uint8_t* obst;     // [ncell] or nullptr
  long long ncell;         // storage cells px * py * nz (pad cells included)
  long long pstride;       // elements per population array (population_stride)
  int nx, ny, nz;
  int px, py;              // row pitch, rows per plane (row_pitch, plane_rows)
  int lattice;             // 0: extended model (Sec. II.A), 1: basic model (Sec. II)
  // Workgroup tiling: tile_x * tile_y == kBlock cells of one z-plane, and a
  // traversal order that keeps stencil reuse inside one XCD's L2.  Tiles are
  // grouped into pencils of pw x ph tiles (pw divides ntx, ph divides nty).
  // order 0 (1D/2D): linear index runs x-tiles of a pencil fastest, then
  //   y-tiles, then z, then pencils; XCD k takes the k-th contiguous chunk.
  // order 1 (3D): XCD k takes z-slab [k zslab, (k+1) zslab); inside it the
  //   index runs the tiles of one pencil plane fastest, then z, then pencils.
  int order;
  int tile_x, tile_y;
  int ntx, nty;
  int pw, ph;
  int zslab;
  long long ntiles;        // tiles in the grid
  long long tiles_per_xcd; // tiles assigned to each XCD (grid = 8 * this)
  // z-marching step of 3D mixed-precision grids (k_step_zm): planes per run
  // (0: off), workgroups (columns x runs) in all and per XCD
  int zm_len;
  long long zm_total;
  long long zm_per_xcd;
  int bc[6];
  // lattice and run constants (FP64)
  double a_scale;   // nu^2 / 27: equilibrium amplitude A = a_scale * eps
  double r;         // c_t / c_0 = sqrt(27) / nu
  double rca;       // (c_t / c_0) c_a
  double ca, ca2;   // c_a = sqrt(13) / nu and its square
  double inv_r;     // c_0 / c_t
  double wp0, wp1, wp2;  // density weights, Eqs. (59)-(60)
  double k1;        // 4 sqrt(13/27): first-order equilibrium coefficient / (A gamma^2)
  double omega_c;   // c_0 nu dt / c_t; omega = omega_c / tau
  double kappa;     // omega_c * alpha (bulk term coefficient, delta x = 1)
  double dtv;       // dt * sqrt(13/27): dt times the streaming speed of |e^a| = 1
  double tau;       // uniform relaxation time
  double nu2_etas;  // nu^2 * eta/s
  int tau_mode;     // 0 uniform, 1 eta/s
  int flux;         // kFluxMinmod (Eqs. (47)-(53)) or kFluxRusanov (not the z-march or segments)
  int guard;        // 0/1
  double m1, mmax, efloor;
  double gmax;      // Lorentz factor at m_max (bounds gamma of projected moments)
  unsigned long long* bad_step;    // atomicMin of the first inadmissible step
  unsigned long long* guard_count; // cell-steps blended by the guard
  long long step_index;
  // Segment mode (many independent 1D domains in one arena, see SegDesc):
  const struct SegDesc* segs;  // device segment table
  const int2* tiles;           // per workgroup: (segment id or -1, tile within segment)
  const long long* gstep;      // device: global step at the start of the chunk
  int step_in_chunk;           // offset of this launch within the chunk
  long long cell0;             // first (dense) cell of k_init / k_moments ranges
  long long range;             // number of dense cells of k_init / k_moments ranges
};

// One independent 1D domain of the batched segment step.  Its cells occupy
// arena indices [base, base + n + 2): a left ghost, n interior cells, a right
// ghost.  Ghosts hold the equilibria of FIXED end states (written once); other
// boundary conditions are folded into the neighbour indices.
struct SegDesc {
  long long base;
  long long start;   // global step at which the segment takes its first step
  long long steps;   // steps to take; afterwards the kernel copies it forward
  int n;
  int bc_lo, bc_hi;
  int id;            // slot of the per-segment counters
  double nu2_etas;   // nu^2 eta/s of this request
  double kappa;      // omega_c * alpha of this request
  double tau;        // uniform relaxation time of this request
  unsigned long long* bad;    // [slots] first inadmissible local step
  unsigned long long* guard;  // [slots] guard events
};

// Launchers (rlb_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_step(const StepParams& p, bool fp64, int act_mask, bool with_h, bool euler,
                       hipStream_t s);
hipError_t launch_init(const StepParams& p, bool fp64, bool with_h, hipStream_t s);
hipError_t launch_face_slots(const StepParams& p, bool fp64, const double* face_states_dev,
                             void* f0, void* f1, void* h0, void* h1, hipStream_t s);
hipError_t launch_moments(const StepParams& p, bool fp64, bool with_h, double* out /*[5][ncell]*/,
                          unsigned long long* bad_flag, hipStream_t s);
hipError_t launch_sums(const StepParams& p, bool fp64, bool with_h, double* partial, int nblocks,
                       double* out5, hipStream_t s);
// Temporal blocking of 1D domains (extended lattice): kb in [1, kTbMaxSteps]
// steps per launch; each workgroup owns tb_cells_per_tile(kb) cells.  seg:
// p.tiles maps the grid onto segments (tiles of that many cells), else the
// grid covers the context's 1D domain.  The previous-step fields move from
// p.hist to p.hist_out, which must be a distinct array (hipErrorInvalidValue
// otherwise).  p.flux == kFluxRusanov selects the Rusanov flux (not in
// segment mode).
constexpr int kTbMaxSteps = 16;
int tb_cells_per_tile(int kb);
hipError_t launch_step_tb(const StepParams& p, bool fp64, bool with_h, bool euler, int kb,
                          bool seg, unsigned grid, hipStream_t s);
// Batched segment step over `grid` workgroups (p.tiles has >= grid entries).
hipError_t launch_seg_step(const StepParams& p, bool fp64, bool with_h, bool euler, unsigned grid,
                           hipStream_t s);
// Largest population stride (elements) of the z-marching step: ten FP32
// arrays of one descriptor group stay below 2^32 bytes.
constexpr long long kZmMaxStride = (1ll << 32) / (10 * 4) - 64;
// Allocation-free field read-back: a fixed device array (one per GPU, held
// until the process ends) that stages the five FP64 fields of k_moments for
// grids of at most kScratchCells cells.  scratch_address() returns its device
// address on `device`, which must be the current device; the first call per
// device looks it up (hipGetSymbolAddress), later calls return the cached
// pointer.  Only that pointer may be handed to kernels or copies.
constexpr long long kScratchCells = 1ll << 20;
constexpr int kScratchFields = 5;
hipError_t scratch_address(int device, double** out);
// Equilibria of a segment's two end states into its ghost cells (both copies).
hipError_t launch_seg_ghosts(const StepParams& p, bool fp64, long long lo_cell, long long hi_cell,
                             const double* states_dev /*2 x 5*/, void* f0, void* f1, void* h0,
                             void* h1, hipStream_t s);

}  // namespace rlb
