// rlb_internal.h -- types shared by the C-ABI host code and the HIP kernels
// of the ultra-relativistic lattice Boltzmann update (arXiv:1302.1125).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rlb {

constexpr int Q = 19;            // extended D3Q19 set, Sec. II.A, Eq. (42)
constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts)
constexpr int kXcds = 8;         // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kBcPeriodic = 0, kBcFixed = 1, kBcOutflow = 2;

// Everything a step kernel needs, passed by value (kernarg segment).
struct StepParams {
  const void* f_in;
  void* f_out;
  const void* h_in;
  void* h_out;
  double* hist;            // [5][ncell]: eps, ux, uy, uz, n of the previous step
  const uint8_t* obst;     // [ncell] or nullptr
  const double* face_eq;   // [6 faces][2: f,h][19] equilibria of FIXED faces
  long long ncell;
  int nx, ny, nz;
  int tile_x, tile_y;      // workgroup tile (tile_x * tile_y == kBlock)
  int ntx, nty;            // tiles along x and y
  long long ntiles;        // ntx * nty * nz
  long long tiles_per_xcd; // ceil(ntiles / kXcds)
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
  int guard;        // 0/1
  double m1, mmax, efloor;
  unsigned long long* bad_step;    // atomicMin of the first inadmissible step
  unsigned long long* guard_count; // cell-steps blended by the guard
  long long step_index;
};

// Launchers (rlb_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_step(const StepParams& p, bool fp64, int act_mask, bool with_h, bool euler,
                       hipStream_t s);
hipError_t launch_init(const StepParams& p, bool fp64, bool with_h, hipStream_t s);
hipError_t launch_face_eq(const StepParams& p, const double* face_states_dev, double* face_eq_dev,
                          hipStream_t s);
hipError_t launch_moments(const StepParams& p, bool fp64, bool with_h, double* out /*[5][ncell]*/,
                          unsigned long long* bad_flag, hipStream_t s);
hipError_t launch_sums(const StepParams& p, bool fp64, bool with_h, double* partial, int nblocks,
                       double* out5, hipStream_t s);

}  // namespace rlb
