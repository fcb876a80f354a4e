// rlb_kernels.hip -- gfx950 kernels of the ultra-relativistic lattice
// Boltzmann update of Mohseni, Mendoza, Succi and Herrmann (arXiv:1302.1125).
//
// Data layout (HBM): populations structure-of-arrays f[i][cell] and
// h[i][cell] with cell = x + px (y + py z) (2D/3D rows and planes padded to
// the 64 x 4 tiles, rlb_internal.h) and a per-population stride that leaves
// six face slots after the cells; two copies (ping-pong).  The fields of the previous step hist[k][cell]
// (FP64, k = eps, ux, uy, uz, n) are read and rewritten in place by their cell;
// the implicit mixed-precision step of 2D/3D grids keeps them in FP32 as
// hist32[k][cell] (k = eps, gamma ux, gamma uy, gamma uz, n) instead.
//
// One fused kernel per step, one thread per cell, one workgroup per tile
// (64 x 4 cells in 2D/3D, 256 cells in 1D).  The thread loads the 38 centre
// values of its cell, forms the moments (FP64 accumulation), recovers the
// fields and builds the equilibrium coefficients in FP64.  In 2D/3D the
// tile's centre values, one halo row per wavefront and the halo cells of
// each row are then staged in LDS a few populations at a time, so that every
// x and y neighbour of the star stencil is an LDS read (z neighbours are
// global loads); in 1D the neighbours are global loads through precomputed,
// boundary-aware offsets.  Per population the thread evaluates the
// minmod-limited flux divergence, the bulk Laplacian and the implicit
// collision in the storage precision and stores the result at once.  The
// admissibility guard is gated by a cheap storage-precision test of the new
// moments with a rounding margin, and re-decided in FP64 from the stored
// values.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "rlb_internal.h"

namespace rlb {
namespace {

// ---------------------------------------------------------------------------
// Velocity set (Sec. II.A, Eq. (42)): rest, the six unit axis vectors and the
// twelve vectors 2(+-1,+-1,0) with permutations.  Canonical order of this
// library (internal; the ABI exposes fields only).
// ---------------------------------------------------------------------------
struct Vel {
  int x, y, z;
};

__host__ __device__ constexpr Vel vel(int i) {
  switch (i) {
    case 0: return {0, 0, 0};
    case 1: return {1, 0, 0};
    case 2: return {-1, 0, 0};
    case 3: return {0, 1, 0};
    case 4: return {0, -1, 0};
    case 5: return {0, 0, 1};
    case 6: return {0, 0, -1};
    case 7: return {2, 2, 0};
    case 8: return {-2, -2, 0};
    case 9: return {2, -2, 0};
    case 10: return {-2, 2, 0};
    case 11: return {2, 0, 2};
    case 12: return {-2, 0, -2};
    case 13: return {2, 0, -2};
    case 14: return {-2, 0, 2};
    case 15: return {0, 2, 2};
    case 16: return {0, -2, -2};
    case 17: return {0, 2, -2};
    default: return {0, -2, 2};
  }
}

__host__ __device__ constexpr int vcomp(int i, int a) {
  return a == 0 ? vel(i).x : (a == 1 ? vel(i).y : vel(i).z);
}

// Weights of the extended set after substituting c_a = sqrt(13)/nu and
// c_t/c_0 = sqrt(27)/nu into Eqs. (43)-(45): nu cancels.
__host__ __device__ constexpr double weight(int i) {
  return i == 0 ? -539.0 / 676.0 : (i <= 6 ? 99.0 / 338.0 : 9.0 / 2704.0);
}

// Lattice L = 0: the extended set above; L = 1: the basic D3Q19 set of
// Sec. II (diagonal links (+-1, +-1, 0), c_a = sqrt(19)/nu), whose weights
// after the same substitution are -44/361, 99/722 and 9/361.
template <int L>
__host__ __device__ constexpr Vel vel_l(int i) {
  const int d = (L == 1 && i >= 7) ? 2 : 1;
  return Vel{vel(i).x / d, vel(i).y / d, vel(i).z / d};
}
template <int L>
__host__ __device__ constexpr double weight_l(int i) {
  return L == 0 ? weight(i) : (i == 0 ? -44.0 / 361.0 : (i <= 6 ? 99.0 / 722.0 : 9.0 / 361.0));
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <int ACT>
__host__ __device__ constexpr bool axis_on(int a) {
  return (ACT >> a) & 1;
}

template <int ACT>
__host__ __device__ constexpr int n_axes() {
  return (ACT & 1) + ((ACT >> 1) & 1) + ((ACT >> 2) & 1);
}

// ---------------------------------------------------------------------------
// Equilibria as linear forms in 10 coefficients:
// bracket_i(K) = K0 + sum_a e^a K[1+a] + sum_a (e^a)^2 K[4+a]
//              + e^x e^y K7 + e^x e^z K8 + e^y e^z K9.
// ---------------------------------------------------------------------------
template <int I, int L = 0, typename C>
__device__ __forceinline__ C bracket(const C* K) {
  constexpr Vel e = vel_l<L>(I);
  C s = K[0];
  if constexpr (e.x != 0) s += C(e.x) * K[1] + C(e.x * e.x) * K[4];
  if constexpr (e.y != 0) s += C(e.y) * K[2] + C(e.y * e.y) * K[5];
  if constexpr (e.z != 0) s += C(e.z) * K[3] + C(e.z * e.z) * K[6];
  if constexpr (e.x * e.y != 0) s += C(e.x * e.y) * K[7];
  if constexpr (e.x * e.z != 0) s += C(e.x * e.z) * K[8];
  if constexpr (e.y * e.z != 0) s += C(e.y * e.z) * K[9];
  return s;
}

// f^eq_i = w_i bracket_i(K) (moment-exact reading of Eq. (29), fixed by
// Eq. (36) with eps = 3p): A = nu^2 eps / 27, G = A gamma^2,
// K0 = A - 16/15 G |u|^2, K_a = 4 sqrt(13/27) G u^a, K_aa = 52/15 G (u^a)^2,
// K_ab = 13 G u^a u^b.  The basic set has the same moments up to fourth
// order, so the same polynomial in xi_i = c_a e_i: with (c_a nu)^2 = 19
// instead of 13, K_a = 4 sqrt(19/27) G u^a (P.k1), K_aa = 76/15 G (u^a)^2,
// K_ab = 19 G u^a u^b.
template <int L = 0>
__device__ __forceinline__ void feq_coeffs(const StepParams& P, double eps, double ux, double uy,
                                           double uz, double g2, double* K) {
  constexpr double kaa = L == 0 ? 52.0 / 15.0 : 76.0 / 15.0;
  constexpr double kab = L == 0 ? 13.0 : 19.0;
  const double A = P.a_scale * eps;
  const double G = A * g2;
  const double u2 = ux * ux + uy * uy + uz * uz;
  K[0] = A - (16.0 / 15.0) * G * u2;
  const double c1 = P.k1 * G;
  K[1] = c1 * ux;
  K[2] = c1 * uy;
  K[3] = c1 * uz;
  const double c2 = kaa * G;
  K[4] = c2 * ux * ux;
  K[5] = c2 * uy * uy;
  K[6] = c2 * uz * uz;
  const double c3 = kab * G;
  K[7] = c3 * ux * uy;
  K[8] = c3 * ux * uz;
  K[9] = c3 * uy * uz;
}

// h^eq_i = w'_i bracket_i(H), Eq. (58): B = n gamma,
// H0 = B (c_0/c_t - 3/2 |u|^2), H_a = 3 c_a B u^a, H_aa = 9/2 c_a^2 B (u^a)^2,
// H_ab = 9 c_a^2 B u^a u^b.
__device__ __forceinline__ void heq_coeffs(const StepParams& P, double n, double ux, double uy,
                                           double uz, double gam, double* H) {
  const double B = n * gam;
  const double u2 = ux * ux + uy * uy + uz * uz;
  H[0] = B * (P.inv_r - 1.5 * u2);
  const double c1 = 3.0 * P.ca * B;
  H[1] = c1 * ux;
  H[2] = c1 * uy;
  H[3] = c1 * uz;
  const double c2 = 4.5 * P.ca2 * B;
  H[4] = c2 * ux * ux;
  H[5] = c2 * uy * uy;
  H[6] = c2 * uz * uz;
  H[7] = 2.0 * c2 * ux * uy;
  H[8] = 2.0 * c2 * ux * uz;
  H[9] = 2.0 * c2 * uy * uz;
}

template <int I>
__device__ __forceinline__ double wprime(const StepParams& P) {
  return I == 0 ? P.wp0 : (I <= 6 ? P.wp1 : P.wp2);
}

// Fields from T^{00} = E, T^{0a} = M^a, N^0 with eps = 3p:
// eps = 3 (E^2 - |M|^2) / (E + sqrt(4 E^2 - 3 |M|^2)), gamma^2 = (3E + eps)/(4 eps),
// u^a = 3 M^a / (4 eps gamma^2), n = N^0 / gamma.
struct Fields {
  double eps, ux, uy, uz, g2, gam, n;
};

template <bool WH>
__device__ __forceinline__ bool recover(double E, double Mx, double My, double Mz, double N0,
                                        Fields& F) {
  const double M2 = Mx * Mx + My * My + Mz * Mz;
  bool ok = (E > 0.0) && (M2 < E * E) && isfinite(E) && isfinite(M2);
  if constexpr (WH) ok = ok && (N0 > 0.0) && isfinite(N0);
  const double Mabs = sqrt(M2);
  const double S = sqrt(fmax(4.0 * E * E - 3.0 * M2, 0.0));
  const double eps = 3.0 * (E - Mabs) * (E + Mabs) / (E + S);
  const double g2 = (3.0 * E + eps) / (4.0 * eps);
  const double k = 3.0 / (4.0 * eps * g2);
  F.eps = ok ? eps : NAN;
  F.ux = k * Mx;
  F.uy = k * My;
  F.uz = k * Mz;
  F.g2 = g2;
  F.gam = sqrt(g2);
  if constexpr (WH) F.n = N0 / F.gam;
  else F.n = pow(eps / 3.0, 0.75);
  return ok;
}

// Local relaxation time: uniform, or Eq. (41) with the entropy density of
// Sec. III, s = n (4 - ln lambda), lambda = n / T^3, T = p / n (lattice units);
// without density lambda = 1 and n = T^3 so tau = 1/2 + nu^2 (eta/s) / T.
// In mixed precision the relaxation time (a rate of the FP32 collision) is
// evaluated in FP32.
#ifndef RLB_TAU_F64
#define RLB_TAU_F64 0
#endif
template <typename T, bool WH>
__device__ __forceinline__ double tau_of(const StepParams& P, const Fields& F, double tau_u,
                                         double nu2_etas) {
  if (P.tau_mode == 0) return tau_u;
  if constexpr (sizeof(T) == 4 && !RLB_TAU_F64) {
    const float eps = static_cast<float>(F.eps), n = static_cast<float>(F.n);
    const float p = eps * (1.0f / 3.0f);
    const float c = static_cast<float>(nu2_etas);
    if constexpr (WH) {
      // ln lambda = ln n - 3 ln T = 4 ln n - 3 ln p (no overflow of T^3)
      const float s = n * (4.0f - (4.0f * __logf(n) - 3.0f * __logf(p)));
      return 0.5 + static_cast<double>(c * s / (eps + p));
    } else {
      return 0.5 + static_cast<double>(c * __frsqrt_rn(__fsqrt_rn(p)));
    }
  } else {
    const double p = F.eps / 3.0;
    if constexpr (WH) {
      const double T_ = p / F.n;
      const double lam = F.n / (T_ * T_ * T_);
      const double s = F.n * (4.0 - log(lam));
      return 0.5 + nu2_etas * s / (F.eps + p);
    } else {
      return 0.5 + nu2_etas / sqrt(sqrt(p));
    }
  }
}

// minmod(X, Y), Eq. (53): the argument of smaller magnitude when both have
// the same sign, otherwise 0.  That is exactly the median of (X, Y, 0): one
// v_med3_f32 in single precision.
__device__ __forceinline__ float mmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double mmod(double a, double b) {
  return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// Difference of limited interface values between x + 1/2 and x - 1/2 for a
// positive streaming speed (left states): values at x-2, x-1, x, x+1.
template <typename T>
__device__ __forceinline__ T dflux_pos(T m2, T m1, T c0, T p1) {
  const T d0 = c0 - m1;
  return d0 + T(0.5) * (mmod(p1 - c0, d0) - mmod(d0, m1 - m2));
}

// Same for a negative speed (right states): values at x-1, x, x+1, x+2.
template <typename T>
__device__ __forceinline__ T dflux_neg(T m1, T c0, T p1, T p2) {
  const T d1 = p1 - c0;
  return d1 - T(0.5) * (mmod(p2 - p1, d1) - mmod(d1, c0 - m1));
}

// Byte offsets (32-bit) of a cell and of its neighbours within one
// population array, for offsets -2, -1, +1, +2 along each active axis, with
// periodic wrap, outflow clamp or the face slot of a FIXED face folded in.
// Loads then take the form base_i + offset with base_i = array + i * stride
// uniform across the wavefront (scalar base, 32-bit vector offset).
template <int ACT>
struct Nbr {
  unsigned c;        // byte offset of the value this lane loads (its cell)
  unsigned cs;       // byte offset its results are stored at (its own storage cell)
  unsigned hr, hx;   // staged tiles: halo row / halo column position this lane loads
  unsigned o[3][4];
};

template <typename T, int ACT>
__device__ __forceinline__ void make_nbr(const StepParams& P, int x, int y, int z, Nbr<ACT>& N) {
  const int co[3] = {x, y, z};
  const int n[3] = {P.nx, P.ny, P.nz};
  const long long st[3] = {1, P.px, static_cast<long long>(P.px) * P.py};
  const long long c = x + static_cast<long long>(P.px) * (y + static_cast<long long>(P.py) * z);
  N.c = static_cast<unsigned>(c) * static_cast<unsigned>(sizeof(T));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!axis_on<ACT>(a)) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = j < 2 ? j - 2 : j - 1;
      const int q = co[a] + k;
      long long idx = c + k * st[a];
      if (q < 0 || q >= n[a]) {
        const int side = q < 0 ? 0 : 1;
        const int b = P.bc[2 * a + side];
        if (b == kBcFixed) idx = P.ncell + 2 * a + side;
        else if (b == kBcPeriodic) idx = c + (q < 0 ? k + n[a] : k - n[a]) * st[a];
        else idx = c + ((q < 0 ? 0 : n[a] - 1) - co[a]) * st[a];
      }
      N.o[a][j] = static_cast<unsigned>(idx) * static_cast<unsigned>(sizeof(T));
    }
  }
  N.cs = N.c;
}

// Neighbour byte offsets of interior cell `local` of a batched 1D segment
// (arena layout of SegDesc: ghost, n cells, ghost).
template <typename T>
__device__ __forceinline__ void make_seg_nbr(const SegDesc& sd, int local, Nbr<1>& N) {
  const long long c = sd.base + 1 + local;
  N.c = static_cast<unsigned>(c) * static_cast<unsigned>(sizeof(T));
  N.cs = N.c;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = j < 2 ? j - 2 : j - 1;
    const int q = local + k;
    long long idx = c + k;
    if (q < 0) {
      idx = sd.bc_lo == kBcFixed ? sd.base : (sd.bc_lo == kBcPeriodic ? c + k + sd.n : sd.base + 1);
    } else if (q >= sd.n) {
      idx = sd.bc_hi == kBcFixed ? sd.base + 1 + sd.n
                                 : (sd.bc_hi == kBcPeriodic ? c + k - sd.n : sd.base + sd.n);
    }
    N.o[0][j] = static_cast<unsigned>(idx) * static_cast<unsigned>(sizeof(T));
  }
}

template <typename T>
__device__ __forceinline__ T ldb(const T* __restrict__ base, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}

template <typename T>
__device__ __forceinline__ void stb(T* __restrict__ base, unsigned off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off) = v;
}

// Streaming (non-temporal) accesses for data touched once per step: the new
// populations and the previous-step fields.  They leave L2 capacity to the
// stencil halos that neighbouring workgroups re-read.
#ifndef RLB_STREAMING
#define RLB_STREAMING 1
#endif
template <typename T>
__device__ __forceinline__ void stb_nt(T* __restrict__ base, unsigned off, T v) {
  T* p = reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
  if constexpr (RLB_STREAMING) __builtin_nontemporal_store(v, p);
  else *p = v;
}
template <typename T>
__device__ __forceinline__ T ldb_nt(const T* __restrict__ base, unsigned off) {
  const T* p = reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
  if constexpr (RLB_STREAMING) return __builtin_nontemporal_load(p);
  else return *p;
}

// ---------------------------------------------------------------------------
// Staged tiles (2D and 3D).  A workgroup updates a tile of kTY rows of 64
// cells (one row per wavefront).  The x and y neighbours of its cells are not
// loaded one by one: per population array, each wavefront writes its own row
// of centre values into an LDS tile of (kTY + 4) x 68 values (rows y0 - 2 ..
// y0 + kTY + 1, columns x0 - 2 .. x0 + 65), loads one halo row (y0 - 2,
// y0 - 1, y0 + kTY, y0 + kTY + 1 for wavefronts 0..3) and the four halo
// cells of its row (lanes 0..3), and after a barrier every x and y
// neighbour is an LDS read.  z neighbours stay global loads.  The arrays go
// through LDS in stages of a few populations (f and h together).  Lanes of
// a ragged tile past the x or y end hold the boundary-mapped value of their
// position, so that every value the tile reads is right; their results go
// to their own pad cell (never read) and they touch no field or counter.
// ---------------------------------------------------------------------------
constexpr int kTY = kBlock / 64;   // rows per tile
constexpr int kLW = 64 + 4;        // LDS row: x0 - 2 .. x0 + 65
constexpr int kLH = kTY + 4;       // LDS rows: y0 - 2 .. y0 + kTY + 1

#ifndef RLB_STAGES_3D
#define RLB_STAGES_3D 4
#endif
#ifndef RLB_STAGES_2D
#define RLB_STAGES_2D 2
#endif
template <typename T, bool WH, int ACT>
struct Stages {
  // stages per step (measured on MI355X: smaller stages keep the 3D working
  // set of a tile's neighbourhood in L2; FP64 with density, 384^3: 4 stages
  // 11.68 ms, 6 stages 11.90, 8 stages 12.17; 2048 x 1024: 2 stages 0.488 ms,
  // 3 stages 0.379, 4 stages 0.386)
  static constexpr int n =
      (WH && sizeof(T) == 8) ? 4 : (ACT == 7 ? RLB_STAGES_3D : RLB_STAGES_2D);
  static constexpr int pops = (Q + n - 1) / n;               // populations per stage
  static constexpr int count = (Q + pops - 1) / pops;        // non-empty stages
  static constexpr int arrays = (WH ? 2 : 1) * pops;         // LDS arrays per stage
};

// Cell index (or face slot) of position (qx, qy) of plane z for qx in
// [-2, nx + 1], qy in [-2, ny + 1], with the x and y boundary conditions.
__device__ __forceinline__ long long map_xy(const StepParams& P, int qx, int qy, int z) {
  const int nx = P.nx, ny = P.ny;
  if (qy < 0 || qy >= ny) {
    const int side = qy < 0 ? 0 : 1;
    const int b = P.bc[2 + side];
    if (b == kBcFixed) return P.ncell + 2 + side;
    qy = b == kBcPeriodic ? (qy < 0 ? qy + ny : qy - ny) : (qy < 0 ? 0 : ny - 1);
  }
  if (qx < 0 || qx >= nx) {
    const int side = qx < 0 ? 0 : 1;
    const int b = P.bc[side];
    if (b == kBcFixed) return P.ncell + side;
    qx = b == kBcPeriodic ? (qx < 0 ? qx + nx : qx - nx) : (qx < 0 ? 0 : nx - 1);
  }
  return static_cast<long long>(P.px) * (qy + static_cast<long long>(P.py) * z) + qx;
}

// Offsets of a staged tile's lane at (x, y, z) (x, y possibly past the end):
// its value, z neighbours, halo row and halo column positions.
template <typename T, int ACT>
__device__ __forceinline__ void make_nbr_stg(const StepParams& P, int x, int y, int z, bool inside,
                                             Nbr<ACT>& N) {
  const int lane = static_cast<int>(__lane_id());
  const int w = static_cast<int>(threadIdx.x) >> 6;
  const int px = x < P.nx + 1 ? x : P.nx + 1;
  const int py = y < P.ny + 1 ? y : P.ny + 1;
  const unsigned sz = static_cast<unsigned>(sizeof(T));
  const long long c = map_xy(P, px, py, z);
  N.c = static_cast<unsigned>(c) * sz;
  // own storage cell (x < px, y < py: the padded planes cover every tile)
  N.cs = static_cast<unsigned>(x + static_cast<long long>(P.px) * (y + static_cast<long long>(P.py) * z)) * sz;
  const int y0 = y - w, x0 = x - lane;
  int hy = y0 - 2 + (w < 2 ? w : kTY + w);
  hy = hy < P.ny + 1 ? hy : P.ny + 1;
  N.hr = static_cast<unsigned>(map_xy(P, px, hy, z)) * sz;
  int hxp = lane < 2 ? x0 - 2 + lane : x0 + 62 + lane;
  hxp = hxp < P.nx + 1 ? hxp : P.nx + 1;
  N.hx = lane < 4 ? static_cast<unsigned>(map_xy(P, hxp, py, z)) * sz : N.c;
  if constexpr (axis_on<ACT>(2)) {
    const long long st = static_cast<long long>(P.px) * P.py;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = j < 2 ? j - 2 : j - 1;
      const int q = z + k;
      long long idx = c + k * st;
      if (q < 0 || q >= P.nz) {
        const int side = q < 0 ? 0 : 1;
        const int b = P.bc[4 + side];
        if (b == kBcFixed) idx = P.ncell + 4 + side;
        else if (b == kBcPeriodic) idx = c + (q < 0 ? k + P.nz : k - P.nz) * st;
        else idx = c + ((q < 0 ? 0 : P.nz - 1) - z) * st;
      }
      // a lane past the x or y end needs no z neighbours: read its own value
      N.o[2][j] = inside ? static_cast<unsigned>(idx) * sz : N.c;
    }
  }
}

// Halo rows of a staged tile: wavefronts 0..3 stage rows y0 - 2, y0 - 1,
// y0 + kTY, y0 + kTY + 1.  A population's y stencil reads, by the sign ey of
// its y velocity component (the diagonal components of the extended set are
// +-2), the two rows below and one above (ey > 0), one below and two above
// (ey < 0) or one on each side (the Laplacian, ey = 0).  So the inner rows
// (sel 0: wavefronts 1, 2) are read by every population with a y stencil,
// y0 - 2 (sel +1, wavefront 0) by ey > 0 only and y0 + kTY + 1 (sel -1,
// wavefront 3) by ey < 0 only.
static_assert(kTY == 4, "four wavefronts stage the four halo rows");
constexpr bool halo_row_sel(int sel, int ey) { return sel == 0 || sel == ey; }

// Workgroup barrier that orders LDS accesses only: the wave's outstanding
// global loads and stores stay in flight across it (a full __syncthreads()
// fence waits for all of them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Fill the LDS tiles of populations [S0, S1) (f in slots 0.., h after them):
// halo loads first, then (after `sync_before`: the previous stage's reads are
// done) the centre row, halo row and halo columns, then a barrier.
template <typename T, int ACT, bool WH, int S0, int S1, bool RUS>
__device__ __forceinline__ void stage_fill(T (*L)[kLH][kLW], const T* __restrict__ fin,
                                           const T* __restrict__ hin, long long S,
                                           const Nbr<ACT>& N, const T* fc, const T* hc,
                                           bool sync_before) {
  constexpr int NP = S1 - S0;
  const int lane = static_cast<int>(__lane_id());
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  T vr[NP], vrh[NP], vx[NP], vxh[NP];
  // halo rows: the inner rows (wavefronts 1, 2) for every population with a
  // y stencil, the outer ones only for the sign of e^y that reads them (f_0
  // has no x/y stencil).  Measured on MI355X: FP32 200 x 100 x 100 Euler step
  // 5% faster, 2048 x 1024 unchanged; FP64 384^3 2.7% slower, so FP64 tiles
  // load every row for every population.
  // With the Rusanov flux (RUS) every population, f_0 and all of h included,
  // reads one cell on each side along every axis: the inner rows only.
  constexpr bool by_sign = sizeof(T) == 4;
  auto load_rows = [&](auto sel) {
    static_for<0, NP>([&](auto k) {
      constexpr int I = S0 + k;
      constexpr int ey = (vcomp(I, 1) > 0) - (vcomp(I, 1) < 0);  // sign
      if constexpr (RUS || (I != 0 && halo_row_sel(sel, ey))) vr[k] = ldb(fin + I * S, N.hr);
      if constexpr (WH && (RUS || (ey != 0 && halo_row_sel(sel, ey)))) vrh[k] = ldb(hin + I * S, N.hr);
    });
  };
  if constexpr (RUS) {
    if (w == 1 || w == 2) load_rows(std::integral_constant<int, 0>{});
  } else if (!by_sign || w == 1 || w == 2) {
    load_rows(std::integral_constant<int, 0>{});
  } else if (w == 0) {
    load_rows(std::integral_constant<int, 1>{});
  } else {
    load_rows(std::integral_constant<int, -1>{});
  }
  if (lane < 4) {
    static_for<0, NP>([&](auto k) {
      constexpr int I = S0 + k;
      vx[k] = ldb(fin + I * S, N.hx);
      if constexpr (WH && (RUS || vcomp(I, 0) != 0)) vxh[k] = ldb(hin + I * S, N.hx);
    });
  }
  if (sync_before) lds_barrier();
  const int hrow = w < 2 ? w : kTY + w;
  const int hcol = lane < 2 ? lane : 64 + lane;
  static_for<0, NP>([&](auto k) {
    constexpr int I = S0 + k;
    L[k][2 + w][2 + lane] = fc[I];
    if constexpr (WH && (RUS || vcomp(I, 0) != 0 || vcomp(I, 1) != 0)) L[NP + k][2 + w][2 + lane] = hc[I];
  });
  auto store_rows = [&](auto sel) {
    static_for<0, NP>([&](auto k) {
      constexpr int I = S0 + k;
      constexpr int ey = (vcomp(I, 1) > 0) - (vcomp(I, 1) < 0);  // sign
      if constexpr (RUS || (I != 0 && halo_row_sel(sel, ey))) L[k][hrow][2 + lane] = vr[k];
      if constexpr (WH && (RUS || (ey != 0 && halo_row_sel(sel, ey)))) L[NP + k][hrow][2 + lane] = vrh[k];
    });
  };
  if constexpr (RUS) {
    if (w == 1 || w == 2) store_rows(std::integral_constant<int, 0>{});
  } else if (!by_sign || w == 1 || w == 2) {
    store_rows(std::integral_constant<int, 0>{});
  } else if (w == 0) {
    store_rows(std::integral_constant<int, 1>{});
  } else {
    store_rows(std::integral_constant<int, -1>{});
  }
  if (lane < 4) {
    static_for<0, NP>([&](auto k) {
      constexpr int I = S0 + k;
      L[k][2 + w][hcol] = vx[k];
      if constexpr (WH && (RUS || vcomp(I, 0) != 0)) L[NP + k][2 + w][hcol] = vxh[k];
    });
  }
  lds_barrier();
}

// Star stencil of one population: per active axis the values the limited
// flux (and, with LAP, the Laplacian) needs: e^a > 0: x-2, x-1, x+1;
// e^a < 0: x-1, x+1, x+2; e^a = 0 with LAP: x-1, x+1.
template <typename T>
struct Sten {
  T v[3][3];
};

template <typename T, int ACT, int I, bool LAP>
__device__ __forceinline__ void gather(const T* __restrict__ arr, const Nbr<ACT>& N, Sten<T>& s) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!axis_on<ACT>(a)) continue;
    const int ea = vcomp(I, a);
    if (ea > 0) {
      s.v[a][0] = ldb(arr, N.o[a][0]);
      s.v[a][1] = ldb(arr, N.o[a][1]);
      s.v[a][2] = ldb(arr, N.o[a][2]);
    } else if (ea < 0) {
      s.v[a][0] = ldb(arr, N.o[a][1]);
      s.v[a][1] = ldb(arr, N.o[a][2]);
      s.v[a][2] = ldb(arr, N.o[a][3]);
    } else if (LAP) {
      s.v[a][0] = ldb(arr, N.o[a][1]);
      s.v[a][1] = ldb(arr, N.o[a][2]);
    }
  }
}

// Stencil of population I of a staged tile: x and y from the LDS tile L
// (this lane at row 2 + wavefront, column 2 + lane), z from the array.
template <typename T, int ACT, int I, bool LAP, bool RUS>
__device__ __forceinline__ void gather_lds(const T (*L)[kLW], const T* __restrict__ arr,
                                           const Nbr<ACT>& N, Sten<T>& s) {
  const int r = 2 + (static_cast<int>(threadIdx.x) >> 6);
  const int c = 2 + static_cast<int>(__lane_id());
  if constexpr (RUS) {
    // the Rusanov flux: one cell on each side along every axis (v[a][0], v[a][1])
    s.v[0][0] = L[r][c - 1];
    s.v[0][1] = L[r][c + 1];
    s.v[1][0] = L[r - 1][c];
    s.v[1][1] = L[r + 1][c];
    if constexpr (axis_on<ACT>(2)) {
      s.v[2][0] = ldb(arr, N.o[2][1]);
      s.v[2][1] = ldb(arr, N.o[2][2]);
    }
    return;
  }
  constexpr int ex = vcomp(I, 0), ey = vcomp(I, 1);
  if constexpr (ex > 0) {
    s.v[0][0] = L[r][c - 2];
    s.v[0][1] = L[r][c - 1];
    s.v[0][2] = L[r][c + 1];
  } else if constexpr (ex < 0) {
    s.v[0][0] = L[r][c - 1];
    s.v[0][1] = L[r][c + 1];
    s.v[0][2] = L[r][c + 2];
  } else if constexpr (LAP) {
    s.v[0][0] = L[r][c - 1];
    s.v[0][1] = L[r][c + 1];
  }
  if constexpr (ey > 0) {
    s.v[1][0] = L[r - 2][c];
    s.v[1][1] = L[r - 1][c];
    s.v[1][2] = L[r + 1][c];
  } else if constexpr (ey < 0) {
    s.v[1][0] = L[r - 1][c];
    s.v[1][1] = L[r + 1][c];
    s.v[1][2] = L[r + 2][c];
  } else if constexpr (LAP) {
    s.v[1][0] = L[r - 1][c];
    s.v[1][1] = L[r + 1][c];
  }
  if constexpr (axis_on<ACT>(2)) {
    constexpr int ez = vcomp(I, 2);
    if constexpr (ez > 0) {
      s.v[2][0] = ldb(arr, N.o[2][0]);
      s.v[2][1] = ldb(arr, N.o[2][1]);
      s.v[2][2] = ldb(arr, N.o[2][2]);
    } else if constexpr (ez < 0) {
      s.v[2][0] = ldb(arr, N.o[2][1]);
      s.v[2][1] = ldb(arr, N.o[2][2]);
      s.v[2][2] = ldb(arr, N.o[2][3]);
    } else if constexpr (LAP) {
      s.v[2][0] = ldb(arr, N.o[2][1]);
      s.v[2][1] = ldb(arr, N.o[2][2]);
    }
  }
}

// delta t * (flux divergence) and the sum of the axis neighbours used by the
// Laplacian (without the -2 f(x) per axis) of population I from its stencil.
template <typename T, int ACT, int I, bool LAP, bool RUS = false>
__device__ __forceinline__ void stream_terms(const Sten<T>& s, T c0, T dtv, T& dD, T& nsum,
                                             T dtc = T(0)) {
  if constexpr (RUS) {
    // the Rusanov flux (rusanov_terms) summed over the active axes; the
    // stencil holds the cells on each side (v[a][0], v[a][1]), dtc = dt times
    // the speed of light
    bool first = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (!axis_on<ACT>(a)) continue;
      const T fm = s.v[a][0], fp = s.v[a][1];
      const T d = T(0.5) * (dtv * T(vcomp(I, a))) * (fp - fm) - T(0.5) * dtc * ((fp - c0) - (c0 - fm));
      dD = first ? d : dD + d;
      nsum = first ? fm + fp : nsum + (fm + fp);
      first = false;
    }
    return;
  }
  bool first_d = true, first_n = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!axis_on<ACT>(a)) continue;
    const int ea = vcomp(I, a);
    T d = T(0), nb = T(0);
    bool has_d = false, has_n = false;
    if (ea > 0) {
      d = (dtv * T(ea)) * dflux_pos(s.v[a][0], s.v[a][1], c0, s.v[a][2]);
      nb = s.v[a][1] + s.v[a][2];
      has_d = true;
      has_n = LAP;
    } else if (ea < 0) {
      d = (dtv * T(ea)) * dflux_neg(s.v[a][0], c0, s.v[a][1], s.v[a][2]);
      nb = s.v[a][0] + s.v[a][1];
      has_d = true;
      has_n = LAP;
    } else if (LAP) {
      nb = s.v[a][0] + s.v[a][1];
      has_n = true;
    }
    if (has_d) {
      dD = first_d ? d : dD + d;
      first_d = false;
    }
    if (has_n) {
      nsum = first_n ? nb : nsum + nb;
      first_n = false;
    }
  }
  if (first_d) dD = T(0);
  if (first_n) nsum = T(0);
}

// Cell of this thread (see StepParams::order); false if the workgroup's tile
// is outside the grid (x and y of a ragged tile may lie past the end).
__device__ __forceinline__ bool cell_of(const StepParams& P, int& x, int& y, int& z) {
  const unsigned b = blockIdx.x;
  const long long l = b / kXcds;
  const int xcd = static_cast<int>(b % kXcds);
  const int tiles_pp = P.pw * P.ph;  // tiles per pencil plane
  const int npx = P.ntx / P.pw;
  int tx, ty;
  if (P.order == 1) {
    const int tin = static_cast<int>(l % tiles_pp);
    const long long r = l / tiles_pp;
    const int zl = static_cast<int>(r % P.zslab);
    const long long pencil = r / P.zslab;
    tx = static_cast<int>(pencil % npx) * P.pw + tin % P.pw;
    ty = static_cast<int>(pencil / npx) * P.ph + tin / P.pw;
    z = xcd * P.zslab + zl;
    if (ty >= P.nty || z >= P.nz) return false;
  } else {
    const long long g = xcd * P.tiles_per_xcd + l;
    if (g >= P.ntiles) return false;
    const int tin = static_cast<int>(g % tiles_pp);
    const long long r = g / tiles_pp;
    const long long npy = P.nty / P.ph;
    const int pyi = static_cast<int>(r % npy);
    const long long r2 = r / npy;
    z = static_cast<int>(r2 % P.nz);
    const int pxi = static_cast<int>(r2 / P.nz);
    tx = pxi * P.pw + tin % P.pw;
    ty = pyi * P.ph + tin / P.pw;
  }
  x = tx * P.tile_x + static_cast<int>(threadIdx.x) % P.tile_x;
  y = ty * P.tile_y + static_cast<int>(threadIdx.x) / P.tile_x;
  return true;
}

// Wavefront-aggregated counter increment.
__device__ __forceinline__ void count_events(unsigned long long* ctr, bool fired) {
  const unsigned long long mask = __ballot(fired);
  if (mask == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll(static_cast<long long>(mask)) - 1;
  if (lane == leader) atomicAdd(ctr, static_cast<unsigned long long>(__popcll(mask)));
}

// Wavefront-aggregated atomicMin of a step index (all lanes of a wave carry
// the same step): one atomic per wave that met an inadmissible cell.
__device__ __forceinline__ void flag_bad(unsigned long long* flag, bool bad, long long step) {
  const unsigned long long mask = __ballot(bad);
  if (mask == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll(static_cast<long long>(mask)) - 1;
  if (lane == leader) atomicMin(flag, static_cast<unsigned long long>(step));
}

// Guard (decided in FP64): projected fields of the new moments and blend
// factors for f and h; true if either factor is below 1.
template <bool WH>
__device__ __forceinline__ bool guard_eval(const StepParams& P, double E, double Mx, double My,
                                           double Mz, double N0, double& thf, double& thh,
                                           Fields& G) {
  thf = 1.0;
  thh = 1.0;
  const double M = sqrt(Mx * Mx + My * My + Mz * Mz);
  if (!(isfinite(E) && isfinite(M))) return false;
  if (WH && !isfinite(N0)) return false;
  double th;
  if (!(E > 0.0)) {
    th = 0.0;
  } else {
    const double m = M / E;
    th = (m <= P.m1) ? 1.0 : ((m >= P.mmax) ? 0.0 : (P.mmax - m) / (P.mmax - P.m1));
  }
  const double Ec = fmax(E, P.efloor);
  const double Mc = fmin(M, P.mmax * Ec);
  const double sc = (M > 0.0) ? Mc / M : 0.0;
  recover<false>(Ec, sc * Mx, sc * My, sc * Mz, 0.0, G);
  double tn = 1.0;
  if constexpr (WH) {
    const double ng = N0 / G.gam;
    tn = (ng >= 2.0 * P.efloor) ? 1.0 : ((ng <= P.efloor) ? 0.0 : (ng - P.efloor) / P.efloor);
    G.n = fmax(ng, P.efloor);
  }
  thf = th;
  thh = fmin(th, tn);
  return th < 1.0 || thh < 1.0;
}

// FP64 moments of 19 (+19) values in canonical order (lattice L).
template <typename T, bool WH, int L = 0, typename LF, typename LH>
__device__ __forceinline__ void moments64(const StepParams& P, LF&& fval, LH&& hval, double& E,
                                          double& Mx, double& My, double& Mz, double& N0) {
  double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0, sh = 0.0;
  static_for<0, Q>([&](auto I) {
    constexpr Vel e = vel_l<L>(I);
    const double v = static_cast<double>(fval(I));
    s0 += v;
    if constexpr (e.x != 0) sx += double(e.x) * v;
    if constexpr (e.y != 0) sy += double(e.y) * v;
    if constexpr (e.z != 0) sz += double(e.z) * v;
    if constexpr (WH) sh += static_cast<double>(hval(I));
  });
  E = P.r * P.r * s0;
  Mx = P.rca * sx;
  My = P.rca * sy;
  Mz = P.rca * sz;
  N0 = P.r * sh;
}

// Per-dimensionality tuning (measured on MI355X): populations gathered per
// batch, and the minimum waves per SIMD the register allocator must allow.
#ifndef RLB_BATCH_3D
#define RLB_BATCH_3D 1
#endif
#ifndef RLB_BATCH_2D
#define RLB_BATCH_2D 3
#endif
#ifndef RLB_BATCH_1D
#define RLB_BATCH_1D 2
#endif
#ifndef RLB_OCC_F32
#define RLB_OCC_F32 3
#endif
#ifndef RLB_OCC_F32_3D
#define RLB_OCC_F32_3D RLB_OCC_F32
#endif
#ifndef RLB_OCC_F64
#define RLB_OCC_F64 2
#endif
template <typename T, int ACT>
struct Occ {
  static constexpr int value =
      sizeof(T) == 4 ? (ACT == 7 ? RLB_OCC_F32_3D : RLB_OCC_F32) : RLB_OCC_F64;
};
template <int ACT>
struct Batch {
  static constexpr int value = ACT == 7 ? RLB_BATCH_3D : (ACT == 3 ? RLB_BATCH_2D : RLB_BATCH_1D);
  static constexpr int count = (Q + value - 1) / value;
};

// ---------------------------------------------------------------------------
// Fused step: moments -> FP64 recovery -> equilibria -> limited streaming,
// bulk term and implicit collision (Eq. (57)) or Euler update -> guard.
// ---------------------------------------------------------------------------
template <typename T, int ACT, bool WH, bool EULER, bool SEG, bool RUS = false>
__global__ __launch_bounds__(kBlock, (Occ<T, ACT>::value)) void k_step(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ hin,
    T* __restrict__ hout, double* __restrict__ hist, const uint8_t* __restrict__ obst,
    const StepParams P) {
  const long long S = P.pstride;
  Nbr<ACT> N;
  bool inside = true;  // the lane holds a cell of the grid
  // run parameters (per request in segment mode)
  double kappa_d = P.kappa, nu2e = P.nu2_etas, tau_u = P.tau;
  unsigned long long* bad_ptr = P.bad_step;
  unsigned long long* guard_ptr = P.guard_count;
  long long step_idx = P.step_index;
  if constexpr (SEG) {
    static_assert(ACT == 1, "segments are one-dimensional");
    const int2 t = P.tiles[blockIdx.x];
    if (t.x < 0) return;
    const SegDesc& sd = P.segs[t.x];
    const int local = t.y * kBlock + static_cast<int>(threadIdx.x);
    if (local >= sd.n) return;
    make_seg_nbr<T>(sd, local, N);
    const long long ls = *P.gstep + P.step_in_chunk - sd.start;
    if (ls >= sd.steps) {
      // finished: carry the state into the other copy until it is retired
      static_for<0, Q>([&](auto I) {
        stb_nt(fout + I * S, N.c, ldb(fin + I * S, N.c));
        if constexpr (WH) stb_nt(hout + I * S, N.c, ldb(hin + I * S, N.c));
      });
      return;
    }
    kappa_d = sd.kappa;
    nu2e = sd.nu2_etas;
    tau_u = sd.tau;
    bad_ptr = sd.bad + sd.id;
    guard_ptr = sd.guard + sd.id;
    step_idx = ls;
  } else {
    int x, y, z;
    if (!cell_of(P, x, y, z)) return;
    if constexpr (ACT == 1) {
      if (x >= P.nx) return;
      make_nbr<T, ACT>(P, x, y, z, N);
    } else {
      // staged tile: every lane stays for the barriers (see make_nbr_stg)
      inside = x < P.nx && y < P.ny;
      make_nbr_stg<T, ACT>(P, x, y, z, inside, N);
    }
  }
  bool real = inside;                                       // this lane updates its cell
  const unsigned cl = N.c;                                  // byte offset loaded from
  const unsigned cb = N.cs;                                 // byte offset stored to
  const unsigned cd = (cl / sizeof(T)) * 8u;                // byte offset in FP64 arrays
  const unsigned cdl = inside ? cd : 0u;                    // previous fields read (any cell if outside)
  const long long NC = P.ncell;
  const double* __restrict__ h0 = hist;
  const double* __restrict__ h1 = hist + NC;
  const double* __restrict__ h2 = hist + 2 * NC;
  const double* __restrict__ h3 = hist + 3 * NC;
  const double* __restrict__ h4 = hist + 4 * NC;

  // Obstacle cells: held at the equilibrium of their prescribed fields (kept
  // in hist).  1D: written here.  In a staged tile the lane stays (its value
  // is a neighbour), touches no field or counter, and its regular stores
  // write that equilibrium (coefficient override below).
  bool solid = false;
  if (!SEG && obst != nullptr && inside && obst[cl / sizeof(T)] != 0) {
    if constexpr (ACT == 1) {
      const double eps = ldb(h0, cd), ux = ldb(h1, cd), uy = ldb(h2, cd), uz = ldb(h3, cd),
                   nn = ldb(h4, cd);
      const double g2 = 1.0 / (1.0 - (ux * ux + uy * uy + uz * uz));
      double K[10];
      feq_coeffs(P, eps, ux, uy, uz, g2, K);
      static_for<0, Q>(
          [&](auto I) { stb(fout + I * S, cl, static_cast<T>(weight(I) * bracket<I>(K))); });
      if constexpr (WH) {
        double H[10];
        heq_coeffs(P, nn, ux, uy, uz, sqrt(g2), H);
        static_for<0, Q>(
            [&](auto I) { stb(hout + I * S, cl, static_cast<T>(wprime<I>(P) * bracket<I>(H))); });
      }
      return;
    }
    solid = true;
    real = false;
  }
  const unsigned cbs = cb;

  T fc[Q];
  T hc[Q];
  static_for<0, Q>([&](auto I) {
    fc[I] = ldb(fin + I * S, cl);
    if constexpr (WH) hc[I] = ldb(hin + I * S, cl);
  });
  // LDS tiles of a stage (2D/3D)
  __shared__ T lds[ACT != 1 ? Stages<T, WH, ACT>::arrays : 1][kLH][kLW];

  static_assert(!RUS || ACT != 1, "the 1D Rusanov flux is built in k_step_tb");
  const T dtv = static_cast<T>(P.dtv);
  const T dtc = static_cast<T>(P.dtv * sqrt(27.0 / 13.0));  // dt times the speed of light
  constexpr T NA2 = T(2 * n_axes<ACT>());
  // the stencils of a batch of populations (f and h) are gathered first so
  // that their loads are in flight together
  constexpr int kBatch = Batch<ACT>::value;
  constexpr int kNumBatches = Batch<ACT>::count;

  // Streaming phase: per_pop(I, stencil of f_I, stencil of h_I) for every
  // population, stencils from the staged LDS tiles (2D/3D, stage by stage) or
  // from the arrays (1D, in batches).
  auto stream_all = [&](auto&& per_pop) {
    if constexpr (ACT != 1) {
      constexpr int NS = Stages<T, WH, ACT>::count, PP = Stages<T, WH, ACT>::pops;
      static_for<0, NS>([&](auto st) {
        constexpr int S0 = st * PP;
        constexpr int S1 = S0 + PP < Q ? S0 + PP : Q;
        stage_fill<T, ACT, WH, S0, S1, RUS>(lds, fin, hin, S, N, fc, hc, st > 0);
        static_for<S0, S1>([&](auto I) {
          Sten<T> sf, sh;
          gather_lds<T, ACT, I, (I != 0), RUS>(lds[I - S0], fin + I * S, N, sf);
          if constexpr (WH)
            gather_lds<T, ACT, I, false, RUS>(lds[(S1 - S0) + (I - S0)], hin + I * S, N, sh);
          per_pop(I, sf, sh);
        });
      });
    } else {
      static_for<0, kNumBatches>([&](auto g) {
        Sten<T> sf[kBatch], sh[kBatch];
        static_for<0, kBatch>([&](auto k) {
          constexpr int I = g * kBatch + k;
          if constexpr (I < Q) {
            gather<T, ACT, I, (I != 0)>(fin + I * S, N, sf[k]);
            if constexpr (WH) gather<T, ACT, I, false>(hin + I * S, N, sh[k]);
          }
        });
        static_for<0, kBatch>([&](auto k) {
          constexpr int I = g * kBatch + k;
          if constexpr (I < Q) per_pop(std::integral_constant<int, I>{}, sf[k], sh[k]);
        });
      });
    }
  };

  if constexpr (EULER) {
    // Streaming and bulk term without collision, then f := f^eq of the
    // post-streaming moments (Sec. III, inviscid case).
    // The post-streaming populations are only needed through their moments:
    // they are summed in FP64 as they are produced (canonical order, as in
    // moments64), so none of them stays live across the stages.
    const T kap = static_cast<T>(kappa_d);
    double m0 = 0.0, mx = 0.0, my = 0.0, mz = 0.0, mh = 0.0;
    stream_all([&](auto I, const Sten<T>& sfI, const Sten<T>& shI) {
      constexpr Vel e = vel(I);
      T dD, ns;
      stream_terms<T, ACT, I, (I != 0), RUS>(sfI, fc[I], dtv, dD, ns, dtc);
      T v;
      if constexpr (I != 0 || RUS) v = (fc[I] - dD) + kap * (ns - NA2 * fc[I]);
      else v = fc[I] - dD;
      const double vd = static_cast<double>(v);
      m0 += vd;
      if constexpr (e.x != 0) mx += double(e.x) * vd;
      if constexpr (e.y != 0) my += double(e.y) * vd;
      if constexpr (e.z != 0) mz += double(e.z) * vd;
      if constexpr (WH) {
        T dH, nh;
        stream_terms<T, ACT, I, false, RUS>(shI, hc[I], dtv, dH, nh, dtc);
        mh += static_cast<double>(hc[I] - dH);
        asm volatile("" : "+v"(mh));
      }
      // keep the sums current: otherwise the compiler defers them past the
      // stage barriers and keeps every stencil value live (register spills)
      asm volatile("" : "+v"(m0), "+v"(mx), "+v"(my), "+v"(mz));
    });
    const double E = P.r * P.r * m0, Mx = P.rca * mx, My = P.rca * my, Mz = P.rca * mz,
                 N0 = P.r * mh;
    Fields F;
    bool ok = true;
    bool fired = false;
    if (P.guard) {
      double thf, thh;
      fired = guard_eval<WH>(P, E, Mx, My, Mz, N0, thf, thh, F);
      count_events(guard_ptr, fired && real);
    }
    if (!fired) ok = recover<WH>(E, Mx, My, Mz, N0, F);
    flag_bad(bad_ptr, !ok && real, step_idx);
    if (solid) {
      // obstacle lane: the equilibrium of its prescribed fields
      F.eps = ldb(h0, cd);
      F.ux = ldb(h1, cd);
      F.uy = ldb(h2, cd);
      F.uz = ldb(h3, cd);
      F.n = ldb(h4, cd);
      F.g2 = 1.0 / (1.0 - (F.ux * F.ux + F.uy * F.uy + F.uz * F.uz));
      F.gam = sqrt(F.g2);
    }
    double K[10];
    feq_coeffs(P, F.eps, F.ux, F.uy, F.uz, F.g2, K);
    T Kt[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) Kt[k] = static_cast<T>(K[k]);
    // lanes past the grid end (staged tiles) store nothing here: no cell
    // reads the pad cells.  (The implicit step below stores them to their own
    // pad cells instead: predicating its interleaved stores cost 10% of the
    // time of unpadded grids.)
    if (!inside) return;
    static_for<0, Q>(
        [&](auto I) { stb_nt(fout + I * S, cbs, static_cast<T>(weight(I)) * bracket<I>(Kt)); });
    if constexpr (WH) {
      double H[10];
      heq_coeffs(P, F.n, F.ux, F.uy, F.uz, F.gam, H);
      T Ht[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) Ht[k] = static_cast<T>(H[k]);
      static_for<0, Q>(
          [&](auto I) { stb_nt(hout + I * S, cbs, static_cast<T>(wprime<I>(P)) * bracket<I>(Ht)); });
    }
    return;
  } else {
    // previous fields: FP64 (eps, u, n), or FP32 (eps, gamma u, n) in the
    // compact form of the mixed-precision 2D/3D step, where gamma^2 =
    // 1 + |gamma u|^2 has no cancellation at high speed
    constexpr bool kCompact = std::is_same<T, float>::value && !SEG && ACT != 1;
    double pe, pux, puy, puz, pn, pg2;
    if constexpr (kCompact) {
      const float* __restrict__ q = P.hist32;
      const unsigned o = inside ? cl : 0u;
      pe = ldb_nt(q, o);
      const double gx = ldb_nt(q + NC, o), gy = ldb_nt(q + 2 * NC, o), gz = ldb_nt(q + 3 * NC, o);
      pn = ldb_nt(q + 4 * NC, o);
      pg2 = 1.0 + (gx * gx + gy * gy + gz * gz);
      const double ig = 1.0 / sqrt(pg2);
      pux = gx * ig;
      puy = gy * ig;
      puz = gz * ig;
    } else {
      pe = ldb_nt(h0, cdl);
      pux = ldb_nt(h1, cdl);
      puy = ldb_nt(h2, cdl);
      puz = ldb_nt(h3, cdl);
      pn = ldb_nt(h4, cdl);
      pg2 = 1.0 / (1.0 - (pux * pux + puy * puy + puz * puz));
    }
    // 1-2: moments and fields at time t.
    double E, Mx, My, Mz, N0;
    moments64<T, WH>(P, [&](auto I) { return fc[I]; }, [&](auto I) { return hc[I]; }, E, Mx, My,
                     Mz, N0);
    Fields F;
    const bool ok = recover<WH>(E, Mx, My, Mz, N0, F);
    flag_bad(bad_ptr, !ok && real, step_idx);

    // 3: the source omega (2 f^eq(t) - f^eq(t - dt)) / (1 + omega) as one
    // coefficient set, computed in FP64 and rounded once to T.
    const double omega = P.omega_c / tau_of<T, WH>(P, F, tau_u, nu2e);
    const double inv1p = 1.0 / (1.0 + omega);
    const double src = omega * inv1p;
    T Kt[10];
    {
      double K[10], Kp[10];
      feq_coeffs(P, F.eps, F.ux, F.uy, F.uz, F.g2, K);
      feq_coeffs(P, pe, pux, puy, puz, pg2, Kp);
      // obstacle lane: the equilibrium of its prescribed fields (held in hist)
#pragma unroll
      for (int k = 0; k < 10; ++k) Kt[k] = static_cast<T>(solid ? Kp[k] : src * (2.0 * K[k] - Kp[k]));
    }
    T Ht[10];
    if constexpr (WH) {
      double H[10], Hp[10];
      heq_coeffs(P, F.n, F.ux, F.uy, F.uz, F.gam, H);
      heq_coeffs(P, pn, pux, puy, puz, sqrt(pg2), Hp);
#pragma unroll
      for (int k = 0; k < 10; ++k) Ht[k] = static_cast<T>(solid ? Hp[k] : src * (2.0 * H[k] - Hp[k]));
    }
    if (real) {
      if constexpr (kCompact) {
        float* __restrict__ q = P.hist32;
        stb_nt(q, cl, static_cast<float>(F.eps));
        stb_nt(q + NC, cl, static_cast<float>(F.gam * F.ux));
        stb_nt(q + 2 * NC, cl, static_cast<float>(F.gam * F.uy));
        stb_nt(q + 3 * NC, cl, static_cast<float>(F.gam * F.uz));
        stb_nt(q + 4 * NC, cl, static_cast<float>(F.n));
      } else {
        double* __restrict__ w0 = hist;
        stb_nt(w0, cd, F.eps);
        stb_nt(w0 + NC, cd, F.ux);
        stb_nt(w0 + 2 * NC, cd, F.uy);
        stb_nt(w0 + 3 * NC, cd, F.uz);
        stb_nt(w0 + 4 * NC, cd, F.n);
      }
    }

    // obstacle lanes keep only the equilibrium term (exact: 0 * finite + y)
    const T tinv = static_cast<T>(solid ? 0.0 : inv1p);
    const T kinv = static_cast<T>(solid ? 0.0 : kappa_d * inv1p);
    const T wp[3] = {static_cast<T>(P.wp0), static_cast<T>(P.wp1), static_cast<T>(P.wp2)};

    // 4-5: limited streaming, bulk term (f only, lambda_0 = 0) and implicit
    // collision, Eq. (57); new moments accumulated for the guard's gate.
    T gE = T(0), gX = T(0), gY = T(0), gZ = T(0), gN = T(0), gA = T(0), gAh = T(0);
    stream_all([&](auto I, const Sten<T>& sfI, const Sten<T>& shI) {
      constexpr Vel e = vel(I);
      T dD, ns;
      stream_terms<T, ACT, I, (I != 0), RUS>(sfI, fc[I], dtv, dD, ns, dtc);
      T v = (fc[I] - dD) * tinv + static_cast<T>(weight(I)) * bracket<I>(Kt);
      if constexpr (I != 0 || RUS) v += kinv * (ns - NA2 * fc[I]);
      stb_nt(fout + I * S, cbs, v);
      gE += v;
      gA += fabs(v);
      if constexpr (e.x != 0) gX += T(e.x) * v;
      if constexpr (e.y != 0) gY += T(e.y) * v;
      if constexpr (e.z != 0) gZ += T(e.z) * v;
      if constexpr (WH) {
        T dH, nh;
        stream_terms<T, ACT, I, false, RUS>(shI, hc[I], dtv, dH, nh, dtc);
        const T wpi = I == 0 ? wp[0] : (I <= 6 ? wp[1] : wp[2]);
        const T hv = (hc[I] - dH) * tinv + wpi * bracket<I>(Ht);
        stb_nt(hout + I * S, cbs, hv);
        gN += hv;
        gAh += fabs(hv);
      }
    });

    // Guard: gate in storage precision with a rounding margin, decide and
    // blend in FP64 from the stored values.
    if (P.guard) {
      constexpr T tol = sizeof(T) == 4 ? T(8e-6) : T(1e-13);
      const T r2 = static_cast<T>(P.r * P.r), rca = static_cast<T>(P.rca);
      const T Eg = r2 * gE, mrg = tol * r2 * gA;
      const T Mg = rca * sqrt(gX * gX + gY * gY + gZ * gZ);
      bool need = real && (!(Eg > mrg) || (Mg + mrg > static_cast<T>(P.m1) * (Eg - mrg)));
      if constexpr (WH) {
        const T Ng = static_cast<T>(P.r) * gN;
        need = need || (real && !(Ng > static_cast<T>(2.0 * P.efloor * P.gmax) +
                                           tol * static_cast<T>(P.r) * gAh));
      }
      bool fired = false;
      if (need) {
        double E2, Mx2, My2, Mz2, N02;
        moments64<T, WH>(P, [&](auto I) { return ldb(fout + I * S, cbs); },
                         [&](auto I) { return ldb(hout + I * S, cbs); }, E2, Mx2, My2, Mz2, N02);
        double thf, thh;
        Fields G;
        fired = guard_eval<WH>(P, E2, Mx2, My2, Mz2, N02, thf, thh, G);
        if (fired) {
          double Kg[10];
          feq_coeffs(P, G.eps, G.ux, G.uy, G.uz, G.g2, Kg);
          static_for<0, Q>([&](auto I) {
            const double ge = weight(I) * bracket<I>(Kg);
            const double v = static_cast<double>(ldb(fout + I * S, cbs));
            stb(fout + I * S, cbs, static_cast<T>(ge + thf * (v - ge)));
          });
          if constexpr (WH) {
            double Hg[10];
            heq_coeffs(P, G.n, G.ux, G.uy, G.uz, G.gam, Hg);
            static_for<0, Q>([&](auto I) {
              const double ge = wprime<I>(P) * bracket<I>(Hg);
              const double v = static_cast<double>(ldb(hout + I * S, cbs));
              stb(hout + I * S, cbs, static_cast<T>(ge + thh * (v - ge)));
            });
          }
        }
      }
      count_events(guard_ptr, fired);
    }
  }
}

// ---------------------------------------------------------------------------
// z-marching step of 3D grids (mixed precision, implicit update).  A
// workgroup owns one 64 x 4 column of the grid and walks a run of zm_len
// z-planes through it.  Each thread keeps, in registers, the z-window of
// the arrays whose stencil reaches along z: the 10 populations with
// e^z != 0 of f and of h (flux, planes z-2..z+1 for e^z > 0, z-1..z+2 for
// e^z < 0) and the 8 populations of f with e^z = 0, i != 0 (bulk term,
// planes z-1..z+1).  Moving to the next plane shifts the windows and loads
// one new plane per array, so every population value is read from HBM once
// per step (plus the first planes of a run); the loads of a plane are in
// flight while the previous one computes.  x and y neighbours come from
// the LDS-staged tiles as in k_step.  The per-cell arithmetic is k_step's,
// in the same order.
// ---------------------------------------------------------------------------

// Window slot of population i: populations with e^z != 0 (flux along z)
constexpr int zf_index(int i) {
  return (i == 5 || i == 6) ? i - 5 : (i >= 11 ? i - 9 : -1);
}
// populations of f with e^z == 0, i != 0 (bulk term along z)
constexpr int zl_index(int i) {
  return (i >= 1 && i <= 4) ? i - 1 : ((i >= 7 && i <= 10) ? i - 3 : -1);
}
// populations of h with e^z == 0 (no z stencil)
constexpr int ho_index(int i) {
  return (i <= 4) ? i : ((i >= 7 && i <= 10) ? i - 2 : -1);
}
// window position of plane z (the centre) for a flux population
constexpr int zf_centre(int i) { return vcomp(i, 2) > 0 ? 2 : 1; }

#ifndef RLB_ZM_OCC
#define RLB_ZM_OCC 2
#endif

// Plane q (uniform across the workgroup) under the z boundary condition:
// either a plane index (periodic wrap, outflow clamp) or the FIXED face slot.
struct ZPlane {
  bool slot;
  unsigned off;  // slot: byte offset of the face slot; else: the plane index
};
__device__ __forceinline__ ZPlane zplane(const StepParams& P, int q, unsigned esz) {
  if (q >= 0 && q < P.nz) return {false, static_cast<unsigned>(q)};
  const int side = q < 0 ? 0 : 1;
  const int b = P.bc[4 + side];
  if (b == kBcFixed) return {true, static_cast<unsigned>(P.ncell + 4 + side) * esz};
  return {false, static_cast<unsigned>(b == kBcPeriodic ? (q < 0 ? q + P.nz : q - P.nz)
                                                       : (q < 0 ? 0 : P.nz - 1))};
}
// Byte offset of a lane's column at plane zp: xy is the column's offset at
// plane 0 and step its plane pitch in bytes (0 for a lane whose column is a
// face slot of an x or y face: every plane reads that slot).
__device__ __forceinline__ unsigned zcol(unsigned xy, unsigned step, ZPlane zp) {
  return zp.slot ? zp.off : xy + zp.off * step;
}

// x and y part of the stencil of population I from the LDS tile L.
template <typename T, int I, bool LAP>
__device__ __forceinline__ void gather_xy_lds(const T (*L)[kLW], Sten<T>& s) {
  const int r = 2 + (static_cast<int>(threadIdx.x) >> 6);
  const int c = 2 + static_cast<int>(__lane_id());
  constexpr int ex = vcomp(I, 0), ey = vcomp(I, 1);
  if constexpr (ex > 0) {
    s.v[0][0] = L[r][c - 2];
    s.v[0][1] = L[r][c - 1];
    s.v[0][2] = L[r][c + 1];
  } else if constexpr (ex < 0) {
    s.v[0][0] = L[r][c - 1];
    s.v[0][1] = L[r][c + 1];
    s.v[0][2] = L[r][c + 2];
  } else if constexpr (LAP) {
    s.v[0][0] = L[r][c - 1];
    s.v[0][1] = L[r][c + 1];
  }
  if constexpr (ey > 0) {
    s.v[1][0] = L[r - 2][c];
    s.v[1][1] = L[r - 1][c];
    s.v[1][2] = L[r + 1][c];
  } else if constexpr (ey < 0) {
    s.v[1][0] = L[r - 1][c];
    s.v[1][1] = L[r + 1][c];
    s.v[1][2] = L[r + 2][c];
  } else if constexpr (LAP) {
    s.v[1][0] = L[r - 1][c];
    s.v[1][1] = L[r + 1][c];
  }
}

// z part of the stencil of a flux population from its window W (planes
// z-2..z+1 for e^z > 0, z-1..z+2 for e^z < 0), in the layout of gather().
template <typename T, int I>
__device__ __forceinline__ void zsten_flux(const T* W, Sten<T>& s) {
  if constexpr (vcomp(I, 2) > 0) {
    s.v[2][0] = W[0];
    s.v[2][1] = W[1];
    s.v[2][2] = W[3];
  } else {
    s.v[2][0] = W[0];
    s.v[2][1] = W[2];
    s.v[2][2] = W[3];
  }
}

// Raw buffer access to the FP32 arrays of the z-marching step.  The 19
// population arrays of one distribution are addressed through two buffer
// descriptors (populations [0, 10) and [10, 19)); an access gives the
// array's offset within its group as the scalar offset and the lane's byte
// offset in the array as the vector offset.  No per-lane 64-bit address
// arithmetic is needed and the descriptors stay in scalar registers for the
// whole kernel.  A group spans at most 10 arrays, below 2^32 bytes for
// population strides up to kZmMaxStride (rlb_internal.h; checked on the host).
constexpr int kZmGroups = 2;
constexpr int zm_grp(int i) { return i < 10 ? 0 : 1; }
constexpr int zm_grp_first(int g) { return g == 0 ? 0 : 10; }
struct PopBuf {
  __amdgpu_buffer_rsrc_t g[kZmGroups];
};
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const float* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, -1, 0x00020000);
}
__device__ __forceinline__ PopBuf pop_buf(const float* base, long long stride) {
  PopBuf b;
#pragma unroll
  for (int k = 0; k < kZmGroups; ++k) b.g[k] = buf_rsrc(base + zm_grp_first(k) * stride);
  return b;
}
// aux 2: non-temporal (data touched once per step)
template <int I, int AUX = 0>
__device__ __forceinline__ float pld(const PopBuf& b, unsigned off, unsigned sb) {
  constexpr int g = zm_grp(I);
  return __builtin_bit_cast(
      float, __builtin_amdgcn_raw_buffer_load_b32(b.g[g], off, (I - zm_grp_first(g)) * sb, AUX));
}
template <int I, int AUX = 0>
__device__ __forceinline__ void pst(const PopBuf& b, unsigned off, unsigned sb, float v) {
  constexpr int g = zm_grp(I);
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), b.g[g], off,
                                        (I - zm_grp_first(g)) * sb, AUX);
}
constexpr int kNT = RLB_STREAMING ? 2 : 0;
#ifndef RLB_ZM_STAGES
#define RLB_ZM_STAGES 2
#endif
// 1: the outer halo rows of a z-marching tile are loaded only for the sign
// of e^y that reads them (0: every row for every population).  Measured on
// MI355X at 384^3 with the centres staged through LDS (RLB_ZM_CENLDS): 1%
// faster (3 spilled values); with the centres in registers 5.6% slower (22).
#ifndef RLB_ZM_ROWS
#define RLB_ZM_ROWS 1
#endif
// wave priority while a z-marching wave issues a burst of loads (0: off);
// measured on MI355X: 0.6% faster at 384^3
#ifndef RLB_ZM_PRIO
#define RLB_ZM_PRIO 1
#endif
// populations staged through LDS together (f and h) in the z-marching step
constexpr int kZmPops = (Q + RLB_ZM_STAGES - 1) / RLB_ZM_STAGES;
// 1: the next plane's centres without a window and previous-step fields are
// loaded straight into LDS (double-buffered per wavefront) instead of
// registers, which frees 15 registers across the recovery and the streaming
// phase (spills 13 -> 3 values; alone no faster, but room for RLB_ZM_ROWS)
#ifndef RLB_ZM_CENLDS
#define RLB_ZM_CENLDS 1
#endif

template <typename T, bool WH>
__global__ __launch_bounds__(kBlock, RLB_ZM_OCC) void k_step_zm(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ hin,
    T* __restrict__ hout, double* __restrict__ hist, const uint8_t* __restrict__ obst,
    const StepParams P) {
  static_assert(std::is_same<T, float>::value, "the z-marching step stores FP32 populations");
  constexpr int ACT = 7;
  const unsigned esz = static_cast<unsigned>(sizeof(T));
  // column and z-run of this workgroup: XCD k takes the k-th contiguous part
  // of the (run, tile row, tile column) order
  const long long g = static_cast<long long>(blockIdx.x % kXcds) * P.zm_per_xcd + blockIdx.x / kXcds;
  if (g >= P.zm_total) return;  // the whole workgroup
  const int tpp = P.ntx * P.nty;
  const int run = static_cast<int>(g / tpp);
  const int rem = static_cast<int>(g % tpp);
  const int ty = rem / P.ntx, tx = rem % P.ntx;
  const int zb = run * P.zm_len;
  const int ze = zb + P.zm_len < P.nz ? zb + P.zm_len : P.nz;
  const int lane = static_cast<int>(__lane_id());
  // wavefront index, uniform (the LDS destinations of the loads into LDS
  // must be scalar)
  const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int x = tx * 64 + lane, y = ty * kTY + wv;
  const bool inside = x < P.nx && y < P.ny;
  const unsigned plane_bytes = static_cast<unsigned>(P.px) * static_cast<unsigned>(P.py) * esz;
  const long long NC = P.ncell;
  // offsets at plane 0 (face slots of x or y faces are the same for every
  // plane: their plane pitch is 0): the lane's value (boundary-mapped past
  // the x or y end), its halo row and halo column, its own storage cell
  const int pxc = x < P.nx + 1 ? x : P.nx + 1;
  const int pyc = y < P.ny + 1 ? y : P.ny + 1;
  const long long c0 = map_xy(P, pxc, pyc, 0);
  const unsigned cxy = static_cast<unsigned>(c0) * esz;
  const unsigned cst = c0 >= NC ? 0u : plane_bytes;
  int hy = ty * kTY - 2 + (wv < 2 ? wv : kTY + wv);
  hy = hy < P.ny + 1 ? hy : P.ny + 1;
  const long long r0 = map_xy(P, pxc, hy, 0);
  const unsigned rxy = static_cast<unsigned>(r0) * esz;
  const unsigned rst = r0 >= NC ? 0u : plane_bytes;
  const unsigned sxy = static_cast<unsigned>(x + static_cast<long long>(P.px) * y) * esz;
  int hxp = lane < 2 ? tx * 64 - 2 + lane : tx * 64 + 62 + lane;
  hxp = hxp < P.nx + 1 ? hxp : P.nx + 1;
  const long long x0 = lane < 4 ? map_xy(P, hxp, pyc, 0) : c0;
  const unsigned xxy = static_cast<unsigned>(x0) * esz;
  const unsigned xst = x0 >= NC ? 0u : plane_bytes;

  unsigned long long* bad_ptr = P.bad_step;
  unsigned long long* guard_ptr = P.guard_count;
  const long long step_idx = P.step_index;
  const double kappa_d = P.kappa, nu2e = P.nu2_etas, tau_u = P.tau;
  const T dtv = static_cast<T>(P.dtv);
  constexpr T NA2 = T(2 * n_axes<ACT>());
  const T wp[3] = {static_cast<T>(P.wp0), static_cast<T>(P.wp1), static_cast<T>(P.wp2)};
  // LDS tiles of one stage: kZmPops populations of f, then of h
  constexpr int NPS = kZmPops;
  __shared__ T lds[(WH ? 2 : 1) * NPS][kLH][kLW];
  // buffer descriptors: populations (in, out) and previous-step fields
  const unsigned sb = static_cast<unsigned>(P.pstride) * esz;   // array pitch in bytes
  const PopBuf Fi = pop_buf(fin, P.pstride), Fo = pop_buf(fout, P.pstride);
  const PopBuf Hi = pop_buf(hin, P.pstride), Ho = pop_buf(hout, P.pstride);
  PopBuf Qh;  // previous-step fields 0..4: one group (5 NC FP32 values)
  Qh.g[0] = buf_rsrc(P.hist32);
  const unsigned qb = static_cast<unsigned>(NC) * 4u;

  // z-windows
  T wf[10][4];
  T wl[8][3];
  T f0c;
  T wh[WH ? 10 : 1][4];
  T ho[WH ? 9 : 1];
  auto fcen = [&](auto I) -> T {
    constexpr int i = I;
    if constexpr (i == 0) return f0c;
    else if constexpr (zf_index(i) >= 0) return wf[zf_index(i)][zf_centre(i)];
    else return wl[zl_index(i)][1];
  };
  auto hcen = [&](auto I) -> T {
    constexpr int i = I;
    if constexpr (zf_index(i) >= 0) return wh[zf_index(i)][zf_centre(i)];
    else return ho[ho_index(i)];
  };
  // centres without a z window and the previous-step fields of a plane
  // (loaded one plane ahead, into LDS or these registers)
  T f0n;
  T hon[WH ? 9 : 1];
  float qn[5];
#if RLB_ZM_CENLDS
  // per wavefront and plane parity: f_0, the 9 centres of h without a
  // window, the 5 previous-step fields (64 lanes each)
  __shared__ float cen[2][kTY][15][64];
  auto dma = [&](__amdgpu_buffer_rsrc_t r, int slot, int zq, unsigned voff, unsigned soff, auto aux) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        r, (__attribute__((address_space(3))) void*)(&cen[zq & 1][wv][slot][0]), 4, voff, soff, 0,
        decltype(aux)::value);
  };
  auto load_centres = [&](int zq) {
    const unsigned c = cxy + static_cast<unsigned>(zq) * cst;
    const unsigned oq = inside ? sxy + static_cast<unsigned>(zq) * plane_bytes : 0u;
    static_for<0, 5>([&](auto k) {
      dma(Qh.g[0], 10 + k, zq, oq, static_cast<unsigned>(k) * qb, std::integral_constant<int, kNT>{});
    });
    dma(Fi.g[0], 0, zq, c, 0u, std::integral_constant<int, 0>{});
    if constexpr (WH) {
      static_for<0, Q>([&](auto I) {
        constexpr int i = I;
        if constexpr (ho_index(i) >= 0)
          dma(Hi.g[zm_grp(i)], 1 + ho_index(i), zq, c, static_cast<unsigned>(i - zm_grp_first(zm_grp(i))) * sb,
              std::integral_constant<int, 0>{});
      });
    }
  };
  auto read_centres = [&](int zq) {
    f0n = cen[zq & 1][wv][0][lane];
    if constexpr (WH) {
#pragma unroll
      for (int k = 0; k < 9; ++k) hon[k] = cen[zq & 1][wv][1 + k][lane];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) qn[k] = cen[zq & 1][wv][10 + k][lane];
  };
#else
  auto load_centres = [&](int zq) {
    const unsigned c = cxy + static_cast<unsigned>(zq) * cst;
    const unsigned oq = inside ? sxy + static_cast<unsigned>(zq) * plane_bytes : 0u;
    static_for<0, 5>([&](auto k) { qn[k] = pld<k, kNT>(Qh, oq, qb); });
    f0n = pld<0>(Fi, c, sb);
    if constexpr (WH) {
      static_for<0, Q>([&](auto I) {
        constexpr int i = I;
        if constexpr (ho_index(i) >= 0) hon[ho_index(i)] = pld<i>(Hi, c, sb);
      });
    }
  };
  auto read_centres = [&](int) {};
#endif
  // first planes of the run
  {
    load_centres(zb);
    static_for<0, Q>([&](auto I) {
      constexpr int i = I;
      if constexpr (zf_index(i) >= 0) {
        constexpr int lo = vcomp(i, 2) > 0 ? -2 : -1;  // window planes lo .. lo + 2
        static_for<0, 3>([&](auto k) {
          const unsigned o = zcol(cxy, cst, zplane(P, zb + lo + k, esz));
          wf[zf_index(i)][k] = pld<i>(Fi, o, sb);
          if constexpr (WH) wh[zf_index(i)][k] = pld<i>(Hi, o, sb);
        });
      } else if constexpr (zl_index(i) >= 0) {
        static_for<0, 2>([&](auto k) {
          wl[zl_index(i)][k] = pld<i>(Fi, zcol(cxy, cst, zplane(P, zb - 1 + k, esz)), sb);
        });
      }
    });
  }

  const int hrow = wv < 2 ? wv : kTY + wv;  // LDS row of this wavefront's halo row
  for (int z = zb; z < ze; ++z) {
    const unsigned pz = static_cast<unsigned>(z) * plane_bytes;
    const unsigned cl = cxy + static_cast<unsigned>(z) * cst;  // this lane's value at z
    const unsigned cbs = sxy + pz;                             // its storage cell
    read_centres(z);  // from LDS (RLB_ZM_CENLDS); the loads' wait is the compiler's
    f0c = f0n;
    if constexpr (WH) {
#pragma unroll
      for (int k = 0; k < 9; ++k) ho[k] = hon[k];
    }
    const double pe = qn[0], gxp = qn[1], gyp = qn[2], gzp = qn[3], pn = qn[4];
    // obstacle cells: held at the equilibrium of their prescribed fields
    const bool solid = obst != nullptr && inside && obst[cl / esz] != 0;
    const bool real = inside && !solid;

    // the planes entering the windows (needed from the streaming phase on):
    // in flight during the recovery and the streaming phase (the stage
    // barriers order LDS only)
    if (RLB_ZM_PRIO) __builtin_amdgcn_s_setprio(RLB_ZM_PRIO);
    {
      const unsigned o1 = zcol(cxy, cst, zplane(P, z + 1, esz));
      const unsigned o2 = zcol(cxy, cst, zplane(P, z + 2, esz));
      static_for<0, Q>([&](auto I) {
        constexpr int i = I;
        if constexpr (zf_index(i) >= 0) {
          const unsigned o = vcomp(i, 2) > 0 ? o1 : o2;
          wf[zf_index(i)][3] = pld<i>(Fi, o, sb);
          if constexpr (WH) wh[zf_index(i)][3] = pld<i>(Hi, o, sb);
        } else if constexpr (zl_index(i) >= 0) {
          wl[zl_index(i)][2] = pld<i>(Fi, o1, sb);
        }
      });
    }
    // the next plane's centres without a window and its previous-step
    // fields (this plane's were copied out above); issued before the
    // recovery, measured 0.5% faster than after it
    if (z + 1 < ze) load_centres(z + 1);
    if (RLB_ZM_PRIO) __builtin_amdgcn_s_setprio(0);
    const double pg2 = 1.0 + (gxp * gxp + gyp * gyp + gzp * gzp);
    const double ig = 1.0 / sqrt(pg2);
    const double pux = gxp * ig, puy = gyp * ig, puz = gzp * ig;
    double E, Mx, My, Mz, N0;
    moments64<T, WH>(P, fcen, hcen, E, Mx, My, Mz, N0);
    Fields F;
    const bool ok = recover<WH>(E, Mx, My, Mz, N0, F);
    flag_bad(bad_ptr, !ok && real, step_idx);
    const double omega = P.omega_c / tau_of<T, WH>(P, F, tau_u, nu2e);
    const double inv1p = 1.0 / (1.0 + omega);
    const double src = omega * inv1p;
    T Kt[10];
    {
      double K[10], Kp[10];
      feq_coeffs(P, F.eps, F.ux, F.uy, F.uz, F.g2, K);
      feq_coeffs(P, pe, pux, puy, puz, pg2, Kp);
#pragma unroll
      for (int k = 0; k < 10; ++k) Kt[k] = static_cast<T>(solid ? Kp[k] : src * (2.0 * K[k] - Kp[k]));
    }
    T Ht[10];
    if constexpr (WH) {
      double H[10], Hp[10];
      heq_coeffs(P, F.n, F.ux, F.uy, F.uz, F.gam, H);
      heq_coeffs(P, pn, pux, puy, puz, sqrt(pg2), Hp);
#pragma unroll
      for (int k = 0; k < 10; ++k) Ht[k] = static_cast<T>(solid ? Hp[k] : src * (2.0 * H[k] - Hp[k]));
    }
    const T tinv = static_cast<T>(solid ? 0.0 : inv1p);
    const T kinv = static_cast<T>(solid ? 0.0 : kappa_d * inv1p);

    if (real) {
      pst<0, kNT>(Qh, cbs, qb, static_cast<float>(F.eps));
      pst<1, kNT>(Qh, cbs, qb, static_cast<float>(F.gam * F.ux));
      pst<2, kNT>(Qh, cbs, qb, static_cast<float>(F.gam * F.uy));
      pst<3, kNT>(Qh, cbs, qb, static_cast<float>(F.gam * F.uz));
      pst<4, kNT>(Qh, cbs, qb, static_cast<float>(F.n));
    }
    const unsigned hr = rxy + static_cast<unsigned>(z) * rst;
    const unsigned hx = xxy + static_cast<unsigned>(z) * xst;
    const int hcol = lane < 2 ? lane : 64 + lane;

    // limited streaming, bulk term and implicit collision, Eq. (57)
    T gE = T(0), gX = T(0), gY = T(0), gZ = T(0), gN = T(0), gA = T(0), gAh = T(0);
    constexpr int NS = (Q + NPS - 1) / NPS;
    static_for<0, NS>([&](auto st) {
      constexpr int S0 = st * NPS;
      constexpr int S1 = S0 + NPS < Q ? S0 + NPS : Q;
      constexpr int NP = S1 - S0;
      {
        // stage the tiles: halo row and halo cells of this plane through
        // registers, centre row from the windows
        static_assert(zm_grp(S0) == zm_grp(S1 - 1), "a stage lies in one descriptor group");
        if (RLB_ZM_PRIO) __builtin_amdgcn_s_setprio(RLB_ZM_PRIO);
        T vr[NP], vrh[NP], vx[NP], vxh[NP];
        // halo rows: the inner rows (wavefronts 1, 2) for every population
        // with a y stencil, the outer ones only for the sign of e^y that
        // reads them (f_0 has no x/y stencil)
        auto load_rows = [&](auto sel) {
          static_for<0, NP>([&](auto k) {
            constexpr int i = S0 + k;
            constexpr int ey = (vcomp(i, 1) > 0) - (vcomp(i, 1) < 0);  // sign
            if constexpr (i != 0 && halo_row_sel(sel, ey)) vr[k] = pld<i>(Fi, hr, sb);
            if constexpr (WH && ey != 0 && halo_row_sel(sel, ey)) vrh[k] = pld<i>(Hi, hr, sb);
          });
        };
        if (!RLB_ZM_ROWS || wv == 1 || wv == 2) load_rows(std::integral_constant<int, 0>{});
        else if (wv == 0) load_rows(std::integral_constant<int, 1>{});
        else load_rows(std::integral_constant<int, -1>{});
        if (lane < 4) {
          static_for<0, NP>([&](auto k) {
            constexpr int i = S0 + k;
            if constexpr (i != 0) vx[k] = pld<i>(Fi, hx, sb);
            if constexpr (WH && vcomp(i, 0) != 0) vxh[k] = pld<i>(Hi, hx, sb);
          });
        }
        if (RLB_ZM_PRIO) __builtin_amdgcn_s_setprio(0);
        // the previous stage's (or plane's) reads of the tiles are done
        if (st > 0 || z > zb) lds_barrier();
        static_for<0, NP>([&](auto k) {
          constexpr int i = S0 + k;
          if constexpr (i != 0) lds[k][2 + wv][2 + lane] = fcen(std::integral_constant<int, i>{});
          if constexpr (WH && (vcomp(i, 0) != 0 || vcomp(i, 1) != 0))
            lds[NP + k][2 + wv][2 + lane] = hcen(std::integral_constant<int, i>{});
        });
        auto store_rows = [&](auto sel) {
          static_for<0, NP>([&](auto k) {
            constexpr int i = S0 + k;
            constexpr int ey = (vcomp(i, 1) > 0) - (vcomp(i, 1) < 0);  // sign
            if constexpr (i != 0 && halo_row_sel(sel, ey)) lds[k][hrow][2 + lane] = vr[k];
            if constexpr (WH && ey != 0 && halo_row_sel(sel, ey)) lds[NP + k][hrow][2 + lane] = vrh[k];
          });
        };
        if (!RLB_ZM_ROWS || wv == 1 || wv == 2) store_rows(std::integral_constant<int, 0>{});
        else if (wv == 0) store_rows(std::integral_constant<int, 1>{});
        else store_rows(std::integral_constant<int, -1>{});
        if (lane < 4) {
          static_for<0, NP>([&](auto k) {
            constexpr int i = S0 + k;
            if constexpr (i != 0) lds[k][2 + wv][hcol] = vx[k];
            if constexpr (WH && vcomp(i, 0) != 0) lds[NP + k][2 + wv][hcol] = vxh[k];
          });
        }
        lds_barrier();
      }
      static_for<S0, S1>([&](auto I) {
        constexpr int i = I;
        constexpr Vel e = vel(i);
        Sten<T> sf, sh;
        if constexpr (i != 0) gather_xy_lds<T, i, true>(lds[i - S0], sf);
        if constexpr (zf_index(i) >= 0) {
          zsten_flux<T, i>(wf[zf_index(i)], sf);
        } else if constexpr (zl_index(i) >= 0) {
          sf.v[2][0] = wl[zl_index(i)][0];
          sf.v[2][1] = wl[zl_index(i)][2];
        }
        const T fci = fcen(I);
        T dD, ns;
        stream_terms<T, ACT, i, (i != 0)>(sf, fci, dtv, dD, ns);
        T v = (fci - dD) * tinv + static_cast<T>(weight(i)) * bracket<i>(Kt);
        if constexpr (i != 0) v += kinv * (ns - NA2 * fci);
        pst<i, kNT>(Fo, cbs, sb, v);
        gE += v;
        gA += fabs(v);
        if constexpr (e.x != 0) gX += T(e.x) * v;
        if constexpr (e.y != 0) gY += T(e.y) * v;
        if constexpr (e.z != 0) gZ += T(e.z) * v;
        if constexpr (WH) {
          gather_xy_lds<T, i, false>(lds[NP + (i - S0)], sh);
          if constexpr (zf_index(i) >= 0) zsten_flux<T, i>(wh[zf_index(i)], sh);
          const T hci = hcen(I);
          T dH, nh;
          stream_terms<T, ACT, i, false>(sh, hci, dtv, dH, nh);
          const T wpi = i == 0 ? wp[0] : (i <= 6 ? wp[1] : wp[2]);
          const T hv = (hci - dH) * tinv + wpi * bracket<i>(Ht);
          pst<i, kNT>(Ho, cbs, sb, hv);
          gN += hv;
          gAh += fabs(hv);
        }
      });
    });

    // guard: gate in storage precision with a rounding margin, decide and
    // blend in FP64 from the stored values (as in k_step)
    if (P.guard) {
      constexpr T tol = T(8e-6);
      const T r2 = static_cast<T>(P.r * P.r), rca = static_cast<T>(P.rca);
      const T Eg = r2 * gE, mrg = tol * r2 * gA;
      const T Mg = rca * sqrt(gX * gX + gY * gY + gZ * gZ);
      bool need = real && (!(Eg > mrg) || (Mg + mrg > static_cast<T>(P.m1) * (Eg - mrg)));
      if constexpr (WH) {
        const T Ng = static_cast<T>(P.r) * gN;
        need = need || (real && !(Ng > static_cast<T>(2.0 * P.efloor * P.gmax) +
                                           tol * static_cast<T>(P.r) * gAh));
      }
      bool fired = false;
      if (need) {
        // the stores of this lane are visible to its own loads
        double E2, Mx2, My2, Mz2, N02;
        moments64<T, WH>(P, [&](auto I) { return pld<I>(Fo, cbs, sb); },
                         [&](auto I) { return pld<I>(Ho, cbs, sb); }, E2, Mx2, My2, Mz2, N02);
        double thf, thh;
        Fields G;
        fired = guard_eval<WH>(P, E2, Mx2, My2, Mz2, N02, thf, thh, G);
        if (fired) {
          double Kg[10];
          feq_coeffs(P, G.eps, G.ux, G.uy, G.uz, G.g2, Kg);
          static_for<0, Q>([&](auto I) {
            const double ge = weight(I) * bracket<I>(Kg);
            const double v = static_cast<double>(pld<I>(Fo, cbs, sb));
            pst<I>(Fo, cbs, sb, static_cast<T>(ge + thf * (v - ge)));
          });
          if constexpr (WH) {
            double Hg[10];
            heq_coeffs(P, G.n, G.ux, G.uy, G.uz, G.gam, Hg);
            static_for<0, Q>([&](auto I) {
              const double ge = wprime<I>(P) * bracket<I>(Hg);
              const double v = static_cast<double>(pld<I>(Ho, cbs, sb));
              pst<I>(Ho, cbs, sb, static_cast<T>(ge + thh * (v - ge)));
            });
          }
        }
      }
      count_events(guard_ptr, fired);
    }

    // next plane: shift the windows
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      wf[k][0] = wf[k][1];
      wf[k][1] = wf[k][2];
      wf[k][2] = wf[k][3];
      if constexpr (WH) {
        wh[k][0] = wh[k][1];
        wh[k][1] = wh[k][2];
        wh[k][2] = wh[k][3];
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      wl[k][0] = wl[k][1];
      wl[k][1] = wl[k][2];
    }
  }
}

// ---------------------------------------------------------------------------
// Temporal blocking of 1D domains: one launch advances KB <= kTbMax steps.
// A workgroup holds a region of kBlock consecutive cells (one per thread):
// its populations and previous fields stay in registers across the steps and
// the population values are exchanged through LDS once per step.  The star
// stencil has radius 2, so after s steps the 2s cells at each end of a region
// are stale; the workgroup owns the kBlock - 4 KB cells in the middle and
// neighbouring regions overlap by 4 KB cells (computed twice, stored once).
// HBM traffic per step falls by the factor KB.  Every owned cell takes the
// single-step kernel's arithmetic in the same order; guard events and
// inadmissible steps are counted by the owner only.  The previous-step fields
// come from hist and go to hist_out (distinct arrays): the halo lanes read
// fields of cells that the neighbouring workgroups own and rewrite, and a
// workgroup may start after its neighbour has finished.  SEG: the region lies in
// one segment of the serving arena (tile table entry (segment, tile)); a
// segment whose steps are done keeps its state.
// ---------------------------------------------------------------------------
constexpr int kTbMax = kTbMaxSteps;

// waves per SIMD the register allocator must allow (measured: FP32 3, which
// spills a few registers in the guarded implicit path but runs large domains
// 8-10% faster than 2; FP64 2)
#ifndef RLB_TB_OCC_F32
#define RLB_TB_OCC_F32 3
#endif
#ifndef RLB_TB_OCC_F64
#define RLB_TB_OCC_F64 2
#endif
template <typename T>
struct TbOcc {
  static constexpr int value = sizeof(T) == 4 ? RLB_TB_OCC_F32 : RLB_TB_OCC_F64;
};
// Rusanov (local Lax-Friedrichs) flux along x, first order -- beyond the
// paper: the interface flux 1/2 p (f_L + f_R) - 1/2 s (f_R - f_L) with one
// dissipation speed s for every population, moving or not (the speed of
// light), so that the moments of the update are the Rusanov scheme of the
// fluid equations.  cx = dt p (the population's Courant number along x),
// cs = dt s.  dD: dt times the flux divergence; nsum: the Laplacian's
// neighbour sum.  With this flux the bulk term acts on the rest population
// too (its weight is negative; without it the term would remove the rest
// population's energy at the cell and break the convexity that keeps the
// moment update admissible).
template <typename T>
__device__ __forceinline__ void rusanov_terms(T fm, T f0, T fp, T cx, T cs, T& dD, T& nsum) {
  dD = T(0.5) * cx * (fp - fm) - T(0.5) * cs * ((fp - f0) - (f0 - fm));
  nsum = fm + fp;
}

template <typename T, bool WH, bool EU, bool SEG, bool RUS>
__global__ __launch_bounds__(kBlock, (TbOcc<T>::value)) void k_step_tb(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ hin,
    T* __restrict__ hout, const double* __restrict__ hist, double* __restrict__ hist_out,
    const uint8_t* __restrict__ obst, const StepParams P, int KB) {
  constexpr int R = kBlock;
  constexpr int NA = WH ? 2 * Q : Q;
  __shared__ T lds[NA][R + 2];  // slots R, R + 1: the fixed end states
  const int p = static_cast<int>(threadIdx.x);
  const int B = R - 4 * KB;
  const long long S = P.pstride;
  // the domain: n cells at storage indices base0 + [0, n), its end conditions
  long long base0, face_lo, face_hi;
  int n, bclo, bchi, tile, nupd;
  long long step0;
  double kappa_d = P.kappa, nu2e = P.nu2_etas, tau_u = P.tau;
  unsigned long long* bad_ptr = P.bad_step;
  unsigned long long* guard_ptr = P.guard_count;
  if constexpr (SEG) {
    const int2 t = P.tiles[blockIdx.x];
    if (t.x < 0) return;  // the whole workgroup: no barrier is skipped
    const SegDesc& sd = P.segs[t.x];
    base0 = sd.base + 1;
    face_lo = sd.base;
    face_hi = sd.base + 1 + sd.n;
    n = sd.n;
    bclo = sd.bc_lo;
    bchi = sd.bc_hi;
    tile = t.y;
    kappa_d = sd.kappa;
    nu2e = sd.nu2_etas;
    tau_u = sd.tau;
    bad_ptr = sd.bad + sd.id;
    guard_ptr = sd.guard + sd.id;
    step0 = *P.gstep + P.step_in_chunk - sd.start;
    const long long left = sd.steps - step0;
    nupd = left <= 0 ? 0 : (left < KB ? static_cast<int>(left) : KB);
  } else {
    base0 = 0;
    face_lo = P.ncell;
    face_hi = P.ncell + 1;
    n = P.nx;
    bclo = P.bc[0];
    bchi = P.bc[1];
    tile = static_cast<int>(blockIdx.x);
    step0 = P.step_index;
    nupd = KB;
  }
  const bool periodic = bclo == kBcPeriodic;
  const long long q = static_cast<long long>(tile) * B - 2 * KB + p;  // this lane's cell
  const bool active = periodic || (q >= 0 && q < n);
  const long long x = periodic ? ((q % n) + n) % n : (active ? q : 0);
  const bool owned = p >= 2 * KB && p < 2 * KB + B && q >= 0 && q < n;
  // LDS positions of the neighbours at offsets -2, -1, +1, +2 (periodic: the
  // region holds the wrapped cells; fixed: the face slot; outflow: the end
  // cell; positions past the region end are clamped and only feed stale lanes)
  int pos[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = j < 2 ? j - 2 : j - 1;
    const long long qq = q + k;
    long long ps = p + k;
    bool face = false;
    if (!periodic && qq < 0) {
      face = bclo == kBcFixed;
      ps = face ? R : p - q;
    } else if (!periodic && qq >= n) {
      face = bchi == kBcFixed;
      ps = face ? R + 1 : p - q + (n - 1);
    }
    if (!face) ps = ps < 0 ? 0 : (ps > R - 1 ? R - 1 : ps);
    pos[j] = static_cast<int>(ps);
  }
  const long long cs = base0 + x;
  const unsigned cl = static_cast<unsigned>(cs) * static_cast<unsigned>(sizeof(T));
  const unsigned cd = static_cast<unsigned>(cs) * 8u;
  const long long NC = P.ncell;
  bool solid = false;
  if constexpr (!SEG) solid = obst != nullptr && active && obst[cs] != 0;

  // fixed end states (the face slots or the segment's ghost cells)
  for (int a = p; a < 2 * NA; a += R) {
    const int arr = a % NA, side = a / NA;
    const long long at = side ? face_hi : face_lo;
    const T* src = arr < Q ? fin + arr * S : hin + (arr - Q) * S;
    lds[arr][R + side] = src[at];
  }
  T fc[Q];
  T hc[Q];
  double pe = 0.0, pux = 0.0, puy = 0.0, puz = 0.0, pn = 1.0;  // previous fields
  if (active) {
    static_for<0, Q>([&](auto I) {
      fc[I] = ldb(fin + I * S, cl);
      if constexpr (WH) hc[I] = ldb(hin + I * S, cl);
    });
    pe = ldb(hist, cd);
    pux = ldb(hist + NC, cd);
    puy = ldb(hist + 2 * NC, cd);
    puz = ldb(hist + 3 * NC, cd);
    pn = ldb(hist + 4 * NC, cd);
  }
  const T dtv = static_cast<T>(P.dtv);
  const T dtc = static_cast<T>(P.dtv * sqrt(27.0 / 13.0));  // dt times the speed of light
  constexpr T NA2 = T(2);

  for (int st = 0; st < KB; ++st) {
    __syncthreads();  // the previous step's neighbour reads are done
    if (active) {
      static_for<0, Q>([&](auto I) {
        lds[I][p] = fc[I];
        if constexpr (WH) lds[Q + I][p] = hc[I];
      });
    }
    __syncthreads();
    if (!active || solid || st >= nupd) continue;
    const long long sidx = step0 + st;
    // stencil of population I (axis x only) from the LDS row
    auto sten = [&](auto I, int arr, bool lap, Sten<T>& sv) {
      constexpr int ea = vcomp(I, 0);
      if constexpr (ea > 0) {
        sv.v[0][0] = lds[arr][pos[0]];
        sv.v[0][1] = lds[arr][pos[1]];
        sv.v[0][2] = lds[arr][pos[2]];
      } else if constexpr (ea < 0) {
        sv.v[0][0] = lds[arr][pos[1]];
        sv.v[0][1] = lds[arr][pos[2]];
        sv.v[0][2] = lds[arr][pos[3]];
      } else {
        if (lap) {
          sv.v[0][0] = lds[arr][pos[1]];
          sv.v[0][1] = lds[arr][pos[2]];
        }
      }
    };
    if constexpr (EU) {
      const T kap = static_cast<T>(kappa_d);
      double m0 = 0.0, mx = 0.0, my = 0.0, mz = 0.0, mh = 0.0;
      static_for<0, Q>([&](auto I) {
        constexpr Vel e = vel(I);
        T dD, ns;
        if constexpr (RUS) {
          rusanov_terms(lds[I][pos[1]], fc[I], lds[I][pos[2]], dtv * T(e.x), dtc, dD, ns);
        } else {
          Sten<T> sf;
          sten(I, I, I != 0, sf);
          stream_terms<T, 1, I, (I != 0)>(sf, fc[I], dtv, dD, ns);
        }
        T v;
        if constexpr (I != 0 || RUS) v = (fc[I] - dD) + kap * (ns - NA2 * fc[I]);
        else v = fc[I] - dD;
        const double vd = static_cast<double>(v);
        m0 += vd;
        if constexpr (e.x != 0) mx += double(e.x) * vd;
        if constexpr (e.y != 0) my += double(e.y) * vd;
        if constexpr (e.z != 0) mz += double(e.z) * vd;
        if constexpr (WH) {
          T dH, nh;
          if constexpr (RUS) {
            rusanov_terms(lds[Q + I][pos[1]], hc[I], lds[Q + I][pos[2]], dtv * T(e.x), dtc, dH, nh);
          } else {
            Sten<T> sh;
            sten(I, Q + I, false, sh);
            stream_terms<T, 1, I, false>(sh, hc[I], dtv, dH, nh);
          }
          mh += static_cast<double>(hc[I] - dH);
        }
      });
      const double E = P.r * P.r * m0, Mx = P.rca * mx, My = P.rca * my, Mz = P.rca * mz,
                   N0 = P.r * mh;
      Fields F;
      bool ok = true, fired = false;
      if (P.guard) {
        double thf, thh;
        fired = guard_eval<WH>(P, E, Mx, My, Mz, N0, thf, thh, F);
        count_events(guard_ptr, fired && owned);
      }
      if (!fired) ok = recover<WH>(E, Mx, My, Mz, N0, F);
      flag_bad(bad_ptr, !ok && owned, sidx);
      double K[10];
      feq_coeffs(P, F.eps, F.ux, F.uy, F.uz, F.g2, K);
      T Kt[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) Kt[k] = static_cast<T>(K[k]);
      static_for<0, Q>([&](auto I) { fc[I] = static_cast<T>(weight(I)) * bracket<I>(Kt); });
      if constexpr (WH) {
        double H[10];
        heq_coeffs(P, F.n, F.ux, F.uy, F.uz, F.gam, H);
        T Ht[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) Ht[k] = static_cast<T>(H[k]);
        static_for<0, Q>([&](auto I) { hc[I] = static_cast<T>(wprime<I>(P)) * bracket<I>(Ht); });
      }
    } else {
      double E, Mx, My, Mz, N0;
      moments64<T, WH>(P, [&](auto I) { return fc[I]; }, [&](auto I) { return hc[I]; }, E, Mx, My,
                       Mz, N0);
      Fields F;
      const bool ok = recover<WH>(E, Mx, My, Mz, N0, F);
      flag_bad(bad_ptr, !ok && owned, sidx);
      const double omega = P.omega_c / tau_of<T, WH>(P, F, tau_u, nu2e);
      const double inv1p = 1.0 / (1.0 + omega);
      const double src = omega * inv1p;
      const double pg2 = 1.0 / (1.0 - (pux * pux + puy * puy + puz * puz));
      T Kt[10];
      {
        double K[10], Kp[10];
        feq_coeffs(P, F.eps, F.ux, F.uy, F.uz, F.g2, K);
        feq_coeffs(P, pe, pux, puy, puz, pg2, Kp);
#pragma unroll
        for (int k = 0; k < 10; ++k) Kt[k] = static_cast<T>(src * (2.0 * K[k] - Kp[k]));
      }
      T Ht[10];
      if constexpr (WH) {
        double H[10], Hp[10];
        heq_coeffs(P, F.n, F.ux, F.uy, F.uz, F.gam, H);
        heq_coeffs(P, pn, pux, puy, puz, sqrt(pg2), Hp);
#pragma unroll
        for (int k = 0; k < 10; ++k) Ht[k] = static_cast<T>(src * (2.0 * H[k] - Hp[k]));
      }
      pe = F.eps;
      pux = F.ux;
      puy = F.uy;
      puz = F.uz;
      pn = F.n;
      const T tinv = static_cast<T>(inv1p);
      const T kinv = static_cast<T>(kappa_d * inv1p);
      const T wp[3] = {static_cast<T>(P.wp0), static_cast<T>(P.wp1), static_cast<T>(P.wp2)};
      T gE = T(0), gX = T(0), gY = T(0), gZ = T(0), gN = T(0), gA = T(0), gAh = T(0);
      static_for<0, Q>([&](auto I) {
        constexpr Vel e = vel(I);
        T dD, ns;
        if constexpr (RUS) {
          rusanov_terms(lds[I][pos[1]], fc[I], lds[I][pos[2]], dtv * T(e.x), dtc, dD, ns);
        } else {
          Sten<T> sf;
          sten(I, I, I != 0, sf);
          stream_terms<T, 1, I, (I != 0)>(sf, fc[I], dtv, dD, ns);
        }
        T v = (fc[I] - dD) * tinv + static_cast<T>(weight(I)) * bracket<I>(Kt);
        if constexpr (I != 0 || RUS) v += kinv * (ns - NA2 * fc[I]);
        fc[I] = v;
        gE += v;
        gA += fabs(v);
        if constexpr (e.x != 0) gX += T(e.x) * v;
        if constexpr (e.y != 0) gY += T(e.y) * v;
        if constexpr (e.z != 0) gZ += T(e.z) * v;
        if constexpr (WH) {
          T dH, nh;
          if constexpr (RUS) {
            rusanov_terms(lds[Q + I][pos[1]], hc[I], lds[Q + I][pos[2]], dtv * T(e.x), dtc, dH, nh);
          } else {
            Sten<T> sh;
            sten(I, Q + I, false, sh);
            stream_terms<T, 1, I, false>(sh, hc[I], dtv, dH, nh);
          }
          const T wpi = I == 0 ? wp[0] : (I <= 6 ? wp[1] : wp[2]);
          const T hv = (hc[I] - dH) * tinv + wpi * bracket<I>(Ht);
          hc[I] = hv;
          gN += hv;
          gAh += fabs(hv);
          asm volatile("" : "+v"(gN), "+v"(gAh));
        }
        asm volatile("" : "+v"(gE), "+v"(gA), "+v"(gX), "+v"(gY), "+v"(gZ));
      });
      if (P.guard) {
        constexpr T tol = sizeof(T) == 4 ? T(8e-6) : T(1e-13);
        const T r2 = static_cast<T>(P.r * P.r), rca = static_cast<T>(P.rca);
        const T Eg = r2 * gE, mrg = tol * r2 * gA;
        const T Mg = rca * sqrt(gX * gX + gY * gY + gZ * gZ);
        bool need = !(Eg > mrg) || (Mg + mrg > static_cast<T>(P.m1) * (Eg - mrg));
        if constexpr (WH) {
          const T Ng = static_cast<T>(P.r) * gN;
          need = need || !(Ng > static_cast<T>(2.0 * P.efloor * P.gmax) + tol * static_cast<T>(P.r) * gAh);
        }
        bool fired = false;
        if (need) {
          double E2, Mx2, My2, Mz2, N02;
          moments64<T, WH>(P, [&](auto I) { return fc[I]; }, [&](auto I) { return hc[I]; }, E2,
                           Mx2, My2, Mz2, N02);
          double thf, thh;
          Fields G;
          fired = guard_eval<WH>(P, E2, Mx2, My2, Mz2, N02, thf, thh, G);
          if (fired) {
            double Kg[10];
            feq_coeffs(P, G.eps, G.ux, G.uy, G.uz, G.g2, Kg);
            static_for<0, Q>([&](auto I) {
              const double ge = weight(I) * bracket<I>(Kg);
              fc[I] = static_cast<T>(ge + thf * (static_cast<double>(fc[I]) - ge));
            });
            if constexpr (WH) {
              double Hg[10];
              heq_coeffs(P, G.n, G.ux, G.uy, G.uz, G.gam, Hg);
              static_for<0, Q>([&](auto I) {
                const double ge = wprime<I>(P) * bracket<I>(Hg);
                hc[I] = static_cast<T>(ge + thh * (static_cast<double>(hc[I]) - ge));
              });
            }
          }
        }
        count_events(guard_ptr, fired && owned);
      }
    }
  }
  if (owned) {
    static_for<0, Q>([&](auto I) {
      stb_nt(fout + I * S, cl, fc[I]);
      if constexpr (WH) stb_nt(hout + I * S, cl, hc[I]);
    });
    if constexpr (!EU) {
      stb_nt(hist_out, cd, pe);
      stb_nt(hist_out + NC, cd, pux);
      stb_nt(hist_out + 2 * NC, cd, puy);
      stb_nt(hist_out + 3 * NC, cd, puz);
      stb_nt(hist_out + 4 * NC, cd, pn);
    }
  }
}

// ---------------------------------------------------------------------------
// Basic model (Sec. II): standard D3Q19 set, exact streaming (dt = c_t dx /
// (c_a c_0) moves every population one link per step), explicit Marle
// collision f' = f - omega (f - f^eq), omega = c_0 nu dt / (c_t tau); no
// limiter, no bulk term, energy-momentum distribution only.  The arrays hold
// post-collision values: a step pulls f_i from x - e_i, forms the moments,
// recovers the fields, collides and stores, one thread per cell with global
// loads (no stencil beyond one link, so no LDS staging).  The pulled cell
// x - e_i is mapped per axis (periodic wrap, outflow clamp); across a FIXED
// face it is that face's slot, and at an edge the later axis's FIXED face
// wins (axis-by-axis ghost filling).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ unsigned pull_offset(const StepParams& P, int x, int y, int z, int ex,
                                                int ey, int ez) {
  int q[3] = {x - ex, y - ey, z - ez};
  const int n[3] = {P.nx, P.ny, P.nz};
  long long face = -1;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (q[a] >= 0 && q[a] < n[a]) continue;
    const int side = q[a] < 0 ? 0 : 1;
    const int b = P.bc[2 * a + side];
    if (b == kBcFixed) {
      face = P.ncell + 2 * a + side;
      q[a] = side ? n[a] - 1 : 0;
    } else if (b == kBcPeriodic) {
      q[a] += side ? -n[a] : n[a];
    } else {
      q[a] = side ? n[a] - 1 : 0;
    }
  }
  const long long idx =
      face >= 0 ? face : q[0] + static_cast<long long>(P.px) * (q[1] + static_cast<long long>(P.py) * q[2]);
  return static_cast<unsigned>(idx) * static_cast<unsigned>(sizeof(T));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_step_basic(const T* __restrict__ fin,
                                                        T* __restrict__ fout,
                                                        const double* __restrict__ hist,
                                                        const uint8_t* __restrict__ obst,
                                                        const StepParams P) {
  int x, y, z;
  if (!cell_of(P, x, y, z)) return;
  if (x >= P.nx || y >= P.ny) return;  // no barriers: lanes past the end leave
  const long long S = P.pstride, NC = P.ncell;
  const long long c = x + static_cast<long long>(P.px) * (y + static_cast<long long>(P.py) * z);
  const unsigned cb = static_cast<unsigned>(c) * static_cast<unsigned>(sizeof(T));
  if (obst != nullptr && obst[c] != 0) {
    // held at the equilibrium of its prescribed fields
    const double eps = hist[c], ux = hist[NC + c], uy = hist[2 * NC + c], uz = hist[3 * NC + c];
    const double g2 = 1.0 / (1.0 - (ux * ux + uy * uy + uz * uz));
    double K[10];
    feq_coeffs<1>(P, eps, ux, uy, uz, g2, K);
    static_for<0, Q>([&](auto I) {
      stb_nt(fout + I * S, cb, static_cast<T>(weight_l<1>(I) * bracket<I, 1>(K)));
    });
    return;
  }
  T f[Q];
  static_for<0, Q>([&](auto I) {
    constexpr Vel e = vel_l<1>(I);
    f[I] = ldb(fin + I * S, pull_offset<T>(P, x, y, z, e.x, e.y, e.z));
  });
  double E, Mx, My, Mz, N0;
  moments64<T, false, 1>(P, [&](auto I) { return f[I]; }, [&](auto I) { return T(0); }, E, Mx, My,
                         Mz, N0);
  Fields F;
  const bool ok = recover<false>(E, Mx, My, Mz, N0, F);
  flag_bad(P.bad_step, !ok, P.step_index);
  const T om = static_cast<T>(P.omega_c / tau_of<T, false>(P, F, P.tau, P.nu2_etas));
  double K[10];
  feq_coeffs<1>(P, F.eps, F.ux, F.uy, F.uz, F.g2, K);
  T Kt[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) Kt[k] = static_cast<T>(K[k]);
  static_for<0, Q>([&](auto I) {
    const T feq = static_cast<T>(weight_l<1>(I)) * bracket<I, 1>(Kt);
    stb_nt(fout + I * S, cb, f[I] - om * (f[I] - feq));
  });
}

// Storage index x + px (y + py z) of dense cell l = x + nx (y + ny z).
__device__ __forceinline__ long long store_index(const StepParams& P, long long l) {
  if (P.px == P.nx && P.py == P.ny) return l;
  const long long row = l / P.nx, z = row / P.ny;
  return (row - z * P.ny + z * P.py) * P.px + (l - row * P.nx);
}

// f := f^eq(fields), h := h^eq(fields) from the fields held in hist; without
// density the lattice equilibrium density (eps/3)^(3/4) is written to hist.
// L: lattice (0 extended, 1 basic).
template <typename T, bool WH, int L>
__global__ __launch_bounds__(kBlock) void k_init(const StepParams P) {
  const long long r = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (r >= P.range) return;
  const long long c = store_index(P, P.cell0 + r);
  const long long NC = P.ncell, S = P.pstride;
  T* __restrict__ f = static_cast<T*>(P.f_out);
  T* __restrict__ h = static_cast<T*>(P.h_out);
  const double eps = P.hist[c], ux = P.hist[NC + c], uy = P.hist[2 * NC + c],
               uz = P.hist[3 * NC + c];
  const double g2 = 1.0 / (1.0 - (ux * ux + uy * uy + uz * uz));
  double K[10];
  feq_coeffs<L>(P, eps, ux, uy, uz, g2, K);
  static_for<0, Q>(
      [&](auto I) { f[I * S + c] = static_cast<T>(weight_l<L>(I) * bracket<I, L>(K)); });
  if constexpr (WH) {
    static_assert(L == 0, "the density distribution is carried by the extended model only");
    double H[10];
    heq_coeffs(P, P.hist[4 * NC + c], ux, uy, uz, sqrt(g2), H);
    static_for<0, Q>([&](auto I) { h[I * S + c] = static_cast<T>(wprime<I>(P) * bracket<I>(H)); });
  } else {
    P.hist[4 * NC + c] = pow(eps / 3.0, 0.75);
  }
  if (P.hist32 != nullptr) {
    // compact previous-step fields (eps, gamma u, n) in FP32
    const double gam = sqrt(g2);
    P.hist32[c] = static_cast<float>(eps);
    P.hist32[NC + c] = static_cast<float>(gam * ux);
    P.hist32[2 * NC + c] = static_cast<float>(gam * uy);
    P.hist32[3 * NC + c] = static_cast<float>(gam * uz);
    P.hist32[4 * NC + c] = static_cast<float>(P.hist[4 * NC + c]);
  }
}

// Face slots: equilibria of the six face states in both ping-pong copies.
template <typename T, int L>
__global__ void k_face_slots(const StepParams P, const double* states, T* f0, T* f1, T* h0, T* h1) {
  const int s = threadIdx.x;
  if (s >= kFaceSlots) return;
  const double* q = states + 5 * s;
  const double g2 = 1.0 / (1.0 - (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]));
  double K[10], H[10];
  feq_coeffs<L>(P, q[0], q[1], q[2], q[3], g2, K);
  heq_coeffs(P, q[4], q[1], q[2], q[3], sqrt(g2), H);
  const long long S = P.pstride, at = P.ncell + s;
  static_for<0, Q>([&](auto I) {
    const T fe = static_cast<T>(weight_l<L>(I) * bracket<I, L>(K));
    f0[I * S + at] = fe;
    f1[I * S + at] = fe;
    if (h0 != nullptr) {
      const T he = static_cast<T>(wprime<I>(P) * bracket<I>(H));
      h0[I * S + at] = he;
      h1[I * S + at] = he;
    }
  });
}

// Fields of the current populations (FP64 recovery); NaN where inadmissible.
template <typename T, bool WH, int L>
__global__ __launch_bounds__(kBlock) void k_moments(const StepParams P, double* out,
                                                     unsigned long long* bad) {
  const long long r = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (r >= P.range) return;
  const long long c = store_index(P, P.cell0 + r);
  const long long NC = P.range, S = P.pstride;
  const T* __restrict__ f = static_cast<const T*>(P.f_in);
  const T* __restrict__ h = static_cast<const T*>(P.h_in);
  double E, Mx, My, Mz, N0;
  moments64<T, WH, L>(P, [&](auto I) { return f[I * S + c]; }, [&](auto I) { return h[I * S + c]; },
                      E, Mx, My, Mz, N0);
  Fields F;
  const bool ok = recover<WH>(E, Mx, My, Mz, N0, F);
  const bool obst = P.obst != nullptr && P.obst[c] != 0;
  flag_bad(bad, !ok && !obst, 0);
  out[r] = ok ? F.eps : NAN;
  out[NC + r] = ok ? F.ux : NAN;
  out[2 * NC + r] = ok ? F.uy : NAN;
  out[3 * NC + r] = ok ? F.uz : NAN;
  out[4 * NC + r] = ok ? F.n : NAN;
}

// Deterministic domain sums of T^{00}, T^{0a}, N^0 over the P.range dense
// cells: per-block tree sums into partial[block][5], then one block adds the
// partials in index order.
template <typename T, bool WH, int L>
__global__ __launch_bounds__(kBlock) void k_sums_partial(const StepParams P, double* partial) {
  __shared__ double red[5][kBlock];
  const long long l = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  double v[5] = {0, 0, 0, 0, 0};
  if (l < P.range) {
    const long long S = P.pstride, c = store_index(P, l);
    const T* __restrict__ f = static_cast<const T*>(P.f_in);
    const T* __restrict__ h = static_cast<const T*>(P.h_in);
    moments64<T, WH, L>(P, [&](auto I) { return f[I * S + c]; }, [&](auto I) { return h[I * S + c]; },
                        v[0], v[1], v[2], v[3], v[4]);
  }
  for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s)
      for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) partial[static_cast<long long>(blockIdx.x) * 5 + k] = red[k][0];
}

__global__ __launch_bounds__(kBlock) void k_sums_final(const double* partial, int nblocks,
                                                        double* out5) {
  __shared__ double red[5][kBlock];
  double v[5] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += kBlock)
    for (int k = 0; k < 5; ++k) v[k] += partial[static_cast<long long>(b) * 5 + k];
  for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s)
      for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) out5[k] = red[k][0];
}

template <typename T, int ACT, bool WH, bool EU>
hipError_t launch_step_t(const StepParams& p, hipStream_t s) {
  if (p.flux == kFluxRusanov) {
    // the staged step (2D/3D); 1D grids take the blocked step (k_step_tb)
    if constexpr (ACT == 1) {
      return hipErrorInvalidValue;
    } else {
      const long long nblk = p.tiles_per_xcd * kXcds;
      hipLaunchKernelGGL((k_step<T, ACT, WH, EU, false, true>), dim3(static_cast<unsigned>(nblk)), dim3(kBlock),
                         0, s, static_cast<const T*>(p.f_in), static_cast<T*>(p.f_out),
                         static_cast<const T*>(p.h_in), static_cast<T*>(p.h_out), p.hist, p.obst, p);
      return hipGetLastError();
    }
  }
  if constexpr (ACT == 7 && !EU && std::is_same<T, float>::value) {
    if (p.zm_len > 0) {
      const long long nblk = p.zm_per_xcd * kXcds;
      hipLaunchKernelGGL((k_step_zm<T, WH>), dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0, s,
                         static_cast<const T*>(p.f_in), static_cast<T*>(p.f_out),
                         static_cast<const T*>(p.h_in), static_cast<T*>(p.h_out), p.hist, p.obst, p);
      return hipGetLastError();
    }
  }
  const long long nblk = p.tiles_per_xcd * kXcds;
  hipLaunchKernelGGL((k_step<T, ACT, WH, EU, false>), dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0,
                     s, static_cast<const T*>(p.f_in), static_cast<T*>(p.f_out),
                     static_cast<const T*>(p.h_in), static_cast<T*>(p.h_out), p.hist, p.obst, p);
  return hipGetLastError();
}

template <typename T, int ACT>
hipError_t launch_step_a(const StepParams& p, bool with_h, bool euler, hipStream_t s) {
  if (with_h) {
    return euler ? launch_step_t<T, ACT, true, true>(p, s) : launch_step_t<T, ACT, true, false>(p, s);
  }
  return euler ? launch_step_t<T, ACT, false, true>(p, s) : launch_step_t<T, ACT, false, false>(p, s);
}

template <typename T>
hipError_t launch_step_p(const StepParams& p, int act, bool with_h, bool euler, hipStream_t s) {
  switch (act) {
    case 1: return launch_step_a<T, 1>(p, with_h, euler, s);
    case 3: return launch_step_a<T, 3>(p, with_h, euler, s);
    case 7: return launch_step_a<T, 7>(p, with_h, euler, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, bool WH, bool EU>
hipError_t launch_seg_t(const StepParams& p, unsigned grid, hipStream_t s) {
  hipLaunchKernelGGL((k_step<T, 1, WH, EU, true>), dim3(grid), dim3(kBlock), 0, s,
                     static_cast<const T*>(p.f_in), static_cast<T*>(p.f_out),
                     static_cast<const T*>(p.h_in), static_cast<T*>(p.h_out), p.hist, nullptr, p);
  return hipGetLastError();
}

template <typename T>
__global__ void k_seg_ghosts(const StepParams P, long long lo, long long hi, const double* states,
                             T* f0, T* f1, T* h0, T* h1) {
  const int s = threadIdx.x;
  if (s >= 2) return;
  const double* q = states + 5 * s;
  const double g2 = 1.0 / (1.0 - (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]));
  double K[10], H[10];
  feq_coeffs(P, q[0], q[1], q[2], q[3], g2, K);
  heq_coeffs(P, q[4], q[1], q[2], q[3], sqrt(g2), H);
  const long long S = P.pstride, at = s == 0 ? lo : hi;
  static_for<0, Q>([&](auto I) {
    const T fe = static_cast<T>(weight(I) * bracket<I>(K));
    f0[I * S + at] = fe;
    f1[I * S + at] = fe;
    if (h0 != nullptr) {
      const T he = static_cast<T>(wprime<I>(P) * bracket<I>(H));
      h0[I * S + at] = he;
      h1[I * S + at] = he;
    }
  });
}

}  // namespace

hipError_t launch_seg_step(const StepParams& p, bool fp64, bool with_h, bool euler, unsigned grid,
                           hipStream_t s) {
  if (grid == 0) return hipSuccess;
  if (fp64) {
    if (with_h) return euler ? launch_seg_t<double, true, true>(p, grid, s) : launch_seg_t<double, true, false>(p, grid, s);
    return euler ? launch_seg_t<double, false, true>(p, grid, s) : launch_seg_t<double, false, false>(p, grid, s);
  }
  if (with_h) return euler ? launch_seg_t<float, true, true>(p, grid, s) : launch_seg_t<float, true, false>(p, grid, s);
  return euler ? launch_seg_t<float, false, true>(p, grid, s) : launch_seg_t<float, false, false>(p, grid, s);
}

hipError_t launch_seg_ghosts(const StepParams& p, bool fp64, long long lo, long long hi,
                             const double* states, void* f0, void* f1, void* h0, void* h1,
                             hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(k_seg_ghosts<double>, dim3(1), dim3(64), 0, s, p, lo, hi, states,
                       static_cast<double*>(f0), static_cast<double*>(f1), static_cast<double*>(h0),
                       static_cast<double*>(h1));
  else
    hipLaunchKernelGGL(k_seg_ghosts<float>, dim3(1), dim3(64), 0, s, p, lo, hi, states,
                       static_cast<float*>(f0), static_cast<float*>(f1), static_cast<float*>(h0),
                       static_cast<float*>(h1));
  return hipGetLastError();
}

hipError_t launch_step(const StepParams& p, bool fp64, int act_mask, bool with_h, bool euler,
                       hipStream_t s) {
  if (p.lattice == 1) {
    // basic model: f only, regular collision (checked by the host)
    if (with_h || euler) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(p.tiles_per_xcd * kXcds));
    if (fp64)
      hipLaunchKernelGGL(k_step_basic<double>, grid, dim3(kBlock), 0, s,
                         static_cast<const double*>(p.f_in), static_cast<double*>(p.f_out), p.hist,
                         p.obst, p);
    else
      hipLaunchKernelGGL(k_step_basic<float>, grid, dim3(kBlock), 0, s,
                         static_cast<const float*>(p.f_in), static_cast<float*>(p.f_out), p.hist,
                         p.obst, p);
    return hipGetLastError();
  }
  return fp64 ? launch_step_p<double>(p, act_mask, with_h, euler, s)
              : launch_step_p<float>(p, act_mask, with_h, euler, s);
}

namespace {
template <typename T, bool WH, bool EU, bool SEG, bool RUS>
void tb_t(const StepParams& p, int kb, unsigned grid, hipStream_t s) {
  hipLaunchKernelGGL((k_step_tb<T, WH, EU, SEG, RUS>), dim3(grid), dim3(kBlock), 0, s,
                     static_cast<const T*>(p.f_in), static_cast<T*>(p.f_out),
                     static_cast<const T*>(p.h_in), static_cast<T*>(p.h_out), p.hist, p.hist_out,
                     SEG ? nullptr : p.obst, p, kb);
}
template <typename T, bool SEG, bool RUS>
void tb_p(const StepParams& p, bool with_h, bool euler, int kb, unsigned grid, hipStream_t s) {
  if (with_h)
    euler ? tb_t<T, true, true, SEG, RUS>(p, kb, grid, s) : tb_t<T, true, false, SEG, RUS>(p, kb, grid, s);
  else
    euler ? tb_t<T, false, true, SEG, RUS>(p, kb, grid, s) : tb_t<T, false, false, SEG, RUS>(p, kb, grid, s);
}
}  // namespace

int tb_cells_per_tile(int kb) { return kBlock - 4 * kb; }

hipError_t launch_step_tb(const StepParams& p, bool fp64, bool with_h, bool euler, int kb,
                          bool seg, unsigned grid, hipStream_t s) {
  if (kb < 1 || kb > kTbMax || p.lattice != 0) return hipErrorInvalidValue;
  if (p.hist_out == nullptr || p.hist_out == p.hist) return hipErrorInvalidValue;
  if (p.flux != kFluxMinmod && (seg || p.flux != kFluxRusanov)) return hipErrorInvalidValue;
  if (grid == 0) return hipSuccess;
  if (p.flux == kFluxRusanov)
    fp64 ? tb_p<double, false, true>(p, with_h, euler, kb, grid, s)
         : tb_p<float, false, true>(p, with_h, euler, kb, grid, s);
  else if (fp64)
    seg ? tb_p<double, true, false>(p, with_h, euler, kb, grid, s)
        : tb_p<double, false, false>(p, with_h, euler, kb, grid, s);
  else
    seg ? tb_p<float, true, false>(p, with_h, euler, kb, grid, s)
        : tb_p<float, false, false>(p, with_h, euler, kb, grid, s);
  return hipGetLastError();
}

namespace {
// Instantiation helpers: (T, with_h, lattice) of the per-cell kernels.  The
// density distribution exists in the extended model only.
template <typename T, bool WH, int L>
void init_t(const StepParams& p, unsigned nb, hipStream_t s) {
  hipLaunchKernelGGL((k_init<T, WH, L>), dim3(nb), dim3(kBlock), 0, s, p);
}
template <typename T>
void init_p(const StepParams& p, bool with_h, unsigned nb, hipStream_t s) {
  if (p.lattice == 1) init_t<T, false, 1>(p, nb, s);
  else if (with_h) init_t<T, true, 0>(p, nb, s);
  else init_t<T, false, 0>(p, nb, s);
}
template <typename T, bool WH, int L>
void moments_t(const StepParams& p, unsigned nb, double* out, unsigned long long* bad, hipStream_t s) {
  hipLaunchKernelGGL((k_moments<T, WH, L>), dim3(nb), dim3(kBlock), 0, s, p, out, bad);
}
template <typename T>
void moments_p(const StepParams& p, bool with_h, unsigned nb, double* out, unsigned long long* bad,
               hipStream_t s) {
  if (p.lattice == 1) moments_t<T, false, 1>(p, nb, out, bad, s);
  else if (with_h) moments_t<T, true, 0>(p, nb, out, bad, s);
  else moments_t<T, false, 0>(p, nb, out, bad, s);
}
template <typename T, bool WH, int L>
void sums_t(const StepParams& p, int nb, double* partial, hipStream_t s) {
  hipLaunchKernelGGL((k_sums_partial<T, WH, L>), dim3(nb), dim3(kBlock), 0, s, p, partial);
}
template <typename T>
void sums_p(const StepParams& p, bool with_h, int nb, double* partial, hipStream_t s) {
  if (p.lattice == 1) sums_t<T, false, 1>(p, nb, partial, s);
  else if (with_h) sums_t<T, true, 0>(p, nb, partial, s);
  else sums_t<T, false, 0>(p, nb, partial, s);
}
template <typename T>
void face_p(const StepParams& p, const double* states, void* f0, void* f1, void* h0, void* h1,
            hipStream_t s) {
  if (p.lattice == 1)
    hipLaunchKernelGGL((k_face_slots<T, 1>), dim3(1), dim3(64), 0, s, p, states, static_cast<T*>(f0),
                       static_cast<T*>(f1), static_cast<T*>(h0), static_cast<T*>(h1));
  else
    hipLaunchKernelGGL((k_face_slots<T, 0>), dim3(1), dim3(64), 0, s, p, states, static_cast<T*>(f0),
                       static_cast<T*>(f1), static_cast<T*>(h0), static_cast<T*>(h1));
}
}  // namespace

hipError_t launch_init(const StepParams& p, bool fp64, bool with_h, hipStream_t s) {
  const unsigned nb = static_cast<unsigned>((p.range + kBlock - 1) / kBlock);
  if (fp64) init_p<double>(p, with_h, nb, s);
  else init_p<float>(p, with_h, nb, s);
  return hipGetLastError();
}

hipError_t launch_face_slots(const StepParams& p, bool fp64, const double* states, void* f0, void* f1,
                             void* h0, void* h1, hipStream_t s) {
  if (fp64) face_p<double>(p, states, f0, f1, h0, h1, s);
  else face_p<float>(p, states, f0, f1, h0, h1, s);
  return hipGetLastError();
}

hipError_t launch_moments(const StepParams& p, bool fp64, bool with_h, double* out,
                          unsigned long long* bad, hipStream_t s) {
  const unsigned nb = static_cast<unsigned>((p.range + kBlock - 1) / kBlock);
  if (fp64) moments_p<double>(p, with_h, nb, out, bad, s);
  else moments_p<float>(p, with_h, nb, out, bad, s);
  return hipGetLastError();
}

hipError_t launch_sums(const StepParams& p, bool fp64, bool with_h, double* partial, int nblocks,
                       double* out5, hipStream_t s) {
  if (fp64) sums_p<double>(p, with_h, nblocks, partial, s);
  else sums_p<float>(p, with_h, nblocks, partial, s);
  hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(kBlock), 0, s, partial, nblocks, out5);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed device scratch for the allocation-free field read-back
// (rlb_moments_noalloc): the staging buffer of k_moments' five FP64 fields
// for up to kScratchCells cells.  Every GPU holds its own copy for the life
// of the process.  In host code the array's name is only a stand-in for the
// symbol: kernels receive the device address that hipGetSymbolAddress
// returns, looked up once per device with that device current.
// ---------------------------------------------------------------------------
namespace {
static __device__ __align__(256) double scratch[kScratchFields * kScratchCells];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace rlb
