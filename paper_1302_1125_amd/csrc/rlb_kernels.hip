// rlb_kernels.hip -- gfx950 kernels of the ultra-relativistic lattice
// Boltzmann update of Mohseni, Mendoza, Succi and Herrmann (arXiv:1302.1125).
//
// Data layout (HBM): populations structure-of-arrays, f[i][cell] and
// h[i][cell], cell = x + nx (y + ny z), two copies (ping-pong); the fields of
// the previous step hist[k][cell] (FP64, k = eps, ux, uy, uz, n) are read and
// rewritten in place by the cell that owns them.
//
// One fused kernel per step: each thread owns one cell, forms its moments
// (FP64 accumulation), recovers the fields in FP64, builds the equilibrium
// coefficients in FP64, and for every population evaluates the minmod
// limited flux divergence, the bulk Laplacian and the implicit collision in
// the storage precision.  Workgroups cover 2D tiles of cells; the tile index
// is remapped so that each XCD (own L2) walks a contiguous range of tiles.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
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

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// XCD-aware tile index: workgroup b runs on XCD b % 8; give XCD x the
// contiguous tile range [x * per, (x + 1) * per).
__device__ __forceinline__ long long xcd_tile(unsigned b, long long per) {
  return static_cast<long long>(b % kXcds) * per + static_cast<long long>(b / kXcds);
}

// Equilibrium as a linear form in 10 coefficients:
// bracket_i(K) = K0 + sum_a e^a K[1+a] + sum_a (e^a)^2 K[4+a]
//              + e^x e^y K7 + e^x e^z K8 + e^y e^z K9.
template <int I>
__device__ __forceinline__ double bracket(const double* K) {
  constexpr Vel e = vel(I);
  double s = K[0];
  if constexpr (e.x != 0) s += double(e.x) * K[1] + double(e.x * e.x) * K[4];
  if constexpr (e.y != 0) s += double(e.y) * K[2] + double(e.y * e.y) * K[5];
  if constexpr (e.z != 0) s += double(e.z) * K[3] + double(e.z * e.z) * K[6];
  if constexpr (e.x * e.y != 0) s += double(e.x * e.y) * K[7];
  if constexpr (e.x * e.z != 0) s += double(e.x * e.z) * K[8];
  if constexpr (e.y * e.z != 0) s += double(e.y * e.z) * K[9];
  return s;
}

// f^eq_i = w_i bracket_i(K) with (moment-exact reading of Eq. (29), fixed by
// Eq. (36) and eps = 3p): A = nu^2 eps / 27, G = A gamma^2,
// K0 = A - 16/15 G |u|^2, K_a = 4 sqrt(13/27) G u^a, K_aa = 52/15 G (u^a)^2,
// K_ab = 13 G u^a u^b.
__device__ __forceinline__ void feq_coeffs(const StepParams& P, double eps, double ux, double uy,
                                           double uz, double g2, double* K) {
  const double A = P.a_scale * eps;
  const double G = A * g2;
  const double u2 = ux * ux + uy * uy + uz * uz;
  K[0] = A - (16.0 / 15.0) * G * u2;
  const double c1 = P.k1 * G;  // 4 sqrt(13/27) G
  K[1] = c1 * ux;
  K[2] = c1 * uy;
  K[3] = c1 * uz;
  const double c2 = (52.0 / 15.0) * G;
  K[4] = c2 * ux * ux;
  K[5] = c2 * uy * uy;
  K[6] = c2 * uz * uz;
  const double c3 = 13.0 * G;
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

__device__ __forceinline__ double wprime(const StepParams& P, int i) {
  return i == 0 ? P.wp0 : (i <= 6 ? P.wp1 : P.wp2);
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
template <bool WH>
__device__ __forceinline__ double tau_of(const StepParams& P, const Fields& F) {
  if (P.tau_mode == 0) return P.tau;
  const double p = F.eps / 3.0;
  if constexpr (WH) {
    const double T = p / F.n;
    const double lam = F.n / (T * T * T);
    const double s = F.n * (4.0 - log(lam));
    return 0.5 + P.nu2_etas * s / (F.eps + p);
  } else {
    return 0.5 + P.nu2_etas / sqrt(sqrt(p));
  }
}

// minmod(X, Y), Eq. (53): the argument of smaller magnitude if both have the
// same sign, else 0.
template <typename T>
__device__ __forceinline__ T mmod(T a, T b) {
  const T lo = fmin(a, b), hi = fmax(a, b);
  return (a > T(0) && b > T(0)) ? lo : ((a < T(0) && b < T(0)) ? hi : T(0));
}

// Difference of limited interface values between x + 1/2 and x - 1/2 for a
// positive streaming speed (left states): values at x-2, x-1, x, x+1.
template <typename T>
__device__ __forceinline__ T dflux_pos(T m2, T m1, T c0, T p1) {
  const T g0 = c0 + T(0.5) * mmod(p1 - c0, c0 - m1);
  const T gm = m1 + T(0.5) * mmod(c0 - m1, m1 - m2);
  return g0 - gm;
}

// Same for a negative speed (right states): values at x-1, x, x+1, x+2.
template <typename T>
__device__ __forceinline__ T dflux_neg(T m1, T c0, T p1, T p2) {
  const T q0 = p1 - T(0.5) * mmod(p2 - p1, p1 - c0);
  const T qm = c0 - T(0.5) * mmod(p1 - c0, c0 - m1);
  return q0 - qm;
}

// Cell coordinates and neighbour addressing with boundary conditions folded
// into the index (periodic wrap, outflow clamp) or the value (fixed face).
template <typename T>
struct Cell {
  int x[3];
  int n[3];
  long long stride[3];
  long long c;
  bool inner;  // every active axis has >= 2 cells on both sides

  __device__ __forceinline__ T load(const T* __restrict__ arr, const StepParams& P, int pop,
                                    int dist, int a, int k) const {
    if (inner) return arr[c + k * stride[a]];
    int q = x[a] + k;
    if (q < 0) {
      const int b = P.bc[2 * a];
      if (b == kBcFixed) return static_cast<T>(P.face_eq[((2 * a) * 2 + dist) * Q + pop]);
      q = (b == kBcPeriodic) ? q + n[a] : 0;
    } else if (q >= n[a]) {
      const int b = P.bc[2 * a + 1];
      if (b == kBcFixed) return static_cast<T>(P.face_eq[((2 * a + 1) * 2 + dist) * Q + pop]);
      q = (b == kBcPeriodic) ? q - n[a] : n[a] - 1;
    }
    return arr[c + static_cast<long long>(q - x[a]) * stride[a]];
  }
};

template <int ACT>
__device__ __forceinline__ bool axis_on(int a) {
  return (ACT >> a) & 1;
}

// delta t * (flux divergence) and the Laplacian of population I at the cell.
template <typename T, int ACT, int I, bool LAP>
__device__ __forceinline__ void stream_terms(const T* __restrict__ arr_i, const StepParams& P,
                                             const Cell<T>& C, int dist, T c0, T dtv, T& dD,
                                             T& lap) {
  dD = T(0);
  lap = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!axis_on<ACT>(a)) continue;
    const int ea = vcomp(I, a);
    if (ea > 0) {
      const T m2 = C.load(arr_i, P, I, dist, a, -2);
      const T m1 = C.load(arr_i, P, I, dist, a, -1);
      const T p1 = C.load(arr_i, P, I, dist, a, +1);
      dD += (dtv * T(ea)) * dflux_pos(m2, m1, c0, p1);
      if (LAP) lap += (m1 + p1) - T(2) * c0;
    } else if (ea < 0) {
      const T m1 = C.load(arr_i, P, I, dist, a, -1);
      const T p1 = C.load(arr_i, P, I, dist, a, +1);
      const T p2 = C.load(arr_i, P, I, dist, a, +2);
      dD += (dtv * T(ea)) * dflux_neg(m1, c0, p1, p2);
      if (LAP) lap += (m1 + p1) - T(2) * c0;
    } else if (LAP) {
      const T m1 = C.load(arr_i, P, I, dist, a, -1);
      const T p1 = C.load(arr_i, P, I, dist, a, +1);
      lap += (m1 + p1) - T(2) * c0;
    }
  }
}

template <typename T>
__device__ __forceinline__ bool cell_of(const StepParams& P, Cell<T>& C) {
  const long long tile = xcd_tile(blockIdx.x, P.tiles_per_xcd);
  if (tile >= P.ntiles) return false;
  const int tx = static_cast<int>(tile % P.ntx);
  const long long r1 = tile / P.ntx;
  const int ty = static_cast<int>(r1 % P.nty);
  const int z = static_cast<int>(r1 / P.nty);
  const int x = tx * P.tile_x + static_cast<int>(threadIdx.x) % P.tile_x;
  const int y = ty * P.tile_y + static_cast<int>(threadIdx.x) / P.tile_x;
  if (x >= P.nx || y >= P.ny) return false;
  C.x[0] = x;
  C.x[1] = y;
  C.x[2] = z;
  C.n[0] = P.nx;
  C.n[1] = P.ny;
  C.n[2] = P.nz;
  C.stride[0] = 1;
  C.stride[1] = P.nx;
  C.stride[2] = static_cast<long long>(P.nx) * P.ny;
  C.c = x + static_cast<long long>(P.nx) * (y + static_cast<long long>(P.ny) * z);
  bool in = true;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (C.n[a] > 1) in = in && C.x[a] >= 2 && C.x[a] < C.n[a] - 2;
  C.inner = in;
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

// Guard (off unless P.guard): projected fields of new moments and the blend
// factors for f and h; returns true if either factor is below 1.
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

template <typename T, bool WH>
__device__ __forceinline__ void moments_of(const T* v_f, const T* v_h, const StepParams& P,
                                           double& E, double& Mx, double& My, double& Mz,
                                           double& N0) {
  double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0, sh = 0.0;
  static_for<0, Q>([&](auto I) {
    constexpr Vel e = vel(I);
    const double v = static_cast<double>(v_f[I]);
    s0 += v;
    if constexpr (e.x != 0) sx += double(e.x) * v;
    if constexpr (e.y != 0) sy += double(e.y) * v;
    if constexpr (e.z != 0) sz += double(e.z) * v;
    if constexpr (WH) sh += static_cast<double>(v_h[I]);
  });
  E = P.r * P.r * s0;
  Mx = P.rca * sx;
  My = P.rca * sy;
  Mz = P.rca * sz;
  N0 = P.r * sh;
}

// ---------------------------------------------------------------------------
// Fused step: moments -> FP64 recovery -> equilibria -> limited streaming,
// bulk term and implicit collision (Eq. (57)) -> guard -> store.
// ---------------------------------------------------------------------------
template <typename T, int ACT, bool WH, bool EULER>
__global__ __launch_bounds__(kBlock) void k_step(const StepParams P) {
  Cell<T> C;
  if (!cell_of<T>(P, C)) return;
  const long long N = P.ncell;
  const long long c = C.c;
  const T* __restrict__ fin = static_cast<const T*>(P.f_in);
  const T* __restrict__ hin = static_cast<const T*>(P.h_in);
  T* __restrict__ fout = static_cast<T*>(P.f_out);
  T* __restrict__ hout = static_cast<T*>(P.h_out);

  // Obstacle cells: held at the equilibrium of their prescribed fields.
  if (P.obst != nullptr && P.obst[c] != 0) {
    const double eps = P.hist[c], ux = P.hist[N + c], uy = P.hist[2 * N + c],
                 uz = P.hist[3 * N + c], nn = P.hist[4 * N + c];
    const double g2 = 1.0 / (1.0 - (ux * ux + uy * uy + uz * uz));
    double K[10];
    feq_coeffs(P, eps, ux, uy, uz, g2, K);
    static_for<0, Q>([&](auto I) { fout[I * N + c] = static_cast<T>(weight(I) * bracket<I>(K)); });
    if constexpr (WH) {
      double H[10];
      heq_coeffs(P, nn, ux, uy, uz, sqrt(g2), H);
      static_for<0, Q>(
          [&](auto I) { hout[I * N + c] = static_cast<T>(wprime(P, I) * bracket<I>(H)); });
    }
    return;
  }

  T fc[Q];
  T hc[Q];
  static_for<0, Q>([&](auto I) {
    fc[I] = fin[I * N + c];
    if constexpr (WH) hc[I] = hin[I * N + c];
  });

  const T dtv = static_cast<T>(P.dtv);
  const T kap = static_cast<T>(P.kappa);

  if constexpr (EULER) {
    // Streaming and bulk term without collision, then f := f^eq of the
    // post-streaming moments (Sec. III, inviscid case).
    T fs[Q];
    T hs[Q];
    static_for<0, Q>([&](auto I) {
      T dD, lap;
      stream_terms<T, ACT, I, (I != 0)>(fin + I * N, P, C, 0, fc[I], dtv, dD, lap);
      fs[I] = fc[I] - dD + kap * lap;
      if constexpr (WH) {
        T dH, lh;
        stream_terms<T, ACT, I, false>(hin + I * N, P, C, 1, hc[I], dtv, dH, lh);
        hs[I] = hc[I] - dH;
      }
    });
    double E, Mx, My, Mz, N0;
    moments_of<T, WH>(fs, hs, P, E, Mx, My, Mz, N0);
    Fields F;
    bool ok;
    bool fired = false;
    if (P.guard) {
      double thf, thh;
      fired = guard_eval<WH>(P, E, Mx, My, Mz, N0, thf, thh, F);
      ok = true;
      if (!fired) ok = recover<WH>(E, Mx, My, Mz, N0, F);
    } else {
      ok = recover<WH>(E, Mx, My, Mz, N0, F);
    }
    if (P.guard) count_events(P.guard_count, fired);
    if (!ok) atomicMin(P.bad_step, static_cast<unsigned long long>(P.step_index));
    double K[10];
    feq_coeffs(P, F.eps, F.ux, F.uy, F.uz, F.g2, K);
    static_for<0, Q>([&](auto I) { fout[I * N + c] = static_cast<T>(weight(I) * bracket<I>(K)); });
    if constexpr (WH) {
      double H[10];
      heq_coeffs(P, F.n, F.ux, F.uy, F.uz, F.gam, H);
      static_for<0, Q>(
          [&](auto I) { hout[I * N + c] = static_cast<T>(wprime(P, I) * bracket<I>(H)); });
    }
    return;
  } else {
    // 1-2: moments and fields at time t.
    double E, Mx, My, Mz, N0;
    moments_of<T, WH>(fc, hc, P, E, Mx, My, Mz, N0);
    Fields F;
    const bool ok = recover<WH>(E, Mx, My, Mz, N0, F);
    if (!ok) atomicMin(P.bad_step, static_cast<unsigned long long>(P.step_index));

    // 3: equilibrium source 2 f^eq(t) - f^eq(t - dt) as one coefficient set.
    const double pe = P.hist[c], pux = P.hist[N + c], puy = P.hist[2 * N + c],
                 puz = P.hist[3 * N + c], pn = P.hist[4 * N + c];
    const double pg2 = 1.0 / (1.0 - (pux * pux + puy * puy + puz * puz));
    double K[10], Kp[10];
    feq_coeffs(P, F.eps, F.ux, F.uy, F.uz, F.g2, K);
    feq_coeffs(P, pe, pux, puy, puz, pg2, Kp);
#pragma unroll
    for (int k = 0; k < 10; ++k) K[k] = 2.0 * K[k] - Kp[k];
    double H[10];
    if constexpr (WH) {
      double Hp[10];
      heq_coeffs(P, F.n, F.ux, F.uy, F.uz, F.gam, H);
      heq_coeffs(P, pn, pux, puy, puz, sqrt(pg2), Hp);
#pragma unroll
      for (int k = 0; k < 10; ++k) H[k] = 2.0 * H[k] - Hp[k];
    }
    const double omega = P.omega_c / tau_of<WH>(P, F);
    const double inv1p = 1.0 / (1.0 + omega);
    const T tinv = static_cast<T>(inv1p);

    // 4-5: limited streaming, bulk term (f only, lambda_0 = 0), implicit
    // collision, Eq. (57).
    T fn[Q];
    T hn[Q];
    static_for<0, Q>([&](auto I) {
      T dD, lap;
      stream_terms<T, ACT, I, (I != 0)>(fin + I * N, P, C, 0, fc[I], dtv, dD, lap);
      const T src = static_cast<T>(omega * (weight(I) * bracket<I>(K)));
      fn[I] = ((fc[I] - dD) + (src + kap * lap)) * tinv;
      if constexpr (WH) {
        T dH, lh;
        stream_terms<T, ACT, I, false>(hin + I * N, P, C, 1, hc[I], dtv, dH, lh);
        const T hsrc = static_cast<T>(omega * (wprime(P, I) * bracket<I>(H)));
        hn[I] = ((hc[I] - dH) + hsrc) * tinv;
      }
    });

    // Guard: blend towards the equilibrium of the projected new moments.
    if (P.guard) {
      double E2, Mx2, My2, Mz2, N02;
      moments_of<T, WH>(fn, hn, P, E2, Mx2, My2, Mz2, N02);
      double thf, thh;
      Fields G;
      const bool fired = guard_eval<WH>(P, E2, Mx2, My2, Mz2, N02, thf, thh, G);
      if (fired) {
        double Kg[10];
        feq_coeffs(P, G.eps, G.ux, G.uy, G.uz, G.g2, Kg);
        static_for<0, Q>([&](auto I) {
          const double ge = weight(I) * bracket<I>(Kg);
          fn[I] = static_cast<T>(ge + thf * (static_cast<double>(fn[I]) - ge));
        });
        if constexpr (WH) {
          double Hg[10];
          heq_coeffs(P, G.n, G.ux, G.uy, G.uz, G.gam, Hg);
          static_for<0, Q>([&](auto I) {
            const double ge = wprime(P, I) * bracket<I>(Hg);
            hn[I] = static_cast<T>(ge + thh * (static_cast<double>(hn[I]) - ge));
          });
        }
      }
      count_events(P.guard_count, fired);
    }

    static_for<0, Q>([&](auto I) {
      fout[I * N + c] = fn[I];
      if constexpr (WH) hout[I * N + c] = hn[I];
    });
    P.hist[c] = F.eps;
    P.hist[N + c] = F.ux;
    P.hist[2 * N + c] = F.uy;
    P.hist[3 * N + c] = F.uz;
    P.hist[4 * N + c] = F.n;
  }
}

// f := f^eq(fields), h := h^eq(fields) from the fields held in hist; without
// density the lattice equilibrium density (eps/3)^(3/4) is written to hist.
template <typename T, bool WH>
__global__ __launch_bounds__(kBlock) void k_init(const StepParams P) {
  const long long c = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (c >= P.ncell) return;
  const long long N = P.ncell;
  T* __restrict__ f = static_cast<T*>(P.f_out);
  T* __restrict__ h = static_cast<T*>(P.h_out);
  const double eps = P.hist[c], ux = P.hist[N + c], uy = P.hist[2 * N + c],
               uz = P.hist[3 * N + c];
  const double g2 = 1.0 / (1.0 - (ux * ux + uy * uy + uz * uz));
  double K[10];
  feq_coeffs(P, eps, ux, uy, uz, g2, K);
  static_for<0, Q>([&](auto I) { f[I * N + c] = static_cast<T>(weight(I) * bracket<I>(K)); });
  if constexpr (WH) {
    double H[10];
    heq_coeffs(P, P.hist[4 * N + c], ux, uy, uz, sqrt(g2), H);
    static_for<0, Q>([&](auto I) { h[I * N + c] = static_cast<T>(wprime(P, I) * bracket<I>(H)); });
  } else {
    P.hist[4 * N + c] = pow(eps / 3.0, 0.75);
  }
}

// Equilibria of the six face states: face_eq[s][0][i] = f^eq, [s][1][i] = h^eq.
__global__ void k_face_eq(const StepParams P, const double* states, double* out) {
  const int s = threadIdx.x;
  if (s >= 6) return;
  const double* q = states + 5 * s;
  const double g2 = 1.0 / (1.0 - (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]));
  double K[10], H[10];
  feq_coeffs(P, q[0], q[1], q[2], q[3], g2, K);
  heq_coeffs(P, q[4], q[1], q[2], q[3], sqrt(g2), H);
  static_for<0, Q>([&](auto I) {
    out[(s * 2 + 0) * Q + I] = weight(I) * bracket<I>(K);
    out[(s * 2 + 1) * Q + I] = wprime(P, I) * bracket<I>(H);
  });
}

// Fields of the current populations (FP64 recovery); NaN where inadmissible.
template <typename T, bool WH>
__global__ __launch_bounds__(kBlock) void k_moments(const StepParams P, double* out,
                                                     unsigned long long* bad) {
  const long long c = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  if (c >= P.ncell) return;
  const long long N = P.ncell;
  const T* __restrict__ f = static_cast<const T*>(P.f_in);
  const T* __restrict__ h = static_cast<const T*>(P.h_in);
  T fc[Q], hc[Q];
  static_for<0, Q>([&](auto I) {
    fc[I] = f[I * N + c];
    if constexpr (WH) hc[I] = h[I * N + c];
  });
  double E, Mx, My, Mz, N0;
  moments_of<T, WH>(fc, hc, P, E, Mx, My, Mz, N0);
  Fields F;
  const bool ok = recover<WH>(E, Mx, My, Mz, N0, F);
  const bool obst = P.obst != nullptr && P.obst[c] != 0;
  if (!ok && !obst) atomicMin(bad, 0ull);
  out[c] = ok ? F.eps : NAN;
  out[N + c] = ok ? F.ux : NAN;
  out[2 * N + c] = ok ? F.uy : NAN;
  out[3 * N + c] = ok ? F.uz : NAN;
  out[4 * N + c] = ok ? F.n : NAN;
}

// Deterministic domain sums of T^{00}, T^{0a}, N^0: per-block tree sums into
// partial[block][5], then one block adds the partials in index order.
template <typename T, bool WH>
__global__ __launch_bounds__(kBlock) void k_sums_partial(const StepParams P, double* partial) {
  __shared__ double red[5][kBlock];
  const long long c = static_cast<long long>(blockIdx.x) * kBlock + threadIdx.x;
  double v[5] = {0, 0, 0, 0, 0};
  if (c < P.ncell) {
    const long long N = P.ncell;
    const T* __restrict__ f = static_cast<const T*>(P.f_in);
    const T* __restrict__ h = static_cast<const T*>(P.h_in);
    T fc[Q], hc[Q];
    static_for<0, Q>([&](auto I) {
      fc[I] = f[I * N + c];
      if constexpr (WH) hc[I] = h[I * N + c];
    });
    moments_of<T, WH>(fc, hc, P, v[0], v[1], v[2], v[3], v[4]);
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
  const long long nblk = p.tiles_per_xcd * kXcds;
  hipLaunchKernelGGL((k_step<T, ACT, WH, EU>), dim3(static_cast<unsigned>(nblk)), dim3(kBlock), 0,
                     s, p);
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

}  // namespace

hipError_t launch_step(const StepParams& p, bool fp64, int act_mask, bool with_h, bool euler,
                       hipStream_t s) {
  return fp64 ? launch_step_p<double>(p, act_mask, with_h, euler, s)
              : launch_step_p<float>(p, act_mask, with_h, euler, s);
}

hipError_t launch_init(const StepParams& p, bool fp64, bool with_h, hipStream_t s) {
  const unsigned nb = static_cast<unsigned>((p.ncell + kBlock - 1) / kBlock);
  if (fp64) {
    if (with_h) hipLaunchKernelGGL((k_init<double, true>), dim3(nb), dim3(kBlock), 0, s, p);
    else hipLaunchKernelGGL((k_init<double, false>), dim3(nb), dim3(kBlock), 0, s, p);
  } else {
    if (with_h) hipLaunchKernelGGL((k_init<float, true>), dim3(nb), dim3(kBlock), 0, s, p);
    else hipLaunchKernelGGL((k_init<float, false>), dim3(nb), dim3(kBlock), 0, s, p);
  }
  return hipGetLastError();
}

hipError_t launch_face_eq(const StepParams& p, const double* states, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_face_eq, dim3(1), dim3(64), 0, s, p, states, out);
  return hipGetLastError();
}

hipError_t launch_moments(const StepParams& p, bool fp64, bool with_h, double* out,
                          unsigned long long* bad, hipStream_t s) {
  const unsigned nb = static_cast<unsigned>((p.ncell + kBlock - 1) / kBlock);
  if (fp64) {
    if (with_h) hipLaunchKernelGGL((k_moments<double, true>), dim3(nb), dim3(kBlock), 0, s, p, out, bad);
    else hipLaunchKernelGGL((k_moments<double, false>), dim3(nb), dim3(kBlock), 0, s, p, out, bad);
  } else {
    if (with_h) hipLaunchKernelGGL((k_moments<float, true>), dim3(nb), dim3(kBlock), 0, s, p, out, bad);
    else hipLaunchKernelGGL((k_moments<float, false>), dim3(nb), dim3(kBlock), 0, s, p, out, bad);
  }
  return hipGetLastError();
}

hipError_t launch_sums(const StepParams& p, bool fp64, bool with_h, double* partial, int nblocks,
                       double* out5, hipStream_t s) {
  if (fp64) {
    if (with_h) hipLaunchKernelGGL((k_sums_partial<double, true>), dim3(nblocks), dim3(kBlock), 0, s, p, partial);
    else hipLaunchKernelGGL((k_sums_partial<double, false>), dim3(nblocks), dim3(kBlock), 0, s, p, partial);
  } else {
    if (with_h) hipLaunchKernelGGL((k_sums_partial<float, true>), dim3(nblocks), dim3(kBlock), 0, s, p, partial);
    else hipLaunchKernelGGL((k_sums_partial<float, false>), dim3(nblocks), dim3(kBlock), 0, s, p, partial);
  }
  hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(kBlock), 0, s, partial, nblocks, out5);
  return hipGetLastError();
}

}  // namespace rlb
