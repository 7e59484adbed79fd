// Device building blocks of the planning step (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aero_internal.h"

namespace aero {

// Pointers known to address device (global) memory.  A pointer read out of a
// descriptor is generic to the compiler, and generic (flat) accesses count on both
// the vector-memory and the LDS/scalar counters, so a wait for one such load also
// waits for every flat store in flight; global accesses keep loads and stores on
// the vector-memory counter only, in order.
#define AERO_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ AERO_GLOBAL T* global_ptr(T* p) {
  return (AERO_GLOBAL T*)p;
}

// ---------------------------------------------------------------------------
// Counter-based noise: Philox4x32 with 10 rounds (Salmon et al., SC'11).  Each
// round multiplies counter words 0 and 2 by the two round constants, folds the
// high halves into words 1 and 3 with the key, and the key advances by the two
// Weyl increments between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo0 = 0xD2511F53u * c[0];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Box-Muller (1958) in binary64: u1 = (a + 1) 2^-32 in (0, 1], u2 = b 2^-32.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& n0, double& n1) {
  const double u1 = ((double)a + 1.0) * 0x1p-32;
  const double u2 = (double)b * 0x1p-32;
  const double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  n0 = r * c;
  n1 = r * s;
}

// Four standard normals for (sample k, step t, instance m) of a problem.
__device__ __forceinline__ void normals4(const DevParams& prm, uint32_t problem_id, uint32_t k,
                                         uint32_t t, uint32_t m, double n[4]) {
  uint32_t c[4] = {k, t, m, prm.iter_base};
  philox4x32_10(c, prm.seed_lo, prm.seed_hi ^ problem_id);
  box_muller(c[0], c[1], n[0], n[1]);
  box_muller(c[2], c[3], n[2], n[3]);
}

// ---------------------------------------------------------------------------
// Quadrotor model (Sec. III-A): x = [p, q(w,x,y,z), v], u = (F_t, omega_body).
// ---------------------------------------------------------------------------
struct Dyn {
  double inv_m, g;
};

// Per-step factors of the held control: half the body rates and twice the mass-
// specific thrust (scalings by powers of two, so every product below rounds exactly
// as the unscaled formula would).
struct HeldControl {
  double hwx, hwy, hwz;  // omega / 2
  double am, am2;        // F / m and 2 F / m
};

__device__ __forceinline__ HeldControl held_control(const double* u, const Dyn& d) {
  HeldControl c;
  c.hwx = 0.5 * u[1];
  c.hwy = 0.5 * u[2];
  c.hwz = 0.5 * u[3];
  c.am = u[0] * d.inv_m;
  c.am2 = 2.0 * c.am;
  return c;
}

__device__ __forceinline__ void xdot_held(const double* x, const HeldControl& c, const Dyn& d,
                                          double* dx) {
  const double qw = x[3], qx = x[4], qy = x[5], qz = x[6];
  dx[0] = x[7];
  dx[1] = x[8];
  dx[2] = x[9];
  // q' = 1/2 q (x) (0, omega)
  dx[3] = -qx * c.hwx - qy * c.hwy - qz * c.hwz;
  dx[4] = qw * c.hwx + qy * c.hwz - qz * c.hwy;
  dx[5] = qw * c.hwy - qx * c.hwz + qz * c.hwx;
  dx[6] = qw * c.hwz + qx * c.hwy - qy * c.hwx;
  // v' = (F/m) R(q) e3 + g, R(q) e3 = (2(xz+wy), 2(yz-wx), 1-2(x^2+y^2))
  dx[7] = c.am2 * (qx * qz + qw * qy);
  dx[8] = c.am2 * (qy * qz - qw * qx);
  dx[9] = c.am * (1.0 - 2.0 * (qx * qx + qy * qy)) - d.g;
}

__device__ __forceinline__ void xdot(const double* x, const double* u, const Dyn& d, double* dx) {
  xdot_held(x, held_control(u, d), d, dx);
}

// 1/sqrt(s) for the quaternion renormalisation: the hardware estimate refined by
// two Newton steps, r <- r (3/2 - s r^2 / 2), each of which doubles the number of
// correct bits (within a couple of ulp of the correctly rounded value; s = |q|^2 is
// close to 1 after every step).
__device__ __forceinline__ double rsqrt_refined(double s) {
  double r = __builtin_amdgcn_rsq(s);
  const double hs = 0.5 * s;
  r = r * fma(-hs * r, r, 1.5);
  r = r * fma(-hs * r, r, 1.5);
  return r;
}

// One RK4 step with the control held, then quaternion renormalisation.
__device__ __forceinline__ void rk4(double* x, const double* u, double dt, const Dyn& d) {
  double k1[10], k2[10], k3[10], k4[10], y[10];
  const HeldControl c = held_control(u, d);
  xdot_held(x, c, d, k1);
#pragma unroll
  for (int i = 0; i < 10; ++i) y[i] = x[i] + 0.5 * dt * k1[i];
  xdot_held(y, c, d, k2);
#pragma unroll
  for (int i = 0; i < 10; ++i) y[i] = x[i] + 0.5 * dt * k2[i];
  xdot_held(y, c, d, k3);
#pragma unroll
  for (int i = 0; i < 10; ++i) y[i] = x[i] + dt * k3[i];
  xdot_held(y, c, d, k4);
  const double h6 = dt / 6.0;
#pragma unroll
  for (int i = 0; i < 10; ++i) x[i] = x[i] + h6 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  const double inv = rsqrt_refined(x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6]);
  x[3] *= inv;
  x[4] *= inv;
  x[5] *= inv;
  x[6] *= inv;
}

// R(q) of a unit quaternion, row-major.
__device__ __forceinline__ void rotmat(double w, double x, double y, double z, double R[9]) {
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// |R(q) Rg^T - I|_F with Rg precomputed.
__device__ __forceinline__ double attitude_err(const double* x, const double Rg[9]) {
  double R[9];
  rotmat(x[3], x[4], x[5], x[6], R);
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double e = R[3 * i] * Rg[3 * j] + R[3 * i + 1] * Rg[3 * j + 1] + R[3 * i + 2] * Rg[3 * j + 2];
      if (i == j) e -= 1.0;
      s += e * e;
    }
  return sqrt(s);
}

// Running goal term Q_p |p - pg| + Q_v |v - vg| + Q_q |R Rg^T - I|_F.
__device__ __forceinline__ double goal_term(const double* x, const double pg[3], const double vg[3],
                                            const double Rg[9], const DevParams& prm) {
  const double ex = x[0] - pg[0], ey = x[1] - pg[1], ez = x[2] - pg[2];
  const double fx = x[7] - vg[0], fy = x[8] - vg[1], fz = x[9] - vg[2];
  return prm.Q_p * sqrt(ex * ex + ey * ey + ez * ez) + prm.Q_v * sqrt(fx * fx + fy * fy + fz * fz) +
         prm.Q_q * attitude_err(x, Rg);
}

// Collision penalty phi(d) (Sec. IV-C, collision cost).
__device__ __forceinline__ double collision_phi(double d, const DevParams& prm) {
  if (d < prm.d_min) return prm.C;
  if (d < prm.d_max) return prm.C * exp(-prm.a * (d - prm.d_min));
  return 0.0;
}

// Order-preserving map of floats to unsigned integers (a < b as floats, NaN aside,
// iff ord_bits(a) < ord_bits(b)), for bounds merged with integer atomics.
__device__ __forceinline__ unsigned ord_bits(float f) {
  const unsigned b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// ---------------------------------------------------------------------------
// Wave64 / block reductions with a fixed combination order (deterministic).
// ---------------------------------------------------------------------------
__device__ inline float wave_minf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline float wave_maxf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Locate the record owning flat index i in an array of prefix bases.
template <typename T, typename F>
__device__ __forceinline__ int find_owner(const T* recs, int n, int64_t i, F base_of) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (base_of(recs[mid]) <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Bounding box of sub-tile `bid` (counted over the two-pass sets in box_base order)
// of a cloud: kSubPts consecutive points, one per thread of a kBlock block.  Read
// by pass A's hit records.
__device__ inline void cloud_box_block(const QuerySet* __restrict__ sets, int n_sets, int64_t bid) {
  static_assert(kSubPts == kBlock, "one point per thread");
  __shared__ float red[6][kBlock / 64];
  const int s = find_owner(sets, n_sets, bid, [](const QuerySet& q) { return q.box_base; });
  const QuerySet& S = sets[s];
  const int64_t sub = bid - S.box_base;
  const int64_t g = sub * kSubPts + threadIdx.x;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (g < S.n_points) {
#pragma unroll
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = S.cloud[3 * g + a];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_minf(lo[a]);
    hi[a] = wave_maxf(hi[a]);
    if (lane == 0) {
      red[a][w] = lo[a];
      red[3 + a][w] = hi[a];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    float v = red[a][0];
    for (int k = 1; k < kBlock / 64; ++k) v = a < 3 ? fminf(v, red[a][k]) : fmaxf(v, red[a][k]);
    S.qbox[6 * sub + a] = v;
  }
}

}  // namespace aero
