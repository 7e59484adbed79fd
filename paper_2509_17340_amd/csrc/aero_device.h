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

// Bytes carried in a kernel argument (descriptors written without a host staging
// buffer).  16-byte aligned, so that records read in place from the argument are
// aligned.
constexpr int kPutBytes = 2048;
struct alignas(16) PutBlob {
  uint32_t n;
  uint32_t pad;
  unsigned char b[kPutBytes];
};

// A launch that carries the call's descriptors in `blob` (blob.n > 0) reads them
// from the argument and has its block 0 write them to the workspace at `dst` for the
// kernels that follow (no separate upload launch).
__device__ inline void put_blob(const PutBlob& blob, unsigned char* dst) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(blob.b);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  for (uint32_t i = threadIdx.x; i < blob.n / 4; i += blockDim.x) d[i] = src[i];
}

// ---------------------------------------------------------------------------
// The same RK4 step spread over the four lanes of a quad (one rollout per quad).
// Lane c (0..3) holds the quaternion component q_c (w, x, y, z) and, for c < 3, the
// position and velocity components p_c and v_c; a lane computes the derivatives of
// its own components only.  The quaternion is the one state the others depend on
// (q' = Omega(omega) q / 2, v' from R(q) e3, p' = v), so after each stage the four
// lanes exchange their components with DPP moves inside the quad.  The per-component
// arithmetic is that of xdot_held and rk4 above.
// ---------------------------------------------------------------------------
constexpr int quad_perm(int a, int b, int c, int d) { return a | b << 2 | c << 4 | d << 6; }

// Lane src_c of the quad's value, for lane c of every quad (Ctrl a quad permutation).
template <int Ctrl>
__device__ __forceinline__ double quad_move(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  // every lane of a quad permutation has a source, so no old value is needed
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, Ctrl, 0xf, 0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), Ctrl, 0xf, 0xf,
                                                         true);
  return __builtin_bit_cast(double, (uint64_t)hi << 32 | lo);
}

__device__ __forceinline__ void quad_gather(double own, double all[4]) {
  all[0] = quad_move<quad_perm(0, 0, 0, 0)>(own);
  all[1] = quad_move<quad_perm(1, 1, 1, 1)>(own);
  all[2] = quad_move<quad_perm(2, 2, 2, 2)>(own);
  all[3] = quad_move<quad_perm(3, 3, 3, 3)>(own);
}

__device__ __forceinline__ double flip_sign(double x, uint32_t sign_hi) {
  uint64_t b = __builtin_bit_cast(uint64_t, x);
  b ^= (uint64_t)sign_hi << 32;
  return __builtin_bit_cast(double, b);
}

// Lane constants of the quad layout.
struct QuadLane {
  int c;                   // component / control channel of this lane
  uint32_t sgn1, sgn2, sgn3;  // sign bits of this lane's row of Omega (columns x, y, z)
};

__device__ __forceinline__ QuadLane quad_lane(int lane) {
  QuadLane L;
  L.c = lane & 3;
  // Row c of Omega(omega/2) over (w, x, y, z):
  //   c=0 ( 0, -hx, -hy, -hz)   c=1 (hx,  0,  hz, -hy)
  //   c=2 (hy, -hz,  0,  hx)    c=3 (hz,  hy, -hx,  0)
  // column 0 is this lane's own held half rate (0 on lane 0), and columns 1..3 are
  // the held half rates of lanes (1,0,3,2), (2,3,0,1), (3,2,1,0) with these signs.
  const uint32_t m = 0x80000000u;
  L.sgn1 = (L.c == 0 || L.c == 2) ? m : 0u;
  L.sgn2 = (L.c == 0 || L.c == 3) ? m : 0u;
  L.sgn3 = (L.c == 0 || L.c == 1) ? m : 0u;
  return L;
}

// The held control of one step in quad form: this lane's row of Omega(omega)/2 and the
// mass-specific thrust (from lane 0's channel).
struct QuadControl {
  double row[4];
  double am, am2;
};

__device__ __forceinline__ QuadControl quad_control(double u_c, const QuadLane& L, const Dyn& d) {
  QuadControl q;
  const double h = L.c == 0 ? 0.0 : 0.5 * u_c;  // omega_c / 2 on lanes 1..3
  q.am = quad_move<quad_perm(0, 0, 0, 0)>(u_c * d.inv_m);
  q.am2 = 2.0 * q.am;
  q.row[0] = h;
  q.row[1] = flip_sign(quad_move<quad_perm(1, 0, 3, 2)>(h), L.sgn1);
  q.row[2] = flip_sign(quad_move<quad_perm(2, 3, 0, 1)>(h), L.sgn2);
  q.row[3] = flip_sign(quad_move<quad_perm(3, 2, 1, 0)>(h), L.sgn3);
  return q;
}

// Derivatives of this lane's quaternion and velocity components at the stage whose
// quaternion (all four components) is qa.
__device__ __forceinline__ void quad_xdot(const double qa[4], const QuadControl& u,
                                          const QuadLane& L, const Dyn& d, double& dq,
                                          double& dv) {
  const double qw = qa[0], qx = qa[1], qy = qa[2], qz = qa[3];
  double r = u.row[0] * qw;
  r = fma(u.row[1], qx, r);
  r = fma(u.row[2], qy, r);
  dq = fma(u.row[3], qz, r);
  const double e0 = qx * qz + qw * qy;
  const double e1 = qy * qz - qw * qx;
  const double e2 = qx * qx + qy * qy;
  const double vxy = u.am2 * (L.c == 0 ? e0 : e1);
  const double vz = u.am * (1.0 - 2.0 * e2) - d.g;
  dv = L.c == 2 ? vz : vxy;
}

// One RK4 step of the quad's rollout with the control held, then the quaternion
// renormalisation.  p, v, q are this lane's components (p, v unused on lane 3); qa
// holds all four quaternion components on entry and on return.
__device__ __forceinline__ void quad_rk4(double& p, double& v, double& q, double qa[4],
                                         const QuadControl& u, const QuadLane& L, double dt,
                                         const Dyn& d) {
  double kq1, kv1, kq2, kv2, kq3, kv3, kq4, kv4, ya[4];
  quad_xdot(qa, u, L, d, kq1, kv1);
  const double kp1 = v;
  const double kp2 = v + 0.5 * dt * kv1;
  quad_gather(q + 0.5 * dt * kq1, ya);
  quad_xdot(ya, u, L, d, kq2, kv2);
  const double kp3 = v + 0.5 * dt * kv2;
  quad_gather(q + 0.5 * dt * kq2, ya);
  quad_xdot(ya, u, L, d, kq3, kv3);
  const double kp4 = v + dt * kv3;
  quad_gather(q + dt * kq3, ya);
  quad_xdot(ya, u, L, d, kq4, kv4);
  const double h6 = dt / 6.0;
  p = p + h6 * (kp1 + 2.0 * kp2 + 2.0 * kp3 + kp4);
  v = v + h6 * (kv1 + 2.0 * kv2 + 2.0 * kv3 + kv4);
  q = q + h6 * (kq1 + 2.0 * kq2 + 2.0 * kq3 + kq4);
  quad_gather(q, qa);
  const double inv = rsqrt_refined(qa[0] * qa[0] + qa[1] * qa[1] + qa[2] * qa[2] + qa[3] * qa[3]);
  q *= inv;
#pragma unroll
  for (int i = 0; i < 4; ++i) qa[i] *= inv;
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

// ---------------------------------------------------------------------------
// Items of the first distance pass: (global query block, sub-tile | order << 31).
// ---------------------------------------------------------------------------

// The two-pass set owning global query block gqb; `c` caches the last lookup
// (items of one block, and mostly of one set, come in runs).
struct SetCache {
  int s;
  int64_t lo, hi;
};
__device__ inline int set_of(const QuerySet* __restrict__ sets, int n_sets, int64_t gqb,
                             SetCache& c) {
  if (gqb >= c.lo && gqb < c.hi) return c.s;
  c.s = find_owner(sets, n_sets, gqb, [](const QuerySet& q) { return q.qb_base; });
  c.lo = sets[c.s].qb_base;
  c.hi = c.lo + sets[c.s].n_qblocks;
  return c.s;
}

// This thread's point of an item's sub-tile (thread i takes point i), from the raw
// cloud or the sorted records; *cnt receives the sub-tile's point count (0 for an
// item that names no sub-tile of the set, which is then skipped).  Addresses are
// always inside the cloud.
__device__ inline void item_point(const QuerySet& S, unsigned ys, float& x, float& y, float& z,
                                  int32_t& idx, bool& in, int& cnt) {
  const int64_t n = S.n_points;
  if (n <= 0) {  // not a set with a cloud: nothing to read
    x = y = z = 0.0f;
    idx = -1;
    in = false;
    cnt = 0;
    return;
  }
  const int64_t g0 = (int64_t)(ys & 0x7fffffffu) * kSubPts;
  const bool srt = (ys >> 31) != 0;
  cnt = (g0 < n && (!srt || S.scloud)) ? (int)min<int64_t>(kSubPts, n - g0) : 0;
  in = (int)threadIdx.x < cnt;
  const int64_t g = in ? g0 + threadIdx.x : 0;
  if (srt && S.scloud) {
    const float4 r = S.scloud[g];
    x = r.x;
    y = r.y;
    z = r.z;
    idx = __float_as_int(r.w);
  } else {
    x = S.cloud[3 * g];
    y = S.cloud[3 * g + 1];
    z = S.cloud[3 * g + 2];
    idx = (int32_t)g;
  }
}

// Whether global block gqb is a block of set S.
__device__ inline bool block_of(const QuerySet& S, int64_t gqb) {
  return gqb >= S.qb_base && gqb < S.qb_base + S.n_qblocks;
}

// Mark item i as hit when some lane of the wave saw a query under its block's bound.
__device__ inline void mark_hit(bool hit, unsigned char* hitf, int64_t i) {
  const unsigned long long hb = __ballot(hit);
  if (hb && (int)(threadIdx.x & 63) == __ffsll((long long)hb) - 1) hitf[i] = 1;
}

// Bounding boxes of cloud tile `t` (kTilePts consecutive points), of its kTileSplit
// sub-tiles and of their kGroupsPerSub groups of 32 points (gbox, when given), from
// the raw points ([n][3], c4 == nullptr) or the sorted records (c4).  One workgroup of
// kBlock threads; sub-tile j's points are taken one per thread.  Sub-tiles past the
// end of the cloud are not written; a group without points gets an empty box.
__device__ inline void tile_boxes(const float* __restrict__ c3, const float4* __restrict__ c4,
                                  int64_t n_points, int64_t t, float* __restrict__ tbox,
                                  float* __restrict__ sbox, float* __restrict__ gbox) {
  static_assert(kSubPts == kBlock, "one point per thread");
  constexpr int kW = kBlock / 64;
  __shared__ float red[kTileSplit][6][kW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kTileSplit; ++j) {
    const int64_t g = t * kTilePts + j * kSubPts + threadIdx.x;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (g < n_points) {
      float p[3];
      if (c4) {
        const float4 r = c4[g];
        p[0] = r.x;
        p[1] = r.y;
        p[2] = r.z;
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) p[a] = c3[3 * g + a];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) lo[a] = hi[a] = p[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // the 32-point group of each half wave first, then the whole wave
#pragma unroll
      for (int o = 1; o < 32; o <<= 1) {
        lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
        hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
      }
      const int64_t sub = t * kTileSplit + j;
      if (gbox && (lane & 31) == 0 && sub * kSubPts < n_points) {
        float* gb = gbox + 6 * (sub * kGroupsPerSub + 2 * w + (lane >> 5));
        gb[a] = lo[a];
        gb[3 + a] = hi[a];
      }
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], 32, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], 32, 64));
      if (lane == 0) {
        red[j][a][w] = lo[a];
        red[j][3 + a][w] = hi[a];
      }
    }
  }
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid < kTileSplit * 6) {  // sub-tile boxes
    const int j = tid / 6, a = tid % 6;
    float v = red[j][a][0];
    for (int k = 1; k < kW; ++k) v = a < 3 ? fminf(v, red[j][a][k]) : fmaxf(v, red[j][a][k]);
    const int64_t sub = t * kTileSplit + j;
    if (sub * kSubPts < n_points) sbox[6 * sub + a] = v;
  } else if (tid < kTileSplit * 6 + 6) {  // the tile's box
    const int a = tid - kTileSplit * 6;
    float v = red[0][a][0];
    for (int j = 0; j < kTileSplit; ++j)
      for (int k = 0; k < kW; ++k) v = a < 3 ? fminf(v, red[j][a][k]) : fmaxf(v, red[j][a][k]);
    tbox[6 * t + a] = v;
  }
}

}  // namespace aero
