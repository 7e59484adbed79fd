// Adjoint of L = g * sum_{m,k} S1[m,k] with respect to u_nom and the five
// term weights (built on Sec. III-A eq. (dynamics), the RK4 step of
// eq. (mppi_rollout) and the Stage-I terms of Sec. IV-C).
//
// The derivative is that of the active smooth piece: the clip mask of every
// perturbed control, the collision branch of every rollout position and its
// nearest cloud point (lowest index on ties) are held fixed.
//
//   k_adjoint      one lane per (instance, sample): forward sweep storing the
//                  state every kSeg steps, then, segment by segment from the last,
//                  recompute the segment's states and run the reverse sweep through
//                  the cost terms, the quaternion renormalisation and the four RK4
//                  stages; writes dS/du_t (masked) per sample
//   k_grad_reduce  fixed-order block sums over samples -> dL/du_nom, dL/dw
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "aero_device.h"
#include "aero_internal.h"

namespace aero {
namespace {

constexpr int kSeg = 8;  // checkpoint interval (steps)

// Perturbed, clipped control of (sample k, step t, instance m) and its clip mask.
__device__ inline void control_at(const DevParams& prm, const DevProblem& P, int m, int k, int t,
                                  double u[4], bool mask[4]) {
  double nz[4];
  const int64_t row = (int64_t)m * P.N + t;
  if (P.noise) {  // the normals the rollout drew (same counters, same values)
#pragma unroll
    for (int c = 0; c < 4; ++c) nz[c] = P.noise[(row * 4 + c) * P.K + k];
  } else if (prm.sigma[0] != 0.0 || prm.sigma[1] != 0.0 || prm.sigma[2] != 0.0 ||
             prm.sigma[3] != 0.0) {
    normals4(prm, P.problem_id, (uint32_t)k, (uint32_t)t, (uint32_t)m, nz);
  } else {  // a noise-free rollout: the noise term vanishes, nothing to draw
#pragma unroll
    for (int c = 0; c < 4; ++c) nz[c] = 0.0;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double v = (double)P.u_nom[row * 4 + c] + prm.sigma[c] * nz[c];
    mask[c] = v >= prm.u_min[c] && v <= prm.u_max[c];
    u[c] = fmin(fmax(v, prm.u_min[c]), prm.u_max[c]);
  }
}

// ly += (d xdot / d y)^T a ; lu += (d xdot / d u)^T a
__device__ inline void xdot_vjp(const double* y, const double* u, const Dyn& d, const double* a,
                                double* ly, double* lu) {
  const double qw = y[3], qx = y[4], qy = y[5], qz = y[6];
  const double wx = u[1], wy = u[2], wz = u[3];
  // p' = v
  ly[7] += a[0];
  ly[8] += a[1];
  ly[9] += a[2];
  // q' = 1/2 q (x) (0, omega): linear in q and in omega
  const double a0 = a[3], a1 = a[4], a2 = a[5], a3 = a[6];
  ly[3] += 0.5 * (a1 * wx + a2 * wy + a3 * wz);
  ly[4] += 0.5 * (-a0 * wx - a2 * wz + a3 * wy);
  ly[5] += 0.5 * (-a0 * wy + a1 * wz - a3 * wx);
  ly[6] += 0.5 * (-a0 * wz - a1 * wy + a2 * wx);
  lu[1] += 0.5 * (-qx * a0 + qw * a1 + qz * a2 - qy * a3);
  lu[2] += 0.5 * (-qy * a0 - qz * a1 + qw * a2 + qx * a3);
  lu[3] += 0.5 * (-qz * a0 + qy * a1 - qx * a2 + qw * a3);
  // v' = (F/m) b(q) + g,  b = (2(xz+wy), 2(yz-wx), 1-2(x^2+y^2))
  const double b0 = 2.0 * (qx * qz + qw * qy), b1 = 2.0 * (qy * qz - qw * qx),
               b2 = 1.0 - 2.0 * (qx * qx + qy * qy);
  const double v0 = a[7], v1 = a[8], v2 = a[9];
  lu[0] += d.inv_m * (b0 * v0 + b1 * v1 + b2 * v2);
  const double am = u[0] * d.inv_m;
  ly[3] += am * (2.0 * qy * v0 - 2.0 * qx * v1);
  ly[4] += am * (2.0 * qz * v0 - 2.0 * qw * v1 - 4.0 * qx * v2);
  ly[5] += am * (2.0 * qw * v0 + 2.0 * qz * v1 - 4.0 * qy * v2);
  ly[6] += am * (2.0 * qx * v0 + 2.0 * qy * v1);
}

// Reverse of x_next = normalise_q(x + dt/6 (k1 + 2k2 + 2k3 + k4)):
// lam (adjoint of x_next) -> lam (adjoint of x), lu += adjoint of u.
__device__ inline void rk4_vjp(const double* x, const double* u, double dt, const Dyn& d,
                               double* lam, double* lu) {
  double k1[10], k2[10], k3[10], y[10], k4[10];
  xdot(x, u, d, k1);
#pragma unroll
  for (int i = 0; i < 10; ++i) y[i] = x[i] + 0.5 * dt * k1[i];
  xdot(y, u, d, k2);
#pragma unroll
  for (int i = 0; i < 10; ++i) y[i] = x[i] + 0.5 * dt * k2[i];
  xdot(y, u, d, k3);
#pragma unroll
  for (int i = 0; i < 10; ++i) y[i] = x[i] + dt * k3[i];
  xdot(y, u, d, k4);
  // renormalisation of the quaternion part
  double zq[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    zq[i] = x[3 + i] + dt / 6.0 * (k1[3 + i] + 2.0 * k2[3 + i] + 2.0 * k3[3 + i] + k4[3 + i]);
  const double nq = sqrt(zq[0] * zq[0] + zq[1] * zq[1] + zq[2] * zq[2] + zq[3] * zq[3]);
  const double inv = 1.0 / nq;
  double qn[4], dot = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    qn[i] = zq[i] * inv;
    dot += qn[i] * lam[3 + i];
  }
  double lz[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) lz[i] = lam[i];
#pragma unroll
  for (int i = 0; i < 4; ++i) lz[3 + i] = (lam[3 + i] - qn[i] * dot) * inv;
  // z = x + dt/6 (k1 + 2 k2 + 2 k3 + k4)
  double lx[10], lk[10], ly[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    lx[i] = lz[i];
    lk[i] = dt / 6.0 * lz[i];  // adjoint of k4
    ly[i] = 0.0;
  }
  // k4 = f(x + dt k3)
#pragma unroll
  for (int i = 0; i < 10; ++i) y[i] = x[i] + dt * k3[i];
  xdot_vjp(y, u, d, lk, ly, lu);
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    lx[i] += ly[i];
    lk[i] = dt / 3.0 * lz[i] + dt * ly[i];  // adjoint of k3
    ly[i] = 0.0;
  }
  // k3 = f(x + dt/2 k2)
#pragma unroll
  for (int i = 0; i < 10; ++i) y[i] = x[i] + 0.5 * dt * k2[i];
  xdot_vjp(y, u, d, lk, ly, lu);
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    lx[i] += ly[i];
    lk[i] = dt / 3.0 * lz[i] + 0.5 * dt * ly[i];  // adjoint of k2
    ly[i] = 0.0;
  }
  // k2 = f(x + dt/2 k1)
#pragma unroll
  for (int i = 0; i < 10; ++i) y[i] = x[i] + 0.5 * dt * k1[i];
  xdot_vjp(y, u, d, lk, ly, lu);
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    lx[i] += ly[i];
    lk[i] = dt / 6.0 * lz[i] + 0.5 * dt * ly[i];  // adjoint of k1
  }
  // k1 = f(x)
  xdot_vjp(x, u, d, lk, lx, lu);
#pragma unroll
  for (int i = 0; i < 10; ++i) lam[i] = lx[i];
}

// d R_ik / d(w, x, y, z) for the unit-quaternion rotation matrix, row-major R.
__device__ inline void drot(double w, double x, double y, double z, double D[9][4]) {
  const double t2 = 2.0, t4 = 4.0;
  D[0][0] = 0; D[0][1] = 0; D[0][2] = -t4 * y; D[0][3] = -t4 * z;
  D[1][0] = -t2 * z; D[1][1] = t2 * y; D[1][2] = t2 * x; D[1][3] = -t2 * w;
  D[2][0] = t2 * y; D[2][1] = t2 * z; D[2][2] = t2 * w; D[2][3] = t2 * x;
  D[3][0] = t2 * z; D[3][1] = t2 * y; D[3][2] = t2 * x; D[3][3] = t2 * w;
  D[4][0] = 0; D[4][1] = -t4 * x; D[4][2] = 0; D[4][3] = -t4 * z;
  D[5][0] = -t2 * x; D[5][1] = -t2 * w; D[5][2] = t2 * z; D[5][3] = t2 * y;
  D[6][0] = -t2 * y; D[6][1] = t2 * z; D[6][2] = -t2 * w; D[6][3] = t2 * x;
  D[7][0] = t2 * x; D[7][1] = t2 * w; D[7][2] = t2 * z; D[7][3] = t2 * y;
  D[8][0] = 0; D[8][1] = -t4 * x; D[8][2] = -t4 * y; D[8][3] = 0;
}

// lam += d(weighted state cost at step t)/d x_{t+1}
__device__ inline void cost_grad(const double* x, int t, const DevParams& prm, const DevProblem& P,
                                 const double cf[3][6], const double pg[3], const double vg[3],
                                 const double Rg[9], int m, int k, double* lam) {
  // tracking: Q_track |p - f((t+1) dt)|
  const double tau = (double)(t + 1) * prm.dt;
  double e[3], n2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double f = cf[a][5];
#pragma unroll
    for (int i = 4; i >= 0; --i) f = f * tau + cf[a][i];
    e[a] = x[a] - f;
    n2 += e[a] * e[a];
  }
  if (n2 > 0.0) {
    const double s = prm.w[0] * prm.Q_track / sqrt(n2);
#pragma unroll
    for (int a = 0; a < 3; ++a) lam[a] += s * e[a];
  }
  // velocity norm: Q_vnorm |v|^2
#pragma unroll
  for (int a = 0; a < 3; ++a) lam[7 + a] += prm.w[1] * prm.Q_vnorm * 2.0 * x[7 + a];
  // goal: Q_p |p - pg| + Q_v |v - vg| + Q_q |R Rg^T - I|_F
  double ep[3], ev[3], np2 = 0.0, nv2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ep[a] = x[a] - pg[a];
    ev[a] = x[7 + a] - vg[a];
    np2 += ep[a] * ep[a];
    nv2 += ev[a] * ev[a];
  }
  if (np2 > 0.0) {
    const double s = prm.w[3] * prm.Q_p / sqrt(np2);
#pragma unroll
    for (int a = 0; a < 3; ++a) lam[a] += s * ep[a];
  }
  if (nv2 > 0.0) {
    const double s = prm.w[3] * prm.Q_v / sqrt(nv2);
#pragma unroll
    for (int a = 0; a < 3; ++a) lam[7 + a] += s * ev[a];
  }
  double R[9];
  rotmat(x[3], x[4], x[5], x[6], R);
  double E[9], ne2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double v = R[3 * i] * Rg[3 * j] + R[3 * i + 1] * Rg[3 * j + 1] + R[3 * i + 2] * Rg[3 * j + 2];
      if (i == j) v -= 1.0;
      E[3 * i + j] = v;
      ne2 += v * v;
    }
  if (ne2 > 0.0) {
    // d|E|/dR_ik = (E Rg)_ik / |E|
    double D[9][4];
    drot(x[3], x[4], x[5], x[6], D);
    const double s = prm.w[3] * prm.Q_q / sqrt(ne2);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        const double G = E[3 * i] * Rg[kk] + E[3 * i + 1] * Rg[3 + kk] + E[3 * i + 2] * Rg[6 + kk];
#pragma unroll
        for (int c = 0; c < 4; ++c) lam[3 + c] += s * G * D[3 * i + kk][c];
      }
  }
  // collision: C exp(-a (d - d_min)) on the middle branch, nearest point held fixed
  if (P.n_points > 0) {
    const int64_t qi = ((int64_t)m * P.N + t) * P.K + k;
    const int idx = P.nidx_in ? P.nidx_in[qi] : P.nidx[qi];
    if (idx >= 0 && idx < P.n_points) {  // caller-given indices may be stale
      const double dx = x[0] - (double)P.cloud[3 * (int64_t)idx];
      const double dy = x[1] - (double)P.cloud[3 * (int64_t)idx + 1];
      const double dz = x[2] - (double)P.cloud[3 * (int64_t)idx + 2];
      const double dd = sqrt(dx * dx + dy * dy + dz * dz);
      if (dd >= prm.d_min && dd < prm.d_max && dd > 0.0) {
        const double s = -prm.w[4] * prm.a * prm.C * exp(-prm.a * (dd - prm.d_min)) / dd;
        lam[0] += s * dx;
        lam[1] += s * dy;
        lam[2] += s * dz;
      }
    }
  }
}

// One wave per workgroup (as the forward rollout): the sequential sweeps are few, one
// lane per sample, and each step stores a state record and four gradients per
// sample, so the waves are spread over as many CUs as there are.
constexpr int kAdjBlock = 64;

__global__ __launch_bounds__(kAdjBlock) void k_adjoint(const DevProblem* __restrict__ prob,
                                                    DevParams prm, int64_t total, double* ckpt,
                                                    double* seg, double* gsamp) {
  const int64_t gid = (int64_t)blockIdx.x * kAdjBlock + threadIdx.x;
  if (gid >= total) return;
  const DevProblem& P = *prob;
  load_weights(P.w_dev, prm);
  const int K = P.K, N = P.N;
  const int m = (int)(gid / K), k = (int)(gid % K);
  const int64_t MK = total;
  const Dyn dyn{1.0 / prm.mass, prm.gravity};
  double cf[3][6];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int i = 0; i < 6; ++i) cf[a][i] = P.coef[(m * 3 + a) * 6 + i];
  const double pg[3] = {P.pg[0], P.pg[1], P.pg[2]}, vg[3] = {P.vg[0], P.vg[1], P.vg[2]};
  double Rg[9];
  rotmat(P.qg[0], P.qg[1], P.qg[2], P.qg[3], Rg);

  // forward sweep with checkpoints (sample-fastest layout: [ckpt][10][M K])
  double x[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) x[i] = P.x0[i];
  for (int t = 0; t < N; ++t) {
    if (t % kSeg == 0) {
      double* c = ckpt + (int64_t)(t / kSeg) * 10 * MK + gid;
#pragma unroll
      for (int i = 0; i < 10; ++i) c[i * MK] = x[i];
    }
    double u[4];
    bool msk[4];
    control_at(prm, P, m, k, t, u, msk);
    rk4(x, u, prm.dt, dyn);
  }
  // x is now x_N
  double lam[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  double xnext[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) xnext[i] = x[i];
  const int n_seg = (N + kSeg - 1) / kSeg;
  double u_after[4] = {0, 0, 0, 0};  // u_{t+1} while sweeping backwards
  // u_t and its clip mask, carried from the step after (its u_{t-1}) once known
  double u[4];
  bool msk[4];
  bool have_u = false;
  for (int sgi = n_seg - 1; sgi >= 0; --sgi) {
    const int t0 = sgi * kSeg, t1 = min(t0 + kSeg, N);
    const double* c = ckpt + (int64_t)sgi * 10 * MK + gid;
#pragma unroll
    for (int i = 0; i < 10; ++i) x[i] = c[i * MK];
    // recompute x_t0 .. x_{t1-1} into the per-lane segment buffer
    for (int t = t0; t < t1; ++t) {
      double* sp = seg + (int64_t)(t - t0) * 10 * MK + gid;
#pragma unroll
      for (int i = 0; i < 10; ++i) sp[i * MK] = x[i];
      if (t + 1 < t1) {
        double uc[4];
        bool mc[4];
        control_at(prm, P, m, k, t, uc, mc);
        rk4(x, uc, prm.dt, dyn);
      }
    }
    for (int t = t1 - 1; t >= t0; --t) {
      // cost of step t sits on x_{t+1}
      cost_grad(xnext, t, prm, P, cf, pg, vg, Rg, m, k, lam);
      const double* sp = seg + (int64_t)(t - t0) * 10 * MK + gid;
      double xt[10];
#pragma unroll
      for (int i = 0; i < 10; ++i) xt[i] = sp[i * MK];
      if (!have_u) control_at(prm, P, m, k, t, u, msk);
      double lu[4] = {0, 0, 0, 0};
      rk4_vjp(xt, u, prm.dt, dyn, lam, lu);
      // control cost: Q_c |u_t|^2 (t <= N-2), Q_cdelta |u_t - u_{t-1}|^2 (1 <= t <= N-2)
      double u_before[4] = {0, 0, 0, 0};
      bool mb[4] = {false, false, false, false};
      if (t >= 1) control_at(prm, P, m, k, t - 1, u_before, mb);
      const int64_t row = (int64_t)m * N + t;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        double g = lu[cc];
        if (t <= N - 2) g += prm.w[2] * prm.Q_c * 2.0 * u[cc];
        if (t >= 1 && t <= N - 2) g += prm.w[2] * prm.Q_cdelta * 2.0 * (u[cc] - u_before[cc]);
        if (t + 1 >= 1 && t + 1 <= N - 2) g -= prm.w[2] * prm.Q_cdelta * 2.0 * (u_after[cc] - u[cc]);
        gsamp[(row * 4 + cc) * K + k] = msk[cc] ? g : 0.0;
        u_after[cc] = u[cc];
        u[cc] = u_before[cc];
        msk[cc] = mb[cc];
      }
      have_u = t >= 1;
#pragma unroll
      for (int i = 0; i < 10; ++i) xnext[i] = xt[i];
    }
  }
}

__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// Blocks 0 .. rows-1: one (instance, step) row each; block `rows`: the weights.
// Sums over samples in a fixed order.  Blocks [0, rows) reduce one (instance, step)
// row of the per-sample control gradients; blocks [rows, rows + 5 kWParts) each sum
// one fixed slice of one cost term for the weight gradient, finished by
// k_grad_w_final in slice order.
constexpr int kWParts = 64;

// The upstream gradient: a device scalar, or 1 when none is given.
__device__ inline double upstream(const float* grad_L) {
  return grad_L ? (double)*grad_L : 1.0;
}

__global__ __launch_bounds__(kBlock) void k_grad_reduce(const DevProblem* __restrict__ prob,
                                                        int64_t rows, const double* gsamp,
                                                        const float* grad_L, float* grad_u,
                                                        double* wpart) {
  __shared__ double sh[4];
  const DevProblem& P = *prob;
  const int K = P.K;
  const double scale = upstream(grad_L);
  if ((int64_t)blockIdx.x < rows) {
    const int64_t row = blockIdx.x;
    for (int c = 0; c < 4; ++c) {
      double acc = 0.0;
      const double* g = gsamp + (row * 4 + c) * K;
      for (int k = threadIdx.x; k < K; k += kBlock) acc += g[k];
      acc = block_sum(acc, sh);
      if (threadIdx.x == 0) grad_u[row * 4 + c] = (float)(scale * acc);
    }
  } else {
    const int64_t j = (int64_t)blockIdx.x - rows;
    const int i = (int)(j / kWParts), part = (int)(j % kWParts);
    const int64_t MK = (int64_t)P.M * K;
    const int64_t per = (MK + kWParts - 1) / kWParts;
    const int64_t a = part * per, b = min<int64_t>(MK, a + per);
    double acc = 0.0;
    for (int64_t q = a + threadIdx.x; q < b; q += kBlock) acc += P.J[i * MK + q];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) wpart[i * kWParts + part] = acc;
  }
}

__global__ void k_grad_w_final(const double* wpart, const float* grad_L, float* grad_w) {
  const int i = threadIdx.x;
  if (i >= 5) return;
  const double scale = upstream(grad_L);
  double acc = 0.0;
  for (int p = 0; p < kWParts; ++p) acc += wpart[i * kWParts + p];
  grad_w[i] = (float)(scale * acc);
}

}  // namespace

hipError_t launch_adjoint(const DevProblem* d_prob, const DevParams& prm, int64_t samples,
                          double* ckpt, double* seg, double* gsamp, hipStream_t s) {
  k_adjoint<<<(unsigned)((samples + kAdjBlock - 1) / kAdjBlock), kAdjBlock, 0, s>>>(
      d_prob, prm, samples, ckpt, seg, gsamp);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const DevProblem* d_prob, const DevParams& prm, int64_t rows,
                              const double* gsamp, const float* grad_L, float* grad_u,
                              float* grad_w, double* wpart, hipStream_t s) {
  (void)prm;
  k_grad_reduce<<<(unsigned)(rows + 5 * kWParts), kBlock, 0, s>>>(d_prob, rows, gsamp, grad_L,
                                                                  grad_u, wpart);
  k_grad_w_final<<<1, 64, 0, s>>>(wpart, grad_L, grad_w);
  return hipGetLastError();
}

size_t grad_w_parts() { return 5 * kWParts; }

}  // namespace aero
