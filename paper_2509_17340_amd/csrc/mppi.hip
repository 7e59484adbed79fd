// Stage I (Sec. III-B, IV-C) and Stage II (Sec. IV-C) kernels.
//
//   k_rollout      one lane per (problem, instance, sample): Philox noise, clip,
//                  RK4 in binary64, smooth cost terms; writes the clipped
//                  perturbations and float32 positions as sample-fastest planes
//   (the nearest-distance kernels live in distance.hip)
//   k_finalize     J_col from the distances, S1 = smooth part + w_col J_col
//   k_update       per (instance, step): rho, eta, and sum_k eps_k delta_eff_k
//                  with fixed-order wave/block reductions in binary64
//   k_sel_rollout  Stage II noise-free rollouts and J_goal
//   k_sel_final    S2 and the argmin per problem
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "aero_device.h"
#include "aero_internal.h"

namespace aero {
namespace {

constexpr unsigned kInfBits = 0x7f800000u;

__device__ inline void load_rg(const float* qg, double Rg[9]) {
  const double w = qg[0], x = qg[1], y = qg[2], z = qg[3];
  rotmat(w, x, y, z, Rg);
}

// The rollout's standard normals for every (instance, step, sample), drawn in
// parallel ahead of the sequential rollout (the same counter-based stream); also
// resets the per-position distance outputs.
__global__ __launch_bounds__(kBlock) void k_noise(const DevProblem* __restrict__ probs, int n,
                                                  int64_t total, DevParams prm) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= total) return;
  const int b = find_owner(probs, n, gid, [](const DevProblem& p) { return p.elem_base; });
  const DevProblem& P = probs[b];
  const int K = P.K, N = P.N;
  const int64_t local = gid - P.elem_base;
  const int64_t row = local / K;
  const int k = (int)(local % K), m = (int)(row / N), t = (int)(row % N);
  double nz[4];
  normals4(prm, P.problem_id, (uint32_t)k, (uint32_t)t, (uint32_t)m, nz);
#pragma unroll
  for (int c = 0; c < 4; ++c) P.noise[(row * 4 + c) * K + k] = nz[c];
  // per-position outputs of this call start empty
  P.mind2[local] = kInfBits;
  if (P.out_slot) P.out_slot[local] = kInfBits;
  if (P.nidx) P.nidx[local] = -1;
}

__global__ __launch_bounds__(kBlock) void k_rollout(const DevProblem* __restrict__ probs, int n,
                                                    int64_t total, DevParams prm) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= total) return;
  const int b = find_owner(probs, n, gid, [](const DevProblem& p) { return p.sample_base; });
  const DevProblem& P = probs[b];
  const int K = P.K, N = P.N;
  const int64_t local = gid - P.sample_base;
  const int m = (int)(local / K), k = (int)(local % K);
  const int64_t MNK = (int64_t)P.M * N * K;
  if (local == 0) {
    if (P.work_count) *P.work_count = 0;  // pass B's work list of this call
    if (P.sort_box)
      for (int a = 0; a < 3; ++a) {
        P.sort_box[a] = 0xffffffffu;      // order-preserving bits: running min, max
        P.sort_box[3 + a] = 0u;
      }
  }

  const Dyn dyn{1.0 / prm.mass, prm.gravity};
  double x[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) x[i] = P.x0[i];
  const double pg[3] = {P.pg[0], P.pg[1], P.pg[2]}, vg[3] = {P.vg[0], P.vg[1], P.vg[2]};
  double Rg[9];
  load_rg(P.qg, Rg);
  double cf[3][6];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int i = 0; i < 6; ++i) cf[a][i] = P.coef[(m * 3 + a) * 6 + i];

  double s_track = 0.0, s_vnorm = 0.0, s_u2 = 0.0, s_du2 = 0.0, s_goal = 0.0;
  double up[4] = {0.0, 0.0, 0.0, 0.0};
  // The step's inputs (nominal control and normals) are loaded one step ahead, so
  // that their memory latency overlaps the previous RK4 step.
  double nz_next[4], un_next[4];
  auto fetch = [&](int t) {
    const int64_t r = (int64_t)m * N + t;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      nz_next[c] = P.noise[(r * 4 + c) * K + k];
      un_next[c] = P.u_nom[r * 4 + c];
    }
  };
  // Cost terms of the state reached at step t: guide error at (t+1) dt, speed and
  // goal terms.  They are evaluated one step late, in the same straight-line code
  // as the following RK4 step, so that the two independent dependency chains
  // interleave; every sum still runs over t = 0 .. N-1 in order.
  auto state_costs = [&](const double* xs, int t) {
    const double tau = (double)(t + 1) * prm.dt;
    double e2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double f = cf[a][5];
#pragma unroll
      for (int i = 4; i >= 0; --i) f = f * tau + cf[a][i];
      const double e = xs[a] - f;
      e2 += e * e;
    }
    s_track += sqrt(e2);
    s_vnorm += xs[7] * xs[7] + xs[8] * xs[8] + xs[9] * xs[9];
    s_goal += goal_term(xs, pg, vg, Rg, prm);
  };
  double xc[10];
  // One step: perturbed, clipped control, its deviation, the RK4 update (the state
  // before it kept in xc) and the control terms (u_t for t <= N-2, the change for
  // 1 <= t <= N-2; predicated, so the body has no branches).
  auto advance = [&](int t) {
    double nz[4], unv[4];
    const int64_t row = (int64_t)m * N + t;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      nz[c] = nz_next[c];
      unv[c] = un_next[c];
    }
    fetch(t + 1 < N ? t + 1 : t);  // in bounds; unused after the last step
    double u[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double un = unv[c];
      const double v = un + prm.sigma[c] * nz[c];
      u[c] = fmin(fmax(v, prm.u_min[c]), prm.u_max[c]);
      P.deff[(row * 4 + c) * K + k] = (float)(u[c] - un);
    }
#pragma unroll
    for (int i = 0; i < 10; ++i) xc[i] = x[i];
    rk4(x, u, prm.dt, dyn);
    const int64_t qi = row * K + k;
    P.pos[qi] = (float)x[0];
    P.pos[MNK + qi] = (float)x[1];
    P.pos[2 * MNK + qi] = (float)x[2];
    const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
    const double d0 = u[0] - up[0], d1 = u[1] - up[1], d2 = u[2] - up[2], d3 = u[3] - up[3];
    const double du2 = d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
    s_u2 += t <= N - 2 ? u2 : 0.0;
    s_du2 += (t >= 1 && t <= N - 2) ? du2 : 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) up[c] = u[c];
  };
  fetch(0);
  advance(0);
  for (int t = 1; t < N; ++t) {
    advance(t);
    state_costs(xc, t - 1);
  }
  state_costs(x, N - 1);
  const double J_track = prm.Q_track * s_track;
  const double J_vnorm = prm.Q_vnorm * s_vnorm;
  const double J_ctrl = prm.Q_c * s_u2 + prm.Q_cdelta * s_du2;
  const int64_t i = (int64_t)m * K + k;
  P.S_smooth[i] = prm.w[0] * J_track + prm.w[1] * J_vnorm + prm.w[2] * J_ctrl + prm.w[3] * s_goal;
  if (P.J) {
    const int64_t MK = (int64_t)P.M * K;
    P.J[i] = J_track;
    P.J[MK + i] = J_vnorm;
    P.J[2 * MK + i] = J_ctrl;
    P.J[3 * MK + i] = s_goal;
  }
}

__global__ __launch_bounds__(kBlock) void k_finalize(const DevProblem* __restrict__ probs, int n,
                                                     int64_t total, DevParams prm) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= total) return;
  const int b = find_owner(probs, n, gid, [](const DevProblem& p) { return p.sample_base; });
  const DevProblem& P = probs[b];
  const int K = P.K, N = P.N;
  const int64_t local = gid - P.sample_base;
  const int m = (int)(local / K), k = (int)(local % K);
  // phi vanishes from d_max on; sqrt is correctly rounded and d_max^2 is exact in
  // binary64, so skipping d^2 >= d_max^2 changes no sum
  const double dmax2 = prm.d_max * prm.d_max;
  double col = 0.0;
#pragma unroll 8
  for (int t = 0; t < N; ++t) {
    const float d2 = __uint_as_float(P.mind2[((int64_t)m * N + t) * K + k]);
    if ((double)d2 < dmax2) col += collision_phi(sqrt((double)d2), prm);
  }
  const int64_t i = (int64_t)m * K + k;
  P.S1[i] = P.S_smooth[i] + prm.w[4] * col;
  if (P.J) P.J[4 * (int64_t)P.M * K + i] = col;
}

// Block-wide reductions (4 waves) in a fixed order; every thread gets the result.
__device__ inline double block_min(double v, double* sh) {
  v = wave_min(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
}

__device__ inline void block_sum5(double v[5], double* sh) {
#pragma unroll
  for (int i = 0; i < 5; ++i) v[i] = wave_sum(v[i]);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int i = 0; i < 5; ++i) sh[i * 4 + w] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 5; ++i) v[i] = ((sh[i * 4] + sh[i * 4 + 1]) + sh[i * 4 + 2]) + sh[i * 4 + 3];
}

__global__ __launch_bounds__(kBlock) void k_update(const DevProblem* __restrict__ probs, int n,
                                                   DevParams prm) {
  __shared__ double sh[20];
  const int64_t gid = blockIdx.x;
  const int b = find_owner(probs, n, gid, [](const DevProblem& p) { return p.row_base; });
  const DevProblem& P = probs[b];
  const int K = P.K, N = P.N;
  const int64_t row = gid - P.row_base;  // m * N + t
  const int m = (int)(row / N);
  const double* S = P.S1 + (int64_t)m * K;
  double mn = INFINITY;
  for (int k = threadIdx.x; k < K; k += kBlock) mn = fmin(mn, S[k]);
  const double rho = block_min(mn, sh);
  const double inv_lam = 1.0 / prm.lambda;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const float* D = P.deff + row * 4 * K;
  for (int k = threadIdx.x; k < K; k += kBlock) {
    const double e = exp(-(S[k] - rho) * inv_lam);
    acc[0] += e;
    acc[1] += e * (double)D[k];
    acc[2] += e * (double)D[K + k];
    acc[3] += e * (double)D[2 * K + k];
    acc[4] += e * (double)D[3 * K + k];
  }
  block_sum5(acc, sh);
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    float* u = P.u_nom + row * 4 + c;
    *u = (float)((double)*u + acc[1 + c] / acc[0]);
  }
}

__global__ __launch_bounds__(kBlock) void k_sel_rollout(const DevSelect* __restrict__ sel, int n,
                                                        int64_t total, DevParams prm) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= total) return;
  const int b = find_owner(sel, n, gid, [](const DevSelect& p) { return p.inst_base; });
  const DevSelect& P = sel[b];
  const int m = (int)(gid - P.inst_base), N = P.N;
  const int64_t MN = (int64_t)P.M * N;
  const Dyn dyn{1.0 / prm.mass, prm.gravity};
  double x[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) x[i] = P.x0[i];
  const double pg[3] = {P.pg[0], P.pg[1], P.pg[2]}, vg[3] = {P.vg[0], P.vg[1], P.vg[2]};
  double Rg[9];
  load_rg(P.qg, Rg);
  double s_goal = 0.0;
  double u_next[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) u_next[c] = P.u_nom[(int64_t)m * N * 4 + c];
  double xc[10];
  for (int t = 0; t < N; ++t) {
    const int64_t row = (int64_t)m * N + t;
    double u[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = u_next[c];
    const int64_t nrow = t + 1 < N ? row + 1 : row;  // next step's control, loaded now
#pragma unroll
    for (int c = 0; c < 4; ++c) u_next[c] = P.u_nom[nrow * 4 + c];
#pragma unroll
    for (int i = 0; i < 10; ++i) xc[i] = x[i];
    rk4(x, u, prm.dt, dyn);
    // goal term of the previous step's state, next to this RK4 step (sum order kept)
    if (t > 0) s_goal += goal_term(xc, pg, vg, Rg, prm);
    P.pos[row] = (float)x[0];
    P.pos[MN + row] = (float)x[1];
    P.pos[2 * MN + row] = (float)x[2];
    P.mind2[row] = kInfBits;
  }
  s_goal += goal_term(x, pg, vg, Rg, prm);
  P.goal_cost[m] = prm.w[3] * s_goal;
}

__global__ __launch_bounds__(kBlock) void k_sel_final(const DevSelect* __restrict__ sel,
                                                      DevParams prm) {
  __shared__ double s2[AERO_M_MAX];
  const DevSelect& P = sel[blockIdx.x];
  const int M = P.M, N = P.N;
  for (int m = threadIdx.x; m < M; m += kBlock) {
    double col = 0.0;
    for (int t = 0; t < N; ++t)
      col += collision_phi(sqrt((double)__uint_as_float(P.mind2[(int64_t)m * N + t])), prm);
    const double v = P.goal_cost[m] + prm.w[4] * col;
    s2[m] = v;
    P.S2[m] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int bi = 0;
    for (int m = 1; m < M; ++m)
      if (s2[m] < s2[bi]) bi = m;
    *P.best = bi;
  }
}

inline unsigned grid1d(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Receding-horizon warm start: every destination instance gets the selected
// source sequence advanced by `shift` steps (last control held).
__global__ void k_shift_controls(const float* __restrict__ src, int M_src, int N,
                                 const int32_t* __restrict__ index, int shift,
                                 float* __restrict__ dst, int M_dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M_dst * N * 4) return;
  int sel = *index;
  sel = sel < 0 ? 0 : (sel >= M_src ? M_src - 1 : sel);
  const int c = (int)(i % 4), t = (int)((i / 4) % N);
  const int ts = t + shift < N ? t + shift : N - 1;
  dst[i] = src[((int64_t)sel * N + ts) * 4 + c];
}

// Step candidates: out[0] = u, out[j] = clip(u - s_j g / max|g|).  One block.
__global__ void k_step_candidates(const float* __restrict__ u, const float* __restrict__ g,
                                  int N, float s0, float beta, int n, DevParams prm,
                                  float* __restrict__ out) {
  __shared__ float red[kBlock];
  float m = 0.0f;
  for (int i = threadIdx.x; i < N * 4; i += blockDim.x) m = fmaxf(m, fabsf(g[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const float gmax = red[0];
  for (int i = threadIdx.x; i < n * N * 4; i += blockDim.x) {
    const int j = i / (N * 4), e = i % (N * 4), c = e % 4;
    if (j == 0 || !(gmax > 0.0f)) {
      out[i] = u[e];
      continue;
    }
    double s = (double)s0;
    for (int k = 1; k < j; ++k) s *= (double)beta;
    const double v = (double)u[e] - s * (double)g[e] / (double)gmax;
    out[i] = (float)fmin(fmax(v, prm.u_min[c]), prm.u_max[c]);
  }
}

// Host bytes carried in the kernel arguments and written to device memory.
constexpr int kPutBytes = 2048;
struct PutBlob {
  uint32_t n;
  uint32_t pad;
  unsigned char b[kPutBytes];
};

__global__ void k_put_bytes(unsigned char* dst, PutBlob blob) {
  for (uint32_t i = threadIdx.x; i < blob.n; i += blockDim.x) dst[i] = blob.b[i];
}

}  // namespace

hipError_t launch_shift_controls(const float* src, int M_src, int N, const int32_t* index,
                                 int shift, float* dst, int M_dst, hipStream_t s) {
  k_shift_controls<<<grid1d((int64_t)M_dst * N * 4), kBlock, 0, s>>>(src, M_src, N, index, shift,
                                                                     dst, M_dst);
  return hipGetLastError();
}

hipError_t launch_step_candidates(const float* u, const float* g, int N, float s0, float beta,
                                  int n, const DevParams& prm, float* out, hipStream_t s) {
  k_step_candidates<<<1, kBlock, 0, s>>>(u, g, N, s0, beta, n, prm, out);
  return hipGetLastError();
}

hipError_t launch_put_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const unsigned char* p = static_cast<const unsigned char*>(src);
  unsigned char* d = static_cast<unsigned char*>(dst);
  for (size_t off = 0; off < bytes; off += kPutBytes) {
    PutBlob blob;
    blob.n = (uint32_t)(bytes - off < (size_t)kPutBytes ? bytes - off : (size_t)kPutBytes);
    blob.pad = 0;
    memcpy(blob.b, p + off, blob.n);
    k_put_bytes<<<1, 256, 0, s>>>(d + off, blob);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_rollout_noise(const DevProblem* d_probs, int n, int64_t total_samples,
                                int64_t total_elems, const DevParams& prm, hipStream_t s) {
  if (total_elems > 0) k_noise<<<grid1d(total_elems), kBlock, 0, s>>>(d_probs, n, total_elems, prm);
  k_rollout<<<grid1d(total_samples), kBlock, 0, s>>>(d_probs, n, total_samples, prm);
  return hipGetLastError();
}

hipError_t launch_rollout(const DevProblem* d_probs, int n, int64_t total, const DevParams& prm,
                          hipStream_t s) {
  k_rollout<<<grid1d(total), kBlock, 0, s>>>(d_probs, n, total, prm);
  return hipGetLastError();
}

hipError_t launch_finalize(const DevProblem* d_probs, int n, int64_t total, const DevParams& prm,
                           hipStream_t s) {
  k_finalize<<<grid1d(total), kBlock, 0, s>>>(d_probs, n, total, prm);
  return hipGetLastError();
}

hipError_t launch_update(const DevProblem* d_probs, int n, int64_t total_rows,
                         const DevParams& prm, hipStream_t s) {
  k_update<<<(unsigned)total_rows, kBlock, 0, s>>>(d_probs, n, prm);
  return hipGetLastError();
}

hipError_t launch_select_rollout(const DevSelect* d_sel, int n, int64_t total_inst,
                                 const DevParams& prm, hipStream_t s) {
  k_sel_rollout<<<grid1d(total_inst), kBlock, 0, s>>>(d_sel, n, total_inst, prm);
  return hipGetLastError();
}

hipError_t launch_select_final(const DevSelect* d_sel, int n, const DevParams& prm,
                               hipStream_t s) {
  k_sel_final<<<(unsigned)n, kBlock, 0, s>>>(d_sel, prm);
  return hipGetLastError();
}

}  // namespace aero
