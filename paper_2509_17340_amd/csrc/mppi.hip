// Stage I (Sec. III-B, IV-C) and Stage II (Sec. IV-C) kernels.
//
//   k_noise        the rollout's standard normals (Philox, Box-Muller), drawn in
//                  parallel; resets the per-call outputs
//   k_rollout      one quad of lanes per (problem, instance, sample): clip, RK4 in
//                  binary64, the control term; writes the clipped perturbations and
//                  float32 positions as sample-fastest planes, the state after
//                  every step rounded to float32 as one 40-byte record per
//                  position, and the positions' bounding box for the spatial sort
//   (the nearest-distance kernels live in distance.hip)
//   k_finalize     per sample, the state terms (tracking, speed, goal) and J_col,
//                  with the horizon split into eight parts per sample; S1
//   k_weights      per instance: rho, e_k and eta
//   k_update       per (instance, step): sum_k e_k delta_eff_k / eta
//                  (both with fixed-order wave/block reductions in binary64)
//   k_sel_rollout  Stage II noise-free rollouts (states and positions)
//   k_sel_final    Stage II goal and collision terms per state, S2 and the argmin
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "aero_device.h"
#include "aero_internal.h"

namespace aero {
namespace {

constexpr unsigned kInfBits = 0x7f800000u;
typedef float fvec2 __attribute__((ext_vector_type(2)));  // 8-byte state accesses

__device__ inline void load_rg(const float* qg, double Rg[9]) {
  const double w = qg[0], x = qg[1], y = qg[2], z = qg[3];
  rotmat(w, x, y, z, Rg);
}

// The rollout's standard normals for every (instance, step, sample), drawn in
// parallel ahead of the sequential rollout (the same counter-based stream); also
// resets the per-position distance outputs (and nearest records), the call's cull
// item counter and the spatial sort's bounding box.
// Blocks from noise_blocks on compute the tile and sub-tile bounding boxes of the
// two-pass sets' clouds instead (independent work, one launch fewer).
__global__ __launch_bounds__(kBlock) void k_noise(const DevProblem* __restrict__ probs, int n,
                                                  int64_t total, DevParams prm,
                                                  const QuerySet* __restrict__ sets, int n_sets,
                                                  int64_t noise_blocks, PutBlob blob,
                                                  int64_t sets_off) {
  if (blob.n > 0) {  // descriptors in the argument (see put_blob)
    if (blockIdx.x == 0) put_blob(blob, (unsigned char*)probs);
    sets = reinterpret_cast<const QuerySet*>(blob.b + sets_off);
    probs = reinterpret_cast<const DevProblem*>(blob.b);
  }
  if ((int64_t)blockIdx.x >= noise_blocks) {
    // tile and sub-tile boxes of the raw clouds of the two-pass sets (tile_base order)
    const int64_t t = (int64_t)blockIdx.x - noise_blocks;
    const int si = find_owner(sets, n_sets, t, [](const QuerySet& q) { return q.tile_base; });
    const QuerySet& S = sets[si];
    tile_boxes(S.cloud, nullptr, S.n_points, t - S.tile_base, S.tbox, S.sbox, S.gbox);
    return;
  }
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= total) return;
  const int b = find_owner(probs, n, gid, [](const DevProblem& p) { return p.elem_base; });
  const DevProblem& P = probs[b];
  const int K = P.K, N = P.N;
  const int64_t local = gid - P.elem_base;
  const int64_t row = local / K;
  const int k = (int)(local % K), m = (int)(row / N), t = (int)(row % N);
  // the descriptor's fields in registers before the first store (a store could alias
  // the descriptor and force it to be read again behind the stores)
  const uint32_t problem_id = P.problem_id;
  AERO_GLOBAL double* __restrict__ noise = global_ptr(P.noise);
  AERO_GLOBAL unsigned* __restrict__ mind2 = global_ptr(P.mind2);
  AERO_GLOBAL unsigned* __restrict__ out_slot = global_ptr(P.out_slot);
  AERO_GLOBAL int32_t* __restrict__ nidx = global_ptr(P.nidx);
  AERO_GLOBAL unsigned long long* __restrict__ nn = global_ptr(P.nn);
  AERO_GLOBAL unsigned* __restrict__ amin = global_ptr(P.amin);
  if (local == 0) {
    AERO_GLOBAL int32_t* __restrict__ item_count = global_ptr(P.item_count);
    AERO_GLOBAL unsigned* __restrict__ sort_box = global_ptr(P.sort_box);
    if (item_count) *item_count = 0;  // the call's (query block, sub-tile) item list
    if (sort_box)
      for (int cp = 0; cp < kBoxCopies; ++cp)
        for (int a = 0; a < 3; ++a) {
          sort_box[cp * kBoxStride + a] = 0xffffffffu;  // order-preserving bits: running
          sort_box[cp * kBoxStride + 3 + a] = 0u;       // min, max
        }
  }
  double nz[4];
  normals4(prm, problem_id, (uint32_t)k, (uint32_t)t, (uint32_t)m, nz);
#pragma unroll
  for (int c = 0; c < 4; ++c) noise[(row * 4 + c) * K + k] = nz[c];
  // per-position outputs of this call start empty
  mind2[local] = kInfBits;
  if (out_slot) out_slot[local] = kInfBits;  // by slot: the slots are a permutation
  if (nidx) nidx[local] = -1;
  if (nn) nn[local] = ~0ull;
  if (amin) amin[local] = kInfBits;  // by slot, as out_slot
}

// Merge the position bounds of a wave's rollouts into their problems' sort boxes
// (the workgroup's copy).  Lane c < 3 of each quad holds the bounds of component c:
// one atomic per wave and component where the wave's active quads share a problem,
// else per lane.
__device__ inline void merge_box_quad(const DevProblem* __restrict__ probs, bool active, int b,
                                      int c, float lo, float hi) {
  const int b0 = __shfl(b, 0, 64);
  const bool one = __all(!active || b == b0);
  if (one) {
#pragma unroll
    for (int o = 4; o < 64; o <<= 1) {
      lo = fminf(lo, __shfl_xor(lo, o, 64));
      hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    }
    unsigned* box = probs[b0].sort_box;
    if ((threadIdx.x & 63) < 3 && box && lo <= hi) {
      box += (blockIdx.x % kBoxCopies) * kBoxStride;
      atomicMin(box + c, ord_bits(lo));
      atomicMax(box + 3 + c, ord_bits(hi));
    }
  } else if (active && c < 3 && lo <= hi) {
    unsigned* box = probs[b].sort_box;
    if (box) {
      box += (blockIdx.x % kBoxCopies) * kBoxStride;
      atomicMin(box + c, ord_bits(lo));
      atomicMax(box + 3 + c, ord_bits(hi));
    }
  }
}

// The sequential part of Stage I: only the dynamics and the control term, so that
// the chain of dependent binary64 operations per step is as short as the model
// allows; the state terms are scored in parallel by k_finalize.
// One rollout per quad of lanes (quad_rk4): lane c perturbs and clips control channel
// c, writes its clipped perturbation, and integrates state components c (quaternion)
// and, for c < 3, position and velocity c.  Four lanes per sample give the
// sequential part four times the waves, and each lane a quarter of the arithmetic.
// One wave per workgroup spreads the waves over as many CUs as possible.
constexpr int kRollBlock = 64;
// Steps of inputs loaded ahead.  Loads and stores share the in-order vector-memory
// counter, so the wait for a step's inputs also waits for the stores issued before
// them: with inputs loaded A steps ahead a step waits only for the stores of step
// t - A - 1, and the latency of a store's acknowledgement is spread over A + 1 steps.
// Each lane has 7 vector-memory operations per step in flight (2 loads, 5 stores),
// within the 63 the counter holds for A <= 8.
#ifndef AERO_ROLL_AHEAD
#define AERO_ROLL_AHEAD 2
#endif
constexpr int kAhead = AERO_ROLL_AHEAD;
static_assert(kAhead >= 1 && 7 * kAhead <= 63, "inputs ahead within the vector-memory counter");
static_assert(kSelCopies == 8, "Stage II: each lane of a quad resets two distance copies");

__global__ __launch_bounds__(kRollBlock) void k_rollout(const DevProblem* __restrict__ probs,
                                                        int n, int64_t total, DevParams prm) {
  const int64_t gid = ((int64_t)blockIdx.x * kRollBlock + threadIdx.x) >> 2;  // sample
  const QuadLane L = quad_lane(threadIdx.x);
  const int c = L.c;
  const bool active = gid < total;  // uniform over the quad
  float lo = INFINITY, hi = -INFINITY;
  int b = 0;
  if (active) {
    b = find_owner(probs, n, gid, [](const DevProblem& p) { return p.sample_base; });
    const DevProblem& P = probs[b];
    const int K = P.K, N = P.N;
    const int64_t local = gid - P.sample_base;
    const int m = (int)(local / K), k = (int)(local % K);
    const int64_t MNK = (int64_t)P.M * N * K;
    // The descriptor's pointers in registers, as global pointers: stores through
    // them could otherwise alias the descriptor, which would then be reloaded (and
    // waited for, behind every store in flight) at each step.
    AERO_GLOBAL const double* __restrict__ noise = global_ptr(P.noise);
    AERO_GLOBAL const float* __restrict__ u_nom = global_ptr(P.u_nom);
    AERO_GLOBAL float* __restrict__ deff = global_ptr(P.deff);
    AERO_GLOBAL float* __restrict__ pos = global_ptr(P.pos);
    AERO_GLOBAL float* __restrict__ state = global_ptr(P.state);
    const Dyn dyn{1.0 / prm.mass, prm.gravity};
    // this lane's channel constants (selected, not indexed: the arrays are kernel
    // arguments)
    const double sig = c == 0 ? prm.sigma[0] : c == 1 ? prm.sigma[1] : c == 2 ? prm.sigma[2]
                                                                              : prm.sigma[3];
    const double umin = c == 0 ? prm.u_min[0] : c == 1 ? prm.u_min[1] : c == 2 ? prm.u_min[2]
                                                                               : prm.u_min[3];
    const double umax = c == 0 ? prm.u_max[0] : c == 1 ? prm.u_max[1] : c == 2 ? prm.u_max[2]
                                                                               : prm.u_max[3];
    const bool pv = c < 3;  // lane 3 carries no position or velocity
    double p = P.x0[pv ? c : 0], v = P.x0[pv ? 7 + c : 7], q = P.x0[3 + c];
    double qa[4] = {P.x0[3], P.x0[4], P.x0[5], P.x0[6]};
    double s_u2 = 0.0, s_du2 = 0.0, up = 0.0;
    // The steps' inputs (normals and nominal controls) are loaded kAhead steps ahead
    // into a ring: a wait for a load also waits for every store issued before it,
    // so a load issued only one step ahead would put that step's stores on the
    // chain of dependent steps.
    // (kept as loaded: converting a value when it is loaded would wait for it there)
    double nzr[kAhead];
    float unr[kAhead];
    auto fetch = [&](int t, double& nz, float& un) {
      const int64_t r = (int64_t)m * N + (t < N ? t : N - 1);  // in bounds; unused past N-1
      nz = noise[(r * 4 + c) * K + k];
      un = u_nom[r * 4 + c];
    };
#pragma unroll
    for (int j = 0; j < kAhead; ++j) fetch(j, nzr[j], unr[j]);
    for (int t0 = 0; t0 < N; t0 += kAhead) {
#pragma unroll
      for (int j = 0; j < kAhead; ++j) {
        const int t = t0 + j;
        if (t >= N) break;
        // perturbed, clipped control channel c and its deviation, the RK4 update, and
        // the control terms (u_t for t <= N-2, the change for 1 <= t <= N-2)
        const int64_t row = (int64_t)m * N + t;
        const double un = unr[j];
        const double u = fmin(fmax(un + sig * nzr[j], umin), umax);
        fetch(t + kAhead, nzr[j], unr[j]);
        const float de = (float)(u - un);
        AERO_GLOBAL float* de_at = deff + (row * 4 + c) * K + k;
        *de_at = de;
        const QuadControl qc = quad_control(u, L, dyn);
        quad_rk4(p, v, q, qa, qc, L, prm.dt, dyn);
        const int64_t qi = row * K + k;
        // one 40-byte record [p, q, v] per position (rounded to float32), written by
        // the quad.  The loop body has no branch (so that the compiler's waits for the
        // loads ahead stay exact): lane 3, which has no position or velocity, stores
        // its own values again to its own addresses instead.
        AERO_GLOBAL float* rec = state + qi * 10;
        const float pf = (float)p, qf = (float)q, vf = (float)v;
        rec[3 + c] = qf;
        *(pv ? pos + c * MNK + qi : de_at) = pv ? pf : de;
        rec[pv ? c : 6] = pv ? pf : qf;
        rec[pv ? 7 + c : 6] = pv ? vf : qf;
        lo = fminf(lo, pv ? pf : INFINITY);
        hi = fmaxf(hi, pv ? pf : -INFINITY);
        const double du = u - up;
        s_u2 += t <= N - 2 ? u * u : 0.0;
        s_du2 += (t >= 1 && t <= N - 2) ? du * du : 0.0;
        up = u;
      }
    }
    // the quad's channel sums, added in a fixed order
    s_u2 += __shfl_xor(s_u2, 1, 64);
    s_du2 += __shfl_xor(s_du2, 1, 64);
    s_u2 += __shfl_xor(s_u2, 2, 64);
    s_du2 += __shfl_xor(s_du2, 2, 64);
    if (c == 0) {
      const double J_ctrl = prm.Q_c * s_u2 + prm.Q_cdelta * s_du2;
      const int64_t i = (int64_t)m * K + k;
      P.J_ctrl[i] = J_ctrl;
      if (P.J) P.J[2 * (int64_t)P.M * K + i] = J_ctrl;
    }
  }
  merge_box_quad(probs, active, b, c, lo, hi);
}

// Per sample: the state terms over the horizon (tracking error to the guide at
// (t+1) dt, speed, goal) and J_col, from the stored states and distances (or, with
// stored nearest indices, from the distance to the stored point, formed exactly as
// the exact distance pass forms it).  A spatially sorted set's distances are read
// by slot through the inverse permutation and written back to min_dist2 here.  A
// block holds kFinSamples consecutive samples; its threads take kFinWaves consecutive
// parts of the horizon (two per wave, so that the blocks spread over all CUs), and
// the parts' sums are added in order.  write_s1 = false leaves S1 alone (the adjoint
// needs the terms only).
constexpr int kFinSamples = 32;
constexpr int kFinWaves = 8;  // parts of the horizon per sample
constexpr int kFinThreads = kFinSamples * kFinWaves;  // two parts per wave

__global__ __launch_bounds__(kFinThreads) void k_finalize(const DevProblem* __restrict__ probs,
                                                             int n, int64_t total, DevParams prm,
                                                             int write_s1) {
  constexpr int kWaves = kFinWaves;
  constexpr int kTerms = 4;  // track, speed, goal, collision
  __shared__ double part[kWaves][kTerms][kFinSamples];
  // lane: the sample within the block; w: the part of the horizon
  const int lane = threadIdx.x % kFinSamples, w = threadIdx.x / kFinSamples;
  const int64_t gid = (int64_t)blockIdx.x * kFinSamples + lane;
  const bool active = gid < total;
  double s[kTerms] = {0.0, 0.0, 0.0, 0.0};
  const int b =
      active ? find_owner(probs, n, gid, [](const DevProblem& p) { return p.sample_base; }) : 0;
  load_weights(probs[b].w_dev, prm);
  if (active) {
    const DevProblem& P = probs[b];
    const int K = P.K, N = P.N;
    const int64_t local = gid - P.sample_base;
    const int m = (int)(local / K), k = (int)(local % K);
    const int64_t MNK = (int64_t)P.M * N * K;
    const int per = (N + kWaves - 1) / kWaves;
    const int t0 = min(N, w * per), t1 = min(N, t0 + per);
    const double pg[3] = {P.pg[0], P.pg[1], P.pg[2]}, vg[3] = {P.vg[0], P.vg[1], P.vg[2]};
    double Rg[9];
    load_rg(P.qg, Rg);
    double cf[3][6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int i = 0; i < 6; ++i) cf[a][i] = P.coef[(m * 3 + a) * 6 + i];
    // phi vanishes from d_max on; sqrt is correctly rounded and d_max^2 is exact in
    // binary64, so skipping d^2 >= d_max^2 changes no sum
    const double dmax2 = prm.d_max * prm.d_max;
    // the next step's state is loaded while this one is scored
    AERO_GLOBAL const float* __restrict__ state = global_ptr(P.state);
    float xn[10];
    auto load_state = [&](int t) {
      const int64_t qi = ((int64_t)m * N + (t < t1 ? t : t1 - 1)) * K + k;
      AERO_GLOBAL const fvec2* st = reinterpret_cast<AERO_GLOBAL const fvec2*>(state + qi * 10);
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        const fvec2 v = st[i];
        xn[2 * i] = v[0];
        xn[2 * i + 1] = v[1];
      }
    };
    // the descriptor's pointers in registers, as global pointers (see k_rollout): the
    // distance write-back could otherwise alias the descriptor, which would then be
    // reloaded at every step
    AERO_GLOBAL const int32_t* __restrict__ nidx_in = global_ptr(P.nidx_in);
    AERO_GLOBAL const int32_t* __restrict__ inv = global_ptr(P.inv);
    AERO_GLOBAL const unsigned* __restrict__ out_slot = global_ptr(P.out_slot);
    AERO_GLOBAL unsigned* __restrict__ mind2 = global_ptr(P.mind2);
    AERO_GLOBAL const float* __restrict__ pos = global_ptr(P.pos);
    AERO_GLOBAL const float* __restrict__ cloud = global_ptr(P.cloud);
    const int n_points = P.n_points;
    if (t0 < t1) load_state(t0);
    for (int t = t0; t < t1; ++t) {
      const int64_t row = (int64_t)m * N + t;
      double x[10];
#pragma unroll
      for (int i = 0; i < 10; ++i) x[i] = xn[i];
      load_state(t + 1);
      const double tau = (double)(t + 1) * prm.dt;
      double e2 = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double f = cf[a][5];
#pragma unroll
        for (int i = 4; i >= 0; --i) f = f * tau + cf[a][i];
        const double e = x[a] - f;
        e2 += e * e;
      }
      s[0] += sqrt(e2);
      s[1] += x[7] * x[7] + x[8] * x[8] + x[9] * x[9];
      s[2] += goal_term(x, pg, vg, Rg, prm);
      const int64_t qi = row * K + k;
      float d2;
      if (nidx_in) {
        const int idx = nidx_in[qi];
        if (idx < 0 || idx >= n_points) continue;
        const float ax = pos[qi] - cloud[3 * (int64_t)idx];
        const float ay = pos[MNK + qi] - cloud[3 * (int64_t)idx + 1];
        const float az = pos[2 * MNK + qi] - cloud[3 * (int64_t)idx + 2];
        d2 = fmaf(az, az, fmaf(ay, ay, ax * ax));
      } else if (inv) {
        // sorted set: the distance by slot, written back to the positions' layout
        // (the min_dist2 output) as it is read
        const int32_t sl = inv[qi];
        const unsigned bits = (sl >= 0 && sl < MNK) ? out_slot[sl] : kInfBits;
        mind2[qi] = bits;
        d2 = __uint_as_float(bits);
      } else {
        d2 = __uint_as_float(mind2[qi]);
      }
      if ((double)d2 < dmax2) s[3] += collision_phi(sqrt((double)d2), prm);
    }
  }
#pragma unroll
  for (int j = 0; j < kTerms; ++j) part[w][j][lane] = s[j];
  __syncthreads();
  if (w != 0 || !active) return;
  double tot[kTerms];
#pragma unroll
  for (int j = 0; j < kTerms; ++j) {
    tot[j] = part[0][j][lane];
#pragma unroll
    for (int v = 1; v < kWaves; ++v) tot[j] += part[v][j][lane];
  }
  const DevProblem& P = probs[b];
  const int K = P.K;
  const int64_t i = gid - P.sample_base;  // m * K + k
  const double J_track = prm.Q_track * tot[0];
  const double J_vnorm = prm.Q_vnorm * tot[1];
  const double J_goal = tot[2], col = tot[3];
  if (write_s1) {
    const double smooth =
        prm.w[0] * J_track + prm.w[1] * J_vnorm + prm.w[2] * P.J_ctrl[i] + prm.w[3] * J_goal;
    P.S1[i] = smooth + prm.w[4] * col;
  }
  if (P.J) {
    const int64_t MK = (int64_t)P.M * K;
    P.J[i] = J_track;
    P.J[MK + i] = J_vnorm;
    P.J[3 * MK + i] = J_goal;
    P.J[4 * MK + i] = col;
  }
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

// Per instance: rho = min_k S1_k, e_k = exp(-(S1_k - rho) / lambda) and eta = sum_k e_k
// (Sec. III-B, eq. (mppi_weights)), once, for every row of the update to read.  Thread
// t sums its samples t, t + kBlock, ... in order, then the block sums in a fixed
// order.
__global__ __launch_bounds__(kBlock) void k_weights(const DevProblem* __restrict__ probs, int n,
                                                    DevParams prm) {
  __shared__ double sh[20];
  const int64_t gid = blockIdx.x;
  const int b = find_owner(probs, n, gid, [](const DevProblem& p) { return p.inst_base; });
  const DevProblem& P = probs[b];
  const int K = P.K;
  const int m = (int)(gid - P.inst_base);
  const double* S = P.S1 + (int64_t)m * K;
  AERO_GLOBAL double* __restrict__ wexp = global_ptr(P.wexp) + (int64_t)m * K;
  double mn = INFINITY;
  for (int k = threadIdx.x; k < K; k += kBlock) mn = fmin(mn, S[k]);
  const double rho = block_min(mn, sh);
  const double inv_lam = 1.0 / prm.lambda;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < K; k += kBlock) {
    const double e = exp(-(S[k] - rho) * inv_lam);
    wexp[k] = e;
    acc[0] += e;
  }
  block_sum5(acc, sh);
  if (threadIdx.x == 0) P.eta[m] = acc[0];
}

// Per (instance, step) row: u_nom += sum_k e_k delta_eff_k / eta (Sec. III-B, eq.
// (mppi_update)), the samples summed per thread in order, then over the block.
__global__ __launch_bounds__(kBlock) void k_update(const DevProblem* __restrict__ probs, int n) {
  __shared__ double sh[20];
  const int64_t gid = blockIdx.x;
  const int b = find_owner(probs, n, gid, [](const DevProblem& p) { return p.row_base; });
  const DevProblem& P = probs[b];
  const int K = P.K, N = P.N;
  const int64_t row = gid - P.row_base;  // m * N + t
  const int m = (int)(row / N);
  const double* __restrict__ W = P.wexp + (int64_t)m * K;
  const float* __restrict__ D = P.deff + row * 4 * K;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < K; k += kBlock) {
    const double e = W[k];
    acc[1] += e * (double)D[k];
    acc[2] += e * (double)D[K + k];
    acc[3] += e * (double)D[2 * K + k];
    acc[4] += e * (double)D[3 * K + k];
  }
  block_sum5(acc, sh);
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    float* u = P.u_nom + row * 4 + c;
    *u = (float)((double)*u + acc[1 + c] / P.eta[m]);
  }
}

// Stage II noise-free rollouts, one per quad of lanes as in k_rollout.
__global__ __launch_bounds__(kBlock) void k_sel_rollout(const DevSelect* __restrict__ sel, int n,
                                                        int64_t total, DevParams prm,
                                                        PutBlob blob) {
  if (blob.n > 0) {  // descriptors in the argument (see put_blob)
    if (blockIdx.x == 0) put_blob(blob, (unsigned char*)sel);
    sel = reinterpret_cast<const DevSelect*>(blob.b);
  }
  const int64_t gid = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 2;  // instance
  if (gid >= total) return;  // whole quads
  const QuadLane L = quad_lane(threadIdx.x);
  const int c = L.c;
  const int b = find_owner(sel, n, gid, [](const DevSelect& p) { return p.inst_base; });
  const DevSelect& P = sel[b];
  const int m = (int)(gid - P.inst_base), N = P.N;
  const int64_t MN = (int64_t)P.M * N;
  const Dyn dyn{1.0 / prm.mass, prm.gravity};
  const bool pv = c < 3;  // lane 3 carries no position or velocity
  double p = P.x0[pv ? c : 0], v = P.x0[pv ? 7 + c : 7], q = P.x0[3 + c];
  double qa[4] = {P.x0[3], P.x0[4], P.x0[5], P.x0[6]};
  // global pointers in registers (see k_rollout)
  AERO_GLOBAL const float* __restrict__ u_nom = global_ptr(P.u_nom);
  AERO_GLOBAL double* __restrict__ state = global_ptr(P.state);
  AERO_GLOBAL float* __restrict__ pos = global_ptr(P.pos);
  AERO_GLOBAL unsigned* __restrict__ mind2 = global_ptr(P.mind2);
  // control channel c loaded kAhead steps ahead (see k_rollout)
  float ur[kAhead];  // as loaded (see k_rollout)
  auto fetch = [&](int t) { return u_nom[((int64_t)m * N + (t < N ? t : N - 1)) * 4 + c]; };
#pragma unroll
  for (int j = 0; j < kAhead; ++j) ur[j] = fetch(j);
  for (int t0 = 0; t0 < N; t0 += kAhead) {
#pragma unroll
    for (int j = 0; j < kAhead; ++j) {
      const int t = t0 + j;
      if (t >= N) break;
      const int64_t row = (int64_t)m * N + t;
      const double u = ur[j];
      ur[j] = fetch(t + kAhead);
      const QuadControl qc = quad_control(u, L, dyn);
      quad_rk4(p, v, q, qa, qc, L, prm.dt, dyn);
      // branch-free stores as in k_rollout (lane 3 repeats its own)
      AERO_GLOBAL double* rec = state + row * 10;
      AERO_GLOBAL unsigned* md = mind2 + (2 * c) * MN + row;
      md[0] = kInfBits;
      md[MN] = kInfBits;
      rec[3 + c] = q;
      rec[pv ? c : 6] = pv ? p : q;
      rec[pv ? 7 + c : 6] = pv ? v : q;
      *(pv ? reinterpret_cast<AERO_GLOBAL unsigned*>(pos + c * MN + row) : md) =
          pv ? __float_as_uint((float)p) : kInfBits;
    }
  }
}

// One block per problem: the goal and collision terms of every (instance, step),
// computed in parallel for a chunk of the horizon at a time into LDS, then added per
// instance in step order; S2 and the argmin (lowest index on ties).
constexpr int kSelTerms = 2048;  // (instance, step) terms per chunk
static_assert(AERO_M_MAX <= kBlock, "one thread per instance sums its terms");

__global__ __launch_bounds__(kBlock) void k_sel_final(const DevSelect* __restrict__ sel,
                                                      DevParams prm) {
  __shared__ double s2[AERO_M_MAX];
  __shared__ double term[2][kSelTerms];
  const DevSelect& P = sel[blockIdx.x];
  load_weights(P.w_dev, prm);
  const int M = P.M, N = P.N;
  const int64_t MN = (int64_t)M * N;
  const double pg[3] = {P.pg[0], P.pg[1], P.pg[2]}, vg[3] = {P.vg[0], P.vg[1], P.vg[2]};
  double Rg[9];
  load_rg(P.qg, Rg);
  const int tc = M >= kSelTerms ? 1 : kSelTerms / M;  // steps per chunk
  double goal = 0.0, col = 0.0;  // running sums of instance threadIdx.x (< M)
  for (int tb = 0; tb < N; tb += tc) {
    const int nt = min(tc, N - tb);
    for (int r = threadIdx.x; r < M * nt; r += kBlock) {
      const int m = r / nt, t = tb + r % nt;
      const int64_t row = (int64_t)m * N + t;
      double x[10];
#pragma unroll
      for (int i = 0; i < 10; ++i) x[i] = P.state[row * 10 + i];
      term[0][r] = goal_term(x, pg, vg, Rg, prm);
      unsigned bits = P.mind2[row];  // merge the distance copies
#pragma unroll
      for (int c = 1; c < kSelCopies; ++c) bits = min(bits, P.mind2[c * MN + row]);
      term[1][r] = collision_phi(sqrt((double)__uint_as_float(bits)), prm);
    }
    __syncthreads();
    if ((int)threadIdx.x < M)
      for (int j = 0; j < nt; ++j) {
        goal += term[0][threadIdx.x * nt + j];
        col += term[1][threadIdx.x * nt + j];
      }
    __syncthreads();
  }
  if ((int)threadIdx.x < M) {
    const double v = prm.w[3] * goal + prm.w[4] * col;
    s2[threadIdx.x] = v;
    P.S2[threadIdx.x] = v;
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

// The descriptors (h_blob, blob_bytes: the image of the workspace from d_probs on)
// travel in the noise launch when they fit in its argument, else by upload launches.
hipError_t launch_rollout_noise(const DevProblem* d_probs, int n, int64_t total_samples,
                                int64_t total_elems, const DevParams& prm, const QuerySet* d_sets,
                                int64_t box_blocks, const void* h_blob, size_t blob_bytes,
                                hipStream_t s) {
  const int64_t nb = (total_elems + kBlock - 1) / kBlock;
  PutBlob blob;
  blob.n = 0;
  blob.pad = 0;
  if (blob_bytes <= (size_t)kPutBytes && blob_bytes % 4 == 0 && nb + box_blocks > 0) {
    blob.n = (uint32_t)blob_bytes;
    memcpy(blob.b, h_blob, blob_bytes);
  } else {
    const hipError_t e = launch_put_bytes((void*)d_probs, h_blob, blob_bytes, s);
    if (e != hipSuccess) return e;
  }
  const int64_t sets_off = (const char*)d_sets - (const char*)d_probs;
  if (nb + box_blocks > 0)
    k_noise<<<(unsigned)(nb + box_blocks), kBlock, 0, s>>>(d_probs, n, total_elems, prm, d_sets, n,
                                                          nb, blob, sets_off);
  k_rollout<<<(unsigned)((4 * total_samples + kRollBlock - 1) / kRollBlock), kRollBlock, 0, s>>>(
      d_probs, n, total_samples, prm);
  return hipGetLastError();
}

hipError_t launch_rollout(const DevProblem* d_probs, int n, int64_t total, const DevParams& prm,
                          hipStream_t s) {
  k_rollout<<<(unsigned)((4 * total + kRollBlock - 1) / kRollBlock), kRollBlock, 0, s>>>(
      d_probs, n, total, prm);
  return hipGetLastError();
}

hipError_t launch_finalize(const DevProblem* d_probs, int n, int64_t total, const DevParams& prm,
                           bool write_s1, hipStream_t s) {
  if (total > 0)
    k_finalize<<<(unsigned)((total + kFinSamples - 1) / kFinSamples), kFinThreads, 0, s>>>(
        d_probs, n, total, prm, write_s1 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_update(const DevProblem* d_probs, int n, int64_t total_inst, int64_t total_rows,
                         const DevParams& prm, hipStream_t s) {
  if (total_inst <= 0) return hipSuccess;
  k_weights<<<(unsigned)total_inst, kBlock, 0, s>>>(d_probs, n, prm);
  k_update<<<(unsigned)total_rows, kBlock, 0, s>>>(d_probs, n);
  return hipGetLastError();
}

// The descriptors (h_blob, blob_bytes: the image of the workspace from d_sel on)
// travel in the rollout launch when they fit in its argument, else by upload launches.
hipError_t launch_select_rollout(const DevSelect* d_sel, int n, int64_t total_inst,
                                 const DevParams& prm, const void* h_blob, size_t blob_bytes,
                                 hipStream_t s) {
  PutBlob blob;
  blob.n = 0;
  blob.pad = 0;
  if (blob_bytes <= (size_t)kPutBytes && blob_bytes % 4 == 0 && total_inst > 0) {
    blob.n = (uint32_t)blob_bytes;
    memcpy(blob.b, h_blob, blob_bytes);
  } else {
    const hipError_t e = launch_put_bytes((void*)d_sel, h_blob, blob_bytes, s);
    if (e != hipSuccess) return e;
  }
  k_sel_rollout<<<grid1d(4 * total_inst), kBlock, 0, s>>>(d_sel, n, total_inst, prm, blob);
  return hipGetLastError();
}

hipError_t launch_select_final(const DevSelect* d_sel, int n, const DevParams& prm,
                               hipStream_t s) {
  k_sel_final<<<(unsigned)n, kBlock, 0, s>>>(d_sel, prm);
  return hipGetLastError();
}

}  // namespace aero
