// Multi-resolution partition, coarse safe directions and anchors
// (Sec. IV-A, eqs. (unit direction), (safe-vector); Sec. IV-B-1/2, eq. (anchor-point)).
//
// Every integer output is decided by exact predicates: IEEE binary64 products and
// sums of float32 operands with contraction disabled, so the result does not
// depend on the order points are visited or on the initial atan2 guess.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "aero_device.h"
#include "aero_internal.h"

namespace aero {
namespace {

struct Grid {
  const float* az_b;  // [n_az][2] boundary (cos, sin)
  const float* el_b;  // [n_el+1][2]
  const float* az_c;  // [n_az][2] centres
  const float* el_c;  // [n_el][2]
  int n_az, n_el;
};

__device__ inline Grid make_grid(const float* tab, int n_az, int n_el) {
  Grid g;
  g.az_b = tab;
  g.el_b = tab + 2 * n_az;
  g.az_c = g.el_b + 2 * (n_el + 1);
  g.el_c = g.az_c + 2 * n_az;
  g.n_az = n_az;
  g.n_el = n_el;
  return g;
}

// (x, y) lies on or counter-clockwise of boundary i: c*y - s*x >= 0 (exact products).
__device__ inline bool az_on_or_after(const Grid& g, int i, double x, double y) {
#pragma clang fp contract(off)
  const double c = (double)g.az_b[2 * i], s = (double)g.az_b[2 * i + 1];
  const double a = c * y;
  const double b = s * x;
  return a - b >= 0.0;
}

// Direction at or above elevation boundary j: z cb >= sb |(x, y)|, compared on squares.
__device__ inline bool el_at_or_above(const Grid& g, int j, double x, double y, double z) {
#pragma clang fp contract(off)
  const double cb = (double)g.el_b[2 * j], sb = (double)g.el_b[2 * j + 1];
  const double zc = z * cb;
  const double A = zc * zc;
  const double xs = x * sb;
  const double ys = y * sb;
  const double xs2 = xs * xs;
  const double ys2 = ys * ys;
  const double B = xs2 + ys2;
  const bool up = z >= 0.0;
  return sb >= 0.0 ? (up && A >= B) : (up || A <= B);
}

__device__ inline int az_bin(const Grid& g, float xf, float yf) {
  if (xf == 0.0f && yf == 0.0f) return 0;
  const double x = xf, y = yf;
  const float ang = atan2f(yf, xf);
  int i = (int)floorf((ang + 3.14159265f) * (g.n_az * 0.159154943f));
  i = min(max(i, 0), g.n_az - 1);
  // Walk to the unique wedge: on/after boundary i and strictly before boundary i+1.
  for (int it = 0; it <= g.n_az; ++it) {
    const int inext = (i + 1 == g.n_az) ? 0 : i + 1;
    const bool lo = az_on_or_after(g, i, x, y);
    const bool hi = az_on_or_after(g, inext, x, y);
    if (lo && !hi) return i;
    i = lo ? inext : (i == 0 ? g.n_az - 1 : i - 1);
  }
  return i;  // unreachable for n_az >= 3
}

__device__ inline int el_bin(const Grid& g, float xf, float yf, float zf) {
  const double x = xf, y = yf, z = zf;
  const float el = atan2f(zf, sqrtf(xf * xf + yf * yf));
  int j = (int)floorf((el + 1.57079633f) * (g.n_el * 0.318309886f));
  j = min(max(j, 0), g.n_el - 1);
  // The predicate is monotone in j: climb while the next boundary holds, then
  // descend while the current one fails.  Band 0 needs no predicate.
  while (j + 1 <= g.n_el - 1 && el_at_or_above(g, j + 1, x, y, z)) ++j;
  while (j >= 1 && !el_at_or_above(g, j, x, y, z)) --j;
  return j;
}

__device__ inline double range_key(float xf, float yf, float zf) {
#pragma clang fp contract(off)
  const double x = xf, y = yf, z = zf;
  const double xx = x * x, yy = y * y, zz = z * z;
  const double s = xx + yy;
  return s + zz;
}

__global__ void k_part_init(unsigned long long* key, unsigned* idx, int n, unsigned long long init) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) {
    key[c] = init;
    idx[c] = 0xFFFFFFFFu;
  }
}

// Pass 1: per cone, the minimum r^2 (positive binary64 bit patterns order as integers).
// Consecutive points of a scan fall into few cones, so the lanes of a wave first
// combine their keys cone by cone (up to kConeRounds cones, one atomic each); lanes
// still left after that issue their own atomic.  The minimum is the same either way.
constexpr int kConeRounds = 8;

__device__ inline void part_key_block(const float* __restrict__ cloud, int n_points,
                                      const float* tab, int n_az, int n_el, double rmax2,
                                      unsigned long long* key, int blk) {
  const int p = blk * blockDim.x + threadIdx.x;
  bool pending = false;
  int c = 0;
  unsigned long long k = ~0ull;
  if (p < n_points) {
    const float x = cloud[3 * p], y = cloud[3 * p + 1], z = cloud[3 * p + 2];
    const double r2 = range_key(x, y, z);
    if (r2 > 0.0 && r2 <= rmax2) {
      const Grid g = make_grid(tab, n_az, n_el);
      c = el_bin(g, x, y, z) * n_az + az_bin(g, x, y);
      k = (unsigned long long)__double_as_longlong(r2);
      pending = true;
    }
  }
  const int lane = threadIdx.x & 63;
  for (int round = 0; round < kConeRounds; ++round) {  // every lane of the wave takes part
    const unsigned long long pm = __ballot(pending);
    if (pm == 0) break;
    const int leader = __ffsll((long long)pm) - 1;
    const int c0 = __shfl(c, leader, 64);
    const bool mine = pending && c == c0;
    unsigned long long m = mine ? k : ~0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long t = __shfl_xor(m, o, 64);
      m = t < m ? t : m;
    }
    if (lane == leader) atomicMin(key + c0, m);
    pending = pending && !mine;
  }
  if (pending) atomicMin(key + c, k);
}

__global__ void k_part_key(const float* __restrict__ cloud, int n_points, const float* tab,
                           int n_az, int n_el, double rmax2, unsigned long long* key) {
  part_key_block(cloud, n_points, tab, n_az, n_el, rmax2, key, blockIdx.x);
}

// Pass 2: the lowest point index attaining the cone minimum.
__device__ inline void part_idx_block(const float* __restrict__ cloud, int n_points,
                                      const float* tab, int n_az, int n_el, double rmax2,
                                      const unsigned long long* key, unsigned* idx, int blk) {
  const int p = blk * blockDim.x + threadIdx.x;
  if (p >= n_points) return;
  const float x = cloud[3 * p], y = cloud[3 * p + 1], z = cloud[3 * p + 2];
  const double r2 = range_key(x, y, z);
  if (!(r2 > 0.0) || r2 > rmax2) return;
  const Grid g = make_grid(tab, n_az, n_el);
  const int c = el_bin(g, x, y, z) * n_az + az_bin(g, x, y);
  if ((unsigned long long)__double_as_longlong(r2) == key[c]) atomicMin(idx + c, (unsigned)p);
}

// Coarse argmax (ties: lowest fine index) and the anchor block around the goal.
__device__ inline void coarse_anchor_block(const float* tab, int n_az_c, int n_el_c, int f_a,
                                           int f_e, const unsigned long long* key,
                                           int32_t* coarse_best, float gx, float gy, float gz,
                                           int M_h, int M_v, float ell, float p0x, float p0y,
                                           float p0z, int32_t* anchor_cell, int32_t* anchor_fine,
                                           float* anchors) {
  const int n_az = n_az_c * f_a, n_el = n_el_c * f_e;
  const int n_coarse = n_az_c * n_el_c;
  for (int C = threadIdx.x; C < n_coarse; C += blockDim.x) {
    const int I = C % n_az_c, J = C / n_az_c;
    unsigned long long best = 0;
    int bc = -1;
    for (int j = J * f_e; j < (J + 1) * f_e; ++j)
      for (int i = I * f_a; i < (I + 1) * f_a; ++i) {
        const int c = j * n_az + i;  // increasing c within the block
        const unsigned long long k = key[c];
        if (bc < 0 || k > best) {
          best = k;
          bc = c;
        }
      }
    coarse_best[C] = bc;
  }
  __syncthreads();
  __shared__ int goal_cell[2];
  if (threadIdx.x == 0) {
    float x = gx, y = gy, z = gz;
    if (x == 0.0f && y == 0.0f && z == 0.0f) x = 1.0f;
    const Grid g = make_grid(tab, n_az, n_el);
    goal_cell[0] = az_bin(g, x, y) / f_a;
    goal_cell[1] = el_bin(g, x, y, z) / f_e;
  }
  __syncthreads();
  const int M = M_h * M_v;
  const int Ig = goal_cell[0], Jg = goal_cell[1];
  int J0 = Jg - (M_v - 1) / 2;
  J0 = min(max(J0, 0), n_el_c - M_v);
  const Grid g = make_grid(tab, n_az, n_el);
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    const int oh = m % M_h, ov = m / M_h;
    int I = (Ig - (M_h - 1) / 2 + oh) % n_az_c;
    if (I < 0) I += n_az_c;
    const int J = J0 + ov;
    const int C = J * n_az_c + I;
    const int c = coarse_best[C];
    anchor_cell[m] = C;
    anchor_fine[m] = c;
    const int i = c % n_az, j = c / n_az;
    const float ca = g.az_c[2 * i], sa = g.az_c[2 * i + 1];
    const float cb = g.el_c[2 * j], sb = g.el_c[2 * j + 1];
    const double dx = (double)cb * ca, dy = (double)cb * sa, dz = sb;
    anchors[3 * m] = (float)(p0x + (double)ell * dx);
    anchors[3 * m + 1] = (float)(p0y + (double)ell * dy);
    anchors[3 * m + 2] = (float)(p0z + (double)ell * dz);
  }
}

// Pass 2 and the coarse step in one launch, since both read only the cone minima
// of pass 1: blocks below n_idx_blocks run pass 2, the last block the coarse argmax
// and the anchors.
__global__ __launch_bounds__(kBlock) void k_part_idx_anchor(
    const float* __restrict__ cloud, int n_points, const float* tab, int n_az_c, int n_el_c,
    int f_a, int f_e, double rmax2, const unsigned long long* key, unsigned* idx,
    int32_t* coarse_best, float gx, float gy, float gz, int M_h, int M_v, float ell, float p0x,
    float p0y, float p0z, int32_t* anchor_cell, int32_t* anchor_fine, float* anchors,
    int n_idx_blocks) {
  if ((int)blockIdx.x < n_idx_blocks) {  // block-uniform
    part_idx_block(cloud, n_points, tab, n_az_c * f_a, n_el_c * f_e, rmax2, key, idx, blockIdx.x);
    return;
  }
  coarse_anchor_block(tab, n_az_c, n_el_c, f_a, f_e, key, coarse_best, gx, gy, gz, M_h, M_v, ell,
                      p0x, p0y, p0z, anchor_cell, anchor_fine, anchors);
}

// Closed-form quintic of anchor m, axis ax: a0 = p0, a1 = v0, a2 = a0/2 and
// a3..a5 from the end conditions.
__device__ inline void guide_axis(const double p0[3], const double v0[3], const double a0[3],
                                  const float* anchors, const float* end_vel,
                                  const float* end_acc, double T, int m, int ax, float* coef) {
  const double pT = anchors[3 * m + ax];
  double vT, aT;
  if (end_vel) {
    vT = end_vel[3 * m + ax];
  } else {
    const double dx = (double)anchors[3 * m] - p0[0], dy = (double)anchors[3 * m + 1] - p0[1],
                 dz = (double)anchors[3 * m + 2] - p0[2];
    const double n = sqrt(dx * dx + dy * dy + dz * dz);
    const double sp = sqrt(v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2]);
    const double d[3] = {dx, dy, dz};
    vT = n > 0.0 ? sp * d[ax] / n : 0.0;
  }
  aT = end_acc ? (double)end_acc[3 * m + ax] : 0.0;
  const double T2 = T * T, T3 = T2 * T, T4 = T3 * T, T5 = T4 * T;
  const double dP = pT - (p0[ax] + v0[ax] * T + 0.5 * a0[ax] * T2);
  const double dV = (vT - v0[ax] - a0[ax] * T) * T;
  const double dA = (aT - a0[ax]) * T2;
  float* c = coef + (m * 3 + ax) * 6;
  c[0] = (float)p0[ax];
  c[1] = (float)v0[ax];
  c[2] = (float)(0.5 * a0[ax]);
  c[3] = (float)((10.0 * dP - 4.0 * dV + 0.5 * dA) / T3);
  c[4] = (float)((-15.0 * dP + 7.0 * dV - dA) / T4);
  c[5] = (float)((6.0 * dP - 3.0 * dV + 0.5 * dA) / T5);
}

__global__ void k_guides(double p0x, double p0y, double p0z, double v0x, double v0y, double v0z,
                         double a0x, double a0y, double a0z, const float* anchors,
                         const float* end_vel, const float* end_acc, double T, int M,
                         float* coef) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= M * 3) return;
  const double p0[3] = {p0x, p0y, p0z}, v0[3] = {v0x, v0y, v0z}, a0[3] = {a0x, a0y, a0z};
  guide_axis(p0, v0, a0, anchors, end_vel, end_acc, T, id / 3, id % 3, coef);
}

// ---------------------------------------------------------------------------
// Batched front end: the same passes for many problems in three launches, with the
// guides computed by the block that finds a problem's anchors.
// ---------------------------------------------------------------------------
__device__ inline const FrontJob& job_of_cell(const FrontJob* jobs, int n, int64_t gid) {
  return jobs[find_owner(jobs, n, gid, [](const FrontJob& j) { return j.cell_base; })];
}

__device__ inline double job_rmax2(const FrontJob& J) {
  return (double)J.r_max * (double)J.r_max;
}

__global__ __launch_bounds__(kBlock) void k_fe_init(FrontJob* jobs, int n, int64_t total_cells,
                                                    PutBlob blob) {
  const FrontJob* jr = jobs;
  if (blob.n > 0) {  // descriptors in the argument (see put_blob)
    if (blockIdx.x == 0) put_blob(blob, (unsigned char*)jobs);
    jr = reinterpret_cast<const FrontJob*>(blob.b);
  }
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= total_cells) return;
  const FrontJob& J = job_of_cell(jr, n, gid);
  const int64_t c = gid - J.cell_base;
  J.key[c] = (unsigned long long)__double_as_longlong(job_rmax2(J));
  J.idx[c] = 0xFFFFFFFFu;
}

__global__ __launch_bounds__(kBlock) void k_fe_key(const FrontJob* __restrict__ jobs, int n) {
  const int j = find_owner(jobs, n, (int64_t)blockIdx.x,
                           [](const FrontJob& q) { return q.block_base; });
  const FrontJob& J = jobs[j];
  part_key_block(J.cloud, J.n_points, J.tables, J.n_az_c * J.f_a, J.n_el_c * J.f_e, job_rmax2(J),
                 J.key, (int)(blockIdx.x - J.block_base));
}

// Blocks below total_blocks: pass 2 of their job; block total_blocks + j: job j's
// coarse argmax, anchors and guides.
__global__ __launch_bounds__(kBlock) void k_fe_idx_anchor(const FrontJob* __restrict__ jobs,
                                                          int n, int64_t total_blocks) {
  if ((int64_t)blockIdx.x < total_blocks) {  // block-uniform
    const int j = find_owner(jobs, n, (int64_t)blockIdx.x,
                             [](const FrontJob& q) { return q.block_base; });
    const FrontJob& J = jobs[j];
    part_idx_block(J.cloud, J.n_points, J.tables, J.n_az_c * J.f_a, J.n_el_c * J.f_e,
                   job_rmax2(J), J.key, J.idx, (int)(blockIdx.x - J.block_base));
    return;
  }
  const FrontJob J = jobs[blockIdx.x - total_blocks];  // a copy: the stores below cannot alias it
  coarse_anchor_block(J.tables, J.n_az_c, J.n_el_c, J.f_a, J.f_e, J.key, J.coarse_best,
                      J.goal[0], J.goal[1], J.goal[2], J.M_h, J.M_v, J.ell, J.p0[0], J.p0[1],
                      J.p0[2], J.anchor_cell, J.anchor_fine, J.anchors);
  __syncthreads();  // the anchors written above are read by other threads below
  const int M = J.M_h * J.M_v;
  const double p0[3] = {J.p0[0], J.p0[1], J.p0[2]}, v0[3] = {J.v0[0], J.v0[1], J.v0[2]},
               a0[3] = {J.a0[0], J.a0[1], J.a0[2]};
  for (int id = threadIdx.x; id < 3 * M; id += kBlock)
    guide_axis(p0, v0, a0, J.anchors, J.end_vel, J.end_acc, (double)J.T, id / 3, id % 3, J.coef);
}

// P_f: the closest point of every fine cone, in cone order, sentinel when empty.
__global__ void k_filter_cloud(const float* __restrict__ cloud, const int32_t* __restrict__ idx,
                               int n_fine, int n_points, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_fine) return;
  const int i = idx[c];
  if (n_points <= 0 || i < 0 || i >= n_points) {
    out[3 * c] = 1.0e18f;
    out[3 * c + 1] = 1.0e18f;
    out[3 * c + 2] = 1.0e18f;
    return;
  }
  out[3 * c] = cloud[3 * (int64_t)i];
  out[3 * c + 1] = cloud[3 * (int64_t)i + 1];
  out[3 * c + 2] = cloud[3 * (int64_t)i + 2];
}

}  // namespace

hipError_t launch_filter_cloud(const float* cloud, int n_points, const int32_t* fine_idx,
                               int n_fine, float* out, hipStream_t s) {
  k_filter_cloud<<<(n_fine + kBlock - 1) / kBlock, kBlock, 0, s>>>(
      n_points > 0 ? cloud : nullptr, fine_idx, n_fine, n_points, out);
  return hipGetLastError();
}

hipError_t launch_partition(const aero_partition_spec& spec, const float* cloud, int n_points,
                            const float goal[3], double* fine_key, int32_t* fine_idx,
                            int32_t* coarse_best, int32_t* anchor_cell, int32_t* anchor_fine,
                            float* anchors, hipStream_t s) {
  const int n_az = spec.n_az_c * spec.f_a, n_el = spec.n_el_c * spec.f_e;
  const int n_fine = n_az * n_el;
  const double rmax2 = (double)spec.r_max * (double)spec.r_max;
  auto* key = reinterpret_cast<unsigned long long*>(fine_key);
  auto* idx = reinterpret_cast<unsigned*>(fine_idx);
  k_part_init<<<(n_fine + kBlock - 1) / kBlock, kBlock, 0, s>>>(
      key, idx, n_fine, (unsigned long long)__builtin_bit_cast(long long, rmax2));
  const int nb = n_points > 0 ? (n_points + kBlock - 1) / kBlock : 0;
  if (nb > 0)
    k_part_key<<<nb, kBlock, 0, s>>>(cloud, n_points, spec.d_tables, n_az, n_el, rmax2, key);
  k_part_idx_anchor<<<nb + 1, kBlock, 0, s>>>(
      cloud, n_points, spec.d_tables, spec.n_az_c, spec.n_el_c, spec.f_a, spec.f_e, rmax2, key,
      idx, coarse_best, goal[0], goal[1], goal[2], spec.M_h, spec.M_v, spec.ell, spec.p0[0],
      spec.p0[1], spec.p0[2], anchor_cell, anchor_fine, anchors, nb);
  return hipGetLastError();
}

hipError_t launch_front_end(FrontJob* d_jobs, const FrontJob* h_jobs, int n, int64_t total_cells,
                            int64_t total_blocks, hipStream_t s) {
  const size_t bytes = (size_t)n * sizeof(FrontJob);
  PutBlob blob;
  blob.n = 0;
  blob.pad = 0;
  if (bytes <= (size_t)kPutBytes && total_cells > 0) {
    blob.n = (uint32_t)bytes;
    memcpy(blob.b, h_jobs, bytes);
  } else {
    const hipError_t e = launch_put_bytes(d_jobs, h_jobs, bytes, s);
    if (e != hipSuccess) return e;
  }
  if (total_cells > 0)
    k_fe_init<<<(unsigned)((total_cells + kBlock - 1) / kBlock), kBlock, 0, s>>>(d_jobs, n,
                                                                               total_cells, blob);
  if (total_blocks > 0) k_fe_key<<<(unsigned)total_blocks, kBlock, 0, s>>>(d_jobs, n);
  k_fe_idx_anchor<<<(unsigned)(total_blocks + n), kBlock, 0, s>>>(d_jobs, n, total_blocks);
  return hipGetLastError();
}

hipError_t launch_guides(const double p0[3], const double v0[3], const double a0[3],
                         const float* anchors, const float* end_vel, const float* end_acc,
                         double T, int M, float* coef, hipStream_t s) {
  const int n = 3 * M;
  k_guides<<<(n + 63) / 64, 64, 0, s>>>(p0[0], p0[1], p0[2], v0[0], v0[1], v0[2], a0[0], a0[1],
                                        a0[2], anchors, end_vel, end_acc, T, M, coef);
  return hipGetLastError();
}

}  // namespace aero
