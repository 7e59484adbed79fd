// Cloud accumulation into the drone-centred frame and the vehicle step of a
// closed loop (Sec. IV-A accumulates LiDAR frames; Sec. III-A/III-B model and RK4).
#include "aero_device.h"
#include "aero_internal.h"

namespace aero {

namespace {

// Frame of point i: the largest f with off[f] <= i, clamped to [0, F) so that
// unordered offsets still give an in-bounds frame.
__device__ __forceinline__ int frame_of(const int32_t* off, int F, int64_t i) {
  int lo = 0, hi = F - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One block writes kBlock consecutive output points.  Output point i belongs to
// frame f = frame_of(i) and is read from ring row start[f] + (i - off[f]), clamped
// into the ring, so inconsistent offsets give wrong values but never an access
// outside the ring or the output.  The block's 3*kBlock input floats (at most two
// contiguous runs per frame boundary) and its output floats move through LDS with
// unit stride; the per-frame rigid maps (binary64) are built once per block.
__global__ void __launch_bounds__(kBlock) k_accumulate_cloud(
    const float* __restrict__ ring, int64_t ring_points, const int32_t* __restrict__ start,
    const int32_t* __restrict__ offsets, int F, int64_t n_points,
    const float* __restrict__ poses, const float* __restrict__ origin, float* __restrict__ out) {
  __shared__ int32_t s_off[AERO_FRAMES_MAX + 1];
  __shared__ int32_t s_start[AERO_FRAMES_MAX];
  __shared__ double s_map[AERO_FRAMES_MAX][12];   // R row-major, then p
  __shared__ float s_pts[3 * kBlock];
  for (int f = threadIdx.x; f <= F; f += kBlock) s_off[f] = offsets[f];
  for (int f = threadIdx.x; f < F; f += kBlock) {
    s_start[f] = start[f];
    const float* ps = poses + 7 * f;
    double w = ps[3], x = ps[4], y = ps[5], z = ps[6];
    const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    w *= inv; x *= inv; y *= inv; z *= inv;
    double* m = s_map[f];
    rotmat(w, x, y, z, m);
    m[9] = ps[0];
    m[10] = ps[1];
    m[11] = ps[2];
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kBlock;
  const int64_t n_here = n_points - base < kBlock ? n_points - base : kBlock;
  const int nf = (int)(3 * n_here);
  for (int j = threadIdx.x; j < nf; j += kBlock) {
    const int64_t i = base + j / 3;
    const int f = frame_of(s_off, F, i);
    int64_t r = (int64_t)s_start[f] + (i - s_off[f]);
    r = r < 0 ? 0 : (r >= ring_points ? ring_points - 1 : r);
    s_pts[j] = ring[3 * r + j % 3];
  }
  __syncthreads();
  // each lane rewrites only the three LDS words of its own point
  if ((int64_t)threadIdx.x < n_here) {
    const int64_t i = base + threadIdx.x;
    const double* m = s_map[frame_of(s_off, F, i)];
    const double a = s_pts[3 * threadIdx.x], b = s_pts[3 * threadIdx.x + 1],
                 c = s_pts[3 * threadIdx.x + 2];
    s_pts[3 * threadIdx.x] = (float)((m[0] * a + m[1] * b + m[2] * c + m[9]) - (double)origin[0]);
    s_pts[3 * threadIdx.x + 1] =
        (float)((m[3] * a + m[4] * b + m[5] * c + m[10]) - (double)origin[1]);
    s_pts[3 * threadIdx.x + 2] =
        (float)((m[6] * a + m[7] * b + m[8] * c + m[11]) - (double)origin[2]);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nf; j += kBlock) out[3 * base + j] = s_pts[j];
}

__global__ void k_advance_state(const float* __restrict__ x0, const float* __restrict__ u, int M,
                                int N, const int32_t* __restrict__ index, DevParams prm,
                                float* __restrict__ x1) {
  if (threadIdx.x != 0) return;
  int i = index[0];
  i = i < 0 ? 0 : (i >= M ? M - 1 : i);
  double x[10], uc[4];
  for (int j = 0; j < 10; ++j) x[j] = x0[j];
  for (int c = 0; c < 4; ++c) uc[c] = u[(int64_t)i * N * 4 + c];
  const Dyn d{1.0 / prm.mass, prm.gravity};
  rk4(x, uc, prm.dt, d);
  for (int j = 0; j < 10; ++j) x1[j] = (float)x[j];
}

}  // namespace

hipError_t launch_accumulate_cloud(const float* ring, int64_t ring_points, const int32_t* start,
                                   const int32_t* offsets, int F, int64_t n_points,
                                   const float* poses, const float* origin, float* out,
                                   hipStream_t s) {
  const int64_t blocks = (n_points + kBlock - 1) / kBlock;
  k_accumulate_cloud<<<(unsigned)blocks, kBlock, 0, s>>>(ring, ring_points, start, offsets, F,
                                                          n_points, poses, origin, out);
  return hipGetLastError();
}

hipError_t launch_advance_state(const float* x0, const float* u, int M, int N,
                                const int32_t* index, const DevParams& prm, float* x1,
                                hipStream_t s) {
  k_advance_state<<<1, 64, 0, s>>>(x0, u, M, N, index, prm, x1);
  return hipGetLastError();
}

}  // namespace aero
