/*
 * aero.h - C ABI of the AERO-MPPI planning-step library for AMD MI355X (gfx950).
 *
 * One planning step of the anchor-guided MPPI ensemble (Chen et al., "AERO-MPPI:
 * Anchor-Guided Ensemble Trajectory Optimization for Agile Mapless Drone
 * Navigation"):
 *
 *   aero_partition_anchors   Sec. IV-A (multi-resolution partition) and
 *                            Sec. IV-B-1/2 (anchor sampling and refinement)
 *   aero_build_guides        Sec. IV-B-3, eq. (polynomial): quintic guides
 *   aero_mppi_step           Sec. III-B eqs. (mppi_rollout), (mppi_weights),
 *                            (mppi_update) with the Stage-I cost of Sec. IV-C
 *   aero_select_best         Sec. IV-C, Stage II: explicit rollouts, S2, argmin
 *   aero_mppi_step_backward  gradient of the summed Stage-I cost with respect to
 *                            the nominal controls and the five term weights
 *
 * Conventions shared by every call
 *   - Pointers named d_* are device pointers (gfx950 global memory) owned by the
 *     caller; h_* pointers are host memory read during the call only.  The
 *     library never keeps or frees a caller pointer after the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *     device work is enqueued asynchronously on it; outputs are valid once the
 *     stream has reached the end of the call's work.
 *   - Arguments are validated on the host before anything is enqueued.  On any
 *     error the call returns a nonzero aero_status, enqueues nothing and leaves
 *     every output untouched.  Non-finite values inside device buffers are not
 *     checked (behaviour undefined).
 *   - Frame: the cloud is given relative to the drone (world axes, z up); the
 *     state, goal and anchors are expressed in the same frame.
 *   - Calls on different streams are re-entrant; calls that share an output
 *     buffer must be ordered by the caller.
 */
#ifndef AERO_H
#define AERO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum aero_status {
  AERO_OK = 0,
  AERO_ERR_NULL = 1,      /* a required pointer is NULL                         */
  AERO_ERR_SHAPE = 2,     /* a size is out of range (see each call)             */
  AERO_ERR_PARAM = 3,     /* a parameter is non-finite or outside its domain    */
  AERO_ERR_WORKSPACE = 4, /* workspace NULL or smaller than the size query      */
  AERO_ERR_DEVICE = 5     /* the HIP runtime reported an error on enqueue       */
} aero_status;

#define AERO_N_MAX 512        /* longest horizon N                                */
#define AERO_M_MAX 256        /* most MPPI instances per problem                  */
#define AERO_K_MAX (1 << 20)  /* most samples per instance                        */
#define AERO_BATCH_MAX 2048   /* most problems per call                           */
#define AERO_GRID_MAX 8192    /* most fine cells along one angular axis           */
#define AERO_FRAMES_MAX 256   /* most LiDAR frames per accumulated cloud          */
#define AERO_POSITIONS_MAX 2147483647LL /* rollout positions M*N*K of one problem and  *
                                         * their sum over one call stay below this     */
#define AERO_NOALLOC_SCRATCH_BYTES (32u << 20) /* device scratch of                  *
                                         * aero_select_best_noalloc, per GPU             */
#define AERO_NOALLOC_BATCH_MAX 16 /* most problems per aero_select_best_noalloc call  */

/* Table I parameters shared by all problems of a call (float32 values). */
typedef struct aero_params {
  float dt;           /* RK4 step [s] (> 0)                                        */
  float lambda;       /* temperature of eq. (mppi_weights) (> 0)                   */
  float mass;         /* m [kg] (> 0)                                              */
  float gravity;      /* |g| [m/s^2], g = (0, 0, -gravity)                         */
  float sigma[4];     /* noise std per channel (F_t, wx, wy, wz) (>= 0)            */
  float u_min[4];     /* control box, u_min <= u_max per channel                   */
  float u_max[4];
  float Q_track, Q_vnorm, Q_c, Q_cdelta, Q_p, Q_v, Q_q;  /* term weights (scalars) */
  float C;            /* collision scale (>= 0)                                    */
  float a;            /* collision slope (>= 0)                                    */
  float d_min, d_max; /* 0 <= d_min < d_max                                        */
  float w[5];         /* multipliers of (J_track, J_vnorm, J_ctrl, J_goal, J_col)  */
  uint64_t seed;      /* noise key: Philox key = (seed_lo, seed_hi ^ problem_id)   */
  uint32_t iter_base; /* noise counter word 3 (the MPPI iteration index)           */
  uint32_t reserved;  /* must be 0                                                 */
} aero_params;

/* One planning problem (host struct; device pointers inside). */
typedef struct aero_problem {
  const float* cloud;   /* device [n_points][3] float32, collision set              */
  int32_t n_points;     /* >= 0 (0 = no obstacles)                                  */
  int32_t M;            /* instances, 1..AERO_M_MAX                                 */
  int32_t K;            /* samples per instance, 1..AERO_K_MAX                      */
  int32_t N;            /* horizon, 2..AERO_N_MAX                                   */
  uint32_t problem_id;  /* mixed into the noise key                                 */
  float x0[10];         /* p (3), q (w, x, y, z), v (3); |q| > 0                    */
  float p_goal[3], v_goal[3], q_goal[4];
  const float* coef;    /* device [M][3][6] guide coefficients a_{i,mu} (Stage I)   */
  float* u_nom;         /* device [M][N][4] nominal controls; updated in place      */
  double* S1;           /* optional device [M][K]: Stage-I cost of every sample     */
  float* delta_eff;     /* optional device [M][N][4][K]: clipped perturbations      */
  float* min_dist2;     /* optional device [M][N][K]: squared nearest distance; exact  *
                         * wherever it is below d_max^2, elsewhere only a value known *
                         * to be >= d_max^2                                           */
  int32_t* nearest_idx; /* optional device [M][N][K]: written by aero_mppi_step and    *
                         * aero_mppi_step_backward, read by                           *
                         * aero_mppi_step_backward_indexed: the nearest cloud point   *
                         * (lowest index on ties) of every position closer than      *
                         * d_max; -1 or an index of a point at least d_max away       *
                         * elsewhere                                                  */
  const float* w;       /* optional device [5]: the term multipliers of this problem   *
                         * (track, vnorm, ctrl, goal, col), read on the device in     *
                         * place of h_prm->w (NULL: use h_prm->w)                     */
} aero_problem;

/* Angular grid of the multi-resolution partition (Sec. IV-A). */
typedef struct aero_partition_spec {
  int32_t n_az_c, n_el_c;  /* coarse cells in azimuth / elevation (>= 1)            */
  int32_t f_a, f_e;        /* pooling factors: fine grid (n_az_c f_a) x (n_el_c f_e) */
  int32_t M_h, M_v;        /* anchor block, 1 <= M_h <= n_az_c, 1 <= M_v <= n_el_c   */
  float r_max;             /* perception range (> 0)                                 */
  float ell;               /* look-ahead distance of the anchors                     */
  float p0[3];             /* drone position in the frame of the anchors             */
  const float* d_tables;   /* device copy of aero_partition_tables() for this grid   */
} aero_partition_spec;

/* ---- host helpers ------------------------------------------------------------ */

/* Number of floats in the direction tables of an n_az x n_el fine grid. */
size_t aero_partition_tables_size(int32_t n_az, int32_t n_el);

/* Fill h_out (aero_partition_tables_size floats, host) with the float32 tables
 * the partition is decided on (Sec. IV-A, eq. (unit direction)):
 *   [0, 2 n_az)            (cos, sin) of azimuth boundaries -pi + 2 pi i / n_az
 *   [.., + 2 (n_el + 1))   (cos, sin) of elevation boundaries -pi/2 + pi j / n_el
 *   [.., + 2 n_az)         (cos, sin) of azimuth cell centres
 *   [.., + 2 n_el)         (cos, sin) of elevation cell centres
 * Angles are formed in binary64 and rounded to float32 after cos/sin.
 * Errors: AERO_ERR_NULL, AERO_ERR_SHAPE (n_az < 3, n_el < 1, either > AERO_GRID_MAX,
 * or n_floats too small).  Host only; touches no device. */
int aero_partition_tables(int32_t n_az, int32_t n_el, float* h_out, size_t n_floats);

/* Which call a workspace is for. */
typedef enum aero_call {
  AERO_CALL_MPPI_STEP = 0,
  AERO_CALL_SELECT_BEST = 1,
  AERO_CALL_BACKWARD = 2
} aero_call;

/* Bytes of device workspace the given call needs for these problems (0 on a
 * NULL or invalid argument).  Pure host arithmetic. */
size_t aero_workspace_size(int which_call, const aero_problem* h_problems, int32_t n_problems);

/* Human-readable text of a status code (static storage). */
const char* aero_status_string(int status);

/* ---- the planning step ---------------------------------------------------------- */

/* Multi-resolution partition and anchors (Sec. IV-A eqs. (unit direction),
 * (safe-vector); Sec. IV-B-1/2 eq. (anchor-point)).
 *   d_cloud       [n_points][3] float32, relative to the drone
 *   h_goal_dir    [3] goal direction (zero vector = +x heading)
 *   d_fine_key    [n_el_f * n_az_f] float64: min r^2 per cone (r_max^2 if empty),
 *                 flat index c = j * n_az_f + i (i azimuth, j elevation)
 *   d_fine_idx    [n_el_f * n_az_f] int32: lowest point index attaining it, -1 if empty
 *   d_coarse_best [n_el_c * n_az_c] int32: fine index of the max-range cone of each
 *                 coarse cell (ties: lowest c), coarse flat index J * n_az_c + I
 *   d_anchor_cell [M_h * M_v] int32 coarse cell of anchor m = o_v * M_h + o_h
 *   d_anchor_fine [M_h * M_v] int32 fine cone of anchor m
 *   d_anchors     [M_h * M_v][3] float32: p0 + ell * d(anchor cone)
 * Integer outputs are decided by exact binary64 predicates on the float32 tables,
 * so they are reproducible bit for bit.
 * Errors: AERO_ERR_NULL, AERO_ERR_SHAPE (grid or block out of range, n_points < 0),
 * AERO_ERR_PARAM (r_max <= 0 or non-finite inputs), AERO_ERR_DEVICE. */
int aero_partition_anchors(const aero_partition_spec* h_spec, const float* d_cloud,
                           int32_t n_points, const float* h_goal_dir, double* d_fine_key,
                           int32_t* d_fine_idx, int32_t* d_coarse_best, int32_t* d_anchor_cell,
                           int32_t* d_anchor_fine, float* d_anchors, void* stream);

/* One problem of a batched front end: the partition of aero_partition_anchors and the
 * guides of aero_build_guides (end conditions as there), for one cloud. */
typedef struct aero_front_end_job {
  aero_partition_spec spec;  /* grid, anchor block, r_max, ell, p0 (also the guides' start
                                position) and the device direction tables                */
  const float* d_cloud;      /* [n_points][3] float32, relative to the drone             */
  int32_t n_points;
  float goal_dir[3];         /* zero vector = +x heading                                  */
  float v0[3], a0[3];        /* the guides' start velocity and acceleration              */
  float horizon_T;           /* the guides' horizon                                       */
  const float* d_end_vel;    /* [M][3] or NULL: |v0| unit(anchor - p0)                    */
  const float* d_end_acc;    /* [M][3] or NULL: 0                                         */
  double* d_fine_key;        /* outputs, as aero_partition_anchors and aero_build_guides  */
  int32_t* d_fine_idx;
  int32_t* d_coarse_best;
  int32_t* d_anchor_cell;
  int32_t* d_anchor_fine;
  float* d_anchors;
  float* d_coef;             /* [M][3][6]                                                 */
} aero_front_end_job;

/* Device workspace of aero_front_end for n_jobs problems (0 for n_jobs out of range). */
size_t aero_front_end_workspace_size(int32_t n_jobs);

/* Partition, anchors and guides of n_jobs problems in three launches (Sec. IV-A,
 * Sec. IV-B, as aero_partition_anchors followed by aero_build_guides for each job;
 * bit for bit the same outputs).  Jobs may differ in grid, cloud and anchor block.
 *   h_jobs  host array [n_jobs], read during the call only
 *   d_ws    device workspace of aero_front_end_workspace_size(n_jobs) bytes
 * Errors: AERO_ERR_NULL, AERO_ERR_SHAPE (n_jobs outside [1, AERO_BATCH_MAX], or a job
 * as aero_partition_anchors / aero_build_guides reject it), AERO_ERR_PARAM,
 * AERO_ERR_WORKSPACE, AERO_ERR_DEVICE; checked for every job before any launch. */
int aero_front_end(const aero_front_end_job* h_jobs, int32_t n_jobs, void* d_ws, size_t ws_bytes,
                   void* stream);

/* Filtered collision set P_f of the collision cost (Sec. IV-C: the closest point of
 * every fine cone of the partition).  out[c] = cloud[fine_idx[c]] in cone order
 * c = 0 .. n_fine-1; a cone without a point holds the sentinel (1e18, 1e18, 1e18),
 * which is never the nearest point of any position, so P_f can be passed to
 * aero_mppi_step / aero_select_best as a cloud of exactly n_fine points.
 *   d_cloud     [n_points][3] float32 (the cloud the partition was built on)
 *   d_fine_idx  [n_fine] int32 from aero_partition_anchors (-1 = empty cone)
 *   d_out       [n_fine][3] float32
 * Errors: AERO_ERR_NULL, AERO_ERR_SHAPE (n_fine < 1, n_points < 0), AERO_ERR_DEVICE. */
int aero_filtered_cloud(const float* d_cloud, int32_t n_points, const int32_t* d_fine_idx,
                        int32_t n_fine, float* d_out, void* stream);

/* Quintic guides (Sec. IV-B-3, eq. (polynomial)): per anchor m and axis mu, the six
 * coefficients of f(t) = sum_i a_i t^i on [0, T] meeting position, velocity and
 * acceleration at both ends.  Start (h_p0, h_v0, h_a0) (host [3] each); end
 * (d_anchors[m], end velocity, end acceleration).  d_end_vel / d_end_acc (device
 * [M][3]) may be NULL: end velocity |v0| * unit(anchor - p0), end acceleration 0.
 *   d_coef [M][3][6] float32 output.
 * Errors: AERO_ERR_NULL, AERO_ERR_SHAPE (M < 1 or > AERO_M_MAX), AERO_ERR_PARAM
 * (horizon_T <= 0 or non-finite), AERO_ERR_DEVICE. */
int aero_build_guides(const float* h_p0, const float* h_v0, const float* h_a0,
                      const float* d_anchors, const float* d_end_vel, const float* d_end_acc,
                      float horizon_T, int32_t M, float* d_coef, void* stream);

/* One Stage-I MPPI iteration for every instance of every problem (Sec. III-B,
 * Sec. IV-C): Philox noise, clipped controls, RK4 rollouts, S1 (J_col from the
 * nearest distance to the raw cloud, exact wherever it is below d_max; a position
 * with no point within d_max, where the penalty is 0, reports a distance of at least
 * d_max), softmax weights and the update of u_nom (in place).  Problems may differ in cloud size, M, K and N; n_problems > 1 runs
 * them in one batched launch sequence.
 *   h_problems  host array [n_problems]
 *   d_ws        device workspace of aero_workspace_size(AERO_CALL_MPPI_STEP, ...)
 * Errors: AERO_ERR_NULL, AERO_ERR_SHAPE (a size outside its range, or M*N*K of a
 * problem or its sum over the call at AERO_POSITIONS_MAX or above: positions are
 * addressed with 32-bit slots), AERO_ERR_PARAM (lambda <= 0, dt <= 0,
 * mass <= 0, sigma < 0, u_min > u_max, d_min >= d_max, non-finite values),
 * AERO_ERR_WORKSPACE, AERO_ERR_DEVICE. */
int aero_mppi_step(const aero_params* h_prm, const aero_problem* h_problems,
                   int32_t n_problems, void* d_ws, size_t ws_bytes, void* stream);

/* Stage II (Sec. IV-C): roll out each instance's u_nom without noise, score it with
 * S2 = w_goal J_goal + w_col J_col and pick the lowest (ties: lowest m).  J_col reads
 * the exact nearest distance wherever it is below d_max (cloud tiles farther than
 * d_max from a group of positions are skipped: the penalty is 0 there).
 *   d_S2    [sum_b M_b] float64, problems concatenated
 *   d_best  [n_problems] int32
 * coef, S1, delta_eff and min_dist2 of the problems are ignored.
 * Errors: as aero_mppi_step. */
int aero_select_best(const aero_params* h_prm, const aero_problem* h_problems,
                     int32_t n_problems, double* d_S2, int32_t* d_best, void* d_ws,
                     size_t ws_bytes, void* stream);

/* aero_select_best without a workspace argument, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same kernels and outputs as aero_select_best (bit for bit);
 * the workspace is a library-internal device array of AERO_NOALLOC_SCRATCH_BYTES
 * (32 MiB) that every GPU the call runs on holds from its first call until the
 * process ends (looked up on the current device, which must own `stream`).  The call
 * allocates nothing and records no timing events.
 * Limits: at most AERO_NOALLOC_BATCH_MAX problems, and the workspace that
 * aero_workspace_size(AERO_CALL_SELECT_BEST, ...) reports for them at most
 * AERO_NOALLOC_SCRATCH_BYTES (about 124 bytes per Stage-II position M*N, so one
 * problem of AERO_M_MAX x AERO_N_MAX fits).
 * Every call on one GPU uses the same array: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * Errors: as aero_select_best; AERO_ERR_SHAPE for more than AERO_NOALLOC_BATCH_MAX
 * problems, AERO_ERR_WORKSPACE when the problems need more than the array holds
 * (both checked on the host before any device work). */
int aero_select_best_noalloc(const aero_params* h_prm, const aero_problem* h_problems,
                             int32_t n_problems, double* d_S2, int32_t* d_best, void* stream);

/* Adjoint of L = g * sum_{m,k} S1[m,k] for one problem, evaluated at the
 * problem's u_nom (read only) with the same noise as aero_mppi_step:
 *   d_grad_L     device float32 scalar g, the upstream gradient (read on the
 *                device, so that an autograd caller needs no host copy; NULL
 *                means g = 1)
 *   d_grad_u_nom [M][N][4] float32 = dL/du_nom (zero where the sample was clipped)
 *   d_grad_w     [5] float32       = dL/dw = g * sum_{m,k} J_i
 * The weights are h_problem->w when given (device memory), else h_prm->w.
 * The derivative is the exact one of the active smooth piece: clip mask, collision
 * branch and nearest point (lowest index on ties) held fixed.  Rollout states are
 * checkpointed every 8 steps and recomputed.  The distance filter pass uses the
 * variant already settled for this shape by aero_mppi_step (else variant 0); the
 * gradients do not depend on it.
 * Errors: as aero_mppi_step. */
int aero_mppi_step_backward(const aero_params* h_prm, const aero_problem* h_problem,
                            const float* d_grad_L, float* d_grad_u_nom, float* d_grad_w,
                            void* d_ws, size_t ws_bytes, void* stream);

/* The same adjoint from nearest indices stored by a previous aero_mppi_step on the
 * same problem (same u_nom, cloud, guides and parameters; the step's in-place update of
 * u_nom must be undone or have been made on a copy): h_problem->nearest_idx is read,
 * not written, and no distance pass runs (the collision terms use the stored point).
 * Gradients equal those of aero_mppi_step_backward bit for bit when the indices came
 * from that step.  Workspace: aero_workspace_size(AERO_CALL_BACKWARD, ...).
 * Errors: as aero_mppi_step_backward; AERO_ERR_NULL if nearest_idx is null. */
int aero_mppi_step_backward_indexed(const aero_params* h_prm, const aero_problem* h_problem,
                                    const float* d_grad_L, float* d_grad_u_nom,
                                    float* d_grad_w, void* d_ws, size_t ws_bytes,
                                    void* stream);

/* ---- receding horizon ----------------------------------------------------------- */

/* Warm start for the next planning step (receding-horizon execution, Sec. III-B):
 * dst[m][t][c] = src[i][min(t + shift, N - 1)][c] for every m < M_dst, where
 * i = *d_index clamped to [0, M_src) (d_index is device memory, e.g. the d_best
 * output of aero_select_best, so no host synchronisation is needed).
 *   d_src [M_src][N][4], d_dst [M_dst][N][4] float32 (must not overlap)
 * Errors: AERO_ERR_NULL, AERO_ERR_SHAPE (M_src, M_dst < 1, N < 1, shift < 0),
 * AERO_ERR_DEVICE. */
int aero_shift_controls(const float* d_src, int32_t M_src, int32_t N, const int32_t* d_index,
                        int32_t shift, float* d_dst, int32_t M_dst, void* stream);

/* Candidates of a gradient step on one control sequence (adjoint refinement of
 * the selected plan; scored afterwards with aero_select_best):
 *   out[0] = u,  out[i] = clip(u - s_i g / max|g|, u_min, u_max),
 *   s_i = s0 beta^(i-1), i = 1 .. n_candidates-1 (g = 0 gives copies of u).
 *   d_u, d_g [N][4]; d_out [n_candidates][N][4]; clip box from h_prm.
 * Errors: AERO_ERR_NULL, AERO_ERR_SHAPE (N < 1, n_candidates < 1 or > AERO_M_MAX),
 * AERO_ERR_PARAM (s0 or beta non-finite or negative), AERO_ERR_DEVICE. */
int aero_step_candidates(const aero_params* h_prm, const float* d_u, const float* d_g, int32_t N,
                         float s0, float beta, int32_t n_candidates, float* d_out, void* stream);

/* ---- closed loop: cloud accumulation and the vehicle step ----------------------- */

/* Accumulated cloud in the drone-centred frame (Sec. IV-A builds the planner's
 * cloud from several recent LiDAR frames; the partition reads it with world axes
 * and the origin at the current position).  Frames sit in a ring of recorded
 * points; frame f has n_f = offsets[f+1] - offsets[f] points from ring row
 * start[f] on, in that frame's sensor coordinates.  Output rows
 * offsets[f] .. offsets[f+1]-1 receive them in order, mapped as
 *   out = (R(q_f / |q_f|) x + p_f) - origin,
 * evaluated in binary64 and rounded once to float32.
 *   d_ring            [ring_points][3] float32
 *   d_frame_start     [n_frames] int32 ring row of each frame's first point
 *   d_frame_offsets   [n_frames + 1] int32, non-decreasing from 0; offsets[n_frames]
 *                     should equal n_points
 *   d_poses           [n_frames][7] float32: p_f (world), then q_f (w, x, y, z),
 *                     sensor to world, non-zero
 *   d_origin          [3] float32 world position of the drone (e.g. p of its state)
 *   d_out             [n_points][3] float32, must not overlap the ring
 * All device memory, owned by the caller.  Starts and offsets are not validated on
 * the host: inconsistent ones give wrong points, but every read is clamped into the
 * ring and exactly n_points rows are written.
 * Errors: AERO_ERR_NULL, AERO_ERR_SHAPE (n_frames < 1 or > AERO_FRAMES_MAX,
 * n_points < 0, ring_points < 0, or ring_points = 0 with n_points > 0),
 * AERO_ERR_DEVICE.  n_points = 0 enqueues nothing. */
int aero_accumulate_cloud(const float* d_ring, int32_t ring_points, const int32_t* d_frame_start,
                          const int32_t* d_frame_offsets, int32_t n_frames, int32_t n_points,
                          const float* d_poses, const float* d_origin, float* d_out,
                          void* stream);

/* One control period of the vehicle under the first control of the executed plan
 * (Sec. III-A model, Sec. III-B RK4 step with the control held and the quaternion
 * renormalised):  x1 = RK4(x0, u[i][0], dt),  i = *d_index clamped to [0, M).
 *   d_x0, d_x1 [10] float32 (may alias), d_u [M][N][4] float32, d_index int32 (device,
 *   e.g. the d_best output of aero_select_best); dt, mass, gravity from h_prm.
 * Errors: as aero_step_candidates' parameter checks; AERO_ERR_NULL, AERO_ERR_SHAPE
 * (M < 1 or > AERO_M_MAX, N < 1), AERO_ERR_DEVICE. */
int aero_advance_state(const aero_params* h_prm, const float* d_x0, const float* d_u, int32_t M,
                       int32_t N, const int32_t* d_index, float* d_x1, void* stream);

/* ---- kernel-variant selection --------------------------------------------------- */

/* The nearest distance d_t of the collision cost (Sec. IV-C) only matters below d_max
 * (the penalty is zero from there on).  Each call therefore cuts the rollout
 * positions into spatially sorted blocks, lists for every block the cloud sub-tiles
 * (256 consecutive points, in the given order or in a Morton order of the cloud)
 * whose bounding box lies within reach of the block's box (the cull step), runs a
 * cheap approximate first pass over those pairs only, and an exact second pass over
 * the positions the first pass finds near the cloud.  The first pass has three
 * implementations: 0 = VALU FMAs on blocks of 2048 positions, 1 = half-precision
 * matrix cores on hi/lo-split coordinates with blocks of 512 positions, 2 = the same
 * with blocks of 1024.  By default (-1) the library autotunes per call shape (sum of
 * M N K, sum of cloud sizes, problem count) over five launch configurations (variant
 * 0 on 1024 persistent workgroups, variants 1 and 2 on 4096 and on 1024): the first
 * five calls of a shape each time one configuration with HIP events on the call's
 * stream, a later call keeps the fastest for that shape.  Costs, controls and selections are bitwise identical for
 * every variant, with or without the cull step; only min_dist2 and nearest_idx
 * entries beyond d_max may differ.  While the stream is being captured into a graph
 * an unsettled shape uses variant 0 and records nothing.
 * aero_set_pass_a_variant forces a variant for all later calls (-1 = autotune);
 * errors: AERO_ERR_PARAM for other values. */
int aero_set_pass_a_variant(int variant);

/* The variant in use for this call shape: 0, 1 or 2, or -1 while still being tuned. */
int aero_pass_a_variant(const aero_problem* h_problems, int32_t n_problems);
/* The persistent workgroups the tuner settled on for pass A at the shape of these
 * problems (it times each variant at two grid sizes, 1024 and 4096 workgroups for
 * the matrix-core variants), the forced variant's default grid, or -1 while the shape
 * is not settled. */
int aero_pass_a_grid(const aero_problem* h_problems, int32_t n_problems);

/* on = 1 (default): the cull step lists only the sub-tiles within reach of each block;
 * on = 0: every sub-tile of every block (the two passes become brute force over the
 * whole cloud; for tests and measurements).  Applies to later calls.  Errors:
 * AERO_ERR_PARAM for other values. */
int aero_set_pass_a_cull(int on);

/* Profiling aid: the work of the two distance passes of the last aero_mppi_step on
 * this workspace (same problems), counted from the cull step's items, pass A's hit
 * words and, for pass_b_eval, by a counting kernel that takes pass B's own work
 * units and group masks (launched on the null stream; the call synchronizes the
 * device).  Reads device memory synchronously: call it once the stream has finished
 * the step and before any other call reuses the workspace (aero_select_best on the
 * same workspace overwrites what it reads).  Errors: AERO_ERR_NULL, AERO_ERR_SHAPE /
 * AERO_ERR_PARAM as aero_mppi_step's size checks, AERO_ERR_WORKSPACE, AERO_ERR_DEVICE. */
typedef struct aero_distance_stats {
  int64_t items;        /* (query block, cloud sub-tile) items the cull step listed      */
  int64_t pairs_a;      /* position-point pairs of those items (pass A evaluates them)   */
  int64_t items_b;      /* items in which some query came under its block's bound        */
  int64_t pairs_b;      /* position-point pairs of pass A's hit words (the listed
                           queries against their items' whole sub-tiles)                 */
  int64_t items_whole;  /* marked items without room for their hit words (pass B takes
                           every query of the block)                                     */
  int64_t positions;    /* rollout positions of the two-pass sets                        */
  int64_t pairs_b_eval; /* position-point pairs pass B evaluates exactly: each listed
                           query against the point groups within its cap                 */
  int64_t pairs_a_eval; /* position-point pairs pass A evaluates: the matrix-core variants
                           skip, per wave, the 32-point groups beyond reach of the wave's
                           positions (the VALU variant: pairs_a)                         */
  int64_t pairs_a_products; /* pairs of the matrix-core products pass A runs (32 points x
                           32 positions each, padding included; VALU: pairs_a)            */
} aero_distance_stats;
int aero_read_distance_stats(const aero_problem* h_problems, int32_t n_problems, const void* d_ws,
                             size_t ws_bytes, aero_distance_stats* h_out);

/* ---- per-kernel timing (profiling aid) ---------------------------------------- */

/* Kernel identifiers for aero_timing_read. */
typedef enum aero_kernel {
  AERO_K_PARTITION = 0,    /* the three partition/anchor kernels of one call        */
  AERO_K_GUIDES = 1,
  AERO_K_ROLLOUT = 2,      /* Stage-I noise (+ cloud tile boxes and the call's
                              descriptors) and RK4 rollout                         */
  AERO_K_MIN_DIST = 3,     /* Stage-I nearest distance, pass A (the listed pairs)    */
  AERO_K_FINALIZE = 4,     /* Stage-I state terms, J_col and S1 (and the write-back
                              of a sorted set's distances to the positions' order) */
  AERO_K_UPDATE = 5,       /* softmax weights and control update                    */
  AERO_K_SEL_ROLLOUT = 6,  /* Stage-II rollout (+ the call's descriptors)           */
  AERO_K_SEL_MIN_DIST = 7, /* Stage-II nearest distance                             */
  AERO_K_SEL_FINAL = 8,    /* Stage-II S2 and argmin                                */
  AERO_K_FLAG = 9,         /* (retired: the exact pass needs no compaction step;
                              reads 0)                                               */
  AERO_K_MIN_DIST_EXACT = 10, /* Stage-I nearest distance, pass B (the hit pairs)   */
  AERO_K_NEAREST = 11,     /* backward: nearest indices of flagged positions         */
  AERO_K_ADJOINT = 12,     /* backward: per-sample reverse sweep                     */
  AERO_K_GRAD_REDUCE = 13, /* backward: sums over samples                            */
  AERO_K_SORT = 14,        /* Stage-I spatial sort of the positions and the cloud
                              (six kernels)                                          */
  AERO_K_CULL = 15,        /* Stage-I cull step (sorted-cloud boxes, block lists)    */
  AERO_K_COUNT = 16
} aero_kernel;

/* on != 0: from now on every launch of the kernels above is bracketed by two HIP
 * events recorded on the launch's own stream (adds a few microseconds per launch);
 * on == 0 stops recording.  Returns AERO_OK. */
int aero_timing_enable(int on);

/* Total event-measured milliseconds and number of launches recorded for `kernel`
 * since the last reset; waits for the recorded events.  reset != 0 clears all
 * counters afterwards.  Errors: AERO_ERR_NULL, AERO_ERR_SHAPE (unknown kernel),
 * AERO_ERR_DEVICE. */
int aero_timing_read(int kernel, double* h_total_ms, int64_t* h_launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* AERO_H */
