"""AERO-MPPI planning step on AMD MI355X: thin Python binding of libaero.so.

Every function here only marshals arguments (tensor pointers, the current HIP
stream, host structs) into the C ABI declared in include/aero.h; all
arithmetic of the planning step runs in the library's HIP kernels.  Importing
the package fails loudly if the library has not been built.
"""
import ctypes
import os

import numpy as np
# torch ships its own HIP runtime under the same soname as the system one; it must
# be mapped before libaero.so so that the library binds to it.  Loading the library
# first maps a second HIP/HSA runtime into the process, and the two then drive the
# same device (kernel launches fail, later calls crash).
import torch  # noqa: F401

__all__ = [
    "AeroError", "lib", "params_struct", "Problem", "partition_tables", "partition_anchors",
    "build_guides", "filtered_cloud", "workspace_size", "mppi_step", "select_best", "mppi_step_backward",
    "CALL_MPPI_STEP", "CALL_SELECT_BEST", "CALL_BACKWARD", "timing_enable", "timing_read",
    "KERNELS", "shift_controls", "step_candidates", "set_pass_a_variant", "pass_a_variant",
    "set_pass_a_cull", "distance_stats", "pass_a_grid", "FrontEndJob", "front_end_job", "front_end",
    "front_end_workspace_size",
    "use_library", "accumulate_cloud", "advance_state", "mppi_step_backward_indexed",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaero.so")

CALL_MPPI_STEP, CALL_SELECT_BEST, CALL_BACKWARD = 0, 1, 2


class AeroError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.aero_status_string(status).decode() if _lib else str(status)
        super().__init__(f"{where}: {msg}")


class Params(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_float), ("lambda_", ctypes.c_float), ("mass", ctypes.c_float),
        ("gravity", ctypes.c_float), ("sigma", ctypes.c_float * 4),
        ("u_min", ctypes.c_float * 4), ("u_max", ctypes.c_float * 4),
        ("Q_track", ctypes.c_float), ("Q_vnorm", ctypes.c_float), ("Q_c", ctypes.c_float),
        ("Q_cdelta", ctypes.c_float), ("Q_p", ctypes.c_float), ("Q_v", ctypes.c_float),
        ("Q_q", ctypes.c_float), ("C", ctypes.c_float), ("a", ctypes.c_float),
        ("d_min", ctypes.c_float), ("d_max", ctypes.c_float), ("w", ctypes.c_float * 5),
        ("seed", ctypes.c_uint64), ("iter_base", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
    ]


class ProblemStruct(ctypes.Structure):
    _fields_ = [
        ("cloud", ctypes.c_void_p), ("n_points", ctypes.c_int32), ("M", ctypes.c_int32),
        ("K", ctypes.c_int32), ("N", ctypes.c_int32), ("problem_id", ctypes.c_uint32),
        ("x0", ctypes.c_float * 10), ("p_goal", ctypes.c_float * 3),
        ("v_goal", ctypes.c_float * 3), ("q_goal", ctypes.c_float * 4),
        ("coef", ctypes.c_void_p), ("u_nom", ctypes.c_void_p), ("S1", ctypes.c_void_p),
        ("delta_eff", ctypes.c_void_p), ("min_dist2", ctypes.c_void_p),
        ("nearest_idx", ctypes.c_void_p), ("w", ctypes.c_void_p),
    ]


class PartitionSpec(ctypes.Structure):
    _fields_ = [
        ("n_az_c", ctypes.c_int32), ("n_el_c", ctypes.c_int32), ("f_a", ctypes.c_int32),
        ("f_e", ctypes.c_int32), ("M_h", ctypes.c_int32), ("M_v", ctypes.c_int32),
        ("r_max", ctypes.c_float), ("ell", ctypes.c_float), ("p0", ctypes.c_float * 3),
        ("d_tables", ctypes.c_void_p),
    ]


_P = ctypes.c_void_p


class FrontEndJob(ctypes.Structure):
    _fields_ = [
        ("spec", PartitionSpec), ("d_cloud", _P), ("n_points", ctypes.c_int32),
        ("goal_dir", ctypes.c_float * 3), ("v0", ctypes.c_float * 3), ("a0", ctypes.c_float * 3),
        ("horizon_T", ctypes.c_float), ("d_end_vel", _P), ("d_end_acc", _P),
        ("d_fine_key", _P), ("d_fine_idx", _P), ("d_coarse_best", _P), ("d_anchor_cell", _P),
        ("d_anchor_fine", _P), ("d_anchors", _P), ("d_coef", _P),
    ]


_SIGS = {
    "aero_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "aero_partition_tables_size": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "aero_partition_tables": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_size_t]),
    "aero_workspace_size": (ctypes.c_size_t, [ctypes.c_int, _P, ctypes.c_int32]),
    "aero_partition_anchors": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P,
                                              _P]),
    "aero_build_guides": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_int32,
                                         _P, _P]),
    "aero_front_end_workspace_size": (ctypes.c_size_t, [ctypes.c_int32]),
    "aero_front_end": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_size_t, _P]),
    "aero_mppi_step": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.c_size_t, _P]),
    "aero_select_best": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P, ctypes.c_size_t, _P]),
    "aero_select_best_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P]),
    "aero_mppi_step_backward": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "aero_mppi_step_backward_indexed": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, ctypes.c_size_t,
                                                       _P]),
    "aero_timing_enable": (ctypes.c_int, [ctypes.c_int]),
    "aero_set_pass_a_variant": (ctypes.c_int, [ctypes.c_int]),
    "aero_set_pass_a_cull": (ctypes.c_int, [ctypes.c_int]),
    "aero_read_distance_stats": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_size_t, _P]),
    "aero_shift_controls": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32,
                                           _P, ctypes.c_int32, _P]),
    "aero_step_candidates": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_int32, _P, _P]),
    "aero_pass_a_variant": (ctypes.c_int, [_P, ctypes.c_int32]),
    "aero_pass_a_grid": (ctypes.c_int, [_P, ctypes.c_int32]),
    "aero_accumulate_cloud": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32,
                                             ctypes.c_int32, _P, _P, _P, _P]),
    "aero_advance_state": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]),
    "aero_filtered_cloud": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P, _P]),
    "aero_timing_read": (ctypes.c_int, [ctypes.c_int, _P, _P, ctypes.c_int]),
}

KERNELS = ("partition", "guides", "rollout", "min_dist", "finalize", "update", "sel_rollout",
           "sel_min_dist", "sel_final", "flag", "min_dist_exact", "nearest", "adjoint",
           "grad_reduce", "sort", "cull")


def _load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_2509_17340_amd/build.py`")
    lib_ = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib_, name)
        fn.restype = res
        fn.argtypes = args
    return lib_


_lib = _load()


def lib():
    return _lib


def use_library(path):
    """Load another build of libaero.so (for example a tuning variant) for all calls."""
    global _lib
    _lib = _load(path)
    return _lib


def _check(status, where):
    if status != 0:
        raise AeroError(status, where)


def _ptr(t):
    """Device (or host) address of a tensor / array, an explicit integer address, or
    None.  Anything else (a Python float such as an upstream gradient given by value)
    is refused: it would otherwise become a bogus address that a kernel dereferences."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    if isinstance(t, (int, np.integer)) and not isinstance(t, (bool, np.bool_)):
        return int(t)
    raise TypeError(f"expected a tensor, an array, an address or None, got {type(t).__name__}")


_DT = {"f32": "torch.float32", "f64": "torch.float64", "i32": "torch.int32", "u8": "torch.uint8"}


def _need(t, numel, kind, name):
    """Host check that a device tensor can hold what the kernels will touch:
    contiguous, of the expected element type and with at least `numel` elements."""
    if t is None:
        return
    if not hasattr(t, "data_ptr") or not hasattr(t, "is_contiguous"):
        return
    if str(t.dtype) != _DT[kind]:
        raise TypeError(f"{name}: expected {_DT[kind]}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, the call needs {numel}")
    if getattr(t, "is_cuda", True) is False:
        raise ValueError(f"{name}: must be a device tensor (the kernels read it on the GPU)")


def _need_device_scalar(g):
    """The upstream gradient of a backward call: None (= 1) or a device float32 tensor
    holding at least one element (the kernels read it on the device)."""
    if g is None:
        return
    if not hasattr(g, "data_ptr"):
        raise TypeError(f"grad_L must be None or a device float32 tensor, got {type(g).__name__}")
    _need(g, 1, "f32", "grad_L")


def _stream(stream=None):
    if stream is not None:
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    import torch
    if torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


def params_struct(prm):
    """aero_params from a dict with the keys of fixtures.table1_params."""
    p = Params()
    p.dt, p.lambda_, p.mass, p.gravity = prm["dt"], prm["lam"], prm["mass"], prm["gravity"]
    for c in range(4):
        p.sigma[c], p.u_min[c], p.u_max[c] = prm["sigma"][c], prm["u_min"][c], prm["u_max"][c]
    for k in ("Q_track", "Q_vnorm", "Q_c", "Q_cdelta", "Q_p", "Q_v", "Q_q", "C", "a", "d_min",
              "d_max"):
        setattr(p, k, float(prm[k]))
    for i in range(5):
        p.w[i] = float(prm["w"][i])
    p.seed = int(prm.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
    p.iter_base = int(prm.get("iter_base", 0))
    p.reserved = 0
    return p


class Problem:
    """One planning problem: device tensors plus host scalars (see aero_problem)."""

    def __init__(self, cloud, M, K, N, x0, p_goal, u_nom, coef=None, v_goal=(0, 0, 0),
                 q_goal=(1, 0, 0, 0), S1=None, delta_eff=None, min_dist2=None, problem_id=0,
                 n_points=None, nearest_idx=None, w=None):
        self.cloud, self.M, self.K, self.N = cloud, int(M), int(K), int(N)
        self.n_points = int(cloud.shape[0]) if n_points is None else int(n_points)
        self.x0 = np.asarray(x0, np.float32)
        self.p_goal = np.asarray(p_goal, np.float32)
        self.v_goal = np.asarray(v_goal, np.float32)
        self.q_goal = np.asarray(q_goal, np.float32)
        self.u_nom, self.coef = u_nom, coef
        self.S1, self.delta_eff, self.min_dist2 = S1, delta_eff, min_dist2
        self.nearest_idx = nearest_idx
        self.w = w  # optional device [5] term weights (replace the call's params["w"])
        self.problem_id = int(problem_id)

    def check(self):
        M, K, N = self.M, self.K, self.N
        _need(self.cloud, 3 * self.n_points, "f32", "cloud")
        _need(self.u_nom, M * N * 4, "f32", "u_nom")
        _need(self.coef, M * 18, "f32", "coef")
        _need(self.S1, M * K, "f64", "S1")
        _need(self.delta_eff, M * N * 4 * K, "f32", "delta_eff")
        _need(self.min_dist2, M * N * K, "f32", "min_dist2")
        _need(self.nearest_idx, M * N * K, "i32", "nearest_idx")
        _need(self.w, 5, "f32", "w")

    def struct(self):
        self.check()
        s = ProblemStruct()
        s.cloud = _ptr(self.cloud) if self.n_points > 0 else None
        s.n_points, s.M, s.K, s.N = self.n_points, self.M, self.K, self.N
        s.problem_id = self.problem_id
        s.x0[:] = [float(v) for v in self.x0]
        s.p_goal[:] = [float(v) for v in self.p_goal]
        s.v_goal[:] = [float(v) for v in self.v_goal]
        s.q_goal[:] = [float(v) for v in self.q_goal]
        s.coef, s.u_nom = _ptr(self.coef), _ptr(self.u_nom)
        s.S1, s.delta_eff, s.min_dist2 = _ptr(self.S1), _ptr(self.delta_eff), _ptr(self.min_dist2)
        s.nearest_idx = _ptr(self.nearest_idx)
        s.w = _ptr(self.w)
        return s


def _problem_array(problems):
    arr = (ProblemStruct * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = p.struct()
    return arr


def partition_tables(n_az, n_el):
    n = _lib.aero_partition_tables_size(n_az, n_el)
    out = np.zeros(max(int(n), 1), np.float32)
    _check(_lib.aero_partition_tables(n_az, n_el, out.ctypes.data, out.size), "aero_partition_tables")
    return out


def partition_anchors(n_az_c, n_el_c, f_a, f_e, M_h, M_v, r_max, ell, p0, d_tables, cloud,
                      goal_dir, fine_key, fine_idx, coarse_best, anchor_cell, anchor_fine, anchors,
                      n_points=None, stream=None):
    spec = PartitionSpec()
    spec.n_az_c, spec.n_el_c, spec.f_a, spec.f_e = n_az_c, n_el_c, f_a, f_e
    spec.M_h, spec.M_v, spec.r_max, spec.ell = M_h, M_v, float(r_max), float(ell)
    spec.p0[:] = [float(v) for v in p0]
    spec.d_tables = _ptr(d_tables)
    g = np.ascontiguousarray(goal_dir, np.float32)
    n = int(cloud.shape[0]) if n_points is None else int(n_points)
    _check(_lib.aero_partition_anchors(
        ctypes.byref(spec), _ptr(cloud) if n > 0 else None, n, g.ctypes.data, _ptr(fine_key),
        _ptr(fine_idx), _ptr(coarse_best), _ptr(anchor_cell), _ptr(anchor_fine), _ptr(anchors),
        _stream(stream)), "aero_partition_anchors")


def filtered_cloud(cloud, fine_idx, out, n_points=None, stream=None):
    """P_f (closest point of every fine cone, cone order, sentinel for empty cones)."""
    n = int(cloud.shape[0]) if n_points is None else int(n_points)
    _check(_lib.aero_filtered_cloud(_ptr(cloud) if n > 0 else None, n, _ptr(fine_idx),
                                    int(fine_idx.shape[0]), _ptr(out), _stream(stream)),
           "aero_filtered_cloud")


def build_guides(p0, v0, a0, anchors, horizon_T, M, coef, end_vel=None, end_acc=None,
                 stream=None):
    p0 = np.ascontiguousarray(p0, np.float32)
    v0 = np.ascontiguousarray(v0, np.float32)
    a0 = np.ascontiguousarray(a0, np.float32)
    _check(_lib.aero_build_guides(p0.ctypes.data, v0.ctypes.data, a0.ctypes.data, _ptr(anchors),
                                  _ptr(end_vel), _ptr(end_acc), float(horizon_T), int(M),
                                  _ptr(coef), _stream(stream)), "aero_build_guides")


def front_end_job(n_az_c, n_el_c, f_a, f_e, M_h, M_v, r_max, ell, p0, d_tables, cloud, goal_dir,
                  v0, a0, horizon_T, fine_key, fine_idx, coarse_best, anchor_cell, anchor_fine,
                  anchors, coef, end_vel=None, end_acc=None, n_points=None):
    """One aero_front_end_job: the arguments of partition_anchors and build_guides
    (the guides start at p0, the partition's origin)."""
    j = FrontEndJob()
    sp = j.spec
    sp.n_az_c, sp.n_el_c, sp.f_a, sp.f_e = n_az_c, n_el_c, f_a, f_e
    sp.M_h, sp.M_v, sp.r_max, sp.ell = M_h, M_v, float(r_max), float(ell)
    sp.p0[:] = [float(v) for v in p0]
    sp.d_tables = _ptr(d_tables)
    n = int(cloud.shape[0]) if n_points is None else int(n_points)
    j.d_cloud = _ptr(cloud) if n > 0 else None
    j.n_points = n
    j.goal_dir[:] = [float(v) for v in goal_dir]
    j.v0[:] = [float(v) for v in v0]
    j.a0[:] = [float(v) for v in a0]
    j.horizon_T = float(horizon_T)
    j.d_end_vel, j.d_end_acc = _ptr(end_vel), _ptr(end_acc)
    j.d_fine_key, j.d_fine_idx = _ptr(fine_key), _ptr(fine_idx)
    j.d_coarse_best, j.d_anchor_cell = _ptr(coarse_best), _ptr(anchor_cell)
    j.d_anchor_fine, j.d_anchors, j.d_coef = _ptr(anchor_fine), _ptr(anchors), _ptr(coef)
    return j


def front_end_workspace_size(n_jobs):
    return int(_lib.aero_front_end_workspace_size(int(n_jobs)))


def front_end(jobs, ws, ws_bytes=None, stream=None):
    """Partition, anchors and guides of all jobs (FrontEndJob list) in three launches."""
    arr = (FrontEndJob * max(len(jobs), 1))(*jobs)
    nbytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.aero_front_end(ctypes.cast(arr, ctypes.c_void_p), len(jobs), _ptr(ws), nbytes,
                               _stream(stream)), "aero_front_end")


def workspace_size(which, problems):
    arr = _problem_array(problems)
    return int(_lib.aero_workspace_size(which, ctypes.cast(arr, ctypes.c_void_p), len(problems)))


def mppi_step(prm, problems, ws, ws_bytes=None, stream=None):
    p = params_struct(prm) if isinstance(prm, dict) else prm
    arr = _problem_array(problems)
    nbytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.aero_mppi_step(ctypes.byref(p), ctypes.cast(arr, ctypes.c_void_p), len(problems),
                               _ptr(ws), nbytes, _stream(stream)), "aero_mppi_step")


def select_best(prm, problems, S2, best, ws, ws_bytes=None, stream=None):
    p = params_struct(prm) if isinstance(prm, dict) else prm
    arr = _problem_array(problems)
    nbytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.aero_select_best(ctypes.byref(p), ctypes.cast(arr, ctypes.c_void_p), len(problems),
                                 _ptr(S2), _ptr(best), _ptr(ws), nbytes, _stream(stream)),
           "aero_select_best")


def select_best_noalloc(prm, problems, S2, best, stream=None):
    """Stage II without a workspace (the library's per-GPU scratch array; see
    aero_select_best_noalloc: calls that overlap on one GPU race)."""
    p = params_struct(prm) if isinstance(prm, dict) else prm
    arr = _problem_array(problems)
    _need(S2, sum(q.M for q in problems), "f64", "S2")
    _need(best, len(problems), "i32", "best")
    _check(_lib.aero_select_best_noalloc(ctypes.byref(p), ctypes.cast(arr, ctypes.c_void_p),
                                         len(problems), _ptr(S2), _ptr(best), _stream(stream)),
           "aero_select_best_noalloc")


def shift_controls(src, index, shift, dst, stream=None):
    """dst[m] = src[index][t + shift] (last control held); index is a device int32."""
    M_src, N = int(src.shape[0]), int(src.shape[1])
    _need(src, M_src * N * 4, "f32", "src")
    _need(index, 1, "i32", "index")
    _need(dst, int(dst.shape[0]) * N * 4, "f32", "dst")
    _check(_lib.aero_shift_controls(_ptr(src), M_src, N, _ptr(index), int(shift), _ptr(dst),
                                    int(dst.shape[0]), _stream(stream)), "aero_shift_controls")


def step_candidates(prm, u, g, s0, beta, out, stream=None):
    """out[0] = u, out[i] = clip(u - s0 beta^(i-1) g / max|g|)."""
    p = params_struct(prm) if isinstance(prm, dict) else prm
    N = int(u.shape[-2])
    _need(u, N * 4, "f32", "u")
    _need(g, N * 4, "f32", "g")
    _need(out, int(out.shape[0]) * N * 4, "f32", "out")
    _check(_lib.aero_step_candidates(ctypes.byref(p), _ptr(u), _ptr(g), int(u.shape[-2]),
                                     float(s0), float(beta), int(out.shape[0]), _ptr(out),
                                     _stream(stream)), "aero_step_candidates")


def accumulate_cloud(ring, frame_start, frame_offsets, poses, origin, out, n_points=None,
                     stream=None):
    """out rows offsets[f]..offsets[f+1] = (R(q_f) x + p_f) - origin for the points of
    frame f read from ring rows start[f].. (see aero_accumulate_cloud).

    ring (R, 3) float32, frame_start (F,) int32, frame_offsets (F+1,) int32,
    poses (F, 7) float32, origin (>= 3,) float32, out (>= n_points, 3) float32 --
    all device tensors; n_points defaults to out's row count."""
    R, F = int(ring.shape[0]), int(poses.shape[0])
    P = int(out.shape[0]) if n_points is None else int(n_points)
    _need(ring, 3 * R, "f32", "ring")
    _need(out, 3 * P, "f32", "out")
    _need(frame_start, F, "i32", "frame_start")
    _need(frame_offsets, F + 1, "i32", "frame_offsets")
    _need(poses, 7 * F, "f32", "poses")
    _need(origin, 3, "f32", "origin")
    _check(_lib.aero_accumulate_cloud(_ptr(ring), R, _ptr(frame_start), _ptr(frame_offsets), F, P,
                                      _ptr(poses), _ptr(origin), _ptr(out), _stream(stream)),
           "aero_accumulate_cloud")


def advance_state(prm, x0, u, index, x1, stream=None):
    """x1 = RK4(x0, u[index][0], dt) (see aero_advance_state); u (M, N, 4)."""
    p = params_struct(prm) if isinstance(prm, dict) else prm
    M, N = int(u.shape[0]), int(u.shape[1])
    _need(x0, 10, "f32", "x0")
    _need(x1, 10, "f32", "x1")
    _need(u, M * N * 4, "f32", "u")
    _need(index, 1, "i32", "index")
    _check(_lib.aero_advance_state(ctypes.byref(p), _ptr(x0), _ptr(u), M, N, _ptr(index), _ptr(x1),
                                   _stream(stream)), "aero_advance_state")


def set_pass_a_variant(variant):
    """Force the first distance pass: 0 = VALU (2048-position blocks), 1 = split-FP16
    matrix cores (512-position blocks), 2 = split-FP16 matrix cores (1024-position
    blocks), -1 = autotune (default)."""
    _check(_lib.aero_set_pass_a_variant(int(variant)), "aero_set_pass_a_variant")


def set_pass_a_cull(on=True):
    """Cull step on (default) or off (every block against the whole cloud)."""
    _check(_lib.aero_set_pass_a_cull(1 if on else 0), "aero_set_pass_a_cull")


class DistanceStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("items", "pairs_a", "items_b", "pairs_b",
                                              "items_whole", "positions", "pairs_b_eval",
                                              "pairs_a_eval", "pairs_a_products")]


def distance_stats(problems, ws, ws_bytes=None):
    """Work of the two distance passes of the last mppi_step on `ws` (synchronous):
    dict with items, pairs_a, items_b, pairs_b, items_whole, positions, pairs_b_eval,
    pairs_a_eval, pairs_a_products."""
    arr = _problem_array(problems)
    out = DistanceStats()
    nbytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.aero_read_distance_stats(ctypes.cast(arr, ctypes.c_void_p), len(problems), _ptr(ws),
                                    nbytes, ctypes.byref(out)), "aero_read_distance_stats")
    return {k: getattr(out, k) for k, _ in DistanceStats._fields_}


def pass_a_variant(problems):
    arr = _problem_array(problems)
    return int(_lib.aero_pass_a_variant(ctypes.cast(arr, ctypes.c_void_p), len(problems)))


def pass_a_grid(problems):
    """Persistent workgroups of the settled pass-A configuration (-1 while tuning)."""
    arr = _problem_array(problems)
    return int(_lib.aero_pass_a_grid(ctypes.cast(arr, ctypes.c_void_p), len(problems)))


def timing_enable(on=True):
    _check(_lib.aero_timing_enable(1 if on else 0), "aero_timing_enable")


def timing_read(reset=False):
    """{kernel name: (total ms, launches)} from the library's event timers."""
    out = {}
    for i, name in enumerate(KERNELS):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        last = reset and i == len(KERNELS) - 1
        _check(_lib.aero_timing_read(i, ctypes.byref(ms), ctypes.byref(n), 1 if last else 0),
               "aero_timing_read")
        out[name] = (ms.value, n.value)
    return out


def mppi_step_backward(prm, problem, grad_L, grad_u_nom, grad_w, ws, ws_bytes=None,
                       stream=None):
    """Adjoint of L = g * sum S1 (see aero_mppi_step_backward); grad_L is the device
    float32 scalar g, or None for g = 1."""
    p = params_struct(prm) if isinstance(prm, dict) else prm
    s = problem.struct()
    _need_device_scalar(grad_L)
    _need(grad_u_nom, problem.M * problem.N * 4, "f32", "grad_u_nom")
    _need(grad_w, 5, "f32", "grad_w")
    nbytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.aero_mppi_step_backward(ctypes.byref(p), ctypes.byref(s), _ptr(grad_L),
                                        _ptr(grad_u_nom), _ptr(grad_w), _ptr(ws), nbytes,
                                        _stream(stream)), "aero_mppi_step_backward")


def mppi_step_backward_indexed(prm, problem, grad_L, grad_u_nom, grad_w, ws, ws_bytes=None,
                               stream=None):
    """Adjoint from the nearest indices a previous mppi_step stored in
    problem.nearest_idx (read here); see aero_mppi_step_backward_indexed.  grad_L is
    the device float32 scalar upstream gradient, or None for 1."""
    p = params_struct(prm) if isinstance(prm, dict) else prm
    s = problem.struct()
    _need_device_scalar(grad_L)
    _need(grad_u_nom, problem.M * problem.N * 4, "f32", "grad_u_nom")
    _need(grad_w, 5, "f32", "grad_w")
    nbytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.aero_mppi_step_backward_indexed(ctypes.byref(p), ctypes.byref(s), _ptr(grad_L),
                                                _ptr(grad_u_nom), _ptr(grad_w), _ptr(ws), nbytes,
                                                _stream(stream)), "aero_mppi_step_backward_indexed")
