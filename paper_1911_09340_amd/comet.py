"""Python binding of the C ABI in include/comet.h (argument marshalling only).

Every function takes torch tensors on the current HIP device, checks their dtype,
shape, device and contiguity, and passes raw pointers plus the current stream to
the library; the work runs in the library's HIP kernels. There is no CPU fallback:
importing this module on a machine without the built library raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcomet.so")

OK, EINVAL, EWORKSPACE, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4

EXPORTS = ("comet_seed_grid", "comet_refine_grid", "comet_extrapolate_seeds",
           "comet_dca_workspace_bytes", "comet_dca_rss", "comet_select_classify",
           "comet_status_string", "comet_last_error", "comet_version")


class CometError(RuntimeError):
    def __init__(self, status: int, call: str, detail: str):
        super().__init__("%s failed: %s (%d): %s" % (call, status_string(status), status, detail))
        self.status = status


class Config(ctypes.Structure):
    """comet_config (host struct)."""
    _fields_ = [("bz_tesla", ctypes.c_double), ("charge_e", ctypes.c_double),
                ("step_mm", ctypes.c_double), ("n_steps", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("lambda_mm", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def load(path: str = LIB_PATH):
    """Load the built library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libcomet.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    I4 = ctypes.POINTER(ctypes.c_int32)
    lib.comet_seed_grid.argtypes = [_vp, I4, _vp, _i64, _vp]
    lib.comet_refine_grid.argtypes = [_vp, I4, _vp, _vp]
    lib.comet_extrapolate_seeds.argtypes = [_vp, _i64, ctypes.POINTER(Config), _vp, _vp]
    lib.comet_dca_workspace_bytes.argtypes = [_i64, _i32, _i32]
    lib.comet_dca_workspace_bytes.restype = ctypes.c_size_t
    lib.comet_dca_rss.argtypes = [_vp, _i64, _i32, _vp, _i32, _vp, _vp, _i32,
                                  ctypes.POINTER(Config), _vp, _vp, ctypes.c_size_t, _vp]
    lib.comet_select_classify.argtypes = [_vp, _i64, _vp, _i32, _vp, _i32, _vp, _vp, _i32,
                                          ctypes.POINTER(Config), _i32, _vp, _vp, _vp, _vp, _vp]
    lib.comet_status_string.argtypes = [ctypes.c_int]
    lib.comet_status_string.restype = ctypes.c_char_p
    lib.comet_last_error.argtypes = []
    lib.comet_last_error.restype = ctypes.c_char_p
    lib.comet_version.restype = ctypes.c_int
    lib.comet_dca_variant_count.restype = ctypes.c_int
    lib.comet_dca_variant_info.argtypes = [ctypes.c_int, I4, I4, I4, I4, I4, I4, I4]
    lib.comet_dca_variant_for.argtypes = [_i64, _i32, _i32]
    lib.comet_dca_variant_for.restype = ctypes.c_int
    lib.comet_dca_autotune.argtypes = [_vp, _i64, _i32, _vp, _i32, _vp, _vp, _i32,
                                       ctypes.POINTER(Config), _vp, _vp, ctypes.c_size_t, _i32,
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_double), _vp]
    lib.comet_dca_autotune.restype = ctypes.c_int
    lib.comet_profile_scan_points.argtypes = [ctypes.POINTER(ctypes.c_int64)]
    lib.comet_profile_scan_points.restype = ctypes.c_int
    lib.comet_profile_begin.restype = ctypes.c_int
    lib.comet_profile_end.restype = ctypes.c_int
    lib.comet_profile_end.argtypes = [ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.comet_dca_set_variant.argtypes = [ctypes.c_int]
    for name in ("comet_seed_grid", "comet_refine_grid", "comet_extrapolate_seeds",
                 "comet_dca_rss", "comet_select_classify", "comet_dca_set_variant",
                 "comet_dca_variant_info"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().comet_status_string(status).decode()


def _check(status: int, call: str):
    if status != OK:
        raise CometError(status, call, load().comet_last_error().decode())


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, name, shape=None, optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError("%s is required" % name)
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError("%s must be a tensor on the GPU" % name)
    if t.device.index is not None and t.device.index != torch.cuda.current_device():
        raise ValueError("%s is on %s but the current device is cuda:%d (the library works "
                         "on the current device)" % (name, t.device, torch.cuda.current_device()))
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return _vp(t.data_ptr())


def _n4(n):
    arr = (ctypes.c_int32 * 4)(*[int(v) for v in n])
    return arr


def make_config(bz: float, charge: float, step_mm: float, n_steps: int, lambda_mm: float):
    return Config(float(bz), float(charge), float(step_mm), int(n_steps), 0, float(lambda_mm))


class Field(ctypes.Structure):
    """comet_field (host struct; b is a device pointer)."""
    _fields_ = [("b", _vp), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("stepper", ctypes.c_int32),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double)]


class FieldMap:
    """A field map on the device: b [nz, ny, nx, 3] (tesla), origin and spacing (mm), and
    the stepper (0 RK4, 1 Runge-Kutta-Nystrom); keeps the tensor alive for the struct's
    pointer."""

    def __init__(self, b, origin, step, stepper: int = 0, device="cuda"):
        self.b = torch.as_tensor(b, dtype=torch.float64, device=device).contiguous()
        if self.b.dim() != 4 or self.b.shape[3] != 3:
            raise ValueError("b must have shape [nz, ny, nx, 3]")
        nz, ny, nx = (int(v) for v in self.b.shape[:3])
        self.struct = Field(_vp(self.b.data_ptr()), nx, ny, nz, int(stepper), float(origin[0]),
                            float(origin[1]), float(origin[2]), float(step[0]), float(step[1]),
                            float(step[2]))


# ------------------------------------------------------------------ entry points
def seed_grid(grid: torch.Tensor, n, seeds: torch.Tensor) -> None:
    """comet_seed_grid: grid f64[14] -> seeds f64[6, S], S = prod(n)."""
    S = int(n[0]) * int(n[1]) * int(n[2]) * int(n[3])
    _check(load().comet_seed_grid(_ptr(grid, torch.float64, "grid", (14,)), _n4(n),
                                  _ptr(seeds, torch.float64, "seeds", (6, S)), S, _stream()),
           "comet_seed_grid")


def refine_grid(grid: torch.Tensor, n, best: torch.Tensor) -> None:
    """comet_refine_grid: re-centre grid f64[14] on best i64[1] in place."""
    _check(load().comet_refine_grid(_ptr(grid, torch.float64, "grid", (14,)), _n4(n),
                                    _ptr(best, torch.int64, "best", (1,)), _stream()),
           "comet_refine_grid")


def extrapolate_seeds(seeds: torch.Tensor, cfg: Config, track: torch.Tensor) -> None:
    """comet_extrapolate_seeds: seeds f64[6, S] -> track f64[3, K+1, S]."""
    S = int(seeds.shape[1]) if seeds.dim() == 2 else -1
    _check(load().comet_extrapolate_seeds(
        _ptr(seeds, torch.float64, "seeds", (6, S)), S, ctypes.byref(cfg),
        _ptr(track, torch.float64, "track", (3, cfg.n_steps + 1, S)), _stream()),
        "comet_extrapolate_seeds")


def extrapolate_seeds_field(seeds: torch.Tensor, cfg: Config, field: FieldMap,
                            track: torch.Tensor) -> None:
    """comet_extrapolate_seeds_field: RK4 in the field map; seeds f64[6, S] -> track."""
    lib = load()
    S = int(seeds.shape[1])
    lib.comet_extrapolate_seeds_field.argtypes = [_vp, _i64, ctypes.POINTER(Config),
                                                  ctypes.POINTER(Field), _vp, _vp]
    lib.comet_extrapolate_seeds_field.restype = ctypes.c_int
    _ptr(field.b, torch.float64, "field.b")
    _check(lib.comet_extrapolate_seeds_field(
        _ptr(seeds, torch.float64, "seeds", (6, S)), S, ctypes.byref(cfg),
        ctypes.byref(field.struct),
        _ptr(track, torch.float64, "track", (3, cfg.n_steps + 1, S)), _stream()),
        "comet_extrapolate_seeds_field")


def dca_workspace_bytes(n_seeds: int, n_points: int, n_wires: int) -> int:
    return int(load().comet_dca_workspace_bytes(int(n_seeds), int(n_points), int(n_wires)))


def dca_workspace(n_seeds: int, n_points: int, n_wires: int, device=None) -> torch.Tensor:
    """A workspace tensor large enough for comet_dca_rss (256-byte aligned)."""
    nbytes = max(dca_workspace_bytes(n_seeds, n_points, n_wires), 8)
    return torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device or "cuda")


def dca_rss(track: torch.Tensor, wire_ends: torch.Tensor, wire_offsets: torch.Tensor,
            drift: torch.Tensor, cfg: Config, rss: torch.Tensor, workspace: torch.Tensor) -> None:
    """comet_dca_rss: Eq. 1 RSS of every seed's recorded track."""
    if track.dim() != 3 or track.shape[0] != 3:
        raise ValueError("track must have shape (3, K+1, S)")
    P, S = int(track.shape[1]), int(track.shape[2])
    n_w = int(wire_ends.shape[0])
    n_h = int(drift.shape[0])
    ws = _ptr(workspace, torch.float64, "workspace")
    _check(load().comet_dca_rss(
        _ptr(track, torch.float64, "track"), S, P,
        _ptr(wire_ends, torch.float64, "wire_ends", (n_w, 6)), n_w,
        _ptr(wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(drift, torch.float64, "drift", (n_h,)), n_h, ctypes.byref(cfg),
        _ptr(rss, torch.float64, "rss", (S,)), ws, workspace.numel() * 8, _stream()),
        "comet_dca_rss")


def track_dca_rss(seeds: torch.Tensor, wire_ends: torch.Tensor, wire_offsets: torch.Tensor,
                  drift: torch.Tensor, cfg: Config, track: torch.Tensor, rss: torch.Tensor,
                  workspace: torch.Tensor, field: FieldMap = None) -> None:
    """comet_track_dca_rss: extrapolate_seeds (or extrapolate_seeds_field) and dca_rss in
    one call; the track's chunk radii are taken while it is recorded."""
    lib = load()
    lib.comet_track_dca_rss.argtypes = [_vp, _i64, ctypes.POINTER(Config), ctypes.POINTER(Field),
                                        _vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp,
                                        ctypes.c_size_t, _vp]
    lib.comet_track_dca_rss.restype = ctypes.c_int
    S = int(seeds.shape[1]) if seeds.dim() == 2 else -1
    n_w, n_h = int(wire_ends.shape[0]), int(drift.shape[0])
    if field is not None:
        _ptr(field.b, torch.float64, "field.b")
    _check(lib.comet_track_dca_rss(
        _ptr(seeds, torch.float64, "seeds", (6, S)), S, ctypes.byref(cfg),
        ctypes.byref(field.struct) if field is not None else None,
        _ptr(wire_ends, torch.float64, "wire_ends", (n_w, 6)), n_w,
        _ptr(wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(drift, torch.float64, "drift", (n_h,)), n_h,
        _ptr(track, torch.float64, "track", (3, cfg.n_steps + 1, S)),
        _ptr(rss, torch.float64, "rss", (S,)), _ptr(workspace, torch.float64, "workspace"),
        workspace.numel() * 8, _stream()), "comet_track_dca_rss")


def static_scratch_bytes() -> int:
    lib = load()
    lib.comet_static_scratch_bytes.restype = ctypes.c_size_t
    lib.comet_static_scratch_bytes.argtypes = []
    return int(lib.comet_static_scratch_bytes())


def track_dca_rss_static(seeds: torch.Tensor, wire_ends: torch.Tensor,
                         wire_offsets: torch.Tensor, drift: torch.Tensor, cfg: Config,
                         track: torch.Tensor, rss: torch.Tensor, field: FieldMap = None) -> None:
    """comet_track_dca_rss_static: track_dca_rss with the library's fixed device workspace
    (no workspace argument, nothing allocated)."""
    lib = load()
    lib.comet_track_dca_rss_static.argtypes = [_vp, _i64, ctypes.POINTER(Config),
                                               ctypes.POINTER(Field), _vp, _i32, _vp, _vp, _i32,
                                               _vp, _vp, _vp]
    lib.comet_track_dca_rss_static.restype = ctypes.c_int
    S = int(seeds.shape[1]) if seeds.dim() == 2 else -1
    n_w, n_h = int(wire_ends.shape[0]), int(drift.shape[0])
    if field is not None:
        _ptr(field.b, torch.float64, "field.b")
    _check(lib.comet_track_dca_rss_static(
        _ptr(seeds, torch.float64, "seeds", (6, S)), S, ctypes.byref(cfg),
        ctypes.byref(field.struct) if field is not None else None,
        _ptr(wire_ends, torch.float64, "wire_ends", (n_w, 6)), n_w,
        _ptr(wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(drift, torch.float64, "drift", (n_h,)), n_h,
        _ptr(track, torch.float64, "track", (3, cfg.n_steps + 1, S)),
        _ptr(rss, torch.float64, "rss", (S,)), _stream()), "comet_track_dca_rss_static")


def select_classify(rss: torch.Tensor, best: torch.Tensor, cfg: Config, track=None,
                    wire_ends=None, wire_offsets=None, drift=None, hit_mask=None,
                    n_borderline=None, dca_best=None, top_k: int = 1) -> None:
    """comet_select_classify: argmin of rss into best; optionally classify the hits."""
    S = int(rss.shape[0])
    n_w = int(wire_ends.shape[0]) if wire_ends is not None else 0
    n_h = int(drift.shape[0]) if drift is not None else 0
    P = int(track.shape[1]) if track is not None else 0
    _check(load().comet_select_classify(
        _ptr(rss, torch.float64, "rss", (S,)), S,
        _ptr(track, torch.float64, "track", optional=True), P,
        _ptr(wire_ends, torch.float64, "wire_ends", (n_w, 6), optional=True), n_w,
        _ptr(wire_offsets, torch.int32, "wire_offsets", (n_w + 1,), optional=True),
        _ptr(drift, torch.float64, "drift", (n_h,), optional=True), n_h, ctypes.byref(cfg),
        int(top_k), _ptr(best, torch.int64, "best", (int(top_k),)),
        _ptr(hit_mask, torch.uint8, "hit_mask", (n_h,), optional=True),
        _ptr(n_borderline, torch.int32, "n_borderline", (1,), optional=True),
        _ptr(dca_best, torch.float64, "dca_best", (n_w,), optional=True), _stream()),
        "comet_select_classify")


# ------------------------------------------------------------------ tuning hooks
def dca_variants():
    lib = load()
    out = []
    for i in range(lib.comet_dca_variant_count()):
        v = [ctypes.c_int32() for _ in range(7)]
        _check(lib.comet_dca_variant_info(i, *[ctypes.byref(x) for x in v]),
               "comet_dca_variant_info")
        form = {0: "lds", 1: "direct", 2: "wide", 3: "wide_cap", 5: "wide_cap_x"}[v[5].value]
        lib.comet_dca_variant_name.restype = ctypes.c_char_p
        lib.comet_dca_variant_name.argtypes = [ctypes.c_int]
        out.append(dict(w=v[0].value, nwv=v[1].value, chunk=v[2].value,
                        chunk_argmin=bool(v[3].value), xcd_remap=bool(v[4].value),
                        direct=form != "lds", form=form, runs=v[6].value,
                        kernel=lib.comet_dca_variant_name(i).decode()))
    return out


def dca_kernel_name(shape: dict) -> str:
    """The kernel symbol (template form) of a DCA shape, as a profiler names it."""
    return shape["kernel"]


def set_dca_variant(i: int) -> None:
    """Force DCA kernel shape i for every call (-1 removes the override)."""
    _check(load().comet_dca_set_variant(int(i)), "comet_dca_set_variant")


def dca_variant_for(n_seeds: int, n_points: int, n_wires: int) -> int:
    return int(load().comet_dca_variant_for(int(n_seeds), int(n_points), int(n_wires)))


def dca_autotune(track: torch.Tensor, wire_ends: torch.Tensor, wire_offsets: torch.Tensor,
                 drift: torch.Tensor, cfg: Config, rss: torch.Tensor, workspace: torch.Tensor,
                 reps: int = 3):
    """comet_dca_autotune: time every DCA shape on these inputs, keep the fastest for
    this shape. Returns (best id, [ms per shape]). Synchronises the current stream."""
    P, S = int(track.shape[1]), int(track.shape[2])
    n_w = int(wire_ends.shape[0])
    n_h = int(drift.shape[0])
    nv = load().comet_dca_variant_count()
    ms = (ctypes.c_double * nv)()
    best = ctypes.c_int32(-1)
    _check(load().comet_dca_autotune(
        _ptr(track, torch.float64, "track"), S, P,
        _ptr(wire_ends, torch.float64, "wire_ends", (n_w, 6)), n_w,
        _ptr(wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(drift, torch.float64, "drift", (n_h,)), n_h, ctypes.byref(cfg),
        _ptr(rss, torch.float64, "rss", (S,)), _ptr(workspace, torch.float64, "workspace"),
        workspace.numel() * 8, int(reps), ctypes.byref(best), ms, _stream()),
        "comet_dca_autotune")
    return best.value, list(ms)


PROFILE_KINDS = ("track", "dca", "rss_sum", "select")


def profile_begin() -> None:
    _check(load().comet_profile_begin(), "comet_profile_begin")


def profile_end() -> dict:
    """{kind: (total_ms, launches)} since profile_begin (waits for the events), plus
    "scan_points": the (seed, wire, point) distance evaluations the DCA scans made."""
    lib = load()
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_int64 * 4)()
    _check(lib.comet_profile_end(ms, n), "comet_profile_end")
    out = {k: (ms[i], n[i]) for i, k in enumerate(PROFILE_KINDS)}
    pts = ctypes.c_int64()
    _check(lib.comet_profile_scan_points(ctypes.byref(pts)), "comet_profile_scan_points")
    out["scan_points"] = pts.value
    return out


# ------------------------------------------------------------------ derivatives
def _bind_derivatives(lib):
    if getattr(lib, "_derivs_bound", False):
        return lib
    lib.comet_rss_adjoint.argtypes = [_vp, _i64, ctypes.POINTER(Config), _vp, _i32, _vp, _vp, _i32,
                                      _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.comet_rss_adjoint.restype = ctypes.c_int
    lib.comet_lm_workspace_bytes.argtypes = [_i64, _i32]
    lib.comet_lm_workspace_bytes.restype = ctypes.c_size_t
    lib.comet_lm_refine.argtypes = [_vp, _i64, ctypes.POINTER(Config), _vp, _i32, _vp, _vp, _i32,
                                    _vp, _vp, _i32, ctypes.c_double, _vp, _vp, _vp,
                                    ctypes.c_size_t, _vp]
    lib.comet_lm_refine.restype = ctypes.c_int
    FP = ctypes.POINTER(Field)
    lib.comet_rss_jacobian_field.argtypes = [_vp, _i64, ctypes.POINTER(Config), FP, _vp, _i32,
                                             _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                             _vp, _vp, _vp]
    lib.comet_rss_jacobian_field.restype = ctypes.c_int
    lib.comet_lm_refine_field.argtypes = [_vp, _i64, ctypes.POINTER(Config), FP, _vp, _i32, _vp,
                                          _vp, _i32, _vp, _vp, _i32, ctypes.c_double, _vp, _vp,
                                          _vp, ctypes.c_size_t, _vp]
    lib.comet_lm_refine_field.restype = ctypes.c_int
    lib._derivs_bound = True
    return lib


def rss_adjoint(seeds: torch.Tensor, cfg: Config, wire_ends: torch.Tensor,
                wire_offsets: torch.Tensor, drift: torch.Tensor, rss=None, grad=None, jtj=None,
                jte=None, dca=None, resid=None, jac=None, event_wires=None,
                seed_event=None, field: "FieldMap" = None) -> None:
    """comet_rss_adjoint: RSS, its seed gradient [S, 6], normal equations and per-wire rows;
    with a field map, comet_rss_jacobian_field (tracks in the map, the same outputs)."""
    lib = _bind_derivatives(load())
    S = int(seeds.shape[1]) if seeds.dim() == 2 else -1
    n_w, n_h = int(wire_ends.shape[0]), int(drift.shape[0])
    if field is None:
        fn, name, head = lib.comet_rss_adjoint, "comet_rss_adjoint", ()
    else:
        fn, name = lib.comet_rss_jacobian_field, "comet_rss_jacobian_field"
        head = (ctypes.byref(field.struct),)
    _check(fn(
        _ptr(seeds, torch.float64, "seeds", (6, S)), S, ctypes.byref(cfg), *head,
        _ptr(wire_ends, torch.float64, "wire_ends", (n_w, 6)), n_w,
        _ptr(wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(drift, torch.float64, "drift", (n_h,)), n_h,
        _ptr(event_wires, torch.int32, "event_wires", optional=True),
        _ptr(seed_event, torch.int32, "seed_event", (S,), optional=True),
        _ptr(rss, torch.float64, "rss", (S,), optional=True),
        _ptr(grad, torch.float64, "grad", (S, 6), optional=True),
        _ptr(jtj, torch.float64, "jtj", (S, 21), optional=True),
        _ptr(jte, torch.float64, "jte", (S, 6), optional=True),
        _ptr(dca, torch.float64, "dca", (S, n_w), optional=True),
        _ptr(resid, torch.float64, "resid", (S, n_w), optional=True),
        _ptr(jac, torch.float64, "jac", (S, n_w, 6), optional=True), _stream()), name)


def lm_workspace(n_seeds: int, n_steps: int, device=None) -> torch.Tensor:
    nbytes = int(_bind_derivatives(load()).comet_lm_workspace_bytes(int(n_seeds), int(n_steps)))
    return torch.empty((max(nbytes, 8) + 7) // 8, dtype=torch.float64, device=device or "cuda")


def lm_refine(seeds: torch.Tensor, cfg: Config, wire_ends: torch.Tensor,
              wire_offsets: torch.Tensor, drift: torch.Tensor, n_iter: int, mu0: float,
              rss: torch.Tensor, workspace: torch.Tensor, n_accepted=None, event_wires=None,
              seed_event=None, field: "FieldMap" = None) -> None:
    """comet_lm_refine: Levenberg-Marquardt refinement of seeds [6, S] in place; with a
    field map, comet_lm_refine_field."""
    lib = _bind_derivatives(load())
    S = int(seeds.shape[1]) if seeds.dim() == 2 else -1
    n_w, n_h = int(wire_ends.shape[0]), int(drift.shape[0])
    if field is None:
        fn, name, head = lib.comet_lm_refine, "comet_lm_refine", ()
    else:
        fn, name = lib.comet_lm_refine_field, "comet_lm_refine_field"
        head = (ctypes.byref(field.struct),)
    _check(fn(
        _ptr(seeds, torch.float64, "seeds", (6, S)), S, ctypes.byref(cfg), *head,
        _ptr(wire_ends, torch.float64, "wire_ends", (n_w, 6)), n_w,
        _ptr(wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(drift, torch.float64, "drift", (n_h,)), n_h,
        _ptr(event_wires, torch.int32, "event_wires", optional=True),
        _ptr(seed_event, torch.int32, "seed_event", (S,), optional=True),
        int(n_iter), float(mu0), _ptr(rss, torch.float64, "rss", (S,)),
        _ptr(n_accepted, torch.int32, "n_accepted", (S,), optional=True),
        _ptr(workspace, torch.float64, "workspace"), workspace.numel() * 8, _stream()), name)


# ------------------------------------------------------------------ batches
def _bind_batch(lib):
    if getattr(lib, "_batch_bound", False):
        return lib
    I4 = ctypes.POINTER(ctypes.c_int32)
    lib.comet_batch_workspace_bytes.argtypes = [_i32, _i32, _i32]
    lib.comet_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.comet_batch_scan.argtypes = [_vp, _i32, _vp, _vp, _i32, _vp, _i32, _vp, _i32, _vp, _vp, I4,
                                     ctypes.POINTER(Config), _i32, _vp, _vp, _vp, _vp, _vp, _i64,
                                     _vp, _i64, _vp, ctypes.c_size_t, _vp]
    lib.comet_batch_scan.restype = ctypes.c_int
    FP = ctypes.POINTER(Field)
    args = list(lib.comet_batch_scan.argtypes)
    lib.comet_batch_scan_field.argtypes = args[:13] + [FP] + args[13:]
    lib.comet_batch_scan_field.restype = ctypes.c_int
    # (..., n_borderline, event_active, workspace, bytes, stream): max_items replaced
    lib.comet_batch_scan_active.argtypes = args[:21] + [_vp] + args[22:]
    lib.comet_batch_scan_active.restype = ctypes.c_int
    lib.comet_batch_variant_count.restype = ctypes.c_int
    lib.comet_batch_variant_info.argtypes = [ctypes.c_int, I4, I4, I4, I4, I4, I4]
    lib.comet_batch_variant_info.restype = ctypes.c_int
    lib.comet_batch_set_variant.argtypes = [ctypes.c_int]
    lib.comet_batch_set_variant.restype = ctypes.c_int
    lib.comet_topk.argtypes = [_vp, _i64, _i32, _i32, _vp, _vp]
    lib.comet_topk.restype = ctypes.c_int
    lib.comet_grid_seeds.argtypes = [_vp, _i32, I4, _vp, _i32, _vp, _vp]
    lib.comet_grid_seeds.restype = ctypes.c_int
    lib.comet_sparse_select.argtypes = [_vp, _vp, _i32, _i32, I4, _i32, _vp, _vp, _vp, _vp, _vp,
                                        _vp]
    lib.comet_sparse_select.restype = ctypes.c_int
    lib.comet_batch_classify.argtypes = [_vp, _i32, I4, _vp, _vp, _vp, _i32, _vp, _vp, _i32, _vp,
                                         _i32, _vp, ctypes.POINTER(Config), _vp, _vp, _vp, _i64,
                                         _vp, _vp]
    lib.comet_batch_classify.restype = ctypes.c_int
    lib.comet_layer_veto.argtypes = [_vp, _i64, _i32, _vp, _vp, _i32, _vp, _vp, _i32, _i32, _vp,
                                     _vp]
    lib.comet_layer_veto.restype = ctypes.c_int
    lib.comet_merge_halves.argtypes = [_vp, _vp, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp]
    lib.comet_merge_halves.restype = ctypes.c_int
    D4 = ctypes.POINTER(ctypes.c_double)
    lib.comet_backward_seeds.argtypes = [_vp, _i32, ctypes.POINTER(Config), ctypes.c_double, _i32,
                                         _vp, _vp, _vp]
    lib.comet_backward_seeds.restype = ctypes.c_int
    lib.comet_stage_grids.argtypes = [_vp, _vp, _i32, D4, _vp, _vp]
    lib.comet_stage_grids.restype = ctypes.c_int
    lib.comet_stage_grids_z.argtypes = [_vp, _vp, _i32, D4, _i32, ctypes.c_double, _vp, _vp]
    lib.comet_stage_grids_z.restype = ctypes.c_int
    lib.comet_exclude_workspace_bytes.argtypes = [_i32]
    lib.comet_exclude_workspace_bytes.restype = ctypes.c_size_t
    lib.comet_exclude_hits.argtypes = [_vp, _i32, _vp, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp,
                                       _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.comet_exclude_hits.restype = ctypes.c_int
    lib.comet_stage_record.argtypes = [_vp, _i64, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp]
    lib.comet_stage_record.restype = ctypes.c_int
    lib.comet_stage_update.argtypes = [_vp, _i32, _vp, _vp, _vp, _i32, _i32, _i32, _vp]
    lib.comet_stage_update.restype = ctypes.c_int
    lib.comet_self_refine.argtypes = [_vp, _i32, _vp, ctypes.POINTER(Config), _vp, _i32, _vp,
                                      _vp, _i32, _vp, _i32, ctypes.c_double, _vp, _vp, _i64, _vp]
    lib.comet_self_refine.restype = ctypes.c_int
    lib.comet_exit_seeds.argtypes = [_vp, _i64, _i32, ctypes.POINTER(Config), ctypes.c_double,
                                     _i32, _vp, _vp, _vp]
    lib.comet_exit_seeds.restype = ctypes.c_int
    lib.comet_half_split.argtypes = [_vp, _i32, _vp, _vp, _i32, _vp, _i32, _vp, _vp, _vp]
    lib.comet_half_split.restype = ctypes.c_int
    lib.comet_wire_layers.argtypes = [_vp, _i32, _vp, _i32, _vp, _vp, _i32, _vp, _vp]
    lib.comet_wire_layers.restype = ctypes.c_int
    lib.comet_union_halves.argtypes = [_vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _i64,
                                       _vp, _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp]
    lib.comet_union_halves.restype = ctypes.c_int
    lib._batch_bound = True
    return lib


def batch_workspace(n_wires: int, n_steps: int, n_partitions: int, device=None) -> torch.Tensor:
    nbytes = int(_bind_batch(load()).comet_batch_workspace_bytes(int(n_wires), int(n_steps),
                                                                 int(n_partitions)))
    return torch.empty((max(nbytes, 8) + 7) // 8, dtype=torch.float64, device=device or "cuda")


def batch_scan(packed, part_event: torch.Tensor, grids: torch.Tensor, n, cfg: Config,
               n_refine: int, rss: torch.Tensor, best: torch.Tensor, workspace: torch.Tensor,
               best_seed=None, best_rss=None, hit_mask=None, n_borderline=None,
               max_items: int = 0, grids_init=None, field: FieldMap = None,
               event_active=None) -> None:
    """comet_batch_scan over packed events (scan.PackedEvents); with a field map,
    comet_batch_scan_field (tracks in the map); with event_active (int32 [n_events]),
    comet_batch_scan_active (only the partitions of active events)."""
    lib = _bind_batch(load())
    NP = int(part_event.shape[0])
    S = int(n[0]) * int(n[1]) * int(n[2]) * int(n[3])
    n_w, n_h = int(packed.wire_ends.shape[0]), int(packed.drift.shape[0])
    n_e = int(packed.event_wires.shape[0]) - 1
    stride = int(hit_mask.shape[1]) if hit_mask is not None else 0
    last = (int(max_items),)
    if field is None and event_active is None:
        fn, name, fld = lib.comet_batch_scan, "comet_batch_scan", ()
    elif field is None:
        if max_items:
            raise ValueError("batch_scan: max_items does not combine with event_active")
        fn, name, fld = lib.comet_batch_scan_active, "comet_batch_scan_active", ()
        last = (_ptr(event_active, torch.int32, "event_active", (n_e,)),)
    else:
        if event_active is not None:
            raise ValueError("batch_scan: event_active is not offered with a field map")
        _ptr(field.b, torch.float64, "field.b")
        fn, name = lib.comet_batch_scan_field, "comet_batch_scan_field"
        fld = (ctypes.byref(field.struct),)
    _check(fn(
        _ptr(packed.wire_ends, torch.float64, "wire_ends", (n_w, 6)), n_w,
        _ptr(packed.wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(packed.drift, torch.float64, "drift", (n_h,)), n_h,
        _ptr(packed.event_wires, torch.int32, "event_wires", (n_e + 1,)), n_e,
        _ptr(part_event, torch.int32, "part_event", (NP,)), NP,
        _ptr(grids_init, torch.float64, "grids_init", (NP, 14), optional=True),
        _ptr(grids, torch.float64, "grids", (NP, 14)), _n4(n), ctypes.byref(cfg), *fld,
        int(n_refine),
        _ptr(rss, torch.float64, "rss", (NP, S)), _ptr(best, torch.int64, "best", (NP,)),
        _ptr(best_seed, torch.float64, "best_seed", (NP, 6), optional=True),
        _ptr(best_rss, torch.float64, "best_rss", (NP,), optional=True),
        _ptr(hit_mask, torch.uint8, "hit_mask", (NP, stride), optional=True), stride,
        _ptr(n_borderline, torch.int32, "n_borderline", (NP,), optional=True), *last,
        _ptr(workspace, torch.float64, "workspace"), workspace.numel() * 8, _stream()), name)


def batch_variants():
    lib = _bind_batch(load())
    out = []
    for i in range(lib.comet_batch_variant_count()):
        v = [ctypes.c_int32() for _ in range(6)]
        _check(lib.comet_batch_variant_info(i, *[ctypes.byref(x) for x in v]),
               "comet_batch_variant_info")
        form = {0: "lds", 1: "direct", 2: "wide", 3: "wide_cap", 4: "wide_cap_az",
                5: "wide_cap_az_x"}[v[4].value]
        out.append(dict(w=v[0].value, nwv=v[1].value, chunk=v[2].value, blocks=v[3].value,
                        direct=form != "lds", form=form, runs=v[5].value))
    return out


def set_batch_variant(i: int) -> None:
    _check(_bind_batch(load()).comet_batch_set_variant(int(i)), "comet_batch_set_variant")


def topk(values: torch.Tensor, k: int, out: torch.Tensor) -> None:
    """comet_topk: values [segments, n] -> out [segments, k] (int64)."""
    lib = _bind_batch(load())
    seg, n = int(values.shape[0]), int(values.shape[1])
    _check(lib.comet_topk(_ptr(values, torch.float64, "values", (seg, n)), n, seg, int(k),
                          _ptr(out, torch.int64, "out", (seg, k)), _stream()), "comet_topk")


def grid_seeds(grids: torch.Tensor, n, idx: torch.Tensor, out: torch.Tensor) -> None:
    """comet_grid_seeds: seeds of grids [NP, 14] at idx [NP, k] -> out [6, NP * k]."""
    lib = _bind_batch(load())
    NP, k = int(idx.shape[0]), int(idx.shape[1])
    _check(lib.comet_grid_seeds(_ptr(grids, torch.float64, "grids", (NP, 14)), NP, _n4(n),
                                _ptr(idx, torch.int64, "idx", (NP, k)), k,
                                _ptr(out, torch.float64, "out", (6, NP * k)), _stream()),
           "comet_grid_seeds")


def sparse_select(grids: torch.Tensor, rss: torch.Tensor, n, n_ref: int, ref_idx: torch.Tensor,
                  new_grids: torch.Tensor, ref_rss=None, ref_grids=None, ref_local=None) -> None:
    """comet_sparse_select: grids [G, n_sub, 14], rss [G, n_sub, S] -> ref_idx [G, n_ref],
    new_grids [G, n_ref, 14] (optional ref_rss [G, n_ref], ref_grids [G, n_ref, 14],
    ref_local [G, n_ref])."""
    lib = _bind_batch(load())
    G, n_sub = int(grids.shape[0]), int(grids.shape[1])
    S = int(n[0]) * int(n[1]) * int(n[2]) * int(n[3])
    R = int(n_ref)
    _check(lib.comet_sparse_select(
        _ptr(grids, torch.float64, "grids", (G, n_sub, 14)),
        _ptr(rss, torch.float64, "rss", (G, n_sub, S)), G, n_sub, _n4(n), R,
        _ptr(ref_idx, torch.int64, "ref_idx", (G, R)),
        _ptr(ref_rss, torch.float64, "ref_rss", (G, R), optional=True),
        _ptr(new_grids, torch.float64, "new_grids", (G, R, 14)),
        _ptr(ref_grids, torch.float64, "ref_grids", (G, R, 14), optional=True),
        _ptr(ref_local, torch.int64, "ref_local", (G, R), optional=True), _stream()),
        "comet_sparse_select")


def batch_classify(packed, part_event: torch.Tensor, grids: torch.Tensor, n, cfg: Config,
                   best: torch.Tensor, rss=None, best_seed=None, best_rss=None, hit_mask=None,
                   n_borderline=None) -> None:
    """comet_batch_classify: classify seed best[p] of grids[p] for every partition p."""
    lib = _bind_batch(load())
    NP = int(part_event.shape[0])
    S = int(n[0]) * int(n[1]) * int(n[2]) * int(n[3])
    n_w, n_h = int(packed.wire_ends.shape[0]), int(packed.drift.shape[0])
    n_e = int(packed.event_wires.shape[0]) - 1
    stride = int(hit_mask.shape[1]) if hit_mask is not None else 0
    _check(lib.comet_batch_classify(
        _ptr(grids, torch.float64, "grids", (NP, 14)), NP, _n4(n),
        _ptr(best, torch.int64, "best", (NP,)),
        _ptr(rss, torch.float64, "rss", (NP, S), optional=True),
        _ptr(packed.wire_ends, torch.float64, "wire_ends", (n_w, 6)), n_w,
        _ptr(packed.wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(packed.drift, torch.float64, "drift", (n_h,)), n_h,
        _ptr(packed.event_wires, torch.int32, "event_wires", (n_e + 1,)), n_e,
        _ptr(part_event, torch.int32, "part_event", (NP,)), ctypes.byref(cfg),
        _ptr(best_seed, torch.float64, "best_seed", (NP, 6), optional=True),
        _ptr(best_rss, torch.float64, "best_rss", (NP,), optional=True),
        _ptr(hit_mask, torch.uint8, "hit_mask", (NP, stride), optional=True), stride,
        _ptr(n_borderline, torch.int32, "n_borderline", (NP,), optional=True), _stream()),
        "comet_batch_classify")


def layer_veto(hit_mask: torch.Tensor, row_event: torch.Tensor, packed, wire_layer: torch.Tensor,
               n_layers: int, veto: torch.Tensor) -> None:
    """comet_layer_veto: hit_mask [rows, stride] (uint8), row_event [rows] -> veto [rows]."""
    lib = _bind_batch(load())
    rows, stride = int(hit_mask.shape[0]), int(hit_mask.shape[1])
    n_w = int(packed.wire_ends.shape[0])
    n_e = int(packed.event_wires.shape[0]) - 1
    _check(lib.comet_layer_veto(
        _ptr(hit_mask, torch.uint8, "hit_mask", (rows, stride)), stride, rows,
        _ptr(row_event, torch.int32, "row_event", (rows,)),
        _ptr(packed.event_wires, torch.int32, "event_wires", (n_e + 1,)), n_e,
        _ptr(packed.wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(wire_layer, torch.int32, "wire_layer", (n_w,)), n_w, int(n_layers),
        _ptr(veto, torch.int32, "veto", (rows,)), _stream()), "comet_layer_veto")


def merge_halves(rss_a: torch.Tensor, veto_a: torch.Tensor, rss_b: torch.Tensor,
                 veto_b: torch.Tensor, pair: torch.Tensor, pair_rss: torch.Tensor,
                 n_complete=None) -> None:
    """comet_merge_halves: [P, F] per side -> pair / pair_rss [P, F * F]."""
    lib = _bind_batch(load())
    P, F = int(rss_a.shape[0]), int(rss_a.shape[1])
    _check(lib.comet_merge_halves(
        _ptr(rss_a, torch.float64, "rss_a", (P, F)), _ptr(veto_a, torch.int32, "veto_a", (P, F)),
        _ptr(rss_b, torch.float64, "rss_b", (P, F)), _ptr(veto_b, torch.int32, "veto_b", (P, F)),
        P, F, _ptr(pair, torch.int32, "pair", (P, F * F)),
        _ptr(pair_rss, torch.float64, "pair_rss", (P, F * F)),
        _ptr(n_complete, torch.int32, "n_complete", (P,), optional=True), _stream()),
        "comet_merge_halves")


# ------------------------------------------------------------------ stage loop
def backward_seeds(seeds: torch.Tensor, cfg: Config, radius: float, max_steps: int,
                   out: torch.Tensor, steps=None) -> None:
    """comet_backward_seeds: seeds [n, 6] -> out [n, 6] (optional steps [n] int32)."""
    lib = _bind_batch(load())
    n = int(seeds.shape[0])
    _check(lib.comet_backward_seeds(_ptr(seeds, torch.float64, "seeds", (n, 6)), n,
                                    ctypes.byref(cfg), float(radius), int(max_steps),
                                    _ptr(out, torch.float64, "out", (n, 6)),
                                    _ptr(steps, torch.int32, "steps", (n,), optional=True),
                                    _stream()), "comet_backward_seeds")


def stage_grids(transverse: torch.Tensor, ext: torch.Tensor, half, grids: torch.Tensor) -> None:
    lib = _bind_batch(load())
    n = int(transverse.shape[0])
    h = (ctypes.c_double * 4)(*[float(v) for v in half])
    _check(lib.comet_stage_grids(_ptr(transverse, torch.float64, "transverse", (n, 6)),
                                 _ptr(ext, torch.float64, "ext", (n, 6)), n, h,
                                 _ptr(grids, torch.float64, "grids", (n, 14)), _stream()),
           "comet_stage_grids")


def stage_grids_z(transverse: torch.Tensor, ext: torch.Tensor, half, n_z: int, z_half: float,
                  grids: torch.Tensor) -> None:
    """comet_stage_grids_z: grids [n, n_z, 14], the seed's z as a fifth axis."""
    lib = _bind_batch(load())
    n = int(transverse.shape[0])
    h = (ctypes.c_double * 4)(*[float(v) for v in half])
    _check(lib.comet_stage_grids_z(_ptr(transverse, torch.float64, "transverse", (n, 6)),
                                   _ptr(ext, torch.float64, "ext", (n, 6)), n, h, int(n_z),
                                   float(z_half),
                                   _ptr(grids, torch.float64, "grids", (n, int(n_z), 14)),
                                   _stream()), "comet_stage_grids_z")


def exclude_workspace(n_events: int, device=None) -> torch.Tensor:
    nbytes = int(_bind_batch(load()).comet_exclude_workspace_bytes(int(n_events)))
    return torch.empty((max(nbytes, 8) + 7) // 8, dtype=torch.float64, device=device or "cuda")


def exclude_hits(src, exclude: torch.Tensor, dst, workspace: torch.Tensor) -> None:
    """comet_exclude_hits from packed events src (with .hit_ids) into dst (same capacities)."""
    lib = _bind_batch(load())
    n_w, n_h = int(src.wire_ends.shape[0]), int(src.drift.shape[0])
    n_e = int(src.event_wires.shape[0]) - 1
    _check(lib.comet_exclude_hits(
        _ptr(src.event_wires, torch.int32, "event_wires", (n_e + 1,)), n_e,
        _ptr(src.wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)), n_w,
        _ptr(src.drift, torch.float64, "drift", (n_h,)),
        _ptr(src.wire_ends, torch.float64, "wire_ends", (n_w, 6)),
        _ptr(src.hit_ids, torch.int32, "hit_ids", (n_h,)), n_h,
        _ptr(exclude, torch.uint8, "exclude", (n_h,)),
        _ptr(dst.event_wires, torch.int32, "event_wires_out", (n_e + 1,)),
        _ptr(dst.wire_offsets, torch.int32, "wire_offsets_out", (n_w + 1,)),
        _ptr(dst.drift, torch.float64, "drift_out", (n_h,)),
        _ptr(dst.wire_ends, torch.float64, "wire_ends_out", (n_w, 6)),
        _ptr(dst.hit_ids, torch.int32, "hit_ids_out", (n_h,)),
        _ptr(workspace, torch.float64, "workspace"), workspace.numel() * 8, _stream()),
        "comet_exclude_hits")


def stage_record(hit_mask: torch.Tensor, packed, active: torch.Tensor, stage: int,
                 stage_of_hit: torch.Tensor, exclude: torch.Tensor) -> None:
    lib = _bind_batch(load())
    n_e, stride = int(hit_mask.shape[0]), int(hit_mask.shape[1])
    n_w, n_h = int(packed.wire_ends.shape[0]), int(packed.drift.shape[0])
    _check(lib.comet_stage_record(
        _ptr(hit_mask, torch.uint8, "hit_mask", (n_e, stride)), stride, n_e,
        _ptr(packed.event_wires, torch.int32, "event_wires", (n_e + 1,)),
        _ptr(packed.wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(packed.hit_ids, torch.int32, "hit_ids", (n_h,)),
        _ptr(active, torch.int32, "active", (n_e,)), int(stage),
        _ptr(stage_of_hit, torch.int32, "stage_of_hit"),
        _ptr(exclude, torch.uint8, "exclude", (n_h,)), _stream()), "comet_stage_record")


def self_refine(seeds: torch.Tensor, row_event: torch.Tensor, cfg: Config, packed, eta: float,
                mask_in: torch.Tensor, mask_out: torch.Tensor) -> None:
    """comet_self_refine: re-classify row r's hits at the fitted seed seeds[r] (double
    [n_rows, 6]) with lambda for the classified hits and eta for wires left without one."""
    lib = _bind_batch(load())
    n_r, stride = int(mask_in.shape[0]), int(mask_in.shape[1])
    n_w, n_h = int(packed.wire_ends.shape[0]), int(packed.drift.shape[0])
    n_e = int(packed.event_wires.shape[0]) - 1
    _check(lib.comet_self_refine(
        _ptr(seeds, torch.float64, "seeds", (n_r, 6)), n_r,
        _ptr(row_event, torch.int32, "row_event", (n_r,)), ctypes.byref(cfg),
        _ptr(packed.wire_ends, torch.float64, "wire_ends", (n_w, 6)), n_w,
        _ptr(packed.wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(packed.drift, torch.float64, "drift", (n_h,)), n_h,
        _ptr(packed.event_wires, torch.int32, "event_wires", (n_e + 1,)), n_e, float(eta),
        _ptr(mask_in, torch.uint8, "mask_in", (n_r, stride)),
        _ptr(mask_out, torch.uint8, "mask_out", (n_r, stride)), stride, _stream()),
        "comet_self_refine")


# ------------------------------------------------------------------ per-stage chain
def exit_seeds(states: torch.Tensor, row_stride: int, cfg: Config, radius: float,
               max_steps: int, out: torch.Tensor, steps=None) -> None:
    """comet_exit_seeds: rows of `states` (double, row_stride doubles apart, the first six
    used) -> out [n, 6], the exit half's seed (optional steps [n] int32)."""
    lib = _bind_batch(load())
    n = int(out.shape[0])
    if states.dtype != torch.float64 or not states.is_contiguous() or \
            states.numel() < (n - 1) * int(row_stride) + 6:
        raise CometError(EINVAL, "exit_seeds: states must be contiguous float64 holding n rows")
    _check(lib.comet_exit_seeds(_ptr(states, torch.float64, "states"), int(row_stride), n,
                                ctypes.byref(cfg), float(radius), int(max_steps),
                                _ptr(out, torch.float64, "out", (n, 6)),
                                _ptr(steps, torch.int32, "steps", (n,), optional=True),
                                _stream()), "comet_exit_seeds")


def half_split(packed, entrance_side: torch.Tensor, exclude_entrance: torch.Tensor,
               exclude_exit: torch.Tensor) -> None:
    """comet_half_split: per hit of `packed` (with .hit_ids), the exclusion masks of the
    entrance and exit halves from entrance_side (uint8, by hit id)."""
    lib = _bind_batch(load())
    n_w, n_h = int(packed.wire_ends.shape[0]), int(packed.drift.shape[0])
    n_e = int(packed.event_wires.shape[0]) - 1
    n_ids = int(entrance_side.shape[0])
    _check(lib.comet_half_split(
        _ptr(packed.event_wires, torch.int32, "event_wires", (n_e + 1,)), n_e,
        _ptr(packed.wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(packed.hit_ids, torch.int32, "hit_ids", (n_h,)), n_h,
        _ptr(entrance_side, torch.uint8, "entrance_side", (n_ids,)), n_ids,
        _ptr(exclude_entrance, torch.uint8, "exclude_entrance", (n_h,)),
        _ptr(exclude_exit, torch.uint8, "exclude_exit", (n_h,)), _stream()), "comet_half_split")


def wire_layers(packed, hit_layer: torch.Tensor, wire_layer: torch.Tensor) -> None:
    """comet_wire_layers: wire_layer [n_wires] from the layer of each wire's first hit."""
    lib = _bind_batch(load())
    n_w, n_h = int(packed.wire_ends.shape[0]), int(packed.drift.shape[0])
    n_e = int(packed.event_wires.shape[0]) - 1
    n_ids = int(hit_layer.shape[0])
    _check(lib.comet_wire_layers(
        _ptr(packed.event_wires, torch.int32, "event_wires", (n_e + 1,)), n_e,
        _ptr(packed.wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)), n_w,
        _ptr(packed.hit_ids, torch.int32, "hit_ids", (n_h,)),
        _ptr(hit_layer, torch.int32, "hit_layer", (n_ids,)), n_ids,
        _ptr(wire_layer, torch.int32, "wire_layer", (n_w,)), _stream()), "comet_wire_layers")


def union_halves(pair: torch.Tensor, n_complete: torch.Tensor, n_final: int, packed,
                 entrance_side: torch.Tensor, mask_a: torch.Tensor, mask_b: torch.Tensor,
                 seeds_a: torch.Tensor, active: torch.Tensor, mask_out: torch.Tensor,
                 seed_out: torch.Tensor, best_out: torch.Tensor) -> None:
    """comet_union_halves: the best complete set of every active event -> its union mask
    on `packed` [E, stride], its entrance seed [E, 6] and pair code [E] (int64)."""
    lib = _bind_batch(load())
    E, F = int(active.shape[0]), int(n_final)
    n_w, n_h = int(packed.wire_ends.shape[0]), int(packed.drift.shape[0])
    n_ids = int(entrance_side.shape[0])
    sa, sb, so = int(mask_a.shape[1]), int(mask_b.shape[1]), int(mask_out.shape[1])
    _check(lib.comet_union_halves(
        _ptr(pair, torch.int32, "pair", (E, F * F)), _ptr(n_complete, torch.int32, "n_complete",
                                                           (E,)), F, E,
        _ptr(packed.event_wires, torch.int32, "event_wires", (E + 1,)),
        _ptr(packed.wire_offsets, torch.int32, "wire_offsets", (n_w + 1,)),
        _ptr(packed.hit_ids, torch.int32, "hit_ids", (n_h,)),
        _ptr(entrance_side, torch.uint8, "entrance_side", (n_ids,)), n_ids,
        _ptr(mask_a, torch.uint8, "mask_a", (E * F, sa)), sa,
        _ptr(mask_b, torch.uint8, "mask_b", (E * F, sb)), sb,
        _ptr(seeds_a, torch.float64, "seeds_a", (E * F, 6)),
        _ptr(active, torch.int32, "active", (E,)),
        _ptr(mask_out, torch.uint8, "mask_out", (E, so)), so,
        _ptr(seed_out, torch.float64, "seed_out", (E, 6)),
        _ptr(best_out, torch.int64, "best_out", (E,)), _stream()), "comet_union_halves")


def stage_update(active: torch.Tensor, best: torch.Tensor, event_wires_next: torch.Tensor,
                 n_turns: torch.Tensor, stage: int, max_stages: int, min_wires: int) -> None:
    lib = _bind_batch(load())
    n_e = int(active.shape[0])
    _check(lib.comet_stage_update(
        _ptr(active, torch.int32, "active", (n_e,)), n_e, _ptr(best, torch.int64, "best", (n_e,)),
        _ptr(event_wires_next, torch.int32, "event_wires_next", (n_e + 1,)),
        _ptr(n_turns, torch.int32, "n_turns", (n_e,)), int(stage), int(max_stages),
        int(min_wires), _stream()), "comet_stage_update")
