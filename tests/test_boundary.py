"""The C ABI on the host: every declared symbol is exported, and host-visible
argument errors are rejected before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1911_09340_amd import comet

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "comet.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(comet_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return comet.load()


def test_header_declares_the_three_calls():
    names = declared_functions()
    for n in ("comet_extrapolate_seeds", "comet_dca_rss", "comet_select_classify"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for st in (comet.OK, comet.EINVAL, comet.EWORKSPACE, comet.EHIP, comet.EUNSUPPORTED):
        assert comet.status_string(st) and comet.status_string(st) != "unknown status"
    assert comet.status_string(42) == "unknown status"
    assert lib.comet_version() >= 100


def _cfg(**kw):
    c = dict(bz=1.0, charge=-1.0, step_mm=2.0, n_steps=10, lambda_mm=1.0)
    c.update(kw)
    return comet.make_config(**c)


def _p(v=0x1000):
    return ctypes.c_void_p(v)


def _n4(*n):
    return (ctypes.c_int32 * 4)(*n)


def test_workspace_bytes(lib):
    assert lib.comet_dca_workspace_bytes(0, 11, 10) == 0
    assert lib.comet_dca_workspace_bytes(10, 11, -1) == 0
    assert lib.comet_dca_workspace_bytes(10, 0, 10) == 0
    a = lib.comet_dca_workspace_bytes(64, 11, 10)
    b = lib.comet_dca_workspace_bytes(128, 11, 10)
    c = lib.comet_dca_workspace_bytes(64, 1001, 10)
    assert a % 256 == 0 and b > a and c > a
    # frames, d^2 per (wire, seed), one chunk radius per 16 points and seed
    assert c >= 8 * 64 * 10 + 8 * 8 * 10 + 8 * 64 * 63


@pytest.mark.parametrize("case", ["null_grid", "bad_n", "count_mismatch"])
def test_seed_grid_rejects(lib, case):
    n = _n4(2, 2, 2, 2)
    args = {"null_grid": (None, n, _p(), 16), "bad_n": (_p(), _n4(2, 0, 2, 2), _p(), 0),
            "count_mismatch": (_p(), n, _p(), 17)}[case]
    assert lib.comet_seed_grid(*args, None) == comet.EINVAL
    assert lib.comet_last_error()


@pytest.mark.parametrize("field,value", [("n_steps", 0), ("step_mm", 0.0), ("step_mm", float("nan")),
                                          ("lambda_mm", -1.0), ("lambda_mm", float("inf")),
                                          ("bz", float("nan")), ("charge", float("inf"))])
def test_extrapolate_rejects_config(lib, field, value):
    cfg = _cfg(**{field: value})
    assert lib.comet_extrapolate_seeds(_p(), 64, ctypes.byref(cfg), _p(), None) == comet.EINVAL


def test_extrapolate_rejects_pointers_and_sizes(lib):
    cfg = _cfg()
    assert lib.comet_extrapolate_seeds(None, 64, ctypes.byref(cfg), _p(), None) == comet.EINVAL
    assert lib.comet_extrapolate_seeds(_p(), 0, ctypes.byref(cfg), _p(), None) == comet.EINVAL
    assert lib.comet_extrapolate_seeds(_p(), 64, None, _p(), None) == comet.EINVAL
    bad = _cfg()
    bad.reserved = 1
    assert lib.comet_extrapolate_seeds(_p(), 64, ctypes.byref(bad), _p(), None) == comet.EINVAL


def _dca(lib, track=_p(), S=64, P=11, ends=_p(), n_w=4, offs=_p(), drift=_p(), n_h=5, cfg=None,
         rss=_p(), ws=_p(0x100000), ws_bytes=1 << 30):
    cfg = cfg or _cfg()
    return lib.comet_dca_rss(track, S, P, ends, n_w, offs, drift, n_h, ctypes.byref(cfg), rss, ws,
                             ws_bytes, None)


def test_dca_rss_rejects(lib):
    assert _dca(lib, track=None) == comet.EINVAL
    assert _dca(lib, rss=None) == comet.EINVAL
    assert _dca(lib, S=0) == comet.EINVAL
    assert _dca(lib, P=10) == comet.EINVAL          # n_points != n_steps + 1
    assert _dca(lib, n_w=-1) == comet.EINVAL
    assert _dca(lib, ends=None) == comet.EINVAL
    assert _dca(lib, offs=None) == comet.EINVAL
    assert _dca(lib, drift=None) == comet.EINVAL
    assert _dca(lib, cfg=_cfg(lambda_mm=0.0)) == comet.EINVAL
    assert _dca(lib, ws=None) == comet.EWORKSPACE
    assert _dca(lib, ws_bytes=16) == comet.EWORKSPACE
    assert _dca(lib, ws=_p(0x100008)) == comet.EINVAL  # misaligned


def test_select_classify_rejects(lib):
    cfg = _cfg()
    best = _p()
    # top_k must be in [1, 1024]
    for k in (0, 1025):
        assert lib.comet_select_classify(_p(), 64, None, 0, None, 0, None, None, 0,
                                         ctypes.byref(cfg), k, best, None, None, None,
                                         None) == comet.EINVAL
    assert lib.comet_select_classify(None, 64, None, 0, None, 0, None, None, 0, ctypes.byref(cfg),
                                     1, best, None, None, None, None) == comet.EINVAL
    assert lib.comet_select_classify(_p(), 64, None, 0, None, 0, None, None, 0, ctypes.byref(cfg),
                                     1, None, None, None, None, None) == comet.EINVAL
    # classification needs the track and a matching point count
    assert lib.comet_select_classify(_p(), 64, None, 11, _p(), 4, _p(), _p(), 5, ctypes.byref(cfg),
                                     1, best, _p(), None, None, None) == comet.EINVAL
    assert lib.comet_select_classify(_p(), 64, _p(), 12, _p(), 4, _p(), _p(), 5, ctypes.byref(cfg),
                                     1, best, _p(), None, None, None) == comet.EINVAL


def test_refine_rejects(lib):
    assert lib.comet_refine_grid(None, _n4(2, 2, 2, 2), _p(), None) == comet.EINVAL
    assert lib.comet_refine_grid(_p(), _n4(2, 2, 0, 2), _p(), None) == comet.EINVAL


def test_valid_call_without_gpu_fails_loudly(lib):
    """On a machine without a GPU a well-formed call reports a HIP error; nothing
    falls back to the CPU."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cfg = _cfg()
    st = lib.comet_extrapolate_seeds(_p(), 64, ctypes.byref(cfg), _p(), None)
    assert st in (comet.EHIP, comet.EUNSUPPORTED)
    assert lib.comet_last_error()


def test_binding_validates_tensors():
    import torch
    cfg = _cfg()
    with pytest.raises(ValueError):
        comet.extrapolate_seeds(torch.zeros(6, 64, dtype=torch.float64), cfg,
                                torch.zeros(3, 11, 64, dtype=torch.float64))


def test_adjoint_and_lm_reject(lib):
    comet._bind_derivatives(lib)
    cfg = _cfg()
    ok = (_p(), 8, ctypes.byref(cfg), _p(), 4, _p(), _p(), 5)
    assert lib.comet_rss_adjoint(None, *ok[1:], None, None, *([None] * 7), None) == comet.EINVAL
    assert lib.comet_rss_adjoint(*ok, _p(), None, *([None] * 7), None) == comet.EINVAL
    long_cfg = _cfg(n_steps=5000)
    assert lib.comet_rss_adjoint(_p(), 8, ctypes.byref(long_cfg), _p(), 4, _p(), _p(), 5, None,
                                 None, *([None] * 7), None) == comet.EUNSUPPORTED
    need = lib.comet_lm_workspace_bytes(8, 10)
    assert need > 0 and need % 256 == 0
    args = ok + (None, None)
    assert lib.comet_lm_refine(*args, 4, 1e-3, _p(), None, _p(0x100000), 16, None) == comet.EWORKSPACE
    assert lib.comet_lm_refine(*args, -1, 1e-3, _p(), None, _p(0x100000), need, None) == comet.EINVAL
    assert lib.comet_lm_refine(*args, 4, 0.0, _p(), None, _p(0x100000), need, None) == comet.EINVAL
    assert lib.comet_lm_refine(*args, 4, 1e-3, None, None, _p(0x100000), need, None) == comet.EINVAL


def test_batch_topk_and_seed_rejects(lib):
    comet._bind_batch(lib)
    assert lib.comet_topk(None, 10, 1, 1, _p(), None) == comet.EINVAL
    assert lib.comet_topk(_p(), 10, 1, 0, _p(), None) == comet.EINVAL
    assert lib.comet_topk(_p(), 0, 1, 1, _p(), None) == comet.EINVAL
    assert lib.comet_grid_seeds(_p(), 2, _n4(2, 2, 0, 2), _p(), 1, _p(), None) == comet.EINVAL
    need = lib.comet_batch_workspace_bytes(100, 1000, 7)
    assert need > 0 and need % 256 == 0
    cfg = _cfg()
    args = [_p(), 10, _p(), _p(), 20, _p(), 2, _p(), 3, None, _p(), _n4(2, 2, 2, 2),
            ctypes.byref(cfg), 1, _p(), _p(), None, None, None, 0, None, 0]
    ws = lib.comet_batch_workspace_bytes(10, 10, 3)
    assert lib.comet_batch_scan(*args, _p(0x100000), 16, None) == comet.EWORKSPACE
    bad = list(args)
    bad[13] = -1  # n_refine
    assert lib.comet_batch_scan(*bad, _p(0x100000), ws, None) == comet.EINVAL
    bad = list(args)
    bad[0] = None
    assert lib.comet_batch_scan(*bad, _p(0x100000), ws, None) == comet.EINVAL
    # the active-events form: event_active in place of max_items, and required
    act = args[:21]
    assert lib.comet_batch_scan_active(*act, None, _p(0x100000), ws, None) == comet.EINVAL
    assert lib.comet_batch_scan_active(*act, _p(), _p(0x100000), 16, None) == comet.EWORKSPACE


def test_static_workspace_call_rejects(lib):
    """The allocation-free entry point checks sizes against its fixed array before any
    device work, and its arguments as the workspace form does."""
    lib.comet_static_scratch_bytes.restype = ctypes.c_size_t
    cap = lib.comet_static_scratch_bytes()
    assert cap == 64 << 20
    lib.comet_dca_workspace_bytes.restype = ctypes.c_size_t
    lib.comet_dca_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
    assert lib.comet_dca_workspace_bytes(65536, 1501, 172) > cap
    assert lib.comet_dca_workspace_bytes(8192, 1501, 172) <= cap
    lib.comet_track_dca_rss_static.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.comet_track_dca_rss_static.restype = ctypes.c_int
    cfg = comet.make_config(1.0, -1.0, 2.0, 1500, 0.8)
    st = lib.comet_track_dca_rss_static(_p(), 65536, ctypes.byref(cfg), None, _p(), 172, _p(),
                                        _p(), 200, _p(), _p(), None)
    assert st == comet.EWORKSPACE and b"split the seeds" in lib.comet_last_error()
    st = lib.comet_track_dca_rss_static(None, 64, ctypes.byref(cfg), None, _p(), 172, _p(),
                                        _p(), 200, _p(), _p(), None)
    assert st == comet.EINVAL


def test_sparse_select_and_classify_reject(lib):
    comet._bind_batch(lib)
    n = _n4(2, 3, 1, 4)
    ok = [_p(), _p(), 3, 2, n, 10, _p(), None, _p(), None, None, None]

    def call(**kw):
        a = list(ok)
        names = ["grids", "rss", "n_groups", "n_sub", "n", "n_ref", "ref_idx", "ref_rss",
                 "new_grids", "ref_grids", "ref_local", "stream"]
        for k, v in kw.items():
            a[names.index(k)] = v
        return lib.comet_sparse_select(*a)

    assert call(grids=None) == comet.EINVAL
    assert call(rss=None) == comet.EINVAL
    assert call(ref_idx=None) == comet.EINVAL
    assert call(new_grids=None) == comet.EINVAL
    assert call(n_groups=0) == comet.EINVAL
    assert call(n_sub=0) == comet.EINVAL
    assert call(n_ref=0) == comet.EINVAL
    assert call(n_ref=65) == comet.EINVAL
    assert call(n=_n4(2, 0, 1, 4)) == comet.EINVAL
    assert call(n=_n4(1024, 1024, 1024, 2), n_sub=1) == comet.EINVAL   # 2^31 candidates
    cfg = _cfg()
    args = [_p(), 3, n, _p(), _p(), _p(), 10, _p(), _p(), 20, _p(), 2, _p(), ctypes.byref(cfg),
            None, None, None, 0, None, None]
    for i in (0, 3, 5, 7, 10, 12):                        # required pointers
        bad = list(args)
        bad[i] = None
        assert lib.comet_batch_classify(*bad) == comet.EINVAL, i
    bad = list(args)
    bad[4], bad[15] = None, _p()                          # best_rss needs rss
    assert lib.comet_batch_classify(*bad) == comet.EINVAL
    bad = list(args)
    bad[16], bad[17] = _p(), 0                            # mask without a stride
    assert lib.comet_batch_classify(*bad) == comet.EINVAL
    bad = list(args)
    bad[1] = 0
    assert lib.comet_batch_classify(*bad) == comet.EINVAL
    long_cfg = _cfg(n_steps=5000)
    bad = list(args)
    bad[13] = ctypes.byref(long_cfg)
    assert lib.comet_batch_classify(*bad) == comet.EUNSUPPORTED


def test_layer_veto_and_merge_reject(lib):
    comet._bind_batch(lib)
    ok = [_p(), 16, 4, _p(), _p(), 2, _p(), _p(), 30, 18, _p(), None]
    for i in (0, 3, 4, 6, 7, 10):
        bad = list(ok)
        bad[i] = None
        assert lib.comet_layer_veto(*bad) == comet.EINVAL, i
    for i, v in ((1, 0), (2, 0), (5, 0), (9, 0), (9, 257)):
        bad = list(ok)
        bad[i] = v
        assert lib.comet_layer_veto(*bad) == comet.EINVAL, (i, v)
    ok = [_p(), _p(), _p(), _p(), 5, 10, _p(), _p(), None, None]
    for i in (0, 1, 2, 3, 6, 7):
        bad = list(ok)
        bad[i] = None
        assert lib.comet_merge_halves(*bad) == comet.EINVAL, i
    for i, v in ((4, 0), (5, 0), (5, 33)):
        bad = list(ok)
        bad[i] = v
        assert lib.comet_merge_halves(*bad) == comet.EINVAL, (i, v)


def test_stage_calls_reject(lib):
    comet._bind_batch(lib)
    cfg = _cfg()
    assert lib.comet_backward_seeds(None, 3, ctypes.byref(cfg), 500.0, 10, _p(), None, None) == comet.EINVAL
    assert lib.comet_backward_seeds(_p(), 0, ctypes.byref(cfg), 500.0, 10, _p(), None, None) == comet.EINVAL
    assert lib.comet_backward_seeds(_p(), 3, ctypes.byref(cfg), -1.0, 10, _p(), None, None) == comet.EINVAL
    assert lib.comet_backward_seeds(_p(), 3, ctypes.byref(cfg), 500.0, 0, _p(), None, None) == comet.EINVAL
    half = (ctypes.c_double * 4)(1.0, 1.0, -1.0, 1.0)
    assert lib.comet_stage_grids(_p(), _p(), 3, half, _p(), None) == comet.EINVAL
    assert lib.comet_exclude_workspace_bytes(0) == 0
    need = lib.comet_exclude_workspace_bytes(10)
    assert need >= 120 and need % 256 == 0
    args = [_p(), 2, _p(), 10, _p(), _p(), _p(), 20, _p(), _p(), _p(), _p(), _p(), _p()]
    assert lib.comet_exclude_hits(*args, _p(0x100000), 16, None) == comet.EWORKSPACE
    bad = list(args)
    bad[0] = None
    assert lib.comet_exclude_hits(*bad, _p(0x100000), need, None) == comet.EINVAL
    assert lib.comet_stage_record(_p(), 0, 2, _p(), _p(), _p(), _p(), 0, _p(), _p(), None) == comet.EINVAL
    assert lib.comet_stage_update(_p(), 2, _p(), _p(), _p(), 0, 0, 30, None) == comet.EINVAL
    ok = [_p(), 4, _p(), ctypes.byref(cfg), _p(), 10, _p(), _p(), 20, _p(), 4, 0.3, _p(), _p(),
          32, None]
    for i in (0, 2, 4, 6, 7, 9, 12, 13):
        bad = list(ok)
        bad[i] = None
        assert lib.comet_self_refine(*bad) == comet.EINVAL, i
    for i, v in ((1, 0), (10, 0), (14, 0), (11, -0.1), (11, float("nan")), (11, float("inf"))):
        bad = list(ok)
        bad[i] = v
        assert lib.comet_self_refine(*bad) == comet.EINVAL, (i, v)
    long_cfg = comet.make_config(1.0, -1.0, 1.0, 2401, 0.8)
    bad = list(ok)
    bad[3] = ctypes.byref(long_cfg)
    assert lib.comet_self_refine(*bad) == comet.EUNSUPPORTED


def test_chain_calls_reject(lib):
    """The per-stage chain's joins reject NULL pointers and bad sizes before device work."""
    comet._bind_batch(lib)
    cfg = _cfg()
    ok = [_p(), 14, 3, ctypes.byref(cfg), 500.0, 10, _p(), None, None]
    assert lib.comet_exit_seeds(*ok) != comet.EINVAL        # valid: fails later (no GPU)
    for i, v in ((0, None), (6, None), (1, 5), (2, 0), (4, -1.0), (4, float("nan")), (5, 0)):
        bad = list(ok)
        bad[i] = v
        assert lib.comet_exit_seeds(*bad) == comet.EINVAL, (i, v)
    ok = [_p(), 2, _p(), _p(), 20, _p(), 20, _p(), _p(), None]
    for i in (0, 2, 3, 5, 7, 8):
        bad = list(ok)
        bad[i] = None
        assert lib.comet_half_split(*bad) == comet.EINVAL, i
    for i in (1, 4, 6):
        bad = list(ok)
        bad[i] = 0
        assert lib.comet_half_split(*bad) == comet.EINVAL, i
    ok = [_p(), 2, _p(), 10, _p(), _p(), 20, _p(), None]
    for i in (0, 2, 4, 5, 7):
        bad = list(ok)
        bad[i] = None
        assert lib.comet_wire_layers(*bad) == comet.EINVAL, i
    for i in (1, 3, 6):
        bad = list(ok)
        bad[i] = 0
        assert lib.comet_wire_layers(*bad) == comet.EINVAL, i
    ok = [_p(), _p(), 4, 2, _p(), _p(), _p(), _p(), 20, _p(), 8, _p(), 8, _p(), _p(), _p(), 8,
          _p(), _p(), None]
    for i in (0, 1, 4, 5, 6, 7, 9, 11, 13, 14, 15, 17, 18):
        bad = list(ok)
        bad[i] = None
        assert lib.comet_union_halves(*bad) == comet.EINVAL, i
    for i, v in ((2, 0), (2, 65), (3, 0), (8, 0), (10, 0), (12, 0), (16, 0)):
        bad = list(ok)
        bad[i] = v
        assert lib.comet_union_halves(*bad) == comet.EINVAL, (i, v)


def test_field_call_rejects(lib):
    lib.comet_extrapolate_seeds_field.argtypes = [ctypes.c_void_p, ctypes.c_int64,
                                                  ctypes.POINTER(comet.Config),
                                                  ctypes.POINTER(comet.Field), ctypes.c_void_p,
                                                  ctypes.c_void_p]
    cfg = _cfg()
    good = comet.Field(_p(), 3, 3, 3, 0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    assert lib.comet_extrapolate_seeds_field(None, 4, ctypes.byref(cfg), ctypes.byref(good), _p(), None) == comet.EINVAL
    for field in (comet.Field(None, 3, 3, 3, 0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0),
                  comet.Field(_p(), 1, 3, 3, 0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0),
                  comet.Field(_p(), 3, 3, 3, 2, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0),
                  comet.Field(_p(), 3, 3, 3, 0, 0.0, 0.0, 0.0, 1.0, 0.0, 1.0)):
        assert lib.comet_extrapolate_seeds_field(_p(), 4, ctypes.byref(cfg), ctypes.byref(field),
                                                 _p(), None) == comet.EINVAL


def test_field_derivative_calls_reject(lib):
    comet._bind_derivatives(lib)
    cfg = _cfg()
    good = comet.Field(_p(), 3, 3, 3, 0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    bad_field = comet.Field(_p(), 3, 1, 3, 0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    outs = [None] * 7
    args = [_p(), 4, ctypes.byref(cfg), ctypes.byref(good), _p(), 10, _p(), _p(), 20, None, None]
    bad = list(args)
    bad[0] = None
    assert lib.comet_rss_jacobian_field(*bad, *outs, None) == comet.EINVAL
    bad = list(args)
    bad[3] = None
    assert lib.comet_rss_jacobian_field(*bad, *outs, None) == comet.EINVAL
    bad[3] = ctypes.byref(bad_field)
    assert lib.comet_rss_jacobian_field(*bad, *outs, None) == comet.EINVAL
    bad = list(args)
    bad[9] = _p()                                   # event_wires without seed_event
    assert lib.comet_rss_jacobian_field(*bad, *outs, None) == comet.EINVAL
    long_cfg = comet.make_config(1.0, -1.0, 1.0, 2401, 0.8)
    bad = list(args)
    bad[2] = ctypes.byref(long_cfg)
    assert lib.comet_rss_jacobian_field(*bad, *outs, None) == comet.EUNSUPPORTED
    lm = [_p(), 4, ctypes.byref(cfg), ctypes.byref(good), _p(), 10, _p(), _p(), 20, None, None,
          8, 1e-3, _p(), None]
    assert lib.comet_lm_refine_field(*lm, _p(0x100000), 16, None) == comet.EWORKSPACE
    bad = list(lm)
    bad[3] = ctypes.byref(bad_field)
    assert lib.comet_lm_refine_field(*bad, _p(0x100000), 1 << 20, None) == comet.EINVAL
    bad = list(lm)
    bad[12] = 0.0
    assert lib.comet_lm_refine_field(*bad, _p(0x100000), 1 << 20, None) == comet.EINVAL


def test_batch_field_calls_reject(lib):
    comet._bind_batch(lib)
    cfg = _cfg()
    n4 = (ctypes.c_int32 * 4)(2, 2, 2, 2)
    bad_field = comet.Field(_p(), 3, 3, 3, 7, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    for field in (None, ctypes.byref(bad_field)):
        assert lib.comet_batch_scan_field(
            _p(), 10, _p(), _p(), 20, _p(), 2, _p(), 3, None, _p(), n4, ctypes.byref(cfg),
            field, 0, _p(), _p(), None, None, None, 0, None, 0, _p(0x100000), 1 << 30,
            None) == comet.EINVAL
    lib.comet_batch_classify_field.argtypes = [ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                               ctypes.POINTER(comet.Config),
                                               ctypes.POINTER(comet.Field), ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                               ctypes.c_void_p, ctypes.c_void_p]
    lib.comet_batch_classify_field.restype = ctypes.c_int
    for field in (None, ctypes.byref(bad_field)):
        assert lib.comet_batch_classify_field(
            _p(), 3, n4, _p(), _p(), _p(), 10, _p(), _p(), 20, _p(), 2, _p(), ctypes.byref(cfg),
            field, None, None, None, 0, None, None) == comet.EINVAL
