"""ctypes front end of the CPU FP64 reference (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg. The GPU library never imports, links or calls it.

Arrays are numpy float64 / int32 / uint8, C-contiguous. Layouts follow the C file:
seeds SoA [6][S], tracks AoS [K+1][3], wire endpoints [n_w][6], CSR offsets [n_w+1].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-Wall", "-Wextra"]


def build(src: str = SRC, out: str = LIB, extra=()) -> str:
    """Compile the oracle with gcc (plain C, no FMA contraction, OpenMP over seeds)."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, *extra, src, "-lm", "-o", tmp], check=True)
    os.replace(tmp, out)
    return out


_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u8 = ctypes.POINTER(ctypes.c_uint8)


def _bind(lib):
    lib.oracle_axis_value.restype = ctypes.c_double
    lib.oracle_axis_value.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                      ctypes.c_int32]
    lib.oracle_seed.restype = None
    lib.oracle_seed.argtypes = [_d, _i32, ctypes.c_int64, _d]
    lib.oracle_seed_grid.restype = None
    lib.oracle_seed_grid.argtypes = [_d, _i32, _d]
    lib.oracle_refine_grid.restype = None
    lib.oracle_refine_grid.argtypes = [_d, _i32, ctypes.c_int64]
    lib.oracle_track.restype = None
    lib.oracle_track.argtypes = [_d, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int32, _d]
    lib.oracle_wire_frame.restype = None
    lib.oracle_wire_frame.argtypes = [_d, _d]
    lib.oracle_dca2.restype = ctypes.c_double
    lib.oracle_dca2.argtypes = [_d, ctypes.c_int32, _d, _i32]
    lib.oracle_rss_track.restype = ctypes.c_double
    lib.oracle_rss_track.argtypes = [_d, ctypes.c_int32, _d, ctypes.c_int32, _i32, _d,
                                     ctypes.c_double]
    lib.oracle_scan.restype = ctypes.c_int32
    lib.oracle_scan.argtypes = [_d, ctypes.c_int64, _d, ctypes.c_int32, _d, ctypes.c_int32,
                                _i32, _d, _d, ctypes.c_int32]
    lib.oracle_argmin.restype = ctypes.c_int64
    lib.oracle_argmin.argtypes = [_d, ctypes.c_int64]
    lib.oracle_classify.restype = ctypes.c_int32
    lib.oracle_classify.argtypes = [_d, _d, ctypes.c_int32, _d, ctypes.c_int32, _i32, _d, _u8,
                                    _d]
    lib.oracle_scan_partition.restype = ctypes.c_int64
    lib.oracle_scan_partition.argtypes = [_d, _i32, _d, ctypes.c_int32, ctypes.c_int32, _d,
                                          ctypes.c_int32, _i32, _d, _d, _d, _d, _u8, _i32,
                                          ctypes.c_int32]
    lib.oracle_scan_partition_field.restype = ctypes.c_int64
    lib.oracle_scan_partition_field.argtypes = [_d, _i32, _d, _i32, _d, _d, ctypes.c_int32, _d,
                                                ctypes.c_int32, ctypes.c_int32, _d,
                                                ctypes.c_int32, _i32, _d, _d, _d, _d, _u8, _i32]
    lib.oracle_rss_jacobian.restype = ctypes.c_double
    lib.oracle_rss_jacobian.argtypes = [_d, _d, ctypes.c_int32, _d, ctypes.c_int32, _i32, _d, _d,
                                        _d, _d, _u8, _d]
    lib.oracle_topk.restype = None
    lib.oracle_topk.argtypes = [_d, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_layer_veto.restype = ctypes.c_int32
    lib.oracle_layer_veto.argtypes = [ctypes.POINTER(ctypes.c_uint8), _i32, ctypes.c_int32, _i32,
                                      ctypes.c_int32]
    lib.oracle_merge_halves.restype = ctypes.c_int32
    lib.oracle_merge_halves.argtypes = [_d, _i32, _d, _i32, ctypes.c_int32, _i32, _d]
    lib.oracle_exit_seed.restype = ctypes.c_int32
    lib.oracle_exit_seed.argtypes = [_d, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int32, _d]
    lib.oracle_backward_seed.restype = ctypes.c_int32
    lib.oracle_backward_seed.argtypes = [_d, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int32, _d]
    lib.oracle_stage_grid.restype = None
    lib.oracle_stage_grid.argtypes = [_d, _d, _d, _d]
    lib.oracle_stage_grids_z.restype = None
    lib.oracle_stage_grids_z.argtypes = [_d, _d, _d, ctypes.c_int32, ctypes.c_double, _d]
    lib.oracle_exclude_hits.restype = ctypes.c_int32
    lib.oracle_exclude_hits.argtypes = [ctypes.c_int32, _i32, _d, _d, ctypes.POINTER(ctypes.c_uint8),
                                        _i32, _d, _d, _i32, _i32]
    lib.oracle_rss_jacobian_field.restype = ctypes.c_double
    lib.oracle_rss_jacobian_field.argtypes = [_d, _d, _i32, _d, _d, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                              _d, ctypes.c_int32, _i32, _d, _d, _d, _d, _u8, _d,
                                              ctypes.c_int32]
    lib.oracle_lm_refine_field.restype = ctypes.c_double
    lib.oracle_lm_refine_field.argtypes = [_d, _d, _i32, _d, _d, _d, ctypes.c_int32, _d,
                                           ctypes.c_int32, _i32, _d, ctypes.c_int32,
                                           ctypes.c_double, _i32, ctypes.c_int32]
    lib.oracle_self_refine.restype = ctypes.c_int32
    lib.oracle_self_refine.argtypes = [_d, _d, ctypes.c_int32, _d, ctypes.c_int32, _i32, _d, _u8,
                                       ctypes.c_double, _u8]
    lib.oracle_field_at.restype = None
    lib.oracle_field_at.argtypes = [_d, _i32, _d, _d, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, _d]
    lib.oracle_track_field.restype = None
    lib.oracle_track_field.argtypes = [_d, _d, _i32, _d, _d, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int32, _d]
    lib.oracle_track_field_rkn.restype = None
    lib.oracle_track_field_rkn.argtypes = lib.oracle_track_field.argtypes
    lib.oracle_sparse_select.restype = ctypes.c_int32
    lib.oracle_sparse_select.argtypes = [_d, _d, ctypes.c_int32, _i32, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int64), _d, _d]
    lib.oracle_lm_refine.restype = ctypes.c_double
    lib.oracle_lm_refine.argtypes = [_d, _d, ctypes.c_int32, _d, ctypes.c_int32, _i32, _d,
                                     ctypes.c_int32, ctypes.c_double, _i32]
    return lib


def load(path: str = LIB, rebuild: bool = False):
    """Load the oracle, building it first when it is missing or older than its source."""
    global _lib
    if path == LIB and _lib is not None and not rebuild:
        return _lib
    if rebuild or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
        build(out=path)
    lib = _bind(ctypes.CDLL(path))
    if path == LIB:
        _lib = lib
    return lib


def _p(a, t=_d):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32a(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Oracle:
    """Thin numpy wrappers over one loaded oracle library."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    def axis_value(self, centre, half, n, i):
        return self.lib.oracle_axis_value(centre, half, n, i)

    def seed(self, grid, n, index):
        out = np.empty(6)
        self.lib.oracle_seed(_p(_f64(grid)), _p(_i32a(n), _i32), index, _p(out))
        return out

    def seed_grid(self, grid, n):
        n = _i32a(n)
        out = np.empty((6, int(np.prod(n.astype(np.int64)))))
        self.lib.oracle_seed_grid(_p(_f64(grid)), _p(n, _i32), _p(out))
        return out

    def refine_grid(self, grid, n, best):
        g = _f64(grid).copy()
        self.lib.oracle_refine_grid(_p(g), _p(_i32a(n), _i32), int(best))
        return g

    def track(self, seed, bz, charge, h, K):
        out = np.empty((K + 1, 3))
        self.lib.oracle_track(_p(_f64(seed)), bz, charge, h, K, _p(out))
        return out

    def wire_frame(self, ends):
        out = np.empty(8)
        self.lib.oracle_wire_frame(_p(_f64(ends)), _p(out))
        return out

    def dca2(self, pts, frame):
        pts = _f64(pts)
        k = np.zeros(1, dtype=np.int32)
        v = self.lib.oracle_dca2(_p(pts), pts.shape[0], _p(_f64(frame)), _p(k, _i32))
        return v, int(k[0])

    def rss_track(self, pts, wire_ends, offsets, drift, lam):
        pts = _f64(pts)
        ends = _f64(wire_ends)
        frames = np.stack([self.wire_frame(e) for e in ends]) if len(ends) else np.zeros((1, 8))
        return self.lib.oracle_rss_track(_p(pts), pts.shape[0], _p(_f64(frames)), len(ends),
                                         _p(_i32a(offsets), _i32), _p(_f64(drift)), lam)

    def scan(self, seeds, cfg, K, wire_ends, offsets, drift, n_threads=0):
        """RSS of every seed (seeds SoA [6][S]); returns (rss, threads used)."""
        seeds = _f64(seeds)
        S = seeds.shape[1]
        rss = np.empty(S)
        ends = _f64(wire_ends).reshape(-1, 6)
        used = self.lib.oracle_scan(_p(seeds), S, _p(_f64(cfg)), K, _p(ends), ends.shape[0],
                                    _p(_i32a(offsets), _i32), _p(_f64(drift)), _p(rss),
                                    n_threads)
        return rss, used

    def argmin(self, rss):
        rss = _f64(rss)
        return int(self.lib.oracle_argmin(_p(rss), rss.size))

    def classify(self, seed, cfg, K, wire_ends, offsets, drift):
        ends = _f64(wire_ends).reshape(-1, 6)
        drift = _f64(drift)
        mask = np.zeros(drift.size, dtype=np.uint8)
        dca = np.empty(ends.shape[0])
        nb = self.lib.oracle_classify(_p(_f64(seed)), _p(_f64(cfg)), K, _p(ends), ends.shape[0],
                                      _p(_i32a(offsets), _i32), _p(drift), _p(mask, _u8),
                                      _p(dca))
        return mask, dca, int(nb)

    def scan_partition(self, grid, n, cfg, K, n_refine, wire_ends, offsets, drift,
                       n_threads=0):
        """Coarse scan, n_refine re-scans, classification. Returns a dict."""
        g = _f64(grid).copy()
        n = _i32a(n)
        S = int(np.prod(n.astype(np.int64)))
        ends = _f64(wire_ends).reshape(-1, 6)
        drift = _f64(drift)
        rss = np.empty(S)
        best_seed = np.zeros(6)
        best_rss = np.zeros(1)
        mask = np.zeros(drift.size, dtype=np.uint8)
        nb = np.zeros(1, dtype=np.int32)
        b = self.lib.oracle_scan_partition(_p(g), _p(n, _i32), _p(_f64(cfg)), K, n_refine,
                                           _p(ends), ends.shape[0], _p(_i32a(offsets), _i32),
                                           _p(drift), _p(rss), _p(best_seed), _p(best_rss),
                                           _p(mask, _u8), _p(nb, _i32), n_threads)
        return {"best": int(b), "grid": g, "rss": rss, "best_seed": best_seed,
                "best_rss": float(best_rss[0]), "mask": mask, "n_borderline": int(nb[0])}

    def scan_partition_field(self, grid, n, fmap, stepper, cfg, K, n_refine, wire_ends, offsets,
                             drift):
        """scan_partition with tracks in a field map (cfg = [unused, charge, h, lambda])."""
        b, origin, step = fmap
        b = np.ascontiguousarray(b, dtype=np.float64)
        nmap = np.array([b.shape[2], b.shape[1], b.shape[0]], np.int32)
        g = _f64(grid).copy()
        n = _i32a(n)
        S = int(np.prod(n.astype(np.int64)))
        ends = _f64(wire_ends).reshape(-1, 6)
        drift = _f64(drift)
        rss = np.empty(S)
        best_seed = np.zeros(6)
        best_rss = np.zeros(1)
        mask = np.zeros(drift.size, dtype=np.uint8)
        nb = np.zeros(1, dtype=np.int32)
        bi = self.lib.oracle_scan_partition_field(
            _p(g), _p(n, _i32), _p(b), _p(nmap, _i32), _p(_f64(origin)), _p(_f64(step)),
            int(stepper), _p(_f64(cfg)), K, n_refine, _p(ends), ends.shape[0],
            _p(_i32a(offsets), _i32), _p(drift), _p(rss), _p(best_seed), _p(best_rss),
            _p(mask, _u8), _p(nb, _i32))
        return {"best": int(bi), "grid": g, "rss": rss, "best_seed": best_seed,
                "best_rss": float(best_rss[0]), "mask": mask, "n_borderline": int(nb[0])}

    def rss_jacobian(self, seed, cfg, K, wire_ends, offsets, drift):
        """Dual-number derivatives: dict(rss, grad[6], D[n_w], J[n_w, 6], resid[n_w], active)."""
        ends = _f64(wire_ends).reshape(-1, 6)
        n_w = ends.shape[0]
        D = np.empty(n_w)
        J = np.empty((n_w, 6))
        e = np.empty(n_w)
        act = np.zeros(n_w, dtype=np.uint8)
        grad = np.empty(6)
        rss = self.lib.oracle_rss_jacobian(_p(_f64(seed)), _p(_f64(cfg)), K, _p(ends), n_w,
                                           _p(_i32a(offsets), _i32), _p(_f64(drift)), _p(D),
                                           _p(J), _p(e), _p(act, _u8), _p(grad))
        return {"rss": rss, "grad": grad, "D": D, "J": J, "resid": e, "active": act.astype(bool)}

    def rss_jacobian_field(self, seed, fmap, charge, h, K, lam, wire_ends, offsets, drift,
                           stepper=0):
        """rss_jacobian for the track in a field map (b [nz, ny, nx, 3], origin, step)."""
        b, origin, step = fmap
        b = np.ascontiguousarray(b, dtype=np.float64)
        n = np.array([b.shape[2], b.shape[1], b.shape[0]], np.int32)
        ends = _f64(wire_ends).reshape(-1, 6)
        n_w = ends.shape[0]
        D, J, e = np.empty(n_w), np.empty((n_w, 6)), np.empty(n_w)
        act = np.zeros(n_w, dtype=np.uint8)
        grad = np.empty(6)
        rss = self.lib.oracle_rss_jacobian_field(
            _p(_f64(seed)), _p(b), _p(n, _i32), _p(_f64(origin)), _p(_f64(step)), float(charge),
            float(h), int(K), float(lam), _p(ends), n_w, _p(_i32a(offsets), _i32),
            _p(_f64(drift)), _p(D), _p(J), _p(e), _p(act, _u8), _p(grad), int(stepper))
        return {"rss": rss, "grad": grad, "D": D, "J": J, "resid": e, "active": act.astype(bool)}

    def lm_refine_field(self, seed, fmap, cfg, K, wire_ends, offsets, drift, n_iter, mu0,
                        stepper=0):
        """lm_refine with tracks in a field map (cfg = [unused, charge, h, lambda])."""
        b, origin, step = fmap
        b = np.ascontiguousarray(b, dtype=np.float64)
        n = np.array([b.shape[2], b.shape[1], b.shape[0]], np.int32)
        s = _f64(seed).copy()
        ends = _f64(wire_ends).reshape(-1, 6)
        acc = np.zeros(1, dtype=np.int32)
        rss = self.lib.oracle_lm_refine_field(_p(s), _p(b), _p(n, _i32), _p(_f64(origin)),
                                              _p(_f64(step)), _p(_f64(cfg)), int(K), _p(ends),
                                              ends.shape[0], _p(_i32a(offsets), _i32),
                                              _p(_f64(drift)), int(n_iter), float(mu0),
                                              _p(acc, _i32), int(stepper))
        return s, rss, int(acc[0])

    def lm_refine(self, seed, cfg, K, wire_ends, offsets, drift, n_iter, mu0):
        """Levenberg-Marquardt refinement of one seed: (seed[6], rss, accepted steps)."""
        s = _f64(seed).copy()
        ends = _f64(wire_ends).reshape(-1, 6)
        acc = np.zeros(1, dtype=np.int32)
        rss = self.lib.oracle_lm_refine(_p(s), _p(_f64(cfg)), K, _p(ends), ends.shape[0],
                                        _p(_i32a(offsets), _i32), _p(_f64(drift)), n_iter,
                                        float(mu0), _p(acc, _i32))
        return s, rss, int(acc[0])

    def sparse_select(self, grids, rss, n, n_ref):
        """Sparse reference seeds of one group of sub-grids: (idx, rss, new_grids, taken)."""
        grids = _f64(grids).reshape(-1, 14)
        rss = _f64(rss).ravel()
        idx = np.empty(n_ref, dtype=np.int64)
        rr = np.empty(n_ref)
        ng = np.empty((n_ref, 14))
        taken = self.lib.oracle_sparse_select(_p(grids), _p(rss), grids.shape[0],
                                              _p(_i32a(n), _i32), n_ref,
                                              idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                              _p(rr), _p(ng))
        return idx, rr, ng, int(taken)

    def layer_veto(self, mask, wire_offsets, wire_layer, n_layers):
        """1 vetoed, 0 kept, -1 a layer out of range (one classified seed of a half)."""
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        if m.size == 0:
            m = np.zeros(1, np.uint8)
        off = _i32a(wire_offsets)
        lay = _i32a(wire_layer)
        return int(self.lib.oracle_layer_veto(m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                              _p(off, _i32), off.size - 1, _p(lay, _i32),
                                              int(n_layers)))

    def merge_halves(self, rss_a, veto_a, rss_b, veto_b):
        """Ranked complete sets of two half sets: (pair, pair_rss, count)."""
        ra, rb = _f64(rss_a).ravel(), _f64(rss_b).ravel()
        va, vb = _i32a(veto_a), _i32a(veto_b)
        F = ra.size
        pair = np.empty(F * F, np.int32)
        prss = np.empty(F * F)
        n = self.lib.oracle_merge_halves(_p(ra), _p(va, _i32), _p(rb), _p(vb, _i32), F,
                                         _p(pair, _i32), _p(prss))
        return pair, prss, int(n)

    def backward_seed(self, seed6, bz, charge, h, radius, max_steps):
        """State at the previous turn's entry through r = radius: (out6, steps)."""
        out = np.empty(6)
        k = self.lib.oracle_backward_seed(_p(_f64(seed6)), bz, charge, h, radius, max_steps,
                                          _p(out))
        return out, int(k)

    def exit_seed(self, seed6, bz, charge, h, radius, max_steps):
        """The exit half track's seed: the state where the turn re-enters r = radius,
        momentum reversed: (out6, steps)."""
        out = np.empty(6)
        k = self.lib.oracle_exit_seed(_p(_f64(seed6)), bz, charge, h, radius, max_steps, _p(out))
        return out, int(k)

    def stage_grid(self, transverse6, ext6, half):
        g = np.empty(14)
        self.lib.oracle_stage_grid(_p(_f64(transverse6)), _p(_f64(ext6)), _p(_f64(half)), _p(g))
        return g

    def stage_grids_z(self, transverse6, ext6, half, n_z, z_half):
        g = np.empty((n_z, 14))
        self.lib.oracle_stage_grids_z(_p(_f64(transverse6)), _p(_f64(ext6)), _p(_f64(half)),
                                      int(n_z), float(z_half), _p(g))
        return g

    def exclude_hits(self, offsets, drift, ends, exclude):
        """(offsets, drift, ends, wire_map, hit_map) without the excluded hits."""
        off = _i32a(offsets)
        nw = off.size - 1
        nh = int(off[-1])
        ex = np.ascontiguousarray(exclude, dtype=np.uint8)
        if ex.size == 0:
            ex = np.zeros(1, np.uint8)
        o2 = np.empty(nw + 1, np.int32)
        d2 = np.empty(max(nh, 1))
        e2 = np.empty((max(nw, 1), 6))
        wm = np.empty(max(nw, 1), np.int32)
        hm = np.empty(max(nh, 1), np.int32)
        n = self.lib.oracle_exclude_hits(nw, _p(off, _i32), _p(_f64(drift) if nh else np.zeros(1)),
                                         _p(_f64(ends).reshape(-1) if nw else np.zeros(6)),
                                         ex.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                         _p(o2, _i32), _p(d2), _p(e2), _p(wm, _i32), _p(hm, _i32))
        n_h = int(o2[n])
        return o2[:n + 1].copy(), d2[:n_h].copy(), e2[:n].copy(), wm[:n].copy(), hm[:n_h].copy()

    def self_refine(self, seed_fit, cfg, K, wire_ends, offsets, drift, mask_in, eta):
        """Classified hits after the self-refining at the fitted seed: (mask, n)."""
        ends = _f64(wire_ends).reshape(-1, 6)
        drift = _f64(drift)
        m_in = np.ascontiguousarray(mask_in, dtype=np.uint8)
        out = np.zeros(max(drift.size, 1), dtype=np.uint8)
        if m_in.size == 0:
            m_in = np.zeros(1, np.uint8)
        n = self.lib.oracle_self_refine(_p(_f64(seed_fit)), _p(_f64(cfg)), K, _p(ends),
                                        ends.shape[0], _p(_i32a(offsets), _i32),
                                        _p(drift if drift.size else np.zeros(1)), _p(m_in, _u8),
                                        float(eta), _p(out, _u8))
        return out[:drift.size].copy(), int(n)

    def field_at(self, fmap, x, y, z):
        """B (tesla) of a field map (b [nz, ny, nx, 3], origin [3], step [3]) at a point."""
        b, origin, step = fmap
        b = _f64(b)
        n = np.array([b.shape[2], b.shape[1], b.shape[0]], np.int32)
        out = np.empty(3)
        self.lib.oracle_field_at(_p(b), _p(n, _i32), _p(_f64(origin)), _p(_f64(step)), x, y, z,
                                 _p(out))
        return out

    def track_field(self, seed, fmap, charge, h, K, stepper=0):
        """Track in a field map, RK4 (stepper 0) or RKN (1): [K + 1, 3] positions."""
        b, origin, step = fmap
        b = _f64(b)
        n = np.array([b.shape[2], b.shape[1], b.shape[0]], np.int32)
        pts = np.empty((K + 1, 3))
        fn = self.lib.oracle_track_field_rkn if stepper == 1 else self.lib.oracle_track_field
        fn(_p(_f64(seed)), _p(b), _p(n, _i32), _p(_f64(origin)), _p(_f64(step)), charge, h, K,
           _p(pts))
        return pts

    def topk(self, values, k):
        v = _f64(values)
        out = np.empty(k, dtype=np.int64)
        self.lib.oracle_topk(_p(v), v.size, k, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        return out
