"""Seeded synthetic CDC-like events: the stand-in for the paper's Geant4 samples.

The paper evaluates its seed scan on simulated COMET Phase-I electrons in the
cylindrical drift chamber (Sec. 1 for the chamber, Sec. 3.2 for the samples).
Those samples are not available, so this module draws events of the same shape:
an 18-layer stereo chamber in a uniform axial field, one electron helix per
event (with a small kink and energy loss at each return through the target
region, standing in for multiple scattering between turns), drift distances
smeared by a Gaussian and clipped to the cell, and optional noise hits.

This module only draws inputs. It holds none of the seed-scan arithmetic (no
stepping, no closest-approach search, no residual sums): the truth hits come
from the closed-form helix and a golden-section search of the helix-to-wire
distance, written independently of both the CPU reference and the GPU library.
Both of those consume its output; neither is imported here.

Units: mm, MeV/c, tesla, charge in units of e.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

KAPPA = 0.299792458  # MeV/c per (T * mm): p_T = KAPPA * |q| * B * R

# Chamber stand-in (Sec. 1: 18 sense layers, stereo tilt ~0.07 rad alternating
# in sign per layer, 1 T solenoid field).
N_LAYERS = 18
WIRES_PER_LAYER = 320
N_WIRES = N_LAYERS * WIRES_PER_LAYER
R_FIRST = 530.0
R_LAST = 830.0
STEREO = 0.070
HALF_LENGTH = 750.0
DRIFT_MAX = 8.0
SEED_RADIUS = 500.0  # seeds sit at a fixed radius in front of the first layer (Sec. 3.1)


def layer_radius(layer):
    return R_FIRST + np.asarray(layer, dtype=np.float64) * ((R_LAST - R_FIRST) / (N_LAYERS - 1))


def chamber_wires() -> np.ndarray:
    """Endpoints of every sense wire, shape [N_WIRES, 6] = (A, B).

    Wire id = layer * 320 + index. Wire w of layer l passes through
    (r_l cos f, r_l sin f, 0), f = 2 pi (w + (l mod 2) / 2) / 320, with direction
    cos(a) z + sin(a) phi_hat, a = +0.07 on even layers and -0.07 on odd ones;
    its endpoints sit at z = -750 and z = +750 mm.
    """
    layer = np.repeat(np.arange(N_LAYERS), WIRES_PER_LAYER)
    idx = np.tile(np.arange(WIRES_PER_LAYER), N_LAYERS)
    r = layer_radius(layer)
    f = 2.0 * np.pi * (idx + 0.5 * (layer % 2)) / WIRES_PER_LAYER
    a = np.where(layer % 2 == 0, STEREO, -STEREO)
    mid = np.stack([r * np.cos(f), r * np.sin(f), np.zeros_like(r)], axis=1)
    phi_hat = np.stack([-np.sin(f), np.cos(f), np.zeros_like(r)], axis=1)
    d = np.cos(a)[:, None] * np.array([0.0, 0.0, 1.0]) + np.sin(a)[:, None] * phi_hat
    t = (HALF_LENGTH / np.cos(a))[:, None]
    return np.concatenate([mid - t * d, mid + t * d], axis=1)


_WIRES = None


def _wires():
    global _WIRES
    if _WIRES is None:
        _WIRES = chamber_wires()
    return _WIRES


# ---------------------------------------------------------------- helix
def helix_state(state0, charge: float, bz: float, s) -> np.ndarray:
    """Exact state after arc length s in a uniform field B = (0, 0, bz).

    The Lorentz force turns the transverse momentum at the constant rate
    c = KAPPA q B / |p| per unit path (clockwise seen from +z for c > 0):
    p_T(s) = p_T(0) exp(-i c s), x_T(s) = x_T(0) + i p_T(0) (exp(-i c s) - 1) / (|p| c),
    z(s) = z(0) + s p_z / |p|. Returns [..., 6].
    """
    x0, y0, z0, px, py, pz = (float(v) for v in state0)
    s = np.asarray(s, dtype=np.float64)
    p = np.sqrt(px * px + py * py + pz * pz)
    c = KAPPA * charge * bz / p
    p0 = complex(px, py)
    rot = np.exp(-1j * c * s)
    pt = p0 * rot
    if c == 0.0:
        xt = complex(x0, y0) + (p0 / p) * s
    else:
        xt = complex(x0, y0) + (1j * p0 / (p * c)) * (rot - 1.0)
    z = z0 + (pz / p) * s
    return np.stack([xt.real, xt.imag, np.broadcast_to(z, xt.shape), pt.real, pt.imag,
                     np.broadcast_to(np.float64(pz), xt.shape)], axis=-1)


def turn_length(state0, charge: float, bz: float) -> float:
    """Path length of one transverse revolution."""
    px, py, pz = state0[3], state0[4], state0[5]
    p = np.sqrt(px * px + py * py + pz * pz)
    return 2.0 * np.pi * p / (KAPPA * abs(charge) * bz)


def _line_distance(pts, a, u):
    """Distance from points [..., 3] to the infinite lines through a with unit direction u."""
    d = pts - a
    cx = d[..., 1] * u[..., 2] - d[..., 2] * u[..., 1]
    cy = d[..., 2] * u[..., 0] - d[..., 0] * u[..., 2]
    cz = d[..., 0] * u[..., 1] - d[..., 1] * u[..., 0]
    return np.sqrt(cx * cx + cy * cy + cz * cz)


def _outward_crossing(state0, charge, bz, s_len, radius=SEED_RADIUS, ds=0.5):
    """First arc length in [0, s_len] where the helix crosses `radius` outward (None if none)."""
    s = np.arange(0.0, s_len + ds, ds)
    st = helix_state(state0, charge, bz, s)
    r = np.hypot(st[:, 0], st[:, 1])
    up = np.nonzero((r[:-1] < radius) & (r[1:] >= radius))[0]
    if up.size == 0:
        return None
    lo, hi = s[up[0]], s[up[0] + 1]
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        st_m = helix_state(state0, charge, bz, mid)
        if np.hypot(st_m[0], st_m[1]) < radius:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _inward_crossing(state0, charge, bz, s_lo, s_hi, radius=SEED_RADIUS, ds=0.5):
    """First arc length in [s_lo, s_hi] where the helix crosses `radius` inward (None if none)."""
    s = np.arange(s_lo, s_hi + ds, ds)
    st = helix_state(state0, charge, bz, s)
    r = np.hypot(st[:, 0], st[:, 1])
    down = np.nonzero((r[:-1] >= radius) & (r[1:] < radius))[0]
    if down.size == 0:
        return None
    lo, hi = s[down[0]], s[down[0] + 1]
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        st_m = helix_state(state0, charge, bz, mid)
        if np.hypot(st_m[0], st_m[1]) >= radius:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def helix_hits(state0, charge: float, bz: float, s_len: float, ds: float = 0.5):
    """Truth hits of one helix segment: (wire_id, dca, s_pca, z_pca) arrays.

    A wire gets a hit when the helix passes within DRIFT_MAX of its line with the
    point of closest approach inside the chamber (|z| <= 750 mm); one hit per wire
    per segment (the closest pass).
    """
    wires = _wires()
    s = np.arange(0.0, s_len + ds, ds)
    st = helix_state(state0, charge, bz, s)
    pos = st[:, :3]
    r = np.hypot(pos[:, 0], pos[:, 1])
    cand_w, cand_s = [], []
    for layer in range(N_LAYERS):
        rl = float(layer_radius(layer))
        sel = np.nonzero(np.abs(r - rl) < 20.0)[0]
        if sel.size == 0:
            continue
        # only wires whose azimuth at the samples' heights lies near the samples
        a_st = STEREO if layer % 2 == 0 else -STEREO
        shift = np.tan(a_st) * pos[sel, 2] / rl
        cell = 2.0 * np.pi / WIRES_PER_LAYER
        centre = (np.arctan2(pos[sel, 1], pos[sel, 0]) - shift) / cell - 0.5 * (layer % 2)
        near = (np.round(centre)[:, None].astype(np.int64) + np.arange(-4, 5)[None]) % WIRES_PER_LAYER
        w_local = np.unique(near)
        w_ids = layer * WIRES_PER_LAYER + w_local
        a = wires[w_ids, :3]
        u = wires[w_ids, 3:] - a
        u = u / np.linalg.norm(u, axis=1, keepdims=True)
        dist = _line_distance(pos[sel][:, None, :], a[None], u[None])  # [n_sel, n_near]
        # local minima along contiguous runs of selected samples
        n = sel.size
        contig_prev = np.zeros(n, dtype=bool)
        contig_prev[1:] = sel[1:] == sel[:-1] + 1
        contig_next = np.zeros(n, dtype=bool)
        contig_next[:-1] = sel[1:] == sel[:-1] + 1
        lm = np.ones_like(dist, dtype=bool)
        lm[1:] &= ~contig_prev[1:, None] | (dist[1:] <= dist[:-1])
        lm[:-1] &= ~contig_next[:-1, None] | (dist[:-1] < dist[1:])
        lm &= dist < DRIFT_MAX + ds
        ii, ww = np.nonzero(lm)
        cand_w.append(w_ids[ww])
        cand_s.append(s[sel[ii]])
    if not cand_w:
        e = np.zeros(0)
        return e.astype(np.int32), e, e, e
    cw = np.concatenate(cand_w)
    cs = np.concatenate(cand_s)
    if cw.size == 0:
        e = np.zeros(0)
        return e.astype(np.int32), e, e, e
    a = wires[cw, :3]
    u = wires[cw, 3:] - a
    u = u / np.linalg.norm(u, axis=1, keepdims=True)

    def f(sv):
        return _line_distance(helix_state(state0, charge, bz, sv)[:, :3], a, u)

    lo = np.maximum(cs - ds, 0.0)
    hi = np.minimum(cs + ds, s_len)
    g = (np.sqrt(5.0) - 1.0) / 2.0
    c = hi - g * (hi - lo)
    d = lo + g * (hi - lo)
    fc, fd = f(c), f(d)
    for _ in range(48):
        left = fc < fd
        hi = np.where(left, d, hi)
        lo = np.where(left, lo, c)
        c_new = hi - g * (hi - lo)
        d_new = lo + g * (hi - lo)
        c, d = c_new, d_new
        fc, fd = f(c), f(d)
    s_pca = 0.5 * (lo + hi)
    dca = f(s_pca)
    z_pca = helix_state(state0, charge, bz, s_pca)[:, 2]
    ok = (dca <= DRIFT_MAX) & (np.abs(z_pca) <= HALF_LENGTH)
    cw, dca, s_pca, z_pca = cw[ok], dca[ok], s_pca[ok], z_pca[ok]
    # one hit per wire: the closest pass
    order = np.lexsort((dca, cw))
    cw, dca, s_pca, z_pca = cw[order], dca[order], s_pca[order], z_pca[order]
    first = np.ones(cw.size, dtype=bool)
    first[1:] = cw[1:] != cw[:-1]
    return cw[first].astype(np.int32), dca[first], s_pca[first], z_pca[first]


# ---------------------------------------------------------------- events
@dataclass
class Event:
    """One event in the CSR layout the seed scan consumes.

    wire_ids [n_w] (sorted), wire_ends [n_w, 6], wire_offsets [n_w + 1] (every wire
    holds at least one hit), drift [n_h]; truth: hit_turn [n_h] (-1 = noise),
    true_dca [n_h] (nan for noise); ref_states [n_turns, 6] = the true state at each
    turn's first outward crossing of r = 500 mm (the seed-grid centre); exit_states
    [n_turns, 6] = the true state where that turn crosses r = 500 mm inward again (NaN
    if it does not within the turn).
    """
    wire_ids: np.ndarray
    wire_ends: np.ndarray
    wire_offsets: np.ndarray
    drift: np.ndarray
    hit_turn: np.ndarray
    true_dca: np.ndarray
    ref_states: np.ndarray
    charge: float = -1.0
    bz: float = 1.0
    meta: dict = field(default_factory=dict)
    exit_states: np.ndarray = None

    @property
    def n_wires(self) -> int:
        return int(self.wire_ids.size)

    @property
    def n_hits(self) -> int:
        return int(self.drift.size)

    @property
    def n_turns(self) -> int:
        return int(self.ref_states.shape[0])


def _kink(state, rng, sigma_ms: float, eloss: float):
    """Small random deflection and momentum loss (stand-in for the target disks)."""
    px, py, pz = state[3], state[4], state[5]
    p = np.sqrt(px * px + py * py + pz * pz)
    th = np.arccos(pz / p) + rng.normal(0.0, sigma_ms)
    ph = np.arctan2(py, px) + rng.normal(0.0, sigma_ms)
    pn = p - eloss
    out = np.array(state, dtype=np.float64)
    out[3:] = pn * np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    return out


def make_event(state0, n_turns: int, rng: np.random.Generator, *, charge: float = -1.0,
               bz: float = 1.0, sigma: float = 0.2, noise: int = 0, noise_per_signal: float = 0.0,
               sigma_ms: float = 0.003, eloss: float = 0.2) -> Event:
    """Draw one event from a helix that starts at `state0` and makes `n_turns` revolutions.

    Between revolutions (where the track returns to its smallest radius) the momentum
    gets a kink of `sigma_ms` rad per angle and loses `eloss` MeV/c. Drift distance =
    clip(true DCA + N(0, sigma), 0, 8). Noise hits (`noise` of them, plus
    round(noise_per_signal * n_signal)) sit on uniformly random wires with drift ~ U[0, 8].
    """
    wires = _wires()
    st = np.array(state0, dtype=np.float64)
    hit_w, hit_d, hit_t = [], [], []
    refs, exits = [], []
    for t in range(n_turns):
        L = turn_length(st, charge, bz)
        w, dca, _, _ = helix_hits(st, charge, bz, L)
        s_ref = _outward_crossing(st, charge, bz, L)
        if s_ref is None:
            raise ValueError("turn %d never crosses r = %.0f mm outward" % (t, SEED_RADIUS))
        refs.append(helix_state(st, charge, bz, s_ref))
        s_exit = _inward_crossing(st, charge, bz, s_ref, L)
        exits.append(np.full(6, np.nan) if s_exit is None else helix_state(st, charge, bz, s_exit))
        hit_w.append(w)
        hit_d.append(dca)
        hit_t.append(np.full(w.size, t, dtype=np.int32))
        st = _kink(helix_state(st, charge, bz, L), rng, sigma_ms, eloss)
    w = np.concatenate(hit_w) if hit_w else np.zeros(0, np.int32)
    true = np.concatenate(hit_d) if hit_d else np.zeros(0)
    turn = np.concatenate(hit_t) if hit_t else np.zeros(0, np.int32)
    if sigma > 0.0:
        drift = np.clip(true + rng.normal(0.0, sigma, size=true.size), 0.0, DRIFT_MAX)
    else:
        drift = np.clip(true, 0.0, DRIFT_MAX)
    noise = int(noise) + int(round(noise_per_signal * true.size))
    if noise > 0:
        nw = rng.integers(0, N_WIRES, size=noise).astype(np.int32)
        nd = rng.uniform(0.0, DRIFT_MAX, size=noise)
        w = np.concatenate([w, nw])
        drift = np.concatenate([drift, nd])
        true = np.concatenate([true, np.full(noise, np.nan)])
        turn = np.concatenate([turn, np.full(noise, -1, dtype=np.int32)])
    order = np.argsort(w, kind="stable")
    w, drift, true, turn = w[order], drift[order], true[order], turn[order]
    uniq, counts = np.unique(w, return_counts=True)
    offsets = np.zeros(uniq.size + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(counts)
    return Event(wire_ids=uniq.astype(np.int32), wire_ends=np.ascontiguousarray(wires[uniq]),
                 wire_offsets=offsets, drift=np.ascontiguousarray(drift, dtype=np.float64),
                 hit_turn=turn.astype(np.int32), true_dca=true,
                 ref_states=np.ascontiguousarray(np.stack(refs)), charge=charge, bz=bz,
                 meta={"n_signal": int(np.sum(turn >= 0)), "n_noise": int(noise)},
                 exit_states=np.ascontiguousarray(np.stack(exits)))


def vertex_state(p: float, polar: float, azimuth: float, vertex=(0.0, 0.0, 0.0)) -> np.ndarray:
    return np.array([vertex[0], vertex[1], vertex[2],
                     p * np.sin(polar) * np.cos(azimuth), p * np.sin(polar) * np.sin(azimuth),
                     p * np.cos(polar)], dtype=np.float64)


# ---------------------------------------------------------------- scan settings
@dataclass
class ScanConfig:
    """Seed-grid and stepping settings of one workload."""
    name: str
    n: tuple            # points per axis (arc offset, |p|, d theta, d phi)
    half: tuple         # half-spans (mm, MeV/c, rad, rad)
    n_steps: int
    step_mm: float
    lambda_mm: float
    n_refine: int = 2

    @property
    def n_seeds(self) -> int:
        return int(np.prod(self.n))


def grid_descriptor(ref_state, cfg: ScanConfig) -> np.ndarray:
    """[14] = reference state (6), axis centres (4), axis half-spans (4).

    Centres: zero offsets and the reference |p|, i.e. the grid is centred on the
    truth state at the seed radius (the Hough / hodoscope seeding is not modelled).
    """
    ref = np.asarray(ref_state, dtype=np.float64)
    p = float(np.sqrt(ref[3] ** 2 + ref[4] ** 2 + ref[5] ** 2))
    return np.concatenate([ref, [0.0, p, 0.0, 0.0], np.asarray(cfg.half, dtype=np.float64)])


# Plain method, one event, one turn (1 T; p = 100 MeV/c at 60 deg polar from the
# origin; 8^4 grid over +-5 mm, +-5 MeV/c, +-50 mrad, +-50 mrad; 1000 x 2 mm; lambda 1 mm).
C0 = ScanConfig("plain-1turn", (8, 8, 8, 8), (5.0, 5.0, 0.05, 0.05), 1000, 2.0, 1.0)
# Plain method, one signal-like event: 104 MeV/c, three turns, 10 % noise, 16^4 grid
# with twice the spans, 1500 x 2 mm, lambda 0.8 mm.
C1 = ScanConfig("signal-3turn", (16, 16, 16, 16), (10.0, 10.0, 0.10, 0.10), 1500, 2.0, 0.8)


def event_plain(seed: int = 0, sigma: float = 0.2) -> Event:
    """One electron, p = 100 MeV/c, polar 60 deg from +z, from the origin; one turn, no noise."""
    rng = np.random.default_rng(seed)
    az = rng.uniform(0.0, 2.0 * np.pi)
    st = vertex_state(100.0, np.deg2rad(60.0), az)
    return make_event(st, 1, rng, sigma=sigma, noise=0)


def event_signal(seed: int = 0, sigma: float = 0.2) -> Event:
    """One signal-like electron: |p| = 104 MeV/c, three turns, 10 % noise hits.

    The polar angle is drawn in [77, 82] deg and the vertex sits at z = -650 mm so
    that three turns fit inside the 1500 mm chamber.
    """
    rng = np.random.default_rng(seed)
    polar = np.deg2rad(rng.uniform(77.0, 82.0))
    az = rng.uniform(0.0, 2.0 * np.pi)
    st = vertex_state(104.0, polar, az, vertex=(0.0, 0.0, -650.0))
    return make_event(st, 3, rng, sigma=sigma, noise_per_signal=0.10)


# ---------------------------------------------------------------- batched event mix
def entry_state(p: float, pz: float, r_max: float, psi: float, z0: float, charge: float = -1.0,
                bz: float = 1.0) -> np.ndarray:
    """Start state on the innermost point of a transverse circle.

    The circle has radius R = p_T / (KAPPA |q| B) and its centre sits at distance
    r_max - R from the axis in direction psi, so the track's largest radius is r_max.
    The start point is the circle's point closest to the axis, with the momentum
    tangent to the circle in the sense the field turns it.
    """
    pt = np.sqrt(p * p - pz * pz)
    R = pt / (KAPPA * abs(charge) * bz)
    d = r_max - R
    u = np.array([np.cos(psi), np.sin(psi)])
    pos = (d - R) * u
    # counter-clockwise (seen from +z) for q B < 0, clockwise otherwise
    sense = 1.0 if charge * bz < 0 else -1.0
    tang = sense * np.array([u[1], -u[0]])
    return np.array([pos[0], pos[1], z0, pt * tang[0], pt * tang[1], pz])


def event_mix(seed: int, sigma: float = 0.2, noise_frac: float = 0.20, turns=(1, 5),
              hits=(40, 400), p_range=(60.0, 105.0), max_tries: int = 200) -> Event:
    """One event of the batched mix (falling momentum spectrum, 1-5 turns, 20 % noise).

    |p| follows (105 - p)^5 on [60, 105] MeV/c; P ~ U{turns}; p_z ~ U[0.3, 1] x 66.8 / P
    MeV/c so that P turns fit in the chamber; the largest track radius ~ U[560, 830] mm;
    the track starts at its innermost point at z = -700 mm (plus a small offset) and
    must cross r = 500 mm outward in every turn. Noise hits make up `noise_frac` of all
    hits. Drawn again until the hit count lies in `hits`.
    """
    rng = np.random.default_rng([seed, 7])
    lo, hi = p_range
    for _ in range(max_tries):
        p = hi - (hi - lo) * rng.uniform() ** (1.0 / 6.0)
        n_turns = int(rng.integers(turns[0], turns[1] + 1))
        pz = rng.uniform(0.3, 1.0) * 66.8 / n_turns
        if pz >= p:
            continue
        r_max = rng.uniform(560.0, 830.0)
        R = np.sqrt(p * p - pz * pz) / KAPPA
        if r_max - 2.0 * R > 480.0 or r_max - R < 0.0:
            continue  # never comes inside the seed radius
        st = entry_state(p, pz, r_max, rng.uniform(0.0, 2.0 * np.pi), -700.0 + rng.uniform(0, 40))
        try:
            ev = make_event(st, n_turns, rng, sigma=sigma,
                            noise_per_signal=noise_frac / (1.0 - noise_frac))
        except ValueError:
            continue
        if hits[0] <= ev.n_hits <= hits[1] and ev.meta["n_signal"] > 0:
            ev.meta.update(p=float(p), n_turns=n_turns, r_max=float(r_max), seed=seed)
            return ev
    raise RuntimeError("event_mix(%d): no event within %s hits" % (seed, hits))


# Batched mix: 32768 seeds per partition (8 x 16 x 16 x 16), 1000 x 2 mm, lambda 0.8 mm.
C2 = ScanConfig("mix-batched", (8, 16, 16, 16), (5.0, 5.0, 0.05, 0.05), 1000, 2.0, 0.8)
# Differentiation workload: coarse 8^4 grid (then Gauss-Newton) vs fine 32^4 grid.
C3_COARSE = ScanConfig("mix-coarse", (8, 8, 8, 8), (5.0, 5.0, 0.05, 0.05), 1000, 2.0, 0.8, 0)
C3_FINE = ScanConfig("mix-fine", (32, 32, 32, 32), (5.0, 5.0, 0.05, 0.05), 1000, 2.0, 0.8, 0)


# Stress workload: up to 6 turns, 200-1200 hits with 30 % noise, 131072 seeds per
# partition (8 x 16 x 32 x 32), RK4 2000 x 1.5 mm; refinement by Levenberg-Marquardt
# from the 64 lowest-RSS seeds of each partition instead of finer grids.
C4 = ScanConfig("stress", (8, 16, 32, 32), (5.0, 5.0, 0.05, 0.05), 2000, 1.5, 0.8, 0)


def event_stress(seed: int) -> Event:
    """One event of the stress mix (event_mix with 1-6 turns, 200-1200 hits, 30 % noise)."""
    return event_mix(seed, noise_frac=0.30, turns=(1, 6), hits=(200, 1200))


def event_mix_batch(seeds, workers: int = 0, kind: str = "mix"):
    """event_mix for many seeds, in worker processes when workers > 1 (numpy only)."""
    seeds = list(seeds)
    fn = {"mix": event_mix, "stress": event_stress}[kind]
    if workers <= 1 or len(seeds) < 8:
        return [fn(s) for s in seeds]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        return pool.map(fn, seeds, chunksize=max(1, len(seeds) // (4 * workers)))


# ---------------------------------------------------------------- half tracks
def circle_centre(state, charge: float, bz: float) -> np.ndarray:
    """Transverse centre of the helix through `state` (x, y)."""
    xt = complex(state[0], state[1])
    pt = complex(state[3], state[4])
    c = xt - 1j * pt / (KAPPA * charge * bz)
    return np.array([c.real, c.imag])


def wire_layers(wire_ids) -> np.ndarray:
    return (np.asarray(wire_ids, dtype=np.int32) // WIRES_PER_LAYER).astype(np.int32)


def _sub_event(ev: Event, wire_sel: np.ndarray, state, charge: float, meta: dict) -> Event:
    wsel = np.nonzero(wire_sel)[0]
    counts = np.diff(ev.wire_offsets)[wsel]
    offsets = np.zeros(wsel.size + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(counts)
    hits = (np.concatenate([np.arange(ev.wire_offsets[i], ev.wire_offsets[i + 1])
                            for i in wsel]) if wsel.size else np.zeros(0, np.int64))
    hits = hits.astype(np.int64)
    return Event(wire_ids=ev.wire_ids[wsel].copy(),
                 wire_ends=np.ascontiguousarray(ev.wire_ends[wsel]).reshape(-1, 6),
                 wire_offsets=offsets, drift=np.ascontiguousarray(ev.drift[hits]),
                 hit_turn=ev.hit_turn[hits].copy(), true_dca=ev.true_dca[hits].copy(),
                 ref_states=np.ascontiguousarray(np.asarray(state, np.float64)[None, :]),
                 charge=charge, bz=ev.bz, meta=dict(meta, hits=hits))


def entrance_sides(ev: Event, turn: int) -> np.ndarray:
    """bool [n_wires]: the wires on the entrance side of the turn (Sec. 3.1's half
    tracks): the side, of the line through the chamber axis and the turn's true circle
    centre, that holds the turn's outward crossing of r = 500 mm; each wire taken at its
    midpoint (z = 0), a wire exactly on the line on the entrance side. The true circle
    stands in for the paper's Hough-transform circle."""
    ref = ev.ref_states[turn]
    c = circle_centre(ref, ev.charge, ev.bz)
    mid = 0.5 * (ev.wire_ends[:, :2] + ev.wire_ends[:, 3:5])
    side = c[0] * mid[:, 1] - c[1] * mid[:, 0]
    s_in = c[0] * ref[1] - c[1] * ref[0]
    return (side == 0.0) | (np.sign(side) == np.sign(s_in))


def half_events(ev: Event, turn: int):
    """The two half tracks of one turn partition (Sec. 3.1) as one-turn pseudo-events.

    Entrance half: the event's wires on the entrance side, seeded at the turn's outward
    crossing of r = 500 mm. Exit half: the wires on the other side, seeded at the
    inward crossing with momentum and charge flipped, so that its tracks run backwards
    from the exit. The two sides are split by the line through the chamber axis and the
    turn's true circle centre (the entrance and exit points are mirror images across
    it), taking each wire at its midpoint (z = 0); a wire exactly on the line goes to the
    entrance side. The true circle stands in for the paper's Hough-transform circle.
    meta["hits"] maps each half's hits to the event's hit indices.
    """
    ref = ev.ref_states[turn]
    ext = ev.exit_states[turn]
    entrance = entrance_sides(ev, turn)
    flipped = np.concatenate([ext[:3], -ext[3:]])
    a = _sub_event(ev, entrance, ref, ev.charge, {"turn": turn, "side": "entrance"})
    b = _sub_event(ev, ~entrance, flipped, -ev.charge, {"turn": turn, "side": "exit"})
    return a, b


# ---------------------------------------------------------------- field map
def solenoid_map(b0: float = 1.0, g: float = 0.1, z_scale: float = 1500.0,
                 half_xy: float = 1000.0, half_z: float = 1500.0, step: float = 25.0):
    """A synthetic solenoid field map (the COMET map is not available): on a regular grid,
    B_z = b0 (1 + g (z / Z)^2), B_x = -b0 g z x / Z^2, B_y = -b0 g z y / Z^2 (tesla),
    which has zero divergence. Returns (b [nz, ny, nx, 3], origin [3], step [3])."""
    xs = np.arange(-half_xy, half_xy + 0.5 * step, step)
    zs = np.arange(-half_z, half_z + 0.5 * step, step)
    Z, Y, X = np.meshgrid(zs, xs, xs, indexing="ij")
    b = np.empty(Z.shape + (3,))
    b[..., 0] = -b0 * g * Z * X / z_scale ** 2
    b[..., 1] = -b0 * g * Z * Y / z_scale ** 2
    b[..., 2] = b0 * (1.0 + g * (Z / z_scale) ** 2)
    return (np.ascontiguousarray(b), np.array([xs[0], xs[0], zs[0]]),
            np.array([step, step, step]))
