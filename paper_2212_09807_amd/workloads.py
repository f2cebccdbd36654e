"""Seeded synthetic inputs shaped like the paper's workloads, and the analytic field-response table.

This module only *prepares inputs*: energy-deposit segment tables (the (r_s, r_e, E) rows of Sec. 2),
detector/response parameters (Sec. 3.1-3.4 constants) and a pixel field-response look-up table.  It holds
none of the simulation's own arithmetic (no recombination, drift, diffusion, induction or electronics);
both the FP64 oracle and the HIP path consume what it returns.  It imports nothing else from this
package and nothing from the oracle.

Workloads (the paper's own inputs are edep-sim/Geant4 segments of cosmic rays and neutrino spills, which
are not available; these generators stand in for them with the same shapes, Sec. 2 and Sec. 6):

* ``cfg1``  one straight muon-like track, 200 segments, one 70x70-pixel Module-0 tile (Sec. 6 geometry).
* ``cfg2``  a module-scale event: 40 tracks (30 muon-like, 10 proton-like), 20,000 segments, 140x140 pixels.
* ``cfg3``  a spill of 64 such events with log-normal segment counts (batched path).
* ``cfg4``  the cfg3 event mix with Poisson arrival times (served path).
* ``cfg5``  a large spill: 30 neutrino-like vertices + 200 cosmic muons over 7x5 tiles, 2,000,000 segments.

Units everywhere: cm, microseconds, MeV, electrons, kV/cm.  The anode plane is z = 0, charge sits at z > 0.

Response table (stand-in for the FEM-derived table of Sec. 3.3.1): the weighting potential of a square pad
of side ``a`` in a grounded plane is the solid angle the pad subtends, divided by 2*pi.  For an electron
drifting straight down the z axis at constant v_d, the charge induced on the pad during tick k is the
change of that potential.  The table is arrival-aligned: entry ``T_R - 1`` is the tick in which the
electron reaches the anode, and entry 0 lumps all induction from beyond the table's reach, so every column
integrates to exactly one electron (bins over the pad) or zero (bins off the pad), which is the
normalisation rule of Sec. 3.3.1.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# --------------------------------------------------------------------------------------------
# Parameter sets (host-side descriptions; mirrored field-for-field by the C structs in ltsim.h)
# --------------------------------------------------------------------------------------------

PITCH_CM = 0.4434          # Module-0 pixel pad pitch (Sec. 6)
TILE_PIXELS_MODULE0 = 70   # 70x70 = 4900 pads per tile (Sec. 6)


@dataclass
class Physics:
    """Charge-transport constants.  Defaults are the paper's values (Sec. 3.1, 3.2)."""
    recomb_model: int = 0           # 0 = Birks (paper default), 1 = modified Box
    e_field: float = 0.5            # kV/cm (Sec. 6 operating field)
    lar_density: float = 1.38       # g/cm^3 (not printed in the paper; standard LAr value)
    w_ion: float = 23.6e-6          # MeV per ionisation electron (not printed; standard LAr value)
    birks_ab: float = 0.800         # ICARUS Birks A_b (Sec. 3.1)
    birks_kb: float = 0.0486        # ICARUS Birks k_b (Sec. 3.1)
    box_alpha: float = 0.93         # ArgoNeuT Box alpha (Sec. 3.1)
    box_beta: float = 0.207         # ArgoNeuT Box beta (Sec. 3.1)
    v_drift: float = 0.1648         # cm/us
    lifetime: float = 2200.0        # us (2.2 ms)
    d_long: float = 4.0e-6          # cm^2/us  (4 cm^2/s, Sec. 3.2)
    d_tran: float = 8.8e-6          # cm^2/us  (8.8 cm^2/s, Sec. 3.2)
    z_anode: float = 0.0            # cm
    sample_step: float = 0.001      # cm: 10 um sampling interval along the segment (Sec. 3.3.2)
    n_sigma: float = 5.0            # diffusion truncation, in sigmas (not printed; shared reading)
    mc_draws: int = 0               # 0: expectation over the diffusion draws; M > 0: M random draws per point
    per_point: int = 0              # 0: lifetime and diffusion at the segment midpoint; 1: at every sample point


@dataclass
class Readout:
    """Pixel plane and time sampling."""
    pitch: float = PITCH_CM         # cm
    n_x: int = TILE_PIXELS_MODULE0
    n_y: int = TILE_PIXELS_MODULE0
    x0: float = 0.0                 # cm, tile origin (lower pixel edge)
    y0: float = 0.0
    n_sub: int = 10                 # sub-pixel bins per pitch (table granularity)
    tick: float = 0.1               # us
    n_ticks: int = 2000
    t_begin: float = 0.0            # us, time of the lower edge of tick 0


@dataclass
class Electronics:
    """LArPix-like front end (Sec. 3.4)."""
    threshold: float = 5000.0       # electrons (paper preset: 7000)
    hold_ticks: int = 16            # 1.6 us between threshold crossing and digitisation
    min_spacing: int = 11           # >= 11 clock cycles (10 MHz) between consecutive samples
    q_lsb: float = 1000.0           # electrons per ADC count
    pedestal: int = 0
    adc_bits: int = 8
    sigma_reset: float = 0.0        # electrons (paper: 900)
    sigma_disc: float = 0.0         # electrons (paper: 650)
    sigma_unc: float = 500.0        # electrons (paper: 500)
    max_packets: int = 128          # per pixel
    seed: int = 0x2212098070000001
    reset_period: int = 0           # periodic reset every N ticks (0 = off)


@dataclass
class TableShape:
    t_r: int = 200                  # ticks in the response table
    b_x: int = 10                   # sub-pixel bins from the pixel centre (reach = b_x * pitch / n_sub)
    b_y: int = 10


@dataclass
class Segments:
    """Structure-of-arrays segment table; coordinates are tile-local."""
    x0: np.ndarray
    y0: np.ndarray
    z0: np.ndarray
    t0: np.ndarray
    x1: np.ndarray
    y1: np.ndarray
    z1: np.ndarray
    t1: np.ndarray
    energy: np.ndarray
    dedx: Optional[np.ndarray] = None   # only needed for zero-length deposits

    FIELDS = ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1", "energy")

    @property
    def n(self) -> int:
        return int(self.x0.shape[0])

    def columns(self):
        return [getattr(self, f) for f in self.FIELDS]

    def subset(self, idx) -> "Segments":
        kw = {f: np.ascontiguousarray(getattr(self, f)[idx]) for f in self.FIELDS}
        kw["dedx"] = None if self.dedx is None else np.ascontiguousarray(self.dedx[idx])
        return Segments(**kw)

    def shifted(self, dx=0.0, dy=0.0, dt=0.0) -> "Segments":
        s = dataclasses.replace(self)
        s.x0 = (self.x0 + np.float32(dx)).astype(np.float32)
        s.x1 = (self.x1 + np.float32(dx)).astype(np.float32)
        s.y0 = (self.y0 + np.float32(dy)).astype(np.float32)
        s.y1 = (self.y1 + np.float32(dy)).astype(np.float32)
        s.t0 = (self.t0 + np.float32(dt)).astype(np.float32)
        s.t1 = (self.t1 + np.float32(dt)).astype(np.float32)
        return s

    @staticmethod
    def concat(parts: List["Segments"]) -> "Segments":
        kw = {f: np.concatenate([getattr(p, f) for p in parts]).astype(np.float32) for f in Segments.FIELDS}
        if any(p.dedx is not None for p in parts):
            kw["dedx"] = np.concatenate([p.dedx if p.dedx is not None else np.full(p.n, np.nan, np.float32)
                                         for p in parts]).astype(np.float32)
        return Segments(**kw)


def make_segments(r0, r1, energy, t0=None, t1=None, dedx=None) -> Segments:
    r0 = np.asarray(r0, np.float64).reshape(-1, 3)
    r1 = np.asarray(r1, np.float64).reshape(-1, 3)
    n = r0.shape[0]
    t0 = np.zeros(n) if t0 is None else np.broadcast_to(np.asarray(t0, np.float64), (n,))
    t1 = np.zeros(n) if t1 is None else np.broadcast_to(np.asarray(t1, np.float64), (n,))
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64), dtype=np.float32)
    return Segments(f(r0[:, 0]), f(r0[:, 1]), f(r0[:, 2]), f(t0), f(r1[:, 0]), f(r1[:, 1]), f(r1[:, 2]), f(t1),
                    f(np.broadcast_to(np.asarray(energy, np.float64), (n,))),
                    None if dedx is None else f(np.broadcast_to(np.asarray(dedx, np.float64), (n,))))


@dataclass
class Workload:
    name: str
    physics: Physics
    readout: Readout
    electronics: Electronics
    table: TableShape
    events: List[Segments] = field(default_factory=list)
    event_ids: List[int] = field(default_factory=list)
    arrivals_s: Optional[np.ndarray] = None     # serving only: arrival times in seconds


# --------------------------------------------------------------------------------------------
# Analytic response table
# --------------------------------------------------------------------------------------------

def pad_weighting_potential(dx, dy, z, side):
    """Weighting potential of a square pad (side ``side``) centred at the origin of a grounded plane,
    at lateral offset (dx, dy) and height z > 0: the pad's solid angle / (2 pi).  z == 0 is the limit
    (1 over the pad, 0 elsewhere)."""
    dx, dy, z = np.broadcast_arrays(np.asarray(dx, np.float64), np.asarray(dy, np.float64),
                                    np.asarray(z, np.float64))
    h = 0.5 * side
    out = np.zeros(dx.shape)
    pos = z > 0
    zz = z[pos]
    acc = np.zeros(zz.shape)
    for sx, X in ((-1.0, -h - dx[pos]), (1.0, h - dx[pos])):
        for sy, Y in ((-1.0, -h - dy[pos]), (1.0, h - dy[pos])):
            acc += sx * sy * np.arctan(X * Y / (zz * np.sqrt(X * X + Y * Y + zz * zz)))
    out[pos] = acc / (2.0 * np.pi)
    inside = (np.abs(dx) < h) & (np.abs(dy) < h)
    out[~pos] = np.where(inside[~pos], 1.0, 0.0)
    return out


def response_table_f64(shape: TableShape, readout: Readout, v_drift: float) -> np.ndarray:
    """R[k, i, j] in FP64, k in [0, T_R): electrons induced during tick k on a pad by one electron whose
    lateral offset from the pad centre is the centre of sub-pixel bin (i, j), ((i+1/2) b, (j+1/2) b),
    b = pitch / n_sub.  Tick T_R-1 ends at arrival; the electron sits at z_k = (T_R - k) * tick * v_d at the
    start of tick k.  R[0] = W(z_1) (everything induced before the table starts), R[k] = W(z_{k+1}) - W(z_k)."""
    T, bx, by = shape.t_r, shape.b_x, shape.b_y
    b = readout.pitch / readout.n_sub
    cx = (np.arange(bx) + 0.5) * b
    cy = (np.arange(by) + 0.5) * b
    zk = (T - np.arange(1, T + 1)) * readout.tick * v_drift          # z_1 .. z_T  (z_T = 0)
    W = pad_weighting_potential(cx[None, :, None], cy[None, None, :], zk[:, None, None], readout.pitch)
    R = np.empty((T, bx, by))
    R[0] = W[0]
    R[1:] = W[1:] - W[:-1]
    return R


def response_table(shape: TableShape, readout: Readout, v_drift: float) -> np.ndarray:
    """The FP32 table that both the oracle and the device consume, layout [T_R][B_x][B_y] C-contiguous."""
    return np.ascontiguousarray(response_table_f64(shape, readout, v_drift), dtype=np.float32)


# --------------------------------------------------------------------------------------------
# Track helpers
# --------------------------------------------------------------------------------------------

def _rng(cfg: int, event: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([2212, 9807, cfg, event])))


_LANDAU_MODE = None


def _landau_mode() -> float:
    global _LANDAU_MODE
    if _LANDAU_MODE is None:
        from scipy.optimize import minimize_scalar
        from scipy.stats import landau
        _LANDAU_MODE = float(minimize_scalar(lambda x: -landau.pdf(x), bracket=(-1.0, 0.0, 1.0)).x)
    return _LANDAU_MODE


def mip_dedx(rng, n) -> np.ndarray:
    """dE/dx of a minimum-ionising particle: 2.1 MeV/cm + 0.2 * (Landau - mode), clipped to [1, 20]."""
    from scipy.stats import landau
    x = landau.rvs(size=n, random_state=rng)
    return np.clip(2.1 + 0.2 * (x - _landau_mode()), 1.0, 20.0)


def proton_dedx(residual_range_cm) -> np.ndarray:
    """Bragg-Kleeman-style stopping power rising toward the end of the range, capped at 40 MeV/cm."""
    r = np.maximum(np.asarray(residual_range_cm, np.float64), 1e-4)
    return np.minimum(13.4 * r ** -0.42, 40.0)


def isotropic(rng, n=None):
    v = rng.normal(size=(3,) if n is None else (n, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def clip_line(p, d, length, lo, hi):
    """Liang-Barsky: parameter range [s0, s1] of p + s*d, s in [0, length], inside the box [lo, hi]."""
    s0, s1 = 0.0, float(length)
    for ax in range(3):
        if abs(d[ax]) < 1e-15:
            if p[ax] < lo[ax] or p[ax] > hi[ax]:
                return None
            continue
        a = (lo[ax] - p[ax]) / d[ax]
        b = (hi[ax] - p[ax]) / d[ax]
        if a > b:
            a, b = b, a
        s0, s1 = max(s0, a), min(s1, b)
        if s0 >= s1:
            return None
    return s0, s1


@dataclass
class Track:
    p: np.ndarray          # start point (unclipped)
    d: np.ndarray          # unit direction
    length: float          # unclipped length
    kind: str              # "mip" or "proton"
    s0: float = 0.0        # clipped parameter range
    s1: float = 0.0
    t0: float = 0.0        # us

    @property
    def clipped_length(self):
        return self.s1 - self.s0


C_CM_PER_US = 2.99792458e4


def segment_tracks(rng, tracks: List[Track], n_total: int) -> Segments:
    """Split the clipped tracks into n_total equal-length-per-track segments, allotted in proportion to
    clipped length (at least one per track)."""
    L = np.array([t.clipped_length for t in tracks])
    raw = n_total * L / L.sum()
    n = np.maximum(1, np.floor(raw).astype(np.int64))
    while n.sum() < n_total:                  # largest remainders first
        n[np.argmax(raw - n)] += 1
    while n.sum() > n_total:
        n[np.argmax(n)] -= 1
    parts = []
    for t, k in zip(tracks, n):
        edges = t.s0 + (t.s1 - t.s0) * np.arange(k + 1) / k
        sa, sb = edges[:-1], edges[1:]
        r0 = t.p[None, :] + sa[:, None] * t.d[None, :]
        r1 = t.p[None, :] + sb[:, None] * t.d[None, :]
        seglen = sb - sa
        if t.kind == "mip":
            dedx = mip_dedx(rng, k)
        else:
            mid = 0.5 * (sa + sb)
            dedx = proton_dedx(t.length - mid)
        parts.append(make_segments(r0, r1, dedx * seglen, t0=t.t0 + sa / C_CM_PER_US,
                                   t1=t.t0 + sb / C_CM_PER_US))
    return Segments.concat(parts)


# --------------------------------------------------------------------------------------------
# Configurations
# --------------------------------------------------------------------------------------------

def _cfg1_event(rng) -> Segments:
    lo = np.zeros(3)
    hi = np.array([TILE_PIXELS_MODULE0 * PITCH_CM, TILE_PIXELS_MODULE0 * PITCH_CM, 30.0])
    ext = hi - lo
    areas = np.array([ext[1] * ext[2], ext[0] * ext[2], ext[0] * ext[1]])

    def surface_point():
        ax = rng.choice(3, p=areas / areas.sum())
        side = rng.integers(2)
        p = lo + rng.random(3) * ext
        p[ax] = hi[ax] if side else lo[ax]
        return p, 2 * ax + side

    while True:
        a, fa = surface_point()
        b, fb = surface_point()
        if fa != fb and np.linalg.norm(b - a) >= 30.0:
            break
    k = 200
    s = np.arange(k + 1) / k
    pts = a[None, :] + s[:, None] * (b - a)[None, :]
    seglen = np.linalg.norm(b - a) / k
    dedx = mip_dedx(rng, k)
    return make_segments(pts[:-1], pts[1:], dedx * seglen)


def _module_tracks(rng, n_mu, n_p, hi) -> List[Track]:
    tracks = []
    for kind, count in (("mip", n_mu), ("proton", n_p)):
        for _ in range(count):
            while True:
                p = rng.random(3) * hi
                d = isotropic(rng)
                length = rng.uniform(50.0, 150.0) if kind == "mip" else rng.uniform(2.0, 20.0)
                c = clip_line(p, d, length, np.zeros(3), hi)
                if c is not None and c[1] - c[0] > 1e-3:
                    break
            tracks.append(Track(p, d, length, kind, c[0], c[1]))
    return tracks


MODULE_W = 140 * PITCH_CM
MODULE_HI = np.array([MODULE_W, MODULE_W, 50.0])


def _cfg2_event(rng, n_segments=20000) -> Segments:
    n_tracks = max(2, int(round(40 * n_segments / 20000)))
    n_p = max(1, n_tracks // 4)
    tracks = _module_tracks(rng, n_tracks - n_p, n_p, MODULE_HI)
    return segment_tracks(rng, tracks, n_segments)


def config(k: int) -> Workload:
    """Parameters of configuration k (1..5) without events."""
    ph = Physics()
    if k == 1:
        ro = Readout(n_x=70, n_y=70, n_ticks=2000)
        el = Electronics(seed=0x2212098070000000 + 1)
        tb = TableShape(200, 10, 10)
    elif k in (2, 3, 4):
        ro = Readout(n_x=140, n_y=140, n_ticks=3000)
        el = Electronics(seed=0x2212098070000000 + k)
        tb = TableShape(1950, 45, 45)
    elif k == 5:
        ro = Readout(n_x=140, n_y=140, n_ticks=5000)
        el = Electronics(sigma_reset=900.0, sigma_disc=650.0, sigma_unc=500.0, seed=0x2212098070000000 + 5)
        tb = TableShape(1950, 45, 45)
    else:
        raise ValueError(f"no configuration {k}")
    return Workload(f"cfg{k}", ph, ro, el, tb)


def spill_sizes(rng, n_events=64) -> np.ndarray:
    return np.clip(np.round(rng.lognormal(np.log(8000.0), 1.2, size=n_events)), 500, 200000).astype(np.int64)


def make_workload(k: int, n_events: Optional[int] = None, event0: int = 0) -> Workload:
    """Configuration k with its seeded events (event ids event0, event0+1, ...)."""
    w = config(k)
    if k == 1:
        ids = list(range(event0, event0 + (n_events or 1)))
        w.events = [_cfg1_event(_rng(1, e)) for e in ids]
    elif k == 2:
        ids = list(range(event0, event0 + (n_events or 1)))
        w.events = [_cfg2_event(_rng(2, e)) for e in ids]
    elif k in (3, 4):
        n = n_events or 64
        sizes = spill_sizes(_rng(k, 1_000_000), max(n, 64))[:n] if n <= 64 else spill_sizes(_rng(k, 1_000_000), n)
        ids = list(range(event0, event0 + n))
        w.events = [_cfg2_event(_rng(k, e), int(s)) for e, s in zip(ids, sizes)]
        if k == 4:
            w.arrivals_s = None    # set by poisson_arrivals() for a chosen rate
    elif k == 5:
        tiles, ids = large_spill(_rng(5, event0))
        w.events = tiles[: n_events] if n_events else tiles
        ids = ids[: len(w.events)]
    w.event_ids = ids
    return w


def poisson_arrivals(rate_hz: float, n: int, seed: int = 0) -> np.ndarray:
    rng = _rng(4, 2_000_000 + seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


# --------------------------------------------------------------------------------------------
# Large spill (cfg5): 7x5 tiles, neutrino-like vertices + cosmic muons, halo replication
# --------------------------------------------------------------------------------------------

TILES_X, TILES_Y = 7, 5


def large_spill(rng, n_segments=2_000_000, halo_cm=2.4):
    hi = np.array([TILES_X * MODULE_W, TILES_Y * MODULE_W, 50.0])
    tracks: List[Track] = []
    for _ in range(30):                                   # neutrino-like vertices
        v = rng.random(3) * hi
        t0 = rng.uniform(0.0, 10.0)
        d_mu = np.array([1.0, 0.0, 0.0]) + 0.5 * isotropic(rng)
        d_mu /= np.linalg.norm(d_mu)
        for kind, d, length in [("mip", d_mu, rng.uniform(50.0, 300.0))] + [
                (("proton", isotropic(rng), rng.uniform(2.0, 20.0)) if rng.random() < 0.5 else
                 ("mip", isotropic(rng), rng.uniform(5.0, 50.0))) for _ in range(int(rng.integers(2, 9)))]:
            c = clip_line(v, d, length, np.zeros(3), hi)
            if c is not None and c[1] - c[0] > 1e-3:
                tracks.append(Track(v, d, length, kind, c[0], c[1], t0))
    for _ in range(200):                                  # cosmic muons entering through the top (y = max)
        while True:
            cos_t = rng.random() ** (1.0 / 3.0)             # pdf ~ cos^2(theta) per solid angle
            sin_t = np.sqrt(1.0 - cos_t * cos_t)
            phi = rng.uniform(0, 2 * np.pi)
            d = np.array([sin_t * np.cos(phi), -cos_t, sin_t * np.sin(phi)])
            p = np.array([rng.uniform(0, hi[0]), hi[1], rng.uniform(0, hi[2])])
            c = clip_line(p, d, 1e4, np.zeros(3), hi)
            if c is not None and c[1] - c[0] > 1.0:
                break
        tracks.append(Track(p, d, c[1], "mip", c[0], c[1], rng.uniform(-300.0, 500.0)))
    segs = segment_tracks(rng, tracks, n_segments)
    mx = 0.5 * (segs.x0.astype(np.float64) + segs.x1)
    my = 0.5 * (segs.y0.astype(np.float64) + segs.y1)
    tiles, ids = [], []
    for ty in range(TILES_Y):
        for tx in range(TILES_X):
            xl, yl = tx * MODULE_W, ty * MODULE_W
            sel = ((mx >= xl - halo_cm) & (mx < xl + MODULE_W + halo_cm) &
                   (my >= yl - halo_cm) & (my < yl + MODULE_W + halo_cm))
            idx = np.nonzero(sel)[0]
            tiles.append(segs.subset(idx).shifted(dx=-xl, dy=-yl))
            ids.append(ty * TILES_X + tx)
    return tiles, ids


# ------------------------------------------------------------------------------------------------ light (Sec. 4)

W_PH_MEV = 19.5e-6                  # MeV per scintillation photon at zero field (not printed; standard LAr value)


@dataclass
class Light:
    """Light readout and scintillation (Sec. 4).  Field order is the C layout of the library's light parameters."""
    tick: float = 1.0               # ns per light tick
    tau_p: float = 7.0              # ns, prompt scintillation decay time (Sec. 4.2: ~7 ns)
    tau_s: float = 1600.0           # ns, slow decay time (Sec. 4.2: ~1600 ns)
    f_prompt: float = 0.3           # prompt light fraction (Sec. 4.2: ~0.3)
    trunc: float = 5.0              # the scintillation kernel is truncated after 5 tau_s (Sec. 4.2)
    gain: float = 8.0               # ADC counts per p.e. (synthetic detector)
    normal_above: float = 30.0      # p.e.: normal approximation above this mean (Sec. 4.2)
    n_det: int = 64                 # light detectors
    n_ticks: int = 16384            # 16.4 us window
    group: int = 8                  # detectors summed for triggering (Sec. 4.3)
    trig_threshold: float = 150.0   # ADC counts on the group sum
    trig_deadtime: int = 2048       # ticks between triggers of a group
    max_trig: int = 16              # triggers kept per group
    seed: int = 0x2212098070000000 + 6


def light_response(n_resp: int = 512, tau_r: float = 20.0, tick: float = 1.0) -> np.ndarray:
    """Unit-normalised impulse response of a synthetic light readout (a CR-RC shape, time constant tau_r ns),
    sampled at the light tick."""
    t = (np.arange(n_resp) + 0.5) * tick / tau_r
    r = t * np.exp(-t)
    return (r / r.sum()).astype(np.float32)


def light_noise_amplitudes(n_freq: int = 2048, sigma: float = 4.0, f_corner: float = 256.0) -> np.ndarray:
    """Amplitudes of the random-phase noise sinusoids (Sec. 4.3) for frequencies f = 1 .. n_freq (in units of one
    cycle per window): a spectrum falling as 1 / (1 + (f / f_corner)^2), scaled to an RMS of sigma ADC counts."""
    f = np.arange(1, n_freq + 1, dtype=np.float64)
    s = 1.0 / (1.0 + (f / f_corner) ** 2)
    return (np.sqrt(2.0 * s / s.sum()) * sigma).astype(np.float32)


def photocurrents(events: List[Segments], t_offsets_ns, light: Light, physics: Physics, module=(62.08, 62.08, 50.0),
                  efficiency: float = 0.005) -> np.ndarray:
    """Synthetic photocurrents I_pe[detector, tick] (p.e. emitted per tick) standing in for the visibility look-up
    table of Sec. 4.1: photons per segment from the same recombination as the charge, dN/dx = (1/W_ph - R/W_ion)
    dE/dx; detectors are 10 x 10 cm pads on the two x = const walls of the module (4 x 8 per wall in y, z); the
    visibility of a segment midpoint is efficiency x the pad's solid-angle fraction (A cos(theta) / (4 pi d^2));
    light arrives at t0 + t_offset + d / (c / 1.38)."""
    nd, T = light.n_det, light.n_ticks
    per_wall = nd // 2
    ny, nz = 4, per_wall // 4
    X, Y, Z = module
    yc = (np.arange(ny) + 0.5) * Y / ny
    zc = (np.arange(nz) + 0.5) * Z / nz
    det = np.array([(wx, y, z) for wx in (0.0, X) for y in yc for z in zc])[:nd]
    ipe = np.zeros((nd, T), np.float64)
    c_lar = 29.9792458 / 1.38                                   # cm/ns
    eps = physics.e_field * physics.lar_density
    for segs, t_off in zip(events, t_offsets_ns):
        r0 = np.stack([segs.x0, segs.y0, segs.z0], 1).astype(np.float64)
        r1 = np.stack([segs.x1, segs.y1, segs.z1], 1).astype(np.float64)
        mid = 0.5 * (r0 + r1)
        L = np.linalg.norm(r1 - r0, axis=1)
        dedx = np.where(L > 0, segs.energy / np.maximum(L, 1e-12), np.nan_to_num(segs.dedx if segs.dedx is not None
                                                                                   else np.zeros(segs.n)))
        R = physics.birks_ab / (1.0 + physics.birks_kb / eps * dedx)
        n_gamma = (1.0 / W_PH_MEV - R / physics.w_ion) * dedx * L
        t0 = 0.5 * (segs.t0 + segs.t1).astype(np.float64) * 1e3 + t_off   # us -> ns
        for i, p in enumerate(det):
            dv = mid - p[None]
            d2 = (dv ** 2).sum(1)
            cos = np.abs(dv[:, 0]) / np.sqrt(d2)
            vis = efficiency * 100.0 * cos / (4.0 * np.pi * d2)
            tick = np.floor((t0 + np.sqrt(d2) / c_lar) / light.tick).astype(np.int64)
            ok = (tick >= 0) & (tick < T)
            np.add.at(ipe[i], tick[ok], (vis * n_gamma)[ok])
    return ipe.astype(np.float32)


def light_workload(n_events: int = 4, light: Optional[Light] = None):
    """A beam-spill light event: n_events module-scale interactions (spill-sized, as cfg3) at seeded times within
    the first 10 us of the window.  Returns (light parameters, photocurrents, response kernel, noise amplitudes)."""
    light = light or Light()
    w = make_workload(3, n_events=n_events)
    rng = _rng(6, 0)
    t_off = np.sort(rng.uniform(200.0, 10000.0, size=n_events))
    ipe = photocurrents(w.events, t_off, light, w.physics)
    return light, ipe, light_response(tick=light.tick), light_noise_amplitudes()
