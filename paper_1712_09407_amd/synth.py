"""Seeded synthetic TPC events: helix tracks crossing the pad rows of 36 sectors.

This module only makes inputs.  It simulates particles (a circle in the
transverse plane, z linear in the transverse arc length), intersects them with
the pad-row planes of each sector, smears the crossings and adds uniform noise.
It holds none of the tracker's arithmetic, imports nothing else from this
package, and is shared by the oracle tests and the GPU tests alike.

Geometry (paper, section 1): two drift volumes of 18 trapezoidal sectors each,
159 pad rows per sector.  The figure with the real row radii is not available,
so rows sit at local x = 85 + 162*r/158 cm (evenly spaced from 85 to 247 cm),
the sector's half opening angle is 10 degrees and the drift length 250 cm.

Sector s has its centre line at angle alpha_s = 20deg*(s mod 18) + 10deg.  Its
local frame is x along the centre line, y perpendicular to it (rotated by
+90deg), z the global z.  Sectors 0..17 see z >= 0, sectors 18..35 see z < 0.

Units: cm, GeV, Tesla.  Positive charge in +Bz turns clockwise seen from +z.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

N_ROWS = 159
N_SECTORS = 36
ROW_X = (85.0 + 162.0 * np.arange(N_ROWS, dtype=np.float64) / 158.0).astype(np.float32)
TAN_HALF = np.float32(math.tan(math.radians(10.0)))
Z_MAX = np.float32(250.0)
R_OUT = 247.0 / math.cos(math.radians(10.0))   # outer corner of the sectors
C_LIGHT = 0.00299792458                          # GeV / (T cm)


def sector_alpha(s: int) -> float:
    """Centre-line angle of sector s in radians."""
    return math.radians(20.0 * (s % 18) + 10.0)


@dataclasses.dataclass
class EventConfig:
    """Recipe of one synthetic event.  All random draws come from `seed`."""
    n_tracks: int = 8000
    sectors: tuple = tuple(range(N_SECTORS))
    phi_range_deg: tuple = (0.0, 360.0)       # azimuth of the primaries
    ignore_membrane: bool = False             # single-sector case: z in [-250, 250]
    sigma: float = 0.1                        # cm, Gaussian smearing of y and z
    noise_frac: float = 0.05                  # noise clusters per signal cluster
    bz: float = 0.5                           # Tesla
    pt_min: float = 0.2                       # GeV: pT = pt_min + Exp(pt_mean)
    pt_mean: float = 0.6
    eta_max: float = 0.9
    vertex_sigma_z: float = 5.0
    n_loopers: int = 0                        # extra low-pT tracks, one full turn
    looper_pt: tuple = (0.1, 0.2)


PRESETS = {
    # one sector, 200 tracks, 2% noise
    "c1_sector": dict(n_tracks=200, sectors=(0,), phi_range_deg=(0.0, 20.0),
                      ignore_membrane=True, noise_frac=0.02),
    # central Pb-Pb-like event, 36 sectors, 8000 primaries, 5% noise
    "c2_central": dict(n_tracks=8000, noise_frac=0.05),
    # stress: 20000 primaries + 6000 loopers, 10% noise, sigma 0.15 cm
    "c5_stress": dict(n_tracks=20000, n_loopers=6000, noise_frac=0.10, sigma=0.15),
}


def preset(name: str, **over) -> EventConfig:
    kw = dict(PRESETS[name])
    kw.update(over)
    return EventConfig(**kw)


def batch_multiplicity(seed: int) -> int:
    """Track count of a batch/serving event: log-uniform between 100 and 8000."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return int(round(math.exp(rng.uniform(math.log(100.0), math.log(8000.0)))))


@dataclasses.dataclass
class Event:
    """One event in the tracker's input layout plus Monte-Carlo truth.

    Clusters are stored structure-of-arrays, sorted by (sector slot, row); the
    order inside a row is random.  Row r of sector slot i holds clusters
    [row_offsets[i*159 + r], row_offsets[i*159 + r + 1]).
    """
    y: np.ndarray            # float32 [N] local y (cm)
    z: np.ndarray            # float32 [N] z (cm)
    row_offsets: np.ndarray  # int32 [n_sectors*159 + 1]
    sector_id: np.ndarray    # int32 [n_sectors] physical sector of each slot
    bz: float
    mc_track: np.ndarray     # int32 [N] generating particle, -1 for noise
    y_true: np.ndarray       # float64 [N] unsmeared crossing (noise: = y)
    z_true: np.ndarray       # float64 [N]
    track_pt: np.ndarray     # float64 [n_particles]
    track_q: np.ndarray      # int8
    track_tanl: np.ndarray   # float64
    track_phi0: np.ndarray   # float64
    track_z0: np.ndarray     # float64
    config: EventConfig = None

    @property
    def n_clusters(self) -> int:
        return int(self.y.shape[0])

    @property
    def n_sectors(self) -> int:
        return int(self.sector_id.shape[0])

    def row_of(self) -> np.ndarray:
        """Global row slot (sector_slot*159 + row) of every cluster."""
        counts = np.diff(self.row_offsets)
        return np.repeat(np.arange(counts.shape[0], dtype=np.int32), counts)


def _crossings(x_r, alpha, pt, q, tanl, phi0, z0, bz, theta_max):
    """All crossings of the particles with the row planes of one sector.

    Returns (track index, row index, local y, z, local sin(phi)) in float64
    for every crossing with 0 < arc <= arc_max.  Both intersections of a
    circle with a plane are considered, which matters for loopers.
    """
    n_t = pt.shape[0]
    ca, sa = math.cos(alpha), math.sin(alpha)
    out = []
    h = np.sign(q * bz)                                  # +1 clockwise
    curved = h != 0
    # --- curved tracks: circle through the origin -------------------------
    if np.any(curved):
        idx = np.nonzero(curved)[0]
        R = pt[idx] / (C_LIGHT * abs(bz))
        hh = h[idx]
        cx = R * hh * np.sin(phi0[idx])
        cy = -R * hh * np.cos(phi0[idx])
        beta0 = np.arctan2(-cy, -cx)
        nc = cx * ca + cy * sa
        g = (x_r[None, :] - nc[:, None]) / R[:, None]       # [t, row]
        ok = np.abs(g) <= 1.0
        ac = np.arccos(np.clip(g, -1.0, 1.0))
        for sgn in (+1.0, -1.0):
            th = np.mod(hh[:, None] * (beta0[:, None] - alpha - sgn * ac), 2.0 * math.pi)
            good = ok & (th > 0.0) & (th <= theta_max[idx][:, None])
            ti, ri = np.nonzero(good)
            th_g = th[ti, ri]
            Rg = R[ti]
            beta = beta0[ti] - hh[ti] * th_g
            X = cx[ti] + Rg * np.cos(beta)
            Y = cy[ti] + Rg * np.sin(beta)
            yl = -X * sa + Y * ca
            zz = z0[idx][ti] + tanl[idx][ti] * Rg * th_g
            phi = phi0[idx][ti] - hh[ti] * th_g
            out.append((idx[ti], ri, yl, zz, np.sin(phi - alpha)))
    # --- straight tracks (q*bz == 0) ----------------------------------------
    if np.any(~curved):
        idx = np.nonzero(~curved)[0]
        cd = np.cos(phi0[idx] - alpha)
        good_t = cd > 0
        s = x_r[None, :] / np.where(good_t, cd, 1.0)[:, None]
        smax = np.minimum(theta_max[idx], R_OUT)             # theta_max holds arc here
        good = good_t[:, None] & (s <= smax[:, None])
        ti, ri = np.nonzero(good)
        sg = s[ti, ri]
        X = sg * np.cos(phi0[idx][ti])
        Y = sg * np.sin(phi0[idx][ti])
        yl = -X * sa + Y * ca
        zz = z0[idx][ti] + tanl[idx][ti] * sg
        out.append((idx[ti], ri, yl, zz, np.sin(phi0[idx][ti] - alpha)))
    if not out:
        return [np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0), np.zeros(0), np.zeros(0)]
    cat = [np.concatenate([o[k] for o in out]) for k in range(5)]
    return cat


def _arc_limit(pt, q, tanl, z0, bz, looper):
    """Turning-angle (curved) or arc-length (straight) limit of each particle."""
    n = pt.shape[0]
    h = np.sign(q * bz)
    lim = np.full(n, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        R = np.where(h != 0, pt / (C_LIGHT * abs(bz) if bz != 0 else 1.0), np.inf)
        # z limit: |z| <= 250 along the arc
        zlim_arc = np.where(tanl > 0, (float(Z_MAX) - z0) / tanl,
                            np.where(tanl < 0, (-float(Z_MAX) - z0) / tanl, np.inf))
        # radial limit for primaries: chord from origin 2R sin(theta/2) <= R_OUT
        curved = h != 0
        th_r = np.where(curved & (2.0 * R > R_OUT),
                        2.0 * np.arcsin(np.clip(R_OUT / (2.0 * R), 0.0, 1.0)), 2.0 * math.pi)
        th_z = zlim_arc / R
        lim = np.where(curved, np.minimum(np.minimum(th_r, th_z), 2.0 * math.pi),
                       np.minimum(zlim_arc, R_OUT))
    return lim


def make_event(cfg: EventConfig, seed: int) -> Event:
    """Build one event from `cfg` using numpy PCG64(seed) for every draw."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_p = int(cfg.n_tracks)
    n_l = int(cfg.n_loopers)
    n_all = n_p + n_l
    # particle draws, in a fixed order
    z0 = rng.normal(0.0, cfg.vertex_sigma_z, n_all)
    pt = np.concatenate([cfg.pt_min + rng.exponential(cfg.pt_mean, n_p),
                         rng.uniform(cfg.looper_pt[0], cfg.looper_pt[1], n_l)])
    eta = rng.uniform(-cfg.eta_max, cfg.eta_max, n_all)
    tanl = np.sinh(eta)
    lo, hi = (math.radians(v) for v in cfg.phi_range_deg)
    phi0 = rng.uniform(lo, hi, n_all)
    q = np.where(rng.uniform(0.0, 1.0, n_all) < 0.5, -1, 1).astype(np.int8)
    looper = np.zeros(n_all, bool)
    looper[n_p:] = True
    lim = _arc_limit(pt, q.astype(np.float64), tanl, z0, cfg.bz, looper)

    x_r = ROW_X.astype(np.float64)
    half_w = (ROW_X * TAN_HALF).astype(np.float64)          # FP32 trapezoid edge, widened
    sectors = list(cfg.sectors)
    ys, zs, yts, zts, rows, secs, mcs = [], [], [], [], [], [], []
    for slot, s in enumerate(sectors):
        ti, ri, yl, zz, _sphi = _crossings(x_r, sector_alpha(s), pt, q.astype(np.float64),
                                           tanl, phi0, z0, cfg.bz, lim)
        order = np.lexsort((ti, ri))                        # deterministic draw order
        ti, ri, yl, zz = ti[order], ri[order], yl[order], zz[order]
        if cfg.sigma > 0:
            dy = rng.normal(0.0, cfg.sigma, ti.shape[0])
            dz = rng.normal(0.0, cfg.sigma, ti.shape[0])
        else:
            dy = np.zeros(ti.shape[0])
            dz = np.zeros(ti.shape[0])
        ym = (yl + dy).astype(np.float32)
        zm = (zz + dz).astype(np.float32)
        keep = np.abs(ym.astype(np.float64)) <= half_w[ri]
        keep &= np.abs(zm) <= Z_MAX
        if not cfg.ignore_membrane:
            keep &= (zm >= 0) if s < 18 else (zm < 0)
        n_sig = int(keep.sum())
        ys.append(ym[keep]); zs.append(zm[keep]); yts.append(yl[keep]); zts.append(zz[keep])
        rows.append(ri[keep].astype(np.int32)); secs.append(np.full(n_sig, slot, np.int32))
        mcs.append(ti[keep].astype(np.int32))
        # noise clusters of this sector
        n_noise = int(round(cfg.noise_frac * n_sig))
        if n_noise:
            nr = rng.integers(0, N_ROWS, n_noise)
            u = rng.uniform(-1.0, 1.0, n_noise)
            yn = (u * half_w[nr]).astype(np.float32)
            if cfg.ignore_membrane:
                zn = rng.uniform(-float(Z_MAX), float(Z_MAX), n_noise)
            elif s < 18:
                zn = rng.uniform(0.0, float(Z_MAX), n_noise)
            else:
                zn = -rng.uniform(0.0, float(Z_MAX), n_noise)
                zn = np.where(zn == 0.0, -1e-3, zn)
            zn = zn.astype(np.float32)
            ys.append(yn); zs.append(zn)
            yts.append(yn.astype(np.float64)); zts.append(zn.astype(np.float64))
            rows.append(nr.astype(np.int32)); secs.append(np.full(n_noise, slot, np.int32))
            mcs.append(np.full(n_noise, -1, np.int32))
    y = np.concatenate(ys); z = np.concatenate(zs)
    yt = np.concatenate(yts); zt = np.concatenate(zts)
    row = np.concatenate(rows); sec = np.concatenate(secs); mc = np.concatenate(mcs)
    # random order inside each (sector, row)
    key = rng.permutation(y.shape[0])
    order = np.lexsort((key, row, sec))
    y, z, yt, zt, row, sec, mc = (a[order] for a in (y, z, yt, zt, row, sec, mc))
    slot_row = sec.astype(np.int64) * N_ROWS + row
    counts = np.bincount(slot_row, minlength=len(sectors) * N_ROWS)
    row_offsets = np.zeros(len(sectors) * N_ROWS + 1, np.int64)
    np.cumsum(counts, out=row_offsets[1:])
    return Event(y=np.ascontiguousarray(y, np.float32), z=np.ascontiguousarray(z, np.float32),
                 row_offsets=row_offsets.astype(np.int32),
                 sector_id=np.asarray(sectors, np.int32), bz=float(cfg.bz),
                 mc_track=mc.astype(np.int32), y_true=yt, z_true=zt,
                 track_pt=pt, track_q=q, track_tanl=tanl, track_phi0=phi0, track_z0=z0,
                 config=cfg)


def make_preset(name: str, seed: int, **over) -> Event:
    return make_event(preset(name, **over), seed)


def batch_event(seed: int, **over) -> Event:
    """An event of the batched / serving workload: 36 sectors, log-uniform multiplicity."""
    return make_event(EventConfig(n_tracks=batch_multiplicity(seed), **over), seed)
