"""Synthetic helix events for the TPC track-finding hot path.

Geometry (a reading of the paper's setting; the paper itself gives none):
  * 152 pad rows per sector, modelled as planes of constant sector-local x,
    x_i = 85 + i * 160/151 cm (85 cm to 245 cm, uniform pitch);
  * 18 sectors of 20 degrees per z side, sector s has its centre at
    ((s mod 18) + 0.5) * 20 degrees; sectors 0..17 are z >= 0, 18..35 z < 0;
  * uniform field B = 0.5 T along +z; a track of charge q and transverse
    momentum pT has signed curvature k = -0.00299792458 * B * q / pT [1/cm],
    so positive charges turn clockwise seen from +z;
  * drift length 250 cm; in continuous read-out the tracker sees
    z* = z - vd * t_collision (side A) with vd = 2.58 cm/us (the paper's
    linear time-to-z scaling with the average drift velocity, section 2).

All geometry is computed in float64 and rounded to float32 once.  Every
random draw comes from numpy's PCG64 seeded generator.
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

N_ROWS = 152
ROW_X64 = 85.0 + np.arange(N_ROWS, dtype=np.float64) * (160.0 / 151.0)
ROW_X = ROW_X64.astype(np.float32)
B_TESLA = 0.5
CURV_PER_QPT64 = -0.00299792458 * B_TESLA       # 1/cm per (GeV/c)^-1
CURV_PER_QPT = np.float32(CURV_PER_QPT64)
SIGMA = 0.1                                    # cm, cluster smear in y and z
DRIFT_LEN = 250.0                              # cm
VD_CM_PER_US = 2.58                            # cm/us
TAN10 = math.tan(math.radians(10.0))
SECTOR_WIDTH = math.radians(20.0)
N_SECTORS_PER_SIDE = 18

CONFIG_SEEDS = {1: 1001, 2: 2002, 3: 3003, 4: 40040000, 5: 5005}


def default_params() -> dict:
    """Physics constants and cuts that define the tracker's outputs.

    These are inputs to both the oracle and the HIP library; the values are
    this project's readings (the paper states none of them)."""
    return dict(
        curv=float(CURV_PER_QPT),   # curvature per unit q/pT
        nb_win_y=2.5,               # neighbour window half-width in y [cm]
        nb_win_z=2.5,               # neighbour window half-width in z [cm]
        nb_d2max=1.0,               # max straight-line deviation^2 [cm^2]
        sigma_y2=SIGMA * SIGMA,     # measurement variance y [cm^2]
        sigma_z2=SIGMA * SIGMA,     # measurement variance z [cm^2]
        chi2_max=16.0,              # hit-search gate (2 d.o.f.)
        search_nsigma=4.0,          # bin window of the hit search, in sigma
        s_max=0.95,                 # stop when |sin(phi)| reaches this
        c_ss0=0.01, c_tt0=0.01, c_ww0=100.0,  # initial variances s, t, q/pT
        max_miss=8,                 # consecutive rows without a hit
        min_tracklet_hits=10,
        min_track_hits=10,
    )


@dataclasses.dataclass
class Event:
    """Clusters of one or more sectors, grouped by sector (CSR)."""
    row: np.ndarray            # uint8 [n]
    y: np.ndarray              # float32 [n], sector-local y [cm]
    z: np.ndarray              # float32 [n], z (or z*) [cm]
    charge: np.ndarray         # float32 [n] (not used by the tracker)
    sector_offsets: np.ndarray  # int64 [n_sectors + 1]
    sector_range: np.ndarray   # float32 [n_sectors, 4]: ymin, ymax, zmin, zmax
    row_x: np.ndarray          # float32 [152]
    label: np.ndarray          # int32 [n]: generating track, -1 for noise
    tracks: dict               # float64 arrays: vx vy vz phi0 tanl qpt
    meta: dict
    sector_side: np.ndarray = None   # int8 [n_sectors]: +1 z >= 0 side, -1 z < 0

    def __post_init__(self):
        if self.sector_side is None:
            self.sector_side = np.ones(self.sector_offsets.shape[0] - 1, np.int8)

    @property
    def n_clusters(self) -> int:
        return int(self.row.shape[0])

    @property
    def n_sectors(self) -> int:
        return int(self.sector_offsets.shape[0] - 1)

    def sector(self, s: int) -> "Event":
        """One sector as a stand-alone single-sector event."""
        a, b = int(self.sector_offsets[s]), int(self.sector_offsets[s + 1])
        return Event(self.row[a:b], self.y[a:b], self.z[a:b], self.charge[a:b],
                     np.array([0, b - a], np.int64), self.sector_range[s:s + 1].copy(),
                     self.row_x, self.label[a:b], self.tracks, dict(self.meta, sector=s),
                     self.sector_side[s:s + 1].copy())


@dataclasses.dataclass
class RefitSet:
    """Found-track hit lists for the calibrated refit (CSR over tracks)."""
    trk_off: np.ndarray   # int32 [n_tracks + 1]
    row: np.ndarray       # uint8 [n_hits]
    y: np.ndarray         # float32 [n_hits], raw (uncalibrated) y
    z: np.ndarray         # float32 [n_hits], raw z
    row_x: np.ndarray     # float32 [152]
    theta_true: np.ndarray  # float64 [16], distortion used to make the data
    theta_eval: np.ndarray  # float32 [16], point where the refit is evaluated
    tracks: dict
    meta: dict

    @property
    def n_tracks(self) -> int:
        return int(self.trk_off.shape[0] - 1)

    @property
    def n_hits(self) -> int:
        return int(self.row.shape[0])


# --------------------------------------------------------------------------
# helix geometry (float64)

def helix_plane_point(vx, vy, vz, phi0, tanl, k, alpha, X, max_turn=math.pi,
                      n_turns=1):
    """Crossings of helices with the sector-local plane x_local = X.

    Helix: vertex (vx, vy, vz), direction phi0 at the vertex, dip tanl,
    signed curvature k [1/cm].  Sector frame rotated by alpha.  Arguments
    broadcast.  Returns a list of (valid, y_local, z, turning_angle), one
    entry per circle solution and turn, turning angle = |k| * arc length.
    """
    xc = vx - np.sin(phi0) / k
    yc = vy + np.cos(phi0) / k
    ca, sa = np.cos(alpha), np.sin(alpha)
    xcl = xc * ca + yc * sa
    ycl = -xc * sa + yc * ca
    phi0l = phi0 - alpha
    u = k * (X - xcl)
    ok = np.abs(u) <= 1.0
    a1 = np.arcsin(np.clip(u, -1.0, 1.0))
    out = []
    for sol in (a1, math.pi - a1):
        dphi = sol - phi0l
        turn0 = np.where(k > 0, np.mod(dphi, 2 * math.pi), np.mod(-dphi, 2 * math.pi))
        yl = ycl - np.cos(sol) / k
        for n in range(n_turns):
            turn = turn0 + 2 * math.pi * n
            z = vz + (turn / np.abs(k)) * tanl
            out.append((ok & (turn <= max_turn), yl, z, turn))
    return out


def _sample_tracks(rng, n, phi_lo, phi_hi, eta_lo, eta_hi, pt_min, pt_mean=0.5):
    """Track kinematics: pT ~ exponential(mean) truncated below at pt_min.

    The truncated exponential equals pt_min + Exp(mean) (memorylessness)."""
    phi0 = rng.uniform(phi_lo, phi_hi, n)
    eta = rng.uniform(eta_lo, eta_hi, n)
    pt = pt_min + rng.exponential(pt_mean, n)
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return dict(vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n), phi0=phi0,
                tanl=np.sinh(eta), qpt=q / pt)


def _concat_tracks(a, b):
    return {k: np.concatenate([a[k], b[k]]) for k in a}


def _smear32(rng, v):
    return (v + rng.normal(0.0, SIGMA, v.shape)).astype(np.float32)


def _instance_clusters(rng, trk, max_turn=math.pi):
    """All first-leg crossings of the 152 planes in one sector frame with no
    azimuthal edge (frame centred at 10 degrees), z >= 0 side."""
    alpha = math.radians(10.0)
    k = CURV_PER_QPT64 * trk["qpt"]
    rows, ys, zs, labs = [], [], [], []
    T = k.shape[0]
    X = ROW_X64[None, :]
    sols = helix_plane_point(
        trk["vx"][:, None], trk["vy"][:, None], trk["vz"][:, None],
        trk["phi0"][:, None], trk["tanl"][:, None], k[:, None], alpha, X,
        max_turn=max_turn)
    # no azimuthal edge: keep the first crossing of each plane only, where the
    # track still moves outwards in local x (the arcsin branch, cos(phi) >= 0)
    for valid, yl, z, _ in sols[:1]:
        m = valid & (z >= 0.0) & (z <= DRIFT_LEN)
        ti, ri = np.nonzero(m)
        rows.append(ri)
        ys.append(yl[ti, ri])
        zs.append(z[ti, ri])
        labs.append(ti)
    row = np.concatenate(rows)
    y = np.concatenate(ys)
    z = np.concatenate(zs)
    lab = np.concatenate(labs)
    del T
    return row, y, z, lab


def _add_noise_and_pack(rng, row, y, z, lab, frac, ylim_rows, zlo, zhi):
    """Append frac * len(row) uniform noise clusters, smear, shuffle."""
    n_noise = int(round(frac * row.shape[0]))
    nrow = rng.integers(0, N_ROWS, n_noise)
    ylim = ylim_rows[nrow]
    ny = rng.uniform(-ylim, ylim)
    nz = rng.uniform(zlo, zhi, n_noise)
    ys = _smear32(rng, y)
    zs = _smear32(rng, z)
    row = np.concatenate([row, nrow]).astype(np.uint8)
    y32 = np.concatenate([ys, ny.astype(np.float32)])
    z32 = np.concatenate([zs, nz.astype(np.float32)])
    lab = np.concatenate([lab, -np.ones(n_noise, np.int64)]).astype(np.int32)
    perm = rng.permutation(row.shape[0])
    return row[perm], y32[perm], z32[perm], lab[perm]


def make_sector_instance(rng, n_tracks, noise_frac=0.05, pt_min=0.1):
    """One single-sector instance with no azimuthal edge: n_tracks primaries
    from the origin, phi0 ~ U(0, 20 deg), eta ~ U(0, 0.9), first leg only."""
    trk = _sample_tracks(rng, n_tracks, 0.0, math.radians(20.0), 0.0, 0.9, pt_min)
    row, y, z, lab = _instance_clusters(rng, trk)
    ylim = ROW_X64 * TAN10
    row, y, z, lab = _add_noise_and_pack(rng, row, y, z, lab, noise_frac, ylim,
                                         0.0, DRIFT_LEN)
    return row, y, z, lab, trk


def _pack_instances(parts, meta):
    rows, ys, zs, qs, labs, offs, rng_ = [], [], [], [], [], [0], []
    tracks = None
    base = 0
    for row, y, z, lab, trk, q in parts:
        rows.append(row)
        ys.append(y)
        zs.append(z)
        qs.append(q)
        labs.append(np.where(lab >= 0, lab + base, -1).astype(np.int32))
        base += trk["qpt"].shape[0]
        tracks = trk if tracks is None else _concat_tracks(tracks, trk)
        offs.append(offs[-1] + row.shape[0])
        if row.shape[0]:
            rng_.append([float(y.min()), float(y.max()), 0.0, DRIFT_LEN])
        else:
            rng_.append([-1.0, 1.0, 0.0, DRIFT_LEN])
    return Event(np.concatenate(rows), np.concatenate(ys), np.concatenate(zs),
                 np.concatenate(qs), np.array(offs, np.int64),
                 np.array(rng_, np.float32), ROW_X.copy(), np.concatenate(labs),
                 tracks, meta)


def make_config1(seed=CONFIG_SEEDS[1], n_tracks=50):
    """Single sector instance: 50 primaries, +5% noise (about 7-8k clusters)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    row, y, z, lab, trk = make_sector_instance(rng, n_tracks)
    q = rng.gamma(2.0, 20.0, row.shape[0]).astype(np.float32)
    return _pack_instances([(row, y, z, lab, trk, q)],
                           dict(config=1, seed=seed, n_tracks=n_tracks))


def make_config4(seed=CONFIG_SEEDS[4], n_instances=512):
    """Batched uneven workload: n_instances single-sector instances, half
    pp-like (20-200 tracks) and half Pb-Pb-like (50-800 tracks), track
    counts log-uniform, instance order shuffled."""
    rng = np.random.Generator(np.random.PCG64(seed))
    half = n_instances // 2
    n_pp = np.exp(rng.uniform(math.log(20), math.log(200), half))
    n_pb = np.exp(rng.uniform(math.log(50), math.log(800), n_instances - half))
    ntrk = np.rint(np.concatenate([n_pp, n_pb])).astype(np.int64)
    ntrk = ntrk[rng.permutation(n_instances)]
    parts = []
    for i in range(n_instances):
        r = np.random.Generator(np.random.PCG64(seed + 1 + i))
        row, y, z, lab, trk = make_sector_instance(r, int(ntrk[i]))
        q = r.gamma(2.0, 20.0, row.shape[0]).astype(np.float32)
        parts.append((row, y, z, lab, trk, q))
    return _pack_instances(parts, dict(config=4, seed=seed, n_instances=n_instances,
                                       tracks_per_instance=ntrk.tolist()))


def _crossings_chunk(trk, k_all, a, b, max_turn, n_turns, offset=0, chunk=512):
    if b - a > chunk:
        parts = [_crossings_chunk(trk, k_all, c, min(b, c + chunk), max_turn, n_turns, offset)
                 for c in range(a, b, chunk)]
        return tuple(np.concatenate([p[i] for p in parts]) for i in range(5))
    alphas = (np.arange(N_SECTORS_PER_SIDE) + 0.5) * SECTOR_WIDTH
    ylim_row = ROW_X64 * TAN10
    sl = slice(a, b)
    k = k_all[sl]
    vx, vy, vz = trk["vx"][sl], trk["vy"][sl], trk["vz"][sl]
    phi0, tanl = trk["phi0"][sl], trk["tanl"][sl]
    # (track, sector) pairs whose circle can reach the sector's rows: the
    # circle's local x extent must meet [x_0, x_last] and its y extent the
    # widest acceptance (a necessary condition; the exact tests follow)
    xc = vx - np.sin(phi0) / k
    yc = vy + np.cos(phi0) / k
    ca, sa = np.cos(alphas), np.sin(alphas)
    xcl = xc[:, None] * ca[None, :] + yc[:, None] * sa[None, :]
    ycl = -xc[:, None] * sa[None, :] + yc[:, None] * ca[None, :]
    R = (1.0 / np.abs(k))[:, None]
    ymax = float(ylim_row[-1])
    keep = ((xcl + R >= ROW_X64[0]) & (xcl - R <= ROW_X64[-1]) &
            (ycl + R >= -ymax) & (ycl - R <= ymax))
    ti, si = np.nonzero(keep)
    # later turns only for helices that stay inside the outer radius of the
    # drift volume; any other track leaves it within its first half turn
    r_out = ROW_X64[-1] / math.cos(SECTOR_WIDTH / 2)
    contained = np.hypot(xc, yc) + 1.0 / np.abs(k) <= r_out
    tmax = np.where(contained, max_turn, min(max_turn, math.pi))
    out = ([], [], [], [], [])
    if ti.shape[0] == 0:
        return tuple(np.zeros(0, d) for d in (np.int64, np.int64, np.float64, np.float64,
                                              np.int64))
    col = lambda v: v[ti][:, None]
    for valid, yl, z, turn in helix_plane_point(col(vx), col(vy), col(vz), col(phi0),
                                                 col(tanl), col(k), alphas[si][:, None],
                                                 ROW_X64[None, :], max_turn=max_turn,
                                                 n_turns=n_turns):
        m = (valid & (turn <= col(tmax)) & (np.abs(yl) <= ylim_row[None, :]) &
             (np.abs(z) <= DRIFT_LEN))
        pi, ri = np.nonzero(m)
        zz = z[pi, ri]
        out[0].append(si[pi] + N_SECTORS_PER_SIDE * (zz < 0))
        out[1].append(ri)
        out[2].append(yl[pi, ri])
        out[3].append(zz)
        out[4].append(ti[pi] + a + offset)
    return tuple(np.concatenate(v) for v in out)


def _crossings_task(args):
    trk, k_all, a, max_turn, n_turns = args
    return _crossings_chunk(trk, k_all, 0, k_all.shape[0], max_turn, n_turns, offset=a)


def _sector_crossings(trk, max_turn=math.pi, n_turns=1, chunk=512, workers=None):
    """Crossings of tracks with the row planes of all 36 real 20-degree
    sectors.  Returns (sector, row, y_local, z, label).  Pure geometry (no
    random numbers): large track sets are split over worker processes
    (started fresh, so that a parent process that uses a GPU is never
    forked), the chunks joined in track order, so the result does not depend
    on the number of workers; TPC_SYNTH_WORKERS sets it)."""
    k_all = CURV_PER_QPT64 * trk["qpt"]
    T = k_all.shape[0]
    ranges = [(a, min(T, a + chunk)) for a in range(0, T, chunk)]
    if workers is None:
        # TPC_SYNTH_WORKERS=1 keeps the work in this process (for runs under a
        # profiler that instruments every child process)
        workers = int(os.environ.get("TPC_SYNTH_WORKERS", min(16, os.cpu_count() or 1)))
    if workers > 1 and len(ranges) >= 16:
        import multiprocessing as mp
        keys = ("vx", "vy", "vz", "phi0", "tanl")
        per = -(-len(ranges) // (4 * workers))          # ranges per task
        tasks = []
        for i in range(0, len(ranges), per):
            a, b = ranges[i][0], ranges[min(i + per, len(ranges)) - 1][1]
            tasks.append(({k: trk[k][a:b] for k in keys}, k_all[a:b], a, max_turn, n_turns))
        with mp.get_context("spawn").Pool(min(workers, len(tasks))) as pool:
            parts = pool.map(_crossings_task, tasks)
    else:
        parts = [_crossings_chunk(trk, k_all, a, b, max_turn, n_turns) for a, b in ranges]
    return tuple(np.concatenate([p[i] for p in parts]) for i in range(5))


def _secondaries(rng, n, pt_min=0.1):
    trk = _sample_tracks(rng, n, 0.0, 2 * math.pi, -0.9, 0.9, pt_min)
    r = 50.0 * rng.random(n) ** (1.0 / 3.0)
    cth = rng.uniform(-1, 1, n)
    ph = rng.uniform(0, 2 * math.pi, n)
    sth = np.sqrt(1 - cth * cth)
    trk["vx"] = r * sth * np.cos(ph)
    trk["vy"] = r * sth * np.sin(ph)
    trk["vz"] = r * cth
    return trk


def make_event(rng, n_primary, sec_frac=0.10, noise_frac=0.05, pt_min=0.1):
    """Clusters of one collision in the 36 real sectors (triggered frame)."""
    prim = _sample_tracks(rng, n_primary, 0.0, 2 * math.pi, -0.9, 0.9, pt_min)
    sec = _secondaries(rng, int(round(sec_frac * n_primary)), pt_min)
    trk = _concat_tracks(prim, sec)
    sector, row, y, z, lab = _sector_crossings(trk)
    y = _smear32(rng, y)
    z = _smear32(rng, z)
    n_noise = int(round(noise_frac * row.shape[0]))
    ns = rng.integers(0, 2 * N_SECTORS_PER_SIDE, n_noise)
    nr = rng.integers(0, N_ROWS, n_noise)
    ylim = ROW_X64[nr] * TAN10
    ny = rng.uniform(-ylim, ylim).astype(np.float32)
    nz = rng.uniform(0.0, DRIFT_LEN, n_noise)
    nz = np.where(ns >= N_SECTORS_PER_SIDE, -nz, nz).astype(np.float32)
    sector = np.concatenate([sector, ns])
    row = np.concatenate([row, nr])
    y = np.concatenate([y, ny])
    z = np.concatenate([z, nz])
    lab = np.concatenate([lab, -np.ones(n_noise, np.int64)])
    return sector, row, y, z, lab, trk


def _pack_sectors(rng, sector, row, y, z, lab, trk, zranges, meta):
    n_sec = 2 * N_SECTORS_PER_SIDE
    key = sector.astype(np.uint8)
    # group by sector, random order inside each sector (a stable sort of a
    # uint8 key is a radix sort)
    perm = rng.permutation(key.shape[0])
    order = perm[np.argsort(key[perm], kind="stable")]
    counts = np.bincount(key, minlength=n_sec)
    offs = np.zeros(n_sec + 1, np.int64)
    offs[1:] = np.cumsum(counts)
    ymax = float(ROW_X64[-1] * TAN10)
    srange = np.array([[-ymax, ymax, zr[0], zr[1]] for zr in zranges], np.float32)
    charge = rng.gamma(2.0, 20.0, row.shape[0]).astype(np.float32)
    side = np.array([1] * N_SECTORS_PER_SIDE + [-1] * N_SECTORS_PER_SIDE, np.int8)
    return Event(row[order].astype(np.uint8), y[order].astype(np.float32),
                 z[order].astype(np.float32), charge, offs, srange, ROW_X.copy(),
                 lab[order].astype(np.int32), trk, meta, side)


def make_config2(seed=CONFIG_SEEDS[2], n_primary=8000):
    """One central Pb-Pb-like event: 36 sectors, 8000 primaries plus 10%
    secondaries from vertices uniform in a 50 cm ball, +5% noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sector, row, y, z, lab, trk = make_event(rng, n_primary)
    zr = [(0.0, DRIFT_LEN)] * N_SECTORS_PER_SIDE + [(-DRIFT_LEN, 0.0)] * N_SECTORS_PER_SIDE
    return _pack_sectors(rng, sector, row, y, z, lab, trk, zr,
                         dict(config=2, seed=seed, n_primary=n_primary))


def make_config3(seed=CONFIG_SEEDS[3], n_collisions=100, rate_khz=50.0,
                 n_primary_central=8000, pt_min=0.05, max_turns=3):
    """Continuous read-out slice: n_collisions collisions with Poisson
    arrival times at rate_khz, multiplicity U(5%, 100%) of the central event,
    loopers followed up to max_turns turns; the tracker sees
    z* = z - sgn(z) * vd * t_collision.  Random draws: arrival times, then
    every collision's tracks, then per collision its smearing and noise (the
    crossings of all tracks are computed in between, in one parallel pass)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t_us = np.cumsum(rng.exponential(1e3 / rate_khz, n_collisions))
    t_us -= t_us[0]
    colls = []
    for c in range(n_collisions):
        f = rng.uniform(0.05, 1.0)
        n_p = int(round(f * n_primary_central))
        prim = _sample_tracks(rng, n_p, 0.0, 2 * math.pi, -0.9, 0.9, pt_min)
        sec = _secondaries(rng, int(round(0.1 * n_p)), pt_min)
        trk = _concat_tracks(prim, sec)
        trk["t_us"] = np.full(trk["qpt"].shape[0], t_us[c])
        colls.append(trk)
    tracks = {k: np.concatenate([t[k] for t in colls]) for k in colls[0]}
    first = np.zeros(n_collisions + 1, np.int64)
    first[1:] = np.cumsum([t["qpt"].shape[0] for t in colls])
    x_sector, x_row, x_y, x_z, x_lab = _sector_crossings(
        tracks, max_turn=2 * math.pi * max_turns, n_turns=max_turns)
    # crossings come in track order
    bounds = np.searchsorted(x_lab, first)
    parts = []
    for c in range(n_collisions):
        a, b = bounds[c], bounds[c + 1]
        sector, row, lab = x_sector[a:b], x_row[a:b], x_lab[a:b]
        y = _smear32(rng, x_y[a:b])
        z = _smear32(rng, x_z[a:b])
        n_noise = int(round(0.05 * row.shape[0]))
        ns = rng.integers(0, 2 * N_SECTORS_PER_SIDE, n_noise)
        nr = rng.integers(0, N_ROWS, n_noise)
        ylim = ROW_X64[nr] * TAN10
        ny = rng.uniform(-ylim, ylim).astype(np.float32)
        nz = rng.uniform(0.0, DRIFT_LEN, n_noise)
        nz = np.where(ns >= N_SECTORS_PER_SIDE, -nz, nz).astype(np.float32)
        sector = np.concatenate([sector, ns])
        row = np.concatenate([row, nr])
        zz = np.concatenate([z, nz]).astype(np.float64)
        shift = VD_CM_PER_US * t_us[c]
        zstar = np.where(sector >= N_SECTORS_PER_SIDE, zz + shift, zz - shift)
        lab = np.concatenate([lab, -np.ones(n_noise, np.int64)])
        parts.append((sector, row, np.concatenate([y, ny]), zstar.astype(np.float32), lab))
    sector, row, y, z, lab = (np.concatenate([p[i] for p in parts]) for i in range(5))
    zmin = -VD_CM_PER_US * float(t_us[-1])
    zr = [(zmin, DRIFT_LEN)] * N_SECTORS_PER_SIDE + [(-DRIFT_LEN, -zmin)] * N_SECTORS_PER_SIDE
    return _pack_sectors(rng, sector, row, y, z, lab, tracks, zr,
                         dict(config=3, seed=seed, n_collisions=n_collisions,
                              collision_t_us=t_us.tolist()))


# --------------------------------------------------------------------------
# calibrated refit workload

def _distortion(theta, xr, y_raw, z_raw, side=1.0):
    """Detector distortion model evaluated at raw coordinates: returns the
    true plane shift, the true y shift and the true z for a raw cluster of a
    sector on z side `side` (+1 or -1).
    theta = (vd scale, t0 [us], a0..a6 radial, c0..c6 azimuthal)."""
    sgn = side
    d_raw = DRIFT_LEN - sgn * z_raw
    d = (1.0 + theta[0]) * (d_raw - VD_CM_PER_US * theta[1])
    z = sgn * (DRIFT_LEN - d)
    u = (xr - 165.0) / 80.0
    v = y_raw / (xr * TAN10)
    w = d / DRIFT_LEN
    basis = (np.ones_like(u), u, v, u * u, u * v, v * v, w)
    dr = sum(theta[2 + j] * basis[j] for j in range(7))
    drphi = sum(theta[9 + j] * basis[j] for j in range(7))
    return dr, drphi, z


def _segment_points(trk, ti, xr):
    """Outgoing (arcsin-branch) crossing of track ti with plane x_local = xr in
    the single-sector frame; origin vertex.  Returns (u = sin(phi_local), y, z,
    turning angle)."""
    alpha = math.radians(10.0)
    k = CURV_PER_QPT64 * trk["qpt"][ti]
    phi0 = trk["phi0"][ti]
    xcl = -np.sin(phi0 - alpha) / k          # circle centre in the local frame
    ycl = np.cos(phi0 - alpha) / k
    u = k * (xr - xcl)
    uc = np.clip(u, -1.0, 1.0)
    dphi = np.arcsin(uc) - (phi0 - alpha)
    turn = np.where(k > 0, np.mod(dphi, 2 * math.pi), np.mod(-dphi, 2 * math.pi))
    y = ycl - np.sqrt(1.0 - uc * uc) / k
    z = (turn / np.abs(k)) * trk["tanl"][ti]
    return u, y, z, turn


def make_config5(seed=CONFIG_SEEDS[5], n_tracks=1_000_000, n_min=40, n_max=152,
                 chunk=200_000):
    """Refit workload: n_tracks truth segments of n_min..n_max consecutive
    rows, helices from the origin in a single-sector frame with pT >= 0.2,
    smeared (Gaussian in calibrated coordinates) and distorted by theta_true;
    the refit is evaluated at theta_eval.
    Segments whose outgoing crossings leave |sin(phi)| <= 0.9 or the drift
    volume are redrawn (same length and first row)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = np.zeros(16)
    theta[0] = 1e-3
    theta[1] = 0.05
    theta[2:9] = rng.uniform(-0.04, 0.04, 7)
    theta[9:16] = rng.uniform(-0.04, 0.04, 7)
    dtheta = np.zeros(16)
    dtheta[0] = 5e-4
    dtheta[1] = 0.02
    dtheta[2:16] = rng.uniform(-0.01, 0.01, 14)
    theta_eval = (theta + dtheta).astype(np.float32)
    nh = rng.integers(n_min, n_max + 1, n_tracks)
    r0 = rng.integers(0, N_ROWS - nh + 1)
    trk = _sample_tracks(rng, n_tracks, 0.0, math.radians(20.0), 0.0, 0.9, 0.2)
    # a segment is valid if its first and last plane crossings are: sin(phi)
    # and z grow monotonically along the outgoing branch
    todo = np.arange(n_tracks)
    for _ in range(100):
        ok = np.ones(todo.shape[0], bool)
        for rr in (r0[todo], r0[todo] + nh[todo] - 1):
            u, _, z, turn = _segment_points(trk, todo, ROW_X64[rr])
            ok &= (np.abs(u) <= 0.9) & (turn <= math.pi) & (z <= DRIFT_LEN - 5.0)
        bad = todo[~ok]
        if bad.shape[0] == 0:
            break
        fresh = _sample_tracks(rng, bad.shape[0], 0.0, math.radians(20.0), 0.0, 0.9, 0.2)
        for key in trk:
            trk[key][bad] = fresh[key]
        todo = bad
    off = np.zeros(n_tracks + 1, np.int64)
    off[1:] = np.cumsum(nh)
    n_hits = int(off[-1])
    row = np.empty(n_hits, np.uint8)
    y = np.empty(n_hits, np.float32)
    z = np.empty(n_hits, np.float32)
    for a in range(0, n_tracks, chunk):
        b = min(n_tracks, a + chunk)
        cnt = nh[a:b]
        ti = np.repeat(np.arange(a, b), cnt)
        ri = (np.arange(ti.shape[0]) - np.repeat(off[a:b] - off[a], cnt)) + np.repeat(r0[a:b], cnt)
        xr = ROW_X64[ri]
        # the cluster error is Gaussian in the calibrated coordinates: the
        # raw point is the one the calibration at theta maps onto the true
        # crossing of the calibrated plane plus the error
        ey = rng.normal(0.0, SIGMA, ti.shape[0])
        ez = rng.normal(0.0, SIGMA, ti.shape[0])
        _, y_raw, z_raw, _ = _segment_points(trk, ti, xr)
        for _ in range(4):     # fixed point: raw -> distortion -> true point
            dr, drphi, _ = _distortion(theta, xr, y_raw, z_raw)
            _, yt, zt, _ = _segment_points(trk, ti, xr + dr)
            y_raw = yt + ey - drphi
            d_raw = (DRIFT_LEN - (zt + ez)) / (1.0 + theta[0]) + VD_CM_PER_US * theta[1]
            z_raw = DRIFT_LEN - d_raw
        sl = slice(int(off[a]), int(off[b]))
        row[sl] = ri.astype(np.uint8)
        y[sl] = y_raw.astype(np.float32)
        z[sl] = z_raw.astype(np.float32)
    return RefitSet(off.astype(np.int32), row, y, z, ROW_X.copy(), theta, theta_eval,
                    dict(trk, n_hits=nh, first_row=r0),
                    dict(config=5, seed=seed, n_tracks=n_tracks))
