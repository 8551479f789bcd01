"""Seeded synthetic workloads for the weighting-field path.

This module only *produces inputs*: sensor cells, resistive columns, frequency
and time grids, carrier drift paths and (for convolution-only checks) synthetic
H fields.  It holds none of the method's arithmetic (no Green's function, no
collocation solve, no frequency-to-time transform, no Eq. 1 convolution), so the
HIP path and the CPU oracle can both be fed from it without sharing any of the
computation they are compared on.

Shapes follow the paper's workload: a 3D pixel with a central readout column
and corner bias columns (Results section, the 2021 test-beam pixel and the
proposed geometry figure), minimum-ionising particles crossing the diamond along
z (workflow section), and O(1e4) charge carriers per particle (GPU section).
The carrier trajectories of the paper come from HEED/Garfield++, which is not
available; they are replaced by straight drift paths (optionally with Gaussian
diffusion) toward the nearest electrode, with a Moyal-distributed number of
electron/hole pairs per micrometre of track.

All quantities are SI (metres, seconds, ohm-metres, coulombs).
"""
from __future__ import annotations

import numpy as np

UM = 1e-6
PS = 1e-12
GHZ = 1e9
OHM_CM = 1e-2            # 1 ohm*cm expressed in ohm*m
E_CHARGE = 1.602176634e-19
SEED_BASE = 13987
DRIFT_SPEED = 1e5        # 1e7 cm/s


def rng_for(k: int) -> np.random.Generator:
    """Generator used for workload ``k`` (PCG64 seeded with 13987 + k)."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + k))


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def make_cell(pitch, thickness, n_xy, n_z, eps_r=5.7):
    """Periodic p x p x T cell on an n_xy x n_xy x n_z grid."""
    return dict(L=(float(pitch), float(pitch), float(thickness)),
                N=(int(n_xy), int(n_xy), int(n_z)),
                eps_r=float(eps_r), sigma_bulk=0.0)


def standard_columns(pitch, thickness, radius, rho_readout, rho_bias,
                     n_colloc=64, length_frac=0.9):
    """Readout column on the cell axis plus the corner bias column.

    The readout column (applied voltage 1) grows from the face z = 0 into the
    bulk; the four corner bias columns coincide under the in-plane periodicity
    and form one column made of four quarter-columns in parallel, growing from
    the opposite face z = T (which is the plane z = 0 of the periodic cell).
    Resistivities are in ohm*m; ``rho_bias`` holds the four quarter values.
    """
    T = float(thickness)
    ro = dict(x=0.5 * pitch, y=0.5 * pitch, radius=float(radius),
              z_contact=0.0, z_free=length_frac * T,
              resistivity=[float(rho_readout)], n_colloc=int(n_colloc),
              v_applied=1.0)
    bias = dict(x=0.0, y=0.0, radius=float(radius),
                z_contact=T, z_free=(1.0 - length_frac) * T,
                resistivity=[float(r) for r in rho_bias], n_colloc=int(n_colloc),
                v_applied=0.0)
    return [ro, bias]


def frequency_grid_to_nyquist(n_freq, dt):
    """Frequency spacing so that n_freq samples span [0, 1/(2 dt)]."""
    return 1.0 / (2.0 * (n_freq - 1) * dt)


# --------------------------------------------------------------------------
# carriers
# --------------------------------------------------------------------------

def _segments(columns, cell):
    """Axis segments (x, y, z_lo, z_hi, radius) of every column."""
    segs = []
    for c in columns:
        z0, z1 = sorted((c["z_contact"], c["z_free"]))
        segs.append((c["x"], c["y"], z0, z1, c["radius"]))
    return segs


def nearest_axis_point(p, seg, L):
    """Nearest point to p (n,3) on a periodic column axis segment.

    Returns (points (n,3), distances (n,)).  The 27 nearest periodic images of
    the segment are searched.
    """
    x, y, z0, z1, _ = seg
    best_d = np.full(p.shape[0], np.inf)
    best = np.zeros_like(p)
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                q = np.empty_like(p)
                q[:, 0] = x + i * L[0]
                q[:, 1] = y + j * L[1]
                q[:, 2] = np.clip(p[:, 2], z0 + k * L[2], z1 + k * L[2])
                d = np.linalg.norm(p - q, axis=1)
                m = d < best_d
                best_d[m] = d[m]
                best[m] = q[m]
    return best, best_d


def inside_any_column(p, columns, cell, margin=0.0):
    L = cell["L"]
    out = np.zeros(p.shape[0], dtype=bool)
    for seg in _segments(columns, cell):
        _, d = nearest_axis_point(p, seg, L)
        out |= d <= seg[4] + margin
    return out


def uniform_starts(rng, n, columns, cell, margin=0.0):
    """n points uniform in the diamond (outside every column capsule)."""
    L = np.asarray(cell["L"])
    pts = np.zeros((0, 3))
    while pts.shape[0] < n:
        cand = rng.random((2 * n, 3)) * L
        cand = cand[~inside_any_column(cand, columns, cell, margin)]
        pts = np.concatenate([pts, cand])
    return pts[:n]


def drift_paths(starts, charges, columns, cell, n_time, dt, speed=DRIFT_SPEED,
                diffusion_sigma=0.0, rng=None):
    """Polylines P_c(t_0..t_{n_time}) of carriers drifting to the electrodes.

    Electrons (negative charge) drift to the nearest image of the readout
    column (applied voltage 1), holes to the nearest image of a bias column.
    Each step moves ``speed*dt`` toward the nearest point of the target axis
    segment, plus an isotropic Gaussian displacement of ``diffusion_sigma`` per
    axis when it is non-zero.  A carrier stops, with a fractional last step, on
    reaching the column surface (distance = radius from the axis segment); from
    then on its position stays constant.  Returns float64 (n, n_time+1, 3).
    """
    L = cell["L"]
    segs = _segments(columns, cell)
    ro = [s for s, c in zip(segs, columns) if c["v_applied"] > 0.5]
    bi = [s for s, c in zip(segs, columns) if c["v_applied"] <= 0.5]
    n = starts.shape[0]
    pos = np.zeros((n, n_time + 1, 3))
    pos[:, 0] = starts
    cur = starts.copy()
    alive = np.ones(n, dtype=bool)
    step_len = speed * dt

    def target(points, neg):
        tgt = np.zeros_like(points)
        dist = np.full(points.shape[0], np.inf)
        rad = np.zeros(points.shape[0])
        for group, sel in ((ro, neg), (bi, ~neg)):
            for seg in group:
                q, d = nearest_axis_point(points, seg, L)
                m = sel & (d < dist)
                tgt[m], dist[m], rad[m] = q[m], d[m], seg[4]
        return tgt, dist, rad

    neg = charges < 0
    if diffusion_sigma <= 0.0:
        # straight line toward a fixed target point: the nearest point of the
        # axis segment stays the nearest one while the carrier moves toward it
        tgt, dist, rad = target(cur, neg)
        u = (tgt - cur) / np.maximum(dist, 1e-30)[:, None]
        travel = np.maximum(dist - rad, 0.0)
        s = np.minimum(np.arange(n_time + 1)[None, :] * step_len, travel[:, None])
        return starts[:, None, :] + s[:, :, None] * u[:, None, :]
    for s in range(n_time):
        tgt, dist, rad = target(cur, neg)
        u = (tgt - cur) / np.maximum(dist, 1e-30)[:, None]
        move = u * step_len
        if diffusion_sigma > 0.0:
            move = move + rng.normal(0.0, diffusion_sigma, size=move.shape)
        nxt = cur + move
        _, d_next, _ = target(nxt, neg)
        hit = alive & (d_next <= rad)
        # fractional last step: stop on the surface along the drift direction
        frac = np.clip((dist - rad) / step_len, 0.0, 1.0)
        stop = cur + u * (frac * step_len)[:, None]
        nxt = np.where(hit[:, None], stop, nxt)
        nxt = np.where(alive[:, None], nxt, cur)
        alive &= ~hit
        cur = nxt
        pos[:, s + 1] = cur
    return pos


def drift_paths_torch(starts, charges, columns, cell, n_time, dt, speed=DRIFT_SPEED, diffusion_sigma=0.0,
                      seed=0, device="cpu", out_dtype=None):
    """``drift_paths`` for large carrier sets, stepped with torch on ``device``.

    Same model: each step moves ``speed*dt`` toward the nearest point of the
    target column's axis segment (electrons to the readout, holes to a bias
    column) plus an isotropic Gaussian displacement of ``diffusion_sigma`` per
    axis from a torch generator seeded with ``seed``; a carrier stops on the
    column surface with a fractional last step.  The nearest periodic image is
    found by wrapping the in-plane offset and trying the segment's images at
    z - L_z, z, z + L_z.  State in float64; the polylines are returned as
    (n, n_time+1, 3) of ``out_dtype`` (default float64) on ``device``.
    """
    import torch

    f64 = torch.float64
    dev = torch.device(device)
    out_dtype = f64 if out_dtype is None else out_dtype
    L = [float(v) for v in cell["L"]]
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    cur = torch.as_tensor(np.asarray(starts), dtype=f64, device=dev).clone()
    neg = torch.as_tensor(np.asarray(charges) < 0, device=dev)
    n = cur.shape[0]
    segs = _segments(columns, cell)
    groups = [[s for s, c in zip(segs, columns) if c["v_applied"] > 0.5],
              [s for s, c in zip(segs, columns) if c["v_applied"] <= 0.5]]

    def target(p):
        tgt = torch.zeros_like(p)
        dist = torch.full((n,), float("inf"), dtype=f64, device=dev)
        rad = torch.zeros(n, dtype=f64, device=dev)
        for gi, group in enumerate(groups):
            sel = neg if gi == 0 else ~neg
            for (x, y, z0, z1, r) in group:
                dx = p[:, 0] - x
                dx = dx - L[0] * torch.round(dx / L[0])
                dy = p[:, 1] - y
                dy = dy - L[1] * torch.round(dy / L[1])
                bz = None
                for k in (-1.0, 0.0, 1.0):
                    cz = torch.clamp(p[:, 2], z0 + k * L[2], z1 + k * L[2])
                    bz = cz if bz is None else torch.where((p[:, 2] - cz).abs() < (p[:, 2] - bz).abs(), cz, bz)
                d = torch.sqrt(dx * dx + dy * dy + (p[:, 2] - bz) ** 2)
                m = sel & (d < dist)
                q = torch.stack([p[:, 0] - dx, p[:, 1] - dy, bz], dim=1)
                tgt = torch.where(m[:, None], q, tgt)
                dist = torch.where(m, d, dist)
                rad = torch.where(m, torch.full_like(rad, r), rad)
        return tgt, dist, rad

    pos = torch.empty((n, n_time + 1, 3), dtype=out_dtype, device=dev)
    pos[:, 0] = cur.to(out_dtype)
    alive = torch.ones(n, dtype=torch.bool, device=dev)
    step_len = speed * dt
    for s in range(n_time):
        tgt, dist, rad = target(cur)
        u = (tgt - cur) / torch.clamp(dist, min=1e-30)[:, None]
        move = u * step_len
        if diffusion_sigma > 0.0:
            move = move + diffusion_sigma * torch.randn(cur.shape, generator=gen, dtype=f64, device=dev)
        nxt = cur + move
        _, d_next, _ = target(nxt)
        hit = alive & (d_next <= rad)
        frac = torch.clamp((dist - rad) / step_len, 0.0, 1.0)
        stop = cur + u * (frac * step_len)[:, None]
        nxt = torch.where(hit[:, None], stop, nxt)
        nxt = torch.where(alive[:, None], nxt, cur)
        alive &= ~hit
        cur = nxt
        pos[:, s + 1] = cur.to(out_dtype)
    return pos


def pairs_to_carriers(starts):
    """One electron (-e) and one hole (+e) at every start point."""
    n = starts.shape[0]
    pts = np.concatenate([starts, starts])
    q = np.concatenate([np.full(n, -E_CHARGE), np.full(n, E_CHARGE)])
    return pts, q


def moyal_counts(rng, n_steps, n_pairs):
    """Electron/hole pairs per track step with Moyal-distributed weights.

    lambda = -ln(g^2), g ~ N(0,1), follows the Moyal approximation of the
    Landau distribution; the weight of a step is max(lambda + 2, 0), and the
    weights are scaled to ``n_pairs`` and rounded by largest remainder.
    """
    g = rng.standard_normal(n_steps)
    lam = -np.log(np.maximum(g * g, 1e-300))
    w = np.maximum(lam + 2.0, 0.0)
    share = w / w.sum() * n_pairs
    counts = np.floor(share).astype(np.int64)
    rest = n_pairs - counts.sum()
    order = np.argsort(-(share - counts), kind="stable")
    counts[order[:rest]] += 1
    return counts


def mip_track_starts(rng, cell, columns, n_pairs, n_steps=300, margin=1.0 * UM):
    """Start points of a minimum-ionising track crossing the cell along z."""
    L = cell["L"]
    while True:
        xy = rng.random(2) * np.asarray(L[:2])
        probe = np.array([[xy[0], xy[1], 0.5 * L[2]]])
        # the track must stay clear of every column for its whole length
        ok = True
        for c in columns:
            dx = (xy[0] - c["x"] + 0.5 * L[0]) % L[0] - 0.5 * L[0]
            dy = (xy[1] - c["y"] + 0.5 * L[1]) % L[1] - 0.5 * L[1]
            if np.hypot(dx, dy) <= c["radius"] + margin:
                ok = False
        if ok and not inside_any_column(probe, columns, cell)[0]:
            break
    counts = moyal_counts(rng, n_steps, n_pairs)
    zs = (np.arange(n_steps) + 0.5) * (L[2] / n_steps)
    z = np.repeat(zs, counts)
    starts = np.stack([np.full(z.size, xy[0]), np.full(z.size, xy[1]), z], axis=1)
    return starts


# --------------------------------------------------------------------------
# synthetic H for convolution-only checks
# --------------------------------------------------------------------------

def synthetic_h_factors(rng, N, n_time, rank=3, scale=1e15):
    """Random separable factors of a synthetic field H_a(ix,iy,iz,t).

    H_a = scale * sum_r fx[r,ix,a] fy[r,iy,a] fz[r,iz,a] ft[r,t,a]; every
    voxel and lag gets a distinct value, so layout or indexing mistakes show.
    """
    nx, ny, nz = N
    return dict(fx=rng.standard_normal((rank, nx, 3)),
                fy=rng.standard_normal((rank, ny, 3)),
                fz=rng.standard_normal((rank, nz, 3)),
                ft=rng.standard_normal((rank, n_time, 3)),
                scale=float(scale))


def synthetic_h_values(f, ix, iy, iz):
    """H at voxels (ix,iy,iz) (arrays of equal length) -> (len, n_time, 3)."""
    acc = 0.0
    for r in range(f["fx"].shape[0]):
        s = f["fx"][r, ix] * f["fy"][r, iy] * f["fz"][r, iz]          # (len,3)
        acc = acc + s[:, None, :] * f["ft"][r][None, :, :]
    return f["scale"] * acc


def synthetic_h_full(f):
    """Whole synthetic H as float64 [nx][ny][nz][n_time][3] (small grids)."""
    nx, ny, nz = f["fx"].shape[1], f["fy"].shape[1], f["fz"].shape[1]
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    v = synthetic_h_values(f, ix.ravel(), iy.ravel(), iz.ravel())
    return v.reshape(nx, ny, nz, v.shape[1], 3)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def _pack(name, cell, columns, spectrum, pos, charge, track, n_tracks, note):
    return dict(name=name, cell=cell, columns=columns, spectrum=spectrum,
                carriers=dict(pos=pos, charge=charge, track=track.astype(np.int32),
                              n_tracks=int(n_tracks)),
                note=note)


def uniform_pixel_32x32x64():
    """32x32x64 grid of a 50x50x300 um cell, 16 frequencies, 64 x 20 ps, 100 carriers."""
    rng = rng_for(1)
    cell = make_cell(50 * UM, 300 * UM, 32, 64)
    cols = standard_columns(50 * UM, 300 * UM, 5 * UM, 0.1 * OHM_CM, [0.1 * OHM_CM] * 4, 64)
    spec = dict(n_freq=16, df=1.25 * GHZ, n_time=64, dt=20 * PS)
    starts = uniform_starts(rng, 50, cols, cell)
    pts, q = pairs_to_carriers(starts)
    pos = drift_paths(pts, q, cols, cell, spec["n_time"], spec["dt"])
    return _pack("px32", cell, cols, spec, pos, q, np.zeros(q.size), 1,
                 "50 e/h pairs, uniform starts, straight drift at 1e5 m/s")


def mip_pixel_128x128x256(n_pairs=10000):
    """128x128x256 grid, seeded resistivities, 256 frequencies, 200 x 10 ps, one MIP track."""
    rng = rng_for(2)
    cell = make_cell(50 * UM, 300 * UM, 128, 256)
    rho = rng.uniform(0.05, 1.0, size=5) * OHM_CM
    cols = standard_columns(50 * UM, 300 * UM, 5 * UM, rho[0], rho[1:], 64)
    dt = 10 * PS
    spec = dict(n_freq=256, df=frequency_grid_to_nyquist(256, dt), n_time=200, dt=dt)
    starts = mip_track_starts(rng, cell, cols, n_pairs)
    pts, q = pairs_to_carriers(starts)
    pos = drift_paths(pts, q, cols, cell, spec["n_time"], spec["dt"])
    return _pack("px128", cell, cols, spec, pos, q, np.zeros(q.size), 1,
                 f"one MIP track along z, {n_pairs} e/h pairs with Moyal weights")


def pixel_256x256x512_tracks(device="cpu", n_tracks=100, n_pairs=5000, out_dtype=None):
    """256x256x512 grid of the 50x50x300 um pixel, 512 frequencies to 50 GHz,
    400 x 10 ps, ``n_tracks`` MIP tracks of ``n_pairs`` e/h pairs each, drift
    at 1e5 m/s plus Gaussian diffusion of 0.5 um per axis per 10 ps step.

    The polylines are stepped with torch on ``device`` (see
    ``drift_paths_torch``); the returned carriers hold torch tensors there.
    """
    import torch

    rng = rng_for(5)
    cell = make_cell(50 * UM, 300 * UM, 256, 512)
    rho = rng.uniform(0.05, 1.0, size=5) * OHM_CM
    cols = standard_columns(50 * UM, 300 * UM, 5 * UM, rho[0], rho[1:], 64)
    dt = 10 * PS
    spec = dict(n_freq=512, df=frequency_grid_to_nyquist(512, dt), n_time=400, dt=dt)
    starts, charge, track = [], [], []
    for k in range(n_tracks):
        pts, q = pairs_to_carriers(mip_track_starts(rng, cell, cols, n_pairs))
        starts.append(pts)
        charge.append(q)
        track.append(np.full(q.size, k, dtype=np.int32))
    starts = np.concatenate(starts)
    charge = np.concatenate(charge)
    pos = drift_paths_torch(starts, charge, cols, cell, spec["n_time"], dt, diffusion_sigma=0.5 * UM,
                            seed=SEED_BASE + 5, device=device, out_dtype=out_dtype)
    car = dict(pos=pos, charge=torch.as_tensor(charge, device=pos.device, dtype=pos.dtype),
               track=torch.as_tensor(np.concatenate(track), device=pos.device), n_tracks=int(n_tracks))
    return dict(name="px256", cell=cell, columns=cols, spectrum=spec, carriers=car,
                note=f"{n_tracks} MIP tracks along z, {n_pairs} e/h pairs each, drift + 0.5 um diffusion per step")


def small_pixel(k=11, n_xy=24, n_z=40, n_freq=12, n_time=40, n_pairs=40,
                 n_colloc=16, to_nyquist=True, rho=None):
    """Small cell for full-grid parity: multi-tile, ragged sizes, a few carriers."""
    rng = rng_for(k)
    cell = make_cell(50 * UM, 300 * UM, n_xy, n_z)
    if rho is None:
        rho = rng.uniform(0.05, 1.0, size=5) * OHM_CM
    cols = standard_columns(50 * UM, 300 * UM, 5 * UM, rho[0], rho[1:], n_colloc)
    dt = 10 * PS
    df = frequency_grid_to_nyquist(n_freq, dt) if to_nyquist else 1.25 * GHZ
    spec = dict(n_freq=n_freq, df=df, n_time=n_time, dt=dt)
    starts = uniform_starts(rng, n_pairs, cols, cell)
    pts, q = pairs_to_carriers(starts)
    pos = drift_paths(pts, q, cols, cell, spec["n_time"], spec["dt"])
    track = (np.arange(q.size) % 3)
    return _pack(f"small-{n_xy}x{n_xy}x{n_z}-seed{k}", cell, cols, spec, pos, q, track, 3,
                 "small full-grid parity case")


CONFIGS = {"px32": uniform_pixel_32x32x64, "px128": mip_pixel_128x128x256}


def describe(cfg):
    c = cfg["cell"]
    s = cfg["spectrum"]
    return (f"{cfg['name']}: grid {c['N'][0]}x{c['N'][1]}x{c['N'][2]}, "
            f"{s['n_freq']} freq, {s['n_time']} x {s['dt'] / PS:.0f} ps, "
            f"{cfg['carriers']['pos'].shape[0]} carriers")


def cr_rc_response(n_time, dt, tau=250 * PS, gain=1.0e3):
    """Sampled impulse response (ohm/s) of a CR-RC front end: transimpedance
    `gain` (ohm, the integral of the response) and shaping time tau, sampled
    on t_n = n dt: gain * t / tau^2 * exp(-t / tau)."""
    t = np.arange(n_time) * dt
    return gain * t / tau ** 2 * np.exp(-t / tau)


def noise_samples(k, n_tracks, n_time):
    """Seeded standard normal samples for the electronics noise."""
    return rng_for(k).standard_normal((n_tracks, n_time))


def smooth_sizes(lo, hi):
    """Even 2*3*5-smooth integers in [lo, hi]."""
    out = []
    for n in range(lo + (lo & 1), hi + 1, 2):
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


def geometry_variant(k, n_pairs=1000, n_time=200):
    """One seeded geometry variant of the batched workload: pitch U(25, 100)
    um, column radius U(3, 10) um clamped to 0.2 pitch, five resistivities
    U(0.01, 1) ohm cm, N_xy an even 2*3*5-smooth size in [64, 160], N_z in
    {N_xy, 2 N_xy} up to 320, N_f in {64, 96, ..., 256} to Nyquist, 200
    samples of 10 ps, one MIP track of n_pairs e/h pairs."""
    rng = rng_for(1000 + k)
    pitch = rng.uniform(25.0, 100.0) * UM
    radius = min(rng.uniform(3.0, 10.0) * UM, 0.2 * pitch)
    rho = rng.uniform(0.01, 1.0, size=5) * OHM_CM
    n_xy = int(rng.choice(smooth_sizes(64, 160)))
    n_z = int(rng.choice([n for n in (n_xy, 2 * n_xy) if n <= 320]))
    n_freq = int(rng.choice(np.arange(64, 257, 32)))
    cell = make_cell(pitch, 300 * UM, n_xy, n_z)
    cols = standard_columns(pitch, 300 * UM, radius, rho[0], rho[1:], 64)
    dt = 10 * PS
    spec = dict(n_freq=n_freq, df=frequency_grid_to_nyquist(n_freq, dt), n_time=n_time, dt=dt)
    starts = mip_track_starts(rng, cell, cols, n_pairs)
    pts, q = pairs_to_carriers(starts)
    pos = drift_paths(pts, q, cols, cell, spec["n_time"], spec["dt"])
    return _pack(f"variant-{k}", cell, cols, spec, pos, q, np.zeros(q.size), 1,
                 f"pitch {pitch / UM:.1f} um, r {radius / UM:.2f} um, {n_pairs} e/h pairs")
