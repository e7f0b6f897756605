"""Seeded synthetic inputs: phantoms, scan descriptions, random rays, noise.

This module holds no part of the transform's arithmetic.  It only produces input
data (numpy arrays and plain parameter dicts) that both the HIP path and the FP64
reference receive unchanged.  It imports numpy only.

Grid dict:  nx, ny, nz (0 for 2D), dx, dy, dz (unit side lengths), cx, cy, cz (centre).
Scan dict:  kind in {par2d, fan2d_flat, fan2d_arc, par3d, cone_flat, cone_arc,
            raylist2d, raylist3d}; angles (per view: phi, alpha, phi1 or phi1');
            ncols, nrows, du, dv, u0, v0 (bin centres (c-(n-1)/2)*du+u0);
            sod, sdd (divergent kinds); view_z (source height per view, helical);
            phi2 (per view, par3d); rays (raylist kinds: (s,phi) or (s1,s2,phi1,phi2)).
Image arrays are [nz][ny][nx] (or [ny][nx]) float32, row j = 0 at the top (+y).
"""
from __future__ import annotations

import numpy as np

# ------------------------------------------------------------------ phantoms


def ellipse_phantom(nx: int, ny: int, n: int, seed: int) -> np.ndarray:
    """Sum of n random ellipses sampled at pixel centres, float32 [ny][nx].

    Normalised coordinates X, Y in (-1, 1) over the image; centre uniform in the disc
    of radius 0.8, semi-axes U[0.05, 0.4], rotation U[0, pi), density U[0, 1]."""
    rng = np.random.default_rng(seed)
    X = ((np.arange(nx) + 0.5) / nx * 2.0 - 1.0)[None, :]
    Y = (1.0 - (np.arange(ny) + 0.5) / ny * 2.0)[:, None]
    img = np.zeros((ny, nx), dtype=np.float64)
    for _ in range(n):
        r = 0.8 * np.sqrt(rng.uniform())
        a = rng.uniform(0, 2 * np.pi)
        x0, y0 = r * np.cos(a), r * np.sin(a)
        ax, ay = rng.uniform(0.05, 0.4, size=2)
        rot = rng.uniform(0, np.pi)
        rho = rng.uniform(0, 1)
        c, s = np.cos(rot), np.sin(rot)
        u = (X - x0) * c + (Y - y0) * s
        v = -(X - x0) * s + (Y - y0) * c
        img += rho * ((u / ax) ** 2 + (v / ay) ** 2 <= 1.0)
    return img.astype(np.float32)


def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def ellipsoid_phantom(nx: int, ny: int, nz: int, n: int, seed: int) -> np.ndarray:
    """Sum of n random ellipsoids sampled at voxel centres, float32 [nz][ny][nx].

    Normalised coordinates in (-1, 1)^3; centre uniform in the ball of radius 0.8,
    semi-axes U[0.05, 0.4], uniformly random rotation, density U[0, 1]."""
    rng = np.random.default_rng(seed)
    params = []
    for _ in range(n):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = 0.8 * rng.uniform() ** (1.0 / 3.0) * d
        ax = rng.uniform(0.05, 0.4, size=3)
        R = _random_rotation(rng)
        rho = rng.uniform(0, 1)
        params.append((c, ax, R, rho))
    X = ((np.arange(nx) + 0.5) / nx * 2.0 - 1.0).astype(np.float32)
    Y = (1.0 - (np.arange(ny) + 0.5) / ny * 2.0).astype(np.float32)
    img = np.zeros((nz, ny, nx), dtype=np.float32)
    for k in range(nz):
        Z = np.float32(1.0 - (k + 0.5) / nz * 2.0)
        sl = np.zeros((ny, nx), dtype=np.float32)
        for c, ax, R, rho in params:
            if abs(Z - c[2]) > ax.max():
                continue
            dx = X[None, :] - np.float32(c[0])
            dy = Y[:, None] - np.float32(c[1])
            dz = Z - np.float32(c[2])
            # body-frame coordinates: R^T (r - c)
            u = R[0, 0] * dx + R[1, 0] * dy + R[2, 0] * dz
            v = R[0, 1] * dx + R[1, 1] * dy + R[2, 1] * dz
            w = R[0, 2] * dx + R[1, 2] * dy + R[2, 2] * dz
            sl += np.float32(rho) * (((u / ax[0]) ** 2 + (v / ax[1]) ** 2 + (w / ax[2]) ** 2) <= 1.0)
        img[k] = sl
    return img


def poisson_sinogram(g: np.ndarray, photons: float, seed: int, max_integral: float = 3.0):
    """Poisson-noisy version of a noiseless sinogram g (float64 result).

    The sinogram is scaled by mu so that its maximum line integral is max_integral;
    counts ~ Poisson(photons * exp(-mu g)), clamped >= 1; returns -ln(counts/photons)/mu."""
    rng = np.random.default_rng(seed)
    gmax = float(np.max(g))
    mu = max_integral / gmax if gmax > 0 else 1.0
    lam = photons * np.exp(-mu * np.asarray(g, dtype=np.float64))
    counts = np.maximum(rng.poisson(lam), 1.0)
    return -np.log(counts / photons) / mu


# ------------------------------------------------------------------ scans of the workloads


def helical_view_z(views_per_turn: int, turns: int, pitch: float, nrows: int, dv: float,
                   sod: float, sdd: float) -> np.ndarray:
    """Source heights of a helical scan: feed per turn F = pitch * nrows * dv * sod/sdd
    (the detector's height at the rotation axis); centred on z = 0, moving +z."""
    F = pitch * nrows * dv * sod / sdd
    k = np.arange(views_per_turn * turns, dtype=np.float64)
    return -(turns * F) / 2.0 + F * k / views_per_turn


WORKLOADS = ("par2d_128", "fan2d_512", "cone_256", "batched_cone_helical", "fan2d_256_sparse")


def workload(name: str) -> dict:
    """Grid, scan and phantom recipe of a named workload.  Phantoms are drawn by
    make_image(cfg); the returned dict holds only parameters.

    par2d_128: 128^2 unit pixels, 180 parallel views over [0, pi), 185 bins of 1.
    fan2d_512: 512^2 pixels of 0.8 centred at (20, -15), 720 fan views over 2 pi, flat
        detector of 1024 bins of 1.2, source-to-centre 1000, source-to-detector 1500.
    cone_256: 256^3 unit voxels, 360 circular cone views over 2 pi, flat 384 x 512
        detector of spacing 1, source-to-centre 1000, source-to-detector 1500.
    batched_cone_helical: 16 uneven cone / helical problems (batched_workload()).
    fan2d_256_sparse: 256^2 unit pixels, 60 fan views over 2 pi, 512 bins of 0.75,
        batches of 64 phantoms with Poisson noise at 1e5 photons per ray."""
    if name == "par2d_128":
        grid = dict(nx=128, ny=128, nz=0, dx=1.0, dy=1.0, cx=0.0, cy=0.0)
        scan = dict(kind="par2d", angles=np.arange(180) * np.pi / 180.0, ncols=185, du=1.0, u0=0.0)
        return dict(name="par2d_128_180x185", grid=grid, scan=scan, phantom=("ellipse", 10), seed=1)
    if name == "fan2d_512":
        grid = dict(nx=512, ny=512, nz=0, dx=0.8, dy=0.8, cx=20.0, cy=-15.0)
        scan = dict(kind="fan2d_flat", angles=np.arange(720) * 2 * np.pi / 720.0, ncols=1024, du=1.2,
                    u0=0.0, sod=1000.0, sdd=1500.0)
        return dict(name="fan2d_512_720x1024", grid=grid, scan=scan, phantom=("ellipse", 10), seed=2)
    if name == "cone_256":
        grid = dict(nx=256, ny=256, nz=256, dx=1.0, dy=1.0, dz=1.0, cx=0.0, cy=0.0, cz=0.0)
        scan = dict(kind="cone_flat", angles=np.arange(360) * 2 * np.pi / 360.0, ncols=512, nrows=384,
                    du=1.0, dv=1.0, u0=0.0, v0=0.0, sod=1000.0, sdd=1500.0)
        return dict(name="cone_256^3_360x384x512", grid=grid, scan=scan, phantom=("ellipsoid", 20), seed=3)
    if name == "fan2d_256_sparse":
        grid = dict(nx=256, ny=256, nz=0, dx=1.0, dy=1.0, cx=0.0, cy=0.0)
        scan = dict(kind="fan2d_flat", angles=np.arange(60) * 2 * np.pi / 60.0, ncols=512, du=0.75,
                    u0=0.0, sod=1000.0, sdd=1500.0)
        return dict(name="fan2d_256_60x512_learned", grid=grid, scan=scan, phantom=("ellipse", 10),
                    seed=5, batch=64, photons=1e5)
    if name == "batched_cone_helical":
        return batched_workload()
    raise ValueError(f"unknown workload {name!r} (known: {', '.join(WORKLOADS)})")


BATCH_DIMS = [(64, 64, 64), (96, 96, 96), (128, 128, 64), (128, 128, 128), (192, 192, 128),
              (256, 256, 128), (256, 256, 256), (512, 512, 256)]


def batched_workload(count: int = 16, seed: int = 4, scale: float = 1.0) -> dict:
    """Uneven batch: even members circular cone (512x384 flat detector, 360 views),
    odd members helical (pitch 1, 3 turns x 720 views, 768x64 detector).  Volume dims
    drawn from BATCH_DIMS; SOD ~ U[800, 1200], SDD/SOD ~ U[1.3, 1.7].  scale < 1
    shrinks every size (for tests)."""
    rng = np.random.default_rng(seed)
    members = []
    for m in range(count):
        nx, ny, nz = BATCH_DIMS[int(rng.integers(len(BATCH_DIMS)))]
        sod = float(rng.uniform(800, 1200))
        sdd = sod * float(rng.uniform(1.3, 1.7))
        nx, ny, nz = (max(4, int(round(v * scale))) for v in (nx, ny, nz))
        grid = dict(nx=nx, ny=ny, nz=nz, dx=1.0, dy=1.0, dz=1.0, cx=0.0, cy=0.0, cz=0.0)
        if m % 2 == 0:
            nv = max(4, int(round(360 * scale)))
            ncols, nrows = max(4, int(round(512 * scale))), max(4, int(round(384 * scale)))
            # detector sized to cover the volume's width at the given magnification
            du = max(nx, ny) * 1.5 * (sdd / sod) / ncols
            dv = nz * 1.2 * (sdd / sod) / nrows
            scan = dict(kind="cone_flat", angles=np.arange(nv) * 2 * np.pi / nv, ncols=ncols,
                        nrows=nrows, du=du, dv=dv, u0=0.0, v0=0.0, sod=sod, sdd=sdd)
        else:
            vpt = max(4, int(round(720 * scale)))
            ncols, nrows = max(4, int(round(768 * scale))), max(2, int(round(64 * scale)))
            du = max(nx, ny) * 1.5 * (sdd / sod) / ncols
            dv = 1.0 * (sdd / sod)
            turns = 3
            vz = helical_view_z(vpt, turns, 1.0, nrows, dv, sod, sdd)
            scan = dict(kind="cone_flat", angles=np.arange(vpt * turns) * 2 * np.pi / vpt,
                        ncols=ncols, nrows=nrows, du=du, dv=dv, u0=0.0, v0=0.0, sod=sod, sdd=sdd,
                        view_z=vz)
        members.append(dict(grid=grid, scan=scan, phantom=("ellipsoid", 20), seed=1000 * seed + m))
    return dict(name=f"batched_{count}_cone_helical", members=members)


def make_image(cfg: dict, seed_offset: int = 0) -> np.ndarray:
    g = cfg["grid"]
    kind, n = cfg["phantom"]
    seed = cfg["seed"] + seed_offset
    if kind == "ellipse":
        return ellipse_phantom(g["nx"], g["ny"], n, seed)
    return ellipsoid_phantom(g["nx"], g["ny"], g["nz"], n, seed)


def sino_shape(scan: dict):
    kind = scan["kind"]
    if kind.startswith("raylist"):
        w = 2 if kind == "raylist2d" else 4
        return (int(np.asarray(scan["rays"]).size // w),)
    nv = len(scan["angles"])
    if kind in ("par2d", "fan2d_flat", "fan2d_arc"):
        return (nv, int(scan["ncols"]))
    return (nv, int(scan.get("nrows", 1)), int(scan["ncols"]))


def image_shape(grid: dict):
    nz = int(grid.get("nz", 0))
    return (int(grid["ny"]), int(grid["nx"])) if nz == 0 else (nz, int(grid["ny"]), int(grid["nx"]))


# ------------------------------------------------------------------ random rays for tests


def random_rays2d(m: int, smax: float, seed: int) -> np.ndarray:
    """m random 2D parallel-beam rays (s, phi): s ~ U[-smax, smax], phi ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-smax, smax, m), rng.uniform(0, 2 * np.pi, m)], axis=1)


def random_rays3d(m: int, smax: float, seed: int) -> np.ndarray:
    """m random 3D rays (s1, s2, phi1, phi2): s ~ U[-smax, smax], phi1 ~ U[0, 2 pi),
    phi2 ~ U[-pi/2, pi/2]."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-smax, smax, m), rng.uniform(-smax, smax, m),
                     rng.uniform(0, 2 * np.pi, m), rng.uniform(-np.pi / 2, np.pi / 2, m)], axis=1)


def random_image(shape, seed: int, positive: bool = True) -> np.ndarray:
    rng = np.random.default_rng(seed)
    a = rng.uniform(0, 1, size=shape) if positive else rng.normal(size=shape)
    return a.astype(np.float32)
