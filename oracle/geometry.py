"""Scan geometry -> rays, following the paper's transforms (FP64, numpy).

TEST INFRASTRUCTURE: only tests/, the smoke check and the benchmark's CPU-baseline
leg use this module.  It shares no code with the HIP path.

Every ray is first mapped to the paper's parallel-beam parameters and then to a line
{p + t*theta}:

* 2D parallel beam (Sec. 2.2.1, eq. direction_normal): theta = (cos phi, sin phi),
  theta_perp = (-sin phi, cos phi); the ray is t*theta + s*theta_perp.
* equiangular fan (Sec. 2.2.2, eq. 2Dparalleltofan): s = D sin(gamma),
  phi = gamma + alpha - pi/2.
* equispaced fan (eq. 2Dparalleltofan_2): s = D t / sqrt(D^2 + t^2),
  phi = arctan(t/D) + alpha - pi/2.
* 3D parallel beam (Sec. 3.2.1, eqs. 3Dparallel_direction, theta_1, theta_2):
  theta = (cos phi2 cos phi1, cos phi2 sin phi1, sin phi2),
  theta_1 = (-sin phi1, cos phi1, 0),
  theta_2 = (-sin phi2 cos phi1, -sin phi2 sin phi1, cos phi2);
  the ray is t*theta + s1*theta_1 + s2*theta_2.
* equiangular circular cone (Sec. 3.2.2, eq. equiangular_cone_beam):
  phi1 = phi1' + alpha, phi2 = beta, s1 = D sin(alpha), s2 = D cos(alpha) sin(beta).
* equispaced circular cone (eq. equispaced_cone_beam): alpha = arctan(t/D),
  beta = arctan(h / sqrt(D^2 + t^2)), s2 = h cos^2(alpha) cos(beta).
* helical cone (Sec. 3.2.3, eqs. Helical_cone_beam_equiangular/_equispaced):
  s2 gains + H cos(beta), H the source height.

Readings where the paper is silent (each listed in the design notes):
* detector bins: centre of bin c is u_c = (c - (n-1)/2) du + u0, rows likewise with +z;
* a flat detector at source-to-detector distance SDD samples the paper's virtual
  detector through the origin at t = u SOD/SDD, h = v SOD/SDD;
* components of magnitude <= 1e-12 of theta, theta_perp, theta_1 and theta_2 are
  snapped to exactly 0 (so that phi = pi/2 in floating point is the axis-parallel case
  of the paper, and a ray placed on a grid line or plane by its offsets stays on it).
"""
from __future__ import annotations

import numpy as np

SNAP = 1e-12

KINDS = ("par2d", "fan2d_flat", "fan2d_arc", "par3d", "cone_flat", "cone_arc",
         "raylist2d", "raylist3d")


# ------------------------------------------------------------------ paper transforms

def fan_equiangular(D, alpha, gamma):
    """(D, alpha, gamma) -> (s, phi), eq. 2Dparalleltofan."""
    gamma = np.asarray(gamma, dtype=np.float64)
    return D * np.sin(gamma), gamma + alpha - np.pi / 2


def fan_equispaced(D, alpha, t):
    """(D, alpha, t) -> (s, phi), eq. 2Dparalleltofan_2."""
    t = np.asarray(t, dtype=np.float64)
    return D * t / np.sqrt(D * D + t * t), np.arctan(t / D) + alpha - np.pi / 2


def cone_equiangular(D, phi1p, alpha, beta, H=0.0):
    """(D, phi1', alpha, beta[, H]) -> (s1, s2, phi1, phi2), eqs. equiangular_cone_beam
    and Helical_cone_beam_equiangular."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    phi1 = phi1p + alpha
    phi2 = beta
    s1 = D * np.sin(alpha)
    s2 = D * np.cos(alpha) * np.sin(beta) + H * np.cos(beta)
    return s1, s2, phi1, phi2


def cone_equispaced(D, phi1p, t, h, H=0.0):
    """(D, phi1', t, h[, H]) -> (s1, s2, phi1, phi2), eqs. equispaced_cone_beam and
    Helical_cone_beam_equispaced."""
    t = np.asarray(t, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    alpha = np.arctan(t / D)
    beta = np.arctan(h / np.sqrt(D * D + t * t))
    phi1 = phi1p + alpha
    phi2 = beta
    s1 = D * np.sin(alpha)
    s2 = h * np.cos(alpha) ** 2 * np.cos(beta) + H * np.cos(beta)
    return s1, s2, phi1, phi2


# ------------------------------------------------------------------ parallel params -> lines

def _snap(v, normalise=True):
    v = np.array(v, dtype=np.float64, copy=True)
    v[np.abs(v) <= SNAP] = 0.0
    if normalise:
        v /= np.linalg.norm(v, axis=-1, keepdims=True)
    return v


def par2d_lines(s, phi):
    """Lines of 2D parallel rays (s, phi): returns p [M,3], theta [M,3]."""
    s = np.atleast_1d(np.asarray(s, dtype=np.float64))
    phi = np.atleast_1d(np.asarray(phi, dtype=np.float64))
    s, phi = np.broadcast_arrays(s, phi)
    th = np.stack([np.cos(phi), np.sin(phi), np.zeros_like(phi)], axis=-1)
    perp = _snap(np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], axis=-1), False)
    p = s[..., None] * perp
    return p.reshape(-1, 3), _snap(th).reshape(-1, 3)


def par3d_lines(s1, s2, phi1, phi2):
    """Lines of 3D parallel rays (s1, s2, phi1, phi2): returns p [M,3], theta [M,3]."""
    s1, s2, phi1, phi2 = np.broadcast_arrays(*[np.atleast_1d(np.asarray(a, dtype=np.float64))
                                               for a in (s1, s2, phi1, phi2)])
    c1, si1, c2, si2 = np.cos(phi1), np.sin(phi1), np.cos(phi2), np.sin(phi2)
    th = np.stack([c2 * c1, c2 * si1, si2], axis=-1)
    th1 = _snap(np.stack([-si1, c1, np.zeros_like(c1)], axis=-1), False)
    th2 = _snap(np.stack([-si2 * c1, -si2 * si1, c2], axis=-1), False)
    p = s1[..., None] * th1 + s2[..., None] * th2
    return p.reshape(-1, 3), _snap(th).reshape(-1, 3)


# ------------------------------------------------------------------ scans

def bins(n, d, off):
    """Bin centres (c - (n-1)/2) d + off, c = 0..n-1."""
    return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * d + off


def parallel_params(scan: dict):
    """Parallel-beam parameters of every ray, in sinogram order [view][row][col].

    Returns ("2d", s, phi) or ("3d", s1, s2, phi1, phi2), flat arrays."""
    kind = scan["kind"]
    if kind == "raylist2d":
        r = np.asarray(scan["rays"], dtype=np.float64).reshape(-1, 2)
        return "2d", r[:, 0], r[:, 1]
    if kind == "raylist3d":
        r = np.asarray(scan["rays"], dtype=np.float64).reshape(-1, 4)
        return "3d", r[:, 0], r[:, 1], r[:, 2], r[:, 3]
    ang = np.asarray(scan["angles"], dtype=np.float64)
    nc = int(scan["ncols"])
    nr = int(scan.get("nrows", 1))
    u = bins(nc, scan["du"], scan.get("u0", 0.0))
    v = bins(nr, scan.get("dv", 1.0), scan.get("v0", 0.0))
    nv = ang.size
    if kind == "par2d":
        phi = np.repeat(ang, nc)
        s = np.tile(u, nv)
        return "2d", s, phi
    if kind in ("fan2d_flat", "fan2d_arc"):
        D = float(scan["sod"])
        A = np.repeat(ang, nc)
        U = np.tile(u, nv)
        if kind == "fan2d_arc":
            s, phi = fan_equiangular(D, A, U)
        else:
            s, phi = fan_equispaced(D, A, U * D / float(scan["sdd"]))
        return "2d", s, phi
    # 3D kinds: [view][row][col]
    V, R, C = np.meshgrid(np.arange(nv), np.arange(nr), np.arange(nc), indexing="ij")
    V, R, C = V.ravel(), R.ravel(), C.ravel()
    if kind == "par3d":
        phi2 = np.asarray(scan["phi2"], dtype=np.float64)
        return "3d", u[C], v[R], ang[V], phi2[V]
    D = float(scan["sod"])
    H = np.zeros(nv) if scan.get("view_z") is None else np.asarray(scan["view_z"], dtype=np.float64)
    if kind == "cone_arc":
        s1, s2, phi1, phi2 = cone_equiangular(D, ang[V], u[C], v[R], H[V])
    elif kind == "cone_flat":
        k = D / float(scan["sdd"])
        s1, s2, phi1, phi2 = cone_equispaced(D, ang[V], u[C] * k, v[R] * k, H[V])
    else:
        raise ValueError(f"unknown scan kind {kind!r}")
    return "3d", s1, s2, phi1, phi2


def expand(scan: dict):
    """Every ray of the scan as a line (p [M,3], theta [M,3]), sinogram order."""
    pp = parallel_params(scan)
    if pp[0] == "2d":
        return par2d_lines(pp[1], pp[2])
    return par3d_lines(*pp[1:])


def sino_shape(scan: dict):
    kind = scan["kind"]
    if kind.startswith("raylist"):
        w = 2 if kind == "raylist2d" else 4
        return (int(np.asarray(scan["rays"]).size // w),)
    nv = len(scan["angles"])
    if kind in ("par2d", "fan2d_flat", "fan2d_arc"):
        return (nv, int(scan["ncols"]))
    return (nv, int(scan.get("nrows", 1)), int(scan["ncols"]))
