"""ctypes front end of the FP64 C reference (xrt_oracle.c) -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may use it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import geometry

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xrt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C reference with gcc (portable flags: the library may run on a
    different host CPU than the one it was built on)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("cz", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        gp = ctypes.POINTER(_Grid)
        lib.ora_forward.argtypes = [gp, ctypes.c_long, dp, dp, dp, dp, ctypes.c_int]
        lib.ora_adjoint.argtypes = [gp, ctypes.c_long, dp, dp, dp, dp, ctypes.c_int]
        lib.ora_ray_hits.argtypes = [gp, dp, dp, lp, dp, ctypes.c_long, ctypes.c_double]
        lib.ora_ray_hits.restype = ctypes.c_long
        lib.ora_hit_counts.argtypes = [gp, ctypes.c_long, dp, dp, ctypes.c_double, lp, ctypes.c_int]
        lib.ora_forward_att.argtypes = [gp, ctypes.c_long, dp, dp, dp, dp, dp, ctypes.c_int]
        lib.ora_adjoint_att.argtypes = [gp, ctypes.c_long, dp, dp, dp, dp, dp, ctypes.c_int]
        lib.ora_forward_simplex.argtypes = [gp, ctypes.c_long, dp, dp, dp, dp, ctypes.c_int]
        lib.ora_adjoint_simplex.argtypes = [gp, ctypes.c_long, dp, dp, dp, dp, ctypes.c_int]
        lib.ora_ray_hits_simplex.argtypes = [gp, dp, dp, lp, dp, ctypes.c_long, ctypes.c_double]
        lib.ora_ray_hits_simplex.restype = ctypes.c_long
        lib.ora_chord.argtypes = [gp, dp, dp]
        lib.ora_chord.restype = ctypes.c_double
        _lib = lib
    return _lib


def _grid(g: dict) -> _Grid:
    nz = int(g.get("nz", 0))
    return _Grid(int(g["nx"]), int(g["ny"]), nz,
                 float(g.get("dx", 1.0)), float(g.get("dy", 1.0)), float(g.get("dz", 1.0)),
                 float(g.get("cx", 0.0)), float(g.get("cy", 0.0)), float(g.get("cz", 0.0)))


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def image_shape(g: dict):
    nz = int(g.get("nz", 0))
    return (int(g["ny"]), int(g["nx"])) if nz == 0 else (nz, int(g["ny"]), int(g["nx"]))


def default_threads() -> int:
    """Threads the oracle uses: the cores this process may run on, capped by
    OMP_NUM_THREADS when that is set (a host shared between jobs sets each one's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def host_info() -> dict:
    """The host the oracle runs on: logical CPUs, the ones this process may use, the
    OpenMP thread setting and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = None
    return {"cpu_count": os.cpu_count(), "affinity": aff, "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "cpu_model": model}


def forward_lines(g: dict, p, th, img, nthreads=None):
    lib = _load()
    p, th = _c(p).reshape(-1, 3), _c(th).reshape(-1, 3)
    img = _c(img)
    out = np.zeros(p.shape[0], dtype=np.float64)
    gg = _grid(g)
    lib.ora_forward(ctypes.byref(gg), p.shape[0], _dptr(p), _dptr(th), _dptr(img), _dptr(out),
                    nthreads or default_threads())
    return out


def adjoint_lines(g: dict, p, th, sino, nthreads=None):
    lib = _load()
    p, th = _c(p).reshape(-1, 3), _c(th).reshape(-1, 3)
    sino = _c(sino).ravel()
    img = np.zeros(int(np.prod(image_shape(g))), dtype=np.float64)
    gg = _grid(g)
    lib.ora_adjoint(ctypes.byref(gg), p.shape[0], _dptr(p), _dptr(th), _dptr(sino), _dptr(img),
                    nthreads or default_threads())
    return img.reshape(image_shape(g))


def forward_att_lines(g: dict, p, th, img, mu, nthreads=None):
    """Attenuated transform (Introduction, eq. generalizedRadontransform, SPECT case)."""
    lib = _load()
    p, th = _c(p).reshape(-1, 3), _c(th).reshape(-1, 3)
    img, mu = _c(img), _c(mu)
    out = np.zeros(p.shape[0], dtype=np.float64)
    gg = _grid(g)
    lib.ora_forward_att(ctypes.byref(gg), p.shape[0], _dptr(p), _dptr(th), _dptr(img), _dptr(mu), _dptr(out),
                        nthreads or default_threads())
    return out


def adjoint_att_lines(g: dict, p, th, sino, mu, nthreads=None):
    lib = _load()
    p, th = _c(p).reshape(-1, 3), _c(th).reshape(-1, 3)
    sino, mu = _c(sino).ravel(), _c(mu)
    img = np.zeros(int(np.prod(image_shape(g))), dtype=np.float64)
    gg = _grid(g)
    lib.ora_adjoint_att(ctypes.byref(gg), p.shape[0], _dptr(p), _dptr(th), _dptr(sino), _dptr(mu), _dptr(img),
                        nthreads or default_threads())
    return img.reshape(image_shape(g))


def forward_weighted_lines(g: dict, p, th, img, w, nthreads=None):
    """PET form of the generalised transform (Introduction, eq. generalizedRadontransform
    with a weight that does not depend on t): the weight of each ray times its X-ray
    transform.  w: one weight per line."""
    return np.asarray(w, dtype=np.float64).ravel() * forward_lines(g, p, th, img, nthreads)


def adjoint_weighted_lines(g: dict, p, th, sino, w, nthreads=None):
    """Transpose of forward_weighted_lines: the plain adjoint of w * sino."""
    ws = np.asarray(w, dtype=np.float64).ravel() * np.asarray(sino, dtype=np.float64).ravel()
    return adjoint_lines(g, p, th, ws, nthreads)


def transmission_lines(g: dict, p, th, mu, nthreads=None):
    """exp(-integral of mu along each line): the PET attenuation weight of the map mu."""
    return np.exp(-forward_lines(g, p, th, mu, nthreads))


def ray_hits_line(g: dict, p, th, eps=0.0):
    """(indices, lengths) of one ray, sorted by 1D index; lengths > eps."""
    lib = _load()
    p, th = _c(p).ravel(), _c(th).ravel()
    cap = int(g["nx"]) + int(g["ny"]) + int(g.get("nz", 0)) + 8
    idx = np.zeros(cap, dtype=np.int64)
    ln = np.zeros(cap, dtype=np.float64)
    gg = _grid(g)
    n = lib.ora_ray_hits(ctypes.byref(gg), _dptr(p), _dptr(th),
                         idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dptr(ln), cap, eps)
    n = min(n, cap)
    return idx[:n].copy(), ln[:n].copy()


def hit_counts_lines(g: dict, p, th, eps=0.0, nthreads=None):
    lib = _load()
    p, th = _c(p).reshape(-1, 3), _c(th).reshape(-1, 3)
    out = np.zeros(p.shape[0], dtype=np.int64)
    gg = _grid(g)
    lib.ora_hit_counts(ctypes.byref(gg), p.shape[0], _dptr(p), _dptr(th), eps,
                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                       nthreads or default_threads())
    return out


def chord_line(g: dict, p, th):
    lib = _load()
    p, th = _c(p).ravel(), _c(th).ravel()
    gg = _grid(g)
    return lib.ora_chord(ctypes.byref(gg), _dptr(p), _dptr(th))


# ------------------------------------------------------------------ scan-level helpers

def forward(g: dict, scan: dict, img, nthreads=None):
    """Sinogram of img for the scan (FP64), shaped like the scan's sinogram."""
    p, th = geometry.expand(scan)
    return forward_lines(g, p, th, img, nthreads).reshape(geometry.sino_shape(scan))


def forward_att(g: dict, scan: dict, img, mu, nthreads=None):
    p, th = geometry.expand(scan)
    return forward_att_lines(g, p, th, img, mu, nthreads).reshape(geometry.sino_shape(scan))


def adjoint_att(g: dict, scan: dict, sino, mu, nthreads=None):
    p, th = geometry.expand(scan)
    return adjoint_att_lines(g, p, th, sino, mu, nthreads)


def forward_weighted(g: dict, scan: dict, img, w, nthreads=None):
    p, th = geometry.expand(scan)
    return forward_weighted_lines(g, p, th, img, w, nthreads).reshape(geometry.sino_shape(scan))


def adjoint_weighted(g: dict, scan: dict, sino, w, nthreads=None):
    p, th = geometry.expand(scan)
    return adjoint_weighted_lines(g, p, th, sino, w, nthreads)


def transmission(g: dict, scan: dict, mu, nthreads=None):
    p, th = geometry.expand(scan)
    return transmission_lines(g, p, th, mu, nthreads).reshape(geometry.sino_shape(scan))


def adjoint(g: dict, scan: dict, sino, nthreads=None):
    p, th = geometry.expand(scan)
    return adjoint_lines(g, p, th, sino, nthreads)


def hit_counts(g: dict, scan: dict, eps=0.0, nthreads=None):
    p, th = geometry.expand(scan)
    return hit_counts_lines(g, p, th, eps, nthreads).reshape(geometry.sino_shape(scan))


# ------------------------------------------------------------------ simplex basis

def simplex_count(g: dict) -> int:
    """Simplices per unit: 2 triangles per pixel, 6 tetrahedra per voxel."""
    return 6 if int(g.get("nz", 0)) > 0 else 2


def simplex_image_shape(g: dict):
    return tuple(image_shape(g)) + (simplex_count(g),)


def forward_simplex_lines(g: dict, p, th, img, nthreads=None):
    """X-ray transform of an image on the simplices of the structured triangulation
    (every pixel cut into 2 triangles, every voxel into 6 tetrahedra; the definition is
    in xrt_oracle.c): out[r] = sum_T img[T] len(r, T)."""
    lib = _load()
    p, th = _c(p).reshape(-1, 3), _c(th).reshape(-1, 3)
    img = _c(img)
    out = np.zeros(p.shape[0], dtype=np.float64)
    gg = _grid(g)
    lib.ora_forward_simplex(ctypes.byref(gg), p.shape[0], _dptr(p), _dptr(th), _dptr(img), _dptr(out),
                            nthreads or default_threads())
    return out


def adjoint_simplex_lines(g: dict, p, th, sino, nthreads=None):
    lib = _load()
    p, th = _c(p).reshape(-1, 3), _c(th).reshape(-1, 3)
    sino = _c(sino).ravel()
    img = np.zeros(int(np.prod(simplex_image_shape(g))), dtype=np.float64)
    gg = _grid(g)
    lib.ora_adjoint_simplex(ctypes.byref(gg), p.shape[0], _dptr(p), _dptr(th), _dptr(sino), _dptr(img),
                            nthreads or default_threads())
    return img.reshape(simplex_image_shape(g))


def ray_hits_simplex_line(g: dict, p, th, eps=0.0):
    """(simplex indices, lengths) of one ray, sorted by index; lengths > eps."""
    lib = _load()
    p, th = _c(p).ravel(), _c(th).ravel()
    cap = 3 * (int(g["nx"]) + int(g["ny"]) + int(g.get("nz", 0))) + 16
    idx = np.zeros(cap, dtype=np.int64)
    ln = np.zeros(cap, dtype=np.float64)
    gg = _grid(g)
    n = lib.ora_ray_hits_simplex(ctypes.byref(gg), _dptr(p), _dptr(th),
                                 idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dptr(ln), cap, eps)
    n = min(n, cap)
    return idx[:n].copy(), ln[:n].copy()
