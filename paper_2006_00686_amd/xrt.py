"""ctypes binding of libxrt.so (include/xrt.h).  Argument marshalling only: every step
of the transform runs in the library's HIP kernels.  torch provides device memory and
the stream.  The library must be built (python -m paper_2006_00686_amd.build); there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxrt.so")

KIND = {"par2d": 1, "fan2d_flat": 2, "fan2d_arc": 3, "par3d": 4, "cone_flat": 5, "cone_arc": 6,
        "raylist2d": 7, "raylist3d": 8}
ADJ = {"auto": 0, "scatter": 1, "gather": 2}


class XrtError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_lib().xrt_status_str(status).decode()} -- "
                         f"{_lib().xrt_last_error().decode()}")


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("cz", ctypes.c_double)]


_dp = ctypes.POINTER(ctypes.c_double)


class Scan(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_views", ctypes.c_int32), ("n_rows", ctypes.c_int32),
                ("n_cols", ctypes.c_int32), ("du", ctypes.c_double), ("dv", ctypes.c_double),
                ("u0", ctypes.c_double), ("v0", ctypes.c_double), ("sod", ctypes.c_double),
                ("sdd", ctypes.c_double), ("view_angle", _dp), ("view_z", _dp), ("view_phi2", _dp),
                ("ray_params", _dp), ("n_rays", ctypes.c_int64)]


class AdjointInfo(ctypes.Structure):
    _fields_ = [("algorithm", ctypes.c_int32), ("voxels_per_lane", ctypes.c_int32), ("row_bound", ctypes.c_int32),
                ("column_slots", ctypes.c_int32), ("helical", ctypes.c_int32), ("zero_row", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("packet_cols", ctypes.c_int32), ("xcd_remap", ctypes.c_int32)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2006_00686_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.xrt_plan_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Scan), ctypes.c_int, ctypes.POINTER(vp)]
        lib.xrt_plan_destroy.argtypes = [vp]
        lib.xrt_plan_sizes.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        lib.xrt_forward.argtypes = [vp, vp, vp, i32, vp]
        lib.xrt_adjoint.argtypes = [vp, vp, vp, i32, i32, vp]
        lib.xrt_ray_hit_counts.argtypes = [vp, i64, i64, ctypes.c_double, vp, vp]
        lib.xrt_ray_hits.argtypes = [vp, i64, i64, ctypes.c_double, vp, vp, vp, vp]
        lib.xrt_status_str.argtypes = [i32]
        lib.xrt_status_str.restype = ctypes.c_char_p
        lib.xrt_last_error.restype = ctypes.c_char_p
        lib.xrt_vec_dot.argtypes = [i64, i32, vp, vp, vp, vp, vp]
        lib.xrt_vec_dot_noalloc.argtypes = [i64, i32, vp, vp, vp, vp]
        lib.xrt_vec_axpy_ratio.argtypes = [i64, i32, vp, vp, ctypes.c_double, vp, vp, vp]
        lib.xrt_vec_xpby_ratio.argtypes = [i64, i32, vp, vp, vp, vp, vp]
        lib.xrt_vec_axpby.argtypes = [i64, ctypes.c_double, vp, ctypes.c_double, vp, vp]
        lib.xrt_conv3x3.argtypes = [i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, i32, vp]
        lib.xrt_conv3x3_wgrad_workspace.argtypes = [i32, i32]
        lib.xrt_conv3x3_wgrad_workspace.restype = i64
        lib.xrt_conv3x3_wgrad.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp, i64, vp, vp]
        lib.xrt_precond_apply.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]
        lib.xrt_plan_adjoint_info.argtypes = [vp, ctypes.POINTER(AdjointInfo)]
        lib.xrt_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        lib.xrt_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        lib.xrt_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
        lib.xrt_batch_destroy.argtypes = [vp]
        lib.xrt_batch_forward.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        lib.xrt_batch_adjoint.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp]
        lib.xrt_forward_attenuated.argtypes = [vp, vp, vp, i32, vp, i32, vp]
        lib.xrt_adjoint_attenuated.argtypes = [vp, vp, vp, i32, vp, i32, vp]
        lib.xrt_forward_simplex.argtypes = [vp, vp, vp, i32, vp]
        lib.xrt_adjoint_simplex.argtypes = [vp, vp, vp, i32, vp]
        lib.xrt_forward_weighted.argtypes = [vp, vp, vp, i32, vp, i32, vp]
        lib.xrt_adjoint_weighted.argtypes = [vp, vp, vp, i32, vp, i32, i32, vp]
        lib.xrt_ray_transmission.argtypes = [vp, vp, vp, i32, vp]
        lib.xrt_forward_interleaved.argtypes = [vp, vp, vp, i32, vp]
        lib.xrt_adjoint_interleaved.argtypes = [vp, vp, vp, i32, vp]
        lib.xrt_scan_workspace.argtypes = [i64]
        lib.xrt_scan_workspace.restype = i64
        lib.xrt_offsets_from_counts.argtypes = [i64, vp, vp, vp, vp]
        lib.xrt_csr_transpose_workspace.argtypes = [i64]
        lib.xrt_csr_transpose_workspace.restype = i64
        lib.xrt_csr_transpose.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp, vp, vp, i64, vp]
        lib.xrt_csr_spmv.argtypes = [i64, i64, vp, vp, vp, i32, vp, vp, vp]
        lib.xrt_interleave.argtypes = [i64, i32, i32, vp, vp, vp]
        lib.xrt_csr_spmv_interleaved.argtypes = [i64, i64, vp, vp, vp, i32, vp, vp, vp]
        for f in ("xrt_plan_create", "xrt_plan_destroy", "xrt_plan_sizes", "xrt_forward", "xrt_adjoint",
                  "xrt_ray_hit_counts", "xrt_ray_hits", "xrt_vec_dot", "xrt_vec_axpy_ratio",
                  "xrt_vec_xpby_ratio", "xrt_vec_axpby", "xrt_conv3x3", "xrt_conv3x3_wgrad"):
            getattr(lib, f).restype = ctypes.c_int32
        _LIB = lib
    return _LIB


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _lib()


def _check(st: int, where: str):
    if st != 0:
        raise XrtError(st, where)


def _arr(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    return a, a.ctypes.data_as(_dp)


def _stream(device: int):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Geometry plan: a grid dict and a scan dict (see paper_2006_00686_amd.inputs)."""

    def __init__(self, grid: dict, scan: dict, device: int = 0):
        lib = _lib()
        self.grid = dict(grid)
        self.scan = dict(scan)
        self.device = int(device)
        nz = int(grid.get("nz", 0))
        g = Grid(int(grid["nx"]), int(grid["ny"]), nz, float(grid.get("dx", 1.0)), float(grid.get("dy", 1.0)),
                 float(grid.get("dz", 1.0)), float(grid.get("cx", 0.0)), float(grid.get("cy", 0.0)),
                 float(grid.get("cz", 0.0)))
        kind = scan["kind"]
        s = Scan()
        s.kind = KIND[kind]
        keep = []
        if kind.startswith("raylist"):
            w = 2 if kind == "raylist2d" else 4
            a, p = _arr(scan["rays"])
            keep.append(a)
            s.ray_params = p
            s.n_rays = a.size // w
            self.sino_shape = (int(s.n_rays),)
        else:
            ang, pa = _arr(scan["angles"])
            keep.append(ang)
            s.n_views = ang.size
            s.n_cols = int(scan["ncols"])
            s.n_rows = int(scan.get("nrows", 1))
            s.du = float(scan["du"])
            s.dv = float(scan.get("dv", 1.0))
            s.u0 = float(scan.get("u0", 0.0))
            s.v0 = float(scan.get("v0", 0.0))
            s.sod = float(scan.get("sod", 0.0))
            s.sdd = float(scan.get("sdd", 0.0))
            s.view_angle = pa
            if scan.get("view_z") is not None:
                z, pz = _arr(scan["view_z"])
                keep.append(z)
                s.view_z = pz
            if scan.get("phi2") is not None:
                q, pq = _arr(scan["phi2"])
                keep.append(q)
                s.view_phi2 = pq
            if kind in ("par2d", "fan2d_flat", "fan2d_arc"):
                self.sino_shape = (s.n_views, s.n_cols)
            else:
                self.sino_shape = (s.n_views, s.n_rows, s.n_cols)
        self.image_shape = (int(grid["ny"]), int(grid["nx"])) if nz == 0 else (nz, int(grid["ny"]), int(grid["nx"]))
        # images on the simplex basis: 2 triangles per pixel, 6 tetrahedra per voxel
        self.simplex_image_shape = tuple(self.image_shape) + (2 if nz == 0 else 6,)
        h = ctypes.c_void_p()
        _check(lib.xrt_plan_create(ctypes.byref(g), ctypes.byref(s), self.device, ctypes.byref(h)),
               "xrt_plan_create")
        self._h = h
        nr, nu = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.xrt_plan_sizes(h, ctypes.byref(nr), ctypes.byref(nu)), "xrt_plan_sizes")
        self.n_rays, self.n_units = nr.value, nu.value
        # the launch shape the plan was created with
        self.default_tuning = self.tuning()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().xrt_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -------------------------------------------------------------- launch shape

    def set_tuning(self, packet_cols: int = 0, xcd_remap: int = 0):
        """Forward launch shape (see xrt_tuning); results do not depend on it."""
        t = Tuning(int(packet_cols), int(xcd_remap))
        _check(_lib().xrt_plan_set_tuning(self._h, ctypes.byref(t)), "xrt_plan_set_tuning")

    def tuning(self) -> dict:
        t = Tuning()
        _check(_lib().xrt_plan_get_tuning(self._h, ctypes.byref(t)), "xrt_plan_get_tuning")
        return {"packet_cols": t.packet_cols, "xcd_remap": t.xcd_remap}

    # -------------------------------------------------------------- operators

    def _batch(self, t: torch.Tensor, inner):
        n = len(inner)
        if tuple(t.shape[-n:]) != tuple(inner):
            raise ValueError(f"expected trailing shape {inner}, got {tuple(t.shape)}")
        lead = tuple(t.shape[:-n])
        return lead, int(np.prod(lead)) if lead else 1

    def _dev_check(self, t: torch.Tensor):
        if t.device.type != "cuda" or t.device.index != self.device:
            raise ValueError(f"tensor must live on cuda:{self.device}")
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("tensor must be contiguous float32")

    def forward(self, img: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._dev_check(img)
        lead, b = self._batch(img, self.image_shape)
        if out is None:
            out = torch.empty(lead + tuple(self.sino_shape), dtype=torch.float32, device=img.device)
        self._dev_check(out)
        _check(_lib().xrt_forward(self._h, _ptr(img), _ptr(out), b, _stream(self.device)), "xrt_forward")
        return out

    def adjoint(self, sino: torch.Tensor, mode: str = "auto", out: torch.Tensor | None = None) -> torch.Tensor:
        self._dev_check(sino)
        lead, b = self._batch(sino, self.sino_shape)
        if out is None:
            out = torch.empty(lead + tuple(self.image_shape), dtype=torch.float32, device=sino.device)
        self._dev_check(out)
        _check(_lib().xrt_adjoint(self._h, _ptr(sino), _ptr(out), b, ADJ[mode], _stream(self.device)),
               "xrt_adjoint")
        return out

    def forward_simplex(self, img: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Transform of an image on the simplex basis ([..., *simplex_image_shape])."""
        self._dev_check(img)
        lead, b = self._batch(img, self.simplex_image_shape)
        if out is None:
            out = torch.empty(lead + tuple(self.sino_shape), dtype=torch.float32, device=img.device)
        self._dev_check(out)
        _check(_lib().xrt_forward_simplex(self._h, _ptr(img), _ptr(out), b, _stream(self.device)),
               "xrt_forward_simplex")
        return out

    def adjoint_simplex(self, sino: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._dev_check(sino)
        lead, b = self._batch(sino, self.sino_shape)
        if out is None:
            out = torch.empty(lead + tuple(self.simplex_image_shape), dtype=torch.float32, device=sino.device)
        self._dev_check(out)
        _check(_lib().xrt_adjoint_simplex(self._h, _ptr(sino), _ptr(out), b, _stream(self.device)),
               "xrt_adjoint_simplex")
        return out

    def _mu(self, mu: torch.Tensor, b: int) -> int:
        self._dev_check(mu)
        lead, mb = self._batch(mu, self.image_shape)
        if mb not in (1, b):
            raise ValueError("mu must hold one attenuation map or one per image")
        return int(mb == b and b > 1)

    def forward_attenuated(self, img: torch.Tensor, mu: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Attenuated transform of img with attenuation map(s) mu (see xrt_forward_attenuated)."""
        self._dev_check(img)
        lead, b = self._batch(img, self.image_shape)
        per = self._mu(mu, b)
        if out is None:
            out = torch.empty(lead + tuple(self.sino_shape), dtype=torch.float32, device=img.device)
        self._dev_check(out)
        _check(_lib().xrt_forward_attenuated(self._h, _ptr(img), _ptr(mu), per, _ptr(out), b, _stream(self.device)),
               "xrt_forward_attenuated")
        return out

    def adjoint_attenuated(self, sino: torch.Tensor, mu: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._dev_check(sino)
        lead, b = self._batch(sino, self.sino_shape)
        per = self._mu(mu, b)
        if out is None:
            out = torch.empty(lead + tuple(self.image_shape), dtype=torch.float32, device=sino.device)
        self._dev_check(out)
        _check(_lib().xrt_adjoint_attenuated(self._h, _ptr(sino), _ptr(mu), per, _ptr(out), b, _stream(self.device)),
               "xrt_adjoint_attenuated")
        return out

    def _weights(self, w: torch.Tensor, b: int) -> int:
        """1 when w holds one set of per-ray weights per image, 0 for one shared set."""
        self._dev_check(w)
        n = w.numel() // self.n_rays if self.n_rays else 0
        if w.numel() != n * self.n_rays or n not in (1, b):
            raise ValueError("w must hold one weight per ray, shared or one set per image")
        return int(n == b and b > 1)

    def forward_weighted(self, img: torch.Tensor, w: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """w * (A img): the PET form of the generalised transform (see xrt_forward_weighted)."""
        self._dev_check(img)
        lead, b = self._batch(img, self.image_shape)
        per = self._weights(w, b)
        if out is None:
            out = torch.empty(lead + tuple(self.sino_shape), dtype=torch.float32, device=img.device)
        self._dev_check(out)
        _check(_lib().xrt_forward_weighted(self._h, _ptr(img), _ptr(w), per, _ptr(out), b, _stream(self.device)),
               "xrt_forward_weighted")
        return out

    def adjoint_weighted(self, sino: torch.Tensor, w: torch.Tensor, mode: str = "auto",
                         out: torch.Tensor | None = None) -> torch.Tensor:
        """A^T (w * sino) (see xrt_adjoint_weighted)."""
        self._dev_check(sino)
        lead, b = self._batch(sino, self.sino_shape)
        per = self._weights(w, b)
        if out is None:
            out = torch.empty(lead + tuple(self.image_shape), dtype=torch.float32, device=sino.device)
        self._dev_check(out)
        _check(_lib().xrt_adjoint_weighted(self._h, _ptr(sino), _ptr(w), per, _ptr(out), b, ADJ[mode],
                                           _stream(self.device)), "xrt_adjoint_weighted")
        return out

    def forward_interleaved(self, img: torch.Tensor, batch: int, out: torch.Tensor | None = None) -> torch.Tensor:
        """Forward of `batch` (1..64) images held interleaved, img (n_units, batch) ->
        (n_rays, batch) (see xrt_forward_interleaved)."""
        self._dev_check(img)
        if img.numel() != self.n_units * batch:
            raise ValueError("img must hold n_units x batch floats")
        if out is None:
            out = torch.empty((self.n_rays, batch), dtype=torch.float32, device=img.device)
        self._dev_check(out)
        if out.numel() != self.n_rays * batch:
            raise ValueError("out must hold n_rays x batch floats")
        _check(_lib().xrt_forward_interleaved(self._h, _ptr(img), _ptr(out), batch, _stream(self.device)),
               "xrt_forward_interleaved")
        return out

    def adjoint_interleaved(self, sino: torch.Tensor, batch: int, out: torch.Tensor | None = None) -> torch.Tensor:
        """Gather adjoint of `batch` (1..64) sinograms held interleaved, sino (n_rays, batch)
        -> (n_units, batch); 2D plans with the voxel-driven gather."""
        self._dev_check(sino)
        if sino.numel() != self.n_rays * batch:
            raise ValueError("sino must hold n_rays x batch floats")
        if out is None:
            out = torch.empty((self.n_units, batch), dtype=torch.float32, device=sino.device)
        self._dev_check(out)
        if out.numel() != self.n_units * batch:
            raise ValueError("out must hold n_units x batch floats")
        _check(_lib().xrt_adjoint_interleaved(self._h, _ptr(sino), _ptr(out), batch, _stream(self.device)),
               "xrt_adjoint_interleaved")
        return out

    def ray_transmission(self, mu: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """exp(-(A mu)) per ray: the PET attenuation weights of map(s) mu."""
        self._dev_check(mu)
        lead, b = self._batch(mu, self.image_shape)
        if out is None:
            out = torch.empty(lead + tuple(self.sino_shape), dtype=torch.float32, device=mu.device)
        self._dev_check(out)
        _check(_lib().xrt_ray_transmission(self._h, _ptr(mu), _ptr(out), b, _stream(self.device)),
               "xrt_ray_transmission")
        return out

    def adjoint_info(self) -> dict:
        """The adjoint AUTO runs and the cone gather's kernel variant (xrt_plan_adjoint_info)."""
        info = AdjointInfo()
        _check(_lib().xrt_plan_adjoint_info(self._h, ctypes.byref(info)), "xrt_plan_adjoint_info")
        out = {f: getattr(info, f) for f, _ in AdjointInfo._fields_}
        out["algorithm"] = {1: "scatter", 2: "gather"}[out["algorithm"]]
        return out

    def hit_counts(self, first: int = 0, n: int | None = None, eps: float = 0.0) -> torch.Tensor:
        n = self.n_rays - first if n is None else n
        out = torch.empty(n, dtype=torch.int32, device=f"cuda:{self.device}")
        _check(_lib().xrt_ray_hit_counts(self._h, first, n, eps, _ptr(out), _stream(self.device)),
               "xrt_ray_hit_counts")
        return out

    def hits(self, first: int = 0, n: int | None = None, eps: float = 0.0):
        """(offsets[n+1], idx, len) CSR of rays [first, first+n), rows sorted by 1D index."""
        counts = self.hit_counts(first, n, eps)
        n = counts.numel()
        offs = offsets_from_counts(counts)
        total = int(offs[-1].item())
        idx = torch.empty(max(total, 1), dtype=torch.int32, device=counts.device)
        ln = torch.empty(max(total, 1), dtype=torch.float32, device=counts.device)
        _check(_lib().xrt_ray_hits(self._h, first, n, eps, _ptr(offs), _ptr(idx), _ptr(ln), _stream(self.device)),
               "xrt_ray_hits")
        return offs, idx[:total], ln[:total]


class Batch:
    """Several plans projected together: the forward of all members is one persistent
    launch (longest rays first); no allocation or synchronisation happens in forward /
    adjoint, so both can be captured in a graph.  Keeps references to its plans."""

    def __init__(self, plans: list):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(_lib().xrt_batch_create(arr, len(self.plans), ctypes.byref(h)), "xrt_batch_create")
        self._h = h
        self.device = self.plans[0].device

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().xrt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, ts, shapes):
        if len(ts) != len(self.plans):
            raise ValueError(f"expected {len(self.plans)} tensors, got {len(ts)}")
        for t, shp, p in zip(ts, shapes, self.plans):
            p._dev_check(t)
            if tuple(t.shape) != tuple(shp):
                raise ValueError(f"expected shape {tuple(shp)}, got {tuple(t.shape)}")
        return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def forward(self, imgs: list, out: list | None = None) -> list:
        if out is None:
            out = [torch.empty(tuple(p.sino_shape), dtype=torch.float32, device=f"cuda:{p.device}")
                   for p in self.plans]
        a = self._ptrs(imgs, [p.image_shape for p in self.plans])
        b = self._ptrs(out, [p.sino_shape for p in self.plans])
        _check(_lib().xrt_batch_forward(self._h, a, b, _stream(self.device)), "xrt_batch_forward")
        return out

    def adjoint(self, sinos: list, mode: str = "auto", out: list | None = None) -> list:
        if out is None:
            out = [torch.empty(tuple(p.image_shape), dtype=torch.float32, device=f"cuda:{p.device}")
                   for p in self.plans]
        a = self._ptrs(sinos, [p.sino_shape for p in self.plans])
        b = self._ptrs(out, [p.image_shape for p in self.plans])
        _check(_lib().xrt_batch_adjoint(self._h, a, b, ADJ[mode], _stream(self.device)), "xrt_batch_adjoint")
        return out


# ------------------------------------------------------------------ batched vector kernels


def _vec_args(t: torch.Tensor, batch: int):
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("vectors must be contiguous float32 on the GPU")
    return t.numel() // batch


def vec_dot(a: torch.Tensor, b: torch.Tensor, batch: int, work: torch.Tensor, out: torch.Tensor):
    """out[b] = <a[b], b[b]> in FP64 (out: float64 [batch]; work: float64 >= 64*batch)."""
    n = _vec_args(a, batch)
    _check(_lib().xrt_vec_dot(n, batch, _ptr(a), _ptr(b), _ptr(work), _ptr(out), _stream(a.device.index)),
           "xrt_vec_dot")
    return out


def vec_dot_noalloc(a: torch.Tensor, b: torch.Tensor, batch: int, out: torch.Tensor):
    """out[k] = <a[k], b[k]> (FP64) like vec_dot, with the library's static scratch instead of
    a workspace (no allocation)."""
    n = _vec_args(a, batch)
    if (_vec_args(b, batch) != n or a.numel() != n * batch or b.numel() != n * batch
            or out.dtype != torch.float64 or not out.is_contiguous() or out.numel() < batch):
        raise ValueError("vec_dot_noalloc: shape or dtype mismatch")
    _check(_lib().xrt_vec_dot_noalloc(n, batch, _ptr(a), _ptr(b), _ptr(out), _stream(a.device.index)),
           "xrt_vec_dot_noalloc")
    return out


def vec_axpy_ratio(num: torch.Tensor, den: torch.Tensor, sign: float, x: torch.Tensor, y: torch.Tensor, batch: int):
    """y[b] += sign * num[b]/den[b] * x[b]."""
    n = _vec_args(x, batch)
    _check(_lib().xrt_vec_axpy_ratio(n, batch, _ptr(num), _ptr(den), float(sign), _ptr(x), _ptr(y),
                                     _stream(x.device.index)), "xrt_vec_axpy_ratio")


def vec_xpby_ratio(num: torch.Tensor, den: torch.Tensor, s: torch.Tensor, p: torch.Tensor, batch: int):
    """p[b] = s[b] + num[b]/den[b] * p[b]."""
    n = _vec_args(s, batch)
    _check(_lib().xrt_vec_xpby_ratio(n, batch, _ptr(num), _ptr(den), _ptr(s), _ptr(p), _stream(s.device.index)),
           "xrt_vec_xpby_ratio")


def vec_axpby(a: float, x: torch.Tensor, b: float, y: torch.Tensor):
    """y = a x + b y."""
    n = _vec_args(x, 1)
    _check(_lib().xrt_vec_axpby(n, float(a), _ptr(x), float(b), _ptr(y), _stream(x.device.index)), "xrt_vec_axpby")


# ------------------------------------------------------------------ CNN convolutions


def _conv_in_check(t: torch.Tensor, ch: int, B: int, H: int, W: int):
    want = (B, H, W) if ch == 1 else (B, H, W, 32)
    dt = torch.float32 if ch == 1 else torch.bfloat16
    if tuple(t.shape) != want or t.dtype != dt or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError(f"expected contiguous {dt} {want}, got {t.dtype} {tuple(t.shape)}")


def conv3x3(x: torch.Tensor, weight: torch.Tensor, cin: int, cout: int, transposed: bool = False,
            residual: torch.Tensor | None = None, out_bf16: bool = True) -> torch.Tensor:
    """One layer (cin -> cout) of 3x3 convolution, or its adjoint (transposed=True)."""
    B, H, W = x.shape[0], x.shape[1], x.shape[2]
    ich, och = (cout, cin) if transposed else (cin, cout)
    _conv_in_check(x, ich, B, H, W)
    if weight.dtype != torch.float32 or not weight.is_contiguous() or weight.numel() != cout * 9 * cin:
        raise ValueError("weight must be contiguous float32 [cout][3][3][cin]")
    if och == 1:
        out = torch.empty((B, H, W), dtype=torch.float32, device=x.device)
    else:
        out = torch.empty((B, H, W, 32), dtype=torch.bfloat16 if out_bf16 else torch.float32, device=x.device)
    res = _ptr(residual) if residual is not None else None
    _check(_lib().xrt_conv3x3(cin, cout, int(transposed), B, H, W, _ptr(x), _ptr(weight), res, _ptr(out),
                              int(out_bf16), _stream(x.device.index)), "xrt_conv3x3")
    return out


def conv3x3_wgrad(x: torch.Tensor, dout: torch.Tensor, cin: int, cout: int) -> torch.Tensor:
    """Weight gradient [cout][3][3][cin] of layer (cin -> cout) for input x, output grad dout."""
    B, H, W = x.shape[0], x.shape[1], x.shape[2]
    _conv_in_check(x, cin, B, H, W)
    _conv_in_check(dout, cout, B, H, W)
    nwork = int(_lib().xrt_conv3x3_wgrad_workspace(cin, cout))
    work = torch.empty(nwork, dtype=torch.float32, device=x.device)
    dw = torch.empty((cout, 3, 3, cin), dtype=torch.float32, device=x.device)
    _check(_lib().xrt_conv3x3_wgrad(cin, cout, B, H, W, _ptr(x), _ptr(dout), _ptr(work), nwork, _ptr(dw),
                                    _stream(x.device.index)), "xrt_conv3x3_wgrad")
    return dw


def precond_apply(x: torch.Tensor, w1: torch.Tensor, w2: torch.Tensor, w3: torch.Tensor, transposed: bool = False,
                  out: torch.Tensor | None = None) -> torch.Tensor:
    """y = x + C3 C2 C1 x (transposed: x + C1^T C2^T C3^T x) in one launch; x float32 [B][H][W]."""
    B, H, W = x.shape[0], x.shape[1], x.shape[2]
    _conv_in_check(x, 1, B, H, W)
    for w, n in ((w1, 32 * 9), (w2, 32 * 9 * 32), (w3, 9 * 32)):
        if w.dtype != torch.float32 or not w.is_contiguous() or w.numel() != n or w.device != x.device:
            raise ValueError("weights must be contiguous float32 [32][3][3][1], [32][3][3][32], [1][3][3][32]")
    if out is None:
        out = torch.empty_like(x)
    else:
        _conv_in_check(out, 1, B, H, W)
    _check(_lib().xrt_precond_apply(int(transposed), B, H, W, _ptr(x), _ptr(w1), _ptr(w2), _ptr(w3), _ptr(out),
                                    _stream(x.device.index)), "xrt_precond_apply")
    return out


# ------------------------------------------------------------------ sparse storage of A


def offsets_from_counts(counts: torch.Tensor) -> torch.Tensor:
    """int64 [n+1] exclusive prefix sums of int32 counts [n] (deterministic)."""
    n = counts.numel()
    dev = counts.device
    if counts.dtype != torch.int32 or not counts.is_contiguous():
        raise ValueError("counts must be contiguous int32")
    offs = torch.empty(n + 1, dtype=torch.int64, device=dev)
    work = torch.empty(int(_lib().xrt_scan_workspace(n)), dtype=torch.int64, device=dev)
    _check(_lib().xrt_offsets_from_counts(n, _ptr(counts) if n else None, _ptr(offs), _ptr(work),
                                          _stream(dev.index)), "xrt_offsets_from_counts")
    return offs


class SparseMatrix:
    """A (and its transpose) in CSR storage on the device: rows are rays, columns units."""

    def __init__(self, n_rows: int, n_cols: int, off: torch.Tensor, col: torch.Tensor, val: torch.Tensor,
                 row_shape=None, col_shape=None):
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)
        self.off, self.col, self.val = off, col, val
        self.nnz = int(col.numel())
        self.row_shape = tuple(row_shape) if row_shape is not None else (self.n_rows,)
        self.col_shape = tuple(col_shape) if col_shape is not None else (self.n_cols,)
        self._t = None

    @classmethod
    def from_plan(cls, plan: "Plan", eps: float = 0.0) -> "SparseMatrix":
        """Hit lists of every ray of the plan (lengths > eps), as rows of A."""
        off, idx, ln = plan.hits(0, None, eps)
        return cls(plan.n_rays, plan.n_units, off, idx.contiguous(), ln.contiguous(), plan.sino_shape,
                   plan.image_shape)

    def transpose(self) -> "SparseMatrix":
        if self._t is None:
            dev = self.off.device
            t_off = torch.empty(self.n_cols + 1, dtype=torch.int64, device=dev)
            t_col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
            t_val = torch.empty(max(self.nnz, 1), dtype=torch.float32, device=dev)
            wl = int(_lib().xrt_csr_transpose_workspace(self.n_cols))
            work = torch.empty(wl, dtype=torch.int64, device=dev)
            _check(_lib().xrt_csr_transpose(self.n_rows, self.n_cols, self.nnz, _ptr(self.off),
                                            _ptr(self.col) if self.nnz else None,
                                            _ptr(self.val) if self.nnz else None, _ptr(t_off), _ptr(t_col),
                                            _ptr(t_val), _ptr(work), wl, _stream(dev.index)), "xrt_csr_transpose")
            t = SparseMatrix(self.n_cols, self.n_rows, t_off, t_col[:self.nnz], t_val[:self.nnz], self.col_shape,
                             self.row_shape)
            t._t = self
            self._t = t
        return self._t

    def matmul(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """y[b] = A x[b] for x [..., *col_shape] float32 contiguous."""
        n = len(self.col_shape)
        if tuple(x.shape[x.dim() - n:]) != self.col_shape or x.dtype != torch.float32 or not x.is_contiguous():
            raise ValueError(f"expected contiguous float32 [..., {self.col_shape}], got {x.dtype} {tuple(x.shape)}")
        lead = tuple(x.shape[:x.dim() - n])
        b = int(np.prod(lead)) if lead else 1
        if out is None:
            out = torch.empty(lead + self.row_shape, dtype=torch.float32, device=x.device)
        _check(_lib().xrt_csr_spmv(self.n_rows, self.n_cols, _ptr(self.off), _ptr(self.col) if self.nnz else None,
                                   _ptr(self.val) if self.nnz else None, b, _ptr(x), _ptr(out),
                                   _stream(x.device.index)), "xrt_csr_spmv")
        return out

    def matmul_interleaved(self, x_il: torch.Tensor, batch: int, out: torch.Tensor | None = None) -> torch.Tensor:
        """y_il [n_rows][batch] = A applied to x_il [n_cols][batch] (batch <= 64)."""
        if x_il.dtype != torch.float32 or not x_il.is_contiguous() or x_il.numel() != self.n_cols * batch:
            raise ValueError("x_il must be contiguous float32 [n_cols][batch]")
        if out is None:
            out = torch.empty((self.n_rows, batch), dtype=torch.float32, device=x_il.device)
        _check(_lib().xrt_csr_spmv_interleaved(self.n_rows, self.n_cols, _ptr(self.off),
                                               _ptr(self.col) if self.nnz else None,
                                               _ptr(self.val) if self.nnz else None, batch, _ptr(x_il), _ptr(out),
                                               _stream(x_il.device.index)), "xrt_csr_spmv_interleaved")
        return out

    def bytes(self) -> int:
        return self.off.numel() * 8 + self.nnz * 8


def interleave(x: torch.Tensor, batch: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """[batch][n] -> [n][batch] (batch <= 64)."""
    n = x.numel() // batch
    if out is None:
        out = torch.empty((n, batch), dtype=torch.float32, device=x.device)
    _check(_lib().xrt_interleave(n, batch, 1, _ptr(x), _ptr(out), _stream(x.device.index)), "xrt_interleave")
    return out


def deinterleave(x_il: torch.Tensor, batch: int, out: torch.Tensor) -> torch.Tensor:
    """[n][batch] -> out [batch][...] (out preallocated with batch * n elements)."""
    n = x_il.numel() // batch
    _check(_lib().xrt_interleave(n, batch, 0, _ptr(x_il), _ptr(out), _stream(x_il.device.index)), "xrt_interleave")
    return out
