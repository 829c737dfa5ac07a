"""ctypes binding of libgpawfd.so: argument marshalling only.

Tensors must be contiguous torch tensors on the GPU. Every call forwards
data pointers, sizes and the current HIP stream to the C ABI declared in
include/gpaw_fd.h; all arithmetic runs in the library's kernels. There is
no fallback: a missing library or a non-zero status raises.
"""
import ctypes
import json
import os

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libgpawfd.so")

GPAW_F64, GPAW_C128, GPAW_F32, GPAW_C64 = 0, 1, 2, 3

STATUS = {0: "GPAW_OK", -1: "GPAW_EINVAL", -2: "GPAW_EDTYPE", -3: "GPAW_ESHAPE",
          -4: "GPAW_EALIAS", -5: "GPAW_EHIP", -6: "GPAW_ENOTPD", -7: "GPAW_ENOMEM",
          -8: "GPAW_ENOCONV", -9: "GPAW_ENONFINITE"}


class GpawError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class Channel(ctypes.Structure):
    _fields_ = [("l", ctypes.c_int32), ("sigma", ctypes.c_double), ("rc", ctypes.c_double)]


class SysDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3), ("k", ctypes.c_double * 3),
                ("dtype", ctypes.c_int32), ("natoms", ctypes.c_int32),
                ("pos", ctypes.POINTER(ctypes.c_double)), ("nchan", ctypes.c_int32),
                ("chan", ctypes.POINTER(Channel)), ("dH", ctypes.POINTER(ctypes.c_double)),
                ("dS", ctypes.POINTER(ctypes.c_double)), ("v", ctypes.POINTER(ctypes.c_double)),
                ("max_bands", ctypes.c_int32), ("boundary", ctypes.c_int32)]


_lib = None

ENTRY_POINTS = ["gpaw_sys_create", "gpaw_sys_destroy", "gpaw_sys_info", "gpaw_project",
                "gpaw_fd_apply_H", "gpaw_fd_apply_S", "gpaw_fd_apply_HS", "gpaw_subspace_matrices",
                "gpaw_subspace_matrices_noalloc", "gpaw_density",
                "gpaw_davidson_correction", "gpaw_davidson_step",
                "gpaw_subspace_diag", "gpaw_rotate", "gpaw_orthonormalize",
                "gpaw_batch_create", "gpaw_batch_destroy", "gpaw_batch_step",
                "gpaw_batch_tune", "gpaw_batch_tuning", "gpaw_batch_set_tuning",
                "gpaw_last_error", "gpaw_version", "gpaw_probe_copy", "gpaw_probe_mfma",
                "gpaw_poisson_create", "gpaw_poisson_destroy", "gpaw_poisson_levels",
                "gpaw_poisson_solve", "gpaw_laplacian_zero", "gpaw_grid_restrict",
                "gpaw_grid_interpolate", "gpaw_td_kick", "gpaw_td_dipole", "gpaw_td_propagate"]


class BatchIO(ctypes.Structure):
    _fields_ = [("psi", ctypes.c_void_p), ("nb", ctypes.c_int32), ("psi_out", ctypes.c_void_p),
                ("eps", ctypes.c_void_p), ("P_out", ctypes.c_void_p), ("H_nn", ctypes.c_void_p),
                ("S_nn", ctypes.c_void_p), ("C_nn", ctypes.c_void_p)]


def library_path():
    return _LIB_PATH


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    lib.gpaw_sys_create.argtypes = [ctypes.POINTER(SysDesc), ctypes.POINTER(vp)]
    lib.gpaw_sys_destroy.argtypes = [vp]
    lib.gpaw_sys_destroy.restype = None
    lib.gpaw_sys_info.argtypes = [vp, i64p]
    lib.gpaw_project.argtypes = [vp, vp, i32, vp, vp]
    lib.gpaw_fd_apply_H.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.gpaw_fd_apply_S.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.gpaw_fd_apply_HS.argtypes = [vp, vp, i32, vp, vp, vp, vp]
    lib.gpaw_subspace_matrices.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp]
    lib.gpaw_subspace_matrices_noalloc.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp]
    lib.gpaw_probe_copy.argtypes = [vp, vp, ctypes.c_int64, vp]
    lib.gpaw_density.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
    lib.gpaw_davidson_correction.argtypes = [vp, vp, vp, vp, i32, vp, vp]
    lib.gpaw_davidson_step.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                       vp]
    lib.gpaw_probe_mfma.argtypes = [i32, vp, i32, i32, vp]
    lib.gpaw_subspace_diag.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
    lib.gpaw_rotate.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
    lib.gpaw_orthonormalize.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.gpaw_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
    lib.gpaw_batch_destroy.argtypes = [vp]
    lib.gpaw_batch_destroy.restype = None
    lib.gpaw_batch_step.argtypes = [vp, ctypes.POINTER(BatchIO), vp, vp]
    lib.gpaw_batch_tune.argtypes = [vp, ctypes.POINTER(BatchIO), vp]
    lib.gpaw_batch_tuning.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.gpaw_batch_set_tuning.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    i32p, f64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    lib.gpaw_poisson_create.argtypes = [i32p, f64p, ctypes.POINTER(vp)]
    lib.gpaw_poisson_destroy.argtypes = [vp]
    lib.gpaw_poisson_destroy.restype = None
    lib.gpaw_poisson_levels.argtypes = [vp, i32p]
    lib.gpaw_poisson_solve.argtypes = [vp, vp, vp, ctypes.c_double, i32, i32p, f64p, vp]
    lib.gpaw_laplacian_zero.argtypes = [i32p, f64p, vp, vp, vp]
    lib.gpaw_grid_restrict.argtypes = [i32p, vp, vp, vp]
    lib.gpaw_grid_interpolate.argtypes = [i32p, vp, vp, i32, vp]
    lib.gpaw_td_kick.argtypes = [vp, vp, i32, f64p, vp]
    lib.gpaw_td_dipole.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.gpaw_td_propagate.argtypes = [vp, vp, i32, ctypes.c_double, ctypes.c_double, i32, i32p,
                                      f64p, vp]
    lib.gpaw_last_error.restype = ctypes.c_char_p
    lib.gpaw_last_error.argtypes = []
    lib.gpaw_version.argtypes = []
    for name in ENTRY_POINTS:
        if name not in ("gpaw_sys_destroy", "gpaw_batch_destroy", "gpaw_last_error",
                        "gpaw_poisson_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise GpawError(rc, load().gpaw_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to the library must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _host(a, dtype=np.float64):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class System:
    """One FD-PAW system on the current GPU (owns the library's gpaw_sys)."""

    def __init__(self, n, h, k, pos, channels, dH, dS, v, max_bands, complex_=None,
                 precision="double", boundary="periodic"):
        lib = load()
        k = tuple(float(x) for x in k)
        if complex_ is None:
            complex_ = any(x != 0.0 for x in k)
        if precision not in ("double", "single"):
            raise ValueError("precision must be 'double' or 'single'")
        single = precision == "single"
        self.precision = precision
        if complex_:
            self.dtype = torch.complex64 if single else torch.complex128
            self.mat_dtype = torch.complex128
            code = GPAW_C64 if single else GPAW_C128
        else:
            self.dtype = torch.float32 if single else torch.float64
            self.mat_dtype = torch.float64
            code = GPAW_F32 if single else GPAW_F64
        self.n = tuple(int(x) for x in n)
        self.ng = int(np.prod(self.n))
        pos = _host(pos).reshape(-1, 3)
        self._keep = [pos, _host(dH), _host(dS), _host(v).ravel()]
        chans = (Channel * max(1, len(channels)))(*[Channel(int(l), float(s), float(r))
                                                    for (l, s, r) in channels])
        self._keep.append(chans)
        d = SysDesc()
        d.n[:] = self.n
        d.h[:] = [float(x) for x in (h if np.ndim(h) else (h, h, h))]
        d.k[:] = k
        d.dtype = code
        d.natoms = pos.shape[0]
        dp = ctypes.POINTER(ctypes.c_double)
        d.pos = self._keep[0].ctypes.data_as(dp)
        d.nchan = len(channels)
        d.chan = chans
        d.dH = self._keep[1].ctypes.data_as(dp)
        d.dS = self._keep[2].ctypes.data_as(dp)
        d.v = self._keep[3].ctypes.data_as(dp)
        d.max_bands = int(max_bands)
        if boundary not in ("periodic", "zero"):
            raise ValueError("boundary must be 'periodic' or 'zero'")
        d.boundary = 1 if boundary == "zero" else 0
        self.boundary = boundary
        handle = ctypes.c_void_p()
        _check(lib.gpaw_sys_create(ctypes.byref(d), ctypes.byref(handle)))
        self._h = handle
        info = (ctypes.c_int64 * 8)()
        _check(lib.gpaw_sys_info(self._h, info))
        self.info = dict(ng=info[0], np=info[1], ni=info[2], natoms=info[3], entries=info[4],
                         covered=info[5], max_bands=info[6], dtype=info[7])
        self.np = int(info[1])
        self.ni = int(info[2])
        self.natoms = int(info[3])
        self.max_bands = int(max_bands)
        self.device = torch.device("cuda", torch.cuda.current_device())

    @classmethod
    def from_synth(cls, s, max_bands=None, precision="double", boundary=None):
        """boundary: 'periodic' or 'zero' (default: the system's own, if it
        names one, else periodic)."""
        boundary = boundary or getattr(s, "meta", {}).get("boundary", "periodic")
        return cls(s.n, s.h, s.k, s.pos, s.channels, s.dH, s.dS, s.v,
                   max_bands or s.nb, complex_=s.is_complex, precision=precision,
                   boundary=boundary)

    # real-time propagation (finite systems, complex128)
    def td_kick(self, psi, kappa, stream=None):
        """gpaw_td_kick: psi <- exp(-i kappa . r) psi, in place."""
        k = (ctypes.c_double * 3)(*[float(x) for x in kappa])
        _check(load().gpaw_td_kick(self._h, _ptr(psi), psi.shape[0], k, _stream(stream)))
        return psi

    def td_dipole(self, psi, f, out=None, stream=None):
        """gpaw_td_dipole: pseudo-density dipole (device tensor of 3)."""
        if out is None:
            out = torch.empty(3, dtype=torch.float64, device=psi.device)
        f = f.to(device=psi.device, dtype=torch.float64).contiguous()
        _check(load().gpaw_td_dipole(self._h, _ptr(psi), psi.shape[0], _ptr(f), _ptr(out),
                                     _stream(stream)))
        return out

    def td_propagate(self, psi, dt, tol=1e-12, max_iter=200, stream=None):
        """gpaw_td_propagate: one Crank-Nicolson step in place; returns
        (iterations, largest relative residual)."""
        it, res = ctypes.c_int32(), ctypes.c_double()
        _check(load().gpaw_td_propagate(self._h, _ptr(psi), psi.shape[0], float(dt), float(tol),
                                        int(max_iter), ctypes.byref(it), ctypes.byref(res),
                                        _stream(stream)))
        return it.value, res.value

    def close(self):
        if getattr(self, "_h", None):
            load().gpaw_sys_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ helpers
    def _new(self, *shape, dtype=None):
        return torch.empty(shape, dtype=dtype or self.dtype, device=self.device)

    def _nb(self, psi):
        if psi.dtype != self.dtype:
            raise TypeError(f"expected {self.dtype}, got {psi.dtype}")
        if psi.numel() % self.ng:
            raise ValueError("psi does not hold whole grids")
        return psi.numel() // self.ng

    # ------------------------------------------------------------ calls
    def project(self, psi, out=None, stream=None):
        nb = self._nb(psi)
        out = self._new(nb, self.np) if out is None else out
        _check(load().gpaw_project(self._h, _ptr(psi), nb, _ptr(out), _stream(stream)))
        return out

    def apply_H(self, psi, P=None, out=None, stream=None):
        nb = self._nb(psi)
        out = torch.empty_like(psi) if out is None else out
        _check(load().gpaw_fd_apply_H(self._h, _ptr(psi), nb, _ptr(P), _ptr(out), _stream(stream)))
        return out

    def apply_S(self, psi, P=None, out=None, stream=None):
        nb = self._nb(psi)
        out = torch.empty_like(psi) if out is None else out
        _check(load().gpaw_fd_apply_S(self._h, _ptr(psi), nb, _ptr(P), _ptr(out), _stream(stream)))
        return out

    def apply_HS(self, psi, P=None, Hpsi=None, Spsi=None, stream=None):
        """H~psi and S~psi in one pass (same results as apply_H and apply_S)."""
        nb = self._nb(psi)
        Hpsi = torch.empty_like(psi) if Hpsi is None else Hpsi
        Spsi = torch.empty_like(psi) if Spsi is None else Spsi
        _check(load().gpaw_fd_apply_HS(self._h, _ptr(psi), nb, _ptr(P), _ptr(Hpsi), _ptr(Spsi),
                                       _stream(stream)))
        return Hpsi, Spsi

    def subspace_matrices(self, psi, Hpsi, Spsi=None, H=None, S=None, stream=None):
        nb = self._nb(psi)
        H = self._new(nb, nb, dtype=self.mat_dtype) if H is None else H
        if Spsi is not None and S is None:
            S = self._new(nb, nb, dtype=self.mat_dtype)
        _check(load().gpaw_subspace_matrices(self._h, _ptr(psi), _ptr(Hpsi), _ptr(Spsi), nb,
                                             _ptr(H), _ptr(S), _stream(stream)))
        return H, S

    def subspace_matrices_noalloc(self, psi, Hpsi, Spsi, H, S, stream=None):
        """gpaw_subspace_matrices_noalloc: caller-provided outputs, nothing
        allocated by the library (partial sums in its static device array)."""
        nb = self._nb(psi)
        _check(load().gpaw_subspace_matrices_noalloc(self._h, _ptr(psi), _ptr(Hpsi), _ptr(Spsi),
                                                     nb, _ptr(H), _ptr(S), _stream(stream)))
        return H, S

    def density(self, psi, f, P=None, n_out=None, D=None, want_D=True, stream=None):
        """Pseudo density [Ng] (float64) and atomic density matrices
        [natoms][ni][ni] (mat dtype) of the block with occupations f."""
        nb = self._nb(psi)
        if f.dtype != torch.float64 or f.numel() != nb:
            raise ValueError("f must be a float64 tensor of nb occupations")
        n_out = self._new(self.ng, dtype=torch.float64) if n_out is None else n_out
        if D is None and want_D and self.natoms > 0:
            D = self._new(self.natoms, self.ni, self.ni, dtype=self.mat_dtype)
        _check(load().gpaw_density(self._h, _ptr(psi), nb, _ptr(f), _ptr(P), _ptr(n_out),
                                   _ptr(D), _stream(stream)))
        return n_out, D

    def davidson_correction(self, Hpsi, Spsi, eps, out=None, stream=None):
        nb = self._nb(Hpsi)
        out = torch.empty_like(Hpsi) if out is None else out
        _check(load().gpaw_davidson_correction(self._h, _ptr(Hpsi), _ptr(Spsi), _ptr(eps), nb,
                                               _ptr(out), _stream(stream)))
        return out

    def davidson_step(self, x, Hx, Sx, Px, eps, out=None, info=None, stream=None):
        """One block Davidson step; x, Hx, Sx: [2nb][Ng] with the Ritz block in
        rows 0..nb-1 (rows nb.. are overwritten), Px [2nb][Np] likewise, eps
        [nb]. Returns dict(psi, P, eps (the lowest nb of eps2), eps2, H2, S2, C2)."""
        n2 = self._nb(x)
        if n2 % 2:
            raise ValueError("x must hold 2 nb bands")
        nb = n2 // 2
        o = out or {}
        psi = o.get("psi", self._new(nb, self.ng))
        P = o.get("P", self._new(nb, self.np)) if self.np else None
        H2 = o.get("H2", self._new(n2, n2, dtype=self.mat_dtype))
        S2 = o.get("S2", self._new(n2, n2, dtype=self.mat_dtype))
        C2 = o.get("C2", self._new(n2, n2, dtype=self.mat_dtype))
        e2 = o.get("eps2", self._new(n2, dtype=torch.float64))
        _check(load().gpaw_davidson_step(self._h, nb, _ptr(x), _ptr(Hx), _ptr(Sx),
                                         _ptr(Px) if self.np else None, _ptr(eps), _ptr(H2),
                                         _ptr(S2), _ptr(C2), _ptr(e2), _ptr(psi), _ptr(P),
                                         _ptr(info), _stream(stream)))
        return dict(psi=psi, P=P, eps=e2[:nb], eps2=e2, H2=H2, S2=S2, C2=C2)

    def subspace_diag(self, H, S, eps=None, C=None, info=None, stream=None):
        nb = H.shape[0]
        eps = self._new(nb, dtype=torch.float64) if eps is None else eps
        C = self._new(nb, nb, dtype=self.mat_dtype) if C is None else C
        _check(load().gpaw_subspace_diag(self._h, _ptr(H), _ptr(S), nb, _ptr(eps), _ptr(C),
                                         _ptr(info), _stream(stream)))
        return eps, C

    def rotate(self, psi, C, out=None, P=None, P_out=None, stream=None):
        nb = self._nb(psi)
        out = torch.empty_like(psi) if out is None else out
        if P is not None and P_out is None:
            P_out = torch.empty_like(P)
        _check(load().gpaw_rotate(self._h, _ptr(psi), _ptr(C), nb, _ptr(out), _ptr(P),
                                  _ptr(P_out), _stream(stream)))
        return out, P_out

    def orthonormalize(self, psi, Spsi, out=None, P=None, P_out=None, info=None, stream=None):
        nb = self._nb(psi)
        out = torch.empty_like(psi) if out is None else out
        if P is not None and P_out is None:
            P_out = torch.empty_like(P)
        _check(load().gpaw_orthonormalize(self._h, _ptr(psi), _ptr(Spsi), nb, _ptr(out), _ptr(P),
                                          _ptr(P_out), _ptr(info), _stream(stream)))
        return out, P_out

    def step(self, psi, stream=None):
        """One block step: P, H~psi, S~psi, H_nm, S_nm, eigensolve, rotation."""
        P = self.project(psi, stream=stream)
        Hpsi, Spsi = self.apply_HS(psi, P, stream=stream)
        H, S = self.subspace_matrices(psi, Hpsi, Spsi, stream=stream)
        eps, C = self.subspace_diag(H, S, stream=stream)
        psi_rot, P_rot = self.rotate(psi, C, P=P, stream=stream)
        return dict(P=P, Hpsi=Hpsi, Spsi=Spsi, H=H, S=S, eps=eps, C=C,
                    psi_rot=psi_rot, P_rot=P_rot)


TUNING_KEYS = ("stencil_ppl", "stencil_ty", "stencil_tz", "stencil_xseg", "subspace_wgs",
               "rotate_rb", "project_nbg")


class Batch:
    """Many independent systems stepped by one graph launch (owns the
    library's gpaw_batch, not the systems)."""

    def __init__(self, systems):
        lib = load()
        self.systems = list(systems)
        arr = (ctypes.c_void_p * len(self.systems))(*[s._h.value for s in self.systems])
        handle = ctypes.c_void_p()
        _check(lib.gpaw_batch_create(arr, len(self.systems), ctypes.byref(handle)))
        self._h = handle

    def close(self):
        if getattr(self, "_h", None):
            load().gpaw_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def io(self, psis, psi_outs, eps, P_outs=None, Hs=None, Ss=None, Cs=None):
        """Host array of per-system buffers (lists of tensors; None entries allowed
        for the optional ones)."""
        n = len(self.systems)
        arr = (BatchIO * n)()
        for i, s in enumerate(self.systems):
            arr[i].psi = _ptr(psis[i])
            arr[i].nb = s._nb(psis[i])
            arr[i].psi_out = _ptr(psi_outs[i])
            arr[i].eps = _ptr(eps[i])
            arr[i].P_out = _ptr(P_outs[i]) if P_outs else None
            arr[i].H_nn = _ptr(Hs[i]) if Hs else None
            arr[i].S_nn = _ptr(Ss[i]) if Ss else None
            arr[i].C_nn = _ptr(Cs[i]) if Cs else None
        return arr

    def step(self, io, info, stream=None):
        _check(load().gpaw_batch_step(self._h, io, _ptr(info), _stream(stream)))

    def tune(self, io, info):
        _check(load().gpaw_batch_tune(self._h, io, _ptr(info)))

    def tuning(self):
        n = len(self.systems)
        out = (ctypes.c_int32 * (1 + 7 * n))()
        _check(load().gpaw_batch_tuning(self._h, out))
        return int(out[0]), [dict(zip(TUNING_KEYS, out[1 + 7 * i: 8 + 7 * i])) for i in range(n)]

    def set_tuning(self, branches, shapes):
        """gpaw_batch_set_tuning: shapes as tuning() returns them."""
        n = len(self.systems)
        if len(shapes) != n:
            raise ValueError("one shape dict per system")
        arr = (ctypes.c_int32 * (1 + 7 * n))()
        arr[0] = int(branches)
        for i, sh in enumerate(shapes):
            for j, key in enumerate(TUNING_KEYS):
                arr[1 + 7 * i + j] = int(sh[key])
        _check(load().gpaw_batch_set_tuning(self._h, arr))

    def signature(self):
        """What a stored tuning is valid for: per system the grid, storage
        type, boundary, band capacity and projector geometry."""
        return [dict(n=list(g.n), dtype=str(g.dtype).replace("torch.", ""), boundary=g.boundary,
                     max_bands=g.max_bands, natoms=g.natoms, np=g.np,
                     entries=int(g.info["entries"])) for g in self.systems]

    def save_tuning(self, path):
        """Writes the current launch shapes and the batch's signature (JSON)."""
        branches, shapes = self.tuning()
        with open(path, "w") as fh:
            json.dump(dict(format="gpaw-fd-tuning", version=1, signature=self.signature(),
                           branches=branches, shapes=shapes), fh, indent=1)

    def load_tuning(self, path):
        """Applies shapes saved by save_tuning when they were made for the
        same systems (same signature): returns True, else False and leaves
        the batch unchanged."""
        with open(path) as fh:
            data = json.load(fh)
        if data.get("format") != "gpaw-fd-tuning" or data.get("signature") != self.signature():
            return False
        self.set_tuning(data["branches"], data["shapes"])
        return True


def probe_copy(src, dst, stream=None):
    """gpaw_probe_copy: dst = src (device tensors of equal byte size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst must have the same size")
    _check(load().gpaw_probe_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)))


def probe_mfma(kind, out, workgroups, iters, stream=None):
    """gpaw_probe_mfma: kind 0 FP64 (out float64), 1 BF16 (out float32)."""
    if out.numel() < workgroups * 256:
        raise ValueError("out needs workgroups x 256 values")
    _check(load().gpaw_probe_mfma(kind, _ptr(out), workgroups, iters, _stream(stream)))


def _i3(n):
    return (ctypes.c_int32 * 3)(*[int(x) for x in n])


def _d3(h):
    return (ctypes.c_double * 3)(*[float(x) for x in h])


def _grid_f64(t, shape, name):
    if t.dtype != torch.float64 or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a float64 tensor of shape {tuple(shape)}")


class Poisson:
    """Multigrid solver of nabla^2 phi = -4 pi rho on a zero-boundary grid
    (gpaw_poisson_create / _solve / _destroy)."""

    def __init__(self, n, h):
        self.n = tuple(int(x) for x in n)
        self.h = tuple(float(x) for x in h)
        handle = ctypes.c_void_p()
        _check(load().gpaw_poisson_create(_i3(self.n), _d3(self.h), ctypes.byref(handle)))
        self._p = handle

    @property
    def levels(self):
        v = ctypes.c_int32()
        _check(load().gpaw_poisson_levels(self._p, ctypes.byref(v)))
        return v.value

    def solve(self, rho, phi=None, tol=1e-12, max_cycles=100, stream=None):
        """phi (initial guess, zeros if None) -> (phi, cycles, relative residual)."""
        _grid_f64(rho, self.n, "rho")
        if phi is None:
            phi = torch.zeros_like(rho)
        _grid_f64(phi, self.n, "phi")
        cyc, res = ctypes.c_int32(), ctypes.c_double()
        _check(load().gpaw_poisson_solve(self._p, _ptr(rho), _ptr(phi), float(tol),
                                         int(max_cycles), ctypes.byref(cyc), ctypes.byref(res),
                                         _stream(stream)))
        return phi, cyc.value, res.value

    def close(self):
        if self._p:
            load().gpaw_poisson_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def laplacian_zero(f, h, out=None, stream=None):
    """gpaw_laplacian_zero: nabla^2 f on the zero-boundary grid."""
    if out is None:
        out = torch.empty_like(f)
    _grid_f64(f, f.shape, "f")
    _grid_f64(out, f.shape, "out")
    _check(load().gpaw_laplacian_zero(_i3(f.shape), _d3(h), _ptr(f), _ptr(out), _stream(stream)))
    return out


def grid_restrict(fine, out=None, stream=None):
    """gpaw_grid_restrict: full weighting onto the (n - 1) / 2 grid."""
    nc = tuple((m - 1) // 2 for m in fine.shape)
    if out is None:
        out = torch.empty(nc, dtype=torch.float64, device=fine.device)
    _grid_f64(fine, fine.shape, "fine")
    _grid_f64(out, nc, "out")
    _check(load().gpaw_grid_restrict(_i3(fine.shape), _ptr(fine), _ptr(out), _stream(stream)))
    return out


def grid_interpolate(coarse, nf, out=None, accumulate=False, stream=None):
    """gpaw_grid_interpolate: trilinear interpolation onto the nf grid."""
    nf = tuple(int(x) for x in nf)
    if out is None:
        out = torch.zeros(nf, dtype=torch.float64, device=coarse.device)
    _grid_f64(coarse, tuple((m - 1) // 2 for m in nf), "coarse")
    _grid_f64(out, nf, "out")
    _check(load().gpaw_grid_interpolate(_i3(nf), _ptr(coarse), _ptr(out), 1 if accumulate else 0,
                                        _stream(stream)))
    return out
