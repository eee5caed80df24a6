"""Thin ctypes binding of liblofqmc (the C ABI declared in include/lofqmc.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device arrays are torch tensors on the GPU (torch supplies device
memory and the stream); complex arrays are torch.complex128, whose storage is
the interleaved (re, im) layout the ABI expects.  The library must have been
built (python -m paper_2202_00832_amd.build); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblofqmc.so")
HEADER_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lofqmc.h")

LO_OK, LO_EINVAL, LO_ENOMEM, LO_EHIP, LO_EUNSUPPORTED, LO_ESOLVER = 0, -1, -2, -3, -4, -5
LO_FP64, LO_FP32, LO_BF16X3, LO_BF16 = 0, 1, 2, 3
LO_THETA_ORBITAL_MAJOR = 1
LO_EXACT_COULOMB = 2
LO_FACTORS_RANDOMIZED = 1
LO_FLAG_SMALL_PIVOT = 4
LO_THETA_TRANSPOSED = 8
RESIDUAL_NFEAT = 4   # per-orbital features of the learned residual
_NAMES = {0: "LO_OK", -1: "LO_EINVAL", -2: "LO_ENOMEM", -3: "LO_EHIP", -4: "LO_EUNSUPPORTED", -5: "LO_ESOLVER"}

_c_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_SIGS = {
    "lo_create": (ctypes.c_int, [ctypes.POINTER(_c_p), _c_p]),
    "lo_set_stream": (ctypes.c_int, [_c_p, _c_p]),
    "lo_synchronize": (ctypes.c_int, [_c_p]),
    "lo_destroy": (ctypes.c_int, [_c_p]),
    "lo_last_error": (ctypes.c_char_p, [_c_p]),
    "lo_profile_enable": (ctypes.c_int, [_c_p, ctypes.c_int]),
    "lo_profile_summary": (ctypes.c_int, [_c_p, ctypes.c_int, _c_p, _c_p, _c_p, ctypes.POINTER(ctypes.c_int)]),
    "build_half_rotated_chol": (ctypes.c_int, [_c_p, _i64, _i64, _i64, _c_p, _c_p, _c_p]),
    "build_lo_factors": (ctypes.c_int, [_c_p, _i64, _i64, _i64, _c_p, ctypes.c_double, ctypes.POINTER(_c_p)]),
    "build_lo_factors_randomized": (ctypes.c_int, [_c_p, _i64, _i64, _i64, _c_p, ctypes.c_double, _i64, ctypes.c_int,
                                                    _c_p, ctypes.POINTER(_c_p)]),
    "lo_factors_destroy": (ctypes.c_int, [_c_p]),
    "lo_factors_info": (ctypes.c_int, [_c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "lo_factors_export": (ctypes.c_int, [_c_p, _c_p, _c_p]),
    "lo_factors_flags": (ctypes.c_int, [_c_p, _c_p]),
    "lo_factors_import": (ctypes.c_int, [_c_p, _i64, _i64, _i64, _c_p, _c_p, _c_p, _c_p, _c_p, ctypes.c_uint,
                                         ctypes.POINTER(_c_p)]),
    "green_theta": (ctypes.c_int, [_c_p, _i64, _i64, _i64, _c_p, _c_p, _c_p, _c_p, _c_p, ctypes.c_uint]),
    "local_energy_full": (ctypes.c_int, [_c_p, _i64, _i64, _i64, _i64, _c_p, _c_p, _c_p, ctypes.c_int,
                                         ctypes.c_uint, _c_p]),
    "local_energy_lo": (ctypes.c_int, [_c_p, _c_p, _i64, _c_p, _c_p, ctypes.c_int, ctypes.c_uint, _c_p, _c_p]),
    "local_energy_lo_noalloc": (ctypes.c_int, [_c_p, _c_p, _i64, _c_p, _c_p, ctypes.c_int, ctypes.c_uint, _c_p,
                                                _c_p]),
    "build_hr_eri": (ctypes.c_int, [_c_p, _i64, _i64, _i64, _c_p, ctypes.POINTER(_c_p)]),
    "lo_localize_boys": (ctypes.c_int, [_c_p, _i64, _i64, _i64, _c_p, _c_p, ctypes.c_int, ctypes.c_double, _c_p]),
    "lo_hr_destroy": (ctypes.c_int, [_c_p]),
    "lo_hr_info": (ctypes.c_int, [_c_p, _c_p, _c_p, _c_p]),
    "local_energy_hr": (ctypes.c_int, [_c_p, _c_p, _i64, _c_p, _c_p, ctypes.c_uint, _c_p]),
    "build_md_trial": (ctypes.c_int, [_c_p, _c_p, _i64, _i64, _c_p, _i64, _i64, _c_p, _c_p, _c_p, _c_p,
                                      ctypes.POINTER(_c_p)]),
    "lo_md_destroy": (ctypes.c_int, [_c_p]),
    "lo_md_info": (ctypes.c_int, [_c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "local_energy_md": (ctypes.c_int, [_c_p, _c_p, _i64, _c_p, _c_p, ctypes.c_uint, _c_p, _c_p]),
    "lo_batch_create": (ctypes.c_int, [_c_p, ctypes.c_int, _c_p, ctypes.c_int, _c_p, ctypes.POINTER(_c_p)]),
    "lo_batch_destroy": (ctypes.c_int, [_c_p]),
    "lo_batch_info": (ctypes.c_int, [_c_p, _c_p, _c_p]),
    "lo_batch_execute": (ctypes.c_int, [_c_p, _c_p]),
    "lo_batch_capture": (ctypes.c_int, [_c_p, _c_p, ctypes.c_int]),
    "lo_batch_replay": (ctypes.c_int, [_c_p, _c_p]),
    "lo_residual_nparam": (ctypes.c_int, []),
    "lo_factors_discarded": (ctypes.c_int, [_c_p, _c_p]),
    "lo_residual_prepare": (ctypes.c_int, [_c_p, _c_p, _i64, _c_p, _c_p, _c_p]),
    "lo_residual_target": (ctypes.c_int, [_c_p, _i64, _c_p, _c_p, ctypes.c_double, ctypes.c_double, _c_p]),
    "lo_residual_apply": (ctypes.c_int, [_c_p, _i64, _c_p, _c_p, ctypes.c_double, ctypes.c_double, _c_p]),
    "lo_residual_features": (ctypes.c_int, [_c_p, _c_p, _i64, _c_p, _c_p]),
    "lo_residual_predict": (ctypes.c_int, [_c_p, _i64, _i64, _c_p, _c_p, ctypes.c_int, _c_p]),
    "lo_residual_train_step": (ctypes.c_int, [_c_p, _i64, _i64, _c_p, _c_p, _c_p, _i64, ctypes.c_double, _c_p,
                                              _c_p, _c_p, _c_p, _c_p]),
}



class _System(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("n_occ", ctypes.c_int64), ("n_chol", ctypes.c_int64), ("nw", ctypes.c_int64),
                ("lbar", ctypes.c_void_p), ("theta", ctypes.c_void_p), ("info", ctypes.c_void_p),
                ("energy", ctypes.c_void_p), ("trial", ctypes.c_void_p), ("phi", ctypes.c_void_p)]


_lib = None


class LoError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, message))
        self.code = code


def load() -> ctypes.CDLL:
    """Loads liblofqmc.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblofqmc.so is not built; run `python -m paper_2202_00832_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def declared_functions() -> list[str]:
    """Names of the functions declared in include/lofqmc.h."""
    with open(HEADER_PATH) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _check_dev(name, t, dtype, shape):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))


class HrEri:
    """Owner of a lo_hr handle: the pair blocks Y^[ij] of the half-rotated ERI (device)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)
        M = ctypes.c_int64()
        n = ctypes.c_int64()
        b = ctypes.c_int64()
        load().lo_hr_info(self._h, ctypes.byref(M), ctypes.byref(n), ctypes.byref(b))
        self.M, self.n_occ, self.bytes = M.value, n.value, b.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load().lo_hr_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MdTrial:
    """Owner of a lo_md handle: a multi-determinant trial over the orbitals of an
    LO factor handle (the handle copies what it needs of the factors, which may
    be closed afterwards)."""

    def __init__(self, handle: int, factors):
        self._h = ctypes.c_void_p(handle)
        vals = [ctypes.c_int64() for _ in range(5)]
        load().lo_md_info(self._h, *[ctypes.byref(v) for v in vals])
        self.n_occ, self.n_cas, self.n_det, self.npairs, self.out_rows = [v.value for v in vals]
        self.M = factors.M

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load().lo_md_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Factors:
    """Owner of a lo_factors handle (device storage held by the library)."""

    def __init__(self, handle: int, n_chol: int = 0):
        self._h = ctypes.c_void_p(handle)
        M = ctypes.c_int64()
        n = ctypes.c_int64()
        load().lo_factors_info(self._h, ctypes.byref(M), ctypes.byref(n), None, None, None, None)
        self.M, self.n_occ = M.value, n.value
        self.n_chol = n_chol

    def checkpoint(self) -> dict:
        """Everything lo_factors_import needs, as numpy arrays (np.savez-able)."""
        inf = self.info()
        M, n = inf["M"], inf["n_occ"]
        rows = np.zeros((inf["total_rows"], M), dtype=np.float64)
        off = np.zeros((n, n), dtype=np.int64)
        lib = load()
        rc = lib.lo_factors_export(self._h, rows.ctypes.data if rows.size else None, off.ctypes.data)
        if rc != LO_OK:
            raise LoError(rc, "lo_factors_export failed")
        fl = ctypes.c_uint()
        lib.lo_factors_flags(self._h, ctypes.byref(fl))
        return {"M": np.int64(M), "n_occ": np.int64(n), "n_chol": np.int64(self.n_chol), "ranks": inf["ranks"],
                "row_offset": off, "first_dropped": inf["first_dropped"], "discarded": self.discarded(),
                "rows": rows, "flags": np.int64(fl.value)}

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load().lo_factors_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        lib = load()
        M = ctypes.c_int64()
        n = ctypes.c_int64()
        lib.lo_factors_info(self._h, ctypes.byref(M), ctypes.byref(n), None, None, None, None)
        ranks = np.zeros((n.value, n.value), dtype=np.int32)
        fd = np.zeros((n.value, n.value), dtype=np.float64)
        rows = ctypes.c_int64()
        nbytes = ctypes.c_int64()
        lib.lo_factors_info(self._h, None, None, ranks.ctypes.data, fd.ctypes.data, ctypes.byref(rows),
                            ctypes.byref(nbytes))
        return {"M": M.value, "n_occ": n.value, "ranks": ranks, "first_dropped": fd,
                "total_rows": rows.value, "bytes": nbytes.value}

    def discarded(self) -> np.ndarray:
        """Sum of the discarded singular values of every pair block, [n][n]."""
        n = self.n_occ
        out = np.zeros((n, n), dtype=np.float64)
        rc = load().lo_factors_discarded(self._h, out.ctypes.data)
        if rc != LO_OK:
            raise LoError(rc, "lo_factors_discarded failed")
        return out

    def export(self) -> dict:
        """{(i, j): (Ubar [M x K], Vbar [K x M], first_dropped)} for i <= j (host copies)."""
        inf = self.info()
        M, n = inf["M"], inf["n_occ"]
        rows = np.zeros((max(inf["total_rows"], 1), M), dtype=np.float64)
        off = np.zeros((n, n), dtype=np.int64)
        rc = load().lo_factors_export(self._h, rows.ctypes.data, off.ctypes.data)
        if rc != LO_OK:
            raise LoError(rc, "lo_factors_export failed")
        out = {}
        for i in range(n):
            for j in range(i, n):
                K = int(inf["ranks"][i, j])
                o = int(off[i, j])
                Ubar = rows[o:o + K].T.copy()
                Vbar = rows[o + K:o + 2 * K].copy()
                out[(i, j)] = (Ubar, Vbar, float(inf["first_dropped"][i, j]))
        return out


class Batch:
    """A plan for the FP32 full-route energies of several systems (lo_batch_*)."""

    def __init__(self, ctx: "Context", systems, chunk=None):
        """systems: list of dicts with lbar [X][M][n] f64, theta [nw][M][n] c128,
        optional info [nw] i32 and energy [nw][2] c128 (device tensors), and
        optionally trial [M][n] f64 and phi [nw][M][n] c128: then every
        evaluation first forms theta and info from them (green_theta)."""
        import torch
        self.ctx = ctx
        self.systems = []
        arr = (_System * len(systems))()
        for k, sd in enumerate(systems):
            lbar, theta = sd["lbar"], sd["theta"]
            X, M, n = lbar.shape
            nw = theta.shape[0]
            _check_dev("lbar", lbar, torch.float64, (X, M, n))
            _check_dev("theta", theta, torch.complex128, (nw, M, n))
            info = sd.get("info")
            if info is not None:
                _check_dev("info", info, torch.int32, (nw,))
            energy = sd.get("energy")
            if energy is None:
                energy = torch.empty((nw, 2), dtype=torch.complex128, device=theta.device)
            _check_dev("energy", energy, torch.complex128, (nw, 2))
            trial, phi = sd.get("trial"), sd.get("phi")
            if phi is not None:
                _check_dev("trial", trial, torch.float64, (M, n))
                _check_dev("phi", phi, torch.complex128, (nw, M, n))
                if info is None:
                    info = torch.zeros((nw,), dtype=torch.int32, device=theta.device)
            self.systems.append({"lbar": lbar, "theta": theta, "info": info, "energy": energy, "trial": trial,
                                 "phi": phi})
            arr[k] = _System(M, n, X, nw, _ptr(lbar), _ptr(theta), _ptr(info), _ptr(energy), _ptr(trial), _ptr(phi))
        ch = None
        if chunk is not None:
            ch = np.ascontiguousarray(chunk, dtype=np.int64)
            assert ch.shape == (len(systems),)
        h = ctypes.c_void_p()
        ctx._check(ctx._lib.lo_batch_create(ctx.handle, len(systems), ctypes.addressof(arr), LO_FP32,
                                            ch.ctypes.data if ch is not None else None, ctypes.byref(h)))
        self._h = h

    @property
    def energies(self):
        return [sd["energy"] for sd in self.systems]

    def info(self):
        nitems = ctypes.c_int64()
        ch = np.zeros(len(self.systems), dtype=np.int64)
        self.ctx._check(self.ctx._lib.lo_batch_info(self._h, ctypes.byref(nitems), ch.ctypes.data))
        return {"items": nitems.value, "chunk": ch}

    def execute(self):
        self.ctx._check(self.ctx._lib.lo_batch_execute(self.ctx.handle, self._h))

    def capture(self, repeats: int):
        self.ctx._check(self.ctx._lib.lo_batch_capture(self.ctx.handle, self._h, int(repeats)))

    def replay(self):
        self.ctx._check(self.ctx._lib.lo_batch_replay(self.ctx.handle, self._h))

    def close(self):
        if self._h:
            load().lo_batch_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



def _theta_layout(theta, M, n, orbital_major, transposed):
    """(nw, layout flag, expected shape) of a theta tensor: [nw][M][n],
    [n][M][nw] (orbital_major) or [nw][n][M] (transposed)."""
    if orbital_major and transposed:
        raise ValueError("theta cannot be orbital-major and transposed")
    if orbital_major:
        nw = theta.shape[2]
        return nw, LO_THETA_ORBITAL_MAJOR, (n, M, nw)
    nw = theta.shape[0]
    if transposed:
        return nw, LO_THETA_TRANSPOSED, (nw, n, M)
    return nw, 0, (nw, M, n)

class Context:
    """A library context bound to a HIP stream (default: torch's current stream)."""

    def __init__(self, stream=None):
        self._lib = load()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
        h = ctypes.c_void_p()
        rc = self._lib.lo_create(ctypes.byref(h), ctypes.c_void_p(stream))
        if rc != LO_OK:
            raise LoError(rc, "lo_create failed")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            self._lib.lo_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != LO_OK:
            raise LoError(rc, self._lib.lo_last_error(self._h).decode())

    def synchronize(self):
        self._check(self._lib.lo_synchronize(self._h))

    # -- kernel timing (diagnostics) --------------------------------------------
    def profile_enable(self, enable: bool = True):
        self._check(self._lib.lo_profile_enable(self._h, 1 if enable else 0))

    def profile_summary(self, max_kernels: int = 32) -> dict:
        """{kernel name: (launches, total ms)} since the last enable/summary."""
        names = ctypes.create_string_buffer(64 * max_kernels)
        launches = np.zeros(max_kernels, dtype=np.int64)
        total = np.zeros(max_kernels, dtype=np.float64)
        count = ctypes.c_int(0)
        self._check(self._lib.lo_profile_summary(self._h, max_kernels, ctypes.addressof(names),
                                                 launches.ctypes.data, total.ctypes.data, ctypes.byref(count)))
        out = {}
        for k in range(min(count.value, max_kernels)):
            name = names.raw[64 * k:64 * (k + 1)].split(b"\0", 1)[0].decode()
            out[name] = (int(launches[k]), float(total[k]))
        return out

    # -- set-up ---------------------------------------------------------------
    def build_half_rotated_chol(self, chol, trial, lbar=None):
        import torch
        X, M, _ = chol.shape
        n = trial.shape[1]
        _check_dev("chol", chol, torch.float64, (X, M, M))
        _check_dev("trial", trial, torch.float64, (M, n))
        if lbar is None:
            lbar = torch.empty((X, M, n), dtype=torch.float64, device=chol.device)
        _check_dev("lbar", lbar, torch.float64, (X, M, n))
        self._check(self._lib.build_half_rotated_chol(self._h, M, n, X, _ptr(chol), _ptr(trial), _ptr(lbar)))
        return lbar

    def build_lo_factors(self, lbar, epsilon: float) -> Factors:
        import torch
        X, M, n = lbar.shape
        _check_dev("lbar", lbar, torch.float64, (X, M, n))
        h = ctypes.c_void_p()
        self._check(self._lib.build_lo_factors(self._h, M, n, X, _ptr(lbar), float(epsilon), ctypes.byref(h)))
        return Factors(h.value, X)

    def import_factors(self, ckpt: dict) -> Factors:
        """A factor handle from Factors.checkpoint() output (host arrays)."""
        n = int(ckpt["n_occ"])
        ranks = np.ascontiguousarray(ckpt["ranks"], dtype=np.int32)
        off = np.ascontiguousarray(ckpt["row_offset"], dtype=np.int64)
        fd = np.ascontiguousarray(ckpt["first_dropped"], dtype=np.float64)
        disc = np.ascontiguousarray(ckpt["discarded"], dtype=np.float64)
        rows = np.ascontiguousarray(ckpt["rows"], dtype=np.float64)
        assert ranks.shape == off.shape == fd.shape == disc.shape == (n, n)
        h = ctypes.c_void_p()
        self._check(self._lib.lo_factors_import(self._h, int(ckpt["M"]), n, int(ckpt["n_chol"]), ranks.ctypes.data,
                                                off.ctypes.data, fd.ctypes.data, disc.ctypes.data,
                                                rows.ctypes.data if rows.size else None, int(ckpt["flags"]),
                                                ctypes.byref(h)))
        return Factors(h.value, int(ckpt["n_chol"]))

    def build_lo_factors_randomized(self, lbar, epsilon: float, omega, power_iters: int = 2) -> Factors:
        """LO factors from a randomized SVD with the test matrix omega [M][sketch] (float64, device)."""
        import torch
        X, M, n = lbar.shape
        _check_dev("lbar", lbar, torch.float64, (X, M, n))
        _check_dev("omega", omega, torch.float64, (M, omega.shape[1]))
        h = ctypes.c_void_p()
        self._check(self._lib.build_lo_factors_randomized(self._h, M, n, X, _ptr(lbar), float(epsilon), omega.shape[1],
                                                          int(power_iters), _ptr(omega), ctypes.byref(h)))
        return Factors(h.value, X)

    def build_hr_eri(self, lbar) -> HrEri:
        import torch
        X, M, n = lbar.shape
        _check_dev("lbar", lbar, torch.float64, (X, M, n))
        h = ctypes.c_void_p()
        self._check(self._lib.build_hr_eri(self._h, M, n, X, _ptr(lbar), ctypes.byref(h)))
        return HrEri(h.value)

    # -- per walker ---------------------------------------------------------------
    def green_theta(self, trial, phi, theta=None, log_ovlp=None, info=None, orbital_major=False,
                    flag_small_pivots=False, transposed=False):
        """theta is [nw][M][n] (walker-major), [n][M][nw] when orbital_major or
        [nw][n][M] when transposed.
        flag_small_pivots: nearly singular overlaps get info < 0 (a warning)."""
        import torch
        nw, M, n = phi.shape
        _check_dev("trial", trial, torch.float64, (M, n))
        _check_dev("phi", phi, torch.complex128, (nw, M, n))
        dev = phi.device
        if orbital_major and transposed:
            raise ValueError("theta cannot be orbital-major and transposed")
        tshape = (n, M, nw) if orbital_major else (nw, n, M) if transposed else (nw, M, n)
        if theta is None:
            theta = torch.empty(tshape, dtype=torch.complex128, device=dev)
        if log_ovlp is None:
            log_ovlp = torch.empty((nw,), dtype=torch.complex128, device=dev)
        if info is None:
            info = torch.empty((nw,), dtype=torch.int32, device=dev)
        _check_dev("theta", theta, torch.complex128, tshape)
        _check_dev("log_ovlp", log_ovlp, torch.complex128, (nw,))
        _check_dev("info", info, torch.int32, (nw,))
        flags = ((LO_THETA_ORBITAL_MAJOR if orbital_major else 0) | (LO_THETA_TRANSPOSED if transposed else 0)
                 | (LO_FLAG_SMALL_PIVOT if flag_small_pivots else 0))
        self._check(self._lib.green_theta(self._h, M, n, nw, _ptr(trial), _ptr(phi), _ptr(theta), _ptr(log_ovlp),
                                          _ptr(info), flags))
        return theta, log_ovlp, info

    def local_energy_full(self, lbar, theta, info=None, energy=None, precision=LO_FP64, flags=0):
        import torch
        X, M, n = lbar.shape
        nw = theta.shape[0]
        _check_dev("lbar", lbar, torch.float64, (X, M, n))
        _check_dev("theta", theta, torch.complex128, (nw, M, n))
        if info is not None:
            _check_dev("info", info, torch.int32, (nw,))
        if energy is None:
            energy = torch.empty((nw, 2), dtype=torch.complex128, device=theta.device)
        _check_dev("energy", energy, torch.complex128, (nw, 2))
        self._check(self._lib.local_energy_full(self._h, M, n, X, nw, _ptr(lbar), _ptr(theta), _ptr(info),
                                                int(precision), int(flags), _ptr(energy)))
        return energy

    def local_energy_lo(self, factors: Factors, theta, info=None, energy=None, precision=LO_FP64, flags=0,
                        orbital_major=False, noalloc=False, lbar=None, transposed=False):
        """theta is [nw][M][n], [n][M][nw] when orbital_major, or [nw][n][M]
        when transposed.  noalloc=True
        calls local_energy_lo_noalloc (fixed scratch, no device allocation in
        the library; `energy` should then be passed in by the caller).  With
        lbar ([X][M][n], the vectors the factors were built from) E_J comes
        from the Cholesky traces (LO_EXACT_COULOMB)."""
        import torch
        if lbar is not None:
            _check_dev("lbar", lbar, torch.float64, (lbar.shape[0], factors.M, factors.n_occ))
            flags = flags | LO_EXACT_COULOMB
        nw, lflag, tshape = _theta_layout(theta, factors.M, factors.n_occ, orbital_major, transposed)
        _check_dev("theta", theta, torch.complex128, tshape)
        flags = flags | lflag
        if info is not None:
            _check_dev("info", info, torch.int32, (nw,))
        if energy is None:
            energy = torch.empty((nw, 2), dtype=torch.complex128, device=theta.device)
        _check_dev("energy", energy, torch.complex128, (nw, 2))
        fn = self._lib.local_energy_lo_noalloc if noalloc else self._lib.local_energy_lo
        self._check(fn(self._h, factors.handle, nw, _ptr(theta), _ptr(info), int(precision), int(flags),
                       _ptr(lbar), _ptr(energy)))
        return energy

    def local_energy_hr(self, hr: HrEri, theta, info=None, energy=None, orbital_major=False):
        """Eq. 17 route; theta is [nw][M][n], or [n][M][nw] when orbital_major."""
        import torch
        flags = 0
        if orbital_major:
            nw = theta.shape[2]
            _check_dev("theta", theta, torch.complex128, (hr.n_occ, hr.M, nw))
            flags = LO_THETA_ORBITAL_MAJOR
        else:
            nw = theta.shape[0]
            _check_dev("theta", theta, torch.complex128, (nw, hr.M, hr.n_occ))
        if info is not None:
            _check_dev("info", info, torch.int32, (nw,))
        if energy is None:
            energy = torch.empty((nw, 2), dtype=torch.complex128, device=theta.device)
        _check_dev("energy", energy, torch.complex128, (nw, 2))
        self._check(self._lib.local_energy_hr(self._h, hr.handle, nw, _ptr(theta), _ptr(info), flags,
                                              _ptr(energy)))
        return energy

    # -- multi-determinant trials ---------------------------------------------------
    def build_md_trial(self, factors, n_occ, n_act_occ, orbitals, holes, particles, coeffs) -> MdTrial:
        """holes / particles: one sequence of column indices per determinant (the
        reference: empty); orbitals: device float64 [M][n_cas]."""
        import numpy as np
        import torch
        _check_dev("orbitals", orbitals, torch.float64, (factors.M, factors.n_occ))
        n_det = len(coeffs)
        if len(holes) != n_det or len(particles) != n_det:
            raise ValueError("holes, particles and coeffs differ in length")
        max_exc = max([len(h) for h in holes] + [0])
        exc = np.zeros(n_det, dtype=np.int32)
        hh = np.zeros((n_det, max(max_exc, 1)), dtype=np.int32)
        pp = np.zeros((n_det, max(max_exc, 1)), dtype=np.int32)
        for d, (h, p) in enumerate(zip(holes, particles)):
            if len(h) != len(p):
                raise ValueError("determinant %d: %d holes, %d particles" % (d, len(h), len(p)))
            exc[d] = len(h)
            hh[d, :len(h)] = h
            pp[d, :len(p)] = p
        if max_exc == 0:
            hh = hh[:, :0].copy()
            pp = pp[:, :0].copy()
        c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
        h = ctypes.c_void_p()
        self._check(self._lib.build_md_trial(
            self._h, factors.handle, n_occ, n_act_occ, _ptr(orbitals), n_det, max_exc,
            exc.ctypes.data, hh.ctypes.data if hh.size else None, pp.ctypes.data if pp.size else None,
            c.ctypes.data, ctypes.byref(h)))
        return MdTrial(h.value, factors)

    def local_energy_md(self, md: MdTrial, theta, info=None, energy=None, ovlp_ratio=None, orbital_major=False,
                        transposed=False):
        """Multi-determinant LO energy; theta from green_theta with the reference
        determinant, [nw][M][n_occ], [n_occ][M][nw] when orbital_major or
        [nw][n_occ][M] when transposed."""
        import torch
        nw, flags, tshape = _theta_layout(theta, md.M, md.n_occ, orbital_major, transposed)
        _check_dev("theta", theta, torch.complex128, tshape)
        if info is not None:
            _check_dev("info", info, torch.int32, (nw,))
        if energy is None:
            energy = torch.empty((nw, 2), dtype=torch.complex128, device=theta.device)
        _check_dev("energy", energy, torch.complex128, (nw, 2))
        if ovlp_ratio is not None:
            _check_dev("ovlp_ratio", ovlp_ratio, torch.complex128, (nw,))
        self._check(self._lib.local_energy_md(self._h, md.handle, nw, _ptr(theta), _ptr(info), flags,
                                              _ptr(energy), _ptr(ovlp_ratio)))
        return energy

    # -- learned residual (extension) ---------------------------------------------
    def residual_nparam(self) -> int:
        return int(self._lib.lo_residual_nparam())

    def residual_prepare(self, factors: Factors, lbar, trial, grad=None):
        """Set-up of the fourth residual feature (the gradient of the dropped
        energy at the trial); lbar [X][M][n] and trial [M][n] are the inputs the
        factors were built from.  grad: optional device float64 [M][n] copy."""
        import torch
        X = lbar.shape[0]
        _check_dev("lbar", lbar, torch.float64, (X, factors.M, factors.n_occ))
        _check_dev("trial", trial, torch.float64, (factors.M, factors.n_occ))
        if grad is not None:
            _check_dev("grad", grad, torch.float64, (factors.M, factors.n_occ))
        self._check(self._lib.lo_residual_prepare(self._h, factors.handle, X, _ptr(lbar), _ptr(trial), _ptr(grad)))
        return grad

    def localize_boys(self, positions, orbitals, max_sweeps=50, tol=1e-14):
        """Foster-Boys localization of orbitals [M][n] (device float64, in
        place) for position operators positions [D][M]; returns (B before,
        B after, sweeps run)."""
        import torch
        M, n = orbitals.shape
        _check_dev("orbitals", orbitals, torch.float64, (M, n))
        D = positions.shape[0]
        _check_dev("positions", positions, torch.float64, (D, M))
        st = (ctypes.c_double * 3)()
        self._check(self._lib.lo_localize_boys(self._h, M, n, D, _ptr(positions), _ptr(orbitals), int(max_sweeps),
                                               float(tol), ctypes.addressof(st)))
        return st[0], st[1], int(st[2])

    def residual_target(self, e_exact, e_lo, shift=0.0, scale=1.0, t=None):
        """(1000 Re(sum e_exact - sum e_lo) - shift) / scale per walker, float64 [nw]."""
        import torch
        nw = e_lo.shape[0]
        _check_dev("e_exact", e_exact, torch.complex128, (nw, 2))
        _check_dev("e_lo", e_lo, torch.complex128, (nw, 2))
        if t is None:
            t = torch.empty((nw,), dtype=torch.float64, device=e_lo.device)
        _check_dev("t", t, torch.float64, (nw,))
        self._check(self._lib.lo_residual_target(self._h, nw, _ptr(e_exact), _ptr(e_lo), float(shift), float(scale),
                                                 _ptr(t)))
        return t

    def residual_apply(self, energy, pred=None, scale=1.0, shift=0.0, out=None):
        """E_J + E_K (+ (pred * scale + shift) / 1000 on the real part), complex128 [nw]."""
        import torch
        nw = energy.shape[0]
        _check_dev("energy", energy, torch.complex128, (nw, 2))
        if pred is not None:
            _check_dev("pred", pred, torch.float64, (nw,))
        if out is None:
            out = torch.empty((nw,), dtype=torch.complex128, device=energy.device)
        _check_dev("out", out, torch.complex128, (nw,))
        self._check(self._lib.lo_residual_apply(self._h, nw, _ptr(energy), _ptr(pred), float(scale), float(shift),
                                                _ptr(out)))
        return out

    def residual_features(self, factors: Factors, theta, x=None):
        """x [nw][n][4] float32 from walker-major theta [nw][M][n]."""
        import torch
        nw = theta.shape[0]
        _check_dev("theta", theta, torch.complex128, (nw, factors.M, factors.n_occ))
        if x is None:
            x = torch.empty((nw, factors.n_occ, RESIDUAL_NFEAT), dtype=torch.float32, device=theta.device)
        _check_dev("x", x, torch.float32, (nw, factors.n_occ, RESIDUAL_NFEAT))
        self._check(self._lib.lo_residual_features(self._h, factors.handle, nw, _ptr(theta), _ptr(x)))
        return x

    def residual_predict(self, params, x, precision=LO_FP32, pred=None):
        import torch
        nw, n, _ = x.shape
        _check_dev("params", params, torch.float32, (self.residual_nparam(),))
        _check_dev("x", x, torch.float32, (nw, n, RESIDUAL_NFEAT))
        if pred is None:
            pred = torch.empty((nw,), dtype=torch.float64, device=x.device)
        _check_dev("pred", pred, torch.float64, (nw,))
        self._check(self._lib.lo_residual_predict(self._h, nw, n, _ptr(params), _ptr(x), int(precision), _ptr(pred)))
        return pred

    def residual_train_step(self, params, adam_m, adam_v, step: int, lr: float, x, target, grad=None, loss=None,
                            pred=None):
        import torch
        nw, n, _ = x.shape
        npar = self.residual_nparam()
        _check_dev("params", params, torch.float32, (npar,))
        _check_dev("x", x, torch.float32, (nw, n, RESIDUAL_NFEAT))
        _check_dev("target", target, torch.float64, (nw,))
        if step > 0:
            _check_dev("adam_m", adam_m, torch.float32, (npar,))
            _check_dev("adam_v", adam_v, torch.float32, (npar,))
        if grad is not None:
            _check_dev("grad", grad, torch.float32, (npar,))
        if loss is not None:
            _check_dev("loss", loss, torch.float64, (1,))
        if pred is not None:
            _check_dev("pred", pred, torch.float64, (nw,))
        self._check(self._lib.lo_residual_train_step(self._h, nw, n, _ptr(params), _ptr(adam_m), _ptr(adam_v),
                                                     int(step), float(lr), _ptr(x), _ptr(target), _ptr(grad),
                                                     _ptr(loss), _ptr(pred)))
