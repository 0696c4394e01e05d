"""Thin ctypes binding of libks (include/ks.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Device buffers are torch tensors on the current HIP device; the
current torch stream is passed to every call.  Importing this module loads
``libks.so`` and raises when it is missing -- there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libks.so")
HEADER = os.path.join(HERE, "..", "include", "ks.h")

KS_OK, KS_EINVAL, KS_ENOMEM, KS_EDEVICE, KS_EUNSUPPORTED = range(5)
KS_FP64, KS_MIXED = 0, 1
KS_XC_NONE, KS_XC_LDA = 0, 1
KERNELS = ["pack", "unpack", "plane_inv", "xproj", "proj_reduce", "xapply", "plane_fwd", "xdens", "dots",
           "gemm", "eig", "sd", "gproj"]


class Info(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int) for f in ("npw", "nplanes", "ncols", "chunk", "natoms", "nproj", "nruns",
                                            "nslots", "npoints", "x_tile", "precision", "x_half", "x_group",
                                            "plane_group", "x_shape", "x_threads", "projection")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("x_group", ctypes.c_int), ("plane_group", ctypes.c_int), ("ms", ctypes.c_double),
                ("from_cache", ctypes.c_int), ("x_shape", ctypes.c_int), ("projection", ctypes.c_int)]


_STATUS = {1: "KS_EINVAL", 2: "KS_ENOMEM", 3: "KS_EDEVICE", 4: "KS_EUNSUPPORTED"}


class KSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def _load():
    # torch ships its own HIP runtime (same SONAME as /opt/rocm's).  Loading
    # torch first makes libks bind to that one copy; the other order would put
    # two HIP runtimes in the process.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2106_03872_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "ks_system_create": (I, [ctypes.POINTER(I), ctypes.POINTER(D), D, I, I, ctypes.POINTER(P)]),
        "ks_system_destroy": (None, [P]),
        "ks_system_create_in": (I, [P, ctypes.POINTER(I), ctypes.POINTER(D), D, I, I, ctypes.POINTER(P)]),
        "ks_system_create_ex": (I, [P, ctypes.POINTER(I), ctypes.POINTER(D), D, I, I, I, ctypes.POINTER(P)]),
        "ks_pool_create": (I, [ctypes.c_ulonglong, ctypes.POINTER(P)]),
        "ks_stream_create": (I, [ctypes.POINTER(P)]),
        "ks_stream_destroy": (None, [P]),
        "ks_batch_create": (I, [ctypes.POINTER(P), I, ctypes.POINTER(P)]),
        "ks_batch_destroy": (None, [P]),
        "ks_batch_propagate": (I, [P, D, I, P]),
        "ks_batch_capture": (I, [P, D, P]),
        "ks_batch_replay": (I, [P, P]),
        "ks_batch_last_error": (ctypes.c_char_p, [P]),
        "ks_propagate_batch": (I, [ctypes.POINTER(P), I, D, I, P]),
        "ks_pool_destroy": (None, [P]),
        "ks_pool_usage": (I, [P, ctypes.POINTER(ctypes.c_ulonglong), ctypes.POINTER(ctypes.c_ulonglong),
                              ctypes.POINTER(ctypes.c_ulonglong)]),
        "ks_last_error": (ctypes.c_char_p, [P]),
        "ks_system_set_vloc": (I, [P, P, P]),
        "ks_system_set_projectors": (I, [P, I, I, P, P, P, P, P]),
        "ks_ham_apply": (I, [P, I, P, P, P]),
        "ks_propagate_step": (I, [P, I, P, D, I, P, P, P]),
        "ks_density": (I, [P, I, P, P, P, P]),
        "ks_reduce": (I, [P, I, P, P, P, P, P]),
        "ks_orthonormalize": (I, [P, I, P, P]),
        "ks_system_npw": (I, [P]),
        "ks_system_chunk": (I, [P]),
        "ks_system_set_chunk": (I, [P, I]),
        "ks_system_info": (I, [P, P]),
        "ks_state_create": (I, [P, I, ctypes.POINTER(P)]),
        "ks_state_destroy": (None, [P]),
        "ks_state_upload": (I, [P, P, P]),
        "ks_state_download": (I, [P, P, P]),
        "ks_state_propagate": (I, [P, D, I, P, P, P, P]),
        "ks_state_propagate_etrs": (I, [P, D, I, P, P, P, P]),
        "ks_hartree": (I, [P, P, P, I, P]),
        "ks_system_set_xc": (I, [P, I]),
        "ks_lda_xc": (I, [P, P, P, I, P]),
        "ks_dipole": (I, [P, P, P, P]),
        "ks_spectrum": (I, [P, I, D, ctypes.POINTER(D), P, I, D, P, P, P]),
        "ks_dipole_noalloc": (I, [ctypes.POINTER(I), ctypes.POINTER(D), P, P, P]),
        "ks_state_kick": (I, [P, ctypes.POINTER(D), P]),
        "ks_state_eigensolve": (I, [P, I, P, P, P]),
        "ks_state_reduce": (I, [P, P, P, P, P]),
        "ks_state_capture": (I, [P, D, P, P, P]),
        "ks_state_replay": (I, [P, P]),
        "ks_plan_footprint": (I, [ctypes.POINTER(I), ctypes.POINTER(D), D, I, I, I, I, I,
                                  ctypes.POINTER(ctypes.c_ulonglong)]),
        "ks_plan_sphere": (I, [ctypes.POINTER(I), ctypes.POINTER(D), D, ctypes.POINTER(I), P]),
        "ks_plan_projectors": (I, [ctypes.POINTER(I), I, I, P, P, P, ctypes.POINTER(I), P, P, P, P]),
        "ks_set_kernel_timing": (I, [P, I]),
        "ks_autotune": (I, [P, I, P, P]),
        "ks_system_set_tuning": (I, [P, P]),
        "ks_kernel_time": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()

# At interpreter exit the process releases every device resource itself;
# finalisers that run after this point (objects collected during shutdown, in
# no particular order) do not call into the runtime.
_exiting = False


def _mark_exiting():
    global _exiting
    _exiting = True


atexit.register(_mark_exiting)


def header_symbols():
    """Entry points declared in include/ks.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ks_status|void|const char\*|int)\s+(ks_\w+)\s*\(", txt, re.M)))


def library():
    return _lib


def plan_sphere(n, L, ecut):
    """Integer frequencies (m0, m1, m2) of the packed plane-wave sphere, in the
    library's packed order (host-only call)."""
    nn = (ctypes.c_int * 3)(*[int(x) for x in n])
    LL = (ctypes.c_double * 3)(*[float(x) for x in L])
    npw = ctypes.c_int()
    st = _lib.ks_plan_sphere(nn, LL, float(ecut), ctypes.byref(npw), None)
    if st != KS_OK:
        raise KSError(st, _lib.ks_last_error(None).decode())
    m = np.zeros((npw.value, 3), np.int32)
    st = _lib.ks_plan_sphere(nn, LL, float(ecut), ctypes.byref(npw), m.ctypes.data_as(ctypes.c_void_p))
    if st != KS_OK:
        raise KSError(st, _lib.ks_last_error(None).decode())
    return m


def plan_projectors(n, npts, idx, beta, nproj=None):
    """Kleinman-Bylander point tables (host-only call): dict with counts and,
    per unique grid point, its flat index and its (atom, input row) entries."""
    npts = np.ascontiguousarray(npts, np.int32)
    idx = np.ascontiguousarray(idx, np.int32)
    beta = np.ascontiguousarray(beta, np.float64)
    nproj = beta.shape[1] if nproj is None else nproj
    nn = (ctypes.c_int * 3)(*[int(x) for x in n])
    counts = (ctypes.c_int * 4)()
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else None
    args = (nn, len(npts), int(nproj), ptr(npts), ptr(idx), ptr(beta), counts)
    st = _lib.ks_plan_projectors(*args, None, None, None, None)
    if st != KS_OK:
        raise KSError(st, _lib.ks_last_error(None).decode())
    nslots, nuniq, nent, nruns = list(counts)
    flat = np.zeros(nuniq, np.int32)
    pent = np.zeros(nuniq + 1, np.int32)
    eatom = np.zeros(nent, np.int32)
    erow = np.zeros(nent, np.int32)
    st = _lib.ks_plan_projectors(*args, flat.ctypes.data_as(ctypes.c_void_p), pent.ctypes.data_as(ctypes.c_void_p),
                                 eatom.ctypes.data_as(ctypes.c_void_p), erow.ctypes.data_as(ctypes.c_void_p))
    if st != KS_OK:
        raise KSError(st, _lib.ks_last_error(None).decode())
    return {"slots": nslots, "unique": nuniq, "entries": nent, "runs": nruns, "point_flat": flat,
            "point_entries": pent, "entry_atom": eatom, "entry_row": erow}


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, shape=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Stream:
    """A non-blocking HIP stream (ks_stream_create) usable as a torch stream
    (``.torch``): graphs can be captured on it while other threads use the
    legacy default stream.  torch may keep the raw stream in its allocators'
    bookkeeping (events of pinned or cross-stream blocks), so the stream is
    destroyed only by an explicit close(), never by garbage collection; long-
    lived users take streams from ``stream_pool``."""

    def __init__(self):
        import torch
        h = ctypes.c_void_p()
        st = _lib.ks_stream_create(ctypes.byref(h))
        if st != KS_OK:
            raise KSError(st, _lib.ks_last_error(None).decode())
        self._h = h
        self.torch = torch.cuda.ExternalStream(h.value)

    def close(self):
        """Destroy the stream after its work (the caller makes sure nothing
        refers to it any more)."""
        if getattr(self, "_h", None):
            self.torch.synchronize()
            _lib.ks_stream_destroy(self._h)
            self._h = None


_stream_pool = []
_stream_pool_lock = None


def stream_pool(i):
    """The i-th process-wide non-blocking Stream (created on first use, kept
    until the process ends), so that repeated users reuse streams."""
    import threading
    global _stream_pool_lock
    if _stream_pool_lock is None:
        _stream_pool_lock = threading.Lock()
    with _stream_pool_lock:
        while len(_stream_pool) <= i:
            _stream_pool.append(Stream())
        return _stream_pool[i]


class Batch:
    """Resident states of distinct systems of one grid stepped together,
    one launch per kernel for all of them (ks_batch_create).  The batch
    keeps the states (and their systems) referenced."""

    def __init__(self, states):
        self.states = list(states)
        arr = (ctypes.c_void_p * len(self.states))(*[s._h.value for s in self.states])
        h = ctypes.c_void_p()
        st = _lib.ks_batch_create(arr, len(self.states), ctypes.byref(h))
        if st != KS_OK:
            raise KSError(st, _lib.ks_batch_last_error(None).decode())
        self._h = h
        self._captured = None

    def _check(self, st):
        if st != KS_OK:
            raise KSError(st, _lib.ks_batch_last_error(self._h).decode())

    @staticmethod
    def _st(stream):
        return ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream()

    def propagate(self, dt, nsteps=1, stream=None):
        self._check(_lib.ks_batch_propagate(self._h, float(dt), int(nsteps), self._st(stream)))

    def capture(self, dt, stream):
        if stream is None:
            raise ValueError("capture needs an explicit non-default stream")
        self._check(_lib.ks_batch_capture(self._h, float(dt), self._st(stream)))

    def replay(self, stream=None):
        self._check(_lib.ks_batch_replay(self._h, self._st(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.ks_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


def propagate_batch(states, dt, nsteps=1, stream=None):
    """ks_propagate_batch: nsteps Taylor-4 steps of the states together."""
    arr = (ctypes.c_void_p * len(states))(*[s._h.value for s in states])
    st = _lib.ks_propagate_batch(arr, len(states), float(dt), int(nsteps),
                                 ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream())
    if st != KS_OK:
        raise KSError(st, _lib.ks_batch_last_error(None).decode())


class Pool:
    """Device memory pool (ks_pool_create): systems created in it allocate
    and free without hipMalloc / hipFree."""

    def __init__(self, nbytes):
        h = ctypes.c_void_p()
        st = _lib.ks_pool_create(int(nbytes), ctypes.byref(h))
        if st != KS_OK:
            raise KSError(st, _lib.ks_last_error(None).decode())
        self._h = h
        self.nbytes = int(nbytes)

    def usage(self):
        """(used, peak, largest free range) in bytes."""
        u, p, f = ctypes.c_ulonglong(), ctypes.c_ulonglong(), ctypes.c_ulonglong()
        st = _lib.ks_pool_usage(self._h, ctypes.byref(u), ctypes.byref(p), ctypes.byref(f))
        if st != KS_OK:
            raise KSError(st, _lib.ks_last_error(None).decode())
        return u.value, p.value, f.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.ks_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


class System:
    """One Kohn-Sham system (grid, cell, cutoff, potential, projectors);
    with `pool`, its device memory comes from that Pool."""

    def __init__(self, n, L, ecut, max_norb, precision=KS_FP64, pool=None, chunk=0):
        self.n = tuple(int(x) for x in n)
        self.L = tuple(float(x) for x in L)
        self.ecut = float(ecut)
        self.max_norb = int(max_norb)
        self.N = int(np.prod(self.n))
        self.pool = pool
        h = ctypes.c_void_p()
        nn, LL = (ctypes.c_int * 3)(*self.n), (ctypes.c_double * 3)(*self.L)
        if chunk:
            st = _lib.ks_system_create_ex(None if pool is None else pool._h, nn, LL, self.ecut, int(precision),
                                          self.max_norb, int(chunk), ctypes.byref(h))
        elif pool is None:
            st = _lib.ks_system_create(nn, LL, self.ecut, int(precision), self.max_norb, ctypes.byref(h))
        else:
            st = _lib.ks_system_create_in(pool._h, nn, LL, self.ecut, int(precision), self.max_norb, ctypes.byref(h))
        if st != KS_OK:
            raise KSError(st, _lib.ks_last_error(None).decode())
        self._h = h

    def _check(self, st):
        if st != KS_OK:
            raise KSError(st, _lib.ks_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            _lib.ks_system_destroy(self._h)
            self._h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass

    @property
    def npw(self):
        return _lib.ks_system_npw(self._h)

    @property
    def chunk(self):
        return _lib.ks_system_chunk(self._h)

    def set_chunk(self, c):
        self._check(_lib.ks_system_set_chunk(self._h, int(c)))

    def info(self):
        inf = Info()
        self._check(_lib.ks_system_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def autotune(self, norb):
        """Time the launch-schedule candidates (x-tile shape and orbital-group
        caps) for H psi over `norb` orbitals and keep the fastest (cached per
        process by grid, precision and size).  Returns {x_group, plane_group,
        ms, from_cache, x_shape, projection}; the projection mode is kept."""
        t = Tuning()
        self._check(_lib.ks_autotune(self._h, int(norb), _stream(), ctypes.byref(t)))
        return {"x_group": t.x_group, "plane_group": t.plane_group, "ms": t.ms, "from_cache": bool(t.from_cache),
                "x_shape": t.x_shape, "projection": t.projection}

    def set_tuning(self, x_group, plane_group, x_shape=None, projection=None):
        """Set the group caps and, unless None, the x-tile shape and the
        projection mode (0: real-space sums; 1: reciprocal-space split-BF16
        product, mixed precision only)."""
        t = Tuning(int(x_group), int(plane_group), 0.0, 0, -1 if x_shape is None else int(x_shape),
                   -1 if projection is None else int(projection))
        self._check(_lib.ks_system_set_tuning(self._h, ctypes.byref(t)))

    def hartree(self, rho, add_vloc=False, out=None):
        """Periodic Hartree potential of the density rho (float64 box on the
        device), plus the static V_loc when add_vloc."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        self._check(_lib.ks_hartree(self._h, _ptr(rho, torch.float64, self.n, "rho"),
                                    _ptr(out, torch.float64, self.n, "out"), int(bool(add_vloc)), _stream()))
        return out

    def set_xc(self, functional):
        """Exchange-correlation term of the density-dependent potential used by
        ETRS: KS_XC_NONE or KS_XC_LDA."""
        self._check(_lib.ks_system_set_xc(self._h, int(functional)))

    def lda_xc(self, rho, out=None, accumulate=False):
        """Local-density exchange-correlation potential of the density rho
        (float64 box on the device); added to out when accumulate."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        self._check(_lib.ks_lda_xc(self._h, _ptr(rho, torch.float64, self.n, "rho"),
                                   _ptr(out, torch.float64, self.n, "out"), int(bool(accumulate)), _stream()))
        return out

    def dipole(self, rho):
        """Dipole moment dV sum_r r rho(r) of a density (float64 box on the
        device); returns a float64 tensor of 3 on the device."""
        import torch
        d = torch.empty(3, dtype=torch.float64, device="cuda")
        self._check(_lib.ks_dipole(self._h, _ptr(rho, torch.float64, self.n, "rho"), _ptr(d, torch.float64), _stream()))
        return d

    def set_kernel_timing(self, enable=True):
        self._check(_lib.ks_set_kernel_timing(self._h, int(bool(enable))))

    def kernel_times(self):
        """{kernel name: (total ms, launches)} since timing was enabled."""
        out = {}
        for k, name in enumerate(KERNELS):
            ms, n = ctypes.c_double(), ctypes.c_longlong()
            self._check(_lib.ks_kernel_time(self._h, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def box_shape(self, norb):
        return (int(norb),) + self.n

    # ---------------------------------------------------------------- set-up
    def set_vloc(self, v):
        import torch
        self._check(_lib.ks_system_set_vloc(self._h, _ptr(v, torch.float64, self.n, "v"), _stream()))

    def set_projectors(self, npts, idx, beta, d):
        npts = np.ascontiguousarray(npts, np.int32)
        idx = np.ascontiguousarray(idx, np.int32)
        beta = np.ascontiguousarray(beta, np.float64)
        d = np.ascontiguousarray(d, np.float64)
        natoms = len(npts)
        nproj = d.shape[1] if d.ndim == 2 and natoms else (beta.shape[1] if beta.ndim == 2 else 1)
        if natoms and (beta.shape[0] != idx.shape[0] or int(npts.sum()) != idx.shape[0]):
            raise ValueError("npts, idx and beta disagree")
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else None
        self._check(_lib.ks_system_set_projectors(self._h, natoms, int(nproj), ptr(npts), ptr(idx),
                                                  ptr(beta), ptr(d), _stream()))
        self._keep = (npts, idx, beta, d)

    # ------------------------------------------------------------- hot path
    def ham_apply(self, psi, hpsi=None):
        import torch
        norb = psi.shape[0]
        if hpsi is None:
            hpsi = torch.empty_like(psi)
        self._check(_lib.ks_ham_apply(self._h, norb, _ptr(psi, torch.complex128, self.box_shape(norb), "psi"),
                                      _ptr(hpsi, torch.complex128, self.box_shape(norb), "hpsi"), _stream()))
        return hpsi

    def propagate_step(self, psi, dt, nsteps=1, occ=None, rho=None):
        import torch
        norb = psi.shape[0]
        self._check(_lib.ks_propagate_step(
            self._h, norb, _ptr(psi, torch.complex128, self.box_shape(norb), "psi"), float(dt), int(nsteps),
            _ptr(occ, torch.float64, (norb,), "occ"),
            _ptr(rho, torch.float64, (int(nsteps),) + self.n, "rho"), _stream()))
        return psi

    def density(self, psi, occ, rho=None):
        import torch
        norb = psi.shape[0]
        if rho is None:
            rho = torch.empty(self.n, dtype=torch.float64, device=psi.device)
        self._check(_lib.ks_density(self._h, norb, _ptr(psi, torch.complex128, self.box_shape(norb), "psi"),
                                    _ptr(occ, torch.float64, (norb,), "occ"),
                                    _ptr(rho, torch.float64, self.n, "rho"), _stream()))
        return rho

    def reduce(self, psi, occ=None, want_energy=True):
        import torch
        norb = psi.shape[0]
        norms = torch.empty(norb, dtype=torch.float64, device=psi.device)
        energy = torch.empty(1, dtype=torch.float64, device=psi.device) if want_energy else None
        self._check(_lib.ks_reduce(self._h, norb, _ptr(psi, torch.complex128, self.box_shape(norb), "psi"),
                                   _ptr(occ, torch.float64, (norb,), "occ"), _ptr(norms, torch.float64),
                                   _ptr(energy, torch.float64), _stream()))
        return norms, energy

    def orthonormalize(self, psi):
        import torch
        norb = psi.shape[0]
        self._check(_lib.ks_orthonormalize(self._h, norb, _ptr(psi, torch.complex128, self.box_shape(norb), "psi"),
                                           _stream()))
        return psi


class State:
    """Orbitals of one system resident on the device (packed FP64 layout)."""

    def __init__(self, system, norb):
        self.system = system
        self.norb = int(norb)
        h = ctypes.c_void_p()
        system._check(_lib.ks_state_create(system._h, self.norb, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.ks_state_destroy(self._h)
            self._h = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass

    def _st(self, stream):
        return ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream()

    def upload(self, psi, stream=None):
        import torch
        self.system._check(_lib.ks_state_upload(
            self._h, _ptr(psi, torch.complex128, self.system.box_shape(self.norb), "psi"), self._st(stream)))

    def download(self, psi=None, stream=None):
        import torch
        if psi is None:
            psi = torch.empty(self.system.box_shape(self.norb), dtype=torch.complex128, device="cuda")
        self.system._check(_lib.ks_state_download(
            self._h, _ptr(psi, torch.complex128, self.system.box_shape(self.norb), "psi"), self._st(stream)))
        return psi

    def propagate(self, dt, nsteps=1, occ=None, rho=None, norms=None, stream=None):
        """nsteps Taylor-4 steps; rho [nsteps][n0][n1][n2] and norms
        [nsteps][norb] (float64, optional) receive the density and the
        orbital norms after each step."""
        import torch
        if rho is not None and rho.numel() < int(nsteps) * int(np.prod(self.system.n)):
            raise ValueError("rho must hold nsteps densities")
        if norms is not None and norms.numel() < int(nsteps) * self.norb:
            raise ValueError("norms must hold nsteps x norb values")
        self.system._check(_lib.ks_state_propagate(
            self._h, float(dt), int(nsteps), _ptr(occ, torch.float64, (self.norb,), "occ"),
            _ptr(rho, torch.float64, None, "rho"), _ptr(norms, torch.float64, None, "norms"), self._st(stream)))

    def kick(self, k, stream=None):
        """psi <- exp(i k.r) psi for every resident orbital (field kick at t = 0)."""
        kk = (ctypes.c_double * 3)(*[float(x) for x in k])
        self.system._check(_lib.ks_state_kick(self._h, kk, self._st(stream)))

    def propagate_etrs(self, dt, nsteps, occ, rho=None, norms=None, stream=None):
        """nsteps ETRS steps under the density-dependent Hamiltonian
        (V_loc + Hartree, + LDA exchange-correlation after
        system.set_xc(KS_XC_LDA)); rho [nsteps][n0][n1][n2] and norms [nsteps][norb]
        (float64, optional) receive the density and norms after each step."""
        import torch
        if rho is not None and rho.numel() < int(nsteps) * int(np.prod(self.system.n)):
            raise ValueError("rho must hold nsteps densities")
        if norms is not None and norms.numel() < int(nsteps) * self.norb:
            raise ValueError("norms must hold nsteps x norb values")
        self.system._check(_lib.ks_state_propagate_etrs(
            self._h, float(dt), int(nsteps), _ptr(occ, torch.float64, (self.norb,), "occ"),
            _ptr(rho, torch.float64, None, "rho"), _ptr(norms, torch.float64, None, "norms"), self._st(stream)))

    def eigensolve(self, niter, eig=None, resid=None, stream=None):
        """niter preconditioned steepest-descent iterations towards the lowest
        norb eigenstates (orthonormal orbitals in and out); returns the Ritz
        values and residual norms of every iteration, float64 [niter][norb]."""
        import torch
        shape = (max(int(niter), 0), self.norb)
        if eig is None:
            eig = torch.empty(shape, dtype=torch.float64, device="cuda")
        if resid is None:
            resid = torch.empty(shape, dtype=torch.float64, device="cuda")
        self.system._check(_lib.ks_state_eigensolve(
            self._h, int(niter), _ptr(eig, torch.float64, shape, "eig"), _ptr(resid, torch.float64, shape, "resid"),
            self._st(stream)))
        return eig, resid

    def reduce(self, occ=None, want_energy=True, stream=None):
        import torch
        norms = torch.empty(self.norb, dtype=torch.float64, device="cuda")
        energy = torch.empty(1, dtype=torch.float64, device="cuda") if want_energy else None
        self.system._check(_lib.ks_state_reduce(self._h, _ptr(occ, torch.float64, (self.norb,), "occ"),
                                                _ptr(norms, torch.float64), _ptr(energy, torch.float64),
                                                self._st(stream)))
        return norms, energy

    def capture(self, dt, occ=None, rho=None, stream=None):
        """Capture one step into a graph.  The graph holds occ and rho, so
        they stay referenced here until the next capture or close."""
        import torch
        if stream is None:
            raise ValueError("capture needs an explicit non-default stream")
        self.system._check(_lib.ks_state_capture(self._h, float(dt), _ptr(occ, torch.float64, (self.norb,), "occ"),
                                                 _ptr(rho, torch.float64, None, "rho"), self._st(stream)))
        self._captured = (occ, rho)

    def replay(self, stream=None):
        self.system._check(_lib.ks_state_replay(self._h, self._st(stream)))


def plan_footprint(n, L, ecut, norb, npoints, nproj=4, precision=KS_FP64, chunk=0):
    """Device bytes of a system plus a resident state (host-only estimate)."""
    out = ctypes.c_ulonglong()
    st = _lib.ks_plan_footprint((ctypes.c_int * 3)(*[int(x) for x in n]), (ctypes.c_double * 3)(*[float(x) for x in L]),
                                float(ecut), int(precision), int(norb), int(npoints), int(nproj), int(chunk),
                                ctypes.byref(out))
    if st != KS_OK:
        raise KSError(st, _lib.ks_last_error(None).decode())
    return int(out.value)


# module-level entry points with the names of the C ABI
def dipole_noalloc(n, L, rho, d):
    """ks_dipole_noalloc: dipole moment of the density rho (float64 box of
    shape n on the device) into d (float64 tensor of 3 on the device), with no
    system and no device allocation."""
    import torch
    n = tuple(int(x) for x in n)
    nn = (ctypes.c_int * 3)(*n)
    LL = (ctypes.c_double * 3)(*[float(x) for x in L])
    st = _lib.ks_dipole_noalloc(nn, LL, _ptr(rho, torch.float64, n, "rho"), _ptr(d, torch.float64, (3,), "d"),
                                _stream())
    if st != KS_OK:
        raise KSError(st, _lib.ks_last_error(None).decode())
    return d


def ham_apply(system, psi, hpsi=None):
    return system.ham_apply(psi, hpsi)


def propagate_step(system, psi, dt, nsteps=1, occ=None, rho=None):
    return system.propagate_step(psi, dt, nsteps, occ, rho)


def density(system, psi, occ, rho=None):
    return system.density(psi, occ, rho)


def reduce(system, psi, occ=None):
    return system.reduce(psi, occ)


def orthonormalize(system, psi):
    return system.orthonormalize(psi)


def system_from_synth(sysm, max_norb=None, ecut=None, precision=KS_FP64, pool=None, chunk=0):
    """Create a System from a synth.System (potential + projectors uploaded);
    chunk > 0 sets the orbitals per pass at creation."""
    import torch
    spec = sysm.spec
    s = System(spec.n, spec.L, spec.ecut if ecut is None else ecut, max_norb or spec.norb, precision, pool, chunk)
    s.set_vloc(torch.from_numpy(sysm.vloc).to("cuda"))
    p = sysm.proj
    s.set_projectors(p.npts, p.idx, p.beta, p.d)
    return s
